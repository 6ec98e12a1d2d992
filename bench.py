#!/usr/bin/env python3
"""Throughput benchmark of the MI355X Tensorized Pauli Decomposition.

Headline (the largest single-GPU configuration): one dense Hermitian
2^16 x 2^16 matrix, A = (G + G^H)/2 with complex N(0,1) G (seed 5),
complex128, decomposed IN PLACE (coefficients in the matrix layout, the
only in-place order for n > 6).  A step is one full decomposition (bitmap
clear + two HBM sweeps, pruning on), timed with HIP events; the input is
restored from a pristine device copy before every step, outside the timed
region.  The K timed steps are spread over several successive allocations
of the in-place buffer (where the driver places a 64 GiB buffer moves the
rate by up to ~15 %): `value` is the median allocation's rate, and the
allocations' figures are listed.  Inputs are generated on the GPU and
resident in HBM before the timed region.  Prints ONE JSON line.

Extras in the same line: the other configurations (n = 8 dense and
integer, n = 12 Hermitian, n = 14 structured with pruning, the 4096-matrix
batched set against a graph of per-matrix launches, n = 16 complex64), the
error against the binary64 oracle for every configuration in both
precisions (with full Parseval sums at n = 16), out-of-place /
Hermitian-mode (complex and real weights) / real-input / synthesis /
partial legs, and the CPU oracle timed on the host.

    python bench.py [--gpus 1] [--steps 20] [--warmup 3] [--extras ...]
"""
import argparse
import hashlib
import json
import math
import re
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBPS = 8000.0
METRIC = "Pauli coeffs/sec + HBM GB/s (% peak) at n=14/16, FP64 vs FP32; batched mats/s"
KERNEL_SOURCES = ["paper_2310_13421_amd/csrc/tpd_sweep.h", "paper_2310_13421_amd/csrc/tpd_core.h",
                  "paper_2310_13421_amd/csrc/tpd_internal.h", "paper_2310_13421_amd/csrc/tpd_batched.h"]


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_source_hash():
    """Hash of the sources of the sweep and batched kernels (their headers
    and the instantiation units), the kernels whose traffic
    profiles/traffic.json records."""
    import glob

    h = hashlib.sha256()
    files = sorted(set(KERNEL_SOURCES) | {os.path.relpath(p, ROOT) for pat in ("tpd_sweep_c*.hip", "tpd_batched_*.hip")
                                          for p in glob.glob(os.path.join(ROOT, "paper_2310_13421_amd", "csrc", pat))})
    for rel in files:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def load_traffic(kernel_name, n):
    """HBM bytes per launch measured with rocprofv3 --pmc (FETCH_SIZE and
    WRITE_SIZE scaled by a plain-copy calibration) for this kernel at this
    n (None: the batched kernel on the 4096-matrix set), if taken on the
    current kernel sources."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    if t.get("kernel_source_sha") != kernel_source_hash():
        return None
    k = t.get("kernels", {}).get(kernel_name)
    # a symbol seen only in the Hermitian / real-symmetric mode (which reads
    # about half) says nothing about the general mode's bytes
    if k and k.get("only_reduced_mode_dispatches"):
        return None
    return k if k and k.get("n") == n else None


def leg_traffic(dt, res, n):
    """Measured HBM bytes per launch of each sweep of a two-sweep leg
    (None where no PMC figures were taken on the current sources)."""
    sched = res.get("schedule") or []
    if len(sched) != 2:
        return None
    out = []
    for w in (1, 2):
        k = load_traffic(sweep_kernel_name(dt, sched, w), n)
        out.append(k["total_bytes"] if k else None)
    return out


LAYOUT_CODE = {"MAT": 0, "CAN": 1, "MID": 2}


def sweep_kernel_name(dt, sched, which):
    """Symbol of the sweep kernel a two-sweep schedule launches (as the
    profiler prints it)."""
    s = sched[which - 1]
    lay = f"{LAYOUT_CODE[s['in']]}, {LAYOUT_CODE[s['out']]}"
    return f"void tpd::k_sweep<{dt}, tpd::Geom<{s['xb']}, {s['db']}, 0, {s['r']}, 0>, {lay}, false>(tpd::SweepArgs)"


def ingest_pmc(pairs, out_path):
    """Turn pairs of rocprofv3 --pmc runs of this script (FETCH_SIZE, then
    WRITE_SIZE, both with --copy-calibration) into profiles/traffic.json.
    Each counter (KiB per dispatch) is scaled by what it reads for the plain
    device copy of 2^32 bytes that --copy-calibration runs.  A kernel seen in
    several pairs takes the figures of the last one, unless an earlier pair
    measured whole general-mode sweeps and the later one only chunks or
    reduced-mode sweeps; the chunk and reduced-mode figures of the entry not
    kept are carried over as its sub-records where the kept one has none."""

    def rank(e):
        if "workload" in e or not (e.get("chunks") or e.get("only_reduced_mode_dispatches")):
            return 2
        return 1 if e.get("chunks") else 0

    def subrecords(e):
        out = {k: e[k] for k in ("reduced_mode_dispatches", "chunked_dispatches") if k in e}
        ratios = {"fetch_over_algorithmic": e.get("fetch_over_algorithmic"),
                  "write_over_algorithmic": e.get("write_over_algorithmic")}
        if e.get("only_reduced_mode_dispatches"):
            out["reduced_mode_dispatches"] = {"count": e["dispatches"], **ratios}
        elif e.get("chunks"):
            out["chunked_dispatches"] = {"count": e["dispatches"], "chunks": e["chunks"], **ratios}
        return out

    kernels, scales = {}, []
    for fetch_csv, write_csv in pairs:
        ks, fs, ws = ingest_pair(fetch_csv, write_csv)
        for name, e in ks.items():
            old = kernels.get(name)
            keep, other = (e, old) if old is None or rank(e) >= rank(old) else (old, e)
            if other is not None and "workload" not in keep and rank(keep) > rank(other):
                for k, v in subrecords(other).items():
                    keep.setdefault(k, v)
            kernels[name] = keep
        scales.append({"fetch_scale": fs, "write_scale": ws})
    doc = {"kernel_source_sha": kernel_source_hash(), "scales": scales,
           "calibration": "plain device copy of 2^32 bytes (__amd_rocclr_copyBuffer via torch copy_)",
           "kernels": kernels}
    with open(out_path, "w") as f:
        json.dump(doc, f, indent=1)
    return doc


def ingest_pair(fetch_csv, write_csv):
    import csv
    from collections import defaultdict

    copy_bytes = float(1 << 32)

    def per_kernel(path):
        agg = defaultdict(list)
        for r in csv.DictReader(open(path)):
            agg[r["Kernel_Name"]].append(float(r["Counter_Value"]) * 1024.0)
        return agg

    fetch, write = per_kernel(fetch_csv), per_kernel(write_csv)

    # The calibration copy is the copy dispatch that writes 2^32 bytes (the
    # write counter reads a plain copy exactly); the input restores of the
    # in-place legs are copies of other sizes.  Both runs dispatch the same
    # kernels in the same order, so the fetch run's copies pair up by index.
    fc = [v for name, vs in fetch.items() if "copyBuffer" in name for v in vs]
    wc = [v for name, vs in write.items() if "copyBuffer" in name for v in vs]
    if len(fc) != len(wc):
        raise SystemExit("copy dispatches differ between the FETCH_SIZE and WRITE_SIZE runs")
    sel = [i for i, w in enumerate(wc) if abs(w / copy_bytes - 1.0) < 0.02]
    if not sel:
        raise SystemExit("no plain-copy dispatch of 2^32 bytes in the WRITE_SIZE run")
    fscale = sum(fc[i] for i in sel) / len(sel) / copy_bytes
    wscale = sum(wc[i] for i in sel) / len(sel) / copy_bytes
    kernels = {}
    for name in fetch:
        if "tpd::k_batched" in name and name in write:
            kernels[name] = batched_traffic(name, fetch[name], write[name], fscale, wscale)
            continue
        if "tpd::k_sweep" not in name or name not in write:
            continue
        if "k_sweep<tpd::Real<double>" in name:
            dt, es = "r64", 8
        elif "k_sweep<tpd::Real<float>" in name:
            dt, es = "r32", 4
        elif "k_sweep<double" in name:
            dt, es = "c128", 16
        else:
            dt, es = "c64", 8
        # layout template arguments: MAT -> MID (sweep 1), MID -> CAN (sweep 2),
        # MAT -> MAT in place (both), MAT -> real canonical weights (sweep 2)
        sweeps = {", 0, 2, false>": 1, ", 2, 1, false>": 2, ", 0, 0, false>": 12, ", 0, 3, false>": 2}
        which = sweeps.get(next((k for k in sweeps if k in name), ""), 0)
        if not which:
            continue  # 12: matrix layout in place, both sweeps share the symbol
        # the profiled legs split an even n into two sweeps of n/2 levels,
        # each with tiles of 2^(n/2) rows: n = 2 x the tile's row bits
        m = re.search(r"Geom<(\d+),", name)
        if not m:
            continue
        n = 2 * int(m.group(1))
        alg = 4 ** n * es
        fr = [v / fscale / alg for v in fetch[name]]
        wr = [v / wscale / alg for v in write[name]]
        # Each dispatch is one of: a whole sweep of the general mode (its
        # fetch ratio near the symbol's largest); a chunk of the chunked order
        # (1/2^k of a sweep, k >= 2), counted per whole sweep; or a sweep of
        # the Hermitian / real-symmetric mode, which shares the symbol and
        # reads about half (1.06 against 2.0 for tiles whose runs are shorter
        # than a line).  The entry takes the whole sweeps, else the chunks,
        # else (flagged) the reduced-mode sweeps.
        if len(fr) != len(wr) or not fr:
            continue
        top = max(fr)
        cls, kexp = [], []
        for r in fr:
            k = round(math.log2(1.0 / r)) if r > 0 else 0
            if r >= 0.75 and r >= 0.75 * top:
                cls.append("full")
            elif k >= 2 and abs(r * 2 ** k - 1.0) < 0.05:
                cls.append("chunk")
            else:
                cls.append("reduced")
            kexp.append(k)
        full = [i for i, c in enumerate(cls) if c == "full"]
        chunk = [i for i, c in enumerate(cls) if c == "chunk"]
        reduced = [i for i, c in enumerate(cls) if c == "reduced"]
        use = full or chunk or reduced
        scale = [2 ** kexp[i] if cls[i] == "chunk" else 1 for i in range(len(fr))]
        fo = sum(fr[i] * scale[i] for i in use) / len(use)
        wo = sum(wr[i] * scale[i] for i in use) / len(use)
        e = {
            "n": n, "sweep": which, "dtype": dt, "dispatches": len(use),
            "fetch_bytes": fo * alg, "write_bytes": wo * alg, "total_bytes": (fo + wo) * alg,
            "algorithmic_bytes": 2 * alg, "fetch_over_algorithmic": fo, "write_over_algorithmic": wo,
        }
        if use is chunk:
            e["chunks"] = sorted({2 ** kexp[i] for i in chunk})
            e["per"] = "whole sweep (the chunked order's dispatches summed over its chunks)"
        elif chunk:
            e["chunked_dispatches"] = {"count": len(chunk), "chunks": sorted({2 ** kexp[i] for i in chunk}),
                                       "fetch_over_algorithmic": sum(fr[i] * scale[i] for i in chunk) / len(chunk),
                                       "write_over_algorithmic": sum(wr[i] * scale[i] for i in chunk) / len(chunk)}
        if use is reduced:
            e["only_reduced_mode_dispatches"] = True  # Hermitian / real-symmetric mode only
        elif reduced:
            e["reduced_mode_dispatches"] = {
                "count": len(reduced),
                "fetch_over_algorithmic": sum(fr[i] for i in reduced) / len(reduced),
                "write_over_algorithmic": sum(wr[i] for i in reduced) / len(reduced),
            }
        kernels[name] = e
    return kernels, fscale, wscale



def batched_elements():
    """Coefficients of the 4096-matrix mixed set (n uniform in 2..9, seed 4)."""
    import workloads as W

    return int(sum(4 ** int(v) for v in W.batched_qubits(4096, seed=4)))


def batched_traffic(name, fetch, write, fscale, wscale):
    """PMC bytes per dispatch of the batched kernel on the 4096-matrix set
    (every dispatch of the profiled run decomposes the whole set)."""
    es = 16 if "k_batched<double" in name else (4 if "Real<float>" in name else 8)
    alg = batched_elements() * es
    fb = sum(fetch) / len(fetch) / fscale
    wb = sum(write) / len(write) / wscale
    return {"workload": "batched 4096 matrices, n in 2..9", "dispatches": len(fetch), "fetch_bytes": fb,
            "write_bytes": wb, "total_bytes": fb + wb, "algorithmic_bytes": 2 * alg,
            "fetch_over_algorithmic": fb / alg, "write_over_algorithmic": wb / alg}


def timed_steps(fn, steps, warmup, torch):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1000.0 / steps


def kernel_avgs(plan):
    ms, cnt = plan.timing(reset=True)
    return [m / c if c else 0.0 for m, c in zip(ms, cnt)], cnt


def event_ms(torch, fn, reps):
    """Median over reps of fn's device time (events on the current stream)."""
    fn()
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        fn()
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1))
    return sorted(ts)[len(ts) // 2]


TUNE = True  # cleared by --no-autotune
SCHED_KEYS = ("xb", "db", "r", "grid", "tile_elems", "threads", "in", "out")


def _sched(desc):
    return [{k: w[k] for k in SCHED_KEYS} for w in desc["sweeps"]]


def sweep_rates(alg, avgs, chunk_bits):
    """Per-sweep rate (bytes of one sweep / its average time).  In the
    chunked order the plan times the whole chunk loop (both sweeps) as
    kernel 0: its entry is then the average over the two sweeps."""
    if chunk_bits:
        return [2 * alg / (avgs[0] / 1e3) / 1e9 if avgs and avgs[0] else None, None]
    return [alg / (a / 1e3) / 1e9 if a else None for a in avgs]


def single_matrix_run(tpd, torch, A, n, dtype_code, steps, warmup, esize, in_place=False, layout="canonical",
                      tune=True, hermitian=False, prune=True):
    out = A.view(-1) if in_place else torch.empty(4 ** n, dtype=A.dtype, device=A.device)
    tuned = None
    if tune and TUNE:
        # pick the schedule by measurement on these buffers (outside the timed
        # region; in place this transforms A repeatedly)
        tuned = tpd.autotune(A, out, layout=layout, prune=prune, hermitian=hermitian).get("chosen")
    plan = tpd.Plan(n, dtype_code, timing=True, in_place=in_place, layout=layout, hermitian=hermitian, prune=prune)
    ms = timed_steps(lambda: plan.execute(A, out), steps, warmup, torch)
    avgs, cnt = kernel_avgs(plan)
    desc = plan.describe()
    plan.close()
    alg = 2 * 4 ** n * esize
    res = {
        "ms_per_step": ms,
        "coeffs_per_s": 4 ** n / (ms / 1e3),
        "algorithmic_GBps": alg / (ms / 1e3) / 1e9,
        "kernel_ms": avgs,
        "kernel_launches": cnt,
        "sweeps": len(desc["sweeps"]),
        "chunk_bits": desc.get("chunk_bits", 0), "chunk_window": desc.get("chunk_window", 0),
        "schedule": _sched(desc),
        "autotuned": tuned,
    }
    # per-sweep rate: achieved where every tile is read and written, an
    # effective (bytes of the dense transform) rate where the Hermitian mode
    # skips tiles (pruned legs rename it themselves)
    res["effective_GBps" if hermitian else "sweep_GBps"] = sweep_rates(alg, avgs, res["chunk_bits"])
    res["pct_peak_algorithmic"] = 100.0 * res["algorithmic_GBps"] / PEAK_HBM_GBPS
    return res, out


def inplace_steps(tpd, torch, A0, B, n, dtype_code, steps, warmup, hermitian=False):
    """Autotune on B (unless --no-autotune), then `steps` timed in-place
    decompositions of B (matrix layout) after `warmup` untimed ones, B
    restored from A0 before each (untimed).  Returns (per-step ms list,
    kernel averages, launch counts, plan description, tuner choice)."""
    flat = B.view(-1)
    tuned = None
    if TUNE:
        B.copy_(A0)
        tuned = tpd.autotune(B, flat, layout="matrix", hermitian=hermitian).get("chosen")
    plan = tpd.Plan(n, dtype_code, timing=True, in_place=True, layout="matrix", hermitian=hermitian)
    times = []
    for step in range(warmup + steps):
        if step == warmup:
            plan.timing(reset=True)
        B.copy_(A0)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        plan.execute(B, flat)
        e1.record()
        torch.cuda.synchronize()
        if step >= warmup:
            times.append(e0.elapsed_time(e1))
    avgs, cnt = kernel_avgs(plan)
    desc = plan.describe()
    plan.close()
    return times, avgs, cnt, desc, tuned


def real_weights_run(tpd, torch, W, A0, B, n, steps, warmup, ms_complex_mode, ms_general):
    """Real weights of the Hermitian A0 into a separate real array
    (tpd_decompose_hermitian_real): B, holding the complex Hermitian mode's
    weights in the matrix layout, gives the reference on 10^5 sampled
    strings, then serves as the first sweep's workspace (restored from A0
    before each step, untimed)."""
    import numpy as np

    qs = torch.from_numpy(W.sampled_strings(n, 100000, seed=163).astype(np.int64))
    h, l = deinterleave(qs.numpy())
    ref = B[torch.from_numpy(h).to("cuda"), torch.from_numpy(l).to("cuda")].real.clone()
    rdt = torch.float64 if A0.dtype == torch.complex128 else torch.float32
    out = torch.empty(4 ** n, dtype=rdt, device="cuda")
    tuned = None
    if TUNE:
        B.copy_(A0)
        tuned = tpd.autotune_hermitian_real(B, out).get("chosen")
    ts = []
    for step in range(warmup + steps):
        B.copy_(A0)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        tpd.decompose_hermitian_real(B, out)
        e1.record()
        torch.cuda.synchronize()
        if step >= warmup:
            ts.append(e0.elapsed_time(e1))
    ms = sum(ts) / len(ts)
    same = bool(torch.equal(out[qs.to("cuda")], ref))
    del out, ref
    return {"ms_per_step": ms, "ms_min": min(ts), "coeffs_per_s": 4 ** n / (ms / 1e3),
            "speedup_vs_complex_hermitian_mode": ms_complex_mode / ms, "speedup_vs_c128_general": ms_general / ms,
            "bitwise_equal_to_complex_mode_real_parts_on_samples": same, "samples": int(qs.numel()),
            "autotuned": tuned}


def inplace_run(tpd, torch, A0, n, dtype_code, steps, warmup, esize, hermitian=False):
    """In-place decomposition (matrix layout) of a copy of A0 on one buffer;
    returns (result dict, the buffer holding the last step's weights)."""
    B = torch.empty_like(A0)
    times, avgs, cnt, desc, tuned = inplace_steps(tpd, torch, A0, B, n, dtype_code, steps, warmup, hermitian)
    ms = sum(times) / len(times)
    alg = 2 * 4 ** n * esize
    res = {
        "ms_per_step": ms,
        "ms_min": min(times),
        "coeffs_per_s": 4 ** n / (ms / 1e3),
        "algorithmic_GBps": alg / (ms / 1e3) / 1e9,
        "kernel_ms": avgs,
        "kernel_launches": cnt,
        "sweeps": len(desc["sweeps"]),
        "chunk_bits": desc.get("chunk_bits", 0), "chunk_window": desc.get("chunk_window", 0),
        "schedule": _sched(desc),
        "autotuned": tuned,
    }
    # the Hermitian mode reads and writes fewer bytes than the dense
    # transform: its per-sweep figure is an effective rate, not HBM traffic
    res["effective_GBps" if hermitian else "sweep_GBps"] = sweep_rates(alg, avgs, res["chunk_bits"])
    res["pct_peak_algorithmic"] = 100.0 * res["algorithmic_GBps"] / PEAK_HBM_GBPS
    return res, B


def headline_run(tpd, torch, A0, n, steps, warmup, allocations):
    """The headline: K = steps timed in-place steps spread over
    `allocations` successive allocations of the in-place buffer (each freed
    before the next is taken, so the driver may place it elsewhere in
    physical memory); every allocation autotunes on its own buffer and runs
    `warmup` untimed steps first.  Returns (per-allocation results, the last
    buffer, holding the weights of A0).  At least one step per allocation:
    fewer steps than allocations use fewer allocations."""
    allocations = max(1, min(allocations, steps))
    per = [steps // allocations + (1 if k < steps % allocations else 0) for k in range(allocations)]
    runs, B = [], None
    for k in range(allocations):
        if B is not None:
            del B
            torch.cuda.empty_cache()
        B = torch.empty_like(A0)
        times, avgs, cnt, desc, tuned = inplace_steps(tpd, torch, A0, B, n, tpd.TPD_C128, per[k], warmup)
        runs.append({"steps": per[k], "ms_mean": sum(times) / len(times), "ms_min": min(times),
                     "ms_max": max(times), "kernel_ms": avgs, "kernel_launches": cnt,
                     "chunk_bits": desc.get("chunk_bits", 0), "chunk_window": desc.get("chunk_window", 0),
                     "schedule": _sched(desc), "autotuned": tuned,
                     "buffer_address": int(B.data_ptr())})
        log(f"main: allocation {k}: {runs[-1]['ms_mean']:.3f} ms/step over {per[k]} steps, kernels {avgs}")
    return runs, B


def rel_err(got, ref, a_max):
    """max over components of |got - ref| / max|a_ij|."""
    import numpy as np

    d = np.asarray(got, np.complex128) - np.asarray(ref, np.complex128)
    if d.size == 0:
        return 0.0
    return float(np.max(np.abs(np.concatenate([d.real.ravel(), d.imag.ravel()])))) / a_max


def a_max_of(torch, A):
    m = 0.0
    rows = max(1, (1 << 26) // A.shape[1])
    for r0 in range(0, A.shape[0], rows):
        blk = A[r0:r0 + rows]
        m = max(m, float((torch.view_as_real(blk) if blk.is_complex() else blk).abs().max()))
    return m


def sum_sq(torch, X):
    """sum |x|^2 over a large tensor in binary64, by row blocks (no
    full-size temporaries)"""
    t = 0.0
    rows = max(1, (1 << 26) // X.shape[1])
    for r0 in range(0, X.shape[0], rows):
        blk = X[r0:r0 + rows]
        t += float((torch.view_as_real(blk) if blk.is_complex() else blk).double().square().sum())
    return t


def parseval_rel(torch, A, B, n):
    """|2^n sum |w|^2 - ||A||_F^2| / ||A||_F^2 for the weights B (any layout)"""
    fro = sum_sq(torch, A)
    return abs(sum_sq(torch, B) * 2 ** n - fro) / fro


def deinterleave(q):
    """canonical q -> (row h, column l) of the matrix layout"""
    import numpy as np

    q = np.asarray(q, np.int64)
    h = np.zeros_like(q)
    l = np.zeros_like(q)
    for b in range(20):
        l |= ((q >> (2 * b)) & 1) << b
        h |= ((q >> (2 * b + 1)) & 1) << b
    return h, l


def sampled_reference(torch, A, n, qs, threads):
    """The oracle's definition at sampled strings of a device matrix: the
    entries each X/Y mask needs are gathered on the device, the per-mask
    sums run on host threads."""
    import numpy as np

    from oracle import oracle as O

    flat = A.view(-1)
    i = torch.arange(1 << n, device=A.device, dtype=torch.int64)

    def fetch(ms):
        xs = torch.from_numpy(np.asarray(ms, np.int64)).to(A.device)
        idx = ((i[None, :] ^ xs[:, None]) << n) + i[None, :]
        return flat[idx.reshape(-1)].to(torch.complex128).reshape(len(ms), -1).cpu().numpy()

    return O.sampled_weights(fetch, n, qs, threads=threads, masks_per_fetch=256)


def host_threads():
    try:
        cpus = len(os.sched_getaffinity(0))
    except AttributeError:
        cpus = os.cpu_count() or 1
    return max(1, min(cpus, int(os.environ.get("OMP_NUM_THREADS", cpus))))


def cpu_info():
    import subprocess

    info = {"nproc": None, "affinity_cpus": None, "lscpu": {}}
    try:
        info["nproc"] = int(subprocess.run(["nproc"], capture_output=True, text=True).stdout.strip())
    except Exception:
        pass
    try:
        info["affinity_cpus"] = len(os.sched_getaffinity(0))
    except AttributeError:
        pass
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True).stdout
        for ln in out.splitlines():
            k, _, v = ln.partition(":")
            if k.strip() in ("Model name", "Socket(s)", "Core(s) per socket", "Thread(s) per core", "CPU(s)",
                             "NUMA node(s)"):
                info["lscpu"][k.strip()] = v.strip()
    except Exception:
        pass
    return info


def cpu_baseline(torch, budget_s=20.0):
    """The oracle timed on the host: Algorithm 2 on all host threads (OpenMP,
    bitwise the serial form) on an n = 14 sample of the headline's
    distribution (dense Hermitian, complex Gaussian G), plus Algorithm 1 on
    one thread and Algorithm 2 on all threads at n = 12.  Bounded: about
    budget_s of CPU time in total."""
    from oracle import oracle as O
    import workloads as W

    th = host_threads()
    res = {"kind": "oracle", "unit": "coeffs/s", "cores": th, "host": cpu_info()}

    def rate(fn, n, min_s):
        reps, t0 = 0, time.perf_counter()
        while True:
            fn()
            reps += 1
            el = time.perf_counter() - t0
            if el >= min_s:
                return reps * 4 ** n / el, reps, el

    A12 = W.gaussian_device(12, seed=5, hermitian=True).cpu().numpy()
    r1, k1, e1 = rate(lambda: O.tpd_recursive(A12), 12, 0.2 * budget_s)
    r2, k2, e2 = rate(lambda: O.tpd_iterative_mt(A12, th), 12, 0.15 * budget_s)
    del A12
    A14 = W.gaussian_device(14, seed=5, hermitian=True).cpu().numpy()
    r3, k3, e3 = rate(lambda: O.tpd_iterative_mt(A14, th), 14, 0.5 * budget_s)
    del A14
    res["value"] = r3
    res["sample"] = (f"oracle Algorithm 2 (level-synchronous, OpenMP on {th} host threads, binary64) on a dense "
                     f"Hermitian n=14 matrix of the headline's distribution, {k3} run(s) in {e3:.1f} s; no n=16 "
                     f"figure is extrapolated")
    res["legs"] = {
        "alg1_recursive_1thread_n12": {"coeffs_per_s": r1, "runs": k1, "seconds": e1, "threads": 1},
        "alg2_openmp_n12": {"coeffs_per_s": r2, "runs": k2, "seconds": e2, "threads": th},
        "alg2_openmp_n14": {"coeffs_per_s": r3, "runs": k3, "seconds": e3, "threads": th,
                            "level_sweep_GBps": 2 * 14 * 4 ** 14 * 16 / (e3 / k3) / 1e9},
    }
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=16)
    ap.add_argument("--allocations", type=int, default=3,
                    help="successive allocations of the headline's in-place buffer the timed steps are spread over")
    ap.add_argument("--samples", type=int, default=100000,
                    help="sampled strings (plus the forced ones) checked against the oracle at n=16")
    ap.add_argument("--extras", default="n8,n12,n14,batched,fp32,hermitian,outofplace,real,synth,partial,n14dense",
                    help="comma list of n8,n12,n14,batched,fp32,hermitian,outofplace,real,synth,partial,n14dense,"
                         "n17, or 'none'")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--legs-only", action="store_true",
                    help="skip the n=16 headline and its legs (profiling runs of the other configurations)")
    ap.add_argument("--no-batched-baseline", action="store_true",
                    help="batched leg without the graph of 4096 per-matrix launches (profiling runs)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="use the schedules already chosen (TPD_AUTOTUNE_CACHE) instead of timing candidates")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain device copy of known size (counter calibration)")
    ap.add_argument("--ingest-pmc", nargs="+", metavar="CSV",
                    help="write profiles/traffic.json from pairs of rocprofv3 --pmc counter CSVs "
                         "(FETCH_SIZE, WRITE_SIZE, ...) and exit")
    args = ap.parse_args()
    global TUNE
    TUNE = not args.no_autotune
    if args.ingest_pmc:
        if len(args.ingest_pmc) % 2:
            raise SystemExit("--ingest-pmc takes FETCH_SIZE/WRITE_SIZE CSV pairs")
        pairs = list(zip(args.ingest_pmc[0::2], args.ingest_pmc[1::2]))
        doc = ingest_pmc(pairs, os.path.join(ROOT, "profiles", "traffic.json"))
        print(json.dumps(doc, indent=1))
        return

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: this build runs on one GPU only; --gpus must be 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from oracle import oracle as O
    from paper_2310_13421_amd import tpd
    import workloads as W

    extras = set() if args.extras == "none" else set(args.extras.split(","))
    torch.cuda.set_device(0)
    threads = host_threads()
    n = args.n
    steps_x = max(3, min(args.steps, 10))
    errors = {}
    if args.copy_calibration:
        nbytes = 1 << 32
        src = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        src.fill_(1.0)
        torch.cuda.synchronize()
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy calibration: 3 copies of {nbytes} bytes")
        del src, dst
        torch.cuda.empty_cache()

    result = {"metric": METRIC, "legs_only": True}
    if not args.legs_only:
        log(f"generating n={n} Hermitian complex128 input on the GPU")
        A = W.gaussian_device(n, seed=5, hermitian=True)
        torch.cuda.synchronize()


        # ---- headline -----------------------------------------------------------
        log(f"main: n={n} complex128 in place (matrix layout), {args.steps} timed steps over {args.allocations} "
            f"buffer allocations ({args.warmup} warmup each), input restored before each step")
        runs, B = headline_run(tpd, torch, A, n, args.steps, args.warmup, max(1, args.allocations))
        order = sorted(range(len(runs)), key=lambda k: runs[k]["ms_mean"])
        med = runs[order[len(order) // 2]]
        ms_step = med["ms_mean"]
        alg_bytes = 2 * 4 ** n * 16  # one complex128 read + one write per coefficient
        a_max = a_max_of(torch, A)

        # config 4 check, complex128: sampled strings against the definition
        qs = W.sampled_strings(n, args.samples, seed=5)
        log(f"oracle: {qs.size} sampled strings of the n={n} matrix on {threads} host threads")
        t0 = time.perf_counter()
        bf = sampled_reference(torch, A, n, qs, threads)
        oracle_s = time.perf_counter() - t0
        h, l = deinterleave(qs.astype(np.int64))
        hb, lb = torch.from_numpy(h).to("cuda"), torch.from_numpy(l).to("cuda")
        got128 = B[hb, lb].cpu().numpy()
        errors["config4_n16_hermitian"] = {
            "samples": int(qs.size), "c128": rel_err(got128, bf, a_max),
            "c128_bound_n_u": n * 2.0 ** -53, "oracle_seconds": oracle_s,
            "c128_parseval_rel": parseval_rel(torch, A, B, n),
            "what": "max |w_gpu - w_oracle| / max|a_ij| over uniformly sampled strings plus I..I, X..X, Y..Y, Z..Z, "
                    "4^16-1; in place, matrix layout; parseval_rel = |2^n sum|w|^2 - ||A||_F^2| / ||A||_F^2 over "
                    "all 4^16 weights",
        }
        del B
        torch.cuda.empty_cache()

        # attainable-bandwidth context on this device: a plain device-to-device
        # copy of 4 GiB (torch copy_), median of 5, read + write bytes / time
        csrc = torch.empty(1 << 29, dtype=torch.float64, device="cuda")
        cdst = torch.empty_like(csrc)
        csrc.fill_(1.0)
        copy_ms = event_ms(torch, lambda: cdst.copy_(csrc), 5)
        copy_gbps = 2 * csrc.numel() * 8 / (copy_ms / 1e3) / 1e9
        del csrc, cdst
        torch.cuda.empty_cache()
        log(f"plain copy on this device: {copy_gbps:.0f} GB/s")

        avgs = med["kernel_ms"]
        k = max(range(len(avgs)), key=lambda i: avgs[i])
        chunked = med["chunk_bits"] > 0
        # bytes per launch of the timed kernel: one sweep moves 2 * 4^n * 16 B
        # (with the chunked order the plan times the whole chunk loop, both sweeps)
        launch_bytes = alg_bytes * (2 if chunked else 1)
        achieved = launch_bytes / (avgs[k] / 1e3) / 1e9
        kname = sweep_kernel_name("double", med["schedule"], k + 1)
        tr_doc = load_traffic(kname, n)
        roofline = {
            "bound": "hbm",
            "kernel": (f"k_sweep (sweep {k + 1} of 2): {kname}" if not chunked else f"k_sweep chunk loop: {kname}"),
            "achieved": achieved,
            "peak": PEAK_HBM_GBPS,
            "unit": "GB/s",
            "frac": achieved / PEAK_HBM_GBPS,
            "traffic": tr_doc["total_bytes"] if tr_doc else None,
            "kernel_ms_per_launch": avgs[k],
            "algorithmic_bytes_per_launch": launch_bytes,
            "method_achieved": alg_bytes / (ms_step / 1e3) / 1e9,
            "method_frac": alg_bytes / (ms_step / 1e3) / 1e9 / PEAK_HBM_GBPS,
            "method_note": "2 * 4^n * 16 B (one read and one write per coefficient) / ms_per_step / peak: the two "
                           "sweeps move twice these bytes",
        }

        result = {
            "metric": METRIC,
            "value": 4 ** n / (ms_step / 1e3),
            "unit": "coeffs/s",
            "n_gpus": 1,
            "steps": args.steps,
            "warmup": args.warmup,
            "ms_per_step": ms_step,
            "higher_is_better": True,
            "scaling": "weak",
            "vs_baseline": None,
            "dtype": "f64",
            "data": "synthetic",
            "config": {
                "workload": f"dense Hermitian {2 ** n}x{2 ** n} complex128 (n={n}), A=(G+G^H)/2, G complex N(0,1) "
                            f"seed 5; in place (coefficients in the matrix layout), input restored from a pristine "
                            f"copy before each timed step (untimed), pruning on; {args.steps} timed steps over "
                            f"{len(runs)} successive buffer allocations, value = the median allocation",
                "n": n,
                "precision": "complex128",
                "layout": "matrix",
                "placement": "in-place",
            },
            "allocations": {
                "ms_per_step": [r["ms_mean"] for r in runs],
                "min": runs[order[0]]["ms_mean"], "median": ms_step, "max": runs[order[-1]]["ms_mean"],
                "runs": runs,
            },
            "hbm_GBps_algorithmic": alg_bytes / (ms_step / 1e3) / 1e9,
            "pct_peak_algorithmic": 100.0 * alg_bytes / (ms_step / 1e3) / 1e9 / PEAK_HBM_GBPS,
            "sweeps": len(med["schedule"]),
            "kernel_ms": avgs,
            "sweep_GBps": [alg_bytes / (a / 1e3) / 1e9 if a else None for a in avgs] if not chunked else None,
            "schedule": med["schedule"],
            "autotuned": med["autotuned"],
            "roofline": roofline,
            "torch_copy_GBps_same_device": copy_gbps,
            "frac_of_copy": achieved / copy_gbps,
        }

        # ---- n = 16 complex64 (config 4, FP32 path) ----------------------------
        if "fp32" in extras:
            log("extra: complex64 (round-to-nearest copy of the same matrix), in place")
            A32 = A.to(torch.complex64)
            r, B32 = inplace_run(tpd, torch, A32, n, tpd.TPD_C64, args.steps, args.warmup, 8)
            r["speedup_vs_c128"] = ms_step / r["ms_per_step"]
            got64 = B32[hb, lb].cpu().numpy()
            e64 = rel_err(got64, bf, a_max)
            errors["config4_n16_hermitian"]["c64"] = e64
            errors["config4_n16_hermitian"]["c64_bound_n_plus_1_u"] = (n + 1) * 2.0 ** -24
            errors["config4_n16_hermitian"]["c64_parseval_rel"] = parseval_rel(torch, A32, B32, n)
            r["max_abs_err_over_max_abs_a"] = e64
            result["fp32"] = r
            del B32
            torch.cuda.empty_cache()
            if "hermitian" in extras:
                r, B32 = inplace_run(tpd, torch, A32, n, tpd.TPD_C64, args.steps, args.warmup, 8, hermitian=True)
                r["speedup_vs_c128_general"] = ms_step / r["ms_per_step"]
                result["hermitian_c64"] = r
                log("extra: Hermitian real weights into a separate float32 array, complex64")
                result["hermitian_c64_real_weights"] = real_weights_run(tpd, torch, W, A32, B32, n, args.steps,
                                                                        args.warmup, r["ms_per_step"], ms_step)
                del B32
                torch.cuda.empty_cache()
            if "outofplace" in extras:
                r, o32 = single_matrix_run(tpd, torch, A32, n, tpd.TPD_C64, args.steps, args.warmup, 8)
                result["fp32_out_of_place_canonical"] = r
                del o32
            del A32
            torch.cuda.empty_cache()

        if extras & {"synth", "partial"}:
            coeffs = tpd.decompose(A)
            torch.cuda.synchronize()
            if "synth" in extras:
                log("extra: synthesis A = sum w_t sigma^t from the n=16 weights, complex128")
                M = torch.empty((2 ** n, 2 ** n), dtype=A.dtype, device="cuda")
                ms = event_ms(torch, lambda: tpd.synthesize(coeffs, M), steps_x)
                err_num = 0.0
                for r0 in range(0, 2 ** n, 2048):  # chunked: no full-size temporaries
                    err_num = max(err_num, float((M[r0:r0 + 2048] - A[r0:r0 + 2048]).abs().max()))
                result["synthesis_c128"] = {
                    "ms_per_step": ms, "coeffs_per_s": 4 ** n / (ms / 1e3),
                    "algorithmic_GBps": 2 * 2 * 4 ** n * 16 / (ms / 1e3) / 1e9,
                    "round_trip_max_abs_err_over_max_abs_a": err_num / a_max,
                }
                total = torch.zeros(1, dtype=torch.int64, device="cuda")
                cms = event_ms(torch, lambda: tpd.lib.tpd_compact(coeffs.data_ptr(), n, tpd.TPD_C128, 0, 0.0, None, None,
                                                                  0, total.data_ptr(), None), steps_x)
                result["compact_count_dense_c128"] = {
                    "ms": cms, "read_GBps": 4 ** n * 16 / (cms / 1e3) / 1e9, "kept": int(total.item()),
                }
                del M
                torch.cuda.empty_cache()
            if "partial" in extras:
                log("extra: partial decomposition of the n=16 matrix, all 1- and 2-local strings")
                qs2 = {0}
                for i in range(n):
                    for a in (1, 2, 3):
                        qs2.add(a << (2 * (n - 1 - i)))
                        for j in range(i + 1, n):
                            for b in (1, 2, 3):
                                qs2.add((a << (2 * (n - 1 - i))) | (b << (2 * (n - 1 - j))))
                req = torch.tensor(sorted(qs2), dtype=torch.int64, device="cuda")
                vals = torch.empty(req.numel(), dtype=A.dtype, device="cuda")
                ms = event_ms(torch, lambda: tpd.decompose_partial(A, req, vals, work=coeffs), steps_x)
                full_ms = event_ms(torch, lambda: tpd.decompose(A, coeffs), steps_x)
                result["partial_2local_c128"] = {
                    "requests": int(req.numel()), "ms": ms, "full_out_of_place_ms": full_ms,
                    "speedup_vs_full": full_ms / ms,
                }
            del coeffs
            torch.cuda.empty_cache()

        if "hermitian" in extras:
            log("extra: Hermitian mode (representatives only, real weights), complex128, in place")
            r, B = inplace_run(tpd, torch, A, n, tpd.TPD_C128, args.steps, args.warmup, 16, hermitian=True)
            r["speedup_vs_general"] = ms_step / r["ms_per_step"]
            result["hermitian_c128"] = r
            log("extra: Hermitian real weights into a separate float64 array, complex128")
            result["hermitian_c128_real_weights"] = real_weights_run(tpd, torch, W, A, B, n, args.steps,
                                                                     args.warmup, r["ms_per_step"], ms_step)
            del B
            torch.cuda.empty_cache()
        if "outofplace" in extras:
            log("extra: out of place, canonical order, complex128")
            r, o = single_matrix_run(tpd, torch, A, n, tpd.TPD_C128, args.steps, args.warmup, 16)
            result["out_of_place_canonical_c128"] = r
            del o
            torch.cuda.empty_cache()
        if "real" in extras:
            log("extra: real input (float64 and float32, real-coded weights): Re A, a real-symmetric matrix, in place")
            Ar = A.real.contiguous()
            d = {}
            for name, herm in (("general", False), ("symmetric_mode", True)):
                r, Bb = inplace_run(tpd, torch, Ar, n, tpd.TPD_R64, args.steps, args.warmup, 8, hermitian=herm)
                r["speedup_vs_c128_general"] = ms_step / r["ms_per_step"]
                d[name] = r
                del Bb
                torch.cuda.empty_cache()
            result["real_r64"] = d
            Ar32 = Ar.to(torch.float32)
            del Ar
            torch.cuda.empty_cache()
            d = {}
            for name, herm in (("general", False), ("symmetric_mode", True)):
                r, Bb = inplace_run(tpd, torch, Ar32, n, tpd.TPD_R32, args.steps, args.warmup, 4, hermitian=herm)
                r["speedup_vs_c128_general"] = ms_step / r["ms_per_step"]
                d[name] = r
                del Bb
                torch.cuda.empty_cache()
            result["real_r32"] = d
            del Ar32
            torch.cuda.empty_cache()
        del A
        torch.cuda.empty_cache()

    # ---- config 0: n = 8 dense Gaussian (and integer entries) --------------
    if "n8" in extras:
        log("extra: n=8 dense complex Gaussian (launch-latency bound), both precisions")
        n8 = 8
        A8 = W.gaussian(n8, seed=1)
        ref8 = O.tpd_recursive(A8)
        am8 = float(np.max(np.abs(np.concatenate([A8.real.ravel(), A8.imag.ravel()]))))
        Z8 = W.integer(n8, seed=1)
        refz = O.tpd_recursive(Z8)
        d = {}
        e = {}
        for name, dt in (("c128", torch.complex128), ("c64", torch.complex64)):
            Ad = torch.from_numpy(A8).to("cuda").to(dt)
            o = torch.empty(4 ** n8, dtype=dt, device="cuda")
            ms = event_ms(torch, lambda: tpd.decompose(Ad, o), 50)
            got = o.cpu().numpy()
            e[name] = rel_err(got, ref8, am8)
            if name == "c128":
                e["c128_bitwise_vs_algorithm_1"] = bool(np.array_equal(got.real, ref8.real) and
                                                        np.array_equal(got.imag, ref8.imag))
            gz = tpd.decompose(torch.from_numpy(Z8).to("cuda").to(dt)).cpu().numpy().astype(np.complex128)
            e[name + "_integer_bit_exact"] = bool(np.array_equal(gz, refz))
            d[name] = {"ms": ms, "coeffs_per_s": 4 ** n8 / (ms / 1e3)}
        e["strings"] = 4 ** n8
        errors["config0_n8"] = e
        result["n8"] = d
    # ---- config 1: n = 12 dense Hermitian ----------------------------------
    if "n12" in extras:
        log("extra: n=12 dense Hermitian, both precisions (MALL-sized: GB/s indicative)")
        n12 = 12
        H = W.gaussian_device(n12, seed=2, hermitian=True)
        Hh = H.cpu().numpy()
        ref12 = O.tpd_iterative_mt(Hh, threads)
        am12 = float(np.max(np.abs(np.concatenate([Hh.real.ravel(), Hh.imag.ravel()]))))
        fro = float(np.sum(np.abs(Hh) ** 2))
        d = {}
        e = {"strings": 4 ** n12}
        for name, dt, es in (("c128", torch.complex128, 16), ("c64", torch.complex64, 8)):
            Hd = H if dt == torch.complex128 else H.to(dt)
            o = torch.empty(4 ** n12, dtype=dt, device="cuda")
            if TUNE:
                tpd.autotune(Hd, o)
            ms = event_ms(torch, lambda: tpd.decompose(Hd, o), 20)
            got = o.cpu().numpy()
            e[name] = rel_err(got, ref12, am12)
            oh = tpd.decompose(Hd, hermitian=True).cpu().numpy()
            e[name + "_hermitian_mode_imag_exactly_zero"] = bool(np.all(oh.imag == 0))
            e[name + "_parseval_rel"] = abs(float(np.sum(np.abs(got.astype(np.complex128)) ** 2)) * 2 ** n12 - fro) / fro
            d[name] = {"ms": ms, "coeffs_per_s": 4 ** n12 / (ms / 1e3),
                       "algorithmic_GBps": 2 * 4 ** n12 * es / (ms / 1e3) / 1e9}
        e["c128_bitwise_vs_algorithm_2"] = bool(e["c128"] == 0.0)
        errors["config1_n12_hermitian"] = e
        result["n12"] = d
        del H, Hh
        torch.cuda.empty_cache()

    if "n14dense" in extras:
        log("extra: n=14 dense Hermitian, complex128 and complex64, out of place and in place")
        n14 = 14
        H = W.gaussian_device(n14, seed=14, hermitian=True)
        d = {}
        for name, dt, code, es in (("c128", torch.complex128, tpd.TPD_C128, 16),
                                   ("c64", torch.complex64, tpd.TPD_C64, 8)):
            Hd = H if dt == torch.complex128 else H.to(dt)
            r, o = single_matrix_run(tpd, torch, Hd, n14, code, args.steps, args.warmup, es)
            d[name] = r
            del o
            r, Bb = inplace_run(tpd, torch, Hd, n14, code, args.steps, args.warmup, es)
            d[name + "_in_place"] = r
            del Bb, Hd
            torch.cuda.empty_cache()
        d["fp32_speedup_in_place"] = d["c128_in_place"]["ms_per_step"] / d["c64_in_place"]["ms_per_step"]
        result["n14_dense"] = d
        del H
        torch.cuda.empty_cache()
    # ---- config 2: n = 14 structured Hamiltonian ---------------------------
    if "n14" in extras:
        log("extra: n=14 Heisenberg chain + 200 4-local strings, pruning, both precisions")
        n14 = 14
        terms = W.heisenberg_terms(n14, seed=3, n_local=200)
        H = W.dense_from_terms_device(terms, n14)
        amh = a_max_of(torch, H)
        qsd = torch.tensor([W.string_index(s_) for s_, _ in terms], dtype=torch.int64, device="cuda")
        exp = torch.zeros(4 ** n14, dtype=torch.complex128, device="cuda")
        exp.index_put_((qsd,), torch.tensor(np.array([c for _, c in terms], np.complex128), device="cuda"),
                       accumulate=True)
        r, o = single_matrix_run(tpd, torch, H, n14, tpd.TPD_C128, args.steps, args.warmup, 16)
        r["effective_GBps"] = r.pop("sweep_GBps")  # pruned tiles move no bytes: an effective rate
        plan = tpd.Plan(n14)
        plan.execute(H, o)
        st = plan.prune_stats()
        plan.close()
        r["live_tile_fraction"] = st["live_tiles"] / st["total_tiles"]
        r["live_prefixes_level"] = st["prefix_level"]
        r["live_prefixes"] = st["live_prefixes"]
        e = {"strings": 4 ** n14, "what": "max |w_gpu - w_generating| / max|a_ij| over all 4^14 strings (zeros "
                                          "where no term was generated)"}
        e["c128"] = float(torch.view_as_real(o - exp).abs().max()) / amh
        rn, o2 = single_matrix_run(tpd, torch, H, n14, tpd.TPD_C128, steps_x, 1, 16, tune=False, prune=False)
        r["ms_per_step_no_prune"] = rn["ms_per_step"]
        r["speedup_from_pruning"] = rn["ms_per_step"] / r["ms_per_step"]
        del o2
        q, w, total = tpd.compact(o)
        cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
        cms = event_ms(torch, lambda: tpd.lib.tpd_compact(o.data_ptr(), n14, tpd.TPD_C128, 0, 0.0, q.data_ptr(),
                                                          w.data_ptr(), total, cnt.data_ptr(), None), steps_x)
        _, _, total_tol = tpd.compact(o, tol=1e-12, capacity=0)
        r["sparse_list"] = {"pairs": total, "compact_ms": cms, "pairs_above_1e-12": total_tol}
        del o, q, w
        H32 = H.to(torch.complex64)
        r32, o32 = single_matrix_run(tpd, torch, H32, n14, tpd.TPD_C64, args.steps, args.warmup, 8)
        r32["effective_GBps"] = r32.pop("sweep_GBps")
        e["c64"] = float(torch.view_as_real(o32.to(torch.complex128) - exp).abs().max()) / amh
        r["c64"] = r32
        errors["config2_n14_structured"] = e
        result["n14_structured"] = r
        del H, H32, o32, exp
        torch.cuda.empty_cache()

    # ---- config 3: batched -------------------------------------------------
    if "batched" in extras:
        log("extra: batched 4096 matrices, n in 2..9")
        ns = [int(v) for v in W.batched_qubits(4096, seed=4)]
        bres = {"count": len(ns), "elements": int(sum(4 ** v for v in ns))}
        e = {}
        check_idx = list(range(0, len(ns), 16))
        refs = {}  # oracle weights of the complex128 matrices (the complex64 set is their rounding)
        for name, dt, code, es in (("c128", torch.complex128, tpd.TPD_C128, 16),
                                   ("c64", torch.complex64, tpd.TPD_C64, 8)):
            buf, mats = W.batched_matrices_packed(ns, seed=4, dtype=dt)
            outs = [torch.empty(4 ** v, dtype=dt, device="cuda") for v in ns]
            plan = tpd.BatchedPlan(ns, code, timing=True)
            dp = tpd.BatchedPlan.pointer_table(mats)
            do = tpd.BatchedPlan.pointer_table(outs)
            plan.execute(dp, do)
            torch.cuda.synchronize()
            plan.timing(reset=True)
            btuned = plan.autotune(dp, do) if TUNE else None
            plan.timing(reset=True)
            ms_eager = timed_steps(lambda: plan.execute(dp, do), args.steps, args.warmup, torch)
            kavg, _ = kernel_avgs(plan)
            plan_g = tpd.BatchedPlan(ns, code)  # takes the tuned grid as its default
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g):
                plan_g.execute(dp, do)
            ms_graph = timed_steps(lambda: g.replay(), args.steps, args.warmup, torch)
            # baseline: the same 4096 decompositions as single-matrix calls,
            # captured in one graph (per-matrix launches, no host overhead);
            # the no-allocation entry point keeps the capture free of hipMalloc
            ms_pm = ms_loop = None
            same = None
            outs2 = []
            if not args.no_batched_baseline:
                outs2 = [torch.empty(4 ** v, dtype=dt, device="cuda") for v in ns]
                for m_, o_ in zip(mats, outs2):
                    tpd.decompose_noalloc(m_, o_)
                torch.cuda.synchronize()
                g2 = torch.cuda.CUDAGraph()
                with torch.cuda.graph(g2):
                    for m_, o_ in zip(mats, outs2):
                        tpd.decompose_noalloc(m_, o_)
                ms_pm = timed_steps(lambda: g2.replay(), max(3, steps_x), 1, torch)

                def loop():
                    for m_, o_ in zip(mats, outs2):
                        tpd.decompose(m_, o_)

                ms_loop = timed_steps(loop, 2, 1, torch)
                same = all(torch.equal(torch.view_as_real(a_), torch.view_as_real(b_)) for a_, b_ in zip(outs, outs2))
                del g2
            errs = []
            for i in check_idx:
                if i not in refs:
                    Mh = mats[i].cpu().numpy().astype(np.complex128)
                    refs[i] = (O.tpd_recursive(Mh),
                               float(np.max(np.abs(np.concatenate([Mh.real.ravel(), Mh.imag.ravel()])))))
                ref, am = refs[i]
                errs.append(rel_err(outs[i].cpu().numpy(), ref, am))
            e[name] = max(errs)
            bytes_ = 2 * bres["elements"] * es
            bres[name] = {
                "graph_ms": ms_graph,
                "mats_per_s": len(ns) / (ms_graph / 1e3),
                "eager_ms": ms_eager,
                "kernel_ms": kavg[0],
                "kernel_GBps": bytes_ / (kavg[0] / 1e3) / 1e9,
                "kernel_frac_of_peak": bytes_ / (kavg[0] / 1e3) / 1e9 / PEAK_HBM_GBPS,
                "per_matrix_graph_ms": ms_pm,
                "per_matrix_graph_mats_per_s": len(ns) / (ms_pm / 1e3) if ms_pm else None,
                "speedup_vs_per_matrix_graph": ms_pm / ms_graph if ms_pm else None,
                "per_matrix_python_loop_ms": ms_loop,
                "batched_equals_per_matrix": same,
                "autotuned": btuned,
                "plan": plan_g.describe(),
                "traffic": load_traffic(f"void tpd::k_batched<{'double' if dt == torch.complex128 else 'float'}, 1, "
                                        f"{12 if dt == torch.complex128 else 13}>(tpd::BatchArgs)", None),
                "algorithmic_GBps": bytes_ / (ms_graph / 1e3) / 1e9,
            }
            plan.close()
            plan_g.close()
            del mats, outs, outs2, g, buf
            torch.cuda.empty_cache()
        e["matrices_checked"] = len(check_idx)
        e["what"] = "max over every 16th matrix of max |w_gpu - w_oracle| / max|a_ij| of that matrix"
        errors["config3_batched"] = e
        result["batched"] = bres

    if "n17" in extras:
        log("extra: n=17 (131072 x 131072): real float32 in place with restores")
        R = W.gaussian_device(17, seed=17, dtype=torch.float32, hermitian=True)  # 64 GiB, real symmetric
        r, Bb = inplace_run(tpd, torch, R, 17, tpd.TPD_R32, args.steps, args.warmup, 4)
        result["n17_r32"] = r
        del Bb, R
        torch.cuda.empty_cache()

    # PMC-measured HBM bytes per launch of each sweep, for the general-mode
    # two-sweep legs whose kernels were profiled on the current sources
    legs = [(result.get("out_of_place_canonical_c128"), "double", n), (result.get("fp32"), "float", n),
            (result.get("fp32_out_of_place_canonical"), "float", n),
            ((result.get("real_r64") or {}).get("general"), "tpd::Real<double>", n),
            ((result.get("real_r32") or {}).get("general"), "tpd::Real<float>", n)]
    legs += [((result.get("n14_dense") or {}).get(k), dt, 14)
             for k, dt in (("c128", "double"), ("c128_in_place", "double"), ("c64", "float"), ("c64_in_place", "float"))]
    for r, dt, nn in legs:
        if r is not None:
            r["traffic_bytes"] = leg_traffic(dt, r, nn)
    result["errors"] = errors

    if not args.no_cpu_baseline:
        log("cpu baseline: oracle on the host")
        result["cpu_baseline"] = cpu_baseline(torch)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
