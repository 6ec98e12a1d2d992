#!/usr/bin/env python3
"""Throughput benchmark of the MI355X Tensorized Pauli Decomposition.

Default workload (the largest single-GPU configuration): one dense Hermitian
2^16 x 2^16 matrix, A = (G + G^H)/2 with complex N(0,1) G (seed 5),
complex128, decomposed out of place into its 4^16 canonical Pauli
coefficients.  A step is one full decomposition (bitmap clear + two HBM
sweeps, pruning on).  Inputs are generated on the GPU and resident in HBM
before the timed region.  Prints ONE JSON line.

Extras in the same line: the complex64 run of the same matrix, the same
matrix in place (matrix layout), the n = 14 structured Hamiltonian with
zero-block pruning, the 4096-matrix batched workload (graph replay vs
per-matrix launches), and the CPU oracle timed on the host.

    python bench.py [--gpus 1] [--steps 20] [--warmup 3] [--extras ...]
"""
import argparse
import hashlib
import json
import re
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBPS = 8000.0
METRIC = "Pauli coeffs/sec + HBM GB/s (% peak) at n=14/16, FP64 vs FP32; batched mats/s"
KERNEL_SOURCES = ["paper_2310_13421_amd/csrc/tpd_sweep.h", "paper_2310_13421_amd/csrc/tpd_core.h",
                  "paper_2310_13421_amd/csrc/tpd_internal.h"]


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_source_hash():
    """Hash of the sources of the sweep kernel (its headers and the
    instantiation units), the kernel whose traffic profiles/traffic.json
    records."""
    import glob

    h = hashlib.sha256()
    files = sorted(set(KERNEL_SOURCES) | {os.path.relpath(p, ROOT) for p in glob.glob(
        os.path.join(ROOT, "paper_2310_13421_amd", "csrc", "tpd_sweep_c*.hip"))})
    for rel in files:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def load_traffic(kernel_name, n):
    """HBM bytes per launch measured with rocprofv3 --pmc (FETCH_SIZE and
    WRITE_SIZE scaled by a plain-copy calibration) for this kernel at this
    n, if taken on the current kernel sources."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    if t.get("kernel_source_sha") != kernel_source_hash():
        return None
    k = t.get("kernels", {}).get(kernel_name)
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
    several pairs takes the figures of the last one."""
    kernels, scales = {}, []
    for fetch_csv, write_csv in pairs:
        ks, fs, ws = ingest_pair(fetch_csv, write_csv)
        kernels.update(ks)
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
        which = {", 0, 2, false>": 1, ", 2, 1, false>": 2, ", 0, 0, false>": 12}.get(
            next((k for k in (", 0, 2, false>", ", 2, 1, false>", ", 0, 0, false>") if k in name), ""), 0)
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
        # Hermitian / real-symmetric mode shares the kernel symbol and reads
        # about half of what the full mode reads (1.06 against 2.0 for tiles
        # whose runs are shorter than a line): its dispatches are reported
        # apart from the full ones
        top = max(fr) if fr else 0.0
        full = [i for i, r in enumerate(fr) if r >= 0.75 and r >= 0.75 * top]
        reduced = [i for i in range(len(fr)) if i not in full] if len(fr) == len(wr) and full else []
        use = full if reduced else list(range(len(fr)))
        only_reduced = not full
        fb = sum(fr[i] for i in use) / len(use) * alg
        wb = sum(wr[i] for i in (use if len(wr) == len(fr) else range(len(wr)))) / (
            len(use) if len(wr) == len(fr) else len(wr)) * alg
        kernels[name] = {
            "n": n, "sweep": which, "dtype": dt, "dispatches": len(use),
            "fetch_bytes": fb, "write_bytes": wb, "total_bytes": fb + wb,
            "algorithmic_bytes": 2 * alg, "fetch_over_algorithmic": fb / alg, "write_over_algorithmic": wb / alg,
        }
        if only_reduced:
            kernels[name]["only_reduced_mode_dispatches"] = True  # Hermitian / real-symmetric mode only
        if reduced:
            kernels[name]["reduced_mode_dispatches"] = {
                "count": len(reduced),
                "fetch_over_algorithmic": sum(fr[i] for i in reduced) / len(reduced),
                "write_over_algorithmic": sum(wr[i] for i in reduced) / len(reduced),
            }
    return kernels, fscale, wscale


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


TUNE = True  # cleared by --no-autotune


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
    plan.timing(reset=True)
    desc = plan.describe()
    plan.close()
    sweep_bytes = 2 * 4 ** n * esize
    res = {
        "ms_per_step": ms,
        "coeffs_per_s": 4 ** n / (ms / 1e3),
        "algorithmic_GBps": sweep_bytes / (ms / 1e3) / 1e9,
        "kernel_ms": avgs,
        "kernel_launches": cnt,
        "sweep_GBps": [sweep_bytes / (a / 1e3) / 1e9 if a else None for a in avgs],
        "sweeps": len(desc["sweeps"]),
        "schedule": [{k: w[k] for k in ("xb", "db", "r", "grid", "tile_elems", "threads", "in", "out")}
                     for w in desc["sweeps"]],
        "autotuned": tuned,
    }
    res["pct_peak_algorithmic"] = 100.0 * res["algorithmic_GBps"] / PEAK_HBM_GBPS
    return res, out


def inplace_run(tpd, torch, A0, n, dtype_code, steps, warmup, esize, hermitian=False):
    """In-place decomposition (matrix layout) of a copy of A0, the copy
    restored from A0 before every step outside the timed region (repeated
    in-place transforms would shrink the values towards zero, where pruning
    and subnormals change the work).  Each step is timed with HIP events
    around the decomposition alone."""
    B = torch.empty_like(A0)
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
    ms = sum(times) / len(times)
    sweep_bytes = 2 * 4 ** n * esize
    res = {
        "ms_per_step": ms,
        "ms_min": min(times),
        "coeffs_per_s": 4 ** n / (ms / 1e3),
        "algorithmic_GBps": sweep_bytes / (ms / 1e3) / 1e9,
        "kernel_ms": avgs,
        "kernel_launches": cnt,
        "sweep_GBps": [sweep_bytes / (a / 1e3) / 1e9 if a else None for a in avgs],
        "sweeps": len(desc["sweeps"]),
        "schedule": [{k: w[k] for k in ("xb", "db", "r", "grid", "tile_elems", "threads", "in", "out")}
                     for w in desc["sweeps"]],
        "autotuned": tuned,
    }
    res["pct_peak_algorithmic"] = 100.0 * res["algorithmic_GBps"] / PEAK_HBM_GBPS
    return res, B


def cpu_baseline(tpd, torch, n_sample=13, min_seconds=10.0):
    """The oracle's Algorithm 1 (plain single-threaded C, binary64) on a
    Hermitian matrix of the workload's distribution at n = n_sample; its
    result also gives the GPU path's error on the same matrix."""
    import numpy as np

    from oracle import oracle as O
    import workloads as W

    A = W.gaussian(n_sample, seed=5, hermitian=True)
    reps = 0
    t0 = time.perf_counter()
    while True:
        ref = O.tpd_recursive(A)
        reps += 1
        el = time.perf_counter() - t0
        if el >= min_seconds:
            break
    rate = reps * 4 ** n_sample / el
    a_max = float(np.max(np.abs(np.concatenate([A.real.ravel(), A.imag.ravel()]))))
    errs = {}
    for name, dt in (("c128", torch.complex128), ("c64", torch.complex64)):
        got = tpd.decompose(torch.from_numpy(A).to("cuda").to(dt)).cpu().numpy().astype(np.complex128)
        d = got - ref
        errs[name] = float(np.max(np.abs(np.concatenate([d.real, d.imag])))) / a_max
    errs["c128_bitwise"] = bool(errs["c128"] == 0.0)
    del A, np
    return {
        "value": rate,
        "unit": "coeffs/s",
        "cores": 1,
        "kind": "oracle",
        "sample": (f"oracle Algorithm 1 recursion (single-threaded C, binary64) on a dense Hermitian "
                   f"n={n_sample} matrix of the workload's distribution, {reps} run(s), {el:.1f} s; its cost per "
                   f"coefficient grows with n, so the n=16 rate is about {n_sample}/16 of this"),
        "seconds": el,
        "gpu_max_abs_err_over_max_abs_a": errs,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=16)
    ap.add_argument("--extras", default="synth,partial,hermitian,outofplace,real,fp32,n14dense,n14,batched,n17",
                    help="comma list of synth,partial,hermitian,outofplace,fp32,n14dense,n14,batched, or 'none'")
    ap.add_argument("--no-cpu-baseline", action="store_true")
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

    import torch

    from paper_2310_13421_amd import tpd
    import workloads as W

    extras = set() if args.extras == "none" else set(args.extras.split(","))
    torch.cuda.set_device(0)
    n = args.n
    log(f"generating n={n} Hermitian complex128 input on the GPU")
    A = W.gaussian_device(n, seed=5, hermitian=True)
    torch.cuda.synchronize()

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

    log(f"main: n={n} complex128 in place (matrix layout), {args.warmup} warmup + {args.steps} timed steps, "
        f"input restored before each")
    main_res, B = inplace_run(tpd, torch, A, n, tpd.TPD_C128, args.steps, args.warmup, 16)
    log(f"main: {main_res['ms_per_step']:.3f} ms/step, {main_res['coeffs_per_s']:.3e} coeffs/s, "
        f"kernels {main_res['kernel_ms']}")
    del B
    torch.cuda.empty_cache()

    # attainable-bandwidth context on this device: a plain device-to-device
    # copy of 4 GiB (torch copy_), median of 5, read + write bytes / time
    csrc = torch.empty(1 << 29, dtype=torch.float64, device="cuda")
    cdst = torch.empty_like(csrc)
    csrc.fill_(1.0)
    cdst.copy_(csrc)
    ctimes = []
    for _ in range(5):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        cdst.copy_(csrc)
        e1.record()
        torch.cuda.synchronize()
        ctimes.append(e0.elapsed_time(e1))
    copy_gbps = 2 * csrc.numel() * 8 / (sorted(ctimes)[2] / 1e3) / 1e9
    del csrc, cdst
    torch.cuda.empty_cache()
    log(f"plain copy on this device: {copy_gbps:.0f} GB/s")

    avgs = main_res["kernel_ms"]
    k = max(range(len(avgs)), key=lambda i: avgs[i])
    unit_bytes = 2 * 16  # one complex128 read + one write per coefficient
    achieved = unit_bytes * 4 ** n / (avgs[k] / 1e3) / 1e9
    kname = sweep_kernel_name("double", main_res["schedule"], k + 1)
    tr_doc = load_traffic(kname, n)
    tr = tr_doc["total_bytes"] if tr_doc else None
    roofline = {
        "bound": "hbm",
        "kernel": f"k_sweep (sweep {k + 1} of 2): {kname}",
        "achieved": achieved,
        "peak": PEAK_HBM_GBPS,
        "unit": "GB/s",
        "frac": achieved / PEAK_HBM_GBPS,
        "traffic": tr,
    }

    result = {
        "metric": METRIC,
        "value": main_res["coeffs_per_s"],
        "unit": "coeffs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_res["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"dense Hermitian {2 ** n}x{2 ** n} complex128 (n={n}), A=(G+G^H)/2, G complex N(0,1) "
                        f"seed 5; in place (coefficients in the matrix layout), input restored from a pristine "
                        f"copy before each timed step (untimed), pruning on",
            "n": n,
            "precision": "complex128",
            "layout": "matrix",
            "placement": "in-place",
        },
        "hbm_GBps_algorithmic": main_res["algorithmic_GBps"],
        "pct_peak_algorithmic": main_res["pct_peak_algorithmic"],
        "sweeps": main_res["sweeps"],
        "kernel_ms": main_res["kernel_ms"],
        "sweep_GBps": main_res["sweep_GBps"],
        "schedule": main_res["schedule"],
        "autotuned": main_res["autotuned"],
        "roofline": roofline,
        "torch_copy_GBps_same_device": copy_gbps,
        "frac_of_copy": achieved / copy_gbps,
    }

    steps_x = max(3, min(args.steps, 10))

    def event_ms(fn, reps):
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

    if extras & {"synth", "partial"}:
        coeffs = tpd.decompose(A)
        torch.cuda.synchronize()
        if "synth" in extras:
            log("extra: synthesis A = sum w_t sigma^t from the n=16 weights, complex128")
            M = torch.empty((2 ** n, 2 ** n), dtype=A.dtype, device="cuda")
            ms = event_ms(lambda: tpd.synthesize(coeffs, M), steps_x)
            err_num, a_max = 0.0, 0.0
            for r0 in range(0, 2 ** n, 2048):  # chunked: no full-size temporaries
                err_num = max(err_num, float((M[r0:r0 + 2048] - A[r0:r0 + 2048]).abs().max()))
                a_max = max(a_max, float(A[r0:r0 + 2048].abs().max()))
            err = err_num / a_max
            result["synthesis_c128"] = {
                "ms_per_step": ms, "coeffs_per_s": 4 ** n / (ms / 1e3),
                "algorithmic_GBps": 2 * 2 * 4 ** n * 16 / (ms / 1e3) / 1e9,
                "round_trip_max_rel_err": err,
            }
            # compaction of the dense weights, count only (one read of 4^n values)
            total = torch.zeros(1, dtype=torch.int64, device="cuda")
            cms = event_ms(lambda: tpd.lib.tpd_compact(coeffs.data_ptr(), n, tpd.TPD_C128, 0, 0.0, None, None, 0,
                                                       total.data_ptr(), None), steps_x)
            result["compact_count_dense_c128"] = {
                "ms": cms, "read_GBps": 4 ** n * 16 / (cms / 1e3) / 1e9, "kept": int(total.item()),
            }
            del M
            torch.cuda.empty_cache()
        if "partial" in extras:
            log("extra: partial decomposition of the n=16 matrix, all 1- and 2-local strings")
            qs = {0}
            for i in range(n):
                for a in (1, 2, 3):
                    qs.add(a << (2 * (n - 1 - i)))
                    for j in range(i + 1, n):
                        for b in (1, 2, 3):
                            qs.add((a << (2 * (n - 1 - i))) | (b << (2 * (n - 1 - j))))
            req = torch.tensor(sorted(qs), dtype=torch.int64, device="cuda")
            vals = torch.empty(req.numel(), dtype=A.dtype, device="cuda")
            ms = event_ms(lambda: tpd.decompose_partial(A, req, vals, work=coeffs), steps_x)
            full_ms = event_ms(lambda: tpd.decompose(A, coeffs), steps_x)
            result["partial_2local_c128"] = {
                "requests": int(req.numel()), "ms": ms, "full_out_of_place_ms": full_ms,
                "speedup_vs_full": full_ms / ms,
            }
        del coeffs
        torch.cuda.empty_cache()

    if "hermitian" in extras:
        log("extra: Hermitian mode (representatives only, real weights), complex128, in place")
        r, B = inplace_run(tpd, torch, A, n, tpd.TPD_C128, args.steps, args.warmup, 16, hermitian=True)
        r["speedup_vs_general"] = main_res["ms_per_step"] / r["ms_per_step"]
        result["hermitian_c128"] = r
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
            r, B = inplace_run(tpd, torch, Ar, n, tpd.TPD_R64, args.steps, args.warmup, 8, hermitian=herm)
            r["speedup_vs_c128_general"] = main_res["ms_per_step"] / r["ms_per_step"]
            d[name] = r
            del B
            torch.cuda.empty_cache()
        result["real_r64"] = d
        Ar32 = Ar.to(torch.float32)
        del Ar
        torch.cuda.empty_cache()
        d = {}
        for name, herm in (("general", False), ("symmetric_mode", True)):
            r, B = inplace_run(tpd, torch, Ar32, n, tpd.TPD_R32, args.steps, args.warmup, 4, hermitian=herm)
            r["speedup_vs_c128_general"] = main_res["ms_per_step"] / r["ms_per_step"]
            d[name] = r
            del B
            torch.cuda.empty_cache()
        result["real_r32"] = d
        del Ar32
        torch.cuda.empty_cache()
    if "fp32" in extras:
        log("extra: complex64 (round-to-nearest copy of the same matrix), in place")
        A32 = A.to(torch.complex64)
        del A
        A = None
        torch.cuda.empty_cache()
        r, B32 = inplace_run(tpd, torch, A32, n, tpd.TPD_C64, args.steps, args.warmup, 8)
        r["speedup_vs_c128"] = main_res["ms_per_step"] / r["ms_per_step"]
        result["fp32"] = r
        del B32
        torch.cuda.empty_cache()
        if "hermitian" in extras:
            r, B32 = inplace_run(tpd, torch, A32, n, tpd.TPD_C64, args.steps, args.warmup, 8, hermitian=True)
            r["speedup_vs_c128_general"] = main_res["ms_per_step"] / r["ms_per_step"]
            result["hermitian_c64"] = r
            del B32
            torch.cuda.empty_cache()
        if "outofplace" in extras:
            r, o32 = single_matrix_run(tpd, torch, A32, n, tpd.TPD_C64, args.steps, args.warmup, 8)
            result["fp32_out_of_place_canonical"] = r
            del o32
        del A32
        torch.cuda.empty_cache()
    if A is not None:
        del A
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
            r, B = inplace_run(tpd, torch, Hd, n14, code, args.steps, args.warmup, es)
            d[name + "_in_place"] = r
            del B, Hd
            torch.cuda.empty_cache()
        result["n14_dense"] = d
        del H
        torch.cuda.empty_cache()
    if "n14" in extras:
        log("extra: n=14 Heisenberg chain + 200 4-local strings, pruning")
        n14 = 14
        H = W.dense_from_terms_device(W.heisenberg_terms(n14, seed=3, n_local=200), n14)
        r, o = single_matrix_run(tpd, torch, H, n14, tpd.TPD_C128, args.steps, args.warmup, 16)
        plan = tpd.Plan(n14)
        plan.execute(H, o)
        st = plan.prune_stats()
        plan.close()
        r["live_tile_fraction"] = st["live_tiles"] / st["total_tiles"]
        r["live_prefixes_level"] = st["prefix_level"]
        r["live_prefixes"] = st["live_prefixes"]
        rn, o2 = single_matrix_run(tpd, torch, H, n14, tpd.TPD_C128, steps_x, 1, 16, tune=False, prune=False)
        r["ms_per_step_no_prune"] = rn["ms_per_step"]
        r["speedup_from_pruning"] = rn["ms_per_step"] / r["ms_per_step"]
        # sparse list of the weights (the paper's output form)
        q, w, total = tpd.compact(o)
        cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
        cms = event_ms(lambda: tpd.lib.tpd_compact(o.data_ptr(), n14, tpd.TPD_C128, 0, 0.0, q.data_ptr(), w.data_ptr(),
                                                   total, cnt.data_ptr(), None), steps_x)
        assert int(cnt.item()) == total
        _, _, total_tol = tpd.compact(o, tol=1e-12, capacity=0)
        r["sparse_list"] = {"pairs": total, "compact_ms": cms, "pairs_above_1e-12": total_tol}
        result["n14_structured"] = r
        del H, o, o2
        torch.cuda.empty_cache()

    if "batched" in extras:
        log("extra: batched 4096 matrices, n in 2..9")
        ns = [int(v) for v in W.batched_qubits(4096, seed=4)]
        bres = {"count": len(ns), "elements": int(sum(4 ** v for v in ns))}
        for name, dt, code, es in (("c128", torch.complex128, tpd.TPD_C128, 16),
                                   ("c64", torch.complex64, tpd.TPD_C64, 8)):
            mats = W.batched_matrices_device(ns, seed=4, dtype=dt)
            outs = [torch.empty(4 ** v, dtype=dt, device="cuda") for v in ns]
            plan = tpd.BatchedPlan(ns, code, timing=True)
            dp = tpd.BatchedPlan.pointer_table(mats)
            do = tpd.BatchedPlan.pointer_table(outs)
            s = torch.cuda.Stream()
            s.wait_stream(torch.cuda.current_stream())
            with torch.cuda.stream(s):
                plan.execute(dp, do)
            torch.cuda.current_stream().wait_stream(s)
            torch.cuda.synchronize()
            plan.timing(reset=True)
            btuned = plan.autotune(dp, do)["chosen"] if TUNE else None
            plan.timing(reset=True)
            ms_eager = timed_steps(lambda: plan.execute(dp, do), args.steps, args.warmup, torch)
            kavg, _ = kernel_avgs(plan)
            plan_g = tpd.BatchedPlan(ns, code)  # takes the tuned grid as its default
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g):
                plan_g.execute(dp, do)
            ms_graph = timed_steps(lambda: g.replay(), args.steps, args.warmup, torch)

            def loop():
                for m, o in zip(mats, outs):
                    tpd.decompose(m, o)

            ms_loop = timed_steps(loop, max(2, steps_x // 3), 1, torch)
            bytes_ = 2 * bres["elements"] * es
            bres[name] = {
                "graph_ms": ms_graph,
                "mats_per_s": len(ns) / (ms_graph / 1e3),
                "eager_ms": ms_eager,
                "kernel_ms": kavg[0],
                "kernel_GBps": bytes_ / (kavg[0] / 1e3) / 1e9,
                "per_matrix_launch_loop_ms": ms_loop,
                "per_matrix_mats_per_s": len(ns) / (ms_loop / 1e3),
                "speedup_vs_per_matrix": ms_loop / ms_graph,
                "autotuned": btuned,
                "algorithmic_GBps": bytes_ / (ms_graph / 1e3) / 1e9,
            }
            plan.close()
            plan_g.close()
            del mats, outs, g
            torch.cuda.empty_cache()
        result["batched"] = bres

    if "n17" in extras:
        log("extra: n=17 (131072 x 131072): real float32 in place with restores, complex64 in place once")
        n17 = 17
        d17 = {}
        R = W.gaussian_device(n17, seed=17, dtype=torch.float32, hermitian=True)  # 64 GiB, real symmetric
        r, B = inplace_run(tpd, torch, R, n17, tpd.TPD_R32, args.steps, args.warmup, 4)
        d17["r32"] = r
        del B, R
        torch.cuda.empty_cache()
        # complex64: 128 GiB, no room for a pristine copy.  The autotuner
        # transforms the buffer repeatedly, so the input is generated again
        # before the one timed decomposition (the plan's events).
        C = W.gaussian_device(n17, seed=17, dtype=torch.complex64, hermitian=True)
        tuned17 = tpd.autotune(C, C.view(-1), layout="matrix").get("chosen") if TUNE else None
        del C
        torch.cuda.empty_cache()
        C = W.gaussian_device(n17, seed=17, dtype=torch.complex64, hermitian=True)
        plan = tpd.Plan(n17, tpd.TPD_C64, timing=True, in_place=True, layout="matrix")
        torch.cuda.synchronize()
        plan.execute(C, C.view(-1))
        torch.cuda.synchronize()
        kav, _ = kernel_avgs(plan)
        desc = plan.describe()
        plan.close()
        ms = sum(kav)
        d17["c64_single"] = {
            "ms": ms, "kernel_ms": kav, "coeffs_per_s": 4 ** n17 / (ms / 1e3), "autotuned": tuned17,
            "sweep_GBps": [2 * 4 ** n17 * 8 / (k / 1e3) / 1e9 for k in kav],
            "schedule": [{k: w[k] for k in ("xb", "db", "r", "grid", "tile_elems", "threads")} for w in desc["sweeps"]],
        }
        del C
        torch.cuda.empty_cache()
        result["n17"] = d17

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

    if not args.no_cpu_baseline:
        log("cpu baseline: oracle on the host")
        result["cpu_baseline"] = cpu_baseline(tpd, torch)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
