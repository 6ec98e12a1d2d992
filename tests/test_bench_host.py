"""Host-side logic of bench.py: PMC ingestion and its calibration, kernel
symbols of a schedule, traffic lookup keyed by source hash, and the
one-GPU guard.  No GPU is used."""
import csv
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402

K1 = "void tpd::k_sweep<double, tpd::Geom<8, 5, 0, 4, 0>, 0, 2, false>(tpd::SweepArgs)"
K2 = "void tpd::k_sweep<double, tpd::Geom<8, 5, 0, 4, 0>, 2, 1, false>(tpd::SweepArgs)"
COPY = "__amd_rocclr_copyBuffer"


def write_csv(path, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Counter_Value"])
        w.writeheader()
        for name, kib in rows:
            w.writerow({"Kernel_Name": name, "Counter_Value": kib})


def test_ingest_scales_by_the_copy_and_keys_by_symbol(tmp_path, monkeypatch):
    alg = 4 ** 16 * 16  # bytes read (or written) by one complex128 sweep at n = 16
    copy = 1 << 32
    # FETCH_SIZE reads half the true bytes, WRITE_SIZE the true bytes
    fetch = [(COPY, 0.5 * copy / 1024), (K1, 0.5 * alg / 1024), (K2, 0.5 * 1.01 * alg / 1024)]
    write = [(COPY, copy / 1024), (K1, alg / 1024), (K2, 1.02 * alg / 1024)]
    f1, w1 = tmp_path / "f.csv", tmp_path / "w.csv"
    write_csv(f1, fetch)
    write_csv(w1, write)
    out = tmp_path / "traffic.json"
    doc = bench.ingest_pmc([(str(f1), str(w1))], str(out))
    assert abs(doc["scales"][0]["fetch_scale"] - 0.5) < 1e-12
    k1, k2 = doc["kernels"][K1], doc["kernels"][K2]
    assert k1["sweep"] == 1 and k2["sweep"] == 2
    assert abs(k1["total_bytes"] - 2 * alg) < 1e-3 * alg
    assert abs(k2["fetch_over_algorithmic"] - 1.01) < 1e-9 and abs(k2["write_over_algorithmic"] - 1.02) < 1e-9
    # lookup: matching sources and n, then a changed source hash
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    os.makedirs(tmp_path / "profiles")
    doc["kernel_source_sha"] = "x"
    with open(tmp_path / "profiles" / "traffic.json", "w") as f:
        json.dump(doc, f)
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "x")
    assert bench.load_traffic(K2, 16)["total_bytes"] == k2["total_bytes"]
    assert bench.load_traffic(K2, 15) is None
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "y")
    assert bench.load_traffic(K2, 16) is None


def test_ingest_calibrates_on_the_2_32_byte_copy_and_splits_reduced_modes(tmp_path):
    # restores of other sizes (in-place legs) must not enter the calibration,
    # and Hermitian / real-symmetric dispatches of a shared symbol are kept
    # apart from the full ones
    copy = 1 << 32
    kr = "void tpd::k_sweep<tpd::Real<float>, tpd::Geom<8, 6, 0, 4, 0>, 0, 0, false>(tpd::SweepArgs)"
    alg = 4 ** 16 * 4  # real float32 sweep bytes read (or written)
    fetch = [(COPY, 0.5 * 4 * copy / 1024), (COPY, 0.5 * copy / 1024), (COPY, 0.5 * 8 * copy / 1024),
             (kr, 0.5 * alg / 1024), (kr, 0.5 * alg / 1024), (kr, 0.5 * 0.5 * alg / 1024), (kr, 0.5 * 0.6 * alg / 1024)]
    write = [(COPY, 4 * copy / 1024), (COPY, copy / 1024), (COPY, 8 * copy / 1024),
             (kr, alg / 1024), (kr, alg / 1024), (kr, 0.5 * alg / 1024), (kr, alg / 1024)]
    f1, w1 = tmp_path / "f.csv", tmp_path / "w.csv"
    write_csv(f1, fetch)
    write_csv(w1, write)
    doc = bench.ingest_pmc([(str(f1), str(w1))], str(tmp_path / "t.json"))
    assert abs(doc["scales"][0]["fetch_scale"] - 0.5) < 1e-12 and doc["scales"][0]["write_scale"] == 1.0
    k = doc["kernels"][kr]
    assert k["dtype"] == "r32" and k["dispatches"] == 2
    assert abs(k["fetch_over_algorithmic"] - 1.0) < 1e-12 and abs(k["write_over_algorithmic"] - 1.0) < 1e-12
    red = k["reduced_mode_dispatches"]
    assert red["count"] == 2 and abs(red["fetch_over_algorithmic"] - 0.55) < 1e-12
    assert abs(red["write_over_algorithmic"] - 0.75) < 1e-12


def test_ingest_splits_reduced_modes_of_tiles_that_fetch_whole_lines(tmp_path):
    # runs shorter than a line: the full mode fetches twice the algorithmic
    # bytes and the reduced mode a little over them; the reduced dispatches
    # are still told apart (they read about half of what the full ones read)
    copy = 1 << 32
    kr = "void tpd::k_sweep<tpd::Real<float>, tpd::Geom<8, 4, 0, 4, 0>, 0, 0, false>(tpd::SweepArgs)"
    alg = 4 ** 16 * 4
    fetch = [(COPY, 0.5 * copy / 1024)] + [(kr, 0.5 * r * alg / 1024) for r in (2.0, 2.0, 1.063, 1.063)]
    write = [(COPY, copy / 1024)] + [(kr, r * alg / 1024) for r in (1.0, 1.0, 0.531, 1.0)]
    f1, w1 = tmp_path / "f.csv", tmp_path / "w.csv"
    write_csv(f1, fetch)
    write_csv(w1, write)
    k = bench.ingest_pmc([(str(f1), str(w1))], str(tmp_path / "t.json"))["kernels"][kr]
    assert k["dispatches"] == 2 and abs(k["fetch_over_algorithmic"] - 2.0) < 1e-12
    assert abs(k["write_over_algorithmic"] - 1.0) < 1e-12
    red = k["reduced_mode_dispatches"]
    assert red["count"] == 2 and abs(red["fetch_over_algorithmic"] - 1.063) < 1e-12


def test_ingest_takes_n_from_the_tile_rows_and_legs_look_it_up(tmp_path, monkeypatch):
    # an n = 14 leg: tiles of 2^7 rows, 4^14 elements per sweep
    copy = 1 << 32
    k14 = "void tpd::k_sweep<double, tpd::Geom<7, 3, 0, 4, 0>, 0, 0, false>(tpd::SweepArgs)"
    alg = 4 ** 14 * 16
    f1, w1 = tmp_path / "f.csv", tmp_path / "w.csv"
    write_csv(f1, [(COPY, 0.5 * copy / 1024), (k14, 0.5 * alg / 1024), (k14, 0.5 * alg / 1024)])
    write_csv(w1, [(COPY, copy / 1024), (k14, 1.001 * alg / 1024), (k14, 1.001 * alg / 1024)])
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    os.makedirs(tmp_path / "profiles")
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "x")
    doc = bench.ingest_pmc([(str(f1), str(w1))], str(tmp_path / "profiles" / "traffic.json"))
    k = doc["kernels"][k14]
    assert k["n"] == 14 and abs(k["fetch_over_algorithmic"] - 1.0) < 1e-12
    assert abs(k["write_over_algorithmic"] - 1.001) < 1e-12
    sched = [{"xb": 7, "db": 3, "r": 4, "in": "MAT", "out": "MAT"}] * 2
    assert bench.leg_traffic("double", {"schedule": sched}, 14) == [k["total_bytes"]] * 2
    assert bench.leg_traffic("double", {"schedule": sched}, 16) == [None, None]
    assert bench.leg_traffic("float", {"schedule": sched}, 14) == [None, None]


def test_ingest_needs_the_copy_calibration(tmp_path):
    f1, w1 = tmp_path / "f.csv", tmp_path / "w.csv"
    write_csv(f1, [(K1, 1.0)])
    write_csv(w1, [(K1, 1.0)])
    with pytest.raises(SystemExit):
        bench.ingest_pmc([(str(f1), str(w1))], str(tmp_path / "t.json"))


def test_kernel_symbol_of_a_schedule():
    sched = [{"xb": 8, "db": 5, "r": 4, "in": "MAT", "out": "MID"}, {"xb": 8, "db": 5, "r": 4, "in": "MID", "out": "CAN"}]
    assert bench.sweep_kernel_name("double", sched, 1) == K1
    assert bench.sweep_kernel_name("double", sched, 2) == K2
    inplace = [{"xb": 8, "db": 4, "r": 4, "in": "MAT", "out": "MAT"}] * 2
    assert bench.sweep_kernel_name("float", inplace, 2) == \
        "void tpd::k_sweep<float, tpd::Geom<8, 4, 0, 4, 0>, 0, 0, false>(tpd::SweepArgs)"


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr


def test_ingest_batched_kernel_against_the_4096_matrix_set(tmp_path):
    # the batched kernel's bytes are compared with the whole set's
    # 2 x sum 4^n x s (every dispatch decomposes all 4096 matrices)
    kb = "void tpd::k_batched<double, 1, 12>(tpd::BatchArgs)"
    copy = 1 << 32
    elems = bench.batched_elements()
    assert elems == sum(4 ** n for n in __import__("workloads").batched_qubits(4096, seed=4))
    alg = elems * 16
    write_csv(tmp_path / "f.csv", [(COPY, 0.5 * copy / 1024), (kb, 0.5 * 1.03 * alg / 1024), (kb, 0.5 * 1.01 * alg / 1024)])
    write_csv(tmp_path / "w.csv", [(COPY, copy / 1024), (kb, alg / 1024), (kb, alg / 1024)])
    doc = bench.ingest_pmc([(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"))], str(tmp_path / "t.json"))
    k = doc["kernels"][kb]
    assert k["dispatches"] == 2 and abs(k["fetch_over_algorithmic"] - 1.02) < 1e-9
    assert abs(k["write_over_algorithmic"] - 1.0) < 1e-9 and abs(k["algorithmic_bytes"] - 2 * alg) < 1


def test_ingest_sums_chunked_dispatches_over_their_chunks(tmp_path):
    # the chunked order launches each sweep once per chunk (here 16 chunks
    # of the n = 14 matrix-layout kernel): its symbol is reported per whole
    # sweep, not as a reduced mode
    k = "void tpd::k_sweep<double, tpd::Geom<7, 3, 0, 4, 0>, 0, 0, false>(tpd::SweepArgs)"
    alg = 4 ** 14 * 16
    copy = 1 << 32
    fetch = [(COPY, 0.5 * copy / 1024)] + [(k, 0.5 * 1.002 * alg / 16 / 1024)] * 32
    write = [(COPY, copy / 1024)] + [(k, 1.001 * alg / 16 / 1024)] * 32
    f1, w1 = tmp_path / "f.csv", tmp_path / "w.csv"
    write_csv(f1, fetch)
    write_csv(w1, write)
    doc = bench.ingest_pmc([(str(f1), str(w1))], str(tmp_path / "t.json"))
    e = doc["kernels"][k]
    assert e["n"] == 14 and e["chunks"] == [16] and e["dispatches"] == 32
    assert abs(e["fetch_over_algorithmic"] - 1.002) < 1e-9 and abs(e["write_over_algorithmic"] - 1.001) < 1e-9
    assert abs(e["total_bytes"] - 2.003 * alg) < 1e-3 * alg
    assert "only_reduced_mode_dispatches" not in e


def test_sweep_rates_of_whole_and_chunked_legs():
    alg = 4 ** 16 * 16
    # whole sweeps: one rate per sweep
    r = bench.sweep_rates(alg, [27.0, 25.0], 0)
    assert abs(r[0] - alg / 27e-3 / 1e9) < 1e-6 and abs(r[1] - alg / 25e-3 / 1e9) < 1e-6
    # chunked: kernel 0 is the whole loop (both sweeps), averaged per sweep
    r = bench.sweep_rates(alg, [52.0, 0.0], 9)
    assert abs(r[0] - 2 * alg / 52e-3 / 1e9) < 1e-6 and r[1] is None


def test_traffic_lookup_ignores_reduced_mode_only_symbols(tmp_path, monkeypatch):
    k = "void tpd::k_sweep<double, tpd::Geom<8, 4, 0, 4, 0>, 0, 0, false>(tpd::SweepArgs)"
    os.makedirs(tmp_path / "profiles")
    doc = {"kernel_source_sha": "x", "kernels": {k: {"n": 16, "total_bytes": 7.3e10,
                                                       "only_reduced_mode_dispatches": True}}}
    with open(tmp_path / "profiles" / "traffic.json", "w") as f:
        json.dump(doc, f)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "x")
    assert bench.load_traffic(k, 16) is None


def test_ingest_mixed_dispatch_kinds_and_merge_keeps_whole_sweeps(tmp_path):
    # one symbol with whole sweeps, chunks of 1/16 and reduced-mode sweeps in
    # one run: the entry is the whole sweeps, the others are listed apart; a
    # later run with reduced-mode sweeps only does not replace it
    k = "void tpd::k_sweep<double, tpd::Geom<8, 4, 0, 4, 0>, 0, 0, false>(tpd::SweepArgs)"
    alg = 4 ** 16 * 16
    copy = 1 << 32
    f1 = [(COPY, 0.5 * copy / 1024)] + [(k, 0.5 * 1.001 * alg / 1024)] * 2 + \
         [(k, 0.5 * alg / 16 / 1024)] * 32 + [(k, 0.5 * 0.53 * alg / 1024)] * 2
    w1 = [(COPY, copy / 1024)] + [(k, 1.002 * alg / 1024)] * 2 + [(k, alg / 16 / 1024)] * 32 + \
         [(k, 0.77 * alg / 1024)] * 2
    f2 = [(COPY, 0.5 * copy / 1024)] + [(k, 0.5 * 0.53 * alg / 1024)] * 2
    w2 = [(COPY, copy / 1024)] + [(k, 0.5 * alg / 1024)] * 2
    paths = []
    for i, rows in enumerate((f1, w1, f2, w2)):
        p = tmp_path / f"{i}.csv"
        write_csv(p, rows)
        paths.append(str(p))
    one = bench.ingest_pmc([(paths[0], paths[1])], str(tmp_path / "a.json"))["kernels"][k]
    assert one["dispatches"] == 2 and abs(one["fetch_over_algorithmic"] - 1.001) < 1e-9
    assert one["chunked_dispatches"]["count"] == 32 and one["chunked_dispatches"]["chunks"] == [16]
    assert one["reduced_mode_dispatches"]["count"] == 2
    both = bench.ingest_pmc([(paths[0], paths[1]), (paths[2], paths[3])], str(tmp_path / "b.json"))["kernels"][k]
    assert both == one
    later = bench.ingest_pmc([(paths[2], paths[3])], str(tmp_path / "c.json"))["kernels"][k]
    assert later["only_reduced_mode_dispatches"]
    # whole sweeps only, then reduced-mode sweeps only: the whole sweeps are
    # kept and the later pair's reduced-mode figures become their sub-record
    # (in either order of the pairs)
    f3 = [(COPY, 0.5 * copy / 1024)] + [(k, 0.5 * 1.001 * alg / 1024)] * 2
    w3 = [(COPY, copy / 1024)] + [(k, 1.002 * alg / 1024)] * 2
    for i, rows in enumerate((f3, w3)):
        p = tmp_path / f"w{i}.csv"
        write_csv(p, rows)
        paths.append(str(p))
    for order in (((paths[4], paths[5]), (paths[2], paths[3])), ((paths[2], paths[3]), (paths[4], paths[5]))):
        m = bench.ingest_pmc(list(order), str(tmp_path / "d.json"))["kernels"][k]
        assert m["dispatches"] == 2 and abs(m["fetch_over_algorithmic"] - 1.001) < 1e-9
        assert "only_reduced_mode_dispatches" not in m
        red = m["reduced_mode_dispatches"]
        assert red["count"] == 2 and abs(red["fetch_over_algorithmic"] - 0.53) < 1e-9
        assert abs(red["write_over_algorithmic"] - 0.5) < 1e-9
