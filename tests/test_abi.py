"""Host-side checks of the C ABI (no GPU): the library loads, exports every
function include/tpd.h declares, validates arguments before touching a
device, and its host helpers and schedule planner behave as documented."""
import ctypes
import json
import os
import re
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tpd.h")

tpd = pytest.importorskip("paper_2310_13421_amd.tpd")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(tpd_[a-z_0-9]+)\s*\(", text)))


def test_every_declared_symbol_is_exported():
    names = declared_functions()
    assert len(names) >= 20
    lib = ctypes.CDLL(tpd.LIB_PATH)
    for name in names:
        assert hasattr(lib, name), name
    # and the binding declares a signature for each of them
    assert set(names) == set(tpd._SIGS)


def test_status_strings_and_limits():
    for code, name in tpd.STATUS.items():
        assert tpd.lib.tpd_status_string(code).decode() == name
    # complex128 stops at 16 (one n = 17 matrix would take 256 GiB); the
    # 8- and 4-byte dtypes reach 17
    assert tpd.max_qubits(tpd.TPD_C128) == 16
    assert tpd.max_qubits(tpd.TPD_C64) == 17
    assert tpd.max_qubits(tpd.TPD_R64) == 17
    assert tpd.max_qubits(tpd.TPD_R32) == 17
    assert tpd.lib.tpd_max_qubits(7) == -1


def test_index_helpers():
    assert tpd.index_from_string("XZ") == 7
    assert tpd.index_from_string("ZX") == 13
    assert tpd.index_from_string("YX") == 9
    assert tpd.index_from_string("I" * 16) == 0
    assert tpd.index_from_string("Z" * 16) == 4 ** 16 - 1
    u64max = 2 ** 64 - 1
    assert tpd.index_from_string("") == u64max
    assert tpd.index_from_string("XQ") == u64max
    assert tpd.index_from_string("X" * 33) == u64max
    for q, n in ((0, 1), (7, 2), (9, 2), (4 ** 16 - 1, 16), (123456789, 16)):
        s = tpd.string_from_index(q, n)
        assert len(s) == n and tpd.index_from_string(s) == q
    buf = ctypes.create_string_buffer(3)
    assert tpd.lib.tpd_string_from_index(16, 2, buf, 3) != 0  # q >= 4^n
    assert tpd.lib.tpd_string_from_index(1, 4, buf, 3) != 0   # buffer too small


FAKE = 0x100000  # never dereferenced: validation fails or the device check stops first


@pytest.mark.parametrize("args,code", [
    ((None, 4, FAKE, 0, 0), 1),            # NULL A
    ((FAKE, 4, None, 0, 0), 1),            # NULL coeffs
    ((FAKE + 8, 4, FAKE * 4, 0, 0), 1),    # misaligned complex128
    ((FAKE, 4, FAKE * 4 + 4, 1, 0), 1),    # misaligned complex64
    ((FAKE, 4, FAKE + 16, 0, 0), 1),       # partial overlap
    ((FAKE, 17, FAKE * 64, 0, 0), 2),      # n too large
    ((FAKE, -1, FAKE * 4, 0, 0), 2),       # n negative
    ((FAKE, 4, FAKE * 4 + 4, 2, 0), 1),    # misaligned real float64
    ((FAKE, 4, FAKE + 8, 2, 0), 1),        # partial overlap, real (8-byte elements)
    ((FAKE, 18, FAKE * 64, 2, 0), 2),      # n too large, real
    ((FAKE, 18, FAKE * 64, 1, 0), 2),      # n too large, complex64
    ((FAKE, 10, FAKE, 2, 0), 2),           # real, in place canonical
    ((FAKE, 4, FAKE * 4 + 2, 3, 0), 1),    # misaligned real float32
    ((FAKE, 4, FAKE + 4, 3, 0), 1),        # partial overlap, real float32 (4-byte elements)
    ((FAKE, 4, FAKE * 4, 5, 0), 1),        # bad dtype
    ((FAKE, 4, FAKE * 4, 0, 0x100), 1),    # unknown flag
    ((FAKE, 8, FAKE, 0, 0), 2),            # in place, canonical, n > 6
    ((FAKE, 10, FAKE, 0, 0), 2),           # in place, canonical, two sweeps
])
def test_decompose_validation_before_device(args, code):
    A, n, C, dt, fl = args
    assert tpd.lib.tpd_decompose_ex(A, n, C, dt, fl, None) == code
    # the no-allocation entry point validates the same way
    assert tpd.lib.tpd_decompose_noalloc(A, n, C, dt, fl, None) == code


def test_hermitian_real_validation_before_device():
    H = tpd.lib.tpd_decompose_hermitian_real
    assert H(None, 4, FAKE * 4, 0, 0, None) == 1                 # NULL A
    assert H(FAKE, 4, None, 0, 0, None) == 1                     # NULL weights
    assert H(FAKE, 4, FAKE * 4, 2, 0, None) == 1                 # real dtypes have no such mode
    assert H(FAKE, 4, FAKE * 4, 3, 0, None) == 1
    assert H(FAKE, 4, FAKE * 4, 0, tpd.FLAG_HERMITIAN, None) == 1  # only TPD_FLAG_NO_PRUNE
    assert H(FAKE, 4, FAKE * 4, 0, tpd.FLAG_LAYOUT_MATRIX, None) == 1
    assert H(FAKE + 8, 4, FAKE * 4, 0, 0, None) == 1             # misaligned complex128 matrix
    assert H(FAKE, 4, FAKE * 4 + 4, 0, 0, None) == 1             # misaligned binary64 weights
    assert H(FAKE, 4, FAKE + 4096 - 8, 0, 0, None) == 1          # weights overlap the matrix's end
    assert H(FAKE, 4, FAKE - 2048 + 8, 0, 0, None) == 1          # matrix starts inside the weights
    assert H(FAKE, 17, FAKE * 64, 0, 0, None) == 2               # n too large
    assert H(FAKE, -1, FAKE * 4, 0, 0, None) == 2
    T = tpd.lib.tpd_autotune_hermitian_real  # validates the same way
    assert T(FAKE, 4, FAKE * 4, 2, 0, None, None, 0) == 1
    assert T(FAKE, 4, FAKE + 4096 - 8, 0, 0, None, None, 0) == 1
    assert T(FAKE, 17, FAKE * 64, 0, 0, None, None, 0) == 2
    D = tpd.lib.tpd_debug_decompose_hermitian_real_tuned
    assert D(FAKE, 4, FAKE * 4, 0, 0, 4, -1, None) == 1                 # negative grid
    assert D(FAKE, 4, FAKE * 4, 0, tpd.FLAG_HERMITIAN, 4, 0, None) == 1


def test_noalloc_rejects_timing_flag():
    assert tpd.lib.tpd_decompose_noalloc(FAKE, 4, FAKE * 4, 0, tpd.FLAG_TIMING, None) == 1


def test_partial_and_compact_validation():
    P = tpd.lib.tpd_decompose_partial
    assert P(FAKE, 4, FAKE * 4, FAKE * 8, 0, FAKE * 16, 0, 0, None) == 0      # nothing requested: no-op
    assert P(FAKE, 4, FAKE * 4, None, 5, FAKE * 16, 0, 0, None) == 1          # NULL requests
    assert P(FAKE, 4, FAKE * 4, FAKE * 8, 5, None, 0, 0, None) == 1           # NULL values
    assert P(FAKE, 4, FAKE * 4, FAKE * 8 + 4, 5, FAKE * 16, 0, 0, None) == 1  # misaligned requests
    assert P(FAKE, 4, FAKE * 4, FAKE * 8, 5, FAKE * 16, 0, 0x4, None) == 1    # timing flag
    assert P(FAKE, 17, FAKE * 64, FAKE * 8, 5, FAKE * 16, 0, 0, None) == 2    # n too large
    assert P(FAKE, 10, FAKE, FAKE * 8, 5, FAKE * 16, 0, 0, None) == 2         # in place canonical
    C = tpd.lib.tpd_compact
    assert C(FAKE, 4, 0, 0, -1.0, FAKE * 2, FAKE * 4, 8, FAKE * 8, None) == 1           # negative tol
    assert C(FAKE, 4, 0, 0, float("nan"), FAKE * 2, FAKE * 4, 8, FAKE * 8, None) == 1   # NaN tol
    assert C(FAKE, 4, 0, 0x1, 0.0, FAKE * 2, FAKE * 4, 8, FAKE * 8, None) == 1          # flag
    assert C(FAKE, 4, 0, 0, 0.0, None, FAKE * 4, 8, FAKE * 8, None) == 1                # NULL list
    assert C(FAKE, 4, 0, 0, 0.0, FAKE * 2, FAKE * 4, 8, None, None) == 1                # NULL count
    assert C(FAKE, 17, 0, 0, 0.0, FAKE * 2, FAKE * 4, 8, FAKE * 8, None) == 2           # n too large


def test_real_input_validation():
    # the real dtypes go through the same host validation as the complex ones
    ns = (ctypes.c_int * 2)(3, 10)
    ptrs = (ctypes.c_void_p * 2)(FAKE, FAKE * 2)
    outs = (ctypes.c_void_p * 2)(FAKE * 4, FAKE * 8)
    for R in (tpd.TPD_R64, tpd.TPD_R32):
        assert tpd.lib.tpd_decompose_batched(ptrs, ns, 2, outs, R, 0, None) == 2  # n > 9
        assert tpd.lib.tpd_decompose_batched(ptrs, ns, -1, outs, R, 0, None) == 1
        assert tpd.lib.tpd_decompose_partial(FAKE, 4, FAKE * 4, None, 5, FAKE * 16, R, 0, None) == 1
        assert tpd.lib.tpd_compact(FAKE, 4, R, 0, -1.0, FAKE * 2, FAKE * 4, 8, FAKE * 8, None) == 1
        assert tpd.lib.tpd_synthesize_ex(FAKE, 4, FAKE * 4, R, 0x4, None) == 1
        h = ctypes.c_void_p()
        assert tpd.lib.tpd_plan_create_batched(ns, 2, R, 0, 0, ctypes.byref(h)) == 2
    # the host replays cover the complex dtypes only
    with pytest.raises(tpd.TPDError):
        tpd.emulate(np.zeros((4, 4)), dtype=tpd.TPD_R64)


def test_batched_validation():
    ns = (ctypes.c_int * 2)(3, 10)
    ptrs = (ctypes.c_void_p * 2)(FAKE, FAKE * 2)
    outs = (ctypes.c_void_p * 2)(FAKE * 4, FAKE * 8)
    assert tpd.lib.tpd_decompose_batched(ptrs, ns, 2, outs, 0, 0, None) == 2   # n > 9
    ns2 = (ctypes.c_int * 2)(3, 8)
    assert tpd.lib.tpd_decompose_batched(ptrs, ns2, 2, None, 0, 0, None) == 2  # in place canonical n = 8
    assert tpd.lib.tpd_decompose_batched(ptrs, ns2, -1, outs, 0, 0, None) == 1
    assert tpd.lib.tpd_decompose_batched(None, ns2, 2, outs, 0, 0, None) == 1
    assert tpd.lib.tpd_decompose_batched(ptrs, ns2, 0, outs, 0, 0, None) == 0  # empty batch is a no-op
    assert tpd.lib.tpd_decompose_batched(ptrs, ns2, 2, outs, 7, 0, None) == 1  # unknown dtype


def test_plan_validation():
    h = ctypes.c_void_p()
    assert tpd.lib.tpd_plan_create(17, 0, 0, 0, ctypes.byref(h)) == 2
    assert tpd.lib.tpd_plan_create(4, 9, 0, 0, ctypes.byref(h)) == 1
    assert tpd.lib.tpd_plan_create(4, 0, 0, 0, None) == 1
    assert tpd.lib.tpd_plan_execute(None, FAKE, FAKE * 4, None) == 1
    assert tpd.lib.tpd_plan_destroy(None) == 1
    assert tpd.lib.tpd_plan_num_kernels(None) == -1


@pytest.mark.parametrize("n", range(0, 18))
def test_schedule_shapes(n):
    for dt in (tpd.TPD_C128, tpd.TPD_C64, tpd.TPD_R64, tpd.TPD_R32):
        if n > tpd.max_qubits(dt):
            with pytest.raises(tpd.TPDError):
                tpd.schedule(n, dt)
            continue
        s = tpd.schedule(n, dt)
        es = {tpd.TPD_C128: 16, tpd.TPD_R32: 4}.get(dt, 8)
        assert s["elements"] == 4 ** n
        assert s["algorithmic_bytes"] == 2 * 4 ** n * es
        if n == 0:
            assert s["sweeps"] == []
            continue
        sw = s["sweeps"]
        assert len(sw) == (1 if n <= 8 else 2)
        # the sweeps transform every x bit exactly once
        bits = sorted(b for w in sw for b in range(w["xlo"], w["xlo"] + w["xb"]))
        assert bits == list(range(n))
        for w in sw:
            assert w["tiles"] * w["tile_elems"] == 4 ** n
            assert w["tile_elems"] * es <= 131072  # one workgroup's LDS tile
            assert w["threads"] <= 1024
        if n >= 9:
            assert sw[0]["bitmap"] == "set" and sw[1]["bitmap"] == "check"
            assert sw[0]["out"] == "MID" and sw[1]["in"] == "MID" and sw[1]["out"] == "CAN"
            # coalescing: every run of the first sweep's reads is 2^db elements,
            # >= 128 B (>= 64 B for 4-byte elements when n = 9 caps db at 4)
            assert (1 << sw[0]["db"]) * es >= (128 if es >= 8 or n >= 10 else 64)


def test_schedule_flags():
    s = tpd.schedule(12, tpd.TPD_C128, tpd.FLAG_LAYOUT_MATRIX, in_place=True)
    assert s["in_place"] and s["layout"] == "matrix"
    assert all(w["in"] == "MAT" and w["out"] == "MAT" for w in s["sweeps"])
    s = tpd.schedule(12, tpd.TPD_C128, tpd.FLAG_NO_PRUNE)
    assert not s["prune"] and all(w["bitmap"] == "none" for w in s["sweeps"])
    with pytest.raises(tpd.TPDError):
        tpd.schedule(12, tpd.TPD_C128, 0, in_place=True)


def test_tune_cache_lines_with_and_without_tile_order(tmp_path):
    # the autotune cache's optional last field selects the second sweep's
    # rotated tile order; older lines without it keep the plain order
    cache = tmp_path / "tune.txt"
    cache.write_text("tpd-tune-v2 gfx950 0 0 16 1 1 0 4 4 2 1\n"
                     "tpd-tune-v2 gfx950 0 1 16 1 1 0 6 4 4\n"
                     "tpd-tune-v2 gfx950 0 0 14 0 0 0 3 4 0 1\n"
                     "garbage line\n")
    code = ("import json; from paper_2310_13421_amd import tpd\n"
            "a = tpd.schedule(16, tpd.TPD_C128, tpd.FLAG_LAYOUT_MATRIX, in_place=True)['sweeps']\n"
            "b = tpd.schedule(16, tpd.TPD_C64, tpd.FLAG_LAYOUT_MATRIX, in_place=True)['sweeps']\n"
            "c = tpd.schedule(14, tpd.TPD_C128)['sweeps']\n"
            "d = tpd.schedule(14, tpd.TPD_C128, tpd.FLAG_ROTATE_TILES | tpd.FLAG_NO_PRUNE)['sweeps']\n"
            "print(json.dumps([[(w['db'], w['tile_order']) for w in x] for x in (a, b, c, d)]))\n")
    env = dict(os.environ, TPD_AUTOTUNE_CACHE=str(cache))
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env, cwd=ROOT, timeout=300)
    assert r.returncode == 0, r.stderr
    a, b, c, d = json.loads(r.stdout.strip().splitlines()[-1])
    assert a == [[4, 0], [4, 1]]  # only the second sweep rotates
    assert b == [[6, 0], [6, 0]]
    assert c == [[3, 0], [3, 1]]
    assert d[1][1] == 1


def test_single_hip_runtime_in_process():
    # the library must share torch's HIP runtime (same soname, different file)
    import torch  # noqa: F401
    assert len(tpd._hip_runtimes()) <= 1, tpd._hip_runtimes()
