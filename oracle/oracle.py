"""CPU FP64 oracle for the Tensorized Pauli Decomposition -- TEST INFRASTRUCTURE.

Thin ctypes front end to ``tpd_oracle.c`` (plain C, binary64, no FMA
contraction; single-threaded except the OpenMP form of Algorithm 2 used to
time the CPU baseline).  Only the test-suite, the package smoke check and the
CPU-baseline leg of the benchmark may import this module; the product path
never does.  It shares no code with the HIP library.

Every function follows a passage of Hantzko, Binkowski, Gupta,
"Tensorized Pauli decomposition algorithm" (arXiv:2310.13421):

* ``weight_dense``     -- eq. (PauliDecomposition), literal double sum over
                          Kronecker-product entries (n <= 5).
* ``weight_sparse``    -- the same sum over the single nonzero per row of each
                          string (section "Existing algorithms" recalls the fact).
* ``weight_from_diagonal`` -- as ``weight_sparse`` given only the entries it reads.
* ``tpd_recursive``    -- Fig. 1, Algorithm 1, with live-CMW counts per level.
* ``tpd_iterative``    -- Fig. 1, Algorithm 2 (n expansions, see its C comment).
* ``tpd_iterative_mt`` -- the same on several OpenMP threads (CPU baseline timing).
* ``tpd_partial``      -- Fig. 2, Algorithm 3.
* ``synthesize``       -- eq. (PauliDecomposition) read as a sum of strings.

Index convention: string t_1..t_n (I=0, X=1, Y=2, Z=3, t_1 the first tensor
factor) has canonical index q = sum_k t_k 4^(n-k).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "tpd_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

_CFLAGS = ["-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared"]


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (no FMA contraction, IEEE semantics)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.run(["gcc", *_CFLAGS, "-o", tmp, _SRC, "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _bind(lib):
    P = ctypes.c_void_p
    I = ctypes.c_int
    S = ctypes.c_size_t
    U = ctypes.c_uint64
    lib.oracle_abi_version.restype = I
    lib.oracle_weight_dense.argtypes = [P, I, P, S, P]
    lib.oracle_weight_sparse.argtypes = [P, I, P, S, P]
    lib.oracle_weight_from_diagonal.argtypes = [P, I, U, P, S, P]
    lib.oracle_xy_mask.argtypes = [U, I]
    lib.oracle_xy_mask.restype = U
    lib.oracle_tpd_recursive.argtypes = [P, I, P, P, P]
    lib.oracle_tpd_iterative.argtypes = [P, I, P, P]
    lib.oracle_tpd_iterative_mt.argtypes = [P, I, P, P, I]
    lib.oracle_tpd_partial.argtypes = [P, I, P, S, P]
    lib.oracle_synthesize.argtypes = [P, I, P]
    for name in ("oracle_weight_dense", "oracle_weight_sparse", "oracle_weight_from_diagonal",
                 "oracle_tpd_recursive", "oracle_tpd_iterative", "oracle_tpd_iterative_mt", "oracle_tpd_partial",
                 "oracle_synthesize"):
        getattr(lib, name).restype = I
    return lib


def _load():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
                build()
            _lib = _bind(ctypes.CDLL(_LIB))
    return _lib


def compile_variant(src_text: str, out_path: str):
    """Compile a modified copy of the oracle source (used by the mutation
    test that plants mistakes in the oracle to show the pins catch them)."""
    c_path = out_path + ".c"
    with open(c_path, "w") as f:
        f.write(src_text)
    subprocess.run(["gcc", *_CFLAGS, "-o", out_path, c_path, "-lm"], check=True)
    return _bind(ctypes.CDLL(out_path))


def source_text() -> str:
    with open(_SRC) as f:
        return f.read()


_override = threading.local()


class use_library:
    """Context manager: route this module's functions to another oracle build."""

    def __init__(self, lib):
        self.lib = lib

    def __enter__(self):
        self.prev = getattr(_override, "lib", None)
        _override.lib = self.lib
        return self

    def __exit__(self, *exc):
        _override.lib = self.prev
        return False


def _cur():
    lib = getattr(_override, "lib", None)
    return lib if lib is not None else _load()


def _mat(A: np.ndarray, n: int | None = None):
    A = np.ascontiguousarray(A, dtype=np.complex128)
    if A.ndim != 2 or A.shape[0] != A.shape[1]:
        raise ValueError("expected a square matrix")
    dim = A.shape[0]
    nn = dim.bit_length() - 1
    if (1 << nn) != dim:
        raise ValueError("dimension must be a power of two")
    if n is not None and n != nn:
        raise ValueError("n does not match the matrix")
    return A, nn


def _check(rc: int, what: str):
    if rc != 0:
        raise RuntimeError(f"oracle {what} failed with code {rc}")


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _qs(qs) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(qs, dtype=np.uint64).reshape(-1))


def weight_dense(A: np.ndarray, qs) -> np.ndarray:
    """omega_q = 2^-n tr(sigma^q A) from the full Kronecker definition (n <= 5)."""
    A, n = _mat(A)
    q = _qs(qs)
    out = np.empty(q.size, np.complex128)
    _check(_cur().oracle_weight_dense(_ptr(A), n, _ptr(q), q.size, _ptr(out)), "weight_dense")
    return out


def weight_sparse(A: np.ndarray, qs) -> np.ndarray:
    """omega_q summed over the single nonzero per row of sigma^q."""
    A, n = _mat(A)
    q = _qs(qs)
    out = np.empty(q.size, np.complex128)
    _check(_cur().oracle_weight_sparse(_ptr(A), n, _ptr(q), q.size, _ptr(out)), "weight_sparse")
    return out


def xy_mask(q: int, n: int) -> int:
    """Bit (n-k) set iff letter t_k is X or Y (column offset of sigma^q's nonzeros)."""
    return int(_cur().oracle_xy_mask(int(q), int(n)))


def weight_from_diagonal(v: np.ndarray, n: int, x: int, qs) -> np.ndarray:
    """omega_q for strings sharing X/Y mask x, given v[i] = A[i ^ x][i]."""
    v = np.ascontiguousarray(v, dtype=np.complex128).reshape(-1)
    if v.size != (1 << n):
        raise ValueError("v must hold 2^n entries")
    q = _qs(qs)
    out = np.empty(q.size, np.complex128)
    _check(_cur().oracle_weight_from_diagonal(_ptr(v), n, int(x), _ptr(q), q.size, _ptr(out)),
           "weight_from_diagonal")
    return out


def sampled_weights(fetch_diagonals, n: int, qs, threads: int = 0, masks_per_fetch: int = 256) -> np.ndarray:
    """omega_q for sampled strings of a matrix too large to copy whole, from
    the definition (weight_from_diagonal).  Strings are grouped by X/Y mask x
    (all strings of one mask read the same 2^n entries v[i] = A[i ^ x][i]);
    fetch_diagonals(xs) must return an array [len(xs), 2^n] of those entries
    (e.g. gathered from a device copy of A).  The per-mask sums run on
    `threads` host threads (0: os.cpu_count()); each call is the
    single-threaded C definition, which releases the GIL."""
    from concurrent.futures import ThreadPoolExecutor

    q = _qs(qs)
    masks = np.array([xy_mask(int(v), n) for v in q], np.int64) if q.size < 4096 else _xy_masks(q, n)
    out = np.empty(q.size, np.complex128)
    order = np.argsort(masks, kind="stable")
    ms = masks[order]
    uniq, starts = np.unique(ms, return_index=True)
    ends = np.append(starts[1:], ms.size)
    nth = threads if threads > 0 else (os.cpu_count() or 1)

    def one(args):
        v, x, sel = args
        out[sel] = weight_from_diagonal(v, n, int(x), q[sel])

    with ThreadPoolExecutor(nth) as ex:
        for c0 in range(0, uniq.size, masks_per_fetch):
            xs = uniq[c0:c0 + masks_per_fetch]
            V = np.asarray(fetch_diagonals(xs))
            jobs = [(V[k], x, order[starts[c0 + k]:ends[c0 + k]]) for k, x in enumerate(xs)]
            list(ex.map(one, jobs))
    return out


def _xy_masks(q: np.ndarray, n: int) -> np.ndarray:
    """X/Y masks of many canonical indices at once (bit n-k set iff letter
    t_k is X or Y, i.e. the digit's two bits differ)."""
    q = q.astype(np.uint64)
    x = np.zeros(q.size, np.int64)
    for k in range(1, n + 1):
        d = (q >> np.uint64(2 * (n - k))) & np.uint64(3)
        x |= ((d == 1) | (d == 2)).astype(np.int64) << (n - k)
    return x


def tpd_recursive(A: np.ndarray, with_stats: bool = False):
    """Algorithm 1.  Returns the 4^n weights (canonical order); with_stats adds
    (live CMW counts per level 0..n, complex entries computed)."""
    A, n = _mat(A)
    out = np.empty(1 << (2 * n), np.complex128)
    live = np.zeros(n + 1, np.uint64)
    ops = ctypes.c_uint64(0)
    _check(_cur().oracle_tpd_recursive(_ptr(A), n, _ptr(out), _ptr(live), ctypes.byref(ops)),
           "tpd_recursive")
    if with_stats:
        return out, live.astype(np.int64), int(ops.value)
    return out


def tpd_iterative(A: np.ndarray, with_stats: bool = False):
    """Algorithm 2 (level-synchronous); bitwise equal to tpd_recursive."""
    A, n = _mat(A)
    out = np.empty(1 << (2 * n), np.complex128)
    live = np.zeros(n + 1, np.uint64)
    _check(_cur().oracle_tpd_iterative(_ptr(A), n, _ptr(out), _ptr(live)), "tpd_iterative")
    if with_stats:
        return out, live.astype(np.int64)
    return out


def tpd_iterative_mt(A: np.ndarray, threads: int = 0, with_stats: bool = False):
    """Algorithm 2 on `threads` OpenMP threads (0: all); bitwise equal to
    tpd_iterative.  For timing the CPU baseline."""
    A, n = _mat(A)
    out = np.empty(1 << (2 * n), np.complex128)
    live = np.zeros(n + 1, np.uint64)
    _check(_cur().oracle_tpd_iterative_mt(_ptr(A), n, _ptr(out), _ptr(live), int(threads)), "tpd_iterative_mt")
    if with_stats:
        return out, live.astype(np.int64)
    return out


def tpd_partial(A: np.ndarray, qs) -> np.ndarray:
    """Algorithm 3: only the requested strings, pruning zero CMWs."""
    A, n = _mat(A)
    q = _qs(qs)
    out = np.empty(q.size, np.complex128)
    _check(_cur().oracle_tpd_partial(_ptr(A), n, _ptr(q), q.size, _ptr(out)), "tpd_partial")
    return out


def synthesize(w: np.ndarray, n: int) -> np.ndarray:
    """A = sum_q w_q sigma^q."""
    w = np.ascontiguousarray(w, dtype=np.complex128).reshape(-1)
    if w.size != 1 << (2 * n):
        raise ValueError("w must hold 4^n weights")
    A = np.empty((1 << n, 1 << n), np.complex128)
    _check(_cur().oracle_synthesize(_ptr(w), n, _ptr(A)), "synthesize")
    return A


def index_of(s: str) -> int:
    """'XYZI...' -> canonical index q (first letter = first tensor factor)."""
    q = 0
    for ch in s:
        q = 4 * q + "IXYZ".index(ch)
    return q


def string_of(q: int, n: int) -> str:
    return "".join("IXYZ"[(q >> (2 * (n - k))) & 3] for k in range(1, n + 1))
