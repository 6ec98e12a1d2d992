"""ctypes binding of libtpd (the C ABI in include/tpd.h).

Argument marshalling only: every step of the decomposition runs in the HIP
kernels of libtpd.so.  PyTorch supplies device memory and the current HIP
stream.  If the library is missing the import fails loudly; there is no
fallback implementation.
"""
from __future__ import annotations

import ctypes
import json
import os
from typing import List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtpd.so")

TPD_C128 = 0
TPD_C64 = 1
TPD_R64 = 2
TPD_R32 = 3
FLAG_NO_PRUNE = 0x1
FLAG_LAYOUT_MATRIX = 0x2
FLAG_TIMING = 0x4
FLAG_ORDER_BOTTOM = 0x8
FLAG_HERMITIAN = 0x10
FLAG_ROTATE_TILES = 0x20

STATUS = {
    0: "TPD_SUCCESS",
    1: "TPD_ERROR_INVALID_VALUE",
    2: "TPD_ERROR_UNSUPPORTED",
    3: "TPD_ERROR_OUT_OF_MEMORY",
    4: "TPD_ERROR_LAUNCH",
    5: "TPD_ERROR_INTERNAL",
    6: "TPD_ERROR_NO_DEVICE",
}

# every symbol include/tpd.h declares, with (restype, argtypes)
_P = ctypes.c_void_p
_I = ctypes.c_int
_U = ctypes.c_uint
_U64 = ctypes.c_uint64
_SZ = ctypes.c_size_t
_SIGS = {
    "tpd_max_qubits": (_I, [_I]),
    "tpd_decompose": (_I, [_P, _I, _P, _P]),
    "tpd_decompose_ex": (_I, [_P, _I, _P, _I, _U, _P]),
    "tpd_decompose_noalloc": (_I, [_P, _I, _P, _I, _U, _P]),
    "tpd_decompose_hermitian_real": (_I, [_P, _I, _P, _I, _U, _P]),
    "tpd_debug_decompose_hermitian_real_tuned": (_I, [_P, _I, _P, _I, _U, _I, _I, _P]),
    "tpd_autotune_hermitian_real": (_I, [_P, _I, _P, _I, _U, _P, _P, ctypes.c_size_t]),
    "tpd_decompose_batched": (_I, [_P, _P, _I, _P, _I, _U, _P]),
    "tpd_plan_create": (_I, [_I, _I, _U, _I, _P]),
    "tpd_plan_create_batched": (_I, [_P, _I, _I, _U, _I, _P]),
    "tpd_plan_execute": (_I, [_P, _P, _P, _P]),
    "tpd_plan_execute_batched": (_I, [_P, _P, _P, _P]),
    "tpd_plan_destroy": (_I, [_P]),
    "tpd_plan_num_kernels": (_I, [_P]),
    "tpd_plan_timing": (_I, [_P, _P, _P, _I]),
    "tpd_plan_prune_stats": (_I, [_P, _P, _P, _P, _P, _P]),
    "tpd_plan_describe": (_I, [_P, ctypes.c_char_p, _SZ]),
    "tpd_release_workspace": (_I, []),
    "tpd_autotune": (_I, [_P, _I, _P, _I, _U, _P, ctypes.c_char_p, _SZ]),
    "tpd_autotune_batched": (_I, [_P, _P, _P, _P, ctypes.c_char_p, _SZ]),
    "tpd_debug_emulate_tuned": (_I, [_P, _I, _P, _I, _U, _I, _I, _I, _I, _I]),
    "tpd_debug_emulate_hermitian_real": (_I, [_P, _I, _P, _I, _U]),
    "tpd_synthesize_ex": (_I, [_P, _I, _P, _I, _U, _P]),
    "tpd_debug_emulate_synth": (_I, [_P, _I, _P, _I, _U, _I]),
    "tpd_status_string": (ctypes.c_char_p, [_I]),
    "tpd_index_from_string": (_U64, [ctypes.c_char_p]),
    "tpd_string_from_index": (_I, [_U64, _I, ctypes.c_char_p, _SZ]),
    "tpd_schedule_describe": (_I, [_I, _I, _U, _I, ctypes.c_char_p, _SZ]),
    "tpd_debug_emulate": (_I, [_P, _I, _P, _I, _U, _I]),
    "tpd_debug_emulate_batched": (_I, [_P, _P, _I, _P, _I, _U, _P]),
    "tpd_debug_plan_batched_codes": (_I, [_P, _P]),
    "tpd_decompose_partial": (_I, [_P, _I, _P, _P, _U64, _P, _I, _U, _P]),
    "tpd_debug_decompose_tuned": (_I, [_P, _I, _P, _I, _U, _I, _I, _I, _I, _I, _P]),
    "tpd_compact": (_I, [_P, _I, _I, _U, ctypes.c_double, _P, _P, _U64, _P, _P]),
    "tpd_debug_emulate_partial": (_I, [_P, _I, _P, _P, _U64, _P, _I, _U, _I]),
    "tpd_debug_emulate_compact": (_I, [_P, _I, _I, _U, ctypes.c_double, _P, _P, _U64, _P]),
}


class TPDError(RuntimeError):
    def __init__(self, code: int, what: str):
        self.code = code
        super().__init__(f"{what}: {STATUS.get(code, code)}")


def _hip_runtimes():
    try:
        with open("/proc/self/maps") as f:
            return sorted({ln.split()[-1] for ln in f if "libamdhip64" in ln})
    except OSError:
        return []


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libtpd.so not built at {LIB_PATH}; run __graft_entry__.build()")
    # torch ships its own HIP runtime under the same soname.  Loading torch
    # first makes the library bind to that runtime, so device pointers and
    # streams created by torch are valid in it; loaded the other way round
    # the process would hold two runtimes with separate device state.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(LIB_PATH)
    runtimes = _hip_runtimes()
    if len(runtimes) > 1:
        raise ImportError("more than one HIP runtime is loaded in this process: " + ", ".join(runtimes))
    for name, (res, args) in _SIGS.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


lib = _load()


def _check(code: int, what: str):
    if code != 0:
        raise TPDError(code, what)


# ----------------------------------------------------------------------------
# host helpers
# ----------------------------------------------------------------------------
def index_from_string(s: str) -> int:
    return int(lib.tpd_index_from_string(s.encode()))


def string_from_index(q: int, n: int) -> str:
    buf = ctypes.create_string_buffer(n + 1)
    _check(lib.tpd_string_from_index(q, n, buf, n + 1), "tpd_string_from_index")
    return buf.value.decode()


def max_qubits(dtype: int = TPD_C128) -> int:
    return int(lib.tpd_max_qubits(dtype))


def schedule(n: int, dtype: int = TPD_C128, flags: int = 0, in_place: bool = False) -> dict:
    buf = ctypes.create_string_buffer(4096)
    _check(lib.tpd_schedule_describe(n, dtype, flags, int(in_place), buf, 4096), "tpd_schedule_describe")
    return json.loads(buf.value.decode())


def _np_dtype(dtype: int):
    if dtype not in (TPD_C128, TPD_C64):
        raise TPDError(2, "the host replays cover the complex dtypes only")
    return np.complex128 if dtype == TPD_C128 else np.complex64


def emulate_hermitian_real(A: np.ndarray, dtype: int = TPD_C128, prune: bool = True) -> np.ndarray:
    """Host replay of decompose_hermitian_real (A is copied, not modified):
    the real weights in canonical order."""
    work = np.ascontiguousarray(A, dtype=_np_dtype(dtype)).copy()
    n = work.shape[0].bit_length() - 1
    out = np.full(work.size, np.nan, np.float64 if dtype == TPD_C128 else np.float32)  # poison
    _check(lib.tpd_debug_emulate_hermitian_real(work.ctypes.data, n, out.ctypes.data, dtype,
                                                0 if prune else FLAG_NO_PRUNE), "tpd_debug_emulate_hermitian_real")
    return out


def emulate(A: np.ndarray, dtype: int = TPD_C128, flags: int = 0, in_place: bool = False, db: int = 0,
            r: int = 0, chunk_bits: int = 0, chunk_window: int = 0) -> np.ndarray:
    """Host replay of the device schedule (debugging aid for small n);
    db/r force a two-sweep tile width 2^db and 2^r elements per thread,
    chunk_bits > 0 the chunked order (2^chunk_bits d-groups per chunk),
    chunk_window >= 2 its pipelined form."""
    A = np.ascontiguousarray(A, dtype=_np_dtype(dtype))
    n = A.shape[0].bit_length() - 1
    if in_place:
        out = A.copy().reshape(-1)
        _check(lib.tpd_debug_emulate_tuned(out.ctypes.data, n, out.ctypes.data, dtype, flags, 1, db, r, chunk_bits,
                                           chunk_window), "tpd_debug_emulate")
        return out
    out = np.full(A.size, np.nan, _np_dtype(dtype))  # poison: every element must be written
    _check(lib.tpd_debug_emulate_tuned(A.ctypes.data, n, out.ctypes.data, dtype, flags, 0, db, r, chunk_bits,
                                       chunk_window), "tpd_debug_emulate")
    return out


def emulate_synth(w: np.ndarray, n: int, dtype: int = TPD_C128, flags: int = 0, in_place: bool = False):
    """Host replay of the synthesis schedule (small n)."""
    w = np.ascontiguousarray(np.asarray(w).reshape(-1), dtype=_np_dtype(dtype))
    if in_place:
        out = w.copy()
        _check(lib.tpd_debug_emulate_synth(out.ctypes.data, n, out.ctypes.data, dtype, flags, 1), "emulate_synth")
        return out.reshape(1 << n, 1 << n)
    out = np.full(w.size, np.nan, _np_dtype(dtype))
    _check(lib.tpd_debug_emulate_synth(w.ctypes.data, n, out.ctypes.data, dtype, flags, 0), "emulate_synth")
    return out.reshape(1 << n, 1 << n)


def emulate_partial(A: np.ndarray, req, dtype: int = TPD_C128, flags: int = 0, in_place: bool = False):
    """Host replay of the partial decomposition; returns (values, work) with
    the work array NaN-poisoned before the call (out of place)."""
    A = np.ascontiguousarray(A, dtype=_np_dtype(dtype))
    n = A.shape[0].bit_length() - 1
    q = np.ascontiguousarray(np.asarray(req, dtype=np.uint64).reshape(-1))
    vals = np.full(q.size, np.nan, _np_dtype(dtype))
    work = A.copy().reshape(-1) if in_place else np.full(A.size, np.nan, _np_dtype(dtype))
    src = work if in_place else A
    _check(lib.tpd_debug_emulate_partial(src.ctypes.data, n, work.ctypes.data, q.ctypes.data, q.size,
                                         vals.ctypes.data, dtype, flags, int(in_place)), "tpd_debug_emulate_partial")
    return vals, work


def emulate_compact(coeffs: np.ndarray, n: int, tol: float = 0.0, capacity: Optional[int] = None,
                    dtype: int = TPD_C128, flags: int = 0):
    """Host replay of the compaction; returns (q, w, total)."""
    c = np.ascontiguousarray(np.asarray(coeffs).reshape(-1), dtype=_np_dtype(dtype))
    cap = c.size if capacity is None else int(capacity)
    q = np.zeros(max(cap, 1), np.uint64)
    w = np.zeros(max(cap, 1), _np_dtype(dtype))
    total = np.zeros(1, np.uint64)
    _check(lib.tpd_debug_emulate_compact(c.ctypes.data, n, dtype, flags, tol, q.ctypes.data, w.ctypes.data, cap,
                                         total.ctypes.data), "tpd_debug_emulate_compact")
    k = min(cap, int(total[0]))
    return q[:k], w[:k], int(total[0])


def _codes(codes):
    """per-n shape codes (sequence of 10, index n) as a C array, or None"""
    if codes is None:
        return None
    codes = list(codes)
    if len(codes) != 10:
        raise ValueError("codes needs one entry per n = 0..9")
    return (ctypes.c_int * 10)(*codes)


def emulate_batched(mats: Sequence[np.ndarray], dtype: int = TPD_C128, flags: int = 0,
                    in_place: bool = False, codes=None) -> List[np.ndarray]:
    """Host replay of the batched kernel; codes: per-n shape codes (see
    BatchedPlan.set_codes) or None for the tuned/default ones."""
    mats = [np.ascontiguousarray(m, dtype=_np_dtype(dtype)) for m in mats]
    ns = (ctypes.c_int * len(mats))(*[m.shape[0].bit_length() - 1 for m in mats])
    ins = (ctypes.c_void_p * len(mats))(*[m.ctypes.data for m in mats])
    if in_place:
        outs_np = [m.copy().reshape(-1) for m in mats]
        ins = (ctypes.c_void_p * len(mats))(*[o.ctypes.data for o in outs_np])
        _check(lib.tpd_debug_emulate_batched(ins, ns, len(mats), None, dtype, flags, _codes(codes)), "emulate_batched")
        return outs_np
    outs_np = [np.empty(m.size, _np_dtype(dtype)) for m in mats]
    outs = (ctypes.c_void_p * len(mats))(*[o.ctypes.data for o in outs_np])
    _check(lib.tpd_debug_emulate_batched(ins, ns, len(mats), outs, dtype, flags, _codes(codes)), "emulate_batched")
    return outs_np


# ----------------------------------------------------------------------------
# device entry points (torch tensors)
# ----------------------------------------------------------------------------
def _torch():
    import torch

    return torch


def _dtype_code(t) -> int:
    torch = _torch()
    if t.dtype == torch.complex128:
        return TPD_C128
    if t.dtype == torch.complex64:
        return TPD_C64
    if t.dtype == torch.float64:
        return TPD_R64
    if t.dtype == torch.float32:
        return TPD_R32
    raise TypeError(f"unsupported dtype {t.dtype}")


def _stream(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _flags(layout: str, prune: bool, order_bottom: bool = False, hermitian: bool = False) -> int:
    f = FLAG_HERMITIAN if hermitian else 0
    if layout == "matrix":
        f |= FLAG_LAYOUT_MATRIX
    elif layout != "canonical":
        raise ValueError("layout must be 'canonical' or 'matrix'")
    if not prune:
        f |= FLAG_NO_PRUNE
    if order_bottom:
        f |= FLAG_ORDER_BOTTOM
    return f


def _check_matrix(A):
    if not A.is_cuda or not A.is_contiguous() or A.dim() != 2 or A.shape[0] != A.shape[1]:
        raise ValueError("A must be a contiguous square CUDA tensor")
    d = A.shape[0]
    n = d.bit_length() - 1
    if (1 << n) != d:
        raise ValueError("dimension must be a power of two")
    return n


def decompose(A, out=None, *, layout: str = "canonical", prune: bool = True, order_bottom: bool = False,
              hermitian: bool = False, stream=None):
    """Pauli coefficients of A (2^n x 2^n complex64/complex128 CUDA tensor,
    or float64/float32 for a real matrix).

    Returns a 1-D tensor of 4^n coefficients (canonical order: index
    q = sum_k t_k 4^(n-k)), or the 2^n x 2^n matrix-layout array.  `out` may
    be A itself for an in-place call (see include/tpd.h).  For real input
    the values are real-coded: w_t = r_t for an even number of Y letters,
    i r_t for an odd number."""
    torch = _torch()
    n = _check_matrix(A)
    dt = _dtype_code(A)
    if out is None:
        out = torch.empty(4 ** n, dtype=A.dtype, device=A.device)
    if out.dtype != A.dtype or not out.is_cuda or not out.is_contiguous() or out.numel() != 4 ** n:
        raise ValueError("out must be a contiguous CUDA tensor of 4^n elements of A's dtype")
    _check(lib.tpd_decompose_ex(A.data_ptr(), n, out.data_ptr(), dt,
                                _flags(layout, prune, order_bottom, hermitian), _stream(stream)), "tpd_decompose_ex")
    return out


def decompose_noalloc(A, out, *, layout: str = "canonical", prune: bool = True, hermitian: bool = False,
                      stream=None):
    """decompose() through tpd_decompose_noalloc: the library allocates
    nothing (its pruning bitmap is a static device array shared by every
    call on the device).  `out` is required."""
    n = _check_matrix(A)
    if out.dtype != A.dtype or not out.is_cuda or not out.is_contiguous() or out.numel() != 4 ** n:
        raise ValueError("out must be a contiguous CUDA tensor of 4^n elements of A's dtype")
    _check(lib.tpd_decompose_noalloc(A.data_ptr(), n, out.data_ptr(), _dtype_code(A),
                                     _flags(layout, prune, False, hermitian), _stream(stream)),
           "tpd_decompose_noalloc")
    return out


def decompose_hermitian_real(A, out=None, *, prune: bool = True, db: int = 0, grid_per_cu: int = 0, stream=None):
    """Real weights of a Hermitian A (complex128 or complex64 CUDA tensor)
    in a separate real tensor (float64 / float32, 4^n, canonical order)
    through tpd_decompose_hermitian_real.  A is destroyed (the first sweep
    works in place in it) for n >= 9.  db > 0 forces the tile width 2^db
    and grid_per_cu the grid (test aid)."""
    torch = _torch()
    n = _check_matrix(A)
    if A.dtype not in (torch.complex128, torch.complex64):
        raise ValueError("A must be complex128 or complex64")
    rdt = torch.float64 if A.dtype == torch.complex128 else torch.float32
    if out is None:
        out = torch.empty(4 ** n, dtype=rdt, device=A.device)
    if out.dtype != rdt or not out.is_cuda or not out.is_contiguous() or out.numel() != 4 ** n:
        raise ValueError("out must be a contiguous CUDA tensor of 4^n real values of A's precision")
    fl = 0 if prune else FLAG_NO_PRUNE
    if db > 0 or grid_per_cu > 0:
        _check(lib.tpd_debug_decompose_hermitian_real_tuned(A.data_ptr(), n, out.data_ptr(), _dtype_code(A), fl, db,
                                                            grid_per_cu, _stream(stream)),
               "tpd_debug_decompose_hermitian_real_tuned")
    else:
        _check(lib.tpd_decompose_hermitian_real(A.data_ptr(), n, out.data_ptr(), _dtype_code(A), fl, _stream(stream)),
               "tpd_decompose_hermitian_real")
    return out


def decompose_tuned(A, out=None, *, db: int, grid_per_cu: int = 0, r: int = 4, layout: str = "canonical",
                    prune: bool = True, hermitian: bool = False, rotate: bool = False, chunk_bits: int = 0,
                    chunk_window: int = 0, stream=None):
    """decompose() with a forced two-sweep schedule (test aid); rotate=True
    selects the second sweep's rotated tile order, chunk_bits > 0 the
    chunked order (sweep 1 then sweep 2 over 2^chunk_bits d-groups at a
    time), chunk_window >= 2 its pipelined form over two streams."""
    torch = _torch()
    n = _check_matrix(A)
    if out is None:
        out = torch.empty(4 ** n, dtype=A.dtype, device=A.device)
    if out.dtype != A.dtype or not out.is_cuda or not out.is_contiguous() or out.numel() != 4 ** n:
        raise ValueError("out must be a contiguous CUDA tensor of 4^n elements of A's dtype")
    _check(lib.tpd_debug_decompose_tuned(A.data_ptr(), n, out.data_ptr(), _dtype_code(A),
                                         _flags(layout, prune, False, hermitian) | (FLAG_ROTATE_TILES if rotate else 0),
                                         db, r, grid_per_cu, chunk_bits, chunk_window, _stream(stream)),
           "tpd_debug_decompose_tuned")
    return out


def autotune(A, out=None, *, layout: str = "canonical", prune: bool = True, hermitian: bool = False,
             stream=None) -> dict:
    """Autotune the schedule for A's (n, dtype, layout, placement) on these
    buffers; later calls with the same key use the choice."""
    torch = _torch()
    n = _check_matrix(A)
    if out is None:
        out = torch.empty(4 ** n, dtype=A.dtype, device=A.device)
    if out.dtype != A.dtype or not out.is_cuda or not out.is_contiguous() or out.numel() != 4 ** n:
        raise ValueError("out must be a contiguous CUDA tensor of 4^n elements of A's dtype")
    buf = ctypes.create_string_buffer(8192)
    _check(lib.tpd_autotune(A.data_ptr(), n, out.data_ptr(), _dtype_code(A), _flags(layout, prune, False, hermitian),
                            _stream(stream), buf, 8192), "tpd_autotune")
    return json.loads(buf.value.decode())


def autotune_hermitian_real(A, out=None, *, prune: bool = True, stream=None) -> dict:
    """Autotune decompose_hermitian_real for A's (n, dtype) on these buffers
    (A is destroyed); later calls use the choice."""
    torch = _torch()
    n = _check_matrix(A)
    rdt = torch.float64 if A.dtype == torch.complex128 else torch.float32
    if out is None:
        out = torch.empty(4 ** n, dtype=rdt, device=A.device)
    buf = ctypes.create_string_buffer(8192)
    _check(lib.tpd_autotune_hermitian_real(A.data_ptr(), n, out.data_ptr(), _dtype_code(A),
                                           0 if prune else FLAG_NO_PRUNE, _stream(stream), buf, 8192),
           "tpd_autotune_hermitian_real")
    return json.loads(buf.value.decode())


def synthesize(coeffs, out=None, *, layout: str = "canonical", stream=None):
    """Inverse transform: A = sum_t w_t sigma^t from 4^n weights (canonical
    order, or the matrix layout).  Returns the 2^n x 2^n matrix."""
    torch = _torch()
    if not coeffs.is_cuda or not coeffs.is_contiguous():
        raise ValueError("coeffs must be a contiguous CUDA tensor")
    m = coeffs.numel()
    n = (m.bit_length() - 1) // 2
    if 4 ** n != m:
        raise ValueError("coeffs must hold 4^n values")
    if out is None:
        out = torch.empty((1 << n, 1 << n), dtype=coeffs.dtype, device=coeffs.device)
    if out.dtype != coeffs.dtype or not out.is_cuda or not out.is_contiguous() or out.numel() != m:
        raise ValueError("out must be a contiguous CUDA tensor of 4^n elements of coeffs' dtype")
    _check(lib.tpd_synthesize_ex(coeffs.data_ptr(), n, out.data_ptr(), _dtype_code(coeffs), _flags(layout, True),
                                 _stream(stream)), "tpd_synthesize_ex")
    return out


def decompose_partial(A, req, values=None, work=None, *, layout: str = "canonical", prune: bool = True,
                      hermitian: bool = False, order_bottom: bool = False, stream=None):
    """Weights of the requested strings only (canonical indices `req`, a
    CUDA int64/uint64 tensor or a sequence).  `work` is the 4^n work array
    (allocated if None; may be A itself for an in-place call in the matrix
    layout).  Returns `values`, one value of A's dtype per request (NaN for
    indices >= 4^n; real-coded for real input)."""
    torch = _torch()
    n = _check_matrix(A)
    dt = _dtype_code(A)
    if not torch.is_tensor(req):
        req = torch.tensor(np.asarray(req, dtype=np.int64), device=A.device)
    if not req.is_cuda or req.dtype not in (torch.int64, torch.uint64) or not req.is_contiguous():
        raise ValueError("req must be a contiguous CUDA int64 tensor of canonical indices")
    count = req.numel()
    if values is None:
        values = torch.empty(count, dtype=A.dtype, device=A.device)
    if values.dtype != A.dtype or not values.is_cuda or not values.is_contiguous() or values.numel() != count:
        raise ValueError("values must be a contiguous CUDA tensor of len(req) elements of A's dtype")
    if work is None:
        work = torch.empty(4 ** n, dtype=A.dtype, device=A.device)
    if work.dtype != A.dtype or not work.is_cuda or not work.is_contiguous() or work.numel() != 4 ** n:
        raise ValueError("work must be a contiguous CUDA tensor of 4^n elements of A's dtype")
    _check(lib.tpd_decompose_partial(A.data_ptr(), n, work.data_ptr(), req.data_ptr(), count, values.data_ptr(), dt,
                                     _flags(layout, prune, order_bottom, hermitian), _stream(stream)),
           "tpd_decompose_partial")
    return values


def compact(coeffs, *, tol: float = 0.0, capacity: Optional[int] = None, layout: str = "canonical", stream=None):
    """Sparse list of the kept weights: (q int64 tensor, w tensor, total).
    With capacity None the count is read back first (one synchronisation)
    and the lists are sized to it."""
    torch = _torch()
    if not coeffs.is_cuda or not coeffs.is_contiguous():
        raise ValueError("coeffs must be a contiguous CUDA tensor")
    m = coeffs.numel()
    n = (m.bit_length() - 1) // 2
    if 4 ** n != m:
        raise ValueError("coeffs must hold 4^n values")
    dt = _dtype_code(coeffs)
    flags = FLAG_LAYOUT_MATRIX if layout == "matrix" else 0
    if layout not in ("canonical", "matrix"):
        raise ValueError("layout must be 'canonical' or 'matrix'")
    total = torch.zeros(1, dtype=torch.int64, device=coeffs.device)
    if capacity is None:
        _check(lib.tpd_compact(coeffs.data_ptr(), n, dt, flags, float(tol), None, None, 0, total.data_ptr(),
                               _stream(stream)), "tpd_compact")
        capacity = int(total.item())
    q = torch.empty(max(capacity, 1), dtype=torch.int64, device=coeffs.device)
    w = torch.empty(max(capacity, 1), dtype=coeffs.dtype, device=coeffs.device)
    _check(lib.tpd_compact(coeffs.data_ptr(), n, dt, flags, float(tol), q.data_ptr(), w.data_ptr(), capacity,
                           total.data_ptr(), _stream(stream)), "tpd_compact")
    k = min(capacity, int(total.item()))
    return q[:k], w[:k], int(total.item())


def decompose_batched(mats, outs=None, *, layout: str = "canonical", stream=None):
    """Decompose a list of square matrices of mixed sizes in one launch.
    outs=None allocates outputs; outs='inplace' overwrites the inputs."""
    torch = _torch()
    if len(mats) == 0:
        return []
    dt = _dtype_code(mats[0])
    ns = [_check_matrix(m) for m in mats]
    for m in mats:
        if m.dtype != mats[0].dtype:
            raise ValueError("all matrices must share one dtype")
    in_place = isinstance(outs, str) and outs == "inplace"
    if outs is None:
        outs = [torch.empty(4 ** n, dtype=mats[0].dtype, device=mats[0].device) for n in ns]
    cnt = len(mats)
    c_ns = (ctypes.c_int * cnt)(*ns)
    c_in = (ctypes.c_void_p * cnt)(*[m.data_ptr() for m in mats])
    c_out = None if in_place else (ctypes.c_void_p * cnt)(*[o.data_ptr() for o in outs])
    _check(lib.tpd_decompose_batched(c_in, c_ns, cnt, c_out, dt, _flags(layout, True), _stream(stream)),
           "tpd_decompose_batched")
    return mats if in_place else outs


class Plan:
    """Single-matrix plan: all allocation at creation; execute() is
    graph-capturable.  timing=True records HIP events around each kernel."""

    def __init__(self, n: int, dtype: int = TPD_C128, *, layout: str = "canonical", prune: bool = True,
                 in_place: bool = False, timing: bool = False, order_bottom: bool = False, hermitian: bool = False,
                 rotate: bool = False):
        self.n = n
        self.dtype = dtype
        self.in_place = in_place
        f = _flags(layout, prune, order_bottom, hermitian) | (FLAG_TIMING if timing else 0)
        f |= FLAG_ROTATE_TILES if rotate else 0
        h = ctypes.c_void_p()
        _check(lib.tpd_plan_create(n, dtype, f, int(in_place), ctypes.byref(h)), "tpd_plan_create")
        self._h = h

    def execute(self, A, out, stream=None):
        _check(lib.tpd_plan_execute(self._h, A.data_ptr(), out.data_ptr(), _stream(stream)), "tpd_plan_execute")
        return out

    def num_kernels(self) -> int:
        return int(lib.tpd_plan_num_kernels(self._h))

    def timing(self, reset: bool = False):
        k = self.num_kernels()
        ms = (ctypes.c_double * k)()
        cnt = (ctypes.c_uint64 * k)()
        _check(lib.tpd_plan_timing(self._h, ms, cnt, int(reset)), "tpd_plan_timing")
        return [float(v) for v in ms], [int(v) for v in cnt]

    def prune_stats(self, stream=None) -> dict:
        lt, tt, lp = ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_uint64()
        lvl = ctypes.c_int()
        _check(lib.tpd_plan_prune_stats(self._h, ctypes.byref(lt), ctypes.byref(tt), ctypes.byref(lp),
                                        ctypes.byref(lvl), _stream(stream)), "tpd_plan_prune_stats")
        return {"live_tiles": lt.value, "total_tiles": tt.value, "live_prefixes": lp.value,
                "prefix_level": lvl.value}

    def describe(self) -> dict:
        buf = ctypes.create_string_buffer(4096)
        _check(lib.tpd_plan_describe(self._h, buf, 4096), "tpd_plan_describe")
        return json.loads(buf.value.decode())

    def close(self):
        if getattr(self, "_h", None):
            lib.tpd_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class BatchedPlan(Plan):
    """Batched plan over fixed qubit counts; execute() takes device arrays of
    device pointers (int64 CUDA tensors), graph-capturable."""

    def __init__(self, ns: Sequence[int], dtype: int = TPD_C128, *, layout: str = "canonical",
                 in_place: bool = False, timing: bool = False):
        self.ns = list(ns)
        self.dtype = dtype
        self.in_place = in_place
        f = _flags(layout, True) | (FLAG_TIMING if timing else 0)
        c_ns = (ctypes.c_int * max(1, len(self.ns)))(*self.ns)
        h = ctypes.c_void_p()
        _check(lib.tpd_plan_create_batched(c_ns, len(self.ns), dtype, f, int(in_place), ctypes.byref(h)),
               "tpd_plan_create_batched")
        self._h = h

    @staticmethod
    def pointer_table(tensors, device=None):
        torch = _torch()
        dev = device or tensors[0].device
        return torch.tensor([t.data_ptr() for t in tensors], dtype=torch.int64, device=dev)

    def autotune(self, d_ptrs, d_out_ptrs=None, stream=None) -> dict:
        buf = ctypes.create_string_buffer(8192)
        _check(lib.tpd_autotune_batched(self._h, d_ptrs.data_ptr(),
                                        None if d_out_ptrs is None else d_out_ptrs.data_ptr(), _stream(stream),
                                        buf, 8192), "tpd_autotune_batched")
        return json.loads(buf.value.decode())

    def set_codes(self, codes):
        """Force per-n shape codes (index n): 0 full tile with prefetch, 1
        full tile without, 2 (n >= 3) half tile with prefetch (test aid)."""
        _check(lib.tpd_debug_plan_batched_codes(self._h, _codes(codes)), "tpd_debug_plan_batched_codes")

    def execute(self, d_ptrs, d_out_ptrs=None, stream=None):
        _check(lib.tpd_plan_execute_batched(self._h, d_ptrs.data_ptr(),
                                            None if d_out_ptrs is None else d_out_ptrs.data_ptr(),
                                            _stream(stream)), "tpd_plan_execute_batched")
