"""GPU test of tpd_decompose_noalloc, the entry point that allocates nothing
(its pruning bitmap is a static device array shared by every call on a
device).  Through the C ABI, its results must be bitwise those of
tpd_decompose_ex with the same arguments, on consecutive calls whose sizes
shrink (the shared array keeps the previous call's bits and must be cleared
before use).
"""
import pytest
import torch

import workloads as W

pytestmark = pytest.mark.gpu

tpd = pytest.importorskip("paper_2310_13421_amd.tpd")

DEV = "cuda"


def _stream():
    return torch.cuda.current_stream().cuda_stream


def _call(fn, A, out, dtype, flags):
    n = A.shape[0].bit_length() - 1
    rc = fn(A.data_ptr(), n, out.data_ptr(), dtype, flags, _stream())
    assert rc == 0, tpd.STATUS.get(rc, rc)
    torch.cuda.synchronize()
    return out


def _same(a, b):
    if a.is_complex():
        a, b = torch.view_as_real(a), torch.view_as_real(b)
    return bool(torch.equal(a, b))


def test_noalloc_equals_decompose_ex_on_shrinking_calls():
    if not torch.cuda.is_available():
        pytest.fail("needs a visible GPU")
    lib = tpd.lib
    cases = []
    # 1: dense Hermitian n = 13, complex128, canonical order, out of place
    cases.append((torch.from_numpy(W.gaussian(13, seed=4100, hermitian=True)).to(DEV), tpd.TPD_C128, 0, False))
    # 2: smaller, structured (zero tiles pruned), Hermitian mode, matrix layout in place
    H = W.dense_from_terms_device(W.heisenberg_terms(12, seed=4101, n_local=50, dyadic=True), 12)
    cases.append((H, tpd.TPD_C128, tpd.FLAG_HERMITIAN | tpd.FLAG_LAYOUT_MATRIX, True))
    # 3: smaller again, complex64 dense, canonical
    cases.append((torch.from_numpy(W.gaussian(10, seed=4102)).to(DEV).to(torch.complex64), tpd.TPD_C64, 0, False))
    # 4: one sweep (n <= 8), real float64
    cases.append((torch.from_numpy(W.real_gaussian(7, seed=4103)).to(DEV), tpd.TPD_R64, 0, False))
    for A, dt, flags, in_place in cases:
        n = A.shape[0].bit_length() - 1
        if in_place:
            X = A.clone()
            got = _call(lib.tpd_decompose_noalloc, X, X.view(-1), dt, flags)
            Y = A.clone()
            ref = _call(lib.tpd_decompose_ex, Y, Y.view(-1), dt, flags)
        else:
            got = _call(lib.tpd_decompose_noalloc, A, torch.full((4 ** n,), float("nan"), dtype=A.dtype, device=DEV),
                        dt, flags)
            ref = _call(lib.tpd_decompose_ex, A, torch.empty(4 ** n, dtype=A.dtype, device=DEV), dt, flags)
        assert _same(got, ref), (n, dt, flags, in_place)
    # the same again in the opposite order of sizes (the array grows back)
    for A, dt, flags, in_place in reversed(cases):
        n = A.shape[0].bit_length() - 1
        if in_place:
            continue
        got = _call(lib.tpd_decompose_noalloc, A, torch.empty(4 ** n, dtype=A.dtype, device=DEV), dt, flags)
        ref = _call(lib.tpd_decompose_ex, A, torch.empty(4 ** n, dtype=A.dtype, device=DEV), dt, flags)
        assert _same(got, ref), (n, dt, flags)


def test_noalloc_argument_errors():
    if not torch.cuda.is_available():
        pytest.fail("needs a visible GPU")
    lib = tpd.lib
    A = torch.zeros((16, 16), dtype=torch.complex128, device=DEV)
    out = torch.empty(256, dtype=torch.complex128, device=DEV)
    s = _stream()
    assert lib.tpd_decompose_noalloc(A.data_ptr(), 4, out.data_ptr(), tpd.TPD_C128, tpd.FLAG_TIMING, s) == 1
    assert lib.tpd_decompose_noalloc(None, 4, out.data_ptr(), tpd.TPD_C128, 0, s) == 1
    assert lib.tpd_decompose_noalloc(A.data_ptr(), 17, out.data_ptr(), tpd.TPD_C128, 0, s) == 2
    assert lib.tpd_decompose_noalloc(A.data_ptr(), 4, A.data_ptr() + 16, tpd.TPD_C128, 0, s) == 1  # overlap
    # canonical order in place is rejected beyond n = 6, as tpd_decompose_ex does
    B = torch.zeros((512, 512), dtype=torch.complex128, device=DEV)
    assert lib.tpd_decompose_noalloc(B.data_ptr(), 9, B.data_ptr(), tpd.TPD_C128, 0, s) == 2
