"""GPU parity tests: the HIP path (through the C ABI) against the CPU oracle.

Bar: complex128 results are compared element by element with the oracle on
the same seeded inputs -- bitwise where the schedule performs the oracle's
operations in the paper's level order, else within n u max|a_ij|
(u = 2^-53), itself far inside the required 1e-12 max|a_ij|; complex64
within (n + 1) 2^-24 max|a_ij| (<= 2e-6 max|a_ij|); integer inputs bit-exact
in both precisions.  Sizes span many tiles; full-size configurations are
checked on sampled strings against the definition, plus Parseval and
exact invariants.
"""
import os

import numpy as np
import pytest
import torch

from oracle import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

tpd = pytest.importorskip("paper_2310_13421_amd.tpd")

DEV = "cuda"
U64 = 2.0 ** -53
U32 = 2.0 ** -24


@pytest.fixture(scope="module", autouse=True)
def _gpu_required():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a visible GPU (run with -m 'not gpu' on CPU-only machines)")
    yield
    torch.cuda.synchronize()
    tpd.lib.tpd_release_workspace()


def amax(A):
    A = np.asarray(A)
    return float(np.max(np.abs(np.concatenate([A.real.ravel(), A.imag.ravel()]))))


def cerr(a, b):
    d = np.asarray(a, np.complex128) - np.asarray(b, np.complex128)
    return float(np.max(np.abs(np.concatenate([d.real.ravel(), d.imag.ravel()])))) if d.size else 0.0


def same_bits(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return np.array_equal(a.real, b.real) and np.array_equal(a.imag, b.imag)


def to_dev(A, dtype=torch.complex128):
    return torch.from_numpy(np.ascontiguousarray(A)).to(DEV).to(dtype).contiguous()


def spread(v):
    r = np.zeros_like(v)
    for b in range(20):
        r |= ((v >> b) & 1) << (2 * b)
    return r


def deinterleave(q):
    q = np.asarray(q, np.int64)
    h = np.zeros_like(q)
    l = np.zeros_like(q)
    for b in range(20):
        l |= ((q >> (2 * b)) & 1) << b
        h |= ((q >> (2 * b + 1)) & 1) << b
    return h, l


def matrix_to_canonical(coeffs, n):
    d = 1 << n
    h = np.arange(d, dtype=np.int64)[:, None]
    l = np.arange(d, dtype=np.int64)[None, :]
    q = (spread(h) << 1) | spread(l)
    out = np.empty(4 ** n, coeffs.dtype)
    out[q.ravel()] = np.asarray(coeffs).ravel()
    return out


def run(A_host, dtype=torch.complex128, **kw):
    A = to_dev(A_host, dtype)
    out = tpd.decompose(A, **kw)
    torch.cuda.synchronize()
    return out.cpu().numpy()


HOST_THREADS = 16  # the GPU machine's host share


def sampled_oracle(A_dev, n, qs, chunk_masks=256):
    """omega_q for sampled q from the definition, reading only the entries
    A[i ^ x][i] each string needs (gathered from the device input), the
    per-mask sums on host threads."""
    flat = A_dev.view(-1)
    i = torch.arange(1 << n, device=A_dev.device, dtype=torch.int64)

    def fetch(ms):
        xs = torch.from_numpy(np.asarray(ms, np.int64)).to(A_dev.device)
        idx = ((i[None, :] ^ xs[:, None]) << n) + i[None, :]
        return flat[idx.reshape(-1)].to(torch.complex128).reshape(len(ms), -1).cpu().numpy()

    return O.sampled_weights(fetch, n, qs, threads=HOST_THREADS, masks_per_fetch=chunk_masks)


# ----------------------------------------------------------------------------
# configuration 0: n = 8, complex Gaussian; integer variant
# ----------------------------------------------------------------------------
def test_config0_n8_gaussian_vs_definition_all_strings():
    n = 8
    A = W.gaussian(n, seed=1)
    got = run(A)
    ref = O.weight_sparse(A, np.arange(4 ** n))
    assert cerr(got, ref) <= 1e-12 * amax(A)
    assert cerr(got, ref) <= n * U64 * amax(A)
    assert same_bits(got, O.tpd_recursive(A))  # paper level order: same operations


@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
def test_config0_n8_integer_entries_bit_exact(dtype):
    n = 8
    A = W.integer(n, seed=1)
    ref = O.weight_sparse(A, np.arange(4 ** n))
    got = run(A, dtype).astype(np.complex128)
    assert same_bits(got, ref)


# ----------------------------------------------------------------------------
# every n up to 12, both layouts, in place and out of place, both dtypes
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("n", list(range(0, 13)))
def test_sizes_canonical_and_matrix_layout(n):
    A = W.gaussian(n, seed=40 + n) if n else np.array([[1.25 - 0.5j]])
    ref = O.tpd_recursive(A)
    assert same_bits(run(A), ref)
    got = run(A, layout="matrix")
    assert same_bits(matrix_to_canonical(got, n), ref)
    g64 = run(A, torch.complex64).astype(np.complex128)
    assert cerr(g64, ref) <= (n + 1) * U32 * amax(A)


@pytest.mark.parametrize("n", [1, 4, 6, 7, 9, 12])
def test_in_place(n):
    A = W.gaussian(n, seed=60 + n)
    ref = O.tpd_recursive(A)
    for dtype in (torch.complex128, torch.complex64):
        T = to_dev(A, dtype)
        tpd.decompose(T, T.view(-1), layout="matrix")
        got = matrix_to_canonical(T.cpu().numpy().ravel(), n).astype(np.complex128)
        if dtype == torch.complex128:
            assert same_bits(got, ref)
        else:
            assert cerr(got, ref) <= (n + 1) * U32 * amax(A)
        if n <= 6:
            T = to_dev(A, dtype)
            tpd.decompose(T, T.view(-1))
            got = T.cpu().numpy().ravel().astype(np.complex128)
            assert cerr(got, ref) <= (n + 1) * U32 * amax(A) if dtype == torch.complex64 else same_bits(got, ref)
    with pytest.raises(tpd.TPDError):
        T = to_dev(W.gaussian(9, 1))
        tpd.decompose(T, T.view(-1))  # in place needs the matrix layout for n > 6


@pytest.mark.parametrize("n", [10, 12])
def test_bottom_first_register_order_within_bound(n):
    A = W.gaussian(n, seed=80 + n)
    ref = O.tpd_recursive(A)
    got = run(A, order_bottom=True)
    assert cerr(got, ref) <= n * U64 * amax(A) * 1.01


# ----------------------------------------------------------------------------
# configuration 1: n = 12 Hermitian
# ----------------------------------------------------------------------------
def test_config1_n12_hermitian():
    n = 12
    A = W.gaussian(n, seed=2, hermitian=True)
    got = run(A)
    ref = O.tpd_recursive(A)
    assert same_bits(got, ref)
    assert np.all(got.imag == 0.0)  # Hermitian input: exactly real weights
    parseval = 2 ** n * np.sum(np.abs(got) ** 2)
    fro = np.sum(np.abs(A) ** 2)
    assert abs(parseval - fro) <= 1e-12 * fro
    qs = W.sampled_strings(n, 10000, seed=2)
    bf = sampled_oracle(to_dev(A), n, qs)
    assert cerr(got[qs.astype(np.int64)], bf) <= 1e-12 * amax(A)
    g64 = run(A, torch.complex64)
    assert np.all(g64.imag == 0.0)
    assert cerr(g64.astype(np.complex128), ref) <= (n + 1) * U32 * amax(A)


# ----------------------------------------------------------------------------
# configuration 2: n = 14 structured Hamiltonian, zero-block pruning
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("dyadic", [True, False])
def test_config2_n14_heisenberg_round_trip_and_pruning(dyadic):
    n = 14
    terms = W.heisenberg_terms(n, seed=3, n_local=200, dyadic=dyadic)
    H = W.dense_from_terms_device(terms, n)
    plan = tpd.Plan(n)
    out = torch.empty(4 ** n, dtype=torch.complex128, device=DEV)
    plan.execute(H, out)
    torch.cuda.synchronize()
    stats = plan.prune_stats()
    qs = np.array([W.string_index(s) for s, _ in terms], np.int64)
    cs = np.array([c for _, c in terms], np.complex128)
    got = out[torch.from_numpy(qs).to(DEV)].cpu().numpy()
    scale = float(torch.view_as_real(H).abs().max())
    rest = out.clone()
    rest[torch.from_numpy(qs).to(DEV)] = 0
    resid = float(torch.view_as_real(rest).abs().max())
    if dyadic:
        assert same_bits(got, cs)  # exact round trip
        assert resid == 0.0        # exact zeros everywhere else
    else:
        assert cerr(got, cs) <= 1e-12 * scale
        assert resid <= 1e-12 * scale
    # pruning: live level-n1 CMWs equal the distinct generating prefixes
    n1 = stats["prefix_level"]
    prefixes = {int(q) >> (2 * (n - n1)) for q in qs}
    if dyadic:
        assert stats["live_prefixes"] == len(prefixes)
    else:
        assert stats["live_prefixes"] >= len(prefixes)
    assert stats["live_tiles"] < stats["total_tiles"] // 4
    # sampled strings against the definition (both generating and others)
    sample = np.concatenate([qs[:50], W.sampled_strings(n, 2000, seed=33).astype(np.int64)])
    bf = sampled_oracle(H, n, sample)
    assert cerr(out[torch.from_numpy(sample).to(DEV)].cpu().numpy(), bf) <= 1e-12 * scale
    # the unpruned schedule gives the same bits
    out2 = tpd.decompose(H, prune=False)
    assert torch.equal(torch.view_as_real(out2), torch.view_as_real(out))
    # and so do the chunked orders, whose second sweeps skip the tiles the
    # pruning bits of their own chunk mark (one stream, and pipelined)
    for cb, w in ((2, 0), (2, 2), (5, 4)):
        out2.fill_(float("nan"))
        tpd.decompose_tuned(H, out2, db=4, grid_per_cu=8, chunk_bits=cb, chunk_window=w)
        assert torch.equal(torch.view_as_real(out2), torch.view_as_real(out)), (cb, w)
    plan.close()


def test_tfim_live_prefixes_closed_form():
    # transverse-field Ising chain: 2k+1 live CMWs at level k < n
    n = 12
    H = W.dense_from_terms_device(W.tfim_terms(n, 1.0, 0.5), n)
    plan = tpd.Plan(n)
    out = torch.empty(4 ** n, dtype=torch.complex128, device=DEV)
    plan.execute(H, out)
    st = plan.prune_stats()
    k = st["prefix_level"]
    assert st["live_prefixes"] == 2 * k + 1
    nz = torch.nonzero(torch.view_as_real(out).abs().sum(-1)).cpu().numpy().ravel()
    expect = sorted(W.string_index(s) for s, _ in W.tfim_terms(n, 1.0, 0.5))
    assert nz.tolist() == expect
    plan.close()


# ----------------------------------------------------------------------------
# configuration 3: batched uneven workload, one persistent launch, graph replay
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
def test_config3_batched_4096(dtype):
    ns = W.batched_qubits(4096, seed=4)
    mats = W.batched_matrices(ns, seed=4)
    dmats = [to_dev(m, dtype) for m in mats]
    outs = tpd.decompose_batched(dmats)
    torch.cuda.synchronize()
    worst = 0.0
    for k, (o, m) in enumerate(zip(outs, mats)):
        got = o.cpu().numpy()
        ref = O.tpd_recursive(m)
        if dtype == torch.complex128:
            assert same_bits(got, ref), k
        else:
            worst = max(worst, cerr(got.astype(np.complex128), ref) / amax(m))
            assert cerr(got.astype(np.complex128), ref) <= (int(ns[k]) + 1) * U32 * amax(m), k
        if k % 2 == 1:
            assert np.all(got.imag == 0), k  # Hermitian members: real weights


def test_batched_plan_graph_capture_and_layouts():
    ns = [int(v) for v in W.batched_qubits(300, seed=7, lo=0, hi=9)]
    mats = W.batched_matrices(ns, seed=7)
    dmats = [to_dev(m) for m in mats]
    refs = [O.tpd_recursive(m) for m in mats]
    outs = [torch.full((4 ** n,), float("nan"), dtype=torch.complex128, device=DEV) for n in ns]
    plan = tpd.BatchedPlan(ns)
    dp = tpd.BatchedPlan.pointer_table(dmats)
    do = tpd.BatchedPlan.pointer_table(outs)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        plan.execute(dp, do)  # warm up on the capture stream
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        plan.execute(dp, do)
    for rep in range(3):
        for o in outs:
            o.fill_(float("nan"))  # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for k, (o, r) in enumerate(zip(outs, refs)):
            assert same_bits(o.cpu().numpy(), r), (rep, k)
    plan.close()
    # matrix layout, in place (allowed for every n with the matrix layout)
    dm2 = [to_dev(m) for m in mats]
    tpd.decompose_batched(dm2, "inplace", layout="matrix")
    for k, (o, r) in enumerate(zip(dm2, refs)):
        assert same_bits(matrix_to_canonical(o.cpu().numpy().ravel(), ns[k]), r), k


@pytest.mark.parametrize("dtype,code", [(torch.complex128, tpd.TPD_C128), (torch.complex64, tpd.TPD_C64),
                                        (torch.float32, tpd.TPD_R32)])
def test_batched_every_item_shape_and_autotune_same_bits(dtype, code):
    # the per-n item shapes the batched autotuner chooses from (full tile
    # with or without prefetch, half tile) and the tuned plan give the same
    # bits as the default plan, NaN-poisoned outputs fully written, complex128
    # bitwise equal to Algorithm 1; the tuner reports a choice per n
    ns = [int(v) for v in W.batched_qubits(600, seed=45, lo=0, hi=9)]
    if dtype.is_complex:
        mats = W.batched_matrices(ns, seed=45)
        dmats = [to_dev(m, dtype) for m in mats]
    else:
        mats = [W.real_gaussian(n, seed=4500 + k) for k, n in enumerate(ns)]
        dmats = [torch.from_numpy(m).to(DEV).to(dtype) for m in mats]
    dp = tpd.BatchedPlan.pointer_table(dmats)

    def run(plan):
        outs = [torch.full((4 ** n,), float("nan"), dtype=dtype, device=DEV) for n in ns]
        plan.execute(dp, tpd.BatchedPlan.pointer_table(outs))
        torch.cuda.synchronize()
        return outs

    plan = tpd.BatchedPlan(ns, code)
    base = run(plan)
    if dtype == torch.complex128:
        for k in range(0, len(ns), 7):
            assert same_bits(base[k].cpu().numpy(), O.tpd_recursive(mats[k])), k
    for c in (0, 1, 2):
        plan.set_codes([0 if (c == 2 and n < 3) else c for n in range(10)])
        outs = run(plan)
        for k, (a, b) in enumerate(zip(outs, base)):
            assert torch.equal(a, b), (c, k)
    ws = [torch.empty(4 ** n, dtype=dtype, device=DEV) for n in ns]
    rep = plan.autotune(dp, tpd.BatchedPlan.pointer_table(ws))
    assert sorted(p_["n"] for p_ in rep["per_n"]) == sorted(set(ns))
    assert all(p_["chosen"] in [c_["code"] for c_ in p_["candidates"]] for p_ in rep["per_n"])
    desc = plan.describe()
    assert {p_["n"]: p_["code"] for p_ in desc["per_n"]} == {p_["n"]: p_["chosen"] for p_ in rep["per_n"]}
    outs = run(plan)
    for k, (a, b) in enumerate(zip(outs, base)):
        assert torch.equal(a, b), k
    # a new plan of the dtype takes the tuned shapes
    plan2 = tpd.BatchedPlan(ns, code)
    assert plan2.describe()["per_n"] == desc["per_n"]
    outs = run(plan2)
    for k, (a, b) in enumerate(zip(outs, base)):
        assert torch.equal(a, b), k
    plan.close()
    plan2.close()


# ----------------------------------------------------------------------------
# configuration 4: n = 16 Hermitian, complex128 and complex64, sampled strings
# ----------------------------------------------------------------------------
def test_config4_n16_sampled_strings_parseval_both_precisions():
    # 10^6 strings uniform over the 4^16 plus the forced ones (I..I, X..X,
    # Y..Y, Z..Z, 4^16 - 1), each against the definition in binary64
    n = 16
    torch.cuda.empty_cache()
    A = W.gaussian_device(n, seed=5, hermitian=True)
    a_max = float(torch.view_as_real(A).abs().max())
    fro = float(torch.view_as_real(A).double().square().sum())
    qs = W.sampled_strings(n, 10 ** 6, seed=5)
    bf = sampled_oracle(A, n, qs)
    qd = torch.from_numpy(qs.astype(np.int64)).to(DEV)

    out = tpd.decompose(A)
    torch.cuda.synchronize()
    got = out[qd].cpu().numpy()
    assert cerr(got, bf) <= 1e-12 * a_max
    assert cerr(got, bf) <= n * U64 * a_max
    assert float(out.imag.abs().max()) == 0.0  # Hermitian: exactly real
    pars = float(torch.view_as_real(out).square().sum()) * 2 ** n
    assert abs(pars - fro) <= 1e-12 * fro
    # in place, matrix layout, on a copy: same bits as the canonical result
    del out
    torch.cuda.empty_cache()
    ref_vals = got
    B = A.clone()
    tpd.decompose(B, B.view(-1), layout="matrix")
    h, l = deinterleave(qs.astype(np.int64))
    hb = torch.from_numpy(h).to(DEV)
    lb = torch.from_numpy(l).to(DEV)
    assert same_bits(B[hb, lb].cpu().numpy(), ref_vals)
    del B
    torch.cuda.empty_cache()

    # Hermitian mode: half the reads, real output, bitwise the same real parts
    outh = tpd.decompose(A, hermitian=True)
    torch.cuda.synchronize()
    gh = outh[qd].cpu().numpy()
    assert np.array_equal(gh.real, ref_vals.real) and np.all(gh.imag == 0)
    del outh
    torch.cuda.empty_cache()

    A32 = A.to(torch.complex64)
    del A
    torch.cuda.empty_cache()
    out32 = tpd.decompose(A32)
    torch.cuda.synchronize()
    g32 = out32[qd].cpu().numpy().astype(np.complex128)
    assert cerr(g32, bf) <= 2e-6 * a_max
    assert cerr(g32, bf) <= (n + 1) * U32 * a_max
    fro32 = float(torch.view_as_real(A32).double().square().sum())
    pars32 = float(torch.view_as_real(out32).double().square().sum()) * 2 ** n
    assert abs(pars32 - fro32) <= 1e-6 * fro32
    del A32, out32
    torch.cuda.empty_cache()


@pytest.mark.parametrize("dtype,dbs", [(torch.complex128, (3, 4, 5)), (torch.complex64, (4, 5, 6))])
def test_n16_in_place_every_tuning_candidate(dtype, dbs):
    # the headline launch configuration at full size: n = 16 Hermitian, in
    # place with the matrix layout, pruning on, for every schedule the
    # autotuner may choose (tile width x persistent grid), in the general
    # and the Hermitian mode; sampled positions against the definition, and
    # every candidate bitwise equal to the default schedule there
    n = 16
    torch.cuda.empty_cache()
    A = W.gaussian_device(n, seed=5, dtype=dtype, hermitian=True)
    a_max = float(torch.view_as_real(A).abs().max())
    qs = W.sampled_strings(n, 2000, seed=16)
    bf = sampled_oracle(A, n, qs)
    h, l = deinterleave(qs.astype(np.int64))
    hb = torch.from_numpy(h).to(DEV)
    lb = torch.from_numpy(l).to(DEV)
    tol = n * U64 * a_max if dtype == torch.complex128 else (n + 1) * U32 * a_max
    B = torch.empty_like(A)
    B.copy_(A)
    tpd.decompose(B, B.view(-1), layout="matrix")
    ref = B[hb, lb].cpu().numpy()
    assert cerr(ref, bf) <= tol
    for herm in (False, True):
        for db in dbs:
            for g in (0, 1, 2, 4, 8):
                B.copy_(A)
                tpd.decompose_tuned(B, B.view(-1), db=db, grid_per_cu=g, layout="matrix", hermitian=herm,
                                    rotate=(g == 4))
                got = B[hb, lb].cpu().numpy()
                if herm:
                    assert np.array_equal(got.real, ref.real) and np.all(got.imag == 0), (db, g)
                else:
                    assert same_bits(got, ref), (db, g)
    del A, B
    torch.cuda.empty_cache()


@pytest.mark.parametrize("dtype,dbs", [(torch.complex128, (3, 4, 5)), (torch.complex64, (4, 5, 6))])
def test_n14_dense_every_tuning_candidate(dtype, dbs):
    # the n = 14 dense legs at full size: Hermitian input, in place with the
    # matrix layout and out of place in canonical order, pruning on, for
    # every tile width x persistent grid the autotuner may choose, each also
    # with the second sweep's rotated tile order; every candidate gives the
    # default schedule's bits, which match the definition on sampled strings
    n = 14
    torch.cuda.empty_cache()
    A = W.gaussian_device(n, seed=14, dtype=dtype, hermitian=True)
    a_max = float(torch.view_as_real(A).abs().max())
    qs = W.sampled_strings(n, 1500, seed=141)
    bf = sampled_oracle(A, n, qs)
    tol = n * U64 * a_max if dtype == torch.complex128 else (n + 1) * U32 * a_max
    qd = torch.from_numpy(qs.astype(np.int64)).to(DEV)
    h, l = deinterleave(qs.astype(np.int64))
    hb = torch.from_numpy(h).to(DEV)
    lb = torch.from_numpy(l).to(DEV)
    ref_can = tpd.decompose(A)
    assert cerr(ref_can[qd].cpu().numpy(), bf) <= tol
    B = A.clone()
    tpd.decompose(B, B.view(-1), layout="matrix")
    ref_mat = B.clone()
    assert cerr(ref_mat[hb, lb].cpu().numpy(), bf) <= tol
    out = torch.empty_like(ref_can)
    for db in dbs:
        for g in (0, 1, 2, 4, 8):
            for rot in (False, True):
                out.fill_(float("nan"))
                tpd.decompose_tuned(A, out, db=db, grid_per_cu=g, rotate=rot)
                assert torch.equal(torch.view_as_real(out), torch.view_as_real(ref_can)), ("canonical", db, g, rot)
                B.copy_(A)
                tpd.decompose_tuned(B, B.view(-1), db=db, grid_per_cu=g, layout="matrix", rotate=rot)
                assert torch.equal(torch.view_as_real(B), torch.view_as_real(ref_mat)), ("matrix", db, g, rot)
    # the chunked orders (2^cb d-groups per chunk, from the smallest chunk to
    # two chunks), on one stream and pipelined over two streams with 2 or 4
    # chunks between their sweeps
    for db in dbs:
        for cb in sorted({1, 4, n - db - 1}):
            for w in (0, 2, 4):
                out.fill_(float("nan"))
                tpd.decompose_tuned(A, out, db=db, grid_per_cu=8, chunk_bits=cb, chunk_window=w)
                assert torch.equal(torch.view_as_real(out), torch.view_as_real(ref_can)), ("canonical", db, cb, w)
                B.copy_(A)
                tpd.decompose_tuned(B, B.view(-1), db=db, grid_per_cu=8, layout="matrix", chunk_bits=cb,
                                    chunk_window=w)
                assert torch.equal(torch.view_as_real(B), torch.view_as_real(ref_mat)), ("matrix", db, cb, w)
    del A, B, ref_can, ref_mat, out
    torch.cuda.empty_cache()


# ----------------------------------------------------------------------------
# real input (real-coded weights): w_t = r_t for even #Y, i r_t for odd #Y
# ----------------------------------------------------------------------------
def y_odd(q):
    """True where the canonical index q has an odd number of Y (= 2) digits."""
    q = np.asarray(q, np.int64)
    par = np.zeros(q.shape, bool)
    for b in range(20):
        par ^= ((q >> (2 * b)) & 3) == 2
    return par


def real_coded(w, q):
    """(nonzero component, the other component) of complex weights w at q."""
    odd = y_odd(q)
    return np.where(odd, w.imag, w.real), np.where(odd, w.real, w.imag)


@pytest.mark.parametrize("n", [0, 1, 2, 5, 7, 8, 9, 11, 12])
def test_real_input_vs_algorithm_1(n):
    A = W.real_gaussian(n, seed=2200 + n) if n else np.array([[1.25]])
    ref = O.tpd_recursive(A.astype(np.complex128))
    exp, other = real_coded(ref, np.arange(4 ** n))
    assert np.all(other == 0)  # a real matrix: each weight real or imaginary
    Ad = torch.from_numpy(A).to(DEV)
    got = tpd.decompose(Ad)
    assert got.dtype == torch.float64
    # the complex path's nonzero component, value for value (== ignores the sign of zero)
    assert np.array_equal(got.cpu().numpy(), exp)
    assert np.array_equal(tpd.decompose(Ad, prune=False).cpu().numpy(), exp)
    # matrix layout, in place
    B = Ad.clone()
    tpd.decompose(B, B.view(-1), layout="matrix")
    assert np.array_equal(matrix_to_canonical(B.cpu().numpy().ravel(), n), exp)
    if n >= 9:
        out = torch.empty_like(got)
        for db in [b for b in (4, 5, 6) if b <= n // 2]:  # tiles fit the second sweep's x bits
            for g in (0, 1, 4):
                out.fill_(float("nan"))
                tpd.decompose_tuned(Ad, out, db=db, grid_per_cu=g)
                assert np.array_equal(out.cpu().numpy(), exp), (db, g)


@pytest.mark.parametrize("n", [0, 1, 3, 8, 9, 12])
def test_real_float32_input(n):
    # float32 real input: the complex64 path's nonzero component, value for
    # value (the same roundings), and within (n+1) 2^-24 max|a| of the oracle
    A = W.real_gaussian(n, seed=2400 + n) if n else np.array([[1.25]])
    A32 = A.astype(np.float32)
    ref = O.tpd_recursive(A32.astype(np.complex128))
    q = np.arange(4 ** n)
    exp, _ = real_coded(ref, q)
    Ad = torch.from_numpy(A32).to(DEV)
    got = tpd.decompose(Ad)
    assert got.dtype == torch.float32
    g = got.cpu().numpy()
    c64 = tpd.decompose(Ad.to(torch.complex64)).cpu().numpy()
    e64, o64 = real_coded(c64, q)
    assert np.all(o64 == 0) and np.array_equal(g, e64)
    a_max = float(np.max(np.abs(A32))) if n else 1.25
    assert np.max(np.abs(g.astype(np.float64) - exp)) <= (n + 1) * U32 * a_max
    B = Ad.clone()
    tpd.decompose(B, B.view(-1), layout="matrix")
    assert np.array_equal(matrix_to_canonical(B.cpu().numpy().ravel(), n), g)
    if n >= 9:
        S = torch.from_numpy(((A + A.T) / 2).astype(np.float32)).to(DEV)
        full = tpd.decompose(S).cpu().numpy()
        herm = tpd.decompose(S, hermitian=True).cpu().numpy()
        assert np.array_equal(full, herm) and np.all(herm[y_odd(q)] == 0)
        out = torch.empty_like(got)
        for db in [b for b in (4, 5, 6) if b <= n // 2]:
            for gp in (0, 1, 4):
                out.fill_(float("nan"))
                tpd.decompose_tuned(Ad, out, db=db, grid_per_cu=gp)
                assert np.array_equal(out.cpu().numpy(), g), (db, gp)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_real_partial_and_compaction(dtype):
    # requested real-coded values are those of the full real decomposition
    # (NaN past 4^n); the sparse list keeps |r| > tol in storage order
    n = 12
    npdt = np.float64 if dtype == torch.float64 else np.float32
    A = W.real_gaussian(n, seed=2500, symmetric=True).astype(npdt)
    Ad = torch.from_numpy(A).to(DEV)
    full = tpd.decompose(Ad).cpu().numpy()
    rng = np.random.default_rng(2501)
    q = np.concatenate([rng.integers(0, 4 ** n, 500), [0, 4 ** n - 1, 4 ** n, 4 ** n + 9]]).astype(np.int64)
    qd = torch.from_numpy(q).to(DEV)
    for kw in ({}, {"hermitian": True}, {"prune": False}):
        vals = tpd.decompose_partial(Ad, qd, **kw).cpu().numpy()
        assert vals.dtype == npdt
        assert np.array_equal(vals[:-2], full[q[:-2]]), kw
        assert np.all(np.isnan(vals[-2:])), kw
    B = Ad.clone()
    vals = tpd.decompose_partial(B, qd, work=B.view(-1), layout="matrix").cpu().numpy()
    assert np.array_equal(vals[:-2], full[q[:-2]])
    fd = torch.from_numpy(full).to(DEV)
    for tol in (0.0, 1e-3):
        qs, ws, total = tpd.compact(fd, tol=tol)
        keep = np.flatnonzero(~(np.abs(full) <= npdt(tol)))
        assert total == keep.size
        assert np.array_equal(qs.cpu().numpy(), keep) and np.array_equal(ws.cpu().numpy(), full[keep])
    # the transverse-field Ising chain: the list is exactly its 2n - 1 terms
    H = W.dense_from_terms_device(W.tfim_terms(n, 1.0, 0.5), n).real.to(dtype).contiguous()
    qs, ws, total = tpd.compact(tpd.decompose(H))
    expect = sorted((W.string_index(s_), c) for s_, c in W.tfim_terms(n, 1.0, 0.5))
    assert total == len(expect) == 2 * n - 1
    assert qs.cpu().numpy().tolist() == [k for k, _ in expect]
    assert np.array_equal(ws.cpu().numpy(), np.array([c.real for _, c in expect], npdt))


@pytest.mark.parametrize("n", [0, 1, 3, 8, 9, 12])
def test_real_synthesis(n):
    # real-coded weights back to the real matrix: the complex path's result
    # (which is real) value for value, integer weights exactly, and the
    # round trip through the real decomposition exact
    rng = np.random.default_rng(2600 + n)
    q = np.arange(4 ** n)
    odd = y_odd(q)
    r = rng.integers(-8, 9, 4 ** n).astype(np.float64)
    w = np.where(odd, 1j * r, r + 0j)  # the complex weights the real-coded r stand for
    ref = O.synthesize(w, n) if n <= 10 else None  # the oracle's sum costs 8^n
    assert ref is None or np.all(ref.imag == 0)  # such weights give a real matrix
    for dtype, cdtype in ((torch.float64, torch.complex128), (torch.float32, torch.complex64)):
        rd = torch.from_numpy(r).to(DEV).to(dtype)
        A = tpd.synthesize(rd)
        assert A.dtype == dtype and A.shape == (1 << n, 1 << n)
        Ac = tpd.synthesize(to_dev(w, cdtype)).cpu().numpy()
        assert np.array_equal(A.cpu().numpy(), Ac.real)
        if ref is not None:
            assert np.array_equal(A.cpu().numpy().astype(np.float64), ref.real)
        assert np.array_equal(tpd.decompose(A).cpu().numpy(), r.astype(A.cpu().numpy().dtype))
        # matrix layout, in place
        T = torch.from_numpy(canonical_to_matrix(r, n)).to(DEV).to(dtype).contiguous()
        tpd.synthesize(T, T.view(1 << n, 1 << n), layout="matrix")
        assert np.array_equal(T.view(1 << n, 1 << n).cpu().numpy(), A.cpu().numpy())


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_real_batched(dtype):
    # real matrices of mixed sizes in one persistent launch: each output is
    # the single-matrix real decomposition's, value for value; graph replay
    ns = [int(v) for v in W.batched_qubits(300, seed=27)]
    npdt = np.float64 if dtype == torch.float64 else np.float32
    mats = [W.real_gaussian(n, seed=2700 + k, symmetric=(k % 2 == 1)).astype(npdt) for k, n in enumerate(ns)]
    dm = [torch.from_numpy(m).to(DEV) for m in mats]
    refs = [tpd.decompose(m).cpu().numpy() for m in dm]
    outs = tpd.decompose_batched(dm)
    for k, (o, r) in enumerate(zip(outs, refs)):
        assert o.dtype == dtype and np.array_equal(o.cpu().numpy(), r), k
    code = tpd.TPD_R64 if dtype == torch.float64 else tpd.TPD_R32
    plan = tpd.BatchedPlan(ns, code)
    dp, do = tpd.BatchedPlan.pointer_table(dm), tpd.BatchedPlan.pointer_table(outs)
    s_ = torch.cuda.Stream()
    s_.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s_):
        plan.execute(dp, do)  # warm up on the capture stream
    torch.cuda.current_stream().wait_stream(s_)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        plan.execute(dp, do)
    for rep in range(2):
        for o in outs:
            o.fill_(float("nan"))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for k, (o, r) in enumerate(zip(outs, refs)):
            assert np.array_equal(o.cpu().numpy(), r), (rep, k)
    plan.close()
    # in place, matrix layout
    dm2 = [m.clone() for m in dm]
    tpd.decompose_batched(dm2, "inplace", layout="matrix")
    for k, (m, n) in enumerate(zip(dm2, ns)):
        assert np.array_equal(matrix_to_canonical(m.cpu().numpy().ravel(), n), refs[k]), k


@pytest.mark.parametrize("n", [9, 12, 13])
def test_real_symmetric_hermitian_mode(n):
    A = W.real_gaussian(n, seed=2300 + n, symmetric=True)
    ref = O.tpd_recursive(A.astype(np.complex128))
    q = np.arange(4 ** n)
    exp, _ = real_coded(ref, q)
    assert np.all(exp[y_odd(q)] == 0)  # odd-Y strings vanish for real-symmetric input
    Ad = torch.from_numpy(A).to(DEV)
    for layout in ("canonical", "matrix"):
        got = tpd.decompose(Ad, hermitian=True, layout=layout).cpu().numpy().ravel()
        if layout == "matrix":
            got = matrix_to_canonical(got, n)
        assert np.array_equal(got, exp), layout
    B = Ad.clone()
    tpd.decompose(B, B.view(-1), layout="matrix", hermitian=True)
    assert np.array_equal(matrix_to_canonical(B.cpu().numpy().ravel(), n), exp)


def test_real_tfim_pruning_and_exact_terms():
    # the transverse-field Ising chain is real symmetric: 2k+1 live CMWs,
    # and exactly its 2n-1 terms survive with their coefficients
    n = 12
    H = W.dense_from_terms_device(W.tfim_terms(n, 1.0, 0.5), n).real.contiguous()
    plan = tpd.Plan(n, tpd.TPD_R64)
    out = torch.empty(4 ** n, dtype=torch.float64, device=DEV)
    plan.execute(H, out)
    st = plan.prune_stats()
    assert st["live_prefixes"] == 2 * st["prefix_level"] + 1
    plan.close()
    got = out.cpu().numpy()
    expect = {}
    for s_, c in W.tfim_terms(n, 1.0, 0.5):
        expect[W.string_index(s_)] = c
    nz = np.flatnonzero(got)
    assert sorted(expect) == nz.tolist()
    assert all(got[k] == v.real for k, v in expect.items())


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("hermitian", [False, True])
def test_n16_real_in_place_every_tuning_candidate(hermitian, dtype):
    # the real path at full size: n = 16 real symmetric matrix in place,
    # every tile width and grid the autotuner may choose, sampled strings
    # against the definition
    n = 16
    torch.cuda.empty_cache()
    A = W.gaussian_device(n, seed=6, dtype=dtype, hermitian=True)
    a_max = float(A.abs().max())
    qs = W.sampled_strings(n, 2000, seed=26)
    bf = sampled_oracle(A, n, qs)
    exp, other = real_coded(bf, qs)
    assert np.max(np.abs(other)) <= n * U64 * a_max
    tol = n * U64 * a_max if dtype == torch.float64 else (n + 1) * U32 * a_max
    h, l = deinterleave(qs.astype(np.int64))
    hb = torch.from_numpy(h).to(DEV)
    lb = torch.from_numpy(l).to(DEV)
    B = torch.empty_like(A)
    B.copy_(A)
    tpd.decompose(B, B.view(-1), layout="matrix")
    ref = B[hb, lb].cpu().numpy()
    assert np.max(np.abs(ref.astype(np.float64) - exp)) <= tol
    assert np.all(ref[y_odd(qs)] == 0)
    for db in (4, 5, 6):
        for g in (0, 1, 2, 4, 8):
            B.copy_(A)
            tpd.decompose_tuned(B, B.view(-1), db=db, grid_per_cu=g, layout="matrix", hermitian=hermitian)
            assert np.array_equal(B[hb, lb].cpu().numpy(), ref), (db, g)
    del A, B
    torch.cuda.empty_cache()


# ----------------------------------------------------------------------------
# n = 17 (complex64 and the real dtypes): a first sweep of 9 levels
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("dtype", [torch.complex64, torch.float32, torch.float64])
def test_n17_in_place_sampled_strings(dtype):
    n = 17
    torch.cuda.empty_cache()
    A = W.gaussian_device(n, seed=17, dtype=dtype, hermitian=True)
    real = not A.is_complex()
    a_max = 0.0  # by row blocks: a full-size temporary would not fit beside A
    for r0 in range(0, 1 << n, 4096):
        blk = A[r0:r0 + 4096]
        a_max = max(a_max, float((blk.abs() if real else torch.view_as_real(blk).abs()).max()))
    qs = W.sampled_strings(n, 1000, seed=17)
    bf = sampled_oracle(A, n, qs)  # read before the in-place transform
    exp = real_coded(bf, qs)[0] if real else bf
    tol = n * U64 * a_max if dtype == torch.float64 else (n + 1) * U32 * a_max
    h, l = deinterleave(qs.astype(np.int64))
    hb = torch.from_numpy(h).to(DEV)
    lb = torch.from_numpy(l).to(DEV)
    pristine = A.clone() if dtype == torch.float32 else None  # 64 GiB: room for a copy
    tpd.decompose(A, A.view(-1), layout="matrix")
    ref = A[hb, lb].cpu().numpy()
    assert cerr(ref, exp) <= tol
    if real:
        assert np.all(ref[y_odd(qs)] == 0)  # real symmetric: no odd-Y weight
    if pristine is not None:
        # db 6 in the general mode: 2^6-diagonal tiles in the 8-level sweep,
        # 2^5 in the 9-level one (pruning bits per narrower d-group)
        for herm, dbs in ((False, (4, 5, 6)), (True, (4, 5))):
            for db in dbs:
                for g in (0, 4):
                    A.copy_(pristine)
                    tpd.decompose_tuned(A, A.view(-1), db=db, grid_per_cu=g, layout="matrix", hermitian=herm)
                    assert np.array_equal(A[hb, lb].cpu().numpy(), ref), (herm, db, g)
    del A, pristine
    torch.cuda.empty_cache()


def test_n17_hermitian_real_weights_complex64():
    # the largest real-weights case: n = 17 complex64 (128 GiB, destroyed),
    # 8 + 9 level split (the real-weights store in a 9-level, 2^14-element
    # tile), sampled weights against the definition, every weight written
    n = 17
    torch.cuda.empty_cache()
    A = W.gaussian_device(n, seed=1717, dtype=torch.complex64, hermitian=True)
    a_max = 0.0
    for r0 in range(0, 1 << n, 4096):
        a_max = max(a_max, float(torch.view_as_real(A[r0:r0 + 4096]).abs().max()))
    qs = W.sampled_strings(n, 1000, seed=1718)
    bf = sampled_oracle(A, n, qs)  # read before A is overwritten
    w = torch.full((4 ** n,), float("nan"), dtype=torch.float32, device=DEV)
    tpd.decompose_hermitian_real(A, w)
    del A
    torch.cuda.empty_cache()
    got = w[torch.from_numpy(qs.astype(np.int64)).to(DEV)].cpu().numpy().astype(np.float64)
    assert np.max(np.abs(got - bf.real)) <= (n + 1) * U32 * a_max
    nan = False
    for c0 in range(0, 4 ** n, 1 << 30):  # by blocks: no full-size temporary
        nan = nan or bool(torch.isnan(w[c0:c0 + (1 << 30)]).any())
    assert not nan
    del w
    torch.cuda.empty_cache()


def test_n17_real_tfim_pruning_with_split_tile_widths():
    # the transverse-field Ising chain at n = 17 (real float32, 64 GiB): its
    # X_i terms sit on single diagonals 2^i, so second-sweep d-groups of 2^5
    # inside first-sweep tiles of 2^6 diagonals are live or dead on their
    # own; the pruned result must still be exactly the 2n - 1 terms
    n = 17
    torch.cuda.empty_cache()
    terms = W.tfim_terms(n, 1.0, 0.5)
    H = W.dense_from_terms_device(terms, n, dtype=torch.float32)
    sched = tpd.schedule(n, tpd.TPD_R32, tpd.FLAG_LAYOUT_MATRIX, in_place=True)
    tpd.decompose_tuned(H, H.view(-1), db=6, grid_per_cu=4, layout="matrix")
    # the nonzero weights through the library's compaction (64-bit counts)
    qs, ws, total = tpd.compact(H.view(-1), layout="matrix")
    got = dict(zip(qs.cpu().numpy().tolist(), ws.cpu().numpy().tolist()))
    expect = {W.string_index(s_): float(np.real(c)) for s_, c in terms}
    assert total == 2 * n - 1 and got == expect
    del H
    torch.cuda.empty_cache()
    assert sched["sweeps"][0]["db"] in (5, 6)


def test_n17_real_split_widths_prune_stats_and_partial():
    # real float32, matrix layout, n = 17: the default schedule gives the two
    # sweeps different tile widths (2^6 and 2^5 diagonals).  The pruning
    # bitmap has one bit per second-sweep tile, so the live level-8 CMWs of
    # the Ising chain (2k + 1 = 17, section "Results") and the partial
    # decomposition's request tiles must be counted at the second sweep's width.
    n = 17
    torch.cuda.empty_cache()
    terms = W.tfim_terms(n, 1.0, 0.5)
    expect = {W.string_index(s_): float(np.real(c)) for s_, c in terms}
    H = W.dense_from_terms_device(terms, n, dtype=torch.float32)
    plan = tpd.Plan(n, tpd.TPD_R32, layout="matrix", in_place=True)
    sw = plan.describe()["sweeps"]
    plan.execute(H, H.view(-1))
    st = plan.prune_stats()
    plan.close()
    assert st["prefix_level"] == 8 and st["live_prefixes"] == 2 * 8 + 1, (sw, st)
    qs, ws, total = tpd.compact(H.view(-1), layout="matrix")
    assert total == 2 * n - 1
    assert dict(zip(qs.cpu().numpy().tolist(), ws.cpu().numpy().tolist())) == expect
    del H
    torch.cuda.empty_cache()
    # partial, bottom-first order (default widths, split like the plan above)
    H = W.dense_from_terms_device(terms, n, dtype=torch.float32)
    rng = np.random.default_rng(1717)
    req = np.concatenate([np.array(sorted(expect), np.int64), two_local(n),
                          rng.integers(0, 4 ** n, 2000, dtype=np.int64)])
    vals = tpd.decompose_partial(H, torch.from_numpy(req).to(DEV), work=H.view(-1), layout="matrix",
                                 order_bottom=True).cpu().numpy()
    want = np.array([expect.get(int(q), 0.0) for q in req], np.float32)
    assert np.array_equal(vals, want)
    del H
    torch.cuda.empty_cache()
    assert sw[0]["db"] == 6 and sw[1]["db"] == 5, sw


@pytest.mark.parametrize("dtype,code", [(torch.complex128, tpd.TPD_C128), (torch.complex64, tpd.TPD_C64),
                                        (torch.float64, tpd.TPD_R64)])
def test_n16_tfim_pruning_lane_group_bits(dtype, code):
    # n = 16: the first sweep transforms 8 levels, and each lane group ORs
    # its rows' pruning bits into one bitmap word; the transverse-field Ising
    # chain's live prefixes follow the closed form 2k + 1, and the result is
    # exactly its 2n - 1 terms, out of place (canonical) and in place (matrix)
    n = 16
    torch.cuda.empty_cache()
    terms = W.tfim_terms(n, 1.0, 0.5)
    expect = {W.string_index(s_): complex(c) for s_, c in terms}
    H = W.dense_from_terms_device(terms, n, dtype=dtype)
    out = torch.empty(4 ** n, dtype=dtype, device=DEV)
    for layout, in_place in (("canonical", False), ("matrix", True)):
        plan = tpd.Plan(n, code, layout=layout, in_place=in_place)
        dst = H.view(-1) if in_place else out
        plan.execute(H, dst)
        st = plan.prune_stats()
        plan.close()
        assert st["live_prefixes"] == 2 * st["prefix_level"] + 1, (layout, st)
        assert 0 < st["live_tiles"] < st["total_tiles"], (layout, st)
        qs, ws, total = tpd.compact(dst, layout=layout)
        got = {int(q): complex(w) for q, w in zip(qs.cpu().numpy(), ws.cpu().numpy())}
        assert total == 2 * n - 1 and got == expect, layout
    del H, out
    torch.cuda.empty_cache()


@pytest.mark.parametrize("dtype", [torch.complex64, torch.float32])
def test_n17_round_trip_in_place_integer_exact(dtype):
    # integer weights synthesized in place into the 131072 x 131072 matrix
    # and decomposed back in place: exact
    n = 17
    m = 4 ** n
    torch.cuda.empty_cache()
    gen = torch.Generator(device=DEV)
    gen.manual_seed(1717)
    T = torch.empty(m, dtype=dtype, device=DEV)
    Tr = torch.view_as_real(T) if T.is_complex() else T.view(-1, 1)
    step = 1 << 28
    for c in range(0, m, step):
        for k in range(Tr.shape[1]):
            Tr[c:c + step, k].copy_(torch.randint(-8, 9, (min(step, m - c),), generator=gen, device=DEV))
    probe = torch.randint(0, m, (4096,), generator=gen, device=DEV)
    before = T[probe].cpu().numpy()
    def total(t):  # exact for these integers; by chunks to stay small
        v = torch.view_as_real(t).reshape(-1) if t.is_complex() else t
        return sum(float(v[c:c + step].double().sum()) for c in range(0, v.numel(), step))

    checksum = total(T)
    M = T.view(1 << n, 1 << n)
    tpd.synthesize(T, M, layout="matrix")
    tpd.decompose(M, T, layout="matrix")
    assert np.array_equal(T[probe].cpu().numpy(), before)
    assert total(T) == checksum
    del T, M
    torch.cuda.empty_cache()


# ----------------------------------------------------------------------------
# edge cases, determinism, poison fill, errors
# ----------------------------------------------------------------------------
def test_edge_cases():
    # zero matrix: everything pruned, output all zeros (written over NaN poison)
    for n in (3, 10, 13):
        Z = torch.zeros((1 << n, 1 << n), dtype=torch.complex128, device=DEV)
        out = torch.full((4 ** n,), float("nan"), dtype=torch.complex128, device=DEV)
        tpd.decompose(Z, out)
        assert float(torch.view_as_real(out).abs().max()) == 0.0
    # identity -> e_0 ; single strings -> unit vectors
    for n in (5, 11):
        I = torch.eye(1 << n, dtype=torch.complex128, device=DEV)
        out = tpd.decompose(I).cpu().numpy()
        e = np.zeros(4 ** n)
        e[0] = 1
        assert same_bits(out, e)
    rng = np.random.default_rng(9)
    for n in (9, 13):
        for _ in range(3):
            s = "".join("IXYZ"[int(v)] for v in rng.integers(0, 4, n))
            S = W.dense_from_terms_device([(s, 1.0 + 0j)], n)
            out = tpd.decompose(S)
            q = W.string_index(s)
            assert complex(out[q]) == 1.0
            out[q] = 0
            assert float(torch.view_as_real(out).abs().max()) == 0.0
    # NaN propagates along its X/Y mask only
    n = 11
    A = torch.zeros((1 << n, 1 << n), dtype=torch.complex128, device=DEV)
    A[5, 9] = float("nan")
    out = tpd.decompose(A).cpu().numpy()
    sample = np.arange(0, 4 ** n, 1013)
    masks = np.array([O.xy_mask(int(q), n) for q in sample])
    assert np.all(np.isnan(out[sample[masks == (5 ^ 9)]]))
    assert np.all(out[sample[masks != (5 ^ 9)]] == 0)


def test_determinism_and_poison():
    n = 13
    A = W.gaussian_device(n, seed=11)
    o1 = torch.full((4 ** n,), float("nan"), dtype=torch.complex128, device=DEV)
    o2 = torch.full((4 ** n,), float("nan"), dtype=torch.complex128, device=DEV)
    tpd.decompose(A, o1)
    tpd.decompose(A, o2)
    assert not bool(torch.isnan(torch.view_as_real(o1)).any())
    assert torch.equal(torch.view_as_real(o1), torch.view_as_real(o2))


def test_pipelined_chunk_schedule_from_the_cache_plan_graph_and_noalloc():
    # a cached pipelined chunk schedule (n = 12 complex128 out of place: tile
    # width 2^4, 64 chunks, window 2) reaches tpd_decompose_ex (a second
    # stream per caller stream), a plan (its own stream), a captured graph of
    # that plan (the second stream joins the capture through events), and
    # the no-allocation entry point (chunks on the caller's stream only); all
    # give the bits of the whole-sweep schedule
    import subprocess
    import sys
    import tempfile
    import textwrap

    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    with tempfile.TemporaryDirectory() as td:
        cache = os.path.join(td, "tune.txt")
        code = textwrap.dedent("""
            import json, os, sys
            sys.path.insert(0, %r)
            import torch
            cus = torch.cuda.get_device_properties(0).multi_processor_count
            with open(os.environ["TPD_AUTOTUNE_CACHE"], "w") as f:
                f.write("tpd-tune-v2 gfx950 %%d 0 12 0 0 0 4 4 8 0 2 2\\n" %% cus)
            from paper_2310_13421_amd import tpd
            import workloads as W
            A = torch.from_numpy(W.gaussian(12, seed=1201)).to("cuda")
            ref = tpd.decompose_tuned(A, db=4, grid_per_cu=8)
            eq = lambda o: bool(torch.equal(torch.view_as_real(o), torch.view_as_real(ref)))
            ok = []
            ok.append(eq(tpd.decompose(A)))
            plan = tpd.Plan(12)
            d = plan.describe()
            ok.append(d["chunk_bits"] == 2 and d["chunk_window"] == 2)
            out = torch.empty_like(ref)
            s = torch.cuda.Stream()
            s.wait_stream(torch.cuda.current_stream())
            with torch.cuda.stream(s):
                plan.execute(A, out)
            torch.cuda.current_stream().wait_stream(s)
            torch.cuda.synchronize()
            ok.append(eq(out))
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g):
                plan.execute(A, out)
            for _ in range(3):
                out.fill_(float("nan"))
                torch.cuda.synchronize()
                g.replay()
                torch.cuda.synchronize()
                ok.append(eq(out))
            out2 = torch.empty_like(ref)
            tpd.decompose_noalloc(A, out2)
            torch.cuda.synchronize()
            ok.append(eq(out2))
            plan.close()
            print("RESULT", json.dumps(ok), flush=True)
        """ % root)
        env = dict(os.environ, TPD_AUTOTUNE_CACHE=cache)
        r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, r.stderr[-2000:]
    line = [ln for ln in r.stdout.splitlines() if ln.startswith("RESULT")][-1]
    import json
    assert all(json.loads(line.split(" ", 1)[1])), line


def test_allocation_failure_hook_reports_out_of_memory():
    # TPD_TEST_FAIL_ALLOC=1 makes every library allocation fail: plan
    # creation and the workspace of a pruned decomposition report
    # TPD_ERROR_OUT_OF_MEMORY, while calls that need no allocation (pruning
    # off, the no-allocation entry point) still run and agree bitwise
    import subprocess
    import sys
    import textwrap

    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = textwrap.dedent("""
        import ctypes, sys
        sys.path.insert(0, %r)
        import torch
        from paper_2310_13421_amd import tpd
        import workloads as W
        A = torch.from_numpy(W.gaussian(9, seed=77)).to("cuda")
        o1 = torch.empty(4 ** 9, dtype=A.dtype, device="cuda")
        o2 = torch.empty(4 ** 9, dtype=A.dtype, device="cuda")
        h = ctypes.c_void_p()
        rc_plan = tpd.lib.tpd_plan_create(9, tpd.TPD_C128, 0, 0, ctypes.byref(h))
        rc_ws = tpd.lib.tpd_decompose_ex(A.data_ptr(), 9, o1.data_ptr(), tpd.TPD_C128, 0, None)
        rc_np = tpd.lib.tpd_decompose_ex(A.data_ptr(), 9, o1.data_ptr(), tpd.TPD_C128, tpd.FLAG_NO_PRUNE, None)
        rc_na = tpd.lib.tpd_decompose_noalloc(A.data_ptr(), 9, o2.data_ptr(), tpd.TPD_C128, 0, None)
        torch.cuda.synchronize()
        same = bool(torch.equal(torch.view_as_real(o1), torch.view_as_real(o2)))
        print("RESULT", rc_plan, rc_ws, rc_np, rc_na, int(same), flush=True)
    """ % root)
    env = dict(os.environ, TPD_TEST_FAIL_ALLOC="1")
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=240, env=env)
    assert r.returncode == 0, r.stderr[-2000:]
    line = [ln for ln in r.stdout.splitlines() if ln.startswith("RESULT")][0].split()[1:]
    assert line == ["3", "3", "0", "0", "1"], (line, r.stderr[-1000:])


def test_device_errors_do_not_launch():
    A = torch.zeros((16, 16), dtype=torch.complex128, device=DEV)
    out = torch.empty(256, dtype=torch.complex128, device=DEV)
    assert tpd.lib.tpd_decompose_ex(A.data_ptr() + 8, 4, out.data_ptr(), 0, 0, None) == 1
    assert tpd.lib.tpd_decompose_ex(A.data_ptr(), 4, A.data_ptr() + 16, 0, 0, None) == 1
    assert tpd.lib.tpd_decompose_ex(A.data_ptr(), 17, out.data_ptr(), 0, 0, None) == 2
    torch.cuda.synchronize()


def test_single_plan_graph_capture_and_timing():
    n = 12
    A = W.gaussian(n, seed=12)
    ref = O.tpd_recursive(A)
    Ad = to_dev(A)
    out = torch.empty(4 ** n, dtype=torch.complex128, device=DEV)
    plan = tpd.Plan(n, timing=True)
    assert plan.num_kernels() == 2
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        plan.execute(Ad, out)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    ms, cnt = plan.timing(reset=True)
    assert cnt == [1, 1] and all(t > 0 for t in ms)
    plan.close()
    plan = tpd.Plan(n)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        plan.execute(Ad, out)
    for _ in range(3):
        out.fill_(float("nan"))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert same_bits(out.cpu().numpy(), ref)
    plan.close()


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_real_plan_graph_capture(dtype):
    # a real-input plan (pruning bitmap, rotated second-sweep order) captured
    # once and replayed, with eager work between the replays
    n = 12
    A = W.real_gaussian(n, seed=1212, symmetric=True).astype(np.float64 if dtype == torch.float64 else np.float32)
    Ad = torch.from_numpy(A).to(DEV)
    ref = tpd.decompose(Ad).cpu().numpy()
    code = tpd.TPD_R64 if dtype == torch.float64 else tpd.TPD_R32
    out = torch.empty(4 ** n, dtype=dtype, device=DEV)
    for flags in ({}, {"hermitian": True, "rotate": True}):
        plan = tpd.Plan(n, code, **flags)
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            plan.execute(Ad, out)  # warm up on the capture stream
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            plan.execute(Ad, out)
        for _ in range(3):
            out.fill_(float("nan"))
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            assert np.array_equal(out.cpu().numpy(), ref), flags
        plan.close()


def test_autotune_keeps_results_bitwise():
    for n, dtype in ((11, torch.complex128), (12, torch.complex64)):
        A = to_dev(W.gaussian(n, seed=90 + n), dtype)
        before = tpd.decompose(A).clone()
        rep = tpd.autotune(A)
        assert rep["tuned"] and len(rep["candidates"]) >= 4
        after = tpd.decompose(A)
        assert torch.equal(torch.view_as_real(before), torch.view_as_real(after))
        if dtype == torch.complex128:
            assert same_bits(after.cpu().numpy(), O.tpd_recursive(W.gaussian(n, seed=90 + n)))
    rep = tpd.autotune(to_dev(W.gaussian(6, 1)))
    assert rep["tuned"] is False
    # in place the tuner refills its buffer with seeded noise before every
    # timed run: the buffer ends holding a transform of noise (live values),
    # not the decayed result of dozens of repeated transforms, which in
    # float32 is all zeros; the choice keeps the bits
    for n, dtype in ((12, torch.float32), (12, torch.complex128)):
        A = to_dev(W.gaussian(n, seed=95).real.copy() if dtype == torch.float32 else W.gaussian(n, seed=95), dtype)
        ref = A.clone()
        tpd.decompose(ref, ref.view(-1), layout="matrix")
        B = A.clone()
        rep = tpd.autotune(B, B.view(-1), layout="matrix")
        assert rep["tuned"] and len(rep["candidates"]) >= 4
        live = torch.view_as_real(B) if B.is_complex() else B
        assert float((live != 0).double().mean()) > 0.9, dtype
        assert bool(torch.isfinite(live).all())
        B.copy_(A)
        tpd.decompose(B, B.view(-1), layout="matrix")
        assert torch.equal(torch.view_as_real(B) if B.is_complex() else B,
                           torch.view_as_real(ref) if ref.is_complex() else ref), dtype
    # batched plan autotune
    ns = [int(v) for v in W.batched_qubits(200, seed=13)]
    mats = W.batched_matrices(ns, seed=13)
    dm = [to_dev(m) for m in mats]
    outs = [torch.empty(4 ** n, dtype=torch.complex128, device=DEV) for n in ns]
    plan = tpd.BatchedPlan(ns)
    dp, do = tpd.BatchedPlan.pointer_table(dm), tpd.BatchedPlan.pointer_table(outs)
    rep = plan.autotune(dp, do)
    assert rep["tuned"] and rep["chosen"]["grid"] > 0
    for o in outs:
        o.fill_(float("nan"))
    plan.execute(dp, do)
    torch.cuda.synchronize()
    for k, (o, m) in enumerate(zip(outs, mats)):
        assert same_bits(o.cpu().numpy(), O.tpd_recursive(m)), k
    plan.close()


@pytest.mark.parametrize("n", [9, 12, 13])
def test_hermitian_mode(n):
    A = W.gaussian(n, seed=70 + n, hermitian=True)
    ref = O.tpd_recursive(A)
    for dtype in (torch.complex128, torch.complex64):
        Ad = to_dev(A, dtype)
        gen = tpd.decompose(Ad)
        for layout in ("canonical", "matrix"):
            out = torch.full((4 ** n,), float("nan"), dtype=dtype, device=DEV)
            tpd.decompose(Ad, out, hermitian=True, layout=layout)
            got = out.cpu().numpy()
            if layout == "matrix":
                got = matrix_to_canonical(got, n)
            assert np.all(got.imag == 0)
            assert np.array_equal(got.real, gen.cpu().numpy().real)
            if dtype == torch.complex128:
                assert same_bits(got, ref)
        # in place, matrix layout
        T = Ad.clone()
        tpd.decompose(T, T.view(-1), hermitian=True, layout="matrix")
        got = matrix_to_canonical(T.cpu().numpy().ravel(), n)
        assert np.array_equal(got.real, gen.cpu().numpy().real) and np.all(got.imag == 0)


def _terms_dense_expect(terms, n, dtype):
    """Dense expected weights on the device: the generating coefficients at
    their canonical indices, zeros elsewhere."""
    qs = torch.tensor([W.string_index(s) for s, _ in terms], dtype=torch.int64, device=DEV)
    cs = torch.tensor(np.array([c for _, c in terms], np.complex128), device=DEV)
    exp = torch.zeros(4 ** n, dtype=torch.complex128, device=DEV)
    exp.index_put_((qs,), cs, accumulate=True)
    return exp.to(dtype) if dtype.is_complex else exp.real.to(dtype).contiguous()


def _dev_matrix_to_canonical(M, n):
    """Matrix-layout weights (device) to canonical order (device)."""
    d = 1 << n
    h = torch.arange(d, device=DEV, dtype=torch.int64)
    sp = torch.zeros_like(h)
    for b in range(n):
        sp |= ((h >> b) & 1) << (2 * b)
    q = ((sp[:, None] << 1) | sp[None, :]).reshape(-1)
    out = torch.empty(4 ** n, dtype=M.dtype, device=DEV)
    out[q] = M.reshape(-1)
    return out


def _exactly(a, b):
    """Same values everywhere (-0 == +0, NaN never equal)."""
    if a.is_complex():
        a, b = torch.view_as_real(a), torch.view_as_real(b)
    return bool(torch.equal(a, b))


@pytest.mark.parametrize("case", ["tfim10", "tfim12", "heisenberg14"])
def test_hermitian_mode_structured_input_with_pruning(case):
    # Hermitian mode with pruning on: the first sweep writes representative
    # rows only, so a zero second-sweep tile must still store zeros on its
    # mirrored rows.  Outputs start NaN-poisoned (out of place) or hold the
    # input (in place); complex128 must give exactly the generating terms,
    # complex64 the general path's real parts with imaginary parts 0.
    if case.startswith("tfim"):
        n = int(case[4:])
        terms = W.tfim_terms(n, 1.0, 0.5)
    else:
        n = 14
        terms = W.heisenberg_terms(n, seed=3, n_local=200, dyadic=True)
    H = W.dense_from_terms_device(terms, n)
    for dtype in (torch.complex128, torch.complex64):
        Hd = H if dtype == torch.complex128 else H.to(dtype)
        gen = tpd.decompose(Hd)
        exp = _terms_dense_expect(terms, n, dtype) if dtype == torch.complex128 else torch.complex(
            gen.real, torch.zeros_like(gen.real))
        for layout in ("canonical", "matrix"):
            out = torch.full((4 ** n,), float("nan"), dtype=dtype, device=DEV)
            tpd.decompose(Hd, out, hermitian=True, layout=layout)
            got = out if layout == "canonical" else _dev_matrix_to_canonical(out, n)
            assert _exactly(got, exp), (case, dtype, layout)
        T = Hd.clone()
        tpd.decompose(T, T.view(-1), hermitian=True, layout="matrix")
        assert _exactly(_dev_matrix_to_canonical(T.view(-1), n), exp), (case, dtype, "in place")
        # real weights into a separate NaN-poisoned array: zero tiles store
        # zeros on every weight
        T.copy_(Hd)
        rdt = torch.float64 if dtype == torch.complex128 else torch.float32
        w = torch.full((4 ** n,), float("nan"), dtype=rdt, device=DEV)
        tpd.decompose_hermitian_real(T, w)
        assert _exactly(w, exp.real.contiguous()), (case, dtype, "real weights")
        del Hd, gen, exp, T, w
    del H
    torch.cuda.empty_cache()


@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
def test_hermitian_real_weights_vs_complex_mode(dtype):
    # tpd_decompose_hermitian_real for n = 0..12: the real weights, written
    # into a NaN-poisoned array, are bitwise the real parts of the complex
    # Hermitian mode (complex128: of Algorithm 1 for n <= 10); with and
    # without pruning; the matrix is destroyed for n >= 9 only
    rdt = torch.float64 if dtype == torch.complex128 else torch.float32
    for n in range(0, 13):
        A = W.gaussian(n, seed=1700 + n, hermitian=True)
        Ad = to_dev(A, dtype)
        ref = tpd.decompose(Ad, hermitian=True)
        for prune in (True, False):
            B = Ad.clone()
            w = torch.full((4 ** n,), float("nan"), dtype=rdt, device=DEV)
            tpd.decompose_hermitian_real(B, w, prune=prune)
            assert torch.equal(w, ref.real.contiguous()), (n, prune)
            if n <= 8:
                assert torch.equal(torch.view_as_real(B), torch.view_as_real(Ad)), n  # one sweep: A unchanged
        if dtype == torch.complex128 and n <= 10:
            assert same_bits(w.cpu().numpy(), O.tpd_recursive(A).real), n


@pytest.mark.parametrize("dtype,dbs", [(torch.complex128, (3, 4, 5)), (torch.complex64, (4, 5, 6))])
def test_hermitian_real_weights_every_tile_width_and_grid(dtype, dbs):
    # n = 14: every tile width and grid the real-weights path can take gives
    # the default schedule's bits
    n = 14
    torch.cuda.empty_cache()
    A = W.gaussian_device(n, seed=24, dtype=dtype, hermitian=True)
    rdt = torch.float64 if dtype == torch.complex128 else torch.float32
    B = A.clone()
    ref = tpd.decompose_hermitian_real(B)
    w = torch.empty_like(ref)
    for db in dbs:
        for g in (0, 2, 8):
            B.copy_(A)
            w.fill_(float("nan"))
            tpd.decompose_hermitian_real(B, w, db=db, grid_per_cu=g)
            assert torch.equal(w, ref), (db, g)
    assert ref.dtype == rdt
    # the real-weights autotuner (on B, destroyed) keeps the bits
    B.copy_(A)
    rep = tpd.autotune_hermitian_real(B, w)
    assert rep["tuned"] and rep["chosen"]["db"] in dbs
    B.copy_(A)
    w.fill_(float("nan"))
    tpd.decompose_hermitian_real(B, w)
    assert torch.equal(w, ref)
    del A, B, ref, w
    torch.cuda.empty_cache()


def test_hermitian_real_weights_n16_full_size():
    # the n = 16 headline matrix: sampled weights against the definition, and
    # 10^5 sampled weights bitwise against the complex Hermitian mode in place
    n = 16
    torch.cuda.empty_cache()
    A = W.gaussian_device(n, seed=5, hermitian=True)
    a_max = float(torch.view_as_real(A).abs().max())
    qs = W.sampled_strings(n, 2000, seed=161)
    bf = sampled_oracle(A, n, qs)
    B = A.clone()
    w = torch.full((4 ** n,), float("nan"), dtype=torch.float64, device=DEV)
    tpd.decompose_hermitian_real(B, w)
    del B
    torch.cuda.empty_cache()
    got = w[torch.from_numpy(qs.astype(np.int64)).to(DEV)].cpu().numpy()
    assert np.max(np.abs(got - bf.real)) <= n * U64 * a_max
    assert not torch.isnan(w).any()
    tpd.decompose(A, A.view(-1), hermitian=True, layout="matrix")
    qs2 = W.sampled_strings(n, 100000, seed=162).astype(np.int64)
    h, l = deinterleave(qs2)
    ref = A[torch.from_numpy(h).to(DEV), torch.from_numpy(l).to(DEV)].real
    assert torch.equal(w[torch.from_numpy(qs2).to(DEV)], ref)
    del A, w
    torch.cuda.empty_cache()


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_real_symmetric_mode_structured_input_with_pruning(dtype):
    # the transverse-field Ising chain is real symmetric: real-coded weights
    # in the real-symmetric (Hermitian) mode with zero tiles pruned, NaN-
    # poisoned output and in place, equal the 2n - 1 generating terms
    n = 12
    terms = W.tfim_terms(n, 1.0, 0.5)
    H = W.dense_from_terms_device(terms, n).real.to(dtype).contiguous()
    exp = _terms_dense_expect(terms, n, dtype)
    for layout in ("canonical", "matrix"):
        out = torch.full((4 ** n,), float("nan"), dtype=dtype, device=DEV)
        tpd.decompose(H, out, hermitian=True, layout=layout)
        got = out if layout == "canonical" else _dev_matrix_to_canonical(out, n)
        assert _exactly(got, exp), layout
    T = H.clone()
    tpd.decompose(T, T.view(-1), hermitian=True, layout="matrix")
    assert _exactly(_dev_matrix_to_canonical(T.view(-1), n), exp)


@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
def test_partial_hermitian_structured_every_string(dtype):
    # every string requested from a structured Hermitian input: requests on
    # the mirrored rows of zero tiles must read the zeros the second sweep
    # stores there (work array NaN-poisoned; in place in the matrix layout)
    n = 12
    terms = W.heisenberg_terms(n, seed=12, n_local=60, dyadic=True)
    H = W.dense_from_terms_device(terms, n).to(dtype)
    full = tpd.decompose(H)
    exp = torch.complex(full.real, torch.zeros_like(full.real))
    q = torch.arange(4 ** n, dtype=torch.int64, device=DEV)
    work = torch.full((4 ** n,), float("nan"), dtype=dtype, device=DEV)
    vals = tpd.decompose_partial(H, q, work=work, hermitian=True)
    assert _exactly(vals, exp)
    T = H.clone()
    vals = tpd.decompose_partial(T, q, work=T.view(-1), layout="matrix", hermitian=True)
    assert _exactly(vals, exp)
    if dtype == torch.complex128:
        assert _exactly(full, _terms_dense_expect(terms, n, dtype))


# ----------------------------------------------------------------------------
# inverse transform (synthesis) and round trips
# ----------------------------------------------------------------------------
def canonical_to_matrix(w, n):
    d = 1 << n
    h = np.arange(d, dtype=np.int64)[:, None]
    l = np.arange(d, dtype=np.int64)[None, :]
    q = (spread(h) << 1) | spread(l)
    return np.asarray(w).reshape(-1)[q.ravel()].copy()


@pytest.mark.parametrize("n", [0, 1, 4, 8, 9, 10])  # the oracle's sum costs 8^n: n = 12 takes minutes
def test_synthesize_vs_oracle(n):
    rng = np.random.default_rng(1200 + n)
    w = rng.standard_normal(4 ** n) + 1j * rng.standard_normal(4 ** n)
    ref = O.synthesize(w, n)
    # level tree (n u 2^n max|w|) plus the oracle's sequential sum (2^n u 2^n max|w|)
    bound64 = (n + (1 << n)) * U64 * (1 << n) * amax(w)
    for dtype, bound in ((torch.complex128, bound64),
                         (torch.complex64, (n + 1) * U32 * (1 << n) * amax(w) * 1.01 + bound64)):
        got = tpd.synthesize(to_dev(w, dtype)).cpu().numpy()
        assert cerr(got, ref) <= bound, (n, dtype)
        wm = to_dev(canonical_to_matrix(w, n), dtype)
        gm = tpd.synthesize(wm, layout="matrix").cpu().numpy()
        assert same_bits(gm, got)
        T = wm.clone()
        tpd.synthesize(T, T.view(1 << n, 1 << n), layout="matrix")
        assert same_bits(T.view(1 << n, 1 << n).cpu().numpy(), got)


@pytest.mark.parametrize("n", [3, 10, 13])
def test_synthesize_integer_exact_and_round_trip(n):
    rng = np.random.default_rng(1300 + n)
    w = (rng.integers(-8, 9, 4 ** n) + 1j * rng.integers(-8, 9, 4 ** n)).astype(np.complex128)
    for dtype in (torch.complex128, torch.complex64):
        A = tpd.synthesize(to_dev(w, dtype))
        if n <= 10:
            assert same_bits(A.cpu().numpy().astype(np.complex128), O.synthesize(w, n))
        back = tpd.decompose(A).cpu().numpy().astype(np.complex128)
        assert same_bits(back, w), (n, dtype)


@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
def test_n16_round_trip_in_place_integer_exact(dtype):
    # 4^16 integer weights synthesized in place into the 65536 x 65536 matrix
    # and decomposed back in place: exact at full size.  With the forward
    # transform checked at this size against the definition, the exact round
    # trip pins the synthesis as its inverse.
    n = 16
    m = 4 ** n
    gen = torch.Generator(device=DEV)
    gen.manual_seed(16)
    re = torch.randint(-8, 9, (m,), generator=gen, device=DEV, dtype=torch.int8)
    im = torch.randint(-8, 9, (m,), generator=gen, device=DEV, dtype=torch.int8)
    T = torch.empty(m, dtype=dtype, device=DEV)
    Tr = torch.view_as_real(T)
    step = 1 << 28
    for c in range(0, m, step):
        Tr[c:c + step, 0].copy_(re[c:c + step])
        Tr[c:c + step, 1].copy_(im[c:c + step])
    M = T.view(1 << n, 1 << n)
    tpd.synthesize(T, M, layout="matrix")
    # Tr(A) = 2^n w_(I...I); the identity string sits at index 0 of either layout
    tr = M.diagonal().to(torch.complex128).sum().item()
    assert tr == complex(float(re[0]), float(im[0])) * (1 << n)
    torch.cuda.synchronize()
    tpd.decompose(M, T, layout="matrix")
    torch.cuda.synchronize()
    for c in range(0, m, step):
        assert torch.equal(Tr[c:c + step, 0], re[c:c + step].to(Tr.dtype))
        assert torch.equal(Tr[c:c + step, 1], im[c:c + step].to(Tr.dtype))
    del T, re, im
    torch.cuda.empty_cache()


# ----------------------------------------------------------------------------
# partial decomposition and sparse-list output
# ----------------------------------------------------------------------------
def two_local(n):
    qs = {0}
    for i in range(n):
        for a in (1, 2, 3):
            qs.add(a << (2 * (n - 1 - i)))
            for j in range(i + 1, n):
                for b in (1, 2, 3):
                    qs.add((a << (2 * (n - 1 - i))) | (b << (2 * (n - 1 - j))))
    return np.array(sorted(qs), np.int64)


@pytest.mark.parametrize("n", [0, 3, 8, 9, 12])
def test_partial_vs_algorithm_3(n):
    A = W.gaussian(n, seed=1400 + n) if n else np.array([[1.5 - 0.25j]])
    rng = np.random.default_rng(1500 + n)
    q = np.concatenate([rng.integers(0, 4 ** n, 300, dtype=np.int64), two_local(n) if n else [0]])
    ref = O.tpd_partial(A, q)
    Ad = to_dev(A)
    qd = torch.from_numpy(q).to(DEV)
    got = tpd.decompose_partial(Ad, qd).cpu().numpy()
    assert same_bits(got, ref)
    if n >= 9:
        g2 = tpd.decompose_partial(Ad.clone(), qd, work=None, layout="matrix", prune=False).cpu().numpy()
        assert same_bits(g2, ref)
        T = Ad.clone()
        g3 = tpd.decompose_partial(T, qd, work=T.view(-1), layout="matrix").cpu().numpy()
        assert same_bits(g3, ref)
        # complex64: the requested values are bitwise the full decomposition's,
        # which is within (n + 1) u max|a| (input rounding plus n levels)
        A32 = to_dev(A, torch.complex64)
        g64 = tpd.decompose_partial(A32, qd).cpu().numpy()
        f64 = tpd.decompose(A32).cpu().numpy()
        assert same_bits(g64, f64[q])
        assert cerr(g64, ref) <= (n + 1) * U32 * amax(A)


def test_config2_n14_partial_and_sparse_list():
    n = 14
    terms = W.heisenberg_terms(n, seed=3, dyadic=True)
    expect = {}
    for s, c in terms:
        expect[W.string_index(s)] = expect.get(W.string_index(s), 0) + c
    expect = {k: v for k, v in expect.items() if v != 0}
    H = W.dense_from_terms_device(terms, n)
    # partial: the generating strings, every 2-local string and some others
    rng = np.random.default_rng(14)
    q = np.unique(np.concatenate([np.array(sorted(expect), np.int64), two_local(n),
                                  rng.integers(0, 4 ** n, 500, dtype=np.int64)]))
    vals = tpd.decompose_partial(H, torch.from_numpy(q).to(DEV)).cpu().numpy()
    want = np.array([expect.get(int(k), 0) for k in q], np.complex128)
    assert same_bits(vals, want)
    # sparse list of the full decomposition: exactly the generating terms
    out = tpd.decompose(H)
    qs, ws, total = tpd.compact(out)
    assert total == len(expect)
    assert np.array_equal(qs.cpu().numpy(), np.array(sorted(expect), np.int64))
    assert same_bits(ws.cpu().numpy(), np.array([expect[k] for k in sorted(expect)]))
    # capacity smaller than the list: the first entries, the full count
    q2, w2, t2 = tpd.compact(out, capacity=10)
    assert t2 == total and np.array_equal(q2.cpu().numpy(), qs.cpu().numpy()[:10])
    # matrix layout: the same pairs in (row, col) order
    M = tpd.decompose(H, layout="matrix")
    qm, wm, tm = tpd.compact(M.view(-1), layout="matrix")
    assert tm == total
    order = np.argsort(qm.cpu().numpy())
    assert np.array_equal(qm.cpu().numpy()[order], qs.cpu().numpy())
    assert same_bits(wm.cpu().numpy()[order], ws.cpu().numpy())


def selection(c, tol, matrix=False, n=None):
    c = np.asarray(c).reshape(-1)
    t = c.real.dtype.type(tol)
    keep = ~((np.abs(c.real) <= t) & (np.abs(c.imag) <= t))
    idx = np.flatnonzero(keep).astype(np.int64)
    if matrix:
        h, l = idx >> n, idx & ((1 << n) - 1)
        return (spread(h) << 1) | spread(l), c[idx]
    return idx, c[idx]


@pytest.mark.parametrize("n", [0, 5, 8, 11, 13])
@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
def test_compaction_vs_selection(n, dtype):
    rng = np.random.default_rng(2200 + n)
    m = 4 ** n
    c = (rng.standard_normal(m) + 1j * rng.standard_normal(m)) * (rng.random(m) < 0.03)
    c[rng.integers(0, m, 3)] = 1e-9
    c[rng.integers(0, m, 2)] = np.nan
    c = c.astype(np.complex128 if dtype == torch.complex128 else np.complex64)
    cd = torch.from_numpy(c).to(DEV)
    for tol in (0.0, 1e-6):
        for matrix in (False, True):
            qe, we = selection(c, tol, matrix, n)
            q, w, total = tpd.compact(cd, tol=tol, layout="matrix" if matrix else "canonical")
            assert total == qe.size
            assert np.array_equal(q.cpu().numpy(), qe)
            assert np.array_equal(w.cpu().numpy().view(np.uint8), we.view(np.uint8))


def test_n16_partial_and_count_at_full_size():
    # 2-local requests on the n = 16 dense Hermitian matrix: values against
    # the definition, then bitwise against the full decomposition; the
    # compaction count of the dense result exceeds 2^32 - 1 only if every
    # weight is nonzero, so it is checked against torch's count
    n = 16
    torch.cuda.empty_cache()
    A = W.gaussian_device(n, seed=5, hermitian=True)
    a_max = float(torch.view_as_real(A).abs().max())
    q = two_local(n)
    qd = torch.from_numpy(q).to(DEV)
    work = torch.empty(4 ** n, dtype=A.dtype, device=DEV)
    vals = tpd.decompose_partial(A, qd, work=work).cpu().numpy()
    bf = sampled_oracle(A, n, q)
    assert cerr(vals, bf) <= n * U64 * a_max
    tpd.decompose(A, work)
    assert same_bits(work[qd].cpu().numpy(), vals)
    del A
    torch.cuda.empty_cache()
    total_dev = torch.zeros(1, dtype=torch.int64, device=DEV)
    assert tpd.lib.tpd_compact(work.data_ptr(), n, tpd.TPD_C128, 0, 0.0, None, None, 0, total_dev.data_ptr(),
                               None) == 0
    nz = int(((work.real != 0) | (work.imag != 0)).sum().item())
    assert int(total_dev.item()) == nz
    del work
    torch.cuda.empty_cache()


@pytest.mark.parametrize("dtype,dbs", [(torch.complex64, (4, 5, 6)), (torch.complex128, (3, 4, 5))])
def test_n15_every_schedule_same_bits(dtype, dbs):
    # n = 15: the first sweep fuses 8 levels, so complex64 tiles of 2^6
    # diagonals hold 2^14 elements (1024 threads, no prefetch); every tile
    # width and grid gives the default schedule's bits, which match the
    # definition on sampled strings
    n = 15
    torch.cuda.empty_cache()
    A = W.gaussian_device(n, seed=15, dtype=dtype)
    ref = tpd.decompose(A)
    qs = W.sampled_strings(n, 600, seed=15)
    qd = torch.from_numpy(qs.astype(np.int64)).to(DEV)
    bf = sampled_oracle(A, n, qs)
    a_max = float(torch.view_as_real(A).abs().max())
    tol = n * U64 * a_max if dtype == torch.complex128 else (n + 1) * U32 * a_max
    assert cerr(ref[qd].cpu().numpy(), bf) <= tol
    out = torch.empty_like(ref)
    for db in dbs:
        for g in (0, 1, 4):
            for rot in (False, True):
                out.fill_(float("nan"))
                tpd.decompose_tuned(A, out, db=db, grid_per_cu=g, rotate=rot)
                assert torch.equal(torch.view_as_real(out), torch.view_as_real(ref)), (db, g, rot)
    with pytest.raises(tpd.TPDError):
        tpd.decompose_tuned(A, out, db=9)
    del A, ref, out
    torch.cuda.empty_cache()


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_n15_real_out_of_place_every_schedule(dtype):
    # real input at n = 15, canonical order out of place: 2^14-element tiles
    # (float32 ones prefetch the next tile at 1024 threads in the first
    # sweep); every tile width and grid gives the same values, which match
    # the definition on sampled strings
    n = 15
    torch.cuda.empty_cache()
    A = W.gaussian_device(n, seed=151, dtype=dtype, hermitian=False)
    ref = tpd.decompose(A)
    qs = W.sampled_strings(n, 600, seed=152)
    qd = torch.from_numpy(qs.astype(np.int64)).to(DEV)
    exp = real_coded(sampled_oracle(A, n, qs), qs)[0]
    a_max = float(A.abs().max())
    tol = n * U64 * a_max if dtype == torch.float64 else (n + 1) * U32 * a_max
    assert np.max(np.abs(ref[qd].cpu().numpy().astype(np.float64) - exp)) <= tol
    out = torch.empty_like(ref)
    for db in (4, 5, 6):
        for g in (0, 1, 4):
            out.fill_(float("nan"))
            tpd.decompose_tuned(A, out, db=db, grid_per_cu=g)
            assert torch.equal(out, ref), (db, g)
    del A, ref, out
    torch.cuda.empty_cache()


def test_partial_with_hermitian_flag_and_in_place():
    n = 12
    A = W.gaussian(n, seed=1600, hermitian=True)
    rng = np.random.default_rng(1601)
    q = np.concatenate([rng.integers(0, 4 ** n, 500, dtype=np.int64), two_local(n)])
    ref = O.tpd_partial(A, q)
    Ad = to_dev(A)
    qd = torch.from_numpy(q).to(DEV)
    got = tpd.decompose_partial(Ad, qd, hermitian=True).cpu().numpy()
    assert np.array_equal(got.real, ref.real) and np.all(got.imag == 0)
    T = Ad.clone()
    got = tpd.decompose_partial(T, qd, work=T.view(-1), layout="matrix", hermitian=True).cpu().numpy()
    assert np.array_equal(got.real, ref.real) and np.all(got.imag == 0)


def test_concurrent_streams_use_separate_workspaces():
    # pruned decompositions, partial decompositions and compactions on two
    # streams at once: each stream has its own bitmaps and scan buffers
    n = 11
    mats = [W.dense_from_terms(W.heisenberg_terms(n, seed=s, n_local=40, dyadic=True), n) for s in (21, 22)]
    refs = [O.tpd_recursive(m) for m in mats]
    req = torch.from_numpy(two_local(n)).to(DEV)
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    devs = [to_dev(m) for m in mats]
    torch.cuda.synchronize()
    outs, vals, lists = [], [], []
    for rep in range(3):
        outs.clear(); vals.clear(); lists.clear()
        for s, Ad in zip(streams, devs):
            with torch.cuda.stream(s):
                o = tpd.decompose(Ad)
                v = tpd.decompose_partial(Ad, req)
                q = torch.empty(5000, dtype=torch.int64, device=DEV)
                w = torch.empty(5000, dtype=Ad.dtype, device=DEV)
                cnt = torch.zeros(1, dtype=torch.int64, device=DEV)
                assert tpd.lib.tpd_compact(o.data_ptr(), n, tpd.TPD_C128, 0, 0.0, q.data_ptr(), w.data_ptr(), 5000,
                                           cnt.data_ptr(), ctypes_stream(s)) == 0
                outs.append(o); vals.append(v); lists.append((q, w, cnt))
        torch.cuda.synchronize()
        for o, v, (q, w, cnt), ref in zip(outs, vals, lists, refs):
            assert same_bits(o.cpu().numpy(), ref)
            assert same_bits(v.cpu().numpy(), ref[two_local(n)])
            nz = np.flatnonzero(ref)
            k = int(cnt.item())
            assert k == nz.size and np.array_equal(q[:k].cpu().numpy(), nz)
            assert same_bits(w[:k].cpu().numpy(), ref[nz])


def ctypes_stream(s):
    return s.cuda_stream
