"""CPU checks of the partial decomposition and the sparse-list compaction.

The host replays run the request marking, tile skips, gather and the
chunked ordered compaction exactly as the HIP kernels do; they are checked
against the oracle's Algorithm 3 (partial decomposition) and against a
plain selection of the coefficients (compaction).
"""
import numpy as np
import pytest

from oracle import oracle as O
import workloads as W

tpd = pytest.importorskip("paper_2310_13421_amd.tpd")


def same_bits(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return np.array_equal(a.real, b.real) and np.array_equal(a.imag, b.imag)


def spread(v):
    r = np.zeros_like(v)
    for b in range(20):
        r |= ((v >> b) & 1) << (2 * b)
    return r


def requests(n, count, seed):
    """Uniformly random canonical indices."""
    rng = np.random.default_rng(seed)
    return rng.integers(0, 4 ** n, count, dtype=np.int64)


@pytest.mark.parametrize("n", [0, 1, 3, 8, 9, 10, 12])
def test_partial_matches_algorithm_3(n):
    A = W.gaussian(n, seed=1400 + n) if n else np.array([[1.5 - 0.25j]])
    q = requests(n, 300, 1500 + n)
    ref = O.tpd_partial(A, q)
    vals, _ = tpd.emulate_partial(A, q)
    assert same_bits(vals, ref)
    # the general path gives the same bits at the requested strings
    full = tpd.emulate(A)
    assert same_bits(vals, full[q])


def two_local(n):
    """All strings with at most two non-identity letters (the request set of
    a 2-local Hamiltonian such as the TFIM or Heisenberg chain)."""
    qs = {0}
    for i in range(n):
        for a in (1, 2, 3):
            qs.add(a << (2 * (n - 1 - i)))
            for j in range(i + 1, n):
                for b in (1, 2, 3):
                    qs.add((a << (2 * (n - 1 - i))) | (b << (2 * (n - 1 - j))))
    return np.array(sorted(qs), np.int64)


@pytest.mark.parametrize("n", [10, 11, 12])
def test_partial_clustered_requests_skip_tiles(n):
    A = W.gaussian(n, seed=1600 + n)
    q = two_local(n)
    vals, work = tpd.emulate_partial(A, q)
    assert same_bits(vals, O.tpd_partial(A, q))
    # X/Y masks of weight <= 2 touch few diagonal groups: most of the work
    # array is never written
    written = np.count_nonzero(~np.isnan(work.real))
    assert written < work.size // 2
    # matrix layout, in place
    vals2, _ = tpd.emulate_partial(A, q, flags=tpd.FLAG_LAYOUT_MATRIX, in_place=True)
    assert same_bits(vals2, vals)
    # no pruning: same values
    vals3, _ = tpd.emulate_partial(A, q, flags=tpd.FLAG_NO_PRUNE)
    assert same_bits(vals3, vals)


def test_partial_structured_with_pruning_and_edge_requests():
    n = 10
    terms = W.heisenberg_terms(n, seed=3, n_local=30, dyadic=True)
    H = W.dense_from_terms(terms, n)
    expect = np.zeros(4 ** n, np.complex128)
    for s, c in terms:
        expect[W.string_index(s)] += c
    gen = np.array(sorted({W.string_index(s) for s, _ in terms}), np.int64)
    zeros = requests(n, 100, 1800)
    q = np.concatenate([gen, zeros, gen[:5], [4 ** n, 4 ** n + 7]])  # repeats and out of range
    vals, _ = tpd.emulate_partial(H, q)
    assert same_bits(vals[:-2], expect[q[:-2]])
    assert np.all(np.isnan(vals[-2:].real)) and np.all(np.isnan(vals[-2:].imag))
    # nothing requested: nothing computed
    v0, w0 = tpd.emulate_partial(H, np.zeros(0, np.int64))
    assert v0.size == 0 and np.all(np.isnan(w0.real))


@pytest.mark.parametrize("n", [9, 12])
def test_partial_hermitian_and_complex64(n):
    A = W.gaussian(n, seed=1900 + n, hermitian=True)
    q = requests(n, 256, 2000 + n)
    ref = O.tpd_partial(A, q)
    vals, _ = tpd.emulate_partial(A, q, flags=tpd.FLAG_HERMITIAN)
    assert np.array_equal(vals.real, ref.real) and np.all(vals.imag == 0)
    v32, _ = tpd.emulate_partial(A, q, dtype=tpd.TPD_C64)
    amax = np.max(np.abs(np.concatenate([A.real.ravel(), A.imag.ravel()])))
    assert np.max(np.abs(v32 - ref)) <= (n + 1) * 2.0 ** -24 * amax * np.sqrt(2)
    assert np.array_equal(v32, tpd.emulate(A, dtype=tpd.TPD_C64)[q])


@pytest.mark.parametrize("kind", ["tfim", "heisenberg"])
def test_partial_hermitian_structured_requests_in_zero_tiles(kind):
    # requests that fall on the mirrored rows of zero tiles: the first sweep
    # never wrote those rows, so the second sweep must store their zeros
    # (every string is requested; the work array starts NaN-poisoned)
    n = 10
    terms = W.tfim_terms(n, 1.0, 0.5) if kind == "tfim" else W.heisenberg_terms(n, seed=9, n_local=30, dyadic=True)
    H = W.dense_from_terms(terms, n)
    expect = np.zeros(4 ** n, np.complex128)
    for s, c in terms:
        expect[W.string_index(s)] += c
    q = np.arange(4 ** n, dtype=np.int64)
    for flags, in_place in ((tpd.FLAG_HERMITIAN, False), (tpd.FLAG_HERMITIAN | tpd.FLAG_LAYOUT_MATRIX, True)):
        vals, _ = tpd.emulate_partial(H, q, flags=flags, in_place=in_place)
        assert same_bits(vals, expect), flags


def selection(c, tol, matrix=False, n=None):
    """Plain definition of the list: storage order, kept unless both parts
    are within tol (in the array's precision)."""
    c = np.asarray(c).reshape(-1)
    t = c.real.dtype.type(tol)
    keep = ~((np.abs(c.real) <= t) & (np.abs(c.imag) <= t))
    idx = np.flatnonzero(keep).astype(np.int64)
    if matrix:
        h, l = idx >> n, idx & ((1 << n) - 1)
        q = (spread(h) << 1) | spread(l)
    else:
        q = idx
    return q, c[idx]


@pytest.mark.parametrize("n", [0, 2, 5, 6, 8, 11])
@pytest.mark.parametrize("dtype", [tpd.TPD_C128, tpd.TPD_C64])
def test_compaction_matches_selection(n, dtype):
    rng = np.random.default_rng(2100 + n)
    m = 4 ** n
    c = (rng.standard_normal(m) + 1j * rng.standard_normal(m)) * (rng.random(m) < 0.05)
    c[rng.integers(0, m, 3)] = 1e-9 + 0j  # below tol
    c[rng.integers(0, m, 2)] = np.nan  # kept
    c = c.astype(np.complex128 if dtype == tpd.TPD_C128 else np.complex64)
    for tol in (0.0, 1e-6):
        for matrix in (False, True):
            flags = tpd.FLAG_LAYOUT_MATRIX if matrix else 0
            qe, we = selection(c, tol, matrix, n)
            q, w, total = tpd.emulate_compact(c, n, tol, dtype=dtype, flags=flags)
            assert total == qe.size
            assert np.array_equal(q.astype(np.int64), qe)
            assert np.array_equal(w.view(np.uint8), we.view(np.uint8))  # NaN payloads too
            if total > 3:
                cap = total // 2
                q2, w2, t2 = tpd.emulate_compact(c, n, tol, capacity=cap, dtype=dtype, flags=flags)
                assert t2 == total and np.array_equal(q2.astype(np.int64), qe[:cap])


def test_compaction_of_structured_decomposition_is_the_term_list():
    n = 10
    terms = W.heisenberg_terms(n, seed=5, n_local=40, dyadic=True)
    H = W.dense_from_terms(terms, n)
    coeffs = O.tpd_recursive(H)
    q, w, total = tpd.emulate_compact(coeffs, n)
    expect = {}
    for s, c in terms:
        expect[W.string_index(s)] = expect.get(W.string_index(s), 0) + c
    expect = {k: v for k, v in expect.items() if v != 0}
    assert total == len(expect)
    assert list(q.astype(np.int64)) == sorted(expect)
    assert all(w[i] == expect[int(k)] for i, k in enumerate(q))


def test_compaction_argument_errors():
    c = np.zeros(16, np.complex128)
    with pytest.raises(tpd.TPDError):
        tpd.emulate_compact(c, 2, -1.0)
    with pytest.raises(tpd.TPDError):
        tpd.emulate_compact(c, 2, float("nan"))
    with pytest.raises(tpd.TPDError):
        tpd.emulate_compact(c, 2, 0.0, flags=tpd.FLAG_NO_PRUNE)
