"""Pins for the CPU FP64 oracle (no GPU needed).

The oracle is checked against things other than itself: hand-derived worked
examples (tests/golden), Pauli strings built with numpy's Kronecker product
and traced with numpy's matmul, closed forms (transverse-field Ising,
single strings, identity, diagonal inputs), exact invariants (Hermitian =>
real weights, real symmetric => no odd-Y weights, Parseval, tensor
factorisation) and brute force on tiny inputs.  Each mistake one could make
in a slicing step (a dropped block, a sign, the factor i, the 1/2, a
transposed block, the digit order of the string index) fails at least one of
these.
"""
import itertools
import os

import numpy as np
import pytest

from oracle import oracle as O
import workloads as W

# Textbook Pauli matrices (sigma^0..3 = I, X, Y, Z).
PAULI = [
    np.array([[1, 0], [0, 1]], np.complex128),
    np.array([[0, 1], [1, 0]], np.complex128),
    np.array([[0, -1j], [1j, 0]], np.complex128),
    np.array([[1, 0], [0, -1]], np.complex128),
]


def kron_string(letters):
    out = np.ones((1, 1), np.complex128)
    for t in letters:
        out = np.kron(out, PAULI[t])
    return out


def q_of(letters):
    q = 0
    for t in letters:
        q = 4 * q + t
    return q


def numpy_weights(A):
    """omega_t = 2^-n tr(sigma^t A) with np.kron / np.matmul / np.trace."""
    n = A.shape[0].bit_length() - 1
    w = np.zeros(4 ** n, np.complex128)
    for letters in itertools.product(range(4), repeat=n):
        w[q_of(letters)] = np.trace(kron_string(letters) @ A) / 2 ** n
    return w


def same_bits(a, b):
    """Bitwise equality with -0 == +0 (signed zeros may differ)."""
    a = np.asarray(a, np.complex128)
    b = np.asarray(b, np.complex128)
    return np.array_equal(a.real, b.real) and np.array_equal(a.imag, b.imag)


# ----------------------------------------------------------------------------
# worked examples
# ----------------------------------------------------------------------------
def _parse_complex(tok):
    re, im = tok.split(",")
    return complex(float(re), float(im))


def load_one_qubit(golden_dir):
    cases = []
    with open(os.path.join(golden_dir, "one_qubit_worked_examples.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            name, a, w = [p.strip() for p in line.split("|")]
            A = np.array([_parse_complex(t) for t in a.split()], np.complex128).reshape(2, 2)
            ws = np.array([_parse_complex(t) for t in w.split()], np.complex128)
            cases.append((name, A, ws))
    return cases


def test_one_qubit_worked_examples(golden_dir):
    cases = load_one_qubit(golden_dir)
    assert len(cases) >= 6
    for name, A, expect in cases:
        for fn in (O.tpd_recursive, O.tpd_iterative, lambda M: O.weight_dense(M, range(4)),
                   lambda M: O.weight_sparse(M, range(4))):
            got = fn(A)
            assert same_bits(got, expect), (name, got, expect)
        # Parseval for the worked example: 2 * sum |w|^2 == ||A||_F^2
        assert 2 * np.sum(np.abs(expect) ** 2) == pytest.approx(np.sum(np.abs(A) ** 2), rel=1e-15)
        np.testing.assert_allclose(O.synthesize(expect, 1), A, rtol=0, atol=1e-15)


def test_tfim_n3_golden(golden_dir):
    expect = {}
    live_expect = None
    with open(os.path.join(golden_dir, "tfim_n3.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            parts = line.split()
            if parts[0] == "live":
                live_expect = [int(v) for v in parts[1:]]
                continue
            s, q, re, im = parts
            assert O.index_of(s) == int(q)
            expect[int(q)] = complex(float(re), float(im))
    # build H from numpy Kronecker products, independently of the generators
    n = 3
    Z, X, I2 = PAULI[3], PAULI[1], PAULI[0]

    def site(op, k):
        mats = [op if j == k else I2 for j in range(n)]
        out = mats[0]
        for m in mats[1:]:
            out = np.kron(out, m)
        return out

    H = np.zeros((8, 8), np.complex128)
    for i in range(n - 1):
        H -= site(Z, i) @ site(Z, i + 1)
    for j in range(n):
        H -= 0.5 * site(X, j)
    w, live, _ = O.tpd_recursive(H, with_stats=True)
    for q in range(64):
        assert w[q] == expect.get(q, 0.0), q
    assert list(live) == live_expect
    w2, live2 = O.tpd_iterative(H, with_stats=True)
    assert same_bits(w, w2) and list(live2) == live_expect


# ----------------------------------------------------------------------------
# index convention and the definition against numpy Kronecker products
# ----------------------------------------------------------------------------
def test_index_convention_order_pins():
    assert O.index_of("XZ") == 7
    assert O.index_of("ZX") == 13
    assert O.index_of("YX") == 9  # the single path Omega_2* -> Omega_21 of Fig. 2
    assert O.index_of("II") == 0
    for n in (1, 2, 3):
        for letters in itertools.product(range(4), repeat=n):
            S = kron_string(letters)
            e = np.zeros(4 ** n, np.complex128)
            e[q_of(letters)] = 1
            for fn in (O.tpd_recursive, O.tpd_iterative):
                assert same_bits(fn(S), e), letters


def test_single_string_live_counts_n4():
    # a single Pauli string keeps exactly one live CMW per level (section "Results")
    rng = np.random.default_rng(0)
    for _ in range(20):
        letters = tuple(int(v) for v in rng.integers(0, 4, size=4))
        _, live, _ = O.tpd_recursive(kron_string(letters), with_stats=True)
        assert list(live) == [1, 1, 1, 1, 1]


@pytest.mark.parametrize("n", [1, 2, 3])
def test_definition_matches_numpy_kron(n):
    A = W.gaussian(n, seed=10 + n)
    ref = numpy_weights(A)
    qs = np.arange(4 ** n)
    for got in (O.weight_dense(A, qs), O.weight_sparse(A, qs), O.tpd_recursive(A), O.tpd_iterative(A),
                O.tpd_partial(A, qs)):
        np.testing.assert_allclose(got, ref, rtol=0, atol=1e-14)


def test_dense_and_sparse_definitions_agree_n4():
    A = W.gaussian(4, seed=3)
    qs = np.arange(256)
    np.testing.assert_allclose(O.weight_dense(A, qs), O.weight_sparse(A, qs), rtol=0, atol=1e-15)


def test_xy_mask_and_diagonal_form():
    n = 5
    A = W.gaussian(n, seed=5)
    rng = np.random.default_rng(1)
    qs = rng.integers(0, 4 ** n, size=64)
    ref = O.weight_sparse(A, qs)
    for q, r in zip(qs, ref):
        x = O.xy_mask(int(q), n)
        letters = O.string_of(int(q), n)
        assert x == int("".join("1" if c in "XY" else "0" for c in letters), 2)
        i = np.arange(1 << n)
        v = A[i ^ x, i]
        assert same_bits(O.weight_from_diagonal(v, n, x, [q]), [r])


# ----------------------------------------------------------------------------
# recursion / iteration / partial against brute force
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("n", [2, 4, 6])
def test_integer_inputs_bit_exact(n):
    A = W.integer(n, seed=100 + n)
    qs = np.arange(4 ** n)
    ref = O.weight_sparse(A, qs)
    rec = O.tpd_recursive(A)
    assert same_bits(rec, ref)
    assert same_bits(O.tpd_iterative(A), rec)


@pytest.mark.parametrize("n", [5, 7])
def test_gaussian_recursion_vs_brute_force(n):
    A = W.gaussian(n, seed=200 + n)
    qs = np.arange(4 ** n)
    ref = O.weight_sparse(A, qs)
    rec = O.tpd_recursive(A)
    amax = np.max(np.abs(np.concatenate([A.real.ravel(), A.imag.ravel()])))
    err = np.max(np.abs(np.concatenate([(rec - ref).real, (rec - ref).imag])))
    # each weight is a +-sum of 2^n entries formed by a depth-n tree of single
    # roundings, scaled exactly: |err| <= n u max|a| (u = 2^-53)
    assert err <= n * 2.0 ** -53 * amax * 1.01
    assert same_bits(O.tpd_iterative(A), rec)


@pytest.mark.parametrize("threads", [1, 2, 3, 8])
def test_multithreaded_algorithm_2_is_the_serial_one(threads):
    # the OpenMP form of Algorithm 2 (CPU baseline) performs the same per-entry
    # operations: bitwise the serial weights and the same live-CMW counts, on
    # dense, integer, structured (pruned), zero and NaN inputs
    cases = [W.gaussian(n, seed=600 + n) for n in (1, 2, 4, 7, 9)]
    cases.append(W.integer(8, seed=610))
    cases.append(W.dense_from_terms(W.tfim_terms(9, 1.0, 0.5), 9))
    cases.append(W.dense_from_terms(W.heisenberg_terms(10, seed=611, n_local=25, dyadic=True), 10))
    cases.append(np.zeros((32, 32), np.complex128))
    nan = np.zeros((64, 64), np.complex128)
    nan[3, 40] = np.nan
    cases.append(nan)
    cases.append(np.array([[0.5 - 2j]]))
    for A in cases:
        w, live = O.tpd_iterative(A, with_stats=True)
        wm, livem = O.tpd_iterative_mt(A, threads, with_stats=True)
        # identical bit patterns (NaN payloads and signed zeros included)
        assert np.array_equal(wm.view(np.uint64), w.view(np.uint64)) and np.array_equal(livem, live)


def test_sampled_weights_grouped_by_mask_on_threads():
    # the sampled-string evaluation used at full size (grouping by X/Y mask,
    # host threads, entries fetched per mask) returns exactly the plain
    # definition's values; the vectorised masks are the C function's
    n = 8
    A = W.gaussian(n, seed=650)
    rng = np.random.default_rng(651)
    qs = np.concatenate([rng.integers(0, 4 ** n, 6000), [0, 4 ** n - 1, 0x5555, 0xAAAA, 0xFFFF]])
    i = np.arange(1 << n)
    got = O.sampled_weights(lambda xs: np.stack([A[i ^ x, i] for x in xs]), n, qs, threads=3, masks_per_fetch=17)
    assert same_bits(got, O.weight_sparse(A, qs))
    assert np.array_equal(O._xy_masks(qs.astype(np.uint64), n), [O.xy_mask(int(q), n) for q in qs])


def test_partial_tpd_matches_full():
    n = 6
    A = W.gaussian(n, seed=7)
    full = O.tpd_recursive(A)
    rng = np.random.default_rng(2)
    req = rng.integers(0, 4 ** n, size=300)
    req = np.concatenate([req, req[:10], [0, 4 ** n - 1]])  # repeats allowed
    got = O.tpd_partial(A, req)
    assert same_bits(got, full[req])
    # requesting a string below a zero CMW yields exactly 0
    D = np.diag(np.arange(1, 2 ** n + 1)).astype(np.complex128)
    q_x = O.index_of("X" + "I" * (n - 1))
    assert O.tpd_partial(D, [q_x])[0] == 0


# ----------------------------------------------------------------------------
# closed forms
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("n", [3, 4, 5, 6, 7])
def test_tfim_closed_form(n):
    J, g = 1.0, 0.5
    H = W.dense_from_terms(W.tfim_terms(n, J, g), n)
    w, live, _ = O.tpd_recursive(H, with_stats=True)
    expect = {W.string_index(s): c for s, c in W.tfim_terms(n, J, g)}
    nz = np.flatnonzero(w)
    assert set(nz.tolist()) == set(expect)
    assert len(nz) == 2 * n - 1
    for q, c in expect.items():
        assert w[q] == c
    # live CMWs per level: 1, then 2k+1 for k < n, then 2n-1
    assert list(live) == [1] + [2 * k + 1 for k in range(1, n)] + [2 * n - 1]


def test_identity_unit_and_diagonal():
    n = 5
    w = O.tpd_recursive(np.eye(2 ** n, dtype=np.complex128))
    e0 = np.zeros(4 ** n, np.complex128)
    e0[0] = 1
    assert same_bits(w, e0)
    D = W.paper_matrix("diagonal", n, seed=3)
    w, live, _ = O.tpd_recursive(D, with_stats=True)
    support = np.flatnonzero(w)
    for q in support:
        assert set(O.string_of(int(q), n)) <= {"I", "Z"}
    # a diagonal input keeps only I/Z children: at most 2^k live CMWs at level k
    assert all(live[k] <= 2 ** k for k in range(n + 1))


def test_dyadic_hamiltonian_round_trip_and_live_prefixes():
    n = 8
    terms = W.heisenberg_terms(n, seed=3, n_local=40, dyadic=True)
    H = W.dense_from_terms(terms, n)
    w, live, _ = O.tpd_recursive(H, with_stats=True)
    expect = np.zeros(4 ** n, np.complex128)
    for s, c in terms:
        expect[W.string_index(s)] += c
    assert same_bits(w, expect)  # exact recovery, exact zeros elsewhere
    gen = [W.string_index(s) for s, _ in terms]
    for k in range(1, n + 1):
        prefixes = {q >> (2 * (n - k)) for q in gen}
        assert live[k] == len(prefixes), k


# ----------------------------------------------------------------------------
# invariants
# ----------------------------------------------------------------------------
def test_parseval_and_reconstruction():
    for n in (3, 6):
        A = W.gaussian(n, seed=50 + n)
        w = O.tpd_recursive(A)
        lhs = 2 ** n * np.sum(np.abs(w) ** 2)
        rhs = np.sum(np.abs(A) ** 2)
        assert abs(lhs - rhs) <= 1e-12 * rhs
        np.testing.assert_allclose(O.synthesize(w, n), A, rtol=0, atol=1e-13)


def test_hermitian_weights_exactly_real():
    for n in (4, 7):
        A = W.gaussian(n, seed=60 + n, hermitian=True)
        w = O.tpd_recursive(A)
        assert np.all(w.imag == 0.0)


def test_real_symmetric_and_real_inputs():
    n = 6
    S = W.paper_matrix("symmetric", n, seed=1)
    w = O.tpd_recursive(S)
    for q in range(4 ** n):
        ny = O.string_of(q, n).count("Y")
        if ny % 2 == 1:
            assert w[q] == 0
    R = W.paper_matrix("random", n, seed=2)
    w = O.tpd_recursive(R)
    for q in range(4 ** n):
        ny = O.string_of(q, n).count("Y")
        if ny % 2 == 0:
            assert w[q].imag == 0
        else:
            assert w[q].real == 0


def test_linearity():
    n = 5
    A, B = W.gaussian(n, 1), W.gaussian(n, 2)
    a, b = 0.75 - 0.5j, -1.25 + 2j
    np.testing.assert_allclose(O.tpd_recursive(a * A + b * B),
                               a * O.tpd_recursive(A) + b * O.tpd_recursive(B), rtol=0, atol=1e-13)


def test_tensor_factorisation():
    # TPD(A (x) B)[q_A 4^{n_B} + q_B] = TPD(A)[q_A] * TPD(B)[q_B]
    A, B = W.gaussian(2, 11), W.gaussian(3, 12)
    wa, wb = O.tpd_recursive(A), O.tpd_recursive(B)
    w = O.tpd_recursive(np.kron(A, B))
    np.testing.assert_allclose(w, np.kron(wa, wb), rtol=0, atol=1e-14)


@pytest.mark.parametrize("kind", W.PAPER_KINDS)
def test_paper_matrix_types(kind):
    n = 5
    A = W.paper_matrix(kind, n, seed=9)
    w = O.tpd_recursive(A)
    np.testing.assert_allclose(O.synthesize(w, n), A, rtol=0, atol=1e-13)
    ref = O.weight_sparse(A, np.arange(4 ** n))
    np.testing.assert_allclose(w, ref, rtol=0, atol=1e-14)


def test_zero_and_nan_semantics():
    n = 3
    Z = np.zeros((8, 8), np.complex128)
    w, live, ops = O.tpd_recursive(Z, with_stats=True)
    assert not np.any(w) and list(live) == [0] * (n + 1) and ops == 0
    A = np.zeros((8, 8), np.complex128)
    A[3, 5] = np.nan
    w = O.tpd_recursive(A)
    # NaN counts as nonzero, so it propagates to every string whose X/Y mask is 3^5
    x = 3 ^ 5
    for q in range(64):
        if O.xy_mask(q, n) == x:
            assert np.isnan(w[q])
        else:
            assert w[q] == 0


def test_generator_matches_numpy_kron():
    # the dense-from-terms generator against explicit Kronecker products
    n = 4
    terms = W.heisenberg_terms(n, seed=8, n_local=10)
    H = W.dense_from_terms(terms, n)
    ref = np.zeros_like(H)
    for s, c in terms:
        ref += c * kron_string(["IXYZ".index(ch) for ch in s])
    np.testing.assert_allclose(H, ref, rtol=0, atol=1e-15)


def test_purely_imaginary_cmw_is_live():
    # A = i (Z (x) X): the level-1 CMW of Z is i X, which has no real part;
    # it must count as nonzero and yield w[ZX] = i exactly.
    A = 1j * kron_string([3, 1])
    w, live, _ = O.tpd_recursive(A, with_stats=True)
    e = np.zeros(16, np.complex128)
    e[O.index_of("ZX")] = 1j
    assert same_bits(w, e)
    assert list(live) == [1, 1, 1]
    assert same_bits(O.tpd_iterative(A), e)
