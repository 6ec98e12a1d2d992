"""Seeded synthetic inputs for the Tensorized Pauli Decomposition.

This module only *builds* matrices; it holds none of the decomposition's
arithmetic and is shared by the tests, the benchmark and the smoke check.
Host-side generators use ``numpy.random.default_rng(seed)``; the large
device-side generators use a seeded ``torch.Generator`` on the GPU.

Workload shapes follow the paper's experiments (section "Results": random,
symmetric, Hermitian, diagonal, unit, sparse, single non-trivial factor and
transverse-field Ising inputs, entries U[0,1]) and the benchmark
configurations:

* dense complex Gaussian, n = 8 (plus an integer-entry variant in [-8, 8]);
* dense Hermitian (G + G^H)/2 with complex Gaussian G, n = 12 and n = 16;
* random-field Heisenberg chain plus 200 random 4-local strings, n = 14;
* 4096 matrices with n uniform in 2..9, every odd one Hermitian.

Pauli strings are given as letter strings ("XIZY", first letter = first
tensor factor) with a coefficient.  A dense matrix is assembled from the
textbook 2x2 matrices I, X, Y = [[0,-i],[i,0]], Z through the one nonzero
every string has per row.
"""
from __future__ import annotations

import math
from typing import Iterable, List, Sequence, Tuple

import numpy as np

Term = Tuple[str, complex]

# row-bit -> entry of the single nonzero in that row of each 2x2 letter
_LETTER_ROW = {
    "I": (1.0 + 0j, 1.0 + 0j),
    "X": (1.0 + 0j, 1.0 + 0j),
    "Y": (-1j, 1j),
    "Z": (1.0 + 0j, -1.0 + 0j),
}
_FLIPS = {"I": 0, "X": 1, "Y": 1, "Z": 0}


# ----------------------------------------------------------------------------
# dense random matrices (host)
# ----------------------------------------------------------------------------
def real_gaussian(n: int, seed: int, symmetric: bool = False) -> np.ndarray:
    """Real matrix with N(0,1) entries; optionally A = (G + G^T)/2."""
    rng = np.random.default_rng(seed)
    d = 1 << n
    G = rng.standard_normal((d, d))
    if symmetric:
        G = (G + G.T) / 2
    return np.ascontiguousarray(G)


def gaussian(n: int, seed: int, hermitian: bool = False) -> np.ndarray:
    """re, im i.i.d. N(0,1); optionally A = (G + G^H)/2."""
    rng = np.random.default_rng(seed)
    d = 1 << n
    G = rng.standard_normal((d, d)) + 1j * rng.standard_normal((d, d))
    if hermitian:
        G = (G + G.conj().T) / 2
    return np.ascontiguousarray(G)


def integer(n: int, seed: int, lo: int = -8, hi: int = 8) -> np.ndarray:
    """re, im i.i.d. uniform integers in [lo, hi]."""
    rng = np.random.default_rng(seed)
    d = 1 << n
    re = rng.integers(lo, hi + 1, size=(d, d)).astype(np.float64)
    im = rng.integers(lo, hi + 1, size=(d, d)).astype(np.float64)
    return np.ascontiguousarray(re + 1j * im)


def uniform01(n: int, seed: int) -> np.ndarray:
    """Real entries U[0,1] (the paper's 'random' input type)."""
    rng = np.random.default_rng(seed)
    d = 1 << n
    return rng.random((d, d)).astype(np.complex128)


def paper_matrix(kind: str, n: int, seed: int) -> np.ndarray:
    """The eight input types of the paper's runtime figure, entries U[0,1]."""
    rng = np.random.default_rng(seed)
    d = 1 << n
    if kind == "random":
        return rng.random((d, d)).astype(np.complex128)
    if kind == "symmetric":
        R = rng.random((d, d))
        return ((R + R.T) / 2).astype(np.complex128)
    if kind == "hermitian":
        R = rng.random((d, d)) + 1j * rng.random((d, d))
        return np.ascontiguousarray((R + R.conj().T) / 2)
    if kind == "diagonal":
        return np.diag(rng.random(d)).astype(np.complex128)
    if kind == "unit":
        return np.eye(d, dtype=np.complex128)
    if kind == "sparse":
        R = rng.random((d, d))
        R[rng.random((d, d)) >= 2.0 / d] = 0.0  # about two nonzeros per row
        return R.astype(np.complex128)
    if kind == "one_factor":
        # a single non-trivial tensor factor: I (x) ... (x) M (x) ... (x) I
        pos = int(rng.integers(0, n))
        M = rng.random((2, 2)).astype(np.complex128)
        out = np.ones((1, 1), np.complex128)
        for k in range(n):
            out = np.kron(out, M if k == pos else np.eye(2))
        return out
    if kind == "tfim":
        return dense_from_terms(tfim_terms(n, 1.0, 0.5), n)
    raise ValueError(kind)


PAPER_KINDS = ("symmetric", "unit", "diagonal", "random", "one_factor", "sparse", "tfim", "hermitian")


# ----------------------------------------------------------------------------
# Hamiltonians given as Pauli terms
# ----------------------------------------------------------------------------
def tfim_terms(n: int, J: float, g: float) -> List[Term]:
    """H = -J (sum_i Z_i Z_{i+1} + g sum_j X_j), open chain (section "Results")."""
    terms: List[Term] = []
    for i in range(n - 1):
        s = ["I"] * n
        s[i] = s[i + 1] = "Z"
        terms.append(("".join(s), -J + 0j))
    for j in range(n):
        s = ["I"] * n
        s[j] = "X"
        terms.append(("".join(s), -J * g + 0j))
    return terms


def _dyadic(v: float, bits: int = 20) -> float:
    return math.ldexp(round(math.ldexp(v, bits)), -bits)


def heisenberg_terms(n: int, seed: int, n_local: int = 200, local_weight: int = 4,
                     dyadic: bool = False) -> List[Term]:
    """Random-field Heisenberg chain sum_i J_i (XX+YY+ZZ)_{i,i+1} + h_i Z_i with
    J_i, h_i ~ U(-1,1) on an open chain, plus ``n_local`` distinct random
    strings with exactly ``local_weight`` non-identity letters (sites uniform
    without replacement, letters uniform in X/Y/Z) and N(0,1) coefficients.
    With ``dyadic`` every coefficient is rounded to a multiple of 2^-20."""
    rng = np.random.default_rng(seed)
    rnd = _dyadic if dyadic else (lambda v: v)
    terms: List[Term] = []
    J = rng.uniform(-1.0, 1.0, size=n - 1)
    h = rng.uniform(-1.0, 1.0, size=n)
    for i in range(n - 1):
        for P in "XYZ":
            s = ["I"] * n
            s[i] = s[i + 1] = P
            terms.append(("".join(s), rnd(float(J[i])) + 0j))
    for i in range(n):
        s = ["I"] * n
        s[i] = "Z"
        terms.append(("".join(s), rnd(float(h[i])) + 0j))
    seen = {t for t, _ in terms}
    added = 0
    while added < n_local:
        sites = rng.choice(n, size=local_weight, replace=False)
        letters = rng.integers(1, 4, size=local_weight)
        s = ["I"] * n
        for site, L in zip(sites, letters):
            s[int(site)] = "IXYZ"[int(L)]
        key = "".join(s)
        c = float(rng.standard_normal())
        if key in seen:
            continue  # duplicates are rejected at draw time
        seen.add(key)
        terms.append((key, rnd(c) + 0j))
        added += 1
    return terms


def string_index(s: str) -> int:
    """Canonical index q = sum_k t_k 4^(n-k) of a letter string."""
    q = 0
    for ch in s:
        q = 4 * q + "IXYZ".index(ch)
    return q


def _row_values(s: str, rows: np.ndarray) -> Tuple[int, np.ndarray]:
    n = len(s)
    x = 0
    val = np.ones(rows.shape, np.complex128)
    for k, ch in enumerate(s):
        bit = n - 1 - k
        x |= _FLIPS[ch] << bit
        b = (rows >> bit) & 1
        lo, hi = _LETTER_ROW[ch]
        val *= np.where(b == 0, lo, hi)
    return x, val


def dense_from_terms(terms: Iterable[Term], n: int) -> np.ndarray:
    """sum_t c_t sigma^t as a dense host matrix."""
    d = 1 << n
    A = np.zeros((d, d), np.complex128)
    rows = np.arange(d, dtype=np.int64)
    for s, c in terms:
        if len(s) != n:
            raise ValueError("term length != n")
        x, val = _row_values(s, rows)
        A[rows, rows ^ x] += c * val
    return A


def dense_from_terms_device(terms: Sequence[Term], n: int, dtype=None, device="cuda"):
    """sum_t c_t sigma^t as a dense torch matrix built on the device."""
    import torch

    dtype = dtype or torch.complex128
    d = 1 << n
    A = torch.zeros((d, d), dtype=dtype, device=device)
    flat = A.view(-1)
    rows_h = np.arange(d, dtype=np.int64)
    rows = torch.arange(d, dtype=torch.int64, device=device)
    for s, c in terms:
        x, val = _row_values(s, rows_h)
        cv = c * val
        if not A.is_complex():  # a real matrix: the terms must be real
            if np.any(np.imag(cv) != 0):
                raise ValueError("a term with imaginary entries in a real matrix")
            cv = np.real(cv)
        v = torch.from_numpy(np.ascontiguousarray(cv)).to(device=device, dtype=dtype)
        flat.index_add_(0, rows * d + (rows ^ x), v)
    return A


# ----------------------------------------------------------------------------
# large dense inputs generated on the device
# ----------------------------------------------------------------------------
def gaussian_device(n: int, seed: int, dtype=None, hermitian: bool = False, device="cuda",
                    block: int = 4096):
    """Complex Gaussian matrix (re, im ~ N(0,1)) generated on the GPU from a
    seeded torch generator, optionally made Hermitian in place blockwise as
    (G + G^H)/2.  A real dtype gives a real N(0,1) matrix (symmetric when
    hermitian=True).  Memory: one matrix plus one block pair of scratch."""
    import torch

    dtype = dtype or torch.complex128
    d = 1 << n
    gen = torch.Generator(device=device)
    gen.manual_seed(seed)
    A = torch.empty((d, d), dtype=dtype, device=device)
    Ar = torch.view_as_real(A) if A.is_complex() else A
    rows = max(1, min(d, (1 << 28) // max(1, d)))
    for r0 in range(0, d, rows):
        Ar[r0:r0 + rows].normal_(0.0, 1.0, generator=gen)
    if hermitian:
        b = min(block, d)
        nb = d // b
        for I in range(nb):
            sI = slice(I * b, (I + 1) * b)
            D = A[sI, sI]
            D.copy_((D + D.conj().transpose(0, 1)) / 2)
            for Jb in range(I + 1, nb):
                sJ = slice(Jb * b, (Jb + 1) * b)
                U = A[sI, sJ]
                L = A[sJ, sI]
                T = (U + L.conj().transpose(0, 1)) / 2
                U.copy_(T)
                L.copy_(T.conj().transpose(0, 1))
                del T
    return A


# ----------------------------------------------------------------------------
# batched uneven workload
# ----------------------------------------------------------------------------
def batched_qubits(count: int = 4096, seed: int = 4, lo: int = 2, hi: int = 9) -> np.ndarray:
    """Qubit counts uniform in [lo, hi]."""
    rng = np.random.default_rng(seed)
    return rng.integers(lo, hi + 1, size=count).astype(np.int32)


def batched_matrices(ns: Sequence[int], seed: int = 4) -> List[np.ndarray]:
    """Complex N(0,1) matrices, every odd-indexed one made Hermitian."""
    rng = np.random.default_rng(seed + 1)
    mats = []
    for k, n in enumerate(ns):
        d = 1 << int(n)
        G = rng.standard_normal((d, d)) + 1j * rng.standard_normal((d, d))
        if k % 2 == 1:
            G = (G + G.conj().T) / 2
        mats.append(np.ascontiguousarray(G))
    return mats


def batched_matrices_device(ns: Sequence[int], seed: int = 4, dtype=None, device="cuda"):
    """Device-side counterpart of ``batched_matrices`` (different random stream)."""
    import torch

    dtype = dtype or torch.complex128
    gen = torch.Generator(device=device)
    gen.manual_seed(seed + 1)
    mats = []
    for k, n in enumerate(ns):
        d = 1 << int(n)
        G = torch.empty((d, d), dtype=dtype, device=device)
        torch.view_as_real(G).normal_(0.0, 1.0, generator=gen)
        if k % 2 == 1:
            G = (G + G.conj().transpose(0, 1)) / 2
        mats.append(G.contiguous())
    return mats


def batched_matrices_packed(ns: Sequence[int], seed: int = 4, dtype=None, device="cuda"):
    """Host-generated counterpart of ``batched_matrices`` packed into one
    device buffer (one upload instead of thousands of small device
    launches): returns (buffer, list of per-matrix 2-D views).  Same
    distribution: complex N(0,1), every odd-indexed matrix (G + G^H)/2."""
    import torch

    dtype = dtype or torch.complex128
    npdt = np.complex128 if dtype == torch.complex128 else np.complex64
    sizes = [1 << (2 * int(n)) for n in ns]
    offs = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    host = np.empty(int(offs[-1]), npdt)
    rng = np.random.default_rng(seed + 2)
    for k, n in enumerate(ns):
        d = 1 << int(n)
        G = rng.standard_normal((d, d)) + 1j * rng.standard_normal((d, d))
        if k % 2 == 1:
            G = (G + G.conj().T) / 2
        host[offs[k]:offs[k + 1]] = G.reshape(-1)
    buf = torch.from_numpy(host).to(device)
    views = [buf[offs[k]:offs[k + 1]].view(1 << int(n), 1 << int(n)) for k, n in enumerate(ns)]
    return buf, views


# ----------------------------------------------------------------------------
# sampled strings for very large n
# ----------------------------------------------------------------------------
def sampled_strings(n: int, count: int, seed: int) -> np.ndarray:
    """``count`` canonical indices uniform in [0, 4^n) (with replacement) plus
    the forced strings I..I, X..X, Y..Y, Z..Z and 4^n - 1."""
    rng = np.random.default_rng(seed)
    top = 1 << (2 * n)
    qs = rng.integers(0, top, size=count, dtype=np.uint64)
    forced = [string_index(c * n) for c in "IXYZ"] + [top - 1]
    return np.concatenate([np.asarray(forced, np.uint64), qs])
