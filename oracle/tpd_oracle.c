/*
 * tpd_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, single-threaded CPU reference in IEEE binary64 for the
 * Tensorized Pauli Decomposition (Hantzko, Binkowski, Gupta,
 * arXiv:2310.13421).  Only the test-suite, the package smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  It shares no
 * code, header, table or helper with the HIP library: the GPU path must
 * never call it, and it never calls the GPU path.
 *
 * Conventions (paper, section "Problem formulation", eq. (PauliString)):
 *   - Pauli letters sigma^0..3 = I, X, Y, Z, with
 *       I = [[1,0],[0,1]]  X = [[0,1],[1,0]]  Y = [[0,-i],[i,0]]  Z = [[1,0],[0,-1]].
 *     (The paper never prints Y; this sign is the only one compatible with
 *     its CMW formula Omega_2 = (i/2)(A12 - A21), eq. (CumulativeWeightsDefinition).)
 *   - A string t = t_1 t_2 ... t_n denotes sigma^{t_1} (x) ... (x) sigma^{t_n};
 *     t_1 is the first (outermost) tensor factor, i.e. it acts on the most
 *     significant bit of the row and column index.
 *   - Its canonical integer index is q(t) = sum_k t_k 4^{n-k}.
 *   - Complex numbers are interleaved (re, im) binary64 pairs; a matrix is
 *     row-major 2^n x 2^n; a coefficient vector has 4^n entries indexed by q.
 *
 * Parity status of each function is stated in its comment; all of them are
 * pinned by the CPU test-suite (hand-derived worked examples, explicit
 * Kronecker products built with a library routine, closed forms such as the
 * transverse-field Ising Hamiltonian, and invariants).
 *
 * Build: gcc -O2 -std=c99 -ffp-contract=off -fno-fast-math -fopenmp -shared
 * -fPIC (no FMA contraction, no flush-to-zero).  OpenMP is used by one
 * function only, the multithreaded form of Algorithm 2 (7), for timing the
 * CPU baseline; every other function runs on one thread.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_OK 0
#define ORACLE_EINVAL -1
#define ORACLE_ENOMEM -2

int oracle_abi_version(void) { return 1; }

/* ------------------------------------------------------------------------ */
/* Pauli letters as exact phase tables.                                      */
/* Every entry of I, X, Y, Z is 0 or a power of i.  pow4[t][a][b] gives the  */
/* exponent e in i^e for a nonzero entry (row a, column b), -1 for a zero.   */
/* Section "Problem formulation".                                            */
/* ------------------------------------------------------------------------ */
static const int pauli_pow4[4][2][2] = {
    /* I */ {{0, -1}, {-1, 0}},
    /* X */ {{-1, 0}, {0, -1}},
    /* Y */ {{-1, 3}, {1, -1}}, /* [0][1] = -i = i^3, [1][0] = +i = i^1 */
    /* Z */ {{0, -1}, {-1, 2}}, /* [1][1] = -1 = i^2 */
};

/* multiply (re, im) by i^e exactly (a permutation and negation) */
static void mul_ipow(int e, double re, double im, double* ore, double* oim) {
  switch (e & 3) {
    case 0: *ore = re; *oim = im; break;
    case 1: *ore = -im; *oim = re; break;
    case 2: *ore = -re; *oim = -im; break;
    default: *ore = im; *oim = -re; break;
  }
}

/* Neumaier-compensated running sum: far more accurate than any fixed
 * summation order used by the decomposition itself. */
typedef struct { double s, c; } nsum_t;
static void nsum_add(nsum_t* a, double x) {
  double t = a->s + x;
  if (fabs(a->s) >= fabs(x)) a->c += (a->s - t) + x;
  else a->c += (x - t) + a->s;
  a->s = t;
}
static double nsum_value(const nsum_t* a) { return a->s + a->c; }

static int digit(uint64_t q, int n, int k /* 1-based factor position */) {
  return (int)((q >> (2 * (n - k))) & 3u);
}
static int rowbit(uint64_t i, int n, int k) { return (int)((i >> (n - k)) & 1u); }

/* ------------------------------------------------------------------------ */
/* (1) The plain definition, written out.                                   */
/*   omega_t = 2^-n tr(sigma^t A) = 2^-n sum_i sum_j sigma^t[i][j] A[j][i]  */
/* with sigma^t[i][j] = prod_k sigma^{t_k}[i_k][j_k] (Kronecker product).   */
/* Eq. (PauliDecomposition) and eq. (PauliString).  Cost 4^n per string,     */
/* so this is meant for n <= 5.                                             */
/* ------------------------------------------------------------------------ */
int oracle_weight_dense(const double* A, int n, const uint64_t* qs, size_t m, double* out) {
  if (n < 0 || n > 12 || (!A && m) || (!qs && m) || (!out && m)) return ORACLE_EINVAL;
  const uint64_t dim = (uint64_t)1 << n;
  for (size_t s = 0; s < m; ++s) {
    const uint64_t q = qs[s];
    if (n < 32 && (q >> (2 * n)) != 0) return ORACLE_EINVAL;
    nsum_t re = {0, 0}, im = {0, 0};
    for (uint64_t i = 0; i < dim; ++i) {
      for (uint64_t j = 0; j < dim; ++j) {
        int e = 0, zero = 0;
        for (int k = 1; k <= n && !zero; ++k) {
          int p = pauli_pow4[digit(q, n, k)][rowbit(i, n, k)][rowbit(j, n, k)];
          if (p < 0) zero = 1; else e += p;
        }
        if (zero) continue;
        const double* a = A + 2 * (j * dim + i); /* A[j][i] */
        double pr, pi;
        mul_ipow(e, a[0], a[1], &pr, &pi);
        nsum_add(&re, pr);
        nsum_add(&im, pi);
      }
    }
    out[2 * s] = ldexp(nsum_value(&re), -n);
    out[2 * s + 1] = ldexp(nsum_value(&im), -n);
  }
  return ORACLE_OK;
}

/* X/Y mask of a string: bit (n-k) set iff t_k is X or Y, i.e. the column
 * offset of the single nonzero in each row of sigma^t. */
uint64_t oracle_xy_mask(uint64_t q, int n) {
  uint64_t x = 0;
  for (int k = 1; k <= n; ++k) {
    int t = digit(q, n, k);
    if (t == 1 || t == 2) x |= (uint64_t)1 << (n - k);
  }
  return x;
}

/* Row phases of sigma^t: sigma^t[i][i ^ x] = i^{e[i]}, built as the
 * Kronecker product of the per-letter 2-vectors (sigma^{t_k}[b][b ^ x_k])_b. */
static void row_phases(uint64_t q, int n, unsigned char* e) {
  e[0] = 0;
  uint64_t len = 1;
  for (int k = 1; k <= n; ++k) {
    const int t = digit(q, n, k);
    const int xk = (t == 1 || t == 2);
    const int p0 = pauli_pow4[t][0][0 ^ xk];
    const int p1 = pauli_pow4[t][1][1 ^ xk];
    /* new index = old index * 2 + b  (b is the k-th most significant bit) */
    for (uint64_t r = len; r-- > 0;) {
      const unsigned char old = e[r];
      e[2 * r] = (unsigned char)((old + p0) & 3);
      e[2 * r + 1] = (unsigned char)((old + p1) & 3);
    }
    len *= 2;
  }
}

/* ------------------------------------------------------------------------ */
/* (2) The same definition summed over the nonzero entries only.            */
/*   omega_t = 2^-n sum_i sigma^t[i][i ^ x(t)] A[i ^ x(t)][i]               */
/* Every Pauli string has exactly one nonzero per row (a fact the paper      */
/* recalls in "Existing algorithms"; it follows from the Kronecker form).    */
/* Cost 2^n per string.                                                      */
/* ------------------------------------------------------------------------ */
int oracle_weight_sparse(const double* A, int n, const uint64_t* qs, size_t m, double* out) {
  if (n < 0 || n > 20 || (!A && m) || (!qs && m) || (!out && m)) return ORACLE_EINVAL;
  const uint64_t dim = (uint64_t)1 << n;
  unsigned char* e = (unsigned char*)malloc(dim);
  if (!e) return ORACLE_ENOMEM;
  for (size_t s = 0; s < m; ++s) {
    const uint64_t q = qs[s];
    if ((q >> (2 * n)) != 0) { free(e); return ORACLE_EINVAL; }
    const uint64_t x = oracle_xy_mask(q, n);
    row_phases(q, n, e);
    nsum_t re = {0, 0}, im = {0, 0};
    for (uint64_t i = 0; i < dim; ++i) {
      const double* a = A + 2 * ((i ^ x) * dim + i); /* A[i^x][i] */
      double pr, pi;
      mul_ipow(e[i], a[0], a[1], &pr, &pi);
      nsum_add(&re, pr);
      nsum_add(&im, pi);
    }
    out[2 * s] = ldexp(nsum_value(&re), -n);
    out[2 * s + 1] = ldexp(nsum_value(&im), -n);
  }
  free(e);
  return ORACLE_OK;
}

/* (2b) As (2), for strings that all share the X/Y mask x, given only the
 * entries the sum reads: v[i] = A[i ^ x][i] for i in [0, 2^n).  This lets a
 * caller evaluate sampled strings of a matrix too large to copy whole. */
int oracle_weight_from_diagonal(const double* v, int n, uint64_t x, const uint64_t* qs, size_t m,
                                double* out) {
  if (n < 0 || n > 24 || (!v && m) || (!qs && m) || (!out && m)) return ORACLE_EINVAL;
  const uint64_t dim = (uint64_t)1 << n;
  unsigned char* e = (unsigned char*)malloc(dim);
  if (!e) return ORACLE_ENOMEM;
  for (size_t s = 0; s < m; ++s) {
    const uint64_t q = qs[s];
    if ((q >> (2 * n)) != 0 || oracle_xy_mask(q, n) != x) { free(e); return ORACLE_EINVAL; }
    row_phases(q, n, e);
    nsum_t re = {0, 0}, im = {0, 0};
    for (uint64_t i = 0; i < dim; ++i) {
      double pr, pi;
      mul_ipow(e[i], v[2 * i], v[2 * i + 1], &pr, &pi);
      nsum_add(&re, pr);
      nsum_add(&im, pi);
    }
    out[2 * s] = ldexp(nsum_value(&re), -n);
    out[2 * s + 1] = ldexp(nsum_value(&im), -n);
  }
  free(e);
  return ORACLE_OK;
}

/* ------------------------------------------------------------------------ */
/* One slicing step: the four cumulative matrix weights (CMWs) of a          */
/* 2^m x 2^m block M (section "Methods", eq. (CumulativeWeightsDefinition)):  */
/*   Omega_0 = (M11 + M22)/2      Omega_1 = (M12 + M21)/2                     */
/*   Omega_2 = (i/2)(M12 - M21)   Omega_3 = (M11 - M22)/2                     */
/* Returns 1 iff the produced block has a nonzero entry (exact comparison,    */
/* a NaN counts as nonzero).                                                  */
/* ------------------------------------------------------------------------ */
/* rows [r0, r1) of the CMW only (used directly by the multithreaded form
 * of Algorithm 2, which splits one CMW over threads) */
static int cmw_rows(const double* M, int m, int t, double* C, uint64_t r0, uint64_t r1) {
  const uint64_t dim = (uint64_t)1 << m, h = dim >> 1;
  int nonzero = 0;
  for (uint64_t r = r0; r < r1; ++r) {
    for (uint64_t c = 0; c < h; ++c) {
      const double* a11 = M + 2 * (r * dim + c);
      const double* a12 = M + 2 * (r * dim + c + h);
      const double* a21 = M + 2 * ((r + h) * dim + c);
      const double* a22 = M + 2 * ((r + h) * dim + c + h);
      double re, im;
      switch (t) {
        case 0: re = (a11[0] + a22[0]) * 0.5; im = (a11[1] + a22[1]) * 0.5; break;
        case 1: re = (a12[0] + a21[0]) * 0.5; im = (a12[1] + a21[1]) * 0.5; break;
        case 2: {
          /* i * (M12 - M21) / 2 : (dr, di) -> (-di, dr), then halve */
          const double dr = a12[0] - a21[0], di = a12[1] - a21[1];
          re = -di * 0.5;
          im = dr * 0.5;
          break;
        }
        default: re = (a11[0] - a22[0]) * 0.5; im = (a11[1] - a22[1]) * 0.5; break;
      }
      C[2 * (r * h + c)] = re;
      C[2 * (r * h + c) + 1] = im;
      if (re != 0.0 || im != 0.0 || re != re || im != im) nonzero = 1;
    }
  }
  return nonzero;
}

static int cmw(const double* M, int m, int t, double* C) {
  return cmw_rows(M, m, t, C, 0, ((uint64_t)1 << m) >> 1);
}

static int block_nonzero(const double* M, uint64_t count) {
  for (uint64_t k = 0; k < 2 * count; ++k)
    if (M[k] != 0.0 || M[k] != M[k]) return 1;
  return 0;
}

/* ------------------------------------------------------------------------ */
/* (3) Recursive TPD, Fig. 1 / Algorithm 1.                                  */
/* Depth-first: compute each child CMW of the current block in the order     */
/* t = 0,1,2,3, recurse into it only when it is nonzero, and record the 1x1  */
/* blocks as weights.  The string grows by one letter per level; the letter  */
/* chosen at depth k is t_k (the k-th tensor factor), so the weight lands at */
/* q = sum_k t_k 4^{n-k}.  Strings never reached stay exactly zero in `out`. */
/* live[k] (k = 1..n) counts the nonzero CMWs produced at depth k; live[0]   */
/* is 1 iff A itself is nonzero.  ops counts complex CMW entries computed.   */
/* ------------------------------------------------------------------------ */
typedef struct {
  int n;
  double* out;
  uint64_t* live;
  uint64_t ops;
  int failed;
} rec_ctx;

static void tpd_rec(rec_ctx* ctx, const double* M, int m, uint64_t prefix) {
  if (m == 0) {
    ctx->out[2 * prefix] = M[0];
    ctx->out[2 * prefix + 1] = M[1];
    return;
  }
  const uint64_t h = (uint64_t)1 << (m - 1);
  double* C = (double*)malloc(sizeof(double) * 2 * h * h);
  if (!C) { ctx->failed = 1; return; }
  const int depth = ctx->n - m + 1;
  for (int t = 0; t < 4 && !ctx->failed; ++t) {
    const int nz = cmw(M, m, t, C);
    ctx->ops += h * h;
    if (nz) {
      if (ctx->live) ctx->live[depth] += 1;
      tpd_rec(ctx, C, m - 1, prefix * 4 + (uint64_t)t);
    }
  }
  free(C);
}

int oracle_tpd_recursive(const double* A, int n, double* out, uint64_t* live, uint64_t* ops) {
  if (n < 0 || n > 16 || !A || !out) return ORACLE_EINVAL;
  const uint64_t count = (uint64_t)1 << (2 * n);
  memset(out, 0, sizeof(double) * 2 * count);
  if (live) memset(live, 0, sizeof(uint64_t) * (size_t)(n + 1));
  rec_ctx ctx = {n, out, live, 0, 0};
  const int nz = block_nonzero(A, count);
  if (live) live[0] = (uint64_t)nz;
  if (nz) tpd_rec(&ctx, A, n, 0);
  if (ops) *ops = ctx.ops;
  return ctx.failed ? ORACLE_ENOMEM : ORACLE_OK;
}

/* ------------------------------------------------------------------------ */
/* (4) Iterative TPD, Fig. 1 / Algorithm 2.                                  */
/* Level-synchronous: the frontier S^i holds the nonzero CMWs of all strings */
/* whose first i-1 letters are fixed.  Iteration i replaces every frontier   */
/* block by its four children, keeping the nonzero ones, and the parent      */
/* storage is released once the next level exists (section "Results", space  */
/* complexity).  The loop runs i = 1..n so that every letter gets expanded   */
/* (the printed bound n-1 would leave the last letter unexpanded).           */
/* Same per-entry operations as (3), hence bitwise the same weights.        */
/* ------------------------------------------------------------------------ */
int oracle_tpd_iterative(const double* A, int n, double* out, uint64_t* live) {
  if (n < 0 || n > 16 || !A || !out) return ORACLE_EINVAL;
  const uint64_t count = (uint64_t)1 << (2 * n);
  memset(out, 0, sizeof(double) * 2 * count);
  if (live) memset(live, 0, sizeof(uint64_t) * (size_t)(n + 1));
  if (!block_nonzero(A, count)) return ORACLE_OK;
  if (live) live[0] = 1;

  /* frontier: `nf` blocks of dimension 2^m, stored back to back */
  uint64_t nf = 1;
  uint64_t* pre = (uint64_t*)malloc(sizeof(uint64_t));
  double* blocks = (double*)malloc(sizeof(double) * 2 * count);
  if (!pre || !blocks) { free(pre); free(blocks); return ORACLE_ENOMEM; }
  pre[0] = 0;
  memcpy(blocks, A, sizeof(double) * 2 * count);

  for (int i = 1; i <= n; ++i) {
    const int m = n - i + 1; /* parent blocks are 2^m x 2^m */
    const uint64_t psize = (uint64_t)1 << (2 * m), csize = psize >> 2;
    uint64_t* npre = (uint64_t*)malloc(sizeof(uint64_t) * 4 * nf);
    double* nblocks = (double*)malloc(sizeof(double) * 2 * csize * 4 * nf);
    if (!npre || !nblocks) {
      free(npre); free(nblocks); free(pre); free(blocks);
      return ORACLE_ENOMEM;
    }
    uint64_t nn = 0;
    for (uint64_t f = 0; f < nf; ++f) {
      for (int t = 0; t < 4; ++t) {
        double* C = nblocks + 2 * csize * nn;
        if (cmw(blocks + 2 * psize * f, m, t, C)) {
          npre[nn] = pre[f] * 4 + (uint64_t)t;
          ++nn;
        }
      }
    }
    if (live) live[i] = nn;
    free(pre);
    free(blocks);
    pre = npre;
    blocks = nblocks;
    nf = nn;
    if (nf == 0) break;
  }
  if (nf && n >= 0) {
    /* after n expansions every frontier block is 1x1 */
    for (uint64_t f = 0; f < nf; ++f) {
      out[2 * pre[f]] = blocks[2 * f];
      out[2 * pre[f] + 1] = blocks[2 * f + 1];
    }
  }
  free(pre);
  free(blocks);
  return ORACLE_OK;
}

/* ------------------------------------------------------------------------ */
/* (7) Algorithm 2 on several threads (OpenMP), for the CPU baseline only.   */
/* The same level loop and the same CMW arithmetic as (4); within a level    */
/* the children of all frontier blocks (4 per block, each split into row     */
/* ranges so that the first levels also spread over the threads) are         */
/* computed independently into their own slots, then the nonzero ones are    */
/* kept in (block, letter) order.  Each entry sees the same operations as    */
/* in (4), so the weights are bitwise those of (4) for any thread count.     */
/* Two buffers of 4^n entries, allocated once and first touched by the       */
/* threads, take turns holding the parents and the children (a level's      */
/* children never need more room than its parents).                          */
/* threads <= 0: the OpenMP default.                                         */
/* ------------------------------------------------------------------------ */
int oracle_tpd_iterative_mt(const double* A, int n, double* out, uint64_t* live, int threads) {
  if (n < 0 || n > 16 || !A || !out) return ORACLE_EINVAL;
  const int nth = threads > 0 ? threads : omp_get_max_threads();
  const int64_t count = (int64_t)1 << (2 * n);
#pragma omp parallel for schedule(static) num_threads(nth)
  for (int64_t k = 0; k < 2 * count; ++k) out[k] = 0.0;
  if (live) memset(live, 0, sizeof(uint64_t) * (size_t)(n + 1));
  if (!block_nonzero(A, (uint64_t)count)) return ORACLE_OK;
  if (live) live[0] = 1;

  uint64_t nf = 1;
  uint64_t* pre = (uint64_t*)malloc(sizeof(uint64_t));
  double* blocks = (double*)malloc(sizeof(double) * 2 * (size_t)count);
  double* all = (double*)malloc(sizeof(double) * 2 * (size_t)count);
  if (!pre || !blocks || !all) { free(pre); free(blocks); free(all); return ORACLE_ENOMEM; }
  pre[0] = 0;
#pragma omp parallel for schedule(static) num_threads(nth)
  for (int64_t k = 0; k < 2 * count; ++k) {
    blocks[k] = A[k];
    all[k] = 0.0;
  }

  for (int i = 1; i <= n; ++i) {
    const int m = n - i + 1;
    const uint64_t psize = (uint64_t)1 << (2 * m), csize = psize >> 2, h = (uint64_t)1 << (m - 1);
    const uint64_t kids = 4 * nf;
    /* jobs: runs of whole children when there are many, else row ranges of
     * one child, so that every thread has work at every level */
    const uint64_t want = 32 * (uint64_t)nth;
    uint64_t split = 1, per = 1;
    while (kids * split < want && split < h) split *= 2;
    while (kids / (per * 2) >= want && kids % (per * 2) == 0) per *= 2;
    const int64_t jobs = (int64_t)(kids / per * split);
    unsigned char* nz = (unsigned char*)calloc(kids, 1);
    uint64_t* npre = (uint64_t*)malloc(sizeof(uint64_t) * kids);
    if (!nz || !npre) {
      free(nz); free(npre); free(pre); free(blocks); free(all);
      return ORACLE_ENOMEM;
    }
#pragma omp parallel for schedule(dynamic, 1) num_threads(nth)
    for (int64_t j = 0; j < jobs; ++j) {
      const uint64_t k0 = (uint64_t)j / split * per, part = (uint64_t)j % split;
      const uint64_t r0 = h * part / split, r1 = h * (part + 1) / split;
      for (uint64_t k = k0; k < k0 + per; ++k) {
        if (cmw_rows(blocks + 2 * psize * (k / 4), m, (int)(k % 4), all + 2 * csize * k, r0, r1)) {
#pragma omp atomic write
          nz[k] = 1;
        }
      }
    }
    /* keep the nonzero children in order (blocks move only towards the
     * front, each after every earlier one: a sequential compaction) */
    uint64_t nn = 0;
    for (uint64_t k = 0; k < kids; ++k) {
      if (!nz[k]) continue;
      if (nn != k) memmove(all + 2 * csize * nn, all + 2 * csize * k, sizeof(double) * 2 * csize);
      npre[nn++] = pre[k / 4] * 4 + (k % 4);
    }
    free(nz);
    if (live) live[i] = nn;
    free(pre);
    pre = npre;
    double* tmp = blocks;
    blocks = all;
    all = tmp;
    nf = nn;
    if (nf == 0) break;
  }
  for (uint64_t f = 0; f < nf; ++f) {
    out[2 * pre[f]] = blocks[2 * f];
    out[2 * pre[f] + 1] = blocks[2 * f + 1];
  }
  free(pre);
  free(blocks);
  free(all);
  return ORACLE_OK;
}

/* ------------------------------------------------------------------------ */
/* (5) Synthesis A = sum_t omega_t sigma^t (eq. (PauliDecomposition), read   */
/* left to right).  Plain sums, for reconstruction checks.  Cost 8^n.        */
/* ------------------------------------------------------------------------ */
int oracle_synthesize(const double* w, int n, double* A) {
  if (n < 0 || n > 12 || !w || !A) return ORACLE_EINVAL;
  const uint64_t dim = (uint64_t)1 << n, count = dim * dim;
  memset(A, 0, sizeof(double) * 2 * count);
  unsigned char* e = (unsigned char*)malloc(dim);
  if (!e) return ORACLE_ENOMEM;
  for (uint64_t q = 0; q < count; ++q) {
    const double wr = w[2 * q], wi = w[2 * q + 1];
    if (wr == 0.0 && wi == 0.0) continue;
    const uint64_t x = oracle_xy_mask(q, n);
    row_phases(q, n, e);
    for (uint64_t i = 0; i < dim; ++i) {
      double pr, pi;
      mul_ipow(e[i], wr, wi, &pr, &pi);
      double* a = A + 2 * (i * dim + (i ^ x)); /* sigma^t[i][i^x] */
      a[0] += pr;
      a[1] += pi;
    }
  }
  free(e);
  return ORACLE_OK;
}

/* ------------------------------------------------------------------------ */
/* (6) Partial TPD, Fig. 2 / Algorithm 3.                                    */
/* Only the strings listed in `req` (canonical indices, any order, repeats   */
/* allowed) are computed.  The request tree T is the set of their prefixes;  */
/* at each node only the children present in T are sliced, and a zero child */
/* CMW ends its branch (its requested weights are zero).  out[s] receives    */
/* the weight of req[s].                                                     */
/* ------------------------------------------------------------------------ */
typedef struct {
  int n;
  const uint64_t* req; /* sorted unique */
  size_t nreq;
  double* vals;        /* per sorted request */
  int failed;
} part_ctx;

/* sorted requests in [lo, hi) all share the prefix of length n-m */
static void tpd_part(part_ctx* ctx, const double* M, int m, size_t lo, size_t hi) {
  if (m == 0) {
    ctx->vals[2 * lo] = M[0];
    ctx->vals[2 * lo + 1] = M[1];
    return;
  }
  const uint64_t h = (uint64_t)1 << (m - 1);
  double* C = (double*)malloc(sizeof(double) * 2 * h * h);
  if (!C) { ctx->failed = 1; return; }
  const int shift = 2 * (m - 1);
  size_t a = lo;
  while (a < hi && !ctx->failed) {
    const int t = (int)((ctx->req[a] >> shift) & 3u);
    size_t b = a;
    while (b < hi && (int)((ctx->req[b] >> shift) & 3u) == t) ++b;
    if (cmw(M, m, t, C)) tpd_part(ctx, C, m - 1, a, b);
    a = b; /* zero CMW: the requested weights below stay 0 */
  }
  free(C);
}

static int cmp_u64(const void* a, const void* b) {
  const uint64_t x = *(const uint64_t*)a, y = *(const uint64_t*)b;
  return (x > y) - (x < y);
}

int oracle_tpd_partial(const double* A, int n, const uint64_t* req, size_t m, double* out) {
  if (n < 0 || n > 16 || !A || (!req && m) || (!out && m)) return ORACLE_EINVAL;
  if (m == 0) return ORACLE_OK;
  for (size_t s = 0; s < m; ++s)
    if ((req[s] >> (2 * n)) != 0) return ORACLE_EINVAL;
  uint64_t* sorted = (uint64_t*)malloc(sizeof(uint64_t) * m);
  double* vals = (double*)calloc(2 * m, sizeof(double));
  if (!sorted || !vals) { free(sorted); free(vals); return ORACLE_ENOMEM; }
  memcpy(sorted, req, sizeof(uint64_t) * m);
  qsort(sorted, m, sizeof(uint64_t), cmp_u64);
  size_t u = 0;
  for (size_t s = 0; s < m; ++s)
    if (s == 0 || sorted[s] != sorted[u - 1]) sorted[u++] = sorted[s];
  part_ctx ctx = {n, sorted, u, vals, 0};
  tpd_part(&ctx, A, n, 0, u);
  for (size_t s = 0; s < m && !ctx.failed; ++s) {
    const uint64_t* hit = (const uint64_t*)bsearch(&req[s], sorted, u, sizeof(uint64_t), cmp_u64);
    const size_t k = (size_t)(hit - sorted);
    out[2 * s] = vals[2 * k];
    out[2 * s + 1] = vals[2 * k + 1];
  }
  free(sorted);
  free(vals);
  return ctx.failed ? ORACLE_ENOMEM : ORACLE_OK;
}
