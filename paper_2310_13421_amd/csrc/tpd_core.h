// tpd_core.h -- index algebra and butterfly of the MI355X TPD kernels.
//
// Shared by the HIP kernels (device) and by the host-side schedule emulator
// used in CPU tests, so both execute the very same address maps, thread
// roles and arithmetic.  Nothing here allocates or launches.
//
// Coordinates.  For an n-qubit matrix A (row-major 2^n x 2^n) every entry is
// addressed by (x, d) with x = row index and d = row XOR column, so
// A[r][c] has x = r, d = r ^ c.  One slicing step of the paper (section
// "Methods", eq. (CumulativeWeightsDefinition)) for qubit level k pairs the
// entries that differ in bit (n-k) of both row and column, i.e. in bit
// (n-k) of x with d fixed:
//   d-bit = 0: (A11, A22) -> (A11+A22)/2 at x-bit 0  [letter I]
//                             (A11-A22)/2 at x-bit 1  [letter Z]
//   d-bit = 1: (A12, A21) -> (A12+A21)/2 at x-bit 0  [letter X]
//                            i(A12-A21)/2 at x-bit 1  [letter Y]
// so a level is a radix-2 butterfly along x whose second output is
// multiplied by i when the d-bit is set.  After all n levels the value at
// (x, d) is the weight of the string with hi(t_k) = x bit (n-k) and
// lo(t_k) = (x ^ d) bit (n-k), where I=(0,0), X=(0,1), Y=(1,0), Z=(1,1):
// the coefficient of sigma^t sits at canonical index
//   q = sum_k t_k 4^(n-k) = interleave(hi bits, lo bits)
// (section "Problem formulation", eq. (PauliString)).
//
// Layouts (all are XOR-linear maps (x, d) -> element offset):
//   MAT : (x << n) | (x ^ d)               the matrix itself / the weights
//                                          kept at "row = hi, column = lo"
//   CAN : interleave(x, x ^ d)             canonical base-4 order
//   MID : CAN with its low 2*DB bits replaced by (x_low << DB) | d_low;
//         the intermediate order between the two sweeps of the
//         out-of-place canonical schedule (see tpd_kernels.hip).
#pragma once
#include <stdint.h>

#if defined(__HIPCC__)
#define TPD_HD __host__ __device__ __forceinline__
#else
#define TPD_HD inline
#endif

namespace tpd {

// L_CANR: the canonical order of L_CAN in an array of real values (the
// weights of a Hermitian matrix are real; only their real parts are stored)
enum Layout : int { L_MAT = 0, L_CAN = 1, L_MID = 2, L_CANR = 3 };

// spread the low 16 bits of v to the even bit positions
TPD_HD uint32_t spread16(uint32_t v) {
  v &= 0xFFFFu;
  v = (v | (v << 8)) & 0x00FF00FFu;
  v = (v | (v << 4)) & 0x0F0F0F0Fu;
  v = (v | (v << 2)) & 0x33333333u;
  v = (v | (v << 1)) & 0x55555555u;
  return v;
}
TPD_HD uint64_t spread32(uint64_t v) {
  return (uint64_t)spread16((uint32_t)v) | ((uint64_t)spread16((uint32_t)(v >> 16)) << 32);
}

template <int L>
TPD_HD uint64_t layout_addr(uint64_t x, uint64_t d, int n, int db) {
  if constexpr (L == L_MAT) {
    return (x << n) | (x ^ d);
  } else if constexpr (L == L_CAN || L == L_CANR) {
    return (spread32(x) << 1) | spread32(x ^ d);
  } else {
    const uint64_t m = ((uint64_t)1 << db) - 1;
    const uint64_t can = (spread32(x) << 1) | spread32(x ^ d);
    return (can & ~((m << db) | m)) | ((x & m) << db) | (d & m);
  }
}
TPD_HD uint64_t layout_addr_rt(int L, uint64_t x, uint64_t d, int n, int db) {
  return L == L_MAT ? layout_addr<L_MAT>(x, d, n, db)
                    : ((L == L_CAN || L == L_CANR) ? layout_addr<L_CAN>(x, d, n, db) : layout_addr<L_MID>(x, d, n, db));
}

// ---------------------------------------------------------------------------
// Tile geometry.  A tile holds 2^B elements, B = DB + XB + MB:
//   tile bits [0, DB)          dl: low d bits (DB contiguous XOR-diagonals)
//   tile bits [DB, DB+XB)      xl: the XB x bits this sweep transforms
//   tile bits [DB+XB, B)       ml: matrix index when small matrices are packed
// Each of the 2^(B-R) threads holds 2^R elements in registers.  A sweep runs
// NPH register phases; between phases the tile is exchanged through LDS.
// ---------------------------------------------------------------------------
constexpr int kMaxPh = 4;

struct Roles {
  int nph;
  int nxf[kMaxPh];       // transform slots of phase p are reg slots 0..nxf-1
  int reg[kMaxPh][4];    // tile bit held by register slot s (-1 = unused)
  int lane[kMaxPh][6];   // tile bit held by lane bit b
  int wave[kMaxPh][4];   // tile bit held by wave bit b
  // store mapping for the canonical order (st_ok): lanes hold d0, x0, d1,
  // x1, d2, x2, which are the six lowest bits of q, so every store
  // instruction of a wave writes 64 consecutive coefficients; registers and
  // waves take d3, x3, d4, x4, ... and then the remaining x bits
  bool st_ok;
  int st_reg[4];
  int st_lane[6];
  int st_wave[4];
};

template <int XB_, int DB_, int MB_, int R_, int ORDER_>
struct Geom {
  static constexpr int XB = XB_, DB = DB_, MB = MB_, R = R_, ORDER = ORDER_;
  static constexpr int B = XB + DB + MB;
  static constexpr int TB = B - R;                 // thread bits
  static constexpr int NT = 1 << TB;
  static constexpr int E = 1 << R;
  static constexpr int LB = TB < 6 ? TB : 6;
  static constexpr int WB = TB - LB;
  static constexpr int NPH = XB == 0 ? 1 : (XB + R - 1) / R;
  static_assert(R >= 0 && R <= 4, "at most 16 elements per thread");
  static_assert(TB >= 0 && WB <= 4, "at most 16 waves");
  static_assert(NPH <= kMaxPh, "too many register phases");
  static_assert(R <= XB + DB, "registers must hold x or d bits of one matrix");
};

// bit roles of every phase, computed at compile time
template <class G>
constexpr Roles make_roles() {
  Roles r{};
  r.nph = G::NPH;
  for (int p = 0; p < kMaxPh; ++p) {
    r.nxf[p] = 0;
    for (int s = 0; s < 4; ++s) r.reg[p][s] = -1;
    for (int s = 0; s < 6; ++s) r.lane[p][s] = -1;
    for (int s = 0; s < 4; ++s) r.wave[p][s] = -1;
  }
  for (int p = 0; p < G::NPH; ++p) {
    bool used[32] = {};
    // transform bits of this phase (xl bit indices), highest first
    int lo, hi;  // [lo, hi)
    if (G::ORDER == 0) {  // top levels first (the paper's level order)
      hi = G::XB - G::R * p;
      lo = hi - G::R < 0 ? 0 : hi - G::R;
    } else {              // bottom group first
      lo = G::R * p;
      hi = lo + G::R > G::XB ? G::XB : lo + G::R;
    }
    int s = 0;
    for (int b = hi - 1; b >= lo; --b) {
      r.reg[p][s++] = G::DB + b;
      used[G::DB + b] = true;
    }
    r.nxf[p] = s;
    // passengers: other xl bits (highest first), then dl bits (highest first)
    for (int b = G::XB - 1; b >= 0 && s < G::R; --b)
      if (!used[G::DB + b]) { r.reg[p][s++] = G::DB + b; used[G::DB + b] = true; }
    for (int b = G::DB - 1; b >= 0 && s < G::R; --b)
      if (!used[b]) { r.reg[p][s++] = b; used[b] = true; }
    // lanes: dl ascending, then xl ascending, then ml ascending; rest -> waves
    int l = 0, w = 0;
    for (int b = 0; b < G::B; ++b) {
      if (used[b]) continue;
      if (l < G::LB) r.lane[p][l++] = b;
      else r.wave[p][w++] = b;
      used[b] = true;
    }
  }
  // canonical-order store mapping
  r.st_ok = G::LB == 6 && G::DB >= 3 && G::XB >= 3 && G::MB == 0;
  for (int s = 0; s < 4; ++s) r.st_reg[s] = -1;
  for (int s = 0; s < 6; ++s) r.st_lane[s] = -1;
  for (int s = 0; s < 4; ++s) r.st_wave[s] = -1;
  if (r.st_ok) {
    int order[32] = {};
    int k = 0;
    for (int b = 0; b < G::DB || b < G::XB; ++b) {
      if (b < G::DB) order[k++] = b;           // d bit b
      if (b < G::XB) order[k++] = G::DB + b;   // x bit b
    }
    int i = 0;
    for (int l = 0; l < 6; ++l) r.st_lane[l] = order[i++];
    for (int s = 0; s < G::R; ++s) r.st_reg[s] = order[i++];
    for (int w = 0; w < G::WB; ++w) r.st_wave[w] = order[i++];
  }
  return r;
}

// tile-element index of (thread, register j) in phase p
template <class G>
TPD_HD uint32_t elem_base(const Roles& r, int p, uint32_t tid) {
  uint32_t e = 0;
  for (int b = 0; b < G::LB; ++b) e |= ((tid >> b) & 1u) << r.lane[p][b];
  for (int b = 0; b < G::WB; ++b) e |= ((tid >> (G::LB + b)) & 1u) << r.wave[p][b];
  return e;
}
template <class G>
TPD_HD constexpr uint32_t elem_reg(const Roles& r, int p, uint32_t j) {
  uint32_t e = 0;
  for (int s = 0; s < G::R; ++s) e |= ((j >> s) & 1u) << r.reg[p][s];
  return e;
}
// the same for the canonical-order store mapping
template <class G>
TPD_HD uint32_t elem_base_st(const Roles& r, uint32_t tid) {
  uint32_t e = 0;
  for (int b = 0; b < G::LB; ++b) e |= ((tid >> b) & 1u) << r.st_lane[b];
  for (int b = 0; b < G::WB; ++b) e |= ((tid >> (G::LB + b)) & 1u) << r.st_wave[b];
  return e;
}
template <class G>
TPD_HD constexpr uint32_t elem_reg_st(const Roles& r, uint32_t j) {
  uint32_t e = 0;
  for (int s = 0; s < G::R; ++s) e |= ((j >> s) & 1u) << r.st_reg[s];
  return e;
}

// ---------------------------------------------------------------------------
// Complex value helpers and the slicing butterfly.
// ---------------------------------------------------------------------------
template <class S>
struct alignas(2 * sizeof(S)) Cx {
  S re, im;
};

// (u, v) at x-bit (0, 1) -> ((u+v)/2, (u-v)/2 * (tw ? i : 1))
template <class S>
TPD_HD void butterfly(Cx<S>& u, Cx<S>& v, bool tw) {
  const S half = (S)0.5;
  const S sr = (u.re + v.re) * half, si = (u.im + v.im) * half;
  const S dr = (u.re - v.re) * half, di = (u.im - v.im) * half;
  u.re = sr;
  u.im = si;
  v.re = tw ? -di : dr;
  v.im = tw ? dr : di;
}

// Real input.  Every value the transform produces from a real matrix is a
// real number times i^k, k = the number of Y letters among the levels done
// so far (a Y output is i times a difference; all other outputs keep the
// phase of their pair, and both members of a pair share it).  A real-coded
// element holds that real factor, so a level is (u, v) -> ((u+v)/2, (u-v)/2)
// on 8 or 4 bytes per element, with the same roundings as the complex
// butterfly applied to the nonzero component.
template <class S>
struct alignas(sizeof(S)) Rl {
  S re;
};
template <class S>
TPD_HD void butterfly(Rl<S>& u, Rl<S>& v, bool) {
  const S half = (S)0.5;
  const S s = (u.re + v.re) * half, d = (u.re - v.re) * half;
  u.re = s;
  v.re = d;
}

// inverse of the real-coded butterfly: (s, t) -> (s + t, s - t).  With
// w = i on X/Y diagonals, t conj(w) = -i t, and t carries one more factor i
// than s (its Y letter), so both outputs keep s's phase: no twiddle.
template <class S>
TPD_HD void butterfly_inv(Rl<S>& u, Rl<S>& v, bool) {
  const S s = u.re, t = v.re;
  u.re = s + t;
  v.re = s - t;
}

// Element type of a kernel instantiation: Cx<S> for complex data, Rl<S> for
// the tag Real<S> (real input, real-coded output).
template <class S>
struct Real {};
template <class S>
struct Elem {
  using type = Cx<S>;
  using scalar = S;
  static constexpr bool real = false;
};
template <class S>
struct Elem<Real<S>> {
  using type = Rl<S>;
  using scalar = S;
  static constexpr bool real = true;
};
template <class S>
TPD_HD bool nonzero(const Cx<S>& z) {
  return z.re != (S)0 || z.im != (S)0;  // NaN counts as nonzero
}
template <class S>
TPD_HD bool nonzero(const Rl<S>& z) {
  return z.re != (S)0;
}

// inverse of butterfly(): (s, t) -> (s + t*conj(w), s - t*conj(w)), w = tw ? i : 1
// (synthesis A = sum_t w_t sigma^t, no scaling)
template <class S>
TPD_HD void butterfly_inv(Cx<S>& u, Cx<S>& v, bool tw) {
  const S tr = tw ? v.im : v.re, ti = tw ? -v.re : v.im;  // t * conj(w)
  const S sr = u.re, si = u.im;
  u.re = sr + tr;
  u.im = si + ti;
  v.re = sr - tr;
  v.im = si - ti;
}

// run the butterflies of phase p on a thread's registers.  d_thread is the
// d coordinate of register 0 (twiddle bits); x bit of transform slot s is
// xlo + (reg bit - DB).  Registers whose d differs (dl passengers) take
// their own twiddle bit.
template <class G, class S, bool INV = false, class E>
TPD_HD void phase_butterflies(const Roles& r, int p, E* v, uint64_t d_thread, int xlo) {
  for (int s = 0; s < r.nxf[p]; ++s) {
    const int xbit = xlo + (r.reg[p][s] - G::DB);
#pragma unroll
    for (int j = 0; j < G::E; ++j) {
      if (j & (1 << s)) continue;
      // d of register j: thread d XOR the dl passenger bits of j
      uint64_t dj = d_thread;
#pragma unroll
      for (int t = 0; t < G::R; ++t)
        if (r.reg[p][t] >= 0 && r.reg[p][t] < G::DB && ((j >> t) & 1)) dj ^= (uint64_t)1 << r.reg[p][t];
      const bool tw = (dj >> xbit) & 1u;
      if constexpr (INV) butterfly_inv(v[j], v[j | (1 << s)], tw);
      else butterfly(v[j], v[j | (1 << s)], tw);
    }
  }
}

}  // namespace tpd
