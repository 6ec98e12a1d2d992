// tpd_kernels.hip -- CDNA4 (gfx950) kernels of the Tensorized Pauli
// Decomposition (Hantzko, Binkowski, Gupta, arXiv:2310.13421).
//
// The transform is n slicing levels (section "Methods",
// eq. (CumulativeWeightsDefinition)); in the (x, d) coordinates of
// tpd_core.h a level is a butterfly along one x bit with d fixed, so the
// work splits into independent XOR-diagonals d and the levels of one sweep
// only need a tile of 2^XB rows x 2^DB diagonals on chip.
//
// Single matrix, n >= 9: two HBM sweeps.
//   sweep 1  levels 1..n1   (x bits [n2, n))  tiles: all 2^n1 row blocks of
//            a 2^DB-diagonal strip; reads A in 2^DB-element aligned runs.
//   sweep 2  levels n1+1..n (x bits [0, n2))  tiles: 2^n2 consecutive rows.
// Out of place, sweep 1 writes the MID order into the output buffer and
// sweep 2 runs in place on it, each tile reading and writing one closed set
// of addresses (16 runs of 2^(2 DB) elements in canonical order).  With the
// matrix layout both sweeps run in place on any buffer.
// n <= 8: one sweep, tiles of all 2^n rows x 2^DB diagonals.
//
// Inside a tile each thread holds 16 elements; up to four levels are done
// in registers per phase, and phases exchange the tile through LDS.  The
// paper's zero-CMW pruning becomes a bitmap with one bit per second-sweep
// tile, set in the first sweep's epilogue; second-sweep tiles whose bit is
// clear hold only zeros and are skipped without touching HBM.
#include "tpd_internal.h"

namespace tpd {

// non-temporal complex loads and stores through native 2-vectors
typedef double tpd_d2 __attribute__((ext_vector_type(2)));
typedef float tpd_f2 __attribute__((ext_vector_type(2)));
template <class S> struct Vec2;
template <> struct Vec2<double> { using type = tpd_d2; };
template <> struct Vec2<float> { using type = tpd_f2; };

template <class S>
__device__ __forceinline__ Cx<S> load_nt(const Cx<S>* p) {
  using V = typename Vec2<S>::type;
  const V v = __builtin_nontemporal_load(reinterpret_cast<const V*>(p));
  return Cx<S>{v.x, v.y};
}
template <class S>
__device__ __forceinline__ void store_nt(Cx<S>* p, const Cx<S>& c) {
  using V = typename Vec2<S>::type;
  V v;
  v.x = c.re;
  v.y = c.im;
  __builtin_nontemporal_store(v, reinterpret_cast<V*>(p));
}

// ---------------------------------------------------------------------------
// single-matrix sweep
// ---------------------------------------------------------------------------
template <class S, class G, int INL, int OUTL>
__global__ void __launch_bounds__(G::NT) k_sweep(SweepArgs a) {
  static constexpr Roles RL = make_roles<G>();
  constexpr int P = G::NPH;
  constexpr int LAST = P - 1;
  constexpr uint32_t DM = (1u << G::DB) - 1;
  constexpr uint32_t XM = (1u << G::XB) - 1;
  constexpr int NBW = (1 << G::XB) >= 32 ? (1 << G::XB) / 32 : 1;
  __shared__ Cx<S> lds[(P > 1) ? (1 << G::B) : 1];
  __shared__ uint32_t bits[NBW];

  const uint32_t tid = threadIdx.x;
  const Cx<S>* __restrict__ in = (const Cx<S>*)a.in;
  Cx<S>* __restrict__ out = (Cx<S>*)a.out;
  const int n = a.n, xlo = a.xlo, db = a.db;
  const uint64_t tdmask = ((uint64_t)1 << a.nfix_d) - 1;

  // register-slot address deltas (layouts are XOR-linear in (x, d))
  uint64_t din[G::R], dout[G::R];
#pragma unroll
  for (int s = 0; s < G::R; ++s) {
    const uint32_t ei = 1u << RL.reg[0][s];
    din[s] = layout_addr<INL>((uint64_t)((ei >> G::DB) & XM) << xlo, ei & DM, n, db);
    const uint32_t eo = 1u << RL.reg[LAST][s];
    dout[s] = layout_addr<OUTL>((uint64_t)((eo >> G::DB) & XM) << xlo, eo & DM, n, db);
  }
  const uint32_t eb0 = elem_base<G>(RL, 0, tid);
  const uint32_t ebl = elem_base<G>(RL, LAST, tid);

  for (uint64_t tile = blockIdx.x; tile < a.ntiles; tile += gridDim.x) {
    const uint64_t td = a.tdn ? a.td0 + tile % a.tdn : (tile & tdmask);
    const uint64_t xf = a.tdn ? tile / a.tdn : (tile >> a.nfix_d);
    const uint64_t xfix = (xf & (((uint64_t)1 << xlo) - 1)) | ((xf >> xlo) << (xlo + G::XB));
    if (a.bitmap_mode == 2) {
      const uint64_t bit = (td << a.bm_xbits) | xf;
      if (!((a.bitmap[bit >> 5] >> (bit & 31)) & 1u)) continue;  // zero subtree
    }
    if (a.bitmap_mode == 1 && tid < NBW) bits[tid] = 0;

    Cx<S> v[G::E];
    {
      const uint64_t x = xfix | ((uint64_t)((eb0 >> G::DB) & XM) << xlo);
      const uint64_t d = (td << G::DB) | (eb0 & DM);
      const uint64_t base = layout_addr<INL>(x, d, n, db);
#pragma unroll
      for (int j = 0; j < G::E; ++j) {
        uint64_t ad = base;
#pragma unroll
        for (int s = 0; s < G::R; ++s)
          if ((j >> s) & 1) ad ^= din[s];
        v[j] = a.nt ? load_nt(&in[ad]) : in[ad];
      }
    }

#pragma unroll
    for (int p = 0; p < P; ++p) {
      const uint32_t ebp = elem_base<G>(RL, p, tid);
      phase_butterflies<G, S>(RL, p, v, (td << G::DB) | (ebp & DM), xlo);
      if (p + 1 < P) {
        __syncthreads();
#pragma unroll
        for (int j = 0; j < G::E; ++j) lds[ebp | elem_reg<G>(RL, p, j)] = v[j];
        __syncthreads();
        const uint32_t ebn = elem_base<G>(RL, p + 1, tid);
#pragma unroll
        for (int j = 0; j < G::E; ++j) v[j] = lds[ebn | elem_reg<G>(RL, p + 1, j)];
      }
    }

    if (a.bitmap_mode == 1) {
      // OR "any nonzero" over the 2^DB diagonals (lanes [0, DB)) of each row
      // block; one bit per second-sweep tile (td, x_hi).  NaN counts as nonzero.
      const uint32_t lane = tid & 63u;
      constexpr uint32_t gsz = 1u << G::DB;
      constexpr uint64_t gmask = gsz >= 64 ? ~0ull : ((1ull << gsz) - 1);
      if (P == 1) __syncthreads();
#pragma unroll
      for (int j = 0; j < G::E; ++j) {
        const bool nz = (v[j].re != (S)0) || (v[j].im != (S)0);
        const uint64_t m = __ballot(nz);
        if ((lane & (gsz - 1)) == 0 && ((m >> lane) & gmask)) {
          const uint32_t xl = ((ebl | elem_reg<G>(RL, LAST, j)) >> G::DB) & XM;
          atomicOr(&bits[xl >> 5], 1u << (xl & 31));
        }
      }
      __syncthreads();
      if (tid < NBW) {
        const uint32_t w = bits[tid];
        if (w) {
          const uint64_t b0 = (td << a.bm_xbits) + 32ull * tid;
          atomicOr(&a.bitmap[b0 >> 5], w << (b0 & 31));
        }
      }
    }

    if (P == 1 && INL != OUTL) __syncthreads();  // in place: all loads before any store
    {
      const uint64_t x = xfix | ((uint64_t)((ebl >> G::DB) & XM) << xlo);
      const uint64_t d = (td << G::DB) | (ebl & DM);
      const uint64_t base = layout_addr<OUTL>(x, d, n, db);
#pragma unroll
      for (int j = 0; j < G::E; ++j) {
        uint64_t ad = base;
#pragma unroll
        for (int s = 0; s < G::R; ++s)
          if ((j >> s) & 1) ad ^= dout[s];
        if (a.nt) store_nt(&out[ad], v[j]);
        else out[ad] = v[j];
      }
    }
  }
}

// ---------------------------------------------------------------------------
// batched persistent kernel: one work item = packed whole matrices (n <= 6)
// or one d-group tile of one matrix (n = 7..9); every item is a single sweep.
// ---------------------------------------------------------------------------
BatchGeom batch_geom(int n) {
  switch (n) {
    case 0: return {0, 0, 8, 0};
    case 1: return {1, 1, 8, 2};
    case 2: return {2, 2, 8, 4};
    case 3: return {3, 3, 6, 4};
    case 4: return {4, 4, 4, 4};
    case 5: return {5, 5, 2, 4};
    case 6: return {6, 6, 0, 4};
    case 7: return {7, 5, 0, 4};
    case 8: return {8, 4, 0, 4};
    case 9: return {9, 3, 0, 4};
    default: return {-1, -1, -1, -1};
  }
}

template <class S, class G, int OUTL>
__device__ __noinline__ void batched_item(const BatchArgs& a, const BatchItem& it, Cx<S>* lds) {
  static constexpr Roles RL = make_roles<G>();
  constexpr int P = G::NPH;
  constexpr int LAST = P - 1;
  constexpr int N = G::XB;  // an item always transforms every level of its matrix
  constexpr uint32_t DM = (1u << G::DB) - 1;
  constexpr uint32_t XM = (1u << G::XB) - 1;
  const uint32_t tid = threadIdx.x;
  const uint64_t td = it.tile;

  Cx<S> v[G::E];
  {
    const uint32_t e = elem_base<G>(RL, 0, tid);
    const uint32_t ml = e >> (G::DB + G::XB);
    if (ml < it.nmat) {
      const Cx<S>* __restrict__ in = (const Cx<S>*)a.in_ptrs[a.perm[it.mat0 + ml]];
      const uint64_t base = layout_addr<L_MAT>((e >> G::DB) & XM, (td << G::DB) | (e & DM), N, G::DB);
#pragma unroll
      for (int j = 0; j < G::E; ++j) {
        const uint32_t er = elem_reg<G>(RL, 0, j);  // compile-time after unrolling
        v[j] = in[base ^ layout_addr<L_MAT>((er >> G::DB) & XM, er & DM, N, G::DB)];
      }
    } else {
#pragma unroll
      for (int j = 0; j < G::E; ++j) v[j] = Cx<S>{(S)0, (S)0};
    }
  }
#pragma unroll
  for (int p = 0; p < P; ++p) {
    const uint32_t ebp = elem_base<G>(RL, p, tid);
    phase_butterflies<G, S>(RL, p, v, (td << G::DB) | (ebp & DM), 0);
    if (p + 1 < P) {
      __syncthreads();
#pragma unroll
      for (int j = 0; j < G::E; ++j) lds[ebp | elem_reg<G>(RL, p, j)] = v[j];
      __syncthreads();
      const uint32_t ebn = elem_base<G>(RL, p + 1, tid);
#pragma unroll
      for (int j = 0; j < G::E; ++j) v[j] = lds[ebn | elem_reg<G>(RL, p + 1, j)];
    }
  }
  // whole matrices in place: every load of the item precedes every store
  __syncthreads();
  {
    const uint32_t e = elem_base<G>(RL, LAST, tid);
    const uint32_t ml = e >> (G::DB + G::XB);
    if (ml < it.nmat) {
      Cx<S>* __restrict__ out = (Cx<S>*)a.out_ptrs[a.perm[it.mat0 + ml]];
      const uint64_t base = layout_addr<OUTL>((e >> G::DB) & XM, (td << G::DB) | (e & DM), N, G::DB);
#pragma unroll
      for (int j = 0; j < G::E; ++j) {
        const uint32_t er = elem_reg<G>(RL, LAST, j);
        out[base ^ layout_addr<OUTL>((er >> G::DB) & XM, er & DM, N, G::DB)] = v[j];
      }
    }
  }
}

template <class S, int OUTL>
__device__ __forceinline__ void batched_dispatch(const BatchArgs& a, const BatchItem& it, Cx<S>* lds) {
  switch (it.n) {
    case 0: batched_item<S, Geom<0, 0, 8, 0, 0>, OUTL>(a, it, lds); break;
    case 1: batched_item<S, Geom<1, 1, 8, 2, 0>, OUTL>(a, it, lds); break;
    case 2: batched_item<S, Geom<2, 2, 8, 4, 0>, OUTL>(a, it, lds); break;
    case 3: batched_item<S, Geom<3, 3, 6, 4, 0>, OUTL>(a, it, lds); break;
    case 4: batched_item<S, Geom<4, 4, 4, 4, 0>, OUTL>(a, it, lds); break;
    case 5: batched_item<S, Geom<5, 5, 2, 4, 0>, OUTL>(a, it, lds); break;
    case 6: batched_item<S, Geom<6, 6, 0, 4, 0>, OUTL>(a, it, lds); break;
    case 7: batched_item<S, Geom<7, 5, 0, 4, 0>, OUTL>(a, it, lds); break;
    case 8: batched_item<S, Geom<8, 4, 0, 4, 0>, OUTL>(a, it, lds); break;
    case 9: batched_item<S, Geom<9, 3, 0, 4, 0>, OUTL>(a, it, lds); break;
    default: break;
  }
}

template <class S, int OUTL>
__global__ void __launch_bounds__(256) k_batched(BatchArgs a) {
  __shared__ Cx<S> lds[4096];
  for (uint32_t i = blockIdx.x; i < a.nitems; i += gridDim.x) {
    const BatchItem it = a.items[i];
    batched_dispatch<S, OUTL>(a, it, lds);
    __syncthreads();  // the next item reuses the LDS tile
  }
}

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------
__global__ void k_fill_u32(uint32_t* p, uint64_t words, uint32_t value) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < words;
       i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = value;
}

__global__ void k_popcount(const uint32_t* p, uint64_t words, unsigned long long* out) {
  unsigned long long c = 0;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < words;
       i += (uint64_t)gridDim.x * blockDim.x)
    c += __popc(p[i]);
  for (int o = 32; o > 0; o >>= 1) c += __shfl_down(c, o);
  if ((threadIdx.x & 63) == 0 && c) atomicAdd(out, c);
}

hipError_t launch_fill_u32(uint32_t* p, uint64_t words, uint32_t value, hipStream_t st) {
  if (words == 0) return hipSuccess;
  uint64_t g = (words + 255) / 256;
  if (g > 4096) g = 4096;
  hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)g), dim3(256), 0, st, p, words, value);
  return hipGetLastError();
}

hipError_t launch_popcount(const uint32_t* p, uint64_t words, unsigned long long* out, hipStream_t st) {
  uint64_t g = (words + 255) / 256;
  if (g > 2048) g = 2048;
  if (g == 0) g = 1;
  hipLaunchKernelGGL(k_popcount, dim3((unsigned)g), dim3(256), 0, st, p, words, out);
  return hipGetLastError();
}

hipError_t launch_batched_perm(Dtype dt, const void* const* in_ptrs, void* const* out_ptrs, const uint32_t* perm,
                               const BatchItem* items, uint32_t nitems, int layout, int grid, hipStream_t st) {
  BatchArgs a{in_ptrs, out_ptrs, perm, items, nitems, layout};
  if (a.nitems == 0) return hipSuccess;
  if (grid <= 0 || (uint32_t)grid > a.nitems) grid = (int)a.nitems;
  if (dt == DT_C128) {
    if (layout == L_CAN) hipLaunchKernelGGL((k_batched<double, L_CAN>), dim3(grid), dim3(256), 0, st, a);
    else hipLaunchKernelGGL((k_batched<double, L_MAT>), dim3(grid), dim3(256), 0, st, a);
  } else {
    if (layout == L_CAN) hipLaunchKernelGGL((k_batched<float, L_CAN>), dim3(grid), dim3(256), 0, st, a);
    else hipLaunchKernelGGL((k_batched<float, L_MAT>), dim3(grid), dim3(256), 0, st, a);
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// sweep dispatch
// ---------------------------------------------------------------------------
template <class S, int XB, int DB, int ORDER, int INL, int OUTL, int RR = 4>
static hipError_t launch_one(const SweepArgs& a, hipStream_t st) {
  // at most 1024 threads per tile, at most 16 registers per thread
  constexpr int R1 = (XB + DB - 10) > RR ? (XB + DB - 10) : RR;
  constexpr int R = (XB + DB) < R1 ? (XB + DB) : R1;
  using G = Geom<XB, DB, 0, R, ORDER>;
  if constexpr (!shape_fits<S>(XB, DB)) {
    return hipErrorInvalidValue;
  } else {
  uint64_t grid = a.ntiles;
  if (grid > 0x7FFFFFFFull) grid = 0x7FFFFFFFull;
  hipLaunchKernelGGL((k_sweep<S, G, INL, OUTL>), dim3((unsigned)grid), dim3(G::NT), 0, st, a);
  return hipGetLastError();
  }
}

template <class S>
static hipError_t dispatch_shape(const SweepDesc& s, const SweepArgs& a, hipStream_t st) {
  const bool one = s.in_layout == L_MAT && s.xlo == 0 && s.xb == a.n;
#define TPD_CASE(XB_, DB_)                                                                   \
  if (one && s.xb == XB_ && s.db == DB_) {                                                   \
    if (s.out_layout == L_CAN) return launch_one<S, XB_, DB_, 0, L_MAT, L_CAN>(a, st);       \
    if (s.out_layout == L_MAT) return launch_one<S, XB_, DB_, 0, L_MAT, L_MAT>(a, st);       \
  }
  TPD_SHAPES_ONE(TPD_CASE)
#undef TPD_CASE
#define TPD_TWO(XB_, DB_, RR_)                                                                        \
  if (s.in_layout == L_MAT && s.out_layout == L_MID) return launch_one<S, XB_, DB_, 0, L_MAT, L_MID, RR_>(a, st); \
  if (s.in_layout == L_MID && s.out_layout == L_CAN)                                                  \
    return s.order ? launch_one<S, XB_, DB_, 1, L_MID, L_CAN, RR_>(a, st)                            \
                   : launch_one<S, XB_, DB_, 0, L_MID, L_CAN, RR_>(a, st);                           \
  if (s.in_layout == L_MAT && s.out_layout == L_MAT)                                                  \
    return s.order ? launch_one<S, XB_, DB_, 1, L_MAT, L_MAT, RR_>(a, st)                            \
                   : launch_one<S, XB_, DB_, 0, L_MAT, L_MAT, RR_>(a, st);
#define TPD_CASE(XB_, DB_)                             \
  if (!one && s.xb == XB_ && s.db == DB_) {            \
    if (s.r == 2) { TPD_TWO(XB_, DB_, 2) }             \
    else if (s.r == 3) { TPD_TWO(XB_, DB_, 3) }        \
    else { TPD_TWO(XB_, DB_, 4) }                      \
  }
  TPD_SHAPES_TWO(TPD_CASE)
#undef TPD_CASE
#undef TPD_TWO
  return hipErrorInvalidValue;
}

bool sweep_supported(Dtype dt, const SweepDesc& s) {
#define TPD_CASE(XB_, DB_) \
  if (s.xb == XB_ && s.db == DB_) return dt == DT_C128 ? shape_fits<double>(XB_, DB_) : shape_fits<float>(XB_, DB_);
  TPD_SHAPES_ONE(TPD_CASE)
  TPD_SHAPES_TWO(TPD_CASE)
#undef TPD_CASE
  return false;
}

hipError_t launch_sweep(Dtype dt, const SweepDesc& s, const SweepArgs& a, hipStream_t st) {
  if (a.ntiles == 0) return hipSuccess;
  return dt == DT_C128 ? dispatch_shape<double>(s, a, st) : dispatch_shape<float>(s, a, st);
}

}  // namespace tpd
