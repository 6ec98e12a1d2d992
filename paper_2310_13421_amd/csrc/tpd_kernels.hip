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

// ---------------------------------------------------------------------------
// batched persistent kernel: one work item = packed whole matrices (n <= 6)
// or one d-group tile of one matrix (n = 7..9); every item is a single sweep.
// ---------------------------------------------------------------------------
// S: double / float (complex), or Real<double> / Real<float> (real input,
// real-coded weights: the store writes each weight's nonzero component).
template <class S, class G, int OUTL>
__device__ __noinline__ void batched_item(const BatchArgs& a, const BatchItem& it, typename Elem<S>::type* lds) {
  using E = typename Elem<S>::type;
  static constexpr Roles RL = make_roles<G>();
  constexpr int P = G::NPH;
  constexpr int LAST = P - 1;
  constexpr int N = G::XB;  // an item always transforms every level of its matrix
  constexpr uint32_t DM = (1u << G::DB) - 1;
  constexpr uint32_t XM = (1u << G::XB) - 1;
  const uint32_t tid = threadIdx.x;
  const uint64_t td = it.tile;

  E v[G::E];
  {
    const uint32_t e = elem_base<G>(RL, 0, tid);
    const uint32_t ml = e >> (G::DB + G::XB);
    if (ml < it.nmat) {
      const E* __restrict__ in = (const E*)a.in_ptrs[a.perm[it.mat0 + ml]];
      const uint64_t base = layout_addr<L_MAT>((e >> G::DB) & XM, (td << G::DB) | (e & DM), N, G::DB);
#pragma unroll
      for (int j = 0; j < G::E; ++j) {
        const uint32_t er = elem_reg<G>(RL, 0, j);  // compile-time after unrolling
        v[j] = in[base ^ layout_addr<L_MAT>((er >> G::DB) & XM, er & DM, N, G::DB)];
      }
    } else {
#pragma unroll
      for (int j = 0; j < G::E; ++j) v[j] = E{};
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
      E* __restrict__ out = (E*)a.out_ptrs[a.perm[it.mat0 + ml]];
      const uint64_t base = layout_addr<OUTL>((e >> G::DB) & XM, (td << G::DB) | (e & DM), N, G::DB);
#pragma unroll
      for (int j = 0; j < G::E; ++j) {
        const uint32_t er = elem_reg<G>(RL, LAST, j);
        if constexpr (Elem<S>::real) {
          // the weight is i^y r, y = popcount(x & d): store its nonzero
          // component (r negated for y mod 4 = 2, 3)
          const uint32_t ee = e | er;
          const uint64_t x = (ee >> G::DB) & XM, d = (td << G::DB) | (ee & DM);
          if ((__popcll(x & d) >> 1) & 1) v[j].re = -v[j].re;
        }
        out[base ^ layout_addr<OUTL>((er >> G::DB) & XM, er & DM, N, G::DB)] = v[j];
      }
    }
  }
}

template <class S, int OUTL, int BT>
__device__ __forceinline__ void batched_dispatch(const BatchArgs& a, const BatchItem& it,
                                                 typename Elem<S>::type* lds) {
  switch (it.n) {
    case 0: batched_item<S, typename BatchShape<0, BT>::G, OUTL>(a, it, lds); break;
    case 1: batched_item<S, typename BatchShape<1, BT>::G, OUTL>(a, it, lds); break;
    case 2: batched_item<S, typename BatchShape<2, BT>::G, OUTL>(a, it, lds); break;
    case 3: batched_item<S, typename BatchShape<3, BT>::G, OUTL>(a, it, lds); break;
    case 4: batched_item<S, typename BatchShape<4, BT>::G, OUTL>(a, it, lds); break;
    case 5: batched_item<S, typename BatchShape<5, BT>::G, OUTL>(a, it, lds); break;
    case 6: batched_item<S, typename BatchShape<6, BT>::G, OUTL>(a, it, lds); break;
    case 7: batched_item<S, typename BatchShape<7, BT>::G, OUTL>(a, it, lds); break;
    case 8: batched_item<S, typename BatchShape<8, BT>::G, OUTL>(a, it, lds); break;
    case 9: batched_item<S, typename BatchShape<9, BT>::G, OUTL>(a, it, lds); break;
    default: break;
  }
}

template <class S, int OUTL, int BT>
__global__ void __launch_bounds__(1 << (BT - 4)) k_batched(BatchArgs a) {
  __shared__ typename Elem<S>::type lds[1 << BT];
  for (uint32_t i = blockIdx.x; i < a.nitems; i += gridDim.x) {
    const BatchItem it = a.items[i];
    batched_dispatch<S, OUTL, BT>(a, it, lds);
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

template <class S, int BT>
static void batched_launch(const BatchArgs& a, int layout, int grid, hipStream_t st) {
  if (layout == L_CAN)
    hipLaunchKernelGGL((k_batched<S, L_CAN, BT>), dim3(grid), dim3(1 << (BT - 4)), 0, st, a);
  else
    hipLaunchKernelGGL((k_batched<S, L_MAT, BT>), dim3(grid), dim3(1 << (BT - 4)), 0, st, a);
}

hipError_t launch_batched_perm(Dtype dt, const void* const* in_ptrs, void* const* out_ptrs, const uint32_t* perm,
                               const BatchItem* items, uint32_t nitems, int layout, int grid, hipStream_t st) {
  BatchArgs a{in_ptrs, out_ptrs, perm, items, nitems, layout};
  if (a.nitems == 0) return hipSuccess;
  if (grid <= 0 || (uint32_t)grid > a.nitems) grid = (int)a.nitems;
  switch (dt) {
    case DT_C128: batched_launch<double, batch_tile_bits(DT_C128)>(a, layout, grid, st); break;
    case DT_C64: batched_launch<float, batch_tile_bits(DT_C64)>(a, layout, grid, st); break;
    case DT_R64: batched_launch<Real<double>, batch_tile_bits(DT_R64)>(a, layout, grid, st); break;
    case DT_R32: batched_launch<Real<float>, batch_tile_bits(DT_R32)>(a, layout, grid, st); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// sweep dispatch (instantiations live in tpd_sweep_c128.hip, tpd_sweep_c64.hip,
// tpd_sweep_r64.hip and tpd_sweep_r32.hip)
// ---------------------------------------------------------------------------
hipError_t launch_sweep_c128(const SweepDesc& s, const SweepArgs& a, hipStream_t st);
hipError_t launch_sweep_c64(const SweepDesc& s, const SweepArgs& a, hipStream_t st);
hipError_t launch_sweep_r64(const SweepDesc& s, const SweepArgs& a, hipStream_t st);
hipError_t launch_sweep_r32(const SweepDesc& s, const SweepArgs& a, hipStream_t st);

hipError_t launch_sweep(Dtype dt, const SweepDesc& s, const SweepArgs& a, hipStream_t st) {
  if (a.ntiles == 0) return hipSuccess;
  switch (dt) {
    case DT_C128: return launch_sweep_c128(s, a, st);
    case DT_C64: return launch_sweep_c64(s, a, st);
    case DT_R64: return launch_sweep_r64(s, a, st);
    case DT_R32: return launch_sweep_r32(s, a, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace tpd
