// tpd_batched.h -- the batched persistent kernel (many independent
// matrices of mixed n in one launch), instantiated once per dtype in
// tpd_batched_{c128,c64,r64,r32}.hip so the four compile in parallel.
//
// The work table lists items sorted by n (largest first): an item is 2^mb
// whole small matrices or one d-group tile of one n = 7..9 matrix, and every
// item is a single sweep over all n levels of its matrices, so items are
// independent (no waits between them).  Runs of items of one shape
// (BatchSeg: n, geometry variant, prefetch or not) are walked in order; in
// each run a workgroup takes the items congruent to its index modulo the
// grid, and with prefetch it issues the next item's loads before it
// transforms and stores the current one.  Every run is inlined into the
// kernel (no device-function calls: the item's descriptor and the kernel
// arguments stay in scalar registers), and the kernel is compiled for the
// residency its 64 KiB LDS tile allows, two workgroups per CU (batch_waves).  The shape tables
// are function-local constants so that every register index folds at
// compile time (as a class member the table was read from memory and the
// tile went to scratch).
#pragma once
#include "tpd_internal.h"

namespace tpd {

template <class S, class G, int OUTL>
struct BatchedOps {
  using E = typename Elem<S>::type;
  static constexpr int P = G::NPH;
  static constexpr int LAST = P - 1;
  static constexpr int N = G::XB;  // an item always transforms every level of its matrices
  static constexpr uint32_t DM = (1u << G::DB) - 1;
  static constexpr uint32_t XM = (1u << G::XB) - 1;

  __device__ __forceinline__ static void load(const BatchArgs& a, const BatchItem& it, E* v, uint32_t tid) {
    static constexpr Roles RL = make_roles<G>();
    const uint64_t td = it.tile;
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

  // transform the loaded item through its register phases and store it
  __device__ __forceinline__ static void process(const BatchArgs& a, const BatchItem& it, E* v, E* lds, uint32_t tid) {
    static constexpr Roles RL = make_roles<G>();
    const uint64_t td = it.tile;
#pragma unroll
    for (int p = 0; p < P; ++p) {
      const uint32_t ebp = elem_base<G>(RL, p, tid);
      phase_butterflies<G, S>(RL, p, v, (td << G::DB) | (ebp & DM), 0);
      if (p + 1 < P) {
        __syncthreads();  // also orders the previous item's LDS reads before these writes
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
};

// one run of items of one shape; PF: prefetch the next item
template <class S, class G, int OUTL, bool PF>
__device__ __forceinline__ void batched_run(const BatchArgs& a, uint32_t first, uint32_t end,
                                         typename Elem<S>::type* lds) {
  using Ops = BatchedOps<S, G, OUTL>;
  using E = typename Elem<S>::type;
  const uint32_t grid = gridDim.x;
  uint32_t i = first + (blockIdx.x + grid - first % grid) % grid;  // first item of this workgroup in the run
  if (i >= end) return;
  // the thread index as an opaque value defined here: otherwise the
  // compiler hoists every shape's per-thread offsets out of the loop over
  // runs and keeps them all live across the kernel (193-254 VGPRs, spills)
  uint32_t tid = threadIdx.x;
  asm volatile("" : "+v"(tid));
  if constexpr (PF) {
    E v[G::E], pf[G::E];
    BatchItem cur = a.items[i], nxt;
    Ops::load(a, cur, v, tid);
    uint32_t next = i + grid;
    if (next < end) {
      nxt = a.items[next];
      Ops::load(a, nxt, pf, tid);
    }
    Ops::process(a, cur, v, lds, tid);
    while (next < end) {
#pragma unroll
      for (int j = 0; j < G::E; ++j) v[j] = pf[j];
      cur = nxt;
      next += grid;
      if (next < end) {
        nxt = a.items[next];
        Ops::load(a, nxt, pf, tid);
      }
      Ops::process(a, cur, v, lds, tid);
    }
  } else {
    for (; i < end; i += grid) {
      E v[G::E];
      const BatchItem it = a.items[i];
      Ops::load(a, it, v, tid);
      Ops::process(a, it, v, lds, tid);
    }
  }
}

template <class S, int OUTL, int BT, int N>
__device__ __forceinline__ void batched_shape(const BatchArgs& a, const BatchSeg& sg, uint32_t code,
                                              typename Elem<S>::type* lds) {
  if (code == 0) batched_run<S, typename BatchShape<N, BT, 0>::G, OUTL, true>(a, sg.first, sg.end, lds);
  else if (code == 1) batched_run<S, typename BatchShape<N, BT, 0>::G, OUTL, false>(a, sg.first, sg.end, lds);
  else if constexpr (N >= 3) batched_run<S, typename BatchShape<N, BT, 1>::G, OUTL, true>(a, sg.first, sg.end, lds);
}

// waves per SIMD the kernel is compiled for: two 64 KiB tiles per CU, i.e.
// 2 waves per SIMD with 256-thread complex128 workgroups and 4 with the
// 512-thread workgroups of the 8- and 4-byte dtypes, except real float64,
// which would spill at 128 VGPRs and keeps one workgroup per CU
template <class S>
constexpr int batch_waves() {
  return (std::is_same_v<S, double> || std::is_same_v<S, Real<double>>) ? 2 : 4;
}

template <class S, int OUTL, int BT>
__global__ void __launch_bounds__(1 << (BT - 4)) __attribute__((amdgpu_waves_per_eu(batch_waves<S>(), batch_waves<S>()))) k_batched(BatchArgs a) {
  __shared__ typename Elem<S>::type lds[1 << BT];
  for (uint32_t s = 0; s < a.nseg; ++s) {
    const BatchSeg sg = a.segs[s];
    const uint32_t n = sg.shape / kBatchCodes, code = sg.shape % kBatchCodes;
    switch (n) {
      case 0: batched_shape<S, OUTL, BT, 0>(a, sg, code, lds); break;
      case 1: batched_shape<S, OUTL, BT, 1>(a, sg, code, lds); break;
      case 2: batched_shape<S, OUTL, BT, 2>(a, sg, code, lds); break;
      case 3: batched_shape<S, OUTL, BT, 3>(a, sg, code, lds); break;
      case 4: batched_shape<S, OUTL, BT, 4>(a, sg, code, lds); break;
      case 5: batched_shape<S, OUTL, BT, 5>(a, sg, code, lds); break;
      case 6: batched_shape<S, OUTL, BT, 6>(a, sg, code, lds); break;
      case 7: batched_shape<S, OUTL, BT, 7>(a, sg, code, lds); break;
      case 8: batched_shape<S, OUTL, BT, 8>(a, sg, code, lds); break;
      case 9: batched_shape<S, OUTL, BT, 9>(a, sg, code, lds); break;
      default: break;
    }
  }
}

template <class S, int BT>
hipError_t batched_launch(const BatchArgs& a, int grid, hipStream_t st) {
  if (a.layout == L_CAN)
    hipLaunchKernelGGL((k_batched<S, L_CAN, BT>), dim3(grid), dim3(1 << (BT - 4)), 0, st, a);
  else
    hipLaunchKernelGGL((k_batched<S, L_MAT, BT>), dim3(grid), dim3(1 << (BT - 4)), 0, st, a);
  return hipGetLastError();
}

}  // namespace tpd
