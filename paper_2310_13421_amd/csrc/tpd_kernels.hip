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

// Seeded noise, uniform in [-1, 1): scalar i is the top bits of
// splitmix64(seed + i) (the published SplitMix64 finaliser).  The in-place
// autotuners refill their buffer with it before every timed run, so that the
// values do not decay towards zero over repeated transforms (all-zero data
// skips the pruning epilogue's atomics and lets the second sweep skip tiles,
// and timed that way the candidates rank differently).
template <class T>
__global__ void k_fill_noise(T* p, uint64_t count, uint64_t seed) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (uint64_t)gridDim.x * blockDim.x) {
    uint64_t z = seed + i * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    if constexpr (sizeof(T) == 8) p[i] = (T)(int64_t)(z >> 11) * (T)0x1p-52 - (T)1;
    else p[i] = (T)(int32_t)(uint32_t)(z >> 40) * (T)0x1p-23 - (T)1;
  }
}

hipError_t launch_fill_noise(void* p, uint64_t scalars, bool f64, uint64_t seed, hipStream_t st) {
  if (scalars == 0) return hipSuccess;
  uint64_t g = (scalars + 255) / 256;
  if (g > 8192) g = 8192;
  if (f64)
    hipLaunchKernelGGL(k_fill_noise<double>, dim3((unsigned)g), dim3(256), 0, st, (double*)p, scalars, seed);
  else
    hipLaunchKernelGGL(k_fill_noise<float>, dim3((unsigned)g), dim3(256), 0, st, (float*)p, scalars, seed);
  return hipGetLastError();
}

hipError_t launch_popcount(const uint32_t* p, uint64_t words, unsigned long long* out, hipStream_t st) {
  uint64_t g = (words + 255) / 256;
  if (g > 2048) g = 2048;
  if (g == 0) g = 1;
  hipLaunchKernelGGL(k_popcount, dim3((unsigned)g), dim3(256), 0, st, p, words, out);
  return hipGetLastError();
}

// batched kernel (tpd_batched.h), one instantiation unit per dtype
hipError_t launch_batched_c128(const BatchArgs& a, int grid, hipStream_t st);
hipError_t launch_batched_c64(const BatchArgs& a, int grid, hipStream_t st);
hipError_t launch_batched_r64(const BatchArgs& a, int grid, hipStream_t st);
hipError_t launch_batched_r32(const BatchArgs& a, int grid, hipStream_t st);

hipError_t launch_batched_perm(Dtype dt, const void* const* in_ptrs, void* const* out_ptrs, const uint32_t* perm,
                               const BatchItem* items, uint32_t nitems, const BatchSeg* segs, uint32_t nseg, int layout,
                               int grid, hipStream_t st) {
  BatchArgs a{in_ptrs, out_ptrs, perm, items, nitems, layout, segs, nseg};
  if (a.nitems == 0 || nseg == 0) return hipSuccess;
  if (grid <= 0 || (uint32_t)grid > a.nitems) grid = (int)a.nitems;
  switch (dt) {
    case DT_C128: return launch_batched_c128(a, grid, st);
    case DT_C64: return launch_batched_c64(a, grid, st);
    case DT_R64: return launch_batched_r64(a, grid, st);
    case DT_R32: return launch_batched_r32(a, grid, st);
    default: return hipErrorInvalidValue;
  }
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
