// tpd_select.hip -- kernels that select strings: request marking and
// gathering for the partial decomposition (the paper's Algorithm 3 at tile
// granularity) and ordered stream compaction of the nonzero weights into a
// sparse (q, w) list (the list L that Algorithms 1 and 2 return).
//
// All of them are memory-bound and simple: grid-stride loops over 64-bit
// element indices, coalesced 4- to 16-byte loads (complex or real-coded
// elements), integer atomics only on request bitmaps.
#include "tpd_internal.h"

namespace tpd {

// ---------------------------------------------------------------------------
// partial decomposition: request bitmaps and gather
// ---------------------------------------------------------------------------
__global__ void k_mark_requests(const uint64_t* __restrict__ req, uint64_t count, int n, int n1, int db1, int db2,
                                uint32_t* groups, uint32_t* tiles) {
  const uint64_t lim = (uint64_t)1 << (2 * n);
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t q = req[i];
    if (q >= lim) continue;  // answered with NaN by the gather
    uint64_t g, t;
    request_bits(q, n, n1, db1, db2, &g, &t);
    atomicOr(&groups[g >> 5], 1u << (g & 31));
    atomicOr(&tiles[t >> 5], 1u << (t & 31));
  }
}

__global__ void k_and_u32(uint32_t* __restrict__ dst, const uint32_t* __restrict__ src, uint64_t words) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < words;
       i += (uint64_t)gridDim.x * blockDim.x)
    dst[i] &= src[i];
}

// indices of the set bits of a bitmap, appended in any order; count must
// start at zero
__global__ void k_bits_to_list(const uint32_t* __restrict__ bits, uint64_t words, uint32_t* __restrict__ list,
                               uint32_t* count) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < words;
       i += (uint64_t)gridDim.x * blockDim.x) {
    uint32_t w = bits[i];
    if (!w) continue;
    uint32_t pos = atomicAdd(count, (uint32_t)__popc(w));
    while (w) {
      const int b = __builtin_ctz(w);
      list[pos++] = (uint32_t)(i * 32 + b);
      w &= w - 1;
    }
  }
}

// element helpers for complex (Cx) and real-coded (Rl) values
template <class S>
__device__ inline void set_nan(Cx<S>& v) {
  v.re = __builtin_nan("");
  v.im = __builtin_nan("");
}
template <class S>
__device__ inline void set_nan(Rl<S>& v) {
  v.re = __builtin_nan("");
}
template <class S>
__device__ inline bool keep_elem(const Cx<S>& v, S tol) {
  return keep_coeff<S>(v.re, v.im, tol);
}
template <class S>
__device__ inline bool keep_elem(const Rl<S>& v, S tol) {
  return keep_coeff<S>(v.re, (S)0, tol);
}

// T: double / float (complex elements) or Real<double> / Real<float>
template <class T>
__global__ void k_gather(const typename Elem<T>::type* __restrict__ c, int n, int matrix_layout,
                         const uint64_t* __restrict__ req, uint64_t count, typename Elem<T>::type* __restrict__ values) {
  const uint64_t lim = (uint64_t)1 << (2 * n);
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t q = req[i];
    typename Elem<T>::type v;
    if (q < lim)
      v = c[storage_of_q(q, n, matrix_layout != 0)];
    else
      set_nan(v);
    values[i] = v;
  }
}

static unsigned grid_for(uint64_t items, unsigned block, unsigned cap) {
  uint64_t g = (items + block - 1) / block;
  if (g > cap) g = cap;
  return g ? (unsigned)g : 1u;
}

hipError_t launch_mark_requests(const uint64_t* req, uint64_t count, int n, int n1, int db1, int db2,
                                uint32_t* groups, uint32_t* tiles, hipStream_t st) {
  if (count == 0) return hipSuccess;
  hipLaunchKernelGGL(k_mark_requests, dim3(grid_for(count, 256, 8192)), dim3(256), 0, st, req, count, n, n1, db1,
                     db2, groups, tiles);
  return hipGetLastError();
}

hipError_t launch_and_u32(uint32_t* dst, const uint32_t* src, uint64_t words, hipStream_t st) {
  if (words == 0) return hipSuccess;
  hipLaunchKernelGGL(k_and_u32, dim3(grid_for(words, 256, 4096)), dim3(256), 0, st, dst, src, words);
  return hipGetLastError();
}

hipError_t launch_bits_to_list(const uint32_t* bits, uint64_t words, uint32_t* list, uint32_t* count,
                               hipStream_t st) {
  if (words == 0) return hipSuccess;
  hipLaunchKernelGGL(k_bits_to_list, dim3(grid_for(words, 256, 4096)), dim3(256), 0, st, bits, words, list, count);
  return hipGetLastError();
}

template <class T>
static void gather_t(const void* coeffs, int n, bool matrix_layout, const uint64_t* req, uint64_t count,
                     void* values, unsigned g, hipStream_t st) {
  using E = typename Elem<T>::type;
  hipLaunchKernelGGL(k_gather<T>, dim3(g), dim3(256), 0, st, (const E*)coeffs, n, (int)matrix_layout, req, count,
                     (E*)values);
}

hipError_t launch_gather(Dtype dt, const void* coeffs, int n, bool matrix_layout, const uint64_t* req,
                         uint64_t count, void* values, hipStream_t st) {
  if (count == 0) return hipSuccess;
  const unsigned g = grid_for(count, 256, 16384);
  switch (dt) {
    case DT_C128: gather_t<double>(coeffs, n, matrix_layout, req, count, values, g, st); break;
    case DT_C64: gather_t<float>(coeffs, n, matrix_layout, req, count, values, g, st); break;
    case DT_R64: gather_t<Real<double>>(coeffs, n, matrix_layout, req, count, values, g, st); break;
    case DT_R32: gather_t<Real<float>>(coeffs, n, matrix_layout, req, count, values, g, st); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// ordered compaction: count per chunk, exclusive scan, write
// ---------------------------------------------------------------------------
// A chunk is kCompactChunk consecutive storage elements, handled by one
// workgroup of 256 threads; element (chunk, j, tid) = chunk * 4096 +
// j * 256 + tid, so every load instruction of a wave reads 64 consecutive
// elements and storage order is (j, wave, lane) order.
constexpr int kCT = 256;
constexpr int kCJ = (int)(kCompactChunk / kCT);  // 16

template <class T, class S = typename Elem<T>::scalar>
__global__ void __launch_bounds__(kCT) k_compact_count(const typename Elem<T>::type* __restrict__ c, uint64_t elems,
                                                       S tol, uint32_t* __restrict__ counts) {
  __shared__ uint32_t wsum[kCT / 64];
  const uint64_t base = (uint64_t)blockIdx.x * kCompactChunk;
  const uint32_t tid = threadIdx.x;
  uint32_t cnt = 0;
#pragma unroll
  for (int j = 0; j < kCJ; ++j) {
    const uint64_t i = base + (uint64_t)j * kCT + tid;
    bool k = false;
    if (i < elems) k = keep_elem(c[i], tol);
    cnt += (uint32_t)__popcll(__ballot(k));
  }
  if ((tid & 63) == 0) wsum[tid >> 6] = cnt;
  __syncthreads();
  if (tid == 0) {
    uint32_t t = 0;
    for (int w = 0; w < kCT / 64; ++w) t += wsum[w];
    counts[blockIdx.x] = t;
  }
}

// one workgroup of 1024 threads; thread t owns a contiguous range of chunks
__global__ void __launch_bounds__(1024) k_compact_scan(const uint32_t* __restrict__ counts, uint64_t nchunks,
                                                       uint64_t* __restrict__ offsets, uint64_t* __restrict__ total) {
  __shared__ uint64_t part[1024];
  const uint32_t tid = threadIdx.x;
  const uint64_t per = (nchunks + 1023) / 1024;
  const uint64_t b = (uint64_t)tid * per;
  const uint64_t e = b + per < nchunks ? b + per : nchunks;
  uint64_t s = 0;
  for (uint64_t k = b; k < e; ++k) s += counts[k];
  part[tid] = s;
  __syncthreads();
  // Hillis-Steele inclusive scan over the 1024 partial sums
  for (uint32_t o = 1; o < 1024; o <<= 1) {
    const uint64_t add = tid >= o ? part[tid - o] : 0;
    __syncthreads();
    part[tid] += add;
    __syncthreads();
  }
  uint64_t run = part[tid] - s;  // exclusive
  for (uint64_t k = b; k < e; ++k) {
    offsets[k] = run;
    run += counts[k];
  }
  if (tid == 1023) *total = part[1023];
}

template <class T, class S = typename Elem<T>::scalar>
__global__ void __launch_bounds__(kCT)
    k_compact_write(const typename Elem<T>::type* __restrict__ c, uint64_t elems, int n, int matrix_layout, S tol,
                    const uint32_t* __restrict__ counts, const uint64_t* __restrict__ offsets, uint64_t capacity,
                    uint64_t* __restrict__ q_out, typename Elem<T>::type* __restrict__ w_out) {
  using E = typename Elem<T>::type;
  __shared__ uint32_t cnt[kCJ * (kCT / 64)];
  __shared__ uint32_t excl[kCJ * (kCT / 64)];
  const uint32_t tid = threadIdx.x, lane = tid & 63u, wave = tid >> 6;
  constexpr int NW = kCT / 64;
  const uint64_t nchunks = (elems + kCompactChunk - 1) / kCompactChunk;
  // persistent grid over the chunks: chunks without kept elements cost one
  // scalar read each, not a workgroup launch.  LDS reuse across iterations is
  // ordered by the two barriers of each iteration (cnt is rewritten only after
  // wave 0 has read it, excl only after every wave has read it).
  for (uint64_t chunk = blockIdx.x; chunk < nchunks; chunk += gridDim.x) {
    if (counts[chunk] == 0) continue;  // uniform per workgroup
    const uint64_t off0 = offsets[chunk];
    if (off0 >= capacity) continue;
    const uint64_t base = chunk * kCompactChunk;

    E v[kCJ];
    uint64_t m[kCJ];
#pragma unroll
    for (int j = 0; j < kCJ; ++j) {
      const uint64_t i = base + (uint64_t)j * kCT + tid;
      bool k = false;
      if (i < elems) {
        v[j] = c[i];
        k = keep_elem(v[j], tol);
      }
      m[j] = __ballot(k);
      if (lane == 0) cnt[j * NW + wave] = (uint32_t)__popcll(m[j]);
    }
    __syncthreads();
    if (wave == 0) {
      // exclusive scan of the kCJ * NW = 64 (j, wave) counts in storage order
      const uint32_t x = cnt[lane];
      uint32_t inc = x;
      for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(inc, o);
        if ((int)lane >= o) inc += y;
      }
      excl[lane] = inc - x;
    }
    __syncthreads();
    const uint64_t below = lane ? (~0ull >> (64 - lane)) : 0ull;
#pragma unroll
    for (int j = 0; j < kCJ; ++j) {
      if (!((m[j] >> lane) & 1ull)) continue;
      const uint64_t pos = off0 + excl[j * NW + wave] + (uint64_t)__popcll(m[j] & below);
      if (pos >= capacity) continue;
      const uint64_t i = base + (uint64_t)j * kCT + tid;
      q_out[pos] = q_of_storage(i, n, matrix_layout != 0);
      w_out[pos] = v[j];
    }
  }
}

template <class T>
static void compact_count_t(const void* coeffs, uint64_t elems, double tol, uint32_t* counts, uint64_t nchunks,
                            hipStream_t st) {
  using E = typename Elem<T>::type;
  using S = typename Elem<T>::scalar;
  hipLaunchKernelGGL((k_compact_count<T>), dim3((unsigned)nchunks), dim3(kCT), 0, st, (const E*)coeffs, elems,
                     (S)tol, counts);
}

hipError_t launch_compact_count(Dtype dt, const void* coeffs, uint64_t elems, double tol, uint32_t* counts,
                                hipStream_t st) {
  const uint64_t nchunks = (elems + kCompactChunk - 1) / kCompactChunk;
  if (nchunks == 0) return hipSuccess;
  switch (dt) {
    case DT_C128: compact_count_t<double>(coeffs, elems, tol, counts, nchunks, st); break;
    case DT_C64: compact_count_t<float>(coeffs, elems, tol, counts, nchunks, st); break;
    case DT_R64: compact_count_t<Real<double>>(coeffs, elems, tol, counts, nchunks, st); break;
    case DT_R32: compact_count_t<Real<float>>(coeffs, elems, tol, counts, nchunks, st); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_compact_scan(const uint32_t* counts, uint64_t nchunks, uint64_t* offsets, uint64_t* total,
                               hipStream_t st) {
  hipLaunchKernelGGL(k_compact_scan, dim3(1), dim3(1024), 0, st, counts, nchunks, offsets, total);
  return hipGetLastError();
}

template <class T>
static void compact_write_t(const void* coeffs, uint64_t elems, int n, bool matrix_layout, double tol,
                            const uint32_t* counts, const uint64_t* offsets, uint64_t capacity, uint64_t* q_out,
                            void* w_out, unsigned grid, hipStream_t st) {
  using E = typename Elem<T>::type;
  using S = typename Elem<T>::scalar;
  hipLaunchKernelGGL((k_compact_write<T>), dim3(grid), dim3(kCT), 0, st, (const E*)coeffs, elems, n,
                     (int)matrix_layout, (S)tol, counts, offsets, capacity, q_out, (E*)w_out);
}

hipError_t launch_compact_write(Dtype dt, const void* coeffs, int n, bool matrix_layout, double tol,
                                const uint32_t* counts, const uint64_t* offsets, uint64_t capacity,
                                uint64_t* q_out, void* w_out, hipStream_t st) {
  const uint64_t elems = (uint64_t)1 << (2 * n);
  const uint64_t nchunks = (elems + kCompactChunk - 1) / kCompactChunk;
  if (capacity == 0 || nchunks == 0) return hipSuccess;
  // a few workgroups per CU loop over the chunks (most are empty for sparse
  // spectra); 2048 covers 256 CUs with eight each
  const unsigned grid = (unsigned)std::min<uint64_t>(nchunks, 2048);
  switch (dt) {
    case DT_C128:
      compact_write_t<double>(coeffs, elems, n, matrix_layout, tol, counts, offsets, capacity, q_out, w_out, grid, st);
      break;
    case DT_C64:
      compact_write_t<float>(coeffs, elems, n, matrix_layout, tol, counts, offsets, capacity, q_out, w_out, grid, st);
      break;
    case DT_R64:
      compact_write_t<Real<double>>(coeffs, elems, n, matrix_layout, tol, counts, offsets, capacity, q_out, w_out,
                                    grid, st);
      break;
    case DT_R32:
      compact_write_t<Real<float>>(coeffs, elems, n, matrix_layout, tol, counts, offsets, capacity, q_out, w_out,
                                   grid, st);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace tpd
