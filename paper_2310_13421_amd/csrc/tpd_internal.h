// tpd_internal.h -- declarations shared by the kernel launchers and the C ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "tpd_core.h"

namespace tpd {

enum Dtype : int { DT_C128 = 0, DT_C64 = 1, DT_R64 = 2, DT_R32 = 3 };

// One HBM sweep over a single matrix: transform x bits [xlo, xlo+xb) for
// every d, tiles of 2^(xb+db) elements.
struct SweepDesc {
  int xlo, xb, db;
  int in_layout, out_layout;
  int bitmap_mode;  // 0 none, 1 set (first sweep), 2 check (second sweep)
  int order;        // register-phase order: 0 top levels first, 1 bottom first
  int r;            // log2 of the elements each thread holds (3 or 4)
  int grid;         // 0: one workgroup per tile; > 0: persistent grid of that size
  bool is_one;      // the single sweep of an n <= 8 schedule
  int herm;         // 1: the input is Hermitian (read representatives only)
  bool inv;         // inverse butterflies (synthesis)
  int tile_order;   // 1: row blocks rotate every 8 d-groups (second sweep, tuning)
  uint64_t ntiles;
};

struct SweepArgs {
  const void* in;
  void* out;
  int n;
  int xlo;
  int db;
  int nfix_d;        // n - db: number of fixed d bits per tile
  uint32_t* bitmap;  // 32-bit words, one bit per second-sweep tile
  int bitmap_mode;
  int bm_xbits;      // x bits of the first sweep (bit index = (td << bm_xbits) | x_hi)
  int bm_db;         // the second sweep's tile width (bitmap d-groups); 0 or db: this sweep's own
  int herm;          // 1: Hermitian input, two-sweep schedule
  const uint32_t* req;  // partial decomposition: bit per d-group td, tiles of unset groups are skipped (null: all)
  // partial decomposition, work list instead of all tiles (null: all):
  // list_shift > 0: list[g] are d-groups, tile t is (xf = t / count, group
  // t mod count), count << list_shift tiles; list_shift = 0: list[t] are
  // second-sweep tiles as bitmap bits (td << bm_xbits) | xf.  count =
  // list_count[0], written by an earlier kernel.
  const uint32_t* list;
  const uint32_t* list_count;
  int list_shift;
  uint64_t ntiles;  // with a list: the most tiles it can hold
  int tile_order;   // 1: rotated tile order (see SweepDesc)
  // chunked two-sweep order: chunk_bits > 0 restricts the launch to the
  // 2^chunk_bits consecutive d-groups starting at td_base (tile t is
  // (xf = t >> chunk_bits, td = td_base + t mod 2^chunk_bits)); 0: every group
  int chunk_bits;
  uint64_t td_base;
};

// Batched work item: `nmat` matrices of the same n starting at `mat0`
// (packed whole matrices), or one d-group tile of one matrix, in the item
// geometry `variant` (see batch_geom).
struct BatchItem {
  uint32_t mat0;
  uint16_t n;
  uint16_t nmat;
  uint32_t tile;
  uint32_t variant;
};

// A run of consecutive work items of one shape: items [first, end) of
// qubit count n in geometry variant `variant`, processed with (prefetch = 1)
// or without (0) the next item's loads issued before the current item is
// transformed.  The shape code n * 3 + code picks the device function:
// code 0 = (variant 0, prefetch), 1 = (variant 0, no prefetch),
// 2 = (variant 1, prefetch).
struct BatchSeg {
  uint32_t first, end;
  uint32_t shape;
  uint32_t pad;
};
constexpr int kBatchCodes = 3;
constexpr int batch_code_variant(int code) { return code == 2 ? 1 : 0; }
constexpr bool batch_code_prefetch(int code) { return code != 1; }
constexpr bool batch_code_ok(int n, int code) { return n >= 0 && n <= 9 && code >= 0 && code < kBatchCodes && (code != 2 || n >= 3); }

struct BatchArgs {
  const void* const* in_ptrs;   // device array of device pointers (caller's order)
  void* const* out_ptrs;        // device array of device pointers (may equal in_ptrs)
  const uint32_t* perm;         // device array: sorted position -> caller's index
  const BatchItem* items;       // device array
  uint32_t nitems;
  int layout;                   // L_CAN or L_MAT output
  const BatchSeg* segs;         // device array of the runs of one shape, in item order
  uint32_t nseg;
};

// scratch of the no-allocation entry point (tpd_scratch.hip): the pruning
// bitmap in a static device array of kNoallocScratchWords 32-bit words.  The
// largest bitmap of any schedule is 2^n1 x 2^(n - db) bits with n1 = 8,
// n - db = 13 (n = 16 at tile width 2^3, n = 17 at 2^4): 2^21 bits = 256 KiB.
constexpr uint64_t kNoallocScratchWords = (uint64_t)1 << 16;
// address of device `dev`'s copy of the array (looked up once per device,
// with that device current); hipSuccess or the lookup's error
hipError_t noalloc_scratch(int dev, uint32_t** out);

// launchers (tpd_kernels.hip)
hipError_t launch_sweep(Dtype dt, const SweepDesc& s, const SweepArgs& a, hipStream_t st);
bool sweep_supported(Dtype dt, const SweepDesc& s);
hipError_t launch_fill_u32(uint32_t* p, uint64_t words, uint32_t value, hipStream_t st);
hipError_t launch_batched_perm(Dtype dt, const void* const* in_ptrs, void* const* out_ptrs, const uint32_t* perm,
                               const BatchItem* items, uint32_t nitems, const BatchSeg* segs, uint32_t nseg, int layout,
                               int grid, hipStream_t st);
hipError_t launch_popcount(const uint32_t* p, uint64_t words, unsigned long long* out, hipStream_t st);

// selection kernels (tpd_select.hip)
hipError_t launch_mark_requests(const uint64_t* req, uint64_t count, int n, int n1, int db1, int db2, uint32_t* req_groups,
                                uint32_t* req_tiles, hipStream_t st);
hipError_t launch_and_u32(uint32_t* dst, const uint32_t* src, uint64_t words, hipStream_t st);
hipError_t launch_bits_to_list(const uint32_t* bits, uint64_t words, uint32_t* list, uint32_t* count,
                               hipStream_t st);
hipError_t launch_gather(Dtype dt, const void* coeffs, int n, bool matrix_layout, const uint64_t* req,
                         uint64_t count, void* values, hipStream_t st);
constexpr uint32_t kCompactChunk = 4096;  // elements per compaction workgroup (256 threads x 16)
hipError_t launch_compact_count(Dtype dt, const void* coeffs, uint64_t elems, double tol, uint32_t* counts,
                                hipStream_t st);
hipError_t launch_compact_scan(const uint32_t* counts, uint64_t nchunks, uint64_t* offsets, uint64_t* total,
                               hipStream_t st);
hipError_t launch_compact_write(Dtype dt, const void* coeffs, int n, bool matrix_layout, double tol,
                                const uint32_t* counts, const uint64_t* offsets, uint64_t capacity,
                                uint64_t* q_out, void* w_out, hipStream_t st);

// ---------------------------------------------------------------------------
// index maps shared by the selection kernels and their host replay
// ---------------------------------------------------------------------------
// even bits of q packed (the low bits of the Pauli digits: the column index)
__host__ __device__ inline uint64_t pack_even_bits(uint64_t q) {
  q &= 0x5555555555555555ull;
  q = (q | (q >> 1)) & 0x3333333333333333ull;
  q = (q | (q >> 2)) & 0x0F0F0F0F0F0F0F0Full;
  q = (q | (q >> 4)) & 0x00FF00FF00FF00FFull;
  q = (q | (q >> 8)) & 0x0000FFFF0000FFFFull;
  q = (q | (q >> 16)) & 0x00000000FFFFFFFFull;
  return q;
}
__host__ __device__ inline uint64_t spread_bits(uint64_t v) {
  v &= 0x00000000FFFFFFFFull;
  v = (v | (v << 16)) & 0x0000FFFF0000FFFFull;
  v = (v | (v << 8)) & 0x00FF00FF00FF00FFull;
  v = (v | (v << 4)) & 0x0F0F0F0F0F0F0F0Full;
  v = (v | (v << 2)) & 0x3333333333333333ull;
  v = (v | (v << 1)) & 0x5555555555555555ull;
  return v;
}
// canonical index q -> element offset in the canonical or matrix layout
// (matrix layout: row = hi bits of the digits, column = lo bits)
__host__ __device__ inline uint64_t storage_of_q(uint64_t q, int n, bool matrix_layout) {
  if (!matrix_layout) return q;
  return (pack_even_bits(q >> 1) << n) | pack_even_bits(q);
}
__host__ __device__ inline uint64_t q_of_storage(uint64_t a, int n, bool matrix_layout) {
  if (!matrix_layout) return a;
  const uint64_t lo = a & (((uint64_t)1 << n) - 1);
  return (spread_bits(a >> n) << 1) | spread_bits(lo);
}
// the two request bits of canonical string q in a two-sweep schedule: its
// first-sweep d-group (row ^ col) >> db1 and its second-sweep tile
// (((row ^ col) >> db2) << n1) | (row >> (n - n1)); db1 and db2 are the
// two sweeps' tile widths (they differ only for split widths)
__host__ __device__ inline void request_bits(uint64_t q, int n, int n1, int db1, int db2, uint64_t* group,
                                             uint64_t* tile) {
  const uint64_t row = pack_even_bits(q >> 1), col = pack_even_bits(q);
  *group = (row ^ col) >> db1;
  *tile = (((row ^ col) >> db2) << n1) | (row >> (n - n1));
}
// Hermitian first sweep: the tiles (fixed low x bits xf, d-group td) whose
// row block holds representatives, enumerated without gaps so that every
// workgroup of a persistent grid gets the same amount of work.  With
// L = n2 - db and dlh = td mod 2^L: a tile is needed when dlh = 0, or when xf
// has bit m = msb(dlh) + db clear.  t < 2^(n2-1+nfix_d): xf is t's high part
// with a zero inserted at bit m (dlh != 0) or with its top bit clear
// (dlh = 0); beyond: the dlh = 0 groups with xf's top bit set.
__host__ __device__ inline uint64_t herm_first_tiles(int n2, int db, int nfix_d) {
  return ((uint64_t)1 << (n2 - 1 + nfix_d)) + ((uint64_t)1 << (n2 - 1 + nfix_d - (n2 - db)));
}
__host__ __device__ inline void herm_first_tile(uint64_t t, int n2, int db, int nfix_d, uint64_t* xf, uint64_t* td) {
  const int L = n2 - db;
  const uint64_t part = (uint64_t)1 << (n2 - 1 + nfix_d);
  if (t < part) {
    const uint64_t xc = t >> nfix_d;
    const uint64_t d = t & (((uint64_t)1 << nfix_d) - 1);
    const uint64_t dlh = d & (((uint64_t)1 << L) - 1);
    *td = d;
    if (dlh) {
      const int m = 63 - __builtin_clzll(dlh) + db;
      *xf = ((xc >> m) << (m + 1)) | (xc & (((uint64_t)1 << m) - 1));
    } else {
      *xf = xc;
    }
  } else {
    const uint64_t u = t - part;
    const int hb = nfix_d - L;
    *td = (u & (((uint64_t)1 << hb) - 1)) << L;
    *xf = (u >> hb) | ((uint64_t)1 << (n2 - 1));
  }
}

// a coefficient is kept in the sparse list unless both parts are within tol
// (compared in the coefficient's own precision; NaN is kept)
template <class S>
__host__ __device__ inline bool keep_coeff(S re, S im, S tol) {
  const S ar = re < (S)0 ? -re : re;
  const S ai = im < (S)0 ? -im : im;
  return !(ar <= tol && ai <= tol);
}

// a sweep tile (plus its small bitmap scratch) must fit the LDS of one
// workgroup; gfx950 gives a workgroup up to 160 KiB, tiles use <= 128 KiB
template <class S>
constexpr bool shape_fits(int xb, int db) {
  return ((size_t)sizeof(typename Elem<S>::type) << (xb + db)) <= 131072;
}

// Batched tile geometry (shared with the host emulator and planner): the
// kernel has 2^(BT-4) threads and one LDS tile of 2^BT elements, 64 KiB for
// every dtype (complex128: BT = 12, the 8- and 4-byte dtypes: 13).  An item
// is 2^mb whole matrices (small n) or one d-group of 2^db XOR-diagonals of
// one matrix, of 2^(BT - v) elements, 2^(4 - v) per thread: variant v = 0
// fills the tile; v = 1 (n >= 3) holds half as much, i.e. half as many
// matrices per item or d-groups half as wide.  n = 0..2 pack whole matrices
// into each thread's registers (variant 0 only).
struct BatchGeom {
  int xb, db, mb, r;  // packed matrices per item = 2^mb, 2^r elements per thread
};
constexpr int batch_tile_bits(Dtype dt) { return dt == DT_C128 ? 12 : 13; }
constexpr BatchGeom batch_geom(int n, int bt, int v = 0) {
  if (n < 0 || n > 9 || v < 0 || v > 1 || (v == 1 && n < 3)) return BatchGeom{-1, -1, -1, -1};
  if (n == 0) return BatchGeom{0, 0, bt - 4, 0};
  if (n <= 2) return BatchGeom{n, n, bt - 4, n == 1 ? 2 : 4};
  const int ib = bt - v;  // item bits
  return 2 * n <= ib ? BatchGeom{n, n, ib - 2 * n, 4 - v} : BatchGeom{n, ib - n, 0, 4 - v};
}
template <int N, int BT, int V = 0>
struct BatchShape {
  static constexpr BatchGeom g = batch_geom(N, BT, V);
  using G = Geom<g.xb, g.db, g.mb, g.r, 0>;
  static_assert(g.xb >= 0, "no such batched geometry");
  static_assert(G::NT == (1 << (BT - 4)), "every batched item uses the whole workgroup");
};

}  // namespace tpd
