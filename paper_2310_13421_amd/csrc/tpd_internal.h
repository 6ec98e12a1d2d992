// tpd_internal.h -- declarations shared by the kernel launchers and the C ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "tpd_core.h"

namespace tpd {

enum Dtype : int { DT_C128 = 0, DT_C64 = 1 };

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
  int herm;          // 1: Hermitian input, two-sweep schedule
  uint64_t ntiles;
};

// Batched work item: `nmat` matrices of the same n starting at `mat0`
// (packed whole matrices), or one d-group tile of one matrix.
struct BatchItem {
  uint32_t mat0;
  uint16_t n;
  uint16_t nmat;
  uint32_t tile;
  uint32_t pad;
};

struct BatchArgs {
  const void* const* in_ptrs;   // device array of device pointers (caller's order)
  void* const* out_ptrs;        // device array of device pointers (may equal in_ptrs)
  const uint32_t* perm;         // device array: sorted position -> caller's index
  const BatchItem* items;       // device array
  uint32_t nitems;
  int layout;                   // L_CAN or L_MAT output
};

// launchers (tpd_kernels.hip)
hipError_t launch_sweep(Dtype dt, const SweepDesc& s, const SweepArgs& a, hipStream_t st);
bool sweep_supported(Dtype dt, const SweepDesc& s);
hipError_t launch_fill_u32(uint32_t* p, uint64_t words, uint32_t value, hipStream_t st);
hipError_t launch_batched_perm(Dtype dt, const void* const* in_ptrs, void* const* out_ptrs, const uint32_t* perm,
                               const BatchItem* items, uint32_t nitems, int layout, int grid, hipStream_t st);
hipError_t launch_popcount(const uint32_t* p, uint64_t words, unsigned long long* out, hipStream_t st);

// a sweep tile (plus its small bitmap scratch) must fit the LDS of one
// workgroup; gfx950 gives a workgroup up to 160 KiB, tiles use <= 128 KiB
template <class S>
constexpr bool shape_fits(int xb, int db) {
  return ((size_t)sizeof(Cx<S>) << (xb + db)) <= 131072;
}

// batched tile geometry per n (shared with the host emulator and planner)
struct BatchGeom {
  int xb, db, mb, r;  // packed matrices per item = 2^mb
};
BatchGeom batch_geom(int n);

}  // namespace tpd
