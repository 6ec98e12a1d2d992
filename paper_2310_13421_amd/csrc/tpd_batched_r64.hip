// tpd_batched_r64.hip -- the batched kernel's r64 instantiation (one
// translation unit per dtype, compiled in parallel).
#include "tpd_batched.h"

namespace tpd {
hipError_t launch_batched_r64(const BatchArgs& a, int grid, hipStream_t st) {
  return batched_launch<Real<double>, batch_tile_bits(DT_R64)>(a, grid, st);
}
}  // namespace tpd
