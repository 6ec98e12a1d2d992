// tpd_batched_r32.hip -- the batched kernel's r32 instantiation (one
// translation unit per dtype, compiled in parallel).
#include "tpd_batched.h"

namespace tpd {
hipError_t launch_batched_r32(const BatchArgs& a, int grid, hipStream_t st) {
  return batched_launch<Real<float>, batch_tile_bits(DT_R32)>(a, grid, st);
}
}  // namespace tpd
