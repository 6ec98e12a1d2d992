// tpd_batched_c64.hip -- the batched kernel's c64 instantiation (one
// translation unit per dtype, compiled in parallel).
#include "tpd_batched.h"

namespace tpd {
hipError_t launch_batched_c64(const BatchArgs& a, int grid, hipStream_t st) {
  return batched_launch<float, batch_tile_bits(DT_C64)>(a, grid, st);
}
}  // namespace tpd
