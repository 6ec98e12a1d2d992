// tpd_batched_c128.hip -- the batched kernel's c128 instantiation (one
// translation unit per dtype, compiled in parallel).
#include "tpd_batched.h"

namespace tpd {
hipError_t launch_batched_c128(const BatchArgs& a, int grid, hipStream_t st) {
  return batched_launch<double, batch_tile_bits(DT_C128)>(a, grid, st);
}
}  // namespace tpd
