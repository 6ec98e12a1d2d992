// Host-only stand-ins for the device launchers of libtpd (the HIP kernels
// are not built into the sanitizer test binary).  The host replays under
// test never launch anything; every stand-in reports an error if reached.
#include "tpd_internal.h"

namespace tpd {
hipError_t launch_sweep(Dtype, const SweepDesc&, const SweepArgs&, hipStream_t) { return hipErrorNoDevice; }
hipError_t launch_fill_u32(uint32_t*, uint64_t, uint32_t, hipStream_t) { return hipErrorNoDevice; }
hipError_t launch_fill_noise(void*, uint64_t, bool, uint64_t, hipStream_t) { return hipErrorNoDevice; }
hipError_t launch_batched_perm(Dtype, const void* const*, void* const*, const uint32_t*, const BatchItem*, uint32_t,
                               const BatchSeg*, uint32_t, int, int, hipStream_t) {
  return hipErrorNoDevice;
}
hipError_t launch_popcount(const uint32_t*, uint64_t, unsigned long long*, hipStream_t) { return hipErrorNoDevice; }
hipError_t launch_mark_requests(const uint64_t*, uint64_t, int, int, int, int, uint32_t*, uint32_t*, hipStream_t) {
  return hipErrorNoDevice;
}
hipError_t launch_and_u32(uint32_t*, const uint32_t*, uint64_t, hipStream_t) { return hipErrorNoDevice; }
hipError_t launch_bits_to_list(const uint32_t*, uint64_t, uint32_t*, uint32_t*, hipStream_t) {
  return hipErrorNoDevice;
}
hipError_t launch_gather(Dtype, const void*, int, bool, const uint64_t*, uint64_t, void*, hipStream_t) {
  return hipErrorNoDevice;
}
hipError_t launch_compact_count(Dtype, const void*, uint64_t, double, uint32_t*, hipStream_t) {
  return hipErrorNoDevice;
}
hipError_t launch_compact_scan(const uint32_t*, uint64_t, uint64_t*, uint64_t*, hipStream_t) {
  return hipErrorNoDevice;
}
hipError_t launch_compact_write(Dtype, const void*, int, bool, double, const uint32_t*, const uint64_t*, uint64_t,
                                uint64_t*, void*, hipStream_t) {
  return hipErrorNoDevice;
}
hipError_t noalloc_scratch(int, uint32_t**) { return hipErrorNoDevice; }
}  // namespace tpd
