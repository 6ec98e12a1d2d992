// tpd_sweep_r32_db5.hip -- two-sweep instantiations of the real-input
// (float32, real-coded) sweep kernel with tiles 2^5 XOR-diagonals wide
// (split out to compile in parallel).
#include "tpd_sweep.h"

namespace tpd {
hipError_t launch_two_r32_db5(const SweepDesc& s, const SweepArgs& a, hipStream_t st) {
  return dispatch_two_xb<Real<float>, 5>(s, a, st);
}
}  // namespace tpd
