// tpd_sweep_r32_db4.hip -- two-sweep instantiations of the real-input
// (float32, real-coded) sweep kernel with tiles 2^4 XOR-diagonals wide
// (split out to compile in parallel).
#include "tpd_sweep.h"

namespace tpd {
hipError_t launch_two_r32_db4(const SweepDesc& s, const SweepArgs& a, hipStream_t st) {
  return dispatch_two_xb<Real<float>, 4>(s, a, st);
}
}  // namespace tpd
