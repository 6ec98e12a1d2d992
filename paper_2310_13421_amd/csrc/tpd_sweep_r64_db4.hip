// tpd_sweep_r64_db4.hip -- two-sweep instantiations of the real-input
// (float64, real-coded) sweep kernel with tiles 2^4 XOR-diagonals wide
// (split out to compile in parallel).
#include "tpd_sweep.h"

namespace tpd {
hipError_t launch_two_r64_db4(const SweepDesc& s, const SweepArgs& a, hipStream_t st) {
  return dispatch_two_xb<Real<double>, 4>(s, a, st);
}
}  // namespace tpd
