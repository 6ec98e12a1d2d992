// tpd_sweep_c128_db3.hip -- two-sweep instantiations of the complex128 sweep
// kernel with tiles 2^3 XOR-diagonals wide (split out to compile in parallel).
#include "tpd_sweep.h"

namespace tpd {
hipError_t launch_two_c128_db3(const SweepDesc& s, const SweepArgs& a, hipStream_t st) {
  return dispatch_two_xb<double, 3>(s, a, st);
}
}  // namespace tpd
