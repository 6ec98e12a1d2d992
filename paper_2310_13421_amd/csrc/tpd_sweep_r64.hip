// tpd_sweep_r64.hip -- real-input float64 instantiations of the sweep kernel
// (8-byte real-coded elements: the same tile shapes as complex64).
// Two-sweep tile widths: 2^4, 2^5 (default) or 2^6 diagonals (128, 256 or
// 512 B runs); the inverse transform with 2^4 or 2^5.
#include "tpd_sweep.h"

namespace tpd {

hipError_t launch_two_r64_db4(const SweepDesc& s, const SweepArgs& a, hipStream_t st);
hipError_t launch_two_r64_db5(const SweepDesc& s, const SweepArgs& a, hipStream_t st);
hipError_t launch_two_r64_db6(const SweepDesc& s, const SweepArgs& a, hipStream_t st);

hipError_t launch_sweep_r64(const SweepDesc& s, const SweepArgs& a, hipStream_t st) {
  if (s.inv) return dispatch_inv<Real<double>>(s, a, st);
  if (s.is_one) return dispatch_one<Real<double>>(s, a, st);
  switch (s.db) {
    case 4: return launch_two_r64_db4(s, a, st);
    case 5: return launch_two_r64_db5(s, a, st);
    case 6: return launch_two_r64_db6(s, a, st);
  }
  return hipErrorInvalidValue;
}

}  // namespace tpd
