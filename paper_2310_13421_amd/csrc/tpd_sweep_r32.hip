// tpd_sweep_r32.hip -- real-input float32 instantiations of the sweep kernel
// (4-byte real-coded elements).
// Two-sweep tile widths: 2^4, 2^5 or 2^6 (default) diagonals (64, 128 or
// 256 B runs); the inverse transform with 2^4 or 2^5.
#include "tpd_sweep.h"

namespace tpd {

hipError_t launch_two_r32_db4(const SweepDesc& s, const SweepArgs& a, hipStream_t st);
hipError_t launch_two_r32_db5(const SweepDesc& s, const SweepArgs& a, hipStream_t st);
hipError_t launch_two_r32_db6(const SweepDesc& s, const SweepArgs& a, hipStream_t st);

hipError_t launch_sweep_r32(const SweepDesc& s, const SweepArgs& a, hipStream_t st) {
  if (s.inv) return dispatch_inv<Real<float>>(s, a, st);
  if (s.is_one) return dispatch_one<Real<float>>(s, a, st);
  switch (s.db) {
    case 4: return launch_two_r32_db4(s, a, st);
    case 5: return launch_two_r32_db5(s, a, st);
    case 6: return launch_two_r32_db6(s, a, st);
  }
  return hipErrorInvalidValue;
}

}  // namespace tpd
