// tpd_sweep_c64.hip -- complex64 instantiations of the sweep kernel.
// Two-sweep tile widths: 2^4, 2^5 (default) or 2^6 diagonals (128, 256 or
// 512 B runs).
#include "tpd_sweep.h"

namespace tpd {

// two-sweep instantiations, one translation unit per tile width
hipError_t launch_two_c64_db4(const SweepDesc& s, const SweepArgs& a, hipStream_t st);
hipError_t launch_two_c64_db5(const SweepDesc& s, const SweepArgs& a, hipStream_t st);
hipError_t launch_two_c64_db6(const SweepDesc& s, const SweepArgs& a, hipStream_t st);

hipError_t launch_sweep_c64(const SweepDesc& s, const SweepArgs& a, hipStream_t st) {
  if (s.inv) return dispatch_inv<float>(s, a, st);
  if (s.is_one) return dispatch_one<float>(s, a, st);
  switch (s.db) {
    case 4: return launch_two_c64_db4(s, a, st);
    case 5: return launch_two_c64_db5(s, a, st);
    case 6: return launch_two_c64_db6(s, a, st);
  }
  return hipErrorInvalidValue;
}

}  // namespace tpd
