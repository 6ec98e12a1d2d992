// tpd_sweep_c128.hip -- complex128 instantiations of the sweep kernel.
// Two-sweep tile widths: 2^3, 2^4 (default) or 2^5 diagonals (128, 256 or
// 512 B runs).
#include "tpd_sweep.h"

namespace tpd {

// two-sweep instantiations, one translation unit per tile width
hipError_t launch_two_c128_db3(const SweepDesc& s, const SweepArgs& a, hipStream_t st);
hipError_t launch_two_c128_db4(const SweepDesc& s, const SweepArgs& a, hipStream_t st);
hipError_t launch_two_c128_db5(const SweepDesc& s, const SweepArgs& a, hipStream_t st);

hipError_t launch_sweep_c128(const SweepDesc& s, const SweepArgs& a, hipStream_t st) {
  if (s.inv) return dispatch_inv<double>(s, a, st);
  if (s.is_one) return dispatch_one<double>(s, a, st);
  switch (s.db) {
    case 3: return launch_two_c128_db3(s, a, st);
    case 4: return launch_two_c128_db4(s, a, st);
    case 5: return launch_two_c128_db5(s, a, st);
  }
  return hipErrorInvalidValue;
}

}  // namespace tpd
