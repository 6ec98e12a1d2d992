// tpd_sweep_r32.hip -- real-input float32 instantiations of the sweep kernel
// (4-byte real-coded elements).
// Two-sweep tile widths: 2^4, 2^5 or 2^6 (default) diagonals (64, 128 or
// 256 B runs); the inverse transform with 2^4 or 2^5.
#include "tpd_sweep.h"

namespace tpd {

hipError_t launch_two_r32_db4(const SweepDesc& s, const SweepArgs& a, hipStream_t st);
hipError_t launch_two_r32_db5(const SweepDesc& s, const SweepArgs& a, hipStream_t st);
hipError_t launch_two_r32_db6(const SweepDesc& s, const SweepArgs& a, hipStream_t st);

bool sweep_supported_r32(const SweepDesc& s) {
  if (s.inv) {
    if (s.out_layout != L_MAT || (s.in_layout != L_CAN && s.in_layout != L_MAT)) return false;
    if (s.is_one)
      return (s.xb == 1 && s.db == 1) || (s.xb == 2 && s.db == 2) || (s.xb == 3 && s.db == 3) ||
             (s.xb == 4 && s.db == 4) || (s.xb == 5 && s.db == 5) || (s.xb == 6 && s.db == 6) ||
             (s.xb == 7 && s.db == 5) || (s.xb == 8 && s.db == 4);
    return s.xb >= 4 && s.xb <= 9 && s.xb + s.db <= 14 && (s.db == 4 || s.db == 5) && s.r == 4 && s.order == 0 &&
           shape_fits<Real<float>>(s.xb, s.db);
  }
  const bool one = s.in_layout == L_MAT && s.xlo == 0 && s.out_layout != L_MID && s.bitmap_mode == 0 &&
                   ((s.xb == 1 && s.db == 1) || (s.xb == 2 && s.db == 2) || (s.xb == 3 && s.db == 3) ||
                    (s.xb == 4 && s.db == 4) || (s.xb == 5 && s.db == 5) || (s.xb == 6 && s.db == 6) ||
                    (s.xb == 7 && s.db == 5) || (s.xb == 8 && s.db == 4));
  if (s.is_one) return one;
  if (s.r != 4) return false;
  if (s.xb < 4 || s.xb > 9 || s.xb + s.db > 14 || s.db < 4 || s.db > 6) return false;
  if (s.order == 1 && s.db != 4 && s.db != 5) return false;
  return shape_fits<Real<float>>(s.xb, s.db);
}

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
