// tpd_shapes.cpp -- which sweep shapes the kernel instantiations cover
// (tpd_sweep_{c128,c64,r64,r32}*.hip).  Plain host C++: the planner asks
// here before it schedules a sweep, and the host emulator and host-only test
// builds link it without any device code.
#include "tpd_internal.h"

namespace tpd {

namespace {
// single-sweep shapes (n <= 8): all 2^n rows x 2^db diagonals
bool one_shape(int xb, int db) {
  static const int dbs[9] = {0, 1, 2, 3, 4, 5, 6, 5, 4};
  return xb >= 1 && xb <= 8 && db == dbs[xb];
}

template <class S>
bool supported(const SweepDesc& s, bool c128) {
  // complex128 tiles stop at 2^13 elements (8 levels of 2^5 diagonals, or
  // 2^4 for the inverse); the 8- and 4-byte elements reach 2^14 (n = 17's
  // 9-level sweeps)
  const int max_xb = c128 ? 8 : 9;
  // the separate real output (Hermitian weights): complex inputs, the matrix
  // layout in, the default phase order
  if (s.out_layout == L_CANR && (Elem<S>::real || s.inv || s.in_layout != L_MAT || s.order != 0)) return false;
  if (s.inv) {
    if (s.out_layout != L_MAT || (s.in_layout != L_CAN && s.in_layout != L_MAT)) return false;
    if (s.is_one) return one_shape(s.xb, s.db);
    const bool db_ok = c128 ? s.db == 4 : (s.db == 4 || s.db == 5);
    return s.xb >= 4 && s.xb <= max_xb && s.xb + s.db <= 14 && db_ok && s.r == 4 && s.order == 0 &&
           shape_fits<S>(s.xb, s.db);
  }
  if (s.is_one)
    return s.in_layout == L_MAT && s.xlo == 0 && s.out_layout != L_MID && s.bitmap_mode == 0 && one_shape(s.xb, s.db);
  if (s.r != 4) return false;
  const int db_lo = c128 ? 3 : 4, db_hi = c128 ? 5 : 6;
  if (s.xb < 4 || s.xb > max_xb || s.xb + s.db > 14 || s.db < db_lo || s.db > db_hi) return false;
  // the bottom-first phase order is instantiated for the default widths only
  if (s.order == 1 && (c128 ? s.db != 4 : (s.db != 4 && s.db != 5))) return false;
  return shape_fits<S>(s.xb, s.db);
}
}  // namespace

bool sweep_supported(Dtype dt, const SweepDesc& s) {
  switch (dt) {
    case DT_C128: return supported<double>(s, true);
    case DT_C64: return supported<float>(s, false);
    case DT_R64: return supported<Real<double>>(s, false);
    case DT_R32: return supported<Real<float>>(s, false);
    default: return false;
  }
}

}  // namespace tpd
