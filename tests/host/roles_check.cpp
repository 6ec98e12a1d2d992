// Host check of the sweep kernel's compile-time register/lane/wave roles
// (tpd_core.h): every phase maps (thread, slot) onto the tile bijectively,
// the last phase puts d bit b on lane bit b for b < min(DB, 6) (the pruning
// epilogue ORs over those lanes), and in 8-level tiles the last phase's
// slots hold rows that differ only in their low 5 bits (the epilogue's
// one-word-per-lane-group form relies on it).  Prints one line per geometry
// and exits nonzero on any violation.
#include <cstdint>
#include <cstdio>
#include <vector>

#include "tpd_core.h"

using namespace tpd;

template <class G>
int check(const char* name, bool want_rows_in_word) {
  constexpr Roles RL = make_roles<G>();
  int bad = 0;
  for (int p = 0; p < G::NPH; ++p) {
    std::vector<int> seen(1u << G::B, 0);
    for (uint32_t t = 0; t < (uint32_t)G::NT; ++t)
      for (int j = 0; j < G::E; ++j) {
        const uint32_t e = elem_base<G>(RL, p, t) | elem_reg<G>(RL, p, j);
        if (e >= (1u << G::B) || (elem_base<G>(RL, p, t) & elem_reg<G>(RL, p, j))) {
          ++bad;
          continue;
        }
        seen[e]++;
      }
    for (int c : seen)
      if (c != 1) ++bad;
  }
  const int last = G::NPH - 1;
  for (int b = 0; b < G::DB && b < 6; ++b)
    if (RL.lane[last][b] != b) ++bad;
  uint32_t rows = 0;
  for (int j = 0; j < G::E; ++j) rows |= (elem_reg<G>(RL, last, j) >> G::DB) & ((1u << G::XB) - 1);
  if (want_rows_in_word && rows >= 32) ++bad;
  std::printf("%s NT=%d slot_rows=0x%x bad=%d\n", name, G::NT, rows, bad);
  return bad;
}

int main() {
  int bad = 0;
  bad += check<Geom<8, 3, 0, 4, 0>>("XB8_DB3", true);
  bad += check<Geom<8, 4, 0, 4, 0>>("XB8_DB4", true);
  bad += check<Geom<8, 5, 0, 4, 0>>("XB8_DB5", true);
  bad += check<Geom<8, 6, 0, 4, 0>>("XB8_DB6", true);
  bad += check<Geom<7, 3, 0, 4, 0>>("XB7_DB3", false);
  bad += check<Geom<7, 6, 0, 4, 0>>("XB7_DB6", false);
  bad += check<Geom<9, 5, 0, 4, 0>>("XB9_DB5", false);
  bad += check<Geom<6, 5, 0, 4, 0>>("XB6_DB5", false);
  bad += check<Geom<5, 5, 0, 4, 0>>("XB5_DB5", false);
  return bad ? 1 : 0;
}
