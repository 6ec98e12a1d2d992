// tpd_emulate.cpp -- sequential host replay of the device schedule.
//
// Executes, thread by thread and phase by phase, exactly what the kernels in
// tpd_kernels.hip execute (same tile decode, thread roles, address maps,
// LDS exchanges, butterflies and pruning-bitmap reduction), and checks on
// the way that every address is in range, that every sweep reads and
// writes each element exactly once, and that in-place tiles write only the
// addresses they read.  It lets the CPU test-suite exercise the index
// algebra before any GPU run.  The library never calls it to produce
// results.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "../../include/tpd.h"
#include "tpd_internal.h"

using namespace tpd;

// A build with TPD_EMULATE_COMPLEX128_ONLY (the host-only sanitizer test
// build, where compile time grows with every instantiation) replays the
// complex128 schedules only; complex64 requests return TPD_ERROR_UNSUPPORTED.
#ifdef TPD_EMULATE_COMPLEX128_ONLY
#define TPD_IF_C64(...) TPD_ERROR_UNSUPPORTED
#else
#define TPD_IF_C64(...) __VA_ARGS__
#endif

namespace {

struct Checker {
  uint64_t count;
  std::vector<uint8_t> reads, writes;
  bool ok = true;
  // second-sweep tiles skipped by the bitmap must hold zeros; with partial
  // requests only the requested tiles that are not live (null: no
  // restriction; zero_check false: no tile)
  const uint32_t* live = nullptr;
  const uint32_t* requested = nullptr;
  bool zero_check = true;
  // chunked order: the chunk that first touched each element of the
  // output buffer (and, in place, of the input), -1 = none; a touch by
  // another chunk fails, so chunks are disjoint and the pipelined streams
  // may interleave their launches in any order their events allow
  int32_t* own_rd = nullptr;
  int32_t* own_wr = nullptr;
  int32_t tag = 0;
  static bool bit(const uint32_t* m, uint64_t b) { return (m[b >> 5] >> (b & 31)) & 1u; }
  explicit Checker(uint64_t c) : count(c), reads(c, 0), writes(c, 0) {}
  void own(int32_t* o, uint64_t a) {
    if (!o) return;
    if (o[a] < 0) o[a] = tag;
    else if (o[a] != tag) ok = false;
  }
  void rd(uint64_t a) {
    if (a >= count) { ok = false; return; }
    if (reads[a]++) ok = false;
    own(own_rd, a);
  }
  void wr(uint64_t a) {
    if (a >= count) { ok = false; return; }
    if (writes[a]++) ok = false;
    own(own_wr, a);
  }
  bool complete() const {
    for (uint64_t i = 0; i < count; ++i)
      if (reads[i] != 1 || writes[i] != 1) return false;
    return true;
  }
};

template <class S, class G, int INL, int OUTL, bool INV = false>
tpd_status_t emulate_sweep(const Cx<S>* in, Cx<S>* out, const SweepArgs& a, uint32_t* bitmap, Checker& ck) {
  constexpr Roles RL = make_roles<G>();
  constexpr int P = G::NPH;
  constexpr int LAST = P - 1;
  constexpr uint32_t DM = (1u << G::DB) - 1;
  constexpr uint32_t XM = (1u << G::XB) - 1;
  constexpr int NBW = (1 << G::XB) >= 32 ? (1 << G::XB) / 32 : 1;
  const int n = a.n, xlo = a.xlo, db = a.db;
  const uint64_t tdmask = ((uint64_t)1 << a.nfix_d) - 1;
  const int tdb = a.chunk_bits > 0 ? a.chunk_bits : a.nfix_d;  // d-group bits of the tile index
  const bool in_place = (const void*)in == (const void*)out;
  std::vector<Cx<S>> v((size_t)G::NT * G::E), lds((size_t)1 << G::B);
  std::vector<uint64_t> rset, wset;
  uint32_t bits[NBW];

  // Hermitian first sweep: the enumeration covers exactly the tiles with
  // representatives; the others are accounted here (nothing is read or
  // written there), so the completeness check also proves the enumeration
  // is a bijection onto the needed tiles
  if (a.herm && xlo) {
    const uint64_t all = ((uint64_t)1 << xlo) << a.nfix_d;
    for (uint64_t tile = 0; tile < all; ++tile) {
      const uint64_t td = tile & tdmask;
      const uint64_t xf = tile >> a.nfix_d;
      const uint64_t dlh = td & (((uint64_t)1 << (xlo - G::DB)) - 1);
      const uint64_t hm = dlh ? (uint64_t)1 << (63 - __builtin_clzll(dlh) + G::DB) : 0;
      if (!(xf & hm)) continue;
      const uint64_t xfix = (xf & (((uint64_t)1 << xlo) - 1)) | ((xf >> xlo) << (xlo + G::XB));
      for (uint32_t tid = 0; tid < (uint32_t)G::NT; ++tid) {
        const uint32_t eb = elem_base<G>(RL, 0, tid);
        for (int j = 0; j < G::E; ++j) {
          const uint32_t e = eb | elem_reg<G>(RL, 0, j);
          const uint64_t x = xfix | ((uint64_t)((e >> G::DB) & XM) << xlo);
          const uint64_t d = (td << G::DB) | (e & DM);
          ck.rd(layout_addr<INL>(x, d, n, db));
          ck.wr(layout_addr<OUTL>(x, d, n, db));
        }
      }
    }
  }
  // work lists (partial decomposition): the listed tiles are processed; the
  // others are accounted after the loop (nothing is read or written there)
  const uint64_t lcount = a.list ? (uint64_t)a.list_count[0] : 0;
  const uint64_t ntiles = a.list ? lcount << a.list_shift : a.ntiles;
  const uint64_t xfbits = (uint64_t)(n - G::XB);
  std::vector<uint8_t> listed(a.list ? ((size_t)1 << (xfbits + a.nfix_d)) : 0, 0);
  for (uint64_t tile = 0; tile < ntiles; ++tile) {
    uint64_t td, xf;
    if (a.list && a.list_shift) {
      xf = tile / lcount;
      td = a.list[tile - xf * lcount];
    } else if (a.list) {
      const uint64_t lt = a.list[tile];
      td = lt >> a.bm_xbits;
      xf = lt & (((uint64_t)1 << a.bm_xbits) - 1);
    } else if (a.herm && xlo) {
      herm_first_tile(tile, xlo, G::DB, a.nfix_d, &xf, &td);
    } else {
      td = a.td_base + (tile & (((uint64_t)1 << tdb) - 1));
      xf = tile >> tdb;
    }
    if (a.list) {
      if (td > tdmask || xf >= ((uint64_t)1 << xfbits)) return TPD_ERROR_INTERNAL;
      if (listed[(xf << a.nfix_d) | td]++) return TPD_ERROR_INTERNAL;  // listed twice
    }
    const uint64_t xfix = (xf & (((uint64_t)1 << xlo) - 1)) | ((xf >> xlo) << (xlo + G::XB));
    if (a.req && !((a.req[td >> 5] >> (td & 31)) & 1u)) {
      // d-group without requested strings: nothing is read or written
      // (account its addresses so completeness still checks)
      for (uint32_t tid = 0; tid < (uint32_t)G::NT; ++tid) {
        const uint32_t eb = elem_base<G>(RL, 0, tid);
        for (int j = 0; j < G::E; ++j) {
          const uint32_t e = eb | elem_reg<G>(RL, 0, j);
          const uint64_t x = xfix | ((uint64_t)((e >> G::DB) & XM) << xlo);
          const uint64_t d = (td << G::DB) | (e & DM);
          ck.rd(layout_addr<INL>(x, d, n, db));
          ck.wr(layout_addr<OUTL>(x, d, n, db));
        }
      }
      continue;
    }
    if (a.bitmap_mode == 2) {
      const uint64_t bit = (td << a.bm_xbits) | xf;
      if (!((bitmap[bit >> 5] >> (bit & 31)) & 1u)) {
        // skipped tile: account its addresses as read and written in place
        const bool must_be_zero = ck.zero_check && (!ck.requested || Checker::bit(ck.requested, bit)) &&
                                  (!ck.live || !Checker::bit(ck.live, bit));
        // Hermitian second sweep: rows that are not representatives were
        // never written by the first sweep and are not read
        uint64_t hskip = 0;
        if (a.herm && !xlo) {
          constexpr int kLh = G::XB > G::DB ? G::XB - G::DB : 0;
          const uint64_t dlh = td & (((uint64_t)1 << kLh) - 1);
          if (dlh) hskip = (uint64_t)1 << (63 - __builtin_clzll(dlh) + G::DB);
        }
        for (uint32_t tid = 0; tid < (uint32_t)G::NT; ++tid) {
          const uint32_t eb = elem_base<G>(RL, 0, tid);
          for (int j = 0; j < G::E; ++j) {
            const uint32_t e = eb | elem_reg<G>(RL, 0, j);
            const uint64_t x = xfix | ((uint64_t)((e >> G::DB) & XM) << xlo);
            const uint64_t d = (td << G::DB) | (e & DM);
            const uint64_t ai = layout_addr<INL>(x, d, n, db);
            const uint64_t ao = layout_addr<OUTL>(x, d, n, db);
            ck.rd(ai);
            ck.wr(ao);
            const bool mirrored = (((uint64_t)((e >> G::DB) & XM)) & hskip) != 0;
            if (must_be_zero && ai < ck.count && !mirrored) {
              const Cx<S> z = in[ai];
              if (z.re != (S)0 || z.im != (S)0) return TPD_ERROR_INTERNAL;  // bit must have been set
            }
            // the kernel stores zeros on the mirrored rows of a Hermitian
            // zero tile (the first sweep never wrote them), and on every
            // element of a separate real output
            if constexpr (OUTL == L_CANR) {
              if (ao < ck.count) ((S*)out)[ao] = (S)0;
            } else if (mirrored && ao < ck.count) {
              out[ao] = Cx<S>{(S)0, (S)0};
            }
          }
        }
        continue;
      }
    }
    uint64_t hm = 0;
    if (a.herm) {
      const int n2 = xlo ? xlo : G::XB;
      const uint64_t dlh = td & (((uint64_t)1 << (n2 - G::DB)) - 1);
      if (dlh) hm = (uint64_t)1 << (63 - __builtin_clzll(dlh) + G::DB);
      if (xlo && (xf & hm)) {
        // the enumeration must never produce a non-representative block
        return TPD_ERROR_INTERNAL;
      }
    }
    for (int w = 0; w < NBW; ++w) bits[w] = 0;
    rset.clear();
    wset.clear();
    for (uint32_t tid = 0; tid < (uint32_t)G::NT; ++tid) {
      const uint32_t eb0 = elem_base<G>(RL, 0, tid);
      const uint64_t x = xfix | ((uint64_t)((eb0 >> G::DB) & XM) << xlo);
      const uint64_t d = (td << G::DB) | (eb0 & DM);
      const uint64_t base = layout_addr<INL>(x, d, n, db);
      for (int j = 0; j < G::E; ++j) {
        uint64_t ad = base;
        for (int s = 0; s < G::R; ++s)
          if ((j >> s) & 1) {
            const uint32_t ei = 1u << RL.reg[0][s];
            ad ^= layout_addr<INL>((uint64_t)((ei >> G::DB) & XM) << xlo, ei & DM, n, db);
          }
        // the delta form must agree with the direct map of the element
        const uint32_t e = eb0 | elem_reg<G>(RL, 0, j);
        const uint64_t xd = xfix | ((uint64_t)((e >> G::DB) & XM) << xlo);
        const uint64_t dd = (td << G::DB) | (e & DM);
        if (ad != layout_addr<INL>(xd, dd, n, db)) return TPD_ERROR_INTERNAL;
        ck.rd(ad);
        if (ad >= ck.count) return TPD_ERROR_INTERNAL;
        rset.push_back(ad);
        if (hm && !xlo && (((uint64_t)((e >> G::DB) & XM)) & hm)) v[(size_t)tid * G::E + j] = Cx<S>{(S)0, (S)0};
        else v[(size_t)tid * G::E + j] = in[ad];
      }
    }
    if (hm && !xlo) {
      const uint64_t dlo_hi = (td << G::DB) & ((((uint64_t)1 << G::XB) - 1));
      std::vector<uint8_t> seen(lds.size(), 0);
      for (uint32_t tid = 0; tid < (uint32_t)G::NT; ++tid) {
        const uint32_t eb0 = elem_base<G>(RL, 0, tid);
        for (int j = 0; j < G::E; ++j) {
          const uint32_t e = eb0 | elem_reg<G>(RL, 0, j);
          if (((uint64_t)((e >> G::DB) & XM)) & hm) continue;
          const uint32_t dlo = (uint32_t)(dlo_hi | (e & DM));
          const uint32_t ep = e ^ (dlo << G::DB);
          if (seen[e]++ || seen[ep]++) return TPD_ERROR_INTERNAL;  // each slot filled exactly once
          const Cx<S> z = v[(size_t)tid * G::E + j];
          lds[e] = z;
          lds[ep] = Cx<S>{z.re, -z.im};
        }
      }
      for (size_t e = 0; e < seen.size(); ++e)
        if (seen[e] != 1) return TPD_ERROR_INTERNAL;
      for (uint32_t tid = 0; tid < (uint32_t)G::NT; ++tid) {
        const uint32_t eb0 = elem_base<G>(RL, 0, tid);
        for (int j = 0; j < G::E; ++j) v[(size_t)tid * G::E + j] = lds[eb0 | elem_reg<G>(RL, 0, j)];
      }
    }
    for (int p = 0; p < P; ++p) {
      for (uint32_t tid = 0; tid < (uint32_t)G::NT; ++tid) {
        const uint32_t ebp = elem_base<G>(RL, p, tid);
        phase_butterflies<G, S, INV>(RL, p, &v[(size_t)tid * G::E], (td << G::DB) | (ebp & DM), xlo);
      }
      if (p + 1 < P) {
        std::vector<uint8_t> seen(lds.size(), 0);
        for (uint32_t tid = 0; tid < (uint32_t)G::NT; ++tid) {
          const uint32_t ebp = elem_base<G>(RL, p, tid);
          for (int j = 0; j < G::E; ++j) {
            const uint32_t e = ebp | elem_reg<G>(RL, p, j);
            if (seen[e]++) return TPD_ERROR_INTERNAL;  // two threads own one element
            lds[e] = v[(size_t)tid * G::E + j];
          }
        }
        for (uint32_t tid = 0; tid < (uint32_t)G::NT; ++tid) {
          const uint32_t ebn = elem_base<G>(RL, p + 1, tid);
          for (int j = 0; j < G::E; ++j) v[(size_t)tid * G::E + j] = lds[ebn | elem_reg<G>(RL, p + 1, j)];
        }
      }
    }
    if (a.bitmap_mode == 1) {
      // mirror the wave ballot: lanes [0, DB) are the diagonals of a row block
      constexpr uint32_t gsz = 1u << G::DB;
      constexpr uint64_t gmask = gsz >= 64 ? ~0ull : ((1ull << gsz) - 1);
      for (uint32_t w0 = 0; w0 < (uint32_t)G::NT; w0 += 64) {
        for (int j = 0; j < G::E; ++j) {
          uint64_t m = 0;
          for (uint32_t lane = 0; lane < 64 && w0 + lane < (uint32_t)G::NT; ++lane) {
            const Cx<S>& z = v[(size_t)(w0 + lane) * G::E + j];
            if (z.re != (S)0 || z.im != (S)0) m |= 1ull << lane;
          }
          for (uint32_t lane = 0; lane < 64 && w0 + lane < (uint32_t)G::NT; ++lane) {
            if ((lane & (gsz - 1)) == 0 && ((m >> lane) & gmask)) {
              const uint32_t ebl = elem_base<G>(RL, LAST, w0 + lane);
              const uint32_t xl = ((ebl | elem_reg<G>(RL, LAST, j)) >> G::DB) & XM;
              bits[xl >> 5] |= 1u << (xl & 31);
            }
          }
        }
      }
      for (int t = 0; t < NBW; ++t)
        if (bits[t]) {
          const uint64_t b0 = (td << a.bm_xbits) + 32ull * t;
          bitmap[b0 >> 5] |= bits[t] << (b0 & 31);
        }
    }
    // canonical-order output: one more pass through LDS into the store mapping
    constexpr bool REMAP = (OUTL == L_CAN || OUTL == L_CANR) && RL.st_ok;
    if (REMAP) {
      std::vector<uint8_t> seen(lds.size(), 0);
      for (uint32_t tid = 0; tid < (uint32_t)G::NT; ++tid) {
        const uint32_t ebl = elem_base<G>(RL, LAST, tid);
        for (int j = 0; j < G::E; ++j) {
          const uint32_t e = ebl | elem_reg<G>(RL, LAST, j);
          if (seen[e]++) return TPD_ERROR_INTERNAL;
          lds[e] = v[(size_t)tid * G::E + j];
        }
      }
      std::vector<uint8_t> got(lds.size(), 0);
      for (uint32_t tid = 0; tid < (uint32_t)G::NT; ++tid) {
        const uint32_t ebs = elem_base_st<G>(RL, tid);
        for (int j = 0; j < G::E; ++j) {
          const uint32_t e = ebs | elem_reg_st<G>(RL, j);
          if (got[e]++) return TPD_ERROR_INTERNAL;  // the store mapping is a bijection
          v[(size_t)tid * G::E + j] = lds[e];
        }
      }
    }
    for (uint32_t tid = 0; tid < (uint32_t)G::NT; ++tid) {
      const uint32_t ebl = REMAP ? elem_base_st<G>(RL, tid) : elem_base<G>(RL, LAST, tid);
      const uint64_t x = xfix | ((uint64_t)((ebl >> G::DB) & XM) << xlo);
      const uint64_t d = (td << G::DB) | (ebl & DM);
      const uint64_t base = layout_addr<OUTL>(x, d, n, db);
      for (int j = 0; j < G::E; ++j) {
        uint64_t ad = base;
        for (int s = 0; s < G::R; ++s)
          if ((j >> s) & 1) {
            const uint32_t eo = 1u << (REMAP ? RL.st_reg[s] : RL.reg[LAST][s]);
            ad ^= layout_addr<OUTL>((uint64_t)((eo >> G::DB) & XM) << xlo, eo & DM, n, db);
          }
        const uint32_t e = ebl | (REMAP ? elem_reg_st<G>(RL, j) : elem_reg<G>(RL, LAST, j));
        if (REMAP && j == 0 && (tid & 63) == 0) {
          // a wave's store instruction covers 64 consecutive coefficients
          uint64_t lo = ~0ull, hi = 0;
          for (uint32_t l = 0; l < 64; ++l) {
            const uint32_t el = elem_base_st<G>(RL, tid + l) | elem_reg_st<G>(RL, 0);
            const uint64_t a2 = layout_addr<OUTL>(xfix | ((uint64_t)((el >> G::DB) & XM) << xlo),
                                                  (td << G::DB) | (el & DM), n, db);
            lo = a2 < lo ? a2 : lo;
            hi = a2 > hi ? a2 : hi;
          }
          if (hi - lo != 63) return TPD_ERROR_INTERNAL;
        }
        const uint64_t xd = xfix | ((uint64_t)((e >> G::DB) & XM) << xlo);
        const uint64_t dd = (td << G::DB) | (e & DM);
        if (ad != layout_addr<OUTL>(xd, dd, n, db)) return TPD_ERROR_INTERNAL;
        ck.wr(ad);
        if (ad >= ck.count) return TPD_ERROR_INTERNAL;
        wset.push_back(ad);
        if (a.herm && !xlo) v[(size_t)tid * G::E + j].im = (S)0;
        if constexpr (OUTL == L_CANR) ((S*)out)[ad] = v[(size_t)tid * G::E + j].re;
        else out[ad] = v[(size_t)tid * G::E + j];
      }
    }
    if (in_place) {
      std::sort(rset.begin(), rset.end());
      std::sort(wset.begin(), wset.end());
      if (rset != wset) return TPD_ERROR_INTERNAL;  // an in-place tile must be closed
    }
  }
  if (a.list) {
    for (uint64_t nt = 0; nt < listed.size(); ++nt) {
      if (listed[nt]) continue;
      const uint64_t td = nt & tdmask, xf = nt >> a.nfix_d;
      const uint64_t xfix = (xf & (((uint64_t)1 << xlo) - 1)) | ((xf >> xlo) << (xlo + G::XB));
      for (uint32_t tid = 0; tid < (uint32_t)G::NT; ++tid) {
        const uint32_t eb = elem_base<G>(RL, 0, tid);
        for (int j = 0; j < G::E; ++j) {
          const uint32_t e = eb | elem_reg<G>(RL, 0, j);
          const uint64_t x = xfix | ((uint64_t)((e >> G::DB) & XM) << xlo);
          const uint64_t d = (td << G::DB) | (e & DM);
          ck.rd(layout_addr<INL>(x, d, n, db));
          ck.wr(layout_addr<OUTL>(x, d, n, db));
        }
      }
    }
  }
  return ck.ok ? TPD_SUCCESS : TPD_ERROR_INTERNAL;
}

template <class S, int XB, int DB, int ORDER, int RR>
tpd_status_t emulate_layouts(const SweepDesc& s, const Cx<S>* in, Cx<S>* out, const SweepArgs& a, uint32_t* bm,
                             Checker& ck) {
  // same thread-count cap as the device launcher
  constexpr int R1 = (XB + DB - 10) > RR ? (XB + DB - 10) : RR;
  constexpr int R = (XB + DB) < R1 ? (XB + DB) : R1;
  using G = Geom<XB, DB, 0, R, ORDER>;
  if (s.inv) {
    if (s.in_layout == L_CAN && s.out_layout == L_MAT) return emulate_sweep<S, G, L_CAN, L_MAT, true>(in, out, a, bm, ck);
    if (s.in_layout == L_MAT && s.out_layout == L_MAT) return emulate_sweep<S, G, L_MAT, L_MAT, true>(in, out, a, bm, ck);
    return TPD_ERROR_INTERNAL;
  }
  if (s.in_layout == L_MAT && s.out_layout == L_CAN) return emulate_sweep<S, G, L_MAT, L_CAN>(in, out, a, bm, ck);
  if (s.in_layout == L_MAT && s.out_layout == L_MAT) return emulate_sweep<S, G, L_MAT, L_MAT>(in, out, a, bm, ck);
  if (s.in_layout == L_MAT && s.out_layout == L_MID) return emulate_sweep<S, G, L_MAT, L_MID>(in, out, a, bm, ck);
  if (s.in_layout == L_MID && s.out_layout == L_CAN) return emulate_sweep<S, G, L_MID, L_CAN>(in, out, a, bm, ck);
  if (s.in_layout == L_MAT && s.out_layout == L_CANR) return emulate_sweep<S, G, L_MAT, L_CANR>(in, out, a, bm, ck);
  return TPD_ERROR_INTERNAL;
}

template <class S, int XB, int DB>
tpd_status_t emulate_r(const SweepDesc& s, const Cx<S>* in, Cx<S>* out, const SweepArgs& a, uint32_t* bm,
                       Checker& ck) {
  if (s.order == 1) return emulate_layouts<S, XB, DB, 1, 4>(s, in, out, a, bm, ck);
  return emulate_layouts<S, XB, DB, 0, 4>(s, in, out, a, bm, ck);
}

template <class S, int DB>
tpd_status_t emulate_xb(const SweepDesc& s, const Cx<S>* in, Cx<S>* out, const SweepArgs& a, uint32_t* bm,
                        Checker& ck) {
  switch (s.xb) {
    case 4: return emulate_r<S, 4, DB>(s, in, out, a, bm, ck);
    case 5: return emulate_r<S, 5, DB>(s, in, out, a, bm, ck);
    case 6: return emulate_r<S, 6, DB>(s, in, out, a, bm, ck);
    case 7: return emulate_r<S, 7, DB>(s, in, out, a, bm, ck);
    case 8: return emulate_r<S, 8, DB>(s, in, out, a, bm, ck);
  }
  return TPD_ERROR_INTERNAL;
}

template <class S>
tpd_status_t emulate_shape(const SweepDesc& s, const Cx<S>* in, Cx<S>* out, const SweepArgs& a, uint32_t* bm,
                           Checker& ck) {
  if (s.is_one) {
#define TPD_CASE(XB_, DB_) \
    if (s.xb == XB_ && s.db == DB_) return emulate_layouts<S, XB_, DB_, 0, 4>(s, in, out, a, bm, ck);
    TPD_CASE(1, 1) TPD_CASE(2, 2) TPD_CASE(3, 3) TPD_CASE(4, 4) TPD_CASE(5, 5) TPD_CASE(6, 6) TPD_CASE(7, 5)
    TPD_CASE(8, 4)
#undef TPD_CASE
    return TPD_ERROR_INTERNAL;
  }
  switch (s.db) {
    case 3: return emulate_xb<S, 3>(s, in, out, a, bm, ck);
    case 4: return emulate_xb<S, 4>(s, in, out, a, bm, ck);
    case 5: return emulate_xb<S, 5>(s, in, out, a, bm, ck);
    case 6: return emulate_xb<S, 6>(s, in, out, a, bm, ck);
  }
  return TPD_ERROR_INTERNAL;
}

// ---- batched ----
template <class S, class G, int OUTL>
tpd_status_t emulate_item(const void* const* ptrs, void* const* outs, const uint32_t* perm, const BatchItem& it) {
  constexpr Roles RL = make_roles<G>();
  constexpr int P = G::NPH;
  constexpr int LAST = P - 1;
  constexpr uint32_t DM = (1u << G::DB) - 1;
  constexpr uint32_t XM = (1u << G::XB) - 1;
  const int n = it.n;
  const uint64_t td = it.tile;
  const uint64_t count = (uint64_t)1 << (2 * n);
  std::vector<Cx<S>> v((size_t)G::NT * G::E), lds((size_t)1 << G::B);
  for (uint32_t tid = 0; tid < (uint32_t)G::NT; ++tid) {
    const uint32_t e = elem_base<G>(RL, 0, tid);
    const uint32_t ml = e >> (G::DB + G::XB);
    for (int j = 0; j < G::E; ++j) {
      Cx<S> z{(S)0, (S)0};
      if (ml < it.nmat) {
        const Cx<S>* in = (const Cx<S>*)ptrs[perm[it.mat0 + ml]];
        const uint32_t ej = e | elem_reg<G>(RL, 0, j);
        const uint64_t ad = layout_addr<L_MAT>((ej >> G::DB) & XM, (td << G::DB) | (ej & DM), n, G::DB);
        if (ad >= count) return TPD_ERROR_INTERNAL;
        z = in[ad];
      }
      v[(size_t)tid * G::E + j] = z;
    }
  }
  for (int p = 0; p < P; ++p) {
    for (uint32_t tid = 0; tid < (uint32_t)G::NT; ++tid) {
      const uint32_t ebp = elem_base<G>(RL, p, tid);
      phase_butterflies<G, S>(RL, p, &v[(size_t)tid * G::E], (td << G::DB) | (ebp & DM), 0);
    }
    if (p + 1 < P) {
      for (uint32_t tid = 0; tid < (uint32_t)G::NT; ++tid) {
        const uint32_t ebp = elem_base<G>(RL, p, tid);
        for (int j = 0; j < G::E; ++j) lds[ebp | elem_reg<G>(RL, p, j)] = v[(size_t)tid * G::E + j];
      }
      for (uint32_t tid = 0; tid < (uint32_t)G::NT; ++tid) {
        const uint32_t ebn = elem_base<G>(RL, p + 1, tid);
        for (int j = 0; j < G::E; ++j) v[(size_t)tid * G::E + j] = lds[ebn | elem_reg<G>(RL, p + 1, j)];
      }
    }
  }
  for (uint32_t tid = 0; tid < (uint32_t)G::NT; ++tid) {
    const uint32_t e = elem_base<G>(RL, LAST, tid);
    const uint32_t ml = e >> (G::DB + G::XB);
    if (ml >= it.nmat) continue;
    Cx<S>* out = (Cx<S>*)outs[perm[it.mat0 + ml]];
    for (int j = 0; j < G::E; ++j) {
      const uint32_t ej = e | elem_reg<G>(RL, LAST, j);
      const uint64_t ad = layout_addr<OUTL>((ej >> G::DB) & XM, (td << G::DB) | (ej & DM), n, G::DB);
      if (ad >= count) return TPD_ERROR_INTERNAL;
      out[ad] = v[(size_t)tid * G::E + j];
    }
  }
  return TPD_SUCCESS;
}

template <class S, int OUTL, int N>
tpd_status_t emulate_item_v(const void* const* ptrs, void* const* outs, const uint32_t* perm, const BatchItem& it) {
  constexpr int BT = batch_tile_bits(sizeof(S) == 8 ? DT_C128 : DT_C64);
  if (it.variant == 0) return emulate_item<S, typename BatchShape<N, BT, 0>::G, OUTL>(ptrs, outs, perm, it);
  if constexpr (N >= 3)
    if (it.variant == 1) return emulate_item<S, typename BatchShape<N, BT, 1>::G, OUTL>(ptrs, outs, perm, it);
  return TPD_ERROR_INTERNAL;
}

template <class S, int OUTL>
tpd_status_t emulate_item_n(const void* const* ptrs, void* const* outs, const uint32_t* perm, const BatchItem& it) {
  switch (it.n) {
    case 0: return emulate_item_v<S, OUTL, 0>(ptrs, outs, perm, it);
    case 1: return emulate_item_v<S, OUTL, 1>(ptrs, outs, perm, it);
    case 2: return emulate_item_v<S, OUTL, 2>(ptrs, outs, perm, it);
    case 3: return emulate_item_v<S, OUTL, 3>(ptrs, outs, perm, it);
    case 4: return emulate_item_v<S, OUTL, 4>(ptrs, outs, perm, it);
    case 5: return emulate_item_v<S, OUTL, 5>(ptrs, outs, perm, it);
    case 6: return emulate_item_v<S, OUTL, 6>(ptrs, outs, perm, it);
    case 7: return emulate_item_v<S, OUTL, 7>(ptrs, outs, perm, it);
    case 8: return emulate_item_v<S, OUTL, 8>(ptrs, outs, perm, it);
    case 9: return emulate_item_v<S, OUTL, 9>(ptrs, outs, perm, it);
  }
  return TPD_ERROR_INTERNAL;
}

}  // namespace

namespace tpd {
// defined in tpd_api.cpp
tpd_status_t host_schedule(int n, int dtype, unsigned flags, bool in_place, const int* tune, SweepDesc* sw,
                           int* nsweep, int* n1, uint64_t* bitmap_words, int* chunk_bits, int* chunk_window);
tpd_status_t host_batch_tables(const int* ns, int count, bool in_place, unsigned flags, int dtype, const int* codes,
                               std::vector<uint32_t>* perm, std::vector<BatchItem>* items);
tpd_status_t host_synth_schedule(int n, int dtype, unsigned flags, bool in_place, SweepDesc* sw, int* nsweep);
tpd_status_t host_partial_schedule(int n, int dtype, unsigned flags, bool in_place, SweepDesc* sw, int* nsweep,
                                   int* n1, uint64_t* bitmap_words, int* prune);
tpd_status_t host_real_out_schedule(int n, int dtype, unsigned flags, SweepDesc* sw, int* nsweep, int* n1,
                                    uint64_t* bitmap_words, int* prune);
}  // namespace tpd

// Host replay of tpd_decompose_hermitian_real: the first sweep in place in
// A, the last from A into the real weights W (HOST pointers, small n).
extern "C" tpd_status_t tpd_debug_emulate_hermitian_real(void* A, int n, void* W, tpd_dtype_t dtype,
                                                         unsigned flags) {
  if (!A || !W) return TPD_ERROR_INVALID_VALUE;
  if (n < 0 || n > 12) return TPD_ERROR_UNSUPPORTED;
  SweepDesc sw[2];
  int nsweep = 0, n1 = 0, prune = 0;
  uint64_t words = 0;
  tpd_status_t st = host_real_out_schedule(n, dtype, flags, sw, &nsweep, &n1, &words, &prune);
  if (st) return st;
  const uint64_t count = (uint64_t)1 << (2 * n);
  if (n == 0) {
    if (dtype == TPD_C128) ((double*)W)[0] = ((const double*)A)[0];
    else ((float*)W)[0] = ((const float*)A)[0];
    return TPD_SUCCESS;
  }
  std::vector<uint32_t> bitmap(words ? words : 1, 0u);
  for (int i = 0; i < nsweep; ++i) {
    const bool last = i == nsweep - 1;
    SweepArgs a{};
    a.in = A;
    a.out = last ? W : A;
    a.n = n;
    a.xlo = sw[i].xlo;
    a.db = sw[i].db;
    a.nfix_d = n - sw[i].db;
    a.bitmap = bitmap.data();
    a.bitmap_mode = sw[i].bitmap_mode;
    a.bm_xbits = n1;
    a.herm = sw[i].herm;
    a.ntiles = sw[i].ntiles;
    Checker ck(count);
    if (dtype == TPD_C128)
      st = emulate_shape<double>(sw[i], (const Cx<double>*)a.in, (Cx<double>*)a.out, a, bitmap.data(), ck);
    else
      st = TPD_IF_C64(emulate_shape<float>(sw[i], (const Cx<float>*)a.in, (Cx<float>*)a.out, a, bitmap.data(), ck));
    if (st) return st;
    if (!ck.complete()) return TPD_ERROR_INTERNAL;
  }
  return TPD_SUCCESS;
}

extern "C" tpd_status_t tpd_debug_emulate_synth(const void* coeffs, int n, void* A, tpd_dtype_t dtype, unsigned flags,
                                                int in_place) {
  if (!coeffs || !A) return TPD_ERROR_INVALID_VALUE;
  if (n < 0 || n > 12) return TPD_ERROR_UNSUPPORTED;
  if (in_place && coeffs != A) return TPD_ERROR_INVALID_VALUE;
  SweepDesc sw[2];
  int nsweep = 0;
  tpd_status_t st = host_synth_schedule(n, dtype, flags, in_place != 0, sw, &nsweep);
  if (st) return st;
  const uint64_t count = (uint64_t)1 << (2 * n);
  const size_t eb = dtype == TPD_C128 ? 16 : 8;
  if (n == 0) {
    if (coeffs != A) std::memcpy(A, coeffs, eb);
    return TPD_SUCCESS;
  }
  for (int i = 0; i < nsweep; ++i) {
    SweepArgs a{};
    a.in = i == 0 ? coeffs : A;
    a.out = A;
    a.n = n;
    a.xlo = sw[i].xlo;
    a.db = sw[i].db;
    a.nfix_d = n - sw[i].db;
    a.bitmap = nullptr;
    a.bitmap_mode = 0;
    a.herm = 0;
    a.ntiles = sw[i].ntiles;
    Checker ck(count);
    if (dtype == TPD_C128)
      st = emulate_shape<double>(sw[i], (const Cx<double>*)a.in, (Cx<double>*)a.out, a, nullptr, ck);
    else
      st = TPD_IF_C64(emulate_shape<float>(sw[i], (const Cx<float>*)a.in, (Cx<float>*)a.out, a, nullptr, ck));
    if (st) return st;
    if (!ck.complete()) return TPD_ERROR_INTERNAL;
  }
  return TPD_SUCCESS;
}

extern "C" tpd_status_t tpd_debug_emulate_tuned(const void* A, int n, void* coeffs, tpd_dtype_t dtype,
                                                unsigned flags, int in_place, int db, int r, int chunk_bits,
                                                int chunk_window) {
  if (!A || !coeffs) return TPD_ERROR_INVALID_VALUE;
  if (n < 0 || n > 12) return TPD_ERROR_UNSUPPORTED;  // host replay is for small n
  if (in_place && A != coeffs) return TPD_ERROR_INVALID_VALUE;
  if (chunk_bits < 0 || (chunk_bits > 0 && db <= 0) || chunk_window < 0) return TPD_ERROR_INVALID_VALUE;
  SweepDesc sw[2];
  int nsweep = 0, n1 = 0, chunk = 0, window = 0;
  uint64_t words = 0;
  const int tune[5] = {db, r, 0, chunk_bits, chunk_window};
  tpd_status_t st = host_schedule(n, dtype, flags, in_place != 0, db > 0 ? tune : nullptr, sw, &nsweep, &n1, &words,
                                  &chunk, &window);
  if (st) return st;
  const uint64_t count = (uint64_t)1 << (2 * n);
  const size_t eb = dtype == TPD_C128 ? 16 : 8;
  if (n == 0) {
    if (A != coeffs) std::memcpy(coeffs, A, eb);
    return TPD_SUCCESS;
  }
  std::vector<uint32_t> bitmap(words ? words : 1, 0u);
  // chunked order: sweep 1 then sweep 2 per chunk of d-groups; each sweep's
  // checker accumulates over the chunks, so completeness covers the union.
  // Pipelined (window w): step k runs sweep 1 of chunk k, then sweep 2 of
  // chunk k - w + 1, the order in which the device streams' dependencies
  // let sweep 1 run furthest ahead.
  const uint64_t nchunks = (nsweep == 2 && chunk > 0) ? ((uint64_t)1 << (n - sw[0].db - chunk)) : 1;
  const uint64_t lag = window >= 2 ? (uint64_t)window - 1 : 0;
  Checker ck0(count), ck1(count);
  Checker* cks[2] = {&ck0, &ck1};
  std::vector<int32_t> own_out, own_in;
  if (nchunks > 1) {
    own_out.assign(count, -1);
    if (!in_place) own_in.assign(count, -1);
    ck0.own_rd = in_place ? own_out.data() : own_in.data();
    ck0.own_wr = own_out.data();
    ck1.own_rd = ck1.own_wr = own_out.data();
  }
  auto run = [&](int i, uint64_t c) -> tpd_status_t {
    SweepArgs a{};
    a.in = i == 0 ? A : coeffs;
    a.out = coeffs;
    a.n = n;
    a.xlo = sw[i].xlo;
    a.db = sw[i].db;
    a.nfix_d = n - sw[i].db;
    a.bitmap = bitmap.data();
    a.bitmap_mode = sw[i].bitmap_mode;
    a.bm_xbits = n1;
    a.herm = sw[i].herm;
    a.ntiles = sw[i].ntiles;
    if (nchunks > 1) {
      a.chunk_bits = chunk + sw[0].db - sw[i].db;
      a.td_base = c << a.chunk_bits;
      a.ntiles = ((uint64_t)1 << (n - sw[i].xb)) << a.chunk_bits;
      cks[i]->tag = (int32_t)c;
    }
    if (dtype == TPD_C128)
      return emulate_shape<double>(sw[i], (const Cx<double>*)a.in, (Cx<double>*)a.out, a, bitmap.data(), *cks[i]);
    return TPD_IF_C64(
        emulate_shape<float>(sw[i], (const Cx<float>*)a.in, (Cx<float>*)a.out, a, bitmap.data(), *cks[i]));
  };
  for (uint64_t k = 0; k < nchunks + lag; ++k) {
    if (k < nchunks) {
      st = run(0, k);
      if (st) return st;
    }
    if (nsweep == 2 && k >= lag) {
      st = run(1, k - lag);
      if (st) return st;
    }
  }
  for (int i = 0; i < nsweep; ++i)
    if (!cks[i]->complete()) return TPD_ERROR_INTERNAL;
  return TPD_SUCCESS;
}

extern "C" tpd_status_t tpd_debug_emulate(const void* A, int n, void* coeffs, tpd_dtype_t dtype, unsigned flags,
                                          int in_place) {
  return tpd_debug_emulate_tuned(A, n, coeffs, dtype, flags, in_place, 0, 0, 0, 0);
}

extern "C" tpd_status_t tpd_debug_emulate_batched(const void* const* ptrs, const int* ns, int count,
                                                  void* const* out_ptrs, tpd_dtype_t dtype, unsigned flags,
                                                  const int* codes) {
  if (count < 0) return TPD_ERROR_INVALID_VALUE;
  if (count == 0) return TPD_SUCCESS;
  if (!ptrs || !ns) return TPD_ERROR_INVALID_VALUE;
  if (dtype != TPD_C128 && dtype != TPD_C64) return TPD_ERROR_INVALID_VALUE;
  std::vector<uint32_t> perm;
  std::vector<BatchItem> items;
  tpd_status_t st = host_batch_tables(ns, count, out_ptrs == nullptr, flags, dtype, codes, &perm, &items);
  if (st) return st;
  void* const* outs = out_ptrs ? out_ptrs : (void* const*)ptrs;
  const bool mat = (flags & TPD_FLAG_LAYOUT_MATRIX) != 0;
  for (const BatchItem& it : items) {
    if (dtype == TPD_C128)
      st = mat ? emulate_item_n<double, L_MAT>(ptrs, outs, perm.data(), it)
               : emulate_item_n<double, L_CAN>(ptrs, outs, perm.data(), it);
    else
      st = TPD_IF_C64(mat ? emulate_item_n<float, L_MAT>(ptrs, outs, perm.data(), it)
                          : emulate_item_n<float, L_CAN>(ptrs, outs, perm.data(), it));
    if (st) return st;
  }
  return TPD_SUCCESS;
}

extern "C" tpd_status_t tpd_debug_emulate_partial(const void* A, int n, void* coeffs, const uint64_t* req,
                                                  uint64_t count, void* values, tpd_dtype_t dtype, unsigned flags,
                                                  int in_place) {
  if (!A || !coeffs || (count && (!req || !values))) return TPD_ERROR_INVALID_VALUE;
  if (n < 0 || n > 12) return TPD_ERROR_UNSUPPORTED;
  if (in_place && A != coeffs) return TPD_ERROR_INVALID_VALUE;
  SweepDesc sw[2];
  int nsweep = 0, n1 = 0, prune = 0;
  uint64_t words = 0;
  tpd_status_t st = host_partial_schedule(n, dtype, flags, in_place != 0, sw, &nsweep, &n1, &words, &prune);
  if (st) return st;
  const uint64_t elems = (uint64_t)1 << (2 * n);
  const size_t eb = dtype == TPD_C128 ? 16 : 8;
  const bool mat = (flags & TPD_FLAG_LAYOUT_MATRIX) != 0;
  if (n == 0) {
    if (A != coeffs) std::memcpy(coeffs, A, eb);
  } else if (nsweep == 1) {
    st = tpd_debug_emulate_tuned(A, n, coeffs, dtype, flags, in_place, 0, 0, 0, 0);
    if (st) return st;
  } else {
    const int db = sw[0].db;
    const uint64_t gw = (((uint64_t)1 << (n - db)) + 31) / 32;
    std::vector<uint32_t> groups(gw, 0u), tiles(words, 0u), live(words, 0u);
    for (uint64_t i = 0; i < count; ++i) {
      if (req[i] >= elems) continue;
      uint64_t g, t;
      request_bits(req[i], n, n1, db, sw[1].db, &g, &t);
      groups[g >> 5] |= 1u << (g & 31);
      tiles[t >> 5] |= 1u << (t & 31);
    }
    // work lists as the device builds them (the order does not matter)
    auto to_list = [](const std::vector<uint32_t>& bits, std::vector<uint32_t>* list) {
      list->clear();
      for (uint64_t w = 0; w < bits.size(); ++w)
        for (int b = 0; b < 32; ++b)
          if ((bits[w] >> b) & 1u) list->push_back((uint32_t)(w * 32 + b));
    };
    std::vector<uint32_t> glist, tlist;
    static const uint32_t kNone = 0;  // an empty list is still a list (never read)
    const bool group_list = !sw[0].herm;
    to_list(groups, &glist);
    for (int i = 0; i < 2; ++i) {
      SweepArgs a{};
      a.in = i == 0 ? A : coeffs;
      a.out = coeffs;
      a.n = n;
      a.xlo = sw[i].xlo;
      a.db = db;
      a.nfix_d = n - db;
      a.bm_xbits = n1;
      a.herm = sw[i].herm;
      a.ntiles = sw[i].ntiles;
      uint32_t lcount = 0;
      if (i == 0) {
        a.bitmap = live.data();
        a.bitmap_mode = sw[i].bitmap_mode;
        if (group_list) {
          lcount = (uint32_t)glist.size();
          a.list = glist.empty() ? &kNone : glist.data();
          a.list_count = &lcount;
          a.list_shift = sw[i].xlo;
        } else {
          a.req = groups.data();
        }
      } else {
        // Hermitian mode: requested zero tiles stay in the list, the kernel
        // stores their mirrored rows (the first sweep never wrote them)
        const bool herm_zero = prune && sw[i].herm;
        if (prune && !herm_zero)
          for (uint64_t w = 0; w < words; ++w) tiles[w] &= live[w];
        to_list(tiles, &tlist);
        lcount = (uint32_t)tlist.size();
        a.bitmap = herm_zero ? live.data() : nullptr;
        a.bitmap_mode = herm_zero ? 2 : 0;
        a.list = tlist.empty() ? &kNone : tlist.data();
        a.list_count = &lcount;
        a.list_shift = 0;
      }
      Checker ck(elems);
      ck.zero_check = false;
      if (dtype == TPD_C128)
        st = emulate_shape<double>(sw[i], (const Cx<double>*)a.in, (Cx<double>*)a.out, a, a.bitmap, ck);
      else
        st = TPD_IF_C64(emulate_shape<float>(sw[i], (const Cx<float>*)a.in, (Cx<float>*)a.out, a, a.bitmap, ck));
      if (st) return st;
      if (!ck.complete()) return TPD_ERROR_INTERNAL;
    }
  }
  for (uint64_t i = 0; i < count; ++i) {
    const uint64_t q = req[i];
    char* dst = (char*)values + i * eb;
    if (q >= elems) {
      if (dtype == TPD_C128) {
        const double nan2[2] = {std::nan(""), std::nan("")};
        std::memcpy(dst, nan2, eb);
      } else {
        const float nan2[2] = {std::nanf(""), std::nanf("")};
        std::memcpy(dst, nan2, eb);
      }
      continue;
    }
    std::memcpy(dst, (const char*)coeffs + storage_of_q(q, n, mat) * eb, eb);
  }
  return TPD_SUCCESS;
}

// host replay of the ordered compaction: the same chunks, per-chunk counts,
// exclusive offsets, capacity clipping and (j, wave, lane) storage order
extern "C" tpd_status_t tpd_debug_emulate_compact(const void* coeffs, int n, tpd_dtype_t dtype, unsigned flags,
                                                  double tol, uint64_t* q_out, void* w_out, uint64_t capacity,
                                                  uint64_t* count) {
  if (!coeffs || !count || (capacity && (!q_out || !w_out))) return TPD_ERROR_INVALID_VALUE;
  if (dtype != TPD_C128 && dtype != TPD_C64) return TPD_ERROR_INVALID_VALUE;
  if (flags & ~TPD_FLAG_LAYOUT_MATRIX) return TPD_ERROR_INVALID_VALUE;
  if (n < 0 || n > 12) return TPD_ERROR_UNSUPPORTED;
  if (!(tol >= 0.0)) return TPD_ERROR_INVALID_VALUE;
  const bool mat = (flags & TPD_FLAG_LAYOUT_MATRIX) != 0;
  const uint64_t elems = (uint64_t)1 << (2 * n);
  const uint64_t nchunks = (elems + kCompactChunk - 1) / kCompactChunk;
  const size_t eb = dtype == TPD_C128 ? 16 : 8;
  auto kept = [&](uint64_t i) {
    if (dtype == TPD_C128) {
      const double* v = (const double*)coeffs + 2 * i;
      return keep_coeff<double>(v[0], v[1], tol);
    }
    const float* v = (const float*)coeffs + 2 * i;
    return keep_coeff<float>(v[0], v[1], (float)tol);
  };
  std::vector<uint32_t> counts(nchunks, 0u);
  for (uint64_t c = 0; c < nchunks; ++c)
    for (uint64_t i = c * kCompactChunk; i < std::min(elems, (c + 1) * kCompactChunk); ++i) counts[c] += kept(i);
  uint64_t run = 0;
  for (uint64_t c = 0; c < nchunks; ++c) {
    uint64_t pos = run;
    run += counts[c];
    if (!counts[c]) continue;
    for (uint64_t i = c * kCompactChunk; i < std::min(elems, (c + 1) * kCompactChunk); ++i) {
      if (!kept(i)) continue;
      if (pos < capacity) {
        q_out[pos] = q_of_storage(i, n, mat);
        std::memcpy((char*)w_out + pos * eb, (const char*)coeffs + i * eb, eb);
      }
      ++pos;
    }
  }
  *count = run;
  return TPD_SUCCESS;
}
