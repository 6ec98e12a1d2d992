// tpd_sweep.h -- the single-matrix sweep kernel template and its
// per-dtype dispatch (instantiated once per dtype in tpd_sweep_c128.hip and
// tpd_sweep_c64.hip so the two compile in parallel).
//
// One launch = one HBM sweep over a single matrix: every tile of
// 2^XB rows x 2^DB XOR-diagonals is loaded (16 B/8 B per element, runs of
// 2^DB elements), transformed on its XB levels through register phases of
// R levels with LDS exchanges between phases, and stored.  See tpd_core.h
// for the coordinates and layouts and tpd_kernels.hip for the schedules.
#pragma once
#include "tpd_internal.h"

namespace tpd {

// ---------------------------------------------------------------------------
// single-matrix sweep
// ---------------------------------------------------------------------------
// A bitmap word that is the same for the whole workgroup and constant for
// the kernel's lifetime (written by an earlier launch), read through the
// constant address space: the load is a scalar one, counted apart from the
// vector memory operations, so deciding on the next tile does not wait for
// the current tile's stores to complete.
__device__ inline uint32_t uniform_word(const uint32_t* p, uint64_t w) {
  typedef const uint32_t __attribute__((address_space(4)))* cptr;
  const uint32_t wi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)w);
  return *(cptr)(p + wi);
}

template <class S, class G, int INL, int OUTL, bool INV = false>
__global__ void __launch_bounds__(G::NT) k_sweep(SweepArgs a) {
  using E = typename Elem<S>::type;  // Cx<double|float>, or Rl<..> for real input
  constexpr bool REAL = Elem<S>::real;
  static constexpr Roles RL = make_roles<G>();
  constexpr int P = G::NPH;
  constexpr int LAST = P - 1;
  constexpr uint32_t DM = (1u << G::DB) - 1;
  constexpr uint32_t XM = (1u << G::XB) - 1;
  constexpr int NBW = (1 << G::XB) >= 32 ? (1 << G::XB) / 32 : 1;
  __shared__ E lds[1 << G::B];
  // split pruning groups (see sub_bits below): only the 8-level, 2^6-wide
  // first sweep of 4-byte elements in the matrix layout takes them
  constexpr bool SPLIT = sizeof(E) <= 4 && INL == L_MAT && OUTL == L_MAT && !INV && G::XB == 8 && G::DB == 6;
  __shared__ uint32_t bits[(SPLIT ? 2 : 1) * NBW];

  static_assert(!(REAL && OUTL == L_CANR), "real-coded elements have no separate real output");
  const uint32_t tid = threadIdx.x;
  const E* __restrict__ in = (const E*)a.in;
  E* __restrict__ out = (E*)a.out;
  // L_CANR: the output is a separate array of real weights
  typename Elem<S>::scalar* __restrict__ outr = (typename Elem<S>::scalar*)a.out;
  const int n = a.n, xlo = a.xlo, db = a.db;
  const int tdb = a.chunk_bits > 0 ? a.chunk_bits : a.nfix_d;  // d-group bits of the tile index
  const uint64_t tdmask = ((uint64_t)1 << tdb) - 1;

  // Canonical-order output: the tile is passed once more through LDS so that
  // each store instruction writes 64 consecutive coefficients (whole cache
  // lines) instead of the last phase's 32-byte pieces.
  constexpr bool REMAP = (OUTL == L_CAN || OUTL == L_CANR) && RL.st_ok;

  // register-slot address deltas (layouts are XOR-linear in (x, d))
  uint64_t din[G::R], dout[G::R];
#pragma unroll
  for (int s = 0; s < G::R; ++s) {
    const uint32_t ei = 1u << RL.reg[0][s];
    din[s] = layout_addr<INL>((uint64_t)((ei >> G::DB) & XM) << xlo, ei & DM, n, db);
    const uint32_t eo = 1u << (REMAP ? RL.st_reg[s] : RL.reg[LAST][s]);
    dout[s] = layout_addr<OUTL>((uint64_t)((eo >> G::DB) & XM) << xlo, eo & DM, n, db);
  }
  // The thread's element bases are recomputed for every tile from an
  // opaque copy of the thread index: hoisted out of the tile loop, every
  // phase's LDS offsets and every register slot's address stayed live
  // across the whole kernel (up to 256 VGPRs, and spills); recomputed, the
  // two-sweep kernels take 58-198 VGPRs and none spills.  The
  // recomputation is a few integer operations per tile.
  auto thread_index = [&]() -> uint32_t {
    uint32_t t = tid;
    asm volatile("" : "+v"(t));
    return t;
  };

  // Tile decode.  A tile is skipped (nothing read or written) when no
  // requested string lies in its d-group, when the pruning bitmap marks its
  // cumulative matrix weight zero, or in the first sweep of a Hermitian
  // input when its row block holds no representatives.
  struct Tile {
    uint64_t td, xf, xfix, hm;
    bool zero;  // Hermitian second sweep, zero tile: only its mirrored rows are stored (zeros)
    bool zall;  // zero tile of a separate real output: every element is stored (zeros)
  };
  // tiles of this launch: all, or the entries of a work list
  const uint64_t lcount = a.list ? (uint64_t)uniform_word(a.list_count, 0) : 0;
  const uint64_t ntiles = a.list ? lcount << a.list_shift : a.ntiles;
  auto decode = [&](uint64_t tile, Tile& t) -> bool {
    if (a.list && a.list_shift) {
      t.xf = tile / lcount;
      t.td = uniform_word(a.list, tile - t.xf * lcount);
    } else if (a.list) {  // second-sweep bitmap bit (td << bm_xbits) | xf
      const uint64_t lt = uniform_word(a.list, tile);
      t.td = lt >> a.bm_xbits;
      t.xf = lt & (((uint64_t)1 << a.bm_xbits) - 1);
    } else if (a.herm && xlo) {
      herm_first_tile(tile, xlo, G::DB, a.nfix_d, &t.xf, &t.td);
    } else {
      t.td = a.td_base + (tile & tdmask);
      t.xf = tile >> tdb;
      if (a.tile_order) {
        // rotated order: the row block index advances with every 8 d-groups,
        // so workgroups running at the same time spread over row blocks (a
        // bijection of the tile index: the tile count is a power of two)
        const uint64_t xmask = (ntiles >> tdb) - 1;
        t.xf = (t.xf ^ (t.td >> 3)) & xmask;
      }
    }
    t.xfix = (t.xf & (((uint64_t)1 << xlo) - 1)) | ((t.xf >> xlo) << (xlo + G::XB));
    if (a.req && !((uniform_word(a.req, t.td >> 5) >> (t.td & 31)) & 1u)) return false;
    // Hermitian input: entry (x, d) is the conjugate of (x ^ d, d), and so
    // is every intermediate value inside one cumulative matrix weight.  With
    // dlh = the d bits of this tile above the diagonal group, below n2, and
    // m the top set bit of d's low n2 bits, only rows with x bit m = 0 are
    // needed ("representatives"); the others follow by conjugation.
    t.hm = 0;  // 1 << m when representatives can be used, else 0
    t.zero = false;
    t.zall = false;
    if (a.herm) {
      const int n2 = xlo ? xlo : G::XB;
      const uint64_t dlh = t.td & (((uint64_t)1 << (n2 - G::DB)) - 1);
      if (dlh) t.hm = (uint64_t)1 << (63 - __builtin_clzll(dlh) + G::DB);
      if (xlo && (t.xf & t.hm)) return false;  // first sweep: never enumerated (herm_first_tile)
    }
    if (a.bitmap_mode == 2) {
      const uint64_t bit = (t.td << a.bm_xbits) | t.xf;
      if (!((uniform_word(a.bitmap, bit >> 5) >> (bit & 31)) & 1u)) {
        // zero subtree: the first sweep already stored its zeros, except, in
        // the Hermitian mode, on the mirrored rows it never visits; those are
        // written here (stores only, nothing is read).  A separate real
        // output receives zeros on every element.
        if constexpr (OUTL == L_CANR) {
          t.zero = true;
          t.zall = true;
          return true;
        }
        if (!(a.herm && !xlo && t.hm)) return false;
        t.zero = true;
      }
    }
    return true;
  };
  auto next_tile = [&](uint64_t tile, Tile& t) -> uint64_t {
    while (tile < ntiles && !decode(tile, t)) tile += gridDim.x;
    return tile;
  };
  auto load = [&](const Tile& t, E* v) {
    if (t.zero) return;
    const uint32_t eb0 = elem_base<G>(RL, 0, thread_index());
    const uint64_t x = t.xfix | ((uint64_t)((eb0 >> G::DB) & XM) << xlo);
    const uint64_t d = (t.td << G::DB) | (eb0 & DM);
    const uint64_t base = layout_addr<INL>(x, d, n, db);
#pragma unroll
    for (int j = 0; j < G::E; ++j) {
      uint64_t ad = base;
#pragma unroll
      for (int s = 0; s < G::R; ++s)
        if ((j >> s) & 1) ad ^= din[s];
      const uint32_t e = eb0 | elem_reg<G>(RL, 0, j);
      if (t.hm && !xlo && (((uint64_t)((e >> G::DB) & XM)) & t.hm)) v[j] = E{};
      else v[j] = in[ad];
      if constexpr (REAL && INV) {
        // synthesis from real-coded weights: back to the raw factor of
        // i^y (the inverse of the forward transform's last store)
        if (!xlo) {
          const uint64_t xe = t.xfix | ((uint64_t)((e >> G::DB) & XM)), de = (t.td << G::DB) | (e & DM);
          if ((__popcll(xe & de) >> 1) & 1) v[j].re = -v[j].re;
        }
      }
    }
  };

  // Pruning bits are per second-sweep tile; with the matrix layout and
  // 4-byte elements that sweep may use d-groups of half this tile's width
  // (sub_bits = 1; only for tiles of >= 32 rows, so every bitmap word belongs
  // to one sub-group).  Lane bit b holds d bit b of the tile in the last
  // phase.  Wider elements keep the plain epilogue: the split's extra
  // per-lane values made the 1024-thread 8-byte kernels spill.
  int sub_bits = 0;
  if constexpr (SPLIT) sub_bits = (G::XB >= 5 && a.bm_db == G::DB - 1) ? 1 : 0;
  // rows held by the last phase's register slots (x offsets of the slots)
  constexpr uint32_t SLOT_ROWS = [] {
    uint32_t r = 0;
    for (int j = 0; j < G::E; ++j) r |= (elem_reg<G>(make_roles<G>(), G::NPH - 1, j) >> G::DB) & ((1u << G::XB) - 1);
    return r;
  }();
  constexpr bool ROWS_IN_WORD = G::XB >= 5 && SLOT_ROWS < 32;
  const int nbw = NBW << sub_bits;

  // Transform one loaded tile and store it.
  auto process = [&](const Tile& t, E* v) {
    const uint64_t td = t.td, hm = t.hm, xfix = t.xfix;
    const uint32_t tid = thread_index();
    const uint32_t eb0 = elem_base<G>(RL, 0, tid);
    const uint32_t ebl = elem_base<G>(RL, LAST, tid);
    const uint32_t ebo = REMAP ? elem_base_st<G>(RL, tid) : ebl;  // element base of the stores
    if (t.zero) {
      // Hermitian zero tile: zeros on the rows with x bit m set (the
      // representatives already hold the first sweep's zeros).  Row bit m
      // of an element is the same in every layout, so these are exactly the
      // addresses the first sweep left unwritten.
      const uint64_t x = xfix | ((uint64_t)((ebo >> G::DB) & XM) << xlo);
      const uint64_t d = (td << G::DB) | (ebo & DM);
      const uint64_t base = layout_addr<OUTL>(x, d, n, db);
#pragma unroll
      for (int j = 0; j < G::E; ++j) {
        const uint32_t e = REMAP ? (ebo | elem_reg_st<G>(RL, j)) : (ebl | elem_reg<G>(RL, LAST, j));
        if (!t.zall && !(((uint64_t)((e >> G::DB) & XM)) & hm)) continue;
        uint64_t ad = base;
#pragma unroll
        for (int s = 0; s < G::R; ++s)
          if ((j >> s) & 1) ad ^= dout[s];
        if constexpr (OUTL == L_CANR) outr[ad] = (typename Elem<S>::scalar)0;
        else out[ad] = E{};
      }
      return;
    }
    if constexpr (SPLIT) {
      if (a.bitmap_mode == 1 && (int)tid < nbw) bits[tid] = 0;
    } else {
      if (a.bitmap_mode == 1 && tid < NBW) bits[tid] = 0;
    }

    if (hm && !xlo) {
      // second sweep: rebuild the non-representative rows by conjugation
      const uint64_t dlo_hi = (td << G::DB) & ((((uint64_t)1 << G::XB) - 1));
      __syncthreads();
#pragma unroll
      for (int j = 0; j < G::E; ++j) {
        const uint32_t e = eb0 | elem_reg<G>(RL, 0, j);
        if (((uint64_t)((e >> G::DB) & XM)) & hm) continue;
        const uint32_t dlo = (uint32_t)(dlo_hi | (e & DM));
        lds[e] = v[j];
        if constexpr (REAL) {
          // conj(i^k r) = i^k (-1)^k r, k = the Y letters of the first
          // sweep's levels (x and d bits from XB up), the same at both rows
          const uint64_t x = xfix | ((e >> G::DB) & XM), d = (td << G::DB) | (e & DM);
          const bool neg = __popcll((x & d) >> G::XB) & 1;
          lds[e ^ (dlo << G::DB)] = E{neg ? -v[j].re : v[j].re};
        } else {
          lds[e ^ (dlo << G::DB)] = Cx<S>{v[j].re, -v[j].im};
        }
      }
      __syncthreads();
#pragma unroll
      for (int j = 0; j < G::E; ++j) v[j] = lds[eb0 | elem_reg<G>(RL, 0, j)];
    }

#pragma unroll
    for (int p = 0; p < P; ++p) {
      const uint32_t ebp = elem_base<G>(RL, p, tid);
      phase_butterflies<G, S, INV>(RL, p, v, (td << G::DB) | (ebp & DM), xlo);
      if (p + 1 < P) {
        __syncthreads();
#pragma unroll
        for (int j = 0; j < G::E; ++j) lds[ebp | elem_reg<G>(RL, p, j)] = v[j];
        __syncthreads();
        const uint32_t ebn = elem_base<G>(RL, p + 1, tid);
#pragma unroll
        for (int j = 0; j < G::E; ++j) v[j] = lds[ebn | elem_reg<G>(RL, p + 1, j)];
      }
    }

    if (a.bitmap_mode == 1 && !SPLIT && ROWS_IN_WORD) {
      // OR "any nonzero" over the 2^DB diagonals (lanes [0, DB)) of each row
      // block; one bit per second-sweep tile (td, x_hi).  NaN counts as nonzero.
      // The register slots of the last phase hold rows that differ only in
      // their low 5 bits, so each lane group's rows share one bitmap word:
      // its leader ORs them in with one global atomic (no LDS pass, and no
      // barrier between the transform and the stores).
      const uint32_t lane = tid & 63u;
      constexpr uint32_t gsz = 1u << G::DB;
      constexpr uint64_t gmask = gsz >= 64 ? ~0ull : ((1ull << gsz) - 1);
      uint32_t wbits = 0;
#pragma unroll
      for (int j = 0; j < G::E; ++j) {
        const uint64_t m = __ballot(nonzero(v[j]));
        if ((m >> (lane & ~(gsz - 1))) & gmask) wbits |= 1u << ((elem_reg<G>(RL, LAST, j) >> G::DB) & XM);
      }
      if ((lane & (gsz - 1)) == 0 && wbits) {
        const uint64_t b0 = (td << a.bm_xbits) + ((ebl >> G::DB) & XM);
        atomicOr(&a.bitmap[b0 >> 5], wbits << (b0 & 31));
      }
    }
    if (a.bitmap_mode == 1 && !SPLIT && !ROWS_IN_WORD) {
      // OR "any nonzero" over the 2^DB diagonals (lanes [0, DB)) of each row
      // block; one bit per second-sweep tile (td, x_hi).  NaN counts as nonzero.
      const uint32_t lane = tid & 63u;
      constexpr uint32_t gsz = 1u << G::DB;
      constexpr uint64_t gmask = gsz >= 64 ? ~0ull : ((1ull << gsz) - 1);
      if (P == 1) __syncthreads();
#pragma unroll
      for (int j = 0; j < G::E; ++j) {
        const bool nz = nonzero(v[j]);
        const uint64_t m = __ballot(nz);
        if ((lane & (gsz - 1)) == 0 && ((m >> lane) & gmask)) {
          const uint32_t xl = ((ebl | elem_reg<G>(RL, LAST, j)) >> G::DB) & XM;
          atomicOr(&bits[xl >> 5], 1u << (xl & 31));
        }
      }
      __syncthreads();
      if (tid < NBW) {
        const uint32_t w = bits[tid];
        if (w) {
          const uint64_t b0 = (td << a.bm_xbits) + 32ull * tid;
          atomicOr(&a.bitmap[b0 >> 5], w << (b0 & 31));
        }
      }
    }
    if (a.bitmap_mode == 1 && SPLIT) {
      // OR "any nonzero" over the diagonals of each second-sweep d-group
      // (2^(DB - sub_bits) consecutive lanes) of each row block; one bit per
      // second-sweep tile (td << sub_bits | sub, x_hi).  NaN counts as nonzero.
      const uint32_t lane = tid & 63u;
      const uint32_t gsz = 1u << (G::DB - sub_bits);
      const uint64_t gmask = gsz >= 64 ? ~0ull : ((1ull << gsz) - 1);
      if (P == 1) __syncthreads();
#pragma unroll
      for (int j = 0; j < G::E; ++j) {
        const bool nz = nonzero(v[j]);
        const uint64_t m = __ballot(nz);
        if ((lane & (gsz - 1)) == 0 && ((m >> lane) & gmask)) {
          const uint32_t xl = ((ebl | elem_reg<G>(RL, LAST, j)) >> G::DB) & XM;
          const uint32_t sub = (lane >> (G::DB - sub_bits)) & ((1u << sub_bits) - 1);
          const uint32_t bi = (sub << G::XB) | xl;
          atomicOr(&bits[bi >> 5], 1u << (bi & 31));
        }
      }
      __syncthreads();
      if ((int)tid < nbw) {
        const uint32_t w = bits[tid];
        if (w) {
          const uint32_t sub = tid / NBW, wi = tid % NBW;
          const uint64_t b0 = ((((uint64_t)td << sub_bits) | sub) << a.bm_xbits) + 32ull * wi;
          atomicOr(&a.bitmap[b0 >> 5], w << (b0 & 31));
        }
      }
    }

    if constexpr (REMAP) {
      __syncthreads();
#pragma unroll
      for (int j = 0; j < G::E; ++j) lds[ebl | elem_reg<G>(RL, LAST, j)] = v[j];
      __syncthreads();
#pragma unroll
      for (int j = 0; j < G::E; ++j) v[j] = lds[ebo | elem_reg_st<G>(RL, j)];
    } else if (P == 1 && INL != OUTL) {
      __syncthreads();  // in place: all loads before any store
    }
    {
      const uint64_t x = xfix | ((uint64_t)((ebo >> G::DB) & XM) << xlo);
      const uint64_t d = (td << G::DB) | (ebo & DM);
      const uint64_t base = layout_addr<OUTL>(x, d, n, db);
      const bool real_out = a.herm && !xlo;  // Hermitian weights are real
#pragma unroll
      for (int j = 0; j < G::E; ++j) {
        uint64_t ad = base;
#pragma unroll
        for (int s = 0; s < G::R; ++s)
          if ((j >> s) & 1) ad ^= dout[s];
        if constexpr (REAL && !INV) {
          // last sweep: the weight is i^y r (y = Y letters = popcount(x & d));
          // store its nonzero component, Re w for even y and Im w for odd y,
          // i.e. r negated when y mod 4 is 2 or 3
          if (!xlo) {
            const uint32_t e = REMAP ? (ebo | elem_reg_st<G>(RL, j)) : (ebl | elem_reg<G>(RL, LAST, j));
            const uint64_t xe = xfix | ((uint64_t)((e >> G::DB) & XM)), de = (td << G::DB) | (e & DM);
            if ((__popcll(xe & de) >> 1) & 1) v[j].re = -v[j].re;
          }
        } else if constexpr (!REAL) {
          if (real_out) v[j].im = (typename Elem<S>::scalar)0;
        }
        if constexpr (OUTL == L_CANR) outr[ad] = v[j].re;
        else out[ad] = v[j];
      }
    }
  };

  // Persistent grids (gridDim.x < ntiles) issue the next tile's loads before
  // transforming and storing the current one.  The first tile is peeled off
  // so that the loop is entered with the same operations in flight as on
  // its back edge (next loads, then current stores): the copy of the
  // prefetched data then waits for those loads only, never for the stores.
  // Workgroups of 1024 threads have 128 registers per thread.  They prefetch
  // for 4-byte elements outside the canonical store's extra LDS pass, and
  // for 8-byte elements read in the matrix layout and stored in place or as
  // real weights (tiles of 2^8 rows or fewer); the others load at the top of
  // each iteration (measured: complex64 n = 16 in place 2.4-3.2 % faster
  // with the prefetch, real float64 1.5 %, complex64 real weights 6 %).
  // Since the element bases are recomputed per tile, a second copy fits
  // without spills in every 1024-thread kernel, but prefetching in the
  // remaining ones measured no gain (complex64, real float64 and real
  // float32 n = 16 out of place, complex64 synthesis: within 1 %).
  constexpr bool PF = G::NT < 1024 || (sizeof(E) <= 4 && OUTL != L_CAN && !INV) ||
                       (sizeof(E) == 8 && INL == L_MAT && (OUTL == L_MAT || OUTL == L_CANR) && !INV && G::XB <= 8);
  if constexpr (PF) {
    Tile cur, nxt;
    const uint64_t first = next_tile(blockIdx.x, cur);
    if (first >= ntiles) return;
    E v[G::E], pf[G::E];
    load(cur, v);
    uint64_t next = next_tile(first + gridDim.x, nxt);
    if (next < ntiles) load(nxt, pf);
    process(cur, v);
    while (next < ntiles) {
#pragma unroll
      for (int j = 0; j < G::E; ++j) v[j] = pf[j];
      cur = nxt;
      next = next_tile(next + gridDim.x, nxt);
      if (next < ntiles) load(nxt, pf);
      process(cur, v);
    }
  } else {
    Tile cur;
    for (uint64_t tile = next_tile(blockIdx.x, cur); tile < ntiles; tile = next_tile(tile + gridDim.x, cur)) {
      E v[G::E];
      load(cur, v);
      process(cur, v);
    }
  }
}

// ---------------------------------------------------------------------------
// launch of one instantiation
// ---------------------------------------------------------------------------
template <class S, int XB, int DB, int ORDER, int INL, int OUTL, int RR, bool INV = false>
hipError_t launch_one(const SweepArgs& a, int grid_req, hipStream_t st) {
  // at most 1024 threads per tile, at most 16 elements per thread
  constexpr int R1 = (XB + DB - 10) > RR ? (XB + DB - 10) : RR;
  constexpr int R = (XB + DB) < R1 ? (XB + DB) : R1;
  using G = Geom<XB, DB, 0, R, ORDER>;
  if constexpr (!shape_fits<S>(XB, DB) || XB + DB > 14) {  // <= 1024 threads of 16 elements
    return hipErrorInvalidValue;
  } else {
    // one workgroup per tile, or a persistent grid that loops over tiles;
    // HIP needs grid * block < 2^32 threads
    uint64_t grid = grid_req > 0 ? (uint64_t)grid_req : a.ntiles;
    if (grid > a.ntiles) grid = a.ntiles;
    const uint64_t cap = 0xFFFFFFFFull / (uint64_t)G::NT;
    if (grid > cap) grid = cap;
    hipLaunchKernelGGL((k_sweep<S, G, INL, OUTL, INV>), dim3((unsigned)grid), dim3(G::NT), 0, st, a);
    return hipGetLastError();
  }
}

// one-sweep shapes (n <= 8): MAT -> CAN or MAT -> MAT, R = 4
#define TPD_ONE_SHAPES(X) X(1, 1) X(2, 2) X(3, 3) X(4, 4) X(5, 5) X(6, 6) X(7, 5) X(8, 4)

template <class S>
hipError_t dispatch_one(const SweepDesc& s, const SweepArgs& a, hipStream_t st) {
#define TPD_CASE(XB_, DB_)                                                                           \
  if (s.xb == XB_ && s.db == DB_) {                                                                  \
    if (s.out_layout == L_CAN) return launch_one<S, XB_, DB_, 0, L_MAT, L_CAN, 4>(a, s.grid, st);    \
    if (s.out_layout == L_MAT) return launch_one<S, XB_, DB_, 0, L_MAT, L_MAT, 4>(a, s.grid, st);    \
    if constexpr (!Elem<S>::real)                                                                    \
      if (s.out_layout == L_CANR) return launch_one<S, XB_, DB_, 0, L_MAT, L_CANR, 4>(a, s.grid, st); \
  }
  TPD_ONE_SHAPES(TPD_CASE)
#undef TPD_CASE
  return hipErrorInvalidValue;
}

// two-sweep halves: XB in 4..9 for the tile widths DB of one dtype, 16
// elements per thread; the bottom-first phase order only for the default
// tile width
template <class S, int XB, int DB, int RR>
hipError_t dispatch_two_layouts(const SweepDesc& s, const SweepArgs& a, hipStream_t st) {
  if (s.in_layout == L_MAT && s.out_layout == L_MID) return launch_one<S, XB, DB, 0, L_MAT, L_MID, RR>(a, s.grid, st);
  if (s.in_layout == L_MID && s.out_layout == L_CAN) return launch_one<S, XB, DB, 0, L_MID, L_CAN, RR>(a, s.grid, st);
  if (s.in_layout == L_MAT && s.out_layout == L_MAT) return launch_one<S, XB, DB, 0, L_MAT, L_MAT, RR>(a, s.grid, st);
  if constexpr (!Elem<S>::real)  // Hermitian second sweep into a separate real output
    if (s.in_layout == L_MAT && s.out_layout == L_CANR) return launch_one<S, XB, DB, 0, L_MAT, L_CANR, RR>(a, s.grid, st);
  return hipErrorInvalidValue;
}
template <class S, int XB, int DB>
hipError_t dispatch_two_bottom(const SweepDesc& s, const SweepArgs& a, hipStream_t st) {
  if (s.in_layout == L_MID && s.out_layout == L_CAN) return launch_one<S, XB, DB, 1, L_MID, L_CAN, 4>(a, s.grid, st);
  if (s.in_layout == L_MAT && s.out_layout == L_MAT) return launch_one<S, XB, DB, 1, L_MAT, L_MAT, 4>(a, s.grid, st);
  return hipErrorInvalidValue;
}
template <class S, int XB, int DB>
hipError_t dispatch_two_r(const SweepDesc& s, const SweepArgs& a, hipStream_t st) {
  if (s.order == 1) return dispatch_two_bottom<S, XB, DB>(s, a, st);
  return dispatch_two_layouts<S, XB, DB, 4>(s, a, st);
}
template <class S, int DB>
hipError_t dispatch_two_xb(const SweepDesc& s, const SweepArgs& a, hipStream_t st) {
  switch (s.xb) {
    case 4: return dispatch_two_r<S, 4, DB>(s, a, st);
    case 5: return dispatch_two_r<S, 5, DB>(s, a, st);
    case 6: return dispatch_two_r<S, 6, DB>(s, a, st);
    case 7: return dispatch_two_r<S, 7, DB>(s, a, st);
    case 8: return dispatch_two_r<S, 8, DB>(s, a, st);
    case 9: return dispatch_two_r<S, 9, DB>(s, a, st);  // n = 17, first sweep
  }
  return hipErrorInvalidValue;
}

// inverse transform (synthesis): one sweep CAN|MAT -> MAT for n <= 8; two
// sweeps for n >= 9 (low levels CAN|MAT -> MAT, then high levels MAT -> MAT
// in place), default tile widths only
template <class S, int XB, int DB>
hipError_t dispatch_inv_layouts(const SweepDesc& s, const SweepArgs& a, hipStream_t st) {
  if (s.out_layout != L_MAT) return hipErrorInvalidValue;
  if (s.in_layout == L_CAN) return launch_one<S, XB, DB, 0, L_CAN, L_MAT, 4, true>(a, s.grid, st);
  if (s.in_layout == L_MAT) return launch_one<S, XB, DB, 0, L_MAT, L_MAT, 4, true>(a, s.grid, st);
  return hipErrorInvalidValue;
}
template <class S, int DB>
hipError_t dispatch_inv_two(const SweepDesc& s, const SweepArgs& a, hipStream_t st) {
  switch (s.xb) {
    case 4: return dispatch_inv_layouts<S, 4, DB>(s, a, st);
    case 5: return dispatch_inv_layouts<S, 5, DB>(s, a, st);
    case 6: return dispatch_inv_layouts<S, 6, DB>(s, a, st);
    case 7: return dispatch_inv_layouts<S, 7, DB>(s, a, st);
    case 8: return dispatch_inv_layouts<S, 8, DB>(s, a, st);
    case 9: return dispatch_inv_layouts<S, 9, DB>(s, a, st);  // n = 17, second synthesis sweep
  }
  return hipErrorInvalidValue;
}
template <class S>
hipError_t dispatch_inv(const SweepDesc& s, const SweepArgs& a, hipStream_t st) {
  if (s.is_one) {
#define TPD_CASE(XB_, DB_) \
    if (s.xb == XB_ && s.db == DB_) return dispatch_inv_layouts<S, XB_, DB_>(s, a, st);
    TPD_ONE_SHAPES(TPD_CASE)
#undef TPD_CASE
    return hipErrorInvalidValue;
  }
  if (s.db == 4) return dispatch_inv_two<S, 4>(s, a, st);
  if (s.db == 5) return dispatch_inv_two<S, 5>(s, a, st);
  return hipErrorInvalidValue;
}

}  // namespace tpd
