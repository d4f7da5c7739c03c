// Neighbour candidate scans and lane-group helpers of the pair passes, their adjoints and the
// pair dump (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "mpsph_device.h"

// The candidate scan ends each chunk with NaN row offsets and relies on every range test failing
// on a NaN distance, which finite-only floating-point modes would not keep.
#if defined(__FAST_MATH__) || (defined(__FINITE_MATH_ONLY__) && __FINITE_MATH_ONLY__)
#error "the pair kernels need IEEE NaN semantics: build without -ffast-math / -ffinite-math-only"
#endif

namespace mpsph {

// Neighbour candidates
//
// Particle i's candidates are the particles of every x-run of cells (fixed y, z) that meets the
// ball of radius rs around it, the run taken at x sub-cell resolution; in the cell order (x
// fastest) each run is one contiguous range of the sorted arrays.  A group of L lanes works on
// one particle (scan_group_table below).
// ------------------------------------------------------------------------------------------
// Lanes per particle of the pair kernels of a context that is not tuned (mpsph_configure and
// mpsph_autotune choose 2, 4 or 8), and of the adjoint's pair kernels.  Measured: 8 lanes are the
// fastest on the 2M-particle graded cube, 4 on the RBF cube's forward steps (8 lanes: 4 % slower)
// and equal on the 64-domain batch; the adjoint's pair kernels run faster at 8.
#ifndef MPSPH_LANES
#define MPSPH_LANES 4
#endif
#ifndef MPSPH_ADJ_LANES
#define MPSPH_ADJ_LANES 8
#endif

// x cell of a particle from its flags word (bits 16-27).  A 3D grid has at most 2^8 cells per
// axis, so there the word's third byte holds it and converts to float in one instruction.
template <int D>
__device__ __forceinline__ float cell_x(uint32_t aux) {
  return D == 3 ? (float)((aux >> 16) & 0xFFu) : (float)((aux >> 16) & 0xFFFu);
}

// x separation in cell units with the minimum image of a periodic box (period P cells); the
// y and z separations come from unwrapped row offsets and need none.  fcxi: the particle's x
// cell as a float (exact); auxj: the neighbour's flags word.
// PER: the launch may contain periodic domains (otherwise the periodic code is compiled out).
template <bool PER, int D>
__device__ __forceinline__ float sep_x(const GridDev &g, float fcxi, uint32_t auxj, float oxi, float oxj) {
  float dx = (fcxi - cell_x<D>(auxj)) + (oxi - oxj);
  if (PER && g.geometry == 0) {
    const float P = (float)(g.gmax + 1);
    dx = dx > 0.5f * P ? dx - P : (dx < -0.5f * P ? dx + P : dx);
  }
  return dx;
}

// Value of lane l - o (o < 16) within the lane's row of 16 lanes, through a DPP row shift (no
// LDS round trip and no lane arithmetic); lanes l < o of the row get 0.  Used for prefix sums
// inside groups of at most 16 lanes, where the lanes that would read across the group's start
// discard the value.
__device__ __forceinline__ uint32_t lane_up(uint32_t x, int o) {
  switch (o) {   // the shift is an immediate of the instruction
    case 1: return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xF, 0xF, true);
    case 2: return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xF, 0xF, true);
    case 4: return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xF, 0xF, true);
    default: return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xF, 0xF, true);
  }
}
// The value of the group's last lane (L lanes, L <= 16), in every lane of the group, through
// ds_swizzle in its bit-mask mode: source lane = (lane & ~(L - 1)) | (L - 1) within 32 lanes.
template <int L>
__device__ __forceinline__ uint32_t group_last(uint32_t x) {
  static_assert(L >= 2 && L <= 16 && (L & (L - 1)) == 0, "groups of 2 to 16 lanes");
  return (uint32_t)__builtin_amdgcn_ds_swizzle((int)x, (0x1F & ~(L - 1)) | ((L - 1) << 5));
}

// Rows per chunk of the LDS row table at 4 lanes per particle (scaled with the lanes, so that
// the table of a 256-thread block stays below 19 KB and 8 blocks fit a CU's LDS).
#ifndef MPSPH_ROW_TABLE
#define MPSPH_ROW_TABLE 18
#endif
template <int L>
constexpr int row_table_rows() {
  return MPSPH_ROW_TABLE * L / 4 < L + 1 ? L + 1 : MPSPH_ROW_TABLE * L / 4;
}
// Entries between two rows of one group's column (one more than the groups of a block, so that
// the columns of a wave's groups start in different banks).
template <int L>
constexpr int row_table_stride() {
  return kBlock / L + 1;
}

// Candidate scan with a row table in LDS (the pair passes, their adjoints and the pair dump).
//
// The group's L lanes take L rows at a time (each reads its row's range from the cell table)
// and lay out the non-empty ones in a table in LDS: base index, end of the run in the flattened
// slot order of the particle's candidates, row offsets.  Then the group visits the slots L at a
// time, lane l taking every L-th one and advancing through the table as its slot index passes
// the end of a row.  A group's loop ends when its own candidates end (no wave-wide rounds of
// rows).  A table holds at most C - 1 rows and an end marker; a particle with more non-empty
// rows is scanned in several chunks.  With CUT the particle's own slot is cut out of its row
// (the row becomes the runs before and after it), so the particle itself is never a slot.
// The end marker (end of run 2^32 - 1, row offsets NaN) stops every lane's walk through the
// table, so the slot loop tests neither the table's length nor the chunk's: a slot past the
// chunk's end reaches the marker and gets the index t - run (in [0, L)) and NaN offsets, which
// make its squared distance NaN and fail every range test of the bodies.
// tab: the group's column of the table, entry e at tab[e * stride]; C > L + 1.
// body(j, dy0, dz0, valid) is called for every slot with the row offsets plus the particle's own
// offsets, dy0 = ci[1] - cy + oi[1] and dz0 = ci[2] - cz + oi[2] (cell units; the y and z
// separations are dy0 - oj[1] and dz0 - oj[2]); valid is false for the particle itself (always
// true with CUT).  A slot
// past the chunk's end carries NaN offsets and an index below L that may still lie outside the
// arrays (fewer than L particles): bodies load through bounds-checked buffer loads or clamp the
// index, and must fail their range tests on a NaN distance.  The return value is the group's
// candidate count (the particle itself excluded), the same in every lane of the group.
// The row's base index goes through remap(cy, cz, a) (a: the global index of the row's first
// candidate) before it enters the table, so that the slots can index a staged copy of the
// neighbours; self is the particle's own index in that numbering.
// A body may also come in two parts, fetch(j) -> payload (the slot's neighbour loads) and
// use(payload, dy0, dz0, valid) (its arithmetic): the scan then issues the loads of a lane's
// next slot round before the arithmetic of the current one, so that their latency overlaps it.
// A fetch past the chunk's end gets an index below 2L (bounds-checked loads again).
struct IdentityRemap {
  __device__ __forceinline__ uint32_t operator()(int, int, uint32_t a) const { return a; }
};
template <typename FetchF, typename UseF>
struct SplitBody {
  FetchF fetch;
  UseF use;
};
// The two-part body when PIPE, else one body that loads and computes in turn (fewer registers
// live across the loop: the kernels that could not hold a second round's loads in 64 registers
// without spilling take it).
template <bool PIPE, typename FetchF, typename UseF>
__device__ __forceinline__ auto pair_body(FetchF fetch, UseF use) {
  if constexpr (PIPE)
    return SplitBody<FetchF, UseF>{fetch, use};
  else
    return [=](uint32_t j, float dy0, float dz0, bool v) { use(fetch(j), dy0, dz0, v); };
}
template <typename T>
struct IsSplitBody {
  static constexpr bool value = false;
};
template <typename F, typename U>
struct IsSplitBody<SplitBody<F, U>> {
  static constexpr bool value = true;
};
template <int D, int L, int C, bool PER = false, bool CUT = true, typename BodyF, typename RemapF = IdentityRemap>
__device__ __forceinline__ uint32_t scan_group_table(int i, int sub, uint4 *tab, int stride, const int *ci,
                                                     const float *oi, float rs, const GridDev &g, uint32_t cellbase,
                                                     const uint32_t *__restrict__ cstart, BodyF &&body,
                                                     RemapF remap = RemapF(), uint32_t self = 0xFFFFFFFFu) {
  if (self == 0xFFFFFFFFu) self = (uint32_t)i;
  static_assert(C > L + 1, "a table chunk holds at least one round of rows (one of them split) and the end marker");
  // one lane per particle is not supported: with no cross-lane operation in the loop nest the
  // compiler merged the chunk loop with the table loop and took the chunk loop's exit mask from a
  // compare of the divergent inner loop, and such a build listed some candidates twice (the same
  // build with the chunk bound passed through a width-1 shuffle listed each once)
  static_assert(L >= 2, "at least two lanes per particle");
  static_assert(L <= 16, "a group's prefix sums use row shifts within 16 lanes");
  rs = fminf(fmaxf(rs, 0.f), 2.f * (float)g.gmax + 2.f);
  const float rs2 = rs * rs;
  const bool per = PER && g.geometry == 0;
  const int P = g.gmax + 1;
  int z0 = D == 3 ? ci[2] + (int)floorf(oi[2] - rs) : 0;
  int z1 = D == 3 ? ci[2] + (int)floorf(oi[2] + rs) : 0;
  int y0 = ci[1] + (int)floorf(oi[1] - rs);
  int y1 = ci[1] + (int)floorf(oi[1] + rs);
  if (per) {
    if (y1 - y0 + 1 > P) {
      y0 = ci[1] - P / 2;
      y1 = y0 + P - 1;
    }
    if (D == 3 && z1 - z0 + 1 > P) {
      z0 = ci[2] - P / 2;
      z1 = z0 + P - 1;
    }
  } else {
    y0 = max(0, y0);
    y1 = min(g.gmax, y1);
    if (D == 3) {
      z0 = max(0, z0);
      z1 = min(g.gmax, z1);
    }
  }
  const int ny = y1 - y0 + 1;
  const int nrows = ny * (z1 - z0 + 1);
  const float inv_ny = 1.f / (float)ny;
  const uint32_t nmax = (uint32_t)g.n;
  const float fx = (float)(1u << g.xe);
  const int xlast = ((g.gmax + 1) << g.xe) - 1;
  const uint32_t kx = g.k + g.xe;
  uint32_t total = 0;   // candidates of the group (the particle itself only without CUT)
  int q0 = 0;
  while (q0 < nrows) {
    // table of the next chunk of rows: whole rounds of L rows while a round surely fits
    uint32_t ne = 0, run = 0;
    while (q0 < nrows && ne + L + 1u < (uint32_t)C) {
      const int q = q0 + sub;
      const int qz = (int)(((float)q + 0.5f) * inv_ny);   // q / ny (q, ny < 2^12)
      const int cz = z0 + qz, cy = y0 + (q - qz * ny);
      float ez = 0.f;
      if constexpr (D == 3) {
        const float lo = (float)(cz - ci[2]) - oi[2], hi = lo + 1.f;
        ez = lo > 0.f ? lo : (hi < 0.f ? -hi : 0.f);
      }
      const float lo = (float)(cy - ci[1]) - oi[1], hi = lo + 1.f;
      const float ey = lo > 0.f ? lo : (hi < 0.f ? -hi : 0.f);
      const float d2 = ey * ey + ez * ez;
      const bool hit = q < nrows && d2 < rs2;
      // the hardware square root (about 1 ulp) is enough: the callers' reach rs exceeds every
      // range test of the bodies by a relative 1e-4
      const float wx = fast_sqrt(fmaxf(rs2 - d2, 0.f));
      int x0 = (ci[0] << g.xe) + (int)floorf((oi[0] - wx) * fx);
      int x1 = (ci[0] << g.xe) + (int)floorf((oi[0] + wx) * fx);
      if (per && (x0 < 0 || x1 > xlast)) {
        x0 = 0;
        x1 = xlast;
      }
      x0 = max(0, x0);
      x1 = min(xlast, x1);
      const int cyw = per ? (cy + P) & g.gmax : cy;
      uint32_t kb;
      if constexpr (D == 3)
        kb = (uint32_t)x0 | (row_index(cyw, per ? (cz + P) & g.gmax : cz, g) << kx);
      else
        kb = (uint32_t)x0 | ((uint32_t)cyw << kx);
      kb += cellbase;
      uint32_t a = 0u, b = 0u;
      if (hit) {
        a = cstart[kb];
        b = min(cstart[kb + (uint32_t)(x1 - x0) + 1u], nmax);
      }
      const uint32_t len = b > a ? b - a : 0u;
      // the particle's own slot is cut out of its row, which becomes the runs before and after it
      // (len1 and len2 candidates; a row without the particle keeps len1 = len)
      uint32_t base = 0u, len1 = len, len2 = 0u;
      if (len > 0u) {
        base = remap(cy, cz, a);
        const uint32_t o = self - base;   // >= len unless the particle lies in this run
        if (CUT && o < len) {
          len1 = o;
          len2 = len - o - 1u;
        }
      }
      const uint32_t lsum = len1 + len2, nl = (len1 > 0u ? 1u : 0u) + (len2 > 0u ? 1u : 0u);
      // prefix sums over the group of the candidates and of the table entries
      uint32_t incl = lsum, nz = nl;
#pragma unroll
      for (int o = 1; o < L; o <<= 1) {
        const uint32_t v = lane_up(incl, o), w = lane_up(nz, o);
        if (sub >= o) {
          incl += v;
          nz += w;
        }
      }
      if (nl > 0u) {
        const float dyo = (float)(ci[1] - cy) + oi[1], dzo = D == 3 ? (float)(ci[2] - cz) + oi[2] : 0.f;
        uint32_t end = run + incl - lsum, en = ne + nz - nl;   // the lane's first slot and entry
        if (len1 > 0u) {
          end += len1;
          tab[en++ * (uint32_t)stride] = make_uint4(base - (end - len1), end, __float_as_uint(dyo), __float_as_uint(dzo));
        }
        if (len2 > 0u) {
          end += len2;
          tab[en * (uint32_t)stride] =
              make_uint4(base + len1 + 1u - (end - len2), end, __float_as_uint(dyo), __float_as_uint(dzo));
        }
      }
      run += group_last<L>(incl);
      ne += group_last<L>(nz);
      q0 += L;
    }
    // end marker (ne < C): base -run, so that slot t past the end maps to index t - run
    if (sub == 0) tab[ne * (uint32_t)stride] = make_uint4(0u - run, 0xFFFFFFFFu, 0x7FC00000u, 0x7FC00000u);
    total += run;
    // the chunk's slots, L at a time; slot t of row e is candidate base_e + t
    if constexpr (IsSplitBody<typename std::decay<BodyF>::type>::value) {
      // one round ahead: the loads of slot t + L are issued before the arithmetic of slot t.  A
      // slot's row is found by walking the rows' ends, and its base and offsets are then read from
      // the table into the slot's own registers, so that none is copied
      using Payload = decltype(body.fetch(0u));
      struct Slot {
        Payload p;
        float dy, dz;
        uint32_t j;
      };
      const uint4 *rp = tab;   // row of the last located slot
      uint32_t y = rp->y;      // its end
      const auto locate = [&](uint32_t tt, Slot &sl) {
        while (tt >= y) {
          rp += stride;
          y = rp->y;
        }
        const uint4 row = *rp;
        sl.j = row.x + tt;
        sl.dy = __uint_as_float(row.z);
        sl.dz = __uint_as_float(row.w);
        sl.p = body.fetch(sl.j);
      };
      uint32_t t = (uint32_t)sub;
      // two slots used in turn (the loop is unrolled twice)
      Slot pa, pb;
      locate(t, pa);
      const auto round = [&](const Slot &now, Slot &next) {
        const uint32_t tn = t + L;
        locate(tn, next);
        body.use(now.p, now.dy, now.dz, CUT || now.j != self);
        t = tn;
      };
      // the lane's rounds end when its next slot t reaches the chunk's end (run + sub)
      const uint32_t tend = run + (uint32_t)sub;
      if (t < tend) {
        while (true) {
          round(pa, pb);
          if (t >= tend) break;
          round(pb, pa);
          if (t >= tend) break;
        }
      }
    } else {
      uint32_t e = 0;
      uint4 cur = tab[0];
      for (uint32_t t0 = 0; t0 < run; t0 += L) {
        const uint32_t t = t0 + (uint32_t)sub;
        while (t >= cur.y) cur = tab[++e * (uint32_t)stride];
        const uint32_t j = cur.x + t;
        body(j, __uint_as_float(cur.z), __uint_as_float(cur.w), CUT || j != self);
      }
    }
  }
  return CUT ? total : (total > 0u ? total - 1u : 0u);
}

// Sum / minimum across the L lanes of a group (fixed butterfly order: lane l combines with lane
// l ^ o for o = L/2, ..., 1).  The partner's value comes through ds_swizzle in its bit-mask mode
// (and-mask 31, xor-mask o), which needs no per-lane address arithmetic; groups never straddle
// the 32-lane halves the swizzle works in (L <= 32).
template <int O>
__device__ __forceinline__ uint32_t xor_lane(uint32_t v) {
  static_assert(O > 0 && O < 32, "swizzle xor masks stay within 32 lanes");
  return (uint32_t)__builtin_amdgcn_ds_swizzle((int)v, 0x1F | (O << 10));
}
template <int L>
__device__ __forceinline__ float group_sum(float x) {
  static_assert(L <= 32, "a group fits in 32 lanes");
  if constexpr (L >= 32) x += __uint_as_float(xor_lane<16>(__float_as_uint(x)));
  if constexpr (L >= 16) x += __uint_as_float(xor_lane<8>(__float_as_uint(x)));
  if constexpr (L >= 8) x += __uint_as_float(xor_lane<4>(__float_as_uint(x)));
  if constexpr (L >= 4) x += __uint_as_float(xor_lane<2>(__float_as_uint(x)));
  if constexpr (L >= 2) x += __uint_as_float(xor_lane<1>(__float_as_uint(x)));
  return x;
}
template <int L>
__device__ __forceinline__ uint32_t group_sum_u(uint32_t x) {
  static_assert(L <= 32, "a group fits in 32 lanes");
  if constexpr (L >= 32) x += xor_lane<16>(x);
  if constexpr (L >= 16) x += xor_lane<8>(x);
  if constexpr (L >= 8) x += xor_lane<4>(x);
  if constexpr (L >= 4) x += xor_lane<2>(x);
  if constexpr (L >= 2) x += xor_lane<1>(x);
  return x;
}
template <int L>
__device__ __forceinline__ float group_min(float x) {
  static_assert(L <= 32, "a group fits in 32 lanes");
  if constexpr (L >= 32) x = fminf(x, __uint_as_float(xor_lane<16>(__float_as_uint(x))));
  if constexpr (L >= 16) x = fminf(x, __uint_as_float(xor_lane<8>(__float_as_uint(x))));
  if constexpr (L >= 8) x = fminf(x, __uint_as_float(xor_lane<4>(__float_as_uint(x))));
  if constexpr (L >= 4) x = fminf(x, __uint_as_float(xor_lane<2>(__float_as_uint(x))));
  if constexpr (L >= 2) x = fminf(x, __uint_as_float(xor_lane<1>(__float_as_uint(x))));
  return x;
}

// First time step (Eq. 29 with v = 0): minimum over the domain's slots, every lane gets it.
__device__ __forceinline__ float read_dt1(const uint32_t *slots) {
  float v = __uint_as_float(slots[threadIdx.x & (kDtSlots - 1)]);
  for (int off = kWave / 2; off > 0; off >>= 1) v = fminf(v, __shfl_xor(v, off, kWave));
  v = v < INFINITY ? v : 0.f;
  // the same value in every lane: held as a wave-uniform (scalar) value
  return __uint_as_float(__builtin_amdgcn_readfirstlane(__float_as_uint(v)));
}

}  // namespace mpsph
