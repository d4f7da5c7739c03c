// Relaxation step of the multi-phase SPH mesh generator (Ji, Fu, Hu & Adams, arXiv 1906.07925)
// on MI355X / gfx950.  The C ABI is declared in include/mpsph.h.
//
// A context holds one or more independent domains of the same dimension (a batch).  Domains
// occupy contiguous ranges of every particle array and of the global cell index space, so one
// launch of each kernel serves all of them; kernels read their domain's parameters from a device
// table.  The step counter lives on the device, so a captured step can be replayed.
//
// Data layout (HBM, structure of arrays, n particles over all domains):
//   state  (order of the previous step's sort): key u32 (domain cell base + packed cell), off
//          float4 (cell offsets), ct u32 (type | colour << 2), id u32 (index at load)
//   work   (order of this step's sort): key u32, pos float4 (offsets, h), jaux u32
//          (colour | cx << 16 | type << 30), id u32
//   per step: acc float4 (a, e = rho_t nu_coeff r_c |a|), cell table u32[ncells+1]; rho, sum|term|,
//             a~, v, dr, nearest distance only in debug mode
// Positions are an integer cell coordinate per axis (packed in the key: x fastest and at
// sub-cell resolution, 3D rows numbered in tiles by row_index) plus a float offset in [0, 1) in
// cell units, so pair separations are formed from exact integer differences plus differences of
// numbers below one.  Lengths inside the kernels are
// in cell units; accelerations and velocities are the domain values divided by the cell size
// (time is unchanged; the EOS constant is scaled by cs^(d-2) to make this exact).
//
// Launch sequence of one step (all on the context stream, no host synchronisation):
//   radix sort of the keys (3 kernels per digit of at most 8 bits)
//   reorder_field   gather the state in key order, evaluate the target field (Eq. 1-2, 16), fill
//                   the cell table
//   pass_density_force  density (Eq. 17), pressure + surface tension (Eq. 18-19, 23-25),
//                   projection (Eq. 30-31), first time step (Eq. 29, block minima); like the
//                   viscous pass, a lane group per particle walks its candidates through a row
//                   table in LDS (scan_group_table in pair_scan.h)
//   pass_viscous_integrate  mid-point velocity (Eq. 26), viscosity (Eq. 21-22), viscous
//                   acceleration (Eq. 20), second time step (Eq. 29), velocity (Eq. 27), drift
//                   (Eq. 28), feature projection and re-tagging (Eq. 32)
//   reduce_partials, finalize   FP64 reduction of the per-block partials in a fixed order
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "mpsph.h"
#include "mpsph_device.h"
#include "adjoint.h"
#include "pair_scan.h"
#include "sort.h"

using namespace mpsph;

namespace {

// ------------------------------------------------------------------------------------------
// Kernels
// ------------------------------------------------------------------------------------------

// Domain units -> (cell, offset) in FP64 (identical inputs give identical keys), validation.
// Internal particles [i0, i1) of one dimension group.
template <int D>
__global__ __launch_bounds__(kBlock) void load_kernel(const DomDev *__restrict__ doms, int ndom, int i0, int i1,
                                                      const float *__restrict__ pos, const int32_t *__restrict__ colour,
                                                      const int32_t *__restrict__ type, uint32_t *__restrict__ key,
                                                      float4 *__restrict__ off, uint32_t *__restrict__ ct,
                                                      uint32_t *__restrict__ id, int *__restrict__ bad) {
  const int i = i0 + blockIdx.x * kBlock + threadIdx.x;
  if (i >= i1) return;
  const DomDev &dd = doms[domain_of(doms, ndom, i)];
  const int local = i - dd.off;
  const int u = dd.uoff + local;
  const float *x = pos + dd.xoff + (int64_t)local * D;
  int c[3] = {0, 0, 0};
  float o[3] = {0.f, 0.f, 0.f};
  bool ok = true;
  for (int a = 0; a < D; ++a) {
    double X = ((double)x[a] - dd.lo[a]) * dd.inv_cs;
    if (!(X >= 0.0 && X <= dd.xhi[a])) ok = false;
    if (dd.g.geometry == 0 && X >= dd.xhi[a]) X -= dd.xhi[a];   // periodic: hi is lo
    double f = floor(X);
    float fo = (float)(X - f);
    if (fo >= 1.0f) {
      fo = 0.0f;
      f += 1.0;
    }
    if (!(f >= 0.0 && f <= (double)dd.g.gmax)) ok = false;
    c[a] = ok ? (int)f : 0;
    o[a] = ok ? fo : 0.f;
  }
  const int col = colour[u];
  const int t = type ? type[u] : 0;
  if (col < 0 || col >= (1 << 16) || t < 0 || t > 3) ok = false;
  if (!ok) atomicOr(bad, 1);
  key[i] = dd.cellbase + pack_key<D>(c, o, dd.g);
  off[i] = make_float4(o[0], o[1], D == 3 ? o[2] : 0.f, 0.f);
  ct[i] = (uint32_t)(t & 3) | ((uint32_t)col << 2);
  id[i] = (uint32_t)u;
}

// Waves per SIMD the pair kernels are compiled for (their register budget: 64 VGPRs and 96 SGPRs
// at 8 waves); 0 leaves it to the compiler, which otherwise settles at 7 waves.  Measured on the
// 2M-particle graded cube: 8 waves make both pair passes 12-13 % faster.
#ifndef MPSPH_PAIR_WAVES
#define MPSPH_PAIR_WAVES 8
#endif
#if MPSPH_PAIR_WAVES > 0
#define MPSPH_PAIR_OCCUPANCY __attribute__((amdgpu_waves_per_eu(MPSPH_PAIR_WAVES, MPSPH_PAIR_WAVES)))
#else
#define MPSPH_PAIR_OCCUPANCY
#endif

// Empty-cell runs of at least this length are filled by fill_gaps instead of one thread.
constexpr uint32_t kShortGap = 64;
constexpr int kGapBlocks = 256;

// Fills the long empty-cell runs listed by reorder_field: block b takes runs b, b + grid, ...,
// its threads stride over the cells of a run.  The last block to finish resets the list (no
// memset, so the launch can be captured in a graph).
__global__ __launch_bounds__(256) void fill_gaps(const uint4 *__restrict__ gaps, uint32_t *__restrict__ gcount,
                                                 uint32_t *__restrict__ gdone, uint32_t *__restrict__ cstart) {
  const uint32_t cnt = *(volatile uint32_t *)gcount;
  for (uint32_t g = blockIdx.x; g < cnt; g += gridDim.x) {
    const uint4 r = gaps[g];
    for (uint32_t c = r.x + threadIdx.x; c <= r.y; c += blockDim.x) cstart[c] = r.z;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    if (atomicAdd(gdone, 1u) == gridDim.x - 1) {
      *gcount = 0u;
      *gdone = 0u;
    }
  }
}

// Gather the state in sorted order, evaluate the size field (h = tau s, Eq. 16) and build the
// cell table: cstart[c] = first sorted index with key >= c, cstart[ncells] = n.  Sorted keys are
// grouped by domain, so the sorted range of domain d is [off_d, off_d + n_d); one launch covers
// the sorted indices [i0, i1) of one dimension group (and the sentinel i = n if i1 = n).  The
// first nreset threads also reset the time-step slots.
template <int D>
__global__ __launch_bounds__(kBlock) void reorder_field(
    const DomDev *__restrict__ doms, int ndom, int i0, int i1, int n, uint32_t ncells, int nreset,
    const uint32_t *__restrict__ skey, const uint32_t *__restrict__ perm, const float4 *__restrict__ soff,
    const uint32_t *__restrict__ sct, const uint32_t *__restrict__ sid, uint32_t *__restrict__ wkey,
    float4 *__restrict__ wpos, uint32_t *__restrict__ wjaux, uint32_t *__restrict__ wid,
    uint32_t *__restrict__ cstart, uint32_t *__restrict__ dtslots, uint4 *__restrict__ gaps,
    uint32_t *__restrict__ gcount) {
  const int t = blockIdx.x * kBlock + threadIdx.x;
  if (t < nreset) dtslots[t] = kInfBits;
  const int i = i0 + t;
  if (i > i1 || (i == i1 && i1 != n)) return;
  // cells (key[i-1], key[i]] start at sorted index i; the sentinel thread i = n closes the table.
  // Long runs of empty cells (regions without particles) go to a list that fill_gaps spreads
  // over many threads.
  const uint32_t lo = i == 0 ? 0u : skey[i - 1] + 1u;
  const uint32_t hi = i == n ? ncells : min(skey[i], ncells);
  if (hi >= lo && hi - lo >= kShortGap) {
    const uint32_t slot = atomicAdd(gcount, 1u);
    gaps[slot] = make_uint4(lo, hi, (uint32_t)i, 0u);
  } else {
    for (uint32_t c = lo; c <= hi; ++c) cstart[c] = (uint32_t)i;
  }
  if (i == n) return;
  const DomDev &dd = doms[domain_of(doms, ndom, i)];
  const uint32_t s = perm[i];
  const uint32_t key = skey[i];
  const float4 o4 = soff[s];
  const uint32_t ct = sct[s];
  int c[3];
  unpack_key<D>(key - dd.cellbase, dd.g, c);
  const float o[3] = {o4.x, o4.y, o4.z};
  const float spc = field_spacing<D>(dd.f, c, o);
  wkey[i] = key;
  wpos[i] = make_float4(o4.x, o4.y, o4.z, dd.sp.tau * spc);
  wjaux[i] = pack_aux((uint32_t)c[0], ct & 3u, ct >> 2);
  wid[i] = sid[s];
}

// Pass 1: density (Eq. 17, self term included, radius kappa h_i) and
//   a_i = -sum_j (1 + beta_ij) (P_i + P_j) dW(r_ij, h_ij)/dr e_ij   (Eq. 18, 23; gamma = 2, Eq. 19)
// with e_ij = r_ij / |r_ij|, r_ij = r_i - r_j, beta_ij = sigma for different colours (Eq. 24),
// P = p0 / rho_t^2, h_ij = (h_i + h_j)/2, over j with r_ij < kappa h_ij that particle i feels.
// Writes acc = (a after the force mapping of Eq. 30-31, e_i) with e_i = rho_t nu_coeff r_c |a_i|,
// the viscosity of Eq. 21-22 per unit of dt1/2, and the first time-step candidate (Eq. 29).
// L lanes per particle (group) sum its pairs; the block's first 256/L threads then finish one
// particle each (the epilogue) and the first wave combines the block's metric partials.
// LDS-staged density pass (3D; pair-kernel variant MPSPH_PAIRS_TILE): the targets of a block share one
// copy of their neighbours in LDS.  The union of the targets' candidate rows (y, z) and, per row,
// of their x-runs is formed with LDS atomics; every union row's particles (offsets and h, flags)
// are copied into LDS once; the targets' row tables then index that copy.  A block whose union
// has more than kTileRows rows or MPSPH_TILE_CAP particles reads its neighbours from global memory.
// Staged particles per block.  Measured on the 2M-particle graded cube (2^6 cells, 8 lanes):
// 768 particles (39 KB of LDS per block with the row table, 4 waves per SIMD) 2.38 ms per density
// pass, 1536 (54 KB, 3 waves) 4.33 ms, against 1.43 ms for the pass that reads its neighbours
// through the caches at 8 waves per SIMD.
#ifndef MPSPH_TILE_CAP
#define MPSPH_TILE_CAP 768
#endif
constexpr int kTileRows = kBlock;
struct TileLds {
  int y0, y1, z0, z1;
  int ux0[kTileRows], ux1[kTileRows];        // union x-run of each row (x sub-cells)
  uint32_t ra[kTileRows];                    // global index of the first staged particle of a row
  uint32_t roff[kTileRows + 1];              // LDS index of a row's first particle; roff[rows] = total
  float4 pos[MPSPH_TILE_CAP];
  uint32_t aux[MPSPH_TILE_CAP];
};
struct TileRemap {
  const TileLds *T;
  int w;   // rows per z of the union
  __device__ __forceinline__ uint32_t operator()(int cy, int cz, uint32_t a) const {
    const int r = (cz - T->z0) * w + (cy - T->y0);
    return T->roff[r] + (a - T->ra[r]);
  }
};

// Exclusive prefix sum over the block's threads; *total receives the sum (every thread).
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t *total) {
  __shared__ uint32_t wsum[kBlock / kWave];
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
  uint32_t incl = v;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const uint32_t t = __shfl_up(incl, o, kWave);
    if (lane >= o) incl += t;
  }
  if (lane == kWave - 1) wsum[w] = incl;
  __syncthreads();
  uint32_t base = 0, tot = 0;
#pragma unroll
  for (int k = 0; k < kBlock / kWave; ++k) {
    if (k < w) base += wsum[k];
    tot += wsum[k];
  }
  __syncthreads();
  *total = tot;
  return base + incl - v;
}

// Stages the neighbours of the block's targets (3D, no periodic wrap); the rows and x-runs are
// those of scan_group_table.  Called by every thread of the block; returns the same value in
// every thread (false: the union does not fit).
template <int L>
__device__ bool stage_tile(TileLds *T, bool active, int sub, const int *ci, const float *oi, float rs,
                           const GridDev &g, uint32_t cellbase, const uint32_t *__restrict__ cstart,
                           const float4 *__restrict__ wpos, const uint32_t *__restrict__ wjaux) {
  rs = fminf(fmaxf(rs, 0.f), 2.f * (float)g.gmax + 2.f);
  const float rs2 = rs * rs;
  int y0 = 0, y1 = -1, z0 = 0, z1 = -1;
  if (active) {
    z0 = max(0, ci[2] + (int)floorf(oi[2] - rs));
    z1 = min(g.gmax, ci[2] + (int)floorf(oi[2] + rs));
    y0 = max(0, ci[1] + (int)floorf(oi[1] - rs));
    y1 = min(g.gmax, ci[1] + (int)floorf(oi[1] + rs));
  }
  if (threadIdx.x == 0) {
    T->y0 = INT_MAX;
    T->y1 = -1;
    T->z0 = INT_MAX;
    T->z1 = -1;
  }
  __syncthreads();
  if (active && sub == 0) {
    atomicMin(&T->y0, y0);
    atomicMax(&T->y1, y1);
    atomicMin(&T->z0, z0);
    atomicMax(&T->z1, z1);
  }
  __syncthreads();
  const int W = T->y1 - T->y0 + 1, H = T->z1 - T->z0 + 1;
  const int nr = T->y1 >= 0 ? W * H : 0;
  if (nr > kTileRows) return false;
  for (int r = threadIdx.x; r < nr; r += kBlock) {
    T->ux0[r] = INT_MAX;
    T->ux1[r] = -1;
  }
  __syncthreads();
  const float fx = (float)(1u << g.xe);
  const int xlast = ((g.gmax + 1) << g.xe) - 1;
  if (active) {
    const int ny = y1 - y0 + 1, nrows = ny * (z1 - z0 + 1);
    for (int q = sub; q < nrows; q += L) {
      const int cz = z0 + q / ny, cy = y0 + q % ny;
      const float lz = (float)(cz - ci[2]) - oi[2], hz = lz + 1.f;
      const float ez = lz > 0.f ? lz : (hz < 0.f ? -hz : 0.f);
      const float ly = (float)(cy - ci[1]) - oi[1], hy = ly + 1.f;
      const float ey = ly > 0.f ? ly : (hy < 0.f ? -hy : 0.f);
      const float d2 = ey * ey + ez * ez;
      if (d2 < rs2) {
        const float wx = fast_sqrt(fmaxf(rs2 - d2, 0.f));
        const int x0 = max(0, (ci[0] << g.xe) + (int)floorf((oi[0] - wx) * fx));
        const int x1 = min(xlast, (ci[0] << g.xe) + (int)floorf((oi[0] + wx) * fx));
        const int r = (cz - T->z0) * W + (cy - T->y0);
        atomicMin(&T->ux0[r], x0);
        atomicMax(&T->ux1[r], x1);
      }
    }
  }
  __syncthreads();
  // global range of each union row (one thread per row), LDS offsets by a prefix sum
  uint32_t a = 0u, cnt = 0u;
  const int r = threadIdx.x;
  if (r < nr && T->ux1[r] >= 0) {
    const int cy = T->y0 + r % W, cz = T->z0 + r / W;
    const int x0 = T->ux0[r], x1 = T->ux1[r];
    const uint32_t kb = cellbase + ((uint32_t)x0 | (row_index(cy, cz, g) << (g.k + g.xe)));
    a = cstart[kb];
    const uint32_t b = min(cstart[kb + (uint32_t)(x1 - x0) + 1u], (uint32_t)g.n);
    cnt = b > a ? b - a : 0u;
  }
  uint32_t total;
  const uint32_t off = block_exclusive_scan(cnt, &total);
  if (r < nr) {
    T->ra[r] = a;
    T->roff[r] = off;
  }
  if (threadIdx.x == 0) T->roff[nr] = total;
  __syncthreads();
  if (total > (uint32_t)MPSPH_TILE_CAP) return false;
  for (uint32_t s = threadIdx.x; s < total; s += kBlock) {
    // the row holding staged slot s: the last row whose offset is <= s (never an empty row)
    int lo = 0, hi = nr - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (T->roff[mid] <= s) lo = mid;
      else hi = mid - 1;
    }
    const uint32_t j = T->ra[lo] + (s - T->roff[lo]);
    T->pos[s] = wpos[j];
    T->aux[s] = wjaux[j];
  }
  __syncthreads();
  return true;
}

// One logical block lb of the pass (blocks of a domain are consecutive; doms is the table the
// block numbers refer to); rowtab is the block's LDS row table, tile the LDS copy of the
// neighbours of the TILE variant (unused otherwise).  With PIPE the scan issues the neighbour
// loads of a lane's next slot before the arithmetic of the current one (same arithmetic, same
// order: the results do not depend on it).  The single-domain passes take it except in 3D
// periodic boxes, where the minimum image's extra registers would spill; the persistent and
// staged variants keep the one-round body.
#define MPSPH_PASS1_PARAMS                                                                                   \
  const DomDev *__restrict__ doms, int ndom, const int64_t *__restrict__ stepctr,                            \
      const uint32_t *__restrict__ wkey, const float4 *__restrict__ wpos, const uint32_t *__restrict__ wjaux, \
      const uint32_t *__restrict__ cstart, float4 *__restrict__ acc, float *__restrict__ rho_out,           \
      float *__restrict__ nn_out, float *__restrict__ aabs_out, uint32_t *__restrict__ dtslots,             \
      const double *__restrict__ metrics, double *__restrict__ partials
#define MPSPH_PASS1_ARGS \
  doms, ndom, stepctr, wkey, wpos, wjaux, cstart, acc, rho_out, nn_out, aabs_out, dtslots, metrics, partials
template <int D, int L, bool PER, bool DBG, bool TILE, bool PIPE>
__device__ __forceinline__ void density_force_block(int lb, uint4 *rowtab, TileLds *tile, MPSPH_PASS1_PARAMS) {
  const int d = domain_of_block(doms, ndom, lb);
  const GridDev g = doms[d].g;
  const StepDev sp = doms[d].sp;
  const uint32_t cellbase = doms[d].cellbase;
  const int local = (lb - doms[d].blk0) * kBlock + threadIdx.x;
  const int li = local / L, sub = local % L;
  const int i = doms[d].off + li;
  const bool active = li < doms[d].n;
  const float sigma = sigma_of(sp, (float)*stepctr, metrics[(size_t)d * 32 + kAutoT0]);
  // the group's sums (wsum, a, nearest distance, counts), valid in lane 0 of each group
  float gw = 0.f, gx = 0.f, gy = 0.f, gz = 0.f, gA = 0.f, gn = INFINITY;
  uint32_t gp = 0u, gi = 0u, gc = 0u;
  bool staged = false;
  uint32_t self_t = 0u;
  int tw = 0;
  if constexpr (TILE) {
    static_assert(D == 3 && !PER, "the staged variant covers 3D regions without periodic wrap");
    int cs[3] = {0, 0, 0};
    float os[3] = {0.f, 0.f, 0.f};
    float rst = 0.f;
    if (active) {
      unpack_key<D>(wkey[i] - cellbase, g, cs);
      const float4 p4 = wpos[i];
      os[0] = p4.x;
      os[1] = p4.y;
      os[2] = p4.z;
      rst = fminf(sp.search_fac * p4.w, sp.kappa * 0.5f * (p4.w + sp.hmax)) * 1.0001f;
    }
    staged = stage_tile<L>(tile, active, sub, cs, os, rst, g, cellbase, cstart, wpos, wjaux);
    if (staged) {
      tw = tile->y1 - tile->y0 + 1;
      if (active) {
        const int r = (cs[2] - tile->z0) * tw + (cs[1] - tile->y0);
        self_t = tile->roff[r] + ((uint32_t)i - tile->ra[r]);
      }
    }
  }
  if (active) {
    int ci[3];
    unpack_key<D>(wkey[i] - cellbase, g, ci);
    const float4 pi = wpos[i];
    const float oi[3] = {pi.x, pi.y, pi.z};
    const uint32_t ai = wjaux[i];
    const int ti = aux_type(ai);
    const float hi = pi.w;
    // P = p0 / rho_t^2 = p0 tau^-2d h^2d and -dW/dr / r = 5 alpha 2^(d+2) (h_i + h_j)^-(d+2) (1 - q/2)^3
    // for the pair's h_ij: the pair sum takes h^2d and (h_i + h_j)^-(d+2), and the factors
    // common to every pair are applied once to the group's total
    const float Phi = powd<D>(hi * hi);
    const float fscale = sp.p0c * powd<D>(sp.inv_tau * sp.inv_tau) * (5.f * sp.alpha) * (D == 3 ? 32.f : 16.f);
    const float ihi = fast_rcp(hi);
    const float rci = sp.kappa * hi, rci2 = rci * rci;
    const float rs = fminf(sp.search_fac * hi, sp.kappa * 0.5f * (hi + sp.hmax)) * 1.0001f;
    const float kh = 0.5f * sp.kappa;
    const float opb = 1.f + sigma;
    float wsum = 0.f, ax = 0.f, ay = 0.f, az = 0.f, A = 0.f, nn2 = INFINITY;
    uint32_t npair = 0, nifc = 0;
    const BufRes rpos = buf_res(wpos, 16, (uint32_t)g.n), raux = buf_res(wjaux, 4, (uint32_t)g.n);
    const auto pair = [&](const float4 pj, const uint32_t aj, float dy0, float dz0, bool v) {
      const float dx = sep_x<PER, D>(g, (float)ci[0], aj, oi[0], pj.x);
      const float dy = dy0 - pj.y;
      float r2 = dx * dx + dy * dy;
      float dz = 0.f;
      if constexpr (D == 3) {
        dz = dz0 - pj.z;
        r2 += dz * dz;
      }
      const float hs = hi + pj.w;                   // 2 h_ij
      const float hij = kh * hs;                    // kappa h_ij
      const bool dens = v && r2 < rci2;
      const bool inter = v && r2 < hij * hij;
      // the counts and the nearest distance in every lane, so that the branch below is taken
      // only for the kernel sums
      const bool diff = colour_differs(aj, ai);
      const bool feel = inter && type_at_least(aj, ti);
      nifc += (inter && diff) ? 1u : 0u;
      npair += feel ? 1u : 0u;
      // an empty statement that reads and writes both counts keeps their additions here, beside
      // the compares, where each becomes one add-with-carry of the compare's lane mask instead
      // of a select and an add after the branch
      asm volatile("" : "+v"(npair), "+v"(nifc));
      if (inter && r2 < nn2) nn2 = r2;
      // coincident particles (two particles clamped into one corner): r = 0, no direction
      const bool apart = r2 > 1e-30f;
      const bool force = feel && apart;
      if (!(dens || force)) return;
      const float r = fast_sqrt(r2);
      if (dens) {
        const float q = r * ihi, u = fmaf(-0.5f, q, 1.f), u2 = u * u;
        wsum += u2 * u2 * fmaf(2.f, q, 1.f);
      }
      if (!force) return;
      const float hj2 = pj.w * pj.w;
      // (P_i + P_j) (-dW/dr / r) over the common factor fscale (>= 0)
      const float s = (diff ? opb : 1.f) * powd_add<D>(hj2, Phi) * kernel_slope_factor<D>(r, fast_rcp(hs));
      ax = fmaf(s, dx, ax);
      ay = fmaf(s, dy, ay);
      az = fmaf(s, dz, az);
      if constexpr (DBG) A = fmaf(s, r, A);        // sum of |pair terms| (debug export only)
    };
    struct Nb {
      float4 p;
      uint32_t a;
    };
    const auto body = pair_body<PIPE>([&](uint32_t j) { return Nb{buf_f4(rpos, j), buf_u32(raux, j)}; },
                                      [&](const Nb &nb, float dy0, float dz0, bool v) { pair(nb.p, nb.a, dy0, dz0, v); });
    uint32_t ncand;
    if constexpr (TILE) {
      if (staged) {
        // slots index the LDS copy; an invalid slot reads entry 0
        const auto tbody = [&](uint32_t j, float dy0, float dz0, bool v) {
          const uint32_t jc = v ? j : 0u;
          pair(tile->pos[jc], tile->aux[jc], dy0, dz0, v);
        };
        ncand = scan_group_table<D, L, row_table_rows<L>(), PER>(i, sub, rowtab + threadIdx.x / L,
                                                                 row_table_stride<L>(), ci, oi, rs, g, cellbase,
                                                                 cstart, tbody, TileRemap{tile, tw}, self_t);
      } else {
        ncand = scan_group_table<D, L, row_table_rows<L>(), PER>(
            i, sub, rowtab + threadIdx.x / L, row_table_stride<L>(), ci, oi, rs, g, cellbase, cstart, body);
      }
    } else {
      ncand = scan_group_table<D, L, row_table_rows<L>(), PER>(
          i, sub, rowtab + threadIdx.x / L, row_table_stride<L>(), ci, oi, rs, g, cellbase, cstart, body);
    }
    gw = group_sum<L>(wsum);
    gx = fscale * group_sum<L>(ax);
    gy = fscale * group_sum<L>(ay);
    if constexpr (D == 3) gz = fscale * group_sum<L>(az);
    if constexpr (DBG) gA = fscale * group_sum<L>(A);
    gn = group_min<L>(nn2);
    gp = group_sum_u<L>(npair);
    gi = group_sum_u<L>(nifc);
    gc = ncand;
  }
  // Per-particle epilogue at one thread per particle: the groups' sums pass through the row
  // table's LDS to the block's first P threads, so that the epilogue does not run in every wave
  // with one lane in L busy.
  constexpr int P = kBlock / L;                  // particles per block
  constexpr int kEp = DBG ? 9 : 8;               // values per particle
  float *ep = reinterpret_cast<float *>(rowtab);
  __syncthreads();                               // every wave is done with the row table
  if (active && sub == 0) {
    const int p = threadIdx.x / L;
    ep[0 * P + p] = gw;
    ep[1 * P + p] = gx;
    ep[2 * P + p] = gy;
    ep[3 * P + p] = gz;
    ep[4 * P + p] = gn;
    ep[5 * P + p] = __uint_as_float(gp);
    ep[6 * P + p] = __uint_as_float(gi);
    ep[7 * P + p] = __uint_as_float(gc);
    if constexpr (DBG) ep[8 * P + p] = gA;
  }
  __syncthreads();
  double red[14];                                // the metrics' partials, interface flag, time-step candidate
#pragma unroll
  for (int s = 0; s < 14; ++s) red[s] = 0.0;
  red[P_ELRMIN] = INFINITY;
  red[13] = INFINITY;
  const int lp = (lb - doms[d].blk0) * P + (int)threadIdx.x;   // the thread's particle of the domain
  if (threadIdx.x < P && lp < doms[d].n) {
    const int ip = doms[d].off + lp;
    const int p = threadIdx.x;
    int ci[3];
    unpack_key<D>(wkey[ip] - cellbase, g, ci);
    const float4 pi = wpos[ip];
    const float oi[3] = {pi.x, pi.y, pi.z};
    const int ti = aux_type(wjaux[ip]);
    const float hi = pi.w, ihi = fast_rcp(hi), si = hi * sp.inv_tau, rci = sp.kappa * hi;
    const float wsum = ep[0 * P + p], nn2 = ep[4 * P + p];
    const uint32_t npair = __float_as_uint(ep[5 * P + p]), nifc = __float_as_uint(ep[6 * P + p]);
    const uint32_t ncand = __float_as_uint(ep[7 * P + p]);
    const float ihd = D == 3 ? ihi * ihi * ihi : ihi * ihi;
    const float rho = sp.alpha * ihd * (1.f + wsum);
    float a[3] = {ep[1 * P + p], ep[2 * P + p], ep[3 * P + p]};
    project_feature<D>(g, ti, ci, oi, a);
    const float am2 = a[0] * a[0] + a[1] * a[1] + (D == 3 ? a[2] * a[2] : 0.f);
    // the hardware square roots below (about 1 ulp) are well inside the step's FP32 error
    const float am = fast_sqrt(am2);
    const float ehat = sp.nu_coeff * rci * am / powd<D>(si);  // rho_t nu_coeff r_c |a|
    acc[ip] = make_float4(a[0], a[1], D == 3 ? a[2] : 0.f, ehat);
    if (rho_out) rho_out[ip] = rho;
    if (nn_out) nn_out[ip] = sqrtf(nn2);
    if constexpr (DBG) {
      if (aabs_out) aabs_out[ip] = ep[8 * P + p];
    }
    if (ti != 3 && am2 > 0.f) red[13] = (double)(sp.c_acc * fast_sqrt(rci * fast_rsq(am2)));
    const bool fin = isfinite(am2) && isfinite(rho);
    if (ti == 0) {
      const double e = (double)(rho * powd<D>(si)) - 1.0;   // rho / rho_t - 1
      red[P_E2] = e * e;
      red[P_EMAX] = fabs(e);
      red[P_NNORM] = 1.0;
      if (nn2 < INFINITY) {
        const double elr = (double)fast_sqrt(nn2) / (double)si;
        red[P_ELR] = elr;
        red[P_ELR2] = elr * elr;
        red[P_ELRMIN] = elr;
        red[P_ELRMAX] = elr;
        red[P_NELR] = 1.0;
      }
    }
    red[P_PAIRS] = (double)npair;
    red[P_IFC] = (double)nifc;
    red[P_CAND] = (double)ncand;
    red[P_NONFIN1] = fin ? 0.0 : 1.0;
    red[12] = nifc > 0 ? 1.0 : 0.0;
  }
  // block results through LDS (after the epilogue's values when both fit in the row table)
  constexpr size_t kEpBytes = (size_t)kEp * P * sizeof(float), kRedBytes = (size_t)(P + 1) * 14 * sizeof(double);
  constexpr size_t kTableBytes = (size_t)row_table_rows<L>() * row_table_stride<L>() * sizeof(uint4);
  constexpr bool kApart = kEpBytes + kRedBytes <= kTableBytes;
  static_assert(kRedBytes <= kTableBytes && kEpBytes <= kTableBytes, "the epilogue and the reduction fit in the row table");
  double *rb = reinterpret_cast<double *>(reinterpret_cast<char *>(rowtab) + (kApart ? (kEpBytes + 15) / 16 * 16 : 0));
  constexpr uint32_t kMinSlots = (1u << P_ELRMIN) | (1u << 13), kMaxSlots = (1u << P_EMAX) | (1u << P_ELRMAX);
  double *out = partials + (size_t)lb * kNumPartials;
  block_reduce_lds<14, P, !kApart>(red, threadIdx.x < P ? (int)threadIdx.x : -1, kMinSlots, kMaxSlots, rb,
                                   [&](int s, double x) {
    if (s < 12) out[s] = x;
    else if (s == 12) out[P_IFCP] = x;
    else if (x < INFINITY) atomic_min_pos(&dtslots[d * kDtSlots + (lb & (kDtSlots - 1))], (float)x);   // one atomic per block
  });
}

// The pass over the logical blocks b0 + [0, gridDim.x) (one dimension group).
template <int D, int L, bool PER, bool DBG>
__global__ __launch_bounds__(kBlock) MPSPH_PAIR_OCCUPANCY void pass_density_force(int b0, MPSPH_PASS1_PARAMS) {
  __shared__ uint4 rowtab[row_table_rows<L>() * row_table_stride<L>()];
  density_force_block<D, L, PER, DBG, false, !PER || D == 2>(b0 + xcd_block(blockIdx.x, gridDim.x), rowtab, nullptr, MPSPH_PASS1_ARGS);
}

// The staged copy limits a CU to 4 blocks (4 waves per SIMD), which the register budget follows.
template <int L, bool DBG>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(4, 4))) void pass_density_force_tile(
    int b0, MPSPH_PASS1_PARAMS) {
  __shared__ uint4 rowtab[row_table_rows<L>() * row_table_stride<L>()];
  __shared__ TileLds tile;
  density_force_block<3, L, false, DBG, true, false>(b0 + xcd_block(blockIdx.x, gridDim.x), rowtab, &tile, MPSPH_PASS1_ARGS);
}


// Box type from the number of faces a particle lies on.
// Mirror image through the lower wall (X = c + o < 0  ->  -X), in (cell, offset) form.
__device__ __forceinline__ void mirror_low(int &c, float &o) {
  int cn = -c - 1;
  float on = 1.f - o;
  if (on >= 1.f) {
    on = 0.f;
    cn += 1;
  }
  c = cn;
  o = on;
}

// Mirror image through the upper wall W = wc + wo (X = c + o > W  ->  2 W - X).
__device__ __forceinline__ void mirror_high(int &c, float &o, int wc, float wo) {
  const float x = wo - ((float)(c - wc) + (o - wo));
  const float fl = floorf(x);
  c = wc + (int)fl;
  o = x - fl;
  if (o >= 1.f) {
    o = 0.f;
    c += 1;
  }
}

__device__ __forceinline__ int type_from_faces(int nf, int d) {
  return nf <= 0 ? 0 : (nf == 1 ? 1 : (nf == 2 ? (d == 3 ? 2 : 3) : 3));
}

// Pass 2: viscous acceleration (Eq. 20 with rho = rho_t, Eq. 22)
//   a~_i = sum_j [2 eta_i eta_j / (eta_i + eta_j)] (1/rho_t,i^2 + 1/rho_t,j^2) dW(r_ij,h_ij)/dr v~_ij / r_ij
// over the same pairs as pass 1, with the mid-point velocity v~ = a dt1 / 2 (Eq. 26 after the
// velocity reset) and eta = rho_t nu_coeff r_c |v~| (Eq. 21-22) formed from pass 1's output.
// Then per particle: projection, v = v~ + a~ dt2 / 2 (Eq. 27), drift r += v dt2 (Eq. 28),
// feature projection / re-tagging (Eq. 32); the new state is written in this step's order.
// With v~ = a dt1/2 the three criteria of Eq. 29 are increasing functions of r_c/|a| and give
// dt2 = dt1 min(1, 2 min(c_vel, c_visc / nu_coeff) / c_acc^2) (sp.dt2_factor).
#define MPSPH_PASS2_PARAMS                                                                                    \
  const DomDev *__restrict__ doms, int ndom, const uint32_t *__restrict__ wkey, const float4 *__restrict__ wpos, \
      const uint32_t *__restrict__ wjaux, const uint32_t *__restrict__ wid, const uint32_t *__restrict__ cstart,  \
      const float4 *__restrict__ acc, const uint32_t *__restrict__ dtslots, uint32_t *__restrict__ skey,         \
      float4 *__restrict__ soff, uint32_t *__restrict__ sct, uint32_t *__restrict__ sid, float4 *__restrict__ at_out, \
      float4 *__restrict__ v_out, float4 *__restrict__ dr_out, double *__restrict__ partials
#define MPSPH_PASS2_ARGS \
  doms, ndom, wkey, wpos, wjaux, wid, cstart, acc, dtslots, skey, soff, sct, sid, at_out, v_out, dr_out, partials
// One logical block lb of the pass; PIPE as for density_force_block.
template <int D, int L, bool PER, bool PIPE>
__device__ __forceinline__ void viscous_integrate_block(int lb, uint4 *rowtab, MPSPH_PASS2_PARAMS) {
  const int d = domain_of_block(doms, ndom, lb);
  const GridDev g = doms[d].g;
  const StepDev sp = doms[d].sp;
  const uint32_t cellbase = doms[d].cellbase;
  const int local = (lb - doms[d].blk0) * kBlock + threadIdx.x;
  const int li = local / L, sub = local % L;
  const int i = doms[d].off + li;
  float gbx = 0.f, gby = 0.f, gbz = 0.f;   // the group's pair sums, valid in lane 0 of each group
  // dt1 is published in LDS and read again after the pair sum, so that no copy of it stays live
  // across the pair loop
  __shared__ float sdt1;
  const float dt1 = read_dt1(dtslots + d * kDtSlots);
  if (threadIdx.x == 0) sdt1 = dt1;
  __syncthreads();
  if (li < doms[d].n) {
    float bx = 0.f, by = 0.f, bz = 0.f;
    {
      // the pair sum; the particle's own data is scoped to it (the epilogue reads it again)
      int ci[3];
      unpack_key<D>(wkey[i] - cellbase, g, ci);
      const float4 pi = wpos[i];
      const float oi[3] = {pi.x, pi.y, pi.z};
      const int ti = aux_type(wjaux[i]);
      const float hi = pi.w;
      // 1 / rho_t^2 = tau^-2d h^2d, v = (dt1/2) a, eta = (dt1/2) e and dW/dr / r =
      // -5 alpha 2^(d+2) (h_i + h_j)^-(d+2) (1 - q/2)^3 for the pair's h_ij: the pair sum takes h^2d,
      // a, e and (h_i + h_j)^-(d+2), and the factors common to every pair are applied once to the
      // group's total
      const float invi = powd<D>(hi * hi);
      const float4 acci = acc[i];
      const float ei = (0.5f * dt1) * acci.w;
      const float rs = fminf(sp.search_fac * hi, sp.kappa * 0.5f * (hi + sp.hmax)) * 1.0001f;
      const float kh = 0.5f * sp.kappa;
      // with eta_i = 0 every harmonic-mean viscosity of particle i vanishes: nothing to sum
      if (ei > 0.f) {
        const BufRes rpos = buf_res(wpos, 16, (uint32_t)g.n), raux = buf_res(wjaux, 4, (uint32_t)g.n);
        const BufRes racc = buf_res(acc, 16, (uint32_t)g.n);
        struct Nb {
          float4 p, acc;
          uint32_t a;
        };
        const auto fetch = [&](uint32_t j) { return Nb{buf_f4(rpos, j), buf_f4(racc, j), buf_u32(raux, j)}; };
        const auto use = [&](const Nb &nb, float dy0, float dz0, bool) {
          const float4 pj = nb.p, accj = nb.acc;
          const uint32_t aj = nb.a;
          const float dx = sep_x<PER, D>(g, (float)ci[0], aj, oi[0], pj.x);
          const float dy = dy0 - pj.y;
          float r2 = dx * dx + dy * dy;
          if constexpr (D == 3) {
            const float dz = dz0 - pj.z;
            r2 += dz * dz;
          }
          const float hs = hi + pj.w;   // 2 h_ij
          const float hij = kh * hs;
          // the particle itself (r = 0 exactly: its own offsets are subtracted from themselves)
          // and coincident particles fail r^2 > 0, so the slot's self flag v is not needed
          if (!(r2 > 1e-30f && r2 < hij * hij && type_at_least(aj, ti))) return;
          const float r = fast_sqrt(r2);
          // e_j / (e_i + e_j): half the harmonic mean e_i e_j / (e_i + e_j) over e_i, which
          // multiplies the sum once; e_i > 0 here and e_j >= 0, so the sum is positive
          const float eh = accj.w * fast_rcp(acci.w + accj.w);
          const float hj2 = pj.w * pj.w;
          const float s = eh * powd_add<D>(hj2, invi) * kernel_slope_factor<D>(r, fast_rcp(hs));
          bx = fmaf(s, acci.x - accj.x, bx);
          by = fmaf(s, acci.y - accj.y, by);
          if constexpr (D == 3) bz = fmaf(s, acci.z - accj.z, bz);
        };
        scan_group_table<D, L, row_table_rows<L>(), PER, false>(i, sub, rowtab + threadIdx.x / L,
                                                                 row_table_stride<L>(), ci, oi, rs, g, cellbase, cstart,
                                                                 pair_body<PIPE>(fetch, use));
        // the factor e_i of every pair term
        bx *= acci.w;
        by *= acci.w;
        bz *= acci.w;
      }
    }
    gbx = group_sum<L>(bx);
    gby = group_sum<L>(by);
    if constexpr (D == 3) gbz = group_sum<L>(bz);
  }
  // Per-particle epilogue at one thread per particle: the groups' sums pass through the row
  // table's LDS to the block's first P threads, so that the epilogue does not run in every wave
  // with one lane in L busy.
  constexpr int P = kBlock / L;                  // particles per block
  float *ep = reinterpret_cast<float *>(rowtab);
  __syncthreads();                               // every wave is done with the row table
  if (li < doms[d].n && sub == 0) {
    const int p = threadIdx.x / L;
    ep[0 * P + p] = gbx;
    ep[1 * P + p] = gby;
    ep[2 * P + p] = gbz;
  }
  __syncthreads();
  double part[3] = {0.0, 0.0, 0.0};
  const int lp = (lb - doms[d].blk0) * P + (int)threadIdx.x;   // the thread's particle of the domain
  if (threadIdx.x < P && lp < doms[d].n) {
    {
      const int io = doms[d].off + lp;
      const int p = threadIdx.x;
      const float hdt = 0.5f * sdt1;
      const float dt2 = sdt1 * sp.dt2_factor;
      // the factors left out of the pair sum: 2 of the harmonic mean, -5 alpha 2^(d+2), tau^-2d and
      // (dt1/2)^2
      const float vscale = (-2.f * 5.f * sp.alpha * (D == 3 ? 32.f : 16.f)) * powd<D>(sp.inv_tau * sp.inv_tau) * hdt * hdt;
      int ci[3];
      unpack_key<D>(wkey[io] - cellbase, g, ci);
      const float4 pe = wpos[io];
      const float oi[3] = {pe.x, pe.y, pe.z};
      const uint32_t ai = wjaux[io];
      int ti = aux_type(ai);
      const float4 acce = acc[io];
      const float vix = hdt * acce.x, viy = hdt * acce.y, viz = hdt * acce.z;
      float b[3] = {vscale * ep[0 * P + p], vscale * ep[1 * P + p], D == 3 ? vscale * ep[2 * P + p] : 0.f};
      project_feature<D>(g, ti, ci, oi, b);
      float v[3] = {vix + 0.5f * b[0] * dt2, viy + 0.5f * b[1] * dt2, viz + 0.5f * b[2] * dt2};
      if (ti == 3) v[0] = v[1] = v[2] = 0.f;
      float dr[3] = {v[0] * dt2, v[1] * dt2, v[2] * dt2};
      float ke = 0.f;
#pragma unroll
      for (int a = 0; a < D; ++a) ke += 0.5f * v[a] * v[a];
      const bool fin = isfinite(b[0]) && isfinite(b[1]) && isfinite(b[2]) && isfinite(dr[0]) && isfinite(dr[1]) &&
                       isfinite(dr[2]);
      // drift in (cell, offset) form with carry
      int c[3] = {ci[0], ci[1], D == 3 ? ci[2] : 0};
      float o[3] = {oi[0], oi[1], D == 3 ? oi[2] : 0.f};
      if (ti != 3 && fin) {
#pragma unroll
        for (int a = 0; a < D; ++a) {
          const float x = o[a] + dr[a];
          const float fl = floorf(x);
          c[a] += (int)fl;
          o[a] = x - fl;
          if (o[a] >= 1.f) {
            o[a] = 0.f;
            c[a] += 1;
          }
        }
        if (PER && g.geometry == 0) {
          // periodic box: wrap into [0, P)
#pragma unroll
          for (int a = 0; a < D; ++a) c[a] = ((c[a] % (g.gmax + 1)) + (g.gmax + 1)) % (g.gmax + 1);
        } else if (g.geometry == 1 && g.seeded) {
          // box with seeded features: a coordinate that left the box is mirrored at the wall it
          // crossed; types never change
#pragma unroll
          for (int a = 0; a < D; ++a) {
            if (c[a] < 0) {
              mirror_low(c[a], o[a]);
              if (c[a] > g.whi_c[a] || (c[a] == g.whi_c[a] && o[a] > g.whi_o[a])) {
                c[a] = g.whi_c[a];
                o[a] = g.whi_o[a];
              }
            } else if (c[a] > g.whi_c[a] || (c[a] == g.whi_c[a] && o[a] > g.whi_o[a])) {
              mirror_high(c[a], o[a], g.whi_c[a], g.whi_o[a]);
              if (c[a] < 0) {
                c[a] = 0;
                o[a] = 0.f;
              }
            }
          }
        } else if (g.geometry == 1) {
          // box: closest-point projection is a clamp to the walls; type from the faces touched
          int nf = 0;
#pragma unroll
          for (int a = 0; a < D; ++a) {
            if (c[a] < 0) {
              c[a] = 0;
              o[a] = 0.f;
            }
            if (c[a] > g.whi_c[a] || (c[a] == g.whi_c[a] && o[a] > g.whi_o[a])) {
              c[a] = g.whi_c[a];
              o[a] = g.whi_o[a];
            }
            if ((c[a] == 0 && o[a] == 0.f) || (c[a] == g.whi_c[a] && o[a] == g.whi_o[a])) ++nf;
          }
          ti = max(ti, type_from_faces(nf, D));
        } else if (g.geometry == 4) {
          // level set on the background mesh: r <- r - phi N (Eq. 32) for feature particles
          // and for normal particles that left the positive phase (re-tagged as surface)
          float gr[3];
          const float phi = mesh_interp<D>(g.phi, g.gn, g.ginv, c, o, gr);
          if (ti != 0 || phi < 0.f) {
            const float gn2 = gr[0] * gr[0] + gr[1] * gr[1] + (D == 3 ? gr[2] * gr[2] : 0.f);
            if (gn2 > 0.f) {
              // seeded features: a normal particle is mirrored through the zero level instead
              const float sc = (g.seeded && ti == 0 ? 2.f : 1.f) * phi * fast_rsq(gn2);
#pragma unroll
              for (int a = 0; a < D; ++a) {
                const float x = o[a] - sc * gr[a];
                const float fl = floorf(x);
                c[a] += (int)fl;
                o[a] = x - fl;
                if (o[a] >= 1.f) {
                  o[a] = 0.f;
                  c[a] += 1;
                }
              }
            }
            if (!g.seeded) ti = max(ti, 1);
          }
        } else {
          // annulus / ball: radial projection onto the nearest boundary circle / sphere
          float rel[3], r2 = 0.f;
#pragma unroll
          for (int a = 0; a < D; ++a) {
            rel[a] = (float)(c[a] - g.gc_c[a]) + (o[a] - g.gc_o[a]);
            r2 += rel[a] * rel[a];
          }
          const float rr = sqrtf(r2);
          const float phi = g.geometry == 2 ? fminf(rr - g.r_in, g.r_out - rr) : g.r_out - rr;
          if ((ti != 0 || phi < 0.f) && rr > 0.f) {
            float rb = g.r_out;
            if (g.geometry == 2 && (rr - g.r_in) < (g.r_out - rr)) rb = g.r_in;
            // seeded features: a normal particle is mirrored through the circle / sphere it crossed
            if (g.seeded && ti == 0) rb = rr > g.r_out ? 2.f * g.r_out - rr : 2.f * g.r_in - rr;
            const float sc = rb / rr;
#pragma unroll
            for (int a = 0; a < D; ++a) {
              // new coordinate relative to the origin of cell c[a]: centre + rel * rb / |rel|
              const float x = (float)(g.gc_c[a] - c[a]) + g.gc_o[a] + rel[a] * sc;
              const float fl = floorf(x);
              c[a] += (int)fl;
              o[a] = x - fl;
              if (o[a] >= 1.f) {
                o[a] = 0.f;
                c[a] += 1;
              }
            }
            if (!g.seeded) ti = max(ti, 1);
          }
        }
      }
      // keys must stay inside the grid whatever the arithmetic above produced
#pragma unroll
      for (int a = 0; a < D; ++a) {
        if (!(o[a] >= 0.f && o[a] < 1.f)) o[a] = 0.f;
        if (c[a] < 0) {
          c[a] = 0;
          o[a] = 0.f;
        }
        if (c[a] > g.gmax) {
          c[a] = g.gmax;
          o[a] = 0.f;
        }
      }
      skey[io] = cellbase + pack_key<D>(c, o, g);
      soff[io] = make_float4(o[0], o[1], D == 3 ? o[2] : 0.f, 0.f);
      sct[io] = (uint32_t)ti | (aux_colour(ai) << 2);
      sid[io] = wid[io];
      if (at_out) at_out[io] = make_float4(b[0], b[1], b[2], 0.f);
      if (v_out) v_out[io] = make_float4(v[0], v[1], v[2], 0.f);
      if (dr_out) dr_out[io] = make_float4(dr[0], dr[1], dr[2], 0.f);
      part[0] = (double)ke;
      part[1] = fin ? 0.0 : 1.0;
      part[2] = ti != 0 ? 1.0 : 0.0;
    }
  }
  // block sums through LDS, after the epilogue's values
  constexpr size_t kEpBytes = (size_t)3 * P * sizeof(float), kRedBytes = (size_t)(P + 1) * 3 * sizeof(double);
  static_assert((kEpBytes + 15) / 16 * 16 + kRedBytes <= (size_t)row_table_rows<L>() * row_table_stride<L>() * sizeof(uint4),
                "the epilogue and the reduction fit in the row table");
  double *rb = reinterpret_cast<double *>(reinterpret_cast<char *>(rowtab) + (kEpBytes + 15) / 16 * 16);
  double *out = partials + (size_t)lb * kNumPartials + P_KE;
  block_reduce_lds<3, P, false>(part, threadIdx.x < P ? (int)threadIdx.x : -1, 0u, 0u, rb,
                                [&](int s, double x) { out[s] = x; });
}

template <int D, int L, bool PER>
__global__ __launch_bounds__(kBlock) MPSPH_PAIR_OCCUPANCY void pass_viscous_integrate(int b0, MPSPH_PASS2_PARAMS) {
  __shared__ uint4 rowtab[row_table_rows<L>() * row_table_stride<L>()];
  viscous_integrate_block<D, L, PER, !PER || D == 2>(b0 + xcd_block(blockIdx.x, gridDim.x), rowtab, MPSPH_PASS2_ARGS);
}


// Persistent launches of the two pair passes: a fixed grid serves the logical blocks
// b0 + [0, nb) from a work queue in device memory, either of one dimension group (DM = 2 or 3) or
// of both in one launch (DM = 5: blocks below nb2 are 2D, the others 3D).  The blocks
// are split into 8 contiguous ranges, one per XCD; a workgroup (XCD blockIdx.x mod 8 under the
// round-robin dispatch) takes the next block of its own range and then of the others.  q[0..7]
// count the blocks taken from each range, q[8] the workgroups that finished; the last one resets
// the queue, so the launch needs no memset and can be captured in a graph.
__device__ __forceinline__ int queue_next(uint32_t *q, int nb) {
  const int x = blockIdx.x & 7, per = nb >> 3, rem = nb & 7;
  for (int k = 0; k < 8; ++k) {
    const int r = (x + k) & 7;
    const int start = r * per + (r < rem ? r : rem), len = per + (r < rem ? 1 : 0);
    const uint32_t t = atomicAdd(&q[r], 1u);
    if ((int)t < len) return start + (int)t;
  }
  return nb;
}
__device__ __forceinline__ void queue_done(uint32_t *q) {
  __threadfence();
  if (atomicAdd(&q[8], 1u) == gridDim.x - 1u) {
    for (int k = 0; k < 9; ++k) q[k] = 0u;
    __threadfence();
  }
}

template <int DM, int L, bool PER, bool DBG>
__global__ __launch_bounds__(kBlock) MPSPH_PAIR_OCCUPANCY void pass_density_force_queue(int b0, int nb2, int nb,
                                                                                        uint32_t *queue,
                                                                                        MPSPH_PASS1_PARAMS) {
  __shared__ uint4 rowtab[row_table_rows<L>() * row_table_stride<L>()];
  __shared__ int sitem;
  for (;;) {
    __syncthreads();   // the previous block's LDS (row table, reductions) is no longer read
    if (threadIdx.x == 0) sitem = queue_next(queue, nb);
    __syncthreads();
    const int it = __builtin_amdgcn_readfirstlane(sitem);   // the same in every lane
    if (it >= nb) break;
    if constexpr (DM == 5) {
      if (it < nb2) density_force_block<2, L, PER, DBG, false, false>(b0 + it, rowtab, nullptr, MPSPH_PASS1_ARGS);
      else density_force_block<3, L, PER, DBG, false, false>(b0 + it, rowtab, nullptr, MPSPH_PASS1_ARGS);
    } else {
      density_force_block<DM, L, PER, DBG, false, false>(b0 + it, rowtab, nullptr, MPSPH_PASS1_ARGS);
    }
  }
  if (threadIdx.x == 0) queue_done(queue);
}

template <int DM, int L, bool PER>
__global__ __launch_bounds__(kBlock) MPSPH_PAIR_OCCUPANCY void pass_viscous_integrate_queue(int b0, int nb2, int nb,
                                                                                            uint32_t *queue,
                                                                                            MPSPH_PASS2_PARAMS) {
  __shared__ uint4 rowtab[row_table_rows<L>() * row_table_stride<L>()];
  __shared__ int sitem;
  for (;;) {
    __syncthreads();   // the previous block's LDS (row table, reductions) is no longer read
    if (threadIdx.x == 0) sitem = queue_next(queue, nb);
    __syncthreads();
    const int it = __builtin_amdgcn_readfirstlane(sitem);   // the same in every lane
    if (it >= nb) break;
    if constexpr (DM == 5) {
      if (it < nb2) viscous_integrate_block<2, L, PER, false>(b0 + it, rowtab, MPSPH_PASS2_ARGS);
      else viscous_integrate_block<3, L, PER, false>(b0 + it, rowtab, MPSPH_PASS2_ARGS);
    } else {
      viscous_integrate_block<DM, L, PER, false>(b0 + it, rowtab, MPSPH_PASS2_ARGS);
    }
  }
  if (threadIdx.x == 0) queue_done(queue);
}


// Debug: ordered geometric neighbour pairs (i, j != i, r_ij < kappa h_ij, no type mask) of the
// last step's start-of-step state, enumerated with the same candidate scan and predicate as the
// pair passes (two lanes per particle).  Pairs go to (out_i, out_j) as load indices while the
// running count stays below cap; *count receives the total.
template <int D, bool PER>
__global__ __launch_bounds__(kBlock) void dump_pairs(const DomDev *__restrict__ doms, int ndom, int i0, int i1,
                                                     const uint32_t *__restrict__ wkey, const float4 *__restrict__ wpos,
                                                     const uint32_t *__restrict__ wjaux, const uint32_t *__restrict__ wid,
                                                     const uint32_t *__restrict__ cstart, unsigned long long cap,
                                                     uint32_t *__restrict__ out_i, uint32_t *__restrict__ out_j,
                                                     unsigned long long *__restrict__ count) {
  constexpr int L = 2;   // lanes per particle, as in the pair passes
  const int t = blockIdx.x * kBlock + threadIdx.x;
  const int i = i0 + t / L, sub = t % L;
  if (i >= i1) return;   // both lanes of a particle leave together
  const DomDev &dd = doms[domain_of(doms, ndom, i)];
  const GridDev &g = dd.g;
  const StepDev &sp = dd.sp;
  int ci[3];
  unpack_key<D>(wkey[i] - dd.cellbase, g, ci);
  const float4 pi = wpos[i];
  const float oi[3] = {pi.x, pi.y, pi.z};
  const float hi = pi.w;
  const float rs = fminf(sp.search_fac * hi, sp.kappa * 0.5f * (hi + sp.hmax)) * 1.0001f;
  const float kh = 0.5f * sp.kappa;
  const uint32_t idi = wid[i];
  __shared__ uint4 rowtab[row_table_rows<L>() * row_table_stride<L>()];
  scan_group_table<D, L, row_table_rows<L>(), PER>(i, sub, rowtab + threadIdx.x / L, row_table_stride<L>(), ci, oi, rs,
                                                   g, dd.cellbase, cstart, [&](uint32_t jr, float dy0, float dz0, bool v) {
    // a slot past the chunk's end may carry an index outside the arrays (and NaN offsets)
    const int j = v && jr < (uint32_t)g.n ? (int)jr : i;
    const float4 pj = wpos[j];
    const uint32_t aj = wjaux[j];
    const float dx = sep_x<PER, D>(g, (float)ci[0], aj, oi[0], pj.x);
    const float dy = dy0 - pj.y;
    float r2 = dx * dx + dy * dy;
    if constexpr (D == 3) {
      const float dz = dz0 - pj.z;
      r2 += dz * dz;
    }
    const float hij = kh * (hi + pj.w);
    if (!(v && r2 < hij * hij)) return;
    const unsigned long long k = atomicAdd(count, 1ull);
    if (k < cap) {
      out_i[k] = idi;
      out_j[k] = wid[j];
    }
  });
}

// Combine partials slot by slot: sums, or min / max for the slots that hold extrema.
__device__ __forceinline__ double combine_slot(int s, double a, double b) {
  return (s == P_EMAX || s == P_ELRMAX) ? fmax(a, b) : (s == P_ELRMIN ? fmin(a, b) : a + b);
}
__device__ __forceinline__ double slot_identity(int s) { return s == P_ELRMIN ? INFINITY : 0.0; }

// Fixed-order reduction of nrows partial rows (kNumPartials doubles each) by one block:
// thread t owns rows t, t + 256, ..., then a fixed tree over the threads.  Result in red[s][0].
__device__ __forceinline__ void reduce_rows(const double *__restrict__ rows, int nrows, double (*red)[257]) {
  double acc[kNumPartials];
#pragma unroll
  for (int s = 0; s < kNumPartials; ++s) acc[s] = slot_identity(s);
  for (int b = threadIdx.x; b < nrows; b += 256) {
    const double *p = rows + (size_t)b * kNumPartials;
#pragma unroll
    for (int s = 0; s < kNumPartials; ++s) acc[s] = combine_slot(s, acc[s], p[s]);
  }
#pragma unroll
  for (int s = 0; s < kNumPartials; ++s) red[s][threadIdx.x] = acc[s];
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
#pragma unroll
      for (int s = 0; s < kNumPartials; ++s)
        red[s][threadIdx.x] = combine_slot(s, red[s][threadIdx.x], red[s][threadIdx.x + w]);
    }
    __syncthreads();
  }
}

// First level of the metric reduction: row group r (never straddling two domains) reduces the
// pair-kernel block partials [groups[r].x, groups[r].y) into one row.
__global__ __launch_bounds__(256) void reduce_partials(const int2 *__restrict__ groups, const double *__restrict__ partials,
                                                       double *__restrict__ out) {
  __shared__ double red[kNumPartials][257];
  const int2 gr = groups[blockIdx.x];
  reduce_rows(partials + (size_t)gr.x * kNumPartials, gr.y - gr.x, red);
  if (threadIdx.x < kNumPartials) out[(size_t)blockIdx.x * kNumPartials + threadIdx.x] = red[threadIdx.x][0];
}

// Second level, one block per domain: the domain's first-level rows into its metrics block m[32 d ...]:
// slots 0..15 as laid out in kNumPartials, 16: dt1, 17: dt2, 18..20: running totals of pairs,
// candidates and steps.  Block 0 then advances the device step counter.
__global__ __launch_bounds__(256) void finalize(const DomDev *__restrict__ doms, const double *__restrict__ rows,
                                                const uint32_t *__restrict__ dtslots, double *__restrict__ m,
                                                int64_t *__restrict__ stepctr) {
  __shared__ double red[kNumPartials][257];
  const int d = blockIdx.x;
  reduce_rows(rows + (size_t)doms[d].row0 * kNumPartials, doms[d].nrow, red);
  double *md = m + (size_t)d * 32;
  if (threadIdx.x < kNumPartials) md[threadIdx.x] = red[threadIdx.x][0];
  if (threadIdx.x == 0) {
    float d1 = INFINITY;
    for (int s = 0; s < kDtSlots; ++s) d1 = fminf(d1, __uint_as_float(dtslots[d * kDtSlots + s]));
    md[16] = d1 < INFINITY ? (double)d1 : 0.0;
    md[17] = d1 < INFINITY ? (double)(d1 * doms[d].sp.dt2_factor) : 0.0;
    // running totals since the last load (exact integers below 2^53)
    md[18] += red[P_PAIRS][0];
    md[19] += red[P_CAND][0];
    md[20] += 1.0;
    // automatic t0 (reading of the paper's "topology static for some iterations"): the
    // interface-pair count and the number of particles with an interface pair stay within
    // t0_tol of a reference for t0_window steps; otherwise the reference restarts here
    const StepDev &sp = doms[d].sp;
    if (sp.auto_t0 && !(md[kAutoT0] > 0.0)) {
      const double t = md[20] - 1.0;  // index of this step since the load
      const double I = red[P_IFC][0] * 0.5, P = red[P_IFCP][0];
      const double tol = (double)sp.t0_tol;
      if (t == 0.0 || fabs(I - md[kAutoT0 + 1]) > tol * md[kAutoT0 + 1] ||
          fabs(P - md[kAutoT0 + 2]) > tol * md[kAutoT0 + 2]) {
        md[kAutoT0 + 1] = I;
        md[kAutoT0 + 2] = P;
        md[kAutoT0 + 3] = t;
      } else if (t - md[kAutoT0 + 3] >= (double)sp.t0_window) {
        md[kAutoT0] = t + 1.0;
      }
    }
    if (d == 0) *stepctr += 1;
  }
}

// Positions back to domain units (FP64) in the load order; state indices [i0, i1).
template <int D>
__global__ __launch_bounds__(kBlock) void store_kernel(const DomDev *__restrict__ doms, int ndom, int i0, int i1,
                                                       const uint32_t *__restrict__ skey, const float4 *__restrict__ soff,
                                                       const uint32_t *__restrict__ sct, const uint32_t *__restrict__ sid,
                                                       float *__restrict__ pos, int32_t *__restrict__ type) {
  const int i = i0 + blockIdx.x * kBlock + threadIdx.x;
  if (i >= i1) return;
  const DomDev &dd = doms[domain_of(doms, ndom, i)];
  int c[3];
  unpack_key<D>(skey[i] - dd.cellbase, dd.g, c);
  const float4 o = soff[i];
  const float oo[3] = {o.x, o.y, o.z};
  const uint32_t id = sid[i];
  if (pos) {
    float *x = pos + dd.xoff + (int64_t)((int)id - dd.uoff) * D;
    for (int a = 0; a < D; ++a) x[a] = (float)(dd.lo[a] + ((double)c[a] + (double)oo[a]) * dd.cs);
  }
  if (type) type[id] = (int32_t)(sct[i] & 3u);
}

// Scatter one per-particle quantity of the last step to load order, converted to domain units;
// sorted indices [i0, i1).  vscale[d] multiplies vector quantities (dt1 / 2 of the domain for
// v~; NULL: 1).
template <int D>
__global__ __launch_bounds__(kBlock) void dump_kernel(const DomDev *__restrict__ doms, int ndom, int i0, int i1,
                                                      int which, const uint32_t *__restrict__ wkey,
                                                      const float4 *__restrict__ wpos, const uint32_t *__restrict__ wid,
                                                      const float *__restrict__ sc, const float4 *__restrict__ vec,
                                                      const float *__restrict__ vscale, float *__restrict__ out) {
  const int i = i0 + blockIdx.x * kBlock + threadIdx.x;
  if (i >= i1) return;
  const int d = domain_of(doms, ndom, i);
  const DomDev &dd = doms[d];
  const uint32_t id = wid[i];
  float *ov = out + dd.xoff + (int64_t)((int)id - dd.uoff) * D;  // row of a vector quantity
  const float4 p = wpos[i];
  const double csd = dd.cs;
  switch (which) {
    case MPSPH_F_RHO:
      out[id] = (float)((double)sc[i] / pow(csd, D));
      break;
    case MPSPH_F_RHO_T: {
      const double s = (double)p.w / dd.sp.tau * csd;
      out[id] = (float)pow(s, -D);
      break;
    }
    case MPSPH_F_H:
      out[id] = (float)((double)p.w * csd);
      break;
    case MPSPH_F_NN:
    case MPSPH_F_A_ABS:
      out[id] = (float)((double)sc[i] * csd);
      break;
    case MPSPH_F_X0: {
      int c[3];
      unpack_key<D>(wkey[i] - dd.cellbase, dd.g, c);
      const float oo[3] = {p.x, p.y, p.z};
      for (int a = 0; a < D; ++a) ov[a] = (float)(dd.lo[a] + ((double)c[a] + (double)oo[a]) * csd);
      break;
    }
    default: {  // vector quantities in cell units per time: scale by cs (and vscale)
      const float4 v = vec[i];
      const float vv[3] = {v.x, v.y, v.z};
      const float f = vscale ? vscale[d] : 1.f;
      for (int a = 0; a < D; ++a) ov[a] = (float)((double)(vv[a] * f) * csd);
    }
  }
}

// ------------------------------------------------------------------------------------------
// Host side
// ------------------------------------------------------------------------------------------

inline size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

struct Derived {
  int dim, k, gmax;
  int xe;                  // x sub-cells per cell in the cell key: 2^xe
  double L, cs, inv_cs, lo[3], xhi[3];
  double smin, smax, lip;  // spacing bounds (domain units), Lipschitz constant of s
  double search_fac;
};

const char *kErr[] = {"ok", "invalid argument", "out of memory", "device error", "bad context state",
                      "non-finite values", "unsupported configuration",
                      "the problem needs more workspace than the static scratch array holds"};

bool valid_params(const mpsph_params *p) {
  if (!p) return false;
  if (p->dim != 2 && p->dim != 3) return false;
  if (p->geometry < MPSPH_PERIODIC || p->geometry > MPSPH_LEVELSET) return false;
  if (p->geometry == MPSPH_PERIODIC)  // periodic: a cube (a square in 2D), every side one period
    for (int a = 1; a < p->dim; ++a)
      if (p->hi[a] - p->lo[a] != p->hi[0] - p->lo[0]) return false;
  if (p->geometry == MPSPH_LEVELSET || p->field == MPSPH_GRID) {
    int64_t nodes = 1;
    for (int a = 0; a < p->dim; ++a) {
      if (p->grid_n[a] < 2 || p->grid_n[a] > (1 << 14)) return false;
      nodes *= p->grid_n[a];
    }
    if (nodes > ((int64_t)1 << 27)) return false;
    if (p->geometry == MPSPH_LEVELSET && !p->grid_phi) return false;
    if (p->field == MPSPH_GRID) {
      if (!p->grid_s) return false;
      for (int64_t k = 0; k < nodes; ++k)
        if (!(p->grid_s[k] > 0) || !std::isfinite(p->grid_s[k])) return false;
    }
  }
  if (p->geometry == MPSPH_ANNULUS && p->dim != 2) return false;
  for (int a = 0; a < p->dim; ++a)
    if (!(p->hi[a] > p->lo[a]) || !std::isfinite(p->lo[a]) || !std::isfinite(p->hi[a])) return false;
  if (p->field < MPSPH_UNIFORM || p->field > MPSPH_GRID) return false;
  if (p->field == MPSPH_RBF_EXP && (p->n_rbf < 0 || p->n_rbf > 64 || (p->n_rbf > 0 && (!p->rbf_centre || !p->rbf_coeff)) ||
                                    !(p->rbf_width > 0)))
    return false;
  // the kernel's support is 2h: a cut-off beyond it would only add zero terms, and the pair
  // kernels evaluate the kernel's polynomial without clamping it to its support
  if (!(p->tau > 0) || !(p->kappa > 0 && p->kappa <= 2) || !(p->p0 > 0) || !(p->sigma0 >= 0)) return false;
  if (p->t0 < -2 || (p->t0 >= 0 && p->t1 < p->t0)) return false;
  if (!(p->nu_coeff >= 0) || !(p->c_acc > 0) || !(p->c_vel > 0) || !(p->c_visc > 0)) return false;
  if ((p->geometry == MPSPH_ANNULUS || p->geometry == MPSPH_BALL) && !(p->r_out > 0)) return false;
  if (p->geometry == MPSPH_ANNULUS && !(p->r_in > 0 && p->r_in < p->r_out)) return false;
  if (p->cell_log2 != -1 && (p->cell_log2 < 1 || p->cell_log2 > 12)) return false;
  return true;
}

double box_dist_range(const mpsph_params *p, const double *c, double *dmax) {
  double dmin2 = 0.0, dmax2 = 0.0;
  for (int a = 0; a < p->dim; ++a) {
    double lo = p->lo[a] - c[a], hi = p->hi[a] - c[a];
    double near = (lo > 0) ? lo : (hi < 0 ? -hi : 0.0);
    double far = std::max(std::fabs(lo), std::fabs(hi));
    dmin2 += near * near;
    dmax2 += far * far;
  }
  *dmax = std::sqrt(dmax2);
  return std::sqrt(dmin2);
}

// Multilinear interpolation on the background mesh (host, FP64), optional gradient.
double host_mesh(const mpsph_params *p, const double *nodes, const double *x, double *grad = nullptr) {
  const int d = p->dim;
  int base[3] = {0, 0, 0};
  double f[3] = {0, 0, 0}, inv[3] = {1, 1, 1};
  for (int a = 0; a < d; ++a) {
    inv[a] = (double)(p->grid_n[a] - 1) / (p->hi[a] - p->lo[a]);
    const double u = (x[a] - p->lo[a]) * inv[a];
    const int i = std::min(std::max((int)std::floor(u), 0), p->grid_n[a] - 2);
    base[a] = i;
    f[a] = u - i;
  }
  double val = 0.0, g[3] = {0, 0, 0};
  for (int cn = 0; cn < (1 << d); ++cn) {
    size_t idx = 0, stride = 1;
    double w = 1.0, dw[3] = {1, 1, 1};
    for (int a = 0; a < d; ++a) {
      const int bit = (cn >> a) & 1;
      idx += (size_t)(base[a] + bit) * stride;
      stride *= (size_t)p->grid_n[a];
      const double wa = bit ? f[a] : 1.0 - f[a];
      for (int b = 0; b < d; ++b) dw[b] *= b == a ? (bit ? inv[a] : -inv[a]) : wa;
      w *= wa;
    }
    val += w * nodes[idx];
    for (int b = 0; b < d; ++b) g[b] += dw[b] * nodes[idx];
  }
  if (grad)
    for (int a = 0; a < 3; ++a) grad[a] = a < d ? g[a] : 0.0;
  return val;
}

// Spacing of the field in domain units at a point (host, FP64), with scale s0.
double host_spacing(const mpsph_params *p, double s0, const double *x) {
  if (p->field == MPSPH_GRID) return s0 * host_mesh(p, p->grid_s, x);
  auto dist = [&](const double *c) {
    double s = 0;
    for (int a = 0; a < p->dim; ++a) s += (x[a] - c[a]) * (x[a] - c[a]);
    return std::sqrt(s);
  };
  switch (p->field) {
    case MPSPH_UNIFORM:
      return s0;
    case MPSPH_RADIAL_LINEAR:
      return s0 * (1.0 + p->fa * (dist(p->fcentre) - p->fb));
    case MPSPH_SPHERE_DISTANCE:
      return s0 * (1.0 + p->fa * std::fabs(dist(p->fcentre) - p->fb));
    default: {
      double e = 0;
      for (int k = 0; k < p->n_rbf; ++k) {
        double r = dist(p->rbf_centre + k * p->dim);
        e += p->rbf_coeff[k] * std::exp(-r * r / (2 * p->rbf_width * p->rbf_width));
      }
      return s0 * std::exp(e);
    }
  }
}

bool inside_region(const mpsph_params *p, const double *x) {
  if (p->geometry == MPSPH_BOX || p->geometry == MPSPH_PERIODIC) return true;
  if (p->geometry == MPSPH_LEVELSET) return host_mesh(p, p->grid_phi, x) > 0.0;
  double r = 0;
  for (int a = 0; a < p->dim; ++a) r += (x[a] - p->centre[a]) * (x[a] - p->centre[a]);
  r = std::sqrt(r);
  if (p->geometry == MPSPH_ANNULUS) return r >= p->r_in && r <= p->r_out;
  return r <= p->r_out;
}

// Gauss-Legendre nodes on [0,1] (8 points).
void gauss8(double *xg, double *wg) {
  static const double t[4] = {0.1834346424956498, 0.5255324099163290, 0.7966664774136267, 0.9602898564975363};
  static const double w[4] = {0.3626837833783620, 0.3137066458778873, 0.2223810344533745, 0.1012285362903763};
  for (int i = 0; i < 4; ++i) {
    xg[3 - i] = 0.5 * (1 - t[i]);
    xg[4 + i] = 0.5 * (1 + t[i]);
    wg[3 - i] = 0.5 * w[i];
    wg[4 + i] = 0.5 * w[i];
  }
}

// Integral of s^-d over the region for s0 = 1: composite 8-point Gauss-Legendre in Cartesian
// panels (box) or polar / spherical coordinates (annulus, ball).
double field_integral_unit(const mpsph_params *p) {
  double xg[8], wg[8];
  gauss8(xg, wg);
  const int d = p->dim;
  const double pi = 3.14159265358979323846;
  double total = 0.0;
  if (p->geometry == MPSPH_LEVELSET) {
    // midpoint rule over sub-cells of the bounding box with the indicator of the positive phase
    const int M = d == 2 ? 1024 : 160;
    double h[3] = {0, 0, 0}, vol = 1.0;
    for (int a = 0; a < d; ++a) {
      h[a] = (p->hi[a] - p->lo[a]) / M;
      vol *= h[a];
    }
    const int64_t cells = d == 2 ? (int64_t)M * M : (int64_t)M * M * M;
    for (int64_t cidx = 0; cidx < cells; ++cidx) {
      double x[3];
      int64_t r = cidx;
      for (int a = 0; a < d; ++a) {
        x[a] = p->lo[a] + ((double)(r % M) + 0.5) * h[a];
        r /= M;
      }
      if (!(host_mesh(p, p->grid_phi, x) > 0.0)) continue;
      total += std::pow(host_spacing(p, 1.0, x), -d);
    }
    return total * vol;
  }
  const bool boxlike = p->geometry == MPSPH_BOX || p->geometry == MPSPH_PERIODIC;
  if (p->field == MPSPH_UNIFORM) {  // s = 1: the measure of the region
    if (boxlike) {
      double v = 1.0;
      for (int a = 0; a < d; ++a) v *= p->hi[a] - p->lo[a];
      return v;
    }
    if (p->geometry == MPSPH_ANNULUS) return pi * (p->r_out * p->r_out - p->r_in * p->r_in);
    return d == 2 ? pi * p->r_out * p->r_out : 4.0 / 3.0 * pi * p->r_out * p->r_out * p->r_out;
  }
  if (boxlike) {
    const int M = d == 2 ? 256 : (p->field == MPSPH_GRID ? 24 : 48);
    const int np = M * 8;
    std::vector<double> node[3], wt[3];
    for (int a = 0; a < d; ++a) {
      double h = (p->hi[a] - p->lo[a]) / M;
      for (int m = 0; m < M; ++m)
        for (int q = 0; q < 8; ++q) {
          node[a].push_back(p->lo[a] + (m + xg[q]) * h);
          wt[a].push_back(wg[q] * h);
        }
    }
    double x[3];
    if (d == 2) {
      for (int i = 0; i < np; ++i)
        for (int j = 0; j < np; ++j) {
          x[0] = node[0][i];
          x[1] = node[1][j];
          total += wt[0][i] * wt[1][j] * std::pow(host_spacing(p, 1.0, x), -d);
        }
    } else {
      for (int i = 0; i < np; ++i) {
        double acc = 0;
        for (int j = 0; j < np; ++j)
          for (int l = 0; l < np; ++l) {
            x[0] = node[0][i];
            x[1] = node[1][j];
            x[2] = node[2][l];
            double s = host_spacing(p, 1.0, x);
            acc += wt[1][j] * wt[2][l] / (s * s * s);
          }
        total += wt[0][i] * acc;
      }
    }
    return total;
  }
  const double r0 = p->geometry == MPSPH_ANNULUS ? p->r_in : 0.0, r1 = p->r_out;
  const int MR = d == 2 ? 128 : 64, MT = d == 2 ? 64 : 16, MP = 32;
  for (int mr = 0; mr < MR; ++mr)
    for (int qr = 0; qr < 8; ++qr) {
      double r = r0 + (mr + xg[qr]) * (r1 - r0) / MR, wr = wg[qr] * (r1 - r0) / MR;
      for (int mt = 0; mt < MT; ++mt)
        for (int qt = 0; qt < 8; ++qt) {
          double th = (mt + xg[qt]) * (d == 2 ? 2 * pi : pi) / MT, wth = wg[qt] * (d == 2 ? 2 * pi : pi) / MT;
          if (d == 2) {
            double x[2] = {p->centre[0] + r * std::cos(th), p->centre[1] + r * std::sin(th)};
            total += wr * wth * r * std::pow(host_spacing(p, 1.0, x), -2);
          } else {
            for (int mp = 0; mp < MP; ++mp)
              for (int qp = 0; qp < 8; ++qp) {
                double ph = (mp + xg[qp]) * 2 * pi / MP, wph = wg[qp] * 2 * pi / MP;
                double x[3] = {p->centre[0] + r * std::sin(th) * std::cos(ph),
                               p->centre[1] + r * std::sin(th) * std::sin(ph), p->centre[2] + r * std::cos(th)};
                total += wr * wth * wph * r * r * std::sin(th) * std::pow(host_spacing(p, 1.0, x), -3);
              }
          }
        }
    }
  return total;
}

// Boundary features of a region (the order the header documents) with the integral, at s0 = 1,
// of s^-k over each: k = dim - 1 on a feature surface, 1 on a feature curve, 0 at a corner.
struct FeatureList {
  int n = 0;
  int type[MPSPH_MAX_FEATURES];
  int power[MPSPH_MAX_FEATURES];
  double I[MPSPH_MAX_FEATURES];
  void add(int t, int k, double v) {
    type[n] = t;
    power[n] = k;
    I[n] = v;
    ++n;
  }
};

// Panels per axis of the composite rule along box axis a: one per background-mesh cell for a
// gridded field (the interpolant is smooth inside a cell), else the given count.
int feature_panels(const mpsph_params *p, int a, int dflt) {
  return p->field == MPSPH_GRID ? std::max(p->grid_n[a] - 1, 1) : dflt;
}

// Integral of s^-k over the parallelogram o + u e1 + v e2 (u, v in [0,1]; e2 = 0 for a segment)
// with m1 x m2 panels of the 8-point Gauss-Legendre rule, s0 = 1.
double flat_integral(const mpsph_params *p, const double *o, const double *e1, const double *e2, int k, int m1,
                     int m2) {
  double xg[8], wg[8];
  gauss8(xg, wg);
  const int d = p->dim;
  double l1 = 0, l2 = 0;
  for (int a = 0; a < d; ++a) {
    l1 += e1[a] * e1[a];
    l2 += e2[a] * e2[a];
  }
  const bool seg = l2 == 0.0;
  const double meas = seg ? std::sqrt(l1) : std::sqrt(l1) * std::sqrt(l2);  // e1, e2 orthogonal
  if (!seg && m2 < 1) m2 = 1;
  const int n2 = seg ? 1 : 8 * m2;
  double total = 0.0;
  for (int i = 0; i < 8 * m1; ++i) {
    const double u = ((i >> 3) + xg[i & 7]) / m1, wu = wg[i & 7] / m1;
    double acc = 0.0;
    for (int j = 0; j < n2; ++j) {
      const double v = seg ? 0.0 : ((j >> 3) + xg[j & 7]) / m2, wv = seg ? 1.0 : wg[j & 7] / m2;
      double x[3] = {0, 0, 0};
      for (int a = 0; a < d; ++a) x[a] = o[a] + u * e1[a] + v * e2[a];
      acc += wv * std::pow(host_spacing(p, 1.0, x), -(double)k);
    }
    total += wu * acc;
  }
  return total * meas;
}

// Integral of s^-k over the sphere (dim 3) or circle (dim 2) of radius R about the region's
// centre, s0 = 1.
double round_integral(const mpsph_params *p, double R, int k) {
  double xg[8], wg[8];
  gauss8(xg, wg);
  const double pi = 3.14159265358979323846;
  const double *c = p->centre;
  double total = 0.0;
  if (p->dim == 2) {
    const int M = 256;
    for (int i = 0; i < 8 * M; ++i) {
      const double th = ((i >> 3) + xg[i & 7]) * 2 * pi / M, w = wg[i & 7] * 2 * pi / M;
      const double x[2] = {c[0] + R * std::cos(th), c[1] + R * std::sin(th)};
      total += w * R * std::pow(host_spacing(p, 1.0, x), -(double)k);
    }
    return total;
  }
  const int MT = 32, MP = 64;
  for (int i = 0; i < 8 * MT; ++i) {
    const double th = ((i >> 3) + xg[i & 7]) * pi / MT, wt = wg[i & 7] * pi / MT;
    double acc = 0.0;
    for (int j = 0; j < 8 * MP; ++j) {
      const double ph = ((j >> 3) + xg[j & 7]) * 2 * pi / MP, wp = wg[j & 7] * 2 * pi / MP;
      const double x[3] = {c[0] + R * std::sin(th) * std::cos(ph), c[1] + R * std::sin(th) * std::sin(ph),
                           c[2] + R * std::cos(th)};
      acc += wp * std::pow(host_spacing(p, 1.0, x), -(double)k);
    }
    total += wt * R * R * std::sin(th) * acc;
  }
  return total;
}

// The features of a region and their integrals at s0 = 1 (§2.3, Eq. 6: a surface integral on the
// feature surfaces and a line integral on the feature curves).
FeatureList feature_integrals(const mpsph_params *p) {
  FeatureList f;
  const int d = p->dim;
  if (p->geometry == MPSPH_PERIODIC) return f;
  if (p->geometry == MPSPH_BALL) {
    f.add(MPSPH_SURFACE, d - 1, round_integral(p, p->r_out, d - 1));
    return f;
  }
  if (p->geometry == MPSPH_ANNULUS) {
    f.add(MPSPH_SURFACE, 1, round_integral(p, p->r_in, 1));
    f.add(MPSPH_SURFACE, 1, round_integral(p, p->r_out, 1));
    return f;
  }
  const double *lo = p->lo, *hi = p->hi;
  auto corner_of = [&](int bits, double *x) {
    for (int a = 0; a < 3; ++a) x[a] = a < d ? ((bits >> a) & 1 ? hi[a] : lo[a]) : 0.0;
  };
  if (d == 2) {
    for (int a = 0; a < 2; ++a)
      for (int side = 0; side < 2; ++side) {
        const int b = 1 - a;
        double o[3] = {0, 0, 0}, e1[3] = {0, 0, 0}, e2[3] = {0, 0, 0};
        o[a] = side ? hi[a] : lo[a];
        o[b] = lo[b];
        e1[b] = hi[b] - lo[b];
        f.add(MPSPH_SURFACE, 1, flat_integral(p, o, e1, e2, 1, feature_panels(p, b, 256), 0));
      }
    for (int c = 0; c < 4; ++c) f.add(MPSPH_FIXED, 0, 1.0);
    return f;
  }
  for (int a = 0; a < 3; ++a)
    for (int side = 0; side < 2; ++side) {
      const int b = (a + 1) % 3, c = (a + 2) % 3;
      double o[3], e1[3] = {0, 0, 0}, e2[3] = {0, 0, 0};
      corner_of(0, o);
      o[a] = side ? hi[a] : lo[a];
      e1[b] = hi[b] - lo[b];
      e2[c] = hi[c] - lo[c];
      f.add(MPSPH_SURFACE, 2, flat_integral(p, o, e1, e2, 2, feature_panels(p, b, 32), feature_panels(p, c, 32)));
    }
  for (int a = 0; a < 3; ++a) {
    const int b = a == 0 ? 1 : 0, c = a == 2 ? 1 : 2;  // the two other axes, lower first
    for (int sc = 0; sc < 2; ++sc)
      for (int sb = 0; sb < 2; ++sb) {
        double o[3], e1[3] = {0, 0, 0}, e2[3] = {0, 0, 0};
        corner_of(0, o);
        o[b] = sb ? hi[b] : lo[b];
        o[c] = sc ? hi[c] : lo[c];
        e1[a] = hi[a] - lo[a];
        f.add(MPSPH_CURVE, 1, flat_integral(p, o, e1, e2, 1, feature_panels(p, a, 256), 0));
      }
  }
  for (int c = 0; c < 8; ++c) f.add(MPSPH_FIXED, 0, 1.0);
  return f;
}

// Bounds of s over the bounding box, and a Lipschitz constant of s (domain units).
// Bounds of the RBF field s = s0 exp(f), f(x) = sum_k c_k G_k(x), G_k = exp(-|x - x_k|^2 / (2 w^2)),
// over the box, from f and grad f on a grid: every point of the box lies within rho (half a grid
// cell's diagonal) of a node n, and |hess G| <= 1 / w^2 everywhere, so with Hf = sum |c_k| / w^2
//   f(x) <= f(n) + |grad f(n)| rho + Hf rho^2 / 2   (Taylor), likewise for the minimum, and
//   |grad f(x)| <= |grad f(n)| + Hf rho.
// Each bound is also capped by its grid-free form (sum of the positive / negative c_k, and
// |grad f| <= sum |c_k| / (w sqrt(e))).  The Lipschitz constant of s is smax * max |grad f|.
void rbf_bounds(const mpsph_params *p, double s0, double *smin, double *smax, double *lip) {
  const int d = p->dim, nr = p->n_rbf;
  const double w = p->rbf_width;
  double pos = 0, neg = 0, abs_sum = 0;
  for (int k = 0; k < nr; ++k) {
    pos += std::max(p->rbf_coeff[k], 0.0);
    neg += std::min(p->rbf_coeff[k], 0.0);
    abs_sum += std::fabs(p->rbf_coeff[k]);
  }
  const double Lf = abs_sum / (w * std::exp(0.5)), Hf = abs_sum / (w * w);
  const int m = d == 3 ? 64 : 256;   // grid nodes per axis
  double step[3] = {0, 0, 0}, rho2 = 0;
  for (int a = 0; a < d; ++a) {
    step[a] = (p->hi[a] - p->lo[a]) / (m - 1);
    rho2 += 0.25 * step[a] * step[a];
  }
  const double rho = std::sqrt(rho2), inv2w2 = 1.0 / (2.0 * w * w);
  double fmax = -INFINITY, fmin = INFINITY, gmax = 0;
  const int mz = d == 3 ? m : 1;
  for (int iz = 0; iz < mz; ++iz)
    for (int iy = 0; iy < m; ++iy)
      for (int ix = 0; ix < m; ++ix) {
        const double x[3] = {p->lo[0] + ix * step[0], p->lo[1] + iy * step[1], d == 3 ? p->lo[2] + iz * step[2] : 0.0};
        double f = 0, g[3] = {0, 0, 0};
        for (int k = 0; k < nr; ++k) {
          double dv[3] = {0, 0, 0}, r2 = 0;
          for (int a = 0; a < d; ++a) {
            dv[a] = x[a] - p->rbf_centre[k * d + a];
            r2 += dv[a] * dv[a];
          }
          const double t = p->rbf_coeff[k] * std::exp(-r2 * inv2w2);
          f += t;
          for (int a = 0; a < d; ++a) g[a] -= t * dv[a] / (w * w);
        }
        const double gn = std::sqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
        const double reach = gn * rho + 0.5 * Hf * rho * rho;
        fmax = std::max(fmax, f + reach);
        fmin = std::min(fmin, f - reach);
        gmax = std::max(gmax, gn);
      }
  fmax = std::min(pos, fmax);
  fmin = std::max(neg, fmin);
  gmax = std::min(Lf, gmax + Hf * rho);
  *smin = s0 * std::exp(fmin);
  *smax = s0 * std::exp(fmax);
  *lip = *smax * gmax;
}

bool spacing_bounds(const mpsph_params *p, double s0, double *smin, double *smax, double *lip) {
  if (p->field == MPSPH_GRID) {
    // the interpolant stays within the node extremes; its slope along an axis is bounded by the
    // largest node difference along that axis over the spacing
    const int d = p->dim;
    size_t nodes = 1;
    for (int a = 0; a < d; ++a) nodes *= (size_t)p->grid_n[a];
    double lo = INFINITY, hi = 0.0, l2 = 0.0;
    for (size_t k = 0; k < nodes; ++k) {
      lo = std::min(lo, p->grid_s[k]);
      hi = std::max(hi, p->grid_s[k]);
    }
    size_t stride = 1;
    for (int a = 0; a < d; ++a) {
      const double hs = (p->hi[a] - p->lo[a]) / (p->grid_n[a] - 1);
      double m = 0.0;
      for (size_t k = 0; k < nodes; ++k) {
        const size_t ia = (k / stride) % (size_t)p->grid_n[a];
        if (ia + 1 < (size_t)p->grid_n[a]) m = std::max(m, std::fabs(p->grid_s[k + stride] - p->grid_s[k]));
      }
      l2 += (m / hs) * (m / hs);
      stride *= (size_t)p->grid_n[a];
    }
    *smin = s0 * lo;
    *smax = s0 * hi;
    *lip = s0 * std::sqrt(l2);
    return *smin > 0 && std::isfinite(*smax);
  }
  switch (p->field) {
    case MPSPH_UNIFORM:
      *smin = *smax = s0;
      *lip = 0;
      break;
    case MPSPH_RADIAL_LINEAR: {
      double rmax, rmin = box_dist_range(p, p->fcentre, &rmax);
      double a = s0 * (1 + p->fa * (rmin - p->fb)), b = s0 * (1 + p->fa * (rmax - p->fb));
      *smin = std::min(a, b);
      *smax = std::max(a, b);
      *lip = s0 * std::fabs(p->fa);
      break;
    }
    case MPSPH_SPHERE_DISTANCE: {
      double rmax, rmin = box_dist_range(p, p->fcentre, &rmax);
      double dlo = (p->fb >= rmin && p->fb <= rmax) ? 0.0 : std::min(std::fabs(rmin - p->fb), std::fabs(rmax - p->fb));
      double dhi = std::max(std::fabs(rmin - p->fb), std::fabs(rmax - p->fb));
      double a = s0 * (1 + p->fa * dlo), b = s0 * (1 + p->fa * dhi);
      *smin = std::min(a, b);
      *smax = std::max(a, b);
      *lip = s0 * std::fabs(p->fa);
      break;
    }
    default:
      rbf_bounds(p, s0, smin, smax, lip);
  }
  return *smin > 0 && std::isfinite(*smax);
}

int derive(const mpsph_params *p, int64_t n, double s0, Derived *d) {
  d->dim = p->dim;
  double L = 0;
  for (int a = 0; a < p->dim; ++a) L = std::max(L, p->hi[a] - p->lo[a]);
  d->L = L;
  for (int a = 0; a < 3; ++a) d->lo[a] = a < p->dim ? p->lo[a] : 0.0;
  if (!spacing_bounds(p, s0, &d->smin, &d->smax, &d->lip)) return MPSPH_E_INVALID;
  int k = p->cell_log2;
  if (k < 0) {
    // cells of about 0.75 of the smallest cut-off radius; at most 2^24 cells, and not many more
    // cells than particles
    double rc_min = p->kappa * p->tau * d->smin;
    double target = L / (0.75 * rc_min) + 1.0;
    k = (int)std::lround(std::log2(std::max(target, 2.0)));
    int kmax = p->dim == 3 ? 8 : 12;
    while (k > 1 && std::pow(2.0, p->dim * k) > 8.0 * std::max<int64_t>(n, 64)) --k;
    k = std::min(std::max(k, 1), kmax);
  }
  if (p->dim * k > 24) return MPSPH_E_UNSUPPORTED;
  // x sub-cells: up to 2^MPSPH_XSUB per cell while the cell table stays within 4 entries per
  // particle (its fill is part of every step) and the key within 26 bits
  int xe = 0;
  while (xe < MPSPH_XSUB && p->dim * k + xe < 26 &&
         std::pow(2.0, p->dim * k + xe + 1) <= 4.0 * (double)std::max<int64_t>(n, 1))
    ++xe;
  d->xe = xe;
  d->k = k;
  d->gmax = (1 << k) - 1;
  // walls at cells 0 and 2^k - 1 (offset 0); a periodic box wraps after 2^k cells
  const double span = p->geometry == MPSPH_PERIODIC ? (double)(1 << k) : (double)d->gmax;
  d->cs = L / span;
  d->inv_cs = span / L;
  for (int a = 0; a < 3; ++a) d->xhi[a] = a < p->dim ? (p->hi[a] - p->lo[a]) * d->inv_cs : 0.0;
  // neighbour search bound: j interacts only if r < kappa (h_i + h_j)/2 and h_j <= h_i + L_h r
  // (L_h = tau * Lipschitz(s)), so r < kappa h_i / (1 - kappa L_h / 2).
  double Lh = p->tau * d->lip;
  double fac = 1e30;
  if (p->kappa * Lh / 2 < 0.95) fac = p->kappa / (1.0 - p->kappa * Lh / 2);
  d->search_fac = std::max(fac, p->kappa) * (1.0 + 1e-4);
  // minimum images are unique only while the cut-off stays below half the period
  if (p->geometry == MPSPH_PERIODIC && !(p->kappa * p->tau * d->smax < 0.5 * L)) return MPSPH_E_UNSUPPORTED;
  return MPSPH_OK;
}


struct EventHook : LaunchHook {
  struct Rec {
    const char *name;
    hipEvent_t a, b;
  };
  hipStream_t stream = nullptr;
  bool on = false;
  bool pairs_only = false;   // record only the pair passes (kernels named pass_*)
  bool open = false;         // the last begin() recorded an event
  std::vector<Rec> pending;
  std::vector<hipEvent_t> pool;
  std::vector<std::string> names;
  std::vector<int64_t> launches;
  std::vector<double> ms;
  hipEvent_t get() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e;
    (void)hipEventCreate(&e);
    return e;
  }
  void begin(const char *name) override {
    open = on && (!pairs_only || std::strncmp(name, "pass_", 5) == 0);
    if (!open) return;
    Rec r{name, get(), get()};
    (void)hipEventRecord(r.a, stream);
    pending.push_back(r);
  }
  void end() override {
    if (!open) return;
    open = false;
    (void)hipEventRecord(pending.back().b, stream);
  }
  void collect() {
    (void)hipStreamSynchronize(stream);
    for (auto &r : pending) {
      float t = 0;
      (void)hipEventElapsedTime(&t, r.a, r.b);
      size_t k = 0;
      for (; k < names.size(); ++k)
        if (names[k] == r.name) break;
      if (k == names.size()) {
        names.emplace_back(r.name);
        launches.push_back(0);
        ms.push_back(0);
      }
      launches[k] += 1;
      ms[k] += t;
      pool.push_back(r.a);
      pool.push_back(r.b);
    }
    pending.clear();
  }
  void reset() {
    names.clear();
    launches.clear();
    ms.clear();
  }
  ~EventHook() override {
    for (auto &r : pending) {
      (void)hipEventDestroy(r.a);
      (void)hipEventDestroy(r.b);
    }
    for (auto e : pool) (void)hipEventDestroy(e);
  }
};


void split_cell(double X, int *c, float *o) {
  double f = std::floor(X);
  *c = (int)f;
  *o = (float)(X - f);
  if (*o >= 1.0f) {
    *o = 0.0f;
    *c += 1;
  }
}

// Surface-tension strength reported for a step (the kernels evaluate the same ramp in FP32).
double sigma_at(const mpsph_params *p, int64_t step, int64_t t0_auto = -1) {
  int64_t t0i = p->t0, t1i = p->t1;
  if (p->t0 == -2) {
    if (t0_auto < 0) return p->sigma0;
    const double th = p->theta > 0 ? p->theta : 0.2;
    t0i = t0_auto;
    // the same single-precision rounding as the kernels (round half to even)
    t1i = t0_auto + std::max<int64_t>(1, (int64_t)std::rint((float)th * (float)t0_auto));
  }
  if (t0i < 0) return p->sigma0;
  double t = (double)step, t0 = (double)t0i, t1 = (double)t1i;
  if (t <= t0) return p->sigma0;
  if (t <= t1) return p->sigma0 * (1.0 - (t - t0) / (t1 - t0));
  return 0.0;
}

// dt2 / dt1: with the velocity reset, v~ = a dt1 / 2 (Eq. 26) and nu = nu_coeff r_c |v~| (Eq. 21),
// so the three criteria of Eq. 29 are c_acc sqrt(m), (2 c_vel / dt1) m and
// (2 c_visc / (nu_coeff dt1)) m in m = r_c / |a|; their minima over the particles are reached at
// the same m = (dt1 / c_acc)^2, which gives dt2 = dt1 min(1, 2 min(c_vel, c_visc/nu_coeff) / c_acc^2).
double dt2_factor(const mpsph_params *p) {
  double c = p->c_vel;
  if (p->nu_coeff > 0) c = std::min(c, p->c_visc / p->nu_coeff);
  return std::min(1.0, 2.0 * c / (p->c_acc * p->c_acc));
}

// One domain of a context: its parameters (RBF arrays copied), derived grid and device constants.
struct Domain {
  mpsph_params p{};
  std::vector<double> rbf_centre, rbf_coeff;
  Derived d{};
  double s0 = 0;
  int64_t n = 0, off = 0;
  uint32_t ncells = 0, cellbase = 0;
  int blk0 = 0, nblk = 0, row0 = 0, nrow = 0;
  size_t rbf0 = 0;  // first RBF term of this domain in the packed RBF arrays
  std::vector<double> gphi, gs;  // background-mesh node values (level set, field)
  size_t gphi0 = 0, gs0 = 0;     // first node of this domain in the packed device arrays
  int uidx = 0;     // index of the domain in the caller's list
  int64_t uoff = 0, xoff = 0;  // first row / first float of the domain in the caller's arrays

  Domain() = default;
  Domain(const Domain &o) { *this = o; }
  Domain(Domain &&o) noexcept = default;
  Domain &operator=(Domain &&o) noexcept = default;
  // p's RBF pointers refer to this domain's own copies of the arrays
  Domain &operator=(const Domain &o) {
    if (this == &o) return *this;
    p = o.p;
    rbf_centre = o.rbf_centre;
    rbf_coeff = o.rbf_coeff;
    d = o.d;
    s0 = o.s0;
    n = o.n;
    off = o.off;
    ncells = o.ncells;
    cellbase = o.cellbase;
    blk0 = o.blk0;
    nblk = o.nblk;
    row0 = o.row0;
    nrow = o.nrow;
    rbf0 = o.rbf0;
    gphi = o.gphi;
    gs = o.gs;
    gphi0 = o.gphi0;
    gs0 = o.gs0;
    uidx = o.uidx;
    uoff = o.uoff;
    xoff = o.xoff;
    if (!rbf_centre.empty()) {
      p.rbf_centre = rbf_centre.data();
      p.rbf_coeff = rbf_coeff.data();
    }
    p.grid_phi = gphi.empty() ? nullptr : gphi.data();
    p.grid_s = gs.empty() ? nullptr : gs.data();
    return *this;
  }
};

// Domains of one dimension occupy consecutive internal domain, particle and block ranges.
struct Group {
  int D = 0;
  bool periodic = false;  // some domain of the group is a periodic box
  int d0 = 0, nd = 0;   // internal domains
  int i0 = 0, i1 = 0;   // internal particles
  int b0 = 0, nb = 0;   // pair-kernel blocks
};

// Parameters copied into a domain; s0 normalised and the grid derived.  n is the domain's count.
int make_domain(const mpsph_params *params, int64_t n, Domain *dm) {
  if (!valid_params(params) || n < 0 || n > (int64_t)1 << 30) return MPSPH_E_INVALID;
  dm->p = *params;
  dm->n = n;
  if (params->field == MPSPH_RBF_EXP && params->n_rbf > 0) {
    dm->rbf_centre.assign(params->rbf_centre, params->rbf_centre + params->n_rbf * params->dim);
    dm->rbf_coeff.assign(params->rbf_coeff, params->rbf_coeff + params->n_rbf);
    dm->p.rbf_centre = dm->rbf_centre.data();
    dm->p.rbf_coeff = dm->rbf_coeff.data();
  } else {
    dm->p.n_rbf = 0;
    dm->p.rbf_centre = nullptr;
    dm->p.rbf_coeff = nullptr;
  }
  size_t nodes = 1;
  for (int a = 0; a < params->dim; ++a) nodes *= (size_t)std::max(params->grid_n[a], 1);
  dm->gphi.clear();
  dm->gs.clear();
  if (params->geometry == MPSPH_LEVELSET) dm->gphi.assign(params->grid_phi, params->grid_phi + nodes);
  if (params->field == MPSPH_GRID) dm->gs.assign(params->grid_s, params->grid_s + nodes);
  dm->p.grid_phi = dm->gphi.empty() ? nullptr : dm->gphi.data();
  dm->p.grid_s = dm->gs.empty() ? nullptr : dm->gs.data();
  double s0 = params->s0;
  if (!(s0 > 0)) {
    double I = field_integral_unit(&dm->p);
    if (!(I > 0) || !std::isfinite(I)) return MPSPH_E_INVALID;
    s0 = std::pow(I / (double)std::max<int64_t>(n, 1), 1.0 / params->dim);
  }
  dm->s0 = s0;
  int rc = derive(&dm->p, n, s0, &dm->d);
  if (rc) return rc;
  dm->ncells = (uint32_t)1u << (params->dim * dm->d.k + dm->d.xe);
  return MPSPH_OK;
}

// Workspace layout of a context (byte offsets, 256-aligned).
struct Layout {
  int ndom = 0;
  Group grp[2];  // 2D domains, then 3D domains
  std::vector<int> internal;  // caller's domain index -> internal index
  int64_t n = 0;
  uint32_t ncells = 0;  // cells of all domains
  int key_bits = 0;
  int nblocks_pair = 0, nrows = 0;
  int lanes = MPSPH_LANES;  // lanes per particle in the forward pair kernels
  int64_t chunk = 1;  // block partials per first-level reduction row
  size_t n_rbf = 0;
  size_t bytes = 0;
  size_t s_key, s_off, s_ct, s_id, w_key, w_pos, w_jaux, w_id, k0, v0, k1, v1, hist, cstart, acc, rho, nn, aabs, at, v,
      dr, partials, partials2, groups, metrics, dtslots, stepctr, bad, paircount, queue, doms, vscale, rbf_c, rbf_o, rbf_k,
      gphi, gs, gaps, gcount;
};

// Orders the domains internally (2D before 3D, otherwise as given), assigns particle offsets,
// cell bases, pair-kernel blocks (lanes per particle) and reduction rows, and lays out the
// workspace.  doms must be in the caller's order.
int plan(std::vector<Domain> &doms, int lanes, Layout *out) {
  Layout L;
  L.ndom = (int)doms.size();
  L.lanes = lanes;
  int64_t uoff = 0, xoff = 0;
  for (int d = 0; d < L.ndom; ++d) {
    doms[d].uidx = d;
    doms[d].uoff = uoff;
    doms[d].xoff = xoff;
    uoff += doms[d].n;
    xoff += doms[d].n * doms[d].p.dim;
  }
  std::stable_sort(doms.begin(), doms.end(), [](const Domain &a, const Domain &b) { return a.p.dim < b.p.dim; });
  L.internal.assign(L.ndom, 0);
  for (int d = 0; d < L.ndom; ++d) L.internal[doms[d].uidx] = d;
  uint64_t cells = 0;
  int64_t n = 0;
  int64_t blocks = 0;
  size_t nrbf = 0, ngphi = 0, ngs = 0;
  for (int gi = 0; gi < 2; ++gi) {
    L.grp[gi].D = 2 + gi;
    L.grp[gi].d0 = 0;
  }
  for (int d = 0; d < L.ndom; ++d) {
    Domain &dm = doms[d];
    Group &g = L.grp[dm.p.dim - 2];
    if (g.nd == 0) {
      g.d0 = d;
      g.i0 = g.i1 = (int)n;
      g.b0 = (int)blocks;
    }
    dm.off = n;
    dm.cellbase = (uint32_t)cells;
    dm.blk0 = (int)blocks;
    dm.nblk = (int)((dm.n * lanes + kBlock - 1) / kBlock);
    dm.rbf0 = nrbf;
    dm.gphi0 = ngphi;
    dm.gs0 = ngs;
    ngphi += dm.gphi.size();
    ngs += dm.gs.size();
    n += dm.n;
    cells += dm.ncells;
    blocks += dm.nblk;
    nrbf += (size_t)dm.p.n_rbf;
    // thread indices of the pair kernels (particles x lanes) stay below 2^31
    if (n > ((int64_t)1 << 30) || n * lanes >= ((int64_t)1 << 31) || cells > ((uint64_t)1 << 28) ||
        blocks > ((int64_t)1 << 30))
      return MPSPH_E_UNSUPPORTED;
    g.nd += 1;
    g.i1 = (int)n;
    g.nb += dm.nblk;
    g.periodic |= dm.p.geometry == MPSPH_PERIODIC;
  }
  // first-level reduction: rows of at most `chunk` block partials, never straddling domains
  const int64_t chunk = std::max<int64_t>(1, (blocks + kReduceBlocks - 1) / kReduceBlocks);
  int rows = 0;
  for (auto &dm : doms) {
    dm.row0 = rows;
    dm.nrow = (int)((dm.nblk + chunk - 1) / chunk);
    rows += dm.nrow;
  }
  L.n = n;
  L.ncells = (uint32_t)cells;
  L.key_bits = 1;
  while (((uint64_t)1 << L.key_bits) < cells) ++L.key_bits;
  L.nblocks_pair = (int)blocks;
  L.nrows = rows;
  L.chunk = chunk;
  L.n_rbf = nrbf;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o += align_up(std::max<size_t>(bytes, 4));
    return at;
  };
  const size_t nn = (size_t)std::max<int64_t>(n, 1);
  L.s_key = take(nn * 4);
  L.s_off = take(nn * 16);
  L.s_ct = take(nn * 4);
  L.s_id = take(nn * 4);
  L.w_key = take(nn * 4);
  L.w_pos = take(nn * 16);
  L.w_jaux = take(nn * 4);
  L.w_id = take(nn * 4);
  L.k0 = take(nn * 4);
  L.v0 = take(nn * 4);
  L.k1 = take(nn * 4);
  L.v1 = take(nn * 4);
  L.hist = take(radix_hist_words((int)n) * 4);
  L.cstart = take(((size_t)L.ncells + 1) * 4);
  L.gaps = take((nn + 1) * sizeof(uint4));   // at most one empty-cell run per sorted particle
  L.gcount = take(8);                       // run count, finished blocks of fill_gaps
  L.acc = take(nn * 16);
  L.rho = take(nn * 4);
  L.nn = take(nn * 4);
  L.aabs = take(nn * 4);
  L.at = take(nn * 16);
  L.v = take(nn * 16);
  L.dr = take(nn * 16);
  L.partials = take((size_t)std::max(L.nblocks_pair, 1) * kNumPartials * 8);
  L.partials2 = take((size_t)std::max(L.nrows, 1) * kNumPartials * 8);
  L.groups = take((size_t)std::max(L.nrows, 1) * sizeof(int2));
  L.metrics = take((size_t)L.ndom * 32 * 8);
  L.dtslots = take((size_t)L.ndom * kDtSlots * 4);
  L.stepctr = take(8);
  L.bad = take(4);
  L.paircount = take(8);
  L.queue = take(32 * 4);                   // work queues of the persistent pair passes (2 x 16 words)
  L.doms = take((size_t)L.ndom * sizeof(DomDev));
  L.vscale = take((size_t)L.ndom * 4);
  L.rbf_c = take(std::max<size_t>(nrbf, 1) * 3 * 4);
  L.rbf_o = take(std::max<size_t>(nrbf, 1) * 3 * 4);
  L.rbf_k = take(std::max<size_t>(nrbf, 1) * 4);
  L.gphi = take(std::max<size_t>(ngphi, 1) * 4);
  L.gs = take(std::max<size_t>(ngs, 1) * 4);
  L.bytes = o;
  *out = L;
  return MPSPH_OK;
}

// Device constants of a domain (grid, region and field in cell units; step constants).
DomDev domain_device(const Domain &dm, const int *rbf_c, const float *rbf_o, const float *rbf_k, const float *gphi,
                     const float *gsv) {
  const mpsph_params &p = dm.p;
  const double cs = dm.d.cs, ics = dm.d.inv_cs;
  const int D = p.dim;
  DomDev dd;
  std::memset(&dd, 0, sizeof(dd));
  GridDev &g = dd.g;
  g.k = dm.d.k;
  g.n = (int)(dm.off + dm.n);
  g.gmax = dm.d.gmax;
  g.xmask = (uint32_t)dm.d.gmax;
  g.geometry = p.geometry;
  for (int a = 0; a < 3; ++a) {
    double Xhi = a < D ? (p.hi[a] - p.lo[a]) * ics : 0.0;
    split_cell(Xhi, &g.whi_c[a], &g.whi_o[a]);
    if (g.whi_c[a] > g.gmax) {
      g.whi_c[a] = g.gmax;
      g.whi_o[a] = 0.f;
    }
    double Xc = a < D ? (p.centre[a] - p.lo[a]) * ics : 0.0;
    split_cell(Xc, &g.gc_c[a], &g.gc_o[a]);
  }
  g.r_in = (float)(p.r_in * ics);
  g.r_out = (float)(p.r_out * ics);
  g.seeded = p.seeded ? 1 : 0;
  // 3D row tiles of 16 x 16 rows (fewer when the grid is smaller)
  g.xe = (uint32_t)dm.d.xe;
  g.ly = D == 3 ? (uint32_t)std::min(MPSPH_TILE_LY, g.k) : 0u;
  g.lz = D == 3 ? (uint32_t)std::min(MPSPH_TILE_LZ, g.k) : 0u;
  // background mesh: node spacing (hi - lo) / (n - 1) in cell units
  for (int a = 0; a < 3; ++a) {
    const int na = a < D ? std::max(p.grid_n[a], 2) : 2;
    g.gn[a] = na;
    g.ginv[a] = a < D ? (double)(na - 1) / ((p.hi[a] - p.lo[a]) * ics) : 1.0;
  }
  g.phi = p.geometry == MPSPH_LEVELSET ? gphi + dm.gphi0 : nullptr;
  FieldDev &f = dd.f;
  f.kind = p.field;
  f.s0 = (float)(dm.s0 * ics);
  f.g = (float)(p.fa * cs);
  f.b = (float)(p.fb * ics);
  for (int a = 0; a < 3; ++a) {
    double Xc = a < D ? (p.fcentre[a] - p.lo[a]) * ics : 0.0;
    split_cell(Xc, &f.fc_c[a], &f.fc_o[a]);
  }
  f.n_rbf = p.n_rbf;
  f.e2 = p.field == MPSPH_RBF_EXP ? (float)(cs * cs / (2.0 * p.rbf_width * p.rbf_width)) : 0.f;
  f.rbf_c = rbf_c + 3 * dm.rbf0;
  f.rbf_o = rbf_o + 3 * dm.rbf0;
  f.rbf_k = rbf_k + dm.rbf0;
  for (int a = 0; a < 3; ++a) {
    f.gn[a] = g.gn[a];
    f.ginv[a] = g.ginv[a];
  }
  f.gs = p.field == MPSPH_GRID ? gsv + dm.gs0 : nullptr;
  StepDev &sp = dd.sp;
  sp.kappa = (float)p.kappa;
  sp.tau = (float)p.tau;
  sp.inv_tau = (float)(1.0 / p.tau);
  sp.p0c = (float)(p.p0 * std::pow(cs, D - 2));
  sp.nu_coeff = (float)p.nu_coeff;
  sp.c_acc = (float)p.c_acc;
  sp.c_vel = (float)p.c_vel;
  sp.c_visc = (float)p.c_visc;
  sp.search_fac = (float)dm.d.search_fac;
  sp.hmax = (float)(p.tau * dm.d.smax / cs * (1.0 + 1e-5));
  sp.alpha = (float)(D == 2 ? 7.0 / (4.0 * M_PI) : 21.0 / (16.0 * M_PI));
  sp.dt2_factor = (float)dt2_factor(&p);
  sp.sigma0 = (float)p.sigma0;
  sp.t0 = p.t0 < 0 ? -1.f : (float)p.t0;
  sp.t1 = (float)p.t1;
  sp.auto_t0 = p.t0 == -2 ? 1 : 0;
  sp.t0_window = p.t0_window > 0 ? p.t0_window : 50;
  sp.t0_tol = (float)(p.t0_tol > 0 ? p.t0_tol : 1e-3);
  sp.theta = (float)(p.theta > 0 ? p.theta : 0.2);
  dd.cellbase = dm.cellbase;
  dd.off = (int)dm.off;
  dd.n = (int)dm.n;
  dd.uoff = (int)dm.uoff;
  dd.xoff = dm.xoff;
  dd.blk0 = dm.blk0;
  dd.nblk = dm.nblk;
  dd.row0 = dm.row0;
  dd.nrow = dm.nrow;
  for (int a = 0; a < 3; ++a) {
    dd.lo[a] = dm.d.lo[a];
    dd.xhi[a] = dm.d.xhi[a];
  }
  dd.cs = cs;
  dd.inv_cs = ics;
  return dd;
}

}  // namespace

struct mpsph_ctx {
  std::vector<Domain> dom;
  Layout L;
  hipStream_t stream = nullptr;
  char *ws = nullptr;
  size_t ws_cap = 0;  // bytes of the workspace
  bool owns = false;
  bool loaded = false;
  bool poisoned = false;
  int64_t steps_done = 0;
  EventHook hook;
  // step graph: nsteps steps captured once on a private stream, replayed on `stream`
  hipStream_t cap_stream = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  int32_t graph_steps = 0;
  // device memory of the gradient driver (checkpoints, step records, adjoint arrays), grown on
  // demand by mpsph_grad and freed with the context
  char *gmem = nullptr;
  size_t gbytes = 0;
  // device whose static scratch array is the workspace (mpsph_create_static), -1 otherwise
  int static_dev = -1;
  // pair-kernel variant (mpsph_set_pair_variant): MPSPH_PAIRS_DEFAULT, _PERSISTENT or _TILE
  int variant = MPSPH_PAIRS_DEFAULT;
  int cus = 256;   // compute units of the device (the persistent grid holds kQueueBlocksPerCU per CU)
  template <typename T>
  T *at(size_t off) {
    return reinterpret_cast<T *>(ws + off);
  }
};

namespace {

int fail(mpsph_ctx *c, int code) {
  if (c && code == MPSPH_E_DEVICE) c->poisoned = true;
  return code;
}

#define HIP_OK(expr)                                            \
  do {                                                          \
    if ((expr) != hipSuccess) return fail(ctx, MPSPH_E_DEVICE); \
  } while (0)

// Kernels of one step for one dimension group.
template <int D>
void launch_group(mpsph_ctx *ctx, const Group &gr, const uint32_t *skeys, const uint32_t *perm, int nreset,
                  hipStream_t st, EventHook *hk) {
  const Layout &L = ctx->L;
  const int n = (int)L.n;
  const DomDev *doms = ctx->at<DomDev>(L.doms) + gr.d0;
  if (hk) hk->begin("reorder_field");
  const int nthr = std::max(gr.i1 - gr.i0 + (gr.i1 == n ? 1 : 0), nreset);
  reorder_field<D><<<(nthr + kBlock - 1) / kBlock, kBlock, 0, st>>>(
      doms, gr.nd, gr.i0, gr.i1, n, L.ncells, nreset, skeys, perm, ctx->at<float4>(L.s_off), ctx->at<uint32_t>(L.s_ct),
      ctx->at<uint32_t>(L.s_id), ctx->at<uint32_t>(L.w_key), ctx->at<float4>(L.w_pos), ctx->at<uint32_t>(L.w_jaux),
      ctx->at<uint32_t>(L.w_id), ctx->at<uint32_t>(L.cstart), ctx->at<uint32_t>(L.dtslots), ctx->at<uint4>(L.gaps),
      ctx->at<uint32_t>(L.gcount));
  fill_gaps<<<kGapBlocks, 256, 0, st>>>(ctx->at<uint4>(L.gaps), ctx->at<uint32_t>(L.gcount),
                                        ctx->at<uint32_t>(L.gcount) + 1, ctx->at<uint32_t>(L.cstart));
  if (hk) hk->end();
}

template <int D, int L_, bool PER>
void launch_pass1_l(mpsph_ctx *ctx, const Group &gr, hipStream_t st) {
  const Layout &L = ctx->L;
  const bool dbg = ctx->dom[0].p.debug != 0;
  auto kern = dbg ? pass_density_force<D, L_, PER, true> : pass_density_force<D, L_, PER, false>;
  if constexpr (D == 3 && !PER)
    if (ctx->variant == MPSPH_PAIRS_TILE) kern = dbg ? pass_density_force_tile<L_, true> : pass_density_force_tile<L_, false>;
  kern<<<gr.nb, kBlock, 0, st>>>(
      gr.b0, ctx->at<DomDev>(L.doms) + gr.d0, gr.nd, ctx->at<int64_t>(L.stepctr), ctx->at<uint32_t>(L.w_key),
      ctx->at<float4>(L.w_pos), ctx->at<uint32_t>(L.w_jaux), ctx->at<uint32_t>(L.cstart), ctx->at<float4>(L.acc),
      dbg ? ctx->at<float>(L.rho) : nullptr, dbg ? ctx->at<float>(L.nn) : nullptr,
      dbg ? ctx->at<float>(L.aabs) : nullptr, ctx->at<uint32_t>(L.dtslots) + (size_t)gr.d0 * kDtSlots,
      ctx->at<double>(L.metrics) + (size_t)gr.d0 * 32, ctx->at<double>(L.partials));
}

template <int D>
void launch_pass1(mpsph_ctx *ctx, const Group &gr, hipStream_t st, EventHook *hk) {
  if (hk) hk->begin("pass_density_force");
  const int sel = ctx->L.lanes * 2 + (gr.periodic ? 1 : 0);
  switch (sel) {
    case 4: launch_pass1_l<D, 2, false>(ctx, gr, st); break;
    case 5: launch_pass1_l<D, 2, true>(ctx, gr, st); break;
    case 16: launch_pass1_l<D, 8, false>(ctx, gr, st); break;
    case 17: launch_pass1_l<D, 8, true>(ctx, gr, st); break;
    case 9: launch_pass1_l<D, 4, true>(ctx, gr, st); break;
    default: launch_pass1_l<D, 4, false>(ctx, gr, st);
  }
  if (hk) hk->end();
}

template <int D, int L_, bool PER>
void launch_pass2_l(mpsph_ctx *ctx, const Group &gr, hipStream_t st, float4 *at_o, float4 *v_o) {
  const Layout &L = ctx->L;
  const bool dbg = ctx->dom[0].p.debug != 0;
  pass_viscous_integrate<D, L_, PER><<<gr.nb, kBlock, 0, st>>>(
      gr.b0, ctx->at<DomDev>(L.doms) + gr.d0, gr.nd, ctx->at<uint32_t>(L.w_key), ctx->at<float4>(L.w_pos),
      ctx->at<uint32_t>(L.w_jaux), ctx->at<uint32_t>(L.w_id), ctx->at<uint32_t>(L.cstart), ctx->at<float4>(L.acc),
      ctx->at<uint32_t>(L.dtslots) + (size_t)gr.d0 * kDtSlots, ctx->at<uint32_t>(L.s_key), ctx->at<float4>(L.s_off),
      ctx->at<uint32_t>(L.s_ct), ctx->at<uint32_t>(L.s_id), at_o, v_o, dbg ? ctx->at<float4>(L.dr) : nullptr,
      ctx->at<double>(L.partials));
}

template <int D>
void launch_pass2(mpsph_ctx *ctx, const Group &gr, hipStream_t st, EventHook *hk, float4 *at_rec = nullptr,
                  float4 *v_rec = nullptr) {
  const Layout &L = ctx->L;
  const bool dbg = ctx->dom[0].p.debug != 0;
  float4 *at_o = at_rec ? at_rec : (dbg ? ctx->at<float4>(L.at) : nullptr);
  float4 *v_o = v_rec ? v_rec : (dbg ? ctx->at<float4>(L.v) : nullptr);
  if (hk) hk->begin("pass_viscous_integrate");
  const int sel = L.lanes * 2 + (gr.periodic ? 1 : 0);
  switch (sel) {
    case 4: launch_pass2_l<D, 2, false>(ctx, gr, st, at_o, v_o); break;
    case 5: launch_pass2_l<D, 2, true>(ctx, gr, st, at_o, v_o); break;
    case 16: launch_pass2_l<D, 8, false>(ctx, gr, st, at_o, v_o); break;
    case 17: launch_pass2_l<D, 8, true>(ctx, gr, st, at_o, v_o); break;
    case 9: launch_pass2_l<D, 4, true>(ctx, gr, st, at_o, v_o); break;
    default: launch_pass2_l<D, 4, false>(ctx, gr, st, at_o, v_o);
  }
  if (hk) hk->end();
}

// Persistent launches of the pair passes (pair-kernel variant MPSPH_PAIRS_PERSISTENT; see
// pass_density_force_queue): one launch per pass serves both dimension groups.
constexpr int kQueueBlocksPerCU = 8;   // blocks of the pair kernels resident per CU (8 waves per SIMD)
int queue_grid(const mpsph_ctx *ctx, int nb) { return std::max(1, std::min(nb, ctx->cus * kQueueBlocksPerCU)); }

template <int DM, int L_, bool PER>
void launch_pass1_queue_l(mpsph_ctx *ctx, int b0, int nb2, int nb, hipStream_t st) {
  const Layout &L = ctx->L;
  const bool dbg = ctx->dom[0].p.debug != 0;
  auto kern = dbg ? pass_density_force_queue<DM, L_, PER, true> : pass_density_force_queue<DM, L_, PER, false>;
  kern<<<queue_grid(ctx, nb), kBlock, 0, st>>>(
      b0, nb2, nb, ctx->at<uint32_t>(L.queue), ctx->at<DomDev>(L.doms), L.ndom, ctx->at<int64_t>(L.stepctr),
      ctx->at<uint32_t>(L.w_key), ctx->at<float4>(L.w_pos), ctx->at<uint32_t>(L.w_jaux), ctx->at<uint32_t>(L.cstart),
      ctx->at<float4>(L.acc), dbg ? ctx->at<float>(L.rho) : nullptr, dbg ? ctx->at<float>(L.nn) : nullptr,
      dbg ? ctx->at<float>(L.aabs) : nullptr, ctx->at<uint32_t>(L.dtslots), ctx->at<double>(L.metrics),
      ctx->at<double>(L.partials));
}

template <int DM, int L_, bool PER>
void launch_pass2_queue_l(mpsph_ctx *ctx, int b0, int nb2, int nb, hipStream_t st) {
  const Layout &L = ctx->L;
  const bool dbg = ctx->dom[0].p.debug != 0;
  pass_viscous_integrate_queue<DM, L_, PER><<<queue_grid(ctx, nb), kBlock, 0, st>>>(
      b0, nb2, nb, ctx->at<uint32_t>(L.queue) + 16, ctx->at<DomDev>(L.doms), L.ndom, ctx->at<uint32_t>(L.w_key),
      ctx->at<float4>(L.w_pos), ctx->at<uint32_t>(L.w_jaux), ctx->at<uint32_t>(L.w_id), ctx->at<uint32_t>(L.cstart),
      ctx->at<float4>(L.acc), ctx->at<uint32_t>(L.dtslots), ctx->at<uint32_t>(L.s_key), ctx->at<float4>(L.s_off),
      ctx->at<uint32_t>(L.s_ct), ctx->at<uint32_t>(L.s_id), dbg ? ctx->at<float4>(L.at) : nullptr,
      dbg ? ctx->at<float4>(L.v) : nullptr, dbg ? ctx->at<float4>(L.dr) : nullptr, ctx->at<double>(L.partials));
}

template <int DM>
void launch_queue_dm(mpsph_ctx *ctx, int pass, int b0, int nb2, int nb, bool per, hipStream_t st) {
  const int sel = ctx->L.lanes * 2 + (per ? 1 : 0);
#define MPSPH_QUEUE_CASE(LN, P)                                 \
  if (pass == 1) launch_pass1_queue_l<DM, LN, P>(ctx, b0, nb2, nb, st); \
  else launch_pass2_queue_l<DM, LN, P>(ctx, b0, nb2, nb, st);
  switch (sel) {
    case 4: MPSPH_QUEUE_CASE(2, false) break;
    case 5: MPSPH_QUEUE_CASE(2, true) break;
    case 16: MPSPH_QUEUE_CASE(8, false) break;
    case 17: MPSPH_QUEUE_CASE(8, true) break;
    case 9: MPSPH_QUEUE_CASE(4, true) break;
    default: MPSPH_QUEUE_CASE(4, false)
  }
#undef MPSPH_QUEUE_CASE
}

void launch_pairs_queue(mpsph_ctx *ctx, hipStream_t st, EventHook *hk) {
  const Layout &L = ctx->L;
  const Group &g2 = L.grp[0], &g3 = L.grp[1];
  for (int pass = 1; pass <= 2; ++pass) {
    if (hk) hk->begin(pass == 1 ? "pass_density_force" : "pass_viscous_integrate");
    if (g2.nb > 0 && g3.nb > 0) {
      launch_queue_dm<5>(ctx, pass, 0, g2.nb, g2.nb + g3.nb, g2.periodic || g3.periodic, st);
    } else {
      if (g2.nb > 0) launch_queue_dm<2>(ctx, pass, g2.b0, g2.nb, g2.nb, g2.periodic, st);
      if (g3.nb > 0) launch_queue_dm<3>(ctx, pass, g3.b0, 0, g3.nb, g3.periodic, st);
    }
    if (hk) hk->end();
  }
}

// Enqueues nsteps steps of every domain on stream st.  No host synchronisation, no memset and
// no host-side state read, so the same launches can be captured into a graph and replayed.
// Each kernel is launched once per non-empty dimension group.
int enqueue(mpsph_ctx *ctx, int nsteps, hipStream_t st, EventHook *hk) {
  const Layout &L = ctx->L;
  const int n = (int)L.n, ndom = L.ndom;
  for (int s = 0; s < nsteps; ++s) {
    if (n > 0) {
      const uint32_t *skeys = nullptr, *perm = nullptr;
      if (radix_sort(ctx->at<uint32_t>(L.s_key), ctx->at<uint32_t>(L.k0), ctx->at<uint32_t>(L.v0),
                     ctx->at<uint32_t>(L.k1), ctx->at<uint32_t>(L.v1), ctx->at<uint32_t>(L.hist), n, L.key_bits, st,
                     &skeys, &perm, hk) != hipSuccess)
        return fail(ctx, MPSPH_E_DEVICE);
      int nreset = ndom * kDtSlots;  // the first launch resets every domain's time-step slots
      for (const Group &gr : L.grp) {
        if (gr.i1 <= gr.i0) continue;
        if (gr.D == 2) launch_group<2>(ctx, gr, skeys, perm, nreset, st, hk);
        else launch_group<3>(ctx, gr, skeys, perm, nreset, st, hk);
        nreset = 0;
      }
      if (ctx->variant == MPSPH_PAIRS_PERSISTENT) {
        launch_pairs_queue(ctx, st, hk);
      } else {
        for (const Group &gr : L.grp) {
          if (gr.nb <= 0) continue;
          if (gr.D == 2) launch_pass1<2>(ctx, gr, st, hk);
          else launch_pass1<3>(ctx, gr, st, hk);
        }
        for (const Group &gr : L.grp) {
          if (gr.nb <= 0) continue;
          if (gr.D == 2) launch_pass2<2>(ctx, gr, st, hk);
          else launch_pass2<3>(ctx, gr, st, hk);
        }
      }
    }
    if (hk) hk->begin("finalize");
    if (L.nrows > 0)
      reduce_partials<<<L.nrows, 256, 0, st>>>(ctx->at<int2>(L.groups), ctx->at<double>(L.partials),
                                               ctx->at<double>(L.partials2));
    finalize<<<ndom, 256, 0, st>>>(ctx->at<DomDev>(L.doms), ctx->at<double>(L.partials2), ctx->at<uint32_t>(L.dtslots),
                                   ctx->at<double>(L.metrics), ctx->at<int64_t>(L.stepctr));
    if (hk) hk->end();
    if (hipGetLastError() != hipSuccess) return fail(ctx, MPSPH_E_DEVICE);
  }
  return MPSPH_OK;
}

void drop_graph(mpsph_ctx *ctx) {
  if (ctx->graph_exec) (void)hipGraphExecDestroy(ctx->graph_exec);
  ctx->graph_exec = nullptr;
  ctx->graph_steps = 0;
}

void fill_metrics(const mpsph_ctx *ctx, int dmi, const double *m, mpsph_metrics_t *out) {
  const Domain &dm = ctx->dom[dmi];
  const double cs = dm.d.cs;
  std::memset(out, 0, sizeof(*out));
  out->step = ctx->steps_done - 1;
  out->pairs = (int64_t)m[P_PAIRS];
  out->interface_pairs = (int64_t)m[P_IFC] / 2;
  out->candidates = (int64_t)m[P_CAND];
  out->n_normal = (int64_t)m[P_NNORM];
  out->n_elr = (int64_t)m[P_NELR];
  out->nonfinite = (int64_t)(m[P_NONFIN1] + m[P_NONFIN2]);
  out->n_feature = (int64_t)m[P_NFEAT];
  out->residual_l2 = m[P_NNORM] > 0 ? std::sqrt(m[P_E2] / m[P_NNORM]) : 0.0;
  out->residual_linf = m[P_EMAX];
  out->pairs_total = (int64_t)m[18];
  out->candidates_total = (int64_t)m[19];
  out->kinetic = m[P_KE] * cs * cs;
  out->dt1 = m[16];
  out->dt2 = m[17];
  const int64_t t0a = m[kAutoT0] > 0 ? (int64_t)m[kAutoT0] - 1 : -1;
  out->sigma = sigma_at(&dm.p, std::max<int64_t>(ctx->steps_done - 1, 0), t0a);
  out->interface_particles = (int64_t)m[P_IFCP];
  out->t0 = dm.p.t0 == -2 ? t0a : dm.p.t0;
  if (m[P_NELR] > 0) {
    double mean = m[P_ELR] / m[P_NELR];
    out->elr_mean = mean;
    out->elr_std = std::sqrt(std::max(0.0, m[P_ELR2] / m[P_NELR] - mean * mean));
    out->elr_min = m[P_ELRMIN];
    out->elr_max = m[P_ELRMAX];
  }
}

int batch_check(int32_t ndom, const mpsph_params *params, const int64_t *n) {
  if (ndom < 1 || ndom > 4096 || !params || !n) return MPSPH_E_INVALID;
  for (int d = 0; d < ndom; ++d) {
    if (!valid_params(&params[d]) || n[d] < 0 || n[d] > (int64_t)1 << 30) return MPSPH_E_INVALID;
    if (params[d].debug != params[0].debug) return MPSPH_E_INVALID;
  }
  return MPSPH_OK;
}

int build_domains(int32_t ndom, const mpsph_params *params, const int64_t *n, std::vector<Domain> *doms, Layout *L) {
  int rc = batch_check(ndom, params, n);
  if (rc) return rc;
  doms->resize(ndom);
  for (int d = 0; d < ndom; ++d)
    if ((rc = make_domain(&params[d], n[d], &(*doms)[d])) != MPSPH_OK) return rc;
  return plan(*doms, MPSPH_LANES, L);
}

// Re-derives every domain's cell grid -- the cell exponent of the size rule plus kdelta for
// domains whose cell_log2 was left to the library, the caller's value otherwise -- and plans
// the workspace for `lanes` lanes per particle.
int replan(std::vector<Domain> &doms, int kdelta, int lanes, Layout *L, int kabs = -1) {
  std::stable_sort(doms.begin(), doms.end(), [](const Domain &a, const Domain &b) { return a.uidx < b.uidx; });
  for (auto &dm : doms) {
    mpsph_params q = dm.p;
    if (kabs >= 1) {
      q.cell_log2 = kabs;
    } else if (q.cell_log2 < 0) {
      Derived r;
      int rc = derive(&q, dm.n, dm.s0, &r);
      if (rc) return rc;
      q.cell_log2 = std::min(std::max(r.k + kdelta, 1), q.dim == 3 ? 8 : 12);
    }
    int rc = derive(&q, dm.n, dm.s0, &dm.d);
    if (rc) return rc;
    dm.ncells = (uint32_t)1u << (q.dim * dm.d.k + dm.d.xe);
  }
  return plan(doms, lanes, L);
}


// Zeroes the workspace and uploads the domain table, the reduction row groups and the RBF
// terms of the current layout.
int setup_device(mpsph_ctx *ctx) {
  const Layout &L = ctx->L;
  const int ndom = L.ndom;
  // a zeroed workspace keeps every table entry a valid index before its first write
  HIP_OK(hipMemset(ctx->ws, 0, L.bytes));
  std::vector<DomDev> dd(ndom);
  std::vector<int2> groups;
  std::vector<int> rc3(3 * std::max<size_t>(L.n_rbf, 1), 0);
  std::vector<float> ro3(3 * std::max<size_t>(L.n_rbf, 1), 0.f), rk(std::max<size_t>(L.n_rbf, 1), 0.f);
  for (int d = 0; d < ndom; ++d) {
    const Domain &dm = ctx->dom[d];
    dd[d] = domain_device(dm, ctx->at<int>(L.rbf_c), ctx->at<float>(L.rbf_o), ctx->at<float>(L.rbf_k),
                          ctx->at<float>(L.gphi), ctx->at<float>(L.gs));
    for (int r = 0; r < dm.nrow; ++r) {
      const int64_t a = dm.blk0 + (int64_t)r * L.chunk;
      groups.push_back(make_int2((int)a, (int)std::min<int64_t>(a + L.chunk, dm.blk0 + dm.nblk)));
    }
    for (int t = 0; t < dm.p.n_rbf; ++t) {
      const size_t kk = dm.rbf0 + t;
      for (int a = 0; a < dm.p.dim; ++a)
        split_cell((dm.p.rbf_centre[t * dm.p.dim + a] - dm.p.lo[a]) * dm.d.inv_cs, &rc3[kk * 3 + a], &ro3[kk * 3 + a]);
      rk[kk] = (float)dm.p.rbf_coeff[t];
    }
  }
  HIP_OK(hipMemcpy(ctx->at<DomDev>(L.doms), dd.data(), dd.size() * sizeof(DomDev), hipMemcpyHostToDevice));
  if (!groups.empty())
    HIP_OK(hipMemcpy(ctx->at<int2>(L.groups), groups.data(), groups.size() * sizeof(int2), hipMemcpyHostToDevice));
  HIP_OK(hipMemcpy(ctx->at<int>(L.rbf_c), rc3.data(), rc3.size() * 4, hipMemcpyHostToDevice));
  HIP_OK(hipMemcpy(ctx->at<float>(L.rbf_o), ro3.data(), ro3.size() * 4, hipMemcpyHostToDevice));
  HIP_OK(hipMemcpy(ctx->at<float>(L.rbf_k), rk.data(), rk.size() * 4, hipMemcpyHostToDevice));
  // background-mesh values: the level set in cell units, the field's relative spacing as given
  for (int d = 0; d < ndom; ++d) {
    const Domain &dm = ctx->dom[d];
    if (!dm.gphi.empty()) {
      std::vector<float> v(dm.gphi.size());
      for (size_t k = 0; k < v.size(); ++k) v[k] = (float)(dm.gphi[k] * dm.d.inv_cs);
      HIP_OK(hipMemcpy(ctx->at<float>(L.gphi) + dm.gphi0, v.data(), v.size() * 4, hipMemcpyHostToDevice));
    }
    if (!dm.gs.empty()) {
      std::vector<float> v(dm.gs.begin(), dm.gs.end());
      HIP_OK(hipMemcpy(ctx->at<float>(L.gs) + dm.gs0, v.data(), v.size() * 4, hipMemcpyHostToDevice));
    }
  }
  return MPSPH_OK;
}

// Re-plans the context for a cell size (rule + kdelta, or kabs >= 1 for every domain) and a
// lane count, growing a library-owned workspace when needed, and resets the device tables.
// The loaded state is lost.  A configuration that does not fit a caller workspace returns
// MPSPH_E_NOMEM and leaves the context unchanged.
int reconfigure(mpsph_ctx *ctx, const std::vector<Domain> &base, int kdelta, int kabs, int lanes) {
  std::vector<Domain> doms = base;
  Layout Lc;
  int rc = replan(doms, kdelta, lanes, &Lc, kabs);
  if (rc) return rc;
  if (Lc.bytes > ctx->ws_cap) {
    if (!ctx->owns) return MPSPH_E_NOMEM;
    (void)hipStreamSynchronize(ctx->stream);
    (void)hipFree(ctx->ws);
    ctx->ws = nullptr;
    ctx->ws_cap = 0;
    if (hipMalloc((void **)&ctx->ws, Lc.bytes) != hipSuccess) return fail(ctx, MPSPH_E_DEVICE);
    ctx->ws_cap = Lc.bytes;
  }
  drop_graph(ctx);
  ctx->dom = doms;
  ctx->L = Lc;
  ctx->loaded = false;
  ctx->steps_done = 0;
  return setup_device(ctx);
}

// ------------------------------------------------------------------------------------------
// Gradient driver: forward with checkpoints, loss, and the reverse sweep.  A segment of
// ckpt steps is recomputed from its checkpoint with every step's sorted state and results
// recorded, then its steps are reversed from last to first.
// ------------------------------------------------------------------------------------------

struct GradPlan {
  int nck = 0, ckpt = 0;
  size_t ck0 = 0, ck_stride = 0, ck_key = 0, ck_off = 0, ck_ct = 0, ck_id = 0;
  size_t tp0 = 0, tp_stride = 0, tp_perm = 0, tp_wkey = 0, tp_wpos = 0, tp_wjaux = 0, tp_acc = 0, tp_at = 0,
         tp_v = 0, tp_cstart = 0, tp_dts = 0;
  size_t xbar = 0, xacc = 0, abv = 0, vtb = 0, abar = 0, fbar = 0, sbar = 0, e = 0, dtc = 0, pa = 0, pb = 0,
         cpart = 0, cbar = 0, scal = 0, mback = 0;
  size_t bytes = 0;
};

GradPlan grad_plan(int64_t n, uint32_t ncells, int nck, int ckpt, int nb1, int nbp) {
  GradPlan P;
  P.nck = nck;
  P.ckpt = ckpt;
  const size_t nn = (size_t)std::max<int64_t>(n, 1);
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o += align_up(std::max<size_t>(bytes, 4));
    return at;
  };
  // checkpoint: the state arrays (key, offsets, type | colour, id)
  size_t c = 0;
  auto ctake = [&](size_t bytes) {
    size_t at = c;
    c += align_up(bytes);
    return at;
  };
  P.ck_key = ctake(nn * 4);
  P.ck_off = ctake(nn * 16);
  P.ck_ct = ctake(nn * 4);
  P.ck_id = ctake(nn * 4);
  P.ck_stride = c;
  P.ck0 = take(P.ck_stride * nck);
  size_t t = 0;
  auto ttake = [&](size_t bytes) {
    size_t at = t;
    t += align_up(bytes);
    return at;
  };
  P.tp_perm = ttake(nn * 4);
  P.tp_wkey = ttake(nn * 4);
  P.tp_wpos = ttake(nn * 16);
  P.tp_wjaux = ttake(nn * 4);
  P.tp_acc = ttake(nn * 16);
  P.tp_at = ttake(nn * 16);
  P.tp_v = ttake(nn * 16);
  P.tp_cstart = ttake(((size_t)ncells + 1) * 4);
  P.tp_dts = ttake(kDtSlots * 4);
  P.tp_stride = t;
  P.tp0 = take(P.tp_stride * ckpt);
  P.xbar = take(nn * 16);
  P.xacc = take(nn * 16);
  P.abv = take(nn * 16);
  P.vtb = take(nn * 16);
  P.abar = take(nn * 16);
  P.fbar = take(nn * 16);
  P.sbar = take(nn * 4);
  P.e = take(nn * 4);
  P.dtc = take(nn * 4);
  P.pa = take((size_t)std::max(nb1, 1) * kNumPartials * 8);
  P.pb = take((size_t)std::max(nbp, 1) * kNumPartials * 8);
  P.cpart = take((size_t)std::max(nb1, 1) * kMaxRbf * 8);
  P.cbar = take(kMaxRbf * 8);
  P.scal = take(64);
  P.mback = take(32 * 8);
  P.bytes = o;
  return P;
}

struct GradRun {
  mpsph_ctx *ctx;
  GradPlan P;
  hipStream_t st;
  const Group *gr;
  int nb1;
  int nbp;  // blocks of the adjoint pair kernels (MPSPH_ADJ_LANES lanes per particle)
  char *g;
  template <typename T>
  T *at(size_t off) {
    return reinterpret_cast<T *>(g + off);
  }
  char *ck(int k) { return g + P.ck0 + P.ck_stride * k; }
  char *tp(int m) { return g + P.tp0 + P.tp_stride * m; }
  TapeView view(int m) {
    char *b = tp(m);
    TapeView v;
    v.wkey = reinterpret_cast<const uint32_t *>(b + P.tp_wkey);
    v.wpos = reinterpret_cast<const float4 *>(b + P.tp_wpos);
    v.wjaux = reinterpret_cast<const uint32_t *>(b + P.tp_wjaux);
    v.cstart = reinterpret_cast<const uint32_t *>(b + P.tp_cstart);
    v.perm = reinterpret_cast<const uint32_t *>(b + P.tp_perm);
    v.acc = reinterpret_cast<const float4 *>(b + P.tp_acc);
    v.at = reinterpret_cast<const float4 *>(b + P.tp_at);
    v.v = reinterpret_cast<const float4 *>(b + P.tp_v);
    v.dts = reinterpret_cast<const uint32_t *>(b + P.tp_dts);
    return v;
  }
};

// Copies the context state arrays to (save) or from (restore) checkpoint k.
int copy_state(GradRun &R, int k, bool save) {
  mpsph_ctx *ctx = R.ctx;
  const Layout &L = ctx->L;
  const size_t n = (size_t)L.n;
  char *c = R.ck(k);
  const size_t off_ws[4] = {L.s_key, L.s_off, L.s_ct, L.s_id};
  const size_t off_ck[4] = {R.P.ck_key, R.P.ck_off, R.P.ck_ct, R.P.ck_id};
  const size_t sz[4] = {n * 4, n * 16, n * 4, n * 4};
  for (int a = 0; a < 4; ++a) {
    void *ws = ctx->ws + off_ws[a];
    void *cp = c + off_ck[a];
    HIP_OK(hipMemcpyAsync(save ? cp : ws, save ? ws : cp, sz[a], hipMemcpyDeviceToDevice, R.st));
  }
  return MPSPH_OK;
}

// One forward step of the single domain with its record in step slot m.
template <int D>
int record_step(GradRun &R, int m) {
  mpsph_ctx *ctx = R.ctx;
  const Layout &L = ctx->L;
  const int n = (int)L.n;
  const uint32_t *skeys = nullptr, *perm = nullptr;
  if (radix_sort(ctx->at<uint32_t>(L.s_key), ctx->at<uint32_t>(L.k0), ctx->at<uint32_t>(L.v0), ctx->at<uint32_t>(L.k1),
                 ctx->at<uint32_t>(L.v1), ctx->at<uint32_t>(L.hist), n, L.key_bits, R.st, &skeys, &perm,
                 nullptr) != hipSuccess)
    return fail(ctx, MPSPH_E_DEVICE);
  char *b = R.tp(m);
  launch_group<D>(ctx, *R.gr, skeys, perm, kDtSlots, R.st, nullptr);
  launch_pass1<D>(ctx, *R.gr, R.st, nullptr);
  launch_pass2<D>(ctx, *R.gr, R.st, nullptr, reinterpret_cast<float4 *>(b + R.P.tp_at),
                  reinterpret_cast<float4 *>(b + R.P.tp_v));
  if (L.nrows > 0)
    reduce_partials<<<L.nrows, 256, 0, R.st>>>(ctx->at<int2>(L.groups), ctx->at<double>(L.partials),
                                                 ctx->at<double>(L.partials2));
  finalize<<<1, 256, 0, R.st>>>(ctx->at<DomDev>(L.doms), ctx->at<double>(L.partials2), ctx->at<uint32_t>(L.dtslots),
                                ctx->at<double>(L.metrics), ctx->at<int64_t>(L.stepctr));
  HIP_OK(hipGetLastError());
  const size_t nn = (size_t)n;
  HIP_OK(hipMemcpyAsync(b + R.P.tp_perm, perm, nn * 4, hipMemcpyDeviceToDevice, R.st));
  HIP_OK(hipMemcpyAsync(b + R.P.tp_wkey, ctx->at<uint32_t>(L.w_key), nn * 4, hipMemcpyDeviceToDevice, R.st));
  HIP_OK(hipMemcpyAsync(b + R.P.tp_wpos, ctx->at<float4>(L.w_pos), nn * 16, hipMemcpyDeviceToDevice, R.st));
  HIP_OK(hipMemcpyAsync(b + R.P.tp_wjaux, ctx->at<uint32_t>(L.w_jaux), nn * 4, hipMemcpyDeviceToDevice, R.st));
  HIP_OK(hipMemcpyAsync(b + R.P.tp_acc, ctx->at<float4>(L.acc), nn * 16, hipMemcpyDeviceToDevice, R.st));
  HIP_OK(hipMemcpyAsync(b + R.P.tp_cstart, ctx->at<uint32_t>(L.cstart), ((size_t)L.ncells + 1) * 4,
                        hipMemcpyDeviceToDevice, R.st));
  HIP_OK(hipMemcpyAsync(b + R.P.tp_dts, ctx->at<uint32_t>(L.dtslots), kDtSlots * 4, hipMemcpyDeviceToDevice, R.st));
  return MPSPH_OK;
}

// Adjoint of the loss at the current state: x-bar (previous state order) and c-bar.
template <int D>
int loss_backward(GradRun &R, double lam) {
  mpsph_ctx *ctx = R.ctx;
  const Layout &L = ctx->L;
  const Domain &dm = ctx->dom[0];
  const int n = (int)L.n;
  const DomDev *dom = ctx->at<DomDev>(L.doms);
  const uint32_t *skeys = nullptr, *perm = nullptr;
  if (radix_sort(ctx->at<uint32_t>(L.s_key), ctx->at<uint32_t>(L.k0), ctx->at<uint32_t>(L.v0), ctx->at<uint32_t>(L.k1),
                 ctx->at<uint32_t>(L.v1), ctx->at<uint32_t>(L.hist), n, L.key_bits, R.st, &skeys, &perm,
                 nullptr) != hipSuccess)
    return fail(ctx, MPSPH_E_DEVICE);
  launch_group<D>(ctx, *R.gr, skeys, perm, kDtSlots, R.st, nullptr);
  const int nbp = R.nbp;
  loss_density<D, MPSPH_ADJ_LANES><<<nbp, kBlock, 0, R.st>>>(dom, ctx->at<uint32_t>(L.w_key), ctx->at<float4>(L.w_pos),
                                                       ctx->at<uint32_t>(L.w_jaux), ctx->at<uint32_t>(L.cstart),
                                                       R.at<float>(R.P.e), R.at<double>(R.P.pb));
  loss_value<<<1, 256, 0, R.st>>>(R.at<double>(R.P.pb), nbp, 1.0 / n, lam, R.at<double>(R.P.scal) + 1);
  // every neighbour j whose support reaches k: r < kappa h_j <= kappa h_k / (1 - kappa L_h)
  const double Lh = dm.p.tau * dm.d.lip;
  const double kl = dm.p.kappa * Lh;
  const float reach = kl < 0.95 ? (float)(dm.p.kappa / (1.0 - kl) * (1.0 + 1e-4)) : 1e30f;
  loss_grad<D, MPSPH_ADJ_LANES><<<nbp, kBlock, 0, R.st>>>(dom, ctx->at<uint32_t>(L.w_key), ctx->at<float4>(L.w_pos),
                                                    ctx->at<uint32_t>(L.w_jaux), ctx->at<uint32_t>(L.cstart),
                                                    R.at<float>(R.P.e), (float)(2.0 / n), (float)(lam / n), reach,
                                                    R.at<float4>(R.P.xacc), R.at<float>(R.P.sbar));
  TapeView tv{};
  tv.wkey = ctx->at<uint32_t>(L.w_key);
  tv.wpos = ctx->at<float4>(L.w_pos);
  tv.perm = perm;
  adj_field<D><<<R.nb1, kBlock, 0, R.st>>>(dom, tv, R.at<float4>(R.P.xacc), R.at<float>(R.P.sbar),
                                           R.at<float4>(R.P.xbar), R.at<double>(R.P.cpart));
  if (dm.p.field == MPSPH_RBF_EXP && dm.p.n_rbf > 0)
    adj_sum_coeff<<<std::max(dm.p.n_rbf, 1), kCoeffSumThreads, 0, R.st>>>(R.at<double>(R.P.cpart), R.nb1, dm.p.n_rbf,
                                                                        R.at<double>(R.P.cbar));
  HIP_OK(hipGetLastError());
  return MPSPH_OK;
}

// Reverse of the recorded step m (step index t of the run).
template <int D>
int step_backward(GradRun &R, int m, int64_t t) {
  mpsph_ctx *ctx = R.ctx;
  const Layout &L = ctx->L;
  const Domain &dm = ctx->dom[0];
  const DomDev *dom = ctx->at<DomDev>(L.doms);
  const TapeView tv = R.view(m);
  const int nbp = R.nbp;
  uint32_t *minbits = reinterpret_cast<uint32_t *>(R.at<char>(R.P.scal) + 32);
  uint32_t *argmin = minbits + 1;
  double *t1bar = R.at<double>(R.P.scal);
  adj_init<<<1, 1, 0, R.st>>>(minbits, argmin);
  adj_drift<D><<<R.nb1, kBlock, 0, R.st>>>(dom, tv, R.at<float4>(R.P.xbar), R.at<float4>(R.P.xacc),
                                           R.at<float4>(R.P.abv), R.at<float4>(R.P.vtb), R.at<float>(R.P.dtc), minbits,
                                           R.at<double>(R.P.pa));
  adj_visc<D, MPSPH_ADJ_LANES><<<nbp, kBlock, 0, R.st>>>(dom, tv, R.at<float4>(R.P.abv), R.at<float4>(R.P.vtb),
                                                   R.at<float4>(R.P.xacc), R.at<float>(R.P.sbar),
                                                   R.at<float4>(R.P.abar), R.at<float>(R.P.dtc), minbits, argmin,
                                                   R.at<double>(R.P.pb));
  adj_sum_dt<<<1, 256, 0, R.st>>>(R.at<double>(R.P.pa), R.nb1, R.at<double>(R.P.pb), nbp,
                                  (float)dt2_factor(&dm.p), t1bar);
  adj_fbar<D><<<R.nb1, kBlock, 0, R.st>>>(dom, tv, R.at<float4>(R.P.abar), t1bar, argmin, R.at<float>(R.P.sbar),
                                          R.at<float4>(R.P.fbar));
  adj_force<D, MPSPH_ADJ_LANES><<<nbp, kBlock, 0, R.st>>>(dom, tv, (float)t, R.at<float4>(R.P.fbar),
                                                    R.at<float4>(R.P.xacc), R.at<float>(R.P.sbar));
  adj_field<D><<<R.nb1, kBlock, 0, R.st>>>(dom, tv, R.at<float4>(R.P.xacc), R.at<float>(R.P.sbar),
                                           R.at<float4>(R.P.xbar), R.at<double>(R.P.cpart));
  if (dm.p.field == MPSPH_RBF_EXP && dm.p.n_rbf > 0)
    adj_sum_coeff<<<std::max(dm.p.n_rbf, 1), kCoeffSumThreads, 0, R.st>>>(R.at<double>(R.P.cpart), R.nb1, dm.p.n_rbf,
                                                                        R.at<double>(R.P.cbar));
  HIP_OK(hipGetLastError());
  return MPSPH_OK;
}

template <int D>
int grad_run(mpsph_ctx *ctx, int nsteps, int ckpt, double lam, double *loss_out, double *grad_coeff,
             float *d_grad_pos) {
  const Layout &L = ctx->L;
  const Domain &dm = ctx->dom[0];
  const int n = (int)L.n;
  GradRun R;
  R.ctx = ctx;
  R.st = ctx->stream;
  R.gr = &L.grp[D - 2];
  R.nb1 = (n + kBlock - 1) / kBlock;
  R.nbp = (int)(((int64_t)n * MPSPH_ADJ_LANES + kBlock - 1) / kBlock);
  const int nseg = nsteps > 0 ? (nsteps + ckpt - 1) / ckpt : 0;
  const int seg_len = std::min(ckpt, std::max(nsteps, 1));
  R.P = grad_plan(n, L.ncells, nseg + 1, seg_len, R.nb1, R.nbp);
  if (ctx->gbytes < R.P.bytes) {
    if (ctx->gmem) (void)hipFree(ctx->gmem);
    ctx->gmem = nullptr;
    ctx->gbytes = 0;
    if (hipMalloc((void **)&ctx->gmem, R.P.bytes) != hipSuccess) return MPSPH_E_NOMEM;
    ctx->gbytes = R.P.bytes;
  }
  R.g = ctx->gmem;
  const int64_t t0 = ctx->steps_done;
  EventHook *hk = ctx->hook.on ? &ctx->hook : nullptr;
  HIP_OK(hipMemsetAsync(R.at<double>(R.P.cbar), 0, kMaxRbf * 8, R.st));
  // forward: checkpoints at the start of every segment, the final state in slot nseg
  if (hk) hk->begin("grad_forward");
  for (int sg = 0; sg < nseg; ++sg) {
    int rc = copy_state(R, sg, true);
    if (rc) return rc;
    const int len = std::min(ckpt, nsteps - sg * ckpt);
    if ((rc = enqueue(ctx, len, R.st, nullptr)) != MPSPH_OK) return rc;
  }
  int rc = copy_state(R, nseg, true);
  if (rc) return rc;
  if (hk) hk->end();
  if (hk) hk->begin("grad_backward");
  HIP_OK(hipMemcpyAsync(R.at<double>(R.P.mback), ctx->at<double>(L.metrics), 32 * 8, hipMemcpyDeviceToDevice, R.st));
  if (n > 0) {
    if ((rc = loss_backward<D>(R, lam)) != MPSPH_OK) return rc;
    for (int sg = nseg - 1; sg >= 0; --sg) {
      const int len = std::min(ckpt, nsteps - sg * ckpt);
      if ((rc = copy_state(R, sg, false)) != MPSPH_OK) return rc;
      set_step<<<1, 1, 0, R.st>>>(ctx->at<int64_t>(L.stepctr), t0 + (int64_t)sg * ckpt);
      for (int m = 0; m < len; ++m)
        if ((rc = record_step<D>(R, m)) != MPSPH_OK) return rc;
      for (int m = len - 1; m >= 0; --m)
        if ((rc = step_backward<D>(R, m, t0 + (int64_t)sg * ckpt + m)) != MPSPH_OK) return rc;
    }
    if (d_grad_pos)
      adj_store_pos<D><<<R.nb1, kBlock, 0, R.st>>>(n, reinterpret_cast<const uint32_t *>(R.ck(0) + R.P.ck_id),
                                                   R.at<float4>(R.P.xbar), (float)dm.d.inv_cs, d_grad_pos);
  } else {
    HIP_OK(hipMemsetAsync(R.at<double>(R.P.scal) + 1, 0, 8, R.st));
  }
  // back to the state after the last step
  if ((rc = copy_state(R, nseg, false)) != MPSPH_OK) return rc;
  HIP_OK(hipMemcpyAsync(ctx->at<double>(L.metrics), R.at<double>(R.P.mback), 32 * 8, hipMemcpyDeviceToDevice, R.st));
  set_step<<<1, 1, 0, R.st>>>(ctx->at<int64_t>(L.stepctr), t0 + nsteps);
  if (hk) hk->end();
  HIP_OK(hipGetLastError());
  double loss = 0.0;
  HIP_OK(hipMemcpyAsync(&loss, R.at<double>(R.P.scal) + 1, 8, hipMemcpyDeviceToHost, R.st));
  std::vector<double> gc(kMaxRbf, 0.0);
  HIP_OK(hipMemcpyAsync(gc.data(), R.at<double>(R.P.cbar), kMaxRbf * 8, hipMemcpyDeviceToHost, R.st));
  HIP_OK(hipStreamSynchronize(R.st));
  ctx->steps_done = t0 + nsteps;
  if (loss_out) *loss_out = loss;
  if (grad_coeff && dm.p.field == MPSPH_RBF_EXP)
    for (int m = 0; m < dm.p.n_rbf; ++m) grad_coeff[m] = gc[m];
  return MPSPH_OK;
}

}  // namespace

// Workspace of mpsph_create_static: one array per GPU, for callers that cannot allocate device
// memory.  Host code never uses the array's name as an address: the device address of each
// GPU's copy comes from hipGetSymbolAddress, taken once per device with that device current.
constexpr size_t kScratchBytes = size_t(64) << 20;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) char scratch[kScratchBytes];

struct ScratchTable {
  std::mutex mu;
  char *ptr[kMaxDevices] = {};
  bool busy[kMaxDevices] = {};
};
ScratchTable &scratch_table() {
  static ScratchTable t;
  return t;
}

extern "C" {

const char *mpsph_strerror(int status) {
  if (status < 0 || status > MPSPH_E_SCRATCH) return "unknown status";
  return kErr[status];
}

int mpsph_field_scale(const mpsph_params *params, int64_t n, double *s0_out) {
  if (!valid_params(params) || n <= 0 || !s0_out) return MPSPH_E_INVALID;
  double I = field_integral_unit(params);
  if (!(I > 0) || !std::isfinite(I)) return MPSPH_E_INVALID;
  *s0_out = std::pow(I / (double)n, 1.0 / params->dim);
  return MPSPH_OK;
}

int mpsph_field_bounds(const mpsph_params *params, int64_t n, double *out) {
  if (!valid_params(params) || n <= 0 || !out) return MPSPH_E_INVALID;
  double s0 = params->s0;
  if (!(s0 > 0)) {
    const double I = field_integral_unit(params);
    if (!(I > 0) || !std::isfinite(I)) return MPSPH_E_INVALID;
    s0 = std::pow(I / (double)n, 1.0 / params->dim);
  }
  double smin, smax, lip;
  if (!spacing_bounds(params, s0, &smin, &smax, &lip)) return MPSPH_E_INVALID;
  out[0] = s0;
  out[1] = smin;
  out[2] = smax;
  out[3] = lip;
  return MPSPH_OK;
}

int mpsph_feature_budget(const mpsph_params *params, int64_t n, mpsph_features_t *out) {
  if (!valid_params(params) || n <= 0 || !out) return MPSPH_E_INVALID;
  if (params->geometry == MPSPH_LEVELSET) return MPSPH_E_UNSUPPORTED;
  const int d = params->dim;
  const double Iv = field_integral_unit(params);
  if (!(Iv > 0) || !std::isfinite(Iv)) return MPSPH_E_INVALID;
  const FeatureList f = feature_integrals(params);
  // n = sum_k c_k u^k with u = 1/s0: the volume term (k = dim) plus every feature's term
  double coef[4] = {0, 0, 0, 0};
  coef[d] = Iv;
  for (int i = 0; i < f.n; ++i) {
    if (!(f.I[i] > 0) || !std::isfinite(f.I[i])) return MPSPH_E_INVALID;
    coef[f.power[i]] += f.I[i];
  }
  const double target = (double)n - coef[0];
  if (!(target > 0)) return MPSPH_E_INVALID;
  // Newton from the volume-only root, which lies at or above the root: the polynomial is convex
  // and increasing for u > 0, so the iterates decrease monotonically onto it
  double u = std::pow(target / Iv, 1.0 / d);
  for (int it = 0; it < 200; ++it) {
    double g = -target, dg = 0.0;
    for (int k = 1; k <= d; ++k) {
      g += coef[k] * std::pow(u, k);
      dg += k * coef[k] * std::pow(u, k - 1);
    }
    const double du = g / dg;
    u -= du;
    if (std::fabs(du) <= 1e-15 * u) break;
  }
  if (!(u > 0) || !std::isfinite(u)) return MPSPH_E_INVALID;
  *out = mpsph_features_t{};
  out->s0 = 1.0 / u;
  out->mass_volume = Iv * std::pow(u, d);
  out->n_features = f.n;
  int64_t used = 0;
  for (int i = 0; i < f.n; ++i) {
    out->type[i] = f.type[i];
    out->mass[i] = f.I[i] * std::pow(u, f.power[i]);
    out->count[i] = f.power[i] == 0 ? 1 : (int64_t)std::llround(out->mass[i]);
    used += out->count[i];
  }
  out->n_volume = n - used;
  return out->n_volume >= 0 ? MPSPH_OK : MPSPH_E_INVALID;
}

size_t mpsph_batch_workspace_bytes(int32_t ndom, const mpsph_params *params, const int64_t *n) {
  std::vector<Domain> doms;
  Layout L;
  if (build_domains(ndom, params, n, &doms, &L) != MPSPH_OK) return 0;
  return L.bytes;
}

size_t mpsph_workspace_bytes(const mpsph_params *params, int64_t n) {
  return mpsph_batch_workspace_bytes(1, params, &n);
}

int mpsph_batch_create(int32_t ndom, const mpsph_params *params, const int64_t *n, void *d_workspace,
                       size_t workspace_bytes, void *hip_stream, mpsph_ctx **out) {
  if (!out) return MPSPH_E_INVALID;
  *out = nullptr;
  mpsph_ctx *ctx = new (std::nothrow) mpsph_ctx();
  if (!ctx) return MPSPH_E_NOMEM;
  int rc = build_domains(ndom, params, n, &ctx->dom, &ctx->L);
  if (rc) {
    delete ctx;
    return rc;
  }
  const Layout &L = ctx->L;
  ctx->stream = (hipStream_t)hip_stream;
  ctx->hook.stream = ctx->stream;
  {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) == hipSuccess && hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) ==
                                                hipSuccess && cus > 0)
      ctx->cus = cus;
  }
  if (d_workspace) {
    if (workspace_bytes < L.bytes || ((uintptr_t)d_workspace & 255)) {
      delete ctx;
      return MPSPH_E_NOMEM;
    }
    ctx->ws = (char *)d_workspace;
  } else {
    if (hipMalloc((void **)&ctx->ws, L.bytes) != hipSuccess) {
      delete ctx;
      return MPSPH_E_NOMEM;
    }
    ctx->owns = true;
  }
  ctx->ws_cap = d_workspace ? workspace_bytes : L.bytes;
  if ((rc = setup_device(ctx)) != MPSPH_OK) {
    mpsph_destroy(ctx);
    return rc;
  }
  *out = ctx;
  return MPSPH_OK;
}

int mpsph_create(const mpsph_params *params, int64_t n, void *d_workspace, size_t workspace_bytes, void *hip_stream,
                 mpsph_ctx **out) {
  return mpsph_batch_create(1, params, &n, d_workspace, workspace_bytes, hip_stream, out);
}

int mpsph_create_static(const mpsph_params *params, int64_t n, void *hip_stream, mpsph_ctx **out) {
  if (!out) return MPSPH_E_INVALID;
  *out = nullptr;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return MPSPH_E_DEVICE;
  if (dev < 0 || dev >= kMaxDevices) return MPSPH_E_UNSUPPORTED;
  ScratchTable &t = scratch_table();
  std::lock_guard<std::mutex> lock(t.mu);
  if (!t.ptr[dev]) {
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return MPSPH_E_DEVICE;
    t.ptr[dev] = static_cast<char *>(p);
  }
  if (t.busy[dev]) return MPSPH_E_STATE;
  const size_t need = mpsph_workspace_bytes(params, n);
  if (need == 0) return MPSPH_E_INVALID;
  if (need > kScratchBytes) return MPSPH_E_SCRATCH;
  // the workspace is zeroed by the set-up of the context, so nothing of an earlier context that
  // used the array survives
  const int rc = mpsph_batch_create(1, params, &n, t.ptr[dev], kScratchBytes, hip_stream, out);
  if (rc != MPSPH_OK) return rc;
  (*out)->static_dev = dev;
  t.busy[dev] = true;
  return MPSPH_OK;
}

int mpsph_configure(mpsph_ctx *ctx, int32_t cell_log2, int32_t lanes) {
  if (!ctx || (lanes != 2 && lanes != 4 && lanes != 8) || cell_log2 == 0 || cell_log2 < -1 || cell_log2 > 12)
    return MPSPH_E_INVALID;
  if (ctx->poisoned) return MPSPH_E_STATE;
  for (const Domain &dm : ctx->dom)
    if (cell_log2 > 0 && dm.p.dim * cell_log2 > 24) return MPSPH_E_UNSUPPORTED;
  const std::vector<Domain> base = ctx->dom;
  return reconfigure(ctx, base, 0, cell_log2, lanes);
}

int mpsph_set_pair_variant(mpsph_ctx *ctx, int32_t variant) {
  if (!ctx || variant < MPSPH_PAIRS_DEFAULT || variant > MPSPH_PAIRS_TILE) return MPSPH_E_INVALID;
  if (ctx->poisoned) return MPSPH_E_STATE;
  if (variant != ctx->variant) drop_graph(ctx);   // a captured graph holds the other kernels
  ctx->variant = variant;
  return MPSPH_OK;
}

int mpsph_autotune(mpsph_ctx *ctx, const float *d_pos, const int32_t *d_colour, const int32_t *d_type,
                   int32_t warm_steps, int32_t probe_steps, int32_t *cell_log2_out, int32_t *lanes_out) {
  if (!ctx || probe_steps < 1 || probe_steps > 1000 || warm_steps < 0 || warm_steps > 10000) return MPSPH_E_INVALID;
  if (ctx->poisoned) return MPSPH_E_STATE;
  bool rule = false;
  for (const Domain &dm : ctx->dom) rule |= dm.p.cell_log2 < 0;
  const std::vector<Domain> base = ctx->dom;
  struct Pick {
    int kd, lanes;
    float ms;
  } best{0, MPSPH_LANES, INFINITY};
  // applies a configuration: plan, workspace, device tables, and the caller's state loaded
  auto apply = [&](int kd, int lanes) -> int {
    int rc = reconfigure(ctx, base, kd, -1, lanes);
    if (rc) return rc;
    return mpsph_load(ctx, d_pos, d_colour, d_type);
  };
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return fail(ctx, MPSPH_E_DEVICE);
  int rc = MPSPH_OK;
  const int lanes_c[3] = {2, 4, 8};
  for (int kd = rule ? -1 : 0; kd <= (rule ? 1 : 0) && rc == MPSPH_OK; ++kd) {
    for (int li = 0; li < 3; ++li) {
      int a = apply(kd, lanes_c[li]);
      if (a == MPSPH_E_NOMEM || a == MPSPH_E_UNSUPPORTED) continue;  // does not fit: not a candidate
      if (a != MPSPH_OK) {
        rc = a;
        break;
      }
      // untimed steps first: the first steps after a load (state still in load order, dense
      // initial neighbourhoods) are not representative of a run
      if ((a = enqueue(ctx, std::max(warm_steps, 1), ctx->stream, nullptr)) != MPSPH_OK) {
        rc = a;
        break;
      }
      if (hipEventRecord(e0, ctx->stream) != hipSuccess || enqueue(ctx, probe_steps, ctx->stream, nullptr) ||
          hipEventRecord(e1, ctx->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
        rc = fail(ctx, MPSPH_E_DEVICE);
        break;
      }
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, e0, e1);
      if (ms < best.ms) best = Pick{kd, lanes_c[li], ms};
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc == MPSPH_OK) rc = apply(best.kd, best.lanes);
  if (rc != MPSPH_OK) return rc;
  if (cell_log2_out) *cell_log2_out = ctx->dom[ctx->L.internal[0]].d.k;
  if (lanes_out) *lanes_out = ctx->L.lanes;
  return MPSPH_OK;
}

int mpsph_load(mpsph_ctx *ctx, const float *d_pos, const int32_t *d_colour, const int32_t *d_type) {
  if (!ctx) return MPSPH_E_INVALID;
  if (ctx->poisoned) return MPSPH_E_STATE;
  const Layout &L = ctx->L;
  const int n = (int)L.n;
  if (n > 0 && (!d_pos || !d_colour)) return MPSPH_E_INVALID;
  HIP_OK(hipMemsetAsync(ctx->at<int>(L.bad), 0, 4, ctx->stream));
  HIP_OK(hipMemsetAsync(ctx->at<double>(L.metrics), 0, (size_t)L.ndom * 32 * 8, ctx->stream));
  HIP_OK(hipMemsetAsync(ctx->at<int64_t>(L.stepctr), 0, 8, ctx->stream));
  for (const Group &gr : L.grp) {
    if (gr.i1 <= gr.i0) continue;
    auto kern = gr.D == 2 ? load_kernel<2> : load_kernel<3>;
    kern<<<(gr.i1 - gr.i0 + kBlock - 1) / kBlock, kBlock, 0, ctx->stream>>>(
        ctx->at<DomDev>(L.doms) + gr.d0, gr.nd, gr.i0, gr.i1, d_pos, d_colour, d_type, ctx->at<uint32_t>(L.s_key),
        ctx->at<float4>(L.s_off), ctx->at<uint32_t>(L.s_ct), ctx->at<uint32_t>(L.s_id), ctx->at<int>(L.bad));
    HIP_OK(hipGetLastError());
  }
  int bad = 0;
  HIP_OK(hipMemcpyAsync(&bad, ctx->at<int>(L.bad), 4, hipMemcpyDeviceToHost, ctx->stream));
  HIP_OK(hipStreamSynchronize(ctx->stream));
  ctx->steps_done = 0;
  if (bad) {
    ctx->loaded = false;
    return MPSPH_E_INVALID;
  }
  ctx->loaded = true;
  return MPSPH_OK;
}

int mpsph_step(mpsph_ctx *ctx, int32_t nsteps) {
  if (!ctx || nsteps < 0) return MPSPH_E_INVALID;
  if (ctx->poisoned || !ctx->loaded) return MPSPH_E_STATE;
  int rc = enqueue(ctx, nsteps, ctx->stream, ctx->hook.on ? &ctx->hook : nullptr);
  if (rc == MPSPH_OK) ctx->steps_done += nsteps;
  return rc;
}

int mpsph_step_graph(mpsph_ctx *ctx, int32_t nsteps) {
  if (!ctx || nsteps < 0) return MPSPH_E_INVALID;
  if (ctx->poisoned || !ctx->loaded) return MPSPH_E_STATE;
  if (nsteps == 0) return MPSPH_OK;
  if (!ctx->graph_exec || ctx->graph_steps != nsteps) {
    drop_graph(ctx);
    if (!ctx->cap_stream) HIP_OK(hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking));
    HIP_OK(hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal));
    const int rc = enqueue(ctx, nsteps, ctx->cap_stream, nullptr);
    hipGraph_t graph = nullptr;
    const hipError_t ec = hipStreamEndCapture(ctx->cap_stream, &graph);
    if (rc != MPSPH_OK || ec != hipSuccess || !graph) {
      if (graph) (void)hipGraphDestroy(graph);
      return fail(ctx, MPSPH_E_DEVICE);
    }
    const hipError_t ei = hipGraphInstantiate(&ctx->graph_exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ei != hipSuccess) {
      ctx->graph_exec = nullptr;
      return fail(ctx, MPSPH_E_DEVICE);
    }
    ctx->graph_steps = nsteps;
  }
  EventHook *hk = ctx->hook.on ? &ctx->hook : nullptr;
  if (hk) hk->begin("step_graph");
  HIP_OK(hipGraphLaunch(ctx->graph_exec, ctx->stream));
  if (hk) hk->end();
  ctx->steps_done += nsteps;
  return MPSPH_OK;
}

int mpsph_domain_count(mpsph_ctx *ctx, int32_t *ndom, int64_t *n_total) {
  if (!ctx) return MPSPH_E_INVALID;
  if (ndom) *ndom = ctx->L.ndom;
  if (n_total) *n_total = ctx->L.n;
  return MPSPH_OK;
}

int mpsph_domain_metrics(mpsph_ctx *ctx, int32_t first, int32_t count, mpsph_metrics_t *out) {
  if (!ctx || !out || first < 0 || count < 1 || first + count > ctx->L.ndom) return MPSPH_E_INVALID;
  if (ctx->poisoned) return MPSPH_E_STATE;
  std::vector<double> m((size_t)ctx->L.ndom * 32);
  HIP_OK(hipMemcpyAsync(m.data(), ctx->at<double>(ctx->L.metrics), m.size() * 8, hipMemcpyDeviceToHost,
                        ctx->stream));
  HIP_OK(hipStreamSynchronize(ctx->stream));
  bool nonfinite = false;
  for (int d = 0; d < count; ++d) {
    const int k = ctx->L.internal[first + d];
    fill_metrics(ctx, k, m.data() + (size_t)k * 32, &out[d]);
    nonfinite |= out[d].nonfinite != 0;
  }
  return nonfinite ? MPSPH_E_NONFINITE : MPSPH_OK;
}

int mpsph_metrics(mpsph_ctx *ctx, mpsph_metrics_t *out) { return mpsph_domain_metrics(ctx, 0, 1, out); }

int mpsph_store(mpsph_ctx *ctx, float *d_pos, int32_t *d_type) {
  if (!ctx) return MPSPH_E_INVALID;
  if (ctx->poisoned || !ctx->loaded) return MPSPH_E_STATE;
  const Layout &L = ctx->L;
  for (const Group &gr : L.grp) {
    if (gr.i1 <= gr.i0) continue;
    auto kern = gr.D == 2 ? store_kernel<2> : store_kernel<3>;
    kern<<<(gr.i1 - gr.i0 + kBlock - 1) / kBlock, kBlock, 0, ctx->stream>>>(
        ctx->at<DomDev>(L.doms) + gr.d0, gr.nd, gr.i0, gr.i1, ctx->at<uint32_t>(L.s_key), ctx->at<float4>(L.s_off),
        ctx->at<uint32_t>(L.s_ct), ctx->at<uint32_t>(L.s_id), d_pos, d_type);
    HIP_OK(hipGetLastError());
  }
  HIP_OK(hipStreamSynchronize(ctx->stream));
  return MPSPH_OK;
}

int mpsph_debug_fields(mpsph_ctx *ctx, int32_t which, float *d_out) {
  if (!ctx || !d_out || which < 0 || which > MPSPH_F_X0) return MPSPH_E_INVALID;
  if (ctx->poisoned || !ctx->loaded || ctx->steps_done == 0) return MPSPH_E_STATE;
  const bool needs_debug = which == MPSPH_F_RHO || which == MPSPH_F_A_ABS || which == MPSPH_F_AT ||
                           which == MPSPH_F_V || which == MPSPH_F_DR || which == MPSPH_F_NN;
  if (needs_debug && !ctx->dom[0].p.debug) return MPSPH_E_STATE;
  const Layout &L = ctx->L;
  const float4 *vec = ctx->at<float4>(L.acc);
  const float *sc = ctx->at<float>(L.rho);
  const float *vscale = nullptr;
  if (which == MPSPH_F_NN) sc = ctx->at<float>(L.nn);
  if (which == MPSPH_F_A_ABS) sc = ctx->at<float>(L.aabs);
  if (which == MPSPH_F_AT) vec = ctx->at<float4>(L.at);
  if (which == MPSPH_F_V) vec = ctx->at<float4>(L.v);
  if (which == MPSPH_F_DR) vec = ctx->at<float4>(L.dr);
  if (which == MPSPH_F_VT) {
    // v~ = a dt1 / 2 (Eq. 26 after the velocity reset) with the domain's dt1; fixed particles
    // carry a = 0
    std::vector<double> m((size_t)L.ndom * 32);
    std::vector<float> vs(L.ndom);
    HIP_OK(hipMemcpyAsync(m.data(), ctx->at<double>(L.metrics), m.size() * 8, hipMemcpyDeviceToHost, ctx->stream));
    HIP_OK(hipStreamSynchronize(ctx->stream));
    for (int d = 0; d < L.ndom; ++d) vs[d] = (float)(0.5 * m[(size_t)d * 32 + 16]);
    HIP_OK(hipMemcpyAsync(ctx->at<float>(L.vscale), vs.data(), vs.size() * 4, hipMemcpyHostToDevice, ctx->stream));
    vscale = ctx->at<float>(L.vscale);
  }
  for (const Group &gr : L.grp) {
    if (gr.i1 <= gr.i0) continue;
    auto kern = gr.D == 2 ? dump_kernel<2> : dump_kernel<3>;
    kern<<<(gr.i1 - gr.i0 + kBlock - 1) / kBlock, kBlock, 0, ctx->stream>>>(
        ctx->at<DomDev>(L.doms) + gr.d0, gr.nd, gr.i0, gr.i1, which, ctx->at<uint32_t>(L.w_key),
        ctx->at<float4>(L.w_pos), ctx->at<uint32_t>(L.w_id), sc, vec, vscale ? vscale + gr.d0 : nullptr, d_out);
    HIP_OK(hipGetLastError());
  }
  HIP_OK(hipStreamSynchronize(ctx->stream));
  return MPSPH_OK;
}

int mpsph_debug_cells(mpsph_ctx *ctx, uint32_t *d_key, uint32_t *d_cell_start, int64_t *ncells, int32_t *cell_log2) {
  if (!ctx) return MPSPH_E_INVALID;
  if (ctx->poisoned) return MPSPH_E_STATE;
  if (ncells) *ncells = ctx->L.ncells;
  if (cell_log2) *cell_log2 = ctx->dom[ctx->L.internal[0]].d.k;
  if ((d_key || d_cell_start) && (!ctx->loaded || ctx->steps_done == 0)) return MPSPH_E_STATE;
  const Layout &L = ctx->L;
  const int n = (int)L.n;
  if (d_key && n > 0) {
    // keys of the last step's start in load order: scatter w_key by w_id
    std::vector<uint32_t> k(n), id(n), outk(n);
    HIP_OK(hipMemcpyAsync(k.data(), ctx->at<uint32_t>(L.w_key), 4 * (size_t)n, hipMemcpyDeviceToHost, ctx->stream));
    HIP_OK(hipMemcpyAsync(id.data(), ctx->at<uint32_t>(L.w_id), 4 * (size_t)n, hipMemcpyDeviceToHost, ctx->stream));
    HIP_OK(hipStreamSynchronize(ctx->stream));
    for (int i = 0; i < n; ++i) outk[id[i]] = k[i];
    HIP_OK(hipMemcpyAsync(d_key, outk.data(), 4 * (size_t)n, hipMemcpyHostToDevice, ctx->stream));
  }
  if (d_cell_start)
    HIP_OK(hipMemcpyAsync(d_cell_start, ctx->at<uint32_t>(L.cstart), 4 * ((size_t)L.ncells + 1),
                          hipMemcpyDeviceToDevice, ctx->stream));
  HIP_OK(hipStreamSynchronize(ctx->stream));
  return MPSPH_OK;
}

int mpsph_debug_pairs(mpsph_ctx *ctx, int64_t cap, uint32_t *d_i, uint32_t *d_j, int64_t *count) {
  if (!ctx || cap < 0 || !count || (cap > 0 && (!d_i || !d_j))) return MPSPH_E_INVALID;
  if (ctx->poisoned || !ctx->loaded || ctx->steps_done == 0) return MPSPH_E_STATE;
  const Layout &L = ctx->L;
  unsigned long long *cnt = ctx->at<unsigned long long>(L.paircount);
  HIP_OK(hipMemsetAsync(cnt, 0, 8, ctx->stream));
  for (const Group &gr : L.grp) {
    if (gr.i1 <= gr.i0) continue;
    auto kern = gr.D == 2 ? (gr.periodic ? dump_pairs<2, true> : dump_pairs<2, false>)
                          : (gr.periodic ? dump_pairs<3, true> : dump_pairs<3, false>);
    // two lanes per particle
    kern<<<(int)((2 * (int64_t)(gr.i1 - gr.i0) + kBlock - 1) / kBlock), kBlock, 0, ctx->stream>>>(
        ctx->at<DomDev>(L.doms) + gr.d0, gr.nd, gr.i0, gr.i1, ctx->at<uint32_t>(L.w_key), ctx->at<float4>(L.w_pos),
        ctx->at<uint32_t>(L.w_jaux), ctx->at<uint32_t>(L.w_id), ctx->at<uint32_t>(L.cstart),
        (unsigned long long)cap, d_i, d_j, cnt);
    HIP_OK(hipGetLastError());
  }
  unsigned long long total = 0;
  HIP_OK(hipMemcpyAsync(&total, cnt, 8, hipMemcpyDeviceToHost, ctx->stream));
  HIP_OK(hipStreamSynchronize(ctx->stream));
  *count = (int64_t)total;
  return MPSPH_OK;
}

int mpsph_set_field_coeff(mpsph_ctx *ctx, int32_t domain, const double *coeff) {
  if (!ctx || !coeff || domain < 0 || domain >= ctx->L.ndom) return MPSPH_E_INVALID;
  if (ctx->poisoned) return MPSPH_E_STATE;
  const int k = ctx->L.internal[domain];
  Domain &dm = ctx->dom[k];
  if (dm.p.field != MPSPH_RBF_EXP) return MPSPH_E_INVALID;
  for (int m = 0; m < dm.p.n_rbf; ++m)
    if (!std::isfinite(coeff[m])) return MPSPH_E_INVALID;
  std::vector<double> saved = dm.rbf_coeff;
  dm.rbf_coeff.assign(coeff, coeff + dm.p.n_rbf);
  dm.p.rbf_coeff = dm.rbf_coeff.data();
  // bounds of the field, search radius and h_max for the new coefficients on the same grid
  mpsph_params q = dm.p;
  q.cell_log2 = dm.d.k;
  Derived nd;
  if (derive(&q, dm.n, dm.s0, &nd) != MPSPH_OK) {
    dm.rbf_coeff = saved;
    dm.p.rbf_coeff = dm.rbf_coeff.data();
    return MPSPH_E_UNSUPPORTED;
  }
  dm.d = nd;
  const Layout &L = ctx->L;
  const DomDev dd = domain_device(dm, ctx->at<int>(L.rbf_c), ctx->at<float>(L.rbf_o), ctx->at<float>(L.rbf_k),
                                  ctx->at<float>(L.gphi), ctx->at<float>(L.gs));
  std::vector<float> rk(std::max(dm.p.n_rbf, 1));
  for (int m = 0; m < dm.p.n_rbf; ++m) rk[m] = (float)coeff[m];
  HIP_OK(hipStreamSynchronize(ctx->stream));
  HIP_OK(hipMemcpy(ctx->at<DomDev>(L.doms) + k, &dd, sizeof(DomDev), hipMemcpyHostToDevice));
  if (dm.p.n_rbf > 0)
    HIP_OK(hipMemcpy(ctx->at<float>(L.rbf_k) + dm.rbf0, rk.data(), (size_t)dm.p.n_rbf * 4, hipMemcpyHostToDevice));
  return MPSPH_OK;
}

int mpsph_grad(mpsph_ctx *ctx, int32_t nsteps, int32_t ckpt_every, double lambda, double *loss_out,
               double *grad_coeff_out, float *d_grad_pos) {
  if (!ctx || nsteps < 0 || ckpt_every < 1 || !std::isfinite(lambda)) return MPSPH_E_INVALID;
  if (ctx->poisoned || !ctx->loaded) return MPSPH_E_STATE;
  // the gradient driver allocates its checkpoint memory; a static-scratch context must not
  if (ctx->static_dev >= 0) return MPSPH_E_UNSUPPORTED;
  const Domain &dm = ctx->dom[0];
  if (ctx->L.ndom != 1 || dm.p.geometry != MPSPH_BOX || dm.p.t0 == -2 || dm.p.seeded ||
      (dm.p.field != MPSPH_RBF_EXP && dm.p.field != MPSPH_UNIFORM))
    return MPSPH_E_UNSUPPORTED;
  return dm.p.dim == 2 ? grad_run<2>(ctx, nsteps, ckpt_every, lambda, loss_out, grad_coeff_out, d_grad_pos)
                       : grad_run<3>(ctx, nsteps, ckpt_every, lambda, loss_out, grad_coeff_out, d_grad_pos);
}

int mpsph_profile(mpsph_ctx *ctx, int32_t enable) {
  if (!ctx || enable < 0 || enable > 2) return MPSPH_E_INVALID;
  if (ctx->poisoned) return MPSPH_E_STATE;
  ctx->hook.collect();
  if (enable) ctx->hook.reset();
  ctx->hook.on = enable != 0;
  ctx->hook.pairs_only = enable == 2;
  return MPSPH_OK;
}

int mpsph_profile_read(mpsph_ctx *ctx, int32_t cap, const char **names, int64_t *launches, double *ms, int32_t *count) {
  if (!ctx || cap < 0 || !count) return MPSPH_E_INVALID;
  if (ctx->poisoned) return MPSPH_E_STATE;
  ctx->hook.collect();
  int m = (int)ctx->hook.names.size();
  *count = m;
  for (int i = 0; i < m && i < cap; ++i) {
    if (names) names[i] = ctx->hook.names[i].c_str();
    if (launches) launches[i] = ctx->hook.launches[i];
    if (ms) ms[i] = ctx->hook.ms[i];
  }
  return MPSPH_OK;
}

void mpsph_destroy(mpsph_ctx *ctx) {
  if (!ctx) return;
  (void)hipStreamSynchronize(ctx->stream);
  drop_graph(ctx);
  if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
  if (ctx->owns && ctx->ws) (void)hipFree(ctx->ws);
  if (ctx->gmem) (void)hipFree(ctx->gmem);
  if (ctx->static_dev >= 0) {
    ScratchTable &t = scratch_table();
    std::lock_guard<std::mutex> lock(t.mu);
    t.busy[ctx->static_dev] = false;
  }
  delete ctx;
}

}  // extern "C"
