// Reverse-mode (adjoint) kernels of the relaxation step and of the relaxation loss (gfx950).
//
// Notation (cell units, one step, the forward kernels in mpsph.hip compute the same values):
//   s_i field spacing, h_i = tau s_i, P_i = p0c s_i^(2d), H = h_ij = (h_i + h_j)/2, q = r/H,
//   u = 1 - q/2, g(r, H) = 5 alpha H^-(d+2) u^3 (= -W'(r, H)/r),  u_ij = X_i - X_j,
//   F_i = sum_j M_ij B_ij (P_i + P_j) g u_ij, a = Pi F (force mapping, Eq. 18, 23, 30),
//   T1 = min_i c_acc sqrt(kappa h_i / |a_i|), T2 = f T1 (Eq. 29), v~ = T1 a / 2 (Eq. 26),
//   eta_i = nu_coeff kappa tau s_i^(1-d) |v~_i| (Eq. 21-22),
//   K_ij = -Hm(eta_i, eta_j) (s_i^(2d) + s_j^(2d)) g, A~_i = sum_j M_ij K_ij (v~_i - v~_j) (Eq. 20),
//   a~ = Pi A~, Delta = T2 (v~ + T2 a~ / 2) (Eq. 27-28), X' = clamp(X + Delta).
// M_ij = [type_j >= type_i] is the interaction mask, B_ij = 1 + sigma [C_i != C_j] (Eq. 24).
// The pair sums are symmetric in everything but the mask, so the adjoint of a pair sum is a
// gather over the same neighbours: particle k collects, for every neighbour j, the terms of the
// pair (k, j) (mask M_kj) and of the pair (j, k) (mask M_jk) -- no atomics, a fixed order.
//
// Loss (after the last step, all n particles):
//   L = (1/n) sum_i e_i^2 + (lambda / n) sum_{i<j, C_i != C_j} w(r_ij / h_ij),
//   e_i = rho_i / rho_t,i - 1 = alpha tau^-d sum_j w(r_ij / h_i) - 1 (Eq. 17, self included),
//   w(q) = (1 - q/2)^4 (1 + 2q), w'(q) = -5 q (1 - q/2)^3.
// Piecewise-constant parts (pair sets, masks, re-tagging, the particle attaining T1) are held
// fixed; the clamp passes the gradient where the coordinate stays inside the box.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mpsph_device.h"
#include "pair_scan.h"

// Waves per SIMD the viscous adjoint is compiled for; 0 leaves it to the compiler.  With the
// particle's own data scoped to the pair loop and its per-group values in LDS, and the neighbour
// loads issued one slot round ahead (four loads held for the next round), 5 waves (88 VGPRs in
// 3D) need no scratch memory; at 6 waves it spills 10 registers.  Reverse sweep of the
// 2^20-particle RBF cube over 50 steps: 106.7 ms at 5 waves, 109.4 ms at 6 with the spills,
// 107.4 ms with one round of loads at 6 waves.
#ifndef MPSPH_ADJ_WAVES
#define MPSPH_ADJ_WAVES 5
#endif
#if MPSPH_ADJ_WAVES > 0
#define MPSPH_ADJ_OCCUPANCY __attribute__((amdgpu_waves_per_eu(MPSPH_ADJ_WAVES, MPSPH_ADJ_WAVES)))
#else
#define MPSPH_ADJ_OCCUPANCY
#endif

namespace mpsph {

constexpr int kMaxRbf = 64;

// One step of the forward record: the sorted state the step started from and its results.
struct TapeView {
  const uint32_t *wkey;
  const float4 *wpos;    // offsets, h
  const uint32_t *wjaux; // colour | cx << 16 | type << 30
  const uint32_t *cstart;
  const uint32_t *perm;  // state index of each sorted index
  const float4 *acc;     // a (after the force mapping), e = rho_t nu_coeff r_c |a|
  const float4 *at;      // a~ after the force mapping
  const float4 *v;       // v_{n+1/2}
  const uint32_t *dts;   // time-step slots of the step
};

template <int D>
__device__ __forceinline__ float pow2d(float s) {  // s^(2d)
  return powd<D>(s * s);
}

// H^-(d+2) and H^-(d+3) from ih = 1/H.
template <int D>
__device__ __forceinline__ void inv_pows(float ih, float &p2, float &p3) {
  const float ih2 = ih * ih;
  if constexpr (D == 3) {
    p2 = ih2 * ih2 * ih;
    p3 = ih2 * ih2 * ih2;
  } else {
    p2 = ih2 * ih2;
    p3 = ih2 * ih2 * ih;
  }
}

// Field spacing s(X) with its gradient (cell units) for the uniform and RBF fields.
template <int D>
__device__ __forceinline__ float field_grad(const FieldDev &f, const int *c, const float *o, float *grad) {
#pragma unroll
  for (int a = 0; a < 3; ++a) grad[a] = 0.f;
  if (f.kind != 3) return f.s0;
  float e = 0.f, gx[3] = {0.f, 0.f, 0.f};
  for (int m = 0; m < f.n_rbf; ++m) {
    float dv[3], r2 = 0.f;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      dv[a] = (float)(c[a] - f.rbf_c[m * 3 + a]) + (o[a] - f.rbf_o[m * 3 + a]);
      r2 += dv[a] * dv[a];
    }
    const float t = f.rbf_k[m] * __expf(-r2 * f.e2);
    e += t;
#pragma unroll
    for (int a = 0; a < D; ++a) gx[a] -= 2.f * f.e2 * t * dv[a];
  }
  const float s = f.s0 * __expf(e);
#pragma unroll
  for (int a = 0; a < D; ++a) grad[a] = s * gx[a];
  return s;
}

// Minimum of non-negative floats over the block into *dst: one atomic per block.
__device__ __forceinline__ void block_min_atomic(float v, uint32_t *dst) {
  __shared__ float wmin[kBlock / kWave];
  for (int off = kWave / 2; off > 0; off >>= 1) v = fminf(v, __shfl_xor(v, off, kWave));
  if ((threadIdx.x & (kWave - 1)) == 0) wmin[threadIdx.x / kWave] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    float m = wmin[0];
    for (int w = 1; w < kBlock / kWave; ++w) m = fminf(m, wmin[w]);
    if (m < INFINITY) atomic_min_pos(dst, m);
  }
}

// Resets the per-step scalars: minimum time-step bits, index attaining it.
__global__ void adj_init(uint32_t *minbits, uint32_t *argmin) {
  *minbits = kInfBits;
  *argmin = 0xffffffffu;
}

// Drift and velocity adjoint, one thread per particle (sorted order of the step).
//   xbar_next: adjoint of the positions after the step (this step's order)
//   xacc <- identity part of the position adjoint, abv <- adjoint of A~ (before the viscous
//   pair sum), vtb <- direct part of the adjoint of v~, dtc <- the particle's candidate of T1.
template <int D>
__global__ __launch_bounds__(kBlock) void adj_drift(const DomDev *__restrict__ dom, TapeView tp,
                                                    const float4 *__restrict__ xbar_next, float4 *__restrict__ xacc,
                                                    float4 *__restrict__ abv, float4 *__restrict__ vtb,
                                                    float *__restrict__ dtc, uint32_t *__restrict__ minbits,
                                                    double *__restrict__ partials) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  const GridDev &g = dom->g;
  const StepDev &sp = dom->sp;
  const float dt1 = read_dt1(tp.dts);
  const float dt2 = dt1 * sp.dt2_factor;
  double part[1] = {0.0};
  const int ops[1] = {0};
  float c1 = INFINITY;   // the particle's candidate of T1
  if (i < dom->n) {
    int ci[3];
    unpack_key<D>(tp.wkey[i], g, ci);
    const float4 pi = tp.wpos[i];
    const float oi[3] = {pi.x, pi.y, pi.z};
    const int ti = aux_type(tp.wjaux[i]);
    const float4 xb4 = xbar_next[i], v4 = tp.v[i], at4 = tp.at[i];
    const float xb[3] = {xb4.x, xb4.y, xb4.z}, vv[3] = {v4.x, v4.y, v4.z}, av[3] = {at4.x, at4.y, at4.z};
    float xd[3] = {0.f, 0.f, 0.f}, db[3] = {0.f, 0.f, 0.f}, ab[3] = {0.f, 0.f, 0.f};
    double t2 = 0.0;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      float keep = 1.f;
      if (ti != 3) {
        // the drift of the forward pass, to find the coordinates the wall clamp fixed
        const float x = oi[a] + vv[a] * dt2;
        const float fl = floorf(x);
        int c = ci[a] + (int)fl;
        float o = x - fl;
        if (o >= 1.f) {
          o = 0.f;
          c += 1;
        }
        if (c < 0 || c > g.whi_c[a] || (c == g.whi_c[a] && o > g.whi_o[a])) keep = 0.f;
      }
      xd[a] = keep * xb[a];
      if (ti != 3) {
        db[a] = xd[a];
        ab[a] = 0.5f * dt2 * dt2 * db[a];
        t2 += (double)db[a] * (double)(vv[a] + 0.5f * dt2 * av[a]);
      }
    }
    project_feature<D>(g, ti, ci, oi, ab);
    xacc[i] = make_float4(xd[0], xd[1], xd[2], 0.f);
    abv[i] = make_float4(ab[0], ab[1], ab[2], 0.f);
    vtb[i] = make_float4(dt2 * db[0], dt2 * db[1], dt2 * db[2], 0.f);
    part[0] = t2;
    // candidate of the first time step (as in the forward pass, from the stored a)
    const float4 a4 = tp.acc[i];
    const float am2 = a4.x * a4.x + a4.y * a4.y + (D == 3 ? a4.z * a4.z : 0.f);
    if (ti != 3 && am2 > 0.f) c1 = sp.c_acc * fast_sqrt(sp.kappa * pi.w * fast_rsq(am2));   // as the density pass
    dtc[i] = c1;
  }
  block_min_atomic(c1, minbits);
  block_reduce_write<1>(part, ops, partials + (size_t)blockIdx.x * kNumPartials);
}

// Viscous adjoint, L lanes per particle.  Gathers over the neighbours j of k the terms of the
// pairs (k, j) and (j, k) of A~ = sum M K (v~_k - v~_j):
//   v~bar_k += K (M_kj Abar_k - M_jk Abar_j),  Kbar = (M_kj Abar_k - M_jk Abar_j).(v~_k - v~_j)
// and Kbar's share of eta_k, s_k, X_k; then eta -> v~, s; a-bar = T1/2 v~bar; T1-bar partials.
template <int D, int L>
__global__ __launch_bounds__(kBlock) MPSPH_ADJ_OCCUPANCY void adj_visc(const DomDev *__restrict__ dom, TapeView tp,
                                                   const float4 *__restrict__ abv, const float4 *__restrict__ vtb,
                                                   float4 *__restrict__ xacc, float *__restrict__ sbar,
                                                   float4 *__restrict__ abar, const float *__restrict__ dtc,
                                                   const uint32_t *__restrict__ minbits, uint32_t *__restrict__ argmin,
                                                   double *__restrict__ partials) {
  const int lb = xcd_block(blockIdx.x, gridDim.x);
  const GridDev &g = dom->g;
  const StepDev &sp = dom->sp;
  const int local = lb * kBlock + threadIdx.x;
  const int i = local / L, sub = local % L;
  __shared__ uint4 rowtab[row_table_rows<L>() * row_table_stride<L>()];
  // per lane group, the particle's (v~, eta) and (a~-bar, d s^(2d)/ds): read from LDS by the
  // pair terms instead of being held in registers across the pair loop
  __shared__ float4 gdat[kBlock / L][2];
  const float dt1 = read_dt1(tp.dts);
  const float hdt = 0.5f * dt1;
  double part[1] = {0.0};
  const int ops[1] = {0};
  if (i < dom->n && sub == 0) {
    const float4 ai = tp.acc[i];
    const float4 abi = abv[i];
    const float si = tp.wpos[i].w * sp.inv_tau;
    gdat[threadIdx.x / L][0] = make_float4(hdt * ai.x, hdt * ai.y, hdt * ai.z, hdt * ai.w);
    gdat[threadIdx.x / L][1] = make_float4(abi.x, abi.y, abi.z, (2.f * (float)D) * pow2d<D>(si) / si);
  }
  __syncthreads();
  if (i < dom->n) {
    float vb[3] = {0.f, 0.f, 0.f}, xb[3] = {0.f, 0.f, 0.f}, eb = 0.f, sb = 0.f;
    {
    // the pair sum; the particle's own data is scoped to it (the epilogue reads it again), so
    // that the kernel fits its register budget without spilling
    int ci[3];
    unpack_key<D>(tp.wkey[i], g, ci);
    const float4 pi = tp.wpos[i];
    const float oi[3] = {pi.x, pi.y, pi.z};
    const int ti = aux_type(tp.wjaux[i]);
    const float hi = pi.w, si = hi * sp.inv_tau;
    const float s2di = pow2d<D>(si);
    const float4 *gd = gdat[threadIdx.x / L];
    const float ei = gd[0].w;
    const float rs = fminf(sp.search_fac * hi, sp.kappa * 0.5f * (hi + sp.hmax)) * 1.0001f;
    const float kh = 0.5f * sp.kappa, a5 = 5.f * sp.alpha, a75 = 7.5f * sp.alpha;
    if (ei > 0.f) {
      const BufRes rpos = buf_res(tp.wpos, 16, (uint32_t)g.n), raux = buf_res(tp.wjaux, 4, (uint32_t)g.n);
      const BufRes racc = buf_res(tp.acc, 16, (uint32_t)g.n), rabv = buf_res(abv, 16, (uint32_t)g.n);
      struct Nb {
        float4 p, a4, ab;
        uint32_t a;
      };
      // the neighbour's loads (bounds-checked: slots past the arrays read zeros) are issued one
      // slot round ahead of the pair's arithmetic
      const auto fetch = [&](uint32_t jr) {
        return Nb{buf_f4(rpos, jr), buf_f4(racc, jr), buf_f4(rabv, jr), buf_u32(raux, jr)};
      };
      const auto use = [&](const Nb &nb, float dy0, float dz0, bool v) {
        const float4 pj = nb.p, aj4 = nb.a4, abj = nb.ab;
        const uint32_t aj = nb.a;
        const float dx = ((float)ci[0] - cell_x<D>(aj)) + (oi[0] - pj.x);
        const float dy = dy0 - pj.y;
        float dz = 0.f;
        float r2 = dx * dx + dy * dy;
        if constexpr (D == 3) {
          dz = dz0 - pj.z;
          r2 += dz * dz;
        }
        const float hij = kh * (hi + pj.w);
        if (!(v && r2 > 1e-30f && r2 < hij * hij)) return;
        const int tj = aux_type(aj);
        const float ej = hdt * aj4.w;
        if (!(ej > 0.f)) return;  // eta_j = 0: the pair's K and every derivative of it vanish
        const float mkj = tj >= ti ? 1.f : 0.f, mjk = ti >= tj ? 1.f : 0.f;
        const float4 vti = gd[0], abi = gd[1];
        const float ds2i = abi.w;
        const float wv[3] = {mkj * abi.x - mjk * abj.x, mkj * abi.y - mjk * abj.y, mkj * abi.z - mjk * abj.z};
        const float rinv = fast_rsq(r2);
        const float r = r2 * rinv;
        const float ih = sp.kappa * fast_rcp(hij);
        const float q = r * ih, u = fmaf(-0.5f, q, 1.f);
        float p2, p3;
        inv_pows<D>(ih, p2, p3);
        const float gg = a5 * p2 * u * u * u;
        const float dgr = -a75 * p3 * u * u;
        const float dgh = a5 * p3 * u * u * (1.5f * q - (float)(D + 2) * u);
        const float sj = pj.w * sp.inv_tau;
        const float S = s2di + pow2d<D>(sj);
        const float esum = ei + ej;
        const float iesum = fast_rcp(esum);
        const float hm = 2.f * ei * ej * iesum;
        const float K = -hm * S * gg;
        vb[0] = fmaf(K, wv[0], vb[0]);
        vb[1] = fmaf(K, wv[1], vb[1]);
        if constexpr (D == 3) vb[2] = fmaf(K, wv[2], vb[2]);
        const float dvx = vti.x - hdt * aj4.x, dvy = vti.y - hdt * aj4.y, dvz = vti.z - hdt * aj4.z;
        const float kb = wv[0] * dvx + wv[1] * dvy + (D == 3 ? wv[2] * dvz : 0.f);
        eb = fmaf(kb * (-S * gg) * 2.f * ej * ej, iesum * iesum, eb);
        sb = fmaf(kb * (-hm), ds2i * gg + S * dgh * (0.5f * sp.tau), sb);
        const float cx = kb * (-hm * S * dgr) * rinv;
        xb[0] = fmaf(cx, dx, xb[0]);
        xb[1] = fmaf(cx, dy, xb[1]);
        if constexpr (D == 3) xb[2] = fmaf(cx, dz, xb[2]);
      };
      scan_group_table<D, L, row_table_rows<L>()>(i, sub, rowtab + threadIdx.x / L, row_table_stride<L>(), ci, oi, rs,
                                                  g, 0u, tp.cstart, pair_body<true>(fetch, use));
    }
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      vb[a] = group_sum<L>(vb[a]);
      xb[a] = group_sum<L>(xb[a]);
    }
    eb = group_sum<L>(eb);
    sb = group_sum<L>(sb);
    if (sub == 0) {
      // the particle's own data again, through an index the compiler cannot tie to i, so that
      // neither values nor addresses stay live across the pair loop
      const int io = __shfl(i, (int)(threadIdx.x & (kWave - 1)));
      const float si = tp.wpos[io].w * sp.inv_tau;
      const int ti = aux_type(tp.wjaux[io]);
      const float4 ai = tp.acc[io];
      const float vti[3] = {hdt * ai.x, hdt * ai.y, hdt * ai.z};
      const float4 vd = vtb[io];
      float vt[3] = {vd.x + vb[0], vd.y + vb[1], vd.z + vb[2]};
      const float vm2 = vti[0] * vti[0] + vti[1] * vti[1] + (D == 3 ? vti[2] * vti[2] : 0.f);
      if (vm2 > 0.f && eb != 0.f) {
        // eta = nu_coeff kappa tau s^(1-d) |v~|
        const float vm = sqrtf(vm2);
        const float c0 = sp.nu_coeff * sp.kappa * sp.tau * (D == 3 ? 1.f / (si * si) : 1.f / si);
        const float f = eb * c0 / vm;
#pragma unroll
        for (int a = 0; a < D; ++a) vt[a] = fmaf(f, vti[a], vt[a]);
        sb = fmaf(eb * c0 * (float)(1 - D) / si, vm, sb);
      }
      float ab[3] = {0.f, 0.f, 0.f};
      const float av[3] = {ai.x, ai.y, ai.z};
      double t1 = 0.0;
      if (ti != 3) {
#pragma unroll
        for (int a = 0; a < D; ++a) {
          ab[a] = hdt * vt[a];
          t1 += 0.5 * (double)av[a] * (double)vt[a];
        }
      }
      abar[io] = make_float4(ab[0], ab[1], ab[2], 0.f);
      sbar[io] = sb;
      const float4 x0 = xacc[io];
      xacc[io] = make_float4(x0.x + xb[0], x0.y + xb[1], x0.z + xb[2], 0.f);
      if (__float_as_uint(dtc[io]) == *minbits) atomicMin(argmin, (uint32_t)io);
      part[0] = t1;
    }
  }
  block_reduce_write<1, L>(part, ops, partials + (size_t)lb * kNumPartials);   // first lanes of the groups
}

// Sum of the time-step adjoints: out[0] = T1-bar + f T2-bar (fixed order, one block).
__global__ __launch_bounds__(256) void adj_sum_dt(const double *__restrict__ pa, int na, const double *__restrict__ pb,
                                                   int nb, float f, double *__restrict__ out) {
  __shared__ double red[256];
  double x = 0.0, y = 0.0;
  for (int b = threadIdx.x; b < na; b += 256) x += pa[(size_t)b * kNumPartials];
  for (int b = threadIdx.x; b < nb; b += 256) y += pb[(size_t)b * kNumPartials];
  red[threadIdx.x] = y + (double)f * x;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0];
}

// Adjoint of the force after the mapping: F-bar = Pi (a-bar + [k attains T1] dT1/da T1-bar);
// the particle attaining T1 also receives dT1/ds T1-bar.
template <int D>
__global__ __launch_bounds__(kBlock) void adj_fbar(const DomDev *__restrict__ dom, TapeView tp,
                                                   const float4 *__restrict__ abar, const double *__restrict__ t1bar,
                                                   const uint32_t *__restrict__ argmin, float *__restrict__ sbar,
                                                   float4 *__restrict__ fbar) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  const float dt1 = read_dt1(tp.dts);
  if (i >= dom->n) return;
  const GridDev &g = dom->g;
  int ci[3];
  unpack_key<D>(tp.wkey[i], g, ci);
  const float4 pi = tp.wpos[i];
  const float oi[3] = {pi.x, pi.y, pi.z};
  const int ti = aux_type(tp.wjaux[i]);
  const float4 ab4 = abar[i];
  float f[3] = {ab4.x, ab4.y, ab4.z};
  if ((uint32_t)i == *argmin) {
    // T1 = c_acc sqrt(kappa h / |a|): dT1/da = -T1 a / (2 |a|^2), dT1/ds = T1 / (2 s)
    const float tb = (float)*t1bar;
    const float4 a4 = tp.acc[i];
    const float am2 = a4.x * a4.x + a4.y * a4.y + (D == 3 ? a4.z * a4.z : 0.f);
    const float c = -0.5f * dt1 * tb / am2;
    f[0] = fmaf(c, a4.x, f[0]);
    f[1] = fmaf(c, a4.y, f[1]);
    if constexpr (D == 3) f[2] = fmaf(c, a4.z, f[2]);
    sbar[i] += 0.5f * dt1 * tb / (pi.w * dom->sp.inv_tau);
  }
  project_feature<D>(g, ti, ci, oi, f);
  fbar[i] = make_float4(f[0], f[1], f[2], 0.f);
}

// Force adjoint, L lanes per particle: for every neighbour j, with W = M_kj Fbar_k - M_jk Fbar_j
// and w = B (P_k + P_j) g(r, H):
//   X-bar_k += w W + B (P_k + P_j) dg/dr (u.W) u / r
//   s-bar_k += (u.W) B [2d p0c s_k^(2d-1) g + (P_k + P_j) dg/dH tau / 2]
template <int D, int L>
__global__ __launch_bounds__(kBlock) void adj_force(const DomDev *__restrict__ dom, TapeView tp, float tstep,
                                                    const float4 *__restrict__ fbar, float4 *__restrict__ xacc,
                                                    float *__restrict__ sbar) {
  const int lb = xcd_block(blockIdx.x, gridDim.x);
  const GridDev &g = dom->g;
  const StepDev &sp = dom->sp;
  const int local = lb * kBlock + threadIdx.x;
  const int i = local / L, sub = local % L;
  __shared__ uint4 rowtab[row_table_rows<L>() * row_table_stride<L>()];
  if (i >= dom->n) return;
  int ci[3];
  unpack_key<D>(tp.wkey[i], g, ci);
  const float4 pi = tp.wpos[i];
  const float oi[3] = {pi.x, pi.y, pi.z};
  const uint32_t ai = tp.wjaux[i];
  const int ti = aux_type(ai);
  const float hi = pi.w, si = hi * sp.inv_tau;
  const float Pi = sp.p0c * pow2d<D>(si);
  const float dPi = (2.f * (float)D) * Pi / si;
  const float4 fi = fbar[i];
  const float rs = fminf(sp.search_fac * hi, sp.kappa * 0.5f * (hi + sp.hmax)) * 1.0001f;
  const float kh = 0.5f * sp.kappa, a5 = 5.f * sp.alpha, a75 = 7.5f * sp.alpha;
  const float opb = 1.f + sigma_of(sp, tstep);   // surface tension of the step (Eq. 24-25)
  float xb[3] = {0.f, 0.f, 0.f}, sb = 0.f;
  const BufRes rpos = buf_res(tp.wpos, 16, (uint32_t)g.n), raux = buf_res(tp.wjaux, 4, (uint32_t)g.n);
  const BufRes rfb = buf_res(fbar, 16, (uint32_t)g.n);
  struct Nb {
    float4 p, f;
    uint32_t a;
  };
  // the neighbour's loads (bounds-checked: slots past the arrays read zeros) are issued one slot
  // round ahead of the pair's arithmetic
  const auto fetch = [&](uint32_t jr) { return Nb{buf_f4(rpos, jr), buf_f4(rfb, jr), buf_u32(raux, jr)}; };
  const auto use = [&](const Nb &nb, float dy0, float dz0, bool v) {
    const float4 pj = nb.p, fj = nb.f;
    const uint32_t aj = nb.a;
    const float dx = ((float)ci[0] - cell_x<D>(aj)) + (oi[0] - pj.x);
    const float dy = dy0 - pj.y;
    float dz = 0.f;
    float r2 = dx * dx + dy * dy;
    if constexpr (D == 3) {
      dz = dz0 - pj.z;
      r2 += dz * dz;
    }
    const float hij = kh * (hi + pj.w);
    if (!(v && r2 > 1e-30f && r2 < hij * hij)) return;
    const int tj = aux_type(aj);
    const float mkj = tj >= ti ? 1.f : 0.f, mjk = ti >= tj ? 1.f : 0.f;
    const float wf[3] = {mkj * fi.x - mjk * fj.x, mkj * fi.y - mjk * fj.y, mkj * fi.z - mjk * fj.z};
    const float rinv = fast_rsq(r2);
    const float r = r2 * rinv;
    const float ih = sp.kappa * fast_rcp(hij);
    const float q = r * ih, u = fmaf(-0.5f, q, 1.f);
    float p2, p3;
    inv_pows<D>(ih, p2, p3);
    const float gg = a5 * p2 * u * u * u;
    const float dgr = -a75 * p3 * u * u;
    const float dgh = a5 * p3 * u * u * (1.5f * q - (float)(D + 2) * u);
    const float B = colour_differs(aj, ai) ? opb : 1.f;
    const float sj = pj.w * sp.inv_tau;
    const float Psum = Pi + sp.p0c * pow2d<D>(sj);
    const float w = B * Psum * gg;
    const float uw = dx * wf[0] + dy * wf[1] + (D == 3 ? dz * wf[2] : 0.f);
    const float cr = B * Psum * dgr * uw * rinv;
    xb[0] += w * wf[0] + cr * dx;
    xb[1] += w * wf[1] + cr * dy;
    if constexpr (D == 3) xb[2] += w * wf[2] + cr * dz;
    sb = fmaf(uw * B, dPi * gg + Psum * dgh * (0.5f * sp.tau), sb);
  };
  scan_group_table<D, L, row_table_rows<L>()>(i, sub, rowtab + threadIdx.x / L, row_table_stride<L>(), ci, oi, rs, g,
                                              0u, tp.cstart, pair_body<true>(fetch, use));
#pragma unroll
  for (int a = 0; a < 3; ++a) xb[a] = group_sum<L>(xb[a]);
  sb = group_sum<L>(sb);
  if (sub == 0) {
    const float4 x0 = xacc[i];
    xacc[i] = make_float4(x0.x + xb[0], x0.y + xb[1], x0.z + xb[2], 0.f);
    sbar[i] += sb;
  }
}

// Field adjoint and hand-over to the previous step, one thread per particle:
//   X-bar_k += s-bar_k grad s(X_k),  c-bar_m += s-bar_k ds/dc_m = s-bar_k s_k G_m(X_k),
// X-bar written at the particle's index in the previous state order (perm), per-block partial
// sums of c-bar to cpart[block * kMaxRbf + m].
template <int D>
__global__ __launch_bounds__(kBlock) void adj_field(const DomDev *__restrict__ dom, TapeView tp,
                                                    const float4 *__restrict__ xacc, const float *__restrict__ sbar,
                                                    float4 *__restrict__ xbar_prev, double *__restrict__ cpart) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  const GridDev &g = dom->g;
  const FieldDev &f = dom->f;
  const bool act = i < dom->n;
  int ci[3] = {0, 0, 0};
  float oi[3] = {0.f, 0.f, 0.f}, sb = 0.f, gs[3] = {0.f, 0.f, 0.f}, sv = 0.f;
  if (act) {
    unpack_key<D>(tp.wkey[i], g, ci);
    const float4 pi = tp.wpos[i];
    oi[0] = pi.x;
    oi[1] = pi.y;
    oi[2] = pi.z;
    sb = sbar[i];
    sv = field_grad<D>(f, ci, oi, gs);
    const float4 x = xacc[i];
    xbar_prev[tp.perm[i]] = make_float4(fmaf(sb, gs[0], x.x), fmaf(sb, gs[1], x.y), fmaf(sb, gs[2], x.z), 0.f);
  }
  if (f.kind != 3) return;  // block-uniform: no coefficient gradient for other fields
  const int ops[16] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  for (int m0 = 0; m0 < f.n_rbf; m0 += 16) {
    double v[16];
#pragma unroll
    for (int t = 0; t < 16; ++t) {
      const int m = m0 + t;
      float c = 0.f;
      if (act && m < f.n_rbf) {
        float r2 = 0.f;
#pragma unroll
        for (int a = 0; a < D; ++a) {
          const float dv = (float)(ci[a] - f.rbf_c[m * 3 + a]) + (oi[a] - f.rbf_o[m * 3 + a]);
          r2 += dv * dv;
        }
        c = sb * sv * __expf(-r2 * f.e2);
      }
      v[t] = (double)c;
    }
    block_reduce_write<16>(v, ops, cpart + (size_t)blockIdx.x * kMaxRbf + m0);
    __syncthreads();
  }
}

// c-bar[m] += sum over blocks of cpart[b][m]: one block per coefficient, each thread summing
// every 256th block partial in order, then a fixed tree over the threads (deterministic).
constexpr int kCoeffSumThreads = 256;
__global__ __launch_bounds__(kCoeffSumThreads) void adj_sum_coeff(const double *__restrict__ cpart, int nblocks,
                                                                  int n_rbf, double *__restrict__ cbar) {
  __shared__ double red[kCoeffSumThreads];
  const int m = blockIdx.x;
  if (m >= n_rbf) return;  // block-uniform
  double s = 0.0;
  for (int b = threadIdx.x; b < nblocks; b += kCoeffSumThreads) s += cpart[(size_t)b * kMaxRbf + m];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int off = kCoeffSumThreads / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) cbar[m] += red[0];
}

// Loss, first pass (L lanes per particle, sorted order of the final state):
//   e_k = alpha tau^-d sum_{r < kappa h_k} w(r / h_k) - 1 (self included), and the ordered
//   interface sum sum_{C_j != C_k, r < kappa H} w(r / H); block partials of sum e^2 (slot 0)
//   and of the interface sum (slot 1).
template <int D, int L>
__global__ __launch_bounds__(kBlock) void loss_density(const DomDev *__restrict__ dom, const uint32_t *__restrict__ wkey,
                                                       const float4 *__restrict__ wpos, const uint32_t *__restrict__ wjaux,
                                                       const uint32_t *__restrict__ cstart, float *__restrict__ e_out,
                                                       double *__restrict__ partials) {
  const int lb = xcd_block(blockIdx.x, gridDim.x);
  const GridDev &g = dom->g;
  const StepDev &sp = dom->sp;
  const int local = lb * kBlock + threadIdx.x;
  const int i = local / L, sub = local % L;
  __shared__ uint4 rowtab[row_table_rows<L>() * row_table_stride<L>()];
  double part[2] = {0.0, 0.0};
  const int ops[2] = {0, 0};
  if (i < dom->n) {
    int ci[3];
    unpack_key<D>(wkey[i], g, ci);
    const float4 pi = wpos[i];
    const float oi[3] = {pi.x, pi.y, pi.z};
    const uint32_t ai = wjaux[i];
    const float hi = pi.w, ihi = fast_rcp(hi);
    const float rci = sp.kappa * hi, rci2 = rci * rci;
    const float rs = fminf(sp.search_fac * hi, sp.kappa * 0.5f * (hi + sp.hmax)) * 1.0001f;
    const float kh = 0.5f * sp.kappa;
    float ws = 0.f, wi = 0.f;
    const BufRes rpos = buf_res(wpos, 16, (uint32_t)g.n), raux = buf_res(wjaux, 4, (uint32_t)g.n);
    scan_group_table<D, L, row_table_rows<L>()>(i, sub, rowtab + threadIdx.x / L, row_table_stride<L>(), ci, oi, rs, g,
                                                 0u, cstart, [&](uint32_t jr, float dy0, float dz0, bool v) {
      // jr lies past the arrays for invalid slots: bounds-checked loads first
      const float4 pj = buf_f4(rpos, jr);
      const uint32_t aj = buf_u32(raux, jr);
      const float dx = ((float)ci[0] - cell_x<D>(aj)) + (oi[0] - pj.x);
      const float dy = dy0 - pj.y;
      float r2 = dx * dx + dy * dy;
      if constexpr (D == 3) {
        const float dz = dz0 - pj.z;
        r2 += dz * dz;
      }
      if (!v) return;
      const float r = sqrtf(r2);
      if (r2 < rci2) {
        const float q = r * ihi, u = fmaf(-0.5f, q, 1.f);
        ws += u * u * u * u * fmaf(2.f, q, 1.f);
      }
      const float hij = kh * (hi + pj.w);
      if (colour_differs(aj, ai) && r2 < hij * hij) {
        const float q = r * sp.kappa * fast_rcp(hij), u = fmaf(-0.5f, q, 1.f);
        wi += u * u * u * u * fmaf(2.f, q, 1.f);
      }
    });
    ws = group_sum<L>(ws);
    wi = group_sum<L>(wi);
    if (sub == 0) {
      const float A = sp.alpha * (D == 3 ? sp.inv_tau * sp.inv_tau * sp.inv_tau : sp.inv_tau * sp.inv_tau);
      const float e = A * (1.f + ws) - 1.f;
      e_out[i] = e;
      part[0] = (double)e * (double)e;
      part[1] = (double)wi;
    }
  }
  block_reduce_write<2, L>(part, ops, partials + (size_t)lb * kNumPartials);   // first lanes of the groups
}

// Loss, gradient pass: with ebar = 2 e / n and the interface weight cl = lambda / n,
//   X-bar_k = sum_j u_kj (-5) [ebar_k A u_k^3 / h_k^2 + ebar_j A u_j^3 / h_j^2 + cl [C_j != C_k] u^3 / H^2]
//   s-bar_k = tau sum_j [ebar_k A 5 q_k^2 u_k^3 / h_k + cl [C_j != C_k] 2.5 q^2 u^3 / H]
// (u_k = 1 - r / (2 h_k) inside the support of particle k, etc.).  The search radius covers
// every j whose support reaches k: r < kappa h_j <= kappa h_k / (1 - kappa L_h).
template <int D, int L>
__global__ __launch_bounds__(kBlock) void loss_grad(const DomDev *__restrict__ dom, const uint32_t *__restrict__ wkey,
                                                    const float4 *__restrict__ wpos, const uint32_t *__restrict__ wjaux,
                                                    const uint32_t *__restrict__ cstart, const float *__restrict__ e,
                                                    float ebar_scale, float cl, float reach_fac,
                                                    float4 *__restrict__ xacc, float *__restrict__ sbar) {
  const int lb = xcd_block(blockIdx.x, gridDim.x);
  const GridDev &g = dom->g;
  const StepDev &sp = dom->sp;
  const int local = lb * kBlock + threadIdx.x;
  const int i = local / L, sub = local % L;
  __shared__ uint4 rowtab[row_table_rows<L>() * row_table_stride<L>()];
  if (i >= dom->n) return;
  int ci[3];
  unpack_key<D>(wkey[i], g, ci);
  const float4 pi = wpos[i];
  const float oi[3] = {pi.x, pi.y, pi.z};
  const uint32_t ai = wjaux[i];
  const float hi = pi.w, ihi = fast_rcp(hi);
  const float A = sp.alpha * (D == 3 ? sp.inv_tau * sp.inv_tau * sp.inv_tau : sp.inv_tau * sp.inv_tau);
  const float ebi = ebar_scale * e[i];
  const float rs = fminf(reach_fac * hi, sp.kappa * sp.hmax) * 1.0001f;
  const float kh = 0.5f * sp.kappa;
  float xb[3] = {0.f, 0.f, 0.f}, sb = 0.f;
  const BufRes rpos = buf_res(wpos, 16, (uint32_t)g.n), raux = buf_res(wjaux, 4, (uint32_t)g.n);
  scan_group_table<D, L, row_table_rows<L>()>(i, sub, rowtab + threadIdx.x / L, row_table_stride<L>(), ci, oi, rs, g,
                                                 0u, cstart, [&](uint32_t jr, float dy0, float dz0, bool v) {
    const int j = (int)jr;  // past the arrays for invalid slots: bounds-checked loads first
    const float4 pj = buf_f4(rpos, jr);
    const uint32_t aj = buf_u32(raux, jr);
    const float dx = ((float)ci[0] - cell_x<D>(aj)) + (oi[0] - pj.x);
    const float dy = dy0 - pj.y;
    float dz = 0.f;
    float r2 = dx * dx + dy * dy;
    if constexpr (D == 3) {
      dz = dz0 - pj.z;
      r2 += dz * dz;
    }
    if (!(v && r2 > 1e-30f)) return;
    const float r = sqrtf(r2);
    float cx = 0.f;
    const float qi = r * ihi;
    if (qi < sp.kappa) {
      const float u = fmaf(-0.5f, qi, 1.f), u3 = u * u * u;
      cx += ebi * A * u3 * ihi * ihi;
      sb = fmaf(ebi * A * 5.f * qi * qi * u3 * ihi, sp.tau, sb);
    }
    const float ihj = fast_rcp(pj.w), qj = r * ihj;
    if (qj < sp.kappa) {
      const float u = fmaf(-0.5f, qj, 1.f);
      cx += ebar_scale * e[j] * A * u * u * u * ihj * ihj;
    }
    const float hij = kh * (hi + pj.w);
    if (colour_differs(aj, ai) && r2 < hij * hij) {
      const float ih = sp.kappa * fast_rcp(hij), q = r * ih, u = fmaf(-0.5f, q, 1.f), u3 = u * u * u;
      cx += cl * u3 * ih * ih;
      sb = fmaf(cl * 2.5f * q * q * u3 * ih, sp.tau, sb);
    }
    cx *= -5.f;
    xb[0] = fmaf(cx, dx, xb[0]);
    xb[1] = fmaf(cx, dy, xb[1]);
    if constexpr (D == 3) xb[2] = fmaf(cx, dz, xb[2]);
  });
#pragma unroll
  for (int a = 0; a < 3; ++a) xb[a] = group_sum<L>(xb[a]);
  sb = group_sum<L>(sb);
  if (sub == 0) {
    xacc[i] = make_float4(xb[0], xb[1], xb[2], 0.f);
    sbar[i] = sb;
  }
}

// Loss value from the first loss pass's partials: sum e^2 / n + lambda sum_ifc / (2 n).
__global__ __launch_bounds__(256) void loss_value(const double *__restrict__ pb, int nb, double inv_n, double lam,
                                                  double *__restrict__ out) {
  __shared__ double r0[256], r1[256];
  double x = 0.0, y = 0.0;
  for (int b = threadIdx.x; b < nb; b += 256) {
    x += pb[(size_t)b * kNumPartials];
    y += pb[(size_t)b * kNumPartials + 1];
  }
  r0[threadIdx.x] = x;
  r1[threadIdx.x] = y;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      r0[threadIdx.x] += r0[threadIdx.x + w];
      r1[threadIdx.x] += r1[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = r0[0] * inv_n + lam * 0.5 * r1[0] * inv_n;
}

// Sets the device step counter (the recomputation of a segment restarts at its first step).
__global__ void set_step(int64_t *stepctr, int64_t t) { *stepctr = t; }

// Positions adjoint of the first step's start state to the caller's layout (domain units).
template <int D>
__global__ __launch_bounds__(kBlock) void adj_store_pos(int n, const uint32_t *__restrict__ sid,
                                                        const float4 *__restrict__ xbar, float inv_cs,
                                                        float *__restrict__ out) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const float4 x = xbar[i];
  const float xv[3] = {x.x, x.y, x.z};
  const uint32_t id = sid[i];
#pragma unroll
  for (int a = 0; a < D; ++a) out[(size_t)id * D + a] = xv[a] * inv_cs;
}

}  // namespace mpsph
