// Device-side building blocks shared by the relaxation-step kernels (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mpsph {

constexpr int kBlock = 256;       // threads per block of the particle kernels (4 waves)
constexpr int kWave = 64;
constexpr int kNumPartials = 16;  // FP64 partial slots per block
constexpr uint32_t kInfBits = 0x7f800000u;
constexpr int kDtSlots = 16;      // words per domain over which the first time-step minimum is spread
constexpr int kReduceBlocks = 256;  // first-level blocks of the metric reduction

// Slots of the per-block FP64 partials.
enum : int {
  P_E2 = 0,      // sum over normal particles of (rho/rho_t - 1)^2
  P_EMAX = 1,    // max |rho/rho_t - 1|
  P_NNORM = 2,   // number of normal particles
  P_ELR = 3,     // sum of nearest distance / s
  P_ELR2 = 4,    // sum of its square
  P_ELRMIN = 5,
  P_ELRMAX = 6,
  P_NELR = 7,
  P_PAIRS = 8,   // ordered interacting pairs passing the type mask
  P_IFC = 9,     // ordered pairs with different colours (geometric)
  P_CAND = 10,   // candidates tested
  P_NONFIN1 = 11,
  P_KE = 12,     // sum 1/2 |v|^2 (cell units)
  P_NONFIN2 = 13,
  P_NFEAT = 14,  // particles of type >= 1 after the step
  P_IFCP = 15   // particles with at least one interface pair
};

// Geometry of the cell grid and of the meshing region, in cell units.  Positions are held as
// an integer cell coordinate per axis plus a float offset in [0, 1).
// Most sub-cells per cell along x in the cell key (log2).  Measured on the 2M-particle graded
// cube at 2^6 cells: 0 / 1 / 2 / 3 / 4 bits give 4.49 / 4.03 / 3.84 / 3.76 / 3.79 ms per step
// (4 lanes, before the row-table scan; with it and 8 lanes 4 bits gain only 0.3 % over 3); with
// the neighbour loads one slot round ahead 3 / 4 / 5 bits give 2.516 / 2.496 / 2.510 ms.
#ifndef MPSPH_XSUB
#define MPSPH_XSUB 4
#endif

// Row tiles of the 3D cell key (log2 of the tile's rows along y and z).  Measured on the
// 2M-particle graded cube (2^6 cells, 8 lanes): tiles of 16 / 32 / 64 x 16 rows give 3.011 /
// 3.033 / 3.394 ms per step.
#ifndef MPSPH_TILE_LY
#define MPSPH_TILE_LY 4
#endif
#ifndef MPSPH_TILE_LZ
#define MPSPH_TILE_LZ 4
#endif

struct GridDev {
  int k;             // cells per axis = 2^k
  int n;             // particles of the context (bound of every sorted index)
  int gmax;          // 2^k - 1
  uint32_t xmask;    // 2^k - 1
  int geometry;      // MPSPH_BOX | MPSPH_ANNULUS | MPSPH_BALL
  int whi_c[3];      // upper box wall: cell + offset (lower wall is cell 0, offset 0)
  float whi_o[3];
  int gc_c[3];       // annulus / ball centre: cell + offset
  float gc_o[3];
  float r_in, r_out; // radii in cell units
  const float *phi;  // MPSPH_LEVELSET: level set at the background-mesh nodes (cell units)
  int gn[3];         // background-mesh nodes per axis
  double ginv[3];    // 1 / node spacing in cell units
  int seeded;        // features seeded explicitly: reflect instead of project-and-retag
  uint32_t ly, lz;   // 3D row tiles of 2^ly x 2^lz rows in the cell key (see row_index)
  uint32_t xe;       // x sub-cells per cell in the cell key: 2^xe
};

// Target size field in cell units: s_cell(x) = s(x) / cs.
struct FieldDev {
  int kind;
  float s0;          // s0 / cs
  float g;           // fa * cs: slope per cell unit of radius
  float b;           // fb / cs
  int fc_c[3];
  float fc_o[3];
  int n_rbf;
  float e2;          // cs^2 / (2 w^2)
  const int *rbf_c;  // n_rbf x 3 cell coordinates of the centres
  const float *rbf_o;// n_rbf x 3 offsets
  const float *rbf_k;// n_rbf coefficients
  const float *gs;   // MPSPH_GRID: relative spacing at the background-mesh nodes
  int gn[3];
  double ginv[3];
};

// Multilinear interpolation of node values on a background mesh (nodes at multiples of the
// node spacing from the box corner, x index fastest) at a position given as cell + offset.
// The node coordinate is formed in FP64 so that it keeps the offset's precision on any grid;
// weights and sums are FP32.  grad (may be null) receives the derivative of the interpolant
// in cell units.
template <int D>
__device__ __forceinline__ float mesh_interp(const float *nodes, const int *gn, const double *ginv, const int *c,
                                             const float *o, float *grad) {
  int base[3] = {0, 0, 0};
  float f[3] = {0.f, 0.f, 0.f};
#pragma unroll
  for (int a = 0; a < D; ++a) {
    const double u = ((double)c[a] + (double)o[a]) * ginv[a];
    int i = (int)floor(u);
    i = min(max(i, 0), gn[a] - 2);
    base[a] = i;
    f[a] = (float)(u - (double)i);
  }
  float val = 0.f, g[3] = {0.f, 0.f, 0.f};
#pragma unroll
  for (int cn = 0; cn < (1 << D); ++cn) {
    size_t idx = 0, stride = 1;
    float w = 1.f, dw[3] = {1.f, 1.f, 1.f};
#pragma unroll
    for (int a = 0; a < D; ++a) {
      const int bit = (cn >> a) & 1;
      idx += (size_t)(base[a] + bit) * stride;
      stride *= (size_t)gn[a];
      const float wa = bit ? f[a] : 1.f - f[a];
      const float da = bit ? (float)ginv[a] : -(float)ginv[a];
#pragma unroll
      for (int b = 0; b < D; ++b) dw[b] *= (b == a) ? da : wa;
      w *= wa;
    }
    const float v = nodes[idx];
    val = fmaf(w, v, val);
#pragma unroll
    for (int b = 0; b < D; ++b) g[b] = fmaf(dw[b], v, g[b]);
  }
  if (grad) {
#pragma unroll
    for (int a = 0; a < 3; ++a) grad[a] = a < D ? g[a] : 0.f;
  }
  return val;
}

// Constants of one step (cell units; time in the caller's units).
struct StepDev {
  float kappa, tau, inv_tau;
  float p0c;         // p0 cs^(d-2): keeps accelerations in cell units = domain units / cs
  float nu_coeff, c_acc, c_vel, c_visc;
  float search_fac;  // neighbour search radius bound: search_fac * h_i
  float hmax;        // upper bound of h over the region (cell units)
  float alpha;       // kernel normalisation alpha_d
  float dt2_factor;  // dt2 / dt1 implied by Eq. 29 after the velocity reset
  float sigma0;      // surface-tension strength before the ramp (Eq. 25)
  float t0, t1;      // ramp over steps (t0, t1]; t0 < 0: constant
  int auto_t0;       // 1: t0 detected on the device (slot kAutoT0 of the domain's metrics)
  int t0_window;     // steps the topology must stay static
  float t0_tol;      // relative tolerance of "static"
  float theta;       // t1 = t0 + max(1, round(theta t0))
};

// Slots of a domain's metrics block used by the automatic t0: detected t0 + 1 (0: not yet),
// reference interface-pair count, reference interface-particle count, reference step.
constexpr int kAutoT0 = 21;

// One domain of a (possibly batched) context.  Domains occupy contiguous particle ranges
// [off, off + n) in every internal particle array, contiguous ranges of the global cell index space
// [cellbase, cellbase + 2^(d k)), and contiguous ranges of the pair-kernel blocks and of the
// first-level reduction rows.
struct DomDev {
  GridDev g;
  FieldDev f;
  StepDev sp;
  uint32_t cellbase;
  int off, n;        // internal particle range (domains grouped by dimension, 2D first)
  int uoff;          // first row of the domain in the caller's colour / type arrays
  int64_t xoff;      // first float of the domain in the caller's position arrays (rows of dim floats)
  int blk0, nblk;    // pair-kernel blocks
  int row0, nrow;    // first-level reduction rows
  double lo[3];      // domain -> cell units: X = (x - lo) * inv_cs
  double cs, inv_cs;
  double xhi[3];     // upper face of the bounding box in cell units
};

// Surface-tension strength at step t (Eq. 25): sigma0 up to t0, linear ramp to 0 on (t0, t1].
// t0_slot: the domain's detected t0 + 1 (automatic mode; 0 while undetected).
__device__ __forceinline__ float sigma_of(const StepDev &sp, float t, double t0_slot = 0.0) {
  float t0 = sp.t0, t1 = sp.t1;
  if (sp.auto_t0) {
    if (!(t0_slot > 0.0)) return sp.sigma0;
    t0 = (float)(t0_slot - 1.0);
    t1 = t0 + fmaxf(1.f, rintf(sp.theta * t0));
  }
  if (t0 < 0.f || t <= t0) return sp.sigma0;
  if (t <= t1) return sp.sigma0 * (1.f - (t - t0) / (t1 - t0));
  return 0.f;
}

// Domain of particle index i (domains sorted by offset).
__device__ __forceinline__ int domain_of(const DomDev *doms, int ndom, int i) {
  int lo = 0, hi = ndom - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (doms[mid].off <= i) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Domain owning pair-kernel block b.
__device__ __forceinline__ int domain_of_block(const DomDev *doms, int ndom, int b) {
  int lo = 0, hi = ndom - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (doms[mid].blk0 <= b) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

__device__ __forceinline__ int xcd_block(int b, int nb) {
  // Blocks are dispatched round-robin over the 8 XCDs; give each XCD a contiguous range of
  // logical blocks so that neighbouring particles share that XCD's L2.
  int q = nb >> 3, r = nb & 7, x = b & 7;
  int start = x * q + (x < r ? x : r);
  return start + (b >> 3);
}

__device__ __forceinline__ float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float fast_rsq(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ float fast_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }  // x >= 0; sqrt(0) = 0

// Flags word of a particle in the sorted order: colour in bits 0-15, x (sub-)cell in bits 16-27
// (16-23 in 3D), type in bits 30-31.  The pair loops test the fields in place: colours with one
// 16-bit compare of the low halves, the type (the top field) with one compare of the whole word,
// and a 3D x cell converts from its byte in one instruction.
__device__ __forceinline__ uint32_t pack_aux(uint32_t cx, uint32_t type, uint32_t colour) {
  return colour | (cx << 16) | (type << 30);
}
__device__ __forceinline__ int aux_type(uint32_t aux) { return (int)(aux >> 30); }
__device__ __forceinline__ uint32_t aux_colour(uint32_t aux) { return aux & 0xFFFFu; }
__device__ __forceinline__ bool colour_differs(uint32_t a, uint32_t b) { return (uint16_t)a != (uint16_t)b; }
// whether the particle of flags word aux has a type of at least t
__device__ __forceinline__ bool type_at_least(uint32_t aux, int t) { return aux >= ((uint32_t)t << 30); }

// (2 h_ij)^-(d+2) (1 - q/2)^3 with q = r / h_ij, from rh = 1 / (2 h_ij): with
// a = rh (1 - r rh) = (1 - q/2) / (2 h_ij) it is a^3 rh^(d-1) (five multiplies and adds).
template <int D>
__device__ __forceinline__ float kernel_slope_factor(float r, float rh) {
  const float rh2 = rh * rh;
  const float a = fmaf(-r, rh2, rh);
  return D == 3 ? a * a * a * rh2 : a * a * a * rh;
}

template <int D>
__device__ __forceinline__ float powd(float s) {  // s^D
  if constexpr (D == 2) return s * s;
  else return s * s * s;
}
template <int D>
__device__ __forceinline__ float powd_add(float s, float c) {  // s^D + c with one rounding of the sum
  if constexpr (D == 2) return fmaf(s, s, c);
  else return fmaf(s, s * s, c);
}

// Spacing of the size field at a position given as cell + offset (cell units).
template <int D>
__device__ __forceinline__ float field_spacing(const FieldDev &f, const int *c, const float *o) {
  if (f.kind == 0) return f.s0;
  if (f.kind == 4) return f.s0 * mesh_interp<D>(f.gs, f.gn, f.ginv, c, o, nullptr);
  if (f.kind == 1 || f.kind == 2) {
    float r2 = 0.f;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      float d = (float)(c[a] - f.fc_c[a]) + (o[a] - f.fc_o[a]);
      r2 += d * d;
    }
    float t = sqrtf(r2) - f.b;
    if (f.kind == 2) t = fabsf(t);
    return f.s0 * (1.f + f.g * t);
  }
  float e = 0.f;
  for (int k2 = 0; k2 < f.n_rbf; ++k2) {
    float r2 = 0.f;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      float d = (float)(c[a] - f.rbf_c[k2 * 3 + a]) + (o[a] - f.rbf_o[k2 * 3 + a]);
      r2 += d * d;
    }
    e += f.rbf_k[k2] * __expf(-r2 * f.e2);
  }
  return f.s0 * __expf(e);
}

// Bounds-checked loads through a buffer resource (structured buffer: element index, the stride
// in the descriptor; vector memory loads): an index at or past the element count reads zeros,
// so candidate slots past the end of a scan round need no clamp and no address arithmetic.
typedef __amdgpu_buffer_rsrc_t BufRes;
typedef float BufF4 __attribute__((ext_vector_type(4)));
__device__ BufF4 struct_load_f4(BufRes rsrc, int vindex, int voffset, int soffset, int aux) __asm(
    "llvm.amdgcn.struct.ptr.buffer.load.v4f32");
__device__ uint32_t struct_load_u32(BufRes rsrc, int vindex, int voffset, int soffset, int aux) __asm(
    "llvm.amdgcn.struct.ptr.buffer.load.i32");
__device__ __forceinline__ BufRes buf_res(const void *p, int stride, uint32_t count) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)stride, (int)count, 0x00020000);
}
__device__ __forceinline__ float4 buf_f4(BufRes r, uint32_t idx) {
  const BufF4 v = struct_load_f4(r, (int)idx, 0, 0, 0);
  return make_float4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ uint32_t buf_u32(BufRes r, uint32_t idx) { return struct_load_u32(r, (int)idx, 0, 0, 0); }

// Cell key = xf + 2^(k+xe) row(cy, cz), with xf = cx 2^xe + floor(ox 2^xe) the x cell index at
// 2^xe sub-cells per cell: the sort orders each row of cells at that finer resolution in x, so
// the candidate scan can take a row's x-range at sub-cell resolution (a tighter run for the
// same number of rows); positions stay (cell, offset) at the coarse size.  In 3D the rows
// (fixed cy, cz) are numbered tile by tile: tiles of 2^ly x 2^lz rows, cy fastest inside a tile,
// then cz; tiles cy-major, then cz.  The cells of a row stay consecutive (the candidate scan
// reads each row as one range), and a run of consecutive particles in key order covers a
// compact block of rows, so the neighbour data a launch window touches is small (ly = lz = 0
// gives the plain row-major order).
__device__ __forceinline__ uint32_t row_index(int cy, int cz, const GridDev &g) {
  const uint32_t y = (uint32_t)cy, z = (uint32_t)cz;
  return (y & ((1u << g.ly) - 1u)) | ((z & ((1u << g.lz) - 1u)) << g.ly) | ((y >> g.ly) << (g.ly + g.lz)) |
         ((z >> g.lz) << (g.k + g.lz));
}

template <int D>
__device__ __forceinline__ void unpack_key(uint32_t key, const GridDev &g, int *c) {
  const uint32_t kx = g.k + g.xe;
  c[0] = (int)((key & ((1u << kx) - 1u)) >> g.xe);
  const uint32_t r = key >> kx;
  if constexpr (D == 2) {
    c[1] = (int)r;
  } else {
    const uint32_t yl = r & ((1u << g.ly) - 1u), zl = (r >> g.ly) & ((1u << g.lz) - 1u);
    const uint32_t yh = (r >> (g.ly + g.lz)) & ((1u << (g.k - g.ly)) - 1u), zh = r >> (g.k + g.lz);
    c[1] = (int)((yh << g.ly) | yl);
    c[2] = (int)((zh << g.lz) | zl);
  }
}

// o[0] in [0, 1): its sub-cell floor(o 2^xe) is exact (a power-of-two scaling).
template <int D>
__device__ __forceinline__ uint32_t pack_key(const int *c, const float *o, const GridDev &g) {
  const uint32_t xf = ((uint32_t)c[0] << g.xe) | (uint32_t)(o[0] * (float)(1u << g.xe));
  const uint32_t kx = g.k + g.xe;
  if constexpr (D == 2) return xf | ((uint32_t)c[1] << kx);
  return xf | (row_index(c[1], c[2], g) << kx);
}

// Remove the components of v along the active constraint normals of a feature particle
// (force mapping of Eq. 30-31).  Box: faces the particle lies on; annulus / ball: radial.
template <int D>
__device__ __forceinline__ void project_feature(const GridDev &g, int type, const int *c,
                                                const float *o, float *v) {
  if (type == 0) return;
  if (type == 3) {
#pragma unroll
    for (int a = 0; a < D; ++a) v[a] = 0.f;
    return;
  }
  if (g.geometry == 0) return;  // periodic box: no walls
  if (g.geometry == 1) {
#pragma unroll
    for (int a = 0; a < D; ++a) {
      bool lo = c[a] == 0 && o[a] == 0.f;
      bool hi = c[a] == g.whi_c[a] && o[a] == g.whi_o[a];
      if (lo || hi) v[a] = 0.f;
    }
  } else if (g.geometry == 4) {
    // level set: N = grad phi / |grad phi| (Eq. 31)
    float n[3], dot = 0.f;
    mesh_interp<D>(g.phi, g.gn, g.ginv, c, o, n);
    float n2 = 0.f;
#pragma unroll
    for (int a = 0; a < D; ++a) n2 += n[a] * n[a];
    if (!(n2 > 0.f)) return;
    const float inv = fast_rsq(n2);
#pragma unroll
    for (int a = 0; a < D; ++a) {
      n[a] *= inv;
      dot += n[a] * v[a];
    }
#pragma unroll
    for (int a = 0; a < D; ++a) v[a] -= dot * n[a];
  } else {
    float n[3], r2 = 0.f, dot = 0.f;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      n[a] = (float)(c[a] - g.gc_c[a]) + (o[a] - g.gc_o[a]);
      r2 += n[a] * n[a];
    }
    float inv = fast_rsq(r2);
#pragma unroll
    for (int a = 0; a < D; ++a) {
      n[a] *= inv;
      dot += n[a] * v[a];
    }
#pragma unroll
    for (int a = 0; a < D; ++a) v[a] -= dot * n[a];
  }
}

// Deterministic block reduction of NP doubles (sum / min / max chosen per slot by op[]).
// op: 0 sum, 1 min, 2 max.  Writes the block result to out[0..NP).
// S: only lanes whose index is a multiple of S hold values (the first lane of each group of S
// lanes), the others the identity of each slot (0 for sums and maxima of non-negative values,
// +inf for minima).  The butterfly then starts at distance S: the skipped steps would only
// combine a value with identities, which leaves it unchanged, so the result is the same bit
// for bit.
template <int NP, int S = 1>
__device__ __forceinline__ void block_reduce_write(double (&v)[NP], const int (&op)[NP], double *out) {
  static_assert(S >= 1 && S <= kWave && (S & (S - 1)) == 0, "S is a power of two within a wave");
  __shared__ double red[kBlock / kWave][NP];
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
#pragma unroll
  for (int s = 0; s < NP; ++s) {
    double x = v[s];
#pragma unroll
    for (int off = kWave / 2; off >= S; off >>= 1) {
      double y = __shfl_xor(x, off, kWave);
      x = op[s] == 0 ? x + y : (op[s] == 1 ? fmin(x, y) : fmax(x, y));
    }
    if (lane == 0) red[w][s] = x;
  }
  __syncthreads();
  if (threadIdx.x < NP) {
    int s = threadIdx.x;
    double x = red[0][s];
    for (int ww = 1; ww < kBlock / kWave; ++ww) {
      double y = red[ww][s];
      x = op[s] == 0 ? x + y : (op[s] == 1 ? fmin(x, y) : fmax(x, y));
    }
    out[s] = x;
  }
}

// Block reduction through LDS of NP doubles from G writer slots, for the pair passes (whose row
// table is free by then): the thread with slot k in [0, G) stores its values (k < 0: the thread
// holds none); then the first wave combines slot s in four threads, each over a quarter of the
// writer slots in slot order, and joins the four in a fixed butterfly, so that the result does
// not depend on timing.  Slots in minmask combine by min, in maxmask by max, the others by sums.
// emit(s, x) is called once per slot with its block result (in one thread).
// lds: (G + 1) * NP doubles of LDS.  SYNC: start with a barrier, for memory that other waves
// may still read; without it the caller guarantees that nobody reads that memory any more.  The
// caller must not reuse it before the next barrier.
template <int NP, int G, bool SYNC, typename EmitF>
__device__ __forceinline__ void block_reduce_lds(const double (&v)[NP], int k, uint32_t minmask, uint32_t maxmask,
                                                 double *lds, EmitF &&emit) {
  constexpr int kStride = G + 1, kPer = G / 4;
  static_assert(NP * 4 <= kWave && G % 4 == 0, "one wave combines the slots, four threads each");
  if constexpr (SYNC) __syncthreads();
  if (k >= 0) {
#pragma unroll
    for (int s = 0; s < NP; ++s) lds[s * kStride + k] = v[s];
  }
  __syncthreads();
  if (threadIdx.x < kWave) {
    const int s = threadIdx.x >> 2, q = threadIdx.x & 3;
    const bool live = s < NP;
    const bool mn = live && ((minmask >> s) & 1u), mx = live && ((maxmask >> s) & 1u);
    const double *row = lds + (live ? s : 0) * kStride + q * kPer;
    double x = row[0];
    if (mn) {
      for (int t = 1; t < kPer; ++t) x = fmin(x, row[t]);
    } else if (mx) {
      for (int t = 1; t < kPer; ++t) x = fmax(x, row[t]);
    } else {
      for (int t = 1; t < kPer; ++t) x += row[t];
    }
#pragma unroll
    for (int off = 1; off < 4; off <<= 1) {
      const double y = __shfl_xor(x, off, kWave);
      x = mn ? fmin(x, y) : (mx ? fmax(x, y) : x + y);
    }
    if (live && q == 0) emit(s, x);
  }
}

__device__ __forceinline__ void atomic_min_pos(uint32_t *cell, float v) {
  // order-free minimum of non-negative floats through their bit patterns
  atomicMin(cell, __float_as_uint(v));
}

}  // namespace mpsph
