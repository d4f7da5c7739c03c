/*
 * mpsph_oracle.c -- FP64 CPU oracle for one relaxation step of the multi-phase SPH mesh
 * generator (Ji, Fu, Hu & Adams, arXiv 1906.07925).
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark; never by the product path.  Shares no code with the GPU library.
 *
 * One call of orc_step() is one pass of the main loop of Algorithm 1:
 *   target density / scale at the particles        (Eq. 1, 2, 16)
 *   neighbour candidates                            (its own uniform grid, or brute force)
 *   density summation                               (Eq. 17)
 *   pressure + surface-tension acceleration         (Eq. 18, 19, 23, 24, 25)
 *   force projection of feature particles           (Eq. 30, 31)
 *   time step and mid-point velocity                (Eq. 29, 26)
 *   viscous acceleration with rho = rho_t           (Eq. 20, 21, 22)
 *   second time step, velocity, drift               (Eq. 29, 27, 28)
 *   feature projection and re-tagging               (Eq. 32, §3.5)
 * in plain double precision, one particle at a time, with no blocking or fusion.
 *
 * Readings of points the paper leaves open (kernel, sign of e_ij, viscosity closure, etc.)
 * are stated next to the code that takes them.
 */
#include "mpsph_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define PI 3.14159265358979323846

int orc_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* ------------------------------------------------------------------------------------
 * Smoothing kernel.  The paper uses "a smooth isotropic kernel" (§2.2, §3.3) without
 * printing it; the reading taken here is the Wendland C2 function with support 2h:
 *   W(r,h) = alpha_d h^-d (1 - q/2)^4 (1 + 2q),  q = r/h < 2,
 *   alpha_2 = 7/(4 pi),  alpha_3 = 21/(16 pi)  (so that the integral of W is one).
 * dW/dr follows by differentiating the polynomial in q.
 * ------------------------------------------------------------------------------------ */
static double kernel_alpha(int dim) { return dim == 2 ? 7.0 / (4.0 * PI) : 21.0 / (16.0 * PI); }

double orc_kernel_w(double r, double h, int32_t dim) {
  double q = r / h;
  if (q >= 2.0) return 0.0;
  double u = 1.0 - 0.5 * q;
  return kernel_alpha(dim) * pow(h, -dim) * u * u * u * u * (1.0 + 2.0 * q);
}

double orc_kernel_dw(double r, double h, int32_t dim) {
  double q = r / h;
  if (q >= 2.0) return 0.0;
  double u = 1.0 - 0.5 * q;
  return kernel_alpha(dim) * pow(h, -dim - 1) * (-5.0 * q) * u * u * u;
}

/* Surface-tension strength sigma(t), Eq. 25: the constant sigma0 (= 3 in the paper) up to
 * t0, a linear ramp to zero on (t0, t1], zero afterwards.  t counts steps. */
double orc_sigma(const orc_params *p, int64_t step) {
  if (p->t0 < 0) return p->sigma0;
  double t = (double)step, t0 = (double)p->t0, t1 = (double)p->t1;
  if (t <= t0) return p->sigma0;
  if (t <= t1) return p->sigma0 * (1.0 - (t0 - t) / (t0 - t1));
  return 0.0;
}

/* ------------------------------------------------------------------------------------
 * Target field (Eq. 1-3, 16).  The configurations give a spacing field s(x); the target
 * density is rho_t = s^-d (unit particle mass, Eq. 15) and the scale is
 * h = tau (m / rho_t)^(1/d) (Eq. 16).
 * ------------------------------------------------------------------------------------ */
static double dist_to(const double *x, const double *c, int dim) {
  double s = 0.0;
  for (int a = 0; a < dim; ++a) s += (x[a] - c[a]) * (x[a] - c[a]);
  return sqrt(s);
}

/* Multilinear interpolation on the Cartesian background mesh (§3.1: the level set and the
 * target information live on that mesh and are interpolated at the particle positions).  The
 * cell is the one containing x (the edge cell outside the mesh); the gradient is the exact
 * derivative of the interpolant in that cell. */
double orc_grid_interp(const orc_params *p, const double *nodes, const double *x, double *grad) {
  int d = p->dim;
  int base[3] = {0, 0, 0};
  double f[3] = {0, 0, 0}, hh[3] = {1, 1, 1};
  for (int a = 0; a < d; ++a) {
    int na = p->grid_n[a];
    hh[a] = (p->hi[a] - p->lo[a]) / (double)(na - 1);
    double u = (x[a] - p->lo[a]) / hh[a];
    int i = (int)floor(u);
    if (i < 0) i = 0;
    if (i > na - 2) i = na - 2;
    base[a] = i;
    f[a] = u - i;
  }
  double val = 0.0, g[3] = {0, 0, 0};
  int corners = 1 << d;
  for (int c = 0; c < corners; ++c) {
    int64_t idx = 0, stride = 1;
    double w = 1.0, dw[3] = {1, 1, 1};
    for (int a = 0; a < d; ++a) {
      int bit = (c >> a) & 1;
      idx += (int64_t)(base[a] + bit) * stride;
      stride *= p->grid_n[a];
      double wa = bit ? f[a] : 1.0 - f[a];
      double da = bit ? 1.0 / hh[a] : -1.0 / hh[a];
      for (int b = 0; b < d; ++b) dw[b] *= (b == a) ? da : wa;
      w *= wa;
    }
    val += w * nodes[idx];
    for (int b = 0; b < d; ++b) g[b] += dw[b] * nodes[idx];
  }
  if (grad)
    for (int a = 0; a < 3; ++a) grad[a] = a < d ? g[a] : 0.0;
  return val;
}

double orc_spacing(const orc_params *p, const double *x) {
  switch (p->field) {
    case ORC_GRID: /* target information interpolated from the background mesh (§3.2) */
      return p->s0 * orc_grid_interp(p, p->grid_s, x, NULL);
    case ORC_UNIFORM:
      return p->s0;
    case ORC_RADIAL_LINEAR: /* s = s0 (1 + fa (|x - c| - fb)) */
      return p->s0 * (1.0 + p->fa * (dist_to(x, p->fcentre, p->dim) - p->fb));
    case ORC_SPHERE_DISTANCE: /* s = s0 (1 + fa | |x - c| - fb |) */
      return p->s0 * (1.0 + p->fa * fabs(dist_to(x, p->fcentre, p->dim) - p->fb));
    case ORC_RBF_EXP: { /* s = s0 exp(sum_k c_k exp(-|x - mu_k|^2 / (2 w^2))) */
      double e = 0.0;
      for (int k = 0; k < p->n_rbf; ++k) {
        double r = dist_to(x, p->rbf_centre + (size_t)k * p->dim, p->dim);
        e += p->rbf_coeff[k] * exp(-r * r / (2.0 * p->rbf_width * p->rbf_width));
      }
      return p->s0 * exp(e);
    }
  }
  return NAN;
}

int orc_field(const orc_params *p, int64_t n, const double *x, double *rho_t, double *h) {
  int d = p->dim;
  for (int64_t i = 0; i < n; ++i) {
    double s = orc_spacing(p, x + i * d);
    double rt = pow(s, -d);
    if (rho_t) rho_t[i] = rt;
    if (h) h[i] = p->tau * pow(1.0 / rt, 1.0 / d);
  }
  return ORC_OK;
}

/* Level set phi (Eq. 14): positive inside the meshing region. */
double orc_level_set(const orc_params *p, const double *x) {
  int d = p->dim;
  switch (p->geometry) {
    case ORC_PERIODIC:
      return INFINITY;
    case ORC_BOX: {
      double m = INFINITY;
      for (int a = 0; a < d; ++a) {
        m = fmin(m, x[a] - p->lo[a]);
        m = fmin(m, p->hi[a] - x[a]);
      }
      return m;
    }
    case ORC_ANNULUS: {
      double r = dist_to(x, p->centre, d);
      return fmin(r - p->r_in, p->r_out - r);
    }
    case ORC_BALL:
      return p->r_out - dist_to(x, p->centre, d);
    case ORC_LEVELSET:
      return orc_grid_interp(p, p->grid_phi, x, NULL);
  }
  return NAN;
}

/* Integral of rho_t over the meshing region (Eq. 4 with the indicator of Eq. 5), by a
 * midpoint rule: Cartesian cells for boxes, polar / spherical shells for annuli and balls
 * (whose fields used here depend on the radius only when centred; the angular direction
 * is still sampled so that off-centre fields are integrated correctly). */
double orc_field_integral(const orc_params *p, int32_t nq) {
  int d = p->dim;
  double total = 0.0;
  if (p->geometry == ORC_PERIODIC || p->geometry == ORC_BOX || p->geometry == ORC_LEVELSET) {
    double dx[3], vol = 1.0;
    for (int a = 0; a < d; ++a) {
      dx[a] = (p->hi[a] - p->lo[a]) / nq;
      vol *= dx[a];
    }
    int64_t ncell = 1;
    for (int a = 0; a < d; ++a) ncell *= nq;
#pragma omp parallel for reduction(+ : total) schedule(static)
    for (int64_t c = 0; c < ncell; ++c) {
      double x[3];
      int64_t r = c;
      for (int a = 0; a < d; ++a) {
        x[a] = p->lo[a] + ((double)(r % nq) + 0.5) * dx[a];
        r /= nq;
      }
      /* indicator of Eq. 5: only the positive phase of the level set counts */
      if (p->geometry == ORC_LEVELSET && !(orc_level_set(p, x) > 0.0)) continue;
      total += pow(orc_spacing(p, x), -d);
    }
    return total * vol;
  }
  double rmin = p->geometry == ORC_ANNULUS ? p->r_in : 0.0, rmax = p->r_out;
  double drr = (rmax - rmin) / nq;
  int nth = nq, nph = d == 3 ? nq : 1;
  double dth = (d == 2 ? 2.0 * PI : PI) / nth, dph = 2.0 * PI / nph;
#pragma omp parallel for reduction(+ : total) schedule(static)
  for (int ir = 0; ir < nq; ++ir) {
    double r = rmin + (ir + 0.5) * drr, acc = 0.0;
    for (int it = 0; it < nth; ++it) {
      double th = (it + 0.5) * dth;
      for (int ip = 0; ip < nph; ++ip) {
        double x[3], jac;
        if (d == 2) {
          x[0] = p->centre[0] + r * cos(th);
          x[1] = p->centre[1] + r * sin(th);
          jac = r * drr * dth;
        } else {
          double ph = (ip + 0.5) * dph;
          x[0] = p->centre[0] + r * sin(th) * cos(ph);
          x[1] = p->centre[1] + r * sin(th) * sin(ph);
          x[2] = p->centre[2] + r * cos(th);
          jac = r * r * sin(th) * drr * dth * dph;
        }
        acc += pow(orc_spacing(p, x), -d) * jac;
      }
    }
    total += acc;
  }
  return total;
}

/* ------------------------------------------------------------------------------------
 * Boundary mass (§2.3, Eq. 5-6, unit particle mass Eq. 15).  Reading: the integrand of Eq. 6
 * is the density of the feature's own dimension at the local target size, s^-(dim-1) on a
 * feature surface and s^-1 on a feature curve; a singularity (a box corner) holds one particle.
 * Midpoint rule with nq intervals per parameter; the sphere is parametrised by (z, phi), whose
 * area element R dz dphi is constant.  Features in the order of the public header.
 * ------------------------------------------------------------------------------------ */

/* integral of s^-k over the segment from a along the vector e (midpoint rule) */
static double segment_integral(const orc_params *p, const double *a, const double *e, int k, int nq) {
  double len = 0.0, total = 0.0;
  for (int c = 0; c < p->dim; ++c) len += e[c] * e[c];
  len = sqrt(len);
  for (int i = 0; i < nq; ++i) {
    double t = (i + 0.5) / nq, x[3] = {0, 0, 0};
    for (int c = 0; c < p->dim; ++c) x[c] = a[c] + t * e[c];
    total += pow(orc_spacing(p, x), -k);
  }
  return total * len / nq;
}

/* integral of s^-2 over the face of the 3D box with coordinate `axis` fixed at `at` */
static double face_integral(const orc_params *p, int axis, double at, int nq) {
  int b = axis == 0 ? 1 : 0, c = axis == 2 ? 1 : 2;
  double db = (p->hi[b] - p->lo[b]) / nq, dc = (p->hi[c] - p->lo[c]) / nq, total = 0.0;
#pragma omp parallel for reduction(+ : total) schedule(static)
  for (int i = 0; i < nq; ++i)
    for (int j = 0; j < nq; ++j) {
      double x[3];
      x[axis] = at;
      x[b] = p->lo[b] + (i + 0.5) * db;
      x[c] = p->lo[c] + (j + 0.5) * dc;
      total += pow(orc_spacing(p, x), -2.0);
    }
  return total * db * dc;
}

/* integral of s^-(dim-1) over the sphere (circle) of radius R about the region centre */
static double round_integral(const orc_params *p, double R, int nq) {
  double total = 0.0;
  if (p->dim == 2) {
    for (int i = 0; i < nq; ++i) {
      double th = (i + 0.5) * 2.0 * PI / nq;
      double x[3] = {p->centre[0] + R * cos(th), p->centre[1] + R * sin(th), 0.0};
      total += pow(orc_spacing(p, x), -1.0);
    }
    return total * R * 2.0 * PI / nq;
  }
#pragma omp parallel for reduction(+ : total) schedule(static)
  for (int i = 0; i < nq; ++i)
    for (int j = 0; j < 2 * nq; ++j) {
      double z = -1.0 + (i + 0.5) * 2.0 / nq, ph = (j + 0.5) * PI / nq;
      double rho = sqrt(1.0 - z * z);
      double x[3] = {p->centre[0] + R * rho * cos(ph), p->centre[1] + R * rho * sin(ph), p->centre[2] + R * z};
      total += pow(orc_spacing(p, x), -2.0);
    }
  return total * R * R * (2.0 / nq) * (PI / nq);
}

int32_t orc_features(const orc_params *p, int32_t nq, double *I, int32_t *type, int32_t *power) {
  int d = p->dim, m = 0;
  if (p->geometry == ORC_PERIODIC || p->geometry == ORC_LEVELSET) return 0;
  if (p->geometry == ORC_BALL || p->geometry == ORC_ANNULUS) {
    if (p->geometry == ORC_ANNULUS) {
      I[m] = round_integral(p, p->r_in, nq); type[m] = ORC_SURFACE; power[m++] = d - 1;
    }
    I[m] = round_integral(p, p->r_out, nq); type[m] = ORC_SURFACE; power[m++] = d - 1;
    return m;
  }
  if (d == 2) {
    for (int a = 0; a < 2; ++a)
      for (int side = 0; side < 2; ++side) {
        double x0[3] = {p->lo[0], p->lo[1], 0.0}, e[3] = {0, 0, 0};
        x0[a] = side ? p->hi[a] : p->lo[a];
        e[1 - a] = p->hi[1 - a] - p->lo[1 - a];
        I[m] = segment_integral(p, x0, e, 1, nq); type[m] = ORC_SURFACE; power[m++] = 1;
      }
  } else {
    for (int a = 0; a < 3; ++a)
      for (int side = 0; side < 2; ++side) {
        I[m] = face_integral(p, a, side ? p->hi[a] : p->lo[a], nq); type[m] = ORC_SURFACE; power[m++] = 2;
      }
    for (int a = 0; a < 3; ++a) {
      int b = a == 0 ? 1 : 0, c = a == 2 ? 1 : 2;
      for (int k = 0; k < 4; ++k) {
        double x0[3], e[3] = {0, 0, 0};
        x0[a] = p->lo[a];
        x0[b] = (k & 1) ? p->hi[b] : p->lo[b];
        x0[c] = (k & 2) ? p->hi[c] : p->lo[c];
        e[a] = p->hi[a] - p->lo[a];
        I[m] = segment_integral(p, x0, e, 1, 64 * nq); type[m] = ORC_CURVE; power[m++] = 1;
      }
    }
  }
  for (int c = 0; c < (1 << d); ++c) {
    I[m] = 1.0; type[m] = ORC_FIXED; power[m++] = 0;
  }
  return m;
}

/* ------------------------------------------------------------------------------------
 * Neighbour candidates.  A plain uniform grid over the bounding box of the particles with
 * cells of side kappa * min(h); a particle visits every cell of the cube that covers its
 * largest possible interaction radius, skipping a cell only when the nearest point of the
 * cell is farther than kappa * max(h_i, (h_i + hmax_cell)/2) (with a small margin).  For
 * periodic boxes every pair is visited with the minimum-image convention.
 * ------------------------------------------------------------------------------------ */
typedef struct {
  double lo[3], cs;
  int64_t nc[3], ncell;
  int64_t *start, *idx;
  double *hmax;
} grid_t;

static void grid_free(grid_t *g) {
  free(g->start);
  free(g->idx);
  free(g->hmax);
}

static int64_t cell_coord(double x, double lo, double cs, int64_t nc) {
  int64_t c = (int64_t)floor((x - lo) / cs);
  if (c < 0) c = 0;
  if (c >= nc) c = nc - 1;
  return c;
}

static int grid_build(grid_t *g, int dim, int64_t n, const double *x, const double *h, double cs) {
  double mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int64_t i = 0; i < n; ++i)
    for (int a = 0; a < dim; ++a) {
      mn[a] = fmin(mn[a], x[i * dim + a]);
      mx[a] = fmax(mx[a], x[i * dim + a]);
    }
  g->cs = cs;
  g->ncell = 1;
  for (int a = 0; a < 3; ++a) {
    if (a < dim) {
      g->lo[a] = mn[a];
      g->nc[a] = (int64_t)floor((mx[a] - mn[a]) / cs) + 1;
    } else {
      g->lo[a] = 0.0;
      g->nc[a] = 1;
    }
    g->ncell *= g->nc[a];
  }
  g->start = (int64_t *)calloc((size_t)g->ncell + 1, sizeof(int64_t));
  g->idx = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
  g->hmax = (double *)calloc((size_t)g->ncell, sizeof(double));
  int64_t *cell = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
  if (!g->start || !g->idx || !g->hmax || !cell) {
    free(cell);
    return ORC_E_NOMEM;
  }
  for (int64_t i = 0; i < n; ++i) {
    int64_t c = 0, mul = 1;
    for (int a = 0; a < dim; ++a) {
      c += cell_coord(x[i * dim + a], g->lo[a], cs, g->nc[a]) * mul;
      mul *= g->nc[a];
    }
    cell[i] = c;
    g->start[c + 1]++;
    if (h[i] > g->hmax[c]) g->hmax[c] = h[i];
  }
  for (int64_t c = 0; c < g->ncell; ++c) g->start[c + 1] += g->start[c];
  int64_t *fill = (int64_t *)malloc((size_t)g->ncell * sizeof(int64_t));
  if (!fill) {
    free(cell);
    return ORC_E_NOMEM;
  }
  memcpy(fill, g->start, (size_t)g->ncell * sizeof(int64_t));
  for (int64_t i = 0; i < n; ++i) g->idx[fill[cell[i]]++] = i;
  free(fill);
  free(cell);
  return ORC_OK;
}

typedef struct {
  int64_t *j;
  int64_t n, cap;
} cand_t;

static int cand_push(cand_t *c, int64_t j) {
  if (c->n == c->cap) {
    int64_t nc = c->cap ? 2 * c->cap : 1024;
    int64_t *nj = (int64_t *)realloc(c->j, (size_t)nc * sizeof(int64_t));
    if (!nj) return ORC_E_NOMEM;
    c->j = nj;
    c->cap = nc;
  }
  c->j[c->n++] = j;
  return ORC_OK;
}

/* Collect the candidates j != i of particle i (ascending cell order, ascending index in a
 * cell, or ascending index in brute-force mode). */
static int candidates(const orc_params *p, const grid_t *g, int64_t n, const double *x,
                      const double *h, double hmax_all, int64_t i, cand_t *out) {
  int d = p->dim;
  out->n = 0;
  if (p->search == 1 || p->geometry == ORC_PERIODIC) {
    for (int64_t j = 0; j < n; ++j)
      if (j != i && cand_push(out, j)) return ORC_E_NOMEM;
    return ORC_OK;
  }
  double margin = 1.0 + 1e-4;
  double rmax = p->kappa * fmax(h[i], 0.5 * (h[i] + hmax_all)) * margin;
  int64_t clo[3] = {0, 0, 0}, chi[3] = {0, 0, 0};
  for (int a = 0; a < d; ++a) {
    clo[a] = cell_coord(x[i * d + a] - rmax, g->lo[a], g->cs, g->nc[a]);
    chi[a] = cell_coord(x[i * d + a] + rmax, g->lo[a], g->cs, g->nc[a]);
  }
  for (int64_t cz = clo[2]; cz <= chi[2]; ++cz)
    for (int64_t cy = clo[1]; cy <= chi[1]; ++cy)
      for (int64_t cx = clo[0]; cx <= chi[0]; ++cx) {
        int64_t cc[3] = {cx, cy, cz};
        int64_t c = cx + g->nc[0] * (cy + g->nc[1] * cz);
        if (g->start[c] == g->start[c + 1]) continue;
        double dist2 = 0.0;
        for (int a = 0; a < d; ++a) {
          double b0 = g->lo[a] + cc[a] * g->cs, b1 = b0 + g->cs, xa = x[i * d + a], e = 0.0;
          /* the outermost cells also hold the particles clamped into them */
          if (cc[a] == 0) b0 = -INFINITY;
          if (cc[a] == g->nc[a] - 1) b1 = INFINITY;
          if (xa < b0) e = b0 - xa;
          if (xa > b1) e = xa - b1;
          dist2 += e * e;
        }
        double need = p->kappa * fmax(h[i], 0.5 * (h[i] + g->hmax[c])) * margin;
        if (dist2 >= need * need) continue;
        for (int64_t k = g->start[c]; k < g->start[c + 1]; ++k)
          if (g->idx[k] != i && cand_push(out, g->idx[k])) return ORC_E_NOMEM;
      }
  return ORC_OK;
}

/* Connecting vector r_ij = r_i - r_j (Eq. 17); minimum image in a periodic box. */
static double separation(const orc_params *p, const double *x, int64_t i, int64_t j, double *e) {
  int d = p->dim;
  double r2 = 0.0;
  for (int a = 0; a < d; ++a) {
    double dx = x[i * d + a] - x[j * d + a];
    if (p->geometry == ORC_PERIODIC) {
      double L = p->hi[a] - p->lo[a];
      dx -= L * round(dx / L);
    }
    e[a] = dx;
    r2 += dx * dx;
  }
  return sqrt(r2);
}

/* Which neighbours particle i feels (§3.5): normal particles feel everybody; feature-
 * surface particles ignore normal particles; feature-curve particles feel only curve and
 * singularity particles.  With types ordered normal < surface < curve < fixed this is
 * "type_j >= type_i". */
static int feels(int32_t ti, int32_t tj) { return tj >= ti; }

/* Force projection for feature particles (Eq. 30, 31): remove the components along the
 * active constraint normals.  Box: the normals of the faces the particle lies on.
 * Annulus / ball: the radial direction.  Fixed particles carry no force. */
static void project_vector(const orc_params *p, const double *xi, int32_t type, double *f) {
  int d = p->dim;
  if (type == ORC_NORMAL) return;
  if (type == ORC_FIXED) {
    for (int a = 0; a < d; ++a) f[a] = 0.0;
    return;
  }
  if (p->geometry == ORC_BOX) {
    for (int a = 0; a < d; ++a)
      if (xi[a] == p->lo[a] || xi[a] == p->hi[a]) f[a] = 0.0;
  } else if (p->geometry == ORC_LEVELSET) {
    /* Eq. 31 with the unit normal N = grad phi / |grad phi| */
    double g[3], gn = 0.0, dot = 0.0;
    orc_grid_interp(p, p->grid_phi, xi, g);
    for (int a = 0; a < d; ++a) gn += g[a] * g[a];
    gn = sqrt(gn);
    if (!(gn > 0.0)) return;
    for (int a = 0; a < d; ++a) dot += g[a] / gn * f[a];
    for (int a = 0; a < d; ++a) f[a] -= dot * g[a] / gn;
  } else if (p->geometry == ORC_ANNULUS || p->geometry == ORC_BALL) {
    double nrm[3], r = dist_to(xi, p->centre, d), dot = 0.0;
    for (int a = 0; a < d; ++a) {
      nrm[a] = (xi[a] - p->centre[a]) / r;
      dot += nrm[a] * f[a];
    }
    for (int a = 0; a < d; ++a) f[a] -= dot * nrm[a];
  }
}

/* Type a box particle takes from the number of faces it lies on. */
static int32_t type_from_faces(int nf, int dim) {
  if (nf <= 0) return ORC_NORMAL;
  if (nf == 1) return ORC_SURFACE;
  if (nf == 2) return dim == 3 ? ORC_CURVE : ORC_FIXED;
  return ORC_FIXED;
}

/* Feature mapping after the drift (Eq. 32 and the last step of the loop in Algorithm 1):
 * a normal particle that left the meshing region (phi < 0) is moved to the closest boundary
 * point and becomes a feature particle (never the reverse); feature particles are projected
 * back onto their boundary.  Box faces: clamping is the closest-point projection. */
static void project_position(const orc_params *p, double *xi, int32_t *type) {
  int d = p->dim;
  if (*type == ORC_FIXED) return;
  if (p->geometry == ORC_PERIODIC) {
    for (int a = 0; a < d; ++a) {
      double L = p->hi[a] - p->lo[a];
      xi[a] -= L * floor((xi[a] - p->lo[a]) / L);
    }
    return;
  }
  if (p->seeded) {
    /* Features seeded explicitly with the counts of the boundary mass (Eq. 6): no particle
     * changes type.  Reading: a normal particle that left the region is reflected back into it
     * (mirror image through the boundary), a feature particle stays on its feature (Eq. 32)
     * and is reflected at the walls that bound its feature. */
    if (p->geometry == ORC_BOX) {
      for (int a = 0; a < d; ++a) {
        if (xi[a] < p->lo[a]) xi[a] = fmin(2.0 * p->lo[a] - xi[a], p->hi[a]);
        if (xi[a] > p->hi[a]) xi[a] = fmax(2.0 * p->hi[a] - xi[a], p->lo[a]);
      }
      return;
    }
    if (p->geometry == ORC_LEVELSET) {
      double g[3], gn = 0.0;
      double phi = orc_grid_interp(p, p->grid_phi, xi, g);
      if (*type == ORC_NORMAL && !(phi < 0.0)) return;
      for (int a = 0; a < d; ++a) gn += g[a] * g[a];
      gn = sqrt(gn);
      double f = *type == ORC_NORMAL ? 2.0 : 1.0;
      if (gn > 0.0)
        for (int a = 0; a < d; ++a) xi[a] -= f * phi * g[a] / gn;
      return;
    }
    double r = dist_to(xi, p->centre, d), phi = orc_level_set(p, xi), rt;
    if (!(r > 0.0)) return;
    if (*type == ORC_NORMAL) {
      if (!(phi < 0.0)) return;
      if (r > p->r_out)
        rt = 2.0 * p->r_out - r;
      else
        rt = 2.0 * p->r_in - r;
    } else {
      rt = p->r_out;
      if (p->geometry == ORC_ANNULUS && (r - p->r_in) < (p->r_out - r)) rt = p->r_in;
    }
    for (int a = 0; a < d; ++a) xi[a] = p->centre[a] + rt * (xi[a] - p->centre[a]) / r;
    return;
  }
  if (p->geometry == ORC_BOX) {
    int nf = 0;
    for (int a = 0; a < d; ++a) {
      if (xi[a] < p->lo[a]) xi[a] = p->lo[a];
      if (xi[a] > p->hi[a]) xi[a] = p->hi[a];
      if (xi[a] == p->lo[a] || xi[a] == p->hi[a]) ++nf;
    }
    int32_t t = type_from_faces(nf, d);
    if (*type == ORC_NORMAL && orc_level_set(p, xi) > 0.0) return;
    if (t > *type) *type = t;
    return;
  }
  if (p->geometry == ORC_LEVELSET) {
    /* Eq. 32: r <- r - phi N, for surface particles and for normal particles that left the
     * positive phase (which become surface particles) */
    double g[3], gn = 0.0;
    double phi = orc_grid_interp(p, p->grid_phi, xi, g);
    if (*type == ORC_NORMAL && !(phi < 0.0)) return;
    for (int a = 0; a < d; ++a) gn += g[a] * g[a];
    gn = sqrt(gn);
    if (gn > 0.0)
      for (int a = 0; a < d; ++a) xi[a] -= phi * g[a] / gn;
    if (*type < ORC_SURFACE) *type = ORC_SURFACE;
    return;
  }
  double r = dist_to(xi, p->centre, d);
  double phi = orc_level_set(p, xi);
  if (*type == ORC_NORMAL && !(phi < 0.0)) return;
  double rb = p->r_out;
  if (p->geometry == ORC_ANNULUS && (r - p->r_in) < (p->r_out - r)) rb = p->r_in;
  for (int a = 0; a < d; ++a) xi[a] = p->centre[a] + rb * (xi[a] - p->centre[a]) / r;
  *type = ORC_SURFACE;
}

static int isfinite_vec(const double *v, int d) {
  for (int a = 0; a < d; ++a)
    if (!isfinite(v[a])) return 0;
  return 1;
}

int orc_step(const orc_params *p, int64_t n, double *x, const int32_t *colour, int32_t *type,
             int64_t step, orc_out *out) {
  if (!p || !x || !colour || !type || !out || n < 0) return ORC_E_INVALID;
  if (p->dim != 2 && p->dim != 3) return ORC_E_INVALID;
  int d = p->dim;
  const double kap = p->kappa;
  size_t nv = (size_t)(n > 0 ? n : 1);
  double *rho_t = malloc(nv * sizeof(double)), *h = malloc(nv * sizeof(double));
  double *P = malloc(nv * sizeof(double)), *rho = malloc(nv * sizeof(double));
  double *a = calloc(nv * d, sizeof(double)), *aabs = calloc(nv, sizeof(double));
  double *vt = calloc(nv * d, sizeof(double)), *at = calloc(nv * d, sizeof(double));
  double *atabs = calloc(nv, sizeof(double)), *v = calloc(nv * d, sizeof(double));
  double *eta = calloc(nv, sizeof(double)), *nn = malloc(nv * sizeof(double));
  int64_t *npair = calloc(nv, sizeof(int64_t)), *nifc = calloc(nv, sizeof(int64_t));
  int64_t *nband = calloc(nv, sizeof(int64_t));
  double *kabs = calloc(nv, sizeof(double));
  int32_t *type0 = malloc(nv * sizeof(int32_t));
  grid_t g;
  memset(&g, 0, sizeof(g));
  int rc = ORC_OK;
  if (!rho_t || !h || !P || !rho || !a || !aabs || !vt || !at || !atabs || !v || !eta || !nn ||
      !npair || !nifc || !nband || !kabs || !type0) {
    rc = ORC_E_NOMEM;
    goto done;
  }

  /* Target density and scale at the start-of-step positions (Eq. 1, 16); the pressure
   * coefficient p0 / rho_t^2 of the gamma = 2 EOS (Eq. 18, 19). */
  orc_field(p, n, x, rho_t, h);
  double hmin = INFINITY, hmax = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    P[i] = p->p0 / (rho_t[i] * rho_t[i]);
    hmin = fmin(hmin, h[i]);
    hmax = fmax(hmax, h[i]);
  }
  const double sigma = orc_sigma(p, step);
  if (n > 0 && p->search == 0 && p->geometry != ORC_PERIODIC) {
    rc = grid_build(&g, d, n, x, h, kap * hmin);
    if (rc) goto done;
  }

  /* Pass 1: density (Eq. 17, self term included), pressure + surface-tension acceleration
   * (Eq. 18, 23).  Reading of the signs: e_ij = r_ij / |r_ij| with r_ij = r_i - r_j, and the
   * momentum balance dv/dt = -F_p + F_s (Eq. 10) gives
   *   a_i = -sum_j (1 + beta_ij) (P_i + P_j) dW(r_ij, h_ij)/dr e_ij,
   * which, with dW/dr <= 0, is repulsive for both terms as the text requires.
   * beta_ij = sigma(t) for different colours, 0 otherwise (Eq. 24). */
#pragma omp parallel
  {
    cand_t cand = {0, 0, 0};
#pragma omp for schedule(dynamic, 256)
    for (int64_t i = 0; i < n; ++i) {
      if (candidates(p, &g, n, x, h, hmax, i, &cand)) {
        rc = ORC_E_NOMEM;
        continue;
      }
      double rs = orc_kernel_w(0.0, h[i], d), ai[3] = {0, 0, 0}, A = 0.0, K = 0.0, nearest = INFINITY;
      int64_t np = 0, ni = 0, nb = 0;
      for (int64_t k = 0; k < cand.n; ++k) {
        int64_t j = cand.j[k];
        double e[3];
        double r = separation(p, x, i, j, e);
        if (r < kap * h[i]) rs += orc_kernel_w(r, h[i], d);
        double hij = 0.5 * (h[i] + h[j]);
        if (fabs(r - kap * hij) < 1e-5 * kap * hij) ++nb;
        if (!(r < kap * hij)) continue;
        if (r < nearest) nearest = r;
        if (colour[i] != colour[j]) ++ni;
        if (!feels(type[i], type[j])) continue;
        ++np;
        if (r == 0.0) continue; /* coincident pair: e_ij undefined, no force */
        double beta = colour[i] != colour[j] ? sigma : 0.0;
        double s = -(1.0 + beta) * (P[i] + P[j]) * orc_kernel_dw(r, hij, d) / r;
        double mag = 0.0;
        for (int c = 0; c < d; ++c) {
          ai[c] += s * e[c];
          mag += (s * e[c]) * (s * e[c]);
        }
        A += sqrt(mag);
        K += sqrt(mag) * (1.0 + 3.0 * (r / hij) / (2.0 - r / hij));
      }
      rho[i] = rs;
      for (int c = 0; c < d; ++c) a[i * d + c] = ai[c];
      aabs[i] = A;
      kabs[i] = K;
      if (out->a_kabs) out->a_kabs[i] = K;
      nn[i] = nearest;
      npair[i] = np;
      nifc[i] = ni;
      nband[i] = nb;
    }
    free(cand.j);
  }
  if (rc) goto done;

  /* Map the forces of feature particles (Eq. 30, 31). */
  for (int64_t i = 0; i < n; ++i) project_vector(p, x + i * d, type[i], a + i * d);

  /* First time step: with the velocity reset (v_n = 0, Algorithm 1) only the body-force
   * criterion of Eq. 29 is active.  Global minimum over movable particles with a != 0;
   * zero when no particle is accelerated. */
  double dt1 = INFINITY;
  for (int64_t i = 0; i < n; ++i) {
    if (type[i] == ORC_FIXED) continue;
    double am = 0.0;
    for (int c = 0; c < d; ++c) am += a[i * d + c] * a[i * d + c];
    am = sqrt(am);
    if (am > 0.0) dt1 = fmin(dt1, p->c_acc * sqrt(kap * h[i] / am));
  }
  if (!(dt1 < INFINITY)) dt1 = 0.0;

  /* Mid-point velocity (Eq. 26 with v_n = 0) and the viscosity closure of Eq. 21, read as
   * nu_i = nu_coeff * r_c,i * |v~_i| with r_c = kappa h_i, and eta_i = rho_t,i nu_i since
   * rho = rho_t in the viscous term (Eq. 22). */
  for (int64_t i = 0; i < n; ++i) {
    double sp = 0.0;
    for (int c = 0; c < d; ++c) {
      vt[i * d + c] = type[i] == ORC_FIXED ? 0.0 : 0.5 * a[i * d + c] * dt1;
      sp += vt[i * d + c] * vt[i * d + c];
    }
    eta[i] = rho_t[i] * p->nu_coeff * kap * h[i] * sqrt(sp);
  }

  /* Pass 2: viscous acceleration (Eq. 20 with rho = rho_t, Eq. 22); a pair whose harmonic
   * mean viscosity has a zero denominator contributes nothing. */
#pragma omp parallel
  {
    cand_t cand = {0, 0, 0};
#pragma omp for schedule(dynamic, 256)
    for (int64_t i = 0; i < n; ++i) {
      if (candidates(p, &g, n, x, h, hmax, i, &cand)) {
        rc = ORC_E_NOMEM;
        continue;
      }
      double ai[3] = {0, 0, 0}, A = 0.0, K = 0.0, Pr[3] = {0.0, 0.0, 0.0};
      for (int64_t k = 0; k < cand.n; ++k) {
        int64_t j = cand.j[k];
        double e[3];
        double r = separation(p, x, i, j, e);
        double hij = 0.5 * (h[i] + h[j]);
        if (!(r < kap * hij) || !feels(type[i], type[j]) || r == 0.0) continue;
        double inv2 = 1.0 / (rho_t[i] * rho_t[i]) + 1.0 / (rho_t[j] * rho_t[j]);
        double gij = inv2 * orc_kernel_dw(r, hij, d) / r;
        if (out->at_prop || out->at_prop_k || out->at_prop_kn) {
          /* conditioning diagnostic only; it does not enter the result.  Weights of particle
           * k: A_k, K_k, K_k / nn_k. */
          double dv = 0.0;
          for (int c = 0; c < d; ++c) dv += (vt[i * d + c] - vt[j * d + c]) * (vt[i * d + c] - vt[j * d + c]);
          double H = eta[i] + eta[j] > 0.0 ? 2.0 * eta[i] * eta[j] / (eta[i] + eta[j]) : 0.0;
          for (int w = 0; w < 3; ++w) {
            double wi = w == 0 ? aabs[i] : (w == 1 ? kabs[i] : (nn[i] > 0.0 && nn[i] < INFINITY ? kabs[i] / nn[i] : 0.0));
            double wj = w == 0 ? aabs[j] : (w == 1 ? kabs[j] : (nn[j] > 0.0 && nn[j] < INFINITY ? kabs[j] / nn[j] : 0.0));
            double dvi = type[i] == ORC_FIXED ? 0.0 : 0.5 * dt1 * wi;
            double dvj = type[j] == ORC_FIXED ? 0.0 : 0.5 * dt1 * wj;
            double dH = 2.0 * (rho_t[i] * p->nu_coeff * kap * h[i] * dvi + rho_t[j] * p->nu_coeff * kap * h[j] * dvj);
            Pr[w] += fabs(gij) * (dH * sqrt(dv) + H * (dvi + dvj));
          }
        }
        if (eta[i] + eta[j] == 0.0) continue;
        double etaij = 2.0 * eta[i] * eta[j] / (eta[i] + eta[j]);
        double s = etaij * inv2 * orc_kernel_dw(r, hij, d) / r;
        double mag = 0.0;
        for (int c = 0; c < d; ++c) {
          double t = s * (vt[i * d + c] - vt[j * d + c]);
          ai[c] += t;
          mag += t * t;
        }
        A += sqrt(mag);
        K += sqrt(mag) * (1.0 + 3.0 * (r / hij) / (2.0 - r / hij));
      }
      for (int c = 0; c < d; ++c) at[i * d + c] = ai[c];
      atabs[i] = A;
      if (out->at_kabs) out->at_kabs[i] = K;
      if (out->at_prop) out->at_prop[i] = Pr[0];
      if (out->at_prop_k) out->at_prop_k[i] = Pr[1];
      if (out->at_prop_kn) out->at_prop_kn[i] = Pr[2];
    }
    free(cand.j);
  }
  if (rc) goto done;
  for (int64_t i = 0; i < n; ++i) project_vector(p, x + i * d, type[i], at + i * d);

  /* Second time step: all three criteria of Eq. 29 with |a| = |a_n|, |v| = |v~| and nu. */
  double dt2 = INFINITY;
  for (int64_t i = 0; i < n; ++i) {
    if (type[i] == ORC_FIXED) continue;
    double am = 0.0, vm = 0.0, rci = kap * h[i];
    for (int c = 0; c < d; ++c) {
      am += a[i * d + c] * a[i * d + c];
      vm += vt[i * d + c] * vt[i * d + c];
    }
    am = sqrt(am);
    vm = sqrt(vm);
    double nu = p->nu_coeff * rci * vm;
    if (am > 0.0) dt2 = fmin(dt2, p->c_acc * sqrt(rci / am));
    if (vm > 0.0) dt2 = fmin(dt2, p->c_vel * rci / vm);
    if (nu > 0.0) dt2 = fmin(dt2, p->c_visc * rci * rci / nu);
  }
  if (!(dt2 < INFINITY)) dt2 = 0.0;

  /* Velocity (Eq. 27), drift (Eq. 28), feature mapping (Eq. 32).  The metrics below use
   * the types at the start of the step, so keep them. */
  for (int64_t i = 0; i < n; ++i) type0[i] = type[i];
  int64_t nonfinite = 0;
  double ke = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    double dri[3] = {0, 0, 0};
    int fixed = type[i] == ORC_FIXED;
    for (int c = 0; c < d; ++c) {
      v[i * d + c] = fixed ? 0.0 : vt[i * d + c] + 0.5 * at[i * d + c] * dt2;
      dri[c] = v[i * d + c] * dt2;
      ke += 0.5 * v[i * d + c] * v[i * d + c];
    }
    if (!isfinite_vec(a + i * d, d) || !isfinite_vec(at + i * d, d)) ++nonfinite;
    if (out->dr)
      for (int c = 0; c < d; ++c) out->dr[i * d + c] = dri[c];
    if (!fixed) {
      for (int c = 0; c < d; ++c) x[i * d + c] += dri[c];
      project_position(p, x + i * d, &type[i]);
    }
    if (!isfinite_vec(x + i * d, d)) ++nonfinite;
  }

  /* Metrics of the step: density residual rho/rho_t - 1 over normal particles (start-of-
   * step positions and types), kinetic energy of v_{n+1/2}, pair counts, and the nearest-
   * neighbour distance over the local target spacing rho_t^(-1/d) ("edge-length ratio"). */
  {
    double s2 = 0.0, linf = 0.0, em = 0.0, em2 = 0.0, emin = INFINITY, emax = 0.0;
    int64_t nnorm = 0, nelr = 0, pairs = 0, ifc = 0, band = 0, ifcp = 0;
    for (int64_t i = 0; i < n; ++i) {
      pairs += npair[i];
      ifc += nifc[i];
      ifcp += nifc[i] > 0;
      band += nband[i];
      if (type0[i] == ORC_NORMAL) {
        double e = rho[i] / rho_t[i] - 1.0;
        s2 += e * e;
        linf = fmax(linf, fabs(e));
        ++nnorm;
        if (nn[i] < INFINITY) {
          double r = nn[i] * pow(rho_t[i], 1.0 / d);
          em += r;
          em2 += r * r;
          emin = fmin(emin, r);
          emax = fmax(emax, r);
          ++nelr;
        }
      }
      if (out->rho) out->rho[i] = rho[i];
      if (out->rho_t) out->rho_t[i] = rho_t[i];
      if (out->h) out->h[i] = h[i];
      if (out->a_abs) out->a_abs[i] = aabs[i];
      if (out->at_abs) out->at_abs[i] = atabs[i];
      if (out->nn) out->nn[i] = nn[i];
      for (int c = 0; c < d; ++c) {
        if (out->a) out->a[i * d + c] = a[i * d + c];
        if (out->vt) out->vt[i * d + c] = vt[i * d + c];
        if (out->at) out->at[i * d + c] = at[i * d + c];
        if (out->v) out->v[i * d + c] = v[i * d + c];
      }
    }
    out->residual_l2 = nnorm ? sqrt(s2 / nnorm) : 0.0;
    out->residual_linf = linf;
    out->n_normal = nnorm;
    out->n_elr = nelr;
    out->elr_mean = nelr ? em / nelr : 0.0;
    out->elr_std = nelr ? sqrt(fmax(em2 / nelr - (em / nelr) * (em / nelr), 0.0)) : 0.0;
    out->elr_min = nelr ? emin : 0.0;
    out->elr_max = emax;
    out->pairs = pairs;
    out->interface_pairs = ifc / 2;
    out->interface_particles = ifcp;
    out->band_pairs = band;
    out->nonfinite = nonfinite;
    out->kinetic = ke;
    out->dt1 = dt1;
    out->dt2 = dt2;
    out->sigma = sigma;
  }
done:
  grid_free(&g);
  free(rho_t);
  free(h);
  free(P);
  free(rho);
  free(a);
  free(aabs);
  free(vt);
  free(at);
  free(atabs);
  free(v);
  free(eta);
  free(nn);
  free(npair);
  free(nifc);
  free(nband);
  free(kabs);
  free(type0);
  return rc;
}

/* Ordered pairs (i, j != i) with r_ij < kappa h_ij at the given positions (no type mask);
 * used to compare neighbour sets.  Writes at most cap pairs, returns the total in count. */
int orc_pairs(const orc_params *p, int64_t n, const double *x, int64_t cap, int64_t *pi,
              int64_t *pj, int64_t *count) {
  if (!p || !x || !count || n < 0) return ORC_E_INVALID;
  int d = p->dim;
  size_t nv = (size_t)(n > 0 ? n : 1);
  double *h = malloc(nv * sizeof(double));
  grid_t g;
  memset(&g, 0, sizeof(g));
  int rc = ORC_OK;
  if (!h) return ORC_E_NOMEM;
  orc_field(p, n, x, NULL, h);
  double hmin = INFINITY, hmax = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    hmin = fmin(hmin, h[i]);
    hmax = fmax(hmax, h[i]);
  }
  if (n > 0 && p->search == 0 && p->geometry != ORC_PERIODIC) rc = grid_build(&g, d, n, x, h, p->kappa * hmin);
  cand_t cand = {0, 0, 0};
  int64_t total = 0;
  for (int64_t i = 0; i < n && !rc; ++i) {
    if ((rc = candidates(p, &g, n, x, h, hmax, i, &cand))) break;
    for (int64_t k = 0; k < cand.n; ++k) {
      int64_t j = cand.j[k];
      double e[3];
      double r = separation(p, x, i, j, e);
      if (!(r < p->kappa * 0.5 * (h[i] + h[j]))) continue;
      if (total < cap) {
        pi[total] = i;
        pj[total] = j;
      }
      ++total;
    }
  }
  *count = total;
  free(cand.j);
  grid_free(&g);
  free(h);
  return rc;
}
