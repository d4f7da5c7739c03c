/*
 * mpsph_oracle.h -- FP64 CPU oracle for one relaxation step of the multi-phase SPH
 * mesh generator of Ji, Fu, Hu & Adams, "A Consistent Parallel Isotropic Unstructured
 * Mesh Generation Method based on Multi-phase SPH" (arXiv 1906.07925).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark may load this library.  It shares no code, header, table or
 * helper with the GPU library; the two agree only on the mathematics.
 *
 * Conventions: positions are FP64, array-of-structs x[i*dim + a], in domain units.
 * Particle types: 0 normal, 1 feature surface, 2 feature curve, 3 singularity (fixed)
 * (paper §3.5).  All functions return 0 on success and a positive code on error.
 */
#ifndef MPSPH_ORACLE_H
#define MPSPH_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_PERIODIC = 0, ORC_BOX = 1, ORC_ANNULUS = 2, ORC_BALL = 3, ORC_LEVELSET = 4 };
enum { ORC_UNIFORM = 0, ORC_RADIAL_LINEAR = 1, ORC_SPHERE_DISTANCE = 2, ORC_RBF_EXP = 3, ORC_GRID = 4 };
enum { ORC_NORMAL = 0, ORC_SURFACE = 1, ORC_CURVE = 2, ORC_FIXED = 3 };
enum { ORC_OK = 0, ORC_E_INVALID = 1, ORC_E_NOMEM = 2 };

typedef struct {
  int32_t dim;          /* 2 or 3 */
  int32_t geometry;     /* ORC_PERIODIC | ORC_BOX | ORC_ANNULUS | ORC_BALL */
  double lo[3], hi[3];  /* box (or bounding box) extents, domain units */
  double centre[3];     /* annulus / ball centre */
  double r_in, r_out;   /* annulus radii; ball radius is r_out */
  int32_t field;        /* ORC_UNIFORM | ORC_RADIAL_LINEAR | ORC_SPHERE_DISTANCE | ORC_RBF_EXP */
  double s0;            /* spacing scale of the size field: rho_t = s(x)^-dim */
  double fcentre[3];    /* centre used by the radial / sphere-distance fields */
  double fa, fb;        /* slope and reference radius of the size field */
  int32_t n_rbf;
  const double *rbf_centre; /* n_rbf*dim */
  const double *rbf_coeff;  /* n_rbf */
  double rbf_width;
  double tau, kappa, p0, sigma0;
  int64_t t0, t1;       /* surface-tension ramp (step index); t0 < 0: sigma constant */
  double nu_coeff, c_acc, c_vel, c_visc;
  int32_t search;       /* 0: cell grid, 1: brute force over all pairs */
  int32_t seeded;       /* 1: the boundary features were seeded explicitly; particles keep
                           their type and are reflected back into the region or onto their
                           feature (see project_position) */
  /* Cartesian background mesh (§3.1-3.2): grid_n[a] nodes per axis spanning [lo, hi], node
   * (i, j, k) at index i + n0 (j + n1 k); values interpolated multilinearly. */
  int32_t grid_n[3];
  int32_t pad2_;
  const double *grid_phi; /* level set of ORC_LEVELSET (positive inside), domain units */
  const double *grid_s;   /* relative spacing of ORC_GRID: s = s0 * interpolated value */
} orc_params;

typedef struct {
  /* per-particle outputs, each may be NULL; vectors are n*dim */
  double *rho, *rho_t, *h, *a, *a_abs, *vt, *at, *at_abs, *v, *dr, *nn;
  /* conditioning diagnostics: sum over pair terms of |term| (1 + 3 q / (2 - q)), q = r/h_ij,
   * the relative sensitivity of a kernel-derivative term to a relative change of r */
  double *a_kabs, *at_kabs;
  /* error of the viscous acceleration propagated from a relative error of one unit in every
   * |a_j| term sum: v~ = a dt1 / 2 carries it into the velocity differences and through
   * |v~| into the viscosities of Eq. 21-22; per particle
   *   sum_j |g_ij| (dH_ij |v~_i - v~_j| + H_ij (dv_i + dv_j)),  dv_k = dt1 A_k / 2,
   *   dH_ij = 2 (c_i dv_i + c_j dv_j),  c_k = rho_t,k nu_coeff kappa h_k,
   * with A_k the sum of |pair terms| of a_k, H_ij the harmonic-mean viscosity and g_ij the
   * rest of the pair coefficient.  at_prop_k and at_prop_kn are the same sum with A_k replaced
   * by K_k (the a_kabs sum of particle k) and by K_k / nn_k (nn_k its nearest interacting
   * distance; 0 where it has none): the error bound of a is linear in these three weights, so
   * its propagation into a~ is their combination */
  double *at_prop, *at_prop_k, *at_prop_kn;
  /* scalars of the step */
  double dt1, dt2, sigma, residual_l2, residual_linf, kinetic;
  double elr_mean, elr_std, elr_min, elr_max;
  int64_t pairs, interface_pairs, band_pairs, n_normal, n_elr, nonfinite;
  int64_t interface_particles; /* particles with at least one pair of a different colour */
} orc_out;

double orc_kernel_w(double r, double h, int32_t dim);
/* Multilinear interpolation of node values on the background mesh, with its gradient (may be
 * NULL). */
double orc_grid_interp(const orc_params *p, const double *nodes, const double *x, double *grad);
double orc_kernel_dw(double r, double h, int32_t dim);
double orc_sigma(const orc_params *p, int64_t step);
double orc_spacing(const orc_params *p, const double *x);
double orc_level_set(const orc_params *p, const double *x);
int orc_field(const orc_params *p, int64_t n, const double *x, double *rho_t, double *h);
double orc_field_integral(const orc_params *p, int32_t nq);
/* Boundary features of the region (§2.3, Eq. 6), in the order of the public header: for each,
 * the integral of s^-power over it with the current s0 (power dim-1 on a surface, 1 on a curve,
 * 0 and integral 1 at a corner) and the particle type it carries.  Returns the feature count
 * (at most 26; 0 for a periodic box or a level set).  Midpoint rule, nq intervals per axis. */
int32_t orc_features(const orc_params *p, int32_t nq, double *I, int32_t *type, int32_t *power);
int orc_step(const orc_params *p, int64_t n, double *x, const int32_t *colour, int32_t *type,
             int64_t step, orc_out *out);
int orc_pairs(const orc_params *p, int64_t n, const double *x, int64_t cap,
              int64_t *pi, int64_t *pj, int64_t *count);
int orc_threads(void);

#ifdef __cplusplus
}
#endif
#endif
