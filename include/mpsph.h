/*
 * mpsph.h -- C ABI of the MI355X (gfx950) relaxation-step library for the multi-phase SPH
 * mesh generator of Ji, Fu, Hu & Adams, "A Consistent Parallel Isotropic Unstructured Mesh
 * Generation Method based on Multi-phase SPH" (arXiv 1906.07925).
 *
 * One call of mpsph_step(ctx, 1) performs one pass of the main loop of the paper's
 * Algorithm 1 on the GPU:
 *   target density and scale at the particles           (§2.3 Eq. 1-2, §3.2 Eq. 15-16)
 *   cell-linked neighbour structure                      (the neighbour-list line of Alg. 1)
 *   density summation                                    (§3.3 Eq. 17)
 *   pressure + surface-tension acceleration, gamma = 2   (§3.3 Eq. 18-19, 23-25)
 *   force mapping of feature particles                   (§3.5 Eq. 30-31)
 *   time step, mid-point velocity                        (§3.4 Eq. 29, 26)
 *   viscous acceleration with rho = rho_t                (§3.3 Eq. 20-22)
 *   time step, velocity, drift                           (§3.4 Eq. 29, 27-28)
 *   feature projection / re-tagging                      (§3.5 Eq. 32, last line of Alg. 1)
 *   FP64 global reductions of the step metrics
 *
 * Conventions shared by every entry point
 *  - Status: every int-returning function returns MPSPH_OK (0) or a positive MPSPH_E_* code.
 *    No exception crosses the ABI.  After a device error the context is poisoned and every
 *    later call returns MPSPH_E_STATE until mpsph_destroy().
 *  - Pointers named d_* are device pointers (HIP device memory on the context's device);
 *    all other pointers are host pointers.  The caller owns every buffer it passes in; the
 *    library never keeps a caller pointer after the call returns (parameter arrays are
 *    copied at mpsph_create).
 *  - Streams: every device operation of a context is enqueued on the hipStream_t given at
 *    creation (NULL = the default stream).  mpsph_step() is asynchronous (no host sync);
 *    mpsph_load(), mpsph_metrics(), mpsph_store(), mpsph_debug_*() synchronise that stream.
 *  - Positions are float32, row-major n x dim (x of particle i at d_pos[i*dim + a]), in the
 *    units of the domain given in mpsph_params.  Colours and types are int32 per particle.
 *  - Particle types (§3.5): 0 normal, 1 feature surface, 2 feature curve, 3 singularity
 *    (never moves).  A particle feels neighbour j only if type_j >= type_i.
 *  - A context is not thread-safe; use one context per host thread / stream.
 */
#ifndef MPSPH_H
#define MPSPH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#if defined(__GNUC__) || defined(__clang__)
#define MPSPH_API __attribute__((visibility("default")))
#else
#define MPSPH_API
#endif

enum {
  MPSPH_OK = 0,
  MPSPH_E_INVALID = 1,     /* bad argument or parameter */
  MPSPH_E_NOMEM = 2,       /* device allocation failed or workspace too small */
  MPSPH_E_DEVICE = 3,      /* a HIP call failed */
  MPSPH_E_STATE = 4,       /* context poisoned by an earlier error, or not loaded */
  MPSPH_E_NONFINITE = 5,   /* the last step produced a non-finite value */
  MPSPH_E_UNSUPPORTED = 6, /* valid but unsupported configuration */
  MPSPH_E_SCRATCH = 7      /* needs more workspace than the static scratch array holds
                              (mpsph_create_static) */
};

/* Meshing region: the positive phase of the level set (§3.1, Eq. 14).  MPSPH_LEVELSET: the
 * level set is given at the nodes of a Cartesian background mesh over [lo, hi] (§3.1-3.2) and
 * interpolated multilinearly; particles leaving it are projected by r <- r - phi N (Eq. 32). */
enum { MPSPH_PERIODIC = 0, MPSPH_BOX = 1, MPSPH_ANNULUS = 2, MPSPH_BALL = 3, MPSPH_LEVELSET = 4 };
/* MPSPH_PERIODIC: a cube (square) [lo, hi) without walls, periodic in every axis (minimum-image
 * separations); the cut-off kappa h must stay below half the side (MPSPH_E_UNSUPPORTED). */

/* Target size field s(x); rho_t = s^-dim (unit particle mass, Eq. 15), h = tau s (Eq. 16). */
enum {
  MPSPH_UNIFORM = 0,         /* s = s0 */
  MPSPH_RADIAL_LINEAR = 1,   /* s = s0 (1 + fa (|x - fcentre| - fb)) */
  MPSPH_SPHERE_DISTANCE = 2, /* s = s0 (1 + fa | |x - fcentre| - fb |) */
  MPSPH_RBF_EXP = 3,         /* s = s0 exp(sum_k c_k exp(-|x - mu_k|^2 / (2 w^2))) */
  MPSPH_GRID = 4             /* s = s0 g(x), g interpolated from the background mesh (§3.2) */
};

/* Per-particle quantities that mpsph_debug_fields() can export (values of the last step). */
enum {
  MPSPH_F_RHO = 0,    /* density summation, Eq. 17 (n) */
  MPSPH_F_RHO_T = 1,  /* target density (n) */
  MPSPH_F_H = 2,      /* smoothing length (n) */
  MPSPH_F_A = 3,      /* pressure + surface-tension acceleration after projection (n x dim) */
  MPSPH_F_A_ABS = 4,  /* sum over pairs of |pair term| of F_A (n) */
  MPSPH_F_VT = 5,     /* mid-point velocity v~ (n x dim) */
  MPSPH_F_AT = 6,     /* viscous acceleration after projection (n x dim) */
  MPSPH_F_V = 7,      /* velocity v_{n+1/2} (n x dim) */
  MPSPH_F_DR = 8,     /* displacement of the drift (n x dim) */
  MPSPH_F_NN = 9,     /* distance to the nearest interacting neighbour, +inf if none (n) */
  MPSPH_F_X0 = 10     /* start-of-step position (n x dim) */
};

typedef struct mpsph_ctx mpsph_ctx;

typedef struct {
  int32_t dim;             /* 2 or 3 */
  int32_t geometry;        /* MPSPH_PERIODIC ... MPSPH_LEVELSET */
  double lo[3], hi[3];     /* box, or bounding box of the annulus / ball, domain units */
  double centre[3];        /* annulus / ball centre */
  double r_in, r_out;      /* annulus radii; ball radius is r_out */
  int32_t field;           /* MPSPH_UNIFORM ... MPSPH_GRID */
  double s0;               /* field scale; <= 0: normalise so that the integral of rho_t is n */
  double fcentre[3];
  double fa, fb;           /* slope and reference radius of the radial fields */
  int32_t n_rbf;           /* number of RBF terms (<= 64) */
  const double *rbf_centre;/* host, n_rbf x dim, copied at create */
  const double *rbf_coeff; /* host, n_rbf, copied at create */
  double rbf_width;
  double tau, kappa;       /* h = tau s; cut-off r_c = kappa h, kappa in (0, 2] (the kernel's support is 2h) */
  double p0, sigma0;       /* EOS constant (Eq. 18); initial surface-tension strength (Eq. 25) */
  int64_t t0, t1;          /* ramp of sigma over steps (t0, t1]; t0 = -1: sigma constant; t0 = -2:
                              automatic (t0 detected, t1 = t0 + max(1, round(theta t0)), §3.3) */
  double nu_coeff;         /* nu = nu_coeff r_c |v~| (Eq. 21), 0.1 in the paper */
  double c_acc, c_vel, c_visc; /* constants of Eq. 29: 0.25, 1/40, 0.125 */
  int32_t cell_log2;       /* cells per axis = 2^cell_log2; -1: chosen from the field */
  int32_t debug;           /* 1: keep rho, sum|term|, a~, v, dr, nearest distance of the last step */
  int32_t t0_window;       /* automatic t0: steps the topology must stay static (<= 0: 50) */
  double t0_tol;           /* automatic t0: relative tolerance of "static" (<= 0: 1e-3) */
  double theta;            /* automatic t0: ramp length as a fraction of t0 (<= 0: 0.2) */
  int32_t grid_n[3];       /* background mesh: nodes per axis (>= 2) spanning [lo, hi] */
  const double *grid_phi;  /* host, prod(grid_n[0..dim)) level-set values (MPSPH_LEVELSET), domain
                              units, positive inside; node (i, j, k) at i + n0 (j + n1 k); copied */
  const double *grid_s;    /* host, node values g of the MPSPH_GRID field (> 0); copied */
  int32_t seeded;          /* 0: a normal particle leaving the region is projected onto the
                              boundary and becomes a feature particle (the feature mapping of
                              Alg. 1); a surface particle reaching a box edge becomes a curve
                              particle.  1: the features were seeded with the counts of
                              mpsph_feature_budget: types never change; a normal particle leaving
                              the region is reflected back into it (mirror image through the
                              boundary) and a feature particle stays on its feature, reflected at
                              the walls that bound it */
} mpsph_params;

typedef struct {
  int64_t step;            /* index of the last completed step (steps done - 1), -1 if none */
  int64_t pairs;           /* ordered pairs (i, j != i), r_ij < kappa h_ij, passing the mask */
  int64_t interface_pairs; /* unordered pairs with r_ij < kappa h_ij and different colours */
  int64_t candidates;      /* pair candidates tested by the first pair pass */
  int64_t n_normal;        /* normal particles at the start of the step */
  int64_t n_elr;           /* normal particles with at least one neighbour */
  int64_t nonfinite;       /* particles with a non-finite acceleration or position */
  int64_t n_feature;       /* particles of type >= 1 after the step */
  int64_t pairs_total;     /* sum of `pairs` over all steps since mpsph_load() */
  int64_t candidates_total;/* sum of `candidates` over all steps since mpsph_load() */
  double residual_l2;      /* sqrt(mean over normal particles of (rho/rho_t - 1)^2) */
  double residual_linf;    /* max over normal particles of |rho/rho_t - 1| */
  double kinetic;          /* 1/2 sum |v_{n+1/2}|^2, domain units */
  double dt1, dt2;         /* the two time steps of Eq. 29 */
  double sigma;            /* sigma(t) used in the step */
  double elr_mean, elr_std, elr_min, elr_max; /* nearest distance x rho_t^(1/d), normal particles */
  int64_t interface_particles; /* particles with at least one interface pair */
  int64_t t0;              /* start of the sigma ramp in effect: params t0, or the detected step
                              (-1 while automatic detection has not fired) */
} mpsph_metrics_t;

/* Field scale s0 for which the integral over the meshing region of rho_t = s^-dim equals n
 * (total mass of Eq. 4 with unit particle mass, used to fix the field constant).  Host-only
 * quadrature; params->s0 is ignored.  Errors: MPSPH_E_INVALID for bad params or n <= 0. */
MPSPH_API int mpsph_field_scale(const mpsph_params *params, int64_t n, double *s0_out);

/* Bounds of the target size field over the region's box that the neighbour search relies on
 * (§3.3: the cut-off r_c = kappa h, h = tau s, Eq. 16): out[0] = s0 (as mpsph_create normalises
 * it for n particles, or params->s0 when that is positive), out[1] = s_min, out[2] = s_max and
 * out[3] = a Lipschitz constant of s (domain units).  A pair can interact only within
 * kappa (h_i + h_j) / 2 and h_j <= h_i + tau L r, so these bounds fix the search radius and the
 * default cell size.  For the RBF field they come from the field sampled on a grid, widened by
 * its derivative bounds between nodes.  Host-only; no device.  Errors: MPSPH_E_INVALID for bad
 * params or n <= 0. */
MPSPH_API int mpsph_field_bounds(const mpsph_params *params, int64_t n, double *out);

/* Particle budget of a region whose boundary features carry their own particles (§2.3, Eq. 4-6,
 * with unit particle mass, Eq. 15, so that the particle count equals the total mass M_t).
 *
 * The boundary mass of Eq. 6 is read with the density of the boundary's own dimension at the
 * local target size: a feature surface carries s^-(dim-1) particles per unit area, a feature curve
 * s^-1 per unit length, and a singularity (a box corner) one particle.  The field scale s0 then
 * solves  n = s0^-dim I_v + s0^-(dim-1) I_s + s0^-1 I_c + N_sing  (I_* the integrals at s0 = 1).
 *
 * Features, in this order (each with its mass at s0, its rounded particle count and the type
 * its particles carry):
 *   box, dim 3: 6 faces, face 2a + h lying on coordinate a = (h ? hi : lo) (MPSPH_SURFACE);
 *               then 12 edges, edge 4a + hb + 2 hc running along axis a with the lower-numbered
 *               other axis b at (hb ? hi : lo) and the higher-numbered one c at (hc ? hi : lo)
 *               (MPSPH_CURVE); then 8 corners, corner c having coordinate a at hi when bit a of c
 *               is set (MPSPH_FIXED);
 *   box, dim 2: 4 sides, side 2a + h on coordinate a = (h ? hi : lo) (MPSPH_SURFACE), then the 4
 *               corners numbered as in 3D (MPSPH_FIXED);
 *   ball:       its sphere (dim 3) or circle (dim 2); annulus: the inner, then the outer circle;
 *   periodic:   none.
 * The remaining particles are the interior (MPSPH_NORMAL) ones.  Host-only FP64 quadrature
 * (composite Gauss-Legendre); params->s0 is ignored.  Errors: MPSPH_E_INVALID for bad params,
 * or a count that leaves no interior particle; MPSPH_E_UNSUPPORTED for a level-set region (its
 * zero level is not reconstructed as a surface). */
#define MPSPH_MAX_FEATURES 26
enum { MPSPH_NORMAL = 0, MPSPH_SURFACE = 1, MPSPH_CURVE = 2, MPSPH_FIXED = 3 };
typedef struct {
  double s0;                       /* field scale with the boundary mass included */
  double mass_volume;              /* s0^-dim I_v */
  int64_t n_volume;                /* interior particles: n minus every feature count */
  int32_t n_features;
  int32_t type[MPSPH_MAX_FEATURES];
  double mass[MPSPH_MAX_FEATURES]; /* per feature at s0 (1 for a corner) */
  int64_t count[MPSPH_MAX_FEATURES]; /* rounded mass */
} mpsph_features_t;
MPSPH_API int mpsph_feature_budget(const mpsph_params *params, int64_t n, mpsph_features_t *out);

/* Device bytes a context for n particles needs (state, sort buffers, cell table, partials). */
MPSPH_API size_t mpsph_workspace_bytes(const mpsph_params *params, int64_t n);

/* Create a context for n >= 0 particles.  d_workspace: caller-owned device memory of at least
 * mpsph_workspace_bytes() bytes that outlives the context, or NULL to let the library
 * allocate (and free at destroy).  hip_stream: a hipStream_t or NULL.
 * Errors: MPSPH_E_INVALID (params), MPSPH_E_NOMEM, MPSPH_E_DEVICE, MPSPH_E_UNSUPPORTED
 * (cell grid too large, or a size field whose slope makes the neighbour bound diverge). */
MPSPH_API int mpsph_create(const mpsph_params *params, int64_t n, void *d_workspace, size_t workspace_bytes,
                 void *hip_stream, mpsph_ctx **out);

/* mpsph_create without any device allocation, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).  The
 * context's workspace is a static array of the library, 64 MiB per GPU (held from its first use
 * on a device until the process ends; about 350,000 particles at the default cell size): the
 * same kernels as a context of mpsph_create, on that array.  The caller still passes inputs and
 * outputs (mpsph_load / mpsph_store, as for any context).  The device is the current one.
 *
 * One array per GPU is shared by every static context on it: at most one static context may exist
 * per device at a time (a second creation before mpsph_destroy of the first returns
 * MPSPH_E_STATE), and work enqueued on it from several streams or threads at once races.  The
 * set-up zeroes the part of the array the context uses, so nothing of an earlier context's
 * contents is read.  mpsph_configure / mpsph_autotune keep within the array (MPSPH_E_NOMEM for a
 * configuration that does not fit); mpsph_grad, which allocates checkpoint memory, returns
 * MPSPH_E_UNSUPPORTED.  load, step, metrics, store and destroy allocate nothing.
 * Errors: MPSPH_E_INVALID (params, n), MPSPH_E_SCRATCH (the workspace mpsph_workspace_bytes
 * reports for (params, n) exceeds 64 MiB), MPSPH_E_STATE (the device's array is in use),
 * MPSPH_E_DEVICE, MPSPH_E_UNSUPPORTED (as mpsph_create, or a device index above 63). */
MPSPH_API int mpsph_create_static(const mpsph_params *params, int64_t n, void *hip_stream, mpsph_ctx **out);

/* Batched context: ndom >= 1 independent domains (one mpsph_params and particle count n[d]
 * each; 2D and 3D domains may be mixed; one debug flag for all) advanced together: each kernel
 * of a step is launched once for all domains of one dimension.  Particle arrays passed to
 * mpsph_load / mpsph_store / mpsph_debug_fields hold the domains one after the other in the
 * given order: domain d owns rows [u_d, u_d + n[d]) of the colour / type / scalar arrays,
 * u_d = n[0] + ... + n[d-1], and the n[d] x dim_d row-major block of positions (or vector
 * quantities) that starts at float n[0] dim_0 + ... + n[d-1] dim_(d-1).  A domain evolves
 * exactly (bit for bit) as it would in a context of its own; domains never interact.
 * Workspace and stream as in mpsph_create (mpsph_batch_workspace_bytes gives the size).
 * Errors: MPSPH_E_INVALID (bad params or counts, mixed debug flags, ndom outside [1, 4096]),
 * MPSPH_E_NOMEM, MPSPH_E_DEVICE, MPSPH_E_UNSUPPORTED (more than 2^30 particles, particles x lanes
 * per particle of 2^31 or more, or more than 2^28 cells). */
MPSPH_API size_t mpsph_batch_workspace_bytes(int32_t ndom, const mpsph_params *params, const int64_t *n);
MPSPH_API int mpsph_batch_create(int32_t ndom, const mpsph_params *params, const int64_t *n, void *d_workspace,
                                 size_t workspace_bytes, void *hip_stream, mpsph_ctx **out);

/* Number of domains and total particle count of a context (either pointer may be NULL). */
MPSPH_API int mpsph_domain_count(mpsph_ctx *ctx, int32_t *ndom, int64_t *n_total);

/* Load the particle set: d_pos (n x dim float32, domain units), d_colour (n int32 in
 * [0, 2^16)), d_type (n int32 in [0,3], or NULL for all normal).  Resets the step counter.
 * Every position must lie inside the bounding box [lo, hi] (MPSPH_E_INVALID otherwise). */
MPSPH_API int mpsph_load(mpsph_ctx *ctx, const float *d_pos, const int32_t *d_colour, const int32_t *d_type);

/* Sets the cell exponent (cells per axis 2^cell_log2 for every domain; -1: the library's size
 * rule, or the value given at creation) and the lanes per particle of the pair kernels (2, 4
 * or 8; 4 at creation).  The workspace is re-planned (a library-owned workspace grows when
 * needed); the loaded state is dropped, so call mpsph_load next.  Errors: MPSPH_E_INVALID,
 * MPSPH_E_STATE, MPSPH_E_UNSUPPORTED (grid too large), MPSPH_E_NOMEM (does not fit a caller
 * workspace; the context is unchanged). */
MPSPH_API int mpsph_configure(mpsph_ctx *ctx, int32_t cell_log2, int32_t lanes);

/* Pair-kernel variants (mpsph_set_pair_variant).  Every variant computes the same step bit for bit;
 * they differ in how the work reaches the GPU:
 *   MPSPH_PAIRS_DEFAULT     one launch per pass and dimension group, a block per 256 threads;
 *   MPSPH_PAIRS_PERSISTENT  one persistent launch per pass for all domains of both dimensions: a
 *                           fixed grid (8 blocks per CU) takes the blocks from a work queue in
 *                           device memory (one range per XCD, then stealing), so that uneven
 *                           domains of a batch share every CU (the paper's parallel environment, §3.8, runs
 *                           many sub-domains per node; here many domains per device);
 *   MPSPH_PAIRS_TILE        the density pass of 3D regions without periodic wrap stages the
 *                           neighbours of each block's particles in LDS once (the union of their
 *                           candidate rows, at most 768 particles; larger blocks read through
 *                           the caches) and reads them from there.
 * Measured on MI355X: the default is the fastest on the graded cube and on a 64-domain batch; the
 * others are kept selectable and tested. */
enum { MPSPH_PAIRS_DEFAULT = 0, MPSPH_PAIRS_PERSISTENT = 1, MPSPH_PAIRS_TILE = 2 };

/* Selects the pair-kernel variant of the context's steps (drops a captured step graph).  The
 * state and the layout are kept.  Errors: MPSPH_E_INVALID (unknown variant), MPSPH_E_STATE. */
MPSPH_API int mpsph_set_pair_variant(mpsph_ctx *ctx, int32_t variant);

/* Autotuner of the cell size and of the lanes per particle of the pair kernels.  For every
 * candidate -- cell exponent of the size rule minus one, the rule's, plus one (for domains
 * whose cell_log2 is -1; a fixed cell_log2 is kept), times 2, 4 or 8 lanes per particle -- the
 * context is re-planned, the state d_pos / d_colour / d_type (as for mpsph_load) is loaded,
 * max(warm_steps, 1) steps (warm_steps <= 10000) are run untimed -- the best lane count changes
 * while a lattice relaxes, so warm_steps chooses the stage of the run to tune for -- and
 * probe_steps steps (1 .. 1000) are timed with HIP events on the context's stream.  The fastest candidate is kept and the state loaded into it (step counter
 * 0).  A library-owned workspace grows when a candidate needs more; with a caller workspace,
 * candidates that do not fit are skipped.  Any captured step graph is dropped.  Outputs (may be
 * NULL): the chosen cell exponent of domain 0 and lanes.  Synchronises.
 * Errors: MPSPH_E_INVALID (arguments or state, as mpsph_load), MPSPH_E_STATE, MPSPH_E_DEVICE. */
MPSPH_API int mpsph_autotune(mpsph_ctx *ctx, const float *d_pos, const int32_t *d_colour, const int32_t *d_type,
                             int32_t warm_steps, int32_t probe_steps, int32_t *cell_log2_out, int32_t *lanes_out);

/* Enqueue nsteps >= 0 relaxation steps on the context's stream; returns without waiting. */
MPSPH_API int mpsph_step(mpsph_ctx *ctx, int32_t nsteps);

/* As mpsph_step, but the nsteps steps run as one HIP graph: captured (on a private stream of
 * the context, default priority) at the first call with this nsteps and replayed by later
 * calls, launched on the context's stream.  Every step reads its step index from device
 * memory, so replays follow the same trajectory as mpsph_step.  The graph holds no memset
 * node.  Profiling records one "step_graph" entry per launch instead of per-kernel entries.
 * Errors: MPSPH_E_STATE (not loaded), MPSPH_E_DEVICE (capture or launch failed). */
MPSPH_API int mpsph_step_graph(mpsph_ctx *ctx, int32_t nsteps);

/* Metrics of the last step (synchronises the stream).  Returns MPSPH_E_NONFINITE (with the
 * metrics still written) when that step produced non-finite values. */
MPSPH_API int mpsph_metrics(mpsph_ctx *ctx, mpsph_metrics_t *out);

/* Metrics of domains first .. first + count - 1 of a batched context into out[0 .. count)
 * (mpsph_metrics reports domain 0).  Same synchronisation and MPSPH_E_NONFINITE rule. */
MPSPH_API int mpsph_domain_metrics(mpsph_ctx *ctx, int32_t first, int32_t count, mpsph_metrics_t *out);

/* Current positions (n x dim float32, domain units) and types (n int32) in the original
 * particle order of mpsph_load().  Either pointer may be NULL.  Synchronises. */
MPSPH_API int mpsph_store(mpsph_ctx *ctx, float *d_pos, int32_t *d_type);

/* Copy one per-particle quantity of the last step (MPSPH_F_*) into d_out (float32, n or
 * n x dim values, original particle order, domain units).  MPSPH_F_RHO, MPSPH_F_A_ABS, MPSPH_F_AT,
 * MPSPH_F_V, MPSPH_F_DR and MPSPH_F_NN need params.debug = 1.  Synchronises.  Errors: MPSPH_E_INVALID (unknown field), MPSPH_E_STATE. */
MPSPH_API int mpsph_debug_fields(mpsph_ctx *ctx, int32_t which, float *d_out);

/* Cell structure of the last step: d_key (n uint32, the cell key of each particle in
 * original order: cellbase + xf + 2^(k+xe) row, where cellbase is 0 for a single domain and in a
 * batch the first cell of the domain's range of the global cell table; xf = cx 2^xe + floor(ox 2^xe)
 * is the x cell at 2^xe sub-cells per cell (ox the float32 offset in [0, 1) within the cell,
 * xe the largest of 0..4 with dim k + xe <= 26 and 2^(dim k + xe) <= 4 n for the domain's n
 * particles, so a domain has 2^(dim k + xe) cells); row = cy in 2D, and in 3D the
 * rows are numbered in tiles of 2^ly x 2^lz rows, ly = min(4, k), lz = min(4, k):
 * row = (cy mod 2^ly) + 2^ly (cz mod 2^lz) + 2^(ly+lz) floor(cy / 2^ly) + 2^(k+lz) floor(cz / 2^lz)),
 * d_cell_start
 * (ncells + 1 uint32: index of the first sorted particle of each cell, last entry n) -- either
 * may be NULL -- and the host values ncells (all domains) and cell_log2 (of domain 0).  The
 * two host values are available from creation on; the arrays need a completed step.
 * Synchronises. */
MPSPH_API int mpsph_debug_cells(mpsph_ctx *ctx, uint32_t *d_key, uint32_t *d_cell_start, int64_t *ncells,
                      int32_t *cell_log2);

/* Neighbour pairs of the last step (for testing at small n): the ordered pairs (i, j), j != i,
 * with |x_i - x_j| < kappa (h_i + h_j) / 2 at the start of that step, before the type mask is
 * applied (the pair set of Alg. 1's neighbour list; §3.3 Eq. 17-20), as load indices.  Up to
 * cap pairs are written to d_i[k], d_j[k] (device, uint32) in an unspecified order; *count
 * (host) receives the total number of pairs, which may exceed cap.  Synchronises.
 * Errors: MPSPH_E_INVALID (cap < 0, NULL arrays with cap > 0), MPSPH_E_STATE (no step yet). */
MPSPH_API int mpsph_debug_pairs(mpsph_ctx *ctx, int64_t cap, uint32_t *d_i, uint32_t *d_j, int64_t *count);

/* Replace the RBF coefficients c_k of the size field s = s0 exp(sum_k c_k G_k(x)) of one domain
 * (n_rbf host doubles, copied).  s0 is kept (the field is not renormalised), the cell grid is
 * kept and the neighbour search bounds are recomputed for the new field.  Synchronises.
 * Errors: MPSPH_E_INVALID (domain out of range, field not MPSPH_RBF_EXP, non-finite value),
 * MPSPH_E_UNSUPPORTED (the new field's slope makes the neighbour bound diverge; the old
 * coefficients stay in place). */
MPSPH_API int mpsph_set_field_coeff(mpsph_ctx *ctx, int32_t domain, const double *coeff);

/* Gradient of a relaxation loss by a hand-written adjoint (reverse mode) of the step.
 * From the current state, runs nsteps steps (the state and step counter advance exactly as
 * with mpsph_step(ctx, nsteps)), evaluates at the final positions
 *   L = (1/n) sum_i (rho_i / rho_t,i - 1)^2 + (lambda / n) sum_{i<j, C_i != C_j} W(r_ij, h_ij) / W(0, h_ij)
 * (density summation of §3.3 Eq. 17 with the target density of Eq. 16; the second term is a
 * smooth measure of the interface between colours, §3.3 Eq. 23-25), and propagates dL back
 * through every step of Algorithm 1's loop: the pair forces (Eq. 18, 23), the force mapping
 * (Eq. 30-31), both time steps (Eq. 29; through the particle that attains the minimum), the
 * viscous pass (Eq. 20-22), the velocity and drift (Eq. 26-28) and the wall clamp (Eq. 32).
 * Pair sets, type masks and re-tagging are held fixed (piecewise constant).
 * Memory: the states at every ckpt_every-th step are kept, and a segment of ckpt_every steps is
 * recomputed with its per-step record (about 80 bytes per particle and step plus the cell table);
 * the library allocates this device memory on first use and keeps it until mpsph_destroy.
 * Outputs (each may be NULL): *loss_out (host), grad_coeff_out[n_rbf] = dL/dc_k (host, only for
 * MPSPH_RBF_EXP fields), d_grad_pos = dL/dx of the positions at the call (device, n x dim
 * float32, load order, domain units).  Debug exports after the call refer to a recomputed
 * step, not to the last one.  Single-domain contexts with a box region and a uniform or RBF
 * field.  Synchronises.  Errors: MPSPH_E_INVALID (nsteps < 0, ckpt_every < 1), MPSPH_E_STATE,
 * MPSPH_E_UNSUPPORTED (batched context, other region or field, seeded features), MPSPH_E_NOMEM. */
MPSPH_API int mpsph_grad(mpsph_ctx *ctx, int32_t nsteps, int32_t ckpt_every, double lambda, double *loss_out,
                         double *grad_coeff_out, float *d_grad_pos);

/* Per-kernel timing with HIP events on the context's stream.  enable = 1 starts recording
 * every kernel, 2 only the pair passes (the kernels named pass_*: two events per launch slow a
 * step by a few per cent, so a throughput measurement records only the kernels it needs), 0
 * stops; 1 and 2 reset the accumulators.  mpsph_profile_read() synchronises and returns, for up
 * to cap kernels, the name, the number of launches and the summed milliseconds.
 * Errors: MPSPH_E_INVALID (enable outside [0, 2]), MPSPH_E_STATE. */
MPSPH_API int mpsph_profile(mpsph_ctx *ctx, int32_t enable);
MPSPH_API int mpsph_profile_read(mpsph_ctx *ctx, int32_t cap, const char **names, int64_t *launches,
                       double *ms, int32_t *count);

MPSPH_API void mpsph_destroy(mpsph_ctx *ctx);
MPSPH_API const char *mpsph_strerror(int status);

#ifdef __cplusplus
}
#endif
#endif /* MPSPH_H */
