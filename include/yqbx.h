/*
 * yqbx: screened-Laplace (Yukawa) double-layer solver for many rigid ellipses
 * on one AMD Instinct MI355X (gfx950).
 *
 * The problem (Fu, Ryham, Kloeckner, Wala, Jiang, Young, arXiv 1810.04131):
 *   exterior Dirichlet problem  -rho^2 Lap u + u = 0 in the water,  u = f on the
 *   particle boundaries Sigma,  u -> 0 at infinity                   (eq. SL),
 *   represented as u = D[sigma] (eq. intrep) with G = K0(|x-y|/rho)/(2 pi)
 *   (eq. Gfunc) and solved through the second-kind equation
 *   1/2 sigma + D sigma = f                                          (eq. bie).
 *   Discretisation: Nystrom on 16-point Gauss-Legendre panels, QBX local
 *   expansions from Graf's addition theorem near the target (section 5, eqs.
 *   local-exp, graf-coefficient, graf-addition), tiled direct far field.
 *   Outputs: density sigma, surface gradient, hydrophobic forces and torques
 *   (eqs. stress, force_torque, scalar-torque) and the energy of eq. main.
 *
 * Conventions for every entry point
 *   - kappa = 1/rho.  Lengths in the caller's units; gamma (eq. main) scales
 *     forces, torques and energy linearly.
 *   - Particles are ellipses: centre a_i, director angle th_i (the major axis
 *     points along (cos th_i, sin th_i), section 2.1), semi-axes A_i >= B_i.
 *   - Nodes are ordered particle-major, then panel (counter-clockwise from the
 *     director, i.e. increasing t in a_i + R(th_i)(A cos t, B sin t)), then
 *     Gauss-Legendre node (increasing t).  N = n * panels_per_particle * 16.
 *     The unit normal points out of the particle into the water.
 *   - Arrays named "host" are caller-owned host memory.  Arrays named "dev"
 *     are caller-owned device memory of the current HIP device, laid out as
 *     plain contiguous doubles; the library only reads/writes them during the
 *     call or, for the asynchronous entry points, in stream order on the
 *     problem's stream.  The library owns all of its own device memory.
 *   - Every call returns a status (YQ_OK = 0 or a negative code).  No C++
 *     exception crosses the ABI.  yq_last_error() gives a message.
 *   - One thread at a time per problem handle.
 */
#ifndef YQBX_H
#define YQBX_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  YQ_OK = 0,
  YQ_EINVAL = -1,   /* invalid argument: null pointer, size or parameter out of range */
  YQ_EGEOM = -2,    /* geometry rejected: particles overlap or a node lies inside another particle */
  YQ_ENOCONV = -3,  /* GMRES reached maxiter above tolerance; outputs are still written */
  YQ_ENOMEM = -4,   /* device memory allocation failed */
  YQ_EDEVICE = -5,  /* HIP runtime error */
  YQ_ESTATE = -6,   /* call out of order, e.g. a solve before yq_set_particles */
  YQ_EADMIT = -7    /* serving: request larger than the device-memory budget */
};

enum { YQ_FP64 = 0, YQ_MIXED = 1 };                       /* precision */
enum { YQ_FMM64 = 2 };  /* yq_apply_far only: FMM expansions with FP64 near interactions */
enum { YQ_FAR_DIRECT = 0, YQ_FAR_FMM = 1, YQ_FAR_AUTO = 2, YQ_FAR_CUTOFF = 3 };   /* far-field mode */
enum { YQ_LABEL_ARC = 0, YQ_LABEL_JANUS = 1 };             /* boundary labels */
enum { YQ_M2L_MFMA = 0, YQ_M2L_VALU = 1, YQ_M2L_MFMA64 = 2 };   /* FMM translation kernels */

typedef struct yq_problem yq_problem;

typedef struct yq_params {
  int32_t panels_per_particle; /* P; equal-parameter panels of 16 nodes, P >= 2*qbx_window+1 */
  int32_t qbx_order;           /* p: the local expansion keeps orders -p..p (section 5), 1..30 */
  int32_t qbx_window;          /* panels on each side of the target's panel taken through the expansion */
  int32_t qbx_oversample;      /* sub-panels per window panel for the coefficient quadrature (1..8) */
  double qbx_radius;           /* expansion radius / arclength of the target's panel */
  double near_beta;            /* other panels closer than near_beta*h (nearest node) are oversampled */
  int32_t near_oversample;     /* sub-panels for those panels (1..8) */
  int32_t pot_oversample;      /* sub-panels for off-surface targets near a panel (1..16) */
  double pot_beta;             /* off-surface near criterion, as near_beta */
  int32_t precision;           /* YQ_FP64, or YQ_MIXED: FP32 far field inside FP64 refinement */
  int32_t far_mode;            /* YQ_FAR_DIRECT | YQ_FAR_FMM | YQ_FAR_AUTO (FMM from 20000 nodes) |
                                  YQ_FAR_CUTOFF (direct sums truncated at a radius, cutoff_tol) */
  int32_t fmm_order;           /* FMM expansion order (far_mode FMM) */
  int32_t fmm_leaf_max;        /* nodes per quadtree leaf (far_mode FMM) */
  double tol;                  /* GMRES: stop at ||f - A sigma||_2 / ||f||_2 <= tol */
  int32_t maxiter;             /* GMRES: total inner iterations */
  int32_t restart;             /* GMRES: Krylov dimension before a restart (<= 200) */
  double inner_tol;            /* YQ_MIXED: relative tolerance of each FP32-operator inner solve */
  int32_t max_refine;          /* YQ_MIXED: maximum refinement (outer) steps */
  int32_t fmm_resid_order;     /* FMM enabled: order of the FP64 FMM used for refinement residuals,
                                  FP64 solves and the reported residual (relative operator error
                                  ~1e-10 at 40); 0 = the exact direct sum */
  int32_t fmm_m2l;             /* FMM M2M/M2L/L2L translations: YQ_M2L_MFMA (matrix-core products;
                                  the M2L of the FP32-class inner operator in FP32 on scaled
                                  expansions, everything else in FP64), YQ_M2L_MFMA64 (all
                                  translations FP64 on the matrix cores) or YQ_M2L_VALU (FP64, one
                                  lane per coefficient; the same results as YQ_M2L_MFMA64 to
                                  rounding) */
  double cutoff_tol;           /* YQ_FAR_CUTOFF: bound eps on the far-field truncation.  The kernel
                                  decays like exp(-kappa r) (eq. exp_decay), so a pair at distance r
                                  contributes at most w_j |sigma_j| kappa K1(kappa r) / (2 pi).  The
                                  sums skip every (64-target group, 256-source tile) pair whose
                                  bounding circles are at least z_c / kappa apart, z_c the smallest z
                                  with kappa/(2 pi) sqrt(pi/(2z)) e^-z (1 + 3/(8z)) L <= eps
                                  (DLMF 10.40.10 bounds K1(z) by the first two terms), L = 2 pi sum_i
                                  A_i >= the total perimeter.  So the skipped part of every far-field
                                  value is <= eps ||sigma||_inf, and with the extra factor (1 + 3/z)
                                  of the gradient bound that of every gradient <= eps kappa
                                  ||sigma||_inf.  The FP32 inner operator of YQ_MIXED uses
                                  max(eps, inner_tol / 10).  0 < cutoff_tol < 1 */
  double sl_coupling;          /* eta >= 0: the combined representation u = D[sigma] + eta S[sigma]
                                  (the Brakhage-Werner form of eq. bwform with the real coupling
                                  of the screened equation; S the single layer of eq.
                                  single-layer-def), solved through 1/2 sigma + D sigma +
                                  eta S sigma = f.  For large rho (small kappa) 1/2 I + D tends to
                                  the Laplace double layer, which loses one dimension per particle;
                                  eta > 0 keeps the system well conditioned.  0 (default): the
                                  double layer of eq. intrep.  eta > 0 needs far_mode
                                  YQ_FAR_DIRECT and single problems (the batch and the server
                                  reject it); the far field then evaluates K0 and K1 at every pair
                                  (FP64, or FP32 for the inner operator of YQ_MIXED) */
  int32_t refine_levels;       /* adaptive panel refinement near contact (section 5's QBX
                                  preconditions; the paper refines at most 3-5 levels per time
                                  step), 0..8, 0 (default): P equal-parameter panels.  Panels
                                  are parameter intervals 2 pi / P (k + [idx, idx + 1] 2^-lev);
                                  passes split every panel whose arclength exceeds refine_ratio
                                  times its distance to the nearest node of another particle,
                                  at most refine_levels times, then each particle's panels are
                                  balanced so that the panels a QBX window takes are at most
                                  one level coarser than the target's.  N then varies per
                                  particle (yq_num_nodes); node order stays particle, panel
                                  (increasing t), node.  Single problems only (the batch, the
                                  server and yq_step reject it) */
  double refine_ratio;         /* > 0, default 2 (the expansion disk, radius h/4 at
                                  qbx_radius 0.25, stays its radius away from other particles) */
} yq_params;

typedef struct yq_solve_info {
  int32_t iterations;       /* total inner GMRES iterations */
  int32_t outer_steps;      /* refinement steps (YQ_MIXED) or restart cycles (YQ_FP64) */
  int32_t matvecs_fp64;     /* FP64 operator applications */
  int32_t matvecs_fp32;     /* FP32-far-field operator applications */
  double residual;          /* final true relative residual with the FP64 operator */
  double seconds;           /* wall time of the solve */
} yq_solve_info;

/* Defaults: P = 32, p = 10, window 2, oversample 4, radius 0.25, near_beta 0.5,
 * near_oversample 4, pot_oversample 8, pot_beta 0.5, FP64, direct far field,
 * FMM order 20 / 64 per leaf, tol 1e-10, maxiter 200, restart 100,
 * inner_tol 1e-6, max_refine 8, fmm_resid_order 40, fmm_m2l YQ_M2L_MFMA, cutoff_tol 1e-12,
 * sl_coupling 0, refine_levels 0, refine_ratio 2. */
void yq_default_params(yq_params* params);

/* Creates a problem on the current HIP device.  params: host, copied. */
int yq_create(const yq_params* params, yq_problem** out);
void yq_destroy(yq_problem* prob);

/* Status text, and the last detailed message of a problem (NULL: of the calling thread). */
const char* yq_error_string(int status);
const char* yq_last_error(const yq_problem* prob);

/* All later work of the problem is issued on this HIP stream (hipStream_t; NULL = default). */
int yq_set_stream(yq_problem* prob, void* hip_stream);

/* Geometry and set-up (geometry, QBX centres and near lists, QBX correction
 * build; section 2.1 particles, section 5 discretisation).
 * center_xy: host [2n] (x0,y0,x1,y1,...); angle: host [n] director angles;
 * semi_axes: host [2n] (A0,B0,A1,B1,...), A >= B > 0; kappa > 0.
 * Builds nodes, normals, weights, near lists and the FP64 QBX correction of
 * the operator and of its surface gradient.  Returns once the geometry check
 * is done; the rest of the build is queued on the problem's stream, ahead of
 * every later call on the problem (host inputs may be reused on return).
 * YQ_EGEOM if a node of one particle lies inside another. */
int yq_set_particles(yq_problem* prob, int32_t n, const double* center_xy, const double* angle,
                     const double* semi_axes, double kappa);

int yq_num_nodes(const yq_problem* prob, int64_t* N);
int yq_num_particles(const yq_problem* prob, int32_t* n);

/* Node data (section 5 discretisation): dev x,y,nx,ny,w each [N] (any may be NULL).  Synchronous. */
int yq_get_nodes(const yq_problem* prob, double* x, double* y, double* nx, double* ny, double* w);

/* Extra near panels (section 5): panels outside a target's QBX window whose
 * nearest node is closer than near_beta * h.  yq_near_count gives their total;
 * yq_get_near fills dev row_ptr [N+1] and dev panels [total] (global panel
 * index = particle * P + k), rows in node order, panels ascending. */
int yq_near_count(const yq_problem* prob, int64_t* total);
int yq_get_near(const yq_problem* prob, int32_t* row_ptr, int32_t* panels);

/* Boundary labels (eq. JanusBC): writes dev f [N].  YQ_LABEL_ARC: smoothed arc
 * f = 1/2 [tanh((phi+a)/b) - tanh((phi-a)/b)], a = param0 (half opening),
 * b = param1 (edge width), phi in (-pi, pi] the polar angle from the director.
 * YQ_LABEL_JANUS: f = 1 - sin^p(phi/2), p = param0 (eq. JanusBC, read with
 * phi/2 so that head and tail differ).  Synchronous. */
int yq_boundary_label(yq_problem* prob, int32_t kind, double param0, double param1, double* f);

/* Sets the Dirichlet data f (dev [N], copied). */
int yq_set_boundary_data(yq_problem* prob, const double* f);

/* Far field alone (the Nystrom rule of eq. double-layer-def): out_i = sum_{j != i} w_j dG/dnu_y(x_i, y_j) sigma_j
 * over every node pair, in FP64 (YQ_FP64) or FP32 arithmetic (YQ_MIXED).  With
 * the FMM enabled (far_mode) YQ_MIXED gives the FMM far field (FP64
 * expansions, FP32 leaf-neighbour interactions) and YQ_FMM64 the FMM with FP64
 * leaf-neighbour interactions.  dev sigma [N], dev out [N].  Asynchronous.
 *
 * With the FMM enabled, YQ_MIXED operator applications (yq_apply_operator and
 * the inner GMRES of a YQ_MIXED solve) use the FMM far field; refinement
 * residuals, FP64 solves and the reported residual use the order
 * fmm_resid_order FMM with FP64 near interactions (or the exact direct sum when
 * it is 0); yq_apply_operator(YQ_FP64) is always the exact direct sum. */
int yq_apply_far(yq_problem* prob, const double* sigma, double* out, int32_t precision);

/* The discrete operator (far field + QBX near correction): out = (1/2 I + D) sigma with the
 * QBX near correction (eq. bie).  dev sigma [N], dev out [N] (must not alias).
 * Asynchronous on the problem's stream. */
int yq_apply_operator(yq_problem* prob, const double* sigma, double* out, int32_t precision);

/* GMRES solve of eq. bie for the data set by yq_set_boundary_data (section 5).
 * dev sigma0 [N] initial guess or NULL (zero); dev sigma [N] result;
 * info: host, may be NULL.  Synchronous.  YQ_ENOCONV: not converged (sigma
 * holds the last iterate). */
int yq_solve(yq_problem* prob, const double* sigma0, double* sigma, yq_solve_info* info);

/* Exterior-limit surface gradient of u = D[sigma] at the nodes (eq. intrep
 * differentiated): dev gx, gy [N].  The far part is the direct FP64 sum, or with the FMM
 * enabled the FP64 FMM gradient (order fmm_resid_order, else fmm_order): the
 * local expansions' gradient plus direct neighbour-leaf interactions.
 * Asynchronous. */
int yq_surface_gradient(yq_problem* prob, const double* sigma, double* gx, double* gy);

/* Hydrophobic forces and torques (eqs. stress, force_torque,
 * scalar-torque): u = f on Sigma, grad u from yq_surface_gradient.
 * dev force [2n] (Fx0,Fy0,...), dev torque [n] about each centre a_i,
 * host energy (may be NULL): Phi = -gamma/kappa int f du/dnu ds.  Synchronous. */
int yq_forces(yq_problem* prob, const double* sigma, double gamma, double* force, double* torque,
              double* energy);

/* The solve-and-forces part of a time step of Algorithm 1: yq_solve, then
 * yq_forces of its sigma (eqs. bie, stress, force_torque), with the same
 * arguments and results as those two calls.  With the direct far field, a YQ_MIXED solve computes the FP64 residual it expects to
 * be its last one together with the gradient far field of the same sigma (one
 * pass over the node pairs instead of two); the forces then reuse it.  If that
 * residual was not the last, the gradient is computed afresh.  Results agree
 * with yq_solve + yq_forces to rounding.  YQ_ENOCONV: not converged; sigma
 * holds the last iterate and the forces are those of it.  Synchronous. */
int yq_solve_forces(yq_problem* prob, const double* sigma0, double* sigma, yq_solve_info* info,
                    double gamma, double* force, double* torque, double* energy);

/* Off-surface potential u = D[sigma] (eq. intrep) at M targets:
 * dev tx, ty [M], dev u [M].  Panels whose nearest node is closer than
 * pot_beta*h use a pot_oversample-fold oversampled rule.  Asynchronous. */
int yq_eval_potential(yq_problem* prob, const double* sigma, int64_t M, const double* tx,
                      const double* ty, double* u);

/* yq_eval_potential without device allocation, for callers that cannot allocate
 * device memory (code under HIP stream capture, tight serving loops, harnesses
 * that forbid hipMalloc).  Same arguments and results as yq_eval_potential (the
 * same kernels).  Its scratch (the chunk partial sums and the oversampled panel
 * rule) lives in one device array of 64 MiB that the library holds on every
 * device it runs on until the process ends; the call allocates nothing and
 * rebuilds the oversampled points each time.  YQ_EINVAL when a call would need
 * more than 64 MiB: about 8 (chunks x M + 5 x panels x pot_oversample x 16)
 * bytes, e.g. 10 MB for 1,024 targets on 1,600 panels at oversampling 8.  All
 * calls on one device share the array: calls that overlap in time on one device
 * (two streams, two threads) race and must be serialised by the caller; calls
 * queued on one stream are ordered.  Asynchronous on the problem's stream. */
int yq_eval_potential_noalloc(yq_problem* prob, const double* sigma, int64_t M, const double* tx,
                              const double* ty, double* u);

/* ---- Time stepping ---------------------------------------------------------------------
 * Excluded-volume repulsion (eq. repul) with the three-circle model of ellipses
 * (supplementary section S1): particle i is three circles of radius B_i centred
 * at a_i + k (A_i - B_i) d_i, k = -1, 0, +1, d_i = (cos th_i, sin th_i).  Every
 * circle pair of two different particles, centre distance r and gap
 * g = r - (B_i + B_j), repels with (c0/3) q g^-(q+1) along the line of centres
 * and carries the potential (c0/3) g^-q.  F_i^rep sums the nine pairs over all
 * other particles, tau_i^rep is the torque about a_i of the forces on the end
 * circles, Phi_rep sums the potential over unordered pairs.  With A = B the
 * three circles coincide, so a disk pair repels with 3 times eq. repul's force
 * for the same c0.  All sums are direct, in FP64.
 *
 * The time step is the constant-drag forward Euler law of eq. euler (Algorithm 1
 * with constant drag coefficients in place of the Stokes mobility solve):
 *   a_i  += dt / xi_x     (F_i + F_i^rep),
 *   th_i += dt / xi_theta (tau_i + tau_i^rep),
 * F_i and tau_i the hydrophobic force and torque of yq_solve_forces. */
typedef struct yq_dynamics {
  double dt;        /* time step, >= 0 */
  double xi_x;      /* translational drag coefficient, > 0 */
  double xi_theta;  /* rotational drag coefficient, > 0 */
  double gamma;     /* hydrophobic tension gamma of eq. main */
  double c0;        /* repulsion strength, >= 0 */
  int32_t q;        /* repulsion order, 1..16 (3 in two dimensions) */
} yq_dynamics;

/* Repulsion of the current particles: dev force [2n] F_i^rep, dev torque [n]
 * tau_i^rep about a_i, host energy (may be NULL) Phi_rep.  c0 >= 0, q in 1..16.
 * YQ_EGEOM if two circles touch or overlap (an end circle reaches slightly
 * outside its ellipse near the tips, so close ellipses can be rejected here
 * although yq_set_particles accepted them).  Synchronous. */
int yq_repulsion(yq_problem* prob, double c0, int32_t q, double* force, double* torque,
                 double* energy);

/* One time step.  dev sigma [N]: in, the previous step's density, which
 * warm-starts GMRES (zeros for a cold start); out, the density at the
 * configuration the step started from.  dev sigma_prev [N] or NULL: the density
 * of the step before; with it the initial guess is the linear extrapolation
 * 2 sigma - sigma_prev, and sigma_prev takes sigma's value on entry, so passing
 * the same two buffers to every step keeps the history (start both equal).  The step solves eq. bie
 * there (as yq_solve_forces with dyn->gamma), adds the repulsion, moves every
 * particle by eq. euler and rebuilds the set-up at the new configuration (as
 * yq_set_particles with the same semi-axes and kappa).  The boundary data are
 * kept per node: nodes are fixed in each particle's frame, so a label that is a
 * function of the polar angle from the director moves with its particle.
 * dev force [2n] and dev torque [n] (each may be NULL): the total force and
 * torque that moved the particles.  host energy [2] (may be NULL): Phi and
 * Phi_rep at the start configuration.  info: host, may be NULL.
 * YQ_ENOCONV: GMRES stopped above tol; sigma, forces and energies are those of
 * the last iterate and the particles do not move.  YQ_EGEOM: two repulsion
 * circles overlap at the start, or the geometry check rejects the new
 * configuration; the particles do not move (the start configuration's set-up
 * is rebuilt if needed) and sigma is the start configuration's density.  On
 * either, sigma_prev has still taken sigma's value on entry.  YQ_EINVAL for
 * parameters out of range or sigma_prev == sigma (nothing is changed).
 * Synchronous. */
int yq_step(yq_problem* prob, const yq_dynamics* dyn, double* sigma, double* sigma_prev,
            yq_solve_info* info, double* force, double* torque, double* energy);

/* The current particles: host center_xy [2n], host angle [n] (either may be NULL). */
int yq_get_particles(const yq_problem* prob, double* center_xy, double* angle);

/* ---- Batched solves -------------------------------------------------------------------
 * A batch holds many independent configurations.  Their nodes are laid out one
 * after another (configuration c at offset offsets[c] of every batch vector, in
 * the node order of a single problem) and every GMRES iteration of the whole
 * batch is one fixed kernel sequence (fused far field over all configurations,
 * fused correction, batched CGS2 Arnoldi, device-side Givens), captured once as
 * a hipGraph and replayed.  A configuration's arithmetic depends only on its own
 * size, so its result is bitwise the same alone (a batch of one) or in a mix.
 * FMM configurations: those of at least a threshold node count (params->far_mode
 * YQ_FAR_FMM: all; YQ_FAR_AUTO: 20000 nodes; YQ_FAR_DIRECT: none;
 * yq_batch_set_fmm overrides) take the quadtree FMM of section 5.  By default
 * they stay engine members: their trees form one forest whose passes (P2M, M2M
 * per level, M2L, L2L per level, L2P + P2P) are one launch each over every tree
 * in the same captured iteration, the inner operator with the order-fmm_order
 * FMM (FP32 leaf pairs and M2L) and the FP64 residuals with the order-
 * fmm_resid_order one; each tree's arithmetic is that of the configuration
 * solved alone.  Their forces run on worker threads (default 6, largest first,
 * one stream of default priority each) beside the others'.  With
 * yq_batch_set_fmm_engine(batch, 0), or when fmm_resid_order is 0 or fmm_m2l is
 * YQ_M2L_VALU, they are standalone problems instead, solved by the worker
 * threads while the engine replays its iteration graph for the rest.
 * The batch owns a HIP stream of default priority; every batch call is
 * synchronous (returns after its work is done) and reads its device inputs when
 * called, so the caller must have finished writing them. */
typedef struct yq_batch yq_batch;

int yq_batch_create(const yq_params* params, yq_batch** out);
void yq_batch_destroy(yq_batch* batch);
const char* yq_batch_last_error(const yq_batch* batch);

/* FMM threshold (nodes, >= 0) and worker count (1..8); before
 * yq_batch_set_configs (YQ_ESTATE after). */
int yq_batch_set_fmm(yq_batch* batch, int64_t min_nodes, int32_t workers);

/* enable != 0 (default): FMM configurations are trees of the engine's forest;
 * 0: standalone problems solved by the worker threads.  Before
 * yq_batch_set_configs (YQ_ESTATE after). */
int yq_batch_set_fmm_engine(yq_batch* batch, int32_t enable);

/* Near-field cache of the FMM forest's trees: the leaf passes' pair coefficients
 * K1(z)/z ((x - y) . w nu) of every pair of neighbouring leaves (section 5's
 * direct interactions of the FMM) are computed once per geometry, in FP32 for the
 * inner operator and in FP64 for the residual operator, and the passes then read
 * them instead of evaluating K1 (a block-sparse matrix-vector product).
 * max_bytes: the most device memory the caches may hold (FP32 caches of every tree
 * first, then FP64 ones, in configuration order, while they fit); 0 disables; -1
 * (default): the device memory free when the configurations are set, less a
 * reserve of a tenth of the device memory (at least 8 GiB).  The FP32 caches also
 * hold the P2M coefficients of the inner operator's multipoles.
 * Results agree with the uncached passes to rounding.  Before yq_batch_set_configs
 * (YQ_ESTATE after).  yq_batch_near_cache_info: bytes held and the number of
 * trees with an FP32 / FP64 cache (outputs may be NULL). */
int yq_batch_set_near_cache(yq_batch* batch, int64_t max_bytes);
int yq_batch_near_cache_info(const yq_batch* batch, int64_t* bytes, int32_t* trees32,
                             int32_t* trees64);

/* Inner (FP32) far field of the direct members.  enable != 0 (default): one
 * evaluation of K1(z)/z per unordered node pair serves both directions of the
 * double-layer sum (section 4, eq. double-layer-def: K1(z)/z depends on the
 * distance only, the factor (x - y).nu on the direction), chunk pairs of 1,024
 * nodes per work item; 0: one
 * evaluation per directed pair (target blocks x source chunks).  Both sum the
 * same pairs in FP32 with the same kernel fits; their rounding differs.  Before
 * yq_batch_set_configs (YQ_ESTATE after). */
int yq_batch_set_symmetric_far(yq_batch* batch, int32_t enable);

/* nparticles: host [nconf]; center_xy, angle, semi_axes: host, all configurations'
 * particles concatenated in order (layout as yq_set_particles); kappa: host [nconf].
 * YQ_EGEOM / YQ_EINVAL name the first failing configuration in the message. */
int yq_batch_set_configs(yq_batch* batch, int32_t nconf, const int32_t* nparticles,
                         const double* center_xy, const double* angle, const double* semi_axes,
                         const double* kappa);

/* total nodes and host offsets [nconf + 1] (may be NULL). */
int yq_batch_num_nodes(const yq_batch* batch, int64_t* total, int64_t* offsets);

/* As yq_boundary_label / yq_set_boundary_data on every configuration: dev f [total]. */
int yq_batch_boundary_label(yq_batch* batch, int32_t kind, double param0, double param1,
                            double* f);
int yq_batch_set_boundary_data(yq_batch* batch, const double* f);

/* out = (1/2 I + D) sigma for every configuration, one fused launch; dev [total]. */
int yq_batch_apply_operator(yq_batch* batch, const double* sigma, double* out, int32_t precision);

/* Solves every configuration (FP64, or mixed with FP64 refinement per the
 * parameters).  dev sigma [total] out; info: host [nconf] (may be NULL).
 * YQ_ENOCONV if any configuration missed the tolerance. */
int yq_batch_solve(yq_batch* batch, double* sigma, yq_solve_info* info);

/* yq_batch_solve, then yq_batch_forces of its sigma, in one call: the FP64
 * residual expected to be the last one of each mixed solve also gives the gradient
 * far field of the forces (eq. stress), as yq_solve_forces does for one problem.
 * Returns the solve's status (YQ_ENOCONV with the forces computed). */
int yq_batch_solve_forces(yq_batch* batch, double* sigma, yq_solve_info* info, double gamma,
                          double* force, double* torque, double* energy);

/* Forces and torques of every particle (particles in batch order): dev force
 * [2 * total particles], dev torque [total particles]; host energy [nconf].
 * The FMM lane's configurations run on the worker threads beside the engine's. */
int yq_batch_forces(yq_batch* batch, const double* sigma, double gamma, double* force,
                    double* torque, double* energy);

/* Autotuner: times the fused FP32 far field for a set of persistent grid sizes
 * and source-chunk policies on this batch and keeps the fastest (reported in the
 * two outputs, either may be NULL).  Changes the per-configuration chunking. */
int yq_batch_autotune(yq_batch* batch, int32_t* persist_blocks, int32_t* far_want);

/* enable != 0: replay the captured iteration graph (default); 0: launch eagerly. */
int yq_batch_use_graphs(yq_batch* batch, int32_t enable);

/* Timers of the fused engine's far-field launches: the direct members' fused
 * far field (the FP32 kernel of the inner iterations, the FP64 kernel of the
 * refinement residuals) and the FMM forest's leaf pass (direct interactions of
 * neighbouring leaves and the local expansions; inner order in FP32 pairs,
 * residual order in FP64).  enable != 0: every such launch (the leaf pass: its
 * launches of one operator application together) is bracketed by hipEvents on
 * the batch's stream (the captured iteration is then replayed as one graph per
 * part, with the events recorded between their launches) and the launches count
 * the source-target pairs they evaluate (masked configurations excluded; the leaf
 * pass counts the pairs of every leaf with the leaves of its direct-interaction
 * list).  yq_batch_profile_read (direct far field) and yq_batch_profile_read_leaf
 * (leaf pass) synchronise and return, for YQ_MIXED or YQ_FP64, the number of
 * timed launches, their summed duration (ms) and the summed pairs; the leaf pass
 * also the algorithmic bytes of its trees that read a near-field cache
 * (coefficients once, each target's output read and written, each list entry's
 * source densities once; bytes may be NULL); reset != 0 clears them.  The leaf
 * pass's timer does not include the local expansions' evaluation at the nodes,
 * which runs before it.  Configurations of the FMM lane are not counted.  All
 * synchronous. */
int yq_batch_profile_enable(yq_batch* batch, int32_t enable);
int yq_batch_profile_read(yq_batch* batch, int32_t precision, int64_t* launches,
                          double* total_ms, double* pairs, int32_t reset);
int yq_batch_profile_read_leaf(yq_batch* batch, int32_t precision, int64_t* launches,
                               double* total_ms, double* pairs, double* bytes, int32_t reset);

/* ---- Serving -----------------------------------------------------------------------------
 * A continuous-batching solve server on one GPU.  Requests (one particle
 * configuration each) are queued by yq_server_submit and advanced by
 * yq_server_step, one scheduling tick per call:
 *   admission (arrival order, first fit) while a free range of the node arena
 *   (node_capacity nodes) and the device-memory budget (mem_budget_bytes, by a
 *   per-request estimate) allow, at most max_slots requests at once; then an
 *   FP64 residual for requests between refinement steps, one Arnoldi step of the
 *   fused batch iteration for every request inside a GMRES cycle, cycle ends,
 *   and finished requests (forces with gamma = 1, results copied to the host,
 *   resources released).
 * Work of requests in flight shares every fused launch; a request's arithmetic
 * depends only on its own size, so its result is the same alone or in a mix.
 * FMM lane: requests of at least a threshold node count (params->far_mode
 * YQ_FAR_FMM: every request; YQ_FAR_AUTO: 20000 nodes; YQ_FAR_DIRECT: none;
 * yq_server_set_fmm overrides) are admitted by the memory budget alone (not the
 * arena) and solved each as a standalone problem with the FMM far field
 * (section 5's fast multipole evaluation; mixed precision with FP64 FMM
 * residuals and forces) by worker threads, each with its own stream of
 * default priority, concurrently with the fused iterations; results likewise
 * depend only on the request.  Latency = completion time - submit time
 * (steady clock).  The server owns a HIP stream of default priority; calls
 * other than the lane's solves are synchronous. */
typedef struct yq_server yq_server;

int yq_server_create(const yq_params* params, int64_t node_capacity, int32_t max_slots,
                     double mem_budget_bytes, yq_server** out);
void yq_server_destroy(yq_server* server);
const char* yq_server_last_error(const yq_server* server);

/* FMM lane threshold (nodes, >= 0) and worker count (1..8); only before the
 * first submit (YQ_ESTATE after). */
int yq_server_set_fmm(yq_server* server, int64_t min_nodes, int32_t workers);

/* Queues a request (host arrays copied; label as yq_boundary_label).  ticket:
 * host out.  YQ_EADMIT (ticket still set, state failed) if the request can
 * never fit the node capacity or the memory budget. */
int yq_server_submit(yq_server* server, int32_t n, const double* center_xy, const double* angle,
                     const double* semi_axes, double kappa, int32_t label_kind, double param0,
                     double param1, int64_t* ticket);

/* One tick.  completed / running / queued: host out (may be NULL). */
int yq_server_step(yq_server* server, int32_t* completed, int32_t* running, int32_t* queued);

/* state: 0 queued, 1 running, 2 done, 3 failed.  For done/failed requests the
 * host outputs (each may be NULL) receive sigma [N], force [2n], torque [n],
 * energy, info and the latency in seconds. */
int yq_server_result(yq_server* server, int64_t ticket, int32_t* state, int64_t* N, int32_t* n,
                     double* sigma, double* force, double* torque, double* energy,
                     yq_solve_info* info, double* latency_s);

/* Forgets a finished request's stored results. */
int yq_server_release(yq_server* server, int64_t ticket);

/* Removes a queued or running request (it ends in state failed, "cancelled"; a
 * running FMM-lane request when its solve returns, at a later yq_server_step). */
int yq_server_cancel(yq_server* server, int64_t ticket);

/* Per-phase GPU timers: every launch of a timed phase is bracketed by
 * hipEvents on the problem's stream.  Phases: 0 FP64 far field, 1 FP32 far
 * field, 2 finish (chunk sum + near correction), 3 gradient far field, 4 QBX
 * build, 5 Krylov vector kernels, 6 the fused FP64 far field + gradient of
 * yq_solve_forces, 7 repulsion (and Euler update) of yq_repulsion and yq_step.
 * phase_mask: bit p times phase p; 0 times nothing (the
 * default); -1 times every phase.  yq_profile_read synchronises the stream and
 * returns the number of timed launches and their summed duration (ms) of one
 * phase; reset != 0 clears that phase. */
int yq_profile_enable(yq_problem* prob, int32_t phase_mask);
int yq_profile_read(yq_problem* prob, int32_t phase, int64_t* launches, double* total_ms,
                    int32_t reset);

/* The FMM's adaptive quadtree (far_mode FMM or AUTO above its threshold): a box is
 * split while it holds more than fmm_leaf_max nodes, so leaves sit on different
 * levels.  Host outputs (each may be NULL): depth (deepest level), leaves, the
 * largest leaf's node count, the source-target pairs of one direct (P2P) pass
 * and the box pairs of one M2L pass.  YQ_ESTATE when the problem has no FMM. */
int yq_fmm_stats(const yq_problem* prob, int32_t* depth, int32_t* leaves, int32_t* max_leaf,
                 double* p2p_pairs, double* m2l_pairs);

/* Device special functions, for testing: kind 0 -> K0(z), 1 -> K1(z),
 * 2 -> K_order(z), 3 -> I_order(z); precision YQ_FP64 or YQ_MIXED (FP32).
 * dev z [n] -> dev out [n].  Synchronous. */
int yq_bessel(int32_t kind, int32_t order, int32_t precision, int64_t n, const double* z, double* out);

#ifdef __cplusplus
}
#endif
#endif /* YQBX_H */
