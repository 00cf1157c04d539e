/*
 * lddmm.h - C ABI of the MI355X (gfx950) library for geodesic-shooting
 * PDE-constrained LDDMM with inexact Gauss-Newton-Krylov optimisation
 * (M. Hernandez, arXiv 1807.04638).
 *
 * Problem (Section 3): minimise over the initial velocity v0
 *     E(v0) = <L v0, v0>_{L2} + sigma^-2 || J_1 - I_1 ||^2_{L2}
 * subject to the EPDiff equation  d_t v + ad^dagger_v v = 0,  v(0) = v0
 * (Section 2.2) and the state equation  d_t J + grad J . v = 0,  J(0) = I_0
 * (Section 2.3), with L = (Id - alpha Laplacian)^s and K = L^-1 (Section 2.1).
 *
 * Discretisation (the paper gives none): periodic box [0, 2 pi)^3 with
 * h_d = 2 pi / N_d; L and K applied spectrally with integer wavenumbers;
 * second-order central differences; ad*_v mu in conservative form; Heun (RK2)
 * time stepping of the momentum mu = L v with dt = 1/nt; semi-Lagrangian
 * transport of the inverse-map displacement u with periodic trilinear
 * interpolation and J_1 = I_0 o (id + u_1).
 *
 * Layouts.  A scalar field is N0*N1*N2 contiguous elements, C order (x2 fastest).
 * A vector field is three such scalar fields back to back (SoA [3][N0][N1][N2]).
 * The element type is float (LDDMM_F32) or double (LDDMM_F64) as chosen at
 * creation; inner products, energies and CG scalars are always accumulated in
 * double.  Every field pointer is a DEVICE pointer on the device that was
 * current when the context was created; the caller owns it and the library
 * keeps no pointer past the call.  Pointers may not alias one another unless a
 * function says so.
 *
 * Streams.  All device work of a context is ordered on the hipStream_t given
 * at creation (NULL = the legacy default stream).  Functions that return host
 * scalars (energies, reports) synchronise that stream before returning; the
 * others only enqueue work.  A context is not thread-safe: use one per host
 * thread.
 *
 * Errors.  Every function returns LDDMM_OK (0) or a negative LDDMM_E* code;
 * outputs are unspecified on error.  lddmm_last_error() gives a message.
 */
#ifndef LDDMM_H
#define LDDMM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LDDMM_OK 0
#define LDDMM_EINVAL (-1)       /* bad argument (NULL pointer, size, dtype)            */
#define LDDMM_EUNSUPPORTED (-2) /* grid size: prime factor > 7, odd N2, N_d < 4, 3N >= 2^31 */
#define LDDMM_ENOMEM (-3)       /* device allocation failed                            */
#define LDDMM_EHIP (-4)         /* a HIP runtime call failed                           */
#define LDDMM_ENONFINITE (-5)   /* an input field holds NaN or Inf                     */
#define LDDMM_ESTATE (-6)       /* call order (e.g. hessvec before any linearization)  */
#define LDDMM_ELINESEARCH (-7)  /* Armijo line search found no decrease               */

#define LDDMM_F32 0
#define LDDMM_F64 1

#define LDDMM_OP_K 0 /* K = (Id - alpha Laplacian)^-s */
#define LDDMM_OP_L 1 /* L = (Id - alpha Laplacian)^s  */

typedef struct lddmm_ctx lddmm_ctx;

/* Model and grid.  n[d] = N_d (each a product of 2, 3, 5, 7; N2 even; N_d >= 4;
 * 3 N0 N1 N2 < 2^31), nt >= 1 Heun steps on [0, 1], s >= 1 and alpha > 0 of L,
 * sigma2 > 0 the image-noise variance of the data term (Section 3 energy).
 *
 * Trajectory memory (the paper's Section 5 names the memory load of the
 * stored geodesic as the method's main drawback):
 *   checkpoint_every > 0   keep the momentum every c steps; each sweep
 *                          recomputes one c-step segment at a time
 *                          (ceil(nt/c) + 4c + 1 vector fields, 2 extra K
 *                          applications per step and sweep)
 *   checkpoint_every < 0   keep mu_0 only and replay (7 vector fields,
 *                          O(nt^2) steps in the adjoint sweep)
 *   checkpoint_every == 0  store every step (4 nt + 2 vector fields), unless
 *                          mem_budget_bytes > 0 and the whole context would not
 *                          fit it: then the largest c that fits, else replay.
 * Every policy gives bitwise the same gradients and Hessian-vector products. */
typedef struct {
  int32_t n[3];
  int32_t nt;
  int32_t s;
  int32_t dtype;
  double alpha;
  double sigma2;
  int64_t mem_budget_bytes;
  int32_t checkpoint_every;
  int32_t reserved;
} lddmm_params;

/* Optimisation methods of lddmm_gn_solve (lddmm_solve_opts.method); the three
 * rows of the paper's comparison that use this hot path (Table 1). */
enum {
  LDDMM_GN_V = 0,  /* inexact Gauss-Newton-Krylov, CG in V (Section 3)             */
  LDDMM_GN_L2 = 1, /* Gauss-Newton with the L2 gradient L g and Hessian L H, PCG
                      with preconditioner K, L2 norms in every stop (Section 3)   */
  LDDMM_GD_V = 2,  /* gradient descent in V, v0 <- v0 - tau g (Section 2.2); the
                      Armijo search starts at tau = 1/2                            */
  LDDMM_NEWTON_V = 3 /* inexact Newton-Krylov, CG in V on the full Newton Hessian
                      (lddmm_hessvec_newton); CG meeting non-positive curvature on
                      its first direction returns -g                             */
};

/* Optimisation settings (Section 3 update and PCG system).  Zero fields take the
 * defaults in brackets.  "||g||" is the norm of the method's space: ||g||_V, or
 * ||L g||_L2 for LDDMM_GN_L2. */
typedef struct {
  int32_t gn_iters;     /* outer iterations [10; 50 for LDDMM_GD_V]               */
  int32_t cg_iters;     /* CG iterations per outer iteration [20]                 */
  int32_t max_halvings; /* Armijo step halvings [10]                              */
  int32_t method;       /* LDDMM_GN_V, LDDMM_GN_L2, LDDMM_GD_V, LDDMM_NEWTON_V [GN_V] */
  double c1;            /* Armijo constant [1e-4]                                 */
  double gtol;          /* stop when ||g|| / ||g_0|| <= gtol [1e-3]               */
  double eta_max;       /* forcing term eta = min(eta_max, sqrt(||g||/||g_0||)) [0.5] */
} lddmm_solve_opts;

/* One record per outer iteration, taken at the iterate before its update. */
typedef struct {
  double E, E_reg, E_data; /* energy and its two terms                          */
  double mse_rel;          /* 100 ||J_1 - I_1||^2 / ||I_0 - I_1||^2 (percent)   */
  double g_norm;           /* ||g|| in the method's space                       */
  double g_inf_rel;        /* ||g||_inf / ||g_0||_inf (the method's gradient)   */
  double eta;              /* CG forcing term                                   */
  double tau;              /* accepted Armijo step (0 = line search failed)     */
  int32_t cg_iters;        /* CG iterations (= Hessian-vector products)         */
  int32_t ls_trials;       /* energies evaluated by the line search             */
} lddmm_iter_log;

typedef struct {
  int32_t iters;       /* outer iterations performed                              */
  int32_t cg_total;    /* sum of CG iterations                                    */
  int32_t hessvecs;    /* Hessian-vector products                                 */
  int32_t gradients;   /* gradients (each = shoot with store + backward sweep)    */
  int32_t shoots;      /* line-search trials; each is a linearization (trajectory
                          store, residual, energy) and an accepted trial is reused
                          as the next iteration's linearization                    */
  int32_t stop_reason; /* 0 iteration cap, 1 gradient tolerance, 2 line search    */
  double E_first, E_final;
  double mse_rel_final;
  double g_rel_final;  /* ||g|| / ||g_0|| at the last linearization                */
} lddmm_solve_report;

/* Create a context: validates params, allocates the workspace and the trajectory
 * store (4 nt + 2 vector fields) on the current device, builds FFT tables.
 * hip_stream is a hipStream_t (may be NULL). */
int lddmm_create(const lddmm_params* params, void* hip_stream, lddmm_ctx** out);
int lddmm_destroy(lddmm_ctx* ctx);

/* Copy the template I_0 and target I_1 (device scalar fields) into the context.
 * Invalidates any linearization.  LDDMM_ENONFINITE if either holds NaN/Inf. */
int lddmm_set_images(lddmm_ctx* ctx, const void* I0, const void* I1);

/* Spectral operator (Section 2.1): out = K in or L in for a field of ncomp
 * components (1 or 3).  in == out is allowed. */
int lddmm_apply_operator(lddmm_ctx* ctx, int op, int ncomp, const void* in, void* out);

/* FP64 L2 inner product h0 h1 h2 sum_i sum_c a_c[i] b_c[i] over ncomp components. */
int lddmm_dot(lddmm_ctx* ctx, int ncomp, const void* a, const void* b, double* out);

/* Forward geodesic shooting (Section 3 constraints): EPDiff from v0 (vector
 * field), transport of the displacement and J_1 = I_0 o (id + u_1).  Any of
 * J1 (scalar), u1, v1 (vector) and energy may be NULL.  Does not store the
 * trajectory and does not change the current linearization.  If energy is not
 * NULL, *energy = E(v0) (needs images; synchronises). */
int lddmm_shoot(lddmm_ctx* ctx, const void* v0, void* J1, void* u1, void* v1, double* energy);

/* Shoot with trajectory store and form the final conditions at v0: residual
 * J_1 - I_1, energy, G = grad_h J_1.  Becomes the current linearization (its
 * counter "lin.epoch" increases).  J1 (scalar field) and energy may be NULL. */
int lddmm_linearize(lddmm_ctx* ctx, const void* v0, void* J1, double* energy);

/* V-gradient g = 2 v0 + w_0 (Section 3: gradient at t = 1, lambda(1) grad J_1,
 * carried to t = 0 by the reduced adjoint Jacobi equations of Section 2.2).
 * Linearizes at v0 first.  energy may be NULL. */
int lddmm_gradient(lddmm_ctx* ctx, const void* v0, void* g, double* energy);

/* Gauss-Newton Hessian-vector product in V (Section 3: incremental EPDiff and
 * incremental state forward, incremental adjoint Jacobi backward):
 * hv = 2 dv + w_0 with w from the final condition -(2/sigma2) dm_1 grad J_1,
 * dm_1 = -grad J_1 . X_1.  v0 == NULL reuses the current linearization
 * (LDDMM_ESTATE if there is none); otherwise linearizes at v0 first.
 * Enqueue-only when v0 == NULL. */
int lddmm_hessvec(lddmm_ctx* ctx, const void* v0, const void* dv, void* hv);

/* Full Newton Hessian-vector product in V (Section 3 incremental adjoint Jacobi
 * equations with nothing dropped): as lddmm_hessvec, plus the terms of the
 * first-order adjoint (U, w) of the gradient in the incremental sweep
 * (ad^dagger_dv U, -ad_dv w, ad^dagger_w dv) and lambda(1) grad(delta m(1)) in its
 * final condition.  Not symmetric on the grid beyond discretisation error and
 * indefinite far from a minimum.  The first call allocates 8 nt vector fields of
 * stage history (LDDMM_ENOMEM if they do not fit); each new linearization costs one
 * extra adjoint sweep to record (U, w).  v0 == NULL reuses the current
 * linearization (LDDMM_ESTATE if there is none). */
int lddmm_hessvec_newton(lddmm_ctx* ctx, const void* v0, const void* dv, void* hv);

/* Backward of J_1 w.r.t. v0 at the current linearization for a plain-array
 * cotangent gbar = dl/dJ_1 (scalar field): the adjoint Jacobi sweep of Section 2.2
 * (the one behind the gradient of Section 3) run as a vector-Jacobian product,
 * with the data term's final condition replaced by U^(1) = -gbar grad J_1;
 * gbar_v0 = L w_0 (the quadrature weights of the pairing cancel).  Layouts as
 * lddmm_gradient; LDDMM_ESTATE without a linearization. */
int lddmm_vjp(lddmm_ctx* ctx, const void* gbar_J1, void* gbar_v0);

/* CG in V for H x = -g at the current linearization (Section 2.3 reduced
 * system with preconditioner K; Section 3 "CG on V"): stops when
 * ||r||_V <= eta ||g||_V or after maxit iterations; *iters = iterations done. */
int lddmm_cg_solve(lddmm_ctx* ctx, const void* g, void* x, double eta, int maxit, int* iters);

/* Solve from v0_inout (updated in place) with opts->method: inexact
 * Gauss-Newton-Krylov in V (default) or with PCG in L2, gradient descent in V, or
 * inexact Newton-Krylov in V.
 * opts may be NULL (defaults); report and log (capacity log_cap) may be NULL.
 * LDDMM_EINVAL for an unknown method. */
int lddmm_gn_solve(lddmm_ctx* ctx, void* v0_inout, const lddmm_solve_opts* opts,
                   lddmm_solve_report* report, lddmm_iter_log* log, int log_cap);

/* PDE-LDDMM, the comparison method of Section 2.3 (energy eq. LS-LDDMM with the
 * state eq. FirstOrder1, adjoint eq. FirstOrder2, gradient eq. FirstOrder3 and the
 * second-order system SecondOrder1-3 with the Gauss-Newton drops of its last
 * paragraph), on the context's grid, nt, L, sigma2 and images.
 * Velocity fields over time: stationary != 0, one vector field v (v_t = v);
 * stationary == 0, nt + 1 vector fields v_0..v_nt at t_n = n / nt, stacked
 * ([nt+1][3][N0][N1][N2]).  Gradients and Hessian products have the same layout.
 * Discretisation: the image transported by the SL step of the main method
 * (m_{n+1} = m_n o X_n); the adjoint lambda (continuity equation) along forward
 * characteristics with a trapezoidal divergence factor exp(dt/2 (div v_n(x) +
 * div v_{n+1}(Y)))); the incremental state with a trapezoidal source; products
 * over time with trapezoid weights.  Optimise-then-discretise: gradient and
 * Hessian agree with the discrete energy to discretisation error.
 * The first call allocates 8 (nt + 1) vector and 2 nt + 8 scalar fields.
 *
 * E = int <L v_t, v_t> dt + sigma2^-1 ||m(1) - I_1||^2; m1 (scalar, may be NULL)
 * = m(1).  Becomes the current PDE linearization. */
int lddmm_pde_energy(lddmm_ctx* ctx, int stationary, const void* v, void* m1, double* energy);
/* L2 gradient 2 L v_t + lambda(t) grad m(t) (stationary: 2 L v + its time
 * integral of lambda grad m); linearizes at v. */
int lddmm_pde_gradient(lddmm_ctx* ctx, int stationary, const void* v, void* g, double* energy);
/* Gauss-Newton Hessian in L2: 2 L dv_t + dlambda(t) grad m(t), dlambda the adjoint
 * of -(2/sigma2) dm(1); v == NULL reuses the current PDE linearization
 * (LDDMM_ESTATE if there is none for this parameterisation). */
int lddmm_pde_hessvec(lddmm_ctx* ctx, int stationary, const void* v, const void* dv, void* hv);
/* Gauss-Newton-Krylov from v_inout (updated in place): PCG in the space-time L2
 * product with preconditioner K per time point, forcing eta = min(eta_max,
 * sqrt(||g|| / ||g_0||)), Armijo backtracking v <- v + tau p; opts->method is
 * ignored.  Report and log as for lddmm_gn_solve (L2 norms). */
int lddmm_pde_gn_solve(lddmm_ctx* ctx, int stationary, void* v_inout, const lddmm_solve_opts* opts,
                       lddmm_solve_report* report, lddmm_iter_log* log, int log_cap);
/* Inverse-map displacement u1 (vector field, caller-owned) of the PDE-LDDMM flow
 * of v: u_0 = 0, u_{n+1}(x) = u_n(X_n) + X_n - x with the Heun foot X_n of the
 * state equation (Section 2.3), so that the warped template is I_0 o (id + u1);
 * det(I + D u1) (lddmm_jacobian_det) gives the Jacobian extrema reported for
 * every method in Table 1.  Needs no images; does not change the PDE
 * linearization.  LDDMM_EINVAL for NULL pointers, LDDMM_ENONFINITE for a
 * non-finite v. */
int lddmm_pde_displacement(lddmm_ctx* ctx, int stationary, const void* v, void* u1);

/* Jacobian determinant det(I + D_h u) (central differences) of a displacement u
 * (vector field) into det (scalar field), plus its extrema (either may be NULL;
 * synchronises when requested). */
int lddmm_jacobian_det(lddmm_ctx* ctx, const void* u, void* det, double* det_min, double* det_max);

/* Per-kernel timing with HIP events recorded on the context stream.  enable=1
 * clears and starts, 0 stops.  lddmm_profile_read fills up to cap entries of
 * names (each a static string), launch counts and total milliseconds and
 * returns the number of kernel kinds (synchronises). */
int lddmm_profile_enable(lddmm_ctx* ctx, int enable);
int lddmm_profile_read(lddmm_ctx* ctx, const char** names, int64_t* counts, double* total_ms, int cap);

/* Launch-shape options of the context's kernels (tuning; results do not change
 * beyond rounding).  Keys:
 *   "fft.plane_threads"   256 | 512 | 1024  threads of an (x1, x2) plane workgroup
 *   "fft.pencil_threads"  256 | 512         threads of a pencil workgroup
 *   "fft.pencil_tb"       1..128            contiguous pencils per workgroup (with half planes:
 *                                           pencil_tb / 2 pairs of half-plane spectra, the
 *                                           pencils of k1 and k1 + N1/2 of each pair)
 *   "fft.rows_rb"         1..64             rows per workgroup (split path)
 *   "fft.force_split"     0 | 1             split transform path even where a plane fits
 *   "fft.static"          0 | 1             compile-time kernels for power-of-two lengths
 *   "fft.plane_grid"      0..65535          0: one (x1, x2) plane per workgroup; G > 0: G
 *                                           workgroups walk the planes (g, g + G, ...), loading
 *                                           the next plane while transforming the current one
 *                                           (compile-time plane kernels; not with 1024 threads
 *                                           in FP64)
 *   "fft.plane_walk"      read-only: workgroups of the plane walk in use (0: none)
 *   "fft.plane_halves"    0 | 1             1: the even and the odd x1 rows of a plane are two
 *                                           workgroups' units (half the LDS, twice the units,
 *                                           so the units spread evenly over the compute
 *                                           units), each transformed along x1 at half length;
 *                                           the x0 pencil pass merges the two halves (the first
 *                                           radix-2 step of the x1 transform) before its
 *                                           transform and splits them after.  Needs an even N1,
 *                                           compile-time kernels for the grid, no plane walk
 *                                           and an even fft.pencil_tb of 8 to 32; otherwise
 *                                           whole planes are used.  Default 1
 *   "fft.plane_halves_used" read-only: 1 if half planes are in use
 *   "fft.fused"           read-only: 1 if the fused plane path is in use
 *   "fft.static_kernels"  read-only: number of passes using compile-time kernels
 *   "traj.policy"         read-only: 0 store-all, 1 checkpoint, 2 recompute
 *   "traj.every"          read-only: checkpoint interval c
 *   "traj.bytes"          read-only: device bytes of the trajectory storage
 *   "lin.epoch"           read-only: number of linearizations made so far
 *   "exec.graph"          0 | 1             replay Hessian-vector products from a captured
 *                                           hipGraph (store-all trajectories; needs a
 *                                           non-default stream)
 *   "exec.branch_k"       0 | 1             in captured graphs, record the transform of a
 *                                           vector field as three independent per-component
 *                                           chains (their passes may overlap); bitwise the
 *                                           same results.  Chosen by lddmm_autotune
 *   "stencil.rowvec"      0, 1, 2, 3, 4     voxels per lane of the row-vectorised stencil
 *                                           kernels (0: one voxel per thread); nonzero
 *                                           values need 32 <= N2 / value <= 64.  Default:
 *                                           the smallest valid width in FP64, the widest
 *                                           in FP32, 0 where none is valid; same
 *                                           operators, summed in another order
 *   "stencil.pair_rows"   0 | 1             with N2 / rowvec = 32 and N1 even a wave holds two
 *                                           x1 rows; 1: the row each half needs from the other
 *                                           comes by a lane swap instead of a load.  Default 1
 * LDDMM_EINVAL for an unknown key or a value out of range, LDDMM_EUNSUPPORTED if
 * the tiles would not fit the LDS of a workgroup (the previous setting stays). */
int lddmm_set_option(lddmm_ctx* ctx, const char* key, int64_t value);
int lddmm_get_option(lddmm_ctx* ctx, const char* key, int64_t* value);

/* Autotuner: time the transform variants (plane workgroup size, pencil tile,
 * compile-time vs generic kernels, plane walk over one workgroup per compute
 * unit or two planes per workgroup), the stencil widths ("stencil.rowvec",
 * "stencil.pair_rows", timed on the tangent stage) and, on a non-default stream,
 * "exec.branch_k" (timed as graph replays) on this context's grid with HIP events
 * (reps repetitions each; a transform shape is timed as a K application followed
 * by a tangent stage, the way the sweeps use it) and keep the fastest; the shape
 * in place when the call starts is kept unless another is more than 3 % faster
 * (0.5 % for "exec.branch_k", whose two graphs of at least 8 K applications are
 * replayed in turn three times and compared by their fastest replay), so
 * repeated calls settle on the same shape.  *tried = variants timed,
 * *ms_per_apply = one K application of a vector field with the chosen shape
 * (either may be NULL).  Synchronises. */
int lddmm_autotune(lddmm_ctx* ctx, int reps, int* tried, double* ms_per_apply);

/* Wait for all work of the context's stream. */
int lddmm_sync(lddmm_ctx* ctx);

/* Bytes of device memory held by the context. */
int lddmm_memory_bytes(lddmm_ctx* ctx, int64_t* bytes);

/* Batches of independent registrations (e.g. many template/target pairs of
 * different sizes).  Each pair gets its own context on its own stream, created
 * by the library (non-blocking, default priority), with graph replay of the
 * Hessian-vector product enabled.  The contexts are used with the functions
 * above (lddmm_batch_get); their calls are ordered on their own streams, so a
 * caller working on another stream synchronises before handing buffers over.
 * lddmm_batch_gn_solve / _hessvec take a mode (argument `concurrent`):
 *   LDDMM_BATCH_SEQUENTIAL  one pair after the other;
 *   LDDMM_BATCH_THREADS     one host thread per pair, each on its pair's stream;
 *   LDDMM_BATCH_LOCKSTEP    every phase of the solve (gradient, each CG
 *                           iteration, <g, p>, each line-search trial) is enqueued
 *                           for all pairs that need it before one wait (the
 *                           launches by one persistent host worker per pair); the
 *                           CG scalars stay on the device, and a CG iteration or a
 *                           Hessian-vector product of several pairs is one graph
 *                           spanning their streams (store-all trajectories).  All
 *                           pairs must share a dtype (else: threads).
 * Every mode gives bitwise the results of lddmm_gn_solve / lddmm_hessvec on each
 * context alone.  They return after every pair has finished and its results are
 * written (each pair's stream is synchronised); the first failing status is
 * returned.  Their pointer arrays hold one entry per pair; a NULL entry gives
 * LDDMM_EINVAL before any work. */
#define LDDMM_BATCH_SEQUENTIAL 0
#define LDDMM_BATCH_THREADS 1
#define LDDMM_BATCH_LOCKSTEP 2
typedef struct lddmm_batch lddmm_batch;
int lddmm_batch_create(const lddmm_params* per_pair, int npairs, lddmm_batch** out);
int lddmm_batch_destroy(lddmm_batch* batch);
int lddmm_batch_get(lddmm_batch* batch, int i, lddmm_ctx** ctx);
int lddmm_batch_sync(lddmm_batch* batch);
/* v0_inout[i]: device vector field of pair i (solved in place); reports may be NULL. */
int lddmm_batch_gn_solve(lddmm_batch* batch, void* const* v0_inout, const lddmm_solve_opts* opts,
                         lddmm_solve_report* reports, int concurrent);
/* reps Hessian-vector products per pair at each pair's current linearization. */
int lddmm_batch_hessvec(lddmm_batch* batch, void* const* dv, void* const* hv, int reps, int concurrent);
/* lddmm_autotune on every context. */
int lddmm_batch_autotune(lddmm_batch* batch, int reps);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * serving loops, harnesses that forbid hipMalloc): lddmm_apply_operator without
 * a context.  out = K in or L in (op) for a field of ncomp (1 or 3) components
 * of dtype on the grid n[3] (same limits as lddmm_params.n), with
 * L = (Id - alpha Laplacian)^s; in == out is allowed; in and out are device
 * pointers on the current device, ordered on hip_stream (NULL = the legacy
 * default stream).  Same kernels and launch shapes as an untuned context.
 * Workspace: nothing is allocated.  The transform tables and the spectrum live in
 * one static device array of LDDMM_NOALLOC_WORKSPACE_BYTES per device, held from
 * the first call on that device until the process ends; the tables take a few
 * KB and the spectrum ncomp * N0 * N1 * (N2/2 + 1) complex values of dtype (e.g.
 * 128^3 vector fields in FP64, 160^3 in FP32).  Larger requests return
 * LDDMM_EUNSUPPORTED with the bytes needed in lddmm_last_error(NULL).
 * The first call for a grid and dtype on a device (and the first after another
 * grid or dtype was used there) copies the tables into the array, synchronising
 * hip_stream before and after; it returns LDDMM_ESTATE while hip_stream is being
 * captured.  Later calls with the same grid and dtype only enqueue kernels.
 * Every call on a device shares that device's array: calls that overlap in time
 * on one device (other streams or host threads without ordering between them)
 * race and give undefined results.  Errors of this call: lddmm_last_error(NULL)
 * gives the calling thread's last message. */
#define LDDMM_NOALLOC_WORKSPACE_BYTES (64 * 1024 * 1024)
int lddmm_apply_operator_noalloc(const int32_t n[3], int dtype, double alpha, int s, int op, int ncomp,
                                 const void* in, void* out, void* hip_stream);

const char* lddmm_strerror(int status);
/* Last error message of ctx; with ctx == NULL, of the calling thread's last failed
 * lddmm_apply_operator_noalloc ("null context" if there was none). */
const char* lddmm_last_error(lddmm_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* LDDMM_H */
