/*
 * dgsw.h -- C ABI of libdgsw, the modal Discontinuous Galerkin right-hand
 * side of the shallow-water equations on a latitude-longitude element mesh
 * of the sphere, and its explicit Runge-Kutta stage loop, for AMD Instinct
 * MI355X (gfx950).
 *
 * The method (Szenes, Discacciati, Bonaventura, Sawyer, "Domain-specific
 * implementation of high-order Discontinuous Galerkin methods in spherical
 * geometry", arXiv:2303.11767):
 *   - section 2, the conservative system d_t U + d_lambda F + d_theta G = S
 *     with U = (h, hu, hv) cos(theta), periodic in longitude, zero flux
 *     through the poles;
 *   - section 2, equation "dg_parts" (weak form), equation "rusanov"
 *     (numerical flux), equation "basis_expansion" (modal Legendre basis of
 *     full tensor degree r), equation "ode" (M dq/dt = h(q)) and the
 *     cos(theta)-weighted local mass matrix;
 *   - section 2, Table "Butcher" (explicit Runge-Kutta tableaux).
 *
 * Conventions shared by every call:
 *   - State layout q[E][3][N], E = n_lon * n_lat elements, element
 *     e = j * n_lon + i (j = 0 is the southernmost row, i = 0 starts at
 *     longitude 0), variables (h, hu, hv), N = (r+1)^2 modes with mode
 *     m = b * (r+1) + a (a: longitude degree, b: latitude degree) of the
 *     orthonormal basis phi_m(xi, eta) = P~_a(xi) P~_b(eta),
 *     P~_a = sqrt((2a+1)/2) P_a.
 *   - Every state pointer (q, dqdt, work, fhat) is caller-owned DEVICE
 *     memory of the context's dtype, contiguous, 16-byte aligned.  The
 *     library never allocates or frees caller state.
 *   - Work is enqueued on the caller's hipStream_t (passed as void*; NULL is
 *     the null stream).  Calls return as soon as the work is enqueued, except
 *     dg_mass, which synchronises the stream.
 *   - Every function returns DG_OK (0) or a negative DG_E* code; nothing is
 *     thrown across the ABI.  dg_last_error() gives a message for the last
 *     failure on the calling thread.
 *   - A context is not used by two host threads at once.
 */
#ifndef DGSW_H
#define DGSW_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DG_ABI_VERSION 1

typedef struct dg_ctx dg_ctx;

enum { DG_F64 = 0, DG_F32 = 1 };

/* Latitude factor of the pressure-metric source -g h^2 sin(theta) / (2R).
 * BALANCED replaces sin(theta) at the quadrature nodes by the degree-r
 * polynomial that makes the discrete integration by parts of the pressure
 * exact (a lake at rest has a zero right-hand side); POINTWISE keeps
 * sin(theta). */
enum { DG_METRIC_BALANCED = 0, DG_METRIC_POINTWISE = 1 };

/* Rusanov stabilisation alpha (equation "rusanov"): LOCAL takes, at every
 * edge quadrature point, the larger of |u_n| + sqrt(g h) over the two
 * sides; GLOBAL uses the fixed speed dg_mesh_desc.alpha [m/s]. */
enum { DG_ALPHA_LOCAL = 0, DG_ALPHA_GLOBAL = 1 };

/* Runge-Kutta schemes of Table "Butcher": RK1 (forward Euler), RK2 (Heun),
 * RK3 (the third tableau, SSP), each applied in Shu-Osher form, and the
 * classical four-stage RK4 (the fourth tableau, the scheme of the spherical
 * runs of Sec. 4.3-4.4; not SSP). */
enum { DG_SSP_RK1 = 1, DG_SSP_RK2 = 2, DG_SSP_RK3 = 3, DG_RK4 = 4 };

enum {
  DG_OK = 0,
  DG_EINVAL = -1,       /* bad argument: null, misaligned, out of range     */
  DG_EDTYPE = -2,       /* dtype not DG_F64 / DG_F32                          */
  DG_ENOMEM = -3,       /* device allocation of the context tables failed     */
  DG_EHIP = -4,         /* a HIP runtime call or kernel launch failed         */
  DG_ENONFINITE = -5,   /* dg_mass found a NaN or Inf in the state            */
  DG_EUNSUPPORTED = -6  /* valid but not supported (e.g. order > 7)           */
};

typedef struct {
  int32_t abi_version;  /* must be DG_ABI_VERSION                                     */
  int32_t n_lon;        /* elements in longitude (periodic), >= 1                     */
  int32_t n_lat;        /* elements in latitude, pole to pole, >= 1                   */
  int32_t order;        /* polynomial degree r in each direction, 0..7                */
  int32_t dtype;        /* DG_F64 or DG_F32: state, right-hand side and arithmetic    */
  int32_t metric;       /* DG_METRIC_*                                                 */
  int32_t alpha_mode;   /* DG_ALPHA_*                                                  */
  int32_t reserved;     /* must be 0                                                   */
  double alpha;         /* [m/s], used iff alpha_mode == DG_ALPHA_GLOBAL, >= 0         */
  double radius;        /* sphere radius R [m], > 0                                    */
  double gravity;       /* g [m/s^2], > 0                                              */
  double omega;         /* rotation rate Omega [1/s]; Coriolis f = 2 Omega sin(theta) */
  double h_ref;         /* reference depth H [m] >= 0.  When > 0 the kernels evaluate  */
                        /* h as H + (h - H) and the pressure as g (h^2 - H^2)/2, a     */
                        /* roundoff-only change under the BALANCED metric (a constant  */
                        /* pressure then contributes exactly zero).  Rejected with     */
                        /* POINTWISE.  0 disables it.                                  */
} dg_mesh_desc;

/* Build a context: host precompute in FP64 (Gauss-Legendre nodes and weights,
 * Legendre values and derivatives, per-latitude-row inverse mass matrices
 * folded with the quadrature tables, metric factors), copied to the device
 * on hip_stream.  Allocates only the context's own tables.  On success
 * *out is a new context; on failure *out is NULL. */
int dg_init_mesh(const dg_mesh_desc *desc, void *hip_stream, dg_ctx **out);

/* The planar shallow-water system of section 4.2 on the doubly periodic
 * rectangle [0, lx] x [0, ly] with nx x ny elements: F = (hu, hu u + g h^2/2,
 * hu v), G = (hv, hv u, hv v + g h^2/2), S = (0, f hv, -f hu) with constant f
 * (the f-plane), no metric terms.  Element e = j nx + i (i along x, j along
 * y), modes as on the sphere (a: x degree, b: y degree).  Every other call
 * (dg_rhs, dg_rk_step, dg_rk_stage, dg_mass, dg_set_forcing, dg_min_width,
 * graphs) works on the context as on a sphere mesh; dg_mass integrates over
 * the rectangle; the learned-correction calls reject it. */
typedef struct {
  int32_t abi_version;  /* must be DG_ABI_VERSION                                     */
  int32_t nx, ny;       /* elements along x and y (both periodic), >= 1               */
  int32_t order;        /* polynomial degree r in each direction, 0..7                */
  int32_t dtype;        /* DG_F64 or DG_F32                                           */
  int32_t alpha_mode;   /* DG_ALPHA_*                                                  */
  double alpha;         /* [m/s], used iff alpha_mode == DG_ALPHA_GLOBAL, >= 0         */
  double lx, ly;        /* domain lengths [m], > 0                                     */
  double gravity;       /* g [m/s^2], > 0                                              */
  double f;             /* Coriolis parameter [1/s], finite                            */
  double h_ref;         /* reference depth H [m] >= 0, as in dg_mesh_desc              */
} dg_plane_desc;
int dg_init_plane(const dg_plane_desc *desc, void *hip_stream, dg_ctx **out);

/* Stage-kernel layout of a context.  DG_KERNEL_LINE: r+1 lanes per element,
 * each lane one modal row / node column.  DG_KERNEL_HALF: 2(r+1) lanes per
 * element, each lane half of a row's outputs and two of the four edges (twice
 * the wavefronts, about half the instructions each).  Both compute the same
 * right-hand side up to rounding (the half layout sums the volume integral
 * in two halves).  dg_init_mesh / dg_init_plane pick one by mesh size; this
 * call overrides it (DG_EINVAL for another value). */
enum { DG_KERNEL_LINE = 0, DG_KERNEL_HALF = 1 };
int dg_set_kernel(dg_ctx *ctx, int32_t kernel);
int dg_get_kernel(const dg_ctx *ctx, int32_t *kernel);

/* Pick the faster stage-kernel layout for this context by timing: two
 * SSP-RK3 stages from q (read only) into work (dg_work_size(DG_SSP_RK3)
 * values, overwritten) with each layout, the best of three repetitions after
 * a warm-up, then dg_set_kernel with the faster one (*chosen, if not NULL,
 * receives it).  Both layouts compute the same right-hand side up to
 * rounding.  Synchronises hip_stream. */
int dg_autotune(dg_ctx *ctx, const void *q, void *work, int32_t *chosen, void *hip_stream);

/* Identical vertical layers (section 5.2.2: decoupled two-dimensional problems
 * stacked in the vertical and solved side by side).  After this call every
 * state-shaped buffer of the context (q, dqdt, q0, out, the work buffers and
 * the forcing) holds n_levels independent copies of the mesh state back to
 * back, [n_levels][E][3][N]; dg_state_size and dg_work_size scale with it;
 * dg_rhs, dg_rk_step, dg_rk_stage and dg_graph_rk advance all layers with one
 * launch per stage; dg_mass returns the integrals summed over the layers.
 * Default 1.  1 <= n_levels <= 65535 and fewer than 2^31 wavefronts over all
 * layers, else DG_EINVAL.  Contexts owned by an ensemble (dg_ens_member) and
 * the learned calls (dg_rhs_learned, dg_rk_step_learned, dg_project,
 * dg_features) accept one layer only (DG_EUNSUPPORTED). */
int dg_set_levels(dg_ctx *ctx, int32_t n_levels);
int dg_get_levels(const dg_ctx *ctx, int32_t *n_levels);

/* Release a context and its device tables.  NULL is accepted.  The caller
 * must make sure no enqueued work still uses the context. */
int dg_free(dg_ctx *ctx);

/* Number of scalars in one state buffer: n_levels * E * 3 * N. */
int dg_state_size(const dg_ctx *ctx, int64_t *n_values);

/* Number of scalars the `work` argument of dg_rk_step must hold for the
 * scheme (1 state buffer for RK1, 2 for RK2/RK3, 3 for RK4). */
int dg_work_size(const dg_ctx *ctx, int32_t scheme, int64_t *n_values);

/* Smallest element width [m] for the Courant number p c dt / H of section 2
 * (where the paper names H the minimum element diameter):
 * H = R * min(dtheta, dlambda * min cos(theta) over the latitude quadrature
 * nodes), i.e. the longitude width at the node nearest a pole.  A caller picks
 * dt = C H / (max(r,1) c_max). */
int dg_min_width(const dg_ctx *ctx, double *meters);

/* dqdt = M^-1 h(q) (+ fhat if a forcing is set): equation "ode".  q and dqdt
 * must not overlap. */
int dg_rhs(dg_ctx *ctx, const void *q, void *dqdt, void *hip_stream);

/* Advance q in place by nsteps >= 0 steps of size dt of the scheme (Shu-Osher
 * form; for RK3: q1 = q + dt L(q); q2 = 3/4 q + 1/4 (q1 + dt L(q1));
 * q <- 1/3 q + 2/3 (q2 + dt L(q2)).  RK4: q1 = q + dt/2 L(q);
 * q2 = q + dt/2 L(q1); q3 = q + dt L(q2);
 * q <- (q1 + 2 q2 + q3 - q)/3 + dt/6 L(q3), which equals the fourth tableau.)
 * work: dg_work_size scalars of scratch, not overlapping q; its contents are
 * undefined afterwards. */
int dg_rk_step(dg_ctx *ctx, void *q, void *work, double dt, int32_t scheme,
               int32_t nsteps, void *hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): dg_rk_step
 * without the `work` argument.  The scheme's stage states live in a library
 * array of DG_NOALLOC_SCRATCH_BYTES per GPU (held from library load until the
 * process ends), so the call allocates and frees nothing; results equal
 * dg_rk_step's bit for bit (same kernels, same order).  Limit: dg_work_size
 * values of the ctx dtype must fit DG_NOALLOC_SCRATCH_BYTES (32 MiB: e.g. an
 * r = 3 mesh of 180 x 90 elements in FP64 with RK4), else DG_EINVAL and
 * nothing is enqueued.  Every call on one GPU shares that GPU's array: calls
 * that overlap in time on one GPU (other streams, other host threads) race
 * and give undefined results; calls in order on one stream are safe.  Other
 * arguments and errors as dg_rk_step. */
#define DG_NOALLOC_SCRATCH_BYTES 33554432
int dg_rk_step_noalloc(dg_ctx *ctx, void *q, double dt, int32_t scheme, int32_t nsteps,
                       void *hip_stream);

/* One Runge-Kutta stage in Shu-Osher form, the building block of
 * dg_rk_step: out = c0 * q0 + c1 * (q + dt * L(q)), L(q) = M^-1 h(q)
 * (+ forcing).  q0 may be NULL iff c0 == 0; q0 may be the same buffer as
 * out (the combination is element-local) but must not partially overlap it;
 * q must not overlap out. */
int dg_rk_stage(dg_ctx *ctx, const void *q, const void *q0, void *out, double c0,
                double c1, double dt, void *hip_stream);

/* out[v] = R^2 * integral over the sphere of q_v cos(theta) dlambda dtheta,
 * v in (h, hu, hv), evaluated exactly for the discrete state with the same
 * mass matrix that is inverted (phi_00 = 1/2, so an element contributes
 * 2 (M q)_00).  Accumulated in FP64 in a fixed order (deterministic).
 * Synchronises hip_stream.  Returns DG_ENONFINITE (out still written) if any
 * state value is NaN or Inf.  out is a HOST pointer to 3 doubles. */
int dg_mass(dg_ctx *ctx, const void *q, double out[3], void *hip_stream);

/* Set (or clear with NULL) a modal forcing fhat[E][3][N] (device, ctx dtype)
 * that every right-hand side evaluation adds to M^-1 h(q); used for
 * manufactured solutions.  The pointer is borrowed: it must stay valid while
 * it is set. */
int dg_set_forcing(dg_ctx *ctx, const void *fhat);

/* ---------------------------------------------------------------------------
 * Ensembles: many independent meshes of different size and order advanced by
 * one kernel launch per Runge-Kutta stage (a batch of independent problems, the
 * generalisation of the paper's identical "vertical levels" of section 5.2 to
 * members of uneven degree and resolution).  All members share the dtype.
 * Member m's state occupies values [offsets[m], offsets[m] + state_m) of the
 * packed buffer, state_m = E_m * 3 * N_m, offsets 16-byte aligned; the gaps
 * between members are never read or written.
 * ------------------------------------------------------------------------- */
typedef struct dg_ens dg_ens;

/* members: n_members >= 1 descriptors, same dtype.  Builds one context per
 * member plus the work list of the persistent kernel.  *out NULL on failure. */
int dg_ens_init(const dg_mesh_desc *members, int32_t n_members, void *hip_stream,
                dg_ens **out);
int dg_ens_free(dg_ens *ens);
/* Values of one packed state buffer (dg_ens_rk_step's work needs twice this). */
int dg_ens_state_size(const dg_ens *ens, int64_t *n_values);
/* offsets[0..n_members] (host array of n_members + 1), in values. */
int dg_ens_offsets(const dg_ens *ens, int64_t *offsets);
/* The context of member m (owned by the ensemble; do not free), e.g. for
 * dg_min_width or dg_mass on the member's slice of the packed state. */
int dg_ens_member(dg_ens *ens, int32_t m, dg_ctx **ctx);
/* Per-member time steps dt[0..n_members) [s], copied to the device
 * (synchronously); used by every following stage or step, and by graphs
 * replayed later. */
int dg_ens_set_dt(dg_ens *ens, const double *dt);
/* dqdt = M^-1 h(q) for every member (one launch); q and dqdt must not overlap. */
int dg_ens_rhs(dg_ens *ens, const void *q, void *dqdt, void *hip_stream);
/* One stage for all members: out = c0 q0 + c1 (q + dt_m L_m(q)); same aliasing
 * rules as dg_rk_stage. */
int dg_ens_rk_stage(dg_ens *ens, const void *q, const void *q0, void *out, double c0,
                    double c1, void *hip_stream);
/* nsteps SSP-RK3 steps of every member (3 launches per step); work = 2 packed
 * states. */
int dg_ens_rk_step(dg_ens *ens, void *q, void *work, int32_t nsteps, void *hip_stream);
/* Schedule of the persistent kernels: wavefronts per workgroup (1, 2 or 4),
 * workgroups in total (each takes one contiguous, cost-balanced range of the
 * work list, sorted by order and layout; 0 = one workgroup per
 * waves_per_group items, the default), and fused = 1 for a single launch
 * covering all orders (its register budget is that of the union of the
 * orders; line-layout members only, else DG_EINVAL) or 0 for one launch per
 * distinct (order, layout) (each compiled for that pair alone). */
int dg_ens_set_schedule(dg_ens *ens, int32_t waves_per_group, int32_t groups, int32_t fused);
int dg_ens_get_schedule(const dg_ens *ens, int32_t *waves_per_group, int32_t *groups,
                        int32_t *fused);
/* Stage-kernel layout (DG_KERNEL_*, as dg_set_kernel) of every member of the
 * given order; at dg_ens_init each member takes the layout a single mesh of
 * its size and order would take.  DG_EINVAL if no member has that order, if
 * the schedule is the fused launch and kernel is not DG_KERNEL_LINE, or while
 * graphs of the ensemble are live.  The schedule's settings are kept. */
int dg_ens_set_kernel(dg_ens *ens, int32_t order, int32_t kernel);
int dg_ens_get_kernel(const dg_ens *ens, int32_t order, int32_t *kernel);
/* Pick the fastest layout per order, then the fastest schedule, by timing
 * stages on q (read only) and work (2 packed states, overwritten); with
 * cache_path, reuse or record the choice keyed by the device and the member
 * list.  Synchronises hip_stream. */
int dg_ens_autotune(dg_ens *ens, const void *q, void *work, const char *cache_path,
                    void *hip_stream);

/* ---------------------------------------------------------------------------
 * HIP graphs of whole step sequences (launch cost paid once per replay).
 * The pointers and step sizes are baked in at capture (an ensemble's dt is
 * read from its device table at run time, so dg_ens_set_dt still applies).
 * A graph pins the context or ensemble it was captured on: dg_free /
 * dg_ens_free called while graphs of it are live return DG_OK but defer the
 * release of its device tables to the last dg_graph_free, and
 * dg_ens_set_schedule / dg_ens_set_kernel / dg_ens_autotune return DG_EINVAL
 * while graphs of the ensemble are live (the schedule is baked into them).  Capturing on an
 * object whose free was deferred returns DG_EINVAL.
 * ------------------------------------------------------------------------- */
typedef struct dg_graph dg_graph;
int dg_graph_rk(dg_ctx *ctx, void *q, void *work, double dt, int32_t scheme,
                int32_t nsteps, dg_graph **out);
int dg_graph_ens(dg_ens *ens, void *q, void *work, int32_t nsteps, dg_graph **out);
int dg_graph_launch(dg_graph *graph, void *hip_stream);
int dg_graph_free(dg_graph *graph);

/* ---------------------------------------------------------------------------
 * Learned right-hand-side correction (an addition to the paper's method): a
 * network 108 -> 256 -> 256 -> 12 with GELU (erf form) after the hidden layers,
 * BF16 operands and FP32 accumulation on the matrix cores, maps the 3 x 3
 * element stencil of an r = 1 state (3 variables x 4 modes per element,
 * periodic in longitude, the pole row repeated across a pole) to a correction
 * of the element's r = 1 right-hand side.
 *
 * Parameters: one FP32 vector of dg_mlp_param_count values, in order
 * W1[108][256], b1[256], W2[256][256], b2[256], W3[256][12], b3[12]
 * (W[k][n] maps input k to output n).  Feature k of element (i, j) is
 * q[(j+dj, i+di)][v][m] with k = ((dj+1)*3 + (di+1))*12 + v*4 + m.
 * ------------------------------------------------------------------------- */
int dg_mlp_param_count(int64_t *n);
/* Device workspace bytes of dg_mlp_forward / dg_mlp_train_step for `rows`. */
int dg_mlp_workspace_size(int64_t rows, int64_t *bytes);
/* Y[rows][12] = net(X[rows][108]) (FP32 in and out, device). */
int dg_mlp_forward(const float *params, const float *X, int64_t rows, float *Y, void *workspace,
                   void *hip_stream);
/* Forward and backward pass of the mean squared error over the outputs with
 * mask[n] = 1 (mask: 12 HOST floats, each 0 or 1, read during the call, at
 * least one 1; else DG_EINVAL) against T[rows][12]; rows a multiple of 32.
 * grads (optional, device, param_count floats) receives the gradient; loss
 * (optional, device float) the mean squared error; with lr > 0 one Adam step
 * (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected with the 1-based step)
 * updates params, adam_m, adam_v in place.  Enqueues only: no
 * synchronisation, so a training loop runs without host round trips. */
int dg_mlp_train_step(float *params, float *adam_m, float *adam_v, int32_t step, float lr,
                      const float *X, const float *T, const float *mask, int64_t rows,
                      float *grads, float *loss, void *workspace, void *hip_stream);
/* Cos-weighted L2 projection q_dst = M_k^-1 int q_src phi_k cos(theta) of a
 * state onto the order-k basis of the same mesh, k = dst's order (the mass
 * matrix of section 2; longitude degrees above k are dropped, latitude
 * degrees mix per row).  For k >= the source order the state already lies
 * in the target space and is copied into it (higher modes zero).  src and
 * dst: same mesh (size, sphere or plane) and dtype, one layer; q_src and
 * q_dst: different device buffers, else DG_EINVAL. */
int dg_project(const dg_ctx *src, const dg_ctx *dst, const void *q_src, void *q_dst,
               void *hip_stream);
/* Stencil features X[E][108] (FP32, device) of an order-1 state, standardised
 * as (x - mean[k]) * istd[k] when both are given (else raw). */
int dg_features(const dg_ctx *ctx, const void *q, const float *feat_mean,
                const float *feat_istd, float *X, void *hip_stream);

/* The learned right-hand side on an order-1 context: L(q) = L1(q) + c(q), with
 * c = out_mean[j] + out_std[j] * net(standardised features) per element of
 * latitude row j.  Trust bound: an element whose correction is not finite, or
 * exceeds kappa * max|L1| over the modes of some variable, falls back to the
 * plain L1 (and is counted).  The (h, mode 00) output of the network is not
 * used: it is replaced by one constant for all elements that makes the total
 * h-mass change of the correction exactly zero. */
typedef struct {
  const float *params;      /* device, dg_mlp_param_count floats                  */
  const float *feat_mean;   /* device, 108 floats                                  */
  const float *feat_istd;   /* device, 108 floats                                  */
  const float *out_mean;    /* device, [n_lat][12]                                 */
  const float *out_std;     /* device, [n_lat][12]                                 */
  double kappa;             /* trust bound, >= 0                                   */
} dg_learned;
int dg_learned_workspace_size(const dg_ctx *ctx, int64_t *bytes);
/* dqdt = L1(q) + c(q).  fallbacks: optional device int64 incremented by the
 * number of elements that fell back. */
int dg_rhs_learned(dg_ctx *ctx, const dg_learned *net, const void *q, void *dqdt,
                   void *workspace, int64_t *fallbacks, void *hip_stream);
/* nsteps SSP-RK3 steps with the learned right-hand side (work: 2 states). */
int dg_rk_step_learned(dg_ctx *ctx, const dg_learned *net, void *q, void *work,
                       void *workspace, double dt, int32_t nsteps, int64_t *fallbacks,
                       void *hip_stream);

/* ---- Planar linear advection (section 4.1's convergence test, equation
 * "lin_adv"): du/dt + div(beta u) = 0 on the periodic rectangle [0, lx] x
 * [0, ly], nx x ny elements, the same modal DG discretisation with the upwind
 * (Rusanov) flux.  One variable: state u[E][N], e = j nx + i, m = b(r+1) + a. */
typedef struct dg_adv dg_adv;
typedef struct {
  int32_t abi_version;  /* must be DG_ABI_VERSION                                     */
  int32_t nx, ny;       /* elements along x and y, >= 1                               */
  int32_t order;        /* polynomial degree r, 0..6                                  */
  int32_t dtype;        /* DG_F64 or DG_F32                                           */
  int32_t reserved;     /* must be 0                                                   */
  double lx, ly;        /* domain lengths, > 0                                         */
  double bx, by;        /* constant velocity beta, finite                              */
} dg_adv_desc;
/* Assembles the linear operator on the host (five (r+1)^2 x (r+1)^2 matrices:
 * the element and its four neighbours) and uploads it; *out NULL on failure. */
int dg_adv_init(const dg_adv_desc *desc, void *hip_stream, dg_adv **out);
int dg_adv_free(dg_adv *adv);
int dg_adv_state_size(const dg_adv *adv, int64_t *n_values);   /* E * N */
/* dqdt = M^-1 h(q); q and dqdt must not overlap. */
int dg_adv_rhs(dg_adv *adv, const void *q, void *dqdt, void *hip_stream);
/* nsteps steps of a DG_SSP_RK* or DG_RK4 scheme, as dg_rk_step (work: 1, 2, 2
 * or 3 states). */
int dg_adv_rk_step(dg_adv *adv, void *q, void *work, double dt, int32_t scheme, int32_t nsteps,
                   void *hip_stream);

/* Message for the last failing call on this thread ("" if none). */
const char *dg_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* DGSW_H */
