/*
 * osbli.h -- C ABI of the MI355X (gfx950) library for the per-Runge-Kutta-
 * substage residual of the explicit compressible Navier-Stokes method of
 * Lusher, Jammy & Sandham (OpenSBLI, arXiv 2007.14933).
 *
 * The library computes, on one GPU, the right-hand side R(U) of the
 * conservation laws of section 2.1 (eq. ns_eqn) on a structured, possibly
 * curvilinear grid, and advances U with the low-storage Runge-Kutta scheme
 * of section 2.7:
 *   - convective terms: characteristic (Roe-averaged) reconstruction with
 *     local Lax-Friedrichs splitting, per direction (section 2.2,
 *     enumerated algorithm): WENO-Z5 (section 2.4), TENO5 or TENO6
 *     (section 2.5), the original WENO-JS5 weights (section 2.3) or the
 *     third-order WENO-Z of section 5.2;
 *   - viscous and heat-flux terms (eqs. heat_flux, stress_tensor, sutherland)
 *     with the fourth-order central scheme and one-sided closures of
 *     section 2.6, in divergence form;
 *   - metrics computed once (section 2.6, last paragraph), in FP64;
 *   - boundary conditions through three ghost nodes per side (section 3.1:
 *     periodic, extrapolation, isothermal and adiabatic no-slip walls; the
 *     Dirichlet ends of section 5.2);
 *   - time advance: the three-stage third-order low-storage scheme, its
 *     strong-stability-preserving version or the five-stage fourth-order
 *     one (section 2.7).
 *
 * Conventions (all calls):
 *   - Arrays are device pointers unless stated otherwise, FP64, owned by the
 *     caller (the library never allocates or frees device memory except in
 *     osbli_init_grid's host-side context).  The state U is laid out
 *     component-major U[c][k][j][i], c = (rho, rho u_0 .. rho u_{ndim-1},
 *     rho E), i fastest, with 3 ghost nodes on both sides of each active
 *     direction (extent n[d] + 6) and extent 1 in unused directions.
 *     R and dU are laid out [c][k][j][i] over interior nodes only.
 *   - `stream` is a hipStream_t (NULL = default stream).  Calls are
 *     stream-ordered and asynchronous unless documented as synchronising.
 *   - Return value: OSBLI_OK (0) or a negative OSBLI_E* code; a message is
 *     kept in the context (osbli_last_error).  No call aborts, exits or
 *     throws across the ABI.
 */
#ifndef OSBLI_H
#define OSBLI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define OSBLI_ABI_VERSION 1
#define OSBLI_NGHOST 3

enum osbli_status {
    OSBLI_OK = 0,
    OSBLI_EINVAL = -1,    /* bad parameters, sizes or arguments */
    OSBLI_EDEVICE = -2,   /* a HIP runtime call failed */
    OSBLI_ENONPHYS = -3,  /* a kernel met rho <= 0, p <= 0 or NaN */
    OSBLI_ENOSPACE = -4   /* workspace too small */
};

/* boundary kinds per (direction, side), section 3.1 */
enum osbli_bc {
    OSBLI_PERIODIC = 0,        /* must be set on both sides of a direction */
    OSBLI_EXTRAPOLATE = 1,     /* zero-gradient copy of the boundary node  */
    OSBLI_ISOTHERMAL_WALL = 2, /* T = wall_T[d][side] at the boundary node */
    OSBLI_ADIABATIC_WALL = 3,  /* dT/dn = 0 (fourth-order one-sided)       */
    OSBLI_DIRICHLET = 4        /* ghost values are boundary data: set by the
                                  caller with the state, never overwritten */
};

/* Reconstructions of section 2.3-2.5 (all in the characteristic LLF frame):
 *   WENOZ5  WENO-Z, eq. wenoz_weights, tau_5 = |beta_0 - beta_2|;
 *   TENO5   TENO with K = 5 (three stencils, tau_5);
 *   TENO6   TENO with K = 6: the three-point stencils plus {i..i+3},
 *           tau_6 = |beta_3 - (beta_0 + beta_2 + 4 beta_1)/6|, optimal
 *           weights (3/10, 9/20, 1/20, 1/5) whose all-kept limit is the
 *           sixth-order reconstruction on i-2..i+3 (teno_CT < 1/4);
 *   WENOJS5 the original weights, eqs. omega and alpha, p = 2 (the paper's
 *           eps for it is 1e-6; eps is the caller's);
 *   WENOZ3  third-order WENO-Z (stencils {i, i+1}, {i-1, i}, weights
 *           (2/3, 1/3), tau_3 = |beta_0 - beta_1|);
 *   WENOZ7  seventh-order WENO-Z (section 5.2): the four-point stencils
 *           {i-r .. i-r+3}, r = 0..3, optimal weights (4/35, 18/35, 12/35,
 *           1/35), tau_7 = |beta_0 + 3 beta_1 - 3 beta_2 - beta_3|; eight
 *           stencil points per interface, so at the two outermost interfaces
 *           of a line it reads one node past the three ghost layers: the
 *           wrapped interior node on periodic lines, the third ghost layer
 *           again otherwise.  Separable meshes; periodic, extrapolated or
 *           Dirichlet ends.
 * The precision form takes WENOZ5 and TENO5; sensor routing TENO5. */
enum osbli_scheme {
    OSBLI_WENOZ5 = 0, OSBLI_TENO5 = 1, OSBLI_TENO6 = 2, OSBLI_WENOJS5 = 3, OSBLI_WENOZ3 = 4,
    OSBLI_CENTRAL4 = 5, /* fourth-order central path, below */
    OSBLI_WENOZ7 = 6
};

/* OSBLI_CENTRAL4 (section 2.6, central schemes for smooth problems; the
 * scheme of the central Taylor-Green benchmark of section 6.1), on separable
 * meshes of uniform spacing per direction (checked at set-up), FP64 form:
 * convection in conservative form, -sum_d D_d(F_d)/h_d with the fourth-order
 * first derivative and its one-sided closures; viscous and heat-flux terms
 * in expanded form: with g_ab = d_b u_a, mu~ = mu(T)/Re, kappa = mu~ /
 * ((gamma-1) M^2 Pr),
 *   d_b tau_ab = sum_b d_b mu~ (g_ab + g_ba) - (2/3) d_a mu~ div
 *              + mu~ [sum_b d_bb u_a + sum_b d_b(g_ba) - (2/3) sum_b d_a(g_bb)],
 *   energy     = sum_ab g_ab tau_ab + sum_a u_a d_b tau_ab
 *              + sum_b (d_b kappa d_b T + kappa d_bb T),
 * pure second derivatives with the printed second-derivative operator and
 * its one-sided closures, mixed ones as first derivatives of first
 * derivatives.  Two storage strategies (section 6.1): StoreSome (default;
 * only the velocity gradients are stored, in the workspace) and store-all
 * (osbli_central_store_all). */

/* Low-storage (2N) Runge-Kutta schemes of section 2.7,
 * dU <- A_s dU + dt R(U), U <- U + B_s dU, A_0 = 0:
 *   RK3      A = (0, -5/9, -153/128), B = (1/3, 15/16, 8/15), 3 stages;
 *   RK3_SSP  the strong-stability-preserving third-order 2N scheme of
 *            Gottlieb and Shu: B_0 = c_2 = 0.924574, the other four from the
 *            third-order conditions and the 2N structure, 3 stages;
 *   RK4      Carpenter and Kennedy's five-stage fourth-order 2N scheme. */
enum osbli_rk { OSBLI_RK3 = 0, OSBLI_RK3_SSP = 1, OSBLI_RK4 = 2 };

/* Arithmetic of the characteristic reconstruction and flux evaluation.
 * OSBLI_FORM_MIXED: per interface, the FP64 flux of node i is the
 * reference; deviations of the six stencil states and fluxes from it are
 * formed in FP64, rounded to FP32, projected, split, reconstructed and
 * back-projected in FP32 (the reconstructions are shift-equivariant), and
 * added to the reference in FP64.  State, RK accumulation, viscous terms,
 * metrics and the dt reduction are FP64 in every form. */
enum osbli_form { OSBLI_FORM_FP64 = 0, OSBLI_FORM_MIXED = 1 };

/* coordinate input of osbli_init_grid */
enum osbli_mesh {
    OSBLI_MESH_SEPARABLE = 0, /* x[n0], y[n1], z[n2]: x_d depends on index d only */
    OSBLI_MESH_GENERAL = 1    /* x, y, z each n0*n1*n2, i fastest              */
};

typedef struct osbli_params {
    int32_t ndim;              /* 1, 2 or 3 */
    int32_t mesh;              /* enum osbli_mesh */
    int64_t n[3];              /* interior nodes per direction; 1 when unused */
    double gamma;              /* ratio of heat capacities */
    double Re;                 /* Reynolds number; <= 0 means inviscid (Euler) */
    double Pr;                 /* Prandtl number */
    double Minf;               /* reference Mach number M_ref */
    int32_t sutherland;        /* 1: Sutherland's law, 0: mu = 1 */
    int32_t scheme;            /* enum osbli_scheme */
    double Ts_over_Tref;       /* Sutherland constant T_s / T_ref */
    double teno_CT;            /* TENO cut-off C_T */
    double eps;                /* epsilon of the nonlinear weights (1e-16; accepted range [1e-40, 1]) */
    int32_t roe_avg;           /* 1: Roe average, 0: arithmetic mean of u, H */
    int32_t form;              /* enum osbli_form */
    int32_t sensor;            /* 1: learned-sensor routing (TENO5, separable mesh) */
    int32_t rk;                /* enum osbli_rk */
    int32_t bc_kind[3][2];     /* enum osbli_bc per (direction, side) */
    double wall_T[3][2];       /* isothermal wall temperature per face */
    double period[3];          /* coordinate shift of a periodic direction */
} osbli_params;

typedef struct osbli_ctx osbli_ctx;

/* Bytes of device workspace osbli_init_grid needs for these parameters
 * (metrics, residual accumulator, viscous fluxes, reduction slots and the
 * coordinate staging used once at set-up).  Pure host function; returns 0
 * for invalid parameters. */
size_t osbli_workspace_bytes(const osbli_params *p);

/* Validate parameters, create the context and compute the metrics and
 * Jacobian once, in FP64, on the device (section 2.6, last paragraph).
 *   x, y, z    host FP64 coordinates of the interior nodes; layout given by
 *              p->mesh; pointers beyond ndim are ignored.  Periodic
 *              directions are shifted by period[d] across the wrap.
 *   workspace  device buffer of at least osbli_workspace_bytes(p) bytes,
 *              owned by the caller, which must outlive the context.
 * Errors: OSBLI_EINVAL (bad ndim / sizes / BC kinds, periodic on one side
 * only, fewer than 5 nodes along a non-periodic direction, fewer than 6
 * along a periodic one), OSBLI_ENOSPACE, OSBLI_EDEVICE.  Synchronising. */
int osbli_init_grid(osbli_ctx **ctx, const osbli_params *p, const double *x, const double *y,
                    const double *z, void *workspace, size_t ws_bytes, void *stream);

/* Impose the boundary conditions on U in place (section 3.1): wall-node
 * momentum and energy of every wall face, then the three ghost layers of
 * each direction in turn. */
int osbli_apply_bc(osbli_ctx *ctx, double *U, void *stream);

/* R = dU/dt at interior nodes: convective part (section 2.2 algorithm, all
 * directions) plus viscous part when Re > 0.  U's ghosts must be valid.
 * R: device, interior layout, may not alias U. */
int osbli_residual(osbli_ctx *ctx, const double *U, double *R, void *stream);

/* One Runge-Kutta substage (section 2.7, 2N form) of the context's scheme
 * (params.rk; stage 0 .. osbli_rk_stages() - 1):
 *   dU <- A_s dU + dt R(U),  U <- U + B_s dU;
 * stage 0 ignores the incoming dU, and the last stage does not store it (the
 * register is not read again before the next stage 0), so dU holds the
 * second-to-last stage's value after a whole step.  Does not apply boundary
 * conditions.  U (ghosted layout) and dU (interior layout) must not alias. */
int osbli_rk_substep(osbli_ctx *ctx, int stage, double dt, double *U, double *dU, void *stream);

/* Number of substages per step of the context's Runge-Kutta scheme (3 or
 * 5), and its coefficients A[s], B[s] (host arrays of at least 5). */
int osbli_rk_stages(const osbli_ctx *ctx);
int osbli_rk_coeffs(const osbli_ctx *ctx, double *A, double *B);

/* Central path, store-all strategy (section 6.1's baseline): every
 * derivative of the residual in its own work array, written by its own pass
 * and read back by an assembling pass.  osbli_central_store_all_bytes gives
 * the work size for params (0 unless scheme is OSBLI_CENTRAL4);
 * osbli_central_store_all(ctx, work, bytes) switches the context to it with
 * the caller's device buffer (256-byte aligned, kept until switched back),
 * or back to StoreSome with work = NULL.  Results agree to rounding. */
size_t osbli_central_store_all_bytes(const osbli_params *params);
int osbli_central_store_all(osbli_ctx *ctx, void *work, size_t bytes);

/* Allocation-free variant of osbli_rk_substep, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments, launches and results as
 * osbli_rk_substep; the per-substage scratch (residual accumulator, and the
 * viscous fluxes when Re > 0) lives in one library-owned static device array
 * of osbli_noalloc_scratch_bytes() = 64 MiB per GPU instead of the context's
 * workspace: 8 nc n bytes plus, when viscous, 8 (ndim (ndim + 1) / 2 + ndim) n
 * bytes on separable meshes (each distinct stress and energy flux once) or
 * 8 ndim (ndim + 1) n on general ones (n interior nodes, each part rounded
 * up to 256) must fit, e.g. a viscous separable 3D grid of up to about
 * 6.0e5 nodes, an inviscid 2D grid of up to about 2.0e6.  Larger grids return OSBLI_ENOSPACE before any launch.  The call
 * allocates nothing (no hipMalloc / hipFree, no profiling events).  Every
 * call on a GPU shares that GPU's one array and leaves its contents behind:
 * calls that overlap on one GPU (several streams or threads) race, so
 * callers serialise them.  OSBLI_EDEVICE if the array's device address
 * could not be resolved when the context was set up. */
int osbli_rk_substep_noalloc(osbli_ctx *ctx, int stage, double dt, double *U, double *dU, void *stream);

/* Size in bytes of the scratch array of osbli_rk_substep_noalloc. */
size_t osbli_noalloc_scratch_bytes(void);

/* dt = cfl / max over interior nodes of
 *   sum_d J|S_d| (|u.n_d| + a) + 2 nu_eff sum_d (J|S_d|)^2,
 * nu_eff = max(4/3, gamma/Pr) mu/(rho Re) when viscous.  Deterministic
 * device max-reduction; synchronising (one host read-back). */
int osbli_compute_dt(osbli_ctx *ctx, const double *U, double cfl, double *dt_out, void *stream);

/* Synchronises the context's last stream; returns OSBLI_ENONPHYS if any
 * kernel met rho <= 0, p <= 0 or NaN since the previous check, and clears
 * the flag. */
int osbli_check(osbli_ctx *ctx);

/* Launch shape of the convective sweeps (not part of the method; results do
 * not depend on it): seg[d] nodes per wave segment along direction d, 0 for
 * the default rule (about 2^18 lanes per sweep, at least 8 nodes). */
int osbli_set_sweep_segments(osbli_ctx *ctx, const int64_t *seg);

/* Last error message of the context (never NULL). */
const char *osbli_last_error(const osbli_ctx *ctx);

/* Release the host-side context (the workspace stays with its owner). */
void osbli_destroy(osbli_ctx *ctx);

/* ---------------------------------------------------------------------
 * Learned shock sensor (not in the paper, which names sensor-switched
 * hybrid central/shock-capturing fluxes as hard to design for every flow).
 * With params.sensor = 1 each interface is routed either to the full
 * characteristic TENO5 flux or to its exact all-stencils-kept limit
 *   F = |S| [C6 f + R diag(alpha) L D6 U],
 *   C6 = (1,-8,37,37,-8,1)/60, D6 = (1,-5,10,-10,5,-1)/60 on i-2..i+3,
 * by a 10 -> 32 -> 32 -> 1 network (ReLU, ReLU, sigmoid) evaluated on the
 * matrix cores (bfloat16 operands, FP32 accumulation).  A misrouted
 * interface is the form's only approximation.
 *
 * Features of interface i+1/2 (float32, ten per interface): Jiang-Shu
 * three-point indicators of rho/rho_bar + p/p_bar + (u.t)/a_bar on the four
 * substencils of i-2..i+3, normalised by their sum (+1e-20); jumps
 * J = |q_{k+1} - q_k| / (q_{k+1} + q_k) of rho and of p over (i-1,i),
 * (i,i+1), (i+1,i+2), as log10(1 + 1e6 J) / 6.  Label: 1 iff every TENO5 stencil
 * of every characteristic field and both splits is kept.
 * Weights: 1441 bfloat16 values in the order W1[10][32] (input-major), b1[32],
 * W2[32][32] (input-major), b2[32], w3[32], b3.
 * --------------------------------------------------------------------- */

/* Copy the routing network's weights (host array) into the context; route
 * an interface to the cheap flux when P(smooth) >= threshold there and at the
 * `dilate` (0, 1 or 2) interfaces on each side along the sweep.  Masks are
 * refreshed at stage 0 of each RK step (every substage with every_substage)
 * and by osbli_residual.  OSBLI_EINVAL for n != 1441, a threshold outside
 * (0, 1) or dilate outside 0..2.  Synchronising. */
int osbli_sensor_set_weights(osbli_ctx *ctx, const uint16_t *w_bf16_host, int n, double threshold, int dilate,
                             int every_substage, void *stream);

/* Recompute the routing masks of every direction from U. */
int osbli_sensor_update(osbli_ctx *ctx, const double *U, void *stream);

/* Number of interfaces routed to the cheap flux by the last mask refresh,
 * and the total number of interfaces.  Synchronising. */
int osbli_sensor_stats(osbli_ctx *ctx, int64_t *smooth, int64_t *total);

/* Copy the routing mask of direction dir as left by the last refresh
 * (one byte per interface, 1 = the network calls it smooth, before the
 * dilation that the sweep applies) into the caller's device buffer dst, in
 * x-fastest order of the direction's interface grid (extent n_dir + 1 along
 * dir).  OSBLI_ENOSPACE if cap is below the direction's interface count.
 * Stream-ordered. */
int osbli_sensor_masks(osbli_ctx *ctx, int dir, uint8_t *dst, int64_t cap, void *stream);

/* Interfaces of all directions: sum_d (n_d + 1) prod_{e != d} n_e. */
int osbli_interface_count(osbli_ctx *ctx, int64_t *count);

/* Training data made by the method: features (device, count x 10 float32)
 * and TENO5 all-kept labels (device, count bytes) of every interface of U,
 * direction by direction, each direction in x-fastest order of its interface
 * grid (extent n_d + 1 along d).  OSBLI_ENOSPACE if cap < count (count is
 * still returned).  Needs TENO5 and a separable mesh. */
int osbli_collect_labels(osbli_ctx *ctx, const double *U, float *feat, uint8_t *label, int64_t cap,
                         int64_t *count, void *stream);

/* Training of the network (context-free; all pointers device, stream-ordered).
 * osbli_mlp_grad: mean class-weighted binary cross-entropy of sigmoid(z)
 * against y over n samples (label-0 samples weigh w_neg), its gradient
 * (1441 float32, with respect to the bfloat16 weights w) and the loss; FP32
 * forward / backward; per-block partial sums in the workspace reduced in a
 * fixed order (deterministic). */
size_t osbli_mlp_workspace_bytes(int64_t n);
int osbli_mlp_grad(const float *X, const uint8_t *y, int64_t n, const uint16_t *w, float w_neg, float *grad,
                   float *loss, void *workspace, size_t ws_bytes, void *stream);

/* Adam step t >= 1 on the FP32 master weights; writes their bfloat16 copy
 * (round to nearest even) to w.  m, v: FP32 moment buffers (1441 each). */
int osbli_mlp_adam(float *master, uint16_t *w, const float *grad, float *m, float *v, int64_t t, float lr,
                   float b1, float b2, float eps, void *stream);

/* Logits of n samples: inference = 0 FP32 VALU (training forward),
 * inference = 1 the bfloat16 MFMA path used for routing. */
int osbli_mlp_forward(const float *X, int64_t n, const uint16_t *w, float *z, int inference, void *stream);

/* ---------------------------------------------------------------------
 * Batched advance of many independent 2D problems of uneven size (not in
 * the paper, whose runs are one block at a time).  Each problem keeps its
 * own context (osbli_init_grid), state U and RK register dU; the batch
 * advances all of them by one RK3 step per osbli_batch_step with its own
 * CFL time step per problem (section 2.7 scheme, dt clipped so that problem
 * p ends exactly at t_end[p], after which it is skipped).  A step is three
 * launches of captured graphs, one per substage, each a fixed sequence of
 * persistent kernels whose workgroups walk a tile queue spanning every
 * problem; dt, t and the active flag live on the device, so no host logic
 * runs between substages.  A batched problem evolves bit for bit as the
 * same problem advanced alone with osbli_compute_dt / osbli_rk_substep /
 * osbli_apply_bc and the same dt clipping.
 *
 * Requirements: every context 2D, separable mesh, inviscid (Re <= 0),
 * periodic or extrapolation boundaries; equal gamma, scheme, form, sensor
 * switch, averaging, C_T and epsilon; with the sensor on, weights set on
 * every context with equal threshold and dilation (context 0's weights are
 * used).  The contexts, their workspaces and the U / dU arrays must outlive
 * the batch.  Problems start at t = 0 with valid ghosts (osbli_apply_bc).
 * --------------------------------------------------------------------- */
typedef struct osbli_batch osbli_batch;

/* Device workspace of a batch of nprob problems (256-byte aligned). */
size_t osbli_batch_workspace_bytes(int nprob);

/* Create a batch over contexts ctxs[0..nprob-1] with device arrays U[p],
 * dU[p] (host arrays of device pointers), end times t_end[p] > 0 (host) and
 * the CFL number.  Tiles start at the single-grid defaults.  *batch is set
 * even on failure (for osbli_batch_last_error); release it with
 * osbli_batch_destroy.  Synchronising. */
int osbli_batch_create(osbli_batch **batch, osbli_ctx *const *ctxs, int nprob, double *const *U,
                       double *const *dU, const double *t_end, double cfl, void *workspace, size_t ws_bytes,
                       void *stream);

/* Sweep tiling of problem p: seg[2 p + 1] = nodes per wave segment of the
 * marching y sweep (clamped to n_y); seg[2 p] = for problems whose x rows
 * hold at least 64 interfaces (swept with lanes along x) the number of
 * 63-interface runs per tile (default 4, clamped to 64), else nodes per wave
 * segment of the marching x sweep.  Values must be positive.  Results do not
 * depend on it.  Drops any
 * captured graphs.  Synchronising. */
int osbli_batch_set_tiles(osbli_batch *batch, const int64_t *seg, void *stream);

/* Workgroups of each persistent sweep launch, 1..65536 (0: the defaults,
 * 2048 for the lanes-along-x sweep, 1024 for the marching ones).  Results do
 * not depend on it.  Drops any captured graphs. */
int osbli_batch_set_grid(osbli_batch *batch, int sweep_blocks);

/* Capture the three substage graphs on `stream` (must not be the NULL
 * stream).  Graph instantiation is the runtime's only allocation. */
int osbli_batch_capture(osbli_batch *batch, void *stream);

/* One RK3 substage (stage 0..2) of every active problem: the stage's
 * captured graph if any, else the same kernels launched directly.  Stage 0
 * also reduces each problem's dt (and refreshes the routing masks); stage 2
 * advances each problem's time and retires problems that reached t_end.
 * Stages must be issued in order 0, 1, 2.  Asynchronous. */
int osbli_batch_substep(osbli_batch *batch, int stage, void *stream);

/* One RK3 step of every active problem: osbli_batch_substep for stages 0, 1
 * and 2.  Asynchronous. */
int osbli_batch_step(osbli_batch *batch, void *stream);

/* Per-problem time and active flag (host arrays of nprob, may be NULL) and
 * the number of active problems.  Synchronising. */
int osbli_batch_status(osbli_batch *batch, double *t, int *active, int *nactive, void *stream);

/* Interior points of all problems, and the number of sweep wave tiles of
 * one step's x and y sweeps together. */
int osbli_batch_interior_points(osbli_batch *batch, int64_t *points, int64_t *wave_tiles);

const char *osbli_batch_last_error(const osbli_batch *batch);
void osbli_batch_destroy(osbli_batch *batch);

/* Kernel classes timed by the optional profiler. */
enum osbli_kernel_class {
    OSBLI_K_SWEEP_X = 0,   /* convective sweep along x (y = 1, z = 2 follow) */
    OSBLI_K_SWEEP_Y = 1,
    OSBLI_K_SWEEP_Z = 2,
    OSBLI_K_VISC_FLUX = 3, /* viscous-flux pass */
    OSBLI_K_FINISH = 4,    /* viscous divergence + RK update (or residual store) */
    OSBLI_K_BC = 5,        /* boundary-condition launches of one osbli_apply_bc */
    OSBLI_K_DT = 6,        /* time-step reduction */
    OSBLI_K_SENSOR = 7,    /* learned-sensor routing masks */
    OSBLI_K_CENTRAL = 8,   /* central path: derivative and residual passes */
    OSBLI_K_COUNT = 9
};

/* Instrumentation (not part of the method): when enabled, each launch group
 * of the classes above is bracketed by HIP events on the stream it runs on.
 * Enabling or disabling clears the totals.  Host-side events only; no device
 * memory is allocated. */
int osbli_profile_enable(osbli_ctx *ctx, int enable);

/* Number of timed launch groups of a class and their summed duration in
 * milliseconds since profiling was enabled.  Synchronises on the events. */
int osbli_profile_read(osbli_ctx *ctx, int kernel_class, int64_t *count, double *total_ms);

/* Version of this ABI (OSBLI_ABI_VERSION). */
int osbli_abi_version(void);

#ifdef __cplusplus
}
#endif

#endif /* OSBLI_H */
