// Internal declarations shared by the HIP translation units of libosbli.
// Not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "osbli.h"

namespace osbli {

constexpr int kGhost = OSBLI_NGHOST;

// Index space of one problem.  "ext" = ghost-extended grid of the state U,
// "int" = compact interior grid of R, dU and the viscous fluxes.
struct Grid {
    int nd, nc;
    int64_t n[3];    // interior nodes per direction (1 when unused)
    int64_t h[3];    // ghosts per side (3 when active, else 0)
    int64_t e[3];    // extended extents
    int64_t es[3];   // extended strides
    int64_t enpts;   // extended nodes (component stride of U)
    int64_t is[3];   // interior strides
    int64_t nint;    // interior nodes (component stride of R, dU)
    int periodic[3];
};

// Physical and scheme constants, precomputed once.
struct Phys {
    double gamma, gm1, Re, Pr, Minf, M2, Ts, CT, eps;
    double teno_fast;  // TENO: every stencil is kept when tau < teno_fast * min_r(beta_r + eps)
    double mu_re;      // 1/Re
    double kheat;      // 1/((gamma-1) M^2 Pr Re)
    double nu_fac;     // max(4/3, gamma/Pr)
    int sutherland, scheme, roe, viscous;
    int mixed;         // FP32 reconstruction / flux evaluation on FP64 deviations
    int dilate;        // routed form: cheap flux only if the interfaces within `dilate` along the line are smooth too
};

// Metric terms.  Separable meshes keep 1/h_d per direction (h_d = D_d x_d);
// general meshes keep node area vectors S[d][m] on the extended grid and J.
struct Metrics {
    int general;
    const double *invh[3];   // separable: n[d] values each
    const double *S;         // general: nd*nd components, stride enpts
    const double *J;         // general: enpts
};

// Device workspace carve-up (byte offsets into the caller's buffer).
struct Layout {
    size_t flags, red, invh[3], S, J, Racc, G, stage, mask[3], wts, total;
};

__host__ __device__ inline int64_t ext_index(const Grid &g, int64_t i, int64_t j, int64_t k) {
    return (i + g.h[0]) + (j + g.h[1]) * g.es[1] + (k + g.h[2]) * g.es[2];
}
__host__ __device__ inline int64_t int_index(const Grid &g, int64_t i, int64_t j, int64_t k) {
    return i + j * g.is[1] + k * g.is[2];
}

// flags word bits
constexpr unsigned kFlagNonPhys = 1u;

// 1/x for positive normal x: the hardware reciprocal estimate refined by two
// Newton-Raphson steps (each squares the relative error), within about one
// ulp of the correctly rounded quotient, in half the instructions of an IEEE
// division (which also rescales for denormals and infinities that the
// kernels' operands never are).
__device__ __forceinline__ double rcp64(double x) {
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(e, r, r);
    e = fma(-x, r, 1.0);
    return fma(e, r, r);
}

// sqrt(x) for positive normal x: g = x rsq(x) ~ sqrt(x) and h = rsq(x)/2,
// one coupled Newton step on both, then g + (x - g^2) h; within about one ulp.
__device__ __forceinline__ double sqrt64(double x) {
    const double y = __builtin_amdgcn_rsq(x);
    double g = x * y, h = 0.5 * y;
    const double r = fma(-g, h, 0.5);
    g = fma(g, r, g);
    h = fma(h, r, h);
    return fma(fma(-g, g, x), h, g);
}


// Stored viscous-flux arrays.  General meshes keep every component of
// G_k = S_k . Fv (nd (nd + 1) arrays); separable meshes store G_k = Fv_k,
// whose momentum part is the symmetric stress tensor, so its nd (nd + 1) / 2
// distinct entries (diagonal first, then (0,1), (0,2), (1,2)) and the nd
// energy fluxes are kept once each: 6 + 3 arrays in 3D instead of 12.
__host__ __device__ constexpr int gflux_count(int nd, bool gen) {
    return gen ? nd * (nd + 1) : nd * (nd + 1) / 2 + nd;
}
template <int ND, bool GEN>
__host__ __device__ constexpr int gslot(int k, int v) {
    if (GEN) return k * (ND + 1) + v;
    if (v == ND) return ND * (ND + 1) / 2 + k;
    const int a = k < v ? k : v, b = k < v ? v : k;
    return a == b ? a : (ND == 2 ? 2 : (a == 0 ? 2 + b : 5));
}

// One stage of a low-storage (2N) Runge-Kutta scheme: dU <- A dU + dt R
// (first: A = 0 and dU is not read), U <- U + B dU (last: dU is not stored,
// the register is not read again before the next step's first stage).
struct RkStage {
    double A, B;
    int first, last;
};

// The three-stage third-order scheme's stages (the batched ensemble's scheme).
inline RkStage rk3_stage(int s) {
    const double A[3] = {0.0, -5.0 / 9.0, -153.0 / 128.0}, B[3] = {1.0 / 3.0, 15.0 / 16.0, 8.0 / 15.0};
    return RkStage{A[s], B[s], s == 0, s == 2};
}

// ---- launchers (each returns hipError_t of the launch) ----
hipError_t launch_metrics_separable(const Grid &g, const double *coord1d, double *invh_out[3],
                                    const double period[3], hipStream_t s);
hipError_t launch_metrics_general(const Grid &g, const double *coords, double *stage,
                                  double *S, double *J, const double period[3], hipStream_t s);
hipError_t launch_bc(const Grid &g, const Phys &ph, const osbli_params &p, double *U, hipStream_t s);
// one convective sweep along dir; first != 0 stores R, otherwise accumulates;
// mask (may be null): routing mask of the direction's interfaces
// segment length (nodes per wave along the sweep) of the single-grid rule:
// about 2^18 lanes per launch, at least 8 nodes per segment
inline int64_t default_segment(int64_t N, int64_t lines) {
    const int64_t target = int64_t(1) << 18;
    int64_t seg = (N * lines + target - 1) / target;
    if (seg < 8) seg = 8;
    return seg < N ? seg : N;
}

// seg_req > 0 overrides the segment length of the sweep
hipError_t launch_convective(const Grid &g, const Phys &ph, const Metrics &m, const double *U,
                             double *R, unsigned *flags, int dir, int first, const uint8_t *mask,
                             int64_t seg_req, hipStream_t s);
// learned sensor
int64_t iface_count(const Grid &g, int d);
hipError_t launch_labels(const Grid &g, const Phys &ph, const double *U, int d, float *feat, uint8_t *lab,
                         hipStream_t s);
hipError_t launch_sensor(const Grid &g, const Phys &ph, const double *U, int d, const uint16_t *w, float zcut,
                         uint8_t *mask, hipStream_t s);
hipError_t launch_count_u8(const uint8_t *a, int64_t n, unsigned long long *out, hipStream_t s);
size_t mlp_workspace_bytes(int64_t n);
hipError_t launch_mlp_grad(const float *X, const uint8_t *y, int64_t n, const uint16_t *w, float wneg,
                           float *grad, float *loss, float *partial, hipStream_t s);
hipError_t launch_mlp_adam(float *master, uint16_t *w, const float *grad, float *m, float *v, int64_t t,
                           float lr, float b1, float b2, float eps, hipStream_t s);
hipError_t launch_mlp_forward(const float *X, int64_t n, const uint16_t *w, float *z, int inference,
                              hipStream_t s);
hipError_t launch_viscous_fluxes(const Grid &g, const Phys &ph, const Metrics &m, const double *U,
                                 double *G, hipStream_t s);
// mode 0: R_out = Racc + viscous;  mode 1: RK update of U, dU with Racc + viscous
hipError_t launch_finish(const Grid &g, const Phys &ph, const Metrics &m, const double *Racc,
                         const double *G, double *Rout, RkStage rs, double dt, double *U, double *dU,
                         int mode, hipStream_t s);
// fourth-order central path: residual R of U (ghosts valid); Gs: velocity
// gradients (nd^2 per node), used by the StoreSome strategy (work == null);
// work: the store-all strategy's arrays (central_work_bytes)
size_t central_work_bytes(const Grid &g, bool viscous);
hipError_t launch_central(const Grid &g, const Phys &ph, const Metrics &m, const double *U, double *Gs, void *work,
                          double *R, hipStream_t s);
hipError_t launch_dt(const Grid &g, const Phys &ph, const Metrics &m, const double *U,
                     unsigned long long *slot, hipStream_t s);
hipError_t launch_fill_u64(unsigned long long *p, unsigned long long v, int n, hipStream_t s);

// ---- batched advance of many 2D problems (batch.hip) ----
struct BProb {             // one problem, device resident
    Grid g;
    double *U, *dU, *R;
    const double *invh[3];
    uint8_t *mask[3];
    int bc[3][2];
    int xl;                            // x sweep with lanes along x (rows of >= 64 interfaces)
    int xlpt;                          // 63-interface runs per tile of that sweep
    int64_t seg[3], nseg[3], wpl[3];   // sweep tiling per direction (marching sweeps)
};

constexpr int kXlPerTile = 4;  // default 63-interface runs per tile of the batched x sweep

struct BState {            // per-problem time state, device resident
    double t, dt, tend;
    unsigned long long smax;
    int active, pad;
};

struct BatchTables {       // device prefix tables (P + 1 entries) and totals
    int64_t *w[2], *wx, *pt, *f[2], *s[2];    // wx: x-lanes sweep waves, w[0]: marching x sweep waves
    int64_t tot_w[2], tot_wx, tot_pt, tot_f[2], tot_s[2];
};

// sweep_blocks > 0: workgroups of each persistent sweep launch (else 2048
// for the lanes-along-x sweep and 1024 for the marching ones)
hipError_t launch_batch_stage(const BProb *pr, BState *st, const BatchTables &T, int P, const Phys &ph, int stage,
                              double cfl, int route, const uint16_t *w, float zcut, unsigned *flags, int sweep_blocks,
                              hipStream_t s);

}  // namespace osbli
