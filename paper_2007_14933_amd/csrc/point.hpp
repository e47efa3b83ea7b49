// Pointwise pieces shared by the single-grid and the batched kernels, so
// that both evaluate the same expressions: viscosity law, the CFL time-step
// denominator of one node, and the low-storage RK update of one value.
#pragma once
#include "internal.hpp"

namespace osbli {

// mu(T) / mu_ref: constant, or Sutherland's law (eq. sutherland)
__device__ __forceinline__ double viscosity(const Phys &ph, double T) {
    if (!ph.sutherland) return 1.0;
    return T * sqrt(T) * (1.0 + ph.Ts) / (T + ph.Ts);
}

// CFL denominator of one node (the dt reduction takes its maximum):
// sum_d J|S_d| (|u.n_d| + a) + 2 nu_eff sum_d (J|S_d|)^2
template <int ND, bool GEN>
__device__ __forceinline__ double dt_node(const double *__restrict__ U, const Grid &g, const Phys &ph,
                                          const Metrics &m, const int64_t (&idx)[3]) {
    const int64_t e = ext_index(g, idx[0], idx[1], idx[2]);
    const int64_t cs = g.enpts;
    const double r = U[e], ri = 1.0 / r;
    double u[3], ke = 0.0;
#pragma unroll
    for (int mm = 0; mm < ND; ++mm) {
        u[mm] = U[e + (1 + mm) * cs] * ri;
        ke += U[e + (1 + mm) * cs] * U[e + (1 + mm) * cs];
    }
    const double p = ph.gm1 * (U[e + (ND + 1) * cs] - 0.5 * ke * ri);
    const double a = sqrt(ph.gamma * p * ri);
    double nu = 0.0;
    if (ph.viscous) {
        const double T = ph.gamma * ph.M2 * p * ri;
        nu = ph.nu_fac * viscosity(ph, T) * ri * ph.mu_re;
    }
    double conv = 0.0, diff = 0.0;
#pragma unroll
    for (int d = 0; d < ND; ++d) {
        double js, un;
        if (!GEN) {
            js = m.invh[d][idx[d]];
            un = u[d];
        } else {
            double s2 = 0.0, us = 0.0;
#pragma unroll
            for (int c = 0; c < ND; ++c) {
                const double sm = m.S[(d * ND + c) * cs + e];
                s2 += sm * sm;
                us += u[c] * sm;
            }
            const double smag = sqrt(s2);
            js = m.J[e] * smag;
            un = us / smag;
        }
        conv += js * (fabs(un) + a);
        diff += js * js;
    }
    double sn = conv + 2.0 * nu * diff;
    if (!(sn >= 0.0)) sn = __builtin_inf();  // NaN state: force dt -> 0
    return sn;
}

// Low-storage (2N) stage: dU <- A_s dU + dt R (A_0 = 0, dU not read),
// U <- U + B_s dU.  The last stage's dU is never read (the next stage 0
// ignores it), so it is not stored.
__device__ __forceinline__ void rk_point(const RkStage &rs, double dt, double R, double *dU, double *U) {
    const double du = (rs.first ? 0.0 : rs.A * *dU) + dt * R;
    if (!rs.last) *dU = du;
    *U += rs.B * du;
}

}  // namespace osbli
