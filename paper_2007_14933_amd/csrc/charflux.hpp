// Device building blocks of the characteristic interface flux (section 2.2,
// enumerated algorithm; reconstructions of sections 2.3-2.5), shared by the
// convective sweeps and the sensor kernels.  Local frame (n, t1, t2): with
// f_k = u_n U_k + p_k (0, n, u_n) the projected flux is
// g_kj = u_n,k V_kj + p_k (l_j,m . n + l_j,E u_n,k), so only V = L U is
// formed per point and L, R are never stored as matrices.
#pragma once

#include "internal.hpp"

namespace osbli {
namespace cf {

template <int ND>
struct Pt {
    double U[ND + 2];
    double ri, p, a;
};

// Local-frame view of one stencil point: normal / tangential momentum.
template <int ND>
struct Loc {
    double r, mn, mt[2], E, p, a, ri;
};

// derived quantities of a point whose conserved state is in w.U
template <int ND>
__device__ __forceinline__ void finish_point(const Phys &ph, Pt<ND> &w, bool &bad) {
    const double ri = rcp64(w.U[0]);
    double ke = 0.0;
#pragma unroll
    for (int m = 0; m < ND; ++m) ke += w.U[1 + m] * w.U[1 + m];
    const double p = ph.gm1 * (w.U[ND + 1] - 0.5 * ke * ri);
    w.ri = ri;
    w.p = p;
    w.a = sqrt64(ph.gamma * p * ri);
    bad |= !(w.U[0] > 0.0 && p > 0.0);
}

// Fifth-order WENO-Z / TENO reconstruction at x_{i+1/2} from f_{i-2..i+2}.
// Candidate stencils S_r = {i-r .. i-r+2}, Jiang-Shu indicators,
// tau_5 = |beta_0 - beta_2|; WENO-Z alpha_r = d_r (1 + (tau/(beta_r+eps))^2);
// TENO gamma_r = (1 + tau/(beta_r+eps))^6, stencil r cut when
// gamma_r / sum(gamma) < C_T (evaluated as gamma_r < C_T * sum), weights
// d_r delta_r / sum(d delta).  The reconstruction is taken in two parts so
// that the two of one LLF split share a single division: the candidate
// values and the indicators (R5), then the weights given
// t = tau / prod_r(beta_r+eps).  TENO's normalisation divides by one of
// seven sums of optimal weights and is skipped when no stencil is cut
// (sum = 1).
struct R5 {
    double q0, q1, q2, tau, e0, e1, e2;
};

__device__ __forceinline__ R5 recon5_ind(double fm2, double fm1, double f0, double fp1, double fp2, double eps4) {
    // from the first differences d1..d4 of f_{i-2..i+2}: each candidate is
    // f_i plus two differences; the indicators are taken times 4,
    // 4 beta_r = (13/3) s_r^2 + t_r^2 (s_r the second difference, t_r the
    // one-sided or central first-difference combination of stencil r), with
    // eps4 = 4 eps, which leaves every ratio tau / (beta_r + eps) unchanged
    const double d1 = fm1 - fm2, d2 = f0 - fm1, d3 = fp1 - f0, d4 = fp2 - fp1;
    R5 r;
    r.q0 = f0 + (2.0 / 3.0) * d3 - (1.0 / 6.0) * d4;
    r.q1 = f0 + (1.0 / 6.0) * d2 + (1.0 / 3.0) * d3;
    r.q2 = f0 - (1.0 / 3.0) * d1 + (5.0 / 6.0) * d2;
    const double s0 = d4 - d3, s1 = d3 - d2, s2 = d2 - d1;
    const double t0 = d4 - 3.0 * d3, t1 = d2 + d3, t2 = 3.0 * d2 - d1;
    const double b0 = ((13.0 / 3.0) * s0) * s0 + t0 * t0;
    const double b1 = ((13.0 / 3.0) * s1) * s1 + t1 * t1;
    const double b2 = ((13.0 / 3.0) * s2) * s2 + t2 * t2;
    r.tau = fabs(b0 - b2);
    r.e0 = b0 + eps4;
    r.e1 = b1 + eps4;
    r.e2 = b2 + eps4;
    return r;
}

// TENO's cut test decided by a bound: tau < X min_r(beta_r + eps) with X =
// ph.teno_fast proves that no stencil is cut (the host derives X from C_T),
// so the value is the linear fifth-order one and the weights, with their
// division, are not evaluated.  Exact: the general path would keep all
// three stencils for these data too.
__device__ __forceinline__ bool teno5_all_kept(const R5 &r, double X) {
    return r.tau < X * fmin(fmin(r.e0, r.e1), r.e2);
}
__device__ __forceinline__ double lin5(const R5 &r) { return 0.3 * r.q0 + 0.6 * r.q1 + 0.1 * r.q2; }

template <int SCHEME>
__device__ __forceinline__ double recon5_fin(const R5 &r, double tinv, double CT, bool *kept) {
    const double x0 = (r.e1 * r.e2) * tinv, x1 = (r.e0 * r.e2) * tinv, x2 = (r.e0 * r.e1) * tinv;
    if (SCHEME == OSBLI_WENOZ5) {
        const double a0 = 0.3 * (1.0 + x0 * x0);
        const double a1 = 0.6 * (1.0 + x1 * x1);
        const double a2 = 0.1 * (1.0 + x2 * x2);
        return (a0 * r.q0 + a1 * r.q1 + a2 * r.q2) * rcp64(a0 + a1 + a2);
    } else {
        double c0 = 1.0 + x0, c1 = 1.0 + x1, c2 = 1.0 + x2;
        c0 = c0 * c0 * c0;
        c1 = c1 * c1 * c1;
        c2 = c2 * c2 * c2;
        const double g0 = c0 * c0, g1 = c1 * c1, g2 = c2 * c2;
        const double lim = CT * (g0 + g1 + g2);
        const bool k0 = !(g0 < lim), k1 = !(g1 < lim), k2 = !(g2 < lim);
        const double w0 = k0 ? 0.3 : 0.0;
        const double w1 = k1 ? 0.6 : 0.0;
        const double w2 = k2 ? 0.1 : 0.0;
        const double num = w0 * r.q0 + w1 * r.q1 + w2 * r.q2;
        if (kept) *kept = *kept && k0 && k1 && k2;
        if (k0 && k1 && k2) return num;
        return num * rcp64(w0 + w1 + w2);
    }
}

// ---- further reconstructions, one side at a time ----
// TENO6 (section 2.5, K = 6) at x_{i+1/2} from f_{i-2..i+3}: the three
// three-point candidates and the cubic on {i..i+3}, value
// f_i/4 + 13 f_{i+1}/12 - 5 f_{i+2}/12 + f_{i+3}/12 and Jiang-Shu indicator
// (1/36)(-11 f_i + 18 f_{i+1} - 9 f_{i+2} + 2 f_{i+3})^2
//   + (13/12)(2 f_i - 5 f_{i+1} + 4 f_{i+2} - f_{i+3})^2
//   + (781/720)(-f_i + 3 f_{i+1} - 3 f_{i+2} + f_{i+3})^2;
// tau_6 = |beta_3 - (beta_0 + beta_2 + 4 beta_1)/6|, gamma_r = (1 +
// tau_6/(beta_r + eps))^6, stencil r cut when gamma_r < C_T sum(gamma),
// optimal weights (3/10, 9/20, 1/20, 1/5) (the sixth-order reconstruction
// when every stencil is kept).  The four ratios tau/(beta_r + eps) share
// one division: x_r = tau prod_{s != r}(beta_s + eps) / prod_s(beta_s + eps).
__device__ __forceinline__ double recon6_teno(double fm2, double fm1, double f0, double fp1, double fp2, double fp3,
                                              double CT, double eps, double X, bool *kept) {
    // from the first differences d1..d5 of f_{i-2..i+3} (as recon5_ind): each
    // candidate is f_i plus differences, and the indicators are taken times 4
    // with 4 eps, which leaves every ratio tau / (beta_r + eps) unchanged
    const double d1 = fm1 - fm2, d2 = f0 - fm1, d3 = fp1 - f0, d4 = fp2 - fp1, d5 = fp3 - fp2;
    const double q0 = f0 + (2.0 / 3.0) * d3 - (1.0 / 6.0) * d4;
    const double q1 = f0 + (1.0 / 6.0) * d2 + (1.0 / 3.0) * d3;
    const double q2 = f0 - (1.0 / 3.0) * d1 + (5.0 / 6.0) * d2;
    const double q3 = f0 + 0.75 * d3 - (1.0 / 3.0) * d4 + (1.0 / 12.0) * d5;
    const double s0 = d4 - d3, s1 = d3 - d2, s2 = d2 - d1;
    const double t0 = d4 - 3.0 * d3, t1 = d2 + d3, t2 = 3.0 * d2 - d1;
    const double b0 = ((13.0 / 3.0) * s0) * s0 + t0 * t0;
    const double b1 = ((13.0 / 3.0) * s1) * s1 + t1 * t1;
    const double b2 = ((13.0 / 3.0) * s2) * s2 + t2 * t2;
    // the cubic's combinations -11 f_i + 18 f_{i+1} - 9 f_{i+2} + 2 f_{i+3},
    // 2 f_i - 5 f_{i+1} + 4 f_{i+2} - f_{i+3}, -f_i + 3 f_{i+1} - 3 f_{i+2} + f_{i+3}
    const double a = 11.0 * d3 - 7.0 * d4 + 2.0 * d5;
    const double b = 3.0 * d4 - 2.0 * d3 - d5;
    const double c = d3 - 2.0 * d4 + d5;
    const double b3 = ((1.0 / 9.0) * a) * a + ((13.0 / 3.0) * b) * b + ((781.0 / 180.0) * c) * c;
    const double tau = fabs(b3 - (b0 + b2 + 4.0 * b1) * (1.0 / 6.0));
    const double eps4 = 4.0 * eps;
    const double e0 = b0 + eps4, e1 = b1 + eps4, e2 = b2 + eps4, e3 = b3 + eps4;
    // cut test decided by the bound (as for TENO5): no stencil cut
    if (tau < X * fmin(fmin(e0, e1), fmin(e2, e3))) return 0.3 * q0 + 0.45 * q1 + 0.05 * q2 + 0.2 * q3;
    const double e01 = e0 * e1, e23 = e2 * e3;
    const double tq = tau * rcp64(e01 * e23);
    double c0 = 1.0 + tq * (e1 * e23), c1 = 1.0 + tq * (e0 * e23);
    double c2 = 1.0 + tq * (e01 * e3), c3 = 1.0 + tq * (e01 * e2);
    c0 = c0 * c0 * c0;
    c1 = c1 * c1 * c1;
    c2 = c2 * c2 * c2;
    c3 = c3 * c3 * c3;
    const double g0 = c0 * c0, g1 = c1 * c1, g2 = c2 * c2, g3 = c3 * c3;
    const double lim = CT * (g0 + g1 + g2 + g3);
    const bool k0 = !(g0 < lim), k1 = !(g1 < lim), k2 = !(g2 < lim), k3 = !(g3 < lim);
    const double w0 = k0 ? 0.3 : 0.0, w1 = k1 ? 0.45 : 0.0, w2 = k2 ? 0.05 : 0.0, w3 = k3 ? 0.2 : 0.0;
    const double num = w0 * q0 + w1 * q1 + w2 * q2 + w3 * q3;
    if (kept) *kept = *kept && k0 && k1 && k2 && k3;
    if (k0 && k1 && k2 && k3) return num;
    return num * rcp64(w0 + w1 + w2 + w3);
}

// WENO-JS5 (section 2.3, eqs. omega and alpha, p = 2): alpha_r = d_r /
// (beta_r + eps)^2; the normalisation cancels the common factor
// prod_s (beta_s + eps)^2, so omega_r = d_r P_r / sum_k d_k P_k with
// P_r = prod_{s != r} (beta_s + eps)^2 and one division per reconstruction.
__device__ __forceinline__ double recon5_js(double fm2, double fm1, double f0, double fp1, double fp2, double eps) {
    const R5 r = recon5_ind(fm2, fm1, f0, fp1, fp2, 4.0 * eps);
    const double s0 = r.e0 * r.e0, s1 = r.e1 * r.e1, s2 = r.e2 * r.e2;
    const double a0 = 0.3 * (s1 * s2), a1 = 0.6 * (s0 * s2), a2 = 0.1 * (s0 * s1);
    return (a0 * r.q0 + a1 * r.q1 + a2 * r.q2) * rcp64(a0 + a1 + a2);
}

// WENO-3Z (third-order WENO-Z, the lowest order of section 5.2) at
// x_{i+1/2} from f_{i-1..i+1}: candidates (f_i + f_{i+1})/2 and
// (3 f_i - f_{i-1})/2, indicators (f_{i+1} - f_i)^2 and (f_i - f_{i-1})^2,
// optimal weights (2/3, 1/3), tau_3 = |beta_0 - beta_1|, alpha_r = d_r (1 +
// (tau/(beta_r + eps))^2); one division for the two ratios.
__device__ __forceinline__ double recon3_z(double fm1, double f0, double fp1, double eps) {
    const double q0 = 0.5 * f0 + 0.5 * fp1, q1 = 1.5 * f0 - 0.5 * fm1;
    const double d0 = fp1 - f0, d1 = f0 - fm1;
    const double b0 = d0 * d0, b1 = d1 * d1;
    const double tau = fabs(b0 - b1);
    const double e0 = b0 + eps, e1 = b1 + eps;
    const double tq = tau * rcp64(e0 * e1);
    const double x0 = tq * e1, x1 = tq * e0;
    const double a0 = (2.0 / 3.0) * (1.0 + x0 * x0), a1 = (1.0 / 3.0) * (1.0 + x1 * x1);
    return (a0 * q0 + a1 * q1) * rcp64(a0 + a1);
}

// WENO-7Z (seventh-order WENO-Z, the highest order of section 5.2) at
// x_{i+1/2} from f_{i-3..i+3}: four candidate stencils S_r = {i-r .. i-r+3},
// each the cell-average reconstruction of its cubic evaluated at x_{i+1/2};
// Jiang-Shu indicator of that cubic over cell i,
//   beta_r = A_r^2/36 + (13/12) B_r^2 + (781/720) C_r^2
// with A_r, B_r, C_r six, two and six times the cubic's first, second and
// third Taylor coefficients about the cell centre (A with the third folded
// in), written on the first differences d1..d6 of the seven values and taken
// times 4 (with 4 eps, which leaves the ratios unchanged); optimal weights
// (4/35, 18/35, 12/35, 1/35), tau_7 = |beta_0 + 3 beta_1 - 3 beta_2 -
// beta_3|, alpha_r = d_r (1 + (tau/(beta_r + eps))^2); the four ratios
// share one division and the normalisation takes another.
__device__ __forceinline__ double recon7_z(double fm3, double fm2, double fm1, double f0, double fp1, double fp2,
                                           double fp3, double eps) {
    const double d1 = fm2 - fm3, d2 = fm1 - fm2, d3 = f0 - fm1, d4 = fp1 - f0, d5 = fp2 - fp1, d6 = fp3 - fp2;
    const double q0 = f0 + 0.75 * d4 - (1.0 / 3.0) * d5 + (1.0 / 12.0) * d6;
    const double q1 = f0 + (1.0 / 12.0) * d3 + 0.5 * d4 - (1.0 / 12.0) * d5;
    const double q2 = f0 - (1.0 / 12.0) * d2 + (1.0 / 3.0) * d3 + 0.25 * d4;
    const double q3 = f0 + 0.25 * d1 - (5.0 / 6.0) * d2 + (13.0 / 12.0) * d3;
    auto ind = [](double a, double b, double c) {
        return ((1.0 / 9.0) * a) * a + ((13.0 / 3.0) * b) * b + ((781.0 / 180.0) * c) * c;
    };
    const double b0 = ind(11.0 * d4 - 7.0 * d5 + 2.0 * d6, 3.0 * d5 - 2.0 * d4 - d6, d4 - 2.0 * d5 + d6);
    const double b1 = ind(2.0 * d3 + 5.0 * d4 - d5, d4 - d3, d3 - 2.0 * d4 + d5);
    const double b2 = ind(5.0 * d3 + 2.0 * d4 - d2, d4 - d3, d2 - 2.0 * d3 + d4);
    const double b3 = ind(2.0 * d1 - 7.0 * d2 + 11.0 * d3, d1 - 3.0 * d2 + 2.0 * d3, d1 - 2.0 * d2 + d3);
    const double tau = fabs(b0 + 3.0 * b1 - 3.0 * b2 - b3);
    const double eps4 = 4.0 * eps;
    const double e0 = b0 + eps4, e1 = b1 + eps4, e2 = b2 + eps4, e3 = b3 + eps4;
    const double e01 = e0 * e1, e23 = e2 * e3;
    const double tq = tau * rcp64(e01 * e23);
    const double x0 = tq * (e1 * e23), x1 = tq * (e0 * e23), x2 = tq * (e01 * e3), x3 = tq * (e01 * e2);
    const double a0 = (4.0 / 35.0) * (1.0 + x0 * x0), a1 = (18.0 / 35.0) * (1.0 + x1 * x1);
    const double a2 = (12.0 / 35.0) * (1.0 + x2 * x2), a3 = (1.0 / 35.0) * (1.0 + x3 * x3);
    return (a0 * q0 + a1 * q1 + a2 * q2 + a3 * q3) * rcp64((a0 + a1) + (a2 + a3));
}

// LLF split of one characteristic field over the six points and the two
// reconstructions: ghat = recon+(g+_{i-2..i+2}) + recon-(g-_{i+3..i-1})
// (TENO6: recon+(g+_{i-2..i+3}) + recon-(g-_{i+3..i-2}); WENO-3Z:
// recon+(g+_{i-1..i+1}) + recon-(g-_{i+2..i}); WENO-7Z reads W = 8 points,
// recon+(g+_{i-3..i+3}) + recon-(g-_{i+4..i-2})).  Takes V, gh = g/2 and
// ha = alpha/2, so g+- = (g +- alpha V)/2 = gh +- ha V.
// SHARED: one division serves both sides: with D+- = prod_r(beta_r+eps),
// tau+/D+ = tau+ D- / (D+ D-) and likewise for the other side (D+ D- >=
// eps^6, which the accepted range of eps keeps a normal number).  This
// saves five divisions per interface but keeps both sides' indicators live
// at once, which the marching sweeps can afford and the lane-per-interface
// sweep cannot (it spills), so that one divides per side.
template <int SCHEME, bool SHARED, int W>
__device__ __forceinline__ double split_recon(const double (&V)[W], const double (&gh)[W], double ha,
                                              const Phys &ph, bool *kept = nullptr) {
    double gp[W], gm[W];
#pragma unroll
    for (int k = 0; k < W; ++k) {
        gp[k] = gh[k] + ha * V[k];
        gm[k] = gh[k] - ha * V[k];
    }
    if constexpr (SCHEME == OSBLI_WENOZ7) {
        // eight points i-3..i+4: recon+(g+_{i-3..i+3}) + recon-(g-_{i+4..i-2})
        return recon7_z(gp[0], gp[1], gp[2], gp[3], gp[4], gp[5], gp[6], ph.eps) +
               recon7_z(gm[7], gm[6], gm[5], gm[4], gm[3], gm[2], gm[1], ph.eps);
    } else if constexpr (SCHEME == OSBLI_TENO6) {
        return recon6_teno(gp[0], gp[1], gp[2], gp[3], gp[4], gp[5], ph.CT, ph.eps, ph.teno_fast, kept) +
               recon6_teno(gm[5], gm[4], gm[3], gm[2], gm[1], gm[0], ph.CT, ph.eps, ph.teno_fast, kept);
    } else if constexpr (SCHEME == OSBLI_WENOJS5) {
        return recon5_js(gp[0], gp[1], gp[2], gp[3], gp[4], ph.eps) +
               recon5_js(gm[5], gm[4], gm[3], gm[2], gm[1], ph.eps);
    } else if constexpr (SCHEME == OSBLI_WENOZ3) {
        return recon3_z(gp[1], gp[2], gp[3], ph.eps) + recon3_z(gm[4], gm[3], gm[2], ph.eps);
    } else if (SHARED) {
        const double eps4 = 4.0 * ph.eps;
        const R5 a = recon5_ind(gp[0], gp[1], gp[2], gp[3], gp[4], eps4);
        const R5 b = recon5_ind(gm[5], gm[4], gm[3], gm[2], gm[1], eps4);
        if (SCHEME == OSBLI_TENO5 && teno5_all_kept(a, ph.teno_fast) && teno5_all_kept(b, ph.teno_fast))
            return lin5(a) + lin5(b);
        const double da = (a.e0 * a.e1) * a.e2, db = (b.e0 * b.e1) * b.e2;
        const double inv = rcp64(da * db);
        return recon5_fin<SCHEME>(a, (a.tau * db) * inv, ph.CT, kept) +
               recon5_fin<SCHEME>(b, (b.tau * da) * inv, ph.CT, kept);
    } else {
        const double eps4 = 4.0 * ph.eps;
        const R5 a = recon5_ind(gp[0], gp[1], gp[2], gp[3], gp[4], eps4);
        double ha5;
        if (SCHEME == OSBLI_TENO5 && teno5_all_kept(a, ph.teno_fast)) ha5 = lin5(a);
        else ha5 = recon5_fin<SCHEME>(a, a.tau * rcp64((a.e0 * a.e1) * a.e2), ph.CT, kept);
        const R5 b = recon5_ind(gm[5], gm[4], gm[3], gm[2], gm[1], eps4);
        if (SCHEME == OSBLI_TENO5 && teno5_all_kept(b, ph.teno_fast)) return ha5 + lin5(b);
        return ha5 + recon5_fin<SCHEME>(b, b.tau * rcp64((b.e0 * b.e1) * b.e2), ph.CT, kept);
    }
}

// Interface flux in the local frame (unit |S|) from the W stencil points
// i-W/2+1 .. i+W/2 (W = 6, or 8 for WENO-7Z).  Outputs: mass, normal
// momentum, tangential momenta, energy.
template <int ND, int SCHEME, bool SHARED = true, int W = 6>
__device__ __forceinline__ void char_flux(const Loc<ND> (&P)[W], const Phys &ph, double &Fr, double &Fn,
                                          double (&Ft)[2], double &FE, bool *kept = nullptr) {
    constexpr int NT = ND - 1;  // tangents
    constexpr int L = W / 2 - 1, R = W / 2;  // the nodes either side of the interface
    // averaged state at the half node (Roe, or arithmetic mean with unit weights)
    double sl = 1.0, sr = 1.0;
    if (ph.roe) {
        sl = sqrt64(P[L].r);
        sr = sqrt64(P[R].r);
    }
    const double iw = rcp64(sl + sr);
    const double un = (sl * (P[L].mn * P[L].ri) + sr * (P[R].mn * P[R].ri)) * iw;
    double ut[2] = {0.0, 0.0};
#pragma unroll
    for (int s = 0; s < NT; ++s) ut[s] = (sl * (P[L].mt[s] * P[L].ri) + sr * (P[R].mt[s] * P[R].ri)) * iw;
    const double Hh = (sl * ((P[L].E + P[L].p) * P[L].ri) + sr * ((P[R].E + P[R].p) * P[R].ri)) * iw;
    double K = un * un;
#pragma unroll
    for (int s = 0; s < NT; ++s) K += ut[s] * ut[s];
    K *= 0.5;
    const double ah = sqrt64(ph.gm1 * (Hh - K));
    const double ia = rcp64(ah);
    const double b = ph.gm1 * ia * ia;
    // Every field is split as g+- = gh +- (alpha/2) V with gh = g/2, built
    // directly from hu = u_n/2 and the halved combinations A, B below, so no
    // product is scaled by 1/2 afterwards (powers of two: exact).
    const double hb = 0.5 * b, hia = 0.5 * ia;
    double hu[W], A[W], B[W], am[W], ap[W], a0 = 0.0;
#pragma unroll
    for (int k = 0; k < W; ++k) {
        hu[k] = P[k].mn * (0.5 * P[k].ri);
        double um = un * P[k].mn;
#pragma unroll
        for (int s = 0; s < NT; ++s) um += ut[s] * P[k].mt[s];
        A[k] = hb * (K * P[k].r - um + P[k].E);
        B[k] = (un * P[k].r - P[k].mn) * hia;
        am[k] = fabs(2.0 * hu[k] - P[k].a);
        ap[k] = fabs(2.0 * hu[k] + P[k].a);
        a0 = fmax(a0, fabs(hu[k]));
    }
    double aminus = am[0], aplus = ap[0];
#pragma unroll
    for (int k = 1; k < W; ++k) {
        aminus = fmax(aminus, am[k]);
        aplus = fmax(aplus, ap[k]);
    }
    double V[W], gh[W];
    // field u_n - a: V = (A + B)|full / 2, g = u_n V + p (b u_n - (b un + 1/a)) / 2
    const double cm = 0.25 * (b * un + ia), cp = 0.25 * (b * un - ia), hbun = hb * un;
#pragma unroll
    for (int k = 0; k < W; ++k) {
        V[k] = A[k] + B[k];
        gh[k] = hu[k] * V[k] + P[k].p * (hb * hu[k] - cm);
    }
    const double h0 = split_recon<SCHEME, SHARED, W>(V, gh, 0.5 * aminus, ph, kept);
    // field u_n + a
#pragma unroll
    for (int k = 0; k < W; ++k) {
        V[k] = A[k] - B[k];
        gh[k] = hu[k] * V[k] + P[k].p * (hb * hu[k] - cp);
    }
    const double h4 = split_recon<SCHEME, SHARED, W>(V, gh, 0.5 * aplus, ph, kept);
    // entropy field: V = rho - b (K rho - u.m + E), g = u_n V + p b (un - u_n)
#pragma unroll
    for (int k = 0; k < W; ++k) {
        V[k] = P[k].r - 2.0 * A[k];
        gh[k] = hu[k] * V[k] + P[k].p * (hbun - b * hu[k]);
    }
    const double h1 = split_recon<SCHEME, SHARED, W>(V, gh, a0, ph, kept);
    // shear fields: V = m_t - ut rho, g = u_n V
    double ht[2] = {0.0, 0.0};
#pragma unroll
    for (int s = 0; s < NT; ++s) {
#pragma unroll
        for (int k = 0; k < W; ++k) {
            V[k] = P[k].mt[s] - ut[s] * P[k].r;
            gh[k] = hu[k] * V[k];
        }
        ht[s] = split_recon<SCHEME, SHARED, W>(V, gh, a0, ph, kept);
    }
    // back to physical space: F = R ghat
    const double hs = h0 + h1 + h4;
    const double hd = h4 - h0;
    Fr = hs;
    Fn = un * hs + ah * hd;
    FE = Hh * (h0 + h4) + ah * un * hd + K * h1;
#pragma unroll
    for (int s = 0; s < NT; ++s) {
        Ft[s] = ut[s] * hs + ht[s];
        FE += ut[s] * ht[s];
    }
}

// ---------------------------------------------------------------- mixed form
// Reconstruction and flux evaluation in FP32 on deviations from an FP64
// reference: with U_ref = U_i, f_ref = f(U_i) (local frame, FP64), the split
// fluxes are g+- = (L f_ref +- alpha L U_ref)/2 + (L df +- alpha L dU)/2, and
// both reconstructions are exactly shift-equivariant (sum of weights 1,
// smoothness indicators use differences only), so
//   F = f_ref + R (recon+(dg+) + recon-(dg-)).
// f_ref and the final sum are FP64; everything between runs on the FP32
// deviations, whose rounding is relative to |df|, not to |f|.
__device__ __forceinline__ float rcpf(float x) { return __builtin_amdgcn_rcpf(x); }

// FP32 WENO-Z / TENO with overflow-safe weights: the TENO cut-off is
// evaluated on c_r / max(c) (gamma_r = (1 + tau/(beta_r+eps))^6 exceeds the
// FP32 range at nearly every jump), WENO-Z's alpha on x_r / max(x) once
// max(x) >= 1.  Both are algebraically the FP64 test.
template <int SCHEME>
__device__ __forceinline__ float recon5f(float fm2, float fm1, float f0, float fp1, float fp2, float CT, float eps,
                                         float X) {
    const float q0 = (1.0f / 3.0f) * f0 + (5.0f / 6.0f) * fp1 - (1.0f / 6.0f) * fp2;
    const float q1 = -(1.0f / 6.0f) * fm1 + (5.0f / 6.0f) * f0 + (1.0f / 3.0f) * fp1;
    const float q2 = (1.0f / 3.0f) * fm2 - (7.0f / 6.0f) * fm1 + (11.0f / 6.0f) * f0;
    float s, t;
    s = f0 - 2.0f * fp1 + fp2;
    t = 3.0f * f0 - 4.0f * fp1 + fp2;
    const float b0 = (13.0f / 12.0f) * s * s + 0.25f * t * t;
    s = fm1 - 2.0f * f0 + fp1;
    t = fm1 - fp1;
    const float b1 = (13.0f / 12.0f) * s * s + 0.25f * t * t;
    s = fm2 - 2.0f * fm1 + f0;
    t = fm2 - 4.0f * fm1 + 3.0f * f0;
    const float b2 = (13.0f / 12.0f) * s * s + 0.25f * t * t;
    const float tau = fabsf(b0 - b2);
    // TENO: no stencil can be cut under the bound (as in FP64)
    if (SCHEME == OSBLI_TENO5 && tau < X * (fminf(fminf(b0, b1), b2) + eps)) return 0.3f * q0 + 0.6f * q1 + 0.1f * q2;
    const float x0 = tau * rcpf(b0 + eps), x1 = tau * rcpf(b1 + eps), x2 = tau * rcpf(b2 + eps);
    if (SCHEME == OSBLI_WENOZ5) {
        const float xm = fmaxf(x0, fmaxf(x1, x2));
        float a0, a1, a2;
        if (xm < 1.0f) {
            a0 = 0.3f * (1.0f + x0 * x0);
            a1 = 0.6f * (1.0f + x1 * x1);
            a2 = 0.1f * (1.0f + x2 * x2);
        } else {
            const float h = rcpf(xm);
            const float w0 = x0 * h, w1 = x1 * h, w2 = x2 * h, h2 = h * h;
            a0 = 0.3f * (h2 + w0 * w0);
            a1 = 0.6f * (h2 + w1 * w1);
            a2 = 0.1f * (h2 + w2 * w2);
        }
        return (a0 * q0 + a1 * q1 + a2 * q2) * rcpf(a0 + a1 + a2);
    } else {
        const float c0 = 1.0f + x0, c1 = 1.0f + x1, c2 = 1.0f + x2;
        const float ic = rcpf(fmaxf(c0, fmaxf(c1, c2)));
        float r0 = c0 * ic, r1 = c1 * ic, r2 = c2 * ic;
        r0 = r0 * r0 * r0;
        r1 = r1 * r1 * r1;
        r2 = r2 * r2 * r2;
        const float g0 = r0 * r0, g1 = r1 * r1, g2 = r2 * r2;
        const float lim = CT * (g0 + g1 + g2);
        const bool k0 = !(g0 < lim), k1 = !(g1 < lim), k2 = !(g2 < lim);
        const float w0 = k0 ? 0.3f : 0.0f, w1 = k1 ? 0.6f : 0.0f, w2 = k2 ? 0.1f : 0.0f;
        const float num = w0 * q0 + w1 * q1 + w2 * q2;
        if (k0 && k1 && k2) return num;
        return num * rcpf(w0 + w1 + w2);
    }
}

template <int SCHEME>
__device__ __forceinline__ float split_reconf(const float (&V)[6], const float (&G)[6], float alpha, float CT,
                                              float eps, float X) {
    float gp[6], gm[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        gp[k] = 0.5f * (G[k] + alpha * V[k]);
        gm[k] = 0.5f * (G[k] - alpha * V[k]);
    }
    return recon5f<SCHEME>(gp[0], gp[1], gp[2], gp[3], gp[4], CT, eps, X) +
           recon5f<SCHEME>(gm[5], gm[4], gm[3], gm[2], gm[1], CT, eps, X);
}

template <int ND, int SCHEME>
__device__ __forceinline__ void char_flux_mixed(const Loc<ND> (&P)[6], const Phys &ph, double &Fr, double &Fn,
                                                double (&Ft)[2], double &FE) {
    constexpr int NT = ND - 1;
    // FP64 reference flux of node i in the local frame:
    // f = u_n (rho, m_n, m_t, E) + p (0, 1, 0, u_n)
    double un64[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) un64[k] = P[k].mn * P[k].ri;
    const double fr0 = P[2].mn;
    const double fn0 = P[2].mn * un64[2] + P[2].p;
    double ft0[2] = {0.0, 0.0};
#pragma unroll
    for (int s = 0; s < NT; ++s) ft0[s] = P[2].mt[s] * un64[2];
    const double fE0 = (P[2].E + P[2].p) * un64[2];

    float dr[6], dmn[6], dmt[2][6], dE[6], gr[6], gmn[6], gmt[2][6], gE[6], unf[6], af[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        dr[k] = (float)(P[k].r - P[2].r);
        dmn[k] = (float)(P[k].mn - P[2].mn);
        dE[k] = (float)(P[k].E - P[2].E);
        gr[k] = (float)(P[k].mn - fr0);
        gmn[k] = (float)(P[k].mn * un64[k] + P[k].p - fn0);
        gE[k] = (float)((P[k].E + P[k].p) * un64[k] - fE0);
#pragma unroll
        for (int s = 0; s < NT; ++s) {
            dmt[s][k] = (float)(P[k].mt[s] - P[2].mt[s]);
            gmt[s][k] = (float)(P[k].mt[s] * un64[k] - ft0[s]);
        }
        unf[k] = (float)un64[k];
        af[k] = (float)P[k].a;
    }
    // averaged state of nodes i, i+1 in FP32
    float sl = 1.0f, sr = 1.0f;
    if (ph.roe) {
        sl = sqrtf((float)P[2].r);
        sr = sqrtf((float)P[3].r);
    }
    const float iw = rcpf(sl + sr);
    const float un = (sl * unf[2] + sr * unf[3]) * iw;
    float ut[2] = {0.0f, 0.0f};
#pragma unroll
    for (int s = 0; s < NT; ++s)
        ut[s] = (sl * (float)(P[2].mt[s] * P[2].ri) + sr * (float)(P[3].mt[s] * P[3].ri)) * iw;
    const float Hl = (float)((P[2].E + P[2].p) * P[2].ri), Hr = (float)((P[3].E + P[3].p) * P[3].ri);
    const float Hh = (sl * Hl + sr * Hr) * iw;
    float K = un * un;
#pragma unroll
    for (int s = 0; s < NT; ++s) K += ut[s] * ut[s];
    K *= 0.5f;
    const float gm1 = (float)ph.gm1;
    const float ah = sqrtf(gm1 * (Hh - K));
    const float ia = rcpf(ah);
    const float b = gm1 * ia * ia;
    const float CT = (float)ph.CT, eps = (float)ph.eps, X = (float)ph.teno_fast;

    float A[6], B[6], Ag[6], Bg[6], aminus = 0.0f, aplus = 0.0f, a0 = 0.0f;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        float um = un * dmn[k], ug = un * gmn[k];
#pragma unroll
        for (int s = 0; s < NT; ++s) {
            um += ut[s] * dmt[s][k];
            ug += ut[s] * gmt[s][k];
        }
        A[k] = b * (K * dr[k] - um + dE[k]);
        B[k] = (un * dr[k] - dmn[k]) * ia;
        Ag[k] = b * (K * gr[k] - ug + gE[k]);
        Bg[k] = (un * gr[k] - gmn[k]) * ia;
        aminus = fmaxf(aminus, fabsf(unf[k] - af[k]));
        aplus = fmaxf(aplus, fabsf(unf[k] + af[k]));
        a0 = fmaxf(a0, fabsf(unf[k]));
    }
    float V[6], G[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        V[k] = 0.5f * (A[k] + B[k]);
        G[k] = 0.5f * (Ag[k] + Bg[k]);
    }
    const float h0 = split_reconf<SCHEME>(V, G, aminus, CT, eps, X);
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        V[k] = 0.5f * (A[k] - B[k]);
        G[k] = 0.5f * (Ag[k] - Bg[k]);
    }
    const float h4 = split_reconf<SCHEME>(V, G, aplus, CT, eps, X);
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        V[k] = dr[k] - A[k];
        G[k] = gr[k] - Ag[k];
    }
    const float h1 = split_reconf<SCHEME>(V, G, a0, CT, eps, X);
    float ht[2] = {0.0f, 0.0f};
#pragma unroll
    for (int s = 0; s < NT; ++s) {
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            V[k] = dmt[s][k] - ut[s] * dr[k];
            G[k] = gmt[s][k] - ut[s] * gr[k];
        }
        ht[s] = split_reconf<SCHEME>(V, G, a0, CT, eps, X);
    }
    const float hs = h0 + h1 + h4, hd = h4 - h0;
    float dFE = Hh * (h0 + h4) + ah * un * hd + K * h1;
    Fr = fr0 + (double)hs;
    Fn = fn0 + (double)(un * hs + ah * hd);
#pragma unroll
    for (int s = 0; s < NT; ++s) {
        Ft[s] = ft0[s] + (double)(ut[s] * hs + ht[s]);
        dFE += ut[s] * ht[s];
    }
    FE = fE0 + (double)dFE;
}


// ------------------------------------------------------------- cheap flux
// Exact all-stencils-kept limit of char_flux: summing the split upwind-5
// reconstructions gives F = C6 f + R diag(alpha) L D6 U with
// C6 = (1, -8, 37, 37, -8, 1)/60 and D6 = (1, -5, 10, -10, 5, -1)/60 on
// i-2..i+3 (same averaged state, L, R and alpha as the full flux).
template <int ND>
__device__ __forceinline__ void cheap_flux(const Loc<ND> (&P)[6], const Phys &ph, double &Fr, double &Fn,
                                           double (&Ft)[2], double &FE) {
    constexpr int NT = ND - 1;
    constexpr double C6[6] = {1.0 / 60.0, -8.0 / 60.0, 37.0 / 60.0, 37.0 / 60.0, -8.0 / 60.0, 1.0 / 60.0};
    constexpr double D6[6] = {1.0 / 60.0, -5.0 / 60.0, 10.0 / 60.0, -10.0 / 60.0, 5.0 / 60.0, -1.0 / 60.0};
    double sl = 1.0, sr = 1.0;
    if (ph.roe) {
        sl = sqrt64(P[2].r);
        sr = sqrt64(P[3].r);
    }
    const double iw = rcp64(sl + sr);
    const double un = (sl * (P[2].mn * P[2].ri) + sr * (P[3].mn * P[3].ri)) * iw;
    double ut[2] = {0.0, 0.0};
#pragma unroll
    for (int s = 0; s < NT; ++s) ut[s] = (sl * (P[2].mt[s] * P[2].ri) + sr * (P[3].mt[s] * P[3].ri)) * iw;
    const double Hh = (sl * ((P[2].E + P[2].p) * P[2].ri) + sr * ((P[3].E + P[3].p) * P[3].ri)) * iw;
    double K = un * un;
#pragma unroll
    for (int s = 0; s < NT; ++s) K += ut[s] * ut[s];
    K *= 0.5;
    const double ah = sqrt64(ph.gm1 * (Hh - K));
    const double ia = rcp64(ah);
    const double b = ph.gm1 * ia * ia;
    double aminus = 0.0, aplus = 0.0, a0 = 0.0;
    double cr = 0.0, cn = 0.0, ct[2] = {0.0, 0.0}, cE = 0.0;   // C6 f
    double dr = 0.0, dn = 0.0, dt[2] = {0.0, 0.0}, dE = 0.0;   // D6 U
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        const double unk = P[k].mn * P[k].ri;
        aminus = fmax(aminus, fabs(unk - P[k].a));
        aplus = fmax(aplus, fabs(unk + P[k].a));
        a0 = fmax(a0, fabs(unk));
        cr += C6[k] * P[k].mn;
        cn += C6[k] * (P[k].mn * unk + P[k].p);
        cE += C6[k] * ((P[k].E + P[k].p) * unk);
        dr += D6[k] * P[k].r;
        dn += D6[k] * P[k].mn;
        dE += D6[k] * P[k].E;
#pragma unroll
        for (int s = 0; s < NT; ++s) {
            ct[s] += C6[k] * (P[k].mt[s] * unk);
            dt[s] += D6[k] * P[k].mt[s];
        }
    }
    double um = un * dn;
#pragma unroll
    for (int s = 0; s < NT; ++s) um += ut[s] * dt[s];
    const double A = b * (K * dr - um + dE);
    const double B = (un * dr - dn) * ia;
    const double v0 = aminus * 0.5 * (A + B);
    const double v4 = aplus * 0.5 * (A - B);
    const double v1 = a0 * (dr - A);
    const double hs = v0 + v1 + v4, hd = v4 - v0;
    Fr = cr + hs;
    Fn = cn + un * hs + ah * hd;
    FE = cE + Hh * (v0 + v4) + ah * un * hd + K * v1;
#pragma unroll
    for (int s = 0; s < NT; ++s) {
        const double vt = a0 * (dt[s] - ut[s] * dr);
        Ft[s] = ct[s] + ut[s] * hs + vt;
        FE += ut[s] * vt;
    }
}

// the cheap flux on FP32 deviations from the FP64 flux of node i
// (C6 sums to 1 and D6 to 0, so F = f_ref + C6 (f - f_ref) + R alpha L D6 (U - U_i))
template <int ND>
__device__ __forceinline__ void cheap_flux_mixed(const Loc<ND> (&P)[6], const Phys &ph, double &Fr, double &Fn,
                                                 double (&Ft)[2], double &FE) {
    constexpr int NT = ND - 1;
    constexpr float C6[6] = {1.0f / 60.0f, -8.0f / 60.0f, 37.0f / 60.0f, 37.0f / 60.0f, -8.0f / 60.0f, 1.0f / 60.0f};
    constexpr float D6[6] = {1.0f / 60.0f, -5.0f / 60.0f, 10.0f / 60.0f, -10.0f / 60.0f, 5.0f / 60.0f, -1.0f / 60.0f};
    double un64[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) un64[k] = P[k].mn * P[k].ri;
    const double fr0 = P[2].mn;
    const double fn0 = P[2].mn * un64[2] + P[2].p;
    double ft0[2] = {0.0, 0.0};
#pragma unroll
    for (int s = 0; s < NT; ++s) ft0[s] = P[2].mt[s] * un64[2];
    const double fE0 = (P[2].E + P[2].p) * un64[2];
    float sl = 1.0f, sr = 1.0f;
    if (ph.roe) {
        sl = sqrtf((float)P[2].r);
        sr = sqrtf((float)P[3].r);
    }
    const float iw = rcpf(sl + sr);
    const float un = (sl * (float)un64[2] + sr * (float)un64[3]) * iw;
    float ut[2] = {0.0f, 0.0f};
#pragma unroll
    for (int s = 0; s < NT; ++s)
        ut[s] = (sl * (float)(P[2].mt[s] * P[2].ri) + sr * (float)(P[3].mt[s] * P[3].ri)) * iw;
    const float Hh = (sl * (float)((P[2].E + P[2].p) * P[2].ri) + sr * (float)((P[3].E + P[3].p) * P[3].ri)) * iw;
    float K = un * un;
#pragma unroll
    for (int s = 0; s < NT; ++s) K += ut[s] * ut[s];
    K *= 0.5f;
    const float gm1 = (float)ph.gm1;
    const float ah = sqrtf(gm1 * (Hh - K));
    const float ia = rcpf(ah);
    const float b = gm1 * ia * ia;
    float aminus = 0.0f, aplus = 0.0f, a0 = 0.0f;
    float cr = 0.0f, cn = 0.0f, ct[2] = {0.0f, 0.0f}, cE = 0.0f;
    float dr = 0.0f, dn = 0.0f, dt[2] = {0.0f, 0.0f}, dE = 0.0f;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        const float unk = (float)un64[k], ak = (float)P[k].a;
        aminus = fmaxf(aminus, fabsf(unk - ak));
        aplus = fmaxf(aplus, fabsf(unk + ak));
        a0 = fmaxf(a0, fabsf(unk));
        cr += C6[k] * (float)(P[k].mn - fr0);
        cn += C6[k] * (float)(P[k].mn * un64[k] + P[k].p - fn0);
        cE += C6[k] * (float)((P[k].E + P[k].p) * un64[k] - fE0);
        dr += D6[k] * (float)(P[k].r - P[2].r);
        dn += D6[k] * (float)(P[k].mn - P[2].mn);
        dE += D6[k] * (float)(P[k].E - P[2].E);
#pragma unroll
        for (int s = 0; s < NT; ++s) {
            ct[s] += C6[k] * (float)(P[k].mt[s] * un64[k] - ft0[s]);
            dt[s] += D6[k] * (float)(P[k].mt[s] - P[2].mt[s]);
        }
    }
    float um = un * dn;
#pragma unroll
    for (int s = 0; s < NT; ++s) um += ut[s] * dt[s];
    const float A = b * (K * dr - um + dE);
    const float B = (un * dr - dn) * ia;
    const float v0 = aminus * 0.5f * (A + B);
    const float v4 = aplus * 0.5f * (A - B);
    const float v1 = a0 * (dr - A);
    const float hs = v0 + v1 + v4, hd = v4 - v0;
    float dFE = cE + Hh * (v0 + v4) + ah * un * hd + K * v1;
    Fr = fr0 + (double)(cr + hs);
    Fn = fn0 + (double)(cn + un * hs + ah * hd);
#pragma unroll
    for (int s = 0; s < NT; ++s) {
        const float vt = a0 * (dt[s] - ut[s] * dr);
        Ft[s] = ft0[s] + (double)(ct[s] + ut[s] * hs + vt);
        dFE += ut[s] * vt;
    }
    FE = fE0 + (double)dFE;
}

}  // namespace cf
}  // namespace osbli
