// Convective residual: characteristic LLF flux reconstruction (WENO-Z5 or
// TENO5) in each direction, section 2.2 (enumerated algorithm), sections
// 2.3-2.5 for the reconstructions.
//
// Thread mapping ("pencil march"): a thread owns one grid line along the sweep
// direction and a segment of it; neighbouring lanes own neighbouring lines
// (adjacent in x for the y and z sweeps, so every load is coalesced).  Each
// thread keeps a six-point register window of the stencil (state + 1/rho, p,
// a computed once per point), marches along the line, computes one interface
// flux per step and the flux difference of the node behind it, so each
// interface is evaluated once (plus one per segment).
//
// The characteristic algebra is written in the local frame (n, t1, t2) of the
// interface: with f_k = u_n U_k + p_k (0, n, u_n) the projected flux is
// g_kj = u_n,k V_kj + p_k (l_j,m . n + l_j,E u_n,k), so only V = L U is
// formed per point, and L, R are never stored as matrices.
#include "internal.hpp"

namespace osbli {
namespace {

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
    const double ri = 1.0 / w.U[0];
    double ke = 0.0;
#pragma unroll
    for (int m = 0; m < ND; ++m) ke += w.U[1 + m] * w.U[1 + m];
    const double p = ph.gm1 * (w.U[ND + 1] - 0.5 * ke * ri);
    w.ri = ri;
    w.p = p;
    w.a = sqrt(ph.gamma * p * ri);
    bad |= !(w.U[0] > 0.0 && p > 0.0);
}

// Fifth-order WENO-Z / TENO reconstruction at x_{i+1/2} from f_{i-2..i+2}.
// Candidate stencils S_r = {i-r .. i-r+2}, Jiang-Shu indicators,
// tau_5 = |beta_0 - beta_2|; WENO-Z alpha_r = d_r (1 + (tau/(beta_r+eps))^2);
// TENO gamma_r = (1 + tau/(beta_r+eps))^6, stencil r cut when
// gamma_r / sum(gamma) < C_T (evaluated as gamma_r < C_T * sum), weights
// d_r delta_r / sum(d delta).  The three ratios tau/(beta_r+eps) share one
// reciprocal of the product of the denominators; TENO's normalisation is a
// reciprocal of one of seven sums of optimal weights, skipped when no
// stencil is cut (sum = 1).
template <int SCHEME>
__device__ __forceinline__ double recon5(double fm2, double fm1, double f0, double fp1, double fp2,
                                         double CT, double eps) {
    const double q0 = (1.0 / 3.0) * f0 + (5.0 / 6.0) * fp1 - (1.0 / 6.0) * fp2;
    const double q1 = -(1.0 / 6.0) * fm1 + (5.0 / 6.0) * f0 + (1.0 / 3.0) * fp1;
    const double q2 = (1.0 / 3.0) * fm2 - (7.0 / 6.0) * fm1 + (11.0 / 6.0) * f0;
    double s, t;
    s = f0 - 2.0 * fp1 + fp2;
    t = 3.0 * f0 - 4.0 * fp1 + fp2;
    const double b0 = (13.0 / 12.0) * s * s + 0.25 * t * t;
    s = fm1 - 2.0 * f0 + fp1;
    t = fm1 - fp1;
    const double b1 = (13.0 / 12.0) * s * s + 0.25 * t * t;
    s = fm2 - 2.0 * fm1 + f0;
    t = fm2 - 4.0 * fm1 + 3.0 * f0;
    const double b2 = (13.0 / 12.0) * s * s + 0.25 * t * t;
    const double tau = fabs(b0 - b2);
    const double e0 = b0 + eps, e1 = b1 + eps, e2 = b2 + eps;
    const double e01 = e0 * e1;
    const double tinv = tau / (e01 * e2);
    const double x0 = (e1 * e2) * tinv, x1 = (e0 * e2) * tinv, x2 = e01 * tinv;
    if (SCHEME == OSBLI_WENOZ5) {
        const double a0 = 0.3 * (1.0 + x0 * x0);
        const double a1 = 0.6 * (1.0 + x1 * x1);
        const double a2 = 0.1 * (1.0 + x2 * x2);
        return (a0 * q0 + a1 * q1 + a2 * q2) / (a0 + a1 + a2);
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
        const double num = w0 * q0 + w1 * q1 + w2 * q2;
        if (k0 && k1 && k2) return num;
        return num / (w0 + w1 + w2);
    }
}

// LLF split of one characteristic field over the six points and the two
// reconstructions: ghat = recon+(g+_{i-2..i+2}) + recon-(g-_{i+3..i-1}).
template <int SCHEME>
__device__ __forceinline__ double split_recon(const double (&V)[6], const double (&g)[6], double alpha,
                                              const Phys &ph) {
    double gp[6], gm[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        gp[k] = 0.5 * (g[k] + alpha * V[k]);
        gm[k] = 0.5 * (g[k] - alpha * V[k]);
    }
    return recon5<SCHEME>(gp[0], gp[1], gp[2], gp[3], gp[4], ph.CT, ph.eps) +
           recon5<SCHEME>(gm[5], gm[4], gm[3], gm[2], gm[1], ph.CT, ph.eps);
}

// Interface flux in the local frame (unit |S|).  Outputs: mass, normal
// momentum, tangential momenta, energy.
template <int ND, int SCHEME>
__device__ __forceinline__ void char_flux(const Loc<ND> (&P)[6], const Phys &ph, double &Fr, double &Fn,
                                          double (&Ft)[2], double &FE) {
    constexpr int NT = ND - 1;  // tangents
    // averaged state at the half node (Roe, or arithmetic mean with unit weights)
    double sl = 1.0, sr = 1.0;
    if (ph.roe) {
        sl = sqrt(P[2].r);
        sr = sqrt(P[3].r);
    }
    const double iw = 1.0 / (sl + sr);
    const double un = (sl * (P[2].mn * P[2].ri) + sr * (P[3].mn * P[3].ri)) * iw;
    double ut[2] = {0.0, 0.0};
#pragma unroll
    for (int s = 0; s < NT; ++s) ut[s] = (sl * (P[2].mt[s] * P[2].ri) + sr * (P[3].mt[s] * P[3].ri)) * iw;
    const double Hh = (sl * ((P[2].E + P[2].p) * P[2].ri) + sr * ((P[3].E + P[3].p) * P[3].ri)) * iw;
    double K = un * un;
#pragma unroll
    for (int s = 0; s < NT; ++s) K += ut[s] * ut[s];
    K *= 0.5;
    const double ah = sqrt(ph.gm1 * (Hh - K));
    const double ia = 1.0 / ah;
    const double b = ph.gm1 * ia * ia;

    double unk[6], A[6], B[6], am[6], ap[6], a0 = 0.0;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        unk[k] = P[k].mn * P[k].ri;
        double um = un * P[k].mn;
#pragma unroll
        for (int s = 0; s < NT; ++s) um += ut[s] * P[k].mt[s];
        A[k] = b * (K * P[k].r - um + P[k].E);
        B[k] = (un * P[k].r - P[k].mn) * ia;
        am[k] = fabs(unk[k] - P[k].a);
        ap[k] = fabs(unk[k] + P[k].a);
        a0 = fmax(a0, fabs(unk[k]));
    }
    double aminus = am[0], aplus = ap[0];
#pragma unroll
    for (int k = 1; k < 6; ++k) {
        aminus = fmax(aminus, am[k]);
        aplus = fmax(aplus, ap[k]);
    }
    double V[6], g[6];
    // field u_n - a
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        V[k] = 0.5 * (A[k] + B[k]);
        g[k] = unk[k] * V[k] + P[k].p * (0.5 * b * unk[k] - 0.5 * (b * un + ia));
    }
    const double h0 = split_recon<SCHEME>(V, g, aminus, ph);
    // field u_n + a
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        V[k] = 0.5 * (A[k] - B[k]);
        g[k] = unk[k] * V[k] + P[k].p * (0.5 * b * unk[k] - 0.5 * (b * un - ia));
    }
    const double h4 = split_recon<SCHEME>(V, g, aplus, ph);
    // entropy field
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        V[k] = P[k].r - A[k];
        g[k] = unk[k] * V[k] + P[k].p * (b * (un - unk[k]));
    }
    const double h1 = split_recon<SCHEME>(V, g, a0, ph);
    // shear fields
    double ht[2] = {0.0, 0.0};
#pragma unroll
    for (int s = 0; s < NT; ++s) {
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            V[k] = P[k].mt[s] - ut[s] * P[k].r;
            g[k] = unk[k] * V[k];
        }
        ht[s] = split_recon<SCHEME>(V, g, a0, ph);
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
__device__ __forceinline__ float recon5f(float fm2, float fm1, float f0, float fp1, float fp2, float CT, float eps) {
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
                                              float eps) {
    float gp[6], gm[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        gp[k] = 0.5f * (G[k] + alpha * V[k]);
        gm[k] = 0.5f * (G[k] - alpha * V[k]);
    }
    return recon5f<SCHEME>(gp[0], gp[1], gp[2], gp[3], gp[4], CT, eps) +
           recon5f<SCHEME>(gm[5], gm[4], gm[3], gm[2], gm[1], CT, eps);
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
    const float CT = (float)ph.CT, eps = (float)ph.eps;

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
    const float h0 = split_reconf<SCHEME>(V, G, aminus, CT, eps);
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        V[k] = 0.5f * (A[k] - B[k]);
        G[k] = 0.5f * (Ag[k] - Bg[k]);
    }
    const float h4 = split_reconf<SCHEME>(V, G, aplus, CT, eps);
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        V[k] = dr[k] - A[k];
        G[k] = gr[k] - Ag[k];
    }
    const float h1 = split_reconf<SCHEME>(V, G, a0, CT, eps);
    float ht[2] = {0.0f, 0.0f};
#pragma unroll
    for (int s = 0; s < NT; ++s) {
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            V[k] = dmt[s][k] - ut[s] * dr[k];
            G[k] = gmt[s][k] - ut[s] * gr[k];
        }
        ht[s] = split_reconf<SCHEME>(V, G, a0, CT, eps);
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

template <int ND, int DIR>
struct Axes {
    static constexpr int T1 = (DIR + 1) % ND;
    static constexpr int T2 = (DIR + 2) % ND;
};

constexpr int kChunk = 8;   // x-points staged per cooperative load (x sweep)
constexpr int kWaves = 4;   // waves per block

// One convective sweep along DIR.  first != 0: R = contribution, else R +=.
// Thread mapping: every wave owns 64 consecutive lines and one segment
// [p0, p1) along DIR (wave-uniform), lane l owns line line0 + l.  Along y and
// z the lanes' loads are contiguous in x.  Along x the lines are strided, so
// the wave stages chunks of kChunk points of its 64 rows through LDS with
// contiguous loads and each lane reads its own row back.
template <int ND, int DIR, int SCHEME, bool GEN, bool MIX>
__global__ void __launch_bounds__(256)
k_sweep(const double *__restrict__ U, double *__restrict__ R, Grid g, Phys ph, Metrics m, int64_t seg,
        int64_t nseg, int first, unsigned *flags) {
    constexpr int NC = ND + 2;
    constexpr int NT = ND - 1;
    constexpr int O1 = DIR == 0 ? 1 : 0;
    constexpr int O2 = DIR == 2 ? 1 : 2;
    const int64_t n1 = g.n[O1], n2 = g.n[O2], N = g.n[DIR];
    const int64_t lines = n1 * n2;
    const int64_t wpl = (lines + 63) >> 6;  // waves per segment
    const int lane = threadIdx.x & 63;
    const int64_t gw = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t sg = gw / wpl;
    if (sg >= nseg) return;  // wave-uniform
    const int64_t line0 = (gw - sg * wpl) << 6;
    const int64_t line = line0 + lane;
    const bool active = line < lines;
    const int64_t lc = active ? line : lines - 1;
    const int64_t p0 = sg * seg;
    const int64_t p1 = p0 + seg < N ? p0 + seg : N;
    int64_t q[3];
    q[DIR] = 0;
    q[O1] = lc % n1;
    q[O2] = lc / n1;
    const int64_t base = ext_index(g, q[0], q[1], q[2]);
    const int64_t st = g.es[DIR];
    const int64_t cs = g.enpts;
    const int64_t ibase = int_index(g, q[0], q[1], q[2]);
    const int64_t ist = g.is[DIR];
    bool bad = false;

    // x sweep staging buffer: [wave][component][chunk point][row]
    __shared__ double sbuf[DIR == 0 ? kWaves : 1][DIR == 0 ? NC : 1][DIR == 0 ? kChunk : 1][64];
    const int wv = DIR == 0 ? (threadIdx.x >> 6) : 0;
    int64_t cbase = p0 - 3 - kChunk;  // first point held in the chunk buffer
    // point q's conserved state into w (from LDS along x, directly otherwise)
    auto fetch = [&](int64_t qp, Pt<ND> &w) {
        if (DIR == 0) {
            if (qp >= cbase + kChunk) {
                cbase = qp;
                const int64_t last = N + kGhost - 1;
#pragma unroll
                for (int s2 = 0; s2 < kChunk; ++s2) {
                    const int e = lane + 64 * s2;
                    const int r = e / kChunk, x = e % kChunk;
                    int64_t rl = line0 + r;
                    if (rl >= lines) rl = lines - 1;
                    const int64_t rb = ext_index(g, 0, rl % n1, rl / n1);
                    int64_t xp = qp + x;
                    if (xp > last) xp = last;
#pragma unroll
                    for (int c = 0; c < NC; ++c) sbuf[wv][c][x][r] = U[rb + xp + c * cs];
                }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            }
            const int xi = (int)(qp - cbase);
#pragma unroll
            for (int c = 0; c < NC; ++c) w.U[c] = sbuf[wv][c][xi][lane];
        } else {
#pragma unroll
            for (int c = 0; c < NC; ++c) w.U[c] = U[base + qp * st + c * cs];
        }
        finish_point<ND>(ph, w, bad);
    };

    Pt<ND> w[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) fetch(p0 - 3 + k, w[k]);

    // general meshes: node area vectors S_DIR at f-1 .. f+2 for interface f+1/2
    double Sw[4][3];
    if (GEN) {
#pragma unroll
        for (int k = 0; k < 4; ++k)
#pragma unroll
            for (int c = 0; c < ND; ++c)
                Sw[k][c] = m.S[(DIR * ND + c) * cs + base + (p0 - 2 + k) * st];
    }

    double Fp[NC];
    for (int64_t f = p0 - 1; f < p1; ++f) {
        if (f >= p0) {
#pragma unroll
            for (int k = 0; k < 5; ++k) w[k] = w[k + 1];
            fetch(f + 3, w[5]);
            if (GEN) {
#pragma unroll
                for (int k = 0; k < 3; ++k)
#pragma unroll
                    for (int c = 0; c < ND; ++c) Sw[k][c] = Sw[k + 1][c];
#pragma unroll
                for (int c = 0; c < ND; ++c) Sw[3][c] = m.S[(DIR * ND + c) * cs + base + (f + 2) * st];
            }
        }
        Loc<ND> P[6];
        double F[NC];
        double Smag = 1.0;
        double nv[3] = {0.0, 0.0, 0.0}, t1[3] = {0.0, 0.0, 0.0}, t2[3] = {0.0, 0.0, 0.0};
        if (!GEN) {
#pragma unroll
            for (int k = 0; k < 6; ++k) {
                P[k].r = w[k].U[0];
                P[k].mn = w[k].U[1 + DIR];
                if (NT >= 1) P[k].mt[0] = w[k].U[1 + Axes<ND, DIR>::T1];
                if (NT >= 2) P[k].mt[1] = w[k].U[1 + Axes<ND, DIR>::T2];
                P[k].E = w[k].U[ND + 1];
                P[k].p = w[k].p;
                P[k].a = w[k].a;
                P[k].ri = w[k].ri;
            }
        } else {
            double Sh[3] = {0.0, 0.0, 0.0};
            double s2 = 0.0;
#pragma unroll
            for (int c = 0; c < ND; ++c) {
                Sh[c] = (-Sw[0][c] + 7.0 * Sw[1][c] + 7.0 * Sw[2][c] - Sw[3][c]) / 12.0;
                s2 += Sh[c] * Sh[c];
            }
            Smag = sqrt(s2);
#pragma unroll
            for (int c = 0; c < ND; ++c) nv[c] = Sh[c] / Smag;
            // tangent basis: t1 = normalise(e_{DIR+1} - (e_{DIR+1}.n) n), t2 = n x t1
            if (ND >= 2) {
                constexpr int TE = (DIR + 1) % (ND > 1 ? ND : 1);
                const double en = nv[TE];
                double tn = 0.0;
#pragma unroll
                for (int c = 0; c < ND; ++c) {
                    t1[c] = (c == TE ? 1.0 : 0.0) - en * nv[c];
                    tn += t1[c] * t1[c];
                }
                tn = sqrt(tn);
#pragma unroll
                for (int c = 0; c < ND; ++c) t1[c] /= tn;
                if (ND == 3) {
                    t2[0] = nv[1] * t1[2] - nv[2] * t1[1];
                    t2[1] = nv[2] * t1[0] - nv[0] * t1[2];
                    t2[2] = nv[0] * t1[1] - nv[1] * t1[0];
                }
            }
#pragma unroll
            for (int k = 0; k < 6; ++k) {
                double mn = 0.0, m1 = 0.0, m2 = 0.0;
#pragma unroll
                for (int c = 0; c < ND; ++c) {
                    mn += w[k].U[1 + c] * nv[c];
                    m1 += w[k].U[1 + c] * t1[c];
                    m2 += w[k].U[1 + c] * t2[c];
                }
                P[k].r = w[k].U[0];
                P[k].mn = mn;
                P[k].mt[0] = m1;
                P[k].mt[1] = m2;
                P[k].E = w[k].U[ND + 1];
                P[k].p = w[k].p;
                P[k].a = w[k].a;
                P[k].ri = w[k].ri;
            }
        }
        double Fr, Fn, Ft[2], FE;
        if (MIX) char_flux_mixed<ND, SCHEME>(P, ph, Fr, Fn, Ft, FE);
        else char_flux<ND, SCHEME>(P, ph, Fr, Fn, Ft, FE);
        F[0] = Fr * Smag;
        F[NC - 1] = FE * Smag;
        if (!GEN) {
            F[1 + DIR] = Fn;
            if (NT >= 1) F[1 + Axes<ND, DIR>::T1] = Ft[0];
            if (NT >= 2) F[1 + Axes<ND, DIR>::T2] = Ft[1];
        } else {
#pragma unroll
            for (int c = 0; c < ND; ++c) {
                double v = Fn * nv[c];
                if (NT >= 1) v += Ft[0] * t1[c];
                if (NT >= 2) v += Ft[1] * t2[c];
                F[1 + c] = v * Smag;
            }
        }
        if (f >= p0 && active) {
            const double sc = GEN ? m.J[base + f * st] : m.invh[DIR][f];
            const int64_t oi = ibase + f * ist;
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                const double v = -sc * (F[c] - Fp[c]);
                double *dst = R + c * g.nint + oi;
                if (first) *dst = v;
                else *dst += v;
            }
        }
#pragma unroll
        for (int c = 0; c < NC; ++c) Fp[c] = F[c];
    }
    if (bad) atomicOr(flags, kFlagNonPhys);
}

template <int ND, int DIR, int SCHEME, bool GEN, bool MIX>
hipError_t launch_one(const Grid &g, const Phys &ph, const Metrics &m, const double *U, double *R,
                      unsigned *flags, int first, hipStream_t s) {
    constexpr int O1 = DIR == 0 ? 1 : 0;
    constexpr int O2 = DIR == 2 ? 1 : 2;
    const int64_t lines = g.n[O1] * g.n[O2];
    const int64_t N = g.n[DIR];
    const int64_t target = int64_t(1) << 18;  // threads in flight to aim for
    int64_t seg = (N * lines + target - 1) / target;
    if (seg < 8) seg = 8;
    if (seg > N) seg = N;
    const int64_t nseg = (N + seg - 1) / seg;
    const int64_t waves = ((lines + 63) / 64) * nseg;
    const int bs = 64 * kWaves;
    const int64_t nb = (waves + kWaves - 1) / kWaves;
    hipLaunchKernelGGL((k_sweep<ND, DIR, SCHEME, GEN, MIX>), dim3((unsigned)nb), dim3(bs), 0, s, U, R, g, ph, m,
                       seg, nseg, first, flags);
    return hipGetLastError();
}

template <int ND, int SCHEME, bool GEN, bool MIX>
hipError_t launch_dir_f(const Grid &g, const Phys &ph, const Metrics &m, const double *U, double *R,
                        unsigned *flags, int dir, int first, hipStream_t s) {
    if (dir == 0) return launch_one<ND, 0, SCHEME, GEN, MIX>(g, ph, m, U, R, flags, first, s);
    if (dir == 1) return launch_one<ND, (ND >= 2 ? 1 : 0), SCHEME, GEN, MIX>(g, ph, m, U, R, flags, first, s);
    return launch_one<ND, (ND >= 3 ? 2 : 0), SCHEME, GEN, MIX>(g, ph, m, U, R, flags, first, s);
}

template <int ND, int SCHEME, bool GEN>
hipError_t launch_dir(const Grid &g, const Phys &ph, const Metrics &m, const double *U, double *R,
                      unsigned *flags, int dir, int first, hipStream_t s) {
    if (ph.mixed) return launch_dir_f<ND, SCHEME, GEN, true>(g, ph, m, U, R, flags, dir, first, s);
    return launch_dir_f<ND, SCHEME, GEN, false>(g, ph, m, U, R, flags, dir, first, s);
}

template <int ND, int SCHEME>
hipError_t launch_mesh(const Grid &g, const Phys &ph, const Metrics &m, const double *U, double *R,
                       unsigned *flags, int dir, int first, hipStream_t s) {
    if (ND >= 2 && m.general) return launch_dir<ND, SCHEME, (ND >= 2)>(g, ph, m, U, R, flags, dir, first, s);
    return launch_dir<ND, SCHEME, false>(g, ph, m, U, R, flags, dir, first, s);
}

template <int ND>
hipError_t launch_scheme(const Grid &g, const Phys &ph, const Metrics &m, const double *U, double *R,
                         unsigned *flags, int dir, int first, hipStream_t s) {
    if (ph.scheme == OSBLI_WENOZ5) return launch_mesh<ND, OSBLI_WENOZ5>(g, ph, m, U, R, flags, dir, first, s);
    return launch_mesh<ND, OSBLI_TENO5>(g, ph, m, U, R, flags, dir, first, s);
}

}  // namespace

hipError_t launch_convective(const Grid &g, const Phys &ph, const Metrics &m, const double *U, double *R,
                             unsigned *flags, int dir, int first, hipStream_t s) {
    if (dir < 0 || dir >= g.nd) return hipErrorInvalidValue;
    switch (g.nd) {
        case 1: return launch_scheme<1>(g, ph, m, U, R, flags, dir, first, s);
        case 2: return launch_scheme<2>(g, ph, m, U, R, flags, dir, first, s);
        default: return launch_scheme<3>(g, ph, m, U, R, flags, dir, first, s);
    }
}

}  // namespace osbli
