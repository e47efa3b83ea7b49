// Device code of the learned sensor shared by the single-grid and the
// batched launches: interface features, the bfloat16 MFMA network and the
// per-interface routing decision.  Arithmetic that decides a route is written
// without FMA contraction so that every translation unit agrees bit for bit.
#pragma once

#include "internal.hpp"

namespace osbli {
namespace sn {

constexpr int kIn = 10, kH = 32;
constexpr int oW1 = 0, oB1 = 320, oW2 = 352, oB2 = 1376, oW3 = 1408, oB3 = 1440;
constexpr int kNP = 1441;
constexpr int kNPad = 1442;  // partial record: 1441 gradients + loss

__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float(((unsigned)b) << 16); }
__device__ __forceinline__ uint16_t f2bf(float x) {  // round to nearest even (v_cvt_pk_bf16_f32)
    const __bf16 b = (__bf16)x;
    uint16_t u;
    __builtin_memcpy(&u, &b, sizeof u);
    return u;
}

// ------------------------------------------------------------ features
// Features 0..3 of interface p+1/2: three-point Jiang-Shu indicators of
// rho/rho_bar + p/p_bar + u_t/a_bar on the four substencils of p-2..p+3
// (each variable's indicator on unscaled values times the inverse square of
// its scale), over their sum + 1e-20; 4..9: log10(1 + 1e6 J)/6 of the rho
// and p jumps J = |q_{k+1} - q_k| / (q_{k+1} + q_k) over (p-1,p), (p,p+1),
// (p+1,p+2).  The FP64 operations follow the definition's order without FMA
// contraction, so every kernel (per interface, marching, batched) computes
// the same features.

// density, pressure and tangential velocities of one point
template <int ND>
struct SPoint {
    double r, p, vt[2];
};

template <int ND, int DIR>
__device__ __forceinline__ void spoint(const double *__restrict__ U, int64_t e, int64_t cs, const Phys &ph,
                                       SPoint<ND> &o) {
#pragma clang fp contract(off)
    const double r = U[e];
    double u[3], ke = 0.0;
#pragma unroll
    for (int m = 0; m < ND; ++m) {
        u[m] = U[e + (1 + m) * cs] / r;
        ke += u[m] * u[m];
    }
    o.r = r;
    o.p = ph.gm1 * (U[e + (ND + 1) * cs] - 0.5 * r * ke);
#pragma unroll
    for (int s = 0; s < ND - 1; ++s) o.vt[s] = u[(DIR + 1 + s) % ND];
}

__device__ __forceinline__ double js3v(double a, double b, double c) {
#pragma clang fp contract(off)
    const double a1 = a - 2.0 * b + c, a2 = a - c;
    return (13.0 / 12.0) * a1 * a1 + 0.25 * a2 * a2;
}

// indicators of one substencil (first point k): rho, p, tangential velocities
template <int ND>
struct STriple {
    double br, bp, bv[2];
};

template <int ND>
__device__ __forceinline__ void striple(const SPoint<ND> &a, const SPoint<ND> &b, const SPoint<ND> &c,
                                        STriple<ND> &o) {
    o.br = js3v(a.r, b.r, c.r);
    o.bp = js3v(a.p, b.p, c.p);
#pragma unroll
    for (int s = 0; s < ND - 1; ++s) o.bv[s] = js3v(a.vt[s], b.vt[s], c.vt[s]);
}

// log-normalised rho and p jumps between two points (inputs of a bfloat16
// network: the logarithm is taken in FP32)
template <int ND>
__device__ __forceinline__ void sjump(const SPoint<ND> &a, const SPoint<ND> &b, float &lr, float &lp) {
#pragma clang fp contract(off)
    const double jr = fabs(b.r - a.r) / (b.r + a.r);
    const double jp = fabs(b.p - a.p) / (b.p + a.p);
    lr = log10f((float)(1.0 + 1e6 * jr)) * (1.0f / 6.0f);
    lp = log10f((float)(1.0 + 1e6 * jp)) * (1.0f / 6.0f);
}

// the ten features from the two middle points, the four substencils'
// indicators and the three jumps
template <int ND>
__device__ __forceinline__ void sfeatures(const SPoint<ND> &m2, const SPoint<ND> &m3, const STriple<ND> (&T)[4],
                                          const float (&lr)[3], const float (&lp)[3], const Phys &ph,
                                          float (&f)[kIn]) {
#pragma clang fp contract(off)
    const double rb = 0.5 * (m2.r + m3.r), pb = 0.5 * (m2.p + m3.p);
    const double sr = 1.0 / (rb * rb), sp = 1.0 / (pb * pb), sv = rb / (ph.gamma * pb);
    double beta[4], sum = 0.0;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        double b = sr * T[m].br + sp * T[m].bp;
#pragma unroll
        for (int s = 0; s < ND - 1; ++s) b += sv * T[m].bv[s];
        beta[m] = b;
        sum += b;
    }
    const double inv = 1.0 / (sum + 1e-20);
#pragma unroll
    for (int m = 0; m < 4; ++m) f[m] = (float)(beta[m] * inv);
#pragma unroll
    for (int m = 0; m < 3; ++m) {
        f[4 + m] = lr[m];
        f[7 + m] = lp[m];
    }
}

// features of interface p+1/2 of a line (separable meshes: n = e_DIR,
// tangents e_{DIR+1}, e_{DIR+2}); stencil points p-2..p+3 start at ext
// index e0 with stride st
template <int ND, int DIR>
__device__ __forceinline__ void features(const double *__restrict__ U, int64_t e0, int64_t st, int64_t cs,
                                         const Phys &ph, float (&f)[kIn]) {
    SPoint<ND> P[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) spoint<ND, DIR>(U, e0 + k * st, cs, ph, P[k]);
    STriple<ND> T[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) striple<ND>(P[m], P[m + 1], P[m + 2], T[m]);
    float lr[3], lp[3];
#pragma unroll
    for (int m = 0; m < 3; ++m) sjump<ND>(P[m + 1], P[m + 2], lr[m], lp[m]);
    sfeatures<ND>(P[2], P[3], T, lr, lp, ph, f);
}

// interface grid of direction d: extent n_d + 1 along d (position p = index - 1)
struct IfaceGrid {
    int64_t E[3], total;
};
__host__ __device__ inline IfaceGrid iface_grid(const Grid &g, int d) {
    IfaceGrid I;
    for (int e = 0; e < 3; ++e) I.E[e] = g.n[e] + (e == d ? 1 : 0);
    I.total = I.E[0] * I.E[1] * I.E[2];
    return I;
}

// ------------------------------------------------------ MFMA inference
typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16;

// Network on the matrix cores, v_mfma_f32_32x32x16_bf16, computed transposed
// (hidden units as rows, 32 samples of the wave as columns) so that each
// layer's accumulators are the next layer's operands without leaving the
// registers.  Operand layouts (lane l, h = l / 32): A holds row l % 32 at
// K = 8h .. 8h+7; B holds column l % 32 at K = 8h .. 8h+7; D register r holds
// row 8 (r / 4) + 4h + r % 4 of column l % 32.  The second layer sums over
// the hidden units in the order the first layer's D registers hold them
// (a permutation of the summation index, applied to W2 as well).
__device__ __forceinline__ int drow(int r, int h) { return 8 * (r >> 2) + 4 * h + (r & 3); }

struct MlpFrag {
    bf16x8 w1;        // W1^T rows: W1[8h + i][l % 32]
    bf16x8 w2[2];     // W2^T rows, summation index in D-register order
    float b1[16], b2[16], w3[16];  // per D register of this lane half
    float b3;
};

__device__ __forceinline__ bf16x8 pack8(const uint16_t (&u)[8]) {
    bf16x8 v;
    __builtin_memcpy(&v, u, sizeof v);
    return v;
}

__device__ __forceinline__ void load_frag(const uint16_t *__restrict__ w, int lane, MlpFrag &F) {
    const int j = lane & 31, h = lane >> 5;
    uint16_t u[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) u[i] = (8 * h + i < kIn) ? w[oW1 + (8 * h + i) * kH + j] : (uint16_t)0;
    F.w1 = pack8(u);
#pragma unroll
    for (int ks = 0; ks < 2; ++ks) {
#pragma unroll
        for (int i = 0; i < 8; ++i) u[i] = w[oW2 + drow(8 * ks + i, h) * kH + j];
        F.w2[ks] = pack8(u);
    }
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        F.b1[r] = bf2f(w[oB1 + drow(r, h)]);
        F.b2[r] = bf2f(w[oB2 + drow(r, h)]);
        F.w3[r] = bf2f(w[oW3 + drow(r, h)]);
    }
    F.b3 = bf2f(w[oB3]);
}

// LDS writes of this wave visible to its other lanes
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ int bf16pair(float a, float b) { return (int)f2bf(a) | ((int)f2bf(b) << 16); }

// logit of the lane's own sample; every lane of the wave must call it.
// Inputs and hidden activations are rounded to bfloat16 (the operands),
// accumulation is FP32.
__device__ __forceinline__ float mlp_mfma(const float (&x)[kIn], const MlpFrag &F, int lane) {
#pragma clang fp contract(off)
    const int h = lane >> 5;
    // columns of tile t are the samples of lanes 32 t .. 32 t + 31: a lane
    // supplies its own features 8h .. 8h+7 to its own tile and receives
    // those of lane l ^ 32 for the other tile
    int own[4], give[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int k0 = 2 * q, k1 = 2 * q + 1;
        const float lo0 = x[k0], lo1 = x[k1];
        const float hi0 = 8 + k0 < kIn ? x[(8 + k0) % kIn] : 0.0f, hi1 = 8 + k1 < kIn ? x[(8 + k1) % kIn] : 0.0f;
        own[q] = h == 0 ? bf16pair(lo0, lo1) : bf16pair(hi0, hi1);
        give[q] = h == 0 ? bf16pair(hi0, hi1) : bf16pair(lo0, lo1);
    }
    int b0[4], b1[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int got = __shfl_xor(give[q], 32, 64);
        b0[q] = h == 0 ? own[q] : got;
        b1[q] = h == 0 ? got : own[q];
    }
    bf16x8 B[2];
    __builtin_memcpy(&B[0], b0, sizeof(bf16x8));
    __builtin_memcpy(&B[1], b1, sizeof(bf16x8));
    float part[2];
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        const f32x16 zero = {0};
        const f32x16 d1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(F.w1, B[t], zero, 0, 0, 0);
        uint16_t a0[8], a1[8];
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            a0[r] = f2bf(fmaxf(d1[r] + F.b1[r], 0.0f));
            a1[r] = f2bf(fmaxf(d1[8 + r] + F.b1[8 + r], 0.0f));
        }
        f32x16 d2 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(F.w2[0], pack8(a0), zero, 0, 0, 0);
        d2 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(F.w2[1], pack8(a1), d2, 0, 0, 0);
        float p = 0.0f;
#pragma unroll
        for (int r = 0; r < 16; ++r) p += bf2f(f2bf(fmaxf(d2[r] + F.b2[r], 0.0f))) * F.w3[r];
        part[t] = p;
    }
    // both halves of a column hold half of the output sum
    const float mine = h == 0 ? part[0] : part[1];
    const float other = __shfl_xor(h == 0 ? part[1] : part[0], 32, 64);
    return F.b3 + (mine + other);
}

// routing decision of interface t (clamped to total - 1) of direction DIR;
// every lane of the wave must call it
template <int ND, int DIR>
__device__ __forceinline__ void sensor_item(const double *__restrict__ U, const Grid &g, const Phys &ph,
                                            const uint16_t *__restrict__ w, float zcut, uint8_t *__restrict__ mask,
                                            int64_t t) {
    const IfaceGrid I = iface_grid(g, DIR);
    const int lane = threadIdx.x & 63;
    const int64_t tc = t < I.total ? t : I.total - 1;
    int64_t q[3];
    q[0] = tc % I.E[0];
    q[1] = (tc / I.E[0]) % I.E[1];
    q[2] = tc / (I.E[0] * I.E[1]);
    q[DIR] -= 1;
    const int64_t st = g.es[DIR], cs = g.enpts;
    const int64_t e0 = ext_index(g, q[0], q[1], q[2]) - 2 * st;
    float f[kIn];
    features<ND, DIR>(U, e0, st, cs, ph, f);
    MlpFrag F;
    load_frag(w, lane, F);
    const float z = mlp_mfma(f, F, lane);
    if (t < I.total) mask[t] = z >= zcut ? 1 : 0;
}

// Routing decisions of the interfaces iq0 .. iq1-1 (iq = p + 1, interface
// p+1/2) of the lane's line along DIR (DIR >= 1: neighbouring lanes own
// neighbouring x, so loads and mask stores are contiguous).  The six points,
// four substencil indicators and three jumps slide along the line, so each
// point, substencil and jump is evaluated once.  Every lane of the wave must
// call it with the same iq0, iq1.
template <int ND, int DIR>
__device__ __forceinline__ void sensor_line(const double *__restrict__ U, const Grid &g, const Phys &ph,
                                            const MlpFrag &F, float zcut, uint8_t *__restrict__ mask, int64_t line0,
                                            int64_t iq0, int64_t iq1) {
    constexpr int O1 = DIR == 0 ? 1 : 0;
    constexpr int O2 = DIR == 2 ? 1 : 2;
    const int lane = threadIdx.x & 63;
    const int64_t n1 = g.n[O1], n2 = g.n[O2], lines = n1 * n2;
    const int64_t line = line0 + lane;
    const bool active = line < lines;
    const int64_t lc = active ? line : lines - 1;
    int64_t q[3];
    q[DIR] = 0;
    q[O1] = lc % n1;
    q[O2] = lc / n1;
    const int64_t base = ext_index(g, q[0], q[1], q[2]);
    const int64_t st = g.es[DIR], cs = g.enpts;
    int64_t E[3] = {g.n[0], g.n[1], g.n[2]};
    E[DIR] += 1;
    const int64_t ms[3] = {1, E[0], E[0] * E[1]};
    const int64_t mbase = q[O1] * ms[O1] + q[O2] * ms[O2], mst = ms[DIR];
    // interface iq: points iq-3 .. iq+2
    SPoint<ND> P[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) spoint<ND, DIR>(U, base + (iq0 - 3 + k) * st, cs, ph, P[k]);
    STriple<ND> T[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) striple<ND>(P[m], P[m + 1], P[m + 2], T[m]);
    float lr[3], lp[3];
#pragma unroll
    for (int m = 0; m < 3; ++m) sjump<ND>(P[m + 1], P[m + 2], lr[m], lp[m]);
    for (int64_t iq = iq0; iq < iq1; ++iq) {
        if (iq > iq0) {
#pragma unroll
            for (int k = 0; k < 5; ++k) P[k] = P[k + 1];
            spoint<ND, DIR>(U, base + (iq + 2) * st, cs, ph, P[5]);
#pragma unroll
            for (int m = 0; m < 3; ++m) T[m] = T[m + 1];
            striple<ND>(P[3], P[4], P[5], T[3]);
#pragma unroll
            for (int m = 0; m < 2; ++m) {
                lr[m] = lr[m + 1];
                lp[m] = lp[m + 1];
            }
            sjump<ND>(P[3], P[4], lr[2], lp[2]);
        }
        float f[kIn];
        sfeatures<ND>(P[2], P[3], T, lr, lp, ph, f);
        const float z = mlp_mfma(f, F, lane);
        if (active) mask[mbase + iq * mst] = z >= zcut ? 1 : 0;
    }
}

// Routing decisions of the x interfaces J0 .. J0+63 of the row-major
// interface numbering J = row (N + 1) + p + 1 (rows of N + 1 >= 64
// interfaces, so a wave spans at most two rows): each lane evaluates the
// point p + 3 of its row once (plus the five points left of lane 0's stencil
// and the first five points of a row starting inside the wave), the stencils
// are gathered from LDS.  Every lane of the wave must call it.
constexpr int kSxSlots = 64 + 10;

template <int ND>
struct SxLds {
    double v[ND + 1][kSxSlots];  // r, p, vt[0..ND-2] of the staged points
};

template <int ND>
__device__ __forceinline__ void sensor_x_lanes(const double *__restrict__ U, const Grid &g, const Phys &ph,
                                               const MlpFrag &F, float zcut, uint8_t *__restrict__ mask, int64_t J0,
                                               int64_t totalJ, SxLds<ND> &sp) {
    const int lane = threadIdx.x & 63;
    const int64_t N = g.n[0], NI = N + 1, n1 = g.n[1], cs = g.enpts;
    const int64_t J = J0 + lane;
    const bool valid = J < totalJ;
    // lane 0's row and interface (wave-uniform), then each lane's row without
    // a per-lane division: a wave spans at most two rows (NI >= 64), whose
    // (y, z) are scalars; lanes past the last interface take the last one
    const bool narrow = totalJ < 0x7fffffff;
    auto sdiv = [narrow](int64_t a, int64_t b) -> int64_t {
        return narrow ? (int64_t)((uint32_t)a / (uint32_t)b) : a / b;
    };
    const int64_t row0 = sdiv(J0, NI), q0 = J0 - row0 * NI - 1;
    const int Lnext = (int)(NI - (q0 + 1));  // first lane of row0 + 1 (>= 64: none)
    const int64_t z0 = sdiv(row0, n1), y0 = row0 - z0 * n1;
    const int64_t y1 = y0 + 1 < n1 ? y0 + 1 : 0, z1 = y0 + 1 < n1 ? z0 : z0 + 1;
    const bool has1 = row0 + 1 < n1 * g.n[2];
    const bool nxt = lane >= Lnext;
    int64_t yl = nxt ? y1 : y0, zl = nxt ? z1 : z0;
    int64_t q = nxt ? (int64_t)(lane - Lnext) - 1 : q0 + lane;
    if (!valid) {
        yl = n1 - 1;
        zl = g.n[2] - 1;
        q = N - 1;
    }
    auto stage = [&](int slot, int64_t y, int64_t z, int64_t pos) {
        SPoint<ND> o;
        spoint<ND, 0>(U, ext_index(g, 0, y, z) + pos, cs, ph, o);
        sp.v[0][slot] = o.r;
        sp.v[1][slot] = o.p;
#pragma unroll
        for (int s = 0; s < ND - 1; ++s) sp.v[2 + s][slot] = o.vt[s];
    };
    stage(lane, yl, zl, q + 3);
    if (lane < 5) {
        stage(64 + lane, y0, z0, q0 - 2 + lane);
    } else if (lane < 10 && Lnext < 64) {
        stage(64 + lane, has1 ? y1 : y0, has1 ? z1 : z0, (int64_t)(lane - 5) - 3);
    }
    wave_sync();
    const bool inrow0 = lane < Lnext;
    SPoint<ND> P[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        const int src = lane - 5 + k;
        int slot;
        if (inrow0) slot = src >= 0 ? src : 64 + lane + k;
        else slot = src >= Lnext ? src : 69 + (lane - Lnext) + k;
        P[k].r = sp.v[0][slot];
        P[k].p = sp.v[1][slot];
#pragma unroll
        for (int s = 0; s < ND - 1; ++s) P[k].vt[s] = sp.v[2 + s][slot];
    }
    STriple<ND> T[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) striple<ND>(P[m], P[m + 1], P[m + 2], T[m]);
    float lr[3], lp[3];
#pragma unroll
    for (int m = 0; m < 3; ++m) sjump<ND>(P[m + 1], P[m + 2], lr[m], lp[m]);
    float f[kIn];
    sfeatures<ND>(P[2], P[3], T, lr, lp, ph, f);
    const float z = mlp_mfma(f, F, lane);
    if (valid) mask[J] = z >= zcut ? 1 : 0;
    wave_sync();  // the staging buffer is reused by the next call
}

}  // namespace sn
}  // namespace osbli
