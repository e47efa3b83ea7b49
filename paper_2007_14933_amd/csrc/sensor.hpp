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
__device__ __forceinline__ uint16_t f2bf(float x) {  // round to nearest even
    unsigned u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// ------------------------------------------------------------ features
__device__ __forceinline__ double js3(const double (&q)[6], int m) {
#pragma clang fp contract(off)
    const double a1 = q[m] - 2.0 * q[m + 1] + q[m + 2], a2 = q[m] - q[m + 2];
    return (13.0 / 12.0) * a1 * a1 + 0.25 * a2 * a2;
}

// Sensor features of interface p+1/2 of a line (separable meshes: n = e_DIR,
// tangents e_{DIR+1}, e_{DIR+2}); stencil points p-2..p+3 start at ext index
// e0 with stride st.  Features 0..3: three-point Jiang-Shu indicators of
// rho/rho_bar + p/p_bar + u_t/a_bar on the four substencils (each variable's
// indicator on unscaled values times the inverse square of its scale), over
// their sum + 1e-20; 4..9: log10(1 + 1e6 J)/6 of the rho and p jumps
// J = |q_{k+1} - q_k| / (q_{k+1} + q_k) over (p-1,p), (p,p+1), (p+1,p+2).
template <int ND, int DIR>
__device__ __forceinline__ void features(const double *__restrict__ U, int64_t e0, int64_t st, int64_t cs,
                                         const Phys &ph, float (&f)[kIn]) {
    // the FP64 operations of the definition in its order, no FMA contraction,
    // so that every translation unit computes the same features
#pragma clang fp contract(off)
    double rho[6], p[6], vt[2][6];
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        const int64_t e = e0 + k * st;
        const double r = U[e];
        double u[3], ke = 0.0;
#pragma unroll
        for (int m = 0; m < ND; ++m) {
            u[m] = U[e + (1 + m) * cs] / r;
            ke += u[m] * u[m];
        }
        rho[k] = r;
        p[k] = ph.gm1 * (U[e + (ND + 1) * cs] - 0.5 * r * ke);
#pragma unroll
        for (int s = 0; s < ND - 1; ++s) vt[s][k] = u[(DIR + 1 + s) % ND];
    }
    const double rb = 0.5 * (rho[2] + rho[3]), pb = 0.5 * (p[2] + p[3]);
    const double sr = 1.0 / (rb * rb), sp = 1.0 / (pb * pb), sv = rb / (ph.gamma * pb);
    double beta[4], sum = 0.0;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        double b = sr * js3(rho, m) + sp * js3(p, m);
#pragma unroll
        for (int s = 0; s < ND - 1; ++s) b += sv * js3(vt[s], m);
        beta[m] = b;
        sum += b;
    }
    const double inv = 1.0 / (sum + 1e-20);
#pragma unroll
    for (int m = 0; m < 4; ++m) f[m] = (float)(beta[m] * inv);
    // jump logarithms in FP32 (inputs of a bfloat16 network)
#pragma unroll
    for (int m = 0; m < 3; ++m) {
        const double jr = fabs(rho[m + 2] - rho[m + 1]) / (rho[m + 2] + rho[m + 1]);
        const double jp = fabs(p[m + 2] - p[m + 1]) / (p[m + 2] + p[m + 1]);
        f[4 + m] = log10f((float)(1.0 + 1e6 * jr)) * (1.0f / 6.0f);
        f[7 + m] = log10f((float)(1.0 + 1e6 * jp)) * (1.0f / 6.0f);
    }
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

// per-lane operand fragments of v_mfma_f32_32x32x16_bf16:
// B (K x N = 16 x 32): lane l holds column l % 32, rows 8 (l / 32) .. + 7
struct MlpFrag {
    bf16x8 w1, w2a, w2b;
    float b1, b2;
};

__device__ __forceinline__ bf16x8 pack8(const uint16_t (&u)[8]) {
    bf16x8 v;
    __builtin_memcpy(&v, u, sizeof v);
    return v;
}

__device__ __forceinline__ void load_frag(const uint16_t *__restrict__ w, int lane, MlpFrag &F) {
    const int j = lane & 31, kh = 8 * (lane >> 5);
    uint16_t u[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) u[i] = (kh + i < kIn) ? w[oW1 + (kh + i) * kH + j] : (uint16_t)0;
    F.w1 = pack8(u);
#pragma unroll
    for (int i = 0; i < 8; ++i) u[i] = w[oW2 + (kh + i) * kH + j];
    F.w2a = pack8(u);
#pragma unroll
    for (int i = 0; i < 8; ++i) u[i] = w[oW2 + (16 + kh + i) * kH + j];
    F.w2b = pack8(u);
    F.b1 = bf2f(w[oB1 + j]);
    F.b2 = bf2f(w[oB2 + j]);
}

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// logit of the lane's own sample; every lane of the wave must call it.
// xs: 64 x 16 bf16 scratch, hs: 64 x 32 bf16 scratch (per wave, LDS);
// w3s: w3[0..31], b3 as floats (LDS).  Inputs and hidden activations are
// rounded to bf16 (the A operands), accumulation is FP32.
__device__ __forceinline__ float mlp_mfma(const float (&x)[kIn], const MlpFrag &F, uint16_t *xs, uint16_t *hs,
                                          const float *w3s, int lane) {
#pragma clang fp contract(off)
#pragma unroll
    for (int k = 0; k < 16; ++k) xs[lane * 16 + k] = k < kIn ? f2bf(x[k]) : (uint16_t)0;
    wave_sync();
    const int r32 = lane & 31, kh = 8 * (lane >> 5), c = lane & 31;
    f32x16 acc[2];
#pragma unroll
    for (int rb = 0; rb < 2; ++rb) {
        bf16x8 a;
        __builtin_memcpy(&a, xs + (rb * 32 + r32) * 16 + kh, sizeof a);
        f32x16 zero = {0};
        acc[rb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, F.w1, zero, 0, 0, 0);
    }
    // D layout: register r of lane l holds row 8 (r / 4) + 4 (l / 32) + r % 4, column l % 32
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int row = rb * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
            hs[row * 32 + c] = f2bf(fmaxf(acc[rb][r] + F.b1, 0.0f));
        }
    wave_sync();
    f32x16 acc2[2];
#pragma unroll
    for (int rb = 0; rb < 2; ++rb) {
        bf16x8 a0, a1;
        __builtin_memcpy(&a0, hs + (rb * 32 + r32) * 32 + kh, sizeof a0);
        __builtin_memcpy(&a1, hs + (rb * 32 + r32) * 32 + 16 + kh, sizeof a1);
        f32x16 zero = {0};
        acc2[rb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0, F.w2a, zero, 0, 0, 0);
        acc2[rb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1, F.w2b, acc2[rb], 0, 0, 0);
    }
    wave_sync();
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int row = rb * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
            hs[row * 32 + c] = f2bf(fmaxf(acc2[rb][r] + F.b2, 0.0f));
        }
    wave_sync();
    float z = w3s[32];
#pragma unroll
    for (int j = 0; j < kH; ++j) z += bf2f(hs[lane * 32 + j]) * w3s[j];
    wave_sync();  // scratch reused by the next call
    return z;
}

// routing decision of interface t (clamped to total - 1) of direction DIR;
// every lane of the wave must call it
template <int ND, int DIR>
__device__ __forceinline__ void sensor_item(const double *__restrict__ U, const Grid &g, const Phys &ph,
                                            const uint16_t *__restrict__ w, float zcut, uint8_t *__restrict__ mask,
                                            int64_t t, uint16_t *xs, uint16_t *hs, const float *w3s) {
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
    const float z = mlp_mfma(f, F, xs, hs, w3s, lane);
    if (t < I.total) mask[t] = z >= zcut ? 1 : 0;
}

}  // namespace sn
}  // namespace osbli
