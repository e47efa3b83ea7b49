// Learned shock sensor (not in the paper; the paper names sensor-switched
// hybrids of central and shock-capturing fluxes as hard to design by hand):
//   - sensor features of an interface and the TENO "all stencils kept" label
//     (training data made by the method itself);
//   - a 10 -> 32 -> 32 -> 1 network (ReLU, ReLU, sigmoid) with bfloat16
//     weights: FP32 training forward / backward, a deterministic gradient
//     reduction and Adam on FP32 master weights;
//   - inference on the matrix cores (bf16 MFMA, FP32 accumulation), 64
//     interfaces per wave, producing per-interface routing masks.
#include "charflux.hpp"
#include "sensor.hpp"

namespace osbli {
namespace {
using namespace cf;
using namespace sn;

// features + label of every interface of direction DIR (TENO5 labels)
template <int ND, int DIR>
__global__ void __launch_bounds__(256)
k_labels(const double *__restrict__ U, Grid g, Phys ph, float *__restrict__ feat, uint8_t *__restrict__ lab) {
    const IfaceGrid I = iface_grid(g, DIR);
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= I.total) return;
    int64_t q[3];
    q[0] = t % I.E[0];
    q[1] = (t / I.E[0]) % I.E[1];
    q[2] = t / (I.E[0] * I.E[1]);
    q[DIR] -= 1;  // interface position p in [-1, N-1]
    const int64_t st = g.es[DIR], cs = g.enpts;
    const int64_t e0 = ext_index(g, q[0], q[1], q[2]) - 2 * st;
    float f[kIn];
    features<ND, DIR>(U, e0, st, cs, ph, f);
#pragma unroll
    for (int m = 0; m < kIn; ++m) feat[t * kIn + m] = f[m];
    Loc<ND> P[6];
    constexpr int T1 = (DIR + 1) % ND, T2 = (DIR + 2) % ND;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        Pt<ND> w;
#pragma unroll
        for (int c = 0; c < ND + 2; ++c) w.U[c] = U[e0 + k * st + c * cs];
        bool bad = false;
        finish_point<ND>(ph, w, bad);
        P[k].r = w.U[0];
        P[k].mn = w.U[1 + DIR];
        P[k].mt[0] = ND >= 2 ? w.U[1 + T1] : 0.0;
        P[k].mt[1] = ND >= 3 ? w.U[1 + T2] : 0.0;
        P[k].E = w.U[ND + 1];
        P[k].p = w.p;
        P[k].a = w.a;
        P[k].ri = w.ri;
    }
    bool kept = true;
    double Fr, Fn, Ft[2], FE;
    char_flux<ND, OSBLI_TENO5>(P, ph, Fr, Fn, Ft, FE, &kept);
    lab[t] = kept ? 1 : 0;
}

// ------------------------------------------------------ FP32 training pass
constexpr int kMB = 64;  // samples per block (one wave)

struct Fwd {
    float a1[kH], a2[kH], z;
};

__device__ __forceinline__ void fwd_fp32(const float (&x)[kIn], const float *W, Fwd &o) {
#pragma unroll
    for (int j = 0; j < kH; ++j) {
        float s = W[oB1 + j];
#pragma unroll
        for (int k = 0; k < kIn; ++k) s += x[k] * W[oW1 + k * kH + j];
        o.a1[j] = s;
    }
#pragma unroll
    for (int j = 0; j < kH; ++j) {
        float s = W[oB2 + j];
#pragma unroll
        for (int k = 0; k < kH; ++k) s += fmaxf(o.a1[k], 0.0f) * W[oW2 + k * kH + j];
        o.a2[j] = s;
    }
    float z = W[oB3];
#pragma unroll
    for (int j = 0; j < kH; ++j) z += fmaxf(o.a2[j], 0.0f) * W[oW3 + j];
    o.z = z;
}

// per-block partial gradients of the mean class-weighted BCE
__global__ void __launch_bounds__(kMB)
k_mlp_grad(const float *__restrict__ X, const uint8_t *__restrict__ y, int64_t n, const uint16_t *__restrict__ w,
           float wneg, float inv_n, float *__restrict__ partial) {
    __shared__ float W[kNP];
    __shared__ float sx[kMB][kIn], sh1[kMB][kH], sd1[kMB][kH], sh2[kMB][kH], sd2[kMB][kH], sdz[kMB], sl[kMB];
    for (int e = threadIdx.x; e < kNP; e += kMB) W[e] = bf2f(w[e]);
    __syncthreads();
    const int tid = threadIdx.x;
    const int64_t s = (int64_t)blockIdx.x * kMB + tid;
    const bool valid = s < n;
    float x[kIn];
#pragma unroll
    for (int k = 0; k < kIn; ++k) x[k] = valid ? X[s * kIn + k] : 0.0f;
    Fwd o;
    fwd_fp32(x, W, o);
    const float yv = valid ? (float)y[s] : 0.0f;
    const float wt = valid ? (yv > 0.5f ? 1.0f : wneg) : 0.0f;
    // sigmoid and the loss term in FP64 (float expf would carry its own
    // rounding into every gradient)
    const double zd = o.z;
    const double sig = 1.0 / (1.0 + exp(-zd));
    const float dz = (float)(wt * (sig - yv) * inv_n);
    const double sp = fmax(zd, 0.0) + log1p(exp(-fabs(zd)));
    sl[tid] = (float)(wt * (sp - yv * zd) * inv_n);
    sdz[tid] = dz;
    float d2[kH];
#pragma unroll
    for (int j = 0; j < kH; ++j) {
        d2[j] = o.a2[j] > 0.0f ? dz * W[oW3 + j] : 0.0f;
        sd2[tid][j] = d2[j];
        sh2[tid][j] = fmaxf(o.a2[j], 0.0f);
        sh1[tid][j] = fmaxf(o.a1[j], 0.0f);
    }
#pragma unroll
    for (int k = 0; k < kH; ++k) {
        float acc = 0.0f;
#pragma unroll
        for (int j = 0; j < kH; ++j) acc += d2[j] * W[oW2 + k * kH + j];
        sd1[tid][k] = o.a1[k] > 0.0f ? acc : 0.0f;
    }
#pragma unroll
    for (int k = 0; k < kIn; ++k) sx[tid][k] = x[k];
    __syncthreads();
    float *out = partial + (int64_t)blockIdx.x * kNPad;
    for (int e = tid; e < kNPad; e += kMB) {
        double acc = 0.0;  // FP64 sums: FP32 sequential sums of same-sign terms drift
        if (e < oB1) {
            const int k = e / kH, j = e % kH;
            for (int t = 0; t < kMB; ++t) acc += (double)sx[t][k] * sd1[t][j];
        } else if (e < oW2) {
            const int j = e - oB1;
            for (int t = 0; t < kMB; ++t) acc += sd1[t][j];
        } else if (e < oB2) {
            const int k = (e - oW2) / kH, j = (e - oW2) % kH;
            for (int t = 0; t < kMB; ++t) acc += (double)(sh1[t][k] * sd2[t][j]);
        } else if (e < oW3) {
            const int j = e - oB2;
            for (int t = 0; t < kMB; ++t) acc += sd2[t][j];
        } else if (e < oB3) {
            const int j = e - oW3;
            for (int t = 0; t < kMB; ++t) acc += (double)(sh2[t][j] * sdz[t]);
        } else if (e == oB3) {
            for (int t = 0; t < kMB; ++t) acc += sdz[t];
        } else {
            for (int t = 0; t < kMB; ++t) acc += sl[t];
        }
        out[e] = (float)acc;
    }
}

// fixed-order sum of the block partials -> gradient (1441) and loss
__global__ void k_mlp_reduce(const float *__restrict__ partial, int64_t nblk, float *__restrict__ grad,
                             float *__restrict__ loss) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= kNPad) return;
    double acc = 0.0;
    for (int64_t b = 0; b < nblk; ++b) acc += partial[b * kNPad + e];
    if (e < kNP) grad[e] = (float)acc;
    else if (loss) *loss = (float)acc;
}

__global__ void k_mlp_adam(float *__restrict__ master, uint16_t *__restrict__ w, const float *__restrict__ grad,
                           float *__restrict__ m, float *__restrict__ v, float lr, float b1, float b2, float eps,
                           float c1, float c2) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= kNP) return;
    const float g = grad[e];
    const float mm = b1 * m[e] + (1.0f - b1) * g;
    const float vv = b2 * v[e] + (1.0f - b2) * g * g;
    m[e] = mm;
    v[e] = vv;
    const float th = master[e] - lr * (mm / c1) / (sqrtf(vv / c2) + eps);
    master[e] = th;
    w[e] = f2bf(th);
}

__global__ void k_mlp_fwd_fp32(const float *__restrict__ X, int64_t n, const uint16_t *__restrict__ w,
                               float *__restrict__ z) {
    __shared__ float W[kNP];
    for (int e = threadIdx.x; e < kNP; e += blockDim.x) W[e] = bf2f(w[e]);
    __syncthreads();
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    float x[kIn];
#pragma unroll
    for (int k = 0; k < kIn; ++k) x[k] = X[s * kIn + k];
    Fwd o;
    fwd_fp32(x, W, o);
    z[s] = o.z;
}

// ------------------------------------------------------ MFMA inference
__global__ void __launch_bounds__(256)
k_mlp_fwd_mfma(const float *__restrict__ X, int64_t n, const uint16_t *__restrict__ w, float *__restrict__ z) {
    const int lane = threadIdx.x & 63;
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t sc = s < n ? s : n - 1;
    float x[kIn];
#pragma unroll
    for (int k = 0; k < kIn; ++k) x[k] = X[sc * kIn + k];
    MlpFrag F;
    load_frag(w, lane, F);
    const float zz = mlp_mfma(x, F, lane);
    if (s < n) z[s] = zz;
}

// routing mask of every interface of direction DIR: 1 when the network's
// logit reaches zcut (P(smooth) >= threshold)
template <int ND, int DIR>
__global__ void __launch_bounds__(256)
k_sensor(const double *__restrict__ U, Grid g, Phys ph, const uint16_t *__restrict__ w, float zcut,
         uint8_t *__restrict__ mask) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    sensor_item<ND, DIR>(U, g, ph, w, zcut, mask, t);
}

template <int ND>
hipError_t labels_nd(const Grid &g, const Phys &ph, const double *U, int d, float *feat, uint8_t *lab,
                     hipStream_t s) {
    const IfaceGrid I = iface_grid(g, d);
    const unsigned nb = (unsigned)((I.total + 255) / 256);
    if (d == 0) hipLaunchKernelGGL((k_labels<ND, 0>), dim3(nb), dim3(256), 0, s, U, g, ph, feat, lab);
    else if (d == 1) hipLaunchKernelGGL((k_labels<ND, (ND >= 2 ? 1 : 0)>), dim3(nb), dim3(256), 0, s, U, g, ph, feat, lab);
    else hipLaunchKernelGGL((k_labels<ND, (ND >= 3 ? 2 : 0)>), dim3(nb), dim3(256), 0, s, U, g, ph, feat, lab);
    return hipGetLastError();
}

// y and z directions: each wave marches a segment of interfaces along 64
// neighbouring lines (sensor_line)
template <int ND, int DIR>
__global__ void __launch_bounds__(256)
k_sensor_line(const double *__restrict__ U, Grid g, Phys ph, const uint16_t *__restrict__ w, float zcut,
              uint8_t *__restrict__ mask, int64_t seg, int64_t nseg) {
    constexpr int O1 = DIR == 0 ? 1 : 0;
    constexpr int O2 = DIR == 2 ? 1 : 2;
    const int64_t lines = g.n[O1] * g.n[O2];
    const int64_t wpl = (lines + 63) >> 6;
    const int64_t gw = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t sg = gw / wpl;
    if (sg >= nseg) return;  // wave-uniform
    const int64_t line0 = (gw - sg * wpl) << 6;
    const int64_t NI = g.n[DIR] + 1;
    const int64_t iq0 = sg * seg, iq1 = iq0 + seg < NI ? iq0 + seg : NI;
    const int lane = threadIdx.x & 63;
    MlpFrag F;
    load_frag(w, lane, F);
    sensor_line<ND, DIR>(U, g, ph, F, zcut, mask, line0, iq0, iq1);
}

// x direction, rows of >= 64 interfaces: 64 interfaces per wave with the
// points staged once (sensor_x_lanes)
template <int ND>
__global__ void __launch_bounds__(256)
k_sensor_xl(const double *__restrict__ U, Grid g, Phys ph, const uint16_t *__restrict__ w, float zcut,
            uint8_t *__restrict__ mask, int64_t totalJ) {
    __shared__ SxLds<ND> sp[4];
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t gw = (int64_t)blockIdx.x * (blockDim.x >> 6) + wv;
    const int64_t J0 = gw * 64;
    if (J0 >= totalJ) return;  // wave-uniform
    const int lane = threadIdx.x & 63;
    MlpFrag F;
    load_frag(w, lane, F);
    sensor_x_lanes<ND>(U, g, ph, F, zcut, mask, J0, totalJ, sp[wv]);
}

template <int ND>
hipError_t sensor_nd(const Grid &g, const Phys &ph, const double *U, int d, const uint16_t *w, float zcut,
                     uint8_t *mask, hipStream_t s) {
    const IfaceGrid I = iface_grid(g, d);
    if (d == 0 && g.n[0] + 1 >= 64) {
        const int64_t waves = (I.total + 63) / 64;
        const unsigned nb = (unsigned)((waves + 3) / 4);
        hipLaunchKernelGGL((k_sensor_xl<ND>), dim3(nb), dim3(256), 0, s, U, g, ph, w, zcut, mask, I.total);
        return hipGetLastError();
    }
    if (d == 0 || ND == 1) {
        const unsigned nb = (unsigned)((I.total + 255) / 256);
        hipLaunchKernelGGL((k_sensor<ND, 0>), dim3(nb), dim3(256), 0, s, U, g, ph, w, zcut, mask);
        return hipGetLastError();
    }
    const int o1 = 0, o2 = d == 2 ? 1 : 2;  // lines of the y and z directions run along x
    const int64_t lines = g.n[o1] * g.n[o2], NI = g.n[d] + 1;
    // about 2^19 lanes (the network's cost per interface does not shrink with
    // longer segments, so parallelism is worth more than the shared prologue)
    int64_t seg = (NI * lines + (int64_t(1) << 19) - 1) >> 19;
    seg = seg < 2 ? 2 : (seg > NI ? NI : seg);
    const int64_t nseg = (NI + seg - 1) / seg;
    const int64_t waves = ((lines + 63) / 64) * nseg;
    const unsigned nb = (unsigned)((waves + 3) / 4);
    if (d == 1)
        hipLaunchKernelGGL((k_sensor_line<ND, (ND >= 2 ? 1 : 0)>), dim3(nb), dim3(256), 0, s, U, g, ph, w, zcut, mask,
                           seg, nseg);
    else
        hipLaunchKernelGGL((k_sensor_line<ND, (ND >= 3 ? 2 : 0)>), dim3(nb), dim3(256), 0, s, U, g, ph, w, zcut, mask,
                           seg, nseg);
    return hipGetLastError();
}

// number of nonzero bytes (integer atomics: order independent)
__global__ void k_count_u8(const uint8_t *__restrict__ a, int64_t n, unsigned long long *out) {
    unsigned long long c = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        c += a[i] != 0;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off, 64);
    if ((threadIdx.x & 63) == 0) atomicAdd(out, c);
}

}  // namespace

hipError_t launch_count_u8(const uint8_t *a, int64_t n, unsigned long long *out, hipStream_t s) {
    int64_t nb = (n + 255) / 256;
    if (nb > 1024) nb = 1024;
    if (nb < 1) nb = 1;
    hipLaunchKernelGGL(k_count_u8, dim3((unsigned)nb), dim3(256), 0, s, a, n, out);
    return hipGetLastError();
}

int64_t iface_count(const Grid &g, int d) { return iface_grid(g, d).total; }

hipError_t launch_labels(const Grid &g, const Phys &ph, const double *U, int d, float *feat, uint8_t *lab,
                         hipStream_t s) {
    switch (g.nd) {
        case 1: return labels_nd<1>(g, ph, U, d, feat, lab, s);
        case 2: return labels_nd<2>(g, ph, U, d, feat, lab, s);
        default: return labels_nd<3>(g, ph, U, d, feat, lab, s);
    }
}

hipError_t launch_sensor(const Grid &g, const Phys &ph, const double *U, int d, const uint16_t *w, float zcut,
                         uint8_t *mask, hipStream_t s) {
    switch (g.nd) {
        case 1: return sensor_nd<1>(g, ph, U, d, w, zcut, mask, s);
        case 2: return sensor_nd<2>(g, ph, U, d, w, zcut, mask, s);
        default: return sensor_nd<3>(g, ph, U, d, w, zcut, mask, s);
    }
}

size_t mlp_workspace_bytes(int64_t n) {
    const int64_t nblk = (n + kMB - 1) / kMB;
    return (size_t)nblk * kNPad * sizeof(float);
}

hipError_t launch_mlp_grad(const float *X, const uint8_t *y, int64_t n, const uint16_t *w, float wneg, float *grad,
                           float *loss, float *partial, hipStream_t s) {
    const int64_t nblk = (n + kMB - 1) / kMB;
    hipLaunchKernelGGL(k_mlp_grad, dim3((unsigned)nblk), dim3(kMB), 0, s, X, y, n, w, wneg, 1.0f / (float)n,
                       partial);
    hipLaunchKernelGGL(k_mlp_reduce, dim3((kNPad + 255) / 256), dim3(256), 0, s, partial, nblk, grad, loss);
    return hipGetLastError();
}

hipError_t launch_mlp_adam(float *master, uint16_t *w, const float *grad, float *m, float *v, int64_t t, float lr,
                           float b1, float b2, float eps, hipStream_t s) {
    const float c1 = 1.0f - powf(b1, (float)t), c2 = 1.0f - powf(b2, (float)t);
    hipLaunchKernelGGL(k_mlp_adam, dim3((kNP + 255) / 256), dim3(256), 0, s, master, w, grad, m, v, lr, b1, b2,
                       eps, c1, c2);
    return hipGetLastError();
}

hipError_t launch_mlp_forward(const float *X, int64_t n, const uint16_t *w, float *z, int inference,
                              hipStream_t s) {
    const unsigned nb = (unsigned)((n + 255) / 256);
    if (inference) hipLaunchKernelGGL(k_mlp_fwd_mfma, dim3(nb), dim3(256), 0, s, X, n, w, z);
    else hipLaunchKernelGGL(k_mlp_fwd_fp32, dim3(nb), dim3(256), 0, s, X, n, w, z);
    return hipGetLastError();
}

}  // namespace osbli
