// Viscous and heat-flux terms (eqs. heat_flux, stress_tensor, sutherland of
// section 2.1) in divergence form with the fourth-order central scheme and
// the one-sided boundary closures of section 2.6; the fused low-storage RK
// update (section 2.7); the CFL time-step reduction.
//
// Pass 1 (k_visc_flux): per node, gradients of (u, T) from the central
// operator (closures at non-periodic ends; periodic ends read the ghost
// copies), stress tensor, heat flux and the contravariant viscous fluxes
// G_k = S_k . Fv, stored once per node.
// Pass 2 (k_finish): per node, J sum_k D_k G_k added to the convective
// residual, then either stored (residual call) or folded into the RK update.
#include "point.hpp"

namespace osbli {
namespace {

// first derivative per unit index at position p of a line of N nodes; `at`
// returns the operand at a line index (periodic lines may be read at
// p +- 1, p +- 2 outside [0, N)).
template <class At>
__device__ __forceinline__ double dline(const At &at, int64_t p, int64_t N, bool periodic) {
    if (periodic || (p >= 2 && p <= N - 3))
        return (2.0 / 3.0) * (at(p + 1) - at(p - 1)) - (1.0 / 12.0) * (at(p + 2) - at(p - 2));
    if (p == 0)
        return (-25.0 * at(0) + 48.0 * at(1) - 36.0 * at(2) + 16.0 * at(3) - 3.0 * at(4)) / 12.0;
    if (p == 1)
        return (-3.0 * at(0) - 10.0 * at(1) + 18.0 * at(2) - 6.0 * at(3) + at(4)) / 12.0;
    if (p == N - 2)
        return (-at(N - 5) + 6.0 * at(N - 4) - 18.0 * at(N - 3) + 10.0 * at(N - 2) + 3.0 * at(N - 1)) / 12.0;
    return (3.0 * at(N - 5) - 16.0 * at(N - 4) + 36.0 * at(N - 3) - 48.0 * at(N - 2) + 25.0 * at(N - 1)) / 12.0;
}

// pointwise kernels: blocks of 64 x 4 threads over (i, j), grid.z over k
constexpr int kBX = 64, kBY = 4;

__device__ __forceinline__ bool node_of_thread(const Grid &g, int64_t (&idx)[3]) {
    idx[0] = (int64_t)blockIdx.x * kBX + threadIdx.x;
    idx[1] = (int64_t)blockIdx.y * kBY + threadIdx.y;
    idx[2] = blockIdx.z;
    return idx[0] < g.n[0] && idx[1] < g.n[1];
}

inline dim3 node_grid(const Grid &g) {
    return dim3((unsigned)((g.n[0] + kBX - 1) / kBX), (unsigned)((g.n[1] + kBY - 1) / kBY), (unsigned)g.n[2]);
}

template <int ND>
__device__ __forceinline__ void phi_at(const double *__restrict__ U, int64_t e, int64_t cs, const Phys &ph,
                                       double (&phi)[ND + 1]) {
    const double r = U[e];
    const double ri = 1.0 / r;
    double ke = 0.0;
#pragma unroll
    for (int m = 0; m < ND; ++m) {
        const double mm = U[e + (1 + m) * cs];
        phi[m] = mm * ri;
        ke += mm * mm;
    }
    const double p = ph.gm1 * (U[e + (ND + 1) * cs] - 0.5 * ke * ri);
    phi[ND] = ph.gamma * ph.M2 * p * ri;
}


template <int ND, bool GEN>
__global__ void __launch_bounds__(256)
k_visc_flux(const double *__restrict__ U, double *__restrict__ G, Grid g, Phys ph, Metrics m) {
    constexpr int NV = ND + 1;
    int64_t idx[3];
    if (!node_of_thread(g, idx)) return;
    const int64_t ci = int_index(g, idx[0], idx[1], idx[2]);
    const int64_t e0 = ext_index(g, idx[0], idx[1], idx[2]);
    const int64_t cs = g.enpts;

    double phi0[NV];
    phi_at<ND>(U, e0, cs, ph, phi0);
    double Dk[ND][NV];
#pragma unroll
    for (int kk = 0; kk < ND; ++kk) {
        const int64_t N = g.n[kk], p = idx[kk], st = g.es[kk];
        const int64_t eline = e0 - p * st;
        const bool per = g.periodic[kk] != 0;
#pragma unroll
        for (int v = 0; v < NV; ++v) Dk[kk][v] = 0.0;
        // evaluate the five-point operator component-wise from one set of loads
        if (per || (p >= 2 && p <= N - 3)) {
            double fm2[NV], fm1[NV], fp1[NV], fp2[NV];
            phi_at<ND>(U, e0 - 2 * st, cs, ph, fm2);
            phi_at<ND>(U, e0 - st, cs, ph, fm1);
            phi_at<ND>(U, e0 + st, cs, ph, fp1);
            phi_at<ND>(U, e0 + 2 * st, cs, ph, fp2);
#pragma unroll
            for (int v = 0; v < NV; ++v)
                Dk[kk][v] = (2.0 / 3.0) * (fp1[v] - fm1[v]) - (1.0 / 12.0) * (fp2[v] - fm2[v]);
        } else {
            double f[5][NV];
            const int64_t q0 = p < 2 ? 0 : N - 5;
#pragma unroll
            for (int r = 0; r < 5; ++r) phi_at<ND>(U, eline + (q0 + r) * st, cs, ph, f[r]);
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                auto at = [&](int64_t q) { return f[q - q0][v]; };
                Dk[kk][v] = dline(at, p, N, false);
            }
        }
    }
    double grad[NV][ND];
    double Jc = 1.0;
    if (GEN) Jc = m.J[e0];
#pragma unroll
    for (int v = 0; v < NV; ++v)
#pragma unroll
        for (int j = 0; j < ND; ++j) {
            if (!GEN) {
                grad[v][j] = m.invh[j][idx[j]] * Dk[j][v];
            } else {
                double s = 0.0;
#pragma unroll
                for (int kk = 0; kk < ND; ++kk) s += m.S[(kk * ND + j) * cs + e0] * Dk[kk][v];
                grad[v][j] = Jc * s;
            }
        }
    const double T = phi0[ND];
    const double mu = viscosity(ph, T);
    double divu = 0.0;
#pragma unroll
    for (int a = 0; a < ND; ++a) divu += grad[a][a];
    const double mre = mu * ph.mu_re;
    double Fv[ND][NV];
#pragma unroll
    for (int b = 0; b < ND; ++b) {
        double work = 0.0;
#pragma unroll
        for (int a = 0; a < ND; ++a) {
            double tab = mre * (grad[a][b] + grad[b][a] - (a == b ? (2.0 / 3.0) * divu : 0.0));
            Fv[b][a] = tab;
            work += phi0[a] * tab;
        }
        const double qb = -mu * ph.kheat * grad[ND][b];
        Fv[b][ND] = work - qb;
    }
#pragma unroll
    for (int kk = 0; kk < ND; ++kk)
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            double s;
            if (!GEN) {
                s = Fv[kk][v];
            } else {
                s = 0.0;
#pragma unroll
                for (int b = 0; b < ND; ++b) s += m.S[(kk * ND + b) * cs + e0] * Fv[b][v];
            }
            G[(kk * NV + v) * g.nint + ci] = s;
        }
}

// R = Racc (+ viscous divergence); mode 0 stores R, mode 1 applies the RK stage.
template <int ND, bool GEN, bool VISC, int MODE>
__global__ void __launch_bounds__(256)
k_finish(const double *Racc, const double *__restrict__ G, double *Rout, Grid g,
         Phys ph, Metrics m, int stage, double dt, double *__restrict__ U, double *__restrict__ dU) {
    constexpr int NC = ND + 2;
    constexpr int NV = ND + 1;
    int64_t idx[3];
    if (!node_of_thread(g, idx)) return;
    const int64_t ci = int_index(g, idx[0], idx[1], idx[2]);
    double R[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) R[c] = Racc[c * g.nint + ci];
    const int64_t e0 = ext_index(g, idx[0], idx[1], idx[2]);
    if (VISC) {
        double acc[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) acc[v] = 0.0;
#pragma unroll
        for (int kk = 0; kk < ND; ++kk) {
            const int64_t N = g.n[kk], p = idx[kk], st = g.is[kk];
            const int64_t line = ci - p * st;
            const bool per = g.periodic[kk] != 0;
            const double sc = GEN ? 1.0 : m.invh[kk][p];
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                const double *Gv = G + (kk * NV + v) * g.nint + line;
                auto at = [&](int64_t q) {
                    int64_t w = q;
                    if (per) w = q < 0 ? q + N : (q >= N ? q - N : q);
                    return Gv[w * st];
                };
                acc[v] += sc * dline(at, p, N, per);
            }
        }
        const double Jc = GEN ? m.J[e0] : 1.0;
#pragma unroll
        for (int v = 0; v < NV; ++v) R[1 + v] += Jc * acc[v];
    }
    if (MODE == 0) {
#pragma unroll
        for (int c = 0; c < NC; ++c) Rout[c * g.nint + ci] = R[c];
    } else {
#pragma unroll
        for (int c = 0; c < NC; ++c) rk_point(stage, dt, R[c], dU + c * g.nint + ci, U + c * g.enpts + e0);
    }
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}

// dt denominator, max over nodes; positive doubles compare as unsigned 64-bit.
// Blocks stride over z planes so that only a few hundred blocks issue the
// final atomic (a max is order independent, so the result is deterministic).
template <int ND, bool GEN>
__global__ void __launch_bounds__(256)
k_dt(const double *__restrict__ U, Grid g, Phys ph, Metrics m, unsigned long long *slot) {
    __shared__ double part[4];
    double s = 0.0;
    int64_t idx[3];
    idx[0] = (int64_t)blockIdx.x * kBX + threadIdx.x;
    idx[1] = (int64_t)blockIdx.y * kBY + threadIdx.y;
    const bool inplane = idx[0] < g.n[0] && idx[1] < g.n[1];
    for (idx[2] = blockIdx.z; inplane && idx[2] < g.n[2]; idx[2] += gridDim.z) {
        double sn = dt_node<ND, GEN>(U, g, ph, m, idx);
        s = fmax(s, sn);
    }
    s = wave_max(s);
    const int lane = threadIdx.x & 63, wv = threadIdx.y;
    if (lane == 0) part[wv] = s;
    __syncthreads();
    if (threadIdx.x == 0 && threadIdx.y == 0) {
        double b = part[0];
        for (int k = 1; k < (int)blockDim.y; ++k) b = fmax(b, part[k]);
        atomicMax(slot, (unsigned long long)__double_as_longlong(b));
    }
}

__global__ void k_fill_u64(unsigned long long *p, unsigned long long v, int n) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

template <int ND, bool GEN>
hipError_t finish_nd(const Grid &g, const Phys &ph, const Metrics &m, const double *Racc, const double *G,
                     double *Rout, int stage, double dt, double *U, double *dU, int mode, hipStream_t s) {
    const dim3 nb = node_grid(g), bs(kBX, kBY);
    if (ph.viscous) {
        if (mode == 0)
            hipLaunchKernelGGL((k_finish<ND, GEN, true, 0>), nb, bs, 0, s, Racc, G, Rout, g, ph, m,
                               stage, dt, U, dU);
        else
            hipLaunchKernelGGL((k_finish<ND, GEN, true, 1>), nb, bs, 0, s, Racc, G, Rout, g, ph, m,
                               stage, dt, U, dU);
    } else {
        if (mode == 0)
            hipLaunchKernelGGL((k_finish<ND, GEN, false, 0>), nb, bs, 0, s, Racc, G, Rout, g, ph,
                               m, stage, dt, U, dU);
        else
            hipLaunchKernelGGL((k_finish<ND, GEN, false, 1>), nb, bs, 0, s, Racc, G, Rout, g, ph,
                               m, stage, dt, U, dU);
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_viscous_fluxes(const Grid &g, const Phys &ph, const Metrics &m, const double *U, double *G,
                                 hipStream_t s) {
    const dim3 nb = node_grid(g), bs(kBX, kBY);
    const bool gen = m.general != 0;
    switch (g.nd) {
        case 1: hipLaunchKernelGGL((k_visc_flux<1, false>), nb, bs, 0, s, U, G, g, ph, m); break;
        case 2:
            if (gen) hipLaunchKernelGGL((k_visc_flux<2, true>), nb, bs, 0, s, U, G, g, ph, m);
            else hipLaunchKernelGGL((k_visc_flux<2, false>), nb, bs, 0, s, U, G, g, ph, m);
            break;
        default:
            if (gen) hipLaunchKernelGGL((k_visc_flux<3, true>), nb, bs, 0, s, U, G, g, ph, m);
            else hipLaunchKernelGGL((k_visc_flux<3, false>), nb, bs, 0, s, U, G, g, ph, m);
    }
    return hipGetLastError();
}

hipError_t launch_finish(const Grid &g, const Phys &ph, const Metrics &m, const double *Racc, const double *G,
                         double *Rout, int stage, double dt, double *U, double *dU, int mode, hipStream_t s) {
    const bool gen = m.general != 0;
    switch (g.nd) {
        case 1: return finish_nd<1, false>(g, ph, m, Racc, G, Rout, stage, dt, U, dU, mode, s);
        case 2:
            return gen ? finish_nd<2, true>(g, ph, m, Racc, G, Rout, stage, dt, U, dU, mode, s)
                       : finish_nd<2, false>(g, ph, m, Racc, G, Rout, stage, dt, U, dU, mode, s);
        default:
            return gen ? finish_nd<3, true>(g, ph, m, Racc, G, Rout, stage, dt, U, dU, mode, s)
                       : finish_nd<3, false>(g, ph, m, Racc, G, Rout, stage, dt, U, dU, mode, s);
    }
}

hipError_t launch_dt(const Grid &g, const Phys &ph, const Metrics &m, const double *U, unsigned long long *slot,
                     hipStream_t s) {
    dim3 nb = node_grid(g);
    const dim3 bs(kBX, kBY);
    const unsigned plane_blocks = nb.x * nb.y;
    unsigned gz = (1024 + plane_blocks - 1) / plane_blocks;
    if (gz < 1) gz = 1;
    if (gz > nb.z) gz = nb.z;
    nb.z = gz;
    const bool gen = m.general != 0;
    switch (g.nd) {
        case 1: hipLaunchKernelGGL((k_dt<1, false>), nb, bs, 0, s, U, g, ph, m, slot); break;
        case 2:
            if (gen) hipLaunchKernelGGL((k_dt<2, true>), nb, bs, 0, s, U, g, ph, m, slot);
            else hipLaunchKernelGGL((k_dt<2, false>), nb, bs, 0, s, U, g, ph, m, slot);
            break;
        default:
            if (gen) hipLaunchKernelGGL((k_dt<3, true>), nb, bs, 0, s, U, g, ph, m, slot);
            else hipLaunchKernelGGL((k_dt<3, false>), nb, bs, 0, s, U, g, ph, m, slot);
    }
    return hipGetLastError();
}

hipError_t launch_fill_u64(unsigned long long *p, unsigned long long v, int n, hipStream_t s) {
    hipLaunchKernelGGL(k_fill_u64, dim3((n + 63) / 64), dim3(64), 0, s, p, v, n);
    return hipGetLastError();
}

}  // namespace osbli
