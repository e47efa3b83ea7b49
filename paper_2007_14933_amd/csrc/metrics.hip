// Metric terms, computed once in FP64 with the same fourth-order central
// operator and one-sided closures as the viscous terms (section 2.6, last
// paragraph).  Strong-conservation form: area vectors S_d = grad(xi_d)/J;
// 2D: S_xi = (y_eta, -x_eta), S_eta = (-y_xi, x_xi); 3D: S_a = x_b x x_c with
// each component in the conservative form D_c(x_q D_b x_p) - D_b(x_q D_c x_p)
// so that sum_d D_d S_d = 0 holds discretely.  Periodic directions shift the
// coordinate component along them by period[d] across the wrap.  Ghost-node
// metrics: periodic copy, otherwise the boundary node's value.
// Separable meshes keep only 1/h_d with h_d = D_d x_d (one array per axis).
#include "internal.hpp"

namespace osbli {
namespace {

struct Coords {
    const double *x[3];   // compact interior arrays (general) or 1D arrays (separable)
    double period[3];
};

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

__device__ __forceinline__ int64_t floordiv(int64_t a, int64_t n) { return a >= 0 ? a / n : -((-a + n - 1) / n); }

// coordinate component comp at a node whose indices may lie outside along
// periodic directions
__device__ __forceinline__ double coord(const Grid &g, const Coords &C, int comp, int64_t i, int64_t j, int64_t k) {
    int64_t q[3] = {i, j, k};
    double shift = 0.0;
    for (int d = 0; d < g.nd; ++d) {
        const int64_t N = g.n[d];
        if (q[d] < 0 || q[d] >= N) {
            const int64_t mm = floordiv(q[d], N);
            q[d] -= mm * N;
            if (comp == d) shift += (double)mm * C.period[d];
        }
    }
    return C.x[comp][int_index(g, q[0], q[1], q[2])] + shift;
}

__global__ void k_metric_sep(Grid g, Coords C, double *invh0, double *invh1, double *invh2) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int d = 0;
    int64_t i = t;
    while (d < g.nd && i >= g.n[d]) {
        i -= g.n[d];
        ++d;
    }
    if (d >= g.nd) return;
    const int64_t N = g.n[d];
    const double *x = C.x[d];
    const double P = C.period[d];
    auto at = [&](int64_t q) {
        const int64_t mm = floordiv(q, N);
        return x[q - mm * N] + (double)mm * P;
    };
    const double h = dline(at, i, N, g.periodic[d] != 0);
    double *out = d == 0 ? invh0 : (d == 1 ? invh1 : invh2);
    out[i] = 1.0 / h;
}

// general 2D: S and J at interior nodes (extended layout)
__global__ void k_metric_gen2(Grid g, Coords C, double *S, double *J) {
    const int64_t ci = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (ci >= g.nint) return;
    const int64_t i = ci % g.n[0], j = ci / g.n[0];
    double X[2][2];
    for (int p = 0; p < 2; ++p) {
        auto ax = [&](int64_t q) { return coord(g, C, p, q, j, 0); };
        auto ay = [&](int64_t q) { return coord(g, C, p, i, q, 0); };
        X[p][0] = dline(ax, i, g.n[0], g.periodic[0] != 0);
        X[p][1] = dline(ay, j, g.n[1], g.periodic[1] != 0);
    }
    const int64_t e = ext_index(g, i, j, 0);
    const int64_t cs = g.enpts;
    S[0 * cs + e] = X[1][1];
    S[1 * cs + e] = -X[0][1];
    S[2 * cs + e] = -X[1][0];
    S[3 * cs + e] = X[0][0];
    J[e] = 1.0 / (X[0][0] * X[1][1] - X[0][1] * X[1][0]);
}

// general 3D, pass A: coordinate derivatives Xd[p*3+b] = D_b x_p at interior nodes
__global__ void k_metric_gen3a(Grid g, Coords C, double *Xd) {
    const int64_t ci = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (ci >= g.nint) return;
    const int64_t q0[3] = {ci % g.n[0], (ci / g.n[0]) % g.n[1], ci / (g.n[0] * g.n[1])};
    for (int p = 0; p < 3; ++p)
        for (int b = 0; b < 3; ++b) {
            auto at = [&](int64_t s) {
                int64_t q[3] = {q0[0], q0[1], q0[2]};
                q[b] = s;
                return coord(g, C, p, q[0], q[1], q[2]);
            };
            Xd[(p * 3 + b) * g.nint + ci] = dline(at, q0[b], g.n[b], g.periodic[b] != 0);
        }
}

// general 3D, pass B: conservative area vectors and J
__global__ void k_metric_gen3b(Grid g, Coords C, const double *__restrict__ Xd, double *S, double *J) {
    const int64_t ci = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (ci >= g.nint) return;
    const int64_t q0[3] = {ci % g.n[0], (ci / g.n[0]) % g.n[1], ci / (g.n[0] * g.n[1])};
    const int64_t e = ext_index(g, q0[0], q0[1], q0[2]);
    const int64_t cs = g.enpts;
    for (int a = 0; a < 3; ++a) {
        const int b = (a + 1) % 3, c = (a + 2) % 3;
        for (int mcomp = 0; mcomp < 3; ++mcomp) {
            const int p = (mcomp + 1) % 3, qc = (mcomp + 2) % 3;
            // D_c(x_q X_{p,b}) - D_b(x_q X_{p,c})
            auto at1 = [&](int64_t s) {
                int64_t q[3] = {q0[0], q0[1], q0[2]};
                q[c] = s;
                const double xq = coord(g, C, qc, q[0], q[1], q[2]);
                int64_t w[3] = {q[0], q[1], q[2]};
                const int64_t N = g.n[c];
                w[c] = s - floordiv(s, N) * N;
                return xq * Xd[(p * 3 + b) * g.nint + int_index(g, w[0], w[1], w[2])];
            };
            auto at2 = [&](int64_t s) {
                int64_t q[3] = {q0[0], q0[1], q0[2]};
                q[b] = s;
                const double xq = coord(g, C, qc, q[0], q[1], q[2]);
                int64_t w[3] = {q[0], q[1], q[2]};
                const int64_t N = g.n[b];
                w[b] = s - floordiv(s, N) * N;
                return xq * Xd[(p * 3 + c) * g.nint + int_index(g, w[0], w[1], w[2])];
            };
            const double t1 = dline(at1, q0[c], g.n[c], g.periodic[c] != 0);
            const double t2 = dline(at2, q0[b], g.n[b], g.periodic[b] != 0);
            S[(a * 3 + mcomp) * cs + e] = t1 - t2;
        }
    }
    auto X = [&](int p, int b) { return Xd[(p * 3 + b) * g.nint + ci]; };
    const double det = X(0, 0) * (X(1, 1) * X(2, 2) - X(1, 2) * X(2, 1)) -
                       X(0, 1) * (X(1, 0) * X(2, 2) - X(1, 2) * X(2, 0)) +
                       X(0, 2) * (X(1, 0) * X(2, 1) - X(1, 1) * X(2, 0));
    J[e] = 1.0 / det;
}

// ghost-node fill of one extended array along direction d over the full
// extent of the other directions
__global__ void k_metric_ghosts(Grid g, double *A, int d) {
    const int o1 = d == 0 ? 1 : 0, o2 = d == 2 ? 1 : 2;
    const int64_t e1 = g.e[o1], e2 = g.e[o2];
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 2 * kGhost * e1 * e2) return;
    const int64_t r = t % (e1 * e2);
    const int64_t gm = t / (e1 * e2);  // 0..2*kGhost-1
    int64_t q[3];
    q[o1] = r % e1 - g.h[o1];
    q[o2] = r / e1 - g.h[o2];
    const int64_t N = g.n[d];
    const int64_t pos = gm < kGhost ? -1 - gm : N + (gm - kGhost);
    int64_t src;
    if (g.periodic[d]) src = pos < 0 ? pos + N : pos - N;
    else src = pos < 0 ? 0 : N - 1;
    q[d] = pos;
    const int64_t ed = ext_index(g, q[0], q[1], q[2]);
    q[d] = src;
    A[ed] = A[ext_index(g, q[0], q[1], q[2])];
}

}  // namespace

hipError_t launch_metrics_separable(const Grid &g, const double *coord1d, double *invh_out[3],
                                    const double period[3], hipStream_t s) {
    Coords C;
    int64_t off = 0;
    for (int d = 0; d < 3; ++d) {
        C.x[d] = d < g.nd ? coord1d + off : nullptr;
        if (d < g.nd) off += g.n[d];
        C.period[d] = period[d];
    }
    const int bs = 256;
    hipLaunchKernelGGL(k_metric_sep, dim3((unsigned)((off + bs - 1) / bs)), dim3(bs), 0, s, g, C, invh_out[0],
                       invh_out[1], invh_out[2]);
    return hipGetLastError();
}

hipError_t launch_metrics_general(const Grid &g, const double *coords, double *stage, double *S, double *J,
                                  const double period[3], hipStream_t s) {
    Coords C;
    for (int d = 0; d < 3; ++d) {
        C.x[d] = d < g.nd ? coords + d * g.nint : nullptr;
        C.period[d] = period[d];
    }
    const int bs = 256;
    const unsigned nb = (unsigned)((g.nint + bs - 1) / bs);
    if (g.nd == 2) {
        hipLaunchKernelGGL(k_metric_gen2, dim3(nb), dim3(bs), 0, s, g, C, S, J);
    } else {
        hipLaunchKernelGGL(k_metric_gen3a, dim3(nb), dim3(bs), 0, s, g, C, stage);
        hipLaunchKernelGGL(k_metric_gen3b, dim3(nb), dim3(bs), 0, s, g, C, stage, S, J);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int ncomp = g.nd * g.nd;
    for (int d = 0; d < g.nd; ++d) {
        const int o1 = d == 0 ? 1 : 0, o2 = d == 2 ? 1 : 2;
        const int64_t nt = 2 * kGhost * g.e[o1] * g.e[o2];
        const unsigned nbg = (unsigned)((nt + bs - 1) / bs);
        for (int c = 0; c < ncomp; ++c)
            hipLaunchKernelGGL(k_metric_ghosts, dim3(nbg), dim3(bs), 0, s, g, S + c * g.enpts, d);
        hipLaunchKernelGGL(k_metric_ghosts, dim3(nbg), dim3(bs), 0, s, g, J, d);
    }
    return hipGetLastError();
}

}  // namespace osbli
