// Fourth-order central path (section 2.6: central schemes for the convective
// terms of smooth problems and for the viscous terms; the scheme of the
// central Taylor-Green benchmark of section 6.1) on separable meshes of
// uniform spacing:
//   convection in conservative form, R_c -= sum_d D_d(F_d,c) / h_d;
//   viscous and heat-flux terms in expanded form: with g_ab = d_b u_a,
//   mu~ = mu(T)/Re and kappa = mu(T)/((gamma-1) M^2 Pr Re),
//     d_b tau_ab = sum_b d_b mu~ (g_ab + g_ba) - (2/3) d_a mu~ div
//                + mu~ [sum_b d_bb u_a + sum_b d_b(g_ba) - (2/3) sum_b d_a(g_bb)],
//     energy     = sum_ab g_ab tau_ab + sum_a u_a d_b tau_ab
//                + sum_b (d_b kappa d_b T + kappa d_bb T);
//   pure second derivatives (d_bb, and d_b(g_bb)) with the second-derivative
//   operator, mixed ones d_b(g_ba), a != b, as the first derivative of the
//   first derivative (outer index as written), d_b mu~ and d_b kappa as
//   first derivatives of their node values.
//
// Two storage strategies for the same arithmetic (section 6.1, "low memory
// intensity algorithms"):
//   StoreSome: only the velocity gradients g_ab are stored (one pointwise
//     pass); everything else is recomputed inside the residual kernel;
//   store-all: every derivative goes to its own work array in its own pass
//     (flux derivatives, first derivatives of u, T, mu~, kappa, second and
//     mixed derivatives), and a pointwise pass assembles them, the practice
//     the paper compares against.
// Both store the residual; the pointwise finish kernel applies the RK update
// (a pass that reads neighbouring states cannot update the state in place).
#include "point.hpp"
#include "stencil.hpp"

namespace osbli {
namespace {

// Node mapping of the central kernels: tiles of kBX x kBY columns, each
// taken plane by plane, numbered with the plane fastest; the linear block id
// b is remapped to item (b % 8) * per + b / 8, so each of the eight XCDs
// (one L2 each) walks one contiguous run of items and the blocks it holds at
// once cover neighbouring planes of the same tile: the z-neighbours of the
// five-point operators are read through that XCD's L2.
struct ColTiles {
    int tx, ty, nz, per, nt;
};

inline ColTiles col_tiles(const Grid &g) {
    ColTiles T;
    T.tx = (int)((g.n[0] + kBX - 1) / kBX);
    T.ty = (int)((g.n[1] + kBY - 1) / kBY);
    T.nz = (int)g.n[2];
    T.nt = T.tx * T.ty * T.nz;
    T.per = (T.nt + 7) / 8;
    return T;
}

__device__ __forceinline__ bool node_of_col_thread(const Grid &g, const ColTiles &T, int64_t (&idx)[3]) {
    const int L = (int)(blockIdx.x % 8) * T.per + (int)(blockIdx.x / 8);
    if (L >= T.nt) return false;
    const int k = L % T.nz, t = L / T.nz;
    idx[0] = (int64_t)(t % T.tx) * kBX + threadIdx.x;
    idx[1] = (int64_t)(t / T.tx) * kBY + threadIdx.y;
    idx[2] = k;
    return idx[0] < g.n[0] && idx[1] < g.n[1];
}

// the five-node operator window of line position p: the nodes q0 .. q0 + 4
// and the row r of the operator (-1: the centred interior / periodic stencil,
// 0, 1: the closures at the start, 3, 4: those at the end)
struct Win {
    int64_t q0;
    int r;
};

__device__ __forceinline__ Win window(int64_t p, int64_t N, bool periodic) {
    if (periodic || (p >= 2 && p <= N - 3)) return Win{p - 2, -1};
    if (p < 2) return Win{0, (int)p};
    return Win{N - 5, (int)(p - (N - 5))};
}

// first derivative per unit index from the window values f[0..4]
__device__ __forceinline__ double d1w(const double (&f)[5], int r) {
    if (r < 0) return (2.0 / 3.0) * (f[3] - f[1]) - (1.0 / 12.0) * (f[4] - f[0]);
    if (r == 0) return (-25.0 * f[0] + 48.0 * f[1] - 36.0 * f[2] + 16.0 * f[3] - 3.0 * f[4]) / 12.0;
    if (r == 1) return (-3.0 * f[0] - 10.0 * f[1] + 18.0 * f[2] - 6.0 * f[3] + f[4]) / 12.0;
    if (r == 3) return (-f[0] + 6.0 * f[1] - 18.0 * f[2] + 10.0 * f[3] + 3.0 * f[4]) / 12.0;
    return (3.0 * f[0] - 16.0 * f[1] + 36.0 * f[2] - 48.0 * f[3] + 25.0 * f[4]) / 12.0;
}

// second derivative per unit index from the window values, on differences
// from the centre (interior) or from the boundary node (closures)
__device__ __forceinline__ double d2w(const double (&f)[5], int r) {
    if (r < 0) {
        const double c = f[2];
        return (4.0 / 3.0) * ((f[3] - c) + (f[1] - c)) - (1.0 / 12.0) * ((f[4] - c) + (f[0] - c));
    }
    double d1, d2, d3, d4;
    if (r <= 1) {
        d1 = f[1] - f[0], d2 = f[2] - f[0], d3 = f[3] - f[0], d4 = f[4] - f[0];
    } else {
        d1 = f[3] - f[4], d2 = f[2] - f[4], d3 = f[1] - f[4], d4 = f[0] - f[4];
    }
    if (r == 0 || r == 4) return (-104.0 * d1 + 114.0 * d2 - 56.0 * d3 + 11.0 * d4) * (1.0 / 12.0);
    return (-20.0 * d1 + 6.0 * d2 + 4.0 * d3 - d4) * (1.0 / 12.0);
}

// node values of one extended node: the flux F_d along e_d (NC values) and
// the viscous primitives u_0..u_{ND-1}, T, mu~, kappa
template <int ND>
struct CNode {
    double F[ND + 2];
    double v[ND + 3];
};

template <int ND, bool VISC>
__device__ __forceinline__ void cnode(const double *__restrict__ U, int64_t e, int64_t cs, const Phys &ph, int d,
                                      CNode<ND> &o) {
    constexpr int NC = ND + 2;
    double q[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) q[c] = U[e + c * cs];
    const double ri = rcp64(q[0]);
    double ke = 0.0;
#pragma unroll
    for (int m = 0; m < ND; ++m) ke += q[1 + m] * q[1 + m];
    const double p = ph.gm1 * (q[ND + 1] - 0.5 * ke * ri);
    const double un = q[1 + d] * ri;
    o.F[0] = q[1 + d];
#pragma unroll
    for (int m = 0; m < ND; ++m) o.F[1 + m] = q[1 + m] * un + (m == d ? p : 0.0);
    o.F[ND + 1] = (q[ND + 1] + p) * un;
    if (VISC) {
#pragma unroll
        for (int m = 0; m < ND; ++m) o.v[m] = q[1 + m] * ri;
        const double T = ph.gamma * ph.M2 * p * ri;
        const double mu = viscosity(ph, T);
        o.v[ND] = T;
        o.v[ND + 1] = mu * ph.mu_re;
        o.v[ND + 2] = mu * ph.kheat;
    }
}

// velocity primitives only (gradient pass)
template <int ND>
__device__ __forceinline__ void cvel(const double *__restrict__ U, int64_t e, int64_t cs, double (&u)[ND]) {
    const double ri = rcp64(U[e]);
#pragma unroll
    for (int m = 0; m < ND; ++m) u[m] = U[e + (1 + m) * cs] * ri;
}

// the five window nodes of direction d around interior node idx (extended
// indices: the periodic stencil reads the ghost copies)
template <int ND>
__device__ __forceinline__ void window_ext(const Grid &g, const int64_t (&idx)[3], int d, Win &w, int64_t (&e)[5]) {
    const int64_t p = idx[d];
    w = window(p, g.n[d], g.periodic[d] != 0);
    const int64_t e0 = ext_index(g, idx[0], idx[1], idx[2]);
#pragma unroll
    for (int k = 0; k < 5; ++k) e[k] = e0 + (w.q0 + k - p) * g.es[d];
}

// the five window nodes of direction d in the interior layout (periodic:
// wrapped indices)
__device__ __forceinline__ void window_int(const Grid &g, const int64_t (&idx)[3], int d, Win &w, int64_t (&ci)[5]) {
    const int64_t p = idx[d], N = g.n[d];
    w = window(p, N, g.periodic[d] != 0);
    const int64_t c0 = int_index(g, idx[0], idx[1], idx[2]) - p * g.is[d];
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        int64_t q = w.q0 + k;
        q = q < 0 ? q + N : (q >= N ? q - N : q);
        ci[k] = c0 + q * g.is[d];
    }
}

// ---------------------------------------------------------------- StoreSome
// pass 1: velocity gradients g_ab = (1/h_b) D_b u_a, stored [(a ND + b)][node]
template <int ND>
__global__ void __launch_bounds__(256) k_c_grad(const double *__restrict__ U, double *__restrict__ Gs, Grid g,
                                                Metrics m, ColTiles T) {
    int64_t idx[3];
    if (!node_of_col_thread(g, T, idx)) return;
    const int64_t ci = int_index(g, idx[0], idx[1], idx[2]);
    const int64_t cs = g.enpts;
#pragma unroll
    for (int b = 0; b < ND; ++b) {
        Win w;
        int64_t e[5];
        window_ext<ND>(g, idx, b, w, e);
        double f[ND][5];
#pragma unroll
        for (int k = 0; k < 5; ++k) {
            double u[ND];
            cvel<ND>(U, e[k], cs, u);
#pragma unroll
            for (int a = 0; a < ND; ++a) f[a][k] = u[a];
        }
        const double ih = m.invh[b][idx[b]];
#pragma unroll
        for (int a = 0; a < ND; ++a) Gs[(a * ND + b) * g.nint + ci] = ih * d1w(f[a], w.r);
    }
}

// the expanded viscous terms of one node from its derivatives
template <int ND>
struct VTerms {
    double G[ND][ND];    // g_ab
    double dT[ND], dmu[ND], dka[ND];
    double s2u[ND][ND];  // d_bb u_a
    double s2T[ND];      // d_bb T
    double X[ND][ND];    // d_b(g_ba), a != b
    double Y[ND][ND];    // d_a(g_bb), a != b
    double u[ND], mu, ka;
};

template <int ND>
__device__ __forceinline__ void visc_assemble(const VTerms<ND> &t, double (&R)[ND + 2]) {
    double div = 0.0;
#pragma unroll
    for (int a = 0; a < ND; ++a) div += t.G[a][a];
    double work = 0.0;
#pragma unroll
    for (int a = 0; a < ND; ++a) {
        double first = -(2.0 / 3.0) * t.dmu[a] * div, second = 0.0;
#pragma unroll
        for (int b = 0; b < ND; ++b) {
            first += t.dmu[b] * (t.G[a][b] + t.G[b][a]);
            second += t.s2u[a][b];
            second += a == b ? t.s2u[b][b] : t.X[a][b];
            second -= (2.0 / 3.0) * (a == b ? t.s2u[b][a] : t.Y[a][b]);
        }
        const double dtau = first + t.mu * second;
#pragma unroll
        for (int b = 0; b < ND; ++b) {
            const double tau = t.mu * (t.G[a][b] + t.G[b][a] - (a == b ? (2.0 / 3.0) * div : 0.0));
            work += t.G[a][b] * tau;
        }
        work += t.u[a] * dtau;
        R[1 + a] += dtau;
    }
    double heat = 0.0;
#pragma unroll
    for (int b = 0; b < ND; ++b) heat += t.dka[b] * t.dT[b] + t.ka * t.s2T[b];
    R[ND + 1] += work + heat;
}

// pass 2: convection and the viscous terms from the stored velocity gradients
// and everything recomputed locally, stored as the residual (the state is
// not updated here: neighbouring nodes still read it)
template <int ND, bool VISC>
__global__ void __launch_bounds__(256)
k_c_resid(const double *__restrict__ U, const double *__restrict__ Gs, Grid g, Phys ph, Metrics m,
          double *__restrict__ Rout, ColTiles T) {
    constexpr int NC = ND + 2;
    int64_t idx[3];
    if (!node_of_col_thread(g, T, idx)) return;
    const int64_t ci = int_index(g, idx[0], idx[1], idx[2]);
    const int64_t cs = g.enpts;
    double R[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) R[c] = 0.0;
    VTerms<ND> t;
#pragma unroll
    for (int d = 0; d < ND; ++d) {
        Win w;
        int64_t e[5];
        window_ext<ND>(g, idx, d, w, e);
        double F[NC][5], V[ND + 3][5];
#pragma unroll
        for (int k = 0; k < 5; ++k) {
            CNode<ND> o;
            cnode<ND, VISC>(U, e[k], cs, ph, d, o);
#pragma unroll
            for (int c = 0; c < NC; ++c) F[c][k] = o.F[c];
            if (VISC) {
#pragma unroll
                for (int v = 0; v < ND + 3; ++v) V[v][k] = o.v[v];
            }
        }
        const double ih = m.invh[d][idx[d]];
#pragma unroll
        for (int c = 0; c < NC; ++c) R[c] -= ih * d1w(F[c], w.r);
        if (VISC) {
            const double ih2 = ih * ih;
            t.dT[d] = ih * d1w(V[ND], w.r);
            t.dmu[d] = ih * d1w(V[ND + 1], w.r);
            t.dka[d] = ih * d1w(V[ND + 2], w.r);
#pragma unroll
            for (int a = 0; a < ND; ++a) t.s2u[a][d] = ih2 * d2w(V[a], w.r);
            t.s2T[d] = ih2 * d2w(V[ND], w.r);
            if (d == 0) {
                // the node itself sits at window row p - q0
                const int rc = (int)(idx[0] - w.q0);
#pragma unroll
                for (int a = 0; a < ND; ++a) t.u[a] = V[a][rc];
                t.mu = V[ND + 1][rc];
                t.ka = V[ND + 2][rc];
            }
        }
    }
    if (VISC) {
#pragma unroll
        for (int a = 0; a < ND; ++a)
#pragma unroll
            for (int b = 0; b < ND; ++b) t.G[a][b] = Gs[(a * ND + b) * g.nint + ci];
#pragma unroll
        for (int b = 0; b < ND; ++b) {
            // along b: g_ba (a != b) for d_b(g_ba), and along b of g_aa for d_b(g_aa) = Y[b][a]
            Win w;
            int64_t cw[5];
            window_int(g, idx, b, w, cw);
            const double ih = m.invh[b][idx[b]];
#pragma unroll
            for (int a = 0; a < ND; ++a) {
                if (a == b) continue;
                double f[5], h[5];
#pragma unroll
                for (int k = 0; k < 5; ++k) {
                    f[k] = Gs[(b * ND + a) * g.nint + cw[k]];
                    h[k] = Gs[(a * ND + a) * g.nint + cw[k]];
                }
                t.X[a][b] = ih * d1w(f, w.r);
                t.Y[b][a] = ih * d1w(h, w.r);
            }
        }
        visc_assemble<ND>(t, R);
    }
#pragma unroll
    for (int c = 0; c < NC; ++c) Rout[c * g.nint + ci] = R[c];
}

// ---------------------------------------------------------------- store-all
// Work arrays (interior layout, [array][node]):
//   F   ND * NC          (1/h_d) D_d F_d,c
//   G   (ND + 3) * ND    (1/h_b) D_b of u_a, T, mu~, kappa
//   S   (ND + 1) * ND    (1/h_b^2) D2_b of u_a, T
//   X   ND * ND          d_b(g_ba), a != b
//   Y   ND * ND          d_a(g_bb), a != b
struct CWork {
    double *F, *G, *S, *X, *Y;
};

template <int ND, bool VISC>
__global__ void __launch_bounds__(256)
k_cb_first(const double *__restrict__ U, CWork W, Grid g, Phys ph, Metrics m, ColTiles T) {
    constexpr int NC = ND + 2;
    int64_t idx[3];
    if (!node_of_col_thread(g, T, idx)) return;
    const int64_t ci = int_index(g, idx[0], idx[1], idx[2]);
    const int64_t cs = g.enpts;
#pragma unroll
    for (int d = 0; d < ND; ++d) {
        Win w;
        int64_t e[5];
        window_ext<ND>(g, idx, d, w, e);
        double F[NC][5], V[ND + 3][5];
#pragma unroll
        for (int k = 0; k < 5; ++k) {
            CNode<ND> o;
            cnode<ND, VISC>(U, e[k], cs, ph, d, o);
#pragma unroll
            for (int c = 0; c < NC; ++c) F[c][k] = o.F[c];
            if (VISC) {
#pragma unroll
                for (int v = 0; v < ND + 3; ++v) V[v][k] = o.v[v];
            }
        }
        const double ih = m.invh[d][idx[d]];
#pragma unroll
        for (int c = 0; c < NC; ++c) W.F[(d * NC + c) * g.nint + ci] = ih * d1w(F[c], w.r);
        if (VISC) {
#pragma unroll
            for (int v = 0; v < ND + 3; ++v) W.G[(v * ND + d) * g.nint + ci] = ih * d1w(V[v], w.r);
        }
    }
}

template <int ND>
__global__ void __launch_bounds__(256)
k_cb_second(const double *__restrict__ U, CWork W, Grid g, Phys ph, Metrics m, ColTiles T) {
    int64_t idx[3];
    if (!node_of_col_thread(g, T, idx)) return;
    const int64_t ci = int_index(g, idx[0], idx[1], idx[2]);
    const int64_t cs = g.enpts;
#pragma unroll
    for (int b = 0; b < ND; ++b) {
        Win w;
        int64_t e[5];
        window_ext<ND>(g, idx, b, w, e);
        double V[ND + 1][5];
#pragma unroll
        for (int k = 0; k < 5; ++k) {
            CNode<ND> o;
            cnode<ND, true>(U, e[k], cs, ph, b, o);
#pragma unroll
            for (int v = 0; v < ND + 1; ++v) V[v][k] = o.v[v];
        }
        const double ih = m.invh[b][idx[b]];
#pragma unroll
        for (int v = 0; v < ND + 1; ++v) W.S[(v * ND + b) * g.nint + ci] = ih * ih * d2w(V[v], w.r);
        Win wi;
        int64_t cw[5];
        window_int(g, idx, b, wi, cw);
#pragma unroll
        for (int a = 0; a < ND; ++a) {
            if (a == b) continue;
            double f[5], h[5];
#pragma unroll
            for (int k = 0; k < 5; ++k) {
                f[k] = W.G[(b * ND + a) * g.nint + cw[k]];   // g_ba along b
                h[k] = W.G[(a * ND + a) * g.nint + cw[k]];   // g_aa along b
            }
            W.X[(a * ND + b) * g.nint + ci] = ih * d1w(f, wi.r);
            W.Y[(b * ND + a) * g.nint + ci] = ih * d1w(h, wi.r);
        }
    }
}

template <int ND, bool VISC>
__global__ void __launch_bounds__(256)
k_cb_assemble(const double *__restrict__ U, CWork W, Grid g, Phys ph, double *__restrict__ Rout, ColTiles T) {
    constexpr int NC = ND + 2;
    int64_t idx[3];
    if (!node_of_col_thread(g, T, idx)) return;
    const int64_t ci = int_index(g, idx[0], idx[1], idx[2]);
    const int64_t e0 = ext_index(g, idx[0], idx[1], idx[2]);
    double R[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        double s = 0.0;
#pragma unroll
        for (int d = 0; d < ND; ++d) s += W.F[(d * NC + c) * g.nint + ci];
        R[c] = -s;
    }
    if (VISC) {
        VTerms<ND> t;
        CNode<ND> o;
        cnode<ND, true>(U, e0, g.enpts, ph, 0, o);
#pragma unroll
        for (int a = 0; a < ND; ++a) t.u[a] = o.v[a];
        t.mu = o.v[ND + 1];
        t.ka = o.v[ND + 2];
#pragma unroll
        for (int a = 0; a < ND; ++a)
#pragma unroll
            for (int b = 0; b < ND; ++b) {
                t.G[a][b] = W.G[(a * ND + b) * g.nint + ci];
                t.s2u[a][b] = W.S[(a * ND + b) * g.nint + ci];
                t.X[a][b] = a == b ? 0.0 : W.X[(a * ND + b) * g.nint + ci];
                t.Y[a][b] = a == b ? 0.0 : W.Y[(a * ND + b) * g.nint + ci];
            }
#pragma unroll
        for (int b = 0; b < ND; ++b) {
            t.dT[b] = W.G[(ND * ND + b) * g.nint + ci];
            t.dmu[b] = W.G[((ND + 1) * ND + b) * g.nint + ci];
            t.dka[b] = W.G[((ND + 2) * ND + b) * g.nint + ci];
            t.s2T[b] = W.S[(ND * ND + b) * g.nint + ci];
        }
        visc_assemble<ND>(t, R);
    }
#pragma unroll
    for (int c = 0; c < NC; ++c) Rout[c * g.nint + ci] = R[c];
}

inline size_t al256(size_t x) { return (x + 255) & ~size_t(255); }

template <int ND, bool VISC>
hipError_t central_nd(const Grid &g, const Phys &ph, const Metrics &m, const double *U, double *Gs, void *work,
                      double *R, hipStream_t s) {
    const ColTiles T = col_tiles(g);
    const dim3 nb((unsigned)(8 * T.per)), bs(kBX, kBY);
    if (!work) {
        if (VISC) hipLaunchKernelGGL((k_c_grad<ND>), nb, bs, 0, s, U, Gs, g, m, T);
        hipLaunchKernelGGL((k_c_resid<ND, VISC>), nb, bs, 0, s, U, Gs, g, ph, m, R, T);
        return hipGetLastError();
    }
    constexpr int NC = ND + 2;
    const size_t a = sizeof(double) * g.nint;
    char *w = static_cast<char *>(work);
    CWork W;
    W.F = reinterpret_cast<double *>(w);
    w += al256(a * ND * NC);
    W.G = reinterpret_cast<double *>(w);
    w += al256(a * (ND + 3) * ND);
    W.S = reinterpret_cast<double *>(w);
    w += al256(a * (ND + 1) * ND);
    W.X = reinterpret_cast<double *>(w);
    w += al256(a * ND * ND);
    W.Y = reinterpret_cast<double *>(w);
    hipLaunchKernelGGL((k_cb_first<ND, VISC>), nb, bs, 0, s, U, W, g, ph, m, T);
    if (VISC) hipLaunchKernelGGL((k_cb_second<ND>), nb, bs, 0, s, U, W, g, ph, m, T);
    hipLaunchKernelGGL((k_cb_assemble<ND, VISC>), nb, bs, 0, s, U, W, g, ph, R, T);
    return hipGetLastError();
}

}  // namespace

size_t central_work_bytes(const Grid &g, bool viscous) {
    const size_t a = sizeof(double) * g.nint;
    const int nd = g.nd, nc = g.nc;
    size_t b = al256(a * nd * nc);
    if (viscous) b += al256(a * (nd + 3) * nd) + al256(a * (nd + 1) * nd) + 2 * al256(a * nd * nd);
    return b;
}

hipError_t launch_central(const Grid &g, const Phys &ph, const Metrics &m, const double *U, double *Gs, void *work,
                          double *R, hipStream_t s) {
    const bool v = ph.viscous != 0;
    switch (g.nd) {
        case 1: return v ? central_nd<1, true>(g, ph, m, U, Gs, work, R, s) : central_nd<1, false>(g, ph, m, U, Gs, work, R, s);
        case 2: return v ? central_nd<2, true>(g, ph, m, U, Gs, work, R, s) : central_nd<2, false>(g, ph, m, U, Gs, work, R, s);
        default: return v ? central_nd<3, true>(g, ph, m, U, Gs, work, R, s) : central_nd<3, false>(g, ph, m, U, Gs, work, R, s);
    }
}

}  // namespace osbli
