// Boundary conditions through three ghost nodes (section 3.1): periodic,
// extrapolation (zero-gradient copy), isothermal and adiabatic no-slip walls
// (eqs. wall_energy and halo_density and the momentum reflection; the
// adiabatic wall temperature from the one-sided fourth-order closure of
// section 2.6 with dT/dn = 0).  Wall-node values of every wall face are set
// first, then ghosts direction by direction over the full extent of the
// other directions.
#include "bc.hpp"

namespace osbli {
namespace {
using namespace bcd;

// wall node of face (dir, side): momentum 0, rho E = rho_w T_w / (M^2 gamma (gamma-1))
template <int ND>
__global__ void k_wall_node(double *__restrict__ U, Grid g, Phys ph, int dir, int side, int kind, double Tw_iso) {
    const int o1 = dir == 0 ? 1 : 0, o2 = dir == 2 ? 1 : 2;
    const int64_t n1 = g.n[o1], n2 = g.n[o2];
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n1 * n2) return;
    int64_t q[3];
    q[o1] = t % n1;
    q[o2] = t / n1;
    q[dir] = side ? g.n[dir] - 1 : 0;
    const int64_t ew = ext_index(g, q[0], q[1], q[2]);
    const int64_t cs = g.enpts;
    const int64_t sgs = (side ? -1 : 1) * g.es[dir];
    double Tw = Tw_iso;
    if (kind == OSBLI_ADIABATIC_WALL) {
        double u[3], T[5];
#pragma unroll
        for (int mm = 1; mm <= 4; ++mm) T[mm] = temp_at<ND>(U, ew + mm * sgs, cs, ph, u);
        Tw = (48.0 * T[1] - 36.0 * T[2] + 16.0 * T[3] - 3.0 * T[4]) / 25.0;
    }
    const double rw = U[ew];
#pragma unroll
    for (int m = 0; m < ND; ++m) U[ew + (1 + m) * cs] = 0.0;
    U[ew + (ND + 1) * cs] = rw * Tw / (ph.M2 * ph.gamma * ph.gm1);
}

// ghosts of direction dir, both sides
template <int ND>
__global__ void k_ghosts(double *__restrict__ U, Grid g, Phys ph, int dir, int kind0, int kind1) {
    const int o1 = dir == 0 ? 1 : 0, o2 = dir == 2 ? 1 : 2;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 2 * g.e[o1] * g.e[o2]) return;
    ghost_fill<ND>(U, g, ph, dir, kind0, kind1, t);
}

// All directions periodic: every ghost node (edges and corners included)
// copies the interior node its wrapped coordinates name, in one launch (the
// three direction passes compose to the same copies).  Items enumerate the
// ghost region as z-ghost planes (full x, y extent), then y-ghost rows of
// interior planes (full x extent), then x-ghost points of interior rows.
template <int ND>
__global__ void k_ghosts_periodic(double *__restrict__ U, Grid g, int64_t c1, int64_t c2, int64_t total) {
    constexpr int NC = ND + 2;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= total) return;
    const int64_t ex = g.e[0], ey = g.e[1];
    int64_t a[3];  // extended coordinates of the ghost node
    if (t < c1) {
        const int64_t pl = t / (ex * ey), r = t - pl * ex * ey;
        a[0] = r % ex;
        a[1] = r / ex;
        a[2] = pl < g.h[2] ? pl : g.n[2] + pl;
    } else if (t < c1 + c2) {
        const int64_t u = t - c1, rg = 2 * g.h[1];
        a[0] = u % ex;
        const int64_t r = u / ex, jg = r % rg;
        a[1] = jg < g.h[1] ? jg : g.n[1] + jg;
        a[2] = r / rg + g.h[2];
    } else {
        const int64_t u = t - c1 - c2, rg = 2 * g.h[0];
        const int64_t ig = u % rg, r = u / rg;
        a[0] = ig < g.h[0] ? ig : g.n[0] + ig;
        a[1] = r % g.n[1] + g.h[1];
        a[2] = r / g.n[1] + g.h[2];
    }
    int64_t b[3];  // extended coordinates of the source
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const int64_t q = a[d] - g.h[d];
        b[d] = (q < 0 ? q + g.n[d] : (q >= g.n[d] ? q - g.n[d] : q)) + g.h[d];
    }
    const int64_t dst = a[0] + a[1] * g.es[1] + a[2] * g.es[2];
    const int64_t src = b[0] + b[1] * g.es[1] + b[2] * g.es[2];
    double v[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) v[c] = U[src + c * g.enpts];
#pragma unroll
    for (int c = 0; c < NC; ++c) U[dst + c * g.enpts] = v[c];
}

template <int ND>
hipError_t bc_nd(const Grid &g, const Phys &ph, const osbli_params &p, double *U, hipStream_t s) {
    const int bs = 256;
    bool allper = true;
    for (int d = 0; d < ND; ++d) allper = allper && p.bc_kind[d][0] == OSBLI_PERIODIC && p.bc_kind[d][1] == OSBLI_PERIODIC;
    if (allper) {
        const int64_t c1 = 2 * g.h[2] * g.e[0] * g.e[1];
        const int64_t c2 = g.n[2] * 2 * g.h[1] * g.e[0];
        const int64_t c3 = g.n[2] * g.n[1] * 2 * g.h[0];
        const int64_t total = c1 + c2 + c3;
        hipLaunchKernelGGL((k_ghosts_periodic<ND>), dim3((unsigned)((total + bs - 1) / bs)), dim3(bs), 0, s, U, g,
                           c1, c2, total);
        return hipGetLastError();
    }
    for (int d = 0; d < ND; ++d)
        for (int side = 0; side < 2; ++side) {
            const int kind = p.bc_kind[d][side];
            if (kind != OSBLI_ISOTHERMAL_WALL && kind != OSBLI_ADIABATIC_WALL) continue;
            const int o1 = d == 0 ? 1 : 0, o2 = d == 2 ? 1 : 2;
            const int64_t nf = g.n[o1] * g.n[o2];
            hipLaunchKernelGGL((k_wall_node<ND>), dim3((unsigned)((nf + bs - 1) / bs)), dim3(bs), 0, s, U, g, ph, d,
                               side, kind, p.wall_T[d][side]);
            hipError_t e = hipGetLastError();
            if (e != hipSuccess) return e;
        }
    for (int d = 0; d < ND; ++d) {
        const int o1 = d == 0 ? 1 : 0, o2 = d == 2 ? 1 : 2;
        const int64_t nt = 2 * g.e[o1] * g.e[o2];
        hipLaunchKernelGGL((k_ghosts<ND>), dim3((unsigned)((nt + bs - 1) / bs)), dim3(bs), 0, s, U, g, ph, d,
                           p.bc_kind[d][0], p.bc_kind[d][1]);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace

hipError_t launch_bc(const Grid &g, const Phys &ph, const osbli_params &p, double *U, hipStream_t s) {
    switch (g.nd) {
        case 1: return bc_nd<1>(g, ph, p, U, s);
        case 2: return bc_nd<2>(g, ph, p, U, s);
        default: return bc_nd<3>(g, ph, p, U, s);
    }
}

}  // namespace osbli
