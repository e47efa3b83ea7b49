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

template <int ND>
hipError_t bc_nd(const Grid &g, const Phys &ph, const osbli_params &p, double *U, hipStream_t s) {
    const int bs = 256;
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
