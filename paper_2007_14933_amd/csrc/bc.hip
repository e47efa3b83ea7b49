// Boundary conditions through three ghost nodes (section 3.1): periodic,
// extrapolation (zero-gradient copy), isothermal and adiabatic no-slip walls
// (eqs. wall_energy and halo_density and the momentum reflection; the
// adiabatic wall temperature from the one-sided fourth-order closure of
// section 2.6 with dT/dn = 0).  Wall-node values of every wall face are set
// first, then ghosts direction by direction over the full extent of the
// other directions.
#include "internal.hpp"

namespace osbli {
namespace {

template <int ND>
__device__ __forceinline__ double temp_at(const double *__restrict__ U, int64_t e, int64_t cs, const Phys &ph,
                                          double (&u)[3]) {
    const double r = U[e];
    const double ri = 1.0 / r;
    double ke = 0.0;
#pragma unroll
    for (int m = 0; m < ND; ++m) {
        const double mm = U[e + (1 + m) * cs];
        u[m] = mm * ri;
        ke += mm * mm;
    }
    const double p = ph.gm1 * (U[e + (ND + 1) * cs] - 0.5 * ke * ri);
    return ph.gamma * ph.M2 * p * ri;
}

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

// ghosts of direction dir, both sides; thread = (face node over the extended
// range of the other directions, side)
template <int ND>
__global__ void k_ghosts(double *__restrict__ U, Grid g, Phys ph, int dir, int kind0, int kind1) {
    constexpr int NC = ND + 2;
    const int o1 = dir == 0 ? 1 : 0, o2 = dir == 2 ? 1 : 2;
    const int64_t e1 = g.e[o1], e2 = g.e[o2];
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 2 * e1 * e2) return;
    const int side = (int)(t / (e1 * e2));
    const int64_t r = t % (e1 * e2);
    int64_t q[3];
    q[o1] = r % e1 - g.h[o1];
    q[o2] = r / e1 - g.h[o2];
    const int64_t N = g.n[dir];
    q[dir] = side ? N - 1 : 0;
    const int kind = side ? kind1 : kind0;
    const int64_t ew = ext_index(g, q[0], q[1], q[2]);
    const int64_t cs = g.enpts;
    const int64_t sg = side ? -1 : 1;
    const int64_t st = g.es[dir];
    if (kind == OSBLI_PERIODIC) {
#pragma unroll
        for (int m = 1; m <= kGhost; ++m) {
            const int64_t eg = ew - sg * m * st;
            const int64_t es = eg + sg * N * st;
#pragma unroll
            for (int c = 0; c < NC; ++c) U[eg + c * cs] = U[es + c * cs];
        }
    } else if (kind == OSBLI_EXTRAPOLATE) {
#pragma unroll
        for (int m = 1; m <= kGhost; ++m) {
            const int64_t eg = ew - sg * m * st;
#pragma unroll
            for (int c = 0; c < NC; ++c) U[eg + c * cs] = U[ew + c * cs];
        }
    } else {
        double uw[3], u1[3];
        const double Tw = temp_at<ND>(U, ew, cs, ph, uw);
        const double T1 = temp_at<ND>(U, ew + sg * st, cs, ph, u1);
        const double rw = U[ew];
        const double pw = rw * Tw / (ph.gamma * ph.M2);
#pragma unroll
        for (int m = 1; m <= kGhost; ++m) {
            double ui[3];
            (void)temp_at<ND>(U, ew + sg * m * st, cs, ph, ui);
            const double Tg = (m + 1) * Tw - m * T1;
            const double rg = ph.gamma * ph.M2 * pw / Tg;
            const int64_t eg = ew - sg * m * st;
            double ke = 0.0;
            U[eg] = rg;
#pragma unroll
            for (int c = 0; c < ND; ++c) {
                U[eg + (1 + c) * cs] = -rg * ui[c];
                ke += ui[c] * ui[c];
            }
            U[eg + (ND + 1) * cs] = pw / ph.gm1 + 0.5 * rg * ke;
        }
    }
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
