// Per-item boundary-condition device code (section 3.1), shared by the
// single-grid and the batched launches.
#pragma once

#include "internal.hpp"

namespace osbli {
namespace bcd {

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

// ghosts of direction dir for face item t in [0, 2 e1 e2): (face node over
// the extended range of the other directions, side)
template <int ND>
__device__ __forceinline__ void ghost_fill(double *__restrict__ U, const Grid &g, const Phys &ph, int dir,
                                           int kind0, int kind1, int64_t t) {
    constexpr int NC = ND + 2;
    const int o1 = dir == 0 ? 1 : 0, o2 = dir == 2 ? 1 : 2;
    const int64_t e1 = g.e[o1], e2 = g.e[o2];
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
    // Periodic and extrapolated ghosts: every source value is read before the
    // first ghost is written (sources are nodes inside the line, ghosts lie
    // outside it, so the two sets are disjoint); interleaved copies would
    // wait out the memory latency once per value.
    if (kind == OSBLI_PERIODIC) {
        double v[kGhost][NC];
#pragma unroll
        for (int m = 1; m <= kGhost; ++m) {
            const int64_t es = ew - sg * m * st + sg * N * st;
#pragma unroll
            for (int c = 0; c < NC; ++c) v[m - 1][c] = U[es + c * cs];
        }
#pragma unroll
        for (int m = 1; m <= kGhost; ++m) {
            const int64_t eg = ew - sg * m * st;
#pragma unroll
            for (int c = 0; c < NC; ++c) U[eg + c * cs] = v[m - 1][c];
        }
    } else if (kind == OSBLI_DIRICHLET) {
        // boundary data: the ghosts keep the values the caller set
    } else if (kind == OSBLI_EXTRAPOLATE) {
        double v[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) v[c] = U[ew + c * cs];
#pragma unroll
        for (int m = 1; m <= kGhost; ++m) {
            const int64_t eg = ew - sg * m * st;
#pragma unroll
            for (int c = 0; c < NC; ++c) U[eg + c * cs] = v[c];
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

}  // namespace bcd
}  // namespace osbli
