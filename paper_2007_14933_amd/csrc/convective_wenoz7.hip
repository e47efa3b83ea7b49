// Convective sweeps with seventh-order WENO-Z (section 5.2), plain FP64
// form, separable meshes.  The reconstruction reads eight points per
// interface, so this scheme has kernels of its own.  Along x a wave owns 64
// consecutive interfaces of one line (63 new nodes), each lane evaluates the
// characteristic flux of its interface from the eight points i-3 .. i+4
// (the wave's 71 points loaded and finished once, into LDS), and the node
// between two lanes takes the
// difference of their fluxes (the left one by a lane shuffle); along y and
// z the lanes lie across 64 consecutive x lines and march.  At the two
// outermost interfaces of a line the stencil reaches one node past the
// three ghost layers: that node is the wrapped interior node on periodic
// lines and the third ghost layer again otherwise.
#include "convective_launch.hpp"

namespace osbli {
namespace cvl {
namespace {

template <int ND, int DIR>
__global__ void __launch_bounds__(64 * kWaves)
k_sweep_wz7(const double *__restrict__ U, double *__restrict__ R, Grid g, Phys ph, Metrics m, int64_t chunks,
            int64_t waves, int first, unsigned *flags) {
    constexpr int NC = ND + 2;
    constexpr int NT = ND - 1;
    constexpr int O1 = DIR == 0 ? 1 : 0;
    constexpr int O2 = DIR == 2 ? 1 : 2;
    const int64_t w = (int64_t)blockIdx.x * kWaves + (threadIdx.x >> 6);
    if (w >= waves) return;  // wave-uniform; no block-wide synchronisation below
    const int lane = threadIdx.x & 63;
    const int64_t line = w / chunks, chunk = w - line * chunks;
    const int64_t N = g.n[DIR];
    // this lane's interface p + 1/2 (p = -1 .. N-1); lanes past the line end
    // write nothing
    const int64_t praw = chunk * 63 - 1 + lane;
    const int64_t p = praw < N ? praw : N - 1;
    int64_t q[3];
    q[DIR] = 0;
    q[O1] = line % g.n[O1];
    q[O2] = line / g.n[O1];
    const int64_t base = ext_index(g, q[0], q[1], q[2]);
    const int64_t st = g.es[DIR], cs = g.enpts;
    const bool per = g.periodic[DIR] != 0;
    const int64_t gl = g.h[DIR];
    bool bad = false;
    // the wave's 71 points (lane 0's stencil start .. lane 63's end), each
    // loaded and finished once into LDS: lane l stages slot l, lanes 0..6
    // also slots 64..70; slot k holds position (chunk * 63 - 1) - 3 + k
    __shared__ double sp[kWaves][NC + 3][72];
    double(*const sw)[72] = sp[threadIdx.x >> 6];
    const int64_t pos0 = chunk * 63 - 4;
    auto stage = [&](int slot) {
        int64_t pos = pos0 + slot;
        if (pos < -gl) pos = per ? pos + N : -gl;
        if (pos > N - 1 + gl) pos = per ? pos - N : N - 1 + gl;
        Pt<ND> pt;
#pragma unroll
        for (int c = 0; c < NC; ++c) pt.U[c] = U[base + pos * st + c * cs];
        finish_point<ND>(ph, pt, bad);
#pragma unroll
        for (int c = 0; c < NC; ++c) sw[c][slot] = pt.U[c];
        sw[NC][slot] = pt.ri;
        sw[NC + 1][slot] = pt.p;
        sw[NC + 2][slot] = pt.a;
    };
    stage(lane);
    if (lane < 7) stage(64 + lane);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // this lane's stencil p - 3 .. p + 4 is slots lane .. lane + 7 (lanes
    // past the line end read valid points and write nothing)
    Loc<ND> P[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const int sl = lane + k;
        P[k].r = sw[0][sl];
        P[k].mn = sw[1 + DIR][sl];
        if (NT >= 1) P[k].mt[0] = sw[1 + Axes<ND, DIR>::T1][sl];
        if (NT >= 2) P[k].mt[1] = sw[1 + Axes<ND, DIR>::T2][sl];
        P[k].E = sw[ND + 1][sl];
        P[k].p = sw[NC + 1][sl];
        P[k].a = sw[NC + 2][sl];
        P[k].ri = sw[NC][sl];
    }
    double Fr, Fn, Ft[2], FE;
    char_flux<ND, OSBLI_WENOZ7, true, 8>(P, ph, Fr, Fn, Ft, FE);
    double F[NC];
    F[0] = Fr;
    F[1 + DIR] = Fn;
    if (NT >= 1) F[1 + Axes<ND, DIR>::T1] = Ft[0];
    if (NT >= 2) F[1 + Axes<ND, DIR>::T2] = Ft[1];
    F[NC - 1] = FE;
    double Fl[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) Fl[c] = __shfl_up(F[c], 1, 64);
    // node p: between the interfaces of lanes lane - 1 and lane
    if (lane >= 1 && praw >= 0 && praw < N) {
        const double sc = m.invh[DIR][p];
        const int64_t oi = int_index(g, q[0], q[1], q[2]) + p * g.is[DIR];
        double v[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) v[c] = -sc * (F[c] - Fl[c]);
        add_residual<NC>(R, g.nint, oi, v, first);
    }
    if (bad) atomicOr(flags, kFlagNonPhys);
}

// y and z: lanes across 64 consecutive lines (consecutive x, so every point
// load of the wave is one contiguous row), each lane marching its line over
// a segment with its eight stencil points in registers (one new point, with
// its 1/rho, p and a, per step): the flux of interface f, the node f from
// this flux and the previous one (kept in registers)
template <int ND, int DIR>
__global__ void __launch_bounds__(64 * kWaves)
k_sweep_wz7_march(const double *__restrict__ U, double *__restrict__ R, Grid g, Phys ph, Metrics m, int64_t seg,
                  int64_t nseg, int64_t waves, int first, unsigned *flags) {
    constexpr int NC = ND + 2;
    constexpr int NT = ND - 1;
    constexpr int O1 = DIR == 0 ? 1 : 0;
    constexpr int O2 = DIR == 2 ? 1 : 2;
    const int64_t w = (int64_t)blockIdx.x * kWaves + (threadIdx.x >> 6);
    if (w >= waves) return;  // wave-uniform; no block-wide synchronisation below
    const int lane = threadIdx.x & 63;
    const int64_t sg = w % nseg, line0 = (w / nseg) * 64;
    const int64_t lines = g.n[O1] * g.n[O2];
    const int64_t line = line0 + lane;
    const bool active = line < lines;
    const int64_t lc = active ? line : lines - 1;
    const int64_t N = g.n[DIR];
    const int64_t p0 = sg * seg, p1 = p0 + seg < N ? p0 + seg : N;
    int64_t q[3];
    q[DIR] = 0;
    q[O1] = lc % g.n[O1];
    q[O2] = lc / g.n[O1];
    const int64_t base = ext_index(g, q[0], q[1], q[2]);
    const int64_t ibase = int_index(g, q[0], q[1], q[2]);
    const int64_t st = g.es[DIR], cs = g.enpts;
    const bool per = g.periodic[DIR] != 0;
    const int64_t gl = g.h[DIR];
    const double *__restrict__ ih = m.invh[DIR];
    bool bad = false;
    // the point at position pos (outer-node reading past the ghost layers)
    auto point = [&](int64_t pos, Loc<ND> &P) {
        if (pos < -gl) pos = per ? pos + N : -gl;
        if (pos > N - 1 + gl) pos = per ? pos - N : N - 1 + gl;
        Pt<ND> pt;
#pragma unroll
        for (int c = 0; c < NC; ++c) pt.U[c] = U[base + pos * st + c * cs];
        finish_point<ND>(ph, pt, bad);
        P.r = pt.U[0];
        P.mn = pt.U[1 + DIR];
        if (NT >= 1) P.mt[0] = pt.U[1 + Axes<ND, DIR>::T1];
        if (NT >= 2) P.mt[1] = pt.U[1 + Axes<ND, DIR>::T2];
        P.E = pt.U[ND + 1];
        P.p = pt.p;
        P.a = pt.a;
        P.ri = pt.ri;
    };
    // window of the eight stencil points f-3 .. f+4, one new point per step
    Loc<ND> P[8];
#pragma unroll
    for (int k = 1; k < 8; ++k) point(p0 - 5 + k, P[k]);
    double Fp[NC];
    for (int64_t f = p0 - 1; f < p1; ++f) {
#pragma unroll
        for (int k = 0; k < 7; ++k) P[k] = P[k + 1];
        point(f + 4, P[7]);
        double Fr, Fn, Ft[2], FE;
        char_flux<ND, OSBLI_WENOZ7, true, 8>(P, ph, Fr, Fn, Ft, FE);
        double F[NC];
        F[0] = Fr;
        F[1 + DIR] = Fn;
        if (NT >= 1) F[1 + Axes<ND, DIR>::T1] = Ft[0];
        if (NT >= 2) F[1 + Axes<ND, DIR>::T2] = Ft[1];
        F[NC - 1] = FE;
        if (f >= p0 && active) {
            const double sc = ih[f];
            double v[NC];
#pragma unroll
            for (int c = 0; c < NC; ++c) v[c] = -sc * (F[c] - Fp[c]);
            add_residual<NC>(R, g.nint, ibase + f * g.is[DIR], v, first);
        }
#pragma unroll
        for (int c = 0; c < NC; ++c) Fp[c] = F[c];
    }
    if (bad) atomicOr(flags, kFlagNonPhys);
}

template <int ND, int DIR>
hipError_t launch_wz7_dir(const Grid &g, const Phys &ph, const Metrics &m, const double *U, double *R,
                          unsigned *flags, int first, hipStream_t s) {
    constexpr int O1 = DIR == 0 ? 1 : 0;
    constexpr int O2 = DIR == 2 ? 1 : 2;
    const int64_t lines = g.n[O1] * g.n[O2];
    const int64_t N = g.n[DIR];
    if (DIR != 0) {
        const int64_t seg = default_segment(N, lines);
        const int64_t nseg = (N + seg - 1) / seg;
        const int64_t waves = ((lines + 63) / 64) * nseg;
        const int64_t nb = (waves + kWaves - 1) / kWaves;
        hipLaunchKernelGGL((k_sweep_wz7_march<ND, DIR>), dim3((unsigned)nb), dim3(64 * kWaves), 0, s, U, R, g, ph, m,
                           seg, nseg, waves, first, flags);
        return hipGetLastError();
    }
    const int64_t chunks = (N + 62) / 63;
    const int64_t waves = lines * chunks;
    const int64_t nb = (waves + kWaves - 1) / kWaves;
    hipLaunchKernelGGL((k_sweep_wz7<ND, DIR>), dim3((unsigned)nb), dim3(64 * kWaves), 0, s, U, R, g, ph, m, chunks,
                       waves, first, flags);
    return hipGetLastError();
}

template <int ND>
hipError_t launch_wz7_nd(const Grid &g, const Phys &ph, const Metrics &m, const double *U, double *R,
                         unsigned *flags, int dir, int first, hipStream_t s) {
    if (dir == 0) return launch_wz7_dir<ND, 0>(g, ph, m, U, R, flags, first, s);
    if (dir == 1) return launch_wz7_dir<ND, (ND >= 2 ? 1 : 0)>(g, ph, m, U, R, flags, first, s);
    return launch_wz7_dir<ND, (ND >= 3 ? 2 : 0)>(g, ph, m, U, R, flags, first, s);
}

}  // namespace

// separable meshes only (validated at set-up); no routing, FP64 form
hipError_t launch_convective_wz7(const Grid &g, const Phys &ph, const Metrics &m, const double *U, double *R,
                                 unsigned *flags, int dir, int first, const uint8_t *, int64_t, hipStream_t s) {
    if (m.general) return hipErrorInvalidValue;
    switch (g.nd) {
        case 1: return launch_wz7_nd<1>(g, ph, m, U, R, flags, dir, first, s);
        case 2: return launch_wz7_nd<2>(g, ph, m, U, R, flags, dir, first, s);
        default: return launch_wz7_nd<3>(g, ph, m, U, R, flags, dir, first, s);
    }
}

}  // namespace cvl
}  // namespace osbli
