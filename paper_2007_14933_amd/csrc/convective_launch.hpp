// Launch templates of the convective sweeps, shared by the translation units
// that instantiate them per reconstruction scheme (each scheme's kernels
// compile in a unit of their own).
#pragma once

#include "sweep.hpp"

namespace osbli {
namespace cvl {
using namespace cf;

template <int ND, int DIR, int SCHEME, bool GEN, bool MIX, bool ROUTE>
hipError_t launch_one(const Grid &g, const Phys &ph, const Metrics &m, const double *U, double *R,
                      unsigned *flags, int first, const uint8_t *mask, int64_t seg_req, hipStream_t s) {
    constexpr int O1 = DIR == 0 ? 1 : 0;
    constexpr int O2 = DIR == 2 ? 1 : 2;
    const int64_t lines = g.n[O1] * g.n[O2];
    const int64_t N = g.n[DIR];
    if (DIR == 0 && !GEN && seg_req <= 0 && N + 1 >= 64) {
        // lanes along x: 63 new interfaces per wave
        const int64_t totalJ = lines * (N + 1);
        const int64_t waves = (totalJ - 2) / 63 + 1;
        const int64_t nb = (waves + kWaves - 1) / kWaves;
        hipLaunchKernelGGL((k_sweep_xl<ND, SCHEME, MIX, ROUTE>), dim3((unsigned)nb), dim3(64 * kWaves), 0, s, U, R,
                           g, ph, m, totalJ, first, flags, mask);
        return hipGetLastError();
    }
    int64_t seg = seg_req > 0 ? seg_req : default_segment(N, lines);
    if (seg > N) seg = N;
    const int64_t nseg = (N + seg - 1) / seg;
    const int64_t waves = ((lines + 63) / 64) * nseg;
    const int bs = 64 * kWaves;
    const int64_t nb = (waves + kWaves - 1) / kWaves;
    hipLaunchKernelGGL((k_sweep<ND, DIR, SCHEME, GEN, MIX, ROUTE>), dim3((unsigned)nb), dim3(bs), 0, s, U, R, g,
                       ph, m, seg, nseg, first, flags, mask);
    return hipGetLastError();
}

template <int ND, int SCHEME, bool GEN, bool MIX, bool ROUTE>
hipError_t launch_dir_r(const Grid &g, const Phys &ph, const Metrics &m, const double *U, double *R,
                        unsigned *flags, int dir, int first, const uint8_t *mask, int64_t sq, hipStream_t s) {
    if (dir == 0) return launch_one<ND, 0, SCHEME, GEN, MIX, ROUTE>(g, ph, m, U, R, flags, first, mask, sq, s);
    if (dir == 1)
        return launch_one<ND, (ND >= 2 ? 1 : 0), SCHEME, GEN, MIX, ROUTE>(g, ph, m, U, R, flags, first, mask, sq, s);
    return launch_one<ND, (ND >= 3 ? 2 : 0), SCHEME, GEN, MIX, ROUTE>(g, ph, m, U, R, flags, first, mask, sq, s);
}

template <int ND, int SCHEME, bool GEN, bool MIX>
hipError_t launch_dir_f(const Grid &g, const Phys &ph, const Metrics &m, const double *U, double *R,
                        unsigned *flags, int dir, int first, const uint8_t *mask, int64_t sq, hipStream_t s) {
    // routing only on separable meshes with TENO5 (validated at set-up)
    if (mask && !GEN && SCHEME == OSBLI_TENO5)
        return launch_dir_r<ND, SCHEME, GEN, MIX, (!GEN && SCHEME == OSBLI_TENO5)>(g, ph, m, U, R, flags, dir, first,
                                                                               mask, sq, s);
    return launch_dir_r<ND, SCHEME, GEN, MIX, false>(g, ph, m, U, R, flags, dir, first, nullptr, sq, s);
}

template <int ND, int SCHEME, bool GEN>
hipError_t launch_dir(const Grid &g, const Phys &ph, const Metrics &m, const double *U, double *R,
                      unsigned *flags, int dir, int first, const uint8_t *mask, int64_t sq, hipStream_t s) {
    // the precision form exists for WENO-Z5 and TENO5 only (validated at set-up)
    if constexpr (SCHEME == OSBLI_WENOZ5 || SCHEME == OSBLI_TENO5)
        if (ph.mixed) return launch_dir_f<ND, SCHEME, GEN, true>(g, ph, m, U, R, flags, dir, first, mask, sq, s);
    return launch_dir_f<ND, SCHEME, GEN, false>(g, ph, m, U, R, flags, dir, first, mask, sq, s);
}

template <int ND, int SCHEME>
hipError_t launch_mesh(const Grid &g, const Phys &ph, const Metrics &m, const double *U, double *R,
                       unsigned *flags, int dir, int first, const uint8_t *mask, int64_t sq, hipStream_t s) {
    if (ND >= 2 && m.general)
        return launch_dir<ND, SCHEME, (ND >= 2)>(g, ph, m, U, R, flags, dir, first, mask, sq, s);
    return launch_dir<ND, SCHEME, false>(g, ph, m, U, R, flags, dir, first, mask, sq, s);
}

// every direction, dimension and mesh kind of one scheme
template <int SCHEME>
hipError_t launch_convective_s(const Grid &g, const Phys &ph, const Metrics &m, const double *U, double *R,
                               unsigned *flags, int dir, int first, const uint8_t *mask, int64_t sq, hipStream_t s) {
    switch (g.nd) {
        case 1: return launch_mesh<1, SCHEME>(g, ph, m, U, R, flags, dir, first, mask, sq, s);
        case 2: return launch_mesh<2, SCHEME>(g, ph, m, U, R, flags, dir, first, mask, sq, s);
        default: return launch_mesh<3, SCHEME>(g, ph, m, U, R, flags, dir, first, mask, sq, s);
    }
}

#define OSBLI_CONVECTIVE_SIG                                                                                 \
    (const Grid &, const Phys &, const Metrics &, const double *, double *, unsigned *, int, int,          \
     const uint8_t *, int64_t, hipStream_t)
extern template hipError_t launch_convective_s<OSBLI_WENOZ5> OSBLI_CONVECTIVE_SIG;
extern template hipError_t launch_convective_s<OSBLI_TENO5> OSBLI_CONVECTIVE_SIG;
extern template hipError_t launch_convective_s<OSBLI_TENO6> OSBLI_CONVECTIVE_SIG;
extern template hipError_t launch_convective_s<OSBLI_WENOJS5> OSBLI_CONVECTIVE_SIG;
extern template hipError_t launch_convective_s<OSBLI_WENOZ3> OSBLI_CONVECTIVE_SIG;
// seventh-order WENO-Z: kernels of its own (eight-point stencils)
hipError_t launch_convective_wz7 OSBLI_CONVECTIVE_SIG;

}  // namespace cvl
}  // namespace osbli
