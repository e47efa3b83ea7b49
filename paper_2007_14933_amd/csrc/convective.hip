// Convective residual: characteristic LLF flux reconstruction in each
// direction, section 2.2 (enumerated algorithm), sections
// 2.3-2.5 for the reconstructions.
//
// Thread mapping ("pencil march"): a thread owns one grid line along the sweep
// direction and a segment of it; neighbouring lanes own neighbouring lines
// (adjacent in x for the y and z sweeps, so every load is coalesced).  Each
// thread keeps a six-point register window of the stencil (state + 1/rho, p,
// a computed once per point), marches along the line, computes one interface
// flux per step and the flux difference of the node behind it, so each
// interface is evaluated once (plus one per segment).
//
// The characteristic algebra is written in the local frame (n, t1, t2) of the
// interface: with f_k = u_n U_k + p_k (0, n, u_n) the projected flux is
// g_kj = u_n,k V_kj + p_k (l_j,m . n + l_j,E u_n,k), so only V = L U is
// formed per point, and L, R are never stored as matrices.
#include "convective_launch.hpp"

namespace osbli {
namespace cvl {
// the two fifth-order schemes of every form (plain, precision, routed)
template hipError_t launch_convective_s<OSBLI_WENOZ5> OSBLI_CONVECTIVE_SIG;
template hipError_t launch_convective_s<OSBLI_TENO5> OSBLI_CONVECTIVE_SIG;
}  // namespace cvl

hipError_t launch_convective(const Grid &g, const Phys &ph, const Metrics &m, const double *U, double *R,
                             unsigned *flags, int dir, int first, const uint8_t *mask, int64_t sq, hipStream_t s) {
    if (dir < 0 || dir >= g.nd) return hipErrorInvalidValue;
    switch (ph.scheme) {
        case OSBLI_WENOZ5: return cvl::launch_convective_s<OSBLI_WENOZ5>(g, ph, m, U, R, flags, dir, first, mask, sq, s);
        case OSBLI_TENO5: return cvl::launch_convective_s<OSBLI_TENO5>(g, ph, m, U, R, flags, dir, first, mask, sq, s);
        case OSBLI_TENO6: return cvl::launch_convective_s<OSBLI_TENO6>(g, ph, m, U, R, flags, dir, first, mask, sq, s);
        case OSBLI_WENOJS5:
            return cvl::launch_convective_s<OSBLI_WENOJS5>(g, ph, m, U, R, flags, dir, first, mask, sq, s);
        case OSBLI_WENOZ3: return cvl::launch_convective_s<OSBLI_WENOZ3>(g, ph, m, U, R, flags, dir, first, mask, sq, s);
        case OSBLI_WENOZ7: return cvl::launch_convective_wz7(g, ph, m, U, R, flags, dir, first, mask, sq, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace osbli
