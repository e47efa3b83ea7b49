// Central-difference building blocks shared by the viscous / finish kernels
// and the fourth-order central path (section 2.6): the first- and
// second-derivative operators on a line with their one-sided closures, and
// the plane-by-plane node mapping of the pointwise kernels.
#pragma once

#include "internal.hpp"

namespace osbli {

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

// second derivative per unit index at position p (section 2.6):
// (-f_{p-2} + 16 f_{p-1} - 30 f_p + 16 f_{p+1} - f_{p+2}) / 12 in the interior
// and on periodic lines, the printed one-sided closures at 0 and 1, mirrored
// at N - 1 and N - 2 (written on differences from the centre or the
// boundary node, so constants give exactly 0)
template <class At>
__device__ __forceinline__ double d2line(const At &at, int64_t p, int64_t N, bool periodic) {
    if (periodic || (p >= 2 && p <= N - 3)) {
        const double c = at(p);
        return (4.0 / 3.0) * ((at(p + 1) - c) + (at(p - 1) - c)) - (1.0 / 12.0) * ((at(p + 2) - c) + (at(p - 2) - c));
    }
    const int64_t m = p <= 1 ? 1 : -1, b = p <= 1 ? 0 : N - 1;
    const double f0 = at(b);
    const double d1 = at(b + m) - f0, d2 = at(b + 2 * m) - f0, d3 = at(b + 3 * m) - f0, d4 = at(b + 4 * m) - f0;
    if (p == 0 || p == N - 1) return (-104.0 * d1 + 114.0 * d2 - 56.0 * d3 + 11.0 * d4) * (1.0 / 12.0);
    return (-20.0 * d1 + 6.0 * d2 + 4.0 * d3 - d4) * (1.0 / 12.0);
}

// pointwise kernels: blocks of 64 x 4 threads over (i, j) of one k plane
constexpr int kBX = 64, kBY = 4;

// the plain 3D grid: blockIdx (x, y) over the plane's tiles, blockIdx.z the plane
__device__ __forceinline__ bool node_of_plane_thread(const Grid &g, int64_t (&idx)[3]) {
    idx[0] = (int64_t)blockIdx.x * kBX + threadIdx.x;
    idx[1] = (int64_t)blockIdx.y * kBY + threadIdx.y;
    idx[2] = blockIdx.z;
    return idx[0] < g.n[0] && idx[1] < g.n[1];
}

inline dim3 node_grid(const Grid &g) {
    return dim3((unsigned)((g.n[0] + kBX - 1) / kBX), (unsigned)((g.n[1] + kBY - 1) / kBY), (unsigned)g.n[2]);
}

}  // namespace osbli
