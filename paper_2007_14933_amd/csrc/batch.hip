// Batched advance of many independent 2D problems of uneven size: every
// substage is one graph of persistent kernels, each of which walks a tile
// queue covering all problems (a tile belongs to one problem; prefix tables
// map a tile index to its problem).  Per-problem dt, time and active flag
// live on the device, so the captured graphs contain no host logic.  The
// per-tile work is the single-grid code (sweep_wave, ghost_fill,
// sensor_item), so a batched problem evolves bit for bit like a solo one.
#include <stdarg.h>
#include <stdio.h>

#include <new>
#include <vector>

#include "bc.hpp"
#include "point.hpp"
#include "sensor.hpp"
#include "sweep.hpp"

namespace osbli {

namespace {
using namespace cf;
using namespace bcd;
using namespace sn;

constexpr int kPT = 256;  // points (or interfaces) per tile of the pointwise kernels

// table index of the tile: the p with off[p] <= item < off[p + 1]
__device__ __forceinline__ int find_prob(const int64_t *__restrict__ off, int P, int64_t item) {
    int lo = 0, hi = P;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (off[mid] <= item) lo = mid;
        else hi = mid;
    }
    return lo;
}

__device__ __forceinline__ Metrics sep_metrics(const BProb &b) {
    Metrics m;
    m.general = 0;
    m.invh[0] = b.invh[0];
    m.invh[1] = b.invh[1];
    m.invh[2] = b.invh[2];
    m.S = nullptr;
    m.J = nullptr;
    return m;
}

__global__ void k_b_dt_reset(BState *st, int P) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < P) st[p].smax = 0ull;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}

// dt denominator of each problem (separable 2D meshes), max per problem.
// Each block walks a contiguous run of tiles and issues one atomic max per
// problem it touches (tiles of a problem are contiguous).
__device__ __forceinline__ void b_dt_flush(BState *st, int p, double run, double *part) {
    run = wave_max(run);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = run;
    __syncthreads();
    if (threadIdx.x == 0) {
        const double m = fmax(fmax(part[0], part[1]), fmax(part[2], part[3]));
        atomicMax(&st[p].smax, (unsigned long long)__double_as_longlong(m));
    }
    __syncthreads();
}

__global__ void __launch_bounds__(256)
k_b_dt(const BProb *__restrict__ pr, BState *st, const int64_t *__restrict__ off, int P, int64_t total, Phys ph) {
    __shared__ double part[4];
    const int64_t per = (total + gridDim.x - 1) / gridDim.x;
    const int64_t t0 = (int64_t)blockIdx.x * per;
    const int64_t t1 = t0 + per < total ? t0 + per : total;
    int cur = -1;
    double run = 0.0;
    for (int64_t tile = t0; tile < t1; ++tile) {
        const int p = find_prob(off, P, tile);  // block-uniform
        if (p != cur) {
            if (cur >= 0) b_dt_flush(st, cur, run, part);
            cur = p;
            run = 0.0;
        }
        const BProb &b = pr[p];
        const int64_t ci = (tile - off[p]) * kPT + threadIdx.x;
        if (st[p].active && ci < b.g.nint) {
            const int64_t idx[3] = {ci % b.g.n[0], ci / b.g.n[0], 0};
            run = fmax(run, dt_node<2, false>(b.U, b.g, ph, sep_metrics(b), idx));
        }
    }
    if (cur >= 0) b_dt_flush(st, cur, run, part);
}

__global__ void k_b_dt_final(BState *st, int P, double cfl, unsigned *flags) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    if (!st[p].active) {
        st[p].dt = 0.0;
        return;
    }
    const double smax = __longlong_as_double((long long)st[p].smax);
    double dt = smax > 0.0 ? cfl / smax : 0.0;
    if (!(smax < __builtin_inf())) {
        dt = 0.0;
        atomicOr(flags, kFlagNonPhys);
    }
    if (st[p].t + dt > st[p].tend) dt = st[p].tend - st[p].t;
    st[p].dt = dt;
}

template <int DIR, int SCHEME, bool MIX, bool ROUTE>
__global__ void __launch_bounds__(256, 2)
k_b_sweep(const BProb *__restrict__ pr, const BState *__restrict__ st, const int64_t *__restrict__ off, int P,
          int64_t total, Phys ph, int first, unsigned *flags) {
    __shared__ double sbuf[DIR == 0 ? kWaves : 1][4][kChunk][64];
    __shared__ double abuf[DIR == 0 ? 1 : kWaves][2][5][64];
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t nw = (int64_t)gridDim.x * kWaves;
    for (int64_t wt = (int64_t)blockIdx.x * kWaves + wv; wt < total; wt += nw) {
        const int p = find_prob(off, P, wt);
        if (!st[p].active) continue;
        const BProb &b = pr[p];
        const int64_t local = wt - off[p];
        const int64_t sg = local / b.wpl[DIR];
        const int64_t line0 = (local - sg * b.wpl[DIR]) << 6;
        const Metrics m = sep_metrics(b);
        const uint8_t *mk = ROUTE ? b.mask[DIR] : nullptr;
        if constexpr (DIR != 0) {
            if ((line0 % b.g.n[0]) + 64 <= b.g.n[0] && line0 + 64 <= b.g.n[0] * b.g.n[2])  // 64 consecutive x nodes
                sweep_wave<2, DIR, SCHEME, false, MIX, ROUTE, true>(b.U, b.R, b.g, ph, m, b.seg[DIR], sg, line0,
                                                                    first, flags, mk, sbuf[0], abuf[wv]);
            else
                sweep_wave<2, DIR, SCHEME, false, MIX, ROUTE, false>(b.U, b.R, b.g, ph, m, b.seg[DIR], sg, line0,
                                                                     first, flags, mk, sbuf[0], abuf[wv]);
        } else {
            sweep_wave<2, DIR, SCHEME, false, MIX, ROUTE, false>(b.U, b.R, b.g, ph, m, b.seg[DIR], sg, line0, first,
                                                                 flags, mk, sbuf[wv], abuf[0]);
        }
    }
}

// x sweep of the problems with rows of >= 64 interfaces: lanes along x, the
// mapping of the single-grid x sweep (63 new interfaces per wave)
template <int SCHEME, bool MIX, bool ROUTE>
__global__ void __launch_bounds__(256, 3)
k_b_sweep_xl(const BProb *__restrict__ pr, const BState *__restrict__ st, const int64_t *__restrict__ off, int P,
             int64_t total, Phys ph, int first, unsigned *flags) {
    __shared__ XlLds<2> sm[kWaves];
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t nw = (int64_t)gridDim.x * kWaves;
    for (int64_t wt = (int64_t)blockIdx.x * kWaves + wv; wt < total; wt += nw) {
        const int p = find_prob(off, P, wt);
        if (!st[p].active) continue;
        const BProb &b = pr[p];
        const int64_t local = wt - off[p];
        const Metrics m = sep_metrics(b);
        const int64_t totalJ = b.g.n[1] * (b.g.n[0] + 1);
        // a tile is b.xlpt consecutive 63-interface runs of the problem
        const int nrun = b.xlpt;
        for (int k = 0; k < nrun; ++k) {
            const int64_t J0 = (local * nrun + k) * 63;
            if (J0 + 1 >= totalJ) break;  // wave-uniform
            sweep_x_lanes<2, SCHEME, MIX, ROUTE>(b.U, b.R, b.g, ph, m, J0, totalJ, first, flags,
                                                 ROUTE ? b.mask[0] : nullptr, sm[wv]);
        }
    }
}

// RK stage update (inviscid)
__global__ void __launch_bounds__(256)
k_b_finish(const BProb *__restrict__ pr, const BState *__restrict__ st, const int64_t *__restrict__ off, int P,
           int64_t total, RkStage rs) {
    for (int64_t tile = blockIdx.x; tile < total; tile += gridDim.x) {
        const int p = find_prob(off, P, tile);
        if (!st[p].active) continue;
        const BProb &b = pr[p];
        const int64_t ci = (tile - off[p]) * kPT + threadIdx.x;
        if (ci >= b.g.nint) continue;
        const int64_t e0 = ext_index(b.g, ci % b.g.n[0], ci / b.g.n[0], 0);
        const double dt = st[p].dt;
#pragma unroll
        for (int c = 0; c < 4; ++c)
            rk_point(rs, dt, b.R[c * b.g.nint + ci], b.dU + c * b.g.nint + ci, b.U + c * b.g.enpts + e0);
    }
}

__global__ void __launch_bounds__(256)
k_b_bc(const BProb *__restrict__ pr, const BState *__restrict__ st, const int64_t *__restrict__ off, int P,
       int64_t total, Phys ph, int dir) {
    for (int64_t it = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; it < total;
         it += (int64_t)gridDim.x * blockDim.x) {
        const int p = find_prob(off, P, it);
        if (!st[p].active) continue;
        const BProb &b = pr[p];
        ghost_fill<2>(b.U, b.g, ph, dir, b.bc[dir][0], b.bc[dir][1], it - off[p]);
    }
}

template <int DIR>
__global__ void __launch_bounds__(256)
k_b_sensor(const BProb *__restrict__ pr, const BState *__restrict__ st, const int64_t *__restrict__ off, int P,
           int64_t total, Phys ph, const uint16_t *__restrict__ w, float zcut) {
    for (int64_t tile = blockIdx.x; tile < total; tile += gridDim.x) {
        const int p = find_prob(off, P, tile);
        if (!st[p].active) continue;
        const BProb &b = pr[p];
        const int64_t t = (tile - off[p]) * kPT + threadIdx.x;
        sensor_item<2, DIR>(b.U, b.g, ph, w, zcut, b.mask[DIR], t);
    }
}

__global__ void k_b_tadvance(BState *st, int P) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P || !st[p].active) return;
    st[p].t += st[p].dt;
    st[p].active = st[p].t < st[p].tend;
}

}  // namespace

static unsigned grid_of(int64_t items, int64_t per_block, unsigned cap) {
    int64_t nb = (items + per_block - 1) / per_block;
    if (nb < 1) nb = 1;
    if (nb > cap) nb = cap;
    return (unsigned)nb;
}

template <int SCHEME, bool MIX, bool ROUTE>
static hipError_t b_sweeps(const BProb *pr, const BState *st, const BatchTables &T, int P, const Phys &ph,
                           unsigned *flags, int nblk, hipStream_t s) {
    const unsigned cx = nblk > 0 ? (unsigned)nblk : 2048u, cm = nblk > 0 ? (unsigned)nblk : 1024u;
    if (T.tot_wx > 0)
        hipLaunchKernelGGL((k_b_sweep_xl<SCHEME, MIX, ROUTE>), dim3(grid_of(T.tot_wx, kWaves, cx)), dim3(256), 0, s,
                           pr, st, T.wx, P, T.tot_wx, ph, 1, flags);
    if (T.tot_w[0] > 0)
        hipLaunchKernelGGL((k_b_sweep<0, SCHEME, MIX, ROUTE>), dim3(grid_of(T.tot_w[0], kWaves, cm)), dim3(256), 0,
                           s, pr, st, T.w[0], P, T.tot_w[0], ph, 1, flags);
    hipLaunchKernelGGL((k_b_sweep<1, SCHEME, MIX, ROUTE>), dim3(grid_of(T.tot_w[1], kWaves, cm)), dim3(256), 0, s,
                       pr, st, T.w[1], P, T.tot_w[1], ph, 0, flags);
    return hipGetLastError();
}

hipError_t launch_batch_stage(const BProb *pr, BState *st, const BatchTables &T, int P, const Phys &ph, int stage,
                              double cfl, int route, const uint16_t *w, float zcut, unsigned *flags, int sweep_blocks,
                              hipStream_t s) {
    if (stage == 0) {
        hipLaunchKernelGGL(k_b_dt_reset, dim3((P + 255) / 256), dim3(256), 0, s, st, P);
        hipLaunchKernelGGL(k_b_dt, dim3(grid_of(T.tot_pt, 1, 2048)), dim3(256), 0, s, pr, st, T.pt, P, T.tot_pt, ph);
        hipLaunchKernelGGL(k_b_dt_final, dim3((P + 255) / 256), dim3(256), 0, s, st, P, cfl, flags);
        if (route) {
            hipLaunchKernelGGL(k_b_sensor<0>, dim3(grid_of(T.tot_s[0], 1, 2048)), dim3(256), 0, s, pr, st, T.s[0], P,
                               T.tot_s[0], ph, w, zcut);
            hipLaunchKernelGGL(k_b_sensor<1>, dim3(grid_of(T.tot_s[1], 1, 2048)), dim3(256), 0, s, pr, st, T.s[1], P,
                               T.tot_s[1], ph, w, zcut);
        }
    }
    hipError_t e;
    const bool mix = ph.mixed != 0;
    if (ph.scheme == OSBLI_WENOZ5) {
        e = mix ? b_sweeps<OSBLI_WENOZ5, true, false>(pr, st, T, P, ph, flags, sweep_blocks, s)
                : b_sweeps<OSBLI_WENOZ5, false, false>(pr, st, T, P, ph, flags, sweep_blocks, s);
    } else if (route) {
        e = mix ? b_sweeps<OSBLI_TENO5, true, true>(pr, st, T, P, ph, flags, sweep_blocks, s)
                : b_sweeps<OSBLI_TENO5, false, true>(pr, st, T, P, ph, flags, sweep_blocks, s);
    } else {
        e = mix ? b_sweeps<OSBLI_TENO5, true, false>(pr, st, T, P, ph, flags, sweep_blocks, s)
                : b_sweeps<OSBLI_TENO5, false, false>(pr, st, T, P, ph, flags, sweep_blocks, s);
    }
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_b_finish, dim3(grid_of(T.tot_pt, 1, 2048)), dim3(256), 0, s, pr, st, T.pt, P, T.tot_pt,
                       rk3_stage(stage));
    for (int d = 0; d < 2; ++d)
        hipLaunchKernelGGL(k_b_bc, dim3(grid_of(T.tot_f[d], 256, 1024)), dim3(256), 0, s, pr, st, T.f[d], P,
                           T.tot_f[d], ph, d);
    if (stage == 2) hipLaunchKernelGGL(k_b_tadvance, dim3((P + 255) / 256), dim3(256), 0, s, st, P);
    return hipGetLastError();
}

}  // namespace osbli
