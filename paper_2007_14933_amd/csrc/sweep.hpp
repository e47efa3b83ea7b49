// Per-wave body of the convective pencil sweep (shared by the single-grid
// and the batched launches).
#pragma once

#include "charflux.hpp"

namespace osbli {
namespace cf {

constexpr int kChunk = 8;   // x-points staged per cooperative load (x sweep)
constexpr int kWaves = 4;   // waves per block

// R += v (first: R = v) over the components of one node, with every load
// issued before the first store: the stores could alias the later loads as
// far as the compiler knows, so one load-add-store per component would wait
// out the memory latency once per component.
template <int NC>
__device__ __forceinline__ void add_residual(double *__restrict__ R, int64_t nint, int64_t oi,
                                             const double (&v)[NC], int first) {
    if (first) {
#pragma unroll
        for (int c = 0; c < NC; ++c) R[c * nint + oi] = v[c];
    } else {
        double old[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) old[c] = R[c * nint + oi];
#pragma unroll
        for (int c = 0; c < NC; ++c) R[c * nint + oi] = old[c] + v[c];
    }
}

template <int ND, int DIR>
struct Axes {
    static constexpr int T1 = (DIR + 1) % ND;
    static constexpr int T2 = (DIR + 2) % ND;
};

template <int ND>
using SweepLds = double[ND + 2][kChunk][64];

// ahead-load buffer of one wave of a y or z sweep: two slots of one point's
// NC component rows (plus a spare row for odd NC)
template <int ND>
using AheadLds = double[2][ND + 3][64];

// The work of one wave: lines line0 .. line0+63 (clamped), segment sg of
// length seg along DIR.  sbuf: this wave's staging buffer (x sweep only);
// ab: this wave's ahead-load buffer (y and z sweeps).
template <int ND, int DIR, int SCHEME, bool GEN, bool MIX, bool ROUTE, bool AHEAD>
__device__ __forceinline__ void sweep_wave(const double *__restrict__ U, double *__restrict__ R, const Grid &g,
                                           const Phys &ph, const Metrics &m, int64_t seg, int64_t sg, int64_t line0,
                                           int first, unsigned *flags, const uint8_t *__restrict__ mask,
                                           SweepLds<ND> &sb, AheadLds<ND> &ab) {
    constexpr int NC = ND + 2;
    constexpr int NT = ND - 1;
    constexpr int O1 = DIR == 0 ? 1 : 0;
    constexpr int O2 = DIR == 2 ? 1 : 2;
    // 1/h along the line, read only for the kernel's lifetime: read through
    // the constant address space, the wave-uniform per-node factor is a
    // scalar load (as a vector load, waiting for it waited for every vector
    // memory operation issued before it)
    const __attribute__((address_space(4))) double *ih = (const __attribute__((address_space(4))) double *)m.invh[DIR];
    const int64_t n1 = g.n[O1], n2 = g.n[O2], N = g.n[DIR];
    const int64_t lines = n1 * n2;
    const int lane = threadIdx.x & 63;
    const int64_t line = line0 + lane;
    const bool active = line < lines;
    const int64_t lc = active ? line : lines - 1;
    const int64_t p0 = sg * seg;
    const int64_t p1 = p0 + seg < N ? p0 + seg : N;
    int64_t q[3];
    q[DIR] = 0;
    q[O1] = lc % n1;
    q[O2] = lc / n1;
    const int64_t base = ext_index(g, q[0], q[1], q[2]);
    const int64_t st = g.es[DIR];
    const int64_t cs = g.enpts;
    const int64_t ibase = int_index(g, q[0], q[1], q[2]);
    const int64_t ist = g.is[DIR];
    bool bad = false;

    // Ahead-loading (AHEAD: y and z sweeps of separable meshes, for waves
    // whose 64 lines are 64 consecutive nodes of one x row, so that each
    // component of a point is one contiguous 512-byte row): the point needed
    // by the next step is copied from HBM straight into LDS while this step
    // computes (global-to-LDS loads, 16 bytes per lane: lanes 0..31 carry one
    // component row, lanes 32..63 the next), and the step after reads it from
    // LDS; without this the march waits out one HBM latency per step.  The
    // caller picks the variant per wave; the two are separate code, so
    // neither pays the other's registers.
    static_assert(!AHEAD || (DIR != 0 && !GEN), "ahead-loading is for y and z sweeps of separable meshes");
    constexpr bool ahead = AHEAD;
    int64_t base0 = 0;
    if (ahead) {
        int64_t q0[3];
        q0[DIR] = 0;
        q0[O1] = line0 % n1;
        q0[O2] = line0 / n1;
        base0 = ext_index(g, q0[0], q0[1], q0[2]);  // lane l's line starts at base0 + l
    }
    auto load_ahead = [&](int64_t qp, int slot) {
        const int half = lane >> 5;
        const int64_t d = 2 * (lane & 31);
#pragma unroll
        for (int i = 0; i < (NC + 1) / 2; ++i) {
            const int c = 2 * i + half < NC ? 2 * i + half : NC - 1;
            __builtin_amdgcn_global_load_lds((const void *)(U + base0 + qp * st + c * cs + d),
                                             (__attribute__((address_space(3))) void *)&ab[slot][2 * i][0], 16,
                                             0, 0);
        }
    };
    auto read_ahead = [&](int slot, Pt<ND> &w, bool after) {
        // wait until the slot's global-to-LDS load has landed.  The vector
        // memory counter drains in issue order, and after that load the
        // previous step issued its NC residual loads (unless first) and its NC
        // residual stores (every lane of an ahead-loading wave is active, and
        // anything else the compiler adds only raises the count), so the wait
        // leaves those stores in flight instead of waiting for them
        if (!after) __builtin_amdgcn_s_waitcnt(0x0F70);           // vmcnt(0)
        else if (first) __builtin_amdgcn_s_waitcnt(0x0F70 | NC);  // vmcnt(NC)
        else __builtin_amdgcn_s_waitcnt(0x0F70 | (2 * NC));       // vmcnt(2 NC)
        __builtin_amdgcn_sched_barrier(0);  // and no LDS read is scheduled above that wait
#pragma unroll
        for (int c = 0; c < NC; ++c) w.U[c] = ab[slot][c][lane];
        finish_point<ND>(ph, w, bad);
    };

    int64_t cbase = p0 - 3 - kChunk;  // first point held in the chunk buffer
    // point q's conserved state into w (from LDS along x, directly otherwise)
    auto fetch = [&](int64_t qp, Pt<ND> &w) {
        if (DIR == 0) {
            if (qp >= cbase + kChunk) {
                cbase = qp;
                const int64_t last = N + kGhost - 1;
#pragma unroll
                for (int s2 = 0; s2 < kChunk; ++s2) {
                    const int e = lane + 64 * s2;
                    const int r = e / kChunk, x = e % kChunk;
                    int64_t rl = line0 + r;
                    if (rl >= lines) rl = lines - 1;
                    const int64_t rb = ext_index(g, 0, rl % n1, rl / n1);
                    int64_t xp = qp + x;
                    if (xp > last) xp = last;
#pragma unroll
                    for (int c = 0; c < NC; ++c) sb[c][x][r] = U[rb + xp + c * cs];
                }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            }
            const int xi = (int)(qp - cbase);
#pragma unroll
            for (int c = 0; c < NC; ++c) w.U[c] = sb[c][xi][lane];
        } else {
#pragma unroll
            for (int c = 0; c < NC; ++c) w.U[c] = U[base + qp * st + c * cs];
        }
        finish_point<ND>(ph, w, bad);
    };

    Pt<ND> w[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) fetch(p0 - 3 + k, w[k]);
    if (ahead && p0 < p1) load_ahead(p0 + 3, (int)((p0 + 3) & 1));

    // general meshes: node area vectors S_DIR at f-1 .. f+2 for interface f+1/2
    double Sw[4][3];
    if (GEN) {
#pragma unroll
        for (int k = 0; k < 4; ++k)
#pragma unroll
            for (int c = 0; c < ND; ++c)
                Sw[k][c] = m.S[(DIR * ND + c) * cs + base + (p0 - 2 + k) * st];
    }

    // routing masks of interfaces f-1, f, f+1 (index p + 1 along DIR of the
    // direction's interface grid, extent N + 1); outside the line: smooth
    int64_t mbase = 0, mst = 1;
    if (ROUTE) {
        int64_t E[3] = {g.n[0], g.n[1], g.n[2]};
        E[DIR] += 1;
        const int64_t ms[3] = {1, E[0], E[0] * E[1]};
        mbase = q[O1] * ms[O1] + q[O2] * ms[O2];
        mst = ms[DIR];
    }
    auto mload = [&](int64_t pp) -> bool {
        if (pp < -1 || pp > N - 1) return true;
        return mask[mbase + (pp + 1) * mst] != 0;
    };
    // masks of interfaces f-2 .. f+2 (f = the interface being evaluated)
    bool mw[5] = {true, true, true, true, true};
    if (ROUTE) {
#pragma unroll
        for (int k = 0; k < 5; ++k) mw[k] = mload(p0 - 3 + k);
    }

    double Fp[NC];
    for (int64_t f = p0 - 1; f < p1; ++f) {
        if (ROUTE && f >= p0) {
#pragma unroll
            for (int k = 0; k < 4; ++k) mw[k] = mw[k + 1];
            mw[4] = mload(f + 2);
        }
        double rold[NC];
        if (f >= p0) {
#pragma unroll
            for (int k = 0; k < 5; ++k) w[k] = w[k + 1];
            if (ahead) {
                read_ahead((int)((f + 3) & 1), w[5], f > p0);
                if (f + 1 < p1) load_ahead(f + 4, (int)((f + 4) & 1));
                __builtin_amdgcn_sched_barrier(0);  // the residual loads stay behind the load
            } else {
                fetch(f + 3, w[5]);
            }
            // this node's residual so far, requested now and used after the
            // flux: its memory latency hides behind the flux arithmetic
            if (!first) {
#pragma unroll
                for (int c = 0; c < NC; ++c) rold[c] = R[c * g.nint + ibase + f * ist];
            }
            if (GEN) {
#pragma unroll
                for (int k = 0; k < 3; ++k)
#pragma unroll
                    for (int c = 0; c < ND; ++c) Sw[k][c] = Sw[k + 1][c];
#pragma unroll
                for (int c = 0; c < ND; ++c) Sw[3][c] = m.S[(DIR * ND + c) * cs + base + (f + 2) * st];
            }
        }
        // the node's metric factor, requested after the new point (whose wait
        // would otherwise cover it too) and used with the residual
        const int64_t fs = f >= p0 ? f : p0;
        const double sc = GEN ? m.J[base + fs * st] : ih[fs];
        Loc<ND> P[6];
        double F[NC];
        double Smag = 1.0;
        double nv[3] = {0.0, 0.0, 0.0}, t1[3] = {0.0, 0.0, 0.0}, t2[3] = {0.0, 0.0, 0.0};
        if (!GEN) {
#pragma unroll
            for (int k = 0; k < 6; ++k) {
                P[k].r = w[k].U[0];
                P[k].mn = w[k].U[1 + DIR];
                if (NT >= 1) P[k].mt[0] = w[k].U[1 + Axes<ND, DIR>::T1];
                if (NT >= 2) P[k].mt[1] = w[k].U[1 + Axes<ND, DIR>::T2];
                P[k].E = w[k].U[ND + 1];
                P[k].p = w[k].p;
                P[k].a = w[k].a;
                P[k].ri = w[k].ri;
            }
        } else {
            double Sh[3] = {0.0, 0.0, 0.0};
            double s2 = 0.0;
#pragma unroll
            for (int c = 0; c < ND; ++c) {
                Sh[c] = (-Sw[0][c] + 7.0 * Sw[1][c] + 7.0 * Sw[2][c] - Sw[3][c]) / 12.0;
                s2 += Sh[c] * Sh[c];
            }
            Smag = sqrt(s2);
#pragma unroll
            for (int c = 0; c < ND; ++c) nv[c] = Sh[c] / Smag;
            // tangent basis: t1 = normalise(e_{DIR+1} - (e_{DIR+1}.n) n), t2 = n x t1
            if (ND >= 2) {
                constexpr int TE = (DIR + 1) % (ND > 1 ? ND : 1);
                const double en = nv[TE];
                double tn = 0.0;
#pragma unroll
                for (int c = 0; c < ND; ++c) {
                    t1[c] = (c == TE ? 1.0 : 0.0) - en * nv[c];
                    tn += t1[c] * t1[c];
                }
                tn = sqrt(tn);
#pragma unroll
                for (int c = 0; c < ND; ++c) t1[c] /= tn;
                if (ND == 3) {
                    t2[0] = nv[1] * t1[2] - nv[2] * t1[1];
                    t2[1] = nv[2] * t1[0] - nv[0] * t1[2];
                    t2[2] = nv[0] * t1[1] - nv[1] * t1[0];
                }
            }
#pragma unroll
            for (int k = 0; k < 6; ++k) {
                double mn = 0.0, m1 = 0.0, m2 = 0.0;
#pragma unroll
                for (int c = 0; c < ND; ++c) {
                    mn += w[k].U[1 + c] * nv[c];
                    m1 += w[k].U[1 + c] * t1[c];
                    m2 += w[k].U[1 + c] * t2[c];
                }
                P[k].r = w[k].U[0];
                P[k].mn = mn;
                P[k].mt[0] = m1;
                P[k].mt[1] = m2;
                P[k].E = w[k].U[ND + 1];
                P[k].p = w[k].p;
                P[k].a = w[k].a;
                P[k].ri = w[k].ri;
            }
        }
        double Fr, Fn, Ft[2], FE;
        // per-interface routing: an interface evaluated by two waves (the
        // first interface of a segment) takes the same flux in both, so the
        // flux differences stay conservative
        const bool cheap = ROUTE && mw[2] && (ph.dilate < 1 || (mw[1] && mw[3])) && (ph.dilate < 2 || (mw[0] && mw[4]));
        if (cheap) {
            if (MIX) cheap_flux_mixed<ND>(P, ph, Fr, Fn, Ft, FE);
            else cheap_flux<ND>(P, ph, Fr, Fn, Ft, FE);
        } else {
            // the routed forms fall back to the full flux in FP64: near a shock
            // the deviations from the reference flux are as large as the jump,
            // and their FP32 rounding is the precision form's main error there
            if (MIX && !ROUTE) char_flux_mixed<ND, SCHEME>(P, ph, Fr, Fn, Ft, FE);
            else char_flux<ND, SCHEME>(P, ph, Fr, Fn, Ft, FE);
        }
        F[0] = Fr * Smag;
        F[NC - 1] = FE * Smag;
        if (!GEN) {
            F[1 + DIR] = Fn;
            if (NT >= 1) F[1 + Axes<ND, DIR>::T1] = Ft[0];
            if (NT >= 2) F[1 + Axes<ND, DIR>::T2] = Ft[1];
        } else {
#pragma unroll
            for (int c = 0; c < ND; ++c) {
                double v = Fn * nv[c];
                if (NT >= 1) v += Ft[0] * t1[c];
                if (NT >= 2) v += Ft[1] * t2[c];
                F[1 + c] = v * Smag;
            }
        }
        if (f >= p0 && active) {
            double v[NC];
#pragma unroll
            for (int c = 0; c < NC; ++c) v[c] = -sc * (F[c] - Fp[c]);
            if (first) {
#pragma unroll
                for (int c = 0; c < NC; ++c) R[c * g.nint + ibase + f * ist] = v[c];
            } else {
#pragma unroll
                for (int c = 0; c < NC; ++c) R[c * g.nint + ibase + f * ist] = rold[c] + v[c];
            }
        }
#pragma unroll
        for (int c = 0; c < NC; ++c) Fp[c] = F[c];
    }
    if (bad) atomicOr(flags, kFlagNonPhys);
}

// One convective sweep along DIR over a whole grid.  first != 0: R =
// contribution, else R +=.  Thread mapping: every wave owns 64 consecutive
// lines and one segment [p0, p1) along DIR (wave-uniform), lane l owns line
// line0 + l.  Along y and z the lanes' loads are contiguous in x; along x
// the lines are strided, so the wave stages chunks of kChunk points of its 64
// rows through LDS with contiguous loads and each lane reads its own row back.
// One wave per SIMD for general meshes and for the mixed-precision routed
// variant (both flux paths plus the FP64 reference in one loop): at two
// waves they spill, which cost more (1.29 vs 0.93 ms at 256^3) than the
// lost occupancy.
template <int ND, int DIR, int SCHEME, bool GEN, bool MIX, bool ROUTE>
__global__ void __launch_bounds__(256, GEN ? 1 : 2)
k_sweep(const double *__restrict__ U, double *__restrict__ R, Grid g, Phys ph, Metrics m, int64_t seg,
        int64_t nseg, int first, unsigned *flags, const uint8_t *__restrict__ mask) {
    __shared__ double sbuf[DIR == 0 ? kWaves : 1][ND + 2][kChunk][64];
    __shared__ double abuf[DIR == 0 || GEN ? 1 : kWaves][2][ND + 3][64];
    constexpr int O1 = DIR == 0 ? 1 : 0;
    constexpr int O2 = DIR == 2 ? 1 : 2;
    const int64_t lines = g.n[O1] * g.n[O2];
    const int64_t wpl = (lines + 63) >> 6;  // waves per segment
    // wave index made explicitly uniform, so that the segment bounds and the
    // loop over it live in scalar registers
    const int64_t gw = (int64_t)blockIdx.x * (blockDim.x >> 6) + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t sg = gw / wpl;
    if (sg >= nseg) return;  // wave-uniform
    const int64_t line0 = (gw - sg * wpl) << 6;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if constexpr (DIR != 0 && !GEN) {
        const int64_t n1 = g.n[O1];
        if ((line0 % n1) + 64 <= n1 && line0 + 64 <= lines)  // wave-uniform: 64 consecutive x nodes
            sweep_wave<ND, DIR, SCHEME, GEN, MIX, ROUTE, true>(U, R, g, ph, m, seg, sg, line0, first, flags, mask,
                                                               sbuf[0], abuf[wv]);
        else
            sweep_wave<ND, DIR, SCHEME, GEN, MIX, ROUTE, false>(U, R, g, ph, m, seg, sg, line0, first, flags, mask,
                                                                sbuf[0], abuf[wv]);
    } else {
        sweep_wave<ND, DIR, SCHEME, GEN, MIX, ROUTE, false>(U, R, g, ph, m, seg, sg, line0, first, flags, mask,
                                                            sbuf[DIR == 0 ? wv : 0], abuf[0]);
    }
}

// ---------------------------------------------------------------------------
// x sweep on separable meshes with lanes along x.  The interfaces of all rows
// are numbered J = row * (N + 1) + (q + 1) for the interface q + 1/2,
// q = -1 .. N-1 (the interface-grid order of the routing masks).  A wave owns
// 64 consecutive interfaces J0 .. J0 + 63, J0 = 63 w: consecutive waves share
// one interface, so every node whose two interfaces lie in the same row is
// written by exactly one wave, and the rows' points are read with contiguous
// loads.  Lane l loads the point q_l + 3 of its row (the right end of its
// stencil); the five points left of lane 0's stencil end, and the first five
// points of a row that starts inside the wave, go to extra slots.  Needs
// N + 1 >= 64 (at most one row start per wave).
constexpr int kXlSlots = 64 + 10;

template <int ND>
struct XlLds {
    double pt[ND + 5][kXlSlots];  // U[0..nc), ri, p, a of the staged points
    double fl[ND + 2][64];        // interface fluxes of the wave
};

template <int ND, int SCHEME, bool MIX, bool ROUTE>
__device__ __forceinline__ void sweep_x_lanes(const double *__restrict__ U, double *__restrict__ R, const Grid &g,
                                              const Phys &ph, const Metrics &m, int64_t J0, int64_t totalJ,
                                              int first, unsigned *flags, const uint8_t *__restrict__ mask,
                                              XlLds<ND> &sm) {
    constexpr int NC = ND + 2;
    constexpr int NT = ND - 1;
    const int lane = threadIdx.x & 63;
    const int64_t N = g.n[0], NI = N + 1, n1 = g.n[1];
    const int64_t cs = g.enpts;
    const int64_t J = J0 + lane;
    const bool valid = J < totalJ;
    const int64_t Jc = valid ? J : totalJ - 1;
    // wave-uniform: lane 0's row and interface, and the first lane of the next row
    // (scalar divisions, in 32 bits whenever the interface count allows)
    const bool narrow = totalJ < 0x7fffffff;
    auto sdiv = [narrow](int64_t a, int64_t b) -> int64_t {
        return narrow ? (int64_t)((uint32_t)a / (uint32_t)b) : a / b;
    };
    const int64_t row0 = sdiv(J0, NI), q0 = J0 - row0 * NI - 1;
    const int Lnext = (int)(NI - (q0 + 1));  // lane index where row0 + 1 starts (>= 64: none)
    // The lane's row and interface without a per-lane division: a wave spans
    // at most two rows (NI >= 64), row0 and row0 + 1, whose (y, z) are
    // scalars; lanes past the last interface take the last one.
    const int64_t z0 = sdiv(row0, n1), y0 = row0 - z0 * n1;
    const int64_t y1 = y0 + 1 < n1 ? y0 + 1 : 0, z1 = y0 + 1 < n1 ? z0 : z0 + 1;
    const int64_t rows = n1 * g.n[2];  // totalJ = rows * NI
    const bool nxt = lane >= Lnext;
    int64_t yl = nxt ? y1 : y0, zl = nxt ? z1 : z0;
    int64_t q = nxt ? (int64_t)(lane - Lnext) - 1 : q0 + lane;
    if (!valid) {
        yl = n1 - 1;
        zl = g.n[2] - 1;
        q = N - 1;
    }
    const int64_t rowb = ext_index(g, 0, yl, zl);
    bool bad = false;

    auto put = [&](int slot, Pt<ND> &w) {
        finish_point<ND>(ph, w, bad);
#pragma unroll
        for (int c = 0; c < NC; ++c) sm.pt[c][slot] = w.U[c];
        sm.pt[NC][slot] = w.ri;
        sm.pt[NC + 1][slot] = w.p;
        sm.pt[NC + 2][slot] = w.a;
    };
    // Every lane stages the point q + 3 of its row.  Lanes 0..4 also stage
    // the points q0 - 2 .. q0 + 2 of lane 0's row, lanes 5..9 the points
    // -3 .. 1 of a row starting inside the wave (the other lanes' second
    // point is their own; the compiler keeps only the extra lanes' loads,
    // inside their branch, so the two batches arrive one after the other).
    int64_t xb = rowb, xp = q + 3;
    bool extra = false;
    if (lane < 5) {
        xb = ext_index(g, 0, y0, z0);
        xp = q0 - 2 + lane;
        extra = true;
    } else if (lane < 10 && Lnext < 64) {
        const bool has1 = row0 + 1 < rows;
        xb = ext_index(g, 0, has1 ? y1 : y0, has1 ? z1 : z0);
        xp = (int64_t)(lane - 5) - 3;
        extra = true;
    }
    Pt<ND> w0, w1;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        w0.U[c] = U[rowb + q + 3 + c * cs];
        w1.U[c] = U[xb + xp + c * cs];
    }
    put(lane, w0);
    if (extra) put(64 + lane, w1);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

    // stencil q - 2 .. q + 3 of this lane
    const bool inrow0 = lane < Lnext;
    Loc<ND> P[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        const int src = lane - 5 + k;
        int slot;
        if (inrow0) slot = src >= 0 ? src : 64 + lane + k;
        else slot = src >= Lnext ? src : 69 + (lane - Lnext) + k;
        P[k].r = sm.pt[0][slot];
        P[k].mn = sm.pt[1][slot];
        if (NT >= 1) P[k].mt[0] = sm.pt[1 + Axes<ND, 0>::T1][slot];
        if (NT >= 2) P[k].mt[1] = sm.pt[1 + Axes<ND, 0>::T2][slot];
        P[k].E = sm.pt[ND + 1][slot];
        P[k].ri = sm.pt[NC][slot];
        P[k].p = sm.pt[NC + 1][slot];
        P[k].a = sm.pt[NC + 2][slot];
    }
    bool cheap = false;
    if (ROUTE) {
        // interfaces outside the line count as smooth
        auto ml = [&](int o) { return (q + o < -1 || q + o > N - 1) ? true : mask[Jc + o] != 0; };
        cheap = ml(0) && (ph.dilate < 1 || (ml(-1) && ml(1))) && (ph.dilate < 2 || (ml(-2) && ml(2)));
    }
    double Fr, Fn, Ft[2], FE;
    if (cheap) {
        if (MIX) cheap_flux_mixed<ND>(P, ph, Fr, Fn, Ft, FE);
        else cheap_flux<ND>(P, ph, Fr, Fn, Ft, FE);
    } else {
        // routed forms: full flux in FP64 (as in the marching sweeps)
        if (MIX && !ROUTE) char_flux_mixed<ND, SCHEME>(P, ph, Fr, Fn, Ft, FE);
        else char_flux<ND, SCHEME, false>(P, ph, Fr, Fn, Ft, FE);
    }
    double F[NC];
    F[0] = Fr;
    F[1] = Fn;
    if (NT >= 1) F[1 + Axes<ND, 0>::T1] = Ft[0];
    if (NT >= 2) F[1 + Axes<ND, 0>::T2] = Ft[1];
    F[NC - 1] = FE;
#pragma unroll
    for (int c = 0; c < NC; ++c) sm.fl[c][lane] = F[c];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // node q: its left interface belongs to lane - 1 of the same row
    if (valid && lane >= 1 && q >= 0 && lane != Lnext) {
        const double sc = m.invh[0][q];
        const int64_t oi = yl * g.is[1] + zl * g.is[2] + q;
        double v[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) v[c] = -sc * (F[c] - sm.fl[c][lane - 1]);
        add_residual<NC>(R, g.nint, oi, v, first);
    }
    if (bad) atomicOr(flags, kFlagNonPhys);
}

// three waves per SIMD (168 registers); TENO6's four stencils spill there,
// so it runs at two (180 registers, x sweep 0.87 -> 0.86 ms at 256^3)
template <int ND, int SCHEME, bool MIX, bool ROUTE>
__global__ void __launch_bounds__(64 * kWaves, SCHEME == OSBLI_TENO6 ? 2 : 3)
k_sweep_xl(const double *__restrict__ U, double *__restrict__ R, Grid g, Phys ph, Metrics m, int64_t totalJ,
           int first, unsigned *flags, const uint8_t *__restrict__ mask) {
    __shared__ XlLds<ND> sm[kWaves];
    const int64_t gw = (int64_t)blockIdx.x * (blockDim.x >> 6) + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t J0 = gw * 63;
    if (J0 + 1 >= totalJ) return;  // wave-uniform: no node left
    sweep_x_lanes<ND, SCHEME, MIX, ROUTE>(U, R, g, ph, m, J0, totalJ, first, flags, mask, sm[threadIdx.x >> 6]);
}

}  // namespace cf
}  // namespace osbli
