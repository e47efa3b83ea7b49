// Viscous and heat-flux terms (eqs. heat_flux, stress_tensor, sutherland of
// section 2.1) in divergence form with the fourth-order central scheme and
// the one-sided boundary closures of section 2.6; the fused low-storage RK
// update (section 2.7); the CFL time-step reduction.
//
// Pass 1 (k_visc_flux): per node, gradients of (u, T) from the central
// operator (closures at non-periodic ends; periodic ends read the ghost
// copies), stress tensor, heat flux and the contravariant viscous fluxes
// G_k = S_k . Fv, stored once per node (separable meshes: each distinct
// stress once, see gslot).
// Pass 2 (k_finish): per node, J sum_k D_k G_k added to the convective
// residual, then either stored (residual call) or folded into the RK update.
#include "point.hpp"
#include "stencil.hpp"

namespace osbli {
namespace {

// Tile placement: workgroups go to the eight XCDs (each with its own L2) in
// turn, so a 1D grid of 8 * per blocks is used and the linear block id b is
// remapped to the tile (b % 8) * per + b / 8: each XCD then owns one
// contiguous run of tiles (x fastest, then y, then z), and the stencil
// neighbours that adjacent tiles share are read through one L2.
constexpr int kXcds = 8;

struct NodeTiles {
    int tx, ty, nt, per;  // tiles along x, along y, in all; tiles per XCD
};

inline NodeTiles node_tiles(const Grid &g) {
    NodeTiles T;
    T.tx = (int)((g.n[0] + kBX - 1) / kBX);
    T.ty = (int)((g.n[1] + kBY - 1) / kBY);
    T.nt = T.tx * T.ty * (int)g.n[2];
    T.per = (T.nt + kXcds - 1) / kXcds;
    return T;
}

inline dim3 node_launch(const NodeTiles &T) { return dim3((unsigned)(T.per * kXcds)); }

__device__ __forceinline__ bool node_of_thread(const Grid &g, const NodeTiles &T, int64_t (&idx)[3]) {
    const int L = (int)(blockIdx.x % kXcds) * T.per + (int)(blockIdx.x / kXcds);
    if (L >= T.nt) return false;
    const int bx = L % T.tx, by = (L / T.tx) % T.ty;
    idx[0] = (int64_t)bx * kBX + threadIdx.x;
    idx[1] = (int64_t)by * kBY + threadIdx.y;
    idx[2] = L / (T.tx * T.ty);
    return idx[0] < g.n[0] && idx[1] < g.n[1];
}

template <int ND>
__device__ __forceinline__ void phi_at(const double *__restrict__ U, int64_t e, int64_t cs, const Phys &ph,
                                       double (&phi)[ND + 1]) {
    const double r = U[e];
    const double ri = 1.0 / r;
    double ke = 0.0;
#pragma unroll
    for (int m = 0; m < ND; ++m) {
        const double mm = U[e + (1 + m) * cs];
        phi[m] = mm * ri;
        ke += mm * mm;
    }
    const double p = ph.gm1 * (U[e + (ND + 1) * cs] - 0.5 * ke * ri);
    phi[ND] = ph.gamma * ph.M2 * p * ri;
}


// D_kk (per unit index) of the node primitives at e0 (position p along kk),
// from global loads: the interior operator on ghost copies for periodic
// directions, the one-sided closures near non-periodic ends
template <int ND>
__device__ __forceinline__ void dk_global(const double *__restrict__ U, int64_t e0, int64_t cs, const Phys &ph,
                                          const Grid &g, int kk, int64_t p, double (&D)[ND + 1]) {
    constexpr int NV = ND + 1;
    const int64_t N = g.n[kk], st = g.es[kk];
    const int64_t eline = e0 - p * st;
    const bool per = g.periodic[kk] != 0;
    // evaluate the five-point operator component-wise from one set of loads
    if (per || (p >= 2 && p <= N - 3)) {
        double fm2[NV], fm1[NV], fp1[NV], fp2[NV];
        phi_at<ND>(U, e0 - 2 * st, cs, ph, fm2);
        phi_at<ND>(U, e0 - st, cs, ph, fm1);
        phi_at<ND>(U, e0 + st, cs, ph, fp1);
        phi_at<ND>(U, e0 + 2 * st, cs, ph, fp2);
#pragma unroll
        for (int v = 0; v < NV; ++v) D[v] = (2.0 / 3.0) * (fp1[v] - fm1[v]) - (1.0 / 12.0) * (fp2[v] - fm2[v]);
    } else {
        // the five nodes at one end; p sits at window position 0, 1, 3 or 4
        double f[5][NV];
        const int64_t q0 = p < 2 ? 0 : N - 5;
        const int r = (int)(p - q0);
#pragma unroll
        for (int k = 0; k < 5; ++k) phi_at<ND>(U, eline + (q0 + k) * st, cs, ph, f[k]);
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const double f0 = f[0][v], f1 = f[1][v], f2 = f[2][v], f3 = f[3][v], f4 = f[4][v];
            if (r == 0) D[v] = (-25.0 * f0 + 48.0 * f1 - 36.0 * f2 + 16.0 * f3 - 3.0 * f4) / 12.0;
            else if (r == 1) D[v] = (-3.0 * f0 - 10.0 * f1 + 18.0 * f2 - 6.0 * f3 + f4) / 12.0;
            else if (r == 3) D[v] = (-f0 + 6.0 * f1 - 18.0 * f2 + 10.0 * f3 + 3.0 * f4) / 12.0;
            else D[v] = (3.0 * f0 - 16.0 * f1 + 36.0 * f2 - 48.0 * f3 + 25.0 * f4) / 12.0;
        }
    }
}

// gradients from D_k, stress tensor, heat flux and the stored contravariant
// viscous fluxes G_k = S_k . Fv of one node
template <int ND, bool GEN>
__device__ __forceinline__ void visc_store(const double (&phi0)[ND + 1], const double (&Dk)[ND][ND + 1],
                                           double *__restrict__ G, const Grid &g, const Phys &ph, const Metrics &m,
                                           const int64_t (&idx)[3], int64_t ci, int64_t e0) {
    constexpr int NV = ND + 1;
    const int64_t cs = g.enpts;
    double grad[NV][ND];
    double Jc = 1.0;
    if (GEN) Jc = m.J[e0];
#pragma unroll
    for (int v = 0; v < NV; ++v)
#pragma unroll
        for (int j = 0; j < ND; ++j) {
            if (!GEN) {
                grad[v][j] = m.invh[j][idx[j]] * Dk[j][v];
            } else {
                double s = 0.0;
#pragma unroll
                for (int kk = 0; kk < ND; ++kk) s += m.S[(kk * ND + j) * cs + e0] * Dk[kk][v];
                grad[v][j] = Jc * s;
            }
        }
    const double T = phi0[ND];
    const double mu = viscosity(ph, T);
    double divu = 0.0;
#pragma unroll
    for (int a = 0; a < ND; ++a) divu += grad[a][a];
    const double mre = mu * ph.mu_re;
    double Fv[ND][NV];
#pragma unroll
    for (int b = 0; b < ND; ++b) {
        double work = 0.0;
#pragma unroll
        for (int a = 0; a < ND; ++a) {
            double tab = mre * (grad[a][b] + grad[b][a] - (a == b ? (2.0 / 3.0) * divu : 0.0));
            Fv[b][a] = tab;
            work += phi0[a] * tab;
        }
        const double qb = -mu * ph.kheat * grad[ND][b];
        Fv[b][ND] = work - qb;
    }
#pragma unroll
    for (int kk = 0; kk < ND; ++kk)
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            double s;
            if (!GEN) {
                s = Fv[kk][v];
            } else {
                s = 0.0;
#pragma unroll
                for (int b = 0; b < ND; ++b) s += m.S[(kk * ND + b) * cs + e0] * Fv[b][v];
            }
            // each distinct stress once (separable meshes)
            if (GEN || v == ND || kk <= v) G[gslot<ND, GEN>(kk, v) * g.nint + ci] = s;
        }
}

template <int ND, bool GEN>
__global__ void __launch_bounds__(256)
k_visc_flux(const double *__restrict__ U, double *__restrict__ G, Grid g, Phys ph, Metrics m, NodeTiles T) {
    constexpr int NV = ND + 1;
    int64_t idx[3];
    if (!node_of_thread(g, T, idx)) return;
    const int64_t ci = int_index(g, idx[0], idx[1], idx[2]);
    const int64_t e0 = ext_index(g, idx[0], idx[1], idx[2]);
    const int64_t cs = g.enpts;
    double phi0[NV];
    phi_at<ND>(U, e0, cs, ph, phi0);
    double Dk[ND][NV];
#pragma unroll
    for (int kk = 0; kk < ND; ++kk) dk_global<ND>(U, e0, cs, ph, g, kk, idx[kk], Dk[kk]);
    visc_store<ND, GEN>(phi0, Dk, G, g, ph, m, idx, ci, e0);
}

// 3D separable meshes: a block owns a kZX x kZY tile of (x, y) columns and
// marches kZC planes along z.  The primitives of the current plane (tile plus
// a two-node halo, read from U including ghost copies) sit in LDS for the x
// and y derivatives; each column keeps its own z-2 .. z+2 primitives in
// registers.  Nodes within two of a non-periodic end take that direction's
// closure from global loads.  The arithmetic per node is that of k_visc_flux.
constexpr int kZX = 64, kZY = 8, kZC = 32;
constexpr int kHX = kZX + 4, kHY = kZY + 4;

// the tile's halo: two rows above and below the tile (kHX wide) and two
// columns either side of its kZY rows; one position per thread
constexpr int kHalo = 4 * kHX + 4 * kZY;
static_assert(kHalo <= kZX * kZY, "one halo position per thread");

__device__ __forceinline__ void halo_pos(int h, int &cx, int &cy) {
    if (h < 4 * kHX) {
        const int r = h / kHX;
        cx = h - r * kHX;
        cy = r < 2 ? r : kZY + r;
    } else {
        const int r = h - 4 * kHX, s = r & 3;
        cy = 2 + (r >> 2);
        cx = s < 2 ? s : kZX + s;
    }
}

// primitives from the conserved values of one node (the arithmetic of phi_at)
__device__ __forceinline__ void phi_of(const double (&u)[5], const Phys &ph, double (&phi)[4]) {
    const double ri = 1.0 / u[0];
    double ke = 0.0;
#pragma unroll
    for (int m = 0; m < 3; ++m) {
        phi[m] = u[1 + m] * ri;
        ke += u[1 + m] * u[1 + m];
    }
    const double p = ph.gm1 * (u[4] - 0.5 * ke * ri);
    phi[3] = ph.gamma * ph.M2 * p * ri;
}

// Tiles are placed on the XCDs as the node tiles are (one contiguous run of
// tiles per XCD).  The loads are issued ahead of their use: a column's
// conserved values at z+3 one step ahead, the halo of plane z+2 two steps
// ahead, together with the columns' own z+2 loads of the neighbouring tiles,
// which read the same nodes at that time, so the halo comes from the L2 (a
// halo read at its own plane was served from HBM: the XCD had streamed two
// planes of every resident tile through the L2 since).  One block per CU
// (at most 256 registers per lane): at four waves per SIMD the loads held in
// flight spilled.
__global__ void __launch_bounds__(kZX * kZY, 2)
k_visc_flux_zm(const double *__restrict__ U, double *__restrict__ G, Grid g, Phys ph, Metrics m, int tx_n,
               int ty_n, int ntiles, int per) {
    constexpr int NV = 4;
    __shared__ double tile[2][NV][kHY][kHX];
    const int L = (int)(blockIdx.x % kXcds) * per + (int)(blockIdx.x / kXcds);
    if (L >= ntiles) return;  // block-uniform
    const int bx = L % tx_n, by = (L / tx_n) % ty_n, bz = L / (tx_n * ty_n);
    const int tx = threadIdx.x, ty = threadIdx.y, tid = ty * kZX + tx;
    const int64_t x0 = (int64_t)bx * kZX, y0 = (int64_t)by * kZY;
    const int64_t x = x0 + tx, y = y0 + ty;
    const int64_t Nx = g.n[0], Ny = g.n[1], Nz = g.n[2];
    const int64_t z0 = (int64_t)bz * kZC;
    const int64_t z1 = z0 + kZC < Nz ? z0 + kZC : Nz;
    const bool own = x < Nx && y < Ny;
    const int64_t cs = g.enpts, sz = g.es[2];
    const bool perx = g.periodic[0] != 0, pery = g.periodic[1] != 0, perz = g.periodic[2] != 0;
    const bool intx = perx || (x >= 2 && x <= Nx - 3);
    const bool inty = pery || (y >= 2 && y <= Ny - 3);
    // a column beyond the grid holds the ghost (or, further out, the last
    // ghost) node of its position: such values reach only unused stencil slots
    const int64_t ecol = ext_index(g, x < Nx + 2 ? x : Nx + 2, y < Ny + 2 ? y : Ny + 2, 0);
    const bool hal = tid < kHalo;
    int hx = 0, hy = 0;
    halo_pos(hal ? tid : 0, hx, hy);
    int64_t hgx = x0 - 2 + hx, hgy = y0 - 2 + hy;
    hgx = hgx > Nx + 2 ? Nx + 2 : hgx;
    hgy = hgy > Ny + 2 ? Ny + 2 : hgy;
    const int64_t hcol = ext_index(g, hgx, hgy, 0);

    double w[5][NV];  // primitives of this column at z-2 .. z+2
#pragma unroll
    for (int k = 1; k < 5; ++k) phi_at<3>(U, ecol + (z0 - 3 + k) * sz, cs, ph, w[k]);
    double ou[5];     // conserved values of this column at z+2
    double hu[2][5];  // conserved values at the halo position, planes z and z+1
#pragma unroll
    for (int c = 0; c < 5; ++c) {
        ou[c] = U[ecol + (z0 + 2) * sz + c * cs];
#pragma unroll
        for (int k = 0; k < 2; ++k) hu[k][c] = hal ? U[hcol + (z0 + k) * sz + c * cs] : 1.0;
    }

#pragma unroll 1
    for (int64_t z = z0; z < z1; ++z) {
#pragma unroll
        for (int k = 0; k < 4; ++k)
#pragma unroll
            for (int v = 0; v < NV; ++v) w[k][v] = w[k + 1][v];
        phi_of(ou, ph, w[4]);
        double hn[5];
#pragma unroll
        for (int c = 0; c < 5; ++c) {
            ou[c] = U[ecol + (z + 3) * sz + c * cs];  // z + 3 <= Nz + 2: the last ghost plane
            hn[c] = hal ? U[hcol + (z + 2) * sz + c * cs] : 1.0;
        }
        const int b = (int)((z - z0) & 1);
        if (hal) {
            double f[NV];
            phi_of(hu[0], ph, f);
#pragma unroll
            for (int v = 0; v < NV; ++v) tile[b][v][hy][hx] = f[v];
        }
#pragma unroll
        for (int v = 0; v < NV; ++v) tile[b][v][ty + 2][tx + 2] = w[2][v];
#pragma unroll
        for (int c = 0; c < 5; ++c) {
            hu[0][c] = hu[1][c];
            hu[1][c] = hn[c];
        }
        __syncthreads();
        if (own) {
            const int64_t idx[3] = {x, y, z};
            const int64_t e0 = ecol + z * sz;
            double Dk[3][NV];
            const int cx = tx + 2, cy = ty + 2;
            if (intx) {
#pragma unroll
                for (int v = 0; v < NV; ++v)
                    Dk[0][v] = (2.0 / 3.0) * (tile[b][v][cy][cx + 1] - tile[b][v][cy][cx - 1]) -
                               (1.0 / 12.0) * (tile[b][v][cy][cx + 2] - tile[b][v][cy][cx - 2]);
            } else {
                dk_global<3>(U, e0, cs, ph, g, 0, x, Dk[0]);
            }
            if (inty) {
#pragma unroll
                for (int v = 0; v < NV; ++v)
                    Dk[1][v] = (2.0 / 3.0) * (tile[b][v][cy + 1][cx] - tile[b][v][cy - 1][cx]) -
                               (1.0 / 12.0) * (tile[b][v][cy + 2][cx] - tile[b][v][cy - 2][cx]);
            } else {
                dk_global<3>(U, e0, cs, ph, g, 1, y, Dk[1]);
            }
            if (perz || (z >= 2 && z <= Nz - 3)) {
#pragma unroll
                for (int v = 0; v < NV; ++v)
                    Dk[2][v] = (2.0 / 3.0) * (w[3][v] - w[1][v]) - (1.0 / 12.0) * (w[4][v] - w[0][v]);
            } else {
                dk_global<3>(U, e0, cs, ph, g, 2, z, Dk[2]);
            }
            visc_store<3, false>(w[2], Dk, G, g, ph, m, idx, int_index(g, x, y, z), e0);
        }
    }
}

// R = Racc (+ viscous divergence); mode 0 stores R, mode 1 applies the RK stage.
template <int ND, bool GEN, bool VISC, int MODE>
__global__ void __launch_bounds__(256)
k_finish(const double *Racc, const double *__restrict__ G, double *Rout, Grid g,
         Phys ph, Metrics m, RkStage rs, double dt, double *__restrict__ U, double *__restrict__ dU) {
    constexpr int NC = ND + 2;
    constexpr int NV = ND + 1;
    int64_t idx[3];
    if (!node_of_plane_thread(g, idx)) return;
    const int64_t ci = int_index(g, idx[0], idx[1], idx[2]);
    double R[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) R[c] = Racc[c * g.nint + ci];
    const int64_t e0 = ext_index(g, idx[0], idx[1], idx[2]);
    if (VISC) {
        double acc[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) acc[v] = 0.0;
#pragma unroll
        for (int kk = 0; kk < ND; ++kk) {
            const int64_t N = g.n[kk], p = idx[kk], st = g.is[kk];
            const int64_t line = ci - p * st;
            const bool per = g.periodic[kk] != 0;
            const double sc = GEN ? 1.0 : m.invh[kk][p];
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                const double *Gv = G + gslot<ND, GEN>(kk, v) * g.nint + line;
                auto at = [&](int64_t q) {
                    int64_t w = q;
                    if (per) w = q < 0 ? q + N : (q >= N ? q - N : q);
                    return Gv[w * st];
                };
                acc[v] += sc * dline(at, p, N, per);
            }
        }
        const double Jc = GEN ? m.J[e0] : 1.0;
#pragma unroll
        for (int v = 0; v < NV; ++v) R[1 + v] += Jc * acc[v];
    }
    if (MODE == 0) {
#pragma unroll
        for (int c = 0; c < NC; ++c) Rout[c * g.nint + ci] = R[c];
    } else {
#pragma unroll
        for (int c = 0; c < NC; ++c) rk_point(rs, dt, R[c], dU + c * g.nint + ci, U + c * g.enpts + e0);
    }
}

// The same finish for 3D separable meshes, RK update only, marching along z:
// a block owns a kBX x kBY tile of columns and kFZ planes; each thread keeps
// its column's G_z at z-2 .. z+2 in registers, so G_z is read once per node
// instead of once per stencil use (the z neighbours' fluxes are otherwise
// re-read from HBM: the plane-by-plane working set overflows the L2).  The
// x and the y neighbours' fluxes are requested a direction at a time, then
// the node's residual, register and state together.  Nodes
// within two of a non-periodic end take that direction's closure from direct
// loads; the arithmetic per node is that of k_finish.
constexpr int kFZ = 16;
constexpr int kFX = 64, kFY = 4;  // columns per block

__global__ void __launch_bounds__(kFX * kFY)
k_finish_zm(const double *__restrict__ Racc, const double *__restrict__ G, Grid g, Metrics m, RkStage rs, double dt,
            double *__restrict__ U, double *__restrict__ dU, int ntx, int nty, int stripe) {
    constexpr int NC = 5, NV = 4;
    // XCD k (blocks b with b % 8 == k) owns the stripe of y tiles
    // [k stripe, (k + 1) stripe); within it x tiles run fastest, then y, then
    // z runs, so every XCD advances through the planes at the same pace and
    // the y neighbours' fluxes are read through the one L2
    const int xcd = (int)(blockIdx.x % kXcds), l = (int)(blockIdx.x / kXcds);
    const int bxt = l % ntx, byt = xcd * stripe + (l / ntx) % stripe, bzt = l / (ntx * stripe);
    if (byt >= nty) return;
    const int64_t x = (int64_t)bxt * kFX + threadIdx.x;
    const int64_t y = (int64_t)byt * kFY + threadIdx.y;
    const int64_t Nx = g.n[0], Ny = g.n[1], Nz = g.n[2];
    if (x >= Nx || y >= Ny) return;  // no block-wide synchronisation below
    const int64_t z0 = (int64_t)bzt * kFZ;
    const int64_t z1 = z0 + kFZ < Nz ? z0 + kFZ : Nz;
    const bool perx = g.periodic[0] != 0, pery = g.periodic[1] != 0, perz = g.periodic[2] != 0;
    const bool intx = perx || (x >= 2 && x <= Nx - 3);
    const bool inty = pery || (y >= 2 && y <= Ny - 3);
    const int64_t sy = g.is[1], sz = g.is[2];
    const int64_t col = x + y * sy;  // interior index of (x, y, 0)
    const double scx = m.invh[0][x], scy = m.invh[1][y];
    auto wrap = [](int64_t q, int64_t N, bool per) -> int64_t {
        if (per) return q < 0 ? q + N : (q >= N ? q - N : q);
        return q < 0 ? 0 : (q >= N ? N - 1 : q);  // clamped: such values are never used
    };
    // neighbour offsets in x and y (p-2, p-1, p+1, p+2), wrapped where periodic
    int64_t ox[4], oy[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int d = k < 2 ? k - 2 : k - 1;
        ox[k] = wrap(x + d, Nx, perx) - x;
        oy[k] = (wrap(y + d, Ny, pery) - y) * sy;
    }
    // component v of G_x, G_y, G_z
    auto Gx = [&](int v) { return G + gslot<3, false>(0, v) * g.nint; };
    auto Gy = [&](int v) { return G + gslot<3, false>(1, v) * g.nint; };
    auto Gz = [&](int v) { return G + gslot<3, false>(2, v) * g.nint; };
    double gz[5][NV];  // G_z of this column at z-2 .. z+2
#pragma unroll
    for (int k = 1; k < 5; ++k) {
        const int64_t zp = wrap(z0 - 3 + k, Nz, perz);
#pragma unroll
        for (int v = 0; v < NV; ++v) gz[k][v] = Gz(v)[col + zp * sz];
    }
#pragma unroll 1
    for (int64_t z = z0; z < z1; ++z) {
#pragma unroll
        for (int k = 0; k < 4; ++k)
#pragma unroll
            for (int v = 0; v < NV; ++v) gz[k][v] = gz[k + 1][v];
        const int64_t ci = col + z * sz;
        const int64_t e0 = ext_index(g, x, y, z);
        const int64_t zn = wrap(z + 2, Nz, perz);
        // the fluxes this node needs: G_z from the window, then the x and the
        // y neighbours, four loads per flux component requested together
#pragma unroll
        for (int v = 0; v < NV; ++v) gz[4][v] = Gz(v)[col + zn * sz];
        double acc[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) acc[v] = 0.0;
        // x, y, z in the order of k_finish
        if (intx) {
            double a[NV][4];
#pragma unroll
            for (int v = 0; v < NV; ++v)
#pragma unroll
                for (int k = 0; k < 4; ++k) a[v][k] = Gx(v)[ci + ox[k]];
#pragma unroll
            for (int v = 0; v < NV; ++v)
                acc[v] += scx * ((2.0 / 3.0) * (a[v][2] - a[v][1]) - (1.0 / 12.0) * (a[v][3] - a[v][0]));
        } else {
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                const double *Gv = Gx(v) + (ci - x);
                auto at = [&](int64_t q) { return Gv[q]; };
                acc[v] += scx * dline(at, x, Nx, false);
            }
        }
        if (inty) {
            double a[NV][4];
#pragma unroll
            for (int v = 0; v < NV; ++v)
#pragma unroll
                for (int k = 0; k < 4; ++k) a[v][k] = Gy(v)[ci + oy[k]];
#pragma unroll
            for (int v = 0; v < NV; ++v)
                acc[v] += scy * ((2.0 / 3.0) * (a[v][2] - a[v][1]) - (1.0 / 12.0) * (a[v][3] - a[v][0]));
        } else {
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                const double *Gv = Gy(v) + (ci - y * sy);
                auto at = [&](int64_t q) { return Gv[q * sy]; };
                acc[v] += scy * dline(at, y, Ny, false);
            }
        }
        const double scz = m.invh[2][z];
        if (perz || (z >= 2 && z <= Nz - 3)) {
#pragma unroll
            for (int v = 0; v < NV; ++v)
                acc[v] += scz * ((2.0 / 3.0) * (gz[3][v] - gz[1][v]) - (1.0 / 12.0) * (gz[4][v] - gz[0][v]));
        } else {
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                const double *Gv = Gz(v) + col;
                auto at = [&](int64_t q) { return Gv[q * sz]; };
                acc[v] += scz * dline(at, z, Nz, false);
            }
        }
        // then the node's residual, register and state, requested together
        double R[NC], d0[NC], u0[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) R[c] = Racc[c * g.nint + ci];
#pragma unroll
        for (int c = 0; c < NC; ++c) d0[c] = rs.first ? 0.0 : dU[c * g.nint + ci];
#pragma unroll
        for (int c = 0; c < NC; ++c) u0[c] = U[c * g.enpts + e0];
#pragma unroll
        for (int v = 0; v < NV; ++v) R[1 + v] += acc[v];
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const double du = (rs.first ? 0.0 : rs.A * d0[c]) + dt * R[c];
            if (!rs.last) dU[c * g.nint + ci] = du;
            U[c * g.enpts + e0] = u0[c] + rs.B * du;
        }
    }
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}

// dt denominator, max over nodes; positive doubles compare as unsigned 64-bit.
// Blocks stride over z planes so that only a few hundred blocks issue the
// final atomic (a max is order independent, so the result is deterministic).
template <int ND, bool GEN>
__global__ void __launch_bounds__(256)
k_dt(const double *__restrict__ U, Grid g, Phys ph, Metrics m, unsigned long long *slot) {
    __shared__ double part[4];
    double s = 0.0;
    int64_t idx[3];
    idx[0] = (int64_t)blockIdx.x * kBX + threadIdx.x;
    idx[1] = (int64_t)blockIdx.y * kBY + threadIdx.y;
    const bool inplane = idx[0] < g.n[0] && idx[1] < g.n[1];
    for (idx[2] = blockIdx.z; inplane && idx[2] < g.n[2]; idx[2] += gridDim.z) {
        double sn = dt_node<ND, GEN>(U, g, ph, m, idx);
        s = fmax(s, sn);
    }
    s = wave_max(s);
    const int lane = threadIdx.x & 63, wv = threadIdx.y;
    if (lane == 0) part[wv] = s;
    __syncthreads();
    if (threadIdx.x == 0 && threadIdx.y == 0) {
        double b = part[0];
        for (int k = 1; k < (int)blockDim.y; ++k) b = fmax(b, part[k]);
        atomicMax(slot, (unsigned long long)__double_as_longlong(b));
    }
}

__global__ void k_fill_u64(unsigned long long *p, unsigned long long v, int n) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

template <int ND, bool GEN>
hipError_t finish_nd(const Grid &g, const Phys &ph, const Metrics &m, const double *Racc, const double *G,
                     double *Rout, RkStage rs, double dt, double *U, double *dU, int mode, hipStream_t s) {
    // plane-major order on every XCD: the finish reads its z neighbours'
    // fluxes best when all XCDs advance through the planes together (the
    // per-XCD runs of node_tiles measured slower here)
    const dim3 nb = node_grid(g), bs(kBX, kBY);
    if (ND == 3 && !GEN && ph.viscous && mode == 1) {
        const int ntx = (int)((g.n[0] + kFX - 1) / kFX), nty = (int)((g.n[1] + kFY - 1) / kFY);
        const int ntz = (int)((g.n[2] + kFZ - 1) / kFZ), stripe = (nty + kXcds - 1) / kXcds;
        const unsigned nblk = (unsigned)kXcds * (unsigned)(ntx * stripe * ntz);
        hipLaunchKernelGGL(k_finish_zm, dim3(nblk), dim3(kFX, kFY), 0, s, Racc, G, g, m, rs, dt, U, dU, ntx, nty,
                           stripe);
        return hipGetLastError();
    }
    if (ph.viscous) {
        if (mode == 0)
            hipLaunchKernelGGL((k_finish<ND, GEN, true, 0>), nb, bs, 0, s, Racc, G, Rout, g, ph, m,
                               rs, dt, U, dU);
        else
            hipLaunchKernelGGL((k_finish<ND, GEN, true, 1>), nb, bs, 0, s, Racc, G, Rout, g, ph, m,
                               rs, dt, U, dU);
    } else {
        if (mode == 0)
            hipLaunchKernelGGL((k_finish<ND, GEN, false, 0>), nb, bs, 0, s, Racc, G, Rout, g, ph,
                               m, rs, dt, U, dU);
        else
            hipLaunchKernelGGL((k_finish<ND, GEN, false, 1>), nb, bs, 0, s, Racc, G, Rout, g, ph,
                               m, rs, dt, U, dU);
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_viscous_fluxes(const Grid &g, const Phys &ph, const Metrics &m, const double *U, double *G,
                                 hipStream_t s) {
    const NodeTiles T = node_tiles(g);
    const dim3 nb = node_launch(T), bs(kBX, kBY);
    const bool gen = m.general != 0;
    switch (g.nd) {
        case 1: hipLaunchKernelGGL((k_visc_flux<1, false>), nb, bs, 0, s, U, G, g, ph, m, T); break;
        case 2:
            if (gen) hipLaunchKernelGGL((k_visc_flux<2, true>), nb, bs, 0, s, U, G, g, ph, m, T);
            else hipLaunchKernelGGL((k_visc_flux<2, false>), nb, bs, 0, s, U, G, g, ph, m, T);
            break;
        default:
            if (gen) {
                hipLaunchKernelGGL((k_visc_flux<3, true>), nb, bs, 0, s, U, G, g, ph, m, T);
            } else {
                const int tx_n = (int)((g.n[0] + kZX - 1) / kZX), ty_n = (int)((g.n[1] + kZY - 1) / kZY);
                const int ntiles = tx_n * ty_n * (int)((g.n[2] + kZC - 1) / kZC);
                const int per = (ntiles + kXcds - 1) / kXcds;
                hipLaunchKernelGGL(k_visc_flux_zm, dim3((unsigned)(per * kXcds)), dim3(kZX, kZY), 0, s, U, G, g, ph,
                                   m, tx_n, ty_n, ntiles, per);
            }
    }
    return hipGetLastError();
}

hipError_t launch_finish(const Grid &g, const Phys &ph, const Metrics &m, const double *Racc, const double *G,
                         double *Rout, RkStage rs, double dt, double *U, double *dU, int mode, hipStream_t s) {
    const bool gen = m.general != 0;
    switch (g.nd) {
        case 1: return finish_nd<1, false>(g, ph, m, Racc, G, Rout, rs, dt, U, dU, mode, s);
        case 2:
            return gen ? finish_nd<2, true>(g, ph, m, Racc, G, Rout, rs, dt, U, dU, mode, s)
                       : finish_nd<2, false>(g, ph, m, Racc, G, Rout, rs, dt, U, dU, mode, s);
        default:
            return gen ? finish_nd<3, true>(g, ph, m, Racc, G, Rout, rs, dt, U, dU, mode, s)
                       : finish_nd<3, false>(g, ph, m, Racc, G, Rout, rs, dt, U, dU, mode, s);
    }
}

hipError_t launch_dt(const Grid &g, const Phys &ph, const Metrics &m, const double *U, unsigned long long *slot,
                     hipStream_t s) {
    dim3 nb = node_grid(g);
    const dim3 bs(kBX, kBY);
    const unsigned plane_blocks = nb.x * nb.y;
    unsigned gz = (1024 + plane_blocks - 1) / plane_blocks;
    if (gz < 1) gz = 1;
    if (gz > nb.z) gz = nb.z;
    nb.z = gz;
    const bool gen = m.general != 0;
    switch (g.nd) {
        case 1: hipLaunchKernelGGL((k_dt<1, false>), nb, bs, 0, s, U, g, ph, m, slot); break;
        case 2:
            if (gen) hipLaunchKernelGGL((k_dt<2, true>), nb, bs, 0, s, U, g, ph, m, slot);
            else hipLaunchKernelGGL((k_dt<2, false>), nb, bs, 0, s, U, g, ph, m, slot);
            break;
        default:
            if (gen) hipLaunchKernelGGL((k_dt<3, true>), nb, bs, 0, s, U, g, ph, m, slot);
            else hipLaunchKernelGGL((k_dt<3, false>), nb, bs, 0, s, U, g, ph, m, slot);
    }
    return hipGetLastError();
}

hipError_t launch_fill_u64(unsigned long long *p, unsigned long long v, int n, hipStream_t s) {
    hipLaunchKernelGGL(k_fill_u64, dim3((n + 63) / 64), dim3(64), 0, s, p, v, n);
    return hipGetLastError();
}

}  // namespace osbli
