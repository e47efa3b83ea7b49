// C ABI of libosbli (declared in include/osbli.h): parameter validation,
// workspace carve-up, context lifecycle and the per-call launch sequences.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <mutex>
#include <new>
#include <vector>

#include "internal.hpp"

using namespace osbli;

// Scratch of the allocation-free substep (osbli_rk_substep_noalloc): the
// residual accumulator and the viscous fluxes of one grid, in one file-scope
// device array that every GPU the library runs on holds until the process
// ends.  Host code never passes the array's name to a kernel: its device
// address is resolved once per device (hipGetSymbolAddress, that device
// current) when a context is set up on it, and kept in scratch_ptr.
constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) char scratch[kScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex scratch_mu;
void *scratch_ptr[kMaxDevices] = {};
hipError_t scratch_err[kMaxDevices] = {};

// the scratch address on device dev (which must be current); nullptr on failure
void *resolve_scratch(int dev, hipError_t *err) {
    *err = hipSuccess;
    if (dev < 0 || dev >= kMaxDevices) {
        *err = hipErrorInvalidDevice;
        return nullptr;
    }
    std::lock_guard<std::mutex> lk(scratch_mu);
    if (!scratch_ptr[dev] && scratch_err[dev] == hipSuccess) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) scratch_err[dev] = e != hipSuccess ? e : hipErrorInvalidSymbol;
        else scratch_ptr[dev] = p;
    }
    *err = scratch_err[dev];
    return scratch_ptr[dev];
}
}  // namespace

// optional HIP-event timing of each kernel class on the launch stream
struct Prof {
    int on = 0;
    std::vector<hipEvent_t> pool;
    struct Pending { int cls; hipEvent_t a, b; };
    std::vector<Pending> pending;
    double ms[OSBLI_K_COUNT] = {0};
    long long cnt[OSBLI_K_COUNT] = {0};
};

struct osbli_ctx {
    Prof prof;
    osbli_params p;
    Grid g;
    Phys ph;
    Metrics m;
    Layout L;
    char *ws;
    size_t ws_bytes;
    unsigned *flags;
    unsigned long long *red;
    double *Racc, *G;
    uint8_t *mask[3];
    uint16_t *wts;
    int sensor_ready;      // weights set
    int sensor_every;      // refresh the routing masks at every substage (else at stage 0)
    float zcut;            // logit of the routing threshold
    int64_t seg[3];        // sweep segment lengths (0: the default rule)
    hipStream_t last;
    int device;
    char *scratch;         // this device's scratch array (allocation-free substep), or null
    hipError_t scratch_err;
    int nstages;           // Runge-Kutta substages per step (3 or 5)
    double rkA[5], rkB[5]; // their 2N coefficients
    void *cwork;           // central path: the store-all strategy's work arrays (null: StoreSome)
    char err[320];
};

namespace {

int set_err(osbli_ctx *c, int code, const char *fmt, ...) {
    if (c) {
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(c->err, sizeof(c->err), fmt, ap);
        va_end(ap);
    }
    return code;
}

#define HIP_TRY(ctx, call)                                                                              \
    do {                                                                                                \
        hipError_t e__ = (call);                                                                        \
        if (e__ != hipSuccess)                                                                          \
            return set_err((ctx), OSBLI_EDEVICE, "%s: %s", #call, hipGetErrorString(e__));             \
    } while (0)

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// validates p; fills Grid; returns 0 or a message in buf
int make_grid(const osbli_params *p, Grid &g, char *buf, size_t nb) {
    if (!p) { snprintf(buf, nb, "null params"); return -1; }
    if (p->ndim < 1 || p->ndim > 3) { snprintf(buf, nb, "ndim must be 1..3"); return -1; }
    g.nd = p->ndim;
    g.nc = p->ndim + 2;
    for (int d = 0; d < 3; ++d) {
        const bool act = d < p->ndim;
        g.n[d] = act ? p->n[d] : 1;
        g.h[d] = act ? kGhost : 0;
        g.e[d] = g.n[d] + 2 * g.h[d];
        g.periodic[d] = 0;
        if (!act) {
            if (p->n[d] != 1 && p->n[d] != 0) { snprintf(buf, nb, "n[%d] must be 1 for unused directions", d); return -1; }
            continue;
        }
        const int k0 = p->bc_kind[d][0], k1 = p->bc_kind[d][1];
        if (k0 < 0 || k0 > 4 || k1 < 0 || k1 > 4) { snprintf(buf, nb, "bad bc kind in direction %d", d); return -1; }
        if ((k0 == OSBLI_PERIODIC) != (k1 == OSBLI_PERIODIC)) {
            snprintf(buf, nb, "periodic must be set on both sides of direction %d", d);
            return -1;
        }
        g.periodic[d] = k0 == OSBLI_PERIODIC;
        const int64_t nmin = g.periodic[d] ? 6 : 5;
        if (p->n[d] < nmin) { snprintf(buf, nb, "n[%d] = %lld below %lld", d, (long long)p->n[d], (long long)nmin); return -1; }
        // grid limits of the pointwise launches (y blocks of 4, z one block per plane)
        const int64_t nmax = d == 0 ? (int64_t(1) << 26) : (d == 1 ? int64_t(4) * 65535 : 65535);
        if (p->n[d] > nmax) { snprintf(buf, nb, "n[%d] too large", d); return -1; }
    }
    g.es[0] = 1;
    g.es[1] = g.e[0];
    g.es[2] = g.e[0] * g.e[1];
    g.enpts = g.e[0] * g.e[1] * g.e[2];
    g.is[0] = 1;
    g.is[1] = g.n[0];
    g.is[2] = g.n[0] * g.n[1];
    g.nint = g.n[0] * g.n[1] * g.n[2];
    if (!(p->gamma > 1.0)) { snprintf(buf, nb, "gamma must exceed 1"); return -1; }
    if (p->scheme < OSBLI_WENOZ5 || p->scheme > OSBLI_WENOZ7) { snprintf(buf, nb, "bad scheme"); return -1; }
    if (p->scheme == OSBLI_WENOZ7) {
        if (p->mesh == OSBLI_MESH_GENERAL && p->ndim > 1) {
            snprintf(buf, nb, "WENO-7Z takes separable meshes");
            return -1;
        }
        for (int d = 0; d < p->ndim; ++d)
            for (int s = 0; s < 2; ++s)
                if (p->bc_kind[d][s] == OSBLI_ISOTHERMAL_WALL || p->bc_kind[d][s] == OSBLI_ADIABATIC_WALL) {
                    snprintf(buf, nb, "WENO-7Z takes periodic, extrapolated or Dirichlet ends");
                    return -1;
                }
        if (p->sensor) { snprintf(buf, nb, "sensor routing needs TENO5"); return -1; }
    }
    if (p->scheme == OSBLI_CENTRAL4 && (p->mesh == OSBLI_MESH_GENERAL && p->ndim > 1)) {
        snprintf(buf, nb, "the central path takes separable meshes of uniform spacing");
        return -1;
    }
    if (p->scheme == OSBLI_CENTRAL4 && p->sensor) { snprintf(buf, nb, "sensor routing needs TENO5"); return -1; }
    if (p->rk < OSBLI_RK3 || p->rk > OSBLI_RK4) { snprintf(buf, nb, "bad Runge-Kutta scheme %d", p->rk); return -1; }
    if (p->form != OSBLI_FORM_FP64 && p->form != OSBLI_FORM_MIXED) { snprintf(buf, nb, "bad form %d", p->form); return -1; }
    if (p->form == OSBLI_FORM_MIXED && p->scheme != OSBLI_WENOZ5 && p->scheme != OSBLI_TENO5) {
        snprintf(buf, nb, "the precision form takes WENO-Z5 or TENO5");
        return -1;
    }
    if (p->sensor != 0 && p->sensor != 1) { snprintf(buf, nb, "bad sensor flag"); return -1; }
    if (p->sensor && (p->scheme != OSBLI_TENO5 || (p->mesh == OSBLI_MESH_GENERAL && p->ndim > 1))) {
        snprintf(buf, nb, "sensor routing needs TENO5 on a separable mesh");
        return -1;
    }
    if (p->mesh != OSBLI_MESH_SEPARABLE && p->mesh != OSBLI_MESH_GENERAL) { snprintf(buf, nb, "bad mesh kind"); return -1; }
    bool walls = false;
    for (int d = 0; d < p->ndim; ++d)
        for (int s = 0; s < 2; ++s)
            walls |= p->bc_kind[d][s] == OSBLI_ISOTHERMAL_WALL || p->bc_kind[d][s] == OSBLI_ADIABATIC_WALL;
    if ((p->Re > 0.0 || walls) && !(p->Minf > 0.0)) { snprintf(buf, nb, "Minf must be positive"); return -1; }
    if (p->Re > 0.0 && !(p->Pr > 0.0)) { snprintf(buf, nb, "Pr must be positive"); return -1; }
    if (p->scheme == OSBLI_TENO5 && !(p->teno_CT > 0.0 && p->teno_CT < 1.0 / 3.0)) {
        snprintf(buf, nb, "teno_CT must lie in (0, 1/3)");
        return -1;
    }
    if (p->scheme == OSBLI_TENO6 && !(p->teno_CT > 0.0 && p->teno_CT < 0.25)) {
        snprintf(buf, nb, "teno_CT must lie in (0, 1/4) for TENO6");
        return -1;
    }
    if (!(p->eps >= 1e-40 && p->eps <= 1.0)) { snprintf(buf, nb, "eps must lie in [1e-40, 1]"); return -1; }
    return 0;
}

bool general_mesh(const osbli_params *p) { return p->mesh == OSBLI_MESH_GENERAL && p->ndim >= 2; }

Layout make_layout(const osbli_params *p, const Grid &g) {
    Layout L;
    size_t off = 0;
    L.flags = off; off += 256;
    L.red = off; off += 256;
    const bool gen = general_mesh(p);
    for (int d = 0; d < 3; ++d) {
        L.invh[d] = off;
        if (!gen && d < g.nd) off += align256(sizeof(double) * g.n[d]);
    }
    L.S = off;
    if (gen) off += align256(sizeof(double) * g.nd * g.nd * g.enpts);
    L.J = off;
    if (gen) off += align256(sizeof(double) * g.enpts);
    // region shared by the per-substage arrays and the one-off coordinate staging
    L.Racc = off;
    size_t racc = align256(sizeof(double) * g.nc * g.nint);
    L.G = L.Racc + racc;
    size_t gsz = p->Re > 0.0 ? align256(sizeof(double) * gflux_count(g.nd, gen) * g.nint) : 0;
    size_t stage;
    if (p->mesh == OSBLI_MESH_GENERAL && g.nd >= 2)
        stage = align256(sizeof(double) * g.nd * g.nint) + (g.nd == 3 ? align256(sizeof(double) * 9 * g.nint) : 0);
    else
        stage = align256(sizeof(double) * (g.n[0] + g.n[1] + g.n[2]));
    L.stage = off;
    size_t region = racc + gsz > stage ? racc + gsz : stage;
    off += region;
    for (int d = 0; d < 3; ++d) {
        L.mask[d] = off;
        if (p->sensor && d < g.nd) off += align256((size_t)iface_count(g, d));
    }
    L.wts = off;
    if (p->sensor) off += align256(2 * 1441);
    L.total = off;
    return L;
}

Phys make_phys(const osbli_params *p) {
    Phys ph;
    ph.gamma = p->gamma;
    ph.gm1 = p->gamma - 1.0;
    ph.Re = p->Re;
    ph.Pr = p->Pr;
    ph.Minf = p->Minf;
    ph.M2 = p->Minf * p->Minf;
    ph.Ts = p->Ts_over_Tref;
    ph.CT = p->teno_CT;
    ph.eps = p->eps;
    // With x_r = tau/(beta_r + eps) <= X for each of the K stencils, every
    // gamma_r = (1 + x_r)^6 >= 1 while C_T sum(gamma) <= K C_T (1 + X)^6;
    // X = (2 K C_T)^(-1/6) - 1 makes that 1/2, so no stencil can be cut (the
    // factor 2 covers the rounding of the kernels' evaluation of x_r).
    {
        const int K = p->scheme == OSBLI_TENO6 ? 4 : 3;
        const double q = 2.0 * K * p->teno_CT;
        ph.teno_fast = (p->scheme == OSBLI_TENO5 || p->scheme == OSBLI_TENO6) && q > 0.0 && q < 1.0
                           ? pow(q, -1.0 / 6.0) - 1.0
                           : 0.0;
    }
    ph.viscous = p->Re > 0.0;
    ph.mu_re = ph.viscous ? 1.0 / p->Re : 0.0;
    ph.kheat = ph.viscous ? 1.0 / ((p->gamma - 1.0) * ph.M2 * p->Pr * p->Re) : 0.0;
    const double gp = ph.viscous ? p->gamma / p->Pr : 0.0;
    ph.nu_fac = gp > 4.0 / 3.0 ? gp : 4.0 / 3.0;
    ph.sutherland = p->sutherland;
    ph.scheme = p->scheme;
    ph.roe = p->roe_avg;
    ph.mixed = p->form == OSBLI_FORM_MIXED;
    ph.dilate = 1;
    return ph;
}

// 2N coefficients of the context's Runge-Kutta scheme (section 2.7; the
// coefficients are cited there, not printed).
//   RK3:     A = (0, -5/9, -153/128), B = (1/3, 15/16, 8/15);
//   RK4:     Carpenter and Kennedy's five-stage fourth-order scheme (their
//            published rationals);
//   RK3_SSP: Gottlieb and Shu's strong-stability-preserving member of the
//            third-order 2N family, fixed by its first node c2 = B_0 =
//            0.924574 (ssp_family below gives the rest).
// ssp_family(c3): with nodes c2 and c3 the third-order conditions fix the
// weights w3 = (2 - 3 c2) / (6 c3 (c3 - c2)), w2 = (2 - 3 c3) / (6 c2 (c2 -
// c3)), w1 = 1 - w2 - w3 and a32 = 1 / (6 w3 c2); the 2N recursion then
// needs B_1 = a32, A_1 = (c3 - c2 - a32) / a32, B_2 = w3, A_2 = (w2 - B_1) /
// B_2, and reproduces the first weight only if
//   w1 = c2 + B_1 A_1 + B_2 A_2 A_1,
// which is the residual returned (its root is the scheme's c3).
double ssp_family(double c3, double *A, double *B) {
    const double c2 = 0.924574;
    const double w3 = (2.0 - 3.0 * c2) / (6.0 * c3 * (c3 - c2));
    const double w2 = (2.0 - 3.0 * c3) / (6.0 * c2 * (c2 - c3));
    const double w1 = 1.0 - w2 - w3;
    const double a32 = 1.0 / (6.0 * w3 * c2);
    A[0] = 0.0;
    B[0] = c2;
    B[1] = a32;
    A[1] = (c3 - c2 - a32) / a32;
    B[2] = w3;
    A[2] = (w2 - B[1]) / B[2];
    return w1 - (c2 + B[1] * A[1] + B[2] * A[2] * A[1]);
}

int rk_setup(int rk, double *A, double *B) {
    if (rk == OSBLI_RK4) {
        const double a[5] = {0.0, -567301805773.0 / 1357537059087.0, -2404267990393.0 / 2016746695238.0,
                             -3550918686646.0 / 2091501179385.0, -1275806237668.0 / 842570457699.0};
        const double b[5] = {1432997174477.0 / 9575080441755.0, 5161836677717.0 / 13612068292357.0,
                             1720146321549.0 / 2090206949498.0, 3134564353537.0 / 4481467310338.0,
                             2277821191437.0 / 14882151754819.0};
        for (int k = 0; k < 5; ++k) {
            A[k] = a[k];
            B[k] = b[k];
        }
        return 5;
    }
    if (rk == OSBLI_RK3_SSP) {
        // secant iteration for the root c3 (about 0.3735) from 0.35 and 0.40
        double x0 = 0.35, x1 = 0.40;
        double f0 = ssp_family(x0, A, B), f1 = ssp_family(x1, A, B);
        for (int it = 0; it < 60 && f1 != 0.0 && x1 != x0; ++it) {
            const double x2 = x1 - f1 * (x1 - x0) / (f1 - f0);
            x0 = x1;
            f0 = f1;
            x1 = x2;
            f1 = ssp_family(x1, A, B);
        }
        ssp_family(x1, A, B);
        return 3;
    }
    const double a[3] = {0.0, -5.0 / 9.0, -153.0 / 128.0}, b[3] = {1.0 / 3.0, 15.0 / 16.0, 8.0 / 15.0};
    for (int k = 0; k < 3; ++k) {
        A[k] = a[k];
        B[k] = b[k];
    }
    return 3;
}

hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

hipEvent_t take_event(osbli_ctx *c) {
    if (!c->prof.pool.empty()) {
        hipEvent_t e = c->prof.pool.back();
        c->prof.pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// brackets one launch group with events when profiling is on
struct Timed {
    osbli_ctx *c;
    int cls;
    hipStream_t s;
    hipEvent_t a = nullptr;
    Timed(osbli_ctx *c_, int cls_, hipStream_t s_) : c(c_), cls(cls_), s(s_) {
        if (c->prof.on && (a = take_event(c)) != nullptr) hipEventRecord(a, s);
    }
    ~Timed() {
        if (!a) return;
        hipEvent_t b = take_event(c);
        if (!b) { c->prof.pool.push_back(a); return; }
        hipEventRecord(b, s);
        c->prof.pending.push_back({cls, a, b});
    }
};

int resolve_profile(osbli_ctx *c) {
    for (auto &p : c->prof.pending) {
        if (hipEventSynchronize(p.b) != hipSuccess) return set_err(c, OSBLI_EDEVICE, "event synchronize failed");
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, p.a, p.b) != hipSuccess) return set_err(c, OSBLI_EDEVICE, "event timing failed");
        c->prof.ms[p.cls] += ms;
        c->prof.cnt[p.cls] += 1;
        c->prof.pool.push_back(p.a);
        c->prof.pool.push_back(p.b);
    }
    c->prof.pending.clear();
    return OSBLI_OK;
}

RkStage stage_of(const osbli_ctx *c, int s) {
    return RkStage{c->rkA[s], c->rkB[s], s == 0, s == c->nstages - 1};
}

// convective sweeps of every direction into R (first stores, later accumulate)
hipError_t convective_all(osbli_ctx *c, const double *U, double *R, hipStream_t s) {
    const bool route = c->p.sensor && c->sensor_ready;
    for (int d = 0; d < c->g.nd; ++d) {
        Timed t(c, OSBLI_K_SWEEP_X + d, s);
        hipError_t e = launch_convective(c->g, c->ph, c->m, U, R, c->flags, d, d == 0, route ? c->mask[d] : nullptr,
                                         c->seg[d], s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t sensor_all(osbli_ctx *c, const double *U, hipStream_t s) {
    Timed t(c, OSBLI_K_SENSOR, s);
    for (int d = 0; d < c->g.nd; ++d) {
        hipError_t e = launch_sensor(c->g, c->ph, U, d, c->wts, c->zcut, c->mask[d], s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace

extern "C" {

int osbli_abi_version(void) { return OSBLI_ABI_VERSION; }

size_t osbli_workspace_bytes(const osbli_params *p) {
    Grid g;
    char buf[200];
    if (make_grid(p, g, buf, sizeof buf) != 0) return 0;
    return make_layout(p, g).total;
}

int osbli_init_grid(osbli_ctx **out, const osbli_params *p, const double *x, const double *y, const double *z,
                    void *workspace, size_t ws_bytes, void *stream) {
    if (!out) return OSBLI_EINVAL;
    *out = nullptr;
    osbli_ctx *c = new (std::nothrow) osbli_ctx();
    if (!c) return OSBLI_EINVAL;
    c->err[0] = 0;
    *out = c;
    if (make_grid(p, c->g, c->err, sizeof c->err) != 0) return OSBLI_EINVAL;
    c->p = *p;
    for (int d = p->ndim; d < 3; ++d) c->p.n[d] = 1;
    c->ph = make_phys(p);
    c->nstages = rk_setup(p->rk, c->rkA, c->rkB);
    c->L = make_layout(p, c->g);
    if (!workspace) return set_err(c, OSBLI_EINVAL, "null workspace");
    if (ws_bytes < c->L.total)
        return set_err(c, OSBLI_ENOSPACE, "workspace %zu bytes, need %zu", ws_bytes, c->L.total);
    if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0) return set_err(c, OSBLI_EINVAL, "workspace not 256-byte aligned");
    const double *X[3] = {x, y, z};
    for (int d = 0; d < p->ndim; ++d)
        if (!X[d]) return set_err(c, OSBLI_EINVAL, "coordinates of direction %d missing", d);
    if (p->scheme == OSBLI_CENTRAL4) {
        // the expanded second derivatives assume a uniform spacing per direction
        for (int d = 0; d < p->ndim; ++d) {
            const int64_t N = c->g.n[d];
            const double h = X[d][1] - X[d][0];
            if (!(h > 0.0)) return set_err(c, OSBLI_EINVAL, "central path: coordinates of direction %d not increasing", d);
            for (int64_t i = 1; i + 1 < N; ++i)
                if (fabs((X[d][i + 1] - X[d][i]) - h) > 1e-10 * h)
                    return set_err(c, OSBLI_EINVAL, "central path: spacing of direction %d not uniform", d);
            if (c->g.periodic[d] && fabs(p->period[d] - N * h) > 1e-10 * N * h)
                return set_err(c, OSBLI_EINVAL, "central path: period of direction %d is not n h", d);
        }
    }
    HIP_TRY(c, hipGetDevice(&c->device));
    // the allocation-free substep's scratch on this device (a failure here
    // only disables that entry point)
    c->scratch = static_cast<char *>(resolve_scratch(c->device, &c->scratch_err));
    hipStream_t s = as_stream(stream);
    c->last = s;
    c->ws = static_cast<char *>(workspace);
    c->ws_bytes = ws_bytes;
    c->flags = reinterpret_cast<unsigned *>(c->ws + c->L.flags);
    c->red = reinterpret_cast<unsigned long long *>(c->ws + c->L.red);
    c->Racc = reinterpret_cast<double *>(c->ws + c->L.Racc);
    c->G = reinterpret_cast<double *>(c->ws + c->L.G);
    for (int d = 0; d < 3; ++d) c->mask[d] = reinterpret_cast<uint8_t *>(c->ws + c->L.mask[d]);
    c->wts = reinterpret_cast<uint16_t *>(c->ws + c->L.wts);
    c->sensor_ready = 0;
    c->sensor_every = 0;
    c->zcut = 0.0f;
    HIP_TRY(c, launch_fill_u64(reinterpret_cast<unsigned long long *>(c->ws), 0ull, 64, s));

    const bool gen = general_mesh(p);
    c->m.general = gen;
    const Grid &g = c->g;
    double *stage = reinterpret_cast<double *>(c->ws + c->L.stage);
    if (!gen) {
        // separable: 1D coordinate arrays (a 1D or separable mesh)
        int64_t off = 0;
        for (int d = 0; d < p->ndim; ++d) {
            if (p->mesh == OSBLI_MESH_SEPARABLE) {
                HIP_TRY(c, hipMemcpyAsync(stage + off, X[d], sizeof(double) * g.n[d], hipMemcpyHostToDevice, s));
            } else {
                // 1D general mesh == separable
                HIP_TRY(c, hipMemcpyAsync(stage + off, X[d], sizeof(double) * g.n[d], hipMemcpyHostToDevice, s));
            }
            off += g.n[d];
        }
        double *invh[3];
        for (int d = 0; d < 3; ++d) {
            invh[d] = reinterpret_cast<double *>(c->ws + c->L.invh[d]);
            c->m.invh[d] = d < p->ndim ? invh[d] : nullptr;
        }
        HIP_TRY(c, launch_metrics_separable(g, stage, invh, p->period, s));
        c->m.S = nullptr;
        c->m.J = nullptr;
    } else {
        for (int d = 0; d < p->ndim; ++d)
            HIP_TRY(c, hipMemcpyAsync(stage + d * g.nint, X[d], sizeof(double) * g.nint, hipMemcpyHostToDevice, s));
        double *S = reinterpret_cast<double *>(c->ws + c->L.S);
        double *J = reinterpret_cast<double *>(c->ws + c->L.J);
        double *extra = stage + ((sizeof(double) * g.nd * g.nint + 255) / 256) * 32;
        HIP_TRY(c, launch_metrics_general(g, stage, extra, S, J, p->period, s));
        c->m.S = S;
        c->m.J = J;
        for (int d = 0; d < 3; ++d) c->m.invh[d] = nullptr;
    }
    HIP_TRY(c, hipStreamSynchronize(s));
    return OSBLI_OK;
}

int osbli_apply_bc(osbli_ctx *c, double *U, void *stream) {
    if (!c || !U) return set_err(c, OSBLI_EINVAL, "null argument");
    hipStream_t s = as_stream(stream);
    c->last = s;
    Timed t(c, OSBLI_K_BC, s);
    HIP_TRY(c, launch_bc(c->g, c->ph, c->p, U, s));
    return OSBLI_OK;
}

int osbli_residual(osbli_ctx *c, const double *U, double *R, void *stream) {
    if (!c || !U || !R) return set_err(c, OSBLI_EINVAL, "null argument");
    if ((const void *)U == (const void *)R) return set_err(c, OSBLI_EINVAL, "R aliases U");
    hipStream_t s = as_stream(stream);
    c->last = s;
    if (c->p.scheme == OSBLI_CENTRAL4) {
        Timed t(c, OSBLI_K_CENTRAL, s);
        HIP_TRY(c, launch_central(c->g, c->ph, c->m, U, c->G, c->cwork, R, s));
        return OSBLI_OK;
    }
    if (c->p.sensor && c->sensor_ready) HIP_TRY(c, sensor_all(c, U, s));
    if (c->ph.viscous) {
        Timed t(c, OSBLI_K_VISC_FLUX, s);
        HIP_TRY(c, launch_viscous_fluxes(c->g, c->ph, c->m, U, c->G, s));
    }
    HIP_TRY(c, convective_all(c, U, R, s));
    if (c->ph.viscous) {
        Timed t(c, OSBLI_K_FINISH, s);
        HIP_TRY(c, launch_finish(c->g, c->ph, c->m, R, c->G, R, RkStage{0.0, 0.0, 1, 1}, 0.0, nullptr, nullptr, 0, s));
    }
    return OSBLI_OK;
}

int osbli_rk_stages(const osbli_ctx *c) { return c ? c->nstages : 0; }

int osbli_rk_coeffs(const osbli_ctx *c, double *A, double *B) {
    if (!c || !A || !B) return OSBLI_EINVAL;
    for (int k = 0; k < c->nstages; ++k) {
        A[k] = c->rkA[k];
        B[k] = c->rkB[k];
    }
    return OSBLI_OK;
}

int osbli_rk_substep(osbli_ctx *c, int stage, double dt, double *U, double *dU, void *stream) {
    if (!c || !U || !dU) return set_err(c, OSBLI_EINVAL, "null argument");
    if (stage < 0 || stage >= c->nstages) return set_err(c, OSBLI_EINVAL, "stage must be 0..%d", c->nstages - 1);
    if ((void *)U == (void *)dU) return set_err(c, OSBLI_EINVAL, "dU aliases U");
    hipStream_t s = as_stream(stream);
    c->last = s;
    if (c->p.scheme == OSBLI_CENTRAL4) {
        {
            Timed t(c, OSBLI_K_CENTRAL, s);
            HIP_TRY(c, launch_central(c->g, c->ph, c->m, U, c->G, c->cwork, c->Racc, s));
        }
        Timed t(c, OSBLI_K_FINISH, s);
        Phys pf = c->ph;
        pf.viscous = 0;  // the residual is complete: the pointwise finish only applies the stage
        HIP_TRY(c, launch_finish(c->g, pf, c->m, c->Racc, nullptr, nullptr, stage_of(c, stage), dt, U, dU, 1, s));
        return OSBLI_OK;
    }
    if (c->p.sensor && c->sensor_ready && (stage == 0 || c->sensor_every)) HIP_TRY(c, sensor_all(c, U, s));
    if (c->ph.viscous) {
        Timed t(c, OSBLI_K_VISC_FLUX, s);
        HIP_TRY(c, launch_viscous_fluxes(c->g, c->ph, c->m, U, c->G, s));
    }
    HIP_TRY(c, convective_all(c, U, c->Racc, s));
    {
        Timed t(c, OSBLI_K_FINISH, s);
        HIP_TRY(c, launch_finish(c->g, c->ph, c->m, c->Racc, c->G, nullptr, stage_of(c, stage), dt, U, dU, 1, s));
    }
    return OSBLI_OK;
}

size_t osbli_noalloc_scratch_bytes(void) { return kScratchBytes; }

int osbli_rk_substep_noalloc(osbli_ctx *c, int stage, double dt, double *U, double *dU, void *stream) {
    if (!c || !U || !dU) return set_err(c, OSBLI_EINVAL, "null argument");
    if (stage < 0 || stage >= c->nstages) return set_err(c, OSBLI_EINVAL, "stage must be 0..%d", c->nstages - 1);
    if ((void *)U == (void *)dU) return set_err(c, OSBLI_EINVAL, "dU aliases U");
    const size_t racc = align256(sizeof(double) * c->g.nc * c->g.nint);
    const size_t gsz =
        c->ph.viscous ? align256(sizeof(double) * gflux_count(c->g.nd, c->m.general != 0) * c->g.nint) : 0;
    if (racc + gsz > kScratchBytes)
        return set_err(c, OSBLI_ENOSPACE, "grid needs %zu bytes of scratch; the allocation-free substep holds %zu",
                       racc + gsz, kScratchBytes);
    if (!c->scratch)
        return set_err(c, OSBLI_EDEVICE, "scratch address of device %d unavailable: %s", c->device,
                       hipGetErrorString(c->scratch_err));
    double *Racc = reinterpret_cast<double *>(c->scratch);
    double *G = reinterpret_cast<double *>(c->scratch + racc);
    hipStream_t s = as_stream(stream);
    c->last = s;
    // the same launches as osbli_rk_substep, with the accumulator (stored,
    // not accumulated, by the first sweep) and the viscous fluxes (every
    // interior node written) in the scratch array; no profiling events
    if (c->p.scheme == OSBLI_CENTRAL4) {
        HIP_TRY(c, launch_central(c->g, c->ph, c->m, U, G, c->cwork, Racc, s));
        Phys pf = c->ph;
        pf.viscous = 0;
        HIP_TRY(c, launch_finish(c->g, pf, c->m, Racc, nullptr, nullptr, stage_of(c, stage), dt, U, dU, 1, s));
        return OSBLI_OK;
    }
    const bool route = c->p.sensor && c->sensor_ready;
    if (route && (stage == 0 || c->sensor_every))
        for (int d = 0; d < c->g.nd; ++d)
            HIP_TRY(c, launch_sensor(c->g, c->ph, U, d, c->wts, c->zcut, c->mask[d], s));
    if (c->ph.viscous) HIP_TRY(c, launch_viscous_fluxes(c->g, c->ph, c->m, U, G, s));
    for (int d = 0; d < c->g.nd; ++d)
        HIP_TRY(c, launch_convective(c->g, c->ph, c->m, U, Racc, c->flags, d, d == 0, route ? c->mask[d] : nullptr,
                                     c->seg[d], s));
    HIP_TRY(c, launch_finish(c->g, c->ph, c->m, Racc, G, nullptr, stage_of(c, stage), dt, U, dU, 1, s));
    return OSBLI_OK;
}

size_t osbli_central_store_all_bytes(const osbli_params *p) {
    Grid g;
    char buf[200];
    if (make_grid(p, g, buf, sizeof buf) != 0 || p->scheme != OSBLI_CENTRAL4) return 0;
    return central_work_bytes(g, p->Re > 0.0);
}

int osbli_central_store_all(osbli_ctx *c, void *work, size_t ws_bytes) {
    if (!c) return OSBLI_EINVAL;
    if (c->p.scheme != OSBLI_CENTRAL4) return set_err(c, OSBLI_EINVAL, "context does not use the central path");
    if (!work) {
        c->cwork = nullptr;
        return OSBLI_OK;
    }
    const size_t need = central_work_bytes(c->g, c->ph.viscous != 0);
    if (ws_bytes < need) return set_err(c, OSBLI_ENOSPACE, "store-all work %zu bytes, need %zu", ws_bytes, need);
    if (reinterpret_cast<uintptr_t>(work) % 256 != 0) return set_err(c, OSBLI_EINVAL, "work not 256-byte aligned");
    c->cwork = work;
    return OSBLI_OK;
}

int osbli_set_sweep_segments(osbli_ctx *c, const int64_t *seg) {
    if (!c || !seg) return set_err(c, OSBLI_EINVAL, "null argument");
    for (int d = 0; d < 3; ++d) {
        if (seg[d] < 0) return set_err(c, OSBLI_EINVAL, "segment length must be >= 0");
        c->seg[d] = seg[d];
    }
    return OSBLI_OK;
}

int osbli_compute_dt(osbli_ctx *c, const double *U, double cfl, double *dt_out, void *stream) {
    if (!c || !U || !dt_out) return set_err(c, OSBLI_EINVAL, "null argument");
    hipStream_t s = as_stream(stream);
    c->last = s;
    {
        Timed t(c, OSBLI_K_DT, s);
        HIP_TRY(c, launch_fill_u64(c->red, 0ull, 1, s));
        HIP_TRY(c, launch_dt(c->g, c->ph, c->m, U, c->red, s));
    }
    unsigned long long bits = 0;
    HIP_TRY(c, hipMemcpyAsync(&bits, c->red, sizeof bits, hipMemcpyDeviceToHost, s));
    HIP_TRY(c, hipStreamSynchronize(s));
    double smax;
    memcpy(&smax, &bits, sizeof smax);
    *dt_out = smax > 0.0 ? cfl / smax : 0.0;
    if (!(smax < __builtin_inf())) return set_err(c, OSBLI_ENONPHYS, "non-physical state in dt reduction");
    return OSBLI_OK;
}

int osbli_check(osbli_ctx *c) {
    if (!c) return OSBLI_EINVAL;
    unsigned f = 0;
    HIP_TRY(c, hipMemcpyAsync(&f, c->flags, sizeof f, hipMemcpyDeviceToHost, c->last));
    HIP_TRY(c, hipStreamSynchronize(c->last));
    if (f) {
        HIP_TRY(c, launch_fill_u64(reinterpret_cast<unsigned long long *>(c->flags), 0ull, 1, c->last));
        HIP_TRY(c, hipStreamSynchronize(c->last));
        return set_err(c, OSBLI_ENONPHYS, "non-physical state (rho <= 0, p <= 0 or NaN) met by a kernel");
    }
    return OSBLI_OK;
}

const char *osbli_last_error(const osbli_ctx *c) { return c ? c->err : "null context"; }

int osbli_sensor_set_weights(osbli_ctx *c, const uint16_t *w, int n, double threshold, int dilate, int every_substage,
                             void *stream) {
    if (!c || !w) return set_err(c, OSBLI_EINVAL, "null argument");
    if (!c->p.sensor) return set_err(c, OSBLI_EINVAL, "context created without sensor routing");
    if (n != 1441) return set_err(c, OSBLI_EINVAL, "expected 1441 bfloat16 weights, got %d", n);
    if (dilate < 0 || dilate > 2) return set_err(c, OSBLI_EINVAL, "dilate must be 0, 1 or 2");
    if (!(threshold > 0.0 && threshold < 1.0)) return set_err(c, OSBLI_EINVAL, "threshold must lie in (0, 1)");
    hipStream_t s = as_stream(stream);
    c->last = s;
    HIP_TRY(c, hipMemcpyAsync(c->wts, w, sizeof(uint16_t) * 1441, hipMemcpyHostToDevice, s));
    HIP_TRY(c, hipStreamSynchronize(s));
    c->zcut = (float)log(threshold / (1.0 - threshold));
    c->ph.dilate = dilate;
    c->sensor_every = every_substage != 0;
    c->sensor_ready = 1;
    return OSBLI_OK;
}

int osbli_sensor_update(osbli_ctx *c, const double *U, void *stream) {
    if (!c || !U) return set_err(c, OSBLI_EINVAL, "null argument");
    if (!c->p.sensor || !c->sensor_ready) return set_err(c, OSBLI_EINVAL, "sensor weights not set");
    hipStream_t s = as_stream(stream);
    c->last = s;
    HIP_TRY(c, sensor_all(c, U, s));
    return OSBLI_OK;
}

int osbli_sensor_stats(osbli_ctx *c, int64_t *smooth, int64_t *total) {
    if (!c || !smooth || !total) return set_err(c, OSBLI_EINVAL, "null argument");
    if (!c->p.sensor || !c->sensor_ready) return set_err(c, OSBLI_EINVAL, "sensor weights not set");
    hipStream_t s = c->last;
    HIP_TRY(c, launch_fill_u64(c->red + 1, 0ull, 1, s));
    int64_t tot = 0;
    for (int d = 0; d < c->g.nd; ++d) {
        HIP_TRY(c, launch_count_u8(c->mask[d], iface_count(c->g, d), c->red + 1, s));
        tot += iface_count(c->g, d);
    }
    unsigned long long cnt = 0;
    HIP_TRY(c, hipMemcpyAsync(&cnt, c->red + 1, sizeof cnt, hipMemcpyDeviceToHost, s));
    HIP_TRY(c, hipStreamSynchronize(s));
    *smooth = (int64_t)cnt;
    *total = tot;
    return OSBLI_OK;
}

int osbli_sensor_masks(osbli_ctx *c, int dir, uint8_t *dst, int64_t cap, void *stream) {
    if (!c || !dst) return set_err(c, OSBLI_EINVAL, "null argument");
    if (!c->p.sensor || !c->sensor_ready) return set_err(c, OSBLI_EINVAL, "sensor weights not set");
    if (dir < 0 || dir >= c->g.nd) return set_err(c, OSBLI_EINVAL, "direction %d out of range", dir);
    const int64_t n = iface_count(c->g, dir);
    if (cap < n) return set_err(c, OSBLI_ENOSPACE, "mask buffer holds %lld, need %lld", (long long)cap, (long long)n);
    hipStream_t s = as_stream(stream);
    c->last = s;
    HIP_TRY(c, hipMemcpyAsync(dst, c->mask[dir], (size_t)n, hipMemcpyDeviceToDevice, s));
    return OSBLI_OK;
}

int osbli_interface_count(osbli_ctx *c, int64_t *count) {
    if (!c || !count) return set_err(c, OSBLI_EINVAL, "null argument");
    int64_t tot = 0;
    for (int d = 0; d < c->g.nd; ++d) tot += iface_count(c->g, d);
    *count = tot;
    return OSBLI_OK;
}

int osbli_collect_labels(osbli_ctx *c, const double *U, float *feat, uint8_t *label, int64_t cap, int64_t *count,
                         void *stream) {
    if (!c || !U || !feat || !label || !count) return set_err(c, OSBLI_EINVAL, "null argument");
    if (c->p.scheme != OSBLI_TENO5) return set_err(c, OSBLI_EINVAL, "labels are TENO5 cut-off decisions");
    if (c->m.general) return set_err(c, OSBLI_EINVAL, "labels need a separable mesh");
    int64_t tot = 0;
    for (int d = 0; d < c->g.nd; ++d) tot += iface_count(c->g, d);
    *count = tot;
    if (cap < tot) return set_err(c, OSBLI_ENOSPACE, "label buffers hold %lld, need %lld", (long long)cap, (long long)tot);
    hipStream_t s = as_stream(stream);
    c->last = s;
    int64_t off = 0;
    for (int d = 0; d < c->g.nd; ++d) {
        HIP_TRY(c, launch_labels(c->g, c->ph, U, d, feat + off * 10, label + off, s));
        off += iface_count(c->g, d);
    }
    return OSBLI_OK;
}

size_t osbli_mlp_workspace_bytes(int64_t n) { return n > 0 ? mlp_workspace_bytes(n) : 0; }

int osbli_mlp_grad(const float *X, const uint8_t *y, int64_t n, const uint16_t *w, float w_neg, float *grad,
                   float *loss, void *workspace, size_t ws_bytes, void *stream) {
    if (!X || !y || !w || !grad || !workspace || n <= 0) return OSBLI_EINVAL;
    if (ws_bytes < mlp_workspace_bytes(n)) return OSBLI_ENOSPACE;
    return launch_mlp_grad(X, y, n, w, w_neg, grad, loss, static_cast<float *>(workspace), as_stream(stream)) ==
                   hipSuccess
               ? OSBLI_OK
               : OSBLI_EDEVICE;
}

int osbli_mlp_adam(float *master, uint16_t *w, const float *grad, float *m, float *v, int64_t t, float lr, float b1,
                   float b2, float eps, void *stream) {
    if (!master || !w || !grad || !m || !v || t < 1) return OSBLI_EINVAL;
    return launch_mlp_adam(master, w, grad, m, v, t, lr, b1, b2, eps, as_stream(stream)) == hipSuccess
               ? OSBLI_OK
               : OSBLI_EDEVICE;
}

int osbli_mlp_forward(const float *X, int64_t n, const uint16_t *w, float *z, int inference, void *stream) {
    if (!X || !w || !z || n <= 0) return OSBLI_EINVAL;
    return launch_mlp_forward(X, n, w, z, inference, as_stream(stream)) == hipSuccess ? OSBLI_OK : OSBLI_EDEVICE;
}

int osbli_profile_enable(osbli_ctx *c, int enable) {
    if (!c) return OSBLI_EINVAL;
    int rc = resolve_profile(c);
    if (rc != OSBLI_OK) return rc;
    for (int k = 0; k < OSBLI_K_COUNT; ++k) {
        c->prof.ms[k] = 0.0;
        c->prof.cnt[k] = 0;
    }
    c->prof.on = enable != 0;
    return OSBLI_OK;
}

int osbli_profile_read(osbli_ctx *c, int kernel_class, int64_t *count, double *total_ms) {
    if (!c || kernel_class < 0 || kernel_class >= OSBLI_K_COUNT || !count || !total_ms)
        return set_err(c, OSBLI_EINVAL, "bad profile query");
    int rc = resolve_profile(c);
    if (rc != OSBLI_OK) return rc;
    *count = c->prof.cnt[kernel_class];
    *total_ms = c->prof.ms[kernel_class];
    return OSBLI_OK;
}

void osbli_destroy(osbli_ctx *c) {
    if (!c) return;
    resolve_profile(c);
    for (hipEvent_t e : c->prof.pool) hipEventDestroy(e);
    delete c;
}

}  // extern "C"

// ===================================================================== batch
struct osbli_batch {
    int P;
    std::vector<osbli_ctx *> ctx;
    std::vector<BProb> hp;
    std::vector<BState> hs;
    Phys ph;
    int route;
    const uint16_t *w;
    float zcut;
    double cfl;
    unsigned *flags;
    BProb *dp;
    BState *ds;
    int64_t *dtab;
    BatchTables T;
    hipGraph_t graph[3];
    hipGraphExec_t exec[3];
    int captured;
    int sweep_blocks;      // workgroups per persistent sweep launch (0: defaults)
    char err[320];
};

namespace {

int bset_err(osbli_batch *b, int code, const char *fmt, ...) {
    if (b) {
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(b->err, sizeof(b->err), fmt, ap);
        va_end(ap);
    }
    return code;
}

#define HIP_BTRY(b, call)                                                                               \
    do {                                                                                                \
        hipError_t e__ = (call);                                                                        \
        if (e__ != hipSuccess)                                                                          \
            return bset_err((b), OSBLI_EDEVICE, "%s: %s", #call, hipGetErrorString(e__));              \
    } while (0)

constexpr int kTables = 8;
size_t batch_table_bytes(int P) { return align256(sizeof(int64_t) * kTables * (size_t)(P + 1)); }

// default segment length of a sweep (the single-grid rule)
int64_t default_seg(const Grid &g, int d) {
    const int o1 = d == 0 ? 1 : 0, o2 = d == 2 ? 1 : 2;
    return default_segment(g.n[d], g.n[o1] * g.n[o2]);
}

// host prefix tables -> device; totals into T
int upload_tables(osbli_batch *b, hipStream_t s) {
    const int P = b->P;
    std::vector<int64_t> h(kTables * (size_t)(P + 1), 0);
    int64_t *W0 = &h[0], *W1 = &h[(P + 1)], *PT = &h[2 * (P + 1)], *F0 = &h[3 * (P + 1)], *F1 = &h[4 * (P + 1)],
            *S0 = &h[5 * (P + 1)], *S1 = &h[6 * (P + 1)], *WX = &h[7 * (P + 1)];
    for (int p = 0; p < P; ++p) {
        BProb &q = b->hp[p];
        for (int d = 0; d < 2; ++d) {
            const int o1 = d == 0 ? 1 : 0;
            q.nseg[d] = (q.g.n[d] + q.seg[d] - 1) / q.seg[d];
            q.wpl[d] = (q.g.n[o1] + 63) / 64;
        }
        // x: lanes along x for rows of >= 64 interfaces (as the single-grid launch)
        const int64_t totalJ = q.g.n[1] * (q.g.n[0] + 1);
        const int64_t nwx = q.xl ? ((totalJ - 2) / 63 + q.xlpt) / q.xlpt : 0;
        const int64_t nw0 = q.xl ? 0 : q.nseg[0] * q.wpl[0];
        const int64_t nw1 = q.nseg[1] * q.wpl[1];
        WX[p + 1] = WX[p] + nwx;
        W0[p + 1] = W0[p] + nw0;
        W1[p + 1] = W1[p] + nw1;
        PT[p + 1] = PT[p] + (q.g.nint + 255) / 256;
        F0[p + 1] = F0[p] + 2 * q.g.e[1] * q.g.e[2];
        F1[p + 1] = F1[p] + 2 * q.g.e[0] * q.g.e[2];
        S0[p + 1] = S0[p] + (iface_count(q.g, 0) + 255) / 256;
        S1[p + 1] = S1[p] + (iface_count(q.g, 1) + 255) / 256;
    }
    HIP_BTRY(b, hipMemcpyAsync(b->dtab, h.data(), sizeof(int64_t) * h.size(), hipMemcpyHostToDevice, s));
    HIP_BTRY(b, hipMemcpyAsync(b->dp, b->hp.data(), sizeof(BProb) * P, hipMemcpyHostToDevice, s));
    HIP_BTRY(b, hipStreamSynchronize(s));
    BatchTables &T = b->T;
    T.w[0] = b->dtab;
    T.w[1] = b->dtab + (P + 1);
    T.pt = b->dtab + 2 * (P + 1);
    T.f[0] = b->dtab + 3 * (P + 1);
    T.f[1] = b->dtab + 4 * (P + 1);
    T.s[0] = b->dtab + 5 * (P + 1);
    T.s[1] = b->dtab + 6 * (P + 1);
    T.wx = b->dtab + 7 * (P + 1);
    T.tot_wx = WX[P];
    T.tot_w[0] = W0[P];
    T.tot_w[1] = W1[P];
    T.tot_pt = PT[P];
    T.tot_f[0] = F0[P];
    T.tot_f[1] = F1[P];
    T.tot_s[0] = S0[P];
    T.tot_s[1] = S1[P];
    return OSBLI_OK;
}

void drop_graphs(osbli_batch *b) {
    if (!b->captured) return;
    for (int s = 0; s < 3; ++s) {
        hipGraphExecDestroy(b->exec[s]);
        hipGraphDestroy(b->graph[s]);
    }
    b->captured = 0;
}

}  // namespace

extern "C" {

size_t osbli_batch_workspace_bytes(int nprob) {
    if (nprob < 1) return 0;
    return align256(sizeof(BProb) * nprob) + align256(sizeof(BState) * nprob) + batch_table_bytes(nprob);
}

int osbli_batch_create(osbli_batch **out, osbli_ctx *const *ctxs, int P, double *const *U, double *const *dU,
                       const double *t_end, double cfl, void *workspace, size_t ws_bytes, void *stream) {
    if (!out) return OSBLI_EINVAL;
    *out = nullptr;
    osbli_batch *b = new (std::nothrow) osbli_batch();
    if (!b) return OSBLI_EINVAL;
    *out = b;
    b->err[0] = 0;
    b->captured = 0;
    b->sweep_blocks = 0;
    if (P < 1 || !ctxs || !U || !dU || !t_end || !workspace) return bset_err(b, OSBLI_EINVAL, "null argument or P < 1");
    if (ws_bytes < osbli_batch_workspace_bytes(P)) return bset_err(b, OSBLI_ENOSPACE, "batch workspace too small");
    if (reinterpret_cast<uintptr_t>(workspace) % 256) return bset_err(b, OSBLI_EINVAL, "workspace not 256-byte aligned");
    if (!(cfl > 0.0)) return bset_err(b, OSBLI_EINVAL, "cfl must be positive");
    const osbli_ctx *c0 = ctxs[0];
    for (int p = 0; p < P; ++p) {
        const osbli_ctx *c = ctxs[p];
        if (!c || !U[p] || !dU[p]) return bset_err(b, OSBLI_EINVAL, "problem %d: null context or state", p);
        if (c->g.nd != 2 || c->m.general || c->ph.viscous)
            return bset_err(b, OSBLI_EINVAL, "problem %d: batching takes inviscid 2D separable problems", p);
        for (int d = 0; d < 2; ++d)
            for (int s2 = 0; s2 < 2; ++s2)
                if (c->p.bc_kind[d][s2] != OSBLI_PERIODIC && c->p.bc_kind[d][s2] != OSBLI_EXTRAPOLATE)
                    return bset_err(b, OSBLI_EINVAL, "problem %d: batching takes periodic / extrapolation BCs", p);
        if (c->p.scheme != OSBLI_WENOZ5 && c->p.scheme != OSBLI_TENO5)
            return bset_err(b, OSBLI_EINVAL, "problem %d: batching takes WENO-Z5 or TENO5", p);
        if (c->p.rk != OSBLI_RK3)
            return bset_err(b, OSBLI_EINVAL, "problem %d: batching takes the three-stage RK3", p);
        if (c->p.gamma != c0->p.gamma || c->p.scheme != c0->p.scheme || c->p.form != c0->p.form ||
            c->p.sensor != c0->p.sensor || c->p.roe_avg != c0->p.roe_avg || c->p.teno_CT != c0->p.teno_CT ||
            c->p.eps != c0->p.eps)
            return bset_err(b, OSBLI_EINVAL, "problem %d: physics differs from problem 0", p);
        if (c->p.sensor && (!c->sensor_ready || c->zcut != c0->zcut || c->ph.dilate != c0->ph.dilate))
            return bset_err(b, OSBLI_EINVAL, "problem %d: sensor weights unset or differ", p);
        if (!(t_end[p] > 0.0)) return bset_err(b, OSBLI_EINVAL, "problem %d: t_end must be positive", p);
    }
    b->P = P;
    b->ctx.assign(ctxs, ctxs + P);
    b->ph = c0->ph;
    b->route = c0->p.sensor && c0->sensor_ready;
    b->w = c0->wts;
    b->zcut = c0->zcut;
    b->cfl = cfl;
    b->flags = c0->flags;
    char *ws = static_cast<char *>(workspace);
    b->dp = reinterpret_cast<BProb *>(ws);
    b->ds = reinterpret_cast<BState *>(ws + align256(sizeof(BProb) * P));
    b->dtab = reinterpret_cast<int64_t *>(ws + align256(sizeof(BProb) * P) + align256(sizeof(BState) * P));
    b->hp.resize(P);
    b->hs.resize(P);
    for (int p = 0; p < P; ++p) {
        const osbli_ctx *c = ctxs[p];
        BProb &q = b->hp[p];
        q.g = c->g;
        q.U = U[p];
        q.dU = dU[p];
        q.R = c->Racc;
        q.xl = c->g.n[0] + 1 >= 64 ? 1 : 0;
        q.xlpt = kXlPerTile;
        for (int d = 0; d < 3; ++d) {
            q.invh[d] = c->m.invh[d];
            q.mask[d] = c->mask[d];
            q.seg[d] = d < 2 ? default_seg(c->g, d) : 1;
            q.nseg[d] = 1;
            q.wpl[d] = 1;
            for (int s2 = 0; s2 < 2; ++s2) q.bc[d][s2] = c->p.bc_kind[d][s2];
        }
        BState &st = b->hs[p];
        st.t = 0.0;
        st.dt = 0.0;
        st.tend = t_end[p];
        st.smax = 0ull;
        st.active = 1;
        st.pad = 0;
    }
    hipStream_t s = as_stream(stream);
    HIP_BTRY(b, hipMemcpyAsync(b->ds, b->hs.data(), sizeof(BState) * P, hipMemcpyHostToDevice, s));
    return upload_tables(b, s);
}

int osbli_batch_set_tiles(osbli_batch *b, const int64_t *seg, void *stream) {
    if (!b || !seg) return bset_err(b, OSBLI_EINVAL, "null argument");
    for (int p = 0; p < b->P; ++p)
        for (int d = 0; d < 2; ++d) {
            const int64_t v = seg[2 * p + d];
            if (v < 1) return bset_err(b, OSBLI_EINVAL, "segment length must be positive");
            if (d == 0 && b->hp[p].xl) {
                // lanes-along-x sweep: 63-interface runs per tile (clamped to 64)
                b->hp[p].xlpt = (int)(v > 64 ? 64 : v);
                continue;
            }
            b->hp[p].seg[d] = v > b->hp[p].g.n[d] ? b->hp[p].g.n[d] : v;
        }
    drop_graphs(b);
    return upload_tables(b, as_stream(stream));
}

int osbli_batch_set_grid(osbli_batch *b, int sweep_blocks) {
    if (!b) return OSBLI_EINVAL;
    if (sweep_blocks < 0 || sweep_blocks > 65536) return bset_err(b, OSBLI_EINVAL, "sweep_blocks must lie in 0..65536");
    b->sweep_blocks = sweep_blocks;
    drop_graphs(b);
    return OSBLI_OK;
}

int osbli_batch_capture(osbli_batch *b, void *stream) {
    if (!b) return OSBLI_EINVAL;
    hipStream_t s = as_stream(stream);
    if (!s) return bset_err(b, OSBLI_EINVAL, "capture needs a non-default stream");
    drop_graphs(b);
    for (int st = 0; st < 3; ++st) {
        HIP_BTRY(b, hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        hipError_t e = launch_batch_stage(b->dp, b->ds, b->T, b->P, b->ph, st, b->cfl, b->route, b->w, b->zcut,
                                          b->flags, b->sweep_blocks, s);
        hipGraph_t g = nullptr;
        hipError_t e2 = hipStreamEndCapture(s, &g);
        if (e != hipSuccess || e2 != hipSuccess) {
            if (g) hipGraphDestroy(g);
            for (int k = 0; k < st; ++k) {
                hipGraphExecDestroy(b->exec[k]);
                hipGraphDestroy(b->graph[k]);
            }
            return bset_err(b, OSBLI_EDEVICE, "graph capture of stage %d failed: %s", st,
                            hipGetErrorString(e != hipSuccess ? e : e2));
        }
        b->graph[st] = g;
        HIP_BTRY(b, hipGraphInstantiate(&b->exec[st], g, nullptr, nullptr, 0));
    }
    b->captured = 1;
    return OSBLI_OK;
}

int osbli_batch_substep(osbli_batch *b, int stage, void *stream) {
    if (!b) return OSBLI_EINVAL;
    if (stage < 0 || stage > 2) return bset_err(b, OSBLI_EINVAL, "stage must be 0..2");
    hipStream_t s = as_stream(stream);
    if (b->captured) {
        HIP_BTRY(b, hipGraphLaunch(b->exec[stage], s));
    } else {
        HIP_BTRY(b, launch_batch_stage(b->dp, b->ds, b->T, b->P, b->ph, stage, b->cfl, b->route, b->w, b->zcut,
                                       b->flags, b->sweep_blocks, s));
    }
    return OSBLI_OK;
}

int osbli_batch_step(osbli_batch *b, void *stream) {
    if (!b) return OSBLI_EINVAL;
    for (int st = 0; st < 3; ++st) {
        const int rc = osbli_batch_substep(b, st, stream);
        if (rc != OSBLI_OK) return rc;
    }
    return OSBLI_OK;
}

int osbli_batch_status(osbli_batch *b, double *t, int *active, int *nactive, void *stream) {
    if (!b) return OSBLI_EINVAL;
    hipStream_t s = as_stream(stream);
    HIP_BTRY(b, hipMemcpyAsync(b->hs.data(), b->ds, sizeof(BState) * b->P, hipMemcpyDeviceToHost, s));
    HIP_BTRY(b, hipStreamSynchronize(s));
    int n = 0;
    for (int p = 0; p < b->P; ++p) {
        if (t) t[p] = b->hs[p].t;
        if (active) active[p] = b->hs[p].active;
        n += b->hs[p].active != 0;
    }
    if (nactive) *nactive = n;
    return OSBLI_OK;
}

int osbli_batch_interior_points(osbli_batch *b, int64_t *points, int64_t *wave_tiles) {
    if (!b || !points) return OSBLI_EINVAL;
    int64_t n = 0;
    for (int p = 0; p < b->P; ++p) n += b->hp[p].g.nint;
    *points = n;
    if (wave_tiles) *wave_tiles = b->T.tot_w[0] + b->T.tot_w[1];
    return OSBLI_OK;
}

const char *osbli_batch_last_error(const osbli_batch *b) { return b ? b->err : "null batch"; }

void osbli_batch_destroy(osbli_batch *b) {
    if (!b) return;
    drop_graphs(b);
    delete b;
}

}  // extern "C"
