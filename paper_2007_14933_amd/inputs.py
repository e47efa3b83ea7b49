"""Seeded synthetic problem generators.

This module is shared by the GPU path's tests and benchmark and by the oracle's
tests.  It holds problem set-ups only (grids, initial states, constants):
no step of the numerical method.  The one piece of physics it uses is the
conversion of a primitive initial state (rho, u, p) to conserved variables,
which is part of stating an initial condition.

Array layout of every state: U[c][k][j][i], c = (rho, rho u_0 .. rho u_{nd-1},
rho E), three ghost nodes on both sides of every active direction (ghosts are
left at zero; the boundary-condition call fills them).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace
from typing import Optional, Tuple

import numpy as np

PERIODIC, EXTRAPOLATE, ISOTHERMAL, ADIABATIC, DIRICHLET = 0, 1, 2, 3, 4
WENOZ5, TENO5, TENO6, WENOJS5, WENOZ3, CENTRAL4, WENOZ7 = 0, 1, 2, 3, 4, 5, 6
RK3, RK3_SSP, RK4 = 0, 1, 2       # low-storage Runge-Kutta schemes (3, 3 and 5 substages)
NGHOST = 3


def rk_stages(rk):
    return 5 if rk == RK4 else 3


@dataclass
class Problem:
    name: str
    ndim: int
    n: Tuple[int, int, int]
    gamma: float = 1.4
    Re: float = 0.0               # <= 0: inviscid
    Pr: float = 0.72
    Minf: float = 1.0
    sutherland: int = 0
    Ts_over_Tref: float = 110.4 / 202.17
    scheme: int = TENO5
    teno_CT: float = 1e-5
    eps: float = 1e-16
    roe_avg: int = 1
    rk: int = RK3
    bc: Tuple = ((PERIODIC, PERIODIC),) * 3
    wall_T: Tuple = ((1.0, 1.0),) * 3
    period: Tuple[float, float, float] = (0.0, 0.0, 0.0)
    body_force: float = 0.0
    # separable meshes: one 1D coordinate array per direction
    coords1d: Optional[Tuple] = None
    # general meshes: full coordinate arrays (nz, ny, nx) per component
    coords_full: Optional[Tuple] = None
    U0: Optional[np.ndarray] = None
    cfl: float = 0.5
    t_end: float = 0.0
    nsteps: int = 0
    dt_fixed: float = 0.0
    meta: dict = field(default_factory=dict)

    @property
    def nc(self):
        return self.ndim + 2

    @property
    def separable(self):
        return self.coords1d is not None

    @property
    def npoints(self):
        return int(np.prod([self.n[d] for d in range(self.ndim)]))

    @property
    def coords(self):
        """Full coordinate arrays (nz, ny, nx) per component (None beyond ndim)."""
        if self.coords_full is not None:
            return self.coords_full
        nd = self.ndim
        shp = tuple(self.n[d] if d < nd else 1 for d in (2, 1, 0))
        out = []
        for d in range(3):
            if d >= nd:
                out.append(None)
                continue
            c = np.asarray(self.coords1d[d], dtype=np.float64)
            view = [1, 1, 1]
            view[2 - d] = c.size
            out.append(np.ascontiguousarray(np.broadcast_to(c.reshape(view), shp)))
        return tuple(out)

    def with_(self, **kw):
        return replace(self, **kw)


def ext_shape(ndim, n):
    e = [n[d] + 2 * NGHOST if d < ndim else 1 for d in range(3)]
    return (ndim + 2, e[2], e[1], e[0])


def int_shape(ndim, n):
    m = [n[d] if d < ndim else 1 for d in range(3)]
    return (ndim + 2, m[2], m[1], m[0])


def interior_view(ndim, U):
    sl = [slice(None)] + [slice(NGHOST, -NGHOST) if d < ndim else slice(None) for d in (2, 1, 0)]
    return U[tuple(sl)]


def conserved(gamma, rho, vel, p):
    """Primitive initial state -> conserved components (list of arrays)."""
    ke = sum(v * v for v in vel)
    return [rho] + [rho * v for v in vel] + [p / (gamma - 1.0) + 0.5 * rho * ke]


def _state(ndim, n, comps):
    U = np.zeros(ext_shape(ndim, n))
    Ui = interior_view(ndim, U)
    for c, a in enumerate(comps):
        Ui[c] = np.broadcast_to(a, Ui[c].shape)
    return U


def _mesh(coords1d, ndim):
    """Broadcast 1D coordinates to (nz, ny, nx) arrays (for evaluating ICs)."""
    axes = [np.asarray(coords1d[d]) if d < ndim else np.zeros(1) for d in range(3)]
    Z, Y, X = np.meshgrid(axes[2], axes[1], axes[0], indexing="ij")
    return X, Y, Z


# --------------------------------------------------------------- 1D Sod
def sod(N=400, scheme=WENOZ5, t_end=0.2, cfl=0.5):
    """Sod shock tube: (rho,u,p) = (1,0,1) | (0.125,0,0.1) split at x = 0.5,
    N cell-centred points on [0,1], zero-gradient ends, inviscid."""
    x = (np.arange(N) + 0.5) / N
    rho = np.where(x < 0.5, 1.0, 0.125)
    p = np.where(x < 0.5, 1.0, 0.1)
    g = 1.4
    U = _state(1, (N, 1, 1), [a.reshape(1, 1, N) for a in conserved(g, rho, [0.0 * x], p)])
    return Problem(name="sod%d" % N, ndim=1, n=(N, 1, 1), gamma=g, Re=0.0, scheme=scheme,
                   bc=((EXTRAPOLATE, EXTRAPOLATE), (PERIODIC, PERIODIC), (PERIODIC, PERIODIC)),
                   period=(1.0, 0.0, 0.0), coords1d=(x, None, None), U0=U, cfl=cfl,
                   t_end=t_end, nsteps=10 ** 9)


# ----------------------------------------------------- 1D Shu-Osher
def shu_osher(N=320, scheme=WENOZ5, t_end=1.8, dt=2e-4):
    """Shock / density-wave interaction: a Mach-3 shock at x = -4 moving into
    rho = 1 + 0.2 sin(5x) on [-5, 5], N cell-centred points, Dirichlet ends
    (ghost nodes hold the initial states: the post-shock state on the left,
    the undisturbed wave on the right), inviscid, fixed dt.  The printed
    right state (u, p) = (1, 0) is read as the standard (0, 1): p = 0 is not
    a gas state, and the standard set-up is a shock running into fluid at
    rest."""
    g = 1.4
    h = 10.0 / N
    xe = -5.0 + (np.arange(-NGHOST, N + NGHOST) + 0.5) * h   # nodes incl. ghosts
    left = xe < -4.0
    rho = np.where(left, 3.857143, 1.0 + 0.2 * np.sin(5.0 * xe))
    u = np.where(left, 2.629369, 0.0)
    p = np.where(left, 10.33333, 1.0)
    U = np.zeros(ext_shape(1, (N, 1, 1)))
    for c, a in enumerate(conserved(g, rho, [u], p)):
        U[c, 0, 0, :] = a
    x = xe[NGHOST:-NGHOST].copy()
    return Problem(name="shuosher%d" % N, ndim=1, n=(N, 1, 1), gamma=g, Re=0.0, scheme=scheme,
                   bc=((DIRICHLET, DIRICHLET), (PERIODIC, PERIODIC), (PERIODIC, PERIODIC)),
                   period=(10.0, 0.0, 0.0), coords1d=(x, None, None), U0=U, t_end=t_end,
                   dt_fixed=dt, nsteps=int(round(t_end / dt)))


# ----------------------------------------------------- 3D Taylor-Green vortex
def tgv(N=256, Re=1600.0, M=0.1, Pr=0.71, scheme=TENO5, nsteps=200, cfl=0.5):
    """Taylor-Green vortex on the periodic box [0, 2 pi)^3: u = sin x cos y cos z,
    v = -cos x sin y cos z, w = 0, p = 1/(gamma M^2) + (cos 2x + cos 2y)(cos 2z + 2)/16,
    T = 1 (rho = gamma M^2 p), constant viscosity."""
    g = 1.4
    L = 2.0 * math.pi
    x = L * np.arange(N) / N
    X, Y, Z = _mesh((x, x, x), 3)
    u = np.sin(X) * np.cos(Y) * np.cos(Z)
    v = -np.cos(X) * np.sin(Y) * np.cos(Z)
    w = np.zeros_like(u)
    p = 1.0 / (g * M * M) + (np.cos(2 * X) + np.cos(2 * Y)) * (np.cos(2 * Z) + 2.0) / 16.0
    rho = g * M * M * p
    U = _state(3, (N, N, N), conserved(g, rho, [u, v, w], p))
    return Problem(name="tgv%d" % N, ndim=3, n=(N, N, N), gamma=g, Re=Re, Pr=Pr, Minf=M,
                   scheme=scheme, period=(L, L, L), coords1d=(x, x, x), U0=U, cfl=cfl,
                   nsteps=nsteps)


# ------------------------------------------- 2D density wave (smooth, periodic)
def sinusoidal_mesh(Nx, Ny, A=0.04, Lx=2.0, Ly=2.0):
    """x = i dx + A sin(6 pi j dy / Ly), y = j dy + A sin(6 pi i dx / Lx) on [0,2)^2."""
    dx, dy = Lx / Nx, Ly / Ny
    J, I = np.meshgrid(np.arange(Ny), np.arange(Nx), indexing="ij")
    X = I * dx + A * np.sin(6 * math.pi * J * dy / Ly)
    Y = J * dy + A * np.sin(6 * math.pi * I * dx / Lx)
    return X.reshape(1, Ny, Nx), Y.reshape(1, Ny, Nx)


def density_wave(N=32, mesh="sinusoidal", scheme=WENOZ5, t=0.0, u=1.0, v=-0.5):
    """rho = 1 + 0.2 sin(pi (x + y - t (u + v))), (u, v) = (1, -0.5), p = 1, periodic."""
    g = 1.4
    if mesh == "sinusoidal":
        X, Y = sinusoidal_mesh(N, N)
        coords1d, coords_full = None, (X, Y, None)
    else:
        x = 2.0 * np.arange(N) / N
        coords1d, coords_full = (x, x, None), None
        X, Y, _ = _mesh(coords1d, 2)
    rho = 1.0 + 0.2 * np.sin(math.pi * (X + Y - t * (u + v)))
    U = _state(2, (N, N, 1), conserved(g, rho, [u + 0 * X, v + 0 * X], 1.0 + 0 * X))
    return Problem(name="dwave%d_%s" % (N, mesh), ndim=2, n=(N, N, 1), gamma=g, Re=0.0,
                   scheme=scheme, period=(2.0, 2.0, 0.0), coords1d=coords1d,
                   coords_full=coords_full, U0=U)


def density_wave_1d(N=32, scheme=WENOZ5, u=1.0, rk=RK3):
    """One-dimensional travelling density wave rho = 1 + 0.2 sin(pi (x - u t)),
    u = 1, p = 1, periodic on [0, 2)."""
    g = 1.4
    x = 2.0 * np.arange(N) / N
    rho = 1.0 + 0.2 * np.sin(math.pi * x)
    U = _state(1, (N, 1, 1), [a.reshape(1, 1, N) for a in conserved(g, rho, [u + 0 * x], 1.0 + 0 * x)])
    return Problem(name="dwave1d_%d" % N, ndim=1, n=(N, 1, 1), gamma=g, Re=0.0, scheme=scheme, rk=rk,
                   period=(2.0, 0.0, 0.0), coords1d=(x, None, None), U0=U, meta={"u": u})


def exact_density_wave(prob, t, u=1.0, v=-0.5):
    if prob.ndim == 1:
        return 1.0 + 0.2 * np.sin(math.pi * (prob.coords[0] - t * prob.meta.get("u", u)))
    X, Y = prob.coords[0], prob.coords[1]
    return 1.0 + 0.2 * np.sin(math.pi * (X + Y - t * (u + v)))


# ----------------------------------- 3D supersonic wall-bounded (precision form)
def tanh_wall_mesh(Ny, Ly, beta=2.5):
    j = np.arange(Ny)
    return Ly * (1.0 - np.tanh(beta * (1.0 - j / (Ny - 1))) / math.tanh(beta))


def wall_flow(nx=512, ny=256, nz=256, L=(100.0, 20.0, 20.0), M=2.0, Re=750.0, Pr=0.72,
              Tref=202.17, delta=3.0, beta=2.5, amp=0.01, nmodes=16, seed=1234,
              nsteps=100, cfl=0.5, scheme=TENO5):
    """Mach-2 flow over an isothermal wall (y = 0), tanh-stretched in y, periodic
    in x and z, extrapolation at the top.  Base profile u = tanh(3 y / delta),
    Crocco-Busemann temperature with T_w equal to the recovery temperature,
    uniform pressure, plus a seeded solenoidal perturbation u' = curl(f(y) A)
    with f = (y/delta)^2 exp(-(y/delta)^2), A a sum of random-phase Fourier
    modes, scaled to max |u'| = amp."""
    g = 1.4
    x = L[0] * np.arange(nx) / nx
    z = L[2] * np.arange(nz) / nz
    y = tanh_wall_mesh(ny, L[1], beta)
    Taw = 1.0 + math.sqrt(Pr) * (g - 1.0) / 2.0 * M * M
    rng = np.random.default_rng(seed)
    kx = rng.integers(1, 5, size=(3, nmodes))
    kz = rng.integers(-4, 5, size=(3, nmodes))
    ph = rng.uniform(0.0, 2.0 * math.pi, size=(3, nmodes))
    am = rng.uniform(0.5, 1.0, size=(3, nmodes))
    # A depends on (x, z) only: evaluate it on one plane, broadcast along y
    X = x[None, None, :]
    Z = z[:, None, None]
    Y = np.broadcast_to(y[None, :, None], (nz, ny, nx))
    f = (Y / delta) ** 2 * np.exp(-(Y / delta) ** 2)
    fy = (2.0 * Y / delta ** 2) * (1.0 - (Y / delta) ** 2) * np.exp(-(Y / delta) ** 2)
    A = [np.zeros((nz, 1, nx)) for _ in range(3)]
    dAx = [np.zeros((nz, 1, nx)) for _ in range(3)]
    dAz = [np.zeros((nz, 1, nx)) for _ in range(3)]
    for c in range(3):
        for m in range(nmodes):
            ax = 2 * math.pi * kx[c, m] / L[0]
            az = 2 * math.pi * kz[c, m] / L[2]
            arg = ax * X + az * Z + ph[c, m]
            A[c] += am[c, m] * np.sin(arg)
            dAx[c] += am[c, m] * ax * np.cos(arg)
            dAz[c] += am[c, m] * az * np.cos(arg)
    # curl(f A) with d/dy acting on f only (A independent of y)
    up = fy * A[2] - f * dAz[1]
    vp = f * dAz[0] - f * dAx[2]
    wp = f * dAx[1] - fy * A[0]
    scale = amp / max(1e-300, float(np.sqrt(up ** 2 + vp ** 2 + wp ** 2).max()))
    ub = np.tanh(3.0 * Y / delta)
    u = ub + scale * up
    v = scale * vp
    w = scale * wp
    T = Taw - (Taw - 1.0) * ub ** 2
    p = np.full_like(T, 1.0 / (g * M * M))
    rho = g * M * M * p / T
    U = _state(3, (nx, ny, nz), conserved(g, rho, [u, v, w], p))
    return Problem(name="wall%dx%dx%d" % (nx, ny, nz), ndim=3, n=(nx, ny, nz), gamma=g, Re=Re,
                   Pr=Pr, Minf=M, sutherland=1, Ts_over_Tref=110.4 / Tref, scheme=scheme,
                   bc=((PERIODIC, PERIODIC), (ISOTHERMAL, EXTRAPOLATE), (PERIODIC, PERIODIC)),
                   wall_T=((1.0, 1.0), (Taw, 1.0), (1.0, 1.0)), period=(L[0], 0.0, L[2]),
                   coords1d=(x, y, z), U0=U, cfl=cfl, nsteps=nsteps)


# -------------------------------------------- 2D shock / vortex fields (sensor)
def shock_vortex(nx=1024, ny=512, seed=42, nvort=6, Ms=1.2, t_end=0.4, cfl=0.5, scheme=TENO5):
    """Stationary Mach-Ms normal shock at x = 0.5 on [0,2]x[0,1] (y periodic,
    x extrapolation) crossed by seeded isentropic vortices: strength eps in
    [0.1, 0.5], radius R in [0.05, 0.2], centres x in [0.1, 0.4]."""
    g = 1.4
    h = 1.0 / ny
    x = (np.arange(nx) + 0.5) * h
    y = (np.arange(ny) + 0.5) * h
    X, Y, _ = _mesh((x, y, None), 2)
    # Rankine-Hugoniot jump of a normal shock (upstream rho = 1, a = 1)
    r2 = (g + 1) * Ms ** 2 / ((g - 1) * Ms ** 2 + 2)
    p2 = 1.0 + 2 * g / (g + 1) * (Ms ** 2 - 1)
    up = X < 0.5
    rho = np.where(up, 1.0, r2)
    p = np.where(up, 1.0, p2) / g
    u = np.where(up, Ms, Ms / r2)
    v = np.zeros_like(u)
    rng = np.random.default_rng(seed)
    alpha = 0.204
    a2 = np.ones_like(u)
    for _ in range(nvort):
        eps_v = rng.uniform(0.1, 0.5)
        R = rng.uniform(0.05, 0.2)
        xc = rng.uniform(0.1, 0.4)
        yc = rng.uniform(0.0, 1.0)
        for img in (-1.0, 0.0, 1.0):
            dx, dy = X - xc, Y - (yc + img)
            tau = np.sqrt(dx * dx + dy * dy) / R
            ee = np.exp(alpha * (1 - tau ** 2))
            # u_theta = eps tau e^{alpha(1-tau^2)} in the counter-clockwise sense
            u = u - eps_v * ee * dy / R
            v = v + eps_v * ee * dx / R
            a2 = a2 - (g - 1) * eps_v ** 2 * ee ** 2 / (4 * alpha)
    # isentropic deficit applied multiplicatively to the base state
    rho = rho * a2 ** (1.0 / (g - 1))
    p = p * a2 ** (g / (g - 1))
    U = _state(2, (nx, ny, 1), conserved(g, rho, [u, v], p))
    return Problem(name="shockvortex%dx%d_s%d" % (nx, ny, seed), ndim=2, n=(nx, ny, 1), gamma=g,
                   Re=0.0, scheme=scheme,
                   bc=((EXTRAPOLATE, EXTRAPOLATE), (PERIODIC, PERIODIC), (PERIODIC, PERIODIC)),
                   period=(2.0, 1.0, 0.0), coords1d=(x, y, None), U0=U, cfl=cfl, t_end=t_end,
                   nsteps=10 ** 9)


# --------------------------------------------- 2D four-quadrant Riemann problems
def riemann2d(N, rng_or_seed, t_end=0.25, cfl=0.5, scheme=TENO5):
    """Four-quadrant Riemann problem on [0,1]^2 split at (0.5, 0.5); quadrant
    states rho ~ U[0.1,2], p ~ U[0.1,10], u, v ~ U[-1,1]; extrapolation BCs."""
    rng = rng_or_seed if isinstance(rng_or_seed, np.random.Generator) else np.random.default_rng(rng_or_seed)
    g = 1.4
    st = [(rng.uniform(0.1, 2.0), rng.uniform(-1, 1), rng.uniform(-1, 1), rng.uniform(0.1, 10.0))
          for _ in range(4)]
    x = (np.arange(N) + 0.5) / N
    X, Y, _ = _mesh((x, x, None), 2)
    q = (X >= 0.5).astype(int) + 2 * (Y >= 0.5).astype(int)
    rho = np.choose(q, [s[0] for s in st])
    u = np.choose(q, [s[1] for s in st])
    v = np.choose(q, [s[2] for s in st])
    p = np.choose(q, [s[3] for s in st])
    U = _state(2, (N, N, 1), conserved(g, rho.astype(float), [u.astype(float), v.astype(float)], p.astype(float)))
    return Problem(name="riemann%d" % N, ndim=2, n=(N, N, 1), gamma=g, Re=0.0, scheme=scheme,
                   bc=((EXTRAPOLATE, EXTRAPOLATE), (EXTRAPOLATE, EXTRAPOLATE), (PERIODIC, PERIODIC)),
                   period=(1.0, 1.0, 0.0), coords1d=(x, x, None), U0=U, cfl=cfl, t_end=t_end,
                   nsteps=10 ** 9, meta={"states": st})


def riemann_batch(nprob=64, seed=2007, nmin=128, nmax=1024, step=64, scale=1.0):
    """The batched ensemble: nprob problems, N_p = nmin + step*k, k uniform."""
    rng = np.random.default_rng(seed)
    ks = rng.integers(0, (nmax - nmin) // step + 1, size=nprob)
    out = []
    for k in ks:
        N = int(round((nmin + step * int(k)) * scale))
        N = max(16, N)
        out.append(riemann2d(N, rng))
    return out


# ------------------------------------------ 2D laminar channel (wall-BC checks)
def laminar_channel(nx=32, ny=64, Re=90.0, Pr=0.72, M=0.01, scheme=TENO5):
    """Channel y in [-1, 1] (nodes on both walls), isothermal wall T = 1 at
    y = -1, adiabatic wall at y = 1, periodic x of length 2 pi, analytic
    profiles u = Re (1 - y^2)/2, T = 1 - Re^2 M^2 Pr (gamma-1)(y^4 - 4y - 5)/12,
    uniform pressure, driven by a unit body force."""
    g = 1.4
    Lx = 2 * math.pi
    x = Lx * np.arange(nx) / nx
    y = -1.0 + 2.0 * np.arange(ny) / (ny - 1)
    X, Y, _ = _mesh((x, y, None), 2)
    u = Re * (1 - Y ** 2) / 2
    T = 1 - Re ** 2 * M ** 2 * Pr * (g - 1) * (Y ** 4 - 4 * Y - 5) / 12
    p = np.full_like(T, 1.0 / (g * M * M))
    rho = g * M * M * p / T
    U = _state(2, (nx, ny, 1), conserved(g, rho, [u, 0 * u], p))
    return Problem(name="channel%dx%d" % (nx, ny), ndim=2, n=(nx, ny, 1), gamma=g, Re=Re, Pr=Pr,
                   Minf=M, scheme=scheme,
                   bc=((PERIODIC, PERIODIC), (ISOTHERMAL, ADIABATIC), (PERIODIC, PERIODIC)),
                   wall_T=((1.0, 1.0), (1.0, 1.0), (1.0, 1.0)), period=(Lx, 0.0, 0.0),
                   coords1d=(x, y, None), U0=U, body_force=1.0)


# ------------------------------------------------------- random smooth states
def smooth_random(ndim, n, seed=0, amp=0.05, mesh="uniform", scheme=TENO5, Re=0.0, M=0.5,
                  bc=None, nmodes=3):
    """Random low-mode perturbation of a uniform state on a periodic box
    [0,1)^ndim (used for conservation / symmetry / parity tests)."""
    rng = np.random.default_rng(seed)
    g = 1.4
    n = tuple(int(n[d]) if d < ndim else 1 for d in range(3))
    axes = [np.arange(n[d]) / n[d] if d < ndim else None for d in range(3)]
    X, Y, Z = _mesh(axes, ndim)
    comps = [X, Y, Z][:ndim]

    def field_(base):
        f = np.full(X.shape, base)
        for _ in range(nmodes):
            k = rng.integers(1, 3, size=ndim)
            ph = rng.uniform(0, 2 * math.pi)
            f = f + amp * rng.uniform(-1, 1) * np.sin(2 * math.pi * sum(k[d] * comps[d] for d in range(ndim)) + ph)
        return f

    rho = field_(1.0)
    vel = [field_(rng.uniform(-0.3, 0.3)) for _ in range(ndim)]
    p = field_(1.0)
    U = _state(ndim, n, conserved(g, rho, vel, p))
    if bc is None:
        bc = ((PERIODIC, PERIODIC),) * 3
    return Problem(name="smooth%dd" % ndim, ndim=ndim, n=n, gamma=g, Re=Re, Minf=M, scheme=scheme,
                   bc=bc, period=tuple(1.0 if d < ndim else 0.0 for d in range(3)),
                   coords1d=tuple(axes), U0=U)


def random_states(nc_dim, count, seed=0):
    """Random physical conserved states (count, ndim+2) for unit tests."""
    rng = np.random.default_rng(seed)
    g = 1.4
    rho = rng.uniform(0.2, 2.0, count)
    vel = [rng.uniform(-1.5, 1.5, count) for _ in range(nc_dim)]
    p = rng.uniform(0.2, 3.0, count)
    return np.stack(conserved(g, rho, vel, p), axis=1)
