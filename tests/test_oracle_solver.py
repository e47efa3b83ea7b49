"""Pins of the oracle's metrics, boundary conditions, viscous terms, time
integration and whole-solver behaviour: exact metrics on polynomial meshes,
the discrete geometric conservation law, free-stream preservation, round-off
conservation, the RK3 stability polynomial, the exact Sod solution, the
density-wave convergence order, exactness of the viscous operator on the
analytic laminar channel and on quadratic fields, wall-ghost formulas, the
closed-form time step and axis-permutation symmetry."""
import math
import os

import numpy as np
import pytest

import exact_riemann as ER
from oracle import oracle as O
from paper_2007_14933_amd import inputs as I

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def read_golden(name):
    out = {}
    for line in open(os.path.join(GOLDEN, name)):
        line = line.strip()
        if line and not line.startswith("#"):
            k, v = line.split()
            out[k] = float(v)
    return out


def nonperiodic(nd):
    return tuple((I.EXTRAPOLATE, I.EXTRAPOLATE) if d < nd else (I.PERIODIC, I.PERIODIC) for d in range(3))


# ---------------------------------------------------------------- metrics
def test_metrics_exact_on_quadratic_mesh_2d():
    """On a quadratic mapping every D is exact, so S and J equal the analytic
    cofactors of dx/dxi."""
    nx, ny = 9, 11
    J_, I_ = np.meshgrid(np.arange(ny, dtype=float), np.arange(nx, dtype=float), indexing="ij")
    X = 0.1 * I_ + 0.02 * J_ + 0.003 * J_ ** 2
    Y = 0.15 * J_ - 0.01 * I_ + 0.002 * I_ * J_
    prob = I.Problem(name="m2", ndim=2, n=(nx, ny, 1), bc=nonperiodic(2),
                     coords_full=(X.reshape(1, ny, nx), Y.reshape(1, ny, nx), None))
    S, J = O.metrics(prob)
    xx, xy = 0.1 + 0 * I_, 0.02 + 0.006 * J_          # x_xi, x_eta
    yx, yy = -0.01 + 0.002 * J_, 0.15 + 0.002 * I_    # y_xi, y_eta
    Si = S[:, :, 0, 3:-3, 3:-3]
    assert np.allclose(Si[0, 0], yy, rtol=0, atol=1e-14)
    assert np.allclose(Si[0, 1], -xy, rtol=0, atol=1e-14)
    assert np.allclose(Si[1, 0], -yx, rtol=0, atol=1e-14)
    assert np.allclose(Si[1, 1], xx, rtol=0, atol=1e-14)
    assert np.allclose(J[0, 3:-3, 3:-3], 1.0 / (xx * yy - xy * yx), rtol=1e-13, atol=0)


def test_metrics_exact_on_quadratic_mesh_3d():
    n = (7, 8, 9)
    K, Jj, Ii = np.meshgrid(*(np.arange(n[d], dtype=float) for d in (2, 1, 0)), indexing="ij")
    X = 0.1 * Ii + 0.01 * Jj + 0.002 * K * Jj
    Y = 0.12 * Jj + 0.003 * Ii ** 2 - 0.01 * K
    Z = 0.09 * K + 0.004 * Ii * Jj + 0.002 * Jj ** 2
    prob = I.Problem(name="m3", ndim=3, n=n, bc=nonperiodic(3), coords_full=(X, Y, Z))
    S, J = O.metrics(prob)
    # analytic Jacobian columns x_xi, x_eta, x_zeta
    Xd = np.zeros((3, 3) + X.shape)  # Xd[p][b] = d x_p / d xi_b
    Xd[0, 0], Xd[0, 1], Xd[0, 2] = 0.1, 0.01 + 0.002 * K, 0.002 * Jj
    Xd[1, 0], Xd[1, 1], Xd[1, 2] = 0.006 * Ii, 0.12, -0.01
    Xd[2, 0], Xd[2, 1], Xd[2, 2] = 0.004 * Jj, 0.004 * Ii + 0.004 * Jj, 0.09
    cols = [Xd[:, b] for b in range(3)]
    det = np.einsum("i...,i...->...", cols[0], np.cross(cols[1], cols[2], axis=0))
    Si = S[:, :, 3:-3, 3:-3, 3:-3]
    for a in range(3):
        ref = np.cross(cols[(a + 1) % 3], cols[(a + 2) % 3], axis=0)
        assert np.abs(Si[a] - ref).max() < 1e-14, a
    assert np.allclose(J[3:-3, 3:-3, 3:-3], 1.0 / det, rtol=1e-13, atol=0)


def test_metrics_uniform_cartesian():
    p = I.tgv(8)
    S, J = O.metrics(p)
    h = 2 * math.pi / 8
    assert np.allclose(S[0, 0], h * h, rtol=1e-14) and np.abs(S[0, 1:]).max() == 0.0
    assert np.allclose(J, 1.0 / h ** 3, rtol=1e-14)


def wavy3d(n=10, A=0.03):
    L = 1.0
    K, Jj, Ii = np.meshgrid(*(np.arange(n, dtype=float) / n for _ in range(3)), indexing="ij")
    X = Ii + A * np.sin(2 * math.pi * Jj) * np.sin(2 * math.pi * K)
    Y = Jj + A * np.sin(2 * math.pi * K) * np.sin(4 * math.pi * Ii)
    Z = K + A * np.sin(2 * math.pi * Ii) * np.sin(2 * math.pi * Jj)
    return (X, Y, Z), (L, L, L)


def test_discrete_gcl_on_curved_meshes():
    """sum_d D_d S_d = 0 to round-off (the reading's metric identity)."""
    X, Y = I.sinusoidal_mesh(16, 16)
    p2 = I.Problem(name="g2", ndim=2, n=(16, 16, 1), period=(2.0, 2.0, 0.0), coords_full=(X, Y, None))
    (X3, Y3, Z3), per = wavy3d()
    p3 = I.Problem(name="g3", ndim=3, n=(10, 10, 10), period=per, coords_full=(X3, Y3, Z3))
    for p in (p2, p3):
        S, _ = O.metrics(p)
        nd = p.ndim
        core = tuple([slice(None)] + [slice(3, -3) if d < nd else slice(None) for d in (2, 1, 0)])
        for m in range(nd):
            tot = sum(O.deriv_field(p, np.ascontiguousarray(S[d, m][core[1:]]), d) for d in range(nd))
            assert np.abs(tot).max() < 1e-14 * (1 + np.abs(S[:nd, m]).max()) * 20


# ---------------------------------------------------- free stream, conservation
def uniform_on(p, rho=1.1, vel=(0.5, -0.3, 0.2), pr=0.9):
    comps = I.conserved(p.gamma, rho, list(vel[: p.ndim]), pr)
    U = np.zeros(O.ext_shape(p))
    Ui = O.interior(p, U)
    for c in range(p.nc):
        Ui[c] = comps[c]
    return U


@pytest.mark.parametrize("scheme", [I.WENOZ5, I.TENO5])
def test_free_stream_preservation_sinusoidal_2d(scheme):
    X, Y = I.sinusoidal_mesh(16, 16)
    p = I.Problem(name="fs2", ndim=2, n=(16, 16, 1), period=(2.0, 2.0, 0.0), scheme=scheme,
                  coords_full=(X, Y, None))
    S, J = O.metrics(p)
    U = uniform_on(p)
    U0 = O.interior(p, U).copy()
    O.run(p, S, J, U, 100, cfl=0.5)
    err = np.abs(O.interior(p, U) - U0).max(axis=(1, 2, 3)) / np.abs(U0).max(axis=(1, 2, 3))
    assert err.max() <= 1e-12, err


def test_free_stream_preservation_wavy_3d_viscous():
    (X, Y, Z), per = wavy3d(8)
    p = I.Problem(name="fs3", ndim=3, n=(8, 8, 8), period=per, scheme=I.TENO5, Re=100.0, Minf=0.5,
                  coords_full=(X, Y, Z))
    S, J = O.metrics(p)
    U = uniform_on(p)
    U0 = O.interior(p, U).copy()
    O.run(p, S, J, U, 30, cfl=0.5)
    err = np.abs(O.interior(p, U) - U0).max() / np.abs(U0).max()
    assert err <= 1e-12, err


def test_free_stream_stretched_wall_mesh():
    """Uniform flow with a periodic / extrapolation set-up on the tanh mesh."""
    p = I.wall_flow(8, 12, 6, nsteps=0)
    p = p.with_(bc=((I.PERIODIC, I.PERIODIC), (I.EXTRAPOLATE, I.EXTRAPOLATE), (I.PERIODIC, I.PERIODIC)))
    S, J = O.metrics(p)
    U = uniform_on(p)
    U0 = O.interior(p, U).copy()
    O.run(p, S, J, U, 20, cfl=0.5)
    assert np.abs(O.interior(p, U) - U0).max() / np.abs(U0).max() <= 1e-12


@pytest.mark.parametrize("viscous", [False, True])
def test_roundoff_conservation_periodic(viscous):
    """sum U/J is conserved to round-off on a periodic curvilinear mesh
    (telescoping flux differences and the divergence-form viscous terms)."""
    X, Y = I.sinusoidal_mesh(16, 16)
    base = I.smooth_random(2, (16, 16), seed=4, amp=0.2, Re=50.0 if viscous else 0.0)
    p = base.with_(period=(2.0, 2.0, 0.0), coords1d=None, coords_full=(X, Y, None), sutherland=int(viscous))
    S, J = O.metrics(p)
    U = p.U0.copy()
    Jin = O.interior(p, J[None])[0]

    def totals():
        Ui = O.interior(p, U)
        return (Ui / Jin).sum(axis=(1, 2, 3)), (np.abs(Ui) / Jin).sum(axis=(1, 2, 3))

    t0, s0 = totals()
    O.run(p, S, J, U, 40, cfl=0.4)
    t1, _ = totals()
    assert (np.abs(t1 - t0) / s0).max() <= 1e-13


# ------------------------------------------------------------- time stepping
def test_rk3_stability_polynomial():
    """One step of the three-stage scheme on u' = z u gives 1 + z + z^2/2 + z^3/6
    exactly (third order, three stages)."""
    p = I.Problem(name="rk", ndim=1, n=(5, 1, 1))
    for z in (-0.7, 0.3, -2.1):
        U = np.zeros(O.ext_shape(p))
        U[:, :, :, 3:-3] = 1.0
        dU = np.zeros(O.int_shape(p))
        for s in range(3):
            R = z * O.interior(p, U).copy()
            O.rk_update(p, s, 1.0, np.ascontiguousarray(R), U, dU)
        assert abs(O.interior(p, U)[0, 0, 0, 0] - (1 + z + z * z / 2 + z ** 3 / 6)) < 1e-15


def test_time_step_closed_form():
    p = I.tgv(8)
    S, J = O.metrics(p)
    U = uniform_on(p, rho=1.0, vel=(0.3, -0.2, 0.1), pr=1.0 / (1.4 * 0.01))
    h = 2 * math.pi / 8
    a = math.sqrt(1.4 * (1.0 / (1.4 * 0.01)) / 1.0)
    inviscid = sum(abs(v) + a for v in (0.3, -0.2, 0.1)) / h
    nu = max(4.0 / 3.0, 1.4 / 0.71) * 1.0 / (1.0 * 1600.0)
    ref = 0.5 / (inviscid + 2 * nu * 3 / h ** 2)
    assert abs(O.compute_dt(p, S, J, U, 0.5) - ref) <= 1e-14 * ref


# -------------------------------------------------------------------- Sod
def test_exact_riemann_solver_matches_toro():
    g = read_golden("sod_star_toro.txt")
    ps, us = ER.star_state(1, 0, 1, 0.125, 0, 0.1)
    assert abs(ps - g["p_star"]) < 6e-6 and abs(us - g["u_star"]) < 6e-6
    rho, _, _ = ER.sample(1, 0, 1, 0.125, 0, 0.1, np.array([us - 1e-9, us + 1e-9]))
    assert abs(rho[0] - g["rho_star_L"]) < 6e-6 and abs(rho[1] - g["rho_star_R"]) < 6e-6


def sod_l1(N, scheme=I.WENOZ5):
    p = I.sod(N, scheme=scheme)
    S, J = O.metrics(p)
    U = p.U0.copy()
    t = O.run(p, S, J, U, 10 ** 6, cfl=0.5, t_end=0.2)
    assert abs(t - 0.2) < 1e-14
    x = (np.arange(N) + 0.5) / N
    rho_ex, _, _ = ER.sample(1, 0, 1, 0.125, 0, 0.1, (x - 0.5) / 0.2)
    return np.abs(O.interior(p, U)[0].ravel() - rho_ex).mean()


@pytest.mark.parametrize("scheme", [I.WENOZ5, I.TENO5])
def test_sod_against_exact_solution(scheme):
    e = [sod_l1(N, scheme) for N in (200, 400, 800)]
    assert e[1] <= 5e-3, e
    assert math.log2(e[0] / e[1]) > 0.7 and math.log2(e[1] / e[2]) > 0.7, e


# ------------------------------------------------------------ density wave
@pytest.mark.parametrize("mesh", ["uniform", "sinusoidal"])
def test_density_wave_convergence_order(mesh):
    """WENO-Z5 on the smooth travelling density wave converges at (at least)
    0.9 x the formal fifth order in L1 and Linf on the paper's grids (32^2,
    64^2, 128^2), as the paper reports for curvilinear meshes.  Fixed dt small
    enough that the time error is negligible."""
    errs1, errsi = [], []
    for N in (32, 64, 128):
        p = I.density_wave(N, mesh=mesh)
        S, J = O.metrics(p)
        U = p.U0.copy()
        t_end = 0.1
        O.run(p, S, J, U, 10 ** 6, dt_fixed=1e-4, t_end=t_end)
        err = O.interior(p, U)[0] - I.exact_density_wave(p, t_end)
        errs1.append(np.abs(err).mean())
        errsi.append(np.abs(err).max())
    o1 = [math.log2(errs1[i] / errs1[i + 1]) for i in range(2)]
    oi = [math.log2(errsi[i] / errsi[i + 1]) for i in range(2)]
    assert o1[-1] >= 4.5 and oi[-1] >= 4.5, (o1, oi, errs1)


# ----------------------------------------------------------------- viscous
def test_viscous_operator_exact_on_laminar_channel():
    """Analytic channel profiles (paper section 5.4): viscous residual plus the
    unit body force vanish at every node including both walls, because the
    central operator and its closures are exact for these polynomials."""
    p = I.laminar_channel(8, 17)
    S, J = O.metrics(p)
    U = p.U0.copy()
    Rv = O.viscous_residual(p, S, J, U)
    Ui = O.interior(p, U)
    u = Ui[1] / Ui[0]
    mom = Rv[1] + 1.0
    en = Rv[3] + 1.0 * u
    assert np.abs(Rv[0]).max() == 0.0
    assert np.abs(mom).max() < 1e-10 and np.abs(Rv[2]).max() < 1e-10
    assert np.abs(en).max() < 1e-9 * np.abs(u).max()


def test_adiabatic_wall_temperature_formula():
    """The one-sided zero-gradient closure recovers T_aw = 1.155520 from the
    analytic profile (to the closure's truncation error)."""
    g = read_golden("laminar_channel.txt")
    p = I.laminar_channel(8, 64)
    U = p.U0.copy()
    O.apply_bc(p, U)
    Ui = O.interior(p, U)
    top = Ui[:, 0, -1, :]
    rho, rE = top[0], top[3]
    T = 1.4 * p.Minf ** 2 * (1.4 - 1.0) * rE / rho   # wall momentum is zero
    assert np.allclose(T, g["T_aw_analytic"], rtol=0, atol=5e-6)
    assert np.abs(top[1:3]).max() == 0.0


def quad_field(rng, X, Y, Z):
    a = rng.uniform(-1, 1)
    b = rng.uniform(-1, 1, 3)
    Cm = rng.uniform(-1, 1, (3, 3))
    Cm = 0.5 * (Cm + Cm.T)
    xs = (X, Y, Z)
    val = a + sum(b[i] * xs[i] for i in range(3)) + sum(Cm[i, j] * xs[i] * xs[j] for i in range(3) for j in range(3))
    grad = [b[i] + 2 * sum(Cm[i, j] * xs[j] for j in range(3)) for i in range(3)]
    hess = 2 * Cm
    return val, grad, hess


def test_viscous_operator_exact_on_quadratic_fields_3d():
    """Quadratic u, v, w, T with constant mu on a non-periodic anisotropic
    Cartesian grid: the discrete divergence-form viscous residual equals the
    continuous one exactly (all operands are polynomials of degree <= 3)."""
    n = (7, 8, 9)
    h = (0.1, 0.07, 0.13)
    axes = [h[d] * np.arange(n[d]) for d in range(3)]
    Z, Y, X = np.meshgrid(axes[2], axes[1], axes[0], indexing="ij")
    rng = np.random.default_rng(12)
    Re, Pr, M, g = 10.0, 0.7, 0.5, 1.4
    vel = [quad_field(rng, X, Y, Z) for _ in range(3)]
    Tq = quad_field(rng, X, Y, Z)
    T = 2.0 + 0.1 * Tq[0]
    Tg = [0.1 * t for t in Tq[1]]
    Th = 0.1 * Tq[2]
    u = [0.3 * v[0] for v in vel]
    ug = [[0.3 * v[1][j] for j in range(3)] for v in vel]
    uh = [0.3 * v[2] for v in vel]
    pr = 1.0 + 0 * X
    rho = g * M * M * pr / T
    prob = I.Problem(name="vq", ndim=3, n=n, Re=Re, Pr=Pr, Minf=M, bc=nonperiodic(3), coords1d=tuple(axes))
    U = np.zeros(O.ext_shape(prob))
    Ui = O.interior(prob, U)
    for c, a in enumerate(I.conserved(g, rho, u, pr)):
        Ui[c] = a
    S, J = O.metrics(prob)
    Rv = O.viscous_residual(prob, S, J, U)
    div = sum(ug[i][i] for i in range(3))
    tau = [[(ug[i][j] + ug[j][i] - (2.0 / 3.0 * div if i == j else 0.0)) / Re for j in range(3)] for i in range(3)]
    # d tau_ij / dx_j = (lap u_i + (1/3) d_i div u) / Re for constant mu
    lap = [np.trace(uh[i]) for i in range(3)]
    ddiv = [sum(uh[j][i, j] for j in range(3)) for i in range(3)]
    dtau = [(lap[i] + ddiv[i] / 3.0) / Re for i in range(3)]
    kc = 1.0 / ((g - 1) * M * M * Pr * Re)
    energy = sum(tau[i][j] * ug[i][j] for i in range(3) for j in range(3)) \
        + sum(u[i] * dtau[i] for i in range(3)) + kc * np.trace(Th)
    for i in range(3):
        assert np.abs(Rv[1 + i] - dtau[i]).max() < 1e-10 * (1 + np.abs(dtau[i]).max())
    assert np.abs(Rv[4] - energy).max() < 1e-9 * (1 + np.abs(energy).max())


def test_sutherland_law():
    p = I.Problem(name="s", ndim=1, n=(5, 1, 1), sutherland=1, Ts_over_Tref=110.4 / 202.17)
    assert abs(O.viscosity(p, 1.0) - 1.0) < 1e-15
    T, Ts = 1.7, 110.4 / 202.17
    assert abs(O.viscosity(p, T) - T ** 1.5 * (1 + Ts) / (T + Ts)) < 1e-15


# -------------------------------------------------------------------- BCs
def test_isothermal_wall_ghosts_linear_temperature():
    """A state whose temperature is linear in y through the wall value gives
    ghost temperatures on the same line; ghost momentum mirrors node i with
    the opposite sign; pressure in the ghosts equals the wall pressure."""
    nx, ny = 6, 10
    g, M = 1.4, 0.5
    y = 0.1 * np.arange(ny)
    x = 0.1 * np.arange(nx)
    Tw = 1.3
    p = I.Problem(name="w", ndim=2, n=(nx, ny, 1), Minf=M, Re=10.0,
                  bc=((I.PERIODIC, I.PERIODIC), (I.ISOTHERMAL, I.EXTRAPOLATE), (I.PERIODIC, I.PERIODIC)),
                  wall_T=((1, 1), (Tw, 1), (1, 1)), period=(0.6, 0, 0), coords1d=(x, y, None))
    Yg, Xg = np.meshgrid(y, x, indexing="ij")
    T = Tw + 0.4 * Yg
    pr = 1.0 / (g * M * M) + 0.0 * Yg
    rho = g * M * M * pr / T
    uvel, vvel = 0.3 + Yg, 0.1 * Xg
    U = np.zeros(O.ext_shape(p))
    Ui = O.interior(p, U)
    for c, a in enumerate(I.conserved(g, rho, [uvel, vvel], pr)):
        Ui[c] = a.reshape(1, ny, nx)
    O.apply_bc(p, U)
    Ui = O.interior(p, U)
    assert np.abs(Ui[1:3, 0, 0, :]).max() == 0.0
    rw = Ui[0, 0, 0, :]
    assert np.allclose(Ui[3, 0, 0, :], rw * Tw / (M * M * g * (g - 1)), rtol=1e-15)
    pw = rw * Tw / (g * M * M)
    for m in (1, 2, 3):
        gh = U[:, 0, 3 - m, 3:-3]
        src = U[:, 0, 3 + m, 3:-3]
        T1 = g * M * M * (g - 1) * (U[3, 0, 4, 3:-3] - 0.5 * (U[1, 0, 4, 3:-3] ** 2 + U[2, 0, 4, 3:-3] ** 2) / U[0, 0, 4, 3:-3]) / U[0, 0, 4, 3:-3]
        Tg_expect = (m + 1) * Tw - m * T1
        pg = (g - 1) * (gh[3] - 0.5 * (gh[1] ** 2 + gh[2] ** 2) / gh[0])
        Tg = g * M * M * pg / gh[0]
        assert np.allclose(Tg, Tg_expect, rtol=1e-12)
        assert np.allclose(pg, pw, rtol=1e-12)
        assert np.allclose(gh[1] / gh[0], -src[1] / src[0], rtol=1e-13)
        assert np.allclose(gh[2] / gh[0], -src[2] / src[0], rtol=1e-13)
    # extrapolation side: copies of the last node; periodic x: wrap copies
    assert np.array_equal(U[:, 0, -1, 3:-3], U[:, 0, -4, 3:-3])
    assert np.array_equal(U[:, 0, 3:-3, 0], U[:, 0, 3:-3, -6])
    assert np.array_equal(U[:, 0, 3:-3, -1], U[:, 0, 3:-3, 5])


def test_adiabatic_wall_temperature_exact_for_quartic():
    """T quartic with zero slope at the wall: the one-sided closure gives T_w
    exactly."""
    nx, ny = 5, 9
    g, M = 1.4, 0.3
    y = np.arange(ny, dtype=float)
    x = np.arange(nx, dtype=float)
    p = I.Problem(name="a", ndim=2, n=(nx, ny, 1), Minf=M, Re=10.0,
                  bc=((I.PERIODIC, I.PERIODIC), (I.ADIABATIC, I.ADIABATIC), (I.PERIODIC, I.PERIODIC)),
                  period=(5.0, 0, 0), coords1d=(x, y, None))
    Yg, _ = np.meshgrid(y, x, indexing="ij")
    T = 1.0 + 0.01 * Yg ** 2 - 0.002 * Yg ** 3 + 0.0001 * Yg ** 4
    pr = 1.0 + 0 * Yg
    rho = g * M * M * pr / T
    U = np.zeros(O.ext_shape(p))
    Ui = O.interior(p, U)
    for c, a in enumerate(I.conserved(g, rho, [0.2 + 0 * Yg, 0 * Yg], pr)):
        Ui[c] = a.reshape(1, ny, nx)
    O.apply_bc(p, U)
    Ui = O.interior(p, U)
    Tw = g * M * M * (g - 1) * Ui[3, 0, 0, :] / Ui[0, 0, 0, :]
    assert np.allclose(Tw, 1.0, rtol=0, atol=1e-13)


# ------------------------------------------------------------- symmetry
def test_axis_permutation_3d():
    """Cycling the axes (x->y->z) of a viscous periodic problem cycles the
    residual (to round-off)."""
    base = I.smooth_random(3, (6, 7, 8), seed=3, amp=0.2, Re=20.0)
    S, J = O.metrics(base)
    U = O.apply_bc(base, base.U0.copy())
    R = O.residual(base, S, J, U)
    # new axes: x' = z, y' = x, z' = y  -> array order (k', j', i') = (y, x, z)
    Up = np.transpose(U, (0, 2, 3, 1)).copy()
    Up = Up[[0, 3, 1, 2, 4]].copy()
    pp = base.with_(n=(8, 6, 7), coords1d=(base.coords1d[2], base.coords1d[0], base.coords1d[1]), U0=Up)
    Sp, Jp = O.metrics(pp)
    Rp = O.residual(pp, Sp, Jp, Up)
    Rref = np.transpose(R, (0, 2, 3, 1))[[0, 3, 1, 2, 4]]
    assert np.abs(Rp - Rref).max() <= 1e-12 * np.abs(R).max()
