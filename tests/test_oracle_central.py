"""Pins of the oracle's fourth-order central path (section 2.6; the scheme of
the central TGV benchmark of section 6.1): the printed second-derivative
operator and its one-sided closures, central convection in conservative
form, and the viscous terms in expanded form.  Each pin is fixed by
mathematics independent of the oracle's code: polynomial exactness, the
continuous operator evaluated analytically, discrete conservation of mass
and momentum, the paper's analytic laminar channel as a steady state, and
convergence orders."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2007_14933_amd import inputs as I


def nonperiodic(nd):
    return tuple((I.EXTRAPOLATE, I.EXTRAPOLATE) if d < nd else (I.PERIODIC, I.PERIODIC) for d in range(3))


# ------------------------------------------------ second-derivative operator
@pytest.mark.parametrize("deg", [0, 1, 2, 3, 4])
def test_second_derivative_exact_for_quartics_with_closures(deg):
    """Interior stencil and the one-sided closures at nodes 0, 1, N-2, N-1 are
    exact for polynomials of degree <= 4 (five-point stencils)."""
    x = np.arange(11, dtype=float) - 3.7
    f = x ** deg
    ref = deg * (deg - 1) * x ** (deg - 2) if deg >= 2 else 0 * x
    out = O.deriv2_line(f, periodic=False)
    assert np.abs(out - ref).max() <= 1e-10 * (1 + np.abs(ref).max()), (deg, out - ref)


def test_second_derivative_closures_are_the_printed_ones():
    """Degree 5: the symmetric interior stencil is still exact, the one-sided
    closures are not, and their errors are those of the printed formulas
    (35, -104, 114, -56, 11)/12 and (11, -20, 6, 4, -1)/12 (an independent
    evaluation on x^5 at unit spacing from node 0)."""
    x = np.arange(10, dtype=float)
    f = x ** 5
    out = O.deriv2_line(f, periodic=False)
    exact = 20 * x ** 3
    assert np.abs(out[2:-2] - exact[2:-2]).max() <= 1e-9 * np.abs(exact).max()
    c0 = np.array([35, -104, 114, -56, 11]) / 12.0
    c1 = np.array([11, -20, 6, 4, -1]) / 12.0
    assert out[0] == pytest.approx(c0 @ f[:5], rel=1e-14, abs=1e-12) and out[0] != exact[0]
    assert out[1] == pytest.approx(c1 @ f[:5], rel=1e-14) and out[1] != pytest.approx(exact[1])
    # mirrored at the far end (a second derivative keeps its sign under x -> -x)
    assert out[-1] == pytest.approx(c0 @ f[::-1][:5], rel=1e-14)
    assert out[-2] == pytest.approx(c1 @ f[::-1][:5], rel=1e-14)


def test_second_derivative_periodic_fourth_order_and_constants():
    errs = []
    for N in (16, 32, 64):
        h = 2 * math.pi / N
        x = h * np.arange(N)
        out = O.deriv2_line(np.sin(x), periodic=True) / h ** 2
        errs.append(np.abs(out + np.sin(x)).max())
    assert math.log2(errs[0] / errs[1]) > 3.8 and math.log2(errs[1] / errs[2]) > 3.8, errs
    assert np.all(O.deriv2_line(np.full(9, 0.3), periodic=False) == 0.0)
    assert np.all(O.deriv2_line(np.full(9, 0.3), periodic=True) == 0.0)


# ---------------------------------------------------------- convection
def test_central_convection_converges_at_fourth_order():
    """1D density wave (u = 1, p = 1): the residual of the central path is
    -dF/dx of the exact state, reached at fourth order."""
    errs = []
    for N in (16, 32, 64):
        p = I.density_wave_1d(N, scheme=I.CENTRAL4)
        S, J = O.metrics(p)
        U = O.apply_bc(p, p.U0.copy())
        R = O.residual(p, S, J, U)
        x = p.coords1d[0]
        drho = 0.2 * math.pi * np.cos(math.pi * x)
        # rho' u, rho' u^2, (rho' u^2 / 2) u with u = 1, p = 1
        ref = [-drho, -drho, -0.5 * drho]
        errs.append(max(np.abs(R[c].ravel() - ref[c]).max() for c in range(3)))
    assert math.log2(errs[0] / errs[1]) > 3.8 and math.log2(errs[1] / errs[2]) > 3.8, errs


@pytest.mark.parametrize("viscous", [False, True])
def test_central_path_conserves_mass_and_momentum(viscous):
    """Periodic box: the conservative central convection telescopes, and so do
    the expanded viscous momentum terms (second differences and differences
    of differences), so sum R = 0 to round-off for mass and momentum; the
    expanded energy terms (products of derivatives) do not telescope."""
    p = I.smooth_random(3, (10, 9, 8), seed=4, amp=0.2, Re=(50.0 if viscous else 0.0), M=0.5,
                        scheme=I.CENTRAL4)
    S, J = O.metrics(p)
    U = O.apply_bc(p, p.U0.copy())
    R = O.residual(p, S, J, U)
    for c in range(4):
        scale = np.abs(R[c]).max() * R[c].size
        assert abs(R[c].sum()) <= 1e-13 * scale, (c, R[c].sum(), scale)
    if viscous:
        assert abs(R[4].sum()) > 1e-10 * np.abs(R[4]).max() * R[4].size


# ------------------------------------------------------------- viscous
def quad_field(rng, X, Y, Z):
    a = rng.uniform(-1, 1)
    b = rng.uniform(-1, 1, 3)
    Cm = rng.uniform(-1, 1, (3, 3))
    Cm = 0.5 * (Cm + Cm.T)
    xs = (X, Y, Z)
    val = a + sum(b[i] * xs[i] for i in range(3)) + sum(Cm[i, j] * xs[i] * xs[j] for i in range(3) for j in range(3))
    grad = [b[i] + 2 * sum(Cm[i, j] * xs[j] for j in range(3)) for i in range(3)]
    return val, grad, 2 * Cm


def test_expanded_viscous_terms_exact_on_quadratic_fields():
    """Quadratic u, v, w, T, constant mu, non-periodic anisotropic grid: the
    expanded viscous terms (the central residual minus its inviscid part)
    equal the continuous ones at every node, closures included."""
    n = (7, 8, 9)
    h = (0.1, 0.07, 0.13)
    axes = [h[d] * np.arange(n[d]) for d in range(3)]
    Z, Y, X = np.meshgrid(axes[2], axes[1], axes[0], indexing="ij")
    rng = np.random.default_rng(13)
    Re, Pr, M, g = 10.0, 0.7, 0.5, 1.4
    vel = [quad_field(rng, X, Y, Z) for _ in range(3)]
    Tq = quad_field(rng, X, Y, Z)
    T = 2.0 + 0.1 * Tq[0]
    Th = 0.1 * Tq[2]
    u = [0.3 * v[0] for v in vel]
    ug = [[0.3 * v[1][j] for j in range(3)] for v in vel]
    uh = [0.3 * v[2] for v in vel]
    pr = 1.0 + 0 * X
    rho = g * M * M * pr / T
    prob = I.Problem(name="vq", ndim=3, n=n, Re=Re, Pr=Pr, Minf=M, bc=nonperiodic(3), coords1d=tuple(axes),
                     scheme=I.CENTRAL4)
    U = np.zeros(O.ext_shape(prob))
    Ui = O.interior(prob, U)
    for c, a in enumerate(I.conserved(g, rho, u, pr)):
        Ui[c] = a
    S, J = O.metrics(prob)
    Rv = O.residual(prob, S, J, U) - O.residual(prob.with_(Re=0.0), S, J, U)
    div = sum(ug[i][i] for i in range(3))
    tau = [[(ug[i][j] + ug[j][i] - (2.0 / 3.0 * div if i == j else 0.0)) / Re for j in range(3)] for i in range(3)]
    dtau = [(np.trace(uh[i]) + sum(uh[j][i, j] for j in range(3)) / 3.0) / Re for i in range(3)]
    kc = 1.0 / ((g - 1) * M * M * Pr * Re)
    energy = sum(tau[i][j] * ug[i][j] for i in range(3) for j in range(3)) \
        + sum(u[i] * dtau[i] for i in range(3)) + kc * np.trace(Th)
    assert np.abs(Rv[0]).max() == 0.0
    for i in range(3):
        assert np.abs(Rv[1 + i] - dtau[i]).max() < 1e-10 * (1 + np.abs(dtau[i]).max())
    assert np.abs(Rv[4] - energy).max() < 1e-9 * (1 + np.abs(energy).max())


def test_expanded_form_steady_on_the_laminar_channel():
    """The paper's analytic channel (section 5.4; u quadratic, T quartic in
    y): with the unit body force the central path's residual vanishes at
    every node, walls included (the second-derivative closures act at the
    wall nodes and their neighbours)."""
    p = I.laminar_channel(8, 17, scheme=I.CENTRAL4)
    S, J = O.metrics(p)
    U = O.apply_bc(p, p.U0.copy())
    R = O.residual(p, S, J, U)
    u = O.interior(p, U)[1] / O.interior(p, U)[0]
    assert np.abs(R[0]).max() == 0.0
    assert np.abs(R[1]).max() < 1e-10 * np.abs(u).max() and np.abs(R[2]).max() < 1e-10
    assert np.abs(R[3]).max() < 1e-9 * np.abs(u).max() ** 2


def test_expanded_and_divergence_forms_agree_in_the_limit():
    """Smooth periodic state with Sutherland viscosity: the two discrete forms
    of the same continuous viscous terms differ by truncation error only,
    falling at fourth order."""
    diffs = []
    for N in (48, 96, 192):
        p = I.smooth_random(2, (N, N), seed=3, amp=0.3, Re=20.0, M=0.4).with_(sutherland=1)
        S, J = O.metrics(p)
        U = O.apply_bc(p, p.U0.copy())
        Rd = O.viscous_residual(p, S, J, U)
        pc = p.with_(scheme=I.CENTRAL4)
        Re_ = O.residual(pc, S, J, U) - O.residual(pc.with_(Re=0.0), S, J, U)
        diffs.append(max(np.abs(Re_[c] - Rd[c]).max() for c in range(1, 4)))
    o = [math.log2(diffs[i] / diffs[i + 1]) for i in range(2)]
    assert min(o) > 3.7, (o, diffs)


def test_central_tgv_runs_and_decays():
    """The central path on the viscous TGV (16^3, a few steps): kinetic energy
    falls, mass is conserved to round-off."""
    p = I.tgv(16, scheme=I.CENTRAL4)
    S, J = O.metrics(p)
    U = p.U0.copy()

    def ke(U):
        Ui = O.interior(p, U)
        return float((0.5 * (Ui[1] ** 2 + Ui[2] ** 2 + Ui[3] ** 2) / Ui[0]).sum())
    m0, k0 = float(O.interior(p, U)[0].sum()), ke(O.apply_bc(p, U.copy()))
    O.run(p, S, J, U, 10, cfl=0.5)
    assert abs(float(O.interior(p, U)[0].sum()) - m0) <= 1e-13 * m0
    assert ke(U) < k0
