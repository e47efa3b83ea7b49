"""Pins of the oracle's pointwise operators against facts fixed by the paper and
by mathematics (never against a retyped copy of the oracle's own formulas):
polynomial exactness of the central operator and its closures, the linear
(upwind-5) limit of WENO-Z and TENO derived here from polynomial exactness,
TENO's cut-off on step data, symmetry, the eigenvectors against the flux
Jacobian, the Roe property, and reductions of the characteristic flux."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2007_14933_amd import inputs as I


# ------------------------------------------------------------ central D
@pytest.mark.parametrize("deg", [0, 1, 2, 3, 4])
def test_central_derivative_exact_for_quartics(deg):
    """Interior operator and the four one-sided closures are exact for
    polynomials of degree <= 4 (fourth order), at every node of a line."""
    N = 13
    x = np.arange(N, dtype=float) + 0.3
    rng = np.random.default_rng(deg)
    c = rng.uniform(-1, 1, deg + 1)
    f = np.polyval(c, x)
    df = np.polyval(np.polyder(c), x) if deg > 0 else np.zeros(N)
    d = O.deriv_line(f, periodic=False)
    scale = np.abs(f).max() + 1.0
    assert np.abs(d - df).max() <= 1e-12 * scale


def test_central_derivative_not_exact_for_quintic():
    """Degree 5 is not reproduced (the operators are fourth order, not more)."""
    N = 13
    x = np.arange(N, dtype=float)
    d = O.deriv_line(x ** 5, periodic=False)
    assert np.abs(d - 5 * x ** 4).max() > 1.0


def test_central_derivative_periodic_fourth_order():
    errs = []
    for N in (16, 32, 64):
        h = 2 * math.pi / N
        x = h * np.arange(N)
        d = O.deriv_line(np.sin(x), periodic=True) / h
        errs.append(np.abs(d - np.cos(x)).max())
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert min(orders) > 3.9, orders


def test_central_derivative_sign():
    """f = x gives +1: the interior sign follows the generated kernel, not the
    garbled displayed formula."""
    d = O.deriv_line(np.arange(20.0), periodic=False)
    assert np.allclose(d, 1.0, rtol=0, atol=1e-13)


# ------------------------------------------------------ reconstructions
def upwind5_weights():
    """Weights w on f_{i-2..i+2} of the fifth-order FD reconstruction: the value
    h(x_{i+1/2}) of any quartic h whose cell averages over [x_j-1/2, x_j+1/2]
    are the f_j.  Derived from exactness on monomials (independent of the
    scheme's ENO tables)."""
    xs = np.arange(-2, 3, dtype=float)
    A = np.zeros((5, 5))
    b = np.zeros(5)
    for p in range(5):
        for m, xj in enumerate(xs):
            A[p, m] = ((xj + 0.5) ** (p + 1) - (xj - 0.5) ** (p + 1)) / (p + 1)
        b[p] = 0.5 ** p
    return np.linalg.solve(A, b)


def test_smoothness_indicators_match_their_integral_definition():
    """beta_r = sum_{l=1,2} int_{cell i} dx^{2l-1} (q_r^{(l)})^2 for the quadratic
    q_r whose cell averages are the data on S_r = {i-r .. i-r+2} (the general
    Jiang-Shu definition, eq. smoothness_indicator), evaluated here by exact
    polynomial algebra, against the oracle's closed forms."""
    rng = np.random.default_rng(11)
    for _ in range(50):
        f = rng.normal(size=5)            # f_{i-2..i+2}, unit spacing, cell i = [-1/2, 1/2]
        beta = O.smoothness5(f)
        for r in range(3):
            centres = np.arange(-r, 3 - r, dtype=float)
            vals = f[2 - r: 5 - r]
            # quadratic c0 + c1 x + c2 x^2 with the given cell averages
            A = np.array([[1.0, xc, xc * xc + 1.0 / 12.0] for xc in centres])
            c = np.linalg.solve(A, vals)
            d1 = np.polynomial.Polynomial([c[1], 2 * c[2]])
            d2 = np.polynomial.Polynomial([2 * c[2]])
            ref = 0.0
            for dp in (d1, d2):
                ip = (dp * dp).integ()
                ref += ip(0.5) - ip(-0.5)
            assert abs(beta[r] - ref) <= 1e-12 * (1 + ref), (r, beta[r], ref)


def test_upwind5_weights_are_the_textbook_ones():
    w = upwind5_weights()
    assert np.allclose(w * 60, [2, -13, 47, 27, -3], atol=1e-12)


@pytest.mark.parametrize("scheme", [I.WENOZ5, I.TENO5])
def test_linear_limit_on_symmetric_integer_data(scheme):
    """Symmetric integer data give beta_0 == beta_2 exactly, so tau = 0 and both
    schemes reduce to the optimal weights: the upwind-5 reconstruction."""
    w = upwind5_weights()
    rng = np.random.default_rng(3)
    for _ in range(50):
        a, b, c = rng.integers(-9, 10, 3).astype(float)
        f = np.array([a, b, c, b, a])
        v, dl = O.recon5(scheme, 1e-5, 1e-16, f)
        assert abs(v - w @ f) <= 1e-13 * (1 + np.abs(f).max())
        assert list(dl) == [1, 1, 1]


def test_teno_keeps_all_stencils_on_smooth_data():
    w = upwind5_weights()
    h = 0.05
    for x0 in np.linspace(0, 1, 17):
        x = x0 + h * np.arange(-2, 3)
        f = np.exp(0.3 * x) + 0.2 * np.sin(x)
        v, dl = O.recon5(I.TENO5, 1e-5, 1e-16, f)
        assert list(dl) == [1, 1, 1]
        assert abs(v - w @ f) <= 1e-14 * np.abs(f).max()


def test_teno_cuts_discontinuous_stencils():
    """Jump between i+1 and i+2: the stencil {i..i+2} crosses it and is removed,
    the kept ones reproduce the constant 0 exactly.  Jump between i and i+1:
    only the upwind stencil {i-2..i} survives."""
    v, dl = O.recon5(I.TENO5, 1e-5, 1e-16, np.array([0.0, 0.0, 0.0, 0.0, 1.0]))
    assert v == 0.0 and list(dl) == [0, 1, 1]
    v, dl = O.recon5(I.TENO5, 1e-5, 1e-16, np.array([0.0, 0.0, 0.0, 1.0, 1.0]))
    assert v == 0.0 and list(dl) == [0, 0, 1]
    v, dl = O.recon5(I.TENO5, 1e-5, 1e-16, np.array([1.0, 1.0, 1.0, 1.0, 3.0]))
    assert v == 1.0


def test_wenoz_is_essentially_non_oscillatory_at_a_jump():
    v, _ = O.recon5(I.WENOZ5, 0, 1e-16, np.array([0.0, 0.0, 0.0, 1.0, 1.0]))
    assert 0.0 <= v < 1e-20
    v, _ = O.recon5(I.WENOZ5, 0, 1e-16, np.array([0.0, 0.0, 1.0, 1.0, 1.0]))
    assert abs(v - 1.0) < 1e-20


@pytest.mark.parametrize("scheme", [I.WENOZ5, I.TENO5])
def test_recon_odd_and_scale_and_shift(scheme):
    rng = np.random.default_rng(5)
    for _ in range(200):
        f = rng.normal(size=5)
        v, d1 = O.recon5(scheme, 1e-5, 1e-16, f)
        vm, d2 = O.recon5(scheme, 1e-5, 1e-16, -f)
        assert vm == -v and list(d1) == list(d2)
        v4, _ = O.recon5(scheme, 1e-5, 1e-16, 4.0 * f)
        assert abs(v4 - 4.0 * v) <= 1e-13 * np.abs(f).max() * 4
        vs, _ = O.recon5(scheme, 1e-5, 1e-16, f + 0.75)
        assert abs(vs - (v + 0.75)) <= 1e-12 * (1 + np.abs(f).max())


def test_wenoz_fifth_order_on_smooth_data():
    """Cell averages of sin(x): the reconstruction error at x_{i+1/2} falls at
    (at least) fifth order."""
    errs = []
    for h in (0.2, 0.1, 0.05):
        x = 0.37 + h * np.arange(-2, 3)
        f = (np.cos(x - h / 2) - np.cos(x + h / 2)) / h
        v, _ = O.recon5(I.WENOZ5, 0, 1e-16, f)
        errs.append(abs(v - math.sin(0.37 + h / 2)))
    assert math.log2(errs[0] / errs[1]) > 4.5 and math.log2(errs[1] / errs[2]) > 4.5


# ----------------------------------------------------------- eigensystem
def _prob(nd):
    return I.Problem(name="unit", ndim=nd, n=(8, 8, 8), gamma=1.4, Minf=1.0)


def _rand_unit(nd, rng):
    v = rng.normal(size=nd)
    return v / np.linalg.norm(v)


def jacobian_fd(prob, U, nv):
    nc = U.size
    A = np.zeros((nc, nc))
    for c in range(nc):
        h = 1e-4 * max(1.0, abs(U[c]))
        e = np.zeros(nc)
        e[c] = h

        def f(s):
            return O.phys_flux(prob, U + s * e, nv)
        # fourth-order central difference (exact for the cubic-or-lower
        # dependence up to round-off)
        A[:, c] = (-f(2) + 8 * f(1) - 8 * f(-1) + f(-2)) / (12 * h)
    return A


@pytest.mark.parametrize("nd", [1, 2, 3])
def test_eigenvectors_diagonalise_flux_jacobian(nd):
    prob = _prob(nd)
    rng = np.random.default_rng(nd)
    Us = I.random_states(nd, 20, seed=nd)
    for U in Us:
        nv = _rand_unit(nd, rng) if nd > 1 else np.array([1.0])
        for d in range(nd):
            L, R, lam = O.eigen(prob, d, U, U, nv)
            assert np.abs(L @ R - np.eye(nd + 2)).max() < 1e-13
            A = jacobian_fd(prob, U, nv)
            A2 = R @ np.diag(lam) @ L
            assert np.abs(A2 - A).max() <= 1e-8 * (1 + np.abs(A).max())


@pytest.mark.parametrize("nd", [1, 2, 3])
def test_roe_average_property(nd):
    """Roe's matrix satisfies f(U_R) - f(U_L) = A_roe (U_R - U_L) exactly."""
    prob = _prob(nd)
    rng = np.random.default_rng(10 + nd)
    Us = I.random_states(nd, 40, seed=10 + nd)
    for a in range(0, 40, 2):
        UL, UR = Us[a], Us[a + 1]
        nv = _rand_unit(nd, rng) if nd > 1 else np.array([1.0])
        L, R, lam = O.eigen(prob, 0, UL, UR, nv)
        lhs = O.phys_flux(prob, UR, nv) - O.phys_flux(prob, UL, nv)
        rhs = R @ (lam * (L @ (UR - UL)))
        assert np.abs(lhs - rhs).max() <= 1e-12 * (1 + np.abs(lhs).max())
    # the arithmetic-mean state does not have the property (sanity)
    p2 = prob.with_(roe_avg=0)
    UL, UR = Us[0], Us[1]
    nv = np.eye(nd)[0]
    L, R, lam = O.eigen(p2, 0, UL, UR, nv)
    lhs = O.phys_flux(p2, UR, nv) - O.phys_flux(p2, UL, nv)
    assert np.abs(lhs - R @ (lam * (L @ (UR - UL)))).max() > 1e-6


# ------------------------------------------------------ interface flux
@pytest.mark.parametrize("nd", [1, 2, 3])
@pytest.mark.parametrize("scheme", [I.WENOZ5, I.TENO5])
def test_iface_flux_uniform_state(nd, scheme):
    prob = _prob(nd).with_(scheme=scheme)
    rng = np.random.default_rng(20 + nd)
    for U in I.random_states(nd, 10, seed=20 + nd):
        S = rng.normal(size=nd) if nd > 1 else np.array([0.7])
        F, dl = O.iface_flux(prob, 0, np.tile(U, (6, 1)), S)
        Sm = np.linalg.norm(S)
        ref = Sm * O.phys_flux(prob, U, S / Sm)
        assert np.abs(F - ref).max() <= 2e-14 * (1 + np.abs(ref).max())
        assert dl.min() == 1


@pytest.mark.parametrize("u", [0.6, -0.6])
@pytest.mark.parametrize("scheme", [I.WENOZ5, I.TENO5])
def test_iface_flux_entropy_wave_is_scalar_upwind(u, scheme):
    """Uniform u and p, varying rho: only the entropy field varies, so the mass
    flux is u times the scalar reconstruction of rho from the upwind side
    (i-2..i+2 for u > 0, the mirror i+3..i-1 for u < 0)."""
    prob = _prob(1).with_(scheme=scheme)
    rng = np.random.default_rng(7)
    for _ in range(20):
        rho = rng.uniform(0.5, 1.5, 6)
        if rng.uniform() < 0.5:
            rho[3:] += 1.0  # a contact discontinuity in the stencil
        U = np.stack(I.conserved(1.4, rho, [u + 0 * rho], 1.0 + 0 * rho), axis=1)
        F, _ = O.iface_flux(prob, 0, U, [1.0])
        src = rho[:5] if u > 0 else rho[::-1][:5]
        r, _ = O.recon5(scheme, 1e-5, 1e-16, src)
        assert abs(F[0] - u * r) <= 1e-13 * (1 + abs(F[0]))
        assert abs(F[1] - (u * u * r + 1.0)) <= 1e-12 * (1 + abs(F[1]))


@pytest.mark.parametrize("scheme", [I.WENOZ5, I.TENO5])
def test_iface_flux_mirror_symmetry(scheme):
    """Reflecting the stencil (k -> 5-k) and the velocity maps F to (-F0, F1, -F2)."""
    prob = _prob(1).with_(scheme=scheme)
    rng = np.random.default_rng(8)
    for _ in range(30):
        U = I.random_states(1, 6, seed=int(rng.integers(1 << 30)))
        Ur = U[::-1].copy()
        Ur[:, 1] *= -1
        F, _ = O.iface_flux(prob, 0, U, [1.0])
        Fr, _ = O.iface_flux(prob, 0, Ur, [1.0])
        assert np.abs(Fr - np.array([-F[0], F[1], -F[2]])).max() <= 1e-13 * (1 + np.abs(F).max())


@pytest.mark.parametrize("scheme", [I.WENOZ5, I.TENO5])
def test_iface_flux_rotation_invariance_2d(scheme):
    """Rotating velocities and the area vector together rotates the momentum
    flux and leaves mass and energy fluxes unchanged (2D: the tangent is fixed
    up to sign, and the reconstruction is odd)."""
    prob = _prob(2).with_(scheme=scheme)
    rng = np.random.default_rng(9)
    for _ in range(30):
        U = I.random_states(2, 6, seed=int(rng.integers(1 << 30)))
        S = rng.normal(size=2)
        th = rng.uniform(0, 2 * math.pi)
        Q = np.array([[math.cos(th), -math.sin(th)], [math.sin(th), math.cos(th)]])
        Uq = U.copy()
        Uq[:, 1:3] = U[:, 1:3] @ Q.T
        F, _ = O.iface_flux(prob, 0, U, S)
        Fq, _ = O.iface_flux(prob, 0, Uq, Q @ S)
        ref = np.concatenate([[F[0]], Q @ F[1:3], [F[3]]])
        assert np.abs(Fq - ref).max() <= 1e-12 * (1 + np.abs(F).max())


def test_iface_flux_linear_limit_equals_central_plus_dissipation():
    """On smooth data (all TENO stencils kept) the flux equals the closed form
    |S| [C6 f + R diag(alpha) L D6 U] obtained by summing the split upwind-5
    reconstructions (C6, D6 derived here from the upwind-5 weights)."""
    w = upwind5_weights()
    cp = np.concatenate([w, [0.0]])           # on i-2..i+3
    cm = np.concatenate([[0.0], w[::-1]])     # mirror
    C6, D6 = 0.5 * (cp + cm), 0.5 * (cp - cm)
    prob = _prob(2).with_(scheme=I.TENO5)
    x = 0.02 * np.arange(6)
    rho = 1.0 + 0.1 * np.sin(x + 0.3)
    u = 0.4 + 0.05 * np.cos(x)
    v = -0.2 + 0.03 * np.sin(2 * x)
    p = 1.0 + 0.1 * np.cos(x + 1.0)
    U = np.stack(I.conserved(1.4, rho, [u, v], p), axis=1)
    S = np.array([0.8, 0.3])
    Sm = np.linalg.norm(S)
    nv = S / Sm
    F, dl = O.iface_flux(prob, 0, U, S)
    assert dl.min() == 1
    L, R, _ = O.eigen(prob, 0, U[2], U[3], nv)
    un = U[:, 1:3] @ nv / U[:, 0]
    a = np.sqrt(1.4 * p / rho)
    alpha = np.array([np.abs(un - a).max(), np.abs(un).max(), np.abs(un).max(), np.abs(un + a).max()])
    f = np.stack([O.phys_flux(prob, U[k], nv) for k in range(6)])
    ref = Sm * (C6 @ f + R @ (alpha * (L @ (D6 @ U))))
    assert np.abs(F - ref).max() <= 1e-13 * np.abs(ref).max()
