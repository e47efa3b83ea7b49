"""Pins of the learned-sensor oracle pieces: the cheap flux is the exact
all-stencils-kept limit of the characteristic flux; features are scale
invariant and bounded; the network's analytic gradient matches central finite
differences; BCE and Adam reduce to their closed forms in special cases."""
import numpy as np
import pytest

from oracle import mlp
from oracle import oracle as O
from paper_2007_14933_amd import inputs as I


def _prob(nd):
    return I.Problem(name="unit", ndim=nd, n=(8, 8, 8), gamma=1.4, Minf=1.0, scheme=I.TENO5)


def smooth_stencil(nd, rng, h=0.02):
    x = h * np.arange(6)
    ph = rng.uniform(0, 6.28, 8)
    rho = 1.0 + 0.1 * np.sin(x + ph[0])
    vel = [0.3 * rng.uniform(-1, 1) + 0.05 * np.cos(x + ph[1 + m]) for m in range(nd)]
    p = 1.0 + 0.1 * np.cos(x + ph[5])
    return np.stack(I.conserved(1.4, rho, vel, p), axis=1)


@pytest.mark.parametrize("nd", [1, 2, 3])
def test_cheap_flux_equals_full_flux_when_all_stencils_kept(nd):
    prob = _prob(nd)
    rng = np.random.default_rng(nd)
    for _ in range(20):
        U = smooth_stencil(nd, rng)
        S = rng.normal(size=nd) if nd > 1 else np.array([1.3])
        F, dl = O.iface_flux(prob, 0, U, S)
        assert dl.min() == 1
        Fc = O.cheap_flux(prob, 0, U, S)
        assert np.abs(F - Fc).max() <= 1e-14 * np.abs(F).max() * 10


def test_cheap_flux_differs_at_a_shock():
    prob = _prob(1)
    rho = np.array([1, 1, 1, 0.125, 0.125, 0.125])
    p = np.array([1, 1, 1, 0.1, 0.1, 0.1])
    U = np.stack(I.conserved(1.4, rho, [0 * rho], p), axis=1)
    F, dl = O.iface_flux(prob, 0, U, [1.0])
    assert dl.min() == 0
    assert np.abs(F - O.cheap_flux(prob, 0, U, [1.0])).max() > 1e-3


@pytest.mark.parametrize("nd", [1, 2, 3])
def test_features_bounded_and_scale_invariant(nd):
    prob = _prob(nd)
    rng = np.random.default_rng(10 + nd)
    for _ in range(20):
        U = I.random_states(nd, 6, seed=int(rng.integers(1 << 30)))
        S = rng.normal(size=nd) if nd > 1 else np.array([1.0])
        f, lab = O.features(prob, 0, U, S)
        assert abs(f[:4].sum() - 1.0) < 1e-12 and f.min() >= 0.0 and f[4:].max() < 1.0 + 1e-12
        # rescaling density (and energy) leaves every feature unchanged:
        # rho/rho_bar, p/p_bar, u/a_bar and the jumps are ratios
        f2, lab2 = O.features(prob, 0, 3.0 * U, S)
        assert np.abs(f2 - f).max() < 1e-12 and lab2 == lab


def test_features_of_uniform_and_step_states():
    prob = _prob(1)
    U = np.tile(I.conserved(1.4, 1.0, [0.3], 1.0), (6, 1)).astype(float)
    f, lab = O.features(prob, 0, U, [1.0])
    assert np.all(f == 0.0) and lab == 1
    rho = np.array([1, 1, 1, 0.125, 0.125, 0.125])
    U = np.stack(I.conserved(1.4, rho, [0 * rho], 0.1 + 0.9 * (rho > 0.5)), axis=1)
    f, lab = O.features(prob, 0, U, [1.0])
    assert lab == 0
    lj = lambda J: np.log10(1 + 1e6 * J) / 6
    assert abs(f[5] - lj(0.875 / 1.125)) < 1e-14 and abs(f[8] - lj(0.9 / 1.1)) < 1e-14
    assert f[4] == 0 and f[6] == 0


def _js_exact(q, m):
    from fractions import Fraction as Fr
    a1 = q[m] - 2 * q[m + 1] + q[m + 2]
    a2 = q[m] - q[m + 2]
    return Fr(13, 12) * a1 * a1 + Fr(1, 4) * a2 * a2


def test_indicator_features_of_one_varying_variable():
    """Only rho varies (u = 0, p uniform): the four indicator features are
    B_m(rho) / sum B(rho) whatever the normalisation, B the three-point
    Jiang-Shu indicator on substencils starting at i-2, i-1, i, i+1 (exact
    rational reference).  With p proportional to rho (p = 7 rho) the two
    variables' normalised indicators coincide, so the features are the same."""
    from fractions import Fraction as Fr
    prob = _prob(1)
    rho = [Fr(1), Fr(11, 10), Fr(13, 10), Fr(8, 5), Fr(17, 10), Fr(19, 10)]
    tot = sum(_js_exact(rho, m) for m in range(4))
    want = np.array([float(_js_exact(rho, m) / tot) for m in range(4)])
    r = np.array([float(v) for v in rho])
    for p in (np.full(6, 2.0), 7.0 * r):
        U = np.stack(I.conserved(1.4, r, [0 * r], p), axis=1)
        f, _ = O.features(prob, 0, U, [1.0])
        assert np.abs(f[:4] - want).max() < 1e-13, (f[:4], want)


@pytest.mark.parametrize("nd", [2, 3])
def test_features_invariant_under_velocity_pressure_scaling(nd):
    """u -> lam u, p -> lam^2 p (rho fixed) scales the sound speed by lam, so
    u_t / a_bar, p / p_bar and the jumps, hence all features, are unchanged;
    a tangential velocity scaled by anything but a_bar would break this."""
    prob = _prob(nd)
    rng = np.random.default_rng(7 + nd)
    x = 0.05 * np.arange(6)
    rho = 1.0 + 0.2 * np.sin(x + 0.3)
    vel = [0.4 * np.cos(3 * x + m) for m in range(nd)]
    p = 1.0 + 0.3 * np.cos(2 * x)
    S = np.eye(nd)[0]
    f0, _ = O.features(prob, 0, np.stack(I.conserved(1.4, rho, vel, p), axis=1), S)
    for lam in (0.1, 3.0):
        f1, _ = O.features(prob, 0, np.stack(I.conserved(1.4, rho, [lam * v for v in vel], lam * lam * p),
                                             axis=1), S)
        assert np.abs(f1 - f0).max() < 1e-12
    # the tangential velocity does enter: changing its profile moves the indicator features
    vel2 = [vel[0]] + [v + 0.3 * x * x for v in vel[1:]]
    f2, _ = O.features(prob, 0, np.stack(I.conserved(1.4, rho, vel2, p), axis=1), S)
    assert np.abs(f2[:4] - f0[:4]).max() > 1e-3
    del rng


def test_bf16_rounding():
    x = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -9, -2.5, 3.0e-3])
    r = mlp.bf16_round(x)
    assert r[0] == 1.0 and r[1] == 1.0          # tie to even
    assert r[2] == 1.0 + 2 ** -7
    assert r[3] == -2.5
    assert abs(r[4] - 3.0e-3) <= 3.0e-3 * 2 ** -8


def test_network_gradient_matches_finite_differences():
    rng = np.random.default_rng(3)
    theta = mlp.bf16_round(mlp.init(1) + 0.01 * rng.normal(size=mlp.NPARAM))
    X = rng.uniform(0, 1, (64, 10))
    y = (rng.uniform(size=64) > 0.4).astype(float)
    g = mlp.grad(theta, X, y)
    h = 1e-6
    idx = rng.choice(mlp.NPARAM, 80, replace=False)
    # finite differences on the function of the (already bf16-exact) weights:
    # perturb the FP64 master values directly, bypassing the bf16 rounding
    def loss_exact(th):
        saved = mlp.bf16_round
        mlp.bf16_round = lambda a: np.asarray(a, dtype=np.float64)
        try:
            return mlp.loss(th, X, y)
        finally:
            mlp.bf16_round = saved
    for i in idx:
        e = np.zeros(mlp.NPARAM)
        e[i] = h
        fd = (loss_exact(theta + e) - loss_exact(theta - e)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 * max(1.0, abs(g).max()), (i, fd, g[i])


def test_bias_only_network_closed_form():
    """All weights zero: z = b3, so loss and its b3-gradient are the weighted
    BCE of a constant prediction."""
    theta = np.zeros(mlp.NPARAM)
    theta[-1] = 0.5
    X = np.random.default_rng(0).uniform(size=(10, 10))
    y = np.array([1, 0, 1, 1, 0, 1, 1, 1, 0, 1], dtype=float)
    s = 1 / (1 + np.exp(-0.5))
    w = np.where(y > 0, 1.0, 10.0)
    ref = np.mean(w * -(y * np.log(s) + (1 - y) * np.log(1 - s)))
    assert abs(mlp.loss(theta, X, y) - ref) < 1e-14
    g = mlp.grad(theta, X, y)
    assert abs(g[-1] - np.mean(w * (s - y))) < 1e-15 and np.abs(g[:-1]).max() == 0.0


def test_adam_first_step_is_signed_lr():
    theta = np.zeros(5)
    g = np.array([0.3, -2.0, 1e-3, 0.0, 5.0])
    t1, m, v = mlp.adam(theta, np.zeros(5), np.zeros(5), g, 1, lr=0.01)
    # bias-corrected first step: -lr * g / (|g| + eps)
    assert np.allclose(t1, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=0)
