"""Pins of three readings of the oracle that the generic operator pins leave
open: TENO's exponent q = 6 and constant C = 1 (section 2.5, eq. TENO_weights
with the cut-off eq. cutoff_eqn), the arithmetic ("simple") half-node average
offered beside Roe's (section 2.2 algorithm, step 2a; the scheme listing of
section 3 selects Roe), and the log-normalised jump features of the learned
sensor.  Every expected value below is derived by hand in the docstrings from
the definitions, not by calling the oracle's formulas."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2007_14933_amd import inputs as I


# ------------------------------------------------------------ TENO q and C
def test_teno_exponent_keeps_stencil_that_q7_would_cut():
    """f = (0, 1, 2, 3, 7) on i-2..i+2.  Jiang-Shu indicators:
    beta_0 = 13/12 (2 - 6 + 7)^2 + 1/4 (6 - 12 + 7)^2 = 13/12 * 9 + 1/4 = 10,
    beta_1 = 13/12 * 0 + 1/4 * (1 - 3)^2 = 1,
    beta_2 = 13/12 * 0 + 1/4 * (0 - 4 + 6)^2 = 1,
    tau_5 = |beta_0 - beta_2| = 9.  With C = 1: 1 + tau/beta_0 = 1.9 and
    1 + tau/beta_{1,2} = 10, so chi_0 = 1 / (1 + 2 (10/1.9)^q).
    q = 6: (10/1.9)^6 = 21 107.3..., chi_0 = 2.369e-5 >= C_T = 1e-5: kept.
    q = 7: chi_0 = 4.50e-6 < C_T: cut.  (C = 0 instead of 1 would give
    chi_0 = 1/(1 + 2 * 10^6): cut.)
    All three kept: the optimal weights (3/10, 3/5, 1/10) on the candidates
    q0 = 2/3 + 5/2 - 7/6 = 2, q1 = -1/6 + 5/3 + 1 = 5/2, q2 = -7/6 + 11/3 = 5/2,
    value 0.3 * 2 + 0.7 * 2.5 = 2.35."""
    v, dl = O.recon5(I.TENO5, 1e-5, 1e-16, np.array([0.0, 1.0, 2.0, 3.0, 7.0]))
    assert list(dl) == [1, 1, 1]
    assert abs(v - 2.35) <= 4e-16 * 2.35


def test_teno_exponent_cuts_stencil_that_q5_would_keep():
    """f = (0, 1, 2, 3, 15/2).  beta_0 = 13/12 (7/2)^2 + 1/4 (3/2)^2 = 83/6,
    beta_1 = beta_2 = 1, tau_5 = 77/6.  1 + tau/beta_0 = 160/83 and
    1 + tau/beta_{1,2} = 83/6, ratio (83/6)/(160/83) = 6889/960 = 7.176...
    q = 6: chi_0 = 1/(1 + 2 * 7.176^6) = 3.66e-6 < 1e-5: stencil 0 cut.
    q = 5: chi_0 = 1/(1 + 2 * 7.176^5) = 2.63e-5: kept.
    With stencil 0 cut the weights are (0, 6/7, 1/7) on q1 = q2 = 5/2
    (the left four points are linear), so the value is 5/2 up to rounding."""
    v, dl = O.recon5(I.TENO5, 1e-5, 1e-16, np.array([0.0, 1.0, 2.0, 3.0, 7.5]))
    assert list(dl) == [0, 1, 1]
    assert abs(v - 2.5) <= 4e-16 * 2.5


def test_teno_cutoff_threshold_position():
    """The cut-off compares chi_r with C_T itself (not C_T times anything):
    the second pin's chi_0 = 3.66e-6 lies between C_T = 1e-6 (kept) and
    C_T = 1e-5 (cut)."""
    _, dl = O.recon5(I.TENO5, 1e-6, 1e-16, np.array([0.0, 1.0, 2.0, 3.0, 7.5]))
    assert list(dl) == [1, 1, 1]
    _, dl = O.recon5(I.TENO5, 1e-5, 1e-16, np.array([0.0, 1.0, 2.0, 3.0, 7.5]))
    assert list(dl) == [0, 1, 1]


# ---------------------------------------------------- simple (arithmetic) average
def _prob1d(roe):
    return I.sod(16).with_(roe_avg=roe)


def test_simple_average_eigensystem_closed_form():
    """Left state (rho, u, p) = (1, 1, 1), right (2, 0, 4/5), gamma = 7/5.
    rho E_L = 1/0.4 + 1/2 = 3, H_L = (3 + 1)/1 = 4;  rho E_R = 0.8/0.4 = 2,
    H_R = (2 + 0.8)/2 = 7/5.  Arithmetic mean: u = 1/2, H = 27/10,
    a^2 = (gamma - 1)(H - u^2/2) = 0.4 * (2.7 - 0.125) = 1.03.
    Eigenvalues u - a, u, u + a; right eigenvectors (columns)
    (1, u - a, H - u a), (1, u, u^2/2), (1, u + a, H + u a).
    (Roe's average would give u = 1/(1 + sqrt 2) = 0.414..., and H = H_L would
    give a^2 = 1.55: both fail.)"""
    prob = _prob1d(0)
    UL = np.array([1.0, 1.0, 3.0])
    UR = np.array([2.0, 0.0, 2.0])
    L, R, lam = O.eigen(prob, 0, UL, UR, [1.0])
    u, H, a = 0.5, 2.7, math.sqrt(1.03)
    assert np.allclose(lam, [u - a, u, u + a], rtol=0, atol=2e-15)
    want_R = np.array([[1.0, 1.0, 1.0], [u - a, u, u + a], [H - u * a, 0.5 * u * u, H + u * a]])
    assert np.allclose(R, want_R, rtol=0, atol=4e-15)
    assert np.allclose(L @ R, np.eye(3), rtol=0, atol=1e-14)


def test_roe_average_differs_from_simple():
    """Same two states, Roe weights sqrt(rho): u = 1/(1 + sqrt 2),
    H = (4 + sqrt 2 * 7/5)/(1 + sqrt 2); a^2 = 0.4 (H - u^2/2)."""
    prob = _prob1d(1)
    L, R, lam = O.eigen(prob, 0, np.array([1.0, 1.0, 3.0]), np.array([2.0, 0.0, 2.0]), [1.0])
    s2 = math.sqrt(2.0)
    u = 1.0 / (1.0 + s2)
    H = (4.0 + s2 * 1.4) / (1.0 + s2)
    a = math.sqrt(0.4 * (H - 0.5 * u * u))
    assert np.allclose(lam, [u - a, u, u + a], rtol=0, atol=4e-15)


def test_simple_average_flux_of_two_state_jump():
    """Characteristic flux at a 1D contact-free jump between the states above,
    each held over three nodes: i-2..i = left, i+1..i+3 = right.  Every split
    field is constant on its upwind side, so TENO keeps exactly the stencils on
    one side and the LLF flux reduces to the characteristic Rusanov flux of
    the two states with the averaged eigenvectors and alpha_j = max |lambda_j|
    over both states:  F = (f_L + f_R)/2 - R diag(alpha) L (U_R - U_L)/2.
    Reference: the closed-form eigenvectors of the first pin (L = R^-1 of that
    matrix), pointwise eigenvalues of the two states."""
    prob = _prob1d(0)
    UL = np.array([1.0, 1.0, 3.0])
    UR = np.array([2.0, 0.0, 2.0])
    Uk = np.stack([UL, UL, UL, UR, UR, UR])
    F, dl = O.iface_flux(prob, 0, Uk, [1.0])
    u, H, a = 0.5, 2.7, math.sqrt(1.03)
    Rm = np.array([[1.0, 1.0, 1.0], [u - a, u, u + a], [H - u * a, 0.5 * u * u, H + u * a]])
    Lm = np.linalg.inv(Rm)
    fL = np.array([1.0, 1.0 + 1.0, (3.0 + 1.0) * 1.0])
    fR = np.array([0.0, 0.8, 0.0])
    aL, aR = math.sqrt(1.4), math.sqrt(1.4 * 0.8 / 2.0)
    alpha = np.array([max(abs(1 - aL), abs(0 - aR)), max(1.0, 0.0), max(abs(1 + aL), abs(0 + aR))])
    want = 0.5 * (fL + fR) - Rm @ (alpha * (Lm @ (UR - UL))) / 2.0
    assert np.abs(F - want).max() <= 1e-13 * np.abs(want).max(), (F, want)


# ----------------------------------------------------------- jump features
def test_log_jump_features_at_decades():
    """Jump features are log10(1 + 1e6 J)/6 with J = |q_R - q_L|/(q_R + q_L)
    (the sensor-input reading).  A density ratio r gives J = (r - 1)/(r + 1);
    choosing r = (1 + J)/(1 - J) with J = (10^k - 1)/1e6 makes 1 + 1e6 J = 10^k,
    so the feature is exactly k/6 (k = 1, 2, 3, 5); pressure uniform gives 0."""
    prob = I.sod(16)
    for k in (1, 2, 3, 5):
        J = (10.0 ** k - 1.0) / 1e6
        r = (1.0 + J) / (1.0 - J)
        rho = np.array([1.0, 1.0, 1.0, r, r, r])
        p = np.full(6, 0.7)
        U = np.stack(I.conserved(1.4, rho, [0 * rho], p), axis=1)
        f, _ = O.features(prob, 0, U, [1.0])
        assert abs(f[5] - k / 6.0) <= 1e-12, (k, f[5])
        assert f[4] == 0.0 and f[6] == 0.0
        assert np.all(f[7:] == 0.0)
