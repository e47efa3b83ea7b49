"""Parity of the HIP fourth-order central path (section 2.6; the scheme of
the central Taylor-Green benchmark of section 6.1) with the FP64 oracle, in
both storage strategies: StoreSome (velocity gradients stored, everything
else recomputed in the residual kernel) and store-all (every derivative in
its own work array).  Bars as the other parity tests: max normwise relative
difference per conserved quantity <= 1e-11 after the run, single residuals
<= 1e-13 of the flux scale.  Every case prints its name before touching the
GPU."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2007_14933_amd import inputs as I
from parity_util import flux_scale, normwise_rel, oracle_run, say

pytestmark = pytest.mark.gpu

TOL_RUN = 1e-11
TOL_ONE = 1e-13
C4 = dict(scheme=I.CENTRAL4)


def cases():
    c = {}
    c["tgv32_central"] = (I.tgv(32, **C4), dict(nsteps=100))
    c["tgv40_central_rk4"] = (I.tgv(40, **C4).with_(rk=I.RK4), dict(nsteps=30))
    ch = I.laminar_channel(16, 33, scheme=I.CENTRAL4)
    c["channel_16x33_walls_central"] = (ch.with_(body_force=0.0), dict(nsteps=100))
    # one-sided closures of both operators in every direction; a central
    # scheme has no dissipation to damp what zero-gradient ends reflect, so
    # the run is kept short (Re 50, 12 steps) while the state stays smooth
    sm = I.smooth_random(3, (22, 9, 13), seed=5, amp=0.05, Re=50.0, M=0.5, scheme=I.CENTRAL4)
    c["smooth3d_22x9x13_extrapolated_central"] = (sm.with_(bc=((I.EXTRAPOLATE,) * 2,) * 3), dict(nsteps=12))
    s2 = I.smooth_random(2, (70, 36), seed=8, amp=0.1, Re=100.0, M=0.4, scheme=I.CENTRAL4).with_(sutherland=1)
    c["smooth2d_70x36_sutherland_central"] = (s2, dict(nsteps=60))
    c["dwave1d_64_central"] = (I.density_wave_1d(64, scheme=I.CENTRAL4), dict(nsteps=100))
    return c


CASES = cases()
STRATEGIES = ["storesome", "storeall"]


def gpu_run(prob, strategy, nsteps, cfl=0.5, dt_fixed=0.0, t_end=0.0):
    from paper_2007_14933_amd.solver import Solver
    s = Solver(prob)
    if strategy == "storeall":
        s.central_store_all(True)
    t = s.run(nsteps, cfl=cfl, dt_fixed=dt_fixed, t_end=t_end)
    s.check()
    return s.state(), t


@pytest.mark.parametrize("strategy", STRATEGIES)
@pytest.mark.parametrize("name", list(CASES))
def test_run_parity(name, strategy):
    prob, kw = CASES[name]
    say("[gpu central run]", name, strategy, prob.n, kw)
    Ug, tg = gpu_run(prob, strategy, **kw)
    Uo, to = oracle_run(prob, **kw)
    assert abs(tg - to) <= 1e-12 * max(1.0, abs(to)), (tg, to)
    err = normwise_rel(O.interior(prob, Ug), O.interior(prob, Uo))
    say("   t=%.6g  normwise rel diff per component:" % tg, err)
    assert np.all(np.isfinite(err)) and err.max() <= TOL_RUN, err


@pytest.mark.parametrize("strategy", STRATEGIES)
@pytest.mark.parametrize("name", list(CASES))
def test_residual_parity(name, strategy):
    prob, _ = CASES[name]
    say("[gpu central residual]", name, strategy, prob.n)
    from paper_2007_14933_amd.solver import Solver
    s = Solver(prob)
    if strategy == "storeall":
        s.central_store_all(True)
    s.apply_bc()
    Rg = s.residual().cpu().numpy()
    Uo = O.apply_bc(prob, prob.U0.copy())
    S, J = O.metrics(prob)
    Ro = O.residual(prob, S, J, Uo)
    err = np.abs(Rg - Ro).max(axis=(1, 2, 3)) / flux_scale(prob, Uo, J, S)
    say("   residual |diff| / flux scale:", err)
    assert err.max() <= TOL_ONE, err
    s.check()


def test_storage_strategies_switch_and_agree():
    from paper_2007_14933_amd.solver import Solver
    prob = I.tgv(24, **C4)
    say("[gpu central] strategy switch on one context")
    s = Solver(prob)
    s.apply_bc()
    a = s.residual().cpu().numpy()
    s.central_store_all(True)
    b = s.residual().cpu().numpy()
    s.central_store_all(False)
    c = s.residual().cpu().numpy()
    assert np.array_equal(a, c)
    scale = np.abs(a).max(axis=(1, 2, 3))
    assert (np.abs(a - b).max(axis=(1, 2, 3)) <= 1e-12 * np.maximum(scale, 1.0)).all()
