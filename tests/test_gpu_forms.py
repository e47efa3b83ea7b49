"""The precision form (FP32 reconstruction and flux evaluation on FP64
deviations; FP64 state, RK accumulation, metrics, dt) checked against the FP64
oracle: density and energy errors are stated per case and bounded."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2007_14933_amd import inputs as I
from parity_util import flux_scale, gpu_run, oracle_run, say

pytestmark = pytest.mark.gpu

MIXED = 1


def rel_errors(prob, Ug, Uo):
    a, b = O.interior(prob, Ug), O.interior(prob, Uo)
    out = {}
    for name, c in (("rho", 0), ("rhoE", prob.nc - 1)):
        d = np.abs(a[c] - b[c])
        out[name + "_L1"] = d.mean() / np.abs(b[c]).mean()
        out[name + "_Linf"] = d.max() / np.abs(b[c]).max()
    return out


CASES = {
    # name: (problem, run kwargs, bounds on relative L1 of rho and of rhoE)
    "tgv32_viscous": (lambda: I.tgv(32), dict(nsteps=100), (1e-6, 1e-6)),
    "wall_24x20x16": (lambda: I.wall_flow(24, 20, 16, L=(10.0, 8.0, 6.0)), dict(nsteps=100), (1e-6, 1e-6)),
    "sod400_wenoz": (lambda: I.sod(400), dict(nsteps=10 ** 6, t_end=0.2), (1e-4, 1e-4)),
    "shockvortex_96x48": (lambda: I.shock_vortex(96, 48, seed=42), dict(nsteps=100), (1e-4, 1e-4)),
    # strong random four-quadrant jumps: FP32 cut-off decisions near shocks
    # differ from FP64 ones; measured rho 7.8e-5, rhoE 1.2e-4
    "riemann2d_70": (lambda: I.riemann2d(70, 5), dict(nsteps=100), (1e-4, 3e-4)),
}


@pytest.mark.parametrize("name", list(CASES))
def test_mixed_form_error_against_oracle(name):
    mk, kw, bound = CASES[name]
    prob = mk()
    say("[gpu mixed form]", name, prob.n, kw)
    Ug, tg, _ = gpu_run(prob, form=MIXED, **kw)
    Uo, to = oracle_run(prob, **kw)
    e = rel_errors(prob, Ug, Uo)
    say("   t=%.5g (oracle %.5g) " % (tg, to) + " ".join("%s=%.3e" % kv for kv in e.items()))
    assert abs(tg - to) <= 1e-4 * to  # CFL dt from the FP32-evaluated state
    assert e["rho_L1"] <= bound[0] and e["rhoE_L1"] <= bound[1], e


@pytest.mark.parametrize("name", ["tgv32_viscous", "shockvortex_96x48", "wall_24x20x16"])
def test_mixed_form_single_residual(name):
    """One residual evaluation: FP32 rounding of the deviations only, i.e.
    ~1e-6 of the flux scale (the FP64 path is at ~1e-15)."""
    from paper_2007_14933_amd.solver import Solver
    prob = CASES[name][0]()
    say("[gpu mixed residual]", name)
    s = Solver(prob, form=MIXED)
    s.apply_bc()
    Rg = s.residual().cpu().numpy()
    Uo = O.apply_bc(prob, prob.U0.copy())
    S, J = O.metrics(prob)
    Ro = O.residual(prob, S, J, Uo)
    err = np.abs(Rg - Ro).max(axis=(1, 2, 3)) / flux_scale(prob, Uo, J, S)
    say("   residual |diff| / flux scale:", err)
    assert err.max() <= 2e-6, err
