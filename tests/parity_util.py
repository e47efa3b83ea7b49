"""Helpers shared by the GPU parity tests: run a problem through the HIP
library and through the oracle on the same seeded input and compare."""
import sys

import numpy as np

from oracle import oracle as O


def normwise_rel(a, b):
    """Parity measure per conserved quantity: max|a_c - b_c| / max|b_q| where q
    is the quantity c belongs to -- density, the momentum vector (all its
    components share one scale, so a component that is zero in the flow,
    e.g. a wall-normal velocity, is measured against the momentum), energy."""
    nc = a.shape[0]
    mom = np.abs(b[1:nc - 1]).max()
    out = np.zeros(nc)
    for c in range(nc):
        den = mom if 0 < c < nc - 1 else np.abs(b[c]).max()
        out[c] = np.abs(a[c] - b[c]).max() / (den if den > 0 else 1.0)
    return out


def flux_scale(prob, U, J, S):
    """Scale of a residual component: max J|S_d| times the largest local
    Lax-Friedrichs flux of that conserved quantity, (|u| + a)|U_c| (+ p for
    momentum, + p|u| for energy).  Flux differences cancel (strongly at low
    Mach number), so rounding of a residual is relative to this scale."""
    from oracle import oracle as O
    nd = prob.ndim
    Ui = O.interior(prob, U)
    rho = Ui[0]
    vel = [Ui[1 + m] / rho for m in range(nd)]
    umag = np.sqrt(sum(v * v for v in vel))
    p = (prob.gamma - 1.0) * (Ui[nd + 1] - 0.5 * rho * umag ** 2)
    lam = umag + np.sqrt(prob.gamma * np.abs(p) / rho)
    js = 0.0
    Ji = O.interior(prob, J[None])[0]
    for d in range(nd):
        smag = np.sqrt(sum(O.interior(prob, S[d, m][None])[0] ** 2 for m in range(nd)))
        js = max(js, float((Ji * smag).max()))
    mmag = np.sqrt(sum(Ui[1 + m] ** 2 for m in range(nd)))
    fl = np.zeros(nd + 2)
    fl[0] = (lam * np.abs(rho)).max()
    fl[1:nd + 1] = (lam * mmag + np.abs(p)).max()
    fl[nd + 1] = (lam * (np.abs(Ui[nd + 1]) + np.abs(p))).max()
    return js * fl


def say(*args):
    print(*args, flush=True)
    sys.stdout.flush()


def oracle_run(prob, nsteps, cfl=0.5, dt_fixed=0.0, t_end=0.0):
    S, J = O.metrics(prob)
    U = prob.U0.copy()
    t = O.run(prob, S, J, U, nsteps, cfl=cfl, dt_fixed=dt_fixed, t_end=t_end)
    return U, t


def gpu_run(prob, nsteps, cfl=0.5, dt_fixed=0.0, t_end=0.0, **kw):
    from paper_2007_14933_amd.solver import Solver
    s = Solver(prob, **kw)
    t = s.run(nsteps, cfl=cfl, dt_fixed=dt_fixed, t_end=t_end)
    s.check()
    return s.state(), t, s
