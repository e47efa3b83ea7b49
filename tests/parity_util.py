"""Helpers shared by the GPU parity tests: run a problem through the HIP
library and through the oracle on the same seeded input and compare."""
import sys

import numpy as np

from oracle import oracle as O


def normwise_rel(a, b):
    """Per component max|a - b| / max|b| (the parity measure)."""
    nc = a.shape[0]
    out = np.zeros(nc)
    for c in range(nc):
        den = np.abs(b[c]).max()
        out[c] = np.abs(a[c] - b[c]).max() / (den if den > 0 else 1.0)
    return out


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
