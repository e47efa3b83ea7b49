"""The allocation-free substep against osbli_rk_substep: the same launches
with the scratch in the library's static device array instead of the
context workspace, so results must be identical bit for bit.  Two problems
in a row, the second smaller than the first (the array keeps the first
call's contents), and a grid beyond the array's size, which must be refused
before any launch."""
import ctypes as C

import numpy as np
import pytest

from paper_2007_14933_amd import binding as B
from paper_2007_14933_amd import inputs as I
from parity_util import say

pytestmark = pytest.mark.gpu


def _ptr(t):
    return C.c_void_p(t.data_ptr())


def _advance(s, noalloc, nsteps):
    lib = s.lib
    fn = lib.osbli_rk_substep_noalloc if noalloc else lib.osbli_rk_substep
    s.apply_bc()
    for _ in range(nsteps):
        dt = s.compute_dt(0.5)
        for st in range(3):
            B.check(fn(s.ctx, st, dt, _ptr(s.U), _ptr(s.dU), s._s()), s.ctx)
            s.apply_bc()
    s.check()
    return s.state(), s.dU.cpu().numpy()


@pytest.mark.parametrize("order", ["large_then_small"])
def test_noalloc_substep_matches_substep(order):
    from paper_2007_14933_amd.solver import Solver
    lib = B.load()
    assert lib.osbli_noalloc_scratch_bytes() == 64 << 20
    # viscous TGV 40^3 (17 doubles of scratch per node: 8.7 MB),
    # then a smaller inviscid 2D Riemann problem on the same scratch
    for prob, nsteps in ((I.tgv(40), 3), (I.riemann2d(70, 5), 5)):
        say("[gpu no-alloc]", prob.name, prob.n, "steps", nsteps)
        a = Solver(prob)
        b = Solver(prob)
        Ua, dUa = _advance(a, False, nsteps)
        Ub, dUb = _advance(b, True, nsteps)
        assert np.array_equal(Ua, Ub), np.abs(Ua - Ub).max()
        assert np.array_equal(dUa, dUb), np.abs(dUa - dUb).max()


def test_noalloc_substep_refuses_oversized_grid():
    from paper_2007_14933_amd.solver import Solver
    say("[gpu no-alloc] oversized grid refused")
    # viscous separable 3D at 90^3: 14 doubles per node (residual 5, viscous
    # fluxes 9) = 81.6 MB > 64 MiB
    s = Solver(I.tgv(90))
    rc = s.lib.osbli_rk_substep_noalloc(s.ctx, 0, 1e-4, _ptr(s.U), _ptr(s.dU), s._s())
    assert rc == B.OSBLI_ENOSPACE
    assert b"scratch" in s.lib.osbli_last_error(s.ctx)
