"""Driver of the HIP library: device buffers owned by PyTorch, calls through
the C ABI.  PyTorch supplies memory and streams only; every step of the
residual and the update runs in libosbli's kernels.

    s = Solver(problem)            # allocates U, dU, workspace on cuda:0
    s.run(nsteps, cfl=0.5)         # BCs at t=0, then dt + the RK substeps per step
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import binding as B
from .inputs import NGHOST


def _ptr(t: torch.Tensor):
    return C.c_void_p(t.data_ptr())


class Solver:
    def __init__(self, prob, device="cuda:0", form=B.FORM_FP64, sensor=0, stream=None):
        if not torch.cuda.is_available():
            raise RuntimeError("the HIP library needs a GPU (torch.cuda is not available)")
        self.lib = B.load()
        self.prob = prob
        self.device = torch.device(device)
        self.params = B.make_params(prob, form=form, sensor=sensor)
        nbytes = self.lib.osbli_workspace_bytes(C.byref(self.params))
        if nbytes == 0:
            raise B.OsbliError(B.OSBLI_EINVAL, "invalid parameters for %s" % prob.name)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        off = (-self.ws.data_ptr()) % 256
        self.ws_ptr = self.ws.data_ptr() + off
        self.ws_bytes = nbytes
        coords = self._coords()
        self.ctx = C.c_void_p()
        rc = self.lib.osbli_init_grid(C.byref(self.ctx), C.byref(self.params), *coords,
                                      C.c_void_p(self.ws_ptr), C.c_size_t(self.ws_bytes), self._s())
        if rc != 0:
            msg = self.lib.osbli_last_error(self.ctx).decode() if self.ctx else ""
            raise B.OsbliError(rc, msg)
        self.U = torch.from_numpy(np.ascontiguousarray(prob.U0)).to(self.device)
        nd = prob.ndim
        ishape = (nd + 2,) + tuple(prob.n[d] if d < nd else 1 for d in (2, 1, 0))
        self.dU = torch.zeros(ishape, dtype=torch.float64, device=self.device)
        self.t = 0.0
        self.nsteps_done = 0
        self.nstages = self.lib.osbli_rk_stages(self.ctx)

    def _s(self):
        return C.c_void_p(self.stream.cuda_stream)

    def _coords(self):
        p = self.prob
        self._coord_keep = []
        out = []
        for d in range(3):
            if d >= p.ndim:
                out.append(None)
                continue
            if p.coords1d is not None:
                a = np.ascontiguousarray(p.coords1d[d], dtype=np.float64)
            else:
                a = np.ascontiguousarray(p.coords_full[d], dtype=np.float64).ravel()
            self._coord_keep.append(a)
            out.append(a.ctypes.data_as(C.POINTER(C.c_double)))
        return out

    def __del__(self):
        try:
            if getattr(self, "ctx", None):
                self.lib.osbli_destroy(self.ctx)
                self.ctx = None
        except Exception:
            pass

    # ---- thin wrappers of the ABI ----
    def apply_bc(self, U=None):
        U = self.U if U is None else U
        B.check(self.lib.osbli_apply_bc(self.ctx, _ptr(U), self._s()), self.ctx)

    def residual(self, U=None, R=None):
        U = self.U if U is None else U
        if R is None:
            R = torch.empty_like(self.dU)
        B.check(self.lib.osbli_residual(self.ctx, _ptr(U), _ptr(R), self._s()), self.ctx)
        return R

    def substep(self, stage, dt):
        B.check(self.lib.osbli_rk_substep(self.ctx, int(stage), float(dt), _ptr(self.U), _ptr(self.dU), self._s()),
                self.ctx)

    def compute_dt(self, cfl):
        out = C.c_double(0.0)
        B.check(self.lib.osbli_compute_dt(self.ctx, _ptr(self.U), float(cfl), C.byref(out), self._s()), self.ctx)
        return out.value

    def set_sweep_segments(self, seg):
        """Nodes per wave segment of each direction's sweep (0: default)."""
        a = (C.c_int64 * 3)(*[int(v) for v in list(seg) + [0] * (3 - len(seg))])
        B.check(self.lib.osbli_set_sweep_segments(self.ctx, a), self.ctx)

    def profile(self, enable=True):
        B.check(self.lib.osbli_profile_enable(self.ctx, int(enable)), self.ctx)

    def profile_read(self):
        """{kernel class: (launch groups, total ms)} since profiling was enabled."""
        out = {}
        for k, name in enumerate(B.K_NAMES):
            cnt, ms = C.c_int64(0), C.c_double(0.0)
            B.check(self.lib.osbli_profile_read(self.ctx, k, C.byref(cnt), C.byref(ms)), self.ctx)
            out[name] = (cnt.value, ms.value)
        return out

    def check(self):
        B.check(self.lib.osbli_check(self.ctx), self.ctx)

    # ---- learned-sensor routing (params.sensor = 1) ----
    def set_sensor(self, bits, threshold, dilate=1, every_substage=0):
        """bits: 1441 bfloat16 weight patterns (uint16, host)."""
        w = np.ascontiguousarray(np.asarray(bits, dtype=np.uint16))
        if w.size != 1441:
            raise ValueError("expected 1441 weights")
        self._sensor_bits = w
        B.check(self.lib.osbli_sensor_set_weights(self.ctx, w.ctypes.data_as(C.c_void_p), 1441, float(threshold),
                                                  int(dilate), int(every_substage), self._s()), self.ctx)

    def sensor_update(self):
        B.check(self.lib.osbli_sensor_update(self.ctx, _ptr(self.U), self._s()), self.ctx)

    def sensor_stats(self):
        sm, tot = C.c_int64(0), C.c_int64(0)
        B.check(self.lib.osbli_sensor_stats(self.ctx, C.byref(sm), C.byref(tot)), self.ctx)
        return sm.value, tot.value

    def sensor_masks(self, d):
        """Direction d's routing mask of the last refresh (numpy uint8, x-fastest
        over the interface grid, extent n_d + 1 along d)."""
        n = [self.prob.n[e] if e < self.prob.ndim else 1 for e in range(3)]
        n[d] += 1
        out = torch.empty(n[0] * n[1] * n[2], dtype=torch.uint8, device=self.device)
        B.check(self.lib.osbli_sensor_masks(self.ctx, int(d), _ptr(out), out.numel(), self._s()), self.ctx)
        torch.cuda.synchronize(self.device)
        return out.cpu().numpy()

    def central_store_all(self, enable=True):
        """Central path: switch to the store-all strategy (every derivative in
        its own work array, allocated here) or back to StoreSome."""
        if not enable:
            B.check(self.lib.osbli_central_store_all(self.ctx, None, 0), self.ctx)
            self._cwork = None
            return
        nb = self.lib.osbli_central_store_all_bytes(C.byref(self.params))
        self._cwork = torch.empty(nb + 256, dtype=torch.uint8, device=self.device)
        off = (-self._cwork.data_ptr()) % 256
        B.check(self.lib.osbli_central_store_all(self.ctx, C.c_void_p(self._cwork.data_ptr() + off), nb), self.ctx)

    def rk_coeffs(self):
        A = (C.c_double * 5)()
        Bc = (C.c_double * 5)()
        B.check(self.lib.osbli_rk_coeffs(self.ctx, A, Bc), self.ctx)
        return list(A)[: self.nstages], list(Bc)[: self.nstages]

    # ---- time loop (section 2.7 ordering: residual, update, BCs) ----
    def step(self, dt):
        for s in range(self.nstages):
            self.substep(s, dt)
            self.apply_bc()
        self.t += dt
        self.nsteps_done += 1

    def run(self, nsteps, cfl=0.5, dt_fixed=0.0, t_end=0.0, start_bc=True):
        if start_bc:
            self.apply_bc()
        for _ in range(int(nsteps)):
            if t_end > 0.0 and self.t >= t_end:
                break
            dt = dt_fixed if dt_fixed > 0.0 else self.compute_dt(cfl)
            if t_end > 0.0 and self.t + dt > t_end:
                dt = t_end - self.t
            self.step(dt)
        return self.t

    def state(self):
        torch.cuda.synchronize(self.device)
        return self.U.cpu().numpy()

    def interior(self):
        nd = self.prob.ndim
        sl = [slice(None)] + [slice(NGHOST, -NGHOST) if d < nd else slice(None) for d in (2, 1, 0)]
        return self.state()[tuple(sl)]
