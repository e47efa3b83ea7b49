"""Batched advance of many independent 2D problems (the C ABI's osbli_batch_*
calls), with a tile autotuner.

Every problem keeps its own context and state; one RK3 step of the whole
ensemble is three launches of captured graphs (one per substage) of
persistent kernels that walk a tile queue over all problems.  Each problem
has its own CFL time step and end time, kept on the device.

    b = Batch(problems, form=1, sensor=1, weights=bits, threshold=thr)
    b.tune()          # optional: measured choice of sweep tiles per grid size
    b.run()           # until every problem reaches its end time

The autotuner chooses, per grid size class, the runs per tile of the
lanes-along-x sweep and the marching y sweep's segment length, then the
workgroups per persistent sweep launch, by coordinate descent on the
measured time of whole-ensemble steps, run on a scratch copy of the ensemble
so that the real one is not advanced; results are cached per (device, form,
sensor, grid size).
"""
from __future__ import annotations

import ctypes as C
import json
import os

import numpy as np
import torch

from . import binding as B
from .solver import Solver

SEG_CANDIDATES = (8, 16, 32, 64, 128)
XL_RUNS = (1, 2, 4, 8, 16)                      # 63-interface runs per tile of the lanes-along-x sweep
GRID_CANDIDATES = (512, 1024, 2048, 4096, 8192)  # workgroups per persistent sweep launch


def default_seg(n_d, lines):
    """The single-grid launch's segment rule (about 2^18 threads per sweep)."""
    target = 1 << 18
    seg = max(8, -(-n_d * lines // target))
    return min(seg, n_d)


def _cache_path():
    return os.environ.get("OSBLI_TILE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "osbli_tiles.json"))


def _cache_load(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _cache_store(path, d):
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(d, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except OSError:
        pass


class Batch:
    def __init__(self, probs, form=B.FORM_FP64, sensor=0, weights=None, threshold=None, dilate=1, cfl=0.5,
                 t_end=None, device="cuda:0", stream=None, capture=True):
        if not torch.cuda.is_available():
            raise RuntimeError("the HIP library needs a GPU (torch.cuda is not available)")
        self.lib = B.load()
        self.device = torch.device(device)
        self.probs = list(probs)
        self.P = len(self.probs)
        self.form, self.sensor, self.cfl = form, int(sensor), float(cfl)
        self.weights, self.threshold, self.dilate = weights, threshold, dilate
        # graph capture needs a stream other than the legacy default one
        self.stream = stream if stream is not None else torch.cuda.Stream(self.device)
        with torch.cuda.stream(self.stream):
            self.solvers = [Solver(p, device, form=form, sensor=sensor, stream=self.stream) for p in self.probs]
            if sensor:
                if weights is None or threshold is None:
                    raise ValueError("sensor routing needs weights and a threshold")
                for s in self.solvers:
                    s.set_sensor(weights, threshold, dilate=dilate)
            for s in self.solvers:
                s.apply_bc()
            nb = self.lib.osbli_batch_workspace_bytes(self.P)
            self.ws = torch.empty(nb + 256, dtype=torch.uint8, device=self.device)
        self.stream.synchronize()
        off = (-self.ws.data_ptr()) % 256
        ends = [float(p.t_end if t_end is None else (t_end[i] if np.ndim(t_end) else t_end))
                for i, p in enumerate(self.probs)]
        self.t_end = np.asarray(ends, dtype=np.float64)
        ctxs = (C.c_void_p * self.P)(*[s.ctx.value for s in self.solvers])
        Us = (C.c_void_p * self.P)(*[s.U.data_ptr() for s in self.solvers])
        dUs = (C.c_void_p * self.P)(*[s.dU.data_ptr() for s in self.solvers])
        self.b = C.c_void_p()
        rc = self.lib.osbli_batch_create(C.byref(self.b), ctxs, self.P, Us, dUs,
                                         self.t_end.ctypes.data_as(C.POINTER(C.c_double)), self.cfl,
                                         C.c_void_p(self.ws.data_ptr() + off), C.c_size_t(nb), self._s())
        B.check_batch(rc, self.b)
        self.captured = False
        # x: runs per tile for rows of >= 64 interfaces (lanes-along-x sweep), else the segment
        self.tiles = np.array([[4 if p.n[0] + 1 >= 64 else default_seg(p.n[0], p.n[1]),
                                default_seg(p.n[1], p.n[0])] for p in self.probs], dtype=np.int64)
        self.sweep_blocks = 0
        self.tune_report = None
        self.steps_done = 0
        if capture:
            self.capture()

    def _s(self):
        return C.c_void_p(self.stream.cuda_stream)

    def __del__(self):
        try:
            if getattr(self, "b", None):
                self.lib.osbli_batch_destroy(self.b)
                self.b = None
        except Exception:
            pass

    # ---- ABI wrappers ----
    def set_tiles(self, seg):
        seg = np.ascontiguousarray(np.asarray(seg, dtype=np.int64).reshape(self.P, 2))
        B.check_batch(self.lib.osbli_batch_set_tiles(self.b, seg.ctypes.data_as(C.POINTER(C.c_int64)), self._s()),
                      self.b)
        lim = np.array([[64 if p.n[0] + 1 >= 64 else p.n[0], p.n[1]] for p in self.probs])
        self.tiles = np.minimum(seg, lim)
        was = self.captured
        self.captured = False
        if was:
            self.capture()

    def capture(self):
        B.check_batch(self.lib.osbli_batch_capture(self.b, self._s()), self.b)
        self.captured = True

    def substep(self, stage):
        B.check_batch(self.lib.osbli_batch_substep(self.b, int(stage), self._s()), self.b)

    def step(self, n=1):
        for _ in range(int(n)):
            for st in range(3):
                self.substep(st)
        self.steps_done += int(n)

    def status(self):
        t = np.zeros(self.P)
        act = np.zeros(self.P, dtype=np.int32)
        na = C.c_int(0)
        B.check_batch(self.lib.osbli_batch_status(self.b, t.ctypes.data_as(C.POINTER(C.c_double)),
                                                  act.ctypes.data_as(C.POINTER(C.c_int)), C.byref(na), self._s()),
                      self.b)
        return t, act.astype(bool), na.value

    def points(self):
        pts, tiles = C.c_int64(0), C.c_int64(0)
        B.check_batch(self.lib.osbli_batch_interior_points(self.b, C.byref(pts), C.byref(tiles)), self.b)
        return pts.value, tiles.value

    def check(self):
        self.solvers[0].check()

    def run(self, max_steps=10 ** 9, poll=64):
        """Step until every problem is done (or max_steps); the host polls the
        device status every `poll` steps.  Returns the number of steps."""
        done = 0
        while done < max_steps:
            k = min(poll, max_steps - done)
            self.step(k)
            done += k
            if self.status()[2] == 0:
                break
        return done

    def state(self, p):
        self.stream.synchronize()
        return self.solvers[p].U.cpu().numpy()

    def interior(self, p):
        self.stream.synchronize()
        return self.solvers[p].interior()

    # ---- autotuner ----
    def time_steps(self, nsteps=3, warm=1):
        """Mean milliseconds per whole-ensemble step (events on the batch's
        stream)."""
        self.step(warm)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(self.stream)
        self.step(nsteps)
        e1.record(self.stream)
        e1.synchronize()
        return e0.elapsed_time(e1) / nsteps

    def set_grid(self, sweep_blocks):
        """Workgroups per persistent sweep launch (0: the library defaults)."""
        B.check_batch(self.lib.osbli_batch_set_grid(self.b, int(sweep_blocks)), self.b)
        self.sweep_blocks = int(sweep_blocks)
        was = self.captured
        self.captured = False
        if was:
            self.capture()

    def tune(self, nsteps=4, cache=True, log=None):
        """Measured choice of the launch knobs that change the ensemble's time:
        per grid-size class, the runs per tile of the lanes-along-x sweep
        (XL_RUNS; the marching x segment for narrow grids) and the marching y
        sweep's segment (SEG_CANDIDATES), then the workgroups per persistent
        sweep launch (GRID_CANDIDATES); coordinate descent on the mean time of
        whole-ensemble steps, run on a scratch copy of the ensemble so the
        real one does not advance.  Results are cached per (device, form,
        sensor, size class).  Returns the choices and the default and tuned
        milliseconds per step."""
        sizes = sorted({(p.n[0], p.n[1]) for p in self.probs}, key=lambda s: -s[0] * s[1])
        dev = torch.cuda.get_device_name(self.device).replace(" ", "_")
        key = lambda s: "v2|%s|form%d|sensor%d|%dx%d" % (dev, self.form, self.sensor, s[0], s[1])
        gkey = "v2|%s|form%d|sensor%d|grid|%d" % (dev, self.form, self.sensor, self.P)
        path = _cache_path()
        store = _cache_load(path) if cache else {}
        scratch = Batch(self.probs, form=self.form, sensor=self.sensor, weights=self.weights,
                        threshold=self.threshold, dilate=self.dilate, cfl=self.cfl,
                        t_end=np.full(self.P, 1e30), device=self.device, capture=True)
        seg = scratch.tiles.copy()
        default_ms = scratch.time_steps(nsteps)
        todo = [s for s in sizes if key(s) not in store]
        fresh = bool(todo) or gkey not in store      # else every choice comes from the cache
        best_t = default_ms
        for s in todo:
            members = [i for i, p in enumerate(self.probs) if (p.n[0], p.n[1]) == s]
            xl = s[0] + 1 >= 64
            for d in (0, 1):
                cands = XL_RUNS if (d == 0 and xl) else [c for c in SEG_CANDIDATES if c <= s[d]]
                for c in cands:
                    if c == seg[members[0], d]:
                        continue
                    trial = seg.copy()
                    trial[members, d] = c
                    scratch.set_tiles(trial)
                    t = scratch.time_steps(nsteps)
                    if t < best_t:
                        best_t, seg = t, trial
            store[key(s)] = [int(v) for v in seg[members[0]]]
            if log:
                log("[tune] %dx%d: %s %d, y segment %d, ensemble step %.3f ms"
                    % (s[0], s[1], "x runs/tile" if xl else "x segment", seg[members[0], 0], seg[members[0], 1],
                       best_t))
        for i, p in enumerate(self.probs):
            seg[i] = store[key((p.n[0], p.n[1]))]
        scratch.set_tiles(seg)
        if gkey not in store:
            best_g, best_t = 0, scratch.time_steps(nsteps)
            for gb in GRID_CANDIDATES:
                scratch.set_grid(gb)
                t = scratch.time_steps(nsteps)
                if t < best_t:
                    best_g, best_t = gb, t
            store[gkey] = best_g
            if log:
                log("[tune] sweep workgroups %s, ensemble step %.3f ms" % (best_g or "default", best_t))
        # the search compares single short timings; confirm the choice against
        # the defaults with interleaved repeats (best of three each) and keep
        # the defaults unless the choice is faster
        dflt = self.tiles.copy()

        def timed(tiles, grid):
            scratch.set_tiles(tiles)
            scratch.set_grid(grid)
            return scratch.time_steps(2 * nsteps)
        t_def, t_tun = [], []
        for _ in range(3):
            t_def.append(timed(dflt, 0))
            t_tun.append(timed(seg, store[gkey]))
        default_ms, tuned_ms = min(t_def), min(t_tun)
        kept = tuned_ms < default_ms or not fresh
        if not kept:
            seg, tuned_ms = dflt, default_ms
            for s in sizes:
                members = [i for i, p in enumerate(self.probs) if (p.n[0], p.n[1]) == s]
                store[key(s)] = [int(v) for v in dflt[members[0]]]
            store[gkey] = 0
        del scratch
        torch.cuda.synchronize(self.device)
        if cache:
            _cache_store(path, store)
        for i, p in enumerate(self.probs):
            seg[i] = store[key((p.n[0], p.n[1]))]
        self.set_tiles(seg)
        self.set_grid(store[gkey])
        self.tune_report = {"default_ms_per_step": round(default_ms, 4), "tuned_ms_per_step": round(tuned_ms, 4),
                            "sweep_blocks": int(store[gkey]), "search_kept": bool(kept)}
        if log:
            log("[tune] confirmed: default %.3f ms, tuned %.3f ms per step (%s)"
                % (default_ms, tuned_ms, "kept" if kept else "defaults kept"))
        out = {s: tuple(store[key(s)]) for s in sizes}
        return out


def solo_run(prob, form=B.FORM_FP64, sensor=0, weights=None, threshold=None, dilate=1, cfl=0.5, device="cuda:0",
             t_end=None):
    """The same problem advanced alone with the single-grid calls (the batch's
    reference)."""
    s = Solver(prob, device, form=form, sensor=sensor)
    if sensor:
        s.set_sensor(weights, threshold, dilate=dilate)
    s.run(10 ** 9, cfl=cfl, t_end=prob.t_end if t_end is None else t_end)
    return s
