#!/usr/bin/env python3
"""Benchmark of the per-Runge-Kutta-substage residual on one MI355X.

Workload: the 3D Taylor-Green vortex, 256^3 periodic box, Re = 1600, M = 0.1,
Pr = 0.71, TENO5 + fourth-order central viscous terms, low-storage RK3 with
dt from CFL = 0.5, plain FP64 (synthetic analytic initial state).  One
"step" = dt reduction + three substages (convective sweeps, viscous fluxes,
viscous divergence fused with the RK update) + boundary conditions after each.

Prints one JSON line:
  value        Mpoint-substeps/s (interior points x 3 substages / wall time)
  roofline     dominant kernel (convective sweep) against the FP64 VALU peak,
               timed live with HIP events on its launch stream
  cpu_baseline the FP64 oracle on a bounded sample (one substage of the same
               256^3 problem) on the host's cores

    python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)


def log(*a):
    """Progress line on stderr (the JSON result is the only stdout line)."""
    print("[bench]", *a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=256, help="TGV grid points per direction")
    ap.add_argument("--cfl", type=float, default=0.5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-forms", action="store_true", help="skip the precision / sensor forms")
    ap.add_argument("--cpu-n", type=int, default=0, help="oracle sample grid (default: same as --n)")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-ensemble line")
    ap.add_argument("--no-central", action="store_true", help="skip the central-path (StoreSome) line")
    ap.add_argument("--central-steps", type=int, default=20)
    ap.add_argument("--no-schemes", action="store_true", help="skip the TENO6 / WENO-JS5 / WENO-3Z / WENO-7Z line")
    ap.add_argument("--scheme-steps", type=int, default=10)
    ap.add_argument("--batch-steps", type=int, default=30)
    ap.add_argument("--batch-full", action="store_true",
                    help="also run both batched forms to t = 0.25 and report their density difference")
    ap.add_argument("--no-tune", action="store_true", help="batched ensemble with default tiles")
    ap.add_argument("--cpu-table", action="store_true",
                    help="also time the oracle on every workload (bounded samples, all threads and one thread)")
    return ap.parse_args()


def cpu_baseline(n):
    """The oracle as it stands: one RK substage (residual + update) of the
    same TGV problem, timed on the host cores it uses (metrics and set-up
    excluded)."""
    import numpy as np
    from oracle import oracle as O
    from paper_2007_14933_amd import inputs
    prob = inputs.tgv(n)
    S, J = O.metrics(prob)
    U = prob.U0.copy()
    O.apply_bc(prob, U)
    dU = np.zeros(O.int_shape(prob))
    dt = O.compute_dt(prob, S, J, U, 0.5)
    t0 = time.perf_counter()
    O.rk_substep(prob, S, J, 0, dt, U, dU)
    el = time.perf_counter() - t0
    threads = O.num_threads()
    out = {"value": round(n ** 3 / el / 1e6, 4), "unit": "Mpoint-substeps/s", "cores": threads,
           "kind": "oracle",
           "sample": "one RK substage (residual + low-storage update) of TGV %d^3, FP64, %.1f s" % (n, el),
           "cpu_model": cpu_model(), "host_cpus": os.cpu_count()}
    out["one_thread"] = one_thread_rate(64)
    return out


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            return next(l.split(":", 1)[1].strip() for l in f if l.startswith("model name"))
    except (OSError, StopIteration):
        return "unknown"


def one_thread_rate(n):
    """The oracle on one thread (a child process with OMP_NUM_THREADS=1): one
    RK substage of TGV n^3, Mpoint-substeps/s."""
    import subprocess
    code = ("import sys, time; sys.path.insert(0, %r); from oracle import oracle as O; "
            "from paper_2007_14933_amd import inputs; import numpy as np; p = inputs.tgv(%d); S, J = O.metrics(p); "
            "U = p.U0.copy(); O.apply_bc(p, U); dU = np.zeros(O.int_shape(p)); dt = O.compute_dt(p, S, J, U, 0.5); "
            "t0 = time.perf_counter(); O.rk_substep(p, S, J, 0, dt, U, dU); el = time.perf_counter() - t0; "
            "print(%d ** 3 / el / 1e6, el, O.num_threads())" % (ROOT, n, n))
    env = dict(os.environ, OMP_NUM_THREADS="1")
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env, timeout=600)
    try:
        v, el, th = r.stdout.split()[-3:]
        return {"value": round(float(v), 4), "unit": "Mpoint-substeps/s", "threads": int(th),
                "sample": "one RK substage of TGV %d^3, %.2f s" % (n, float(el))}
    except ValueError:
        return {"error": r.stderr[-300:]}


SWEEP_SOURCES = ("paper_2007_14933_amd/csrc/sweep.hpp", "paper_2007_14933_amd/csrc/charflux.hpp",
                 "paper_2007_14933_amd/csrc/convective.hip", "paper_2007_14933_amd/csrc/internal.hpp")
TRAFFIC_PROFILE = "profiles/tgv256_sweep_hbm_traffic.txt"


def sweep_source_hash():
    import hashlib
    h = hashlib.sha1()
    for f in SWEEP_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def sweep_profile():
    """Per-launch figures of the sweeps from the committed rocprofv3 counter
    summary: HBM bytes (FETCH_SIZE and WRITE_SIZE, scaled by a copy kernel of
    known size) and executed FP64 flops (SQ_INSTS_VALU_FLOPS_FP64), or {}
    when the sweep sources changed since the counters were taken."""
    path = os.path.join(ROOT, TRAFFIC_PROFILE)
    if not os.path.exists(path):
        return {}
    vals = {}
    with open(path) as f:
        for line in f:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                vals[k.strip()] = v.strip()
    if vals.get("source_hash") != sweep_source_hash():
        return {}
    out = {}
    for key in ("traffic_bytes_per_launch", "executed_fp64_flops_per_launch"):
        try:
            out[key] = float(vals[key])
        except (KeyError, ValueError):
            pass
    return out


def copy_ceiling(nbytes=1 << 30, reps=5):
    """Device-to-device copy of `nbytes` (read + write) as the achievable HBM
    rate, GB/s."""
    import torch
    src = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda:0").fill_(1.0)
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    e1.synchronize()
    gbs = 2 * nbytes * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del src, dst
    torch.cuda.empty_cache()
    return gbs


def cpu_table():
    """The oracle on each workload (bounded samples) on all host threads, and
    one TGV 64^3 substage on one thread (a child process)."""
    import subprocess
    import numpy as np
    from oracle import oracle as O
    from paper_2007_14933_amd import inputs

    out = {"threads": O.num_threads(), "cpu": cpu_model()}
    cases = [("sod400_full_run", inputs.sod(400), 10 ** 6, 0.2),
             ("tgv256_2_steps", inputs.tgv(256), 2, 0.0),
             ("tgv64_100_steps", inputs.tgv(64), 100, 0.0),
             ("wall512x256x256_1_step", inputs.wall_flow(), 1, 0.0),
             ("shockvortex1024x512_10_steps", inputs.shock_vortex(1024, 512, seed=42), 10, 0.0)]
    rng = np.random.default_rng(2007)
    for n in (128, 448, 768, 1024):
        cases.append(("riemann%d_10_steps" % n, inputs.riemann2d(n, rng), 10, 0.0))
    for name, prob, nst, te in cases:
        S, J = O.metrics(prob)
        U = prob.U0.copy()
        t0 = time.perf_counter()
        if te > 0.0:
            steps, tt = 0, 0.0
            while tt < te and steps < 10 ** 6:
                tt = O.run(prob, S, J, U, 1, cfl=0.5, t_end=te, t0=tt)
                steps += 1
        else:
            O.run(prob, S, J, U, nst, cfl=0.5)
            steps = nst
        el = time.perf_counter() - t0
        out[name] = {"seconds": round(el, 3), "steps": steps,
                     "Mpoint_substeps_per_s": round(prob.npoints * 3 * steps / el / 1e6, 3)}
    code = ("import sys, time; sys.path.insert(0, %r); from oracle import oracle as O; "
            "from paper_2007_14933_amd import inputs; import numpy as np; p = inputs.tgv(64); S, J = O.metrics(p); "
            "U = p.U0.copy(); O.apply_bc(p, U); dU = np.zeros(O.int_shape(p)); dt = O.compute_dt(p, S, J, U, 0.5); "
            "t0 = time.perf_counter(); O.rk_substep(p, S, J, 0, dt, U, dU); "
            "print(64 ** 3 / (time.perf_counter() - t0) / 1e6, O.num_threads())" % ROOT)
    env = dict(os.environ, OMP_NUM_THREADS="1")
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env, timeout=600)
    try:
        v, th = r.stdout.split()[-2:]
        out["tgv64_1_substage_one_thread"] = {"Mpoint_substeps_per_s": round(float(v), 3), "threads": int(th)}
    except ValueError:
        out["tgv64_1_substage_one_thread"] = {"error": r.stderr[-300:]}
    return out


def timed_run(prob, form, steps, warmup, cfl, sensor=0, bits=None, thr=None, keep_rho=False, dilate=1):
    """W warm-up steps, then K timed steps (dt reduction + the RK substages +
    BCs each) with the library's per-kernel event timing on."""
    import torch
    from paper_2007_14933_amd.solver import Solver
    s = Solver(prob, form=form, sensor=sensor)
    if sensor:
        s.set_sensor(bits, thr, dilate=dilate)
    stream = s.stream
    s.apply_bc()
    for _ in range(warmup):
        s.step(s.compute_dt(cfl))
    s.check()
    torch.cuda.synchronize()
    s.profile(True)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(steps):
        s.step(s.compute_dt(cfl))
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    s.check()
    prof = s.profile_read()
    s.profile(False)
    gpu_ms = ev0.elapsed_time(ev1)
    extra = {}
    if sensor:
        sm, tot = s.sensor_stats()
        extra["smooth_fraction_last"] = round(sm / tot, 4)
    if keep_rho:
        extra["rho"] = s.interior()[0]
        extra["t"] = s.t
    del s
    torch.cuda.empty_cache()
    return wall, gpu_ms, prof, extra


def form_error(prob, form, steps, cfl):
    """Relative L1 / Linf of rho and rho E of a form against plain FP64 after
    `steps` steps with the same fixed dt (from the initial state)."""
    import numpy as np
    import torch
    from paper_2007_14933_amd.solver import Solver
    outs = []
    dt = None
    for f in (0, form):
        s = Solver(prob, form=f)
        s.apply_bc()
        if dt is None:
            dt = s.compute_dt(cfl)
        for _ in range(steps):
            s.step(dt)
        s.check()
        outs.append(s.interior())
        del s
        torch.cuda.empty_cache()
    a, b = outs[1], outs[0]
    res = {}
    for name, c in (("rho", 0), ("rhoE", prob.nc - 1)):
        d = np.abs(a[c] - b[c])
        res["rel_L1_" + name] = float("%.3e" % (d.mean() / np.abs(b[c]).mean()))
        res["rel_Linf_" + name] = float("%.3e" % (d.max() / np.abs(b[c]).max()))
    res["steps"] = steps
    return res


def sweep_valu_frac(prob, sweep_ms, launches):
    """Effective rate of the convective sweeps against the FP64 vector peak
    (the precision form's FP32 runs at the same rate: packed FP32 is not
    used): nominal TENO5 flops of the interfaces of `launches` sweep launches
    (averaged over the directions) over their measured time."""
    from paper_2007_14933_amd import cost
    nd = prob.ndim
    per = cost.flops_per_interface(nd, 1) * sum(cost.interfaces_per_sweep(prob.n, nd, d) for d in range(nd)) / nd
    if sweep_ms <= 0.0:
        return None
    return round(per * launches / (sweep_ms * 1e-3) / 1e12 / cost.PEAK_FP64_VALU_TFLOPS, 4)


def tgv_learned(prob, args, plain_value, plain_extra):
    """The headline TGV with learned routing (FP64 and FP32 reconstruction):
    same steps as the plain run; relative L1 of rho against the plain run's
    final state."""
    import numpy as np
    from paper_2007_14933_amd import sensor as SN
    if not os.path.exists(SN.DEFAULT_WEIGHTS):
        return {"skipped": "no trained weights"}
    bits, thr = SN.load()
    dil = SN.load_dilate()
    npts = prob.npoints
    ref = plain_extra["rho"]
    res = {"threshold": thr, "dilate": dil}
    for name, form in (("fp64_learned", 0), ("fp32_learned", 1)):
        w, _, p, ex = timed_run(prob, form, args.steps, args.warmup, args.cfl, sensor=1, bits=bits, thr=thr,
                                keep_rho=True, dilate=dil)
        v = npts * 3 * args.steps / w / 1e6
        sw = sum(p["sweep_%s" % a][1] for a in "xyz") / max(1, sum(p["sweep_%s" % a][0] for a in "xyz"))
        res[name] = {"value": round(v, 3), "speedup_vs_plain": round(v / plain_value, 3),
                     "sweep_avg_ms": round(sw, 4), "valu_frac_effective": sweep_valu_frac(prob, sw, 1),
                     "sensor_ms_per_step": round(p["sensor"][1] / max(1, args.steps), 4),
                     "smooth_fraction_last": ex["smooth_fraction_last"],
                     "rel_L1_rho_vs_plain": float("%.3e" % (np.abs(ex["rho"] - ref).mean() / np.abs(ref).mean())),
                     "t_diff_vs_plain": float("%.3e" % (ex["t"] - plain_extra["t"]))}
        res[name]["meets_1e-4"] = bool(res[name]["rel_L1_rho_vs_plain"] <= 1e-4)
    return res


def wall_precision(cfl, steps=100):
    """Supersonic wall-bounded flow 512 x 256 x 256 (tanh wall mesh): plain
    FP64 and the precision form, `steps` steps each with the CFL time step of
    the initial state held fixed (both forms reach the same time); relative
    L1 / Linf of rho and rho E of the precision form against plain."""
    import numpy as np
    import torch
    from paper_2007_14933_amd import inputs
    from paper_2007_14933_amd.solver import Solver
    prob = inputs.wall_flow()
    npts = prob.npoints
    outs, res, dt = [], {}, None
    for name, form in (("plain_fp64", 0), ("fp32_recon", 1)):
        s = Solver(prob, form=form)
        s.apply_bc()
        if dt is None:
            dt = s.compute_dt(cfl)
        s.step(dt)  # warm-up step (kernels loaded, caches warm)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps - 1):
            s.step(dt)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        s.check()
        res[name] = {"value": round(npts * 3 * (steps - 1) / wall / 1e6, 3),
                     "ms_per_step": round(wall * 1e3 / (steps - 1), 3)}
        outs.append(s.interior())
        del s
        torch.cuda.empty_cache()
    a, b = outs[1], outs[0]
    err = {}
    for q, c in (("rho", 0), ("rhoE", prob.nc - 1)):
        d = np.abs(a[c] - b[c])
        err["rel_L1_" + q] = float("%.3e" % (d.mean() / np.abs(b[c]).mean()))
        err["rel_Linf_" + q] = float("%.3e" % (d.max() / np.abs(b[c]).max()))
    res["fp32_recon"]["speedup_vs_plain"] = round(res["fp32_recon"]["value"] / res["plain_fp64"]["value"], 3)
    res["fp32_recon"]["error_vs_plain_after_%d_steps" % steps] = err
    res["workload"] = ("wall-bounded Mach 2, 512x256x256 tanh mesh (beta 2.5), isothermal wall, Sutherland, "
                       "TENO5 + viscous, dt %.4e fixed" % dt)
    return res


def sensor_form(cfl):
    """Shock-vortex field 1024 x 512 (seed 42) run to t = 0.4: plain FP64,
    FP64 + learned routing, FP32 reconstruction + learned routing.  Whole
    runs (dt reduction, sensor refresh, sweeps, updates, BCs), timed with
    events on the solver's stream; error = relative L1 of rho against plain
    at the end time."""
    import numpy as np
    import torch
    from paper_2007_14933_amd import cost, inputs
    from paper_2007_14933_amd import sensor as SN
    from paper_2007_14933_amd.solver import Solver
    if not os.path.exists(SN.DEFAULT_WEIGHTS):
        return {"skipped": "no trained weights at %s" % os.path.relpath(SN.DEFAULT_WEIGHTS, ROOT)}
    bits, thr = SN.load()
    dil = SN.load_dilate()
    prob = inputs.shock_vortex(1024, 512, seed=42)
    npts = prob.npoints
    res, ref = {}, None
    for name, form, sensor in (("plain_fp64", 0, 0), ("fp64_learned", 0, 1), ("fp32_learned", 1, 1),
                               ("fp32_plain", 1, 0)):
        s = Solver(prob, form=form, sensor=sensor)
        if sensor:
            s.set_sensor(bits, thr, dilate=dil)
        s.apply_bc()
        torch.cuda.synchronize()
        s.profile(True)
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        ev0.record(s.stream)
        s.run(10 ** 9, cfl=cfl, t_end=prob.t_end, start_bc=False)
        ev1.record(s.stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        s.check()
        prof = s.profile_read()
        rho = s.interior()[0]
        v = npts * 3 * s.nsteps_done / wall / 1e6
        sweeps = sum(prof["sweep_%s" % a][1] for a in "xy")
        r = {"value": round(v, 3), "steps": s.nsteps_done, "t_end": round(s.t, 6),
             "gpu_ms": round(ev0.elapsed_time(ev1), 3), "sweep_ms": round(sweeps, 3),
             "valu_frac_effective": sweep_valu_frac(prob, sweeps, sum(prof["sweep_%s" % a][0] for a in "xy")),
             "sensor_ms": round(prof["sensor"][1], 3),
             "hbm_compulsory_frac": round(npts * 3 * s.nsteps_done * cost.compulsory_bytes_per_point(2) / wall
                                          / 1e9 / cost.PEAK_HBM_GBS, 4)}
        if sensor:
            sm, tot = s.sensor_stats()
            r["smooth_fraction_last"] = round(sm / tot, 4)
        if ref is None:
            ref = rho
        else:
            r["rel_L1_rho_vs_plain"] = float("%.3e" % (np.abs(rho - ref).mean() / np.abs(ref).mean()))
            r["meets_1e-4"] = bool(r["rel_L1_rho_vs_plain"] <= 1e-4)
            r["speedup_vs_plain"] = round(v / res["plain_fp64"]["value"], 3)
        res[name] = r
        del s
        torch.cuda.empty_cache()
    res["plain_sensitivity_floor_rel_L1_rho"] = float("%.3e" % SN.sensitivity_floor(prob))
    res["workload"] = "shock-vortex 1024x512 seed 42, TENO5, CFL 0.5, to t=0.4; threshold %.3f, dilate %d" % (thr, dil)
    return res


def schemes_form(steps, warmup, cfl, n=256):
    """The further schemes on the headline TGV n^3 (viscous, FP64): TENO6 with
    the SSP RK3 (the paper's production configuration), WENO-JS5 with the
    five-stage RK4, WENO-3Z and WENO-7Z with RK3; same timing as the
    headline line."""
    from paper_2007_14933_amd import inputs
    out = {}
    for name, kw in (("teno6_ssp_rk3", dict(scheme=inputs.TENO6, rk=inputs.RK3_SSP)),
                     ("wenojs5_rk4", dict(scheme=inputs.WENOJS5, rk=inputs.RK4, eps=1e-6)),
                     ("wenoz3_rk3", dict(scheme=inputs.WENOZ3)),
                     ("wenoz7_rk3", dict(scheme=inputs.WENOZ7))):
        prob = inputs.tgv(n).with_(**kw)
        nst = inputs.rk_stages(prob.rk)
        wall, _, prof, _ = timed_run(prob, 0, steps, warmup, cfl)
        sw = sum(prof["sweep_%s" % a][1] for a in "xyz") / max(1, sum(prof["sweep_%s" % a][0] for a in "xyz"))
        out[name] = {"value": round(n ** 3 * nst * steps / wall / 1e6, 3), "ms_per_step": round(wall * 1e3 / steps, 4),
                     "substages_per_step": nst, "sweep_avg_ms": round(sw, 4)}
    out["workload"] = "TGV %d^3 periodic, Re=1600, M=0.1, viscous, CFL 0.5, FP64; %d timed steps" % (n, steps)
    return out


def central_form(steps, warmup, cfl, sizes=(192, 256)):
    """The fourth-order central path on the viscous TGV (the paper's central
    benchmark; 192^3 is its one-GPU size): StoreSome (velocity gradients
    stored) against store-all (every derivative in its own work array), same
    steps, same kernels otherwise."""
    import torch
    from paper_2007_14933_amd import inputs
    from paper_2007_14933_amd.solver import Solver
    out = {}
    for n in sizes:
        prob = inputs.tgv(n, scheme=inputs.CENTRAL4)
        r = {}
        for name, store_all in (("storesome", False), ("storeall", True)):
            s = Solver(prob)
            if store_all:
                s.central_store_all(True)
            s.apply_bc()
            for _ in range(warmup):
                s.step(s.compute_dt(cfl))
            torch.cuda.synchronize()
            s.profile(True)
            t0 = time.perf_counter()
            for _ in range(steps):
                s.step(s.compute_dt(cfl))
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            s.check()
            prof = s.profile_read()
            s.profile(False)
            nst = s.nstages
            r[name] = {"value": round(prob.npoints * nst * steps / wall / 1e6, 3),
                       "ms_per_step": round(wall * 1e3 / steps, 4),
                       "central_ms_per_substage": round(prof["central"][1] / max(1, prof["central"][0]), 4),
                       "finish_ms_per_substage": round(prof["finish"][1] / max(1, prof["finish"][0]), 4)}
            del s
            torch.cuda.empty_cache()
        r["storesome_speedup"] = round(r["storesome"]["value"] / r["storeall"]["value"], 3)
        out["tgv%d" % n] = r
    out["workload"] = ("TGV n^3 periodic, Re=1600, M=0.1, fourth-order central convection + expanded viscous terms, "
                       "RK3 CFL=0.5, FP64; %d timed steps" % steps)
    out["arrays_per_node"] = {"storesome": "U 5 + dU 5 + velocity gradients 9 + residual 5 = 24",
                              "storeall": "U 5 + dU 5 + 57 derivative arrays (63 slots) + residual 5 = 72"}
    return out


def batch_form(steps, warmup, cfl, tune, full):
    """The batched ensemble: 64 seeded four-quadrant Riemann problems,
    N in {128, 192, ..., 1024}, each with its own dt.  Timed over `steps`
    whole-ensemble steps (three graph launches each); value counts the
    points of active problems.  Also the same problems advanced one by one
    (single-grid calls, a few steps each) for the batching gain."""
    import numpy as np
    import torch
    from paper_2007_14933_amd import cost, inputs
    from paper_2007_14933_amd import sensor as SN
    from paper_2007_14933_amd.batch import Batch
    from paper_2007_14933_amd.solver import Solver
    probs = inputs.riemann_batch(64, seed=2007)
    npts = sum(p.npoints for p in probs)
    out = {"workload": "64 four-quadrant Riemann problems (seed 2007), N in 128..1024 step 64, "
                       "%d points, TENO5, CFL 0.5, per-problem dt, t_end 0.25" % npts}
    have_w = os.path.exists(SN.DEFAULT_WEIGHTS)
    forms = [("plain_fp64", 0, 0)] + ([("fp32_learned", 1, 1)] if have_w else [])
    bits, thr = SN.load() if have_w else (None, None)
    dil = SN.load_dilate() if have_w else 1
    finals, snaps = {}, {}
    for name, form, sensor in forms:
        kw = dict(form=form, sensor=sensor, weights=bits, threshold=thr, cfl=cfl, dilate=dil)
        b = Batch(probs, **kw)
        tiles = b.tune(nsteps=3) if tune else None
        b.step(warmup)
        b.stream.synchronize()
        _, act, _ = b.status()
        act_pts = sum(p.npoints for p, a in zip(probs, act) if a)
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        ev0.record(b.stream)
        b.step(steps)
        ev1.record(b.stream)
        b.stream.synchronize()
        wall = time.perf_counter() - t0
        b.check()
        r = {"value": round(act_pts * 3 * steps / wall / 1e6, 3), "ms_per_step": round(wall * 1e3 / steps, 4),
             "gpu_ms_per_step": round(ev0.elapsed_time(ev1) / steps, 4), "steps": steps,
             "hbm_compulsory_frac": round(act_pts * 3 * steps * cost.compulsory_bytes_per_point(2) / wall / 1e9
                                          / cost.PEAK_HBM_GBS, 4),
             "tiles_tuned": bool(tune)}
        if tiles:
            r["tiles"] = {"%dx%d" % k: list(v) for k, v in sorted(tiles.items())}
            r["tiles_note"] = ("per size class: [runs per tile of the lanes-along-x sweep, y segment]; "
                               "sweep workgroups %d (0 = defaults)" % b.tune_report["sweep_blocks"])
            r["tuned_vs_default"] = {"default_ms_per_step": b.tune_report["default_ms_per_step"],
                                     "tuned_ms_per_step": b.tune_report["tuned_ms_per_step"],
                                     "ratio": round(b.tune_report["default_ms_per_step"]
                                                    / b.tune_report["tuned_ms_per_step"], 3)}
        # both forms start from the same states and advance the same number of
        # ensemble steps: their densities are compared after them (the whole
        # run to t = 0.25 with --batch-full)
        snaps[name] = [b.interior(p)[0] for p in range(len(probs))]
        if full:
            n = b.run()
            b.check()
            r["full_run_steps"] = n + steps + warmup
            finals[name] = [b.interior(p)[0] for p in range(len(probs))]
        out[name] = r
        del b
        torch.cuda.empty_cache()
    if "fp32_learned" in out:
        out["fp32_learned"]["speedup_vs_plain"] = round(out["fp32_learned"]["value"] / out["plain_fp64"]["value"], 3)
        errs = [float(np.abs(a - b).mean() / np.abs(b).mean()) for a, b in zip(snaps["fp32_learned"],
                                                                                 snaps["plain_fp64"])]
        out["fp32_learned"]["rel_L1_rho_vs_plain_after_%d_steps" % (steps + warmup)] = {
            "median": float("%.3e" % np.median(errs)), "max": float("%.3e" % max(errs)),
            "meets_1e-4": bool(max(errs) <= 1e-4)}
    if full and len(finals) == 2:
        errs = [float(np.abs(a - b).mean() / np.abs(b).mean()) for a, b in zip(finals["fp32_learned"],
                                                                                 finals["plain_fp64"])]
        out["fp32_learned"]["rel_L1_rho_vs_plain_at_t_end"] = {
            "median": float("%.3e" % np.median(errs)), "max": float("%.3e" % max(errs))}
    # one by one: every problem through the single-grid calls, a few steps each
    solo_ms = 0.0
    k = 4
    for p in probs:
        s = Solver(p)
        s.apply_bc()
        s.step(s.compute_dt(cfl))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(k):
            s.step(s.compute_dt(cfl))
        torch.cuda.synchronize()
        solo_ms += (time.perf_counter() - t0) * 1e3 / k
        del s
    torch.cuda.empty_cache()
    out["one_by_one_plain_fp64"] = {"ms_per_ensemble_step": round(solo_ms, 3),
                                    "value": round(npts * 3 / solo_ms / 1e3, 3)}
    out["plain_fp64"]["batching_gain"] = round(solo_ms / out["plain_fp64"]["ms_per_step"], 3)
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only (got --gpus %d); the multi-GPU halo exchange "
              "is described in the design notes but not built" % args.gpus, file=sys.stderr)
        sys.exit(2)
    from paper_2007_14933_amd import cost, inputs

    n = args.n
    prob = inputs.tgv(n)
    log("copy ceiling")
    copy_gbs = copy_ceiling()
    log("TGV %d^3 plain FP64, %d warm-up + %d timed steps" % (n, args.warmup, args.steps))
    npts = n ** 3
    wall, gpu_ms, prof, plain_extra = timed_run(prob, 0, args.steps, args.warmup, args.cfl, keep_rho=not args.no_forms)
    value = npts * 3 * args.steps / wall / 1e6

    # dominant kernel: the convective sweeps (one launch per direction and substage)
    sweep_cnt = sum(prof["sweep_%s" % a][0] for a in "xyz")
    sweep_ms = sum(prof["sweep_%s" % a][1] for a in "xyz")
    fl_if = cost.flops_per_interface(3, prob.scheme)
    fl_launch = fl_if * sum(cost.interfaces_per_sweep(prob.n, 3, d) for d in range(3)) / 3.0
    avg_ms = sweep_ms / max(1, sweep_cnt)
    achieved = fl_launch / (avg_ms * 1e-3) / 1e12
    peak = cost.PEAK_FP64_VALU_TFLOPS
    sp = sweep_profile()
    traffic = sp.get("traffic_bytes_per_launch")
    executed = sp.get("executed_fp64_flops_per_launch")
    sweep_alg_bytes = npts * sum(cost.sweep_bytes_per_point(3, d == 0) for d in range(3)) / 3.0
    roofline = {"bound": "alu", "achieved": round(achieved, 3), "peak": peak, "unit": "TFLOP/s",
                "frac": round(achieved / peak, 4), "traffic": traffic,
                "traffic_vs_algorithmic": (round(traffic / sweep_alg_bytes, 3) if traffic else None),
                "algorithmic_bytes_per_launch": sweep_alg_bytes,
                "kernel": "k_sweep<3,d,TENO5> (average over x, y, z)", "avg_ms": round(avg_ms, 4),
                "flops_per_launch": fl_launch,
                "flops_model": ("nominal: the full TENO5 characteristic flux, weights at every reconstruction "
                                "(%d flops per interface); the kernel skips the weights where a bound proves no "
                                "stencil is cut" % fl_if),
                "executed_fp64_flops_per_launch": executed,
                "executed_achieved": (round(executed / (avg_ms * 1e-3) / 1e12, 3) if executed else None),
                "executed_frac": (round(executed / (avg_ms * 1e-3) / 1e12 / peak, 4) if executed else None)}
    breakdown = {k: {"launch_groups": c, "avg_ms": round(ms / c, 4) if c else 0.0} for k, (c, ms) in prof.items()}

    out = {
        "metric": "Mpoint-substeps/s: plain FP64 vs FP32+learned sensor at rel L1≤1e-4; %HBM peak",
        "value": round(value, 3),
        "unit": "Mpoint-substeps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall * 1e3 / args.steps, 4),
        "gpu_ms_per_step": round(gpu_ms / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "TGV %d^3 periodic, Re=1600, M=0.1, Pr=0.71, TENO5 + 4th-order central "
                               "viscous, RK3 CFL=0.5, plain FP64" % n, "points": npts, "form": "plain FP64",
                   "parallelism": "single GPU"},
        "hbm_compulsory_frac": round(npts * 3 * args.steps * cost.compulsory_bytes_per_point(3) / wall / 1e9
                                     / cost.PEAK_HBM_GBS, 4),
        "copy_ceiling_GBs": round(copy_gbs, 1),
        "hbm_compulsory_frac_of_copy_ceiling": round(npts * 3 * args.steps * cost.compulsory_bytes_per_point(3)
                                                     / wall / 1e9 / copy_gbs, 4),
        "roofline": roofline,
        "kernels": breakdown,
    }
    if not args.no_forms:
        log("precision form on TGV")
        wm, _, pm, _ = timed_run(prob, 1, args.steps, args.warmup, args.cfl)
        vm = npts * 3 * args.steps / wm / 1e6
        sm = sum(pm["sweep_%s" % a][1] for a in "xyz") / max(1, sum(pm["sweep_%s" % a][0] for a in "xyz"))
        out["forms"] = {"mixed_fp32": {
            "value": round(vm, 3), "speedup_vs_fp64": round(vm / value, 3),
            "sweep_avg_ms": round(sm, 4), "valu_frac_effective": sweep_valu_frac(prob, sm, 1),
            "error_vs_fp64": form_error(prob, 1, 10, args.cfl)}}
        log("learned routing on TGV")
        out["forms"]["tgv_learned"] = tgv_learned(prob, args, value, plain_extra)
        log("shock-vortex 1024x512: plain and learned forms to t = 0.4")
        out["forms"]["learned_sensor"] = sensor_form(args.cfl)
        log("wall flow 512x256x256: plain and precision form")
        out["forms"]["wall_precision"] = wall_precision(args.cfl)
    if not args.no_schemes:
        log("further schemes on TGV")
        out["schemes"] = schemes_form(args.scheme_steps, args.warmup, args.cfl, n)
    if not args.no_central:
        log("central path: StoreSome against store-all")
        out["central"] = central_form(args.central_steps, args.warmup, args.cfl)
    if not args.no_batch:
        log("batched Riemann ensemble")
        out["batch"] = batch_form(args.batch_steps, args.warmup, args.cfl, not args.no_tune, args.batch_full)
    if not args.no_cpu_baseline:
        log("oracle on the host cores")
        out["cpu_baseline"] = cpu_baseline(args.cpu_n or n)
    if args.cpu_table:
        log("oracle table")
        out["cpu_table"] = cpu_table()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
