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
    return {"value": round(n ** 3 / el / 1e6, 4), "unit": "Mpoint-substeps/s", "cores": threads,
            "kind": "oracle",
            "sample": "one RK substage (residual + low-storage update) of TGV %d^3, FP64, %.1f s" % (n, el)}


def timed_run(prob, form, steps, warmup, cfl):
    """W warm-up steps, then K timed steps (dt reduction + 3 substages + BCs
    each) with the library's per-kernel event timing on."""
    import torch
    from paper_2007_14933_amd.solver import Solver
    s = Solver(prob, form=form)
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
    del s
    torch.cuda.empty_cache()
    return wall, gpu_ms, prof


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


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only (got --gpus %d); the multi-GPU halo exchange "
              "is described in the design notes but not built" % args.gpus, file=sys.stderr)
        sys.exit(2)
    from paper_2007_14933_amd import cost, inputs

    n = args.n
    prob = inputs.tgv(n)
    npts = n ** 3
    wall, gpu_ms, prof = timed_run(prob, 0, args.steps, args.warmup, args.cfl)
    value = npts * 3 * args.steps / wall / 1e6

    # dominant kernel: the convective sweeps (one launch per direction and substage)
    sweep_cnt = sum(prof["sweep_%s" % a][0] for a in "xyz")
    sweep_ms = sum(prof["sweep_%s" % a][1] for a in "xyz")
    fl_if = cost.flops_per_interface(3, prob.scheme)
    fl_launch = fl_if * sum(cost.interfaces_per_sweep(prob.n, 3, d) for d in range(3)) / 3.0
    avg_ms = sweep_ms / max(1, sweep_cnt)
    achieved = fl_launch / (avg_ms * 1e-3) / 1e12
    peak = cost.PEAK_FP64_VALU_TFLOPS
    roofline = {"bound": "alu", "achieved": round(achieved, 3), "peak": peak, "unit": "TFLOP/s",
                "frac": round(achieved / peak, 4), "traffic": None,
                "kernel": "k_sweep<3,d,TENO5> (average over x, y, z)", "avg_ms": round(avg_ms, 4),
                "flops_per_launch": fl_launch}
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
        "roofline": roofline,
        "kernels": breakdown,
    }
    if not args.no_forms:
        wm, _, pm = timed_run(prob, 1, args.steps, args.warmup, args.cfl)
        vm = npts * 3 * args.steps / wm / 1e6
        sm = sum(pm["sweep_%s" % a][1] for a in "xyz") / max(1, sum(pm["sweep_%s" % a][0] for a in "xyz"))
        out["forms"] = {"mixed_fp32": {
            "value": round(vm, 3), "speedup_vs_fp64": round(vm / value, 3),
            "sweep_avg_ms": round(sm, 4),
            "error_vs_fp64": form_error(prob, 1, 10, args.cfl)}}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.cpu_n or n)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
