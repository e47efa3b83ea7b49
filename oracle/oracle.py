"""ctypes front end of the plain FP64 CPU oracle (``osbli_oracle.c``).

TEST INFRASTRUCTURE ONLY.  The test-suite, the smoke check and the CPU
baseline leg of the benchmark are the only callers.  This module imports
neither the GPU library nor its Python binding; problems are passed in as any
object carrying the problem attributes (``ndim, n, gamma, Re, Pr, Minf,
sutherland, Ts_over_Tref, scheme, teno_CT, eps, roe_avg, bc, wall_T, period,
body_force, coords``), e.g. the ``Problem`` records of the seeded input
generators.

Array layout: U[c][k][j][i] with three ghost nodes on each side of every active
direction; residual and RK register arrays over interior nodes only.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "osbli_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

GCC_FLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-shared", "-fPIC", "-std=c99"]


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (no FMA contraction, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", *GCC_FLAGS, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class Params(C.Structure):
    _fields_ = [
        ("ndim", C.c_int32), ("pad0", C.c_int32),
        ("n", C.c_int64 * 3),
        ("gamma", C.c_double), ("Re", C.c_double), ("Pr", C.c_double), ("Minf", C.c_double),
        ("sutherland", C.c_int32), ("scheme", C.c_int32),
        ("Ts_over_Tref", C.c_double), ("teno_CT", C.c_double), ("eps", C.c_double),
        ("roe_avg", C.c_int32), ("rk", C.c_int32),
        ("bc", (C.c_int32 * 2) * 3),
        ("wall_T", (C.c_double * 2) * 3),
        ("period", C.c_double * 3),
        ("body_force", C.c_double),
    ]


_D = C.POINTER(C.c_double)
_I = C.POINTER(C.c_int)


def _load():
    global _lib
    with _lock:
        if _lib is None:
            build()
            lib = C.CDLL(_LIB)
            P = C.POINTER(Params)
            sig = {
                "orc_metrics": (C.c_int, [P, _D, _D, _D, _D, _D]),
                "orc_apply_bc": (None, [P, _D]),
                "orc_residual": (C.c_int, [P, _D, _D, _D, _D]),
                "orc_viscous_residual": (C.c_int, [P, _D, _D, _D, _D]),
                "orc_rk_update": (C.c_int, [P, C.c_int, C.c_double, _D, _D, _D]),
                "orc_rk_substep": (C.c_int, [P, _D, _D, C.c_int, C.c_double, _D, _D]),
                "orc_compute_dt": (C.c_double, [P, _D, _D, _D, C.c_double]),
                "orc_run": (C.c_int, [P, _D, _D, _D, _D, C.c_int64, C.c_double, C.c_double,
                                      C.c_double, _D]),
                "orc_recon5": (C.c_double, [C.c_int, C.c_double, C.c_double, _D, _I]),
                "orc_recon": (C.c_double, [C.c_int, C.c_double, C.c_double, _D, _I]),
                "orc_rk_coeffs": (None, [P, _D, _D, _I]),
                "orc_smoothness6": (C.c_double, [_D, _D]),
                "orc_recon_wenoz7": (C.c_double, [C.c_double, _D]),
                "orc_smoothness7": (None, [_D, _D, _D]),
                "orc_smoothness5": (None, [_D, _D]),
                "orc_iface_flux": (None, [P, C.c_int, _D, _D, _D, _I]),
                "orc_phys_flux": (None, [P, _D, _D, _D]),
                "orc_eigen": (None, [P, C.c_int, _D, _D, _D, _D, _D, _D]),
                "orc_deriv_line": (None, [_D, C.c_int64, C.c_int, _D]),
                "orc_deriv2_line": (None, [_D, C.c_int64, C.c_int, _D]),
                "orc_deriv_field": (None, [P, _D, C.c_int, _D]),
                "orc_viscosity": (C.c_double, [P, C.c_double]),
                "orc_num_threads": (C.c_int, []),
                "orc_cheap_flux": (None, [P, C.c_int, _D, _D, _D]),
                "orc_features": (None, [P, C.c_int, _D, _D, _D, _I]),
            }
            for name, (res, args) in sig.items():
                f = getattr(lib, name)
                f.restype = res
                f.argtypes = args
            _lib = lib
    return _lib


def _dp(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_D)


def _ip(a: np.ndarray):
    assert a.dtype == np.intc and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_I)


def params(prob) -> Params:
    p = Params()
    p.ndim = int(prob.ndim)
    for d in range(3):
        p.n[d] = int(prob.n[d]) if d < prob.ndim else 1
        p.period[d] = float(prob.period[d])
        for s in range(2):
            p.bc[d][s] = int(prob.bc[d][s])
            p.wall_T[d][s] = float(prob.wall_T[d][s])
    p.gamma, p.Re, p.Pr, p.Minf = float(prob.gamma), float(prob.Re), float(prob.Pr), float(prob.Minf)
    p.sutherland = int(prob.sutherland)
    p.Ts_over_Tref = float(prob.Ts_over_Tref)
    p.scheme = int(prob.scheme)
    p.teno_CT = float(prob.teno_CT)
    p.eps = float(prob.eps)
    p.roe_avg = int(prob.roe_avg)
    p.rk = int(getattr(prob, "rk", 0))
    p.body_force = float(getattr(prob, "body_force", 0.0))
    return p


def ext_shape(prob):
    nd = prob.ndim
    e = [int(prob.n[d]) + 6 if d < nd else 1 for d in range(3)]
    return (nd + 2, e[2], e[1], e[0])


def int_shape(prob):
    nd = prob.ndim
    n = [int(prob.n[d]) if d < nd else 1 for d in range(3)]
    return (nd + 2, n[2], n[1], n[0])


def interior(prob, U):
    nd = prob.ndim
    sl = [slice(None)] + [slice(3, -3) if d < nd else slice(None) for d in (2, 1, 0)]
    return U[tuple(sl)]


def metrics(prob):
    """Node area vectors S[d][m] and J on the ghost-extended grid."""
    lib = _load()
    p = params(prob)
    shp = ext_shape(prob)[1:]
    S = np.zeros((3, 3) + shp)
    J = np.zeros(shp)
    cs = []
    for d in range(3):
        c = prob.coords[d] if d < prob.ndim else None
        cs.append(None if c is None else np.ascontiguousarray(c, dtype=np.float64))
    ptrs = [(_dp(c) if c is not None else None) for c in cs]
    rc = lib.orc_metrics(C.byref(p), ptrs[0], ptrs[1], ptrs[2], _dp(S), _dp(J))
    if rc != 0:
        raise RuntimeError("orc_metrics failed")
    return S, J


def apply_bc(prob, U):
    _load().orc_apply_bc(C.byref(params(prob)), _dp(U))
    return U


def residual(prob, S, J, U):
    R = np.zeros(int_shape(prob))
    _load().orc_residual(C.byref(params(prob)), _dp(S), _dp(J), _dp(U), _dp(R))
    return R


def viscous_residual(prob, S, J, U):
    R = np.zeros(int_shape(prob))
    _load().orc_viscous_residual(C.byref(params(prob)), _dp(S), _dp(J), _dp(U), _dp(R))
    return R


def rk_update(prob, stage, dt, R, U, dU):
    _load().orc_rk_update(C.byref(params(prob)), int(stage), float(dt), _dp(R), _dp(U), _dp(dU))


def rk_substep(prob, S, J, stage, dt, U, dU):
    _load().orc_rk_substep(C.byref(params(prob)), _dp(S), _dp(J), int(stage), float(dt), _dp(U), _dp(dU))


def compute_dt(prob, S, J, U, cfl):
    return _load().orc_compute_dt(C.byref(params(prob)), _dp(S), _dp(J), _dp(U), float(cfl))


def run(prob, S, J, U, nsteps, cfl=0.5, dt_fixed=0.0, t_end=0.0, t0=0.0, dU=None):
    """Advance U in place: BCs at the start, then nsteps (or until t_end)."""
    if dU is None:
        dU = np.zeros(int_shape(prob))
    t = C.c_double(t0)
    _load().orc_run(C.byref(params(prob)), _dp(S), _dp(J), _dp(U), _dp(dU), int(nsteps), float(cfl),
                    float(dt_fixed), float(t_end), C.byref(t))
    return t.value


def recon5(scheme, CT, eps, f):
    f = np.ascontiguousarray(f, dtype=np.float64)
    dl = np.zeros(3, dtype=np.intc)
    v = _load().orc_recon5(int(scheme), float(CT), float(eps), _dp(f), _ip(dl))
    return v, dl


def recon(scheme, CT, eps, f):
    """Reconstruction at x_{i+1/2} from f_{i-2..i+3} (six values); four
    cut-off flags (1 for stencils a scheme does not have)."""
    f = np.ascontiguousarray(f, dtype=np.float64)
    assert f.size == 6
    dl = np.zeros(4, dtype=np.intc)
    v = _load().orc_recon(int(scheme), float(CT), float(eps), _dp(f), _ip(dl))
    return v, dl


def recon_wenoz7(eps, f):
    """WENO-7Z at x_{i+1/2} from f_{i-3..i+3} (seven values)."""
    f = np.ascontiguousarray(f, dtype=np.float64)
    assert f.size == 7
    return _load().orc_recon_wenoz7(float(eps), _dp(f))


def smoothness7(f):
    """WENO-7Z indicators beta_0..beta_3 and candidates q_0..q_3 of f_{i-3..i+3}."""
    f = np.ascontiguousarray(f, dtype=np.float64)
    assert f.size == 7
    b = np.zeros(4)
    q = np.zeros(4)
    _load().orc_smoothness7(_dp(f), _dp(b), _dp(q))
    return b, q


def smoothness6(f):
    """TENO6 indicators beta_0..beta_3 and tau_6 of f_{i-2..i+3}."""
    f = np.ascontiguousarray(f, dtype=np.float64)
    b = np.zeros(4)
    tau = _load().orc_smoothness6(_dp(f), _dp(b))
    return b, tau


def rk_coeffs(prob):
    """(A, B) of the problem's low-storage RK scheme."""
    A = np.zeros(5)
    B = np.zeros(5)
    ns = np.zeros(1, dtype=np.intc)
    _load().orc_rk_coeffs(C.byref(params(prob)), _dp(A), _dp(B), _ip(ns))
    return A[: ns[0]], B[: ns[0]]


def smoothness5(f):
    f = np.ascontiguousarray(f, dtype=np.float64)
    b = np.zeros(3)
    _load().orc_smoothness5(_dp(f), _dp(b))
    return b


def iface_flux(prob, d, Uk, S):
    """Uk: (6, nc) stencil states at i-2..i+3; S: half-node area vector."""
    nc = prob.ndim + 2
    Uk = np.ascontiguousarray(Uk, dtype=np.float64).reshape(6 * nc)
    S3 = np.zeros(3)
    S3[: prob.ndim] = np.asarray(S, dtype=np.float64)[: prob.ndim]
    F = np.zeros(nc)
    dl = np.zeros(nc * 2 * 4, dtype=np.intc)
    _load().orc_iface_flux(C.byref(params(prob)), int(d), _dp(Uk), _dp(S3), _dp(F), _ip(dl))
    return F, dl.reshape(nc, 2, 4)


def phys_flux(prob, U, nv):
    nc = prob.ndim + 2
    U = np.ascontiguousarray(U, dtype=np.float64)
    n3 = np.zeros(3)
    n3[: prob.ndim] = np.asarray(nv, dtype=np.float64)[: prob.ndim]
    f = np.zeros(nc)
    _load().orc_phys_flux(C.byref(params(prob)), _dp(U), _dp(n3), _dp(f))
    return f


def eigen(prob, d, UL, UR, nv):
    nc = prob.ndim + 2
    n3 = np.zeros(3)
    n3[: prob.ndim] = np.asarray(nv, dtype=np.float64)[: prob.ndim]
    L = np.zeros((nc, nc))
    R = np.zeros((nc, nc))
    lam = np.zeros(nc)
    _load().orc_eigen(C.byref(params(prob)), int(d), _dp(np.ascontiguousarray(UL, dtype=np.float64)),
                      _dp(np.ascontiguousarray(UR, dtype=np.float64)), _dp(n3), _dp(L), _dp(R), _dp(lam))
    return L, R, lam


def deriv_line(f, periodic):
    f = np.ascontiguousarray(f, dtype=np.float64)
    out = np.zeros_like(f)
    _load().orc_deriv_line(_dp(f), f.size, int(bool(periodic)), _dp(out))
    return out


def deriv2_line(f, periodic):
    """Second-derivative operator along a line (unit spacing)."""
    f = np.ascontiguousarray(f, dtype=np.float64)
    out = np.zeros_like(f)
    _load().orc_deriv2_line(_dp(f), f.size, int(bool(periodic)), _dp(out))
    return out


def deriv_field(prob, a, d):
    a = np.ascontiguousarray(a, dtype=np.float64)
    out = np.zeros_like(a)
    _load().orc_deriv_field(C.byref(params(prob)), _dp(a), int(d), _dp(out))
    return out


def viscosity(prob, T):
    return _load().orc_viscosity(C.byref(params(prob)), float(T))


def num_threads():
    return int(_load().orc_num_threads())


def cheap_flux(prob, d, Uk, S):
    """Exact all-stencils-kept limit of the characteristic flux."""
    nc = prob.ndim + 2
    Uk = np.ascontiguousarray(Uk, dtype=np.float64).reshape(6 * nc)
    S3 = np.zeros(3)
    S3[: prob.ndim] = np.asarray(S, dtype=np.float64)[: prob.ndim]
    F = np.zeros(nc)
    _load().orc_cheap_flux(C.byref(params(prob)), int(d), _dp(Uk), _dp(S3), _dp(F))
    return F


def features(prob, d, Uk, S):
    """Ten sensor features and the TENO all-kept label of one interface."""
    nc = prob.ndim + 2
    Uk = np.ascontiguousarray(Uk, dtype=np.float64).reshape(6 * nc)
    S3 = np.zeros(3)
    S3[: prob.ndim] = np.asarray(S, dtype=np.float64)[: prob.ndim]
    f = np.zeros(10)
    lab = np.zeros(1, dtype=np.intc)
    _load().orc_features(C.byref(params(prob)), int(d), _dp(Uk), _dp(S3), _dp(f), _ip(lab))
    return f, int(lab[0])

