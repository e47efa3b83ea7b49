"""ctypes binding of libosbli.so (the C ABI of include/osbli.h).

Argument marshalling only: every step of the method runs in the library's
HIP kernels.  The library must have been built in-tree
(``python -m paper_2007_14933_amd.build``); a missing library raises at load
time -- there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os
import threading

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libosbli.so")

OSBLI_OK, OSBLI_EINVAL, OSBLI_EDEVICE, OSBLI_ENONPHYS, OSBLI_ENOSPACE = 0, -1, -2, -3, -4
PERIODIC, EXTRAPOLATE, ISOTHERMAL_WALL, ADIABATIC_WALL, DIRICHLET = 0, 1, 2, 3, 4
WENOZ5, TENO5, TENO6, WENOJS5, WENOZ3, CENTRAL4, WENOZ7 = 0, 1, 2, 3, 4, 5, 6
RK3, RK3_SSP, RK4 = 0, 1, 2
FORM_FP64, FORM_MIXED = 0, 1
MESH_SEPARABLE, MESH_GENERAL = 0, 1


class OsbliError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("osbli error %d: %s" % (code, msg))
        self.code = code


class Params(C.Structure):
    _fields_ = [
        ("ndim", C.c_int32), ("mesh", C.c_int32),
        ("n", C.c_int64 * 3),
        ("gamma", C.c_double), ("Re", C.c_double), ("Pr", C.c_double), ("Minf", C.c_double),
        ("sutherland", C.c_int32), ("scheme", C.c_int32),
        ("Ts_over_Tref", C.c_double), ("teno_CT", C.c_double), ("eps", C.c_double),
        ("roe_avg", C.c_int32), ("form", C.c_int32), ("sensor", C.c_int32), ("rk", C.c_int32),
        ("bc_kind", (C.c_int32 * 2) * 3),
        ("wall_T", (C.c_double * 2) * 3),
        ("period", C.c_double * 3),
    ]


_lock = threading.Lock()
_lib = None

_VP = C.c_void_p
_DP = C.POINTER(C.c_double)
_SIGS = {
    "osbli_abi_version": (C.c_int, []),
    "osbli_workspace_bytes": (C.c_size_t, [C.POINTER(Params)]),
    "osbli_init_grid": (C.c_int, [C.POINTER(_VP), C.POINTER(Params), _DP, _DP, _DP, _VP, C.c_size_t, _VP]),
    "osbli_apply_bc": (C.c_int, [_VP, _VP, _VP]),
    "osbli_residual": (C.c_int, [_VP, _VP, _VP, _VP]),
    "osbli_rk_substep": (C.c_int, [_VP, C.c_int, C.c_double, _VP, _VP, _VP]),
    "osbli_rk_substep_noalloc": (C.c_int, [_VP, C.c_int, C.c_double, _VP, _VP, _VP]),
    "osbli_noalloc_scratch_bytes": (C.c_size_t, []),
    "osbli_rk_stages": (C.c_int, [_VP]),
    "osbli_central_store_all_bytes": (C.c_size_t, [C.POINTER(Params)]),
    "osbli_central_store_all": (C.c_int, [_VP, _VP, C.c_size_t]),
    "osbli_rk_coeffs": (C.c_int, [_VP, _DP, _DP]),
    "osbli_compute_dt": (C.c_int, [_VP, _VP, C.c_double, _DP, _VP]),
    "osbli_check": (C.c_int, [_VP]),
    "osbli_last_error": (C.c_char_p, [_VP]),
    "osbli_destroy": (None, [_VP]),
    "osbli_profile_enable": (C.c_int, [_VP, C.c_int]),
    "osbli_profile_read": (C.c_int, [_VP, C.c_int, C.POINTER(C.c_int64), _DP]),
    "osbli_sensor_set_weights": (C.c_int, [_VP, _VP, C.c_int, C.c_double, C.c_int, C.c_int, _VP]),
    "osbli_sensor_update": (C.c_int, [_VP, _VP, _VP]),
    "osbli_sensor_stats": (C.c_int, [_VP, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
    "osbli_sensor_masks": (C.c_int, [_VP, C.c_int, _VP, C.c_int64, _VP]),
    "osbli_interface_count": (C.c_int, [_VP, C.POINTER(C.c_int64)]),
    "osbli_collect_labels": (C.c_int, [_VP, _VP, _VP, _VP, C.c_int64, C.POINTER(C.c_int64), _VP]),
    "osbli_mlp_workspace_bytes": (C.c_size_t, [C.c_int64]),
    "osbli_mlp_grad": (C.c_int, [_VP, _VP, C.c_int64, _VP, C.c_float, _VP, _VP, _VP, C.c_size_t, _VP]),
    "osbli_mlp_adam": (C.c_int, [_VP, _VP, _VP, _VP, _VP, C.c_int64, C.c_float, C.c_float, C.c_float, C.c_float, _VP]),
    "osbli_mlp_forward": (C.c_int, [_VP, C.c_int64, _VP, _VP, C.c_int, _VP]),
    "osbli_set_sweep_segments": (C.c_int, [_VP, C.POINTER(C.c_int64)]),
    "osbli_batch_workspace_bytes": (C.c_size_t, [C.c_int]),
    "osbli_batch_create": (C.c_int, [C.POINTER(_VP), C.POINTER(_VP), C.c_int, C.POINTER(_VP), C.POINTER(_VP), _DP,
                                     C.c_double, _VP, C.c_size_t, _VP]),
    "osbli_batch_set_tiles": (C.c_int, [_VP, C.POINTER(C.c_int64), _VP]),
    "osbli_batch_set_grid": (C.c_int, [_VP, C.c_int]),
    "osbli_batch_capture": (C.c_int, [_VP, _VP]),
    "osbli_batch_step": (C.c_int, [_VP, _VP]),
    "osbli_batch_substep": (C.c_int, [_VP, C.c_int, _VP]),
    "osbli_batch_status": (C.c_int, [_VP, _DP, C.POINTER(C.c_int), C.POINTER(C.c_int), _VP]),
    "osbli_batch_interior_points": (C.c_int, [_VP, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
    "osbli_batch_last_error": (C.c_char_p, [_VP]),
    "osbli_batch_destroy": (None, [_VP]),
}

K_SWEEP_X, K_SWEEP_Y, K_SWEEP_Z, K_VISC_FLUX, K_FINISH, K_BC, K_DT, K_SENSOR, K_CENTRAL = range(9)
K_NAMES = ["sweep_x", "sweep_y", "sweep_z", "visc_flux", "finish", "bc", "dt", "sensor", "central"]


def load():
    """Load libosbli.so (raises if it has not been built).

    torch is imported first so that its HIP runtime is the one in the process:
    the library and torch then share one runtime (same SONAME), hence one set
    of streams and allocations."""
    global _lib
    with _lock:
        if _lib is None:
            import torch  # noqa: F401  (loads the process's HIP runtime first)
            if not os.path.exists(LIB_PATH):
                raise ImportError("libosbli.so not built: run `python -m paper_2007_14933_amd.build`")
            lib = C.CDLL(LIB_PATH)
            for name, (res, args) in _SIGS.items():
                fn = getattr(lib, name)
                fn.restype = res
                fn.argtypes = args
            _lib = lib
    return _lib


def exported_symbols():
    return list(_SIGS)


def make_params(prob, form=FORM_FP64, sensor=0) -> Params:
    p = Params()
    p.ndim = int(prob.ndim)
    p.mesh = MESH_SEPARABLE if prob.coords1d is not None else MESH_GENERAL
    for d in range(3):
        p.n[d] = int(prob.n[d]) if d < prob.ndim else 1
        p.period[d] = float(prob.period[d])
        for s in range(2):
            p.bc_kind[d][s] = int(prob.bc[d][s])
            p.wall_T[d][s] = float(prob.wall_T[d][s])
    p.gamma, p.Re, p.Pr, p.Minf = float(prob.gamma), float(prob.Re), float(prob.Pr), float(prob.Minf)
    p.sutherland = int(prob.sutherland)
    p.Ts_over_Tref = float(prob.Ts_over_Tref)
    p.scheme = int(prob.scheme)
    p.teno_CT = float(prob.teno_CT)
    p.eps = float(prob.eps)
    p.roe_avg = int(prob.roe_avg)
    p.rk = int(getattr(prob, "rk", RK3))
    p.form = int(form)
    p.sensor = int(sensor)
    return p


def check_batch(code, batch):
    if code != OSBLI_OK:
        msg = load().osbli_batch_last_error(batch).decode() if batch else "(no batch)"
        raise OsbliError(code, msg)
    return code


def check(code, ctx=None):
    if code != OSBLI_OK:
        msg = load().osbli_last_error(ctx).decode() if ctx else "(no context)"
        raise OsbliError(code, msg)
    return code
