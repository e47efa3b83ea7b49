"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every symbol the public header declares, sizes its workspace, and rejects
invalid parameters before any device call."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2007_14933_amd import binding as B
from paper_2007_14933_amd import inputs as I

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    txt = open(os.path.join(ROOT, "include", "osbli.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(osbli_[a-z_0-9]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(B.LIB_PATH):
        from paper_2007_14933_amd import build
        build.build()
    return B.load()


def test_exports_every_declared_symbol(lib):
    names = header_functions()
    assert "osbli_rk_substep" in names and "osbli_init_grid" in names
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) <= set(B.exported_symbols()) | {"osbli_abi_version"}
    assert lib.osbli_abi_version() == 1


def test_params_struct_matches_header_layout(lib):
    # the ctypes mirror must have the size the C compiler gives the struct
    assert C.sizeof(B.Params) == 8 + 24 + 32 + 8 + 24 + 16 + 24 + 48 + 24


def _ws(prob, **kw):
    p = B.make_params(prob, **kw)
    return B.load().osbli_workspace_bytes(C.byref(p))


def test_workspace_sizes(lib):
    tgv = I.tgv(16)
    n = 16 ** 3
    ws = _ws(tgv)
    # residual accumulator 5n + viscous fluxes 9n doubles (separable mesh:
    # six distinct stresses and three energy fluxes), plus small tables
    assert ws >= 8 * (5 * n + 9 * n)
    assert ws < 8 * (5 * n + 9 * n) + 64 * 1024
    sod = I.sod(400)
    assert 8 * 3 * 400 <= _ws(sod) < 64 * 1024


@pytest.mark.parametrize("mutate,why", [
    (lambda p: setattr(p, "ndim", 4), "ndim"),
    (lambda p: p.bc_kind[0].__setitem__(1, B.EXTRAPOLATE), "periodic on one side"),
    (lambda p: p.n.__setitem__(0, 5), "too few periodic nodes"),
    (lambda p: setattr(p, "scheme", 7), "scheme"),
    (lambda p: setattr(p, "gamma", 1.0), "gamma"),
    (lambda p: setattr(p, "teno_CT", 0.5), "C_T"),
    (lambda p: setattr(p, "form", 9), "form"),
    (lambda p: setattr(p, "eps", 1e-60), "eps below the range whose sixth power stays normal"),
    (lambda p: setattr(p, "eps", 0.0), "eps zero"),
    (lambda p: (setattr(p, "scheme", B.TENO6), setattr(p, "teno_CT", 0.3)), "TENO6 needs C_T < 1/4"),
    (lambda p: (setattr(p, "scheme", B.TENO6), setattr(p, "form", B.FORM_MIXED)), "precision form: fifth order only"),
    (lambda p: (setattr(p, "scheme", B.WENOJS5), setattr(p, "sensor", 1)), "routing needs TENO5"),
    (lambda p: setattr(p, "rk", 3), "Runge-Kutta scheme"),
    (lambda p: setattr(p, "scheme", 7), "scheme past WENO-7Z"),
    (lambda p: (setattr(p, "scheme", B.WENOZ7), setattr(p, "form", B.FORM_MIXED)), "precision form: WENO-7Z"),
    (lambda p: (setattr(p, "scheme", B.WENOZ7), setattr(p, "sensor", 1)), "routing needs TENO5 (WENO-7Z)"),
    (lambda p: (setattr(p, "scheme", B.WENOZ7), setattr(p, "mesh", B.MESH_GENERAL)), "WENO-7Z general mesh"),
    (lambda p: (setattr(p, "scheme", B.WENOZ7), p.bc_kind[1].__setitem__(0, B.ISOTHERMAL_WALL),
                p.bc_kind[1].__setitem__(1, B.ISOTHERMAL_WALL)), "WENO-7Z with walls"),
    (lambda p: (p.bc_kind[0].__setitem__(0, 5), p.bc_kind[0].__setitem__(1, 5)), "bc kind"),
])
def test_invalid_parameters_rejected_without_device(lib, mutate, why):
    p = B.make_params(I.tgv(8))
    mutate(p)
    assert lib.osbli_workspace_bytes(C.byref(p)) == 0, why
    ctx = C.c_void_p()
    rc = lib.osbli_init_grid(C.byref(ctx), C.byref(p), None, None, None, None, 0, None)
    assert rc == B.OSBLI_EINVAL
    assert lib.osbli_last_error(ctx)
    lib.osbli_destroy(ctx)


def test_too_few_wall_nodes_rejected(lib):
    p = B.make_params(I.laminar_channel(8, 9))
    p.n[1] = 4
    ctx = C.c_void_p()
    assert lib.osbli_init_grid(C.byref(ctx), C.byref(p), None, None, None, None, 0, None) == B.OSBLI_EINVAL
    assert b"below" in lib.osbli_last_error(ctx)
    lib.osbli_destroy(ctx)


@pytest.mark.parametrize("why", ["non-uniform", "period"])
def test_central_path_needs_uniform_spacing(lib, why):
    """The central path's expanded second derivatives assume uniform spacing:
    a stretched mesh (or a period other than n h) is refused at set-up, on
    the host, before any device call."""
    prob = I.tgv(8, scheme=I.CENTRAL4)
    p = B.make_params(prob)
    x = np.ascontiguousarray(prob.coords1d[0], dtype=np.float64).copy()
    if why == "non-uniform":
        x[3] += 1e-3
    else:
        p.period[0] = 1.01 * p.period[0]
    xs = [x.ctypes.data_as(C.POINTER(C.c_double))] + [
        np.ascontiguousarray(prob.coords1d[d]).ctypes.data_as(C.POINTER(C.c_double)) for d in (1, 2)]
    need = lib.osbli_workspace_bytes(C.byref(p))
    ctx = C.c_void_p()
    rc = lib.osbli_init_grid(C.byref(ctx), C.byref(p), *xs, C.c_void_p(256), need, None)
    assert rc == B.OSBLI_EINVAL and b"central path" in lib.osbli_last_error(ctx)
    lib.osbli_destroy(ctx)


def test_central_store_all_sizes(lib):
    p = B.make_params(I.tgv(16, scheme=I.CENTRAL4))
    n = 16 ** 3
    # F 15, G 18, S 12, X 9, Y 9 arrays of n doubles
    assert lib.osbli_central_store_all_bytes(C.byref(p)) == 8 * n * (15 + 18 + 12 + 9 + 9)
    assert lib.osbli_central_store_all_bytes(C.byref(B.make_params(I.tgv(16)))) == 0


def test_small_workspace_rejected(lib):
    prob = I.sod(50)
    p = B.make_params(prob)
    need = lib.osbli_workspace_bytes(C.byref(p))
    ctx = C.c_void_p()
    x = (C.c_double * 50)()
    rc = lib.osbli_init_grid(C.byref(ctx), C.byref(p), x, None, None, C.c_void_p(256), need - 8, None)
    assert rc == B.OSBLI_ENOSPACE
    lib.osbli_destroy(ctx)


def _gpu_test_problems():
    """Every problem the GPU tests construct, as (name, problem, form, sensor)."""
    import sys
    here = os.path.dirname(os.path.abspath(__file__))
    sys.path.insert(0, here)
    import test_gpu_batch as TB
    import test_gpu_forms as TF
    import test_gpu_parity as TP
    out = []
    for name, mk in TP.X_SWEEP_CASES.items():
        for form in (0, 1):
            out.append((name, mk(), form, 0))
    for name, (mk, _, _) in TF.CASES.items():
        out.append((name, mk(), 1, 0))
    for sensor in (0, 1):
        for p in TB.ensemble(TB.SIZES, 11, TB.T_ENDS):
            out.append((p.name, p, 1, sensor))
    out.append(("sod80_teno", I.sod(80).with_(scheme=I.TENO5), 0, 1))
    import test_gpu_schemes as TS
    for name, (prob, _) in TS.CASES.items():
        out.append((name, prob, 0, 0))
    import test_gpu_central as TC
    for name, (prob, _) in TC.CASES.items():
        out.append((name, prob, 0, 0))
    return out


def test_gpu_test_problems_are_valid_parameters(lib):
    """The parameter check of osbli_workspace_bytes runs on the host: every
    grid the GPU tests build must pass it (a size or BC mistake in a test
    then shows here, without a GPU)."""
    for name, prob, form, sensor in _gpu_test_problems():
        p = B.make_params(prob, form=form, sensor=sensor)
        assert lib.osbli_workspace_bytes(C.byref(p)) > 0, (name, form, sensor)
