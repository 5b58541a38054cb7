"""Host-side checks of the C ABI that need no GPU: the library loads, it
exports every symbol include/dgsw.h declares, and descriptor validation
rejects bad meshes before any device call."""
import ctypes
import os
import re

import pytest

from paper_2303_11767_amd import _lib

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "dgsw.h")


def header_functions():
    src = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int|const char \*)\s*(dg_\w+)\s*\(", src, re.M)))


def test_header_and_binding_agree():
    assert header_functions() == sorted(_lib.EXPORTS)


def test_header_constants_match_binding():
    """Every enumerator the header defines has the same value in the binding."""
    src = open(HEADER).read()
    found = 0
    for body in re.findall(r"enum\s*\{([^}]*)\}", src):
        for name, val in re.findall(r"(DG_\w+)\s*=\s*(-?\d+)", body):
            if hasattr(_lib, name):
                assert getattr(_lib, name) == int(val), name
                found += 1
    assert found >= 10
    assert _lib.DG_RK4 == 4


def test_library_exports_every_declared_symbol():
    lib = _lib.load()
    for name in header_functions():
        assert hasattr(lib, name), name


def _desc(**kw):
    d = _lib.MeshDesc()
    d.abi_version, d.n_lon, d.n_lat, d.order = 1, 8, 4, 2
    d.dtype, d.metric, d.alpha_mode, d.reserved = 0, 0, 0, 0
    d.alpha, d.radius, d.gravity, d.omega, d.h_ref = 0.0, 6.371e6, 9.80616, 7.292e-5, 0.0
    for k, v in kw.items():
        setattr(d, k, v)
    return d


@pytest.mark.parametrize("kw,code", [
    ({"abi_version": 2}, -1), ({"n_lon": 0}, -1), ({"n_lat": -3}, -1), ({"order": -1}, -1),
    ({"order": 8}, -6), ({"dtype": 7}, -2), ({"metric": 5}, -1), ({"alpha_mode": 3}, -1),
    ({"reserved": 1}, -1), ({"radius": 0.0}, -1), ({"gravity": -1.0}, -1),
    ({"omega": float("nan")}, -1), ({"h_ref": -1.0}, -1),
    ({"h_ref": 100.0, "metric": 1}, -1), ({"alpha_mode": 1, "alpha": -2.0}, -1),
    ({"n_lon": 70000, "n_lat": 70000}, -1),
])
def test_descriptor_validation(kw, code):
    lib = _lib.load()
    ctx = ctypes.c_void_p(123)
    d = _desc(**kw)
    rc = lib.dg_init_mesh(ctypes.byref(d), None, ctypes.byref(ctx))
    assert rc == code
    assert ctx.value is None
    assert len(lib.dg_last_error()) > 0


def _plane(**kw):
    d = _lib.PlaneDesc()
    d.abi_version, d.nx, d.ny, d.order, d.dtype, d.alpha_mode = 1, 8, 6, 3, 0, 0
    d.alpha, d.lx, d.ly, d.gravity, d.f, d.h_ref = 0.0, 1e7, 1e7, 9.81, 1e-4, 0.0
    for k, v in kw.items():
        setattr(d, k, v)
    return d


@pytest.mark.parametrize("kw,code", [
    ({"abi_version": 0}, -1), ({"nx": 0}, -1), ({"ny": -1}, -1), ({"order": 8}, -6),
    ({"dtype": 3}, -2), ({"alpha_mode": 2}, -1), ({"lx": 0.0}, -1), ({"ly": float("inf")}, -1),
    ({"gravity": 0.0}, -1), ({"f": float("nan")}, -1), ({"h_ref": -5.0}, -1),
])
def test_plane_descriptor_validation(kw, code):
    lib = _lib.load()
    ctx = ctypes.c_void_p(123)
    rc = lib.dg_init_plane(ctypes.byref(_plane(**kw)), None, ctypes.byref(ctx))
    assert rc == code
    assert ctx.value is None
    assert len(lib.dg_last_error()) > 0


@pytest.mark.parametrize("kw,code", [
    ({"abi_version": 0}, -1), ({"nx": 0}, -1), ({"order": 7}, -6), ({"order": -1}, -1),
    ({"dtype": 2}, -2), ({"reserved": 1}, -1), ({"lx": 0.0}, -1), ({"by": float("nan")}, -1),
])
def test_advection_descriptor_validation(kw, code):
    lib = _lib.load()
    d = _lib.AdvDesc()
    d.abi_version, d.nx, d.ny, d.order, d.dtype, d.reserved = 1, 8, 8, 3, 0, 0
    d.lx, d.ly, d.bx, d.by = 1.0, 1.0, 1.0, 1.0
    for k, v in kw.items():
        setattr(d, k, v)
    h = ctypes.c_void_p(123)
    assert lib.dg_adv_init(ctypes.byref(d), None, ctypes.byref(h)) == code
    assert h.value is None


def test_null_arguments():
    lib = _lib.load()
    assert lib.dg_init_mesh(None, None, None) == -1
    assert lib.dg_init_plane(None, None, None) == -1
    assert lib.dg_adv_init(None, None, None) == -1
    assert lib.dg_adv_free(None) == 0
    assert lib.dg_free(None) == 0
    n = ctypes.c_int64()
    assert lib.dg_state_size(None, ctypes.byref(n)) == -1
    assert lib.dg_rhs(None, None, None, None) == -1
    assert lib.dg_rk_step(None, None, None, 1.0, 3, 1, None) == -1
    out = (ctypes.c_double * 3)()
    assert lib.dg_mass(None, None, out, None) == -1
    assert lib.dg_set_forcing(None, None) == -1
    assert lib.dg_set_levels(None, 2) == -1
    assert lib.dg_autotune(None, None, None, None, None) == -1
    k = ctypes.c_int32()
    assert lib.dg_get_levels(None, ctypes.byref(k)) == -1
