"""Host-side checks of the C ABI library (no GPU needed): it loads, exports
every entry point include/*.h declares, its ns_params layout matches the
binding, and parameter validation rejects bad or unstable input before any
device call."""
import ctypes
import os
import re
import subprocess

import pytest

import nsworkloads as W
from paper_1201_2118_amd import abi
from paper_1201_2118_amd.solver import make_params

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    names = set()
    inc = os.path.join(ROOT, "include")
    for f in os.listdir(inc):
        if f.endswith(".h"):
            src = open(os.path.join(inc, f)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            names |= set(re.findall(r"\b(ns_[a-z_]+)\s*\(", src))
    return names


def test_library_exports_every_declared_symbol():
    lib = abi.load()
    declared = _declared_symbols()
    assert {"ns_create", "ns_set_state", "ns_step", "ns_get_state", "ns_backward"} <= declared
    for name in declared:
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", abi.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (ns_[a-z_]+)\b", out))
    assert declared <= exported
    assert set(abi.EXPORTED) == declared


def test_library_is_gfx950_only():
    """Every device code object in our own build targets gfx950."""
    blob = open(abi.LIB_PATH, "rb").read()
    targets = set(re.findall(rb"amdgcn-amd-amdhsa--(gfx[0-9a-z]+)", blob))
    assert targets == {b"gfx950"}, targets


def test_params_layout_and_defaults():
    p = abi.ns_params()
    assert abi.ns_params_default(p) == abi.NS_OK
    assert p.struct_size == ctypes.sizeof(abi.ns_params)
    assert (p.nx, p.ny, p.nz) == (16, 16, 16)
    assert p.re == 100.0 and p.dt == 0.01 and p.gamma == 0.5 and p.omega == 1.7
    assert p.tol == 1e-6 and p.itermax == 200 and p.wall_vel[5][0] == 1.0
    assert abi.load().ns_params_default(None) == abi.NS_E_INVALID


def _create(prm, flags=0, edit=None):
    p = make_params(dict(prm, flags=flags))
    if edit:
        edit(p)
    h = ctypes.c_void_p()
    arr = (abi.ns_params * 1)(p)
    code = abi.ns_create(arr, 1, None, h)
    return code, h


@pytest.mark.parametrize("edit,msg", [
    (lambda p: setattr(p, "nx", 1), "at least 2"),
    (lambda p: setattr(p, "omega", 2.0), "omega"),
    (lambda p: setattr(p, "omega", 0.0), "omega"),
    (lambda p: setattr(p, "re", -1.0), "re"),
    (lambda p: setattr(p, "gamma", 1.5), "gamma"),
    (lambda p: setattr(p, "itermax", -1), "itermax"),
    (lambda p: setattr(p, "precision", 7), "precision"),
    (lambda p: setattr(p, "struct_size", 8), "struct_size"),
    (lambda p: setattr(p, "tol", float("nan")), "tol"),
    (lambda p: p.tile.__setitem__(0, 20), "tile[0]"),
    (lambda p: p.tile.__setitem__(0, 24), "16 rows"),
    (lambda p: (p.tile.__setitem__(0, 16), p.bc.__setitem__(2, 1), setattr(p, "nz", 2)), "at least 4 cells"),
    (lambda p: (p.tile.__setitem__(0, 8), setattr(p, "nx", 24000), setattr(p, "ny", 24000), setattr(p, "nz", 2)),
     "unfused"),
])
def test_invalid_parameters_are_rejected(edit, msg):
    code, h = _create(W.cavity(8), edit=edit)
    assert code == abi.NS_E_INVALID
    assert msg in abi.ns_last_error(None)
    assert not h.value


def test_periodic_axis_needs_even_size():
    prm = W.periodic_box(8, nz=5)
    code, _ = _create(prm)
    assert code == abi.NS_E_INVALID and "even" in abi.ns_last_error(None)


def test_recording_needs_fp64_and_fixed_dt():
    code, _ = _create(dict(W.cavity(8), precision="mixed", checkpoint_every=2))
    assert code == abi.NS_E_INVALID
    code, _ = _create(dict(W.cavity(8, dt=0.0), checkpoint_every=2))
    assert code == abi.NS_E_INVALID


@pytest.mark.parametrize("prm", [W.cavity(128, dt=0.01), W.cavity(512, re=1000.0, dt=0.002)])
def test_literal_unstable_steps_are_refused(prm):
    """128^3 with dt 0.01 (diffusion number 4.9) and 512^3 with dt 0.002
    (1.57) exceed the explicit bound of 1/2."""
    code, _ = _create(prm)
    assert code == abi.NS_E_UNSTABLE
    assert "NS_ALLOW_UNSTABLE" in abi.ns_last_error(None)


def test_null_arguments():
    lib = abi.load()
    assert lib.ns_create(None, 1, None, None) == abi.NS_E_INVALID
    assert lib.ns_step(None, 1, None) == abi.NS_E_INVALID
    assert lib.ns_set_state(None, 0, 0, None, 0) == abi.NS_E_INVALID
    assert lib.ns_get_state(None, 0, 0, None, 0) == abi.NS_E_INVALID
    lib.ns_destroy(None)


def test_noalloc_step_validates_before_any_device_call():
    """ns_step_noalloc rejects bad arguments and grids beyond its static
    scratch on the host, before it touches a device."""
    prm = W.cavity(80, ny=80, nz=80, dt=5e-4)  # 82^3 padded entries > 524288
    code = abi.ns_step_noalloc(make_params(prm), 1, 1, 1, 1, 1, None, None)
    assert code == abi.NS_E_INVALID and "static scratch" in abi.ns_last_error(None)
    for edit in (dict(precision="mixed"), dict(checkpoint_every=2), dict(flags=abi.NS_TIMING)):
        code = abi.ns_step_noalloc(make_params(dict(W.cavity(8), **edit)), 1, 1, 1, 1, 1, None, None)
        assert code == abi.NS_E_INVALID, edit
    code = abi.ns_step_noalloc(make_params(W.cavity(8)), 0, 1, 1, 1, 1, None, None)
    assert code == abi.NS_E_INVALID
    code = abi.ns_step_noalloc(make_params(W.cavity(8)), 1, 1, 1, 1, -1, None, None)
    assert code == abi.NS_E_INVALID


def test_advective_form_refuses_unsupported_combinations():
    """NS_ADVECTIVE: one instance, not with recording for the adjoint
    (host-side validation)."""
    prm = dict(W.cavity(8), convection="advective")
    assert _create(dict(prm, checkpoint_every=2))[0] == abi.NS_E_INVALID
    arr = (abi.ns_params * 2)(make_params(prm), make_params(prm))
    h = ctypes.c_void_p()
    assert abi.ns_create(arr, 2, None, h) == abi.NS_E_INVALID
    assert "one instance" in abi.ns_last_error(None)


def test_rk2_refuses_unsupported_combinations():
    """NS_RK2: one instance, not with recording for the adjoint, not through
    ns_step_noalloc (host-side validation); an unknown integrator name is
    refused by the binding."""
    prm = dict(W.cavity(8), integrator="rk2")
    assert make_params(prm).flags & abi.NS_RK2
    assert _create(dict(prm, checkpoint_every=2))[0] == abi.NS_E_INVALID
    assert "NS_RK2" in abi.ns_last_error(None)
    arr = (abi.ns_params * 2)(make_params(prm), make_params(prm))
    h = ctypes.c_void_p()
    assert abi.ns_create(arr, 2, None, h) == abi.NS_E_INVALID
    assert "one instance" in abi.ns_last_error(None)
    code = abi.ns_step_noalloc(make_params(prm), 1, 1, 1, 1, 1, None, None)
    assert code == abi.NS_E_INVALID and "Euler" in abi.ns_last_error(None)
    with pytest.raises(ValueError):
        make_params(dict(W.cavity(8), integrator="rk4"))
