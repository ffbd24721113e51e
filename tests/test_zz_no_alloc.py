"""ns_step_noalloc (the allocation-free step over caller-owned FP64 fields,
scratch in one static device array) against the handle path
ns_create + ns_set_state + ns_step + ns_get_state, through the C ABI.

Two calls in a row on the same device, the second on a smaller grid with
other parameters, so the second call starts from the scratch contents the
first one left.  Bar: FP64 1e-12 relative (the same kernels and sweep
shapes run on both paths) with equal sweep counts.
"""
import ctypes

import numpy as np
import pytest
import torch

import nsworkloads as W
from tests import gpu_util as U

pytestmark = pytest.mark.gpu


def _noalloc(prm, init, nsteps):
    from paper_1201_2118_amd import abi
    from paper_1201_2118_amd.solver import make_params
    dev = torch.device("cuda:0")
    f = {k: torch.tensor(init[k], dtype=torch.float64, device=dev).contiguous() for k in "uvwp"}
    st = abi.ns_stats()
    torch.cuda.synchronize()
    code = abi.ns_step_noalloc(make_params(prm), f["u"].data_ptr(), f["v"].data_ptr(), f["w"].data_ptr(),
                               f["p"].data_ptr(), nsteps, torch.cuda.current_stream(dev).cuda_stream, st)
    if code != abi.NS_OK:
        raise abi.NSError(code, abi.ns_last_error(None))
    return {k: t.cpu().numpy() for k, t in f.items()}, st.as_dict()


def _handle(prm, init, nsteps):
    s = U.gpu_run(prm, nsteps, init)
    out = {k: s.get_np(k) for k in "uvwp"}
    st = s.stats()
    s.close()
    return out, st


def _compare(a, b, prm):
    m = U.masks(prm)
    scale = U.velocity_scale([b[k] for k in "uvw"], prm)
    errs = {k: U.vel_rel(a[k], b[k], m[c], scale) for c, k in enumerate("uvw")}
    errs["p"] = U.pressure_rel(a["p"], b["p"], m[3])
    return errs


def test_noalloc_step_equals_handle_step_two_calls():
    cases = [
        (dict(W.cavity(40, ny=36, nz=30, re=150.0, dt=0.004), tile=(16, 0)), 4, 31),
        (dict(W.cavity(20, ny=18, nz=12, re=60.0, dt=0.0, tau=0.5), gamma=0.3), 3, 32),
    ]
    for prm, nsteps, seed in cases:
        init = U.random_state(prm, seed, amp=0.2)
        a, sa = _noalloc(prm, init, nsteps)
        b, sb = _handle(prm, init, nsteps)
        assert sa["steps"] == sb["steps"] == nsteps
        assert sa["sweeps_total"] == sb["sweeps_total"], (sa, sb)
        assert sa["t"] == sb["t"]
        errs = _compare(a, b, prm)
        print(f"{prm['nx']}x{prm['ny']}x{prm['nz']}: noalloc vs handle {errs}", flush=True)
        assert max(errs.values()) < 1e-12, errs


def test_noalloc_rejects_oversize_and_host_pointers():
    from paper_1201_2118_amd import abi
    from paper_1201_2118_amd.solver import make_params
    big = W.cavity(80, ny=80, nz=80, dt=5e-4)  # 82^3 > 524288 padded entries
    dev = torch.device("cuda:0")
    t = torch.zeros(1, dtype=torch.float64, device=dev)
    code = abi.ns_step_noalloc(make_params(big), t.data_ptr(), t.data_ptr(), t.data_ptr(), t.data_ptr(), 1,
                               None, None)
    assert code == abi.NS_E_INVALID and "static scratch" in abi.ns_last_error(None)
    small = W.cavity(8)
    h = np.zeros(W.shape(small))
    hp = h.ctypes.data_as(ctypes.c_void_p).value
    code = abi.ns_step_noalloc(make_params(small), hp, hp, hp, hp, 1, None, None)
    assert code == abi.NS_E_INVALID and "memory of the current device" in abi.ns_last_error(None)
