"""GPU tests of the two binding paths the step tests do not take:

* ``NSRollout`` -- the torch.autograd.Function over set / step / get whose
  backward calls ns_backward: ``torch.autograd.grad`` of the loss
  0.5 sum over the velocity unknowns of (u(T) - u_target)^2 against the
  oracle's FP64 reverse-mode gradient (1e-10) and against Solver.backward
  (bitwise: the same library calls).
* host pointers (``on_device = 0``) in ns_set_state, ns_get_state and
  ns_backward: bitwise equal to the device-pointer path, FP64 and FP32
  storage (the FP32 form converts host data through the staging buffer).
"""
import ctypes

import numpy as np
import pytest
import torch

import nsworkloads as W
import oracle
from tests import gpu_util as U

pytestmark = pytest.mark.gpu


def _adjoint_case(n=10, steps=4, k=2):
    prm = W.cavity(n, ny=n - 2, nz=n + 1, re=400.0, dt=0.005, tol=1e-13, itermax=20000)
    prm["checkpoint_every"] = k
    mk = [oracle.unknown_mask(prm, c) for c in range(3)]
    u0 = [np.where(mk[c], f, 0.0) for c, f in enumerate(W.gaussian_velocity(prm, 1e-2, 5))]
    tgt = [np.where(mk[c], f, 0.0) for c, f in enumerate(W.gaussian_velocity(prm, 1e-2, 6))]
    return prm, u0, tgt, mk, steps


def test_nsrollout_autograd_matches_oracle_gradient():
    from paper_1201_2118_amd.solver import NSRollout
    prm, u0, tgt, mk, steps = _adjoint_case()
    loss_o, grad_o, final_o = oracle.gradient(prm, *u0, tgt, steps)
    dev = torch.device("cuda:0")
    x = [torch.tensor(a, device=dev, requires_grad=True) for a in u0]
    masks = [torch.tensor(m, device=dev) for m in mk]
    tg = [torch.tensor(a, device=dev) for a in tgt]
    u, v, w = NSRollout.apply(x[0], x[1], x[2], prm, steps)
    loss = 0.5 * sum(torch.sum(torch.where(m, q - t, torch.zeros_like(q)) ** 2)
                     for q, t, m in zip((u, v, w), tg, masks))
    assert abs(loss.detach().item() - loss_o) <= 1e-10 * abs(loss_o)
    gx = torch.autograd.grad(loss, x)
    for c in range(3):
        g = gx[c].cpu().numpy()
        assert U.rel(g, grad_o[c], mk[c]) < 1e-10, c
        assert not np.any(g[~mk[c]])
    # the same library calls through Solver.backward give the same bits
    s = U.gpu_run(prm, steps, {"u": u0[0], "v": u0[1], "w": u0[2]})
    gf = [np.where(mk[c], s.get_np(f) - tgt[c], 0.0) for c, f in enumerate("uvw")]
    gs = [t.cpu().numpy() for t in s.backward(gf)]
    for c in range(3):
        assert np.array_equal(gs[c], gx[c].cpu().numpy()), c


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p).value


@pytest.mark.parametrize("form", ["fp64", "mixed"])
def test_host_pointer_state_paths_equal_device_paths(form):
    from paper_1201_2118_amd import abi
    from paper_1201_2118_amd.solver import Solver
    prm = dict(W.cavity(13, ny=11, nz=9, re=80.0, dt=0.004), precision=form)
    init = U.random_state(prm, 21, amp=0.2)
    # a: device pointers (Solver.set / get); b: host pointers through the ABI
    a = Solver(prm)
    b = Solver(prm)
    for name, arr in init.items():
        a.set(name, arr)
        src = np.ascontiguousarray(arr, dtype=np.float64)
        abi.check(abi.ns_set_state(b.handle, 0, abi.FIELD_IDS[name], _ptr(src), 0), b.handle)
    for name in "uvwp":
        h = np.full(W.shape(prm), np.nan)
        abi.check(abi.ns_get_state(b.handle, 0, abi.FIELD_IDS[name], _ptr(h), 0), b.handle)
        assert np.array_equal(h, a.get_np(name)), name
    a.step(3)
    b.step(3)
    assert a.stats()["sweeps_total"] == b.stats()["sweeps_total"]
    for name in ("u", "v", "w", "p", "F", "G", "H", "rhs"):
        h = np.full(W.shape(prm), np.nan)
        abi.check(abi.ns_get_state(b.handle, 0, abi.FIELD_IDS[name], _ptr(h), 0), b.handle)
        assert np.array_equal(h, a.get_np(name)), name
    # force fields never set read as zero through either path
    h = np.full(W.shape(prm), np.nan)
    abi.check(abi.ns_get_state(b.handle, 0, abi.NS_FX, _ptr(h), 0), b.handle)
    assert not np.any(h) and not np.any(a.get_np("fx"))


def test_host_pointer_backward_equals_device_backward():
    from paper_1201_2118_amd import abi
    prm, u0, tgt, mk, steps = _adjoint_case(n=9, steps=3, k=2)
    s = U.gpu_run(prm, steps, {"u": u0[0], "v": u0[1], "w": u0[2]})
    gf = [np.ascontiguousarray(np.where(mk[c], s.get_np(f) - tgt[c], 0.0)) for c, f in enumerate("uvw")]
    gd = [t.cpu().numpy() for t in s.backward(gf)]
    gh = [np.full(W.shape(prm), np.nan) for _ in range(3)]
    abi.check(abi.ns_backward(s.handle, 0, [_ptr(g) for g in gf], [_ptr(g) for g in gh], 0), s.handle)
    for c in range(3):
        assert np.array_equal(gh[c], gd[c]), c
    loss_o, grad_o, _ = oracle.gradient(prm, *u0, tgt, steps)
    for c in range(3):
        assert U.rel(gh[c], grad_o[c], mk[c]) < 1e-10, c


def test_bad_arguments_on_a_live_handle():
    """Argument errors on a live handle return NS_E_INVALID with a message and
    leave the handle usable: an instance out of range, an unknown field id,
    null data pointers, a negative step count, ns_backward without
    recording."""
    from paper_1201_2118_amd import abi
    from paper_1201_2118_amd.solver import Solver
    prm = W.cavity(10, ny=9, nz=8)
    s = Solver([prm, prm])
    h = s.handle
    t = torch.zeros(s.shape(), dtype=torch.float64, device="cuda:0")
    torch.cuda.synchronize()
    cases = [
        (lambda: abi.ns_set_state(h, 2, abi.NS_U, t.data_ptr(), 1), "instance out of range"),
        (lambda: abi.ns_get_state(h, -1, abi.NS_U, t.data_ptr(), 1), "instance out of range"),
        (lambda: abi.ns_set_state(h, 0, 99, t.data_ptr(), 1), "unknown field id"),
        (lambda: abi.ns_get_state(h, 1, -3, t.data_ptr(), 1), "unknown field id"),
        (lambda: abi.ns_set_state(h, 0, abi.NS_P, None, 1), "src is NULL"),
        (lambda: abi.ns_get_state(h, 0, abi.NS_P, None, 0), "dst is NULL"),
        (lambda: abi.ns_step(h, -1, None), "nsteps must be >= 0"),
    ]
    for call, msg in cases:
        assert call() == abi.NS_E_INVALID, msg
        assert msg in abi.ns_last_error(h), (msg, abi.ns_last_error(h))
    gi = [torch.zeros(s.shape(), dtype=torch.float64, device="cuda:0") for _ in range(3)]
    code = abi.ns_backward(h, 0, [g.data_ptr() for g in gi], [g.data_ptr() for g in gi], 1)
    assert code == abi.NS_E_INVALID, code  # no recording (checkpoint_every = 0)
    # still usable
    s.step(2)
    o, rc = U.oracle_run(prm, 2)
    assert rc == 0
    for i in range(2):
        assert s.stats(i)["sweeps_total"] == o.stats.sweeps_total
    s.close()
