"""The two-stage SSP Runge-Kutta (Heun) integrator (NS_RK2) on the GPU
against the oracle's two-stage integrator: FP64 to 1e-12 with equal sweep
counts (both stages' solves), mixed precision to 1e-5; the closed-form
amplification of a viscous shear wave; the combinations with the advective
form and with the generated kernels."""
import math

import numpy as np
import pytest

import nsworkloads as W
from paper_1201_2118_amd import abi
from tests import gpu_util as U

pytestmark = pytest.mark.gpu

CASES = [
    (dict(nx=20, ny=16, nz=12), (0, 0, 0), 0.0),     # cavity, adaptive dt
    (dict(nx=16, ny=16, nz=8), (1, 1, 1), 2e-3),     # periodic box
    (dict(nx=18, ny=11, nz=14), (1, 0, 0), 1e-3),    # mixed boundaries
    (dict(nx=70, ny=37, nz=19), (0, 0, 0), 2e-3),    # several tiles, ragged
]


def _prm(dims, bc, dt, precision="fp64", **kw):
    prm = W.cavity(dims["nx"], ny=dims["ny"], nz=dims["nz"], re=80.0, dt=dt, gamma=0.3, tau=0.5)
    prm.update(bc=bc, integrator="rk2", precision=precision, **kw)
    prm["wall_vel"][5] = [1.0, 0.2, 0.0]
    return prm


@pytest.mark.parametrize("dims,bc,dt", CASES)
def test_rk2_matches_oracle_fp64(dims, bc, dt):
    prm = _prm(dims, bc, dt)
    init = U.random_state(prm, 11, amp=0.2)
    s = U.gpu_run(prm, 3, init)
    o, rc = U.oracle_run(prm, 3, init)
    assert rc == 0
    st = s.stats()
    assert st["sweeps_total"] == o.stats.sweeps_total
    assert st["steps"] == 3 == o.stats.steps
    assert abs(st["t"] - o.stats.t) <= 1e-15 * max(o.stats.t, 1e-300)
    assert st["steps_unconverged"] == o.stats.steps_unconverged
    U.compare_state(s, o, prm, 1e-12)


@pytest.mark.parametrize("dims,bc,dt", CASES[:3])
def test_rk2_mixed_matches_oracle(dims, bc, dt):
    prm = _prm(dims, bc, dt, precision="mixed")
    init = U.random_state(prm, 12, amp=0.2)
    s = U.gpu_run(prm, 3, init)
    o, rc = U.oracle_run(dict(prm, precision="fp64"), 3, init, mode=1)
    assert rc == 0
    m = U.masks(prm)
    sc = U.velocity_scale([o.field(f) for f in "uvw"], prm)
    for c, f in enumerate("uvw"):
        assert U.vel_rel(s.get_np(f), o.field(f), m[c], sc) < 1e-5, f


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_rk2_shear_wave_amplification(precision):
    """u = A sin(2 pi z) in a periodic box: no convection, zero rhs; each step
    multiplies A by 1 - z + z^2/2, z = dt nu (2 - 2 cos(2 pi h)) / h^2."""
    n = 32
    prm = W.periodic_box(4, nz=n, re=10.0, dt=1e-3, gamma=0.5)
    prm.update(integrator="rk2", precision=precision, tol=1e-12)
    _, _, z = W.coords(prm, 0)
    s_ = np.sin(2 * math.pi * z)
    zero = np.zeros(W.shape(prm))
    s = U.gpu_run(prm, 20, {"u": 0.5 * s_, "v": zero, "w": zero, "p": zero})
    h = 1.0 / n
    zz = prm["dt"] / prm["re"] * (2.0 - 2.0 * math.cos(2 * math.pi * h)) / (h * h)
    expect = 0.5 * (1.0 - zz + zz * zz / 2.0) ** 20 * s_
    m = U.masks(prm)
    bar = 1e-13 if precision == "fp64" else 2e-6
    assert np.abs(s.get_np("u")[m[0]] - expect[m[0]]).max() <= bar * 0.5
    assert s.stats()["sweeps_total"] == 0


def test_rk2_advective_matches_oracle():
    prm = dict(_prm(dict(nx=14, ny=12, nz=10), (0, 1, 0), 2e-3), convection="advective")
    init = U.random_state(prm, 13, amp=0.2)
    s = U.gpu_run(prm, 2, init)
    o, rc = U.oracle_run(prm, 2, init)
    assert rc == 0 and s.stats()["sweeps_total"] == o.stats.sweeps_total
    U.compare_state(s, o, prm, 1e-12)


def test_rk2_generated_equals_hand_written():
    prm = _prm(dict(nx=30, ny=10, nz=9), (0, 0, 0), 2e-3)
    init = U.random_state(prm, 14, amp=0.2)
    a = U.gpu_run(prm, 2, init)
    b = U.gpu_run(dict(prm, flags=abi.NS_GENERATED), 2, init)
    assert a.stats()["sweeps_total"] == b.stats()["sweeps_total"]
    m = U.masks(prm)
    sc = U.velocity_scale([a.get_np(f) for f in "uvw"], prm)
    for c, f in enumerate("uvw"):
        assert U.vel_rel(b.get_np(f), a.get_np(f), m[c], sc) <= 1e-13, f
