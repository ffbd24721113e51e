"""The kernels generated from the kernel descriptors.

PREDICT_VELOCITY (3DSTREAM: streamed through z, the velocity in an LDS
plane ring) is the predictor of every single-domain handle; its F, G, H
equal, bit for bit, the hand-written predictor cells the batched launches
run (a two-domain handle, persistent or multi-launch, with no sweeps).
UPDATE_VELOCITY (3DBLOCK) replaces the hand-written projection under
NS_GENERATED: every field of the state and of the last predictor and rhs
equals the default step's bit for bit, FP64 and mixed, on ragged, periodic
and mixed-boundary grids, with body-force fields and adaptive dt; the FP64
result matches the oracle to 1e-12."""
import numpy as np
import pytest

import nsworkloads as W
from tests import gpu_util as U

pytestmark = pytest.mark.gpu

CASES = [((70, 20, 13), (0, 0, 0), False, 0.002), ((16, 12, 8), (1, 1, 1), False, 5e-4),
         ((61, 10, 7), (0, 1, 0), True, 0.0), ((5, 130, 9), (0, 0, 0), False, 0.001),
         ((130, 40, 10), (1, 0, 1), True, 0.001)]


@pytest.mark.parametrize("form", ["fp64", "mixed"])
@pytest.mark.parametrize("dims,bc,force,dt", CASES)
def test_generated_kernels_equal_hand_written(form, dims, bc, force, dt):
    from paper_1201_2118_amd import abi
    prm = W.cavity(dims[0], ny=dims[1], nz=dims[2], re=80.0, dt=dt, tau=0.5, gamma=0.37)
    prm.update(bc=bc, precision=form, lx=1.1, ly=0.9, lz=1.3)
    prm["wall_vel"][2] = [0.2, 0.0, -0.3]
    prm["g"] = (0.1, -0.2, 0.3)
    init = U.random_state(prm, 17, amp=0.3)
    frc = W.gaussian_velocity(prm, 0.2, 23) if force else None
    a = U.gpu_run(prm, 3, init, force=frc)
    b = U.gpu_run(dict(prm, flags=abi.NS_GENERATED), 3, init, force=frc)
    assert a.stats()["sweeps_total"] == b.stats()["sweeps_total"]
    for name in ("u", "v", "w", "p", "F", "G", "H", "rhs"):
        assert np.array_equal(a.get_np(name), b.get_np(name)), name
    if form == "fp64":
        o, _ = U.oracle_run(prm, 3, init, force=frc)
        assert b.stats()["sweeps_total"] == o.stats.sweeps_total
        U.compare_state(b, o, prm, 1e-12)


def test_generated_kernels_need_one_instance():
    from paper_1201_2118_amd import abi
    from paper_1201_2118_amd.solver import Solver
    prm = dict(W.cavity(8), flags=abi.NS_GENERATED)
    with pytest.raises(abi.NSError) as e:
        Solver([prm, prm])
    assert e.value.code == abi.NS_E_INVALID


@pytest.mark.parametrize("launches", [0, 1])
@pytest.mark.parametrize("form", ["fp64", "mixed"])
@pytest.mark.parametrize("dims,bc,force,dt", CASES)
def test_generated_predictor_equals_hand_written_cells(form, dims, bc, force, dt, launches):
    from paper_1201_2118_amd import abi
    from paper_1201_2118_amd.solver import Solver
    prm = W.cavity(dims[0], ny=dims[1], nz=dims[2], re=80.0, dt=dt, tau=0.5, gamma=0.37, itermax=0)
    prm.update(bc=bc, precision=form, lx=1.1, ly=0.9, lz=1.3)
    prm["wall_vel"][2] = [0.2, 0.0, -0.3]
    prm["g"] = (0.1, -0.2, 0.3)
    init = U.random_state(prm, 19, amp=0.3)
    frc = W.gaussian_velocity(prm, 0.2, 29) if force else None
    a = U.gpu_run(prm, 1, init, force=frc)
    other = W.cavity(12, ny=9, nz=7, dt=0.001, itermax=0)
    other["precision"] = form
    flags = abi.NS_BATCH_LAUNCHES if launches else 0
    b = Solver([dict(prm, flags=flags), other])
    for name, arr in init.items():
        b.set(name, arr, 0)
    if frc is not None:
        for name, arr in zip(("fx", "fy", "fz"), frc):
            b.set(name, arr, 0)
    b.step(1)
    for name in ("F", "G", "H", "rhs", "u", "v", "w"):
        assert np.array_equal(a.get_np(name), b.get_np(name, 0)), name
