"""Translation symmetry of the discrete step (the premise of the GPU test at
the library's size limit): on a grid periodic in x and y, an initial state
that repeats with an even period P in both stays periodic under the step --
red-black colours repeat with any even period and, with tol = 0, every solve
takes the same fixed sweeps -- so the oracle's run on a 3P x 2P grid equals
its run on one P x P period, repeated, to rounding of the pressure mean."""
import numpy as np
import pytest

import nsworkloads as W
from tests import gpu_util as U

P, NZ = 8, 3


def _params(nx, ny):
    h = 1.0 / 16
    prm = W.cavity(nx, ny=ny, nz=NZ, re=80.0, dt=1e-3, gamma=0.4, omega=1.5, tol=0.0, itermax=7)
    prm.update(lx=nx * h, ly=ny * h, lz=NZ * h, bc=(1, 1, 0))
    prm["wall_vel"][5] = [0.9, -0.4, 0.0]
    prm["g"] = (0.1, 0.0, -0.2)
    return prm


@pytest.mark.parametrize("mode", [0, 1])
def test_periodic_tiling_commutes_with_the_step(mode):
    small, big = _params(P, P), _params(3 * P, 2 * P)
    init, tiled = {}, {}
    for name, arr in U.random_state(small, 77, amp=0.3).items():
        z = np.zeros_like(arr)
        z[1:-1, 1:-1, 1:-1] = arr[1:-1, 1:-1, 1:-1]
        init[name] = z
        t = np.zeros((NZ + 2, 2 * P + 2, 3 * P + 2))
        t[1:-1, 1:-1, 1:-1] = np.tile(arr[1:-1, 1:-1, 1:-1], (1, 2, 3))
        tiled[name] = t
    a, rca = U.oracle_run(small, 2, init, mode=mode)
    b, rcb = U.oracle_run(big, 2, tiled, mode=mode)
    assert rca == rcb == 0 and a.stats.sweeps_total == b.stats.sweeps_total == 14
    for f in "uvw":
        sa = a.field(f)[1:-1, 1:-1, 1:-1]
        sb = b.field(f)[1:-1, 1:-1, 1:-1]
        assert np.array_equal(sb, np.tile(sa, (1, 2, 3))), f
    pa = a.p[1:-1, 1:-1, 1:-1]
    pb = b.p[1:-1, 1:-1, 1:-1]
    d = np.abs((pb - pb.mean()) - np.tile(pa - pa.mean(), (1, 2, 3))).max()
    assert d <= 1e-13 * np.abs(pa - pa.mean()).max(), d
