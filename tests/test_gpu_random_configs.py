"""Seeded random combinations of the step's options against the oracle:
grid sizes (with ragged tiles), the boundary kind of each axis, storage
precision, fixed or adaptive dt, body-force fields, the sweep shape, the
time integrator, the convective form and the generated projection.  FP64
must match to 1e-12 with equal sweep counts, mixed precision to 1e-5."""
import numpy as np
import pytest

import nsworkloads as W
from paper_1201_2118_amd import abi
from tests import gpu_util as U

pytestmark = pytest.mark.gpu

TILES = [(0, 0), (4, 0), (8, 16), (12, 0), (16, 0), (16, 9), (24, 0), (32, 5), (-1, 0)]


def _draw(seed, long_axis=False):
    rng = np.random.default_rng(1000 + seed)
    bc = tuple(int(b) for b in rng.integers(0, 2, 3))
    dims = []
    la = int(rng.integers(0, 3)) if long_axis else -1
    for a in range(3):
        n = int(rng.integers(60, 151)) if a == la else int(rng.integers(2, 40))
        if bc[a]:
            n = max(4, n + (n % 2))  # periodic: even, at least the pass tile's halo
        dims.append(n)
    precision = "mixed" if rng.random() < 0.4 else "fp64"
    prm = W.cavity(dims[0], ny=dims[1], nz=dims[2], re=float(rng.uniform(30, 400)),
                   gamma=float(rng.uniform(0, 1)), omega=float(rng.uniform(1.2, 1.8)),
                   dt=0.0 if rng.random() < 0.4 else 1e-3, tau=0.5, itermax=int(rng.integers(5, 120)))
    prm.update(bc=bc, precision=precision, lx=float(rng.uniform(0.7, 1.4)), ly=float(rng.uniform(0.7, 1.4)),
               lz=float(rng.uniform(0.7, 1.4)))
    if la >= 0:  # the long axis keeps a cell size like the others'
        key = ("lx", "ly", "lz")[la]
        prm[key] = prm[key] * dims[la] / 30.0
    prm["wall_vel"][5] = [float(rng.uniform(-1, 1)), float(rng.uniform(-0.3, 0.3)), 0.0]
    prm["g"] = tuple(float(x) for x in rng.uniform(-0.2, 0.2, 3))
    tile = TILES[int(rng.integers(0, len(TILES)))]
    if precision == "fp64" and tile[0] > 16:
        tile = (16, tile[1])
    prm["tile"] = tile
    flags = 0
    r = rng.random()
    if r < 0.2:
        prm["integrator"] = "rk2"
    elif r < 0.35:
        prm["convection"] = "advective"
    if rng.random() < 0.25:
        flags |= abi.NS_GENERATED
    prm["flags"] = flags
    force = rng.random() < 0.4
    return prm, force


def _check(prm, force, seed):
    init = U.random_state(prm, 300 + seed, amp=0.2)
    frc = W.gaussian_velocity(prm, 0.1, 400 + seed) if force else None
    s = U.gpu_run(prm, 2, init, force=frc)
    oprm = {k: v for k, v in prm.items() if k not in ("tile", "flags")}
    mixed = prm["precision"] == "mixed"
    o, rc = U.oracle_run(dict(oprm, precision="fp64"), 2, init, force=frc, mode=1 if mixed else 0)
    assert rc == 0
    if mixed:
        m = U.masks(prm)
        sc = U.velocity_scale([o.field(f) for f in "uvw"], prm)
        for c, f in enumerate("uvw"):
            assert U.vel_rel(s.get_np(f), o.field(f), m[c], sc) < 1e-5, (f, prm)
    else:
        assert s.stats()["sweeps_total"] == o.stats.sweeps_total, prm
        U.compare_state(s, o, prm, 1e-12)


@pytest.mark.parametrize("seed", range(48))
def test_random_configuration_matches_oracle(seed):
    prm, force = _draw(seed)
    _check(prm, force, seed)


@pytest.mark.parametrize("seed", range(16))
def test_random_configuration_with_a_long_axis_matches_oracle(seed):
    """As above with one axis of 60-150 cells, so that the sweep tiles
    (56 or 60 cells wide in x, 8-24 rows in y, z chunks) meet at tile
    boundaries under every boundary kind and option."""
    prm, force = _draw(100 + seed, long_axis=True)
    _check(prm, force, 100 + seed)
