"""Seeded random batches of uneven domains in one persistent launch (and in
the multi-launch form) against each domain's standalone run: equal sweep
counts, simulated time to rounding (1e-14: adaptive steps come from velocity
maxima, and the sweep shapes differ in rounding), velocities to 1e-12 (FP64)
or 1e-6 (mixed: the sweep shapes differ in their FP32 rounding)."""
import numpy as np
import pytest

import nsworkloads as W
from paper_1201_2118_amd import abi
from tests import gpu_util as U

pytestmark = pytest.mark.gpu


def _domain(rng, precision):
    bc = tuple(int(b) for b in rng.integers(0, 2, 3))
    dims = []
    for a in range(3):
        n = int(rng.integers(2, 48))
        if bc[a]:
            n = max(4, n + (n % 2))
        dims.append(n)
    prm = W.cavity(dims[0], ny=dims[1], nz=dims[2], re=float(rng.uniform(30, 600)),
                   gamma=float(rng.uniform(0, 1)), dt=0.0 if rng.random() < 0.5 else 1e-3, tau=0.5,
                   itermax=int(rng.integers(4, 150)))
    prm.update(bc=bc, precision=precision)
    prm["wall_vel"][5] = [float(rng.uniform(-1, 1)), 0.0, 0.0]
    return prm


@pytest.mark.parametrize("launches", [0, 1])
@pytest.mark.parametrize("seed", range(12))
def test_random_batch_matches_standalone_runs(seed, launches):
    from paper_1201_2118_amd.solver import Solver
    rng = np.random.default_rng(2000 + seed)
    precision = "mixed" if rng.random() < 0.5 else "fp64"
    prms = [_domain(rng, precision) for _ in range(int(rng.integers(2, 7)))]
    inits = [U.random_state(p, 500 + 10 * seed + i, amp=0.2) for i, p in enumerate(prms)]
    flags = abi.NS_BATCH_LAUNCHES if launches else 0
    s = Solver([dict(p, flags=flags if i == 0 else 0) for i, p in enumerate(prms)])
    for i, init in enumerate(inits):
        for name, arr in init.items():
            s.set(name, arr, i)
    s.step(2)
    for i, p in enumerate(prms):
        one = U.gpu_run(p, 2, inits[i])
        st, so = s.stats(i), one.stats()
        assert st["sweeps_total"] == so["sweeps_total"], (i, p, st, so)
        assert U.close_time(st["t"], so["t"]), (i, p)
        m = U.masks(p)
        ref = [one.get_np(f) for f in "uvw"]
        sc = U.velocity_scale(ref, p)
        bar = 1e-12 if precision == "fp64" else 1e-6
        for c, f in enumerate("uvw"):
            assert U.vel_rel(s.get_np(f, i), ref[c], m[c], sc) < bar, (i, f, p)
