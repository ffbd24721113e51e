"""Guard bands around every device buffer (NS_GUARD): each kernel family runs
with 4 KiB pattern bands on both sides of every buffer the library allocates,
and no band may change -- a kernel writing past the end of a buffer into a
neighbouring allocation would not fault, but it would be counted here.  The
cases cover the predictor (generated, hand-written batched, advective), rhs,
every sweep shape (fused 4/8/12 rows, two-sweep pass 16/24/32 rows, unfused),
the defect correction, the projection (hand-written and generated), the time
step, body forces, the two-stage integrator, the adjoint, the persistent and
the multi-launch batched forms and the autotuner's trial sweeps.  The check's
own detector is shown to count a byte set past a buffer's end by a host-side
fill, and results with and without the bands are bitwise equal."""
import numpy as np
import pytest

import nsworkloads as W
from paper_1201_2118_amd import abi
from tests import gpu_util as U

pytestmark = pytest.mark.gpu


def _single_cases():
    base = W.cavity(37, ny=25, nz=30, re=300.0, dt=0.0, tau=0.5, itermax=60)
    per = dict(W.cavity(34, ny=20, nz=18, re=150.0, dt=1e-3, itermax=60), bc=(1, 0, 1))
    per["wall_vel"][5] = [0.0, 0.0, 0.0]
    per["wall_vel"][3] = [0.7, 0.0, 0.2]
    cases = [(base, False)]
    for tile in [(4, 0), (8, 16), (12, 0), (16, 0), (16, 9), (-1, 0)]:
        cases.append((dict(per, tile=tile), tile == (8, 16)))
    for tile in [(8, 0), (16, 0), (24, 5), (32, 0)]:
        cases.append((dict(per, precision="mixed", tile=tile), False))
    cases += [(dict(base, integrator="rk2"), False),
              (dict(base, convection="advective"), True),
              (dict(base, flags=abi.NS_GENERATED), False),
              (dict(base, precision="mixed", integrator="rk2", flags=abi.NS_GENERATED), False)]
    return cases


def _run_all():
    from paper_1201_2118_amd.solver import Solver
    for k, (prm, force) in enumerate(_single_cases()):
        init = U.random_state(prm, 700 + k, amp=0.2)
        frc = W.gaussian_velocity(prm, 0.1, 800 + k) if force else None
        s = U.gpu_run(prm, 3, init, force=frc)
        s.close()
    # the adjoint (checkpoints, recomputation, the adjoint kernels)
    prm = W.cavity(14, ny=12, nz=10, dt=0.005, itermax=80)
    prm["checkpoint_every"] = 2
    s = U.gpu_run(prm, 5, U.random_state(prm, 900, amp=0.1))
    s.backward([np.ones(s.shape()) for _ in range(3)])
    s.close()
    # batched: persistent (mixed and FP64) and multi-launch with each sweep kind
    doms = [W.cavity(10, ny=12, nz=8), W.cavity(16, re=300.0, dt=0.004), W.periodic_box(8, nz=6, dt=1e-3),
            W.cavity(37, ny=25, nz=30, re=700.0, dt=0.0, tau=0.5)]
    for form in ("mixed", "fp64"):
        s = Solver([dict(d, precision=form) for d in doms])
        s.step(2)
        s.close()
    for tile in [(8, 0), (16, 0), (24, 0)]:
        s = Solver([dict(d, precision="mixed", tile=tile, flags=abi.NS_BATCH_LAUNCHES) for d in doms])
        s.step(2)
        s.close()
    s = Solver([dict(d, precision="fp64", flags=abi.NS_BATCH_LAUNCHES) for d in doms])
    s.step(2)
    s.close()
    # the autotuner's trial sweeps (a grid above its 2^21-cell threshold)
    for form in ("fp64", "mixed"):
        s = Solver(dict(W.cavity(136, ny=130, nz=126, dt=3e-4, itermax=20), precision=form))
        s.step(1)
        s.close()


def test_no_kernel_writes_past_a_buffer(monkeypatch):
    monkeypatch.setenv("NS_TUNE_CACHE", "off")
    before = abi.ns_guard_check(0)
    monkeypatch.setenv("NS_GUARD", "1")
    _run_all()
    assert abi.ns_guard_check(0) == before
    # the detector counts a byte set past a guarded buffer's end
    assert abi.ns_guard_check(1) == before + 1


def test_guard_bands_leave_results_unchanged(monkeypatch):
    prm = dict(W.cavity(37, ny=25, nz=30, re=300.0, dt=0.0, tau=0.5, itermax=60), tile=(16, 0))
    init = U.random_state(prm, 701, amp=0.2)
    monkeypatch.delenv("NS_GUARD", raising=False)
    a = U.gpu_run(prm, 3, init)
    monkeypatch.setenv("NS_GUARD", "1")
    b = U.gpu_run(prm, 3, init)
    assert a.stats()["sweeps_total"] == b.stats()["sweeps_total"]
    for f in "uvwp":
        assert np.array_equal(a.get_np(f), b.get_np(f)), f
    a.close()
    b.close()
