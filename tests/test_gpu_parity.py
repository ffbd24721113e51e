"""GPU parity of the HIP step against the FP64 oracle, through the C ABI.

FP64 bar: 1e-12 relative (max-norm over the unknowns, pressure after mean
removal) with equal sweep counts; the GPU contracts multiply-adds and sums
residuals in another order, and both effects stay far below it because SOR
is contractive.  Mixed precision: the stated 1e-5 relative velocity error.
"""
import numpy as np
import pytest

import nsworkloads as W
import oracle
from tests import gpu_util as U

pytestmark = pytest.mark.gpu


def _fixed_sweeps(prm, k):
    return dict(prm, tol=0.0, itermax=k)


# ---- single stages, via parameters that isolate them ----------------------

@pytest.mark.parametrize("dims,bc", [((24, 20, 18), (0, 0, 0)), ((17, 13, 11), (0, 0, 0)),
                                     ((16, 12, 8), (1, 1, 1)), ((12, 9, 10), (1, 0, 0)),
                                     ((2, 2, 2), (0, 0, 0)), ((70, 3, 5), (0, 0, 0))])
def test_predictor_rhs_and_projection(dims, bc):
    """itermax = 0: boundary fill, predictor, rhs, (no sweep), projection."""
    prm = W.cavity(dims[0], ny=dims[1], nz=dims[2], re=37.0, gamma=0.37)
    prm.update(bc=bc, lx=1.1, ly=0.9, lz=1.3, itermax=0, dt=0.002)
    prm["wall_vel"][2] = [0.2, 0.0, -0.3]
    prm["g"] = (0.1, -0.2, 0.3)
    init = U.random_state(prm, 1, amp=0.5)
    s = U.gpu_run(prm, 1, init)
    o, _ = U.oracle_run(prm, 1, init)
    m = U.masks(prm)
    for c, name in enumerate(("F", "G", "H")):
        assert U.rel(s.get_np(name), o.work[c], m[c]) < 1e-13, name
    assert U.rel(s.get_np("rhs"), o.rhs, m[3]) < 1e-12
    assert np.array_equal(s.get_np("p")[m[3]], init["p"][m[3]])
    U.compare_state(s, o, prm, 1e-13)


@pytest.mark.parametrize("k", [1, 2, 7])
@pytest.mark.parametrize("dims,bc", [((20, 16, 12), (0, 0, 0)), ((13, 11, 9), (0, 0, 0)),
                                     ((16, 16, 6), (1, 1, 1)), ((10, 12, 7), (0, 1, 0))])
def test_fixed_sweep_count(dims, bc, k):
    """tol = 0: exactly k red-black sweeps, so the Poisson stage is compared
    without any stop-rule decision."""
    prm = W.cavity(dims[0], ny=dims[1], nz=dims[2], re=50.0, dt=0.003)
    prm.update(_fixed_sweeps(prm, k), bc=bc)
    init = U.random_state(prm, 2, amp=0.3)
    s = U.gpu_run(prm, 1, init)
    o, _ = U.oracle_run(prm, 1, init)
    assert s.stats()["sweeps_total"] == k == o.stats.sweeps_total
    U.compare_state(s, o, prm, 1e-12)
    assert abs(s.stats()["res_last"] - o.stats.res_last) <= 1e-12 * o.stats.res_last


# ---- whole steps ----------------------------------------------------------------

@pytest.mark.parametrize("tile", [(0, 0), (4, 0), (8, 3), (12, 0), (-1, 0)])
@pytest.mark.parametrize("dims,bc", [((2, 2, 2), (1, 1, 1)), ((2, 6, 4), (1, 0, 1)), ((4, 2, 3), (1, 1, 0)),
                                     ((5, 2, 2), (0, 1, 1))])
@pytest.mark.parametrize("form", ["fp64", "mixed"])
def test_two_cell_periodic_axes(dims, bc, tile, form):
    """Periodic axes of two cells, the shortest the library accepts: a cell's
    two neighbours along such an axis are the same cell, and the sweep tiles'
    two-cell halos wrap exactly once.  Three steps against the oracle, every
    one-sweep shape (the two-sweep pass needs periodic axes of four cells)."""
    prm = W.cavity(dims[0], ny=dims[1], nz=dims[2], re=60.0, dt=0.002, tol=1e-10, itermax=80)
    prm.update(bc=bc, precision=form, tile=tile, lx=0.4, ly=0.5, lz=0.6)
    prm["wall_vel"] = [[0.0] * 3 for _ in range(6)]
    for a in range(3):
        if not bc[a]:
            prm["wall_vel"][2 * a + 1] = [0.8 if a != 0 else 0.0, 0.5 if a != 1 else 0.0, 0.3 if a != 2 else 0.0]
    prm["g"] = (0.2, -0.1, 0.3)
    init = U.random_state(prm, 31, amp=0.4)
    s = U.gpu_run(prm, 3, init)
    o, rc = U.oracle_run(dict(prm, precision="fp64"), 3, init, mode=1 if form == "mixed" else 0)
    assert rc == 0
    if form == "fp64":
        assert s.stats()["sweeps_total"] == o.stats.sweeps_total
        U.compare_state(s, o, prm, 1e-12)
    else:
        U.compare_state(s, o, prm, 1e-5, ptol=1e-4)


@pytest.mark.parametrize("n_dom", [1, 3])
@pytest.mark.parametrize("form", ["fp64", "mixed"])
def test_zero_steps_leave_state_unchanged(n_dom, form):
    """ns_step(0) on a single and a batched (persistent) handle: no step, the
    state and the statistics as they were."""
    from paper_1201_2118_amd.solver import Solver
    prms = [dict(W.cavity(12 + 2 * i, ny=10, nz=9 + i, dt=0.0, tau=0.5), precision=form) for i in range(n_dom)]
    s = Solver(prms)
    inits = [U.random_state(p, 60 + i, amp=0.2) for i, p in enumerate(prms)]
    for i, init in enumerate(inits):
        for name, arr in init.items():
            s.set(name, arr, i)
    s.step(1)
    before = [{f: s.get_np(f, i) for f in "uvwp"} for i in range(n_dom)]
    st0 = [s.stats(i) for i in range(n_dom)]
    s.step(0)
    for i in range(n_dom):
        assert s.stats(i) == st0[i]
        for f in "uvwp":
            assert np.array_equal(s.get_np(f, i), before[i][f]), (i, f)
    s.close()


def test_cavity_16_ten_steps():
    """The 16^3 lid-driven cavity, Re 100, dt 0.01, gamma 0.5, omega 1.7,
    tol 1e-6, 200 sweeps, 10 steps."""
    prm, n = W.cavity_small()
    s = U.gpu_run(prm, n)
    o, rc = U.oracle_run(prm, n)
    assert rc == 0
    st = s.stats()
    assert st["steps"] == 10 and st["steps_unconverged"] == 0
    assert st["sweeps_total"] == o.stats.sweeps_total
    assert st["sweeps_max"] == o.stats.sweeps_max
    U.compare_state(s, o, prm, 1e-12)
    assert abs(st["t"] - o.stats.t) < 1e-15


@pytest.mark.parametrize("dims", [(17, 15, 13), (32, 8, 16), (9, 30, 5)])
def test_cavity_ragged_sizes(dims):
    prm = W.cavity(dims[0], ny=dims[1], nz=dims[2], dt=0.005)
    s = U.gpu_run(prm, 4)
    o, _ = U.oracle_run(prm, 4)
    assert s.stats()["sweeps_total"] == o.stats.sweeps_total
    U.compare_state(s, o, prm, 1e-12)


def test_periodic_taylor_green():
    prm = W.periodic_box(32, nz=4, dt=5e-4, gamma=0.0)
    u, v, w, p = W.taylor_green(prm, amp=1.0, pert=1e-3, seed=2)
    init = {"u": u, "v": v, "w": w, "p": p}
    s = U.gpu_run(prm, 5, init)
    o, _ = U.oracle_run(prm, 5, init)
    assert s.stats()["sweeps_total"] == o.stats.sweeps_total
    U.compare_state(s, o, prm, 1e-12)


def test_cavity_128_parity():
    """The 128^3 cavity (dt 5e-4), three steps: the sweep cap binds."""
    prm, _ = W.cavity_128()
    s = U.gpu_run(prm, 3)
    o, _ = U.oracle_run(prm, 3)
    assert s.stats()["sweeps_total"] == o.stats.sweeps_total == 600
    U.compare_state(s, o, prm, 1e-12)


def test_body_force_fields_and_adaptive_dt():
    prm = W.cavity(12, ny=10, nz=14, re=80.0, dt=0.0, tau=0.5)
    fx, fy, fz = W.gaussian_velocity(prm, 0.3, 9)
    init = U.random_state(prm, 3, amp=0.2)
    s = U.gpu_run(prm, 3, init, force=(fx, fy, fz))
    o, _ = U.oracle_run(prm, 3, init, force=(fx, fy, fz))
    assert abs(s.stats()["dt_last"] - o.stats.dt_last) <= 1e-15 * o.stats.dt_last
    assert s.stats()["sweeps_total"] == o.stats.sweeps_total
    U.compare_state(s, o, prm, 1e-12)


@pytest.mark.parametrize("form", ["fp64", "mixed"])
def test_single_body_force_field(form):
    """Setting only fy: the other two force fields read as zero (they are
    allocated with it), the same as the oracle given (0, fy, 0)."""
    import numpy as np
    from paper_1201_2118_amd.solver import Solver
    prm = dict(W.cavity(12, ny=10, nz=14, re=80.0, dt=0.004), precision=form)
    _, fy, _ = W.gaussian_velocity(prm, 0.3, 11)
    init = U.random_state(prm, 5, amp=0.2)
    s = Solver(prm)
    for name, arr in init.items():
        s.set(name, arr)
    s.set("fy", fy)
    s.step(3)
    zero = np.zeros_like(fy)
    o, _ = U.oracle_run(dict(prm, precision="fp64"), 3, init, force=(zero, fy, zero), mode=0 if form == "fp64" else 1)
    if form == "fp64":
        assert s.stats()["sweeps_total"] == o.stats.sweeps_total
        U.compare_state(s, o, prm, 1e-12)
    else:
        m = U.masks(prm)
        sc = U.velocity_scale([o.field(f) for f in "uvw"], prm)
        for c, f in enumerate("uvw"):
            assert U.vel_rel(s.get_np(f), o.field(f), m[c], sc) < 1e-5, f


def test_restart_and_determinism_are_bitwise():
    prm = W.cavity(14, ny=12, nz=10)
    a = U.gpu_run(prm, 6)
    b = U.gpu_run(prm, 3)
    c = U.gpu_run(prm, 0, {f: b.get_np(f) for f in "uvwp"})
    c.step(3)
    d = U.gpu_run(prm, 6)
    for f in "uvwp":
        assert np.array_equal(a.get_np(f), c.get_np(f)), f
        assert np.array_equal(a.get_np(f), d.get_np(f)), f


@pytest.mark.parametrize("tile", [None, (8, 0), (16, 0), (16, 5), (24, 5), (32, 0), (16, -7), (32, -12), (8, -5)])
@pytest.mark.parametrize("form", ["fp64", "mixed"])
def test_batched_instances_match_standalone_runs_and_oracle(form, tile):
    """Several domains in one handle share one launch per sweep (one-sweep
    shapes) or per pair of sweeps (pass shapes); each keeps its own stop
    rule, so it equals its standalone run (same sweep counts, fields to
    rounding: the sweep shapes differ) and the oracle.  With pass shapes the
    per-step sweep counts include odd ones (a domain that stops on the
    iterate a pass held only in registers is swept again)."""
    prms = [W.cavity(10, ny=12, nz=8), W.cavity(16, re=300.0, dt=0.004), W.periodic_box(8, nz=6, dt=1e-3),
            W.cavity(37, ny=25, nz=30, re=700.0, dt=0.0, tau=0.5), W.cavity(61, ny=9, nz=14, re=90.0, dt=0.0)]
    prms = [dict(p, precision=form) for p in prms]
    if tile is not None:
        prms = [dict(p, tile=tile) for p in prms]
    from paper_1201_2118_amd import abi
    from paper_1201_2118_amd.solver import Solver
    if form == "fp64" and tile is not None and tile[0] > 16:
        with pytest.raises(abi.NSError) as e:  # FP64 two-sweep tiles have 16 rows
            Solver(prms)
        assert e.value.code == abi.NS_E_INVALID
        return
    s = Solver(prms)
    counts = []
    for _ in range(3):
        before = [s.stats(i)["sweeps_total"] for i in range(len(prms))]
        s.step(1)
        counts += [s.stats(i)["sweeps_total"] - b for i, b in enumerate(before)]
    if tile is not None:
        assert list(s.timing().sor_tile) == list(tile)
        if tile[0] >= 16 and form == "fp64":
            assert any(c % 2 for c in counts), counts
    for i, prm in enumerate(prms):
        prm = dict(prm, tile=(0, 0))
        one = U.gpu_run(prm, 3)
        st, so = s.stats(i), one.stats()
        assert st["sweeps_total"] == so["sweeps_total"], (i, st, so)
        assert U.close_time(st["t"], so["t"]), (i, st["t"], so["t"])
        m = U.masks(prm)
        ref = [one.get_np(f) for f in "uvw"]
        sc = U.velocity_scale(ref, prm)
        # different sweep shapes round differently (FP32 arithmetic in the
        # mixed correction sweeps)
        # (the default shape is the persistent launch: two-sweep pass tiles)
        same = (1e-12 if tile is None or tile[0] >= 16 else 1e-13) if form == "fp64" else 1e-6
        for c, f in enumerate("uvw"):
            assert U.vel_rel(s.get_np(f, i), ref[c], m[c], sc) < same, (i, f)
        o, _ = U.oracle_run(dict(prm, precision="fp64"), 3, mode=0 if form == "fp64" else 1)
        so = U.velocity_scale([o.field(f) for f in "uvw"], prm)
        for c, f in enumerate("uvw"):
            assert U.vel_rel(s.get_np(f, i), o.field(f), m[c], so) < (1e-12 if form == "fp64" else 1e-5), (i, f)


def test_batched_workload_runs():
    """The 64-cavity workload (sizes U{24..96}, Re U[50, 1000], adaptive dt,
    mixed precision) in the persistent launch, two steps: every instance
    equals its standalone run (same sweep counts, velocity to 1e-6 of its
    scale: the sweep shapes round differently in FP32)."""
    prms, _ = W.batched_64()
    prms = [dict(p, precision="mixed") for p in prms]
    from paper_1201_2118_amd.solver import Solver
    s = Solver(prms)
    s.step(2)
    worst = 0.0
    for i in range(len(prms)):
        st = s.stats(i)
        assert st["steps"] == 2 and st["dt_last"] > 0 and np.isfinite(st["res_last"])
        one = U.gpu_run(prms[i], 2)
        assert st["sweeps_total"] == one.stats()["sweeps_total"], i
        assert U.close_time(st["t"], one.stats()["t"]), i
        m = U.masks(prms[i])
        ref = [one.get_np(f) for f in "uvw"]
        sc = U.velocity_scale(ref, prms[i])
        for c, f in enumerate("uvw"):
            e = U.vel_rel(s.get_np(f, i), ref[c], m[c], sc)
            worst = max(worst, e)
            assert e < 1e-6, (i, f, e)
        one.close()
    print(f"64 cavities, 2 steps: worst velocity difference to the standalone runs {worst:.2e}", flush=True)


@pytest.mark.parametrize("launch,form,tile", [("multi", "mixed", (24, 0)), ("multi", "mixed", (32, 0)),
                                               ("multi", "fp64", (16, 0)), ("persistent", "mixed", (32, 0)),
                                               ("persistent", "fp64", (16, 0))])
def test_batched_workload_bitwise_equal_to_standalone_same_tile(launch, form, tile):
    """The 64-cavity workload, batched, against each cavity's standalone run
    with the same two-sweep tile: the per-cell arithmetic is the same, so
    with equal sweep counts every field is bit for bit equal.  Multi-launch
    form with explicit 24- and 32-row (FP32) and 16-row (FP64) tiles; the
    persistent launch, whose teams sweep 32-row (FP32) / 16-row (FP64) tiles
    cut into z ranges instead of fixed chunks."""
    prms, _ = W.batched_64()
    prms = [dict(p, precision=form) for p in prms]
    from paper_1201_2118_amd import abi
    from paper_1201_2118_amd.solver import Solver
    if launch == "multi":
        s = Solver([dict(p, tile=tile, flags=abi.NS_BATCH_LAUNCHES) for p in prms])
    else:
        s = Solver([dict(p, flags=abi.NS_TIMING if i == 0 else 0) for i, p in enumerate(prms)])
    s.step(2)
    if launch == "multi":
        assert list(s.timing().sor_tile) == list(tile)
    else:
        assert s.timing().launches[abi.NS_T_SOR] == 1  # the persistent launch
    for i, prm in enumerate(prms):
        st = s.stats(i)
        one = U.gpu_run(dict(prm, tile=tile), 2)
        assert st["sweeps_total"] == one.stats()["sweeps_total"], (i, st, one.stats())
        assert st["t"] == one.stats()["t"], i
        for f in "uvwp":
            assert np.array_equal(s.get_np(f, i), one.get_np(f)), (i, f)
        one.close()
    s.close()


def test_nonfinite_state_is_reported():
    from paper_1201_2118_amd import abi
    prm = W.cavity(10)
    init = U.random_state(prm, 4)
    init["u"][5, 5, 5] = np.nan
    s = U.gpu_run(prm, 0, init)
    assert s.step(2, check=False) == abi.NS_E_NONFINITE
    assert "non-finite" in s.last_error()


@pytest.mark.parametrize("variant", [dict(precision="mixed"), dict(integrator="rk2"),
                                     dict(convection="advective"), dict(precision="mixed", integrator="rk2"),
                                     dict(tile=(16, 0)), dict(tile=(-1, 0)), dict(dt=0.0, tau=0.5)])
@pytest.mark.parametrize("field", ["u", "w", "p"])
def test_nonfinite_state_is_reported_in_every_form(variant, field):
    """A NaN in the velocity or the pressure is reported as NS_E_NONFINITE
    by every form of the step (mixed precision, two-stage integrator,
    advective form, every sweep family, adaptive dt), and the handle stays
    usable: a finite state set afterwards steps normally."""
    from paper_1201_2118_amd import abi
    prm = dict(W.cavity(10, ny=9, nz=8), **variant)
    init = U.random_state(prm, 4)
    bad = {k: v.copy() for k, v in init.items()}
    bad[field][4, 5, 5] = np.nan
    s = U.gpu_run(prm, 0, bad)
    assert s.step(2, check=False) == abi.NS_E_NONFINITE
    assert "non-finite" in s.last_error()
    for name, arr in init.items():
        s.set(name, arr)
    assert s.step(1, check=False) == abi.NS_OK, s.last_error()
    for f in "uvwp":
        assert np.isfinite(s.get_np(f)).all(), f
    s.close()


@pytest.mark.parametrize("launches", [0, 1])
def test_nonfinite_state_is_reported_in_a_batch(launches):
    """A NaN in one domain of a batched handle (persistent and multi-launch
    form) is reported as NS_E_NONFINITE; with finite states set again the
    handle steps normally."""
    from paper_1201_2118_amd import abi
    from paper_1201_2118_amd.solver import Solver
    prms = [dict(W.cavity(10 + i, ny=9, nz=8), precision="mixed") for i in range(3)]
    s = Solver([dict(p, flags=abi.NS_BATCH_LAUNCHES if launches else 0) for p in prms])
    inits = [U.random_state(p, 40 + i) for i, p in enumerate(prms)]
    for i, init in enumerate(inits):
        for name, arr in init.items():
            a = arr.copy()
            if i == 1 and name == "v":
                a[3, 4, 5] = np.nan
            s.set(name, a, i)
    assert s.step(2, check=False) == abi.NS_E_NONFINITE
    for i, init in enumerate(inits):
        for name, arr in init.items():
            s.set(name, arr, i)
    assert s.step(1, check=False) == abi.NS_OK, s.last_error()
    for i in range(3):
        for f in "uvwp":
            assert np.isfinite(s.get_np(f, i)).all(), (i, f)
    s.close()


@pytest.mark.parametrize("form", ["fp64", "mixed"])
@pytest.mark.parametrize("itermax", [1, 3])
def test_unconverged_solves_are_counted(form, itermax):
    """A sweep budget too small for the tolerance is not an error: every step
    proceeds after itermax sweeps and counts as unconverged, as in the
    oracle; a batched handle (persistent launch) counts per domain."""
    from paper_1201_2118_amd.solver import Solver
    prm = dict(W.cavity(14, ny=12, nz=10, tol=1e-12, itermax=itermax), precision=form)
    s = U.gpu_run(prm, 4)
    o, rc = U.oracle_run(dict(prm, precision="fp64"), 4, mode=1 if form == "mixed" else 0)
    st = s.stats()
    assert st["steps"] == 4 and st["steps_unconverged"] == o.stats.steps_unconverged == 4
    assert st["sweeps_max"] == o.stats.sweeps_max == itermax
    assert st["sweeps_total"] == o.stats.sweeps_total == 4 * itermax
    b = Solver([prm, dict(prm, nx=12, tol=1e-3, itermax=200)])
    b.step(4)
    assert b.stats(0)["steps_unconverged"] == 4 and b.stats(0)["sweeps_total"] == 4 * itermax
    assert b.stats(1)["steps_unconverged"] == 0
    b.close()
    s.close()


@pytest.mark.parametrize("form", ["fp64", "mixed"])
def test_unstable_dt_when_allowed_ends_nonfinite(form):
    """A fixed dt 40 times the explicit diffusion bound, accepted with
    NS_ALLOW_UNSTABLE: the state overflows within a few steps (the oracle's
    run of the same case after 6), and ns_step reports NS_E_NONFINITE with
    the completed steps counted -- an error code, not a crash."""
    from paper_1201_2118_amd import abi
    n, re = 12, 100.0
    bound = 0.5 * re / (3 * n * n)  # diffusion number 1/2 on the unit cube
    prm = dict(W.cavity(n, re=re, dt=40 * bound, itermax=50), precision=form, flags=abi.NS_ALLOW_UNSTABLE)
    s = U.gpu_run(prm, 0, U.random_state(prm, 9, amp=0.1))
    code = s.step(400, check=False)
    assert code == abi.NS_E_NONFINITE, (code, s.last_error())
    assert 0 < s.stats()["steps"] < 400
    s.close()


# ---- mixed precision ---------------------------------------------------------------

def test_mixed_matches_its_fp64_algorithm_and_fp64_oracle():
    """FP32 storage and sweeps inside FP64 defect correction: against the
    oracle running the same defect-correction algorithm in FP64 and against
    the plain FP64 oracle, relative velocity error <= 1e-5."""
    prm, n = W.cavity_small()
    mp = dict(prm, precision="mixed")
    s = U.gpu_run(mp, n)
    od, _ = U.oracle_run(prm, n, mode=1)
    o, _ = U.oracle_run(prm, n, mode=0)
    m = U.masks(prm)
    sd = U.velocity_scale([od.field(f) for f in "uvw"], prm)
    so = U.velocity_scale([o.field(f) for f in "uvw"], prm)
    for c, f in enumerate("uvw"):
        assert U.vel_rel(s.get_np(f), od.field(f), m[c], sd) < 1e-5, f
        assert U.vel_rel(s.get_np(f), o.field(f), m[c], so) < 1e-5, f
    assert s.stats()["steps_unconverged"] == 0


def test_mixed_fixed_budget_128():
    prm, _ = W.cavity_128()
    mp = dict(prm, precision="mixed")
    s = U.gpu_run(mp, 2)
    o, _ = U.oracle_run(prm, 2)
    m = U.masks(prm)
    sc = U.velocity_scale([o.field(f) for f in "uvw"], prm)
    for c, f in enumerate("uvw"):
        assert U.vel_rel(s.get_np(f), o.field(f), m[c], sc) < 1e-5, f
    assert s.stats()["sweeps_total"] == 400


# ---- adjoint ------------------------------------------------------------------------

def _adjoint_case(n=10, steps=4, k=2, bc=(0, 0, 0)):
    prm = W.cavity(n, ny=n - 2, nz=n + 1, re=400.0, dt=0.005, tol=1e-13, itermax=20000)
    if bc[0]:
        prm = W.periodic_box(n, ny=n - 2, nz=4, re=400.0, dt=0.005, gamma=0.5, tol=1e-13, itermax=20000)
    prm["checkpoint_every"] = k
    mk = [oracle.unknown_mask(prm, c) for c in range(3)]
    u0 = [np.where(mk[c], f, 0.0) for c, f in enumerate(W.gaussian_velocity(prm, 1e-2, 5))]
    tgt = [np.where(mk[c], f, 0.0) for c, f in enumerate(W.gaussian_velocity(prm, 1e-2, 6))]
    return prm, u0, tgt, mk, steps


@pytest.mark.parametrize("bc,k", [((0, 0, 0), 2), ((0, 0, 0), 3), ((1, 1, 1), 4)])
def test_backward_matches_oracle_gradient(bc, k):
    prm, u0, tgt, mk, steps = _adjoint_case(bc=bc, k=k, steps=5)
    loss, grad, final = oracle.gradient(prm, *u0, tgt, steps)
    s = U.gpu_run(prm, steps, {"u": u0[0], "v": u0[1], "w": u0[2]})
    sc = U.velocity_scale(final, prm)
    for c, f in enumerate("uvw"):
        assert U.vel_rel(s.get_np(f), final[c], mk[c], sc) < 1e-12
    gf = [np.where(mk[c], s.get_np(f) - tgt[c], 0.0) for c, f in enumerate("uvw")]
    gi = [g.cpu().numpy() for g in s.backward(gf)]
    for c in range(3):
        assert U.rel(gi[c], grad[c], mk[c]) < 1e-10, c
        assert not np.any(gi[c][~mk[c]])
    # the forward state is untouched by the backward pass
    for c, f in enumerate("uvw"):
        assert U.vel_rel(s.get_np(f), final[c], mk[c], sc) < 1e-12


def test_backward_needs_a_recording():
    from paper_1201_2118_amd import abi
    prm, u0, tgt, mk, steps = _adjoint_case()
    s = U.gpu_run(prm, 0, {"u": u0[0], "v": u0[1], "w": u0[2]})
    with pytest.raises(abi.NSError) as e:
        s.backward(tgt)
    assert e.value.code == abi.NS_E_STATE


# ---- fused sweep shapes ------------------------------------------------------------

@pytest.mark.parametrize("tile", [(4, 0), (8, 5), (12, 3), (8, 1), (4, 2), (8, -4)])
@pytest.mark.parametrize("dims,bc", [((70, 20, 13), (0, 0, 0)), ((16, 12, 8), (1, 1, 1)),
                                     ((61, 10, 7), (0, 1, 0)), ((3, 130, 4), (0, 0, 0)),
                                     ((122, 7, 6), (1, 0, 1))])
def test_fused_sweep_shapes_match_unfused_and_oracle(dims, bc, tile):
    """Every workgroup shape and z chunking (ragged tiles in x, y and z)
    gives the unfused sweeps' result and the oracle's, for fixed sweeps, and
    the 8-row whole-column shape's result bit for bit (the tiling changes no
    cell's arithmetic)."""
    prm = W.cavity(dims[0], ny=dims[1], nz=dims[2], re=50.0, dt=5e-4, tol=0.0, itermax=5)
    prm["bc"] = bc
    init = U.random_state(prm, 8, amp=0.3)
    f = U.gpu_run(dict(prm, tile=tile), 1, init)
    ref = U.gpu_run(dict(prm, tile=(-1, 0)), 1, init)
    fam = U.gpu_run(dict(prm, tile=(8, 0)), 1, init)
    o, _ = U.oracle_run(prm, 1, init)
    m = U.masks(prm)
    for name in "uvwp":
        assert np.array_equal(f.get_np(name), fam.get_np(name)), name
    for name, c in (("p", 3), ("u", 0), ("v", 1), ("w", 2)):
        a, b = f.get_np(name), ref.get_np(name)
        assert np.abs(a[m[c]] - b[m[c]]).max() <= 1e-13 * np.abs(b[m[c]]).max(), name
    U.compare_state(f, o, prm, 1e-12)
    assert abs(f.stats()["res_last"] - ref.stats()["res_last"]) <= 1e-13 * ref.stats()["res_last"]


# ---- two-sweep pass shapes (temporal blocking) ----------------------------------

@pytest.mark.parametrize("tile", [(16, 0), (16, 5), (16, 3), (16, 1), (16, 2), (16, -4)])
@pytest.mark.parametrize("dims,bc", [((70, 20, 13), (0, 0, 0)), ((16, 12, 8), (1, 1, 1)),
                                     ((61, 10, 7), (0, 1, 0)), ((3, 130, 4), (0, 0, 0)),
                                     ((122, 7, 6), (1, 0, 1)), ((130, 40, 9), (0, 0, 0))])
def test_pass_shapes_match_unfused_and_oracle(dims, bc, tile):
    """Two sweeps per launch, every pass shape and z chunking, ragged tiles;
    5 fixed sweeps = two passes, a single sweep and the residual pass.  Equal
    to the whole-column 16-row pass bit for bit."""
    prm = W.cavity(dims[0], ny=dims[1], nz=dims[2], re=50.0, dt=5e-4, tol=0.0, itermax=5)
    prm["bc"] = bc
    init = U.random_state(prm, 8, amp=0.3)
    f = U.gpu_run(dict(prm, tile=tile), 1, init)
    ref = U.gpu_run(dict(prm, tile=(-1, 0)), 1, init)
    fam = U.gpu_run(dict(prm, tile=(16, 0)), 1, init)
    o, _ = U.oracle_run(prm, 1, init)
    m = U.masks(prm)
    for name in "uvwp":
        assert np.array_equal(f.get_np(name), fam.get_np(name)), name
    for name, c in (("p", 3), ("u", 0), ("v", 1), ("w", 2)):
        a, b = f.get_np(name), ref.get_np(name)
        assert np.abs(a[m[c]] - b[m[c]]).max() <= 1e-13 * np.abs(b[m[c]]).max(), name
    U.compare_state(f, o, prm, 1e-12)
    assert abs(f.stats()["res_last"] - ref.stats()["res_last"]) <= 1e-13 * ref.stats()["res_last"]
    assert list(f.timing().sor_tile) == list(tile)


@pytest.mark.parametrize("itermax", [1, 2, 3, 4, 6])
def test_pass_sweep_budgets(itermax):
    """Budgets that end on a pass, on a single sweep, and itermax 1."""
    prm = W.cavity(40, ny=30, nz=20, re=50.0, dt=5e-4, tol=0.0, itermax=itermax)
    init = U.random_state(prm, 12, amp=0.3)
    f = U.gpu_run(dict(prm, tile=(16, 0)), 2, init)
    o, _ = U.oracle_run(prm, 2, init)
    assert f.stats()["sweeps_total"] == o.stats.sweeps_total == 2 * itermax
    U.compare_state(f, o, prm, 1e-12)


@pytest.mark.parametrize("tile", [(16, 0), (16, 4)])
def test_pass_converges_on_either_sweep_of_a_pass(tile):
    """The 16^3 cavity, tol 1e-6: sweep counts per step of both parities
    (152, 117, 116, ...), so some solves stop on the iterate a pass held
    only in registers; every count and the state match the oracle."""
    prm, n = W.cavity_small()
    from paper_1201_2118_amd.solver import Solver
    s = Solver(dict(prm, tile=tile))
    o = oracle.Oracle(prm)
    counts = []
    for _ in range(n):
        before = s.stats()["sweeps_total"]
        s.step(1)
        o.run(1)
        counts.append(s.stats()["sweeps_total"] - before)
        assert s.stats()["sweeps_total"] == o.stats.sweeps_total
    assert any(c % 2 for c in counts) and any(c % 2 == 0 for c in counts), counts
    U.compare_state(s, o, prm, 1e-12)


def test_pass_periodic_taylor_green():
    prm = W.periodic_box(32, nz=4, dt=5e-4, gamma=0.0)
    u, v, w, p = W.taylor_green(prm, amp=1.0, pert=1e-3, seed=2)
    init = {"u": u, "v": v, "w": w, "p": p}
    s = U.gpu_run(dict(prm, tile=(16, 0)), 5, init)
    o, _ = U.oracle_run(prm, 5, init)
    assert s.stats()["sweeps_total"] == o.stats.sweeps_total
    U.compare_state(s, o, prm, 1e-12)


@pytest.mark.parametrize("tile", [(4, 16), (12, 0), (16, 0), (32, 5), (24, 3), (32, 1), (24, 0), (32, -6)])
def test_fused_mixed_precision_shapes(tile):
    """Mixed precision, every family's shapes: against the unfused sweeps and
    the oracle, and bit for bit against the same family's whole-column shape
    (8 rows fused; 16 rows pass) when the sweep counts agree."""
    prm = W.cavity(70, ny=24, nz=20, dt=0.002)
    a = U.gpu_run(dict(prm, precision="mixed", tile=tile), 2)
    b = U.gpu_run(dict(prm, precision="mixed", tile=(-1, 0)), 2)
    fam = U.gpu_run(dict(prm, precision="mixed", tile=(8, 0) if tile[0] < 16 else (16, 0)), 2)
    if a.stats()["sweeps_total"] == fam.stats()["sweeps_total"]:
        for name in "uvwp":
            assert np.array_equal(a.get_np(name), fam.get_np(name)), name
    o, _ = U.oracle_run(prm, 2)
    m = U.masks(prm)
    sc = U.velocity_scale([o.field(f) for f in "uvw"], prm)
    for c, f in enumerate("uvw"):
        assert U.vel_rel(a.get_np(f), b.get_np(f), m[c], sc) < 1e-6, f
        assert U.vel_rel(a.get_np(f), o.field(f), m[c], sc) < 1e-5, f


def test_autotuner_picks_a_valid_shape():
    prm = W.cavity(160, ny=120, nz=128, dt=5e-4, itermax=3, tol=0.0)
    from paper_1201_2118_amd.solver import Solver
    s = Solver(prm)
    t = s.timing()
    assert t.sor_tile[0] in (4, 8, 12, 16, 24, 32) and (t.sor_tile[1] == 0 or t.sor_tile[1] >= 8)
    s.step(1)
    o, _ = U.oracle_run(prm, 1)
    U.compare_state(s, o, prm, 1e-12)
