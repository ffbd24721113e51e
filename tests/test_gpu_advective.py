"""The advective convective form (NS_ADVECTIVE: the SOLA / NASA-VOF2D form
weighted by alpha = gamma) on the GPU against the oracle running the same
form: the predictor alone (itermax 0) to 1e-13, whole steps to 1e-12 with
equal sweep counts (FP64) and the mixed form to 1e-5, on wall, periodic
and mixed-boundary grids with body-force fields and adaptive dt."""
import pytest

import nsworkloads as W
from tests import gpu_util as U

pytestmark = pytest.mark.gpu

GRIDS = [((24, 20, 18), (0, 0, 0)), ((17, 13, 11), (0, 0, 0)), ((16, 12, 8), (1, 1, 1)),
         ((12, 9, 10), (1, 0, 0)), ((70, 3, 6), (0, 0, 1))]


@pytest.mark.parametrize("alpha", [0.0, 0.37, 1.0])
@pytest.mark.parametrize("dims,bc", GRIDS)
def test_advective_predictor_matches_oracle(dims, bc, alpha):
    prm = W.cavity(dims[0], ny=dims[1], nz=dims[2], re=37.0, gamma=alpha)
    prm.update(bc=bc, lx=1.1, ly=0.9, lz=1.3, itermax=0, dt=0.002, convection="advective")
    prm["wall_vel"][2] = [0.2, 0.0, -0.3]
    prm["g"] = (0.1, -0.2, 0.3)
    init = U.random_state(prm, 1, amp=0.5)
    frc = W.gaussian_velocity(prm, 0.3, 29)
    s = U.gpu_run(prm, 1, init, force=frc)
    o, _ = U.oracle_run(prm, 1, init, force=frc)
    m = U.masks(prm)
    for c, name in enumerate(("F", "G", "H")):
        assert U.rel(s.get_np(name), o.work[c], m[c]) < 1e-13, name
    U.compare_state(s, o, prm, 1e-13)


@pytest.mark.parametrize("alpha", [0.0, 0.5])
@pytest.mark.parametrize("dims,bc,dt", [((20, 16, 12), (0, 0, 0), 0.004), ((16, 16, 6), (1, 1, 1), 1e-3),
                                        ((13, 12, 9), (0, 1, 0), 0.0)])
def test_advective_steps_match_oracle(dims, bc, dt, alpha):
    prm = W.cavity(dims[0], ny=dims[1], nz=dims[2], re=60.0, dt=dt, tau=0.5, gamma=alpha)
    prm.update(bc=bc, convection="advective")
    init = U.random_state(prm, 2, amp=0.3)
    s = U.gpu_run(prm, 4, init)
    o, _ = U.oracle_run(prm, 4, init)
    assert s.stats()["sweeps_total"] == o.stats.sweeps_total
    U.compare_state(s, o, prm, 1e-12)
    mp = dict(prm, precision="mixed")
    sm = U.gpu_run(mp, 4, init)
    od, _ = U.oracle_run(prm, 4, init, mode=1)
    m = U.masks(prm)
    sc = U.velocity_scale([od.field(f) for f in "uvw"], prm)
    for c, f in enumerate("uvw"):
        assert U.vel_rel(sm.get_np(f), od.field(f), m[c], sc) < 1e-5, f


def test_advective_cavity_differs_from_conservative_at_first_order():
    """Same 32^3 cavity, both forms with weight 0.5, 20 steps: the velocity
    fields differ (the upwind terms differ at O(h)), by far more than the
    parity bar and far less than the velocity scale."""
    prm = W.cavity(32, dt=0.005)
    a = U.gpu_run(prm, 20)
    b = U.gpu_run(dict(prm, convection="advective"), 20)
    m = U.masks(prm)
    sc = U.velocity_scale([a.get_np(f) for f in "uvw"], prm)
    d = max(U.vel_rel(b.get_np(f), a.get_np(f), m[c], sc) for c, f in enumerate("uvw"))
    assert 1e-4 < d < 0.2, d
