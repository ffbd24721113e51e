"""Pins of the oracle's moving-wall boundary term (no GPU).

Plane Couette flow: walls on one axis, periodic on the other two, one wall
sliding in a tangential direction.  The exact steady solution of eq. (1)
(incompressible Navier-Stokes, "Background and Governing Equations") is the
linear profile between the wall speeds; it has no convective term (the
velocity is parallel to the walls and varies only across them) and no
pressure gradient.  On the cell-centred tangential unknowns it is also an
exact discrete steady state of a scheme whose ghost value makes the average
across the wall equal the wall speed: the second difference of a linear
profile vanishes and the ghost continues it linearly.  A missing factor 2
in the reflection, a wrong face index of the wall speed or a wrong
tangential component breaks the fixed point and changes the state the
run converges to.
"""
import numpy as np
import pytest

import nsworkloads as W
import oracle

FACES = [(f, c) for f in range(6) for c in range(3) if c != f // 2]


def _couette_params(face, comp, speed, n_wall=8, n_per=4, re=1.0, dt=None):
    axis = face // 2
    bc = [1, 1, 1]
    bc[axis] = 0
    n = [n_per, n_per, n_per]
    n[axis] = n_wall
    prm = W.periodic_box(n[0], ny=n[1], nz=n[2], re=re, gamma=0.5, tol=1e-12, itermax=500)
    prm["bc"] = tuple(bc)
    wall = np.zeros((6, 3))
    wall[face, comp] = speed
    prm["wall_vel"] = wall.tolist()
    if dt is None:
        h2 = sum((1.0 / m) ** -2 for m in n)
        dt = 0.4 / (h2 / re)
    prm["dt"] = dt
    return prm


def _profile(prm, face, comp, speed):
    """Exact Couette profile of component comp on its own staggered
    positions: speed at the moving wall, 0 at the opposite one, linear in
    between (the tangential unknowns sit at cell centres along the wall
    axis)."""
    axis = face // 2
    X = W.coords(prm, comp)[axis]
    s = X / 1.0
    return speed * (s if face % 2 == 1 else 1.0 - s)


@pytest.mark.parametrize("face,comp", FACES)
def test_linear_couette_profile_is_a_fixed_point(oracle_mod, face, comp):
    speed = 0.7
    prm = _couette_params(face, comp, speed)
    o = oracle_mod.Oracle(prm)
    prof = _profile(prm, face, comp, speed)
    o.set("uvw"[comp], prof)
    assert o.run(4) == 0
    for c in range(3):
        m = oracle.unknown_mask(prm, c)
        want = prof[m] if c == comp else 0.0
        assert np.abs(o.field("uvw"[c])[m] - want).max() < 1e-13, (face, comp, c)
    # the ghosts beyond the walls continue the profile linearly
    axis = face // 2
    got = o.field("uvw"[comp])
    sl_lo = [slice(1, -1)] * 3
    sl_hi = [slice(1, -1)] * 3
    sl_lo[2 - axis] = 0
    sl_hi[2 - axis] = -1
    assert np.abs(got[tuple(sl_lo)] - prof[tuple(sl_lo)]).max() < 1e-13
    assert np.abs(got[tuple(sl_hi)] - prof[tuple(sl_hi)]).max() < 1e-13


@pytest.mark.parametrize("face,comp", FACES)
def test_couette_from_rest_converges_to_linear_profile(oracle_mod, face, comp):
    """Started from rest, the flow diffuses to the linear profile: with the
    reflection ghost the slowest discrete mode decays by
    1 - nu dt (4/h^2) sin^2(pi h / 2) per step, so 1200 steps at diffusion
    number 0.4 take it far below 1e-12."""
    speed = -1.3
    prm = _couette_params(face, comp, speed)
    o = oracle_mod.Oracle(prm)
    assert o.run(1200) == 0
    prof = _profile(prm, face, comp, speed)
    m = oracle.unknown_mask(prm, comp)
    assert np.abs(o.field("uvw"[comp])[m] - prof[m]).max() < 1e-12 * abs(speed)
    # mid-channel value: the mean of the two wall speeds
    mid = np.abs(o.field("uvw"[comp])[m]).mean()
    assert abs(mid - abs(speed) / 2) < 1e-12


def test_two_moving_walls_superpose(oracle_mod):
    """Both walls of the z axis moving, in different tangential directions:
    the steady state is the sum of the two single-wall profiles."""
    prm = _couette_params(5, 0, 0.9)
    wall = np.zeros((6, 3))
    wall[5, 0] = 0.9
    wall[4, 1] = -0.4
    prm["wall_vel"] = wall.tolist()
    o = oracle_mod.Oracle(prm)
    assert o.run(1200) == 0
    pu = _profile(prm, 5, 0, 0.9)
    pv = _profile(prm, 4, 1, -0.4)
    for c, want in ((0, pu), (1, pv)):
        m = oracle.unknown_mask(prm, c)
        assert np.abs(o.field("uvw"[c])[m] - want[m]).max() < 1e-12


def test_wall_normal_speed_is_ignored(oracle_mod):
    """Only the tangential parts of a wall velocity enter the fill (the
    wall-normal face velocity is the no-penetration value 0)."""
    base = W.cavity(6, ny=5, nz=7, dt=0.01)
    a = oracle_mod.Oracle(base)
    wall = np.asarray(base["wall_vel"], float).copy()
    for f in range(6):
        wall[f, f // 2] = 0.37 * (f + 1)
    b = oracle_mod.Oracle(dict(base, wall_vel=wall.tolist()))
    a.run(3)
    b.run(3)
    for c in range(3):
        m = oracle.unknown_mask(base, c)
        assert np.array_equal(a.field("uvw"[c])[m], b.field("uvw"[c])[m])
