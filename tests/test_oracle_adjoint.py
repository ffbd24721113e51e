"""Pins of the oracle's hand-written adjoint (no GPU).

The forward map of one step is u -> P Phi(B u): boundary fill B, predictor
Phi, exact projection P.  Each transpose is checked against the forward
code itself through directional derivatives (central differences, which
are exact up to round-off for the quadratic predictor away from the kinks
of |t|), and the whole multi-step gradient against central finite
differences of the loss.
"""
import numpy as np
import pytest

import nsworkloads as W
import oracle


def _masked(prm, fields):
    return [np.where(oracle.unknown_mask(prm, c), f, 0.0) for c, f in enumerate(fields)]


def _dot(a, b):
    return sum(float(np.sum(x * y)) for x, y in zip(a, b))


def _cases():
    cav = W.cavity(7, ny=6, nz=5, re=40.0, gamma=0.5)
    cav["wall_vel"][2] = [0.3, 0.0, -0.2]
    per = W.periodic_box(6, ny=4, nz=8, gamma=1.0, re=25.0)
    mix = W.cavity(6, ny=5, nz=4, re=60.0, gamma=0.0)
    mix["bc"] = (1, 0, 0)
    return [cav, per, mix]


@pytest.mark.parametrize("prm", _cases())
def test_predictor_transpose_dot_product(prm):
    o = oracle.Oracle(prm)
    dt = 0.02
    u = list(W.gaussian_velocity(prm, 1.0, 1))
    o.bc_vel(*u)
    d = _masked(prm, W.gaussian_velocity(prm, 1.0, 2))
    mu = _masked(prm, W.gaussian_velocity(prm, 1.0, 3))
    eps = 1e-6

    def phi(s):
        x = [a + s * b for a, b in zip(u, d)]
        o.bc_vel(*x)
        return _masked(prm, o.fgh(dt, *x))

    jd = [(a - b) / (2 * eps) for a, b in zip(phi(eps), phi(-eps))]
    lhs = _dot(jd, mu)
    jt = o.adj_fgh(dt, *u, *mu)
    rhs = _dot(d, jt)
    assert abs(lhs - rhs) < 1e-8 * abs(lhs)
    # the transpose lives on the unknowns only
    for c in range(3):
        assert not np.any(jt[c][~oracle.unknown_mask(prm, c)])


@pytest.mark.parametrize("prm", _cases())
def test_projection_is_a_symmetric_projector(prm):
    prm = dict(prm, tol=1e-14, itermax=50000)
    o = oracle.Oracle(prm)

    def P(fields):
        f = [x.copy() for x in fields]
        o.adj_project(*f)
        return f

    a = _masked(prm, W.gaussian_velocity(prm, 1.0, 5))
    b = _masked(prm, W.gaussian_velocity(prm, 1.0, 6))
    pa, pb = P(a), P(b)
    assert abs(_dot(pa, b) - _dot(a, pb)) < 1e-11 * abs(_dot(a, b)) + 1e-11
    ppa = P(pa)
    scale = max(np.abs(x).max() for x in pa)
    assert max(np.abs(x - y).max() for x, y in zip(ppa, pa)) < 1e-10 * scale
    filled = [x.copy() for x in pa]
    o.bc_vel(*filled)  # periodic images of face 0 for the divergence
    assert np.abs(o.divergence(*filled)[oracle.unknown_mask(prm, 3)]).max() < 1e-9 * scale * prm["nx"]


@pytest.mark.slow
@pytest.mark.parametrize("bc", [(0, 0, 0), (1, 1, 1)])
def test_gradient_matches_central_differences(bc):
    prm = W.cavity(8, ny=6, nz=7, re=400.0, dt=0.005, tol=1e-13, itermax=20000)
    if bc[0]:
        prm = W.periodic_box(8, ny=6, nz=4, re=400.0, dt=0.005, gamma=0.5, tol=1e-13, itermax=20000)
    nsteps = 4
    u0 = _masked(prm, W.gaussian_velocity(prm, 1e-2, 5))
    if bc[0]:
        u0 = _masked(prm, W.gaussian_velocity(prm, 0.5, 5))
    tgt = _masked(prm, W.gaussian_velocity(prm, 1e-2, 6))
    loss, grad, _ = oracle.gradient(prm, *u0, tgt, nsteps)
    for c in range(3):
        assert not np.any(grad[c][~oracle.unknown_mask(prm, c)])

    def L(x):
        o = oracle.Oracle(prm)
        o.set("u", x[0]); o.set("v", x[1]); o.set("w", x[2])
        o.run(nsteps)
        r = _masked(prm, [o.u - tgt[0], o.v - tgt[1], o.w - tgt[2]])
        return 0.5 * sum(float(np.sum(a * a)) for a in r)

    # O(1) random velocities with gamma > 0 put some |t| within 1e-4 of its
    # kink at 0, where a central difference of that width is wrong; a
    # narrower step stays on one side
    eps = 1e-6 if bc[0] else 1e-4
    for k, dvec in enumerate(W.directions(prm, 4, 7)):
        dvec = _masked(prm, dvec)
        nrm = np.sqrt(_dot(dvec, dvec))
        dvec = [x / nrm for x in dvec]
        fd = (L([a + eps * b for a, b in zip(u0, dvec)]) -
              L([a - eps * b for a, b in zip(u0, dvec)])) / (2 * eps)
        an = _dot(grad, dvec)
        assert abs(fd - an) < 1e-5 * max(abs(an), 1e-12), (k, fd, an)
