"""Pins of the oracle's two-stage time integrator (the second-order
strong-stability-preserving Runge-Kutta method of Heun, in the
method-of-lines form the Cactus time integrator offers, with a projected
Euler step as each stage) that do not rest on its own code:

* a viscous shear wave u = A s(z), v = w = 0 (s a sine sampled at the
  u positions, periodic or between resting walls) has no convective term
  and a zero Poisson right-hand side, so one Euler stage multiplies A by
  1 - z exactly, z = dt nu lambda_h with the exact discrete eigenvalue
  lambda_h = (2 - 2 cos theta) / h^2; the two-stage step must multiply it
  by 1 - z + z^2/2 (the stability polynomial of any two-stage second-order
  Runge-Kutta method), which fails for a missing average, weights other
  than one half, a second stage from u^n or with another dt;
* on a perturbed Taylor-Green flow (convection, pressure and projection all
  active; the perturbation projected onto the divergence-free fields) the
  error against a run with a step 16 times smaller than the smallest
  falls by ~2 per halving of dt for Euler and by ~4 for the two-stage
  method (measured rates 1.05, 1.06 and 2.08, 2.04);
* the averaged step stays divergence-free (the projection is linear);
* an unknown integrator name is refused.
"""
import math

import numpy as np
import pytest

import nsworkloads as W
import oracle


def _shear(walls_z, stages):
    n = 16
    prm = W.periodic_box(4, nz=n, re=10.0, dt=1e-3, gamma=0.5)
    prm.update(tol=1e-13, itermax=50, integrator="rk2" if stages == 2 else "euler")
    if walls_z:
        prm["bc"] = (1, 1, 0)
    o = oracle.Oracle(prm)
    _, _, z = W.coords(prm, 0)
    theta = (math.pi if walls_z else 2 * math.pi) / n
    s = np.sin((math.pi if walls_z else 2 * math.pi) * z)
    o.set("u", 0.8 * s)
    return prm, o, s, theta


@pytest.mark.parametrize("walls_z", [False, True])
@pytest.mark.parametrize("stages", [1, 2])
def test_shear_wave_amplitude_follows_the_stability_polynomial(walls_z, stages):
    prm, o, s, theta = _shear(walls_z, stages)
    nsteps = 25
    assert o.run(nsteps) == 0
    h = 1.0 / prm["nz"]
    zz = prm["dt"] / prm["re"] * (2.0 - 2.0 * math.cos(theta)) / (h * h)
    g = 1.0 - zz if stages == 1 else 1.0 - zz + zz * zz / 2.0
    m = oracle.unknown_mask(prm, 0)
    expect = 0.8 * g ** nsteps * s
    assert np.abs(o.u[m] - expect[m]).max() <= 1e-13 * 0.8
    for c, f in ((1, o.v), (2, o.w)):
        assert not np.any(f[oracle.unknown_mask(prm, c)])
    assert o.stats.steps == nsteps
    assert abs(o.stats.t - nsteps * prm["dt"]) <= 1e-15 * nsteps


def _tg(dt, stages, T=0.08):
    prm = W.periodic_box(16, nz=8, re=50.0, dt=dt, gamma=0.0)
    prm.update(tol=1e-12, itermax=5000, integrator="rk2" if stages == 2 else "euler")
    u, v, w, p = W.taylor_green(prm, pert=0.05, seed=3)
    o = oracle.Oracle(prm)
    # the averaged step keeps half of the state it starts from: start it
    # divergence-free (the projector with dt = 1 on the perturbed field),
    # or the initial divergence would only halve per step, an error that
    # scales with the step count, not with dt
    o.adj_project(u, v, w)
    o.set("p", p)
    for name, arr in zip("uvw", (u, v, w)):
        o.set(name, arr)
    o.bc_vel()
    nsteps = int(round(T / dt))
    assert o.run(nsteps) == 0 and o.stats.steps_unconverged == 0
    return prm, o


@pytest.mark.parametrize("stages,order", [(1, 1.0), (2, 2.0)])
def test_time_order_on_a_perturbed_taylor_green_flow(stages, order):
    prm, ref = _tg(0.08 / 1024, stages)
    errs = []
    for dt in (0.005, 0.0025, 0.00125):
        _, o = _tg(dt, stages)
        e = 0.0
        for c, name in enumerate("uvw"):
            m = oracle.unknown_mask(prm, c)
            e = max(e, float(np.abs(o.field(name)[m] - ref.field(name)[m]).max()))
        errs.append(e)
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert all(abs(r - order) < 0.15 for r in rates), (errs, rates)


def test_two_stage_step_stays_divergence_free():
    prm, o = _tg(0.01, 2, T=0.05)
    d = o.divergence()
    m = oracle.unknown_mask(prm, 3)
    assert np.abs(d[m]).max() <= 1e-9


def test_unknown_integrator_is_refused():
    with pytest.raises(ValueError):
        oracle.Oracle(dict(W.periodic_box(4), integrator="rk4"))
