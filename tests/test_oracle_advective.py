"""Pins of the oracle's advective convective form (the SOLA / NASA-VOF2D
form weighted by alpha = gamma) that do not rest on its own code; the
order-of-accuracy pins on the manufactured solution are in
test_oracle_mms.py (parametrised over both forms).

* uniform flow in a periodic box is a fixed point of the predictor for
  every alpha (all differences vanish): F = u + dt g exactly;
* a shear mode u = A sin(2 pi y), v = w = 0 has no convective term at all
  in either form (u does not vary along x, the transport velocities in y
  and z are zero), so F = u + dt nu lap_h u with the exact discrete
  eigenvalue lap_h u = -(4/h^2) sin^2(pi h) u;
* the two forms agree to second order in h on a smooth divergence-free
  field at alpha = gamma = 0 (they discretise the same operator), but
  differ at first order when the weight is 0.5 (their upwind terms differ);
* the adjoint refuses the advective form.
"""
import math

import numpy as np
import pytest

import nsworkloads as W
import oracle


@pytest.mark.parametrize("alpha", [0.0, 0.5, 1.0])
def test_uniform_flow_is_a_fixed_point(alpha):
    prm = dict(W.periodic_box(8, ny=6, nz=4, gamma=alpha, dt=1e-3), convection="advective")
    prm["g"] = (0.3, -0.1, 0.2)
    o = oracle.Oracle(prm)
    shape = W.shape(prm)
    u, v, w = np.full(shape, 0.7), np.full(shape, -1.3), np.full(shape, 0.4)
    o.bc_vel(u, v, w)
    F, G, H = o.fgh(1e-3, u, v, w)
    for c, (q, Q) in enumerate(((u, F), (v, G), (w, H))):
        m = oracle.unknown_mask(prm, c)
        assert np.array_equal(Q[m], q[m] + 1e-3 * prm["g"][c]), c


@pytest.mark.parametrize("convection", ["conservative", "advective"])
@pytest.mark.parametrize("alpha", [0.0, 0.5])
def test_shear_mode_has_no_convective_term(convection, alpha):
    n, A, dt, re = 16, 0.8, 1e-3, 50.0
    prm = dict(W.periodic_box(n, gamma=alpha, dt=dt, re=re), convection=convection)
    o = oracle.Oracle(prm)
    _, y, _ = W.coords(prm, 0)
    u = A * np.sin(2 * math.pi * y)
    zero = np.zeros_like(u)
    o.bc_vel(u, zero, zero.copy())
    F, G, H = o.fgh(dt, u, zero, zero)
    h = 1.0 / n
    lam = -(4.0 / h ** 2) * math.sin(math.pi * h) ** 2
    m = oracle.unknown_mask(prm, 0)
    exact = u * (1.0 + dt * lam / re)
    assert np.abs(F[m] - exact[m]).max() < 1e-14
    for c, Q in ((1, G), (2, H)):
        assert np.abs(Q[oracle.unknown_mask(prm, c)]).max() == 0.0


def _tg_fields(prm):
    x, y, _ = W.coords(prm, 0)
    u = np.sin(2 * math.pi * x) * np.cos(2 * math.pi * y)
    x, y, _ = W.coords(prm, 1)
    v = -np.cos(2 * math.pi * x) * np.sin(2 * math.pi * y)
    return u, v, np.zeros_like(u)


def _form_gap(n, weight):
    dt = 1e-3
    out = []
    for conv in ("conservative", "advective"):
        prm = dict(W.periodic_box(n, nz=4, gamma=weight, dt=dt), convection=conv)
        o = oracle.Oracle(prm)
        u, v, w = _tg_fields(prm)
        o.bc_vel(u, v, w)
        out.append(o.fgh(dt, u, v, w)[0])
    m = oracle.unknown_mask(prm, 0)
    return float(np.abs(out[0][m] - out[1][m]).max()) / dt


def test_forms_agree_to_second_order_central_first_order_upwinded():
    c = [_form_gap(n, 0.0) for n in (16, 32, 64)]
    assert 3.5 < c[0] / c[1] < 4.5 and 3.5 < c[1] / c[2] < 4.5, c
    d = [_form_gap(n, 0.5) for n in (16, 32, 64)]
    assert 1.6 < d[0] / d[1] < 2.4 and 1.6 < d[1] / d[2] < 2.4, d


def test_adjoint_refuses_the_advective_form():
    prm = dict(W.cavity(6, dt=0.005), convection="advective")
    z = np.zeros(W.shape(prm))
    with pytest.raises(ValueError):
        oracle.gradient(prm, z, z, z, [z, z, z], 1)
