"""Manufactured-solution pins of the oracle with no-slip walls (no GPU).

The solution and its forcing come from tests/golden/mms_forcing.json,
written by tests/golden/make_mms.py with sympy from eq. (1) of the paper
(incompressible Navier-Stokes, rho = 1).  Every tangential component is
odd about each wall, so the ghost reflection reproduces it exactly.
"""
import json
import os

import numpy as np
import pytest
import sympy as sp

import nsworkloads as W
import oracle

_G = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "mms_forcing.json")))
_x, _y, _z, _nu = sp.symbols("x y z nu")
_FN = {k: sp.lambdify((_x, _y, _z, _nu), sp.sympify(v), "numpy") for k, v in _G.items()}


def _sample(prm, key, comp, nu):
    X, Y, Z = W.coords(prm, comp)
    return np.broadcast_to(_FN[key](X, Y, Z, nu), X.shape).astype(np.float64).copy()


def _setup(n, re, gamma, convection="conservative", **kw):
    prm = dict(W.cavity(n, lid=0.0, re=re, gamma=gamma, **kw), convection=convection)
    nu = 1.0 / re
    o = oracle.Oracle(prm)
    u, v, w = (_sample(prm, k, c, nu) for c, k in enumerate("uvw"))
    p = _sample(prm, "p", 3, nu)
    o.set_force(*(_sample(prm, k, c, nu) for c, k in enumerate(("fx", "fy", "fz"))))
    return prm, o, (u, v, w), p


def _momentum_truncation(n, gamma, convection="conservative"):
    """max over unknowns of (F - u)/dt - G_h p at the exact solution: the
    local truncation error of the momentum predictor (walls included)."""
    prm, o, (u, v, w), p = _setup(n, 1.0, gamma, convection)
    o.bc_vel(u, v, w)
    dt = 1e-3
    F, G, H = o.fgh(dt, u, v, w)
    h = 1.0 / n
    err = 0.0
    for c, (q, Q) in enumerate(((u, F), (v, G), (w, H))):
        m = oracle.unknown_mask(prm, c)
        shift = [1, n + 2, (n + 2) ** 2][c]
        gp = (np.roll(p.ravel(), -shift).reshape(p.shape) - p) / h
        err = max(err, float(np.abs(((Q - q) / dt - gp)[m]).max()))
    return err


FORMS = ["conservative", "advective"]


@pytest.mark.parametrize("convection", FORMS)
def test_momentum_truncation_second_order_central(convection):
    """gamma (conservative) or alpha (advective) = 0: second order."""
    e = [_momentum_truncation(n, 0.0, convection) for n in (16, 32, 64)]
    for k in range(2):
        assert 3.6 < e[k] / e[k + 1] < 4.4, e


def test_momentum_truncation_first_order_donor_cell():
    e = [_momentum_truncation(n, 0.5) for n in (32, 64, 128)]
    # the donor-cell blend adds an O(gamma h) flux term: the max-norm
    # truncation falls at first order, not second
    assert 1.4 < e[0] / e[1] < 2.6, e
    assert 1.4 < e[1] / e[2] < 2.6, e


def test_momentum_truncation_first_order_advective_upwind():
    """The advective form with alpha = 1 (full upwind): observed order near
    1 (second order would give 2); the first-order term comes out of the
    second-order one only past n = 64 on this solution."""
    ns = (64, 128, 192)
    e = [_momentum_truncation(n, 1.0, "advective") for n in ns]
    orders = [np.log(e[k] / e[k + 1]) / np.log(ns[k + 1] / ns[k]) for k in range(2)]
    assert all(0.7 < q < 1.3 for q in orders), (e, orders)


def _steady_error(n, convection="conservative"):
    prm, o, (u, v, w), p = _setup(n, 1.0, 0.0, convection, tol=1e-12, itermax=20000)
    h = 1.0 / n
    prm["dt"] = 0.9 * h * h / 6.0
    o = oracle.Oracle(prm)
    nu = 1.0
    o.set_force(*(_sample(prm, k, c, nu) for c, k in enumerate(("fx", "fy", "fz"))))
    o.set("u", u); o.set("v", v); o.set("w", w); o.set("p", p)
    for _ in range(400):
        u0 = o.u.copy()
        o.run(20)
        if np.abs(o.u - u0).max() < 1e-11:
            break
    m = oracle.unknown_mask(prm, 0)
    return float(np.abs(o.u[m] - u[m]).max())


@pytest.mark.parametrize("convection", FORMS)
def test_steady_manufactured_solution_second_order(convection):
    """Run the full step (walls, forcing, SOR, projection) to its steady
    state; the distance to the exact solution falls by about 4 per halving
    of h (gamma / alpha = 0)."""
    e8, e16 = _steady_error(8, convection), _steady_error(16, convection)
    assert 3.3 < e8 / e16 < 4.7, (e8, e16)
