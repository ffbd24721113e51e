"""Steady lid-driven cavity at Re 100 (the paper's verification case,
"Code Validation and Verification"): grid self-convergence of the steady
centreline profiles on the GPU (FP64).

The published reference profiles the paper compares with are not available
here, so the check is internal: the cavity is run to a steady state at 16^3,
32^3 and 64^3 (t = 20, dt 0.0025, SOR to 1e-8; a steady state of the
projection step does not depend on dt, so the three grids share it and run
in one batched handle), the centreline
profiles u(z) at x = y = 1/2 and w(x) at y = z = 1/2 are restricted to the
coarser grid (mean of the two fine values around a coarse point) and the
differences between successive grids must fall at an observed order above
1 (the donor-cell blend gamma = 0.5 makes the scheme formally first order in
the convective terms, second order elsewhere).
"""
import numpy as np
import pytest

import nsworkloads as W
from tests import gpu_util as U

pytestmark = pytest.mark.gpu


def _steady_profiles(ns, dt=0.0025, t_end=20.0):
    """{n: (u(z), w(x), change of u over the last 2 time units)} for every
    grid size n in ns, all in one batched handle (one persistent launch per
    call; each domain keeps its own stop rule)."""
    from paper_1201_2118_amd.solver import Solver
    prms = [W.cavity(n, re=100.0, dt=dt, tol=1e-8, itermax=500) for n in ns]
    s = Solver(prms)
    nsteps = int(round(t_end / dt))
    tail = int(round(2.0 / dt))

    def advance(k):  # in calls of at most 800 steps (short launches)
        while k > 0:
            s.step(min(k, 800))
            k -= 800

    advance(nsteps - tail)
    u_before = [s.get_np("u", i) for i in range(len(ns))]
    advance(tail)
    out = {}
    for i, n in enumerate(ns):
        u = s.get_np("u", i)
        w = s.get_np("w", i)
        change = np.abs(u - u_before[i]).max()
        h = n // 2
        uc = 0.5 * (u[1:n + 1, h, h] + u[1:n + 1, h + 1, h])    # u(z) at x = 1/2, y = 1/2
        wc = 0.5 * (w[h, h, 1:n + 1] + w[h, h + 1, 1:n + 1])    # w(x) at z = 1/2, y = 1/2
        out[n] = (uc, wc, change)
    s.close()
    return out


def _restrict(a):
    return 0.5 * (a[0::2] + a[1::2])


@pytest.mark.timeout(900)
def test_steady_cavity_re100_self_convergence():
    runs = _steady_profiles((16, 32, 64))
    for n, (_, _, change) in runs.items():
        print(f"{n}^3: change of u over the last 2 time units {change:.2e}", flush=True)
        assert change < 1e-4, (n, change)
    for q, name in ((0, "u(z)"), (1, "w(x)")):
        e1 = np.abs(runs[16][q] - _restrict(runs[32][q])).max()
        e2 = np.abs(runs[32][q] - _restrict(runs[64][q])).max()
        order = np.log2(e1 / e2)
        print(f"{name}: |16-32| {e1:.3e}  |32-64| {e2:.3e}  observed order {order:.2f}", flush=True)
        assert order > 1.0, (name, e1, e2)
    # the primary vortex: reversed flow below the lid on the vertical centreline
    uc = runs[64][0]
    assert uc.min() < 0 and uc[-1] > 0.5


@pytest.mark.timeout(600)
def test_steady_cavity_re100_matches_oracle():
    n, dt, t_end = 16, 0.01, 20.0
    prm = W.cavity(n, re=100.0, dt=dt, tol=1e-8, itermax=500)
    nsteps = int(round(t_end / dt))
    s = U.gpu_run(prm, nsteps)
    o, rc = U.oracle_run(prm, nsteps)
    assert rc == 0
    st = s.stats()
    print(f"{n}^3 steady cavity: GPU {st['sweeps_total']} sweeps, oracle {o.stats.sweeps_total}", flush=True)
    assert st["steps"] == nsteps and abs(st["t"] - o.stats.t) < 1e-12
    assert st["sweeps_total"] == o.stats.sweeps_total
    errs = U.compare_state(s, o, prm, 1e-12)
    h = n // 2
    u, w = s.get_np("u"), s.get_np("w")
    uo, wo = o.field("u"), o.field("w")
    uc = 0.5 * (u[1:n + 1, h, h] + u[1:n + 1, h + 1, h])
    uco = 0.5 * (uo[1:n + 1, h, h] + uo[1:n + 1, h + 1, h])
    wc = 0.5 * (w[h, h, 1:n + 1] + w[h, h + 1, 1:n + 1])
    wco = 0.5 * (wo[h, h, 1:n + 1] + wo[h, h + 1, 1:n + 1])
    assert np.abs(uc - uco).max() <= 1e-12 * np.abs(uco).max()
    assert np.abs(wc - wco).max() <= 1e-12 * np.abs(wco).max()
    print(f"{n}^3 steady cavity vs oracle: {errs}", flush=True)


def test_steady_cavity_re100_32_matches_oracle_golden():
    """The 32^3 cavity to t = 20 against the oracle's run of the same 4000
    steps (tests/golden/steady_32.npz, written by make_steady_32.py, which
    calls only the oracle): equal sweep counts, every unknown and both
    centreline profiles to 1e-12."""
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "steady_32.npz")
    gold = np.load(path)
    n, dt = 32, 0.005
    prm = W.cavity(n, re=100.0, dt=dt, tol=1e-8, itermax=500)
    nsteps = int(gold["steps"])
    s = U.gpu_run(prm, nsteps)
    st = s.stats()
    print(f"32^3 steady cavity: GPU {st['sweeps_total']} sweeps, oracle {int(gold['sweeps_total'])}", flush=True)
    assert st["steps"] == nsteps and abs(st["t"] - float(gold["t"])) < 1e-12
    assert st["sweeps_total"] == int(gold["sweeps_total"])
    m = U.masks(prm)
    ref = [gold[f] for f in "uvw"]
    sc = U.velocity_scale(ref, prm)
    for c, f in enumerate("uvw"):
        assert U.vel_rel(s.get_np(f), ref[c], m[c], sc) <= 1e-12, f
        assert U.own_rel(s.get_np(f), ref[c], m[c], sc) <= 1e-10, f
    assert U.pressure_rel(s.get_np("p"), gold["p"], m[3]) <= 1e-12
    h = n // 2
    u, w = s.get_np("u"), s.get_np("w")
    uc = 0.5 * (u[1:n + 1, h, h] + u[1:n + 1, h + 1, h])
    wc = 0.5 * (w[h, h, 1:n + 1] + w[h, h + 1, 1:n + 1])
    assert np.abs(uc - gold["u_centre"]).max() <= 1e-12 * np.abs(gold["u_centre"]).max()
    assert np.abs(wc - gold["w_centre"]).max() <= 1e-12 * np.abs(gold["w_centre"]).max()
