"""Writes steady_32.npz: the FP64 oracle's run of the Re 100 lid-driven
cavity on a 32^3 grid from rest to t = 20 (dt 0.005, 4000 steps, gamma 0.5,
omega 1.7, tol 1e-8, at most 500 sweeps per step), the paper's verification
case ("Code Validation and Verification") at the second resolution of the
steady-state tests, reduced to what a GPU test compares without re-running
the oracle (the run takes minutes on a CPU): the full u, v, w, p fields over
the padded array, the two centreline profiles (u along z through the cavity
centre, w along x) and the run's statistics.

Calls only the oracle and the seeded input generators.
Run: python tests/golden/make_steady_32.py   (about 4 minutes on 8 cores)
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import nsworkloads as W  # noqa: E402
import oracle  # noqa: E402

OUT = os.path.join(HERE, "steady_32.npz")
N, DT, T_END = 32, 0.005, 20.0


def params():
    return W.cavity(N, re=100.0, dt=DT, tol=1e-8, itermax=500)


def centrelines(u, w, n):
    h = n // 2
    uc = 0.5 * (u[1:n + 1, h, h] + u[1:n + 1, h + 1, h])
    wc = 0.5 * (w[h, h, 1:n + 1] + w[h, h + 1, 1:n + 1])
    return uc, wc


def main():
    prm = params()
    nsteps = int(round(T_END / DT))
    o = oracle.Oracle(prm)
    t0 = time.time()
    rc = o.run(nsteps)
    assert rc == 0, rc
    uc, wc = centrelines(o.field("u"), o.field("w"), N)
    st = o.stats
    np.savez_compressed(OUT, u=o.u, v=o.v, w=o.w, p=o.p, u_centre=uc, w_centre=wc, steps=st.steps,
                        sweeps_total=st.sweeps_total, t=st.t, res_last=st.res_last,
                        steps_unconverged=st.steps_unconverged)
    print(f"wrote {OUT}: {nsteps} steps, {st.sweeps_total} sweeps, {time.time() - t0:.0f} s")


if __name__ == "__main__":
    main()
