"""Writes configs_128.npz: the FP64 oracle's full 100-step runs of the two
128^3 workloads, reduced to what a GPU test can compare without re-running
the oracle (each run takes minutes on a CPU):

* ``cavity``: the 128^3 lid-driven cavity, Re 100, dt 5e-4, gamma 0.5,
  omega 1.7, tol 1e-6, 200 sweeps, from rest;
* ``tg``: the 128^3 periodic z-extruded Taylor-Green vortex, amplitude 1,
  nu 0.01, U(-1e-3, 1e-3) perturbations (seed 2), gamma 0, dt 5e-4.

Per workload and field (u, v, w over their unknowns; p over the cells after
removing its mean): 4096 entries at seeded random unknowns (flat indices
into the padded array and their values), the max-norm, the 2-norm, and two
projections sum(w_k * q) on seeded N(0, 1) weights w_k drawn over the padded
array (seed 1000 + 10 * field + k, numpy default_rng) restricted to the
unknowns; the run's statistics; for the Taylor-Green run the least-squares
amplitude of sin(2 pi x) cos(2 pi y) in u.

Calls only the oracle and the seeded input generators.
Run: python tests/golden/make_configs_128.py   (about 10 minutes on 8 cores)
"""
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import nsworkloads as W  # noqa: E402
import oracle  # noqa: E402

OUT = os.path.join(HERE, "configs_128.npz")
NSAMPLE = 4096
FIELDS = "uvwp"


def weights(shape, field, k):
    return np.random.default_rng(1000 + 10 * field + k).standard_normal(shape)


def mode_amplitude(prm, u):
    x, y, _ = W.coords(prm, 0)
    mode = np.sin(2 * math.pi * x) * np.cos(2 * math.pi * y)
    m = oracle.unknown_mask(prm, 0)
    return float(np.sum(u[m] * mode[m]) / np.sum(mode[m] ** 2))


def reduce_run(tag, prm, o, out):
    st = o.stats
    out[f"{tag}_stats"] = np.array([st.t, st.res_last, st.sweeps_total, st.steps, st.steps_unconverged],
                                   dtype=np.float64)
    for fi, name in enumerate(FIELDS):
        comp = fi if name != "p" else 3
        m = oracle.unknown_mask(prm, comp)
        q = o.field(name) if name != "p" else o.p
        q = q.copy()
        if name == "p":
            q[m] -= q[m].mean()
        flat = np.flatnonzero(m.ravel())
        rng = np.random.default_rng(500 + fi)
        idx = np.sort(rng.choice(flat, size=NSAMPLE, replace=False))
        out[f"{tag}_{name}_idx"] = idx.astype(np.int64)
        out[f"{tag}_{name}_val"] = q.ravel()[idx]
        qm = np.where(m, q, 0.0)
        proj = [float(np.sum(weights(q.shape, fi, k) * qm)) for k in range(2)]
        out[f"{tag}_{name}_norms"] = np.array([np.abs(qm).max(), np.sqrt(np.sum(qm * qm))] + proj)


def main():
    out = {}
    prm, n = W.cavity_128()
    o = oracle.Oracle(prm)
    a = time.time()
    assert o.run(n) == 0
    print(f"cavity 128^3, {n} steps: {time.time() - a:.0f} s, {o.stats.as_dict()}", flush=True)
    reduce_run("cavity", prm, o, out)

    prm, n = W.taylor_green_128()
    u, v, w, p = W.taylor_green(prm, amp=1.0, pert=1e-3, seed=2)
    o = oracle.Oracle(prm)
    for name, arr in zip(FIELDS, (u, v, w, p)):
        o.set(name, arr)
    a = time.time()
    assert o.run(n) == 0
    print(f"taylor-green 128^3, {n} steps: {time.time() - a:.0f} s, {o.stats.as_dict()}", flush=True)
    reduce_run("tg", prm, o, out)
    out["tg_amplitude"] = np.array([mode_amplitude(prm, u), mode_amplitude(prm, o.field("u"))])
    np.savez_compressed(OUT, **out)
    print(f"wrote {OUT}")


if __name__ == "__main__":
    main()
