"""Helpers shared by the GPU parity tests: run the same seeded case through
the HIP library (C ABI via the binding) and through the FP64 oracle."""
import numpy as np

import nsworkloads as W
import oracle


def masks(prm):
    return [oracle.unknown_mask(prm, c) for c in range(4)]


def rel(a, b, m):
    """max |a - b| / max |b| over the mask."""
    den = np.abs(b[m]).max()
    return float(np.abs(a[m] - b[m]).max() / (den if den > 0 else 1.0))


def pressure_rel(a, b, m):
    """pressure is unique up to a constant: compare after removing the
    interior mean."""
    x = a[m] - a[m].mean()
    y = b[m] - b[m].mean()
    den = np.abs(y).max()
    return float(np.abs(x - y).max() / (den if den > 0 else 1.0))


def gpu_run(prm, nsteps, init=None, force=None):
    from paper_1201_2118_amd.solver import Solver
    s = Solver(prm)
    if init is not None:
        for name, arr in init.items():
            s.set(name, arr)
    if force is not None:
        for name, arr in zip(("fx", "fy", "fz"), force):
            s.set(name, arr)
    if nsteps:
        s.step(nsteps)
    return s


def oracle_run(prm, nsteps, init=None, force=None, mode=0):
    o = oracle.Oracle(prm)
    if init is not None:
        for name, arr in init.items():
            o.set(name, arr)
    if force is not None:
        o.set_force(*force)
    rc = o.run(nsteps, mode) if nsteps else 0
    return o, rc


def velocity_scale(fields, prm):
    """max |velocity| over the unknowns of all three components."""
    m = masks(prm)
    return max(float(np.abs(f[m[c]]).max()) for c, f in enumerate(fields))


def vel_rel(a, b, m, scale):
    """max |a - b| over the unknowns / the velocity scale of the reference.
    A component can vanish by symmetry (v in the x-lid cavity is ~1e-4 of
    u), so each component is measured against the velocity scale, not
    against its own maximum."""
    return float(np.abs(a[m] - b[m]).max() / (scale if scale > 0 else 1.0))


def own_rel(a, b, m, scale, floor=1e-4):
    """max |a - b| over the unknowns of one component / that component's
    own max |b|, floored at `floor` times the velocity scale (a component that
    vanishes up to rounding is then held to an absolute bar)."""
    own = max(float(np.abs(b[m]).max()), floor * scale)
    return float(np.abs(a[m] - b[m]).max() / (own if own > 0 else 1.0))


def compare_state(s, o, prm, tol, ptol=None, own_tol=None):
    """Velocity (each component against the velocity scale) and pressure
    against the oracle.  FP64 comparisons (tol below 1e-9) also hold each
    velocity component to own_tol (default 1e-10) of its own maximum, so a
    small component (v in the x-lid cavity) cannot drift further relative to
    itself than that."""
    m = masks(prm)
    ref = [o.field(f) for f in "uvw"]
    scale = velocity_scale(ref, prm)
    errs = {}
    for c, name in enumerate("uvw"):
        errs[name] = vel_rel(s.get_np(name), ref[c], m[c], scale)
    errs["p"] = pressure_rel(s.get_np("p"), o.p, m[3])
    bad = {k: v for k, v in errs.items() if v > (ptol if (k == "p" and ptol) else tol)}
    if own_tol is None and tol < 1e-9:
        own_tol = 1e-10
    if own_tol is not None:
        for c, name in enumerate("uvw"):
            e = own_rel(s.get_np(name), ref[c], m[c], scale)
            errs[name + "_own"] = e
            if e > own_tol:
                bad[name + "_own"] = e
    assert not bad, errs
    return errs


def close_time(a, b):
    """Simulated times of two runs whose sweep shapes differ: with an
    adaptive dt the step sizes come from velocity maxima that can differ in
    the last bit between sweep-kernel families (each sums the stencil in its
    own order), so the times agree to rounding, not bit for bit."""
    return abs(a - b) <= 1e-14 * max(abs(b), 1e-300)


def random_state(prm, seed, amp=0.1):
    u, v, w = W.gaussian_velocity(prm, amp, seed)
    p = W.random_field(prm, seed + 100, 0.01)
    return {"u": u, "v": v, "w": w, "p": p}
