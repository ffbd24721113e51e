"""Seeded synthetic inputs for the Navier-Stokes step.

This module builds parameter dictionaries and initial fields only; it holds
none of the method's arithmetic, so both the FP64 oracle and the HIP path
can take their inputs from it.  Fields use the padded layout
``(nz+2, ny+2, nx+2)``, x fastest, with the staggered (MAC) positions

    u[k, j, i] at (i dx, (j - 1/2) dy, (k - 1/2) dz)
    v[k, j, i] at ((i - 1/2) dx, j dy, (k - 1/2) dz)
    w[k, j, i] at ((i - 1/2) dx, (j - 1/2) dy, k dz)
    p[k, j, i] at ((i - 1/2) dx, (j - 1/2) dy, (k - 1/2) dz).

Workloads (the lid-driven cavity of the paper's "Code Validation and
Verification" section and the derived cases):

* ``cavity_small``  16^3, Re 100, dt 0.01, gamma 0.5, omega 1.7, tol 1e-6,
  200 sweeps, 10 steps.
* ``cavity_128``    the same cavity at 128^3 with dt 5e-4 (the literal 0.01
  violates the explicit stability bounds at this spacing).
* ``taylor_green_128``  periodic z-extruded 2D Taylor-Green vortex,
  amplitude 1, nu = 0.01, U(-1e-3, 1e-3) perturbations (seed 2), gamma 0.
* ``cavity_512``    Re 1000, dt 3e-4 (literal 0.002 is unstable), tol 1e-8,
  200 sweeps, 50 steps: the throughput case.
* ``batched_64``    64 cavities, per-axis sizes U{24..96}, Re U[50, 1000]
  (seed 4), adaptive dt with tau = 0.5, 200 steps.
* ``adjoint_64``    64^3 cavity, Re 400, dt 0.005, 20 steps, Gaussian initial
  velocity sigma 1e-2 (seed 5), target from seed 6, 16 directions (seed 7).
"""
from __future__ import annotations

import math

import numpy as np

WALL, PERIODIC = 0, 1


def cavity(n, re=100.0, dt=0.01, gamma=0.5, omega=1.7, tol=1e-6, itermax=200,
           lid=1.0, ny=None, nz=None, tau=0.5, eta=1e-2):
    """Lid-driven cavity on the unit cube: lid (lid, 0, 0) on the z = 1 face,
    no-slip on the other five walls."""
    wall = np.zeros((6, 3))
    wall[5, 0] = lid
    return dict(nx=int(n), ny=int(ny or n), nz=int(nz or n), lx=1.0, ly=1.0, lz=1.0,
                re=float(re), dt=float(dt), tau=float(tau), gamma=float(gamma),
                omega=float(omega), tol=float(tol), itermax=int(itermax),
                bc=(WALL, WALL, WALL), wall_vel=wall.tolist(), g=(0.0, 0.0, 0.0),
                eta=float(eta))


def periodic_box(n, re=100.0, dt=5e-4, gamma=0.0, omega=1.7, tol=1e-6, itermax=200,
                 nz=None, ny=None):
    return dict(nx=int(n), ny=int(ny or n), nz=int(nz or n), lx=1.0, ly=1.0, lz=1.0,
                re=float(re), dt=float(dt), tau=0.5, gamma=float(gamma), omega=float(omega),
                tol=float(tol), itermax=int(itermax), bc=(PERIODIC, PERIODIC, PERIODIC),
                wall_vel=np.zeros((6, 3)).tolist(), g=(0.0, 0.0, 0.0), eta=1e-2)


def cavity_small():
    return cavity(16), 10


def cavity_128():
    return cavity(128, dt=5e-4), 100


def cavity_512():
    return cavity(512, re=1000.0, dt=3e-4, tol=1e-8), 50


def taylor_green_128():
    return periodic_box(128, re=100.0, dt=5e-4, gamma=0.0), 100


def adjoint_64():
    p = cavity(64, re=400.0, dt=0.005)
    return p, 20


def shape(params):
    return (params["nz"] + 2, params["ny"] + 2, params["nx"] + 2)


def coords(params, comp):
    """Physical coordinates (x, y, z) of every padded entry of a field:
    comp 0/1/2 = u/v/w faces, 3 = cell centres."""
    n = (params["nx"], params["ny"], params["nz"])
    L = (params.get("lx", 1.0), params.get("ly", 1.0), params.get("lz", 1.0))
    axes = []
    for a in range(3):
        h = L[a] / n[a]
        idx = np.arange(n[a] + 2, dtype=np.float64)
        axes.append(idx * h if comp == a else (idx - 0.5) * h)
    z, y, x = np.meshgrid(axes[2], axes[1], axes[0], indexing="ij")
    return x, y, z


def taylor_green(params, amp=1.0, pert=0.0, seed=2):
    """z-extruded 2D Taylor-Green vortex sampled at the staggered positions:
    u = A sin(2 pi x) cos(2 pi y), v = -A cos(2 pi x) sin(2 pi y), w = 0,
    p = (A^2/4)(cos 4 pi x + cos 4 pi y); plus i.i.d. U(-pert, pert) on every
    padded entry of u, v, w (ghosts are overwritten by the boundary fill)."""
    x, y, _ = coords(params, 0)
    u = amp * np.sin(2 * math.pi * x) * np.cos(2 * math.pi * y)
    x, y, _ = coords(params, 1)
    v = -amp * np.cos(2 * math.pi * x) * np.sin(2 * math.pi * y)
    w = np.zeros(shape(params))
    x, y, _ = coords(params, 3)
    p = amp * amp / 4.0 * (np.cos(4 * math.pi * x) + np.cos(4 * math.pi * y))
    if pert > 0.0:
        rng = np.random.default_rng(seed)
        u = u + rng.uniform(-pert, pert, u.shape)
        v = v + rng.uniform(-pert, pert, v.shape)
        w = w + rng.uniform(-pert, pert, w.shape)
    return u, v, w, p


def taylor_green_decay(params, t):
    """Amplitude factor of the exact Taylor-Green solution at time t
    (wavenumber 2 pi in x and y): exp(-8 pi^2 nu t)."""
    return math.exp(-8.0 * math.pi ** 2 * t / params["re"])


def gaussian_velocity(params, sigma, seed):
    """i.i.d. N(0, sigma^2) on every padded entry of u, v, w."""
    rng = np.random.default_rng(seed)
    s = shape(params)
    return tuple(sigma * rng.standard_normal(s) for _ in range(3))


def random_field(params, seed, scale=1.0):
    rng = np.random.default_rng(seed)
    return scale * rng.standard_normal(shape(params))


def directions(params, count, seed):
    """``count`` Gaussian directions over (u, v, w), each normalised to unit
    2-norm over all padded entries (entries that are not unknowns are
    masked by the caller)."""
    rng = np.random.default_rng(seed)
    s = shape(params)
    out = []
    for _ in range(count):
        d = [rng.standard_normal(s) for _ in range(3)]
        out.append(d)
    return out


def batched_draws(count=64, seed=4, lo=24, hi=96, re_lo=50.0, re_hi=1000.0):
    """Per-instance (nx, ny, nz, Re): sizes integer-uniform in [lo, hi]
    inclusive, Re continuous-uniform in [re_lo, re_hi]."""
    rng = np.random.default_rng(seed)
    sizes = rng.integers(lo, hi + 1, size=(count, 3))
    res = rng.uniform(re_lo, re_hi, size=count)
    return [(int(s[0]), int(s[1]), int(s[2]), float(r)) for s, r in zip(sizes, res)]


def batched_64(count=64, seed=4):
    """64 cavities with mixed precision and adaptive dt (tau 0.5)."""
    out = []
    for nx, ny, nz, re in batched_draws(count, seed):
        p = cavity(nx, ny=ny, nz=nz, re=re, dt=0.0, tau=0.5)
        out.append(p)
    return out, 200
