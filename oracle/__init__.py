"""FP64 CPU oracle for the staggered-grid Navier-Stokes step.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this package; the product library
never does.  It wraps ``libns_oracle.so`` (plain C, built from
``ns_oracle.c`` with ``build()``) through ctypes and works on numpy arrays of
shape ``(nz+2, ny+2, nx+2)`` (x fastest, one ghost layer).

Every function follows the method the paper's CFD section states (eq. (1)
in "Background and Governing Equations": incompressible Navier-Stokes on a
regular staggered grid, finite differences in stencil form); the discrete
choices are documented in ``ns_oracle.c``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ns_oracle.c")
_LIB = os.path.join(_HERE, "libns_oracle.so")


def build(verbose: bool = False) -> str:
    """Compile the oracle with gcc (-O3 for any x86-64-v3 host, OpenMP, no FP
    contraction; without -ffast-math the optimiser keeps every rounding, so
    the results equal those of an unoptimised build)."""
    cmd = ["gcc", "-O3", "-march=x86-64-v3", "-std=c99", "-fopenmp", "-ffp-contract=off", "-fPIC",
           "-shared", "-Wall", "-o", _LIB + ".tmp", _SRC, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class _Cfg(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
        ("per", ctypes.c_int * 3),
        ("dx", ctypes.c_double), ("dy", ctypes.c_double), ("dz", ctypes.c_double),
        ("re", ctypes.c_double), ("dt", ctypes.c_double), ("tau", ctypes.c_double),
        ("gamma", ctypes.c_double), ("omega", ctypes.c_double), ("tol", ctypes.c_double),
        ("itermax", ctypes.c_int),
        ("wall", (ctypes.c_double * 3) * 6),
        ("g", ctypes.c_double * 3),
        ("eta", ctypes.c_double),
        ("advective", ctypes.c_int),
        ("stages", ctypes.c_int),
    ]


class Stats(ctypes.Structure):
    _fields_ = [
        ("t", ctypes.c_double), ("dt_last", ctypes.c_double), ("res_last", ctypes.c_double),
        ("sweeps_total", ctypes.c_longlong),
        ("steps", ctypes.c_int), ("sweeps_max", ctypes.c_int),
        ("steps_unconverged", ctypes.c_int), ("outer_max", ctypes.c_int),
    ]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.POINTER(ctypes.c_double)
        C = ctypes.POINTER(_Cfg)
        d = ctypes.c_double
        sig = {
            "nso_bc_vel": (None, [C, P, P, P]),
            "nso_p_ghosts": (None, [C, P]),
            "nso_fgh": (None, [C, d, P, P, P, P, P, P, P, P, P]),
            "nso_rhs": (None, [C, d, P, P, P, P]),
            "nso_residual": (d, [C, P, P, P]),
            "nso_rms": (d, [C, P]),
            "nso_sor_sweep": (None, [C, P, P, d]),
            "nso_sor_solve": (ctypes.c_int, [C, P, P, P]),
            "nso_sor_defect": (ctypes.c_int, [C, P, P, P, ctypes.POINTER(ctypes.c_int)]),
            "nso_project": (None, [C, d, P, P, P, P, P, P, P]),
            "nso_divergence": (None, [C, P, P, P, P]),
            "nso_dt": (d, [C, P, P, P]),
            "nso_run": (ctypes.c_int, [C, P, P, P, P, P, P, P, P, ctypes.c_int, ctypes.c_int,
                                       ctypes.POINTER(Stats)]),
            "nso_adj_project": (ctypes.c_int, [C, P, P, P, P, P]),
            "nso_adj_fgh": (None, [C, d, P, P, P, P, P, P, P, P, P]),
            "nso_threads": (ctypes.c_int, []),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _p(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


class Oracle:
    """One cavity / periodic box.  ``params`` uses the same keys as the
    product binding: nx, ny, nz, lx, ly, lz, re, dt, tau, gamma, omega, tol,
    itermax, bc (3 ints, 0 wall / 1 periodic), wall_vel (6x3), g (3), eta."""

    def __init__(self, params: dict):
        self.params = dict(params)
        c = _Cfg()
        c.nx, c.ny, c.nz = int(params["nx"]), int(params["ny"]), int(params["nz"])
        bc = params.get("bc", (0, 0, 0))
        for a in range(3):
            c.per[a] = int(bc[a])
        c.dx = params.get("lx", 1.0) / c.nx
        c.dy = params.get("ly", 1.0) / c.ny
        c.dz = params.get("lz", 1.0) / c.nz
        c.re = float(params["re"])
        c.dt = float(params["dt"])
        c.tau = float(params.get("tau", 0.5))
        c.gamma = float(params["gamma"])
        c.omega = float(params["omega"])
        c.tol = float(params["tol"])
        c.itermax = int(params["itermax"])
        wv = np.zeros((6, 3)) if params.get("wall_vel") is None else np.asarray(params["wall_vel"], float)
        for f in range(6):
            for q in range(3):
                c.wall[f][q] = float(wv[f, q])
        g = params.get("g", (0.0, 0.0, 0.0))
        for q in range(3):
            c.g[q] = float(g[q])
        c.eta = float(params.get("eta", 1e-2))
        c.advective = 1 if params.get("convection", "conservative") == "advective" else 0
        integ = params.get("integrator", "euler")
        if integ not in ("euler", "rk2"):
            raise ValueError(f"integrator must be 'euler' or 'rk2', not {integ!r}")
        c.stages = 2 if integ == "rk2" else 1
        self.cfg = c
        self.shape = (c.nz + 2, c.ny + 2, c.nx + 2)
        self.u, self.v, self.w, self.p = (np.zeros(self.shape) for _ in range(4))
        self.work = np.zeros((4,) + self.shape)
        self.force = [None, None, None]
        self.stats = Stats()

    # -- state -------------------------------------------------------------
    def field(self, name):
        return {"u": self.u, "v": self.v, "w": self.w, "p": self.p}[name]

    def set(self, name, arr):
        self.field(name)[...] = np.asarray(arr, dtype=np.float64)

    def set_force(self, fx, fy, fz):
        self.force = [None if f is None else np.ascontiguousarray(f, dtype=np.float64)
                      for f in (fx, fy, fz)]

    @property
    def F(self):
        return self.work[0]

    @property
    def G(self):
        return self.work[1]

    @property
    def H(self):
        return self.work[2]

    @property
    def rhs(self):
        return self.work[3]

    def run(self, nsteps: int, mode: int = 0) -> int:
        """``nsteps`` full steps; mode 0 = SOR, 1 = defect-correction form."""
        c = ctypes.byref(self.cfg)
        return lib().nso_run(c, _p(self.u), _p(self.v), _p(self.w), _p(self.p),
                             _p(self.force[0]), _p(self.force[1]), _p(self.force[2]),
                             _p(self.work), nsteps, mode, ctypes.byref(self.stats))

    # -- stages --------------------------------------------------------------
    def bc_vel(self, u=None, v=None, w=None):
        u = self.u if u is None else u
        v = self.v if v is None else v
        w = self.w if w is None else w
        lib().nso_bc_vel(ctypes.byref(self.cfg), _p(u), _p(v), _p(w))

    def p_ghosts(self, p=None):
        lib().nso_p_ghosts(ctypes.byref(self.cfg), _p(self.p if p is None else p))

    def fgh(self, dt, u=None, v=None, w=None):
        u = self.u if u is None else u
        v = self.v if v is None else v
        w = self.w if w is None else w
        F, G, H = (np.zeros(self.shape) for _ in range(3))
        lib().nso_fgh(ctypes.byref(self.cfg), dt, _p(u), _p(v), _p(w),
                      _p(self.force[0]), _p(self.force[1]), _p(self.force[2]), _p(F), _p(G), _p(H))
        return F, G, H

    def rhs_of(self, dt, F, G, H):
        r = np.zeros(self.shape)
        lib().nso_rhs(ctypes.byref(self.cfg), dt, _p(F), _p(G), _p(H), _p(r))
        return r

    def residual(self, p, rhs):
        r = np.zeros(self.shape)
        rms = lib().nso_residual(ctypes.byref(self.cfg), _p(p), _p(rhs), _p(r))
        return rms, r

    def rms(self, q):
        return lib().nso_rms(ctypes.byref(self.cfg), _p(q))

    def sor_sweep(self, p, rhs, omega=None):
        om = self.cfg.omega if omega is None else omega
        lib().nso_sor_sweep(ctypes.byref(self.cfg), _p(p), _p(rhs), om)

    def sor_solve(self, p, rhs):
        res = ctypes.c_double()
        n = lib().nso_sor_solve(ctypes.byref(self.cfg), _p(p), _p(rhs), ctypes.byref(res))
        return n, res.value

    def sor_defect(self, p, rhs):
        res = ctypes.c_double()
        outer = ctypes.c_int()
        n = lib().nso_sor_defect(ctypes.byref(self.cfg), _p(p), _p(rhs), ctypes.byref(res),
                                 ctypes.byref(outer))
        return n, res.value, outer.value

    def project(self, dt, F, G, H, p, u, v, w):
        lib().nso_project(ctypes.byref(self.cfg), dt, _p(F), _p(G), _p(H), _p(p), _p(u), _p(v), _p(w))

    def divergence(self, u=None, v=None, w=None):
        u = self.u if u is None else u
        v = self.v if v is None else v
        w = self.w if w is None else w
        d = np.zeros(self.shape)
        lib().nso_divergence(ctypes.byref(self.cfg), _p(u), _p(v), _p(w), _p(d))
        return d

    def dt_adaptive(self):
        return lib().nso_dt(ctypes.byref(self.cfg), _p(self.u), _p(self.v), _p(self.w))

    # -- adjoint ---------------------------------------------------------------
    def adj_project(self, lu, lv, lw, q=None):
        q = np.zeros(self.shape) if q is None else q
        rhs = np.zeros(self.shape)
        n = lib().nso_adj_project(ctypes.byref(self.cfg), _p(lu), _p(lv), _p(lw), _p(q), _p(rhs))
        return n

    def adj_fgh(self, dt, u, v, w, mu, mv, mw):
        ou, ov, ow = (np.zeros(self.shape) for _ in range(3))
        lib().nso_adj_fgh(ctypes.byref(self.cfg), dt, _p(u), _p(v), _p(w), _p(mu), _p(mv), _p(mw),
                          _p(ou), _p(ov), _p(ow))
        return ou, ov, ow


def threads() -> int:
    return lib().nso_threads()


def unknown_mask(params: dict, comp: int) -> np.ndarray:
    """Boolean mask of the unknowns of velocity component ``comp`` (0,1,2)
    or of the cells (comp = 3) in the padded layout."""
    n = [int(params["nx"]), int(params["ny"]), int(params["nz"])]
    bc = params.get("bc", (0, 0, 0))
    hi = list(n)
    if comp < 3 and not bc[comp]:
        hi[comp] = n[comp] - 1
    m = np.zeros((n[2] + 2, n[1] + 2, n[0] + 2), dtype=bool)
    m[1:hi[2] + 1, 1:hi[1] + 1, 1:hi[0] + 1] = True
    return m


def gradient(params: dict, u0, v0, w0, target, nsteps: int):
    """dL/du0 for L = 1/2 sum over the unknowns of (u^N - target)^2, by the
    reverse sweep: lambda^N = u^N - target, then for n = N-1..0
    mu = P lambda^{n+1} (transpose of the exact projection) and
    lambda^n = B^T J_Phi(u^n)^T mu.  Fixed dt only; the conservative form of
    the convective term only (the transpose is written for it).  The forward
    keeps every state (no checkpointing needed at oracle sizes)."""
    if params.get("convection", "conservative") != "conservative":
        raise ValueError("the oracle adjoint covers the conservative convective form only")
    o = Oracle(params)
    o.set("u", u0); o.set("v", v0); o.set("w", w0)
    o.bc_vel()
    states = []
    for _ in range(nsteps):
        states.append((o.u.copy(), o.v.copy(), o.w.copy()))
        o.run(1)
    masks = [unknown_mask(params, c) for c in range(3)]
    lam = [np.where(masks[c], f - t, 0.0) for c, (f, t) in enumerate(zip((o.u, o.v, o.w), target))]
    loss = 0.5 * sum(float(np.sum(l * l)) for l in lam)
    dt = float(params["dt"])
    q = np.zeros(o.shape)
    for n in range(nsteps - 1, -1, -1):
        o.adj_project(lam[0], lam[1], lam[2], q)
        lam = list(o.adj_fgh(dt, *states[n], lam[0], lam[1], lam[2]))
    return loss, lam, (o.u.copy(), o.v.copy(), o.w.copy())
