"""Python front end of libns.so: parameter marshalling, torch tensors for
device memory, the current torch stream as the handle's stream, and the
reverse-mode gradient as a torch.autograd.Function.

Nothing here computes any part of the step; it only moves arguments.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import abi


def make_params(prm: dict) -> abi.ns_params:
    """dict (keys as in the oracle / workload dictionaries) -> ns_params."""
    p = abi.ns_params()
    abi.check(abi.ns_params_default(p))
    p.nx, p.ny, p.nz = int(prm["nx"]), int(prm["ny"]), int(prm["nz"])
    p.lx, p.ly, p.lz = float(prm.get("lx", 1.0)), float(prm.get("ly", 1.0)), float(prm.get("lz", 1.0))
    p.re = float(prm["re"])
    p.dt = float(prm["dt"])
    p.tau = float(prm.get("tau", 0.5))
    p.gamma = float(prm["gamma"])
    p.omega = float(prm["omega"])
    p.tol = float(prm["tol"])
    p.itermax = int(prm["itermax"])
    bc = prm.get("bc", (0, 0, 0))
    for a in range(3):
        p.bc[a] = int(bc[a])
    wv = np.zeros((6, 3)) if prm.get("wall_vel") is None else np.asarray(prm["wall_vel"], float)
    for f in range(6):
        for c in range(3):
            p.wall_vel[f][c] = float(wv[f, c])
    g = prm.get("g", (0.0, 0.0, 0.0))
    for c in range(3):
        p.g[c] = float(g[c])
    p.eta = float(prm.get("eta", 1e-2))
    prec = prm.get("precision", "fp64")
    p.precision = abi.NS_MIXED if prec in ("mixed", abi.NS_MIXED) else abi.NS_FP64
    p.checkpoint_every = int(prm.get("checkpoint_every", 0))
    p.flags = int(prm.get("flags", 0))
    if prm.get("convection", "conservative") == "advective":
        p.flags |= abi.NS_ADVECTIVE
    integ = prm.get("integrator", "euler")
    if integ not in ("euler", "rk2"):
        raise ValueError(f"integrator must be 'euler' or 'rk2', not {integ!r}")
    if integ == "rk2":
        p.flags |= abi.NS_RK2
    tile = prm.get("tile", (0, 0))
    p.tile[0], p.tile[1] = int(tile[0]), int(tile[1])
    return p


class Solver:
    """One libns handle over one or more independent domains.

    Fields are exchanged as float64 tensors of shape (nz+2, ny+2, nx+2) on
    the torch device (default ``cuda:0``), on the torch stream current at
    construction."""

    def __init__(self, params, device="cuda:0", stream=None):
        if isinstance(params, dict):
            params = [params]
        self.params = [dict(p) for p in params]
        self.device = torch.device(device)
        arr = (abi.ns_params * len(params))(*[make_params(p) for p in params])
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self.stream = stream
        self.handle = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            abi.check(abi.ns_create(arr, len(params), stream.cuda_stream, self.handle))
        self.n = len(params)
        self._stats = (abi.ns_stats * self.n)()

    def shape(self, inst=0):
        p = self.params[inst]
        return (p["nz"] + 2, p["ny"] + 2, p["nx"] + 2)

    def set(self, name, value, inst=0):
        t = torch.as_tensor(value, dtype=torch.float64, device=self.device).contiguous()
        if tuple(t.shape) != self.shape(inst):
            raise ValueError(f"{name}: expected shape {self.shape(inst)}, got {tuple(t.shape)}")
        self.stream.synchronize() if t.device != self.device else None
        torch.cuda.current_stream(self.device).synchronize()
        abi.check(abi.ns_set_state(self.handle, inst, abi.FIELD_IDS[name], t.data_ptr(), 1), self.handle)

    def get(self, name, inst=0) -> torch.Tensor:
        t = torch.empty(self.shape(inst), dtype=torch.float64, device=self.device)
        torch.cuda.current_stream(self.device).synchronize()
        abi.check(abi.ns_get_state(self.handle, inst, abi.FIELD_IDS[name], t.data_ptr(), 1), self.handle)
        return t

    def get_np(self, name, inst=0) -> np.ndarray:
        return self.get(name, inst).cpu().numpy()

    def step(self, nsteps=1, check=True) -> int:
        code = abi.ns_step(self.handle, nsteps, self._stats)
        if check:
            abi.check(code, self.handle)
        return code

    def stats(self, inst=0) -> dict:
        return self._stats[inst].as_dict()

    def timing(self) -> abi.ns_timing:
        t = abi.ns_timing()
        abi.check(abi.ns_get_timing(self.handle, t), self.handle)
        return t

    def backward(self, g_final, inst=0):
        gf = [torch.as_tensor(g, dtype=torch.float64, device=self.device).contiguous() for g in g_final]
        gi = [torch.zeros(self.shape(inst), dtype=torch.float64, device=self.device) for _ in range(3)]
        torch.cuda.current_stream(self.device).synchronize()
        abi.check(abi.ns_backward(self.handle, inst, [t.data_ptr() for t in gf],
                                  [t.data_ptr() for t in gi], 1), self.handle)
        return gi

    def last_error(self) -> str:
        return abi.ns_last_error(self.handle)

    def close(self):
        if self.handle:
            abi.ns_destroy(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class NSRollout(torch.autograd.Function):
    """(u0, v0, w0) -> (u, v, w) after ``nsteps`` steps of one FP64 domain
    with checkpointing; backward runs the library's hand-written adjoint
    (ns_backward).  ``params`` must have a fixed dt and checkpoint_every > 0."""

    @staticmethod
    def forward(ctx, u0, v0, w0, params, nsteps):
        s = Solver(params, device=u0.device)
        s.set("u", u0.detach()); s.set("v", v0.detach()); s.set("w", w0.detach())
        s.step(nsteps)
        ctx.solver = s
        return s.get("u"), s.get("v"), s.get("w")

    @staticmethod
    def backward(ctx, gu, gv, gw):
        s = ctx.solver
        g = s.backward([gu, gv, gw])
        s.close()
        return g[0], g[1], g[2], None, None
