"""Writes mms_forcing.json: the manufactured solution used by the oracle's
order-of-accuracy pins and the body force that makes it an exact steady
solution of the incompressible Navier-Stokes equations (the paper's eq. (1)
with rho = 1):  f = (u.grad)u + grad p - nu lap u.

    u = sin^2(pi x) sin(2 pi y) sin(pi z)
    v = -sin(2 pi x) sin^2(pi y) sin(pi z)
    w = 0
    p = cos(pi x) cos(pi y) cos(pi z)

div u = 0; u, v, w vanish on every face of the unit cube; dp/dn = 0 there;
every tangential component is odd about each wall, so the ghost reflection
2*0 - u_interior reproduces the exact solution.  nu is left symbolic.
Run: python tests/golden/make_mms.py
"""
import json
import os

import sympy as sp

x, y, z, nu = sp.symbols("x y z nu")
u = sp.sin(sp.pi * x) ** 2 * sp.sin(2 * sp.pi * y) * sp.sin(sp.pi * z)
v = -sp.sin(2 * sp.pi * x) * sp.sin(sp.pi * y) ** 2 * sp.sin(sp.pi * z)
w = sp.Integer(0)
p = sp.cos(sp.pi * x) * sp.cos(sp.pi * y) * sp.cos(sp.pi * z)
vel = (u, v, w)
X = (x, y, z)
assert sp.simplify(sum(sp.diff(vel[a], X[a]) for a in range(3))) == 0
f = []
for c in range(3):
    conv = sum(vel[d] * sp.diff(vel[c], X[d]) for d in range(3))
    lap = sum(sp.diff(vel[c], X[d], 2) for d in range(3))
    f.append(sp.simplify(conv + sp.diff(p, X[c]) - nu * lap))
out = {"u": str(u), "v": str(v), "w": str(w), "p": str(p),
       "fx": str(f[0]), "fy": str(f[1]), "fz": str(f[2])}
with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "mms_forcing.json"), "w") as fh:
    json.dump(out, fh, indent=1)
print(json.dumps(out, indent=1))
