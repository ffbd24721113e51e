"""Independent constructions used to pin the oracle (not the oracle's code).

* The Neumann / periodic Poisson matrix is built from 1D second-difference
  matrices by Kronecker products (the textbook construction), not from the
  oracle's per-cell coefficient loop.
* Exact spectral solves use scipy's DCT-II (homogeneous Neumann on cell
  centres) and FFT (periodic), whose eigenvalues are the closed forms
  -(4/h^2) sin^2(pi m / 2n) and -(4/h^2) sin^2(pi m / n).
* Young's theory gives the asymptotic red-black SOR contraction from the
  Jacobi spectral radius mu.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.fft as sfft


def lap1d(n: int, h: float, periodic: bool) -> np.ndarray:
    """1D second difference on n cell centres; Neumann rows drop the missing
    neighbour (boundary elimination), periodic rows wrap."""
    A = np.zeros((n, n))
    for i in range(n):
        if i > 0:
            A[i, i - 1] += 1.0
            A[i, i] -= 1.0
        elif periodic:
            A[i, n - 1] += 1.0
            A[i, i] -= 1.0
        if i < n - 1:
            A[i, i + 1] += 1.0
            A[i, i] -= 1.0
        elif periodic:
            A[i, 0] += 1.0
            A[i, i] -= 1.0
    return A / (h * h)


def poisson_matrix(params) -> np.ndarray:
    """3D operator over interior cells, ordering (k, j, i) with i fastest."""
    n = (params["nx"], params["ny"], params["nz"])
    L = (params.get("lx", 1.0), params.get("ly", 1.0), params.get("lz", 1.0))
    bc = params.get("bc", (0, 0, 0))
    Ax, Ay, Az = (lap1d(n[a], L[a] / n[a], bool(bc[a])) for a in range(3))
    Ix, Iy, Iz = (np.eye(m) for m in n)
    return (np.kron(Iz, np.kron(Iy, Ax)) + np.kron(Iz, np.kron(Ay, Ix))
            + np.kron(Az, np.kron(Iy, Ix)))


def interior(a: np.ndarray) -> np.ndarray:
    return a[1:-1, 1:-1, 1:-1]


def dense_solve(params, rhs_interior: np.ndarray) -> np.ndarray:
    """Mean-zero solution of A p = rhs (singular Neumann / periodic system),
    by a bordered system [[A, 1], [1^T, 0]]."""
    A = poisson_matrix(params)
    N = A.shape[0]
    M = np.zeros((N + 1, N + 1))
    M[:N, :N] = A
    M[:N, N] = 1.0
    M[N, :N] = 1.0
    b = np.zeros(N + 1)
    b[:N] = rhs_interior.ravel()
    x = np.linalg.solve(M, b)
    return x[:N].reshape(rhs_interior.shape)


def spectral_solve(params, rhs_interior: np.ndarray) -> np.ndarray:
    """Mean-zero exact solve by diagonalisation: DCT-II on Neumann axes,
    FFT on periodic axes (all axes of one kind)."""
    n = (params["nx"], params["ny"], params["nz"])
    L = (params.get("lx", 1.0), params.get("ly", 1.0), params.get("lz", 1.0))
    bc = params.get("bc", (0, 0, 0))
    assert len(set(bc)) == 1
    periodic = bool(bc[0])
    lam = np.zeros(rhs_interior.shape)
    for a in range(3):
        h = L[a] / n[a]
        m = np.arange(n[a])
        if periodic:
            ev = -(4.0 / h ** 2) * np.sin(np.pi * m / n[a]) ** 2
        else:
            ev = -(4.0 / h ** 2) * np.sin(np.pi * m / (2 * n[a])) ** 2
        shape = [1, 1, 1]
        shape[2 - a] = n[a]
        lam = lam + ev.reshape(shape)
    if periodic:
        fh = np.fft.fftn(rhs_interior)
        lam[0, 0, 0] = 1.0
        fh = fh / lam
        fh[0, 0, 0] = 0.0
        return np.real(np.fft.ifftn(fh))
    fh = sfft.dctn(rhs_interior, type=2, norm="ortho")
    lam[0, 0, 0] = 1.0
    fh = fh / lam
    fh[0, 0, 0] = 0.0
    return sfft.idctn(fh, type=2, norm="ortho")


def jacobi_mu(params) -> float:
    """Largest Jacobi eigenvalue below 1 (the null mode excluded)."""
    A = poisson_matrix(params)
    d = -np.diag(A)
    S = (A + np.diag(d)) / np.sqrt(np.outer(d, d))  # symmetric similar of D^-1 N
    ev = np.linalg.eigvalsh(S)
    ev = ev[ev < 1.0 - 1e-10]
    return float(ev.max())


def young_rate(mu: float, omega: float) -> float:
    """Spectral radius of red-black SOR for a consistently ordered matrix:
    (lambda + omega - 1)^2 = lambda omega^2 mu^2; past omega_opt the
    eigenvalues are complex with modulus omega - 1."""
    disc = omega * omega * mu * mu - 4.0 * (omega - 1.0)
    if disc < 0:
        return omega - 1.0
    return ((omega * mu + math.sqrt(disc)) / 2.0) ** 2


def rel(a, b) -> float:
    """max |a - b| / max |b|"""
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))
