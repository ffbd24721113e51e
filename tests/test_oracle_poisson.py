"""Pins of the oracle's Poisson operator and red-black SOR (no GPU).

The operator is pinned by a dense direct solve of an independently built
Kronecker-product matrix and by exact DCT / FFT diagonalisation; the SOR
ordering and relaxation by Young's theory of red-black SOR.
"""
import numpy as np
import pytest

import nsworkloads as W
from tests import _pins

pytestmark = pytest.mark.filterwarnings("ignore")


def _prm(nx, ny, nz, bc, lx=1.0, ly=1.0, lz=1.0, tol=1e-13, itermax=20000, omega=1.7):
    p = W.cavity(nx, ny=ny, nz=nz, tol=tol, itermax=itermax, omega=omega)
    p.update(bc=bc, lx=lx, ly=ly, lz=lz)
    return p


def _zero_mean_rhs(params, seed):
    r = W.random_field(params, seed)
    core = r[1:-1, 1:-1, 1:-1]
    core -= core.mean()
    return r


@pytest.mark.parametrize("dims,bc,ext", [
    ((8, 8, 8), (0, 0, 0), (1.0, 1.0, 1.0)),
    ((8, 6, 5), (0, 0, 0), (1.0, 0.7, 1.3)),
    ((8, 6, 4), (1, 1, 1), (1.0, 0.7, 1.3)),
    ((6, 8, 5), (1, 0, 0), (1.2, 1.0, 0.8)),
    ((7, 6, 5), (0, 1, 0), (1.0, 1.0, 1.0)),
])
def test_sor_fixed_point_matches_dense_solve(oracle_mod, dims, bc, ext):
    prm = _prm(*dims, bc=bc, lx=ext[0], ly=ext[1], lz=ext[2])
    o = oracle_mod.Oracle(prm)
    rhs = _zero_mean_rhs(prm, 11)
    p = np.zeros(o.shape)
    n, res = o.sor_solve(p, rhs)
    assert n < prm["itermax"]
    got = _pins.interior(p) - _pins.interior(p).mean()
    want = _pins.dense_solve(prm, _pins.interior(rhs))
    assert _pins.rel(got, want) < 1e-10


@pytest.mark.parametrize("n,bc", [(16, (0, 0, 0)), (24, (0, 0, 0)), (16, (1, 1, 1))])
def test_sor_fixed_point_matches_spectral_solve(oracle_mod, n, bc):
    prm = _prm(n, n - 4 if not bc[0] else n, n + 4 if not bc[0] else n, bc=bc,
               lx=1.0, ly=0.8, lz=1.1)
    o = oracle_mod.Oracle(prm)
    rhs = _zero_mean_rhs(prm, 12)
    p = np.zeros(o.shape)
    o.sor_solve(p, rhs)
    got = _pins.interior(p) - _pins.interior(p).mean()
    want = _pins.spectral_solve(prm, _pins.interior(rhs))
    assert _pins.rel(got, want) < 1e-10


def test_residual_is_the_kronecker_operator(oracle_mod):
    prm = _prm(7, 6, 5, bc=(0, 0, 0), lx=1.0, ly=0.6, lz=1.4)
    o = oracle_mod.Oracle(prm)
    p = W.random_field(prm, 3)
    rhs = W.random_field(prm, 4)
    rms, r = o.residual(p, rhs)
    A = _pins.poisson_matrix(prm)
    want = (A @ _pins.interior(p).ravel() - _pins.interior(rhs).ravel()).reshape(5, 6, 7)
    assert _pins.rel(_pins.interior(r), want) < 1e-13
    assert abs(rms - np.sqrt(np.mean(want ** 2))) < 1e-12 * rms


@pytest.mark.parametrize("bc,dims,omega", [
    ((0, 0, 0), (12, 10, 8), 1.2),
    ((0, 0, 0), (12, 10, 8), 1.0),
    ((1, 1, 1), (8, 8, 8), 1.25),
])
def test_red_black_sor_rate_matches_young(oracle_mod, bc, dims, omega):
    prm = _prm(*dims, bc=bc, omega=omega)
    o = oracle_mod.Oracle(prm)
    rhs = _zero_mean_rhs(prm, 21)
    p = W.random_field(prm, 22)
    res = [o.residual(p, rhs)[0]]
    # stop well before round-off so the ratio is the asymptotic one
    while res[-1] > 1e-9 * res[0] and len(res) < 400:
        o.sor_sweep(p, rhs)
        res.append(o.residual(p, rhs)[0])
    ratio = res[-1] / res[-2]
    theory = _pins.young_rate(_pins.jacobi_mu(prm), omega)
    assert abs(ratio - theory) < 2e-3 * theory, (ratio, theory)


def test_overrelaxed_rate_is_omega_minus_one(oracle_mod):
    # omega above omega_opt: all SOR eigenvalues have modulus omega - 1.
    prm = _prm(8, 8, 8, bc=(1, 1, 1), omega=1.7)
    o = oracle_mod.Oracle(prm)
    rhs = _zero_mean_rhs(prm, 31)
    p = W.random_field(prm, 32)
    res = []
    for _ in range(50):
        o.sor_sweep(p, rhs)
        res.append(o.residual(p, rhs)[0])
    gm = (res[-1] / res[-31]) ** (1.0 / 30.0)
    assert abs(gm - 0.7) < 0.02 * 0.7, gm


def test_zero_rhs_needs_no_sweep(oracle_mod):
    prm = _prm(6, 6, 6, bc=(0, 0, 0))
    o = oracle_mod.Oracle(prm)
    p = W.random_field(prm, 5)
    p0 = p.copy()
    n, res = o.sor_solve(p, np.zeros(o.shape))
    assert n == 0 and res == 0.0
    assert np.array_equal(p, p0)


def test_stop_rule_first_sweep_below_tolerance(oracle_mod):
    prm = _prm(10, 10, 10, bc=(0, 0, 0), tol=1e-5, itermax=500)
    o = oracle_mod.Oracle(prm)
    rhs = _zero_mean_rhs(prm, 41)
    p = np.zeros(o.shape)
    n, res = o.sor_solve(p, rhs)
    thr = prm["tol"] * o.rms(rhs)
    assert res <= thr
    # one sweep fewer does not meet the tolerance
    q = np.zeros(o.shape)
    for _ in range(n - 1):
        o.sor_sweep(q, rhs)
    assert o.residual(q, rhs)[0] > thr


def test_defect_correction_reaches_dense_solution(oracle_mod):
    prm = _prm(8, 8, 8, bc=(0, 0, 0), tol=1e-12, itermax=5000)
    o = oracle_mod.Oracle(prm)
    rhs = _zero_mean_rhs(prm, 51)
    p = np.zeros(o.shape)
    n, res, outer = o.sor_defect(p, rhs)
    assert outer >= 3 and res <= 1e-12 * o.rms(rhs)
    got = _pins.interior(p) - _pins.interior(p).mean()
    want = _pins.dense_solve(prm, _pins.interior(rhs))
    assert _pins.rel(got, want) < 1e-9


@pytest.mark.parametrize("eta,tol", [(0.1, 1e-9), (0.03, 1e-11)])
def test_defect_correction_inner_stop_rule(oracle_mod, eta, tol):
    """Replay of the defect-correction solve with every residual taken from
    the Kronecker-product matrix: outer residual r = rhs - A p; the inner
    sweeps on A e = r start from e = 0 and stop at the first sweep with
    RMS(r - A e) <= eta RMS(r); then p += e; the outer loop stops once
    RMS(r) <= tol RMS(rhs).  The oracle's sweep and outer counts and its
    pressure must equal the replay's (an inner rule one sweep early or
    late, or measured against RMS(rhs), changes the counts)."""
    prm = _prm(7, 6, 5, bc=(0, 0, 0), lx=1.0, ly=0.8, lz=1.2, tol=tol, itermax=5000)
    prm["eta"] = eta
    o = oracle_mod.Oracle(prm)
    rhs = _zero_mean_rhs(prm, 61)
    p0 = W.random_field(prm, 62, 0.1)
    p = p0.copy()
    n, res, outer = o.sor_defect(p, rhs)

    A = _pins.poisson_matrix(prm)
    b = _pins.interior(rhs).ravel()
    rms = lambda x: float(np.sqrt(np.mean(x * x)))
    thr = tol * rms(b)
    q = p0.copy()
    sweeps = outers = 0
    inner_counts = []
    while True:
        r = b - A @ _pins.interior(q).ravel()
        ro = rms(r)
        if ro <= thr or sweeps >= prm["itermax"]:
            break
        outers += 1
        rf = np.zeros(o.shape)
        _pins.interior(rf)[...] = r.reshape(5, 6, 7)
        e = np.zeros(o.shape)
        k = 0
        prev = None
        while sweeps < prm["itermax"]:
            o.sor_sweep(e, rf)
            sweeps += 1
            k += 1
            re_ = rms(r - A @ _pins.interior(e).ravel())
            if re_ <= eta * ro:
                assert prev is None or prev > eta * ro
                break
            prev = re_
        inner_counts.append(k)
        _pins.interior(q)[...] += _pins.interior(e)
    assert outers >= 3 and min(inner_counts) >= 2, inner_counts
    assert (n, outer) == (sweeps, outers), ((n, outer), (sweeps, outers), inner_counts)
    assert abs(res - ro) <= 1e-6 * ro
    assert _pins.rel(_pins.interior(p), _pins.interior(q)) < 1e-12
