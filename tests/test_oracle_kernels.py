"""Pins of the oracle's fundamental solutions against closed forms and invariants.

Sec. 2.1 gives U_ij, T_ij = G_ikj n_k and phi/psi; these tests check the
oracle's Laplace-domain reading of them without re-typing its formulas:
Kelvin's static solution (textbook, written out in oracle.closed_form),
Hooke's law applied to finite differences of U, the Navier equation
mu Lap u + (lam + mu) grad div u = rho s^2 u, symmetries, and agreement of the
small-|z| series with the closed form where both are accurate.
"""

import numpy as np
import pytest

from oracle import kernels as K
from oracle import closed_form as CF

def _pairs(n=6, scale=0.8, seed=1212):
    RNG = np.random.default_rng(seed)
    x = RNG.standard_normal((n, 3))
    d = RNG.standard_normal((n, 3))
    d *= scale / np.linalg.norm(d, axis=1, keepdims=True) * RNG.uniform(0.3, 2.0, (n, 1))
    nrm = RNG.standard_normal((n, 3))
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    return x, x + d, nrm


def _rel(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


# ---- pins written as functions so that the planted-mistake tests reuse them


def kelvin_gap(s, mat):
    x, y, n = _pairs()
    eU = _rel(K.U_kernel(x, y, s, mat), CF.kelvin_U(x, y, mat))
    eT = _rel(K.T_kernel(x, y, n, s, mat), CF.kelvin_T(x, y, n, mat))
    return eU, eT


def hooke_gap(s, mat, h=1e-4):
    """max |T - T_hooke| / max |T| with T_hooke from central differences of U
    in the field point: sigma_jk = lam delta_jk dU_il/dy_l
    + mu (dU_ij/dy_k + dU_ik/dy_j), T_ij = sigma_jk n_k."""
    x, y, n = _pairs()
    h = h / max(1.0, abs(s))      # keep the step small against the wavelength
    lam, mu = mat["lam"], mat["mu"]
    dU = np.zeros((len(x), 3, 3, 3), np.complex128)   # [p, i, j, k] = dU_ij/dy_k
    for k in range(3):
        e = np.zeros(3)
        e[k] = h
        dU[..., k] = (K.U_kernel(x, y + e, s, mat) - K.U_kernel(x, y - e, s, mat)) / (2 * h)
    div = np.einsum("pill->pi", dU)
    sig = (lam * div[:, :, None, None] * np.eye(3)[None, None]
           + mu * (dU + np.swapaxes(dU, 2, 3)))              # [p, i, j, k]
    Th = np.einsum("pijk,pk->pij", sig, n)
    T = K.T_kernel(x, y, n, s, mat)
    return _rel(T, Th)


def navier_gap(s, mat, h=2e-3):
    """Residual of mu Lap u + (lam+mu) grad div u - rho s^2 u for the field
    u_j(y) = U_ij(x, y), relative to the size of mu Lap u."""
    x, y, _ = _pairs(4)
    lam, mu, rho = mat["lam"], mat["mu"], mat["rho"]
    E = np.eye(3) * h
    u0 = K.U_kernel(x, y, s, mat)
    lap = np.zeros_like(u0)
    for k in range(3):
        lap += (K.U_kernel(x, y + E[k], s, mat) - 2 * u0 + K.U_kernel(x, y - E[k], s, mat)) / h ** 2
    # grad div: d/dy_j sum_k dU_ik/dy_k
    gd = np.zeros_like(u0)
    for j in range(3):
        for k in range(3):
            f = lambda a, b: K.U_kernel(x, y + a * E[j] + b * E[k], s, mat)[:, :, k]
            if j == k:
                d2 = (K.U_kernel(x, y + E[k], s, mat)[:, :, k] - 2 * u0[:, :, k]
                      + K.U_kernel(x, y - E[k], s, mat)[:, :, k]) / h ** 2
            else:
                d2 = (f(1, 1) - f(1, -1) - f(-1, 1) + f(-1, -1)) / (4 * h * h)
            gd[:, :, j] += d2
    res = mu * lap + (lam + mu) * gd - rho * s * s * u0
    return np.abs(res).max() / np.abs(mu * lap).max()


# ---- the pins


def test_static_limit_is_kelvin_exactly(mat):
    """At s = 0 only the n = 2 terms survive: U and T are Kelvin's kernels."""
    eU, eT = kelvin_gap(0.0, mat)
    assert eU < 1e-14 and eT < 1e-14


def test_kelvin_limit_rates(mat):
    """U - U_Kelvin = O(s) (a rigid-translation term), T - T_Kelvin = O(s^2)."""
    eU1, eT1 = kelvin_gap(1e-2, mat)
    eU2, eT2 = kelvin_gap(1e-3, mat)
    assert 8.0 < eU1 / eU2 < 12.0
    assert 80.0 < eT1 / eT2 < 120.0
    assert eT2 < 1e-6


@pytest.mark.parametrize("s", [0.75, 0.75 + 3.0j, 0.75 + 25.0j, 0.05 + 0.05j, 2.0 - 1.0j])
def test_traction_is_hooke_of_displacement(mat, s):
    assert hooke_gap(s, mat) < 2e-7


@pytest.mark.parametrize("s", [0.75, 0.75 + 3.0j, 0.3 + 8.0j])
def test_displacement_solves_navier(mat, s):
    """The finite-difference residual vanishes as O(h^2)."""
    e1 = navier_gap(s, mat, h=1e-3)
    e2 = navier_gap(s, mat, h=5e-4)
    assert e2 < 1e-5
    assert 3.5 < e1 / e2 < 4.5


def test_symmetries(mat):
    x, y, n = _pairs()
    for s in (0.75 + 2.0j, 0.1 + 0.02j):
        U = K.U_kernel(x, y, s, mat)
        assert np.abs(U - np.swapaxes(U, 1, 2)).max() < 1e-15 * np.abs(U).max() + 1e-300
        assert _rel(K.U_kernel(y, x, s, mat), U) < 1e-14
        T = K.T_kernel(x, y, n, s, mat)
        assert _rel(-K.T_kernel(y, x, n, s, mat), T) < 1e-14
        assert _rel(K.U_kernel(x, y, np.conj(s), mat), np.conj(U)) < 1e-14
        assert _rel(K.T_kernel(x, y, n, np.conj(s), mat), np.conj(T)) < 1e-14


def test_series_matches_closed_form(mat):
    for s in (0.75 + 0.3j, 1.0, 0.2 + 0.9j, -0.3 + 0.5j):
        r = np.linspace(0.15, 1.0, 40) / abs(s)
        a = K.radial(r, s, mat, force="series")
        b = K.radial(r, s, mat, force="direct")
        for p, q in zip(a, b):
            assert np.abs(p - q).max() < 1e-12


def test_series_tail_is_small_near_zero(mat):
    """The static terms carry the singular part: the tails vanish as r -> 0."""
    r = np.array([1e-6, 1e-4, 1e-2])
    rphi, rpsi, r2dphi, r2dpsi = K.radial(r, 0.75 + 2j, mat, tail=True)
    assert np.abs(rphi[0]) < 1e-5 and np.abs(rpsi[0]) < 1e-10
    assert np.abs(r2dphi[0]) < 1e-10 and np.abs(r2dpsi[0]) < 1e-10


def test_gamma_squared_reading(mat):
    """Without the factor gamma^2 on the P-wave terms (as printed) U blows
    up as s -> 0; with it U tends to Kelvin."""
    x, y, _ = _pairs(3)
    s = 1e-3
    g = mat["gamma"]
    r = np.linalg.norm(y - x, axis=1)
    z = s * r / mat["cs"]
    zp = g * z
    printed = (np.exp(-z) * (1 + 1 / z + 1 / z ** 2) - np.exp(-zp) * (1 / zp + 1 / zp ** 2)) / r
    kel = (3 - 4 * mat["nu"]) / (4 * (1 - mat["nu"]) * r)
    assert np.abs(printed - kel).max() > 1e3
    assert np.abs(K.radial(r, s, mat)[0] / r - kel).max() < 1e-2


# ---- planted mistakes: each must be caught by one of the pins above


def test_planted_missing_gamma_is_caught(mat, monkeypatch):
    orig = K._direct

    def bad(z, g):
        zs, zp = z, g * z
        es, ep = np.exp(-zs), np.exp(-zp)
        out = list(orig(z, g))
        out[0] = es * (1 + 1 / zs + 1 / zs ** 2) - ep * (1 / zp + 1 / zp ** 2)
        return tuple(out)

    monkeypatch.setattr(K, "_direct", bad)
    assert navier_gap(0.75 + 3.0j, mat) > 1e-2


def test_planted_sign_error_in_T_is_caught(mat, monkeypatch):
    orig = K.radial

    def bad(r, s, m, tail=False, force=None):
        a, b, c, d = orig(r, s, m, tail=tail, force=force)
        return a, b, c, -d

    monkeypatch.setattr(K, "radial", bad)
    assert hooke_gap(0.75 + 3.0j, mat) > 1e-2
    assert kelvin_gap(0.0, mat)[1] > 1e-2


def test_planted_series_error_is_caught(mat, monkeypatch):
    orig = K.series_coefficients

    def bad(g, n_terms=K.N_SERIES):
        a, b, c, d = orig(g, n_terms)
        a = list(a)
        a[3] *= 1.01
        return a, b, c, d

    monkeypatch.setattr(K, "series_coefficients", bad)
    r = np.linspace(0.15, 1.0, 10)
    a = K.radial(r, 1.0, mat, force="series")
    b = K.radial(r, 1.0, mat, force="direct")
    assert np.abs(a[0] - b[0]).max() > 1e-6
