"""Laplace-domain elastodynamic fundamental solutions (oracle; test infrastructure).

Sec. 2.1 defines the displacement kernel U_ij = (phi delta_ij - psi r_i r_j)
/ (4 pi mu) and the traction kernel T_ij = G_ikj n_k(y), with phi and psi
built from exp(i k r) terms in the wavenumbers k_s = omega/c_s and
k_p = omega/c_p.  This module writes them in the Laplace variable
s = sigma + i omega_k used by the exponential window (Sec. 3.1): i k r becomes
-s r / c, so with z_s = s r / c_s, z_p = s r / c_p and gamma = c_s / c_p

  r phi = e^{-z_s}(1 + 1/z_s + 1/z_s^2) - gamma^2 e^{-z_p}(1/z_p + 1/z_p^2)
  r psi = e^{-z_s}(1 + 3/z_s + 3/z_s^2) - gamma^2 e^{-z_p}(1 + 3/z_p + 3/z_p^2)

Readings of the printed formulas (each pinned by a test):
  * the P-wave terms of phi and psi carry the factor gamma^2; without it U
    does not reduce to the Kelvin solution as s -> 0;
  * r_i in U_ij and in G_ikj is the unit vector (y - x)/|y - x|, pointing
    from the source point x to the field point y; the 1/(4 pi r) prefactor of
    G_ikj together with non-unit r_i is the same thing;
  * derivatives are taken with respect to the field point y, so T_ij is the
    traction at y (normal n(y)) of the field of a unit force at x along i.

T_ij expands to (1/4pi)[A(delta_ij dr/dn + rh_j n_i) + B rh_i rh_j dr/dn
+ C rh_i n_j] with A = phi' - psi/r, B = 2(2 psi/r - psi'),
C = (c_p/c_s)^2 (phi' - psi' - 2 psi/r) - 2 (phi' - psi' - psi/r).

For |z_s| < SERIES_Z the closed forms cancel catastrophically, so the Taylor
series of r phi, r psi, r^2 phi', r^2 psi' in z = z_s is used instead:
  r phi     = sum_{n>=2} (-1)^n (n-1)(n-1+gamma^n) z^{n-2} / n!
  r psi     = sum_{n>=2} (-1)^n (n-1)(n-3)(1-gamma^n) z^{n-2} / n!
  r^2 phi'  = sum (n-3) * [coefficient of r phi] z^{n-2}, likewise psi.
The n = 2 terms are the static (Kelvin) parts.
"""

from math import factorial, pi, sqrt

import numpy as np

SERIES_Z = 0.5
N_SERIES = 30


def material(rho, mu, nu):
    """Lame constant, wave speeds and gamma = c_s/c_p (Sec. 2.1)."""
    lam = 2.0 * mu * nu / (1.0 - 2.0 * nu)
    cs = sqrt(mu / rho)
    cp = sqrt((lam + 2.0 * mu) / rho)
    return dict(rho=rho, mu=mu, nu=nu, lam=lam, cs=cs, cp=cp, gamma=cs / cp)


def series_coefficients(g, n_terms=N_SERIES):
    """Coefficients (index m = n - 2) of r phi, r psi, r^2 phi', r^2 psi'."""
    c_phi, c_psi, c_dphi, c_dpsi = [], [], [], []
    for n in range(2, n_terms + 2):
        c = (-1.0) ** n / factorial(n)
        cphi = c * (n - 1) * (n - 1 + g ** n)
        cpsi = c * (n - 1) * (n - 3) * (1.0 - g ** n)
        c_phi.append(cphi)
        c_psi.append(cpsi)
        c_dphi.append((n - 3) * cphi)
        c_dpsi.append((n - 3) * cpsi)
    return c_phi, c_psi, c_dphi, c_dpsi


def _series(z, g):
    out = []
    for coef in series_coefficients(g):
        acc = np.zeros_like(z)
        for c in reversed(coef):          # Horner
            acc = acc * z + c
        out.append(acc)
    return tuple(out)


def _direct(z, g):
    zs = z
    zp = g * z
    es = np.exp(-zs)
    ep = np.exp(-zp)
    g2 = g * g
    rphi = es * (1 + 1 / zs + 1 / zs ** 2) - g2 * ep * (1 / zp + 1 / zp ** 2)
    rpsi = es * (1 + 3 / zs + 3 / zs ** 2) - g2 * ep * (1 + 3 / zp + 3 / zp ** 2)
    r2dphi = -rphi - (es * (zs + 1 + 2 / zs + 2 / zs ** 2)
                      - g2 * ep * (1 + 2 / zp + 2 / zp ** 2))
    r2dpsi = -rpsi - (es * (zs + 3 + 6 / zs + 6 / zs ** 2)
                      - g2 * ep * (zp + 3 + 6 / zp + 6 / zp ** 2))
    return rphi, rpsi, r2dphi, r2dpsi


def static_terms(g):
    """n = 2 (Kelvin) terms of r phi, r psi, r^2 phi', r^2 psi'."""
    a2 = (1.0 + g * g) / 2.0
    b2 = -(1.0 - g * g) / 2.0
    return a2, b2, -a2, -b2


def radial(r, s, mat, tail=False, force=None):
    """r*phi, r*psi, r^2*phi', r^2*psi' at distances ``r`` and complex ``s``.

    ``tail=True`` drops the static n = 2 terms (the part that stays bounded
    at r -> 0).  ``force`` = "series" or "direct" selects one branch for all
    points (used by tests); by default |z_s| < SERIES_Z uses the series."""
    r = np.asarray(r, dtype=np.float64)
    g = mat["gamma"]
    z = (complex(s) / mat["cs"]) * r.astype(np.complex128)
    if force == "series":
        small = np.ones(z.shape, bool)
    elif force == "direct":
        small = np.zeros(z.shape, bool)
    else:
        small = np.abs(z) < SERIES_Z
    out = [np.zeros(z.shape, np.complex128) for _ in range(4)]
    if small.any():
        vals = _series(z[small], g)
        for o, v in zip(out, vals):
            o[small] = v
    big = ~small
    if big.any():
        vals = _direct(z[big], g)
        for o, v in zip(out, vals):
            o[big] = v
    if tail:
        for o, st in zip(out, static_terms(g)):
            o -= st
    return tuple(out)


def _geom(x, y):
    d = np.asarray(y, dtype=np.float64) - np.asarray(x, dtype=np.float64)
    r = np.linalg.norm(d, axis=-1)
    rh = d / r[..., None]
    return r, rh


def U_kernel(x, y, s, mat, tail=False):
    """U_ij(x, y; s), shape (..., 3, 3); i = force direction at x."""
    r, rh = _geom(x, y)
    rphi, rpsi, _, _ = radial(r, s, mat, tail=tail)
    phi = rphi / r
    psi = rpsi / r
    eye = np.eye(3)
    U = (phi[..., None, None] * eye
         - psi[..., None, None] * rh[..., :, None] * rh[..., None, :])
    return U / (4.0 * pi * mat["mu"])


def T_kernel(x, y, ny, s, mat, tail=False):
    """T_ij(x, y; n(y), s), shape (..., 3, 3): traction component j at y on
    the surface with normal n(y), for a unit force at x along i."""
    r, rh = _geom(x, y)
    n = np.broadcast_to(np.asarray(ny, dtype=np.float64), rh.shape)
    rphi, rpsi, r2dphi, r2dpsi = radial(r, s, mat, tail=tail)
    psi = rpsi / r
    dphi = r2dphi / r ** 2
    dpsi = r2dpsi / r ** 2
    A = dphi - psi / r
    B = 2.0 * (2.0 * psi / r - dpsi)
    ratio = (mat["cp"] / mat["cs"]) ** 2
    C = ratio * (dphi - dpsi - 2.0 * psi / r) - 2.0 * (dphi - dpsi - psi / r)
    drdn = np.einsum("...k,...k->...", rh, n)
    eye = np.eye(3)
    T = (A[..., None, None] * (eye * drdn[..., None, None]
                               + n[..., :, None] * rh[..., None, :])
         + (B * drdn)[..., None, None] * rh[..., :, None] * rh[..., None, :]
         + C[..., None, None] * rh[..., :, None] * n[..., None, :])
    return T / (4.0 * pi)


def T_static_flat(x, y, ny, mat):
    """Static traction kernel when dr/dn = 0 (field point in the plane of a
    flat element through x): gamma^2/(4 pi r^2) (rh_i n_j - rh_j n_i)."""
    r, rh = _geom(x, y)
    n = np.broadcast_to(np.asarray(ny, dtype=np.float64), rh.shape)
    g2 = mat["gamma"] ** 2
    K = rh[..., :, None] * n[..., None, :] - n[..., :, None] * rh[..., None, :]
    return (g2 / (4.0 * pi * r ** 2))[..., None, None] * K
