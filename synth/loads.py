"""Seeded load inputs: per-element pressure amplitudes and sampled histories."""

import numpy as np
from scipy import special


def ramp_history(n_f, period, t_rise):
    """Samples ``P(n dt) = min(n dt / t_rise, 1)`` for ``n = 0..n_f-1`` with
    ``dt = period / n_f`` (a Heaviside step with a linear rise)."""
    t = np.arange(n_f, dtype=np.float64) * (period / n_f)
    if t_rise <= 0:
        return (t > 0).astype(np.float64)
    return np.minimum(t / t_rise, 1.0)


def ricker_history(n_f, period, fc, delay):
    """Ricker wavelet ``(1 - 2 a) exp(-a)``, ``a = (pi fc (t - delay))^2``."""
    t = np.arange(n_f, dtype=np.float64) * (period / n_f)
    a = (np.pi * fc * (t - delay)) ** 2
    return (1.0 - 2.0 * a) * np.exp(-a)


def uniform_pressure(nt, amplitude=1.0):
    return np.full(int(nt), float(amplitude), dtype=np.float64)


def _real_sh(l, m, theta, phi):
    """Real spherical harmonic of degree l, order m (theta polar, phi azimuth)."""
    if m == 0:
        return np.real(special.sph_harm_y(l, 0, theta, phi))
    y = special.sph_harm_y(l, abs(m), theta, phi)
    if m > 0:
        return np.sqrt(2.0) * (-1) ** m * np.real(y)
    return np.sqrt(2.0) * (-1) ** m * np.imag(y)


def sh_pressure(xyz, tri, rng, n_terms=4, lmax=6, centre=(0.0, 0.0, 0.0)):
    """Pressure field as a sum of ``n_terms`` real spherical harmonics with
    (l, m) drawn uniformly among the (lmax+1)^2 pairs with l <= lmax and
    N(0, 1) coefficients, evaluated in the direction of each triangle's
    vertex mean as seen from ``centre``."""
    pairs = [(l, m) for l in range(lmax + 1) for m in range(-l, l + 1)]
    pick = rng.integers(0, len(pairs), size=n_terms)
    coef = rng.standard_normal(n_terms)
    d = xyz[tri].mean(axis=1) - np.asarray(centre)
    d = d / np.linalg.norm(d, axis=1, keepdims=True)
    theta = np.arccos(np.clip(d[:, 2], -1.0, 1.0))
    phi = np.arctan2(d[:, 1], d[:, 0])
    p = np.zeros(len(tri))
    for c, k in zip(coef, pick):
        l, m = pairs[k]
        p += c * _real_sh(l, m, theta, phi)
    return p, [(pairs[k], float(c)) for c, k in zip(coef, pick)]
