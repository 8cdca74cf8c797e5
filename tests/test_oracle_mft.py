"""Pins of the oracle's modified Fourier transform, closed forms and SEM.

* the damped DFT is numpy's FFT of the damped samples, divided by N_f;
* forward then inverse transform without a window returns the samples;
* the Hann and Blackman windows are scipy's periodic windows shifted by
  half a period (the paper's windows peak at k = 0);
* the cavity's residue-form step response has the Laplace transform H(s)/s;
* the sphere's transfer function through the transform reproduces the
  closed-form transient, and the Hann window reduces the late-time Gibbs
  error (Sec. 3.2);
* SEM is exact on its span and never worse than any other combination.
"""

import numpy as np
import pytest
from scipy import integrate
from scipy.signal import windows

from oracle import closed_form as CF, mft, sem
from synth import ramp_history


def test_load_spectrum_is_fft():
    rng = np.random.default_rng(3)
    P = rng.standard_normal(32)
    T, sigma = 8.0, 0.75
    got = mft.load_spectrum(P, T, sigma)
    n = np.arange(32)
    ref = np.fft.fft(np.exp(-sigma * n * T / 32) * P)[:17] / 32
    assert np.abs(got - ref).max() < 1e-14


def test_round_trip_without_window():
    rng = np.random.default_rng(4)
    P = rng.standard_normal(64)
    T, sigma = 8.0, 0.75
    spec = mft.load_spectrum(P, T, sigma)
    back = mft.inverse(spec, T, sigma, mft.WINDOW_NONE)
    assert np.abs(back - P).max() < 1e-12 * np.abs(P).max()


def test_windows_match_scipy():
    for n in (16, 32, 128):
        assert np.abs(mft.window(n, mft.WINDOW_HANN)
                      - np.roll(windows.hann(n, sym=False), n // 2)).max() < 1e-15
        assert np.abs(mft.window(n, mft.WINDOW_BLACKMAN)
                      - np.roll(windows.blackman(n, sym=False), n // 2)).max() < 1e-15


def test_sigma_rule():
    assert abs(mft.sigma_from_kappa(4.0, 8.0) - 4.0 * np.log(10.0) / 8.0) < 1e-15


def test_step_response_transforms_to_H(mat):
    assert abs(CF.sphere_step_response(0.0, 1.0, mat)) < 1e-14
    assert abs(CF.sphere_step_response(60.0, 1.0, mat) - 0.25) < 1e-12
    for s in (0.75, 0.75 + 2.0j, 1.5 - 0.5j):
        f = lambda t: CF.sphere_step_response(t, 1.0, mat) * np.exp(-s * t)
        re, _ = integrate.quad(lambda t: np.real(f(t)), 0, 80, limit=400)
        im, _ = integrate.quad(lambda t: np.imag(f(t)), 0, 80, limit=400)
        assert abs((re + 1j * im) - CF.sphere_H(s, 1.0, mat) / s) < 1e-9


def _mft_sphere(mat, n_f, kind, period=8.0, t_rise=0.05):
    sigma = 6.0 / period
    P = ramp_history(n_f, period, t_rise)
    s = mft.freq_grid(period, n_f, sigma)
    spec = mft.load_spectrum(P, period, sigma) * CF.sphere_H(s, 1.0, mat)
    u = mft.inverse(spec, period, sigma, kind)
    t = np.arange(n_f) * period / n_f
    # the sampled load is a step at t = dt (the rise is shorter than dt)
    ref = CF.sphere_ramp_response(t - period / n_f, 1.0, mat, 0.0)
    return np.linalg.norm(u - ref) / np.linalg.norm(ref)


def test_hann_reduces_gibbs_error(mat):
    e_none = _mft_sphere(mat, 32, mft.WINDOW_NONE)
    e_hann = _mft_sphere(mat, 32, mft.WINDOW_HANN)
    e_black = _mft_sphere(mat, 32, mft.WINDOW_BLACKMAN)
    assert e_hann < 0.5 * e_none
    # Blackman removes the Gibbs error as well; on this smooth response its
    # wider main lobe costs up to twice Hann's error
    assert e_black < 0.5 * e_none and e_black < 2.5 * e_hann
    # refining the sampling reduces the intrinsic error of the transform
    assert _mft_sphere(mat, 128, mft.WINDOW_HANN) < 0.5 * e_hann


# ---- SEM (Sec. 4.2)


def _sys(n=40, seed=5):
    rng = np.random.default_rng(seed)
    A = np.eye(n) * 3 + (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / np.sqrt(n)
    return A, rng


def test_sem_exact_on_span():
    A, rng = _sys()
    X = rng.standard_normal((40, 3)) + 1j * rng.standard_normal((40, 3))
    c = np.array([0.7, -0.2 + 0.1j, 0.05j])
    b = A @ (X @ c)
    x0 = sem.sem_guess(lambda M: A @ M, X, b)
    assert np.linalg.norm(x0 - X @ c) < 1e-12 * np.linalg.norm(X @ c)


def test_sem_least_squares_optimal():
    A, rng = _sys()
    X = rng.standard_normal((40, 3)) + 1j * rng.standard_normal((40, 3))
    b = rng.standard_normal(40) + 0j
    x0 = sem.sem_guess(lambda M: A @ M, X, b)
    r0 = np.linalg.norm(b - A @ x0)
    for _ in range(50):
        c = rng.standard_normal(3) + 1j * rng.standard_normal(3)
        assert r0 <= np.linalg.norm(b - A @ (X @ c)) + 1e-12
    q = sem.quadratic_extrapolation([X[:, 0], X[:, 1], X[:, 2]])
    assert r0 <= np.linalg.norm(b - A @ q) + 1e-12


def test_sem_drops_dependent_columns():
    A, rng = _sys()
    x = rng.standard_normal(40) + 1j * rng.standard_normal(40)
    X = np.stack([x, 2 * x, x + 1e-15], axis=1)
    b = A @ (0.5 * x)
    x0 = sem.sem_guess(lambda M: A @ M, X, b)
    assert np.linalg.norm(x0 - 0.5 * x) < 1e-10 * np.linalg.norm(x)
    assert np.array_equal(sem.sem_guess(lambda M: A @ M, X[:, :0], b), np.zeros_like(b))


def test_quadratic_extrapolation_exact_on_quadratics():
    # Lagrange extrapolation through the three previous equispaced samples
    # reproduces any vector sequence quadratic in k, and on a cubic it
    # leaves exactly the third difference (6 c for c k^3).  The shorter
    # histories are the constant and linear extrapolations.
    rng = np.random.default_rng(11)
    c0, c1, c2, c3 = (rng.standard_normal(17) + 1j * rng.standard_normal(17) for _ in range(4))
    for k in (3, 7, 40):
        quad = lambda j: c0 + c1 * j + c2 * j * j
        hist = [quad(k - 1), quad(k - 2), quad(k - 3)]
        x = sem.quadratic_extrapolation(hist)
        assert np.linalg.norm(x - quad(k)) <= 1e-12 * np.linalg.norm(quad(k))
        cub = lambda j: quad(j) + c3 * j ** 3
        x = sem.quadratic_extrapolation([cub(k - 1), cub(k - 2), cub(k - 3)])
        assert np.linalg.norm((cub(k) - x) - 6.0 * c3) <= 1e-9 * np.linalg.norm(cub(k))
        lin = lambda j: c0 + c1 * j
        x = sem.quadratic_extrapolation([lin(k - 1), lin(k - 2)])
        assert np.linalg.norm(x - lin(k)) <= 1e-12 * np.linalg.norm(lin(k))
        x = sem.quadratic_extrapolation([quad(k - 1), quad(k - 2)])
        assert np.linalg.norm((quad(k) - x) - 2.0 * c2) <= 1e-10 * np.linalg.norm(quad(k))
        assert np.array_equal(sem.quadratic_extrapolation([c0]), c0)
    assert sem.quadratic_extrapolation([]) is None
    # a planted mistake in the coefficients (2 a1 - a2, the linear rule on
    # three samples) is caught by the quadratic case
    bad = 2.0 * quad(39) - quad(38)
    assert np.linalg.norm(bad - quad(40)) > 1e-3 * np.linalg.norm(quad(40))
