"""Modified Fourier transform (oracle; test infrastructure).

Sec. 2.2: with N_f samples over the period T, d omega = 2 pi / T and
dt = T / N_f; only k = 0..N_f/2 are solved and the rest follow from
R_k = conj(R_{N_f - k}).  Sec. 3.1: the exponential window damps the history
by exp(-eta t), which moves the frequencies to omega_k - i eta; in the Laplace
variable used here that is s_k = sigma + i k d omega with sigma = eta.
Sec. 3.2: the spectrum is multiplied by a Hann or Blackman window before
inversion.  Sec. 3.3 gives the two transforms:
  P_k  = (1/N_f) sum_n exp(-sigma n dt) P(n dt) exp(-2 pi i n k / N_f)
  R(n dt) = exp(sigma n dt) sum_k W_k R_k exp(2 pi i n k / N_f).
Reading: the solved Nyquist bin k = N_f/2 is kept as solved, and the real
part of the inverse sum is the time response.
"""

from math import log, pi

import numpy as np

WINDOW_NONE, WINDOW_HANN, WINDOW_BLACKMAN = 0, 1, 2


def sigma_from_kappa(kappa, period):
    """Rule of thumb of Sec. 3.1: eta = kappa ln(10) / T."""
    return kappa * log(10.0) / period


def freq_grid(period, n_f, sigma):
    """s_k = sigma + i k (2 pi / T), k = 0..N_f/2."""
    k = np.arange(n_f // 2 + 1)
    return sigma + 1j * k * (2.0 * pi / period)


def window(n_f, kind):
    """W_k for k = 0..N_f-1 (Sec. 3.2)."""
    k = np.arange(n_f)
    if kind == WINDOW_NONE:
        return np.ones(n_f)
    if kind == WINDOW_HANN:
        return 0.5 * (1.0 + np.cos(2.0 * pi * k / n_f))
    if kind == WINDOW_BLACKMAN:
        return (0.42 + 0.5 * np.cos(2.0 * pi * k / n_f)
                + 0.08 * np.cos(4.0 * pi * k / n_f))
    raise ValueError(kind)


def load_spectrum(history, period, sigma):
    """Damped DFT of the sampled history, k = 0..N_f/2, by the direct sum."""
    P = np.asarray(history, dtype=np.float64)
    n_f = len(P)
    dt = period / n_f
    out = np.zeros(n_f // 2 + 1, np.complex128)
    for k in range(n_f // 2 + 1):
        acc = 0.0 + 0.0j
        for n in range(n_f):
            acc += np.exp(-sigma * n * dt) * P[n] * np.exp(-2j * pi * n * k / n_f)
        out[k] = acc / n_f
    return out


def full_spectrum(half):
    """Fill k = N_f/2+1..N_f-1 by conjugate symmetry; ``half`` has N_f/2+1
    rows (any trailing shape)."""
    half = np.asarray(half)
    n_f = 2 * (half.shape[0] - 1)
    full = np.zeros((n_f,) + half.shape[1:], np.complex128)
    full[:n_f // 2 + 1] = half
    for k in range(n_f // 2 + 1, n_f):
        full[k] = np.conj(half[n_f - k])
    return full


def inverse(half, period, sigma, window_kind):
    """Time samples R(n dt), n = 0..N_f-1, from the solved half spectrum
    (shape (N_f/2+1, ...)), windowed and de-damped; real part returned."""
    full = full_spectrum(half)
    n_f = full.shape[0]
    dt = period / n_f
    W = window(n_f, window_kind)
    n = np.arange(n_f)
    k = np.arange(n_f)
    E = np.exp(2j * pi * np.outer(n, k) / n_f)            # (n, k)
    flat = (W[:, None] * full.reshape(n_f, -1))
    out = np.exp(sigma * n * dt)[:, None] * (E @ flat)
    return np.real(out).reshape((n_f,) + full.shape[1:])
