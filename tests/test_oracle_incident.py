"""Plane S-wave load (the scattering workload), pinned on the CPU.

  * the Laplace-domain plane wave pol exp(-s d.x / c_s) satisfies Navier's
    equation, and its stress formula equals the stress of finite-difference
    strains;
  * transforming the sampled wavelet with the damped DFT, multiplying by
    exp(-s_k d.x / c_s) and inverting (Sec. 3.3) gives back the wavelet
    delayed by d.x / c_s (so the sign of the delay and the spectrum's
    convention are right);
  * manufactured solution: a solid ball (interior problem, Sec. 2.1) loaded
    by the scattered-field traction of the wave, -sigma_inc n, has the exact
    solution -u_inc on its surface; the oracle's BEM converges to it;
  * the total-field formulation: the identity it rests on, T u_inc - U t_inc
    = u_inc on a cavity's surface (u_inc regular inside it), holds to the
    discretisation error and converges; and the total-field solution equals
    the scattered one plus u_inc in the limit (their difference shrinks
    under refinement).
"""

import numpy as np
import pytest

from oracle import bem, closed_form as CF, kernels as K, mft
from synth import icosphere, ricker_history


@pytest.fixture(scope="module")
def mat():
    return K.material(1.0, 1.0, 0.25)


DIRS = [(np.array([1.0, 0.0, 0.0]), np.array([0.0, 0.0, 1.0])),
        (np.array([1.0, 2.0, -2.0]) / 3.0, np.array([2.0, 1.0, 2.0]) / 3.0)]


@pytest.mark.parametrize("s", [0.75 + 2.0j, 0.3 + 7.0j])
@pytest.mark.parametrize("dp", DIRS)
def test_plane_wave_satisfies_navier_and_stress_formula(mat, s, dp):
    d, q = dp
    assert abs(d @ q) < 1e-15
    x0 = np.array([0.3, -0.4, 0.5])
    u = lambda x: CF.plane_s_wave(x, s, mat, d, q)[0]
    h = 2e-4  # truncation error ~ (|s| h / c_s)^2 / 6 < 1e-6
    J = np.zeros((3, 3), complex)
    lap = np.zeros(3, complex)
    for j in range(3):
        e = np.zeros(3)
        e[j] = h
        J[:, j] = (u(x0 + e) - u(x0 - e)) / (2 * h)
        lap += (u(x0 + e) - 2 * u(x0) + u(x0 - e)) / h ** 2
    # divergence free, so Navier reduces to mu lap u = rho s^2 u
    assert abs(np.trace(J)) < 1e-6 * np.abs(J).max()
    res = mat["mu"] * lap - mat["rho"] * s * s * u(x0)
    assert np.linalg.norm(res) < 1e-5 * mat["rho"] * abs(s) ** 2 * np.linalg.norm(u(x0))
    eps = 0.5 * (J + J.T)
    sig = mat["lam"] * np.trace(eps) * np.eye(3) + 2 * mat["mu"] * eps
    S = CF.plane_s_wave_stress(x0, s, mat, d, q)[0]
    assert np.abs(S - sig).max() < 1e-5 * np.abs(S).max()


def test_transformed_wave_is_the_delayed_wavelet(mat):
    period, n_f, fc, t0 = 16.0, 256, 0.5, 3.0
    sigma = 6.0 / period
    hist = ricker_history(n_f, period, fc, t0)
    s_k = mft.freq_grid(period, n_f, sigma)
    phat = mft.load_spectrum(hist, period, sigma)
    d, q = DIRS[0]
    x = np.array([[1.7, 0.2, -0.3]])
    spec = np.array([phat[k] * CF.plane_s_wave(x, s, mat, d, q)[0] for k, s in enumerate(s_k)])
    u = mft.inverse(spec, period, sigma, 0)
    t = np.arange(n_f) * period / n_f
    tau = (x[0] @ d) / mat["cs"]
    a = (np.pi * fc * (t - t0 - tau)) ** 2
    ref = (1 - 2 * a) * np.exp(-a)
    assert np.abs(u[:, 2] - ref).max() < 2e-3
    assert np.abs(u[:, :2]).max() < 1e-12


def test_interior_ball_reproduces_minus_the_incident_wave(mat):
    s = 0.75 + 3.0j
    errs = []
    for sub in (1, 2):
        for d, q in DIRS:
            xyz, tri = icosphere(sub)
            g = bem.geometry(xyz, tri, exterior=False)
            T, U = bem.assemble_dense(g, s, mat)
            a = np.linalg.solve(T, U @ bem.incident_s_load(g, s, mat, d, q)).reshape(-1, 3)
            ref = -CF.plane_s_wave(g["cen"], s, mat, d, q)
            errs.append(np.linalg.norm(a - ref) / np.linalg.norm(ref))
    # level 1 then level 2, for both directions
    assert max(errs[2:]) < 0.06
    assert errs[2] < 0.7 * errs[0] and errs[3] < 0.7 * errs[1]


def test_interior_identity_behind_the_total_field(mat):
    """T u_inc - U t_inc = u_inc for the cavity (T with its free term 1/2):
    Somigliana's identity inside the cavity, where the plane wave is
    regular.  A sign error in either term, or a free term of 1, breaks it."""
    s = 0.75 + 3.0j
    errs, bad = [], []
    for sub in (1, 2):
        d, q = DIRS[1]
        xyz, tri = icosphere(sub)
        g = bem.geometry(xyz, tri, exterior=True)
        T, U = bem.assemble_dense(g, s, mat)
        v = bem.incident_s_total_rhs(g, s, mat, d, q)
        t_inc = -bem.incident_s_load(g, s, mat, d, q)   # the wave's own traction (n out of the solid)
        errs.append(np.linalg.norm(T @ v - U @ t_inc - v) / np.linalg.norm(v))
        bad.append(np.linalg.norm(T @ v + U @ t_inc - v) / np.linalg.norm(v))
    assert errs[1] < 0.05 and errs[1] < 0.6 * errs[0]
    assert min(bad) > 0.3


def test_total_field_converges_to_scattered_plus_incident(mat):
    s = 0.75 + 2.0j
    diffs = []
    for sub in (1, 2):
        d, q = DIRS[0]
        xyz, tri = icosphere(sub)
        g = bem.geometry(xyz, tri, exterior=True)
        T, U = bem.assemble_dense(g, s, mat)
        u_tot = np.linalg.solve(T, bem.incident_s_total_rhs(g, s, mat, d, q))
        u_sc = np.linalg.solve(T, U @ bem.incident_s_load(g, s, mat, d, q))
        u_inc = bem.incident_s_total_rhs(g, s, mat, d, q)
        diffs.append(np.linalg.norm(u_tot - u_sc - u_inc) / np.linalg.norm(u_tot))
    assert diffs[1] < 0.05 and diffs[1] < 0.6 * diffs[0]
