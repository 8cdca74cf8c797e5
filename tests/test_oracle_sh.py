"""Closed form for a spherical cavity under a spherical-harmonic wall
pressure, pinned against the mathematics and against the oracle's BEM.

The closed form (oracle/closed_form.py) builds the exterior field from two
potentials with decaying modified spherical Bessel functions.  Pins:
  * l = 0 reduces to the uniform-pressure transfer function H(s), which is
    written out independently;
  * k_l solves the modified spherical Bessel equation, and the returned
    derivatives are derivatives (finite differences);
  * the field satisfies Navier's equation mu lap u + (lambda + mu) grad div u
    = rho s^2 u outside the cavity (finite differences in 3-D);
  * at the wall the traction is -p Y e_r with no shear (finite-difference
    strains);
  * the oracle's dense BEM solution (Sec. 2.1) for the same load converges to
    it: the error at level 3 is about half that at level 2.
"""

import numpy as np
import pytest

from oracle import bem, closed_form as CF, kernels as K
from synth import icosphere


@pytest.fixture(scope="module")
def mat():
    return K.material(1.0, 1.0, 0.25)


S_VALUES = (0.75 + 1.0j, 0.75 + 4.0j, 2.0 + 9.0j)


@pytest.mark.parametrize("s", S_VALUES)
def test_l0_is_uniform_pressure_closed_form(mat, s):
    _, _, Hr, Ht = CF.sphere_sh_modes(s, 0, 1.0, mat)
    assert abs(Hr - CF.sphere_H(s, 1.0, mat)) < 1e-13 * abs(Hr)


@pytest.mark.parametrize("l", [0, 1, 2, 3, 5])
def test_kl_solves_modified_spherical_bessel_equation(l):
    x = np.array([0.7 + 0.2j, 1.5 + 3.0j, 4.0 - 1.0j])
    k, k1, k2 = CF.mod_sph_bessel_k(l, x)
    res = x * x * k2 + 2 * x * k1 - (x * x + l * (l + 1)) * k
    assert np.all(np.abs(res) < 1e-12 * np.abs(x * x * k))
    h = 1e-6
    kp = CF.mod_sph_bessel_k(l, x + h)
    km = CF.mod_sph_bessel_k(l, x - h)
    assert np.allclose((kp[0] - km[0]) / (2 * h), k1, rtol=1e-7)
    assert np.allclose((kp[1] - km[1]) / (2 * h), k2, rtol=1e-7)
    if l == 0:
        assert np.allclose(k, np.exp(-x) / x, rtol=1e-14)


def _field(mat, s, l):
    Y, gY = CF.legendre_Y(l)
    return lambda pts: CF.sphere_sh_displacement(np.atleast_2d(pts), s, l, 1.0, mat, Y, gY)


def _jacobian(u, x, h):
    """du_i/dx_j at x by central differences."""
    J = np.zeros((3, 3), complex)
    for j in range(3):
        e = np.zeros(3)
        e[j] = h
        J[:, j] = (u(x + e)[0] - u(x - e)[0]) / (2 * h)
    return J


@pytest.mark.parametrize("l", [1, 2, 3])
@pytest.mark.parametrize("s", S_VALUES[:2])
def test_field_satisfies_navier_equation(mat, s, l):
    u = _field(mat, s, l)
    h = 2e-3
    rng = np.random.default_rng(l)
    for _ in range(3):
        d = rng.standard_normal(3)
        x = (1.4 + rng.random()) * d / np.linalg.norm(d)
        u0 = u(x)[0]
        lap = np.zeros(3, complex)
        for j in range(3):
            e = np.zeros(3)
            e[j] = h
            lap += (u(x + e)[0] - 2 * u0 + u(x - e)[0]) / h ** 2
        # grad div by differences of the divergence
        gdiv = np.zeros(3, complex)
        for j in range(3):
            e = np.zeros(3)
            e[j] = h
            gdiv[j] = (np.trace(_jacobian(u, x + e, h)) - np.trace(_jacobian(u, x - e, h))) / (2 * h)
        res = mat["mu"] * lap + (mat["lam"] + mat["mu"]) * gdiv - mat["rho"] * s * s * u0
        scale = mat["rho"] * abs(s) ** 2 * np.linalg.norm(u0) + mat["mu"] * np.linalg.norm(lap)
        assert np.linalg.norm(res) < 2e-4 * scale


@pytest.mark.parametrize("l", [1, 2, 3])
def test_wall_traction_is_the_pressure(mat, l):
    s = S_VALUES[1]
    u = _field(mat, s, l)
    Y, _ = CF.legendre_Y(l)
    h = 1e-4
    rng = np.random.default_rng(10 + l)
    for _ in range(4):
        d = rng.standard_normal(3)
        er = d / np.linalg.norm(d)
        x = er * (1.0 + 2 * h)  # just outside the wall, so the stencil stays in the solid
        J = _jacobian(u, x, h)
        eps = 0.5 * (J + J.T)
        sig = mat["lam"] * np.trace(eps) * np.eye(3) + 2 * mat["mu"] * eps
        t = sig @ er
        # the traction varies smoothly: compare with the load at the wall,
        # first order in the 2h offset
        p = Y(er[None])[0]
        assert np.linalg.norm(t - (-p) * er) < 5e-3 * max(abs(p), 0.1)


def test_oracle_bem_converges_to_sh_closed_form(mat):
    s = 0.75 + 4.0j
    errs = {}
    for sub in (2, 3):
        xyz, tri = icosphere(sub)
        g = bem.geometry(xyz, tri, exterior=True)
        T, U = bem.assemble_dense(g, s, mat)
        xh = g["cen"] / np.linalg.norm(g["cen"], axis=1, keepdims=True)
        for l in (1, 2, 3):
            Y, gY = CF.legendre_Y(l)
            t0 = bem.traction_from_pressure(g, Y(xh))
            a = np.linalg.solve(T, U @ t0).reshape(-1, 3)
            ref = CF.sphere_sh_displacement(xh, s, l, 1.0, mat, Y, gY)
            errs[sub, l] = np.linalg.norm(a - ref) / np.linalg.norm(ref)
    for l in (1, 2, 3):
        assert errs[2, l] < 0.08
        assert errs[3, l] < 0.03
        assert errs[3, l] < 0.7 * errs[2, l]


def test_surface_gradient_by_differences_matches_legendre():
    rng = np.random.default_rng(3)
    d = rng.standard_normal((20, 3))
    xh = d / np.linalg.norm(d, axis=1, keepdims=True)
    for l in (1, 2, 4):
        Y, gY = CF.legendre_Y(l)
        assert np.allclose(CF.surface_gradient(Y, xh), gY(xh), atol=1e-8)
        # tangent to the sphere
        assert np.allclose(np.einsum("ij,ij->i", gY(xh), xh), 0.0, atol=1e-13)
