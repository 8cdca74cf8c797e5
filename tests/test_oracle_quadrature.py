"""Pins of the oracle's quadrature and singular self-element integrals.

* the 7-point rule integrates every monomial of degree <= 5 exactly;
* the polar rule (used by the oracle) and the Duffy rule (kept as a check)
  reproduce the closed-form integral of 1/r over a triangle;
* the principal value of the static antisymmetric traction kernel agrees
  with its divergence-theorem form (a line integral of 1/r around the edges)
  and vanishes on an equilateral triangle;
* the self-element U and T agree with a high-order Duffy integration and
  with an adaptive polar-coordinate integration.
"""

from math import factorial, pi

import numpy as np
import pytest
from scipy import integrate

from oracle import bem, kernels as K, quadrature as Q

TRI = np.array([[0.1, -0.2, 0.05], [1.3, 0.1, -0.1], [0.3, 0.9, 0.4]])


def _normal(v):
    g = np.cross(v[1] - v[0], v[2] - v[0])
    return g / np.linalg.norm(g)


def test_radon7_degree5_exact():
    bary, w = Q.radon7()
    x, y = bary[:, 1], bary[:, 2]          # reference triangle (0,0),(1,0),(0,1)
    for a in range(6):
        for b in range(6 - a):
            exact = factorial(a) * factorial(b) / factorial(a + b + 2)
            got = 0.5 * np.sum(w * x ** a * y ** b)
            assert abs(got - exact) < 1e-16 + 1e-14 * exact
    # and it is not exact at degree 6
    errs = [abs(0.5 * np.sum(w * x ** a * y ** (6 - a))
                - factorial(a) * factorial(6 - a) / factorial(8)) for a in range(7)]
    assert max(errs) > 1e-6


def _edge_geom(x, pa, pb):
    """Perpendicular distance h and signed in-line coordinates of the
    endpoints measured from the foot of the perpendicular from x."""
    t = (pb - pa) / np.linalg.norm(pb - pa)
    foot = pa + t * np.dot(x - pa, t)
    h = np.linalg.norm(x - foot)
    return h, np.dot(pa - foot, t), np.dot(pb - foot, t), t, foot


@pytest.mark.parametrize("rule,order", [("polar", 24), ("duffy", 48)])
def test_singular_rules_integrate_inverse_distance(rule, order):
    x = TRI.mean(axis=0)
    exact = 0.0
    got = 0.0
    area = 0.0
    for a in range(3):
        pa, pb = TRI[a], TRI[(a + 1) % 3]
        h, l1, l2, _, _ = _edge_geom(x, pa, pb)
        exact += h * abs(np.arcsinh(l2 / h) - np.arcsinh(l1 / h))
        if rule == "polar":
            pts, w = Q.polar_rule(x, pa, pb, order, order)
        else:
            pts, w = Q.duffy_rule(x, pa, pb, order)
        got += np.sum(w / np.linalg.norm(pts - x, axis=-1))
        area += np.sum(w)
    assert abs(got - exact) < 1e-13 * exact
    assert abs(area - 0.5 * np.linalg.norm(np.cross(TRI[1] - TRI[0], TRI[2] - TRI[0]))) < 1e-14


def _cpv_divergence(x, v, n, mat):
    """PV int rh_i / r^2 dA = -sum_edges m_i int_edge dl / r (m: outward
    in-plane edge normal), so the static kernel's principal value is
    gamma^2/(4 pi) (C_i n_j - n_i C_j)."""
    C = np.zeros(3)
    e3 = _normal(v)
    for a in range(3):
        pa, pb = v[a], v[(a + 1) % 3]
        h, l1, l2, t, foot = _edge_geom(x, pa, pb)
        m = np.cross(t, e3)
        if np.dot(m, foot - x) < 0:
            m = -m
        C -= m * abs(np.arcsinh(l2 / h) - np.arcsinh(l1 / h))
    g2 = mat["gamma"] ** 2
    return g2 / (4 * pi) * (C[:, None] * n[None, :] - n[:, None] * C[None, :])


@pytest.mark.parametrize("flip", [False, True])
def test_cpv_matches_divergence_theorem(mat, flip):
    x = TRI.mean(axis=0)
    n = _normal(TRI) * (-1 if flip else 1)
    got = bem.cpv_static(x[None], TRI[None], n[None], mat)[0]
    ref = _cpv_divergence(x, TRI, n, mat)
    assert np.abs(got - ref).max() < 1e-13
    assert np.abs(ref).max() > 1e-3          # not trivially zero


def test_cpv_vanishes_on_equilateral(mat):
    v = np.array([[1.0, 0, 0], [-0.5, np.sqrt(3) / 2, 0], [-0.5, -np.sqrt(3) / 2, 0]])
    got = bem.cpv_static(v.mean(axis=0)[None], v[None], np.array([[0, 0, 1.0]]), mat)[0]
    assert np.abs(got).max() < 1e-15


def test_self_rule_converges(mat):
    x = TRI.mean(axis=0)
    n = -_normal(TRI)
    # |s| times the element size is ~4 here, beyond what the meshes reach
    for s in (0.75, 0.75 + 3.0j):
        U1, T1 = bem.self_integrals(x, TRI, n, s, mat, order=24)
        U2, T2 = bem.self_integrals(x, TRI, n, s, mat, order=40)
        assert np.abs(U1 - U2).max() < 1e-13 * np.abs(U2).max()
        assert np.abs(T1 - T2).max() < 1e-13 * np.abs(T2).max()


def _polar_self(x, v, n, s, mat, kind):
    """int over the triangle in polar coordinates about x: adaptive in theta
    per edge, 48-point Gauss-Legendre in rho on [0, R(theta)].  For T the
    static part enters through its polar principal value g(theta) ln R."""
    e3 = _normal(v)
    e1 = v[0] - x
    e1 -= e3 * np.dot(e1, e3)
    e1 /= np.linalg.norm(e1)
    e2 = np.cross(e3, e1)
    t, wt = Q.gauss_legendre_01(48)
    g2 = mat["gamma"] ** 2
    total = np.zeros((3, 3), np.complex128)
    for a in range(3):
        pa, pb = v[a], v[(a + 1) % 3]
        ta = np.arctan2(np.dot(pa - x, e2), np.dot(pa - x, e1))
        tb = np.arctan2(np.dot(pb - x, e2), np.dot(pb - x, e1))
        dth = (tb - ta) % (2 * pi)
        h, _, _, tt, foot = _edge_geom(x, pa, pb)
        m = (foot - x) / np.linalg.norm(foot - x)

        def f(th):
            rh = np.cos(th) * e1 + np.sin(th) * e2
            R = h / np.dot(rh, m)
            rho = t * R
            pts = x + rho[:, None] * rh
            if kind == "U":
                ker = K.U_kernel(x, pts, s, mat)
                val = np.einsum("q,qij->ij", wt * rho * R, ker)
            else:
                ker = K.T_kernel(x, pts, n, s, mat, tail=True)
                val = np.einsum("q,qij->ij", wt * rho * R, ker)
                Kst = np.outer(rh, n) - np.outer(n, rh)
                val = val + g2 / (4 * pi) * Kst * np.log(R)
            return np.concatenate([val.real.ravel(), val.imag.ravel()])

        res, _ = integrate.quad_vec(f, ta, ta + dth, epsabs=1e-15, epsrel=1e-13)
        total += (res[:9] + 1j * res[9:]).reshape(3, 3)
    return total


def _duffy_self(x, v, n, s, mat, order=64):
    U = np.zeros((3, 3), np.complex128)
    T = np.zeros((3, 3), np.complex128)
    for a in range(3):
        pts, w = Q.duffy_rule(x, v[a], v[(a + 1) % 3], order)
        U += np.einsum("q,qij->ij", w[0], K.U_kernel(x, pts[0], s, mat))
        T += np.einsum("q,qij->ij", w[0], K.T_kernel(x, pts[0], n, s, mat, tail=True))
    return U, T


@pytest.mark.parametrize("s", [0.75, 0.75 + 6.0j])
def test_self_integrals_match_brute_force(mat, s):
    x = TRI.mean(axis=0)
    n = -_normal(TRI)
    U, T = bem.self_integrals(x, TRI, n, s, mat)
    Ub = _polar_self(x, TRI, n, s, mat, "U")
    Tb = _polar_self(x, TRI, n, s, mat, "T") + 0.5 * np.eye(3)
    assert np.abs(U[0] - Ub).max() < 1e-12 * np.abs(Ub).max()
    assert np.abs(T[0] - Tb).max() < 1e-12 * np.abs(Tb).max()
    Ud, Td = _duffy_self(x, TRI, n, s, mat)
    Td = Td + 0.5 * np.eye(3) + _cpv_divergence(x, TRI, n, mat)
    assert np.abs(U[0] - Ud).max() < 1e-12 * np.abs(Ud).max()
    assert np.abs(T[0] - Td).max() < 1e-12 * np.abs(Td).max()
