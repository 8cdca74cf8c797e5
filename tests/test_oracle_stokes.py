"""Stokes' transient point-force solution (oracle.closed_form), pinned
against the Laplace-domain fundamental solution it must transform into, and
against Kelvin's static solution for a force held constant.

  * its Laplace transform, taken by quadrature in time at complex s, equals
    U(x0, x; s) d F(s) with U the oracle's Laplace-domain kernel (Sec. 2.1)
    and F(s) the transform of the force history -- at points in the near
    field (r < one wavelength) and beyond, for two values of s;
  * a force ramped to 1 and then held gives, once both waves have passed,
    Kelvin's static displacement;
  * planted errors in the material the formula is given (c_s for c_p, or
    c_s off by 10%) break the first check.
"""

import numpy as np
import pytest

from oracle import closed_form as CF, kernels as K


@pytest.fixture(scope="module")
def mat():
    return K.material(1.0, 1.0, 0.25)


def _pulse(t, tc=3.0, w=0.6):
    t = np.asarray(t, float)
    return np.where(t > 0, np.exp(-((t - tc) / w) ** 2), 0.0)


def _laplace(fn, s, T=40.0, n=8000):
    # composite Gauss-Legendre on [0, T]; the pulse and the responses decay well before T
    xg, wg = np.polynomial.legendre.leggauss(16)
    edges = np.linspace(0.0, T, n // 16 + 1)
    tt = (0.5 * (edges[1:] - edges[:-1])[:, None] * xg[None, :] + 0.5 * (edges[1:] + edges[:-1])[:, None]).ravel()
    ww = (0.5 * (edges[1:] - edges[:-1])[:, None] * wg[None, :]).ravel()
    v = fn(tt)
    return np.tensordot(ww * np.exp(-s * tt), v, axes=(0, 0))


def test_stokes_transforms_into_the_laplace_kernel(mat):
    x0 = np.array([0.1, -0.2, 0.05])
    d = np.array([0.3, -0.5, 0.8])
    d /= np.linalg.norm(d)
    pts = np.array([[0.6, 0.1, -0.2], [1.5, 2.0, 1.0], [-3.0, 1.0, 2.5]])
    for s in (0.4 + 1.3j, 1.0 + 0.2j):
        Fs = _laplace(_pulse, s)
        lap = _laplace(lambda tt: CF.stokes_point_force(pts, x0, d, tt, _pulse, mat), s)
        ref = np.einsum("i,pij->pj", d, K.U_kernel(x0, pts, s, mat)) * Fs
        e = np.abs(lap - ref).max() / np.abs(ref).max()
        assert e < 1e-7, (s, e)


def test_stokes_static_limit_is_kelvin(mat):
    x0 = np.zeros(3)
    d = np.array([0.0, 0.0, 1.0])
    pts = np.array([[0.7, 0.2, -0.3], [1.2, -0.4, 0.9]])
    ramp = lambda t: np.clip(np.asarray(t, float) / 0.5, 0.0, 1.0)
    u = CF.stokes_point_force(pts, x0, d, np.array([30.0]), ramp, mat)[0]
    ref = np.einsum("i,pij->pj", d, CF.kelvin_U(x0, pts, mat))
    assert np.abs(u - ref).max() < 1e-10 * np.abs(ref).max()


def test_planted_errors_are_caught(mat):
    x0 = np.zeros(3)
    d = np.array([1.0, 0.0, 0.0])
    pts = np.array([[0.5, 0.3, 0.2]])
    s = 0.4 + 1.3j
    Fs = _laplace(_pulse, s)
    ref = np.einsum("i,pij->pj", d, K.U_kernel(x0, pts, s, mat)) * Fs
    for bad in (dict(mat, cp=mat["cs"]), dict(mat, cs=1.1 * mat["cs"])):
        lap = _laplace(lambda tt: CF.stokes_point_force(pts, x0, d, tt, _pulse, bad), s)
        assert np.abs(lap - ref).max() > 1e-3 * np.abs(ref).max()
