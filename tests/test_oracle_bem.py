"""Pins of the oracle's assembled operator and frequency solve.

* rigid-body identity at s -> 0: c_ij + PV int T_ij = delta_ij for a cavity
  (n pointing into it) and 0 for a bounded body;
* the pressurised spherical cavity: the solved wall displacement converges
  to the closed form p H(s) as the mesh is refined (first order for
  constant elements), with no tangential part;
* a manufactured solution: the field of a point force placed inside the
  cavity is an exact exterior solution, so its traction must return its
  displacement, for any shape.
"""

import numpy as np
import pytest

from oracle import bem, closed_form as CF, kernels as K
from synth import icosphere, ellipsoid


def _geom(sub, exterior=True, axes=None):
    xyz, tri = icosphere(sub) if axes is None else ellipsoid(sub, axes)
    return bem.geometry(xyz, tri, exterior=exterior)


def _rigid_gap(g, mat):
    T, _ = bem.assemble_dense(g, 1e-7, mat)
    ne = g["ne"]
    return T.reshape(ne, 3, ne, 3).sum(axis=2)          # (a, i, j)


def test_rigid_body_exterior(mat):
    gaps = []
    for sub in (1, 2):
        rs = _rigid_gap(_geom(sub), mat)
        gaps.append(np.abs(rs - np.eye(3)).max())
    assert gaps[1] < 5e-3
    assert gaps[1] < 0.7 * gaps[0]


def test_rigid_body_interior(mat):
    rs = _rigid_gap(_geom(2, exterior=False), mat)
    assert np.abs(rs).max() < 5e-3


def _sphere_err(sub, s, mat):
    g = _geom(sub)
    t0 = bem.traction_from_pressure(g, np.ones(g["ne"]))
    T, U = bem.assemble_dense(g, s, mat)
    a = np.linalg.solve(T, U @ t0).reshape(-1, 3)
    rh = g["cen"] / np.linalg.norm(g["cen"], axis=1, keepdims=True)
    ur = np.einsum("ek,ek->e", a, rh)
    tang = a - ur[:, None] * rh
    H = CF.sphere_H(s, 1.0, mat)
    return abs(ur.mean() - H) / abs(H), np.sqrt(np.mean(np.abs(tang) ** 2)) / abs(H)


@pytest.mark.parametrize("s", [0.75, 0.75 + 3.1416j, 0.75 + 9.4248j])
def test_sphere_closed_form(mat, s):
    e1, t1 = _sphere_err(1, s, mat)
    e2, t2 = _sphere_err(2, s, mat)
    assert e2 < 0.06
    assert e2 < 0.65 * e1
    assert t2 < 0.01


def test_point_source_manufactured(mat):
    """u_j(y) = e_i U_ij(x0, y), t_j(y) = e_i T_ij(x0, y; n(y)) with x0 inside
    the cavity; the ellipsoid makes the check shape-independent."""
    x0 = np.array([0.15, -0.1, 0.2])
    e = np.array([0.3, 0.5, -0.8])
    e /= np.linalg.norm(e)
    s = 0.75 + 2.0j
    errs = []
    for sub in (1, 2):
        g = _geom(sub, axes=(1.2, 0.9, 1.0))
        t = np.einsum("i,bij->bj", e, K.T_kernel(x0, g["cen"], g["n"], s, mat)).reshape(-1)
        u = np.einsum("i,bij->bj", e, K.U_kernel(x0, g["cen"], s, mat)).reshape(-1)
        T, U = bem.assemble_dense(g, s, mat)
        a = np.linalg.solve(T, U @ t)
        errs.append(np.linalg.norm(a - u) / np.linalg.norm(u))
    assert errs[1] < 0.08
    assert errs[1] < 0.7 * errs[0]


def test_rows_match_dense(mat):
    g = _geom(1)
    T, U = bem.assemble_dense(g, 0.75 + 1j, mat)
    rows = bem.assemble_rows(g, 0.75 + 1j, mat, [3, 17, 40])
    for r, a in enumerate([3, 17, 40]):
        for w, M in (("T", T), ("U", U)):
            d = np.abs(rows[w][3 * r:3 * r + 3] - M[3 * a:3 * a + 3]).max()
            assert d < 1e-15 * np.abs(M).max()
