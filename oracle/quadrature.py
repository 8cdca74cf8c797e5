"""Quadrature rules on flat triangles (oracle; test infrastructure).

Sec. 2.1 discretises the boundary into flat triangles with one constant
value per element and collocation; the paper does not state the rules.  The
reading used here: the 7-point degree-5 rule of Radon for every pair of
distinct elements, and for the element that carries the collocation point a
product rule in polar coordinates about that point (Gauss-Legendre in the
angle over each edge, Gauss-Legendre in the radius), which cancels the 1/r
singularity of U and leaves a smooth integrand.  The Duffy rule is kept as
an independent cross-check.
"""

import numpy as np


def radon7():
    """Barycentric points (7, 3) and weights (7,) of the degree-5 rule; the
    weights sum to one (multiply by the triangle area)."""
    s15 = np.sqrt(15.0)
    a = (6.0 - s15) / 21.0
    b = (6.0 + s15) / 21.0
    wa = (155.0 - s15) / 1200.0
    wb = (155.0 + s15) / 1200.0
    pts = [(1 / 3, 1 / 3, 1 / 3),
           (a, a, 1 - 2 * a), (a, 1 - 2 * a, a), (1 - 2 * a, a, a),
           (b, b, 1 - 2 * b), (b, 1 - 2 * b, b), (1 - 2 * b, b, b)]
    w = [9.0 / 40.0] + [wa] * 3 + [wb] * 3
    return np.array(pts), np.array(w)


def triangle_rule(v0, v1, v2):
    """Physical points (7, 3) and weights (7,) of the 7-point rule."""
    bary, w = radon7()
    pts = bary[:, 0:1] * v0 + bary[:, 1:2] * v1 + bary[:, 2:3] * v2
    area = 0.5 * np.linalg.norm(np.cross(v1 - v0, v2 - v0))
    return pts, w * area


def gauss_legendre_01(n):
    """n-point Gauss-Legendre nodes and weights on [0, 1]."""
    t, w = np.polynomial.legendre.leggauss(int(n))
    return 0.5 * (t + 1.0), 0.5 * w


def duffy_rule(x, pa, pb, n):
    """Product rule on triangles (x, pa, pb) with the singular vertex at x.

    The square (u, v) in [0,1]^2 maps to y = x + u((pa - x) + v (pb - pa));
    the area element is u * |(pa - x) x (pb - pa)| du dv, so a 1/|y - x|
    singularity at x is cancelled by the factor u.  Inputs are (E, 3) (or
    (3,)); returns points (E, n*n, 3) and weights (E, n*n)."""
    x, pa, pb = (np.atleast_2d(np.asarray(a, dtype=np.float64)) for a in (x, pa, pb))
    u, wu = gauss_legendre_01(n)
    v, wv = gauss_legendre_01(n)
    e1 = pa - x
    e2 = pb - pa
    jac = np.linalg.norm(np.cross(e1, e2), axis=1)                  # (E,)
    U, V = np.meshgrid(u, v, indexing="ij")
    W = (np.outer(wu, wv) * U).reshape(-1)                          # (q,)
    Uf, Vf = U.reshape(-1), V.reshape(-1)
    pts = (x[:, None, :] + Uf[None, :, None]
           * (e1[:, None, :] + Vf[None, :, None] * e2[:, None, :]))
    return pts, W[None, :] * jac[:, None]


def polar_rule(x, pa, pb, n_theta, n_rho):
    """Product rule on triangles (x, pa, pb) in polar coordinates about x.

    theta runs over the angle the edge (pa, pb) subtends at x, rho over
    [0, R(theta)] with R(theta) = h / cos(theta - theta_0) the distance to
    the edge line (h its distance from x, theta_0 the direction of the foot
    of the perpendicular).  dA = rho d rho d theta.  Inputs (E, 3); returns
    points (E, n_theta*n_rho, 3) and weights (E, n_theta*n_rho)."""
    x, pa, pb = (np.atleast_2d(np.asarray(a, dtype=np.float64)) for a in (x, pa, pb))
    e3 = np.cross(pa - x, pb - x)
    e3 /= np.linalg.norm(e3, axis=1, keepdims=True)
    da = pa - x
    la = np.linalg.norm(da, axis=1)
    e1 = da / la[:, None]
    e2 = np.cross(e3, e1)
    db = pb - x
    tb = np.arctan2(np.einsum("ek,ek->e", db, e2), np.einsum("ek,ek->e", db, e1))
    # edge line: foot of the perpendicular from x
    t = (pb - pa) / np.linalg.norm(pb - pa, axis=1, keepdims=True)
    foot = pa - t * np.einsum("ek,ek->e", pa - x, t)[:, None]
    h = np.linalg.norm(foot - x, axis=1)
    m = (foot - x) / h[:, None]
    th, wth = gauss_legendre_01(n_theta)
    u, wu = gauss_legendre_01(n_rho)
    theta = th[None, :] * tb[:, None]                                   # (E, a)
    rh = (np.cos(theta)[..., None] * e1[:, None, :]
          + np.sin(theta)[..., None] * e2[:, None, :])                  # (E, a, 3)
    R = h[:, None] / np.einsum("eak,ek->ea", rh, m)                     # (E, a)
    rho = R[:, :, None] * u[None, None, :]                              # (E, a, b)
    pts = x[:, None, None, :] + rho[..., None] * rh[:, :, None, :]
    w = (wth[None, :, None] * tb[:, None, None]) * wu[None, None, :] * rho * R[:, :, None]
    E = len(x)
    return pts.reshape(E, -1, 3), w.reshape(E, -1)
