"""Dense collocation BEM with constant flat triangles (oracle; test infrastructure).

Sec. 2.1: the boundary integral equation
    c_ij u_j(x) + PV int_Gamma T_ij(x, y) u_j(y) dGamma_y
        = int_Gamma U_ij(x, y) t_j(y) dGamma_y
is collocated at one point per element with constant u and t per element,
giving N x N matrices T (free term included) and U with N = 3 N_e and the
system T u = U t.  Degree of freedom 3 e + i is component i (global axes) of
element e.

Readings (where the paper is silent): the collocation point is the element
centroid; c_ij = delta_ij / 2 there (the flat element is smooth at its
centroid); distinct elements use the 7-point rule; the element holding the
collocation point uses a polar-coordinate rule about the centroid for U, and
for T the sum of the free term, the Cauchy principal value of the static
kernel and the polar-rule integral of the bounded remainder T - T_static.
"""

from math import pi

import numpy as np

from . import kernels as K
from . import quadrature as Q


def geometry(xyz, tri, exterior=True):
    """Centroids, unit normals n (pointing out of the solid Omega), areas,
    and the 7-point rule of every element.

    Triangles are counter-clockwise seen from outside the closed surface.
    For ``exterior`` (Omega outside the surface, a cavity) n points into
    the enclosed volume; otherwise it points out of it."""
    xyz = np.asarray(xyz, dtype=np.float64)
    tri = np.asarray(tri, dtype=np.int64)
    v0, v1, v2 = xyz[tri[:, 0]], xyz[tri[:, 1]], xyz[tri[:, 2]]
    cr = np.cross(v1 - v0, v2 - v0)
    area = 0.5 * np.linalg.norm(cr, axis=1)
    n = cr / (2.0 * area[:, None])
    if exterior:
        n = -n
    cen = (v0 + v1 + v2) / 3.0
    bary, w = Q.radon7()
    qp = (bary[None, :, 0:1] * v0[:, None, :] + bary[None, :, 1:2] * v1[:, None, :]
          + bary[None, :, 2:3] * v2[:, None, :])
    qw = w[None, :] * area[:, None]
    return dict(v=np.stack([v0, v1, v2], axis=1), cen=cen, n=n, area=area,
                qp=qp, qw=qw, ne=len(tri))


def cpv_static(x, verts, n, mat, order=64):
    """CPV over flat triangles of the static kernel
    gamma^2/(4 pi r^2)(rh_i n_j - rh_j n_i) from interior points x.

    In polar coordinates about x the integrand is g(theta)/rho^2 with
    int_0^{2 pi} g = 0, so the principal value is int g(theta) ln R(theta)
    d theta, R(theta) being the distance from x to the boundary.  Each edge
    is integrated over the angle it subtends with Gauss-Legendre.

    Shapes: x (E, 3), verts (E, 3, 3), n (E, 3) -> (E, 3, 3)."""
    g2 = mat["gamma"] ** 2
    e3 = np.cross(verts[:, 1] - verts[:, 0], verts[:, 2] - verts[:, 0])
    e3 /= np.linalg.norm(e3, axis=1, keepdims=True)
    e1 = verts[:, 0] - x
    e1 -= e3 * np.einsum("ek,ek->e", e1, e3)[:, None]
    e1 /= np.linalg.norm(e1, axis=1, keepdims=True)
    e2 = np.cross(e3, e1)
    t, wt = np.polynomial.legendre.leggauss(order)
    out = np.zeros((len(x), 3, 3))
    dot = lambda a, b: np.einsum("ek,ek->e", a, b)
    for a in range(3):
        pa, pb = verts[:, a], verts[:, (a + 1) % 3]
        ta = np.arctan2(dot(pa - x, e2), dot(pa - x, e1))
        tb = np.arctan2(dot(pb - x, e2), dot(pb - x, e1))
        dth = (tb - ta) % (2.0 * pi)
        m = np.cross(pb - pa, e3)
        m /= np.linalg.norm(m, axis=1, keepdims=True)
        h = dot(pa - x, m)
        m = m * np.sign(h)[:, None]
        h = np.abs(h)
        th = ta[:, None] + 0.5 * dth[:, None] * (t[None, :] + 1.0)     # (E, q)
        w = 0.5 * dth[:, None] * wt[None, :]
        rh = (np.cos(th)[..., None] * e1[:, None, :]
              + np.sin(th)[..., None] * e2[:, None, :])                 # (E, q, 3)
        lnR = np.log(h[:, None] / np.einsum("eqk,ek->eq", rh, m))
        Kij = (rh[..., :, None] * n[:, None, None, :]
               - n[:, None, :, None] * rh[..., None, :])
        out += np.einsum("eq,eq,eqij->eij", w, lnR, Kij)
    return g2 / (4.0 * pi) * out


def self_integrals(x, verts, n, s, mat, order=24):
    """U and T blocks (E, 3, 3) of the elements that hold the collocation
    points x (their centroids).  T includes the free term delta_ij / 2.

    Shapes: x (E, 3), verts (E, 3, 3), n (E, 3)."""
    x = np.atleast_2d(x)
    verts = np.asarray(verts).reshape(-1, 3, 3)
    n = np.atleast_2d(n)
    Uself = np.zeros((len(x), 3, 3), np.complex128)
    Tself = np.zeros((len(x), 3, 3), np.complex128)
    for a in range(3):
        pts, w = Q.polar_rule(x, verts[:, a], verts[:, (a + 1) % 3], order, order)
        xx = x[:, None, :]
        Uself += np.einsum("eq,eqij->eij", w, K.U_kernel(xx, pts, s, mat))
        Tself += np.einsum("eq,eqij->eij", w,
                           K.T_kernel(xx, pts, n[:, None, :], s, mat, tail=True))
    Tself += 0.5 * np.eye(3) + cpv_static(x, verts, n, mat)
    return Uself, Tself


def assemble_rows(geom, s, mat, elems, which=("T", "U"), self_order=24, chunk=None):
    """Rows 3a..3a+2 of T and U for every element a in ``elems``.

    Returns a dict with arrays of shape (3 len(elems), N)."""
    elems = np.asarray(elems, dtype=np.int64)
    ne = geom["ne"]
    N = 3 * ne
    out = {w: np.zeros((3 * len(elems), N), np.complex128) for w in which}
    qp, qw, nrm = geom["qp"], geom["qw"], geom["n"]
    if chunk is None:
        chunk = max(1, int(1.5e6 // (7 * ne)))
    for c0 in range(0, len(elems), chunk):
        ea = elems[c0:c0 + chunk]
        x = geom["cen"][ea]                                   # (m, 3)
        y = np.broadcast_to(qp[None], (len(ea),) + qp.shape).copy()
        # keep the self element out of the regular rule (its centroid is a
        # quadrature point); it is overwritten below
        y[np.arange(len(ea)), ea] = x[:, None, :] + 10.0
        xx = x[:, None, None, :]
        for w in which:
            if w == "T":
                ker = K.T_kernel(xx, y, nrm[None, :, None, :], s, mat)
            else:
                ker = K.U_kernel(xx, y, s, mat)
            blk = np.einsum("bq,abqij->aibj", qw, ker)           # (m,3,ne,3)
            out[w][3 * c0:3 * (c0 + len(ea))] = blk.reshape(3 * len(ea), N)
        Us, Ts = self_integrals(x, geom["v"][ea], nrm[ea], s, mat, order=self_order)
        for i, a in enumerate(ea):
            r = 3 * (c0 + i)
            if "T" in which:
                out["T"][r:r + 3, 3 * a:3 * a + 3] = Ts[i]
            if "U" in which:
                out["U"][r:r + 3, 3 * a:3 * a + 3] = Us[i]
    return out


def assemble_dense(geom, s, mat, self_order=24):
    """Dense T (free term included) and U at Laplace parameter s."""
    rows = assemble_rows(geom, s, mat, np.arange(geom["ne"]), self_order=self_order)
    return rows["T"], rows["U"]


def traction_from_pressure(geom, p):
    """t = -p n: a cavity pressure p pushes on the solid against n, which
    points out of Omega (Sec. 2.1 defines n as the outward normal)."""
    return (-np.asarray(p, dtype=np.float64)[:, None] * geom["n"]).reshape(-1)


def incident_s_load(geom, s, mat, direction, polarisation):
    """Scattered-field load of a plane S-wave on a traction-free boundary, for
    a unit wavelet spectrum: t_sc = -sigma_inc n at each element's centroid
    (n out of the solid), flattened to 3 N_e."""
    from .closed_form import plane_s_wave_stress
    S = plane_s_wave_stress(geom["cen"], s, mat, direction, polarisation)
    return (-np.einsum("eij,ej->ei", S, geom["n"])).reshape(-1)


def incident_s_total_rhs(geom, s, mat, direction, polarisation):
    """Total-field right-hand side of a plane S-wave on traction-free
    cavities, for a unit wavelet spectrum: the incident displacement
    pol exp(-s d.x / c_s) at each element's centroid, flattened to 3 N_e.
    The total displacement u = u_sc + u_inc then solves T u = u_inc (T with
    its free term), because u_inc, regular inside the cavities, satisfies
    T u_inc - U t_inc = u_inc there (Somigliana's identity for the
    cavities' interior with the normal reversed)."""
    from .closed_form import plane_s_wave
    return plane_s_wave(geom["cen"], s, mat, direction, polarisation).reshape(-1)


def mixed_system(T, U, bc, given):
    """Sec. 2.1, eq. Aa_b: the boundary conditions move the known boundary
    values to the right-hand side of T u = U t.  For an element with a given
    traction (bc = 0) the unknown is its displacement and its columns of T
    stay in A; for a given displacement (bc = 1) the unknown is its traction
    and its columns of -U go into A.  ``given`` (N_e x 3) holds the given
    traction or displacement of each element.  Returns (A, b) with
    b = sum_trac U t_given - sum_disp T u_given."""
    bc = np.asarray(bc)
    dof = np.repeat(bc, 3).astype(bool)          # True: displacement given
    g = np.asarray(given).reshape(-1)
    A = np.where(dof[None, :], -U, T)
    b = U[:, ~dof] @ g[~dof] - T[:, dof] @ g[dof]
    return A, b
