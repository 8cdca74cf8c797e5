"""Closed-form solutions used to pin the oracle (test infrastructure).

Pressurised spherical cavity of radius a in an infinite elastic solid: the
radial displacement of the wall for a wall pressure with Laplace transform
p(s) is u_r(a, s) = p(s) H(s),

    H(s) = a (1 + s a / c_p) / (rho a^2 s^2 + 4 mu (1 + s a / c_p)),

from the compressional potential exp(-s r / c_p) / r with the wall condition
sigma_rr = -p.  H(0) = a / (4 mu) is Lame's static result.  The transient
responses follow by residues at the two poles of H.

Prismatic rod with Poisson ratio 0 (Sec. 5.1): length L along x, fixed at
x = 0, traction p(t) along x on the end x = L, the other faces free.  With
nu = 0 there is no lateral contraction and the 3-D field is the 1-D bar
u_tt = c^2 u_xx with c^2 = E / rho = 2 mu / rho, so in the Laplace domain

    u(L, s)      = p(s) (c / (E s)) tanh(s L / c)
    sigma(0, s)  = p(s) / cosh(s L / c)

and for a unit step the end displacement is a triangle wave rising to
2 L / E at t = 2 L / c and the stress at the fixed end a square wave
between 0 and 2, both of period 4 L / c.

Kelvin's static kernels (the s -> 0 limit of U and T) are written out
independently of the oracle's dynamic kernels.
"""

from math import pi

import numpy as np


def sphere_H(s, a, mat):
    s = np.asarray(s, dtype=np.complex128)
    q = 1.0 + s * a / mat["cp"]
    return a * q / (mat["rho"] * a * a * s * s + 4.0 * mat["mu"] * q)


def sphere_poles(a, mat):
    """Roots of rho a^2 s^2 + (4 mu a / c_p) s + 4 mu (upper one first)."""
    r = np.roots([mat["rho"] * a * a, 4.0 * mat["mu"] * a / mat["cp"], 4.0 * mat["mu"]])
    return tuple(sorted(r, key=lambda z: -z.imag))


def _residue(a, mat):
    sp, sm = sphere_poles(a, mat)
    Rp = a * (1.0 + sp * a / mat["cp"]) / (mat["rho"] * a * a * sp * (sp - sm))
    return sp, Rp


def sphere_step_response(t, a, mat):
    """Wall displacement for a unit pressure step: H(0) + 2 Re[R+ e^{s+ t}]."""
    t = np.asarray(t, dtype=np.float64)
    sp, Rp = _residue(a, mat)
    g = a / (4.0 * mat["mu"]) + 2.0 * np.real(Rp * np.exp(sp * t))
    return np.where(t >= 0, g, 0.0)


def _step_integral(t, a, mat):
    sp, Rp = _residue(a, mat)
    G = a / (4.0 * mat["mu"]) * t + 2.0 * np.real(Rp * (np.exp(sp * t) - 1.0) / sp)
    return np.where(t >= 0, G, 0.0)


def sphere_ramp_response(t, a, mat, t_rise):
    """Wall displacement for a pressure rising linearly to 1 over t_rise."""
    t = np.asarray(t, dtype=np.float64)
    if t_rise <= 0:
        return sphere_step_response(t, a, mat)
    return (_step_integral(t, a, mat) - _step_integral(t - t_rise, a, mat)) / t_rise


def kelvin_U(x, y, mat):
    d = np.asarray(y, float) - np.asarray(x, float)
    r = np.linalg.norm(d, axis=-1)
    rh = d / r[..., None]
    nu, mu = mat["nu"], mat["mu"]
    c = 1.0 / (16.0 * pi * mu * (1.0 - nu) * r)
    return c[..., None, None] * ((3.0 - 4.0 * nu) * np.eye(3)
                                 + rh[..., :, None] * rh[..., None, :])


def kelvin_T(x, y, n, mat):
    d = np.asarray(y, float) - np.asarray(x, float)
    r = np.linalg.norm(d, axis=-1)
    rh = d / r[..., None]
    n = np.broadcast_to(np.asarray(n, float), rh.shape)
    nu = mat["nu"]
    drdn = np.einsum("...k,...k->...", rh, n)
    c = -1.0 / (8.0 * pi * (1.0 - nu) * r * r)
    inner = (drdn[..., None, None] * ((1.0 - 2.0 * nu) * np.eye(3)
                                      + 3.0 * rh[..., :, None] * rh[..., None, :])
             - (1.0 - 2.0 * nu) * (rh[..., :, None] * n[..., None, :]
                                    - n[..., :, None] * rh[..., None, :]))
    return c[..., None, None] * inner


def rod_wave_speed(mat):
    """c = sqrt(E / rho) of the 1-D bar (equals c_p when nu = 0)."""
    E = 2.0 * mat["mu"] * (1.0 + mat["nu"])
    return np.sqrt(E / mat["rho"]), E


def rod_end_displacement_H(s, L, mat):
    c, E = rod_wave_speed(mat)
    s = np.asarray(s, dtype=np.complex128)
    return (c / (E * s)) * np.tanh(s * L / c)


def rod_fixed_stress_H(s, L, mat):
    c, _ = rod_wave_speed(mat)
    s = np.asarray(s, dtype=np.complex128)
    return 1.0 / np.cosh(s * L / c)


def rod_step_end_displacement(t, L, mat):
    """u(L, t) for a unit step traction: triangle wave of period 4L/c."""
    c, E = rod_wave_speed(mat)
    t = np.asarray(t, dtype=np.float64)
    tau = np.mod(t, 4.0 * L / c)
    tri = np.where(tau <= 2.0 * L / c, tau, 4.0 * L / c - tau)
    return np.where(t >= 0, c * tri / E, 0.0)


def rod_step_fixed_stress(t, L, mat):
    """sigma_xx(0, t) for a unit step traction: 0 before L/c, then 2 and 0
    alternating every 2L/c."""
    c, _ = rod_wave_speed(mat)
    t = np.asarray(t, dtype=np.float64)
    tau = np.mod(t - L / c, 4.0 * L / c)
    return np.where((t >= L / c) & (tau < 2.0 * L / c), 2.0, 0.0)
