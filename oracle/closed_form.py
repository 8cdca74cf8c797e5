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

Spherical cavity under a wall pressure p(s) Y(x) with Y a spherical
harmonic of degree l (the pressure pushes the solid away from the cavity, so
sigma_rr = -p Y and the wall shear vanishes).  In the Laplace domain the
displacement outside the cavity is u = grad Phi + curl curl (x Psi) with
Phi = A k_l(s r / c_p) Y and Psi = B k_l(s r / c_s) Y, where k_l is the
decaying modified spherical Bessel function, so that
    u = u_r(r) Y e_r + u_t(r) grad_1 Y,
    u_r = f' + l(l+1) g / r,   u_t = (f + g) / r + g',
with f = A k_l(k_p r), g = B k_l(k_s r) and grad_1 Y = r grad Y the surface
gradient on the unit sphere.  The two wall conditions,
    lambda k_p^2 f + 2 mu u_r' = -p,
    2 f'/r - 2 f / r^2 + g'' + (l(l+1) - 2) g / r^2 = 0,
fix A and B (for l = 0 only the first applies and the field is the uniform
case above).
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


# ---- spherical-harmonic wall pressure on a spherical cavity

def _kl_coeffs(l):
    """k_l(x) = exp(-x) sum_n c[n] x^{-n} (n = 1..l+1), the reverse Bessel
    polynomial form of the decaying modified spherical Bessel function."""
    from math import factorial
    c = np.zeros(l + 3)
    for j in range(l + 1):
        c[j + 1] = factorial(l + j) / (factorial(j) * factorial(l - j) * 2.0 ** j)
    return c


def _kl_derivative(c):
    """Coefficients of d/dx of exp(-x) sum c[n] x^{-n}."""
    d = np.zeros(len(c) + 1)
    for n, cn in enumerate(c):
        d[n] -= cn              # from exp(-x)'
        d[n + 1] -= n * cn      # from (x^{-n})'
    return d


def mod_sph_bessel_k(l, x):
    """k_l(x), k_l'(x), k_l''(x) for complex x (normalised so that
    k_0(x) = exp(-x) / x)."""
    x = np.asarray(x, dtype=np.complex128)
    c0 = _kl_coeffs(l)
    c1 = _kl_derivative(c0)
    c2 = _kl_derivative(c1)
    out = []
    for c in (c0, c1, c2):
        v = np.zeros_like(x)
        for n, cn in enumerate(c):
            if cn != 0.0:
                v = v + cn * x ** (-n)
        out.append(np.exp(-x) * v)
    return tuple(out)


def sphere_sh_modes(s, l, a, mat):
    """Amplitudes (A, B) of the two potentials for a unit wall pressure
    coefficient, and the wall displacement factors (Hr, Ht): at r = a,
    u = Hr Y e_r + Ht grad_1 Y."""
    s = complex(s)
    kp, ks = s / mat["cp"], s / mat["cs"]
    lam, mu = mat["lam"], mat["mu"]
    L = l * (l + 1)
    fp = mod_sph_bessel_k(l, kp * a)   # values at r = a of k_l(kp r) and its x-derivatives
    gs = mod_sph_bessel_k(l, ks * a)
    # f, f', f'' per unit A; g, g', g'' per unit B (derivatives in r)
    f = (fp[0], kp * fp[1], kp * kp * fp[2])
    g = (gs[0], ks * gs[1], ks * ks * gs[2])
    # sigma_rr: lambda kp^2 f + 2 mu (f'' + L (g'/a - g/a^2))
    m11 = lam * kp * kp * f[0] + 2 * mu * f[2]
    m12 = 2 * mu * L * (g[1] / a - g[0] / a ** 2)
    if l == 0:
        A, B = -1.0 / m11, 0.0
    else:
        # shear: 2 f'/a - 2 f / a^2 + g'' + (L - 2) g / a^2 = 0
        m21 = 2 * f[1] / a - 2 * f[0] / a ** 2
        m22 = g[2] + (L - 2) * g[0] / a ** 2
        A, B = np.linalg.solve(np.array([[m11, m12], [m21, m22]]), np.array([-1.0, 0.0]))
    Hr = A * f[1] + L * B * g[0] / a
    Ht = (A * f[0] + B * g[0]) / a + B * g[1]
    return A, B, Hr, Ht


def sphere_sh_radial(r, s, l, a, mat):
    """u_r(r), u_t(r) outside the cavity for a unit wall pressure coefficient."""
    A, B, _, _ = sphere_sh_modes(s, l, a, mat)
    s = complex(s)
    kp, ks = s / mat["cp"], s / mat["cs"]
    r = np.asarray(r, dtype=np.float64)
    fp = mod_sph_bessel_k(l, kp * r)
    gs = mod_sph_bessel_k(l, ks * r)
    f, f1 = A * fp[0], A * kp * fp[1]
    g, g1 = B * gs[0], B * ks * gs[1]
    L = l * (l + 1)
    return f1 + L * g / r, (f + g) / r + g1


def surface_gradient(Y, xhat, h=1e-5):
    """grad_1 Y at unit vectors xhat by central differences in the tangent
    plane (Y takes an (n, 3) array of unit vectors)."""
    xhat = np.asarray(xhat, dtype=np.float64)
    ref = np.where(np.abs(xhat[:, :1]) < 0.9, [[1.0, 0.0, 0.0]], [[0.0, 1.0, 0.0]])
    e1 = np.cross(xhat, ref)
    e1 /= np.linalg.norm(e1, axis=1, keepdims=True)
    e2 = np.cross(xhat, e1)
    out = np.zeros_like(xhat)
    for e in (e1, e2):
        fp = Y((xhat + h * e) / np.linalg.norm(xhat + h * e, axis=1, keepdims=True))
        fm = Y((xhat - h * e) / np.linalg.norm(xhat - h * e, axis=1, keepdims=True))
        out += ((fp - fm) / (2 * h))[:, None] * e
    return out


def sphere_sh_displacement(x, s, l, a, mat, Y, gradY=None):
    """Displacement at points x (|x| >= a, cavity centred at the origin) for
    the wall pressure coefficient 1 times Y (degree l).  Y maps unit vectors
    to values; gradY (optional) to surface gradients."""
    x = np.asarray(x, dtype=np.float64)
    r = np.linalg.norm(x, axis=1)
    xh = x / r[:, None]
    ur, ut = sphere_sh_radial(r, s, l, a, mat)
    yv = Y(xh)
    gy = surface_gradient(Y, xh) if gradY is None else gradY(xh)
    return (ur * yv)[:, None] * xh + ut[:, None] * gy


def legendre_Y(l):
    """Axisymmetric harmonic P_l(cos theta) and its exact surface gradient."""
    from numpy.polynomial import legendre as Lg
    c = np.zeros(l + 1)
    c[l] = 1.0
    dc = Lg.legder(c)

    def Y(xh):
        return Lg.legval(xh[:, 2], c)

    def gradY(xh):
        # grad_1 P_l(z) = P_l'(z) (e_z - z xhat)
        z = xh[:, 2]
        ez = np.zeros_like(xh)
        ez[:, 2] = 1.0
        return Lg.legval(z, dc)[:, None] * (ez - z[:, None] * xh)

    return Y, gradY


# ---- plane S-wave (the incident field of the scattering load)

def plane_s_wave(x, s, mat, direction, polarisation):
    """Laplace transform of u(x, t) = pol f(t - dir . x / c_s) for a unit
    spectrum F(s) = 1: pol exp(-s dir . x / c_s), shape (n, 3)."""
    d = np.asarray(direction, float)
    q = np.asarray(polarisation, float)
    x = np.atleast_2d(np.asarray(x, float))
    return np.exp(-complex(s) * (x @ d) / mat["cs"])[:, None] * q[None, :]


def plane_s_wave_stress(x, s, mat, direction, polarisation):
    """Its stress, sigma = 2 mu eps with eps = -(s / 2 c_s) (pol d^T + d pol^T)
    times the phase (the wave is divergence free), shape (n, 3, 3)."""
    d = np.asarray(direction, float)
    q = np.asarray(polarisation, float)
    x = np.atleast_2d(np.asarray(x, float))
    ph = np.exp(-complex(s) * (x @ d) / mat["cs"])
    S = -(mat["mu"] * complex(s) / mat["cs"]) * (np.outer(q, d) + np.outer(d, q))
    return ph[:, None, None] * S[None]


# ---- Stokes' solution: a point force with a time history in the infinite solid

def stokes_point_force(x, x0, direction, t, F, mat, n_quad=96):
    """Displacement u(x, t) of the infinite solid under the point force
    F(t) d at x0 (Stokes, 1849; in the form of Aki and Richards, eq. 4.23):
      4 pi rho u_i = (3 g_i g_j - delta_ij) r^-3 int_{r/c_p}^{r/c_s} tau F(t - tau) dtau
                   + g_i g_j r^-1 c_p^-2 F(t - r/c_p)
                   - (g_i g_j - delta_ij) r^-1 c_s^-2 F(t - r/c_s)
    with r = |x - x0|, g = (x - x0)/r, summed over j with d_j.  F: callable
    of an array of times (zero before its onset); the near-field integral by
    Gauss-Legendre with n_quad nodes.  Returns (len(t), n_points, 3)."""
    x = np.atleast_2d(np.asarray(x, float))
    d = np.asarray(direction, float)
    t = np.asarray(t, float)
    dx = x - np.asarray(x0, float)[None, :]
    r = np.linalg.norm(dx, axis=1)
    g = dx / r[:, None]
    gd = g @ d
    cp, cs, rho = mat["cp"], mat["cs"], mat["rho"]
    xg, wg = np.polynomial.legendre.leggauss(n_quad)
    out = np.zeros((len(t), len(r), 3))
    for p in range(len(r)):
        a, b = r[p] / cp, r[p] / cs
        tau = 0.5 * (b - a) * xg + 0.5 * (b + a)
        wq = 0.5 * (b - a) * wg
        near = np.array([np.sum(wq * tau * F(ti - tau)) for ti in t])
        fp, fs = F(t - a), F(t - b)
        A = (3 * gd[p] * g[p] - d) / r[p] ** 3           # (3 g_i g_j - delta_ij) d_j
        B = gd[p] * g[p] / (r[p] * cp ** 2)                # g_i g_j d_j
        C = (gd[p] * g[p] - d) / (r[p] * cs ** 2)          # (g_i g_j - delta_ij) d_j
        out[:, p, :] = (near[:, None] * A[None, :] + fp[:, None] * B[None, :] - fs[:, None] * C[None, :]) / (4 * pi * rho)
    return out
