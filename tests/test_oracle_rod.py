"""Pins for mixed boundary conditions and the prismatic rod (Sec. 2.1,
eq. Aa_b; Sec. 5.1).

* the column swap of the mixed system is checked on a consistent pair
  (u, t) with T u = U t built from a random matrix pair;
* the rod's closed-form step responses transform to the Laplace-domain
  closed forms H(s)/s (quadrature);
* the oracle's 3-D rod (nu = 0, fixed end, traction at the other end)
  converges to the 1-D solution as the mesh is refined.
"""

import numpy as np
import pytest
from scipy import integrate

from oracle import bem, closed_form as CF, kernels as K
from synth import box_mesh


def test_mixed_system_column_swap():
    rng = np.random.default_rng(8)
    ne = 6
    N = 3 * ne
    T = rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N)) + 4 * np.eye(N)
    U = rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))
    t = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    u = np.linalg.solve(T, U @ t)            # a consistent boundary state
    bc = np.array([0, 1, 0, 1, 1, 0])
    dof = np.repeat(bc, 3).astype(bool)
    given = np.where(dof, u, t).reshape(ne, 3)
    A, b = bem.mixed_system(T, U, bc, given)
    a = np.linalg.solve(A, b)
    assert np.allclose(a, np.where(dof, t, u), atol=1e-12)


def test_rod_step_responses_transform_to_closed_forms():
    mat = K.material(1.0, 1.0, 0.0)
    L = 3.0
    for s in (0.5, 0.5 + 1.0j, 0.8 - 0.3j):
        for f_t, H in ((CF.rod_step_end_displacement, CF.rod_end_displacement_H),
                       (CF.rod_step_fixed_stress, CF.rod_fixed_stress_H)):
            c, _ = CF.rod_wave_speed(mat)
            brk = [k * L / c for k in range(1, 60)]
            g = lambda t: f_t(t, L, mat) * np.exp(-s * t)
            re, _ = integrate.quad(lambda t: np.real(g(t)), 0, 120, limit=2000, points=brk)
            im, _ = integrate.quad(lambda t: np.imag(g(t)), 0, 120, limit=2000, points=brk)
            ref = H(s, L, mat) / s
            assert abs((re + 1j * im) - ref) < 1e-7 * abs(ref)


def _rod(div, s):
    mat = K.material(1.0, 1.0, 0.0)
    L = 3.0
    xyz, tri, face = box_mesh((L, 1, 1), div, origin=(0, -0.5, -0.5))
    g = bem.geometry(xyz, tri, exterior=False)
    bc = (face == 0).astype(int)
    given = np.zeros((len(tri), 3))
    given[face == 1, 0] = 1.0
    T, U = bem.assemble_dense(g, s, mat)
    A, b = bem.mixed_system(T, U, bc, given)
    a = np.linalg.solve(A, b).reshape(-1, 3)
    uL = a[face == 1, 0].mean()
    sig0 = -a[face == 0, 0].mean()       # traction t_x = -sigma_xx on the x = 0 face
    eu = abs(uL - CF.rod_end_displacement_H(s, L, mat)) / abs(CF.rod_end_displacement_H(s, L, mat))
    es = abs(sig0 - CF.rod_fixed_stress_H(s, L, mat)) / abs(CF.rod_fixed_stress_H(s, L, mat))
    return eu, es


@pytest.mark.slow
def test_rod_converges_to_one_dimensional_solution():
    s = 0.5 + 1.0j
    eu1, es1 = _rod((6, 2, 2), s)
    eu2, es2 = _rod((12, 4, 4), s)
    assert eu2 < 0.02 and es2 < 0.04
    assert eu2 < 0.7 * eu1 and es2 < 0.7 * es1
