"""The frequency loop of the method with dense LU (oracle; test infrastructure).

Sec. 2.2 lists the steps: sample and transform the load, solve the system at
k = 0..N_f/2, fill the rest by conjugate symmetry, invert.  Sec. 3 moves the
frequencies off the real axis and windows the spectrum; Sec. 4 writes the
frequency loop as the sequence A_k a_k = b_k.  For a pure traction problem
(every element loaded by a known traction) the boundary condition step of
Sec. 2.1 leaves A = T and b = U t.  The history enters as a scalar factor:
b_k = P_k U(s_k) t0 for a traction t(x, t) = t0(x) P(t).
"""

import time

import numpy as np

from . import bem, mft
from .kernels import material


def frequency_system(geom, s, mat, t0, self_order=24):
    """A = T(s), b_unit = U(s) t0 for a pure traction problem."""
    T, U = bem.assemble_dense(geom, s, mat, self_order=self_order)
    return T, U @ t0


def transient(xyz, tri, mat_params, period, n_f, sigma, window_kind,
              pressure, history, exterior=True, self_order=24, timings=None,
              bc=None, given=None):
    """Boundary unknowns a(n dt) for n = 0..N_f-1 at every degree of freedom:
    displacements, and for elements with a given displacement (``bc`` = 1)
    tractions.  The load is the pressure field times the history, or, when
    ``bc`` is given, the per-element given values (``given``, N_e x 3)
    times the history.

    Returns dict(s, phat, spec (N_f/2+1, N), u (N_f, N))."""
    mat = material(**mat_params)
    geom = bem.geometry(xyz, tri, exterior=exterior)
    t0 = None if bc is not None else bem.traction_from_pressure(geom, pressure)
    s_k = mft.freq_grid(period, n_f, sigma)
    phat = mft.load_spectrum(history, period, sigma)
    spec = np.zeros((len(s_k), 3 * geom["ne"]), np.complex128)
    for k, s in enumerate(s_k):
        t_a = time.perf_counter()
        if bc is None:
            A, bu = frequency_system(geom, s, mat, t0, self_order=self_order)
        else:
            T, U = bem.assemble_dense(geom, s, mat, self_order=self_order)
            A, bu = bem.mixed_system(T, U, bc, given)
        t_b = time.perf_counter()
        spec[k] = np.linalg.solve(A, phat[k] * bu)
        t_c = time.perf_counter()
        if timings is not None:
            timings.append((t_b - t_a, t_c - t_b))
    u = mft.inverse(spec, period, sigma, window_kind)
    return dict(s=s_k, phat=phat, spec=spec, u=u, geom=geom, mat=mat, t0=t0)


def transient_incident_s(xyz, tri, mat_params, period, n_f, sigma, window_kind, direction, polarisation,
                         history, exterior=True, self_order=24):
    """Scattered displacement on a traction-free boundary under the plane
    S-wave u_inc = pol f(t - dir . x / c_s), f sampled in ``history``:
    b_k = U(s_k) t_sc(s_k) F_k with t_sc the negated traction of the incident
    wave (Sec. 2.1 equation with the scattered field as the unknown).

    Returns dict(s, phat, spec (N_f/2+1, N), u (N_f, N))."""
    mat = material(**mat_params)
    geom = bem.geometry(xyz, tri, exterior=exterior)
    s_k = mft.freq_grid(period, n_f, sigma)
    phat = mft.load_spectrum(history, period, sigma)
    spec = np.zeros((len(s_k), 3 * geom["ne"]), np.complex128)
    for k, s in enumerate(s_k):
        T, U = bem.assemble_dense(geom, s, mat, self_order=self_order)
        t_sc = bem.incident_s_load(geom, s, mat, direction, polarisation)
        spec[k] = np.linalg.solve(T, phat[k] * (U @ t_sc))
    u = mft.inverse(spec, period, sigma, window_kind)
    return dict(s=s_k, phat=phat, spec=spec, u=u, geom=geom, mat=mat)


def transient_incident_s_total(xyz, tri, mat_params, period, n_f, sigma, window_kind, direction,
                               polarisation, history, self_order=24):
    """Total displacement on traction-free cavities under the same plane
    S-wave, total-field formulation: b_k = F_k u_inc(x_i, s_k), A_k = T(s_k).

    Returns dict(s, phat, spec (N_f/2+1, N), u (N_f, N))."""
    mat = material(**mat_params)
    geom = bem.geometry(xyz, tri, exterior=True)
    s_k = mft.freq_grid(period, n_f, sigma)
    phat = mft.load_spectrum(history, period, sigma)
    spec = np.zeros((len(s_k), 3 * geom["ne"]), np.complex128)
    for k, s in enumerate(s_k):
        T, _ = bem.assemble_dense(geom, s, mat, self_order=self_order)
        spec[k] = np.linalg.solve(T, phat[k] * bem.incident_s_total_rhs(geom, s, mat, direction, polarisation))
    u = mft.inverse(spec, period, sigma, window_kind)
    return dict(s=s_k, phat=phat, spec=spec, u=u, geom=geom, mat=mat)
