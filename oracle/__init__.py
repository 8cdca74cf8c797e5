"""CPU oracle for the exponential-window frequency-domain BEM (test infrastructure).

This package is test infrastructure, not part of the product.  Only the test
suite, the smoke check and the CPU-baseline leg of the benchmark import it;
the GPU library never links, imports or calls it, and it shares no code,
tables or constants with the GPU path.  Its only common dependency with the
GPU side is the ``synth`` input generator, which holds none of the method's
arithmetic.

It is plain, dense and slow on purpose: complex128 throughout, every matrix
entry assembled explicitly, each frequency solved by LU, the inverse
transform done as a direct O(N_f^2) sum.

Modules
-------
kernels      Laplace-domain displacement/traction fundamental solutions
             (Sec. 2.1, the U_ij, T_ij = G_ikj n_k and phi/psi definitions).
quadrature   7-point triangle rule, Duffy rule, Gauss-Legendre on [0, 1].
bem          geometry, singular self-element integrals, dense T and U
             (Sec. 2.1, boundary integral equation and the system T u = U t).
mft          frequency grid, damped DFT, windows, de-damped inverse DFT
             (Sec. 2.2 and Sec. 3).
sem          least-squares solution extrapolation (Sec. 4.2).
solve        the frequency loop with LU and the transient result.
closed_form  pressurised spherical cavity, Kelvin static kernels.

Parity status: every function here is pinned by a CPU test against a closed
form, an invariant, a textbook rule or brute force (tests/test_oracle_*.py).
"""
