"""Solution extrapolation method (oracle; test infrastructure).

Sec. 4.2: the initial guess for A_k a_k = b_k is a combination X s of the K
previous solutions X = (a_{k-1}, ..., a_{k-K}); with Y = A_k X and the QR
factorisation Y = Q R, the least-squares coefficients are s = R^{-1} Q^H b_k
(the printed formula omits the conjugate transpose, which a complex least
squares problem needs).  Readings: k = 0 starts from zero, k < K uses the
solutions that exist, and columns whose |R_ii| falls below 1e-12 |R_11| are
dropped (a rank-deficient history).
"""

import numpy as np


def sem_guess(A_apply, X, b, drop=1e-12):
    """x0 = X R^{-1} Q^H b, Y = A X = Q R.  ``A_apply`` maps an (N, K) array
    to A times it; ``X`` is (N, K) with K >= 0 columns."""
    X = np.asarray(X)
    if X.ndim == 1:
        X = X[:, None]
    if X.shape[1] == 0:
        return np.zeros_like(b)
    Y = A_apply(X)
    Q, R = np.linalg.qr(Y)
    d = np.abs(np.diag(R))
    keep = d > drop * d[0]
    if not keep.all():
        X = X[:, keep]
        Q, R = np.linalg.qr(Y[:, keep])
    s = np.linalg.solve(R, Q.conj().T @ b)
    return X @ s


def quadratic_extrapolation(history):
    """Lagrange extrapolation to the next equispaced frequency from the last
    three solutions (newest first): 3 a1 - 3 a2 + a3."""
    if len(history) == 0:
        return None
    if len(history) == 1:
        return history[0].copy()
    if len(history) == 2:
        return 2.0 * history[0] - history[1]
    return 3.0 * history[0] - 3.0 * history[1] + history[2]
