"""Learned initial guess (oracle; test infrastructure).

An addition to the method, not part of the paper: Sec. 4.2's extrapolation
takes one more column, a network's prediction of the next frequency's
solution.  What is defined here, plainly and in float64:

* proper orthogonal decomposition: the basis is the r leading left singular
  vectors of the snapshot matrix (numpy's SVD), optionally of the snapshots
  scaled to unit norm;
* the learned column: the quadratic extrapolation of the last three
  solutions plus the network's correction mapped through the basis;
* a regularised least-squares map per frequency from the three previous
  coordinate vectors to the next (dual form over the training cases), its
  predictions of the training cases and its leave-one-out residuals;
* the learned guess: the least-squares extrapolation with its part in the
  basis moved towards the predicted coordinates by a residual-minimising
  step;
* reduced coordinates c = Phi^H a, and the samples: input
  [Re c1, Im c1, Re c2, Im c2, Re c3, Im c3] / nu followed by f and f^2,
  target [Re e, Im e] / nu with e = c_k - (3 c1 - 3 c2 + c3), where
  c1, c2, c3 are the coordinates at k-1, k-2, k-3, nu = |c1| (1 when zero)
  and f = k / (N_f / 2);
* the network y = W_L g(... g(W_1 x + b_1) ...) + b_L, g(z) = z Phi(z)
  (GELU with the normal CDF), its mean squared error and the gradient by
  the chain rule, and Adam (Kingma and Ba, Algorithm 1) with bias
  correction;
* the precision the GPU kernels use (an implementation choice, mirrored so
  that parity can be tight): with ``bf16=True`` every operand of a matrix
  product -- weights, layer inputs and the back-propagated gradients -- is
  first rounded to float32 and then to bfloat16 (round to nearest, ties to
  even); sums, biases, activations and the loss stay in float64.

Pins (tests/test_oracle_learn.py): bfloat16 rounding against torch's CPU
conversion and hand-checked bit patterns; GELU against values of the normal
CDF; the gradient against central differences; the forward pass of a net in
its linear regime against the product of its affine maps; the first Adam
steps against their closed form; the basis against Eckart-Young on matrices
of known singular values; the samples against exactly quadratic coordinate
sequences (zero target).
"""

import math

import numpy as np
from scipy.special import erf


# ---- bfloat16

def round_bf16(x):
    """float64 array -> float64 array of the nearest bfloat16 values, going
    through float32 (round to nearest even at both steps)."""
    f = np.ascontiguousarray(np.asarray(x, dtype=np.float64).astype(np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    special = (u & 0x7F800000) == 0x7F800000
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    quiet = np.where((u & 0x007FFFFF) != 0, np.uint64(0x00400000), np.uint64(0))
    r = np.where(special, (u & np.uint64(0xFFFF0000)) | quiet, r)
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


# ---- network

def gelu(z):
    return 0.5 * z * (1.0 + erf(z / math.sqrt(2.0)))


def gelu_grad(z):
    return 0.5 * (1.0 + erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


def unpack(params, dims):
    """Flat parameters -> [(W_l, b_l)], W_l of shape (dims[l+1], dims[l])."""
    out, o = [], 0
    for l in range(len(dims) - 1):
        n_w = dims[l + 1] * dims[l]
        W = np.asarray(params[o:o + n_w], dtype=np.float64).reshape(dims[l + 1], dims[l])
        o += n_w
        b = np.asarray(params[o:o + dims[l + 1]], dtype=np.float64)
        o += dims[l + 1]
        out.append((W, b))
    if o != len(params):
        raise ValueError("parameter count does not match the widths")
    return out


def n_params(dims):
    return sum(dims[l + 1] * dims[l] + dims[l + 1] for l in range(len(dims) - 1))


def forward(params, dims, X, bf16=False):
    """Output (M, dims[-1]) and the cache of inputs and pre-activations."""
    rnd = round_bf16 if bf16 else (lambda a: a)
    layers = unpack(params, dims)
    h = np.asarray(X, dtype=np.float64)
    cache = []
    for l, (W, b) in enumerate(layers):
        z = rnd(h) @ rnd(W).T + b
        cache.append((h, z))
        h = gelu(z) if l + 1 < len(layers) else z
    return h, cache


def loss_and_grad(params, dims, X, T, bf16=False):
    """Mean squared error over all entries and its gradient (flat)."""
    rnd = round_bf16 if bf16 else (lambda a: a)
    layers = unpack(params, dims)
    Y, cache = forward(params, dims, X, bf16)
    E = Y - np.asarray(T, dtype=np.float64)
    n = E.size
    loss = float(np.sum(E * E) / n)
    dz = 2.0 * E / n
    grads = [None] * len(layers)
    for l in range(len(layers) - 1, -1, -1):
        W, _ = layers[l]
        h_in, _ = cache[l]
        gW = rnd(dz).T @ rnd(h_in)
        gb = dz.sum(axis=0)
        grads[l] = (gW, gb)
        if l > 0:
            dz = (rnd(dz) @ rnd(W)) * gelu_grad(cache[l - 1][1])
    flat = np.concatenate([np.concatenate([gW.ravel(), gb]) for gW, gb in grads])
    return loss, flat


def adam(params, grad_fn, steps, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """``steps`` Adam steps from zero moments with a constant step size;
    grad_fn(params) -> (loss, gradient).  Returns the parameters and the
    losses before the first and after the last step."""
    p = np.asarray(params, dtype=np.float64).copy()
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    first = None
    for t in range(1, steps + 1):
        loss, g = grad_fn(p)
        if first is None:
            first = loss
        m = beta1 * m + (1 - beta1) * g
        v = beta2 * v + (1 - beta2) * g * g
        p = p - lr * (m / (1 - beta1 ** t)) / (np.sqrt(v / (1 - beta2 ** t)) + eps)
    last = grad_fn(p)[0]
    return p, (last if first is None else first), last


# ---- reduced coordinates and samples

def pod_basis(S, r, unit=False):
    """The r leading left singular vectors of S (N x M) and the fraction of
    |S|_F^2 they capture; with ``unit`` those of S with every nonzero column
    scaled to unit norm (each snapshot weighted alike)."""
    S = np.asarray(S)
    if unit:
        n = np.linalg.norm(S, axis=0)
        S = S / np.where(n > 0, n, 1.0)[None, :]
    U, sv, _ = np.linalg.svd(S, full_matrices=False)
    e = sv ** 2
    return U[:, :r], float(e[:r].sum() / e.sum()) if e.sum() > 0 else 1.0


def sample(c1, c2, c3, f, c0=None, base=None):
    """Network input (6 r + 2), target (2 r, or None) and nu from the
    coordinates at k-1, k-2, k-3 (and k).  The target is the correction to
    ``base`` (default: the quadratic extrapolation 3 c1 - 3 c2 + c3)."""
    c1, c2, c3 = (np.asarray(c, dtype=complex) for c in (c1, c2, c3))
    nu = float(np.linalg.norm(c1))
    if nu == 0.0:
        nu = 1.0
    x = np.concatenate([c1.real, c1.imag, c2.real, c2.imag, c3.real, c3.imag]) / nu
    x = np.concatenate([x, [f, f * f]])
    t = None
    if c0 is not None:
        b = (3 * c1 - 3 * c2 + c3) if base is None else np.asarray(base, dtype=complex)
        e = np.asarray(c0, dtype=complex) - b
        t = np.concatenate([e.real, e.imag]) / nu
    return x, t, nu


# ---- the linear part of the prediction: a regularised least-squares map per
# frequency from the three previous coordinate vectors to the next

def ridge_fit(C, k, eps=1e-8):
    """C: coordinates of the training cases, shape (n_cases, n_k, r).  For
    frequency k >= 3 the history of case i is h_i = [c_{k-1}; c_{k-2};
    c_{k-3}] (3 r) and its target y_i = c_k.  The map y = W X^H h minimises
    sum_i |y_i - W X^H h_i|^2 + lam |W|^2-type penalty in its dual form:
    with X = [h_1 .. h_n] (3 r x n), Y = [y_1 .. y_n] (r x n),
    G = X^H X and lam = eps tr(G) / n, A = (G + lam I)^{-1} and W = Y A.
    Returns X, W and diag(A)."""
    C = np.asarray(C, dtype=complex)
    X = np.concatenate([C[:, k - 1, :], C[:, k - 2, :], C[:, k - 3, :]], axis=1).T
    Y = C[:, k, :].T
    G = X.conj().T @ X
    n = G.shape[0]
    lam = eps * np.trace(G).real / n
    A = np.linalg.inv(G + lam * np.eye(n))
    return X, Y @ A, np.diag(A).copy()


def ridge_predict(X, W, h):
    """Prediction W X^H h for the history h = [c_{k-1}; c_{k-2}; c_{k-3}]."""
    return W @ (X.conj().T @ np.asarray(h, dtype=complex))


def ridge_train_predictions(X, W):
    """The map's predictions of its own training cases, W X^H X (r x n)."""
    return W @ (X.conj().T @ X)


def learned_guess(xs, rs, Phi, p, A):
    """The learned initial guess from the least-squares extrapolation xs
    (residual rs = b - A xs) and predicted coordinates p: the part of xs in
    the basis is moved towards p along v = Phi (p - Phi^H xs) by the step
    gamma minimising |rs - gamma A v|.  A: callable x -> A x.  Returns
    (x0, r0, gamma)."""
    v = Phi @ (np.asarray(p) - Phi.conj().T @ xs)
    y = A(v)
    yy = np.vdot(y, y).real
    gamma = np.vdot(y, rs) / yy if yy > 0 else 0.0
    return xs + gamma * v, rs - gamma * y, gamma


def ridge_loo(W, adiag):
    """Leave-one-out residuals of the dual fit: y_i minus the prediction of a
    fit without case i, which is column i of W divided by A_ii (the
    Sherman-Morrison identity for the kernel form)."""
    return W / np.asarray(adiag)[None, :]


def compose(c1, c2, c3, nu, y, base=None):
    """Predicted coordinates: base + nu (y_re + i y_im), base defaulting to
    the quadratic extrapolation 3 c1 - 3 c2 + c3."""
    r = len(c1)
    b = (3 * np.asarray(c1) - 3 * np.asarray(c2) + np.asarray(c3)) if base is None else np.asarray(base)
    return b + nu * (y[:r] + 1j * y[r:])


def learned_column(a1, a2, a3, Phi, nu, y, base=None):
    """The learned column of the extrapolation: the quadratic extrapolation
    of the last three solutions with its coordinates replaced by the
    prediction, 3 a1 - 3 a2 + a3 + Phi (p - (3 c1 - 3 c2 + c3)) where
    p = compose(c1, c2, c3, nu, y, base) and c_j = Phi^H a_j.  Its part
    outside the basis is that of the extrapolation."""
    a1, a2, a3 = (np.asarray(a) for a in (a1, a2, a3))
    c = [Phi.conj().T @ a for a in (a1, a2, a3)]
    q = 3 * c[0] - 3 * c[1] + c[2]
    p = compose(c[0], c[1], c[2], nu, y, base)
    return 3 * a1 - 3 * a2 + a3 + Phi @ (p - q)
