"""Pins of the learned-guess oracle (network, Adam, basis, samples) on the CPU."""

import math

import numpy as np
import pytest

from oracle import learn as OL


def test_bf16_rounding_matches_torch_and_bit_patterns():
    import torch
    rng = np.random.default_rng(5)
    x = np.concatenate([rng.standard_normal(20000) * 10.0 ** rng.integers(-30, 30, 20000),
                        [0.0, -0.0, 1.0, -2.5, 3.0e38, 1e-40, np.inf, -np.inf]])
    ref = torch.from_numpy(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    got = OL.round_bf16(x)
    assert np.array_equal(np.isinf(got), np.isinf(ref))
    fin = np.isfinite(ref)
    assert np.array_equal(got[fin], ref[fin])
    # ties go to the even neighbour: 1 + 2^-8 lies halfway between 1 and
    # 1 + 2^-7 (odd); 1 + 3 2^-8 halfway between 1 + 2^-7 and 1 + 2^-6 (even)
    assert OL.round_bf16(np.array([1 + 2.0 ** -8]))[0] == 1.0
    assert OL.round_bf16(np.array([1 + 3 * 2.0 ** -8]))[0] == 1 + 2.0 ** -6
    assert OL.round_bf16(np.array([1 + 2.0 ** -8 + 2.0 ** -20]))[0] == 1 + 2.0 ** -7
    assert np.isnan(OL.round_bf16(np.array([np.nan]))[0])


def test_gelu_values_and_derivative():
    # gelu(z) = z Phi(z): Phi(1) = 0.841344746068543, Phi(-1) = 0.158655253931457
    assert abs(OL.gelu(np.array(1.0)) - 0.8413447460685429) < 1e-15
    assert abs(OL.gelu(np.array(-1.0)) + 0.15865525393145707) < 1e-15
    assert OL.gelu(np.array(0.0)) == 0.0
    z = np.linspace(-6, 6, 101)
    h = 1e-5
    fd = (OL.gelu(z + h) - OL.gelu(z - h)) / (2 * h)
    assert np.abs(fd - OL.gelu_grad(z)).max() < 1e-9


def _net(dims, rng, scale=1.0):
    p = []
    for l in range(len(dims) - 1):
        p.append(rng.standard_normal(dims[l + 1] * dims[l]) * scale / math.sqrt(dims[l]))
        p.append(rng.standard_normal(dims[l + 1]) * 0.1)
    return np.concatenate(p)


@pytest.mark.parametrize("dims", [[7, 5, 4, 3], [3, 6, 2], [4, 2]])
def test_gradient_matches_central_differences(dims):
    rng = np.random.default_rng(11)
    p = _net(dims, rng)
    X = rng.standard_normal((6, dims[0]))
    T = rng.standard_normal((6, dims[-1]))
    loss, g = OL.loss_and_grad(p, dims, X, T)
    h = 1e-6
    fd = np.empty_like(p)
    for i in range(p.size):
        e = np.zeros_like(p)
        e[i] = h
        fd[i] = (OL.loss_and_grad(p + e, dims, X, T)[0] - OL.loss_and_grad(p - e, dims, X, T)[0]) / (2 * h)
    assert np.abs(fd - g).max() < 1e-7 * max(1.0, np.abs(g).max())
    assert loss == pytest.approx(np.mean((OL.forward(p, dims, X)[0] - T) ** 2))


def test_forward_in_the_linear_regime_is_the_composed_affine_map():
    # GELU(z) = z to double precision for z >= 10, so with biases that keep
    # every pre-activation above 10 the network is the composition of its
    # affine maps, evaluated here as one product in the opposite order
    rng = np.random.default_rng(3)
    dims = [5, 7, 4, 3]
    layers = [(rng.uniform(-0.3, 0.3, (dims[l + 1], dims[l])), np.zeros(dims[l + 1])) for l in range(3)]
    X = rng.uniform(-1, 1, (9, dims[0]))
    h = X
    for l, (W, b) in enumerate(layers[:-1]):
        z = h @ W.T
        b[:] = 12.0 - z.min(axis=0)
        h = z + b
    W1, b1 = layers[0]
    W2, b2 = layers[1]
    W3, b3 = layers[2]
    b3[:] = rng.standard_normal(dims[3])
    A = W3 @ W2 @ W1
    c = W3 @ (W2 @ b1 + b2) + b3
    p = np.concatenate([np.concatenate([W.ravel(), b]) for W, b in layers])
    Y, _ = OL.forward(p, dims, X)
    assert np.abs(Y - (X @ A.T + c)).max() < 1e-12


def test_adam_first_steps_have_the_closed_form():
    # with a constant gradient the bias-corrected moments are g and g^2, so
    # every step moves each parameter by lr g / (|g| + eps)
    rng = np.random.default_rng(2)
    p0 = rng.standard_normal(50)
    g = rng.standard_normal(50)
    p, _, _ = OL.adam(p0, lambda q: (0.0, g), steps=3, lr=1e-2)
    assert np.abs(p - (p0 - 3e-2 * g / (np.abs(g) + 1e-8))).max() < 1e-14
    # on f(p) = |p|^2 / 2 the first step is p0 - lr sign(p0), the second
    # uses the moments of the two gradients
    p, l0, _ = OL.adam(p0, lambda q: (0.5 * q @ q, q.copy()), steps=2, lr=0.1)
    p1 = p0 - 0.1 * p0 / (np.abs(p0) + 1e-8)
    m = 0.9 * 0.1 * p0 + 0.1 * p1
    v = 0.999 * 0.001 * p0 ** 2 + 0.001 * p1 ** 2
    p2 = p1 - 0.1 * (m / (1 - 0.81)) / (np.sqrt(v / (1 - 0.999 ** 2)) + 1e-8)
    assert np.abs(p - p2).max() < 1e-12
    assert l0 == pytest.approx(0.5 * p0 @ p0)


def test_pod_basis_is_eckart_young():
    rng = np.random.default_rng(8)
    N, M, n = 60, 40, 30
    U, _ = np.linalg.qr(rng.standard_normal((N, n)) + 1j * rng.standard_normal((N, n)))
    V, _ = np.linalg.qr(rng.standard_normal((M, n)) + 1j * rng.standard_normal((M, n)))
    sv = 2.0 ** -np.arange(n, dtype=float)
    S = (U * sv) @ V.conj().T
    for r in (1, 5, 12):
        Phi, e = OL.pod_basis(S, r)
        assert np.abs(Phi.conj().T @ Phi - np.eye(r)).max() < 1e-12
        res = np.linalg.norm(S - Phi @ (Phi.conj().T @ S)) ** 2
        assert res == pytest.approx((sv[r:] ** 2).sum(), rel=1e-8)
        assert e == pytest.approx((sv[:r] ** 2).sum() / (sv ** 2).sum(), rel=1e-12)


def test_pod_basis_of_unit_snapshots():
    """Scaling snapshots does not change the unit-norm basis (its projector),
    the unit-norm basis of unit-norm snapshots is the plain one, and with
    snapshots of very different sizes the unit weighting keeps directions
    the plain basis drops."""
    rng = np.random.default_rng(9)
    N, M = 50, 30
    S = rng.standard_normal((N, M)) + 1j * rng.standard_normal((N, M))
    proj = lambda P: P @ P.conj().T
    P1, e1 = OL.pod_basis(S, 7, unit=True)
    P2, e2 = OL.pod_basis(S * (10.0 ** rng.uniform(-6, 6, M))[None, :], 7, unit=True)
    assert np.abs(proj(P1) - proj(P2)).max() < 1e-9 and e1 == pytest.approx(e2, rel=1e-10)
    Su = S / np.linalg.norm(S, axis=0)[None, :]
    P3, e3 = OL.pod_basis(Su, 7)
    assert np.abs(proj(P1) - proj(P3)).max() < 1e-9 and e1 == pytest.approx(e3, rel=1e-12)
    # one large snapshot among small orthogonal ones: the plain basis of rank 1
    # is that snapshot; the unit basis weights all alike
    Q, _ = np.linalg.qr(rng.standard_normal((N, 4)))
    T = Q * np.array([1e6, 1.0, 1.0, 1.0])[None, :]
    Pp, _ = OL.pod_basis(T, 1)
    assert abs(abs(Pp[:, 0] @ Q[:, 0]) - 1) < 1e-12
    Pu, eu = OL.pod_basis(T, 3, unit=True)
    assert eu == pytest.approx(0.75, rel=1e-12)


def test_learned_column_has_the_predicted_coordinates():
    """The column's coordinates are the composed prediction and its part
    outside the basis is the quadratic extrapolation's."""
    rng = np.random.default_rng(10)
    N, r = 40, 6
    Phi, _ = np.linalg.qr(rng.standard_normal((N, r)) + 1j * rng.standard_normal((N, r)))
    a1, a2, a3 = (rng.standard_normal(N) + 1j * rng.standard_normal(N) for _ in range(3))
    y = rng.standard_normal(2 * r)
    nu = 0.37
    x = OL.learned_column(a1, a2, a3, Phi, nu, y)
    c = [Phi.conj().T @ a for a in (a1, a2, a3)]
    assert np.abs(Phi.conj().T @ x - OL.compose(c[0], c[1], c[2], nu, y)).max() < 1e-12
    out = lambda v: v - Phi @ (Phi.conj().T @ v)
    assert np.abs(out(x) - out(3 * a1 - 3 * a2 + a3)).max() < 1e-12
    # a zero correction gives the extrapolation itself
    assert np.abs(OL.learned_column(a1, a2, a3, Phi, nu, np.zeros(2 * r)) - (3 * a1 - 3 * a2 + a3)).max() < 1e-13
    # with a base prediction the coordinates are base + nu y, the outside part unchanged
    base = rng.standard_normal(r) + 1j * rng.standard_normal(r)
    xb = OL.learned_column(a1, a2, a3, Phi, nu, y, base=base)
    assert np.abs(Phi.conj().T @ xb - (base + nu * (y[:r] + 1j * y[r:]))).max() < 1e-12
    assert np.abs(out(xb) - out(3 * a1 - 3 * a2 + a3)).max() < 1e-12


def test_samples_of_a_quadratic_sequence_have_zero_target():
    rng = np.random.default_rng(4)
    r = 9
    a, b, c = (rng.standard_normal(r) + 1j * rng.standard_normal(r) for _ in range(3))
    coef = lambda k: a + b * k + c * k * k
    k = 7
    x, t, nu = OL.sample(coef(k - 1), coef(k - 2), coef(k - 3), k / 16, coef(k))
    assert x.shape == (6 * r + 2,) and t.shape == (2 * r,)
    assert np.abs(t).max() < 1e-13 * np.abs(coef(k)).max()
    assert nu == pytest.approx(np.linalg.norm(coef(k - 1)))
    assert x[-2] == k / 16 and x[-1] == (k / 16) ** 2
    # homogeneous: scaled coordinates give the same sample
    x2, t2, nu2 = OL.sample(5 * coef(k - 1), 5 * coef(k - 2), 5 * coef(k - 3), k / 16, 5 * coef(k) + 1.0)
    assert np.abs(x2 - x).max() < 1e-15 and nu2 == pytest.approx(5 * nu)
    # compose inverts the target
    c0 = rng.standard_normal(r) + 1j * rng.standard_normal(r)
    x, t, nu = OL.sample(coef(k - 1), coef(k - 2), coef(k - 3), 0.5, c0)
    assert np.abs(OL.compose(coef(k - 1), coef(k - 2), coef(k - 3), nu, t) - c0).max() < 1e-12
    # a zero history has nu = 1 and a zero input
    x, _, nu = OL.sample(np.zeros(r), np.zeros(r), np.zeros(r), 0.25)
    assert nu == 1.0 and np.all(x[:-2] == 0)


def _cases(rng, n, nk, r):
    return rng.standard_normal((n, nk, r)) + 1j * rng.standard_normal((n, nk, r))


def test_ridge_recovers_an_exact_linear_recurrence():
    """Coordinates that follow c_k = M_k [c_{k-1}; c_{k-2}; c_{k-3}] exactly,
    with more cases than history entries, give back M_k on a new history."""
    rng = np.random.default_rng(11)
    n, nk, r, k = 40, 6, 4, 5
    C = _cases(rng, n, nk, r)
    M = (rng.standard_normal((r, 3 * r)) + 1j * rng.standard_normal((r, 3 * r))) / 4
    C[:, k, :] = (M @ np.concatenate([C[:, k - 1], C[:, k - 2], C[:, k - 3]], axis=1).T).T
    # (more cases than entries make the dual Gram matrix singular, so the
    # regularisation sets the accuracy: bias ~ eps, rounding ~ 1e-16 / eps)
    X, W, ad = OL.ridge_fit(C, k, eps=1e-10)
    h = rng.standard_normal(3 * r) + 1j * rng.standard_normal(3 * r)
    assert np.abs(OL.ridge_predict(X, W, h) - M @ h).max() < 1e-5 * np.abs(M @ h).max()


def test_ridge_interpolates_and_combines_training_cases():
    """With fewer cases than history entries the fit reproduces each
    training target, and a combination of training histories is mapped to
    the same combination of their targets (the solution is linear in the
    load, so this is what a combined load needs)."""
    rng = np.random.default_rng(12)
    n, nk, r, k = 7, 5, 6, 4
    C = _cases(rng, n, nk, r)
    X, W, ad = OL.ridge_fit(C, k, eps=1e-12)
    for i in range(n):
        assert np.abs(OL.ridge_predict(X, W, X[:, i]) - C[i, k]).max() < 1e-9
    w = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    assert np.abs(OL.ridge_predict(X, W, X @ w) - C[:, k, :].T @ w).max() < 1e-8


def test_ridge_leave_one_out_matches_refitting():
    rng = np.random.default_rng(13)
    n, nk, r, k = 9, 5, 3, 3
    C = _cases(rng, n, nk, r)
    X, W, ad = OL.ridge_fit(C, k, eps=1e-3)
    R = OL.ridge_loo(W, ad)
    G = X.conj().T @ X
    lam = 1e-3 * np.trace(G).real / n
    for i in range(n):
        keep = [j for j in range(n) if j != i]
        Xi, Yi = X[:, keep], C[keep, k, :].T
        Wi = Yi @ np.linalg.inv(Xi.conj().T @ Xi + lam * np.eye(n - 1))
        ref = C[i, k] - Wi @ (Xi.conj().T @ X[:, i])
        assert np.abs(R[:, i] - ref).max() < 1e-10 * np.abs(ref).max()


def test_ridge_training_predictions_closed_form():
    """W X^H X = Y - lam W: the dual form's own residual on its training
    cases is lam times its coefficients."""
    rng = np.random.default_rng(14)
    n, nk, r, k = 6, 5, 4, 4
    C = _cases(rng, n, nk, r)
    eps = 1e-3
    X, W, ad = OL.ridge_fit(C, k, eps=eps)
    G = X.conj().T @ X
    lam = eps * np.trace(G).real / n
    assert np.abs(OL.ridge_train_predictions(X, W) - (C[:, k, :].T - lam * W)).max() < 1e-10


def test_learned_guess_step():
    """The step is the least-squares one (the new residual is orthogonal to
    A v); exact coordinates of a solution whose extrapolation error lies in
    the basis give that solution; a prediction equal to the extrapolation's
    own coordinates changes nothing."""
    rng = np.random.default_rng(15)
    N, r = 30, 5
    A = rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N)) + 6 * np.eye(N)
    Phi, _ = np.linalg.qr(rng.standard_normal((N, r)) + 1j * rng.standard_normal((N, r)))
    a = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    b = A @ a
    xs = a + Phi @ (rng.standard_normal(r) + 1j * rng.standard_normal(r))
    rs = b - A @ xs
    x0, r0, g = OL.learned_guess(xs, rs, Phi, Phi.conj().T @ a, lambda v: A @ v)
    assert abs(g - 1) < 1e-12 and np.abs(x0 - a).max() < 1e-12 and np.abs(r0).max() < 1e-10
    p = rng.standard_normal(r) + 1j * rng.standard_normal(r)
    x0, r0, g = OL.learned_guess(xs, rs, Phi, p, lambda v: A @ v)
    v = Phi @ (p - Phi.conj().T @ xs)
    assert abs(np.vdot(A @ v, r0)) < 1e-10 * np.linalg.norm(A @ v) * np.linalg.norm(r0)
    assert np.linalg.norm(r0) <= np.linalg.norm(rs)
    assert np.abs(r0 - (b - A @ x0)).max() < 1e-10
    x0, r0, g = OL.learned_guess(xs, rs, Phi, Phi.conj().T @ xs, lambda v: A @ v)
    assert g == 0.0 and np.array_equal(x0, xs)
