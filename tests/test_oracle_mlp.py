"""Pins of the FP64 warm-start network reference (CPU only): gradients against
central finite differences, the loss's invariances and its closed-form values."""
import numpy as np
import pytest

from oracle import mlp as R


def _problem(n=300, k=6, seed=0):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n, 11))
    T = np.linalg.qr(rng.standard_normal((n, k)))[0]
    d = rng.uniform(0.5, 2.0, size=n)
    p = R.init_params(k, seed=seed)
    return X, T, d, p


def test_param_count():
    assert R.param_count(32) == 128 * 11 + 128 + 2 * (128 * 128 + 128) + 32 * 128 + 32


def test_gradient_matches_finite_differences():
    X, T, d, p = _problem()
    k = T.shape[1]
    L, g = R.loss_and_grad(p, X, T, d, k)
    rng = np.random.default_rng(1)
    idx = rng.choice(p.size, size=40, replace=False)
    for i in idx:
        h = 1e-6 * max(1.0, abs(p[i]))
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        fd = (R.loss_and_grad(pp, X, T, d, k)[0] - R.loss_and_grad(pm, X, T, d, k)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, np.abs(g).max())


def test_loss_invariances_and_range():
    X, T, d, p = _problem()
    k = T.shape[1]
    Y = R.forward(p, X, k)
    L, _ = R.subspace_loss(Y, T, d)
    assert 0.0 <= L <= k
    rng = np.random.default_rng(2)
    Q = rng.standard_normal((k, k))                 # any invertible mixing of the columns
    L2, _ = R.subspace_loss(Y @ Q, T, d)
    L3, _ = R.subspace_loss(Y, T @ Q, d)
    assert abs(L2 - L) <= 1e-9 and abs(L3 - L) <= 1e-9
    # the same subspace gives zero loss; a D-orthogonal one gives k
    L0, g0 = R.subspace_loss(T @ Q, T, d)
    assert abs(L0) <= 1e-10 and np.abs(g0).max() <= 1e-8
    D = np.diag(d)
    Tp = rng.standard_normal((X.shape[0], k))
    Tp -= T @ np.linalg.solve(T.T @ D @ T, T.T @ D @ Tp)
    Lk, _ = R.subspace_loss(Tp, T, d)
    assert abs(Lk - k) <= 1e-9


def test_gelu_is_the_exact_erf_form():
    from scipy.stats import norm
    z = np.linspace(-6, 6, 101)
    assert np.allclose(R.gelu(z), z * norm.cdf(z), rtol=0, atol=1e-15)
    h = 1e-6
    assert np.allclose(R.gelu_grad(z), (R.gelu(z + h) - R.gelu(z - h)) / (2 * h), atol=1e-8)


def test_adam_moves_against_the_gradient_and_lowers_the_loss():
    X, T, d, p = _problem(n=400, k=4, seed=3)
    k = 4
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    L0, _ = R.loss_and_grad(p, X, T, d, k)
    for t in range(1, 61):
        L, g = R.loss_and_grad(p, X, T, d, k)
        p, m, v = R.adam_step(p, g, m, v, t, lr=3e-3)
    assert L < L0
