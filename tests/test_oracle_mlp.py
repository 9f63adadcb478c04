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


def _lattice(m=7, a=0.1, jitter=0.0, seed=0):
    g = np.arange(m) * a
    X = np.stack(np.meshgrid(g, g, g, indexing="ij"), axis=-1).reshape(-1, 3)
    if jitter:
        X = X + np.random.default_rng(seed).uniform(-jitter, jitter, X.shape)
    return X


def _features(oracle, X, h, kernel=0):
    off, ids = oracle.neighbors_brute(X, X, h)
    return R.rkpm_features(X, X, off, ids, h, kernel), off


@pytest.mark.parametrize("kernel", [0, 1])
def test_features_symmetric_lattice_interior(oracle, kernel):
    """At the centre of a cubic lattice the neighbourhood is symmetric: the first
    moments vanish (boundary indicator 0) and the normalised moment matrix is
    diag(1, s, s, s) with s < 1, so three eigenvalues coincide and the largest is 1."""
    X = _lattice()
    h = 0.25
    F, off = _features(oracle, X, h, kernel)
    c = int(np.argmin(((X - X.mean(axis=0)) ** 2).sum(axis=1)))
    f = F[c]
    assert abs(f[6]) <= 1e-14
    assert abs(f[3] - 1.0) <= 1e-14
    assert np.ptp(f[0:3]) <= 1e-14 and 0 < f[0] < 1
    assert f[4] == off[c + 1] - off[c]
    # 4/3 pi (h/a)^3 lattice points in the ball, up to the shell: a count check by enumeration
    g = np.arange(-3, 4)
    cnt = sum(1 for i in g for j in g for k in g if (i * i + j * j + k * k) * 0.01 < h * h)
    assert f[4] == cnt


def test_features_face_points_inward(oracle):
    """On the z = 0 face the kernel-weighted offset points into the body (+z)."""
    X = _lattice()
    h = 0.25
    off, ids = oracle.neighbors_brute(X, X, h)
    face = np.where((X[:, 2] == 0) & (np.abs(X[:, 0] - 0.3) < 1e-9) & (np.abs(X[:, 1] - 0.3) < 1e-9))[0][0]
    f = R.rkpm_features(X, X, off, ids, h)[face]
    nb = X[ids[off[face]:off[face + 1]]]
    w = R._raw_kernel(np.linalg.norm(nb - X[face], axis=1), h, 0)
    v = (w[:, None] * (nb - X[face])).sum(axis=0)
    assert abs(v[0]) <= 1e-14 and abs(v[1]) <= 1e-14 and v[2] > 0
    assert f[6] > 0.1


def test_features_rigid_motion_invariant(oracle):
    X = _lattice(m=6, jitter=0.02, seed=4)
    h = 0.25
    F, _ = _features(oracle, X, h)
    Q = np.linalg.qr(np.random.default_rng(5).standard_normal((3, 3)))[0]
    Y = X @ Q.T + np.array([3.0, -1.0, 0.5])
    G, _ = _features(oracle, Y, h)
    assert np.allclose(F, G, rtol=1e-10, atol=1e-12)


def test_features_flat_kernel_limit(oracle):
    """Gaussian with support far beyond the cloud: every phi~ is about 1, so the
    spread tends to 0, the sum to n, and the moment matrix to [[1, m^T], [m, C]]
    with C the second moments of (p - X)/h, all small next to 1."""
    X = _lattice(m=4, a=0.01, jitter=0.002, seed=1)
    h = 1000.0
    F, _ = _features(oracle, X, h, kernel=1)
    n = X.shape[0]
    assert np.all(F[:, 4] == n)
    assert np.allclose(F[:, 5], n, rtol=1e-7)
    assert np.all(F[:, 7] <= 1e-7)
    assert np.all(np.abs(F[:, 3] - 1.0) <= 1e-7) and np.all(np.abs(F[:, 0:3]) <= 1e-7)
    Xc = X - X.mean(axis=0)
    assert np.allclose(F[:, 6], np.linalg.norm(-Xc, axis=1) / h, rtol=1e-6)


def test_position_encoding_octaves():
    """Each octave doubles the angle of the previous one: sin 2t = 2 sin t cos t,
    cos 2t = cos^2 t - sin^2 t; the first octave is sin/cos(pi x) of the normalised
    position; the base 11 inputs are unchanged."""
    rng = np.random.default_rng(3)
    xyz = rng.uniform(-2, 5, size=(200, 3))
    feat = rng.uniform(0.1, 1.0, size=(200, 8))
    base = R.inputs(xyz, feat)
    enc = R.inputs(xyz, feat, n_freq=5)
    assert enc.shape == (200, 41)
    assert np.array_equal(enc[:, :11], base)
    x = base[:, 0:3]
    assert np.abs(x).max() == pytest.approx(1.0)
    assert np.allclose(enc[:, 11:14], np.sin(np.pi * x), atol=1e-15)
    for l in range(1, 5):
        s0, c0 = enc[:, 5 + 6 * l: 8 + 6 * l], enc[:, 8 + 6 * l: 11 + 6 * l]
        s1, c1 = enc[:, 11 + 6 * l: 14 + 6 * l], enc[:, 14 + 6 * l: 17 + 6 * l]
        assert np.allclose(s1, 2 * s0 * c0, atol=1e-12)
        assert np.allclose(c1, c0 * c0 - s0 * s0, atol=1e-12)


def test_gradient_with_encoded_inputs():
    rng = np.random.default_rng(4)
    n, k, n_in = 200, 5, 23
    X = rng.standard_normal((n, n_in))
    T = np.linalg.qr(rng.standard_normal((n, k)))[0]
    d = rng.uniform(0.5, 2.0, size=n)
    p = R.init_params(k, seed=1, n_in=n_in)
    assert p.size == R.param_count(k, n_in) and R.input_width(p, k) == n_in
    L, g = R.loss_and_grad(p, X, T, d, k)
    for i in rng.choice(128 * n_in, size=20, replace=False):     # first-layer weights
        h = 1e-6
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        fd = (R.loss_and_grad(pp, X, T, d, k)[0] - R.loss_and_grad(pm, X, T, d, k)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, np.abs(g).max())


def test_blend_closed_forms():
    """The blended block: blending a block with itself gives (1 + w) X / rms(X); with columns
    of X and R orthogonal, every output column has rms sqrt(1 + w^2); w = 0 leaves X's
    directions, each column at rms 1; scaling X or R by any positive factors per column
    changes nothing."""
    rng = np.random.default_rng(3)
    n, m = 400, 6
    X = rng.standard_normal((n, m)) * rng.uniform(0.1, 10.0, m)
    rmsX = np.sqrt((X * X).sum(axis=0) / n)
    assert np.allclose(R.blend(X, X, 2.5), 3.5 * X / rmsX, rtol=1e-14, atol=0)
    Q, _ = np.linalg.qr(rng.standard_normal((n, 2 * m)))
    Xo, Ro = Q[:, :m] * 7.0, Q[:, m:] * 0.01
    for w in (0.0, 1.0, 3.0):
        Y = R.blend(Xo, Ro, w)
        assert np.allclose(np.sqrt((Y * Y).sum(axis=0) / n), np.sqrt(1 + w * w), rtol=1e-12)
    Y0 = R.blend(X, Ro, 0.0)
    assert np.allclose(Y0 * rmsX, X, rtol=1e-13)
    s1, s2 = rng.uniform(0.5, 4.0, m), rng.uniform(0.5, 4.0, m)
    assert np.allclose(R.blend(X * s1, Ro * s2, 3.0), R.blend(X, Ro, 3.0), rtol=1e-13)
