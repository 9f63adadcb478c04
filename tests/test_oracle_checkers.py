"""Pins of the oracle's checkers, CPU only: the CSR product and norm, the residual,
the principal angles between subspaces, the cluster-safe mode count and the
Chebyshev-Jacobi preconditioner used by the oracle's large solves.

Every GPU parity test of a product or an eigenpair is judged through these
functions, so each is fixed here against something other than itself: scipy's
sparse product, values worked out by hand on hand-built inputs, subspaces
built with prescribed principal angles, and the Chebyshev polynomial's closed
form.
"""
import numpy as np
import pytest
import scipy.sparse as sp


def _random_csr(n, seed, empty_rows=(3, 17, 18), long_rows=(5, 40), long_len=None):
    rng = np.random.default_rng(seed)
    rows = []
    for r in range(n):
        if r in empty_rows:
            cols = np.array([], dtype=np.int64)
        elif r in long_rows:
            cols = np.sort(rng.choice(n, size=long_len or n - 7, replace=False))
        else:
            cols = np.sort(rng.choice(n, size=int(rng.integers(1, 9)), replace=False))
        rows.append(cols)
    indptr = np.concatenate([[0], np.cumsum([len(c) for c in rows])]).astype(np.int64)
    indices = np.concatenate(rows).astype(np.int32)
    data = rng.standard_normal(indices.size) * np.exp(rng.uniform(-3, 3, indices.size))
    return indptr, indices, data


@pytest.mark.parametrize("m", [1, 3, 8])
def test_spmm_matches_scipy(oracle, m):
    n = 300
    rp, col, val = _random_csr(n, seed=m)
    A = sp.csr_matrix((val, col, rp), shape=(n, n))
    X = np.random.default_rng(9).standard_normal((n, m))
    Y = oracle.spmm(rp, col, val, X)
    ref = A @ X
    # same terms in the same (storage) order: equal up to the last bit, within a hair for safety
    assert np.abs(Y - ref).max() <= 1e-14 * np.abs(A).dot(np.abs(X)).max()
    # empty rows give zero rows
    assert np.all(Y[[3, 17, 18]] == 0.0)
    # the vector form and the scipy-operand wrapper agree
    assert np.array_equal(oracle.spmm(rp, col, val, X[:, 0]), Y[:, 0])
    assert np.array_equal(oracle.matmul(A, X), Y)


def test_spmm_rectangular(oracle):
    """A q x n matrix (the lists of q integration points over n nodes) times an n x m block."""
    rng = np.random.default_rng(2)
    q, n, m = 50, 20, 3
    rows = [np.sort(rng.choice(n, size=int(rng.integers(0, 6)), replace=False)) for _ in range(q)]
    rp = np.concatenate([[0], np.cumsum([len(r) for r in rows])]).astype(np.int64)
    col = np.concatenate(rows).astype(np.int32)
    val = rng.standard_normal(col.size)
    X = rng.standard_normal((n, m))
    Y = oracle.spmm(rp, col, val, X)
    assert Y.shape == (q, m)
    assert np.abs(Y - sp.csr_matrix((val, col, rp), shape=(q, n)) @ X).max() <= 1e-14
    with pytest.raises(ValueError):
        oracle.spmm(rp, col, val, X[:5])


def test_norm_inf_matches_definition(oracle):
    n = 250
    rp, col, val = _random_csr(n, seed=4, long_rows=(77,))
    A = sp.csr_matrix((val, col, rp), shape=(n, n))
    ref = float(np.abs(A).sum(axis=1).max())
    assert abs(oracle.norm_inf(rp, val) - ref) <= 1e-14 * ref
    # the maximum sits on the long row here; an all-empty matrix has norm 0
    assert int(np.argmax(np.asarray(np.abs(A).sum(axis=1)).ravel())) == 77
    z = np.zeros(n + 1, dtype=np.int64)
    assert oracle.norm_inf(z, np.zeros(1)) == 0.0


def test_residual_hand_computed(oracle):
    """Diagonal pencil, eigenvector e0 perturbed by eps e1: r = eps |h1 - lam m1| / ((|H| + lam |M|) |w|)."""
    h = np.array([2.0, 7.0, 11.0, 5.0])
    mm = np.array([0.5, 2.0, 1.0, 4.0])
    H = sp.csr_matrix(np.diag(h))
    M = sp.csr_matrix(np.diag(mm))
    lam0 = h[0] / mm[0]                                  # 4
    eps = 1e-3
    W = np.zeros((4, 2))
    W[0, 0], W[1, 0] = 1.0, eps                          # perturbed first pair
    W[3, 1] = 3.0                                        # exact pair (5 / 4), scaled
    lam = np.array([lam0, h[3] / mm[3]])
    r = oracle.residuals(H, M, lam, W)
    normH, normM = 11.0, 4.0
    ref0 = eps * abs(h[1] - lam0 * mm[1]) / ((normH + lam0 * normM) * np.sqrt(1.0 + eps * eps))
    assert abs(r[0] - ref0) <= 1e-15 * ref0
    assert r[1] == 0.0
    # explicit norms are used as given
    r2 = oracle.residuals(H, M, lam, W, normH=1.0, normM=0.0)
    assert abs(r2[0] - eps * abs(h[1] - lam0 * mm[1]) / np.sqrt(1 + eps * eps)) <= 1e-15
    # a non-diagonal pencil: 2x2 by hand
    H2 = sp.csr_matrix(np.array([[2.0, -1.0], [-1.0, 2.0]]))
    M2 = sp.csr_matrix(np.eye(2))
    w = np.array([[1.0], [0.0]])
    rr = oracle.residuals(H2, M2, np.array([2.0]), w)
    # H w - 2 w = (0, -1); |H|_inf = 3, |M|_inf = 1
    assert abs(rr[0] - 1.0 / (3.0 + 2.0)) <= 1e-16


def _m_orthonormal_basis(n, seed):
    """A dense SPD M (not the identity) and a basis U with U^T M U = I."""
    rng = np.random.default_rng(seed)
    B = rng.standard_normal((n, n))
    Md = B @ B.T / n + np.diag(rng.uniform(0.5, 3.0, n))
    L = np.linalg.cholesky(Md)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    U = np.linalg.solve(L.T, Q)                          # U^T M U = Q^T L^-1 L L^T L^-T Q = I
    return sp.csr_matrix(Md), U


@pytest.mark.parametrize("angles", [(0.5, 1e-3, 1e-8), (1e-8,), (1e-3,), (0.5,), (np.pi / 2, 0.25)])
def test_subspace_sines_prescribed_angles(oracle, angles):
    n = 40
    M, U = _m_orthonormal_basis(n, seed=len(angles))
    p = len(angles)
    Wa = U[:, :p].copy()
    Wb = np.stack([np.cos(a) * U[:, j] + np.sin(a) * U[:, p + j] for j, a in enumerate(angles)], axis=1)
    # mixing the columns of either block does not change the subspaces
    rng = np.random.default_rng(11)
    Wa = Wa @ (np.eye(p) + 0.3 * rng.standard_normal((p, p)))
    Wb = Wb @ (np.eye(p) + 0.3 * rng.standard_normal((p, p)))
    s = oracle.subspace_sines(Wa, Wb, M)
    ref = np.sort(np.sin(np.array(angles)))[::-1]
    assert s.shape == (p,)
    big = ref.max()
    for got, want in zip(s, ref):
        # the sines come from the eigenvalues of a Gram matrix of the complement: absolute
        # accuracy ~ 1e-16 relative to the largest sine squared, hence the floor below
        assert abs(got - want) <= 1e-9 * want + 2e-8 * big, (got, want)
    # identical subspaces: all sines zero
    assert oracle.subspace_sines(Wa, Wa @ np.diag(np.arange(1.0, p + 1)), M).max() <= 1e-7


def test_subspace_sines_uses_the_M_inner_product(oracle):
    """Two vectors orthogonal in the Euclidean sense but not in M give a sine below 1."""
    Md = np.array([[2.0, 1.0], [1.0, 2.0]])
    M = sp.csr_matrix(Md)
    a = np.array([[1.0], [0.0]])
    b = np.array([[0.0], [1.0]])
    s = oracle.subspace_sines(a, b, M)
    cos = (a[:, 0] @ Md @ b[:, 0]) / np.sqrt((a[:, 0] @ Md @ a[:, 0]) * (b[:, 0] @ Md @ b[:, 0]))
    assert abs(s[0] - np.sqrt(1 - cos * cos)) <= 1e-15


def test_cluster_safe_k_hand_built_spectra(oracle):
    lam = np.array([0.0, 1.0, 1.0000001, 2.0, 3.0, 3.0005, 4.0])
    # relative gaps to the next value: 1, 1e-7, 0.5, 0.333, 1.7e-4, 0.25
    assert oracle.cluster_safe_k(lam, 3) == 3          # gap after lam[2] is wide
    assert oracle.cluster_safe_k(lam, 2) == 1          # k = 2 splits the cluster {1, 1.0000001}
    assert oracle.cluster_safe_k(lam, 5) == 4          # k = 5 splits {3, 3.0005}
    assert oracle.cluster_safe_k(lam, 6) == 6
    assert oracle.cluster_safe_k(lam, 7) == 6          # the value after the last is unknown
    assert oracle.cluster_safe_k(lam, 1) == 1
    assert oracle.cluster_safe_k(np.array([1.0, 1.0, 1.0]), 2) == 0
    # the threshold is relative to the larger value and inclusive
    assert oracle.cluster_safe_k(np.array([0.0, 1.0, 1.001]), 2) == 1
    assert oracle.cluster_safe_k(np.array([0.0, 1.0, 1.002]), 2) == 2
    assert oracle.cluster_safe_k(np.array([0.0, 1.0, 1.0015]), 2, rel_gap=1e-3) == 2


def test_chebyshev_preconditioner_is_the_chebyshev_polynomial(oracle):
    """T = p(D^-1 H) D^-1 with the closed form p(t) = (1 - T_d((theta - t) / delta) /
    T_d(theta / delta)) / t of the Chebyshev semi-iteration on [a, b], built here from the
    eigendecomposition of D^-1/2 H D^-1/2; p > 0 on (0, b] and T is symmetric."""
    rng = np.random.default_rng(3)
    n = 30
    B = sp.random(n, n, density=0.2, random_state=4, format="csr")
    L = sp.csgraph.laplacian(abs(B + B.T)).tocsr()
    H = (L + sp.diags(rng.uniform(0.01, 0.1, n))).tocsr()
    d = H.diagonal()
    S = (H.toarray() / np.sqrt(d)[:, None]) / np.sqrt(d)[None, :]
    lam, V = np.linalg.eigh(S)
    upper, ratio, deg = 1.01 * lam.max(), 40.0, 6
    T = oracle.chebyshev_jacobi(H, degree=deg, ratio=ratio, upper=upper)
    lo = upper / ratio
    theta, delta = 0.5 * (upper + lo), 0.5 * (upper - lo)

    def cheb(x):
        if abs(x) <= 1:
            return np.cos(deg * np.arccos(x))
        return np.sign(x) ** deg * np.cosh(deg * np.arccosh(abs(x)))
    p = np.array([(1 - cheb((theta - t) / delta) / cheb(theta / delta)) / t for t in lam])
    assert np.all(p > 0)
    Dm = 1.0 / np.sqrt(d)
    Tref = (Dm[:, None] * (V * p[None, :]) @ V.T) * Dm[None, :]
    R = rng.standard_normal((n, 4))
    Z = T(R)
    assert np.abs(Z - Tref @ R).max() <= 1e-10 * np.abs(Tref @ R).max()
    Tm = T(np.eye(n))
    assert np.abs(Tm - Tm.T).max() <= 1e-10 * np.abs(Tm).max()
    # the default upper bound comes from ARPACK and covers the spectrum
    Td = oracle.chebyshev_jacobi(H)
    assert lam.max() <= Td.upper <= 1.06 * lam.max()


def test_lobpcg_with_chebyshev_matches_dense(oracle):
    from paper_2605_29318_amd import synth
    c = synth.random_cloud(1200, seed=21, hetero=True)
    P = oracle.pipeline(c)
    H, M = P.Hs(), P.Ms()
    k = 8
    wd, Vd = oracle.dense_eigh(H, M, k + 2)
    X0 = synth.initial_block(c.n, k + 4, seed=2)
    wl, Vl, it, res = oracle.lobpcg(H, M, X0, k=k, tol=1e-10, precond="chebyshev", maxiter=2000)
    assert res.max() <= 1e-10
    assert np.abs(wl[1:] - wd[1:k]).max() / wd[1:k].min() <= 1e-8
    kk = oracle.cluster_safe_k(wd, k)
    assert oracle.subspace_sines(Vd[:, :kk], Vl[:, :kk], M).max() <= 1e-6
