"""Pins of the oracle's generalized eigensolve (Eq. (15)), CPU only.

Dense LAPACK is the plain definition on small inputs; the oracle's FP64
LOBPCG must agree with it. The homogeneous cube approaches the Neumann
Laplacian spectrum pi^2 * {0, 1, 1, 1, 2, 2, 2, 3, ...} scaled by lam + 4 mu
(Eq. (17)), the constant mode has eigenvalue 0 (Supp. B.1), and the spectrum
is invariant to input order, translation and quadrature-weight scaling.
"""
import numpy as np
import pytest

from paper_2605_29318_amd import synth


def test_constant_mode_and_orthonormality(oracle):
    c = synth.cube_lattice()
    P = oracle.pipeline(c)
    H, M = P.Hs(), P.Ms()
    w, V = oracle.dense_eigh(H, M, 10)
    assert abs(w[0]) <= 1e-10 * w[1]
    const = np.ones(c.n) / np.sqrt(np.ones(c.n) @ (M @ np.ones(c.n)))
    assert abs(abs(V[:, 0] @ (M @ const)) - 1.0) <= 1e-8
    G = V.T @ (M @ V)
    assert np.abs(G - np.eye(10)).max() <= 1e-10
    r = oracle.residuals(H, M, w, V)
    assert r.max() <= 1e-12


def test_neumann_laplacian_limit():
    """lam_2 / (lam + 4 mu) tends to pi^2 under refinement of the unjittered cube."""
    from oracle import oracle as O
    errs = []
    for m in (8, 12, 16):
        c = synth.cube_lattice(m=m, spacing=1.0 / m, jitter=0.0)
        P = O.pipeline(c)
        w, _ = O.dense_eigh(P.Hs(), P.Ms(), 5)
        s = c.lam[0] + 4 * c.mu[0]
        ratio = w[1:4] / s
        # the first cluster is threefold degenerate on the symmetric cube
        assert np.ptp(ratio) <= 1e-8 * ratio.mean()
        errs.append(abs(ratio.mean() - np.pi ** 2) / np.pi ** 2)
    assert errs[-1] < errs[0]
    assert errs[-1] < 0.05


def test_lobpcg_matches_dense(oracle):
    c = synth.random_cloud(1500, seed=12, hetero=True)
    P = oracle.pipeline(c)
    H, M = P.Hs(), P.Ms()
    k = 8
    wd, Vd = oracle.dense_eigh(H, M, k + 4)
    X0 = synth.initial_block(c.n, k + 2, seed=1)
    wl, Vl, it, res = oracle.lobpcg(H, M, X0, k=k, tol=1e-10, precond="jacobi", maxiter=4000)
    assert res.max() <= 1e-10
    assert np.abs(wl[1:] - wd[1:k]).max() / wd[1:k].min() <= 1e-8
    assert abs(wl[0]) <= 1e-8 * wd[1]
    kk = oracle.cluster_safe_k(wd, k)
    s = oracle.subspace_sines(Vd[:, :kk], Vl[:, :kk], M)
    assert s.max() <= 1e-6


def test_invariances(oracle):
    c = synth.random_cloud(800, seed=19)
    P = oracle.pipeline(c)
    w0, _ = oracle.dense_eigh(P.Hs(), P.Ms(), 8)
    # input order
    rng = np.random.default_rng(5)
    p = rng.permutation(c.n)
    c2 = synth.Cloud("perm", c.xyz[p].copy(), c.vol[p], c.lam[p], c.mu[p], c.rho[p], c.h, c.k, 0)
    w1, _ = oracle.dense_eigh(oracle.pipeline(c2).Hs(), oracle.pipeline(c2).Ms(), 8)
    assert np.abs(w1[1:] - w0[1:]).max() <= 1e-9 * w0[1:].max()
    # translation
    c3 = synth.Cloud("shift", c.xyz + np.array([3.25, -1.5, 0.75]), c.vol, c.lam, c.mu, c.rho,
                     c.h, c.k, 0)
    w3, _ = oracle.dense_eigh(oracle.pipeline(c3).Hs(), oracle.pipeline(c3).Ms(), 8)
    assert np.abs(w3[1:] - w0[1:]).max() <= 1e-7 * w0[1:].max()
    # quadrature-weight scaling leaves the eigenvalues unchanged
    c4 = synth.Cloud("vscale", c.xyz, c.vol * 7.0, c.lam, c.mu, c.rho, c.h, c.k, 0)
    P4 = oracle.pipeline(c4)
    w4, _ = oracle.dense_eigh(P4.Hs(), P4.Ms(), 8)
    assert np.abs(w4[1:] - w0[1:]).max() <= 1e-9 * w0[1:].max()


def test_disconnected_cloud_has_two_zero_modes(oracle):
    a = synth.random_cloud(400, seed=2)
    b = synth.random_cloud(400, seed=3)
    xyz = np.concatenate([a.xyz, b.xyz + np.array([2.0, 0, 0])])
    c = synth.Cloud("two", xyz, np.concatenate([a.vol, b.vol]), np.concatenate([a.lam, b.lam]),
                    np.concatenate([a.mu, b.mu]), np.concatenate([a.rho, b.rho]), a.h, 4, 0)
    P = oracle.pipeline(c)
    w, _ = oracle.dense_eigh(P.Hs(), P.Ms(), 4)
    assert abs(w[0]) <= 1e-10 * w[2] and abs(w[1]) <= 1e-10 * w[2]
