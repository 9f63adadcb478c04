"""Pins of the oracle's Hessian (Prop. 1) and mass matrix (Eq. (14)), CPU only.

The key pin differentiates the quadrature of the Neo-Hookean energy of
Eq. (16) numerically (Supp. C, Eq. (S5)): the sum of its xx, yy and zz blocks
at d = 0 must equal the assembled H. The remaining pins are structural
(bitwise symmetry, constant null vector, PSD), exact energies of linear
fields, a dense re-assembly from the shape-function matrices, and material
scaling.
"""
import numpy as np
import pytest

from paper_2605_29318_amd import synth


def _problem(oracle, c, rho=False):
    return oracle.pipeline(c, use_rho=rho)


def _dense_shape_matrices(P, n):
    q = len(P.nbr_off) - 1
    rows = np.repeat(np.arange(q), np.diff(P.nbr_off))
    Phi = np.zeros((q, n))
    G = np.zeros((3, q, n))
    Phi[rows, P.nbr_id] = P.phi
    for s in range(3):
        G[s, rows, P.nbr_id] = P.dphi[:, s]
    return Phi, G


def _neo_hookean_energy(F, lam, mu):
    """Psi(F) = 1/2 [ lb (det F - g)^2 + mb tr(F^T F) - E0 ], lb = lam + mu, mb = mu,
    g = 1 + mb/lb, E0 chosen so that Psi(I) = 0 (Eq. (16))."""
    lb = lam + mu
    mb = mu
    g = 1.0 + mb / lb
    J = np.linalg.det(F)
    E0 = lb * (1.0 - g) ** 2 + 3.0 * mb
    return 0.5 * (lb * (J - g) ** 2 + mb * np.einsum("...ij,...ij->...", F, F) - E0)


def test_prop1_by_finite_differences(oracle):
    c = synth.random_cloud(40, seed=3, hetero=True, support_factor=3.2)
    P = _problem(oracle, c)
    n = c.n
    Phi, G = _dense_shape_matrices(P, n)
    gradphi = np.transpose(G, (1, 2, 0))          # (q, n, 3): grad phi_k at X_i

    def energy(d):                                 # d: (n, 3) nodal displacements
        F = np.eye(3)[None] + np.einsum("kr,iks->irs", d, gradphi)   # F = I + d^T grad phi
        return np.sum(P.vol * _neo_hookean_energy(F, P.lam, P.mu))

    delta = 1e-4
    Hw = np.zeros((n, n))
    for axis in range(3):                          # H_xx + H_yy + H_zz
        for a in range(n):
            for b in range(a, n):
                def e(sa, sb):
                    d = np.zeros((n, 3))
                    d[a, axis] += sa * delta
                    d[b, axis] += sb * delta
                    return energy(d)
                v = (e(1, 1) - e(1, -1) - e(-1, 1) + e(-1, -1)) / (4 * delta * delta)
                Hw[a, b] += v
                if a != b:
                    Hw[b, a] += v
    H = P.Hs().toarray()
    scale = np.abs(H).max()
    assert np.abs(Hw - H).max() <= 1e-5 * scale


def test_symmetry_nullspace_and_definiteness(oracle):
    c = synth.cube_lattice()
    P = _problem(oracle, c)
    H, M = P.Hs(), P.Ms()
    assert (H != H.T).nnz == 0            # bitwise symmetric
    assert (M != M.T).nnz == 0
    rowabs = abs(H).sum(axis=1).max()
    assert np.abs(H @ np.ones(c.n)).max() <= 1e-12 * rowabs
    Hd, Md = H.toarray(), M.toarray()
    eh = np.linalg.eigvalsh(Hd)
    em = np.linalg.eigvalsh(Md)
    assert eh.min() >= -1e-12 * eh.max()
    assert em.min() > 0
    # cond(M) of the one-point-per-particle quadrature on this cube (recorded)
    assert em.max() / em.min() < 1e8


def test_linear_fields_exact(oracle):
    c = synth.random_cloud(1200, seed=7, hetero=True)
    P = _problem(oracle, c)
    H, M = P.Hs(), P.Ms()
    rng = np.random.default_rng(0)
    a = rng.normal()
    b = rng.normal(size=3)
    cvec = a + P.xyz @ b
    w = P.vol * (P.lam + 4 * P.mu)
    eH = cvec @ (H @ cvec)
    assert abs(eH - (b @ b) * w.sum()) <= 1e-10 * abs(eH)
    eM = cvec @ (M @ cvec)
    ref = np.sum(P.vol * (a + P.xyz @ b) ** 2)
    assert abs(eM - ref) <= 1e-12 * abs(ref)


def test_dense_reassembly(oracle):
    """H = sum_s G_s^T diag(v (lam + 4 mu)) G_s and M = Phi^T diag(v rho) Phi as dense products."""
    c = synth.random_cloud(700, seed=31, hetero=True)
    for rho in (False, True):
        P = _problem(oracle, c, rho=rho)
        Phi, G = _dense_shape_matrices(P, c.n)
        w = P.vol * (P.lam + 4 * P.mu)
        Hd = sum(G[s].T @ (w[:, None] * G[s]) for s in range(3))
        mw = P.vol * (P.rho if rho else 1.0)
        Md = Phi.T @ (mw[:, None] * Phi)
        H, M = P.Hs().toarray(), P.Ms().toarray()
        assert np.abs(H - Hd).max() <= 1e-12 * np.abs(Hd).max()
        assert np.abs(M - Md).max() <= 1e-12 * np.abs(Md).max()
        # the pattern is the structural union: every dense nonzero is stored
        assert np.all((Hd != 0) <= (P.Hs().toarray() != 0) | (np.abs(Hd) < 1e-300))


def test_material_scaling(oracle):
    """Homogeneous material: H / (lam + 4 mu) does not depend on E or nu (Eq. (17))."""
    c1 = synth.cube_lattice(E=1e5, nu=0.45)
    c2 = synth.cube_lattice(E=3e6, nu=0.3)
    P1, P2 = _problem(oracle, c1), _problem(oracle, c2)
    s1 = c1.lam[0] + 4 * c1.mu[0]
    s2 = c2.lam[0] + 4 * c2.mu[0]
    assert np.array_equal(P1.col, P2.col)
    assert np.abs(P1.H / s1 - P2.H / s2).max() <= 1e-12 * np.abs(P1.H / s1).max()
    assert np.array_equal(P1.M, P2.M)


def test_rows_sorted_and_pattern_radius(oracle):
    c = synth.random_cloud(900, seed=41)
    P = _problem(oracle, c)
    for r in range(0, c.n, 17):
        cols = P.col[P.row_ptr[r]:P.row_ptr[r + 1]]
        assert np.all(np.diff(cols) > 0)
        d = np.sqrt(np.sum((P.xyz[cols] - P.xyz[r]) ** 2, axis=1))
        assert d.max() < 2 * c.h
