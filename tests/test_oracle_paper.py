"""Pins of the oracle's version of the paper's own construction (Supp. B.1, "RKPM
construction"), CPU only: farthest point sampling of the centres among grid
integration points, each centre's Gaussian radius (the distance reaching two other
centres), neighbour lists with a radius per centre, the cut Gaussian, and the three
bases of Sec. 3.2 / Fig. 3b (plain RBF, partition-of-unity RBF, RKPM).

Pins: FPS sequences worked out by hand, the separation property every FPS sequence
has, radii by hand, brute-force neighbour search, the cut kernel's closed-form
value at the centre and its quadratic vanishing at the cut, reproducing
conditions to 1e-12, central finite differences, and the continuum limit of the
first non-zero mode of a box (the Neumann Laplacian's (pi / L)^2, cos(pi x / L)).
"""
import numpy as np
import pytest

from paper_2605_29318_amd import synth


def test_fps_by_hand(oracle):
    line = np.stack([np.arange(11.0), np.zeros(11), np.zeros(11)], axis=1)
    # 0, then 10 (farthest), 5 (middle), then four points at distance 2 tie: the lowest, 2; then 7
    # (distance 2 from {5, 10}), then the six points at distance 1 tie: 1
    assert oracle.fps(line, 6).tolist() == [0, 10, 5, 2, 7, 1]
    cube = np.array([[x, y, z] for z in (0.0, 1.0) for y in (0.0, 1.0) for x in (0.0, 1.0)] + [[0.5, 0.5, 0.5]])
    # from corner 0 the opposite corner 7 (d^2 = 3); then every corner is at distance 1 from the
    # picked set and the centre at sqrt(0.75): the corners in index order, the centre last
    assert oracle.fps(cube, 9).tolist() == [0, 7, 1, 2, 3, 4, 5, 6, 8]
    assert oracle.fps(cube, 9, start=8).tolist()[:2] == [8, 0]     # all corners tie from the centre
    assert oracle.fps(cube, 1, start=3).tolist() == [3]
    with pytest.raises(ValueError):
        oracle.fps(cube, 10)


def test_fps_separation_property(oracle):
    """Each pick is at least the current covering radius from every earlier pick, and the
    covering radius never grows: checked by brute force on random points."""
    rng = np.random.default_rng(4)
    p = rng.uniform(size=(600, 3))
    K = 60
    idx = oracle.fps(p, K)
    assert len(set(idx.tolist())) == K
    D = np.sqrt(((p[:, None, :] - p[None, :, :]) ** 2).sum(-1))
    cover = [D[:, idx[:t]].min(axis=1).max() for t in range(1, K + 1)]
    assert np.all(np.diff(cover) <= 0)
    for t in range(1, K):
        # the t-th pick realises the covering radius of the first t picks
        assert abs(D[idx[t], idx[:t]].min() - cover[t - 1]) <= 1e-15
        assert D[np.ix_(idx[:t + 1], idx[:t + 1])][np.triu_indices(t + 1, 1)].min() >= cover[t] - 1e-15


def test_radii_by_hand(oracle):
    c = np.array([[0.0, 0, 0], [1.0, 0, 0], [3.0, 0, 0], [6.0, 0, 0]])
    r, R = oracle.radii(c, cut=2.5)
    # second-nearest distances: 0 -> {1, 3, 6}: 3; 1 -> {1, 2, 5}: 2; 3 -> {3, 2, 3}: 3; 6 -> {6, 5, 3}: 5
    assert r.tolist() == [3.0, 2.0, 3.0, 5.0]
    assert R.tolist() == [7.5, 5.0, 7.5, 12.5]
    with pytest.raises(ValueError):
        oracle.radii(c[:2])


def test_neighbors_var_match_brute_force(oracle):
    rng = np.random.default_rng(9)
    cen = rng.uniform(size=(300, 3))
    R = rng.uniform(0.05, 0.2, size=300)
    h = float(R.max())
    perm, cs, origin, dims = oracle.bin_nodes(cen, h)
    xs, Rs = np.ascontiguousarray(cen[perm]), R[perm]
    q = rng.uniform(-0.1, 1.1, size=(700, 3))
    off, ids = oracle.neighbors_var(q, xs, Rs, h, origin, dims, cs)
    offb, idsb = oracle.neighbors_var_brute(q, xs, Rs)
    assert np.array_equal(off, offb) and np.array_equal(ids, idsb)
    assert off[-1] > 0


def test_cut_gaussian_shape(oracle):
    """Plain-RBF basis returns the raw kernel: 1 - e^-c^2 (1 + c^2) at the centre, and near the
    cut s -> c^2 it vanishes quadratically, w ~ e^-c^2 (c^2 - s)^2 / 2."""
    cut, r = 3.0, 0.2
    xs = np.array([[0.0, 0.0, 0.0]])
    rs = np.array([r])
    for d in (0.0, 0.5 * r, (1 - 1e-4) * cut * r):
        q = np.array([[d, 0.0, 0.0]])
        off = np.array([0, 1], dtype=np.int64)
        ids = np.array([0], dtype=np.int32)
        phi, dphi = oracle.rkpm_var(q, xs, rs, off, ids, 1.0, cut, oracle.BASIS_RBF)
        s = d * d / (r * r)
        if d == 0.0:
            assert abs(phi[0] - (1 - np.exp(-9.0) * 10.0)) <= 1e-15
            assert np.all(dphi == 0.0)
        elif d < r:
            assert abs(phi[0] - (np.exp(-s) - np.exp(-9.0) * (10.0 - s))) <= 1e-15
        else:
            delta = cut * cut - s
            assert abs(phi[0] - np.exp(-9.0) * delta * delta / 2) <= 1e-3 * np.exp(-9.0) * delta * delta
            assert abs(dphi[0, 0]) <= 2 * np.exp(-9.0) * delta * 2 * d / (r * r)


def _beam(oracle, basis, K=220, spacing=0.1, length=3.0):
    S = synth.beam(spacing=spacing, K=K, length=length)
    P = oracle.paper_pipeline(S.xyz, S.vol, S.lam, S.mu, S.K, basis=basis)
    return S, P


@pytest.mark.parametrize("basis", [0, 1, 2])
def test_paper_bases_reproduction_and_gradient(oracle, basis):
    S, P = _beam(oracle, basis)
    q = S.q
    rows = np.repeat(np.arange(q), np.diff(P.nbr_off))
    s0 = np.bincount(rows, weights=P.phi, minlength=q)
    g0 = np.stack([np.bincount(rows, weights=P.dphi[:, a], minlength=q) for a in range(3)], 1)
    if basis >= 1:                       # partition of unity (PU-RBF and RKPM)
        assert np.abs(s0 - 1).max() <= 1e-12 and np.abs(g0).max() * P.h <= 1e-12
    else:
        assert np.abs(s0 - 1).max() > 1e-3                           # plain RBF does not reproduce
    p = P.xyz[P.nbr_id]
    for a in range(3):
        lin = np.bincount(rows, weights=P.phi * p[:, a], minlength=q)
        err = np.abs(lin - S.xyz[:, a]).max() / P.h
        if basis == 2:
            assert err <= 1e-12
            for s in range(3):
                gl = np.bincount(rows, weights=P.dphi[:, s] * p[:, a], minlength=q)
                assert np.abs(gl - (1.0 if a == s else 0.0)).max() <= 1e-12
        else:
            assert err > 1e-6                                          # only RKPM reproduces x
    # central finite differences of phi at a sample of points, same lists
    sel = np.arange(0, q, 97)
    d = 1e-6 * P.h
    sub_off = np.concatenate([[0], np.cumsum(np.diff(P.nbr_off)[sel])])
    sub_ids = np.concatenate([P.nbr_id[P.nbr_off[i]:P.nbr_off[i + 1]] for i in sel]).astype(np.int32)
    ref = np.concatenate([P.dphi[P.nbr_off[i]:P.nbr_off[i + 1]] for i in sel])
    for s in range(3):
        e = np.zeros(3)
        e[s] = d
        pp, _ = oracle.rkpm_var(S.xyz[sel] + e, P.xyz, P.r, sub_off, sub_ids, P.h, 3.0, basis)
        pm, _ = oracle.rkpm_var(S.xyz[sel] - e, P.xyz, P.r, sub_off, sub_ids, P.h, 3.0, basis)
        assert np.abs((pp - pm) / (2 * d) - ref[:, s]).max() <= 1e-6 * np.abs(ref).max()


def test_paper_assembly_properties_and_conditioning(oracle):
    """H bitwise symmetric with the constant field in its null space; M far better conditioned
    with many integration points per centre than with one quadrature point per node (the
    regime the rest of the path runs in)."""
    S, P = _beam(oracle, 2)
    H, M = P.Hs(), P.Ms()
    assert (H != H.T).nnz == 0 and (M != M.T).nnz == 0
    ones = np.ones(P.K)
    assert np.abs(H @ ones).max() <= 1e-12 * np.abs(H).sum(axis=1).max()
    cond_many = np.linalg.cond(M.toarray())
    # one quadrature point per node, as in the particle workloads
    c = synth.random_cloud(P.K, seed=3)
    Pk = oracle.pipeline(c)
    cond_one = np.linalg.cond(Pk.Ms().toarray())
    assert cond_many < 1e4 and cond_one > 100 * cond_many, (cond_many, cond_one)


def test_first_mode_of_a_box_by_basis(oracle):
    """The first non-zero mode of a 3 x 1 x 1 box tends to the Neumann Laplacian's, eigenvalue
    (pi / 3)^2 (times lambda + 4 mu) and shape cos(pi x / 3). RKPM is closest in both, the
    plain RBF farthest (the paper's Fig. 3b shows RBF and partition-of-unity RBF modes as
    irregular and RKPM's as the expected field)."""
    import scipy.linalg as sl
    out = {}
    for basis in (0, 1, 2):
        S, P = _beam(oracle, basis)
        w, V = sl.eigh(P.Hs().toarray(), P.Ms().toarray(), subset_by_index=[0, 3])
        s = S.lam[0] + 4 * S.mu[0]
        lam2 = w[1] / s
        # the mode at the integration points, against the best a cos(pi x / 3) + b
        rows = np.repeat(np.arange(S.q), np.diff(P.nbr_off))
        u = np.bincount(rows, weights=P.phi * V[P.nbr_id, 1], minlength=S.q)
        A = np.stack([np.cos(np.pi * S.xyz[:, 0] / 3.0), np.ones(S.q)], 1)
        coef = np.linalg.lstsq(A, u, rcond=None)[0]
        shape_err = np.linalg.norm(u - A @ coef) / np.linalg.norm(u - u.mean())
        out[basis] = (abs(lam2 - (np.pi / 3) ** 2) / (np.pi / 3) ** 2, shape_err)
    assert out[2][0] < out[1][0] < out[0][0], out
    assert out[2][1] < out[0][1], out
    assert out[2][0] < 2e-3 and out[2][1] < 1e-2, out
