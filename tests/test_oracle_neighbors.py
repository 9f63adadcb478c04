"""Pins of the oracle's cell binning and neighbour lists (CPU only).

Binning is checked against the definition of a cell (a box of edge h from the
origin), of its 4x4x4 sub-cells and of the (cell, sub-cell Morton code, original
index) order; the cell-list neighbour search is checked
against exhaustive search and against scipy's KD-tree.
"""
import numpy as np
import pytest

from paper_2605_29318_amd import synth


def _clouds():
    yield synth.cube_lattice()
    yield synth.cube_lattice(m=7, jitter=0.0, seed=3)
    yield synth.random_cloud(1500, seed=5)
    c = synth.random_cloud(800, seed=9)
    c.xyz[:, 2] *= 0.05           # flat slab: one cell layer in z
    yield c


@pytest.mark.parametrize("ci", range(4))
def test_binning_orders_by_cell_and_subcell(oracle, ci):
    c = list(_clouds())[ci]
    perm, cs, origin, dims = oracle.bin_nodes(c.xyz, c.h)
    n = c.n
    assert sorted(perm.tolist()) == list(range(n))
    assert cs[0] == 0 and cs[-1] == n and np.all(np.diff(cs) >= 0)
    assert np.allclose(origin, c.xyz.min(axis=0), rtol=0, atol=0)
    # every node of cell id lies in that cell's box (the last cell of an axis is closed)
    cid = np.repeat(np.arange(len(cs) - 1), np.diff(cs))
    cx = cid % dims[0]
    cy = (cid // dims[0]) % dims[1]
    cz = cid // (dims[0] * dims[1])
    cc = np.stack([cx, cy, cz], axis=1)
    x = c.xyz[perm]
    lo = origin + cc * c.h
    hi = origin + (cc + 1) * c.h
    eps = 1e-12
    assert np.all(x >= lo - eps)
    last = cc == (dims - 1)[None, :]
    assert np.all((x < hi + eps) | last)
    # the grid just covers the nodes
    assert np.all(origin + (dims - 1) * c.h <= c.xyz.max(axis=0) + eps)
    # inside a cell: ascending Morton code of the 4x4x4 sub-cell, ties by original index;
    # each node lies in its sub-cell's box (the last sub-cell of a clamped axis is closed)
    t = (c.xyz[perm] - origin) / c.h
    q = np.clip(np.floor(t), 0, dims - 1)
    sub = np.clip(np.floor((t - q) * 4.0), 0, 3).astype(np.int64)
    code = np.zeros(n, dtype=np.int64)
    for b in range(2):
        for a in range(3):
            code |= ((sub[:, a] >> b) & 1) << (3 * b + a)
    slo = lo + sub * (c.h / 4)
    assert np.all(x >= slo - eps)
    assert np.all((x < slo + c.h / 4 + eps) | (sub == 3))
    for a, b in zip(cs[:-1], cs[1:]):
        key = code[a:b] * (n + 1) + perm[a:b]
        assert np.all(np.diff(key) > 0)


@pytest.mark.parametrize("ci", range(4))
def test_cell_list_equals_brute_force(oracle, ci):
    c = list(_clouds())[ci]
    perm, cs, origin, dims = oracle.bin_nodes(c.xyz, c.h)
    xs = np.ascontiguousarray(c.xyz[perm])
    off, ids = oracle.neighbors(xs, xs, c.h, origin, dims, cs)
    boff, bids = oracle.neighbors_brute(xs, xs, c.h)
    assert np.array_equal(off, boff)
    assert np.array_equal(ids, bids)
    # self is always a neighbour and the relation is symmetric when Q = K
    n = c.n
    A = np.zeros((n, n), dtype=bool)
    rows = np.repeat(np.arange(n), np.diff(off))
    A[rows, ids] = True
    assert np.all(np.diag(A))
    assert np.array_equal(A, A.T)
    # ascending within each list
    for i in range(0, n, 37):
        seg = ids[off[i]:off[i + 1]]
        assert np.all(np.diff(seg) > 0)


def test_separate_quadrature_points_with_outside_points(oracle):
    c = synth.random_cloud(1200, seed=11)
    rng = np.random.default_rng(2)
    q = rng.uniform(-0.2, 1.2, size=(700, 3))      # some far outside the node box
    perm, cs, origin, dims = oracle.bin_nodes(c.xyz, c.h)
    xs = np.ascontiguousarray(c.xyz[perm])
    off, ids = oracle.neighbors(q, xs, c.h, origin, dims, cs)
    boff, bids = oracle.neighbors_brute(q, xs, c.h)
    assert np.array_equal(off, boff)
    assert np.array_equal(ids, bids)


def test_against_kdtree(oracle):
    from scipy.spatial import cKDTree
    c = synth.random_cloud(3000, seed=21)
    perm, cs, origin, dims = oracle.bin_nodes(c.xyz, c.h)
    xs = np.ascontiguousarray(c.xyz[perm])
    off, ids = oracle.neighbors(xs, xs, c.h, origin, dims, cs)
    tree = cKDTree(xs)
    lists = tree.query_ball_point(xs, r=c.h)
    for i in range(0, c.n, 7):
        ref = sorted(j for j in lists[i] if np.sum((xs[i] - xs[j]) ** 2) < c.h * c.h)
        assert ids[off[i]:off[i + 1]].tolist() == ref


def test_config1_neighbour_statistics(oracle):
    """The 1,000-particle cube: about 52 neighbours per point at h = 2.5 spacing."""
    c = synth.cube_lattice()
    perm, cs, origin, dims = oracle.bin_nodes(c.xyz, c.h)
    xs = np.ascontiguousarray(c.xyz[perm])
    off, ids = oracle.neighbors(xs, xs, c.h, origin, dims, cs)
    deg = np.diff(off)
    assert 45 < deg.mean() < 60
    assert deg.max() <= 81 + 10
