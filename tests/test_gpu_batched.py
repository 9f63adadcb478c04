"""GPU tests of the batched eigensolver (many objects, one launch per stage), hipGraph
replay of the iteration, and the SpMM autotuner."""
import numpy as np
import pytest

from paper_2605_29318_amd import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ff():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2605_29318_amd import freeform
    return freeform


@pytest.fixture(scope="module")
def ctx(ff):
    c = ff.Context(0)
    yield c
    c.close()


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), device="cuda")


def _objects():
    # uneven sizes and materials; small enough for dense oracle eigensolves
    clouds = [synth.cube_lattice(k=16), synth.random_cloud(1800, seed=41, hetero=True, k=16),
              synth.cube_lattice(m=12, spacing=1 / 12, jitter=0.015, seed=7, E=7e5, nu=0.3, k=16),
              synth.random_cloud(700, seed=43, k=16), synth.sphere_union(n=2400, seed=5, mc_samples=200_000, k=16)]
    return clouds


@pytest.fixture(scope="module")
def batch(oracle, ctx, ff):
    clouds = _objects()
    parts = [ff.assemble_cloud(ctx, dev(c.xyz), dev(c.vol), dev(c.lam), dev(c.mu), c.h) for c in clouds]
    refs = []
    for c in clouds:
        P = oracle.pipeline(c)
        wd, Vd = oracle.dense_eigh(P.Hs(), P.Ms(), 20)
        refs.append((P, wd, Vd))
    return clouds, parts, refs


@pytest.mark.parametrize("precision,graph,precond", [(0, False, 1), (1, False, 1), (1, True, 1), (1, True, 2),
                                                     (0, False, 2)])
def test_batched_matches_oracle(batch, oracle, ctx, ff, precision, graph, precond):
    clouds, parts, refs = batch
    k = 16
    off, rp, col, H, M, hm = ff.concat_objects(parts)
    lam, W, res, infos, rc = ff.eigenmodes_batched(ctx, off, rp, col, H, M, hm, k=k, precision=precision,
                                                   tol=1e-8, max_iter=8000, use_graph=graph, precond=precond)
    assert rc == 0
    Wh = W.cpu().numpy()
    for o, (P, wd, Vd) in enumerate(refs):
        assert infos[o]["converged"] == 1
        assert infos[o]["graph"] == int(graph)
        assert np.abs(lam[o, 1:] - wd[1:k]).max() / wd[1:k].min() <= 1e-5
        Wo = Wh[off[o]:off[o + 1]]
        r = oracle.residuals(P.Hs(), P.Ms(), lam[o], Wo)
        assert r.max() <= 2e-8
        kk = oracle.cluster_safe_k(wd, k)
        if kk:
            assert oracle.subspace_sines(Vd[:, :kk], Wo[:, :kk], P.Ms()).max() <= 1e-3
    # objects converge at different iteration counts and are masked independently
    its = [i["iters_fp32"] + i["iters_fp64"] for i in infos]
    assert len(set(its)) > 1


@pytest.mark.parametrize("graph", [False, True])
def test_batched_matrix_core_chebyshev(batch, oracle, ctx, ff, graph):
    """k = 32: the Chebyshev steps run on the matrix cores (binary16 H and iterate), each
    object's columns scaled by their own maxima; objects finish at different iterations
    and are masked while the rest go on."""
    clouds, parts, refs = batch
    k = 32
    off, rp, col, H, M, hm = ff.concat_objects(parts)
    lam, W, res, infos, rc = ff.eigenmodes_batched(ctx, off, rp, col, H, M, hm, k=k, precision=1, tol=1e-8,
                                                   max_iter=8000, use_graph=graph, precond=2, precond_values=3)
    assert rc == 0
    Wh = W.cpu().numpy()
    for o, (P, wd, Vd) in enumerate(refs):
        assert infos[o]["converged"] == 1 and infos[o]["graph"] == int(graph)
        assert np.abs(lam[o, 1:20] - wd[1:20]).max() / wd[1:20].min() <= 1e-5
        Wo = Wh[off[o]:off[o + 1]]
        assert oracle.residuals(P.Hs(), P.Ms(), lam[o], Wo).max() <= 2e-8
        assert np.abs(Wo.T @ (P.Ms() @ Wo) - np.eye(k)).max() <= 1e-6
        assert np.all(np.diff(lam[o]) >= -1e-9 * abs(lam[o, -1]))


def test_batched_equals_single_object_solves(batch, ctx, ff):
    clouds, parts, refs = batch
    k = 16
    off, rp, col, H, M, hm = ff.concat_objects(parts)
    lam, W, res, infos, rc = ff.eigenmodes_batched(ctx, off, rp, col, H, M, hm, k=k, precision=0, tol=1e-9,
                                                   max_iter=8000)
    for o, a in enumerate(parts):
        l1, W1, r1, i1 = ff.eigenmodes(ctx, a.n, a.row_ptr, a.col, a.H, a.M, a.hm32, k=k, precision=0, tol=1e-9,
                                      max_iter=8000)
        assert np.abs(lam[o, 1:] - l1[1:]).max() / l1[1:].max() <= 1e-9


def test_graph_replay_is_deterministic(batch, ctx, ff):
    """Replaying the captured iteration gives bitwise the same results as launching it directly."""
    clouds, parts, refs = batch
    off, rp, col, H, M, hm = ff.concat_objects(parts)
    outs = []
    for graph in (False, True, True):
        lam, W, res, infos, rc = ff.eigenmodes_batched(ctx, off, rp, col, H, M, hm, k=16, precision=1, tol=1e-7,
                                                       max_iter=8000, use_graph=graph)
        outs.append((lam.copy(), W.cpu().numpy()))
    for lam, W in outs[1:]:
        assert np.array_equal(lam, outs[0][0])
        assert np.array_equal(W, outs[0][1])


def test_batched_rejects_too_small_object(ctx, ff):
    c = synth.random_cloud(400, seed=3)
    a = ff.assemble_cloud(ctx, dev(c.xyz), dev(c.vol), dev(c.lam), dev(c.mu), c.h)
    off, rp, col, H, M, hm = ff.concat_objects([a])
    with pytest.raises(ff.FFError) as ei:
        ff.eigenmodes_batched(ctx, np.array([0, 10, c.n]), rp, col, H, M, hm, k=16)
    assert ei.value.code == ff.FF_ERR_INVALID_ARG


def test_autotuner_picks_a_valid_variant_and_caches(tmp_path, ctx, ff):
    c = synth.random_cloud(20000, seed=9)
    a = ff.assemble_cloud(ctx, dev(c.xyz), dev(c.vol), dev(c.lam), dev(c.mu), c.h)
    path = str(tmp_path / "tune.json")
    v, ms = ff.spmm_autotune(ctx, a.n, a.row_ptr, a.col, a.H, a.M, a.hm32, 1, 32, path)
    assert 0 <= v < len(ff.spmm_variant_names()) and ms > 0
    import json
    data = json.load(open(path))
    assert len(data) == 1 and list(data.values())[0]["variant"] == v
    v2, ms2 = ff.spmm_autotune(ctx, a.n, a.row_ptr, a.col, a.H, a.M, a.hm32, 1, 32, path)
    assert v2 == v and ms2 == pytest.approx(ms, rel=1e-4)
