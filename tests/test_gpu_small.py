"""The whole device path on objects smaller than its tiles: 27, 40 and 160 particles (one to twenty
eight-row tiles, ragged last tile, every row's neighbourhood nearly the whole object), against the
oracle's pipeline and its dense generalized eigensolver (Eq. (15)).

Binning, neighbours and the CSR pattern are integer work and bit-exact; values within 1e-12 of the
largest (the FP64 sums in another order). Eigenvalues: the FP64 path to residual 1e-10 within 1e-8
relative; the mixed path (FP32 products, at k = 32 the binary16 matrix-core Chebyshev steps) to
residual 1e-6 within 1e-5 relative and its residual recomputed by the oracle within 2e-6, as the
larger objects' tests state. An object with fewer rows than the block, and an empty one, are refused.
"""
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
    freeform.lib()
    return freeform


@pytest.fixture(scope="module")
def ctx(ff):
    c = ff.Context(0)
    yield c
    c.close()


def dev(a, dt=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device="cuda")


def host(t):
    return t.detach().cpu().numpy()


SMALL = {
    "lattice27": (lambda: synth.cube_lattice(m=3, seed=4), 4),
    "random40": (lambda: synth.random_cloud(40, seed=3, hetero=True, support_factor=3.2), 8),
    "random160": (lambda: synth.random_cloud(160, seed=4, hetero=True, support_factor=3.2), 32),
}


@pytest.fixture(scope="module", params=sorted(SMALL))
def small(request, oracle, ctx, ff):
    make, k = SMALL[request.param]
    c = make()
    P = oracle.pipeline(c)
    A = ff.assemble_cloud(ctx, dev(c.xyz), dev(c.vol), dev(c.lam), dev(c.mu), c.h)
    return request.param, c, P, A, k


def test_small_object_assembly(small):
    name, c, P, A, k = small
    assert np.array_equal(host(A.row_ptr), P.row_ptr), name
    assert np.array_equal(host(A.col), P.col), name
    assert np.abs(host(A.H) - P.H).max() <= 1e-12 * np.abs(P.H).max(), name
    assert np.abs(host(A.M) - P.M).max() <= 1e-12 * np.abs(P.M).max(), name


@pytest.mark.parametrize("precision", [0, 1])
def test_small_object_eigenpairs(small, oracle, ctx, ff, precision):
    name, c, P, A, k = small
    tol = 1e-10 if precision == 0 else 1e-6
    lam, W, res, info = ff.eigenmodes(ctx, c.n, A.row_ptr, A.col, A.H, A.M, A.hm32, k=k, precision=precision,
                                      tol=tol, max_iter=4000)
    assert info["converged"] == 1, name
    H, M = P.Hs(), P.Ms()
    wd, _ = oracle.dense_eigh(H, M, k)
    rel = np.abs(lam[1:] - wd[1:k]) / wd[1:k]
    print(f"\n[small] {name} n={c.n} k={k} precision {precision}: iterations {info['iters_fp32']}+"
          f"{info['iters_fp64']}, max relative eigenvalue error {rel.max():.2e}")
    assert rel.max() <= (1e-8 if precision == 0 else 1e-5), (name, rel.max())
    assert abs(lam[0]) <= (1e-8 if precision == 0 else 1e-5) * wd[1], name
    r_cpu = oracle.residuals(H, M, lam, host(W))
    assert r_cpu.max() <= 2 * tol, (name, r_cpu.max())
    G = host(W).T @ (M @ host(W))
    assert np.abs(G - np.eye(k)).max() <= 1e-6, name


def test_block_wider_than_object_is_refused(oracle, ctx, ff):
    c = synth.cube_lattice(m=3, seed=4)
    A = ff.assemble_cloud(ctx, dev(c.xyz), dev(c.vol), dev(c.lam), dev(c.mu), c.h)
    with pytest.raises(ff.FFError) as ei:
        ff.eigenmodes(ctx, c.n, A.row_ptr, A.col, A.H, A.M, A.hm32, k=32)
    assert ei.value.code == ff.FF_ERR_INVALID_ARG


def test_empty_object_is_refused(ctx, ff):
    """No particles: the entry points refuse the call (FF_ERR_INVALID_ARG), nothing is launched."""
    with pytest.raises(ff.FFError) as ei:
        ff.build_neighbors(ctx, dev(np.zeros((0, 3))), 0.5)
    assert ei.value.code == ff.FF_ERR_INVALID_ARG
    empty_i64 = torch.zeros(1, dtype=torch.int64, device="cuda")
    empty_i32 = torch.zeros(0, dtype=torch.int32, device="cuda")
    empty_f64 = torch.zeros(0, dtype=torch.float64, device="cuda")
    empty_f32 = torch.zeros(0, dtype=torch.float32, device="cuda")
    with pytest.raises(ff.FFError) as ei:
        ff.eigenmodes(ctx, 0, empty_i64, empty_i32, empty_f64, empty_f64, empty_f32, k=4)
    assert ei.value.code == ff.FF_ERR_INVALID_ARG
