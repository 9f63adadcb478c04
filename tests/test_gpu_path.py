"""GPU parity of the HIP path against the FP64 CPU oracle, through the C ABI.

Integer outputs (permutation, cell starts, neighbour lists, CSR pattern) must
be bit-exact; FP64 values within 1e-12 of the oracle relative to their scale;
eigenpairs to the eigenvalue, angle and residual bounds stated per test.
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


def _slab():
    c = synth.random_cloud(1700, seed=9)
    c.xyz[:, 2] *= 0.05
    return c


CLOUDS = {
    "cube1k": lambda: synth.cube_lattice(),
    "cube_unjittered": lambda: synth.cube_lattice(m=9, jitter=0.0, seed=1),
    "random3k_hetero": lambda: synth.random_cloud(3000, seed=5, hetero=True),
    "spheres4k": lambda: synth.sphere_union(n=4000, seed=2, mc_samples=200_000),
    "slab1700": _slab,
}


@pytest.fixture(scope="module", params=sorted(CLOUDS))
def case(request, oracle, ctx, ff):
    c = CLOUDS[request.param]()
    P = oracle.pipeline(c)
    xyz = dev(c.xyz)
    A = ff.assemble_cloud(ctx, xyz, dev(c.vol), dev(c.lam), dev(c.mu), c.h)
    torch.cuda.synchronize()
    return request.param, c, P, A


def test_binning_bitexact(case):
    name, c, P, A = case
    g = A.nb.grid
    assert tuple(g.dims) == tuple(P.dims)
    assert tuple(g.origin) == tuple(P.origin)
    assert np.array_equal(host(A.nb.perm), P.perm)
    assert np.array_equal(host(A.nb.cell_start), P.cell_start)
    assert np.array_equal(host(A.nb.xyz_sorted), P.xyz)


def test_neighbors_bitexact(case):
    name, c, P, A = case
    assert np.array_equal(host(A.nb.nbr_off), P.nbr_off)
    assert np.array_equal(host(A.nb.nbr_id), P.nbr_id)


def test_shape_functions(case):
    name, c, P, A = case
    phi, dphi = host(A.phi), host(A.dphi)
    assert np.abs(phi - P.phi).max() <= 1e-12
    assert np.abs(dphi - P.dphi).max() <= 1e-12 * np.abs(P.dphi).max()


def test_shape_functions_gaussian(case, oracle, ctx, ff):
    """kernel 1 (the Gaussian of Sec. 3.2, r = h/2, cut at h) on the same lists."""
    name, c, P, A = case
    phi_o, dphi_o = oracle.rkpm(P.xyz, P.xyz, P.nbr_off, P.nbr_id, c.h, kernel=1)
    phi, dphi, _ = ff.rkpm_shape(ctx, A.nb.xyz_sorted, A.nb.nbr_off, A.nb.nbr_id, c.h, kernel=1)
    assert np.abs(host(phi) - phi_o).max() <= 1e-12
    assert np.abs(host(dphi) - dphi_o).max() <= 1e-12 * np.abs(dphi_o).max()


def test_assembly(case):
    name, c, P, A = case
    assert np.array_equal(host(A.row_ptr), P.row_ptr)
    assert np.array_equal(host(A.col), P.col)
    H, M = host(A.H), host(A.M)
    assert np.abs(H - P.H).max() <= 1e-12 * np.abs(P.H).max()
    assert np.abs(M - P.M).max() <= 1e-12 * np.abs(P.M).max()
    hm = host(A.hm32)
    assert np.array_equal(hm[:, 0], H.astype(np.float32))
    assert np.array_equal(hm[:, 1], M.astype(np.float32))


def test_assembly_bitwise_symmetric_and_deterministic(case, ctx, ff):
    name, c, P, A = case
    import scipy.sparse as sp
    n = c.n
    Hs = sp.csr_matrix((host(A.H), host(A.col), host(A.row_ptr)), shape=(n, n))
    assert (Hs != Hs.T).nnz == 0
    B = ff.assemble_cloud(ctx, dev(c.xyz), dev(c.vol), dev(c.lam), dev(c.mu), c.h)
    assert torch.equal(A.H, B.H) and torch.equal(A.M, B.M) and torch.equal(A.col, B.col)


def test_assembly_sizing_state_reuse(oracle, ctx, ff):
    """The sizing call keeps its symbolic state for the next call on the same arrays; any
    other call in between (here the sizing of another object) makes the fill call recompute
    it. Both routes give the oracle's CSR bit for bit."""
    import ctypes
    L = ff.lib()
    objs = [synth.random_cloud(2100, seed=61, hetero=True), synth.cube_lattice()]
    pre = []
    for c in objs:
        nb = ff.build_neighbors(ctx, dev(c.xyz), c.h)
        phi, dphi, _ = ff.rkpm_shape(ctx, nb.xyz_sorted, nb.nbr_off, nb.nbr_id, c.h)
        keep = (dev(c.vol), dev(c.lam), dev(c.mu))      # alive while their addresses are in use
        row_ptr = torch.empty(c.n + 1, dtype=torch.int64, device="cuda")
        args = (ctx.h, c.n, c.n, ff._p(nb.nbr_off), ff._p(nb.nbr_id), ff._p(phi), ff._p(dphi), ff._p(keep[0]),
                ff._p(keep[1]), ff._p(keep[2]), None, ff._p(nb.perm), ctypes.byref(nb.grid), ff._p(nb.cell_start),
                ff._p(row_ptr))
        pre.append((c, nb, phi, dphi, keep, row_ptr, args))
    def size(a):
        nnz = ctypes.c_int64()
        ctx.check(L.assemble_HM(*a, None, None, None, None, 0, ctypes.byref(nnz)))
        return nnz.value
    def fill(a, m):
        col = torch.empty(m, dtype=torch.int32, device="cuda")
        H = torch.empty(m, dtype=torch.float64, device="cuda")
        M = torch.empty(m, dtype=torch.float64, device="cuda")
        nnz = ctypes.c_int64()
        ctx.check(L.assemble_HM(*a, ff._p(col), ff._p(H), ff._p(M), None, m, ctypes.byref(nnz)))
        assert nnz.value == m
        return col, H, M
    (c0, _, _, _, _, rp0, a0), (c1, _, _, _, _, rp1, a1) = pre
    m0 = size(a0)
    m1 = size(a1)                         # replaces object 0's state
    fresh = fill(a0, m0)                  # recomputes the symbolic phase
    assert size(a0) == m0
    reused = fill(a0, m0)                 # reuses it
    P = oracle.pipeline(c0)
    assert np.array_equal(host(rp0), P.row_ptr)
    for col, H, M in (fresh, reused):
        assert np.array_equal(host(col), P.col)
        assert np.abs(host(H) - P.H).max() <= 1e-12 * np.abs(P.H).max()
        assert np.abs(host(M) - P.M).max() <= 1e-12 * np.abs(P.M).max()
    assert all(torch.equal(x, y) for x, y in zip(fresh, reused))
    for sized in (False, True):              # a fill short of capacity is refused on either route
        if sized:
            size(a1)
        with pytest.raises(ff.FFError) as ei:
            fill(a1, m1 - 1)
        assert ei.value.code == ff.FF_ERR_CAPACITY


def test_assembly_without_stored_bitmaps(oracle, ctx, ff):
    """The numeric pass reads each row's column bitmap kept by the symbolic pass, or, where
    that store would be too large (FF_ASM_BITMAP_BYTES=0 here), marks the rows itself: the
    same CSR bit for bit, and the oracle's."""
    import os
    c = synth.random_cloud(2100, seed=61, hetero=True)
    A = ff.assemble_cloud(ctx, dev(c.xyz), dev(c.vol), dev(c.lam), dev(c.mu), c.h)
    os.environ["FF_ASM_BITMAP_BYTES"] = "0"
    try:
        ctx2 = ff.Context(0)
    finally:
        del os.environ["FF_ASM_BITMAP_BYTES"]
    B = ff.assemble_cloud(ctx2, dev(c.xyz), dev(c.vol), dev(c.lam), dev(c.mu), c.h)
    for x, y in ((A.row_ptr, B.row_ptr), (A.col, B.col), (A.H, B.H), (A.M, B.M)):
        assert torch.equal(x, y)
    P = oracle.pipeline(c)
    assert np.array_equal(host(B.col), P.col)
    assert np.abs(host(B.H) - P.H).max() <= 1e-12 * np.abs(P.H).max()
    ctx2.close()


def test_separate_quadrature_points(oracle, ctx, ff):
    c = synth.random_cloud(2000, seed=14)
    rng = np.random.default_rng(3)
    q = rng.uniform(-0.1, 1.1, size=(1500, 3))
    nb = ff.build_neighbors(ctx, dev(c.xyz), c.h, qxyz=dev(q))
    perm, cs, origin, dims = oracle.bin_nodes(c.xyz, c.h)
    xs = np.ascontiguousarray(c.xyz[perm])
    off, ids = oracle.neighbors(q, xs, c.h, origin, dims, cs)
    assert np.array_equal(host(nb.nbr_off), off)
    assert np.array_equal(host(nb.nbr_id), ids)
    # points with too few neighbours make the moment matrix singular: report the first
    with pytest.raises(ff.FFError) as ei:
        ff.rkpm_shape(ctx, nb.xyz_sorted, nb.nbr_off, nb.nbr_id, c.h, qxyz=dev(q))
    cnt = np.diff(off)
    if (cnt >= 4).all():
        pytest.skip("no singular point in this draw")
    assert ei.value.code == ff.FF_ERR_SINGULAR_MOMENT


@pytest.mark.parametrize("shuffled", [False, True])
@pytest.mark.parametrize("kernel", [0, 1])
def test_assembly_separate_quadrature_points(oracle, ctx, ff, kernel, shuffled):
    """q != n: 2,600 quadrature points on a jittered grid inside the node box (every one sees
    enough nodes), their own weights and material; the per-point arrays either in quadrature
    order (perm NULL) or shuffled, with perm[i] naming point i's entry. Pattern bit-exact,
    values to 1e-12 of their scale."""
    c = synth.random_cloud(2000, seed=44, hetero=True)
    rng = np.random.default_rng(8)
    g = (np.arange(14) + 0.5) / 14
    q = np.stack(np.meshgrid(g, g, g, indexing="ij"), axis=-1).reshape(-1, 3)[:2600]
    q = np.clip(q + rng.uniform(-0.01, 0.01, q.shape), 0.02, 0.98)
    nq = q.shape[0]
    vol = np.full(nq, 1.0 / nq)
    E = np.exp(rng.uniform(np.log(1e4), np.log(1e6), nq))
    lam, mu = synth.lame_from_young(E, rng.uniform(0.3, 0.48, nq))
    perm_n, cs, origin, dims = oracle.bin_nodes(c.xyz, c.h)
    xs = np.ascontiguousarray(c.xyz[perm_n])
    off, ids = oracle.neighbors(q, xs, c.h, origin, dims, cs)
    phi, dphi = oracle.rkpm(q, xs, off, ids, c.h, kernel=kernel)
    rp, col, H, M = oracle.assemble(c.n, off, ids, phi, dphi, vol, lam, mu)
    nb = ff.build_neighbors(ctx, dev(c.xyz), c.h, qxyz=dev(q))
    assert np.array_equal(host(nb.nbr_id), ids)
    gphi, gdphi, _ = ff.rkpm_shape(ctx, nb.xyz_sorted, nb.nbr_off, nb.nbr_id, c.h, qxyz=dev(q), kernel=kernel)
    assert np.abs(host(gphi) - phi).max() <= 1e-12
    assert np.abs(host(gdphi) - dphi).max() <= 1e-12 * np.abs(dphi).max()
    if shuffled:
        sig = rng.permutation(nq).astype(np.int32)       # point i's values sit at entry sig[i]
        store = lambda a: np.empty_like(a)
        v2, l2, m2 = store(vol), store(lam), store(mu)
        v2[sig], l2[sig], m2[sig] = vol, lam, mu
        args = dict(perm=dev(sig, torch.int32))
        vol_d, lam_d, mu_d = dev(v2), dev(l2), dev(m2)
    else:
        args = {}
        vol_d, lam_d, mu_d = dev(vol), dev(lam), dev(mu)
    grp, gcol, gH, gM, _ = ff.assemble_HM(ctx, c.n, nb.nbr_off, nb.nbr_id, gphi, gdphi, vol_d, lam_d, mu_d, nb.grid,
                                         nb.cell_start, **args)
    assert np.array_equal(host(grp), rp)
    assert np.array_equal(host(gcol), col)
    assert np.abs(host(gH) - H).max() <= 1e-12 * np.abs(H).max()
    assert np.abs(host(gM) - M).max() <= 1e-12 * np.abs(M).max()


def test_singular_moment_index(ctx, ff):
    xs = dev(np.array([[0.0, 0.0, 0.0], [0.1, 0.0, 0.0], [0.2, 0.0, 0.0], [0.9, 0.9, 0.9]]))
    nb = ff.build_neighbors(ctx, xs, 0.25)
    with pytest.raises(ff.FFError) as ei:
        ff.rkpm_shape(ctx, nb.xyz_sorted, nb.nbr_off, nb.nbr_id, 0.25)
    assert ei.value.code == ff.FF_ERR_SINGULAR_MOMENT
    assert ei.value.bad_index == 0


def test_invalid_arguments(ctx, ff):
    bad = dev(np.array([[0.0, np.nan, 0.0], [1.0, 1.0, 1.0]]))
    with pytest.raises(ff.FFError) as ei:
        ff.build_neighbors(ctx, bad, 0.5)
    assert ei.value.code == ff.FF_ERR_INVALID_ARG
    with pytest.raises(ff.FFError):
        ff.build_neighbors(ctx, dev(np.zeros((4, 3))), -1.0)


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("m", [8, 16, 24, 32, 64])
def test_spmm(oracle, ctx, ff, precision, m):
    c = synth.random_cloud(2500, seed=21, hetero=True)
    P = oracle.pipeline(c)
    A = ff.assemble_cloud(ctx, dev(c.xyz), dev(c.vol), dev(c.lam), dev(c.mu), c.h)
    rng = np.random.default_rng(m)
    Y = rng.standard_normal((c.n, m))
    dt = torch.float32 if precision else torch.float64
    refH = oracle.spmm(P.row_ptr, P.col, P.H, Y)
    refM = oracle.spmm(P.row_ptr, P.col, P.M, Y)
    absH = oracle.spmm(P.row_ptr, P.col, np.abs(P.H), np.abs(Y))
    absM = oracle.spmm(P.row_ptr, P.col, np.abs(P.M), np.abs(Y))
    out = {}
    for v, name in enumerate(ff.spmm_variant_names()):
        if name.startswith("rowtile8_mfma") and (precision == 0 or m not in (8, 16, 32, 64)):
            # the eight-row FP64-MFMA variants take FP32 blocks of these widths only
            with pytest.raises(ff.FFError):
                ff.spmm_hm(ctx, A.row_ptr, A.col, A.H, A.M, A.hm32, dev(Y, dt), precision, variant=v)
            continue
        # outputs filled with NaN first, so that a row a kernel does not write cannot pass on what an
        # earlier variant left in the same memory
        out_nan = (torch.full((c.n, m), float("nan"), dtype=dt, device="cuda"),
                   torch.full((c.n, m), float("nan"), dtype=dt, device="cuda"))
        HY, MY = ff.spmm_hm(ctx, A.row_ptr, A.col, A.H, A.M, A.hm32, dev(Y, dt), precision, variant=v, out=out_nan)
        eps = 2e-6 if precision else 1e-13
        assert np.all(np.abs(host(HY) - refH) <= eps * absH + 1e-300), name
        assert np.all(np.abs(host(MY) - refM) <= eps * absM + 1e-300), name
        out[name] = (host(HY), host(MY))
    # the pipelined eight-row kernels issue the same matrix-core steps in the same order
    for a, b in (("rowtile8_mfma64_pipelined_waves4", "rowtile8_mfma64_waves4_batch8"),
                 ("rowtile8_mfma64_pipelined_waves2", "rowtile8_mfma64_waves4_batch8"),
                 ("rowtile8_mfma32x64_pipelined_waves4", "rowtile8_mfma32x64_waves4_batch8")):
        if a in out:
            assert np.array_equal(out[a][0], out[b][0]) and np.array_equal(out[a][1], out[b][1]), (a, m)


@pytest.mark.parametrize("precision", [0, 1])
def test_rowtiles_spmm(oracle, ctx, ff, precision):
    """The row-tile copy (tiles of four rows, ragged last tile) gives the same products;
    its union entries are at least the largest row and at most the sum of four rows."""
    c = synth.random_cloud(2501, seed=23, hetero=True)
    P = oracle.pipeline(c)
    A = ff.assemble_cloud(ctx, dev(c.xyz), dev(c.vol), dev(c.lam), dev(c.mu), c.h)
    rt = ff.RowTiles(ctx, A.n, A.row_ptr, A.col, A.H, A.M, precision=precision)
    ntiles, entries = rt.info()
    assert ntiles == (c.n + 3) // 4
    rl = np.diff(P.row_ptr)
    assert rl.max() <= entries <= rl.sum()
    dt = torch.float32 if precision else torch.float64
    eps = 2e-6 if precision else 1e-13
    nan = lambda m: torch.full((c.n, m), float("nan"), dtype=dt, device="cuda")
    # m = 64 at FP64 leaves two lane groups per wave (fewer than the tile's four rows); outputs start
    # as NaN so that a row a kernel does not write fails
    for m in (8, 24, 32, 64):
        Y = np.random.default_rng(m).standard_normal((c.n, m))
        refH = oracle.spmm(P.row_ptr, P.col, P.H, Y)
        refM = oracle.spmm(P.row_ptr, P.col, P.M, Y)
        absH = oracle.spmm(P.row_ptr, P.col, np.abs(P.H), np.abs(Y))
        absM = oracle.spmm(P.row_ptr, P.col, np.abs(P.M), np.abs(Y))
        for sub in range(3):
            HY, MY = rt.spmm(dev(Y, dt), precision, sub, out=(nan(m), nan(m)))
            assert np.all(np.abs(host(HY) - refH) <= eps * absH + 1e-300)
            assert np.all(np.abs(host(MY) - refM) <= eps * absM + 1e-300)
            # H alone (the preconditioner's product): FP32 accumulation at precision 1, whose
            # longest chain of roundings is a lane group's share of a tile (at most 4 rows / 8)
            # plus the three cross-group additions and the rounding of the values and of Y
            HO, none = rt.spmm(dev(Y, dt), precision, sub, h_only=True, out=(nan(m), None))
            assert none is None
            eps_h = (4 * rl.max() // 8 + 6) * 2.0 ** -24 if precision else 1e-13
            assert np.all(np.abs(host(HO) - refH) <= eps_h * absH + 1e-300)
    rt.close()


@pytest.mark.parametrize("bitmap", [True, False])
@pytest.mark.parametrize("rows,hf", [(8, 1.0), (16, 1.0), (8, 1.3)])
def test_rowtiles_h_only_copies(oracle, ctx, ff, rows, hf, bitmap):
    """The preconditioner's H-only copies in tiles of eight rows (VALU kernel) and of
    sixteen rows (MFMA kernel), ragged last tile: H Y in FP32 accumulation, every launch
    shape and the block widths the kernels take; other forms are rejected. The copies are
    built one workgroup per tile: from a bitmap of the tile's column range in LDS, or
    (FF_UNION_BITS=0, as for a range beyond the bitmap) from the rows' columns in LDS by
    binary search, tiles beyond that capacity by the serial merge: the sixteen-row tiles of
    this cloud and the eight-row tiles at a 1.3x support radius (up to 7766 entries per
    tile) take both of the latter."""
    import os
    c = synth.random_cloud(2503, seed=29, hetero=True)
    c.h *= hf
    P = oracle.pipeline(c)
    A = ff.assemble_cloud(ctx, dev(c.xyz), dev(c.vol), dev(c.lam), dev(c.mu), c.h)
    if not bitmap:
        os.environ["FF_UNION_BITS"] = "0"
        try:
            ctx = ff.Context(0)
        finally:
            del os.environ["FF_UNION_BITS"]
    rt = ff.RowTiles(ctx, A.n, A.row_ptr, A.col, A.H, A.M, precision=3 if rows == 8 else 4)
    ntiles, entries = rt.info()
    assert ntiles == (c.n + rows - 1) // rows
    rl = np.diff(P.row_ptr)
    assert rl.max() <= entries <= rl.sum()
    # longest rounding chain: the entries one accumulator sums (a lane group's share of a
    # tile, at most rows x the longest row over 8 groups, or a whole tile's union in the
    # MFMA), the butterfly's additions, the rounding of the values and of Y
    eps = ((rl.max() if rows == 8 else 16 * rl.max()) + 8) * 2.0 ** -24
    for m in ((8, 16, 32, 64) if rows == 8 else (4, 8, 12, 16, 32, 64)):
        Y = np.random.default_rng(m).standard_normal((c.n, m))
        refH = oracle.spmm(P.row_ptr, P.col, P.H, Y)
        absH = oracle.spmm(P.row_ptr, P.col, np.abs(P.H), np.abs(Y))
        for sub in range(3):
            HO, none = rt.spmm(dev(Y, torch.float32), 1, sub, h_only=True)
            assert none is None
            assert np.all(np.abs(host(HO) - refH) <= eps * absH + 1e-300), (m, sub)
    Y = dev(np.ones((c.n, 24)), torch.float32)
    with pytest.raises(ff.FFError):
        rt.spmm(Y, 1, 0, h_only=True)                      # a width neither kernel takes
    with pytest.raises(ff.FFError):
        rt.spmm(dev(np.ones((c.n, 32)), torch.float32), 1, 0)   # MY requested
    rt.close()
    if not bitmap:
        ctx.close()


def _fp16_storage(H):
    """H as the FP16 tile copy stores it (rowtiles_build precision 5): FP32 rounding, scale
    2^e with the largest magnitude in [2^14, 2^15), binary16 rounding to nearest even."""
    h32 = H.astype(np.float32)
    amax = float(np.abs(h32).max())
    e = 15 - int(np.frexp(amax)[1]) if amax > 0 else 0
    q = (h32.astype(np.float64) * 2.0 ** e).astype(np.float16)
    assert np.all(np.isfinite(q))
    return q.astype(np.float64) * 2.0 ** -e, e


def _banded_csr(seed=5):
    """A CSR whose row bands grow along the rows, so that eight-row tiles hold from a few to
    several hundred union entries: rows 0-999 reach at most 4 columns either side, rows
    1000-1399 40-59, rows 1400-1799 60-89, rows 1800-2199 90-159, the rest 160-399; n = 3001
    leaves a ragged last tile."""
    rng = np.random.default_rng(seed)
    n = 3001
    band = np.concatenate([rng.integers(0, 5, 1000), rng.integers(40, 60, 400), rng.integers(60, 90, 400),
                           rng.integers(90, 160, 400), rng.integers(160, 400, n - 2200)])
    cols = [np.arange(max(0, i - b), min(n, i + b + 1)) for i, b in enumerate(band)]
    row_ptr = np.concatenate([[0], np.cumsum([len(c) for c in cols])]).astype(np.int64)
    col = np.concatenate(cols).astype(np.int32)
    H = rng.standard_normal(len(col))
    M = rng.uniform(0.1, 1.0, len(col))
    E = np.array([len(np.unique(col[row_ptr[t]:row_ptr[min(t + 8, n)]])) for t in range(0, n, 8)])
    return n, row_ptr, col, H, M, E


def test_rowtile_kernels_short_tiles(oracle, ctx, ff):
    """The pipelined product kernels on tiles of every length, including the shortest tails
    (one and two chunks of 64 entries for the fused [H, M] product, one and two super-blocks
    of four K-blocks for the binary16 product): against the plain CSR product of the oracle,
    and bitwise against the unpipelined kernels."""
    n, row_ptr, col, H, M, E = _banded_csr()
    chunks, superblocks = set(((E + 63) // 64).tolist()), set((((E + 15) // 16 + 3) // 4).tolist())
    assert {1, 2, 3, 4, 5} <= chunks and {1, 2, 3, 4, 5} <= superblocks
    rp, cl, Hd, Md = dev(row_ptr, torch.int64), dev(col, torch.int32), dev(H), dev(M)
    hm32 = torch.stack([Hd.float(), Md.float()], dim=1).reshape(-1).contiguous()
    names = ff.spmm_variant_names()
    for m in (8, 32, 64):
        Y = np.random.default_rng(m).standard_normal((n, m))
        refH, refM = oracle.spmm(row_ptr, col, H, Y), oracle.spmm(row_ptr, col, M, Y)
        absH = oracle.spmm(row_ptr, col, np.abs(H), np.abs(Y))
        absM = oracle.spmm(row_ptr, col, np.abs(M), np.abs(Y))
        out = {}
        for v, name in enumerate(names):
            if not name.startswith("rowtile8_mfma"):
                continue
            HY, MY = ff.spmm_hm(ctx, rp, cl, Hd, Md, hm32, dev(Y, torch.float32), 1, variant=v)
            HY, MY = host(HY), host(MY)
            assert np.all(np.abs(HY - refH) <= 2e-6 * absH + 1e-300), (name, m)
            assert np.all(np.abs(MY - refM) <= 2e-6 * absM + 1e-300), (name, m)
            out[name] = (HY, MY)
        # the zero-free copy gives the same operands as the full tiles: the same sums
        for a, b in (("rowtile8_mfma64_pipelined_waves4", "rowtile8_mfma64_waves4_batch8"),
                     ("rowtile8_mfma64_pipelined_waves2", "rowtile8_mfma64_waves4_batch8"),
                     ("rowtile8_mfma64_zerofree_waves2", "rowtile8_mfma64_waves4_batch8"),
                     ("rowtile8_mfma64_zerofree_waves4", "rowtile8_mfma64_waves4_batch8"),
                     ("rowtile8_mfma32x64_pipelined_waves4", "rowtile8_mfma32x64_waves4_batch8")):
            assert np.array_equal(out[a][0], out[b][0]) and np.array_equal(out[a][1], out[b][1]), (a, m)
    rt = ff.RowTiles(ctx, n, rp, cl, Hd, None, precision=6)
    Hq, _ = _fp16_storage(H)
    rl = np.diff(row_ptr)
    eps = (8 * rl.max() + 8) * 2.0 ** -24
    for m in (32, 64):
        Y = np.random.default_rng(m).standard_normal((n, m)).astype(np.float16).astype(np.float64)
        refq = oracle.spmm(row_ptr, col, Hq, Y)
        absq = oracle.spmm(row_ptr, col, np.abs(Hq), np.abs(Y))
        HO, _ = rt.spmm(dev(Y, torch.float16), 2, 0)
        HO = host(HO)
        assert np.all(np.abs(HO - refq) <= eps * absq + 1e-300), m
        for sub in range(1, 15):
            HS, _ = rt.spmm(dev(Y, torch.float16), 2, sub)
            assert np.array_equal(host(HS), HO), (m, sub)
    rt.close()


def test_rowtiles_fp16_copy(oracle, ctx, ff):
    """The preconditioner's default copy: H in binary16 (scaled by a power of two) in
    tiles of eight rows, ragged last tile. Against H as stored it obeys the same FP32
    accumulation bound as the FP32 copy; against the exact H each value adds at most
    2^-11 relative (or half a subnormal step)."""
    c = synth.random_cloud(2503, seed=29, hetero=True)
    P = oracle.pipeline(c)
    A = ff.assemble_cloud(ctx, dev(c.xyz), dev(c.vol), dev(c.lam), dev(c.mu), c.h)
    rt = ff.RowTiles(ctx, A.n, A.row_ptr, A.col, A.H, None, precision=5)
    ntiles, entries = rt.info()
    assert ntiles == (c.n + 7) // 8
    Hq, e = _fp16_storage(P.H)
    rl = np.diff(P.row_ptr)
    eps = (rl.max() + 8) * 2.0 ** -24
    for m in (8, 16, 32, 64):
        Y = np.random.default_rng(m).standard_normal((c.n, m))
        refq = oracle.spmm(P.row_ptr, P.col, Hq, Y)
        absq = oracle.spmm(P.row_ptr, P.col, np.abs(Hq), np.abs(Y))
        ref = oracle.spmm(P.row_ptr, P.col, P.H, Y)
        absH = oracle.spmm(P.row_ptr, P.col, np.abs(P.H), np.abs(Y))
        absY = oracle.spmm(P.row_ptr, P.col, np.ones_like(P.H), np.abs(Y))
        for sub in range(3):
            HO, none = rt.spmm(dev(Y, torch.float32), 1, sub, h_only=True)
            assert none is None
            HO = host(HO)
            assert np.all(np.abs(HO - refq) <= eps * absq + 1e-300), (m, sub)
            assert np.all(np.abs(HO - ref) <= (2.0 ** -11 + 2 * eps) * absH + 2.0 ** (-24 - e) * absY), (m, sub)
    rt.close()
    with pytest.raises(ff.FFError):
        ff.RowTiles(ctx, A.n, A.row_ptr, A.col, A.H, None, precision=7)


def test_rowtiles_fp16_kblocked_matrix_core(oracle, ctx, ff):
    """The matrix-core product: H in binary16 K-blocks (rowtiles_build precision 6),
    a binary16 block Y, FP32 sums on v_mfma_f32_16x16x16_f16, ragged last tile and
    tiles whose entry count is not a multiple of 16. Against H as stored (and Y exactly,
    being binary16) the FP32 accumulation bound holds; against the exact H each value
    adds at most 2^-11 relative."""
    c = synth.random_cloud(2503, seed=29, hetero=True)
    P = oracle.pipeline(c)
    A = ff.assemble_cloud(ctx, dev(c.xyz), dev(c.vol), dev(c.lam), dev(c.mu), c.h)
    rt = ff.RowTiles(ctx, A.n, A.row_ptr, A.col, A.H, None, precision=6)
    Hq, e = _fp16_storage(P.H)
    rl = np.diff(P.row_ptr)
    eps = (8 * rl.max() + 8) * 2.0 ** -24
    for m in (32, 64):
        Y = np.random.default_rng(m).standard_normal((c.n, m)).astype(np.float16).astype(np.float64)
        refq = oracle.spmm(P.row_ptr, P.col, Hq, Y)
        absq = oracle.spmm(P.row_ptr, P.col, np.abs(Hq), np.abs(Y))
        ref = oracle.spmm(P.row_ptr, P.col, P.H, Y)
        absH = oracle.spmm(P.row_ptr, P.col, np.abs(P.H), np.abs(Y))
        absY = oracle.spmm(P.row_ptr, P.col, np.ones_like(P.H), np.abs(Y))
        HO, none = rt.spmm(dev(Y, torch.float16), 2)
        assert none is None and HO.dtype == torch.float32
        HO = host(HO)
        assert np.all(np.abs(HO - refq) <= eps * absq + 1e-300), m
        assert np.all(np.abs(HO - ref) <= (2.0 ** -11 + 2 * eps) * absH + 2.0 ** (-24 - e) * absY), m
        # every launch shape (the ring of K-blocks and the super-block pipeline, several waves per
        # workgroup) sums the K-blocks in the same order: bitwise the same result
        # (shapes 8 .. 14 read the K-blocks without their zeros and rebuild them in LDS: the same
        # operands, so the same sums; 13 and 14 keep one buffer of gathers)
        for sub in range(1, 15):
            HS, _ = rt.spmm(dev(Y, torch.float16), 2, sub)
            assert np.array_equal(host(HS), HO), (m, sub)
        with pytest.raises(ff.FFError):
            rt.spmm(dev(Y, torch.float16), 2, 15)
        # the FP32 forms of the same handle agree with the binary16 one to the stored values' rounding
        HF, _ = rt.spmm(dev(Y, torch.float32), 1, h_only=True)
        assert np.all(np.abs(host(HF) - ref) <= 2 * eps * absH + 1e-300), m
    for m in (16, 48):
        with pytest.raises(ff.FFError):
            rt.spmm(dev(np.ones((c.n, m)), torch.float16), 2)
    with pytest.raises(ff.FFError):      # binary16 products need the K-blocked copy
        rt5 = ff.RowTiles(ctx, A.n, A.row_ptr, A.col, A.H, None, precision=5)
        try:
            rt5.spmm(dev(np.ones((c.n, 32)), torch.float16), 2)
        finally:
            rt5.close()
    rt.close()


def test_philox_known_answers(ctx, ff):
    """Known-answer vectors of Philox-4x32-10 (Salmon et al., SC'11, Random123 distribution)."""
    import os
    rows = []
    with open(os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                rows.append([int(x, 16) for x in line.split()])
    rows = np.array(rows, dtype=np.uint64)
    ctr = dev(rows[:, 0:4].astype(np.int64).astype(np.uint32).view(np.int32), torch.int32)
    key = dev(rows[:, 4:6].astype(np.int64).astype(np.uint32).view(np.int32), torch.int32)
    out = host(ff.philox4x32_10(ctx, ctr, key)).view(np.uint32)
    assert np.array_equal(out.astype(np.uint64), rows[:, 6:10])


def _check_modes(oracle, P, lam, W, res, k, rel_tol, sin_tol, resid_tol):
    H, M = P.Hs(), P.Ms()
    wd, Vd = oracle.dense_eigh(H, M, k + 4)
    assert np.abs(lam[1:] - wd[1:k]).max() / wd[1:k].min() <= rel_tol
    assert abs(lam[0]) <= rel_tol * wd[1]
    assert res.max() <= resid_tol
    # residuals recomputed on the CPU with the oracle's matrices
    r_cpu = oracle.residuals(H, M, lam, W)
    assert r_cpu.max() <= 2 * resid_tol
    # M-orthonormal
    G = W.T @ (M @ W)
    assert np.abs(G - np.eye(k)).max() <= 1e-6
    kk = oracle.cluster_safe_k(wd, k)
    if kk > 0:
        s = oracle.subspace_sines(Vd[:, :kk], W[:, :kk], M)
        assert s.max() <= sin_tol
    # sign rule
    idx = np.argmax(np.abs(W), axis=0)
    assert np.all(W[idx, np.arange(k)] > 0)


@pytest.mark.parametrize("precision,precond,degree,values", [(0, 1, 0, 0), (1, 1, 0, 0), (0, 2, 0, 0), (1, 2, 3, 0),
                                                            (1, 2, 8, 0), (1, 2, 16, 0), (1, 2, 0, 1),
                                                            (1, 2, 0, 2)])
def test_eigenmodes_cube(oracle, ctx, ff, precision, precond, degree, values):
    c = synth.cube_lattice()
    P = oracle.pipeline(c)
    A = ff.assemble_cloud(ctx, dev(c.xyz), dev(c.vol), dev(c.lam), dev(c.mu), c.h)
    k = 8
    lam, W, res, info = ff.eigenmodes(ctx, c.n, A.row_ptr, A.col, A.H, A.M, A.hm32, k=k, precision=precision,
                                      tol=1e-8 if precision == 0 else 1e-6, max_iter=4000, precond=precond,
                                      precond_degree=degree, precond_values=values)
    _check_modes(oracle, P, lam, host(W), res, k, 1e-8 if precision == 0 else 1e-5,
                 1e-6 if precision == 0 else 1e-3, 1e-8 if precision == 0 else 1e-6)


@pytest.mark.parametrize("precision,precond", [(0, 1), (1, 1), (0, 2), (1, 2)])
def test_eigenmodes_random_hetero(oracle, ctx, ff, precision, precond):
    """i.i.d. random particles give cond(M) ~ 2e7: a backward-error residual of 1e-6
    leaves ~3e-4 eigenvalue error even in exact FP64, so parity is checked at 1e-8
    (where the oracle's own solve is accurate to ~4e-8)."""
    c = synth.random_cloud(2500, seed=33, hetero=True)
    P = oracle.pipeline(c)
    A = ff.assemble_cloud(ctx, dev(c.xyz), dev(c.vol), dev(c.lam), dev(c.mu), c.h)
    k = 16
    lam, W, res, info = ff.eigenmodes(ctx, c.n, A.row_ptr, A.col, A.H, A.M, A.hm32, k=k, precision=precision,
                                      tol=1e-8, max_iter=8000, precond=precond)
    _check_modes(oracle, P, lam, host(W), res, k, 1e-5, 1e-3, 1e-8)


@pytest.mark.parametrize("values", [1, 2, 3, 4])
def test_eigenmodes_chebyshev_number_formats(oracle, ctx, ff, values):
    """k = 32 (the benchmark's block width): the Chebyshev-Jacobi products with H and the
    iterate in FP32 (1), H in binary16 (2), and both in binary16 on the matrix cores (3,
    the default at this width, with per-column scaling of the recurrence); the converged
    eigenpairs meet the same bounds in every case."""
    c = synth.random_cloud(2500, seed=33, hetero=True)
    P = oracle.pipeline(c)
    A = ff.assemble_cloud(ctx, dev(c.xyz), dev(c.vol), dev(c.lam), dev(c.mu), c.h)
    k = 32
    lam, W, res, info = ff.eigenmodes(ctx, c.n, A.row_ptr, A.col, A.H, A.M, A.hm32, k=k, precision=1, tol=1e-8,
                                      max_iter=8000, precond=2, precond_values=values)
    assert info["converged"] == 1
    _check_modes(oracle, P, lam, host(W), res, k, 1e-5, 1e-3, 1e-8)


@pytest.mark.parametrize("values", [3, 4])
@pytest.mark.parametrize("degree", [2, 3, 9])
def test_eigenmodes_matrix_core_chebyshev_degrees(oracle, ctx, ff, degree, values):
    """k = 32 on the matrix cores with step counts 1, 2 and 8: the block W takes the iterates of
    two steps at every second step, and the last step's own when the count is odd, so a single
    step, one pair and an even count (the last step adding two iterates) all reach the same
    eigenpairs."""
    c = synth.random_cloud(2500, seed=33, hetero=True)
    P = oracle.pipeline(c)
    A = ff.assemble_cloud(ctx, dev(c.xyz), dev(c.vol), dev(c.lam), dev(c.mu), c.h)
    k = 32
    lam, W, res, info = ff.eigenmodes(ctx, c.n, A.row_ptr, A.col, A.H, A.M, A.hm32, k=k, precision=1, tol=1e-8,
                                      max_iter=8000, precond=2, precond_degree=degree, precond_values=values)
    assert info["converged"] == 1
    _check_modes(oracle, P, lam, host(W), res, k, 1e-5, 1e-3, 1e-8)


@pytest.mark.parametrize("values,seed", [(1, 0), (2, 1), (3, 0), (3, 1), (4, 0)])
def test_eigenmodes_stable_near_convergence(oracle, ctx, ff, values, seed):
    """k = 32 on the 1000-particle lattice, residual 1e-8: most pairs converge long before the
    last one and their P columns shrink to rounding level, where their implicitly updated
    images are noise. The Rayleigh-Ritz step drops such columns (M-norm below 1e-6 in FP32,
    1e-12 in FP64); without that every residual jumped back to ~1e-3 after reaching 4e-8 and
    the basis lost rank."""
    c = synth.cube_lattice()
    P = oracle.pipeline(c)
    A = ff.assemble_cloud(ctx, dev(c.xyz), dev(c.vol), dev(c.lam), dev(c.mu), c.h)
    k = 32
    lam, W, res, info = ff.eigenmodes(ctx, c.n, A.row_ptr, A.col, A.H, A.M, A.hm32, k=k, precision=1, tol=1e-8,
                                      max_iter=3000, precond=2, precond_values=values, seed=seed)
    assert info["converged"] == 1
    _check_modes(oracle, P, lam, host(W), res, k, 1e-5, 1e-3, 1e-8)


def test_eigenmodes_given_start_block(oracle, ctx, ff):
    c = synth.cube_lattice()
    P = oracle.pipeline(c)
    A = ff.assemble_cloud(ctx, dev(c.xyz), dev(c.vol), dev(c.lam), dev(c.mu), c.h)
    X0 = synth.initial_block(c.n, 8, seed=4)
    perm = P.perm
    lam, W, res, info = ff.eigenmodes(ctx, c.n, A.row_ptr, A.col, A.H, A.M, A.hm32, k=8, precision=0, tol=1e-8,
                                      X0=dev(X0[perm]))
    _check_modes(oracle, P, lam, host(W), res, 8, 1e-8, 1e-6, 1e-8)


def test_chebyshev_parameters_are_validated(ctx, ff):
    c = synth.cube_lattice()
    A = ff.assemble_cloud(ctx, dev(c.xyz), dev(c.vol), dev(c.lam), dev(c.mu), c.h)
    for bad in (1, 17, -2):
        with pytest.raises(ff.FFError):
            ff.eigenmodes(ctx, c.n, A.row_ptr, A.col, A.H, A.M, A.hm32, k=8, precond=2, precond_degree=bad)
    with pytest.raises(ff.FFError):
        ff.eigenmodes(ctx, c.n, A.row_ptr, A.col, A.H, A.M, A.hm32, k=8, precond=3)
    for bad in (0.5, 1.0, -3.0):
        with pytest.raises(ff.FFError):
            ff.eigenmodes(ctx, c.n, A.row_ptr, A.col, A.H, A.M, A.hm32, k=8, precond=2, precond_ratio=bad)
    for bad in (-1, 5, 4, 3):     # 3 and 4 need block width 32 or 64
        with pytest.raises(ff.FFError):
            ff.eigenmodes(ctx, c.n, A.row_ptr, A.col, A.H, A.M, A.hm32, k=8, precond=2, precond_values=bad)


def test_not_converged_still_returns(ctx, ff):
    c = synth.cube_lattice()
    A = ff.assemble_cloud(ctx, dev(c.xyz), dev(c.vol), dev(c.lam), dev(c.mu), c.h)
    lam, W, res, info = ff.eigenmodes(ctx, c.n, A.row_ptr, A.col, A.H, A.M, A.hm32, k=8, precision=0, tol=1e-12,
                                      max_iter=3, allow_unconverged=True)
    assert info["status"] == ff.FF_ERR_NOT_CONVERGED
    assert np.all(np.isfinite(lam)) and np.all(res > 0)


def test_stage_timing(ctx, ff):
    """Per-stage HIP-event times: off by default (only the total), on they cover every
    stage, the Chebyshev products count degree - 1 launches per body pass, and the
    stage sums stay within the call's wall time."""
    c = synth.cube_lattice()
    A = ff.assemble_cloud(ctx, dev(c.xyz), dev(c.vol), dev(c.lam), dev(c.mu), c.h)
    run = lambda: ff.eigenmodes(ctx, c.n, A.row_ptr, A.col, A.H, A.M, A.hm32, k=8, precision=1, tol=1e-6,
                                precond=2, precond_degree=3)
    run()
    st = ctx.stage_times()
    assert set(st) == {"spmm", "precond_product", "precond_other", "gram", "rayleigh_ritz", "update", "resid",
                       "fp64_phase", "total"}
    assert all(v == (0.0, 0) for k, v in st.items() if k != "total") and st["total"][0] > 0
    ctx.set_stage_timing(True)
    try:
        lam, W, res, info = run()
        st = ctx.stage_times()
    finally:
        ctx.set_stage_timing(False)
    for k in ("spmm", "precond_product", "precond_other", "gram", "rayleigh_ritz", "update", "resid", "fp64_phase"):
        assert st[k][0] > 0 and st[k][1] > 0, k
    # the mixed path's FP64 phase is one stage: the Chebyshev launches are the FP32 iterations' (degree 3:
    # two per pass, passes up to the next convergence check)
    assert st["fp64_phase"][1] == 1
    assert st["precond_product"][1] % 2 == 0
    assert 2 * info["iters_fp32"] <= st["precond_product"][1] <= 2 * (info["iters_fp32"] + 10)
    assert sum(v[0] for k, v in st.items() if k != "total") <= st["total"][0] * 1.01
