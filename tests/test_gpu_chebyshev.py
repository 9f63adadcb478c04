"""The eigensolver's Chebyshev-Jacobi preconditioner alone (chebyshev_apply, the same set-up and
launches as inside eigenmodes) against the oracle's FP64 Chebyshev semi-iteration
(oracle.chebyshev_jacobi) on the same interval, through the C ABI.

Every degree's output is the sum of its increments; the matrix-core steps fold two
increments into the output block at every second step and the last one alone when the
count is odd, so the degrees 2, 3, 9 and 12 cover a single step, one pair, an odd and an
even count. A dropped or doubled increment moves the output by at least the smallest
increment's share of it, which the test computes from the oracle's increments and requires
to be at least twice the tolerance, so no such mistake passes.

Tolerances: FP32 products (values 1) 2e-5 relative per column; binary16 H (2) and binary16 H
and iterate on the matrix cores (3, 4) 5e-3 (each stored value and each iterate rounds to 11
significant bits). With values 3 and 4 the library scales column c of the input by
1 / max |D^-1 r_c| before the recurrence (the binary16 range), so its output is the exact one
times that factor.
"""
import numpy as np
import pytest

from paper_2605_29318_amd import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

TOL = {1: 2e-5, 2: 5e-3, 3: 5e-3, 4: 5e-3}


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


@pytest.fixture(scope="module")
def cloud(oracle, ctx, ff):
    c = synth.random_cloud(2500, seed=33, hetero=True)
    P = oracle.pipeline(c)
    A = ff.assemble_cloud(ctx, dev(c.xyz), dev(c.vol), dev(c.lam), dev(c.mu), c.h)
    T = oracle.chebyshev_jacobi(P.Hs(), degree=2)          # its default interval: 1.05 x ARPACK's top
    return c, P, A, T.upper


def _scaled_reference(oracle, P, R, degree, upper, values):
    T = oracle.chebyshev_jacobi(P.Hs(), degree=degree, upper=upper)
    rec = []
    ref = T(R, record=rec)
    if values >= 3:
        d = np.asarray(P.Hs().diagonal())
        dinv32 = (1.0 / d).astype(np.float32).astype(np.float64)
        w = (R * dinv32[:, None]).astype(np.float32)       # D^-1 r as the library forms it (FP32)
        ref = ref / np.abs(w).max(axis=0).astype(np.float64)[None, :]
    share = min(np.min(np.linalg.norm(s, axis=0) / np.linalg.norm(T(R), axis=0)) for s in rec)
    return ref, share


@pytest.mark.parametrize("values", [1, 2, 3, 4])
@pytest.mark.parametrize("degree", [2, 3, 9, 12])
def test_chebyshev_apply_matches_the_recurrence(cloud, oracle, ctx, ff, degree, values):
    c, P, A, upper = cloud
    m = 32
    R = np.random.default_rng(100 * degree + values).standard_normal((c.n, m)).astype(np.float32).astype(np.float64)
    Z, b = ff.chebyshev_apply(ctx, c.n, A.row_ptr, A.col, A.H, A.M, A.hm32, dev(R, torch.float32), degree=degree,
                              values=values, upper=upper)
    assert b == upper
    ref, share = _scaled_reference(oracle, P, R, degree, upper, values)
    err = np.linalg.norm(host(Z).astype(np.float64) - ref, axis=0) / np.linalg.norm(ref, axis=0)
    print(f"\n[chebyshev] degree {degree} values {values}: max column error {err.max():.2e}, "
          f"smallest increment share {share:.3g}")
    assert err.max() <= TOL[values], err.max()
    assert share >= 2 * TOL[values]


@pytest.mark.parametrize("values", [1, 3, 4])
def test_chebyshev_apply_block64(cloud, oracle, ctx, ff, values):
    """Block width 64 (the matrix-core steps' other width: two tiles per workgroup from the
    zero-free K-blocks, with values 4), degree 12."""
    c, P, A, upper = cloud
    R = np.random.default_rng(64 + values).standard_normal((c.n, 64)).astype(np.float32).astype(np.float64)
    Z, b = ff.chebyshev_apply(ctx, c.n, A.row_ptr, A.col, A.H, A.M, A.hm32, dev(R, torch.float32), degree=12,
                              values=values, upper=upper)
    ref, share = _scaled_reference(oracle, P, R, 12, upper, values)
    err = np.linalg.norm(host(Z).astype(np.float64) - ref, axis=0) / np.linalg.norm(ref, axis=0)
    assert err.max() <= TOL[values], err.max()
    assert share >= 2 * TOL[values]


def test_chebyshev_interval_estimate(cloud, oracle, ctx, ff):
    """With upper = 0 the library takes min(1.1 x the Rayleigh quotient after 30 power steps,
    the Gershgorin bound): at least the top of D^-1 H's spectrum (the oracle's ARPACK value)
    up to the power method's shortfall, and at most 1.1 times it."""
    c, P, A, upper = cloud
    top = upper / 1.05
    R = np.random.default_rng(5).standard_normal((c.n, 32)).astype(np.float32)
    for values in (1, 4):
        _, b = ff.chebyshev_apply(ctx, c.n, A.row_ptr, A.col, A.H, A.M, A.hm32, dev(R, torch.float32), degree=12,
                                  values=values)
        assert 0.98 * top <= b <= 1.1 * top * (1 + 1e-3), (values, b, top)


def test_chebyshev_apply_validates(cloud, ctx, ff):
    c, P, A, upper = cloud
    R = dev(np.zeros((c.n, 32)), torch.float32)
    for kw in (dict(degree=1), dict(degree=17), dict(values=0), dict(values=5), dict(upper=-1.0)):
        with pytest.raises(ff.FFError):
            ff.chebyshev_apply(ctx, c.n, A.row_ptr, A.col, A.H, A.M, A.hm32, R, **kw)
    with pytest.raises(ff.FFError):
        ff.chebyshev_apply(ctx, c.n, A.row_ptr, A.col, A.H, A.M, A.hm32, R[:, :24].contiguous(), values=3)
    with pytest.raises(ff.FFError):
        ff.chebyshev_apply(ctx, c.n, A.row_ptr, A.col, A.H, A.M, A.hm32, R.double())


def test_chebyshev_shape_override(cloud, ctx, ff, monkeypatch):
    """FF_CHEB_SHAPE (read at context creation) runs the matrix-core steps in another launch shape:
    every shape sums alike, so the result is bitwise the default's; a shape of the other K-block
    form is refused."""
    c, P, A, upper = cloud
    R = dev(np.random.default_rng(7).standard_normal((c.n, 32)), torch.float32)
    Z0, _ = ff.chebyshev_apply(ctx, c.n, A.row_ptr, A.col, A.H, A.M, A.hm32, R, degree=12, values=4, upper=upper)
    monkeypatch.setenv("FF_CHEB_SHAPE", "11")
    c11 = ff.Context(0)
    try:
        Z1, _ = ff.chebyshev_apply(c11, c.n, A.row_ptr, A.col, A.H, A.M, A.hm32, R, degree=12, values=4, upper=upper)
        assert torch.equal(Z0, Z1)
    finally:
        c11.close()
    monkeypatch.setenv("FF_CHEB_SHAPE", "3")
    c3 = ff.Context(0)
    try:
        with pytest.raises(ff.FFError):
            ff.chebyshev_apply(c3, c.n, A.row_ptr, A.col, A.H, A.M, A.hm32, R, degree=12, values=4, upper=upper)
    finally:
        c3.close()
