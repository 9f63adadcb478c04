"""rayleigh_ritz_noalloc (fixed per-GPU scratch, no device allocation) against rayleigh_ritz,
through the C ABI: the same kernels on the same pencil give the same eigenvalues and
coefficients bit for bit, on two calls in a row (the second smaller, so the scratch holds
the first call's larger contents), and sizes beyond the scratch are refused."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _pencil(w, seed):
    rng = np.random.default_rng(seed)
    B = rng.standard_normal((w, w))
    D = np.exp(rng.uniform(-3, 3, size=w))
    GM = (B @ B.T + w * np.eye(w)) * D[:, None] * D[None, :]
    A = rng.standard_normal((w, w))
    GH = (A + A.T) * D[:, None] * D[None, :]
    return np.stack([GH, GM])


def _call(ff, ctx, name, G, m, tau=1e-13):
    w = G.shape[1]
    C = torch.full((w, m), np.nan, dtype=torch.float64, device="cuda")
    theta = torch.full((m,), np.nan, dtype=torch.float64, device="cuda")
    kept = ctypes.c_int(-1)
    rc = getattr(ff.lib(), name)(ctx.h, w, m, ff._p(G), tau, ff._p(C), ff._p(theta), ctypes.byref(kept))
    return rc, C.cpu().numpy(), theta.cpu().numpy(), kept.value


def test_noalloc_matches_rayleigh_ritz():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import scipy.linalg as sl
    from paper_2605_29318_amd import freeform as ff
    ctx = ff.Context(0)
    try:
        for w, m, seed in ((192, 64, 1), (48, 16, 2)):
            Gh = _pencil(w, seed)
            G = torch.as_tensor(Gh, device="cuda")
            rc0, C0, th0, k0 = _call(ff, ctx, "rayleigh_ritz", G, m)
            rc1, C1, th1, k1 = _call(ff, ctx, "rayleigh_ritz_noalloc", G, m)
            assert rc0 == 0 and rc1 == 0, ff.lib().ff_last_error(ctx.h)
            assert k0 == k1 == w
            assert np.array_equal(th0, th1) and np.array_equal(C0, C1)
            ref = sl.eigh(Gh[0], Gh[1], eigvals_only=True)[:m]
            assert np.abs(th1 - ref).max() <= 1e-10 * np.abs(ref).max()
            assert np.abs(C1.T @ Gh[1] @ C1 - np.eye(m)).max() <= 1e-10
        G = torch.as_tensor(_pencil(8, 3), device="cuda")
        for w, m in ((193, 8), (192, 65)):
            Gb = torch.zeros((2, w, w), dtype=torch.float64, device="cuda")
            rc, _, _, _ = _call(ff, ctx, "rayleigh_ritz_noalloc", Gb, m)
            assert rc == ff.FF_ERR_INVALID_ARG
            assert b"fixed scratch" in ff.lib().ff_last_error(ctx.h)
    finally:
        ctx.close()
