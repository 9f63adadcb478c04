"""GPU parity of the eigensolver's dense stages (Gram products, Rayleigh-Ritz) against numpy/LAPACK."""
import numpy as np
import pytest

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


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("n,w", [(5, 8), (64, 16), (1000, 24), (4099, 48), (3001, 96), (2500, 130), (777, 192)])
def test_gram(ctx, ff, dtype, n, w):
    rng = np.random.default_rng(n + w)
    S = rng.standard_normal((n, w))
    HS = rng.standard_normal((n, w))
    MS = rng.standard_normal((n, w))
    dt = torch.float32 if dtype == "f32" else torch.float64
    if dtype == "f32":
        S, HS, MS = (a.astype(np.float32).astype(np.float64) for a in (S, HS, MS))
    t = lambda a: torch.as_tensor(a, dtype=dt, device="cuda")
    G = ff.gram_hm(ctx, t(S), t(HS), t(MS)).cpu().numpy()
    refH, refM = S.T @ HS, S.T @ MS
    bound = np.abs(S).T @ np.abs(HS)
    tol = 1e-6 if dtype == "f32" else 1e-14
    assert np.all(np.abs(G[0] - refH) <= tol * bound + 1e-300)
    assert np.all(np.abs(G[1] - refM) <= tol * (np.abs(S).T @ np.abs(MS)) + 1e-300)


@pytest.mark.parametrize("w,m", [(8, 8), (16, 8), (24, 8), (48, 16), (96, 32), (64, 32), (192, 64), (120, 40)])
def test_rayleigh_ritz(ctx, ff, w, m):
    import scipy.linalg as sl
    rng = np.random.default_rng(w * 7 + m)
    B = rng.standard_normal((w, w))
    GM = B @ B.T + w * np.eye(w)
    D = np.exp(rng.uniform(-3, 3, size=w))          # badly scaled columns
    GM = GM * D[:, None] * D[None, :]
    A = rng.standard_normal((w, w))
    GH = (A + A.T) * D[:, None] * D[None, :]
    G = torch.as_tensor(np.stack([GH, GM]), device="cuda")
    theta, C, kept = ff.rayleigh_ritz(ctx, G, m)
    theta, C = theta.cpu().numpy(), C.cpu().numpy()
    ref = sl.eigh(GH, GM, eigvals_only=True)[:m]
    assert kept == w
    scale = np.abs(ref).max()
    assert np.abs(theta - ref).max() <= 1e-10 * scale
    assert np.abs(C.T @ GM @ C - np.eye(m)).max() <= 1e-10
    assert np.abs(C.T @ GH @ C - np.diag(theta)).max() <= 1e-10 * scale


def test_rayleigh_ritz_drops_dependent_columns(ctx, ff):
    import scipy.linalg as sl
    rng = np.random.default_rng(5)
    n, w, m = 200, 24, 8
    S = rng.standard_normal((n, w))
    S[:, 20] = S[:, 3] + S[:, 9]                    # exactly dependent directions
    S[:, 21] = 2.0 * S[:, 10]
    K = rng.standard_normal((n, n))
    Hm = K @ K.T
    GH, GM = S.T @ Hm @ S, S.T @ S
    G = torch.as_tensor(np.stack([GH, GM]), device="cuda")
    theta, C, kept = ff.rayleigh_ritz(ctx, G, m, tau=1e-12)
    assert kept == w - 2
    keep = [j for j in range(w) if j not in (20, 21)]
    ref = sl.eigh(GH[np.ix_(keep, keep)], GM[np.ix_(keep, keep)], eigvals_only=True)[:m]
    assert np.abs(theta.cpu().numpy() - ref).max() <= 1e-8 * np.abs(ref).max()
