"""GPU tests of the warm-start network through the C ABI against the FP64
reference in oracle/mlp.py.

Tolerances: the GPU network stores weights and hidden activations in BF16
(unit roundoff 2^-9 after round-to-nearest-even) and accumulates in FP32, so
with BF16-representable parameters the output carries about three BF16
roundings: relative Frobenius error <= 2e-2. Gradients go through the same
roundings plus the FP32 loss algebra: cosine similarity with the FP64
gradient >= 0.999. The features and inputs are FP32 results of FP64 sums:
relative 2e-6.
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


@pytest.fixture(scope="module")
def R():
    from oracle import mlp
    return mlp


def dev(a, dt=None):
    t = torch.as_tensor(np.ascontiguousarray(a), device="cuda")
    return t if dt is None else t.to(dt)


def bf16_round(a):
    """Round FP32 values to the nearest BF16 (ties to even), kept in FP32."""
    u = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32)


def _problem(R, n, k, seed, n_in=11):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n, n_in)).astype(np.float32)
    T = np.linalg.qr(rng.standard_normal((n, k)))[0]
    d = rng.uniform(0.5, 2.0, size=n)
    p = bf16_round(R.init_params(k, seed=seed, n_in=n_in)).astype(np.float64)
    return X, T, d, p


@pytest.mark.parametrize("name", ["cube1k", "spheres4k"])
def test_features_match_oracle(oracle, R, ctx, ff, name):
    c = synth.cube_lattice() if name == "cube1k" else synth.sphere_union(n=4000, seed=2, mc_samples=200_000)
    P = oracle.pipeline(c)
    ref = R.rkpm_features(P.xyz, P.xyz, P.nbr_off, P.nbr_id, c.h)
    A = ff.assemble_cloud(ctx, dev(c.xyz), dev(c.vol), dev(c.lam), dev(c.mu), c.h, features=True)
    f = A.feat.cpu().numpy().astype(np.float64)
    assert np.array_equal(f[:, 4], ref[:, 4])
    err = np.abs(f - ref) / np.maximum(np.abs(ref), 1e-3)
    assert err.max() <= 2e-6, (err.max(axis=0))


@pytest.mark.parametrize("n_freq", [0, 6, 19])
def test_inputs_match_oracle(oracle, R, ctx, ff, n_freq):
    c = synth.sphere_union(n=4000, seed=2, mc_samples=200_000)
    P = oracle.pipeline(c)
    feat = R.rkpm_features(P.xyz, P.xyz, P.nbr_off, P.nbr_id, c.h).astype(np.float32)
    ref = R.inputs(P.xyz, feat.astype(np.float64), n_freq=n_freq)
    got = ff.mlp_inputs(ctx, dev(P.xyz), dev(feat), n_freq=n_freq).cpu().numpy()
    assert got.shape == ref.shape
    # FP32 results; the highest octave (2^18 pi x) also carries the FP64 rounding of x times 2^18
    tol = 2e-6 * max(1.0, np.abs(ref[:, :11]).max()) + (2.0 ** max(0, n_freq - 1) * np.pi * 4e-16 if n_freq else 0)
    assert np.abs(got - ref).max() <= tol


def test_lumped_mass_is_row_sum(oracle, ctx, ff):
    c = synth.random_cloud(1500, seed=8)
    P = oracle.pipeline(c)
    A = ff.assemble_cloud(ctx, dev(c.xyz), dev(c.vol), dev(c.lam), dev(c.mu), c.h)
    d = ff.lumped_mass(ctx, A.n, A.row_ptr, A.M).cpu().numpy()
    ref = np.asarray(P.Ms().sum(axis=1)).ravel()
    assert np.abs(d - ref).max() <= 1e-13 * np.abs(ref).max()


@pytest.mark.parametrize("n,k,n_in", [(1037, 8, 11), (1037, 24, 11), (64, 32, 11), (2500, 64, 11), (1037, 32, 47),
                                      (300, 16, 128)])
def test_forward_matches_oracle(R, ctx, ff, n, k, n_in):
    X, T, d, p = _problem(R, n, k, seed=n + k, n_in=n_in)
    net = ff.MLP(ctx, k, n_in=n_in, seed=0)
    net.set_params(p.astype(np.float32))
    assert np.array_equal(net.get_params(), p.astype(np.float32))
    ld = k + 3
    Y = net.forward(dev(X), ldy=ld).cpu().numpy()
    ref = R.forward(p, X.astype(np.float64), k)
    assert np.linalg.norm(Y[:, :k] - ref) <= 2e-2 * np.linalg.norm(ref)
    assert np.all(Y[:, k:] == 0.0)          # columns beyond k untouched
    net.close()


@pytest.mark.parametrize("n,k,n_in", [(1037, 8, 11), (3000, 32, 11), (2000, 16, 47)])
def test_gradient_matches_oracle(R, ctx, ff, n, k, n_in):
    X, T, d, p = _problem(R, n, k, seed=7 * n + k, n_in=n_in)
    net = ff.MLP(ctx, k, n_in=n_in, seed=0)
    net.set_params(p.astype(np.float32))
    loss = net.train_step(dev(X), dev(T), dev(d), 0.0)
    g = net.get_grad().astype(np.float64)
    L_ref, g_ref = R.loss_and_grad(p, X.astype(np.float64), T, d, k)
    assert abs(loss - L_ref) <= 2e-2 * max(1.0, L_ref)
    cos = g @ g_ref / (np.linalg.norm(g) * np.linalg.norm(g_ref))
    assert cos >= 0.999, cos
    # with lr = 0 the parameters stay as they were
    assert np.array_equal(net.get_params(), p.astype(np.float32))
    net.close()


def test_adam_first_step(R, ctx, ff):
    """The first Adam step moves each parameter by lr * g / (|g| + eps): lr against
    the sign of its gradient, as the FP64 reference does."""
    n, k, lr = 1500, 16, 1e-3
    X, T, d, p = _problem(R, n, k, seed=11)
    net = ff.MLP(ctx, k, seed=0)
    net.set_params(p.astype(np.float32))
    net.train_step(dev(X), dev(T), dev(d), lr)
    p1 = net.get_params().astype(np.float64)
    _, g_ref = R.loss_and_grad(p, X.astype(np.float64), T, d, k)
    ref = R.adam_step(p, g_ref, np.zeros_like(p), np.zeros_like(p), 1, lr=lr)[0]
    big = np.abs(g_ref) > 1e-2 * np.abs(g_ref).max()
    assert big.sum() > 1000
    assert np.abs((p1 - p)[big] - (ref - p)[big]).max() <= 1e-2 * lr
    net.close()


def test_training_lowers_the_loss(R, ctx, ff):
    n, k = 4000, 16
    X, T, d, p = _problem(R, n, k, seed=5)
    # targets that the network can represent: smooth functions of the inputs
    Xf = X.astype(np.float64)
    T = np.linalg.qr(np.hstack([np.ones((n, 1)), Xf[:, :3], np.sin(Xf), Xf[:, :1] * Xf[:, 1:2]]))[0]
    assert T.shape == (n, k)
    net = ff.MLP(ctx, k, seed=3)
    Xd, Td, dd = dev(X), dev(T), dev(d)
    losses = [net.train_step(Xd, Td, dd, 3e-3) for _ in range(150)]
    assert losses[-1] < 0.3 * losses[0], (losses[0], losses[-1])
    net.close()


def test_mlp_rejects_bad_arguments(ctx, ff):
    with pytest.raises(ff.FFError):
        ff.MLP(ctx, 65)
    net = ff.MLP(ctx, 8)
    X = torch.zeros((4, 11), dtype=torch.float32, device="cuda")
    T = torch.zeros((4, 8), dtype=torch.float64, device="cuda")
    d = torch.ones(4, dtype=torch.float64, device="cuda")
    with pytest.raises(ff.FFError) as ei:
        net.train_step(X, T, d, 1e-3)          # n < k
    assert ei.value.code == ff.FF_ERR_INVALID_ARG
    net.close()


@pytest.mark.parametrize("n,m,w", [(1, 1, 3.0), (1037, 8, 3.0), (5000, 32, 1.0), (70000, 33, 0.0), (3001, 64, 2.5)])
def test_block_blend(ctx, ff, R, n, m, w):
    """The warm start's column blend in the library against the FP64 reference: FP64 sums
    (chunk partials added in a fixed order), 1e-13 relative; a strided X, and the argument checks."""
    rng = np.random.default_rng(n + m)
    X = rng.standard_normal((n, m)) * rng.uniform(0.1, 10.0, m)
    Rb = rng.uniform(-1.0, 1.0, (n, m))
    ref = R.blend(X, Rb, w)
    Xd = dev(X)
    ff.block_blend(ctx, Xd, dev(Rb), w)
    assert np.abs(Xd.cpu().numpy() - ref).max() <= 1e-13 * np.abs(ref).max()
    wide = dev(np.zeros((n, m + 5)))
    wide[:, :m] = dev(X)
    ff.block_blend(ctx, wide[:, :m], dev(Rb), w)
    assert np.abs(wide[:, :m].cpu().numpy() - ref).max() <= 1e-13 * np.abs(ref).max()
    assert np.all(wide[:, m:].cpu().numpy() == 0.0)
    with pytest.raises(ff.FFError):
        ff.block_blend(ctx, dev(X).float(), dev(Rb), w)
    with pytest.raises(ff.FFError):
        ff.block_blend(ctx, dev(X), dev(Rb), -1.0)
