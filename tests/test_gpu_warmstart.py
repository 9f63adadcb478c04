"""End-to-end test of the learned warm start on the GPU: the network is trained
by the library's own kernels on modes that eigenmodes computes for seeded
ellipsoid-union shapes, then starts eigenmodes on held-out shapes.

The converged answer is the reference: from the network's block the solver must
reach the same eigenpairs (eigenvalues against a tight FP64 solve, within the
error the residual tolerance allows) and the residual tolerance itself. The
gain is the number of iterations against a random start on the same shapes.
"""
import numpy as np
import pytest

from paper_2605_29318_amd import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

K = 16


@pytest.fixture(scope="module")
def env():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2605_29318_amd import freeform as ff, warmstart as ws
    ctx = ff.Context(0)
    train = []
    for j in range(12):
        c = synth.ellipsoid_union(n=10000, seed=700 + j, hetero=False, k=K, mc_samples=200_000)
        try:
            train.append(ws.with_targets(ctx, ws.prepare(ctx, c), K, tol=1e-6))
        except ff.FFError:
            continue
    assert len(train) >= 8
    log = []
    net = ws.train(ctx, train, K, 60, lr=3e-3, lr_final=3e-4, log=log.append)
    tests = [ws.prepare(ctx, synth.ellipsoid_union(n=40000, seed=800 + j, hetero=False, k=K, mc_samples=200_000))
             for j in range(3)]
    yield ff, ws, ctx, net, train, tests, log
    net.close()
    ctx.close()


def test_training_lowers_the_loss(env):
    ff, ws, ctx, net, train, tests, log = env
    first = float(log[0].split("loss")[1].split()[0])
    last = float(log[-1].split("loss")[1].split()[0])
    assert last < first - 0.5, (first, last)


def _ratios(env, precond, random_weight=0.0):
    ff, ws, ctx, net, train, tests, log = env
    m = K
    ratios = []
    for s in tests:
        ref, _, rinfo = ws.solve(ctx, s, K, precision=0, tol=1e-9, seed=5)
        assert rinfo["converged"] == 1
        its = {}
        for mode in ("random", "warm"):
            X0, used = ws.warm_block(ctx, net if mode == "warm" else None, s, m, seed=1, fallback=False,
                                     random_weight=random_weight)
            lam, W, info = ws.solve(ctx, s, K, X0=X0, precision=1, tol=1e-6, precond=precond)
            assert info["converged"] == 1 and info["max_resid"] <= 1e-6
            # Ritz values bound the eigenvalues from above; residual 1e-6 allowed at most 1.1e-4 of lambda_max on these shapes
            assert np.all(lam[1:] >= ref[1:] * (1 - 1e-7))
            print("max eigenvalue excess", mode, np.abs(lam[1:] - ref[1:]).max() / ref[1:].max())
            assert np.abs(lam[1:] - ref[1:]).max() <= 1e-3 * ref[1:].max()
            its[mode] = info["iters_fp32"] + info["iters_fp64"]
        ratios.append(its["warm"] / its["random"])
    print("precond", precond, "warm/random iteration ratios", ratios)
    return ratios


def test_warm_start_reaches_the_same_eigenpairs_in_fewer_iterations(env):
    """With the Jacobi preconditioner (several hundred iterations from a random start)
    the network's block saves iterations."""
    ratios = _ratios(env, precond=1)
    assert np.mean(ratios) < 1.0, ratios


def test_warm_start_with_chebyshev_preconditioner(env):
    """With the default Chebyshev-Jacobi preconditioner (a few dozen iterations from any start)
    the network's block alone costs iterations (mean ratio 1.29 on these shapes: it lacks a
    component along some wanted mode, which the strong preconditioner cannot grow quickly);
    blended with random columns of three times its RMS it reaches the same eigenpairs, and at
    the large configuration's scale (512 training shapes, 100 held-out shapes of 1e5-5e5
    particles) its iteration ratio is 0.995 +- 0.039 (95% interval): no measurable gain and no
    loss. The test checks the same eigenpairs and no loss beyond that interval on its shapes."""
    ratios = _ratios(env, precond=2, random_weight=3.0)
    mean = float(np.mean(ratios))
    half = 1.96 * float(np.std(ratios, ddof=1)) / np.sqrt(len(ratios))
    print(f"chebyshev: warm/random iteration ratio {mean:.3f} +- {half:.3f} over {len(ratios)} shapes")
    assert mean <= 1.1, ratios


def test_fallback_keeps_the_block_with_the_lower_ritz_sum(env):
    ff, ws, ctx, net, train, tests, log = env
    s = tests[0]
    X0, used = ws.warm_block(ctx, net, s, K, seed=1, fallback=True)
    R = ff.rand_block(ctx, s.n, K, 1)
    Xw, _ = ws.warm_block(ctx, net, s, K, seed=1, fallback=False)
    rw, rr = ws.ritz_sum(ctx, s, Xw), ws.ritz_sum(ctx, s, R)
    assert used == (rw <= rr)
    assert torch.equal(X0, Xw if used else R)
    Xn, used_n = ws.warm_block(ctx, None, s, K, seed=1)
    assert not used_n and torch.equal(Xn, R)
