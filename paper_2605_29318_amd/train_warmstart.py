"""Train the warm-start network on seeded ellipsoid-union shapes and evaluate it
on held-out shapes: LOBPCG iterations and seconds to residual tol from the
network's block against a random block, on the same GPU.

    python -m paper_2605_29318_amd.train_warmstart --train 48 --test 6 \
        --train-n 20000 40000 --test-n 100000 100000 --k 32 --freq 6 --out weights.npy

The full workload trains on 512 shapes of 20,000-100,000 particles and tests on
100 shapes of 100,000-500,000 (--train 512 --train-n 20000 100000 --test 100
--test-n 100000 500000). Shapes are homogeneous (one E per shape): the inputs
carry no material, and homogeneous modes do not depend on E. Prints one JSON
line per held-out shape and a summary line.
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np

from . import freeform as ff
from . import synth
from . import warmstart as ws


def _log(msg: str):
    print(msg, flush=True)


def _make_shape(args):
    n, seed, k = args
    return synth.ellipsoid_union(n=n, seed=seed, hetero=False, k=k, mc_samples=400_000)


def _shapes(count: int, nmin: int, nmax: int, seed0: int, rng, k: int, workers: int = 1):
    """Shapes j = 0 .. count - 1 (particle counts log-uniform in [nmin, nmax], seed seed0 + j); with
    workers > 1 built ahead in freshly started worker processes (each shape from its own seed, so
    the same shapes), yielded in order."""
    jobs = [(int(round(math.exp(rng.uniform(math.log(nmin), math.log(nmax))))), seed0 + j, k) for j in range(count)]
    if workers <= 1:
        for j, a in enumerate(jobs):
            yield j, _make_shape(a)
        return
    import multiprocessing as mp
    with mp.get_context("spawn").Pool(min(workers, count)) as pool:
        for j, c in enumerate(pool.imap(_make_shape, jobs, chunksize=1)):
            yield j, c


def _ci95(x):
    """Mean and the half-width of its 95% confidence interval (normal approximation)."""
    x = np.asarray(x, dtype=np.float64)
    if x.size < 2:
        return float(x.mean()) if x.size else float("nan"), float("nan")
    return float(x.mean()), float(1.96 * x.std(ddof=1) / math.sqrt(x.size))


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--train", type=int, default=48)
    ap.add_argument("--test", type=int, default=6)
    ap.add_argument("--train-n", type=int, nargs=2, default=[20000, 40000])
    ap.add_argument("--test-n", type=int, nargs=2, default=[100000, 100000])
    ap.add_argument("--k", type=int, default=32)
    ap.add_argument("--freq", type=int, default=ws.DEFAULT_FREQ)
    ap.add_argument("--epochs", type=int, default=100)
    ap.add_argument("--lr", type=float, default=3e-3)
    ap.add_argument("--lr-final", type=float, default=3e-4)
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--precision", type=int, nargs="+", default=[1, 0])
    ap.add_argument("--precond", type=int, nargs="+", default=[2, 1],
                    help="preconditioners to evaluate (2 Chebyshev-Jacobi, 1 Jacobi)")
    ap.add_argument("--random-weight", type=float, nargs="+", default=[3.0, 0.0],
                    help="random_weight of warm_block per preconditioner in --precond order")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--out", type=str, default=None, help="save the FP32 parameters (.npy)")
    ap.add_argument("--workers", type=int, default=1, help="worker processes building the shapes")
    a = ap.parse_args(argv)

    import torch
    if not torch.cuda.is_available():
        _log("no GPU: the warm start trains and runs only on the device")
        return 2
    ctx = ff.Context(0)
    k = a.k
    rng = np.random.default_rng(a.seed)
    t0 = time.time()
    train = []
    for j, c in _shapes(a.train, a.train_n[0], a.train_n[1], 10_000, rng, k, a.workers):
        try:
            s = ws.with_targets(ctx, ws.prepare(ctx, c, n_freq=a.freq), k, tol=a.tol)
        except ff.FFError as e:            # e.g. a thin part sampled too sparsely for the kernel support
            _log(f"train shape {j}: skipped ({e})")
            continue
        s.A = None                         # training reads only the inputs, lumped mass and targets
        train.append(s)
        _log(f"train shape {j}: n={s.n} iters={s.info['iters_fp32']}+{s.info['iters_fp64']} "
             f"({time.time() - t0:.1f} s)")
    t1 = time.time()
    net = ws.train(ctx, train, k, a.epochs, lr=a.lr, lr_final=a.lr_final, seed=a.seed,
                   log=lambda m: _log(m) if int(m.split()[1].split("/")[0]) % 10 == 0 else None)
    torch.cuda.synchronize()
    train_s = time.time() - t1
    if a.out:
        np.save(a.out, net.get_params(), allow_pickle=False)
    rows = []
    for j, c in _shapes(a.test, a.test_n[0], a.test_n[1], 90_000, rng, k, a.workers):
        try:
            s = ws.prepare(ctx, c, n_freq=a.freq)
        except ff.FFError as e:
            _log(f"test shape {j}: skipped ({e})")
            continue
        m = ((k + 7) // 8) * 8
        row = dict(shape=j, n=s.n)
        for prec in a.precision:
            for ip, pc in enumerate(a.precond):
                key = f"p{prec}c{pc}"
                rw = a.random_weight[ip] if ip < len(a.random_weight) else 0.0
                for mode in ("random", "warm"):
                    X0, used = ws.warm_block(ctx, net if mode == "warm" else None, s, m, seed=a.seed + 1,
                                             random_weight=rw)
                    lam, W, info = ws.solve(ctx, s, k, X0=X0, precision=prec, tol=a.tol, precond=pc)
                    row[f"{key}_{mode}"] = dict(iters=info["iters_fp32"] + info["iters_fp64"],
                                                seconds=round(info["seconds"], 3), converged=info["converged"],
                                                used_network=used, max_resid=info["max_resid"])
                    if mode == "random":
                        lam_r = lam
                    else:
                        row[f"{key}_dlam"] = float(np.abs(lam[1:] - lam_r[1:]).max() / np.abs(lam_r[1:]).max())
        rows.append(row)
        _log(json.dumps(row))
    summ = dict(train_shapes=len(train), train_n=a.train_n, test_n=a.test_n, train_seconds=round(train_s, 2), k=k,
                freq=a.freq, epochs=a.epochs, random_weight=a.random_weight, precond=a.precond)
    for prec in a.precision:
        for pc in a.precond:
            key = f"p{prec}c{pc}"
            r = [x[f"{key}_random"]["iters"] for x in rows]
            w = [x[f"{key}_warm"]["iters"] for x in rows]
            rs = [x[f"{key}_random"]["seconds"] for x in rows]
            wsec = [x[f"{key}_warm"]["seconds"] for x in rows]
            ratio, ci = _ci95(np.array(w) / np.array(r))
            sratio, sci = _ci95(np.array(wsec) / np.array(rs))
            summ[key] = dict(shapes=len(rows), iters_random=float(np.mean(r)), iters_warm=float(np.mean(w)),
                             seconds_random=float(np.mean(rs)), seconds_warm=float(np.mean(wsec)),
                             iter_ratio=ratio, iter_ratio_ci95=ci, seconds_ratio=sratio, seconds_ratio_ci95=sci,
                             used_network=sum(x[f"{key}_warm"]["used_network"] for x in rows))
    _log("SUMMARY " + json.dumps(summ))
    net.close()
    ctx.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
