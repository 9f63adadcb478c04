"""Learned warm start of the eigensolver: training data, training and inference.

Everything numeric runs in the library (mlp_inputs, mlp_forward,
mlp_train_step, lumped_mass, eigenmodes, spmm_hm, gram_hm, rayleigh_ritz);
this module only orders the calls. The network is trained on modes that
eigenmodes itself computes for seeded synthetic shapes, and it is judged by
the iterations eigenmodes needs from its block against a random start: the
converged answer is the same either way, only the starting block differs.
"""
from __future__ import annotations

import time
from dataclasses import dataclass
from typing import Callable, List, Optional

import numpy as np

from . import freeform as ff


DEFAULT_FREQ = 6      # octaves of sine/cosine position encoding


@dataclass
class Sample:
    n: int
    A: ff.Assembled
    x: "object"         # [n][11 + 6 n_freq] FP32 network inputs
    d: "object"         # [n] lumped mass
    T: "object"         # [n][k] target modes (M-orthonormal), or None
    lam: Optional[np.ndarray]
    info: Optional[dict]


def prepare(ctx: ff.Context, cloud, n_freq: int = DEFAULT_FREQ, device="cuda") -> Sample:
    """Assemble H, M with the per-point features and build the network inputs."""
    import torch

    def dev(a):
        return torch.as_tensor(np.ascontiguousarray(a), device=device)

    A = ff.assemble_cloud(ctx, dev(cloud.xyz), dev(cloud.vol), dev(cloud.lam), dev(cloud.mu), cloud.h,
                          features=True)
    x = ff.mlp_inputs(ctx, A.nb.xyz_sorted, A.feat, n_freq=n_freq)
    d = ff.lumped_mass(ctx, A.n, A.row_ptr, A.M)
    return Sample(A.n, A, x, d, None, None, None)


def solve(ctx: ff.Context, s: Sample, k: int, X0=None, precision: int = 1, tol: float = 1e-6,
          max_iter: int = 20000, seed: int = 0, precond: int = 2):
    """eigenmodes on a prepared sample; returns (lam, W, info)."""
    A = s.A
    lam, W, res, info = ff.eigenmodes(ctx, A.n, A.row_ptr, A.col, A.H, A.M, A.hm32, k=k, precision=precision,
                                      tol=tol, max_iter=max_iter, X0=X0, seed=seed, allow_unconverged=True,
                                      precond=precond)
    return lam, W, info


def with_targets(ctx: ff.Context, s: Sample, k: int, tol: float = 1e-6, precision: int = 1) -> Sample:
    lam, W, info = solve(ctx, s, k, precision=precision, tol=tol)
    s.T, s.lam, s.info = W, lam, info
    return s


def train(ctx: ff.Context, samples: List[Sample], k: int, epochs: int, lr: float = 1e-3, seed: int = 0,
          lr_final: float = 1e-4, log: Optional[Callable[[str], None]] = None) -> ff.MLP:
    """Adam over the samples in a seeded shuffled order each epoch, one step per
    sample; the step size decays geometrically from lr to lr_final."""
    net = ff.MLP(ctx, k, n_in=samples[0].x.shape[1], seed=seed)
    rng = np.random.default_rng(seed)
    total = epochs * len(samples)
    step = 0
    t0 = time.time()
    for ep in range(epochs):
        losses = []
        for j in rng.permutation(len(samples)):
            s = samples[j]
            a = lr * (lr_final / lr) ** (step / max(1, total - 1))
            losses.append(net.train_step(s.x, s.T, s.d, a))
            step += 1
        if log:
            log(f"epoch {ep + 1}/{epochs} mean loss {np.mean(losses):.4f} ({time.time() - t0:.1f} s)")
    return net


def ritz_sum(ctx: ff.Context, s: Sample, X) -> float:
    """Sum of the Ritz values of (H, M) on span(X): tr((X^T M X)^-1 X^T H X)."""
    A = s.A
    HX, MX = ff.spmm_hm(ctx, A.row_ptr, A.col, A.H, A.M, A.hm32, X, precision=0)
    G = ff.gram_hm(ctx, X, HX, MX)
    theta, C, kept = ff.rayleigh_ritz(ctx, G, X.shape[1])
    return float(theta.sum().item())


def warm_block(ctx: ff.Context, net: Optional[ff.MLP], s: Sample, block: int, seed: int = 0,
               fallback: bool = True, random_weight: float = 0.0):
    """Starting block [n][block]: the network's k columns, random columns
    (rand_block, seed) beyond k. With random_weight w > 0 every column is
    X/rms(X) + w R/rms(R): a strong preconditioner needs the start to keep a
    component along every mode, which the network's columns alone may lack
    (measured with Chebyshev-Jacobi: w = 0 costs 1.29x the iterations of a
    random start, w = 3 saves 2.6%; with Jacobi w = 0 is best). Returns (X0,
    used_network). Falls back to the random block when there is no network,
    when its block is rank deficient, or when its Ritz-value sum exceeds that
    of the random block."""
    R = ff.rand_block(ctx, s.n, block, seed)
    if net is None:
        return R, False
    X = R.clone()
    net.forward(s.x, out=X)        # writes the first k columns
    if random_weight > 0.0:
        ff.block_blend(ctx, X, R, random_weight)
    if not fallback:
        return X, True
    try:
        warm = ritz_sum(ctx, s, X)
    except ff.FFError:
        return R, False
    cold = ritz_sum(ctx, s, R)
    return (X, True) if warm <= cold else (R, False)
