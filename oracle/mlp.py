"""FP64 reference of the learned warm start (not part of the paper: the paper's
only MLP is the Simplicits baseline).

TEST INFRASTRUCTURE ONLY: used by the tests to check the GPU network's forward
pass and gradients; the product path never imports it.

Network: n_in -> 128 -> 128 -> 128 -> k, GELU(z) = z * Phi(z) (exact erf
form) after the three hidden layers; n_in = 11 + 6 F for the 11 base inputs and
F octaves of sine/cosine position encoding (see inputs). Parameters are laid
out flat as [W1 (128 x n_in), b1, W2 (128x128), b2, W3 (128x128), b3,
W4 (k x 128), b4], each W stored output-major (row = output unit).

Loss for one shape with lumped mass D = diag(M 1) and target modes T (n x k):
    A = Y^T D Y,  B = Y^T D T,  E = (T^T D T)^-1
    L = k - tr(A^-1 B E B^T)
the sum of squared cosines of the principal angles between span(Y) and
span(T) in the D inner product, subtracted from k: invariant to any
invertible mixing of the columns of Y or T (signs, rotations, scales).
Gradient: dL/dY = D (T G1 + Y G2), G1 = -2 E B^T A^-1, G2 = 2 A^-1 B E B^T A^-1.
"""
from __future__ import annotations

import math

import numpy as np

HIDDEN = 128
N_IN = 11


def shapes(k, n_in=N_IN):
    return [(HIDDEN, n_in), (HIDDEN,), (HIDDEN, HIDDEN), (HIDDEN,), (HIDDEN, HIDDEN), (HIDDEN,), (k, HIDDEN), (k,)]


def param_count(k, n_in=N_IN):
    return sum(int(np.prod(s)) for s in shapes(k, n_in))


def input_width(p, k):
    """n_in of a flat parameter vector for output width k."""
    rest = len(p) - param_count(k, 0)
    assert rest % HIDDEN == 0
    return rest // HIDDEN


def unpack(p, k):
    out = []
    o = 0
    for s in shapes(k, input_width(p, k)):
        c = int(np.prod(s))
        out.append(np.asarray(p[o:o + c], dtype=np.float64).reshape(s))
        o += c
    return out


def pack(arrs):
    return np.concatenate([np.asarray(a, dtype=np.float64).ravel() for a in arrs])


def init_params(k, seed=0, n_in=N_IN):
    """Uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) weights, zero biases (seeded numpy)."""
    rng = np.random.default_rng(seed)
    arrs = []
    for s in shapes(k, n_in):
        if len(s) == 2:
            b = 1.0 / math.sqrt(s[1])
            arrs.append(rng.uniform(-b, b, size=s))
        else:
            arrs.append(np.zeros(s))
    return pack(arrs)


_SQRT2 = math.sqrt(2.0)
_INV_SQRT2PI = 1.0 / math.sqrt(2.0 * math.pi)


def gelu(z):
    from scipy.special import erf
    return 0.5 * z * (1.0 + erf(z / _SQRT2))


def gelu_grad(z):
    from scipy.special import erf
    return 0.5 * (1.0 + erf(z / _SQRT2)) + z * _INV_SQRT2PI * np.exp(-0.5 * z * z)


def forward(p, X, k, keep=False):
    W1, b1, W2, b2, W3, b3, W4, b4 = unpack(p, k)
    Z1 = X @ W1.T + b1
    A1 = gelu(Z1)
    Z2 = A1 @ W2.T + b2
    A2 = gelu(Z2)
    Z3 = A2 @ W3.T + b3
    A3 = gelu(Z3)
    Y = A3 @ W4.T + b4
    if keep:
        return Y, (X, Z1, A1, Z2, A2, Z3, A3)
    return Y


def subspace_loss(Y, T, d):
    """Returns L and dL/dY (see module docstring)."""
    k = Y.shape[1]
    DY = d[:, None] * Y
    DT = d[:, None] * T
    A = Y.T @ DY
    B = Y.T @ DT
    Cm = T.T @ DT
    Ainv = np.linalg.inv(A)
    E = np.linalg.inv(Cm)
    L = k - np.trace(Ainv @ B @ E @ B.T)
    G1 = -2.0 * E @ B.T @ Ainv
    G2 = 2.0 * Ainv @ B @ E @ B.T @ Ainv
    dY = DT @ G1 + DY @ G2
    return L, dY


def loss_and_grad(p, X, T, d, k):
    Y, (X0, Z1, A1, Z2, A2, Z3, A3) = forward(p, X, k, keep=True)
    L, dY = subspace_loss(Y, T, d)
    W1, b1, W2, b2, W3, b3, W4, b4 = unpack(p, k)
    gW4 = dY.T @ A3
    gb4 = dY.sum(axis=0)
    dZ3 = (dY @ W4) * gelu_grad(Z3)
    gW3 = dZ3.T @ A2
    gb3 = dZ3.sum(axis=0)
    dZ2 = (dZ3 @ W3) * gelu_grad(Z2)
    gW2 = dZ2.T @ A1
    gb2 = dZ2.sum(axis=0)
    dZ1 = (dZ2 @ W2) * gelu_grad(Z1)
    gW1 = dZ1.T @ X0
    gb1 = dZ1.sum(axis=0)
    return L, pack([gW1, gb1, gW2, gb2, gW3, gb3, gW4, gb4])


def adam_step(p, g, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """Adam (Kingma & Ba 2015) with bias correction; returns new p, m, v."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def blend(X, R, w):
    """The warm start's blended starting block: each column of X divided by its root mean
    square, plus w times the matching column of R divided by its own."""
    X = np.asarray(X, dtype=np.float64)
    R = np.asarray(R, dtype=np.float64)
    rms = lambda A: np.sqrt(np.mean(A * A, axis=0))
    return X / rms(X)[None, :] + w * R / rms(R)[None, :]


def inputs(xyz, feat, n_freq=0):
    """The network inputs from positions and the 8 raw RKPM features of rkpm_shape:
    position normalised to [-1, 1]^3 about the box centre by the largest half extent,
    the 4 moment-matrix eigenvalues, neighbour count / mean count, kernel sum / mean
    kernel sum, the boundary indicator and std/mean of the raw kernel values; then for
    each octave l < n_freq, sin(pi 2^l x_a) for a = 0, 1, 2 and cos(pi 2^l x_a) for
    a = 0, 1, 2 of the normalised position x (Fourier features, which let a small
    network represent the sharp variation of low modes across thin necks)."""
    xyz = np.asarray(xyz, dtype=np.float64)
    f = np.asarray(feat, dtype=np.float64)
    lo, hi = xyz.min(axis=0), xyz.max(axis=0)
    c = 0.5 * (lo + hi)
    half = 0.5 * (hi - lo).max()
    pos = (xyz - c) / half
    out = np.empty((xyz.shape[0], 11 + 6 * n_freq))
    out[:, 0:3] = pos
    out[:, 3:7] = f[:, 0:4]
    out[:, 7] = f[:, 4] / f[:, 4].mean()
    out[:, 8] = f[:, 5] / f[:, 5].mean()
    out[:, 9] = f[:, 6]
    out[:, 10] = f[:, 7]
    for l in range(n_freq):
        out[:, 11 + 6 * l: 14 + 6 * l] = np.sin(np.pi * 2.0 ** l * pos)
        out[:, 14 + 6 * l: 17 + 6 * l] = np.cos(np.pi * 2.0 ** l * pos)
    return out


def _raw_kernel(d, h, kernel):
    """Kernel values phi~ of distance d: cubic B-spline of z = d/h with support 1
    (kernel 0), or the Gaussian exp(-d^2/r^2), r = h/2, of Sec. 3.2 (kernel 1)."""
    d = np.asarray(d, dtype=np.float64)
    if kernel == 1:
        return np.where(d < h, np.exp(-(d * d) / (0.25 * h * h)), 0.0)
    z = d / h
    inner = 2.0 / 3.0 - 4.0 * z ** 2 + 4.0 * z ** 3
    outer = 4.0 / 3.0 * (1.0 - z) ** 3
    return np.where(z <= 0.5, inner, np.where(z < 1.0, outer, 0.0))


def rkpm_features(qxyz, xyz_sorted, off, ids, h, kernel=0):
    """The 8 raw per-point features of rkpm_shape, from their definitions, one
    point at a time: with phi~ the kernel values over the neighbour list and
    P = [1, (p - X)/h] the shifted scaled linear basis of Sec. 3.2,
      0-3  eigenvalues (ascending) of sum phi~ P P^T / sum phi~,
      4    neighbour count,
      5    sum phi~,
      6    |sum phi~ (p - X)| / (h sum phi~),
      7    population std / mean of phi~ over the list."""
    q = len(off) - 1
    out = np.zeros((q, 8))
    for i in range(q):
        X = np.asarray(qxyz[i], dtype=np.float64)
        nb = np.asarray(xyz_sorted)[np.asarray(ids[off[i]:off[i + 1]])]
        r = nb - X
        w = _raw_kernel(np.sqrt((r ** 2).sum(axis=1)), h, kernel)
        P = np.hstack([np.ones((len(w), 1)), r / h])
        S = (P * w[:, None]).T @ P
        sw = w.sum()
        out[i, 0:4] = np.linalg.eigvalsh(S / sw)
        out[i, 4] = len(w)
        out[i, 5] = sw
        out[i, 6] = np.linalg.norm((w[:, None] * r).sum(axis=0)) / (h * sw)
        out[i, 7] = w.std() / w.mean()
    return out
