"""Seeded synthetic particle clouds for the subspace-construction path.

This module only builds inputs: particle positions, quadrature volumes, the
support radius and per-point material parameters. It contains none of the
method's arithmetic (no kernel, no shape functions, no assembly, no
eigensolve), so both the CPU oracle and the GPU path can take their inputs
from here.

The paper fits skinning eigenmodes on objects given by an inside/outside test
and sampled by points (Sec. 3, Supp. B.1). Its own datasets (Thingi10K,
Simready, 3DGS scenes) are not available, so these generators stand in for
them with unions of spheres or ellipsoids clipped to the unit box:

* ``cube_lattice``   - jittered 10x10x10 lattice in the unit cube (small case).
* ``sphere_union``   - Poisson-disk samples inside a union of random spheres.
* ``ellipsoid_union``- uniform samples inside a union of random ellipsoids,
                       optionally with heterogeneous per-particle material.
* ``batch_objects``  - many sphere-union objects of log-uniform sizes.

Every generator is deterministic in its seed (numpy ``default_rng``).
"""
from __future__ import annotations

import dataclasses
import hashlib
import math
from typing import List, Optional

import numpy as np


@dataclasses.dataclass
class Cloud:
    """One object: nodes are also the quadrature points (one per particle)."""
    name: str
    xyz: np.ndarray          # (n, 3) float64, original (unsorted) order
    vol: np.ndarray          # (n,) float64 quadrature weight v_i
    lam: np.ndarray          # (n,) float64 Lame lambda
    mu: np.ndarray           # (n,) float64 Lame mu
    rho: np.ndarray          # (n,) float64 density
    h: float                 # kernel support radius
    k: int                   # number of eigenpairs requested (constant mode included)
    seed: int
    meta: dict = dataclasses.field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.xyz.shape[0])

    def sha256(self) -> str:
        m = hashlib.sha256()
        for a in (self.xyz, self.vol, self.lam, self.mu, self.rho):
            m.update(np.ascontiguousarray(a).tobytes())
        m.update(np.float64(self.h).tobytes())
        return m.hexdigest()


def lame_from_young(E, nu):
    """Standard conversion from Young's modulus and Poisson ratio to Lame parameters."""
    E = np.asarray(E, dtype=np.float64)
    nu = np.asarray(nu, dtype=np.float64)
    lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    mu = E / (2.0 * (1.0 + nu))
    return lam, mu


# ----------------------------------------------------------------------------
# small clouds
# ----------------------------------------------------------------------------

def cube_lattice(m: int = 10, spacing: float = 0.1, jitter: float = 0.02, seed: int = 0,
                 E: float = 1e5, nu: float = 0.45, rho: float = 1000.0, k: int = 8,
                 support: float = 2.5) -> Cloud:
    """Jittered m^3 lattice: x = (i + 0.5) * spacing, index (iz*m + iy)*m + ix.

    The default is the 1,000-particle unit-cube case (spacing 0.1, jitter
    U(-0.02, 0.02) per coordinate, h = 2.5 spacing, v = spacing^3).
    """
    rng = np.random.default_rng(seed)
    i = np.arange(m, dtype=np.float64)
    iz, iy, ix = np.meshgrid(i, i, i, indexing="ij")
    base = np.stack([ix.ravel(), iy.ravel(), iz.ravel()], axis=1)
    xyz = (base + 0.5) * spacing
    if jitter > 0:
        xyz = xyz + rng.uniform(-jitter, jitter, size=xyz.shape)
    n = xyz.shape[0]
    lam, mu = lame_from_young(np.full(n, E), np.full(n, nu))
    return Cloud(name=f"cube{m}", xyz=np.ascontiguousarray(xyz), vol=np.full(n, spacing ** 3),
                 lam=lam, mu=mu, rho=np.full(n, rho), h=support * spacing, k=k, seed=seed,
                 meta=dict(spacing=spacing, jitter=jitter, E=E, nu=nu))


def random_cloud(n: int, seed: int, box: float = 1.0, support_factor: float = 2.5,
                 hetero: bool = False, k: int = 8) -> Cloud:
    """Uniform random points in a box (tiny cases for brute-force checks)."""
    rng = np.random.default_rng(seed)
    xyz = rng.uniform(0.0, box, size=(n, 3))
    s = box / n ** (1.0 / 3.0)
    if hetero:
        E = np.exp(rng.uniform(math.log(1e4), math.log(1e6), size=n))
        nu = rng.uniform(0.3, 0.48, size=n)
    else:
        E = np.full(n, 1e5)
        nu = np.full(n, 0.45)
    lam, mu = lame_from_young(E, nu)
    return Cloud(name=f"rand{n}", xyz=xyz, vol=np.full(n, box ** 3 / n), lam=lam, mu=mu,
                 rho=np.full(n, 1000.0), h=support_factor * s, k=k, seed=seed)


# ----------------------------------------------------------------------------
# shapes: unions of spheres / ellipsoids clipped to the unit box
# ----------------------------------------------------------------------------

class _Union:
    """Inside test for a union of ellipsoids (spheres are a special case)."""

    def __init__(self, centres, axes, rots):
        self.c = np.asarray(centres, dtype=np.float64)      # (m, 3)
        self.a = np.asarray(axes, dtype=np.float64)         # (m, 3) semi-axes
        self.R = np.asarray(rots, dtype=np.float64)         # (m, 3, 3) body->world
        # axis-aligned bodies skip the rotation (a product with the identity is exact)
        self.eye = [bool(np.array_equal(R, np.eye(3))) for R in self.R]

    def inside(self, p: np.ndarray) -> np.ndarray:
        p = np.asarray(p, dtype=np.float64)
        ok = np.zeros(p.shape[0], dtype=bool)
        step = 1 << 16                  # cache-sized pieces (the same arithmetic per point)
        for s0 in range(0, p.shape[0], step):
            ps = p[s0:s0 + step]
            oks = ok[s0:s0 + step]
            for c, a, R, eye in zip(self.c, self.a, self.R, self.eye):
                q = ps - c if eye else (ps - c) @ R     # world -> body coordinates
                t = q / a
                oks |= ((t[:, 0] * t[:, 0] + t[:, 1] * t[:, 1]) + t[:, 2] * t[:, 2]) <= 1.0
            for ax in range(3):
                oks &= (ps[:, ax] >= 0.0) & (ps[:, ax] <= 1.0)
        return ok


def _quat_to_rot(q):
    w, x, y, z = q / np.linalg.norm(q)
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
                     [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
                     [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)]])


def _sphere_union(rng, count=8, rmin=0.1, rmax=0.3):
    c = rng.uniform(0.0, 1.0, size=(count, 3))
    r = rng.uniform(rmin, rmax, size=count)
    return _Union(c, np.repeat(r[:, None], 3, axis=1), np.repeat(np.eye(3)[None], count, axis=0))


def _ellipsoid_union(rng, count=20, amin=0.05, amax=0.4):
    c = rng.uniform(0.0, 1.0, size=(count, 3))
    a = rng.uniform(amin, amax, size=(count, 3))
    R = np.stack([_quat_to_rot(rng.standard_normal(4)) for _ in range(count)])
    return _Union(c, a, R)


def _mc_volume(shape: _Union, rng, samples: int) -> float:
    hits = 0
    chunk = 1_000_000
    done = 0
    while done < samples:
        m = min(chunk, samples - done)
        hits += int(np.count_nonzero(shape.inside(rng.uniform(0.0, 1.0, size=(m, 3)))))
        done += m
    return hits / samples


def _connected(shape: _Union, res: int = 96) -> bool:
    """Connectivity of the voxelised shape (6-connected voxel components)."""
    from scipy import ndimage
    g = (np.arange(res) + 0.5) / res
    Z, Y, X = np.meshgrid(g, g, g, indexing="ij")
    occ = shape.inside(np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)).reshape(res, res, res)
    _, ncomp = ndimage.label(occ)
    return ncomp == 1


def _rejection_sample(shape: _Union, rng, n: int) -> np.ndarray:
    out = []
    have = 0
    while have < n:
        cand = rng.uniform(0.0, 1.0, size=(max(2 * (n - have), 4096), 3))
        cand = cand[shape.inside(cand)]
        out.append(cand)
        have += cand.shape[0]
    return np.ascontiguousarray(np.concatenate(out)[:n])


def _poisson_disk(shape: _Union, rng, n: int, r: float, max_rounds: int = 4000) -> np.ndarray:
    """Dart throwing with minimum distance r until n points are placed.

    Candidates arrive in batches; a candidate is kept if it is at least r from
    every kept point and from every earlier kept candidate of its batch.
    """
    from scipy.spatial import cKDTree
    pts = np.zeros((0, 3))
    rounds = 0
    while pts.shape[0] < n:
        rounds += 1
        if rounds > max_rounds:
            raise RuntimeError(f"Poisson-disk sampling stalled at {pts.shape[0]} / {n} points")
        need = n - pts.shape[0]
        cand = rng.uniform(0.0, 1.0, size=(max(4 * need, 2048), 3))
        cand = cand[shape.inside(cand)]
        if pts.shape[0]:
            d, _ = cKDTree(pts).query(cand, k=1, distance_upper_bound=r)
            cand = cand[~(d < r)]
        if cand.shape[0] == 0:
            continue
        # resolve conflicts inside the batch greedily in candidate order (walk the
        # candidates in order, dropping the later partners of each kept one): the
        # same selection is reached in rounds, a candidate being kept once every
        # earlier partner is dropped and dropped once an earlier partner is kept
        pairs = cKDTree(cand).query_pairs(r, output_type="ndarray")
        keep = np.ones(cand.shape[0], dtype=bool)
        if pairs.size:
            lo = np.minimum(pairs[:, 0], pairs[:, 1])
            hi = np.maximum(pairs[:, 0], pairs[:, 1])
            state = np.zeros(cand.shape[0], dtype=np.int8)       # 0 open, 1 kept, 2 dropped
            nc = cand.shape[0]
            while True:
                open_lo = np.bincount(hi, weights=(state[lo] != 2), minlength=nc)
                newly_kept = (state == 0) & (open_lo == 0)
                state[newly_kept] = 1
                kept_lo = np.bincount(hi, weights=(state[lo] == 1), minlength=nc)
                state[(state == 0) & (kept_lo > 0)] = 2
                if not np.any(state == 0):
                    break
            keep = state == 1
        cand = cand[keep][:need]
        pts = np.concatenate([pts, cand])
    return np.ascontiguousarray(pts[:n])


def sphere_union(n: int = 100_000, seed: int = 1, r_disk: Optional[float] = None,
                 E: float = 1e5, nu: float = 0.45, rho: float = 1000.0, k: int = 32,
                 support: float = 2.5, mc_samples: int = 2_000_000, min_volume: float = 0.2) -> Cloud:
    """Poisson-disk samples inside 8 random spheres (radii U(0.1, 0.3)) in the unit box.

    The shape is redrawn while its volume is below ``min_volume`` or it is not
    connected. Mean spacing s = (V/n)^(1/3), h = support * s, v = V/n.
    ``r_disk`` defaults to 0.7 s.
    """
    rng = np.random.default_rng(seed)
    while True:
        shape = _sphere_union(rng)
        V = _mc_volume(shape, rng, mc_samples)
        if V >= min_volume and _connected(shape):
            break
    s = (V / n) ** (1.0 / 3.0)
    r = 0.7 * s if r_disk is None else r_disk
    xyz = _poisson_disk(shape, rng, n, r)
    lam, mu = lame_from_young(np.full(n, E), np.full(n, nu))
    return Cloud(name=f"spheres{n}", xyz=xyz, vol=np.full(n, V / n), lam=lam, mu=mu,
                 rho=np.full(n, rho), h=support * s, k=k, seed=seed,
                 meta=dict(volume=V, spacing=s, r_disk=r, E=E, nu=nu))


def ellipsoid_union(n: int = 1_000_000, seed: int = 3, hetero: bool = True, k: int = 32,
                    count: int = 20, support: float = 2.5, mc_samples: int = 4_000_000,
                    E: Optional[float] = None, nu: float = 0.45, rho: float = 1000.0,
                    min_volume: float = 0.05, sample_seed: Optional[int] = None) -> Cloud:
    """Uniform samples inside a union of 20 random ellipsoids (semi-axes U(0.05, 0.4)).

    ``hetero`` draws per-particle E log-uniform in [1e4, 1e6] Pa and nu
    uniform in [0.3, 0.48]; otherwise E (default: log-uniform per shape) and
    nu are uniform over the object. ``sample_seed`` (optional) seeds the
    particle positions and materials separately from the shape, so one shape
    can be sampled at several resolutions.
    """
    rng = np.random.default_rng(seed)
    while True:
        shape = _ellipsoid_union(rng, count=count)
        V = _mc_volume(shape, rng, mc_samples)
        if V >= min_volume and _connected(shape):
            break
    if sample_seed is not None:
        rng = np.random.default_rng([seed, sample_seed])
    xyz = _rejection_sample(shape, rng, n)
    s = (V / n) ** (1.0 / 3.0)
    if hetero:
        Ev = np.exp(rng.uniform(math.log(1e4), math.log(1e6), size=n))
        nuv = rng.uniform(0.3, 0.48, size=n)
    else:
        e0 = float(np.exp(rng.uniform(math.log(1e4), math.log(1e6)))) if E is None else E
        Ev = np.full(n, e0)
        nuv = np.full(n, nu)
    lam, mu = lame_from_young(Ev, nuv)
    return Cloud(name=f"ellipsoids{n}", xyz=xyz, vol=np.full(n, V / n), lam=lam, mu=mu,
                 rho=np.full(n, rho), h=support * s, k=k, seed=seed,
                 meta=dict(volume=V, spacing=s, hetero=hetero))


def _batch_member(args) -> Cloud:
    nj, sj, Ej, k, mc_samples = args
    return sphere_union(n=nj, seed=sj, E=Ej, k=k, mc_samples=mc_samples)


def batch_objects(count: int = 64, nmin: int = 2_000, nmax: int = 200_000, seed: int = 100,
                  k: int = 16, mc_samples: int = 400_000, workers: int = 1) -> List[Cloud]:
    """Sphere-union objects with n log-uniform in [nmin, nmax] and E uniform in [1e4, 1e6].

    Each object draws from its own seed, so ``workers`` > 1 builds them in
    freshly started worker processes with the same result."""
    rng = np.random.default_rng(seed)
    jobs = []
    for j in range(count):
        nj = int(round(math.exp(rng.uniform(math.log(nmin), math.log(nmax)))))
        Ej = float(rng.uniform(1e4, 1e6))
        jobs.append((nj, seed * 1000 + j, Ej, k, mc_samples))
    if workers <= 1:
        return [_batch_member(a) for a in jobs]
    import multiprocessing as mp
    order = sorted(range(count), key=lambda j: -jobs[j][0])       # largest first
    with mp.get_context("spawn").Pool(min(workers, count)) as pool:
        built = pool.map(_batch_member, [jobs[j] for j in order], chunksize=1)
    out = [None] * count
    for j, c in zip(order, built):
        out[j] = c
    return out


# ----------------------------------------------------------------------------
# integration points of the paper's own construction (Supp. B.1): a uniform grid
# over the bounding box, points outside the object rejected
# ----------------------------------------------------------------------------

@dataclasses.dataclass
class IntegrationSet:
    """Grid integration points inside an object, their weights and material, and the number
    of kernel centres to pick from them."""
    name: str
    xyz: np.ndarray          # (Q, 3) grid points inside the object, grid order (x fastest)
    vol: np.ndarray          # (Q,) weight = grid cell volume
    lam: np.ndarray
    mu: np.ndarray
    rho: np.ndarray
    spacing: float
    K: int                   # kernel centres to pick
    k: int                   # eigenpairs wanted (constant mode included)
    meta: dict = dataclasses.field(default_factory=dict)

    @property
    def q(self) -> int:
        return int(self.xyz.shape[0])

    def sha256(self) -> str:
        m = hashlib.sha256()
        for a in (self.xyz, self.vol, self.lam, self.mu, self.rho):
            m.update(np.ascontiguousarray(a).tobytes())
        m.update(np.int64(self.K).tobytes())
        return m.hexdigest()


def grid_inside(inside, lo, hi, spacing: float) -> np.ndarray:
    """Cell centres lo + (i + 1/2) g of a uniform grid over the box [lo, hi] that pass the
    inside test, x fastest."""
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    cnt = np.maximum(1, np.round((hi - lo) / spacing).astype(np.int64))
    axes = [lo[a] + (np.arange(cnt[a]) + 0.5) * spacing for a in range(3)]
    z, y, x = np.meshgrid(axes[2], axes[1], axes[0], indexing="ij")
    p = np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1)
    return np.ascontiguousarray(p[inside(p)])


def _set(name, xyz, spacing, E, nu, rho, K, k, meta):
    q = xyz.shape[0]
    E = np.broadcast_to(np.asarray(E, dtype=np.float64), (q,)).copy()
    nu = np.broadcast_to(np.asarray(nu, dtype=np.float64), (q,)).copy()
    lam, mu = lame_from_young(E, nu)
    return IntegrationSet(name, xyz, np.full(q, spacing ** 3), lam, mu, np.full(q, float(rho)), spacing, K, k,
                          meta)


def beam(spacing: float = 0.05, K: int = 1000, k: int = 17, E: float = 5e6, nu: float = 0.45,
         rho: float = 1000.0, length: float = 5.0) -> IntegrationSet:
    """The standard beam of Sec. 4: a length x 1 x 1 m cuboid (5 m by default), E = 5e6 Pa,
    nu = 0.45, density 1000; every grid point of the box is inside."""
    xyz = grid_inside(lambda p: np.ones(p.shape[0], dtype=bool), (0, 0, 0), (length, 1, 1), spacing)
    return _set(f"beam{length:g}", xyz, spacing, E, nu, rho, K, k, dict(length=length))


def layered_sphere(spacing: float = 0.025, K: int = 1000, k: int = 33, radius: float = 0.5,
                   E_stiff: float = 1e6, E_soft: float = 1e4, nu: float = 0.45, rho: float = 1000.0,
                   layers: int = 4) -> IntegrationSet:
    """The heterogeneous sphere of the supplementary multi-layer test: concentric shells of equal
    thickness, stiff and soft alternating from the centre outwards (stiff-soft-stiff-soft)."""
    inside = lambda p: np.sum(p * p, axis=1) <= radius * radius
    xyz = grid_inside(inside, (-radius,) * 3, (radius,) * 3, spacing)
    shell = np.minimum((np.sqrt(np.sum(xyz * xyz, axis=1)) / radius * layers).astype(np.int64), layers - 1)
    E = np.where(shell % 2 == 0, E_stiff, E_soft)
    return _set("layered_sphere", xyz, spacing, E, nu, rho, K, k, dict(radius=radius, layers=layers))


def ellipsoid_blob(spacing: float = 0.02, K: int = 1000, k: int = 33, seed: int = 3, E: float = 1e5,
                   nu: float = 0.45, rho: float = 1000.0) -> IntegrationSet:
    """An object of the kind the paper's datasets hold (a closed shape with an inside test),
    here the seeded union of 20 ellipsoids of the large-object workload, on a grid."""
    rng = np.random.default_rng(seed)
    while True:
        shape = _ellipsoid_union(rng, count=20)
        if _mc_volume(shape, rng, 400_000) >= 0.05 and _connected(shape):
            break
    xyz = grid_inside(shape.inside, (0, 0, 0), (1, 1, 1), spacing)
    return _set(f"ellipsoid_blob{seed}", xyz, spacing, E, nu, rho, K, k, dict(seed=seed))


def initial_block(n: int, m: int, seed: int) -> np.ndarray:
    """Seeded starting block for the eigensolver, uniform in [-1, 1), row-major (n, m)."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-1.0, 1.0, size=(n, m))


# ----------------------------------------------------------------------------
# named workloads
# ----------------------------------------------------------------------------

def workload(name: str) -> Cloud:
    """The named synthetic workloads, built by the generators above."""
    if name == "cube1k":
        return cube_lattice()
    if name == "spheres100k":
        return sphere_union(n=100_000, seed=1, r_disk=0.01, k=32)
    if name == "ellipsoids1m":
        return ellipsoid_union(n=1_000_000, seed=3, hetero=True, k=32)
    if name.startswith("ellipsoids"):
        n = int(float(name[len("ellipsoids"):].replace("k", "e3").replace("m", "e6")))
        return ellipsoid_union(n=n, seed=3, hetero=True, k=32)
    raise KeyError(name)
