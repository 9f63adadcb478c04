"""FP64 CPU oracle of the FreeForm subspace-construction path (arXiv 2605.29318).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg of
the benchmark may import this module; the product library never does. It
shares no code with the GPU path (the seeded input generators, which hold none
of the method's arithmetic, are the only common module).

Layers:
  * ``ff_oracle.c`` (built here with gcc, no FMA contraction): cell binning,
    neighbour lists, RKPM shape functions (Sec. 3.2 Eq. (7)-(11)), the
    transpose of the neighbour relation, the Hessian of Prop. 1 and the mass
    matrix of Eq. (14), CSR products.
  * this file: the generalized eigenproblem of Eq. (15) - dense LAPACK
    ``eigh`` for small n, and an FP64 block LOBPCG (Knyazev 2001) with SVQB
    orthonormalisation (Stathopoulos & Wu 2002) and an optional Jacobi
    (diag(H)^-1) or Chebyshev-Jacobi polynomial preconditioner for larger n -
    plus the residual, subspace-angle and cluster metrics used to compare
    results.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ff_oracle.c")
_LIB = os.path.join(_HERE, "libff_oracle.so")

_i64p = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
_i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")


def build(force: bool = False) -> str:
    """Compile the C oracle (gcc, OpenMP, -ffp-contract=off)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
                               "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        vp = ctypes.c_void_p
        L.orc_grid.argtypes = [ctypes.c_int64, _f64p, ctypes.c_double, _f64p, _i64p]
        L.orc_grid.restype = ctypes.c_int
        L.orc_bin.argtypes = [ctypes.c_int64, _f64p, ctypes.c_double, _f64p, _i64p, _i32p, _i64p]
        L.orc_bin.restype = ctypes.c_int
        L.orc_neighbors.argtypes = [ctypes.c_int64, _f64p, _f64p, ctypes.c_double, _f64p, _i64p,
                                    _i64p, _i64p, vp]
        L.orc_neighbors.restype = ctypes.c_int64
        L.orc_neighbors_brute.argtypes = [ctypes.c_int64, _f64p, ctypes.c_int64, _f64p,
                                          ctypes.c_double, _i64p, vp]
        L.orc_neighbors_brute.restype = ctypes.c_int64
        L.orc_rkpm.argtypes = [ctypes.c_int64, _f64p, _f64p, _i64p, _i32p, ctypes.c_double,
                               ctypes.c_int, _f64p, _f64p, ctypes.POINTER(ctypes.c_int64)]
        L.orc_rkpm.restype = ctypes.c_int
        L.orc_transpose.argtypes = [ctypes.c_int64, ctypes.c_int64, _i64p, _i32p, _i64p, _i32p,
                                    _i32p]
        L.orc_transpose.restype = ctypes.c_int
        L.orc_assemble.argtypes = [ctypes.c_int64, ctypes.c_int64, _i64p, _i32p, _f64p, _f64p,
                                   _f64p, _f64p, _f64p, vp, _i64p, _i32p, _i32p, _i64p, vp, vp, vp]
        L.orc_assemble.restype = ctypes.c_int64
        L.orc_spmm.argtypes = [ctypes.c_int64, _i64p, _i32p, _f64p, ctypes.c_int64, _f64p, _f64p]
        L.orc_spmm.restype = None
        L.orc_norm_inf.argtypes = [ctypes.c_int64, _i64p, _f64p]
        L.orc_norm_inf.restype = ctypes.c_double
        L.orc_fps.argtypes = [ctypes.c_int64, _f64p, ctypes.c_int64, ctypes.c_int64, _i32p]
        L.orc_fps.restype = ctypes.c_int
        L.orc_radii.argtypes = [ctypes.c_int64, _f64p, ctypes.c_double, _f64p, _f64p]
        L.orc_radii.restype = ctypes.c_int
        L.orc_neighbors_var.argtypes = [ctypes.c_int64, _f64p, _f64p, _f64p, ctypes.c_double, _f64p, _i64p,
                                        _i64p, _i64p, vp]
        L.orc_neighbors_var.restype = ctypes.c_int64
        L.orc_neighbors_var_brute.argtypes = [ctypes.c_int64, _f64p, ctypes.c_int64, _f64p, _f64p, _i64p, vp]
        L.orc_neighbors_var_brute.restype = ctypes.c_int64
        L.orc_rkpm_var.argtypes = [ctypes.c_int64, _f64p, _f64p, _f64p, _i64p, _i32p, ctypes.c_double,
                                   ctypes.c_double, ctypes.c_int, _f64p, _f64p, ctypes.POINTER(ctypes.c_int64)]
        L.orc_rkpm_var.restype = ctypes.c_int
        _lib = L
    return _lib


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


# ----------------------------------------------------------------------------
# binning and neighbours
# ----------------------------------------------------------------------------

def grid(xyz, h):
    xyz = _c(xyz, np.float64)
    origin = np.zeros(3)
    dims = np.zeros(3, dtype=np.int64)
    rc = lib().orc_grid(xyz.shape[0], xyz, float(h), origin, dims)
    if rc != 0:
        raise ValueError("bad grid arguments")
    return origin, dims


def bin_nodes(xyz, h):
    """Counting sort of the nodes by (cell, Morton code of the 4x4x4 sub-cell, original
    index). Returns perm, cell_start, origin, dims."""
    xyz = _c(xyz, np.float64)
    origin, dims = grid(xyz, h)
    n = xyz.shape[0]
    perm = np.zeros(n, dtype=np.int32)
    cell_start = np.zeros(int(np.prod(dims)) + 1, dtype=np.int64)
    lib().orc_bin(n, xyz, float(h), origin, dims, perm, cell_start)
    return perm, cell_start, origin, dims


def neighbors(qxyz, xyz_sorted, h, origin, dims, cell_start):
    qxyz = _c(qxyz, np.float64)
    xyz_sorted = _c(xyz_sorted, np.float64)
    q = qxyz.shape[0]
    off = np.zeros(q + 1, dtype=np.int64)
    tot = lib().orc_neighbors(q, qxyz, xyz_sorted, float(h), _c(origin, np.float64),
                              _c(dims, np.int64), _c(cell_start, np.int64), off, None)
    ids = np.zeros(max(tot, 1), dtype=np.int32)
    lib().orc_neighbors(q, qxyz, xyz_sorted, float(h), _c(origin, np.float64), _c(dims, np.int64),
                        _c(cell_start, np.int64), off, _ptr(ids))
    return off, ids[:tot]


def neighbors_brute(qxyz, xyz_sorted, h):
    qxyz = _c(qxyz, np.float64)
    xyz_sorted = _c(xyz_sorted, np.float64)
    q = qxyz.shape[0]
    off = np.zeros(q + 1, dtype=np.int64)
    tot = lib().orc_neighbors_brute(q, qxyz, xyz_sorted.shape[0], xyz_sorted, float(h), off, None)
    ids = np.zeros(max(tot, 1), dtype=np.int32)
    lib().orc_neighbors_brute(q, qxyz, xyz_sorted.shape[0], xyz_sorted, float(h), off, _ptr(ids))
    return off, ids[:tot]


# ----------------------------------------------------------------------------
# shape functions and assembly
# ----------------------------------------------------------------------------

class SingularMoment(RuntimeError):
    def __init__(self, index):
        super().__init__(f"singular moment matrix at quadrature point {index}")
        self.index = index


def rkpm(qxyz, xyz_sorted, off, ids, h, kernel=0):
    """phi[e], dphi[e, 3] for each neighbour entry e (Sec. 3.2 Eq. (7)-(11))."""
    nnz = int(off[-1])
    phi = np.zeros(max(nnz, 1))
    dphi = np.zeros((max(nnz, 1), 3))
    bad = ctypes.c_int64(-1)
    rc = lib().orc_rkpm(len(off) - 1, _c(qxyz, np.float64), _c(xyz_sorted, np.float64),
                        _c(off, np.int64), _c(ids, np.int32), float(h), int(kernel), phi, dphi,
                        ctypes.byref(bad))
    if rc != 0:
        raise SingularMoment(bad.value)
    return phi[:nnz], dphi[:nnz]


def transpose(n, off, ids):
    off = _c(off, np.int64)
    ids = _c(ids, np.int32)
    nt_off = np.zeros(n + 1, dtype=np.int64)
    nt_id = np.zeros(max(len(ids), 1), dtype=np.int32)
    nt_slot = np.zeros(max(len(ids), 1), dtype=np.int32)
    lib().orc_transpose(n, len(off) - 1, off, ids, nt_off, nt_id, nt_slot)
    return nt_off, nt_id, nt_slot


def assemble(n, off, ids, phi, dphi, vol, lam, mu, rho=None):
    """CSR (row_ptr, col, H, M) of Prop. 1 and Eq. (14), rows and columns in sorted numbering."""
    off = _c(off, np.int64)
    ids = _c(ids, np.int32)
    q = len(off) - 1
    phi = _c(phi, np.float64)
    dphi = _c(dphi, np.float64).reshape(-1)
    vol = _c(vol, np.float64)
    lam = _c(lam, np.float64)
    mu = _c(mu, np.float64)
    rho = None if rho is None else _c(rho, np.float64)
    nt_off, nt_id, nt_slot = transpose(n, off, ids)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    nnz = lib().orc_assemble(n, q, off, ids, phi, dphi, vol, lam, mu, _ptr(rho), nt_off, nt_id,
                             nt_slot, row_ptr, None, None, None)
    col = np.zeros(max(nnz, 1), dtype=np.int32)
    H = np.zeros(max(nnz, 1))
    M = np.zeros(max(nnz, 1))
    lib().orc_assemble(n, q, off, ids, phi, dphi, vol, lam, mu, _ptr(rho), nt_off, nt_id, nt_slot,
                       row_ptr, _ptr(col), _ptr(H), _ptr(M))
    return row_ptr, col[:nnz], H[:nnz], M[:nnz]


def spmm(row_ptr, col, val, X):
    """Y = A X for a CSR matrix given by its arrays (row-major blocks, threaded C loop)."""
    X = _c(X, np.float64)
    two = X.ndim == 2
    X2 = X if two else X[:, None]
    X2 = np.ascontiguousarray(X2)
    col = _c(col, np.int32)
    if col.size and (int(col.max()) >= X2.shape[0] or int(col.min()) < 0):
        raise ValueError("column index outside the block")
    Y = np.zeros((len(row_ptr) - 1, X2.shape[1]))       # as many rows as the matrix (it may be rectangular)
    lib().orc_spmm(len(row_ptr) - 1, _c(row_ptr, np.int64), col,
                   _c(val, np.float64), X2.shape[1], X2, Y)
    return Y if two else Y[:, 0]


def norm_inf(row_ptr, val):
    return float(lib().orc_norm_inf(len(row_ptr) - 1, _c(row_ptr, np.int64), _c(val, np.float64)))


def matmul(A, X):
    """A @ X for a scipy CSR matrix, through the threaded C product of ``spmm`` (the same
    definition as scipy's, one row at a time in storage order); other operands use ``@``."""
    import scipy.sparse as sp
    if not sp.isspmatrix_csr(A) and not isinstance(A, getattr(sp, "csr_array", ())):
        return A @ X
    arrs = getattr(A, "_orc_arrays", None)
    if arrs is None:
        arrs = (np.ascontiguousarray(A.indptr, dtype=np.int64), np.ascontiguousarray(A.indices, dtype=np.int32),
                np.ascontiguousarray(A.data, dtype=np.float64))
        try:
            A._orc_arrays = arrs
        except AttributeError:
            pass
    return spmm(arrs[0], arrs[1], arrs[2], X)


def to_scipy(n, row_ptr, col, val):
    import scipy.sparse as sp
    return sp.csr_matrix((val, col, row_ptr), shape=(n, n))


@dataclass
class Problem:
    """Everything the path produces for one object, in sorted numbering."""
    n: int
    h: float
    perm: np.ndarray
    cell_start: np.ndarray
    origin: np.ndarray
    dims: np.ndarray
    xyz: np.ndarray
    nbr_off: np.ndarray
    nbr_id: np.ndarray
    phi: np.ndarray
    dphi: np.ndarray
    vol: np.ndarray
    lam: np.ndarray
    mu: np.ndarray
    rho: Optional[np.ndarray]
    row_ptr: np.ndarray
    col: np.ndarray
    H: np.ndarray
    M: np.ndarray

    def Hs(self):
        return to_scipy(self.n, self.row_ptr, self.col, self.H)

    def Ms(self):
        return to_scipy(self.n, self.row_ptr, self.col, self.M)


def pipeline(cloud, use_rho: bool = False, kernel: int = 0) -> Problem:
    """Binning -> neighbours -> shape functions -> H, M for a synthetic cloud.

    Quadrature points are the particles themselves (one per particle), so the
    per-point arrays are permuted into sorted numbering with ``perm``.
    """
    perm, cs, origin, dims = bin_nodes(cloud.xyz, cloud.h)
    xs = np.ascontiguousarray(cloud.xyz[perm])
    off, ids = neighbors(xs, xs, cloud.h, origin, dims, cs)
    phi, dphi = rkpm(xs, xs, off, ids, cloud.h, kernel=kernel)
    vol, lam, mu = cloud.vol[perm], cloud.lam[perm], cloud.mu[perm]
    rho = cloud.rho[perm] if use_rho else None
    rp, col, H, M = assemble(cloud.n, off, ids, phi, dphi, vol, lam, mu, rho)
    return Problem(cloud.n, cloud.h, perm, cs, origin, dims, xs, off, ids, phi, dphi,
                   np.ascontiguousarray(vol), np.ascontiguousarray(lam), np.ascontiguousarray(mu),
                   rho, rp, col, H, M)


# ----------------------------------------------------------------------------
# the paper's own construction (Supp. B.1 "RKPM construction"): integration points,
# farthest-point-sampled centres, a Gaussian per centre whose radius reaches two other
# centres; plain RBF, partition-of-unity RBF and RKPM bases (Sec. 3.2, Fig. 3b)
# ----------------------------------------------------------------------------

BASIS_RBF, BASIS_PU, BASIS_RKPM = 0, 1, 2


def fps(xyz, K, start=0):
    """Farthest point sampling of K of the points, from ``start``; ties to the lowest index."""
    xyz = _c(xyz, np.float64)
    out = np.zeros(int(K), dtype=np.int32)
    if lib().orc_fps(xyz.shape[0], xyz, int(K), int(start), out) != 0:
        raise ValueError("bad FPS arguments")
    return out


def radii(centres, cut=3.0):
    """r_k = distance to the 2nd-nearest other centre; R_k = cut * r_k (support of the cut kernel)."""
    c = _c(centres, np.float64)
    r = np.zeros(c.shape[0])
    R = np.zeros(c.shape[0])
    if lib().orc_radii(c.shape[0], c, float(cut), r, R) != 0:
        raise ValueError("need at least 3 centres")
    return r, R


def neighbors_var(qxyz, xyz_sorted, R_sorted, h, origin, dims, cell_start):
    qxyz = _c(qxyz, np.float64)
    q = qxyz.shape[0]
    off = np.zeros(q + 1, dtype=np.int64)
    args = (_c(xyz_sorted, np.float64), _c(R_sorted, np.float64), float(h), _c(origin, np.float64),
            _c(dims, np.int64), _c(cell_start, np.int64), off)
    tot = lib().orc_neighbors_var(q, qxyz, *args, None)
    ids = np.zeros(max(tot, 1), dtype=np.int32)
    lib().orc_neighbors_var(q, qxyz, *args, _ptr(ids))
    return off, ids[:tot]


def neighbors_var_brute(qxyz, xyz_sorted, R_sorted):
    qxyz = _c(qxyz, np.float64)
    xs = _c(xyz_sorted, np.float64)
    q = qxyz.shape[0]
    off = np.zeros(q + 1, dtype=np.int64)
    tot = lib().orc_neighbors_var_brute(q, qxyz, xs.shape[0], xs, _c(R_sorted, np.float64), off, None)
    ids = np.zeros(max(tot, 1), dtype=np.int32)
    lib().orc_neighbors_var_brute(q, qxyz, xs.shape[0], xs, _c(R_sorted, np.float64), off, _ptr(ids))
    return off, ids[:tot]


def rkpm_var(qxyz, xyz_sorted, r_sorted, off, ids, h, cut=3.0, basis=BASIS_RKPM):
    """phi, dphi on the centres' cut Gaussians for the given basis (0 RBF, 1 PU-RBF, 2 RKPM)."""
    nnz = int(off[-1])
    phi = np.zeros(max(nnz, 1))
    dphi = np.zeros((max(nnz, 1), 3))
    bad = ctypes.c_int64(-1)
    rc = lib().orc_rkpm_var(len(off) - 1, _c(qxyz, np.float64), _c(xyz_sorted, np.float64),
                            _c(r_sorted, np.float64), _c(off, np.int64), _c(ids, np.int32), float(h),
                            float(cut), int(basis), phi, dphi, ctypes.byref(bad))
    if rc != 0:
        raise SingularMoment(bad.value)
    return phi[:nnz], dphi[:nnz]


@dataclass
class PaperProblem:
    """The paper's construction for one object, centres in sorted (cell) numbering."""
    K: int
    centre_idx: np.ndarray      # [K] FPS picks: indices into the integration points, in pick order
    perm: np.ndarray            # [K] sorted centre j = pick perm[j]
    xyz: np.ndarray             # [K][3] centres, sorted
    r: np.ndarray               # [K] Gaussian radius, sorted
    R: np.ndarray               # [K] support radius, sorted
    h: float                    # cell edge = max R
    origin: np.ndarray
    dims: np.ndarray
    cell_start: np.ndarray
    qxyz: np.ndarray
    nbr_off: np.ndarray
    nbr_id: np.ndarray
    phi: np.ndarray
    dphi: np.ndarray
    row_ptr: np.ndarray
    col: np.ndarray
    H: np.ndarray
    M: np.ndarray

    def Hs(self):
        return to_scipy(self.K, self.row_ptr, self.col, self.H)

    def Ms(self):
        return to_scipy(self.K, self.row_ptr, self.col, self.M)


def paper_pipeline(qxyz, vol, lam, mu, K, cut=3.0, basis=BASIS_RKPM, start=0, rho=None) -> PaperProblem:
    """Supp. B.1: K centres by FPS over the integration points, r_k to the 2nd-nearest centre,
    neighbour lists d^2 < R_k^2 on a grid of edge max R, shape functions (Sec. 3.2) and
    H (Prop. 1), M (Eq. (14)) with the integration points as quadrature (weights vol)."""
    qxyz = _c(qxyz, np.float64)
    pick = fps(qxyz, K, start)
    cen = qxyz[pick]
    r, R = radii(cen, cut)
    h = float(R.max())
    perm, cs, origin, dims = bin_nodes(cen, h)
    xs = np.ascontiguousarray(cen[perm])
    rs, Rs = r[perm], R[perm]
    off, ids = neighbors_var(qxyz, xs, Rs, h, origin, dims, cs)
    phi, dphi = rkpm_var(qxyz, xs, rs, off, ids, h, cut, basis)
    rp, col, H, M = assemble(K, off, ids, phi, dphi, vol, lam, mu, rho)
    return PaperProblem(int(K), pick, perm, xs, rs, Rs, h, origin, dims, cs, qxyz, off, ids, phi, dphi,
                        rp, col, H, M)


# ----------------------------------------------------------------------------
# eigenproblem (Eq. (15)): H w = lambda M w, k smallest, W^T M W = I
# ----------------------------------------------------------------------------

def sign_fix(W):
    """Sign rule: in every column the entry of largest magnitude is positive (first on ties)."""
    W = np.array(W, copy=True)
    idx = np.argmax(np.abs(W), axis=0)
    s = np.sign(W[idx, np.arange(W.shape[1])])
    s[s == 0] = 1.0
    return W * s


def dense_eigh(H, M, k):
    """Plain definition for small n: LAPACK generalized symmetric eigensolver."""
    import scipy.linalg as sl
    Hd = H.toarray() if hasattr(H, "toarray") else np.asarray(H)
    Md = M.toarray() if hasattr(M, "toarray") else np.asarray(M)
    w, V = sl.eigh(Hd, Md, subset_by_index=[0, k - 1])
    return w, sign_fix(V)


def residuals(H, M, lam, W, normH=None, normM=None):
    """r_j = ||H w_j - lam_j M w_j|| / ((||H||_inf + |lam_j| ||M||_inf) ||w_j||)."""
    if normH is None:
        normH = float(abs(H).sum(axis=1).max())
    if normM is None:
        normM = float(abs(M).sum(axis=1).max())
    W = np.ascontiguousarray(W, dtype=np.float64)
    R = matmul(H, W) - matmul(M, W) * lam[None, :]
    return np.linalg.norm(R, axis=0) / ((normH + np.abs(lam) * normM) * np.linalg.norm(W, axis=0))


def _svqb(S, MS, tau):
    """M-orthonormalise the columns of S (Stathopoulos & Wu 2002); returns T with S T orthonormal."""
    G = S.T @ MS
    G = 0.5 * (G + G.T)
    d = np.sqrt(np.maximum(np.diag(G), 1e-300))
    Dinv = 1.0 / d
    Gs = G * Dinv[:, None] * Dinv[None, :]
    s, U = np.linalg.eigh(Gs)
    keep = s > tau * s.max()
    return (Dinv[:, None] * U[:, keep]) / np.sqrt(s[keep])[None, :]


def chebyshev_jacobi(H, degree=12, ratio=1000.0, upper=None, mul=None):
    """Polynomial preconditioner T r = p(D^-1 H) D^-1 r, D = diag(H).

    p is the Chebyshev semi-iteration for D^-1 H z = D^-1 r on the interval
    [upper / ratio, upper] (Saad, "Iterative Methods for Sparse Linear Systems",
    Chebyshev acceleration), started from z = 0 and stopped after ``degree``
    updates of z, i.e. ``degree - 1`` products with H. p is positive on
    (0, upper], so T is symmetric positive definite when ``upper`` bounds the
    spectrum of D^-1 H; by default ``upper`` is 1.05 times the largest
    eigenvalue of D^-1/2 H D^-1/2 from ARPACK. The eigenproblem's answer does
    not depend on T, only the number of iterations does.
    """
    mul = matmul if mul is None else mul
    d = np.asarray(H.diagonal(), dtype=np.float64)
    if upper is None:
        import scipy.sparse.linalg as sla
        s = 1.0 / np.sqrt(d)
        op = sla.LinearOperator(H.shape, dtype=np.float64,
                                matvec=lambda v: s * mul(H, np.ascontiguousarray(s * np.ravel(v))))
        lmax = float(sla.eigsh(op, k=1, which="LA", tol=1e-4, return_eigenvectors=False)[0])
        upper = 1.05 * lmax
    lo = upper / ratio
    theta, delta = 0.5 * (upper + lo), 0.5 * (upper - lo)
    sigma = theta / delta

    def apply(R, record=None):
        # record (a list, optional) receives a copy of each of the ``degree`` increments of z
        f = R / d[:, None]                     # right-hand side D^-1 r
        z = np.zeros_like(f)
        res = f.copy()                         # residual f - A z of the Chebyshev iteration
        step = res / theta
        rho = 1.0 / sigma
        for j in range(degree):
            z += step
            if record is not None:
                record.append(step.copy())
            if j == degree - 1:
                break
            res -= mul(H, step) / d[:, None]
            rho_next = 1.0 / (2.0 * sigma - rho)
            step = (rho_next * rho) * step + (2.0 * rho_next / delta) * res
            rho = rho_next
        return z

    apply.upper = upper
    return apply


def lobpcg(H, M, X0, k=None, tol=1e-10, maxiter=5000, precond=None, normH=None, normM=None,
           verbose=False, mul=None, callback=None):
    """Block LOBPCG (Knyazev 2001) in FP64 for the smallest eigenpairs of (H, M).

    Search space S = [X, W, P] with W the (optionally preconditioned) block
    residual and P the previous search direction; the Rayleigh-Ritz step is
    done in an M-orthonormal basis of S. Converged when the first k columns
    satisfy the backward-error residual of ``residuals`` <= tol. ``precond``
    is None, "jacobi" (diag(H)^-1), "chebyshev" (``chebyshev_jacobi`` with its
    defaults) or a callable R -> W. Products with H and M go through ``mul``
    (default ``matmul``, the threaded C loop for CSR operands). With ``verbose``
    = v, every v-th iteration prints the largest residual of the first k columns
    and calls ``callback(iteration, ritz_values, residuals)`` when given.
    """
    mul = matmul if mul is None else mul
    X = np.array(X0, dtype=np.float64, copy=True)
    m = X.shape[1]
    if isinstance(precond, str):
        if precond == "jacobi":
            dH = np.asarray(H.diagonal(), dtype=np.float64)
            precond = (lambda R, d=dH: R / d[:, None])
        elif precond == "chebyshev":
            precond = chebyshev_jacobi(H, mul=mul)
        else:
            raise ValueError(precond)
    k = m if k is None else k
    if normH is None:
        normH = float(abs(H).sum(axis=1).max())
    if normM is None:
        normM = float(abs(M).sum(axis=1).max())
    MX = mul(M, X)
    T = _svqb(X, MX, 1e-14)
    X = X @ T
    HX, MX = mul(H, X), mul(M, X)
    A = X.T @ HX
    th, Y = np.linalg.eigh(0.5 * (A + A.T))
    X, HX, MX = X @ Y, HX @ Y, MX @ Y
    P = HP = MP = None
    it = 0
    res = None
    for it in range(1, maxiter + 1):
        R = HX - MX * th[None, :]
        res = np.linalg.norm(R, axis=0) / ((normH + np.abs(th) * normM) *
                                           np.linalg.norm(X, axis=0))
        if verbose and it % verbose == 0:
            print(it, res[:k].max(), flush=True)
            if callback is not None:
                callback(it, th, res)
        if res[:k].max() <= tol:
            break
        W = R if precond is None else precond(R)
        HW, MW = mul(H, W), mul(M, W)
        blocks = [X, W] + ([P] if P is not None else [])
        S = np.concatenate(blocks, axis=1)
        HS = np.concatenate([HX, HW] + ([HP] if P is not None else []), axis=1)
        MS = np.concatenate([MX, MW] + ([MP] if P is not None else []), axis=1)
        T = _svqb(S, MS, 1e-14)
        A = T.T @ (S.T @ HS) @ T
        th_all, Y = np.linalg.eigh(0.5 * (A + A.T))
        C = T @ Y[:, :m]
        th = th_all[:m]
        Cn = C.copy()
        Cn[:m, :] = 0.0                      # the part of the update outside span(X)
        X, HX, MX = S @ C, HS @ C, MS @ C
        P, HP, MP = S @ Cn, HS @ Cn, MS @ Cn
    order = np.argsort(th)
    th, X = th[order], X[:, order]
    return th[:k], sign_fix(X[:, :k]), it, res[order][:k]


def subspace_sines(Wa, Wb, M):
    """Sines of the principal angles between span(Wa) and span(Wb) in the M inner product."""
    Wa = np.ascontiguousarray(Wa, dtype=np.float64)
    Wb = np.ascontiguousarray(Wb, dtype=np.float64)
    Ta = _svqb(Wa, matmul(M, Wa), 1e-14)
    Qa = Wa @ Ta
    Tb = _svqb(Wb, matmul(M, Wb), 1e-14)
    Qb = Wb @ Tb
    E = Qb - Qa @ (Qa.T @ matmul(M, Qb))
    G = E.T @ matmul(M, E)
    s = np.linalg.eigvalsh(0.5 * (G + G.T))
    return np.sqrt(np.clip(s, 0.0, None))[::-1]


def cluster_safe_k(lam, k, rel_gap=1e-3):
    """Largest k' <= k with (lam[k'] - lam[k'-1]) / lam[k'] >= rel_gap (no split cluster)."""
    for kk in range(k, 0, -1):
        if kk == len(lam):
            continue
        a, b = lam[kk - 1], lam[kk]
        if b > 0 and (b - a) / b >= rel_gap:
            return kk
    return 0


def philox4x32_10(ctr, key):
    """Philox-4x32-10 (Salmon et al., SC'11): ten rounds of two 32x32->64 multiplies
    with multipliers 0xD2511F53 and 0xCD9E8D57 and a Weyl key schedule
    (0x9E3779B9, 0xBB67AE85). Returns the four output words."""
    c = [int(x) & 0xFFFFFFFF for x in ctr]
    k0, k1 = int(key[0]) & 0xFFFFFFFF, int(key[1]) & 0xFFFFFFFF
    for _ in range(10):
        p0 = 0xD2511F53 * c[0]
        p1 = 0xCD9E8D57 * c[2]
        c = [((p1 >> 32) ^ c[1] ^ k0) & 0xFFFFFFFF, p1 & 0xFFFFFFFF,
             ((p0 >> 32) ^ c[3] ^ k1) & 0xFFFFFFFF, p0 & 0xFFFFFFFF]
        k0 = (k0 + 0x9E3779B9) & 0xFFFFFFFF
        k1 = (k1 + 0xBB67AE85) & 0xFFFFFFFF
    return c
