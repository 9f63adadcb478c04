"""Python binding of libfreeform.so (the C ABI declared in include/freeform.h).

Argument marshalling only: every step of the path runs in the library's HIP
kernels. Device arrays are torch tensors on a ROCm device; the functions
allocate the outputs with torch and pass raw pointers plus sizes. The names
follow the C entry points.

The library must be built (``python -m paper_2605_29318_amd.build``); loading
fails loudly if it is missing - there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
import weakref
from dataclasses import dataclass
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfreeform.so")

FF_OK = 0
FF_ERR_INVALID_ARG = -1
FF_ERR_OOM = -2
FF_ERR_HIP = -3
FF_ERR_CAPACITY = -4
FF_ERR_SINGULAR_MOMENT = -5
FF_ERR_NOT_CONVERGED = -6
FF_ERR_BREAKDOWN = -7


class FFError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"freeform error {code}: {msg}")
        self.code = code
        self.msg = msg


class ff_grid(ctypes.Structure):
    _fields_ = [("origin", ctypes.c_double * 3), ("h", ctypes.c_double),
                ("dims", ctypes.c_int64 * 3), ("n_cells", ctypes.c_int64)]


class ff_eig_params(ctypes.Structure):
    _fields_ = [("k", ctypes.c_int), ("block", ctypes.c_int), ("precision", ctypes.c_int),
                ("tol", ctypes.c_double), ("max_iter", ctypes.c_int), ("precond", ctypes.c_int),
                ("seed", ctypes.c_uint64), ("check_every", ctypes.c_int), ("use_graph", ctypes.c_int),
                ("refresh_every", ctypes.c_int), ("precond_degree", ctypes.c_int), ("precond_ratio", ctypes.c_double),
                ("precond_values", ctypes.c_int), ("eig_tol", ctypes.c_double), ("angle_tol", ctypes.c_double)]


class ff_eig_info(ctypes.Structure):
    _fields_ = [("iters_fp32", ctypes.c_int), ("iters_fp64", ctypes.c_int), ("converged", ctypes.c_int),
                ("restarts", ctypes.c_int), ("max_resid", ctypes.c_double), ("seconds", ctypes.c_double),
                ("graph", ctypes.c_int), ("max_eig_bound", ctypes.c_double), ("max_angle_bound", ctypes.c_double),
                ("eig_certified", ctypes.c_int)]


_lib = None
vp = ctypes.c_void_p
i64 = ctypes.c_int64
i32 = ctypes.c_int
f64 = ctypes.c_double


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise FileNotFoundError(f"{LIB_PATH} is not built; run python -m paper_2605_29318_amd.build")
    L = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    sig = {
        "ff_ctx_create": (i32, [P(vp), i32, vp]),
        "ff_ctx_destroy": (None, [vp]),
        "ff_last_error": (ctypes.c_char_p, [vp]),
        "ff_ctx_set_stage_timing": (i32, [vp, i32]),
        "ff_ctx_stage_times": (i32, [vp, i32, P(f64), P(i64)]),
        "ff_stage_name": (ctypes.c_char_p, [i32]),
        "build_neighbors": (i32, [vp, i64, vp, i64, vp, f64, P(ff_grid), vp, vp, vp, i64, vp, vp, i64,
                                  P(i64)]),
        "rkpm_shape": (i32, [vp, i64, vp, i64, vp, vp, vp, i64, f64, i32, vp, vp, vp, P(i64)]),
        "build_neighbors_radii": (i32, [vp, i64, vp, vp, i64, vp, P(ff_grid), vp, vp, vp, i64, vp, vp, i64, P(i64)]),
        "fps_centers": (i32, [vp, i64, vp, i32, i64, vp, vp]),
        "kernel_radii": (i32, [vp, i64, vp, f64, vp, vp]),
        "rkpm_shape_radii": (i32, [vp, i64, vp, vp, vp, i64, vp, vp, vp, i64, f64, f64, i32, vp, vp, P(i64)]),
        "assemble_HM": (i32, [vp, i64, i64, vp, vp, vp, vp, vp, vp, vp, vp, vp, P(ff_grid), vp, vp, vp,
                              vp, vp, vp, i64, P(i64)]),
        "eigenmodes": (i32, [vp, i64, vp, vp, vp, vp, vp, P(ff_eig_params), vp, vp, vp, vp,
                             P(ff_eig_info)]),
        "eigenmodes_batched": (i32, [vp, i32, vp, vp, vp, vp, vp, vp, P(ff_eig_params), vp, vp, vp, vp,
                                     vp]),
        "eig_bounds": (i32, [vp, i32, i32, vp, vp]),
        "chebyshev_apply": (i32, [vp, i64, vp, vp, vp, vp, vp, i32, i32, f64, i32, f64, vp, i64, vp, i64, P(f64)]),
        "spmm_hm": (i32, [vp, i64, vp, vp, vp, vp, vp, i32, i32, vp, i64, vp, vp, i64, i32]),
        "spmm_autotune": (i32, [vp, i64, vp, vp, vp, vp, vp, i32, i32, ctypes.c_char_p, P(i32), P(f64)]),
        "gram_hm": (i32, [vp, i64, i32, i32, vp, vp, vp, i64, vp]),
        "rayleigh_ritz": (i32, [vp, i32, i32, vp, f64, vp, vp, P(i32)]),
        "rayleigh_ritz_noalloc": (i32, [vp, i32, i32, vp, f64, vp, vp, P(i32)]),
        "spmm_variant_count": (i32, []),
        "spmm_variant_name": (ctypes.c_char_p, [i32]),
        "spmm_variant_selected": (i32, [vp, i64, i64, i32, i32]),
        "rowtiles_build": (i32, [vp, i64, vp, vp, vp, vp, i32, P(vp)]),
        "rowtiles_info": (i32, [vp, P(i64), P(i64)]),
        "spmm_rowtiles": (i32, [vp, vp, i32, i32, vp, i64, vp, vp, i64, i32]),
        "rowtiles_destroy": (None, [vp]),
        "mf_build": (i32, [vp, i64, i64, vp, vp, vp, vp, vp, vp, vp, vp, vp, i32, P(vp)]),
        "mf_apply": (i32, [vp, vp, i32, vp, i64, vp, vp, i64]),
        "mf_interpolate": (i32, [vp, vp, i32, vp, i64, vp, i64]),
        "mf_destroy": (None, [vp]),
        "rand_block": (i32, [vp, i64, i32, ctypes.c_uint64, vp]),
        "philox4x32_10": (i32, [vp, i32, vp, vp, vp]),
        "mlp_param_count": (i32, [i32, i32]),
        "mlp_create": (i32, [vp, i32, i32, ctypes.c_uint64, P(vp)]),
        "mlp_destroy": (None, [vp]),
        "mlp_set_params": (i32, [vp, vp]),
        "mlp_get_params": (i32, [vp, vp]),
        "mlp_get_grad": (i32, [vp, vp]),
        "mlp_inputs": (i32, [vp, i64, vp, vp, i32, vp]),
        "mlp_forward": (i32, [vp, i64, vp, vp, i64]),
        "mlp_train_step": (i32, [vp, i64, vp, vp, i64, vp, ctypes.c_float, P(f64)]),
        "lumped_mass": (i32, [vp, i64, vp, vp, vp]),
        "block_blend": (i32, [vp, i64, i32, vp, i64, vp, i64, f64]),
        "sym_build": (i32, [vp, i64, vp, vp, vp, vp, i32, P(vp)]),
        "sym_info": (i32, [vp, P(i64), P(i64)]),
        "spmm_sym": (i32, [vp, vp, i32, vp, i64, vp, vp, i64]),
        "sym_destroy": (None, [vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def _p(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


_POISON = os.environ.get("FF_POISON_OUTPUTS") == "1"


def _out(shape, dtype, device):
    """A buffer for the library to fill: uninitialised, or, with FF_POISON_OUTPUTS=1 (the tests set
    it), filled with NaN (floating point) or -1 (integers), so that an element the library fails to
    write cannot pass on what earlier work left in the same memory."""
    import torch
    if not _POISON:
        return torch.empty(shape, dtype=dtype, device=device)
    shape = (int(shape),) if isinstance(shape, (int, np.integer)) else tuple(shape)
    if dtype.is_floating_point:
        fill = float("nan")
    else:
        fill = -1 if dtype.is_signed else torch.iinfo(dtype).max
    return torch.full(shape, fill, dtype=dtype, device=device)


class Context:
    """A library context bound to a device and the current torch stream."""

    def __init__(self, device: int = 0, stream=None):
        import torch
        self.device = device
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.stream = stream
        h = ctypes.c_void_p()
        rc = lib().ff_ctx_create(ctypes.byref(h), device, ctypes.c_void_p(stream.cuda_stream))
        if rc != 0:
            raise FFError(rc, "ff_ctx_create failed")
        self.h = h
        self._children = weakref.WeakSet()   # handles that must be released before the context

    def check(self, rc: int):
        if rc != 0:
            raise FFError(rc, lib().ff_last_error(self.h).decode())

    def set_stage_timing(self, enable: bool):
        """Per-stage HIP-event timing of the eigensolver (off by default)."""
        self.check(lib().ff_ctx_set_stage_timing(self.h, int(bool(enable))))

    def stage_times(self):
        """{stage name: (milliseconds, launches)} of the last eigenmodes call."""
        L = lib()
        n = L.ff_ctx_stage_times(self.h, 0, None, None)
        if n < 0:
            self.check(n)
        ms = (ctypes.c_double * n)()
        la = (ctypes.c_int64 * n)()
        L.ff_ctx_stage_times(self.h, n, ms, la)
        return {L.ff_stage_name(i).decode(): (ms[i], la[i]) for i in range(n)}

    def close(self):
        if self.h:
            for c in list(self._children):
                c.close()
            lib().ff_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


@dataclass
class Neighbors:
    grid: ff_grid
    perm: "object"
    xyz_sorted: "object"
    cell_start: "object"
    nbr_off: "object"
    nbr_id: "object"


def build_neighbors(ctx: Context, xyz, h: float, qxyz=None) -> Neighbors:
    import torch
    dev = xyz.device
    xyz = xyz.contiguous()
    n = xyz.shape[0]
    q = n if qxyz is None else qxyz.shape[0]
    grid = ff_grid()
    perm = _out(n, torch.int32, dev)
    xs = _out((n, 3), torch.float64, dev)
    off = _out(q + 1, torch.int64, dev)
    tot = ctypes.c_int64()
    L = lib()
    ctx.check(L.build_neighbors(ctx.h, n, _p(xyz), q, _p(qxyz), float(h), ctypes.byref(grid), _p(perm), _p(xs),
                                None, 0, _p(off), None, 0, ctypes.byref(tot)))
    cs = _out(grid.n_cells + 1, torch.int64, dev)
    ids = _out(max(tot.value, 1), torch.int32, dev)
    ctx.check(L.build_neighbors(ctx.h, n, _p(xyz), q, _p(qxyz), float(h), ctypes.byref(grid), _p(perm), _p(xs),
                                _p(cs), cs.numel(), _p(off), _p(ids), ids.numel(), ctypes.byref(tot)))
    return Neighbors(grid, perm, xs, cs, off, ids[:tot.value])


def rkpm_shape(ctx: Context, xyz_sorted, nbr_off, nbr_id, h: float, qxyz=None, kernel: int = 0,
               features: bool = False):
    import torch
    dev = xyz_sorted.device
    n = xyz_sorted.shape[0]
    q = nbr_off.shape[0] - 1
    tot = nbr_id.shape[0]
    phi = _out(max(tot, 1), torch.float64, dev)
    dphi = _out((max(tot, 1), 3), torch.float64, dev)
    feat = _out((q, 8), torch.float32, dev) if features else None
    bad = ctypes.c_int64(-1)
    rc = lib().rkpm_shape(ctx.h, n, _p(xyz_sorted), q, _p(qxyz), _p(nbr_off), _p(nbr_id), tot, float(h), kernel,
                          _p(phi), _p(dphi), _p(feat), ctypes.byref(bad))
    if rc != 0:
        e = FFError(rc, lib().ff_last_error(ctx.h).decode())
        e.bad_index = bad.value
        raise e
    return phi[:tot], dphi[:tot], feat


def build_neighbors_radii(ctx: Context, xyz, radius, qxyz) -> Neighbors:
    """Neighbour lists d^2 < R_j^2 with a support radius per node (original order)."""
    import torch
    dev = xyz.device
    xyz = xyz.contiguous()
    radius = radius.contiguous()
    qxyz = qxyz.contiguous()
    n, q = xyz.shape[0], qxyz.shape[0]
    if radius.dtype != torch.float64 or radius.shape != (n,):
        raise FFError(FF_ERR_INVALID_ARG, "radius must be float64 [n]")
    grid = ff_grid()
    perm = _out(n, torch.int32, dev)
    xs = _out((n, 3), torch.float64, dev)
    off = _out(q + 1, torch.int64, dev)
    tot = ctypes.c_int64()
    L = lib()
    ctx.check(L.build_neighbors_radii(ctx.h, n, _p(xyz), _p(radius), q, _p(qxyz), ctypes.byref(grid), _p(perm),
                                      _p(xs), None, 0, _p(off), None, 0, ctypes.byref(tot)))
    cs = _out(grid.n_cells + 1, torch.int64, dev)
    ids = _out(max(tot.value, 1), torch.int32, dev)
    ctx.check(L.build_neighbors_radii(ctx.h, n, _p(xyz), _p(radius), q, _p(qxyz), ctypes.byref(grid), _p(perm),
                                      _p(xs), _p(cs), cs.numel(), _p(off), _p(ids), ids.numel(), ctypes.byref(tot)))
    return Neighbors(grid, perm, xs, cs, off, ids[:tot.value])


def fps_centers(ctx: Context, qxyz, K: int, start: int = 0):
    """(indices [K] int32, centres [K][3]) of farthest point sampling over the points."""
    import torch
    qxyz = qxyz.contiguous()
    idx = _out(K, torch.int32, qxyz.device)
    cen = _out((K, 3), torch.float64, qxyz.device)
    ctx.check(lib().fps_centers(ctx.h, qxyz.shape[0], _p(qxyz), K, start, _p(idx), _p(cen)))
    return idx, cen


def kernel_radii(ctx: Context, centres, cut: float = 3.0):
    """(r, R): each centre's Gaussian radius (distance to its 2nd-nearest centre) and cut * r."""
    import torch
    centres = centres.contiguous()
    K = centres.shape[0]
    r = _out(K, torch.float64, centres.device)
    R = _out(K, torch.float64, centres.device)
    ctx.check(lib().kernel_radii(ctx.h, K, _p(centres), float(cut), _p(r), _p(R)))
    return r, R


def rkpm_shape_radii(ctx: Context, xyz_sorted, node_r, nbr_off, nbr_id, h: float, qxyz, cut: float = 3.0,
                     basis: int = 2, perm=None):
    import torch
    dev = xyz_sorted.device
    n = xyz_sorted.shape[0]
    q = nbr_off.shape[0] - 1
    tot = nbr_id.shape[0]
    qxyz = qxyz.contiguous()
    phi = _out(max(tot, 1), torch.float64, dev)
    dphi = _out((max(tot, 1), 3), torch.float64, dev)
    bad = ctypes.c_int64(-1)
    rc = lib().rkpm_shape_radii(ctx.h, n, _p(xyz_sorted), _p(node_r.contiguous()), _p(perm), q, _p(qxyz),
                                _p(nbr_off), _p(nbr_id), tot, float(h), float(cut), int(basis), _p(phi), _p(dphi),
                                ctypes.byref(bad))
    if rc != 0:
        e = FFError(rc, lib().ff_last_error(ctx.h).decode())
        e.bad_index = bad.value
        raise e
    return phi[:tot], dphi[:tot]


def assemble_HM(ctx: Context, n: int, nbr_off, nbr_id, phi, dphi, vol, lam, mu, grid: ff_grid, cell_start,
                rho=None, perm=None, fp32: bool = True):
    import torch
    dev = phi.device
    q = nbr_off.shape[0] - 1
    row_ptr = _out(n + 1, torch.int64, dev)
    nnz = ctypes.c_int64()
    L = lib()
    args = (ctx.h, n, q, _p(nbr_off), _p(nbr_id), _p(phi), _p(dphi), _p(vol), _p(lam), _p(mu), _p(rho), _p(perm),
            ctypes.byref(grid), _p(cell_start), _p(row_ptr))
    ctx.check(L.assemble_HM(*args, None, None, None, None, 0, ctypes.byref(nnz)))
    m = nnz.value
    col = _out(max(m, 1), torch.int32, dev)
    H = _out(max(m, 1), torch.float64, dev)
    M = _out(max(m, 1), torch.float64, dev)
    hm32 = _out((max(m, 1), 2), torch.float32, dev) if fp32 else None
    ctx.check(L.assemble_HM(*args, _p(col), _p(H), _p(M), _p(hm32), m, ctypes.byref(nnz)))
    return row_ptr, col[:m], H[:m], M[:m], (hm32[:m] if fp32 else None)


def _params(k, block, precision, tol, max_iter, precond, seed, check_every, use_graph, refresh_every,
            precond_degree=0, precond_ratio=0.0, precond_values=0, eig_tol=0.0, angle_tol=0.0):
    return ff_eig_params(k, block, precision, tol, max_iter, precond, seed, check_every, int(use_graph),
                         refresh_every, precond_degree, float(precond_ratio), precond_values, float(eig_tol),
                         float(angle_tol))


def _info_dict(i):
    return dict(iters_fp32=i.iters_fp32, iters_fp64=i.iters_fp64, converged=i.converged, restarts=i.restarts,
                max_resid=i.max_resid, seconds=i.seconds, graph=i.graph, max_eig_bound=i.max_eig_bound,
                max_angle_bound=i.max_angle_bound, eig_certified=i.eig_certified)


def eigenmodes(ctx: Context, n: int, row_ptr, col, H, M, hm32, k: int, block: int = 0, precision: int = 1,
               tol: float = 1e-6, max_iter: int = 5000, precond: int = 2, seed: int = 0, X0=None,
               check_every: int = 10, use_graph: bool = False, refresh_every: int = 0, allow_unconverged=False,
               precond_degree: int = 0, precond_ratio: float = 0.0, precond_values: int = 0, eig_tol: float = 0.0,
               angle_tol: float = 0.0):
    import torch
    p = _params(k, block, precision, tol, max_iter, precond, seed, check_every, use_graph, refresh_every,
                precond_degree, precond_ratio, precond_values, eig_tol, angle_tol)
    m = block if block > 0 else (k + 7) // 8 * 8
    _check_block(X0, n, m, H.device)
    lam = np.zeros(k)
    res = np.zeros(k)
    W = _out((n, k), torch.float64, H.device)
    info = ff_eig_info()
    rc = lib().eigenmodes(ctx.h, n, _p(row_ptr), _p(col), _p(H), _p(M), _p(hm32), ctypes.byref(p),
                          _p(X0), lam.ctypes.data_as(vp), _p(W), res.ctypes.data_as(vp), ctypes.byref(info))
    out = _info_dict(info)
    out["status"] = rc
    if rc != 0 and not (allow_unconverged and rc == FF_ERR_NOT_CONVERGED):
        ctx.check(rc)
    return lam, W, res, out


def eigenmodes_batched(ctx: Context, obj_row_off, row_ptr, col, H, M, hm32, k: int, block: int = 0,
                       precision: int = 1, tol: float = 1e-6, max_iter: int = 5000, precond: int = 2,
                       seed: int = 0, X0=None, check_every: int = 10, use_graph: bool = False,
                       refresh_every: int = 0, allow_unconverged=False, precond_degree: int = 0,
                       precond_ratio: float = 0.0, precond_values: int = 0, eig_tol: float = 0.0,
                       angle_tol: float = 0.0):
    import torch
    off = np.ascontiguousarray(obj_row_off, dtype=np.int64)
    n_obj = len(off) - 1
    N = int(off[-1])
    p = _params(k, block, precision, tol, max_iter, precond, seed, check_every, use_graph, refresh_every,
                precond_degree, precond_ratio, precond_values, eig_tol, angle_tol)
    _check_block(X0, N, block if block > 0 else (k + 7) // 8 * 8, H.device)
    lam = np.zeros((n_obj, k))
    res = np.zeros((n_obj, k))
    W = _out((N, k), torch.float64, H.device)
    info = (ff_eig_info * n_obj)()
    rc = lib().eigenmodes_batched(ctx.h, n_obj, off.ctypes.data_as(vp), _p(row_ptr), _p(col), _p(H), _p(M),
                                  _p(hm32), ctypes.byref(p), _p(X0), lam.ctypes.data_as(vp), _p(W),
                                  res.ctypes.data_as(vp), ctypes.cast(info, vp))
    infos = [_info_dict(i) for i in info]
    if rc != 0 and not (allow_unconverged and rc == FF_ERR_NOT_CONVERGED):
        ctx.check(rc)
    return lam, W, res, infos, rc


def eig_bounds(ctx: Context, n_obj: int, k: int):
    """(eig_bound, angle_bound), each [n_obj][k], of the last eigensolve on the context."""
    e = np.zeros((n_obj, k))
    a = np.zeros((n_obj, k))
    ctx.check(lib().eig_bounds(ctx.h, n_obj, k, e.ctypes.data_as(vp), a.ctypes.data_as(vp)))
    return e, a


def chebyshev_apply(ctx: Context, n: int, row_ptr, col, H, M, hm32, R, degree: int = 12, ratio: float = 0.0,
                    values: int = 1, upper: float = 0.0):
    """(Z, b): Z = q(D^-1 H) D^-1 R, the eigensolver's preconditioner alone on one object, R a
    float32 [n][m] block on the device; b the interval's upper end taken (upper, or the library's
    estimate when 0). With values 3 and 4 each column of Z is scaled by 1 / max |D^-1 r|."""
    import torch
    if R.dtype != torch.float32 or R.dim() != 2 or R.shape[0] != n or R.stride(1) != 1:
        raise FFError(FF_ERR_INVALID_ARG, f"R must be a float32 [{n}][m] block with unit column stride")
    Z = _out((n, R.shape[1]), torch.float32, R.device)
    b = ctypes.c_double()
    ctx.check(lib().chebyshev_apply(ctx.h, n, _p(row_ptr), _p(col), _p(H), _p(M), _p(hm32), R.shape[1], degree,
                                    float(ratio), values, float(upper), _p(R), R.stride(0), _p(Z), Z.stride(0),
                                    ctypes.byref(b)))
    return Z, b.value


def _check_block(X0, n, m, device):
    """A starting block must be FP64, contiguous, on the solver's device and [n][m] (the library
    reads n * m doubles from it)."""
    import torch
    if X0 is None:
        return
    if X0.dtype != torch.float64 or not X0.is_contiguous() or X0.device != device or tuple(X0.shape) != (n, m):
        raise FFError(FF_ERR_INVALID_ARG, f"X0 must be a contiguous float64 [{n}][{m}] tensor on {device}, got "
                      f"{X0.dtype} {tuple(X0.shape)} on {X0.device} (contiguous={X0.is_contiguous()})")


def spmm_hm(ctx: Context, row_ptr, col, H, M, hm32, Y, precision: int, variant: int = -1, out=None):
    import torch
    n, m = Y.shape
    if out is None:
        HY = _out(Y.shape, Y.dtype, Y.device)
        MY = _out(Y.shape, Y.dtype, Y.device)
    else:
        HY, MY = out
    ctx.check(lib().spmm_hm(ctx.h, n, _p(row_ptr), _p(col), _p(H), _p(M), _p(hm32), precision, m, _p(Y),
                            Y.stride(0), _p(HY), _p(MY), HY.stride(0), variant))
    return HY, MY


def spmm_autotune(ctx: Context, n: int, row_ptr, col, H, M, hm32, precision: int, m: int,
                  cache_path: Optional[str] = None):
    best = ctypes.c_int()
    ms = ctypes.c_double()
    ctx.check(lib().spmm_autotune(ctx.h, n, _p(row_ptr), _p(col), _p(H), _p(M), _p(hm32), precision, m,
                                  None if cache_path is None else cache_path.encode(), ctypes.byref(best),
                                  ctypes.byref(ms)))
    return best.value, ms.value


def gram_hm(ctx: Context, S, HS, MS, w: int = None):
    """G[0] = S^T HS, G[1] = S^T MS over the first w columns (FP64 result)."""
    import torch
    n = S.shape[0]
    w = S.shape[1] if w is None else w
    precision = 1 if S.dtype == torch.float32 else 0
    G = _out((2, w, w), torch.float64, S.device)
    ctx.check(lib().gram_hm(ctx.h, n, w, precision, _p(S), _p(HS), _p(MS), S.stride(0), _p(G)))
    return G


def rayleigh_ritz(ctx: Context, G, m: int, tau: float = 1e-13):
    import torch
    w = G.shape[1]
    C = _out((w, m), torch.float64, G.device)
    theta = _out(m, torch.float64, G.device)
    kept = ctypes.c_int()
    ctx.check(lib().rayleigh_ritz(ctx.h, w, m, _p(G.contiguous()), tau, _p(C), _p(theta), ctypes.byref(kept)))
    return theta, C, kept.value


class RowTiles:
    """Handle of an ff_rowtiles copy of [H, M] (tiles of four rows sharing one column list)."""

    def __init__(self, ctx: Context, n: int, row_ptr, col, H, M, precision: int = 1):
        self.ctx = ctx
        self.h = None
        h = ctypes.c_void_p()
        ctx.check(lib().rowtiles_build(ctx.h, n, _p(row_ptr), _p(col), _p(H), _p(M), precision, ctypes.byref(h)))
        self.h = h
        ctx._children.add(self)

    def info(self):
        nt, ne = ctypes.c_int64(), ctypes.c_int64()
        lib().rowtiles_info(self.h, ctypes.byref(nt), ctypes.byref(ne))
        return nt.value, ne.value

    def spmm(self, Y, precision: int, sub: int = 0, out=None, h_only: bool = False):
        """[HY, MY] = [H, M] Y; with h_only, (HY, None) from the preconditioner's product.
        precision 2 takes a binary16 Y (a handle built with precision 6) and returns HY in FP32."""
        import torch
        n, m = Y.shape
        if precision == 2:
            if Y.dtype != torch.float16:
                raise TypeError("precision 2 takes a float16 block")
            h_only = True
        if out is None:
            HY = _out(Y.shape, torch.float32 if precision == 2 else Y.dtype, Y.device)
            MY = None if h_only else _out(Y.shape, Y.dtype, Y.device)
        else:
            HY, MY = out
            if h_only:
                MY = None
        self.ctx.check(lib().spmm_rowtiles(self.ctx.h, self.h, precision, m, _p(Y), Y.stride(0), _p(HY),
                                           None if MY is None else _p(MY), HY.stride(0), sub))
        return HY, MY

    def close(self):
        if self.h:
            lib().rowtiles_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class SymCSR:
    """Handle of an ff_sym copy of [H, M]: the upper triangles' values and, per lower entry, the
    position of its mirror (sym_build); precision 0 keeps FP64 values, 1 FP32."""

    def __init__(self, ctx: Context, n: int, row_ptr, col, H, M=None, precision: int = 0):
        self.ctx = ctx
        self.h = None
        self.n = n
        self.precision = precision
        self.has_m = M is not None
        h = ctypes.c_void_p()
        ctx.check(lib().sym_build(ctx.h, n, _p(row_ptr), _p(col), _p(H), _p(M), precision, ctypes.byref(h)))
        self.h = h
        ctx._children.add(self)

    def info(self):
        u, l = ctypes.c_int64(), ctypes.c_int64()
        lib().sym_info(self.h, ctypes.byref(u), ctypes.byref(l))
        return u.value, l.value

    def spmm(self, Y, h_only: bool = False, out=None):
        """(HY, MY) = [H, M] Y for Y [n][m] (float64 at precision 0, float32 at 1); MY is None
        with h_only or a copy built without M."""
        import torch
        dt = torch.float32 if self.precision else torch.float64
        if Y.dtype != dt or Y.dim() != 2 or Y.shape[0] != self.n or Y.stride(1) != 1:
            raise FFError(FF_ERR_INVALID_ARG, f"Y must be [{self.n}][m] {dt} with unit column stride")
        want_m = self.has_m and not h_only
        if out is None:
            HY = _out(Y.shape, dt, Y.device)
            MY = _out(Y.shape, dt, Y.device) if want_m else None
        else:
            HY, MY = out
            MY = MY if want_m else None
        self.ctx.check(lib().spmm_sym(self.ctx.h, self.h, Y.shape[1], _p(Y), Y.stride(0), _p(HY), _p(MY),
                                      HY.stride(0)))
        return HY, MY

    def close(self):
        if self.h:
            lib().sym_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class MatFree:
    """Handle of the matrix-free products [H Y, M Y] = [G^T D G Y, Phi^T V Phi Y] (mf_build)."""

    def __init__(self, ctx: Context, n: int, nbr_off, nbr_id, phi, dphi, vol, lam, mu, rho=None, perm=None,
                 precision: int = 1):
        self.ctx = ctx
        self.h = None
        self.n = n
        self.q = nbr_off.shape[0] - 1
        self.precision = precision
        self._keep = (nbr_off, nbr_id)          # the handle reads these lists on every product
        h = ctypes.c_void_p()
        ctx.check(lib().mf_build(ctx.h, n, self.q, _p(nbr_off), _p(nbr_id), _p(phi), _p(dphi), _p(vol), _p(lam),
                                 _p(mu), _p(rho), _p(perm), precision, ctypes.byref(h)))
        self.h = h
        ctx._children.add(self)

    def apply(self, Y, h: bool = True, m: bool = True, out=None):
        """(HY, MY) for Y [n][m] (float32 at precision 1, float64 at 0); either may be skipped."""
        import torch
        dt = torch.float32 if self.precision else torch.float64
        if Y.dtype != dt or Y.shape[0] != self.n or Y.stride(1) != 1:
            raise FFError(FF_ERR_INVALID_ARG, f"Y must be [{self.n}][m] {dt} with unit column stride")
        k = Y.shape[1]
        if out is None:
            HY = _out((self.n, k), dt, Y.device) if h else None
            MY = _out((self.n, k), dt, Y.device) if m else None
        else:
            HY, MY = out
        ld = (HY if HY is not None else MY).stride(0)
        self.ctx.check(lib().mf_apply(self.ctx.h, self.h, k, _p(Y), Y.stride(0), _p(HY), _p(MY), ld))
        return HY, MY

    def interpolate(self, Y):
        """U [q][m] = Phi Y: the fields at the integration points."""
        import torch
        dt = torch.float32 if self.precision else torch.float64
        if Y.dtype != dt or Y.shape[0] != self.n or Y.stride(1) != 1:
            raise FFError(FF_ERR_INVALID_ARG, f"Y must be [{self.n}][m] {dt} with unit column stride")
        U = _out((self.q, Y.shape[1]), dt, Y.device)
        self.ctx.check(lib().mf_interpolate(self.ctx.h, self.h, Y.shape[1], _p(Y), Y.stride(0), _p(U), U.stride(0)))
        return U

    def close(self):
        if self.h:
            lib().mf_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def spmm_variant_selected(ctx: Context, n: int, nnz: int, m: int, precision: int) -> int:
    v = lib().spmm_variant_selected(ctx.h, n, nnz, m, precision)
    ctx.check(min(v, 0))
    return v


def spmm_variant_names():
    L = lib()
    return [L.spmm_variant_name(i).decode() for i in range(L.spmm_variant_count())]


def rand_block(ctx: Context, n: int, m: int, seed: int, device="cuda"):
    import torch
    out = _out((n, m), torch.float64, device)
    ctx.check(lib().rand_block(ctx.h, n, m, seed, _p(out)))
    return out


def philox4x32_10(ctx: Context, ctr, key):
    """ctr: uint32 tensor (count, 4), key: (count, 2) on the device; returns (count, 4)."""
    import torch
    out = _out(ctr.shape, ctr.dtype, ctr.device)
    ctx.check(lib().philox4x32_10(ctx.h, ctr.shape[0], _p(ctr), _p(key), _p(out)))
    return out


# ----------------------------------------------------------------------------
# learned warm start
# ----------------------------------------------------------------------------

def mlp_param_count(k: int, n_in: int = 11) -> int:
    return lib().mlp_param_count(k, n_in)


class MLP:
    """Handle of an ff_mlp (the warm-start network) on a context."""

    def __init__(self, ctx: Context, k: int, n_in: int = 11, seed: int = 0):
        self.ctx = ctx
        self.k = k
        self.n_in = n_in
        self.h = None
        self.P = mlp_param_count(k, n_in)
        if self.P < 0:
            raise FFError(FF_ERR_INVALID_ARG, f"k = {k} or n_in = {n_in} out of range")
        h = ctypes.c_void_p()
        ctx.check(lib().mlp_create(ctx.h, k, n_in, seed, ctypes.byref(h)))
        self.h = h
        ctx._children.add(self)

    def close(self):
        if self.h:
            lib().mlp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, params):
        a = np.ascontiguousarray(params, dtype=np.float32)
        assert a.size == self.P
        self.ctx.check(lib().mlp_set_params(self.h, a.ctypes.data_as(vp)))

    def get_params(self):
        a = np.empty(self.P, dtype=np.float32)
        self.ctx.check(lib().mlp_get_params(self.h, a.ctypes.data_as(vp)))
        return a

    def get_grad(self):
        a = np.empty(self.P, dtype=np.float32)
        self.ctx.check(lib().mlp_get_grad(self.h, a.ctypes.data_as(vp)))
        return a

    def _check_in(self, x):
        if x.shape[1] != self.n_in or x.stride(0) != self.n_in:
            raise FFError(FF_ERR_INVALID_ARG, f"inputs must be contiguous [n][{self.n_in}]")

    def forward(self, x, ldy: Optional[int] = None, out=None):
        """Y [n][ldy] FP64 with the first k columns written."""
        import torch
        self._check_in(x)
        n = x.shape[0]
        if out is None:
            out = torch.zeros((n, ldy or self.k), dtype=torch.float64, device=x.device)
        self.ctx.check(lib().mlp_forward(self.h, n, _p(x), _p(out), out.stride(0)))
        return out

    def train_step(self, x, T, d, lr: float) -> float:
        self._check_in(x)
        loss = ctypes.c_double()
        self.ctx.check(lib().mlp_train_step(self.h, x.shape[0], _p(x), _p(T), T.stride(0), _p(d), lr,
                                            ctypes.byref(loss)))
        return loss.value


def mlp_inputs(ctx: Context, xyz_sorted, feat, n_freq: int = 0):
    import torch
    n = xyz_sorted.shape[0]
    out = _out((n, 11 + 6 * n_freq), torch.float32, xyz_sorted.device)
    ctx.check(lib().mlp_inputs(ctx.h, n, _p(xyz_sorted), _p(feat), n_freq, _p(out)))
    return out


def lumped_mass(ctx: Context, n: int, row_ptr, M):
    import torch
    d = _out(n, torch.float64, M.device)
    ctx.check(lib().lumped_mass(ctx.h, n, _p(row_ptr), _p(M), _p(d)))
    return d


def block_blend(ctx: Context, X, R, w: float):
    """In place, column by column: X_c <- X_c / rms(X_c) + w R_c / rms(R_c) (FP64 [n][m] blocks on
    the device, unit column stride). Returns X."""
    import torch
    for name, A in (("X", X), ("R", R)):
        if A.dtype != torch.float64 or A.dim() != 2 or A.stride(1) != 1:
            raise FFError(FF_ERR_INVALID_ARG, f"{name} must be a float64 [n][m] block with unit column stride")
    if tuple(R.shape) != tuple(X.shape) or R.device != X.device:
        raise FFError(FF_ERR_INVALID_ARG, "X and R must have the same shape and device")
    ctx.check(lib().block_blend(ctx.h, X.shape[0], X.shape[1], _p(X), X.stride(0), _p(R), R.stride(0), float(w)))
    return X


# ----------------------------------------------------------------------------
# convenience: the whole path for one synthetic cloud
# ----------------------------------------------------------------------------

@dataclass
class Assembled:
    n: int
    h: float
    nb: Neighbors
    phi: "object"
    dphi: "object"
    feat: "object"
    row_ptr: "object"
    col: "object"
    H: "object"
    M: "object"
    hm32: "object"


def assemble_cloud(ctx: Context, xyz, vol, lam, mu, h: float, rho=None, features: bool = False,
                   kernel: int = 0) -> Assembled:
    """build_neighbors -> rkpm_shape -> assemble_HM; per-point arrays in original order."""
    nb = build_neighbors(ctx, xyz, h)
    phi, dphi, feat = rkpm_shape(ctx, nb.xyz_sorted, nb.nbr_off, nb.nbr_id, h, kernel=kernel, features=features)
    n = xyz.shape[0]
    rp, col, H, M, hm32 = assemble_HM(ctx, n, nb.nbr_off, nb.nbr_id, phi, dphi, vol, lam, mu, nb.grid,
                                      nb.cell_start, rho=rho, perm=nb.perm)
    return Assembled(n, h, nb, phi, dphi, feat, rp, col, H, M, hm32)


@dataclass
class PaperAssembled:
    """The paper's construction on the device (Supp. B.1): FPS centres, radii, lists, shape
    functions, H and M in sorted centre numbering."""
    K: int
    pick: "object"
    centres: "object"
    r: "object"
    R: "object"
    nb: Neighbors
    phi: "object"
    dphi: "object"
    row_ptr: "object"
    col: "object"
    H: "object"
    M: "object"
    hm32: "object"


def paper_construction(ctx: Context, qxyz, vol, lam, mu, K: int, cut: float = 3.0, basis: int = 2,
                       start: int = 0, rho=None) -> PaperAssembled:
    """fps_centers -> kernel_radii -> build_neighbors_radii -> rkpm_shape_radii -> assemble_HM, with
    the integration points as quadrature points (their arrays in their own order)."""
    pick, cen = fps_centers(ctx, qxyz, K, start)
    r, R = kernel_radii(ctx, cen, cut)
    nb = build_neighbors_radii(ctx, cen, R, qxyz)
    phi, dphi = rkpm_shape_radii(ctx, nb.xyz_sorted, r, nb.nbr_off, nb.nbr_id, nb.grid.h, qxyz, cut, basis,
                                 perm=nb.perm)
    rp, col, H, M, hm32 = assemble_HM(ctx, K, nb.nbr_off, nb.nbr_id, phi, dphi, vol, lam, mu, nb.grid,
                                      nb.cell_start, rho=rho)
    return PaperAssembled(K, pick, cen, r, R, nb, phi, dphi, rp, col, H, M, hm32)


def concat_objects(parts):
    """Block-diagonal concatenation of assembled objects for eigenmodes_batched.

    Marshalling only: CSR arrays are concatenated and column / row-pointer
    offsets shifted with torch; returns (obj_row_off (numpy), row_ptr, col, H, M, hm32).
    """
    import torch
    offs = [0]
    rps, cols, Hs, Ms, hms = [], [], [], [], []
    nnz_off = 0
    for a in parts:
        rp = a.row_ptr
        rps.append((rp[:-1] if len(rps) < len(parts) - 1 else rp) + nnz_off)
        cols.append(a.col + offs[-1])
        Hs.append(a.H)
        Ms.append(a.M)
        hms.append(a.hm32)
        nnz_off += int(a.col.numel())
        offs.append(offs[-1] + a.n)
    return (np.array(offs, dtype=np.int64), torch.cat(rps), torch.cat(cols).to(torch.int32), torch.cat(Hs),
            torch.cat(Ms), torch.cat(hms))
