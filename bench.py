"""Benchmark: seconds to the 32 smallest skinning eigenmodes of a 1,000,000-particle object.

One step is the whole subspace-construction path on one synthetic object:
cell binning and neighbour lists, RKPM shape functions, assembly of H and M,
and the mixed-precision LOBPCG (FP32 products, FP64 Rayleigh-Ritz, FP64
certification) to residual 1e-6. Inputs are generated on the host once and
are resident in HBM before the timed region. Step s starts the eigensolver
from the seeded random block of seed s (the iteration count depends on the
start), so the reported time is a mean over starts.

Workload: 1,000,000 particles drawn uniformly inside a seeded union of 20
random ellipsoids (semi-axes U(0.05, 0.4)) clipped to the unit box,
per-particle E log-uniform in [1e4, 1e6] Pa and nu uniform in [0.3, 0.48],
support radius 2.5 x mean spacing, k = 32 (constant mode included).

Also reported (same JSON line): the plain FP64 path on the same object, the
per-stage device times of the timed solve (HIP events the library records on
its stream), the achieved HBM rate of the dominant kernel (the Chebyshev step:
H-only product fused with the preconditioner's vector update) against the
MI355X peak, and the FP64 CPU oracle timed on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "s to 32 eigenmodes @1M particles (resid≤1e-6), mixed vs FP64; SpMM GB/s"
HBM_PEAK_GBS = 8000.0
PRECOND = 2            # Chebyshev-Jacobi
PRECOND_DEGREE = 0     # library default


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def run_step(ff, ctx, dev_in, n, h, k, precision, tol, max_iter, use_graph=False, seed=0, eig_tol=0.0):
    import torch
    xyz, vol, lam, mu = dev_in
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    A = ff.assemble_cloud(ctx, xyz, vol, lam, mu, h)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ev, W, res, info = ff.eigenmodes(ctx, n, A.row_ptr, A.col, A.H, A.M, A.hm32, k=k, precision=precision,
                                     tol=tol, max_iter=max_iter, use_graph=use_graph, allow_unconverged=True,
                                     precond=PRECOND, precond_degree=PRECOND_DEGREE, seed=seed, eig_tol=eig_tol)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    return dict(total=t2 - t0, build=t1 - t0, solve=t2 - t1, ev=ev, res=res, info=info, A=A, W=W)


KERNEL_SRC = os.path.join(ROOT, "paper_2605_29318_amd", "csrc", "k_rowtile.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "cheb_step_ellipsoids1m_k32_hbm_traffic.txt")


def kernel_source_hash():
    import hashlib
    return hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()[:16]


def cheb_step_bytes(nnz, n, m, value_bytes=2, iter_bytes=2, degree=12):
    """Algorithmic HBM bytes of one Chebyshev step launch (m columns), independent of the
    tiling, averaged over the degree - 1 steps of one application: the H value (binary16,
    value_bytes) and int32 column of every nonzero, the row pointers, D^-1 and the row's
    object index, the iterate DZ (binary16, iter_bytes) read once and the next one written,
    R (FP32) read and written, and W (FP32) read and written at ceil((degree - 1) / 2) of the
    steps (every second step adds two iterates, the last step its own when the count is odd)."""
    steps = degree - 1
    w_frac = ((steps + 1) // 2) / steps
    return nnz * (value_bytes + 4) + 8 * (n + 1) + n * (4 + 4) + n * m * (2 * iter_bytes + 8 + 8 * w_frac)


def spmm_hm_bytes(nnz, n, m):
    """Algorithmic HBM bytes of one fused [H, M] Y launch (FP32): H, M values and a column
    per nonzero, the row pointers, Y read once, HY and MY written."""
    return nnz * 12 + 8 * (n + 1) + 4 * n * m + 8 * n * m


def measured_traffic():
    """HBM bytes per Chebyshev step launch from the committed counter summary (FETCH_SIZE
    and WRITE_SIZE passes, each scaled by the same counter on a copy of known size), or
    None when the summary is missing or was taken on another version of the kernel."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    vals = {}
    for line in open(TRAFFIC_FILE):
        if ":" in line:
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def stream_copy_gbps():
    """Achievable HBM bandwidth on this device: a 1 GiB device-to-device copy (reads and writes
    1 GiB), mean of 10 after 3 untimed, timed with events on torch's stream."""
    import torch
    src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(10):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / 10
    del src, dst
    return 2 * (1 << 30) / (ms * 1e-3) / 1e9


def counters_run(args):
    """Counter-collection helper: a short solve of the benchmark workload (its Chebyshev
    step and SpMM launches) and an elementwise kernel that reads and writes 1 GiB (the
    counters' calibration)."""
    import numpy as np
    import torch
    from paper_2605_29318_amd import freeform as ff
    from paper_2605_29318_amd import synth
    c = synth.ellipsoid_union(n=args.n, seed=3, hetero=True, k=args.k, mc_samples=4_000_000)
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a), device="cuda")
    ctx = ff.Context(0)
    A = ff.assemble_cloud(ctx, dev(c.xyz), dev(c.vol), dev(c.lam), dev(c.mu), c.h)
    ff.eigenmodes(ctx, c.n, A.row_ptr, A.col, A.H, A.M, A.hm32, k=args.k, precision=1, tol=args.tol,
                  max_iter=args.steps, allow_unconverged=True, precond=PRECOND, precond_degree=PRECOND_DEGREE)
    src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")     # 1 GiB
    dst = torch.empty_like(src)
    for _ in range(3):
        torch.mul(src, 1.0, out=dst)
    torch.cuda.synchronize()
    log(f"[bench] counters: {args.steps} solver iterations, 3 calibration passes over 1 GiB")
    ctx.close()


CPU_LEG = r"""
import json, os, sys, time
sys.path.insert(0, sys.argv[1])
from oracle import oracle as O
from paper_2605_29318_amd import synth
n, k, tol = int(sys.argv[2]), int(sys.argv[3]), float(sys.argv[4])
c = synth.ellipsoid_union(n=n, seed=3, hetero=True, k=k, mc_samples=1_000_000)
O.build()
t = [time.perf_counter()]
perm, cs, origin, dims = O.bin_nodes(c.xyz, c.h)
xs = c.xyz[perm].copy()
off, ids = O.neighbors(xs, xs, c.h, origin, dims, cs)
t.append(time.perf_counter())
phi, dphi = O.rkpm(xs, xs, off, ids, c.h)
t.append(time.perf_counter())
rp, col, H, M = O.assemble(c.n, off, ids, phi, dphi, c.vol[perm], c.lam[perm], c.mu[perm])
t.append(time.perf_counter())
Hs, Ms = O.to_scipy(c.n, rp, col, H), O.to_scipy(c.n, rp, col, M)
lam, W, it, res = O.lobpcg(Hs, Ms, synth.initial_block(c.n, k, seed=1), k=k, tol=tol, maxiter=3000,
                           precond="chebyshev")
t.append(time.perf_counter())
print(json.dumps(dict(n=n, nnz=int(rp[-1]), iters=int(it), max_resid=float(res.max()),
                      stages=dict(binning_neighbours=t[1] - t[0], rkpm=t[2] - t[1], assembly=t[3] - t[2],
                                  eigensolve=t[4] - t[3]))))
"""


def cpu_leg(n_sample, k, tol, threads):
    """The FP64 oracle's own pipeline and its own eigensolver (LOBPCG with its Chebyshev-Jacobi
    preconditioner) to its own convergence on a sample of the benchmark recipe, in a child
    process with the given thread count (OpenMP and BLAS)."""
    import subprocess
    env = dict(os.environ)
    if threads:
        env["OMP_NUM_THREADS"] = env["OPENBLAS_NUM_THREADS"] = str(threads)
    r = subprocess.run([sys.executable, "-c", CPU_LEG, ROOT, str(n_sample), str(k), str(tol)], env=env,
                       capture_output=True, text=True, timeout=900)
    if r.returncode != 0:
        raise RuntimeError(r.stderr[-2000:])
    return json.loads(r.stdout.strip().splitlines()[-1])


def cpu_baseline(k, tol, n_full, n_all=20_000, n_one=5_000):
    """The oracle on bounded samples: on all host cores (n_all particles) and on one core (n_one),
    each stage timed; the projection to n_full scales every stage linearly in the particle count
    at the sample's own iteration count (the GPU's count at n_full is of the same order)."""
    cores = os.cpu_count() or 1
    allc = cpu_leg(n_all, k, tol, None)
    one = cpu_leg(n_one, k, tol, 1)
    scale = n_full / n_all
    est = sum(allc["stages"].values()) * scale
    fmt = lambda d: ", ".join(f"{a} {b:.2f} s" for a, b in d["stages"].items())
    return dict(value=round(est, 1), unit="s", cores=int(os.environ.get("OMP_NUM_THREADS", cores)), kind="oracle",
                sample=(f"the oracle's whole path to its own convergence (its FP64 LOBPCG with its Chebyshev-Jacobi "
                        f"preconditioner, k = {k}, residual {tol:g}) on {n_all} particles of the same recipe "
                        f"on all cores ({fmt(allc)}; {allc['iters']} iterations), every stage scaled linearly to "
                        f"{n_full} particles; on one core, {n_one} particles: {fmt(one)} ({one['iters']} iterations)"),
                all_cores=allc, one_core=one,
                one_core_projection_s=round(sum(one["stages"].values()) * n_full / n_one, 1))


GOLDEN_DIR = os.path.join(ROOT, "tests", "golden")


def golden_eigs(name, cloud, k=32):
    """The oracle's reference eigenvalues of a named workload (stored with the input's SHA-256
    and the residual the oracle's solve reached by tests/golden/make_reference_eigs.py), as
    dict(ev, tol), or None if absent or for another input."""
    import numpy as np
    path = os.path.join(GOLDEN_DIR, f"ref_eigs_{name}_k{k}.json")
    if not os.path.exists(path):
        return None
    d = json.load(open(path))
    if d.get("sha256") != cloud.sha256():
        return None
    return dict(ev=np.array(d["eigenvalues"][:k]), tol=float(d["tol"]))


def eig_rel_err(ev, ref):
    """max over j >= 2 of |lambda_j - ref_j| / ref_j, the signed extremes of (lambda_j - ref_j) / ref_j
    (the reference's Ritz values lie above the exact eigenvalues, by more the larger its residual),
    |lambda_1| / ref_2 for the constant mode, and the reference's residual."""
    import numpy as np
    if ref is None:
        return None
    r = ref["ev"]
    sig = (ev[1:len(r)] - r[1:]) / r[1:]
    return dict(max_rel=float(np.abs(sig).max()), min_signed=float(sig.min()), max_signed=float(sig.max()),
                const_mode=float(abs(ev[0]) / r[1]), reference_residual=ref["tol"])


def time_solves(ff, ctx, dev_in, c, k, precision, seeds, tol, max_iter, eig_tol=0.0):
    out = []
    for sd in seeds:
        r = run_step(ff, ctx, dev_in, c.n, c.h, k, precision, tol, max_iter, seed=sd, eig_tol=eig_tol)
        out.append(r)
    return out


def batched_config(ff, ctx, tol, max_iter):
    """64 sphere-union objects (particle counts log-uniform in 2e3-2e5, E uniform in 1e4-1e6 Pa),
    k = 16, one launch per stage for all objects with the LOBPCG iteration replayed from a hipGraph."""
    import numpy as np
    import torch
    from paper_2605_29318_amd import synth
    t0 = time.perf_counter()
    clouds = synth.batch_objects(count=64, workers=16)
    gen = time.perf_counter() - t0
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a), device="cuda")
    ins = [(dev(c.xyz), dev(c.vol), dev(c.lam), dev(c.mu), c.h) for c in clouds]
    res = []
    for rep in range(2):                      # the first call also autotunes nothing: same shapes both times
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        parts = [ff.assemble_cloud(ctx, *a) for a in ins]
        off, rp, col, H, M, hm = ff.concat_objects(parts)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        lam, W, rs, infos, rc = ff.eigenmodes_batched(ctx, off, rp, col, H, M, hm, k=16, tol=tol, max_iter=max_iter,
                                                      use_graph=True, allow_unconverged=True)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        res.append((t1 - t0, t2 - t1, infos, rc))
        del parts, rp, col, H, M, hm, W
    build, solve, infos, rc = res[-1]
    its = [i["iters_fp32"] + i["iters_fp64"] for i in infos]
    return dict(objects=64, particles=int(sum(c.n for c in clouds)), k=16, graph=bool(infos[0]["graph"]),
                seconds=round(build + solve, 3), build_s=round(build, 3), solve_s=round(solve, 3),
                iters_mean=round(float(np.mean(its)), 1), iters_max=int(max(its)),
                converged=int(sum(i["converged"] for i in infos)), status=rc, generate_s=round(gen, 1))


def paper_training(ff, ctx, S, k, reps=3):
    """The paper's own construction and eigensolve on one object ("training time", Sec. 4): FPS
    centres, radii, neighbour lists, RKPM shape functions, H and M, then k modes (mixed path,
    refined to eigenvalue bound 1e-5) with a block of 64 (at K = 1000 the guard columns cut the
    iterations from 223 to 18: the solve is launch-bound at this size)."""
    import numpy as np
    import torch
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a), device="cuda")
    ins = (dev(S.xyz), dev(S.vol), dev(S.lam), dev(S.mu))
    times = []
    for rep in range(reps + 1):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        A = ff.paper_construction(ctx, *ins, S.K)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        lam, W, res, info = ff.eigenmodes(ctx, S.K, A.row_ptr, A.col, A.H, A.M, A.hm32, k=k, block=64, tol=1e-6,
                                          eig_tol=1e-5, allow_unconverged=True)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        if rep:
            times.append((t2 - t0, t1 - t0, t2 - t1))
    tt = np.array(times).mean(axis=0)
    return dict(integration_points=S.q, centres=S.K, k=k, seconds=round(float(tt[0]), 4),
                construction_s=round(float(tt[1]), 4), eigensolve_s=round(float(tt[2]), 4),
                nnz=int(A.col.numel()), block=64, iters=info["iters_fp32"] + info["iters_fp64"],
                converged=bool(info["converged"]), max_eig_bound=info["max_eig_bound"])


def matfree_timing(ff, ctx, A, vol, lam, mu, m, reps=10):
    """Matrix-free [H Y, M Y] (two passes over the neighbour lists, FP32) on the benchmark object,
    timed with HIP events on torch's stream (the context's)."""
    import torch
    n = A.n
    mf = ff.MatFree(ctx, n, A.nb.nbr_off, A.nb.nbr_id, A.phi, A.dphi, vol, lam, mu, perm=A.nb.perm, precision=1)
    Y = torch.randn((n, m), dtype=torch.float32, device="cuda")
    HY = torch.empty_like(Y)
    MY = torch.empty_like(Y)
    for _ in range(2):
        mf.apply(Y, out=(HY, MY))
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        mf.apply(Y, out=(HY, MY))
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    entries = int(A.nb.nbr_id.numel())
    q = n
    # per list entry: id + (phi, grad phi) FP32, once in each pass; per point: offset, two weights,
    # the 4m-value pass buffer written and read; per node: offset, Y read, HY and MY written
    alg = entries * 2 * (4 + 16) + q * (8 + 8 + 2 * 16 * m) + n * (8 + 4 * m + 8 * m)
    mf.close()
    return dict(launch_ms=round(ms, 4), bytes_per_launch=alg, achieved_gbps=round(alg / (ms * 1e-3) / 1e9, 1),
                list_entries=entries, m=m)


def _event_ms(fn, reps):
    import torch
    for _ in range(2):
        fn()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def sym_timing(ff, ctx, A, m, reps=10):
    """FP64 [H, M] Y from the upper triangles (sym_build / spmm_sym) against the FP64 path's own
    fused products on the benchmark object: the four-row tile copy (the FP64 solve's) and the CSR
    (the mixed path's certification); HIP events on torch's stream (the context's)."""
    import torch
    n = A.n
    nnz = int(A.col.numel())
    s = ff.SymCSR(ctx, n, A.row_ptr, A.col, A.H, A.M, precision=0)
    nu, nl = s.info()
    Y = torch.randn((n, m), dtype=torch.float64, device="cuda")
    HY, MY = torch.empty_like(Y), torch.empty_like(Y)
    ms_sym = _event_ms(lambda: s.spmm(Y, out=(HY, MY)), reps)
    s.close()
    names = ff.spmm_variant_names()
    csr = names.index("chunk64_waves4_batch4_occ8")
    ms_csr = _event_ms(lambda: ff.spmm_hm(ctx, A.row_ptr, A.col, A.H, A.M, A.hm32, Y, 0, variant=csr,
                                          out=(HY, MY)), reps)
    rt = ff.RowTiles(ctx, n, A.row_ptr, A.col, A.H, A.M, precision=0)
    ms_rt = _event_ms(lambda: rt.spmm(Y, 0, 0, out=(HY, MY)), reps)
    rt.close()
    # algorithmic bytes: per upper entry its column and two FP64 values, per lower entry its column
    # and position (its values are the upper entries' own), two row pointers per row, Y read once,
    # HY and MY written; the full CSR reads a column and two values per nonzero
    alg_sym = nu * (4 + 16) + nl * (4 + 4) + 16 * (n + 1) + 8 * n * m * 3
    alg_full = nnz * (4 + 16) + 8 * (n + 1) + 8 * n * m * 3
    return dict(m=m, upper_entries=nu, lower_entries=nl, sym_ms=round(ms_sym, 4), csr_ms=round(ms_csr, 4),
                rowtile4_ms=round(ms_rt, 4), sym_bytes=alg_sym, csr_bytes=alg_full,
                sym_gbps=round(alg_sym / (ms_sym * 1e-3) / 1e9, 1), csr_gbps=round(alg_full / (ms_csr * 1e-3) / 1e9, 1))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=1_000_000)
    ap.add_argument("--k", type=int, default=32)
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--max-iter", type=int, default=3000)
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--graph", action="store_true")
    ap.add_argument("--no-k64", action="store_true", help="skip the k = 64 solve of the large-object configuration")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the other configurations (100k sphere union, 64-object batch, paper construction)")
    ap.add_argument("--counters", action="store_true",
                    help="run a short solve (--steps iterations) and a 1 GiB calibration kernel (for counter passes)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(run with --gpus 1).", file=sys.stderr)
        sys.exit(2)
    if args.counters:
        counters_run(args)
        return

    import numpy as np
    import torch
    from paper_2605_29318_amd import freeform as ff
    from paper_2605_29318_amd import synth

    t = time.perf_counter()
    c = synth.ellipsoid_union(n=args.n, seed=3, hetero=True, k=args.k, mc_samples=4_000_000)
    log(f"[bench] generated {c.n} particles in {time.perf_counter() - t:.1f} s, h = {c.h:.5f}")
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a), device="cuda")
    dev_in = (dev(c.xyz), dev(c.vol), dev(c.lam), dev(c.mu))
    ctx = ff.Context(0)

    for w in range(args.warmup):
        r = run_step(ff, ctx, dev_in, c.n, c.h, args.k, 1, args.tol, args.max_iter, args.graph, seed=1000 + w)
        log(f"[bench] warmup {w}: {r['total']:.3f} s (build {r['build']:.3f}, solve {r['solve']:.3f}), "
            f"iters {r['info']['iters_fp32']}+{r['info']['iters_fp64']}")
    torch.cuda.synchronize()
    times = []
    last = None
    ctx.set_stage_timing(True)
    t_start = time.perf_counter()
    step_iters = []
    for s in range(args.steps):
        # step s starts LOBPCG from the seeded random block of seed s: the iteration count of a
        # solve depends on its start (the last pair's convergence), so the steps average over starts
        last = run_step(ff, ctx, dev_in, c.n, c.h, args.k, 1, args.tol, args.max_iter, args.graph, seed=s)
        times.append(last["total"])
        step_iters.append(last["info"]["iters_fp32"] + last["info"]["iters_fp64"])
        log(f"[bench] step {s}: {last['total']:.3f} s (build {last['build']:.3f}, solve {last['solve']:.3f}), "
            f"iters {last['info']['iters_fp32']}+{last['info']['iters_fp64']}, max resid {last['res'].max():.2e}")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    stages = ctx.stage_times()          # of the last timed solve
    ctx.set_stage_timing(False)
    ms_per_step = 1e3 * wall / args.steps
    A = last["A"]
    nnz = int(A.col.numel())

    ref = golden_eigs("ellipsoids1m", c) if args.n == 1_000_000 and args.k <= 32 else None
    fp64 = None
    if not args.no_fp64:
        # the plain FP64 path from the same starts as the timed mixed steps
        r64s = []
        for sd in range(args.steps):
            r64 = run_step(ff, ctx, dev_in, c.n, c.h, args.k, 0, args.tol, args.max_iter, args.graph, seed=sd)
            r64s.append(r64)
            log(f"[bench] fp64 seed {sd}: {r64['total']:.3f} s, iters {r64['info']['iters_fp64']}")
        t64 = [r["total"] for r in r64s]
        rel = np.abs(last["ev"][1:] - r64s[-1]["ev"][1:]) / np.abs(r64s[-1]["ev"][1:])
        fp64 = dict(seconds=round(float(np.mean(t64)), 3), seconds_per_seed=[round(x, 3) for x in t64],
                    iters_per_seed=[r["info"]["iters_fp64"] for r in r64s],
                    max_resid=float(max(r["res"].max() for r in r64s)),
                    converged=bool(all(r["info"]["converged"] for r in r64s)),
                    speedup_per_seed=[round(a / b, 3) for a, b in zip(t64, times)],
                    mixed_vs_fp64_eig_rel_diff_last_seed=float(rel.max()),
                    eig_err_vs_reference=eig_rel_err(r64s[-1]["ev"], ref))
        del r64s

    # time to the eigenvalue tolerance: both paths refined until every pair's a-posteriori bound is
    # <= 1e-5, then the eigenvalues' measured error against the oracle's reference
    eig_tol_runs = {}
    for prec, name in ((1, "mixed"), (0, "fp64")):
        if prec == 0 and args.no_fp64:
            continue
        rs = time_solves(ff, ctx, dev_in, c, args.k, prec, range(min(args.steps, 3)), args.tol, args.max_iter,
                         eig_tol=1e-5)
        eig_tol_runs[name] = dict(
            seconds=round(float(np.mean([r["total"] for r in rs])), 3),
            iters=[(r["info"]["iters_fp32"], r["info"]["iters_fp64"]) for r in rs],
            max_eig_bound=float(max(r["info"]["max_eig_bound"] for r in rs)),
            max_angle_bound=float(max(r["info"]["max_angle_bound"] for r in rs)),
            certified=bool(all(r["info"]["eig_certified"] for r in rs)),
            eig_err_vs_reference=[eig_rel_err(r["ev"], ref) for r in rs])
        log(f"[bench] {name} to eigenvalue bound 1e-5: {eig_tol_runs[name]}")
        del rs

    k64 = None
    if not args.no_k64 and args.k == 32:
        # the large-object configuration asks for 64 modes of the same object (mixed path, start seed 0)
        r = run_step(ff, ctx, dev_in, c.n, c.h, 64, 1, args.tol, args.max_iter, args.graph, seed=0)
        k64 = dict(seconds=round(r["total"], 3), build_s=round(r["build"], 4), solve_s=round(r["solve"], 4),
                   iters=r["info"]["iters_fp32"] + r["info"]["iters_fp64"], max_resid=float(r["res"].max()),
                   converged=bool(r["info"]["converged"]))
        log(f"[bench] k = 64 step: {r['total']:.3f} s, iters {r['info']['iters_fp32']}+{r['info']['iters_fp64']}")
        del r
    extra = {}
    if not args.no_extra and args.k == 32:
        mf = matfree_timing(ff, ctx, last["A"], dev_in[1], dev_in[2], dev_in[3], m=32)
        extra["matfree_hm"] = mf
        log(f"[bench] matrix-free [H, M] Y: {mf}")
        extra["sym_hm_fp64"] = sym_timing(ff, ctx, last["A"], m=32)
        log(f"[bench] upper-triangle FP64 [H, M] Y: {extra['sym_hm_fp64']}")
        cs = synth.workload("spheres100k")
        ds = (dev(cs.xyz), dev(cs.vol), dev(cs.lam), dev(cs.mu))
        ref2 = golden_eigs("spheres100k", cs)
        time_solves(ff, ctx, ds, cs, 32, 1, [100], args.tol, args.max_iter)              # warm-up
        mx = time_solves(ff, ctx, ds, cs, 32, 1, range(3), args.tol, args.max_iter)
        f64 = time_solves(ff, ctx, ds, cs, 32, 0, range(3), args.tol, args.max_iter)
        ce = time_solves(ff, ctx, ds, cs, 32, 1, range(3), args.tol, args.max_iter, eig_tol=1e-5)
        extra["spheres100k"] = dict(
            particles=cs.n, k=32, nnz=int(mx[-1]["A"].col.numel()),
            mixed_s=round(float(np.mean([r["total"] for r in mx])), 4),
            mixed_iters=[r["info"]["iters_fp32"] + r["info"]["iters_fp64"] for r in mx],
            fp64_s=round(float(np.mean([r["total"] for r in f64])), 4),
            fp64_iters=[r["info"]["iters_fp64"] for r in f64],
            mixed_eig_tol_s=round(float(np.mean([r["total"] for r in ce])), 4),
            eig_err_vs_reference=dict(mixed=eig_rel_err(mx[0]["ev"], ref2), fp64=eig_rel_err(f64[0]["ev"], ref2),
                                      mixed_eig_tol=eig_rel_err(ce[0]["ev"], ref2)))
        log(f"[bench] spheres100k: {extra['spheres100k']}")
        del mx, f64, ce, ds
        extra["paper_beam"] = paper_training(ff, ctx, synth.beam(spacing=0.05, K=1000), k=33)
        log(f"[bench] paper construction, beam: {extra['paper_beam']}")
        extra["paper_ellipsoid_blob"] = paper_training(ff, ctx, synth.ellipsoid_blob(spacing=0.02, K=1000), k=33)
        log(f"[bench] paper construction, ellipsoid blob: {extra['paper_ellipsoid_blob']}")
        try:
            extra["batched64"] = batched_config(ff, ctx, args.tol, args.max_iter)
            log(f"[bench] batched 64 objects: {extra['batched64']}")
        except Exception as e:          # the batch's generator uses worker processes
            extra["batched64"] = dict(error=str(e)[:300])
    copy_gbps = stream_copy_gbps()
    log(f"[bench] stream copy (1 GiB, device to device): {copy_gbps:.0f} GB/s")

    m = args.k if args.k % 8 == 0 else ((args.k + 7) // 8) * 8
    cheb_ms, cheb_n = stages["precond_product"]
    spmm_ms, spmm_n = stages["spmm"]
    cheb_avg = cheb_ms / max(cheb_n, 1)
    spmm_avg = spmm_ms / max(spmm_n, 1)
    cheb_alg = cheb_step_bytes(nnz, c.n, m, degree=PRECOND_DEGREE or 12)
    spmm_alg = spmm_hm_bytes(nnz, c.n, m)
    achieved = cheb_alg / (cheb_avg * 1e-3) / 1e9
    spmm_gbps = spmm_alg / (spmm_avg * 1e-3) / 1e9
    traffic = measured_traffic()
    log(f"[bench] stage times of the last solve (ms, launches): "
        + ", ".join(f"{k} {v[0]:.1f}/{v[1]}" for k, v in stages.items()))
    log(f"[bench] chebyshev step: {cheb_avg:.3f} ms/launch, {achieved:.0f} GB/s algorithmic; "
        f"fused [H,M] spmm: {spmm_avg:.3f} ms/launch, {spmm_gbps:.0f} GB/s")

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(args.k, args.tol, c.n)
        log(f"[bench] cpu baseline: {cpu}")

    info = last["info"]
    out = {
        "metric": METRIC,
        "value": round(ms_per_step / 1e3, 4),
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 2),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f16+f32+f64",
        "data": "synthetic",
        "config": {"workload": "ellipsoids1m_hetero", "particles": c.n, "k": args.k, "tol": args.tol,
                   "nnz": nnz, "nnz_per_row": round(nnz / c.n, 1), "h": round(c.h, 6),
                   "precond": "chebyshev-jacobi", "precond_degree": PRECOND_DEGREE or 12, "precond_ratio": 1000,
                   "precond_values": "fp16 H and iterate (matrix cores)",
                   "graph": bool(args.graph)},
        "build_s": round(last["build"], 4),
        "solve_s": round(last["solve"], 4),
        "iters": {"fp32": info["iters_fp32"], "fp64": info["iters_fp64"]},
        "iters_per_step": step_iters,
        "start_seeds": list(range(args.steps)),
        "max_resid": float(last["res"].max()),
        # a-posteriori estimates of the timed answer (relative eigenvalue error, sine of the largest
        # subspace angle), residual in the norm of diag(M)^-1, clusters as blocks
        "max_eig_bound": float(info["max_eig_bound"]),
        "max_angle_bound": float(info["max_angle_bound"]),
        "converged": bool(info["converged"]),
        "fp64": fp64,
        "speedup_vs_fp64": (round(fp64["seconds"] / (ms_per_step / 1e3), 3) if fp64 else None),
        "eig_err_vs_reference": eig_rel_err(last["ev"], ref),
        "eig_tol_1e-5": eig_tol_runs,
        "k64": k64,
        "stream_copy_gbps": round(copy_gbps, 1),
        "spmm_gbps": round(spmm_gbps, 1),
        "stages_ms": {k: round(v[0], 2) for k, v in stages.items()},
        "stage_launches": {k: int(v[1]) for k, v in stages.items()},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "kernel": "spmm_tq_sb_kernel<%d, true, %d, 2, true> (Chebyshev step on the matrix cores: "
                               "binary16 H in K-blocks of the eight-row tiles, read without their zeros (a mask per "
                               "K-block, the values rebuilt in LDS), times the binary16 iterate, FP32 accumulation "
                               "on v_mfma_f32_16x16x16_f16, loads pipelined a super-block of four K-blocks ahead, "
                               "fused with the step's vector update, m=%d)" % (m // 16, 4 if m == 32 else 2, m),
                     "bytes_per_launch": cheb_alg, "launch_ms": round(cheb_avg, 4),
                     "share_of_solve": round(cheb_ms / max(stages["total"][0], 1e-9), 3)},
        "spmm_hm": {"kernel": "spmm_hm8p_kernel<2, 2, 2, true, 4> (fused [H, M] Y on the eight-row tiles, "
                              "FP32 matrix cores, four four-entry steps chained before each FP64 addition)"
                              if args.k == 32 else "fused [H, M] Y (default variant)",
                    "achieved": round(spmm_gbps, 1), "peak": 8000.0, "unit": "GB/s",
                    "frac": round(spmm_gbps / 8000.0, 4), "bytes_per_launch": spmm_alg,
                    "launch_ms": round(spmm_avg, 4)},
        "cpu_baseline": cpu,
    }
    out.update(extra)
    print(json.dumps(out), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
