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


def run_step(ff, ctx, dev_in, n, h, k, precision, tol, max_iter, use_graph=False, seed=0):
    import torch
    xyz, vol, lam, mu = dev_in
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    A = ff.assemble_cloud(ctx, xyz, vol, lam, mu, h)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ev, W, res, info = ff.eigenmodes(ctx, n, A.row_ptr, A.col, A.H, A.M, A.hm32, k=k, precision=precision,
                                     tol=tol, max_iter=max_iter, use_graph=use_graph, allow_unconverged=True,
                                     precond=PRECOND, precond_degree=PRECOND_DEGREE, seed=seed)
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


def cpu_baseline(n_sample, k, iters, gpu_iters, n_full):
    """The FP64 oracle on a bounded sample: its build stages on n_sample particles and
    `iters` LOBPCG iterations, scaled linearly in n to n_full and to the GPU's
    iteration count."""
    import numpy as np
    from oracle import oracle as O
    from paper_2605_29318_amd import synth
    c = synth.ellipsoid_union(n=n_sample, seed=3, hetero=True, k=k, mc_samples=1_000_000)
    t0 = time.perf_counter()
    P = O.pipeline(c)
    t1 = time.perf_counter()
    H, M = P.Hs(), P.Ms()
    X0 = synth.initial_block(c.n, k, seed=1)
    t2 = time.perf_counter()
    O.lobpcg(H, M, X0, k=k, tol=1e-30, maxiter=iters, precond="jacobi")
    t3 = time.perf_counter()
    build = t1 - t0
    per_iter = (t3 - t2) / iters
    scale = n_full / n_sample
    est = build * scale + per_iter * scale * gpu_iters
    return dict(value=round(est, 2), unit="s", cores=os.cpu_count(), kind="oracle",
                sample=(f"oracle binning+neighbours+RKPM+assembly on {n_sample} particles of the same recipe "
                        f"({build:.2f} s) and {iters} FP64 Jacobi-preconditioned LOBPCG iterations "
                        f"({per_iter*1e3:.1f} ms/iter), scaled linearly to {n_full} particles and the GPU's "
                        f"{gpu_iters} iterations (a lower bound: each GPU iteration also applies the "
                        f"Chebyshev polynomial, the oracle's applies diag(H)^-1)"),
                measured_s=round(t3 - t0, 2))


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

    fp64 = None
    if not args.no_fp64:
        r64 = run_step(ff, ctx, dev_in, c.n, c.h, args.k, 0, args.tol, args.max_iter, args.graph,
                       seed=args.steps - 1)
        rel = np.abs(last["ev"][1:] - r64["ev"][1:]) / np.abs(r64["ev"][1:])
        fp64 = dict(seconds=round(r64["total"], 3), iters=r64["info"]["iters_fp64"],
                    max_resid=float(r64["res"].max()), converged=bool(r64["info"]["converged"]),
                    mixed_vs_fp64_eig_rel_diff=float(rel.max()))
        log(f"[bench] fp64 step: {r64['total']:.3f} s, iters {r64['info']['iters_fp64']}")

    k64 = None
    if not args.no_k64 and args.k == 32:
        # the large-object configuration asks for 64 modes of the same object (mixed path, start seed 0)
        r = run_step(ff, ctx, dev_in, c.n, c.h, 64, 1, args.tol, args.max_iter, args.graph, seed=0)
        k64 = dict(seconds=round(r["total"], 3), build_s=round(r["build"], 4), solve_s=round(r["solve"], 4),
                   iters=r["info"]["iters_fp32"] + r["info"]["iters_fp64"], max_resid=float(r["res"].max()),
                   converged=bool(r["info"]["converged"]))
        log(f"[bench] k = 64 step: {r['total']:.3f} s, iters {r['info']['iters_fp32']}+{r['info']['iters_fp64']}")
        del r
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
        gpu_iters = int(round(sum(step_iters) / len(step_iters)))
        cpu = cpu_baseline(50_000, args.k, 10, gpu_iters, c.n)
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
        "dtype": "f32+f64",
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
        "converged": bool(info["converged"]),
        "fp64": fp64,
        "speedup_vs_fp64": (round(fp64["seconds"] / (ms_per_step / 1e3), 3) if fp64 else None),
        "k64": k64,
        "stream_copy_gbps": round(copy_gbps, 1),
        "spmm_gbps": round(spmm_gbps, 1),
        "stages_ms": {k: round(v[0], 2) for k, v in stages.items()},
        "stage_launches": {k: int(v[1]) for k, v in stages.items()},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "kernel": "spmm_tq_sb_kernel<%d, true> (Chebyshev step on the matrix cores: binary16 H in "
                               "K-blocks of the eight-row tiles times the binary16 iterate, FP32 accumulation on "
                               "v_mfma_f32_16x16x16_f16, loads pipelined a super-block of four K-blocks ahead, "
                               "fused with the step's vector update, m=%d)" % (m // 16, m),
                     "bytes_per_launch": cheb_alg, "launch_ms": round(cheb_avg, 4),
                     "share_of_solve": round(cheb_ms / max(stages["total"][0], 1e-9), 3)},
        "spmm_hm": {"achieved": round(spmm_gbps, 1), "unit": "GB/s", "bytes_per_launch": spmm_alg,
                    "launch_ms": round(spmm_avg, 4)},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
