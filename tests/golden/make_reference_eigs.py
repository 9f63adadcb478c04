"""Reference eigenvalues of the named workloads, computed by the FP64 oracle alone.

    python tests/golden/make_reference_eigs.py spheres100k 32
    python tests/golden/make_reference_eigs.py ellipsoids1m 32 --tol 5e-8 --guard 16 --kc 36
    python tests/golden/make_reference_eigs.py ellipsoids1m 32 --tol 1.5e-8 --guard 16 --kc 32 --partial P
    python tests/golden/make_reference_eigs.py ellipsoids1m 32 --guard 16 --kc 32 --from-partial P

Builds the seeded workload (``synth.workload``), runs the oracle's whole
pipeline (binning, neighbours, RKPM shape functions of Sec. 3.2 Eq. (7)-(11),
the Hessian of Prop. 1 and the mass matrix of Eq. (14)), then the oracle's FP64
block LOBPCG for the generalized eigenproblem of Eq. (15) with its
Chebyshev-Jacobi preconditioner, from a seeded random start, with k + guard
columns (``--guard``, default 8) of which the first k + guard / 2 (or ``--kc``) must reach the
backward-error residual ``tol``. The result file ``ref_eigs_<workload>_k<k>.json`` next to this script
holds the input's SHA-256 (so a test can tell that it checks the same object),
the eigenvalues and residuals of every column, the iteration count and the
host threads used. Nothing here reads a GPU result.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("workload")
    ap.add_argument("k", type=int)
    ap.add_argument("--tol", type=float, default=1e-10)
    ap.add_argument("--guard", type=int, default=8)
    ap.add_argument("--seed", type=int, default=7)
    ap.add_argument("--maxiter", type=int, default=3000)
    ap.add_argument("--kc", type=int, default=None,
                    help="columns that must reach tol (default k + guard / 2)")
    ap.add_argument("--out", default=None)
    ap.add_argument("--partial", default=None,
                    help="rewrite this file with the Ritz values and residuals every 10 iterations")
    ap.add_argument("--from-partial", default=None,
                    help="write the reference from such a progress file of a run with the same arguments "
                         "(the solve stopped there: its Ritz values, its own residuals) instead of solving")
    a = ap.parse_args(argv)

    import numpy as np
    from oracle import oracle as O
    from paper_2605_29318_amd import synth

    t0 = time.time()
    cloud = synth.workload(a.workload)
    P = O.pipeline(cloud)
    t_build = time.time() - t0
    H, M = P.Hs(), P.Ms()
    m = a.k + a.guard
    kc = a.kc if a.kc is not None else a.k + a.guard // 2
    assert a.k <= kc <= m
    if a.from_partial:
        d = json.load(open(a.from_partial))
        lam, res = d["ritz_values"], d["residuals"]
        assert len(lam) == m and all(x <= y for x, y in zip(lam, lam[1:]))
        out = {
            "workload": a.workload, "sha256": cloud.sha256(), "n": int(cloud.n), "nnz": int(P.row_ptr[-1]),
            "h": float(cloud.h), "k": a.k, "block": m, "k_converged": kc,
            "tol": float(max(res[:kc])), "max_resid_first_kc": float(max(res[:kc])),
            "iterations": int(d["iteration"]), "stopped": "at the progress file's iteration, before tol",
            "start": f"synth.initial_block(n, {m}, seed={a.seed})",
            "precond": "oracle.chebyshev_jacobi defaults (degree 12, ratio 1000)",
            "eigenvalues": [float(x) for x in lam], "residuals": [float(x) for x in res],
            "residual_kind": "the solve's own (from its implicitly updated products)",
        }
        path = a.out or os.path.join(HERE, f"ref_eigs_{a.workload}_k{a.k}.json")
        with open(path, "w") as f:
            json.dump(out, f, indent=1)
        print(json.dumps({k: v for k, v in out.items() if k not in ("eigenvalues", "residuals")}))
        return 0
    X0 = synth.initial_block(cloud.n, m, seed=a.seed)
    t1 = time.time()
    def partial(it, th, res):
        if a.partial:
            with open(a.partial, "w") as f:
                json.dump({"iteration": it, "max_resid_first_kc": float(res[:kc].max()),
                           "ritz_values": [float(x) for x in th], "residuals": [float(x) for x in res]}, f)
    lam, W, it, res = O.lobpcg(H, M, X0, k=kc, tol=a.tol, maxiter=a.maxiter, precond="chebyshev", verbose=10,
                               callback=partial)
    t_solve = time.time() - t1
    res_all = O.residuals(H, M, lam, W)
    out = {
        "workload": a.workload,
        "sha256": cloud.sha256(),
        "n": int(cloud.n),
        "nnz": int(P.row_ptr[-1]),
        "h": float(cloud.h),
        "k": a.k,
        "block": m,
        "k_converged": kc,
        "tol": a.tol,
        "max_resid_first_kc": float(res_all[:kc].max()),
        "iterations": int(it),
        "start": f"synth.initial_block(n, {m}, seed={a.seed})",
        "precond": "oracle.chebyshev_jacobi defaults (degree 12, ratio 1000)",
        "eigenvalues": [float(x) for x in lam],
        "residuals": [float(x) for x in res_all],
        "build_seconds": round(t_build, 1),
        "solve_seconds": round(t_solve, 1),
        "host_threads": int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1)),
    }
    path = a.out or os.path.join(HERE, f"ref_eigs_{a.workload}_k{a.k}.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps({k: v for k, v in out.items() if k not in ("eigenvalues", "residuals")}))
    if res_all[:kc].max() > a.tol:
        print("NOT CONVERGED to tol in the first", kc, "columns", file=sys.stderr)
        return 1
    return 0


if __name__ == "__main__":
    sys.exit(main())
