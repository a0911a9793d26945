"""Benchmark: time to a 1e-10 relative residual (setup + solve) of lAIR on one
MI355X, mixed precision against plain FP64.

Default workload: one implicit Euler step of 3-D advection-diffusion, 7-point
upwind finite differences on a 128^3 grid (2,097,152 unknowns), velocity
(1, 0.7, 0.4)/|.|, eps = 1e-4, dt = h, 16 seeded N(0,1) right-hand sides,
distance-1 lAIR with classical direct interpolation, F-F-C Jacobi.

One step = lair_setup (CF splitting per level given) + lair_solve of all 16
right-hand sides from x = 0 to ||b - A x|| <= 1e-10 ||b|| each.  Inputs are
resident in HBM before the timed region.  The CF splitting (the classical
first pass, a sequential host algorithm) is computed once by the library
before timing and reported separately.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--workload c5|c1|c4]
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_workload(name):
    import workloads as W
    if name == "c5":
        w = W.workload_c5()
        return w, dict(interp="direct", distance=1), \
            {"workload": "implicit_euler_adr3d_128^3_16rhs", "n": w["n"], "nnz": w["nnz"],
             "nrhs": 16, "grid": "128^3", "eps": 1e-4, "dt": "h", "distance": 1,
             "interp": "direct", "relaxation": "FFC-Jacobi", "rtol": 1e-10}
    if name == "c1":
        w = W.workload_c1()
        return w, dict(interp="one_point", distance=1), \
            {"workload": "steady_upwind_transport_64x64", "n": w["n"], "nnz": w["nnz"],
             "nrhs": 1, "distance": 1, "interp": "one_point", "rtol": 1e-10}
    if name == "c4":
        import scipy.sparse as sp
        w = W.workload_c4()
        from_csr = sp.csr_matrix((w["val"], w["col"], w["rowptr"]), shape=(w["n"],) * 2)
        A = (from_csr + sp.diags(w["c"])).tocsr()
        A.sort_indices()
        w = dict(w, rowptr=A.indptr.astype(np.int32), col=A.indices.astype(np.int32),
                 val=A.data, nnz=A.nnz)
        return w, dict(interp="direct", distance=1), \
            {"workload": "adr_reaction_64x64", "n": w["n"], "nnz": w["nnz"], "nrhs": 1,
             "distance": 1, "interp": "direct", "rtol": 1e-10}
    raise SystemExit("unknown workload %s" % name)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="c5")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the lAIR hot path here is a "
              "single-GPU build (see the sharding notes in the design document); "
              "--gpus %d is not supported" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1708_06065_amd as lair
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    lair.load_library()

    t0 = time.time()
    w, kw, cfg = make_workload(args.workload)
    log("workload %s generated in %.1fs (n=%d nnz=%d)" % (cfg["workload"], time.time() - t0,
                                                          w["n"], w["nnz"]))
    rp = torch.as_tensor(w["rowptr"], device=dev)
    cj = torch.as_tensor(w["col"], device=dev)
    vv = torch.as_tensor(w["val"], device=dev)
    rhs = np.asarray(w["rhs"], dtype=np.float64)
    B = torch.as_tensor(np.ascontiguousarray(rhs), device=dev)
    nrhs = 1 if B.dim() == 1 else B.shape[1]
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()

    # CF splitting per level by the library's own first pass (untimed)
    t0 = time.perf_counter()
    h0 = lair.setup(rp, cj, vv, **kw)
    torch.cuda.synchronize()
    t_full_setup = (time.perf_counter() - t0) * 1e3
    cfl = [h0.export(l, "cf") for l in range(h0.nlevels - 1)]
    nlev = h0.nlevels
    h0.free()
    log("library CF split + setup: %.1f ms, %d levels" % (t_full_setup, nlev))

    def step(precision):
        h = lair.setup(rp, cj, vv, cf_levels=cfl, precision=precision, **kw)
        X, info = h.solve(B, rtol=1e-10, maxit=100)
        return h, X, info

    results = {}
    for prec in (["mixed"] if args.no_fp64 else ["mixed", "fp64"]):
        for _ in range(args.warmup):
            h, X, info = step(prec)
            h.free()
        torch.cuda.synchronize()
        times, infos = [], []
        for k in range(args.steps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            h, X, info = step(prec)
            torch.cuda.synchronize()
            times.append((time.perf_counter() - t0) * 1e3)
            infos.append(info)
            if k < args.steps - 1:
                h.free()
        # verify the last step's solution independently in FP64 on the GPU
        A = torch.sparse_csr_tensor(rp.long(), cj.long(), vv, size=(w["n"], w["n"]))
        R = B - (A @ X if X.dim() > 1 else (A @ X.unsqueeze(1)).squeeze(1))
        rel = (torch.linalg.vector_norm(R, dim=0) / torch.linalg.vector_norm(B, dim=0)).max().item()
        h.free()
        results[prec] = dict(ms=float(np.median(times)), ms_all=times, iters=infos[-1]["iters"],
                             relres=infos[-1]["relres"], relres_check=rel,
                             setup_ms=infos[-1]["setup_ms"], solve_ms=infos[-1]["solve_ms"],
                             rho=infos[-1]["rho"], cc=infos[-1]["cycle_complexity"],
                             oc=infos[-1]["op_complexity"])
        log(prec, json.dumps(results[prec]))

    main_prec = "mixed"
    r = results[main_prec]
    out = {
        "metric": "time to 1e-10 rel. residual (setup+solve), mixed vs FP64",
        "value": r["ms"],
        "unit": "ms",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms"],
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 cycle/local LU + f64 outer",
        "data": "synthetic",
        "config": cfg,
        "iters": r["iters"],
        "relres": r["relres"],
        "relres_check_fp64": r["relres_check"],
        "setup_ms": r["setup_ms"],
        "solve_ms": r["solve_ms"],
        "cf_split_plus_setup_ms_untimed": t_full_setup,
        "levels": nlev,
    }
    if "fp64" in results:
        out["fp64"] = {k: results["fp64"][k] for k in ("ms", "iters", "relres", "setup_ms",
                                                        "solve_ms")}
        out["speedup_mixed_vs_fp64"] = results["fp64"]["ms"] / r["ms"]
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
