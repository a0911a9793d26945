"""Benchmark: time to a 1e-10 relative residual (setup + solve) of lAIR on one
MI355X, mixed precision against plain FP64.

Default workload: one implicit Euler step of 3-D advection-diffusion, 7-point
upwind finite differences on a 128^3 grid (2,097,152 unknowns), velocity
(1, 0.7, 0.4)/|.|, eps = 1e-4, dt = h, 16 seeded N(0,1) right-hand sides,
distance-1 lAIR with classical direct interpolation, F-F-C Jacobi.

One step = lair_setup (CF splitting per level given) + lair_solve of all 16
right-hand sides from x = 0 until ||b - A x|| <= 1e-10 ||b|| for each.  The
matrix and right-hand sides are resident in HBM before the timed region.  The
CF splitting (the classical first pass, a sequential host algorithm) is
computed once by the library before timing and reported separately.

During the timed steps the library's profiler brackets every launch of the
dominant kernel category with HIP events on its stream; the roofline entry is
that category's algorithmic bytes divided by its measured time.

Workload c3: a batch of 512 independent 2-D advection-diffusion-reaction
systems of uneven size (N x N grids, N log-uniform in [32, 320], 10.8 M
unknowns in all), set up and solved as one block-diagonal union with
per-system convergence; one step = lair_setup_batch (union CF splittings
given) + lair_solve_batch to 1e-10 for every system.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--workload c5|c3|c4|c1]
"""
import argparse
import json
import os
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E peak, GB/s


def measured_traffic(workload, category, lump_tol):
    """HBM bytes per launch of a kernel category from the committed
    rocprofv3 FETCH_SIZE / WRITE_SIZE record, or None when there is none for
    this workload, category and lumping tolerance or the kernel sources
    changed since."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "%s_%s_traffic.json" % (workload, category))
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("lump_tol", 0.0) != lump_tol:
        return None
    for f, sha in rec.get("source_sha256", {}).items():
        fp = os.path.join(ROOT, f)
        if not os.path.exists(fp) or hashlib.sha256(open(fp, "rb").read()).hexdigest() != sha:
            return None
    return rec["fetch"]["bytes_per_launch"] + rec["write"]["bytes_per_launch"]


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
    if name == "c3":
        w = W.workload_c3()
        return w, dict(interp="direct", distance=1), \
            {"workload": "adr2d_batch_512_systems", "n": w["n"], "nnz": w["nnz"],
             "nsys": 512, "grid": "N x N, N log-uniform in [32, 320]", "nrhs": 1,
             "distance": 1, "interp": "direct", "relaxation": "FFC-Jacobi", "rtol": 1e-10}
    if name == "c1":
        w = W.workload_c1()
        return w, dict(interp="one_point", distance=1), \
            {"workload": "steady_upwind_transport_64x64", "n": w["n"], "nnz": w["nnz"],
             "nrhs": 1, "distance": 1, "interp": "one_point", "rtol": 1e-10}
    if name == "c4":
        import scipy.sparse as sp
        w = W.workload_c4()
        A = (sp.csr_matrix((w["val"], w["col"], w["rowptr"]), shape=(w["n"],) * 2)
             + sp.diags(w["c"])).tocsr()
        A.sort_indices()
        w = dict(w, rowptr=A.indptr.astype(np.int32), col=A.indices.astype(np.int32),
                 val=A.data, nnz=A.nnz)
        return w, dict(interp="direct", distance=1), \
            {"workload": "adr_reaction_64x64", "n": w["n"], "nnz": w["nnz"], "nrhs": 1,
             "distance": 1, "interp": "direct", "rtol": 1e-10}
    if name == "dg":
        w = W.workload_dg_curved(256)
        return w, dict(interp="one_point", distance=2, block_size=6, nodal=True), \
            {"workload": w["name"], "n": w["n"], "nnz": w["nnz"], "nrhs": 1, "block": 6,
             "treatment": "nodal", "interp": "one_point by block", "distance": 2,
             "relaxation": "FFC block Jacobi", "rtol": 1e-10}
    raise SystemExit("unknown workload %s" % name)


def cpu_baseline_batch(kw, budget_s=15.0):
    """Oracle on a bounded sample of the batch: setup + solve of the systems
    in order until budget_s seconds have been spent, scaled to the whole
    batch by stored entries.  Child process, one OpenMP thread."""
    code = r'''
import json, sys, time
sys.path.insert(0, %r)
import workloads as W
from oracle import lair as O
systems = W.adr_batch(512, seed=3)
tot = sum(w["nnz"] for w in systems)
t0 = time.perf_counter(); done = 0; nz = 0; its = []
for w in systems:
    A = O.csr(w["rowptr"], w["col"], w["val"])
    H = O.setup(A, interp=O.INTERP_DIRECT, lump_tol=%r)
    x, it, _ = O.solve(H, w["rhs"], rtol=1e-10, maxit=100)
    done += 1; nz += w["nnz"]; its.append(it)
    if time.perf_counter() - t0 > %r:
        break
el = time.perf_counter() - t0
print(json.dumps({"s": el, "done": done, "nnz": nz, "tot": tot, "iters_max": max(its)}))
''' % (ROOT, kw.get("lump_tol", 0.0), budget_s)
    env = dict(os.environ, OMP_NUM_THREADS="1")
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env,
                       timeout=600)
    if r.returncode != 0:
        log("cpu baseline failed:", r.stderr[-2000:])
        return None
    d = json.loads(r.stdout.strip().splitlines()[-1])
    scale = d["tot"] / d["nnz"]
    return {"value": 1e3 * d["s"] * scale, "unit": "ms", "cores": 1, "kind": "oracle",
            "sample": "oracle setup + solve to 1e-10 of the first %d of 512 systems "
                      "(%.1f s, %.1f%% of the stored entries), scaled x%.1f by stored entries"
                      % (d["done"], d["s"], 100.0 / scale, scale)}


def cpu_baseline_nodal(kw, n_full, m_sample=96):
    """The oracle's nodal setup + solve to 1e-10 on the same DG problem at
    m_sample x m_sample x 2 triangles (its Python loops over nodes would
    take minutes at full size), scaled to the full problem by rows.  Child
    process, one OpenMP thread."""
    code = r'''
import json, sys, time
sys.path.insert(0, %r)
import workloads as W
from oracle import lair as O
w = W.workload_dg_curved(%d)
A = O.csr(w["rowptr"], w["col"], w["val"])
t0 = time.perf_counter()
H = O.setup(A, block=6, distance=%d)
t1 = time.perf_counter()
x, it, _ = O.solve(H, w["rhs"], rtol=1e-10, maxit=300)
t2 = time.perf_counter()
print(json.dumps({"setup_s": t1 - t0, "solve_s": t2 - t1, "iters": it, "n": w["n"]}))
''' % (ROOT, m_sample, kw["distance"])
    env = dict(os.environ, OMP_NUM_THREADS="1")
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env,
                       timeout=600)
    if r.returncode != 0:
        log("cpu baseline failed:", r.stderr[-2000:])
        return None
    d = json.loads(r.stdout.strip().splitlines()[-1])
    scale = n_full / d["n"]
    return {"value": 1e3 * (d["setup_s"] + d["solve_s"]) * scale, "unit": "ms", "cores": 1,
            "kind": "oracle",
            "sample": "oracle nodal setup (%.1f s) + solve to 1e-10 (%.1f s, %d cycles) of the "
                      "same problem on %dx%dx2 triangles (%d rows), scaled x%.0f by rows"
                      % (d["setup_s"], d["solve_s"], d["iters"], m_sample, m_sample, d["n"],
                         scale)}


def cpu_baseline(workload, kw):
    """Time the CPU oracle on a bounded sample: the full setup of the
    workload plus the solve of its first right-hand side; the solve time is
    scaled by the number of right-hand sides.  Runs in a child process with
    one OpenMP thread."""
    code = r'''
import json, sys, time
sys.path.insert(0, %r)
import numpy as np
import bench
from oracle import lair as O
w, kw, cfg = bench.make_workload(%r)
A = O.csr(w["rowptr"], w["col"], w["val"])
interp = O.INTERP_DIRECT if kw["interp"] == "direct" else O.INTERP_ONE_POINT
t0 = time.perf_counter()
H = O.setup(A, interp=interp, distance=kw["distance"], lump_tol=%r)
t1 = time.perf_counter()
b = np.asarray(w["rhs"])
b0 = b[:, 0] if b.ndim > 1 else b
x, it, hist = O.solve(H, b0, rtol=1e-10, maxit=100)
t2 = time.perf_counter()
print(json.dumps({"setup_s": t1 - t0, "solve_s": t2 - t1, "iters": it,
                  "nrhs": 1 if b.ndim == 1 else b.shape[1]}))
''' % (ROOT, workload, kw.get("lump_tol", 0.0))
    env = dict(os.environ, OMP_NUM_THREADS="1")
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env,
                       timeout=600)
    if r.returncode != 0:
        log("cpu baseline failed:", r.stderr[-2000:])
        return None
    d = json.loads(r.stdout.strip().splitlines()[-1])
    total_ms = 1e3 * (d["setup_s"] + d["nrhs"] * d["solve_s"])
    return {"value": total_ms, "unit": "ms", "cores": 1, "kind": "oracle",
            "sample": "full-size oracle setup (%.1f s, CF split included) + solve of "
                      "right-hand side 0 of %d to 1e-10 (%.1f s, %d cycles), solve time "
                      "scaled x%d" % (d["setup_s"], d["nrhs"], d["solve_s"], d["iters"],
                                      d["nrhs"])}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="c5")
    ap.add_argument("--split", choices=("rs", "pmis"), default="rs",
                    help="rs: the paper's first pass on the host, computed once untimed and "
                         "passed in; pmis: the parallel splitting on the device, inside the "
                         "timed setup")
    ap.add_argument("--distance", type=int, choices=(1, 2), default=None,
                    help="neighbourhood distance instead of the workload's own")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-graphs", action="store_true",
                    help="launch the solve's kernels eagerly instead of replaying captured iterations")
    ap.add_argument("--solver", choices=("stationary", "fgmres"), default="stationary",
                    help="outer iteration: the stationary V-cycle iteration (the default "
                         "hot path) or flexible GMRES with the V-cycle as preconditioner")
    ap.add_argument("--restart", type=int, default=20, help="FGMRES restart length")
    ap.add_argument("--lump", type=float, default=1e-3,
                    help="lump every coarse operator at this tolerance (0: off); the paper "
                         "lumps all its lAIR results at 0.001")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="run one device copy of this size first (for HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this lAIR build is single-GPU (the "
              "design notes describe how it would shard); --gpus %d is not "
              "supported" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1708_06065_amd as lair
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    lair.load_library()

    if args.copy_calibration_mib:
        nb = args.copy_calibration_mib << 20
        a = torch.ones(nb // 4, dtype=torch.float32, device=dev)
        c = torch.empty_like(a)
        c.copy_(a)
        torch.cuda.synchronize()
        log("copy calibration: %d bytes read, %d bytes written" % (nb, nb))
        del a, c

    t0 = time.time()
    w, kw, cfg = make_workload(args.workload)
    if args.solver == "fgmres":
        if "systems" in w:
            print("--solver fgmres is for a single system", file=sys.stderr)
            sys.exit(2)
        cfg = dict(cfg, outer="FGMRES(%d), V-cycle as right preconditioner" % args.restart)
        args.no_cpu_baseline = True
    log("workload %s generated in %.1fs (n=%d nnz=%d)" % (cfg["workload"], time.time() - t0,
                                                          w["n"], w["nnz"]))
    batch = "systems" in w
    rp = torch.as_tensor(w["rowptr"], device=dev)
    cj = torch.as_tensor(w["col"], device=dev)
    vv = torch.as_tensor(w["val"], device=dev)
    B = torch.as_tensor(np.ascontiguousarray(np.asarray(w["rhs"], dtype=np.float64)),
                        device=dev)
    if batch:
        members = [(torch.as_tensor(q["rowptr"], device=dev),
                    torch.as_tensor(q["col"], device=dev),
                    torch.as_tensor(q["val"], device=dev)) for q in w["systems"]]
    torch.cuda.synchronize()

    if args.no_graphs:
        kw = dict(kw, graphs=False)
    if args.split == "pmis":
        kw = dict(kw, split="pmis")
        cfg = dict(cfg, splitting="PMIS on the device, timed")
        args.no_cpu_baseline = True
    if args.distance is not None:
        kw = dict(kw, distance=args.distance)
        cfg = dict(cfg, distance=args.distance)
        args.no_cpu_baseline = True
    if kw.get("nodal"):
        # lumping would break the dense blocks a nodal hierarchy keeps
        args.lump = 0.0
    kw = dict(kw, lump_tol=args.lump)
    cfg = dict(cfg, lumping=args.lump)

    def build(cf_levels=None, precision="fp64"):
        if batch:
            return lair.setup_batch(members, cf_levels=cf_levels, precision=precision, **kw)
        return lair.setup(rp, cj, vv, cf_levels=cf_levels, precision=precision, **kw)

    # CF splitting per level by the library's own first pass (untimed)
    t0 = time.perf_counter()
    h0 = build()
    torch.cuda.synchronize()
    t_full_setup = (time.perf_counter() - t0) * 1e3
    cfl = [h0.export(l, "cf") for l in range(h0.nlevels - 1)]
    nlev = h0.nlevels
    h0.free()
    log("library CF split + setup: %.1f ms, %d levels" % (t_full_setup, nlev))

    # the nodal DG workload needs 54 cycles at 256 x 256 x 2 (101 at distance 1)
    maxit = 300 if kw.get("nodal") else 100

    def step(precision):
        h = build(None if args.split == "pmis" else cfl, precision)
        if batch:
            X, info = h.solve_batch(B, rtol=1e-10, maxit=maxit)
        elif args.solver == "fgmres":
            X, info = h.solve_fgmres(B, rtol=1e-10, maxit=maxit, restart=args.restart)
        else:
            X, info = h.solve(B, rtol=1e-10, maxit=maxit)
        return h, X, info

    # which kernel category dominates a step: one profiled, untimed step
    # after a warm-up step (so that first-use allocations are not in it)
    h, X, info = step("mixed")
    h.free()
    lair.profile_begin(None)
    h, X, info = step("mixed")
    torch.cuda.synchronize()
    prof_all = lair.profile_end()
    h.free()
    dominant = max(prof_all.items(), key=lambda kv: kv[1]["ms"])[0]
    log("profiled step, per category:", json.dumps(prof_all))
    log("per-category GPU time of one mixed step (ms):",
        json.dumps({k: round(v["ms"], 3) for k, v in sorted(prof_all.items(),
                                                              key=lambda kv: -kv[1]["ms"])}))

    results, prof_timed = {}, None
    for prec in (["mixed"] if args.no_fp64 else ["mixed", "fp64"]):
        for _ in range(args.warmup):
            h, X, info = step(prec)
            h.free()
        torch.cuda.synchronize()
        times, infos = [], []
        if prec == "mixed":
            lair.profile_begin([dominant])
        for k in range(args.steps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            h, X, info = step(prec)
            torch.cuda.synchronize()
            times.append((time.perf_counter() - t0) * 1e3)
            infos.append(info)
            if k < args.steps - 1:
                h.free()
        if prec == "mixed":
            prof_timed = lair.profile_end()
        # independent FP64 check of the last step's solution
        try:
            A = torch.sparse_csr_tensor(rp.long(), cj.long(), vv, size=(w["n"], w["n"]))
            Xm = X if X.dim() > 1 else X.unsqueeze(1)
            Bm = B if B.dim() > 1 else B.unsqueeze(1)
            R = Bm - A @ Xm
            rel = (torch.linalg.vector_norm(R, dim=0) /
                   torch.linalg.vector_norm(Bm, dim=0)).max().item()
        except Exception as e:  # the check is optional
            log("residual check skipped:", e)
            rel = None
        h.free()
        if batch:
            its = np.asarray(infos[-1]["sys_iters"], dtype=np.float64)
            nz = np.array([q["nnz"] for q in w["systems"]], dtype=np.float64)
            log("%s: cycles per system min %d median %d max %d; useful share of the union's "
                "cycle work %.3f" % (prec, its.min(), np.median(its), its.max(),
                                     (nz * its).sum() / (nz.sum() * its.max())))
        results[prec] = dict(ms=float(np.median(times)), ms_all=times, iters=infos[-1]["iters"],
                             relres=infos[-1]["relres"], relres_check=rel,
                             setup_ms=infos[-1]["setup_ms"], solve_ms=infos[-1]["solve_ms"],
                             rho=infos[-1]["rho"], cc=infos[-1]["cycle_complexity"],
                             oc=infos[-1]["op_complexity"])
        log(prec, json.dumps(results[prec]))

    r = results["mixed"]
    d = prof_timed.get(dominant, {"launches": 0, "ms": 1.0, "alg_bytes": 0.0})
    achieved = d["alg_bytes"] / (d["ms"] * 1e-3) / 1e9 if d["ms"] > 0 else 0.0
    roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS,
                "traffic": measured_traffic(args.workload, dominant, args.lump), "kernel": dominant,
                "launches": d["launches"], "avg_launch_us": 1e3 * d["ms"] / max(d["launches"], 1),
                "alg_bytes_per_launch": d["alg_bytes"] / max(d["launches"], 1)}
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
        "roofline": roofline,
        "gpu_ms_by_category": {k: round(v["ms"], 3) for k, v in prof_all.items()},
    }
    if "fp64" in results:
        out["fp64"] = {k: results["fp64"][k] for k in ("ms", "iters", "relres", "setup_ms",
                                                        "solve_ms")}
        out["speedup_mixed_vs_fp64"] = results["fp64"]["ms"] / r["ms"]
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a bounded sample ...")
        if batch:
            cb = cpu_baseline_batch(kw)
        elif kw.get("nodal"):
            cb = cpu_baseline_nodal(kw, w["n"])
        else:
            cb = cpu_baseline(args.workload, kw)
        if cb:
            out["cpu_baseline"] = cb
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
