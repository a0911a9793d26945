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

The timed steps run as a caller would run them (iterations replayed from HIP
graphs, no profiler).  As many steps again follow with the library's
profiler bracketing every launch of the dominant kernel category with HIP
events on its stream (those cycles run eagerly); the roofline entry is that
category's algorithmic bytes divided by its measured kernel time.

Workload c3: a batch of 512 independent 2-D advection-diffusion-reaction
systems of uneven size (N x N grids, N log-uniform in [32, 320], 10.8 M
unknowns in all), set up and solved as one block-diagonal union with
per-system convergence; one step = lair_setup_batch (union CF splittings
given) + lair_solve_batch to 1e-10 for every system.

Workload c2: P2 upwind DG on 256 x 256 x 2 triangles (786,432 unknowns),
recirculating pure advection, block-scaled, distance-2 neighbourhoods.  The
stationary iteration does not reach 1e-10 on this problem (closed
streamlines: the paper calls the steady limit ill-posed), so one step is the
setup plus a fixed number of cycles, and the line says so.

Workload dg: nodal (block) lAIR at distance 2 on P2 upwind DG along the
curved field b = (y^2, cos^2(pi x/2)), 256 x 256 x 2 triangles, dense 6 x 6
blocks.  Workload dgu: the same with the DGu problem's total cross section
(1e4 in the central square, 1e-4 outside) and interior-penalty diffusion
kappa = 1e-3.  Both solve to 1e-10.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--workload c5|c3|c2|c4|c1|dg|dgu]

Summaries of rocprofv3 runs (written under profiles/):

    python bench.py --summarize-trace DIR --out FILE.md --title T --command CMD
    python bench.py --summarize-counters FETCH_DIR WRITE_DIR --workload W
          --category C --kernel-regex RE --out FILE.json --command CMD ...
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
FP64_VALU_PEAK_TFS = 78.6      # MI355X FP64 vector peak, TFLOP/s
C2_CYCLES = 20                 # fixed cycles per step on the non-converging DG problem
DGU_KAPPA = 1e-3               # diffusion of the DGu workload (one of the paper's values)


CSRC = os.path.join("paper_1708_06065_amd", "csrc")


def source_hashes():
    """SHA-256 of every source of the library (kernels and host code): a
    counter record describes the sources it was taken on."""
    import hashlib
    out = {}
    d = os.path.join(ROOT, CSRC)
    for f in sorted(os.listdir(d)):
        if f.endswith((".hip", ".cpp", ".hpp")):
            out[os.path.join(CSRC, f)] = hashlib.sha256(
                open(os.path.join(d, f), "rb").read()).hexdigest()
    return out


def measured_traffic(workload, category, cfg_key, alg_per_launch):
    """HBM bytes per launch of a kernel category from the committed
    rocprofv3 FETCH_SIZE / WRITE_SIZE record, or None when there is none for
    this workload, category and configuration, when any library source
    changed since the counters were taken, or when the record's algorithmic
    bytes per launch differ from this run's (another hierarchy)."""
    path = os.path.join(ROOT, "profiles", "%s_%s_traffic.json" % (workload, category))
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("config") != cfg_key:
        return None
    if rec.get("source_sha256") != source_hashes():
        return None
    a = rec.get("algorithmic_bytes_per_launch", 0.0)
    if not alg_per_launch or abs(a - alg_per_launch) > 0.005 * alg_per_launch:
        return None
    return rec["fetch"]["bytes_per_launch"] + rec["write"]["bytes_per_launch"]


def host_cpu():
    """(threads available to this process, CPU model name)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return n, model


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
    if name == "c2":
        w = W.workload_c2(256)
        return w, dict(interp="one_point", distance=2, block_size=6), \
            {"workload": "dg_p2_recirculating_256x256x2", "n": w["n"], "nnz": w["nnz"],
             "nrhs": 1, "block_scaling": 6, "distance": 2, "interp": "one_point",
             "relaxation": "FFC-Jacobi", "cycles": C2_CYCLES}
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
    if name == "dgu":
        w = W.workload_dgu(256, DGU_KAPPA)
        return w, dict(interp="one_point", distance=2, block_size=6, nodal=True), \
            {"workload": w["name"], "n": w["n"], "nnz": w["nnz"], "nrhs": 1, "block": 6,
             "kappa": DGU_KAPPA, "gamma": "1e4 in (0.25,0.75)^2, 1e-4 elsewhere",
             "beta": "(y^2, cos^2(pi x/2))", "diffusion": "symmetric interior penalty",
             "treatment": "nodal", "interp": "one_point by block", "distance": 2,
             "relaxation": "FFC block Jacobi", "rtol": 1e-10}
    raise SystemExit("unknown workload %s" % name)


def _oracle_child(code, threads, timeout=900):
    """Run oracle code in a child process with `threads` OpenMP threads
    (the oracle's C loops over C-points); returns its last JSON line."""
    env = dict(os.environ, OMP_NUM_THREADS=str(threads))
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env,
                       timeout=timeout)
    if r.returncode != 0:
        log("cpu baseline failed:", r.stderr[-2000:])
        return None
    return json.loads(r.stdout.strip().splitlines()[-1])


def _both_thread_counts(make_code, to_ms, describe):
    """The oracle timed on one host core and on every core this process
    may use; the all-core figure is the baseline value."""
    ncpu, model = host_cpu()
    one = _oracle_child(make_code(True), 1)
    allc = _oracle_child(make_code(False), ncpu) if ncpu > 1 else one
    if not one or not allc:
        return None
    return {"value": to_ms(allc), "unit": "ms", "cores": ncpu, "kind": "oracle",
            "single_core_ms": to_ms(one), "cpu_model": model,
            "sample": describe(allc) + "; the same on one core: %.1f ms" % to_ms(one)}


def cpu_baseline_batch(kw, budget_s=15.0, x_path=None):
    """Oracle on a bounded sample of the batch: setup + solve of the systems
    in order until budget_s seconds have been spent, scaled to the whole
    batch by stored entries.  The one-core run also writes the oracle's
    solutions of the systems it solved, one after another, to x_path."""
    def code(first):
        return r"""
import json, sys, time
sys.path.insert(0, %r)
import numpy as np
import workloads as W
from oracle import lair as O
systems = W.adr_batch(512, seed=3)
tot = sum(w["nnz"] for w in systems)
t0 = time.perf_counter(); done = 0; nz = 0; its = []; xs = []
for w in systems:
    A = O.csr(w["rowptr"], w["col"], w["val"])
    H = O.setup(A, interp=O.INTERP_DIRECT, lump_tol=%r)
    x, it, _ = O.solve(H, w["rhs"], rtol=1e-10, maxit=100)
    done += 1; nz += w["nnz"]; its.append(it); xs.append(x)
    if time.perf_counter() - t0 > %r:
        break
el = time.perf_counter() - t0
xp = %r
if xp:
    np.save(xp, np.concatenate(xs))
print(json.dumps({"s": el, "done": done, "nnz": nz, "tot": tot, "iters_max": max(its)}))
""" % (ROOT, kw.get("lump_tol", 0.0), budget_s, x_path if first else None)

    def to_ms(d):
        return 1e3 * d["s"] * d["tot"] / d["nnz"]

    def describe(d):
        scale = d["tot"] / d["nnz"]
        return ("oracle setup + solve to 1e-10 of the first %d of 512 systems (%.1f s, %.1f%% "
                "of the stored entries), scaled x%.1f by stored entries"
                % (d["done"], d["s"], 100.0 / scale, scale))
    return _both_thread_counts(code, to_ms, describe)


DG_ORACLE_SAMPLE = 96     # mesh of the nodal workloads' oracle sample


def cpu_baseline_nodal(kw, n_full, gen, m_sample=DG_ORACLE_SAMPLE, x_path=None):
    """The oracle's nodal setup + solve to 1e-10 on the same DG problem at
    m_sample x m_sample x 2 triangles (its Python loops over nodes would
    take minutes at full size), scaled to the full problem by rows.  gen:
    the workload call with %d for the mesh size.  The one-core run also
    writes the oracle's solution to x_path."""
    def code(first):
        return (r"""
import json, sys, time
sys.path.insert(0, %r)
import numpy as np
import workloads as W
from oracle import lair as O
w = W.""" + gen + r"""
A = O.csr(w["rowptr"], w["col"], w["val"])
t0 = time.perf_counter()
H = O.setup(A, block=6, distance=%d)
t1 = time.perf_counter()
x, it, _ = O.solve(H, w["rhs"], rtol=1e-10, maxit=300)
t2 = time.perf_counter()
xp = %r
if xp:
    np.save(xp, x)
print(json.dumps({"setup_s": t1 - t0, "solve_s": t2 - t1, "iters": it, "n": w["n"]}))
""") % (ROOT, m_sample, kw["distance"], x_path if first else None)

    def to_ms(d):
        return 1e3 * (d["setup_s"] + d["solve_s"]) * n_full / d["n"]

    def describe(d):
        return ("oracle nodal setup (%.1f s) + solve to 1e-10 (%.1f s, %d cycles) of the same "
                "problem on %dx%dx2 triangles (%d rows), scaled x%.0f by rows"
                % (d["setup_s"], d["solve_s"], d["iters"], m_sample, m_sample, d["n"],
                   n_full / d["n"]))
    return _both_thread_counts(code, to_ms, describe)


def cpu_baseline(workload, kw, x_path=None, cycles=None):
    """Time the CPU oracle on a bounded sample: the full setup of the
    workload plus the solve of its first right-hand side, the solve time
    scaled by the number of right-hand sides (with `cycles`, that many
    cycles instead of a solve to 1e-10).  The one-core run also writes the
    oracle's solution of right-hand side 0 to x_path."""
    def code(first):
        return r"""
import json, sys, time
sys.path.insert(0, %r)
import numpy as np
import bench
from oracle import lair as O
w, kw, cfg = bench.make_workload(%r)
A = O.csr(w["rowptr"], w["col"], w["val"])
interp = O.INTERP_DIRECT if kw["interp"] == "direct" else O.INTERP_ONE_POINT
b = np.asarray(w["rhs"])
b0 = b[:, 0] if b.ndim > 1 else b
t0 = time.perf_counter()
if kw.get("block_size"):
    A, b0 = O.block_scale(A, b0, kw["block_size"])
H = O.setup(A, interp=interp, distance=kw["distance"], lump_tol=%r)
t1 = time.perf_counter()
cyc = %r
if cyc:
    x, it, hist = O.solve(H, b0, rtol=0.0, maxit=cyc)
else:
    x, it, hist = O.solve(H, b0, rtol=1e-10, maxit=100)
t2 = time.perf_counter()
xp = %r
if xp:
    np.save(xp, x)
print(json.dumps({"setup_s": t1 - t0, "solve_s": t2 - t1, "iters": it,
                  "relres": float(hist[-1] / hist[0]),
                  "nrhs": 1 if b.ndim == 1 else b.shape[1]}))
""" % (ROOT, workload, kw.get("lump_tol", 0.0), cycles, x_path if first else None)

    def to_ms(d):
        return 1e3 * (d["setup_s"] + d["nrhs"] * d["solve_s"])

    def describe(d):
        what = ("%d cycles (relres %.2e)" % (d["iters"], d["relres"]) if cycles
                else "to 1e-10 (%d cycles)" % d["iters"])
        return ("full-size oracle setup (%.1f s, CF split included) + solve of right-hand "
                "side 0 of %d %s in %.1f s, solve time scaled x%d"
                % (d["setup_s"], d["nrhs"], what, d["solve_s"], d["nrhs"]))
    return _both_thread_counts(code, to_ms, describe)


def summarize_trace(d, out, title, command, top=30):
    """Markdown summary of a rocprofv3 --kernel-trace --stats run (the
    kernel_stats CSV under d): the top kernels by total time."""
    import csv
    import glob
    files = glob.glob(os.path.join(d, "**", "*kernel_stats.csv"), recursive=True)
    if not files:
        raise SystemExit("no kernel_stats.csv under %s" % d)
    rows = list(csv.DictReader(open(files[0])))
    tot = sum(float(r["TotalDurationNs"]) for r in rows)
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    lines = ["# Kernel profile: %s" % title, "", "Command (repository root, one MI355X, "
             "`cd /tmp && export TMPDIR=/tmp` for the profiler's files):", "", "```",
             command, "```", "",
             "## Kernel time (rocprofv3 --stats), top %d of %.1f ms" % (top, tot * 1e-6), "",
             "| kernel | calls | total ms | avg us | % |", "|---|---|---|---|---|"]
    for r in rows[:top]:
        lines.append("| `%s` | %s | %.3f | %.1f | %.1f |" % (
            r["Name"], r["Calls"], float(r["TotalDurationNs"]) * 1e-6,
            float(r["AverageNs"]) * 1e-3, 100.0 * float(r["TotalDurationNs"]) / tot))
    open(out, "w").write("\n".join(lines) + "\n")
    print(out)


def _counter_per_launch(d, counter, kernel_regex):
    """(KiB per launch of the kernels matching kernel_regex, launches, KiB
    of the calibration copy kernel) from a rocprofv3 --pmc CSV run."""
    import csv
    import glob
    import re
    files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise SystemExit("no counter_collection.csv under %s" % d)
    rx = re.compile(kernel_regex)
    per, copy = {}, []
    for f in files:
        for r in csv.DictReader(open(f)):
            if r.get("Counter_Name") != counter:
                continue
            name = r["Kernel_Name"]
            v = float(r["Counter_Value"])
            if "copyBuffer" in name:
                copy.append(v)
            if rx.search(name):
                per[r["Dispatch_Id"]] = per.get(r["Dispatch_Id"], 0.0) + v
    if not per or not copy:
        raise SystemExit("counter %s: no launch of %s or no copy kernel" % (counter, kernel_regex))
    return sum(per.values()) / len(per), len(per), max(copy)


def summarize_counters(fetch_dir, write_dir, workload, category, kernel_regex, cfg_key,
                       alg_per_launch, calib_mib, commands, out):
    """HBM bytes per launch of a kernel category from two rocprofv3 --pmc
    runs (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch), each scaled by
    what the counter reads for the calibration copy of calib_mib MiB."""
    rec = {"workload": workload, "category": category, "config": cfg_key,
           "kernel_regex": kernel_regex,
           "calibration": "%d MiB device copy (copyBuffer) read and written once: counted KiB "
                          "scaled to %d" % (calib_mib, calib_mib * 1024),
           "commands": commands, "algorithmic_bytes_per_launch": alg_per_launch,
           "source_sha256": source_hashes()}
    for key, d, ctr in (("fetch", fetch_dir, "FETCH_SIZE"), ("write", write_dir, "WRITE_SIZE")):
        kib, n, copy = _counter_per_launch(d, ctr, kernel_regex)
        factor = calib_mib * 1024.0 / copy
        rec[key] = {"counter": ctr, "copy_kib": copy, "factor": factor, "launches": n,
                    "kib_per_launch": kib, "bytes_per_launch": kib * factor * 1024.0}
    rec["traffic_over_algorithmic"] = (rec["fetch"]["bytes_per_launch"] +
                                       rec["write"]["bytes_per_launch"]) / alg_per_launch
    json.dump(rec, open(out, "w"), indent=1)
    print(out, "traffic / algorithmic = %.3f" % rec["traffic_over_algorithmic"])


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
    ap.add_argument("--summarize-trace", metavar="DIR", default=None)
    ap.add_argument("--summarize-counters", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    default=None)
    ap.add_argument("--category", default="jacobi")
    ap.add_argument("--kernel-regex", default=None)
    ap.add_argument("--alg-bytes-per-launch", type=float, default=0.0)
    ap.add_argument("--out", default=None)
    ap.add_argument("--title", default="")
    ap.add_argument("--command", action="append", default=[])
    args = ap.parse_args()
    if args.summarize_trace:
        summarize_trace(args.summarize_trace, args.out, args.title, "\n".join(args.command))
        return
    if args.gpus != 1:
        print("bench.py measures one GPU: this lAIR build is single-GPU (the "
              "design notes describe how it would shard); --gpus %d is not "
              "supported" % args.gpus, file=sys.stderr)
        sys.exit(2)
    c2 = args.workload == "c2"

    def cfg_key():
        return {"workload": args.workload, "lump_tol": 0.0 if c2 else args.lump,
                "split": args.split, "distance": args.distance, "solver": args.solver,
                "precision": "mixed_local" if c2 else "mixed"}

    if args.summarize_counters:
        summarize_counters(args.summarize_counters[0], args.summarize_counters[1],
                           args.workload, args.category, args.kernel_regex, cfg_key(),
                           args.alg_bytes_per_launch, args.copy_calibration_mib, args.command,
                           args.out)
        return

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
    if kw.get("nodal") or c2:
        # lumping would break the dense blocks a nodal hierarchy keeps; the
        # DG configuration is defined without it
        args.lump = 0.0
    kw = dict(kw, lump_tol=args.lump)
    cfg = dict(cfg, lumping=args.lump)
    # the variant timed for the value, and the plain FP64 one beside it
    main_prec = "mixed_local" if c2 else "mixed"

    def build(cf_levels=None, precision="fp64"):
        if batch:
            return lair.setup_batch(members, cf_levels=cf_levels, precision=precision, **kw)
        return lair.setup(rp, cj, vv, cf_levels=cf_levels, precision=precision, **kw)

    # CF splitting per level by the library's own first pass (untimed); its
    # host time is reported on its own
    t0 = time.perf_counter()
    h0 = build()
    torch.cuda.synchronize()
    t_full_setup = (time.perf_counter() - t0) * 1e3
    # the splittings stay in device memory for the timed setups
    cfl = [torch.as_tensor(h0.export(l, "cf"), device=dev) for l in range(h0.nlevels - 1)]
    nlev = h0.nlevels
    if batch:
        _, i0 = h0.solve_batch(B, rtol=1e-10, maxit=0)
    else:
        _, i0 = h0.solve(B, rtol=1e-10, maxit=0)
    split_ms = i0["split_ms"]
    h0.free()
    log("library CF split + setup: %.1f ms (host first pass %.1f ms), %d levels"
        % (t_full_setup, split_ms, nlev))

    # the nodal DG workload needs 54 cycles at 256 x 256 x 2 (101 at distance 1)
    maxit = C2_CYCLES if c2 else (300 if kw.get("nodal") else 100)
    rtol = 1e-30 if c2 else 1e-10

    def step(precision):
        h = build(None if args.split == "pmis" else cfl, precision)
        if batch:
            X, info = h.solve_batch(B, rtol=rtol, maxit=maxit)
        elif args.solver == "fgmres":
            X, info = h.solve_fgmres(B, rtol=rtol, maxit=maxit, restart=args.restart)
        else:
            X, info = h.solve(B, rtol=rtol, maxit=maxit)
        return h, X, info

    # which kernel category dominates a step: one profiled, untimed step
    # after a warm-up step (so that first-use allocations are not in it)
    h, X, info = step(main_prec)
    h.free()
    lair.profile_begin(None)
    h, X, info = step(main_prec)
    torch.cuda.synchronize()
    prof_all = lair.profile_end()
    h.free()
    dominant = max(prof_all.items(), key=lambda kv: kv[1]["ms"])[0]
    log("profiled step, per category:", json.dumps(prof_all))
    log("per-category GPU time of one %s step (ms):" % main_prec,
        json.dumps({k: round(v["ms"], 3) for k, v in sorted(prof_all.items(),
                                                              key=lambda kv: -kv[1]["ms"])}))

    results, prof_timed, x_main = {}, None, None
    for prec in ([main_prec] if args.no_fp64 else [main_prec, "fp64"]):
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
        if prec == main_prec:
            x_main = (X[:, 0] if X.dim() > 1 else X).cpu().numpy()
            # the dominant category's kernels timed with HIP events on their
            # streams over as many steps again (the profiler launches a
            # profiled cycle's kernels one by one, so it stays out of the
            # timed steps above)
            h.free()
            lair.profile_begin([dominant])
            for k in range(args.steps):
                h, X, info = step(prec)
                if k < args.steps - 1:
                    h.free()
            torch.cuda.synchronize()
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
        last = infos[-1]
        results[prec] = dict(ms=float(np.median(times)), ms_all=times, iters=last["iters"],
                             relres=last["relres"], relres_check=rel,
                             setup_ms=last["setup_ms"], solve_ms=last["solve_ms"],
                             rho=last["rho"], cc=last["cycle_complexity"],
                             oc=last["op_complexity"], wpd=last["wpd"],
                             setup_phase_ms=last["setup_phase_ms"][:6],
                             relres_hist=last["relres_hist"])
        log(prec, json.dumps(results[prec]))

    r = results[main_prec]
    d = prof_timed.get(dominant, {"launches": 0, "ms": 1.0, "alg_bytes": 0.0})
    achieved = d["alg_bytes"] / (d["ms"] * 1e-3) / 1e9 if d["ms"] > 0 else 0.0
    per_launch = d["alg_bytes"] / max(d["launches"], 1)
    roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS,
                "traffic": measured_traffic(args.workload, dominant, cfg_key(), per_launch),
                "kernel": dominant, "launches": d["launches"],
                "avg_launch_us": 1e3 * d["ms"] / max(d["launches"], 1),
                "alg_bytes_per_launch": per_launch}
    # the whole step: every category's algorithmic bytes over the step time
    step_bytes = sum(v["alg_bytes"] for v in prof_all.values())
    step_flops = sum(v["alg_flops"] for v in prof_all.values())
    step_roof = {"alg_bytes": step_bytes, "achieved": step_bytes / (r["ms"] * 1e-3) / 1e9,
                 "peak": HBM_PEAK_GBS, "unit": "GB/s",
                 "frac": step_bytes / (r["ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS,
                 "gpu_busy_ms": sum(v["ms"] for v in prof_all.values())}
    local = {k: v for k, v in prof_all.items() if k.startswith("local")}
    local_roof = None
    if local:
        lf = sum(v["alg_flops"] for v in local.values())
        lms = sum(v["ms"] for v in local.values())
        local_roof = {"bound": "valu_fp64" if main_prec == "fp64" else "valu",
                      "alg_flops": lf, "ms": lms,
                      "achieved_tflops": lf / (lms * 1e-3) / 1e12 if lms > 0 else 0.0,
                      "fp64_peak_tflops": FP64_VALU_PEAK_TFS,
                      "frac_of_fp64_peak": lf / (lms * 1e-3) / 1e12 / FP64_VALU_PEAK_TFS
                      if lms > 0 else 0.0}
    metric = ("setup + %d V-cycles (the stationary iteration does not reach 1e-10 on this "
              "recirculating problem), FP32 local LU + FP64 refinement vs FP64" % C2_CYCLES
              if c2 else "time to 1e-10 rel. residual (setup+solve), mixed vs FP64")
    out = {
        "metric": metric,
        "value": r["ms"],
        "unit": "ms",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms"],
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": ("f32 local LU + f64 refinement, f64 cycle" if c2
                  else "f32 cycle/local LU + f64 outer"),
        "data": "synthetic",
        "config": cfg,
        "iters": r["iters"],
        "relres": r["relres"],
        "relres_check_fp64": r["relres_check"],
        "rho": r["rho"],
        "wpd": r["wpd"],
        "cycle_complexity": r["cc"],
        "op_complexity": r["oc"],
        "relres_hist": r["relres_hist"],
        "setup_ms": r["setup_ms"],
        "setup_phase_ms": dict(zip(("input", "strength_split", "nbr_interp_local",
                                    "galerkin_lump", "coarsest", "cycle_operators"),
                                   r["setup_phase_ms"])),
        "solve_ms": r["solve_ms"],
        "cf_split_host_ms_untimed": split_ms,
        "cf_split_plus_setup_ms_untimed": t_full_setup,
        "levels": nlev,
        "roofline": roofline,
        "step_roofline": step_roof,
        "gpu_ms_by_category": {k: round(v["ms"], 3) for k, v in prof_all.items()},
        # per category of the profiled step: launches, algorithmic bytes and
        # the fraction of the HBM peak they reach
        "category_roofline": {k: {"launches": v["launches"],
                                  "alg_gb": round(v["alg_bytes"] * 1e-9, 4),
                                  "frac": round(v["alg_bytes"] / (max(v["ms"], 1e-9) * 1e-3)
                                                * 1e-9 / HBM_PEAK_GBS, 4)}
                              for k, v in prof_all.items()},
    }
    if c2:
        out["converged"] = False
    if local_roof:
        out["local_solve_roofline"] = local_roof
    if "fp64" in results:
        out["fp64"] = {k: results["fp64"][k] for k in ("ms", "iters", "relres", "setup_ms",
                                                        "solve_ms", "wpd")}
        out["speedup_mixed_vs_fp64"] = results["fp64"]["ms"] / r["ms"]
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a bounded sample (one core, then every core) ...")
        import tempfile
        xp = os.path.join(tempfile.mkdtemp(prefix="lair_bench_"), "x0.npy")
        if batch:
            cb = cpu_baseline_batch(kw, x_path=xp)
        elif kw.get("nodal"):
            gen = ("workload_dgu(%%d, %r)" % DGU_KAPPA if args.workload == "dgu"
                   else "workload_dg_curved(%d)")
            cb = cpu_baseline_nodal(kw, w["n"], gen, x_path=xp)
        else:
            cb = cpu_baseline(args.workload, kw, xp, cycles=C2_CYCLES if c2 else None)
        if cb:
            out["cpu_baseline"] = cb
        if x_main is not None and os.path.exists(xp) and batch:
            # every system the oracle solved (the first ones of the union)
            xo = np.load(xp)
            sys_n = [q["n"] for q in w["systems"]]
            errs, lo = [], 0
            for nq in sys_n:
                if lo + nq > xo.size:
                    break
                xq = xo[lo:lo + nq]
                errs.append(float(np.linalg.norm(x_main[lo:lo + nq] - xq) /
                                  max(np.linalg.norm(xq), 1e-300)))
                lo += nq
            out["err_vs_fp64_oracle"] = {"max_rel": max(errs), "median_rel": float(np.median(errs)),
                                         "systems": len(errs),
                                         "sample": "the first %d of 512 systems, each against the "
                                                   "oracle's FP64 solve to 1e-10" % len(errs)}
        elif kw.get("nodal") and os.path.exists(xp):
            # the full-size oracle would take minutes: the GPU solves the
            # oracle's sample problem in the timed precision and is
            # compared there
            import workloads as W
            m = DG_ORACLE_SAMPLE
            ws = (W.workload_dgu(m, DGU_KAPPA) if args.workload == "dgu"
                  else W.workload_dg_curved(m))
            hs = lair.setup(torch.as_tensor(ws["rowptr"], device=dev),
                            torch.as_tensor(ws["col"], device=dev),
                            torch.as_tensor(ws["val"], device=dev), precision=main_prec, **kw)
            bs = torch.as_tensor(np.ascontiguousarray(np.asarray(ws["rhs"], dtype=np.float64)),
                                 device=dev)
            xs, _ = hs.solve(bs, rtol=1e-10, maxit=maxit)
            hs.free()
            xo = np.load(xp)
            out["err_vs_fp64_oracle"] = {
                "rel": float(np.linalg.norm(xs.cpu().numpy() - xo) / np.linalg.norm(xo)),
                "sample": "the same problem on %dx%dx2 triangles (%d rows), GPU in the timed "
                          "precision against the oracle's FP64 solve to 1e-10" % (m, m, ws["n"])}
        elif x_main is not None and os.path.exists(xp):
            xo = np.load(xp)
            out["err_vs_fp64_oracle_rhs0"] = float(np.linalg.norm(x_main - xo) /
                                                   np.linalg.norm(xo))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
