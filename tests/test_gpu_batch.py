"""GPU tests of the batched path and of graph-captured iterations.

A batch of independent advection-diffusion-reaction systems of uneven size
(the recipe of the 512-system workload at reduced sizes, plus a 1 x 1
system) is set up and solved as one block-diagonal union.  Every member must
equal the oracle's own single-system run, level by level on the GPU's member
block of A_l: strength pattern, CF splitting, neighbourhoods, fallback flags
and the R, P and K patterns bit-exact; R rows within 1e-12 (row-relative), K
within 1e-12 of |R||A||P|.  A member that stopped coarsening passes through
later levels unchanged (all C-points, identity R and P, its block of K
bitwise its block of A).  Its level count and its FP64 iteration count to
1e-10 equal the oracle's; mixed precision takes at most one more cycle.

Graph capture: solves replaying captured iterations give bitwise the result
of eager launches, over several solves with new right-hand sides in the same
buffers and other GPU work in between.
"""
import sys

import numpy as np
import pytest
import scipy.sparse as sp

import workloads as W
from oracle import lair as O
from tests.parity import _lump_scale, gpu_A, rows_rel_err

pytestmark = pytest.mark.gpu

MC = 40   # max_coarse for the small batch


@pytest.fixture(scope="module")
def lair():
    import torch
    import paper_1708_06065_amd as lair
    assert torch.cuda.is_available()
    lair.load_library()
    return lair


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _dev(x):
    import torch
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


def _systems():
    sy = W.adr_batch(nsys=10, nmin=6, nmax=40, seed=3)
    one = dict(n=1, nnz=1, rowptr=np.array([0, 1], np.int32), col=np.array([0], np.int32),
               val=np.array([2.5]), rhs=np.array([1.0]))
    sy.insert(3, one)
    return sy


def _level_segs(h, seg0):
    """Row offsets of the members on every level (from the exported CF)."""
    segs = [np.asarray(seg0, dtype=np.int64)]
    for l in range(h.nlevels - 1):
        cf = h.export(l, "cf").astype(np.int64)
        s = segs[-1]
        c = np.concatenate([[0], np.cumsum(cf)])
        segs.append(c[s])
    return segs


def _block(M, r0, r1, c0, c1):
    B = M[r0:r1, c0:c1].tocsr()
    assert M[r0:r1].nnz == B.nnz, "entries outside the member's block"
    return B


def _identity_check(B):
    n = B.shape[0]
    assert B.shape[0] == B.shape[1]
    assert np.array_equal(B.indptr, np.arange(n + 1))
    assert np.array_equal(B.indices, np.arange(n))
    assert np.all(B.data == 1.0)


def _check_member_levels(h, systems, segs, interp, lump_tol=0.0):
    nl = h.nlevels
    sys_levels = h.system_levels()
    worst = {"z": 0.0, "k": 0.0}
    As = [gpu_A(h, l) for l in range(nl)]
    for l in range(nl - 1):
        A = As[l]
        Anext = As[l + 1]
        n = A.shape[0]
        nc = Anext.shape[0]
        sm = h.export(l, "smask")
        cf = h.export(l, "cf")
        nbp = h.export(l, "nbr_ptr")
        nbr = h.export(l, "nbr")
        flg = h.export(l, "flags")
        R = O.csr(h.export(l, "R.rowptr"), h.export(l, "R.col"), h.export(l, "R.val"),
                  shape=(nc, n))
        P = O.csr(h.export(l, "P.rowptr"), h.export(l, "P.col"), h.export(l, "P.val"),
                  shape=(n, nc))
        for q in range(len(systems)):
            s0, s1 = segs[l][q], segs[l][q + 1]
            c0, c1 = segs[l + 1][q], segs[l + 1][q + 1]
            Aq = _block(A, s0, s1, s0, s1)
            Kq = _block(Anext, c0, c1, c0, c1)
            Rq = _block(R, c0, c1, s0, s1)
            Pq = _block(P, s0, s1, c0, c1)
            if l >= sys_levels[q] - 1:
                # pass-through: all C, identity transfer, K block == A block
                assert np.all(cf[s0:s1] == 1), (l, q)
                _identity_check(Rq)
                _identity_check(Pq)
                assert np.array_equal(Kq.indptr, Aq.indptr) and np.array_equal(Kq.indices, Aq.indices)
                assert np.array_equal(Kq.data, Aq.data), (l, q)
                continue
            sm_o = O.strength(Aq, 0.25)
            assert np.array_equal(sm_o, sm[A.indptr[s0]:A.indptr[s1]]), (l, q)
            cf_o = O.rs_split(Aq, sm_o)
            assert np.array_equal(cf_o, cf[s0:s1]), (l, q)
            cpts, nptr, nb = O.neighbourhoods(Aq, sm_o, cf_o, 1)
            assert np.array_equal(nptr, nbp[c0:c1 + 1] - nbp[c0]), (l, q)
            assert np.array_equal(nb, nbr[nbp[c0]:nbp[c1]] - s0), (l, q)
            z, flags = O.local_solves(Aq, cpts, nptr, nb)
            assert np.array_equal(flags.astype(np.int8), flg[c0:c1]), (l, q)
            Ro = O.restriction(Aq.shape[0], cpts, nptr, nb, z)
            assert np.array_equal(Ro.indptr, Rq.indptr) and np.array_equal(Ro.indices, Rq.indices)
            ze = rows_rel_err(Rq.indptr, Rq.data, Ro.data)
            assert ze <= 1e-12, (l, q, ze)
            Po = O.interp_direct(Aq, sm_o, cf_o) if interp == "direct" else \
                O.interp_one_point(Aq, sm_o, cf_o)
            assert np.array_equal(Po.indptr, Pq.indptr) and np.array_equal(Po.indices, Pq.indices)
            assert np.allclose(Pq.data, Po.data, rtol=1e-13, atol=1e-15)
            Ko = O.galerkin(Ro, Aq, Po)
            S = O.galerkin(abs(Ro), abs(Aq), abs(Po))
            if lump_tol > 0.0:
                Ko.sort_indices()
                S.sort_indices()
                S = _lump_scale(Ko, S, lump_tol)
                Ko = O.lump(Ko, lump_tol)
            assert np.array_equal(Ko.indptr, Kq.indptr) and np.array_equal(Ko.indices, Kq.indices)
            scale = S.data
            ke = float((np.abs(Kq.data - Ko.data) / np.maximum(scale, 1e-300)).max()) \
                if scale.shape[0] else 0.0
            assert ke <= 1e-12, (l, q, ke)
            worst["z"] = max(worst["z"], ze)
            worst["k"] = max(worst["k"], ke)
    return worst


@pytest.mark.parametrize("interp", ["direct", "one_point"])
def test_batch_members_equal_single_runs(lair, interp):
    systems = _systems()
    seg0 = np.concatenate([[0], np.cumsum([w["n"] for w in systems])])
    h = lair.setup_batch([(w["rowptr"], w["col"], w["val"]) for w in systems],
                         interp=interp, max_coarse=MC)
    assert h.nsys == len(systems)
    _say("  batch of %d systems, sizes %s, union levels %d, member levels %s"
         % (len(systems), [w["n"] for w in systems], h.nlevels, list(h.system_levels())))
    okw = dict(interp=O.INTERP_DIRECT if interp == "direct" else O.INTERP_ONE_POINT,
               max_coarse=MC)
    Hs = [O.setup(O.csr(w["rowptr"], w["col"], w["val"]), **okw) for w in systems]
    assert list(h.system_levels()) == [H.nlevels for H in Hs]
    assert h.nlevels == max(H.nlevels for H in Hs)
    segs = _level_segs(h, seg0)
    worst = _check_member_levels(h, systems, segs, interp)
    _say("  worst R row error %.2e, worst K error %.2e" % (worst["z"], worst["k"]))
    # solve: per-system iteration counts equal the oracle's
    b = np.concatenate([w["rhs"] for w in systems])
    x, info = h.solve_batch(_dev(b), rtol=1e-10)
    assert info["converged"]
    X = x.cpu().numpy()
    for q, (w, H) in enumerate(zip(systems, Hs)):
        _, ito, _ = O.solve(H, w["rhs"], rtol=1e-10)
        assert info["sys_iters"][q] == ito, (q, info["sys_iters"][q], ito)
        Aq = O.csr(w["rowptr"], w["col"], w["val"])
        xq = X[seg0[q]:seg0[q + 1]]
        assert np.linalg.norm(w["rhs"] - Aq @ xq) <= 1e-10 * np.linalg.norm(w["rhs"])
        assert info["sys_relres"][q] <= 1e-10
    _say("  iterations per system:", list(info["sys_iters"]))


def _c3_sample():
    """The first 24 systems of the 512-system workload (seed 3, drawn in
    order) plus its largest and its smallest system."""
    allsys = W.adr_batch(512, seed=3)
    sizes = np.array([w["n"] for w in allsys])
    pick = list(range(24))
    for q in (int(np.argmax(sizes)), int(np.argmin(sizes))):
        if q not in pick:
            pick.append(q)
    return [allsys[q] for q in pick]


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_c3_recipe_batch_members_against_oracle(lair, precision):
    """Systems of the 512-system workload at their own sizes (N from 32 to
    320), set up and solved as the benchmark does (direct interpolation,
    coarse operators lumped at 0.001, default coarsest size): every member's
    levels against the oracle's single-system run on the GPU's member
    blocks, pass-through blocks unchanged, and each member's cycle count
    equal to the oracle's (mixed precision: at most one more), its solution
    within 1e-8 of the oracle's."""
    systems = _c3_sample()
    seg0 = np.concatenate([[0], np.cumsum([w["n"] for w in systems])])
    _say("case: C3 recipe batch, %d systems, N %s, %s" %
         (len(systems), [int(round(np.sqrt(w["n"]))) for w in systems], precision))
    h = lair.setup_batch([(w["rowptr"], w["col"], w["val"]) for w in systems],
                         interp="direct", lump_tol=1e-3, precision=precision)
    Hs = [O.setup(O.csr(w["rowptr"], w["col"], w["val"]), interp=O.INTERP_DIRECT,
                  lump_tol=1e-3) for w in systems]
    assert list(h.system_levels()) == [H.nlevels for H in Hs]
    if precision == "fp64":
        segs = _level_segs(h, seg0)
        worst = _check_member_levels(h, systems, segs, "direct", lump_tol=1e-3)
        _say("  worst R row error %.2e, worst K error %.2e" % (worst["z"], worst["k"]))
    b = np.concatenate([w["rhs"] for w in systems])
    x, info = h.solve_batch(_dev(b), rtol=1e-10, maxit=100)
    assert info["converged"]
    X = x.cpu().numpy()
    worst_err = 0.0
    for q, (w, H) in enumerate(zip(systems, Hs)):
        xo, ito, _ = O.solve(H, w["rhs"], rtol=1e-10, maxit=100)
        it = int(info["sys_iters"][q])
        if precision == "fp64":
            assert it == ito, (q, it, ito)
        else:
            assert it <= ito + 1, (q, it, ito)
        xq = X[seg0[q]:seg0[q + 1]]
        err = np.linalg.norm(xq - xo) / np.linalg.norm(xo)
        worst_err = max(worst_err, err)
        assert err <= 1e-8, (q, err)
    _say("  cycles per system:", list(info["sys_iters"]),
         "max rel err vs FP64 oracle %.2e" % worst_err)


def test_batch_mixed_precision(lair):
    systems = _systems()
    seg0 = np.concatenate([[0], np.cumsum([w["n"] for w in systems])])
    h = lair.setup_batch([(w["rowptr"], w["col"], w["val"]) for w in systems],
                         interp="direct", precision="mixed", max_coarse=MC)
    b = np.concatenate([w["rhs"] for w in systems])
    x, info = h.solve_batch(_dev(b), rtol=1e-10)
    assert info["converged"]
    X = x.cpu().numpy()
    for q, w in enumerate(systems):
        H = O.setup(O.csr(w["rowptr"], w["col"], w["val"]), interp=O.INTERP_DIRECT,
                    max_coarse=MC)
        _, ito, _ = O.solve(H, w["rhs"], rtol=1e-10)
        assert info["sys_iters"][q] <= ito + 1, (q, info["sys_iters"][q], ito)
        Aq = O.csr(w["rowptr"], w["col"], w["val"])
        r = w["rhs"] - Aq @ X[seg0[q]:seg0[q + 1]]
        assert np.linalg.norm(r) <= 1e-10 * np.linalg.norm(w["rhs"])
    _say("  mixed iterations per system:", list(info["sys_iters"]))


def test_batch_from_device_arrays_equals_host(lair):
    import torch
    systems = _systems()
    hh = lair.setup_batch([(w["rowptr"], w["col"], w["val"]) for w in systems],
                          interp="direct", max_coarse=MC)
    dev = [(torch.as_tensor(w["rowptr"], device="cuda"), torch.as_tensor(w["col"], device="cuda"),
            torch.as_tensor(w["val"], device="cuda")) for w in systems]
    hd = lair.setup_batch(dev, interp="direct", max_coarse=MC)
    assert hh.nlevels == hd.nlevels
    for l in range(hh.nlevels):
        for what in ("A.rowptr", "A.col", "A.val"):
            assert np.array_equal(hh.export(l, what), hd.export(l, what)), (l, what)


def test_batch_errors(lair):
    import torch
    from paper_1708_06065_amd import LairError
    systems = _systems()[:3]
    h1 = lair.setup(systems[0]["rowptr"], systems[0]["col"], systems[0]["val"])
    with pytest.raises(LairError):
        h1.solve_batch(_dev(systems[0]["rhs"]))
    hb = lair.setup_batch([(w["rowptr"], w["col"], w["val"]) for w in systems],
                          max_coarse=MC)
    n = sum(w["n"] for w in systems)
    with pytest.raises(LairError):
        hb.solve(torch.zeros((n, 2), dtype=torch.float64, device="cuda"))
    bad = dict(systems[1])
    bad_col = bad["col"].copy()
    bad_col[-1] = bad["n"]            # column outside the member's rows
    dev = [(torch.as_tensor(w["rowptr"], device="cuda"), torch.as_tensor(w["col"], device="cuda"),
            torch.as_tensor(w["val"], device="cuda")) for w in systems]
    dev[1] = (dev[1][0], torch.as_tensor(bad_col, device="cuda"), dev[1][2])
    with pytest.raises(LairError):
        lair.setup_batch(dev)


# ------------------------------------------------------------------ graphs

def _busy(torch):
    a = torch.randn(512, 512, device="cuda", dtype=torch.float32)
    return float((a @ a).sum().item())


@pytest.mark.parametrize("precision,nrhs", [("fp64", 4), ("mixed", 1), ("fp64", 1)])
def test_graph_replays_equal_eager(lair, precision, nrhs):
    import torch
    w = W.implicit_euler_adr_3d(m=20, nrhs=nrhs, seed=7)
    kw = dict(interp="direct", precision=precision)
    hg = lair.setup(w["rowptr"], w["col"], w["val"], **kw)
    he = lair.setup(w["rowptr"], w["col"], w["val"], graphs=False, **kw)
    for l in range(hg.nlevels):
        assert np.array_equal(hg.export(l, "A.val"), he.export(l, "A.val"))
    n = w["n"]
    shape = (n,) if nrhs == 1 else (n, nrhs)
    B = torch.zeros(shape, dtype=torch.float64, device="cuda")
    Xg = torch.zeros_like(B)
    Xe = torch.zeros_like(B)
    rng = np.random.default_rng(11)
    for rep in range(3):
        B.copy_(_dev(rng.standard_normal(shape)))
        Xg.zero_()
        Xe.zero_()
        _busy(torch)
        _, ig = hg.solve(B, Xg, rtol=1e-10)
        _busy(torch)
        _, ie = he.solve(B, Xe, rtol=1e-10)
        torch.cuda.synchronize()
        assert ig["iters"] == ie["iters"] and ig["converged"]
        assert torch.equal(Xg, Xe), "replay %d differs from eager" % rep
        _say("  replay round %d: %d iterations, bitwise equal" % (rep, ig["iters"]))


def test_batch_graph_replays_equal_eager(lair):
    import torch
    systems = _systems()
    mats = [(w["rowptr"], w["col"], w["val"]) for w in systems]
    hg = lair.setup_batch(mats, interp="direct", max_coarse=MC)
    he = lair.setup_batch(mats, interp="direct", max_coarse=MC, graphs=False)
    n = sum(w["n"] for w in systems)
    B = torch.zeros(n, dtype=torch.float64, device="cuda")
    Xg = torch.zeros_like(B)
    Xe = torch.zeros_like(B)
    rng = np.random.default_rng(12)
    for rep in range(3):
        B.copy_(_dev(rng.standard_normal(n)))
        Xg.zero_()
        Xe.zero_()
        _busy(torch)
        _, ig = hg.solve_batch(B, Xg, rtol=1e-10)
        _busy(torch)
        _, ie = he.solve_batch(B, Xe, rtol=1e-10)
        torch.cuda.synchronize()
        assert np.array_equal(ig["sys_iters"], ie["sys_iters"])
        assert torch.equal(Xg, Xe), "batch replay %d differs from eager" % rep


def test_c3_full_batch_sampled_members(lair):
    """The whole 512-system workload in one batch, as the benchmark runs it
    (direct interpolation, lumped at 0.001, mixed precision): every member
    converges with its own residual below 1e-10 (checked independently),
    and sampled members (the largest, the smallest and ten seeded picks)
    have the oracle's level count, at most one cycle more than the oracle's
    single-system solve, and its solution to 1e-8."""
    allsys = W.adr_batch(512, seed=3)
    sizes = np.array([w["n"] for w in allsys])
    seg0 = np.concatenate([[0], np.cumsum(sizes)])
    _say("case: C3 full batch, 512 systems, %d rows" % seg0[-1])
    h = lair.setup_batch([(w["rowptr"], w["col"], w["val"]) for w in allsys],
                         interp="direct", lump_tol=1e-3, precision="mixed")
    b = np.concatenate([w["rhs"] for w in allsys])
    x, info = h.solve_batch(_dev(b), rtol=1e-10, maxit=100)
    assert info["converged"]
    X = x.cpu().numpy()
    worst_res = 0.0
    for q, w in enumerate(allsys):
        A = O.csr(w["rowptr"], w["col"], w["val"])
        xq = X[seg0[q]:seg0[q + 1]]
        worst_res = max(worst_res, np.linalg.norm(w["rhs"] - A @ xq) / np.linalg.norm(w["rhs"]))
    _say("  largest member relative residual %.2e, cycles %d" % (worst_res, info["iters"]))
    assert worst_res <= 1e-10 * (1 + 1e-6)
    rng = np.random.default_rng(11)
    pick = sorted({int(np.argmax(sizes)), int(np.argmin(sizes))} |
                  set(int(q) for q in rng.choice(512, size=10, replace=False)))
    levels = h.system_levels()
    for q in pick:
        w = allsys[q]
        H = O.setup(O.csr(w["rowptr"], w["col"], w["val"]), interp=O.INTERP_DIRECT,
                    lump_tol=1e-3)
        assert levels[q] == H.nlevels, (q, levels[q], H.nlevels)
        xo, ito, _ = O.solve(H, w["rhs"], rtol=1e-10, maxit=100)
        it = int(info["sys_iters"][q])
        err = np.linalg.norm(X[seg0[q]:seg0[q + 1]] - xo) / np.linalg.norm(xo)
        _say("  system %d (N = %d): cycles gpu %d oracle %d, rel. error %.2e"
             % (q, int(round(np.sqrt(w["n"]))), it, ito, err))
        assert ito <= it <= ito + 1
        assert err <= 1e-8
    h.free()
