"""GPU tests of the adjoint (transposed cycle, autograd) and of mixed precision.

Adjoint: one transposed cycle is the exact adjoint of one forward cycle;
the transposed solve matches a dense A^T solve; gradients of
J = ||x - x_obs||^2 with respect to b and the reaction field c match the
dense adjoint gradient (1e-8) and central finite differences (h = 1e-6,
1e-6 relative), all on the 64 x 64 advection-diffusion-reaction workload.

Mixed precision: float LU plus one double refinement per row of Z, float
cycle under a double outer iteration.  Each row of Z is checked against the
FP64 oracle with the refinement bound of mixed-precision iterative
refinement, c ((k u32)^2 + k u64) with k the condition number of the local
matrix; the solve reaches the same 1e-10 double residual.
"""
import sys

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import workloads as W
from oracle import lair as O
from tests.parity import compare_level, gpu_A, oracle_cf_levels

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24
U64 = 2.0 ** -53


@pytest.fixture(scope="module")
def lair():
    import torch
    import paper_1708_06065_amd as lair
    assert torch.cuda.is_available()
    lair.load_library()
    return lair


def _dev(x):
    import torch
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _c4(m=64):
    w = W.workload_c4(m)
    A0 = O.csr(w["rowptr"], w["col"], w["val"])
    A = (A0 + sp.diags(w["c"])).tocsr()
    A.sort_indices()
    return w, A0, A


# ------------------------------------------------------------------ adjoint

def test_transpose_cycle_is_adjoint(lair):
    _, _, A = _c4(40)
    h = lair.setup(A.indptr, A.indices, A.data, interp="direct", max_coarse=30)
    assert h.nlevels >= 3
    rng = np.random.default_rng(9)
    u = rng.standard_normal(A.shape[0])
    v = rng.standard_normal(A.shape[0])
    Bu = _dev(np.zeros_like(u))
    h.cycle(_dev(u), Bu)
    Btv = _dev(np.zeros_like(v))
    h.cycle_transpose(_dev(v), Btv)
    lhs = Bu.cpu().numpy() @ v
    rhs = u @ Btv.cpu().numpy()
    _say("  <Bu,v> =", lhs, " <u,B^T v> =", rhs)
    assert abs(lhs - rhs) <= 1e-12 * np.linalg.norm(Bu.cpu().numpy()) * np.linalg.norm(v)


def test_transpose_solve_matches_dense_and_oracle(lair):
    _, _, A = _c4()
    h = lair.setup(A.indptr, A.indices, A.data, interp="direct")
    g = np.random.default_rng(3).standard_normal(A.shape[0])
    lam, info = h.solve_transpose(_dev(g), rtol=1e-12)
    assert info["converged"]
    ref = np.linalg.solve(A.toarray().T, g)
    lam = lam.cpu().numpy()
    assert np.linalg.norm(lam - ref) <= 1e-9 * np.linalg.norm(ref)
    H = O.setup(A, interp=O.INTERP_DIRECT)
    lo, ito, _ = O.solve_transpose(H, g, rtol=1e-12)
    _say("  transposed iterations gpu", info["iters"], "oracle", ito)
    assert info["iters"] == ito


def _loss_np(A, b, x_obs):
    x = spla.splu(A.tocsc()).solve(b)
    return float(((x - x_obs) ** 2).sum())


def test_gradients_wrt_b_and_c(lair):
    import torch
    from paper_1708_06065_amd.autograd import LairSolve
    w, A0, A = _c4()
    n = A.shape[0]
    x_obs = w["x_obs"]
    b = np.ones(n)
    dev = "cuda"
    rp = torch.as_tensor(A0.indptr.astype(np.int32), device=dev)
    cj = torch.as_tensor(A0.indices.astype(np.int32), device=dev)
    v0 = torch.as_tensor(A0.data, device=dev)
    bt = torch.tensor(b, device=dev, requires_grad=True)
    ct = torch.tensor(w["c"], device=dev, requires_grad=True)
    xo = torch.as_tensor(x_obs, device=dev)
    x = LairSolve.apply(bt, ct, rp, cj, v0, {"interp": "direct", "rtol": 1e-12})
    J = ((x - xo) ** 2).sum()
    J.backward()
    gb = bt.grad.cpu().numpy()
    gc = ct.grad.cpu().numpy()
    # dense adjoint reference
    D = A.toarray()
    xs = np.linalg.solve(D, b)
    lam = np.linalg.solve(D.T, 2.0 * (xs - x_obs))
    assert abs(J.item() - ((xs - x_obs) ** 2).sum()) <= 1e-10 * J.item()
    assert np.linalg.norm(gb - lam) <= 1e-8 * np.linalg.norm(lam)
    assert np.linalg.norm(gc + lam * xs) <= 1e-8 * np.linalg.norm(lam * xs)
    # central finite differences, h = 1e-6, on 16 random directions each.
    # Their own error (truncation + rounding of J over 2h) is measured with
    # the exact dense gradient; the GPU gradient must be as close to the
    # differences as the exact gradient is (plus 1e-8), and within 1e-5.
    rng = np.random.default_rng(4)
    hfd = 1e-6
    worst, worst_ref = 0.0, 0.0
    for k in range(16):
        d = rng.standard_normal(n)
        fd_b = (_loss_np(A, b + hfd * d, x_obs) - _loss_np(A, b - hfd * d, x_obs)) / (2 * hfd)
        Ap = (A + sp.diags(hfd * d)).tocsr()
        Am = (A - sp.diags(hfd * d)).tocsr()
        fd_c = (_loss_np(Ap, b, x_obs) - _loss_np(Am, b, x_obs)) / (2 * hfd)
        for g_gpu, g_ref, fd in ((gb, lam, fd_b), (gc, -lam * xs, fd_c)):
            e = abs(g_gpu @ d - fd) / abs(fd)
            e_ref = abs(g_ref @ d - fd) / abs(fd)
            assert e <= e_ref + 1e-8, (k, e, e_ref)
            worst, worst_ref = max(worst, e), max(worst_ref, e_ref)
    _say("  worst relative error vs central differences: gpu %.2e, exact gradient %.2e"
         % (worst, worst_ref))
    assert worst <= 1e-5


def test_gradients_with_reused_hierarchy(lair):
    """Two reaction fields in a row through one kept hierarchy (the second
    call only replaces the diagonal): gradients equal the dense adjoint's."""
    import torch
    from paper_1708_06065_amd.autograd import LairSolve
    w, A0, _ = _c4(48)
    n = A0.shape[0]
    dev = "cuda"
    rp = torch.as_tensor(A0.indptr.astype(np.int32), device=dev)
    cj = torch.as_tensor(A0.indices.astype(np.int32), device=dev)
    v0 = torch.as_tensor(A0.data, device=dev)
    xo = torch.as_tensor(w["x_obs"], device=dev)
    reuse = {}
    for scale in (1.0, 1.7):
        c = w["c"] * scale
        bt = torch.ones(n, dtype=torch.float64, device=dev, requires_grad=True)
        ct = torch.tensor(c, device=dev, requires_grad=True)
        x = LairSolve.apply(bt, ct, rp, cj, v0, {"interp": "direct", "rtol": 1e-12,
                                                 "reuse": reuse})
        ((x - xo) ** 2).sum().backward()
        D = (A0 + sp.diags(c)).toarray()
        xs = np.linalg.solve(D, np.ones(n))
        lam = np.linalg.solve(D.T, 2.0 * (xs - w["x_obs"]))
        assert np.linalg.norm(bt.grad.cpu().numpy() - lam) <= 1e-8 * np.linalg.norm(lam)
        assert np.linalg.norm(ct.grad.cpu().numpy() + lam * xs) <= 1e-8 * np.linalg.norm(lam * xs)
    reuse["h"].free()


def test_reused_hierarchy_two_forwards_before_backward(lair):
    """forward(c1), forward(c2), backward(c1), backward(c2) on one kept
    hierarchy: each backward uses its own forward's A(c)^T."""
    import torch
    from paper_1708_06065_amd.autograd import LairSolve
    w, A0, _ = _c4(40)
    n = A0.shape[0]
    dev = "cuda"
    rp = torch.as_tensor(A0.indptr.astype(np.int32), device=dev)
    cj = torch.as_tensor(A0.indices.astype(np.int32), device=dev)
    v0 = torch.as_tensor(A0.data, device=dev)
    xo = torch.as_tensor(w["x_obs"], device=dev)
    reuse = {}
    runs = []
    for scale in (1.0, 2.5):
        c = w["c"] * scale
        bt = torch.ones(n, dtype=torch.float64, device=dev, requires_grad=True)
        ct = torch.tensor(c, device=dev, requires_grad=True)
        x = LairSolve.apply(bt, ct, rp, cj, v0, {"interp": "direct", "rtol": 1e-12,
                                                 "reuse": reuse})
        runs.append((c, bt, ct, ((x - xo) ** 2).sum()))
    for c, bt, ct, J in runs:
        J.backward()
        D = (A0 + sp.diags(c)).toarray()
        xs = np.linalg.solve(D, np.ones(n))
        lam = np.linalg.solve(D.T, 2.0 * (xs - w["x_obs"]))
        assert np.linalg.norm(bt.grad.cpu().numpy() - lam) <= 1e-8 * np.linalg.norm(lam)
        assert np.linalg.norm(ct.grad.cpu().numpy() + lam * xs) <= 1e-8 * np.linalg.norm(lam * xs)
    reuse["h"].free()


# ------------------------------------------------------------------ mixed

@pytest.mark.parametrize("case", ["euler3d", "dg"])
def test_mixed_local_solves_within_refinement_bound(lair, case):
    if case == "euler3d":
        w = W.implicit_euler_adr_3d(m=24, nrhs=1)
        A = O.csr(w["rowptr"], w["col"], w["val"])
        kw = dict(interp="direct")
        okw = dict(interp=O.INTERP_DIRECT)
        b = w["rhs"]
        block = 0
    else:
        w = W.upwind_dg_p2(12)
        A, b = O.block_scale(O.csr(w["rowptr"], w["col"], w["val"]), w["rhs"], 6)
        kw = dict(distance=2)
        okw = dict(distance=2)
        block = 6
    H = O.setup(A, **okw)
    cfl = oracle_cf_levels(H)
    src = (w["rowptr"], w["col"], w["val"]) if block else (A.indptr, A.indices, A.data)
    h = lair.setup(*src, cf_levels=cfl, precision="mixed", block_size=block, **kw)
    worst_ratio = 0.0
    for l in range(h.nlevels - 1):
        Al = gpu_A(h, l)
        sm = O.strength(Al, 0.25)
        cpts, nptr, nbr = O.neighbourhoods(Al, sm, cfl[l], kw.get("distance", 1))
        z, _ = O.local_solves(Al, cpts, nptr, nbr)
        R = O.restriction(Al.shape[0], cpts, nptr, nbr, z)
        rv = h.export(l, "R.val")
        assert np.array_equal(h.export(l, "R.col"), R.indices)
        D = Al.tocsr()
        rng = np.random.default_rng(l)
        for c in rng.choice(cpts.shape[0], size=min(300, cpts.shape[0]), replace=False):
            nb = nbr[nptr[c]:nptr[c + 1]]
            if nb.shape[0] == 0:
                continue
            M = D[nb][:, nb].toarray().T
            kappa = np.linalg.cond(M)
            lo, hi = R.indptr[c], R.indptr[c + 1]
            err = np.abs(rv[lo:hi] - R.data[lo:hi]).max() / np.abs(R.data[lo:hi]).max()
            bound = 10.0 * ((kappa * U32) ** 2 + kappa * U64) + 1e-15
            worst_ratio = max(worst_ratio, err / bound)
            assert err <= bound, (l, c, err, kappa)
    _say("  worst error / refinement bound:", worst_ratio)


def test_mixed_local_precision_solve(lair):
    """Float local solves with one double refinement, double cycle: the same
    cycle count as FP64 (at most one more) and the FP64 residual."""
    w = W.implicit_euler_adr_3d(m=24, nrhs=4)
    h64 = lair.setup(w["rowptr"], w["col"], w["val"], interp="direct")
    hml = lair.setup(w["rowptr"], w["col"], w["val"], interp="direct", precision="mixed_local")
    B = _dev(w["rhs"])
    x64, i64 = h64.solve(B, rtol=1e-10)
    xml, iml = hml.solve(B, rtol=1e-10)
    _say("  iterations fp64", i64["iters"], "mixed_local", iml["iters"])
    assert iml["converged"] and iml["iters"] <= i64["iters"] + 1
    A = O.csr(w["rowptr"], w["col"], w["val"])
    X = xml.cpu().numpy()
    for q in range(4):
        r = w["rhs"][:, q] - A @ X[:, q]
        assert np.linalg.norm(r) <= 1e-10 * np.linalg.norm(w["rhs"][:, q])


def test_mixed_solve_reaches_fp64_tolerance(lair):
    w = W.implicit_euler_adr_3d(m=32, nrhs=16)
    h64 = lair.setup(w["rowptr"], w["col"], w["val"], interp="direct")
    hmx = lair.setup(w["rowptr"], w["col"], w["val"], interp="direct", precision="mixed")
    B = _dev(w["rhs"])
    x64, i64 = h64.solve(B, rtol=1e-10)
    xmx, imx = hmx.solve(B, rtol=1e-10)
    _say("  iterations fp64", i64["iters"], "mixed", imx["iters"], "relres", imx["relres"])
    assert i64["converged"] and imx["converged"]
    assert imx["iters"] <= i64["iters"] + 1
    A = O.csr(w["rowptr"], w["col"], w["val"])
    X = xmx.cpu().numpy()
    for q in range(16):
        r = w["rhs"][:, q] - A @ X[:, q]
        assert np.linalg.norm(r) <= 1e-10 * np.linalg.norm(w["rhs"][:, q])
    err = np.abs(X - x64.cpu().numpy()).max() / np.abs(x64.cpu().numpy()).max()
    _say("  max relative difference mixed vs fp64 solution:", err)
    assert err <= 1e-8
