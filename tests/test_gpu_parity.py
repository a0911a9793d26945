"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Bit-exact: strength masks, CF splittings, neighbourhoods, the patterns of R,
P and every coarse operator, fallback flags.  Floating point: each row of Z
within 1e-12 of the row's largest |z|; K entries within 1e-12 of the scale of
the terms summed (|R||A||P|); equal V-cycle counts to 1e-10.
"""
import sys

import numpy as np
import pytest
import scipy.sparse as sp

import workloads as W
from oracle import lair as O
from tests.parity import compare_level, gpu_A, oracle_cf_levels

pytestmark = pytest.mark.gpu


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


def _solve_both(lair, h, H, b, rtol=1e-10, maxit=200):
    x, info = h.solve(_dev(b), rtol=rtol, maxit=maxit)
    xo, ito, hist = O.solve(H, b, rtol=rtol, maxit=maxit)
    return x.cpu().numpy(), info, xo, ito, hist


# ------------------------------------------------------------------- C1

def test_c1_levelwise_and_iterations(lair):
    _say("case: C1 64x64 steady transport, oracle CF passed in")
    w = W.workload_c1()
    A = O.csr(w["rowptr"], w["col"], w["val"])
    H = O.setup(A)
    cfl = oracle_cf_levels(H)
    h = lair.setup(w["rowptr"], w["col"], w["val"], cf_levels=cfl)
    assert h.nlevels == H.nlevels
    for l in range(h.nlevels - 1):
        e = compare_level(h, l, cf=cfl[l])
        _say("  level", l, e)
    # end-to-end: the GPU's coarse operators equal the oracle's own chain
    for l in range(1, h.nlevels):
        Kg = gpu_A(h, l)
        Ko = H.levels[l].A
        assert np.array_equal(Kg.indptr, Ko.indptr) and np.array_equal(Kg.indices, Ko.indices)
    x, info, xo, ito, hist = _solve_both(lair, h, H, w["rhs"])
    _say("  iters gpu", info["iters"], "oracle", ito, "relres", info["relres"])
    assert info["converged"]
    assert info["iters"] == ito
    assert np.abs(x - xo).max() <= 1e-9 * np.abs(xo).max()
    h.free()


def test_device_cf_levels_equal_host(lair):
    """Splittings handed over in device memory (checked and counted on the
    device) give the hierarchy the host arrays give; a bad value or a
    wrong length is refused."""
    import torch
    from paper_1708_06065_amd import LairError
    w = W.implicit_euler_adr_3d(m=24, nrhs=1)
    A = O.csr(w["rowptr"], w["col"], w["val"])
    H = O.setup(A, interp=O.INTERP_DIRECT, max_coarse=16)
    cfl = oracle_cf_levels(H)
    hh = lair.setup(w["rowptr"], w["col"], w["val"], cf_levels=cfl, interp="direct",
                    max_coarse=16)
    dcf = [torch.as_tensor(c, device="cuda") for c in cfl]
    hd = lair.setup(w["rowptr"], w["col"], w["val"], cf_levels=dcf, interp="direct",
                    max_coarse=16)
    assert hh.nlevels == hd.nlevels == H.nlevels
    for l in range(hh.nlevels):
        for what in ("A.rowptr", "A.col", "A.val"):
            assert np.array_equal(hh.export(l, what), hd.export(l, what)), (l, what)
    bad = [c.clone() for c in dcf]
    bad[1][3] = 2
    with pytest.raises(LairError) as e:
        lair.setup(w["rowptr"], w["col"], w["val"], cf_levels=bad, interp="direct",
                   max_coarse=16)
    assert e.value.status == -1
    short = [dcf[0], dcf[1][:-1]]
    with pytest.raises(LairError):
        lair.setup(w["rowptr"], w["col"], w["val"], cf_levels=short, interp="direct",
                   max_coarse=16)
    hh.free()
    hd.free()


def test_c1_library_rs_split(lair):
    """No CF given: the library's own first-pass splitting equals the oracle's."""
    w = W.workload_c1()
    h = lair.setup(w["rowptr"], w["col"], w["val"])
    for l in range(h.nlevels - 1):
        compare_level(h, l)
    H = O.setup(O.csr(w["rowptr"], w["col"], w["val"]))
    assert h.nlevels == H.nlevels


@pytest.mark.parametrize("m", [5, 17, 33])
def test_chain_and_small_grids_ragged(lair, m):
    """Ragged sizes, tiny coarsest grids, chain closed form (one cycle)."""
    w = W.chain_1d(m * 7 + 3)
    h = lair.setup(w["rowptr"], w["col"], w["val"], max_coarse=2)
    for l in range(h.nlevels - 1):
        compare_level(h, l)
    b = np.random.default_rng(m).standard_normal(w["n"])
    x = _dev(np.zeros(w["n"]))
    h.cycle(_dev(b), x)
    A = O.csr(w["rowptr"], w["col"], w["val"])
    r = b - A @ x.cpu().numpy()
    assert np.abs(r).max() <= 1e-12 * np.abs(b).max() * w["n"]


# ------------------------------------------------------------------- distance 2, DG

@pytest.mark.parametrize("m", [6, 16])
def test_dg_block_scaled_distance2(lair, m):
    _say("case: DG P2 %dx%dx2, block scaling, distance 2" % (m, m))
    w = W.upwind_dg_p2(m)
    A = O.csr(w["rowptr"], w["col"], w["val"])
    As, bs = O.block_scale(A, w["rhs"], 6)
    H = O.setup(As, distance=2, max_coarse=20)
    cfl = oracle_cf_levels(H)
    h = lair.setup(w["rowptr"], w["col"], w["val"], cf_levels=cfl, distance=2,
                   block_size=6, max_coarse=20)
    # scaled operator: pattern bit-exact, values to rounding
    Ag = gpu_A(h, 0)
    assert np.array_equal(Ag.indptr, As.indptr) and np.array_equal(Ag.indices, As.indices)
    assert np.abs(Ag.data - As.data).max() <= 1e-12 * np.abs(As.data).max()
    for l in range(h.nlevels - 1):
        e = compare_level(h, l, distance=2, cf=cfl[l])
        _say("  level", l, e)
    # a few cycles: residual histories agree (the stationary iteration does
    # not converge on this ill-posed recirculating problem)
    x, info = h.solve(_dev(w["rhs"]), rtol=1e-10, maxit=5)
    xo, ito, hist = O.solve(H, bs, maxit=5)
    assert info["iters"] == ito == 5
    assert abs(info["relres"] - hist[-1] / hist[0]) <= 1e-6 * hist[-1] / hist[0]


# ------------------------------------------------------------------- direct P, ADR

@pytest.mark.parametrize("case", ["c4", "euler3d", "adr_diffusive"])
def test_direct_interp_levelwise_and_iterations(lair, case):
    _say("case: direct interpolation", case)
    if case == "c4":
        w = W.workload_c4(40)
        A = (O.csr(w["rowptr"], w["col"], w["val"]) + sp.diags(w["c"])).tocsr()
        A.sort_indices()
        b = w["rhs"]
    elif case == "euler3d":
        w = W.implicit_euler_adr_3d(m=18, nrhs=1)
        A = O.csr(w["rowptr"], w["col"], w["val"])
        b = w["rhs"]
    else:
        w = W.adr_2d(45, 1.0, 1.0, 0.0)
        A = O.csr(w["rowptr"], w["col"], w["val"])
        b = np.random.default_rng(1).standard_normal(A.shape[0])
    H = O.setup(A, interp=O.INTERP_DIRECT)
    cfl = oracle_cf_levels(H)
    h = lair.setup(A.indptr, A.indices, A.data, cf_levels=cfl, interp="direct")
    assert h.nlevels == H.nlevels
    for l in range(h.nlevels - 1):
        e = compare_level(h, l, interp=O.INTERP_DIRECT, cf=cfl[l])
        _say("  level", l, e)
    x, info, xo, ito, hist = _solve_both(lair, h, H, b)
    _say("  iters gpu", info["iters"], "oracle", ito)
    assert info["converged"] and info["iters"] == ito
    assert np.linalg.norm(x - xo) <= 1e-8 * np.linalg.norm(xo)


@pytest.mark.parametrize("m", [128, 129])
def test_scan_size_boundary_levelwise(lair, m):
    """n = 16,384 and 16,641 on level 0: the setup's prefix sums over n take
    the one-launch path and the tiled path; every level against the oracle
    and the same iteration count (direct P, a diffusive case with levels of
    all sizes below)."""
    _say("case: scan size boundary, m =", m)
    w = W.adr_2d(m, 1.0, 0.7, 0.0)
    A = O.csr(w["rowptr"], w["col"], w["val"])
    b = np.random.default_rng(2).standard_normal(A.shape[0])
    H = O.setup(A, interp=O.INTERP_DIRECT)
    cfl = oracle_cf_levels(H)
    h = lair.setup(A.indptr, A.indices, A.data, cf_levels=cfl, interp="direct")
    assert h.nlevels == H.nlevels
    for l in range(h.nlevels - 1):
        compare_level(h, l, interp=O.INTERP_DIRECT, cf=cfl[l])
    x, info, xo, ito, hist = _solve_both(lair, h, H, b)
    assert info["converged"] and info["iters"] == ito
    assert np.linalg.norm(x - xo) <= 1e-8 * np.linalg.norm(xo)
    h.free()


def test_large_levels_levelwise(lair):
    """64^3 implicit Euler step (262,144 rows): levels 1 and 2 have 65,536
    rows or more, so their products size the hash tables from the level
    above and redo the rows that overflow, and levels 0 to 2 run the cycle
    renumbered.  Every level against the oracle, same iteration count."""
    _say("case: 64^3 levelwise")
    w = W.implicit_euler_adr_3d(m=64, nrhs=1)
    A = O.csr(w["rowptr"], w["col"], w["val"])
    H = O.setup(A, interp=O.INTERP_DIRECT)
    cfl = oracle_cf_levels(H)
    h = lair.setup(A.indptr, A.indices, A.data, cf_levels=cfl, interp="direct")
    assert h.nlevels == H.nlevels
    for l in range(h.nlevels - 1):
        compare_level(h, l, interp=O.INTERP_DIRECT, cf=cfl[l])
    x, info, xo, ito, hist = _solve_both(lair, h, H, w["rhs"])
    _say("  iters gpu", info["iters"], "oracle", ito)
    assert info["converged"] and info["iters"] == ito
    assert np.linalg.norm(x - xo) <= 1e-8 * np.linalg.norm(xo)
    h.free()


def test_multi_rhs_equals_single(lair):
    import torch
    w = W.implicit_euler_adr_3d(m=14, nrhs=16)
    h = lair.setup(w["rowptr"], w["col"], w["val"], interp="direct")
    B = _dev(w["rhs"])
    X, info = h.solve(B, rtol=1e-10)
    assert info["converged"]
    A = O.csr(w["rowptr"], w["col"], w["val"])
    Xh = X.cpu().numpy()
    for q in (0, 7, 15):
        x1, i1 = h.solve(_dev(w["rhs"][:, q]), rtol=1e-10)
        assert np.abs(x1.cpu().numpy() - Xh[:, q]).max() <= 1e-9 * np.abs(Xh[:, q]).max()
        r = w["rhs"][:, q] - A @ Xh[:, q]
        assert np.linalg.norm(r) <= 1e-10 * np.linalg.norm(w["rhs"][:, q])
    # right-hand sides and solution at an 8-byte offset (not 16-byte aligned):
    # the library takes its scalar-lane kernels; same iteration, same answer
    n = w["n"]
    flat_b = torch.zeros(n * 16 + 1, dtype=torch.float64, device="cuda")
    flat_x = torch.zeros(n * 16 + 1, dtype=torch.float64, device="cuda")
    Bu = flat_b[1:].view(n, 16)
    Xu = flat_x[1:].view(n, 16)
    Bu.copy_(B)
    assert Bu.data_ptr() % 16 == 8
    _, iu = h.solve(Bu, Xu, rtol=1e-10)
    assert iu["iters"] == info["iters"]
    assert np.abs(Xu.cpu().numpy() - Xh).max() <= 1e-12 * np.abs(Xh).max()


# ------------------------------------------------------------------- special cases

@pytest.mark.parametrize("n", [90, 300])
def test_all_f_neighbourhood_is_ideal(lair, n):
    # n = 300 puts ~3000 products in a row of R (A P): the product's widest
    # staging kernel and its row-merge fallback both run
    w = W.random_ff_digraph(n, 4, 17)
    A = O.csr(w["rowptr"], w["col"], w["val"])
    h = lair.setup(w["rowptr"], w["col"], w["val"], distance="all_f", max_coarse=8,
                   max_levels=2)
    e = compare_level(h, 0, distance=O.DIST_ALL_F, ztol=1e-11)
    D = A.toarray()
    cf = h.export(0, "cf")
    F = np.flatnonzero(cf == 0)
    C = np.flatnonzero(cf == 1)
    Zi = -D[np.ix_(C, F)] @ np.linalg.inv(D[np.ix_(F, F)])
    rrp, rcj, rv = (h.export(0, k) for k in ("R.rowptr", "R.col", "R.val"))
    Rg = sp.csr_matrix((rv, rcj, rrp), shape=(C.shape[0], n)).toarray()
    assert np.abs(Rg[:, F] - Zi).max() <= 1e-11 * np.abs(Zi).max()


def test_singular_local_system_uses_least_squares(lair):
    """C-point 0 with N = {1, 2} has a singular local matrix (Sec. 3.1
    footnote): the GPU's SVD-based minimal-norm solution equals pinv."""
    rp = np.array([0, 3, 5, 8, 9], dtype=np.int32)
    cj = np.array([0, 1, 2, 1, 3, 1, 2, 3, 3], dtype=np.int32)
    v = np.array([4.0, -1.0, -1.0, 1.0, -1.0, 1.0, 1e-300, -1.0, 2.0])
    # a_22 must be a nonzero diagonal for the CSR checks; 1e-300 keeps the
    # local matrix singular to working precision
    cf = np.array([1, 0, 0, 1], dtype=np.int8)
    h = lair.setup(rp, cj, v, cf_levels=[cf], max_coarse=1, max_levels=2,
                   theta=0.0)
    flags = h.export(0, "flags")
    A = O.csr(rp, cj, v)
    sm = O.strength(A, 0.0)
    cpts, nptr, nbr = O.neighbourhoods(A, sm, cf, 1)
    z, fo = O.local_solves(A, cpts, nptr, nbr)
    assert flags.tolist() == fo.tolist()
    rv = h.export(0, "R.val")
    R = O.restriction(4, cpts, nptr, nbr, z)
    assert np.allclose(rv, R.data, rtol=1e-12, atol=1e-14)


# ------------------------------------------------------------------- errors

def test_error_paths(lair):
    from paper_1708_06065_amd import LairError
    w = W.workload_c1(8)
    bad = w["col"].copy()
    bad[[1, 2]] = bad[[2, 1]]
    with pytest.raises(LairError) as e:
        lair.setup(w["rowptr"], bad, w["val"])
    assert e.value.status == -1
    v = w["val"].copy()
    v[5] = np.nan
    with pytest.raises(LairError):
        lair.setup(w["rowptr"], w["col"], v)
    with pytest.raises(LairError):
        lair.setup(w["rowptr"], w["col"], w["val"], cf_levels=[np.zeros(3, np.int8)],
                   max_coarse=4)
    with pytest.raises(LairError):
        lair.setup(w["rowptr"], w["col"], w["val"], cf_levels=[np.full(64, 2, np.int8)],
                   max_coarse=4)
    h = lair.setup(w["rowptr"], w["col"], w["val"], max_coarse=4)
    x, info = h.solve(_dev(w["rhs"]), maxit=1, rtol=1e-30)
    assert not info["converged"] and info["iters"] == 1


@pytest.mark.parametrize("lump_tol", [0.0, 1e-3])
def test_given_splitting_equals_computed_splitting(lair, lump_tol):
    """With the splitting given per level, the strength pass also takes the
    counting pass of direct interpolation (one read of each row instead of
    two); with the splitting computed by the library's first pass the two
    passes stay apart.  Handing the second setup the first one's splittings
    must rebuild the same hierarchy bit for bit: masks, P, R, the coarse
    operators and the solution.  48^3, 4 right-hand sides, direct
    interpolation, mixed precision."""
    _say("case: given vs computed splitting, lump", lump_tol)
    w = W.implicit_euler_adr_3d(m=48, nrhs=4)
    kw = dict(interp="direct", precision="mixed", lump_tol=lump_tol)
    hc = lair.setup(w["rowptr"], w["col"], w["val"], **kw)
    cfs = [hc.export(l, "cf") for l in range(hc.nlevels - 1)]
    hg = lair.setup(w["rowptr"], w["col"], w["val"], cf_levels=cfs, **kw)
    assert hc.nlevels == hg.nlevels
    for l in range(hc.nlevels - 1):
        for what in ("smask", "cf", "P.rowptr", "P.col", "P.val", "R.rowptr", "R.col", "R.val",
                     "A.rowptr", "A.col", "A.val"):
            assert np.array_equal(hc.export(l, what), hg.export(l, what)), (l, what)
    b = _dev(w["rhs"])
    xc, ic = hc.solve(b, rtol=1e-10)
    xg, ig = hg.solve(b, rtol=1e-10)
    _say("  levels", hc.nlevels, "iterations", ic["iters"], ig["iters"])
    assert ic["converged"] and ic["iters"] == ig["iters"]
    assert np.array_equal(xc.cpu().numpy(), xg.cpu().numpy())
    hc.free()
    hg.free()
