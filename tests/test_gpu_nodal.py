"""GPU: nodal (block) lAIR (LAIR_FLAG_NODAL, Sec. 3.1 block form of
Eq. (system), Sec. 4.2 treatment (iii)) against the oracle's nodal setup.

Level by level on the GPU's own A_l: strength masks, node splittings,
neighbourhoods, fallback flags and the R, P and K patterns bit-exact; each
row of Z within 1e-12 of its largest entry; K within 1e-12 of the scale of
the terms summed; the same number of cycles to 1e-10 and the solution
within 1e-8.  Cases: a Kronecker product ADR (x) B (k = 3), a perturbed
dense-block matrix (k = 2), P2 upwind DG along a curved field (k = 6), the
DGu problem of Sec. 4.2 (gamma jump, interior-penalty diffusion kappa in
{0, 1e-3, 1}; k = 6; on 24 x 24 x 2 triangles its systems pass 72 rows),
and a random sparse graph (x) 3 x 3 blocks whose distance-2 systems pass
128 rows.
"""
import sys

import numpy as np
import pytest
import scipy.sparse as sp

import workloads as W
from oracle import lair as O
from tests.parity import gpu_A, gpu_level_csr, rows_rel_err

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


def _adr(m):
    w = W.workload_c4(m)
    A = (O.csr(w["rowptr"], w["col"], w["val"]) + sp.diags(w["c"])).tocsr()
    A.sort_indices()
    return A, w["rhs"]


def _case(name):
    if name == "kron3":
        As, bs = _adr(20)
        B = np.random.default_rng(0).standard_normal((3, 3)) + 3.0 * np.eye(3)
        A = sp.kron(As, sp.csr_matrix(B)).tocsr()
        A.sort_indices()
        return A, np.kron(bs, [1.0, -2.0, 0.5]), 3
    if name == "perturbed2":
        As, bs = _adr(24)
        rng = np.random.default_rng(1)
        B = rng.standard_normal((2, 2)) + 3.0 * np.eye(2)
        A = sp.kron(As, sp.csr_matrix(B)).tocsr()
        A.sort_indices()
        A.data = A.data * (1.0 + 0.3 * rng.standard_normal(A.nnz))
        return A, np.kron(bs, [1.0, 1.0]), 2
    if name == "rand8k3":
        # a random sparse graph (8 couplings per row) (x) 3 x 3 blocks: at
        # distance 2 the first level's systems reach 141 rows
        As = W.random_ff_digraph(300, 8, seed=1)
        As = O.csr(As["rowptr"], As["col"], As["val"])
        B = np.random.default_rng(0).standard_normal((3, 3)) + 3.0 * np.eye(3)
        A = sp.kron(As, sp.csr_matrix(B)).tocsr()
        A.sort_indices()
        return A, np.kron(np.ones(300), [1.0, -1.0, 0.5]), 3
    if name == "dgu24":
        # 24 x 24 x 2 triangles, kappa 1e-3: at distance 2 level 1 holds
        # systems of up to 78 rows, past the register form's 72
        w = W.workload_dgu(24, 1e-3)
        return O.csr(w["rowptr"], w["col"], w["val"]), w["rhs"], 6
    if name.startswith("dgu"):
        # the DGu problem of Sec. 4.2 (gamma jump, curved field) with
        # diffusion kappa = the number after "dgu"
        w = W.workload_dgu(16, float(name[3:]))
        return O.csr(w["rowptr"], w["col"], w["val"]), w["rhs"], 6
    w = W.workload_dg_curved(16)
    return O.csr(w["rowptr"], w["col"], w["val"]), w["rhs"], 6


def compare_nodal_level(h, l, k, theta=0.25, cf=None, distance=1):
    A = gpu_A(h, l)
    n = A.shape[0]
    nrp, ncol, nsq = O.node_graph(A, k)
    nsm = O.node_strength(nrp, ncol, nsq, theta)
    assert np.array_equal(O.node_entry_mask(A, k, nrp, nsm), h.export(l, "smask")), \
        "strength mask differs at level %d" % l
    if cf is None:
        G = O.csr(nrp.astype(np.int32), ncol, np.ones(ncol.shape[0]), shape=(n // k,) * 2)
        cf_node = O.rs_split(G, nsm)
    else:
        cf_node = np.asarray(cf, dtype=np.int8)[::k]
    cf_o = O.expand_nodes(cf_node, k).astype(np.int8)
    assert np.array_equal(cf_o, h.export(l, "cf")), "CF splitting differs at level %d" % l
    cpts, nptr, nbr = O.node_neighbourhoods(nrp, ncol, nsm, cf_node, k, distance)
    assert np.array_equal(nptr.astype(np.int32), h.export(l, "nbr_ptr"))
    assert np.array_equal(nbr.astype(np.int32), h.export(l, "nbr"))
    z, flags = O.node_local_solves(A, k, cpts, nptr, nbr)
    assert np.array_equal(flags.astype(np.int8), h.export(l, "flags"))
    R = O.restriction(n, cpts, nptr, nbr, z)
    rrp, rcj, rv = gpu_level_csr(h, l, "R")
    assert np.array_equal(R.indptr.astype(np.int32), rrp)
    assert np.array_equal(R.indices.astype(np.int32), rcj)
    z_err = rows_rel_err(rrp, rv, R.data)
    assert z_err <= 1e-12, "R values differ by %g at level %d" % (z_err, l)
    P = O.node_interp_one_point(nrp, ncol, nsq, nsm, cf_node, k)
    prp, pcj, pv = gpu_level_csr(h, l, "P")
    assert np.array_equal(P.indptr.astype(np.int32), prp)
    assert np.array_equal(P.indices.astype(np.int32), pcj)
    assert np.array_equal(pv, P.data)
    K = O.galerkin(R, A, P)
    scale = O.galerkin(abs(R), abs(A), abs(P))
    Kg = gpu_A(h, l + 1)
    assert np.array_equal(K.indptr, Kg.indptr) and np.array_equal(K.indices, Kg.indices)
    assert np.all(np.abs(Kg.data - K.data) <= 1e-12 * scale.data + 1e-300)
    return z_err


@pytest.mark.parametrize("name", ["kron3", "perturbed2", "dg_curved", "dgu0", "dgu0.001",
                                  "dgu1"])
@pytest.mark.parametrize("own_split", [False, True])
def test_nodal_levels_and_iterations(lair, name, own_split):
    _say("case: nodal", name, "own split" if own_split else "oracle split")
    A, b, k = _case(name)
    H = O.setup(A, block=k)
    cfl = None if own_split else [L.cf for L in H.levels[:-1]]
    h = lair.setup(A.indptr, A.indices, A.data, cf_levels=cfl, block_size=k, nodal=True)
    assert h.nlevels == H.nlevels
    for l in range(h.nlevels - 1):
        compare_nodal_level(h, l, k, cf=None if cfl is None else cfl[l])
    x, info = h.solve(_dev(b), rtol=1e-10)
    xo, ito, _ = O.solve(H, b, rtol=1e-10)
    _say("  levels", h.nlevels, "iters", info["iters"], ito)
    assert info["converged"] and info["iters"] == ito
    assert np.linalg.norm(x.cpu().numpy() - xo) <= 1e-8 * np.linalg.norm(xo)
    h.free()


@pytest.mark.parametrize("name", ["perturbed2", "dg_curved", "dgu0", "dgu0.001", "dgu1",
                                  "dgu24", "rand8k3"])
def test_nodal_distance_two(lair, name):
    """F-F-C paths on the graph of blocks: the node-expanded strength mask
    makes the scalar distance-two merge give the nodal sets."""
    _say("case: nodal distance 2", name)
    A, b, k = _case(name)
    H = O.setup(A, block=k, distance=2)
    h = lair.setup(A.indptr, A.indices, A.data, block_size=k, nodal=True, distance=2)
    assert h.nlevels == H.nlevels
    for l in range(h.nlevels - 1):
        compare_nodal_level(h, l, k, distance=2)
    x, info = h.solve(_dev(b), rtol=1e-10)
    xo, ito, _ = O.solve(H, b, rtol=1e-10)
    _say("  levels", h.nlevels, "iters", info["iters"], ito, "s_max",
         max(h.level_stats(l)["s_max"] for l in range(h.nlevels - 1)))
    assert info["converged"] and info["iters"] == ito
    assert np.linalg.norm(x.cpu().numpy() - xo) <= 1e-8 * np.linalg.norm(xo)
    h.free()


def test_nodal_cycle_matches_oracle(lair):
    """Single cycles from a nonzero iterate, 4 right-hand sides at once."""
    A, b, k = _case("dg_curved")
    H = O.setup(A, block=k)
    h = lair.setup(A.indptr, A.indices, A.data, cf_levels=[L.cf for L in H.levels[:-1]],
                   block_size=k, nodal=True)
    rng = np.random.default_rng(5)
    n = A.shape[0]
    B = rng.standard_normal((n, 4))
    X0 = rng.standard_normal((n, 4))
    X = _dev(X0)
    h.cycle(_dev(B), X)
    X = X.cpu().numpy()
    for q in range(4):
        xo = O.cycle(H, B[:, q], X0[:, q].copy())
        assert np.linalg.norm(X[:, q] - xo) <= 1e-11 * np.linalg.norm(xo)
    h.free()


@pytest.mark.parametrize("name", ["dg_curved", "dgu0.001"])
def test_nodal_mixed_and_fgmres(lair, name):
    _say("case: nodal mixed + fgmres", name)
    A, b, k = _case(name)
    H = O.setup(A, block=k)
    cfl = [L.cf for L in H.levels[:-1]]
    _, ito, _ = O.solve(H, b, rtol=1e-10)
    hm = lair.setup(A.indptr, A.indices, A.data, cf_levels=cfl, block_size=k, nodal=True,
                    precision="mixed")
    x, info = hm.solve(_dev(b), rtol=1e-10)
    _say("  mixed iters", info["iters"], "oracle", ito)
    assert info["converged"] and ito <= info["iters"] <= ito + 1
    assert np.linalg.norm(b - A @ x.cpu().numpy()) <= 1e-10 * np.linalg.norm(b) * (1 + 1e-6)
    hm.free()
    h = lair.setup(A.indptr, A.indices, A.data, cf_levels=cfl, block_size=k, nodal=True)
    xo, itg, _, _ = O.fgmres_cycle(H, b, rtol=1e-10, restart=20)
    x, info = h.solve_fgmres(_dev(b), rtol=1e-10, restart=20)
    _say("  fgmres steps", info["iters"], "oracle", itg)
    assert info["converged"] and info["iters"] == itg
    assert np.linalg.norm(x.cpu().numpy() - xo) <= 1e-8 * np.linalg.norm(xo)
    h.free()


def test_nodal_argument_errors(lair):
    A, b, k = _case("perturbed2")
    with pytest.raises(Exception):      # one-point interpolation only
        lair.setup(A.indptr, A.indices, A.data, block_size=k, nodal=True, interp="direct")
    with pytest.raises(Exception):      # no lumping
        lair.setup(A.indptr, A.indices, A.data, block_size=k, nodal=True, lump_tol=1e-3)
    Ad, _ = _adr(12)                     # scalar ADR: rows do not store whole 2 x 2 blocks
    with pytest.raises(Exception):
        lair.setup(Ad.indptr, Ad.indices, Ad.data, block_size=2, nodal=True)
    H = O.setup(A, block=k)
    cf = H.levels[0].cf.copy()
    cf[1] = 1 - cf[1]                    # splits node 0
    with pytest.raises(Exception):
        lair.setup(A.indptr, A.indices, A.data, cf_levels=[cf], block_size=k, nodal=True)
    h = lair.setup(A.indptr, A.indices, A.data, block_size=k, nodal=True)
    with pytest.raises(Exception):
        h.update_diag(A.diagonal())
    with pytest.raises(Exception):
        h.solve_transpose(_dev(b))
    h.free()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("name,distance", [("kron3", 1), ("dg_curved", 1), ("dg_curved", 2),
                                           ("perturbed2", 2), ("dgu0.001", 2), ("dgu24", 2),
                                           ("rand8k3", 2)])
def test_node_solves_equal_row_solves(lair, monkeypatch, name, distance, precision):
    """The nodal local systems of a C-node (one matrix A(N,N)^T, one
    right-hand side per row of the node; Sec. 3.1, block form of
    Eq. (system)) solved as one factorisation with k right-hand sides give
    the same R, bit for bit, as k separate solves of the scalar rows, with
    the node's matrix in registers or in LDS; the node path is the one that
    ran (its profiler category)."""
    _say("case: node solves", name, "distance", distance, precision)
    A, b, k = _case(name)
    Rs = {}
    # scalar rows; nodes with M in registers (systems up to 72 rows) and in
    # LDS above; nodes all in LDS
    for mode in ("rows", "nodes", "nodes_lds"):
        monkeypatch.delenv("LAIR_NODAL_ROW_SOLVES", raising=False)
        monkeypatch.delenv("LAIR_NODE_LDS_SOLVES", raising=False)
        if mode == "rows":
            monkeypatch.setenv("LAIR_NODAL_ROW_SOLVES", "1")
        if mode == "nodes_lds":
            monkeypatch.setenv("LAIR_NODE_LDS_SOLVES", "1")
        lair.profile_begin(["local_node", "local_small"])
        h = lair.setup(A.indptr, A.indices, A.data, block_size=k, nodal=True,
                       distance=distance, precision=precision)
        prof = lair.profile_end()
        Rs[mode] = [gpu_level_csr(h, l, "R") for l in range(h.nlevels - 1)]
        smax = max(h.level_stats(l)["s_max"] for l in range(h.nlevels - 1))
        _say("  " + mode, "levels", h.nlevels, "s_max", smax,
             {c: (round(v["ms"], 3), v["launches"]) for c, v in prof.items()})
        if name == "dgu24":
            assert smax > 72        # the LDS form takes the largest systems
        if name == "rand8k3":
            assert smax > 128       # past the searches' first power of two
        if mode == "rows":
            assert "local_node" not in prof
        else:
            assert prof.get("local_node", {}).get("launches", 0) > 0
        h.free()
    monkeypatch.delenv("LAIR_NODE_LDS_SOLVES", raising=False)
    for mode in ("nodes", "nodes_lds"):
        assert len(Rs["rows"]) == len(Rs[mode])
        for l, (a, c) in enumerate(zip(Rs["rows"], Rs[mode])):
            for u, w in zip(a, c):
                assert np.array_equal(u, w), "R differs at level %d (%s)" % (l, mode)
