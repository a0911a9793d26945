"""GPU: the parallel PMIS-type CF splitting on the device (split="pmis",
LAIR_FLAG_PMIS) against the oracle's pmis_split.

Level by level on the GPU's own A_l: the splitting bit-exact, and the rest
of the level (neighbourhoods, R, P, K) to the usual parity bar; the same
number of cycles to 1e-10 as the oracle's hierarchy on the same splitting
rule; a batch's splitting of every level equals the oracle's on the union.
"""
import sys

import numpy as np
import pytest
import scipy.sparse as sp

import workloads as W
from oracle import lair as O
from tests.parity import compare_level, gpu_A

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


def _case(name):
    if name == "c4":
        w = W.workload_c4(40)
        A = (O.csr(w["rowptr"], w["col"], w["val"]) + sp.diags(w["c"])).tocsr()
        A.sort_indices()
        return A, w["rhs"], O.INTERP_DIRECT, "direct"
    if name == "c1":
        w = W.workload_c1(48)
        return O.csr(w["rowptr"], w["col"], w["val"]), w["rhs"], O.INTERP_ONE_POINT, "one_point"
    w = W.implicit_euler_adr_3d(m=40, nrhs=1)
    return O.csr(w["rowptr"], w["col"], w["val"]), w["rhs"], O.INTERP_DIRECT, "direct"


@pytest.mark.parametrize("name", ["c4", "c1", "euler3d"])
def test_pmis_levels_and_iterations(lair, name):
    _say("case: pmis", name)
    A, b, oi, gi = _case(name)
    h = lair.setup(A.indptr, A.indices, A.data, interp=gi, split="pmis")
    for l in range(h.nlevels - 1):
        Al = gpu_A(h, l)
        cf = O.pmis_split(Al, O.strength(Al, 0.25))
        compare_level(h, l, interp=oi, cf=cf)
    H = O.setup(A, interp=oi, split="pmis")
    assert h.nlevels == H.nlevels
    x, info = h.solve(_dev(b), rtol=1e-10)
    xo, ito, _ = O.solve(H, b, rtol=1e-10)
    _say("  levels", h.nlevels, "iters", info["iters"], ito)
    assert info["converged"] and info["iters"] == ito
    assert np.linalg.norm(x.cpu().numpy() - xo) <= 1e-8 * np.linalg.norm(xo)
    h.free()


def test_pmis_batch_every_level(lair):
    """A batch split in parallel: on every level, each system still
    coarsening has the oracle's splitting of the GPU's union A_l on its rows
    (the weights' hash takes union indices, so the union is split as one
    matrix), and a system that has stopped has all its points as C-points."""
    systems = W.adr_batch(6, seed=11)
    mats = [(q["rowptr"], q["col"], q["val"]) for q in systems]
    hb = lair.setup_batch(mats, interp="direct", split="pmis", max_coarse=40)
    sys_levels = hb.system_levels()
    _say("  batch levels", hb.nlevels, "per system", list(sys_levels))
    assert hb.nlevels >= 3
    seg = np.concatenate([[0], np.cumsum([q["n"] for q in systems])]).astype(np.int64)
    for l in range(hb.nlevels - 1):
        Ul = gpu_A(hb, l)
        cf_o = O.pmis_split(Ul, O.strength(Ul, 0.25))
        cf_g = hb.export(l, "cf")
        for q in range(len(systems)):
            s0, s1 = seg[q], seg[q + 1]
            if l >= sys_levels[q] - 1:
                assert np.all(cf_g[s0:s1] == 1), (l, q)
            else:
                assert np.array_equal(cf_g[s0:s1], cf_o[s0:s1]), (l, q)
        c = np.concatenate([[0], np.cumsum(cf_g.astype(np.int64))])
        seg = c[seg]
    U = sp.block_diag([O.csr(*m) for m in mats]).tocsr()
    U.sort_indices()
    b = np.concatenate([q["rhs"] for q in systems])
    x, info = hb.solve_batch(_dev(b), rtol=1e-10)
    assert info["converged"]
    assert np.linalg.norm(b - U @ x.cpu().numpy()) <= 1e-9 * np.linalg.norm(b)
    hb.free()


def test_pmis_refused_with_nodal(lair):
    A, b, oi, gi = _case("c4")
    with pytest.raises(Exception):
        lair.setup(A.indptr, A.indices, A.data, block_size=1, nodal=True, split="pmis")
