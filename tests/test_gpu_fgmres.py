"""GPU: flexible GMRES with the V-cycle as right preconditioner
(lair_solve_fgmres) against the oracle's fgmres_cycle.

FP64: the same number of Arnoldi steps to 1e-10 per right-hand side, the
solution within 1e-8 of the oracle's, the true residual below the
tolerance.  Mixed precision: at most one step more, the same residual bound.
The oracle's FGMRES is itself pinned to least squares over the Krylov space
(tests/test_oracle_pins.py).
"""
import sys

import numpy as np
import pytest
import scipy.sparse as sp

import workloads as W
from oracle import lair as O
from tests.parity import oracle_cf_levels

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


def _problem(case):
    if case == "c4":
        w = W.workload_c4(40)
        A = (O.csr(w["rowptr"], w["col"], w["val"]) + sp.diags(w["c"])).tocsr()
        A.sort_indices()
        return A, w["rhs"], "direct"
    if case == "c1":
        w = W.workload_c1(48)
        return O.csr(w["rowptr"], w["col"], w["val"]), w["rhs"], "one_point"
    w = W.implicit_euler_adr_3d(m=48, nrhs=1)      # 110,592 rows: level 0 renumbered
    return O.csr(w["rowptr"], w["col"], w["val"]), w["rhs"], "direct"


@pytest.mark.parametrize("case,restart", [("c4", 20), ("c4", 2), ("c1", 20), ("euler3d", 20)])
def test_fgmres_matches_oracle(lair, case, restart):
    _say("case: fgmres fp64", case, "restart", restart)
    A, b, interp = _problem(case)
    H = O.setup(A, interp=O.INTERP_DIRECT if interp == "direct" else O.INTERP_ONE_POINT)
    cfl = oracle_cf_levels(H)
    h = lair.setup(A.indptr, A.indices, A.data, cf_levels=cfl, interp=interp)
    xo, ito, _, _ = O.fgmres_cycle(H, b, rtol=1e-10, restart=restart)
    x, info = h.solve_fgmres(_dev(b), rtol=1e-10, restart=restart)
    x = x.cpu().numpy()
    _say("  steps gpu", info["iters"], "oracle", ito, "relres", info["relres"])
    assert info["converged"] and info["iters"] == ito
    assert np.linalg.norm(b - A @ x) <= 1e-10 * np.linalg.norm(b) * (1 + 1e-6)
    assert np.linalg.norm(x - xo) <= 1e-8 * np.linalg.norm(xo)
    h.free()


def test_fgmres_mixed_precision(lair):
    _say("case: fgmres mixed, 48^3")
    A, b, _ = _problem("euler3d")
    H = O.setup(A, interp=O.INTERP_DIRECT)
    cfl = oracle_cf_levels(H)
    h = lair.setup(A.indptr, A.indices, A.data, cf_levels=cfl, interp="direct",
                   precision="mixed")
    _, ito, _, _ = O.fgmres_cycle(H, b, rtol=1e-10)
    x, info = h.solve_fgmres(_dev(b), rtol=1e-10)
    x = x.cpu().numpy()
    _say("  steps gpu", info["iters"], "oracle", ito)
    assert info["converged"] and ito <= info["iters"] <= ito + 1
    assert np.linalg.norm(b - A @ x) <= 1e-10 * np.linalg.norm(b) * (1 + 1e-6)
    h.free()


def test_fgmres_columns_are_independent(lair):
    """Four right-hand sides at once (one of them zero, one a multiple of
    another) give each column what it gets alone, with its own step count."""
    import torch
    A, b, _ = _problem("c4")
    n = A.shape[0]
    rng = np.random.default_rng(7)
    B = np.stack([b, np.zeros(n), rng.standard_normal(n), 1e3 * b], axis=1)
    H = O.setup(A, interp=O.INTERP_DIRECT)
    h = lair.setup(A.indptr, A.indices, A.data, cf_levels=oracle_cf_levels(H),
                   interp="direct")
    X, info = h.solve_fgmres(_dev(B), rtol=1e-10, restart=5)
    X = X.cpu().numpy()
    steps = []
    for q in range(4):
        xq, iq = h.solve_fgmres(_dev(B[:, q]), rtol=1e-10, restart=5)
        xq = xq.cpu().numpy()
        steps.append(iq["iters"])
        assert np.linalg.norm(X[:, q] - xq) <= 1e-9 * max(np.linalg.norm(xq), 1e-300)
        assert np.linalg.norm(B[:, q] - A @ X[:, q]) <= 1e-10 * np.linalg.norm(B[:, q]) * (1 + 1e-6)
    assert steps[1] == 0 and np.all(X[:, 1] == 0.0)
    assert info["converged"] and info["iters"] == max(steps)
    h.free()


def test_fgmres_argument_errors(lair):
    from paper_1708_06065_amd import _lib as L
    A, b, _ = _problem("c4")
    h = lair.setup(A.indptr, A.indices, A.data, interp="direct")
    for r in (0, 65):
        with pytest.raises(Exception):
            h.solve_fgmres(_dev(b), restart=r)
    assert b"restart" in L.load().lair_last_error()
    # maxit reached first: ENOCONV reported, the iterate returned
    x, info = h.solve_fgmres(_dev(b), rtol=1e-14, maxit=2, restart=20)
    assert not info["converged"] and info["iters"] == 2
    h.free()
    hb = lair.setup_batch([(A.indptr, A.indices, A.data)] * 2, interp="direct")
    with pytest.raises(Exception):
        hb.solve_fgmres(_dev(np.concatenate([b, b])))
    hb.free()
