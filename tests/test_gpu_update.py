"""GPU tests of lair_update_diag: a new diagonal on a kept hierarchy.

The GPU hierarchy (oracle splittings passed in) and the oracle's are both
updated with the same new diagonal; level by level the strength masks,
splittings and every pattern are unchanged and bit-exact, R rows agree to
1e-12 (row-relative), P to 1e-13 and K to 1e-12 of |R||A||P|; the V-cycle
counts to 1e-10 are equal.  A zero diagonal entry is rejected and leaves the
hierarchy as it was.
"""
import sys

import numpy as np
import pytest
import scipy.sparse as sp

import workloads as W
from oracle import lair as O
from tests.parity import gpu_A, gpu_level_csr, oracle_cf_levels, rows_rel_err

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


def _c4(m=40):
    w = W.workload_c4(m)
    A = (O.csr(w["rowptr"], w["col"], w["val"]) + sp.diags(w["c"])).tocsr()
    A.sort_indices()
    return w, A


def _compare(h, H):
    for l in range(h.nlevels - 1):
        L = H.levels[l]
        Ag = gpu_A(h, l)
        assert np.array_equal(Ag.indptr, L.A.indptr) and np.array_equal(Ag.indices, L.A.indices)
        assert np.array_equal(h.export(l, "cf"), L.cf)
        rrp, rcj, rv = gpu_level_csr(h, l, "R")
        assert np.array_equal(rrp, L.R.indptr) and np.array_equal(rcj, L.R.indices)
        assert rows_rel_err(rrp, rv, L.R.data) <= 1e-12, l
        prp, pcj, pv = gpu_level_csr(h, l, "P")
        assert np.array_equal(prp, L.P.indptr) and np.array_equal(pcj, L.P.indices)
        assert np.allclose(pv, L.P.data, rtol=1e-13, atol=1e-15)
        K = H.levels[l + 1].A
        Kg = gpu_A(h, l + 1)
        assert np.array_equal(Kg.indptr, K.indptr) and np.array_equal(Kg.indices, K.indices)
        scale = O.galerkin(abs(L.R), abs(L.A), abs(L.P)).data
        assert np.all(np.abs(Kg.data - K.data) <= 1e-12 * scale + 1e-300), l


@pytest.mark.parametrize("on_device", [True, False])
def test_update_diag_matches_oracle(lair, on_device):
    w, A = _c4()
    H = O.setup(A, interp=O.INTERP_DIRECT)
    cfl = oracle_cf_levels(H)
    h = lair.setup(A.indptr, A.indices, A.data, cf_levels=cfl, interp="direct")
    sm0 = [h.export(l, "smask") for l in range(h.nlevels - 1)]
    d = A.diagonal() * (1.0 + np.random.default_rng(5).random(A.shape[0]))
    h.update_diag(_dev(d) if on_device else d)
    O.update_diag(H, d)
    for l in range(h.nlevels - 1):
        assert np.array_equal(h.export(l, "smask"), sm0[l])
    _compare(h, H)
    b = w["rhs"]
    x, info = h.solve(_dev(b), rtol=1e-10)
    xo, ito, _ = O.solve(H, b, rtol=1e-10)
    print("  iterations after update: gpu", info["iters"], "oracle", ito, flush=True)
    sys.stdout.flush()
    assert info["converged"] and info["iters"] == ito
    assert np.linalg.norm(x.cpu().numpy() - xo) <= 1e-8 * np.linalg.norm(xo)


def test_update_diag_mixed_and_rejects_zero(lair):
    from paper_1708_06065_amd import LairError
    w, A = _c4(32)
    h = lair.setup(A.indptr, A.indices, A.data, interp="direct", precision="mixed")
    d = A.diagonal() * 1.5
    h.update_diag(d)
    A_new = A.tocsr(copy=True)
    A_new.setdiag(d)
    x, info = h.solve(_dev(w["rhs"]), rtol=1e-10)
    assert info["converged"]
    r = w["rhs"] - A_new @ x.cpu().numpy()
    assert np.linalg.norm(r) <= 1e-10 * np.linalg.norm(w["rhs"])
    bad = d.copy()
    bad[3] = 0.0
    with pytest.raises(LairError):
        h.update_diag(bad)
    x2, info2 = h.solve(_dev(w["rhs"]), rtol=1e-10)
    assert info2["iters"] == info["iters"]
