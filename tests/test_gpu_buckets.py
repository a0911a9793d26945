"""GPU: the size buckets of the local solves change speed only.

Every bucket path (one lane, teams of 8/16/32 lanes, one wave) performs the
same floating-point operations in the same order, so R must come out bit for
bit the same whatever the bucket edges, in FP64 and in mixed precision, and
the tuned edges must equal one of the fixed choices' results.  The values
themselves are pinned to the oracle by the parity tests.
"""
import sys

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

EDGES = [(4, 8, 16, 32, 0), (0, 8, 16, 32, 0), (4, 8, 16, 32, 1), (2, 6, 12, 24, 1),
         (0, 0, 0, 0, 0), (4, 4, 4, 4, 1), (3, 5, 9, 17, 0)]


@pytest.fixture(scope="module")
def lair():
    import torch
    import paper_1708_06065_amd as lair
    assert torch.cuda.is_available()
    lair.load_library()
    yield lair
    lair.set_local_buckets(None)


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _problem(case):
    if case == "euler3d":
        w = W.implicit_euler_adr_3d(m=20, nrhs=1)
        return w, dict(interp="direct")
    if case == "dg_d2":
        w = W.upwind_dg_p2(8)
        return w, dict(distance=2, block_size=6, max_coarse=20)
    if case == "all_f":
        w = W.random_ff_digraph(120, 4, 17)
        return w, dict(distance="all_f", max_coarse=8, max_levels=2)
    if case == "singular":
        # C-point 0 with N = {1, 2} has a singular local matrix: the
        # least-squares path
        w = dict(rowptr=np.array([0, 3, 5, 8, 9], dtype=np.int32),
                 col=np.array([0, 1, 2, 1, 3, 1, 2, 3, 3], dtype=np.int32),
                 val=np.array([4.0, -1.0, -1.0, 1.0, -1.0, 1.0, 1e-300, -1.0, 2.0]))
        return w, dict(cf_levels=[np.array([1, 0, 0, 1], dtype=np.int8)], max_coarse=1,
                       max_levels=2, theta=0.0)
    w = W.workload_c1(40)
    return w, dict()


def _r_values(lair, w, kw):
    h = lair.setup(w["rowptr"], w["col"], w["val"], **kw)
    out = [(h.export(l, "R.col"), h.export(l, "R.val"), h.export(l, "flags"))
           for l in range(h.nlevels - 1)]
    used = [tuple(h.local_buckets(l)) for l in range(h.nlevels - 1)]
    h.free()
    return out, used


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("case", ["euler3d", "dg_d2", "all_f", "c1", "singular"])
def test_bucket_edges_do_not_change_r(lair, case, precision):
    _say("case: bucket edges,", case, precision)
    w, kw = _problem(case)
    kw = dict(kw, precision=precision)
    ref = None
    if case == "singular":
        lair.set_local_buckets(None)
        got, _ = _r_values(lair, w, kw)
        assert got[0][2].tolist() == [1, 0]
    try:
        for e in EDGES:
            lair.set_local_buckets(e)
            got, used = _r_values(lair, w, kw)
            assert all(u == e for u in used)
            if ref is None:
                ref = got
                continue
            for (c0, v0, f0), (c1, v1, f1) in zip(ref, got):
                assert np.array_equal(c0, c1)
                assert np.array_equal(f0, f1)
                assert np.array_equal(v0, v1), "edges %s" % (e,)
        lair.set_local_buckets(None)
        got, used = _r_values(lair, w, kw)
        _say("  tuned edges per level:", used)
        for (c0, v0, f0), (c1, v1, f1) in zip(ref, got):
            assert np.array_equal(v0, v1) and np.array_equal(f0, f1)
    finally:
        lair.set_local_buckets(None)


def test_bucket_edges_rejected(lair):
    from paper_1708_06065_amd import LairError
    for e in [(5, 8, 16, 32, 0), (4, 9, 16, 32, 0), (4, 8, 17, 32, 0), (4, 8, 16, 33, 0),
              (4, 2, 16, 32, 0), (4, 8, 16, 32, 2)]:
        with pytest.raises(LairError):
            lair.set_local_buckets(e)
    lair.set_local_buckets(None)
