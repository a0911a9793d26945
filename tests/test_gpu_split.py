"""GPU: the cycle on split-ordered copies (each level's F-points first, then
its C-points) against the cycle on the natural matrices.

Renumbering rows and columns keeps every row's entries in their stored
order, so each row sum of the cycle is formed in the same order: solutions
and single cycles must agree bit for bit, and so must the iteration counts.
The natural-ordering solve is itself pinned to the oracle by the parity
tests.
"""
import sys

import numpy as np
import pytest

import workloads as W
from oracle import lair as O

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


def _cases():
    return ["c1_one_point", "euler3d_direct_16rhs", "euler3d_direct_mixed",
            "dg_block_distance2", "adr_mixed_1rhs"]


def _build(lair, case, ordering):
    if case == "c1_one_point":
        w = W.workload_c1(48)
        kw = dict()
        b = w["rhs"]
    elif case.startswith("euler3d"):
        nr = 16 if case.endswith("16rhs") else 4
        w = W.implicit_euler_adr_3d(m=16, nrhs=nr)
        kw = dict(interp="direct", precision="mixed" if case.endswith("mixed") else "fp64")
        b = w["rhs"]
    elif case == "dg_block_distance2":
        w = W.upwind_dg_p2(8)
        kw = dict(distance=2, block_size=6, max_coarse=20)
        b = w["rhs"]
    else:
        w = W.adr_2d(60, 1.0, 0.5, 0.0)
        kw = dict(interp="direct", precision="mixed")
        b = np.random.default_rng(3).standard_normal(w["n"])
    h = lair.setup(w["rowptr"], w["col"], w["val"], ordering=ordering, **kw)
    return h, b


@pytest.mark.parametrize("case", _cases())
def test_split_solve_equals_natural(lair, case):
    _say("case: split vs natural ordering,", case)
    hs, b = _build(lair, case, "split")
    hn, _ = _build(lair, case, "natural")
    assert hs.nlevels == hn.nlevels
    maxit = 5 if case.startswith("dg") else 200
    xs, infs = hs.solve(_dev(b), rtol=1e-10, maxit=maxit)
    xn, infn = hn.solve(_dev(b), rtol=1e-10, maxit=maxit)
    _say("  iterations", infs["iters"], infn["iters"])
    assert infs["iters"] == infn["iters"]
    assert np.array_equal(xs.cpu().numpy(), xn.cpu().numpy())
    # a nonzero initial guess and a single cycle
    x0 = np.random.default_rng(5).standard_normal(np.shape(b))
    ys = hs.cycle(_dev(b), _dev(x0))
    yn = hn.cycle(_dev(b), _dev(x0))
    assert np.array_equal(ys.cpu().numpy(), yn.cpu().numpy())
    # the caller's initial guess is used (warm start equals continuing)
    xw, infw = hs.solve(_dev(b), x=_dev(x0), rtol=1e-10, maxit=maxit)
    xw2, _ = hn.solve(_dev(b), x=_dev(x0), rtol=1e-10, maxit=maxit)
    assert np.array_equal(xw.cpu().numpy(), xw2.cpu().numpy())
    hs.free()
    hn.free()


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_auto_ordering_renumbers_a_prefix(lair, precision):
    """48^3 grid: level 0 (110,592 rows, 7 per row) is renumbered by the
    default ordering, the next level (below 65,536 rows) is not, so the
    transfer operators between them map one side only."""
    _say("case: auto ordering, 48^3,", precision)
    w = W.implicit_euler_adr_3d(m=48, nrhs=4)
    kw = dict(interp="direct", precision=precision)
    ha = lair.setup(w["rowptr"], w["col"], w["val"], **kw)
    hn = lair.setup(w["rowptr"], w["col"], w["val"], ordering="natural", **kw)
    xa, ia = ha.solve(_dev(w["rhs"]), rtol=1e-10)
    xn, inn = hn.solve(_dev(w["rhs"]), rtol=1e-10)
    _say("  iterations", ia["iters"], inn["iters"])
    assert ia["converged"] and ia["iters"] == inn["iters"]
    assert np.array_equal(xa.cpu().numpy(), xn.cpu().numpy())
    ha.free()
    hn.free()


def test_split_levels_export_natural(lair):
    """Exports stay in the natural ordering: the split copies are private to
    the cycle, the hierarchy's matrices still match the oracle."""
    w = W.workload_c1(40)
    A = O.csr(w["rowptr"], w["col"], w["val"])
    H = O.setup(A)
    h = lair.setup(w["rowptr"], w["col"], w["val"])
    from tests.parity import compare_level
    for l in range(h.nlevels - 1):
        compare_level(h, l)
    x, info = h.solve(_dev(w["rhs"]), rtol=1e-10)
    xo, ito, _ = O.solve(H, w["rhs"], rtol=1e-10)
    assert info["iters"] == ito
    assert np.abs(x.cpu().numpy() - xo).max() <= 1e-9 * np.abs(xo).max()


@pytest.mark.parametrize("ordering", ["auto", "split"])
def test_copies_behind_readbacks_equal_copies_at_the_end(lair, ordering):
    """The split-ordered copies are queued behind the setup's readbacks, level
    by level as their inputs appear; with the profiler on they are all made
    at the end of setup instead.  The two hierarchies must solve alike, bit
    for bit (the profiler also runs the cycles without graphs, which the
    graph tests pin to the captured cycles).  48^3, 16 right-hand sides,
    lumped, mixed precision: the timed configuration at a smaller size."""
    _say("case: copies behind readbacks vs at the end,", ordering)
    w = W.implicit_euler_adr_3d(m=48, nrhs=16)
    kw = dict(interp="direct", precision="mixed", lump_tol=1e-3, ordering=ordering)
    b = _dev(w["rhs"])
    hq = lair.setup(w["rowptr"], w["col"], w["val"], **kw)
    xq, iq = hq.solve(b, rtol=1e-10)
    lair.profile_begin(None)
    try:
        he = lair.setup(w["rowptr"], w["col"], w["val"], **kw)
        xe, ie = he.solve(b, rtol=1e-10)
    finally:
        lair.profile_end()
    _say("  levels", hq.nlevels, he.nlevels, "iterations", iq["iters"], ie["iters"])
    assert hq.nlevels == he.nlevels
    assert iq["converged"] and iq["iters"] == ie["iters"]
    assert np.array_equal(xq.cpu().numpy(), xe.cpu().numpy())
    hq.free()
    he.free()
