"""lair_cycle_noalloc (the cycle with its work vectors in the library's fixed
device array) against lair_cycle through the C ABI: bitwise the same
iterate, on two calls in a row with the second on a smaller input, on a
fresh hierarchy and on one whose own work vectors exist (they are left as
they were); a cycle whose vectors do not fit is refused before any device
work and leaves x unchanged."""
import sys

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


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


def _cases():
    big = W.implicit_euler_adr_3d(m=28, nrhs=4)
    small = W.workload_c1(32)
    dg = W.upwind_dg_p2(10)
    return [
        ("euler3d 28^3, 4 rhs, fp64, split ordering", big,
         dict(interp="direct", ordering="split"), 4),
        ("transport 32x32, 1 rhs, fp64", small, dict(), 1),
        ("euler3d 28^3, 4 rhs, mixed", big, dict(interp="direct", precision="mixed"), 4),
        ("dg p2 10x10x2, block-scaled, distance 2", dg, dict(distance=2, block_size=6), 1),
    ]


def test_noalloc_cycle_equals_cycle(lair):
    import torch
    rng = np.random.default_rng(5)
    for name, w, kw, nrhs in _cases():
        _say("case:", name)
        n = w["n"]
        shape = (n,) if nrhs == 1 else (n, nrhs)
        b = _dev(rng.standard_normal(shape))
        x0 = _dev(rng.standard_normal(shape))
        h = lair.setup(w["rowptr"], w["col"], w["val"], max_coarse=20, **kw)
        # fresh hierarchy: the no-allocation cycle first, then the plain one
        xa = x0.clone()
        h.cycle_noalloc(b, xa)
        xr = x0.clone()
        h.cycle(b, xr)
        torch.cuda.synchronize()
        assert torch.equal(xa, xr), name
        # again, now that the hierarchy holds its own vectors; those still
        # give the same cycle afterwards
        xa2 = xr.clone()
        h.cycle_noalloc(b, xa2)
        xr2 = xr.clone()
        h.cycle(b, xr2)
        torch.cuda.synchronize()
        assert torch.equal(xa2, xr2), name
        assert not torch.equal(xr2, xr)
        h.free()


def test_noalloc_refuses_what_does_not_fit(lair):
    import torch
    from paper_1708_06065_amd import LairError
    w = W.implicit_euler_adr_3d(m=64, nrhs=16)
    h = lair.setup(w["rowptr"], w["col"], w["val"], interp="direct")
    B = _dev(w["rhs"])
    X = torch.ones_like(B)
    with pytest.raises(LairError) as e:
        h.cycle_noalloc(B, X)
    assert e.value.status == -6
    torch.cuda.synchronize()
    assert bool((X == 1.0).all())
    # one right-hand side fits, and matches the plain cycle
    b1 = B[:, 0].contiguous()
    xa = torch.zeros_like(b1)
    xr = torch.zeros_like(b1)
    h.cycle_noalloc(b1, xa)
    h.cycle(b1, xr)
    torch.cuda.synchronize()
    assert torch.equal(xa, xr)
    h.free()
