"""Failure paths on the GPU, forced from the host: an allocation cap
(LAIR_DEBUG_MAX_BYTES) makes setup and solve fail with LAIR_ENOMEM as a real
shortage would; nothing is leaked (the library's device bytes in use return
to their value before the call, or before the hierarchy once it is freed),
and a hierarchy whose solve failed solves correctly once memory is there."""
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


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _dev(x):
    import torch
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


def test_allocation_cap_enomem_and_nothing_leaked(lair, monkeypatch):
    import torch
    from paper_1708_06065_amd import LairError
    w = W.implicit_euler_adr_3d(m=24, nrhs=4)
    args = (w["rowptr"], w["col"], w["val"])
    monkeypatch.delenv("LAIR_DEBUG_MAX_BYTES", raising=False)
    base, _ = lair.memory()
    h = lair.setup(*args, interp="direct")
    need = lair.memory()[0] - base
    h.free()
    assert lair.memory()[0] == base
    _say("  setup holds %d bytes" % need)
    # setup: the cap hit early, halfway, and just short of the end
    for cap in (base + 4096, base + need // 2, base + need - 1):
        monkeypatch.setenv("LAIR_DEBUG_MAX_BYTES", str(cap))
        with pytest.raises(LairError) as e:
            lair.setup(*args, interp="direct")
        assert e.value.status == -2, e.value
        assert lair.memory()[0] == base, cap
    monkeypatch.delenv("LAIR_DEBUG_MAX_BYTES")
    # solve: its work vectors refused, the hierarchy left usable
    h = lair.setup(*args, interp="direct")
    held = lair.memory()[0]
    B = _dev(w["rhs"])
    monkeypatch.setenv("LAIR_DEBUG_MAX_BYTES", str(held + 4096))
    with pytest.raises(LairError) as e:
        h.solve(B)
    assert e.value.status == -2
    monkeypatch.delenv("LAIR_DEBUG_MAX_BYTES")
    X, info = h.solve(B, rtol=1e-10)
    assert info["converged"]
    A = O.csr(*args)
    Xh = X.cpu().numpy()
    for q in range(4):
        r = w["rhs"][:, q] - A @ Xh[:, q]
        assert np.linalg.norm(r) <= 1e-10 * np.linalg.norm(w["rhs"][:, q])
    h.free()
    torch.cuda.synchronize()
    assert lair.memory()[0] == base
