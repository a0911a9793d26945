"""lAIR on MI355X: Python binding of liblair (argument marshalling only).

Every step of the setup and of the cycles runs in the HIP kernels of
liblair.so (include/lair.h).  PyTorch supplies device memory and the current
HIP stream.  There is no CPU fallback: if the library is not built or no GPU
is visible, the calls raise.

    import paper_1708_06065_amd as lair
    h = lair.setup(rowptr, col, val, distance=2, interp="one_point")
    x, info = h.solve(b)                 # b: torch tensor on the GPU
"""
import ctypes

import numpy as np

from . import _lib as L
from ._lib import LairError  # noqa: F401

__all__ = ["setup", "setup_batch", "Hierarchy", "LairError", "load_library",
           "memory", "profile_begin", "profile_end"]

_KINDS = {"abs": L.SOC_ABS, "neg": L.SOC_NEG}
_INTERP = {"one_point": L.P_ONE_POINT, "direct": L.P_DIRECT}
_PREC = {"fp64": L.FP64, "mixed": L.MIXED, "mixed_local": L.MIXED_LOCAL}
_ORDERING = {"auto": 0, "natural": L.FLAG_NATURAL_ORDER, "split": L.FLAG_SPLIT_ALL}
_DIST = {1: 1, 2: 2, "all_f": L.DIST_ALL_F, 0: L.DIST_ALL_F}

EXPORT_WHAT = {
    "A.rowptr": (0, np.int32), "A.col": (1, np.int32), "A.val": (2, np.float64),
    "cf": (3, np.int8), "smask": (4, np.uint8),
    "R.rowptr": (5, np.int32), "R.col": (6, np.int32), "R.val": (7, np.float64),
    "P.rowptr": (8, np.int32), "P.col": (9, np.int32), "P.val": (10, np.float64),
    "nbr_ptr": (11, np.int32), "nbr": (12, np.int32), "flags": (13, np.int8),
}


def load_library():
    return L.load()


def _torch():
    import torch
    return torch


def _stream_ptr(stream):
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _dev_ptr(t, dtype, name):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a CUDA (HIP) tensor" % name)
    if t.dtype != dtype or not t.is_contiguous():
        raise TypeError("%s must be contiguous %s" % (name, dtype))
    return ctypes.c_void_p(t.data_ptr())


class Hierarchy:
    """An lAIR hierarchy living on the GPU (owns liblair's handle)."""

    def __init__(self, handle, n, options):
        self._h = handle
        self.n = n
        self.options = options

    # -- lifetime ---------------------------------------------------------
    def free(self):
        if self._h:
            L.load().lair_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    @property
    def handle(self):
        if not self._h:
            raise RuntimeError("hierarchy has been freed")
        return self._h

    # -- introspection ----------------------------------------------------
    @property
    def nlevels(self):
        return L.load().lair_num_levels(self.handle)

    def level_stats(self, level):
        st = L.LevelStats()
        L.check(L.load().lair_level_stats_get(self.handle, level, ctypes.byref(st)),
                "lair_level_stats_get")
        return st.as_dict()

    def export(self, level, what):
        code, dt = EXPORT_WHAT[what]
        nb = ctypes.c_int64(0)
        lib = L.load()
        L.check(lib.lair_export(self.handle, level, code, None, ctypes.byref(nb)),
                "lair_export")
        out = np.zeros(nb.value // np.dtype(dt).itemsize, dtype=dt)
        if nb.value:
            L.check(lib.lair_export(self.handle, level, code,
                                    out.ctypes.data_as(ctypes.c_void_p),
                                    ctypes.byref(nb)), "lair_export")
        return out

    # -- cycles and solves --------------------------------------------------
    def _nrhs(self, b):
        if b.dim() == 1:
            return 1
        return b.shape[1]

    def local_buckets(self, level):
        """Size-bucket edges and fused flag the local solves of `level` used."""
        e = np.zeros(5, dtype=np.int32)
        L.check(L.load().lair_local_buckets(self.handle, int(level),
                                            e.ctypes.data_as(ctypes.c_void_p)),
                "lair_local_buckets")
        return e

    def cycle(self, b, x, stream=None):
        """x <- x + B (b - A x): one V-cycle, in place on device tensors."""
        torch = _torch()
        nr = self._nrhs(b)
        L.check(L.load().lair_cycle(self.handle, _dev_ptr(b, torch.float64, "b"),
                                    _dev_ptr(x, torch.float64, "x"), nr,
                                    _stream_ptr(stream)), "lair_cycle")
        return x

    def cycle_noalloc(self, b, x, stream=None):
        """The same cycle with the work vectors in the library's fixed device
        array (lair_cycle_noalloc): no device allocation in the call."""
        torch = _torch()
        nr = self._nrhs(b)
        L.check(L.load().lair_cycle_noalloc(self.handle, _dev_ptr(b, torch.float64, "b"),
                                            _dev_ptr(x, torch.float64, "x"), nr,
                                            _stream_ptr(stream)), "lair_cycle_noalloc")
        return x

    def cycle_transpose(self, g, lam, stream=None):
        torch = _torch()
        nr = self._nrhs(g)
        L.check(L.load().lair_cycle_transpose(self.handle, _dev_ptr(g, torch.float64, "g"),
                                              _dev_ptr(lam, torch.float64, "lam"), nr,
                                              _stream_ptr(stream)),
                "lair_cycle_transpose")
        return lam

    def solve(self, b, x=None, rtol=1e-10, maxit=200, stream=None,
              raise_on_noconv=False):
        """Stationary V-cycle iteration.  Returns (x, info dict)."""
        torch = _torch()
        if x is None:
            x = torch.zeros_like(b)
        info = L.Info()
        st = L.load().lair_solve(self.handle, _dev_ptr(b, torch.float64, "b"),
                                 _dev_ptr(x, torch.float64, "x"), self._nrhs(b),
                                 float(rtol), int(maxit), ctypes.byref(info),
                                 _stream_ptr(stream))
        if st != L.LAIR_OK and (st != L.LAIR_ENOCONV or raise_on_noconv):
            L.check(st, "lair_solve")
        d = info.as_dict()
        d["converged"] = st == L.LAIR_OK
        return x, d

    def solve_fgmres(self, b, x=None, rtol=1e-10, maxit=200, restart=20, stream=None,
                     raise_on_noconv=False):
        """Flexible GMRES(restart) with one V-cycle as the preconditioner.
        Returns (x, info dict); iters counts Arnoldi steps (V-cycles)."""
        torch = _torch()
        if x is None:
            x = torch.zeros_like(b)
        info = L.Info()
        st = L.load().lair_solve_fgmres(self.handle, _dev_ptr(b, torch.float64, "b"),
                                        _dev_ptr(x, torch.float64, "x"), self._nrhs(b),
                                        float(rtol), int(maxit), int(restart),
                                        ctypes.byref(info), _stream_ptr(stream))
        if st != L.LAIR_OK and (st != L.LAIR_ENOCONV or raise_on_noconv):
            L.check(st, "lair_solve_fgmres")
        d = info.as_dict()
        d["converged"] = st == L.LAIR_OK
        return x, d

    def update_diag(self, diag, stream=None):
        """New diagonal of A (NumPy array or CUDA float64 tensor of n values):
        same structure, values rebuilt."""
        torch = _torch()
        if isinstance(diag, torch.Tensor) and diag.is_cuda:
            ptr, dev = _dev_ptr(diag, torch.float64, "diag"), 1
            keep = diag
        else:
            keep = np.ascontiguousarray(diag, dtype=np.float64)
            ptr, dev = keep.ctypes.data_as(ctypes.c_void_p), 0
        L.check(L.load().lair_update_diag(self.handle, ptr, dev, _stream_ptr(stream)),
                "lair_update_diag")
        del keep
        return self

    @property
    def nsys(self):
        return L.load().lair_num_systems(self.handle)

    def system_levels(self):
        """Levels of each system of a batch on its own (int32 array)."""
        out = np.zeros(self.nsys, dtype=np.int32)
        L.check(L.load().lair_system_levels(self.handle, out.ctypes.data_as(ctypes.c_void_p)),
                "lair_system_levels")
        return out

    def solve_batch(self, b, x=None, rtol=1e-10, maxit=200, stream=None,
                    raise_on_noconv=False):
        """Per-system stationary iteration on a batch's union vectors.
        Returns (x, info dict with per-system 'iters' and 'relres' arrays)."""
        torch = _torch()
        if x is None:
            x = torch.zeros_like(b)
        ns = self.nsys
        its = np.zeros(ns, dtype=np.int32)
        rel = np.zeros(ns, dtype=np.float64)
        info = L.Info()
        st = L.load().lair_solve_batch(self.handle, _dev_ptr(b, torch.float64, "b"),
                                       _dev_ptr(x, torch.float64, "x"), float(rtol), int(maxit),
                                       its.ctypes.data_as(ctypes.c_void_p),
                                       rel.ctypes.data_as(ctypes.c_void_p),
                                       ctypes.byref(info), _stream_ptr(stream))
        if st != L.LAIR_OK and (st != L.LAIR_ENOCONV or raise_on_noconv):
            L.check(st, "lair_solve_batch")
        d = info.as_dict()
        d["converged"] = st == L.LAIR_OK
        d["sys_iters"] = its
        d["sys_relres"] = rel
        return x, d

    def solve_transpose(self, g, lam=None, rtol=1e-10, maxit=200, stream=None,
                        raise_on_noconv=False):
        torch = _torch()
        if lam is None:
            lam = torch.zeros_like(g)
        info = L.Info()
        st = L.load().lair_solve_transpose(self.handle, _dev_ptr(g, torch.float64, "g"),
                                           _dev_ptr(lam, torch.float64, "lam"),
                                           self._nrhs(g), float(rtol), int(maxit),
                                           ctypes.byref(info), _stream_ptr(stream))
        if st != L.LAIR_OK and (st != L.LAIR_ENOCONV or raise_on_noconv):
            L.check(st, "lair_solve_transpose")
        d = info.as_dict()
        d["converged"] = st == L.LAIR_OK
        return lam, d


def memory():
    """(bytes in use, bytes cached) of the library's device memory."""
    a, b = ctypes.c_int64(0), ctypes.c_int64(0)
    L.load().lair_memory(ctypes.byref(a), ctypes.byref(b))
    return a.value, b.value


def profile_begin(categories=None):
    """Start the library's kernel profiler (HIP events per launch) for the
    given categories (list or comma-separated string; None = all)."""
    if isinstance(categories, (list, tuple)):
        categories = ",".join(categories)
    L.check(L.load().lair_profile_begin(None if categories is None else categories.encode()),
            "lair_profile_begin")


def profile_end():
    """Stop profiling; returns {category: {launches, ms, ms_max, alg_bytes,
    alg_flops}} summed over the profiled launches."""
    import json
    lib = L.load()
    n = ctypes.c_int64(0)
    lib.lair_profile_end(None, ctypes.byref(n))
    buf = ctypes.create_string_buffer(int(n.value) + 16)
    n2 = ctypes.c_int64(len(buf))
    L.check(lib.lair_profile_end(buf, ctypes.byref(n2)), "lair_profile_end")
    return json.loads(buf.value.decode() or "{}")


def _csr(rowptr, col, val, keep):
    """lair_csr for NumPy (host) or CUDA-tensor (device) arrays."""
    torch = _torch()
    on_dev = isinstance(val, torch.Tensor) and val.is_cuda
    if on_dev:
        rp = _dev_ptr(rowptr, torch.int32, "rowptr")
        cj = _dev_ptr(col, torch.int32, "col")
        vx = _dev_ptr(val, torch.float64, "val")
        n = rowptr.shape[0] - 1
        nnz = col.shape[0]
    else:
        a = np.ascontiguousarray(rowptr, dtype=np.int32)
        c = np.ascontiguousarray(col, dtype=np.int32)
        v = np.ascontiguousarray(val, dtype=np.float64)
        keep += [a, c, v]
        rp, cj, vx = (x.ctypes.data_as(ctypes.c_void_p) for x in (a, c, v))
        n = a.shape[0] - 1
        nnz = c.shape[0]
    return L.Csr(n, nnz, rp, cj, vx, 1 if on_dev else 0), n


def _cf_levels(cf_levels, keep):
    """lair_cf_levels pointer (or None) for a list of per-level splittings:
    NumPy arrays (host), or CUDA int8 tensors (device, concatenated on the
    device)."""
    if cf_levels is None:
        return None
    torch = _torch()
    on_dev = len(cf_levels) > 0 and all(isinstance(x, torch.Tensor) and x.is_cuda
                                        for x in cf_levels)
    sizes = [int(x.shape[0]) for x in cf_levels]
    offs = np.zeros(len(sizes) + 1, dtype=np.int64)
    offs[1:] = np.cumsum(sizes)
    if on_dev:
        flat = torch.cat([x.to(torch.int8).contiguous() for x in cf_levels])
        ptr = ctypes.c_void_p(flat.data_ptr())
    else:
        arrs = [np.ascontiguousarray(x, dtype=np.int8) for x in cf_levels]
        flat = np.concatenate(arrs) if arrs else np.zeros(1, np.int8)
        ptr = flat.ctypes.data_as(ctypes.c_void_p)
    keep += [offs, flat]
    cfl = L.CfLevels(len(sizes), offs.ctypes.data_as(ctypes.c_void_p), ptr,
                     1 if on_dev else 0)
    keep.append(cfl)
    return ctypes.byref(cfl)


_SPLIT = {"rs": 0, "pmis": L.FLAG_PMIS}


def _params(theta, theta_c, kind, distance, interp, precision, omega, max_levels,
            max_coarse, stall, block_size, graphs, ordering="auto", lump_tol=0.0,
            nodal=False, split="rs"):
    s = L.Strength(float(theta), float(theta if theta_c is None else theta_c),
                   _KINDS[kind], _DIST[distance])
    o = L.Options(_INTERP[interp], _PREC[precision], float(omega), int(max_levels),
                  int(max_coarse), float(stall), int(block_size),
                  (0 if graphs else L.FLAG_NO_GRAPH) | _ORDERING[ordering] |
                  (L.FLAG_NODAL if nodal else 0) | _SPLIT[split],
                  float(lump_tol))
    opts = dict(theta=theta, theta_c=theta_c, kind=kind, distance=distance,
                interp=interp, precision=precision, omega=omega,
                max_levels=max_levels, max_coarse=max_coarse, stall=stall,
                block_size=block_size, graphs=graphs, ordering=ordering,
                lump_tol=lump_tol, nodal=nodal, split=split)
    return s, o, opts


def set_local_buckets(edges=None):
    """Fix the size buckets of the local solves for every later setup of the
    process (5 ints: largest S_i per lane, per 8-, 16- and 32-lane team, and
    1 to run the first three buckets in the shared persistent kernel), or
    with None let the library tune them per level shape.  The choice
    changes speed only; the results are bitwise the same."""
    lib = L.load()
    if edges is None:
        L.check(lib.lair_set_local_buckets(None), "lair_set_local_buckets")
        return
    e = np.ascontiguousarray(edges, dtype=np.int32)
    if e.shape != (5,):
        raise ValueError("edges: 5 values")
    L.check(lib.lair_set_local_buckets(e.ctypes.data_as(ctypes.c_void_p)),
            "lair_set_local_buckets")


def setup_batch(systems, cf_levels=None, theta=0.25, theta_c=None, kind="abs",
                distance=1, interp="one_point", precision="fp64", omega=1.0,
                max_levels=25, max_coarse=128, stall=0.9, block_size=0, graphs=True,
                lump_tol=0.0, split="rs", stream=None):
    """One hierarchy for a batch of independent systems.

    systems: list of (rowptr, col, val), all NumPy (host) or all CUDA
    tensors.  Vectors of the returned hierarchy are the concatenation of the
    systems' vectors in list order.  cf_levels: optional per-level
    splittings of the union (as exported by a previous batch setup).
    """
    lib = L.load()
    keep = []
    mats = []
    for (rp, cj, v) in systems:
        A, _ = _csr(rp, cj, v, keep)
        mats.append(A)
    arr = (L.Csr * len(mats))(*mats)
    s, o, opts = _params(theta, theta_c, kind, distance, interp, precision, omega,
                         max_levels, max_coarse, stall, block_size, graphs,
                         lump_tol=lump_tol, split=split)
    out = ctypes.c_void_p()
    cfp = _cf_levels(cf_levels, keep)
    st = lib.lair_setup_batch(len(mats), arr, cfp, ctypes.byref(s), ctypes.byref(o),
                              _stream_ptr(stream), ctypes.byref(out))
    L.check(st, "lair_setup_batch")
    return Hierarchy(out, int(sum(m.n for m in mats)), opts)


def setup(rowptr, col, val, cf_levels=None, theta=0.25, theta_c=None,
          kind="abs", distance=1, interp="one_point", precision="fp64",
          omega=1.0, max_levels=25, max_coarse=128, stall=0.9, block_size=0,
          graphs=True, ordering="auto", lump_tol=0.0, nodal=False, split="rs", stream=None):
    """Build a hierarchy for the CSR matrix (rowptr, col, val).

    The arrays may be NumPy arrays (host) or contiguous CUDA tensors
    (int32, int32, float64).  cf_levels is an optional list of per-level
    int8 CF splittings (1 = C): NumPy arrays, or CUDA tensors (checked and
    counted on the device).  graphs=False launches the
    solve's kernels eagerly instead of replaying captured iterations.
    ordering: "auto" runs the cycle on F-first renumbered copies of the
    large sparse levels, "natural" on the natural matrices everywhere,
    "split" renumbers every level but the coarsest; the results are bitwise
    the same.  lump_tol > 0 lumps every coarse operator (Sec. 3.3).
    nodal=True with block_size=k builds the hierarchy by k x k blocks (the
    nodal treatment of Sec. 4.2) instead of scaling by the block diagonal.
    split="pmis" splits the levels without a given splitting on the device
    by a parallel PMIS-type splitting instead of the host first pass.
    """
    lib = L.load()
    keep = []
    A, n = _csr(rowptr, col, val, keep)
    s, o, opts = _params(theta, theta_c, kind, distance, interp, precision, omega,
                         max_levels, max_coarse, stall, block_size, graphs, ordering,
                         lump_tol, nodal, split)
    cfp = _cf_levels(cf_levels, keep)
    out = ctypes.c_void_p()
    st = lib.lair_setup(ctypes.byref(A), cfp, ctypes.byref(s), ctypes.byref(o),
                        _stream_ptr(stream), ctypes.byref(out))
    L.check(st, "lair_setup")
    return Hierarchy(out, n, opts)
