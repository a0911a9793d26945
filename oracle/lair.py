"""FP64 CPU oracle for lAIR (arXiv:1708.06065).

TEST INFRASTRUCTURE ONLY: this module is the reference the GPU library is
checked against.  Only tests, the smoke check and the benchmark's CPU-baseline
leg may import it; the solver library never does, and the two share no code.

The heavy per-row loops (strength, Ruge-Stueben split, neighbourhoods, local
solves, interpolation, sparse products) are in ``lair_oracle.c``; this module
strings them together in the paper's order and adds the parts that are plain
library calls (SciPy sparse products with vectors, a dense LU for the
coarsest grid, minimal-norm least squares for singular local systems).

Steps and where the paper defines them:
  strength          Sec. 4 (strong neighbourhood with a hard minimum)
  rs_split          Sec. 4 (classical CF splitting, first pass only)
  neighbourhoods    Sec. 3.1 (distance-one or -two strong F-neighbours) and
                    Sec. 4 (F-F-C paths only at distance two)
  local_solves      Sec. 3.1, Eq. (johnair) / Eq. (system) and its footnote
  restriction       Eq. (PR): R = [Z I]
  interp_one_point  Sec. 4 (one-point interpolation)
  interp_direct     classical direct interpolation (Stueben 2001) as a
                    stand-in for the classical formulas cited in Sec. 4
  galerkin          Sec. 2.1: K = R A P
  lump              Sec. 3.3 (filtering and lumping): entries of a coarse
                    row below theta_D times the row's largest magnitude
                    (diagonal included) move to the diagonal
  block_scale       Sec. 4.2.1: D_B^{-1} A with the element block diagonal
  cycle             Sec. 2.1 coarse-grid correction followed by F-F-C Jacobi
                    (Sec. 4, relaxation paragraph; Eq. (jacobi_err))
  solve             stationary iteration on the V-cycle to a relative
                    residual tolerance
  cycle_transpose   the exact adjoint of ``cycle`` (for gradients)
  fgmres            flexible GMRES(m) with one V-cycle as the right
                    preconditioner (the outer solver of Sec. 4's results)
  setup(block=k)    nodal treatment of a k x k block structure (Sec. 3.1, the
                    block form of Eq. (system); Sec. 4.2, treatment (iii)):
                    strength and CF splitting on the graph of blocks, local
                    systems by block with k right-hand sides, one-point
                    interpolation by block, block Jacobi relaxation
  update_diag       a new diagonal on a kept hierarchy structure: Eq. (system)
                    solves, interpolation weights and Sec. 2.1 Galerkin
                    products recomputed on the same neighbourhoods, splittings
                    and patterns
"""
import ctypes
import math
import os

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from . import build as _build

SOC_ABS, SOC_NEG = 0, 1
DIST_ALL_F = 0
INTERP_ONE_POINT, INTERP_DIRECT = 0, 1

_lib = None


def lib():
    global _lib
    if _lib is None:
        path = _build.build(force=False)
        L = ctypes.CDLL(path)
        P = ctypes.c_void_p
        i64, i32, f64 = ctypes.c_int64, ctypes.c_int32, ctypes.c_double
        L.orc_strength.argtypes = [i64, P, P, P, f64, i32, P]
        L.orc_strength.restype = None
        L.orc_rs_split.argtypes = [i64, P, P, P, P]
        L.orc_rs_split.restype = i32
        L.orc_nbr_count.argtypes = [i64, P, P, P, P, i32, i64, P, P]
        L.orc_nbr_count.restype = i32
        L.orc_nbr_fill.argtypes = [i64, P, P, P, P, i32, i64, P, P, P]
        L.orc_nbr_fill.restype = i32
        L.orc_local_solves.argtypes = [P, P, P, i64, P, P, P, P, P]
        L.orc_local_solves.restype = i32
        L.orc_interp_one_point.argtypes = [i64, P, P, P, P, P, P, P]
        L.orc_interp_one_point.restype = None
        L.orc_interp_direct.argtypes = [i64, P, P, P, P, P, P, i32, P, P, P]
        L.orc_interp_direct.restype = None
        L.orc_spgemm_count.argtypes = [i64, i64, P, P, P, P, P]
        L.orc_spgemm_count.restype = i32
        L.orc_spgemm_fill.argtypes = [i64, i64, P, P, P, P, P, P, P, P, P]
        L.orc_spgemm_fill.restype = i32
        L.orc_lump.argtypes = [i64, P, P, P, f64, i32, P, P, P, P, P]
        L.orc_lump.restype = None
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def csr(rowptr, col, val, shape=None):
    """scipy CSR from raw arrays, keeping every stored entry (even zeros)."""
    rowptr = np.ascontiguousarray(rowptr, dtype=np.int32)
    n = rowptr.shape[0] - 1
    if shape is None:
        shape = (n, n)
    m = sp.csr_matrix((np.ascontiguousarray(val, dtype=np.float64),
                       np.ascontiguousarray(col, dtype=np.int32), rowptr),
                      shape=shape)
    return m


def _arrays(A):
    return (np.ascontiguousarray(A.indptr, dtype=np.int32),
            np.ascontiguousarray(A.indices, dtype=np.int32),
            np.ascontiguousarray(A.data, dtype=np.float64))


# --------------------------------------------------------------------------
# Setup steps
# --------------------------------------------------------------------------

def strength(A, theta=0.25, kind=SOC_ABS):
    """Strong-connection mask over A's stored entries (uint8[nnz])."""
    rp, cj, vx = _arrays(A)
    smask = np.zeros(cj.shape[0], dtype=np.uint8)
    lib().orc_strength(A.shape[0], _p(rp), _p(cj), _p(vx), float(theta),
                       int(kind), _p(smask))
    return smask


def rs_split(A, smask):
    """Classical Ruge-Stueben first pass: int8[n], 1 = C, 0 = F."""
    rp, cj, _ = _arrays(A)
    cf = np.zeros(A.shape[0], dtype=np.int8)
    st = lib().orc_rs_split(A.shape[0], _p(rp), _p(cj),
                            _p(np.ascontiguousarray(smask, dtype=np.uint8)),
                            _p(cf))
    if st != 0:
        raise MemoryError("rs_split")
    return cf


def hash32(i):
    """MurmurHash3's 32-bit finalizer (fmix32, A. Appleby) of the indices:
    the deterministic tie-breaking weight of the parallel splitting."""
    h = np.asarray(i, dtype=np.uint64) & np.uint64(0xFFFFFFFF)
    m = np.uint64(0xFFFFFFFF)
    h ^= h >> np.uint64(16)
    h = (h * np.uint64(0x85EBCA6B)) & m
    h ^= h >> np.uint64(13)
    h = (h * np.uint64(0xC2B2AE35)) & m
    h ^= h >> np.uint64(16)
    return h


def pmis_split(A, smask):
    """A parallel CF splitting of the PMIS type (De Sterck, Yang and Heys,
    2006), an alternative to the Ruge-Stueben first pass of Sec. 4 that
    needs no sequential greedy step.  Weight of point i: the number of
    points that strongly depend on it, then hash32(i), then i.  Points on
    which no point strongly depends are F.  Each round, every undecided
    point whose weight exceeds that of every undecided point it is strongly
    connected to (either direction) becomes C, then every undecided point
    that strongly depends on a C-point becomes F.  int8[n], 1 = C, 0 = F."""
    A = A.tocsr()
    n = A.shape[0]
    rows = np.repeat(np.arange(n), np.diff(A.indptr))
    sm = np.asarray(smask).astype(bool) & (A.indices != rows)
    sj, si = rows[sm], A.indices[sm]            # j strongly depends on i
    cnt = np.bincount(si, minlength=n).astype(np.uint64)
    key = (cnt << np.uint64(32)) | hash32(np.arange(n))
    state = np.where(cnt == 0, 0, -1).astype(np.int8)
    while (state == -1).any():
        und = state == -1
        cand = und.copy()
        live = und[sj] & und[si]
        a, b = sj[live], si[live]
        b_wins = (key[b] > key[a]) | ((key[b] == key[a]) & (b > a))
        cand[a[b_wins]] = False
        cand[b[~b_wins]] = False
        state[cand] = 1
        hit = (state[sj] == -1) & (state[si] == 1)
        state[sj[hit]] = 0
    return state


def coarse_index(cf):
    """C-points numbered in increasing fine index; -1 for F-points."""
    cf = np.asarray(cf)
    cidx = np.full(cf.shape[0], -1, dtype=np.int32)
    cpts = np.flatnonzero(cf == 1).astype(np.int32)
    cidx[cpts] = np.arange(cpts.shape[0], dtype=np.int32)
    return cidx, cpts


def neighbourhoods(A, smask, cf, distance=1):
    """Sorted restriction neighbourhoods N_i of every C-point.

    Returns (cpts, nptr int64[nc+1], nbr int32[sum S_i]).
    """
    rp, cj, _ = _arrays(A)
    cf = np.ascontiguousarray(cf, dtype=np.int8)
    smask = np.ascontiguousarray(smask, dtype=np.uint8)
    _, cpts = coarse_index(cf)
    nc = cpts.shape[0]
    cnt = np.zeros(nc, dtype=np.int64)
    L = lib()
    L.orc_nbr_count(A.shape[0], _p(rp), _p(cj), _p(smask), _p(cf),
                    int(distance), nc, _p(cpts), _p(cnt))
    nptr = np.zeros(nc + 1, dtype=np.int64)
    np.cumsum(cnt, out=nptr[1:])
    nbr = np.zeros(max(int(nptr[-1]), 1), dtype=np.int32)
    L.orc_nbr_fill(A.shape[0], _p(rp), _p(cj), _p(smask), _p(cf),
                   int(distance), nc, _p(cpts), _p(nptr), _p(nbr))
    return cpts, nptr, nbr[:nptr[-1]]


def local_system(A, i, nb):
    """Dense M = A(N,N)^T and f = -A(i,N)^T of Eq. (system) for one C-point."""
    sub = A[nb][:, nb].toarray()
    M = sub.T.copy()
    f = -A[i][:, nb].toarray().ravel()
    return M, f


def local_solves(A, cpts, nptr, nbr):
    """Solve every local system; singular ones by minimal-norm least squares.

    Returns (z float64[sum S_i], flags int8[nc]) with flag 1 where the
    least-squares fallback was taken.
    """
    rp, cj, vx = _arrays(A)
    nc = cpts.shape[0]
    z = np.zeros(max(int(nptr[-1]), 1), dtype=np.float64)
    flag = np.zeros(max(nc, 1), dtype=np.int8)
    nb = np.ascontiguousarray(nbr if nbr.shape[0] else np.zeros(1, np.int32),
                              dtype=np.int32)
    st = lib().orc_local_solves(_p(rp), _p(cj), _p(vx), nc,
                                _p(np.ascontiguousarray(cpts, np.int32)),
                                _p(np.ascontiguousarray(nptr, np.int64)),
                                _p(nb), _p(z), _p(flag))
    if st != 0:
        raise MemoryError("local_solves")
    flag = flag[:nc]
    for c in np.flatnonzero(flag):
        nbc = nbr[nptr[c]:nptr[c + 1]]
        M, f = local_system(A, int(cpts[c]), nbc)
        z[nptr[c]:nptr[c + 1]] = np.linalg.lstsq(M, f, rcond=None)[0]
    return z[:nptr[-1]], flag


def restriction(n, cpts, nptr, nbr, z):
    """R = [Z I]: row c holds z on N_c and 1 at the C-point, sorted columns."""
    nc = cpts.shape[0]
    rows = np.concatenate([np.repeat(np.arange(nc), np.diff(nptr)),
                           np.arange(nc)])
    cols = np.concatenate([nbr.astype(np.int64), cpts.astype(np.int64)])
    vals = np.concatenate([z, np.ones(nc)])
    order = np.lexsort((cols, rows))
    rowptr = np.zeros(nc + 1, dtype=np.int32)
    np.cumsum(np.bincount(rows, minlength=nc), out=rowptr[1:])
    return csr(rowptr, cols[order], vals[order], shape=(nc, n))


def interp_one_point(A, smask, cf):
    rp, cj, vx = _arrays(A)
    cidx, cpts = coarse_index(cf)
    n = A.shape[0]
    pcol = np.zeros(n, dtype=np.int32)
    lib().orc_interp_one_point(n, _p(rp), _p(cj), _p(vx),
                               _p(np.ascontiguousarray(smask, np.uint8)),
                               _p(np.ascontiguousarray(cf, np.int8)),
                               _p(cidx), _p(pcol))
    has = pcol >= 0
    rowptr = np.zeros(n + 1, dtype=np.int32)
    np.cumsum(has, out=rowptr[1:])
    return csr(rowptr, pcol[has], np.ones(int(has.sum())),
               shape=(n, cpts.shape[0]))


def interp_direct(A, smask, cf):
    rp, cj, vx = _arrays(A)
    cidx, cpts = coarse_index(cf)
    n = A.shape[0]
    L = lib()
    args = (n, _p(rp), _p(cj), _p(vx),
            _p(np.ascontiguousarray(smask, np.uint8)),
            _p(np.ascontiguousarray(cf, np.int8)), _p(cidx))
    pptr = np.zeros(n + 1, dtype=np.int64)
    dummy_i = np.zeros(1, np.int32)
    dummy_d = np.zeros(1, np.float64)
    L.orc_interp_direct(*args, 0, _p(pptr), _p(dummy_i), _p(dummy_d))
    np.cumsum(pptr, out=pptr)
    nnz = int(pptr[-1])
    pcol = np.zeros(max(nnz, 1), np.int32)
    pval = np.zeros(max(nnz, 1), np.float64)
    L.orc_interp_direct(*args, 1, _p(pptr), _p(pcol), _p(pval))
    return csr(pptr.astype(np.int32), pcol[:nnz], pval[:nnz],
               shape=(n, cpts.shape[0]))


def spgemm(A, B):
    """C = A B with the symbolic pattern (no value-based dropping)."""
    m = A.shape[0]
    nb = B.shape[1]
    ap = np.ascontiguousarray(A.indptr, np.int64)
    aj = np.ascontiguousarray(A.indices, np.int32)
    ax = np.ascontiguousarray(A.data, np.float64)
    bp = np.ascontiguousarray(B.indptr, np.int64)
    bj = np.ascontiguousarray(B.indices, np.int32)
    bx = np.ascontiguousarray(B.data, np.float64)
    if aj.shape[0] == 0:
        aj = np.zeros(1, np.int32); ax = np.zeros(1)
    if bj.shape[0] == 0:
        bj = np.zeros(1, np.int32); bx = np.zeros(1)
    cnt = np.zeros(m, np.int64)
    L = lib()
    L.orc_spgemm_count(m, nb, _p(ap), _p(aj), _p(bp), _p(bj), _p(cnt))
    cp = np.zeros(m + 1, np.int64)
    np.cumsum(cnt, out=cp[1:])
    nnz = int(cp[-1])
    cj = np.zeros(max(nnz, 1), np.int32)
    cx = np.zeros(max(nnz, 1), np.float64)
    L.orc_spgemm_fill(m, nb, _p(ap), _p(aj), _p(ax), _p(bp), _p(bj), _p(bx),
                      _p(cp), _p(cj), _p(cx))
    return csr(cp.astype(np.int32), cj[:nnz], cx[:nnz], shape=(m, nb))


def galerkin(R, A, P):
    """K = R (A P), symbolic pattern."""
    return spgemm(R, spgemm(A, P))


def block_scale(A, b, k):
    """D_B^{-1} A and D_B^{-1} b for the k x k diagonal blocks (Sec. 4.2.1).

    Each block row is multiplied by the inverse of its diagonal block; the
    product keeps the symbolic pattern, so every row of a block carries the
    union of that block row's columns.  The diagonal blocks of D_B^{-1} A
    are the identity by definition; they are stored as exact ones and zeros
    instead of the rounded products, whose noise (about 1e-17) would
    otherwise decide the strength of connection in rows without other
    couplings.
    """
    n = A.shape[0]
    assert n % k == 0
    nb = n // k
    D = np.zeros((nb, k, k))
    Ac = A.tocoo()
    r, c = Ac.row, Ac.col
    inblk = (r // k) == (c // k)
    D[r[inblk] // k, r[inblk] % k, c[inblk] % k] = Ac.data[inblk]
    Dinv = np.linalg.inv(D)
    rowptr = np.arange(0, n * k + 1, k, dtype=np.int32)
    col = (np.repeat(np.arange(nb) * k, k * k) +
           np.tile(np.arange(k), nb * k)).astype(np.int32)
    Bd = csr(rowptr, col, Dinv.reshape(-1), shape=(n, n))
    bs = np.einsum("eij,ej->ei", Dinv, np.asarray(b).reshape(nb, k)).ravel()
    S = spgemm(Bd, A)
    rows = np.repeat(np.arange(n), np.diff(S.indptr))
    inb = (rows // k) == (S.indices // k)
    S.data[inb] = np.where(S.indices[inb] == rows[inb], 1.0, 0.0)
    return S, bs


# --------------------------------------------------------------------------
# Nodal (block) treatment: every step taken on the k x k blocks of A
# (Sec. 3.1, block form of Eq. (system); Sec. 4.2, treatment (iii)).  A is
# held as a scalar CSR matrix whose stored blocks are dense: the k rows of a
# node store the same columns, in whole groups of k.
# --------------------------------------------------------------------------

def node_graph(A, k):
    """The graph of blocks: node CSR (rowptr, col) and, per stored block,
    its squared Frobenius norm summed row by row then column by column
    (a fixed order, so that a comparison of two norms is reproducible).
    Checks that every stored block is dense."""
    A = A.tocsr()
    n = A.shape[0]
    assert n % k == 0
    nn = n // k
    rp, cj, vx = A.indptr, A.indices, A.data
    nrp = np.zeros(nn + 1, dtype=np.int64)
    ncol, nsq = [], []
    for i in range(nn):
        r0 = i * k
        len0 = rp[r0 + 1] - rp[r0]
        if len0 % k:
            raise ValueError("node %d: a row does not store whole blocks" % i)
        cols0 = cj[rp[r0]:rp[r0 + 1]]
        for a in range(k):
            ca = cj[rp[r0 + a]:rp[r0 + a + 1]]
            if ca.shape[0] != len0 or np.any(ca != cols0):
                raise ValueError("node %d: its rows store different columns" % i)
        g = cols0.reshape(-1, k)
        if np.any(g[:, 0] % k) or np.any(g - g[:, :1] != np.arange(k)):
            raise ValueError("node %d: a stored block is not dense" % i)
        for t in range(g.shape[0]):
            acc = 0.0
            for a in range(k):
                base = rp[r0 + a] + t * k
                for u in range(k):
                    acc = acc + vx[base + u] * vx[base + u]
            ncol.append(g[t, 0] // k)
            nsq.append(acc)
        nrp[i + 1] = nrp[i] + g.shape[0]
    return nrp, np.array(ncol, dtype=np.int32), np.array(nsq, dtype=np.float64)


def node_strength(nrp, ncol, nsq, theta=0.25):
    """Strong blocks: ||A_ij||_F >= theta max_{l != i} ||A_il||_F, taken on
    squared norms (||A_ij||^2 >= theta^2 max ||A_il||^2); a zero block or a
    node without off-diagonal blocks has no strong connection.  uint8 per
    stored block."""
    nn = nrp.shape[0] - 1
    th2 = theta * theta
    sm = np.zeros(ncol.shape[0], dtype=np.uint8)
    for i in range(nn):
        lo, hi = nrp[i], nrp[i + 1]
        off = ncol[lo:hi] != i
        if not off.any():
            continue
        m = nsq[lo:hi][off].max()
        if m <= 0.0:
            continue
        cut = th2 * m
        for p in range(lo, hi):
            if ncol[p] != i and nsq[p] > 0.0 and nsq[p] >= cut:
                sm[p] = 1
    return sm


def node_entry_mask(A, k, nrp, nsm):
    """The strength mask over A's stored entries: every entry of a strong
    block (uint8 per entry)."""
    sm = np.zeros(A.nnz, dtype=np.uint8)
    for i in range(nrp.shape[0] - 1):
        for a in range(k):
            lo = A.indptr[i * k + a]
            for t, p in enumerate(range(nrp[i], nrp[i + 1])):
                if nsm[p]:
                    sm[lo + t * k:lo + (t + 1) * k] = 1
    return sm


def expand_nodes(x_node, k):
    """A per-node array repeated for each of the node's k rows."""
    return np.repeat(np.asarray(x_node), k)


def node_neighbourhoods(nrp, ncol, nsm, cf_node, k, distance=1):
    """N_i of every C-node on the graph of blocks: its strong F-neighbour
    nodes, and at distance two also theirs (F-F-C paths only, Sec. 4),
    given per C-row: every row of C-node i gets the k rows of each node of
    N_i, ascending.  Returns (cpts, nptr, nbr) over the rows of A."""
    nn = nrp.shape[0] - 1

    def strong_f(i):
        return [int(ncol[p]) for p in range(nrp[i], nrp[i + 1])
                if ncol[p] != i and nsm[p] and cf_node[ncol[p]] == 0]
    rows, lists = [], []
    for i in range(nn):
        if cf_node[i] != 1:
            continue
        nb = set(strong_f(i))
        if distance == 2:
            for j in list(nb):
                nb.update(strong_f(j))
        dof = (np.repeat(np.array(sorted(nb), dtype=np.int64), k) * k +
               np.tile(np.arange(k), len(nb))).astype(np.int32)
        for a in range(k):
            rows.append(i * k + a)
            lists.append(dof)
    cpts = np.array(rows, dtype=np.int32)
    nptr = np.zeros(len(lists) + 1, dtype=np.int64)
    np.cumsum([l.shape[0] for l in lists], out=nptr[1:])
    nbr = np.concatenate(lists).astype(np.int32) if lists else np.zeros(0, np.int32)
    return cpts, nptr, nbr


def node_local_solves(A, k, cpts, nptr, nbr):
    """Block form of Eq. (system): for C-node i with neighbour rows N,
    A(N,N)^T Y = -A(i-rows, N)^T with k right-hand sides, one per row of the
    node; row a of the block row Z_i is column a of Y.  A singular system
    (a pivot of its LU with |u_kk| <= 1e-14 ||M||_inf) is solved for each
    right-hand side in the minimal-norm least-squares sense.  Returns
    (z over nbr, flags per C-row)."""
    A = A.tocsr()
    z = np.zeros(int(nptr[-1]), dtype=np.float64)
    flags = np.zeros(cpts.shape[0], dtype=np.int8)
    for q0 in range(0, cpts.shape[0], k):
        nb = nbr[nptr[q0]:nptr[q0 + 1]]
        if nb.shape[0] == 0:
            continue
        node_rows = cpts[q0:q0 + k]
        M = A[nb][:, nb].toarray().T
        F = -A[node_rows][:, nb].toarray().T           # (kS) x k
        lu, piv = sla.lu_factor(M, check_finite=False)
        if np.any(np.abs(np.diag(lu)) <= 1e-14 * np.abs(M).sum(axis=1).max()):
            Y = np.linalg.lstsq(M, F, rcond=None)[0]
            flags[q0:q0 + k] = 1
        else:
            Y = sla.lu_solve((lu, piv), F)
        for a in range(k):
            z[nptr[q0 + a]:nptr[q0 + a + 1]] = Y[:, a]
    return z, flags


def node_interp_one_point(nrp, ncol, nsq, nsm, cf_node, k):
    """One-point interpolation by block (Sec. 4.2): an F-node takes the
    identity block from its strong C-neighbour node with the largest block
    norm (the first in column order on a tie); a C-node injects; an F-node
    without a strong C-neighbour gets zero rows."""
    nn = nrp.shape[0] - 1
    cidx_n, cnodes = coarse_index(cf_node)
    pick = np.full(nn, -1, dtype=np.int64)
    for i in range(nn):
        if cf_node[i] == 1:
            pick[i] = cidx_n[i]
            continue
        best, bv = -1, -1.0
        for p in range(nrp[i], nrp[i + 1]):
            j = ncol[p]
            if j == i or not nsm[p] or cf_node[j] != 1:
                continue
            if nsq[p] > bv:
                bv, best = nsq[p], j
        pick[i] = cidx_n[best] if best >= 0 else -1
    n = nn * k
    pcol = np.full(n, -1, dtype=np.int64)
    for i in range(nn):
        if pick[i] >= 0:
            pcol[i * k:(i + 1) * k] = pick[i] * k + np.arange(k)
    has = pcol >= 0
    rowptr = np.zeros(n + 1, dtype=np.int32)
    np.cumsum(has, out=rowptr[1:])
    return csr(rowptr, pcol[has].astype(np.int32), np.ones(int(has.sum())),
               shape=(n, cnodes.shape[0] * k))


def diag_blocks(A, k):
    """The k x k diagonal blocks of A, shape (n/k, k, k)."""
    n = A.shape[0]
    Ac = A.tocoo()
    D = np.zeros((n // k, k, k))
    inb = (Ac.row // k) == (Ac.col // k)
    D[Ac.row[inb] // k, Ac.row[inb] % k, Ac.col[inb] % k] = Ac.data[inb]
    return D


# --------------------------------------------------------------------------
# Hierarchy
# --------------------------------------------------------------------------

class Level:
    pass


class Hierarchy:
    def __init__(self):
        self.levels = []
        self.coarse_lu = None

    @property
    def nlevels(self):
        return len(self.levels)

    def op_complexity(self):
        return sum(l.A.nnz for l in self.levels) / self.levels[0].A.nnz

    def cycle_complexity(self):
        """Work units per V-cycle; one WU = one SpMV with A_0 (2 nnz flops)."""
        wu = 2.0 * self.levels[0].A.nnz
        flops = 0.0
        for l in self.levels[:-1]:
            nf = l.A.indptr[1:] - l.A.indptr[:-1]
            nnz_f = float(nf[l.cf == 0].sum())
            nnz_c = float(nf[l.cf == 1].sum())
            flops += 2.0 * l.A.nnz                    # residual
            flops += 2.0 * l.R.nnz + 2.0 * l.P.nnz    # restrict, interpolate
            flops += 2.0 * (2.0 * nnz_f + nnz_c)      # F, F, C Jacobi
        nL = self.levels[-1].A.shape[0]
        flops += 2.0 * nL * nL                        # coarsest triangular solves
        return flops / wu


def _lump_pass(K, theta_d):
    K = K.tocsr()
    rp, cj, vx = _arrays(K)
    m = K.shape[0]
    keep = np.zeros(max(cj.shape[0], 1), dtype=np.uint8)
    cnt = np.zeros(m, dtype=np.int64)
    dummy_i = np.zeros(1, np.int64)
    lib().orc_lump(m, _p(rp), _p(cj), _p(vx), float(theta_d), 0, _p(keep),
                   _p(cnt), _p(dummy_i), _p(np.zeros(1, np.int32)),
                   _p(np.zeros(1)))
    return K, rp, cj, vx, keep[:cj.shape[0]], cnt


def lump_keep(K, theta_d):
    """Entries of K that lumping keeps: the diagonal, and off-diagonal
    entries with |k_ij| >= theta_d * max_j |k_ij|, the maximum taken over
    the whole row, diagonal included (Sec. 3.3 and the caption of its
    filtering table).  Rows without a stored diagonal or without an
    off-diagonal entry are kept whole.  Boolean per stored entry."""
    return _lump_pass(K, theta_d)[4].astype(bool)


def lump(K, theta_d):
    """Sec. 3.3: each removed entry of row i is added to k_ii, so row sums
    stay.  The removed entries are summed in column order, then added."""
    K, rp, cj, vx, keep, cnt = _lump_pass(K, theta_d)
    m = K.shape[0]
    optr = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(cnt, out=optr[1:])
    nnz = int(optr[-1])
    ocj = np.zeros(max(nnz, 1), np.int32)
    ov = np.zeros(max(nnz, 1), np.float64)
    if cj.shape[0] == 0:
        keep = np.zeros(1, np.uint8)
    lib().orc_lump(m, _p(rp), _p(cj), _p(vx), float(theta_d), 1,
                   _p(np.ascontiguousarray(keep, np.uint8)), _p(cnt), _p(optr),
                   _p(ocj), _p(ov))
    return csr(optr.astype(np.int32), ocj[:nnz], ov[:nnz], shape=K.shape)


def setup(A, cf_levels=None, theta=0.25, theta_c=None, kind=SOC_ABS,
          distance=1, interp=INTERP_ONE_POINT, max_levels=25, max_coarse=128,
          stall=0.9, lump_tol=0.0, block=0, split="rs"):
    """Build the lAIR hierarchy.

    cf_levels: optional list of per-level CF splits (int8 arrays, 1 = C);
    levels beyond the list use the Ruge-Stueben first pass.
    Coarsening stops when n <= max_coarse, when max_levels is reached, when
    no C-point is found, or when n_c > stall * n.  lump_tol > 0 lumps every
    coarse operator (Sec. 3.3; level 0 is the caller's matrix).  block = k
    builds the hierarchy by k x k blocks (nodal treatment; distance one or
    two on the graph of blocks, one-point interpolation by block, SOC on
    block norms, block Jacobi).  split="pmis" takes the parallel splitting
    of pmis_split instead of the Ruge-Stueben first pass.
    """
    if theta_c is None:
        theta_c = theta
    if block:
        return _setup_nodal(A, block, cf_levels, theta, theta_c, max_levels,
                            max_coarse, stall, distance)
    H = Hierarchy()
    Al = A.tocsr()
    lvl = 0
    while True:
        L = Level()
        L.A = Al
        n = Al.shape[0]
        H.levels.append(L)
        if n <= max_coarse or lvl + 1 >= max_levels:
            break
        L.smask = strength(Al, theta, kind)
        if cf_levels is not None and lvl < len(cf_levels):
            cf = np.ascontiguousarray(cf_levels[lvl], dtype=np.int8)
        else:
            sm_c = L.smask if theta_c == theta else strength(Al, theta_c, kind)
            cf = pmis_split(Al, sm_c) if split == "pmis" else rs_split(Al, sm_c)
        nc = int((cf == 1).sum())
        if nc == 0 or nc > stall * n:
            del L.smask
            break
        L.cf = cf
        L.cidx, L.cpts = coarse_index(cf)
        cpts, L.nptr, L.nbr = neighbourhoods(Al, L.smask, cf, distance)
        L.z, L.flags = local_solves(Al, cpts, L.nptr, L.nbr)
        L.R = restriction(n, cpts, L.nptr, L.nbr, L.z)
        if interp == INTERP_ONE_POINT:
            L.P = interp_one_point(Al, L.smask, cf)
        else:
            L.P = interp_direct(Al, L.smask, cf)
        L.AP = spgemm(Al, L.P)
        Al = spgemm(L.R, L.AP)
        if lump_tol > 0.0:
            L.K_full = Al
            Al = lump(Al, lump_tol)
        lvl += 1
    last = H.levels[-1]
    last.cf = None
    H.coarse_lu = sla.lu_factor(last.A.toarray())
    H.interp = interp
    return H


def _setup_nodal(A, k, cf_levels, theta, theta_c, max_levels, max_coarse, stall, distance=1):
    H = Hierarchy()
    H.block = k
    Al = A.tocsr()
    lvl = 0
    while True:
        L = Level()
        L.A = Al
        n = Al.shape[0]
        H.levels.append(L)
        if n <= max_coarse or lvl + 1 >= max_levels:
            break
        nrp, ncol, nsq = node_graph(Al, k)
        nsm = node_strength(nrp, ncol, nsq, theta)
        if cf_levels is not None and lvl < len(cf_levels):
            cf = np.ascontiguousarray(cf_levels[lvl], dtype=np.int8)
            cf_node = cf[::k].copy()
            assert np.array_equal(expand_nodes(cf_node, k), cf)
        else:
            nsm_c = nsm if theta_c == theta else node_strength(nrp, ncol, nsq, theta_c)
            G = csr(nrp.astype(np.int32), ncol, np.ones(ncol.shape[0]),
                    shape=(n // k, n // k))
            cf_node = rs_split(G, nsm_c)
            cf = expand_nodes(cf_node, k).astype(np.int8)
        nc = int((cf == 1).sum())
        if nc == 0 or nc > stall * n:
            break
        L.cf = cf
        L.node_graph = (nrp, ncol, nsq)
        L.nsmask = nsm
        L.smask = node_entry_mask(Al, k, nrp, nsm)
        L.cidx, L.cpts = coarse_index(cf)
        cpts, L.nptr, L.nbr = node_neighbourhoods(nrp, ncol, nsm, cf_node, k, distance)
        assert np.array_equal(cpts, L.cpts)
        L.z, L.flags = node_local_solves(Al, k, cpts, L.nptr, L.nbr)
        L.R = restriction(n, cpts, L.nptr, L.nbr, L.z)
        L.P = node_interp_one_point(nrp, ncol, nsq, nsm, cf_node, k)
        L.AP = spgemm(Al, L.P)
        Al = spgemm(L.R, L.AP)
        lvl += 1
    last = H.levels[-1]
    last.cf = None
    H.coarse_lu = sla.lu_factor(last.A.toarray())
    H.interp = INTERP_ONE_POINT
    return H


def update_diag(H, d):
    """Replace the diagonal of A_0 by d and recompute every value of the
    hierarchy on its kept structure.

    The strength masks, CF splittings, neighbourhoods and the sparsity
    patterns of R, P and every A_l stay as set up.  For each level in turn
    the local systems of Eq. (system) are solved again on the same N_i, the
    interpolation weights are recomputed (direct interpolation; one-point
    weights are 1 on a kept pattern), and the next operator is the Galerkin
    product R (A P) of Sec. 2.1.  The hierarchy is modified in place.
    """
    A = H.levels[0].A.tocsr(copy=True)
    d = np.asarray(d, dtype=np.float64)
    n = A.shape[0]
    for i in range(n):
        lo, hi = A.indptr[i], A.indptr[i + 1]
        k = lo + int(np.searchsorted(A.indices[lo:hi], i))
        A.data[k] = d[i]
    for L in H.levels[:-1]:
        L.A = A
        cpts = L.cpts
        L.z, L.flags = local_solves(A, cpts, L.nptr, L.nbr)
        L.R = restriction(n, cpts, L.nptr, L.nbr, L.z)
        if H.interp == INTERP_DIRECT:
            L.P = interp_direct(A, L.smask, L.cf)
        L.AP = spgemm(A, L.P)
        A = spgemm(L.R, L.AP)
        n = A.shape[0]
    H.levels[-1].A = A
    H.coarse_lu = sla.lu_factor(A.toarray())
    return H


def _jacobi(A, diag, b, x, rows, omega=1.0):
    """One Jacobi sweep restricted to ``rows``; every row reads the old x."""
    r = b[rows] - A[rows] @ x
    y = x.copy()
    y[rows] = x[rows] + omega * r / diag[rows]
    return y


def _jacobi_block(A, D, k, b, x, rows, omega=1.0):
    """One block Jacobi sweep over the nodes whose rows are ``rows``:
    x_i + omega D_i^{-1} (b - A x)_i with D_i the node's diagonal block."""
    r = b[rows] - A[rows] @ x
    nodes = rows[::k] // k
    c = np.linalg.solve(D[nodes], r.reshape(-1, k, 1)).reshape(-1)
    y = x.copy()
    y[rows] = x[rows] + omega * c
    return y


def cycle(H, b, x, lvl=0, omega=1.0):
    """One V-cycle: coarse-grid correction, then F, F, C Jacobi sweeps
    (block Jacobi on the nodes for a nodal hierarchy)."""
    L = H.levels[lvl]
    if lvl == H.nlevels - 1:
        return sla.lu_solve(H.coarse_lu, b)
    A = L.A
    r = b - A @ x
    bc = L.R @ r
    xc = cycle(H, bc, np.zeros(bc.shape[0]), lvl + 1, omega)
    x = x + L.P @ xc
    F = np.flatnonzero(L.cf == 0)
    C = np.flatnonzero(L.cf == 1)
    k = getattr(H, "block", 0)
    if k:
        D = diag_blocks(A, k)
        x = _jacobi_block(A, D, k, b, x, F, omega)
        x = _jacobi_block(A, D, k, b, x, F, omega)
        x = _jacobi_block(A, D, k, b, x, C, omega)
        return x
    diag = A.diagonal()
    x = _jacobi(A, diag, b, x, F, omega)
    x = _jacobi(A, diag, b, x, F, omega)
    x = _jacobi(A, diag, b, x, C, omega)
    return x


def solve(H, b, x0=None, rtol=1e-10, maxit=200, omega=1.0):
    """Stationary V-cycle iteration until ||b - A x|| <= rtol ||b||.

    Returns (x, iterations, residual-norm history).
    """
    A = H.levels[0].A
    x = np.zeros_like(b) if x0 is None else x0.copy()
    nb = np.linalg.norm(b)
    hist = [np.linalg.norm(b - A @ x)]
    it = 0
    while hist[-1] > rtol * nb and it < maxit:
        x = cycle(H, b, x, 0, omega)
        it += 1
        hist.append(np.linalg.norm(b - A @ x))
    return x, it, np.array(hist)


# --------------------------------------------------------------------------
# Adjoint: the exact transpose of the V-cycle map x <- x + B (b - A x).
# B^T applies, per level, Jacobi C, F, F on A^T (same diagonal), restricts
# with P^T, recurses on K^T and interpolates with R^T.
# --------------------------------------------------------------------------

def cycle_transpose(H, g, lam, lvl=0, omega=1.0):
    L = H.levels[lvl]
    if lvl == H.nlevels - 1:
        return sla.lu_solve(H.coarse_lu, g, trans=1)
    At = L.A.T.tocsr()
    diag = L.A.diagonal()
    F = np.flatnonzero(L.cf == 0)
    C = np.flatnonzero(L.cf == 1)
    lam = _jacobi(At, diag, g, lam, C, omega)
    lam = _jacobi(At, diag, g, lam, F, omega)
    lam = _jacobi(At, diag, g, lam, F, omega)
    r = g - At @ lam
    gc = L.P.T @ r
    lc = cycle_transpose(H, gc, np.zeros(gc.shape[0]), lvl + 1, omega)
    return lam + L.R.T @ lc


def solve_transpose(H, g, rtol=1e-10, maxit=200, omega=1.0):
    At = H.levels[0].A.T.tocsr()
    lam = np.zeros_like(g)
    ng = np.linalg.norm(g)
    hist = [np.linalg.norm(g - At @ lam)]
    it = 0
    while hist[-1] > rtol * ng and it < maxit:
        lam = cycle_transpose(H, g, lam, 0, omega)
        it += 1
        hist.append(np.linalg.norm(g - At @ lam))
    return lam, it, np.array(hist)


# --------------------------------------------------------------------------
# Flexible GMRES(m), right preconditioned (Saad 1993): the Krylov solver the
# paper wraps its cycles in.  Arnoldi by classical Gram-Schmidt applied
# twice, the small least-squares problem by Givens rotations.
# --------------------------------------------------------------------------

def fgmres(A, b, precond, x0=None, rtol=1e-10, maxit=200, restart=20):
    """Solve A x = b; precond(v) returns an approximation of A^{-1} v.

    One iteration is one Arnoldi step (one preconditioner application).
    Stops when the residual estimate |g_{j+1}| <= rtol ||b|| or after maxit
    steps; after each cycle of at most ``restart`` steps the true residual
    decides whether to restart.  Returns (x, iterations, history of true
    residual norms at the restarts, estimates at every step).
    """
    n = b.shape[0]
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=float)
    nb = np.linalg.norm(b)
    tol = rtol * nb
    r = b - A @ x
    beta = np.linalg.norm(r)
    hist = [beta]
    est = [beta]
    it = 0
    while beta > tol and it < maxit:
        m = restart
        V = np.zeros((n, m + 1))
        Z = np.zeros((n, m))
        Hh = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        V[:, 0] = r / beta
        k = 0
        for j in range(m):
            Z[:, j] = precond(V[:, j])
            w = A @ Z[:, j]
            h = np.zeros(j + 1)
            for _ in range(2):                      # Gram-Schmidt, twice
                c = V[:, :j + 1].T @ w
                w = w - V[:, :j + 1] @ c
                h += c
            hn = np.linalg.norm(w)
            Hh[:j + 1, j] = h
            Hh[j + 1, j] = hn
            V[:, j + 1] = w / hn if hn > 0 else 0.0
            for i in range(j):                      # earlier rotations
                t = cs[i] * Hh[i, j] + sn[i] * Hh[i + 1, j]
                Hh[i + 1, j] = -sn[i] * Hh[i, j] + cs[i] * Hh[i + 1, j]
                Hh[i, j] = t
            d = math.hypot(Hh[j, j], Hh[j + 1, j])
            cs[j], sn[j] = (Hh[j, j] / d, Hh[j + 1, j] / d) if d > 0 else (1.0, 0.0)
            Hh[j, j] = d
            Hh[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            it += 1
            k = j + 1
            est.append(abs(g[j + 1]))
            if abs(g[j + 1]) <= tol or it >= maxit:
                break
        y = sla.solve_triangular(Hh[:k, :k], g[:k])
        x = x + Z[:, :k] @ y
        r = b - A @ x
        beta = np.linalg.norm(r)
        hist.append(beta)
    return x, it, np.array(hist), np.array(est)


def fgmres_cycle(H, b, x0=None, rtol=1e-10, maxit=200, restart=20, omega=1.0):
    """FGMRES(m) on level 0 with one V-cycle from zero as the preconditioner."""
    A = H.levels[0].A
    return fgmres(A, b, lambda v: cycle(H, v, np.zeros_like(v), 0, omega), x0, rtol,
                  maxit, restart)


def convergence_factor(hist):
    """Geometric mean residual reduction per iteration."""
    k = len(hist) - 1
    if k <= 0 or hist[0] == 0:
        return 0.0
    return float((hist[-1] / hist[0]) ** (1.0 / k))
