"""Finite-difference advection-diffusion-reaction matrices (seeded, synthetic).

Upwind first-order finite differences on uniform grids of interior nodes with
zero Dirichlet boundary values, which drop out of every row.  Node numbering
is lexicographic with x fastest.  A coupling whose coefficient is exactly zero
(for example the downwind neighbour of a pure-advection row) is not stored.

The 2-D row for node P with diffusion eps, velocity (bx, by), reaction c is

    (4 eps/h^2 + |bx|/h + |by|/h + c) u_P - (eps/h^2 + bx+/h) u_W
      - (eps/h^2 + bx-/h) u_E - (eps/h^2 + by+/h) u_S - (eps/h^2 + by-/h) u_N

with b+ = max(b, 0) and b- = max(-b, 0); the 3-D row adds the z pair.
"""
import math

import numpy as np
import scipy.sparse as sp


def _to_csr(n, rows, cols, vals):
    m = sp.coo_matrix((vals, (rows, cols)), shape=(n, n)).tocsr()
    m.sum_duplicates()
    m.sort_indices()
    return (m.indptr.astype(np.int32), m.indices.astype(np.int32),
            m.data.astype(np.float64))


def _pack(rowptr, col, val, rhs, **meta):
    d = dict(rowptr=rowptr, col=col, val=val, rhs=rhs)
    d["n"] = int(rowptr.shape[0] - 1)
    d["nnz"] = int(col.shape[0])
    d.update(meta)
    return d


def adr_2d_csr(nx, ny, h, eps, bx, by, c=0.0):
    """5-point upwind ADR operator on an nx-by-ny interior grid (x fastest).

    ``c`` is a scalar or an array of n = nx*ny reaction values.
    """
    n = nx * ny
    k = np.arange(n, dtype=np.int64)
    i = k % nx
    j = k // nx
    e = eps / (h * h)
    bxp, bxm = max(bx, 0.0) / h, max(-bx, 0.0) / h
    byp, bym = max(by, 0.0) / h, max(-by, 0.0) / h
    diag = 4.0 * e + abs(bx) / h + abs(by) / h + np.broadcast_to(
        np.asarray(c, dtype=np.float64), (n,))
    rows = [k]
    cols = [k]
    vals = [diag.astype(np.float64)]
    for coef, mask, off in ((e + bxp, i > 0, -1), (e + bxm, i < nx - 1, +1),
                            (e + byp, j > 0, -nx), (e + bym, j < ny - 1, +nx)):
        if coef == 0.0:
            continue
        kk = k[mask]
        rows.append(kk)
        cols.append(kk + off)
        vals.append(np.full(kk.shape, -coef))
    return _to_csr(n, np.concatenate(rows), np.concatenate(cols),
                   np.concatenate(vals))


def upwind_transport_2d(m=64, theta=3.0 * math.pi / 16.0):
    """Steady pure advection b.grad u = 1 on (0,1)^2, m x m interior nodes.

    h = 1/(m+1), constant velocity (cos theta, sin theta), zero inflow values.
    The matrix is lower triangular with at most 3 entries per row.
    """
    h = 1.0 / (m + 1)
    rowptr, col, val = adr_2d_csr(m, m, h, 0.0, math.cos(theta),
                                  math.sin(theta), 0.0)
    rhs = np.ones(m * m)
    return _pack(rowptr, col, val, rhs, grid=(m, m), h=h)


def adr_2d(m, eps, phi, c, rhs=None):
    """Upwind ADR on an m x m grid, unit speed at angle phi, reaction c."""
    h = 1.0 / (m + 1)
    rowptr, col, val = adr_2d_csr(m, m, h, eps, math.cos(phi), math.sin(phi),
                                  c)
    if rhs is None:
        rhs = np.ones(m * m)
    return _pack(rowptr, col, val, rhs, grid=(m, m), h=h)


def reaction_field_2d(m, rng, modes=8):
    """c(x) = exp(0.5 xi(x)), xi a smooth Gaussian cosine series.

    xi(x, y) = sum_{p,q<modes} g_pq cos(p pi x) cos(q pi y) / (1 + p^2 + q^2)
    with g_pq ~ N(0, 1) drawn from ``rng`` in row-major (p, q) order.
    Returns (c over the m*m interior nodes, g).
    """
    g = rng.standard_normal((modes, modes))
    h = 1.0 / (m + 1)
    xs = h * np.arange(1, m + 1)
    p = np.arange(modes)
    cx = np.cos(np.pi * np.outer(xs, p))            # [m, modes]
    w = g / (1.0 + p[:, None] ** 2 + p[None, :] ** 2)
    xi = cx @ w @ cx.T                              # xi[ix, iy]
    c = np.exp(0.5 * xi.T.reshape(-1))              # x fastest
    return c, g


def implicit_euler_adr_3d(m=128, eps=1e-4, b=(1.0, 0.7, 0.4), dt=None,
                          nrhs=16, seed=5):
    """One implicit Euler step (I + dt S) of 7-point upwind 3-D ADR.

    m^3 interior nodes, h = 1/(m+1), dt = h unless given, velocity b
    normalised to unit length, c = 0.  Right-hand sides are N(0,1) stored
    n x nrhs row-major.
    """
    h = 1.0 / (m + 1)
    if dt is None:
        dt = h
    bn = math.sqrt(sum(x * x for x in b))
    b = [x / bn for x in b]
    n = m * m * m
    k = np.arange(n, dtype=np.int64)
    i = k % m
    j = (k // m) % m
    l = k // (m * m)
    e = eps / (h * h)
    diag = np.full(n, 1.0 + dt * (6.0 * e + sum(abs(x) for x in b) / h))
    rows, cols, vals = [k], [k], [diag]
    strides = (1, m, m * m)
    for ax, idx in enumerate((i, j, l)):
        bp, bm = max(b[ax], 0.0) / h, max(-b[ax], 0.0) / h
        for coef, mask, off in ((e + bp, idx > 0, -strides[ax]),
                                (e + bm, idx < m - 1, strides[ax])):
            if coef == 0.0:
                continue
            kk = k[mask]
            rows.append(kk)
            cols.append(kk + off)
            vals.append(np.full(kk.shape, -dt * coef))
    rowptr, col, val = _to_csr(n, np.concatenate(rows), np.concatenate(cols),
                               np.concatenate(vals))
    rng = np.random.default_rng(seed)
    rhs = rng.standard_normal((n, nrhs)) if nrhs > 1 else rng.standard_normal(n)
    return _pack(rowptr, col, val, rhs, grid=(m, m, m), h=h, dt=dt,
                 velocity=tuple(b), eps=eps)


def chain_1d(n):
    """1-D upwind chain: a_ii = 1, a_{i,i-1} = -1."""
    k = np.arange(n, dtype=np.int64)
    rows = np.concatenate([k, k[1:]])
    cols = np.concatenate([k, k[1:] - 1])
    vals = np.concatenate([np.ones(n), -np.ones(n - 1)])
    rowptr, col, val = _to_csr(n, rows, cols, vals)
    return _pack(rowptr, col, val, np.ones(n))


def random_ff_digraph(n, deg, seed, dominance=2.0, symmetric_pattern=False):
    """Small random sparse matrix with a diagonally dominant diagonal.

    Each row gets ``deg`` distinct random off-diagonal columns with values
    in -U[0.1, 1]; the diagonal is dominance * (row abs sum) + 0.1.
    """
    rng = np.random.default_rng(seed)
    rows, cols, vals = [], [], []
    for r in range(n):
        others = np.setdiff1d(np.arange(n), [r])
        cs = rng.choice(others, size=min(deg, n - 1), replace=False)
        vs = -rng.uniform(0.1, 1.0, size=cs.shape[0])
        rows += [r] * len(cs)
        cols += list(cs)
        vals += list(vs)
    rows, cols, vals = map(np.asarray, (rows, cols, vals))
    if symmetric_pattern:
        rows, cols = np.concatenate([rows, cols]), np.concatenate([cols, rows])
        vals = np.concatenate([vals, vals])
    off = sp.coo_matrix((vals, (rows, cols)), shape=(n, n)).tocsr()
    off.sum_duplicates()
    d = dominance * np.asarray(abs(off).sum(axis=1)).ravel() + 0.1
    m = (off + sp.diags(d)).tocsr()
    m.sort_indices()
    return _pack(m.indptr.astype(np.int32), m.indices.astype(np.int32),
                 m.data.astype(np.float64), np.ones(n))


# --------------------------------------------------------------------------
# Named workloads
# --------------------------------------------------------------------------

def workload_c1(m=64):
    """Steady 2-D pure advection, 64 x 64, angle 3 pi/16, rhs = 1."""
    w = upwind_transport_2d(m)
    w["name"] = "steady_upwind_transport_%dx%d" % (m, m)
    return w


def workload_c4(m=64, eps=1e-3, seed=4):
    """C1 grid with eps = 1e-3 diffusion and reaction exp(0.5 xi)."""
    rng = np.random.default_rng(seed)
    c, g = reaction_field_2d(m, rng)
    x_obs = rng.standard_normal(m * m)
    theta = 3.0 * math.pi / 16.0
    h = 1.0 / (m + 1)
    rowptr0, col0, val0 = adr_2d_csr(m, m, h, eps, math.cos(theta),
                                     math.sin(theta), 0.0)
    w = _pack(rowptr0, col0, val0, np.ones(m * m), grid=(m, m), h=h, eps=eps)
    w["c"] = c
    w["g"] = g
    w["x_obs"] = x_obs
    w["name"] = "adjoint_adr_%dx%d" % (m, m)
    return w


def workload_c5(m=128, nrhs=16):
    """One implicit Euler step of 3-D ADR on an m^3 grid, nrhs right sides."""
    w = implicit_euler_adr_3d(m=m, nrhs=nrhs)
    w["name"] = "implicit_euler_adr3d_%d^3_x%d" % (m, nrhs)
    return w


def adr_batch(nsys=512, nmin=32, nmax=320, seed=3):
    """Batch of 2-D ADR systems of uneven size (per-system draws in order).

    For each system: N = round(exp(U[ln nmin, ln nmax])), eps = 10^U[-6,0],
    c ~ U[0,1], phi ~ U[0, 2 pi), then rhs ~ N(0,1)^(N^2).
    """
    rng = np.random.default_rng(seed)
    systems = []
    for s in range(nsys):
        m = int(round(math.exp(rng.uniform(math.log(nmin), math.log(nmax)))))
        eps = 10.0 ** rng.uniform(-6.0, 0.0)
        c = rng.uniform(0.0, 1.0)
        phi = rng.uniform(0.0, 2.0 * math.pi)
        rhs = rng.standard_normal(m * m)
        w = adr_2d(m, eps, phi, c, rhs=rhs)
        w.update(eps=eps, c=c, phi=phi)
        systems.append(w)
    return systems


def block_union(systems):
    """Block-diagonal union of several CSR systems plus segment offsets."""
    offs = np.zeros(len(systems) + 1, dtype=np.int64)
    nzo = np.zeros(len(systems) + 1, dtype=np.int64)
    for s, w in enumerate(systems):
        offs[s + 1] = offs[s] + w["n"]
        nzo[s + 1] = nzo[s] + w["nnz"]
    rowptr = np.empty(offs[-1] + 1, dtype=np.int64)
    rowptr[0] = 0
    cols, vals, rhs = [], [], []
    for s, w in enumerate(systems):
        rowptr[offs[s] + 1:offs[s + 1] + 1] = w["rowptr"][1:].astype(np.int64) + nzo[s]
        cols.append(w["col"].astype(np.int64) + offs[s])
        vals.append(w["val"])
        rhs.append(w["rhs"])
    return _pack(rowptr.astype(np.int32), np.concatenate(cols).astype(np.int32),
                 np.concatenate(vals), np.concatenate(rhs), offs=offs)


def workload_c3(nsys=512, seed=3):
    systems = adr_batch(nsys=nsys, seed=seed)
    u = block_union(systems)
    u["systems"] = systems
    u["name"] = "adr_batch_%d" % nsys
    return u
