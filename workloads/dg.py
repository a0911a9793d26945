"""Upwind discontinuous Galerkin (P2 on triangles) for steady advection.

Discretises  b . grad u = f  on (0,1)^2 with u = g on the inflow boundary
(b . n < 0), using the conservative upwind DG form for a divergence-free b:

    sum_K [ -int_K u (b . grad v) + int_{dK} (b . n_K) u_hat v ] = int f v

with the pointwise upwind trace u_hat (own trace where b . n_K >= 0, the
neighbour's trace where b . n_K < 0, g on inflow boundary edges, moved to
the right-hand side).  The face integral is evaluated with 3-point
Gauss-Legendre per edge and upwinding is decided per quadrature point.

Mesh: m x m squares on (0,1)^2, each cut by its SW-NE diagonal into two
counter-clockwise triangles (SW, SE, NE) and (SW, NE, NW); interior vertices
are jittered by U[-jitter h, jitter h]^2 (seeded), boundary vertices stay.
DoFs are element-contiguous: 6 per triangle, the 3 vertices then the
midpoints of edges (0,1), (1,2), (2,0).  Element t of square (ix, iy) is
2 (iy m + ix) + {0, 1}.

With f = 0, g = 1 and div b = 0 the discrete solution is exactly u = 1
(constants are reproduced), which the tests use as a check of the assembly.
"""
import numpy as np
import scipy.sparse as sp

# Symmetric 6-point degree-4 rule on the triangle (Dunavant 1985):
# barycentric points and weights normalised to sum to 1.
_A1, _B1, _W1 = 0.108103018168070, 0.445948490915965, 0.223381589678011
_A2, _B2, _W2 = 0.816847572980459, 0.091576213509771, 0.109951743655322
TRI_Q = np.array([[_A1, _B1, _B1], [_B1, _A1, _B1], [_B1, _B1, _A1],
                  [_A2, _B2, _B2], [_B2, _A2, _B2], [_B2, _B2, _A2]])
TRI_W = np.array([_W1] * 3 + [_W2] * 3)
# 3-point Gauss-Legendre on [0, 1].
_g = 0.5 * np.sqrt(3.0 / 5.0)
EDGE_S = np.array([0.5 - _g, 0.5, 0.5 + _g])
EDGE_W = np.array([5.0, 8.0, 5.0]) / 18.0

_EDGES = ((0, 1), (1, 2), (2, 0))


def _p2_values(lam):
    """P2 Lagrange basis at barycentric points lam[..., 3] -> [..., 6]."""
    l0, l1, l2 = lam[..., 0], lam[..., 1], lam[..., 2]
    return np.stack([l0 * (2 * l0 - 1), l1 * (2 * l1 - 1), l2 * (2 * l2 - 1),
                     4 * l0 * l1, 4 * l1 * l2, 4 * l2 * l0], axis=-1)


def _p2_grads(lam, glam):
    """Gradients of the P2 basis.

    lam: [Q, 3] barycentrics; glam: [E, 3, 2] gradients of the barycentric
    coordinates per element.  Returns [E, Q, 6, 2].
    """
    L = lam[None, :, :, None]               # [1, Q, 3, 1]
    G = glam[:, None, :, :]                 # [E, 1, 3, 2]
    gv = (4.0 * L - 1.0) * G                # vertex functions
    mids = []
    for a, b in _EDGES:
        mids.append(4.0 * (L[:, :, a] * G[:, :, b] + L[:, :, b] * G[:, :, a]))
    gm = np.stack(mids, axis=2)
    return np.concatenate([gv, gm], axis=2)


def jittered_mesh(m, jitter=0.2, seed=2):
    h = 1.0 / m
    iy, ix = np.meshgrid(np.arange(m + 1), np.arange(m + 1), indexing="ij")
    xy = np.stack([ix.ravel() * h, iy.ravel() * h], axis=1).astype(np.float64)
    rng = np.random.default_rng(seed)
    d = rng.uniform(-jitter * h, jitter * h, size=xy.shape)
    interior = ((ix.ravel() > 0) & (ix.ravel() < m) &
                (iy.ravel() > 0) & (iy.ravel() < m))
    xy[interior] += d[interior]
    sq_y, sq_x = np.meshgrid(np.arange(m), np.arange(m), indexing="ij")
    sw = (sq_y * (m + 1) + sq_x).ravel()
    se, nw = sw + 1, sw + (m + 1)
    ne = nw + 1
    tri = np.empty((2 * m * m, 3), dtype=np.int64)
    tri[0::2] = np.stack([sw, se, ne], axis=1)
    tri[1::2] = np.stack([sw, ne, nw], axis=1)
    return xy, tri


def upwind_dg_p2(m=256, velocity=None, g=1.0, jitter=0.2, seed=2):
    """Assemble the P2 upwind DG advection system on an m x m mesh.

    ``velocity(x, y) -> (bx, by)`` must be divergence free; the default is
    the recirculating field b = (-y + 0.5, x - 0.5).
    """
    if velocity is None:
        def velocity(x, y):
            return -y + 0.5, x - 0.5
    xy, tri = jittered_mesh(m, jitter, seed)
    ne = tri.shape[0]
    n = 6 * ne
    P = xy[tri]                                     # [E, 3, 2]
    J = np.stack([P[:, 1] - P[:, 0], P[:, 2] - P[:, 0]], axis=2)  # cols
    det = J[:, 0, 0] * J[:, 1, 1] - J[:, 0, 1] * J[:, 1, 0]
    assert np.all(det > 0), "mesh has inverted triangles"
    area = 0.5 * det
    # grad lambda_1, lambda_2 are the rows of J^{-1}.
    inv = np.empty_like(J)
    inv[:, 0, 0] = J[:, 1, 1] / det
    inv[:, 0, 1] = -J[:, 0, 1] / det
    inv[:, 1, 0] = -J[:, 1, 0] / det
    inv[:, 1, 1] = J[:, 0, 0] / det
    glam = np.empty((ne, 3, 2))
    glam[:, 1] = inv[:, 0]
    glam[:, 2] = inv[:, 1]
    glam[:, 0] = -glam[:, 1] - glam[:, 2]

    # ---- volume term  -int_K phi_j (b . grad phi_i) ----
    xq = np.einsum("qa,eak->eqk", TRI_Q, P)         # [E, Q, 2]
    bx, by = velocity(xq[..., 0], xq[..., 1])
    phi = _p2_values(TRI_Q)                         # [Q, 6]
    gphi = _p2_grads(TRI_Q, glam)                   # [E, Q, 6, 2]
    bgrad = gphi[..., 0] * bx[..., None] + gphi[..., 1] * by[..., None]
    vol = -np.einsum("q,e,eqi,qj->eij", TRI_W, area, bgrad, phi)
    base = 6 * np.arange(ne)
    li, lj = np.meshgrid(np.arange(6), np.arange(6), indexing="ij")
    rows = [(base[:, None, None] + li[None]).ravel()]
    cols = [(base[:, None, None] + lj[None]).ravel()]
    vals = [vol.ravel()]
    rhs = np.zeros(n)

    # ---- faces ----
    occ_t = np.repeat(np.arange(ne), 3)
    occ_e = np.tile(np.arange(3), ne)
    va = tri[occ_t, [_EDGES[e][0] for e in occ_e]]
    vb = tri[occ_t, [_EDGES[e][1] for e in occ_e]]
    key = np.minimum(va, vb) * (xy.shape[0]) + np.maximum(va, vb)
    order = np.argsort(key, kind="stable")
    ks = key[order]
    first = np.ones(ks.shape[0], dtype=bool)
    first[1:] = ks[1:] != ks[:-1]
    grp = np.cumsum(first) - 1
    counts = np.bincount(grp)
    assert counts.max() <= 2
    nbr = -np.ones(occ_t.shape[0], dtype=np.int64)   # partner occurrence
    pair_start = np.flatnonzero(first)
    two = counts == 2
    o1 = order[pair_start[two]]
    o2 = order[pair_start[two] + 1]
    nbr[o1] = o2
    nbr[o2] = o1

    # Edge DoF local indices in orientation (a -> b): vertex a, vertex b, mid.
    def edge_dofs(t, e):
        a = np.array([_EDGES[k][0] for k in e])
        b = np.array([_EDGES[k][1] for k in e])
        return np.stack([6 * t + a, 6 * t + b, 6 * t + 3 + e], axis=1)

    def edge_phi(s):
        """Basis values of (vertex a, vertex b, mid) at parameter s."""
        la, lb = 1.0 - s, s
        return np.stack([la * (2 * la - 1), lb * (2 * lb - 1), 4 * la * lb],
                        axis=-1)

    pa, pb = xy[va], xy[vb]
    d = pb - pa
    length = np.sqrt((d ** 2).sum(axis=1))
    nrm = np.stack([d[:, 1], -d[:, 0]], axis=1) / length[:, None]
    cen = P[occ_t].mean(axis=1)
    mid = 0.5 * (pa + pb)
    assert np.all(((mid - cen) * nrm).sum(axis=1) > 0)
    dofs = edge_dofs(occ_t, occ_e)                  # [O, 3]
    # physical quadrature points along a -> b
    xq = pa[:, None, :] + EDGE_S[None, :, None] * d[:, None, :]   # [O, 3, 2]
    bqx, bqy = velocity(xq[..., 0], xq[..., 1])
    bn = bqx * nrm[:, None, 0] + bqy * nrm[:, None, 1]             # [O, 3]
    wq = EDGE_W[None, :] * length[:, None]                         # [O, 3]
    ph = edge_phi(EDGE_S)                                          # [3q, 3]
    # Own-trace outflow part:  (b.n)+ phi_j phi_i on this element.
    outw = wq * np.maximum(bn, 0.0)
    own = np.einsum("oq,qi,qj->oij", outw, ph, ph)
    rows.append(np.repeat(dofs, 3, axis=1).ravel())
    cols.append(np.tile(dofs, (1, 3)).ravel())
    vals.append(own.ravel())
    # Inflow part: (b.n)- couples to the neighbour trace or to g.
    inw = wq * np.minimum(bn, 0.0)                                 # <= 0
    has = nbr >= 0
    bnd = ~has
    # boundary inflow -> rhs:  rhs_i -= (b.n) g phi_i
    rb = -g * np.einsum("oq,qi->oi", inw[bnd], ph)
    np.add.at(rhs, dofs[bnd].ravel(), rb.ravel())
    # interior inflow: neighbour trial functions in the neighbour's own
    # orientation; same physical point has parameter 1 - s there when the
    # neighbour runs the edge b -> a (always true for consistently oriented
    # triangles, checked below).
    oi = np.flatnonzero(has)
    on = nbr[oi]
    assert np.all(va[on] == vb[oi]) and np.all(vb[on] == va[oi])
    phn = edge_phi(1.0 - EDGE_S)                                   # [q, 3]
    cpl = np.einsum("oq,qi,qj->oij", inw[oi], ph, phn)
    nd = dofs[on]
    rows.append(np.repeat(dofs[oi], 3, axis=1).ravel())
    cols.append(np.tile(nd, (1, 3)).ravel())
    vals.append(cpl.ravel())
    # Couplings that vanish identically (edge fully outflow for this side)
    # are not stored: keep only element-face pairs with an inflow point.
    keep_last = np.repeat(np.any(inw[oi] < 0.0, axis=1), 9)
    rows[-1] = rows[-1][keep_last]
    cols[-1] = cols[-1][keep_last]
    vals[-1] = vals[-1][keep_last]

    A = sp.coo_matrix((np.concatenate(vals),
                       (np.concatenate(rows), np.concatenate(cols))),
                      shape=(n, n)).tocsr()
    A.sum_duplicates()
    A.sort_indices()
    return dict(rowptr=A.indptr.astype(np.int32),
                col=A.indices.astype(np.int32),
                val=A.data.astype(np.float64), rhs=rhs, n=n, nnz=int(A.nnz),
                block=6, nelem=ne, h=1.0 / m, xy=xy, tri=tri)


def workload_c2(m=256):
    """Recirculating pure advection, P2 upwind DG, m x m x 2 triangles."""
    w = upwind_dg_p2(m)
    w["name"] = "dg_p2_recirculating_%dx%dx2" % (m, m)
    return w


def dense_blocks(w, k=6):
    """The same system stored with whole dense k x k blocks (explicit zeros
    where a coupling block has structural zeros): the layout a nodal
    hierarchy reads."""
    A = sp.csr_matrix((w["val"], w["col"], w["rowptr"]), shape=(w["n"],) * 2)
    B = sp.bsr_matrix(A, blocksize=(k, k)).tocsr()
    B.sort_indices()
    return dict(w, rowptr=B.indptr.astype(np.int32), col=B.indices.astype(np.int32),
                val=B.data.astype(np.float64), nnz=int(B.nnz))


def workload_dg_curved(m=256):
    """Pure advection along the curved, divergence-free field
    b = (y^2, cos^2(pi x / 2)) (the advective field of the paper's DGu
    problem, Sec. 4.2, without its diffusion), P2 upwind DG on m x m x 2
    triangles, stored in dense 6 x 6 blocks.  Every streamline enters at
    x = 0 or y = 0 and leaves, so the steady problem is well posed."""
    def velocity(x, y):
        return y * y, np.cos(0.5 * np.pi * x) ** 2
    w = dense_blocks(upwind_dg_p2(m, velocity=velocity))
    w["name"] = "dg_p2_curved_%dx%dx2" % (m, m)
    return w
