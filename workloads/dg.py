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


def _dgu_gamma(x, y):
    """Total cross section of the DGu problem (Sec. 4.2): 1e4 in the
    square (0.25, 0.75)^2, 1e-4 elsewhere."""
    inside = (x > 0.25) & (x < 0.75) & (y > 0.25) & (y < 0.75)
    return np.where(inside, 1e4, 1e-4)


def _dgu_velocity(x, y):
    return y * y, np.cos(0.5 * np.pi * x) ** 2


def diffusion_reaction_dg_p2(m, kappa, gamma, jitter=0.2, seed=2, g=1.0, penalty=20.0,
                             dirichlet=None):
    """Diffusion and reaction parts of a P2 DG discretisation on the mesh of
    upwind_dg_p2 (same m, jitter, seed, so the DoF numbering matches).

    Reaction: int_K gamma_K u v with gamma_K = gamma(centroid of K).
    Diffusion: symmetric interior penalty,
        sum_K int_K kappa grad u . grad v
      - sum_F int_F ({kappa grad u} . [v] + {kappa grad v} . [u])
      + sum_F int_F (penalty kappa / |F|) [u] . [v]
    over interior faces F and the Dirichlet faces (where the jump is the
    trace minus g, moved to the right-hand side: Nitsche's method); the
    other boundary faces carry the natural (zero flux) condition.  g is
    the Dirichlet value, a number or a function g(x, y).
    ``dirichlet(xm, ym) -> bool`` selects Dirichlet boundary faces by their
    midpoint (default: the south and west sides, y = 0 or x = 0).
    Returns (A, rhs) as a scipy CSR matrix and a vector."""
    if dirichlet is None:
        def dirichlet(xm, ym):
            return (ym < 1e-12) | (xm < 1e-12)
    xy, tri = jittered_mesh(m, jitter, seed)
    ne = tri.shape[0]
    n = 6 * ne
    P = xy[tri]
    J = np.stack([P[:, 1] - P[:, 0], P[:, 2] - P[:, 0]], axis=2)
    det = J[:, 0, 0] * J[:, 1, 1] - J[:, 0, 1] * J[:, 1, 0]
    area = 0.5 * det
    glam = np.empty((ne, 3, 2))
    glam[:, 1, 0], glam[:, 1, 1] = J[:, 1, 1] / det, -J[:, 0, 1] / det
    glam[:, 2, 0], glam[:, 2, 1] = -J[:, 1, 0] / det, J[:, 0, 0] / det
    glam[:, 0] = -glam[:, 1] - glam[:, 2]
    base = 6 * np.arange(ne)
    li, lj = np.meshgrid(np.arange(6), np.arange(6), indexing="ij")
    rows, cols, vals = [], [], []
    rhs = np.zeros(n)

    def add_blocks(ti, tj, blk):
        # blk[o, i, j]: test function i of element ti, trial j of element tj
        rows.append((6 * ti[:, None, None] + li[None]).ravel())
        cols.append((6 * tj[:, None, None] + lj[None]).ravel())
        vals.append(blk.ravel())

    # ---- volume: kappa stiffness + gamma mass ----
    phi = _p2_values(TRI_Q)                          # [Q, 6]
    gphi = _p2_grads(TRI_Q, glam)                    # [E, Q, 6, 2]
    cen = P.mean(axis=1)
    gam = gamma(cen[:, 0], cen[:, 1])
    stiff = kappa * np.einsum("q,e,eqik,eqjk->eij", TRI_W, area, gphi, gphi)
    mass = np.einsum("q,e,qi,qj->eij", TRI_W, area * gam, phi, phi)
    add_blocks(np.arange(ne), np.arange(ne), stiff + mass)

    if kappa > 0.0:
        # ---- faces ----
        occ_t = np.repeat(np.arange(ne), 3)
        occ_e = np.tile(np.arange(3), ne)
        ea = np.array([_EDGES[e][0] for e in occ_e])
        eb = np.array([_EDGES[e][1] for e in occ_e])
        va, vb = tri[occ_t, ea], tri[occ_t, eb]
        key = np.minimum(va, vb) * xy.shape[0] + np.maximum(va, vb)
        order = np.argsort(key, kind="stable")
        ks = key[order]
        first = np.ones(ks.shape[0], dtype=bool)
        first[1:] = ks[1:] != ks[:-1]
        grp = np.cumsum(first) - 1
        counts = np.bincount(grp)
        pair_start = np.flatnonzero(first)
        two = counts == 2
        o1 = order[pair_start[two]]
        o2 = order[pair_start[two] + 1]
        ob = order[pair_start[~two]]
        pa, pb = xy[va], xy[vb]
        d = pb - pa
        length = np.sqrt((d ** 2).sum(axis=1))
        nrm = np.stack([d[:, 1], -d[:, 0]], axis=1) / length[:, None]

        def face_basis(o, s):
            """Values [O, q, 6] and gradients [O, q, 6, 2] of the basis of
            occurrence o's element at parameter s along its edge a -> b."""
            nq = s.shape[0]
            lam = np.zeros((o.shape[0], nq, 3))
            lam[np.arange(o.shape[0])[:, None], np.arange(nq)[None], ea[o][:, None]] = 1.0 - s
            lam[np.arange(o.shape[0])[:, None], np.arange(nq)[None], eb[o][:, None]] = s
            val = _p2_values(lam)
            Lm = lam[..., None]                      # [O, q, 3, 1]
            G = glam[occ_t[o]][:, None]              # [O, 1, 3, 2]
            gv = (4.0 * Lm - 1.0) * G
            mids = [4.0 * (Lm[:, :, a] * G[:, :, b] + Lm[:, :, b] * G[:, :, a])
                    for a, b in _EDGES]
            grad = np.concatenate([gv, np.stack(mids, axis=2)], axis=2)
            return val, grad

        # interior faces: o1 runs a -> b, o2 the same edge b -> a
        w = EDGE_W[None, :] * length[o1][:, None]                    # [F, q]
        n1 = nrm[o1]
        v1, g1 = face_basis(o1, EDGE_S)
        v2, g2 = face_basis(o2, 1.0 - EDGE_S)
        dn1 = np.einsum("fqik,fk->fqi", g1, n1)                       # grad . n1
        dn2 = np.einsum("fqik,fk->fqi", g2, n1)
        sig = penalty * kappa / length[o1]
        t1, t2 = occ_t[o1], occ_t[o2]
        # test i, trial j; [u] = (u1 - u2) n1, {grad u} . n1 = (dn_u1 + dn_u2) / 2
        for (ti, vi, di, si), (tj, vj, dj, sj) in (
                ((t1, v1, dn1, 1.0), (t1, v1, dn1, 1.0)),
                ((t1, v1, dn1, 1.0), (t2, v2, dn2, -1.0)),
                ((t2, v2, dn2, -1.0), (t1, v1, dn1, 1.0)),
                ((t2, v2, dn2, -1.0), (t2, v2, dn2, -1.0))):
            blk = (-0.5 * kappa * si * np.einsum("fq,fqi,fqj->fij", w, vi, dj)
                   - 0.5 * kappa * sj * np.einsum("fq,fqi,fqj->fij", w, di, vj)
                   + si * sj * np.einsum("f,fq,fqi,fqj->fij", sig, w, vi, vj))
            add_blocks(ti, tj, blk)
        # Dirichlet boundary faces (Nitsche): trace u, outward normal
        mid = 0.5 * (pa[ob] + pb[ob])
        od = ob[dirichlet(mid[:, 0], mid[:, 1])]
        if od.shape[0]:
            w = EDGE_W[None, :] * length[od][:, None]
            vb_, gb_ = face_basis(od, EDGE_S)
            dnb = np.einsum("fqik,fk->fqi", gb_, nrm[od])
            sigb = penalty * kappa / length[od]
            blk = (-kappa * np.einsum("fq,fqi,fqj->fij", w, vb_, dnb)
                   - kappa * np.einsum("fq,fqi,fqj->fij", w, dnb, vb_)
                   + np.einsum("f,fq,fqi,fqj->fij", sigb, w, vb_, vb_))
            tb = occ_t[od]
            add_blocks(tb, tb, blk)
            if callable(g):
                xq = pa[od][:, None, :] + EDGE_S[None, :, None] * d[od][:, None, :]
                gq = g(xq[..., 0], xq[..., 1])                   # [F, q]
            else:
                gq = np.full(w.shape, float(g))
            rb = (-kappa * np.einsum("fq,fq,fqi->fi", w, gq, dnb)
                  + np.einsum("f,fq,fq,fqi->fi", sigb, w, gq, vb_))
            np.add.at(rhs, (6 * tb[:, None] + np.arange(6)[None]).ravel(), rb.ravel())
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(n, n)).tocsr()
    A.sum_duplicates()
    return A, rhs


def workload_dgu(m=256, kappa=1e-3, jitter=0.2, seed=2):
    """The DGu problem of Sec. 4.2: div(-kappa grad u + beta u) + gamma u = 0
    on (0,1)^2 with beta = (y^2, cos^2(pi x / 2)), gamma = 1e4 in
    (0.25, 0.75)^2 and 1e-4 elsewhere, u = 1 on the inflow sides (south and
    west), zero diffusive flux on the outflow sides (north and east).  P2
    upwind DG for the advection, symmetric interior penalty for the
    diffusion (kappa = 0: advection-reaction only), m x m x 2 jittered
    triangles, stored in dense 6 x 6 blocks."""
    adv = upwind_dg_p2(m, velocity=_dgu_velocity, g=1.0, jitter=jitter, seed=seed)
    Aa = sp.csr_matrix((adv["val"], adv["col"], adv["rowptr"]), shape=(adv["n"],) * 2)
    Ad, rd = diffusion_reaction_dg_p2(m, kappa, _dgu_gamma, jitter=jitter, seed=seed)
    A = (Aa + Ad).tocsr()
    A.sum_duplicates()
    A.sort_indices()
    w = dict(adv, rowptr=A.indptr.astype(np.int32), col=A.indices.astype(np.int32),
             val=A.data.astype(np.float64), nnz=int(A.nnz), rhs=adv["rhs"] + rd,
             kappa=kappa)
    w = dense_blocks(w)
    w["name"] = "dgu_p2_%dx%dx2_kappa%g" % (m, m, kappa)
    return w
