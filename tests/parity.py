"""Helpers for comparing the GPU hierarchy with the CPU oracle.

Level-wise parity: the oracle is fed the GPU's own A_l, so a floating-point
decision that flips on one side cannot cascade into later levels.
"""
import numpy as np
import scipy.sparse as sp

from oracle import lair as O


def gpu_level_csr(h, l, what="A"):
    rp = h.export(l, what + ".rowptr")
    cj = h.export(l, what + ".col")
    v = h.export(l, what + ".val")
    return rp, cj, v


def gpu_A(h, l):
    rp, cj, v = gpu_level_csr(h, l, "A")
    return O.csr(rp, cj, v)


def rows_rel_err(a_rp, a_v, b_v):
    """max over rows of max|a-b| / max|b| (row-wise relative error)."""
    worst = 0.0
    diff = np.abs(a_v - b_v)
    for i in range(a_rp.shape[0] - 1):
        lo, hi = a_rp[i], a_rp[i + 1]
        if hi == lo:
            continue
        scale = np.abs(b_v[lo:hi]).max()
        if scale == 0:
            scale = 1.0
        worst = max(worst, diff[lo:hi].max() / scale)
    return worst


def _lump_scale(K, S, theta_d):
    """The scale matrix S (|R||A||P| on K's pattern) moved like K's lumped
    entries: kept entries keep their scale, removed ones add to the
    diagonal's."""
    assert np.array_equal(K.indptr, S.indptr) and np.array_equal(K.indices, S.indices)
    keep = O.lump_keep(K, theta_d)
    data = S.data.copy()
    for i in range(K.shape[0]):
        lo, hi = K.indptr[i], K.indptr[i + 1]
        gone = data[lo:hi][~keep[lo:hi]].sum()
        if gone:
            d = lo + int(np.flatnonzero(K.indices[lo:hi] == i)[0])
            data[d] += gone
    rows = np.repeat(np.arange(K.shape[0]), np.diff(K.indptr))
    out = sp.csr_matrix((data[keep], (rows[keep], K.indices[keep])), shape=K.shape)
    out.sort_indices()
    return out


def compare_level(h, l, theta=0.25, kind=O.SOC_ABS, distance=1,
                  interp=O.INTERP_ONE_POINT, cf=None, ztol=1e-12, ktol=1e-12, lump_tol=0.0):
    """Check level l of the GPU hierarchy against the oracle run on the GPU's
    A_l.  Returns a dict of measured errors; asserts the bit-exact parts."""
    A = gpu_A(h, l)
    n = A.shape[0]
    out = {"n": n}
    sm_o = O.strength(A, theta, kind)
    sm_g = h.export(l, "smask")
    assert np.array_equal(sm_o, sm_g), "strength mask differs at level %d" % l
    cf_g = h.export(l, "cf")
    if cf is None:
        cf_o = O.rs_split(A, sm_o)
    else:
        cf_o = np.asarray(cf, dtype=np.int8)
    assert np.array_equal(cf_o, cf_g), "CF splitting differs at level %d" % l
    cpts, nptr, nbr = O.neighbourhoods(A, sm_o, cf_o, distance)
    assert np.array_equal(nptr.astype(np.int32), h.export(l, "nbr_ptr"))
    assert np.array_equal(nbr.astype(np.int32), h.export(l, "nbr"))
    # the level's statistics (sizes the setup may first bound, then reads)
    st = h.level_stats(l)
    sizes = np.diff(np.asarray(nptr, dtype=np.int64))
    assert st["nc"] == len(cpts) and st["nnz_R"] == int(sizes.sum()) + len(cpts)
    if len(sizes):
        assert st["s_max"] == int(sizes.max()), "largest neighbourhood differs at level %d" % l
        assert abs(st["s_mean"] - sizes.mean()) <= 1e-12 * max(1.0, sizes.mean())
    z, flags = O.local_solves(A, cpts, nptr, nbr)
    assert np.array_equal(flags.astype(np.int8), h.export(l, "flags"))
    R = O.restriction(n, cpts, nptr, nbr, z)
    rrp, rcj, rv = gpu_level_csr(h, l, "R")
    assert np.array_equal(R.indptr.astype(np.int32), rrp)
    assert np.array_equal(R.indices.astype(np.int32), rcj)
    out["z_err"] = rows_rel_err(rrp, rv, R.data)
    assert out["z_err"] <= ztol, "R values differ by %g at level %d" % (out["z_err"], l)
    if interp == O.INTERP_ONE_POINT:
        P = O.interp_one_point(A, sm_o, cf_o)
    else:
        P = O.interp_direct(A, sm_o, cf_o)
    prp, pcj, pv = gpu_level_csr(h, l, "P")
    assert np.array_equal(P.indptr.astype(np.int32), prp)
    assert np.array_equal(P.indices.astype(np.int32), pcj)
    out["p_err"] = float(np.abs(P.data - pv).max()) if pv.shape[0] else 0.0
    assert np.allclose(pv, P.data, rtol=1e-13, atol=1e-15)
    K = O.galerkin(R, A, P)
    scale = O.galerkin(abs(R), abs(A), abs(P))
    if lump_tol > 0.0:
        K.sort_indices()
        scale.sort_indices()
        scale = _lump_scale(K, scale, lump_tol)
        K = O.lump(K, lump_tol)
    Kg = gpu_A(h, l + 1)
    assert np.array_equal(K.indptr, Kg.indptr), "K pattern (rowptr) differs at level %d" % l
    assert np.array_equal(K.indices, Kg.indices), "K pattern (col) differs at level %d" % l
    err = np.abs(Kg.data - K.data)
    bound = ktol * scale.data + 1e-300
    out["k_err"] = float((err / np.maximum(scale.data, 1e-300)).max()) if err.shape[0] else 0.0
    assert np.all(err <= bound), "K values differ (%g of scale) at level %d" % (out["k_err"], l)
    return out


def oracle_cf_levels(H):
    return [l.cf for l in H.levels[:-1]]
