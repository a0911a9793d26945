"""The DGu workload (Sec. 4.2): checks of its diffusion and reaction
assembly (symmetric interior penalty, Nitsche boundary terms, P2 on
triangles) against properties the discretisation must have, independent of
the solver: exactness for harmonic polynomials of degree <= 2, symmetry and
positive definiteness of the diffusion operator, the reaction mass matrix,
and the advective part reproducing the transport problem's constant."""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spl

import workloads as W
from workloads.dg import diffusion_reaction_dg_p2, jittered_mesh, upwind_dg_p2


def _nodes(m, jitter=0.2, seed=2):
    """Coordinates of the P2 DoFs (vertices, then edge midpoints (0,1),
    (1,2), (2,0)), element by element."""
    xy, tri = jittered_mesh(m, jitter, seed)
    P = xy[tri]
    mids = [0.5 * (P[:, a] + P[:, b]) for a, b in ((0, 1), (1, 2), (2, 0))]
    return np.concatenate([P, np.stack(mids, axis=1)], axis=1).reshape(-1, 2)


def _everywhere(xm, ym):
    return np.ones_like(xm, dtype=bool)


def test_sipg_reproduces_harmonic_quadratics():
    """-div grad u = 0 with u = g on the whole boundary: SIPG is consistent,
    so the discrete solution is the interpolant of any harmonic polynomial
    of degree <= 2 (A u_I = rhs to rounding)."""
    m = 6
    X = _nodes(m)
    zero = lambda x, y: np.zeros_like(x)
    for u in (lambda x, y: np.ones_like(x), lambda x, y: x + 2.0 * y,
              lambda x, y: x * x - y * y + 3.0 * x * y):
        A, rhs = diffusion_reaction_dg_p2(m, 1.0, zero, g=u, dirichlet=_everywhere)
        ui = u(X[:, 0], X[:, 1])
        res = A @ ui - rhs
        assert np.abs(res).max() <= 1e-9 * (np.abs(A).max() + np.abs(rhs).max())


def test_sipg_symmetric_positive_definite():
    m = 5
    zero = lambda x, y: np.zeros_like(x)
    A, _ = diffusion_reaction_dg_p2(m, 0.7, zero, dirichlet=_everywhere)
    A = A.toarray()
    assert np.abs(A - A.T).max() <= 1e-12 * np.abs(A).max()
    assert np.linalg.eigvalsh(0.5 * (A + A.T)).min() > 0.0


def test_reaction_is_gamma_mass_matrix():
    """kappa = 0: the assembly is the element mass matrix scaled by gamma;
    1^T M 1 is the area weighted by gamma (the domain's area for gamma = 1)."""
    m = 4
    one = lambda x, y: np.ones_like(x)
    M, rhs = diffusion_reaction_dg_p2(m, 0.0, one)
    assert np.abs(rhs).max() == 0.0
    e = np.ones(M.shape[0])
    assert abs(e @ (M @ e) - 1.0) <= 1e-12
    two = lambda x, y: np.where(x < 0.5, 2.0, 1.0)
    M2, _ = diffusion_reaction_dg_p2(m, 0.0, two)
    xy, tri = jittered_mesh(m)
    P = xy[tri]
    area = 0.5 * np.abs((P[:, 1, 0] - P[:, 0, 0]) * (P[:, 2, 1] - P[:, 0, 1]) -
                        (P[:, 1, 1] - P[:, 0, 1]) * (P[:, 2, 0] - P[:, 0, 0]))
    g = np.where(P.mean(axis=1)[:, 0] < 0.5, 2.0, 1.0)
    assert abs(e @ (M2 @ e) - (area * g).sum()) <= 1e-12


def test_dgu_transport_limit_constant_to_quadrature_error():
    """The advective part alone: u = 1 solves the transport problem with
    inflow value 1 exactly, and the discrete form reproduces it up to the
    quadrature error of the curved (non-polynomial) field, which falls
    with the mesh size at high order."""
    res = []
    for m in (4, 8):
        w = upwind_dg_p2(m, velocity=lambda x, y: (y * y, np.cos(0.5 * np.pi * x) ** 2))
        A = sp.csr_matrix((w["val"], w["col"], w["rowptr"]), shape=(w["n"],) * 2)
        e = np.ones(w["n"])
        res.append(np.abs(A @ e - w["rhs"]).max())
    assert res[0] < 1e-4 and res[1] < res[0] / 8.0


def test_dgu_workload_shape_and_blocks():
    """Dense 6 x 6 blocks (the nodal layout), gamma jump present, inflow
    data in the right-hand side, a solution near 1 upstream of the thick
    region for the diffusive case."""
    for kappa in (0.0, 1e-3):
        w = W.workload_dgu(8, kappa)
        n = w["n"]
        A = sp.csr_matrix((w["val"], w["col"], w["rowptr"]), shape=(n, n))
        rp, cj = w["rowptr"], w["col"]
        lens = np.diff(rp)
        assert np.all(lens % 6 == 0)
        for r in range(0, n, 6):
            assert np.array_equal(cj[rp[r]:rp[r + 1]], cj[rp[r + 5]:rp[r + 6]])
        assert np.abs(A.diagonal()).max() > 1e3 * np.abs(A.diagonal()).min()
        x = spl.spsolve(A.tocsc(), w["rhs"])
        assert np.isfinite(x).all() and np.abs(w["rhs"]).max() > 0
