"""Pins of the CPU oracle against facts the paper and the mathematics fix.

None of these tests compares the oracle with itself: every expected value
comes from a hand trace, a closed form, a dense re-derivation with NumPy, or
an independent brute-force implementation written here.
"""
import math
import os

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import workloads as W
from oracle import lair as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _read_golden(name):
    out = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            k, v = line.split(":", 1)
            out[k.strip()] = v.split()
    return out


def _mat(w):
    return O.csr(w["rowptr"], w["col"], w["val"])


# ---------------------------------------------------------------- brute force

def brute_strength(A, theta, kind):
    """Strong sets from a dense copy, written independently of the oracle."""
    D = A.toarray()
    n = D.shape[0]
    S = []
    for i in range(n):
        off = [abs(D[i, k]) for k in range(n) if k != i]
        m = max(off) if off else 0.0
        s = set()
        for j in range(n):
            if j == i or D[i, j] == 0.0 or m <= 0.0:
                continue
            a = -D[i, j] if kind == O.SOC_NEG else abs(D[i, j])
            if a >= theta * m:
                s.add(j)
        S.append(s)
    return S


def brute_rs(S):
    """Ruge-Stueben first pass by linear scans over sets (no tree)."""
    n = len(S)
    ST = [set() for _ in range(n)]
    for i in range(n):
        for j in S[i]:
            ST[j].add(i)
    lam = [len(ST[i]) for i in range(n)]
    state = [None] * n
    for i in range(n):
        if not S[i] and not ST[i]:
            state[i] = 0
    while True:
        U = [i for i in range(n) if state[i] is None]
        if not U:
            break
        best = max(U, key=lambda i: (lam[i], -i))
        if lam[best] == 0:
            for i in U:
                state[i] = 0
            break
        state[best] = 1
        for j in sorted(ST[best]):
            if state[j] is None:
                state[j] = 0
                for k in S[j]:
                    if state[k] is None:
                        lam[k] += 1
        for j in S[best]:
            if state[j] is None:
                lam[j] -= 1
    return np.array(state, dtype=np.int8)


def brute_nbr(S, cf, i, distance):
    F = {j for j in range(len(cf)) if cf[j] == 0}
    if distance == 0:
        return sorted(F)
    d1 = S[i] & F
    out = set(d1)
    if distance == 2:
        for j in d1:
            out |= S[j] & F
    return sorted(out)


def smask_to_sets(A, smask):
    S = []
    for i in range(A.shape[0]):
        lo, hi = A.indptr[i], A.indptr[i + 1]
        S.append({int(A.indices[p]) for p in range(lo, hi) if smask[p]})
    return S


# ---------------------------------------------------------------- O1 strength

def test_strength_c1_hand_values():
    """C1 interior rows: |a_W|/max = 1 and |a_S|/max = tan(3pi/16) >= 0.25."""
    w = W.workload_c1()
    A = _mat(w)
    sm = O.strength(A, 0.25, O.SOC_ABS)
    cnt = np.add.reduceat(sm.astype(np.int64), A.indptr[:-1]) * (np.diff(A.indptr) > 0)
    m = 64
    i = np.arange(m * m) % m
    j = np.arange(m * m) // m
    assert math.tan(3 * math.pi / 16) >= 0.25
    assert cnt[0] == 0
    assert np.all(cnt[(i > 0) & (j > 0)] == 2)
    assert np.all(cnt[(i == 0) & (j > 0)] == 1)
    assert np.all(cnt[(i > 0) & (j == 0)] == 1)


@pytest.mark.parametrize("kind", [O.SOC_ABS, O.SOC_NEG])
@pytest.mark.parametrize("theta", [0.1, 0.25, 0.6])
def test_strength_vs_bruteforce(kind, theta):
    rng = np.random.default_rng(7)
    D = rng.standard_normal((30, 30)) * (rng.uniform(size=(30, 30)) < 0.2)
    D[np.arange(30), np.arange(30)] = 5.0
    D[3, :] = 0.0
    D[3, 3] = 1.0                      # a row with no off-diagonal: no strong
    A = sp.csr_matrix(D)
    A.sort_indices()
    sm = O.strength(A, theta, kind)
    assert smask_to_sets(A, sm) == brute_strength(A, theta, kind)


def test_strength_keeps_explicit_zero_weak():
    A = O.csr(np.array([0, 2, 4]), np.array([0, 1, 0, 1]),
              np.array([2.0, 0.0, -1.0, 3.0]))
    sm = O.strength(A, 0.25)
    assert sm.tolist() == [0, 0, 1, 0]


# ---------------------------------------------------------------- O2 RS split

def test_rs_chain_hand_trace():
    g = _read_golden("chain5.txt")
    A = _mat(W.chain_1d(5))
    sm = O.strength(A, 0.25)
    cf = O.rs_split(A, sm)
    assert cf.tolist() == [int(v) for v in g["cf"]]
    cnt = [int(sm[A.indptr[i]:A.indptr[i + 1]].sum()) for i in range(5)]
    assert cnt == [int(v) for v in g["strong_per_row"]]


@pytest.mark.parametrize("seed", range(8))
def test_rs_vs_bruteforce(seed):
    w = W.random_ff_digraph(40, 3, seed)
    A = _mat(w)
    sm = O.strength(A, 0.25)
    S = smask_to_sets(A, sm)
    assert O.rs_split(A, sm).tolist() == brute_rs(S).tolist()


def test_rs_small_grid_vs_bruteforce():
    w = W.adr_2d(9, 1e-2, 0.3, 0.5)
    A = _mat(w)
    sm = O.strength(A, 0.25)
    assert O.rs_split(A, sm).tolist() == brute_rs(smask_to_sets(A, sm)).tolist()


# ---------------------------------------------------------------- O3 N_i

@pytest.mark.parametrize("distance", [0, 1, 2])
@pytest.mark.parametrize("seed", range(5))
def test_neighbourhoods_vs_bruteforce(distance, seed):
    w = W.random_ff_digraph(35, 4, seed + 100)
    A = _mat(w)
    sm = O.strength(A, 0.25)
    cf = O.rs_split(A, sm)
    cpts, nptr, nbr = O.neighbourhoods(A, sm, cf, distance)
    S = smask_to_sets(A, sm)
    for c, i in enumerate(cpts):
        got = nbr[nptr[c]:nptr[c + 1]].tolist()
        assert got == brute_nbr(S, cf, int(i), distance)


def test_neighbourhoods_chain():
    g = _read_golden("chain5.txt")
    A = _mat(W.chain_1d(5))
    sm = O.strength(A, 0.25)
    cf = O.rs_split(A, sm)
    cpts, nptr, nbr = O.neighbourhoods(A, sm, cf, 1)
    assert nptr.tolist() == [int(v) for v in g["nbr_ptr"]]
    assert nbr.tolist() == [int(v) for v in g["nbr"]]


# ---------------------------------------------------------------- O4-O5 Z

def _ideal_Z(A, cf):
    D = A.toarray()
    F = np.flatnonzero(cf == 0)
    C = np.flatnonzero(cf == 1)
    return -D[np.ix_(C, F)] @ np.linalg.inv(D[np.ix_(F, F)]), F, C


@pytest.mark.parametrize("seed", range(4))
def test_all_f_neighbourhood_gives_ideal_restriction(seed):
    """N_i = all F-points makes Z = -A_cf A_ff^{-1} exactly (Eq. r_ideal)."""
    w = W.random_ff_digraph(60, 4, seed + 200)
    A = _mat(w)
    sm = O.strength(A, 0.25)
    cf = O.rs_split(A, sm)
    cpts, nptr, nbr = O.neighbourhoods(A, sm, cf, O.DIST_ALL_F)
    z, flags = O.local_solves(A, cpts, nptr, nbr)
    R = O.restriction(A.shape[0], cpts, nptr, nbr, z).toarray()
    Zi, F, C = _ideal_Z(A, cf)
    assert flags.sum() == 0
    assert np.abs(R[:, F] - Zi).max() <= 1e-12 * max(1.0, np.abs(Zi).max())
    assert np.array_equal(R[:, C], np.eye(C.shape[0]))


def test_ideal_restriction_on_small_transport():
    w = W.upwind_transport_2d(12)
    A = _mat(w)
    sm = O.strength(A, 0.25)
    cf = O.rs_split(A, sm)
    cpts, nptr, nbr = O.neighbourhoods(A, sm, cf, O.DIST_ALL_F)
    z, _ = O.local_solves(A, cpts, nptr, nbr)
    R = O.restriction(A.shape[0], cpts, nptr, nbr, z).toarray()
    Zi, F, C = _ideal_Z(A, cf)
    assert np.abs(R[:, F] - Zi).max() <= 1e-12 * np.abs(Zi).max()


@pytest.mark.parametrize("distance", [1, 2])
@pytest.mark.parametrize("case", ["adr", "dg"])
def test_RA_vanishes_on_neighbourhood(distance, case):
    """Eq. (johnair): (Z A_ff + A_cf)(i, N_i) = 0, i.e. (R A)(i, N_i) = 0."""
    if case == "adr":
        A = _mat(W.adr_2d(14, 1e-2, 0.7, 0.3))
    else:
        w = W.upwind_dg_p2(6)
        A, _ = O.block_scale(_mat(w), w["rhs"], 6)
    sm = O.strength(A, 0.25)
    cf = O.rs_split(A, sm)
    cpts, nptr, nbr = O.neighbourhoods(A, sm, cf, distance)
    z, flags = O.local_solves(A, cpts, nptr, nbr)
    R = O.restriction(A.shape[0], cpts, nptr, nbr, z)
    RA = (R @ A).toarray()
    scale = (abs(R) @ abs(A)).toarray()
    for c in range(cpts.shape[0]):
        nb = nbr[nptr[c]:nptr[c + 1]]
        if nb.shape[0]:
            assert np.all(np.abs(RA[c, nb]) <= 1e-12 * scale[c, nb] + 1e-300)


def test_local_solves_vs_numpy():
    A = _mat(W.adr_2d(12, 1e-1, 2.0, 0.1))
    sm = O.strength(A, 0.25)
    cf = O.rs_split(A, sm)
    cpts, nptr, nbr = O.neighbourhoods(A, sm, cf, 2)
    z, flags = O.local_solves(A, cpts, nptr, nbr)
    D = A.toarray()
    for c, i in enumerate(cpts):
        nb = nbr[nptr[c]:nptr[c + 1]]
        if not nb.shape[0]:
            continue
        M = D[np.ix_(nb, nb)].T
        f = -D[i, nb]
        ref = np.linalg.solve(M, f)
        assert np.abs(z[nptr[c]:nptr[c + 1]] - ref).max() <= 1e-12 * max(1, np.abs(ref).max())


def test_singular_local_system_takes_min_norm_lstsq():
    """Footnote of Sec. 3.1: a singular local system is solved as a
    minimal-norm least-squares problem.  Rows 1 and 2 are identical, so the
    local matrix of C-point 0 (N = {1, 2}) is singular; a_22 is a stored
    zero."""
    A = O.csr(np.array([0, 3, 5, 8, 9]), np.array([0, 1, 2, 1, 3, 1, 2, 3, 3]),
              np.array([4.0, -1.0, -1.0, 1.0, -1.0, 1.0, 0.0, -1.0, 2.0]))
    cf = np.array([1, 0, 0, 1], dtype=np.int8)
    cpts = np.array([0, 3], dtype=np.int32)
    nptr = np.array([0, 2, 2], dtype=np.int64)
    nbr = np.array([1, 2], dtype=np.int32)
    z, flags = O.local_solves(A, cpts, nptr, nbr)
    assert flags.tolist() == [1, 0]
    M = np.array([[1.0, 1.0], [0.0, 0.0]])      # A(N,N)^T
    f = np.array([1.0, 1.0])
    assert np.allclose(z, np.linalg.pinv(M) @ f, rtol=0, atol=1e-14)


def test_chain_z_is_one():
    g = _read_golden("chain5.txt")
    A = _mat(W.chain_1d(5))
    sm = O.strength(A, 0.25)
    cf = O.rs_split(A, sm)
    cpts, nptr, nbr = O.neighbourhoods(A, sm, cf, 1)
    z, _ = O.local_solves(A, cpts, nptr, nbr)
    assert z.tolist() == [float(v) for v in g["z"]]
    R = O.restriction(5, cpts, nptr, nbr, z)
    assert R.indptr.tolist() == [int(v) for v in g["R_rowptr"]]
    assert R.indices.tolist() == [int(v) for v in g["R_col"]]
    assert R.data.tolist() == [float(v) for v in g["R_val"]]


# ---------------------------------------------------------------- O6-O8 P, K

def test_one_point_interp_chain_and_strongest():
    g = _read_golden("chain5.txt")
    A = _mat(W.chain_1d(5))
    sm = O.strength(A, 0.25)
    cf = O.rs_split(A, sm)
    P = O.interp_one_point(A, sm, cf)
    want = [int(v) for v in g["P_one_point_col"]]
    for i in range(5):
        cols = P.indices[P.indptr[i]:P.indptr[i + 1]].tolist()
        assert cols == ([] if want[i] < 0 else [want[i]])
    # strongest C-neighbour, ties to the smallest index
    A2 = O.csr(np.array([0, 4, 5, 6, 7]), np.array([0, 1, 2, 3, 1, 2, 3]),
               np.array([3.0, -1.0, -2.0, 2.0, 1.0, 1.0, 1.0]))
    cf2 = np.array([0, 1, 1, 1], dtype=np.int8)
    sm2 = O.strength(A2, 0.25)
    P2 = O.interp_one_point(A2, sm2, cf2)
    assert P2.indices[P2.indptr[0]:P2.indptr[1]].tolist() == [1]   # col 2 -> c1


def test_direct_interp_reproduces_constants():
    """Zero row sums: sum_k w_ik = -(sum_{j != i} a_ij)/a_ii = 1."""
    w = W.adr_2d(15, 1.0, 0.4, 0.0)
    A = _mat(w)
    rs = np.asarray(A.sum(axis=1)).ravel()
    sm = O.strength(A, 0.25)
    cf = O.rs_split(A, sm)
    P = O.interp_direct(A, sm, cf)
    p1 = P @ np.ones(P.shape[1])
    rows = (np.abs(rs) < 1e-12 * np.abs(A.diagonal())) & (np.diff(P.indptr) > 0)
    assert rows.sum() > 10
    assert np.allclose(p1[rows], 1.0, rtol=0, atol=1e-12)


def _golden_direct():
    g = _read_golden("direct_interp7.txt")
    A = O.csr(np.array(g["A_rowptr"], np.int32), np.array(g["A_col"], np.int32),
              np.array(g["A_val"], np.float64))
    P = O.csr(np.array(g["P_rowptr"], np.int32), np.array(g["P_col"], np.int32),
              np.array(g["P_val"], np.float64), shape=(A.shape[0], 3))
    return g, A, P


def test_direct_interp_hand_worked_rows():
    """Direct interpolation (Stueben 2001) worked by hand on rows with both
    sign classes (beta weights for positive couplings, a weak positive
    neighbour in N_i but not in P_i), with no positive interpolatory
    coupling (their sum goes to the diagonal), with no negative one, and
    with no strong C-neighbour (zero row)."""
    g, A, Pw = _golden_direct()
    sm = O.strength(A, 0.25, O.SOC_ABS)
    assert np.array_equal(sm, np.array(g["strong"], np.uint8))
    cf = np.array(g["cf"], np.int8)
    P = O.interp_direct(A, sm, cf)
    assert np.array_equal(P.indptr, Pw.indptr)
    assert np.array_equal(P.indices, Pw.indices)
    assert np.allclose(P.data, Pw.data, rtol=4e-16, atol=0.0)


def test_galerkin_matches_dense_products():
    A = _mat(W.adr_2d(10, 1e-2, 1.1, 0.2))
    H = O.setup(A, interp=O.INTERP_DIRECT, max_coarse=10)
    L0 = H.levels[0]
    K = H.levels[1].A.toarray()
    Kd = L0.R.toarray() @ L0.A.toarray() @ L0.P.toarray()
    assert np.abs(K - Kd).max() <= 1e-12 * np.abs(Kd).max()


def test_galerkin_pattern_is_symbolic():
    """Entries that cancel to zero stay in K's pattern (chain: R A has an
    exact 0 in every F column, Eq. (johnair))."""
    g = _read_golden("chain5.txt")
    A = _mat(W.chain_1d(5))
    H = O.setup(A, max_coarse=1, max_levels=2)
    K = H.levels[1].A
    assert K.indptr.tolist() == [int(v) for v in g["K_rowptr"]]
    assert K.indices.tolist() == [int(v) for v in g["K_col"]]
    assert K.data.tolist() == [float(v) for v in g["K_val"]]
    AP = H.levels[0].AP
    assert 0.0 in AP.data.tolist()        # the kept cancellation


def test_ideal_R_gives_schur_complement():
    """With ideal R, R A P = A_cc - A_cf A_ff^{-1} A_fc for any P."""
    w = W.random_ff_digraph(50, 4, 321)
    A = _mat(w)
    sm = O.strength(A, 0.25)
    cf = O.rs_split(A, sm)
    cpts, nptr, nbr = O.neighbourhoods(A, sm, cf, O.DIST_ALL_F)
    z, _ = O.local_solves(A, cpts, nptr, nbr)
    R = O.restriction(A.shape[0], cpts, nptr, nbr, z)
    D = A.toarray()
    F = np.flatnonzero(cf == 0)
    C = np.flatnonzero(cf == 1)
    S = D[np.ix_(C, C)] - D[np.ix_(C, F)] @ np.linalg.solve(D[np.ix_(F, F)], D[np.ix_(F, C)])
    for P in (O.interp_one_point(A, sm, cf), O.interp_direct(A, sm, cf)):
        K = O.galerkin(R, A, P).toarray()
        assert np.abs(K - S).max() <= 1e-11 * np.abs(S).max()


def test_row_scaling_invariance():
    """Remark (row scaling): A -> D A keeps the splitting and patterns,
    Z -> D_c Z D_f^{-1}, K -> D_c K (same P)."""
    w = W.adr_2d(12, 1e-2, 0.9, 0.3)
    A = _mat(w)
    d = np.random.default_rng(5).uniform(0.5, 4.0, A.shape[0])
    DA = (sp.diags(d) @ A).tocsr()
    DA.sort_indices()
    sm = O.strength(A, 0.25)
    cf = O.rs_split(A, sm)
    smd = O.strength(DA, 0.25)
    assert np.array_equal(sm, smd)
    assert np.array_equal(cf, O.rs_split(DA, smd))
    cpts, nptr, nbr = O.neighbourhoods(A, sm, cf, 2)
    z, _ = O.local_solves(A, cpts, nptr, nbr)
    zd, _ = O.local_solves(DA, cpts, nptr, nbr)
    rows = np.repeat(cpts, np.diff(nptr))
    assert np.allclose(zd, d[rows] * z / d[nbr], rtol=1e-12, atol=0)
    P = O.interp_one_point(A, sm, cf)
    R = O.restriction(A.shape[0], cpts, nptr, nbr, z)
    Rd = O.restriction(A.shape[0], cpts, nptr, nbr, zd)
    K = O.galerkin(R, A, P).toarray()
    Kd = O.galerkin(Rd, DA, P).toarray()
    assert np.abs(Kd - d[cpts][:, None] * K).max() <= 1e-12 * np.abs(Kd).max()


# ---------------------------------------------------------------- O10 cycle

def test_chain_one_cycle_is_exact():
    """F-F-C Jacobi after the distance-one lAIR correction solves the upwind
    chain in one V-cycle, for any length and depth."""
    for n in (5, 64, 257):
        A = _mat(W.chain_1d(n))
        H = O.setup(A, max_coarse=2)
        b = np.random.default_rng(n).standard_normal(n)
        x = O.cycle(H, b, np.zeros(n))
        xs = spla.spsolve(A.tocsc(), b)
        assert np.abs(x - xs).max() <= 1e-12 * np.abs(xs).max()
        for l in H.levels[1:]:
            K = l.A
            assert np.all(np.diff(K.indptr)[1:] == 2)


def _two_grid_error_operator(H):
    """E = (I - Pi_C D^-1 A)(I - Pi_F D^-1 A)^2 (I - P K^-1 R A), written from
    Eq. (err_prop) and Eq. (jacobi_err) with Delta = D_ff^{-1}."""
    L = H.levels[0]
    A = L.A.toarray()
    n = A.shape[0]
    R, P = L.R.toarray(), L.P.toarray()
    K = R @ A @ P
    Dinv = np.diag(1.0 / np.diag(A))
    PiF = np.diag((L.cf == 0).astype(float))
    PiC = np.diag((L.cf == 1).astype(float))
    I = np.eye(n)
    cgc = I - P @ np.linalg.solve(K, R @ A)
    fr = I - PiF @ Dinv @ A
    cr = I - PiC @ Dinv @ A
    return cr @ fr @ fr @ cgc


def test_two_grid_cycle_matches_error_propagation():
    A = _mat(W.adr_2d(9, 1e-2, 0.6, 0.2))
    H = O.setup(A, max_levels=2, max_coarse=10, distance=2)
    assert H.nlevels == 2
    E = _two_grid_error_operator(H)
    rng = np.random.default_rng(3)
    xs = rng.standard_normal(A.shape[0])
    b = A @ xs
    x0 = rng.standard_normal(A.shape[0])
    x1 = O.cycle(H, b, x0)
    assert np.abs((xs - x1) - E @ (xs - x0)).max() <= 1e-11 * np.abs(xs - x0).max()


def test_exact_f_solve_and_ideal_R_converge_in_one_step():
    """Eq. (cgc_rho): exact F-solve with ideal restriction gives rho = 0."""
    w = W.random_ff_digraph(40, 3, 11)
    A = _mat(w)
    D = A.toarray()
    sm = O.strength(A, 0.25)
    cf = O.rs_split(A, sm)
    cpts, nptr, nbr = O.neighbourhoods(A, sm, cf, O.DIST_ALL_F)
    z, _ = O.local_solves(A, cpts, nptr, nbr)
    R = O.restriction(A.shape[0], cpts, nptr, nbr, z).toarray()
    P = O.interp_one_point(A, sm, cf).toarray()
    F = np.flatnonzero(cf == 0)
    n = A.shape[0]
    Delta = np.zeros((n, n))
    Delta[np.ix_(F, F)] = np.linalg.inv(D[np.ix_(F, F)])
    K = R @ D @ P
    E = (np.eye(n) - Delta @ D) @ (np.eye(n) - P @ np.linalg.solve(K, R @ D))
    assert np.abs(np.linalg.eigvals(E)).max() <= 1e-10


def test_row_scaling_gives_same_iterates():
    w = W.adr_2d(16, 1e-2, 2.5, 0.1)
    A = _mat(w)
    d = np.random.default_rng(8).uniform(0.3, 3.0, A.shape[0])
    DA = (sp.diags(d) @ A).tocsr()
    DA.sort_indices()
    H = O.setup(A, interp=O.INTERP_ONE_POINT)
    Hd = O.setup(DA, interp=O.INTERP_ONE_POINT)
    b = np.ones(A.shape[0])
    x = O.cycle(H, b, np.zeros_like(b))
    xd = O.cycle(Hd, d * b, np.zeros_like(b))
    x2 = O.cycle(H, b, x)
    xd2 = O.cycle(Hd, d * b, xd)
    assert np.abs(x2 - xd2).max() <= 1e-11 * np.abs(x2).max()


# ---------------------------------------------------------------- O11 solve

@pytest.mark.parametrize("case", ["c1", "c4", "euler3d"])
def test_solve_matches_direct_solution(case):
    if case == "c1":
        w = W.workload_c1(32)
        A = _mat(w)
        kw = {}
    elif case == "c4":
        w = W.workload_c4(32)
        A = (_mat(w) + sp.diags(w["c"])).tocsr()
        A.sort_indices()
        kw = dict(interp=O.INTERP_DIRECT)
    else:
        w = W.implicit_euler_adr_3d(m=14, nrhs=1)
        A = _mat(w)
        kw = dict(interp=O.INTERP_DIRECT)
    H = O.setup(A, **kw)
    x, it, hist = O.solve(H, w["rhs"], rtol=1e-10)
    assert hist[-1] <= 1e-10 * np.linalg.norm(w["rhs"])
    xs = spla.spsolve(A.tocsc(), w["rhs"])
    cond_est = np.linalg.cond(A.toarray()) if A.shape[0] <= 3000 else 1e4
    assert np.linalg.norm(x - xs) <= 2e-10 * cond_est * np.linalg.norm(xs)


# ---------------------------------------------------------------- adjoint

def test_transpose_cycle_is_adjoint():
    """<B u, v> = <u, B^T v> for one cycle from zero (x = B b)."""
    w = W.workload_c4(24)
    A = (_mat(w) + sp.diags(w["c"])).tocsr()
    A.sort_indices()
    H = O.setup(A, interp=O.INTERP_DIRECT, max_coarse=20)
    assert H.nlevels >= 3
    rng = np.random.default_rng(2)
    u = rng.standard_normal(A.shape[0])
    v = rng.standard_normal(A.shape[0])
    Bu = O.cycle(H, u, np.zeros_like(u))
    Btv = O.cycle_transpose(H, v, np.zeros_like(v))
    assert abs(Bu @ v - u @ Btv) <= 1e-13 * np.linalg.norm(Bu) * np.linalg.norm(v) * 10


def test_transpose_solve_matches_dense():
    w = W.workload_c4(20)
    A = (_mat(w) + sp.diags(w["c"])).tocsr()
    A.sort_indices()
    H = O.setup(A, interp=O.INTERP_DIRECT)
    g = np.random.default_rng(4).standard_normal(A.shape[0])
    lam, it, hist = O.solve_transpose(H, g, rtol=1e-12)
    ref = np.linalg.solve(A.toarray().T, g)
    assert np.linalg.norm(lam - ref) <= 1e-9 * np.linalg.norm(ref)


# ---------------------------------------------------------------- DG / block

def test_dg_reproduces_constants_and_block_scaling():
    w = W.upwind_dg_p2(5)
    A = _mat(w)
    assert np.abs(A @ np.ones(A.shape[0]) - w["rhs"]).max() <= 1e-14
    As, bs = O.block_scale(A, w["rhs"], 6)
    D = As.toarray()
    Ad = A.toarray()
    for e in range(A.shape[0] // 6):
        sl = slice(6 * e, 6 * e + 6)
        # the identity exactly, whatever the rounding of D_B^{-1} D_B
        assert np.array_equal(D[sl, sl], np.eye(6))
        # the rest of the block row: D_B^{-1} times A's block row (dense)
        want = np.linalg.solve(Ad[sl, sl], Ad[sl, :])
        off = np.ones(A.shape[0], bool)
        off[sl] = False
        assert np.abs(D[sl][:, off] - want[:, off]).max() <= 1e-12 * np.abs(want).max()
    assert np.abs(As @ np.ones(A.shape[0]) - bs).max() <= 1e-12


# ---------------------------------------------------------------- new diagonal

def _with_diag(A, d):
    B = A.tocsr(copy=True)
    B.setdiag(d)
    B.sort_indices()
    return B


def test_update_diag_satisfies_the_local_systems_and_galerkin():
    """After a new diagonal, every row of Z solves its local system with the
    new values on the kept N_i (Eq. (johnair): (Z A + A_cf)(i, N_i) = 0,
    checked densely) and each coarse operator is R A P (dense products)."""
    w = W.workload_c4(16)
    A = (_mat(w) + sp.diags(w["c"])).tocsr()
    A.sort_indices()
    H = O.setup(A, interp=O.INTERP_DIRECT, max_coarse=20)
    assert H.nlevels >= 3
    d_new = A.diagonal() * (1.0 + 0.5 * np.random.default_rng(7).random(A.shape[0]))
    O.update_diag(H, d_new)
    A_new = _with_diag(A, d_new)
    assert np.array_equal(H.levels[0].A.toarray(), A_new.toarray())
    for l, L in enumerate(H.levels[:-1]):
        D = L.A.toarray()
        R = L.R.toarray()
        for c, i in enumerate(L.cpts):
            nb = L.nbr[L.nptr[c]:L.nptr[c + 1]]
            if nb.shape[0] == 0:
                continue
            res = R[c] @ D[:, nb]
            assert np.abs(res).max() <= 1e-10 * np.abs(D[i]).max(), (l, c)
        K = R @ D @ L.P.toarray()
        Kn = H.levels[l + 1].A.toarray()
        assert np.abs(Kn - K).max() <= 1e-12 * np.abs(K).max()


def test_update_diag_keeps_structure_and_identity():
    """The same diagonal gives back the same hierarchy, bit for bit; a new
    one keeps every pattern and the splittings."""
    w = W.workload_c4(16)
    A = (_mat(w) + sp.diags(w["c"])).tocsr()
    A.sort_indices()
    H = O.setup(A, interp=O.INTERP_DIRECT, max_coarse=20)
    ref = [(L.A.copy(), L.R.copy(), L.P.copy()) for L in H.levels[:-1]]
    O.update_diag(H, A.diagonal())
    for (A0, R0, P0), L in zip(ref, H.levels[:-1]):
        for X, Y in ((A0, L.A), (R0, L.R), (P0, L.P)):
            assert np.array_equal(X.indptr, Y.indptr) and np.array_equal(X.indices, Y.indices)
            assert np.array_equal(X.data, Y.data)
    O.update_diag(H, 2.0 * A.diagonal())
    for (A0, R0, P0), L in zip(ref, H.levels[:-1]):
        for X, Y in ((A0, L.A), (R0, L.R), (P0, L.P)):
            assert np.array_equal(X.indptr, Y.indptr) and np.array_equal(X.indices, Y.indices)
    # direct weights are -alpha a_ik / a_ii with alpha free of the diagonal:
    # doubling the diagonal halves the F rows of P_0 and keeps its C rows
    P0, P1 = ref[0][2].toarray(), H.levels[0].P.toarray()
    F = H.levels[0].cf == 0
    assert np.abs(P1[F] - 0.5 * P0[F]).max() <= 1e-15 * np.abs(P0[F]).max()
    assert np.array_equal(P1[~F], P0[~F])


def test_update_diag_chain_still_solves_in_one_cycle():
    """On the upwind chain the structure does not depend on the diagonal, so
    after a new (positive) diagonal one V-cycle is still an exact solve."""
    n = 129
    A = _mat(W.chain_1d(n))
    H = O.setup(A, max_coarse=2)
    d = 1.0 + np.random.default_rng(3).random(n)
    O.update_diag(H, d)
    A_new = _with_diag(A, d)
    b = np.random.default_rng(4).standard_normal(n)
    x = O.cycle(H, b, np.zeros(n))
    xs = spla.spsolve(A_new.tocsc(), b)
    assert np.abs(x - xs).max() <= 1e-12 * np.abs(xs).max()


# ----------------------------------------------------------------- FGMRES

def _nonsym(n, seed):
    rng = np.random.default_rng(seed)
    A = 4.0 * np.eye(n) + 0.6 * rng.standard_normal((n, n))
    return A, rng.standard_normal(n)


@pytest.mark.parametrize("seed", [0, 1])
def test_fgmres_minimises_over_the_krylov_space(seed):
    """Unpreconditioned, no restart: after k steps the residual is the least
    one over x0 + K_k(A, r0), here found by an independent least-squares fit
    on an orthonormal basis of the Krylov matrix."""
    A, b = _nonsym(24, seed)
    x0 = np.random.default_rng(seed + 10).standard_normal(24)
    r0 = b - A @ x0
    for k in range(1, 9):
        xk, it, _, _ = O.fgmres(A, b, lambda v: v, x0=x0, rtol=0.0, maxit=k, restart=50)
        assert it == k
        K = np.empty((24, k))
        K[:, 0] = r0
        for j in range(1, k):
            K[:, j] = A @ K[:, j - 1]
        Q, _ = np.linalg.qr(K)
        y, *_ = np.linalg.lstsq(A @ Q, r0, rcond=None)
        best = np.linalg.norm(r0 - A @ Q @ y)
        got = np.linalg.norm(b - A @ xk)
        assert abs(got - best) <= 1e-9 * np.linalg.norm(r0)


def test_fgmres_estimate_is_the_true_residual():
    A, b = _nonsym(20, 3)
    for k in (1, 4, 9):
        xk, _, _, est = O.fgmres(A, b, lambda v: v, rtol=0.0, maxit=k, restart=30)
        assert abs(est[-1] - np.linalg.norm(b - A @ xk)) <= 1e-10 * np.linalg.norm(b)


def test_fgmres_exact_preconditioner_one_step():
    A, b = _nonsym(16, 4)
    x, it, hist, _ = O.fgmres(A, b, lambda v: np.linalg.solve(A, v), rtol=1e-12)
    assert it == 1
    assert np.linalg.norm(x - np.linalg.solve(A, b)) <= 1e-12 * np.linalg.norm(x)


def test_fgmres_restart_is_a_fresh_start():
    """GMRES(3) for 9 steps equals three GMRES(3) runs of 3 steps, each
    starting from the last iterate."""
    A, b = _nonsym(18, 5)
    x9, it, _, _ = O.fgmres(A, b, lambda v: v, rtol=0.0, maxit=9, restart=3)
    assert it == 9
    x = np.zeros(18)
    for _ in range(3):
        x, _, _, _ = O.fgmres(A, b, lambda v: v, x0=x, rtol=0.0, maxit=3, restart=3)
    assert np.linalg.norm(x9 - x) <= 1e-12 * np.linalg.norm(x)


def test_fgmres_cycle_no_slower_than_stationary():
    """With the V-cycle as a fixed preconditioner B, the k-th FGMRES iterate
    minimises the residual over x0 + B K_k(A B, r0), which holds the k-th
    stationary iterate: never more iterations to the same tolerance."""
    w = W.workload_c4(24)
    A = (O.csr(w["rowptr"], w["col"], w["val"]) + sp.diags(w["c"])).tocsr()
    A.sort_indices()
    H = O.setup(A, interp=O.INTERP_DIRECT)
    b = w["rhs"]
    xs, its, _ = O.solve(H, b, rtol=1e-10)
    xg, itg, hist, _ = O.fgmres_cycle(H, b, rtol=1e-10, restart=20)
    assert itg <= its
    assert np.linalg.norm(b - A @ xg) <= 1e-10 * np.linalg.norm(b)


# ----------------------------------------------------------------- lumping

def test_lump_hand_example():
    """Sec. 3.3 by hand, theta_D = 1e-3: each row's cut is 1e-3 times the
    largest magnitude of the row, diagonal included (10, 5, 6, 3: cuts 0.01,
    0.005, 0.006, 0.003); the off-diagonal entries below it move onto the
    diagonal.  Rows 0 and 2 hold an entry (-0.005, -0.004) that a maximum
    over the off-diagonal entries alone (2, 2) would keep."""
    K = sp.csr_matrix(np.array([[10.0, -0.005, -2.0, 0.0],
                                [-1.0, 5.0, -1e-5, -3.0],
                                [0.0, -2.0, 6.0, -0.004],
                                [-0.0015, 0.0, -3.0, 1.0]]))
    want = np.array([[10.0 - 0.005, 0.0, -2.0, 0.0],
                     [-1.0, 5.0 - 1e-5, 0.0, -3.0],
                     [0.0, -2.0, 6.0 - 0.004, 0.0],
                     [0.0, 0.0, -3.0, 1.0 - 0.0015]])
    L = O.lump(K, 1e-3)
    assert np.array_equal(L.toarray(), want)
    assert L.nnz == 9
    # a row without its diagonal, or without an off-diagonal entry, stays whole
    K2 = sp.csr_matrix((np.array([1e-9, 4.0, 7.0]), np.array([1, 2, 1]),
                        np.array([0, 2, 3])), shape=(2, 3))
    L2 = O.lump(K2, 1e-3)
    assert L2.nnz == 3 and np.array_equal(L2.toarray(), K2.toarray())


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_lump_keeps_row_sums_and_limits(seed):
    rng = np.random.default_rng(seed)
    n = 40
    K = sp.random(n, n, density=0.3, random_state=seed, format="csr") * 2.0 - \
        sp.random(n, n, density=0.3, random_state=seed + 7, format="csr")
    K = (K + sp.diags(5.0 + rng.random(n))).tocsr()
    K.sum_duplicates()
    K.sort_indices()
    one = np.ones(n)
    scale = abs(K) @ one
    for th in (1e-3, 0.1, 0.5, 1.0):
        L = O.lump(K, th)
        assert np.all(np.abs(L @ one - K @ one) <= 1e-14 * scale)
        assert L.nnz <= K.nnz
    assert (O.lump(K, 0.0) != K).nnz == 0          # nothing below a zero cut
    # at theta_D = 1 an off-diagonal entry stays only when its magnitude is
    # the row's largest, diagonal included
    L1 = O.lump(K, 1.0)
    for i in range(n):
        row = K.getrow(i).toarray().ravel()
        mag = np.abs(row)
        off = mag.copy()
        off[i] = 0.0
        kept = set(L1.getrow(i).indices) - {i}
        want = set(np.flatnonzero(off == mag.max())) - {i} if off.max() > 0 else set()
        assert kept == want


def test_lumped_hierarchy_is_smaller_and_converges():
    """Lumping at the paper's 1e-3 lowers the operator complexity and leaves
    convergence about where it was (Sec. 3.3)."""
    w = W.workload_c4(32)
    A = (O.csr(w["rowptr"], w["col"], w["val"]) + sp.diags(w["c"])).tocsr()
    A.sort_indices()
    H0 = O.setup(A, interp=O.INTERP_DIRECT)
    H1 = O.setup(A, interp=O.INTERP_DIRECT, lump_tol=1e-3,
                 cf_levels=[l.cf for l in H0.levels[:-1]])
    assert H1.op_complexity() < H0.op_complexity()
    _, i0, _ = O.solve(H0, w["rhs"], rtol=1e-10)
    x1, i1, _ = O.solve(H1, w["rhs"], rtol=1e-10)
    assert i1 <= i0 + 3
    assert np.linalg.norm(w["rhs"] - A @ x1) <= 1e-10 * np.linalg.norm(w["rhs"])


# --------------------------------------------------------------------------
# Nodal (block) treatment, Sec. 3.1 block form of Eq. (system), Sec. 4.2 (iii)
# --------------------------------------------------------------------------

def _adr(m):
    w = W.workload_c4(m)
    A = (O.csr(w["rowptr"], w["col"], w["val"]) + sp.diags(w["c"])).tocsr()
    A.sort_indices()
    return A, w["rhs"]


@pytest.mark.parametrize("distance", [1, 2])
def test_nodal_with_unit_blocks_is_scalar_lair(distance):
    """k = 1: block norms are magnitudes, so every step reduces to scalar
    lAIR with one-point interpolation, at distance one and two."""
    A, b = _adr(24)
    H = O.setup(A, interp=O.INTERP_ONE_POINT, distance=distance)
    G = O.setup(A, block=1, distance=distance)
    assert G.nlevels == H.nlevels
    for l in range(H.nlevels - 1):
        assert np.array_equal(G.levels[l].cf, H.levels[l].cf)
        assert np.array_equal(G.levels[l].smask, H.levels[l].smask)
        for M in ("R", "P"):
            a, c = getattr(G.levels[l], M), getattr(H.levels[l], M)
            assert np.array_equal(a.indptr, c.indptr) and np.array_equal(a.indices, c.indices)
            assert np.abs(a.data - c.data).max() <= 1e-12 * np.abs(c.data).max()
    _, it_h, _ = O.solve(H, b, rtol=1e-10)
    x, it_g, _ = O.solve(G, b, rtol=1e-10)
    assert it_g == it_h
    assert np.linalg.norm(b - A @ x) <= 1e-10 * np.linalg.norm(b)


def _kron_case(k=3, m=20, seed=0):
    As, bs = _adr(m)
    rng = np.random.default_rng(seed)
    B = rng.standard_normal((k, k)) + 3.0 * np.eye(k)
    A = sp.kron(As, sp.csr_matrix(B)).tocsr()
    A.sort_indices()
    return As, bs, B, A


@pytest.mark.parametrize("distance", [1, 2])
def test_nodal_kronecker_is_scalar_times_identity(distance):
    """A = A_s (x) B: the block norms are |a_ij| ||B||_F, so the nodes split
    as the scalar points of A_s; Z_il = z_il I solves the block system
    (z (a B) summed = -a_ij B), so R = R_s (x) I, P = P_s (x) I, K = K_s (x) B,
    and block Jacobi with D_i = a_ii B maps x_s (x) B^{-1} w as the scalar
    sweep maps x_s: every cycle's iterate is the scalar one (x) B^{-1} w."""
    k = 3
    As, bs, B, A = _kron_case(k)
    Hs = O.setup(As, interp=O.INTERP_ONE_POINT, distance=distance)
    Hb = O.setup(A, block=k, max_coarse=128 * k, distance=distance)   # the same stop in nodes
    assert Hb.nlevels == Hs.nlevels >= 3
    I = sp.identity(k)
    for l in range(Hs.nlevels - 1):
        Ls, Lb = Hs.levels[l], Hb.levels[l]
        assert np.array_equal(Lb.cf, np.repeat(Ls.cf, k))
        Rk = sp.kron(Ls.R, I).toarray()
        assert np.abs(Lb.R.toarray() - Rk).max() <= 1e-12 * np.abs(Rk).max()
        assert (Lb.P != sp.kron(Ls.P, I)).nnz == 0
        Kk = sp.kron(Hs.levels[l + 1].A, sp.csr_matrix(B)).toarray()
        assert np.abs(Hb.levels[l + 1].A.toarray() - Kk).max() <= 1e-11 * np.abs(Kk).max()
    w = np.array([1.0, -2.0, 0.5])
    u = np.linalg.solve(B, w)
    xs = np.zeros_like(bs)
    xb = np.zeros(A.shape[0])
    bb = np.kron(bs, w)
    for _ in range(3):
        xs = O.cycle(Hs, bs, xs)
        xb = O.cycle(Hb, bb, xb)
        ref = np.kron(xs, u)
        assert np.linalg.norm(xb - ref) <= 1e-10 * np.linalg.norm(ref)


def _dense_block_case(k=2, m=16, seed=1):
    """A dense-block matrix that is not a Kronecker product: A_s (x) B with
    every stored entry perturbed."""
    As, bs, B, A = _kron_case(k, m, seed)
    rng = np.random.default_rng(seed + 10)
    A = A.copy()
    A.data = A.data * (1.0 + 0.3 * rng.standard_normal(A.nnz))
    return A, np.kron(bs, np.ones(k))


def test_nodal_strength_and_one_point_brute_force():
    k = 2
    A, _ = _dense_block_case(k)
    nrp, ncol, nsq = O.node_graph(A, k)
    nsm = O.node_strength(nrp, ncol, nsq, 0.25)
    Ad = A.toarray()
    nn = A.shape[0] // k
    blk = lambda i, j: Ad[i * k:(i + 1) * k, j * k:(j + 1) * k]
    for i in range(nn):
        js = ncol[nrp[i]:nrp[i + 1]]
        norms = {j: np.linalg.norm(blk(i, j)) for j in js}
        m = max([norms[j] for j in js if j != i], default=0.0)
        for t, j in enumerate(js):
            want = j != i and norms[j] > 0 and m > 0 and norms[j] >= 0.25 * m
            assert bool(nsm[nrp[i] + t]) == want
    cf_node = O.rs_split(O.csr(nrp.astype(np.int32), ncol, np.ones(ncol.shape[0]),
                               shape=(nn, nn)), nsm)
    P = O.node_interp_one_point(nrp, ncol, nsq, nsm, cf_node, k).toarray()
    cidx, _ = O.coarse_index(cf_node)
    for i in range(nn):
        rows = P[i * k:(i + 1) * k]
        if cf_node[i] == 1:
            want = cidx[i]
        else:
            cand = [j for t, j in enumerate(ncol[nrp[i]:nrp[i + 1]])
                    if nsm[nrp[i] + t] and cf_node[j] == 1]
            want = cidx[max(cand, key=lambda j: (np.linalg.norm(blk(i, j)), -j))] \
                if cand else -1
        if want < 0:
            assert not rows.any()
        else:
            assert np.array_equal(rows[:, want * k:(want + 1) * k], np.eye(k))
            assert rows.sum() == k


def test_nodal_restriction_annihilates_neighbourhood_blocks():
    """Block form of Eq. (johnair): (R A)(i, N_i) = 0 as a k x k block for
    every C-node i and every node of N_i; the hierarchy solves."""
    k = 2
    A, b = _dense_block_case(k)
    H = O.setup(A, block=k)
    L = H.levels[0]
    RA = (L.R @ A).toarray()
    scale = (abs(L.R) @ abs(A)).toarray()
    for q in range(L.cpts.shape[0]):
        nb = L.nbr[L.nptr[q]:L.nptr[q + 1]]
        assert np.all(np.abs(RA[q, nb]) <= 1e-12 * scale[q, nb] + 1e-300)
    x, it, _ = O.solve(H, b, rtol=1e-10)
    assert np.linalg.norm(b - A @ x) <= 1e-10 * np.linalg.norm(b)


def test_nodal_rejects_blocks_that_are_not_dense():
    A, _ = _adr(8)
    with pytest.raises(ValueError):
        O.node_graph(A, 2)


# --------------------------------------------------------------------------
# Parallel (PMIS-type) CF splitting
# --------------------------------------------------------------------------

def test_hash32_published_values():
    """fmix32 of MurmurHash3: 0 maps to 0; the finalizer is a bijection on
    32-bit words (no two of 2^16 inputs collide); a hand-worked value."""
    assert int(O.hash32(0)) == 0
    h = O.hash32(np.arange(1 << 16))
    assert np.unique(h).shape[0] == 1 << 16
    x = 1
    x ^= x >> 16
    x = (x * 0x85EBCA6B) & 0xFFFFFFFF
    x ^= x >> 13
    x = (x * 0xC2B2AE35) & 0xFFFFFFFF
    x ^= x >> 16
    assert int(O.hash32(1)) == x


def _strong_pairs(A, sm):
    n = A.shape[0]
    rows = np.repeat(np.arange(n), np.diff(A.indptr))
    s = sm.astype(bool) & (A.indices != rows)
    return rows[s], A.indices[s]                  # j strongly depends on i


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_pmis_split_dominates_and_takes_local_maxima(seed):
    """Points on which nothing strongly depends are F; every other F-point
    strongly depends on a C-point; a point whose weight (count of
    dependants, hash, index) beats every point it is strongly connected to
    is C (it wins the first round); some points are C, some F."""
    A, _ = _adr(20 + 4 * seed)
    rng = np.random.default_rng(seed)
    A = A.copy()
    A.data = A.data * (1.0 + 0.5 * rng.random(A.nnz))
    sm = O.strength(A, 0.25)
    cf = O.pmis_split(A, sm)
    n = A.shape[0]
    j, i = _strong_pairs(A, sm)
    cnt = np.bincount(i, minlength=n)
    assert np.all(cf[cnt == 0] == 0)
    hasc = np.zeros(n, bool)
    hasc[j[cf[i] == 1]] = True
    assert np.all((cf == 1) | (cnt == 0) | hasc)
    key = [(int(cnt[q]), int(O.hash32(q)), q) for q in range(n)]
    nbrs = [set() for _ in range(n)]
    for a, b in zip(j, i):
        nbrs[a].add(b)
        nbrs[b].add(a)
    for q in range(n):
        if cnt[q] > 0 and all(key[q] > key[r] for r in nbrs[q] if cnt[r] > 0):
            assert cf[q] == 1
    assert 0 < (cf == 1).sum() < n


def test_pmis_split_on_a_chain_and_the_hierarchy_solves():
    """Upwind chain: point i strongly depends on i - 1 only.  The last point
    influences nothing and is F; every other F-point has its upwind
    neighbour as C.  The lAIR hierarchy built on the parallel splitting
    solves ADR to 1e-10."""
    n = 50
    A = sp.diags([np.ones(n), -np.ones(n - 1)], [0, -1], format="csr")
    A.sort_indices()
    cf = O.pmis_split(A, O.strength(A, 0.25))
    assert cf[-1] == 0
    for q in range(1, n):
        if cf[q] == 0 and q < n - 1:
            assert cf[q - 1] == 1
    B, b = _adr(24)
    H = O.setup(B, interp=O.INTERP_DIRECT, split="pmis")
    x, it, _ = O.solve(H, b, rtol=1e-10)
    assert H.nlevels >= 3 and np.linalg.norm(b - B @ x) <= 1e-10 * np.linalg.norm(b)
