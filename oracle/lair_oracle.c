/*
 * lair_oracle.c -- plain FP64 CPU reference for the lAIR setup steps.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the oracle that the GPU library is
 * checked against.  Only the tests, the smoke check and the benchmark's
 * CPU-baseline leg may load it; the solver library never does.  It shares no
 * source with the GPU path.
 *
 * Method: Manteuffel, Ruge, Southworth, "Nonsymmetric algebraic multigrid
 * based on local approximate ideal restriction (lAIR)", arXiv:1708.06065.
 * Each function is a direct, unblocked transcription of one step:
 *
 *   orc_strength      classical strength of connection (Sec. 4, the hard
 *                     minimum definition of the strong neighbourhood)
 *   orc_rs_split      classical Ruge-Stueben first pass, no second pass
 *                     (Sec. 4, coarsening paragraph; Ruge & Stueben 1987)
 *   orc_nbr_*         restriction neighbourhoods: strong F-neighbours at
 *                     distance one, or F-F-C paths at distance two (Sec. 3.1
 *                     and Sec. 4)
 *   orc_local_solves  the dense local system of Eq. (system), Sec. 3.1:
 *                     A(N,N)^T z = -A(i,N)^T, Gaussian elimination with
 *                     partial pivoting; singular systems are flagged so the
 *                     caller can take the minimal-norm least-squares solution
 *                     (Sec. 3.1, footnote on singular local systems)
 *   orc_interp_*      one-point interpolation (Sec. 4) and classical direct
 *                     interpolation (Stueben 2001, a stand-in for the
 *                     classical formulas the paper cites but does not state)
 *   orc_spgemm_*      sparse product for the Galerkin operator K = R A P
 *                     (Sec. 2.1), symbolic pattern, nothing dropped
 *   orc_lump          lumping of a coarse operator (Sec. 3.3 and the caption
 *                     of its filtering table): small entries of a row move
 *                     onto the diagonal
 *
 * All arrays are caller-owned.  Indices are int32 (CSR rowptr/col), values
 * double.  Rows of every input CSR have sorted, unique column indices.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_SOC_ABS 0
#define ORC_SOC_NEG 1

/* ------------------------------------------------------------------------ */
/* Strength of connection.                                                   */
/* j is strong for i  <=>  j != i, a_ij != 0, m_i > 0 and                    */
/*   |a_ij| >= theta m_i  (ABS)   or   -a_ij >= theta m_i  (NEG),            */
/* with m_i = max_{k != i} |a_ik|.                                            */
/* ------------------------------------------------------------------------ */
void orc_strength(int64_t n, const int32_t *rowptr, const int32_t *col,
                  const double *val, double theta, int32_t kind,
                  uint8_t *smask)
{
    for (int64_t i = 0; i < n; ++i) {
        double m = 0.0;
        for (int32_t p = rowptr[i]; p < rowptr[i + 1]; ++p)
            if (col[p] != i && fabs(val[p]) > m) m = fabs(val[p]);
        for (int32_t p = rowptr[i]; p < rowptr[i + 1]; ++p) {
            int s = 0;
            if (col[p] != i && val[p] != 0.0 && m > 0.0) {
                double a = (kind == ORC_SOC_NEG) ? -val[p] : fabs(val[p]);
                s = (a >= theta * m);
            }
            smask[p] = (uint8_t)s;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Ruge-Stueben first pass.                                                  */
/* S_i = {j : smask(i,j)} (what i strongly depends on), S_i^T = {j : i in S_j}*/
/* lambda_i = |S_i^T|.  Points with S_i and S_i^T both empty are F.          */
/* Repeat: take the undecided point of largest lambda (smallest index on a   */
/* tie); if that lambda is 0 every undecided point becomes F and we stop;    */
/* else it becomes C, every undecided j in S_i^T becomes F and each          */
/* undecided k in S_j gains 1, then every undecided j in S_i loses 1.        */
/* The arg-max is kept in a segment tree over point indices.                 */
/* ------------------------------------------------------------------------ */
typedef struct { int64_t lam; int64_t idx; } orc_key;

static int orc_better(orc_key a, orc_key b)
{
    if (a.lam != b.lam) return a.lam > b.lam;
    return a.idx < b.idx;
}

static void orc_tree_set(orc_key *t, int64_t size, int64_t i, int64_t lam)
{
    int64_t p = size + i;
    t[p].lam = lam;
    t[p].idx = i;
    for (p >>= 1; p >= 1; p >>= 1)
        t[p] = orc_better(t[2 * p], t[2 * p + 1]) ? t[2 * p] : t[2 * p + 1];
}

int32_t orc_rs_split(int64_t n, const int32_t *rowptr, const int32_t *col,
                     const uint8_t *smask, int8_t *cf)
{
    /* transpose of the strength pattern */
    int64_t *tp = calloc((size_t)n + 1, sizeof(int64_t));
    int64_t nnz = rowptr[n];
    int64_t *tj = malloc(sizeof(int64_t) * (size_t)(nnz > 0 ? nnz : 1));
    int64_t *fill = malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    int64_t *lam = calloc((size_t)n + 1, sizeof(int64_t));
    int8_t *state = malloc((size_t)(n > 0 ? n : 1)); /* -1 undecided, 0 F, 1 C */
    int64_t size = 1;
    while (size < n) size <<= 1;
    orc_key *tree = malloc(sizeof(orc_key) * (size_t)(2 * size));
    if (!tp || !tj || !fill || !lam || !state || !tree) {
        free(tp); free(tj); free(fill); free(lam); free(state); free(tree);
        return -2;
    }
    for (int64_t i = 0; i < n; ++i)
        for (int32_t p = rowptr[i]; p < rowptr[i + 1]; ++p)
            if (smask[p]) tp[col[p] + 1]++;
    for (int64_t i = 0; i < n; ++i) tp[i + 1] += tp[i];
    for (int64_t i = 0; i < n; ++i) fill[i] = tp[i];
    for (int64_t i = 0; i < n; ++i)
        for (int32_t p = rowptr[i]; p < rowptr[i + 1]; ++p)
            if (smask[p]) tj[fill[col[p]]++] = i;

    for (int64_t p = 0; p < 2 * size; ++p) { tree[p].lam = -1; tree[p].idx = INT64_MAX; }
    for (int64_t i = 0; i < n; ++i) {
        int64_t ns = 0;
        for (int32_t p = rowptr[i]; p < rowptr[i + 1]; ++p) ns += smask[p];
        lam[i] = tp[i + 1] - tp[i];
        if (ns == 0 && lam[i] == 0) {
            state[i] = 0;
        } else {
            state[i] = -1;
            tree[size + i].lam = lam[i];
            tree[size + i].idx = i;
        }
    }
    for (int64_t p = size - 1; p >= 1; --p)
        tree[p] = orc_better(tree[2 * p], tree[2 * p + 1]) ? tree[2 * p] : tree[2 * p + 1];

    for (;;) {
        orc_key top = tree[1];
        if (top.lam < 0) break;                       /* nothing undecided */
        if (top.lam == 0) {                           /* leftovers -> F */
            for (int64_t i = 0; i < n; ++i)
                if (state[i] < 0) state[i] = 0;
            break;
        }
        int64_t i = top.idx;
        state[i] = 1;
        orc_tree_set(tree, size, i, -1);
        for (int64_t q = tp[i]; q < tp[i + 1]; ++q) {
            int64_t j = tj[q];
            if (state[j] >= 0) continue;
            state[j] = 0;
            orc_tree_set(tree, size, j, -1);
            for (int32_t p = rowptr[j]; p < rowptr[j + 1]; ++p) {
                int64_t k = col[p];
                if (!smask[p] || state[k] >= 0) continue;
                lam[k] += 1;
                orc_tree_set(tree, size, k, lam[k]);
            }
        }
        for (int32_t p = rowptr[i]; p < rowptr[i + 1]; ++p) {
            int64_t j = col[p];
            if (!smask[p] || state[j] >= 0) continue;
            lam[j] -= 1;
            orc_tree_set(tree, size, j, lam[j]);
        }
    }
    for (int64_t i = 0; i < n; ++i) cf[i] = (int8_t)state[i];
    free(tp); free(tj); free(fill); free(lam); free(state); free(tree);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Restriction neighbourhoods N_i for each C-point i (ascending order).      */
/*   distance 1:  S_i intersect F                                            */
/*   distance 2:  (S_i n F)  union  (S_j n F for j in S_i n F)   (F-F-C only) */
/*   distance 0:  every F-point (test mode giving the ideal restriction)     */
/* cpts lists the C-points in increasing fine index.                         */
/* ------------------------------------------------------------------------ */
static int orc_cmp_i32(const void *a, const void *b)
{
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

static int64_t orc_nbr_one(int64_t i, int64_t n, const int32_t *rowptr,
                           const int32_t *col, const uint8_t *smask,
                           const int8_t *cf, int32_t distance,
                           int32_t *mark, int32_t stamp, int32_t *out)
{
    int64_t cnt = 0;
    if (distance == 0) {
        for (int64_t j = 0; j < n; ++j)
            if (cf[j] == 0) { if (out) out[cnt] = (int32_t)j; cnt++; }
        return cnt;
    }
    for (int32_t p = rowptr[i]; p < rowptr[i + 1]; ++p) {
        int32_t j = col[p];
        if (!smask[p] || cf[j] != 0) continue;
        if (mark[j] != stamp) { mark[j] = stamp; if (out) out[cnt] = j; cnt++; }
        if (distance >= 2) {
            for (int32_t q = rowptr[j]; q < rowptr[j + 1]; ++q) {
                int32_t k = col[q];
                if (!smask[q] || cf[k] != 0) continue;
                if (mark[k] != stamp) { mark[k] = stamp; if (out) out[cnt] = k; cnt++; }
            }
        }
    }
    if (out) qsort(out, (size_t)cnt, sizeof(int32_t), orc_cmp_i32);
    return cnt;
}

int32_t orc_nbr_count(int64_t n, const int32_t *rowptr, const int32_t *col,
                      const uint8_t *smask, const int8_t *cf, int32_t distance,
                      int64_t nc, const int32_t *cpts, int64_t *counts)
{
    int32_t *mark = malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    if (!mark) return -2;
    for (int64_t j = 0; j < n; ++j) mark[j] = -1;
    for (int64_t c = 0; c < nc; ++c)
        counts[c] = orc_nbr_one(cpts[c], n, rowptr, col, smask, cf, distance,
                                mark, (int32_t)c, NULL);
    free(mark);
    return 0;
}

int32_t orc_nbr_fill(int64_t n, const int32_t *rowptr, const int32_t *col,
                     const uint8_t *smask, const int8_t *cf, int32_t distance,
                     int64_t nc, const int32_t *cpts, const int64_t *nptr,
                     int32_t *nbr)
{
    int32_t *mark = malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    if (!mark) return -2;
    for (int64_t j = 0; j < n; ++j) mark[j] = -1;
    for (int64_t c = 0; c < nc; ++c)
        orc_nbr_one(cpts[c], n, rowptr, col, smask, cf, distance, mark,
                    (int32_t)c, nbr + nptr[c]);
    free(mark);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Local lAIR systems, Eq. (system):                                         */
/*   M[p][q] = a(l_q, l_p)   (M = A(N,N)^T),   f[p] = -a(i, l_p),            */
/* solved by Gaussian elimination with partial pivoting (largest |pivot|,    */
/* smallest row on ties).  If a pivot satisfies |u_kk| <= 1e-14 ||M||_inf    */
/* the system is flagged singular (flag = 1) and z is left at zero; the      */
/* caller then takes the minimal-norm least-squares solution.                */
/* ------------------------------------------------------------------------ */
static double orc_entry(const int32_t *rowptr, const int32_t *col,
                        const double *val, int32_t r, int32_t c)
{
    int32_t lo = rowptr[r], hi = rowptr[r + 1] - 1;
    while (lo <= hi) {
        int32_t mid = lo + (hi - lo) / 2;
        if (col[mid] == c) return val[mid];
        if (col[mid] < c) lo = mid + 1; else hi = mid - 1;
    }
    return 0.0;
}

int32_t orc_local_solves(const int32_t *rowptr, const int32_t *col,
                         const double *val, int64_t nc, const int32_t *cpts,
                         const int64_t *nptr, const int32_t *nbr, double *z,
                         int8_t *flag)
{
    int32_t status = 0;
    #pragma omp parallel
    {
        int64_t cap = 0;
        double *M = NULL, *f = NULL;
        #pragma omp for schedule(dynamic, 64)
        for (int64_t c = 0; c < nc; ++c) {
            int64_t s = nptr[c + 1] - nptr[c];
            const int32_t *l = nbr + nptr[c];
            int32_t i = cpts[c];
            flag[c] = 0;
            if (s == 0) continue;
            if (s > cap) {
                free(M); free(f);
                cap = s;
                M = malloc(sizeof(double) * (size_t)(s * s));
                f = malloc(sizeof(double) * (size_t)s);
                if (!M || !f) {
                    #pragma omp atomic write
                    status = -2;
                    cap = 0;
                    continue;
                }
            }
            for (int64_t p = 0; p < s; ++p) {
                for (int64_t q = 0; q < s; ++q)
                    M[p * s + q] = orc_entry(rowptr, col, val, l[q], l[p]);
                f[p] = -orc_entry(rowptr, col, val, i, l[p]);
            }
            double mnorm = 0.0;
            for (int64_t p = 0; p < s; ++p) {
                double r = 0.0;
                for (int64_t q = 0; q < s; ++q) r += fabs(M[p * s + q]);
                if (r > mnorm) mnorm = r;
            }
            double tol = 1e-14 * mnorm;
            int singular = 0;
            for (int64_t k = 0; k < s && !singular; ++k) {
                int64_t pr = k;
                double pv = fabs(M[k * s + k]);
                for (int64_t r = k + 1; r < s; ++r)
                    if (fabs(M[r * s + k]) > pv) { pv = fabs(M[r * s + k]); pr = r; }
                if (pv <= tol) { singular = 1; break; }
                if (pr != k) {
                    for (int64_t q = 0; q < s; ++q) {
                        double t = M[k * s + q]; M[k * s + q] = M[pr * s + q]; M[pr * s + q] = t;
                    }
                    double t = f[k]; f[k] = f[pr]; f[pr] = t;
                }
                for (int64_t r = k + 1; r < s; ++r) {
                    double mult = M[r * s + k] / M[k * s + k];
                    for (int64_t q = k + 1; q < s; ++q)
                        M[r * s + q] -= mult * M[k * s + q];
                    f[r] -= mult * f[k];
                }
            }
            double *zc = z + nptr[c];
            if (singular) {
                flag[c] = 1;
                for (int64_t p = 0; p < s; ++p) zc[p] = 0.0;
                continue;
            }
            for (int64_t k = s - 1; k >= 0; --k) {
                double acc = f[k];
                for (int64_t q = k + 1; q < s; ++q) acc -= M[k * s + q] * zc[q];
                zc[k] = acc / M[k * s + k];
            }
        }
        free(M); free(f);
    }
    return status;
}

/* ------------------------------------------------------------------------ */
/* One-point interpolation (Sec. 4): an F-point takes the value of its       */
/* strongest C-neighbour j* = argmax_{j in S_i n C} |a_ij| (smallest j on a  */
/* tie); no strong C-neighbour gives a zero row.  A C-point j injects:       */
/* P(j, cidx[j]) = 1.  pcol[i] receives the coarse column or -1.             */
/* ------------------------------------------------------------------------ */
void orc_interp_one_point(int64_t n, const int32_t *rowptr, const int32_t *col,
                          const double *val, const uint8_t *smask,
                          const int8_t *cf, const int32_t *cidx, int32_t *pcol)
{
    for (int64_t i = 0; i < n; ++i) {
        if (cf[i] == 1) { pcol[i] = cidx[i]; continue; }
        int32_t best = -1;
        double bv = -1.0;
        for (int32_t p = rowptr[i]; p < rowptr[i + 1]; ++p) {
            int32_t j = col[p];
            if (!smask[p] || cf[j] != 1) continue;
            if (fabs(val[p]) > bv) { bv = fabs(val[p]); best = j; }
        }
        pcol[i] = best >= 0 ? cidx[best] : -1;
    }
}

/* ------------------------------------------------------------------------ */
/* Classical direct interpolation (Stueben, "A review of algebraic           */
/* multigrid", 2001).  For an F-point i with interpolatory set               */
/* P_i = S_i n C and all neighbours N_i = {j != i : a_ij != 0}:              */
/*   alpha = sum_{N_i} a_ij^- / sum_{P_i} a_ik^-,                            */
/*   beta  = sum_{N_i} a_ij^+ / sum_{P_i} a_ik^+,                            */
/*   w_ik = -alpha a_ik / a_ii (a_ik < 0),  w_ik = -beta a_ik / a_ii (> 0).  */
/* When P_i has no negative (positive) entry, the negative (positive)        */
/* neighbour sum is added to the diagonal instead.  A C-point injects.       */
/* Pass 1 (fill == 0) writes per-row counts into pptr[i+1]; pass 2 fills.    */
/* ------------------------------------------------------------------------ */
void orc_interp_direct(int64_t n, const int32_t *rowptr, const int32_t *col,
                       const double *val, const uint8_t *smask,
                       const int8_t *cf, const int32_t *cidx, int32_t fill,
                       int64_t *pptr, int32_t *pcol, double *pval)
{
    for (int64_t i = 0; i < n; ++i) {
        if (cf[i] == 1) {
            if (!fill) pptr[i + 1] = 1;
            else { pcol[pptr[i]] = cidx[i]; pval[pptr[i]] = 1.0; }
            continue;
        }
        double diag = 0.0, sn = 0.0, sp = 0.0, pn = 0.0, pp = 0.0;
        int64_t cnt = 0;
        for (int32_t p = rowptr[i]; p < rowptr[i + 1]; ++p) {
            int32_t j = col[p];
            double a = val[p];
            if (j == i) { diag = a; continue; }
            if (a < 0.0) sn += a; else sp += a;
            if (smask[p] && cf[j] == 1) {
                if (a < 0.0) pn += a; else pp += a;
                cnt++;
            }
        }
        double d = diag;
        if (pn == 0.0) d += sn;
        if (pp == 0.0) d += sp;
        double alpha = (pn != 0.0) ? sn / pn : 0.0;
        double beta = (pp != 0.0) ? sp / pp : 0.0;
        if (cnt == 0 || d == 0.0) {
            if (!fill) pptr[i + 1] = 0;
            continue;
        }
        if (!fill) { pptr[i + 1] = cnt; continue; }
        int64_t o = pptr[i];
        for (int32_t p = rowptr[i]; p < rowptr[i + 1]; ++p) {
            int32_t j = col[p];
            double a = val[p];
            if (j == i || !smask[p] || cf[j] != 1) continue;
            pcol[o] = cidx[j];
            pval[o] = -(a < 0.0 ? alpha : beta) * a / d;
            o++;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Sparse product C = A B with the symbolic pattern: every (i, j) reached by */
/* a path a_ik b_kj is kept, whatever its value.  Columns come out sorted;   */
/* values are accumulated in the order of A's row entries.                   */
/* ------------------------------------------------------------------------ */
int32_t orc_spgemm_count(int64_t m, int64_t ncol_b, const int64_t *ap,
                         const int32_t *aj, const int64_t *bp,
                         const int32_t *bj, int64_t *cnt)
{
    int32_t *mark = malloc(sizeof(int32_t) * (size_t)(ncol_b > 0 ? ncol_b : 1));
    if (!mark) return -2;
    for (int64_t j = 0; j < ncol_b; ++j) mark[j] = -1;
    for (int64_t i = 0; i < m; ++i) {
        int64_t c = 0;
        for (int64_t p = ap[i]; p < ap[i + 1]; ++p) {
            int32_t k = aj[p];
            for (int64_t q = bp[k]; q < bp[k + 1]; ++q) {
                int32_t j = bj[q];
                if (mark[j] != (int32_t)i) { mark[j] = (int32_t)i; c++; }
            }
        }
        cnt[i] = c;
    }
    free(mark);
    return 0;
}

int32_t orc_spgemm_fill(int64_t m, int64_t ncol_b, const int64_t *ap,
                        const int32_t *aj, const double *ax, const int64_t *bp,
                        const int32_t *bj, const double *bx, const int64_t *cp,
                        int32_t *cj, double *cx)
{
    int64_t *pos = malloc(sizeof(int64_t) * (size_t)(ncol_b > 0 ? ncol_b : 1));
    double *acc = malloc(sizeof(double) * (size_t)(ncol_b > 0 ? ncol_b : 1));
    if (!pos || !acc) { free(pos); free(acc); return -2; }
    for (int64_t j = 0; j < ncol_b; ++j) { pos[j] = -1; acc[j] = 0.0; }
    for (int64_t i = 0; i < m; ++i) {
        int64_t c = cp[i];
        for (int64_t p = ap[i]; p < ap[i + 1]; ++p) {
            int32_t k = aj[p];
            for (int64_t q = bp[k]; q < bp[k + 1]; ++q) {
                int32_t j = bj[q];
                if (pos[j] < 0) { pos[j] = c; cj[c] = j; c++; }
                acc[j] += ax[p] * bx[q];
            }
        }
        qsort(cj + cp[i], (size_t)(c - cp[i]), sizeof(int32_t), orc_cmp_i32);
        for (int64_t t = cp[i]; t < c; ++t) {
            int32_t j = cj[t];
            cx[t] = acc[j];
            acc[j] = 0.0;
            pos[j] = -1;
        }
    }
    free(pos); free(acc);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Lumping (Sec. 3.3).  In row i, an off-diagonal entry with                 */
/*   |k_ij| < theta_D max_j |k_ij|   (the maximum over the whole row, the    */
/*                                    diagonal included)                     */
/* is removed and added to k_ii, so the row sum is kept.  The removed        */
/* entries are summed in column order first, then added to k_ii.  A row      */
/* without a stored diagonal, or without an off-diagonal entry, is kept      */
/* whole.  keep[p] = 1 for every entry that stays; pass 1 (fill == 0)        */
/* writes keep and the kept count of row i into cnt[i]; pass 2 writes the    */
/* lumped row at out_ptr[i].                                                 */
/* ------------------------------------------------------------------------ */
void orc_lump(int64_t m, const int32_t *rp, const int32_t *cj, const double *v,
              double theta, int32_t fill, uint8_t *keep, int64_t *cnt,
              const int64_t *out_ptr, int32_t *out_cj, double *out_v)
{
    for (int64_t i = 0; i < m; ++i) {
        if (!fill) {
            double mx = 0.0;
            int has_d = 0, has_o = 0;
            for (int32_t p = rp[i]; p < rp[i + 1]; ++p) {
                if (cj[p] == i) has_d = 1; else has_o = 1;
                if (fabs(v[p]) > mx) mx = fabs(v[p]);
            }
            int64_t c = 0;
            for (int32_t p = rp[i]; p < rp[i + 1]; ++p) {
                int k = 1;
                if (has_d && has_o && cj[p] != i && fabs(v[p]) < theta * mx) k = 0;
                keep[p] = (uint8_t)k;
                c += k;
            }
            cnt[i] = c;
            continue;
        }
        double gone = 0.0;
        for (int32_t p = rp[i]; p < rp[i + 1]; ++p)
            if (!keep[p]) gone += v[p];
        int64_t o = out_ptr[i];
        for (int32_t p = rp[i]; p < rp[i + 1]; ++p) {
            if (!keep[p]) continue;
            out_cj[o] = cj[p];
            out_v[o] = (cj[p] == i) ? v[p] + gone : v[p];
            o++;
        }
    }
}
