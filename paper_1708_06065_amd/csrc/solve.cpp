// liblair cycles and solves: the V-cycle schedule (coarse-grid correction,
// then F, F, C Jacobi), its transpose, the outer iterations (stationary,
// flexible GMRES, per-system batch) and their HIP graphs.  Every arithmetic
// step runs in the HIP kernels of k_cycle.hip, k_krylov.hip and k_batch.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <climits>
#include <cmath>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "hierarchy.hpp"

namespace lair {

__global__ void k_add(double *x, const double *e, int64_t m) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m) x[i] += e[i];
}

// ---------------------------------------------------------------------------
// Cycle
// ---------------------------------------------------------------------------
static void ensure_vectors(lair_hierarchy *h, int32_t nrhs, hipStream_t s) {
    if (nrhs <= h->nrhs_cap) return;
    h->drop_graphs();     // captured iterations refer to the old buffers
    // a failed allocation below leaves no capacity claimed, so the next call
    // allocates every vector again
    h->nrhs_cap = 0;
    for_each_cycle_vector(h, nrhs, [&](auto &a, size_t count) { a.alloc(count, s); });
    h->partial.alloc((size_t)NPARTIAL * nrhs, s);
    h->norms.alloc((size_t)nrhs, s);
    h->nrhs_cap = nrhs;
}

// Algorithmic bytes of the cycle operations (w = value size, R = number of
// right-hand sides): every matrix entry (index + value), row pointer, source
// vector entry and destination entry counted once.
static double ab_rowdot(const DevCSR &M, int w, int R, int vec_in_out) {
    return (4.0 + w) * (double)M.nnz + 4.0 * (M.nrows + 1) + (double)w * R * M.ncols +
           (double)w * R * M.nrows * vec_in_out;
}
static double ab_jacobi(int64_t nnz_x, int32_t nx, int32_t n, int w, int R, bool sel) {
    return (4.0 + w) * (double)nnz_x + 12.0 * nx + (double)w * R * n + 2.0 * w * R * nx +
           (sel ? (double)n : 0.0);
}

template <class VT>
static void coarse_solve(lair_hierarchy *h, const VT *b, VT *x, int32_t nrhs,
                         bool transpose, hipStream_t s) {
    const int w = sizeof(VT);
    ProfScope ps("coarse_solve", s, 8.0 * h->coarse_entries + 2.0 * w * nrhs * h->nL,
                 2.0 * h->coarse_entries * nrhs);
    if (h->nsys > 1) {
        Level &Lb = *h->L.back();
        const uint8_t *act = h->use_act ? h->active_dev.get() : nullptr;
        auto block_solve = [&](const double *bb, double *xx) {
            if (h->binv.get())
                launch_block_apply_inv(h->nsys, Lb.seg_dev.get(), h->dense_off.get(),
                                       h->binv.get(), bb, xx, transpose, s, act,
                                       h->use_inv.get());
            launch_block_solve(h->nsys, Lb.seg_dev.get(), h->dense_off.get(), h->lu.get(),
                               h->piv.get(), bb, xx, transpose, s, act,
                               h->binv.get() ? h->use_inv.get() : nullptr);
        };
        if constexpr (std::is_same<VT, double>::value) {
            block_solve(b, x);
        } else {
            op_cast_f64(b, Lb.r.get(), h->nL, s);
            block_solve(Lb.r.get(), Lb.x.get());
            op_cast_f32(Lb.x.get(), x, h->nL, s);
        }
        return;
    }
    if (h->kinv.get()) {
        op_coarse_apply<VT>(h->nL, h->kinv.get(), b, x, nrhs, transpose, s);
        return;
    }
    Level &Lc = *h->L.back();
    if constexpr (std::is_same<VT, double>::value) {
        op_dense_solve<double>(h->nL, h->lu.get(), h->piv.get(), b, x, nrhs, transpose, s);
    } else {
        int64_t m = (int64_t)h->nL * nrhs;
        op_cast_f64(b, Lc.r.get(), m, s);
        op_dense_solve<double>(h->nL, h->lu.get(), h->piv.get(), Lc.r.get(), Lc.x.get(),
                               nrhs, transpose, s);
        op_cast_f32(Lc.x.get(), x, m, s);
    }
}

// F, F, C Jacobi sweeps on a level, every sweep reading the previous iterate.
// X is the iterate, Y a level-sized buffer:
//   F sweep 1 reads X, writes Y at the F rows;
//   F sweep 2 reads Y at F-points and X at C-points, writes X at the F rows
//     (X's F entries are not read by this sweep);
//   C sweep reads X, writes a compact buffer that is then scattered to X.
// With leave_c the C sweep writes Y's C rows instead and nothing is copied:
// the result is X at the F rows and Y at the C rows (on a split-ordered
// level, X below nf and Y from nf on).  Returns whether it did so.
template <class VT>
static bool ffc(lair_hierarchy *h, Level &Lv, const VT *b, VT *x, int32_t nrhs,
                hipStream_t s, bool leave_c) {
    const bool split = Lv.split;
    CsrView<VT> A = view<VT>(split ? Lv.As : Lv.A, Lv.team_A);
    if (nodal(h->opt)) {
        // block Jacobi x_X + D_X^{-1} (b - A x)_X is the scalar Jacobi sweep
        // on D^{-1} A (unit diagonal blocks) with right-hand side D^{-1} b
        VT *bt = vec<VT>(Lv.bt, Lv.bt32);
        {
            ProfScope ps("jacobi", s, 8.0 * Lv.n * h->opt.block_size +
                                          2.0 * sizeof(VT) * nrhs * Lv.n,
                         2.0 * Lv.n * h->opt.block_size * nrhs);
            op_node_rhs<VT>(Lv.n, h->opt.block_size, nrhs, Lv.ndinv.get(), b, bt, s);
        }
        b = bt;
        if constexpr (std::is_same<VT, double>::value) A.v = Lv.av.get();
        else A.v = Lv.av32.get();
    }
    VT *y = vec<VT>(Lv.t, Lv.t32);
    double om = h->opt.omega;
    const int w = sizeof(VT);
    // batch solve: only the rows of the systems still iterated (device lists)
    const bool act = h->use_act;
    // split ordering: F rows are 0 .. nf-1 and C rows nf .. n-1 (no list)
    const int32_t *frows = act ? Lv.act_f.get() : (split ? nullptr : Lv.flist.get());
    const int32_t *fcnt = act ? Lv.act_cnt + 1 : nullptr;
    {
        ProfScope ps("jacobi", s, ab_jacobi(Lv.nnzF, Lv.nf, Lv.n, w, nrhs, false),
                     2.0 * Lv.nnzF * nrhs);
        op_jacobi<VT>(A, frows, Lv.nf, b, x, x, nullptr, y, false, om, nrhs, s, fcnt);
    }
    {
        ProfScope ps("jacobi", s, ab_jacobi(Lv.nnzF, Lv.nf, Lv.n, w, nrhs, true),
                     2.0 * Lv.nnzF * nrhs);
        CsrView<VT> At = A;
        At.cjt = split ? Lv.cjt_split.get() : Lv.cjt.get();
        op_jacobi<VT>(At, frows, Lv.nf, b, y, x, split ? Lv.cf_split.get() : Lv.cf.get(), x,
                      false, om, nrhs, s, fcnt);
    }
    const int32_t *crows = act ? Lv.act_c.get()
                               : split ? nullptr
                               : (Lv.nrc >= 0 ? Lv.rclist.get() : Lv.clist.get());
    const int32_t *ccnt = act ? Lv.act_cnt + 2 : nullptr;
    const int32_t ncr = Lv.nrc >= 0 ? Lv.nrc : Lv.nc;
    const int32_t c0 = split ? Lv.nf : 0;
    leave_c = leave_c && !act && Lv.nrc < 0;
    {
        ProfScope ps("jacobi", s, ab_jacobi(Lv.nnzC, ncr, Lv.n, w, nrhs, false),
                     2.0 * Lv.nnzC * nrhs);
        op_jacobi<VT>(A, crows, ncr, b, x, x, nullptr, y, !leave_c, om, nrhs, s, ccnt, c0);
    }
    if (leave_c) return true;
    {
        ProfScope ps("scatter", s, 4.0 * ncr + 2.0 * w * nrhs * ncr);
        op_scatter<VT>(crows, ncr, y, x, nrhs, s, ccnt, c0);
    }
    return false;
}

// V-cycle from level l.  With x_zero the incoming iterate is zero: the
// residual is b itself and the interpolated correction is assigned.  When
// r is non-null it already holds b - A x.  With split_out the result may be
// left split (see ffc): the return value is then the buffer that holds its
// C rows, otherwise nullptr (x holds all of it).
template <class VT>
static const VT *vcycle(lair_hierarchy *h, size_t l, const VT *b, VT *x, bool x_zero,
                        const VT *r, int32_t nrhs, hipStream_t s, bool split_out = false) {
    Level &Lv = *h->L[l];
    const int w = sizeof(VT);
    if (l + 1 == h->L.size()) {
        coarse_solve<VT>(h, b, x, nrhs, false, s);
        return nullptr;
    }
    Level &Nx = *h->L[l + 1];
    const VT *res = b;
    if (!x_zero) {
        if (r) {
            res = r;
        } else {
            VT *rr = vec<VT>(Lv.r, Lv.r32);
            ProfScope ps("residual", s, ab_rowdot(Lv.A, w, nrhs, 2), 2.0 * Lv.A.nnz * nrhs);
            op_residual<VT>(view<VT>(Lv.split ? Lv.As : Lv.A, Lv.team_A), b, x, rr, nrhs, s);
            res = rr;
        }
    }
    VT *bc = vec<VT>(Nx.b, Nx.b32);
    VT *xc = vec<VT>(Nx.x, Nx.x32);
    {
        ProfScope ps("restrict", s, ab_rowdot(Lv.R, w, nrhs, 1), 2.0 * Lv.R.nnz * nrhs);
        if (h->use_act)
            op_rowdot_list<VT>(view<VT>(Lv.R, Lv.team_R), 1, Nx.act_rows.get(),
                               Nx.act_cnt, Nx.n, res, nullptr, bc, s);
        else
            op_spmv<VT>(view<VT>(Lv.Rs.rp.get() ? Lv.Rs : Lv.R, Lv.team_R), res, bc, nrhs, false,
                        s);
    }
    // the coarse correction may come back in two buffers (its C rows in the
    // level's work buffer); the interpolation then reads those columns there
    const bool coarse_split = !h->use_act &&
                              op_spmv_split_ok(nrhs, xc, vec<VT>(Nx.t, Nx.t32), x);
    const VT *xc_hi = vcycle<VT>(h, l + 1, bc, xc, true, nullptr, nrhs, s, coarse_split);
    {
        ProfScope ps("interpolate", s, ab_rowdot(Lv.P, w, nrhs, x_zero ? 1 : 2),
                     2.0 * Lv.P.nnz * nrhs);
        if (h->use_act)
            op_rowdot_list<VT>(view<VT>(Lv.P, Lv.team_P), x_zero ? 1 : 2, Lv.act_rows.get(),
                               Lv.act_cnt, Lv.n, xc, nullptr, x, s);
        else
            op_spmv<VT>(view<VT>(Lv.Ps.rp.get() ? Lv.Ps : Lv.P, Lv.team_P), xc, x, nrhs, !x_zero,
                        s, xc_hi, Nx.split && nrhs > 1 ? Nx.nf : -1,
                        Nx.split ? Nx.cf_split.get() : Nx.cf.get());
    }
    return ffc<VT>(h, Lv, b, x, nrhs, s, split_out) ? vec<VT>(Lv.t, Lv.t32) : nullptr;
}

// Transposed cycle: C, F, F Jacobi on A^T, restriction with P^T, recursion
// on K^T, interpolation with R^T.
static void ensure_transposes(lair_hierarchy *h) {
    if (h->have_transpose) return;
    hipStream_t s = h->stream;
    DevArr<int64_t> tmp;
    for (size_t l = 0; l < h->L.size(); ++l) {
        Level &Lv = *h->L[l];
        transpose(Lv.A, Lv.At, s, tmp);
        Lv.team_At = team_of(Lv.At);
        if (l + 1 == h->L.size()) break;
        transpose(Lv.R, Lv.Rt, s, tmp);
        transpose(Lv.P, Lv.Pt, s, tmp);
        Lv.team_Rt = team_of(Lv.Rt);
        Lv.team_Pt = team_of(Lv.Pt);
    }
    LAIR_HIP(hipStreamSynchronize(s));
    h->have_transpose = true;
}

static void vcycle_t(lair_hierarchy *h, size_t l, const double *g, double *lam,
                     bool lam_zero, int32_t nrhs, hipStream_t s) {
    Level &Lv = *h->L[l];
    if (l + 1 == h->L.size()) {
        coarse_solve<double>(h, g, lam, nrhs, true, s);
        return;
    }
    if (lam_zero) op_fill<double>(lam, 0.0, (int64_t)Lv.n * nrhs, s);
    CsrView<double> At = view<double>(Lv.At, Lv.team_At);
    double om = h->opt.omega;
    const int32_t *crows = Lv.nrc >= 0 ? Lv.rclist.get() : Lv.clist.get();
    const int32_t ncr = Lv.nrc >= 0 ? Lv.nrc : Lv.nc;
    for (int sweep = 0; sweep < 3; ++sweep) {
        const int32_t *rows = sweep == 0 ? crows : Lv.flist.get();
        int32_t nx = sweep == 0 ? ncr : Lv.nf;
        op_jacobi<double>(At, rows, nx, g, lam, lam, nullptr, Lv.t.get(), true, om, nrhs, s);
        op_scatter<double>(rows, nx, Lv.t.get(), lam, nrhs, s);
    }
    op_residual<double>(At, g, lam, Lv.r.get(), nrhs, s);
    Level &Nx = *h->L[l + 1];
    op_spmv<double>(view<double>(Lv.Pt, Lv.team_Pt), Lv.r.get(), Nx.b.get(), nrhs, false, s);
    vcycle_t(h, l + 1, Nx.b.get(), Nx.x.get(), true, nrhs, s);
    op_spmv<double>(view<double>(Lv.Rt, Lv.team_Rt), Nx.x.get(), lam, nrhs, true, s);
}

static bool valid_nrhs(int32_t nrhs) {
    return nrhs == 1 || nrhs == 2 || nrhs == 4 || nrhs == 8 || nrhs == 16 || nrhs == 32;
}

void check_nrhs(const lair_hierarchy *h, int32_t nrhs) {
    if (!valid_nrhs(nrhs)) fail(LAIR_EINVAL, "nrhs must be 1, 2, 4, 8, 16 or 32");
    if (h->nsys > 1 && nrhs != 1)
        fail(LAIR_EINVAL, "a hierarchy of a batch takes one right-hand side per system");
}

static void sumsq_dev(lair_hierarchy *h, const double *r, int32_t nrhs, hipStream_t s) {
    ProfScope ps("norm", s, 8.0 * nrhs * h->L[0]->n, 2.0 * nrhs * h->L[0]->n);
    op_sumsq(r, h->L[0]->n, nrhs, h->partial.get(), NPARTIAL, h->norms.get(), s);
}

// Square roots of the m sums of squares at dev (synchronises s).
static void read_norms(const double *dev, int32_t m, hipStream_t s, std::vector<double> &out) {
    out.resize((size_t)m);
    {
        Readback rb(s);
        rb.add(out.data(), dev, sizeof(double) * m);
        rb.run();
    }
    for (auto &v : out) v = std::sqrt(v);
}

static void norms_host(lair_hierarchy *h, const double *r, int32_t nrhs,
                       hipStream_t s, std::vector<double> &out) {
    sumsq_dev(h, r, nrhs, s);
    read_norms(h->norms.get(), nrhs, s, out);
}

// Kinds of captured iterations.
enum { IT_FP64 = 0, IT_MIXED = 1, IT_BATCH_FP64 = 2, IT_BATCH_MIXED = 3 };

static const char *const CYCLE_CATEGORIES[] = {
    "jacobi", "scatter", "residual", "restrict", "interpolate", "coarse_solve", "norm", "cast"};

// Iterations are captured unless the caller asked for eager launches or the
// profiler times one of the cycle's categories (its events would have to be
// recorded launch by launch).
static bool use_graphs(const lair_hierarchy *h) {
    if (h->opt.flags & LAIR_FLAG_NO_GRAPH) return false;
    for (const char *c : CYCLE_CATEGORIES)
        if (prof_selected(c)) return false;
    return true;
}

static const size_t MAX_GRAPHS = 8;

// Run body(stream) on s: replay its captured graph.  The first iteration of
// a kind is launched directly on s and then captured on the hierarchy's
// private stream, so that the capture and the instantiation (host work of
// a few hundred microseconds for a deep cycle) run while the device executes
// that first iteration; later ones replay the graph.  body must launch
// kernels only (no allocation, no host synchronisation, no memset).
template <class Body>
static void run_iteration(lair_hierarchy *h, int kind, int32_t nrhs, const void *b, void *x,
                          hipStream_t s, Body &&body) {
    if (!use_graphs(h)) {
        body(s);
        return;
    }
    for (auto &g : h->graphs)
        if (g.kind == kind && g.nrhs == nrhs && g.b == b && g.x == x) {
            LAIR_HIP(hipGraphLaunch(g.exec, s));
            return;
        }
    body(s);
    if (!h->gstream) LAIR_HIP(hipStreamCreateWithFlags(&h->gstream, hipStreamNonBlocking));
    hipGraph_t graph = nullptr;
    LAIR_HIP(hipStreamBeginCapture(h->gstream, hipStreamCaptureModeThreadLocal));
    try {
        body(h->gstream);
    } catch (...) {
        if (hipStreamEndCapture(h->gstream, &graph) == hipSuccess && graph)
            (void)hipGraphDestroy(graph);
        throw;
    }
    LAIR_HIP(hipStreamEndCapture(h->gstream, &graph));
    hipGraphExec_t exec = nullptr;
    hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) fail(LAIR_EDEVICE, "graph instantiation failed: %s", hipGetErrorString(e));
    if (h->graphs.size() >= MAX_GRAPHS) {
        (void)hipGraphExecDestroy(h->graphs.front().exec);
        h->graphs.erase(h->graphs.begin());
    }
    h->graphs.push_back({kind, nrhs, b, x, exec});
}

static void check_solve_args(lair_hierarchy *h, const double *b, double *x, double rtol,
                             int32_t maxit) {
    if (!h) fail(LAIR_EINVAL, "hierarchy is NULL");
    if (!b || !x) fail(LAIR_EINVAL, "b and x must not be NULL");
    if (!(rtol > 0.0) || maxit < 0) fail(LAIR_EINVAL, "need rtol > 0 and maxit >= 0");
}

void info_common(const lair_hierarchy *h, lair_info *info) {
    info->nlevels = (int32_t)h->L.size();
    info->cycle_complexity = h->cc;
    info->op_complexity = h->oc;
    info->n_singular_local = h->n_singular;
    info->setup_ms = h->setup_ms;
    info->split_ms = h->split_ms;
    for (int k = 0; k < 8; ++k) info->setup_phase_ms[k] = h->phase_ms[k];
    // Sec. 4: work units per digit of accuracy, -CC / log10(rho)
    info->wpd = (info->rho > 0.0 && info->rho < 1.0)
                    ? -h->cc / std::log10(info->rho) : 0.0;
    info->hist_len = 0;
}

static void set_history(lair_info *info, const std::vector<double> &hist) {
    const size_t m = std::min(hist.size(), (size_t)LAIR_HIST_MAX);
    for (size_t k = 0; k < m; ++k) info->relres_hist[k] = hist[k];
    info->hist_len = (int32_t)m;
}

lair_status solve_impl(lair_hierarchy *h, const double *b, double *x,
                       int32_t nrhs, double rtol, int32_t maxit,
                       lair_info *info, hipStream_t s, bool transpose) {
    auto t0 = Clock::now();
    check_solve_args(h, b, x, rtol, maxit);
    check_nrhs(h, nrhs);
    ensure_vectors(h, nrhs, s);
    if (transpose) ensure_transposes(h);
    Level &L0 = *h->L[0];
    const int64_t n = L0.n;
    const double *bb = b;
    if (scaled(h->opt) && !transpose) {
        op_block_apply(n / h->opt.block_size, h->opt.block_size, h->dinv.get(), b,
                       h->bscaled.get(), nrhs, s);
        bb = h->bscaled.get();
    }
    bool mixed = h->opt.precision == LAIR_MIXED && !transpose;
    // level 0 renumbered for the cycle: the FP64 iteration carries b and x
    // in the split ordering (x is written back at the end); the mixed one
    // keeps them natural, writes its float residual in the split ordering
    // and adds the correction back row by row
    const bool split = L0.split && !transpose;
    const bool vec_split = split && !mixed;
    const int32_t *orow = split && mixed ? L0.iperm.get() : nullptr;
    double *const xu = x;
    if (vec_split) {
        op_permute_rows(n, nrhs, L0.perm.get(), bb, h->bsplit.get(), true, s);
        op_permute_rows(n, nrhs, L0.perm.get(), x, h->xsplit.get(), true, s);
        bb = h->bsplit.get();
        x = h->xsplit.get();
    }
    std::vector<double> nb, rn, r_first;
    norms_host(h, bb, nrhs, s, nb);
    CsrView<double> A0 = transpose ? view<double>(L0.At, L0.team_At)
                                   : view<double>(vec_split ? L0.As : L0.A, L0.team_A);
    const DevCSR &M0 = transpose ? L0.At : L0.A;
    // fused residual + norms (+ float copy in mixed precision) unless the
    // caller's vectors are not 16-byte aligned
    const bool fused = nrhs == 1 || (((uintptr_t)bb | (uintptr_t)x) & 15u) == 0;
    auto residual_and_norms = [&](hipStream_t st) {
        if (fused) {
            ProfScope ps("residual", st, ab_rowdot(M0, 8, nrhs, 1) + (mixed ? 4.0 : 8.0) *
                         nrhs * (double)M0.nrows, 2.0 * M0.nnz * nrhs);
            if (!op_residual_norm(A0, bb, x, mixed ? nullptr : h->r0.get(),
                                  mixed ? h->r0_32.get() : nullptr, nrhs, h->partial.get(),
                                  NPARTIAL, h->norms.get(), st, orow))
                fail(LAIR_EDEVICE, "fused residual not applicable");
            return;
        }
        {
            ProfScope ps("residual", st, ab_rowdot(M0, 8, nrhs, 2), 2.0 * M0.nnz * nrhs);
            op_residual<double>(A0, bb, x, h->r0.get(), nrhs, st);
        }
        sumsq_dev(h, h->r0.get(), nrhs, st);
    };
    residual_and_norms(s);
    read_norms(h->norms.get(), nrhs, s, rn);
    r_first = rn;
    int32_t it = 0;
    double relmax = 0.0;
    std::vector<double> hist;
    for (;;) {
        relmax = 0.0;
        bool done = true;
        for (int32_t q = 0; q < nrhs; ++q) {
            double rel = nb[q] > 0 ? rn[q] / nb[q] : rn[q];
            relmax = std::max(relmax, rel);
            if (!(rel <= rtol)) done = false;
        }
        hist.push_back(relmax);
        if (done || it >= maxit) break;
        if (transpose) {
            // lambda <- lambda + B^T (g - A^T lambda): cycle on the residual
            DevArr<double> &e = L0.b;
            vcycle_t(h, 0, h->r0.get(), e.get(), true, nrhs, s);
            LAIR_LAUNCH(k_add, dim3(blocks_for(n * nrhs, 256)), dim3(256), 0, s,
                               x, e.get(), n * nrhs);
            LAIR_LAUNCH_CHECK();
            residual_and_norms(s);
        } else if (!mixed) {
            run_iteration(h, IT_FP64, nrhs, bb, x, s, [&](hipStream_t st) {
                vcycle<double>(h, 0, bb, x, false, h->r0.get(), nrhs, st);
                residual_and_norms(st);
            });
        } else {
            run_iteration(h, IT_MIXED, nrhs, bb, x, s, [&](hipStream_t st) {
                if (!fused) {
                    ProfScope ps("cast", st, 12.0 * n * nrhs);
                    if (orow) op_cast_f32_rows(h->r0.get(), h->r0_32.get(), orow, n, nrhs, st);
                    else op_cast_f32(h->r0.get(), h->r0_32.get(), n * nrhs, st);
                }
                // the split-ordered correction may come back in two pieces
                const float *e_hi = vcycle<float>(h, 0, h->r0_32.get(), h->e32.get(), true,
                                                  nullptr, nrhs, st, orow != nullptr);
                {
                    ProfScope ps("cast", st, 20.0 * n * nrhs);
                    if (orow) op_axpy_f32_rows(x, h->e32.get(), orow, n, nrhs, st, e_hi, L0.nf);
                    else op_axpy_f32(x, h->e32.get(), n * nrhs, st);
                }
                residual_and_norms(st);
            });
        }
        read_norms(h->norms.get(), nrhs, s, rn);
        ++it;
    }
    if (vec_split) op_permute_rows(n, nrhs, L0.perm.get(), x, xu, false, s);
    LAIR_HIP(hipStreamSynchronize(s));
    if (info) {
        info->iters = it;
        info->relres = relmax;
        double rho = 0.0;
        if (it > 0 && !r_first.empty()) {
            for (int32_t q = 0; q < nrhs; ++q)
                if (r_first[q] > 0) rho = std::max(rho, std::pow(rn[q] / r_first[q], 1.0 / it));
        }
        info->rho = rho;
        info_common(h, info);
        set_history(info, hist);
        info->solve_ms = ms_since(t0);
    }
    return relmax <= rtol ? LAIR_OK : LAIR_ENOCONV;
}

// Flexible GMRES(m), right preconditioned (Saad 1993), with one V-cycle from
// zero as the preconditioner: the outer solver of the paper's results
// (Sec. 4).  Each right-hand side has its own Krylov space, Hessenberg
// matrix and Givens rotations (host), in shared device bases V (m + 1
// vectors) and Z (m vectors) of n x nrhs doubles in the natural ordering.
// Arnoldi: classical Gram-Schmidt applied twice.  A right-hand side whose
// residual estimate reaches rtol ||b|| is frozen (its next basis vectors are
// zero) and updated with its own number of steps; a cycle of m steps ends
// with the true residual, which decides whether to restart.
lair_status solve_fgmres_impl(lair_hierarchy *h, const double *b, double *x,
                              int32_t nrhs, double rtol, int32_t maxit, int32_t m,
                              lair_info *info, hipStream_t s) {
    auto t0 = Clock::now();
    check_solve_args(h, b, x, rtol, maxit);
    check_nrhs(h, nrhs);
    if (h->batch) fail(LAIR_EUNSUPPORTED, "FGMRES is for a single system");
    if (m < 1 || m > 64) fail(LAIR_EINVAL, "restart must be in [1, 64] (got %d)", m);
    ensure_vectors(h, nrhs, s);
    Level &L0 = *h->L[0];
    const int64_t n = L0.n;
    const int32_t R = nrhs;
    const int64_t nv = n * R;
    const bool mixed = h->opt.precision == LAIR_MIXED;
    const bool split = L0.split;
    const double *bb = b;
    if (scaled(h->opt)) {
        op_block_apply(n / h->opt.block_size, h->opt.block_size, h->dinv.get(), b,
                       h->bscaled.get(), nrhs, s);
        bb = h->bscaled.get();
    }
    CsrView<double> A0 = view<double>(L0.A, L0.team_A);
    DevArr<double> V, Z, w, coef, dots, partial, scale;
    V.alloc((size_t)(m + 1) * nv, s);
    Z.alloc((size_t)m * nv, s);
    w.alloc((size_t)nv, s);
    coef.alloc((size_t)(m + 1) * R, s);
    // dots: both Gram-Schmidt passes' coefficients, then |w|^2
    const size_t HOFF = (size_t)(m + 1) * R;
    dots.alloc(2 * HOFF + R, s);
    partial.alloc((size_t)kry_dot_blocks(nv) * (m + 1) * R, s);
    scale.alloc((size_t)R, s);
    double *Vp = V.get(), *Zp = Z.get();
    auto Vk = [&](int k) { return Vp + (int64_t)k * nv; };
    auto Zk = [&](int k) { return Zp + (int64_t)k * nv; };
    // z = B v: one V-cycle from zero, in the cycle's ordering and precision
    auto precond = [&](const double *v, double *z) {
        if (mixed) {
            if (split) op_cast_f32_rows(v, h->r0_32.get(), L0.iperm.get(), n, R, s);
            else op_cast_f32(v, h->r0_32.get(), nv, s);
            vcycle<float>(h, 0, h->r0_32.get(), h->e32.get(), true, nullptr, R, s);
            op_fill<double>(z, 0.0, nv, s);
            if (split) op_axpy_f32_rows(z, h->e32.get(), L0.iperm.get(), n, R, s);
            else op_axpy_f32(z, h->e32.get(), nv, s);
        } else if (split) {
            op_permute_rows(n, R, L0.perm.get(), v, h->bsplit.get(), true, s);
            vcycle<double>(h, 0, h->bsplit.get(), h->xsplit.get(), true, nullptr, R, s);
            op_permute_rows(n, R, L0.perm.get(), h->xsplit.get(), z, false, s);
        } else {
            vcycle<double>(h, 0, v, z, true, nullptr, R, s);
        }
    };
    auto upload = [&](double *dev, const std::vector<double> &hv) {
        double *st = (double *)pinned_upload(sizeof(double) * hv.size());
        memcpy(st, hv.data(), sizeof(double) * hv.size());
        LAIR_HIP(hipMemcpyAsync(dev, st, sizeof(double) * hv.size(), hipMemcpyHostToDevice, s));
        LAIR_HIP(hipStreamSynchronize(s));     // the staging area is reused
    };
    // r = b - A x into V_0 and its norms
    auto true_residual = [&](std::vector<double> &beta) {
        op_residual<double>(A0, bb, x, Vk(0), R, s);
        op_mdot(n, R, Vk(0), nv, 1, Vk(0), partial.get(), dots.get(), s);
        read_norms(dots.get(), R, s, beta);
    };
    std::vector<double> nb, beta, r_first;
    norms_host(h, bb, R, s, nb);
    std::vector<double> tol((size_t)R);
    for (int32_t q = 0; q < R; ++q) tol[q] = rtol * nb[q];
    true_residual(beta);
    r_first = beta;
    std::vector<int32_t> its((size_t)R, 0);
    const size_t H1 = (size_t)m + 1;
    std::vector<double> Hh(H1 * m * R), cs((size_t)m * R), sn((size_t)m * R), g(H1 * R);
    std::vector<double> hc(2 * HOFF + R), sc((size_t)R), cf((size_t)(m + 1) * R);
    std::vector<int32_t> kq((size_t)R);
    std::vector<char> act((size_t)R);
    int32_t it = 0;
    for (;;) {
        bool any = false;
        for (int32_t q = 0; q < R; ++q) {
            act[q] = !(beta[q] <= tol[q]);
            any = any || act[q];
        }
        if (!any || it >= maxit) break;
        // V_0 = r / beta for the right-hand sides still iterated
        for (int32_t q = 0; q < R; ++q) {
            sc[q] = act[q] ? 1.0 / beta[q] : 0.0;
            kq[q] = 0;
            g[q] = act[q] ? beta[q] : 0.0;
            for (size_t i = 1; i < H1; ++i) g[i * R + q] = 0.0;
        }
        upload(scale.get(), sc);
        op_scale_rhs(n, R, Vk(0), scale.get(), Vk(0), s);
        for (int j = 0; j < m; ++j) {
            precond(Vk(j), Zk(j));
            op_spmv<double>(A0, Zk(j), w.get(), R, false, s);
            // Gram-Schmidt twice: c = V^T w, w -= V c; h = c1 + c2
            for (int pass = 0; pass < 2; ++pass) {
                double *cd = dots.get() + (size_t)pass * HOFF;
                op_mdot(n, R, Vp, nv, j + 1, w.get(), partial.get(), cd, s);
                op_maxpy(n, R, Vp, nv, j + 1, cd, w.get(), s);
            }
            op_mdot(n, R, w.get(), nv, 1, w.get(), partial.get(), dots.get() + 2 * HOFF, s);
            {
                Readback rb(s);
                rb.add(hc.data(), dots.get(), sizeof(double) * (j + 1) * R);
                rb.add(hc.data() + HOFF, dots.get() + HOFF, sizeof(double) * (j + 1) * R);
                rb.add(hc.data() + 2 * HOFF, dots.get() + 2 * HOFF, sizeof(double) * R);
                rb.run();
            }
            for (int i = 0; i <= j; ++i)
                for (int32_t q = 0; q < R; ++q)
                    Hh[((size_t)i * m + j) * R + q] =
                        hc[(size_t)i * R + q] + hc[HOFF + (size_t)i * R + q];
            std::vector<double> hn((size_t)R);
            for (int32_t q = 0; q < R; ++q) hn[q] = std::sqrt(hc[2 * HOFF + q]);
            ++it;
            bool still = false;
            for (int32_t q = 0; q < R; ++q) {
                sc[q] = 0.0;
                if (!act[q]) continue;
                auto H = [&](size_t i, size_t jj) -> double & { return Hh[(i * m + jj) * R + q]; };
                H(j + 1, j) = hn[q];
                for (int i = 0; i < j; ++i) {
                    const double c = cs[(size_t)i * R + q], sg = sn[(size_t)i * R + q];
                    const double t = c * H(i, j) + sg * H(i + 1, j);
                    H(i + 1, j) = -sg * H(i, j) + c * H(i + 1, j);
                    H(i, j) = t;
                }
                const double d = std::hypot(H(j, j), H(j + 1, j));
                double c = 1.0, sg = 0.0;
                if (d > 0) { c = H(j, j) / d; sg = H(j + 1, j) / d; }
                cs[(size_t)j * R + q] = c;
                sn[(size_t)j * R + q] = sg;
                H(j, j) = d;
                H(j + 1, j) = 0.0;
                g[(size_t)(j + 1) * R + q] = -sg * g[(size_t)j * R + q];
                g[(size_t)j * R + q] = c * g[(size_t)j * R + q];
                kq[q] = j + 1;
                its[q] += 1;
                if (std::fabs(g[(size_t)(j + 1) * R + q]) <= tol[q]) {
                    act[q] = 0;          // frozen: its next basis vectors are zero
                } else {
                    still = true;
                    sc[q] = hn[q] > 0 ? 1.0 / hn[q] : 0.0;
                }
            }
            if (!still || it >= maxit || j + 1 == m) break;
            upload(scale.get(), sc);
            op_scale_rhs(n, R, w.get(), scale.get(), Vk(j + 1), s);
        }
        // x += Z y, y from the triangular systems (each right-hand side its
        // own number of steps; missing steps weigh zero)
        int kmax = 0;
        std::fill(cf.begin(), cf.end(), 0.0);
        for (int32_t q = 0; q < R; ++q) {
            const int k = kq[q];
            kmax = std::max(kmax, k);
            std::vector<double> y((size_t)k);
            for (int i = k - 1; i >= 0; --i) {
                double t = g[(size_t)i * R + q];
                for (int l = i + 1; l < k; ++l) t -= Hh[((size_t)i * m + l) * R + q] * y[l];
                y[i] = t / Hh[((size_t)i * m + i) * R + q];
            }
            for (int i = 0; i < k; ++i) cf[(size_t)i * R + q] = -y[i];
        }
        if (kmax > 0) {
            upload(coef.get(), cf);
            op_maxpy(n, R, Zp, nv, kmax, coef.get(), x, s);
        }
        true_residual(beta);
    }
    LAIR_HIP(hipStreamSynchronize(s));
    double relmax = 0.0;
    int32_t itmax = 0;
    for (int32_t q = 0; q < R; ++q) {
        relmax = std::max(relmax, nb[q] > 0 ? beta[q] / nb[q] : beta[q]);
        itmax = std::max(itmax, its[q]);
    }
    if (info) {
        info->iters = itmax;
        info->relres = relmax;
        double rho = 0.0;
        if (itmax > 0)
            for (int32_t q = 0; q < R; ++q)
                if (r_first[q] > 0 && its[q] > 0)
                    rho = std::max(rho, std::pow(beta[q] / r_first[q], 1.0 / its[q]));
        info->rho = rho;
        info_common(h, info);
        info->solve_ms = ms_since(t0);
    }
    return relmax <= rtol ? LAIR_OK : LAIR_ENOCONV;
}

// Batch of independent systems (one right-hand side each): the correction
// form x += B (b - A x) on the union, with the residual rows of converged
// systems zeroed so that their corrections vanish.  Each system stops at its
// own relative residual.
lair_status solve_batch_impl(lair_hierarchy *h, const double *b, double *x,
                             double rtol, int32_t maxit, int32_t *iters,
                             double *relres, lair_info *info, hipStream_t s) {
    auto t0 = Clock::now();
    check_solve_args(h, b, x, rtol, maxit);
    if (!h->batch) fail(LAIR_EINVAL, "the hierarchy was not built by lair_setup_batch");
    ensure_vectors(h, 1, s);
    Level &L0 = *h->L[0];
    const int32_t ns = h->nsys;
    const int64_t n = L0.n;
    bool mixed = h->opt.precision == LAIR_MIXED;
    // grow-only: captured iterations keep these addresses
    bool moved = false;
    if (h->seg_norm.get() == nullptr) { h->seg_norm.alloc((size_t)ns, s); moved = true; }
    if (h->active_dev.get() == nullptr) { h->active_dev.alloc((size_t)ns, s); moved = true; }
    if (!mixed && h->e64.get() == nullptr) { h->e64.alloc((size_t)n, s); moved = true; }
    // one system: the iteration stops when it converges, no lists needed
    const bool lists = ns > 1;
    const size_t cnt_bytes = (3 * sizeof(int32_t) * h->L.size() + 15) & ~(size_t)15;
    if (lists && L0.act_cnt == nullptr) {
        const size_t maxseg = 3 * h->L.size() * (size_t)ns;
        h->act_upload.alloc(cnt_bytes + sizeof(int64_t) * (maxseg + 1) +
                                3 * sizeof(int32_t) * maxseg + 64, s);
        for (size_t l = 0; l < h->L.size(); ++l) {
            Level &Lv = *h->L[l];
            Lv.act_cnt = reinterpret_cast<int32_t *>(h->act_upload.get()) + 3 * l;
            Lv.act_rows.alloc((size_t)std::max(Lv.n, 1), s);
            if (l + 1 < h->L.size()) {
                Lv.act_f.alloc((size_t)std::max(Lv.nf, 1), s);
                Lv.act_c.alloc((size_t)std::max(Lv.nrc >= 0 ? Lv.nrc : Lv.nc, 1), s);
            }
        }
        moved = true;
    }
    if (h->ss_nblk == 0) {
        // per-system norms: blocks of at most seg_sum_chunk() rows
        const int64_t ch = seg_sum_chunk();
        std::vector<int32_t> bsys;
        std::vector<int64_t> blo, bstart{0};
        for (int32_t q = 0; q < ns; ++q) {
            for (int64_t lo = L0.seg[q]; lo < L0.seg[q + 1]; lo += ch) {
                bsys.push_back(q);
                blo.push_back(lo);
            }
            bstart.push_back((int64_t)bsys.size());
        }
        h->ss_nblk = (int32_t)bsys.size();
        h->ss_sys.alloc(bsys.size(), s);
        h->ss_lo.alloc(blo.size(), s);
        h->ss_start.alloc(bstart.size(), s);
        h->ss_part.alloc(bsys.size(), s);
        LAIR_HIP(hipMemcpyAsync(h->ss_sys.get(), bsys.data(), sizeof(int32_t) * bsys.size(),
                                hipMemcpyHostToDevice, s));
        LAIR_HIP(hipMemcpyAsync(h->ss_lo.get(), blo.data(), sizeof(int64_t) * blo.size(),
                                hipMemcpyHostToDevice, s));
        LAIR_HIP(hipMemcpyAsync(h->ss_start.get(), bstart.data(),
                                sizeof(int64_t) * bstart.size(), hipMemcpyHostToDevice, s));
        LAIR_HIP(hipStreamSynchronize(s));     // pageable sources
        moved = true;
    }
    if (moved) h->drop_graphs();
    auto seg_norms = [&](const double *r, const uint8_t *act, hipStream_t st) {
        ProfScope ps("norm", st, 8.0 * n, 2.0 * n);
        launch_seg_sumsq_blocks(ns, h->ss_nblk, h->ss_sys.get(), h->ss_lo.get(),
                                h->ss_start.get(), L0.seg_dev.get(), act, r,
                                h->ss_part.get(), h->seg_norm.get(), st);
    };
    // rows of the systems still iterated, on every level.  A system's rows,
    // F rows and relaxed C rows are contiguous runs of the level's row range,
    // F list and relaxed-C list; the host lays out the runs of the active
    // systems and one kernel copies them (no atomics, fixed order).
    const size_t nlev = h->L.size();
    std::vector<std::array<std::vector<int32_t>, 3>> runs(nlev);   // per list: prefix over systems
    for (size_t l = 0; lists && l < nlev; ++l) {
        Level &Lv = *h->L[l];
        for (int t = 0; t < 3; ++t) runs[l][t].assign((size_t)ns + 1, 0);
        const bool last = l + 1 == nlev;
        for (int32_t q = 0; q < ns; ++q) {
            const int32_t nq = (int32_t)(Lv.seg[q + 1] - Lv.seg[q]);
            int32_t cq = 0, rq = 0;
            if (!last) {
                cq = (int32_t)(Lv.next_seg[q + 1] - Lv.next_seg[q]);
                rq = Lv.stopped[q] ? 0 : cq;     // stopped systems' C rows are not relaxed
            }
            runs[l][0][q + 1] = runs[l][0][q] + nq;
            runs[l][1][q + 1] = runs[l][1][q] + (last ? 0 : nq - cq);
            runs[l][2][q + 1] = runs[l][2][q] + rq;
        }
    }
    DevArr<const int32_t *> d_src;
    DevArr<int32_t *> d_dst;
    if (lists) {
        std::vector<const int32_t *> srcs(3 * nlev, nullptr);
        std::vector<int32_t *> dsts(3 * nlev, nullptr);
        for (size_t l = 0; l < nlev; ++l) {
            Level &Lv = *h->L[l];
            dsts[3 * l] = Lv.act_rows.get();
            if (l + 1 < nlev) {
                srcs[3 * l + 1] = Lv.flist.get();
                dsts[3 * l + 1] = Lv.act_f.get();
                srcs[3 * l + 2] = Lv.nrc >= 0 ? Lv.rclist.get() : Lv.clist.get();
                dsts[3 * l + 2] = Lv.act_c.get();
            }
        }
        d_src.alloc(3 * nlev, s);
        d_dst.alloc(3 * nlev, s);
        LAIR_HIP(hipMemcpyAsync(d_src.get(), srcs.data(), sizeof(void *) * 3 * nlev,
                                hipMemcpyHostToDevice, s));
        LAIR_HIP(hipMemcpyAsync(d_dst.get(), dsts.data(), sizeof(void *) * 3 * nlev,
                                hipMemcpyHostToDevice, s));
        LAIR_HIP(hipStreamSynchronize(s));     // the pointer tables are pageable host memory
    }
    auto rebuild_lists = [&]() {
        std::vector<int64_t> out{0};
        std::vector<int32_t> src, dst, lst;
        std::vector<int32_t> counts(3 * nlev, 0);
        for (size_t l = 0; l < nlev; ++l)
            for (int t = 0; t < 3; ++t) {
                if (t > 0 && l + 1 == nlev) continue;
                int32_t pos = 0;
                for (int32_t q = 0; q < ns; ++q) {
                    if (!h->active[q]) continue;
                    const int32_t len = runs[l][t][q + 1] - runs[l][t][q];
                    if (len == 0) continue;
                    const int32_t start = t == 0 ? (int32_t)h->L[l]->seg[q] : runs[l][t][q];
                    out.push_back(out.back() + len);
                    src.push_back(start);
                    dst.push_back(pos);
                    lst.push_back((int32_t)(3 * l + t));
                    pos += len;
                }
                counts[3 * l + t] = pos;
            }
        const int32_t nseg = (int32_t)lst.size();
        // one pinned upload area with the device layout: the list lengths
        // (fixed addresses), then the segment offsets, sources, targets and
        // list numbers; one copy in stream order.  It is rewritten only at
        // the next rebuild, after the readback that follows this iteration.
        const size_t b_out = sizeof(int64_t) * out.size(), b_i = sizeof(int32_t) * nseg;
        const size_t total = cnt_bytes + b_out + 3 * b_i;
        char *st = (char *)pinned_upload(total + 64);
        memset(st, 0, cnt_bytes);
        memcpy(st, counts.data(), sizeof(int32_t) * counts.size());
        memcpy(st + cnt_bytes, out.data(), b_out);
        memcpy(st + cnt_bytes + b_out, src.data(), b_i);
        memcpy(st + cnt_bytes + b_out + b_i, dst.data(), b_i);
        memcpy(st + cnt_bytes + b_out + 2 * b_i, lst.data(), b_i);
        char *dev = h->act_upload.get();
        LAIR_HIP(hipMemcpyAsync(dev, st, total, hipMemcpyHostToDevice, s));
        const int64_t *d_out = reinterpret_cast<const int64_t *>(dev + cnt_bytes);
        const int32_t *d_meta = reinterpret_cast<const int32_t *>(dev + cnt_bytes + b_out);
        launch_materialize(nseg, out.back(), d_out, d_meta, d_meta + nseg, d_meta + 2 * nseg,
                           d_src.get(), d_dst.get(), s);
    };
    struct ActGuard {
        lair_hierarchy *h;
        ~ActGuard() { h->use_act = false; }
    } act_guard{h};
    const double *bb = b;
    if (scaled(h->opt)) {
        op_block_apply(n / h->opt.block_size, h->opt.block_size, h->dinv.get(), b,
                       h->bscaled.get(), 1, s);
        bb = h->bscaled.get();
    }
    std::vector<double> nb, rn, rfirst;
    seg_norms(bb, nullptr, s);
    read_norms(h->seg_norm.get(), ns, s, nb);
    CsrView<double> A0 = view<double>(L0.A, L0.team_A);
    auto residual_and_norms = [&](hipStream_t st) {
        {
            ProfScope ps("residual", st, ab_rowdot(L0.A, 8, 1, 2), 2.0 * L0.A.nnz);
            op_residual<double>(A0, bb, x, h->r0.get(), 1, st);
        }
        seg_norms(h->r0.get(), nullptr, st);
    };
    residual_and_norms(s);
    read_norms(h->seg_norm.get(), ns, s, rn);
    rfirst = rn;
    h->active.assign((size_t)ns, 1);
    std::vector<int32_t> its((size_t)ns, 0);
    std::vector<double> rel((size_t)ns, 0.0);
    bool upload = true;
    int32_t it = 0;
    std::vector<double> hist;
    for (;;) {
        int32_t nact = 0;
        for (int32_t q = 0; q < ns; ++q) {
            if (!h->active[q]) continue;
            rel[q] = nb[q] > 0 ? rn[q] / nb[q] : rn[q];
            its[q] = it;
            if (rel[q] <= rtol) {
                h->active[q] = 0;
                upload = true;
            } else {
                ++nact;
            }
        }
        hist.push_back(*std::max_element(rel.begin(), rel.end()));
        if (nact == 0 || it >= maxit) break;
        if (upload) {
            LAIR_HIP(hipMemcpyAsync(h->active_dev.get(), h->active.data(), (size_t)ns,
                                    hipMemcpyHostToDevice, s));
            if (lists) rebuild_lists();
            upload = false;
        }
        // the cycle touches only the rows of systems still iterated; the
        // others keep their x (their corrections would be zero)
        h->use_act = lists;
        run_iteration(h, mixed ? IT_BATCH_MIXED : IT_BATCH_FP64, 1, bb, x, s,
                      [&](hipStream_t st) {
            if (mixed) {
                {
                    ProfScope ps("cast", st, 12.0 * n);
                    op_cast_f32(h->r0.get(), h->r0_32.get(), n, st);
                }
                vcycle<float>(h, 0, h->r0_32.get(), h->e32.get(), true, nullptr, 1, st);
                ProfScope ps("cast", st, 20.0 * n);
                if (lists)
                    op_update_list<float>(L0.act_rows.get(), L0.act_cnt, (int32_t)n, x,
                                          h->e32.get(), st);
                else
                    op_axpy_f32(x, h->e32.get(), n, st);
            } else {
                vcycle<double>(h, 0, h->r0.get(), h->e64.get(), true, nullptr, 1, st);
                if (lists) {
                    op_update_list<double>(L0.act_rows.get(), L0.act_cnt, (int32_t)n, x,
                                           h->e64.get(), st);
                } else {
                    LAIR_LAUNCH(k_add, dim3(blocks_for(n, 256)), dim3(256), 0, st, x,
                                h->e64.get(), n);
                    LAIR_LAUNCH_CHECK();
                }
            }
            {
                ProfScope ps("residual", st, ab_rowdot(L0.A, 8, 1, 2), 2.0 * L0.A.nnz);
                if (lists)
                    op_rowdot_list<double>(A0, 0, L0.act_rows.get(), L0.act_cnt,
                                           (int32_t)n, x, bb, h->r0.get(), st);
                else
                    op_residual<double>(A0, bb, x, h->r0.get(), 1, st);
            }
            seg_norms(h->r0.get(), h->active_dev.get(), st);
        });
        h->use_act = false;
        read_norms(h->seg_norm.get(), ns, s, rn);
        ++it;
    }
    LAIR_HIP(hipStreamSynchronize(s));
    double relmax = 0.0;
    int32_t itmax = 0;
    bool conv = true;
    for (int32_t q = 0; q < ns; ++q) {
        if (iters) iters[q] = its[q];
        if (relres) relres[q] = rel[q];
        relmax = std::max(relmax, rel[q]);
        itmax = std::max(itmax, its[q]);
        conv = conv && rel[q] <= rtol;
    }
    if (info) {
        info->iters = itmax;
        info->relres = relmax;
        double rho = 0.0;
        for (int32_t q = 0; q < ns; ++q)
            if (its[q] > 0 && rfirst[q] > 0)
                rho = std::max(rho, std::pow(rel[q] * nb[q] / rfirst[q], 1.0 / its[q]));
        info->rho = rho;
        info_common(h, info);
        set_history(info, hist);
        info->solve_ms = ms_since(t0);
    }
    return conv ? LAIR_OK : LAIR_ENOCONV;
}

// ---------------------------------------------------------------------------
// One cycle from a given iterate (lair_cycle) and its transpose
// ---------------------------------------------------------------------------
void cycle_impl(lair_hierarchy *h, const double *b, double *x, int32_t nrhs, hipStream_t s) {
    if (!h || !b || !x) fail(LAIR_EINVAL, "NULL argument");
    check_nrhs(h, nrhs);
    ensure_vectors(h, nrhs, s);
    cycle_body(h, b, x, nrhs, s);
}

void cycle_body(lair_hierarchy *h, const double *b, double *x, int32_t nrhs, hipStream_t s) {
    const double *bb = b;
    int64_t n = h->L[0]->n;
    if (scaled(h->opt)) {
        op_block_apply(n / h->opt.block_size, h->opt.block_size, h->dinv.get(), b,
                       h->bscaled.get(), nrhs, s);
        bb = h->bscaled.get();
    }
    Level &L0 = *h->L[0];
    if (h->opt.precision == LAIR_MIXED) {
        op_residual<double>(view<double>(L0.A, L0.team_A), bb, x, h->r0.get(), nrhs, s);
        if (L0.split) op_cast_f32_rows(h->r0.get(), h->r0_32.get(), L0.iperm.get(), n,
                                       nrhs, s);
        else op_cast_f32(h->r0.get(), h->r0_32.get(), n * nrhs, s);
        vcycle<float>(h, 0, h->r0_32.get(), h->e32.get(), true, nullptr, nrhs, s);
        if (L0.split) op_axpy_f32_rows(x, h->e32.get(), L0.iperm.get(), n, nrhs, s);
        else op_axpy_f32(x, h->e32.get(), n * nrhs, s);
    } else if (L0.split) {
        op_permute_rows(n, nrhs, L0.perm.get(), bb, h->bsplit.get(), true, s);
        op_permute_rows(n, nrhs, L0.perm.get(), x, h->xsplit.get(), true, s);
        vcycle<double>(h, 0, h->bsplit.get(), h->xsplit.get(), false, nullptr, nrhs, s);
        op_permute_rows(n, nrhs, L0.perm.get(), h->xsplit.get(), x, false, s);
    } else {
        vcycle<double>(h, 0, bb, x, false, nullptr, nrhs, s);
    }
}

void cycle_transpose_impl(lair_hierarchy *h, const double *g, double *lam, int32_t nrhs,
                          hipStream_t s) {
    if (!h || !g || !lam) fail(LAIR_EINVAL, "NULL argument");
    check_nrhs(h, nrhs);
    if (nodal(h->opt)) fail(LAIR_EUNSUPPORTED, "transposed cycle on a nodal hierarchy");
    ensure_vectors(h, nrhs, s);
    ensure_transposes(h);
    // lam <- lam + B^T (g - A^T lam)
    Level &L0 = *h->L[0];
    int64_t n = L0.n;
    op_residual<double>(view<double>(L0.At, L0.team_At), g, lam, h->r0.get(), nrhs, s);
    vcycle_t(h, 0, h->r0.get(), L0.b.get(), true, nrhs, s);
    LAIR_LAUNCH(k_add, dim3(blocks_for(n * nrhs, 256)), dim3(256), 0, s,
                       lam, L0.b.get(), n * nrhs);
    LAIR_LAUNCH_CHECK();
}

}  // namespace lair
