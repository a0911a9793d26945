// hierarchy.hpp -- the host-side hierarchy of liblair (levels, their
// matrices, transfer operators and work vectors) and the functions shared by
// the setup (setup.cpp), the cycles and solves (solve.cpp) and the C ABI
// (lair_api.cpp).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdint>
#include <memory>
#include <type_traits>
#include <vector>

#include "lair_internal.hpp"

namespace lair {

// ---------------------------------------------------------------------------
// Hierarchy storage
// ---------------------------------------------------------------------------
struct Level {
    DevCSR A, R, P;            // A_l (n x n), R_l (nc x n), P_l (n x nc)
    DevCSR At, Rt, Pt;         // transposes for the adjoint cycle
    int32_t n = 0, nc = 0, nf = 0;
    int64_t nnzF = 0, nnzC = 0;     // stored entries in the F rows / C rows
    DevArr<unsigned long long> fc_acc;   // their device sums until read at the end of setup
    int32_t max_row = 0;
    int32_t team_A = 8, team_R = 8, team_P = 2;
    int32_t team_At = 8, team_Rt = 2, team_Pt = 8;
    DevArr<int8_t> cf;
    DevArr<uint8_t> smask;
    DevArr<int32_t> cidx, clist, flist, nptr, nbr;
    DevArr<int32_t> cjt;           // A's columns tagged with the C/F type
    DevArr<int8_t> flags;
    lair_level_stats st{};
    // batch of systems: row offsets of every system at this level, the
    // systems that no longer coarsen (pass-through rows), and the C rows
    // that are relaxed (C-points of systems still coarsening)
    std::vector<int64_t> seg, next_seg;
    DevArr<int64_t> seg_dev;
    std::vector<uint8_t> stopped;
    DevArr<uint8_t> stopped_dev;
    DevArr<int32_t> rclist;
    int32_t nrc = -1;                 // -1: relax every C row (clist)
    // rows of the systems still iterated (batch solve): all rows, F rows,
    // relaxed C rows; their lengths in act_cnt[0..2] on the device (inside
    // the hierarchy's list upload area)
    DevArr<int32_t> act_rows, act_f, act_c;
    int32_t *act_cnt = nullptr;
    // cycle work vectors (capacity h->nrhs_cap right-hand sides)
    DevArr<double> b, x, t, r;
    DevArr<float> b32, x32, t32, r32;
    // split ordering of a single system's level for the cycle: F-points
    // first, then C-points.  perm[new] = old, iperm[old] = new, ids[k] = k
    // (F rows ids[0..nf), C rows ids[nf..n)), cf_split[k] = (k >= nf); As,
    // Rs, Ps are A, R, P in the split orderings of their row and column
    // levels, cjt_split As's columns tagged where they are C-points
    DevArr<int32_t> perm, iperm, ids, cjt_split;
    DevArr<int8_t> cf_split;
    DevCSR As, Rs, Ps;
    bool split = false;
    // size-bucket edges (and the fused flag) the local solves used here
    int32_t buckets[5] = {0, 0, 0, 0, 0};
    // nodal hierarchy (k x k blocks): inverses of the diagonal blocks, the
    // values of D^{-1} A on A's pattern (double and float) that the block
    // Jacobi sweeps read, and the sweeps' right-hand side D^{-1} b
    DevArr<double> ndinv, av, bt;
    DevArr<float> av32, bt32;
};

}  // namespace lair

struct lair_hierarchy {
    std::vector<std::unique_ptr<lair::Level>> L;
    lair_strength str{};
    lair_options opt{};
    hipStream_t stream = nullptr;
    int32_t nL = 0;                          // coarsest size
    double coarse_entries = 0.0;             // entries of the coarsest dense factors:
                                             // nL^2, or the sum of the systems' n_q^2
    lair::DevArr<double> lu;
    lair::DevArr<int32_t> piv;
    lair::DevArr<double> kinv;               // explicit inverse when nL <= 512
    lair::DevArr<int8_t> cf_dev;             // caller's CF splittings (all levels)
    std::vector<int64_t> cf_count;           // their numbers of C-points
    lair::DevArr<double> dinv;               // block scaling (block_size > 0)
    int32_t nrhs_cap = 0;
    lair::DevArr<double> bscaled, r0, partial, norms;
    lair::DevArr<float> r0_32, e32;
    bool have_transpose = false;
    // batch of independent systems (nsys > 1): per-system coarsest blocks
    int32_t nsys = 1;
    lair::DevArr<int64_t> dense_off;
    lair::DevArr<double> binv;               // per-system coarsest inverses (small blocks)
    lair::DevArr<uint8_t> use_inv;           // 1: the system's block is applied by its inverse
    // per-system norms over several blocks per system (level-0 rows)
    lair::DevArr<int32_t> ss_sys;
    lair::DevArr<int64_t> ss_lo, ss_start;
    lair::DevArr<double> ss_part;
    int32_t ss_nblk = 0;
    std::vector<int32_t> sys_levels;
    lair::DevArr<uint8_t> active_dev;
    // batch solve: the active-row list lengths of every level (3 per level,
    // at fixed addresses read by captured iterations) followed by the
    // segment tables of the last list rebuild, uploaded in one copy
    lair::DevArr<char> act_upload;
    lair::DevArr<double> seg_norm;
    lair::DevArr<double> e64;
    // single system: the cycle runs on split-ordered copies (Level::As ...)
    // of the levels marked split; an FP64 solve carries b and x in level 0's
    // split ordering
    lair::DevArr<double> bsplit, xsplit;
    // captured correction cycles, keyed by (precision, nrhs); replayed on a
    // private stream ordered against the caller's stream with events
    bool batch = false;                      // built by lair_setup_batch
    bool use_act = false;                    // cycles restricted to the active rows
    std::vector<uint8_t> active;             // systems still iterated
    // captured solve iterations (cycle + residual + norms), keyed by the
    // iteration kind, the number of right-hand sides and the caller's b and
    // x; captured on a private stream, replayed on the caller's stream
    struct Graph { int kind; int32_t nrhs; const void *b; void *x; hipGraphExec_t exec; };
    std::vector<Graph> graphs;
    hipStream_t gstream = nullptr;
    void drop_graphs() {
        for (auto &g : graphs) (void)hipGraphExecDestroy(g.exec);
        graphs.clear();
    }
    ~lair_hierarchy() {
        drop_graphs();
        if (gstream) (void)hipStreamDestroy(gstream);
    }
    int64_t n_singular = 0;
    double setup_ms = 0.0;
    double split_ms = 0.0;                   // host first-pass splittings in setup
    double phase_ms[8] = {0, 0, 0, 0, 0, 0, 0, 0};   // setup wall time by phase
    std::chrono::steady_clock::time_point phase_t0;
    // charge the wall time since the last mark to phase k
    void phase_mark(int k) {
        const auto t = std::chrono::steady_clock::now();
        phase_ms[k] += std::chrono::duration<double, std::milli>(t - phase_t0).count();
        phase_t0 = t;
    }
    double cc = 0.0, oc = 0.0;
};

namespace lair {

using Clock = std::chrono::steady_clock;

inline double ms_since(Clock::time_point t0) {
    return std::chrono::duration<double, std::milli>(Clock::now() - t0).count();
}

// block_size k with the nodal flag builds the hierarchy by blocks; without
// it the system is scaled by its block diagonal first
inline bool nodal(const lair_options &o) {
    return o.block_size > 0 && (o.flags & LAIR_FLAG_NODAL) != 0;
}
inline bool scaled(const lair_options &o) { return o.block_size > 0 && !nodal(o); }

inline int32_t team_of(const DevCSR &M) {
    double mean = M.nrows ? (double)M.nnz / (double)M.nrows : 1.0;
    int t = 1;
    while (t < 64 && t < mean) t <<= 1;
    return t;
}

template <class VT>
inline CsrView<VT> view(const DevCSR &M, int32_t team) {
    CsrView<VT> v;
    v.nrows = M.nrows;
    v.ncols = M.ncols;
    v.rp = M.rp.get();
    v.cj = M.cj.get();
    if constexpr (std::is_same<VT, double>::value) v.v = M.v.get();
    else v.v = M.v32.get();
    v.team = team;
    return v;
}

constexpr int32_t NPARTIAL = 4096;   // blocks of the fused residual (and partial sums)

template <class VT>
inline VT *vec(DevArr<double> &d, DevArr<float> &f) {
    if constexpr (std::is_same<VT, double>::value) { (void)f; return d.get(); }
    else { (void)d; return f.get(); }
}

// ---------------------------------------------------------------------------
// Shared between the translation units
// ---------------------------------------------------------------------------
void rs_first_pass(int64_t n, const int32_t *rp, const int32_t *cj,
                   const uint8_t *sm, int8_t *cf);
void check_options(const lair_strength *s, const lair_options *o);
// T = M^T (CSR), with the team sizes of its rows
void transpose(const DevCSR &M, DevCSR &T, hipStream_t s, DevArr<int64_t> &tmp);
lair_hierarchy *setup_impl(const lair_csr *Ain, const lair_cf_levels *cfl,
                           const lair_strength *str, const lair_options *opt,
                           hipStream_t s, const std::vector<int64_t> *seg = nullptr);
lair_hierarchy *setup_batch_impl(int32_t nsys, const lair_csr *sys, const lair_cf_levels *cfl,
                                 const lair_strength *str, const lair_options *opt,
                                 hipStream_t s);
void update_diag_impl(lair_hierarchy *h, const double *diag, int32_t on_device,
                      hipStream_t s);

void check_nrhs(const lair_hierarchy *h, int32_t nrhs);
lair_status solve_impl(lair_hierarchy *h, const double *b, double *x, int32_t nrhs,
                       double rtol, int32_t maxit, lair_info *info, hipStream_t s,
                       bool transpose);
lair_status solve_fgmres_impl(lair_hierarchy *h, const double *b, double *x, int32_t nrhs,
                              double rtol, int32_t maxit, int32_t restart, lair_info *info,
                              hipStream_t s);
lair_status solve_batch_impl(lair_hierarchy *h, const double *b, double *x, double rtol,
                             int32_t maxit, int32_t *iters, double *relres, lair_info *info,
                             hipStream_t s);
// The fields of lair_info every solve fills the same way: level count,
// complexities, setup figures, and the work units per digit from rho.
void info_common(const lair_hierarchy *h, lair_info *info);
// x <- x + B (b - A x), the work vectors taken from the hierarchy
void cycle_impl(lair_hierarchy *h, const double *b, double *x, int32_t nrhs, hipStream_t s);
// the same with the arguments checked and the work vectors in place (the
// arrays ensure_vectors sizes, for nrhs right-hand sides)
void cycle_body(lair_hierarchy *h, const double *b, double *x, int32_t nrhs, hipStream_t s);
// Visit every work vector of a cycle with nrhs right-hand sides as
// f(array, count), array a DevArr<double> or DevArr<float> of the hierarchy:
// the level vectors b, x, r, t (and their float copies in mixed precision),
// a nodal hierarchy's sweep right-hand sides, and the level-0 vectors of
// block scaling, mixed precision and the split ordering.  ensure_vectors
// allocates exactly these (plus the norms' partial sums).
template <class F>
void for_each_cycle_vector(lair_hierarchy *h, int32_t nrhs, F &&f) {
    const bool mixed = h->opt.precision == LAIR_MIXED;
    for (size_t l = 0; l < h->L.size(); ++l) {
        Level &Lv = *h->L[l];
        const size_t n = (size_t)Lv.n * nrhs;
        const size_t tn = (size_t)std::max(Lv.n, 1) * nrhs;
        f(Lv.b, n);
        f(Lv.x, n);
        f(Lv.r, n);
        f(Lv.t, tn);
        if (mixed) {
            f(Lv.b32, n);
            f(Lv.x32, n);
            f(Lv.r32, n);
            f(Lv.t32, tn);
        }
    }
    const size_t n0 = (size_t)h->L[0]->n * nrhs;
    f(h->r0, n0);
    if (scaled(h->opt)) f(h->bscaled, n0);
    if (nodal(h->opt))
        for (size_t l = 0; l + 1 < h->L.size(); ++l) {
            Level &Lv = *h->L[l];
            const size_t n = (size_t)std::max(Lv.n, 1) * nrhs;
            f(Lv.bt, n);
            if (mixed) f(Lv.bt32, n);
        }
    if (mixed) {
        f(h->r0_32, n0);
        f(h->e32, n0);
    }
    if (h->L[0]->split && !mixed) {
        f(h->bsplit, n0);
        f(h->xsplit, n0);
    }
}
// lair_cycle_noalloc: cycle_body with the work vectors in the fixed device
// array of noalloc.cpp
void cycle_noalloc_impl(lair_hierarchy *h, const double *b, double *x, int32_t nrhs,
                        hipStream_t s);
// lam <- lam + B^T (g - A^T lam)
void cycle_transpose_impl(lair_hierarchy *h, const double *g, double *lam, int32_t nrhs,
                          hipStream_t s);

}  // namespace lair
