// liblair host side: argument checking, the level loop of the setup, the
// V-cycle schedule and the outer iteration.  Every arithmetic step runs in
// the HIP kernels of k_setup.hip and k_cycle.hip; the host only sizes
// buffers, launches, and (for the classical CF splitting, a sequential
// greedy algorithm) runs rs_first_pass on a host copy of the strength mask.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <chrono>
#include <climits>
#include <cmath>
#include <cstdarg>
#include <cstring>
#include <memory>
#include <new>
#include <string>
#include <type_traits>
#include <vector>

#include "lair_internal.hpp"

namespace lair {

void rs_first_pass(int64_t n, const int32_t *rp, const int32_t *cj,
                   const uint8_t *sm, int8_t *cf);

static thread_local std::string g_last_error;

void set_last_error(const std::string &m) { g_last_error = m; }

void fail(lair_status st, const char *fmt, ...) {
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    throw Error{st, std::string(buf)};
}

// ---------------------------------------------------------------------------
// Hierarchy storage
// ---------------------------------------------------------------------------
struct Level {
    DevCSR A, R, P;            // A_l (n x n), R_l (nc x n), P_l (n x nc)
    DevCSR At, Rt, Pt;         // transposes for the adjoint cycle
    int32_t n = 0, nc = 0, nf = 0;
    int64_t nnzF = 0, nnzC = 0;     // stored entries in the F rows / C rows
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
    lair::DevArr<double> lu;
    lair::DevArr<int32_t> piv;
    lair::DevArr<double> kinv;               // explicit inverse when nL <= 512
    lair::DevArr<int8_t> cf_dev;             // caller's CF splittings (all levels)
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
    double cc = 0.0, oc = 0.0;
};

namespace lair {

using Clock = std::chrono::steady_clock;

static double ms_since(Clock::time_point t0) {
    return std::chrono::duration<double, std::milli>(Clock::now() - t0).count();
}

// block_size k with the nodal flag builds the hierarchy by blocks; without
// it the system is scaled by its block diagonal first
static bool nodal(const lair_options &o) {
    return o.block_size > 0 && (o.flags & LAIR_FLAG_NODAL) != 0;
}
static bool scaled(const lair_options &o) { return o.block_size > 0 && !nodal(o); }

static int32_t team_of(const DevCSR &M) {
    double mean = M.nrows ? (double)M.nnz / (double)M.nrows : 1.0;
    int t = 1;
    while (t < 64 && t < mean) t <<= 1;
    return t;
}

template <class VT>
static CsrView<VT> view(const DevCSR &M, int32_t team) {
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

static const int32_t NPARTIAL = 4096;   // blocks of the fused residual (and partial sums)

__global__ void k_nonneg_flag(int32_t n, const int32_t *pc, int32_t *hs) {
    int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) hs[i] = pc[i] >= 0 ? 1 : 0;
}

__global__ void k_add(double *x, const double *e, int64_t m) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m) x[i] += e[i];
}

__global__ void k_r_rowptr(int32_t nc, const int32_t *nptr, int32_t *rrp) {
    int32_t c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c <= nc) rrp[c] = nptr[c] + c;
}

__global__ void k_block_diag_csr(int32_t nblk, int32_t k, const double *dinv,
                                 int32_t *rp, int32_t *cj, double *v) {
    int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t n = (int64_t)nblk * k;
    if (g <= n) rp[g] = (int32_t)(g * k);
    if (g >= n * k) return;
    int64_t row = g / k;
    int c = (int)(g % k);
    cj[g] = (int32_t)((row / k) * k + c);
    v[g] = dinv[(row / k) * k * k + (row % k) * k + c];
}

// The diagonal blocks of D_B^{-1} A are the identity by definition: store
// exact ones and zeros there instead of the rounded products, whose noise
// would otherwise decide the strength of connection in rows that have no
// other coupling.  A team of 8 lanes per row.
__global__ void k_unit_diag_blocks(int32_t n, int32_t k, const int32_t *rp, const int32_t *cj,
                                   double *v) {
    int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int32_t r = (int32_t)(g / 8);
    if (r >= n) return;
    const int32_t blk = r / k;
    for (int32_t p = rp[r] + (int32_t)(g % 8); p < rp[r + 1]; p += 8) {
        const int32_t c = cj[p];
        if (c / k == blk) v[p] = (c == r) ? 1.0 : 0.0;
    }
}

// Sizes of a CSR matrix produced on the device (nnz, longest row, an
// overflow flag) whose host copies wait for a later readback, so that the
// setup does not stop for each of them.
struct PendingSizes {
    DevArr<int64_t> d;               // [0] nnz, [1] longest row, [2] flag (low word)
    int64_t *dp = nullptr;           // d, or three zeroed slots of the caller
    int64_t h[3] = {0, 0, 0};
    DevCSR *m = nullptr;
    const char *what = "";
    void arm(DevCSR *mat, const char *w, hipStream_t s) {
        d.alloc(3, s);
        LAIR_HIP(hipMemsetAsync(d.get(), 0, 3 * sizeof(int64_t), s));
        arm_at(d.get(), mat, w);
    }
    // slots already zeroed in stream order (no memset here)
    void arm_at(int64_t *slots, DevCSR *mat, const char *w) {
        dp = slots;
        m = mat;
        what = w;
    }
    int64_t *tot() { return dp; }
    int32_t *flag() { return reinterpret_cast<int32_t *>(dp + 2); }
    void add(Readback &rb) {
        if (m) rb.add(h, dp, sizeof(h));
    }
    // after the readback that carried them
    void apply() {
        if (!m) return;
        DevCSR *mat = m;
        m = nullptr;
        if ((int32_t)h[2]) fail(LAIR_EUNSUPPORTED, "%s", what);
        mat->nnz = h[0];
        mat->max_row = (int32_t)h[1];
    }
    void settle(hipStream_t s) {
        if (!m) return;
        Readback rb(s);
        add(rb);
        rb.run();
        apply();
    }
};

// The profiler attributes algorithmic bytes from host-side sizes as it
// launches; while it times the setup categories every size is read at once.
static bool setup_sizes_eager() {
    return prof_selected("spgemm_fill") || prof_selected("spgemm_compact") ||
           prof_selected("spgemm_count") || prof_selected("interp");
}

// C = A B with the symbolic pattern, in two parts: spgemm_count launches
// the products-per-row count and its scan, leaving the total and the
// longest count on the device (st.tot) for the caller's next readback;
// spgemm_finish then stages, accumulates and compacts the rows.  With
// `defer` the sizes of C stay on the device too (C's arrays are sized by
// the number of products, an upper bound) and reach the host with a later
// readback; otherwise they are read at once.
struct SpgemmState {
    int32_t m = 0;
    DevArr<int32_t> cnt;
    DevArr<int64_t> eoff, tot;       // tot: [0] products, [1] most in a row
    // work: [0..5] three int64 slots (C's sizes, or [2] the overflow flag),
    // then the product's retry counters and lists; the head is zeroed once
    DevArr<int32_t> work;
    static constexpr int HEAD = 6;
    int64_t *ctl() { return reinterpret_cast<int64_t *>(work.get()); }
    int32_t *lists() { return work.get() + HEAD; }
    int64_t h[2] = {0, 0};
};

// The counters the product needs zeroed are cleared here, while earlier
// work still runs, rather than after the readback that spgemm_finish waits
// for.
static void spgemm_count(const DevCSR &A, const DevCSR &B, SpgemmState &st, hipStream_t s,
                         DevArr<int64_t> &tmp) {
    const int32_t m = A.nrows;
    st.m = m;
    st.cnt.alloc((size_t)m + 1, s);
    st.eoff.alloc((size_t)m + 1, s);
    st.work.alloc(SpgemmState::HEAD + 4 + 3 * (size_t)m, s);
    st.tot.alloc(2, s);
    LAIR_HIP(hipMemsetAsync(st.work.get(), 0, (SpgemmState::HEAD + 4) * sizeof(int32_t), s));
    // products per row: A's indices and B's row pointers
    ProfScope ps("spgemm_count", s, 4.0 * A.nnz + 4.0 * (A.nrows + 1) +
                                        8.0 * (B.nrows + 1) + 12.0 * m);
    launch_prod_count(m, A.rp.get(), A.cj.get(), B.rp.get(), st.cnt.get(), s);
    scan_counts_i64_to(st.cnt.get(), st.eoff.get(), m, s, tmp, st.tot.get());
}

// st.h must hold the readback of st.tot.  Returns C's longest row (0 when
// deferred).
// ratio: products per distinct column expected for C's rows (from a
// similar product; 0 when unknown), which sizes the hash tables.
// lump_tol > 0 (not deferred): C is written lumped (Sec. 3.3) straight from
// the staged rows, in place of the plain compaction.
// *distinct receives the size C has before lumping.
static int32_t spgemm_finish(const DevCSR &A, const DevCSR &B, DevCSR &C, SpgemmState &st,
                             hipStream_t s, DevArr<int64_t> &tmp, PendingSizes *defer,
                             double ratio = 0.0, double lump_tol = 0.0,
                             int64_t *distinct = nullptr, const int8_t *whole_rows = nullptr) {
    const int32_t m = st.m;
    const int64_t etot = st.h[0], emax = st.h[1];
    C.nrows = m;
    C.ncols = B.ncols;
    int32_t *ovp = reinterpret_cast<int32_t *>(st.ctl() + 2);
    if (defer) defer->arm_at(st.ctl(), &C, "sparse product row with more than 1024 terms");
    DevArr<int32_t> tcj;
    DevArr<double> tcx;
    tcj.alloc((size_t)std::max<int64_t>(etot, 1), s);
    tcx.alloc((size_t)std::max<int64_t>(etot, 1), s);
    {
        // A, the rows of B and the rows of C each touched once
        ProfScope ps("spgemm_fill", s, 12.0 * (A.nnz + B.nnz) + 4.0 * (A.nrows + 1) +
                                           4.0 * (B.nrows + 1));
        const double mean_e = m ? (double)etot / m : 0.0;
        launch_spgemm(m, A.rp.get(), A.cj.get(), A.v.get(), B.rp.get(), B.cj.get(),
                      B.v.get(), st.eoff.get(), emax, mean_e, ratio > 1.0 ? mean_e / ratio : 0.0,
                      st.cnt.get(), tcj.get(), tcx.get(), st.lists(), ovp, s);
    }
    C.rp.alloc((size_t)m + 1, s);
    int64_t mx = 0;
    if (lump_tol > 0.0 && !defer) {
        DevArr<int32_t> kcnt;
        kcnt.alloc((size_t)m + 1, s);
        // mean row of C before lumping, from the products per distinct
        // column of the level above when known
        const double mean_e = m ? (double)etot / m : 1.0;
        const double mean_c = ratio > 1.0 ? mean_e / ratio : mean_e / 2.0;
        // algorithmic bytes: the distinct entries of each staged row (column
        // and value), its offset and length, and the count written; the
        // number of distinct entries reaches the host with the readback below
        int count_slot = -1;
        {
            ProfScope ps("lump", s, 12.0 * etot + 16.0 * m);
            launch_lump(m, nullptr, st.eoff.get(), st.cnt.get(), tcj.get(), tcx.get(), lump_tol,
                        whole_rows, mean_c, kcnt.get(), nullptr, nullptr, nullptr, s);
            count_slot = ps.slot;
        }
        // kept entries (offsets of C) and, for the hash-table estimate of
        // the next level, the distinct columns before lumping: one readback
        DevArr<int32_t> dscan;
        dscan.alloc((size_t)m + 1, s);
        DevArr<int64_t> tots;
        tots.alloc(4, s);
        scan_counts_i32_to(kcnt.get(), C.rp.get(), m, s, tmp, tots.get());
        scan_counts_i32_to(st.cnt.get(), dscan.get(), m, s, tmp, tots.get() + 2);
        int64_t ht[4] = {0, 0, 0, 0};
        int32_t ov = 0;
        {
            Readback rb(s);
            rb.add(ht, tots.get(), sizeof(ht));
            rb.add(&ov, ovp, sizeof(ov));
            rb.run();
        }
        if (ov) fail(LAIR_EUNSUPPORTED, "sparse product row with more than 1024 terms");
        if (ht[0] > INT32_MAX)
            fail(LAIR_EUNSUPPORTED, "offset array exceeds 2^31 entries (%lld)", (long long)ht[0]);
        C.nnz = ht[0];
        mx = ht[1];
        if (distinct) *distinct = ht[2];
        prof_set_bytes(count_slot, 12.0 * ht[2] + 16.0 * m);
        C.max_row = (int32_t)mx;
        C.cj.alloc((size_t)std::max<int64_t>(C.nnz, 1), s);
        C.v.alloc((size_t)std::max<int64_t>(C.nnz, 1), s);
        {
            // the distinct entries read again, C's offsets read, C written
            ProfScope ps("lump", s, 12.0 * ht[2] + 20.0 * m + 12.0 * C.nnz);
            launch_lump(m, nullptr, st.eoff.get(), st.cnt.get(), tcj.get(), tcx.get(), lump_tol,
                        whole_rows, mean_c, nullptr, C.rp.get(), C.cj.get(), C.v.get(), s);
        }
        return (int32_t)mx;
    }
    if (defer) {
        scan_counts_i32_to(st.cnt.get(), C.rp.get(), m, s, tmp, defer->tot());
        C.nnz = etot;                // an upper bound until the sizes arrive
        C.max_row = -1;
    } else {
        int32_t ov = 0;
        C.nnz = scan_counts_i32(st.cnt.get(), C.rp.get(), m, s, tmp, &mx, ovp, &ov);
        if (ov) fail(LAIR_EUNSUPPORTED, "sparse product row with more than 1024 terms");
        C.max_row = (int32_t)mx;
    }
    C.cj.alloc((size_t)std::max<int64_t>(C.nnz, 1), s);
    C.v.alloc((size_t)std::max<int64_t>(C.nnz, 1), s);
    {
        ProfScope ps("spgemm_compact", s, 24.0 * C.nnz + 8.0 * (m + 1) + 4.0 * (m + 1));
        launch_spgemm_compact(m, st.eoff.get(), C.rp.get(), tcj.get(), tcx.get(), C.cj.get(),
                              C.v.get(), m ? (double)C.nnz / m : 1.0, s);
    }
    return (int32_t)mx;
}

// C = A B at once (count, readback, product, sizes).  Returns the longest
// row of C.
// c_nnz: C's size when known beforehand (0 if not), which sizes the hash
// tables.
static int32_t spgemm(const DevCSR &A, int32_t max_row_a, const DevCSR &B,
                      DevCSR &C, hipStream_t s, DevArr<int64_t> &tmp, int64_t c_nnz = 0) {
    (void)max_row_a;
    SpgemmState st;
    spgemm_count(A, B, st, s, tmp);
    {
        Readback rb(s);
        rb.add(st.h, st.tot.get(), sizeof(st.h));
        rb.run();
    }
    return spgemm_finish(A, B, C, st, s, tmp, nullptr,
                         c_nnz > 0 ? (double)st.h[0] / (double)c_nnz : 0.0);
}

static void transpose(const DevCSR &M, DevCSR &T, hipStream_t s,
                      DevArr<int64_t> &tmp) {
    T.nrows = M.ncols;
    T.ncols = M.nrows;
    T.nnz = M.nnz;
    DevArr<int32_t> cnt, cur;
    cnt.alloc((size_t)M.ncols + 1, s);
    cur.alloc((size_t)M.ncols + 1, s);
    T.rp.alloc((size_t)M.ncols + 1, s);
    T.cj.alloc((size_t)std::max<int64_t>(M.nnz, 1), s);
    T.v.alloc((size_t)std::max<int64_t>(M.nnz, 1), s);
    launch_transpose(M.nrows, M.ncols, M.nnz, M.rp.get(), M.cj.get(), M.v.get(),
                     cnt.get(), T.rp.get(), T.cj.get(), T.v.get(), cur.get(), s, tmp);
    if (M.v32.get()) {
        T.v32.alloc((size_t)std::max<int64_t>(M.nnz, 1), s);
        launch_to_float(T.v.get(), T.v32.get(), T.nnz, s);
    }
}

static void check_options(const lair_strength *s, const lair_options *o) {
    if (!s || !o) fail(LAIR_EINVAL, "strength and options must not be NULL");
    if (!(s->theta >= 0.0 && s->theta <= 1.0) || !(s->theta_c >= 0.0 && s->theta_c <= 1.0))
        fail(LAIR_EINVAL, "strength thresholds must lie in [0, 1]");
    if (s->kind != LAIR_SOC_ABS && s->kind != LAIR_SOC_NEG)
        fail(LAIR_EINVAL, "unknown strength kind %d", s->kind);
    if (s->distance != 1 && s->distance != 2 && s->distance != LAIR_DIST_ALL_F)
        fail(LAIR_EINVAL, "distance must be 1, 2 or LAIR_DIST_ALL_F");
    if (o->interp != LAIR_P_ONE_POINT && o->interp != LAIR_P_DIRECT)
        fail(LAIR_EINVAL, "unknown interpolation %d", o->interp);
    if (o->precision != LAIR_FP64 && o->precision != LAIR_MIXED &&
        o->precision != LAIR_MIXED_LOCAL)
        fail(LAIR_EINVAL, "unknown precision %d", o->precision);
    if (!(o->omega > 0.0 && o->omega <= 2.0)) fail(LAIR_EINVAL, "omega must lie in (0, 2]");
    if (o->max_levels < 1 || o->max_levels > 64) fail(LAIR_EINVAL, "max_levels must lie in [1, 64]");
    if (o->max_coarse < 1) fail(LAIR_EINVAL, "max_coarse must be >= 1");
    if (!(o->stall > 0.0 && o->stall <= 1.0)) fail(LAIR_EINVAL, "stall must lie in (0, 1]");
    if (o->block_size < 0 || o->block_size > 8) fail(LAIR_EINVAL, "block_size must lie in [0, 8]");
    if (o->flags & ~(LAIR_FLAG_NO_GRAPH | LAIR_FLAG_NATURAL_ORDER | LAIR_FLAG_SPLIT_ALL |
                     LAIR_FLAG_NODAL | LAIR_FLAG_PMIS))
        fail(LAIR_EINVAL, "unknown option flags 0x%x", o->flags);
    if (o->flags & LAIR_FLAG_NODAL) {
        if (o->block_size < 1) fail(LAIR_EINVAL, "the nodal treatment needs block_size >= 1");
        if (o->interp != LAIR_P_ONE_POINT)
            fail(LAIR_EUNSUPPORTED, "the nodal treatment interpolates by one point");
        if (s->distance != 1 && s->distance != 2)
            fail(LAIR_EUNSUPPORTED, "the nodal treatment uses distance 1 or 2");
        if (o->lump_tol > 0.0)
            fail(LAIR_EUNSUPPORTED, "lumping would break the dense blocks of a nodal hierarchy");
        if (o->flags & LAIR_FLAG_PMIS)
            fail(LAIR_EUNSUPPORTED, "a nodal hierarchy splits the graph of blocks on the host");
    }
    if ((o->flags & LAIR_FLAG_NATURAL_ORDER) && (o->flags & LAIR_FLAG_SPLIT_ALL))
        fail(LAIR_EINVAL, "NATURAL_ORDER and SPLIT_ALL exclude each other");
    if (!(o->lump_tol >= 0.0 && o->lump_tol <= 1.0))
        fail(LAIR_EINVAL, "lump_tol must lie in [0, 1]");
}

static const int32_t MAX_DENSE = 4096;

// ---------------------------------------------------------------------------
// Setup
// ---------------------------------------------------------------------------
// Strength, splitting, neighbourhoods, local solves, R and P of one level,
// and the product counts of A P (left in ap for the caller's product).
// Host synchronisations: the number of C-points with the F/C row lists,
// the neighbourhood sizes, and one readback after the local solves that
// also carries P's sizes and the count of products of A P.
static void build_level_transfer(lair_hierarchy *h, Level &Lv, int32_t lvl,
                                 const lair_cf_levels *cfl, bool &coarsest,
                                 DevArr<int64_t> &tmp, SpgemmState &ap) {
    hipStream_t s = h->stream;
    const int32_t n = Lv.n;
    const DevCSR &A = Lv.A;
    double mean = n ? (double)A.nnz / n : 1.0;
    const bool nod = nodal(h->opt);
    const int32_t kb = h->opt.block_size;
    if (nod) {
        // every level of a nodal hierarchy stores dense blocks (the Galerkin
        // product of dense blocks with identity-block P keeps them); the
        // kernels below index by that layout, so it is checked first
        if (n % kb != 0) fail(LAIR_EINVAL, "level %d: n = %d is not whole nodes", lvl, n);
        if (!node_check(n, kb, A.rp.get(), A.cj.get(), s))
            fail(LAIR_EINVAL, "level %d: the nodal treatment needs the k rows of a node to store "
                 "the same whole dense blocks", lvl);
    }
    Lv.smask.alloc((size_t)std::max<int64_t>(A.nnz, 1), s);
    if (nod)
        launch_node_strength(n, kb, A.rp.get(), A.cj.get(), A.v.get(), h->str.theta,
                             Lv.smask.get(), s);
    else
        launch_strength(n, A.rp.get(), A.cj.get(), A.v.get(), h->str.theta, h->str.kind,
                        Lv.smask.get(), mean, s);
    Lv.cf.alloc((size_t)n, s);
    if (cfl && lvl < cfl->nlevels) {
        int64_t lo = cfl->offs[lvl], hi = cfl->offs[lvl + 1];
        if (hi - lo != n)
            fail(LAIR_EINVAL, "CF splitting of level %d has %lld entries, level size is %d",
                 lvl, (long long)(hi - lo), n);
        // the splittings were uploaded (and checked) at the start of setup
        LAIR_HIP(hipMemcpyAsync(Lv.cf.get(), h->cf_dev.get() + lo, (size_t)n,
                                hipMemcpyDeviceToDevice, s));
    } else if (h->opt.flags & LAIR_FLAG_PMIS) {
        // the parallel splitting on the device
        const uint8_t *sm_dev = Lv.smask.get();
        DevArr<uint8_t> smc;
        if (h->str.theta_c != h->str.theta) {
            smc.alloc((size_t)std::max<int64_t>(A.nnz, 1), s);
            launch_strength(n, A.rp.get(), A.cj.get(), A.v.get(), h->str.theta_c,
                            h->str.kind, smc.get(), mean, s);
            sm_dev = smc.get();
        }
        ProfScope ps("split", s, 13.0 * A.nnz + 4.0 * n);
        launch_pmis_split(n, A.rp.get(), A.cj.get(), sm_dev, Lv.cf.get(), s);
    } else {
        // library's own classical first pass on a host copy of the pattern
        const uint8_t *sm_dev = Lv.smask.get();
        DevArr<uint8_t> smc;
        if (h->str.theta_c != h->str.theta) {
            smc.alloc((size_t)std::max<int64_t>(A.nnz, 1), s);
            if (nod)
                launch_node_strength(n, kb, A.rp.get(), A.cj.get(), A.v.get(), h->str.theta_c,
                                     smc.get(), s);
            else
                launch_strength(n, A.rp.get(), A.cj.get(), A.v.get(), h->str.theta_c,
                                h->str.kind, smc.get(), mean, s);
            sm_dev = smc.get();
        }
        std::vector<int32_t> hrp((size_t)n + 1), hcj((size_t)A.nnz);
        std::vector<uint8_t> hsm((size_t)A.nnz);
        std::vector<int8_t> hcf((size_t)n);
        LAIR_HIP(hipMemcpyAsync(hrp.data(), A.rp.get(), sizeof(int32_t) * (n + 1), hipMemcpyDeviceToHost, s));
        if (A.nnz) {
            LAIR_HIP(hipMemcpyAsync(hcj.data(), A.cj.get(), sizeof(int32_t) * A.nnz, hipMemcpyDeviceToHost, s));
            LAIR_HIP(hipMemcpyAsync(hsm.data(), sm_dev, (size_t)A.nnz, hipMemcpyDeviceToHost, s));
        }
        LAIR_HIP(hipStreamSynchronize(s));
        if (nod) {
            // the first pass on the graph of blocks (node i's first row, one
            // entry per block), each node's type given to its k rows
            const int32_t nn = n / kb;
            std::vector<int32_t> nrp((size_t)nn + 1, 0), ncj;
            std::vector<uint8_t> nsm;
            ncj.reserve((size_t)A.nnz / kb / kb + 1);
            nsm.reserve((size_t)A.nnz / kb / kb + 1);
            for (int32_t i = 0; i < nn; ++i) {
                for (int32_t p = hrp[(size_t)i * kb]; p < hrp[(size_t)i * kb + 1]; p += kb) {
                    ncj.push_back(hcj[p] / kb);
                    nsm.push_back(hsm[p]);
                }
                nrp[i + 1] = (int32_t)ncj.size();
            }
            std::vector<int8_t> ncf((size_t)nn);
            rs_first_pass(nn, nrp.data(), ncj.data(), nsm.data(), ncf.data());
            for (int32_t r = 0; r < n; ++r) hcf[r] = ncf[r / kb];
        } else {
            rs_first_pass(n, hrp.data(), hcj.data(), hsm.data(), hcf.data());
        }
        LAIR_HIP(hipMemcpyAsync(Lv.cf.get(), hcf.data(), (size_t)n, hipMemcpyHostToDevice, s));
        LAIR_HIP(hipStreamSynchronize(s));
    }
    std::vector<int64_t> seg_next;
    if (h->nsys > 1) {
        // systems that stopped coarsening keep all their points as C-points;
        // a system whose splitting has no C-point or stalls stops here
        const int32_t ns = h->nsys;
        Lv.stopped_dev.alloc((size_t)ns, s);
        LAIR_HIP(hipMemcpyAsync(Lv.stopped_dev.get(), Lv.stopped.data(), (size_t)ns,
                                hipMemcpyHostToDevice, s));
        launch_force_c(ns, Lv.seg_dev.get(), Lv.stopped_dev.get(), Lv.cf.get(), n, s);
        DevArr<int32_t> cnt;
        cnt.alloc((size_t)ns, s);
        launch_seg_count_c(ns, Lv.seg_dev.get(), Lv.cf.get(), cnt.get(), s);
        std::vector<int32_t> ncs((size_t)ns);
        {
            Readback rb(s);
            rb.add(ncs.data(), cnt.get(), sizeof(int32_t) * ns);
            rb.run();
        }
        bool newly = false, all = true;
        for (int32_t q = 0; q < ns; ++q) {
            int64_t nq = Lv.seg[q + 1] - Lv.seg[q];
            if (!Lv.stopped[q] && (ncs[q] == 0 || (double)ncs[q] > h->opt.stall * (double)nq)) {
                Lv.stopped[q] = 1;
                h->sys_levels[q] = lvl + 1;
                newly = true;
            }
            all = all && Lv.stopped[q];
        }
        if (all) {
            coarsest = true;
            Lv.smask.release();
            Lv.cf.release();
            return;
        }
        if (newly) {
            LAIR_HIP(hipMemcpyAsync(Lv.stopped_dev.get(), Lv.stopped.data(), (size_t)ns,
                                    hipMemcpyHostToDevice, s));
            launch_force_c(ns, Lv.seg_dev.get(), Lv.stopped_dev.get(), Lv.cf.get(), n, s);
        }
        seg_next.assign((size_t)ns + 1, 0);
        for (int32_t q = 0; q < ns; ++q) {
            int64_t nq = Lv.seg[q + 1] - Lv.seg[q];
            seg_next[q + 1] = seg_next[q] + (Lv.stopped[q] ? nq : (int64_t)ncs[q]);
        }
    }
    // coarse numbering and the F/C row lists in one pass with the count of
    // C-points (the lists are sized for every point until it is known)
    DevArr<int32_t> scan;
    scan.alloc((size_t)n + 1, s);
    DevArr<int64_t> nct;
    nct.alloc(2, s);
    scan_flags_i8_to(Lv.cf.get(), 1, scan.get(), n, s, tmp, nct.get());
    Lv.cidx.alloc((size_t)n, s);
    Lv.clist.alloc((size_t)std::max(n, 1), s);
    Lv.flist.alloc((size_t)std::max(n, 1), s);
    // the neighbourhoods' overflow flag, cleared before the readback below
    DevArr<int32_t> over;
    over.alloc(1, s);
    LAIR_HIP(hipMemsetAsync(over.get(), 0, sizeof(int32_t), s));
    int64_t nc = 0;
    {
        DevArr<unsigned long long> acc;
        acc.alloc(2 + 2 * (size_t)blocks_for(n, 256), s);
        ProfScope ps("cf_lists", s, 13.0 * n + 4.0 * n);
        launch_cf_lists(n, Lv.cf.get(), scan.get(), A.rp.get(), Lv.cidx.get(), Lv.clist.get(),
                        Lv.flist.get(), acc.get(), s);
        unsigned long long hacc[2];
        int64_t hn[2];
        Readback rb(s);
        rb.add(hacc, acc.get(), sizeof(hacc));
        rb.add(hn, nct.get(), sizeof(hn));
        rb.run();
        nc = hn[0];
        Lv.nnzF = (int64_t)hacc[0];
        Lv.nnzC = (int64_t)hacc[1];
    }
    if (h->nsys == 1 && (nc == 0 || (double)nc > h->opt.stall * (double)n)) {
        coarsest = true;
        Lv.smask.release();
        Lv.cf.release();
        Lv.cidx.release();
        Lv.clist.release();
        Lv.flist.release();
        return;
    }
    Lv.nc = (int32_t)nc;
    Lv.nf = n - Lv.nc;
    Lv.next_seg = std::move(seg_next);
    if (h->nsys > 1) {
        bool any = false;
        for (auto q : Lv.stopped) any = any || q;
        if (any)
            Lv.nrc = relax_list(h->nsys, Lv.seg_dev.get(), Lv.stopped_dev.get(), Lv.clist.get(),
                                Lv.nc, Lv.rclist, s, tmp);
    }

    // neighbourhoods
    DevArr<int32_t> cnt;
    cnt.alloc((size_t)Lv.nc + 1, s);
    launch_neighbourhoods(Lv.nc, n, Lv.clist.get(), A.rp.get(), A.cj.get(), Lv.smask.get(),
                          Lv.cf.get(), h->str.distance, Lv.flist.get(), Lv.nf, cnt.get(),
                          nullptr, nullptr, over.get(), Lv.max_row, s);
    Lv.nptr.alloc((size_t)Lv.nc + 1, s);
    // distance 1: N_i lies in row i without i, so the C rows' lengths bound
    // the lists' total and the longest row bounds each list; when that bound
    // keeps every system within the one-wave LDS kernel, the exact sizes wait
    // for the local solves' readback instead of a wait of their own
    const bool defer_nbr = h->str.distance == 1 && Lv.max_row > 0 && Lv.max_row - 1 <= WSMAX;
    DevArr<int64_t> ntot;
    int64_t smax64 = 0, nn = 0;
    if (defer_nbr) {
        ntot.alloc(2, s);
        scan_counts_i32_to(cnt.get(), Lv.nptr.get(), Lv.nc, s, tmp, ntot.get());
        nn = std::max<int64_t>(0, Lv.nnzC - Lv.nc);
        smax64 = Lv.max_row - 1;
    } else {
        int32_t ov = 0;
        nn = scan_counts_i32(cnt.get(), Lv.nptr.get(), Lv.nc, s, tmp, &smax64, over.get(), &ov);
        if (ov) fail(LAIR_EUNSUPPORTED, "level %d: a distance-2 neighbourhood merges more than 256 rows", lvl);
    }
    Lv.nbr.alloc((size_t)std::max<int64_t>(nn, 1), s);
    launch_neighbourhoods(Lv.nc, n, Lv.clist.get(), A.rp.get(), A.cj.get(), Lv.smask.get(),
                          Lv.cf.get(), h->str.distance, Lv.flist.get(), Lv.nf, nullptr,
                          Lv.nptr.get(), Lv.nbr.get(), over.get(), Lv.max_row, s);
    Lv.st.s_max = (int32_t)smax64;
    Lv.st.s_mean = Lv.nc ? (double)nn / Lv.nc : 0.0;
    Lv.st.s_min = -1;   // filled on demand by lair_level_stats_get

    // R = [Z I] (its size an upper bound until the readback when deferred)
    DevCSR &R = Lv.R;
    R.nrows = Lv.nc;
    R.ncols = n;
    R.nnz = nn + Lv.nc;
    R.rp.alloc((size_t)Lv.nc + 1, s);
    R.cj.alloc((size_t)R.nnz, s);
    R.v.alloc((size_t)R.nnz, s);
    LAIR_LAUNCH(k_r_rowptr, dim3(blocks_for(Lv.nc + 1, 256)), dim3(256), 0, s,
                       Lv.nc, Lv.nptr.get(), R.rp.get());
    LAIR_LAUNCH_CHECK();
    // P; its sizes stay on the device until the local solves' readback
    // (arrays sized by an upper bound: a row of P has at most as many
    // entries as the row of A)
    const bool eager = setup_sizes_eager();
    PendingSizes p_pend;
    DevCSR &P = Lv.P;
    P.nrows = n;
    P.ncols = Lv.nc;
    P.rp.alloc((size_t)n + 1, s);
    p_pend.arm(&P, "", s);
    if (h->opt.interp == LAIR_P_ONE_POINT) {
        DevArr<int32_t> pcol;
        pcol.alloc((size_t)n, s);
        {
            ProfScope ps("interp", s, 13.0 * A.nnz + 9.0 * n);
            if (nod)
                launch_interp_1p_node(n, kb, A.rp.get(), A.cj.get(), A.v.get(), Lv.smask.get(),
                                      Lv.cf.get(), Lv.cidx.get(), pcol.get(), s);
            else
                launch_interp_one_point(n, A.rp.get(), A.cj.get(), A.v.get(), Lv.smask.get(),
                                        Lv.cf.get(), Lv.cidx.get(), pcol.get(), s);
        }
        DevArr<int32_t> has;
        has.alloc((size_t)n, s);
        LAIR_LAUNCH(k_nonneg_flag, dim3(blocks_for(n, 256)), dim3(256), 0, s,
                           n, pcol.get(), has.get());
        LAIR_LAUNCH_CHECK();
        scan_counts_i32_to(has.get(), P.rp.get(), n, s, tmp, p_pend.tot());
        if (eager) p_pend.settle(s);
        else P.nnz = n;
        P.cj.alloc((size_t)std::max<int64_t>(P.nnz, 1), s);
        P.v.alloc((size_t)std::max<int64_t>(P.nnz, 1), s);
        launch_compact_one_point(n, pcol.get(), P.rp.get(), P.cj.get(), P.v.get(), s);
    } else {
        DevArr<int32_t> pc;
        pc.alloc((size_t)n, s);
        DevArr<double> coef;
        coef.alloc(3 * (size_t)std::max(n, 1), s);
        {
            ProfScope ps("interp", s, 6.0 * A.nnz + 9.0 * n);
            launch_interp_direct(n, A.rp.get(), A.cj.get(), A.v.get(), Lv.smask.get(),
                                 Lv.cf.get(), Lv.cidx.get(), false, pc.get(), nullptr, nullptr,
                                 nullptr, mean, s, coef.get());
        }
        scan_counts_i32_to(pc.get(), P.rp.get(), n, s, tmp, p_pend.tot());
        if (eager) p_pend.settle(s);
        else P.nnz = A.nnz;
        P.cj.alloc((size_t)std::max<int64_t>(P.nnz, 1), s);
        P.v.alloc((size_t)std::max<int64_t>(P.nnz, 1), s);
        {
            ProfScope ps("interp", s, 14.0 * A.nnz + 13.0 * n + 12.0 * P.nnz);
            launch_interp_direct(n, A.rp.get(), A.cj.get(), A.v.get(), Lv.smask.get(),
                                 Lv.cf.get(), Lv.cidx.get(), true, nullptr, P.rp.get(),
                                 P.cj.get(), P.v.get(), mean, s, coef.get());
        }
    }
    // products of A P counted now, read with the local solves
    spgemm_count(A, P, ap, s, tmp);
    Readback rb(s);
    p_pend.add(rb);
    rb.add(ap.h, ap.tot.get(), sizeof(ap.h));
    int64_t hnt[2] = {nn, smax64};
    if (defer_nbr) rb.add(hnt, ntot.get(), sizeof(hnt));

    Lv.flags.alloc((size_t)Lv.nc, s);
    LocalSolveOut out{R.rp.get(), R.cj.get(), R.v.get(), Lv.flags.get()};
    int64_t nsing = local_solves(Lv.nc, Lv.clist.get(), Lv.nptr.get(), Lv.nbr.get(),
                                 A.rp.get(), A.cj.get(), A.v.get(),
                                 h->opt.precision == LAIR_FP64 ? LAIR_FP64 : LAIR_MIXED,
                                 Lv.st.s_max, n ? (double)A.nnz / n : 0.0, out, s,
                                 Lv.buckets, &rb);
    p_pend.apply();
    if (defer_nbr) {
        R.nnz = hnt[0] + Lv.nc;
        Lv.st.s_max = (int32_t)hnt[1];
        Lv.st.s_mean = Lv.nc ? (double)hnt[0] / Lv.nc : 0.0;
    }
    Lv.st.n_singular = nsing;
    h->n_singular += nsing;
}

static const int32_t MAX_INVERSE = 512;

static void finish_coarsest_batch(lair_hierarchy *h) {
    hipStream_t s = h->stream;
    Level &Lc = *h->L.back();
    const int32_t ns = h->nsys;
    std::vector<int64_t> doff((size_t)ns + 1, 0);
    for (int32_t q = 0; q < ns; ++q) {
        int64_t m = Lc.seg[q + 1] - Lc.seg[q];
        if (m > MAX_DENSE)
            fail(LAIR_EUNSUPPORTED, "system %d has a coarsest level of %lld rows (> %d)", q,
                 (long long)m, MAX_DENSE);
        doff[q + 1] = doff[q] + m * m;
    }
    ProfScope ps("coarse_setup", s, 8.0 * (double)doff[ns], 0.0);
    h->nL = Lc.n;
    h->dense_off.alloc((size_t)ns + 1, s);
    LAIR_HIP(hipMemcpyAsync(h->dense_off.get(), doff.data(), sizeof(int64_t) * (ns + 1),
                            hipMemcpyHostToDevice, s));
    h->lu.alloc((size_t)std::max<int64_t>(doff[ns], 1), s);
    h->piv.alloc((size_t)std::max(Lc.n, 1), s);
    DevArr<int32_t> info;
    info.alloc(1, s);
    LAIR_HIP(hipMemsetAsync(info.get(), 0, sizeof(int32_t), s));
    launch_dense_blocks(ns, Lc.seg_dev.get(), h->dense_off.get(), Lc.A.rp.get(), Lc.A.cj.get(),
                        Lc.A.v.get(), h->lu.get(), Lc.n, s);
    // blocks up to small_dense_max() rows: LU and inverse in LDS, one wave
    // each; up to mid_dense_max() rows: LU, then the inverse in LDS chunks;
    // a product with the inverse per solve.  Larger blocks: LU, and
    // triangular solves per solve
    const int32_t small = small_dense_max();
    std::vector<uint8_t> ui((size_t)ns, 0);
    int64_t mmax = 0;
    bool any = false;
    for (int32_t q = 0; q < ns; ++q) {
        const int64_t m = Lc.seg[q + 1] - Lc.seg[q];
        if (m <= mid_dense_max()) {
            ui[q] = 1;
            any = true;
        }
        mmax = std::max(mmax, m);
    }
    h->use_inv.alloc((size_t)ns, s);
    LAIR_HIP(hipMemcpyAsync(h->use_inv.get(), ui.data(), (size_t)ns, hipMemcpyHostToDevice, s));
    if (any) h->binv.alloc((size_t)std::max<int64_t>(doff[ns], 1), s);
    else h->binv.release();
    launch_block_lu_inv_small(ns, Lc.seg_dev.get(), h->dense_off.get(), h->lu.get(),
                              h->piv.get(), h->binv.get(), info.get(), s);
    if (mmax > small) {
        launch_block_lu(ns, Lc.seg_dev.get(), h->dense_off.get(), h->lu.get(), h->piv.get(),
                        info.get(), s, small + 1);
        launch_block_inv_mid(ns, (int32_t)std::min<int64_t>(mmax, mid_dense_max()),
                             Lc.seg_dev.get(), h->dense_off.get(), h->lu.get(), h->piv.get(),
                             h->binv.get(), h->use_inv.get(), s);
    }
    int32_t hinfo = 0;
    {
        Readback rb(s);
        rb.add(&hinfo, info.get(), sizeof(int32_t));
        rb.run();
    }
    if (hinfo != 0)
        fail(LAIR_ESINGULAR, "the coarsest matrix of system %d is singular", hinfo - 1);
}

static void finish_coarsest(lair_hierarchy *h) {
    if (h->nsys > 1) {
        finish_coarsest_batch(h);
        return;
    }
    hipStream_t s = h->stream;
    Level &Lc = *h->L.back();
    int32_t n = Lc.n;
    if (n > MAX_DENSE)
        fail(LAIR_EUNSUPPORTED, "coarsest level has %d rows (> %d) after coarsening stalled",
             n, MAX_DENSE);
    ProfScope ps("coarse_setup", s, 8.0 * n * (double)n, 2.0 / 3.0 * n * (double)n * n);
    h->nL = n;
    h->lu.alloc((size_t)n * n, s);
    h->piv.alloc((size_t)std::max(n, 1), s);
    DevArr<int32_t> info;
    info.alloc(1, s);
    launch_dense_from_csr(n, Lc.A.rp.get(), Lc.A.cj.get(), Lc.A.v.get(), h->lu.get(), s);
    bool have_inv = false;
    if (n <= MAX_INVERSE) h->kinv.alloc((size_t)n * n, s);
    // small grids: the inverse directly, in one workgroup (the cycle only
    // applies the inverse; no factors are kept)
    if (n <= MAX_INVERSE && launch_dense_gj_inv(n, h->lu.get(), h->kinv.get(), info.get(), s))
        have_inv = true;
    else
        launch_dense_lu(n, h->lu.get(), h->piv.get(), info.get(), s);
    int32_t hinfo = 0;
    {
        Readback rb(s);
        rb.add(&hinfo, info.get(), sizeof(int32_t));
        rb.run();
    }
    if (hinfo != 0) {
        h->kinv.release();
        fail(LAIR_ESINGULAR, "coarsest matrix (n = %d) is singular at pivot %d", n, hinfo);
    }
    if (n <= MAX_INVERSE && !have_inv) {
        // K^{-1} from the LU factors, eight columns of the identity per block
        launch_dense_inverse(n, h->lu.get(), h->piv.get(), h->kinv.get(), s);
    }
}

static void level_stats_and_cc(lair_hierarchy *h) {
    double nnz0 = (double)h->L[0]->A.nnz;
    double flops = 0.0, sum = 0.0;
    for (size_t l = 0; l < h->L.size(); ++l) {
        Level &Lv = *h->L[l];
        Lv.st.n = Lv.n;
        Lv.st.nnz_A = Lv.A.nnz;
        Lv.st.nc = Lv.nc;
        Lv.st.nnz_R = Lv.R.nnz;
        Lv.st.nnz_P = Lv.P.nnz;
        sum += (double)Lv.A.nnz;
        if (l + 1 == h->L.size()) break;
        // residual, restriction, interpolation, then F, F, C Jacobi sweeps
        flops += 2.0 * Lv.A.nnz + 2.0 * Lv.R.nnz + 2.0 * Lv.P.nnz;
        flops += 2.0 * (2.0 * (double)Lv.nnzF + (double)Lv.nnzC);
    }
    double nl = (double)h->L.back()->n;
    flops += 2.0 * nl * nl;
    h->cc = flops / (2.0 * nnz0);
    h->oc = sum / nnz0;
}

// Split-ordered copies of the cycle operators (single systems).  A level is
// renumbered when it is large (in the natural ordering its F and C sweeps
// read and write the vectors line by line for half of the data); the
// renumbered levels form a prefix of the hierarchy and the coarsest level
// keeps its natural ordering (its dense solve).  Mixed precision keeps
// float values only.
constexpr int32_t SPLIT_MIN_ROWS = 65536;

static void build_split(lair_hierarchy *h, hipStream_t s) {
    const size_t nL = h->L.size();
    const bool mixed = h->opt.precision == LAIR_MIXED;
    const bool allowed = h->nsys == 1 && nL > 1 && !(h->opt.flags & LAIR_FLAG_NATURAL_ORDER) &&
                         !nodal(h->opt);
    const bool all = (h->opt.flags & LAIR_FLAG_SPLIT_ALL) != 0;
    bool prev = allowed;
    for (size_t l = 0; l < nL; ++l) {
        Level &Lv = *h->L[l];
        const bool big = Lv.n >= SPLIT_MIN_ROWS;
        Lv.split = prev && l + 1 < nL && (all || big);
        prev = Lv.split;
    }
    DevArr<int64_t> tmp;
    for (size_t l = 0; l + 1 < nL; ++l) {
        Level &Lv = *h->L[l];
        if (!Lv.split) continue;
        const size_t n = (size_t)std::max(Lv.n, 1);
        Lv.perm.alloc(n, s);
        Lv.iperm.alloc(n, s);
        Lv.ids.alloc(n, s);
        Lv.cf_split.alloc(n, s);
        launch_split_perm(Lv.nf, Lv.nc, Lv.flist.get(), Lv.clist.get(), Lv.perm.get(),
                          Lv.iperm.get(), Lv.ids.get(), Lv.cf_split.get(), s);
    }
    auto copy = [&](const DevCSR &M, DevCSR &O, const int32_t *rowmap, const int32_t *colmap,
                    DevArr<int32_t> *cjt, int32_t nsplit) {
        O.nrows = M.nrows;
        O.ncols = M.ncols;
        O.nnz = M.nnz;
        O.max_row = M.max_row;
        const size_t z = (size_t)std::max<int64_t>(M.nnz, 1);
        O.rp.alloc((size_t)M.nrows + 1, s);
        O.cj.alloc(z, s);
        if (!mixed) O.v.alloc(z, s); else O.v.release();
        if (mixed) O.v32.alloc(z, s); else O.v32.release();
        if (cjt) cjt->alloc(z, s);
        launch_permute_csr(M.nrows, M.nnz, M.nrows ? (double)M.nnz / M.nrows : 0.0, rowmap,
                           colmap, M.rp.get(), M.cj.get(), M.v.get(), O.rp.get(), O.cj.get(),
                           mixed ? nullptr : O.v.get(), mixed ? O.v32.get() : nullptr,
                           cjt ? cjt->get() : nullptr, nsplit, tmp, s);
    };
    auto drop = [](DevCSR &O) {
        O.rp.release(); O.cj.release(); O.v.release(); O.v32.release();
        O.nrows = O.ncols = 0; O.nnz = 0;
    };
    for (size_t l = 0; l + 1 < nL; ++l) {
        Level &Lv = *h->L[l];
        Level &Nx = *h->L[l + 1];
        const int32_t *perm = Lv.split ? Lv.perm.get() : nullptr;
        const int32_t *iperm = Lv.split ? Lv.iperm.get() : nullptr;
        const int32_t *nperm = Nx.split ? Nx.perm.get() : nullptr;
        const int32_t *niperm = Nx.split ? Nx.iperm.get() : nullptr;
        if (Lv.split) {
            copy(Lv.A, Lv.As, perm, iperm, &Lv.cjt_split, Lv.nf);
        } else {
            drop(Lv.As);
            Lv.cjt_split.release();
        }
        if (Lv.split || Nx.split) {
            copy(Lv.R, Lv.Rs, nperm, iperm, nullptr, 0);
            copy(Lv.P, Lv.Ps, perm, niperm, nullptr, 0);
        } else {
            drop(Lv.Rs);
            drop(Lv.Ps);
        }
    }
}

// After the values of a hierarchy are set: split-ordered copies, the tagged
// columns and float values of whatever the cycle reads in the natural
// ordering.
static void finish_cycle_operators(lair_hierarchy *h, hipStream_t s) {
    build_split(h, s);
    const bool mixed = h->opt.precision == LAIR_MIXED;
    if (nodal(h->opt)) {
        // block Jacobi: D^{-1} of every level's diagonal blocks and the
        // values of D^{-1} A, read by the sweeps as a scalar Jacobi on them
        const int32_t k = h->opt.block_size;
        DevArr<int32_t> bad;
        bad.alloc(1, s);
        LAIR_HIP(hipMemsetAsync(bad.get(), 0, sizeof(int32_t), s));
        for (size_t l = 0; l + 1 < h->L.size(); ++l) {
            Level &Lv = *h->L[l];
            const int32_t nblk = Lv.n / k;
            Lv.ndinv.alloc((size_t)std::max(nblk, 1) * k * k, s);
            launch_block_inverse(nblk, k, Lv.A.rp.get(), Lv.A.cj.get(), Lv.A.v.get(),
                                 Lv.ndinv.get(), bad.get(), s);
            Lv.av.alloc((size_t)std::max<int64_t>(Lv.A.nnz, 1), s);
            launch_node_scale(Lv.n, k, Lv.A.rp.get(), Lv.A.v.get(), Lv.ndinv.get(), Lv.av.get(),
                              s);
            if (mixed) {
                Lv.av32.alloc((size_t)std::max<int64_t>(Lv.A.nnz, 1), s);
                launch_to_float(Lv.av.get(), Lv.av32.get(), Lv.A.nnz, s);
            }
        }
        int32_t hb = 0;
        Readback rb(s);
        rb.add(&hb, bad.get(), sizeof(int32_t));
        rb.run();
        if (hb) fail(LAIR_ESINGULAR, "a %dx%d diagonal block of a nodal level is singular", k, k);
    }
    for (size_t l = 0; l < h->L.size(); ++l) {
        Level &Lv = *h->L[l];
        if (l + 1 < h->L.size() && !Lv.split && !Lv.cjt.get()) {
            Lv.cjt.alloc((size_t)std::max<int64_t>(Lv.A.nnz, 1), s);
            launch_tag_columns(Lv.A.nnz, Lv.A.cj.get(), Lv.cf.get(), Lv.cjt.get(), s);
        }
        if (!mixed) continue;
        if (!Lv.split) {
            if (Lv.A.v32.get() == nullptr)
                Lv.A.v32.alloc((size_t)std::max<int64_t>(Lv.A.nnz, 1), s);
            launch_to_float(Lv.A.v.get(), Lv.A.v32.get(), Lv.A.nnz, s);
        }
        if (Lv.R.nnz && !Lv.Rs.rp.get()) {
            if (Lv.R.v32.get() == nullptr) Lv.R.v32.alloc((size_t)Lv.R.nnz, s);
            launch_to_float(Lv.R.v.get(), Lv.R.v32.get(), Lv.R.nnz, s);
        }
        if (Lv.P.nnz && !Lv.Ps.rp.get()) {
            if (Lv.P.v32.get() == nullptr) Lv.P.v32.alloc((size_t)Lv.P.nnz, s);
            launch_to_float(Lv.P.v.get(), Lv.P.v32.get(), Lv.P.nnz, s);
        }
    }
}

static void upload_seg(Level &Lv, hipStream_t s) {
    Lv.seg_dev.alloc(Lv.seg.size(), s);
    LAIR_HIP(hipMemcpyAsync(Lv.seg_dev.get(), Lv.seg.data(), sizeof(int64_t) * Lv.seg.size(),
                            hipMemcpyHostToDevice, s));
}

// seg: row offsets of the systems of a batch (nsys + 1 entries), or NULL.
static lair_hierarchy *setup_impl(const lair_csr *Ain, const lair_cf_levels *cfl,
                                  const lair_strength *str, const lair_options *opt,
                                  hipStream_t s, const std::vector<int64_t> *seg = nullptr) {
    auto t0 = Clock::now();
    if (!Ain) fail(LAIR_EINVAL, "A must not be NULL");
    check_options(str, opt);
    if (Ain->n < 1 || Ain->n >= INT32_MAX) fail(LAIR_EINVAL, "n = %lld out of range", (long long)Ain->n);
    if (Ain->nnz < Ain->n || Ain->nnz >= INT32_MAX)
        fail(LAIR_EINVAL, "nnz = %lld out of range (needs n <= nnz < 2^31)", (long long)Ain->nnz);
    if (!Ain->rowptr || !Ain->col || !Ain->val) fail(LAIR_EINVAL, "CSR arrays must not be NULL");
    if (cfl && cfl->nlevels > 0 && (!cfl->offs || !cfl->cf))
        fail(LAIR_EINVAL, "cf levels given without arrays");
    if (cfl && cfl->nlevels < 0) fail(LAIR_EINVAL, "negative number of CF levels");
    if (opt->block_size > 0 && Ain->n % opt->block_size != 0)
        fail(LAIR_EINVAL, "n is not a multiple of block_size");
    int dev_count = 0;
    if (hipGetDeviceCount(&dev_count) != hipSuccess || dev_count < 1)
        fail(LAIR_EDEVICE, "no HIP device available");
    std::unique_ptr<lair_hierarchy> h(new lair_hierarchy());
    h->str = *str;
    h->opt = *opt;
    h->stream = s;
    DevArr<int64_t> tmp;

    const int32_t n = (int32_t)Ain->n;
    const int64_t nnz = Ain->nnz;
    if (cfl && cfl->nlevels > 0) {
        // check the caller's splittings and upload them in one pinned copy
        int64_t total = cfl->offs[cfl->nlevels];
        if (cfl->offs[0] != 0 || total < 0) fail(LAIR_EINVAL, "bad CF level offsets");
        for (int32_t l = 0; l < cfl->nlevels; ++l)
            if (cfl->offs[l + 1] < cfl->offs[l]) fail(LAIR_EINVAL, "bad CF level offsets");
        uint8_t bad = 0;
        const uint8_t *cfb = (const uint8_t *)cfl->cf;
        for (int64_t k = 0; k < total; ++k) bad |= cfb[k] & 0xFE;
        if (bad) fail(LAIR_EINVAL, "a CF splitting holds a value other than 0/1");
        if (total > 0) {
            int8_t *stage = (int8_t *)pinned_staging((size_t)total);
            memcpy(stage, cfl->cf, (size_t)total);
            h->cf_dev.alloc((size_t)total, s);
            LAIR_HIP(hipMemcpyAsync(h->cf_dev.get(), stage, (size_t)total,
                                    hipMemcpyHostToDevice, s));
            LAIR_HIP(hipStreamSynchronize(s));   // the staging buffer is reused
        }
    }
    std::unique_ptr<Level> L0(new Level());
    L0->n = n;
    if (seg) {
        h->batch = true;
        h->nsys = (int32_t)seg->size() - 1;
        h->sys_levels.assign((size_t)h->nsys, 0);
        L0->seg = *seg;
        L0->stopped.assign((size_t)h->nsys, 0);
        upload_seg(*L0, s);
    }
    DevCSR &A = L0->A;
    A.nrows = A.ncols = n;
    A.nnz = nnz;
    A.rp.alloc((size_t)n + 1, s);
    A.cj.alloc((size_t)nnz, s);
    A.v.alloc((size_t)nnz, s);
    hipMemcpyKind kind = Ain->on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    LAIR_HIP(hipMemcpyAsync(A.rp.get(), Ain->rowptr, sizeof(int32_t) * (n + 1), kind, s));
    LAIR_HIP(hipMemcpyAsync(A.cj.get(), Ain->col, sizeof(int32_t) * nnz, kind, s));
    LAIR_HIP(hipMemcpyAsync(A.v.get(), Ain->val, sizeof(double) * nnz, kind, s));
    L0->max_row = validate_csr(n, nnz, A.rp.get(), A.cj.get(), A.v.get(), s);
    A.max_row = L0->max_row;

    if (nodal(*opt) && cfl && cfl->nlevels > 0) {
        // the caller's splittings must give the k rows of a node one type
        const int32_t k = opt->block_size;
        for (int32_t l = 0; l < cfl->nlevels; ++l) {
            const int64_t lo = cfl->offs[l], hi = cfl->offs[l + 1];
            if ((hi - lo) % k) fail(LAIR_EINVAL, "CF splitting of level %d is not whole nodes", l);
            for (int64_t q = lo; q < hi; ++q)
                if (cfl->cf[q] != cfl->cf[lo + (q - lo) / k * k])
                    fail(LAIR_EINVAL, "CF splitting of level %d splits a node", l);
        }
    }
    if (scaled(*opt)) {
        int32_t k = opt->block_size;
        int32_t nblk = n / k;
        h->dinv.alloc((size_t)nblk * k * k, s);
        DevArr<int32_t> bad;
        bad.alloc(1, s);
        LAIR_HIP(hipMemsetAsync(bad.get(), 0, sizeof(int32_t), s));
        launch_block_inverse(nblk, k, A.rp.get(), A.cj.get(), A.v.get(), h->dinv.get(),
                             bad.get(), s);
        int32_t hb = 0;
        {
            Readback rb(s);
            rb.add(&hb, bad.get(), sizeof(int32_t));
            rb.run();
        }
        if (hb) fail(LAIR_ESINGULAR, "a %dx%d diagonal block is singular", k, k);
        DevCSR D;
        D.nrows = D.ncols = n;
        D.nnz = (int64_t)n * k;
        D.rp.alloc((size_t)n + 1, s);
        D.cj.alloc((size_t)D.nnz, s);
        D.v.alloc((size_t)D.nnz, s);
        LAIR_LAUNCH(k_block_diag_csr, dim3(blocks_for(D.nnz + 1, 256)), dim3(256), 0, s,
                           nblk, k, h->dinv.get(), D.rp.get(), D.cj.get(), D.v.get());
        LAIR_LAUNCH_CHECK();
        DevCSR As;
        L0->max_row = spgemm(D, k, A, As, s, tmp);
        LAIR_LAUNCH(k_unit_diag_blocks, dim3(blocks_for((int64_t)n * 8, 256)), dim3(256), 0, s,
                    n, k, As.rp.get(), As.cj.get(), As.v.get());
        LAIR_LAUNCH_CHECK();
        L0->A = std::move(As);
    }
    h->L.push_back(std::move(L0));

    // products per distinct column of A P and of R (A P) on the level above:
    // the next level's hash tables are sized from them
    double ap_ratio = 0.0, k_ratio = 0.0;
    for (int32_t lvl = 0;; ++lvl) {
        Level &Lv = *h->L.back();
        if (h->nsys == 1) {
            if (Lv.n <= opt->max_coarse || lvl + 1 >= opt->max_levels) break;
        } else {
            // each system stops under the single-system rules
            bool all = true;
            for (int32_t q = 0; q < h->nsys; ++q) {
                int64_t nq = Lv.seg[q + 1] - Lv.seg[q];
                if (!Lv.stopped[q] && (nq <= opt->max_coarse || lvl + 1 >= opt->max_levels)) {
                    Lv.stopped[q] = 1;
                    h->sys_levels[q] = lvl + 1;
                }
                all = all && Lv.stopped[q];
            }
            if (all) break;
        }
        bool coarsest = false;
        SpgemmState ap_st;
        build_level_transfer(h.get(), Lv, lvl, cfl, coarsest, tmp, ap_st);
        if (coarsest) break;
        // Galerkin product K = R (A P): the sizes of A P reach the host with
        // the count of products of R (A P)
        DevCSR AP;
        PendingSizes ap_pend;
        const bool eager = setup_sizes_eager();
        spgemm_finish(Lv.A, Lv.P, AP, ap_st, s, tmp, eager ? nullptr : &ap_pend, ap_ratio);
        std::unique_ptr<Level> nx(new Level());
        nx->n = Lv.nc;
        if (h->nsys > 1) {
            nx->seg = Lv.next_seg;
            nx->stopped = Lv.stopped;
            upload_seg(*nx, s);
        }
        // a batch keeps the blocks of its stopped systems as they are: the
        // single-system hierarchy lumps a coarse operator once, when it is
        // formed, and never the coarsest level again
        DevArr<int8_t> whole;
        if (h->nsys > 1 && opt->lump_tol > 0.0) {
            whole.alloc((size_t)std::max(Lv.nc, 1), s);
            launch_stopped_rows(h->nsys, nx->seg_dev.get(), Lv.stopped_dev.get(), whole.get(),
                                Lv.nc, s);
        }
        SpgemmState k_st;
        spgemm_count(Lv.R, AP, k_st, s, tmp);
        {
            Readback rb(s);
            rb.add(k_st.h, k_st.tot.get(), sizeof(k_st.h));
            ap_pend.add(rb);
            rb.run();
            ap_pend.apply();
        }
        if (AP.nnz > 0) ap_ratio = (double)ap_st.h[0] / (double)AP.nnz;
        // rows of K are sorted and unique by construction of the product
        int64_t k_distinct = -1;
        nx->max_row = spgemm_finish(Lv.R, AP, nx->A, k_st, s, tmp, nullptr, k_ratio,
                                    opt->lump_tol, &k_distinct, whole.get());
        if (k_distinct < 0) k_distinct = nx->A.nnz;
        if (k_distinct > 0) k_ratio = (double)k_st.h[0] / (double)k_distinct;
        h->L.push_back(std::move(nx));
    }
    finish_coarsest(h.get());
    for (auto &lp : h->L) {
        Level &Lv = *lp;
        Lv.team_A = team_of(Lv.A);
        Lv.team_R = team_of(Lv.R);
        Lv.team_P = team_of(Lv.P);
    }
    finish_cycle_operators(h.get(), s);
    level_stats_and_cc(h.get());
    LAIR_HIP(hipStreamSynchronize(s));
    h->setup_ms = ms_since(t0);
    return h.release();
}

// ---------------------------------------------------------------------------
// Cycle
// ---------------------------------------------------------------------------
static void ensure_vectors(lair_hierarchy *h, int32_t nrhs, hipStream_t s) {
    if (nrhs <= h->nrhs_cap) return;
    h->drop_graphs();     // captured iterations refer to the old buffers
    bool mixed = h->opt.precision == LAIR_MIXED;
    for (size_t l = 0; l < h->L.size(); ++l) {
        Level &Lv = *h->L[l];
        size_t n = (size_t)Lv.n * nrhs;
        size_t tn = (size_t)std::max(Lv.n, 1) * nrhs;
        Lv.b.alloc(n, s);
        Lv.x.alloc(n, s);
        Lv.r.alloc(n, s);
        Lv.t.alloc(tn, s);
        if (mixed) {
            Lv.b32.alloc(n, s);
            Lv.x32.alloc(n, s);
            Lv.r32.alloc(n, s);
            Lv.t32.alloc(tn, s);
        }
    }
    size_t n0 = (size_t)h->L[0]->n * nrhs;
    h->r0.alloc(n0, s);
    if (scaled(h->opt)) h->bscaled.alloc(n0, s);
    if (nodal(h->opt))
        for (size_t l = 0; l + 1 < h->L.size(); ++l) {
            Level &Lv = *h->L[l];
            size_t n = (size_t)std::max(Lv.n, 1) * nrhs;
            Lv.bt.alloc(n, s);
            if (mixed) Lv.bt32.alloc(n, s);
        }
    if (mixed) {
        h->r0_32.alloc(n0, s);
        h->e32.alloc(n0, s);
    }
    if (h->L[0]->split && !mixed) {
        h->bsplit.alloc(n0, s);
        h->xsplit.alloc(n0, s);
    }
    h->partial.alloc((size_t)NPARTIAL * nrhs, s);
    h->norms.alloc((size_t)nrhs, s);
    h->nrhs_cap = nrhs;
}

template <class VT>
static VT *vec(DevArr<double> &d, DevArr<float> &f) {
    if constexpr (std::is_same<VT, double>::value) { (void)f; return d.get(); }
    else { (void)d; return f.get(); }
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
    ProfScope ps("coarse_solve", s, 8.0 * h->nL * (double)h->nL + 2.0 * w * nrhs * h->nL,
                 2.0 * h->nL * (double)h->nL * nrhs);
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
template <class VT>
static void ffc(lair_hierarchy *h, Level &Lv, const VT *b, VT *x, int32_t nrhs,
                hipStream_t s) {
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
    {
        ProfScope ps("jacobi", s, ab_jacobi(Lv.nnzC, ncr, Lv.n, w, nrhs, false),
                     2.0 * Lv.nnzC * nrhs);
        op_jacobi<VT>(A, crows, ncr, b, x, x, nullptr, y, true, om, nrhs, s, ccnt, c0);
    }
    {
        ProfScope ps("scatter", s, 4.0 * ncr + 2.0 * w * nrhs * ncr);
        op_scatter<VT>(crows, ncr, y, x, nrhs, s, ccnt, c0);
    }
}

// V-cycle from level l.  With x_zero the incoming iterate is zero: the
// residual is b itself and the interpolated correction is assigned.  When
// r is non-null it already holds b - A x.
template <class VT>
static void vcycle(lair_hierarchy *h, size_t l, const VT *b, VT *x, bool x_zero,
                   const VT *r, int32_t nrhs, hipStream_t s) {
    Level &Lv = *h->L[l];
    const int w = sizeof(VT);
    if (l + 1 == h->L.size()) {
        coarse_solve<VT>(h, b, x, nrhs, false, s);
        return;
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
    vcycle<VT>(h, l + 1, bc, xc, true, nullptr, nrhs, s);
    {
        ProfScope ps("interpolate", s, ab_rowdot(Lv.P, w, nrhs, x_zero ? 1 : 2),
                     2.0 * Lv.P.nnz * nrhs);
        if (h->use_act)
            op_rowdot_list<VT>(view<VT>(Lv.P, Lv.team_P), x_zero ? 1 : 2, Lv.act_rows.get(),
                               Lv.act_cnt, Lv.n, xc, nullptr, x, s);
        else
            op_spmv<VT>(view<VT>(Lv.Ps.rp.get() ? Lv.Ps : Lv.P, Lv.team_P), xc, x, nrhs, !x_zero,
                        s);
    }
    ffc<VT>(h, Lv, b, x, nrhs, s);
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

static void check_nrhs(const lair_hierarchy *h, int32_t nrhs) {
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

// Run body(stream) on s: replay its captured graph, capturing it first on
// the hierarchy's private stream.  body must launch kernels only (no
// allocation, no host synchronisation, no memset).
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
    LAIR_HIP(hipGraphLaunch(exec, s));
}

static void check_solve_args(lair_hierarchy *h, const double *b, double *x, double rtol,
                             int32_t maxit) {
    if (!h) fail(LAIR_EINVAL, "hierarchy is NULL");
    if (!b || !x) fail(LAIR_EINVAL, "b and x must not be NULL");
    if (!(rtol > 0.0) || maxit < 0) fail(LAIR_EINVAL, "need rtol > 0 and maxit >= 0");
}

static lair_status solve_impl(lair_hierarchy *h, const double *b, double *x,
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
    for (;;) {
        relmax = 0.0;
        bool done = true;
        for (int32_t q = 0; q < nrhs; ++q) {
            double rel = nb[q] > 0 ? rn[q] / nb[q] : rn[q];
            relmax = std::max(relmax, rel);
            if (!(rel <= rtol)) done = false;
        }
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
                vcycle<float>(h, 0, h->r0_32.get(), h->e32.get(), true, nullptr, nrhs, st);
                {
                    ProfScope ps("cast", st, 20.0 * n * nrhs);
                    if (orow) op_axpy_f32_rows(x, h->e32.get(), orow, n, nrhs, st);
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
        info->nlevels = (int32_t)h->L.size();
        info->relres = relmax;
        double rho = 0.0;
        if (it > 0 && !r_first.empty()) {
            for (int32_t q = 0; q < nrhs; ++q)
                if (r_first[q] > 0) rho = std::max(rho, std::pow(rn[q] / r_first[q], 1.0 / it));
        }
        info->rho = rho;
        info->cycle_complexity = h->cc;
        info->op_complexity = h->oc;
        info->n_singular_local = h->n_singular;
        info->setup_ms = h->setup_ms;
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
static lair_status solve_fgmres_impl(lair_hierarchy *h, const double *b, double *x,
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
        info->nlevels = (int32_t)h->L.size();
        info->relres = relmax;
        double rho = 0.0;
        if (itmax > 0)
            for (int32_t q = 0; q < R; ++q)
                if (r_first[q] > 0 && its[q] > 0)
                    rho = std::max(rho, std::pow(beta[q] / r_first[q], 1.0 / its[q]));
        info->rho = rho;
        info->cycle_complexity = h->cc;
        info->op_complexity = h->oc;
        info->n_singular_local = h->n_singular;
        info->setup_ms = h->setup_ms;
        info->solve_ms = ms_since(t0);
    }
    return relmax <= rtol ? LAIR_OK : LAIR_ENOCONV;
}

// Batch of independent systems (one right-hand side each): the correction
// form x += B (b - A x) on the union, with the residual rows of converged
// systems zeroed so that their corrections vanish.  Each system stops at its
// own relative residual.
static lair_status solve_batch_impl(lair_hierarchy *h, const double *b, double *x,
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
        info->nlevels = (int32_t)h->L.size();
        info->relres = relmax;
        double rho = 0.0;
        for (int32_t q = 0; q < ns; ++q)
            if (its[q] > 0 && rfirst[q] > 0)
                rho = std::max(rho, std::pow(rel[q] * nb[q] / rfirst[q], 1.0 / its[q]));
        info->rho = rho;
        info->cycle_complexity = h->cc;
        info->op_complexity = h->oc;
        info->n_singular_local = h->n_singular;
        info->setup_ms = h->setup_ms;
        info->solve_ms = ms_since(t0);
    }
    return conv ? LAIR_OK : LAIR_ENOCONV;
}

// ---------------------------------------------------------------------------
// New diagonal, same hierarchy structure: the strength masks, splittings,
// neighbourhoods and every sparsity pattern are kept; the local solves, the
// interpolation weights, the Galerkin products and the coarsest factors are
// recomputed from the new level-0 values.
// ---------------------------------------------------------------------------
__global__ void k_check_diag(int32_t n, const double *d, int32_t *bad) {
    int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double x = d[i];
    if (!isfinite(x) || x == 0.0) atomicOr(bad, 1);
}

__global__ void k_set_diag(int32_t n, const int32_t *rp, const int32_t *cj, double *v,
                           const double *d) {
    int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int lo = rp[i], hi = rp[i + 1] - 1;
    while (lo <= hi) {                         // columns are sorted; the diagonal is stored
        int mid = (lo + hi) >> 1;
        int c = cj[mid];
        if (c == i) { v[mid] = d[i]; return; }
        if (c < i) lo = mid + 1; else hi = mid - 1;
    }
}

static void update_diag_impl(lair_hierarchy *h, const double *diag, int32_t on_device,
                             hipStream_t s) {
    if (!h || !diag) fail(LAIR_EINVAL, "hierarchy and diag must not be NULL");
    if (scaled(h->opt))
        fail(LAIR_EUNSUPPORTED, "a new diagonal changes the block scaling: set up again");
    if (nodal(h->opt))
        fail(LAIR_EUNSUPPORTED, "a new diagonal on a nodal hierarchy: set up again");
    if (h->opt.lump_tol > 0.0)
        fail(LAIR_EUNSUPPORTED, "lumped coarse patterns depend on the values: set up again");
    h->stream = s;
    Level &L0 = *h->L[0];
    const int32_t n = L0.n;
    DevArr<double> d;
    const double *dd = diag;
    if (!on_device) {
        d.alloc((size_t)n, s);
        LAIR_HIP(hipMemcpyAsync(d.get(), diag, sizeof(double) * n, hipMemcpyHostToDevice, s));
        LAIR_HIP(hipStreamSynchronize(s));     // diag is pageable caller memory
        dd = d.get();
    }
    DevArr<int32_t> bad;
    bad.alloc(1, s);
    LAIR_HIP(hipMemsetAsync(bad.get(), 0, sizeof(int32_t), s));
    LAIR_LAUNCH(k_check_diag, dim3(blocks_for(n, 256)), dim3(256), 0, s, n, dd, bad.get());
    LAIR_LAUNCH_CHECK();
    int32_t hb = 0;
    {
        Readback rb(s);
        rb.add(&hb, bad.get(), sizeof(int32_t));
        rb.run();
    }
    if (hb) fail(LAIR_EINVAL, "the new diagonal has a zero or non-finite entry");
    LAIR_LAUNCH(k_set_diag, dim3(blocks_for(n, 256)), dim3(256), 0, s, n, L0.A.rp.get(),
                L0.A.cj.get(), L0.A.v.get(), dd);
    LAIR_LAUNCH_CHECK();
    h->drop_graphs();
    h->have_transpose = false;
    h->n_singular = 0;
    DevArr<int64_t> tmp;
    const int32_t prec = h->opt.precision == LAIR_FP64 ? LAIR_FP64 : LAIR_MIXED;
    for (size_t l = 0; l + 1 < h->L.size(); ++l) {
        Level &Lv = *h->L[l];
        const DevCSR &A = Lv.A;
        LocalSolveOut out{Lv.R.rp.get(), Lv.R.cj.get(), Lv.R.v.get(), Lv.flags.get()};
        int64_t nsing = local_solves(Lv.nc, Lv.clist.get(), Lv.nptr.get(), Lv.nbr.get(),
                                     A.rp.get(), A.cj.get(), A.v.get(), prec, Lv.st.s_max,
                                     Lv.n ? (double)A.nnz / Lv.n : 0.0, out, s, Lv.buckets);
        Lv.st.n_singular = nsing;
        h->n_singular += nsing;
        if (h->opt.interp == LAIR_P_DIRECT) {
            // one-point weights are 1 on a kept pattern; direct weights use values
            ProfScope ps("interp", s, 14.0 * A.nnz + 13.0 * Lv.n + 12.0 * Lv.P.nnz);
            launch_interp_direct(Lv.n, A.rp.get(), A.cj.get(), A.v.get(), Lv.smask.get(),
                                 Lv.cf.get(), Lv.cidx.get(), true, nullptr, Lv.P.rp.get(),
                                 Lv.P.cj.get(), Lv.P.v.get(),
                                 Lv.n ? (double)A.nnz / Lv.n : 1.0, s);
        }
        DevCSR AP, K;
        spgemm(Lv.A, Lv.max_row, Lv.P, AP, s, tmp);
        int32_t mr = spgemm(Lv.R, Lv.st.s_max + 1, AP, K, s, tmp, h->L[l + 1]->A.nnz);
        Level &Nx = *h->L[l + 1];
        if (K.nnz != Nx.A.nnz)
            fail(LAIR_EDEVICE, "coarse operator pattern changed on update (level %zu)", l + 1);
        Nx.A = std::move(K);
        Nx.max_row = mr;
    }
    finish_coarsest(h);
    finish_cycle_operators(h, s);
    level_stats_and_cc(h);
    LAIR_HIP(hipStreamSynchronize(s));
}

// Union of a batch: the systems' matrices placed block-diagonally, rows of
// system q at [seg[q], seg[q+1]).
static lair_hierarchy *setup_batch_impl(int32_t nsys, const lair_csr *sys,
                                        const lair_cf_levels *cfl, const lair_strength *str,
                                        const lair_options *opt, hipStream_t s) {
    if (nsys < 1) fail(LAIR_EINVAL, "nsys must be >= 1");
    if (!sys) fail(LAIR_EINVAL, "the system array must not be NULL");
    check_options(str, opt);
    if (nodal(*opt)) fail(LAIR_EUNSUPPORTED, "batches are not built by nodes");
    std::vector<int64_t> seg((size_t)nsys + 1, 0), nzo((size_t)nsys + 1, 0);
    const int32_t dev = sys[0].on_device;
    for (int32_t q = 0; q < nsys; ++q) {
        const lair_csr &M = sys[q];
        if (M.n < 1 || M.nnz < M.n) fail(LAIR_EINVAL, "system %d: need n >= 1 and nnz >= n", q);
        if (!M.rowptr || !M.col || !M.val) fail(LAIR_EINVAL, "system %d: NULL CSR array", q);
        if ((M.on_device != 0) != (dev != 0))
            fail(LAIR_EINVAL, "all systems must be on the host or all on the device");
        if (opt->block_size > 0 && M.n % opt->block_size != 0)
            fail(LAIR_EINVAL, "system %d: n is not a multiple of block_size", q);
        seg[q + 1] = seg[q] + M.n;
        nzo[q + 1] = nzo[q] + M.nnz;
    }
    if (seg[nsys] >= INT32_MAX || nzo[nsys] >= INT32_MAX)
        fail(LAIR_EINVAL, "the union has %lld rows and %lld entries (each must be < 2^31)",
             (long long)seg[nsys], (long long)nzo[nsys]);
    const int64_t n = seg[nsys], nnz = nzo[nsys];
    lair_csr U{n, nnz, nullptr, nullptr, nullptr, 0};
    std::vector<int32_t> hrp, hcj;
    std::vector<double> hv;
    DevArr<int32_t> drp, dcj;
    DevArr<double> dv;
    if (!dev) {
        hrp.resize((size_t)n + 1);
        hcj.resize((size_t)nnz);
        hv.resize((size_t)nnz);
        for (int32_t q = 0; q < nsys; ++q) {
            const lair_csr &M = sys[q];
            if (M.rowptr[0] != 0 || M.rowptr[M.n] != M.nnz)
                fail(LAIR_EINVAL, "system %d: rowptr must run from 0 to nnz", q);
            for (int64_t i = 0; i < M.n; ++i) hrp[seg[q] + i] = (int32_t)(nzo[q] + M.rowptr[i]);
            for (int64_t p = 0; p < M.nnz; ++p) {
                int32_t c = M.col[p];
                if (c < 0 || c >= M.n) fail(LAIR_EINVAL, "system %d: column %d out of range", q, c);
                hcj[nzo[q] + p] = (int32_t)(c + seg[q]);
            }
            memcpy(hv.data() + nzo[q], M.val, sizeof(double) * M.nnz);
        }
        hrp[n] = (int32_t)nnz;
        U.rowptr = hrp.data();
        U.col = hcj.data();
        U.val = hv.data();
    } else {
        std::vector<SysCsr> hs((size_t)nsys);
        for (int32_t q = 0; q < nsys; ++q)
            hs[q] = SysCsr{sys[q].rowptr, sys[q].col, sys[q].val, sys[q].n, sys[q].nnz};
        DevArr<SysCsr> ds;
        DevArr<int64_t> dseg, dnzo;
        DevArr<int32_t> bad;
        ds.alloc((size_t)nsys, s);
        dseg.alloc((size_t)nsys + 1, s);
        dnzo.alloc((size_t)nsys + 1, s);
        bad.alloc(1, s);
        drp.alloc((size_t)n + 1, s);
        dcj.alloc((size_t)nnz, s);
        dv.alloc((size_t)nnz, s);
        LAIR_HIP(hipMemcpyAsync(ds.get(), hs.data(), sizeof(SysCsr) * nsys,
                                hipMemcpyHostToDevice, s));
        LAIR_HIP(hipMemcpyAsync(dseg.get(), seg.data(), sizeof(int64_t) * (nsys + 1),
                                hipMemcpyHostToDevice, s));
        LAIR_HIP(hipMemcpyAsync(dnzo.get(), nzo.data(), sizeof(int64_t) * (nsys + 1),
                                hipMemcpyHostToDevice, s));
        LAIR_HIP(hipMemsetAsync(bad.get(), 0, sizeof(int32_t), s));
        int64_t max_nnz = 0;
        for (int32_t q = 0; q < nsys; ++q) max_nnz = std::max(max_nnz, sys[q].nnz);
        launch_union_gather(nsys, ds.get(), dseg.get(), dnzo.get(), drp.get(), dcj.get(),
                            dv.get(), bad.get(), max_nnz, s);
        int32_t hb = 0;
        {
            Readback rb(s);
            rb.add(&hb, bad.get(), sizeof(int32_t));
            rb.run();
        }
        if (hb) fail(LAIR_EINVAL, "a system's rowptr does not run from 0 to nnz or a column "
                                  "lies outside its rows");
        U.rowptr = drp.get();
        U.col = dcj.get();
        U.val = dv.get();
        U.on_device = 1;
    }
    return setup_impl(&U, cfl, str, opt, s, &seg);
}

}  // namespace lair

// ===========================================================================
// C ABI
// ===========================================================================
using namespace lair;

template <class F>
static lair_status guarded(F &&f) {
    try {
        return f();
    } catch (const Error &e) {
        set_last_error(e.msg);
        return e.status;
    } catch (const std::bad_alloc &) {
        set_last_error("host allocation failed");
        return LAIR_ENOMEM;
    } catch (const std::exception &e) {
        set_last_error(e.what());
        return LAIR_EDEVICE;
    } catch (...) {
        set_last_error("unknown error");
        return LAIR_EDEVICE;
    }
}

extern "C" {

void lair_default_options(lair_strength *s, lair_options *o) {
    if (s) {
        s->theta = 0.25;
        s->theta_c = 0.25;
        s->kind = LAIR_SOC_ABS;
        s->distance = 1;
    }
    if (o) {
        o->interp = LAIR_P_ONE_POINT;
        o->precision = LAIR_FP64;
        o->omega = 1.0;
        o->max_levels = 25;
        o->max_coarse = 128;
        o->stall = 0.9;
        o->block_size = 0;
        o->flags = 0;
        o->lump_tol = 0.0;
    }
}

lair_status lair_setup(const lair_csr *A, const lair_cf_levels *cf,
                       const lair_strength *s, const lair_options *o,
                       void *stream, lair_hierarchy **out) {
    return guarded([&]() -> lair_status {
        if (!out) fail(LAIR_EINVAL, "out must not be NULL");
        *out = nullptr;
        *out = setup_impl(A, cf, s, o, (hipStream_t)stream);
        return LAIR_OK;
    });
}

lair_status lair_setup_batch(int32_t nsys, const lair_csr *A, const lair_cf_levels *cf,
                             const lair_strength *s, const lair_options *o, void *stream,
                             lair_hierarchy **out) {
    return guarded([&]() -> lair_status {
        if (!out) fail(LAIR_EINVAL, "out must not be NULL");
        *out = nullptr;
        *out = setup_batch_impl(nsys, A, cf, s, o, (hipStream_t)stream);
        return LAIR_OK;
    });
}

lair_status lair_solve_batch(lair_hierarchy *h, const double *b, double *x, double rtol,
                             int32_t maxit, int32_t *iters, double *relres, lair_info *info,
                             void *stream) {
    return guarded([&]() -> lair_status {
        return solve_batch_impl(h, b, x, rtol, maxit, iters, relres, info,
                                (hipStream_t)stream);
    });
}

int32_t lair_num_systems(const lair_hierarchy *h) { return h ? h->nsys : 0; }

lair_status lair_update_diag(lair_hierarchy *h, const double *diag, int32_t on_device,
                             void *stream) {
    return guarded([&]() -> lair_status {
        update_diag_impl(h, diag, on_device, (hipStream_t)stream);
        return LAIR_OK;
    });
}

lair_status lair_system_levels(const lair_hierarchy *h, int32_t *levels) {
    return guarded([&]() -> lair_status {
        if (!h || !levels) fail(LAIR_EINVAL, "hierarchy and levels must not be NULL");
        if (!h->batch) fail(LAIR_EINVAL, "the hierarchy was not built by lair_setup_batch");
        for (int32_t q = 0; q < h->nsys; ++q)
            levels[q] = h->nsys > 1 ? h->sys_levels[q] : (int32_t)h->L.size();
        return LAIR_OK;
    });
}

lair_status lair_set_local_buckets(const int32_t *edges) {
    return guarded([&]() -> lair_status {
        set_local_buckets(edges);
        return LAIR_OK;
    });
}

lair_status lair_local_buckets(const lair_hierarchy *h, int32_t level, int32_t *edges) {
    return guarded([&]() -> lair_status {
        if (!h || !edges) fail(LAIR_EINVAL, "hierarchy and edges must not be NULL");
        if (level < 0 || level + 1 >= (int32_t)h->L.size())
            fail(LAIR_EINVAL, "level %d has no local solves", level);
        for (int k = 0; k < 5; ++k) edges[k] = h->L[level]->buckets[k];
        return LAIR_OK;
    });
}

lair_status lair_cycle(lair_hierarchy *h, const double *b, double *x,
                       int32_t nrhs, void *stream) {
    return guarded([&]() -> lair_status {
        if (!h || !b || !x) fail(LAIR_EINVAL, "NULL argument");
        check_nrhs(h, nrhs);
        hipStream_t s = (hipStream_t)stream;
        ensure_vectors(h, nrhs, s);
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
        return LAIR_OK;
    });
}

lair_status lair_cycle_transpose(lair_hierarchy *h, const double *g, double *lam,
                                 int32_t nrhs, void *stream) {
    return guarded([&]() -> lair_status {
        if (!h || !g || !lam) fail(LAIR_EINVAL, "NULL argument");
        check_nrhs(h, nrhs);
        hipStream_t s = (hipStream_t)stream;
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
        return LAIR_OK;
    });
}

lair_status lair_solve(lair_hierarchy *h, const double *b, double *x, int32_t nrhs,
                       double rtol, int32_t maxit, lair_info *info, void *stream) {
    return guarded([&]() -> lair_status {
        return solve_impl(h, b, x, nrhs, rtol, maxit, info, (hipStream_t)stream, false);
    });
}

lair_status lair_solve_transpose(lair_hierarchy *h, const double *g, double *lam,
                                 int32_t nrhs, double rtol, int32_t maxit,
                                 lair_info *info, void *stream) {
    return guarded([&]() -> lair_status {
        if (h && scaled(h->opt))
            fail(LAIR_EUNSUPPORTED, "transposed solve with block scaling");
        if (h && nodal(h->opt))
            fail(LAIR_EUNSUPPORTED, "transposed solve on a nodal hierarchy");
        return solve_impl(h, g, lam, nrhs, rtol, maxit, info, (hipStream_t)stream, true);
    });
}

lair_status lair_solve_fgmres(lair_hierarchy *h, const double *b, double *x, int32_t nrhs,
                              double rtol, int32_t maxit, int32_t restart, lair_info *info,
                              void *stream) {
    return guarded([&]() -> lair_status {
        return solve_fgmres_impl(h, b, x, nrhs, rtol, maxit, restart, info,
                                 (hipStream_t)stream);
    });
}

int32_t lair_num_levels(const lair_hierarchy *h) { return h ? (int32_t)h->L.size() : 0; }

lair_status lair_level_stats_get(const lair_hierarchy *h, int32_t level,
                                 lair_level_stats *st) {
    return guarded([&]() -> lair_status {
        if (!h || !st) fail(LAIR_EINVAL, "NULL argument");
        if (level < 0 || level >= (int32_t)h->L.size()) fail(LAIR_EINVAL, "bad level %d", level);
        *st = h->L[level]->st;
        const Level &Lv = *h->L[level];
        if (Lv.nptr.get() && Lv.nc > 0) {
            std::vector<int32_t> hn((size_t)Lv.nc + 1);
            LAIR_HIP(hipStreamSynchronize(h->stream));
            LAIR_HIP(hipMemcpy(hn.data(), Lv.nptr.get(), sizeof(int32_t) * (Lv.nc + 1),
                               hipMemcpyDeviceToHost));
            int32_t smin = INT_MAX;
            for (int32_t c = 0; c < Lv.nc; ++c) smin = std::min(smin, hn[c + 1] - hn[c]);
            st->s_min = smin;
        } else {
            st->s_min = 0;
        }
        return LAIR_OK;
    });
}

lair_status lair_export(const lair_hierarchy *h, int32_t level, int32_t what,
                        void *host_buf, int64_t *bytes) {
    return guarded([&]() -> lair_status {
        if (!h || !bytes) fail(LAIR_EINVAL, "NULL argument");
        if (level < 0 || level >= (int32_t)h->L.size()) fail(LAIR_EINVAL, "bad level %d", level);
        const Level &Lv = *h->L[level];
        const void *src = nullptr;
        int64_t nb = 0;
        switch (what) {
            case 0: src = Lv.A.rp.get(); nb = 4 * ((int64_t)Lv.n + 1); break;
            case 1: src = Lv.A.cj.get(); nb = 4 * Lv.A.nnz; break;
            case 2: src = Lv.A.v.get(); nb = 8 * Lv.A.nnz; break;
            case 3: src = Lv.cf.get(); nb = Lv.cf.get() ? Lv.n : 0; break;
            case 4: src = Lv.smask.get(); nb = Lv.smask.get() ? Lv.A.nnz : 0; break;
            case 5: src = Lv.R.rp.get(); nb = Lv.R.rp.get() ? 4 * ((int64_t)Lv.nc + 1) : 0; break;
            case 6: src = Lv.R.cj.get(); nb = 4 * Lv.R.nnz; break;
            case 7: src = Lv.R.v.get(); nb = 8 * Lv.R.nnz; break;
            case 8: src = Lv.P.rp.get(); nb = Lv.P.rp.get() ? 4 * ((int64_t)Lv.n + 1) : 0; break;
            case 9: src = Lv.P.cj.get(); nb = 4 * Lv.P.nnz; break;
            case 10: src = Lv.P.v.get(); nb = 8 * Lv.P.nnz; break;
            case 11: src = Lv.nptr.get(); nb = Lv.nptr.get() ? 4 * ((int64_t)Lv.nc + 1) : 0; break;
            case 12: src = Lv.nbr.get(); nb = Lv.nptr.get() ? 4 * (Lv.R.nnz - Lv.nc) : 0; break;
            case 13: src = Lv.flags.get(); nb = Lv.flags.get() ? Lv.nc : 0; break;
            default: fail(LAIR_EINVAL, "unknown export selector %d", what);
        }
        int64_t cap = *bytes;
        *bytes = nb;
        if (!host_buf) return LAIR_OK;
        if (cap < nb) fail(LAIR_EINVAL, "export buffer too small (%lld < %lld)",
                           (long long)cap, (long long)nb);
        if (nb > 0) {
            LAIR_HIP(hipStreamSynchronize(h->stream));
            LAIR_HIP(hipMemcpy(host_buf, src, (size_t)nb, hipMemcpyDeviceToHost));
        }
        return LAIR_OK;
    });
}

void lair_free(lair_hierarchy *h) {
    if (!h) return;
    try {
        // the memory goes back to the allocator's cache: wait for every
        // launch that may still read it
        (void)hipDeviceSynchronize();
        delete h;
    } catch (...) {
    }
}

void lair_trim(void) { dev_trim(); }

const char *lair_status_string(lair_status s) {
    switch (s) {
        case LAIR_OK: return "LAIR_OK";
        case LAIR_EINVAL: return "LAIR_EINVAL: invalid argument";
        case LAIR_ENOMEM: return "LAIR_ENOMEM: out of memory";
        case LAIR_EDEVICE: return "LAIR_EDEVICE: HIP device error";
        case LAIR_ESINGULAR: return "LAIR_ESINGULAR: singular coarsest matrix";
        case LAIR_ENOCONV: return "LAIR_ENOCONV: tolerance not reached";
        case LAIR_EUNSUPPORTED: return "LAIR_EUNSUPPORTED: size limit exceeded";
        default: return "unknown status";
    }
}

const char *lair_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
