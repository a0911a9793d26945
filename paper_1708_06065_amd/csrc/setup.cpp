// liblair setup: the level loop (strength, splitting, neighbourhoods, local
// solves, interpolation, Galerkin product, lumping), the coarsest level, the
// cycle's renumbered operators, a batch's union and a new diagonal on a kept
// hierarchy.  Every arithmetic step runs in the HIP kernels of k_setup.hip,
// k_batch.hip, k_nodal.hip and k_split.hip; the host only sizes buffers,
// launches, and (for the classical CF splitting, a sequential greedy
// algorithm) runs rs_first_pass on a host copy of the strength mask.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <climits>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <functional>
#include <memory>
#include <string>
#include <vector>

#include "hierarchy.hpp"

namespace lair {

__global__ void k_nonneg_flag(int32_t n, const int32_t *pc, int32_t *hs) {
    int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) hs[i] = pc[i] >= 0 ? 1 : 0;
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
    int64_t *dp = nullptr;           // three zeroed slots: [0] nnz, [1] longest row, [2] flag
    int64_t h[3] = {0, 0, 0};
    int64_t *nnz = nullptr;          // where the sizes go (null: nothing pending)
    int32_t *max_row = nullptr;
    const char *what = "";
    void arm(DevCSR *mat, const char *w, hipStream_t s) {
        arm_at(zeroed_slots(3, s), mat, w);
    }
    // slots already zeroed in stream order (no memset here)
    void arm_at(int64_t *slots, DevCSR *mat, const char *w) {
        arm_sizes(slots, &mat->nnz, &mat->max_row, w);
    }
    void arm_sizes(int64_t *slots, int64_t *n, int32_t *mx, const char *w) {
        dp = slots;
        nnz = n;
        max_row = mx;
        what = w;
    }
    int64_t *tot() { return dp; }
    int32_t *flag() { return reinterpret_cast<int32_t *>(dp + 2); }
    // a profiled launch whose algorithmic bytes include 12 per entry of the
    // matrix whose size is pending (set when the size arrives)
    int prof_slot = -1;
    double prof_base = 0.0;
    void add(Readback &rb) {
        if (nnz) rb.add(h, dp, sizeof(h));
    }
    // after the readback that carried them
    void apply() {
        if (!nnz) return;
        int64_t *n = nnz;
        nnz = nullptr;
        if ((int32_t)h[2]) fail(LAIR_EUNSUPPORTED, "%s", what);
        *n = h[0];
        *max_row = (int32_t)h[1];
        if (prof_slot >= 0) prof_set_bytes(prof_slot, prof_base + 12.0 * (double)h[0]);
        prof_slot = -1;
    }
    void settle(hipStream_t s) {
        if (!nnz) return;
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
// The right factor of a product: a CSR matrix, or the rows an earlier
// product left staged (at their product offsets, with their lengths).
struct StagedB {
    DevArr<int64_t> off;
    DevArr<int32_t> len, cj;
    DevArr<double> v;
    int32_t nrows = 0, ncols = 0;
    int64_t nnz = 0;                 // distinct entries (once read back)
    int32_t max_row = -1;
};
struct BSrc {
    BRows rows;
    const int32_t *cj = nullptr;
    const double *v = nullptr;
    int32_t nrows = 0, ncols = 0;
    int64_t nnz = 0;
    static BSrc of(const DevCSR &B) {
        BSrc b;
        b.rows.rp = B.rp.get();
        b.cj = B.cj.get();
        b.v = B.v.get();
        b.nrows = B.nrows;
        b.ncols = B.ncols;
        b.nnz = B.nnz;
        return b;
    }
    static BSrc of(const StagedB &B) {
        BSrc b;
        b.rows.off = B.off.get();
        b.rows.len = B.len.get();
        b.cj = B.cj.get();
        b.v = B.v.get();
        b.nrows = B.nrows;
        b.ncols = B.ncols;
        b.nnz = B.nnz;
        return b;
    }
};

struct SpgemmState {
    int32_t m = 0;
    DevArr<int32_t> cnt;
    DevArr<int64_t> eoff, tot;       // tot: [0] products, [1] most in a row
    // ctl: five zeroed int64 slots: [0..2] C's sizes (or [2] the overflow
    // flag), then the product's four retry-list counters (int32); lists:
    // the retry lists
    int64_t *ctl_ = nullptr;
    DevArr<int32_t> lists_;
    int64_t *ctl() { return ctl_; }
    int32_t *counts() { return reinterpret_cast<int32_t *>(ctl_ + 3); }
    int32_t *lists() { return lists_.get(); }
    int64_t h[2] = {0, 0};
};

// The counters the product needs zeroed are cleared here, while earlier
// work still runs, rather than after the readback that spgemm_finish waits
// for.
static void spgemm_count(const DevCSR &A, const BSrc &B, SpgemmState &st, hipStream_t s,
                         DevArr<int64_t> &tmp) {
    const int32_t m = A.nrows;
    st.m = m;
    st.cnt.alloc((size_t)m + 1, s);
    st.eoff.alloc((size_t)m + 1, s);
    st.ctl_ = zeroed_slots(5, s);
    st.lists_.alloc(3 * (size_t)std::max(m, 1), s);
    st.tot.alloc(2, s);
    // products per row: A's indices and B's row pointers
    ProfScope ps("spgemm_count", s, 4.0 * A.nnz + 4.0 * (A.nrows + 1) +
                                        8.0 * (B.nrows + 1) + 12.0 * m);
    launch_prod_count(m, A.rp.get(), A.cj.get(), B.rows, st.cnt.get(), s);
    scan_counts_i64_to(st.cnt.get(), st.eoff.get(), m, s, tmp, st.tot.get());
}

// st.h must hold the readback of st.tot.  Returns C's longest row (0 when
// deferred).
// ratio: products per distinct column expected for C's rows (from a
// similar product; 0 when unknown), which sizes the hash tables.
// lump_tol > 0 (not deferred): C is written lumped (Sec. 3.3) straight from
// the staged rows, in place of the plain compaction.
// *distinct receives the size C has before lumping.
// The hash pass of C = A B: C's rows sorted at their product offsets in the
// staging arrays tcj, tcx (sized here by st.h), their lengths in st.cnt.
// *slot / *base: the profiler slot of the pass and its algorithmic bytes
// before C's entries (12 per distinct entry written, added by the caller
// once the number is known).
static void spgemm_hash(const DevCSR &A, const BSrc &B, SpgemmState &st, hipStream_t s,
                        double ratio, DevArr<int32_t> &tcj, DevArr<double> &tcx,
                        int *slot = nullptr, double *base = nullptr) {
    const int32_t m = st.m;
    const int64_t etot = st.h[0], emax = st.h[1];
    if (etot > INT32_MAX)
        fail(LAIR_EUNSUPPORTED, "sparse product with more than 2^31 terms (%lld)", (long long)etot);
    int32_t *ovp = reinterpret_cast<int32_t *>(st.ctl() + 2);
    tcj.alloc((size_t)std::max<int64_t>(etot, 1), s);
    tcx.alloc((size_t)std::max<int64_t>(etot, 1), s);
    // A, the rows of B and the rows of C each touched once
    const double bytes = 12.0 * (A.nnz + B.nnz) + 4.0 * (A.nrows + 1) + 4.0 * (B.nrows + 1);
    ProfScope ps("spgemm_fill", s, bytes);
    if (slot) *slot = ps.slot;
    if (base) *base = bytes;
    const double mean_e = m ? (double)etot / m : 0.0;
    launch_spgemm(m, A.rp.get(), A.cj.get(), A.v.get(), B.rows, B.cj, B.v, st.eoff.get(),
                  emax, mean_e, ratio > 1.0 ? mean_e / ratio : 0.0, st.cnt.get(), tcj.get(),
                  tcx.get(), st.counts(), st.lists(), ovp, s);
}

// C = A B left staged for a following product (no compaction): its sizes
// (distinct entries, longest row, the overflow flag) wait in `pend` for a
// later readback.
static void spgemm_to_staged(const DevCSR &A, const BSrc &B, StagedB &C, SpgemmState &st,
                             hipStream_t s, DevArr<int64_t> &tmp, PendingSizes &pend,
                             double ratio) {
    DevArr<int32_t> tcj;
    DevArr<double> tcx;
    int slot = -1;
    double base = 0.0;
    spgemm_hash(A, B, st, s, ratio, tcj, tcx, &slot, &base);
    C.nrows = st.m;
    C.ncols = B.ncols;
    C.nnz = st.h[0];                 // an upper bound until the sizes arrive
    // the totals of the lengths (a scratch scan)
    DevArr<int32_t> rp;
    rp.alloc((size_t)st.m + 1, s);
    pend.arm_sizes(st.ctl(), &C.nnz, &C.max_row, "sparse product row with more than 1024 terms");
    pend.prof_slot = slot;
    pend.prof_base = base;
    scan_counts_i32_to(st.cnt.get(), rp.get(), st.m, s, tmp, pend.tot());
    C.off = std::move(st.eoff);
    C.len = std::move(st.cnt);
    C.cj = std::move(tcj);
    C.v = std::move(tcx);
}

static int32_t spgemm_finish(const DevCSR &A, const BSrc &B, DevCSR &C, SpgemmState &st,
                             hipStream_t s, DevArr<int64_t> &tmp, PendingSizes *defer,
                             double ratio = 0.0, double lump_tol = 0.0,
                             int64_t *distinct = nullptr, const int8_t *whole_rows = nullptr) {
    const int32_t m = st.m;
    const int64_t etot = st.h[0];
    C.nrows = m;
    C.ncols = B.ncols;
    int32_t *ovp = reinterpret_cast<int32_t *>(st.ctl() + 2);
    if (defer) defer->arm_at(st.ctl(), &C, "sparse product row with more than 1024 terms");
    DevArr<int32_t> tcj;
    DevArr<double> tcx;
    int fill_slot = -1;
    double fill_base = 0.0;
    spgemm_hash(A, B, st, s, ratio, tcj, tcx, &fill_slot, &fill_base);
    if (defer) {
        defer->prof_slot = fill_slot;
        defer->prof_base = fill_base;
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
        prof_set_bytes(fill_slot, fill_base + 12.0 * ht[2]);
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
        prof_set_bytes(fill_slot, fill_base + 12.0 * C.nnz);
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
    spgemm_count(A, BSrc::of(B), st, s, tmp);
    {
        Readback rb(s);
        rb.add(st.h, st.tot.get(), sizeof(st.h));
        rb.run();
    }
    return spgemm_finish(A, BSrc::of(B), C, st, s, tmp, nullptr,
                         c_nnz > 0 ? (double)st.h[0] / (double)c_nnz : 0.0);
}

void transpose(const DevCSR &M, DevCSR &T, hipStream_t s, DevArr<int64_t> &tmp) {
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

void check_options(const lair_strength *s, const lair_options *o) {
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
        if (!node_check(n, kb, A.rp.get(), A.cj.get(), A.nnz, s))
            fail(LAIR_EINVAL, "level %d: the nodal treatment needs the k rows of a node to store "
                 "the same whole dense blocks", lvl);
    }
    Lv.smask.alloc((size_t)std::max<int64_t>(A.nnz, 1), s);
    Lv.cf.alloc((size_t)n, s);
    const bool given = cfl && lvl < cfl->nlevels;
    if (given) {
        int64_t lo = cfl->offs[lvl], hi = cfl->offs[lvl + 1];
        if (hi - lo != n)
            fail(LAIR_EINVAL, "CF splitting of level %d has %lld entries, level size is %d",
                 lvl, (long long)(hi - lo), n);
        // the splittings were uploaded (and checked) at the start of setup
        LAIR_HIP(hipMemcpyAsync(Lv.cf.get(), h->cf_dev.get() + lo, (size_t)n,
                                hipMemcpyDeviceToDevice, s));
    }
    // a given splitting of one system (not changed after the strength) lets
    // the strength pass also take the counting pass of direct interpolation
    const bool strength_interp = given && !nod && h->nsys == 1 &&
                                 h->opt.interp == LAIR_P_DIRECT;
    DevArr<int32_t> pc_early;
    DevArr<double> coef_early;
    if (nod) {
        launch_node_strength(n, kb, A.rp.get(), A.cj.get(), A.v.get(), A.nnz, h->str.theta,
                             Lv.smask.get(), s);
    } else if (strength_interp) {
        pc_early.alloc((size_t)n, s);
        coef_early.alloc(3 * (size_t)std::max(n, 1), s);
        launch_strength_interp(n, A.rp.get(), A.cj.get(), A.v.get(), h->str.theta,
                               h->str.kind, Lv.cf.get(), Lv.smask.get(), pc_early.get(),
                               coef_early.get(), mean, s);
    } else {
        launch_strength(n, A.rp.get(), A.cj.get(), A.v.get(), h->str.theta, h->str.kind,
                        Lv.smask.get(), mean, s);
    }
    if (given) {
        // copied above, before the strength pass
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
        // (timed from the moment the device has produced the mask)
        LAIR_HIP(hipStreamSynchronize(s));
        const auto t_split = Clock::now();
        const uint8_t *sm_dev = Lv.smask.get();
        DevArr<uint8_t> smc;
        if (h->str.theta_c != h->str.theta) {
            smc.alloc((size_t)std::max<int64_t>(A.nnz, 1), s);
            if (nod)
                launch_node_strength(n, kb, A.rp.get(), A.cj.get(), A.v.get(), A.nnz,
                                     h->str.theta_c, smc.get(), s);
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
        h->split_ms += ms_since(t_split);
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
    // the neighbourhoods' overflow flag
    struct { int32_t *p; int32_t *get() const { return p; } } over{
        reinterpret_cast<int32_t *>(zeroed_slots(1, s))};
    int64_t nc = 0;
    // a caller's splitting gives the count of C-points on the host: the
    // entries of the F and C rows (for the cycle's accounting) then wait on
    // the device until the end of the setup instead of a wait here
    const bool nc_known = h->nsys == 1 && cfl && lvl < cfl->nlevels;
    {
        DevArr<unsigned long long> acc;
        acc.alloc(2 + 2 * (size_t)blocks_for(n, 256), s);
        ProfScope ps("cf_lists", s, 13.0 * n + 4.0 * n);
        launch_cf_lists(n, Lv.cf.get(), scan.get(), A.rp.get(), Lv.cidx.get(), Lv.clist.get(),
                        Lv.flist.get(), acc.get(), s);
        if (nc_known) {
            nc = h->cf_count[(size_t)lvl];
            Lv.nnzF = Lv.nnzC = -1;
            Lv.fc_acc = std::move(acc);
        } else {
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
    }
    h->phase_mark(1);
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
    // nodal levels: the rows of a C-node share one neighbourhood, merged once
    const int32_t knbr = nodal(h->opt) ? h->opt.block_size : 1;
    launch_neighbourhoods(Lv.nc, n, Lv.clist.get(), A.rp.get(), A.cj.get(), Lv.smask.get(),
                          Lv.cf.get(), h->str.distance, Lv.flist.get(), Lv.nf, cnt.get(),
                          nullptr, nullptr, over.get(), Lv.max_row, s, knbr);
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
        // N_i holds at most the entries of row i but its diagonal
        nn = std::max<int64_t>(0, (Lv.nnzC >= 0 ? Lv.nnzC : A.nnz) - Lv.nc);
        smax64 = Lv.max_row - 1;
    } else {
        int32_t ov = 0;
        nn = scan_counts_i32(cnt.get(), Lv.nptr.get(), Lv.nc, s, tmp, &smax64, over.get(), &ov);
        if (ov) fail(LAIR_EUNSUPPORTED, "level %d: a distance-2 neighbourhood merges more than 256 rows", lvl);
    }
    Lv.nbr.alloc((size_t)std::max<int64_t>(nn, 1), s);
    launch_neighbourhoods(Lv.nc, n, Lv.clist.get(), A.rp.get(), A.cj.get(), Lv.smask.get(),
                          Lv.cf.get(), h->str.distance, Lv.flist.get(), Lv.nf, nullptr,
                          Lv.nptr.get(), Lv.nbr.get(), over.get(), Lv.max_row, s, knbr);
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
                launch_interp_1p_node(n, kb, A.rp.get(), A.cj.get(), A.v.get(), A.nnz,
                                      Lv.smask.get(), Lv.cf.get(), Lv.cidx.get(), pcol.get(), s);
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
        DevArr<double> coef;
        if (strength_interp) {
            // counted by the strength pass
            pc = std::move(pc_early);
            coef = std::move(coef_early);
        } else {
            pc.alloc((size_t)n, s);
            coef.alloc(3 * (size_t)std::max(n, 1), s);
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
    spgemm_count(A, BSrc::of(P), ap, s, tmp);
    Readback rb(s);
    p_pend.add(rb);
    rb.add(ap.h, ap.tot.get(), sizeof(ap.h));
    int64_t hnt[2] = {nn, smax64};
    if (defer_nbr) rb.add(hnt, ntot.get(), sizeof(hnt));

    Lv.flags.alloc((size_t)Lv.nc, s);
    LocalSolveOut out{R.rp.get(), R.cj.get(), R.v.get(), Lv.flags.get()};
    const int32_t lprec = h->opt.precision == LAIR_FP64 ? LAIR_FP64 : LAIR_MIXED;
    // nodal: the k rows of a C-node share N, one factorisation per node
    // (LAIR_NODAL_ROW_SOLVES=1 solves every row on its own instead, the
    // same numbers; for checks)
    const int32_t knode = nod && node_solves_fit(kb, Lv.st.s_max, lprec) &&
                                  !env_flag("LAIR_NODAL_ROW_SOLVES") ? kb : 1;
    int64_t nsing = local_solves(Lv.nc, Lv.clist.get(), Lv.nptr.get(), Lv.nbr.get(),
                                 A.rp.get(), A.cj.get(), A.v.get(), lprec,
                                 Lv.st.s_max, n ? (double)A.nnz / n : 0.0, out, s,
                                 Lv.buckets, &rb, knode);
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
    h->coarse_entries = (double)doff[ns];
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
    h->coarse_entries = (double)n * (double)n;
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
    // the F/C row entries left on the device, in one readback
    {
        std::vector<unsigned long long> v(2 * h->L.size(), 0);
        Readback rb(h->stream);
        bool any = false;
        for (size_t l = 0; l < h->L.size(); ++l)
            if (h->L[l]->fc_acc.get()) {
                rb.add(&v[2 * l], h->L[l]->fc_acc.get(), 2 * sizeof(unsigned long long));
                any = true;
            }
        if (any) rb.run();
        for (size_t l = 0; l < h->L.size(); ++l)
            if (h->L[l]->fc_acc.get()) {
                h->L[l]->nnzF = (int64_t)v[2 * l];
                h->L[l]->nnzC = (int64_t)v[2 * l + 1];
                h->L[l]->fc_acc.release();
            }
    }
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
    // the coarsest dense solve(s): one per system of a batch
    flops += 2.0 * h->coarse_entries;
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

// The work level by level: whether level l is renumbered (decide, once the
// level is known not to be the coarsest), its permutation and its copy of A
// (once its splitting exists), and its copies of R and P (once the next
// level is decided and permuted).
struct SplitCopies {
    lair_hierarchy *h;
    hipStream_t s;
    bool mixed, allowed, all;
    DevArr<int64_t> tmp;
    SplitCopies(lair_hierarchy *h_, hipStream_t s_) : h(h_), s(s_) {
        mixed = h->opt.precision == LAIR_MIXED;
        allowed = h->nsys == 1 && !(h->opt.flags & LAIR_FLAG_NATURAL_ORDER) && !nodal(h->opt);
        all = (h->opt.flags & LAIR_FLAG_SPLIT_ALL) != 0;
    }
    // renumbered levels form a prefix of the hierarchy, the coarsest excluded
    void decide(size_t l, bool coarsest) {
        Level &Lv = *h->L[l];
        const bool prev = l == 0 ? allowed : h->L[l - 1]->split;
        Lv.split = prev && !coarsest && (all || Lv.n >= SPLIT_MIN_ROWS);
    }
    void perm(size_t l) {
        Level &Lv = *h->L[l];
        if (!Lv.split) return;
        const size_t n = (size_t)std::max(Lv.n, 1);
        Lv.perm.alloc(n, s);
        Lv.iperm.alloc(n, s);
        Lv.ids.alloc(n, s);
        Lv.cf_split.alloc(n, s);
        launch_split_perm(Lv.nf, Lv.nc, Lv.flist.get(), Lv.clist.get(), Lv.perm.get(),
                          Lv.iperm.get(), Lv.ids.get(), Lv.cf_split.get(), s);
    }
    void copy(const DevCSR &M, DevCSR &O, const int32_t *rowmap, const int32_t *irowmap,
              const int32_t *colmap, DevArr<int32_t> *cjt, int32_t nsplit) {
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
                           irowmap, colmap, M.rp.get(), M.cj.get(), M.v.get(), O.rp.get(),
                           O.cj.get(),
                           mixed ? nullptr : O.v.get(), mixed ? O.v32.get() : nullptr,
                           cjt ? cjt->get() : nullptr, nsplit, tmp, s);
    }
    static void drop(DevCSR &O) {
        O.rp.release(); O.cj.release(); O.v.release(); O.v32.release();
        O.nrows = O.ncols = 0; O.nnz = 0;
    }
    void copy_A(size_t l) {
        Level &Lv = *h->L[l];
        if (Lv.split) {
            copy(Lv.A, Lv.As, Lv.perm.get(), Lv.iperm.get(), Lv.iperm.get(), &Lv.cjt_split,
                 Lv.nf);
        } else {
            drop(Lv.As);
            Lv.cjt_split.release();
        }
    }
    void copy_RP(size_t l) {
        Level &Lv = *h->L[l];
        Level &Nx = *h->L[l + 1];
        if (Lv.split || Nx.split) {
            const int32_t *perm = Lv.split ? Lv.perm.get() : nullptr;
            const int32_t *iperm = Lv.split ? Lv.iperm.get() : nullptr;
            const int32_t *nperm = Nx.split ? Nx.perm.get() : nullptr;
            const int32_t *niperm = Nx.split ? Nx.iperm.get() : nullptr;
            copy(Lv.R, Lv.Rs, nperm, niperm, iperm, nullptr, 0);
            copy(Lv.P, Lv.Ps, perm, iperm, niperm, nullptr, 0);
        } else {
            drop(Lv.Rs);
            drop(Lv.Ps);
        }
    }
};

// Every level at once (a hierarchy whose values have changed).
static void build_split(lair_hierarchy *h, hipStream_t s) {
    const size_t nL = h->L.size();
    SplitCopies sc(h, s);
    for (size_t l = 0; l < nL; ++l) sc.decide(l, l + 1 == nL);
    for (size_t l = 0; l + 1 < nL; ++l) sc.perm(l);
    for (size_t l = 0; l + 1 < nL; ++l) {
        sc.copy_A(l);
        sc.copy_RP(l);
    }
}

// After the values of a hierarchy are set: split-ordered copies, the tagged
// columns and float values of whatever the cycle reads in the natural
// ordering.
static void finish_cycle_operators(lair_hierarchy *h, hipStream_t s, bool split_built = false) {
    if (!split_built) build_split(h, s);
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
            launch_node_scale(Lv.n, k, Lv.A.rp.get(), Lv.A.v.get(), Lv.A.nnz, Lv.ndinv.get(),
                              Lv.av.get(), s);
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
lair_hierarchy *setup_impl(const lair_csr *Ain, const lair_cf_levels *cfl,
                           const lair_strength *str, const lair_options *opt,
                           hipStream_t s, const std::vector<int64_t> *seg) {
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
    h->phase_t0 = t0;
    zeroed_slots_reserve(4096, s);
    DevArr<int64_t> tmp;

    const int32_t n = (int32_t)Ain->n;
    const int64_t nnz = Ain->nnz;
    if (cfl && cfl->nlevels > 0) {
        // check the caller's splittings and upload them in one pinned copy
        int64_t total = cfl->offs[cfl->nlevels];
        if (cfl->offs[0] != 0 || total < 0) fail(LAIR_EINVAL, "bad CF level offsets");
        for (int32_t l = 0; l < cfl->nlevels; ++l)
            if (cfl->offs[l + 1] < cfl->offs[l]) fail(LAIR_EINVAL, "bad CF level offsets");
        h->cf_count.assign((size_t)cfl->nlevels, 0);
        if (cfl->on_device) {
            // copied, checked and counted on the device; one readback
            const int32_t nl = cfl->nlevels;
            h->cf_dev.alloc((size_t)std::max<int64_t>(total, 1), s);
            if (total > 0)
                LAIR_HIP(hipMemcpyAsync(h->cf_dev.get(), cfl->cf, (size_t)total,
                                        hipMemcpyDeviceToDevice, s));
            int64_t *stage = (int64_t *)pinned_upload(sizeof(int64_t) * (nl + 1));
            memcpy(stage, cfl->offs, sizeof(int64_t) * (nl + 1));
            DevArr<int64_t> doffs;
            doffs.alloc((size_t)nl + 1, s);
            LAIR_HIP(hipMemcpyAsync(doffs.get(), stage, sizeof(int64_t) * (nl + 1),
                                    hipMemcpyHostToDevice, s));
            int64_t *cnt = zeroed_slots((size_t)nl + 1, s);
            int32_t *badp = reinterpret_cast<int32_t *>(cnt + nl);
            launch_cf_check(nl, doffs.get(), total, h->cf_dev.get(),
                            nodal(*opt) ? opt->block_size : 1, cnt, badp, s);
            std::vector<int64_t> hc((size_t)nl + 1, 0);
            {
                Readback rb(s);
                rb.add(hc.data(), cnt, sizeof(int64_t) * (nl + 1));
                rb.run();
            }
            if ((int32_t)hc[(size_t)nl])
                fail(LAIR_EINVAL, nodal(*opt) ? "a CF splitting holds a value other than 0/1 "
                                                "or splits a node"
                                              : "a CF splitting holds a value other than 0/1");
            for (int32_t l = 0; l < nl; ++l) h->cf_count[(size_t)l] = hc[(size_t)l];
        }
        uint8_t bad = 0;
        const uint8_t *cfb = (const uint8_t *)cfl->cf;
        if (!cfl->on_device) {
            for (int32_t l = 0; l < cfl->nlevels; ++l) {
                int64_t c = 0;
                for (int64_t k = cfl->offs[l]; k < cfl->offs[l + 1]; ++k) {
                    bad |= cfb[k] & 0xFE;
                    c += cfb[k] & 1;
                }
                h->cf_count[(size_t)l] = c;
            }
        }
        if (bad) fail(LAIR_EINVAL, "a CF splitting holds a value other than 0/1");
        if (total > 0 && !cfl->on_device) {
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

    if (nodal(*opt) && cfl && cfl->nlevels > 0 && !cfl->on_device) {
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
    // The split-ordered copies of a level wait in a queue once their inputs
    // exist; every readback of the levels below takes one item and queues its
    // kernels behind the readback, so the device copies while the host waits
    // for the sizes (not while profiling: the profiler times categories
    // launch by launch).
    SplitCopies sc(h.get(), s);
    std::deque<std::function<void()>> fillq;
    const std::function<void()> fill = [&fillq]() {
        if (fillq.empty()) return;
        std::function<void()> f = std::move(fillq.front());
        fillq.pop_front();
        f();
    };
    struct FillGuard {
        const std::function<void()> *prev;
        ~FillGuard() { set_readback_fill(prev); }
    } fill_guard{set_readback_fill(prof_active() ? nullptr : &fill)};
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
        h->phase_mark(lvl == 0 ? 0 : 3);
        build_level_transfer(h.get(), Lv, lvl, cfl, coarsest, tmp, ap_st);
        h->phase_mark(2);
        if (coarsest) break;
        // level lvl is not the coarsest: its permutation and copy of A, then
        // the copies of the transfer operators of the level above it
        sc.decide((size_t)lvl, false);
        fillq.push_back([&sc, lvl] {
            sc.perm((size_t)lvl);
            sc.copy_A((size_t)lvl);
        });
        if (lvl > 0) fillq.push_back([&sc, lvl] { sc.copy_RP((size_t)lvl - 1); });
        // Galerkin product K = R (A P): the sizes of A P reach the host with
        // the count of products of R (A P)
        // A P stays in the product's staging arrays (rows at their product
        // offsets): R (A P) reads it there, so it is never compacted
        StagedB AP;
        PendingSizes ap_pend;
        spgemm_to_staged(Lv.A, BSrc::of(Lv.P), AP, ap_st, s, tmp, ap_pend, ap_ratio);
        if (setup_sizes_eager()) ap_pend.settle(s);
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
        spgemm_count(Lv.R, BSrc::of(AP), k_st, s, tmp);
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
        nx->max_row = spgemm_finish(Lv.R, BSrc::of(AP), nx->A, k_st, s, tmp, nullptr, k_ratio,
                                    opt->lump_tol, &k_distinct, whole.get());
        if (k_distinct < 0) k_distinct = nx->A.nnz;
        if (k_distinct > 0) k_ratio = (double)k_st.h[0] / (double)k_distinct;
        h->L.push_back(std::move(nx));
    }
    h->phase_mark(h->L.size() == 1 ? 0 : 3);
    finish_coarsest(h.get());
    // what the readbacks have not taken
    set_readback_fill(fill_guard.prev);
    while (!fillq.empty()) fill();
    {
        const size_t nL = h->L.size();
        sc.decide(nL - 1, true);
        if (nL >= 2) sc.copy_RP(nL - 2);
    }
    h->phase_mark(4);
    for (auto &lp : h->L) {
        Level &Lv = *lp;
        Lv.team_A = team_of(Lv.A);
        Lv.team_R = team_of(Lv.R);
        Lv.team_P = team_of(Lv.P);
    }
    finish_cycle_operators(h.get(), s, true);
    level_stats_and_cc(h.get());
    LAIR_HIP(hipStreamSynchronize(s));
    h->phase_mark(5);
    h->setup_ms = ms_since(t0);
    return h.release();
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

void update_diag_impl(lair_hierarchy *h, const double *diag, int32_t on_device,
                      hipStream_t s) {
    if (!h || !diag) fail(LAIR_EINVAL, "hierarchy and diag must not be NULL");
    if (scaled(h->opt))
        fail(LAIR_EUNSUPPORTED, "a new diagonal changes the block scaling: set up again");
    if (nodal(h->opt))
        fail(LAIR_EUNSUPPORTED, "a new diagonal on a nodal hierarchy: set up again");
    if (h->opt.lump_tol > 0.0)
        fail(LAIR_EUNSUPPORTED, "lumped coarse patterns depend on the values: set up again");
    h->stream = s;
    zeroed_slots_reserve(4096, s);
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
lair_hierarchy *setup_batch_impl(int32_t nsys, const lair_csr *sys,
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
