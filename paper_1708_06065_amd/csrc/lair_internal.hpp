// Internal declarations shared by the liblair translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <stdexcept>
#include <string>
#include <utility>
#include <vector>

#include "../../include/lair.h"

namespace lair {

// ---------------------------------------------------------------------------
// Errors: thrown inside the library, turned into a status at the ABI.
// ---------------------------------------------------------------------------
struct Error {
    lair_status status;
    std::string msg;
};

[[noreturn]] void fail(lair_status st, const char *fmt, ...);
void set_last_error(const std::string &m);

#define LAIR_HIP(call)                                                         \
    do {                                                                       \
        hipError_t e_ = (call);                                                \
        if (e_ != hipSuccess)                                                  \
            ::lair::fail(e_ == hipErrorOutOfMemory ? LAIR_ENOMEM : LAIR_EDEVICE,\
                         "%s failed: %s (%s:%d)", #call, hipGetErrorString(e_),\
                         __FILE__, __LINE__);                                  \
    } while (0)

#define LAIR_LAUNCH_CHECK() LAIR_HIP(hipGetLastError())

// ---------------------------------------------------------------------------
// Stream-ordered device array, freed on the stream it was allocated on.
// ---------------------------------------------------------------------------
// Caching device allocator (alloc.cpp): blocks released on a stream are
// reused by later requests on the same stream.
void *dev_alloc(size_t bytes, hipStream_t s);
void dev_free(void *p, hipStream_t s) noexcept;
void dev_trim() noexcept;
size_t dev_cached_bytes() noexcept;
size_t dev_in_use_bytes() noexcept;
// `count` int64 slots of device memory that are zero in stream order on s,
// each handed out once (flags, sizes and counters of the setup); reserve at
// the start of a call so that its slots come from one cleared block.
int64_t *zeroed_slots(size_t count, hipStream_t s);
void zeroed_slots_reserve(size_t count, hipStream_t s);

template <class T>
struct DevArr {
    T *p = nullptr;
    size_t n = 0;
    hipStream_t s = nullptr;
    bool own = true;       // false: a view of memory the array does not free

    DevArr() = default;
    DevArr(const DevArr &) = delete;
    DevArr &operator=(const DevArr &) = delete;
    DevArr(DevArr &&o) noexcept { swap(o); }
    DevArr &operator=(DevArr &&o) noexcept {
        if (this != &o) { release(); swap(o); }
        return *this;
    }
    ~DevArr() { release(); }

    void swap(DevArr &o) noexcept {
        std::swap(p, o.p);
        std::swap(n, o.n);
        std::swap(s, o.s);
        std::swap(own, o.own);
    }
    void release() noexcept {
        if (p && own) dev_free(p, s);
        p = nullptr;
        n = 0;
        own = true;
    }
    // view `count` elements at `ptr` (memory owned elsewhere)
    void borrow(T *ptr, size_t count) noexcept {
        release();
        p = ptr;
        n = count;
        own = false;
    }
    void alloc(size_t count, hipStream_t stream) {
        release();
        s = stream;
        n = count;
        if (count == 0) return;
        try {
            p = (T *)dev_alloc(count * sizeof(T), stream);
        } catch (...) {
            p = nullptr;
            n = 0;
            throw;
        }
    }
    void ensure(size_t count, hipStream_t stream) {
        if (count > n || p == nullptr) alloc(count, stream);
    }
    T *get() const { return p; }
    size_t bytes() const { return n * sizeof(T); }
};

// ---------------------------------------------------------------------------
// Small device-to-host readbacks through a pinned host buffer (per host
// thread): reads never go through pageable memory.  Every readback waits
// for the stream.
// ---------------------------------------------------------------------------
struct Readback {
    explicit Readback(hipStream_t s) : stream(s) {}
    // queue a copy of `bytes` from device pointer `src` into host `dst`
    void add(void *dst, const void *src, size_t bytes);
    // issue the copies, wait for the stream, deliver to the destinations
    void run();
    hipStream_t stream;
    std::vector<std::pair<void *, size_t>> dst;   // destination, offset
    std::vector<std::pair<const void *, size_t>> src;
    size_t used = 0;
};
// Install (or, with null, remove) a hook that every Readback::run of this
// host thread calls after queueing its copies and before waiting for them:
// the hook may queue work on the readback's stream that does not feed the
// values read back, and the wait then covers the readback alone.  Returns
// the hook it replaces.
const std::function<void()> *set_readback_fill(const std::function<void()> *fill);
// pinned host staging buffer of at least `bytes` (reused; per host thread)
// A second pinned host buffer for host-to-device uploads that stay in
// flight across later readbacks (the readback buffer is pinned_staging).
void *pinned_upload(size_t bytes);
void *pinned_staging(size_t bytes);

// A square or rectangular CSR matrix on the device (int32 indices).
struct DevCSR {
    int32_t nrows = 0, ncols = 0;
    int64_t nnz = 0;
    int32_t max_row = -1;  // longest row when known, else -1
    DevArr<int32_t> rp, cj;
    DevArr<double> v;
    DevArr<float> v32;    // float copy of the values (mixed precision)
};

// ---------------------------------------------------------------------------
// Kernel profiler: when enabled (lair_profile_begin), launches of the
// selected categories are bracketed by HIP events on their own stream and
// tagged with their algorithmic bytes and flops.  Disabled it costs one
// branch per launch.
// ---------------------------------------------------------------------------
struct ProfScope {
    ProfScope(const char *category, hipStream_t s, double bytes, double flops = 0.0);
    ~ProfScope();
    ProfScope(const ProfScope &) = delete;
    ProfScope &operator=(const ProfScope &) = delete;
    int slot = -1, prev_slot = -1;
    hipStream_t stream = nullptr, prev_stream = nullptr;
};
// true while profiling is on and `category` is selected
bool prof_selected(const char *category);
// true while profiling is on
bool prof_active();
// Replace the algorithmic bytes of a closed scope's record (slot from
// ProfScope::slot; ignored when negative or profiling has restarted), for
// sizes that reach the host only after the scope's launches.
void prof_set_bytes(int slot, double bytes);
// Start/stop events for a kernel about to be launched on s inside a
// selected scope (false: launch without events).
bool prof_kernel_events(hipStream_t s, hipEvent_t *e0, hipEvent_t *e1);

// Every kernel launch of the library: with the profiler on, the launch
// carries its own start/stop events.
#define LAIR_LAUNCH(K, G, B, SH, S, ...)                                            \
    do {                                                                           \
        hipEvent_t lair_e0_ = nullptr, lair_e1_ = nullptr;                         \
        if (::lair::prof_kernel_events((S), &lair_e0_, &lair_e1_))                 \
            hipExtLaunchKernelGGL(K, G, B, SH, S, lair_e0_, lair_e1_, 0, __VA_ARGS__); \
        else                                                                       \
            hipLaunchKernelGGL(K, G, B, SH, S, __VA_ARGS__);                       \
    } while (0)

// An environment switch: set and not "0".
inline bool env_flag(const char *name) {
    const char *e = std::getenv(name);
    return e && *e && std::strcmp(e, "0") != 0;
}

// ---------------------------------------------------------------------------
// Launch helpers
// ---------------------------------------------------------------------------
inline unsigned blocks_for(int64_t threads, int bs) {
    int64_t b = (threads + bs - 1) / bs;
    return (unsigned)(b < 1 ? 1 : b);
}

// Team size for row-parallel kernels from the mean row length.
inline int team_for_mean(double mean_len) {
    int t = 2;
    while (t < 64 && t < mean_len) t <<= 1;
    return t;
}

// ---------------------------------------------------------------------------
// Setup kernels (k_setup.hip)
// ---------------------------------------------------------------------------
// exclusive scan of f(i) for i < n into out[0..n], returns out[n]
// optionally also returns the largest count and copies a device flag back
// in the same synchronisation
int64_t scan_counts_i64(const int32_t *cnt, int64_t *out, int64_t n, hipStream_t s,
                        DevArr<int64_t> &tmp, int64_t *max_out = nullptr);
int64_t scan_counts_i32(const int32_t *cnt, int32_t *out, int64_t n,
                        hipStream_t s, DevArr<int64_t> &tmp,
                        int64_t *max_out = nullptr, const int32_t *flag = nullptr,
                        int32_t *flag_out = nullptr);
int64_t scan_flags_i8(const int8_t *flags, int8_t want, int32_t *out, int64_t n,
                      hipStream_t s, DevArr<int64_t> &tmp);
// the same scans without a readback: tot[0] = total, tot[1] = largest value
// are written to device memory the caller reads later
// Check a caller's device CF splittings (0/1 values, whole nodes of k) and
// count each level's C-points into cnt[0..nlevels) (zeroed int64); bad[0]
// (zeroed) becomes nonzero on a bad value.  offs_dev: device level offsets.
void launch_cf_check(int32_t nlevels, const int64_t *offs_dev, int64_t total, const int8_t *cf,
                     int32_t k, int64_t *cnt, int32_t *bad, hipStream_t s);
void scan_counts_i32_to(const int32_t *cnt, int32_t *out, int64_t n, hipStream_t s,
                        DevArr<int64_t> &tmp, int64_t *tot);
void scan_counts_i64_to(const int32_t *cnt, int64_t *out, int64_t n, hipStream_t s,
                        DevArr<int64_t> &tmp, int64_t *tot);
void scan_flags_i8_to(const int8_t *flags, int8_t want, int32_t *out, int64_t n, hipStream_t s,
                      DevArr<int64_t> &tmp, int64_t *tot);
// split ordering (F-points, then C-points): perm[new] = old, iperm[old] =
// new, ids[k] = k, cf_split[k] = (k >= nf)
void launch_split_perm(int32_t nf, int32_t nc, const int32_t *flist, const int32_t *clist,
                       int32_t *perm, int32_t *iperm, int32_t *ids, int8_t *cf_split,
                       hipStream_t s);
// permuted copy of a CSR matrix: row k of the copy is row rowmap[k], column
// c becomes colmap[c] (nullptr: identity); rp_out is written on the device
// (no synchronisation); v_out, v32_out, cjt_out optional
void launch_permute_csr(int32_t nrows, int64_t nnz, double mean_row, const int32_t *rowmap,
                        const int32_t *irowmap, const int32_t *colmap, const int32_t *rp,
                        const int32_t *cj, const double *v, int32_t *rp_out, int32_t *cj_out,
                        double *v_out, float *v32_out, int32_t *cjt_out, int32_t nsplit,
                        DevArr<int64_t> &tmp, hipStream_t s);

int32_t validate_csr(int64_t n, int64_t nnz, const int32_t *rp,
                     const int32_t *cj, const double *v, hipStream_t s);
void launch_strength(int32_t n, const int32_t *rp, const int32_t *cj,
                     const double *v, double theta, int32_t kind,
                     uint8_t *smask, double mean_len, hipStream_t s);
// launch_strength and, on the same reads of each row, the counting pass of
// launch_interp_direct (cnt, coef: the same values, bit for bit), for a
// splitting cf known before the strength (the counting pass then need not
// read the matrix again).
void launch_strength_interp(int32_t n, const int32_t *rp, const int32_t *cj,
                            const double *v, double theta, int32_t kind, const int8_t *cf,
                            uint8_t *smask, int32_t *cnt, double *coef, double mean_len,
                            hipStream_t s);
// cidx, C and F row lists; acc[0] += nnz of F rows, acc[1] += nnz of C rows
void launch_cf_lists(int32_t n, const int8_t *cf, const int32_t *cidx_scan,
                     const int32_t *rp, int32_t *cidx, int32_t *clist,
                     int32_t *flist, unsigned long long *acc, hipStream_t s);
// neighbourhood sizes (fill = false) or lists (fill = true)
void launch_neighbourhoods(int32_t nc, int32_t n, const int32_t *clist,
                           const int32_t *rp, const int32_t *cj,
                           const uint8_t *smask, const int8_t *cf,
                           int32_t distance, const int32_t *flist, int32_t nf,
                           int32_t *cnt, const int32_t *nptr, int32_t *nbr,
                           int32_t *overflow, int32_t max_row_strong,
                           hipStream_t s, int32_t knode = 1);
struct LocalSolveOut {
    int32_t *r_rp, *r_cj;
    double *r_v;
    int8_t *flags;
};
// Lumping of a coarse operator (k_lump): counts of kept entries per row
// (cnt != nullptr), or the lumped rows written at rp_out.  The rows are CSR
// rows (rp), or staged rows at row_off[i] of length row_len[i] (row_off
// non-null; sorted columns, as the product leaves them).  Rows with
// whole_rows[i] != 0 are kept whole (whole_rows may be null).
void launch_lump(int32_t n, const int32_t *rp, const int64_t *row_off, const int32_t *row_len,
                 const int32_t *cj, const double *v, double theta, const int8_t *whole_rows,
                 double mean_len, int32_t *cnt, const int32_t *rp_out, int32_t *cj_out,
                 double *v_out, hipStream_t s);

// Flexible GMRES kernels (vectors of n rows x R interleaved right-hand
// sides, R a power of two up to 32; a basis: kc vectors ldv apart).
// op_mdot: out[k R + q] = (V_k, w)_q for k < kc (partial: kry_dot_blocks(n R)
// x kc x R doubles of scratch); op_maxpy: w -= sum_k coef[k R + q] V_k per
// right-hand side; op_scale_rhs: out = w * s[q] per right-hand side (out may
// be w).
int32_t kry_dot_blocks(int64_t m);
void op_mdot(int64_t n, int32_t R, const double *V, int64_t ldv, int32_t kc, const double *w,
             double *partial, double *out, hipStream_t s);
void op_maxpy(int64_t n, int32_t R, const double *V, int64_t ldv, int32_t kc,
              const double *coef, double *w, hipStream_t s);
void op_scale_rhs(int64_t n, int32_t R, const double *w, const double *sc, double *out,
                  hipStream_t s);

// Largest local system the one-wave kernel keeps in LDS (larger ones use a
// global slab).
constexpr int32_t WSMAX = 64;
// returns the number of systems solved by least squares.  smax may be an
// upper bound of the largest system (it selects kernels and tables).
// knode > 1: the C-rows form nodes of knode consecutive rows that share
// one neighbourhood (the nodal treatment), solved as one system with knode
// right-hand sides each; needs node_solves_fit(knode, smax, precision).
int64_t local_solves(int32_t nc, const int32_t *clist, const int32_t *nptr,
                     const int32_t *nbr, const int32_t *rp, const int32_t *cj,
                     const double *v, int32_t precision, int32_t smax, double mean_row,
                     LocalSolveOut out, hipStream_t s, int32_t *edges_used = nullptr,
                     Readback *rb_extra = nullptr, int32_t knode = 1);
bool node_solves_fit(int32_t k, int32_t smax, int32_t precision);
// process-wide bucket edges of the local solves and the fused flag (5
// values; nullptr: tune per shape); edges_used receives 5 values
void set_local_buckets(const int32_t *edges);
void launch_interp_one_point(int32_t n, const int32_t *rp, const int32_t *cj,
                             const double *v, const uint8_t *smask,
                             const int8_t *cf, const int32_t *cidx,
                             int32_t *pcol, hipStream_t s);
void launch_compact_one_point(int32_t n, const int32_t *pcol,
                              const int32_t *prp, int32_t *pcj, double *pv,
                              hipStream_t s);
// Direct interpolation: fill = false counts each row's entries into cnt,
// fill = true writes them.  coef (3 n doubles, optional): the counting pass
// keeps each F row's alpha, beta and lumped diagonal there and the filling
// pass reuses them instead of summing the row again.
void launch_interp_direct(int32_t n, const int32_t *rp, const int32_t *cj,
                          const double *v, const uint8_t *smask,
                          const int8_t *cf, const int32_t *cidx, bool fill,
                          int32_t *cnt, const int32_t *prp, int32_t *pcj,
                          double *pv, double mean_len, hipStream_t s,
                          double *coef = nullptr);
// C = A B in three steps: launch_prod_count gives the products of every row
// (an upper bound of its length); launch_spgemm writes each row of C,
// sorted, at its product offset eoff[i] of the staging arrays (tcj, tcx)
// and its length into cnt; launch_spgemm_compact copies the rows to C
// (row pointers crp from a scan of cnt).  work: 4 + 3 m int32, the first
// four zeroed by the caller; *overflow zeroed by the caller.  mean_c_hint:
// an estimate of the distinct columns per row of C (0: none), which sizes
// the first pass's tables.
// Rows of the right factor B of a sparse product: CSR (rp), or rows staged
// by an earlier product at offsets off[k] with lengths len[k] (rp null;
// offsets below 2^31).
struct BRows {
    const int32_t *rp = nullptr;
    const int64_t *off = nullptr;
    const int32_t *len = nullptr;
    __device__ __forceinline__ int start(int k) const { return rp ? rp[k] : (int)off[k]; }
    __device__ __forceinline__ int length(int k) const {
        return rp ? rp[k + 1] - rp[k] : len[k];
    }
};
void launch_prod_count(int32_t m, const int32_t *ap, const int32_t *aj, BRows bp,
                       int32_t *e, hipStream_t s);
void launch_spgemm(int32_t m, const int32_t *ap, const int32_t *aj, const double *ax,
                   BRows bp, const int32_t *bj, const double *bx,
                   const int64_t *eoff, int64_t max_e, double mean_e, double mean_c_hint,
                   int32_t *cnt, int32_t *tcj, double *tcx, int32_t *counts, int32_t *lists,
                   int32_t *overflow, hipStream_t s);
void launch_spgemm_compact(int32_t m, const int64_t *eoff, const int32_t *crp,
                           const int32_t *tcj, const double *tcx, int32_t *cj, double *cx,
                           double mean_c, hipStream_t s);
void launch_transpose(int32_t nrows, int32_t ncols, int64_t nnz,
                      const int32_t *rp, const int32_t *cj, const double *v,
                      int32_t *tcount, int32_t *trp, int32_t *tcj, double *tv,
                      int32_t *cursor, hipStream_t s, DevArr<int64_t> &tmp);
void launch_to_float(const double *in, float *out, int64_t n, hipStream_t s);
void launch_block_inverse(int32_t nblk, int32_t k, const int32_t *rp,
                          const int32_t *cj, const double *v, double *dinv,
                          int32_t *bad, hipStream_t s);
// dense coarsest factorisation
void launch_dense_from_csr(int32_t n, const int32_t *rp, const int32_t *cj,
                           const double *v, double *dense, hipStream_t s);
// n <= 128 and n^2 doubles fit one workgroup's LDS: the explicit inverse of
// the dense matrix by Gauss-Jordan in one kernel; false when it does not apply
bool launch_dense_gj_inv(int32_t n, const double *dense, double *inv, int32_t *info,
                         hipStream_t s);
void launch_dense_lu(int32_t n, double *lu, int32_t *piv, int32_t *info,
                     hipStream_t s);
// inv = K^{-1} from the factors of launch_dense_lu (n <= 4096)
void launch_dense_inverse(int32_t n, const double *lu, const int32_t *piv,
                          double *inv, hipStream_t s);

// ---------------------------------------------------------------------------
// Cycle kernels (k_cycle.hip)
// ---------------------------------------------------------------------------
template <class VT>
struct CsrView {
    int32_t nrows, ncols;
    const int32_t *rp, *cj;
    const VT *v;
    int32_t team;      // lanes per row for single right-hand sides
    const int32_t *cjt = nullptr;   // columns tagged with the C/F type, or null
};
// cjt[p] = cj[p] with bit 31 set when cf[cj[p]] = 1 (C-point)
void launch_tag_columns(int64_t nnz, const int32_t *cj, const int8_t *cf, int32_t *cjt,
                        hipStream_t s);

template <class VT>
void op_residual(const CsrView<VT> &A, const VT *b, const VT *x, VT *r,
                 int32_t nrhs, hipStream_t s);
// y = A x (or y += A x).  With x_hi, some rows of x are read from x_hi
// instead (a vector left in two buffers): the rows >= csplit when csplit >= 0
// (aligned multi-vectors only), else the rows with cf_hi[c] = 1; see
// op_spmv_split_ok.
template <class VT>
void op_spmv(const CsrView<VT> &A, const VT *x, VT *y, int32_t nrhs,
             bool accumulate, hipStream_t s, const VT *x_hi = nullptr, int32_t csplit = -1,
             const int8_t *cf_hi = nullptr);
bool op_spmv_split_ok(int32_t nrhs, const void *x, const void *x_hi, const void *y);
// Jacobi on rows X: out[k] (compact) or out[i] = x_i + omega (b - A x)_i / a_ii.
// With cf non-null, neighbour values come from xC at C-points and from xF
// at F-points; otherwise everything is read from xF.  rows == nullptr
// means the contiguous rows row0 .. row0 + nrows - 1.
template <class VT>
void op_jacobi(const CsrView<VT> &A, const int32_t *rows, int32_t nrows,
               const VT *b, const VT *xF, const VT *xC, const int8_t *cf,
               VT *out, bool compact, double omega, int32_t nrhs,
               hipStream_t s, const int32_t *cnt = nullptr, int32_t row0 = 0);
template <class VT>
void op_coarse_apply(int32_t n, const double *kinv, const VT *b, VT *x,
                     int32_t nrhs, bool transpose, hipStream_t s);
template <class VT>
void op_scatter(const int32_t *rows, int32_t nrows, const VT *t, VT *x,
                int32_t nrhs, hipStream_t s, const int32_t *cnt = nullptr,
                int32_t row0 = 0);
template <class VT>
void op_fill(VT *x, VT val, int64_t n, hipStream_t s);
template <class VT>
void op_copy(const VT *x, VT *y, int64_t n, hipStream_t s);
template <class VT>
void op_dense_solve(int32_t n, const double *lu, const int32_t *piv,
                    const VT *b, VT *x, int32_t nrhs, bool transpose,
                    hipStream_t s);
// per right-hand side sum of squares into out[0..nrhs) (double, fixed order)
// One right-hand side over the listed rows rows[k], k < *cnt (device list of
// capacity cap): mode 0 y = b - A x, 1 y = A x, 2 y += A x.
template <class VT>
void op_rowdot_list(const CsrView<VT> &A, int mode, const int32_t *rows, const int32_t *cnt,
                    int32_t cap, const VT *x, const VT *b, VT *y, hipStream_t s);
// x[i] += e[i] for the listed rows
template <class ET>
void op_update_list(const int32_t *rows, const int32_t *cnt, int32_t cap, double *x,
                    const ET *e, hipStream_t s);
// r = b - A x with its per-column sums of squares (out, nrhs entries) in one
// pass, written as r64 and/or r32.  Returns false (nothing launched) when the
// vectors are not 16-byte aligned for nrhs > 1.  partial: npartial * nrhs.
bool op_residual_norm(const CsrView<double> &A, const double *b, const double *x,
                      double *r64, float *r32, int32_t nrhs, double *partial,
                      int32_t npartial, double *out, hipStream_t s,
                      const int32_t *orow = nullptr);
void op_sumsq(const double *r, int64_t n, int32_t nrhs, double *partial,
              int32_t npartial, double *out, hipStream_t s);
void op_axpy_f32(double *x, const float *e, int64_t n, hipStream_t s);
// x[i] += e[map[i]], out[map[i]] = (float) in[i] (rows of nrhs); with e_hi
// the rows map[i] >= split of e are read from e_hi
void op_axpy_f32_rows(double *x, const float *e, const int32_t *map, int64_t n, int32_t nrhs,
                      hipStream_t s, const float *e_hi = nullptr, int32_t split = 0);
void op_cast_f32_rows(const double *in, float *out, const int32_t *map, int64_t n,
                      int32_t nrhs, hipStream_t s);
void op_cast_f32(const double *in, float *out, int64_t n, hipStream_t s);
// to_split: out[k] = in[perm[k]]; else out[perm[k]] = in[k] (rows of nrhs)
void op_permute_rows(int64_t n, int32_t nrhs, const int32_t *perm, const double *in,
                     double *out, bool to_split, hipStream_t s);
void op_cast_f64(const float *in, double *out, int64_t n, hipStream_t s);
void op_block_apply(int32_t nblk, int32_t k, const double *dinv,
                    const double *b, double *out, int32_t nrhs, hipStream_t s);

// ---------------------------------------------------------------------------
// Nodal treatment of k x k blocks (k_nodal.hip).  The matrix is scalar CSR
// whose k rows of a node store the same whole dense blocks.
// ---------------------------------------------------------------------------
// true when every row of every node stores its node's whole dense blocks
// (waits for the answer)
bool node_check(int32_t n, int32_t k, const int32_t *rp, const int32_t *cj, int64_t nnz,
                hipStream_t s);
// smask over A's entries: every entry of a block with
// ||A_ij||_F^2 >= theta^2 max_{l != i} ||A_il||_F^2 (nonzero)
void launch_node_strength(int32_t n, int32_t k, const int32_t *rp, const int32_t *cj,
                          const double *v, int64_t nnz, double theta, uint8_t *smask,
                          hipStream_t s);
// one-point interpolation by block: pcol[r] = coarse column of row r or -1
void launch_interp_1p_node(int32_t n, int32_t k, const int32_t *rp, const int32_t *cj,
                           const double *v, int64_t nnz, const uint8_t *smask, const int8_t *cf,
                           const int32_t *cidx, int32_t *pcol, hipStream_t s);
// out = D^{-1} A on A's pattern (dinv: the inverse diagonal blocks)
void launch_node_scale(int32_t n, int32_t k, const int32_t *rp, const double *v, int64_t nnz,
                       const double *dinv, double *out, hipStream_t s);
// parallel PMIS-type CF splitting on the device (k_split.hip): cf[i] = 1
// for C, 0 for F
void launch_pmis_split(int32_t n, const int32_t *rp, const int32_t *cj, const uint8_t *smask,
                       int8_t *cf, hipStream_t s);
// out = D^{-1} b for nrhs interleaved right-hand sides
template <class VT>
void op_node_rhs(int32_t n, int32_t k, int32_t nrhs, const double *dinv, const VT *b, VT *out,
                 hipStream_t s);

// ---------------------------------------------------------------------------
// Batch kernels (k_batch.hip)
// ---------------------------------------------------------------------------
struct SysCsr {
    const int32_t *rp;
    const int32_t *cj;
    const double *v;
    int64_t n, nnz;
};
void launch_union_gather(int32_t nsys, const SysCsr *sys, const int64_t *seg,
                         const int64_t *nzo, int32_t *rp, int32_t *cj, double *v, int32_t *bad,
                         int64_t max_nnz, hipStream_t s);
void launch_seg_count_c(int32_t nsys, const int64_t *seg, const int8_t *cf, int32_t *count,
                        hipStream_t s);
void launch_force_c(int32_t nsys, const int64_t *seg, const uint8_t *stopped, int8_t *cf,
                    int64_t nrows, hipStream_t s);
// flag[r] = 1 for the rows (seg: nsys + 1 offsets) of the stopped systems
void launch_stopped_rows(int32_t nsys, const int64_t *seg, const uint8_t *stopped, int8_t *flag,
                         int64_t nrows, hipStream_t s);
int32_t relax_list(int32_t nsys, const int64_t *seg, const uint8_t *stopped,
                   const int32_t *clist, int32_t nc, DevArr<int32_t> &out,
                   hipStream_t s, DevArr<int64_t> &tmp);
void launch_seg_sumsq(int32_t nsys, const int64_t *seg, const double *r, double *out,
                      hipStream_t s, const uint8_t *active = nullptr);
int64_t seg_sum_chunk();
void launch_seg_sumsq_blocks(int32_t nsys, int32_t nblk, const int32_t *bsys,
                             const int64_t *blo, const int64_t *bstart, const int64_t *seg,
                             const uint8_t *active, const double *r, double *part,
                             double *out, hipStream_t s);
void launch_block_apply_inv(int32_t nsys, const int64_t *seg, const int64_t *doff,
                            const double *inv, const double *b, double *x, bool transpose,
                            hipStream_t s, const uint8_t *active, const uint8_t *use_inv);
void launch_materialize(int32_t nseg, int64_t total, const int64_t *seg_out,
                        const int32_t *seg_src, const int32_t *seg_dst, const int32_t *lst,
                        const int32_t *const *srcs, int32_t *const *dsts, hipStream_t s);
void launch_dense_blocks(int32_t nsys, const int64_t *seg, const int64_t *doff,
                         const int32_t *rp, const int32_t *cj, const double *v,
                         double *dense, int64_t nrows, hipStream_t s);
void launch_block_lu(int32_t nsys, const int64_t *seg, const int64_t *doff, double *dense,
                     int32_t *piv, int32_t *info, hipStream_t s, int32_t min_n = 0);
// blocks of at most small_dense_max() rows: LU and inverse in one kernel
int32_t small_dense_max();
// blocks of small_dense_max()+1 .. mid_dense_max() rows: inverse from the LU
int32_t mid_dense_max();
void launch_block_inv_mid(int32_t nsys, int32_t maxn, const int64_t *seg, const int64_t *doff,
                          const double *lu, const int32_t *piv, double *inv,
                          const uint8_t *use_inv, hipStream_t s);
void launch_block_lu_inv_small(int32_t nsys, const int64_t *seg, const int64_t *doff,
                               double *dense, int32_t *piv, double *inv, int32_t *info,
                               hipStream_t s);
void launch_block_solve(int32_t nsys, const int64_t *seg, const int64_t *doff,
                        const double *dense, const int32_t *piv, const double *b, double *x,
                        bool transpose, hipStream_t s, const uint8_t *active = nullptr,
                        const uint8_t *skip = nullptr);

}  // namespace lair
