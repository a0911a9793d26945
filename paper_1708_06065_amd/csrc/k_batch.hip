// Kernels for a batch of independent systems solved as one block-diagonal
// union: building the union, per-system (segmented) counts and norms,
// per-system activity masks, and the per-system coarsest-grid solves.
//
// Segments: system s owns rows [seg[s], seg[s+1]) of a level; seg has
// nsys + 1 entries (int64).  The system of a row is found by binary search.
#include <cmath>

#include "k_common.hpp"
#include "lair_internal.hpp"

namespace lair {

__device__ __forceinline__ int32_t seg_of(const int64_t *seg, int32_t nsys, int64_t row) {
    int lo = 0, hi = nsys - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (seg[mid] <= row) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Union of the systems, gathered from device arrays: one workgroup per
// system copies its rows and entries to its row offset seg[s] and entry
// offset nzo[s], shifting row pointers and columns.  Malformed members
// (rowptr[0] != 0, rowptr[n_s] != nnz_s, a column outside [0, n_s)) set
// *bad; the union is then validated as one matrix.
__global__ void __launch_bounds__(256)
k_union_gather(int32_t nsys, const SysCsr *sys, const int64_t *seg, const int64_t *nzo,
               int32_t *rp, int32_t *cj, double *v, int32_t *bad) {
    const int32_t s = blockIdx.x;
    const SysCsr q = sys[s];
    const int64_t r0 = seg[s], z0 = nzo[s];
    int flag = 0;
    for (int64_t i = threadIdx.x; i <= q.n; i += 256) {
        int32_t p = q.rp[i];
        if ((i == 0 && p != 0) || (i == q.n && (int64_t)p != q.nnz)) flag = 1;
        if (i < q.n) rp[r0 + i] = (int32_t)(z0 + p);
    }
    for (int64_t p = threadIdx.x; p < q.nnz; p += 256) {
        int32_t c = q.cj[p];
        if (c < 0 || (int64_t)c >= q.n) flag = 1;
        cj[z0 + p] = (int32_t)(c + r0);
        v[z0 + p] = q.v[p];
    }
    if (flag) atomicOr(bad, 1);
    if (s == nsys - 1 && threadIdx.x == 0) rp[seg[nsys]] = (int32_t)nzo[nsys];
}

void launch_union_gather(int32_t nsys, const SysCsr *sys, const int64_t *seg,
                         const int64_t *nzo, int32_t *rp, int32_t *cj, double *v, int32_t *bad,
                         hipStream_t s) {
    LAIR_LAUNCH(k_union_gather, dim3(nsys), dim3(256), 0, s, nsys, sys, seg, nzo, rp,
                       cj, v, bad);
    LAIR_LAUNCH_CHECK();
}

// Number of C-points of every system (one block per system, fixed order).
__global__ void __launch_bounds__(256)
k_seg_count_c(const int64_t *seg, const int8_t *cf, int32_t *count) {
    __shared__ int32_t sh[256];
    int32_t s = blockIdx.x;
    int32_t acc = 0;
    for (int64_t r = seg[s] + threadIdx.x; r < seg[s + 1]; r += 256) acc += (cf[r] == 1);
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) count[s] = sh[0];
}

void launch_seg_count_c(int32_t nsys, const int64_t *seg, const int8_t *cf, int32_t *count,
                        hipStream_t s) {
    LAIR_LAUNCH(k_seg_count_c, dim3(nsys), dim3(256), 0, s, seg, cf, count);
    LAIR_LAUNCH_CHECK();
}

// Rows of systems that stopped coarsening become C-points (identity
// transfer: their coarse operator is their current operator).
__global__ void k_force_c(int32_t nsys, const int64_t *seg, const uint8_t *stopped,
                          int8_t *cf, int64_t nrows) {
    int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nrows) return;
    if (stopped[seg_of(seg, nsys, r)]) cf[r] = 1;
}

void launch_force_c(int32_t nsys, const int64_t *seg, const uint8_t *stopped, int8_t *cf,
                    int64_t nrows, hipStream_t s) {
    LAIR_LAUNCH(k_force_c, dim3(blocks_for(nrows, 256)), dim3(256), 0, s,
                       nsys, seg, stopped, cf, nrows);
    LAIR_LAUNCH_CHECK();
}

// flag[k] = 1 when C-point clist[k] belongs to a system still coarsening
// (the only C rows that are relaxed).
__global__ void k_relax_flags(int32_t nsys, const int64_t *seg, const uint8_t *stopped,
                              const int32_t *clist, int32_t nc, int8_t *flag) {
    int32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nc) return;
    flag[k] = stopped[seg_of(seg, nsys, clist[k])] ? 0 : 1;
}

__global__ void k_compact_list(const int8_t *flag, const int32_t *scan,
                               const int32_t *src, int32_t n, int32_t *dst) {
    int32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n && flag[k]) dst[scan[k]] = src[k];
}

int32_t relax_list(int32_t nsys, const int64_t *seg, const uint8_t *stopped,
                   const int32_t *clist, int32_t nc, DevArr<int32_t> &out,
                   hipStream_t s, DevArr<int64_t> &tmp) {
    DevArr<int8_t> flag;
    DevArr<int32_t> scan;
    flag.alloc((size_t)std::max(nc, 1), s);
    scan.alloc((size_t)nc + 1, s);
    LAIR_LAUNCH(k_relax_flags, dim3(blocks_for(nc, 256)), dim3(256), 0, s,
                       nsys, seg, stopped, clist, nc, flag.get());
    LAIR_LAUNCH_CHECK();
    int64_t cnt = scan_flags_i8(flag.get(), 1, scan.get(), nc, s, tmp);
    out.alloc((size_t)std::max<int64_t>(cnt, 1), s);
    LAIR_LAUNCH(k_compact_list, dim3(blocks_for(nc, 256)), dim3(256), 0, s,
                       flag.get(), scan.get(), clist, nc, out.get());
    LAIR_LAUNCH_CHECK();
    return (int32_t)cnt;
}

// All active-row lists of a batch in one launch.  The outputs are laid end
// to end in one index space; segment j covers [seg_out[j], seg_out[j+1]) of
// it and copies `len` consecutive entries of list `lst[j]`'s source from
// seg_src[j] (or the row ids themselves when that list has no source) to
// its output at seg_dst[j].  No atomics: every position has one writer.
__global__ void k_materialize(int32_t nseg, const int64_t *seg_out, const int32_t *seg_src,
                              const int32_t *seg_dst, const int32_t *lst,
                              const int32_t *const *srcs, int32_t *const *dsts) {
    const int64_t total = seg_out[nseg];
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < total;
         k += (int64_t)gridDim.x * blockDim.x) {
        int lo = 0, hi = nseg - 1;
        while (lo < hi) {
            int mid = (lo + hi + 1) >> 1;
            if (seg_out[mid] <= k) lo = mid; else hi = mid - 1;
        }
        const int32_t off = (int32_t)(k - seg_out[lo]);
        const int32_t *src = srcs[lst[lo]];
        const int32_t v = src ? src[seg_src[lo] + off] : seg_src[lo] + off;
        dsts[lst[lo]][seg_dst[lo] + off] = v;
    }
}

void launch_materialize(int32_t nseg, int64_t total, const int64_t *seg_out,
                        const int32_t *seg_src, const int32_t *seg_dst, const int32_t *lst,
                        const int32_t *const *srcs, int32_t *const *dsts, hipStream_t s) {
    if (nseg == 0 || total == 0) return;
    const int64_t b = (total + 255) / 256;
    LAIR_LAUNCH(k_materialize, dim3((unsigned)(b < 4096 ? b : 4096)), dim3(256), 0, s, nseg,
                seg_out, seg_src, seg_dst, lst, srcs, dsts);
    LAIR_LAUNCH_CHECK();
}

// Per-system sum of squares (one block per system, fixed order).
__global__ void __launch_bounds__(256)
k_seg_sumsq(const int64_t *seg, const uint8_t *active, const double *r, double *out) {
    __shared__ double sh[256];
    int32_t s = blockIdx.x;
    if (active && !active[s]) return;      // a finished system keeps its last norm
    double acc = 0.0;
    for (int64_t i = seg[s] + threadIdx.x; i < seg[s + 1]; i += 256) acc += r[i] * r[i];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[s] = sh[0];
}

void launch_seg_sumsq(int32_t nsys, const int64_t *seg, const double *r, double *out,
                      hipStream_t s, const uint8_t *active) {
    LAIR_LAUNCH(k_seg_sumsq, dim3(nsys), dim3(256), 0, s, seg, active, r, out);
    LAIR_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// Per-system coarsest grids.  System s owns the dense block at doff[s] of
// size m_s = seg[s+1] - seg[s] (row-major).
// ---------------------------------------------------------------------------
__global__ void k_dense_blocks(int32_t nsys, const int64_t *seg, const int64_t *doff,
                               const int32_t *rp, const int32_t *cj, const double *v,
                               double *dense, int64_t nrows) {
    int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nrows) return;
    int32_t s = seg_of(seg, nsys, r);
    int64_t m = seg[s + 1] - seg[s];
    int64_t i = r - seg[s];
    double *row = dense + doff[s] + i * m;
    for (int64_t q = 0; q < m; ++q) row[q] = 0.0;
    for (int p = rp[r]; p < rp[r + 1]; ++p) {
        int64_t c = cj[p] - seg[s];
        if (c >= 0 && c < m) row[c] = v[p];   // the union is block-diagonal
    }
}

// LU with partial pivoting of every block, one workgroup per system.
__global__ void __launch_bounds__(256)
k_block_lu(const int64_t *seg, const int64_t *doff, double *dense, int32_t *piv,
           int32_t *info) {
    __shared__ double sv[256];
    __shared__ int si[256];
    int32_t s = blockIdx.x;
    int t = threadIdx.x;
    const int n = (int)(seg[s + 1] - seg[s]);
    double *a = dense + doff[s];
    int32_t *pv = piv + seg[s];
    for (int k = 0; k < n; ++k) {
        double best = -1.0;
        int bi = INT_MAX;
        for (int r = k + t; r < n; r += 256) {
            double x = fabs(a[(size_t)r * n + k]);
            if (x > best) { best = x; bi = r; }
        }
        sv[t] = best;
        si[t] = bi;
        __syncthreads();
        for (int o = 128; o > 0; o >>= 1) {
            if (t < o) {
                double ov = sv[t + o];
                int oi = si[t + o];
                if (ov > sv[t] || (ov == sv[t] && oi < si[t])) { sv[t] = ov; si[t] = oi; }
            }
            __syncthreads();
        }
        int pr = si[0];
        double pvv = sv[0];
        __syncthreads();
        if (pvv == 0.0) {
            if (t == 0) atomicMax(info, s + 1);
            return;
        }
        if (t == 0) pv[k] = pr;
        if (pr != k)
            for (int q = t; q < n; q += 256) {
                double x = a[(size_t)k * n + q];
                a[(size_t)k * n + q] = a[(size_t)pr * n + q];
                a[(size_t)pr * n + q] = x;
            }
        __syncthreads();
        double inv = 1.0 / a[(size_t)k * n + k];
        for (int r = k + 1 + t; r < n; r += 256) a[(size_t)r * n + k] *= inv;
        __syncthreads();
        int w = n - k - 1;
        for (int idx = t; idx < w * w; idx += 256) {
            int r = k + 1 + idx / w;
            int q = k + 1 + idx % w;
            a[(size_t)r * n + q] -= a[(size_t)r * n + k] * a[(size_t)k * n + q];
        }
        __syncthreads();
    }
}

// x = K_s^{-1} b (or K_s^{-T} b) for every system, one workgroup per system
// and right-hand side column held in place (nrhs = 1).
__global__ void __launch_bounds__(256)
k_block_solve(const int64_t *seg, const int64_t *doff, const double *dense,
              const int32_t *piv, const double *b, double *x, int transpose,
              const uint8_t *active) {
    int32_t s = blockIdx.x;
    if (active && !active[s]) return;
    int t = threadIdx.x;
    const int n = (int)(seg[s + 1] - seg[s]);
    const double *a = dense + doff[s];
    const int32_t *pv = piv + seg[s];
    double *xs = x + seg[s];
    const double *bs = b + seg[s];
    for (int i = t; i < n; i += 256) xs[i] = bs[i];
    __syncthreads();
    if (!transpose) {
        if (t == 0)
            for (int k = 0; k < n; ++k)
                if (pv[k] != k) { double q = xs[k]; xs[k] = xs[pv[k]]; xs[pv[k]] = q; }
        __syncthreads();
        for (int k = 0; k < n; ++k) {
            for (int r = k + 1 + t; r < n; r += 256) xs[r] -= a[(size_t)r * n + k] * xs[k];
            __syncthreads();
        }
        for (int k = n - 1; k >= 0; --k) {
            if (t == 0) xs[k] /= a[(size_t)k * n + k];
            __syncthreads();
            for (int r = t; r < k; r += 256) xs[r] -= a[(size_t)r * n + k] * xs[k];
            __syncthreads();
        }
    } else {
        for (int k = 0; k < n; ++k) {
            if (t == 0) xs[k] /= a[(size_t)k * n + k];
            __syncthreads();
            for (int r = k + 1 + t; r < n; r += 256) xs[r] -= a[(size_t)k * n + r] * xs[k];
            __syncthreads();
        }
        for (int k = n - 1; k >= 0; --k) {
            for (int r = t; r < k; r += 256) xs[r] -= a[(size_t)k * n + r] * xs[k];
            __syncthreads();
        }
        if (t == 0)
            for (int k = n - 1; k >= 0; --k)
                if (pv[k] != k) { double q = xs[k]; xs[k] = xs[pv[k]]; xs[pv[k]] = q; }
    }
}

void launch_dense_blocks(int32_t nsys, const int64_t *seg, const int64_t *doff,
                         const int32_t *rp, const int32_t *cj, const double *v,
                         double *dense, int64_t nrows, hipStream_t s) {
    LAIR_LAUNCH(k_dense_blocks, dim3(blocks_for(nrows, 64)), dim3(64), 0, s,
                       nsys, seg, doff, rp, cj, v, dense, nrows);
    LAIR_LAUNCH_CHECK();
}

void launch_block_lu(int32_t nsys, const int64_t *seg, const int64_t *doff, double *dense,
                     int32_t *piv, int32_t *info, hipStream_t s) {
    LAIR_LAUNCH(k_block_lu, dim3(nsys), dim3(256), 0, s, seg, doff, dense, piv, info);
    LAIR_LAUNCH_CHECK();
}

void launch_block_solve(int32_t nsys, const int64_t *seg, const int64_t *doff,
                        const double *dense, const int32_t *piv, const double *b, double *x,
                        bool transpose, hipStream_t s, const uint8_t *active) {
    LAIR_LAUNCH(k_block_solve, dim3(nsys), dim3(256), 0, s, seg, doff, dense, piv, b, x,
                       transpose ? 1 : 0, active);
    LAIR_LAUNCH_CHECK();
}

}  // namespace lair
