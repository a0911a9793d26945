// Kernels for a batch of independent systems solved as one block-diagonal
// union: building the union, per-system (segmented) counts and norms,
// per-system activity masks, and the per-system coarsest-grid solves.
//
// Segments: system s owns rows [seg[s], seg[s+1]) of a level; seg has
// nsys + 1 entries (int64).  The system of a row is found by binary search.
#include <algorithm>
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
    // blockIdx.y takes one of gridDim.y slices of the rows and of the entries
    const int64_t gy = gridDim.y, y = blockIdx.y;
    const int64_t rlo = (q.n + 1) * y / gy, rhi = (q.n + 1) * (y + 1) / gy;
    const int64_t plo = q.nnz * y / gy, phi = q.nnz * (y + 1) / gy;
    int flag = 0;
    for (int64_t i = rlo + threadIdx.x; i < rhi; i += 256) {
        int32_t p = q.rp[i];
        if ((i == 0 && p != 0) || (i == q.n && (int64_t)p != q.nnz)) flag = 1;
        if (i < q.n) rp[r0 + i] = (int32_t)(z0 + p);
    }
    for (int64_t p = plo + threadIdx.x; p < phi; p += 256) {
        int32_t c = q.cj[p];
        if (c < 0 || (int64_t)c >= q.n) flag = 1;
        cj[z0 + p] = (int32_t)(c + r0);
        v[z0 + p] = q.v[p];
    }
    if (flag) atomicOr(bad, 1);
    if (s == nsys - 1 && y == 0 && threadIdx.x == 0) rp[seg[nsys]] = (int32_t)nzo[nsys];
}

void launch_union_gather(int32_t nsys, const SysCsr *sys, const int64_t *seg,
                         const int64_t *nzo, int32_t *rp, int32_t *cj, double *v, int32_t *bad,
                         int64_t max_nnz, hipStream_t s) {
    int64_t gy = (max_nnz + 16383) / 16384;
    if (gy < 1) gy = 1;
    if (gy > 256) gy = 256;
    LAIR_LAUNCH(k_union_gather, dim3(nsys, (unsigned)gy), dim3(256), 0, s, nsys, sys, seg, nzo,
                rp, cj, v, bad);
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

// flag[r] = 1 for the rows of the systems that have stopped coarsening.
__global__ void k_stopped_rows(int32_t nsys, const int64_t *seg, const uint8_t *stopped,
                               int8_t *flag, int64_t nrows) {
    int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nrows) return;
    flag[r] = stopped[seg_of(seg, nsys, r)] ? 1 : 0;
}

void launch_stopped_rows(int32_t nsys, const int64_t *seg, const uint8_t *stopped, int8_t *flag,
                         int64_t nrows, hipStream_t s) {
    if (nrows == 0) return;
    LAIR_LAUNCH(k_stopped_rows, dim3(blocks_for(nrows, 256)), dim3(256), 0, s,
                nsys, seg, stopped, flag, nrows);
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
__global__ void __launch_bounds__(256)
k_materialize(int32_t nseg, const int64_t *seg_out, const int32_t *seg_src,
              const int32_t *seg_dst, const int32_t *lst, const int32_t *const *srcs,
              int32_t *const *dsts) {
    // one block per segment (grid-stride over segments): a straight copy of
    // its run, coalesced, with no search per entry
    for (int32_t g = blockIdx.x; g < nseg; g += gridDim.x) {
        const int64_t len = seg_out[g + 1] - seg_out[g];
        const int32_t *src = srcs[lst[g]];
        int32_t *dst = dsts[lst[g]] + seg_dst[g];
        const int32_t s0 = seg_src[g];
        if (src) {
            for (int64_t o = threadIdx.x; o < len; o += blockDim.x) dst[o] = src[s0 + o];
        } else {
            for (int64_t o = threadIdx.x; o < len; o += blockDim.x) dst[o] = s0 + (int32_t)o;
        }
    }
}

void launch_materialize(int32_t nseg, int64_t total, const int64_t *seg_out,
                        const int32_t *seg_src, const int32_t *seg_dst, const int32_t *lst,
                        const int32_t *const *srcs, int32_t *const *dsts, hipStream_t s) {
    if (nseg == 0 || total == 0) return;
    LAIR_LAUNCH(k_materialize, dim3((unsigned)std::min(nseg, 8192)), dim3(256), 0, s, nseg,
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

// Per-system sums of squares over several blocks per system: block b sums
// rows [blo[b], min(blo[b] + SEG_CHUNK, end of its system)) into part[b];
// then one block per system adds its blocks' partials in order.
constexpr int64_t SEG_CHUNK = 8192;

__global__ void __launch_bounds__(256)
k_seg_sumsq_part(const int32_t *bsys, const int64_t *blo, const int64_t *seg,
                 const uint8_t *active, const double *r, double *part) {
    __shared__ double sh[256];
    const int32_t b = blockIdx.x;
    const int32_t q = bsys[b];
    if (active && !active[q]) return;
    const int64_t lo = blo[b];
    const int64_t hi = lo + SEG_CHUNK < seg[q + 1] ? lo + SEG_CHUNK : seg[q + 1];
    double acc = 0.0;
    for (int64_t i = lo + threadIdx.x; i < hi; i += 256) acc += r[i] * r[i];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[b] = sh[0];
}

__global__ void __launch_bounds__(256)
k_seg_sumsq_final(const int64_t *bstart, const uint8_t *active, const double *part,
                  double *out) {
    __shared__ double sh[256];
    const int32_t q = blockIdx.x;
    if (active && !active[q]) return;
    double acc = 0.0;
    for (int64_t b = bstart[q] + threadIdx.x; b < bstart[q + 1]; b += 256) acc += part[b];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[q] = sh[0];
}

int64_t seg_sum_chunk() { return SEG_CHUNK; }

void launch_seg_sumsq_blocks(int32_t nsys, int32_t nblk, const int32_t *bsys,
                             const int64_t *blo, const int64_t *bstart, const int64_t *seg,
                             const uint8_t *active, const double *r, double *part,
                             double *out, hipStream_t s) {
    LAIR_LAUNCH(k_seg_sumsq_part, dim3(nblk), dim3(256), 0, s, bsys, blo, seg, active, r, part);
    LAIR_LAUNCH_CHECK();
    LAIR_LAUNCH(k_seg_sumsq_final, dim3(nsys), dim3(256), 0, s, bstart, active, part, out);
    LAIR_LAUNCH_CHECK();
}

// Systems whose coarsest block has at most 64 rows: one wave per system does
// the LU with partial pivoting and the inverse in LDS (the block and the
// inverse, 32 KB each).  Ties in the pivot search go to the smallest row,
// as in k_block_lu, so the factors and pivots are the same.
constexpr int SMALL_DENSE = 64;

__global__ void __launch_bounds__(64)
k_block_lu_inv_small(const int64_t *seg, const int64_t *doff, double *dense, int32_t *piv,
                     double *inv, int32_t *info) {
    __shared__ double a[SMALL_DENSE * SMALL_DENSE];
    __shared__ double x[SMALL_DENSE * SMALL_DENSE];
    __shared__ int32_t spv[SMALL_DENSE];
    const int32_t s = blockIdx.x;
    const int n = (int)(seg[s + 1] - seg[s]);
    if (n > SMALL_DENSE) return;
    const int t = threadIdx.x;
    double *g = dense + doff[s];
    for (int e = t; e < n * n; e += 64) a[e] = g[e];
    wave_lds_sync();
    int32_t *pv = piv + seg[s];
    for (int k = 0; k < n; ++k) {
        double bv = -1.0;
        int bi = INT_MAX;
        if (t >= k && t < n) { bv = fabs(a[t * n + k]); bi = t; }
        team_argmax<WAVE>(bv, bi);
        if (bv == 0.0) {
            if (t == 0) atomicMax(info, s + 1);
            return;
        }
        if (t == 0) { pv[k] = bi; spv[k] = bi; }
        if (bi != k && t < n) {
            double q = a[k * n + t];
            a[k * n + t] = a[bi * n + t];
            a[bi * n + t] = q;
        }
        wave_lds_sync();
        const double inv_p = 1.0 / a[k * n + k];
        if (t > k && t < n) {
            const double l = a[t * n + k] * inv_p;
            a[t * n + k] = l;
            for (int j = k + 1; j < n; ++j) a[t * n + j] -= l * a[k * n + j];
        }
        wave_lds_sync();
    }
    for (int e = t; e < n * n; e += 64) g[e] = a[e];
    // inverse: lane j solves K x = e_j
    if (t < n) {
        for (int i = 0; i < n; ++i) x[i * n + t] = (i == t) ? 1.0 : 0.0;
        for (int k = 0; k < n; ++k) {
            const int p = spv[k];
            if (p != k) {
                double q = x[k * n + t];
                x[k * n + t] = x[p * n + t];
                x[p * n + t] = q;
            }
        }
        for (int k = 0; k < n; ++k) {
            const double xk = x[k * n + t];
            for (int i = k + 1; i < n; ++i) x[i * n + t] -= a[i * n + k] * xk;
        }
        for (int k = n - 1; k >= 0; --k) {
            const double xk = x[k * n + t] / a[k * n + k];
            x[k * n + t] = xk;
            for (int i = 0; i < k; ++i) x[i * n + t] -= a[i * n + k] * xk;
        }
    }
    wave_lds_sync();
    double *o = inv + doff[s];
    for (int e = t; e < n * n; e += 64) o[e] = x[e];
}

void launch_block_lu_inv_small(int32_t nsys, const int64_t *seg, const int64_t *doff,
                               double *dense, int32_t *piv, double *inv, int32_t *info,
                               hipStream_t s) {
    LAIR_LAUNCH(k_block_lu_inv_small, dim3(nsys), dim3(64), 0, s, seg, doff, dense, piv, inv,
                info);
    LAIR_LAUNCH_CHECK();
}

int32_t small_dense_max() { return SMALL_DENSE; }

// Inverse of a block of 65..256 rows from its LU factors (P K = L U): one
// wave per chunk of 32 columns of the inverse (blockIdx.y), the chunk held in
// LDS (at most 256 x 32 doubles).  Lanes take a column each and one of two
// row parities; rows of L and U are read from global memory.
constexpr int MID_DENSE = 256, MID_COLS = 32;

__global__ void __launch_bounds__(64)
k_block_inv_mid(const int64_t *seg, const int64_t *doff, const double *__restrict__ lu,
                const int32_t *piv, double *__restrict__ inv, const uint8_t *use_inv) {
    __shared__ double y[MID_DENSE * MID_COLS];
    const int32_t s = blockIdx.x;
    if (!use_inv[s]) return;
    const int n = (int)(seg[s + 1] - seg[s]);
    if (n <= SMALL_DENSE || n > MID_DENSE) return;
    const int j0 = blockIdx.y * MID_COLS;
    if (j0 >= n) return;
    const int c = threadIdx.x % MID_COLS, par = threadIdx.x / MID_COLS;
    const double *a = lu + doff[s];
    const int32_t *pv = piv + seg[s];
    // column j0 + c of P: where the row swaps take e_j
    int pos = j0 + c;
    for (int k = 0; k < n; ++k) {
        const int p = pv[k];
        if (pos == k) pos = p;
        else if (pos == p) pos = k;
    }
    for (int i = par; i < n; i += 2) y[i * MID_COLS + c] = (i == pos) ? 1.0 : 0.0;
    wave_lds_sync();
    for (int k = 0; k < n; ++k) {                     // L Y = P E
        const double yk = y[k * MID_COLS + c];
#pragma unroll 4
        for (int i = k + 1 + par; i < n; i += 2) y[i * MID_COLS + c] -= a[(size_t)i * n + k] * yk;
        wave_lds_sync();
    }
    for (int k = n - 1; k >= 0; --k) {                // U X = Y
        if (par == 0) y[k * MID_COLS + c] /= a[(size_t)k * n + k];
        wave_lds_sync();
        const double xk = y[k * MID_COLS + c];
#pragma unroll 4
        for (int i = par; i < k; i += 2) y[i * MID_COLS + c] -= a[(size_t)i * n + k] * xk;
        wave_lds_sync();
    }
    double *o = inv + doff[s];
    if (j0 + c < n)
        for (int i = par; i < n; i += 2) o[(size_t)i * n + j0 + c] = y[i * MID_COLS + c];
}

void launch_block_inv_mid(int32_t nsys, int32_t maxn, const int64_t *seg, const int64_t *doff,
                          const double *lu, const int32_t *piv, double *inv,
                          const uint8_t *use_inv, hipStream_t s) {
    const int gy = (maxn + MID_COLS - 1) / MID_COLS;
    LAIR_LAUNCH(k_block_inv_mid, dim3(nsys, gy), dim3(64), 0, s, seg, doff, lu, piv, inv,
                use_inv);
    LAIR_LAUNCH_CHECK();
}

int32_t mid_dense_max() { return MID_DENSE; }

// x_s = K_s^{-1} b_s (or K_s^{-T} b_s) with the explicit inverses, one
// block per system: a wave per row of the inverse (coalesced), or for the
// transpose a thread per column.
__global__ void __launch_bounds__(256)
k_block_apply_inv(const int64_t *seg, const int64_t *doff, const double *inv, const double *b,
                  double *x, int transpose, const uint8_t *active, const uint8_t *use_inv) {
    const int32_t s = blockIdx.x;
    if ((active && !active[s]) || !use_inv[s]) return;
    const int n = (int)(seg[s + 1] - seg[s]);
    const double *m = inv + doff[s];
    const double *bs = b + seg[s];
    double *xs = x + seg[s];
    if (transpose) {
        for (int i = threadIdx.x; i < n; i += blockDim.x) {
            double acc = 0.0;
            for (int j = 0; j < n; ++j) acc += m[(size_t)j * n + i] * bs[j];
            xs[i] = acc;
        }
        return;
    }
    const int lane = threadIdx.x & (WAVE - 1), wv = threadIdx.x / WAVE;
    const int nw = blockDim.x / WAVE;
    for (int i = wv; i < n; i += nw) {
        double acc = 0.0;
        for (int j = lane; j < n; j += WAVE) acc += m[(size_t)i * n + j] * bs[j];
        acc = team_sum<WAVE>(acc);
        if (lane == 0) xs[i] = acc;
    }
}

void launch_block_apply_inv(int32_t nsys, const int64_t *seg, const int64_t *doff,
                            const double *inv, const double *b, double *x, bool transpose,
                            hipStream_t s, const uint8_t *active, const uint8_t *use_inv) {
    LAIR_LAUNCH(k_block_apply_inv, dim3(nsys), dim3(256), 0, s, seg, doff, inv, b, x,
                transpose ? 1 : 0, active, use_inv);
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
           int32_t *info, int32_t min_n) {
    __shared__ double sv[256];
    __shared__ int si[256];
    int32_t s = blockIdx.x;
    int t = threadIdx.x;
    const int n = (int)(seg[s + 1] - seg[s]);
    if (n < min_n) return;
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

// x = K_s^{-1} b (or K_s^{-T} b) for every system from its LU factors, one
// wave per system: the unknowns sit in LDS and every substitution step is
// a row-times-vector product over the wave (coalesced reads of a row of L,
// U, or for the transpose of a column), so the only synchronisation is the
// wave's own.  Systems applied by an explicit inverse are skipped.
constexpr int SOLVE_LDS = 4096;     // unknowns per system held in LDS (= the size limit)

__global__ void __launch_bounds__(64)
k_block_solve(const int64_t *seg, const int64_t *doff, const double *dense,
              const int32_t *piv, const double *b, double *x, int transpose,
              const uint8_t *active, const uint8_t *skip) {
    __shared__ double xs[SOLVE_LDS];
    const int32_t s = blockIdx.x;
    if ((active && !active[s]) || (skip && skip[s])) return;
    const int n = (int)(seg[s + 1] - seg[s]);
    const int lane = threadIdx.x;
    const double *a = dense + doff[s];
    const int32_t *pv = piv + seg[s];
    const double *bs = b + seg[s];
    for (int i = lane; i < n; i += WAVE) xs[i] = bs[i];
    wave_lds_sync();
    if (!transpose) {
        if (lane == 0)
            for (int k = 0; k < n; ++k)
                if (pv[k] != k) { double q = xs[k]; xs[k] = xs[pv[k]]; xs[pv[k]] = q; }
        wave_lds_sync();
        for (int r = 1; r < n; ++r) {               // L y = P b (unit diagonal)
            double acc = 0.0;
            for (int k = lane; k < r; k += WAVE) acc += a[(size_t)r * n + k] * xs[k];
            acc = team_sum<WAVE>(acc);
            if (lane == 0) xs[r] -= acc;
            wave_lds_sync();
        }
        for (int r = n - 1; r >= 0; --r) {          // U x = y
            double acc = 0.0;
            for (int k = r + 1 + lane; k < n; k += WAVE) acc += a[(size_t)r * n + k] * xs[k];
            acc = team_sum<WAVE>(acc);
            if (lane == 0) xs[r] = (xs[r] - acc) / a[(size_t)r * n + r];
            wave_lds_sync();
        }
    } else {
        for (int r = 0; r < n; ++r) {               // U^T y = b
            double acc = 0.0;
            for (int k = lane; k < r; k += WAVE) acc += a[(size_t)k * n + r] * xs[k];
            acc = team_sum<WAVE>(acc);
            if (lane == 0) xs[r] = (xs[r] - acc) / a[(size_t)r * n + r];
            wave_lds_sync();
        }
        for (int r = n - 2; r >= 0; --r) {          // L^T z = y (unit diagonal)
            double acc = 0.0;
            for (int k = r + 1 + lane; k < n; k += WAVE) acc += a[(size_t)k * n + r] * xs[k];
            acc = team_sum<WAVE>(acc);
            if (lane == 0) xs[r] -= acc;
            wave_lds_sync();
        }
        if (lane == 0)                               // x = P^T z
            for (int k = n - 1; k >= 0; --k)
                if (pv[k] != k) { double q = xs[k]; xs[k] = xs[pv[k]]; xs[pv[k]] = q; }
        wave_lds_sync();
    }
    double *xo = x + seg[s];
    for (int i = lane; i < n; i += WAVE) xo[i] = xs[i];
}

void launch_dense_blocks(int32_t nsys, const int64_t *seg, const int64_t *doff,
                         const int32_t *rp, const int32_t *cj, const double *v,
                         double *dense, int64_t nrows, hipStream_t s) {
    LAIR_LAUNCH(k_dense_blocks, dim3(blocks_for(nrows, 64)), dim3(64), 0, s,
                       nsys, seg, doff, rp, cj, v, dense, nrows);
    LAIR_LAUNCH_CHECK();
}

void launch_block_lu(int32_t nsys, const int64_t *seg, const int64_t *doff, double *dense,
                     int32_t *piv, int32_t *info, hipStream_t s, int32_t min_n) {
    LAIR_LAUNCH(k_block_lu, dim3(nsys), dim3(256), 0, s, seg, doff, dense, piv, info, min_n);
    LAIR_LAUNCH_CHECK();
}

void launch_block_solve(int32_t nsys, const int64_t *seg, const int64_t *doff,
                        const double *dense, const int32_t *piv, const double *b, double *x,
                        bool transpose, hipStream_t s, const uint8_t *active,
                        const uint8_t *skip) {
    LAIR_LAUNCH(k_block_solve, dim3(nsys), dim3(64), 0, s, seg, doff, dense, piv, b, x,
                       transpose ? 1 : 0, active, skip);
    LAIR_LAUNCH_CHECK();
}

}  // namespace lair
