// Setup kernels of the lAIR hierarchy on gfx950 (wave64).
//
//   validate / strength     one team of lanes per row
//   scan                    three-phase tile scan (counts -> offsets)
//   neighbourhoods          one team per C-point; distance 2 is a k-way
//                           merge of sorted strong-F lists (F-F-C paths)
//   local solves            Eq. (system): M = A(N,N)^T, f = -A(i,N)^T,
//                           partial-pivot LU; small systems one lane each in
//                           registers, larger ones one wave each in LDS (or
//                           global scratch beyond the LDS limit); singular
//                           systems take the minimal-norm least-squares
//                           solution by one-sided Jacobi SVD
//   interpolation           one-point and classical direct, one lane per row
//   sparse product          row-merge: one team per output row merges the
//                           sorted rows of B selected by a row of A
//   transpose, coarsest LU  support for the cycle and its adjoint
#include <algorithm>
#include <array>
#include <cfloat>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>
#include <type_traits>
#include <vector>

#include "k_common.hpp"
#include "lair_internal.hpp"

namespace lair {

// ===========================================================================
// Scan: out[i] = sum_{j<i} f(j), out[n] = total.
// ===========================================================================
constexpr int SCAN_BS = 256;
constexpr int SCAN_IPT = 8;
constexpr int SCAN_TILE = SCAN_BS * SCAN_IPT;

struct CountsF {
    const int32_t *c;
    __device__ int64_t operator()(int64_t i) const { return c[i]; }
};
struct FlagsF {
    const int8_t *f;
    int8_t want;
    __device__ int64_t operator()(int64_t i) const { return f[i] == want ? 1 : 0; }
};
// length of row map[k] of a CSR matrix (map == nullptr: row k)
struct RowLenF {
    const int32_t *rp, *map;
    __device__ int64_t operator()(int64_t k) const {
        const int64_t r = map ? map[k] : k;
        return rp[r + 1] - rp[r];
    }
};

// Longer inputs in two launches.  k_scan_reduce writes the sum and the
// largest value of every tile of SCAN_TILE entries; k_scan_down gives each
// tile its offset by summing the sums of the tiles before it (the block's
// threads share the reads) and writes the tile's offsets.  The last tile
// also writes out[n], the total and the largest value.
__device__ __forceinline__ int64_t block_scan_threads(int64_t v, int64_t *s_w, int64_t &total) {
    // exclusive scan of one value per thread over a block of SCAN_BS threads
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    int64_t inc = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int64_t u = __shfl_up(inc, o);
        if (lane >= o) inc += u;
    }
    if (lane == 63) s_w[w] = inc;
    __syncthreads();
    int64_t pre = inc - v;
    total = 0;
#pragma unroll
    for (int k = 0; k < SCAN_BS / 64; ++k) {
        if (k < w) pre += s_w[k];
        total += s_w[k];
    }
    __syncthreads();
    return pre;
}

__device__ __forceinline__ int64_t block_sum_threads(int64_t v, int64_t *s_w) {
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    if (lane == 0) s_w[w] = v;
    __syncthreads();
    int64_t r = 0;
#pragma unroll
    for (int k = 0; k < SCAN_BS / 64; ++k) r += s_w[k];
    __syncthreads();
    return r;
}

__device__ __forceinline__ int64_t block_max_threads(int64_t v, int64_t *s_w) {
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const int64_t u = __shfl_xor(v, o);
        v = u > v ? u : v;
    }
    if (lane == 0) s_w[w] = v;
    __syncthreads();
    int64_t r = 0;
#pragma unroll
    for (int k = 0; k < SCAN_BS / 64; ++k) r = s_w[k] > r ? s_w[k] : r;
    __syncthreads();
    return r;
}

template <class F>
__global__ void __launch_bounds__(SCAN_BS)
k_scan_reduce(F f, int64_t n, int64_t *blocksum, int64_t *blockmax) {
    __shared__ int64_t s_w[SCAN_BS / 64];
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_IPT;
    int64_t sum = 0, mx = 0;
#pragma unroll
    for (int j = 0; j < SCAN_IPT; ++j) {
        const int64_t i = base + j;
        const int64_t v = (i < n) ? f(i) : 0;
        sum += v;
        mx = v > mx ? v : mx;
    }
    sum = block_sum_threads(sum, s_w);
    mx = block_max_threads(mx, s_w);
    if (threadIdx.x == 0) {
        blocksum[blockIdx.x] = sum;
        blockmax[blockIdx.x] = mx;
    }
}

template <class F, class OUT>
__global__ void __launch_bounds__(SCAN_BS)
k_scan_down(F f, int64_t n, int64_t nb, const int64_t *blocksum, const int64_t *blockmax,
            OUT *out, int64_t *tot) {
    __shared__ int64_t s_w[SCAN_BS / 64];
    const int64_t b = blockIdx.x;
    // this tile's offset: the sums of the tiles before it
    int64_t part = 0;
    for (int64_t k = threadIdx.x; k < b; k += SCAN_BS) part += blocksum[k];
    const int64_t off = block_sum_threads(part, s_w);
    const int64_t base = b * SCAN_TILE + (int64_t)threadIdx.x * SCAN_IPT;
    int64_t v[SCAN_IPT];
    int64_t sum = 0;
#pragma unroll
    for (int j = 0; j < SCAN_IPT; ++j) {
        const int64_t i = base + j;
        v[j] = (i < n) ? f(i) : 0;
        sum += v[j];
    }
    int64_t tile_total;
    int64_t pre = off + block_scan_threads(sum, s_w, tile_total);
#pragma unroll
    for (int j = 0; j < SCAN_IPT; ++j) {
        const int64_t i = base + j;
        if (i < n) out[i] = (OUT)pre;
        pre += v[j];
    }
    if (b == nb - 1) {
        int64_t mx = 0;
        for (int64_t k = threadIdx.x; k < nb; k += SCAN_BS)
            mx = blockmax[k] > mx ? blockmax[k] : mx;
        mx = block_max_threads(mx, s_w);
        if (threadIdx.x == 0) {
            out[n] = (OUT)(off + tile_total);
            tot[0] = off + tile_total;
            tot[1] = mx;
        }
    }
}

// ===========================================================================
// Caller's CF splittings in device memory: every value 0 or 1 (else bad[0]
// is set), with k > 1 every node's k entries alike (else bad[0]), and the
// C-points of every level counted into cnt[l] (int64).  offs: nlevels + 1
// level offsets.  The lanes of a wave that lie in the level of the wave's
// first entry add their count with one atomic; the others (a wave across a
// level boundary) add one by one.
// ===========================================================================
constexpr int CF_LDS_LEVELS = 64;

__global__ void __launch_bounds__(256)
k_cf_check(int32_t nlevels, const int64_t *offs, const int8_t *cf, int32_t k, int64_t *cnt,
           int32_t *bad) {
    __shared__ unsigned long long s_cnt[CF_LDS_LEVELS];
    for (int l = threadIdx.x; l < CF_LDS_LEVELS; l += blockDim.x) s_cnt[l] = 0;
    __syncthreads();
    const int64_t total = offs[nlevels];
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t rounds = (total + stride - 1) / stride;
    int any_bad = 0;
    for (int64_t r = 0; r < rounds; ++r) {
        const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x + r * stride;
        const bool in = q < total;
        int lev = 0;
        int8_t v = 0;
        if (in) {
            while (lev + 1 < nlevels && offs[lev + 1] <= q) ++lev;
            v = cf[q];
            bool b = (v & ~1) != 0;
            if (k > 1) {
                const int64_t lo = offs[lev];
                b = b || v != cf[lo + (q - lo) / k * k];
            }
            any_bad |= b ? 1 : 0;
        }
        // the lanes in the level of the wave's first entry: one LDS add
        const int first = __shfl(lev, 0);
        const bool same = in && lev == first;
        const uint64_t ones = __ballot(same && v == 1);
        if ((threadIdx.x & (WAVE - 1)) == 0 && ones) {
            if (first < CF_LDS_LEVELS) atomicAdd(&s_cnt[first], (unsigned long long)__popcll(ones));
            else atomicAdd((unsigned long long *)&cnt[first], (unsigned long long)__popcll(ones));
        }
        if (in && !same && v == 1) {
            if (lev < CF_LDS_LEVELS) atomicAdd(&s_cnt[lev], 1ull);
            else atomicAdd((unsigned long long *)&cnt[lev], 1ull);
        }
    }
    if (any_bad) atomicOr(bad, 1);
    __syncthreads();
    for (int l = threadIdx.x; l < CF_LDS_LEVELS && l < nlevels; l += blockDim.x)
        if (s_cnt[l]) atomicAdd((unsigned long long *)&cnt[l], s_cnt[l]);
}

void launch_cf_check(int32_t nlevels, const int64_t *offs_dev, int64_t total, const int8_t *cf,
                     int32_t k, int64_t *cnt, int32_t *bad, hipStream_t s) {
    if (total <= 0) return;
    const unsigned grid = std::min<unsigned>(blocks_for(total, 256), 1024u);
    LAIR_LAUNCH(k_cf_check, dim3(grid), dim3(256), 0, s, nlevels, offs_dev, cf, k, cnt, bad);
    LAIR_LAUNCH_CHECK();
}

// Short inputs in one launch: one block of SCAN1_BS threads, each thread
// scanning ipt consecutive entries (read twice: sums, then offsets), the
// waves' sums combined through LDS.
constexpr int SCAN1_BS = 1024;
constexpr int64_t SCAN1_MAX = 16 * SCAN1_BS;

template <class F, class OUT>
__global__ void __launch_bounds__(SCAN1_BS)
k_scan_one(F f, int64_t n, int ipt, OUT *out, int64_t *tot) {
    __shared__ int64_t s_sum[SCAN1_BS / 64], s_max[SCAN1_BS / 64];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int64_t b0 = (int64_t)t * ipt;
    int64_t sum = 0, mx = 0;
    for (int j = 0; j < ipt; ++j) {
        const int64_t i = b0 + j;
        if (i < n) {
            const int64_t v = f(i);
            sum += v;
            mx = v > mx ? v : mx;
        }
    }
    int64_t inc = sum;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int64_t u = __shfl_up(inc, o);
        if (lane >= o) inc += u;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const int64_t u = __shfl_xor(mx, o);
        mx = u > mx ? u : mx;
    }
    if (lane == 63) s_sum[w] = inc;
    if (lane == 0) s_max[w] = mx;
    __syncthreads();
    int64_t pre = inc - sum, total = 0, big = 0;
    for (int k = 0; k < SCAN1_BS / 64; ++k) {
        if (k < w) pre += s_sum[k];
        total += s_sum[k];
        big = s_max[k] > big ? s_max[k] : big;
    }
    for (int j = 0; j < ipt; ++j) {
        const int64_t i = b0 + j;
        if (i < n) {
            out[i] = (OUT)pre;
            pre += f(i);
        }
    }
    if (t == 0) {
        out[n] = (OUT)total;
        tot[0] = total;
        tot[1] = big;
    }
}

// Launches only: out[0..n] and tot[0] = total, tot[1] = largest value on
// the device.
template <class F, class OUT>
static int64_t *scan_launch(F f, OUT *out, int64_t n, hipStream_t s, DevArr<int64_t> &tmp,
                            int64_t *tot_out = nullptr) {
    if (n <= SCAN1_MAX) {
        int64_t *tot = tot_out;
        if (!tot) {
            tmp.ensure(2, s);
            tot = tmp.get();
        }
        const int ipt = (int)((n + SCAN1_BS - 1) / SCAN1_BS);
        LAIR_LAUNCH((k_scan_one<F, OUT>), dim3(1), dim3(SCAN1_BS), 0, s, f, n, ipt, out, tot);
        LAIR_LAUNCH_CHECK();
        return tot;
    }
    int64_t nb = (n + SCAN_TILE - 1) / SCAN_TILE;
    if (nb < 1) nb = 1;
    tmp.ensure((size_t)2 * nb + 2, s);
    int64_t *bs = tmp.get();
    int64_t *bmax = bs + nb;
    // tot[0] = total, tot[1] = largest value (in tmp, or where the caller
    // keeps them for a later readback)
    int64_t *tot = tot_out ? tot_out : bmax + nb;
    LAIR_LAUNCH((k_scan_reduce<F>), dim3((unsigned)nb), dim3(SCAN_BS), 0, s, f, n, bs, bmax);
    LAIR_LAUNCH_CHECK();
    LAIR_LAUNCH((k_scan_down<F, OUT>), dim3((unsigned)nb), dim3(SCAN_BS), 0, s, f, n, nb, bs,
                bmax, out, tot);
    LAIR_LAUNCH_CHECK();
    return tot;
}

template <class F, class OUT>
static int64_t scan_impl(F f, OUT *out, int64_t n, hipStream_t s,
                         DevArr<int64_t> &tmp, int64_t *max_out,
                         const int32_t *flag, int32_t *flag_out) {
    int64_t *tot = scan_launch(f, out, n, s, tmp);
    int64_t h[2] = {0, 0};
    Readback rb(s);
    rb.add(h, tot, sizeof(h));
    if (flag && flag_out) rb.add(flag_out, flag, sizeof(int32_t));
    rb.run();
    if (sizeof(OUT) == 4 && h[0] > INT32_MAX)
        fail(LAIR_EUNSUPPORTED, "offset array exceeds 2^31 entries (%lld)",
             (long long)h[0]);
    if (max_out) *max_out = h[1];
    return h[0];
}

void scan_counts_i32_to(const int32_t *cnt, int32_t *out, int64_t n, hipStream_t s,
                        DevArr<int64_t> &tmp, int64_t *tot) {
    scan_launch(CountsF{cnt}, out, n, s, tmp, tot);
}

void scan_counts_i64_to(const int32_t *cnt, int64_t *out, int64_t n, hipStream_t s,
                        DevArr<int64_t> &tmp, int64_t *tot) {
    scan_launch(CountsF{cnt}, out, n, s, tmp, tot);
}

void scan_flags_i8_to(const int8_t *flags, int8_t want, int32_t *out, int64_t n, hipStream_t s,
                      DevArr<int64_t> &tmp, int64_t *tot) {
    scan_launch(FlagsF{flags, want}, out, n, s, tmp, tot);
}

int64_t scan_counts_i32(const int32_t *cnt, int32_t *out, int64_t n,
                        hipStream_t s, DevArr<int64_t> &tmp, int64_t *max_out,
                        const int32_t *flag, int32_t *flag_out) {
    return scan_impl(CountsF{cnt}, out, n, s, tmp, max_out, flag, flag_out);
}

int64_t scan_counts_i64(const int32_t *cnt, int64_t *out, int64_t n, hipStream_t s,
                        DevArr<int64_t> &tmp, int64_t *max_out) {
    return scan_impl(CountsF{cnt}, out, n, s, tmp, max_out, nullptr, nullptr);
}

int64_t scan_flags_i8(const int8_t *flags, int8_t want, int32_t *out, int64_t n,
                      hipStream_t s, DevArr<int64_t> &tmp) {
    return scan_impl(FlagsF{flags, want}, out, n, s, tmp, nullptr, nullptr, nullptr);
}

// ===========================================================================
// CSR validation.  Error bits: 1 bad row pointers, 2 column out of range,
// 4 columns not strictly increasing, 8 non-finite value, 16 zero diagonal,
// 32 missing diagonal.  stat[1] receives the longest row.
// ===========================================================================
// Team of VT lanes per row (lanes take every VT-th entry); each block
// writes its error bits and longest row to part[2 b], part[2 b + 1], and one
// block combines the partials (no contended atomics).
constexpr int VT = 8;

__global__ void __launch_bounds__(256)
k_validate(int64_t n, int64_t nnz, const int32_t *rp, const int32_t *cj,
           const double *v, int32_t *part) {
    __shared__ int se[256], sm[256];
    // a fixed grid, rows taken grid-stride (few partial results to combine)
    const int64_t gt = xcd_block_id() * blockDim.x + threadIdx.x;
    const int lane = (int)(gt % VT);
    const int64_t nteam = (int64_t)gridDim.x * blockDim.x / VT;
    int err = 0, len = 0;
    if (gt == 0 && (rp[0] != 0 || (int64_t)rp[n] != nnz)) err = 1;
    const int64_t rounds = (n + nteam - 1) / nteam;
    for (int64_t k = 0; k < rounds; ++k) {
        const int64_t i = gt / VT + k * nteam;
        bool diag = false;
        if (i < n) {
            int64_t lo = rp[i], hi = rp[i + 1];
            if (lo < 0 || hi < lo || hi > nnz) {
                err |= 1;
                diag = true;        // reported as bad row pointers only
            } else {
                for (int64_t p = lo + lane; p < hi; p += VT) {
                    int c = cj[p];
                    if (c < 0 || c >= n) err |= 2;
                    if (p > lo && c <= cj[p - 1]) err |= 4;
                    double a = v[p];
                    if (!isfinite(a)) err |= 8;
                    if (c == i) { diag = true; if (a == 0.0) err |= 16; }
                }
                len = max(len, (int)(hi - lo));
            }
        } else {
            diag = true;
        }
        if (team_bits<VT>(diag) == 0 && lane == 0) err |= 32;
    }
    se[threadIdx.x] = err;
    sm[threadIdx.x] = len;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            se[threadIdx.x] |= se[threadIdx.x + o];
            sm[threadIdx.x] = max(sm[threadIdx.x], sm[threadIdx.x + o]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = se[0];
        part[2 * blockIdx.x + 1] = sm[0];
    }
}

__global__ void __launch_bounds__(256)
k_validate_final(const int32_t *part, int64_t nb, int32_t *stat) {
    __shared__ int se[256], sm[256];
    int e = 0, m = 0;
    for (int64_t b = threadIdx.x; b < nb; b += 256) {
        e |= part[2 * b];
        m = max(m, part[2 * b + 1]);
    }
    se[threadIdx.x] = e;
    sm[threadIdx.x] = m;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            se[threadIdx.x] |= se[threadIdx.x + o];
            sm[threadIdx.x] = max(sm[threadIdx.x], sm[threadIdx.x + o]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) { stat[0] = se[0]; stat[1] = sm[0]; }
}

int32_t validate_csr(int64_t n, int64_t nnz, const int32_t *rp,
                     const int32_t *cj, const double *v, hipStream_t s) {
    const unsigned nb = std::min<unsigned>(blocks_for(n * VT, 256), 2048u);
    DevArr<int32_t> st;
    st.alloc(2 + 2 * (size_t)nb, s);
    ProfScope ps("validate", s, 12.0 * nnz + 4.0 * (n + 1));
    LAIR_LAUNCH(k_validate, dim3(nb), dim3(256), 0, s, n, nnz, rp, cj, v,
                       st.get() + 2);
    LAIR_LAUNCH_CHECK();
    LAIR_LAUNCH(k_validate_final, dim3(1), dim3(256), 0, s, st.get() + 2, (int64_t)nb,
                       st.get());
    LAIR_LAUNCH_CHECK();
    int32_t h[2];
    {
        Readback rb(s);
        rb.add(h, st.get(), sizeof(h));
        rb.run();
    }
    if (h[0]) {
        fail(LAIR_EINVAL, "invalid CSR matrix (error bits 0x%x: %s%s%s%s%s%s)", h[0],
             (h[0] & 1) ? "row pointers " : "", (h[0] & 2) ? "column range " : "",
             (h[0] & 4) ? "unsorted/duplicate columns " : "",
             (h[0] & 8) ? "non-finite values " : "",
             (h[0] & 16) ? "zero diagonal " : "",
             (h[0] & 32) ? "missing diagonal" : "");
    }
    return h[1];
}

// ===========================================================================
// Strength of connection (Sec. 4).  j is strong for i iff j != i, a_ij != 0,
// m_i = max_{k!=i} |a_ik| > 0 and |a_ij| (ABS) or -a_ij (NEG) >= theta m_i.
// ===========================================================================
template <int T>
__global__ void k_strength(int32_t n, const int32_t *rp, const int32_t *cj,
                           const double *v, double theta, int32_t kind,
                           uint8_t *smask) {
    int64_t gt = xcd_block_id() * blockDim.x + threadIdx.x;
    int32_t i = (int32_t)(gt / T);
    int lane = (int)(gt % T);
    if (i >= n) return;
    int lo = rp[i], hi = rp[i + 1];
    double m = 0.0;
    for (int p = lo + lane; p < hi; p += T)
        if (cj[p] != i) m = fmax(m, fabs(v[p]));
    m = team_max<T>(m);
    double thr = theta * m;
    for (int p = lo + lane; p < hi; p += T) {
        double a = v[p];
        bool s = (cj[p] != i) && (a != 0.0) && (m > 0.0) &&
                 (((kind == LAIR_SOC_NEG) ? -a : fabs(a)) >= thr);
        smask[p] = s ? 1 : 0;
    }
}

template <int T>
static void strength_t(int32_t n, const int32_t *rp, const int32_t *cj,
                       const double *v, double theta, int32_t kind,
                       uint8_t *smask, hipStream_t s) {
    LAIR_LAUNCH(k_strength<T>, dim3(blocks_for((int64_t)n * T, 256)),
                       dim3(256), 0, s, n, rp, cj, v, theta, kind, smask);
    LAIR_LAUNCH_CHECK();
}

void launch_strength(int32_t n, const int32_t *rp, const int32_t *cj,
                     const double *v, double theta, int32_t kind,
                     uint8_t *smask, double mean_len, hipStream_t s) {
    int t = team_for_mean(mean_len / 2.0);
    double nnz = mean_len * n;
    ProfScope ps("strength", s, 13.0 * nnz + 4.0 * (n + 1));
    switch (t) {
        case 2: strength_t<2>(n, rp, cj, v, theta, kind, smask, s); break;
        case 4: strength_t<4>(n, rp, cj, v, theta, kind, smask, s); break;
        case 8: strength_t<8>(n, rp, cj, v, theta, kind, smask, s); break;
        case 16: strength_t<16>(n, rp, cj, v, theta, kind, smask, s); break;
        case 32: strength_t<32>(n, rp, cj, v, theta, kind, smask, s); break;
        default: strength_t<64>(n, rp, cj, v, theta, kind, smask, s); break;
    }
}

// ===========================================================================
// Coarse numbering (C-points in increasing fine index) and row lists.
// ===========================================================================
__global__ void __launch_bounds__(256)
k_cf_lists(int32_t n, const int8_t *cf, const int32_t *scan, const int32_t *rp,
           int32_t *cidx, int32_t *clist, int32_t *flist,
           unsigned long long *acc) {
    __shared__ unsigned long long sf[256], sc[256];
    int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    unsigned long long nf = 0, ncc = 0;
    if (i < n) {
        int32_t c = scan[i];
        unsigned long long len = (unsigned long long)(rp[i + 1] - rp[i]);
        if (cf[i] == 1) {
            cidx[i] = c;
            clist[c] = i;
            ncc = len;
        } else {
            cidx[i] = -1;
            flist[i - c] = i;
            nf = len;
        }
    }
    sf[threadIdx.x] = nf;
    sc[threadIdx.x] = ncc;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            sf[threadIdx.x] += sf[threadIdx.x + o];
            sc[threadIdx.x] += sc[threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        acc[2 * blockIdx.x] = sf[0];
        acc[2 * blockIdx.x + 1] = sc[0];
    }
}

// Fixed-order sum of nb pairs of block partials into out[0], out[1].
__global__ void __launch_bounds__(256)
k_sum_pairs(const unsigned long long *part, int64_t nb, unsigned long long *out) {
    __shared__ unsigned long long s0[256], s1[256];
    unsigned long long a = 0, b = 0;
    for (int64_t k = threadIdx.x; k < nb; k += 256) {
        a += part[2 * k];
        b += part[2 * k + 1];
    }
    s0[threadIdx.x] = a;
    s1[threadIdx.x] = b;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            s0[threadIdx.x] += s0[threadIdx.x + o];
            s1[threadIdx.x] += s1[threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) { out[0] = s0[0]; out[1] = s1[0]; }
}

// acc: 2 + 2 * ceil(n / 256) entries; acc[0], acc[1] receive the entries of
// the F rows and of the C rows.
void launch_cf_lists(int32_t n, const int8_t *cf, const int32_t *cidx_scan,
                     const int32_t *rp, int32_t *cidx, int32_t *clist,
                     int32_t *flist, unsigned long long *acc, hipStream_t s) {
    const unsigned nb = blocks_for(n, 256);
    LAIR_LAUNCH(k_cf_lists, dim3(nb), dim3(256), 0, s,
                       n, cf, cidx_scan, rp, cidx, clist, flist, acc + 2);
    LAIR_LAUNCH_CHECK();
    LAIR_LAUNCH(k_sum_pairs, dim3(1), dim3(256), 0, s, acc + 2, (int64_t)nb, acc);
    LAIR_LAUNCH_CHECK();
}

// ===========================================================================
// Restriction neighbourhoods N_i (Sec. 3.1; F-F-C paths at distance two,
// Sec. 4).  One team of T lanes per C-point.  Distance 1 compacts the strong
// F entries of row i (already sorted).  Distance 2 merges the sorted lists
// {row i} and {row j : j strong F-neighbour of i}, each filtered to strong
// F entries; list k belongs to lane k % T, slot k / T (LPL slots per lane).
// ===========================================================================
constexpr int NBR_LPL = 4;

__device__ __forceinline__ bool nbr_ok(const uint8_t *sm, const int8_t *cf,
                                       const int32_t *cj, int p) {
    return sm[p] && cf[cj[p]] == 0;
}

template <int T>
__global__ void k_nbr(int32_t nc, const int32_t *clist, const int32_t *rp,
                      const int32_t *cj, const uint8_t *sm, const int8_t *cf,
                      int32_t distance, const int32_t *flist, int32_t nf,
                      bool fill, int32_t *cnt, const int32_t *nptr,
                      int32_t *nbr, int32_t *overflow, int32_t knode) {
    // knode > 1 (nodal levels): the knode consecutive C rows of a C-node
    // share their neighbourhood (the strength mask is node-expanded), so one
    // team merges it once, from the node's first row, and writes it for each
    int64_t gt = xcd_block_id() * blockDim.x + threadIdx.x;
    int32_t c = (int32_t)(gt / T) * knode;
    int lane = (int)(gt % T);
    if (c >= nc) return;
    if (distance == LAIR_DIST_ALL_F) {
        for (int32_t a = 0; a < knode; ++a) {
            if (fill)
                for (int q = lane; q < nf; q += T) nbr[nptr[c + a] + q] = flist[q];
            else if (lane == 0)
                cnt[c + a] = nf;
        }
        return;
    }
    int32_t i = clist[c];
    int lo = rp[i], hi = rp[i + 1];
    if (distance == 1) {
        int o = 0;
        for (int p0 = lo; p0 < hi; p0 += T) {
            int p = p0 + lane;
            bool q = (p < hi) && nbr_ok(sm, cf, cj, p);
            uint64_t bits = team_bits<T>(q);
            int before = __popcll(bits & ((1ull << lane) - 1ull));
            if (fill && q)
                for (int32_t a = 0; a < knode; ++a) nbr[nptr[c + a] + o + before] = cj[p];
            o += __popcll(bits);
        }
        if (!fill && lane == 0)
            for (int32_t a = 0; a < knode; ++a) cnt[c + a] = o;
        return;
    }
    // distance 2: assign lists to (lane, slot)
    int pos[NBR_LPL], end[NBR_LPL], head[NBR_LPL];
#pragma unroll
    for (int m = 0; m < NBR_LPL; ++m) { pos[m] = 0; end[m] = 0; head[m] = INT_MAX; }
    int k = 1;                // list 0 is row i itself
    bool over = false;
    if (lane == 0) { pos[0] = lo; end[0] = hi; }
    for (int p = lo; p < hi; ++p) {
        if (!nbr_ok(sm, cf, cj, p)) continue;
        if ((k % T) == lane) {
            int m = k / T;
            if (m >= NBR_LPL) {
                over = true;
            } else {
                int j = cj[p];
#pragma unroll
                for (int mm = 0; mm < NBR_LPL; ++mm)
                    if (mm == m) { pos[mm] = rp[j]; end[mm] = rp[j + 1]; }
            }
        }
        ++k;
    }
    if (k > T * NBR_LPL) {
        if (lane == 0) atomicOr(overflow, 1);
        if (!fill && lane == 0)
            for (int32_t a = 0; a < knode; ++a) cnt[c + a] = 0;
        return;
    }
    (void)over;
#pragma unroll
    for (int m = 0; m < NBR_LPL; ++m) {
        while (pos[m] < end[m] && !nbr_ok(sm, cf, cj, pos[m])) ++pos[m];
        head[m] = (pos[m] < end[m]) ? cj[pos[m]] : INT_MAX;
    }
    // lanes a < knode write copy a of each merged entry
    const int32_t base = (fill && lane < knode) ? nptr[c + lane] : 0;
    int o = 0;
    for (;;) {
        int h = INT_MAX;
#pragma unroll
        for (int m = 0; m < NBR_LPL; ++m) h = min(h, head[m]);
        int mn = team_min<T>(h);
        if (mn == INT_MAX) break;
        if (fill) {
            if (lane < knode) nbr[base + o] = mn;
            for (int32_t a = T + lane; a < knode; a += T) nbr[nptr[c + a] + o] = mn;
        }
        ++o;
#pragma unroll
        for (int m = 0; m < NBR_LPL; ++m) {
            if (head[m] == mn) {
                ++pos[m];
                while (pos[m] < end[m] && !nbr_ok(sm, cf, cj, pos[m])) ++pos[m];
                head[m] = (pos[m] < end[m]) ? cj[pos[m]] : INT_MAX;
            }
        }
    }
    if (!fill && lane == 0)
        for (int32_t a = 0; a < knode; ++a) cnt[c + a] = o;
}

template <int T>
static void nbr_t(int32_t nc, const int32_t *clist, const int32_t *rp,
                  const int32_t *cj, const uint8_t *sm, const int8_t *cf,
                  int32_t distance, const int32_t *flist, int32_t nf, bool fill,
                  int32_t *cnt, const int32_t *nptr, int32_t *nbr,
                  int32_t *overflow, int32_t knode, hipStream_t s) {
    LAIR_LAUNCH(k_nbr<T>, dim3(blocks_for((int64_t)(nc / knode) * T, 256)), dim3(256),
                       0, s, nc, clist, rp, cj, sm, cf, distance, flist, nf, fill,
                       cnt, nptr, nbr, overflow, knode);
    LAIR_LAUNCH_CHECK();
}

void launch_neighbourhoods(int32_t nc, int32_t n, const int32_t *clist,
                           const int32_t *rp, const int32_t *cj,
                           const uint8_t *smask, const int8_t *cf,
                           int32_t distance, const int32_t *flist, int32_t nf,
                           int32_t *cnt, const int32_t *nptr, int32_t *nbr,
                           int32_t *overflow, int32_t max_row,
                           hipStream_t s, int32_t knode) {
    (void)n;
    if (nc == 0) return;
    if (knode < 1 || nc % knode != 0)
        fail(LAIR_EINVAL, "neighbourhoods: %d C rows in nodes of %d", nc, knode);
    bool fill = (nbr != nullptr);
    ProfScope ps("nbr", s, 4.0 * nc);
    int t;
    if (distance == 2) {
        int need = (max_row + 1 + NBR_LPL - 1) / NBR_LPL;
        t = 4;
        while (t < 64 && t < need) t <<= 1;
    } else {
        t = team_for_mean(distance == 1 ? (double)max_row : 64.0);
        if (t > 16 && distance == 1) t = 16;
    }
    switch (t) {
        case 2: nbr_t<2>(nc, clist, rp, cj, smask, cf, distance, flist, nf, fill, cnt, nptr, nbr, overflow, knode, s); break;
        case 4: nbr_t<4>(nc, clist, rp, cj, smask, cf, distance, flist, nf, fill, cnt, nptr, nbr, overflow, knode, s); break;
        case 8: nbr_t<8>(nc, clist, rp, cj, smask, cf, distance, flist, nf, fill, cnt, nptr, nbr, overflow, knode, s); break;
        case 16: nbr_t<16>(nc, clist, rp, cj, smask, cf, distance, flist, nf, fill, cnt, nptr, nbr, overflow, knode, s); break;
        case 32: nbr_t<32>(nc, clist, rp, cj, smask, cf, distance, flist, nf, fill, cnt, nptr, nbr, overflow, knode, s); break;
        default: nbr_t<64>(nc, clist, rp, cj, smask, cf, distance, flist, nf, fill, cnt, nptr, nbr, overflow, knode, s); break;
    }
}

// ===========================================================================
// Local lAIR solves, Eq. (system): for C-point i with N = (l_0 .. l_{s-1})
//   M[p][q] = a(l_q, l_p),   f[p] = -a(i, l_p),   M z = f.
// Row c of R is written in place: sorted N with z, and 1 at column i.
// Singular systems (|pivot| <= 1e-14 ||M||_inf) are listed for the
// least-squares kernel.
// ===========================================================================
constexpr double SING_TOL = 1e-14;

__device__ __forceinline__ void write_r_row(int32_t rbase, int s, int32_t i,
                                            const int32_t *l, const double *z,
                                            int32_t *r_cj, double *r_v) {
    // position of the C-point among the sorted columns
    int ip = 0;
    for (int q = 0; q < s; ++q) ip += (l[q] < i);
    for (int q = 0; q < s; ++q) {
        int o = rbase + q + (q >= ip ? 1 : 0);
        r_cj[o] = l[q];
        r_v[o] = z[q];
    }
    r_cj[rbase + ip] = i;
    r_v[rbase + ip] = 1.0;
}

// Every solver below performs the same floating-point operations in the
// same order, so a system's z does not depend on which of them takes it
// (the size buckets only change speed):
//   * pivot of step k: the largest |M[r][k]| among the rows not yet used,
//     ties to the row at the smallest position, positions being those of
//     partial pivoting with row exchanges;
//   * each remaining row r: m = M[r][k] / M[k][k]; M[r][j] -= m M[k][j]
//     for j > k; f_r -= m f_k;
//   * back substitution column by column from the last: z_k = f_k / U[k][k],
//     then f_r -= U[r][k] z_k for the rows above;
//   * MIXED: the factorisation runs in float; the double residual
//     r_p = f_p - sum_k M[p][k] z_k is summed from the last column down,
//     then the same eliminations and back substitution run on r and z += d.

// One lane per system, s <= SM, everything in registers.
template <int SM, bool MIXED>
__device__ __forceinline__ void lane_solve(int32_t c, const int32_t *clist, const int32_t *nptr,
                           const int32_t *nbr, const int32_t *rp, const int32_t *cj,
                           const double *v, int32_t *r_cj, double *r_v, int8_t *flags,
                           int32_t *sing, int32_t *nsing) {
    using FT = typename std::conditional<MIXED, float, double>::type;
    const int32_t i = clist[c];
    const int32_t n0 = nptr[c];
    const int s = nptr[c + 1] - n0;
    const int32_t rbase = n0 + c;
    if (s == 0) {
        r_cj[rbase] = i;
        r_v[rbase] = 1.0;
        return;
    }
    int li[SM];
#pragma unroll
    for (int q = 0; q < SM; ++q) li[q] = (q < s) ? nbr[n0 + q] : -1;
    // Md holds M in double (kept for the refinement residual in MIXED);
    // M is the copy that gets factorised (float in MIXED)
    double Md[SM][SM];
    FT M[SM][SM];
    double f[SM];
#pragma unroll
    for (int p = 0; p < SM; ++p) {
        f[p] = 0.0;
#pragma unroll
        for (int q = 0; q < SM; ++q) Md[p][q] = 0.0;
    }
    // column p of M comes from row l_p of A: M[q][p] = a(l_p, l_q)
#pragma unroll
    for (int p = 0; p < SM; ++p) {
        if (p < s) {
            int r = li[p];
            for (int e = rp[r]; e < rp[r + 1]; ++e) {
                int col = cj[e];
                double a = v[e];
#pragma unroll
                for (int q = 0; q < SM; ++q)
                    if (li[q] == col) Md[q][p] = a;
            }
        }
    }
#pragma unroll
    for (int p = 0; p < SM; ++p)
#pragma unroll
        for (int q = 0; q < SM; ++q) M[p][q] = (FT)Md[p][q];
    for (int e = rp[i]; e < rp[i + 1]; ++e) {
        int col = cj[e];
        double a = v[e];
#pragma unroll
        for (int p = 0; p < SM; ++p)
            if (li[p] == col) f[p] = -a;
    }
    double mnorm = 0.0;
#pragma unroll
    for (int p = 0; p < SM; ++p) {
        double rs = 0.0;
#pragma unroll
        for (int q = 0; q < SM; ++q) rs += fabs(Md[p][q]);
        mnorm = fmax(mnorm, rs);
    }
    const double tol = SING_TOL * mnorm;
    int perm[SM];
#pragma unroll
    for (int p = 0; p < SM; ++p) perm[p] = p;
    bool singular = false;
    FT fw[SM];
#pragma unroll
    for (int p = 0; p < SM; ++p) fw[p] = (FT)f[p];
#pragma unroll
    for (int k = 0; k < SM; ++k) {
        if (k < s && !singular) {
            int pr = k;
            double pv = fabs((double)M[k][k]);
#pragma unroll
            for (int r = k + 1; r < SM; ++r)
                if (r < s && fabs((double)M[r][k]) > pv) { pv = fabs((double)M[r][k]); pr = r; }
            if (pv <= tol) {
                singular = true;
            } else {
#pragma unroll
                for (int r = k + 1; r < SM; ++r) {
                    if (r == pr) {
#pragma unroll
                        for (int q = 0; q < SM; ++q) {
                            FT t = M[k][q]; M[k][q] = M[r][q]; M[r][q] = t;
                        }
                        FT t = fw[k]; fw[k] = fw[r]; fw[r] = t;
                        int tp = perm[k]; perm[k] = perm[r]; perm[r] = tp;
                    }
                }
#pragma unroll
                for (int r = k + 1; r < SM; ++r) {
                    if (r < s) {
                        const FT mult = M[r][k] / M[k][k];
                        M[r][k] = mult;               // kept for the refinement
#pragma unroll
                        for (int q = k + 1; q < SM; ++q) M[r][q] -= mult * M[k][q];
                        fw[r] -= mult * fw[k];
                    }
                }
            }
        }
    }
    if (singular) {
        flags[c] = 1;
        sing[atomicAdd(nsing, 1)] = c;
        return;
    }
    double z[SM];
    double res[SM];
#pragma unroll
    for (int p = 0; p < SM; ++p) res[p] = f[p];
#pragma unroll
    for (int k = SM - 1; k >= 0; --k) {
        z[k] = 0.0;
        if (k < s) {
            const FT zk = fw[k] / M[k][k];
#pragma unroll
            for (int r = 0; r < k; ++r) fw[r] -= M[r][k] * zk;
            z[k] = (double)zk;
            if (MIXED) {
#pragma unroll
                for (int p = 0; p < SM; ++p) res[p] -= Md[p][k] * (double)zk;
            }
        }
    }
    if (MIXED) {
        // the residual in pivot order, then L, then U
        FT w[SM];
#pragma unroll
        for (int k = 0; k < SM; ++k) {
            FT acc = (FT)0;
#pragma unroll
            for (int p = 0; p < SM; ++p)
                if (perm[k] == p) acc = (FT)res[p];
            w[k] = acc;
        }
#pragma unroll
        for (int k = 0; k < SM; ++k)
#pragma unroll
            for (int r = k + 1; r < SM; ++r)
                if (r < s) w[r] -= M[r][k] * w[k];
#pragma unroll
        for (int k = SM - 1; k >= 0; --k) {
            if (k < s) {
                const FT dk = w[k] / M[k][k];
#pragma unroll
                for (int r = 0; r < k; ++r) w[r] -= M[r][k] * dk;
                z[k] += (double)dk;
            }
        }
    }
    int32_t lw[SM];
#pragma unroll
    for (int q = 0; q < SM; ++q) lw[q] = li[q];
    // sorted write of the R row
    int ip = 0;
#pragma unroll
    for (int q = 0; q < SM; ++q) ip += (q < s && lw[q] < i) ? 1 : 0;
#pragma unroll
    for (int q = 0; q < SM; ++q) {
        if (q < s) {
            int o = rbase + q + (q >= ip ? 1 : 0);
            r_cj[o] = lw[q];
            r_v[o] = z[q];
        }
    }
    r_cj[rbase + ip] = i;
    r_v[rbase + ip] = 1.0;
}

// Inclusive prefix sum over a team of T consecutive lanes.
template <int T>
__device__ __forceinline__ int team_scan_incl(int x) {
    const int p = threadIdx.x % T;
#pragma unroll
    for (int o = 1; o < T; o <<= 1) {
        int u = __shfl_up(x, o, T);
        if (p >= o) x += u;
    }
    return x;
}

// Gathers the local matrix M[k][q] = a(l_q, l_k) (row stride ldm) for the
// sorted neighbourhood ln[0..s): the entries of the s rows l_q are numbered
// as one flat range and each lane of the team takes every T-th of them,
// U at a time, so a lane's loads do not wait on each other (the row-by-row
// walk of long coarse-grid rows was bound by load latency).  off (s + 1)
// and st (s) are the team's scratch; BLOCK selects a block barrier (the
// one-wave kernel, whose scratch may sit in global memory) over a wave
// fence.  Md, when given, receives the same entries in double.
template <int T, int U, bool BLOCK, class FT>
__device__ __forceinline__ void gather_local(int p, int s, const int32_t *ln, int32_t *off, int32_t *st,
                             const int32_t *rp, const int32_t *cj, const double *v,
                             FT *M, int ldm, double *Md) {
    int carry = 0;
    for (int q0 = 0; q0 < s; q0 += T) {
        const int q = q0 + p;
        int a = 0, len = 0;
        if (q < s) {
            const int r = ln[q];
            a = rp[r];
            len = rp[r + 1] - a;
        }
        const int incl = team_scan_incl<T>(len);
        if (q < s) {
            st[q] = a;
            off[q] = carry + incl - len;
        }
        carry += __shfl(incl, T - 1, T);
    }
    if (p == 0) off[s] = carry;
    if (BLOCK) __syncthreads(); else wave_lds_sync();
    const int E = carry;
    int q = 0;
    for (int base = p; base < E; base += U * T) {
        int e[U], qq[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int idx = base + u * T;
            e[u] = -1;
            qq[u] = 0;
            if (idx < E) {
                while (off[q + 1] <= idx) ++q;
                qq[u] = q;
                e[u] = st[q] + idx - off[q];
            }
        }
        int col[U];
        double val[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            col[u] = -1;
            val[u] = 0.0;
            if (e[u] >= 0) {
                col[u] = cj[e[u]];
                val[u] = v[e[u]];
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (e[u] >= 0) {
                const int k = bsearch_i32(ln, s, col[u]);
                if (k >= 0) {
                    M[(size_t)k * ldm + qq[u]] = (FT)val[u];
                    if (Md) Md[(size_t)k * ldm + qq[u]] = val[u];
                }
            }
        }
    }
}

// One team of T lanes (part of one wave) per system with s <= T.  The
// gather writes M into the team's LDS tile; lane p then holds row p of M in
// registers.  Rows stay in place: at step k the pivot row is found by an
// arg-max over the unused lanes, broadcast by shuffles, and the other
// unused rows eliminate column k.  Back substitution: the pivot lane of
// step k yields z_k and every lane removes column k from its right-hand
// side.  LDS of the team: M (T x T doubles), f (T doubles), ln, pv, st
// (T ints each) and off (T + 1 ints), as typed LDS arrays.
template <int T, bool MIXED>
__device__ __forceinline__ void team_solve(int p, int32_t c, const int32_t *clist, const int32_t *nptr,
                           const int32_t *nbr, const int32_t *rp, const int32_t *cj,
                           const double *v, int32_t *r_cj, double *r_v, int8_t *flags,
                           int32_t *sing, int32_t *nsing, double *M, double *f, int32_t *ln,
                           int32_t *pv, int32_t *sst, int32_t *soff) {
    using FT = typename std::conditional<MIXED, float, double>::type;
    const int32_t i = clist[c];
    const int32_t n0 = nptr[c];
    const int s = nptr[c + 1] - n0;
    const int32_t rbase = n0 + c;
    const int32_t lp = (p < s) ? nbr[n0 + p] : INT_MAX;
    ln[p] = lp;
    f[p] = 0.0;
    pv[p] = p;
#pragma unroll
    for (int j = 0; j < T; ++j) M[j * T + p] = 0.0;
    wave_lds_sync();
    gather_local<T, 4, false, double>(p, s, ln, soff, sst, rp, cj, v, M, T, nullptr);
    for (int e = rp[i] + p; e < rp[i + 1]; e += T) {
        int q = bsearch_i32(ln, s, cj[e]);
        if (q >= 0) f[q] = -v[e];
    }
    wave_lds_sync();
    FT Mr[T];
    double rs = 0.0;
#pragma unroll
    for (int j = 0; j < T; ++j) {
        const double a = M[p * T + j];
        Mr[j] = (FT)a;
        rs += fabs(a);
    }
    const double f0 = f[p];
    const double tol = SING_TOL * team_max<T>(p < s ? rs : 0.0);
    FT fr = (FT)f0;
    FT Lr[T];
    // the steps run without branches (k >= s contributes zeros), so the
    // compiler keeps the row arrays in place instead of copying them at
    // every join
    bool used = (p >= s);
    bool singular = false;
    int pos = p;          // this row's position under the row exchanges
#pragma unroll
    for (int k = 0; k < T; ++k) {
        const bool act = k < s;
        double cand;
        int key = (pos << 8) | p;
        if constexpr (MIXED) {
            // the same arg-max in one 64-bit key: |pivot| bits + 1 above (0
            // for rows out of the race, below every candidate), the
            // complement of the key below (ties to the smallest key)
            uint64_t pk = (uint64_t)(~(uint32_t)key);
            if (!(used || !act))
                pk |= (uint64_t)(__float_as_uint(fabsf(Mr[k])) + 1u) << 32;
            pk = team_max_u64<T>(pk);
            key = (int)~(uint32_t)pk;
            const uint32_t hi = (uint32_t)(pk >> 32);
            cand = hi ? (double)__uint_as_float(hi - 1u) : -1.0;
        } else {
            cand = (used || !act) ? -1.0 : fabs((double)Mr[k]);
            team_argmax<T>(cand, key);
        }
        const int who = key & 0xff;
        const int wpos = key >> 8;
        if (act) pos = (p == who) ? k : (pos == k ? wpos : pos);
        singular = singular || (act && cand <= tol);
        if (p == 0 && act) pv[k] = who;
        const FT pk = __shfl(Mr[k], who, T);
        const FT fk = __shfl(fr, who, T);
        used = used || (act && p == who);
        const FT mult = (used || !act) ? (FT)0 : Mr[k] / pk;
        Lr[k] = mult;
#pragma unroll
        for (int j = k + 1; j < T; ++j) {
            const FT pj = __shfl(Mr[j], who, T);
            Mr[j] -= mult * pj;
        }
        fr -= mult * fk;
    }
    if (singular) {
        if (p == 0) {
            flags[c] = 1;
            sing[atomicAdd(nsing, 1)] = c;
        }
        return;
    }
    wave_lds_sync();
    double zq = 0.0;
    double r = f0;
#pragma unroll
    for (int k = T - 1; k >= 0; --k) {
        const bool act = k < s;
        const FT q = fr / Mr[k];
        const FT zk = act ? __shfl(q, pv[k], T) : (FT)0;
        fr -= Mr[k] * zk;
        zq = (k == p) ? (double)zk : zq;
        if (MIXED) r -= M[p * T + k] * (double)zk;
    }
    if (MIXED) {
        FT rr = (FT)r;
#pragma unroll
        for (int k = 0; k < T; ++k) {
            const FT rk = __shfl(rr, pv[k], T);
            rr -= Lr[k] * rk;
        }
#pragma unroll
        for (int k = T - 1; k >= 0; --k) {
            const bool act = k < s;
            const FT q = rr / Mr[k];
            const FT dk = act ? __shfl(q, pv[k], T) : (FT)0;
            rr -= Mr[k] * dk;
            zq = (k == p) ? zq + (double)dk : zq;
        }
    }
    // sorted write of the R row: lane q writes entry q
    int ip = team_sum_int<T>((p < s && lp < i) ? 1 : 0);
    if (p < s) {
        int o = rbase + p + (p >= ip ? 1 : 0);
        r_cj[o] = lp;
        r_v[o] = zq;
    }
    if (p == 0) {
        r_cj[rbase + ip] = i;
        r_v[rbase + ip] = 1.0;
    }
}

// Size buckets: 0 one lane (s <= e0 <= 4), 1 eight lanes (s <= e1 <= 8),
// 2 sixteen (s <= e2 <= 16), 3 thirty-two (s <= e3 <= 32), 4 one wave.
// fused: buckets 0-2 share the persistent kernel, else each has its own.
struct Buckets {
    int32_t e[4];
    int32_t fused;
};
constexpr int NBUCKET = 5;

// List every C-point under its bucket.  Positions come from LDS counters
// per block and one global atomic per block and bucket (the order within a
// bucket does not affect any result).
__global__ void __launch_bounds__(256)
k_local_bin(int32_t nc, const int32_t *nptr, Buckets bk, int32_t *cnt, int32_t *lists,
            int8_t *flags) {
    __shared__ int32_t s_cnt[NBUCKET], s_base[NBUCKET];
    if (threadIdx.x < NBUCKET) s_cnt[threadIdx.x] = 0;
    __syncthreads();
    const int32_t c = (int32_t)(xcd_block_id() * blockDim.x + threadIdx.x);
    int b = -1, pos = 0;
    if (c < nc) {
        const int s = nptr[c + 1] - nptr[c];
        b = s <= bk.e[0] ? 0 : s <= bk.e[1] ? 1 : s <= bk.e[2] ? 2 : s <= bk.e[3] ? 3 : 4;
        flags[c] = 0;
        pos = atomicAdd(&s_cnt[b], 1);
    }
    __syncthreads();
    if (threadIdx.x < NBUCKET)
        s_base[threadIdx.x] = s_cnt[threadIdx.x] ? atomicAdd(&cnt[threadIdx.x], s_cnt[threadIdx.x])
                                                 : 0;
    __syncthreads();
    if (b >= 0) lists[(int64_t)b * nc + s_base[b] + pos] = c;
}

// The persistent local-solve kernel: every block takes tiles from one
// queue (a ticket counter) until none is left, a tile being 32 systems of
// the 8-lane bucket, 16 of the 16-lane bucket or 256 of the one-lane bucket
// (larger buckets first).  Bucket lengths are read on the device, so no
// host synchronisation separates binning from solving.  The 32-lane and
// one-wave buckets always run as kernels of their own (their registers and
// LDS would halve the residency of the others); whether buckets 0-2 share
// this kernel or take one each is part of the tuned choice, since sharing
// takes the footprint of the 16-lane path for all three.
constexpr int PERSIST_BS = 256;
// LDS of the shared kernel: the 8-lane (32 teams) and 16-lane (16 teams)
// layouts over the same typed arrays
constexpr int PSM = 16 * 16 * 16;      // M tiles (doubles), >= 32 * 8 * 8
constexpr int PSV = 256;               // f, ln, pv, st (per team T entries)
constexpr int PSO = 32 * 9;            // off (T + 1 per team), >= 16 * 17

template <bool MIXED>
__global__ void __launch_bounds__(PERSIST_BS)
k_local_persist(const int32_t *cnt, const int32_t *lists, int32_t nc, int32_t *ticket,
                const int32_t *clist, const int32_t *nptr, const int32_t *nbr,
                const int32_t *rp, const int32_t *cj, const double *v, int32_t *r_cj,
                double *r_v, int8_t *flags, int32_t *sing, int32_t *nsing) {
    __shared__ double sM[PSM];
    __shared__ double sf[PSV];
    __shared__ int32_t sl[PSV], spv[PSV], sst[PSV], soff[PSO];
    __shared__ int32_t s_tile;
    const int32_t n1 = cnt[0], n8 = cnt[1], n16 = cnt[2];
    constexpr int P16 = PERSIST_BS / 16, P8 = PERSIST_BS / 8, P1 = PERSIST_BS;
    const int32_t t16 = (n16 + P16 - 1) / P16, t8 = (n8 + P8 - 1) / P8,
                  t1 = (n1 + P1 - 1) / P1;
    const int32_t total = t16 + t8 + t1;
    for (;;) {
        if (threadIdx.x == 0) s_tile = atomicAdd(ticket, 1);
        __syncthreads();
        int32_t t = s_tile;
        __syncthreads();
        if (t >= total) break;
        if (t < t16) {
            const int team = threadIdx.x / 16;
            const int32_t idx = t * P16 + team;
            if (idx < n16)
                team_solve<16, MIXED>(threadIdx.x % 16, lists[2 * (int64_t)nc + idx], clist, nptr,
                                      nbr, rp, cj, v, r_cj, r_v, flags, sing, nsing,
                                      sM + team * 256, sf + team * 16, sl + team * 16,
                                      spv + team * 16, sst + team * 16, soff + team * 17);
        } else if ((t -= t16) < t8) {
            const int team = threadIdx.x / 8;
            const int32_t idx = t * P8 + team;
            if (idx < n8)
                team_solve<8, MIXED>(threadIdx.x % 8, lists[(int64_t)nc + idx], clist, nptr, nbr,
                                     rp, cj, v, r_cj, r_v, flags, sing, nsing, sM + team * 64,
                                     sf + team * 8, sl + team * 8, spv + team * 8,
                                     sst + team * 8, soff + team * 9);
        } else {
            t -= t8;
            const int32_t idx = t * P1 + (int32_t)threadIdx.x;
            if (idx < n1)
                lane_solve<4, MIXED>(lists[idx], clist, nptr, nbr, rp, cj, v, r_cj, r_v, flags,
                                     sing, nsing);
        }
    }
}

// One bucket on its own: teams of T lanes (bucket b); the grid covers every
// C-point (the bucket's length is only known on the device).
template <int T, bool MIXED>
__global__ void __launch_bounds__(T >= 32 ? 128 : 256)
k_local_teams(const int32_t *cnt, int b, const int32_t *list, const int32_t *clist,
              const int32_t *nptr, const int32_t *nbr, const int32_t *rp, const int32_t *cj,
              const double *v, int32_t *r_cj, double *r_v, int8_t *flags, int32_t *sing,
              int32_t *nsing) {
    constexpr int TEAMS = (T >= 32 ? 128 : 256) / T;
    __shared__ double sM[TEAMS][T * T];
    __shared__ double sf[TEAMS][T];
    __shared__ int32_t sl[TEAMS][T], spv[TEAMS][T], sst[TEAMS][T], soff[TEAMS][T + 1];
    const int team = threadIdx.x / T;
    const int32_t n = cnt[b];
    // one system per team: a loop over several would keep more registers
    // live across iterations and cost residency
    const int64_t t = (int64_t)xcd_block_id() * TEAMS + team;
    if (t < n)
        team_solve<T, MIXED>(threadIdx.x % T, list[t], clist, nptr, nbr, rp, cj, v, r_cj, r_v,
                             flags, sing, nsing, sM[team], sf[team], sl[team], spv[team],
                             sst[team], soff[team]);
}

// The one-lane bucket on its own: one system per thread.
template <bool MIXED>
__global__ void __launch_bounds__(256)
k_local_lane(const int32_t *cnt, const int32_t *list, const int32_t *clist,
             const int32_t *nptr, const int32_t *nbr, const int32_t *rp, const int32_t *cj,
             const double *v, int32_t *r_cj, double *r_v, int8_t *flags, int32_t *sing,
             int32_t *nsing) {
    const int64_t t = xcd_block_id() * blockDim.x + threadIdx.x;
    if (t >= cnt[0]) return;
    lane_solve<4, MIXED>(list[t], clist, nptr, nbr, rp, cj, v, r_cj, r_v, flags, sing, nsing);
}

// One wave per system (blockDim = 64), rows exchanged in LDS.  M lives in
// dynamic LDS sized for the level's largest system up to WSMAX, beyond that
// in a global scratch slab of 3 smax^2 doubles per block.  The gather
// enumerates the entries of the rows l_p as one flat range over the lanes.
// MIXED keeps a double copy of M for the refinement residual.  (WSMAX: 64.)

template <class FT>
__host__ __device__ constexpr size_t wave_lds_bytes(int cap) {
    return (size_t)cap * cap * sizeof(FT) +
           (sizeof(FT) == sizeof(float) ? (size_t)cap * cap * sizeof(double) : 0) +
           (size_t)cap * (2 * sizeof(double) + sizeof(FT) + 4 * sizeof(int32_t)) + 64;
}

template <bool MIXED>
__device__ __forceinline__ void wave_solve(int32_t c, const int32_t *clist, const int32_t *nptr,
                           const int32_t *nbr, const int32_t *rp, const int32_t *cj,
                           const double *v, int32_t *r_cj, double *r_v, int8_t *flags,
                           int32_t *sing, int32_t *nsing, double *dyn, double *slab,
                           int32_t smax, int32_t cap) {
    using FT = typename std::conditional<MIXED, float, double>::type;
    int lane = threadIdx.x;
    int32_t i = clist[c];
    int32_t n0 = nptr[c];
    int s = nptr[c + 1] - n0;
    int32_t rbase = n0 + c;
    const int32_t *l = nbr + n0;
    if (lane == 0) flags[c] = 0;
    const int32_t m = (s <= cap) ? cap : smax;   // capacity of this layout
    // layout: z, f, Md (double; Md only in MIXED), M, w (FT), ln, perm,
    // off, st (int)
    double *z = (s <= cap) ? dyn : slab;
    double *f = z + m;
    double *Md = MIXED ? f + m : nullptr;
    FT *M = (FT *)(f + m + (MIXED ? (size_t)m * m : 0));
    FT *w = M + (size_t)m * m;
    int32_t *ln = (int32_t *)(w + m);
    int32_t *perm = ln + m;
    int32_t *off = perm + m;
    int32_t *st = off + m + 1;
    for (int idx = lane; idx < s * s; idx += 64) {
        M[idx] = (FT)0;
        if (MIXED) Md[idx] = 0.0;
    }
    for (int p = lane; p < s; p += 64) { f[p] = 0.0; ln[p] = l[p]; perm[p] = p; }
    __syncthreads();
    // column p of M is row l_p of A restricted to N: M[q][p] = a(l_p, l_q)
    gather_local<64, 4, true, FT>(lane, s, ln, off, st, rp, cj, v, M, s, Md);
    for (int e = rp[i] + lane; e < rp[i + 1]; e += 64) {
        int p = bsearch_i32(ln, s, cj[e]);
        if (p >= 0) f[p] = -v[e];
    }
    __syncthreads();
    double rs = 0.0;
    for (int p = lane; p < s; p += 64) {
        double a = 0.0;
        for (int q = 0; q < s; ++q) a += fabs(MIXED ? Md[p * s + q] : (double)M[p * s + q]);
        rs = fmax(rs, a);
    }
    double tol = SING_TOL * team_max<64>(rs);
    for (int p = lane; p < s; p += 64) w[p] = (FT)f[p];
    __syncthreads();
    bool singular = false;
    for (int k = 0; k < s; ++k) {
        double pv = -1.0;
        int pr = INT_MAX;
        for (int r = k + lane; r < s; r += 64) {
            double a = fabs((double)M[r * s + k]);
            if (a > pv) { pv = a; pr = r; }
        }
        team_argmax<64>(pv, pr);
        if (pv <= tol) { singular = true; break; }
        if (pr != k) {
            for (int q = lane; q < s; q += 64) {
                FT t = M[k * s + q]; M[k * s + q] = M[pr * s + q]; M[pr * s + q] = t;
            }
            if (lane == 0) {
                FT t = w[k]; w[k] = w[pr]; w[pr] = t;
                int tp = perm[k]; perm[k] = perm[pr]; perm[pr] = tp;
            }
        }
        __syncthreads();
        for (int r = k + 1 + lane; r < s; r += 64) {
            const FT mult = M[r * s + k] / M[k * s + k];
            M[r * s + k] = mult;
            w[r] -= mult * w[k];
        }
        __syncthreads();
        int wdt = s - k - 1;
        for (int idx = lane; idx < wdt * wdt; idx += 64) {
            int r = k + 1 + idx / wdt;
            int q = k + 1 + idx % wdt;
            M[r * s + q] -= M[r * s + k] * M[k * s + q];
        }
        __syncthreads();
    }
    if (singular) {
        if (lane == 0) {
            flags[c] = 1;
            sing[atomicAdd(nsing, 1)] = c;
        }
        return;
    }
    // back substitution, column oriented: z_k = w_k / u_kk; w_r -= u_rk z_k
    for (int k = s - 1; k >= 0; --k) {
        FT zk = w[k] / M[k * s + k];
        __syncthreads();
        if (lane == 0) z[k] = (double)zk;
        for (int r = lane; r < k; r += 64) w[r] -= M[r * s + k] * zk;
        __syncthreads();
    }
    if (MIXED) {
        // one refinement in double: r = f - M z from the double copy of M
        // (rows in their original order), then z += LU^{-1} r with the
        // float factors
        double *res = f;
        for (int p = lane; p < s; p += 64) {
            double acc = res[p];
            for (int q = s - 1; q >= 0; --q) acc -= Md[p * s + q] * z[q];
            res[p] = acc;
        }
        __syncthreads();
        for (int k = lane; k < s; k += 64) w[k] = (FT)res[perm[k]];
        __syncthreads();
        for (int k = 0; k < s; ++k) {
            FT wk = w[k];
            for (int r = k + 1 + lane; r < s; r += 64) w[r] -= M[r * s + k] * wk;
            __syncthreads();
        }
        for (int k = s - 1; k >= 0; --k) {
            FT zk = w[k] / M[k * s + k];
            __syncthreads();
            if (lane == 0) z[k] += (double)zk;
            for (int r = lane; r < k; r += 64) w[r] -= M[r * s + k] * zk;
            __syncthreads();
        }
    }
    __syncthreads();
    int ip = 0;
    for (int q = lane; q < s; q += 64) ip += (ln[q] < i) ? 1 : 0;
    ip = team_sum_int<64>(ip);
    for (int q = lane; q < s; q += 64) {
        int o = rbase + q + (q >= ip ? 1 : 0);
        r_cj[o] = ln[q];
        r_v[o] = z[q];
    }
    if (lane == 0) {
        r_cj[rbase + ip] = i;
        r_v[rbase + ip] = 1.0;
    }
}

// Binary searches of a trip count fixed by n alone (steps from the largest
// power of two <= n down), so a lane's searches for several keys proceed
// side by side.  Entries of a[0..n) below key, and at or below.
__device__ __forceinline__ int count_below(const int32_t *a, int n, int key) {
    int p = 0;
    if (n <= 0) return 0;
    for (int step = 1 << (31 - __clz(n)); step > 0; step >>= 1) {
        const int t = p + step;
        const int x = a[min(t, n) - 1];
        if (t <= n && x < key) p = t;
    }
    return p;
}
__device__ __forceinline__ int count_upto(const int32_t *a, int n, int key) {
    int p = 0;
    if (n <= 0) return 0;
    for (int step = 1 << (31 - __clz(n)); step > 0; step >>= 1) {
        const int t = p + step;
        const int x = a[min(t, n) - 1];
        if (t <= n && x <= key) p = t;
    }
    return p;
}

// The gather of gather_local for one wave (a block of 64 threads):
// M[k][q] = a(l_q, l_k) (row stride ldm), and the same entries in double in
// Md when given.  Each entry's row in the flat range and its column's place
// in N come from the searches above, so the U entries of a lane are found
// side by side instead of one walk after another.
template <int U, class FT>
__device__ __forceinline__ void gather_wave(int lane, int s, const int32_t *ln, int32_t *off,
                                            int32_t *st, const int32_t *rp, const int32_t *cj,
                                            const double *v, FT *M, int ldm, double *Md) {
    int carry = 0;
    for (int q0 = 0; q0 < s; q0 += 64) {
        const int q = q0 + lane;
        int a = 0, len = 0;
        if (q < s) {
            const int r = ln[q];
            a = rp[r];
            len = rp[r + 1] - a;
        }
        const int incl = team_scan_incl<64>(len);
        if (q < s) {
            st[q] = a;
            off[q] = carry + incl - len;
        }
        carry += __shfl(incl, 63);
    }
    if (lane == 0) off[s] = carry;
    __syncthreads();
    const int E = carry;
    for (int base = lane; base < E; base += U * 64) {
        int qq[U], e[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int idx = min(base + u * 64, E - 1);
            qq[u] = count_upto(off + 1, s - 1, idx);     // off[qq] <= idx < off[qq + 1]
            e[u] = st[qq[u]] + idx - off[qq[u]];
        }
        int col[U];
        double val[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            col[u] = cj[e[u]];
            val[u] = v[e[u]];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int kp = count_below(ln, s, col[u]);
            if (base + u * 64 < E && kp < s && ln[kp] == col[u]) {
                M[(size_t)kp * ldm + qq[u]] = (FT)val[u];
                if (Md) Md[(size_t)kp * ldm + qq[u]] = val[u];
            }
        }
    }
}

// Block form of the local systems (Sec. 3.1): the k rows of a C-node share
// their neighbourhood, so the k systems A(N,N)^T z_a = -A(i_a,N)^T have one
// matrix and k right-hand sides.  One wave per node factors M once (the
// pivoting of wave_solve) and carries the k right-hand sides through the
// elimination, the back substitution and, in MIXED, the refinement; every
// right-hand side sees exactly the operations wave_solve applies to it, so
// the rows of R equal those of k separate solves bit for bit.  The node's
// rows are clist[c0 .. c0 + k - 1] = i0 .. i0 + k - 1 with c0 = node k;
// a node whose rows do not have that form or whose lists differ in length
// is counted in *bad and left alone.  The work arrays of a system live in
// LDS when they fit, else partly (the double copy of M) or wholly in a
// global slab per block.
constexpr size_t NODE_LDS_MAX = 64 * 1024;   // LDS of one node's block
constexpr size_t NODE_LDS_CU = 152 * 1024;   // at most, when one block takes a CU

// Bytes of one node's work arrays for systems up to `cap` rows: with_md
// includes the double copy of M that MIXED keeps for the refinement.
template <class FT>
__host__ __device__ constexpr size_t node_lds_bytes(int cap, int k, bool with_md = true) {
    return (size_t)cap * cap * sizeof(FT) +
           (sizeof(FT) == sizeof(float) && with_md ? (size_t)cap * cap * sizeof(double) : 0) +
           (size_t)k * cap * (2 * sizeof(double) + sizeof(FT)) +
           (size_t)cap * 4 * sizeof(int32_t) + 64;
}

// Largest system size whose work arrays fit `bytes` (0 if none).
template <class FT>
static int node_cap_for(size_t bytes, int k, bool with_md, int limit) {
    int c = 0;
    while (c < limit && node_lds_bytes<FT>(c + 1, k, with_md) <= bytes) ++c;
    return c;
}

// q / d for 0 <= q < 2^22, d >= 1 by a float reciprocal and one correction
// step (the estimate is off by at most one): the loops below would
// otherwise spend most of their instructions on integer divisions.
struct SmallDiv {
    float inv;
    int d;
    __device__ explicit SmallDiv(int dd) : inv(1.0f / (float)dd), d(dd) {}
    __device__ int quot(int q) const {
        int r = (int)(((float)q + 0.5f) * inv);
        if (r * d > q) --r;
        else if ((r + 1) * d <= q) ++r;
        return r;
    }
};

template <bool MIXED>
__global__ void __launch_bounds__(64)
k_local_node(int32_t nnode, int32_t k, const int32_t *clist, const int32_t *nptr,
             const int32_t *nbr, const int32_t *rp, const int32_t *cj, const double *v,
             int32_t *r_cj, double *r_v, int8_t *flags, int32_t *sing, int32_t *nsing,
             int32_t *bad, int32_t cap, int32_t cap_nomd, double *gscratch, int64_t slab,
             int32_t smax, int32_t s_lo, int32_t s_hi) {
    using FT = typename std::conditional<MIXED, float, double>::type;
    extern __shared__ double dyn[];
    const int lane = threadIdx.x;
    double *gslab = gscratch ? gscratch + blockIdx.x * slab : nullptr;
    for (int64_t node = blockIdx.x; node < nnode; node += gridDim.x) {
        const int32_t c0 = (int32_t)(node * k);
        const int32_t i0 = clist[c0];
        const int32_t n0 = nptr[c0];
        const int s = nptr[c0 + 1] - n0;
        if (s < s_lo || s > s_hi) continue;      // outside this launch's size range
        // where the work arrays live: all in LDS (s <= cap); in LDS but the
        // double copy of M in this block's global slab (MIXED, s <= cap_nomd);
        // all in the slab (s <= smax)
        const bool all_lds = s <= cap;
        const bool md_out = MIXED && !all_lds && s <= cap_nomd;
        const int32_t m = all_lds ? cap : md_out ? cap_nomd : smax;
        double *base = (all_lds || md_out) ? dyn : gslab;
        // layout: z[k][m], f[k][m], Md[m][m] (MIXED, unless md_out), M[m][m],
        // w[k][m] (FT), ln, perm, off, st (int)
        double *z = base;
        double *f = z + (size_t)k * m;
        const bool md_here = MIXED && !md_out;
        double *Md = !MIXED ? nullptr : md_out ? gslab : f + (size_t)k * m;
        FT *M = (FT *)(f + (size_t)k * m + (md_here ? (size_t)m * m : 0));
        FT *w = M + (size_t)m * m;
        int32_t *ln = (int32_t *)(w + (size_t)k * m);
        int32_t *perm = ln + m;
        int32_t *off = perm + m;
        int32_t *st = off + m + 1;
        bool ok = all_lds || md_out || (gslab && s <= smax);
        for (int a = 1; a < k; ++a)
            ok = ok && clist[c0 + a] == i0 + a && nptr[c0 + a + 1] - nptr[c0 + a] == s;
        if (!ok) {
            if (lane == 0) atomicAdd(bad, 1);
            continue;
        }
        const int32_t *l = nbr + n0;
        const SmallDiv ds(s > 0 ? s : 1);
        if (lane < k) flags[c0 + lane] = 0;
        __syncthreads();
        for (int idx = lane; idx < s * s; idx += 64) {
            M[idx] = (FT)0;
            if (MIXED) Md[idx] = 0.0;
        }
        for (int idx = lane; idx < k * s; idx += 64) f[idx] = 0.0;
        for (int p = lane; p < s; p += 64) { ln[p] = l[p]; perm[p] = p; }
        __syncthreads();
        gather_wave<8, FT>(lane, s, ln, off, st, rp, cj, v, M, s, Md);
        // right-hand side a: -A(i_a, N)^T
        for (int a = 0; a < k; ++a)
            for (int e = rp[i0 + a] + lane; e < rp[i0 + a + 1]; e += 64) {
                int p = bsearch_i32(ln, s, cj[e]);
                if (p >= 0) f[a * s + p] = -v[e];
            }
        __syncthreads();
        double rs = 0.0;
        for (int p = lane; p < s; p += 64) {
            double acc = 0.0;
            for (int q = 0; q < s; ++q) acc += fabs(MIXED ? Md[p * s + q] : (double)M[p * s + q]);
            rs = fmax(rs, acc);
        }
        const double tol = SING_TOL * team_max<64>(rs);
        for (int idx = lane; idx < k * s; idx += 64) w[idx] = (FT)f[idx];
        __syncthreads();
        bool singular = false;
        for (int kk = 0; kk < s; ++kk) {
            double pv = -1.0;
            int pr = INT_MAX;
            for (int r = kk + lane; r < s; r += 64) {
                double av = fabs((double)M[r * s + kk]);
                if (av > pv) { pv = av; pr = r; }
            }
            team_argmax<64>(pv, pr);
            if (pv <= tol) { singular = true; break; }
            if (pr != kk) {
                for (int q = lane; q < s; q += 64) {
                    FT t = M[kk * s + q]; M[kk * s + q] = M[pr * s + q]; M[pr * s + q] = t;
                }
                if (lane < k) {
                    FT t = w[lane * s + kk]; w[lane * s + kk] = w[lane * s + pr];
                    w[lane * s + pr] = t;
                }
                if (lane == 0) { int tp = perm[kk]; perm[kk] = perm[pr]; perm[pr] = tp; }
            }
            __syncthreads();
            // multipliers, then every right-hand side (its pivot entry is
            // final: the multipliers of this step only touch rows below)
            for (int r = kk + 1 + lane; r < s; r += 64) M[r * s + kk] = M[r * s + kk] / M[kk * s + kk];
            __syncthreads();
            // the right-hand sides' rows below, then the trailing matrix:
            // each lane takes columns, runs down the rows eight at a time,
            // every load of a batch before its stores (the entries of a step
            // are independent), so their LDS latencies overlap
            for (int a = 0; a < k; ++a) {
                const FT wk = w[a * s + kk];
                for (int r = kk + 1 + lane; r < s; r += 64) w[a * s + r] -= M[r * s + kk] * wk;
            }
            for (int q = kk + 1 + lane; q < s; q += 64) {
                const FT pq = M[kk * s + q];
                for (int r0 = kk + 1; r0 < s; r0 += 8) {
                    FT mb[8], mx[8];
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        const int r = min(r0 + u, s - 1);
                        mb[u] = M[r * s + kk];
                        mx[u] = M[r * s + q];
                    }
#pragma unroll
                    for (int u = 0; u < 8; ++u)
                        if (r0 + u < s) M[(r0 + u) * s + q] = mx[u] - mb[u] * pq;
                }
            }
            __syncthreads();
        }
        if (singular) {
            if (lane == 0) {
                const int32_t o = atomicAdd(nsing, k);
                for (int a = 0; a < k; ++a) {
                    flags[c0 + a] = 1;
                    sing[o + a] = c0 + a;
                }
            }
            __syncthreads();
            continue;
        }
        // back substitution, column oriented for each right-hand side: z_kk
        // (every lane forms the same quotient), then the rows above
        for (int kk = s - 1; kk >= 0; --kk) {
            for (int a = 0; a < k; ++a) {
                const FT zk = w[a * s + kk] / M[kk * s + kk];
                if (lane == 0) z[a * s + kk] = (double)zk;
                for (int r = lane; r < kk; r += 64) w[a * s + r] -= M[r * s + kk] * zk;
            }
            __syncthreads();
        }
        if (MIXED) {
            // one refinement per right-hand side in double (as wave_solve):
            // each residual entry summed over the columns from the last down,
            // a lane's entries eight side by side
            for (int base = lane; base < k * s; base += 8 * 64) {
                double acc[8];
                int bm[8], bz[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int idx = min(base + u * 64, k * s - 1);
                    const int a = ds.quot(idx), p = idx - a * s;
                    bm[u] = p * s;
                    bz[u] = a * s;
                    acc[u] = f[idx];
                }
                for (int q = s - 1; q >= 0; --q) {
#pragma unroll
                    for (int u = 0; u < 8; ++u) acc[u] -= Md[bm[u] + q] * z[bz[u] + q];
                }
#pragma unroll
                for (int u = 0; u < 8; ++u)
                    if (base + u * 64 < k * s) f[base + u * 64] = acc[u];
            }
            __syncthreads();
            for (int idx = lane; idx < k * s; idx += 64) {
                const int a = ds.quot(idx), kk = idx - a * s;
                w[a * s + kk] = (FT)f[a * s + perm[kk]];
            }
            __syncthreads();
            for (int kk = 0; kk < s; ++kk) {
                for (int a = 0; a < k; ++a) {
                    const FT wk = w[a * s + kk];
                    for (int r = kk + 1 + lane; r < s; r += 64)
                        w[a * s + r] -= M[r * s + kk] * wk;
                }
                __syncthreads();
            }
            for (int kk = s - 1; kk >= 0; --kk) {
                for (int a = 0; a < k; ++a) {
                    const FT zk = w[a * s + kk] / M[kk * s + kk];
                    if (lane == 0) z[a * s + kk] += (double)zk;
                    for (int r = lane; r < kk; r += 64) w[a * s + r] -= M[r * s + kk] * zk;
                }
                __syncthreads();
            }
        }
        // rows of R: N with the identity entry at the row's place
        int ip = 0;
        for (int q = lane; q < s; q += 64) ip += (ln[q] < i0) ? 1 : 0;
        ip = team_sum_int<64>(ip);
        for (int idx = lane; idx < k * s; idx += 64) {
            const int a = ds.quot(idx), q = idx - a * s;
            const int64_t o = (int64_t)nptr[c0 + a] + c0 + a + q + (q >= ip ? 1 : 0);
            r_cj[o] = ln[q];
            r_v[o] = z[a * s + q];
        }
        if (lane < k) {
            const int64_t o = (int64_t)nptr[c0 + lane] + c0 + lane + ip;
            r_cj[o] = i0 + lane;
            r_v[o] = 1.0;
        }
        __syncthreads();
    }
}

// The node solve with M in registers, for systems up to 8R rows.  The wave
// is an 8 x 8 grid of lanes: lane (lr, lq) keeps the entries (r, q) of M
// with r = lr + 8i, q = lq + 8j in m[i][j], and in column slot R the entry
// of right-hand side lq (lq < k) at row r.  Rows never move: each keeps its
// position under the row exchanges beside it, and the pivot of step kk is
// the arg-max of |M[r][kk]| over the rows at positions >= kk, ties to the
// smallest position, as in the LDS form.  Every lane of a row of lanes
// holds column kk of its rows (cur), so the arg-max needs only a reduction
// across the rows of lanes and every lane forms its rows' multipliers; the
// pivot row goes through LDS from its row of lanes, and after the update the
// next column is shared along each row of lanes.  The substitutions
// take the column of U or L the same way; in MIXED the refinement's
// residual f - M z comes from the double matrix in LDS, summed in the order
// of the LDS form.  Every
// entry sees the operations of the LDS form in the same order, so the rows
// of R are the same bit for bit.  LDS holds the gathered matrix in double,
// the right-hand sides and the neighbourhood.
template <int R>
__host__ __device__ constexpr size_t node_reg_lds_bytes(int k, bool mg_in_lds = true) {
    return (mg_in_lds ? (size_t)64 * R * R * sizeof(double) : 0) +
           2 * (size_t)k * 8 * R * sizeof(double) +
           2 * (size_t)8 * (R + 1) * sizeof(double) + (4 * (size_t)8 * R + 1) * sizeof(int32_t) +
           64;
}

template <int R, bool MIXED, bool GMG>
__global__ void __launch_bounds__(64)
k_local_node_reg(int32_t nnode, int32_t k, const int32_t *clist, const int32_t *nptr,
                 const int32_t *nbr, const int32_t *rp, const int32_t *cj, const double *v,
                 int32_t *r_cj, double *r_v, int8_t *flags, int32_t *sing, int32_t *nsing,
                 int32_t *bad, int32_t s_lo, int32_t s_hi, double *gslab) {
    using FT = typename std::conditional<MIXED, float, double>::type;
    constexpr int SC = 8 * R, C = R + 1;
    extern __shared__ double dyn[];
    const int lane = threadIdx.x, lr = lane >> 3, lq = lane & 7;
    // layout: Mg[s][s] (in this block's global slab when GMG: LDS then
    // leaves room for more waves per CU), f[k][s] and zs[k][s] (double), two
    // pivot-row buffers of 8C (FT), ln, off, st, rowat (int)
    double *Mg = GMG ? gslab + (size_t)blockIdx.x * SC * SC : dyn;
    double *f = GMG ? dyn : dyn + (size_t)SC * SC;
    double *zs = f + (size_t)k * SC;
    FT *prow = (FT *)(zs + (size_t)k * SC);
    int32_t *ln = (int32_t *)(prow + 2 * 8 * C);
    int32_t *off = ln + SC;
    int32_t *st = off + SC + 1;
    int32_t *rowat = st + SC;
    for (int64_t node = blockIdx.x; node < nnode; node += gridDim.x) {
        const int32_t c0 = (int32_t)(node * k);
        const int32_t i0 = clist[c0];
        const int32_t n0 = nptr[c0];
        const int s = nptr[c0 + 1] - n0;
        if (s < s_lo || s > s_hi) continue;      // outside this launch's size range
        bool ok = s <= SC;
        for (int a = 1; a < k; ++a)
            ok = ok && clist[c0 + a] == i0 + a && nptr[c0 + a + 1] - nptr[c0 + a] == s;
        if (!ok) {
            if (lane == 0) atomicAdd(bad, 1);
            continue;
        }
        const int32_t *l = nbr + n0;
        if (lane < k) flags[c0 + lane] = 0;
        __syncthreads();
        for (int idx = lane; idx < s * s; idx += 64) Mg[idx] = 0.0;
        for (int idx = lane; idx < k * s; idx += 64) f[idx] = 0.0;
        for (int p = lane; p < s; p += 64) ln[p] = l[p];
        __syncthreads();
        gather_wave<8, double>(lane, s, ln, off, st, rp, cj, v, Mg, s, nullptr);
        for (int a = 0; a < k; ++a)
            for (int e = rp[i0 + a] + lane; e < rp[i0 + a + 1]; e += 64) {
                int p = bsearch_i32(ln, s, cj[e]);
                if (p >= 0) f[a * s + p] = -v[e];
            }
        __syncthreads();
        double rs = 0.0;
        for (int p = lane; p < s; p += 64) {
            double acc = 0.0;
            for (int q = 0; q < s; ++q) acc += fabs(Mg[p * s + q]);
            rs = fmax(rs, acc);
        }
        const double tol = SING_TOL * team_max<64>(rs);
        FT m[R][C];
        FT cur[R];
        int pos[R];
#pragma unroll
        for (int i = 0; i < R; ++i) {
            const int r = lr + 8 * i;
            pos[i] = r < s ? r : -1;
#pragma unroll
            for (int j = 0; j < R; ++j) {
                const int q = lq + 8 * j;
                m[i][j] = (r < s && q < s) ? (FT)Mg[r * s + q] : (FT)0;
            }
            m[i][R] = (r < s && lq < k) ? (FT)f[lq * s + r] : (FT)0;
            cur[i] = r < s ? (FT)Mg[r * s] : (FT)0;
        }
        bool singular = false;
#pragma unroll
        for (int jb = 0; jb < R; ++jb) {
#pragma unroll 1
            for (int kl = 0; kl < 8; ++kl) {
                const int kk = 8 * jb + kl;
                if (kk >= s) break;
                // arg-max over the unused rows, then across the rows of lanes
                double pv = -1.0;
                int key = INT_MAX;
                FT pval = (FT)0;
#pragma unroll
                for (int i = 0; i < R; ++i) {
                    const double a = fabs((double)cur[i]);
                    const int ki = pos[i] * 256 + lr + 8 * i;
                    if (pos[i] >= kk && (a > pv || (a == pv && ki < key))) {
                        pv = a;
                        key = ki;
                        pval = cur[i];
                    }
                }
#pragma unroll
                for (int o = 8; o < 64; o <<= 1) {
                    const double ov = __shfl_xor(pv, o);
                    const int ok2 = __shfl_xor(key, o);
                    const FT oval = __shfl_xor(pval, o);
                    if (ov > pv || (ov == pv && ok2 < key)) { pv = ov; key = ok2; pval = oval; }
                }
                key = __builtin_amdgcn_readfirstlane(key);
                // (no candidate at all, key INT_MAX, only with a NaN norm)
                if (__builtin_amdgcn_readfirstlane(pv <= tol || key == INT_MAX ? 1 : 0)) {
                    singular = true;
                    break;
                }
                const int pp = key >> 8;
                // exchange positions kk and pp
#pragma unroll
                for (int i = 0; i < R; ++i)
                    pos[i] = pos[i] == kk ? pp : (pos[i] == pp ? kk : pos[i]);
                FT mult[R];
#pragma unroll
                for (int i = 0; i < R; ++i) mult[i] = cur[i] / pval;
                // the pivot row through LDS: its row of lanes writes it (the
                // pivot is the row now at position kk; selecting its slot by
                // a test on each slot keeps m out of indexed memory)
                FT *pb = prow + (kk & 1) * 8 * C;
#pragma unroll
                for (int i = 0; i < R; ++i)
                    if (pos[i] == kk) {
#pragma unroll
                        for (int j = 0; j < C; ++j)
                            if (j >= jb) pb[j * 8 + lq] = m[i][j];
                    }
                wave_lds_sync();
                FT pj[C];
#pragma unroll
                for (int j = 0; j < C; ++j) pj[j] = j >= jb ? pb[j * 8 + lq] : (FT)0;
#pragma unroll
                for (int i = 0; i < R; ++i) {
                    if (pos[i] > kk) {
                        const FT mu = mult[i];
                        m[i][jb] = lq > kl ? m[i][jb] - mu * pj[jb]
                                           : (lq == kl ? mu : m[i][jb]);
#pragma unroll
                        for (int j = 0; j < R; ++j)
                            if (j > jb) m[i][j] -= mu * pj[j];
                        m[i][R] = lq < k ? m[i][R] - mu * pj[R] : m[i][R];
                    }
                }
                // the next column along each row of lanes
                if (kl < 7) {
#pragma unroll
                    for (int i = 0; i < R; ++i) cur[i] = __shfl(m[i][jb], lr * 8 + kl + 1);
                } else if (jb + 1 < R) {
#pragma unroll
                    for (int i = 0; i < R; ++i) cur[i] = __shfl(m[i][jb + 1 < R ? jb + 1 : jb], lr * 8);
                }
            }
            if (singular) break;
        }
        if (singular) {
            if (lane == 0) {
                const int32_t o = atomicAdd(nsing, k);
                for (int a = 0; a < k; ++a) {
                    flags[c0 + a] = 1;
                    sing[o + a] = c0 + a;
                }
            }
            __syncthreads();
            continue;
        }
        // the row at each position, read per step by readlane
        if (lq == 0) {
#pragma unroll
            for (int i = 0; i < R; ++i)
                if (pos[i] >= 0) rowat[pos[i]] = lr + 8 * i;
        }
        wave_lds_sync();
        const int ra0 = lane < s ? rowat[lane] : 0;
        const int ra1 = (SC > 64 && 64 + lane < s) ? rowat[64 + lane] : 0;
        // solution entries q = lr + 8i of right-hand side lq (lanes lq < k)
        double zr[R];
#pragma unroll
        for (int i = 0; i < R; ++i) zr[i] = 0.0;
        for (int pass = 0; pass < (MIXED && s > 0 ? 2 : 1); ++pass) {
            if (pass == 1) {
                // residual f - M z in double from the gathered matrix, each
                // entry summed over the columns from the last down; a lane
                // runs its entries side by side
                if (lq < k) {
#pragma unroll
                    for (int i = 0; i < R; ++i) {
                        const int q = lr + 8 * i;
                        if (q < s) zs[lq * s + q] = zr[i];
                    }
                }
                wave_lds_sync();
                constexpr int NT = (8 * SC + 63) / 64;     // entries per lane, k <= 8
                const SmallDiv ds(s > 0 ? s : 1);
                double acc[NT];
                int bm[NT], bz[NT];
#pragma unroll
                for (int t = 0; t < NT; ++t) {
                    const int idx = min(lane + 64 * t, k * s - 1);
                    const int a = ds.quot(idx), p = idx - a * s;
                    bm[t] = p * s;
                    bz[t] = a * s;
                    acc[t] = f[idx];
                }
                for (int q = s - 1; q >= 0; --q) {
#pragma unroll
                    for (int t = 0; t < NT; ++t) acc[t] -= Mg[bm[t] + q] * zs[bz[t] + q];
                }
                wave_lds_sync();
#pragma unroll
                for (int t = 0; t < NT; ++t)
                    if (lane + 64 * t < k * s) f[lane + 64 * t] = acc[t];
                wave_lds_sync();
                // the residual as right-hand side (row r takes residual r:
                // rows never moved), then forward substitution with L
#pragma unroll
                for (int i = 0; i < R; ++i) {
                    const int r = lr + 8 * i;
                    m[i][R] = (r < s && lq < k) ? (FT)f[lq * s + r] : (FT)0;
                }
#pragma unroll
                for (int jb = 0; jb < R; ++jb) {
#pragma unroll 1
                    for (int kl = 0; kl < 8; ++kl) {
                        const int kk = 8 * jb + kl;
                        if (kk >= s) break;
                        const int ph = __builtin_amdgcn_readlane(kk < 64 ? ra0 : ra1, kk & 63);
                        FT wl = (FT)0;
#pragma unroll
                        for (int i = 0; i < R; ++i) wl = pos[i] == kk ? m[i][R] : wl;
                        const FT wk = __shfl(wl, (ph & 7) * 8 + lq);
#pragma unroll
                        for (int i = 0; i < R; ++i) {
                            const FT lv = __shfl(m[i][jb], lr * 8 + kl);
                            const FT t = m[i][R] - lv * wk;
                            m[i][R] = (lq < k && pos[i] > kk) ? t : m[i][R];
                        }
                    }
                }
            }
            // back substitution: z_kk = w(row at kk) / U(kk, kk), then the
            // rows above remove column kk
#pragma unroll
            for (int jb = R - 1; jb >= 0; --jb) {
#pragma unroll 1
                for (int kl = 7; kl >= 0; --kl) {
                    const int kk = 8 * jb + kl;
                    if (kk >= s) continue;
                    const int ph = __builtin_amdgcn_readlane(kk < 64 ? ra0 : ra1, kk & 63);
                    FT ucol[R];
#pragma unroll
                    for (int i = 0; i < R; ++i) ucol[i] = __shfl(m[i][jb], lr * 8 + kl);
                    FT num = (FT)0, den = (FT)1;
#pragma unroll
                    for (int i = 0; i < R; ++i) {
                        num = pos[i] == kk ? m[i][R] : num;
                        den = pos[i] == kk ? ucol[i] : den;
                    }
                    const FT zk = __shfl(num / den, (ph & 7) * 8 + lq);
                    if (lr == kl) zr[jb] = pass == 0 ? (double)zk : zr[jb] + (double)zk;
#pragma unroll
                    for (int i = 0; i < R; ++i) {
                        const FT t = m[i][R] - ucol[i] * zk;
                        m[i][R] = (lq < k && pos[i] >= 0 && pos[i] < kk) ? t : m[i][R];
                    }
                }
            }
        }
        // rows of R: N with the identity entry at the row's place
        int ip = 0;
        for (int q = lane; q < s; q += 64) ip += (ln[q] < i0) ? 1 : 0;
        ip = team_sum_int<64>(ip);
        if (lq < k) {
#pragma unroll
            for (int i = 0; i < R; ++i) {
                const int q = lr + 8 * i;
                if (q < s) {
                    const int64_t o = (int64_t)nptr[c0 + lq] + c0 + lq + q + (q >= ip ? 1 : 0);
                    r_cj[o] = ln[q];
                    r_v[o] = zr[i];
                }
            }
        }
        if (lane < k) {
            const int64_t o = (int64_t)nptr[c0 + lane] + c0 + lane + ip;
            r_cj[o] = i0 + lane;
            r_v[o] = 1.0;
        }
        __syncthreads();
    }
}

// The one-wave bucket: a fixed grid striding over the bucket's length on
// the device, one global slab per block.
template <bool MIXED>
__global__ void __launch_bounds__(64)
k_local_wave(const int32_t *cnt, const int32_t *list, const int32_t *clist,
             const int32_t *nptr, const int32_t *nbr, const int32_t *rp, const int32_t *cj,
             const double *v, int32_t *r_cj, double *r_v, int8_t *flags, int32_t *sing,
             int32_t *nsing, double *gscratch, int32_t smax, int32_t cap) {
    extern __shared__ double dyn[];
    const int32_t n = cnt[4];
    double *slab = gscratch ? gscratch + (size_t)blockIdx.x * (size_t)smax * (size_t)smax * 3
                            : nullptr;
    for (int64_t t = blockIdx.x; t < n; t += gridDim.x) {
        wave_solve<MIXED>(list[t], clist, nptr, nbr, rp, cj, v, r_cj, r_v, flags, sing, nsing,
                          dyn, slab, smax, cap);
        __syncthreads();
    }
}

// Minimal-norm least squares for flagged systems (footnote of Sec. 3.1):
// one-sided Jacobi SVD, W = M V with orthogonal columns, then
// z = sum_{sigma_j > cut} (w_j . f / sigma_j^2) v_j, cut = eps s sigma_max.
// One wave per system, W and V column-major in global scratch.
__global__ void __launch_bounds__(64)
k_local_lstsq(const int32_t *list, int32_t nlist, const int32_t *clist,
              const int32_t *nptr, const int32_t *nbr, const int32_t *rp,
              const int32_t *cj, const double *v, int32_t *r_cj, double *r_v,
              double *gscratch, int32_t smax) {
    int lane = threadIdx.x;
    int32_t b = blockIdx.x;
    if (b >= nlist) return;
    int32_t c = list[b];
    int32_t i = clist[c];
    int32_t n0 = nptr[c];
    int s = nptr[c + 1] - n0;
    int32_t rbase = n0 + c;
    const int32_t *l = nbr + n0;
    size_t ss = (size_t)smax * smax;
    double *W = gscratch + (size_t)b * (2 * ss + 2 * (size_t)smax);
    double *V = W + ss;
    double *f = V + ss;
    double *z = f + smax;
    for (int idx = lane; idx < s * s; idx += 64) {
        W[idx] = 0.0;
        V[idx] = ((idx % s) == (idx / s)) ? 1.0 : 0.0;
    }
    for (int p = lane; p < s; p += 64) { f[p] = 0.0; z[p] = 0.0; }
    __syncthreads();
    // W column p, row q = M[q][p] = a(l_p, l_q)  (column-major: W[p*s + q])
    for (int p = lane; p < s; p += 64) {
        int r = l[p];
        for (int e = rp[r]; e < rp[r + 1]; ++e) {
            int q = bsearch_i32(l, s, cj[e]);
            if (q >= 0) W[p * s + q] = v[e];
        }
    }
    for (int e = rp[i] + lane; e < rp[i + 1]; e += 64) {
        int p = bsearch_i32(l, s, cj[e]);
        if (p >= 0) f[p] = -v[e];
    }
    __syncthreads();
    for (int sweep = 0; sweep < 60; ++sweep) {
        int rotated = 0;
        for (int j = 0; j < s - 1; ++j) {
            for (int k = j + 1; k < s; ++k) {
                double a = 0.0, bb = 0.0, g = 0.0;
                for (int q = lane; q < s; q += 64) {
                    double wj = W[j * s + q], wk = W[k * s + q];
                    a += wj * wj; bb += wk * wk; g += wj * wk;
                }
                a = team_sum<64>(a); bb = team_sum<64>(bb); g = team_sum<64>(g);
                if (fabs(g) <= DBL_EPSILON * sqrt(a * bb) || g == 0.0) continue;
                rotated = 1;
                double zeta = (bb - a) / (2.0 * g);
                double t = (zeta >= 0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                double cs = 1.0 / sqrt(1.0 + t * t), sn = cs * t;
                for (int q = lane; q < s; q += 64) {
                    double wj = W[j * s + q], wk = W[k * s + q];
                    W[j * s + q] = cs * wj - sn * wk;
                    W[k * s + q] = sn * wj + cs * wk;
                    double vj = V[j * s + q], vk = V[k * s + q];
                    V[j * s + q] = cs * vj - sn * vk;
                    V[k * s + q] = sn * vj + cs * vk;
                }
                __syncthreads();
            }
        }
        if (!rotated) break;
    }
    double smx = 0.0;
    for (int j = 0; j < s; ++j) {
        double a = 0.0;
        for (int q = lane; q < s; q += 64) a += W[j * s + q] * W[j * s + q];
        a = team_sum<64>(a);
        smx = fmax(smx, sqrt(a));
    }
    double cut = DBL_EPSILON * (double)s * smx;
    for (int j = 0; j < s; ++j) {
        double a = 0.0, d = 0.0;
        for (int q = lane; q < s; q += 64) {
            double wj = W[j * s + q];
            a += wj * wj;
            d += wj * f[q];
        }
        a = team_sum<64>(a);
        d = team_sum<64>(d);
        if (sqrt(a) <= cut) continue;
        double coef = d / a;
        for (int q = lane; q < s; q += 64) z[q] += coef * V[j * s + q];
        __syncthreads();
    }
    __syncthreads();
    int ip = 0;
    for (int q = lane; q < s; q += 64) ip += (l[q] < i) ? 1 : 0;
    ip = team_sum_int<64>(ip);
    for (int q = lane; q < s; q += 64) {
        int o = rbase + q + (q >= ip ? 1 : 0);
        r_cj[o] = l[q];
        r_v[o] = z[q];
    }
    if (lane == 0) {
        r_cj[rbase + ip] = i;
        r_v[rbase + ip] = 1.0;
    }
}


// Algorithmic cost of the local solves, split at s <= lim / s > lim:
// bytes = (|row i| + sum_{j in N_i} |row j|) 12 + (s + 1) 12 (gather and R
// row), flops = 2 s^3 / 3 + 2 s^2 (LU and triangular solves).
__global__ void __launch_bounds__(256)
k_local_cost(int32_t nc, const int32_t *clist, const int32_t *nptr,
             const int32_t *nbr, const int32_t *rp, int32_t lim, double *acc,
             int32_t knode) {
    __shared__ double sh[4][256];
    int32_t c = blockIdx.x * blockDim.x + threadIdx.x;
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    if (c < nc && knode > 1 && c % knode != 0) {
        // a node's later rows: their right-hand side, substitutions and row
        // of R (the gather and the factorisation are the first row's)
        int32_t i = clist[c];
        double ds = (double)(nptr[c + 1] - nptr[c]);
        v[0] = 12.0 * (double)(rp[i + 1] - rp[i]) + 12.0 * (ds + 1);
        v[1] = 2.0 * ds * ds;
    } else if (c < nc) {
        int32_t i = clist[c];
        int s = nptr[c + 1] - nptr[c];
        double rows = (double)(rp[i + 1] - rp[i]);
        for (int q = 0; q < s; ++q) {
            int j = nbr[nptr[c] + q];
            rows += (double)(rp[j + 1] - rp[j]);
        }
        double ds = (double)s;
        int k = (s <= lim) ? 0 : 2;
        v[k] = 12.0 * rows + 12.0 * (s + 1);
        v[k + 1] = 2.0 * ds * ds * ds / 3.0 + 2.0 * ds * ds;
    }
    for (int k = 0; k < 4; ++k) sh[k][threadIdx.x] = v[k];
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o)
            for (int k = 0; k < 4; ++k) sh[k][threadIdx.x] += sh[k][threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int k = 0; k < 4; ++k) atomicAdd(acc + k, sh[k][0]);
}

// ---------------------------------------------------------------------------
// Bucket edges.  Fixed by the caller (set_local_buckets), else chosen per
// level shape (precision, size class, mean row length, largest system) by
// timing a few candidates the first time the process meets that shape.
// Every candidate yields the same z bit for bit; only the speed differs.
// ---------------------------------------------------------------------------
namespace {
std::mutex g_bk_mu;
bool g_bk_fixed = false;
Buckets g_bk_edges{{4, 8, 16, 32}, 0};
std::map<std::array<int32_t, 4>, Buckets> g_bk_cache;
const Buckets BK_CANDIDATES[] = {{{4, 8, 16, 32}, 0}, {{0, 8, 16, 32}, 0},
                                 {{4, 8, 16, 32}, 1}, {{0, 8, 16, 32}, 1},
                                 {{2, 6, 12, 32}, 0}, {{4, 8, 12, 24}, 0},
                                 {{4, 8, 16, 16}, 0}, {{0, 8, 16, 16}, 1}};

// LAIR_TUNE_LOG=1 prints every tuning measurement to stderr
bool tune_log() {
    static const bool on = [] {
        const char *e = getenv("LAIR_TUNE_LOG");
        return e && e[0] == '1';
    }();
    return on;
}

int ilog2_floor(int64_t v) {
    int l = 0;
    while (v > 1) { v >>= 1; ++l; }
    return l;
}

// resident blocks of the persistent kernel on the current device
unsigned persist_resident(bool mixed) {
    static int cache[2][16] = {};
    int dev = 0;
    LAIR_HIP(hipGetDevice(&dev));
    int &c = cache[mixed ? 1 : 0][dev & 15];
    if (c == 0) {
        int ncu = 0, per = 0;
        LAIR_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
        if (mixed)
            LAIR_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_local_persist<true>,
                                                                  PERSIST_BS, 0));
        else
            LAIR_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_local_persist<false>,
                                                                  PERSIST_BS, 0));
        c = std::max(1, ncu) * std::max(1, per);
    }
    return (unsigned)c;
}
}  // namespace

void set_local_buckets(const int32_t *e) {
    std::lock_guard<std::mutex> g(g_bk_mu);
    if (!e) {
        g_bk_fixed = false;
        return;
    }
    if (!(e[0] >= 0 && e[0] <= 4 && e[1] >= e[0] && e[1] <= 8 && e[2] >= e[1] && e[2] <= 16 &&
          e[3] >= e[2] && e[3] <= 32 && (e[4] == 0 || e[4] == 1)))
        fail(LAIR_EINVAL, "bucket edges must satisfy 0 <= e0 <= 4, e0 <= e1 <= 8, "
                          "e1 <= e2 <= 16, e2 <= e3 <= 32, and the fused flag be 0 or 1");
    g_bk_fixed = true;
    for (int k = 0; k < 4; ++k) g_bk_edges.e[k] = e[k];
    g_bk_edges.fused = e[4];
}

namespace {
struct LocalRun {
    int32_t nc;
    const int32_t *clist, *nptr, *nbr, *rp, *cj;
    const double *v;
    bool mixed;
    int32_t smax;
    LocalSolveOut out;
    int32_t *cnt, *lists, *sing;          // cnt[0..4] buckets, cnt[5] ticket, cnt[6] nsing
    double *gscratch;
    unsigned gw;
};

// Binning, the persistent kernel, the 32-lane and one-wave buckets: no
// host synchronisation.
void run_buckets(LocalRun &r, const Buckets &bk, hipStream_t s) {
    r.cnt = reinterpret_cast<int32_t *>(zeroed_slots(4, s));   // 7 zeroed counters
    int32_t *ticket = r.cnt + 5, *nsing = r.cnt + 6;
    LAIR_LAUNCH(k_local_bin, dim3(blocks_for(r.nc, 256)), dim3(256), 0, s, r.nc, r.nptr, bk,
                r.cnt, r.lists, r.out.flags);
    LAIR_LAUNCH_CHECK();
    const int32_t *l1 = r.lists, *l8 = r.lists + (int64_t)r.nc,
                  *l16 = r.lists + 2 * (int64_t)r.nc, *l32 = r.lists + 3 * (int64_t)r.nc;
    // teams of T over bucket b, a team for every C-point at most
    auto teams = [&](auto tag, int b, const int32_t *list) {
        constexpr int T = decltype(tag)::value;
        constexpr int BS = T >= 32 ? 128 : 256;
        const unsigned g = (unsigned)((r.nc + BS / T - 1) / (BS / T));
        if (r.mixed)
            LAIR_LAUNCH((k_local_teams<T, true>), dim3(g), dim3(BS), 0, s, r.cnt, b, list,
                        r.clist, r.nptr, r.nbr, r.rp, r.cj, r.v, r.out.r_cj, r.out.r_v,
                        r.out.flags, r.sing, nsing);
        else
            LAIR_LAUNCH((k_local_teams<T, false>), dim3(g), dim3(BS), 0, s, r.cnt, b, list,
                        r.clist, r.nptr, r.nbr, r.rp, r.cj, r.v, r.out.r_cj, r.out.r_v,
                        r.out.flags, r.sing, nsing);
        LAIR_LAUNCH_CHECK();
    };
    if (bk.fused) {
        const unsigned gp = (unsigned)std::min<int64_t>(persist_resident(r.mixed),
                                                        std::max<int64_t>(1, (r.nc + 15) / 16));
        if (r.mixed)
            LAIR_LAUNCH(k_local_persist<true>, dim3(gp), dim3(PERSIST_BS), 0, s, r.cnt, r.lists,
                        r.nc, ticket, r.clist, r.nptr, r.nbr, r.rp, r.cj, r.v, r.out.r_cj,
                        r.out.r_v, r.out.flags, r.sing, nsing);
        else
            LAIR_LAUNCH(k_local_persist<false>, dim3(gp), dim3(PERSIST_BS), 0, s, r.cnt,
                        r.lists, r.nc, ticket, r.clist, r.nptr, r.nbr, r.rp, r.cj, r.v,
                        r.out.r_cj, r.out.r_v, r.out.flags, r.sing, nsing);
        LAIR_LAUNCH_CHECK();
    } else {
        if (r.mixed)
            LAIR_LAUNCH(k_local_lane<true>, dim3(blocks_for(r.nc, 256)), dim3(256), 0, s, r.cnt,
                        l1, r.clist, r.nptr, r.nbr, r.rp, r.cj, r.v, r.out.r_cj, r.out.r_v,
                        r.out.flags, r.sing, nsing);
        else
            LAIR_LAUNCH(k_local_lane<false>, dim3(blocks_for(r.nc, 256)), dim3(256), 0, s,
                        r.cnt, l1, r.clist, r.nptr, r.nbr, r.rp, r.cj, r.v, r.out.r_cj,
                        r.out.r_v, r.out.flags, r.sing, nsing);
        LAIR_LAUNCH_CHECK();
        if (r.smax > bk.e[0]) teams(std::integral_constant<int, 8>{}, 1, l8);
        if (r.smax > bk.e[1]) teams(std::integral_constant<int, 16>{}, 2, l16);
    }
    if (r.smax > bk.e[2]) teams(std::integral_constant<int, 32>{}, 3, l32);
    if (r.smax > bk.e[3]) {
        const int32_t cap = r.smax < WSMAX ? r.smax : WSMAX;
        const int32_t *l4 = r.lists + 4 * (int64_t)r.nc;
        const size_t lds = r.mixed ? wave_lds_bytes<float>(cap) : wave_lds_bytes<double>(cap);
        if (r.mixed)
            LAIR_LAUNCH(k_local_wave<true>, dim3(r.gw), dim3(64), lds, s, r.cnt, l4, r.clist,
                        r.nptr, r.nbr, r.rp, r.cj, r.v, r.out.r_cj, r.out.r_v, r.out.flags,
                        r.sing, nsing, r.gscratch, r.smax, cap);
        else
            LAIR_LAUNCH(k_local_wave<false>, dim3(r.gw), dim3(64), lds, s, r.cnt, l4, r.clist,
                        r.nptr, r.nbr, r.rp, r.cj, r.v, r.out.r_cj, r.out.r_v, r.out.flags,
                        r.sing, nsing, r.gscratch, r.smax, cap);
        LAIR_LAUNCH_CHECK();
    }
}
}  // namespace

// Local solves of one level: bucket edges (fixed, cached or tuned), one
// pass over the buckets, one readback (bucket sizes and the number of
// singular systems), then least squares for the singular ones.
bool node_solves_fit(int32_t k, int32_t smax, int32_t precision) {
    if (k < 2) return false;
    // the smallest systems must fit in LDS; larger ones go to the slab
    const size_t b = precision == LAIR_MIXED ? node_lds_bytes<float>(1, k)
                                             : node_lds_bytes<double>(1, k);
    return b <= NODE_LDS_MAX && smax >= 0;
}

int64_t local_solves(int32_t nc, const int32_t *clist, const int32_t *nptr,
                     const int32_t *nbr, const int32_t *rp, const int32_t *cj,
                     const double *v, int32_t precision, int32_t smax, double mean_row,
                     LocalSolveOut out, hipStream_t s, int32_t *edges_used,
                     Readback *rb_extra, int32_t knode) {
    if (nc == 0) {
        if (rb_extra) rb_extra->run();
        return 0;
    }
    const bool mixed = (precision == LAIR_MIXED);
    if (knode > 1) {
        // one factorisation per node, k right-hand sides (the caller checked
        // node_solves_fit)
        if (nc % knode != 0 || !node_solves_fit(knode, smax, precision))
            fail(LAIR_EINVAL, "node local solves: %d C-rows, nodes of %d, systems up to %d",
                 nc, knode, smax);
        DevArr<int32_t> sing;
        sing.alloc((size_t)nc, s);
        int32_t *cnt = reinterpret_cast<int32_t *>(zeroed_slots(4, s));   // [0] bad, [6] nsing
        const int32_t nnode = nc / knode;
        double cost[4] = {0, 0, 0, 0};
        if (prof_selected("local_node")) {
            DevArr<double> acc;
            acc.alloc(4, s);
            LAIR_HIP(hipMemsetAsync(acc.get(), 0, 4 * sizeof(double), s));
            LAIR_LAUNCH(k_local_cost, dim3(blocks_for(nc, 256)), dim3(256), 0, s, nc, clist,
                        nptr, nbr, rp, WSMAX, acc.get(), knode);
            LAIR_LAUNCH_CHECK();
            Readback rb(s);
            rb.add(cost, acc.get(), sizeof(cost));
            rb.run();
        }
        // Systems up to 72 rows run with M in registers, in three size
        // classes (the smaller tiles leave more waves per CU); the LDS form
        // takes the rest.  Its work arrays: in at most 64 KB of LDS (several
        // blocks per CU) when it takes every system, all of them up to `cap`
        // rows, all but the double copy of M (MIXED) up to `cap_nomd`; larger
        // systems use a global slab per block, the grid then kept small
        // enough for 256 MB of slabs.  When it takes only the few systems
        // above 72 rows it gets the LDS of a whole CU, which keeps them out
        // of the slab.  (For the bulk, blocks with the whole LDS of a CU ran
        // slower: one wave per CU leaves the elimination's latency exposed.)
        const bool reg = knode <= 8 && !env_flag("LAIR_NODE_LDS_SOLVES");
        size_t budget = NODE_LDS_MAX;
        if (reg && smax > 72) {
            const size_t big = mixed ? std::max(node_lds_bytes<float>(smax, knode),
                                                node_lds_bytes<float>(smax, knode, false))
                                     : node_lds_bytes<double>(smax, knode);
            const size_t want = std::min<size_t>(big, NODE_LDS_CU);
            const void *kern = mixed ? (const void *)k_local_node<true>
                                     : (const void *)k_local_node<false>;
            if (want > NODE_LDS_MAX &&
                hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)want) == hipSuccess)
                budget = want;
            (void)hipGetLastError();
        }
        const int sm1 = std::max(1, smax);
        const int cap = mixed ? node_cap_for<float>(budget, knode, true, sm1)
                              : node_cap_for<double>(budget, knode, true, sm1);
        const int cap_nomd = mixed ? node_cap_for<float>(budget, knode, false, sm1) : cap;
        const size_t lds = mixed ? std::max(node_lds_bytes<float>(cap, knode),
                                            node_lds_bytes<float>(cap_nomd, knode, false))
                                 : node_lds_bytes<double>(cap, knode);
        unsigned g = (unsigned)std::min<int64_t>(nnode, 8192);
        DevArr<double> gscratch;
        int64_t slab = 0;
        if (smax > cap_nomd) {
            const size_t sb = mixed ? node_lds_bytes<float>(smax, knode)
                                    : node_lds_bytes<double>(smax, knode);
            slab = (int64_t)((sb + 255) / 256 * 256 / sizeof(double));
        } else if (smax > cap) {
            slab = ((int64_t)smax * smax + 31) / 32 * 32;   // the double copies of M only
        }
        if (slab) {
            g = (unsigned)std::max<int64_t>(
                1, std::min<int64_t>(g, ((int64_t)256 << 20) / (slab * (int64_t)sizeof(double))));
            gscratch.alloc((size_t)g * slab, s);
        }
        {
            ProfScope ps("local_node", s, cost[0], cost[1]);
            const unsigned gr = (unsigned)std::min<int64_t>(nnode, 8192);
            int lo = 0;
            if (reg) {
                auto run = [&](auto kern, int hi, size_t bytes, unsigned grid, double *slabs) {
                    if (lo > smax) return;
                    LAIR_LAUNCH(kern, dim3(grid), dim3(64), bytes, s, nnode, knode, clist, nptr,
                                nbr, rp, cj, v, out.r_cj, out.r_v, out.flags, sing.get(),
                                cnt + 6, cnt, lo, hi, slabs);
                    LAIR_LAUNCH_CHECK();
                    lo = hi + 1;
                };
                if (mixed) {
                    run(k_local_node_reg<3, true, false>, 24, node_reg_lds_bytes<3>(knode), gr,
                        nullptr);
                    run(k_local_node_reg<5, true, false>, 40, node_reg_lds_bytes<5>(knode), gr,
                        nullptr);
                    if (lo <= smax) {
                        // the largest class keeps its double matrix in a
                        // global slab per block (then registers, not LDS,
                        // bound the waves per CU)
                        const unsigned g9 = (unsigned)std::min<int64_t>(nnode, 2048);
                        DevArr<double> slabs;
                        slabs.alloc((size_t)g9 * 72 * 72, s);
                        run(k_local_node_reg<9, true, true>, 72,
                            node_reg_lds_bytes<9>(knode, false), g9, slabs.get());
                    }
                } else {
                    run(k_local_node_reg<3, false, false>, 24, node_reg_lds_bytes<3>(knode), gr,
                        nullptr);
                    run(k_local_node_reg<5, false, false>, 40, node_reg_lds_bytes<5>(knode), gr,
                        nullptr);
                    if (lo <= smax) {
                        const unsigned g9 = (unsigned)std::min<int64_t>(nnode, 2048);
                        DevArr<double> slabs;
                        slabs.alloc((size_t)g9 * 72 * 72, s);
                        run(k_local_node_reg<9, false, true>, 72,
                            node_reg_lds_bytes<9>(knode, false), g9, slabs.get());
                    }
                }
            }
            if (lo <= smax) {
                if (mixed)
                    LAIR_LAUNCH(k_local_node<true>, dim3(g), dim3(64), lds, s, nnode, knode,
                                clist, nptr, nbr, rp, cj, v, out.r_cj, out.r_v, out.flags,
                                sing.get(), cnt + 6, cnt, cap, cap_nomd, gscratch.get(), slab,
                                smax, lo, smax);
                else
                    LAIR_LAUNCH(k_local_node<false>, dim3(g), dim3(64), lds, s, nnode, knode,
                                clist, nptr, nbr, rp, cj, v, out.r_cj, out.r_v, out.flags,
                                sing.get(), cnt + 6, cnt, cap, cap_nomd, gscratch.get(), slab,
                                smax, lo, smax);
                LAIR_LAUNCH_CHECK();
            }
        }
        int32_t h[7] = {0, 0, 0, 0, 0, 0, 0};
        {
            Readback own(s);
            Readback &rb = rb_extra ? *rb_extra : own;
            rb.add(h, cnt, sizeof(h));
            rb.run();
        }
        if (h[0] > 0)
            fail(LAIR_EINVAL, "%d C-node(s) whose rows do not share one neighbourhood", h[0]);
        const int32_t nsing = h[6];
        if (nsing > 0) {
            DevArr<double> scratch;
            scratch.alloc((size_t)nsing * (2 * (size_t)smax * smax + 2 * (size_t)smax), s);
            ProfScope ps_ls("local_lstsq", s, 0.0);
            LAIR_LAUNCH(k_local_lstsq, dim3((unsigned)nsing), dim3(64), 0, s,
                        sing.get(), nsing, clist, nptr, nbr, rp, cj, v, out.r_cj, out.r_v,
                        scratch.get(), smax);
            LAIR_LAUNCH_CHECK();
            LAIR_HIP(hipStreamSynchronize(s));
        }
        return nsing;
    }
    DevArr<int32_t> work;
    work.alloc((size_t)nc * (NBUCKET + 1) + 8, s);
    LocalRun r{nc, clist, nptr, nbr, rp, cj, v, mixed, smax, out, nullptr,
               work.get() + 8, work.get() + 8 + (size_t)nc * NBUCKET, nullptr, 1};
    // the one-wave bucket: a fixed grid; systems above WSMAX use a global
    // slab per block, the grid kept small enough for 256 MB of slabs
    DevArr<double> gscratch;
    {
        const int32_t cap = smax < WSMAX ? smax : WSMAX;
        int64_t gw = std::min<int64_t>(nc, 2048);
        if (smax > cap) {
            const int64_t slab = 3 * (int64_t)smax * smax * (int64_t)sizeof(double);
            gw = std::max<int64_t>(1, std::min<int64_t>(gw, ((int64_t)256 << 20) / slab));
            gscratch.alloc((size_t)gw * 3 * (size_t)smax * smax, s);
            r.gscratch = gscratch.get();
        }
        r.gw = (unsigned)gw;
    }
    double cost[4] = {0, 0, 0, 0};
    if (prof_selected("local_small") || prof_selected("local_wave")) {
        DevArr<double> acc;
        acc.alloc(4, s);
        LAIR_HIP(hipMemsetAsync(acc.get(), 0, 4 * sizeof(double), s));
        LAIR_LAUNCH(k_local_cost, dim3(blocks_for(nc, 256)), dim3(256), 0, s,
                           nc, clist, nptr, nbr, rp, 32, acc.get(), 1);
        LAIR_LAUNCH_CHECK();
        Readback rb(s);
        rb.add(cost, acc.get(), sizeof(cost));
        rb.run();
    }
    Buckets bk;
    bool tune = false;
    const std::array<int32_t, 4> key{mixed ? 1 : 0, ilog2_floor(nc),
                                     (int32_t)std::lround(mean_row), std::min(smax, 33)};
    {
        std::lock_guard<std::mutex> g(g_bk_mu);
        if (g_bk_fixed) {
            bk = g_bk_edges;
        } else {
            auto it = g_bk_cache.find(key);
            if (it != g_bk_cache.end()) bk = it->second;
            else tune = true;
        }
    }
    if (tune) {
        // every candidate runs TUNE_REPS times in turn (the first pass also
        // loads the kernels' code) and keeps its fastest time; each run
        // overwrites the same outputs with the same values
        constexpr int TUNE_REPS = 3;
        const int nk = (int)(sizeof(BK_CANDIDATES) / sizeof(BK_CANDIDATES[0]));
        std::vector<hipEvent_t> ev(2 * nk * TUNE_REPS, nullptr);
        for (auto &e : ev) LAIR_HIP(hipEventCreate(&e));
        for (int rep = 0; rep < TUNE_REPS; ++rep)
            for (int k = 0; k < nk; ++k) {
                LAIR_HIP(hipEventRecord(ev[2 * (rep * nk + k)], s));
                run_buckets(r, BK_CANDIDATES[k], s);
                LAIR_HIP(hipEventRecord(ev[2 * (rep * nk + k) + 1], s));
            }
        LAIR_HIP(hipStreamSynchronize(s));
        float best = 0.0f;
        int arg = 0;
        for (int k = 0; k < nk; ++k) {
            float mk = 0.0f;
            for (int rep = 1; rep < TUNE_REPS; ++rep) {
                float ms = 0.0f;
                LAIR_HIP(hipEventElapsedTime(&ms, ev[2 * (rep * nk + k)],
                                             ev[2 * (rep * nk + k) + 1]));
                mk = (rep == 1) ? ms : std::min(mk, ms);
            }
            if (k == 0 || mk < best) { best = mk; arg = k; }
            if (tune_log())
                fprintf(stderr, "lair tune: nc %d mean_row %.1f smax %d %s edges %d %d %d %d "
                        "fused %d: %.1f us\n", nc, mean_row, smax, mixed ? "mixed" : "fp64",
                        BK_CANDIDATES[k].e[0], BK_CANDIDATES[k].e[1], BK_CANDIDATES[k].e[2],
                        BK_CANDIDATES[k].e[3], BK_CANDIDATES[k].fused, 1e3 * mk);
        }
        for (auto &e : ev) (void)hipEventDestroy(e);
        bk = BK_CANDIDATES[arg];
        std::lock_guard<std::mutex> g(g_bk_mu);
        g_bk_cache[key] = bk;
    } else {
        ProfScope ps_small("local_small", s, cost[0] + cost[2], cost[1] + cost[3]);
        run_buckets(r, bk, s);
    }
    if (edges_used) {
        for (int k = 0; k < 4; ++k) edges_used[k] = bk.e[k];
        edges_used[4] = bk.fused;
    }
    int32_t h[7] = {0, 0, 0, 0, 0, 0, 0};
    {
        // the caller's pending items travel with this readback
        Readback own(s);
        Readback &rb = rb_extra ? *rb_extra : own;
        rb.add(h, r.cnt, sizeof(h));
        rb.run();
    }
    const int32_t nsing = h[6];
    if (nsing > 0) {
        DevArr<double> scratch;
        scratch.alloc((size_t)nsing * (2 * (size_t)smax * smax + 2 * (size_t)smax), s);
        ProfScope ps_ls("local_lstsq", s, 0.0);
        LAIR_LAUNCH(k_local_lstsq, dim3((unsigned)nsing), dim3(64), 0, s,
                           r.sing, nsing, clist, nptr, nbr, rp, cj, v, out.r_cj,
                           out.r_v, scratch.get(), smax);
        LAIR_LAUNCH_CHECK();
        LAIR_HIP(hipStreamSynchronize(s));
    }
    return nsing;
}

// ===========================================================================
// Interpolation.
// ===========================================================================
// One-point (Sec. 4): F-point i takes the value at its strongest C-neighbour
// (largest |a_ij| over strong C entries, smallest j on a tie); C-points
// inject.  pcol[i] = coarse column or -1.
__global__ void k_interp_1p(int32_t n, const int32_t *rp, const int32_t *cj,
                            const double *v, const uint8_t *sm,
                            const int8_t *cf, const int32_t *cidx,
                            int32_t *pcol) {
    int32_t i = (int32_t)xcd_block_id() * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (cf[i] == 1) { pcol[i] = cidx[i]; return; }
    int best = -1;
    double bv = -1.0;
    for (int p = rp[i]; p < rp[i + 1]; ++p) {
        int j = cj[p];
        if (!sm[p] || cf[j] != 1) continue;
        double a = fabs(v[p]);
        if (a > bv) { bv = a; best = j; }
    }
    pcol[i] = best >= 0 ? cidx[best] : -1;
}

void launch_interp_one_point(int32_t n, const int32_t *rp, const int32_t *cj,
                             const double *v, const uint8_t *smask,
                             const int8_t *cf, const int32_t *cidx,
                             int32_t *pcol, hipStream_t s) {
    LAIR_LAUNCH(k_interp_1p, dim3(blocks_for(n, 256)), dim3(256), 0, s,
                       n, rp, cj, v, smask, cf, cidx, pcol);
    LAIR_LAUNCH_CHECK();
}

__global__ void k_compact_1p(int32_t n, const int32_t *pcol, const int32_t *prp,
                             int32_t *pcj, double *pv) {
    int32_t i = (int32_t)xcd_block_id() * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (pcol[i] >= 0) {
        pcj[prp[i]] = pcol[i];
        pv[prp[i]] = 1.0;
    }
}

void launch_compact_one_point(int32_t n, const int32_t *pcol,
                              const int32_t *prp, int32_t *pcj, double *pv,
                              hipStream_t s) {
    LAIR_LAUNCH(k_compact_1p, dim3(blocks_for(n, 256)), dim3(256), 0, s,
                       n, pcol, prp, pcj, pv);
    LAIR_LAUNCH_CHECK();
}

// Classical direct interpolation (Stueben 2001): for F-point i with
// P_i = S_i n C, alpha = sum_{j!=i} a_ij^- / sum_{P_i} a_ik^-, beta likewise
// for positive entries, w_ik = -(alpha or beta) a_ik / a_ii; a sign class
// missing from P_i is lumped into the diagonal.  Columns follow A's order,
// which is increasing in coarse index.  One team of T lanes per row: the
// sums are team reductions and the fill compacts in order with a ballot.
// Direct weights of F row i in the row's order: w_ij = -(alpha or beta) a_ij / d
// for the strong C-points j (alpha for negative entries, beta otherwise).
template <int T>
__device__ __forceinline__ void interp_direct_write(int32_t i, int lo, int hi, int lane,
                                                    const int32_t *cj, const double *v,
                                                    const uint8_t *sm, const int8_t *cf,
                                                    const int32_t *cidx, int o, double alpha,
                                                    double beta, double d, int32_t *pcj,
                                                    double *pv) {
    for (int p0 = lo; p0 < hi; p0 += T) {
        int p = p0 + lane;
        int j = -1;
        double a = 0.0;
        bool take = false;
        if (p < hi) {
            j = cj[p];
            a = v[p];
            take = (j != i) && sm[p] && cf[j] == 1;
        }
        uint64_t bits = team_bits<T>(take);
        int before = __popcll(bits & ((1ull << lane) - 1ull));
        if (take) {
            pcj[o + before] = cidx[j];
            pv[o + before] = -(a < 0.0 ? alpha : beta) * a / d;
        }
        o += __popcll(bits);
    }
}

template <int T>
__global__ void __launch_bounds__(256)
k_interp_direct(int32_t n, const int32_t *rp, const int32_t *cj,
                const double *v, const uint8_t *sm, const int8_t *cf,
                const int32_t *cidx, bool fill, int32_t *cnt,
                const int32_t *prp, int32_t *pcj, double *pv, double *coef) {
    int64_t gt = xcd_block_id() * blockDim.x + threadIdx.x;
    int32_t i = (int32_t)(gt / T);
    int lane = (int)(gt % T);
    if (i >= n) return;
    if (cf[i] == 1) {
        if (lane == 0) {
            if (!fill) cnt[i] = 1;
            else { pcj[prp[i]] = cidx[i]; pv[prp[i]] = 1.0; }
        }
        return;
    }
    const int lo = rp[i], hi = rp[i + 1];
    if (fill && coef) {
        // the sizing pass kept alpha, beta and the lumped diagonal (0: no row)
        const double alpha = coef[3 * (int64_t)i], beta = coef[3 * (int64_t)i + 1];
        const double d = coef[3 * (int64_t)i + 2];
        if (d == 0.0) return;
        interp_direct_write<T>(i, lo, hi, lane, cj, v, sm, cf, cidx, prp[i], alpha, beta, d,
                               pcj, pv);
        return;
    }
    double diag = 0.0, sn = 0.0, sp = 0.0, pn = 0.0, pp = 0.0;
    int k = 0;
    for (int p = lo + lane; p < hi; p += T) {
        int j = cj[p];
        double a = v[p];
        if (j == i) { diag = a; continue; }
        if (a < 0.0) sn += a; else sp += a;
        if (sm[p] && cf[j] == 1) {
            if (a < 0.0) pn += a; else pp += a;
            ++k;
        }
    }
    diag = team_sum<T>(diag);
    sn = team_sum<T>(sn);
    sp = team_sum<T>(sp);
    pn = team_sum<T>(pn);
    pp = team_sum<T>(pp);
    k = team_sum_int<T>(k);
    double d = diag;
    if (pn == 0.0) d += sn;
    if (pp == 0.0) d += sp;
    bool empty = (k == 0 || d == 0.0);
    double alpha = (pn != 0.0) ? sn / pn : 0.0;
    double beta = (pp != 0.0) ? sp / pp : 0.0;
    if (!fill) {
        if (lane == 0) {
            cnt[i] = empty ? 0 : k;
            if (coef) {
                coef[3 * (int64_t)i] = alpha;
                coef[3 * (int64_t)i + 1] = beta;
                coef[3 * (int64_t)i + 2] = empty ? 0.0 : d;
            }
        }
        return;
    }
    if (empty) return;
    interp_direct_write<T>(i, lo, hi, lane, cj, v, sm, cf, cidx, prp[i], alpha, beta, d, pcj, pv);
}

void launch_interp_direct(int32_t n, const int32_t *rp, const int32_t *cj,
                          const double *v, const uint8_t *smask,
                          const int8_t *cf, const int32_t *cidx, bool fill,
                          int32_t *cnt, const int32_t *prp, int32_t *pcj,
                          double *pv, double mean_len, hipStream_t s, double *coef) {
    int t = team_for_mean(mean_len);
    if (t > 16) t = 16;
#define LAIR_ID(TT)                                                              \
    LAIR_LAUNCH(k_interp_direct<TT>, dim3(blocks_for((int64_t)n * TT, 256)), \
                       dim3(256), 0, s, n, rp, cj, v, smask, cf, cidx, fill, cnt, prp, \
                       pcj, pv, coef)
    switch (t) {
        case 2: LAIR_ID(2); break;
        case 4: LAIR_ID(4); break;
        case 8: LAIR_ID(8); break;
        default: LAIR_ID(16); break;
    }
#undef LAIR_ID
    LAIR_LAUNCH_CHECK();
}

// The strength of k_strength and the counting pass of k_interp_direct in one
// pass over each row, for a splitting known beforehand: the team shape, the
// loop over the row and the team sums are those of k_interp_direct, so cnt
// and coef are its values bit for bit (the strength does not depend on the
// team: a maximum and comparisons).
template <int T>
__global__ void __launch_bounds__(256)
k_strength_interp(int32_t n, const int32_t *rp, const int32_t *cj, const double *v,
                  double theta, int32_t kind, const int8_t *cf, uint8_t *smask,
                  int32_t *cnt, double *coef) {
    int64_t gt = xcd_block_id() * blockDim.x + threadIdx.x;
    int32_t i = (int32_t)(gt / T);
    int lane = (int)(gt % T);
    if (i >= n) return;
    const int lo = rp[i], hi = rp[i + 1];
    double m = 0.0;
    for (int p = lo + lane; p < hi; p += T)
        if (cj[p] != i) m = fmax(m, fabs(v[p]));
    m = team_max<T>(m);
    const double thr = theta * m;
    const bool frow = cf[i] != 1;
    double diag = 0.0, sn = 0.0, sp = 0.0, pn = 0.0, pp = 0.0;
    int k = 0;
    for (int p = lo + lane; p < hi; p += T) {
        const int j = cj[p];
        const double a = v[p];
        const bool st = (j != i) && (a != 0.0) && (m > 0.0) &&
                        (((kind == LAIR_SOC_NEG) ? -a : fabs(a)) >= thr);
        smask[p] = st ? 1 : 0;
        if (!frow) continue;
        if (j == i) { diag = a; continue; }
        if (a < 0.0) sn += a; else sp += a;
        if (st && cf[j] == 1) {
            if (a < 0.0) pn += a; else pp += a;
            ++k;
        }
    }
    if (!frow) {
        if (lane == 0) cnt[i] = 1;
        return;
    }
    diag = team_sum<T>(diag);
    sn = team_sum<T>(sn);
    sp = team_sum<T>(sp);
    pn = team_sum<T>(pn);
    pp = team_sum<T>(pp);
    k = team_sum_int<T>(k);
    double d = diag;
    if (pn == 0.0) d += sn;
    if (pp == 0.0) d += sp;
    const bool empty = (k == 0 || d == 0.0);
    if (lane == 0) {
        cnt[i] = empty ? 0 : k;
        coef[3 * (int64_t)i] = (pn != 0.0) ? sn / pn : 0.0;
        coef[3 * (int64_t)i + 1] = (pp != 0.0) ? sp / pp : 0.0;
        coef[3 * (int64_t)i + 2] = empty ? 0.0 : d;
    }
}

void launch_strength_interp(int32_t n, const int32_t *rp, const int32_t *cj,
                            const double *v, double theta, int32_t kind, const int8_t *cf,
                            uint8_t *smask, int32_t *cnt, double *coef, double mean_len,
                            hipStream_t s) {
    if (n == 0) return;
    // the team of launch_interp_direct
    int t = team_for_mean(mean_len);
    if (t > 16) t = 16;
    const double nnz = mean_len * n;
    ProfScope ps("strength", s, 13.0 * nnz + 4.0 * (n + 1) + 1.0 * n + 16.0 * n);
#define LAIR_SI(TT)                                                                      \
    LAIR_LAUNCH(k_strength_interp<TT>, dim3(blocks_for((int64_t)n * TT, 256)), dim3(256), \
                0, s, n, rp, cj, v, theta, kind, cf, smask, cnt, coef)
    switch (t) {
        case 2: LAIR_SI(2); break;
        case 4: LAIR_SI(4); break;
        case 8: LAIR_SI(8); break;
        default: LAIR_SI(16); break;
    }
#undef LAIR_SI
    LAIR_LAUNCH_CHECK();
}

// ===========================================================================
// Lumping of a coarse operator (Sec. 3.3 and the caption of its filtering
// table): in row i, an off-diagonal entry with |k_ij| < theta_D max_j |k_ij|
// (the maximum over the whole row, diagonal included) leaves the pattern and
// is added to k_ii (the removed entries summed in column order, then added), so the
// row sum stays.  A row without a diagonal or without off-diagonal entries
// is kept whole, and so is row i when whole_rows[i] != 0 (whole_rows may be
// null).  cnt != nullptr: count the kept entries of every row; otherwise
// write them at rp_out.  A team of T lanes per row.
// ===========================================================================
constexpr int LUMP_E = 4;     // entries per lane held in registers

template <int T>
__global__ void __launch_bounds__(256)
k_lump(int32_t n, const int32_t *rp, const int64_t *row_off, const int32_t *row_len,
       const int32_t *cj, const double *v, double theta, const int8_t *whole_rows,
       int32_t *cnt, const int32_t *rp_out, int32_t *cj_out, double *v_out) {
    const int64_t gt = xcd_block_id() * blockDim.x + threadIdx.x;
    const int32_t i = (int32_t)(gt / T);
    const int lane = (int)(gt % T);
    if (i >= n) return;
    // a CSR row, or a staged row (offset and length)
    const int64_t lo = row_off ? row_off[i] : (int64_t)rp[i];
    const int64_t hi = row_off ? lo + row_len[i] : (int64_t)rp[i + 1];
    if (hi - lo <= (int64_t)LUMP_E * T) {
        // the row in registers: step e of the team holds entries
        // lo + e T .. lo + e T + T - 1, so steps in order are column order
        int32_t c[LUMP_E];
        double a[LUMP_E];
        double mx = 0.0;
        int has_d = 0, has_o = 0;
#pragma unroll
        for (int e = 0; e < LUMP_E; ++e) {
            const int64_t p = lo + e * T + lane;
            c[e] = -1;
            a[e] = 0.0;
            if (p < hi) {
                c[e] = cj[p];
                a[e] = v[p];
                if (c[e] == i) has_d = 1;
                else has_o = 1;
                mx = fmax(mx, fabs(a[e]));
            }
        }
        mx = team_max<T>(mx);
        has_d = team_sum_int<T>(has_d);
        has_o = team_sum_int<T>(has_o);
        const bool whole = !has_d || !has_o || (whole_rows && whole_rows[i]);
        const double cut = theta * mx;
        bool keep[LUMP_E];
#pragma unroll
        for (int e = 0; e < LUMP_E; ++e)
            keep[e] = c[e] >= 0 && (whole || c[e] == i || !(fabs(a[e]) < cut));
        if (cnt) {
            int k = 0;
#pragma unroll
            for (int e = 0; e < LUMP_E; ++e) k += keep[e] ? 1 : 0;
            k = team_sum_int<T>(k);
            if (lane == 0) cnt[i] = k;
            return;
        }
        double gone = 0.0;
        if (!whole) {
#pragma unroll
            for (int e = 0; e < LUMP_E; ++e) {
                const bool rm = c[e] >= 0 && !keep[e];
                const double x = rm ? a[e] : 0.0;
                if (team_bits<T>(rm) == 0) continue;
                for (int k = 0; k < T; ++k) gone += __shfl(x, k, T);
            }
        }
        int o = rp_out[i];
#pragma unroll
        for (int e = 0; e < LUMP_E; ++e) {
            const uint64_t bits = team_bits<T>(keep[e]);
            const int before = __popcll(bits & ((1ull << lane) - 1ull));
            if (keep[e]) {
                cj_out[o + before] = c[e];
                v_out[o + before] = (c[e] == i && !whole) ? a[e] + gone : a[e];
            }
            o += __popcll(bits);
        }
        return;
    }
    // longer rows: streamed, the same operations in the same order
    double mx = 0.0;
    int has_d = 0, has_o = 0;
    for (int64_t p = lo + lane; p < hi; p += T) {
        if (cj[p] == i) has_d = 1;
        else has_o = 1;
        mx = fmax(mx, fabs(v[p]));
    }
    mx = team_max<T>(mx);
    has_d = team_sum_int<T>(has_d);
    has_o = team_sum_int<T>(has_o);
    const bool whole = !has_d || !has_o || (whole_rows && whole_rows[i]);
    const double cut = theta * mx;
    auto kept = [&](int64_t p) { return whole || cj[p] == i || !(fabs(v[p]) < cut); };
    if (cnt) {
        int k = 0;
        for (int64_t p = lo + lane; p < hi; p += T) k += kept(p) ? 1 : 0;
        k = team_sum_int<T>(k);
        if (lane == 0) cnt[i] = k;
        return;
    }
    // the removed entries' sum in column order: each step of T entries is
    // loaded by the team, then added entry by entry (kept ones add +0)
    double gone = 0.0;
    if (!whole) {
        for (int64_t p0 = lo; p0 < hi; p0 += T) {
            const int64_t p = p0 + lane;
            const bool rm = p < hi && !kept(p);
            const double x = rm ? v[p] : 0.0;
            if (team_bits<T>(rm) == 0) continue;
#pragma unroll 8
            for (int k = 0; k < T; ++k) gone += __shfl(x, k, T);
        }
    }
    int o = rp_out[i];
    for (int64_t p0 = lo; p0 < hi; p0 += T) {
        const int64_t p = p0 + lane;
        const bool take = p < hi && kept(p);
        const uint64_t bits = team_bits<T>(take);
        const int before = __popcll(bits & ((1ull << lane) - 1ull));
        if (take) {
            const int32_t j = cj[p];
            cj_out[o + before] = j;
            v_out[o + before] = (j == i && !whole) ? v[p] + gone : v[p];
        }
        o += __popcll(bits);
    }
}

void launch_lump(int32_t n, const int32_t *rp, const int64_t *row_off, const int32_t *row_len,
                 const int32_t *cj, const double *v, double theta, const int8_t *whole_rows,
                 double mean_len, int32_t *cnt, const int32_t *rp_out, int32_t *cj_out,
                 double *v_out, hipStream_t s) {
    if (n == 0) return;
    // about four entries per lane: several rows share a wavefront
    int t = team_for_mean(mean_len / 4.0);
    if (t > 16) t = 16;
#define LAIR_LU(TT)                                                                        \
    LAIR_LAUNCH(k_lump<TT>, dim3(blocks_for((int64_t)n * TT, 256)), dim3(256), 0, s, n, rp, \
                row_off, row_len, cj, v, theta, whole_rows, cnt, rp_out, cj_out, v_out)
    switch (t) {
        case 1: LAIR_LU(1); break;
        case 2: LAIR_LU(2); break;
        case 4: LAIR_LU(4); break;
        case 8: LAIR_LU(8); break;
        case 16: LAIR_LU(16); break;
        case 32: LAIR_LU(32); break;
        default: LAIR_LU(64); break;
    }
#undef LAIR_LU
    LAIR_LAUNCH_CHECK();
}

// ===========================================================================
// Sparse product C = A B with the symbolic pattern, rows of C sorted.
//
// Row i of C has at most E_i = sum over the entries a_ik of |row k of B|
// products.  One pass writes row i (sorted, distinct columns) into a staging
// buffer at the row's product offset, a scan of the row lengths gives C's
// row pointers, and a copy compacts the rows.
//
// Main kernel (hash accumulation): one team of T lanes per row, inside one
// wave, with a private open-addressing table in LDS.  The products are
// enumerated flat (the team scans the lengths of the selected rows of B;
// each lane takes every T-th product); each product's column is found or
// inserted in the table and a_ik b_kj added to its slot.  The adds of a
// round are one LDS instruction of the team's wave, rounds follow in
// program order, and no other wave touches the table, so every sum is
// formed in the same order on every run.  The rank of each distinct column
// among the row's columns is its output position.  Rows with more distinct
// columns than the table holds go to a list redone by a one-team block with
// a larger table, and beyond that by the row-merge kernel.
//
// Fallback (row-merge): one team per row; the row's entries select rows of
// B (sorted lists) merged in increasing column order, list k held by lane
// k % T, slot k / T.
// ===========================================================================
constexpr int GEMM_PF = 4;   // entries of each merge list held in registers

// Rows processed by a team: all rows (rows == nullptr), or the *nlist rows
// of a list, grid-stride.
struct RowSrc {
    const int32_t *rows;
    const int32_t *nlist;
};

__global__ void __launch_bounds__(256)
k_prod_count(int32_t m, const int32_t *ap, const int32_t *aj, BRows bp, int32_t *e) {
    const int64_t gt = xcd_block_id() * blockDim.x + threadIdx.x;
    const int32_t i = (int32_t)(gt / 8);
    const int lane = (int)(gt % 8);
    if (i >= m) return;
    int64_t t = 0;
    for (int p = ap[i] + lane; p < ap[i + 1]; p += 8) {
        int k = aj[p];
        t += bp.length(k);
    }
#pragma unroll
    for (int o = 4; o > 0; o >>= 1) t += __shfl_xor(t, o, 8);
    if (lane == 0) e[i] = (int32_t)min<int64_t>(t, INT32_MAX);
}

template <int T, int LPL>
__global__ void __launch_bounds__(256)
k_spgemm_merge(RowSrc src, const int32_t *ap, const int32_t *aj, const double *ax,
               BRows bp, const int32_t *bj, const double *bx, const int64_t *off,
               int32_t *cnt, int32_t *cj, double *cx, int32_t *overflow) {
    const int64_t gt = xcd_block_id() * blockDim.x + threadIdx.x;
    const int lane = (int)(gt % T);
    const int64_t nteams = (int64_t)gridDim.x * (blockDim.x / T);
    const int64_t nr = (int64_t)*src.nlist;
    for (int64_t t = gt / T; t < nr; t += nteams) {
        const int32_t i = src.rows[t];
        int lo = ap[i], ka = ap[i + 1] - lo;
        if (ka > T * LPL) {
            if (lane == 0) { atomicOr(overflow, 1); cnt[i] = 0; }
            continue;
        }
        // Each slot holds the next GEMM_PF entries of its list (columns and
        // scaled values) as a shift register, reloaded when empty.
        int pos[LPL], end[LPL];
        int hb[LPL][GEMM_PF];
        double vb[LPL][GEMM_PF];
        double mul[LPL];
#pragma unroll
        for (int s = 0; s < LPL; ++s) {
            int k = lane + s * T;
            pos[s] = 0;
            end[s] = 0;
            mul[s] = 0.0;
            if (k < ka) {
                int r = aj[lo + k];
                pos[s] = bp.start(r);
                end[s] = pos[s] + bp.length(r);
                mul[s] = ax[lo + k];
            }
#pragma unroll
            for (int d = 0; d < GEMM_PF; ++d) {
                int idx = pos[s] + d;
                bool ok = idx < end[s];
                hb[s][d] = ok ? bj[idx] : INT_MAX;
                vb[s][d] = ok ? mul[s] * bx[idx] : 0.0;
            }
            pos[s] += GEMM_PF;
        }
        int64_t o = off[i];
        int nout = 0;
        for (;;) {
            int h = INT_MAX;
#pragma unroll
            for (int s = 0; s < LPL; ++s) h = min(h, hb[s][0]);
            int mn = team_min<T>(h);
            if (mn == INT_MAX) break;
            double acc = 0.0;
#pragma unroll
            for (int s = 0; s < LPL; ++s) {
                if (hb[s][0] == mn) {
                    acc += vb[s][0];
#pragma unroll
                    for (int d = 0; d + 1 < GEMM_PF; ++d) {
                        hb[s][d] = hb[s][d + 1];
                        vb[s][d] = vb[s][d + 1];
                    }
                    hb[s][GEMM_PF - 1] = INT_MAX;
                    if (hb[s][0] == INT_MAX && pos[s] < end[s]) {
#pragma unroll
                        for (int d = 0; d < GEMM_PF; ++d) {
                            int idx = pos[s] + d;
                            bool ok = idx < end[s];
                            hb[s][d] = ok ? bj[idx] : INT_MAX;
                            vb[s][d] = ok ? mul[s] * bx[idx] : 0.0;
                        }
                        pos[s] += GEMM_PF;
                    }
                }
            }
            acc = team_sum<T>(acc);
            if (lane == 0) { cj[o + nout] = mn; cx[o + nout] = acc; }
            ++nout;
        }
        if (lane == 0) cnt[i] = nout;
    }
}

__device__ __forceinline__ int gemm_hash(int32_t col, int bits) {
    return (int)(((uint32_t)col * 0x9E3779B1u) >> (32 - bits));
}

template <int HS>
constexpr int log2_const() { return HS <= 1 ? 0 : 1 + log2_const<HS / 2>(); }

// Eight waves per SIMD asked for: the ranking below holds up to four columns
// per lane, whose scalar registers would otherwise lower the occupancy of the
// tables that fit eight (a few scalars then live in vector lanes).
template <int T, int HS, int BLOCK>
__global__ void __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(8)))
k_spgemm_hacc(int32_t m, RowSrc src, const int32_t *ap, const int32_t *aj, const double *ax,
              BRows bp, const int32_t *bj, const double *bx, const int64_t *eoff,
              int32_t *cnt, int32_t *tcj, double *tcx, int32_t *next, int32_t *nnext) {
    constexpr int TEAMS = BLOCK / T;
    constexpr int HC = HS / 2;              // distinct columns a table holds
    constexpr int BITS = log2_const<HS>();
    __shared__ int32_t s_key[TEAMS * HS];
    __shared__ double s_val[TEAMS * HS];
    __shared__ __align__(16) int32_t s_col[TEAMS * HC];   // distinct columns, insertion order
    __shared__ int16_t s_slot[TEAMS * HC];  // and their slots
    __shared__ int32_t s_n[TEAMS];
    const int team = threadIdx.x / T;
    const int lane = threadIdx.x % T;
    int32_t *key = s_key + team * HS;
    double *val = s_val + team * HS;
    int32_t *lcol = s_col + team * HC;
    int16_t *lslot = s_slot + team * HC;
    const int64_t gteam = (xcd_block_id() * BLOCK + threadIdx.x) / T;
    const int64_t nteams = (int64_t)gridDim.x * TEAMS;
    const int64_t nr = src.rows ? (int64_t)*src.nlist : (int64_t)m;
    for (int64_t t = gteam; t < nr; t += nteams) {
        const int32_t i = src.rows ? src.rows[t] : (int32_t)t;
        const int lo = ap[i], ka = ap[i + 1] - lo;
        for (int q = lane; q < HS; q += T) { key[q] = -1; val[q] = 0.0; }
        if (lane == 0) s_n[team] = 0;
        wave_lds_sync();
        bool full = false;
        for (int c0 = 0; c0 < ka && !full; c0 += T) {
            const int p = c0 + lane;
            int b0 = 0, len = 0;
            double a = 0.0;
            if (p < ka) {
                int k = aj[lo + p];
                b0 = bp.start(k);
                len = bp.length(k);
                a = ax[lo + p];
            }
            int inc = len;
#pragma unroll
            for (int o = 1; o < T; o <<= 1) {
                int u = __shfl_up(inc, o, T);
                if (lane >= o) inc += u;
            }
            const int tot = __shfl(inc, T - 1, T);
            const int exc = inc - len;
            for (int e0 = 0; e0 < tot; e0 += T) {
                const int e = e0 + lane;
                // owner of product e: the last lane whose offset is <= e
                int q = 0;
#pragma unroll
                for (int st = T / 2; st > 0; st >>= 1) {
                    int ex = __shfl(exc, q + st, T);
                    if (ex <= e) q += st;
                }
                const int bq = __shfl(b0, q, T);
                const int xq = __shfl(exc, q, T);
                const double aq = __shfl(a, q, T);
                int h = -1;
                double v = 0.0;
                bool ovf = false;
                if (e < tot) {
                    const int idx = bq + e - xq;
                    const int32_t col = bj[idx];
                    v = aq * bx[idx];
                    h = gemm_hash(col, BITS);
                    for (int probe = 0;; ++probe) {
                        int old = atomicCAS(&key[h], -1, col);
                        if (old == -1) {
                            int ps = atomicAdd(&s_n[team], 1);
                            if (ps < HC) { lcol[ps] = col; lslot[ps] = (int16_t)h; }
                            else ovf = true;
                            break;
                        }
                        if (old == col) break;
                        if (probe == HS - 1) { h = -1; break; }
                        h = (h + 1) & (HS - 1);
                    }
                }
                // one add per product, issued together by the team; the
                // wave's LDS atomics complete in issue order, so the sums do
                // not depend on timing, and no wait is needed between steps
                if (h >= 0) atomicAdd(&val[h], v);
                // past HC distinct columns the row goes to a larger table
                if (team_bits<T>(ovf)) { full = true; break; }
            }
        }
        wave_lds_sync();
        const int n = s_n[team];
        if (n > HC) {
            // more distinct columns than this table holds: a larger one redoes it
            if (lane == 0) next[atomicAdd(nnext, 1)] = i;
            wave_lds_sync();
            continue;
        }
        const int64_t o = eoff[i];
        // rank of each distinct column among them (reads four at a time;
        // lcol is 16-byte aligned, entries past n are masked).  A lane holds
        // at most HC / T columns; up to four of them are ranked in one pass
        // over the list, each read compared with all of them.
        constexpr int KR = HC / T;
        if constexpr (KR <= 4) {
            int cc[KR], rk[KR];
#pragma unroll
            for (int k = 0; k < KR; ++k) {
                const int u = lane + k * T;
                cc[k] = u < n ? lcol[u] : INT_MAX;
                rk[k] = 0;
            }
            for (int w = 0; w < n; w += 4) {
                int4 q = *reinterpret_cast<const int4 *>(lcol + w);
                // entries past n rank below nothing
                q.y = w + 1 < n ? q.y : INT_MAX;
                q.z = w + 2 < n ? q.z : INT_MAX;
                q.w = w + 3 < n ? q.w : INT_MAX;
#pragma unroll
                for (int k = 0; k < KR; ++k)
                    rk[k] += (q.x < cc[k]) + (q.y < cc[k]) + (q.z < cc[k]) + (q.w < cc[k]);
            }
#pragma unroll
            for (int k = 0; k < KR; ++k) {
                const int u = lane + k * T;
                if (u < n) {
                    tcj[o + rk[k]] = cc[k];
                    tcx[o + rk[k]] = val[lslot[u]];
                }
            }
        } else {
            for (int u = lane; u < n; u += T) {
                const int32_t c = lcol[u];
                auto rank4 = [&](int w) {
                    const int4 q = *reinterpret_cast<const int4 *>(lcol + w);
                    return (q.x < c) + (w + 1 < n && q.y < c) + (w + 2 < n && q.z < c) +
                           (w + 3 < n && q.w < c);
                };
                int r = 0;
                if constexpr (HC >= 64) {
                    // long lists: more reads in flight (small tables keep the
                    // registers for occupancy)
#pragma unroll 4
                    for (int w = 0; w < n; w += 4) r += rank4(w);
                } else {
                    for (int w = 0; w < n; w += 4) r += rank4(w);
                }
                tcj[o + r] = c;
                tcx[o + r] = val[lslot[u]];
            }
        }
        if (lane == 0) cnt[i] = n;
        wave_lds_sync();
    }
}

template <int T, int HS, int BLOCK>
static void spgemm_hacc(int32_t m, RowSrc src, unsigned grid, const int32_t *ap,
                        const int32_t *aj, const double *ax, BRows bp,
                        const int32_t *bj, const double *bx, const int64_t *eoff, int32_t *cnt,
                        int32_t *tcj, double *tcx, int32_t *next, int32_t *nnext,
                        hipStream_t s) {
    LAIR_LAUNCH((k_spgemm_hacc<T, HS, BLOCK>), dim3(grid), dim3(BLOCK), 0, s, m, src,
                       ap, aj, ax, bp, bj, bx, eoff, cnt, tcj, tcx, next, nnext);
    LAIR_LAUNCH_CHECK();
}

// Team size from the mean number of products per row: about three or four
// steps of T products per row (more rows per wave) measured faster than one
// or two on the Galerkin products of the 3-D and batched 2-D problems.
static int hacc_team(double mean_e) {
    if (mean_e <= 32.0) return 8;
    if (mean_e <= 96.0) return 16;
    if (mean_e <= 256.0) return 32;
    return 64;
}

constexpr int HACC_BIG = 4096;   // table of the one-team kernel

void launch_prod_count(int32_t m, const int32_t *ap, const int32_t *aj, BRows bp,
                       int32_t *e, hipStream_t s) {
    if (m == 0) return;
    LAIR_LAUNCH(k_prod_count, dim3(blocks_for((int64_t)m * 8, 256)), dim3(256), 0, s, m,
                       ap, aj, bp, e);
    LAIR_LAUNCH_CHECK();
}

void launch_spgemm(int32_t m, const int32_t *ap, const int32_t *aj, const double *ax,
                   BRows bp, const int32_t *bj, const double *bx,
                   const int64_t *eoff, int64_t max_e, double mean_e, double mean_c_hint,
                   int32_t *cnt, int32_t *tcj, double *tcx, int32_t *counts, int32_t *lists,
                   int32_t *overflow, hipStream_t s) {
    if (m == 0) return;
    // counts[0..2] (the lengths of the retry lists) arrive zeroed; lists
    // holds three lists of m rows
    int32_t *n1 = counts, *n2 = counts + 1, *n3 = counts + 2;
    int32_t *l1 = lists, *l2 = lists + m, *l3 = lists + 2 * (int64_t)m;
    const int T = hacc_team(mean_e);
    const RowSrc all{nullptr, nullptr};
    const unsigned g = blocks_for((int64_t)m * T, 256);
    // table: twice the mean products (a row has at most that many distinct
    // columns in the common case), at most 2048 slots per block; smaller
    // tables leave LDS for more resident waves
    const int cap = 2048 / (256 / T);
    int HS = 16;
    while (HS < cap && HS < 2.0 * mean_e) HS <<= 1;
    if (HS < cap / 4) HS = cap / 4;
    // with an estimate of the distinct columns per row, a large product's
    // first pass takes a table three times that size (more waves per CU);
    // rows that do not fit are redone by the table above, then by the large
    // one.  Small products keep one pass (a retry costs a launch).
    int HS1 = HS;
    if (mean_c_hint > 0.0 && m >= 65536) {
        HS1 = 16;
        while (HS1 < HS && HS1 < 3.0 * mean_c_hint) HS1 <<= 1;
        if (HS1 < cap / 4) HS1 = cap / 4;
    }
#define LAIR_HA(TT, HH, SRC, GRID, NL, NN)                                                 \
    if (T == TT && hs == HH)                                                               \
        spgemm_hacc<TT, HH, 256>(m, SRC, GRID, ap, aj, ax, bp, bj, bx, eoff, cnt, tcj, tcx, \
                                 NL, NN, s);
#define LAIR_HA_ALL(SRC, GRID, NL, NN)                                                     \
    LAIR_HA(8, 16, SRC, GRID, NL, NN) LAIR_HA(8, 32, SRC, GRID, NL, NN)                    \
    LAIR_HA(8, 64, SRC, GRID, NL, NN) LAIR_HA(16, 32, SRC, GRID, NL, NN)                   \
    LAIR_HA(16, 64, SRC, GRID, NL, NN) LAIR_HA(16, 128, SRC, GRID, NL, NN)                 \
    LAIR_HA(32, 64, SRC, GRID, NL, NN) LAIR_HA(32, 128, SRC, GRID, NL, NN)                 \
    LAIR_HA(32, 256, SRC, GRID, NL, NN) LAIR_HA(64, 128, SRC, GRID, NL, NN)                \
    LAIR_HA(64, 256, SRC, GRID, NL, NN) LAIR_HA(64, 512, SRC, GRID, NL, NN)
    {
        const int hs = HS1;
        LAIR_HA_ALL(all, g, l1, n1)
    }
    if (max_e <= HS1 / 2) return;     // no row can have more distinct columns
    int32_t *lbig = l1, *nbig = n1;
    if (HS1 < HS) {
        const int hs = HS;
        const RowSrc retry{l1, n1};
        const unsigned g2 = g < 4096u ? g : 4096u;
        LAIR_HA_ALL(retry, g2, l2, n2)
        if (max_e <= HS / 2) return;
        lbig = l2;
        nbig = n2;
    }
#undef LAIR_HA_ALL
#undef LAIR_HA
    // wider rows: one 64-lane team per block with a large table, then the merge
    spgemm_hacc<64, HACC_BIG, 64>(m, RowSrc{lbig, nbig}, 2048, ap, aj, ax, bp, bj, bx, eoff,
                                  cnt, tcj, tcx, l3, n3, s);
    if (max_e <= HACC_BIG / 2) return;
    LAIR_LAUNCH((k_spgemm_merge<64, 16>), dim3(256), dim3(256), 0, s, RowSrc{l3, n3},
                       ap, aj, ax, bp, bj, bx, eoff, cnt, tcj, tcx, overflow);
    LAIR_LAUNCH_CHECK();
}

// Copy the staged rows (at their product offsets) to C's rows, a team of T
// lanes per row.
template <int T>
__global__ void __launch_bounds__(256)
k_spgemm_compact(int32_t m, const int64_t *eoff, const int32_t *crp, const int32_t *tcj,
                 const double *tcx, int32_t *cj, double *cx) {
    const int64_t gt = xcd_block_id() * blockDim.x + threadIdx.x;
    const int32_t i = (int32_t)(gt / T);
    const int lane = (int)(gt % T);
    if (i >= m) return;
    const int64_t src = eoff[i];
    const int32_t dst = crp[i], len = crp[i + 1] - dst;
    for (int q = lane; q < len; q += T) {
        cj[dst + q] = tcj[src + q];
        cx[dst + q] = tcx[src + q];
    }
}

void launch_spgemm_compact(int32_t m, const int64_t *eoff, const int32_t *crp,
                           const int32_t *tcj, const double *tcx, int32_t *cj, double *cx,
                           double mean_c, hipStream_t s) {
    if (m == 0) return;
    const int t = team_for_mean(mean_c / 2.0);
#define LAIR_CP(TT)                                                                      \
    LAIR_LAUNCH(k_spgemm_compact<TT>, dim3(blocks_for((int64_t)m * TT, 256)),     \
                       dim3(256), 0, s, m, eoff, crp, tcj, tcx, cj, cx)
    switch (t) {
        case 2: LAIR_CP(2); break;
        case 4: LAIR_CP(4); break;
        case 8: LAIR_CP(8); break;
        case 16: LAIR_CP(16); break;
        case 32: LAIR_CP(32); break;
        default: LAIR_CP(64); break;
    }
#undef LAIR_CP
    LAIR_LAUNCH_CHECK();
}

// ===========================================================================
// Transpose (deterministic): count per column, scan, scatter with atomic
// cursors, then sort each output row by column (the source row index).
// ===========================================================================
__global__ void k_tcount(int32_t nrows, const int32_t *rp, const int32_t *cj,
                         int32_t *tcount) {
    int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nrows) return;
    for (int p = rp[i]; p < rp[i + 1]; ++p) atomicAdd(&tcount[cj[p]], 1);
}

__global__ void k_tscatter(int32_t nrows, const int32_t *rp, const int32_t *cj,
                           const double *v, const int32_t *trp,
                           int32_t *cursor, int32_t *tcj, double *tv) {
    int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nrows) return;
    for (int p = rp[i]; p < rp[i + 1]; ++p) {
        int c = cj[p];
        int o = trp[c] + atomicAdd(&cursor[c], 1);
        tcj[o] = i;
        tv[o] = v[p];
    }
}

__global__ void k_tsort(int32_t ncols, const int32_t *trp, int32_t *tcj,
                        double *tv) {
    int32_t r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= ncols) return;
    int lo = trp[r], hi = trp[r + 1];
    for (int a = lo + 1; a < hi; ++a) {
        int kc = tcj[a];
        double kv = tv[a];
        int b = a - 1;
        while (b >= lo && tcj[b] > kc) {
            tcj[b + 1] = tcj[b];
            tv[b + 1] = tv[b];
            --b;
        }
        tcj[b + 1] = kc;
        tv[b + 1] = kv;
    }
}

void launch_transpose(int32_t nrows, int32_t ncols, int64_t nnz,
                      const int32_t *rp, const int32_t *cj, const double *v,
                      int32_t *tcount, int32_t *trp, int32_t *tcj, double *tv,
                      int32_t *cursor, hipStream_t s, DevArr<int64_t> &tmp) {
    (void)nnz;
    LAIR_HIP(hipMemsetAsync(tcount, 0, sizeof(int32_t) * (size_t)ncols, s));
    LAIR_HIP(hipMemsetAsync(cursor, 0, sizeof(int32_t) * (size_t)ncols, s));
    LAIR_LAUNCH(k_tcount, dim3(blocks_for(nrows, 256)), dim3(256), 0, s,
                       nrows, rp, cj, tcount);
    LAIR_LAUNCH_CHECK();
    scan_counts_i32(tcount, trp, ncols, s, tmp);
    LAIR_LAUNCH(k_tscatter, dim3(blocks_for(nrows, 256)), dim3(256), 0, s,
                       nrows, rp, cj, v, trp, cursor, tcj, tv);
    LAIR_LAUNCH_CHECK();
    LAIR_LAUNCH(k_tsort, dim3(blocks_for(ncols, 256)), dim3(256), 0, s,
                       ncols, trp, tcj, tv);
    LAIR_LAUNCH_CHECK();
}

__global__ void k_to_float(const double *in, float *out, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = (float)in[i];
}

void launch_to_float(const double *in, float *out, int64_t n, hipStream_t s) {
    if (n == 0) return;
    LAIR_LAUNCH(k_to_float, dim3(blocks_for(n, 256)), dim3(256), 0, s,
                       in, out, n);
    LAIR_LAUNCH_CHECK();
}

// ===========================================================================
// Block-diagonal inverse (Sec. 4.2.1): the k x k diagonal blocks by
// Gauss-Jordan with partial pivoting.  bad = 1 for a singular block.
// ===========================================================================
constexpr int BLK_MAX = 8;

// A team of BLK_MAX lanes per block, lane r holding row r of [D_e | I] in
// registers (every index below is a compile-time one, so nothing spills):
// lane r finds the block's entries in its row by a binary search for
// column e k; the Gauss-Jordan steps are those of a serial elimination
// (pivot: the largest magnitude in the column, the first row on a tie; the
// pivot row scaled by 1 / pivot, then every other row with a nonzero
// multiplier updated), one row per lane.
__global__ void __launch_bounds__(256)
k_block_inverse(int32_t nblk, int32_t k, const int32_t *rp, const int32_t *cj,
                const double *v, double *dinv, int32_t *bad) {
    constexpr int B = BLK_MAX;
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int32_t e = (int32_t)(g / B);
    const int r = (int)(g % B);
    if (e >= nblk) return;
    const int32_t b0 = e * k;
    double a[2 * B];
#pragma unroll
    for (int q = 0; q < 2 * B; ++q) a[q] = (r < k && q == k + r) ? 1.0 : 0.0;
    if (r < k) {
        const int32_t row = b0 + r;
        int32_t lo = rp[row], hi = rp[row + 1];
        while (lo < hi) {                       // first column >= b0
            const int32_t mid = (lo + hi) >> 1;
            if (cj[mid] < b0) lo = mid + 1; else hi = mid;
        }
        for (int32_t p = lo; p < rp[row + 1] && cj[p] < b0 + k; ++p) {
            const int c = cj[p] - b0;
            const double val = v[p];
#pragma unroll
            for (int q = 0; q < B; ++q)
                if (q == c) a[q] = val;
        }
    }
    bool singular = false;
#pragma unroll
    for (int col = 0; col < B; ++col) {
        if (col >= k) break;
        double cand = (r >= col && r < k) ? fabs(a[col]) : -1.0;
        int pr = r;
        team_argmax<B>(cand, pr);
        if (cand == 0.0) { singular = true; break; }
        const int src = (r == col) ? pr : (r == pr ? col : r);
#pragma unroll
        for (int q = 0; q < 2 * B; ++q) a[q] = __shfl(a[q], src, B);
        const double inv = 1.0 / __shfl(a[col], col, B);
        if (r == col) {
#pragma unroll
            for (int q = 0; q < 2 * B; ++q)
                if (q < 2 * k) a[q] *= inv;
        }
        const double f = a[col];
#pragma unroll
        for (int q = 0; q < 2 * B; ++q) {
            const double pq = __shfl(a[q], col, B);
            if (r != col && r < k && f != 0.0 && q < 2 * k) a[q] -= f * pq;
        }
    }
    if (singular) {
        if (r == 0) atomicOr(bad, 1);
        return;
    }
    if (r < k) {
        double *out = dinv + (size_t)e * k * k + (size_t)r * k;
#pragma unroll
        for (int q = 0; q < 2 * B; ++q)
            if (q >= k && q < 2 * k) out[q - k] = a[q];
    }
}

void launch_block_inverse(int32_t nblk, int32_t k, const int32_t *rp,
                          const int32_t *cj, const double *v, double *dinv,
                          int32_t *bad, hipStream_t s) {
    if (k > BLK_MAX) fail(LAIR_EUNSUPPORTED, "block size %d > %d", k, BLK_MAX);
    if (nblk == 0) return;
    LAIR_LAUNCH(k_block_inverse, dim3(blocks_for((int64_t)nblk * BLK_MAX, 256)), dim3(256), 0, s,
                nblk, k, rp, cj, v, dinv, bad);
    LAIR_LAUNCH_CHECK();
}

// ===========================================================================
// Coarsest grid: dense copy and LU with partial pivoting (one block).
// ===========================================================================
__global__ void k_dense_from_csr(int32_t n, const int32_t *rp, const int32_t *cj,
                                 const double *v, double *dense) {
    int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double *row = dense + (size_t)i * n;
    for (int q = 0; q < n; ++q) row[q] = 0.0;
    for (int p = rp[i]; p < rp[i + 1]; ++p) row[cj[p]] = v[p];
}

void launch_dense_from_csr(int32_t n, const int32_t *rp, const int32_t *cj,
                           const double *v, double *dense, hipStream_t s) {
    LAIR_LAUNCH(k_dense_from_csr, dim3(blocks_for(n, 64)), dim3(64), 0, s,
                       n, rp, cj, v, dense);
    LAIR_LAUNCH_CHECK();
}

__global__ void __launch_bounds__(1024)
k_dense_lu(int32_t n, double *a, int32_t *piv, int32_t *info) {
    __shared__ double sv[1024];
    __shared__ int si[1024];
    int t = threadIdx.x;
    int nt = blockDim.x;
    for (int k = 0; k < n; ++k) {
        double best = -1.0;
        int bi = INT_MAX;
        for (int r = k + t; r < n; r += nt) {
            double x = fabs(a[(size_t)r * n + k]);
            if (x > best || (x == best && r < bi)) { best = x; bi = r; }
        }
        sv[t] = best;
        si[t] = bi;
        __syncthreads();
        for (int o = nt / 2; o > 0; o >>= 1) {
            if (t < o) {
                double ov = sv[t + o];
                int oi = si[t + o];
                if (ov > sv[t] || (ov == sv[t] && oi < si[t])) { sv[t] = ov; si[t] = oi; }
            }
            __syncthreads();
        }
        int pr = si[0];
        double pv = sv[0];
        __syncthreads();
        if (pv == 0.0) {
            if (t == 0) *info = k + 1;
            return;
        }
        if (t == 0) piv[k] = pr;
        if (pr != k)
            for (int q = t; q < n; q += nt) {
                double x = a[(size_t)k * n + q];
                a[(size_t)k * n + q] = a[(size_t)pr * n + q];
                a[(size_t)pr * n + q] = x;
            }
        __syncthreads();
        double inv = 1.0 / a[(size_t)k * n + k];
        for (int r = k + 1 + t; r < n; r += nt) a[(size_t)r * n + k] *= inv;
        __syncthreads();
        int w = n - k - 1;
        for (int64_t idx = t; idx < (int64_t)w * w; idx += nt) {
            int r = k + 1 + (int)(idx / w);
            int q = k + 1 + (int)(idx % w);
            a[(size_t)r * n + q] -= a[(size_t)r * n + k] * a[(size_t)k * n + q];
        }
        __syncthreads();
    }
    if (t == 0) *info = 0;
}

// Small coarsest grids (n <= 128): the whole factorisation in LDS, pivot
// search by the first wave with shuffles (largest |a|, smallest row on ties).
__global__ void __launch_bounds__(256)
k_dense_lu_lds(int32_t n, double *lu, int32_t *piv, int32_t *info) {
    extern __shared__ double a[];
    __shared__ int s_piv;
    __shared__ double s_val;
    int t = threadIdx.x, nt = blockDim.x;
    for (int idx = t; idx < n * n; idx += nt) a[idx] = lu[idx];
    __syncthreads();
    for (int k = 0; k < n; ++k) {
        if (t < 64) {
            double best = -1.0;
            int bi = INT_MAX;
            for (int r = k + t; r < n; r += 64) {
                double x = fabs(a[r * n + k]);
                if (x > best) { best = x; bi = r; }
            }
            team_argmax<64>(best, bi);
            if (t == 0) { s_piv = bi; s_val = best; }
        }
        __syncthreads();
        int pr = s_piv;
        if (s_val == 0.0) {
            if (t == 0) *info = k + 1;
            return;
        }
        if (t == 0) piv[k] = pr;
        if (pr != k)
            for (int q = t; q < n; q += nt) {
                double x = a[k * n + q];
                a[k * n + q] = a[pr * n + q];
                a[pr * n + q] = x;
            }
        __syncthreads();
        double inv = 1.0 / a[k * n + k];
        for (int r = k + 1 + t; r < n; r += nt) a[r * n + k] *= inv;
        __syncthreads();
        int w = n - k - 1;
        for (int idx = t; idx < w * w; idx += nt) {
            int r = k + 1 + idx / w;
            int q = k + 1 + idx % w;
            a[r * n + q] -= a[r * n + k] * a[k * n + q];
        }
        __syncthreads();
    }
    for (int idx = t; idx < n * n; idx += nt) lu[idx] = a[idx];
    if (t == 0) *info = 0;
}

// Small coarsest grids (n <= 128): the explicit inverse in one workgroup by
// Gauss-Jordan elimination in place with partial pivoting (largest |a_rk|
// among the rows not yet used, smallest row on ties, rows exchanged), n
// steps of one rank-1 update each; the row exchanges are undone at the end
// as column exchanges (inv(A) = inv(PA) P).  info = k + 1 for a zero pivot
// at step k.
constexpr int LUI_ROWS = 128;
constexpr int LUI_BS = 1024;
constexpr int LUI_WAVES = LUI_BS / 64;
constexpr int LUI_RPW = LUI_ROWS / LUI_WAVES;    // row positions per wave

// Gauss-Jordan inverse with partial pivoting in place, in one workgroup.
// Row positions are dealt to the waves cyclically; lane q of a wave holds
// columns q and q + 64 of the rows it updates.  Each step: every wave finds
// the pivot itself (same reads, same answer: no exchange) and reads the
// pivot row and its own rows; after one barrier it writes its rows, and a
// second barrier ends the step.  The row exchanges are undone as a column
// permutation on the way out.
__global__ void __launch_bounds__(LUI_BS)
k_dense_gj_inv(int32_t n, const double *dense, double *inv, int32_t *info) {
    extern __shared__ double a[];
    __shared__ int s_piv[LUI_ROWS];
    __shared__ int s_perm[LUI_ROWS];
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    for (int idx = tid; idx < n * n; idx += LUI_BS) a[idx] = dense[idx];
    __syncthreads();
    const int q0 = lane, q1 = lane + 64;
    const bool h0 = q0 < n, h1 = q1 < n;
    for (int k = 0; k < n; ++k) {
        double bv = -1.0;
        int bi = INT_MAX;
        if (h0 && q0 >= k) { bv = fabs(a[q0 * n + k]); bi = q0; }
        if (h1 && q1 >= k) {
            const double v1 = fabs(a[q1 * n + k]);
            if (v1 > bv) { bv = v1; bi = q1; }
        }
        team_argmax<64>(bv, bi);
        if (bv == 0.0) {            // the same in every wave: all leave together
            if (tid == 0) *info = k + 1;
            return;
        }
        const int pr = bi;
        const double d = 1.0 / a[pr * n + k];
        // scaled pivot row (its column k becomes the inverse's entry d)
        const double p0 = h0 ? (q0 == k ? 1.0 : a[pr * n + q0]) * d : 0.0;
        const double p1 = h1 ? (q1 == k ? 1.0 : a[pr * n + q1]) * d : 0.0;
        // this wave's rows; position pr receives old row k
        double f[LUI_RPW], s0[LUI_RPW], s1[LUI_RPW];
#pragma unroll
        for (int t = 0; t < LUI_RPW; ++t) {
            const int r = wave + t * LUI_WAVES;
            const int src = (r == pr) ? k : r;
            f[t] = 0.0;
            s0[t] = 0.0;
            s1[t] = 0.0;
            if (r < n && r != k) {
                f[t] = a[src * n + k];
                if (h0) s0[t] = a[src * n + q0];
                if (h1) s1[t] = a[src * n + q1];
            }
        }
        if (tid == 0) s_piv[k] = pr;
        __syncthreads();
#pragma unroll
        for (int t = 0; t < LUI_RPW; ++t) {
            const int r = wave + t * LUI_WAVES;
            if (r >= n) break;
            if (r == k) {
                if (h0) a[k * n + q0] = p0;
                if (h1) a[k * n + q1] = p1;
            } else {
                if (h0) a[r * n + q0] = (q0 == k) ? -f[t] * d : s0[t] - f[t] * p0;
                if (h1) a[r * n + q1] = (q1 == k) ? -f[t] * d : s1[t] - f[t] * p1;
            }
        }
        __syncthreads();
    }
    // the row exchanges, undone last first as column exchanges, compose to
    // one column permutation: inv[r][c] = a[r][perm[c]]
    if (tid == 0) {
        for (int c = 0; c < n; ++c) s_perm[c] = c;
        for (int j = n - 1; j >= 0; --j) {
            const int jp = s_piv[j];
            const int t = s_perm[j];
            s_perm[j] = s_perm[jp];
            s_perm[jp] = t;
        }
    }
    __syncthreads();
    for (int r = wave; r < n; r += LUI_WAVES) {
        if (h0) inv[r * n + q0] = a[r * n + s_perm[q0]];
        if (h1) inv[r * n + q1] = a[r * n + s_perm[q1]];
    }
    if (tid == 0) *info = 0;
}

// n <= 128 and the matrix fits LDS: the inverse in one kernel
bool launch_dense_gj_inv(int32_t n, const double *dense, double *inv, int32_t *info,
                         hipStream_t s);

static size_t max_lds_per_block() {
    static size_t cached = 0;
    if (!cached) {
        int dev = 0, v = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess &&
            v > 0)
            cached = (size_t)v;
        else
            cached = 65536;
    }
    return cached;
}

bool launch_dense_gj_inv(int32_t n, const double *dense, double *inv, int32_t *info,
                         hipStream_t s) {
    if (n < 1 || n > LUI_ROWS || (size_t)n * n * sizeof(double) + 4096 > max_lds_per_block())
        return false;
    LAIR_LAUNCH(k_dense_gj_inv, dim3(1), dim3(LUI_BS), (size_t)n * n * sizeof(double), s, n,
                dense, inv, info);
    LAIR_LAUNCH_CHECK();
    return true;
}

void launch_dense_lu(int32_t n, double *lu, int32_t *piv, int32_t *info,
                     hipStream_t s) {
    if (n <= 128 && (size_t)n * n * sizeof(double) + 64 <= max_lds_per_block()) {
        LAIR_LAUNCH(k_dense_lu_lds, dim3(1), dim3(256), (size_t)n * n * sizeof(double),
                           s, n, lu, piv, info);
        LAIR_LAUNCH_CHECK();
        return;
    }
    int bs = 64;
    while (bs < 1024 && bs < n) bs <<= 1;
    LAIR_LAUNCH(k_dense_lu, dim3(1), dim3(bs), 0, s, n, lu, piv, info);
    LAIR_LAUNCH_CHECK();
}

// Explicit inverse from P K = L U: block b solves for identity columns
// 8b .. 8b+7 (one wave per block, the columns kept in LDS).
constexpr int INV_COLS = 8;

__global__ void __launch_bounds__(64)
k_dense_inverse(int32_t n, const double *lu, const int32_t *piv, double *inv) {
    extern __shared__ double xs[];
    const int c0 = blockIdx.x * INV_COLS;
    const int t = threadIdx.x;
    for (int idx = t; idx < n * INV_COLS; idx += 64) {
        int r = idx / INV_COLS, q = idx % INV_COLS;
        xs[idx] = (r == c0 + q) ? 1.0 : 0.0;
    }
    __syncthreads();
    if (t < INV_COLS)
        for (int k = 0; k < n; ++k) {
            int p = piv[k];
            if (p != k) {
                double x = xs[k * INV_COLS + t];
                xs[k * INV_COLS + t] = xs[p * INV_COLS + t];
                xs[p * INV_COLS + t] = x;
            }
        }
    __syncthreads();
    for (int k = 0; k < n; ++k) {
        int w = (n - k - 1) * INV_COLS;
        for (int idx = t; idx < w; idx += 64) {
            int r = k + 1 + idx / INV_COLS, q = idx % INV_COLS;
            xs[r * INV_COLS + q] -= lu[(size_t)r * n + k] * xs[k * INV_COLS + q];
        }
        __syncthreads();
    }
    for (int k = n - 1; k >= 0; --k) {
        if (t < INV_COLS) xs[k * INV_COLS + t] /= lu[(size_t)k * n + k];
        __syncthreads();
        int w = k * INV_COLS;
        for (int idx = t; idx < w; idx += 64) {
            int r = idx / INV_COLS, q = idx % INV_COLS;
            xs[r * INV_COLS + q] -= lu[(size_t)r * n + k] * xs[k * INV_COLS + q];
        }
        __syncthreads();
    }
    for (int idx = t; idx < n * INV_COLS; idx += 64) {
        int r = idx / INV_COLS, q = idx % INV_COLS;
        if (c0 + q < n) inv[(size_t)r * n + c0 + q] = xs[idx];
    }
}

void launch_dense_inverse(int32_t n, const double *lu, const int32_t *piv,
                          double *inv, hipStream_t s) {
    int nb = (n + INV_COLS - 1) / INV_COLS;
    LAIR_LAUNCH(k_dense_inverse, dim3(nb), dim3(64),
                       (size_t)n * INV_COLS * sizeof(double), s, n, lu, piv, inv);
    LAIR_LAUNCH_CHECK();
}

// ===========================================================================
// Split ordering of a level for the cycle: F-points first (ascending), then
// C-points (ascending, i.e. in coarse-index order).  A permuted copy keeps
// every row's entries in their stored order with renumbered columns, so a
// row's sum in the cycle runs in the same order as on the natural matrix.
// ===========================================================================
__global__ void k_split_perm(int32_t nf, int32_t nc, const int32_t *flist,
                             const int32_t *clist, int32_t *perm, int32_t *iperm,
                             int32_t *ids, int8_t *cf_split) {
    const int32_t n = nf + nc;
    const int32_t k = (int32_t)((int64_t)blockIdx.x * blockDim.x + threadIdx.x);
    if (k >= n) return;
    const int32_t old = k < nf ? flist[k] : clist[k - nf];
    perm[k] = old;
    iperm[old] = k;
    ids[k] = k;
    cf_split[k] = k < nf ? 0 : 1;
}

void launch_split_perm(int32_t nf, int32_t nc, const int32_t *flist, const int32_t *clist,
                       int32_t *perm, int32_t *iperm, int32_t *ids, int8_t *cf_split,
                       hipStream_t s) {
    if (nf + nc == 0) return;
    LAIR_LAUNCH(k_split_perm, dim3(blocks_for(nf + nc, 256)), dim3(256), 0, s, nf, nc, flist,
                clist, perm, iperm, ids, cf_split);
    LAIR_LAUNCH_CHECK();
}

// New row k is old row rowmap[k]; columns become colmap[c] (nullptr maps
// are identities).  Values go to v_out and/or v32_out; cjt_out receives
// the new columns tagged (sign bit) where they are >= nsplit.
template <int T>
__global__ void __launch_bounds__(256)
k_permute_csr(int32_t nrows, const int32_t *irowmap, const int32_t *colmap, const int32_t *rp,
              const int32_t *cj, const double *v, const int32_t *rp_out, int32_t *cj_out,
              double *v_out, float *v32_out, int32_t *cjt_out, int32_t nsplit) {
    // teams walk the input rows in order (reads stream; output row
    // k = irowmap[r] is written at its place)
    const int64_t gt = xcd_block_id() * blockDim.x + threadIdx.x;
    const int32_t r = (int32_t)(gt / T);
    const int t = (int)(gt % T);
    if (r >= nrows) return;
    const int32_t k = irowmap ? irowmap[r] : r;
    const int32_t lo = rp[r], hi = rp[r + 1];
    const int64_t o = (int64_t)rp_out[k] - lo;
    // four entries per lane in flight: loads first, then the column map,
    // then the stores
    constexpr int U = 4;
    for (int32_t base = lo + t; base < hi; base += U * T) {
        int32_t c[U];
        double a[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int32_t e = base + u * T;
            c[u] = e < hi ? cj[e] : 0;
            a[u] = e < hi ? v[e] : 0.0;
        }
        if (colmap) {
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (base + u * T < hi) c[u] = colmap[c[u]];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int32_t e = base + u * T;
            if (e < hi) {
                cj_out[o + e] = c[u];
                if (v_out) v_out[o + e] = a[u];
                if (v32_out) v32_out[o + e] = (float)a[u];
                if (cjt_out)
                    cjt_out[o + e] = c[u] >= nsplit ? (int32_t)((uint32_t)c[u] | 0x80000000u)
                                                    : c[u];
            }
        }
    }
}

void launch_permute_csr(int32_t nrows, int64_t nnz, double mean_row, const int32_t *rowmap,
                        const int32_t *irowmap, const int32_t *colmap, const int32_t *rp,
                        const int32_t *cj, const double *v, int32_t *rp_out, int32_t *cj_out,
                        double *v_out, float *v32_out, int32_t *cjt_out, int32_t nsplit,
                        DevArr<int64_t> &tmp, hipStream_t s) {
    if ((rowmap == nullptr) != (irowmap == nullptr))
        fail(LAIR_EINVAL, "a row permutation needs its inverse");
    (void)nnz;
    scan_launch(RowLenF{rp, rowmap}, rp_out, nrows, s, tmp);
    if (nrows == 0) return;
    // about four entries per lane
    const int T = mean_row > 96 ? 32 : mean_row > 48 ? 16 : mean_row > 24 ? 8
                : mean_row > 12 ? 4 : mean_row > 6 ? 2 : 1;
#define LAIR_PC(TT)                                                                      \
    LAIR_LAUNCH((k_permute_csr<TT>), dim3(blocks_for((int64_t)nrows * TT, 256)), dim3(256), \
                0, s, nrows, irowmap, colmap, rp, cj, v, rp_out, cj_out, v_out, v32_out, \
                cjt_out, nsplit)
    switch (T) {
        case 1: LAIR_PC(1); break;
        case 2: LAIR_PC(2); break;
        case 4: LAIR_PC(4); break;
        case 8: LAIR_PC(8); break;
        case 16: LAIR_PC(16); break;
        default: LAIR_PC(32); break;
    }
#undef LAIR_PC
    LAIR_LAUNCH_CHECK();
}

}  // namespace lair
