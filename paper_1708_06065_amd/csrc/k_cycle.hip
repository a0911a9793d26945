// V-cycle kernels on gfx950: residual, sparse matrix-vector products for
// restriction and interpolation, masked Jacobi sweeps (every row of a sweep
// reads the previous iterate), norms and the coarsest-grid triangular
// solves.  All are memory bound: CSR rows are streamed with a team of T
// lanes per row for one right-hand side, or one lane per (row, right-hand
// side) when several interleaved right-hand sides share each matrix row.
#include <cmath>

#include "k_common.hpp"
#include "lair_internal.hpp"

namespace lair {

// ---------------------------------------------------------------------------
// Row products.  Source vectors may be split by point type: with SEL the
// value of neighbour c is read from xC when cf[c] = 1 (C-point) and from xF
// otherwise, which lets two Jacobi sweeps read and write without a copy.
// ---------------------------------------------------------------------------
enum { MODE_RESID = 0, MODE_SET = 1, MODE_ADD = 2 };

template <class VT, bool SEL>
__device__ __forceinline__ VT src_val(const VT *xF, const VT *xC, const int8_t *cf,
                                      int64_t idx, int c) {
    if (SEL) return cf[c] ? xC[idx] : xF[idx];
    return xF[idx];
}

// One right-hand side, a team of T lanes per row (lanes take every T-th
// entry of the row).  A lane loads four of its entries, then their four
// gathers, before it sums them in entry order, so the loads of a row are in
// flight together (the sums are those of the plain loop).
template <class VT, int T, bool SEL>
__device__ __forceinline__ void row_acc1(int lo, int hi, int lane, int diag_col,
                                         const int32_t *cj, const VT *v,
                                         const VT *xF, const VT *xC,
                                         const int8_t *cf, VT &acc, VT &d) {
    constexpr int U = 4;
    for (int p0 = lo + lane; p0 < hi; p0 += U * T) {
        int c[U];
        VT a[U], xv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int p = p0 + u * T;
            c[u] = p < hi ? cj[p] : -1;
            a[u] = p < hi ? v[p] : (VT)0;
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
            xv[u] = c[u] >= 0 ? src_val<VT, SEL>(xF, xC, cf, c[u], c[u]) : (VT)0;
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (c[u] >= 0) {
                acc += a[u] * xv[u];
                if (c[u] == diag_col) d = a[u];
            }
        }
    }
}

// NR interleaved right-hand sides, one lane per right-hand side.  The team
// loads NR consecutive entries of the row (one per lane) and broadcasts them
// by shuffles in chunks of CH, so the gathers of a chunk are independent
// loads issued together.  Padding entries use column 0 with value 0.
template <class VT, int NR, bool SEL>
__device__ __forceinline__ void row_accM(int lo, int hi, int q, int diag_col,
                                         const int32_t *cj, const VT *v,
                                         const VT *xF, const VT *xC,
                                         const int8_t *cf, VT &acc, VT &d) {
    constexpr int CH = NR < 8 ? NR : 8;
    for (int base = lo; base < hi; base += NR) {
        int p = base + q;
        int c = -1;
        VT a = (VT)0;
        if (p < hi) { c = cj[p]; a = v[p]; }
        int cnt = hi - base;
#pragma unroll
        for (int ch = 0; ch < NR; ch += CH) {
            if (ch < cnt) {
                int ce[CH];
                VT ae[CH], xe[CH];
#pragma unroll
                for (int e = 0; e < CH; ++e) {
                    ce[e] = __shfl(c, ch + e, NR);
                    ae[e] = __shfl(a, ch + e, NR);
                }
#pragma unroll
                for (int e = 0; e < CH; ++e) {
                    int cc = ce[e] < 0 ? 0 : ce[e];
                    xe[e] = src_val<VT, SEL>(xF, xC, cf, (int64_t)cc * NR + q, cc);
                }
#pragma unroll
                for (int e = 0; e < CH; ++e) {
                    acc += ae[e] * xe[e];
                    if (ce[e] == diag_col) d = ae[e];
                }
            }
        }
    }
}

// NR interleaved right-hand sides held VW to a lane as one 16-byte vector
// (4 floats or 2 doubles): L = NR / VW lanes per row, so a wave covers 64 / L
// rows.  The L lanes load L consecutive entries of the row, broadcast them by
// shuffles, and each lane gathers its VW values of every neighbour with one
// vector load.  Pointers must be 16-byte aligned (checked by the launchers).
template <class VT, int VW> struct VecT;
template <> struct VecT<double, 1> { using T = double; };
template <> struct VecT<float, 1> { using T = float; };
template <> struct VecT<float, 4> { using T = float4; };
template <> struct VecT<float, 2> { using T = float2; };
template <> struct VecT<double, 2> { using T = double2; };

template <class VT, int VW>
struct Pack {
    VT v[VW];
    __device__ __forceinline__ void zero() {
#pragma unroll
        for (int k = 0; k < VW; ++k) v[k] = (VT)0;
    }
    __device__ __forceinline__ void load(const VT *p) {
        typename VecT<VT, VW>::T t = *reinterpret_cast<const typename VecT<VT, VW>::T *>(p);
        const VT *q = reinterpret_cast<const VT *>(&t);
#pragma unroll
        for (int k = 0; k < VW; ++k) v[k] = q[k];
    }
    __device__ __forceinline__ void store(VT *p) const {
        typename VecT<VT, VW>::T t;
        VT *q = reinterpret_cast<VT *>(&t);
#pragma unroll
        for (int k = 0; k < VW; ++k) q[k] = v[k];
        *reinterpret_cast<typename VecT<VT, VW>::T *>(p) = t;
    }
    // streaming load (data read once, far larger than the caches)
    __device__ __forceinline__ void load_nt(const VT *p) {
        if constexpr (VW == 1) {
            v[0] = ld_stream(p);
        } else {
            const ExtVec<VT, VW> t = ld_stream(reinterpret_cast<const ExtVec<VT, VW> *>(p));
#pragma unroll
            for (int k = 0; k < VW; ++k) v[k] = t[k];
        }
    }
};

// Row k of a row list: rows[k], or row0 + k for a contiguous range
// (rows == nullptr).
__device__ __forceinline__ int32_t list_row(const int32_t *rows, int32_t row0, int64_t k) {
    return rows ? rows[k] : row0 + (int32_t)k;
}

// A team of T = G L lanes per row (G a power of two chosen from the row
// length): the team loads T consecutive entries, group g of L lanes takes
// entries g L .. g L + L - 1 of them, and the G partial sums are added by
// shuffles at the end.
// TAG: the column indices carry the point type in their sign bit (C-point
// columns are stored as c | 2^31), which spares SEL the load of cf[c].
// U: steps of T entries taken together (their loads all in flight before
// the first product); a lane still adds its entries in increasing order, so
// the sums do not depend on U.
// NTA: the row's entries are streamed (read once).
// RNG: columns >= csplit are read from xC, the others from xF (a vector
// whose rows from csplit on were left in another buffer).
template <class VT, int NR, int VW, bool SEL, bool TAG = false, int U = 1, bool NTA = false,
          bool RNG = false>
__device__ __forceinline__ void row_accV(int lo, int hi, int t, int T, int diag_col,
                                         const int32_t *cj, const VT *v,
                                         const VT *xF, const VT *xC,
                                         const int8_t *cf, Pack<VT, VW> &acc, VT &d,
                                         int csplit = 0) {
    constexpr int L = NR / VW;
    const int q = t % L;
    const int g0 = (t / L) * L;      // first entry of this lane's group
    for (int base = lo; base < hi; base += U * T) {
        int c[U];
        VT a[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int p = base + u * T + t;
            c[u] = 0;
            a[u] = (VT)0;
            if (p < hi) {
                c[u] = NTA ? ld_stream(cj + p) : cj[p];
                a[u] = NTA ? ld_stream(v + p) : v[p];
            }
        }
        int ce[U][L];
        VT ae[U][L];
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int e = 0; e < L; ++e) {
                ce[u][e] = __shfl(c[u], e, L);
                ae[u][e] = __shfl(a[u], e, L);
            }
        Pack<VT, VW> xe[U][L];
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int e = 0; e < L; ++e) {
                if (base + u * T + g0 + e < hi) {
                    const int col = TAG ? (ce[u][e] & 0x7fffffff) : ce[u][e];
                    const VT *src = TAG ? (ce[u][e] < 0 ? xC : xF)
                                  : SEL ? (cf[col] ? xC : xF)
                                  : RNG ? (col >= csplit ? xC : xF)
                                        : xF;
                    xe[u][e].load(src + (int64_t)col * NR + q * VW);
                    if (col == diag_col) d = ae[u][e];
                } else {
                    xe[u][e].zero();
                }
            }
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int e = 0; e < L; ++e) {
#pragma unroll
                for (int k = 0; k < VW; ++k) acc.v[k] += ae[u][e] * xe[u][e].v[k];
            }
    }
    for (int o = L; o < T; o <<= 1) {
#pragma unroll
        for (int k = 0; k < VW; ++k) acc.v[k] += __shfl_xor(acc.v[k], o);
        d += __shfl_xor(d, o);
    }
}

// SRC: 0 one source; 1 columns >= csplit read from xhi; 2 columns with
// cf[c] = 1 read from xhi.
template <class VT, int NR, int VW, int MODE, int U, int SRC>
__global__ void __launch_bounds__(256)
k_rowdotV(int32_t nrows, int T, const int32_t *rp, const int32_t *cj, const VT *v,
          const VT *x, const VT *xhi, int32_t csplit, const int8_t *cf, const VT *b, VT *y) {
    constexpr int L = NR / VW;
    int64_t gt = xcd_block_id() * blockDim.x + threadIdx.x;
    int32_t i = (int32_t)(gt / T);
    int t = (int)(gt % T);
    if (i >= nrows) return;
    Pack<VT, VW> acc;
    acc.zero();
    VT d = (VT)0;
    row_accV<VT, NR, VW, SRC == 2, false, U, false, SRC == 1>(rp[i], rp[i + 1], t, T, -1, cj, v,
                                                             x, SRC ? xhi : x, cf, acc, d,
                                                             csplit);
    if (t >= L) return;
    const int64_t o = (int64_t)i * NR + t * VW;
    Pack<VT, VW> out;
    if (MODE == MODE_RESID) {
        out.load(b + o);
#pragma unroll
        for (int k = 0; k < VW; ++k) out.v[k] -= acc.v[k];
    } else if (MODE == MODE_ADD) {
        out.load(y + o);
#pragma unroll
        for (int k = 0; k < VW; ++k) out.v[k] += acc.v[k];
    } else {
        out = acc;
    }
    out.store(y + o);
}

template <class VT, int NR, int VW, bool SEL, bool TAG, int U>
__global__ void __launch_bounds__(256)
k_jacobiV(int32_t nx, int T, const int32_t *rows, int32_t row0, const int32_t *rp,
          const int32_t *cj, const VT *v, const VT *b, const VT *xF, const VT *xC,
          const int8_t *cf, VT *out, int compact, VT omega) {
    constexpr int L = NR / VW;
    int64_t gt = xcd_block_id() * blockDim.x + threadIdx.x;
    int32_t k = (int32_t)(gt / T);
    int t = (int)(gt % T);
    if (k >= nx) return;
    const int32_t i = list_row(rows, row0, k);
    // the row's own old value and right-hand side load beside the row
    const int64_t oi = (int64_t)i * NR + (t % L) * VW;
    Pack<VT, VW> xi, bi, r;
    if (t < L) {
        xi.load((SEL ? (cf[i] ? xC : xF) : xF) + oi);
        bi.load(b + oi);
    }
    Pack<VT, VW> acc;
    acc.zero();
    VT d = (VT)0;
    row_accV<VT, NR, VW, SEL, TAG, U>(rp[i], rp[i + 1], t, T, i, cj, v, xF, xC, cf, acc, d);
    if (t >= L) return;
#pragma unroll
    for (int e = 0; e < VW; ++e) r.v[e] = xi.v[e] + omega * (bi.v[e] - acc.v[e]) / d;
    r.store(out + (compact ? (int64_t)k * NR + t * VW : oi));
}

// Lanes per row for the vector kernels: L = nrhs / VW, times G groups so
// that a team covers about half of a mean row per step (team: the matrix's
// single-vector team, a power of two >= its mean row length).
static inline int vec_team(int L, int team) {
    int g = 1;
    while (g * L * 2 < team && g * L < 64) g <<= 1;
    return g * L;
}

// Jacobi sweeps: half as many lanes per row as the products above (a
// quarter on long rows, mean 32 or more), at least one row vector, so that
// each lane keeps more steps of gathers in flight and more rows share a
// wavefront (measured on 16 right-hand sides: the sweeps of the coarse
// levels ran about 6 % faster in total than with twice the lanes).
static inline int vec_team_jacobi(int L, int team) {
    const int T = vec_team(L, team);
    return std::max(L, team >= 32 ? T / 4 : T / 2);
}

// Steps of T entries per loop turn: two when a mean row (team) needs more
// than one step and the doubled gathers still fit the registers.
template <class VT>
static inline int vec_unroll(int nrhs, int T, int team) {
    return team > T && nrhs <= (sizeof(VT) == 4 ? 16 : 8) ? 2 : 1;
}

// Outer residual of the double iteration fused with its norms and the
// float copy for the cycle: r = b - A x for every row (teams as above,
// grid-stride over a fixed grid), written as r64 and/or r32, and each
// block's sum of r^2 per right-hand side into partial[block][nrhs]
// (fixed order: thread sums, then a fixed walk over the block's threads).
template <int NR, int VW, bool OUT64, bool OUT32, int U>
__global__ void __launch_bounds__(256)
k_resid_norm(int32_t nrows, int T, const int32_t *rp, const int32_t *cj, const double *v,
             const double *x, const double *b, double *r64, float *r32, double *partial,
             const int32_t *orow) {
    constexpr int L = NR / VW;
    __shared__ double sh[256 * VW];
    const int t = (int)(threadIdx.x % T);
    // the blocks of one XCD (consecutive ids under xcd_block_id) take one
    // contiguous share of the rows, their teams striding through it: a
    // row's neighbours a few strides away then stay in that XCD's L2
    // instead of being fetched again by another XCD
    const int64_t nb = gridDim.x, xb = blockIdx.x % NXCD;
    const int64_t q = nb / NXCD, rr = nb % NXCD;
    const int64_t nbx = q + (xb < rr ? 1 : 0);
    const int64_t b0 = xb < rr ? xb * (q + 1) : rr * (q + 1) + (xb - rr) * q;
    const int64_t tpb = blockDim.x / T;
    const int64_t tl = (xcd_block_id() - b0) * tpb + threadIdx.x / T;
    const int64_t lo = b0 * (int64_t)nrows / nb, hi = (b0 + nbx) * (int64_t)nrows / nb;
    double sq[VW];
#pragma unroll
    for (int k = 0; k < VW; ++k) sq[k] = 0.0;
    for (int64_t i = lo + tl; i < hi; i += nbx * tpb) {
        Pack<double, VW> acc;
        acc.zero();
        double d = 0.0;
        // the matrix and b are streamed (read once), x is gathered
        row_accV<double, NR, VW, false, false, U, true>(ld_stream(rp + i), ld_stream(rp + i + 1),
                                                        t, T, -1, cj, v, x, x, nullptr, acc, d);
        if (t < L) {
            const int64_t o = i * NR + t * VW;
            // the residual goes to row orow[i] (another ordering) if given
            const int64_t oo = orow ? (int64_t)orow[i] * NR + t * VW : o;
            Pack<double, VW> r;
            r.load_nt(b + o);
#pragma unroll
            for (int k = 0; k < VW; ++k) {
                r.v[k] -= acc.v[k];
                sq[k] += r.v[k] * r.v[k];
            }
            if (OUT64) r.store(r64 + oo);
            if (OUT32) {
                Pack<float, VW> rf;
#pragma unroll
                for (int k = 0; k < VW; ++k) rf.v[k] = (float)r.v[k];
                rf.store(r32 + oo);
            }
        }
    }
#pragma unroll
    for (int k = 0; k < VW; ++k) sh[threadIdx.x * VW + k] = sq[k];
    __syncthreads();
    if ((int)threadIdx.x < NR) {
        const int lane = threadIdx.x / VW, k = threadIdx.x % VW;
        double a = 0.0;
        for (int th = lane; th < (int)blockDim.x; th += T) a += sh[th * VW + k];
        partial[(int64_t)blockIdx.x * NR + threadIdx.x] = a;
    }
}

// Lanes per row for one right-hand side: about four entries per lane (a
// power of two >= the mean row length gives `team`).
static inline int scalar_team(int team) { return team >= 4 ? team / 4 : 1; }

static inline bool aligned16(const void *p) { return ((uintptr_t)p & 15u) == 0; }

// SEL: the source is split by point type (x at F columns, xC where
// cf[c] = 1).
template <class VT, int T, int MODE, bool SEL>
__global__ void __launch_bounds__(256)
k_rowdot1(int32_t nrows, const int32_t *rp, const int32_t *cj, const VT *v,
          const VT *x, const VT *xC, const int8_t *cf, const VT *b, VT *y) {
    int64_t gt = xcd_block_id() * blockDim.x + threadIdx.x;
    int32_t i = (int32_t)(gt / T);
    int lane = (int)(gt % T);
    if (i >= nrows) return;
    VT acc = (VT)0, d = (VT)0;
    row_acc1<VT, T, SEL>(rp[i], rp[i + 1], lane, -1, cj, v, x, SEL ? xC : x, cf, acc, d);
    acc = team_sum<T>(acc);
    if (lane == 0) {
        if (MODE == MODE_RESID) y[i] = b[i] - acc;
        else if (MODE == MODE_SET) y[i] = acc;
        else y[i] += acc;
    }
}

// One right-hand side over a listed subset of rows: rows[k] for k < *cnt
// (the list and its length live on the device; the grid covers the list's
// capacity).
template <class VT, int T, int MODE>
__global__ void __launch_bounds__(256)
k_rowdot_list(const int32_t *rows, const int32_t *cnt, const int32_t *rp, const int32_t *cj,
              const VT *v, const VT *x, const VT *b, VT *y) {
    const int64_t gt = xcd_block_id() * blockDim.x + threadIdx.x;
    const int lane = (int)(gt % T);
    const int64_t nteams = (int64_t)gridDim.x * (blockDim.x / T);
    const int32_t n = *cnt;
    for (int64_t k = gt / T; k < n; k += nteams) {
        const int32_t i = rows[k];
        VT acc = (VT)0, d = (VT)0;
        row_acc1<VT, T, false>(rp[i], rp[i + 1], lane, -1, cj, v, x, x, nullptr, acc, d);
        acc = team_sum<T>(acc);
        if (lane == 0) {
            if (MODE == MODE_RESID) y[i] = b[i] - acc;
            else if (MODE == MODE_SET) y[i] = acc;
            else y[i] += acc;
        }
    }
}

// Grid for kernels that stride over a device-side count: the blocks that
// fill every CU once (more would mostly find nothing to do).
constexpr int64_t LIST_GRID = 2048;
static inline unsigned list_grid(int64_t threads) {
    const int64_t b = (threads + 255) / 256;
    return (unsigned)(b < 1 ? 1 : (b < LIST_GRID ? b : LIST_GRID));
}

template <class VT, int NR, int MODE>
__global__ void __launch_bounds__(256)
k_rowdotM(int32_t nrows, const int32_t *rp, const int32_t *cj, const VT *v,
          const VT *x, const VT *b, VT *y) {
    int64_t gt = xcd_block_id() * blockDim.x + threadIdx.x;
    int32_t i = (int32_t)(gt / NR);
    int q = (int)(gt % NR);
    if (i >= nrows) return;
    VT acc = (VT)0, d = (VT)0;
    row_accM<VT, NR, false>(rp[i], rp[i + 1], q, -1, cj, v, x, x, nullptr, acc, d);
    int64_t o = (int64_t)i * NR + q;
    if (MODE == MODE_RESID) y[o] = b[o] - acc;
    else if (MODE == MODE_SET) y[o] = acc;
    else y[o] += acc;
}

// x_hi (optional): a source vector left in two buffers.  With csplit >= 0
// its rows from csplit on are read from x_hi, else the rows with
// cf_hi[c] = 1 (the vector path takes either, the one-right-hand-side path
// the point types; see op_spmv_split_ok).
template <class VT, int MODE>
static void rowdot(const CsrView<VT> &A, const VT *x, const VT *b, VT *y,
                   int32_t nrhs, hipStream_t s, const VT *x_hi = nullptr, int32_t csplit = -1,
                   const int8_t *cf_hi = nullptr) {
    if (A.nrows == 0) return;
    if (x_hi && csplit < 0 && !cf_hi) fail(LAIR_EINVAL, "a split source needs its split");
    if (nrhs > 1 && aligned16(x) && aligned16(y) && (!b || aligned16(b)) &&
        (!x_hi || aligned16(x_hi))) {
        constexpr int VW = sizeof(VT) == 4 ? 4 : 2;
#define LAIR_RVU(NN, WW, UU)                                                      \
        if (x_hi && csplit >= 0)                                                  \
            LAIR_LAUNCH((k_rowdotV<VT, NN, WW, MODE, UU, 1>),                     \
                        dim3(blocks_for((int64_t)A.nrows * T, 256)), dim3(256), 0, s, \
                        A.nrows, T, A.rp, A.cj, A.v, x, x_hi, csplit, nullptr, b, y); \
        else if (x_hi)                                                            \
            LAIR_LAUNCH((k_rowdotV<VT, NN, WW, MODE, UU, 2>),                     \
                        dim3(blocks_for((int64_t)A.nrows * T, 256)), dim3(256), 0, s, \
                        A.nrows, T, A.rp, A.cj, A.v, x, x_hi, 0, cf_hi, b, y);    \
        else                                                                      \
            LAIR_LAUNCH((k_rowdotV<VT, NN, WW, MODE, UU, 0>),                     \
                        dim3(blocks_for((int64_t)A.nrows * T, 256)), dim3(256), 0, s, \
                        A.nrows, T, A.rp, A.cj, A.v, x, x, 0, nullptr, b, y);
#define LAIR_RV(NN, WW)                                                           \
    {                                                                             \
        const int T = vec_team(NN / WW, A.team);                                  \
        if (vec_unroll<VT>(NN, T, A.team) == 2) { LAIR_RVU(NN, WW, 2) }           \
        else { LAIR_RVU(NN, WW, 1) }                                              \
    }
        switch (nrhs) {
            case 2: LAIR_RV(2, 2); break;
            case 4: LAIR_RV(4, VW); break;
            case 8: LAIR_RV(8, VW); break;
            case 16: LAIR_RV(16, VW); break;
            default: LAIR_RV(32, VW); break;
        }
#undef LAIR_RV
#undef LAIR_RVU
        LAIR_LAUNCH_CHECK();
        return;
    }
    if (x_hi && (nrhs > 1 || !cf_hi))
        fail(LAIR_EINVAL, "a vector split over two buffers needs aligned multi-vectors or "
             "point types");
    if (nrhs > 1) {
#define LAIR_RM(NN)                                                               \
    LAIR_LAUNCH((k_rowdotM<VT, NN, MODE>),                                 \
                       dim3(blocks_for((int64_t)A.nrows * NN, 256)), dim3(256), 0, s, \
                       A.nrows, A.rp, A.cj, A.v, x, b, y)
        switch (nrhs) {
            case 2: LAIR_RM(2); break;
            case 4: LAIR_RM(4); break;
            case 8: LAIR_RM(8); break;
            case 16: LAIR_RM(16); break;
            default: LAIR_RM(32); break;
        }
#undef LAIR_RM
        LAIR_LAUNCH_CHECK();
        return;
    }
#define LAIR_RD(TT)                                                              \
    if (x_hi)                                                                    \
        LAIR_LAUNCH((k_rowdot1<VT, TT, MODE, true>),                             \
                    dim3(blocks_for((int64_t)A.nrows * TT, 256)), dim3(256), 0, s, \
                    A.nrows, A.rp, A.cj, A.v, x, x_hi, cf_hi, b, y);             \
    else                                                                         \
        LAIR_LAUNCH((k_rowdot1<VT, TT, MODE, false>),                            \
                    dim3(blocks_for((int64_t)A.nrows * TT, 256)), dim3(256), 0, s, \
                    A.nrows, A.rp, A.cj, A.v, x, x, nullptr, b, y)
    switch (scalar_team(A.team)) {
        case 1: LAIR_RD(1); break;
        case 2: LAIR_RD(2); break;
        case 4: LAIR_RD(4); break;
        case 8: LAIR_RD(8); break;
        case 16: LAIR_RD(16); break;
        case 32: LAIR_RD(32); break;
        default: LAIR_RD(64); break;
    }
#undef LAIR_RD
    LAIR_LAUNCH_CHECK();
}

template <class VT>
void op_residual(const CsrView<VT> &A, const VT *b, const VT *x, VT *r,
                 int32_t nrhs, hipStream_t s) {
    rowdot<VT, MODE_RESID>(A, x, b, r, nrhs, s);
}

template <class VT>
void op_spmv(const CsrView<VT> &A, const VT *x, VT *y, int32_t nrhs,
             bool accumulate, hipStream_t s, const VT *x_hi, int32_t csplit,
             const int8_t *cf_hi) {
    if (accumulate) rowdot<VT, MODE_ADD>(A, x, nullptr, y, nrhs, s, x_hi, csplit, cf_hi);
    else rowdot<VT, MODE_SET>(A, x, nullptr, y, nrhs, s, x_hi, csplit, cf_hi);
}

bool op_spmv_split_ok(int32_t nrhs, const void *x, const void *x_hi, const void *y) {
    return nrhs == 1 || (aligned16(x) && aligned16(x_hi) && aligned16(y));
}

template <class VT, int MODE>
static void rowdot_list_t(const CsrView<VT> &A, const int32_t *rows, const int32_t *cnt,
                          int32_t cap, const VT *x, const VT *b, VT *y, hipStream_t s) {
#define LAIR_RL(TT)                                                                    \
    LAIR_LAUNCH((k_rowdot_list<VT, TT, MODE>), dim3(list_grid((int64_t)cap * TT)),     \
                dim3(256), 0, s, rows, cnt, A.rp, A.cj, A.v, x, b, y)
    switch (scalar_team(A.team)) {
        case 1: LAIR_RL(1); break;
        case 2: LAIR_RL(2); break;
        case 4: LAIR_RL(4); break;
        case 8: LAIR_RL(8); break;
        case 16: LAIR_RL(16); break;
        case 32: LAIR_RL(32); break;
        default: LAIR_RL(64); break;
    }
#undef LAIR_RL
    LAIR_LAUNCH_CHECK();
}

template <class VT>
void op_rowdot_list(const CsrView<VT> &A, int mode, const int32_t *rows, const int32_t *cnt,
                    int32_t cap, const VT *x, const VT *b, VT *y, hipStream_t s) {
    if (cap == 0) return;
    if (mode == MODE_RESID) rowdot_list_t<VT, MODE_RESID>(A, rows, cnt, cap, x, b, y, s);
    else if (mode == MODE_SET) rowdot_list_t<VT, MODE_SET>(A, rows, cnt, cap, x, b, y, s);
    else rowdot_list_t<VT, MODE_ADD>(A, rows, cnt, cap, x, b, y, s);
}

// ---------------------------------------------------------------------------
// Jacobi on a row set X:  new_i = x_i + omega (b_i - (A x)_i) / a_ii for
// i = X[k], written to out[k] (compact) or out[i].  Every row reads the
// previous iterate; the diagonal is found while streaming the row.
// ---------------------------------------------------------------------------
template <class VT, int T, bool SEL>
__global__ void __launch_bounds__(256)
k_jacobi1(int32_t nx, const int32_t *cnt, const int32_t *rows, int32_t row0, const int32_t *rp,
          const int32_t *cj, const VT *v, const VT *b, const VT *xF, const VT *xC,
          const int8_t *cf, VT *out, int compact, VT omega) {
    const int64_t gt = xcd_block_id() * blockDim.x + threadIdx.x;
    const int lane = (int)(gt % T);
    const int64_t nteams = (int64_t)gridDim.x * (blockDim.x / T);
    const int32_t n = cnt ? *cnt : nx;
    for (int64_t k = gt / T; k < n; k += nteams) {
        const int32_t i = list_row(rows, row0, k);
        VT acc = (VT)0, d = (VT)0;
        row_acc1<VT, T, SEL>(rp[i], rp[i + 1], lane, i, cj, v, xF, xC, cf, acc, d);
        acc = team_sum<T>(acc);
        d = team_sum<T>(d);
        if (lane == 0) {
            VT xi = src_val<VT, SEL>(xF, xC, cf, i, i);
            out[compact ? k : i] = xi + omega * (b[i] - acc) / d;
        }
    }
}

template <class VT, int NR, bool SEL>
__global__ void __launch_bounds__(256)
k_jacobiM(int32_t nx, const int32_t *rows, int32_t row0, const int32_t *rp, const int32_t *cj,
          const VT *v, const VT *b, const VT *xF, const VT *xC, const int8_t *cf,
          VT *out, int compact, VT omega) {
    int64_t gt = xcd_block_id() * blockDim.x + threadIdx.x;
    int32_t k = (int32_t)(gt / NR);
    int q = (int)(gt % NR);
    if (k >= nx) return;
    const int32_t i = list_row(rows, row0, k);
    VT acc = (VT)0, d = (VT)0;
    row_accM<VT, NR, SEL>(rp[i], rp[i + 1], q, i, cj, v, xF, xC, cf, acc, d);
    int64_t oi = (int64_t)i * NR + q;
    VT xi = src_val<VT, SEL>(xF, xC, cf, oi, i);
    out[(compact ? (int64_t)k * NR : oi - q) + q] = xi + omega * (b[oi] - acc) / d;
}

template <class VT, bool SEL>
static void jacobi_launch(const CsrView<VT> &A, const int32_t *rows, int32_t row0, int32_t nx,
                          const int32_t *cnt, const VT *b, const VT *xF, const VT *xC,
                          const int8_t *cf, VT *out, int compact, VT om, int32_t nrhs,
                          hipStream_t s) {
    if (cnt && nrhs != 1) fail(LAIR_EINVAL, "listed Jacobi rows take one right-hand side");
    if (nrhs > 1 && aligned16(b) && aligned16(xF) && aligned16(xC) && aligned16(out)) {
        constexpr int VW = sizeof(VT) == 4 ? 4 : 2;
#define LAIR_JVU(NN, WW, UU)                                                      \
    {                                                                             \
        if (SEL && A.cjt)                                                         \
            LAIR_LAUNCH((k_jacobiV<VT, NN, WW, SEL, true, UU>),                   \
                        dim3(blocks_for((int64_t)nx * T, 256)), dim3(256), 0, s,  \
                        nx, T, rows, row0, A.rp, A.cjt, A.v, b, xF, xC, cf, out, compact, om); \
        else                                                                      \
            LAIR_LAUNCH((k_jacobiV<VT, NN, WW, SEL, false, UU>),                  \
                        dim3(blocks_for((int64_t)nx * T, 256)), dim3(256), 0, s,  \
                        nx, T, rows, row0, A.rp, A.cj, A.v, b, xF, xC, cf, out, compact, om); \
    }
#define LAIR_JV(NN, WW)                                                           \
    {                                                                             \
        const int T = vec_team_jacobi(NN / WW, A.team);                          \
        if (vec_unroll<VT>(NN, T, A.team) == 2) LAIR_JVU(NN, WW, 2)               \
        else LAIR_JVU(NN, WW, 1)                                                  \
    }
        switch (nrhs) {
            case 2: LAIR_JV(2, 2); break;
            case 4: LAIR_JV(4, VW); break;
            case 8: LAIR_JV(8, VW); break;
            case 16: LAIR_JV(16, VW); break;
            default: LAIR_JV(32, VW); break;
        }
#undef LAIR_JV
#undef LAIR_JVU
        LAIR_LAUNCH_CHECK();
        return;
    }
    if (nrhs > 1) {
#define LAIR_JM(NN)                                                               \
    LAIR_LAUNCH((k_jacobiM<VT, NN, SEL>),                                  \
                       dim3(blocks_for((int64_t)nx * NN, 256)), dim3(256), 0, s,  \
                       nx, rows, row0, A.rp, A.cj, A.v, b, xF, xC, cf, out, compact, om)
        switch (nrhs) {
            case 2: LAIR_JM(2); break;
            case 4: LAIR_JM(4); break;
            case 8: LAIR_JM(8); break;
            case 16: LAIR_JM(16); break;
            default: LAIR_JM(32); break;
        }
#undef LAIR_JM
        LAIR_LAUNCH_CHECK();
        return;
    }
#define LAIR_JC(TT)                                                              \
    LAIR_LAUNCH((k_jacobi1<VT, TT, SEL>),                                 \
                       dim3(cnt ? list_grid((int64_t)nx * TT) : blocks_for((int64_t)nx * TT, 256)), \
                       dim3(256), 0, s, nx, cnt, rows, row0, A.rp, A.cj, A.v, b, xF, xC, cf, out, compact, om)
    switch (scalar_team(A.team)) {
        case 1: LAIR_JC(1); break;
        case 2: LAIR_JC(2); break;
        case 4: LAIR_JC(4); break;
        case 8: LAIR_JC(8); break;
        case 16: LAIR_JC(16); break;
        case 32: LAIR_JC(32); break;
        default: LAIR_JC(64); break;
    }
#undef LAIR_JC
    LAIR_LAUNCH_CHECK();
}

template <class VT>
void op_jacobi(const CsrView<VT> &A, const int32_t *rows, int32_t nx,
               const VT *b, const VT *xF, const VT *xC, const int8_t *cf,
               VT *out, bool compact, double omega, int32_t nrhs,
               hipStream_t s, const int32_t *cnt, int32_t row0) {
    if (nx == 0) return;
    if (!rows && cnt) fail(LAIR_EINVAL, "a counted row list needs its rows");
    VT om = (VT)omega;
    if (cf)
        jacobi_launch<VT, true>(A, rows, row0, nx, cnt, b, xF, xC, cf, out, compact ? 1 : 0,
                                om, nrhs, s);
    else
        jacobi_launch<VT, false>(A, rows, row0, nx, cnt, b, xF, xF, nullptr, out,
                                 compact ? 1 : 0, om, nrhs, s);
}

template <class VT>
__global__ void k_scatter(int64_t total, int32_t nrhs, const int32_t *rows, int32_t row0,
                          const int32_t *cnt, const VT *t, VT *x) {
    const int64_t n = cnt ? (int64_t)*cnt * nrhs : total;
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < n;
         g += (int64_t)gridDim.x * blockDim.x) {
        int64_t k = g / nrhs;
        int q = (int)(g % nrhs);
        x[(int64_t)list_row(rows, row0, k) * nrhs + q] = t[g];
    }
}

// A contiguous row range: a straight copy, 16 bytes per thread.
__global__ void k_copy16(int64_t n16, const int4 *src, int4 *dst) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g < n16) dst[g] = src[g];
}

template <class VT>
void op_scatter(const int32_t *rows, int32_t nx, const VT *t, VT *x,
                int32_t nrhs, hipStream_t s, const int32_t *cnt, int32_t row0) {
    if (nx == 0) return;
    if (!rows && cnt) fail(LAIR_EINVAL, "a counted row list needs its rows");
    int64_t total = (int64_t)nx * nrhs;
    VT *dst = x + (int64_t)row0 * nrhs;
    if (!rows && (total * (int64_t)sizeof(VT)) % 16 == 0 && aligned16(t) && aligned16(dst)) {
        const int64_t n16 = total * (int64_t)sizeof(VT) / 16;
        LAIR_LAUNCH(k_copy16, dim3(blocks_for(n16, 256)), dim3(256), 0, s, n16,
                    reinterpret_cast<const int4 *>(t), reinterpret_cast<int4 *>(dst));
        LAIR_LAUNCH_CHECK();
        return;
    }
    LAIR_LAUNCH((k_scatter<VT>), dim3(cnt ? list_grid(total) : blocks_for(total, 256)),
                dim3(256), 0, s, total, nrhs, rows, row0, cnt, t, x);
    LAIR_LAUNCH_CHECK();
}

template <class VT>
__global__ void k_fill(VT *x, VT val, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] = val;
}

template <class VT>
void op_fill(VT *x, VT val, int64_t n, hipStream_t s) {
    if (n == 0) return;
    LAIR_LAUNCH((k_fill<VT>), dim3(blocks_for(n, 256)), dim3(256), 0, s, x, val, n);
    LAIR_LAUNCH_CHECK();
}

template <class VT>
__global__ void k_copy(const VT *x, VT *y, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = x[i];
}

template <class VT>
void op_copy(const VT *x, VT *y, int64_t n, hipStream_t s) {
    if (n == 0) return;
    LAIR_LAUNCH((k_copy<VT>), dim3(blocks_for(n, 256)), dim3(256), 0, s, x, y, n);
    LAIR_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// Coarsest grid: x = K^{-1} b (or K^{-T} b) from P K = L U, one block,
// right-hand sides in parallel.
// ---------------------------------------------------------------------------
template <class VT>
__global__ void __launch_bounds__(256)
k_dense_solve(int32_t n, const double *lu, const int32_t *piv, const VT *b,
              VT *x, int32_t nrhs, int transpose) {
    int t = threadIdx.x, nt = blockDim.x;
    int64_t tot = (int64_t)n * nrhs;
    for (int64_t g = t; g < tot; g += nt) x[g] = b[g];
    __syncthreads();
    if (!transpose) {
        for (int q = t; q < nrhs; q += nt)
            for (int k = 0; k < n; ++k) {
                int p = piv[k];
                if (p != k) {
                    VT a = x[(int64_t)k * nrhs + q];
                    x[(int64_t)k * nrhs + q] = x[(int64_t)p * nrhs + q];
                    x[(int64_t)p * nrhs + q] = a;
                }
            }
        __syncthreads();
        for (int k = 0; k < n; ++k) {                 // L y = P b (unit)
            int64_t w = (int64_t)(n - k - 1) * nrhs;
            for (int64_t g = t; g < w; g += nt) {
                int r = k + 1 + (int)(g / nrhs);
                int q = (int)(g % nrhs);
                x[(int64_t)r * nrhs + q] -= (VT)lu[(size_t)r * n + k] * x[(int64_t)k * nrhs + q];
            }
            __syncthreads();
        }
        for (int k = n - 1; k >= 0; --k) {            // U x = y
            for (int q = t; q < nrhs; q += nt)
                x[(int64_t)k * nrhs + q] /= (VT)lu[(size_t)k * n + k];
            __syncthreads();
            int64_t w = (int64_t)k * nrhs;
            for (int64_t g = t; g < w; g += nt) {
                int r = (int)(g / nrhs);
                int q = (int)(g % nrhs);
                x[(int64_t)r * nrhs + q] -= (VT)lu[(size_t)r * n + k] * x[(int64_t)k * nrhs + q];
            }
            __syncthreads();
        }
    } else {
        for (int k = 0; k < n; ++k) {                 // U^T w = b
            for (int q = t; q < nrhs; q += nt)
                x[(int64_t)k * nrhs + q] /= (VT)lu[(size_t)k * n + k];
            __syncthreads();
            int64_t w = (int64_t)(n - k - 1) * nrhs;
            for (int64_t g = t; g < w; g += nt) {
                int r = k + 1 + (int)(g / nrhs);
                int q = (int)(g % nrhs);
                x[(int64_t)r * nrhs + q] -= (VT)lu[(size_t)k * n + r] * x[(int64_t)k * nrhs + q];
            }
            __syncthreads();
        }
        for (int k = n - 1; k >= 0; --k) {            // L^T y = w (unit)
            int64_t w = (int64_t)k * nrhs;
            for (int64_t g = t; g < w; g += nt) {
                int r = (int)(g / nrhs);
                int q = (int)(g % nrhs);
                x[(int64_t)r * nrhs + q] -= (VT)lu[(size_t)k * n + r] * x[(int64_t)k * nrhs + q];
            }
            __syncthreads();
        }
        for (int q = t; q < nrhs; q += nt)            // x = P^T y
            for (int k = n - 1; k >= 0; --k) {
                int p = piv[k];
                if (p != k) {
                    VT a = x[(int64_t)k * nrhs + q];
                    x[(int64_t)k * nrhs + q] = x[(int64_t)p * nrhs + q];
                    x[(int64_t)p * nrhs + q] = a;
                }
            }
    }
}

template <class VT>
void op_dense_solve(int32_t n, const double *lu, const int32_t *piv,
                    const VT *b, VT *x, int32_t nrhs, bool transpose,
                    hipStream_t s) {
    LAIR_LAUNCH((k_dense_solve<VT>), dim3(1), dim3(256), 0, s, n, lu, piv, b, x,
                       nrhs, transpose ? 1 : 0);
    LAIR_LAUNCH_CHECK();
}

// Coarsest grid through its explicit inverse (small grids): x = Kinv b or
// Kinv^T b, accumulated in double whatever the vector type.
// x = K^{-1} b (or K^{-T} b) with the explicit inverse: a team of
// COARSE_T lanes per output entry, each lane summing every COARSE_T-th
// term, then a fixed shuffle tree.
constexpr int COARSE_T = 16;

template <class VT>
__global__ void __launch_bounds__(256)
k_coarse_apply(int32_t n, const double *kinv, const VT *b, VT *x, int32_t nrhs,
               int transpose) {
    const int64_t g = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / COARSE_T;
    const int lane = threadIdx.x % COARSE_T;
    if (g >= (int64_t)n * nrhs) return;
    const int32_t i = (int32_t)(g / nrhs);
    const int q = (int)(g % nrhs);
    double acc = 0.0;
    if (!transpose)
        for (int j = lane; j < n; j += COARSE_T)
            acc += kinv[(size_t)i * n + j] * (double)b[(int64_t)j * nrhs + q];
    else
        for (int j = lane; j < n; j += COARSE_T)
            acc += kinv[(size_t)j * n + i] * (double)b[(int64_t)j * nrhs + q];
    acc = team_sum<COARSE_T>(acc);
    if (lane == 0) x[g] = (VT)acc;
}

template <class VT>
void op_coarse_apply(int32_t n, const double *kinv, const VT *b, VT *x,
                     int32_t nrhs, bool transpose, hipStream_t s) {
    LAIR_LAUNCH((k_coarse_apply<VT>), dim3(blocks_for((int64_t)n * nrhs * COARSE_T, 256)),
                       dim3(256), 0, s, n, kinv, b, x, nrhs, transpose ? 1 : 0);
    LAIR_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// Sum of squares per right-hand side, fixed reduction order.
// ---------------------------------------------------------------------------
constexpr int NRM_BS = 256;

__global__ void __launch_bounds__(NRM_BS)
k_sumsq_partial(const double *r, int64_t total, int32_t nrhs, int64_t chunk,
                double *partial) {
    __shared__ double sh[NRM_BS];
    int t = threadIdx.x;
    int64_t lo = (int64_t)blockIdx.x * chunk;
    int64_t hi = lo + chunk < total ? lo + chunk : total;
    double acc = 0.0;
    for (int64_t g = lo + t; g < hi; g += NRM_BS) acc += r[g] * r[g];
    sh[t] = acc;
    __syncthreads();
    for (int o = NRM_BS / 2; o >= nrhs; o >>= 1) {
        if (t < o) sh[t] += sh[t + o];
        __syncthreads();
    }
    if (t < nrhs) partial[(int64_t)blockIdx.x * nrhs + t] = sh[t];
}

// one block per right-hand side; strided partial sums then a fixed tree
__global__ void __launch_bounds__(NRM_BS)
k_sumsq_final(const double *partial, int32_t nblk, int32_t nrhs, double *out) {
    __shared__ double sh[NRM_BS];
    int q = blockIdx.x;
    int t = threadIdx.x;
    double acc = 0.0;
    for (int b = t; b < nblk; b += NRM_BS) acc += partial[(int64_t)b * nrhs + q];
    sh[t] = acc;
    __syncthreads();
    for (int o = NRM_BS / 2; o > 0; o >>= 1) {
        if (t < o) sh[t] += sh[t + o];
        __syncthreads();
    }
    if (t == 0) out[q] = sh[0];
}

void op_sumsq(const double *r, int64_t n, int32_t nrhs, double *partial,
              int32_t npartial, double *out, hipStream_t s) {
    int64_t total = n * nrhs;
    // chunks are multiples of NRM_BS, so lane t always sees rhs t % nrhs
    int64_t per = (total + npartial - 1) / npartial;
    int64_t chunk = ((per + NRM_BS - 1) / NRM_BS) * NRM_BS;
    if (chunk < NRM_BS) chunk = NRM_BS;
    int32_t nblk = (int32_t)((total + chunk - 1) / chunk);
    if (nblk < 1) nblk = 1;
    LAIR_LAUNCH(k_sumsq_partial, dim3(nblk), dim3(NRM_BS), 0, s, r, total,
                       nrhs, chunk, partial);
    LAIR_LAUNCH_CHECK();
    LAIR_LAUNCH(k_sumsq_final, dim3(nrhs), dim3(NRM_BS), 0, s, partial, nblk, nrhs, out);
    LAIR_LAUNCH_CHECK();
}

template <int NR, int VW>
static void resid_norm_t(const CsrView<double> &A, const double *b, const double *x,
                         double *r64, float *r32, double *partial, unsigned grid, int T,
                         hipStream_t s, const int32_t *orow) {
    // two steps of a row's gathers in flight where a row needs more than one
    // (the sums keep their order)
    const bool u2 = vec_unroll<double>(NR, T, A.team) == 2;
#define LAIR_RN(O64, O32)                                                                  \
    {                                                                                      \
        if (u2)                                                                            \
            LAIR_LAUNCH((k_resid_norm<NR, VW, O64, O32, 2>), dim3(grid), dim3(256), 0, s,  \
                        A.nrows, T, A.rp, A.cj, A.v, x, b, r64, r32, partial, orow);       \
        else                                                                               \
            LAIR_LAUNCH((k_resid_norm<NR, VW, O64, O32, 1>), dim3(grid), dim3(256), 0, s,  \
                        A.nrows, T, A.rp, A.cj, A.v, x, b, r64, r32, partial, orow);       \
    }
    if (r64 && r32) LAIR_RN(true, true)
    else if (r64) LAIR_RN(true, false)
    else LAIR_RN(false, true)
#undef LAIR_RN
    LAIR_LAUNCH_CHECK();
}

bool op_residual_norm(const CsrView<double> &A, const double *b, const double *x,
                      double *r64, float *r32, int32_t nrhs, double *partial,
                      int32_t npartial, double *out, hipStream_t s, const int32_t *orow) {
    if (A.nrows == 0 || (!r64 && !r32)) return false;
    const int VW = nrhs == 1 ? 1 : 2;
    if (VW == 2 && !(aligned16(b) && aligned16(x) && (!r64 || aligned16(r64))))
        return false;
    const int L = nrhs / VW;
    const int T = vec_team(L, A.team);
    int64_t blocks = ((int64_t)A.nrows * T + 255) / 256;
    unsigned grid = (unsigned)(blocks < npartial ? (blocks < 1 ? 1 : blocks) : npartial);
    switch (nrhs) {
        case 1: resid_norm_t<1, 1>(A, b, x, r64, r32, partial, grid, T, s, orow); break;
        case 2: resid_norm_t<2, 2>(A, b, x, r64, r32, partial, grid, T, s, orow); break;
        case 4: resid_norm_t<4, 2>(A, b, x, r64, r32, partial, grid, T, s, orow); break;
        case 8: resid_norm_t<8, 2>(A, b, x, r64, r32, partial, grid, T, s, orow); break;
        case 16: resid_norm_t<16, 2>(A, b, x, r64, r32, partial, grid, T, s, orow); break;
        default: resid_norm_t<32, 2>(A, b, x, r64, r32, partial, grid, T, s, orow); break;
    }
    LAIR_LAUNCH(k_sumsq_final, dim3(nrhs), dim3(NRM_BS), 0, s, partial, (int32_t)grid,
                       nrhs, out);
    LAIR_LAUNCH_CHECK();
    return true;
}

__global__ void k_tag_columns(int64_t nnz, const int32_t *cj, const int8_t *cf, int32_t *cjt) {
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= nnz) return;
    const int32_t c = cj[p];
    cjt[p] = cf[c] == 1 ? (int32_t)((uint32_t)c | 0x80000000u) : c;
}

void launch_tag_columns(int64_t nnz, const int32_t *cj, const int8_t *cf, int32_t *cjt,
                        hipStream_t s) {
    if (nnz == 0) return;
    LAIR_LAUNCH(k_tag_columns, dim3(blocks_for(nnz, 256)), dim3(256), 0, s, nnz, cj, cf, cjt);
    LAIR_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// Mixed precision helpers and block scaling of right-hand sides.
// ---------------------------------------------------------------------------
template <class ET>
__global__ void k_update_list(const int32_t *rows, const int32_t *cnt, double *x, const ET *e) {
    const int32_t n = *cnt;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n;
         k += (int64_t)gridDim.x * blockDim.x) {
        const int32_t i = rows[k];
        x[i] += (double)e[i];
    }
}

template <class ET>
void op_update_list(const int32_t *rows, const int32_t *cnt, int32_t cap, double *x,
                    const ET *e, hipStream_t s) {
    if (cap == 0) return;
    LAIR_LAUNCH((k_update_list<ET>), dim3(list_grid(cap)), dim3(256), 0, s, rows, cnt, x, e);
    LAIR_LAUNCH_CHECK();
}

__global__ void k_axpy_f32(double *x, const float *e, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] += (double)e[i];
}

// Row-mapped vector operations on n x nrhs blocks (nrhs a power of two),
// VW consecutive entries of a row per thread; lgv = log2(nrhs / VW).
// x[i] += e[map[i]] (e in another ordering)
template <int VW>
__global__ void k_axpy_f32_rows(double *x, const float *e, const float *e_hi, int32_t split,
                                const int32_t *map, int64_t nv, int lgv) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= nv) return;
    const int64_t i = g >> lgv;
    const int32_t m = map[i];
    if (e_hi && m >= split) e = e_hi;
    const int64_t src = (((int64_t)m << lgv) | (g & ((1 << lgv) - 1))) * VW;
    constexpr int XW = VW >= 2 ? 2 : 1;    // x in 16-byte pieces
    Pack<float, VW> ev;
    ev.load(e + src);
#pragma unroll
    for (int h = 0; h < VW / XW; ++h) {
        Pack<double, XW> xv;
        xv.load(x + g * VW + h * XW);
#pragma unroll
        for (int k = 0; k < XW; ++k) xv.v[k] += (double)ev.v[h * XW + k];
        xv.store(x + g * VW + h * XW);
    }
}

// out[map[i]] = (float) in[i]
template <int VW>
__global__ void k_cast_f32_rows(const double *in, float *out, const int32_t *map, int64_t nv,
                                int lgv) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= nv) return;
    const int64_t i = g >> lgv;
    const int64_t dst = (((int64_t)map[i] << lgv) | (g & ((1 << lgv) - 1))) * VW;
    constexpr int XW = VW >= 2 ? 2 : 1;
    Pack<float, VW> ov;
#pragma unroll
    for (int h = 0; h < VW / XW; ++h) {
        Pack<double, XW> iv;
        iv.load(in + g * VW + h * XW);
#pragma unroll
        for (int k = 0; k < XW; ++k) ov.v[h * XW + k] = (float)iv.v[k];
    }
    ov.store(out + dst);
}

static int ilog2(int32_t v) {
    int l = 0;
    while ((1 << l) < v) ++l;
    return l;
}

void op_axpy_f32_rows(double *x, const float *e, const int32_t *map, int64_t n, int32_t nrhs,
                      hipStream_t s, const float *e_hi, int32_t split) {
    if (n == 0) return;
    if (nrhs % 4 == 0 && aligned16(x) && aligned16(e) && (!e_hi || aligned16(e_hi))) {
        const int64_t nv = n * nrhs / 4;
        LAIR_LAUNCH(k_axpy_f32_rows<4>, dim3(blocks_for(nv, 256)), dim3(256), 0, s, x, e, e_hi,
                    split, map, nv, ilog2(nrhs / 4));
    } else {
        LAIR_LAUNCH(k_axpy_f32_rows<1>, dim3(blocks_for(n * nrhs, 256)), dim3(256), 0, s, x, e,
                    e_hi, split, map, n * nrhs, ilog2(nrhs));
    }
    LAIR_LAUNCH_CHECK();
}

void op_cast_f32_rows(const double *in, float *out, const int32_t *map, int64_t n,
                      int32_t nrhs, hipStream_t s) {
    if (n == 0) return;
    if (nrhs % 4 == 0 && aligned16(in)) {
        const int64_t nv = n * nrhs / 4;
        LAIR_LAUNCH(k_cast_f32_rows<4>, dim3(blocks_for(nv, 256)), dim3(256), 0, s, in, out,
                    map, nv, ilog2(nrhs / 4));
    } else {
        LAIR_LAUNCH(k_cast_f32_rows<1>, dim3(blocks_for(n * nrhs, 256)), dim3(256), 0, s, in,
                    out, map, n * nrhs, ilog2(nrhs));
    }
    LAIR_LAUNCH_CHECK();
}

void op_axpy_f32(double *x, const float *e, int64_t n, hipStream_t s) {
    if (n == 0) return;
    LAIR_LAUNCH(k_axpy_f32, dim3(blocks_for(n, 256)), dim3(256), 0, s, x, e, n);
    LAIR_LAUNCH_CHECK();
}

__global__ void k_cast_f32(const double *in, float *out, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = (float)in[i];
}

void op_cast_f32(const double *in, float *out, int64_t n, hipStream_t s) {
    if (n == 0) return;
    LAIR_LAUNCH(k_cast_f32, dim3(blocks_for(n, 256)), dim3(256), 0, s, in, out, n);
    LAIR_LAUNCH_CHECK();
}

__global__ void k_cast_f64(const float *in, double *out, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = (double)in[i];
}

void op_cast_f64(const float *in, double *out, int64_t n, hipStream_t s) {
    if (n == 0) return;
    LAIR_LAUNCH(k_cast_f64, dim3(blocks_for(n, 256)), dim3(256), 0, s, in, out, n);
    LAIR_LAUNCH_CHECK();
}

__global__ void k_block_apply(int32_t nblk, int32_t k, const double *dinv,
                              const double *b, double *out, int32_t nrhs) {
    int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t n = (int64_t)nblk * k;
    if (g >= n * nrhs) return;
    int64_t i = g / nrhs;
    int q = (int)(g % nrhs);
    int64_t e = i / k;
    int r = (int)(i % k);
    const double *d = dinv + (size_t)e * k * k + (size_t)r * k;
    double acc = 0.0;
    for (int c = 0; c < k; ++c) acc += d[c] * b[(e * k + c) * nrhs + q];
    out[g] = acc;
}

void op_block_apply(int32_t nblk, int32_t k, const double *dinv,
                    const double *b, double *out, int32_t nrhs, hipStream_t s) {
    int64_t tot = (int64_t)nblk * k * nrhs;
    LAIR_LAUNCH(k_block_apply, dim3(blocks_for(tot, 256)), dim3(256), 0, s,
                       nblk, k, dinv, b, out, nrhs);
    LAIR_LAUNCH_CHECK();
}

// explicit instantiations
template void op_residual<double>(const CsrView<double> &, const double *, const double *, double *, int32_t, hipStream_t);
template void op_residual<float>(const CsrView<float> &, const float *, const float *, float *, int32_t, hipStream_t);
template void op_spmv<double>(const CsrView<double> &, const double *, double *, int32_t, bool, hipStream_t, const double *, int32_t, const int8_t *);
template void op_spmv<float>(const CsrView<float> &, const float *, float *, int32_t, bool, hipStream_t, const float *, int32_t, const int8_t *);
template void op_jacobi<double>(const CsrView<double> &, const int32_t *, int32_t, const double *, const double *, const double *, const int8_t *, double *, bool, double, int32_t, hipStream_t, const int32_t *, int32_t);
template void op_jacobi<float>(const CsrView<float> &, const int32_t *, int32_t, const float *, const float *, const float *, const int8_t *, float *, bool, double, int32_t, hipStream_t, const int32_t *, int32_t);
template void op_rowdot_list<double>(const CsrView<double> &, int, const int32_t *, const int32_t *, int32_t, const double *, const double *, double *, hipStream_t);
template void op_rowdot_list<float>(const CsrView<float> &, int, const int32_t *, const int32_t *, int32_t, const float *, const float *, float *, hipStream_t);
template void op_update_list<double>(const int32_t *, const int32_t *, int32_t, double *, const double *, hipStream_t);
template void op_update_list<float>(const int32_t *, const int32_t *, int32_t, double *, const float *, hipStream_t);
template void op_coarse_apply<double>(int32_t, const double *, const double *, double *, int32_t, bool, hipStream_t);
template void op_coarse_apply<float>(int32_t, const double *, const float *, float *, int32_t, bool, hipStream_t);
template void op_scatter<double>(const int32_t *, int32_t, const double *, double *, int32_t, hipStream_t, const int32_t *, int32_t);
template void op_scatter<float>(const int32_t *, int32_t, const float *, float *, int32_t, hipStream_t, const int32_t *, int32_t);
template void op_fill<double>(double *, double, int64_t, hipStream_t);
template void op_fill<float>(float *, float, int64_t, hipStream_t);
template void op_copy<double>(const double *, double *, int64_t, hipStream_t);
template void op_copy<float>(const float *, float *, int64_t, hipStream_t);
template void op_dense_solve<double>(int32_t, const double *, const int32_t *, const double *, double *, int32_t, bool, hipStream_t);
template void op_dense_solve<float>(int32_t, const double *, const int32_t *, const float *, float *, int32_t, bool, hipStream_t);

// Row permutation of an n x nrhs block (row-major, nrhs a power of two):
// to_split gathers out[k] = in[perm[k]], otherwise out[perm[k]] = in[k]
// (back to natural); VW entries per thread, lgv = log2(nrhs / VW).
template <int VW>
__global__ void k_permute_rows(const int32_t *perm, const double *in, double *out, int64_t nv,
                               int lgv, int to_split) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= nv) return;
    const int64_t k = g >> lgv;
    const int64_t o = (((int64_t)perm[k] << lgv) | (g & ((1 << lgv) - 1))) * VW;
    Pack<double, VW> v;
    if (to_split) {
        v.load(in + o);
        v.store(out + g * VW);
    } else {
        v.load(in + g * VW);
        v.store(out + o);
    }
}

void op_permute_rows(int64_t n, int32_t nrhs, const int32_t *perm, const double *in,
                     double *out, bool to_split, hipStream_t s) {
    if (n == 0) return;
    if (nrhs % 2 == 0 && aligned16(in) && aligned16(out)) {
        const int64_t nv = n * nrhs / 2;
        LAIR_LAUNCH(k_permute_rows<2>, dim3(blocks_for(nv, 256)), dim3(256), 0, s, perm, in,
                    out, nv, ilog2(nrhs / 2), to_split ? 1 : 0);
    } else {
        LAIR_LAUNCH(k_permute_rows<1>, dim3(blocks_for(n * nrhs, 256)), dim3(256), 0, s, perm,
                    in, out, n * nrhs, ilog2(nrhs), to_split ? 1 : 0);
    }
    LAIR_LAUNCH_CHECK();
}

}  // namespace lair
