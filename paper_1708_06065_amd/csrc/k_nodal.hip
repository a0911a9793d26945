// Nodal treatment of a k x k block structure (Sec. 3.1, the block form of
// Eq. (system); Sec. 4.2, treatment (iii)): strength by block norms,
// one-point interpolation by block, and the block-scaled copies the block
// Jacobi sweeps read.  A is a scalar CSR matrix whose stored blocks are
// dense: the k rows of node i (rows i k .. i k + k - 1) store the same
// columns, in whole ascending groups of k that start at a multiple of k.
// The local systems of a node are the scalar ones of its k rows (the same
// matrix A(N,N)^T, one right-hand side per row), so they need no kernel of
// their own.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>

#include "k_common.hpp"
#include "lair_internal.hpp"

namespace lair {

constexpr int NODE_BS = 256;

// Teams: the kernels below give a team of T lanes (a power of two, 4 ..
// 64) to each row or node; the lanes take the row's entries or the node's
// blocks in turn, so that the long rows of the coarse levels (hundreds of
// blocks) are spread over lanes instead of one lane walking them.  T is
// chosen from the mean row length.
static int node_team(int64_t nnz, int32_t n, int32_t per) {
    const double m = n ? (double)nnz / n / per : 1.0;
    int t = 4;
    while (t < 64 && t < m) t <<= 1;
    return t;
}

#define LAIR_NODE_TEAMS(T_EXPR, LAUNCH)                   \
    switch (T_EXPR) {                                     \
        case 4: { constexpr int T = 4; LAUNCH; } break;   \
        case 8: { constexpr int T = 8; LAUNCH; } break;   \
        case 16: { constexpr int T = 16; LAUNCH; } break; \
        case 32: { constexpr int T = 32; LAUNCH; } break; \
        default: { constexpr int T = 64; LAUNCH; } break; \
    }

// bad |= 1 when a row of node i stores other columns than the node's first
// row, or a group of k columns is not one whole block.  A team per row;
// entry p of a group starting at column c0 must be c0 + (p mod k) in the
// row and in the node's first row, with c0 a multiple of k.
template <int T>
__global__ void __launch_bounds__(NODE_BS)
k_node_check(int32_t n, int32_t k, const int32_t *rp, const int32_t *cj, int32_t *bad) {
    const int64_t g = (int64_t)blockIdx.x * NODE_BS + threadIdx.x;
    const int32_t r = (int32_t)(g / T);
    const int lane = (int)(g % T);
    if (r >= n) return;
    const int32_t r0 = (r / k) * k;
    const int32_t lo = rp[r], len = rp[r + 1] - lo;
    const int32_t lo0 = rp[r0], len0 = rp[r0 + 1] - lo0;
    bool ok = len == len0 && len % k == 0;
    for (int32_t p = lane; ok && p < len; p += T) {
        const int32_t u = p % k;
        const int32_t c0 = cj[lo + p - u];
        ok = c0 % k == 0 && cj[lo + p] == c0 + u && cj[lo0 + p] == c0 + u;
    }
    if (!ok) atomicOr(bad, 1);
}

// Squared Frobenius norm of block t of node i: rows ascending, then columns
// ascending, every product rounded before it is added (no fused
// multiply-add), so that both sides of a comparison are reproducible.
__device__ __forceinline__ double node_block_sq(const int32_t *rp, const double *v, int32_t i,
                                                int32_t k, int32_t t) {
#pragma clang fp contract(off)
    double acc = 0.0;
    for (int32_t a = 0; a < k; ++a) {
        const double *row = v + rp[i * k + a] + (int64_t)t * k;
        for (int32_t u = 0; u < k; ++u) {
            const double sq = row[u] * row[u];
            acc = acc + sq;
        }
    }
    return acc;
}

// Strength by blocks: block (i, j) is strong when
// ||A_ij||^2 >= theta^2 max_{l != i} ||A_il||^2 (norms squared as above), it
// is not zero and the node has a nonzero off-diagonal block.  Every stored
// entry of a strong block is marked in smask (the scalar strength mask the
// neighbourhoods and the interpolation read).  A team per node, lanes over
// the node's blocks.
template <int T>
__global__ void __launch_bounds__(NODE_BS)
k_node_strength(int32_t nn, int32_t k, const int32_t *rp, const int32_t *cj, const double *v,
                double theta, uint8_t *smask) {
    const int64_t g = (int64_t)blockIdx.x * NODE_BS + threadIdx.x;
    const int32_t i = (int32_t)(g / T);
    const int lane = (int)(g % T);
    if (i >= nn) return;
    const int32_t lo0 = rp[i * k];
    const int32_t nb = (rp[i * k + 1] - lo0) / k;
    double m = 0.0;
    for (int32_t t = lane; t < nb; t += T) {
        if (cj[lo0 + t * k] / k == i) continue;
        const double sq = node_block_sq(rp, v, i, k, t);
        if (sq > m) m = sq;
    }
    m = team_max<T>(m);
    const double th2 = theta * theta;
    const double cut = th2 * m;
    for (int32_t t = lane; t < nb; t += T) {
        uint8_t s = 0;
        if (cj[lo0 + t * k] / k != i && m > 0.0) {
            const double sq = node_block_sq(rp, v, i, k, t);
            s = (sq > 0.0 && sq >= cut) ? 1 : 0;
        }
        for (int32_t a = 0; a < k; ++a) {
            uint8_t *row = smask + rp[i * k + a] + (int64_t)t * k;
            for (int32_t u = 0; u < k; ++u) row[u] = s;
        }
    }
}

// One-point interpolation by block: F-node i takes the identity block from
// the strong C-node neighbour with the largest block norm (the first in
// column order on a tie); row a of the node interpolates from row a of that
// C-node.  A C-row injects.  pcol[r] = coarse column or -1.  A team per
// node, lanes over the node's blocks.
template <int T>
__global__ void __launch_bounds__(NODE_BS)
k_interp_1p_node(int32_t nn, int32_t k, const int32_t *rp, const int32_t *cj, const double *v,
                 const uint8_t *smask, const int8_t *cf, const int32_t *cidx, int32_t *pcol) {
    const int64_t g = (int64_t)blockIdx.x * NODE_BS + threadIdx.x;
    const int32_t i = (int32_t)(g / T);
    const int lane = (int)(g % T);
    if (i >= nn) return;
    const int32_t lo0 = rp[i * k];
    const int32_t nb = (rp[i * k + 1] - lo0) / k;
    int best = INT_MAX;
    double bv = -1.0;
    for (int32_t t = lane; t < nb; t += T) {
        const int32_t c0 = cj[lo0 + t * k];
        if (c0 / k == i || !smask[lo0 + t * k] || cf[c0] != 1) continue;
        const double sq = node_block_sq(rp, v, i, k, t);
        if (sq > bv) {
            bv = sq;
            best = t;
        }
    }
    team_argmax<T>(bv, best);
    const int32_t bc = best < nb ? cj[lo0 + best * k] : -1;
    for (int32_t a = lane; a < k; a += T) {
        const int32_t r = i * k + a;
        pcol[r] = cf[r] == 1 ? cidx[r] : (bc >= 0 ? cidx[bc + a] : -1);
    }
}

// out = D^{-1} A on A's pattern: out[p] for row (i, a) at offset o of the
// row is sum_b dinv_i[a][b] v[rp[i k + b] + o], b ascending.  A team per
// node, lanes over the offsets (the k rows of a node have one length): a
// lane loads the node's k values at its offset once and writes all k rows.
constexpr int NODE_KMAX = 8;

template <int T>
__global__ void __launch_bounds__(NODE_BS)
k_node_scale(int32_t nn, int32_t k, const int32_t *rp, const double *v, const double *dinv,
             double *out) {
    const int64_t g = (int64_t)blockIdx.x * NODE_BS + threadIdx.x;
    const int32_t i = (int32_t)(g / T);
    const int lane = (int)(g % T);
    if (i >= nn) return;
    int32_t lo[NODE_KMAX];
#pragma unroll
    for (int b = 0; b < NODE_KMAX; ++b) lo[b] = b < k ? rp[i * k + b] : 0;
    const int32_t len = rp[i * k + 1] - lo[0];
    const double *d = dinv + (int64_t)i * k * k;
    for (int32_t o = lane; o < len; o += T) {
        double vb[NODE_KMAX];
#pragma unroll
        for (int b = 0; b < NODE_KMAX; ++b) vb[b] = b < k ? v[lo[b] + o] : 0.0;
#pragma unroll
        for (int a = 0; a < NODE_KMAX; ++a) {
            if (a >= k) break;
            double acc = 0.0;
#pragma unroll
            for (int b = 0; b < NODE_KMAX; ++b)
                if (b < k) acc += d[a * k + b] * vb[b];
            out[lo[a] + o] = acc;
        }
    }
}

// out[(i k + a) R + q] = sum_b dinv_i[a][b] b[(i k + b) R + q]: the
// right-hand side of the block Jacobi sweeps.  One thread per element.
template <class VT>
__global__ void __launch_bounds__(NODE_BS)
k_node_rhs(int64_t m, int32_t k, int32_t R, const double *dinv, const VT *b, VT *out) {
    const int64_t g = (int64_t)blockIdx.x * NODE_BS + threadIdx.x;
    if (g >= m) return;
    const int64_t row = g / R;
    const int32_t q = (int32_t)(g - row * R);
    const int64_t i = row / k;
    const int32_t a = (int32_t)(row - i * k);
    const double *d = dinv + (i * k + a) * k;
    const VT *bb = b + i * k * R + q;
    double acc = 0.0;
    for (int32_t c = 0; c < k; ++c) acc += d[c] * (double)bb[(int64_t)c * R];
    out[g] = (VT)acc;
}

bool node_check(int32_t n, int32_t k, const int32_t *rp, const int32_t *cj, int64_t nnz,
                hipStream_t s) {
    if (n == 0) return true;
    DevArr<int32_t> bad;
    bad.alloc(1, s);
    LAIR_HIP(hipMemsetAsync(bad.get(), 0, sizeof(int32_t), s));
    LAIR_NODE_TEAMS(node_team(nnz, n, 1),
                    LAIR_LAUNCH(k_node_check<T>, dim3(blocks_for((int64_t)n * T, NODE_BS)),
                                dim3(NODE_BS), 0, s, n, k, rp, cj, bad.get()));
    LAIR_LAUNCH_CHECK();
    int32_t hb = 0;
    Readback rb(s);
    rb.add(&hb, bad.get(), sizeof(int32_t));
    rb.run();
    return hb == 0;
}

void launch_node_strength(int32_t n, int32_t k, const int32_t *rp, const int32_t *cj,
                          const double *v, int64_t nnz, double theta, uint8_t *smask,
                          hipStream_t s) {
    const int32_t nn = n / k;
    if (nn == 0) return;
    LAIR_NODE_TEAMS(node_team(nnz, n, k),
                    LAIR_LAUNCH(k_node_strength<T>, dim3(blocks_for((int64_t)nn * T, NODE_BS)),
                                dim3(NODE_BS), 0, s, nn, k, rp, cj, v, theta, smask));
    LAIR_LAUNCH_CHECK();
}

void launch_interp_1p_node(int32_t n, int32_t k, const int32_t *rp, const int32_t *cj,
                           const double *v, int64_t nnz, const uint8_t *smask, const int8_t *cf,
                           const int32_t *cidx, int32_t *pcol, hipStream_t s) {
    const int32_t nn = n / k;
    if (nn == 0) return;
    LAIR_NODE_TEAMS(node_team(nnz, n, k),
                    LAIR_LAUNCH(k_interp_1p_node<T>, dim3(blocks_for((int64_t)nn * T, NODE_BS)),
                                dim3(NODE_BS), 0, s, nn, k, rp, cj, v, smask, cf, cidx, pcol));
    LAIR_LAUNCH_CHECK();
}

void launch_node_scale(int32_t n, int32_t k, const int32_t *rp, const double *v, int64_t nnz,
                       const double *dinv, double *out, hipStream_t s) {
    const int32_t nn = n / k;
    if (nn == 0) return;
    if (k > NODE_KMAX) fail(LAIR_EUNSUPPORTED, "block size %d > %d", k, NODE_KMAX);
    LAIR_NODE_TEAMS(node_team(nnz, n, 1),
                    LAIR_LAUNCH(k_node_scale<T>, dim3(blocks_for((int64_t)nn * T, NODE_BS)),
                                dim3(NODE_BS), 0, s, nn, k, rp, v, dinv, out));
    LAIR_LAUNCH_CHECK();
}

template <class VT>
void op_node_rhs(int32_t n, int32_t k, int32_t nrhs, const double *dinv, const VT *b, VT *out,
                 hipStream_t s) {
    const int64_t m = (int64_t)n * nrhs;
    if (m == 0) return;
    LAIR_LAUNCH(k_node_rhs<VT>, dim3(blocks_for(m, NODE_BS)), dim3(NODE_BS), 0, s, m, k, nrhs,
                dinv, b, out);
    LAIR_LAUNCH_CHECK();
}

template void op_node_rhs<double>(int32_t, int32_t, int32_t, const double *, const double *,
                                  double *, hipStream_t);
template void op_node_rhs<float>(int32_t, int32_t, int32_t, const double *, const float *,
                                 float *, hipStream_t);

}  // namespace lair
