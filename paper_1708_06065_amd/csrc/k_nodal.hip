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

#include "k_common.hpp"
#include "lair_internal.hpp"

namespace lair {

constexpr int NODE_BS = 256;

// bad |= 1 when a row of node i stores other columns than the node's first
// row, or a group of k columns is not one whole block.  One thread per row.
__global__ void __launch_bounds__(NODE_BS)
k_node_check(int32_t n, int32_t k, const int32_t *rp, const int32_t *cj, int32_t *bad) {
    const int32_t r = blockIdx.x * NODE_BS + threadIdx.x;
    if (r >= n) return;
    const int32_t r0 = (r / k) * k;
    const int32_t lo = rp[r], len = rp[r + 1] - lo;
    const int32_t lo0 = rp[r0], len0 = rp[r0 + 1] - lo0;
    bool ok = len == len0 && len % k == 0;
    for (int32_t p = 0; ok && p < len; p += k) {
        const int32_t c0 = cj[lo + p];
        ok = c0 % k == 0;
        for (int32_t u = 0; ok && u < k; ++u)
            ok = cj[lo + p + u] == c0 + u && cj[lo0 + p + u] == c0 + u;
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
// neighbourhoods and the interpolation read).  One thread per node.
__global__ void __launch_bounds__(NODE_BS)
k_node_strength(int32_t nn, int32_t k, const int32_t *rp, const int32_t *cj, const double *v,
                double theta, uint8_t *smask) {
    const int32_t i = blockIdx.x * NODE_BS + threadIdx.x;
    if (i >= nn) return;
    const int32_t lo0 = rp[i * k];
    const int32_t nb = (rp[i * k + 1] - lo0) / k;
    double m = 0.0;
    for (int32_t t = 0; t < nb; ++t) {
        if (cj[lo0 + t * k] / k == i) continue;
        const double sq = node_block_sq(rp, v, i, k, t);
        if (sq > m) m = sq;
    }
    const double th2 = theta * theta;
    const double cut = th2 * m;
    for (int32_t t = 0; t < nb; ++t) {
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
// C-node.  A C-row injects.  pcol[r] = coarse column or -1.  One thread per
// row.
__global__ void __launch_bounds__(NODE_BS)
k_interp_1p_node(int32_t n, int32_t k, const int32_t *rp, const int32_t *cj, const double *v,
                 const uint8_t *smask, const int8_t *cf, const int32_t *cidx, int32_t *pcol) {
    const int32_t r = blockIdx.x * NODE_BS + threadIdx.x;
    if (r >= n) return;
    if (cf[r] == 1) {
        pcol[r] = cidx[r];
        return;
    }
    const int32_t i = r / k, a = r - i * k;
    const int32_t lo0 = rp[i * k];
    const int32_t nb = (rp[i * k + 1] - lo0) / k;
    int32_t best = -1;
    double bv = -1.0;
    for (int32_t t = 0; t < nb; ++t) {
        const int32_t c0 = cj[lo0 + t * k];
        if (c0 / k == i || !smask[lo0 + t * k] || cf[c0] != 1) continue;
        const double sq = node_block_sq(rp, v, i, k, t);
        if (sq > bv) {
            bv = sq;
            best = c0;
        }
    }
    pcol[r] = best >= 0 ? cidx[best + a] : -1;
}

// out = D^{-1} A on A's pattern: out[p] for row (i, a) at offset o of the
// row is sum_b dinv_i[a][b] v[rp[i k + b] + o], b ascending.  One thread per
// row.
__global__ void __launch_bounds__(NODE_BS)
k_node_scale(int32_t n, int32_t k, const int32_t *rp, const double *v, const double *dinv,
             double *out) {
    const int32_t r = blockIdx.x * NODE_BS + threadIdx.x;
    if (r >= n) return;
    const int32_t i = r / k, a = r - i * k;
    const double *d = dinv + ((int64_t)i * k + a) * k;
    const int32_t lo = rp[r], len = rp[r + 1] - lo;
    for (int32_t o = 0; o < len; ++o) {
        double acc = 0.0;
        for (int32_t b = 0; b < k; ++b) acc += d[b] * v[rp[i * k + b] + o];
        out[lo + o] = acc;
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

bool node_check(int32_t n, int32_t k, const int32_t *rp, const int32_t *cj, hipStream_t s) {
    if (n == 0) return true;
    DevArr<int32_t> bad;
    bad.alloc(1, s);
    LAIR_HIP(hipMemsetAsync(bad.get(), 0, sizeof(int32_t), s));
    LAIR_LAUNCH(k_node_check, dim3(blocks_for(n, NODE_BS)), dim3(NODE_BS), 0, s, n, k, rp, cj,
                bad.get());
    LAIR_LAUNCH_CHECK();
    int32_t hb = 0;
    Readback rb(s);
    rb.add(&hb, bad.get(), sizeof(int32_t));
    rb.run();
    return hb == 0;
}

void launch_node_strength(int32_t n, int32_t k, const int32_t *rp, const int32_t *cj,
                          const double *v, double theta, uint8_t *smask, hipStream_t s) {
    const int32_t nn = n / k;
    if (nn == 0) return;
    LAIR_LAUNCH(k_node_strength, dim3(blocks_for(nn, NODE_BS)), dim3(NODE_BS), 0, s, nn, k, rp,
                cj, v, theta, smask);
    LAIR_LAUNCH_CHECK();
}

void launch_interp_1p_node(int32_t n, int32_t k, const int32_t *rp, const int32_t *cj,
                           const double *v, const uint8_t *smask, const int8_t *cf,
                           const int32_t *cidx, int32_t *pcol, hipStream_t s) {
    if (n == 0) return;
    LAIR_LAUNCH(k_interp_1p_node, dim3(blocks_for(n, NODE_BS)), dim3(NODE_BS), 0, s, n, k, rp,
                cj, v, smask, cf, cidx, pcol);
    LAIR_LAUNCH_CHECK();
}

void launch_node_scale(int32_t n, int32_t k, const int32_t *rp, const double *v,
                       const double *dinv, double *out, hipStream_t s) {
    if (n == 0) return;
    LAIR_LAUNCH(k_node_scale, dim3(blocks_for(n, NODE_BS)), dim3(NODE_BS), 0, s, n, k, rp, v,
                dinv, out);
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
