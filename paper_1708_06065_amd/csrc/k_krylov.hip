// Kernels of the flexible GMRES outer iteration (the Krylov solver the paper
// wraps its V-cycles in, Sec. 4).  Vectors hold R right-hand sides
// interleaved (element (i, q) at i R + q, R a power of two up to 32), as in
// the cycle; a basis is kc such vectors ldv elements apart.  Every kernel is
// a stream over HBM; the dot products reduce in a fixed order (per thread,
// then a fixed tree per block, then over the blocks in order), so their
// results do not depend on timing.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "k_common.hpp"
#include "lair_internal.hpp"

namespace lair {

constexpr int KRY_BS = 256;
constexpr int KRY_KC = 8;        // basis vectors per dot-product pass

// partial[(blk * kstride + kbase + k) * R + q] = the block's part of
// sum_i V_{kbase+k}[i R + q] w[i R + q], k < kc <= KRY_KC.  The grid stride
// is a multiple of R, so each thread keeps one right-hand side.
__global__ void __launch_bounds__(KRY_BS)
k_mdot(int64_t m, int R, const double *V, int64_t ldv, int kbase, int kc, int kstride,
       const double *w, double *partial) {
    __shared__ double sh[KRY_BS];
    double acc[KRY_KC];
#pragma unroll
    for (int k = 0; k < KRY_KC; ++k) acc[k] = 0.0;
    const double *Vb = V + (int64_t)kbase * ldv;
    const int64_t stride = (int64_t)gridDim.x * KRY_BS;
    for (int64_t e = (int64_t)blockIdx.x * KRY_BS + threadIdx.x; e < m; e += stride) {
        const double wv = w[e];
#pragma unroll
        for (int k = 0; k < KRY_KC; ++k)
            if (k < kc) acc[k] += Vb[(int64_t)k * ldv + e] * wv;
    }
    const int t = threadIdx.x;
    for (int k = 0; k < kc; ++k) {
        sh[t] = acc[k];
        __syncthreads();
        for (int o = KRY_BS / 2; o >= R; o >>= 1) {
            if (t < o) sh[t] += sh[t + o];
            __syncthreads();
        }
        if (t < R) partial[((int64_t)blockIdx.x * kstride + kbase + k) * R + t] = sh[t];
        __syncthreads();
    }
}

// out[k R + q] = sum over the blocks, in order, of their parts.
__global__ void __launch_bounds__(KRY_BS)
k_mdot_final(int nblk, int kc, int R, const double *partial, double *out) {
    const int idx = blockIdx.x * KRY_BS + threadIdx.x;
    if (idx >= kc * R) return;
    double a = 0.0;
    for (int b = 0; b < nblk; ++b) a += partial[(int64_t)b * kc * R + idx];
    out[idx] = a;
}

// w[i R + q] -= sum_k coef[k R + q] V_k[i R + q], k ascending.
__global__ void __launch_bounds__(KRY_BS)
k_maxpy(int64_t m, int R, const double *V, int64_t ldv, int kc, const double *coef,
        double *w) {
    const int64_t e = (int64_t)blockIdx.x * KRY_BS + threadIdx.x;
    if (e >= m) return;
    const int q = (int)(e & (R - 1));
    double a = 0.0;
    for (int k = 0; k < kc; ++k) a += coef[k * R + q] * V[(int64_t)k * ldv + e];
    w[e] -= a;
}

// out[i R + q] = w[i R + q] * s[q]
__global__ void __launch_bounds__(KRY_BS)
k_scale_rhs(int64_t m, int R, const double *w, const double *s, double *out) {
    const int64_t e = (int64_t)blockIdx.x * KRY_BS + threadIdx.x;
    if (e >= m) return;
    out[e] = w[e] * s[e & (R - 1)];
}

static bool pow2_rhs(int R) { return R >= 1 && R <= 32 && (R & (R - 1)) == 0; }

int32_t kry_dot_blocks(int64_t m) {
    const int64_t b = (m + KRY_BS - 1) / KRY_BS;
    return (int32_t)std::max<int64_t>(1, std::min<int64_t>(b, 1024));
}

void op_mdot(int64_t n, int32_t R, const double *V, int64_t ldv, int32_t kc, const double *w,
             double *partial, double *out, hipStream_t s) {
    if (!pow2_rhs(R)) fail(LAIR_EINVAL, "right-hand sides must be a power of two up to 32");
    if (kc < 1) return;
    const int64_t m = n * R;
    const int32_t nblk = kry_dot_blocks(m);
    for (int kb = 0; kb < kc; kb += KRY_KC) {
        const int c = std::min(KRY_KC, kc - kb);
        LAIR_LAUNCH(k_mdot, dim3(nblk), dim3(KRY_BS), 0, s, m, R, V, ldv, kb, c, kc, w,
                    partial);
        LAIR_LAUNCH_CHECK();
    }
    LAIR_LAUNCH(k_mdot_final, dim3((kc * R + KRY_BS - 1) / KRY_BS), dim3(KRY_BS), 0, s, nblk,
                kc, R, partial, out);
    LAIR_LAUNCH_CHECK();
}

void op_maxpy(int64_t n, int32_t R, const double *V, int64_t ldv, int32_t kc,
              const double *coef, double *w, hipStream_t s) {
    if (!pow2_rhs(R)) fail(LAIR_EINVAL, "right-hand sides must be a power of two up to 32");
    if (kc < 1 || n == 0) return;
    const int64_t m = n * R;
    LAIR_LAUNCH(k_maxpy, dim3(blocks_for(m, KRY_BS)), dim3(KRY_BS), 0, s, m, R, V, ldv, kc,
                coef, w);
    LAIR_LAUNCH_CHECK();
}

void op_scale_rhs(int64_t n, int32_t R, const double *w, const double *sc, double *out,
                  hipStream_t s) {
    if (!pow2_rhs(R)) fail(LAIR_EINVAL, "right-hand sides must be a power of two up to 32");
    if (n == 0) return;
    const int64_t m = n * R;
    LAIR_LAUNCH(k_scale_rhs, dim3(blocks_for(m, KRY_BS)), dim3(KRY_BS), 0, s, m, R, w, sc, out);
    LAIR_LAUNCH_CHECK();
}

}  // namespace lair
