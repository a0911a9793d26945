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
// y = b - A x   (or y = A x, y += A x), one right-hand side, T lanes per row
// ---------------------------------------------------------------------------
enum { MODE_RESID = 0, MODE_SET = 1, MODE_ADD = 2 };

template <class VT, int T, int MODE>
__global__ void __launch_bounds__(256)
k_rowdot1(int32_t nrows, const int32_t *rp, const int32_t *cj, const VT *v,
          const VT *x, const VT *b, VT *y) {
    int64_t gt = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int32_t i = (int32_t)(gt / T);
    int lane = (int)(gt % T);
    if (i >= nrows) return;
    VT acc = (VT)0;
    for (int p = rp[i] + lane; p < rp[i + 1]; p += T) acc += v[p] * x[cj[p]];
    acc = team_sum<T>(acc);
    if (lane == 0) {
        if (MODE == MODE_RESID) y[i] = b[i] - acc;
        else if (MODE == MODE_SET) y[i] = acc;
        else y[i] += acc;
    }
}

// one lane per (row, right-hand side), nrhs interleaved
template <class VT, int MODE>
__global__ void __launch_bounds__(256)
k_rowdotM(int32_t nrows, int32_t nrhs, const int32_t *rp, const int32_t *cj,
          const VT *v, const VT *x, const VT *b, VT *y) {
    int64_t gt = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int32_t i = (int32_t)(gt / nrhs);
    int q = (int)(gt % nrhs);
    if (i >= nrows) return;
    VT acc = (VT)0;
    for (int p = rp[i]; p < rp[i + 1]; ++p) acc += v[p] * x[(int64_t)cj[p] * nrhs + q];
    int64_t o = (int64_t)i * nrhs + q;
    if (MODE == MODE_RESID) y[o] = b[o] - acc;
    else if (MODE == MODE_SET) y[o] = acc;
    else y[o] += acc;
}

template <class VT, int MODE>
static void rowdot(const CsrView<VT> &A, const VT *x, const VT *b, VT *y,
                   int32_t nrhs, hipStream_t s) {
    if (A.nrows == 0) return;
    if (nrhs > 1) {
        hipLaunchKernelGGL((k_rowdotM<VT, MODE>),
                           dim3(blocks_for((int64_t)A.nrows * nrhs, 256)), dim3(256),
                           0, s, A.nrows, nrhs, A.rp, A.cj, A.v, x, b, y);
        LAIR_LAUNCH_CHECK();
        return;
    }
#define LAIR_RD(TT)                                                              \
    hipLaunchKernelGGL((k_rowdot1<VT, TT, MODE>),                                \
                       dim3(blocks_for((int64_t)A.nrows * TT, 256)), dim3(256), 0, s, \
                       A.nrows, A.rp, A.cj, A.v, x, b, y)
    switch (A.team) {
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
             bool accumulate, hipStream_t s) {
    if (accumulate) rowdot<VT, MODE_ADD>(A, x, nullptr, y, nrhs, s);
    else rowdot<VT, MODE_SET>(A, x, nullptr, y, nrhs, s);
}

// ---------------------------------------------------------------------------
// Jacobi on a row set X:  t[k] = x_i + omega (b_i - (A x)_i) / a_ii, i = X[k].
// The diagonal is found while streaming the row.
// ---------------------------------------------------------------------------
template <class VT, int T>
__global__ void __launch_bounds__(256)
k_jacobi1(int32_t nx, const int32_t *rows, const int32_t *rp, const int32_t *cj,
          const VT *v, const VT *b, const VT *x, VT *t, VT omega) {
    int64_t gt = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int32_t k = (int32_t)(gt / T);
    int lane = (int)(gt % T);
    if (k >= nx) return;
    int32_t i = rows[k];
    VT acc = (VT)0, d = (VT)0;
    for (int p = rp[i] + lane; p < rp[i + 1]; p += T) {
        int c = cj[p];
        VT a = v[p];
        acc += a * x[c];
        if (c == i) d = a;
    }
    acc = team_sum<T>(acc);
    d = team_sum<T>(d);
    if (lane == 0) t[k] = x[i] + omega * (b[i] - acc) / d;
}

template <class VT>
__global__ void __launch_bounds__(256)
k_jacobiM(int32_t nx, int32_t nrhs, const int32_t *rows, const int32_t *rp,
          const int32_t *cj, const VT *v, const VT *b, const VT *x, VT *t,
          VT omega) {
    int64_t gt = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int32_t k = (int32_t)(gt / nrhs);
    int q = (int)(gt % nrhs);
    if (k >= nx) return;
    int32_t i = rows[k];
    VT acc = (VT)0, d = (VT)0;
    for (int p = rp[i]; p < rp[i + 1]; ++p) {
        int c = cj[p];
        VT a = v[p];
        acc += a * x[(int64_t)c * nrhs + q];
        if (c == i) d = a;
    }
    int64_t oi = (int64_t)i * nrhs + q;
    t[(int64_t)k * nrhs + q] = x[oi] + omega * (b[oi] - acc) / d;
}

template <class VT>
void op_jacobi(const CsrView<VT> &A, const int32_t *rows, int32_t nx,
               const VT *b, const VT *x, VT *t, double omega, int32_t nrhs,
               hipStream_t s) {
    if (nx == 0) return;
    VT om = (VT)omega;
    if (nrhs > 1) {
        hipLaunchKernelGGL((k_jacobiM<VT>), dim3(blocks_for((int64_t)nx * nrhs, 256)),
                           dim3(256), 0, s, nx, nrhs, rows, A.rp, A.cj, A.v, b, x, t, om);
        LAIR_LAUNCH_CHECK();
        return;
    }
#define LAIR_JC(TT)                                                             \
    hipLaunchKernelGGL((k_jacobi1<VT, TT>), dim3(blocks_for((int64_t)nx * TT, 256)), \
                       dim3(256), 0, s, nx, rows, A.rp, A.cj, A.v, b, x, t, om)
    switch (A.team) {
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
__global__ void k_scatter(int64_t total, int32_t nrhs, const int32_t *rows,
                          const VT *t, VT *x) {
    int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= total) return;
    int64_t k = g / nrhs;
    int q = (int)(g % nrhs);
    x[(int64_t)rows[k] * nrhs + q] = t[g];
}

template <class VT>
void op_scatter(const int32_t *rows, int32_t nx, const VT *t, VT *x,
                int32_t nrhs, hipStream_t s) {
    if (nx == 0) return;
    int64_t total = (int64_t)nx * nrhs;
    hipLaunchKernelGGL((k_scatter<VT>), dim3(blocks_for(total, 256)), dim3(256), 0, s,
                       total, nrhs, rows, t, x);
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
    hipLaunchKernelGGL((k_fill<VT>), dim3(blocks_for(n, 256)), dim3(256), 0, s, x, val, n);
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
    hipLaunchKernelGGL((k_copy<VT>), dim3(blocks_for(n, 256)), dim3(256), 0, s, x, y, n);
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
    hipLaunchKernelGGL((k_dense_solve<VT>), dim3(1), dim3(256), 0, s, n, lu, piv, b, x,
                       nrhs, transpose ? 1 : 0);
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

__global__ void k_sumsq_final(const double *partial, int32_t nblk, int32_t nrhs,
                              double *out) {
    int q = threadIdx.x;
    if (q >= nrhs) return;
    double acc = 0.0;
    for (int b = 0; b < nblk; ++b) acc += partial[(int64_t)b * nrhs + q];
    out[q] = acc;
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
    hipLaunchKernelGGL(k_sumsq_partial, dim3(nblk), dim3(NRM_BS), 0, s, r, total,
                       nrhs, chunk, partial);
    LAIR_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_sumsq_final, dim3(1), dim3(64), 0, s, partial, nblk, nrhs, out);
    LAIR_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// Mixed precision helpers and block scaling of right-hand sides.
// ---------------------------------------------------------------------------
__global__ void k_axpy_f32(double *x, const float *e, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] += (double)e[i];
}

void op_axpy_f32(double *x, const float *e, int64_t n, hipStream_t s) {
    if (n == 0) return;
    hipLaunchKernelGGL(k_axpy_f32, dim3(blocks_for(n, 256)), dim3(256), 0, s, x, e, n);
    LAIR_LAUNCH_CHECK();
}

__global__ void k_cast_f32(const double *in, float *out, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = (float)in[i];
}

void op_cast_f32(const double *in, float *out, int64_t n, hipStream_t s) {
    if (n == 0) return;
    hipLaunchKernelGGL(k_cast_f32, dim3(blocks_for(n, 256)), dim3(256), 0, s, in, out, n);
    LAIR_LAUNCH_CHECK();
}

__global__ void k_cast_f64(const float *in, double *out, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = (double)in[i];
}

void op_cast_f64(const float *in, double *out, int64_t n, hipStream_t s) {
    if (n == 0) return;
    hipLaunchKernelGGL(k_cast_f64, dim3(blocks_for(n, 256)), dim3(256), 0, s, in, out, n);
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
    hipLaunchKernelGGL(k_block_apply, dim3(blocks_for(tot, 256)), dim3(256), 0, s,
                       nblk, k, dinv, b, out, nrhs);
    LAIR_LAUNCH_CHECK();
}

// explicit instantiations
template void op_residual<double>(const CsrView<double> &, const double *, const double *, double *, int32_t, hipStream_t);
template void op_residual<float>(const CsrView<float> &, const float *, const float *, float *, int32_t, hipStream_t);
template void op_spmv<double>(const CsrView<double> &, const double *, double *, int32_t, bool, hipStream_t);
template void op_spmv<float>(const CsrView<float> &, const float *, float *, int32_t, bool, hipStream_t);
template void op_jacobi<double>(const CsrView<double> &, const int32_t *, int32_t, const double *, const double *, double *, double, int32_t, hipStream_t);
template void op_jacobi<float>(const CsrView<float> &, const int32_t *, int32_t, const float *, const float *, float *, double, int32_t, hipStream_t);
template void op_scatter<double>(const int32_t *, int32_t, const double *, double *, int32_t, hipStream_t);
template void op_scatter<float>(const int32_t *, int32_t, const float *, float *, int32_t, hipStream_t);
template void op_fill<double>(double *, double, int64_t, hipStream_t);
template void op_fill<float>(float *, float, int64_t, hipStream_t);
template void op_copy<double>(const double *, double *, int64_t, hipStream_t);
template void op_copy<float>(const float *, float *, int64_t, hipStream_t);
template void op_dense_solve<double>(int32_t, const double *, const int32_t *, const double *, double *, int32_t, bool, hipStream_t);
template void op_dense_solve<float>(int32_t, const double *, const int32_t *, const float *, float *, int32_t, bool, hipStream_t);

}  // namespace lair
