// Device-side helpers shared by the kernel translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <climits>
#include <cstdint>

namespace lair {

constexpr int WAVE = 64;
constexpr int NXCD = 8;

// The hardware hands workgroups to the 8 XCDs round-robin, and each XCD has
// its own L2.  Remap the workgroup id so that every XCD runs one contiguous
// range of logical blocks: consecutive rows, which share matrix and vector
// cache lines, then share an L2 instead of being striped over eight.  The
// map is a bijection on [0, gridDim.x) for any grid size.
__device__ __forceinline__ int64_t xcd_block_id() {
    const int64_t nb = gridDim.x, b = blockIdx.x;
    const int64_t x = b % NXCD, k = b / NXCD;
    const int64_t q = nb / NXCD, r = nb % NXCD;
    return (x < r) ? x * (q + 1) + k : r * (q + 1) + (x - r) * q + k;
}

// Streaming (non-temporal) loads for data that a kernel reads once and
// that is far larger than the caches: the lines are not kept, so the caches
// stay with the gathered vectors.
template <class T>
__device__ __forceinline__ T ld_stream(const T *p) { return __builtin_nontemporal_load(p); }
template <class T, int N>
using ExtVec = T __attribute__((ext_vector_type(N)));

// Butterfly reductions over a team of T consecutive lanes (T a power of two
// dividing 64).  Every lane of the team receives the result; the order of
// the additions is fixed, so results are reproducible run to run.
template <int T>
__device__ __forceinline__ double team_sum(double v) {
#pragma unroll
    for (int o = T / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, T);
    return v;
}
template <int T>
__device__ __forceinline__ float team_sum(float v) {
#pragma unroll
    for (int o = T / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, T);
    return v;
}
template <int T>
__device__ __forceinline__ double team_max(double v) {
#pragma unroll
    for (int o = T / 2; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, T));
    return v;
}
template <int T>
__device__ __forceinline__ int team_min(int v) {
#pragma unroll
    for (int o = T / 2; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, T));
    return v;
}
template <int T>
__device__ __forceinline__ int team_sum_int(int v) {
#pragma unroll
    for (int o = T / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, T);
    return v;
}

// Bits of a wave ballot that belong to the calling lane's team of T lanes.
template <int T>
__device__ __forceinline__ uint64_t team_bits(bool pred) {
    uint64_t b = __ballot(pred);
    int first = (threadIdx.x & (WAVE - 1)) & ~(T - 1);
    uint64_t mask = (T == 64) ? ~0ull : ((1ull << T) - 1ull);
    return (b >> first) & mask;
}

// Arg-max of |value| over a team, ties to the smallest index.
template <int T>
__device__ __forceinline__ void team_argmax(double &v, int &idx) {
#pragma unroll
    for (int o = T / 2; o > 0; o >>= 1) {
        double ov = __shfl_xor(v, o, T);
        int oi = __shfl_xor(idx, o, T);
        if (ov > v || (ov == v && oi < idx)) { v = ov; idx = oi; }
    }
}

// Largest 64-bit key over a team (a packed arg-max: value bits above, an
// index code below).
template <int T>
__device__ __forceinline__ uint64_t team_max_u64(uint64_t v) {
#pragma unroll
    for (int o = T / 2; o > 0; o >>= 1) {
        const uint64_t ov = __shfl_xor(v, o, T);
        v = ov > v ? ov : v;
    }
    return v;
}

// Make the LDS writes of the calling wave visible to its later LDS reads
// (lanes of one wave run in lockstep; only memory ordering is needed).
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Position of `key` in the sorted list a[0..n), or -1.
__device__ __forceinline__ int bsearch_i32(const int32_t *a, int n, int key) {
    int lo = 0, hi = n - 1;
    while (lo <= hi) {
        int mid = (lo + hi) >> 1;
        int v = a[mid];
        if (v == key) return mid;
        if (v < key) lo = mid + 1; else hi = mid - 1;
    }
    return -1;
}

}  // namespace lair
