// Parallel CF splitting of the PMIS type (De Sterck, Yang and Heys, 2006):
// the device alternative to the sequential Ruge-Stueben first pass of
// Sec. 4.  Weight of point i: the number of points that strongly depend on
// it, then fmix32(i) (MurmurHash3's 32-bit finalizer), then i.  Points on
// which nothing strongly depends are F.  A round: every undecided point that
// beats every undecided point it is strongly connected to (either
// direction) becomes C, then every undecided point that strongly depends on
// a C-point becomes F.  Every kernel only ever moves a point's state one
// way (undecided to "not a candidate", undecided to C or F), so the rounds'
// results do not depend on the order of the threads.
#include <hip/hip_runtime.h>

#include "k_common.hpp"
#include "lair_internal.hpp"

namespace lair {

constexpr int SPLIT_BS = 256;
constexpr int8_t ST_U = -1, ST_F = 0, ST_C = 1;

__device__ __forceinline__ uint32_t fmix32(uint32_t h) {
    h ^= h >> 16;
    h *= 0x85EBCA6Bu;
    h ^= h >> 13;
    h *= 0xC2B2AE35u;
    h ^= h >> 16;
    return h;
}

// cnt[i] += 1 for every strong entry (j, i), j != i
__global__ void __launch_bounds__(SPLIT_BS)
k_pmis_count(int32_t n, const int32_t *rp, const int32_t *cj, const uint8_t *smask,
             int32_t *cnt) {
    const int32_t j = blockIdx.x * SPLIT_BS + threadIdx.x;
    if (j >= n) return;
    for (int32_t p = rp[j]; p < rp[j + 1]; ++p)
        if (smask[p] && cj[p] != j) atomicAdd(&cnt[cj[p]], 1);
}

// weights and the first states; every undecided point starts a candidate
__global__ void __launch_bounds__(SPLIT_BS)
k_pmis_init(int32_t n, const int32_t *cnt, uint64_t *key, int8_t *state, uint8_t *cand) {
    const int32_t i = blockIdx.x * SPLIT_BS + threadIdx.x;
    if (i >= n) return;
    key[i] = ((uint64_t)(uint32_t)cnt[i] << 32) | fmix32((uint32_t)i);
    state[i] = cnt[i] == 0 ? ST_F : ST_U;
    cand[i] = cnt[i] == 0 ? 0 : 1;
}

__device__ __forceinline__ bool pmis_beats(const uint64_t *key, int32_t a, int32_t b) {
    return key[a] > key[b] || (key[a] == key[b] && a > b);
}

// cand[i] is 1 for the undecided points at the start of a round; the loser
// of every strong pair of undecided points is cleared (stores of 0 only)
__global__ void __launch_bounds__(SPLIT_BS)
k_pmis_compete(int32_t n, const int32_t *rp, const int32_t *cj, const uint8_t *smask,
               const uint64_t *key, const int8_t *state, uint8_t *cand) {
    const int32_t j = blockIdx.x * SPLIT_BS + threadIdx.x;
    if (j >= n || state[j] != ST_U) return;
    for (int32_t p = rp[j]; p < rp[j + 1]; ++p) {
        const int32_t i = cj[p];
        if (!smask[p] || i == j || state[i] != ST_U) continue;
        if (pmis_beats(key, i, j)) cand[j] = 0;
        else cand[i] = 0;
    }
}

__global__ void __launch_bounds__(SPLIT_BS)
k_pmis_select(int32_t n, const uint8_t *cand, int8_t *state) {
    const int32_t i = blockIdx.x * SPLIT_BS + threadIdx.x;
    if (i >= n) return;
    if (cand[i]) state[i] = ST_C;
}

// undecided points that strongly depend on a C-point become F; the points
// still undecided are the next round's candidates (a thread writes only its
// own point's state and candidate flag) and are counted, one atomic per
// wavefront (every lane reaches the ballot: no early return)
__global__ void __launch_bounds__(SPLIT_BS)
k_pmis_fpass(int32_t n, const int32_t *rp, const int32_t *cj, const uint8_t *smask,
             int8_t *state, uint8_t *cand, int32_t *left) {
    const int32_t j = blockIdx.x * SPLIT_BS + threadIdx.x;
    bool und = false;
    if (j < n) {
        if (state[j] == ST_U) {
            bool to_f = false;
            for (int32_t p = rp[j]; p < rp[j + 1] && !to_f; ++p) {
                const int32_t i = cj[p];
                to_f = smask[p] && i != j && state[i] == ST_C;
            }
            if (to_f) state[j] = ST_F;
            und = !to_f;
        }
        cand[j] = und ? 1 : 0;
    }
    const unsigned long long m = __ballot(und);
    if ((threadIdx.x & 63) == 0 && m != 0ull) atomicAdd(left, (int32_t)__popcll(m));
}

void launch_pmis_split(int32_t n, const int32_t *rp, const int32_t *cj, const uint8_t *smask,
                       int8_t *cf, hipStream_t s) {
    if (n == 0) return;
    const dim3 grid(blocks_for(n, SPLIT_BS)), blk(SPLIT_BS);
    DevArr<int32_t> cnt, left;
    DevArr<uint64_t> key;
    DevArr<uint8_t> cand;
    cnt.alloc((size_t)n, s);
    key.alloc((size_t)n, s);
    cand.alloc((size_t)n, s);
    // one counter per round of a batch of rounds
    constexpr int ROUNDS = 8;
    left.alloc(ROUNDS, s);
    LAIR_HIP(hipMemsetAsync(cnt.get(), 0, sizeof(int32_t) * n, s));
    LAIR_LAUNCH(k_pmis_count, grid, blk, 0, s, n, rp, cj, smask, cnt.get());
    LAIR_LAUNCH_CHECK();
    LAIR_LAUNCH(k_pmis_init, grid, blk, 0, s, n, cnt.get(), key.get(), cf, cand.get());
    LAIR_LAUNCH_CHECK();
    // every round turns at least the undecided point of largest weight into
    // a C-point, so n rounds always suffice; rounds are launched in batches
    // and the count of undecided points read after each batch
    for (int64_t done = 0; done < n; done += ROUNDS) {
        LAIR_HIP(hipMemsetAsync(left.get(), 0, sizeof(int32_t) * ROUNDS, s));
        for (int r = 0; r < ROUNDS; ++r) {
            LAIR_LAUNCH(k_pmis_compete, grid, blk, 0, s, n, rp, cj, smask, key.get(), cf,
                        cand.get());
            LAIR_LAUNCH_CHECK();
            LAIR_LAUNCH(k_pmis_select, grid, blk, 0, s, n, cand.get(), cf);
            LAIR_LAUNCH_CHECK();
            LAIR_LAUNCH(k_pmis_fpass, grid, blk, 0, s, n, rp, cj, smask, cf, cand.get(),
                        left.get() + r);
            LAIR_LAUNCH_CHECK();
        }
        int32_t hl[ROUNDS];
        Readback rb(s);
        rb.add(hl, left.get(), sizeof(hl));
        rb.run();
        if (hl[ROUNDS - 1] == 0) return;
    }
    fail(LAIR_EDEVICE, "parallel splitting did not finish");
}

}  // namespace lair
