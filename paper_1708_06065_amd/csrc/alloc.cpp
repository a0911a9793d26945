// Device memory for the library: a caching allocator.
//
// The setup allocates and releases many large temporaries (staging rows of
// the sparse products, per-level work arrays) on every call; returning them
// to the runtime and mapping them again costs far more than the kernels
// that use them.  Released blocks are kept per device and per stream and
// handed out again to requests on the same stream, where stream order makes
// the reuse safe.  lair_trim returns the cached blocks to the runtime.
//
// Failure testing: when the environment variable LAIR_DEBUG_MAX_BYTES holds a
// positive number, a request that would raise the bytes in use by the
// library above it fails with LAIR_ENOMEM, as a real shortage would.
#include <hip/hip_runtime.h>

#include <cstdlib>
#include <map>
#include <mutex>
#include <unordered_map>

#include "lair_internal.hpp"

namespace lair {
namespace {

struct Block {
    size_t size;
    int device;
    hipStream_t stream;
};

struct Cache {
    std::mutex mu;
    std::unordered_map<void *, Block> live;
    std::multimap<size_t, std::pair<void *, Block>> idle;   // by size
    size_t cached = 0;
    size_t in_use = 0;       // bytes of the live blocks
};

Cache &cache() {
    static Cache *c = new Cache();   // outlives static destructors of callers
    return *c;
}

size_t round_size(size_t b) {
    if (b <= 512) return 512;
    if (b <= (1u << 20)) {
        size_t r = 512;
        while (r < b) r <<= 1;
        return r;
    }
    const size_t q = (size_t)2 << 20;   // 2 MiB granules above 1 MiB
    return (b + q - 1) / q * q;
}

void release_idle(Cache &c, int device) {
    for (auto it = c.idle.begin(); it != c.idle.end();) {
        if (device < 0 || it->second.second.device == device) {
            (void)hipFree(it->second.first);
            c.cached -= it->second.second.size;
            it = c.idle.erase(it);
        } else {
            ++it;
        }
    }
}

// LAIR_DEBUG_MAX_BYTES, read at every request (0: no cap)
size_t debug_cap() {
    const char *e = std::getenv("LAIR_DEBUG_MAX_BYTES");
    if (!e || !*e) return 0;
    char *end = nullptr;
    unsigned long long v = std::strtoull(e, &end, 10);
    return (end && *end == 0) ? (size_t)v : 0;
}

}  // namespace

void *dev_alloc(size_t bytes, hipStream_t s) {
    if (bytes == 0) return nullptr;
    int dev = 0;
    LAIR_HIP(hipGetDevice(&dev));
    const size_t want = round_size(bytes);
    Cache &c = cache();
    std::lock_guard<std::mutex> g(c.mu);
    const size_t cap = debug_cap();
    if (cap && c.in_use + want > cap)
        fail(LAIR_ENOMEM, "device allocation of %zu bytes refused: %zu bytes in use, "
             "LAIR_DEBUG_MAX_BYTES = %zu", bytes, c.in_use, cap);
    // smallest idle block of this device and stream that fits without
    // wasting more than half of it
    for (auto it = c.idle.lower_bound(want); it != c.idle.end() && it->first <= 2 * want; ++it) {
        const Block &b = it->second.second;
        if (b.device == dev && b.stream == s) {
            void *p = it->second.first;
            c.live[p] = b;
            c.cached -= b.size;
            c.in_use += b.size;
            c.idle.erase(it);
            return p;
        }
    }
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, want);
    if (e == hipErrorOutOfMemory) {
        (void)hipGetLastError();
        release_idle(c, dev);
        e = hipMalloc(&p, want);
    }
    if (e != hipSuccess) {
        (void)hipGetLastError();
        fail(e == hipErrorOutOfMemory ? LAIR_ENOMEM : LAIR_EDEVICE,
             "device allocation of %zu bytes failed: %s", bytes, hipGetErrorString(e));
    }
    c.live[p] = Block{want, dev, s};
    c.in_use += want;
    return p;
}

void dev_free(void *p, hipStream_t s) noexcept {
    if (!p) return;
    Cache &c = cache();
    std::lock_guard<std::mutex> g(c.mu);
    auto it = c.live.find(p);
    if (it == c.live.end()) return;
    Block b = it->second;
    b.stream = s;
    c.live.erase(it);
    c.in_use -= b.size;
    c.idle.emplace(b.size, std::make_pair(p, b));
    c.cached += b.size;
}

void dev_trim() noexcept {
    Cache &c = cache();
    std::lock_guard<std::mutex> g(c.mu);
    (void)hipDeviceSynchronize();
    release_idle(c, -1);
}

size_t dev_cached_bytes() noexcept {
    Cache &c = cache();
    std::lock_guard<std::mutex> g(c.mu);
    return c.cached;
}

size_t dev_in_use_bytes() noexcept {
    Cache &c = cache();
    std::lock_guard<std::mutex> g(c.mu);
    return c.in_use;
}

// ---------------------------------------------------------------------------
// Zeroed counter slots.  Flags, sizes and queue counters of the setup must
// start at zero; instead of a memset for each, they are handed out from a
// block per device and stream that one memset clears, each slot once.
// zeroed_slots_reserve (at the start of a setup) clears the block again when
// fewer slots than asked remain: every slot handed out before belongs to an
// earlier call whose work and readbacks are complete in stream order.  A
// block that runs out within a call is replaced by a fresh one.  The blocks
// are held until the process ends and are not counted as memory in use.
// ---------------------------------------------------------------------------
namespace {
constexpr size_t ZBLOCK = (size_t)1 << 16;   // slots (int64) per block

struct ZArena {
    int64_t *block = nullptr;
    size_t next = ZBLOCK;
};

std::mutex g_zmu;
std::map<std::pair<int, hipStream_t>, ZArena> g_zarena;

ZArena &zarena(hipStream_t s) {
    int dev = 0;
    LAIR_HIP(hipGetDevice(&dev));
    return g_zarena[{dev, s}];
}

void zfresh(ZArena &a, hipStream_t s) {
    if (!a.block) {
        void *p = nullptr;
        if (hipMalloc(&p, ZBLOCK * sizeof(int64_t)) != hipSuccess) {
            (void)hipGetLastError();
            fail(LAIR_ENOMEM, "device allocation of the counter slots failed");
        }
        a.block = (int64_t *)p;
    }
    LAIR_HIP(hipMemsetAsync(a.block, 0, ZBLOCK * sizeof(int64_t), s));
    a.next = 0;
}
}  // namespace

void zeroed_slots_reserve(size_t count, hipStream_t s) {
    std::lock_guard<std::mutex> g(g_zmu);
    ZArena &a = zarena(s);
    if (!a.block || ZBLOCK - a.next < count) zfresh(a, s);
}

int64_t *zeroed_slots(size_t count, hipStream_t s) {
    if (count > ZBLOCK) fail(LAIR_EUNSUPPORTED, "too many counter slots (%zu)", count);
    std::lock_guard<std::mutex> g(g_zmu);
    ZArena &a = zarena(s);
    if (!a.block || ZBLOCK - a.next < count) {
        // mid-call: a new block, so that slots still to be read stay intact
        a.block = nullptr;
        zfresh(a, s);
    }
    int64_t *p = a.block + a.next;
    a.next += count;
    return p;
}

}  // namespace lair
