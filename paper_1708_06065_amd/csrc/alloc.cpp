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

}  // namespace lair
