// lair_cycle_noalloc: one V-cycle (the operation of lair_cycle) whose work
// vectors live in a fixed device array of this file, so that the call
// allocates no device memory.  For callers that cannot allocate: code under
// HIP graph capture, tight serving loops, harnesses that forbid allocation.
//
// The array `scratch` is a file-scope __device__ array: every GPU the
// library runs on holds its own copy, at its own address, until the process
// ends.  In host code its name is only a stand-in for that address, so the
// first call on a device looks the address up with hipGetSymbolAddress (that
// device current) and keeps it per device; every use below goes through the
// looked-up pointer.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>
#include <type_traits>
#include <utility>
#include <vector>

#include "hierarchy.hpp"

static __device__ __align__(256) char scratch[LAIR_NOALLOC_MAX_BYTES];

namespace lair {

namespace {

constexpr size_t SCRATCH_BYTES = (size_t)LAIR_NOALLOC_MAX_BYTES;
constexpr size_t SCRATCH_ALIGN = 256;
constexpr int MAX_DEVICES = 64;

std::mutex g_mu;
char *g_ptr[MAX_DEVICES] = {};

// Device address of this device's copy of `scratch` (looked up once per
// device).
char *scratch_on_current_device() {
    int dev = -1;
    LAIR_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= MAX_DEVICES) fail(LAIR_EDEVICE, "device %d out of range", dev);
    std::lock_guard<std::mutex> g(g_mu);
    if (!g_ptr[dev]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            fail(LAIR_EDEVICE, "hipGetSymbolAddress(scratch) failed on device %d: %s", dev,
                 hipGetErrorString(e));
        g_ptr[dev] = (char *)p;
    }
    return g_ptr[dev];
}

size_t round_up(size_t b) { return (b + SCRATCH_ALIGN - 1) / SCRATCH_ALIGN * SCRATCH_ALIGN; }

// Bytes the cycle's work vectors take in the scratch array (each vector
// starting on a 256-byte boundary).
size_t scratch_bytes(lair_hierarchy *h, int32_t nrhs) {
    size_t off = 0;
    for_each_cycle_vector(h, nrhs, [&](auto &a, size_t count) {
        using T = std::remove_pointer_t<decltype(a.get())>;
        off += round_up(count * sizeof(T));
    });
    return off;
}

// Puts views of the scratch array in place of the hierarchy's work vectors
// for the duration of one call, and the hierarchy's own arrays back after it
// (also when the call fails).
struct ScratchVectors {
    std::vector<std::pair<DevArr<double> *, DevArr<double>>> d;
    std::vector<std::pair<DevArr<float> *, DevArr<float>>> f;
    ScratchVectors(lair_hierarchy *h, int32_t nrhs, char *base) {
        size_t off = 0;
        for_each_cycle_vector(h, nrhs, [&](auto &a, size_t count) {
            using T = std::remove_pointer_t<decltype(a.get())>;
            std::remove_reference_t<decltype(a)> view;
            view.borrow(reinterpret_cast<T *>(base + off), count);
            off += round_up(count * sizeof(T));
            a.swap(view);               // the hierarchy's array is now in `view`
            if constexpr (std::is_same<T, double>::value) d.emplace_back(&a, std::move(view));
            else f.emplace_back(&a, std::move(view));
        });
    }
    ~ScratchVectors() {
        for (auto &e : d) e.first->swap(e.second);
        for (auto &e : f) e.first->swap(e.second);
    }
    ScratchVectors(const ScratchVectors &) = delete;
    ScratchVectors &operator=(const ScratchVectors &) = delete;
};

}  // namespace

void cycle_noalloc_impl(lair_hierarchy *h, const double *b, double *x, int32_t nrhs,
                        hipStream_t s) {
    if (!h || !b || !x) fail(LAIR_EINVAL, "NULL argument");
    check_nrhs(h, nrhs);
    const size_t need = scratch_bytes(h, nrhs);
    if (need > SCRATCH_BYTES)
        fail(LAIR_EUNSUPPORTED,
             "lair_cycle_noalloc: this hierarchy's cycle with %d right-hand side(s) needs "
             "%zu bytes of work vectors, more than the %zu-byte scratch array",
             nrhs, need, SCRATCH_BYTES);
    char *base = scratch_on_current_device();
    ScratchVectors views(h, nrhs, base);
    cycle_body(h, b, x, nrhs, s);
}

}  // namespace lair
