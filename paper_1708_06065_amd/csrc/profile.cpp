// Kernel profiler behind lair_profile_begin / lair_profile_end.
//
// A ProfScope of a selected category makes every kernel launched inside it
// (on the scope's stream, through LAIR_LAUNCH) carry a start and a stop HIP
// event of its own dispatch (hipExtLaunchKernelGGL), so the time is that of
// the kernels as the stream executes them, without the dispatch latency
// that events recorded between launches would add.  Records carry the
// algorithmic bytes and flops of the operation (the data it must touch at
// least once), from which the caller derives achieved bandwidth.
// Process-wide; not for concurrent use from several host threads.
#include <hip/hip_runtime.h>

#include <cstring>
#include <functional>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "lair_internal.hpp"

namespace lair {

namespace {
struct Rec {
    std::string cat;
    double bytes, flops;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> kev;   // one pair per kernel
};
struct Prof {
    bool on = false;
    std::string filter;            // empty: every category
    std::vector<Rec> recs;
    std::vector<hipEvent_t> pool;
    std::mutex mu;
};
Prof &prof() {
    static Prof p;
    return p;
}
thread_local int t_slot = -1;                 // record of the innermost scope
thread_local hipStream_t t_stream = nullptr;
hipEvent_t take_event(Prof &p) {
    if (!p.pool.empty()) {
        hipEvent_t e = p.pool.back();
        p.pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}
bool selected(const Prof &p, const char *cat) {
    if (p.filter.empty()) return true;
    // comma-separated list of category names
    size_t pos = 0;
    while (pos <= p.filter.size()) {
        size_t c = p.filter.find(',', pos);
        std::string tok = p.filter.substr(pos, c == std::string::npos ? std::string::npos : c - pos);
        if (tok == cat) return true;
        if (c == std::string::npos) break;
        pos = c + 1;
    }
    return false;
}
}  // namespace

bool prof_selected(const char *category) {
    Prof &p = prof();
    if (!p.on) return false;
    std::lock_guard<std::mutex> g(p.mu);
    return selected(p, category);
}

ProfScope::ProfScope(const char *category, hipStream_t s, double bytes, double flops) {
    Prof &p = prof();
    if (!p.on) return;
    std::lock_guard<std::mutex> g(p.mu);
    if (!selected(p, category)) return;
    prev_slot = t_slot;
    prev_stream = t_stream;
    slot = (int)p.recs.size();
    stream = s;
    p.recs.push_back(Rec{category, bytes, flops, {}});
    t_slot = slot;
    t_stream = s;
}

void prof_set_bytes(int slot, double bytes) {
    if (slot < 0) return;
    Prof &p = prof();
    std::lock_guard<std::mutex> g(p.mu);
    if (!p.on || slot >= (int)p.recs.size()) return;
    p.recs[slot].bytes = bytes;
}

ProfScope::~ProfScope() {
    if (slot < 0) return;
    t_slot = prev_slot;
    t_stream = prev_stream;
}

bool prof_kernel_events(hipStream_t s, hipEvent_t *e0, hipEvent_t *e1) {
    if (t_slot < 0 || s != t_stream) return false;
    Prof &p = prof();
    std::lock_guard<std::mutex> g(p.mu);
    if (!p.on || t_slot >= (int)p.recs.size()) return false;
    hipEvent_t a = take_event(p), b = take_event(p);
    if (!a || !b) return false;
    p.recs[t_slot].kev.push_back({a, b});
    *e0 = a;
    *e1 = b;
    return true;
}

namespace {
struct PinnedBuf {
    void *p = nullptr;
    size_t n = 0;
    ~PinnedBuf() {
        if (p) (void)hipHostFree(p);
    }
};
}  // namespace

static void *pinned_grow(PinnedBuf &buf, size_t bytes);

void *pinned_staging(size_t bytes) {
    static thread_local PinnedBuf buf;
    return pinned_grow(buf, bytes);
}

void *pinned_upload(size_t bytes) {
    static thread_local PinnedBuf buf;
    return pinned_grow(buf, bytes);
}

static void *pinned_grow(PinnedBuf &buf, size_t bytes) {
    if (bytes > buf.n) {
        if (buf.p) (void)hipHostFree(buf.p);
        buf.p = nullptr;
        buf.n = 0;
        size_t want = bytes < 65536 ? 65536 : bytes;
        if (hipHostMalloc(&buf.p, want, hipHostMallocDefault) != hipSuccess) {
            buf.p = nullptr;
            fail(LAIR_ENOMEM, "pinned host allocation of %zu bytes failed", want);
        }
        buf.n = want;
    }
    return buf.p;
}

void Readback::add(void *d, const void *sp, size_t bytes) {
    size_t off = (used + 15) & ~(size_t)15;
    dst.push_back({d, off});
    src.push_back({sp, bytes});
    used = off + bytes;
}

// Small readbacks: one kernel gathers every source into coherent pinned
// host memory (vector stores, then a system-scope fence), instead of one
// copy per source.
namespace {
constexpr int GATHER_MAX = 8;
constexpr size_t GATHER_BYTES = 16384;
struct GatherArgs {
    const uint32_t *src[GATHER_MAX];
    uint32_t off[GATHER_MAX];     // in 4-byte words
    uint32_t len[GATHER_MAX];     // in 4-byte words
    int32_t n;
};

__global__ void __launch_bounds__(256) k_gather_host(GatherArgs a, uint32_t *dst) {
    for (int k = 0; k < a.n; ++k)
        for (uint32_t w = threadIdx.x; w < a.len[k]; w += blockDim.x)
            dst[a.off[k] + w] = a.src[k][w];
    __threadfence_system();
}

struct CoherentBuf {
    void *p = nullptr;
    ~CoherentBuf() {
        if (p) (void)hipHostFree(p);
    }
};

void *gather_buffer() {
    static thread_local CoherentBuf buf;
    if (!buf.p) {
        if (hipHostMalloc(&buf.p, GATHER_BYTES, hipHostMallocCoherent) != hipSuccess) {
            buf.p = nullptr;
            (void)hipGetLastError();
            fail(LAIR_ENOMEM, "pinned host allocation of %zu bytes failed", GATHER_BYTES);
        }
    }
    return buf.p;
}
}  // namespace

namespace {
thread_local const std::function<void()> *t_fill = nullptr;
hipEvent_t readback_event() {
    thread_local hipEvent_t e = nullptr;
    if (!e) LAIR_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    return e;
}
// Wait for everything queued on s so far.  With a fill hook installed, the
// hook first queues independent work behind the readback, which the device
// runs while this thread waits for the readback alone (an event recorded
// before the hook's work).
void wait_readback(hipStream_t s) {
    if (t_fill && *t_fill) {
        hipEvent_t e = readback_event();
        LAIR_HIP(hipEventRecord(e, s));
        const std::function<void()> *f = t_fill;
        t_fill = nullptr;                    // no hook inside the hook
        try {
            (*f)();
        } catch (...) {
            t_fill = f;
            throw;
        }
        t_fill = f;
        LAIR_HIP(hipEventSynchronize(e));
        return;
    }
    LAIR_HIP(hipStreamSynchronize(s));
}
}  // namespace

const std::function<void()> *set_readback_fill(const std::function<void()> *fill) {
    const std::function<void()> *prev = t_fill;
    t_fill = fill;
    return prev;
}

bool prof_active() { return prof().on; }

void Readback::run() {
    bool small = src.size() <= (size_t)GATHER_MAX && used <= GATHER_BYTES;
    for (size_t k = 0; k < src.size() && small; ++k)
        small = (src[k].second % 4 == 0) && ((uintptr_t)src[k].first % 4 == 0);
    if (small && !src.empty()) {
        GatherArgs a{};
        a.n = (int32_t)src.size();
        for (size_t k = 0; k < src.size(); ++k) {
            a.src[k] = (const uint32_t *)src[k].first;
            a.off[k] = (uint32_t)(dst[k].second / 4);
            a.len[k] = (uint32_t)(src[k].second / 4);
        }
        char *stage = (char *)gather_buffer();
        // (not a profiled operation: launched without the profiler's events)
        hipLaunchKernelGGL(k_gather_host, dim3(1), dim3(256), 0, stream, a, (uint32_t *)stage);
        LAIR_LAUNCH_CHECK();
        wait_readback(stream);
        for (size_t k = 0; k < src.size(); ++k)
            memcpy(dst[k].first, stage + dst[k].second, src[k].second);
        dst.clear();
        src.clear();
        used = 0;
        return;
    }
    char *stage = (char *)pinned_staging(used);
    for (size_t k = 0; k < src.size(); ++k)
        LAIR_HIP(hipMemcpyAsync(stage + dst[k].second, src[k].first, src[k].second,
                                hipMemcpyDeviceToHost, stream));
    wait_readback(stream);
    for (size_t k = 0; k < src.size(); ++k)
        memcpy(dst[k].first, stage + dst[k].second, src[k].second);
    dst.clear();
    src.clear();
    used = 0;
}

}  // namespace lair

using namespace lair;

extern "C" {

lair_status lair_profile_begin(const char *categories) {
    Prof &p = prof();
    std::lock_guard<std::mutex> g(p.mu);
    for (auto &r : p.recs)
        for (auto &e : r.kev) {
            p.pool.push_back(e.first);
            p.pool.push_back(e.second);
        }
    p.recs.clear();
    p.filter = categories ? categories : "";
    p.on = true;
    return LAIR_OK;
}

lair_status lair_profile_end(char *json, int64_t *len) {
    Prof &p = prof();
    std::lock_guard<std::mutex> g(p.mu);
    p.on = false;
    struct Agg { long n = 0; double ms = 0, bytes = 0, flops = 0, ms_max = 0; };
    std::map<std::string, Agg> agg;
    lair_status st = LAIR_OK;
    for (auto &r : p.recs) {
        if (r.kev.empty()) continue;          // no kernel ran in the scope
        double ms = 0.0;
        bool ok = true;
        for (auto &e : r.kev) {
            float k = 0.f;
            if (hipEventSynchronize(e.second) != hipSuccess ||
                hipEventElapsedTime(&k, e.first, e.second) != hipSuccess) {
                ok = false;
                break;
            }
            ms += k;
        }
        if (!ok) {
            st = LAIR_EDEVICE;
            continue;
        }
        Agg &a = agg[r.cat];
        a.n += (long)r.kev.size();
        a.ms += ms;
        a.bytes += r.bytes;
        a.flops += r.flops;
        if (ms > a.ms_max) a.ms_max = ms;
    }
    std::string out = "{";
    bool first = true;
    for (auto &kv : agg) {
        char buf[512];
        snprintf(buf, sizeof(buf),
                 "%s\"%s\": {\"launches\": %ld, \"ms\": %.6f, \"ms_max\": %.6f, "
                 "\"alg_bytes\": %.1f, \"alg_flops\": %.1f}",
                 first ? "" : ", ", kv.first.c_str(), kv.second.n, kv.second.ms,
                 kv.second.ms_max, kv.second.bytes, kv.second.flops);
        out += buf;
        first = false;
    }
    out += "}";
    if (len) {
        int64_t cap = *len;
        *len = (int64_t)out.size() + 1;
        if (json && cap >= (int64_t)out.size() + 1) memcpy(json, out.c_str(), out.size() + 1);
        else if (json) st = LAIR_EINVAL;
    }
    return st;
}

}  // extern "C"
