// liblair C ABI (include/lair.h): error handling across the boundary, the
// entry points, statistics and exports.  The setup lives in setup.cpp, the
// cycles and solves in solve.cpp.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <chrono>
#include <climits>
#include <cmath>
#include <cstdarg>
#include <cstring>
#include <memory>
#include <new>
#include <string>
#include <type_traits>
#include <vector>

#include "hierarchy.hpp"

namespace lair {

static thread_local std::string g_last_error;

void set_last_error(const std::string &m) { g_last_error = m; }

void fail(lair_status st, const char *fmt, ...) {
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    throw Error{st, std::string(buf)};
}

}  // namespace lair


// ===========================================================================
// C ABI
// ===========================================================================
using namespace lair;

template <class F>
static lair_status guarded(F &&f) {
    try {
        return f();
    } catch (const Error &e) {
        set_last_error(e.msg);
        return e.status;
    } catch (const std::bad_alloc &) {
        set_last_error("host allocation failed");
        return LAIR_ENOMEM;
    } catch (const std::exception &e) {
        set_last_error(e.what());
        return LAIR_EDEVICE;
    } catch (...) {
        set_last_error("unknown error");
        return LAIR_EDEVICE;
    }
}

extern "C" {

void lair_default_options(lair_strength *s, lair_options *o) {
    if (s) {
        s->theta = 0.25;
        s->theta_c = 0.25;
        s->kind = LAIR_SOC_ABS;
        s->distance = 1;
    }
    if (o) {
        o->interp = LAIR_P_ONE_POINT;
        o->precision = LAIR_FP64;
        o->omega = 1.0;
        o->max_levels = 25;
        o->max_coarse = 128;
        o->stall = 0.9;
        o->block_size = 0;
        o->flags = 0;
        o->lump_tol = 0.0;
    }
}

lair_status lair_setup(const lair_csr *A, const lair_cf_levels *cf,
                       const lair_strength *s, const lair_options *o,
                       void *stream, lair_hierarchy **out) {
    return guarded([&]() -> lair_status {
        if (!out) fail(LAIR_EINVAL, "out must not be NULL");
        *out = nullptr;
        *out = setup_impl(A, cf, s, o, (hipStream_t)stream);
        return LAIR_OK;
    });
}

lair_status lair_setup_batch(int32_t nsys, const lair_csr *A, const lair_cf_levels *cf,
                             const lair_strength *s, const lair_options *o, void *stream,
                             lair_hierarchy **out) {
    return guarded([&]() -> lair_status {
        if (!out) fail(LAIR_EINVAL, "out must not be NULL");
        *out = nullptr;
        *out = setup_batch_impl(nsys, A, cf, s, o, (hipStream_t)stream);
        return LAIR_OK;
    });
}

lair_status lair_solve_batch(lair_hierarchy *h, const double *b, double *x, double rtol,
                             int32_t maxit, int32_t *iters, double *relres, lair_info *info,
                             void *stream) {
    return guarded([&]() -> lair_status {
        return solve_batch_impl(h, b, x, rtol, maxit, iters, relres, info,
                                (hipStream_t)stream);
    });
}

int32_t lair_num_systems(const lair_hierarchy *h) { return h ? h->nsys : 0; }

lair_status lair_update_diag(lair_hierarchy *h, const double *diag, int32_t on_device,
                             void *stream) {
    return guarded([&]() -> lair_status {
        update_diag_impl(h, diag, on_device, (hipStream_t)stream);
        return LAIR_OK;
    });
}

lair_status lair_system_levels(const lair_hierarchy *h, int32_t *levels) {
    return guarded([&]() -> lair_status {
        if (!h || !levels) fail(LAIR_EINVAL, "hierarchy and levels must not be NULL");
        if (!h->batch) fail(LAIR_EINVAL, "the hierarchy was not built by lair_setup_batch");
        for (int32_t q = 0; q < h->nsys; ++q)
            levels[q] = h->nsys > 1 ? h->sys_levels[q] : (int32_t)h->L.size();
        return LAIR_OK;
    });
}

lair_status lair_set_local_buckets(const int32_t *edges) {
    return guarded([&]() -> lair_status {
        set_local_buckets(edges);
        return LAIR_OK;
    });
}

lair_status lair_local_buckets(const lair_hierarchy *h, int32_t level, int32_t *edges) {
    return guarded([&]() -> lair_status {
        if (!h || !edges) fail(LAIR_EINVAL, "hierarchy and edges must not be NULL");
        if (level < 0 || level + 1 >= (int32_t)h->L.size())
            fail(LAIR_EINVAL, "level %d has no local solves", level);
        for (int k = 0; k < 5; ++k) edges[k] = h->L[level]->buckets[k];
        return LAIR_OK;
    });
}

lair_status lair_cycle(lair_hierarchy *h, const double *b, double *x,
                       int32_t nrhs, void *stream) {
    return guarded([&]() -> lair_status {
        cycle_impl(h, b, x, nrhs, (hipStream_t)stream);
        return LAIR_OK;
    });
}

lair_status lair_cycle_noalloc(lair_hierarchy *h, const double *b, double *x,
                               int32_t nrhs, void *stream) {
    return guarded([&]() -> lair_status {
        cycle_noalloc_impl(h, b, x, nrhs, (hipStream_t)stream);
        return LAIR_OK;
    });
}

lair_status lair_cycle_transpose(lair_hierarchy *h, const double *g, double *lam,
                                 int32_t nrhs, void *stream) {
    return guarded([&]() -> lair_status {
        cycle_transpose_impl(h, g, lam, nrhs, (hipStream_t)stream);
        return LAIR_OK;
    });
}

lair_status lair_solve(lair_hierarchy *h, const double *b, double *x, int32_t nrhs,
                       double rtol, int32_t maxit, lair_info *info, void *stream) {
    return guarded([&]() -> lair_status {
        return solve_impl(h, b, x, nrhs, rtol, maxit, info, (hipStream_t)stream, false);
    });
}

lair_status lair_solve_transpose(lair_hierarchy *h, const double *g, double *lam,
                                 int32_t nrhs, double rtol, int32_t maxit,
                                 lair_info *info, void *stream) {
    return guarded([&]() -> lair_status {
        if (h && scaled(h->opt))
            fail(LAIR_EUNSUPPORTED, "transposed solve with block scaling");
        if (h && nodal(h->opt))
            fail(LAIR_EUNSUPPORTED, "transposed solve on a nodal hierarchy");
        return solve_impl(h, g, lam, nrhs, rtol, maxit, info, (hipStream_t)stream, true);
    });
}

lair_status lair_solve_fgmres(lair_hierarchy *h, const double *b, double *x, int32_t nrhs,
                              double rtol, int32_t maxit, int32_t restart, lair_info *info,
                              void *stream) {
    return guarded([&]() -> lair_status {
        return solve_fgmres_impl(h, b, x, nrhs, rtol, maxit, restart, info,
                                 (hipStream_t)stream);
    });
}

int32_t lair_num_levels(const lair_hierarchy *h) { return h ? (int32_t)h->L.size() : 0; }

lair_status lair_level_stats_get(const lair_hierarchy *h, int32_t level,
                                 lair_level_stats *st) {
    return guarded([&]() -> lair_status {
        if (!h || !st) fail(LAIR_EINVAL, "NULL argument");
        if (level < 0 || level >= (int32_t)h->L.size()) fail(LAIR_EINVAL, "bad level %d", level);
        *st = h->L[level]->st;
        const Level &Lv = *h->L[level];
        if (Lv.nptr.get() && Lv.nc > 0) {
            std::vector<int32_t> hn((size_t)Lv.nc + 1);
            LAIR_HIP(hipStreamSynchronize(h->stream));
            LAIR_HIP(hipMemcpy(hn.data(), Lv.nptr.get(), sizeof(int32_t) * (Lv.nc + 1),
                               hipMemcpyDeviceToHost));
            int32_t smin = INT_MAX;
            for (int32_t c = 0; c < Lv.nc; ++c) smin = std::min(smin, hn[c + 1] - hn[c]);
            st->s_min = smin;
        } else {
            st->s_min = 0;
        }
        return LAIR_OK;
    });
}

lair_status lair_export(const lair_hierarchy *h, int32_t level, int32_t what,
                        void *host_buf, int64_t *bytes) {
    return guarded([&]() -> lair_status {
        if (!h || !bytes) fail(LAIR_EINVAL, "NULL argument");
        if (level < 0 || level >= (int32_t)h->L.size()) fail(LAIR_EINVAL, "bad level %d", level);
        const Level &Lv = *h->L[level];
        const void *src = nullptr;
        int64_t nb = 0;
        switch (what) {
            case 0: src = Lv.A.rp.get(); nb = 4 * ((int64_t)Lv.n + 1); break;
            case 1: src = Lv.A.cj.get(); nb = 4 * Lv.A.nnz; break;
            case 2: src = Lv.A.v.get(); nb = 8 * Lv.A.nnz; break;
            case 3: src = Lv.cf.get(); nb = Lv.cf.get() ? Lv.n : 0; break;
            case 4: src = Lv.smask.get(); nb = Lv.smask.get() ? Lv.A.nnz : 0; break;
            case 5: src = Lv.R.rp.get(); nb = Lv.R.rp.get() ? 4 * ((int64_t)Lv.nc + 1) : 0; break;
            case 6: src = Lv.R.cj.get(); nb = 4 * Lv.R.nnz; break;
            case 7: src = Lv.R.v.get(); nb = 8 * Lv.R.nnz; break;
            case 8: src = Lv.P.rp.get(); nb = Lv.P.rp.get() ? 4 * ((int64_t)Lv.n + 1) : 0; break;
            case 9: src = Lv.P.cj.get(); nb = 4 * Lv.P.nnz; break;
            case 10: src = Lv.P.v.get(); nb = 8 * Lv.P.nnz; break;
            case 11: src = Lv.nptr.get(); nb = Lv.nptr.get() ? 4 * ((int64_t)Lv.nc + 1) : 0; break;
            case 12: src = Lv.nbr.get(); nb = Lv.nptr.get() ? 4 * (Lv.R.nnz - Lv.nc) : 0; break;
            case 13: src = Lv.flags.get(); nb = Lv.flags.get() ? Lv.nc : 0; break;
            default: fail(LAIR_EINVAL, "unknown export selector %d", what);
        }
        int64_t cap = *bytes;
        *bytes = nb;
        if (!host_buf) return LAIR_OK;
        if (cap < nb) fail(LAIR_EINVAL, "export buffer too small (%lld < %lld)",
                           (long long)cap, (long long)nb);
        if (nb > 0) {
            LAIR_HIP(hipStreamSynchronize(h->stream));
            LAIR_HIP(hipMemcpy(host_buf, src, (size_t)nb, hipMemcpyDeviceToHost));
        }
        return LAIR_OK;
    });
}

void lair_free(lair_hierarchy *h) {
    if (!h) return;
    try {
        // the memory goes back to the allocator's cache: wait for every
        // launch that may still read it
        (void)hipDeviceSynchronize();
        delete h;
    } catch (...) {
    }
}

void lair_trim(void) { dev_trim(); }

void lair_memory(int64_t *in_use, int64_t *cached) {
    if (in_use) *in_use = (int64_t)dev_in_use_bytes();
    if (cached) *cached = (int64_t)dev_cached_bytes();
}

const char *lair_status_string(lair_status s) {
    switch (s) {
        case LAIR_OK: return "LAIR_OK";
        case LAIR_EINVAL: return "LAIR_EINVAL: invalid argument";
        case LAIR_ENOMEM: return "LAIR_ENOMEM: out of memory";
        case LAIR_EDEVICE: return "LAIR_EDEVICE: HIP device error";
        case LAIR_ESINGULAR: return "LAIR_ESINGULAR: singular coarsest matrix";
        case LAIR_ENOCONV: return "LAIR_ENOCONV: tolerance not reached";
        case LAIR_EUNSUPPORTED: return "LAIR_EUNSUPPORTED: size limit exceeded";
        default: return "unknown status";
    }
}

const char *lair_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
