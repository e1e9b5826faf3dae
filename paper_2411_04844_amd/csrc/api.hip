// Status strings, thread-local error text, argument checks and dgr_check.
#include <cmath>
#include <cstdarg>
#include <cstring>

#include "internal.h"

namespace dgr {

static thread_local char g_err[512] = "";

dgr_status fail(dgr_status s, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return s;
}

static bool finite_pos(float x) { return std::isfinite(x) && x > 0.0f; }

dgr_status check_grid(const dgr_grid *g) {
    DGR_CHECK(g != nullptr, "grid is null");
    for (int a = 0; a < 3; ++a) {
        DGR_CHECK(g->dims[a] >= 1 && g->dims[a] <= 16384, "grid dims[%d] = %d outside [1, 16384]", a,
                  g->dims[a]);
        DGR_CHECK(finite_pos(g->inv_h[a]), "grid inv_h[%d] must be finite and > 0", a);
        DGR_CHECK(std::isfinite(g->lo[a]), "grid lo[%d] must be finite", a);
    }
    int64_t nvox = (int64_t)g->dims[0] * g->dims[1] * g->dims[2];
    DGR_CHECK(nvox < (int64_t(1) << 34), "grid has too many voxels");
    return DGR_OK;
}

dgr_status check_trunc(const dgr_trunc *t) {
    DGR_CHECK(t != nullptr, "trunc is null");
    DGR_CHECK(std::isfinite(t->k_sigma), "k_sigma must be finite");
    if (t->k_sigma <= 0.0f)
        DGR_CHECK(t->box_half >= 0 && t->box_half <= 1024, "box_half %d outside [0, 1024]",
                  t->box_half);
    return DGR_OK;
}

dgr_status check_geometry(const dgr_geometry *g) {
    DGR_CHECK(g != nullptr, "geometry is null");
    DGR_CHECK(g->kind == DGR_PARALLEL || g->kind == DGR_CONE || g->kind == DGR_FAN, "geometry kind %d unknown",
              g->kind);
    DGR_CHECK(g->n_views >= 1 && g->nu >= 1 && g->nv >= 1, "geometry sizes must be >= 1");
    DGR_CHECK(g->nu <= 65536 && g->nv <= 65536 && g->n_views <= 65535,
              "geometry sizes too large (nu, nv <= 65536, n_views <= 65535)");
    DGR_CHECK(g->views != nullptr, "geometry views is null");
    DGR_CHECK(finite_pos(g->step), "geometry step must be finite and > 0");
    DGR_CHECK(std::isfinite(g->length_scale), "geometry length_scale must be finite");
    return DGR_OK;
}

}  // namespace dgr

using namespace dgr;

extern "C" const char *dgr_status_string(dgr_status s) {
    switch (s) {
        case DGR_OK: return "ok";
        case DGR_ERR_INVALID_ARG: return "invalid argument";
        case DGR_ERR_WORKSPACE: return "workspace too small or misaligned";
        case DGR_ERR_CAPACITY: return "pair capacity exceeded";
        case DGR_ERR_HIP: return "HIP runtime error";
    }
    return "unknown status";
}

extern "C" const char *dgr_last_error(void) { return g_err; }

extern "C" int32_t dgr_version(void) { return 1; }

extern "C" dgr_status dgr_check(void *ws, void *stream) {
    if (!ws) return fail(DGR_ERR_INVALID_ARG, "ws is null");
    hipStream_t st = as_stream(stream);
    VoxHeader h;
    DGR_TRY_HIP(hipMemcpyAsync(&h, ws, sizeof(h), hipMemcpyDeviceToHost, st));
    DGR_TRY_HIP(hipStreamSynchronize(st));
    if (h.overflow) {
        uint32_t zero = 0;
        DGR_TRY_HIP(hipMemcpyAsync(ws, &zero, sizeof(zero), hipMemcpyHostToDevice, st));
        DGR_TRY_HIP(hipStreamSynchronize(st));
        return fail(DGR_ERR_CAPACITY, "voxelization needed %llu pairs, more than the workspace holds",
                    (unsigned long long)h.total);
    }
    return DGR_OK;
}
