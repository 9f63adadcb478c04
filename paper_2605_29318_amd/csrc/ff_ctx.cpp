// Context lifetime, error reporting and workspace management.
#include "ff_internal.h"

#include <cstdlib>

namespace ff {

int set_error(ff_ctx *ctx, int code, const char *fmt, ...) {
    if (ctx) {
        char buf[1024];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof(buf), fmt, ap);
        va_end(ap);
        ctx->last_error = buf;
    }
    return code;
}

void *ws_get(ff_ctx *ctx, int slot, size_t bytes) {
    if (bytes == 0) bytes = 256;
    if (ctx->ws_size[slot] >= bytes) return ctx->ws[slot];
    if (ctx->ws[slot]) {
        (void)hipStreamSynchronize(ctx->stream);
        (void)hipFree(ctx->ws[slot]);
        ctx->ws[slot] = nullptr;
        ctx->ws_size[slot] = 0;
    }
    size_t want = bytes + bytes / 8;           // headroom for slightly larger reuse
    want = (want + 255) & ~(size_t)255;
    void *p = nullptr;
    if (hipMalloc(&p, want) != hipSuccess) {
        (void)hipGetLastError();
        set_error(ctx, FF_ERR_OOM, "device allocation of %zu bytes (workspace slot %d) failed",
                  want, slot);
        return nullptr;
    }
    ctx->ws[slot] = p;
    ctx->ws_size[slot] = want;
    return p;
}

void *pinned_get(ff_ctx *ctx, size_t bytes) {
    if (ctx->pinned_size >= bytes) return ctx->pinned;
    if (ctx->pinned) {
        (void)hipStreamSynchronize(ctx->stream);
        (void)hipHostFree(ctx->pinned);
        ctx->pinned = nullptr;
        ctx->pinned_size = 0;
    }
    size_t want = bytes < 65536 ? 65536 : bytes;
    void *p = nullptr;
    if (hipHostMalloc(&p, want, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        set_error(ctx, FF_ERR_OOM, "pinned host allocation of %zu bytes failed", want);
        return nullptr;
    }
    ctx->pinned = p;
    ctx->pinned_size = want;
    return p;
}

}  // namespace ff

extern "C" {

int ff_ctx_create(ff_ctx **out, int device, void *hip_stream) {
    if (!out) return FF_ERR_INVALID_ARG;
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count <= 0) {
        (void)hipGetLastError();
        return FF_ERR_HIP;
    }
    if (device < 0 || device >= count) return FF_ERR_INVALID_ARG;
    if (hipSetDevice(device) != hipSuccess) return FF_ERR_HIP;
    ff_ctx *ctx = new ff_ctx();
    ctx->device = device;
    ctx->stream = (hipStream_t)hip_stream;
    const char *v = getenv("FF_VERBOSE");
    ctx->verbose = v && v[0] == '1';
    *out = ctx;
    return FF_OK;
}

void ff_ctx_destroy(ff_ctx *ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    for (int i = 0; i < ff::WS_COUNT; ++i)
        if (ctx->ws[i]) (void)hipFree(ctx->ws[i]);
    if (ctx->pinned) (void)hipHostFree(ctx->pinned);
    if (ctx->graph_stream) (void)hipStreamDestroy(ctx->graph_stream);
    delete ctx;
}

const char *ff_last_error(const ff_ctx *ctx) {
    return ctx ? ctx->last_error.c_str() : "null context";
}

int ff_ctx_stage_times(const ff_ctx *ctx, double *spmm_ms, double *gram_ms, double *rr_ms,
                       double *update_ms, double *total_ms) {
    if (!ctx) return FF_ERR_INVALID_ARG;
    if (spmm_ms) *spmm_ms = ctx->stage_ms[0];
    if (gram_ms) *gram_ms = ctx->stage_ms[1];
    if (rr_ms) *rr_ms = ctx->stage_ms[2];
    if (update_ms) *update_ms = ctx->stage_ms[3];
    if (total_ms) *total_ms = ctx->stage_ms[4];
    return FF_OK;
}

}  // extern "C"
