// Context lifetime, error reporting and workspace management.
#include "ff_internal.h"
#include "k_lobpcg.h"

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

void timing_reset(ff_ctx *ctx) {
    ctx->ev_used = 0;
    ctx->marks.clear();
    for (int i = 0; i < FF_STAGE_COUNT; ++i) {
        ctx->stage_ms[i] = 0.0;
        ctx->stage_launches[i] = 0;
    }
}

int timing_event(ff_ctx *ctx, hipStream_t st) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) {
        (void)hipGetLastError();
        return -1;
    }
    if (ctx->ev_used == ctx->ev_pool.size()) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) {
            (void)hipGetLastError();
            return -1;
        }
        ctx->ev_pool.push_back(e);
    }
    const int idx = (int)ctx->ev_used;
    if (hipEventRecord(ctx->ev_pool[idx], st) != hipSuccess) {
        (void)hipGetLastError();
        return -1;
    }
    ++ctx->ev_used;
    return idx;
}

void timing_collect(ff_ctx *ctx) {
    for (const auto &mk : ctx->marks) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, ctx->ev_pool[mk[2]], ctx->ev_pool[mk[3]]) != hipSuccess) {
            (void)hipGetLastError();
            continue;
        }
        ctx->stage_ms[mk[0]] += ms;
        ctx->stage_launches[mk[0]] += mk[1];
    }
    ctx->marks.clear();
    ctx->ev_used = 0;
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
    // a cap on the LDS bitmap of the tile-copy build, so that its other paths can be exercised
    if (const char *b = getenv("FF_UNION_BITS")) ctx->union_bits = atoi(b) < 0 ? 0 : atoi(b);
    // a cap on the row bitmaps the assembly's symbolic pass keeps, so that the numeric pass's own
    // marking can be exercised
    if (const char *b = getenv("FF_ASM_BITMAP_BYTES")) ctx->asm_bm_cap = atoll(b) < 0 ? 0 : atoll(b);
    // the launch shape of the matrix-core Chebyshev steps, for tuning (every shape sums alike)
    if (const char *b = getenv("FF_CHEB_SHAPE")) ctx->cheb_shape = atoi(b) < 0 ? -1 : atoi(b);
    // the fixed scratch of rayleigh_ritz_noalloc: its device address, once per device
    if (ff::lob::noalloc_setup(ctx) != FF_OK) {
        delete ctx;
        return FF_ERR_HIP;
    }
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
    for (hipEvent_t e : ctx->ev_pool) (void)hipEventDestroy(e);
    delete ctx;
}

const char *ff_last_error(const ff_ctx *ctx) {
    return ctx ? ctx->last_error.c_str() : "null context";
}

int ff_ctx_set_stage_timing(ff_ctx *ctx, int enable) {
    if (!ctx) return FF_ERR_INVALID_ARG;
    ctx->timing = enable != 0;
    return FF_OK;
}

int ff_ctx_stage_times(const ff_ctx *ctx, int n, double *ms, int64_t *launches) {
    if (!ctx || n < 0) return FF_ERR_INVALID_ARG;
    for (int i = 0; i < n && i < FF_STAGE_COUNT; ++i) {
        if (ms) ms[i] = ctx->stage_ms[i];
        if (launches) launches[i] = ctx->stage_launches[i];
    }
    return FF_STAGE_COUNT;
}

const char *ff_stage_name(int stage) {
    static const char *names[FF_STAGE_COUNT] = {"spmm",          "precond_product", "precond_other", "gram",
                                                "rayleigh_ritz", "update",          "resid",         "fp64_phase",
                                                "total"};
    return stage >= 0 && stage < FF_STAGE_COUNT ? names[stage] : "";
}

}  // extern "C"
