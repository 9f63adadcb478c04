// Internal runtime of the freeform library: context, error reporting,
// device workspace and small launch helpers shared by the kernel files.
#pragma once

#include <hip/hip_runtime.h>

#include <array>
#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/freeform.h"

namespace ff {

// Workspace slots: each names one reusable device buffer owned by the context.
enum WsSlot {
    WS_BBOX = 0, WS_KEYS, WS_COUNTS, WS_CURSOR, WS_CELLS, WS_SCAN, WS_FLAG,
    WS_NT_OFF, WS_NT, WS_ROWLEN, WS_ASM_FLAG, WS_ZYN, WS_ZYE, WS_ASM_BM,
    WS_S0, WS_S1, WS_HS0, WS_HS1, WS_MS0, WS_MS1,            // working precision blocks
    WS_D0, WS_D1, WS_HD0, WS_HD1, WS_MD0, WS_MD1,            // FP64 blocks of the mixed path
    WS_GPART, WS_G, WS_C, WS_C32, WS_THETA, WS_RPART, WS_RES, WS_STATE, WS_RRSCR,
    WS_DINV, WS_DINV32, WS_NORMS, WS_CHUNKS, WS_GCHUNKS, WS_OBJ, WS_SIGN, WS_TUNE,
    WS_MLP0, WS_MLP1, WS_MLP2, WS_MLP3, WS_MLP4, WS_MLP5, WS_MLP6, WS_MLP7,
    WS_RT_CNT, WS_RT_PTR, WS_RT_COL, WS_RT_VAL32, WS_RT_VAL64,   // row-tile SpMM copies
    WS_CHEB0, WS_CHEB1, WS_CHEB2, WS_CHEB3, WS_CHEB4,             // Chebyshev-Jacobi work
    WS_RT8_CNT, WS_RT8_PTR, WS_RT8_COL, WS_RT8_VAL, WS_RT8_VALM,  // eight-row tile copy (H, and M)
    WS_RT8_VAL16, WS_RT8_MAX,                                     // its FP16 copy of H and |H| max
    WS_RTQ_CNT, WS_RTQ_PTR, WS_RTQ_VAL,                           // K-blocked FP16 copy (matrix cores)
    WS_CHEBQ,                                                     // column maxima of the scaled recurrence
    WS_RT16_CNT, WS_RT16_PTR, WS_RT16_COL, WS_RT16_VAL,           // sixteen-row H-only tile copy
    WS_SUBCELL,                                                   // sub-cell codes of the binning
    WS_MDINV,                                                     // diag(M)^-1 for the eigenvalue bounds
    WS_FPS, WS_RADMAX,                                            // farthest point sampling, radius maxima
    WS_MF,                                                        // matrix-free build: transposed entries
    WS_NT_TMP,                                                    // assembly: sort buffer of long transposed lists
    WS_RTQ_PMASK, WS_RTQ_POFF, WS_RTQ_PCNT, WS_RTQ_PVAL,          // zero-free K-blocked copy
    WS_BLEND,                                                     // warm start: column blend partials
    WS_SYM,                                                       // symmetric copy: row counts
    WS_T8Z_CNT, WS_T8Z_OFF, WS_T8Z_MASK, WS_T8Z_VAL,              // zero-free eight-row [H, M] copy
    WS_DENSE, WS_DENSE_X,                                         // small objects: dense pencil, start block
    WS_COUNT
};

}  // namespace ff

struct ff_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string last_error;
    void *ws[ff::WS_COUNT] = {};
    size_t ws_size[ff::WS_COUNT] = {};
    void *pinned = nullptr;          // small pinned host staging area
    size_t pinned_size = 0;
    std::unordered_map<std::string, int> tuned;   // SpMM shape key -> variant
    int timing = 0;                               // per-stage HIP-event timing of the solver
    int timing_mute = 0;                          // stage marks inside a region timed as one stage
    std::vector<hipEvent_t> ev_pool;              // reusable timing events
    size_t ev_used = 0;
    std::vector<std::array<int, 4>> marks;        // stage, launches, start event, end event
    double stage_ms[FF_STAGE_COUNT] = {};
    int64_t stage_launches[FF_STAGE_COUNT] = {};
    int verbose = 0;                 // FF_VERBOSE=1: residual trace on stderr
    int union_bits = -1;             // FF_UNION_BITS: cap on the tile-copy build's bitmap words (-1: none)
    // symbolic state of assemble_HM's sizing call, reused by a matching next call
    bool asm_valid = false;
    const void *asm_ptr[4] = {};
    int64_t asm_size[5] = {};
    int64_t asm_nnz = 0;
    int asm_rowmax = 0;
    int asm_wwords = 0;              // largest row window of that call, in bitmap words
    bool asm_bm = false;             // the sizing call kept its row bitmaps (workspace slot WS_ASM_BM)
    int64_t asm_bm_cap = -1;         // FF_ASM_BITMAP_BYTES: cap on that store (-1: the built-in 8 GiB)
    int cheb_shape = -1;             // FF_CHEB_SHAPE: launch shape of the matrix-core Chebyshev steps (-1: default)
    hipStream_t graph_stream = nullptr;   // private stream for graph capture
    // a-posteriori bounds of the last eigensolve, [n_obj][k] each
    int eb_nobj = 0, eb_k = 0;
    std::vector<double> eb_eig, eb_angle;
};

namespace ff {

int set_error(ff_ctx *ctx, int code, const char *fmt, ...);

// Stage timing: timing_reset at the start of a solve, StageMark around each
// stage (records a start and an end event on the stream when timing is on and
// the stream is not being captured), timing_collect after the final
// synchronisation (sums the marks' elapsed times into stage_ms).
void timing_reset(ff_ctx *ctx);
void timing_collect(ff_ctx *ctx);
int timing_event(ff_ctx *ctx, hipStream_t st);
struct StageMark {
    ff_ctx *ctx;
    hipStream_t st;
    int stage, launches, e0 = -1;
    StageMark(ff_ctx *c, hipStream_t s, int stg, int n = 1) : ctx(c), st(s), stage(stg), launches(n) {
        if (ctx->timing && !ctx->timing_mute) e0 = timing_event(ctx, st);
    }
    void end() {
        if (e0 < 0) return;
        const int e1 = timing_event(ctx, st);
        if (e1 >= 0) ctx->marks.push_back({stage, launches, e0, e1});
        e0 = -1;
    }
    ~StageMark() { end(); }
    StageMark(const StageMark &) = delete;
    StageMark &operator=(const StageMark &) = delete;
};
// while alive (and on), StageMarks inside record nothing: an enclosing mark times the region as one stage
struct TimingMute {
    ff_ctx *ctx;
    int prev;
    TimingMute(ff_ctx *c, bool on) : ctx(c), prev(c->timing_mute) { if (on) ctx->timing_mute = 1; }
    ~TimingMute() { ctx->timing_mute = prev; }
    TimingMute(const TimingMute &) = delete;
    TimingMute &operator=(const TimingMute &) = delete;
};

// Grow-only device buffer for a workspace slot; returns nullptr on failure
// (and records FF_ERR_OOM in the context).
void *ws_get(ff_ctx *ctx, int slot, size_t bytes);
void *pinned_get(ff_ctx *ctx, size_t bytes);

#define FF_HIP(ctx, call)                                                              \
    do {                                                                               \
        hipError_t e_ = (call);                                                        \
        if (e_ != hipSuccess)                                                          \
            return ff::set_error((ctx), FF_ERR_HIP, "%s failed: %s (%s:%d)", #call,    \
                                 hipGetErrorString(e_), __FILE__, __LINE__);           \
    } while (0)

#define FF_CHECK_LAUNCH(ctx)                                                           \
    do {                                                                               \
        hipError_t e_ = hipGetLastError();                                             \
        if (e_ != hipSuccess)                                                          \
            return ff::set_error((ctx), FF_ERR_HIP, "kernel launch failed: %s (%s:%d)", \
                                 hipGetErrorString(e_), __FILE__, __LINE__);           \
    } while (0)

#define FF_REQUIRE(ctx, cond, ...)                                                     \
    do {                                                                               \
        if (!(cond)) return ff::set_error((ctx), FF_ERR_INVALID_ARG, __VA_ARGS__);     \
    } while (0)

// Device-wide exclusive scan of int64 values: out[0] = 0, out[i+1] = out[i] + in[i].
// `in` and `out` may alias only if out == in + 1 is not required; out has len+1 entries.
int scan_exclusive_i64(ff_ctx *ctx, const int64_t *in, int64_t *out, int64_t len);
// Same for int32 counts into int64 offsets.
int scan_exclusive_i32_to_i64(ff_ctx *ctx, const int32_t *in, int64_t *out, int64_t len);

// The transpose of the neighbour relation: NT(k) = {(i, slot) : N(i)[slot] = k} in ascending i,
// nt_off [n+1] and nt [total] device out; empty_node (device, or NULL) receives the smallest
// node with an empty list (all ones if none).
int build_transpose(ff_ctx *ctx, hipStream_t st, int64_t n, int64_t q, int64_t total, const int64_t *nbr_off,
                    const int32_t *nbr_id, int64_t *nt_off, int2 *nt, unsigned long long *empty_node);

inline unsigned grid_for(int64_t items, int per_block) {
    int64_t g = (items + per_block - 1) / per_block;
    return (unsigned)(g < 1 ? 1 : g);
}

}  // namespace ff
