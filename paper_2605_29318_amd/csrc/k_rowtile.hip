// Row-tile SpMM: tiles of four consecutive rows share one merged column list.
#include "k_rowtile.h"

#include <climits>

struct ff_rowtiles {
    int device = 0;
    hipStream_t stream = nullptr;                  // the context's stream, kept for destruction
    ff::rt::RTView v;
    void *mem[4] = {nullptr, nullptr, nullptr, nullptr};
};

namespace ff {
namespace rt {

const char *kSubNames[kSubs] = {"rowtile4_waves4_batch4", "rowtile4_waves2_batch8", "rowtile4_waves4_batch4_occ4"};

// consecutive workgroups go round-robin to the 8 XCDs; give each XCD a contiguous range of tiles
__device__ inline int xcd_remap(int b, int nb) {
    const int xcd = b & 7, idx = b >> 3, per = nb >> 3, rem = nb & 7;
    const int start = xcd * per + (xcd < rem ? xcd : rem);
    const int cnt = per + (xcd < rem ? 1 : 0);
    return idx < cnt ? start + idx : b;
}

// ---------------------------------------------------------------------------
// building the tile copy: one thread per tile merges its (sorted) rows
// ---------------------------------------------------------------------------

struct Merge4 {
    int64_t p[kTileRows], e[kTileRows];
    int32_t h[kTileRows];
};

__device__ inline void merge_init(Merge4 &s, int64_t nrows, int64_t r0, const int64_t *row_ptr, const int32_t *col) {
#pragma unroll
    for (int i = 0; i < kTileRows; ++i) {
        const bool in = r0 + i < nrows;
        s.p[i] = in ? row_ptr[r0 + i] : 0;
        s.e[i] = in ? row_ptr[r0 + i + 1] : 0;
        s.h[i] = s.p[i] < s.e[i] ? col[s.p[i]] : INT_MAX;
    }
}
__device__ inline int32_t merge_head(const Merge4 &s) {
    int32_t c = s.h[0];
#pragma unroll
    for (int i = 1; i < kTileRows; ++i) c = min(c, s.h[i]);
    return c;
}

__global__ void rt_count_kernel(int64_t nrows, int64_t ntiles, const int64_t *row_ptr, const int32_t *col,
                                int64_t *cnt) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ntiles) return;
    Merge4 s;
    merge_init(s, nrows, t * kTileRows, row_ptr, col);
    int64_t k = 0;
    for (int32_t cur = merge_head(s); cur != INT_MAX; cur = merge_head(s)) {
        ++k;
#pragma unroll
        for (int i = 0; i < kTileRows; ++i)
            if (s.h[i] == cur) {
                ++s.p[i];
                s.h[i] = s.p[i] < s.e[i] ? col[s.p[i]] : INT_MAX;
            }
    }
    cnt[t] = k;
}

template <typename T>
__global__ void rt_fill_kernel(int64_t nrows, int64_t ntiles, const int64_t *row_ptr, const int32_t *col,
                               const double *H, const double *M, const int64_t *tptr, int32_t *tcol, T *tval,
                               int write_col) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ntiles) return;
    Merge4 s;
    merge_init(s, nrows, t * kTileRows, row_ptr, col);
    int64_t o = tptr[t];
    for (int32_t cur = merge_head(s); cur != INT_MAX; cur = merge_head(s), ++o) {
        if (write_col) tcol[o] = cur;
        T *v = tval + o * 8;
#pragma unroll
        for (int i = 0; i < kTileRows; ++i) {
            const bool hit = s.h[i] == cur;
            v[i] = hit ? (T)H[s.p[i]] : (T)0;
            v[4 + i] = hit ? (T)M[s.p[i]] : (T)0;
            if (hit) {
                ++s.p[i];
                s.h[i] = s.p[i] < s.e[i] ? col[s.p[i]] : INT_MAX;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// SpMM on the tile copy: one wavefront per tile
// ---------------------------------------------------------------------------

template <typename T> struct Vec;
template <> struct Vec<float> { typedef float4 type; static constexpr int n = 4; };
template <> struct Vec<double> { typedef double2 type; static constexpr int n = 2; };

// Accumulators: FP64 for the products of the eigensolver (a product of two FP32
// numbers is exact in FP64), FP32 for the H-only products of the preconditioner.
template <typename A> struct Acc4 { A v[4]; };
__device__ inline void acc_fma(Acc4<double> &a, float h, const float4 &x) {
    const double d = (double)h;
    a.v[0] += d * (double)x.x;
    a.v[1] += d * (double)x.y;
    a.v[2] += d * (double)x.z;
    a.v[3] += d * (double)x.w;
}
__device__ inline void acc_fma(Acc4<float> &a, float h, const float4 &x) {
    a.v[0] = fmaf(h, x.x, a.v[0]);
    a.v[1] = fmaf(h, x.y, a.v[1]);
    a.v[2] = fmaf(h, x.z, a.v[2]);
    a.v[3] = fmaf(h, x.w, a.v[3]);
}
__device__ inline void acc_fma(Acc4<double> &a, double h, const double2 &x) {
    a.v[0] += h * x.x;
    a.v[1] += h * x.y;
}
template <typename A>
__device__ inline void acc_store(float *p, const Acc4<A> &a) {
    *(float4 *)p = make_float4((float)a.v[0], (float)a.v[1], (float)a.v[2], (float)a.v[3]);
}
__device__ inline void acc_store(double *p, const Acc4<double> &a) { *(double2 *)p = make_double2(a.v[0], a.v[1]); }

typedef float f32x4 __attribute__((ext_vector_type(4)));

// Chunk of 64 union entries: column and the eight values of entry l in lane l.
// With kHM false only the H values are loaded and staged (stride 4 in LDS).
template <typename T, bool kHM> struct Chunk;
template <bool kHM> struct Chunk<float, kHM> {
    int32_t j;
    f32x4 a, b;                                    // H rows 0..3, M rows 0..3
    __device__ void load(const int32_t *tcol, const float *tval, int64_t e, bool in) {
        j = 0;
        a = b = f32x4{0.f, 0.f, 0.f, 0.f};
        if (in) {
            j = __builtin_nontemporal_load(tcol + e);
            a = __builtin_nontemporal_load((const f32x4 *)(tval + e * 8));
            if (kHM) b = __builtin_nontemporal_load((const f32x4 *)(tval + e * 8 + 4));
        }
    }
    __device__ void stage(float *sv, int lane) const {
        if (kHM) {
            *(f32x4 *)(sv + lane * 8) = a;
            *(f32x4 *)(sv + lane * 8 + 4) = b;
        } else {
            *(f32x4 *)(sv + lane * 4) = a;
        }
    }
};
typedef double f64x2 __attribute__((ext_vector_type(2)));
template <bool kHM> struct Chunk<double, kHM> {
    static constexpr int NQ = kHM ? 4 : 2;
    int32_t j;
    f64x2 v[NQ];
    __device__ void load(const int32_t *tcol, const double *tval, int64_t e, bool in) {
        j = 0;
#pragma unroll
        for (int q = 0; q < NQ; ++q) v[q] = f64x2{0.0, 0.0};
        if (in) {
            j = __builtin_nontemporal_load(tcol + e);
#pragma unroll
            for (int q = 0; q < NQ; ++q) v[q] = __builtin_nontemporal_load((const f64x2 *)(tval + e * 8 + 2 * q));
        }
    }
    __device__ void stage(double *sv, int lane) const {
#pragma unroll
        for (int q = 0; q < NQ; ++q) *(f64x2 *)(sv + lane * 2 * NQ + 2 * q) = v[q];
    }
};

// One wavefront per tile. The wave reads 64 union entries (column and eight
// values) with one coalesced load per lane, prefetches the next 64 while it
// works on these, keeps the values in a wave-private LDS area (each lane group
// reads its entry's values as a broadcast) and hands each column to the lane
// group that needs it by a cross-lane shuffle. Lanes form groups of
// G = m / VN; group g takes entries g, g + NG, ... of the chunk; each lane holds
// VN columns of the gathered row of Y and accumulates all four rows of the tile
// in FP64; the groups are summed at the end. With kHM false the kernel forms
// H Y alone (MY is not touched), accumulating in A.
template <typename T, typename A, bool kHM, int kWaves, int kBatch, int kOcc>
__global__ void __launch_bounds__(64 * kWaves) __attribute__((amdgpu_waves_per_eu(kOcc, 8)))
spmm_rt_kernel(int64_t nrows, int64_t ntiles, const int64_t *tptr, const int32_t *tcol, const T *tval, const T *Y,
               int64_t ldy, T *HY, T *MY, int64_t ldo, int m, const int *row_obj, const int *obj_status) {
    typedef typename Vec<T>::type V;
    constexpr int VN = Vec<T>::n;
    constexpr int NV = kHM ? 8 : 4;                // staged values per entry
    __shared__ __align__(16) T svals[kWaves][64 * NV];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t t = (int64_t)xcd_remap(blockIdx.x, gridDim.x) * kWaves + wv;
    if (t >= ntiles) return;
    const int64_t r0 = t * kTileRows;
    bool act[kTileRows];
    bool any = false;
#pragma unroll
    for (int i = 0; i < kTileRows; ++i) {
        act[i] = r0 + i < nrows && (!obj_status || obj_status[row_obj[r0 + i]] == 0);
        any = any || act[i];
    }
    if (!any) return;
    const int G = m / VN;
    const int NG = 64 / G;
    const int g = lane / G, c = lane - g * G;
    const bool on = g < NG;
    const int steps = (64 + NG - 1) / NG;
    T *sv = svals[wv];
    const int64_t e0 = tptr[t], e1 = tptr[t + 1];
    Acc4<A> aH[kTileRows], aM[kHM ? kTileRows : 1];
#pragma unroll
    for (int i = 0; i < kTileRows; ++i)
#pragma unroll
        for (int q = 0; q < 4; ++q) aH[i].v[q] = 0;
#pragma unroll
    for (int i = 0; i < (kHM ? kTileRows : 1); ++i)
#pragma unroll
        for (int q = 0; q < 4; ++q) aM[i].v[q] = 0;
    Chunk<T, kHM> nxt;
    nxt.load(tcol, tval, e0 + lane, e0 + lane < e1);
    for (int64_t base = e0; base < e1; base += 64) {
        const int cnt = (int)(e1 - base < 64 ? e1 - base : 64);
        const int32_t jc = nxt.j;
        __builtin_amdgcn_wave_barrier();
        nxt.stage(sv, lane);
        __builtin_amdgcn_wave_barrier();
        nxt.load(tcol, tval, base + 64 + lane, base + 64 + lane < e1);
        for (int s0 = 0; s0 < steps; s0 += kBatch) {
            V x[kBatch];
#pragma unroll
            for (int u = 0; u < kBatch; ++u) {
                const int src = (s0 + u) * NG + g;
                const int32_t j = __shfl(jc, src < 64 ? src : 63, 64);
                const bool ok = on && (s0 + u < steps) && src < cnt;
                if (ok)
                    x[u] = *(const V *)(Y + (int64_t)j * ldy + c * VN);
                else
                    x[u] = V{};
            }
#pragma unroll
            for (int u = 0; u < kBatch; ++u) {
                const int src = (s0 + u) * NG + g;
                const bool ok = on && (s0 + u < steps) && src < cnt;
                if (ok) {
                    const T *vv = sv + src * NV;
#pragma unroll
                    for (int i = 0; i < kTileRows; ++i) {
                        acc_fma(aH[i], vv[i], x[u]);
                        if (kHM) acc_fma(aM[i], vv[4 + i], x[u]);
                    }
                }
            }
        }
    }
    if ((64 % G) == 0) {
#pragma unroll
        for (int i = 0; i < kTileRows; ++i)
            for (int d = G; d < 64; d <<= 1)
#pragma unroll
                for (int q = 0; q < VN; ++q) {
                    aH[i].v[q] += __shfl_xor(aH[i].v[q], d, 64);
                    if (kHM) aM[i].v[q] += __shfl_xor(aM[i].v[q], d, 64);
                }
    } else {
        __shared__ A red[kWaves][2][4][64];
#pragma unroll
        for (int i = 0; i < kTileRows; ++i) {
            for (int q = 0; q < VN; ++q) {
                red[wv][0][q][lane] = aH[i].v[q];
                if (kHM) red[wv][1][q][lane] = aM[i].v[q];
            }
            __builtin_amdgcn_wave_barrier();
            if (g == 0)
                for (int tt = 1; tt < NG; ++tt)
                    for (int q = 0; q < VN; ++q) {
                        aH[i].v[q] += red[wv][0][q][tt * G + c];
                        if (kHM) aM[i].v[q] += red[wv][1][q][tt * G + c];
                    }
            __builtin_amdgcn_wave_barrier();
        }
    }
    if (g == 0) {
#pragma unroll
        for (int i = 0; i < kTileRows; ++i)
            if (act[i]) {
                acc_store(HY + (r0 + i) * ldo + c * VN, aH[i]);
                if (kHM) acc_store(MY + (r0 + i) * ldo + c * VN, aM[kHM ? i : 0]);
            }
    }
}

template <typename T, typename A = double, bool kHM = true>
int launch(ff_ctx *ctx, hipStream_t st, const RTView &v, const T *tval, int sub, int m, const T *Y, int64_t ldy,
           T *HY, T *MY, int64_t ldo, const int *row_obj, const int *status) {
    // each lane holds one 16-byte access of the gathered row (narrower loads cost the texture unit as many cycles)
#define FF_RT(W, B, O)                                                                                      \
    hipLaunchKernelGGL((spmm_rt_kernel<T, A, kHM, W, B, O>), dim3(grid_for(v.ntiles, W)), dim3(64 * W), 0, st, \
                       v.n, v.ntiles, v.tptr, v.tcol, tval, Y, ldy, HY, MY, ldo, m, row_obj, status)
    switch (sub) {
        case 1: FF_RT(2, 8, 1); break;
        case 2: FF_RT(4, 4, 4); break;
        default: FF_RT(4, 4, 1); break;
    }
#undef FF_RT
    FF_CHECK_LAUNCH(ctx);
    return FF_OK;
}

int spmm32(ff_ctx *ctx, hipStream_t st, const RTView &v, int sub, int m, const float *Y, int64_t ldy, float *HY,
           float *MY, int64_t ldo, const int *row_obj, const int *status) {
    FF_REQUIRE(ctx, v.v32 != nullptr, "row tiles have no FP32 values");
    return launch<float>(ctx, st, v, v.v32, sub, m, Y, ldy, HY, MY, ldo, row_obj, status);
}
int spmm64(ff_ctx *ctx, hipStream_t st, const RTView &v, int sub, int m, const double *Y, int64_t ldy, double *HY,
           double *MY, int64_t ldo, const int *row_obj, const int *status) {
    FF_REQUIRE(ctx, v.v64 != nullptr, "row tiles have no FP64 values");
    return launch<double>(ctx, st, v, v.v64, sub, m, Y, ldy, HY, MY, ldo, row_obj, status);
}
int spmm_h32(ff_ctx *ctx, hipStream_t st, const RTView &v, int sub, int m, const float *Y, int64_t ldy, float *HY,
             int64_t ldo, const int *row_obj, const int *status) {
    FF_REQUIRE(ctx, v.v32 != nullptr, "row tiles have no FP32 values");
    return launch<float, float, false>(ctx, st, v, v.v32, sub, m, Y, ldy, HY, nullptr, ldo, row_obj, status);
}
int spmm_h64(ff_ctx *ctx, hipStream_t st, const RTView &v, int sub, int m, const double *Y, int64_t ldy, double *HY,
             int64_t ldo, const int *row_obj, const int *status) {
    FF_REQUIRE(ctx, v.v64 != nullptr, "row tiles have no FP64 values");
    return launch<double, double, false>(ctx, st, v, v.v64, sub, m, Y, ldy, HY, nullptr, ldo, row_obj, status);
}

// tile pointers and the number of union entries (host), in caller-provided memory
static int build_ptr(ff_ctx *ctx, hipStream_t st, int64_t n, const int64_t *row_ptr, const int32_t *col,
                     int64_t *cnt, int64_t *tptr, int64_t ntiles, int64_t *entries) {
    hipLaunchKernelGGL(rt_count_kernel, dim3(grid_for(ntiles, 256)), dim3(256), 0, st, n, ntiles, row_ptr, col, cnt);
    FF_CHECK_LAUNCH(ctx);
    int rc = scan_exclusive_i64(ctx, cnt, tptr, ntiles);
    if (rc) return rc;
    int64_t *h = (int64_t *)pinned_get(ctx, 64);
    if (!h) return FF_ERR_OOM;
    FF_HIP(ctx, hipMemcpyAsync(h, tptr + ntiles, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    FF_HIP(ctx, hipStreamSynchronize(st));
    *entries = h[0];
    return FF_OK;
}

static int fill(ff_ctx *ctx, hipStream_t st, int64_t n, int64_t ntiles, const int64_t *row_ptr, const int32_t *col,
                const double *H, const double *M, const int64_t *tptr, int32_t *tcol, float *v32, double *v64) {
    if (v32)
        hipLaunchKernelGGL(rt_fill_kernel<float>, dim3(grid_for(ntiles, 256)), dim3(256), 0, st, n, ntiles, row_ptr,
                           col, H, M, tptr, tcol, v32, 1);
    if (v64)
        hipLaunchKernelGGL(rt_fill_kernel<double>, dim3(grid_for(ntiles, 256)), dim3(256), 0, st, n, ntiles, row_ptr,
                           col, H, M, tptr, tcol, v64, v32 ? 0 : 1);
    FF_CHECK_LAUNCH(ctx);
    return FF_OK;
}

int build_ws(ff_ctx *ctx, hipStream_t st, int64_t n, const int64_t *row_ptr, const int32_t *col, const double *H,
             const double *M, int want32, int want64, RTView *out) {
    FF_REQUIRE(ctx, n > 0 && row_ptr && col && H && M && out, "bad arguments");
    const int64_t ntiles = (n + kTileRows - 1) / kTileRows;
    int64_t *cnt = (int64_t *)ws_get(ctx, WS_RT_CNT, (size_t)(ntiles + 1) * sizeof(int64_t));
    int64_t *tptr = (int64_t *)ws_get(ctx, WS_RT_PTR, (size_t)(ntiles + 1) * sizeof(int64_t));
    if (!cnt || !tptr) return FF_ERR_OOM;
    int64_t entries = 0;
    int rc = build_ptr(ctx, st, n, row_ptr, col, cnt, tptr, ntiles, &entries);
    if (rc) return rc;
    int32_t *tcol = (int32_t *)ws_get(ctx, WS_RT_COL, (size_t)std::max<int64_t>(entries, 1) * sizeof(int32_t));
    float *v32 = want32 ? (float *)ws_get(ctx, WS_RT_VAL32, (size_t)std::max<int64_t>(entries, 1) * 8 * sizeof(float))
                        : nullptr;
    double *v64 = want64 ? (double *)ws_get(ctx, WS_RT_VAL64,
                                            (size_t)std::max<int64_t>(entries, 1) * 8 * sizeof(double))
                         : nullptr;
    if (!tcol || (want32 && !v32) || (want64 && !v64)) return FF_ERR_OOM;
    if ((rc = fill(ctx, st, n, ntiles, row_ptr, col, H, M, tptr, tcol, v32, v64))) return rc;
    out->n = n;
    out->ntiles = ntiles;
    out->entries = entries;
    out->tptr = tptr;
    out->tcol = tcol;
    out->v32 = v32;
    out->v64 = v64;
    return FF_OK;
}

}  // namespace rt
}  // namespace ff

using namespace ff;

extern "C" {

int rowtiles_build(ff_ctx *ctx, int64_t n, const int64_t *row_ptr, const int32_t *col, const double *H,
                   const double *M, int precision, ff_rowtiles **out) {
    if (!ctx || !out) return FF_ERR_INVALID_ARG;
    *out = nullptr;
    FF_REQUIRE(ctx, n > 0 && row_ptr && col && H && M, "bad arguments");
    FF_REQUIRE(ctx, precision >= 0 && precision <= 2, "precision must be 0 (FP64), 1 (FP32) or 2 (both)");
    FF_HIP(ctx, hipSetDevice(ctx->device));
    hipStream_t st = ctx->stream;
    ff_rowtiles *h = new ff_rowtiles();
    h->device = ctx->device;
    h->stream = ctx->stream;
    const int64_t ntiles = (n + rt::kTileRows - 1) / rt::kTileRows;
    auto alloc = [&](int slot, size_t bytes) -> void * {
        void *p = nullptr;
        if (hipMalloc(&p, bytes < 256 ? 256 : bytes) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
        h->mem[slot] = p;
        return p;
    };
    int rc = FF_OK;
    int64_t *cnt = nullptr, *tptr = (int64_t *)alloc(0, (size_t)(ntiles + 1) * sizeof(int64_t));
    if (hipMalloc((void **)&cnt, (size_t)(ntiles + 1) * sizeof(int64_t)) != hipSuccess) {
        (void)hipGetLastError();
        cnt = nullptr;
    }
    int64_t entries = 0;
    if (!tptr || !cnt) rc = set_error(ctx, FF_ERR_OOM, "row-tile allocation failed");
    if (!rc) rc = rt::build_ptr(ctx, st, n, row_ptr, col, cnt, tptr, ntiles, &entries);
    if (cnt) (void)hipFree(cnt);
    int32_t *tcol = nullptr;
    float *v32 = nullptr;
    double *v64 = nullptr;
    if (!rc) {
        const size_t ne = (size_t)std::max<int64_t>(entries, 1);
        tcol = (int32_t *)alloc(1, ne * sizeof(int32_t));
        if (precision != 0) v32 = (float *)alloc(2, ne * 8 * sizeof(float));
        if (precision != 1) v64 = (double *)alloc(3, ne * 8 * sizeof(double));
        if (!tcol || (precision != 0 && !v32) || (precision != 1 && !v64))
            rc = set_error(ctx, FF_ERR_OOM, "row-tile allocation of %lld entries failed", (long long)entries);
    }
    if (!rc) rc = rt::fill(ctx, st, n, ntiles, row_ptr, col, H, M, tptr, tcol, v32, v64);
    if (!rc && hipStreamSynchronize(st) != hipSuccess) rc = set_error(ctx, FF_ERR_HIP, "row-tile build failed");
    if (rc) {
        rowtiles_destroy(h);
        return rc;
    }
    h->v.n = n;
    h->v.ntiles = ntiles;
    h->v.entries = entries;
    h->v.tptr = tptr;
    h->v.tcol = tcol;
    h->v.v32 = v32;
    h->v.v64 = v64;
    *out = h;
    return FF_OK;
}

int rowtiles_info(const ff_rowtiles *rt, int64_t *ntiles, int64_t *entries) {
    if (!rt) return FF_ERR_INVALID_ARG;
    if (ntiles) *ntiles = rt->v.ntiles;
    if (entries) *entries = rt->v.entries;
    return FF_OK;
}

int spmm_rowtiles(ff_ctx *ctx, const ff_rowtiles *rt, int precision, int m, const void *Y, int64_t ld_y, void *HY,
                  void *MY, int64_t ld_out, int sub) {
    if (!ctx || !rt) return FF_ERR_INVALID_ARG;
    FF_REQUIRE(ctx, Y && HY, "required pointer is NULL");
    FF_REQUIRE(ctx, precision == 0 || precision == 1, "precision must be 0 or 1");
    const int vn = precision ? 4 : 2;
    FF_REQUIRE(ctx, m > 0 && m % vn == 0 && m / vn <= 64, "block width %d not supported", m);
    FF_REQUIRE(ctx, ld_y >= m && ld_out >= m && ld_y % vn == 0 && ld_out % vn == 0, "bad leading dimension");
    FF_REQUIRE(ctx, sub >= 0 && sub < rt::kSubs, "launch shape %d out of range", sub);
    FF_HIP(ctx, hipSetDevice(ctx->device));
    if (!MY)
        return precision ? rt::spmm_h32(ctx, ctx->stream, rt->v, sub, m, (const float *)Y, ld_y, (float *)HY, ld_out,
                                        nullptr, nullptr)
                         : rt::spmm_h64(ctx, ctx->stream, rt->v, sub, m, (const double *)Y, ld_y, (double *)HY,
                                        ld_out, nullptr, nullptr);
    if (precision)
        return rt::spmm32(ctx, ctx->stream, rt->v, sub, m, (const float *)Y, ld_y, (float *)HY, (float *)MY, ld_out,
                          nullptr, nullptr);
    return rt::spmm64(ctx, ctx->stream, rt->v, sub, m, (const double *)Y, ld_y, (double *)HY, (double *)MY, ld_out,
                      nullptr, nullptr);
}

void rowtiles_destroy(ff_rowtiles *rt) {
    if (!rt) return;
    (void)hipSetDevice(rt->device);
    (void)hipStreamSynchronize(rt->stream);
    for (void *p : rt->mem)
        if (p) (void)hipFree(p);
    delete rt;
}

}  // extern "C"
