// [H, M] Y from the upper triangles of H and M (H and M of Prop. 1 and Eq. (14) are symmetric):
// the values of the diagonal and above are stored once, and the strict lower triangle of each
// row keeps only its columns and, per entry (i, j < i), the position of (j, i) in the upper
// arrays, from which the value is read. The product runs one wavefront per row over the row's
// lower entries (ascending column) and then its upper ones, lane groups gathering 16-byte pieces
// of the Y rows and accumulating in FP64; the groups' sums are added by shuffles in a fixed
// order, so every call gives the same result.
#include "ff_internal.h"

struct ff_sym {
    ff_ctx *ctx = nullptr;
    int64_t n = 0, nnz_u = 0, nnz_l = 0;
    int precision = 0;
    bool has_m = false;
    void *mem = nullptr;
    int64_t *uptr = nullptr, *lptr = nullptr;
    int32_t *ucol = nullptr, *lcol = nullptr, *lidx = nullptr;
    void *uh = nullptr, *um = nullptr;
};

namespace ff {
namespace {

// first entry of row r at or right of the diagonal (the CSR rows are sorted)
__device__ inline int64_t diag_pos(const int64_t *row_ptr, const int32_t *col, int64_t r) {
    int64_t lo = row_ptr[r], hi = row_ptr[r + 1];
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (col[mid] < r) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// per row the entries at or right of the diagonal and left of it; *strict_upper gathers the
// entries right of the diagonal (a symmetric pattern has as many as left of it)
__global__ void __launch_bounds__(256) sym_count_kernel(int64_t n, const int64_t *row_ptr, const int32_t *col,
                                                        int64_t *nu, int64_t *nl,
                                                        unsigned long long *strict_upper) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    unsigned long long su = 0;
    if (r < n) {
        const int64_t p = diag_pos(row_ptr, col, r), e1 = row_ptr[r + 1];
        nu[r] = e1 - p;
        nl[r] = p - row_ptr[r];
        su = (unsigned long long)(e1 - p) - ((p < e1 && col[p] == r) ? 1ull : 0ull);
    }
    for (int d = 32; d >= 1; d >>= 1) su += __shfl_xor(su, d, 64);
    if ((threadIdx.x & 63) == 0 && su) atomicAdd(strict_upper, su);
}

// one wavefront per row: the upper part's columns and values, then for each lower entry (r, j)
// the position of r among row j's upper columns (a binary search; not found means the pattern
// is not symmetric)
template <typename T>
__global__ void sym_fill_kernel(int64_t n, const int64_t *row_ptr, const int32_t *col, const double *H,
                                const double *M, const int64_t *uptr, const int64_t *lptr, int32_t *ucol, T *uh,
                                T *um, int32_t *lcol, int32_t *lidx, int *bad) {
    const int64_t r = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (r >= n) return;
    const int64_t e0 = row_ptr[r], e1 = row_ptr[r + 1];
    const int64_t nl = lptr[r + 1] - lptr[r], p = e0 + nl;
    for (int64_t e = p + lane; e < e1; e += 64) {
        const int64_t o = uptr[r] + (e - p);
        ucol[o] = col[e];
        uh[o] = (T)H[e];
        if (M) um[o] = (T)M[e];
    }
    for (int64_t e = e0 + lane; e < p; e += 64) {
        const int32_t j = col[e];
        int64_t lo = uptr[j], hi = uptr[j + 1];
        while (lo < hi) {
            const int64_t mid = (lo + hi) >> 1;
            if (col[row_ptr[j + 1] - (uptr[j + 1] - mid)] < r) lo = mid + 1;
            else hi = mid;
        }
        const bool found = lo < uptr[j + 1] && col[row_ptr[j + 1] - (uptr[j + 1] - lo)] == r;
        if (!found) atomicOr(bad, 1);
        lcol[lptr[r] + (e - e0)] = j;
        lidx[lptr[r] + (e - e0)] = found ? (int32_t)lo : 0;
    }
}

template <typename T> struct SymVec;
template <> struct SymVec<float> {
    typedef float4 V;
    static constexpr int n = 4;
    static __device__ inline double at(const V &v, int q) { return q == 0 ? v.x : q == 1 ? v.y : q == 2 ? v.z : v.w; }
    static __device__ inline void store(float *p, const double *a) {
        *(float4 *)p = make_float4((float)a[0], (float)a[1], (float)a[2], (float)a[3]);
    }
};
template <> struct SymVec<double> {
    typedef double2 V;
    static constexpr int n = 2;
    static __device__ inline double at(const V &v, int q) { return q == 0 ? v.x : v.y; }
    static __device__ inline void store(double *p, const double *a) { *(double2 *)p = make_double2(a[0], a[1]); }
};

// One wavefront per row over the row's entries taken as one list, its lower part (ascending
// column) then its upper part: the wave loads 64 entries at a time (column, and the two values,
// direct for an upper entry, through its mirror's position for a lower one; one entry per lane)
// with the next 64 requested before these are used; lane groups of G = m / VN lanes take the
// chunk's entries g, g + NG, ... from their lanes by cross-lane reads, kBatch gathers of Y rows
// in flight per lane, and accumulate in FP64; the groups are added by shuffles.
template <typename T, bool kM, int kBatch>
__global__ void __launch_bounds__(256) spmm_sym_kernel(int64_t n, int m, const int64_t *uptr, const int32_t *ucol,
                                                       const T *uh, const T *um, const int64_t *lptr,
                                                       const int32_t *lcol, const int32_t *lidx, const T *Y,
                                                       int64_t ldy, T *HY, T *MY, int64_t ldo) {
    typedef SymVec<T> SV;
    typedef typename SV::V V;
    constexpr int VN = SV::n;
    const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (r >= n) return;
    const int lane = threadIdx.x & 63;
    const int G = m / VN, NG = 64 / G;
    const int g = lane / G, c = lane - g * G;
    const int steps = 64 / NG;
    const int64_t l0 = lptr[r], nl = lptr[r + 1] - l0, u0 = uptr[r], len = nl + (uptr[r + 1] - u0);
    // entry t of the row's list: its column and values
    auto fetch = [&](int64_t t, int32_t &j, T &h, T &mm) {
        j = 0;
        h = mm = T(0);
        if (t < nl) {
            j = lcol[l0 + t];
            const int32_t v = lidx[l0 + t];
            h = uh[v];
            if (kM) mm = um[v];
        } else if (t < len) {
            j = ucol[u0 + t - nl];
            h = uh[u0 + t - nl];
            if (kM) mm = um[u0 + t - nl];
        }
    };
    double aH[VN], aM[VN];
#pragma unroll
    for (int q = 0; q < VN; ++q) aH[q] = aM[q] = 0.0;
    int32_t jn;
    T hn, mn;
    fetch(lane, jn, hn, mn);
    for (int64_t base = 0; base < len; base += 64) {
        const int cnt = (int)(len - base < 64 ? len - base : 64);
        const int32_t jc = jn;
        const T hc = hn, mc = mn;
        fetch(base + 64 + lane, jn, hn, mn);
        for (int s0 = 0; s0 < steps; s0 += kBatch) {
            V x[kBatch];
#pragma unroll
            for (int u = 0; u < kBatch; ++u) {
                const int src = (s0 + u) * NG + g;
                const int32_t j = __shfl(jc, src < 64 ? src : 63, 64);
                x[u] = (s0 + u < steps && src < cnt) ? *(const V *)(Y + (int64_t)j * ldy + c * VN) : V{};
            }
#pragma unroll
            for (int u = 0; u < kBatch; ++u) {
                const int src = (s0 + u) * NG + g;
                const int sl = src < 64 ? src : 63;
                const bool ok = (s0 + u < steps) && src < cnt;
                const T hv = __shfl(hc, sl, 64), mv = kM ? __shfl(mc, sl, 64) : T(0);
#pragma unroll
                for (int q = 0; q < VN; ++q) {
                    aH[q] += (double)(ok ? hv : T(0)) * SV::at(x[u], q);
                    if (kM) aM[q] += (double)(ok ? mv : T(0)) * SV::at(x[u], q);
                }
            }
        }
    }
    for (int d = G; d < 64; d <<= 1)
#pragma unroll
        for (int q = 0; q < VN; ++q) {
            aH[q] += __shfl_xor(aH[q], d, 64);
            if (kM) aM[q] += __shfl_xor(aM[q], d, 64);
        }
    if (g == 0) {
        SV::store(HY + r * ldo + c * VN, aH);
        if (kM) SV::store(MY + r * ldo + c * VN, aM);
    }
}

}  // namespace
}  // namespace ff

using namespace ff;

extern "C" int sym_build(ff_ctx *ctx, int64_t n, const int64_t *row_ptr, const int32_t *col, const double *H,
                         const double *M, int precision, ff_sym **out) {
    if (!ctx) return FF_ERR_INVALID_ARG;
    FF_REQUIRE(ctx, out && row_ptr && col && H, "required pointer is NULL");
    FF_REQUIRE(ctx, n > 0 && n < INT32_MAX, "n out of range");
    FF_REQUIRE(ctx, precision == 0 || precision == 1, "precision must be 0 (FP64) or 1 (FP32)");
    *out = nullptr;
    FF_HIP(ctx, hipSetDevice(ctx->device));
    hipStream_t st = ctx->stream;
    int64_t *cnt = (int64_t *)ws_get(ctx, WS_SYM, (size_t)(2 * n + 2) * sizeof(int64_t));
    int *flag = (int *)ws_get(ctx, WS_FLAG, 64);
    int64_t *h = (int64_t *)pinned_get(ctx, 4096);
    if (!cnt || !flag || !h) return FF_ERR_OOM;
    int64_t *nu = cnt, *nl = cnt + n + 1;
    unsigned long long *su = (unsigned long long *)(flag + 2);
    FF_HIP(ctx, hipMemsetAsync(flag, 0, 64, st));
    hipLaunchKernelGGL(sym_count_kernel, dim3(grid_for(n, 256)), dim3(256), 0, st, n, row_ptr, col, nu, nl, su);
    FF_CHECK_LAUNCH(ctx);
    const size_t tsz = precision ? sizeof(float) : sizeof(double);
    auto up = [](size_t b) { return (b + 255) & ~(size_t)255; };
    ff_sym *s = new ff_sym();
    s->ctx = ctx;
    s->n = n;
    s->precision = precision;
    s->has_m = M != nullptr;
    // offsets first (their totals size the rest)
    const size_t b_ptr = up((size_t)(n + 1) * 8);
    int64_t *ptrs = nullptr;
    if (hipMalloc((void **)&ptrs, 2 * b_ptr) != hipSuccess) {
        (void)hipGetLastError();
        delete s;
        return set_error(ctx, FF_ERR_OOM, "symmetric copy: device allocation failed");
    }
    int64_t *uptr = ptrs, *lptr = (int64_t *)((char *)ptrs + b_ptr);
    int rc = scan_exclusive_i64(ctx, nu, uptr, n);
    if (!rc) rc = scan_exclusive_i64(ctx, nl, lptr, n);
    if (!rc) {
        if (hipMemcpyAsync(h, uptr + n, 8, hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipMemcpyAsync(h + 1, lptr + n, 8, hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipMemcpyAsync(h + 3, su, 8, hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess)
            rc = set_error(ctx, FF_ERR_HIP, "symmetric copy: count failed");
    }
    // every lower entry finds its mirror below (checked by the fill), and there are as many
    // entries right of the diagonal as left of it: then the pattern is symmetric
    if (!rc && h[3] != h[1])
        rc = set_error(ctx, FF_ERR_INVALID_ARG, "symmetric copy: the sparsity pattern is not symmetric");
    if (!rc && (h[0] >= INT32_MAX || h[1] >= INT32_MAX))
        rc = set_error(ctx, FF_ERR_INVALID_ARG, "symmetric copy: %lld upper entries exceed 32-bit positions",
                       (long long)h[0]);
    if (!rc) {
        s->nnz_u = h[0];
        s->nnz_l = h[1];
        const size_t b_uc = up((size_t)std::max<int64_t>(s->nnz_u, 1) * 4), b_uv = up((size_t)std::max<int64_t>(s->nnz_u, 1) * tsz),
                     b_l = up((size_t)std::max<int64_t>(s->nnz_l, 1) * 4);
        if (hipMalloc(&s->mem, b_uc + (s->has_m ? 2 : 1) * b_uv + 2 * b_l) != hipSuccess) {
            (void)hipGetLastError();
            rc = set_error(ctx, FF_ERR_OOM, "symmetric copy: device allocation failed");
        } else {
            char *p = (char *)s->mem;
            s->ucol = (int32_t *)p;
            s->uh = p + b_uc;
            s->um = s->has_m ? p + b_uc + b_uv : nullptr;
            s->lcol = (int32_t *)(p + b_uc + (s->has_m ? 2 : 1) * b_uv);
            s->lidx = (int32_t *)(p + b_uc + (s->has_m ? 2 : 1) * b_uv + b_l);
        }
    }
    s->uptr = uptr;
    s->lptr = lptr;
    if (!rc) {
        if (precision)
            hipLaunchKernelGGL(sym_fill_kernel<float>, dim3(grid_for(n, 4)), dim3(256), 0, st, n, row_ptr, col, H, M,
                               (const int64_t *)uptr, (const int64_t *)lptr, s->ucol, (float *)s->uh, (float *)s->um,
                               s->lcol, s->lidx, flag);
        else
            hipLaunchKernelGGL(sym_fill_kernel<double>, dim3(grid_for(n, 4)), dim3(256), 0, st, n, row_ptr, col, H,
                               M, (const int64_t *)uptr, (const int64_t *)lptr, s->ucol, (double *)s->uh,
                               (double *)s->um, s->lcol, s->lidx, flag);
        if (hipGetLastError() != hipSuccess) rc = set_error(ctx, FF_ERR_HIP, "symmetric copy: fill launch failed");
        int *hf = (int *)(h + 2);
        if (!rc && (hipMemcpyAsync(hf, flag, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess ||
                    hipStreamSynchronize(st) != hipSuccess))
            rc = set_error(ctx, FF_ERR_HIP, "symmetric copy: fill failed");
        if (!rc && hf[0])
            rc = set_error(ctx, FF_ERR_INVALID_ARG, "symmetric copy: the sparsity pattern is not symmetric");
    }
    if (rc) {
        (void)hipFree(s->mem);
        (void)hipFree(ptrs);
        delete s;
        return rc;
    }
    *out = s;
    return FF_OK;
}

extern "C" int sym_info(const ff_sym *s, int64_t *nnz_upper, int64_t *nnz_lower) {
    if (!s) return FF_ERR_INVALID_ARG;
    if (nnz_upper) *nnz_upper = s->nnz_u;
    if (nnz_lower) *nnz_lower = s->nnz_l;
    return FF_OK;
}

extern "C" int spmm_sym(ff_ctx *ctx, const ff_sym *s, int m, const void *Y, int64_t ld_y, void *HY, void *MY,
                        int64_t ld_out) {
    if (!ctx) return FF_ERR_INVALID_ARG;
    FF_REQUIRE(ctx, s && Y && HY, "required pointer is NULL");
    FF_REQUIRE(ctx, !MY || s->has_m, "MY requested from a copy built without M");
    FF_REQUIRE(ctx, m == 8 || m == 16 || m == 32 || m == 64, "block width %d must be 8, 16, 32 or 64", m);
    const int vn = s->precision ? 4 : 2;
    FF_REQUIRE(ctx, ld_y >= m && ld_out >= m && ld_y % vn == 0 && ld_out % vn == 0,
               "leading dimensions must be >= m and multiples of %d", vn);
    FF_REQUIRE(ctx, (uintptr_t)Y % 16 == 0 && (uintptr_t)HY % 16 == 0 && (uintptr_t)MY % 16 == 0,
               "Y, HY and MY must be 16-byte aligned");
    FF_HIP(ctx, hipSetDevice(ctx->device));
    hipStream_t st = ctx->stream;
    const dim3 grid(grid_for(s->n, 4)), block(256);
#define FF_SYM(T, KM)                                                                                              \
    hipLaunchKernelGGL((spmm_sym_kernel<T, KM, 8>), grid, block, 0, st, s->n, m, (const int64_t *)s->uptr,        \
                       (const int32_t *)s->ucol, (const T *)s->uh, (const T *)s->um, (const int64_t *)s->lptr,     \
                       (const int32_t *)s->lcol, (const int32_t *)s->lidx, (const T *)Y, ld_y, (T *)HY, (T *)MY, \
                       ld_out)
    if (s->precision) {
        if (MY) FF_SYM(float, true);
        else FF_SYM(float, false);
    } else {
        if (MY) FF_SYM(double, true);
        else FF_SYM(double, false);
    }
#undef FF_SYM
    FF_CHECK_LAUNCH(ctx);
    return FF_OK;
}

extern "C" void sym_destroy(ff_sym *s) {
    if (!s) return;
    (void)hipFree(s->mem);
    (void)hipFree(s->uptr);
    delete s;
}
