// Matrix-free products with the weight-space Hessian and the mass matrix on gfx950.
//
// Prop. 1 with the quadrature of Supp. C writes H as a sum over integration points,
// H = G^T D G with G the 3q x n matrix of shape-function gradients and D = diag of
// v_i (lambda_i + 4 mu_i) (three times per point), and Eq. (14) writes M = Phi^T V Phi with
// Phi the q x n matrix of shape-function values and V = diag(v_i [rho_i]). So
//   [H Y, M Y] = [G^T (D (G Y)), Phi^T (V (Phi Y))]
// in two passes over the neighbour lists, without the assembled CSR:
//   pass 1 (gather, per integration point i):  UG_i = [v_i (Phi Y)_i, w_i (G Y)_i]  (4 m values)
//   pass 2 (per node k, over the points whose list holds k, in ascending i):
//       (M Y)_k = sum_i phi_k(X_i) u_i,   (H Y)_k = sum_i grad phi_k(X_i) . g_i
// The transposed lists (with each entry's phi and grad phi copied into transposed order, so
// the second pass reads them contiguously) are built once per handle. Both passes give a
// group of Lp lanes to one point or node, a lane per column of Y; the group's list entries
// are loaded a chunk at a time, one per lane, and broadcast within the group with
// ds_bpermute (a group only reads its own lanes, which share its control flow), several
// gathers in flight. Every sum runs in a fixed order (deterministic).
#include "ff_internal.h"

#include <algorithm>

namespace ff {
namespace {

template <typename T> struct MfVals;
template <> struct MfVals<float> { typedef float4 V; };
template <> struct MfVals<double> { typedef double4 V; };

// value (x) and gradient (y, z, w) of one list entry
template <typename T> __device__ inline typename MfVals<T>::V mf_entry(const double *phi, const double *dphi, int64_t e) {
    typename MfVals<T>::V v;
    v.x = (T)phi[e];
    v.y = (T)dphi[3 * e];
    v.z = (T)dphi[3 * e + 1];
    v.w = (T)dphi[3 * e + 2];
    return v;
}

// ---------------------------------------------------------------------------
// build: the transposed lists (shared with the assembly), value copies, weights
// ---------------------------------------------------------------------------

// the transposed entries' point and (phi, grad phi), from the transposed lists (i, slot)
template <typename T>
__global__ void mf_transposed_values_kernel(const int2 *nt, int64_t total, const int64_t *off, const double *phi,
                                            const double *dphi, int32_t *tpt, typename MfVals<T>::V *tval) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= total) return;
    const int2 v = nt[t];
    tpt[t] = v.x;
    tval[t] = mf_entry<T>(phi, dphi, off[v.x] + v.y);
}

template <typename T>
__global__ void mf_values_kernel(int64_t total, const double *phi, const double *dphi, typename MfVals<T>::V *val) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < total) val[e] = mf_entry<T>(phi, dphi, e);
}

// per-point weights: v_i [rho_i] for M, v_i (lambda_i + 4 mu_i) for H (Prop. 1)
template <typename T>
__global__ void mf_weights_kernel(int64_t q, const double *vol, const double *lam, const double *mu,
                                  const double *rho, const int32_t *perm, T *wm, T *wh) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= q) return;
    const int64_t j = perm ? perm[i] : i;
    wh[i] = (T)(vol[j] * (lam[j] + 4.0 * mu[j]));
    wm[i] = (T)(rho ? vol[j] * rho[j] : vol[j]);
}

// ---------------------------------------------------------------------------
// the two passes
// ---------------------------------------------------------------------------

template <typename T>
__device__ inline T bperm(T v, int src_lane) {
    if constexpr (sizeof(T) == 4) {
        return __int_as_float(__builtin_amdgcn_ds_bpermute(src_lane << 2, __float_as_int(v)));
    } else {
        const long long b = __double_as_longlong(v);
        const int lo = __builtin_amdgcn_ds_bpermute(src_lane << 2, (int)(b & 0xffffffff));
        const int hi = __builtin_amdgcn_ds_bpermute(src_lane << 2, (int)(b >> 32));
        return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
    }
}
__device__ inline int bperm_i(int v, int src_lane) { return __builtin_amdgcn_ds_bpermute(src_lane << 2, v); }

// Pass 1. Lane group of kLp lanes per point, lane c of the group owns column c (< m):
//   u = sum_e phi_e Y[id_e][c], g_s = sum_e dphi_e[s] Y[id_e][c];  UG[i] = [wm u, wh g0, wh g1, wh g2]
template <typename T, int kLp>
__global__ void __launch_bounds__(256) mf_pass1_kernel(int64_t q, int m, const int64_t *off, const int32_t *ids,
                                                       const typename MfVals<T>::V *val, const T *wm, const T *wh,
                                                       const T *Y, int64_t ldy, T *UG) {
    const int lane = threadIdx.x & 63, c = lane % kLp, base = lane - c;
    const int64_t i = (((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6) * (64 / kLp) + lane / kLp;
    const bool live = i < q;
    const int64_t e0 = live ? off[i] : 0, e1 = live ? off[i + 1] : 0;
    const bool col = c < m;
    T u = 0, g0 = 0, g1 = 0, g2 = 0;
    // the group's longest remaining chunk decides the wave's trip count; groups past their end idle
    int64_t len = e1 - e0;
    for (int d = kLp; d < 64; d <<= 1) len = std::max<int64_t>(len, __shfl_xor(len, d, 64));
    for (int64_t s = 0; s < len; s += kLp) {
        const int64_t e = e0 + s + c;
        const bool has = e < e1;
        const int id = has ? ids[e] : 0;
        typename MfVals<T>::V v;
        if (has) v = val[e]; else v.x = v.y = v.z = v.w = 0;
        const int cnt = (int)std::min<int64_t>(kLp, std::max<int64_t>(0, e1 - e0 - s));
        int t = 0;
        for (; t + 4 <= cnt; t += 4) {
            T y[4], a[4][4];
            int kk[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) kk[r] = bperm_i(id, base + t + r);
#pragma unroll
            for (int r = 0; r < 4; ++r) y[r] = col ? Y[(int64_t)kk[r] * ldy + c] : (T)0;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                a[r][0] = bperm(v.x, base + t + r);
                a[r][1] = bperm(v.y, base + t + r);
                a[r][2] = bperm(v.z, base + t + r);
                a[r][3] = bperm(v.w, base + t + r);
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                u += a[r][0] * y[r];
                g0 += a[r][1] * y[r];
                g1 += a[r][2] * y[r];
                g2 += a[r][3] * y[r];
            }
        }
        for (; t < cnt; ++t) {
            const int k = bperm_i(id, base + t);
            const T y = col ? Y[(int64_t)k * ldy + c] : (T)0;
            u += bperm(v.x, base + t) * y;
            g0 += bperm(v.y, base + t) * y;
            g1 += bperm(v.z, base + t) * y;
            g2 += bperm(v.w, base + t) * y;
        }
    }
    if (live && col) {
        const T a = wm[i], b = wh[i];
        T *o = UG + (size_t)i * 4 * m;
        o[c] = a * u;
        o[m + c] = b * g0;
        o[2 * m + c] = b * g1;
        o[3 * m + c] = b * g2;
    }
}

// Pass 2: per node k, MY[k][c] = sum phi u_i[c], HY[k][c] = sum grad phi . g_i[c] over the
// transposed entries in ascending point order.
template <typename T, int kLp>
__global__ void __launch_bounds__(256) mf_pass2_kernel(int64_t n, int m, const int64_t *toff, const int32_t *tpt,
                                                       const typename MfVals<T>::V *tval, const T *UG, T *HY, T *MY,
                                                       int64_t ldo) {
    const int lane = threadIdx.x & 63, c = lane % kLp, base = lane - c;
    const int64_t k = (((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6) * (64 / kLp) + lane / kLp;
    const bool live = k < n;
    const int64_t e0 = live ? toff[k] : 0, e1 = live ? toff[k + 1] : 0;
    const bool col = c < m;
    T hy = 0, my = 0;
    int64_t len = e1 - e0;
    for (int d = kLp; d < 64; d <<= 1) len = std::max<int64_t>(len, __shfl_xor(len, d, 64));
    const int64_t m4 = 4 * (int64_t)m;
    for (int64_t s = 0; s < len; s += kLp) {
        const int64_t e = e0 + s + c;
        const bool has = e < e1;
        const int pt = has ? tpt[e] : 0;
        typename MfVals<T>::V v;
        if (has) v = tval[e]; else v.x = v.y = v.z = v.w = 0;
        const int cnt = (int)std::min<int64_t>(kLp, std::max<int64_t>(0, e1 - e0 - s));
        int t = 0;
        for (; t + 2 <= cnt; t += 2) {
            T g[2][4];
            int ii[2];
#pragma unroll
            for (int r = 0; r < 2; ++r) ii[r] = bperm_i(pt, base + t + r);
#pragma unroll
            for (int r = 0; r < 2; ++r) {
                const T *src = UG + (int64_t)ii[r] * m4 + c;
#pragma unroll
                for (int q4 = 0; q4 < 4; ++q4) g[r][q4] = col ? src[q4 * m] : (T)0;
            }
#pragma unroll
            for (int r = 0; r < 2; ++r) {
                my += bperm(v.x, base + t + r) * g[r][0];
                hy += bperm(v.y, base + t + r) * g[r][1];
                hy += bperm(v.z, base + t + r) * g[r][2];
                hy += bperm(v.w, base + t + r) * g[r][3];
            }
        }
        for (; t < cnt; ++t) {
            const int i = bperm_i(pt, base + t);
            const T *src = UG + (int64_t)i * m4 + c;
            const T g0 = col ? src[0] : (T)0, g1 = col ? src[m] : (T)0, g2 = col ? src[2 * m] : (T)0,
                    g3 = col ? src[3 * m] : (T)0;
            my += bperm(v.x, base + t) * g0;
            hy += bperm(v.y, base + t) * g1;
            hy += bperm(v.z, base + t) * g2;
            hy += bperm(v.w, base + t) * g3;
        }
    }
    if (live && col) {
        if (HY) HY[k * ldo + c] = hy;
        if (MY) MY[k * ldo + c] = my;
    }
}

// U[i][c] = sum_e phi_e Y[id_e][c] (the weight field at the integration points, no weights)
template <typename T, int kLp>
__global__ void __launch_bounds__(256) mf_interp_kernel(int64_t q, int m, const int64_t *off, const int32_t *ids,
                                                        const typename MfVals<T>::V *val, const T *Y, int64_t ldy,
                                                        T *U, int64_t ldu) {
    const int lane = threadIdx.x & 63, c = lane % kLp, base = lane - c;
    const int64_t i = (((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6) * (64 / kLp) + lane / kLp;
    const bool live = i < q;
    const int64_t e0 = live ? off[i] : 0, e1 = live ? off[i + 1] : 0;
    const bool col = c < m;
    T u = 0;
    int64_t len = e1 - e0;
    for (int d = kLp; d < 64; d <<= 1) len = std::max<int64_t>(len, __shfl_xor(len, d, 64));
    for (int64_t s = 0; s < len; s += kLp) {
        const int64_t e = e0 + s + c;
        const bool has = e < e1;
        const int id = has ? ids[e] : 0;
        const T p = has ? val[e].x : (T)0;
        const int cnt = (int)std::min<int64_t>(kLp, std::max<int64_t>(0, e1 - e0 - s));
        for (int t = 0; t < cnt; ++t) {
            const int k = bperm_i(id, base + t);
            const T y = col ? Y[(int64_t)k * ldy + c] : (T)0;
            u += bperm(p, base + t) * y;
        }
    }
    if (live && col) U[i * ldu + c] = u;
}

int lanes_for(int m) { return m <= 16 ? 16 : (m <= 32 ? 32 : 64); }

}  // namespace
}  // namespace ff

struct ff_mf {
    ff_ctx *ctx = nullptr;
    int64_t n = 0, q = 0, total = 0;
    int precision = 1;
    const int64_t *off = nullptr;     // the caller's lists (must stay alive and unchanged)
    const int32_t *ids = nullptr;
    void *mem = nullptr;              // one allocation: toff, tpt, val, tval, wm, wh
    int64_t *toff = nullptr;
    int32_t *tpt = nullptr;
    void *val = nullptr, *tval = nullptr, *wm = nullptr, *wh = nullptr;
    void *ug = nullptr;               // pass-1 buffer [q][4][m] (grown on demand)
    size_t ug_bytes = 0;
};

using namespace ff;

extern "C" int mf_build(ff_ctx *ctx, int64_t n, int64_t q, const int64_t *nbr_off, const int32_t *nbr_id,
                        const double *phi, const double *dphi, const double *vol, const double *lam,
                        const double *mu, const double *rho, const int32_t *perm, int precision, ff_mf **out) {
    if (!ctx) return FF_ERR_INVALID_ARG;
    FF_REQUIRE(ctx, out && nbr_off && nbr_id && phi && dphi && vol && lam && mu, "required pointer is NULL");
    FF_REQUIRE(ctx, n > 0 && n < INT32_MAX && q > 0 && q < INT32_MAX, "n or q out of range");
    FF_REQUIRE(ctx, precision == 0 || precision == 1, "precision must be 0 (FP64) or 1 (FP32)");
    *out = nullptr;
    FF_HIP(ctx, hipSetDevice(ctx->device));
    hipStream_t st = ctx->stream;
    int64_t *h = (int64_t *)pinned_get(ctx, 4096);
    if (!h) return FF_ERR_OOM;
    FF_HIP(ctx, hipMemcpyAsync(h, nbr_off + q, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    FF_HIP(ctx, hipStreamSynchronize(st));
    const int64_t total = h[0];
    FF_REQUIRE(ctx, total >= 0 && total < INT32_MAX, "list total %lld out of range", (long long)total);
    const size_t tsz = precision ? sizeof(float) : sizeof(double);
    auto up = [](size_t b) { return (b + 255) & ~(size_t)255; };
    const size_t b_toff = up((size_t)(n + 1) * 8), b_tpt = up((size_t)std::max<int64_t>(total, 1) * 4),
                 b_val = up((size_t)std::max<int64_t>(total, 1) * 4 * tsz), b_w = up((size_t)q * tsz);
    ff_mf *mf = new ff_mf();
    mf->ctx = ctx;
    mf->n = n;
    mf->q = q;
    mf->total = total;
    mf->precision = precision;
    mf->off = nbr_off;
    mf->ids = nbr_id;
    if (hipMalloc(&mf->mem, b_toff + b_tpt + 2 * b_val + 2 * b_w) != hipSuccess) {
        (void)hipGetLastError();
        delete mf;
        return set_error(ctx, FF_ERR_OOM, "matrix-free handle: device allocation failed");
    }
    char *p = (char *)mf->mem;
    mf->toff = (int64_t *)p;
    mf->tpt = (int32_t *)(p + b_toff);
    mf->val = p + b_toff + b_tpt;
    mf->tval = p + b_toff + b_tpt + b_val;
    mf->wm = p + b_toff + b_tpt + 2 * b_val;
    mf->wh = p + b_toff + b_tpt + 2 * b_val + b_w;
    int rc = FF_OK;
    int2 *nt = (int2 *)ws_get(ctx, WS_MF, (size_t)std::max<int64_t>(total, 1) * sizeof(int2));
    if (!nt) rc = FF_ERR_OOM;
    if (!rc) rc = build_transpose(ctx, st, n, q, total, nbr_off, nbr_id, mf->toff, nt, nullptr);
    if (!rc) {
        if (precision) {
            hipLaunchKernelGGL(mf_transposed_values_kernel<float>, dim3(grid_for(total, 256)), dim3(256), 0, st,
                               (const int2 *)nt, total, nbr_off, phi, dphi, mf->tpt, (float4 *)mf->tval);
            hipLaunchKernelGGL(mf_values_kernel<float>, dim3(grid_for(total, 256)), dim3(256), 0, st, total, phi,
                               dphi, (float4 *)mf->val);
            hipLaunchKernelGGL(mf_weights_kernel<float>, dim3(grid_for(q, 256)), dim3(256), 0, st, q, vol, lam, mu,
                               rho, perm, (float *)mf->wm, (float *)mf->wh);
        } else {
            hipLaunchKernelGGL(mf_transposed_values_kernel<double>, dim3(grid_for(total, 256)), dim3(256), 0, st,
                               (const int2 *)nt, total, nbr_off, phi, dphi, mf->tpt, (double4 *)mf->tval);
            hipLaunchKernelGGL(mf_values_kernel<double>, dim3(grid_for(total, 256)), dim3(256), 0, st, total, phi,
                               dphi, (double4 *)mf->val);
            hipLaunchKernelGGL(mf_weights_kernel<double>, dim3(grid_for(q, 256)), dim3(256), 0, st, q, vol, lam, mu,
                               rho, perm, (double *)mf->wm, (double *)mf->wh);
        }
        if (hipGetLastError() != hipSuccess) rc = set_error(ctx, FF_ERR_HIP, "matrix-free build launch failed");
    }
    if (!rc && hipStreamSynchronize(st) != hipSuccess) rc = set_error(ctx, FF_ERR_HIP, "matrix-free build failed");
    if (rc) {
        (void)hipFree(mf->mem);
        delete mf;
        return rc;
    }
    *out = mf;
    return FF_OK;
}

namespace {
template <typename T>
int mf_launch_apply(ff_ctx *ctx, ff_mf *mf, int m, const T *Y, int64_t ldy, T *HY, T *MY, int64_t ldo) {
    hipStream_t st = ctx->stream;
    const size_t need = (size_t)mf->q * 4 * m * sizeof(T);
    if (mf->ug_bytes < need) {
        if (mf->ug) {
            (void)hipStreamSynchronize(st);
            (void)hipFree(mf->ug);
            mf->ug = nullptr;
            mf->ug_bytes = 0;
        }
        if (hipMalloc(&mf->ug, need) != hipSuccess) {
            (void)hipGetLastError();
            return set_error(ctx, FF_ERR_OOM, "matrix-free pass buffer: device allocation failed");
        }
        mf->ug_bytes = need;
    }
    typedef typename MfVals<T>::V V;
    const int lp = lanes_for(m);
    const unsigned g1 = grid_for(mf->q, 4 * (64 / lp)), g2 = grid_for(mf->n, 4 * (64 / lp));
#define FF_MF_LAUNCH(LP)                                                                                         \
    hipLaunchKernelGGL((mf_pass1_kernel<T, LP>), dim3(g1), dim3(256), 0, st, mf->q, m, mf->off, mf->ids,          \
                       (const V *)mf->val, (const T *)mf->wm, (const T *)mf->wh, Y, ldy, (T *)mf->ug);            \
    hipLaunchKernelGGL((mf_pass2_kernel<T, LP>), dim3(g2), dim3(256), 0, st, mf->n, m, (const int64_t *)mf->toff, \
                       (const int32_t *)mf->tpt, (const V *)mf->tval, (const T *)mf->ug, HY, MY, ldo)
    if (lp == 16) {
        FF_MF_LAUNCH(16);
    } else if (lp == 32) {
        FF_MF_LAUNCH(32);
    } else {
        FF_MF_LAUNCH(64);
    }
#undef FF_MF_LAUNCH
    FF_CHECK_LAUNCH(ctx);
    return FF_OK;
}

template <typename T>
int mf_launch_interp(ff_ctx *ctx, const ff_mf *mf, int m, const T *Y, int64_t ldy, T *U, int64_t ldu) {
    typedef typename MfVals<T>::V V;
    const int lp = lanes_for(m);
    const unsigned g1 = grid_for(mf->q, 4 * (64 / lp));
    if (lp == 16)
        hipLaunchKernelGGL((mf_interp_kernel<T, 16>), dim3(g1), dim3(256), 0, ctx->stream, mf->q, m, mf->off, mf->ids,
                           (const V *)mf->val, Y, ldy, U, ldu);
    else if (lp == 32)
        hipLaunchKernelGGL((mf_interp_kernel<T, 32>), dim3(g1), dim3(256), 0, ctx->stream, mf->q, m, mf->off, mf->ids,
                           (const V *)mf->val, Y, ldy, U, ldu);
    else
        hipLaunchKernelGGL((mf_interp_kernel<T, 64>), dim3(g1), dim3(256), 0, ctx->stream, mf->q, m, mf->off, mf->ids,
                           (const V *)mf->val, Y, ldy, U, ldu);
    FF_CHECK_LAUNCH(ctx);
    return FF_OK;
}
}  // namespace

extern "C" int mf_apply(ff_ctx *ctx, ff_mf *mf, int m, const void *Y, int64_t ld_y, void *HY, void *MY,
                        int64_t ld_out) {
    if (!ctx) return FF_ERR_INVALID_ARG;
    FF_REQUIRE(ctx, mf && mf->ctx == ctx, "handle missing or built on another context");
    FF_REQUIRE(ctx, Y && (HY || MY), "Y and at least one of HY, MY are required");
    FF_REQUIRE(ctx, m >= 1 && m <= 64, "block width %d outside [1, 64]", m);
    FF_REQUIRE(ctx, ld_y >= m && (ld_out >= m), "bad leading dimension");
    FF_HIP(ctx, hipSetDevice(ctx->device));
    if (mf->precision)
        return mf_launch_apply<float>(ctx, mf, m, (const float *)Y, ld_y, (float *)HY, (float *)MY, ld_out);
    return mf_launch_apply<double>(ctx, mf, m, (const double *)Y, ld_y, (double *)HY, (double *)MY, ld_out);
}

extern "C" int mf_interpolate(ff_ctx *ctx, const ff_mf *mf, int m, const void *Y, int64_t ld_y, void *U,
                              int64_t ld_u) {
    if (!ctx) return FF_ERR_INVALID_ARG;
    FF_REQUIRE(ctx, mf && mf->ctx == ctx, "handle missing or built on another context");
    FF_REQUIRE(ctx, Y && U, "required pointer is NULL");
    FF_REQUIRE(ctx, m >= 1 && m <= 64 && ld_y >= m && ld_u >= m, "bad block width or leading dimension");
    FF_HIP(ctx, hipSetDevice(ctx->device));
    if (mf->precision)
        return mf_launch_interp<float>(ctx, mf, m, (const float *)Y, ld_y, (float *)U, ld_u);
    return mf_launch_interp<double>(ctx, mf, m, (const double *)Y, ld_y, (double *)U, ld_u);
}

extern "C" void mf_destroy(ff_mf *mf) {
    if (!mf) return;
    if (mf->ctx) {
        (void)hipSetDevice(mf->ctx->device);
        (void)hipStreamSynchronize(mf->ctx->stream);
    }
    if (mf->ug) (void)hipFree(mf->ug);
    if (mf->mem) (void)hipFree(mf->mem);
    delete mf;
}
