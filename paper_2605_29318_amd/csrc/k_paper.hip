// The paper's own kernel construction (Supp. B.1, "RKPM construction") on gfx950:
// farthest point sampling of the kernel centres among the integration points, and
// the radius of each centre's Gaussian (the distance that reaches two other centres).
//
// Both decide integers (which point is picked) or feed a predicate (d^2 < R^2) from
// FP64 distances, so the file builds without contraction and every distance is
// d^2 = ((dx*dx) + (dy*dy)) + (dz*dz), dx = a.x - b.x, as in the neighbour search.
#include "ff_internal.h"

namespace ff {
namespace {

constexpr int kFpsThreads = 256;
constexpr int kFpsMaxBlocks = 1024;

__device__ inline double dist2(const double *a, const double *b) {
    const double dx = a[0] - b[0], dy = a[1] - b[1], dz = a[2] - b[2];
    return ((dx * dx) + (dy * dy)) + (dz * dz);
}

// (value, index) with the larger value first and, on equal values, the lower index
struct VI {
    double v;
    int64_t i;
};
__device__ inline VI better(VI a, VI b) {
    return (b.v > a.v || (b.v == a.v && b.i < a.i)) ? b : a;
}

// Block-wide argmax of one (value, index) per thread; every thread gets the result.
__device__ inline VI block_argmax(VI x, double *sv, int64_t *si) {
    const int t = threadIdx.x;
    sv[t] = x.v;
    si[t] = x.i;
    __syncthreads();
    for (int s = kFpsThreads / 2; s > 0; s >>= 1) {
        if (t < s) {
            const VI o = better(VI{sv[t], si[t]}, VI{sv[t + s], si[t + s]});
            sv[t] = o.v;
            si[t] = o.i;
        }
        __syncthreads();
    }
    const VI r{sv[0], si[0]};
    __syncthreads();
    return r;
}

// The pick of the previous step: the argmax over the blocks' partials (every block
// reduces all of them in the same way, so all agree).
__device__ inline int64_t previous_pick(int step, int64_t start, const double *pv, const int64_t *pi, int nb,
                                        double *sv, int64_t *si) {
    if (step == 1) return start;
    VI x{-1.0, INT64_MAX};
    for (int b = threadIdx.x; b < nb; b += kFpsThreads) x = better(x, VI{pv[b], pi[b]});
    return block_argmax(x, sv, si).i;
}

// Step t (1 <= t < K) of farthest point sampling: find the point picked at step t - 1
// (the start at t = 1) and record it, lower each point's squared distance to the chosen
// set by its distance to that pick, and leave each block's largest (value, index) for
// step t + 1. Partials alternate between two buffers by the parity of t.
__global__ void __launch_bounds__(kFpsThreads) fps_step_kernel(const double *xyz, int64_t q, int step, int64_t start,
                                                               double *md, double *pv, int64_t *pi, int nb,
                                                               int32_t *out) {
    __shared__ double sv[kFpsThreads];
    __shared__ int64_t si[kFpsThreads];
    __shared__ double cpos[3];
    const int prev = (step - 1) & 1, cur = step & 1;
    const int64_t c = previous_pick(step, start, pv + (size_t)prev * nb, pi + (size_t)prev * nb, nb, sv, si);
    if (threadIdx.x < 3) cpos[threadIdx.x] = xyz[3 * c + threadIdx.x];
    if (blockIdx.x == 0 && threadIdx.x == 0) out[step - 1] = (int32_t)c;
    __syncthreads();
    VI best{-1.0, INT64_MAX};
    for (int64_t i = (int64_t)blockIdx.x * kFpsThreads + threadIdx.x; i < q; i += (int64_t)nb * kFpsThreads) {
        const double d = dist2(xyz + 3 * i, cpos);
        double m = step == 1 ? INFINITY : md[i];
        if (d < m) m = d;
        md[i] = m;
        best = better(best, VI{m, i});
    }
    const VI r = block_argmax(best, sv, si);
    if (threadIdx.x == 0) {
        pv[(size_t)cur * nb + blockIdx.x] = r.v;
        pi[(size_t)cur * nb + blockIdx.x] = r.i;
    }
}

// the last pick (after step K - 1)
__global__ void __launch_bounds__(kFpsThreads) fps_last_kernel(int K, int64_t start, const double *pv,
                                                               const int64_t *pi, int nb, int32_t *out) {
    __shared__ double sv[kFpsThreads];
    __shared__ int64_t si[kFpsThreads];
    const int prev = (K - 1) & 1;
    const int64_t c = previous_pick(K, start, pv + (size_t)prev * nb, pi + (size_t)prev * nb, nb, sv, si);
    if (threadIdx.x == 0) out[K - 1] = (int32_t)c;
}

// r_k = sqrt of the second smallest squared distance from centre k to the other centres;
// R_k = cut * r_k. Centres are staged through LDS in tiles of 256.
__global__ void __launch_bounds__(256) radii_kernel(const double *c, int64_t K, double cut, double *r, double *R) {
    __shared__ double tile[256 * 3];
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    double me[3] = {0.0, 0.0, 0.0};
    if (k < K)
        for (int a = 0; a < 3; ++a) me[a] = c[3 * k + a];
    double d1 = INFINITY, d2 = INFINITY;
    for (int64_t base = 0; base < K; base += 256) {
        __syncthreads();
        for (int t = threadIdx.x; t < 256 * 3; t += 256) {
            const int64_t e = base * 3 + t;
            tile[t] = e < 3 * K ? c[e] : 0.0;
        }
        __syncthreads();
        if (k < K) {
            const int64_t lim = K - base < 256 ? K - base : 256;
            for (int j = 0; j < lim; ++j) {
                if (base + j == k) continue;
                const double d = dist2(me, tile + 3 * j);
                if (d < d1) {
                    d2 = d1;
                    d1 = d;
                } else if (d < d2) {
                    d2 = d;
                }
            }
        }
    }
    if (k < K) {
        r[k] = sqrt(d2);
        R[k] = cut * r[k];
    }
}

__global__ void gather_centres_kernel(const double *xyz, const int32_t *idx, int K, double *out) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < 3 * K) out[t] = xyz[3 * (int64_t)idx[t / 3] + t % 3];
}

__global__ void nonfinite_kernel(const double *a, int64_t count, int *flag) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        if (!isfinite(a[i])) atomicOr(flag, 1);
}

}  // namespace
}  // namespace ff

using namespace ff;

extern "C" int fps_centers(ff_ctx *ctx, int64_t q, const double *qxyz, int K, int64_t start, int32_t *out_idx,
                           double *out_xyz) {
    if (!ctx) return FF_ERR_INVALID_ARG;
    FF_REQUIRE(ctx, qxyz && out_idx, "required pointer is NULL");
    FF_REQUIRE(ctx, q > 0 && q < INT32_MAX, "q = %lld out of range", (long long)q);
    FF_REQUIRE(ctx, K >= 1 && K <= q, "K = %d must be in [1, q = %lld]", K, (long long)q);
    FF_REQUIRE(ctx, start >= 0 && start < q, "start %lld out of range", (long long)start);
    FF_HIP(ctx, hipSetDevice(ctx->device));
    hipStream_t st = ctx->stream;
    int *flag = (int *)ws_get(ctx, WS_FLAG, 64);
    int *hflag = (int *)pinned_get(ctx, 4096);
    if (!flag || !hflag) return FF_ERR_OOM;
    FF_HIP(ctx, hipMemsetAsync(flag, 0, sizeof(int), st));
    hipLaunchKernelGGL(nonfinite_kernel, dim3(256), dim3(256), 0, st, qxyz, 3 * q, flag);
    FF_CHECK_LAUNCH(ctx);
    FF_HIP(ctx, hipMemcpyAsync(hflag, flag, sizeof(int), hipMemcpyDeviceToHost, st));
    FF_HIP(ctx, hipStreamSynchronize(st));
    FF_REQUIRE(ctx, hflag[0] == 0, "non-finite integration point coordinate");
    const int nb = (int)std::min<int64_t>(kFpsMaxBlocks, (q + kFpsThreads - 1) / kFpsThreads);
    double *md = (double *)ws_get(ctx, WS_FPS, (size_t)q * sizeof(double) + (size_t)2 * nb * 16 + 64);
    if (!md) return FF_ERR_OOM;
    double *pv = md + q;
    int64_t *pi = (int64_t *)(pv + 2 * nb);
    for (int t = 1; t < K; ++t) {
        hipLaunchKernelGGL(fps_step_kernel, dim3(nb), dim3(kFpsThreads), 0, st, qxyz, q, t, start, md, pv, pi, nb,
                           out_idx);
        FF_CHECK_LAUNCH(ctx);
    }
    hipLaunchKernelGGL(fps_last_kernel, dim3(1), dim3(kFpsThreads), 0, st, K, start, pv, pi, nb, out_idx);
    FF_CHECK_LAUNCH(ctx);
    if (out_xyz) {
        hipLaunchKernelGGL(gather_centres_kernel, dim3(grid_for(3 * (int64_t)K, 256)), dim3(256), 0, st, qxyz,
                           (const int32_t *)out_idx, K, out_xyz);
        FF_CHECK_LAUNCH(ctx);
    }
    return FF_OK;
}

extern "C" int kernel_radii(ff_ctx *ctx, int64_t K, const double *centres, double cut, double *r, double *R) {
    if (!ctx) return FF_ERR_INVALID_ARG;
    FF_REQUIRE(ctx, centres && r && R, "required pointer is NULL");
    FF_REQUIRE(ctx, K >= 3 && K < INT32_MAX, "K = %lld: need at least 3 centres", (long long)K);
    FF_REQUIRE(ctx, std::isfinite(cut) && cut > 0.0, "cut must be finite and positive");
    FF_HIP(ctx, hipSetDevice(ctx->device));
    hipLaunchKernelGGL(radii_kernel, dim3(grid_for(K, 256)), dim3(256), 0, ctx->stream, centres, K, cut, r, R);
    FF_CHECK_LAUNCH(ctx);
    return FF_OK;
}
