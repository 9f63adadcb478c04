// Cell binning (stable counting sort) and neighbour lists on gfx950.
//
// Compiled with -ffp-contract=off: the cell index floor((x - o)/h) and the
// predicate d^2 < h^2 decide integers, so they must be evaluated exactly as
// written (IEEE double subtraction, multiplication and division, no FMA).
#include "ff_internal.h"

namespace ff {
namespace {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanThreads * kScanItems;   // elements per block
constexpr int kMaxCell = 4096;                           // nodes per cell (sort limit)

struct GridDev {
    double o[3];
    double h;
    double hh;
    int64_t d[3];
};

// ---------------------------------------------------------------------------
// block-level scan helpers (wave64)
// ---------------------------------------------------------------------------

__device__ inline int64_t wave_incl_scan(int64_t v) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        int64_t t = __shfl_up(v, d, 64);
        if (lane >= d) v += t;
    }
    return v;
}

// exclusive scan across the block; returns the block total through *total
__device__ inline int64_t block_excl_scan(int64_t v, int64_t *total) {
    __shared__ int64_t wsum[kScanThreads / 64];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    int64_t inc = wave_incl_scan(v);
    if (lane == 63) wsum[wid] = inc;
    __syncthreads();
    int64_t before = 0, tot = 0;
    for (int w = 0; w < kScanThreads / 64; ++w) {
        if (w < wid) before += wsum[w];
        tot += wsum[w];
    }
    __syncthreads();
    *total = tot;
    return before + inc - v;
}

template <typename T>
__global__ void __launch_bounds__(kScanThreads) scan_sums_kernel(const T *in, int64_t len, int64_t *sums) {
    int64_t base = (int64_t)blockIdx.x * kScanTile;
    int64_t s = 0;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        int64_t i = base + threadIdx.x + (int64_t)j * kScanThreads;
        if (i < len) s += (int64_t)in[i];
    }
    int64_t total;
    (void)block_excl_scan(s, &total);
    if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

template <typename T>
__global__ void __launch_bounds__(kScanThreads) scan_apply_kernel(const T *in, int64_t len, const int64_t *offs,
                                                                  int64_t *out) {
    int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int64_t v[kScanItems];
    int64_t local = 0;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        v[j] = (base + j < len) ? (int64_t)in[base + j] : 0;
        local += v[j];
    }
    int64_t total;
    int64_t run = offs[blockIdx.x] + block_excl_scan(local, &total);
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        if (base + j < len) out[base + j] = run;
        run += v[j];
        if (base + j == len - 1) out[len] = run;
    }
}

__global__ void scan_single_kernel(const int64_t *in, int64_t len, int64_t *out) {
    // len <= kScanTile, one block
    int64_t base = (int64_t)threadIdx.x * kScanItems;
    int64_t v[kScanItems];
    int64_t local = 0;
    for (int j = 0; j < kScanItems; ++j) {
        v[j] = (base + j < len) ? in[base + j] : 0;
        local += v[j];
    }
    int64_t total;
    int64_t run = block_excl_scan(local, &total);
    for (int j = 0; j < kScanItems; ++j) {
        if (base + j < len) out[base + j] = run;
        run += v[j];
    }
    if (threadIdx.x == 0) out[len] = total;
}

// Bytes of level storage for a scan of len elements and all its recursive levels.
size_t scan_scratch_bytes(int64_t len) {
    size_t need = 0;
    int64_t l = (len + kScanTile - 1) / kScanTile;
    while (true) {
        need += (size_t)(2 * l + 2) * sizeof(int64_t);
        if (l <= kScanTile) break;
        l = (l + kScanTile - 1) / kScanTile;
    }
    return need;
}

// Each level takes [sums | offs] at the front of its scratch and hands the
// rest to the next level, so no two levels share storage.
template <typename T>
int scan_impl(ff_ctx *ctx, const T *in, int64_t *out, int64_t len, int64_t *scratch) {
    int64_t nb = (len + kScanTile - 1) / kScanTile;
    int64_t *sums = scratch;
    int64_t *offs = sums + nb + 1;
    int64_t *next = offs + nb + 1;
    hipLaunchKernelGGL(scan_sums_kernel<T>, dim3((unsigned)nb), dim3(kScanThreads), 0, ctx->stream, in, len,
                       sums);
    FF_CHECK_LAUNCH(ctx);
    if (nb <= kScanTile) {
        hipLaunchKernelGGL(scan_single_kernel, dim3(1), dim3(kScanThreads), 0, ctx->stream, sums, nb, offs);
        FF_CHECK_LAUNCH(ctx);
    } else {
        int rc = scan_impl<int64_t>(ctx, sums, offs, nb, next);
        if (rc) return rc;
    }
    hipLaunchKernelGGL(scan_apply_kernel<T>, dim3((unsigned)nb), dim3(kScanThreads), 0, ctx->stream, in, len,
                       offs, out);
    FF_CHECK_LAUNCH(ctx);
    return FF_OK;
}

template <typename T>
int scan_top(ff_ctx *ctx, const T *in, int64_t *out, int64_t len) {
    if (len <= 0) {
        FF_HIP(ctx, hipMemsetAsync(out, 0, sizeof(int64_t), ctx->stream));
        return FF_OK;
    }
    int64_t *scratch = (int64_t *)ws_get(ctx, WS_SCAN, scan_scratch_bytes(len) + 256);
    if (!scratch) return FF_ERR_OOM;
    return scan_impl<T>(ctx, in, out, len, scratch);
}

// ---------------------------------------------------------------------------
// bounding box
// ---------------------------------------------------------------------------

constexpr int kBboxBlocks = 256;

__global__ void __launch_bounds__(256) bbox_partial_kernel(const double *xyz, int64_t n, double *part,
                                                           int *nonfinite) {
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    int bad = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        for (int a = 0; a < 3; ++a) {
            double v = xyz[3 * i + a];
            if (!isfinite(v)) bad = 1;
            lo[a] = fmin(lo[a], v);
            hi[a] = fmax(hi[a], v);
        }
    }
    __shared__ double s[6][256];
    for (int a = 0; a < 3; ++a) {
        s[a][threadIdx.x] = lo[a];
        s[3 + a][threadIdx.x] = hi[a];
    }
    if (bad) atomicOr(nonfinite, 1);
    __syncthreads();
    for (int stride = 128; stride > 0; stride >>= 1) {
        if ((int)threadIdx.x < stride)
            for (int a = 0; a < 3; ++a) {
                s[a][threadIdx.x] = fmin(s[a][threadIdx.x], s[a][threadIdx.x + stride]);
                s[3 + a][threadIdx.x] = fmax(s[3 + a][threadIdx.x], s[3 + a][threadIdx.x + stride]);
            }
        __syncthreads();
    }
    if (threadIdx.x < 6) part[blockIdx.x * 6 + threadIdx.x] = s[threadIdx.x][0];
}

__global__ void bbox_final_kernel(const double *part, int nb, double *out) {
    int a = threadIdx.x;
    if (a >= 6) return;
    double v = part[a];
    for (int b = 1; b < nb; ++b) v = (a < 3) ? fmin(v, part[b * 6 + a]) : fmax(v, part[b * 6 + a]);
    out[a] = v;
}

// ---------------------------------------------------------------------------
// binning
// ---------------------------------------------------------------------------

__device__ inline int64_t axis_cell(double x, double o, double h, int64_t D) {
    double t = floor((x - o) / h);
    t = t < 0.0 ? 0.0 : t;
    double top = (double)(D - 1);
    t = t > top ? top : t;
    return (int64_t)t;
}

// Sub-cell index along one axis: the cell split in 4, s = clamp(floor((t - q) * 4), 0, 3)
// with t = (x - o)/h and q the clamped cell coordinate (t - q and the product are exact).
__device__ inline int axis_sub(double x, double o, double h, int64_t D) {
    const double t = (x - o) / h;
    double q = floor(t);
    q = q < 0.0 ? 0.0 : q;
    const double top = (double)(D - 1);
    q = q > top ? top : q;
    double s = floor((t - q) * 4.0);
    s = s < 0.0 ? 0.0 : (s > 3.0 ? 3.0 : s);
    return (int)s;
}

// Cell of each node and the Morton code (x lowest) of its 4x4x4 sub-cell: nodes
// are ordered by cell, then sub-cell, so consecutive rows are spatially compact
// (the SpMM's row tiles share more columns).
__global__ void __launch_bounds__(256) cell_key_kernel(const double *xyz, int64_t n, GridDev g, int32_t *key,
                                                       int32_t *count, int32_t *sub) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int64_t cx = axis_cell(xyz[3 * i + 0], g.o[0], g.h, g.d[0]);
    int64_t cy = axis_cell(xyz[3 * i + 1], g.o[1], g.h, g.d[1]);
    int64_t cz = axis_cell(xyz[3 * i + 2], g.o[2], g.h, g.d[2]);
    int32_t c = (int32_t)((cz * g.d[1] + cy) * g.d[0] + cx);
    key[i] = c;
    const int sx = axis_sub(xyz[3 * i + 0], g.o[0], g.h, g.d[0]);
    const int sy = axis_sub(xyz[3 * i + 1], g.o[1], g.h, g.d[1]);
    const int sz = axis_sub(xyz[3 * i + 2], g.o[2], g.h, g.d[2]);
    int code = 0;
#pragma unroll
    for (int b = 0; b < 2; ++b)
        code |= (((sx >> b) & 1) << (3 * b)) | (((sy >> b) & 1) << (3 * b + 1)) | (((sz >> b) & 1) << (3 * b + 2));
    sub[i] = code;
    atomicAdd(&count[c], 1);
}

// Unordered placement into the cell's slot range; the per-cell sort below
// restores the (cell, sub-cell code, original index) order deterministically.
__global__ void __launch_bounds__(256) cell_scatter_kernel(const int32_t *key, int64_t n, const int64_t *cell_start,
                                                           int32_t *cursor, int32_t *perm) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int32_t c = key[i];
    int64_t pos = cell_start[c] + atomicAdd(&cursor[c], 1);
    perm[pos] = (int32_t)i;
}

__global__ void __launch_bounds__(256) cell_sort_kernel(const int64_t *cell_start, int64_t ncell, int32_t *perm,
                                                        const int32_t *sub, int *too_full) {
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncell) return;
    int64_t a = cell_start[c], b = cell_start[c + 1];
    if (b - a > kMaxCell) {
        atomicOr(too_full, 1);
        return;
    }
    for (int64_t j = a + 1; j < b; ++j) {
        const int32_t v = perm[j];
        const int64_t kv = ((int64_t)sub[v] << 32) | (uint32_t)v;
        int64_t t = j - 1;
        while (t >= a && (((int64_t)sub[perm[t]] << 32) | (uint32_t)perm[t]) > kv) {
            perm[t + 1] = perm[t];
            --t;
        }
        perm[t + 1] = v;
    }
}

__global__ void __launch_bounds__(256) gather_xyz_kernel(const double *xyz, const int32_t *perm, int64_t n,
                                                         double *out) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 3 * n) return;
    int64_t j = t / 3, a = t - 3 * j;
    out[t] = xyz[3 * (int64_t)perm[j] + a];
}

// ---------------------------------------------------------------------------
// neighbour lists: one wavefront per quadrature point, lanes over candidates
// ---------------------------------------------------------------------------

// With rad (support radius per node, original order, read through perm) the predicate is
// d^2 < R_j R_j for sorted node j, else d^2 < h h.
template <bool kFill>
__global__ void __launch_bounds__(256) neighbor_kernel(const double *qxyz, int64_t q, const double *xs, GridDev g,
                                                       const int64_t *cell_start, const int64_t *off,
                                                       int32_t *ids, int32_t *counts, const double *rad,
                                                       const int32_t *perm) {
    const int lane = threadIdx.x & 63;
    const int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    if (i >= q) return;
    const double X0 = qxyz[3 * i], X1 = qxyz[3 * i + 1], X2 = qxyz[3 * i + 2];
    const int64_t cx = axis_cell(X0, g.o[0], g.h, g.d[0]);
    const int64_t cy = axis_cell(X1, g.o[1], g.h, g.d[1]);
    const int64_t cz = axis_cell(X2, g.o[2], g.h, g.d[2]);
    const int64_t x0 = cx > 0 ? cx - 1 : 0;
    const int64_t x1 = cx + 1 < g.d[0] ? cx + 1 : g.d[0] - 1;
    int64_t pos = kFill ? off[i] : 0;
    int64_t cnt = 0;
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    for (int64_t z = cz - 1; z <= cz + 1; ++z) {
        if (z < 0 || z >= g.d[2]) continue;
        for (int64_t y = cy - 1; y <= cy + 1; ++y) {
            if (y < 0 || y >= g.d[1]) continue;
            const int64_t row = (z * g.d[1] + y) * g.d[0];
            const int64_t j0 = cell_start[row + x0], j1 = cell_start[row + x1 + 1];
            for (int64_t base = j0; base < j1; base += 64) {
                const int64_t j = base + lane;
                bool hit = false;
                if (j < j1) {
                    const double dx = X0 - xs[3 * j], dy = X1 - xs[3 * j + 1], dz = X2 - xs[3 * j + 2];
                    const double d2 = ((dx * dx) + (dy * dy)) + (dz * dz);
                    if (rad) {
                        const double Rj = rad[perm[j]];
                        hit = d2 < Rj * Rj;
                    } else {
                        hit = d2 < g.hh;
                    }
                }
                const uint64_t mask = __ballot(hit);
                if (kFill && hit) ids[pos + __popcll(mask & below)] = (int32_t)j;
                pos += __popcll(mask);
                cnt += __popcll(mask);
            }
        }
    }
    if (!kFill && lane == 0) counts[i] = (int32_t)cnt;
}

}  // namespace

int scan_exclusive_i64(ff_ctx *ctx, const int64_t *in, int64_t *out, int64_t len) {
    return scan_top<int64_t>(ctx, in, out, len);
}

int scan_exclusive_i32_to_i64(ff_ctx *ctx, const int32_t *in, int64_t *out, int64_t len) {
    return scan_top<int32_t>(ctx, in, out, len);
}

}  // namespace ff

using namespace ff;

namespace {

// largest radius per block and a flag for a radius that is not finite and positive
__global__ void __launch_bounds__(256) radius_max_kernel(const double *rad, int64_t n, double *part, int *bad) {
    __shared__ double s[256];
    double m = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const double v = rad[i];
        if (!(v > 0.0) || !isfinite(v)) atomicOr(bad, 1);
        m = fmax(m, v);
    }
    s[threadIdx.x] = m;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) s[threadIdx.x] = fmax(s[threadIdx.x], s[threadIdx.x + st]);
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = s[0];
}

int build_impl(ff_ctx *ctx, int64_t n, const double *xyz, int64_t q, const double *qxyz, double h,
               const double *rad, ff_grid *grid, int32_t *perm, double *xyz_sorted, int64_t *cell_start,
               int64_t cell_cap, int64_t *nbr_off, int32_t *nbr_id, int64_t nbr_cap, int64_t *nbr_total);

}  // namespace

extern "C" int build_neighbors(ff_ctx *ctx, int64_t n, const double *xyz, int64_t q, const double *qxyz,
                               double h, ff_grid *grid, int32_t *perm, double *xyz_sorted, int64_t *cell_start,
                               int64_t cell_cap, int64_t *nbr_off, int32_t *nbr_id, int64_t nbr_cap,
                               int64_t *nbr_total) {
    if (!ctx) return FF_ERR_INVALID_ARG;
    return build_impl(ctx, n, xyz, q, qxyz, h, nullptr, grid, perm, xyz_sorted, cell_start, cell_cap, nbr_off,
                      nbr_id, nbr_cap, nbr_total);
}

extern "C" int build_neighbors_radii(ff_ctx *ctx, int64_t n, const double *xyz, const double *radius, int64_t q,
                                     const double *qxyz, ff_grid *grid, int32_t *perm, double *xyz_sorted,
                                     int64_t *cell_start, int64_t cell_cap, int64_t *nbr_off, int32_t *nbr_id,
                                     int64_t nbr_cap, int64_t *nbr_total) {
    if (!ctx) return FF_ERR_INVALID_ARG;
    FF_REQUIRE(ctx, radius != nullptr, "radius is NULL");
    FF_REQUIRE(ctx, n > 0 && n < INT32_MAX, "n = %lld out of range", (long long)n);
    FF_HIP(ctx, hipSetDevice(ctx->device));
    hipStream_t st = ctx->stream;
    constexpr int kBlocks = 256;
    double *part = (double *)ws_get(ctx, WS_RADMAX, kBlocks * sizeof(double) + 64);
    int *flag = (int *)(part ? part + kBlocks : nullptr);
    double *host = (double *)pinned_get(ctx, 4096);
    if (!part || !host) return FF_ERR_OOM;
    FF_HIP(ctx, hipMemsetAsync(flag, 0, sizeof(int), st));
    hipLaunchKernelGGL(radius_max_kernel, dim3(kBlocks), dim3(256), 0, st, radius, n, part, flag);
    FF_CHECK_LAUNCH(ctx);
    FF_HIP(ctx, hipMemcpyAsync(host, part, kBlocks * sizeof(double) + sizeof(int), hipMemcpyDeviceToHost, st));
    FF_HIP(ctx, hipStreamSynchronize(st));
    FF_REQUIRE(ctx, ((const int *)(host + kBlocks))[0] == 0, "a support radius is not finite and positive");
    double h = 0.0;
    for (int b = 0; b < kBlocks; ++b) h = std::max(h, host[b]);
    return build_impl(ctx, n, xyz, q, qxyz, h, radius, grid, perm, xyz_sorted, cell_start, cell_cap, nbr_off,
                      nbr_id, nbr_cap, nbr_total);
}

namespace {

int build_impl(ff_ctx *ctx, int64_t n, const double *xyz, int64_t q, const double *qxyz, double h,
               const double *rad, ff_grid *grid, int32_t *perm, double *xyz_sorted, int64_t *cell_start,
               int64_t cell_cap, int64_t *nbr_off, int32_t *nbr_id, int64_t nbr_cap, int64_t *nbr_total) {
    FF_REQUIRE(ctx, n > 0 && n < INT32_MAX, "n = %lld out of range", (long long)n);
    FF_REQUIRE(ctx, xyz && perm && xyz_sorted && nbr_off && grid && nbr_total, "required pointer is NULL");
    FF_REQUIRE(ctx, std::isfinite(h) && h > 0.0, "support radius h must be finite and positive");
    if (!qxyz) FF_REQUIRE(ctx, q == n, "qxyz == NULL requires q == n");
    FF_REQUIRE(ctx, q > 0 && q < INT32_MAX, "q = %lld out of range", (long long)q);
    FF_HIP(ctx, hipSetDevice(ctx->device));
    hipStream_t st = ctx->stream;

    // 1. bounding box (and a finite-input check)
    double *part = (double *)ws_get(ctx, WS_BBOX, (kBboxBlocks * 6 + 6) * sizeof(double) + 64);
    int *flag = (int *)ws_get(ctx, WS_FLAG, 64);
    double *host = (double *)pinned_get(ctx, 4096);
    if (!part || !flag || !host) return FF_ERR_OOM;
    FF_HIP(ctx, hipMemsetAsync(flag, 0, 64, st));
    hipLaunchKernelGGL(bbox_partial_kernel, dim3(kBboxBlocks), dim3(256), 0, st, xyz, n, part, flag);
    FF_CHECK_LAUNCH(ctx);
    hipLaunchKernelGGL(bbox_final_kernel, dim3(1), dim3(64), 0, st, part, kBboxBlocks, part + kBboxBlocks * 6);
    FF_CHECK_LAUNCH(ctx);
    if (qxyz) {
        // finite check of the quadrature points (box of nodes is what defines the grid)
        hipLaunchKernelGGL(bbox_partial_kernel, dim3(kBboxBlocks), dim3(256), 0, st, qxyz, q, part, flag + 1);
        FF_CHECK_LAUNCH(ctx);
    }
    FF_HIP(ctx, hipMemcpyAsync(host, part + kBboxBlocks * 6, 6 * sizeof(double), hipMemcpyDeviceToHost, st));
    FF_HIP(ctx, hipMemcpyAsync(host + 6, flag, 2 * sizeof(int), hipMemcpyDeviceToHost, st));
    FF_HIP(ctx, hipStreamSynchronize(st));
    const int *hflag = (const int *)(host + 6);
    FF_REQUIRE(ctx, hflag[0] == 0, "non-finite node coordinate");
    FF_REQUIRE(ctx, hflag[1] == 0, "non-finite quadrature point coordinate");

    GridDev g;
    int64_t ncell = 1;
    for (int a = 0; a < 3; ++a) {
        g.o[a] = host[a];
        double span = std::floor((host[3 + a] - host[a]) / h);
        FF_REQUIRE(ctx, span < 2.0e9, "grid too fine: %g cells along axis %d", span, a);
        g.d[a] = (int64_t)span + 1;
        ncell *= g.d[a];
        FF_REQUIRE(ctx, ncell < INT32_MAX, "more than 2^31-1 cells; increase h");
    }
    g.h = h;
    g.hh = h * h;
    for (int a = 0; a < 3; ++a) {
        grid->origin[a] = g.o[a];
        grid->dims[a] = g.d[a];
    }
    grid->h = h;
    grid->n_cells = ncell;

    int64_t *cs = cell_start;
    if (!cs) {
        cs = (int64_t *)ws_get(ctx, WS_CELLS, (size_t)(ncell + 1) * sizeof(int64_t));
        if (!cs) return FF_ERR_OOM;
    } else if (cell_cap < ncell + 1) {
        return set_error(ctx, FF_ERR_CAPACITY, "cell_start needs %lld entries, capacity %lld",
                         (long long)(ncell + 1), (long long)cell_cap);
    }

    // 2. counting sort of the nodes by cell
    int32_t *key = (int32_t *)ws_get(ctx, WS_KEYS, (size_t)n * sizeof(int32_t));
    int32_t *count = (int32_t *)ws_get(ctx, WS_COUNTS, (size_t)(ncell > q ? ncell : q) * sizeof(int32_t));
    int32_t *cursor = (int32_t *)ws_get(ctx, WS_CURSOR, (size_t)ncell * sizeof(int32_t));
    int32_t *sub = (int32_t *)ws_get(ctx, WS_SUBCELL, (size_t)n * sizeof(int32_t));
    if (!key || !count || !cursor || !sub) return FF_ERR_OOM;
    FF_HIP(ctx, hipMemsetAsync(count, 0, (size_t)ncell * sizeof(int32_t), st));
    FF_HIP(ctx, hipMemsetAsync(cursor, 0, (size_t)ncell * sizeof(int32_t), st));
    hipLaunchKernelGGL(cell_key_kernel, dim3(grid_for(n, 256)), dim3(256), 0, st, xyz, n, g, key, count, sub);
    FF_CHECK_LAUNCH(ctx);
    int rc = scan_exclusive_i32_to_i64(ctx, count, cs, ncell);
    if (rc) return rc;
    hipLaunchKernelGGL(cell_scatter_kernel, dim3(grid_for(n, 256)), dim3(256), 0, st, key, n, cs, cursor, perm);
    FF_CHECK_LAUNCH(ctx);
    hipLaunchKernelGGL(cell_sort_kernel, dim3(grid_for(ncell, 256)), dim3(256), 0, st, cs, ncell, perm, sub,
                       flag + 2);
    FF_CHECK_LAUNCH(ctx);
    hipLaunchKernelGGL(gather_xyz_kernel, dim3(grid_for(3 * n, 256)), dim3(256), 0, st, xyz, perm, n, xyz_sorted);
    FF_CHECK_LAUNCH(ctx);

    // 3. neighbour counts, offsets, then the lists
    const double *Q = qxyz ? qxyz : xyz_sorted;
    const unsigned nbq = grid_for(q, 4);   // 4 waves of 64 per block
    hipLaunchKernelGGL(neighbor_kernel<false>, dim3(nbq), dim3(256), 0, st, Q, q, xyz_sorted, g, cs,
                       (const int64_t *)nullptr, (int32_t *)nullptr, count, rad, (const int32_t *)perm);
    FF_CHECK_LAUNCH(ctx);
    rc = scan_exclusive_i32_to_i64(ctx, count, nbr_off, q);
    if (rc) return rc;
    FF_HIP(ctx, hipMemcpyAsync(host, nbr_off + q, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    FF_HIP(ctx, hipMemcpyAsync(host + 1, flag + 2, sizeof(int), hipMemcpyDeviceToHost, st));
    FF_HIP(ctx, hipStreamSynchronize(st));
    int64_t total = ((const int64_t *)host)[0];
    FF_REQUIRE(ctx, ((const int *)(host + 1))[0] == 0, "a cell holds more than %d nodes; decrease h", kMaxCell);
    *nbr_total = total;
    if (!nbr_id) return FF_OK;
    if (nbr_cap < total)
        return set_error(ctx, FF_ERR_CAPACITY, "nbr_id needs %lld entries, capacity %lld", (long long)total,
                         (long long)nbr_cap);
    hipLaunchKernelGGL(neighbor_kernel<true>, dim3(nbq), dim3(256), 0, st, Q, q, xyz_sorted, g, cs, nbr_off,
                       nbr_id, (int32_t *)nullptr, rad, (const int32_t *)perm);
    FF_CHECK_LAUNCH(ctx);
    return FF_OK;
}

}  // namespace
