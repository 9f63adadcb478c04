// Row-tile SpMM: tiles of four consecutive rows share one merged column list.
#include "k_rowtile.h"

#include <climits>
#include <cmath>
#include <cstring>

struct ff_rowtiles {
    int device = 0;
    hipStream_t stream = nullptr;                  // the context's stream, kept for destruction
    int hrows = 0;                                 // 8 or 16: an H-only copy in tiles of that many rows
    ff::rt::RTView v;
    ff::rt::RT8View v8;
    ff::rt::RT16View v16;
    ff::rt::RTQView vq;                            // K-blocked binary16 copy (precision 6)
    void *mem[9] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
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

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));

template <int R> struct Merge {
    int64_t p[R], e[R];
    int32_t h[R];
};

template <int R>
__device__ inline void merge_init(Merge<R> &s, int64_t nrows, int64_t r0, const int64_t *row_ptr, const int32_t *col) {
#pragma unroll
    for (int i = 0; i < R; ++i) {
        const bool in = r0 + i < nrows;
        s.p[i] = in ? row_ptr[r0 + i] : 0;
        s.e[i] = in ? row_ptr[r0 + i + 1] : 0;
        s.h[i] = s.p[i] < s.e[i] ? col[s.p[i]] : INT_MAX;
    }
}
template <int R>
__device__ inline int32_t merge_head(const Merge<R> &s) {
    int32_t c = s.h[0];
#pragma unroll
    for (int i = 1; i < R; ++i) c = min(c, s.h[i]);
    return c;
}

template <int R>
__device__ int64_t merge_count(int64_t nrows, int64_t t, const int64_t *row_ptr, const int32_t *col) {
    Merge<R> s;
    merge_init(s, nrows, t * R, row_ptr, col);
    int64_t k = 0;
    for (int32_t cur = merge_head(s); cur != INT_MAX; cur = merge_head(s)) {
        ++k;
#pragma unroll
        for (int i = 0; i < R; ++i)
            if (s.h[i] == cur) {
                ++s.p[i];
                s.h[i] = s.p[i] < s.e[i] ? col[s.p[i]] : INT_MAX;
            }
    }
    return k;
}

// FP32 copy of tile t in tiles of R rows: vh[entry][R] (H) and, when vm is given, vm[entry][R] (M)
template <int R>
__device__ void merge_fill(int64_t nrows, int64_t t, const int64_t *row_ptr, const int32_t *col, const double *H,
                           const double *M, const int64_t *tptr, int32_t *tcol, float *vh, float *vm) {
    Merge<R> s;
    merge_init(s, nrows, t * R, row_ptr, col);
    int64_t o = tptr[t];
    for (int32_t cur = merge_head(s); cur != INT_MAX; cur = merge_head(s), ++o) {
        tcol[o] = cur;
        float *v = vh + o * R;
#pragma unroll
        for (int i = 0; i < R; ++i) {
            const bool hit = s.h[i] == cur;
            v[i] = hit ? (float)H[s.p[i]] : 0.f;
            if (vm) vm[o * R + i] = hit ? (float)M[s.p[i]] : 0.f;
            if (hit) {
                ++s.p[i];
                s.h[i] = s.p[i] < s.e[i] ? col[s.p[i]] : INT_MAX;
            }
        }
    }
}

template <int R>
__global__ void rt_count_kernel(int64_t nrows, int64_t ntiles, const int64_t *row_ptr, const int32_t *col,
                                int64_t *cnt) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ntiles) return;
    cnt[t] = merge_count<R>(nrows, t, row_ptr, col);
}

// ---------------------------------------------------------------------------
// building the eight- and sixteen-row copies: one workgroup per tile
// ---------------------------------------------------------------------------
//
// A tile's union holds each column of its rows once. The entry (row r, column c) represents c
// in the union when no earlier row of the tile holds c. With G the exclusive prefix count of
// representatives over the tile's entries in row order, c's union slot is the number of
// representatives with a smaller column: the sum over rows q of G[start q + lower_bound(q, c)]
// - G[start q]. Each representative writes its slot, the column and the R values (zero where a
// row lacks it), so every slot is written once and the copy equals the serial merge's. The
// column lists sit in LDS (cap entries per tile); a larger tile takes the serial merge.
//
// The common case is faster still: a tile's columns lie in the range [cmin, cmax] of its rows' first
// and last columns (its rows' two-hop neighbourhood, 2.6e3 words of 32 columns at the median on the
// benchmark's clouds), so a bitmap of that range in LDS marks the union and a prefix popcount over
// its words gives every column's slot directly. The tile's value block is then cleared and every
// entry writes its own value into its slot and row (each slot's column is written by each of its
// entries, the same value). Tiles whose range exceeds the bitmap take the path above.
constexpr int kUnionCap = 6144;                   // entries per tile held in LDS (49 KB with G)
constexpr int kUnionThreads = 256;
constexpr int kUnionBitWords = 4096;              // bitmap words (32 KB with their prefix)

// mx[0]: the largest entry count of a tile, mx[1]: the largest bitmap of a tile's column range in words
template <int R>
__global__ void tile_entries_max_kernel(int64_t nrows, int64_t ntiles, const int64_t *row_ptr, const int32_t *col,
                                        int *mx) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int v = 0, words = 0;
    if (t < ntiles) {
        const int64_t r1 = (t + 1) * R < nrows ? (t + 1) * R : nrows;
        const int64_t e = row_ptr[r1] - row_ptr[t * R];
        v = e < INT_MAX ? (int)e : INT_MAX;
        int32_t lo = INT_MAX, hi = -1;
        for (int64_t r = t * R; r < r1; ++r)
            if (row_ptr[r + 1] > row_ptr[r]) {
                lo = min(lo, col[row_ptr[r]]);
                hi = max(hi, col[row_ptr[r + 1] - 1]);
            }
        if (hi >= lo) words = (int)(((int64_t)hi - lo) / 32 + 1);
    }
    for (int d = 32; d >= 1; d >>= 1) {
        v = max(v, __shfl_xor(v, d, 64));
        words = max(words, __shfl_xor(words, d, 64));
    }
    if ((threadIdx.x & 63) == 0) {
        atomicMax(mx, v);
        atomicMax(mx + 1, words);
    }
}

__device__ inline int lower_bound_lds(const int32_t *a, int len, int32_t c) {
    int lo = 0, hi = len;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (a[mid] < c)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

template <int R, bool kFill>
__global__ void __launch_bounds__(kUnionThreads) tile_union_kernel(int64_t nrows, int64_t ntiles,
                                                                   const int64_t *row_ptr, const int32_t *col,
                                                                   int cap, int bits, int64_t *cnt,
                                                                   const double *H, const double *M,
                                                                   const int64_t *tptr, int32_t *tcol, float *vh,
                                                                   float *vm) {
    extern __shared__ __align__(16) int32_t lds[];
    int32_t *lcol = lds;                           // [cap] the rows' columns, row after row
    int32_t *G = lds + cap;                        // [cap + 1] representative flags, then their prefix
    __shared__ int rs[R + 1];                      // row starts in lcol
    __shared__ int64_t gs[R];                      // row starts in the CSR
    __shared__ int wsum[kUnionThreads / 64];
    __shared__ int32_t crange[2];                  // first and last column of the tile
    const int64_t t = blockIdx.x;
    if (t >= ntiles) return;
    const int tid = threadIdx.x;
    const int64_t r0 = t * R;
    if (tid < 64) {                                // lane r reads row r's range and end columns at once
        const bool in = tid < R && r0 + tid < nrows;
        const int64_t b = in ? row_ptr[r0 + tid] : 0, e = in ? row_ptr[r0 + tid + 1] : 0;
        const int len = (int)(e - b);
        int32_t lo = INT_MAX, hi = -1;
        if (e > b) {
            lo = col[b];
            hi = col[e - 1];
        }
        int incl = len;                            // row starts: inclusive scan over the R lanes
        for (int d = 1; d < R; d <<= 1) {
            const int u = __shfl_up(incl, d, 64);
            if (tid >= d) incl += u;
        }
        for (int d = 1; d < 64; d <<= 1) {
            lo = min(lo, __shfl_xor(lo, d, 64));
            hi = max(hi, __shfl_xor(hi, d, 64));
        }
        if (tid < R) {
            gs[tid] = b;
            rs[tid] = incl - len;
        }
        if (tid == R - 1) rs[R] = incl;
        if (tid == 0) {
            crange[0] = lo;
            crange[1] = hi;
        }
    }
    __syncthreads();
    const int E = rs[R];
    auto row_of = [&](int x) {
        int r = 0;
        while (r + 1 < R && rs[r + 1] <= x) ++r;
        return r;
    };
    const int32_t cmin = crange[0];
    const int nw = E > 0 ? (int)(((int64_t)crange[1] - cmin) / 32 + 1) : 0;
    if (nw <= bits) {
        uint32_t *bm = (uint32_t *)lds;            // [bits] the union's columns, relative to cmin
        int32_t *pre = lds + bits;                 // [bits] set bits in the words before
        for (int w = tid; w < nw; w += kUnionThreads) bm[w] = 0u;
        __syncthreads();
        // four entries per thread per pass, their columns loaded before any is used (an index past
        // E reads entry E - 1 and marks nothing)
        for (int x0 = tid; x0 < E; x0 += 4 * kUnionThreads) {
            int32_t c[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int x = min(x0 + u * kUnionThreads, E - 1);
                const int r = row_of(x);
                c[u] = col[gs[r] + (x - rs[r])];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
                if (x0 + u * kUnionThreads < E) {
                    const int b = c[u] - cmin;
                    atomicOr(&bm[b >> 5], 1u << (b & 31));
                }
        }
        __syncthreads();
        const int per = (nw + kUnionThreads - 1) / kUnionThreads;
        const int w0 = min(nw, tid * per), w1 = min(nw, w0 + per);
        int local = 0;
        for (int w = w0; w < w1; ++w) local += __popc(bm[w]);
        const int lane = tid & 63, wv = tid >> 6;
        int incl = local;
        for (int d = 1; d < 64; d <<= 1) {
            const int u = __shfl_up(incl, d, 64);
            if (lane >= d) incl += u;
        }
        if (lane == 63) wsum[wv] = incl;
        __syncthreads();
        int run = incl - local, U = 0;
        for (int w = 0; w < kUnionThreads / 64; ++w) {
            if (w < wv) run += wsum[w];
            U += wsum[w];
        }
        for (int w = w0; w < w1; ++w) {
            pre[w] = run;
            run += __popc(bm[w]);
        }
        if (!kFill) {
            if (tid == 0) cnt[t] = U;
            return;
        }
        const int64_t o = tptr[t];
        // clear the tile's values, then every entry writes its own; the barrier orders the two
        for (int i = tid; i < U * R / 4; i += kUnionThreads) {
            *(f32x4 *)(vh + o * R + 4 * i) = f32x4{0.f, 0.f, 0.f, 0.f};
            if (vm) *(f32x4 *)(vm + o * R + 4 * i) = f32x4{0.f, 0.f, 0.f, 0.f};
        }
        __syncthreads();
        for (int x0 = tid; x0 < E; x0 += 4 * kUnionThreads) {   // as above: loads first
            int32_t c[4];
            double hv[4], mv[4];
            int rr[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int x = min(x0 + u * kUnionThreads, E - 1);
                rr[u] = row_of(x);
                const int64_t g = gs[rr[u]] + (x - rs[rr[u]]);
                c[u] = col[g];
                hv[u] = H[g];
                mv[u] = vm ? M[g] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
                if (x0 + u * kUnionThreads < E) {
                    const int b = c[u] - cmin;
                    const int rank = pre[b >> 5] + __popc(bm[b >> 5] & ((1u << (b & 31)) - 1u));
                    tcol[o + rank] = c[u];
                    vh[(o + rank) * R + rr[u]] = (float)hv[u];
                    if (vm) vm[(o + rank) * R + rr[u]] = (float)mv[u];
                }
        }
        return;
    }
    if (E > cap) {
        if (tid == 0) {
            if (kFill)
                merge_fill<R>(nrows, t, row_ptr, col, H, M, tptr, tcol, vh, vm);
            else
                cnt[t] = merge_count<R>(nrows, t, row_ptr, col);
        }
        return;
    }
    for (int x = tid; x < E; x += kUnionThreads) {
        const int r = row_of(x);
        lcol[x] = col[gs[r] + (x - rs[r])];
    }
    __syncthreads();
    // representatives over a contiguous chunk per thread, then a workgroup-wide exclusive scan
    const int per = (E + kUnionThreads - 1) / kUnionThreads;
    const int x0 = min(E, tid * per), x1 = min(E, x0 + per);
    int local = 0;
    for (int x = x0, r = x0 < E ? row_of(x0) : 0; x < x1; ++x) {
        while (x >= rs[r + 1]) ++r;
        const int32_t c = lcol[x];
        bool rep = true;
        for (int q = 0; q < r && rep; ++q) {
            const int len = rs[q + 1] - rs[q];
            const int lb = lower_bound_lds(lcol + rs[q], len, c);
            rep = !(lb < len && lcol[rs[q] + lb] == c);
        }
        G[x] = rep ? 1 : 0;
        local += rep ? 1 : 0;
    }
    const int lane = tid & 63, wv = tid >> 6;
    int incl = local;
    for (int d = 1; d < 64; d <<= 1) {
        const int u = __shfl_up(incl, d, 64);
        if (lane >= d) incl += u;
    }
    if (lane == 63) wsum[wv] = incl;
    __syncthreads();
    int run = incl - local, U = 0;
    for (int w = 0; w < kUnionThreads / 64; ++w) {
        if (w < wv) run += wsum[w];
        U += wsum[w];
    }
    for (int x = x0; x < x1; ++x) {
        const int f = G[x];
        G[x] = run;
        run += f;
    }
    if (tid == 0) G[E] = U;
    __syncthreads();
    if (!kFill) {
        if (tid == 0) cnt[t] = U;
        return;
    }
    const int64_t o = tptr[t];
    for (int x = tid; x < E; x += kUnionThreads) {
        if (G[x + 1] == G[x]) continue;            // not a representative
        const int r = row_of(x);
        const int32_t c = lcol[x];
        int rank = G[x] - G[rs[r]];
        float v[R], w[R];
#pragma unroll
        for (int q = 0; q < R; ++q) {
            const int len = rs[q + 1] - rs[q];
            int lb;
            if (q == r) {
                lb = x - rs[r];
            } else {
                lb = lower_bound_lds(lcol + rs[q], len, c);
                rank += G[rs[q] + lb] - G[rs[q]];
            }
            const bool hit = lb < len && lcol[rs[q] + lb] == c;
            v[q] = hit ? (float)H[gs[q] + lb] : 0.f;
            w[q] = hit && vm ? (float)M[gs[q] + lb] : 0.f;
        }
        tcol[o + rank] = c;
#pragma unroll
        for (int q = 0; q < R; q += 4) {
            *(f32x4 *)(vh + (o + rank) * R + q) = f32x4{v[q], v[q + 1], v[q + 2], v[q + 3]};
            if (vm) *(f32x4 *)(vm + (o + rank) * R + q) = f32x4{w[q], w[q + 1], w[q + 2], w[q + 3]};
        }
    }
}

template <typename T>
__global__ void rt_fill_kernel(int64_t nrows, int64_t ntiles, const int64_t *row_ptr, const int32_t *col,
                               const double *H, const double *M, const int64_t *tptr, int32_t *tcol, T *tval,
                               int64_t entries, int write_col) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ntiles) return;
    Merge<kTileRows> s;
    merge_init(s, nrows, t * kTileRows, row_ptr, col);
    int64_t o = tptr[t];
    for (int32_t cur = merge_head(s); cur != INT_MAX; cur = merge_head(s), ++o) {
        if (write_col) tcol[o] = cur;
        T *vh = tval + o * 4, *vm = tval + (entries + o) * 4;
#pragma unroll
        for (int i = 0; i < kTileRows; ++i) {
            const bool hit = s.h[i] == cur;
            vh[i] = hit ? (T)H[s.p[i]] : (T)0;
            vm[i] = hit ? (T)M[s.p[i]] : (T)0;
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
__device__ inline float vget(const float4 &v, int q) { return q == 0 ? v.x : q == 1 ? v.y : q == 2 ? v.z : v.w; }
__device__ inline double vget(const double2 &v, int q) { return q == 0 ? v.x : v.y; }
__device__ inline void vset(float4 &v, int q, float x) {
    if (q == 0) v.x = x; else if (q == 1) v.y = x; else if (q == 2) v.z = x; else v.w = x;
}
__device__ inline void vset(double2 &v, int q, double x) {
    if (q == 0) v.x = x; else v.y = x;
}

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


// Chunk of 64 union entries: column and the eight values of entry l in lane l.
// With kHM false only the H values are loaded and staged (stride 4 in LDS).
template <typename T, bool kHM> struct Chunk;
template <bool kHM> struct Chunk<float, kHM> {
    int32_t j;
    f32x4 a, b;                                    // H rows 0..3, M rows 0..3
    __device__ void load(const int32_t *tcol, const float *th, const float *tm, int64_t e, bool in) {
        j = 0;
        a = b = f32x4{0.f, 0.f, 0.f, 0.f};
        if (in) {
            j = __builtin_nontemporal_load(tcol + e);
            a = __builtin_nontemporal_load((const f32x4 *)(th + e * 4));
            if (kHM) b = __builtin_nontemporal_load((const f32x4 *)(tm + e * 4));
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
    __device__ void load(const int32_t *tcol, const double *th, const double *tm, int64_t e, bool in) {
        j = 0;
#pragma unroll
        for (int q = 0; q < NQ; ++q) v[q] = f64x2{0.0, 0.0};
        if (in) {
            j = __builtin_nontemporal_load(tcol + e);
#pragma unroll
            for (int q = 0; q < NQ; ++q)
                v[q] = __builtin_nontemporal_load((const f64x2 *)((q < 2 ? th : tm) + e * 4 + 2 * (q & 1)));
        }
    }
    __device__ void stage(double *sv, int lane) const {
#pragma unroll
        for (int q = 0; q < NQ; ++q) *(f64x2 *)(sv + lane * 2 * NQ + 2 * q) = v[q];
    }
};

// One 64-entry chunk of a tile: stage its values in LDS, request the chunk
// kAhead chunks ahead into the same registers, then gather and accumulate.
template <typename T, typename A, bool kHM, int kBatch, int kAhead>
__device__ __forceinline__ void rt_chunk(Chunk<T, kHM> &ch, int64_t base, int64_t e1, const int32_t *tcol,
                                         const T *tval_h, const T *tval_m, T *sv, int lane, bool on, int g, int c,
                                         int NG, int steps, const T *Y, int64_t ldy, Acc4<A> (&aH)[kTileRows],
                                         Acc4<A> (&aM)[kHM ? kTileRows : 1]) {
    typedef typename Vec<T>::type V;
    constexpr int VN = Vec<T>::n;
    constexpr int NV = kHM ? 8 : 4;
    const int cnt = (int)(e1 - base < 64 ? e1 - base : 64);
    const int32_t jc = ch.j;
    __builtin_amdgcn_wave_barrier();
    ch.stage(sv, lane);
    __builtin_amdgcn_wave_barrier();
    ch.load(tcol, tval_h, tval_m, base + 64 * kAhead + lane, base + 64 * kAhead + lane < e1);
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

// One wavefront per tile. The wave reads 64 union entries (column and eight
// values) with one coalesced load per lane, keeps the next chunk of 64 (two
// in the H-only form) in flight while it works on one, keeps the values in a wave-private LDS area (each lane group
// reads its entry's values as a broadcast) and hands each column to the lane
// group that needs it by a cross-lane shuffle. Lanes form groups of
// G = m / VN; group g takes entries g, g + NG, ... of the chunk; each lane holds
// VN columns of the gathered row of Y and accumulates all four rows of the tile
// in FP64; the groups are summed at the end. With kHM false the kernel forms
// H Y alone (MY is not touched), accumulating in A.
template <typename T, typename A, bool kHM, bool kEpi, int kWaves, int kBatch, int kOcc>
__global__ void __launch_bounds__(64 * kWaves) __attribute__((amdgpu_waves_per_eu(kOcc, 8)))
spmm_rt_kernel(int64_t nrows, int64_t ntiles, const int64_t *tptr, const int32_t *tcol, const T *tval_h,
               const T *tval_m, const T *Y, int64_t ldy, T *HY, T *MY, int64_t ldo, int m, const int *row_obj,
               const int *obj_status, ChebStep<T> cs) {
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
    // the H-only (FP32-accumulating) form keeps two chunks in flight: chunk k + 2 is requested as
    // soon as chunk k is staged; the fused form, with twice the accumulators in FP64, keeps one
    // (a second would cost it occupancy)
    Chunk<T, kHM> ca, cb;
    ca.load(tcol, tval_h, tval_m, e0 + lane, e0 + lane < e1);
    if (!kHM) {
        cb.load(tcol, tval_h, tval_m, e0 + 64 + lane, e0 + 64 + lane < e1);
        for (int64_t base = e0; base < e1; base += 128) {
            rt_chunk<T, A, kHM, kBatch, 2>(ca, base, e1, tcol, tval_h, tval_m, sv, lane, on, g, c, NG, steps, Y, ldy,
                                           aH, aM);
            if (base + 64 < e1)
                rt_chunk<T, A, kHM, kBatch, 2>(cb, base + 64, e1, tcol, tval_h, tval_m, sv, lane, on, g, c, NG, steps,
                                               Y, ldy, aH, aM);
        }
    } else {
        for (int64_t base = e0; base < e1; base += 64)
            rt_chunk<T, A, kHM, kBatch, 1>(ca, base, e1, tcol, tval_h, tval_m, sv, lane, on, g, c, NG, steps, Y, ldy,
                                           aH, aM);
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
    // after the butterfly every lane holds the sums and lane group i < 4 stores row i when there are
    // at least four groups (FP64 at m = 64 has two); otherwise group 0 stores all four rows
    const bool all = (64 % G) == 0 && NG >= kTileRows;
    if (all ? g < kTileRows : g == 0) {
#pragma unroll
        for (int i = 0; i < kTileRows; ++i) {
            if (all && i != g) continue;
            if (!act[i]) continue;
            const int64_t r = r0 + i;
            if (kEpi) {
                // Chebyshev step on the row: r -= D^-1 H dz, dz' = f1 dz + f2 r, w += dz'
                const int o = row_obj[r];
                const double f1 = cs.coef[(size_t)o * cs.stride + 2 * cs.step - 1];
                const double f2 = cs.coef[(size_t)o * cs.stride + 2 * cs.step];
                const double dv = (double)cs.dinv[r];
                const V rv0 = *(const V *)(cs.R + r * ldo + c * VN);
                const V dz0 = *(const V *)(Y + r * ldy + c * VN);
                const V w0 = *(const V *)(cs.W + r * cs.ldw + c * VN);
                V rv1, dz1, w1;
#pragma unroll
                for (int q = 0; q < VN; ++q) {
                    const double rv = (double)vget(rv0, q) - dv * (double)(T)aH[i].v[q];
                    const double dz = f1 * (double)vget(dz0, q) + f2 * rv;
                    vset(rv1, q, (T)rv);
                    vset(dz1, q, (T)dz);
                    vset(w1, q, (T)((double)vget(w0, q) + dz));
                }
                *(V *)(cs.R + r * ldo + c * VN) = rv1;
                *(V *)(cs.dz_out + r * ldo + c * VN) = dz1;
                *(V *)(cs.W + r * cs.ldw + c * VN) = w1;
            } else {
                acc_store(HY + r * ldo + c * VN, aH[i]);
                if (kHM) acc_store(MY + r * ldo + c * VN, aM[kHM ? i : 0]);
            }
        }
    }
}

template <int kBatch>
__device__ __forceinline__ void h8_chunk(Chunk<float, false> &ch, int64_t base, int64_t e1, const int32_t *tcol,
                                         const float *tval_h, float *sv, int lane, int g, int c, int NG, int steps,
                                         const float *Y, int64_t ldy, float (&acc)[kTileRows][8]) {
    const int cnt = (int)(e1 - base < 64 ? e1 - base : 64);
    const int32_t jc = ch.j;
    __builtin_amdgcn_wave_barrier();
    ch.stage(sv, lane);
    __builtin_amdgcn_wave_barrier();
    ch.load(tcol, tval_h, nullptr, base + 128 + lane, base + 128 + lane < e1);
    for (int s0 = 0; s0 < steps; s0 += kBatch) {
        f32x4 x[kBatch][2];
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
            const int src = (s0 + u) * NG + g;
            const int32_t j = __shfl(jc, src < 64 ? src : 63, 64);
            const bool ok = (s0 + u < steps) && src < cnt;
            x[u][0] = x[u][1] = f32x4{0.f, 0.f, 0.f, 0.f};
            if (ok) {
                const float *yp = Y + (int64_t)j * ldy + c * 8;
                x[u][0] = *(const f32x4 *)yp;
                x[u][1] = *(const f32x4 *)(yp + 4);
            }
        }
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
            const int src = (s0 + u) * NG + g;
            if ((s0 + u < steps) && src < cnt) {
                const f32x4 hv = *(const f32x4 *)(sv + src * 4);
#pragma unroll
                for (int i = 0; i < kTileRows; ++i)
#pragma unroll
                    for (int q = 0; q < 8; ++q) acc[i][q] = fmaf(hv[i], x[u][q >> 2][q & 3], acc[i][q]);
            }
        }
    }
}

// H-only FP32 product (FP32 accumulation) with eight columns per lane: two
// 16-byte pieces of each gathered row, so the per-entry work that does not
// scale with the columns (column shuffle, value read, address) is spread over
// twice the FMAs of the four-column kernel. Needs m % 8 == 0 and 64 % (m / 8)
// == 0; after the butterfly every lane holds the sums and lane group i stores
// row i. With kEpi the Chebyshev step replaces the store; its operands for the
// lane group's row are loaded before the product so their latency is hidden.
template <bool kEpi, int kWaves, int kBatch, int kOcc>
__global__ void __launch_bounds__(64 * kWaves) __attribute__((amdgpu_waves_per_eu(kOcc, 8)))
spmm_rt_h8_kernel(int64_t nrows, int64_t ntiles, const int64_t *tptr, const int32_t *tcol, const float *tval_h,
                  const float *Y, int64_t ldy, float *HY, int64_t ldo, int m, const int *row_obj,
                  const int *obj_status, ChebStep<float> cs) {
    __shared__ __align__(16) float svals[kWaves][64 * 4];
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
    const int G = m >> 3, NG = 64 / G;
    const int g = lane / G, c = lane - g * G;
    const int steps = NG < 64 ? 64 / NG : 1;
    const bool mine = g < kTileRows && act[g < kTileRows ? g : 0];
    const int64_t rme = r0 + (g < kTileRows ? g : 0);
    f32x4 er[2], ez[2], ew[2];
    if (kEpi && mine) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            er[h] = *(const f32x4 *)(cs.R + rme * ldo + c * 8 + 4 * h);
            ez[h] = *(const f32x4 *)(Y + rme * ldy + c * 8 + 4 * h);
            ew[h] = *(const f32x4 *)(cs.W + rme * cs.ldw + c * 8 + 4 * h);
        }
    }
    float *sv = svals[wv];
    const int64_t e0 = tptr[t], e1 = tptr[t + 1];
    float acc[kTileRows][8];
#pragma unroll
    for (int i = 0; i < kTileRows; ++i)
#pragma unroll
        for (int q = 0; q < 8; ++q) acc[i][q] = 0.f;
    Chunk<float, false> ca, cb;
    ca.load(tcol, tval_h, nullptr, e0 + lane, e0 + lane < e1);
    cb.load(tcol, tval_h, nullptr, e0 + 64 + lane, e0 + 64 + lane < e1);
    for (int64_t base = e0; base < e1; base += 128) {
        h8_chunk<kBatch>(ca, base, e1, tcol, tval_h, sv, lane, g, c, NG, steps, Y, ldy, acc);
        if (base + 64 < e1) h8_chunk<kBatch>(cb, base + 64, e1, tcol, tval_h, sv, lane, g, c, NG, steps, Y, ldy, acc);
    }
#pragma unroll
    for (int i = 0; i < kTileRows; ++i)
        for (int d = G; d < 64; d <<= 1)
#pragma unroll
            for (int q = 0; q < 8; ++q) acc[i][q] += __shfl_xor(acc[i][q], d, 64);
    if (!mine) return;
    float a8[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        a8[q] = acc[0][q];
#pragma unroll
        for (int i = 1; i < kTileRows; ++i)
            if (g == i) a8[q] = acc[i][q];
    }
    if (kEpi) {
        // Chebyshev step on the row: r -= D^-1 H dz, dz' = f1 dz + f2 r, w += dz'
        const int o = row_obj[rme];
        const double f1 = cs.coef[(size_t)o * cs.stride + 2 * cs.step - 1];
        const double f2 = cs.coef[(size_t)o * cs.stride + 2 * cs.step];
        const double dv = (double)cs.dinv[rme];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            f32x4 rv1, dz1, w1;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const double rv = (double)er[h][q] - dv * (double)a8[4 * h + q];
                const double dz = f1 * (double)ez[h][q] + f2 * rv;
                rv1[q] = (float)rv;
                dz1[q] = (float)dz;
                w1[q] = (float)((double)ew[h][q] + dz);
            }
            *(f32x4 *)(cs.R + rme * ldo + c * 8 + 4 * h) = rv1;
            *(f32x4 *)(cs.dz_out + rme * ldo + c * 8 + 4 * h) = dz1;
            *(f32x4 *)(cs.W + rme * cs.ldw + c * 8 + 4 * h) = w1;
        }
    } else {
#pragma unroll
        for (int h = 0; h < 2; ++h)
            *(f32x4 *)(HY + rme * ldo + c * 8 + 4 * h) =
                f32x4{a8[4 * h], a8[4 * h + 1], a8[4 * h + 2], a8[4 * h + 3]};
    }
}

inline bool h8_ok(int m, int64_t ldy, int64_t ldo) {
    return m % 8 == 0 && m <= 512 && 64 % (m / 8) == 0 && ldy % 4 == 0 && ldo % 4 == 0;
}

template <bool kEpi>
int launch_h8(ff_ctx *ctx, hipStream_t st, const RTView &v, int sub, int m, const float *Y, int64_t ldy, float *HY,
              int64_t ldo, const int *row_obj, const int *status, const ChebStep<float> &cs) {
#define FF_RT8(W, B, O)                                                                                     \
    hipLaunchKernelGGL((spmm_rt_h8_kernel<kEpi, W, B, O>), dim3(grid_for(v.ntiles, W)), dim3(64 * W), 0, st, \
                       v.n, v.ntiles, v.tptr, v.tcol, v.v32, Y, ldy, HY, ldo, m, row_obj, status, cs)
    switch (sub) {
        case 1: FF_RT8(2, 4, 1); break;
        case 2: FF_RT8(4, 2, 4); break;
        default: FF_RT8(4, 4, 1); break;
    }
#undef FF_RT8
    FF_CHECK_LAUNCH(ctx);
    return FF_OK;
}

template <typename T, typename A = double, bool kHM = true, bool kEpi = false>
int launch(ff_ctx *ctx, hipStream_t st, const RTView &v, const T *tval, int sub, int m, const T *Y, int64_t ldy,
           T *HY, T *MY, int64_t ldo, const int *row_obj, const int *status, ChebStep<T> cs = ChebStep<T>{}) {
    // each lane holds one 16-byte access of the gathered row (narrower loads cost the texture unit as many cycles)
#define FF_RT(W, B, O)                                                                                             \
    hipLaunchKernelGGL((spmm_rt_kernel<T, A, kHM, kEpi, W, B, O>), dim3(grid_for(v.ntiles, W)), dim3(64 * W), 0, st, \
                       v.n, v.ntiles, v.tptr, v.tcol, tval, tval + 4 * v.entries, Y, ldy, HY, MY, ldo, m, row_obj,  \
                       status, cs)
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
    if (h8_ok(m, ldy, ldo))
        return launch_h8<false>(ctx, st, v, sub, m, Y, ldy, HY, ldo, row_obj, status, ChebStep<float>{});
    return launch<float, float, false>(ctx, st, v, v.v32, sub, m, Y, ldy, HY, nullptr, ldo, row_obj, status);
}
int spmm_h64(ff_ctx *ctx, hipStream_t st, const RTView &v, int sub, int m, const double *Y, int64_t ldy, double *HY,
             int64_t ldo, const int *row_obj, const int *status) {
    FF_REQUIRE(ctx, v.v64 != nullptr, "row tiles have no FP64 values");
    return launch<double, double, false>(ctx, st, v, v.v64, sub, m, Y, ldy, HY, nullptr, ldo, row_obj, status);
}
int cheb_step32(ff_ctx *ctx, hipStream_t st, const RTView &v, int sub, int m, const float *DZ, int64_t ld,
                const int *row_obj, const int *status, const ChebStep<float> &cs) {
    FF_REQUIRE(ctx, v.v32 != nullptr && row_obj != nullptr, "row tiles have no FP32 values");
    if (h8_ok(m, ld, ld) && cs.ldw % 4 == 0)
        return launch_h8<true>(ctx, st, v, sub, m, DZ, ld, nullptr, ld, row_obj, status, cs);
    return launch<float, float, false, true>(ctx, st, v, v.v32, sub, m, DZ, ld, nullptr, nullptr, ld, row_obj, status,
                                             cs);
}
int cheb_step64(ff_ctx *ctx, hipStream_t st, const RTView &v, int sub, int m, const double *DZ, int64_t ld,
                const int *row_obj, const int *status, const ChebStep<double> &cs) {
    FF_REQUIRE(ctx, v.v64 != nullptr && row_obj != nullptr, "row tiles have no FP64 values");
    return launch<double, double, false, true>(ctx, st, v, v.v64, sub, m, DZ, ld, nullptr, nullptr, ld, row_obj,
                                               status, cs);
}

// tile pointers and the number of union entries (host), in caller-provided memory
template <int R = kTileRows>
static int build_ptr(ff_ctx *ctx, hipStream_t st, int64_t n, const int64_t *row_ptr, const int32_t *col,
                     int64_t *cnt, int64_t *tptr, int64_t ntiles, int64_t *entries) {
    hipLaunchKernelGGL(rt_count_kernel<R>, dim3(grid_for(ntiles, 256)), dim3(256), 0, st, n, ntiles, row_ptr, col,
                       cnt);
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

// the eight- and sixteen-row copies: the LDS cap of the workgroup-per-tile kernels (the largest
// tile's entry count, at most kUnionCap), tile pointers and the number of union entries (host)
template <int R>
static int build_ptr_union(ff_ctx *ctx, hipStream_t st, int64_t n, const int64_t *row_ptr, const int32_t *col,
                           int64_t *cnt, int64_t *tptr, int64_t ntiles, int64_t *entries, int *cap, int *bits) {
    int *mx0 = (int *)ws_get(ctx, WS_RT8_MAX, 256);
    int64_t *h = (int64_t *)pinned_get(ctx, 64);
    if (!mx0 || !h) return FF_ERR_OOM;
    int *mx = mx0 + 1;                             // word 0 serves the binary16 copies' |H| maximum
    FF_HIP(ctx, hipMemsetAsync(mx, 0, 2 * sizeof(int), st));
    hipLaunchKernelGGL(tile_entries_max_kernel<R>, dim3(grid_for(ntiles, 256)), dim3(256), 0, st, n, ntiles, row_ptr,
                       col, mx);
    FF_CHECK_LAUNCH(ctx);
    FF_HIP(ctx, hipMemcpyAsync(h, mx, 2 * sizeof(int), hipMemcpyDeviceToHost, st));
    FF_HIP(ctx, hipStreamSynchronize(st));
    *cap = std::min(((int *)h)[0], kUnionCap);
    *bits = std::min(((int *)h)[1], ctx->union_bits >= 0 ? std::min(ctx->union_bits, kUnionBitWords) : kUnionBitWords);
    const size_t lds = (size_t)std::max(2 * *cap + 1, 2 * *bits) * sizeof(int32_t);
    hipLaunchKernelGGL((tile_union_kernel<R, false>), dim3(ntiles), dim3(kUnionThreads), lds, st, n, ntiles, row_ptr,
                       col, *cap, *bits, cnt, (const double *)nullptr, (const double *)nullptr,
                       (const int64_t *)nullptr, (int32_t *)nullptr, (float *)nullptr, (float *)nullptr);
    FF_CHECK_LAUNCH(ctx);
    int rc = scan_exclusive_i64(ctx, cnt, tptr, ntiles);
    if (rc) return rc;
    FF_HIP(ctx, hipMemcpyAsync(h, tptr + ntiles, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    FF_HIP(ctx, hipStreamSynchronize(st));
    *entries = h[0];
    return FF_OK;
}

template <int R>
static int fill_union(ff_ctx *ctx, hipStream_t st, int64_t n, int64_t ntiles, const int64_t *row_ptr,
                      const int32_t *col, int cap, int bits, const double *H, const int64_t *tptr, int32_t *tcol,
                      float *vh, const double *M = nullptr, float *vm = nullptr) {
    const size_t lds = (size_t)std::max(2 * cap + 1, 2 * bits) * sizeof(int32_t);
    hipLaunchKernelGGL((tile_union_kernel<R, true>), dim3(ntiles), dim3(kUnionThreads), lds, st, n, ntiles, row_ptr,
                       col, cap, bits, (int64_t *)nullptr, H, M, tptr, tcol, vh, vm);
    FF_CHECK_LAUNCH(ctx);
    return FF_OK;
}

static int fill(ff_ctx *ctx, hipStream_t st, int64_t n, int64_t ntiles, const int64_t *row_ptr, const int32_t *col,
                const double *H, const double *M, const int64_t *tptr, int64_t entries, int32_t *tcol, float *v32,
                double *v64) {
    if (v32)
        hipLaunchKernelGGL(rt_fill_kernel<float>, dim3(grid_for(ntiles, 256)), dim3(256), 0, st, n, ntiles, row_ptr,
                           col, H, M, tptr, tcol, v32, entries, 1);
    if (v64)
        hipLaunchKernelGGL(rt_fill_kernel<double>, dim3(grid_for(ntiles, 256)), dim3(256), 0, st, n, ntiles, row_ptr,
                           col, H, M, tptr, tcol, v64, entries, v32 ? 0 : 1);
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
    if ((rc = fill(ctx, st, n, ntiles, row_ptr, col, H, M, tptr, entries, tcol, v32, v64))) return rc;
    out->n = n;
    out->ntiles = ntiles;
    out->entries = entries;
    out->tptr = tptr;
    out->tcol = tcol;
    out->v32 = v32;
    out->v64 = v64;
    return FF_OK;
}

// ---------------------------------------------------------------------------
// The preconditioner's H-only product on tiles of eight rows
// ---------------------------------------------------------------------------
//
// Eight rows per tile cut the gathered rows of the block from 0.39 to 0.23 per
// nonzero on the benchmark's clouds (the H values grow from 1.55 to 1.86 slots
// per nonzero): the product gathers about 40% fewer bytes through the caches.
// Same scheme as the eight-column kernel: lane groups of G = m / 8 lanes take
// entries of a 64-entry chunk, each lane accumulates 8 rows x 8 columns in
// FP32, the groups are summed by a butterfly, and lane group i stores row i.
template <typename V> struct Chunk8;
template <> struct Chunk8<float> {
    int32_t j;
    f32x4 a, b;                                    // H rows 0..3 and 4..7
    __device__ void load(const int32_t *tcol, const float *vh, int64_t e, bool in) {
        j = 0;
        a = b = f32x4{0.f, 0.f, 0.f, 0.f};
        if (in) {
            j = __builtin_nontemporal_load(tcol + e);
            a = __builtin_nontemporal_load((const f32x4 *)(vh + e * 8));
            b = __builtin_nontemporal_load((const f32x4 *)(vh + e * 8 + 4));
        }
    }
    __device__ void stage(float *sv, int lane) const {
        *(f32x4 *)(sv + lane * 8) = a;
        *(f32x4 *)(sv + lane * 8 + 4) = b;
    }
};
// the FP16 copy: one 16-byte load per entry, widened to FP32 as it is staged
template <> struct Chunk8<_Float16> {
    int32_t j;
    f32x4 a;                                       // H rows 0..7 as eight binary16 values
    __device__ void load(const int32_t *tcol, const _Float16 *vh, int64_t e, bool in) {
        j = 0;
        a = f32x4{0.f, 0.f, 0.f, 0.f};
        if (in) {
            j = __builtin_nontemporal_load(tcol + e);
            a = __builtin_nontemporal_load((const f32x4 *)(vh + e * 8));
        }
    }
    __device__ void stage(float *sv, int lane) const {
        const f16x8 h = __builtin_bit_cast(f16x8, a);
        *(f32x4 *)(sv + lane * 8) = f32x4{(float)h[0], (float)h[1], (float)h[2], (float)h[3]};
        *(f32x4 *)(sv + lane * 8 + 4) = f32x4{(float)h[4], (float)h[5], (float)h[6], (float)h[7]};
    }
};

template <typename V, int kBatch, int kAhead>
__device__ __forceinline__ void t8_chunk(Chunk8<V> &ch, int64_t base, int64_t e1, const int32_t *tcol, const V *vh,
                                         float *sv, int lane, int g, int c, int NG, int steps, const float *Y,
                                         int64_t ldy, float (&acc)[kTile8][8]) {
    const int cnt = (int)(e1 - base < 64 ? e1 - base : 64);
    const int32_t jc = ch.j;
    __builtin_amdgcn_wave_barrier();
    ch.stage(sv, lane);
    __builtin_amdgcn_wave_barrier();
    ch.load(tcol, vh, base + 64 * kAhead + lane, base + 64 * kAhead + lane < e1);
    (void)cnt;
    // entries past the chunk's end have column 0 and zero values: their loads are valid and
    // add nothing, so the loads carry no per-lane condition (a conditional load into a
    // register the previous step loaded makes the wave wait for every load in flight)
    for (int s0 = 0; s0 < steps; s0 += kBatch) {
        f32x4 x[kBatch][2];
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
            if (s0 + u < steps) {
                const int src = (s0 + u) * NG + g;
                const uint32_t j = (uint32_t)__shfl(jc, src, 64);
                const float *yp = Y + (size_t)(j * (uint32_t)ldy) + c * 8;
                x[u][0] = *(const f32x4 *)yp;
                x[u][1] = *(const f32x4 *)(yp + 4);
            }
        }
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
            const int src = (s0 + u) * NG + g;
            if (s0 + u < steps) {
                const f32x4 h0 = *(const f32x4 *)(sv + src * 8), h1 = *(const f32x4 *)(sv + src * 8 + 4);
#pragma unroll
                for (int i = 0; i < kTile8; ++i) {
                    const float hv = i < 4 ? h0[i & 3] : h1[i & 3];
#pragma unroll
                    for (int q = 0; q < 8; ++q) acc[i][q] = fmaf(hv, x[u][q >> 2][q & 3], acc[i][q]);
                }
            }
        }
    }
}

template <typename V, bool kEpi, int kWaves, int kBatch, int kAhead, int kOcc, bool kPre>
__global__ void __launch_bounds__(64 * kWaves) __attribute__((amdgpu_waves_per_eu(kOcc, 8)))
spmm_t8_kernel(int64_t nrows, int64_t ntiles, const int64_t *tptr, const int32_t *tcol, const V *vh, float vscale,
               const float *Y, int64_t ldy, float *HY, int64_t ldo, int m, const int *row_obj, const int *obj_status,
               ChebStep<float> cs) {
    __shared__ __align__(16) float svals[kWaves][64 * 8];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t t = (int64_t)xcd_remap(blockIdx.x, gridDim.x) * kWaves + wv;
    if (t >= ntiles) return;
    const int64_t r0 = t * kTile8;
    const int G = m >> 3, NG = 64 / G;             // NG >= 8 (m <= 64)
    const int g = lane / G, c = lane - g * G;
    const int steps = 64 / NG;
    const int64_t rme = r0 + (g < kTile8 ? g : 0);
    const bool mine = g < kTile8 && rme < nrows && (!obj_status || obj_status[row_obj[rme]] == 0);
    bool any = false;
#pragma unroll
    for (int i = 0; i < kTile8; ++i)
        any = any || (r0 + i < nrows && (!obj_status || obj_status[row_obj[r0 + i]] == 0));
    if (!any) return;
    f32x4 er[2], ez[2], ew[2];
    auto epi_load = [&]() {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            er[h] = *(const f32x4 *)(cs.R + rme * ldo + c * 8 + 4 * h);
            ez[h] = *(const f32x4 *)(Y + rme * ldy + c * 8 + 4 * h);
            ew[h] = *(const f32x4 *)(cs.W + rme * cs.ldw + c * 8 + 4 * h);
        }
    };
    if (kEpi && kPre && mine) epi_load();
    float *sv = svals[wv];
    const int64_t e0 = tptr[t], e1 = tptr[t + 1];
    float acc[kTile8][8];
#pragma unroll
    for (int i = 0; i < kTile8; ++i)
#pragma unroll
        for (int q = 0; q < 8; ++q) acc[i][q] = 0.f;
    Chunk8<V> ca, cb;
    ca.load(tcol, vh, e0 + lane, e0 + lane < e1);
    if (kAhead == 2) {
        cb.load(tcol, vh, e0 + 64 + lane, e0 + 64 + lane < e1);
        for (int64_t base = e0; base < e1; base += 128) {
            t8_chunk<V, kBatch, 2>(ca, base, e1, tcol, vh, sv, lane, g, c, NG, steps, Y, ldy, acc);
            if (base + 64 < e1)
                t8_chunk<V, kBatch, 2>(cb, base + 64, e1, tcol, vh, sv, lane, g, c, NG, steps, Y, ldy, acc);
        }
    } else {
        for (int64_t base = e0; base < e1; base += 64)
            t8_chunk<V, kBatch, 1>(ca, base, e1, tcol, vh, sv, lane, g, c, NG, steps, Y, ldy, acc);
    }
    if (kEpi && !kPre && mine) epi_load();
    if (!kEpi && G == 1) {
        // m = 8: the sum over the 64 lanes as a reduce-scatter. Step d (1, 2, .., 32, the order of the
        // butterfly below) halves each lane's set, the lanes with bit d set keeping the upper half, so
        // every element is the butterfly's sum bit for bit (the same pairs in the same order); lane l
        // ends with element k = bit-reverse6(l) of the 8 x 8 block, row k / 8 and column k % 8
        float v[64];
#pragma unroll
        for (int i = 0; i < kTile8; ++i)
#pragma unroll
            for (int q = 0; q < 8; ++q) v[8 * i + q] = acc[i][q];
#pragma unroll
        for (int st = 0, h = 32; st < 6; ++st, h >>= 1) {
            const int d = 1 << st;
            const bool up = (lane & d) != 0;
#pragma unroll
            for (int k = 0; k < h; ++k) {
                const float keep = up ? v[k + h] : v[k], send = up ? v[k] : v[k + h];
                v[k] = keep + __shfl_xor(send, d, 64);
            }
        }
        const int k = (int)(__builtin_bitreverse32((uint32_t)lane) >> 26);
        const int64_t r = r0 + (k >> 3);
        if (r < nrows && (!obj_status || obj_status[row_obj[r]] == 0)) HY[r * ldo + (k & 7)] = v[0] * vscale;
        return;
    }
#pragma unroll
    for (int i = 0; i < kTile8; ++i)
        for (int d = G; d < 64; d <<= 1)
#pragma unroll
            for (int q = 0; q < 8; ++q) acc[i][q] += __shfl_xor(acc[i][q], d, 64);
    if (!mine) return;
    float a8[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        a8[q] = acc[0][q];
#pragma unroll
        for (int i = 1; i < kTile8; ++i)
            if (g == i) a8[q] = acc[i][q];
    }
    if (kEpi) {
        const int o = row_obj[rme];
        const double f1 = cs.coef[(size_t)o * cs.stride + 2 * cs.step - 1];
        const double f2 = cs.coef[(size_t)o * cs.stride + 2 * cs.step];
        const double dv = (double)cs.dinv[rme] * (double)vscale;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            f32x4 rv1, dz1, w1;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const double rv = (double)er[h][q] - dv * (double)a8[4 * h + q];
                const double dz = f1 * (double)ez[h][q] + f2 * rv;
                rv1[q] = (float)rv;
                dz1[q] = (float)dz;
                w1[q] = (float)((double)ew[h][q] + dz);
            }
            *(f32x4 *)(cs.R + rme * ldo + c * 8 + 4 * h) = rv1;
            *(f32x4 *)(cs.dz_out + rme * ldo + c * 8 + 4 * h) = dz1;
            *(f32x4 *)(cs.W + rme * cs.ldw + c * 8 + 4 * h) = w1;
        }
    } else {
#pragma unroll
        for (int h = 0; h < 2; ++h)
            *(f32x4 *)(HY + rme * ldo + c * 8 + 4 * h) = f32x4{a8[4 * h] * vscale, a8[4 * h + 1] * vscale,
                                                                a8[4 * h + 2] * vscale, a8[4 * h + 3] * vscale};
    }
}

bool t8_ok(int m, int64_t ldy, int64_t ldo) {
    return m % 8 == 0 && m >= 8 && m <= 64 && 64 % (m / 8) == 0 && ldy % 4 == 0 && ldo % 4 == 0;
}

template <bool kEpi>
int launch_t8(ff_ctx *ctx, hipStream_t st, const RT8View &v, int sub, int m, const float *Y, int64_t ldy, float *HY,
              int64_t ldo, const int *row_obj, const int *status, const ChebStep<float> &cs) {
#define FF_T8(VT, VP, SC, W, B, A, O, P)                                                                          \
    hipLaunchKernelGGL((spmm_t8_kernel<VT, kEpi, W, B, A, O, P>), dim3(grid_for(v.ntiles, W)), dim3(64 * W), 0, st, \
                       v.n, v.ntiles, v.tptr, v.tcol, VP, SC, Y, ldy, HY, ldo, m, row_obj, status, cs)
    // H-only product on the benchmark workload (m = 32, FP32 values): 1.18 / 1.24 ms for the first two
    if (v.vh16) {
        const _Float16 *vp = (const _Float16 *)v.vh16;
        switch (sub) {
            case 1: FF_T8(_Float16, vp, v.hscale, 4, 2, 2, 1, true); break;
            case 2: FF_T8(_Float16, vp, v.hscale, 4, 2, 1, 1, false); break;
            default: FF_T8(_Float16, vp, v.hscale, 2, 4, 2, 1, true); break;
        }
    } else {
        switch (sub) {
            case 1: FF_T8(float, v.vh, 1.f, 4, 2, 2, 1, true); break;
            case 2: FF_T8(float, v.vh, 1.f, 4, 2, 1, 1, false); break;
            default: FF_T8(float, v.vh, 1.f, 2, 4, 2, 1, true); break;
        }
    }
#undef FF_T8
    FF_CHECK_LAUNCH(ctx);
    return FF_OK;
}

// the gathers index rows with 32-bit offsets
inline bool off32_ok(int64_t n, int64_t ld) { return n * ld < ((int64_t)1 << 32); }

int spmm_h_t8(ff_ctx *ctx, hipStream_t st, const RT8View &v, int sub, int m, const float *Y, int64_t ldy, float *HY,
              int64_t ldo, const int *row_obj, const int *status) {
    FF_REQUIRE(ctx, (v.vh != nullptr || v.vh16 != nullptr) && t8_ok(m, ldy, ldo),
               "eight-row tiles: bad copy or block shape (m = %d)", m);
    FF_REQUIRE(ctx, off32_ok(v.n, ldy), "block of %lld rows x %lld too large for 32-bit row offsets", (long long)v.n,
               (long long)ldy);
    return launch_t8<false>(ctx, st, v, sub, m, Y, ldy, HY, ldo, row_obj, status, ChebStep<float>{});
}

int cheb_step_t8(ff_ctx *ctx, hipStream_t st, const RT8View &v, int sub, int m, const float *DZ, int64_t ld,
                 const int *row_obj, const int *status, const ChebStep<float> &cs) {
    FF_REQUIRE(ctx, (v.vh != nullptr || v.vh16 != nullptr) && row_obj != nullptr && t8_ok(m, ld, ld) && cs.ldw % 4 == 0,
               "eight-row tiles: bad copy or block shape (m = %d)", m);
    FF_REQUIRE(ctx, off32_ok(v.n, ld), "block of %lld rows x %lld too large for 32-bit row offsets", (long long)v.n,
               (long long)ld);
    return launch_t8<true>(ctx, st, v, sub, m, DZ, ld, nullptr, ld, row_obj, status, cs);
}

int build_t8_ws(ff_ctx *ctx, hipStream_t st, int64_t n, const int64_t *row_ptr, const int32_t *col, const double *H,
                RT8View *out, const double *M) {
    FF_REQUIRE(ctx, n > 0 && row_ptr && col && H && out, "bad arguments");
    const int64_t ntiles = (n + kTile8 - 1) / kTile8;
    int64_t *cnt = (int64_t *)ws_get(ctx, WS_RT8_CNT, (size_t)(ntiles + 1) * sizeof(int64_t));
    int64_t *tptr = (int64_t *)ws_get(ctx, WS_RT8_PTR, (size_t)(ntiles + 1) * sizeof(int64_t));
    if (!cnt || !tptr) return FF_ERR_OOM;
    int64_t entries = 0;
    int cap = 0, bits = 0;
    int rc = build_ptr_union<kTile8>(ctx, st, n, row_ptr, col, cnt, tptr, ntiles, &entries, &cap, &bits);
    if (rc) return rc;
    const size_t ne = (size_t)std::max<int64_t>(entries, 1);
    int32_t *tcol = (int32_t *)ws_get(ctx, WS_RT8_COL, ne * sizeof(int32_t));
    float *vh = (float *)ws_get(ctx, WS_RT8_VAL, ne * kTile8 * sizeof(float));
    float *vm = M ? (float *)ws_get(ctx, WS_RT8_VALM, ne * kTile8 * sizeof(float)) : nullptr;
    if (!tcol || !vh || (M && !vm)) return FF_ERR_OOM;
    if ((rc = fill_union<kTile8>(ctx, st, n, ntiles, row_ptr, col, cap, bits, H, tptr, tcol, vh, M, vm))) return rc;
    out->n = n;
    out->ntiles = ntiles;
    out->entries = entries;
    out->tptr = tptr;
    out->tcol = tcol;
    out->vh = vh;
    out->vm = vm;
    return FF_OK;
}

// largest |v| over n4 groups of four FP32 values, as the bit pattern of a non-negative float
// (those order as unsigned integers, so one atomic max per wavefront combines them)
__global__ void absmax_f32_kernel(int64_t n4, const float *v, uint32_t *out) {
    float a = 0.f;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += (int64_t)gridDim.x * blockDim.x) {
        const f32x4 x = __builtin_nontemporal_load((const f32x4 *)v + i);
        a = fmaxf(a, fmaxf(fmaxf(fabsf(x[0]), fabsf(x[1])), fmaxf(fabsf(x[2]), fabsf(x[3]))));
    }
    for (int d = 32; d >= 1; d >>= 1) a = fmaxf(a, __shfl_xor(a, d, 64));
    if ((threadIdx.x & 63) == 0) atomicMax(out, __float_as_uint(a));
}

// out[i] = binary16(scale * v[i]), eight values per thread; scale is a power of two, so the only
// rounding is the one to binary16 (to nearest even)
__global__ void to_half_kernel(int64_t n8, const float *v, float scale, f32x4 *out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n8) return;
    const f32x4 a = __builtin_nontemporal_load((const f32x4 *)v + 2 * i);
    const f32x4 b = __builtin_nontemporal_load((const f32x4 *)v + 2 * i + 1);
    f16x8 h;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        h[q] = (_Float16)(a[q] * scale);
        h[4 + q] = (_Float16)(b[q] * scale);
    }
    out[i] = __builtin_bit_cast(f32x4, h);
}

// the exponent e of the binary16 copies: 2^e puts the largest |vh| in [2^14, 2^15), so binary16 holds
// it with room to spare and the relative rounding error stays 2^-11 down to 2^-29 of it (below that
// subnormal, then zero); synchronises the stream once
static int half_exponent(ff_ctx *ctx, hipStream_t st, const float *vh, int64_t n8, int *e_out) {
    uint32_t *mx = (uint32_t *)ws_get(ctx, WS_RT8_MAX, 256);
    uint32_t *hbuf = (uint32_t *)pinned_get(ctx, 64);
    if (!mx || !hbuf) return FF_ERR_OOM;
    FF_HIP(ctx, hipMemsetAsync(mx, 0, sizeof(uint32_t), st));
    if (n8 > 0) {
        const int64_t blocks = std::min<int64_t>(grid_for(2 * n8, 256), 8192);
        hipLaunchKernelGGL(absmax_f32_kernel, dim3(blocks), dim3(256), 0, st, 2 * n8, vh, mx);
        FF_CHECK_LAUNCH(ctx);
    }
    FF_HIP(ctx, hipMemcpyAsync(hbuf, mx, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
    FF_HIP(ctx, hipStreamSynchronize(st));
    float amax;
    std::memcpy(&amax, hbuf, sizeof(float));
    FF_REQUIRE(ctx, std::isfinite(amax), "non-finite value in H");
    int e = 0;
    if (amax > 0.f) {
        int p;
        (void)std::frexp(amax, &p);                // amax in [2^(p-1), 2^p)
        e = std::max(-126, std::min(126, 15 - p));
    }
    *e_out = e;
    return FF_OK;
}

int build_t8_half(ff_ctx *ctx, hipStream_t st, RT8View *v, uint16_t *out16) {
    FF_REQUIRE(ctx, v != nullptr && v->vh != nullptr && v->entries >= 0, "FP16 tile copy needs a built FP32 copy");
    const int64_t n8 = v->entries;                 // one group of eight values per entry
    if (!out16) out16 = (uint16_t *)ws_get(ctx, WS_RT8_VAL16, (size_t)std::max<int64_t>(n8, 1) * 8 * 2);
    if (!out16) return FF_ERR_OOM;
    int e = 0;
    int rc = half_exponent(ctx, st, v->vh, n8, &e);
    if (rc) return rc;
    if (n8 > 0) {
        hipLaunchKernelGGL(to_half_kernel, dim3(grid_for(n8, 256)), dim3(256), 0, st, n8, v->vh,
                           std::ldexp(1.f, e), (f32x4 *)out16);
        FF_CHECK_LAUNCH(ctx);
    }
    v->vh16 = out16;
    v->hscale = std::ldexp(1.f, -e);
    return FF_OK;
}

// ---------------------------------------------------------------------------
// The preconditioner's Chebyshev step on the matrix cores (binary16 operands)
// ---------------------------------------------------------------------------
//
// Per tile, (H DZ)^T [columns][8 rows] = DZ^T [columns][entries] . V^T [entries]
// [rows] on v_mfma_f32_16x16x16_f16: 16 columns of the block form the A/D row
// index, 16 union entries the contraction index, the tile's rows the B/D column
// index (8 of its 16 slots carry rows, the other 8 are never stored). A lane's
// A operand holds one column of four consecutive entries, i.e. four different
// gathered rows of DZ: the wave loads the K-block's 16 rows of DZ with 16-byte
// loads, stages them in LDS and reads the fragments back column-wise. The B
// operand is read straight from the K-blocked copy (8 bytes per lane). Lane l
// ends up with rows l % 16 (< 8 kept) at columns 16 cb + 4 (l / 16) + 0..3.
typedef _Float16 f16x4 __attribute__((ext_vector_type(4)));

// The A fragment of v_mfma_f32_16x16x16_f16 for lane (m, g) = (lane % 16, lane / 16) of a 16 x 16
// tile held row-major in LDS (row k at sy + k * stride, 16 binary16 columns from column c0): the
// four values of column c0 + m in rows 4 g .. 4 g + 3, by one transposing LDS read
// (ds_read_b64_tr_b16). In each group of 16 lanes, lane j supplies the 8 bytes of row
// 4 g + j / 4, columns c0 + 4 (j % 4) .. + 3, and lane m receives element m of each of the four
// rows the group read (so the source must be 8-byte aligned).
__device__ inline f16x4 lds_a_frag(const unsigned char *sy, int stride, int c0, int lane) {
    const int g = lane >> 4, j = lane & 15;
    const unsigned char *src = sy + (4 * g + (j >> 2)) * stride + (c0 + 4 * (j & 3)) * 2;
    typedef short i16x4 __attribute__((ext_vector_type(4)));
    typedef __attribute__((address_space(3))) i16x4 *LdsI16x4;
    const i16x4 v = __builtin_amdgcn_ds_read_tr16_b64_v4i16((LdsI16x4)(__attribute__((address_space(3))) void *)(void *)src);
    return __builtin_bit_cast(f16x4, v);
}

__global__ void tq_count_kernel(int64_t ntiles, const int64_t *tptr, int64_t *cnt) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < ntiles) cnt[t] = (tptr[t + 1] - tptr[t] + 15) / 16;
}

// one 64-thread block per tile; K-block kb holds the tile's entries 16 kb .. 16 kb + 15: thread s
// takes values s and s + 64 of the block's 128 (entry-major in vh, so the reads are contiguous)
// and writes them to [row][entry]
__global__ void __launch_bounds__(64) tq_fill_kernel(int64_t ntiles, const int64_t *tptr, const int64_t *kptr,
                                                    const float *vh, float scale, _Float16 *vq) {
    const int64_t t = blockIdx.x;
    if (t >= ntiles) return;
    const int64_t e0 = tptr[t], e1 = tptr[t + 1], k0 = kptr[t], nk = kptr[t + 1] - k0;
    for (int64_t kb = 0; kb < nk; ++kb) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int s = threadIdx.x + 64 * h;
            const int k = s >> 3, r = s & 7;
            const int64_t e = e0 + 16 * kb + k;
            const float v = e < e1 ? vh[e * kTile8 + r] * scale : 0.f;
            vq[(k0 + kb) * 128 + r * 16 + k] = (_Float16)v;
        }
    }
}

// K-block pointers of the tiles (kptr[ntiles + 1]; cnt[ntiles + 1] scratch) and their total
int build_tq_ptr(ff_ctx *ctx, hipStream_t st, const RT8View &v8, int64_t *kptr, int64_t *cnt, int64_t *nkb) {
    FF_REQUIRE(ctx, v8.vh != nullptr && v8.tptr != nullptr && v8.ntiles > 0 && kptr && cnt && nkb,
               "K-blocked copy needs a built eight-row FP32 copy");
    hipLaunchKernelGGL(tq_count_kernel, dim3(grid_for(v8.ntiles, 256)), dim3(256), 0, st, v8.ntiles, v8.tptr, cnt);
    FF_CHECK_LAUNCH(ctx);
    int rc = scan_exclusive_i64(ctx, cnt, kptr, v8.ntiles);
    if (rc) return rc;
    int64_t *h = (int64_t *)pinned_get(ctx, 64);
    if (!h) return FF_ERR_OOM;
    FF_HIP(ctx, hipMemcpyAsync(h, kptr + v8.ntiles, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    FF_HIP(ctx, hipStreamSynchronize(st));
    *nkb = h[0];
    return FF_OK;
}

// the binary16 values into vq (nkb * 128 halves), scaled as the eight-row binary16 copy
int build_tq_fill(ff_ctx *ctx, hipStream_t st, const RT8View &v8, const int64_t *kptr, int64_t nkb, uint16_t *vq,
                  RTQView *out) {
    FF_REQUIRE(ctx, out && vq && kptr, "bad arguments");
    int e = 0;
    int rc = half_exponent(ctx, st, v8.vh, v8.entries, &e);
    if (rc) return rc;
    hipLaunchKernelGGL(tq_fill_kernel, dim3(v8.ntiles), dim3(64), 0, st, v8.ntiles, v8.tptr, kptr, v8.vh,
                       std::ldexp(1.f, e), (_Float16 *)vq);
    FF_CHECK_LAUNCH(ctx);
    out->n = v8.n;
    out->ntiles = v8.ntiles;
    out->nkb = nkb;
    out->tptr = v8.tptr;
    out->tcol = v8.tcol;
    out->kptr = kptr;
    out->vq = vq;
    out->hscale = std::ldexp(1.f, -e);
    return FF_OK;
}

int build_tq(ff_ctx *ctx, hipStream_t st, const RT8View &v8, RTQView *out) {
    const int64_t ntiles = v8.ntiles;
    int64_t *kptr = (int64_t *)ws_get(ctx, WS_RTQ_PTR, (size_t)(ntiles + 1) * sizeof(int64_t));
    int64_t *cnt = (int64_t *)ws_get(ctx, WS_RTQ_CNT, (size_t)(ntiles + 1) * sizeof(int64_t));
    if (!kptr || !cnt) return FF_ERR_OOM;
    int64_t nkb = 0;
    int rc = build_tq_ptr(ctx, st, v8, kptr, cnt, &nkb);
    if (rc) return rc;
    uint16_t *vq = (uint16_t *)ws_get(ctx, WS_RTQ_VAL, (size_t)std::max<int64_t>(nkb, 1) * 128 * 2);
    if (!vq) return FF_ERR_OOM;
    return build_tq_fill(ctx, st, v8, kptr, nkb, vq, out);
}

// halves each tile's zero-free values take: the values present in each group of kTqPackGroup
// consecutive K-blocks (a binary16 value counts when it is not +-0), each group rounded up to a
// multiple of eight halves so that every group starts 16-byte aligned
__global__ void __launch_bounds__(64) tqp_count_kernel(int64_t ntiles, const int64_t *kptr, const uint16_t *vq,
                                                       int64_t *cnt) {
    const int64_t t = blockIdx.x;
    if (t >= ntiles) return;
    const int64_t k0 = kptr[t], nk = kptr[t + 1] - k0;
    int64_t total = 0;
    for (int64_t g = 0; g < nk; g += kTqPackGroup) {
        int c = 0;
        for (int64_t kb = g; kb < nk && kb < g + kTqPackGroup; ++kb)
#pragma unroll
            for (int h = 0; h < 2; ++h) c += (vq[(k0 + kb) * 128 + threadIdx.x + 64 * h] & 0x7fffu) != 0;
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) c += __shfl_xor(c, d, 64);
        total += (c + 7) & ~7;
    }
    if (threadIdx.x == 0) cnt[t] = total;
}

// one 64-thread block per tile: thread s takes values s (rows 0-3) and s + 64 (rows 4-7) of each
// K-block in [row][entry] order; the ballots are the K-block's mask words, the prefix counts
// place the present values (zeros pad each group of K-blocks to a multiple of eight halves)
__global__ void __launch_bounds__(64) tqp_fill_kernel(int64_t ntiles, const int64_t *kptr, const uint16_t *vq,
                                                      const int64_t *pvoff, uint64_t *pmask, uint16_t *pval) {
    const int64_t t = blockIdx.x;
    if (t >= ntiles) return;
    const int lane = threadIdx.x;
    const uint64_t below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    const int64_t k0 = kptr[t], nk = kptr[t + 1] - k0;
    int64_t run = pvoff[t];
    for (int64_t kb = 0; kb < nk; ++kb) {
        if (kb % kTqPackGroup == 0) run = (run + 7) & ~(int64_t)7;      // each group starts 16-byte aligned
        const uint16_t a = vq[(k0 + kb) * 128 + lane], b = vq[(k0 + kb) * 128 + 64 + lane];
        const bool pa = (a & 0x7fffu) != 0, pb = (b & 0x7fffu) != 0;
        const uint64_t lo = __ballot(pa), hi = __ballot(pb);
        if (pa) pval[run + __popcll(lo & below)] = a;
        if (pb) pval[run + __popcll(lo) + __popcll(hi & below)] = b;
        if (lane == 0) {
            pmask[2 * (k0 + kb)] = lo;
            pmask[2 * (k0 + kb) + 1] = hi;
        }
        run += __popcll(lo) + __popcll(hi);
    }
}

__global__ void fill_u16_kernel(uint16_t *a, int64_t count) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) a[i] = 0;
}

int build_tq_pack(ff_ctx *ctx, hipStream_t st, RTQView *v, uint64_t *pmask, int64_t *pvoff, int64_t *cnt,
                  void *(*alloc)(void *, size_t), void *alloc_arg) {
    FF_REQUIRE(ctx, v && v->vq && v->kptr && v->ntiles > 0 && pmask && pvoff && cnt, "zero-free copy: bad arguments");
    hipLaunchKernelGGL(tqp_count_kernel, dim3(v->ntiles), dim3(64), 0, st, v->ntiles, v->kptr, v->vq, cnt);
    FF_CHECK_LAUNCH(ctx);
    int rc = scan_exclusive_i64(ctx, cnt, pvoff, v->ntiles);
    if (rc) return rc;
    int64_t *h = (int64_t *)pinned_get(ctx, 64);
    if (!h) return FF_ERR_OOM;
    FF_HIP(ctx, hipMemcpyAsync(h, pvoff + v->ntiles, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    FF_HIP(ctx, hipStreamSynchronize(st));
    const int64_t total = h[0];
    // eight halves of padding: a lane's window of four values is read as three aligned dwords
    uint16_t *pval = (uint16_t *)alloc(alloc_arg, (size_t)(total + 8) * sizeof(uint16_t));
    if (!pval) return set_error(ctx, FF_ERR_OOM, "zero-free copy: allocation of %lld values failed", (long long)total);
    hipLaunchKernelGGL(fill_u16_kernel, dim3(grid_for(total + 8, 256)), dim3(256), 0, st, pval, total + 8);
    hipLaunchKernelGGL(tqp_fill_kernel, dim3(v->ntiles), dim3(64), 0, st, v->ntiles, v->kptr, v->vq,
                       (const int64_t *)pvoff, pmask, pval);
    FF_CHECK_LAUNCH(ctx);
    v->pmask = pmask;
    v->pvoff = pvoff;
    v->pval = pval;
    return FF_OK;
}

namespace {
struct WsAlloc {
    ff_ctx *ctx;
    int slot;
};
void *ws_alloc(void *arg, size_t bytes) {
    WsAlloc *a = (WsAlloc *)arg;
    return ws_get(a->ctx, a->slot, bytes);
}
}  // namespace

int build_tq_pack_ws(ff_ctx *ctx, hipStream_t st, RTQView *v) {
    uint64_t *pmask = (uint64_t *)ws_get(ctx, WS_RTQ_PMASK, (size_t)std::max<int64_t>(v->nkb, 1) * 16);
    int64_t *pvoff = (int64_t *)ws_get(ctx, WS_RTQ_POFF, (size_t)(v->ntiles + 1) * sizeof(int64_t));
    int64_t *cnt = (int64_t *)ws_get(ctx, WS_RTQ_PCNT, (size_t)(v->ntiles + 1) * sizeof(int64_t));
    if (!pmask || !pvoff || !cnt) return FF_ERR_OOM;
    WsAlloc a{ctx, WS_RTQ_PVAL};
    return build_tq_pack(ctx, st, v, pmask, pvoff, cnt, ws_alloc, &a);
}

bool tq_ok(int m) { return m == 32 || m == 64; }

// The Chebyshev step of the binary16 matrix-core products on one lane's columns 16 cb + 4 quad .. + 3
// of row rme, acc holding (H dz) / vscale there: r -= D^-1 H dz, dz' = f1 dz + f2 r (stored in binary16,
// clamped to its range), w += dz' (wmode 1) or w += dz + dz' (wmode 2, two steps' iterates at once).
// FP32 arithmetic with fused multiply-adds: the iterate is rounded to binary16 (2^-11) at every step,
// far above the FP32 rounding of these few operations.
template <int kMB>
__device__ __forceinline__ void cheb_q_epilogue(const ChebStepQ &cs, const f32x4 (&acc)[kMB], const _Float16 *Y,
                                                int64_t rme, int quad, float vscale, int o) {
    constexpr int m = 16 * kMB;
    const float f1 = (float)cs.coef[(size_t)o * cs.stride + 2 * cs.step - 1];
    const float f2 = (float)cs.coef[(size_t)o * cs.stride + 2 * cs.step];
    const float dv = cs.dinv[rme] * vscale;
    _Float16 *dzo = (_Float16 *)cs.dz_out;
#pragma unroll
    for (int cb = 0; cb < kMB; ++cb) {
        const int c0 = 16 * cb + 4 * quad;
        float *rp = cs.R + rme * m + c0, *wp = cs.W + rme * cs.ldw + c0;
        const f32x4 er = *(const f32x4 *)rp;
        const f32x4 ew = cs.wmode ? *(const f32x4 *)wp : f32x4{0.f, 0.f, 0.f, 0.f};
        const f16x4 ez = *(const f16x4 *)(Y + rme * m + c0);
        f32x4 rv1, w1;
        f16x4 dz1;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const float rv = __builtin_fmaf(-dv, acc[cb][q], er[q]);
            float dz = __builtin_fmaf(f1, (float)ez[q], f2 * rv);
            dz = dz > 65504.f ? 65504.f : (dz < -65504.f ? -65504.f : dz);   // binary16 range
            rv1[q] = rv;
            dz1[q] = (_Float16)dz;
            w1[q] = cs.wmode == 2 ? (ew[q] + (float)ez[q]) + (float)dz1[q] : ew[q] + (float)dz1[q];
        }
        *(f32x4 *)rp = rv1;
        *(f16x4 *)(dzo + rme * m + c0) = dz1;
        if (cs.wmode) *(f32x4 *)wp = w1;
    }
}

template <int kMB, bool kEpi, int kWaves, int kOcc, int kD>
__global__ void __launch_bounds__(64 * kWaves) __attribute__((amdgpu_waves_per_eu(kOcc, 8)))
spmm_tq_kernel(int64_t nrows, int64_t ntiles, const int64_t *tptr, const int32_t *tcol, const int64_t *kptr,
               const _Float16 *vq, float vscale, const _Float16 *Y, float *HY, int64_t ldo, const int *row_obj,
               const int *obj_status, ChebStepQ cs) {
    constexpr int m = 16 * kMB;
    constexpr int kPieces = m / 8;                 // 16-byte pieces of a binary16 row of the block
    constexpr int kRowsPer = 64 / kPieces;         // rows one wave-wide load covers (16 or 8)
    constexpr int kLoads = 16 / kRowsPer;          // loads per K-block (1 or 2)
    constexpr int kStride = 2 * m + 16;            // LDS row stride in bytes: the four entry quads of a
                                                   // fragment read fall on different banks
    __shared__ __align__(16) unsigned char ys[kWaves][16 * kStride];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t t = (int64_t)xcd_remap(blockIdx.x, gridDim.x) * kWaves + wv;
    if (t >= ntiles) return;
    const int64_t r0 = t * kTile8;
    const int rr = lane & 15, quad = lane >> 4;
    const int64_t rme = r0 + (rr & 7);
    const bool mine = rr < 8 && rme < nrows && (!obj_status || obj_status[row_obj[rme]] == 0);
    bool any = false;
#pragma unroll
    for (int i = 0; i < kTile8; ++i)
        any = any || (r0 + i < nrows && (!obj_status || obj_status[row_obj[r0 + i]] == 0));
    if (!any) return;
    const int64_t e0 = tptr[t], e1 = tptr[t + 1], k0 = kptr[t];
    const int nk = (int)(kptr[t + 1] - k0);
    const int piece = lane % kPieces, slot = lane / kPieces;
    unsigned char *sy = ys[wv];
    // entries past the tile's end read its last column (their values are zero), so every load is
    // unconditional
    auto col_of = [&](int kb, int i) -> uint32_t {
        const int64_t e = e0 + 16 * kb + slot + kRowsPer * i;
        return (uint32_t)tcol[e < e1 ? e : e1 - 1];
    };
    auto load_y = [&](uint32_t j) -> f32x4 {
        return *(const f32x4 *)(Y + (size_t)(j * (uint32_t)m) + piece * 8);
    };
    auto load_v = [&](int kb) -> f16x4 {
        return __builtin_nontemporal_load((const f16x4 *)(vq + (k0 + kb) * 128 + (rr & 7) * 16 + 4 * quad));
    };
    f32x4 acc[kMB];
#pragma unroll
    for (int cb = 0; cb < kMB; ++cb) acc[cb] = f32x4{0.f, 0.f, 0.f, 0.f};
    if (nk > 0) {
        // a ring of kD K-blocks: kD - 1 in flight while one is multiplied. The passes of a partial
        // last round reload the tile's last block and multiply a zero B operand.
        f32x4 y[kD][kLoads];
        f16x4 b[kD];
        uint32_t jn[kLoads];
#pragma unroll
        for (int d = 0; d < kD - 1; ++d) {
            const int kb = d < nk ? d : nk - 1;
#pragma unroll
            for (int i = 0; i < kLoads; ++i) y[d][i] = load_y(col_of(kb, i));
            b[d] = load_v(kb);
        }
#pragma unroll
        for (int i = 0; i < kLoads; ++i) jn[i] = col_of(kD - 1 < nk ? kD - 1 : nk - 1, i);
        for (int kb0 = 0; kb0 < nk; kb0 += kD) {
#pragma unroll
            for (int d = 0; d < kD; ++d) {
                const int kb = kb0 + d;
                // block kb + kD - 1's rows (their columns are loaded), then block kb + kD's columns
                const int si = (d + kD - 1) % kD;
                const int kbi = kb + kD - 1 < nk ? kb + kD - 1 : nk - 1;
#pragma unroll
                for (int i = 0; i < kLoads; ++i) y[si][i] = load_y(jn[i]);
                b[si] = load_v(kbi);
                const int kbn = kb + kD < nk ? kb + kD : nk - 1;
#pragma unroll
                for (int i = 0; i < kLoads; ++i) jn[i] = col_of(kbn, i);
                __builtin_amdgcn_wave_barrier();
#pragma unroll
                for (int i = 0; i < kLoads; ++i)
                    *(f32x4 *)(sy + (slot + kRowsPer * i) * kStride + piece * 16) = y[d][i];
                __builtin_amdgcn_wave_barrier();
                const f16x4 bv = kb < nk ? b[d] : f16x4{0, 0, 0, 0};
#pragma unroll
                for (int cb = 0; cb < kMB; ++cb) {
                    const f16x4 a = lds_a_frag(sy, kStride, 16 * cb, lane);
                    acc[cb] = __builtin_amdgcn_mfma_f32_16x16x16f16(a, bv, acc[cb], 0, 0, 0);
                }
            }
        }
    }
    if (!mine) return;
    if (kEpi) {
        cheb_q_epilogue<kMB>(cs, acc, Y, rme, quad, vscale, row_obj[rme]);
    } else {
#pragma unroll
        for (int cb = 0; cb < kMB; ++cb)
            *(f32x4 *)(HY + rme * ldo + 16 * cb + 4 * quad) = acc[cb] * vscale;
    }
}

// The same product with the gathers pipelined a super-block of four K-blocks (64 union entries) ahead.
// Vector loads retire in order, so in the ring above the wait for a K-block's columns also waits for
// every gather issued before them and at most one or two K-blocks of gathers are in flight. Here each
// lane loads one column of a super-block (coalesced, two super-blocks ahead) and the lanes that
// gather a row take its column from that lane by a cross-lane read; the gathers and value loads of
// super-block s + 1 are issued before super-block s is multiplied. The four K-blocks of a super-block
// use separate LDS buffers.
//
// With kPacked the values come from the zero-free copy. A super-block's four pairs of mask words
// are loaded two super-blocks ahead (so waiting for them does not wait for the gathers in flight)
// and read into scalar registers; their counts give the super-block's span of values, which the
// wave reads at once, 16 bytes a lane from its 16-byte aligned start, and stages in LDS beside the
// gathered rows. Lane j then rebuilds entries j and 64 + j of each K-block in LDS (its mask bit
// selects the value at the count of set bits below it, or zero) and each lane reads its B fragment
// from there, so the B operand, and every sum, is the same as from the full K-block.
struct PackedQ {
    const uint64_t *pmask = nullptr;
    const int64_t *pvoff = nullptr;
    const uint16_t *pval = nullptr;
};
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef const __attribute__((address_space(4))) int64_t *ConstI64;
// the super-block's values staged in LDS: at most 4 * 128 halves
constexpr int kPkStage = 4 * 128 * 2;

template <int kMB, bool kEpi, int kWaves, int kOcc, bool kPacked = false, int kDepth = 2, bool kPadRows = true>
__global__ void __launch_bounds__(64 * kWaves) __attribute__((amdgpu_waves_per_eu(kOcc, 8)))
spmm_tq_sb_kernel(int64_t nrows, int64_t ntiles, const int64_t *tptr, const int32_t *tcol, const int64_t *kptr,
                  const _Float16 *vq, float vscale, const _Float16 *Y, float *HY, int64_t ldo, const int *row_obj,
                  const int *obj_status, ChebStepQ cs, PackedQ pq) {
    constexpr int m = 16 * kMB;
    constexpr int kPieces = m / 8;                 // 16-byte pieces of a binary16 row of the block
    constexpr int kRowsPer = 64 / kPieces;         // rows one wave-wide load covers (16 or 8)
    constexpr int kLoads = 16 / kRowsPer;          // loads per K-block (1 or 2)
    // LDS row stride in bytes (2m + 32, which puts the eight rows a half-wave reads by the transposing
    // read on distinct banks and cut the bank-conflict cycles by a quarter, measured 3% slower at
    // m = 32: 0.526 against 0.512 ms)
    // (unpadded rows: 2m bytes, so that eight four-wave workgroups fit a CU's LDS)
    constexpr int kStride = kPadRows ? 2 * m + 16 : 2 * m;
    constexpr int kQ = 4;                          // K-blocks per super-block
    static_assert(kQ == kTqPackGroup, "the zero-free copy aligns groups of four K-blocks");
    __shared__ __align__(16) unsigned char ys[kWaves][kQ][16 * kStride];
    // the super-block's staged values, rebuilt in place into its four dense K-blocks (4 x 256 bytes)
    __shared__ __align__(16) unsigned char pvs[kWaves][kPacked ? kPkStage : 16];
    const int lane = threadIdx.x & 63, wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t t = (int64_t)xcd_remap(blockIdx.x, gridDim.x) * kWaves + wv;
    if (t >= ntiles) return;
    const int64_t r0 = t * kTile8;
    const int rr = lane & 15, quad = lane >> 4;
    const int64_t rme = r0 + (rr & 7);
    const bool mine = rr < 8 && rme < nrows && (!obj_status || obj_status[row_obj[rme]] == 0);
    bool any = false;
#pragma unroll
    for (int i = 0; i < kTile8; ++i)
        any = any || (r0 + i < nrows && (!obj_status || obj_status[row_obj[r0 + i]] == 0));
    if (!any) return;
    const int64_t e0 = tptr[t], e1 = tptr[t + 1], k0 = kptr[t];
    const int nk = (int)(kptr[t + 1] - k0);
    const int ns = (nk + kQ - 1) / kQ;
    const int piece = lane % kPieces, slot = lane / kPieces;
    // entries past the tile's end read its last column (their values are zero)
    auto cols_of = [&](int s) -> int {
        const int64_t e = e0 + 64 * (int64_t)s + lane;
        return tcol[e < e1 ? e : e1 - 1];
    };
    const _Float16 *vb = vq + k0 * 128 + (rr & 7) * 16 + 4 * quad;   // this lane's values in the tile's K-blocks
    // packed copy: the start of the next super-block's values (uniform)
    int64_t pk_run = kPacked ? ((ConstI64)pq.pvoff)[t] : 0;
    struct PkSB {
        u32x4 pv;              // this lane's 16 bytes of the super-block's values
        uint64_t lo[kQ], hi[kQ];
        uint32_t mk;           // lanes 0-15: the mask dwords of the next super-block this buffer takes
    };
    // the four K-blocks' mask words of super-block sb, one dword a lane in lanes 0-15 (K-blocks past
    // the tile's end read its last one; they are not used)
    auto load_masks = [&](int sb) -> uint32_t {
        const int kb = kQ * sb + ((lane >> 2) & 3);
        const uint32_t *mp = (const uint32_t *)(pq.pmask + 2 * (k0 + (kb < nk ? kb : nk - 1)));
        return lane < 16 ? mp[lane & 3] : 0u;
    };
    // the gathers of a super-block, then its value loads (consumed in that order); whole: all four
    // K-blocks lie inside the tile
    auto issue = [&](int s, int cols, f32x4 (&y)[kQ][kLoads], f16x4 (&b)[kQ], PkSB &pk, bool whole) {
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int q = 0; q < kQ; ++q)
#pragma unroll
            for (int i = 0; i < kLoads; ++i) {
                const uint32_t j = (uint32_t)__shfl(cols, 16 * q + slot + kRowsPer * i, 64);
                y[q][i] = *(const f32x4 *)(Y + (size_t)(j * (uint32_t)m) + piece * 8);
            }
        __builtin_amdgcn_sched_barrier(0);
        if constexpr (!kPacked) {
#pragma unroll
            for (int q = 0; q < kQ; ++q) {
                const int kb = whole || kQ * s + q < nk ? kQ * s + q : nk - 1;
                b[q] = __builtin_nontemporal_load((const f16x4 *)(vb + kb * 128));
            }
        } else {
            // this super-block's masks were loaded two super-blocks ago: the wait for them does not
            // wait for the gathers in flight
            int span = 0;
#pragma unroll
            for (int q = 0; q < kQ; ++q) {
                const bool in = whole || kQ * s + q < nk;
                const uint64_t lo = (uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)pk.mk, 4 * q) |
                                    ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)pk.mk, 4 * q + 1) << 32);
                const uint64_t hi = (uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)pk.mk, 4 * q + 2) |
                                    ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)pk.mk, 4 * q + 3) << 32);
                pk.lo[q] = in ? lo : 0ull;
                pk.hi[q] = in ? hi : 0ull;
                span += __popcll(pk.lo[q]) + __popcll(pk.hi[q]);
            }
            pk.pv = 8 * lane < span ? __builtin_nontemporal_load((const u32x4 *)(pq.pval + pk_run) + lane)
                                    : u32x4{0u, 0u, 0u, 0u};
            pk_run += (span + 7) & ~7;
            pk.mk = load_masks(s + (kDepth == 1 ? 1 : 2));
        }
        __builtin_amdgcn_sched_barrier(0);
    };
    f32x4 acc[kMB];
#pragma unroll
    for (int cb = 0; cb < kMB; ++cb) acc[cb] = f32x4{0.f, 0.f, 0.f, 0.f};
    // multiplies super-block s; full: all four of its K-blocks lie inside the tile
    // the gathered rows and the staged values of a super-block into LDS
    auto stage_lds = [&](const f32x4 (&y)[kQ][kLoads], const PkSB &pk) __attribute__((always_inline)) {
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int q = 0; q < kQ; ++q)
#pragma unroll
            for (int i = 0; i < kLoads; ++i)
                *(f32x4 *)(&ys[wv][q][0] + (slot + kRowsPer * i) * kStride + piece * 16) = y[q][i];
        if constexpr (kPacked) *(u32x4 *)(&pvs[wv][0] + 16 * lane) = pk.pv;
        __builtin_amdgcn_wave_barrier();
    };
    // multiplies the staged super-block s (lo, hi: its K-blocks' masks)
    auto compute = [&](int s, const f16x4 (&b)[kQ], const uint64_t (&mlo)[kQ], const uint64_t (&mhi)[kQ], bool full)
        __attribute__((always_inline)) {
        f16x4 bp[kQ];
        if constexpr (kPacked) {
            // expand the four K-blocks in place, lane j taking entries j (rows 0-3) and 64 + j
            // (rows 4-7) of each: present when its mask bit is set, then the value at the count of
            // present entries before it. Every value is read before any is written (a wave's LDS
            // instructions execute in order), so the dense blocks can overwrite the staged values.
            uint16_t *ps = (uint16_t *)&pvs[wv][0];
            uint16_t v0[kQ], v1[kQ];
            int base = 0;                                              // halves before K-block q
#pragma unroll
            for (int q = 0; q < kQ; ++q) {
                const uint64_t lo = mlo[q], hi = mhi[q];
                const int nlo = __popcll(lo);
                const int ilo = __builtin_amdgcn_mbcnt_hi((uint32_t)(lo >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)lo, 0));
                const int ihi = __builtin_amdgcn_mbcnt_hi((uint32_t)(hi >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)hi, 0));
                v0[q] = ps[base + ilo];
                v1[q] = ps[base + nlo + ihi];
                base += nlo + __popcll(hi);
            }
            uint16_t *pd = ps;
#pragma unroll
            for (int q = 0; q < kQ; ++q) {
                pd[q * 128 + lane] = __builtin_amdgcn_inverse_ballot_w64(mlo[q]) ? v0[q] : (uint16_t)0;
                pd[q * 128 + 64 + lane] = __builtin_amdgcn_inverse_ballot_w64(mhi[q]) ? v1[q] : (uint16_t)0;
            }
            __builtin_amdgcn_wave_barrier();
#pragma unroll
            for (int q = 0; q < kQ; ++q) bp[q] = *(const f16x4 *)(pd + q * 128 + (rr & 7) * 16 + 4 * quad);
        }
#pragma unroll
        for (int q = 0; q < kQ; ++q) {
            if (!full && kQ * s + q >= nk) break;
            const unsigned char *sy = &ys[wv][q][0];
#pragma unroll
            for (int cb = 0; cb < kMB; ++cb) {
                const f16x4 a = lds_a_frag(sy, kStride, 16 * cb, lane);
                acc[cb] = __builtin_amdgcn_mfma_f32_16x16x16f16(a, kPacked ? bp[q] : b[q], acc[cb], 0, 0, 0);
            }
        }
    };
    auto consume = [&](int s, const f32x4 (&y)[kQ][kLoads], const f16x4 (&b)[kQ], const PkSB &pk, bool full)
        __attribute__((always_inline)) {
        stage_lds(y, pk);
        compute(s, b, pk.lo, pk.hi, full);
    };
    if constexpr (kDepth == 1) {
        // one buffer: super-block s + 1 is gathered into the registers that held s once s is staged
        // in LDS, while s is multiplied from there; its masks are loaded one super-block ahead (the
        // wait for them only waits for loads that staging s waited for already)
        static_assert(kPacked, "the single-buffer form reads the zero-free copy");
        if (nk > 0) {
            f32x4 y1[kQ][kLoads];
            f16x4 b1[kQ];
            PkSB p1;
            p1.mk = load_masks(0);
            issue(0, cols_of(0), y1, b1, p1, false);
            int cn = cols_of(ns > 1 ? 1 : 0);
            for (int s = 0; s < ns; ++s) {
                stage_lds(y1, p1);
                uint64_t mlo[kQ], mhi[kQ];
#pragma unroll
                for (int q = 0; q < kQ; ++q) {
                    mlo[q] = p1.lo[q];
                    mhi[q] = p1.hi[q];
                }
                if (s + 1 < ns) {
                    issue(s + 1, cn, y1, b1, p1, false);
                    cn = cols_of(s + 2 < ns ? s + 2 : ns - 1);
                }
                compute(s, b1, mlo, mhi, false);
            }
        }
    } else {
        if (nk > 0) {
            f32x4 ya[kQ][kLoads], yb[kQ][kLoads];
            f16x4 ba[kQ], bb[kQ];
            PkSB pa, pb;
            if constexpr (kPacked) {
                pa.mk = load_masks(0);
                pb.mk = load_masks(1);
            }
            const int c0 = cols_of(0);
            int c1 = cols_of(ns > 1 ? 1 : 0);
            issue(0, c0, ya, ba, pa, ns > 1);
            int s = 0;
            // steady state: super-blocks s and s + 1 are whole, s + 2 exists
            for (; s + 2 < ns; s += 2) {
                const int c2 = cols_of(s + 2);
                issue(s + 1, c1, yb, bb, pb, true);
                consume(s, ya, ba, pa, true);
                c1 = cols_of(s + 3 < ns ? s + 3 : ns - 1);
                issue(s + 2, c2, ya, ba, pa, false);
                consume(s + 1, yb, bb, pb, true);
            }
            // the last one or two super-blocks
            if (s + 1 < ns) {
                issue(s + 1, c1, yb, bb, pb, false);
                consume(s, ya, ba, pa, true);
                consume(s + 1, yb, bb, pb, false);
            } else {
                consume(s, ya, ba, pa, false);
            }
        }
    }
    if (!mine) return;
    if (kEpi) {
        cheb_q_epilogue<kMB>(cs, acc, Y, rme, quad, vscale, row_obj[rme]);
    } else {
#pragma unroll
        for (int cb = 0; cb < kMB; ++cb)
            *(f32x4 *)(HY + rme * ldo + 16 * cb + 4 * quad) = acc[cb] * vscale;
    }
}

template <bool kEpi>
static int launch_tq(ff_ctx *ctx, hipStream_t st, const RTQView &v, int sub, int m, const uint16_t *Y, float *HY,
                     int64_t ldo, const int *row_obj, const int *status, const ChebStepQ &cs) {
    FF_REQUIRE(ctx, v.vq != nullptr && tq_ok(m), "matrix-core Chebyshev step: no K-blocked copy or m = %d", m);
    FF_REQUIRE(ctx, sub >= 0 && sub < kTqSubs, "launch shape %d out of range", sub);
    FF_REQUIRE(ctx, sub < kTqPacked || (v.pmask && v.pval && v.pvoff), "launch shape %d needs the zero-free copy", sub);
    PackedQ pq;
    pq.pmask = v.pmask;
    pq.pvoff = v.pvoff;
    pq.pval = v.pval;
    FF_REQUIRE(ctx, v.n * (int64_t)m < ((int64_t)1 << 32), "block of %lld rows x %d too large for 32-bit offsets",
               (long long)v.n, m);
    const _Float16 *vq = (const _Float16 *)v.vq, *y = (const _Float16 *)Y;
    // Ring shapes 0 .. 4 (waves per block, occupancy floor, K-blocks in the ring); product alone at 1M
    // particles, m = 32 / 64: 0.607 / 0.888, 0.610 / 0.887, 0.656 / 0.962, 0.631 / 0.889, 0.612 / 0.892 ms.
    // Super-block shapes 5 .. 7 (waves per block, occupancy floor), measured in one run with shape 0 at
    // 0.622 / 0.897 ms: 0.551 / 0.863, 0.561 / 0.825, 0.552 / 0.864 ms. Eight consecutive tiles per
    // workgroup share most gathered rows in the CU's cache.
#define FF_TQ(MB, W, O, D)                                                                                        \
    hipLaunchKernelGGL((spmm_tq_kernel<MB, kEpi, W, O, D>), dim3(grid_for(v.ntiles, W)), dim3(64 * W), 0, st, v.n, \
                       v.ntiles, v.tptr, v.tcol, v.kptr, vq, v.hscale, y, HY, ldo, row_obj, status, cs)
#define FF_TQS(MB, W, O)                                                                                       \
    hipLaunchKernelGGL((spmm_tq_sb_kernel<MB, kEpi, W, O>), dim3(grid_for(v.ntiles, W)), dim3(64 * W), 0, st, v.n, \
                       v.ntiles, v.tptr, v.tcol, v.kptr, vq, v.hscale, y, HY, ldo, row_obj, status, cs, pq)
#define FF_TQP(MB, W, O)                                                                                       \
    hipLaunchKernelGGL((spmm_tq_sb_kernel<MB, kEpi, W, O, true>), dim3(grid_for(v.ntiles, W)), dim3(64 * W), 0, st,  \
                       v.n, v.ntiles, v.tptr, v.tcol, v.kptr, vq, v.hscale, y, HY, ldo, row_obj, status, cs, pq)
#define FF_TQP1(MB, W, O)                                                                                     \
    hipLaunchKernelGGL((spmm_tq_sb_kernel<MB, kEpi, W, O, true, 1>), dim3(grid_for(v.ntiles, W)), dim3(64 * W), 0,  \
                       st, v.n, v.ntiles, v.tptr, v.tcol, v.kptr, vq, v.hscale, y, HY, ldo, row_obj, status, cs, pq)
#define FF_TQP1U(MB, W, O)                                                                                    \
    hipLaunchKernelGGL((spmm_tq_sb_kernel<MB, kEpi, W, O, true, 1, false>), dim3(grid_for(v.ntiles, W)),          \
                       dim3(64 * W), 0, st, v.n, v.ntiles, v.tptr, v.tcol, v.kptr, vq, v.hscale, y, HY, ldo, row_obj,  \
                       status, cs, pq)
#define FF_TQ_SHAPES(MB)                   \
    switch (sub) {                         \
        case 1: FF_TQ(MB, 8, 4, 3); break; \
        case 2: FF_TQ(MB, 4, 4, 2); break; \
        case 3: FF_TQ(MB, 4, 4, 3); break; \
        case 4: FF_TQ(MB, 16, 4, 2); break; \
        case 5: FF_TQS(MB, 8, 2); break;   \
        case 6: FF_TQS(MB, 4, 2); break;   \
        case 7: FF_TQS(MB, 8, MB == 2 ? 5 : 3); break; \
        case 8: FF_TQP(MB, 8, 2); break;   \
        case 9: FF_TQP(MB, 4, 2); break;   \
        case 10: FF_TQP(MB, 8, MB == 2 ? 5 : 3); break; \
        case 11: FF_TQP(MB, 4, 4); break;  \
        case 12: FF_TQP(MB, 2, 2); break;  \
        case 13: FF_TQP1(MB, 4, 6); break; \
        case 14: FF_TQP1U(MB, 4, 8); break; \
        default: FF_TQ(MB, 8, 4, 2); break; \
    }
    if (m == 32) {
        FF_TQ_SHAPES(2)
    } else {
        FF_TQ_SHAPES(4)
    }
#undef FF_TQ_SHAPES
#undef FF_TQP
#undef FF_TQP1
#undef FF_TQP1U
#undef FF_TQS
#undef FF_TQ
    FF_CHECK_LAUNCH(ctx);
    return FF_OK;
}

int cheb_step_tq(ff_ctx *ctx, hipStream_t st, const RTQView &v, int sub, int m, const uint16_t *DZ,
                 const int *row_obj, const int *status, const ChebStepQ &cs) {
    FF_REQUIRE(ctx, DZ && row_obj && cs.R && cs.W && cs.dz_out && cs.dinv && cs.coef && cs.ldw % 4 == 0,
               "matrix-core Chebyshev step: bad arguments");
    return launch_tq<true>(ctx, st, v, sub, m, DZ, nullptr, 0, row_obj, status, cs);
}

int spmm_h_tq(ff_ctx *ctx, hipStream_t st, const RTQView &v, int sub, int m, const uint16_t *Y, float *HY,
              int64_t ldo) {
    FF_REQUIRE(ctx, Y && HY && ldo >= m && ldo % 4 == 0, "matrix-core product: bad arguments");
    return launch_tq<false>(ctx, st, v, sub, m, Y, HY, ldo, nullptr, nullptr, ChebStepQ{});
}

// ---------------------------------------------------------------------------
// The preconditioner's H-only product on tiles of sixteen rows, on MFMA
// ---------------------------------------------------------------------------
//
// Per tile the product is dense: (H Y)[tile rows][columns] = V[tile rows][entries]
// . Y[entries][columns], V the tile's value block and the entries' rows of Y
// gathered. It runs on v_mfma_f32_16x16x4f32 with the 16 tile rows as the B/D
// column index and 16 column slots as the A/D row index: slot i of MFMA t holds
// column kMT * i + t (kMT = m / 16), so the lane that supplies slot i for entry
// k reads kMT consecutive floats of that entry's row with one load. The MFMA
// sums over the entries itself (no cross-lane reduction), and lane l ends up
// holding row l % 16 of the tile at 4 kMT consecutive columns, which it then
// stores or uses for the Chebyshev step. m <= 16 (kMT = 1) masks slots >= m.
struct Chunk16 {
    int32_t j;
    f32x4 v[4];                                    // H of the tile's rows 0..15
    __device__ void load(const int32_t *tcol, const float *vh, int64_t e, bool in) {
        j = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q) v[q] = f32x4{0.f, 0.f, 0.f, 0.f};
        if (in) {
            j = __builtin_nontemporal_load(tcol + e);
#pragma unroll
            for (int q = 0; q < 4; ++q) v[q] = __builtin_nontemporal_load((const f32x4 *)(vh + e * 16 + 4 * q));
        }
    }
    __device__ void stage(float *sv, int lane) const {
#pragma unroll
        for (int q = 0; q < 4; ++q) *(f32x4 *)(sv + lane * 16 + 4 * q) = v[q];
    }
};

template <int kMT> struct YVec;
template <> struct YVec<1> { typedef float type; };
template <> struct YVec<2> { typedef float2 type; };
template <> struct YVec<4> { typedef f32x4 type; };
__device__ inline float yget(const float &v, int) { return v; }
__device__ inline float yget(const float2 &v, int t) { return t == 0 ? v.x : v.y; }
__device__ inline float yget(const f32x4 &v, int t) { return v[t]; }

__device__ inline f32x4 mfma16(float a, float b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

template <int kMT, int kBatch, int kAhead>
__device__ __forceinline__ void t16_chunk(Chunk16 &ch, int64_t base, int64_t e1, const int32_t *tcol, const float *vh,
                                          float *sv, int lane, int li, int lk, int m, const float *Y, int64_t ldy,
                                          f32x4 (&d)[kMT]) {
    typedef typename YVec<kMT>::type YV;
    const int cnt = (int)(e1 - base < 64 ? e1 - base : 64);
    const int32_t jc = ch.j;
    __builtin_amdgcn_wave_barrier();
    ch.stage(sv, lane);
    __builtin_amdgcn_wave_barrier();
    ch.load(tcol, vh, base + 64 * kAhead + lane, base + 64 * kAhead + lane < e1);
    const bool slot_ok = kMT > 1 || li < m;
    const int nq = (cnt + 3) >> 2;                 // k-steps of 4 entries
    for (int q0 = 0; q0 < nq; q0 += kBatch) {
        YV y[kBatch];
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
            const int e = 4 * (q0 + u) + lk;
            const int32_t j = __shfl(jc, e < 64 ? e : 63, 64);
            y[u] = YV{};
            if (e < cnt && slot_ok) y[u] = *(const YV *)(Y + (int64_t)j * ldy + kMT * li);
        }
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
            const int e = 4 * (q0 + u) + lk;
            const float b = (q0 + u < nq && e < cnt) ? sv[e * 16 + li] : 0.f;
#pragma unroll
            for (int t = 0; t < kMT; ++t) d[t] = mfma16(yget(y[u], t), b, d[t]);
        }
    }
}

template <bool kEpi, int kMT, int kWaves, int kBatch, int kAhead, int kOcc, bool kPre>
__global__ void __launch_bounds__(64 * kWaves) __attribute__((amdgpu_waves_per_eu(kOcc, 8)))
spmm_t16_kernel(int64_t nrows, int64_t ntiles, const int64_t *tptr, const int32_t *tcol, const float *vh,
                const float *Y, int64_t ldy, float *HY, int64_t ldo, int m, const int *row_obj, const int *obj_status,
                ChebStep<float> cs) {
    __shared__ __align__(16) float svals[kWaves][64 * 16];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t t = (int64_t)xcd_remap(blockIdx.x, gridDim.x) * kWaves + wv;
    if (t >= ntiles) return;
    const int li = lane & 15, lk = lane >> 4;
    const int64_t r = t * kTile16 + li;           // the row this lane stores
    const int c0 = lk * 4 * kMT;                   // its first column
    const bool mine = r < nrows && c0 < m && (!obj_status || obj_status[row_obj[r]] == 0);
    if (!__any(r < nrows && (!obj_status || obj_status[row_obj[r]] == 0))) return;
    f32x4 er[kMT], ez[kMT], ew[kMT];
    auto epi_load = [&]() {
#pragma unroll
        for (int h = 0; h < kMT; ++h) {
            er[h] = *(const f32x4 *)(cs.R + r * ldo + c0 + 4 * h);
            ez[h] = *(const f32x4 *)(Y + r * ldy + c0 + 4 * h);
            ew[h] = *(const f32x4 *)(cs.W + r * cs.ldw + c0 + 4 * h);
        }
    };
    if (kEpi && kPre && mine) epi_load();
    float *sv = svals[wv];
    const int64_t e0 = tptr[t], e1 = tptr[t + 1];
    f32x4 d[kMT];
#pragma unroll
    for (int q = 0; q < kMT; ++q) d[q] = f32x4{0.f, 0.f, 0.f, 0.f};
    Chunk16 ca, cb;
    ca.load(tcol, vh, e0 + lane, e0 + lane < e1);
    if (kAhead == 2) {
        cb.load(tcol, vh, e0 + 64 + lane, e0 + 64 + lane < e1);
        for (int64_t base = e0; base < e1; base += 128) {
            t16_chunk<kMT, kBatch, 2>(ca, base, e1, tcol, vh, sv, lane, li, lk, m, Y, ldy, d);
            if (base + 64 < e1) t16_chunk<kMT, kBatch, 2>(cb, base + 64, e1, tcol, vh, sv, lane, li, lk, m, Y, ldy, d);
        }
    } else {
        for (int64_t base = e0; base < e1; base += 64)
            t16_chunk<kMT, kBatch, 1>(ca, base, e1, tcol, vh, sv, lane, li, lk, m, Y, ldy, d);
    }
    if (!mine) return;
    if (kEpi && !kPre) epi_load();
    // d[t][v] is column kMT * (4 lk + v) + t = c0 + kMT * v + t
    f32x4 out[kMT];
#pragma unroll
    for (int v = 0; v < 4; ++v)
#pragma unroll
        for (int tt = 0; tt < kMT; ++tt) {
            const int cc = kMT * v + tt;
            out[cc >> 2][cc & 3] = d[tt][v];
        }
    if (kEpi) {
        const int o = row_obj[r];
        const double f1 = cs.coef[(size_t)o * cs.stride + 2 * cs.step - 1];
        const double f2 = cs.coef[(size_t)o * cs.stride + 2 * cs.step];
        const double dv = (double)cs.dinv[r];
#pragma unroll
        for (int h = 0; h < kMT; ++h) {
            f32x4 rv1, dz1, w1;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const double rv = (double)er[h][q] - dv * (double)out[h][q];
                const double dz = f1 * (double)ez[h][q] + f2 * rv;
                rv1[q] = (float)rv;
                dz1[q] = (float)dz;
                w1[q] = (float)((double)ew[h][q] + dz);
            }
            *(f32x4 *)(cs.R + r * ldo + c0 + 4 * h) = rv1;
            *(f32x4 *)(cs.dz_out + r * ldo + c0 + 4 * h) = dz1;
            *(f32x4 *)(cs.W + r * cs.ldw + c0 + 4 * h) = w1;
        }
    } else {
#pragma unroll
        for (int h = 0; h < kMT; ++h) *(f32x4 *)(HY + r * ldo + c0 + 4 * h) = out[h];
    }
}

bool t16_ok(int m, int64_t ldy, int64_t ldo) {
    return (m == 32 || m == 64 || (m % 4 == 0 && m >= 4 && m <= 16)) && ldy % 4 == 0 && ldo % 4 == 0;
}

template <bool kEpi>
int launch_t16(ff_ctx *ctx, hipStream_t st, const RT16View &v, int sub, int m, const float *Y, int64_t ldy, float *HY,
               int64_t ldo, const int *row_obj, const int *status, const ChebStep<float> &cs) {
#define FF_T16(MT, W, B, A, O, P)                                                                            \
    hipLaunchKernelGGL((spmm_t16_kernel<kEpi, MT, W, B, A, O, P>), dim3(grid_for(v.ntiles, W)), dim3(64 * W), 0, \
                       st, v.n, v.ntiles, v.tptr, v.tcol, v.vh, Y, ldy, HY, ldo, m, row_obj, status, cs)
    const int mt = m <= 16 ? 1 : m / 16;
    if (mt == 1) {
        FF_T16(1, 4, 4, 1, 4, false);
    } else if (mt == 2) {
        // measured on the benchmark workload: 1.38 / 1.43 / 1.47 ms
        switch (sub) {
            case 1: FF_T16(2, 4, 8, 1, 4, false); break;
            case 2: FF_T16(2, 4, 16, 1, 1, true); break;
            default: FF_T16(2, 2, 16, 1, 4, false); break;
        }
    } else {
        FF_T16(4, 4, 2, 1, 4, false);
    }
#undef FF_T16
    FF_CHECK_LAUNCH(ctx);
    return FF_OK;
}

int spmm_h_t16(ff_ctx *ctx, hipStream_t st, const RT16View &v, int sub, int m, const float *Y, int64_t ldy, float *HY,
               int64_t ldo, const int *row_obj, const int *status) {
    FF_REQUIRE(ctx, v.vh != nullptr && t16_ok(m, ldy, ldo), "sixteen-row tiles: bad copy or block shape (m = %d)", m);
    return launch_t16<false>(ctx, st, v, sub, m, Y, ldy, HY, ldo, row_obj, status, ChebStep<float>{});
}

int cheb_step_t16(ff_ctx *ctx, hipStream_t st, const RT16View &v, int sub, int m, const float *DZ, int64_t ld,
                  const int *row_obj, const int *status, const ChebStep<float> &cs) {
    FF_REQUIRE(ctx, v.vh != nullptr && row_obj != nullptr && t16_ok(m, ld, ld) && cs.ldw % 4 == 0,
               "sixteen-row tiles: bad copy or block shape (m = %d)", m);
    return launch_t16<true>(ctx, st, v, sub, m, DZ, ld, nullptr, ld, row_obj, status, cs);
}

int build_t16_ws(ff_ctx *ctx, hipStream_t st, int64_t n, const int64_t *row_ptr, const int32_t *col, const double *H,
                 RT16View *out) {
    FF_REQUIRE(ctx, n > 0 && row_ptr && col && H && out, "bad arguments");
    const int64_t ntiles = (n + kTile16 - 1) / kTile16;
    int64_t *cnt = (int64_t *)ws_get(ctx, WS_RT16_CNT, (size_t)(ntiles + 1) * sizeof(int64_t));
    int64_t *tptr = (int64_t *)ws_get(ctx, WS_RT16_PTR, (size_t)(ntiles + 1) * sizeof(int64_t));
    if (!cnt || !tptr) return FF_ERR_OOM;
    int64_t entries = 0;
    int cap = 0, bits = 0;
    int rc = build_ptr_union<kTile16>(ctx, st, n, row_ptr, col, cnt, tptr, ntiles, &entries, &cap, &bits);
    if (rc) return rc;
    const size_t ne = (size_t)std::max<int64_t>(entries, 1);
    int32_t *tcol = (int32_t *)ws_get(ctx, WS_RT16_COL, ne * sizeof(int32_t));
    float *vh = (float *)ws_get(ctx, WS_RT16_VAL, ne * kTile16 * sizeof(float));
    if (!tcol || !vh) return FF_ERR_OOM;
    if ((rc = fill_union<kTile16>(ctx, st, n, ntiles, row_ptr, col, cap, bits, H, tptr, tcol, vh))) return rc;
    out->n = n;
    out->ntiles = ntiles;
    out->entries = entries;
    out->tptr = tptr;
    out->tcol = tcol;
    out->vh = vh;
    return FF_OK;
}

// ---------------------------------------------------------------------------
// Fused [H, M] Y on the eight-row [H, M] copy, on FP64 MFMA
// ---------------------------------------------------------------------------
//
// Per tile (HY; MY)[16 outputs][columns] = V[16 outputs][entries] . Y[entries]
// [columns], the 16 outputs being H of the tile's eight rows and M of the same
// rows. v_mfma_f64_16x16x4f64 takes the outputs as its A/D row index and 16
// column slots as the B/D column index (slot j of MFMA t is column kMT j + t),
// so a lane reads kMT consecutive floats of a gathered row with one load. The
// FP32 values and block entries are exact in FP64 and the sums accumulate in
// FP64, as in the VALU kernel; the VALU keeps only the conversions and the
// address arithmetic. Lanes with the same output write one contiguous row.
struct ChunkHM8 {
    int32_t j;
    f32x4 v[4];                                    // H rows 0..3, 4..7, M rows 0..3, 4..7
    __device__ void load(const int32_t *tcol, const float *vh, const float *vm, int64_t e, bool in) {
        j = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q) v[q] = f32x4{0.f, 0.f, 0.f, 0.f};
        if (in) {
            j = __builtin_nontemporal_load(tcol + e);
            v[0] = __builtin_nontemporal_load((const f32x4 *)(vh + e * 8));
            v[1] = __builtin_nontemporal_load((const f32x4 *)(vh + e * 8 + 4));
            v[2] = __builtin_nontemporal_load((const f32x4 *)(vm + e * 8));
            v[3] = __builtin_nontemporal_load((const f32x4 *)(vm + e * 8 + 4));
        }
    }
    __device__ void stage(float *sv, int lane) const {
#pragma unroll
        for (int q = 0; q < 4; ++q) *(f32x4 *)(sv + lane * 16 + 4 * q) = v[q];
    }
};

typedef double f64x4r __attribute__((ext_vector_type(4)));
__device__ inline f64x4r mfma64(double a, double b, f64x4r c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

template <int kMT, int kBatch, bool kF32>
__device__ __forceinline__ void hm8_chunk(ChunkHM8 &ch, int64_t base, int64_t e1, const int32_t *tcol,
                                          const float *vh, const float *vm, float *sv, int lane, int li, int lk, int m,
                                          const float *Y, int64_t ldy, f64x4r (&d)[kMT]) {
    typedef typename YVec<kMT>::type YV;
    const int cnt = (int)(e1 - base < 64 ? e1 - base : 64);
    const int32_t jc = ch.j;
    __builtin_amdgcn_wave_barrier();
    ch.stage(sv, lane);
    __builtin_amdgcn_wave_barrier();
    ch.load(tcol, vh, vm, base + 64 + lane, base + 64 + lane < e1);
    // entries past the chunk's end have column 0 and zero values, and a masked slot (m < 16)
    // reads column 0: every load is valid, so none carries a per-lane condition
    const int col = kMT * (kMT > 1 || li < m ? li : 0);
    const int nq = (cnt + 3) >> 2;
    for (int q0 = 0; q0 < nq; q0 += kBatch) {
        YV y[kBatch];
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
            if (q0 + u < nq) {
                const int e = 4 * (q0 + u) + lk;
                const uint32_t j = (uint32_t)__shfl(jc, e, 64);
                y[u] = *(const YV *)(Y + (size_t)(j * (uint32_t)ldy) + col);
            }
        }
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
            if (q0 + u < nq) {
                const int e = 4 * (q0 + u) + lk;
                if (kF32) {
                    // each step of four entries on the FP32 matrix cores from a zero accumulator, its
                    // sums added in FP64: a step rounds once at 2^-24 of its terms, the order of the
                    // FP32 rounding of the stored values themselves
                    const float a = sv[e * 16 + li];
#pragma unroll
                    for (int t = 0; t < kMT; ++t) {
                        const f32x4 p = __builtin_amdgcn_mfma_f32_16x16x4f32(a, yget(y[u], t),
                                                                            f32x4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
#pragma unroll
                        for (int v = 0; v < 4; ++v) d[t][v] += (double)p[v];
                    }
                } else {
                    const double a = (double)sv[e * 16 + li];
#pragma unroll
                    for (int t = 0; t < kMT; ++t) d[t] = mfma64(a, (double)yget(y[u], t), d[t]);
                }
            }
        }
    }
}

template <int kMT, int kWaves, int kBatch, int kOcc, bool kF32>
__global__ void __launch_bounds__(64 * kWaves) __attribute__((amdgpu_waves_per_eu(kOcc, 8)))
spmm_hm8_kernel(int64_t nrows, int64_t ntiles, const int64_t *tptr, const int32_t *tcol, const float *vh,
                const float *vm, const float *Y, int64_t ldy, float *HY, float *MY, int64_t ldo, int m,
                const int *row_obj, const int *obj_status) {
    __shared__ __align__(16) float svals[kWaves][64 * 16];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t t = (int64_t)xcd_remap(blockIdx.x, gridDim.x) * kWaves + wv;
    if (t >= ntiles) return;
    const int li = lane & 15, lk = lane >> 4;
    const int64_t r0 = t * kTile8;
    bool any = false;
#pragma unroll
    for (int i = 0; i < kTile8; ++i)
        any = any || (r0 + i < nrows && (!obj_status || obj_status[row_obj[r0 + i]] == 0));
    if (!any) return;
    float *sv = svals[wv];
    const int64_t e0 = tptr[t], e1 = tptr[t + 1];
    f64x4r d[kMT];
#pragma unroll
    for (int q = 0; q < kMT; ++q) d[q] = f64x4r{0.0, 0.0, 0.0, 0.0};
    ChunkHM8 ch;
    ch.load(tcol, vh, vm, e0 + lane, e0 + lane < e1);
    for (int64_t base = e0; base < e1; base += 64)
        hm8_chunk<kMT, kBatch, kF32>(ch, base, e1, tcol, vh, vm, sv, lane, li, lk, m, Y, ldy, d);
    if (kMT == 1 && li >= m) return;
    // lane holds D[o][li] for v = 0..3 with o = 4 v + lk on the FP64 matrix cores and o = 4 lk + v on the
    // FP32 ones (their result layouts differ); outputs o: H rows 0..7, then M rows 0..7; columns kMT li + t
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int o = kF32 ? 4 * lk + v : 4 * v + lk;
        const int64_t r = r0 + (o & 7);
        if (r >= nrows || (obj_status && obj_status[row_obj[r]] != 0)) continue;
        float *dst = (o < 8 ? HY : MY) + r * ldo + kMT * li;
        if (kMT == 1) {
            dst[0] = (float)d[0][v];
        } else if (kMT == 2) {
            *(float2 *)dst = make_float2((float)d[0][v], (float)d[1][v]);
        } else {
            *(f32x4 *)dst = f32x4{(float)d[0][v], (float)d[1][v], (float)d[2][v], (float)d[3][v]};
        }
    }
}

// The same product with its loads pipelined. Vector loads retire in order, so above the wait for a
// batch's gathers also waits for the next chunk's columns and values, issued just before them. Here
// a chunk's columns and values are loaded two batches ahead of their use and each batch of eight
// quads (32 entries) is gathered while the previous one is multiplied:
//   chunk c: stage values(c) in LDS; gather batch 2c+1; multiply batch 2c; gather batch 2c+2
//   (columns of chunk c+1); load columns and values of chunk c+2; multiply batch 2c+1.
// The MFMA sequence (entries in order, one accumulator per column group) is that of the kernel above.
// With kF32 and kChain > 1 the FP32 matrix-core steps accumulate kChain four-entry steps in FP32 before
// each FP64 addition (a bound of about 4 kChain units of FP32 rounding of the summed magnitudes, the
// order of the rounding of the FP32 values themselves), which divides the FP64 additions by kChain.
template <int kMT, int kWaves, int kOcc, bool kF32, int kChain = 1>
__global__ void __launch_bounds__(64 * kWaves) __attribute__((amdgpu_waves_per_eu(kOcc, 8)))
spmm_hm8p_kernel(int64_t nrows, int64_t ntiles, const int64_t *tptr, const int32_t *tcol, const float *vh,
                 const float *vm, const float *Y, int64_t ldy, float *HY, float *MY, int64_t ldo, int m,
                 const int *row_obj, const int *obj_status) {
    typedef typename YVec<kMT>::type YV;
    constexpr int kB = 8;                          // quads (of four entries) per batch
    __shared__ __align__(16) float svals[kWaves][64 * 16];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t t = (int64_t)xcd_remap(blockIdx.x, gridDim.x) * kWaves + wv;
    if (t >= ntiles) return;
    const int li = lane & 15, lk = lane >> 4;
    const int64_t r0 = t * kTile8;
    bool any = false;
#pragma unroll
    for (int i = 0; i < kTile8; ++i)
        any = any || (r0 + i < nrows && (!obj_status || obj_status[row_obj[r0 + i]] == 0));
    if (!any) return;
    float *sv = svals[wv];
    const int64_t e0 = tptr[t], e1 = tptr[t + 1];
    const int nch = (int)((e1 - e0 + 63) >> 6);
    const int col = kMT * (kMT > 1 || li < m ? li : 0);
    f64x4r d[kMT];
#pragma unroll
    for (int q = 0; q < kMT; ++q) d[q] = f64x4r{0.0, 0.0, 0.0, 0.0};
    // quads of chunk c: entries past the tile's end have column 0 and zero values
    auto nquads = [&](int c) __attribute__((always_inline)) -> int {
        const int64_t cnt = e1 - e0 - 64 * (int64_t)c;
        return cnt >= 64 ? 16 : (int)((cnt + 3) >> 2);
    };
    // a chunk's columns and values without a branch: the index is clamped to the tile's last entry and
    // the lanes past the end take column 0 and zero values where they are used (staging, gathers), so
    // that no instruction touches the loaded registers before then
    struct Chunk {
        int32_t j;
        f32x4 v[4];
        bool in;
    };
    auto load_chunk = [&](Chunk &ch, int c) __attribute__((always_inline)) {
        const int64_t e = e0 + 64 * (int64_t)c + lane;
        ch.in = e < e1;
        const int64_t ec = ch.in ? e : e1 - 1;
        __builtin_amdgcn_sched_barrier(0);
        ch.j = __builtin_nontemporal_load(tcol + ec);
        ch.v[0] = __builtin_nontemporal_load((const f32x4 *)(vh + ec * 8));
        ch.v[1] = __builtin_nontemporal_load((const f32x4 *)(vh + ec * 8 + 4));
        ch.v[2] = __builtin_nontemporal_load((const f32x4 *)(vm + ec * 8));
        ch.v[3] = __builtin_nontemporal_load((const f32x4 *)(vm + ec * 8 + 4));
        __builtin_amdgcn_sched_barrier(0);
    };
    auto stage = [&](const Chunk &ch) __attribute__((always_inline)) {
#pragma unroll
        for (int q = 0; q < 4; ++q)
            *(f32x4 *)(sv + lane * 16 + 4 * q) = ch.in ? ch.v[q] : f32x4{0.f, 0.f, 0.f, 0.f};
    };
    // batch h (0 or 1) of a chunk whose columns are jc; every quad is gathered (past the end: row 0)
    auto gather = [&](YV (&y)[kB], const Chunk &ch, int h) __attribute__((always_inline)) {
        const int32_t jc = ch.in ? ch.j : 0;
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int u = 0; u < kB; ++u) {
            const uint32_t j = (uint32_t)__shfl(jc, 4 * (kB * h + u) + lk, 64);
            y[u] = *(const YV *)(Y + (size_t)(j * (uint32_t)ldy) + col);
        }
        __builtin_amdgcn_sched_barrier(0);
    };
    // the quads below nq (all of them when full)
    auto multiply = [&](const YV (&y)[kB], int h, int nq, bool full) __attribute__((always_inline)) {
        f32x4 pc[kMT];                             // the FP32 chain (kChain > 1)
#pragma unroll
        for (int tt = 0; tt < kMT; ++tt) pc[tt] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int u = 0; u < kB; ++u) {
            if (full || kB * h + u < nq) {
                const int e = 4 * (kB * h + u) + lk;
                if (kF32 && kChain > 1) {
                    const float a = sv[e * 16 + li];
#pragma unroll
                    for (int tt = 0; tt < kMT; ++tt)
                        pc[tt] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, yget(y[u], tt), pc[tt], 0, 0, 0);
                } else if (kF32) {
                    const float a = sv[e * 16 + li];
#pragma unroll
                    for (int tt = 0; tt < kMT; ++tt) {
                        const f32x4 p = __builtin_amdgcn_mfma_f32_16x16x4f32(a, yget(y[u], tt),
                                                                            f32x4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
#pragma unroll
                        for (int v = 0; v < 4; ++v) d[tt][v] += (double)p[v];
                    }
                } else {
                    const double a = (double)sv[e * 16 + li];
#pragma unroll
                    for (int tt = 0; tt < kMT; ++tt) d[tt] = mfma64(a, (double)yget(y[u], tt), d[tt]);
                }
            }
            if (kF32 && kChain > 1 && (u % kChain == kChain - 1 || u == kB - 1)) {
#pragma unroll
                for (int tt = 0; tt < kMT; ++tt) {
#pragma unroll
                    for (int v = 0; v < 4; ++v) d[tt][v] += (double)pc[tt][v];
                    pc[tt] = f32x4{0.f, 0.f, 0.f, 0.f};
                }
            }
        }
    };
    // chunk c: cur holds its columns and values, nxt those of chunk c + 1; cur is then reloaded with
    // chunk c + 2. steady: chunk c is whole and chunks c + 1 and c + 2 exist (no branch)
    YV ya[kB], yb[kB];
    auto step = [&](int c, Chunk &cur, Chunk &nxt, bool steady) __attribute__((always_inline)) {
        const int nq = steady ? 16 : nquads(c);
        __builtin_amdgcn_wave_barrier();
        stage(cur);
        __builtin_amdgcn_wave_barrier();
        if (steady || nq > kB) gather(yb, cur, 1);
        multiply(ya, 0, nq, steady);
        if (steady || c + 1 < nch) gather(ya, nxt, 0);
        if (steady || c + 2 < nch) load_chunk(cur, c + 2);
        if (steady || nq > kB) multiply(yb, 1, nq, steady);
    };
    if (nch > 0) {
        Chunk pa, pb;
        load_chunk(pa, 0);
        if (nch > 1) load_chunk(pb, 1);
        gather(ya, pa, 0);
        int c = 0;
        for (; c + 3 < nch; c += 2) {
            step(c, pa, pb, true);
            step(c + 1, pb, pa, true);
        }
        // the last one to three chunks
        step(c, pa, pb, false);
        if (c + 1 < nch) step(c + 1, pb, pa, false);
        if (c + 2 < nch) step(c + 2, pa, pb, false);
    }
    if (kMT == 1 && li >= m) return;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int o = kF32 ? 4 * lk + v : 4 * v + lk;
        const int64_t r = r0 + (o & 7);
        if (r >= nrows || (obj_status && obj_status[row_obj[r]] != 0)) continue;
        float *dst = (o < 8 ? HY : MY) + r * ldo + kMT * li;
        if (kMT == 1) {
            dst[0] = (float)d[0][v];
        } else if (kMT == 2) {
            *(float2 *)dst = make_float2((float)d[0][v], (float)d[1][v]);
        } else {
            *(f32x4 *)dst = f32x4{(float)d[0][v], (float)d[1][v], (float)d[2][v], (float)d[3][v]};
        }
    }
}

// The pipelined [H, M] product of spmm_hm8p_kernel (FP64 matrix cores) reading the zero-free copy
// of the eight-row tiles: per union entry a byte mask of the tile rows present and, in entry order,
// their (H, M) value pairs. The columns and masks of a chunk of 64 entries are loaded two chunks
// ahead and its pairs one chunk ahead (so waiting for a mask waits only for loads that were needed
// already); each lane reads the 64 bytes from its entry's first pair (its pairs and, past them,
// its neighbours', which it does not use), the wave's prefix count of present rows locating them,
// and rebuilds the entry in LDS as the full tiles hold it: row r's pair is the one at the count of
// mask bits below r (zeros when the bit is clear). The same operands as from the full tiles, so the
// same sums bit for bit.
template <int kMT, int kWaves, int kOcc>
__global__ void __launch_bounds__(64 * kWaves) __attribute__((amdgpu_waves_per_eu(kOcc, 8)))
spmm_hm8z_kernel(int64_t nrows, int64_t ntiles, const int64_t *tptr, const int32_t *tcol, const uint8_t *m8,
                 const int64_t *poff, const float *pv, const float *Y, int64_t ldy, float *HY, float *MY, int64_t ldo,
                 int m, const int *row_obj, const int *obj_status) {
    typedef typename YVec<kMT>::type YV;
    constexpr int kB = 8;                          // quads (of four entries) per batch
    __shared__ __align__(16) float sraw[kWaves][64 * 16];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t t = (int64_t)xcd_remap(blockIdx.x, gridDim.x) * kWaves + wv;
    if (t >= ntiles) return;
    const int li = lane & 15, lk = lane >> 4;
    const int64_t r0 = t * kTile8;
    bool any = false;
#pragma unroll
    for (int i = 0; i < kTile8; ++i)
        any = any || (r0 + i < nrows && (!obj_status || obj_status[row_obj[r0 + i]] == 0));
    if (!any) return;
    float *sv = sraw[wv];
    const int64_t e0 = tptr[t], e1 = tptr[t + 1];
    const int nch = (int)((e1 - e0 + 63) >> 6);
    const int col = kMT * (kMT > 1 || li < m ? li : 0);
    int64_t pbase = poff[t];                       // first pair of the next chunk whose pairs are loaded
    f64x4r d[kMT];
#pragma unroll
    for (int q = 0; q < kMT; ++q) d[q] = f64x4r{0.0, 0.0, 0.0, 0.0};
    auto nquads = [&](int c) __attribute__((always_inline)) -> int {
        const int64_t cnt = e1 - e0 - 64 * (int64_t)c;
        return cnt >= 64 ? 16 : (int)((cnt + 3) >> 2);
    };
    struct Chunk {
        int32_t j;
        uint32_t mk;
        bool in;
        f32x4 v[4];
    };
    // columns and masks of chunk c (lanes past the tile's end: the last entry's column, no rows)
    auto load_cols = [&](Chunk &ch, int c) __attribute__((always_inline)) {
        const int64_t e = e0 + 64 * (int64_t)c + lane;
        ch.in = e < e1;
        const int64_t ec = ch.in ? e : e1 - 1;
        __builtin_amdgcn_sched_barrier(0);
        ch.j = __builtin_nontemporal_load(tcol + ec);
        ch.mk = (uint32_t)m8[ec];
        __builtin_amdgcn_sched_barrier(0);
    };
    // the pairs of the chunk whose masks ch holds: 64 bytes from the lane's first pair
    auto load_vals = [&](Chunk &ch) __attribute__((always_inline)) {
        const uint32_t mk = ch.in ? ch.mk : 0u;
        const int cnt = __popc(mk);
        int incl = cnt;
#pragma unroll
        for (int dd = 1; dd < 64; dd <<= 1) {
            const int v = __shfl_up(incl, dd, 64);
            if (lane >= dd) incl += v;
        }
        const float *src = pv + 2 * (pbase + incl - cnt);
        pbase += __shfl(incl, 63, 64);
        __builtin_amdgcn_sched_barrier(0);
        // pairs are 8-byte aligned: 16-byte loads at 8-byte alignment (the hardware takes dword alignment)
        typedef float f32x4a8 __attribute__((ext_vector_type(4), aligned(8)));
#pragma unroll
        for (int q = 0; q < 4; ++q) ch.v[q] = __builtin_nontemporal_load((const f32x4a8 *)(src + 4 * q));
        __builtin_amdgcn_sched_barrier(0);
    };
    // the lane's entry laid out as the full tiles' (H rows 0-7, M rows 0-7, zeros for absent rows) in
    // its LDS area: its pairs are written there, read back by rank, and the expanded entry written
    // over them (only the lane touches its area here)
    auto stage = [&](const Chunk &ch) __attribute__((always_inline)) {
        float *a = sv + lane * 16;
#pragma unroll
        for (int q = 0; q < 4; ++q) *(f32x4 *)(a + 4 * q) = ch.v[q];
        const uint32_t mk = ch.in ? ch.mk : 0u;
        float hv[8], mv[8];
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            const float2 pr = *(const float2 *)(a + 2 * __popc(mk & ((1u << r) - 1u)));
            const bool on = (mk >> r) & 1u;
            hv[r] = on ? pr.x : 0.f;
            mv[r] = on ? pr.y : 0.f;
        }
        *(f32x4 *)(a + 0) = f32x4{hv[0], hv[1], hv[2], hv[3]};
        *(f32x4 *)(a + 4) = f32x4{hv[4], hv[5], hv[6], hv[7]};
        *(f32x4 *)(a + 8) = f32x4{mv[0], mv[1], mv[2], mv[3]};
        *(f32x4 *)(a + 12) = f32x4{mv[4], mv[5], mv[6], mv[7]};
    };
    auto gather = [&](YV (&y)[kB], const Chunk &ch, int h) __attribute__((always_inline)) {
        const int32_t jc = ch.in ? ch.j : 0;
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int u = 0; u < kB; ++u) {
            const uint32_t j = (uint32_t)__shfl(jc, 4 * (kB * h + u) + lk, 64);
            y[u] = *(const YV *)(Y + (size_t)(j * (uint32_t)ldy) + col);
        }
        __builtin_amdgcn_sched_barrier(0);
    };
    auto multiply = [&](const YV (&y)[kB], int h, int nq, bool full) __attribute__((always_inline)) {
#pragma unroll
        for (int u = 0; u < kB; ++u) {
            if (full || kB * h + u < nq) {
                const int e = 4 * (kB * h + u) + lk;
                const double a = (double)sv[e * 16 + li];
#pragma unroll
                for (int tt = 0; tt < kMT; ++tt) d[tt] = mfma64(a, (double)yget(y[u], tt), d[tt]);
            }
        }
    };
    // chunk c: cur holds its columns, masks and pairs, nxt the columns and masks of chunk c + 1, whose
    // pairs are loaded here; cur is then reloaded with the columns of chunk c + 2
    YV ya[kB], yb[kB];
    auto step = [&](int c, Chunk &cur, Chunk &nxt, bool steady) __attribute__((always_inline)) {
        const int nq = steady ? 16 : nquads(c);
        __builtin_amdgcn_wave_barrier();
        stage(cur);
        __builtin_amdgcn_wave_barrier();
        if (steady || nq > kB) gather(yb, cur, 1);
        multiply(ya, 0, nq, steady);
        if (steady || c + 1 < nch) {
            gather(ya, nxt, 0);
            load_vals(nxt);
        }
        if (steady || c + 2 < nch) load_cols(cur, c + 2);
        if (steady || nq > kB) multiply(yb, 1, nq, steady);
    };
    if (nch > 0) {
        Chunk pa, pb;
        load_cols(pa, 0);
        if (nch > 1) load_cols(pb, 1);
        load_vals(pa);
        gather(ya, pa, 0);
        int c = 0;
        for (; c + 3 < nch; c += 2) {
            step(c, pa, pb, true);
            step(c + 1, pb, pa, true);
        }
        step(c, pa, pb, false);
        if (c + 1 < nch) step(c + 1, pb, pa, false);
        if (c + 2 < nch) step(c + 2, pa, pb, false);
    }
    if (kMT == 1 && li >= m) return;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int o = 4 * v + lk;
        const int64_t r = r0 + (o & 7);
        if (r >= nrows || (obj_status && obj_status[row_obj[r]] != 0)) continue;
        float *dst = (o < 8 ? HY : MY) + r * ldo + kMT * li;
        if (kMT == 1) {
            dst[0] = (float)d[0][v];
        } else if (kMT == 2) {
            *(float2 *)dst = make_float2((float)d[0][v], (float)d[1][v]);
        } else {
            *(f32x4 *)dst = f32x4{(float)d[0][v], (float)d[1][v], (float)d[2][v], (float)d[3][v]};
        }
    }
}

// value pairs present in each tile's entries (a row is present when its H or its M value is not +-0)
__global__ void __launch_bounds__(64) t8z_count_kernel(int64_t ntiles, const int64_t *tptr, const float *vh,
                                                       const float *vm, int64_t *cnt) {
    const int64_t t = blockIdx.x;
    if (t >= ntiles) return;
    int c = 0;
    for (int64_t e = tptr[t] + threadIdx.x; e < tptr[t + 1]; e += 64)
#pragma unroll
        for (int r = 0; r < 8; ++r) c += (vh[e * 8 + r] != 0.f || vm[e * 8 + r] != 0.f);
#pragma unroll
    for (int dd = 32; dd >= 1; dd >>= 1) c += __shfl_xor(c, dd, 64);
    if (threadIdx.x == 0) cnt[t] = c;
}

// one 64-thread block per tile, an entry per lane per chunk of 64: its mask and its present pairs,
// placed by the prefix count over the chunk's lanes after the tile's earlier chunks
__global__ void __launch_bounds__(64) t8z_fill_kernel(int64_t ntiles, const int64_t *tptr, const float *vh,
                                                      const float *vm, const int64_t *poff, uint8_t *m8, float *pv) {
    const int64_t t = blockIdx.x;
    if (t >= ntiles) return;
    const int lane = threadIdx.x;
    int64_t run = poff[t];
    for (int64_t base = tptr[t]; base < tptr[t + 1]; base += 64) {
        const int64_t e = base + lane;
        const bool in = e < tptr[t + 1];
        uint32_t mk = 0;
        if (in)
#pragma unroll
            for (int r = 0; r < 8; ++r) mk |= (vh[e * 8 + r] != 0.f || vm[e * 8 + r] != 0.f) ? (1u << r) : 0u;
        const int cnt = __popc(mk);
        int incl = cnt;
#pragma unroll
        for (int dd = 1; dd < 64; dd <<= 1) {
            const int v = __shfl_up(incl, dd, 64);
            if (lane >= dd) incl += v;
        }
        if (in) {
            m8[e] = (uint8_t)mk;
            int64_t o = run + incl - cnt;
            for (int r = 0; r < 8; ++r)
                if ((mk >> r) & 1u) {
                    pv[2 * o] = vh[e * 8 + r];
                    pv[2 * o + 1] = vm[e * 8 + r];
                    ++o;
                }
        }
        run += __shfl(incl, 63, 64);
    }
}

int build_t8z_ws(ff_ctx *ctx, hipStream_t st, RT8View *v) {
    FF_REQUIRE(ctx, v && v->vh && v->vm && v->tptr && v->ntiles > 0, "zero-free [H, M] tiles: no eight-row copy");
    int64_t *cnt = (int64_t *)ws_get(ctx, WS_T8Z_CNT, (size_t)(v->ntiles + 1) * sizeof(int64_t));
    int64_t *poff = (int64_t *)ws_get(ctx, WS_T8Z_OFF, (size_t)(v->ntiles + 1) * sizeof(int64_t));
    uint8_t *m8 = (uint8_t *)ws_get(ctx, WS_T8Z_MASK, (size_t)std::max<int64_t>(v->entries, 1));
    if (!cnt || !poff || !m8) return FF_ERR_OOM;
    hipLaunchKernelGGL(t8z_count_kernel, dim3(v->ntiles), dim3(64), 0, st, v->ntiles, v->tptr, v->vh, v->vm, cnt);
    FF_CHECK_LAUNCH(ctx);
    int rc = scan_exclusive_i64(ctx, cnt, poff, v->ntiles);
    if (rc) return rc;
    int64_t *h = (int64_t *)pinned_get(ctx, 64);
    if (!h) return FF_ERR_OOM;
    FF_HIP(ctx, hipMemcpyAsync(h, poff + v->ntiles, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    FF_HIP(ctx, hipStreamSynchronize(st));
    const int64_t total = h[0];
    // sixteen floats of padding: the last lanes read 64 bytes from their first pair
    float *pv = (float *)ws_get(ctx, WS_T8Z_VAL, (size_t)(2 * total + 16) * sizeof(float));
    if (!pv) return FF_ERR_OOM;
    FF_HIP(ctx, hipMemsetAsync(pv + 2 * total, 0, 16 * sizeof(float), st));
    hipLaunchKernelGGL(t8z_fill_kernel, dim3(v->ntiles), dim3(64), 0, st, v->ntiles, v->tptr, v->vh, v->vm,
                       (const int64_t *)poff, m8, pv);
    FF_CHECK_LAUNCH(ctx);
    v->m8 = m8;
    v->poff = poff;
    v->pv = pv;
    return FF_OK;
}

bool hm8_ok(int m, int64_t ldy, int64_t ldo) { return t16_ok(m, ldy, ldo); }

int spmm_hm8(ff_ctx *ctx, hipStream_t st, const RT8View &v, int sub, int m, const float *Y, int64_t ldy, float *HY,
             float *MY, int64_t ldo, const int *row_obj, const int *status) {
    FF_REQUIRE(ctx, v.vh != nullptr && v.vm != nullptr && hm8_ok(m, ldy, ldo),
               "eight-row [H, M] tiles: bad copy or block shape (m = %d)", m);
    FF_REQUIRE(ctx, off32_ok(v.n, ldy), "block of %lld rows x %lld too large for 32-bit row offsets", (long long)v.n,
               (long long)ldy);
#define FF_HM8(MT, W, B, O, F)                                                                                \
    hipLaunchKernelGGL((spmm_hm8_kernel<MT, W, B, O, F>), dim3(grid_for(v.ntiles, W)), dim3(64 * W), 0, st, v.n, \
                       v.ntiles, v.tptr, v.tcol, v.vh, v.vm, Y, ldy, HY, MY, ldo, m, row_obj, status)
#define FF_HM8P(MT, W, O, F)                                                                                  \
    hipLaunchKernelGGL((spmm_hm8p_kernel<MT, W, O, F>), dim3(grid_for(v.ntiles, W)), dim3(64 * W), 0, st, v.n, \
                       v.ntiles, v.tptr, v.tcol, v.vh, v.vm, Y, ldy, HY, MY, ldo, m, row_obj, status)
#define FF_HM8PC(MT, W, O, C)                                                                                 \
    hipLaunchKernelGGL((spmm_hm8p_kernel<MT, W, O, true, C>), dim3(grid_for(v.ntiles, W)), dim3(64 * W), 0, st, \
                       v.n, v.ntiles, v.tptr, v.tcol, v.vh, v.vm, Y, ldy, HY, MY, ldo, m, row_obj, status)
    // sub 0..2: FP64 matrix cores; 3, 4: FP32 matrix cores with FP64 accumulation of each four-entry step;
    // 5, 6: the pipelined kernel on the FP64 and the FP32 matrix cores; 7: the former with two waves per
    // workgroup at m = 32 (as 5 at other widths); 8, 9: the pipelined kernel on the FP64 matrix cores from
    // the zero-free copy, two and four waves per workgroup
    // 10: the pipelined kernel on the FP32 matrix cores with four four-entry steps chained in FP32 before
    // each FP64 addition, two waves per workgroup
    FF_REQUIRE(ctx, sub >= 0 && sub < kHm8Subs, "launch shape %d out of range", sub);
    const int mt = m <= 16 ? 1 : m / 16;
    if (sub == 10) {
        if (mt == 1) FF_HM8PC(1, 2, 2, 4);
        else if (mt == 2) FF_HM8PC(2, 2, 2, 4);
        else FF_HM8PC(4, 2, 2, 4);
        FF_CHECK_LAUNCH(ctx);
        return FF_OK;
    }
    if (sub == 8 || sub == 9) {
        FF_REQUIRE(ctx, v.m8 && v.poff && v.pv, "launch shape %d needs the zero-free copy", sub);
#define FF_HM8Z(MT, W, O)                                                                                        \
    hipLaunchKernelGGL((spmm_hm8z_kernel<MT, W, O>), dim3(grid_for(v.ntiles, W)), dim3(64 * W), 0, st, v.n,       \
                       v.ntiles, v.tptr, v.tcol, v.m8, v.poff, v.pv, Y, ldy, HY, MY, ldo, m, row_obj, status)
        const bool two = sub == 8;
        if (mt == 1) {
            if (two) FF_HM8Z(1, 2, 2); else FF_HM8Z(1, 4, 2);
        } else if (mt == 2) {
            if (two) FF_HM8Z(2, 2, 2); else FF_HM8Z(2, 4, 2);
        } else {
            if (two) FF_HM8Z(4, 2, 2); else FF_HM8Z(4, 4, 2);
        }
#undef FF_HM8Z
        FF_CHECK_LAUNCH(ctx);
        return FF_OK;
    }
    if (sub >= 5) {
        const bool f32p = sub == 6;
        if (mt == 1) {
            if (f32p) FF_HM8P(1, 4, 2, true); else FF_HM8P(1, 4, 2, false);
        } else if (mt == 2) {
            if (sub == 7) FF_HM8P(2, 2, 2, false);
            else if (f32p) FF_HM8P(2, 4, 2, true);
            else FF_HM8P(2, 4, 2, false);
        } else {
            if (f32p) FF_HM8P(4, 4, 2, true); else FF_HM8P(4, 4, 2, false);
        }
        FF_CHECK_LAUNCH(ctx);
        return FF_OK;
    }
#undef FF_HM8P
#undef FF_HM8PC
    const bool f32 = sub >= 3;
    if (mt == 1) {
        if (f32) FF_HM8(1, 4, 8, 4, true); else FF_HM8(1, 4, 8, 4, false);
    } else if (mt == 2) {
        switch (sub) {
            case 1: FF_HM8(2, 2, 8, 4, false); break;
            case 2: FF_HM8(2, 4, 4, 6, false); break;
            case 3: FF_HM8(2, 4, 8, 4, true); break;
            case 4: FF_HM8(2, 2, 8, 4, true); break;
            default: FF_HM8(2, 4, 8, 4, false); break;
        }
    } else {
        if (f32) {
            if (sub == 4) FF_HM8(4, 2, 4, 4, true); else FF_HM8(4, 4, 4, 4, true);
        } else {
            if (sub == 1) FF_HM8(4, 2, 4, 4, false); else FF_HM8(4, 4, 4, 4, false);
        }
    }
#undef FF_HM8
    FF_CHECK_LAUNCH(ctx);
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
    FF_REQUIRE(ctx, n > 0 && row_ptr && col && H && (M || precision >= 3), "bad arguments");
    FF_REQUIRE(ctx, precision >= 0 && precision <= 6,
               "precision must be 0 (FP64), 1 (FP32), 2 (both), 3 or 4 (FP32 H only, eight- or sixteen-row tiles), "
               "5 (H only in binary16, eight-row tiles) or 6 (5 in K-blocks for the matrix cores)");
    FF_HIP(ctx, hipSetDevice(ctx->device));
    hipStream_t st = ctx->stream;
    ff_rowtiles *h = new ff_rowtiles();
    h->device = ctx->device;
    h->stream = ctx->stream;
    if (precision >= 3) {
        const int R = precision == 4 ? rt::kTile16 : rt::kTile8;
        h->hrows = R;
        const int64_t nt8 = (n + R - 1) / R;
        int64_t *cnt8 = nullptr, *tptr8 = nullptr;
        int rc8 = FF_OK;
        if (hipMalloc((void **)&cnt8, (size_t)(nt8 + 1) * sizeof(int64_t)) != hipSuccess ||
            hipMalloc((void **)&tptr8, (size_t)(nt8 + 1) * sizeof(int64_t)) != hipSuccess) {
            (void)hipGetLastError();
            rc8 = set_error(ctx, FF_ERR_OOM, "row-tile allocation failed");
        }
        h->mem[0] = tptr8;
        int64_t ent8 = 0;
        int cap8 = 0, bits8 = 0;
        if (!rc8)
            rc8 = R == rt::kTile8 ? rt::build_ptr_union<rt::kTile8>(ctx, st, n, row_ptr, col, cnt8, tptr8, nt8, &ent8,
                                                                    &cap8, &bits8)
                                  : rt::build_ptr_union<rt::kTile16>(ctx, st, n, row_ptr, col, cnt8, tptr8, nt8, &ent8,
                                                                     &cap8, &bits8);
        if (cnt8) (void)hipFree(cnt8);
        int32_t *tcol8 = nullptr;
        float *vh = nullptr;
        if (!rc8) {
            const size_t ne = (size_t)std::max<int64_t>(ent8, 1);
            if (hipMalloc((void **)&tcol8, ne * sizeof(int32_t)) != hipSuccess ||
                hipMalloc((void **)&vh, ne * R * sizeof(float)) != hipSuccess) {
                (void)hipGetLastError();
                rc8 = set_error(ctx, FF_ERR_OOM, "row-tile allocation of %lld entries failed", (long long)ent8);
            }
            h->mem[1] = tcol8;
            h->mem[2] = vh;
        }
        if (!rc8)
            rc8 = R == rt::kTile8
                      ? rt::fill_union<rt::kTile8>(ctx, st, n, nt8, row_ptr, col, cap8, bits8, H, tptr8, tcol8, vh)
                      : rt::fill_union<rt::kTile16>(ctx, st, n, nt8, row_ptr, col, cap8, bits8, H, tptr8, tcol8, vh);
        h->v8.n = h->v16.n = n;
        h->v8.ntiles = h->v16.ntiles = nt8;
        h->v8.entries = h->v16.entries = ent8;
        h->v8.tptr = h->v16.tptr = tptr8;
        h->v8.tcol = h->v16.tcol = tcol8;
        h->v8.vh = h->v16.vh = vh;
        if (!rc8 && precision == 5) {
            uint16_t *v16 = nullptr;
            if (hipMalloc((void **)&v16, (size_t)std::max<int64_t>(ent8, 1) * rt::kTile8 * 2) != hipSuccess) {
                (void)hipGetLastError();
                rc8 = set_error(ctx, FF_ERR_OOM, "row-tile allocation of %lld entries failed", (long long)ent8);
            }
            h->mem[3] = v16;
            if (!rc8) rc8 = rt::build_t8_half(ctx, st, &h->v8, v16);
        }
        if (!rc8 && precision == 6) {
            int64_t *kp = nullptr, *kc = nullptr, nkb = 0;
            if (hipMalloc((void **)&kp, (size_t)(nt8 + 1) * sizeof(int64_t)) != hipSuccess ||
                hipMalloc((void **)&kc, (size_t)(nt8 + 1) * sizeof(int64_t)) != hipSuccess) {
                (void)hipGetLastError();
                rc8 = set_error(ctx, FF_ERR_OOM, "row-tile allocation failed");
            }
            h->mem[4] = kp;
            if (!rc8) rc8 = rt::build_tq_ptr(ctx, st, h->v8, kp, kc, &nkb);
            if (kc) {
                (void)hipStreamSynchronize(st);
                (void)hipFree(kc);
            }
            uint16_t *vq = nullptr;
            if (!rc8 && hipMalloc((void **)&vq, (size_t)std::max<int64_t>(nkb, 1) * 128 * 2) != hipSuccess) {
                (void)hipGetLastError();
                rc8 = set_error(ctx, FF_ERR_OOM, "row-tile allocation of %lld K-blocks failed", (long long)nkb);
            }
            h->mem[5] = vq;
            if (!rc8) rc8 = rt::build_tq_fill(ctx, st, h->v8, kp, nkb, vq, &h->vq);
            // and without its zeros (the packed launch shapes)
            uint64_t *pm = nullptr;
            int64_t *po = nullptr, *pc = nullptr;
            if (!rc8 && (hipMalloc((void **)&pm, (size_t)std::max<int64_t>(nkb, 1) * 16) != hipSuccess ||
                         hipMalloc((void **)&po, (size_t)(nt8 + 1) * sizeof(int64_t)) != hipSuccess ||
                         hipMalloc((void **)&pc, (size_t)(nt8 + 1) * sizeof(int64_t)) != hipSuccess)) {
                (void)hipGetLastError();
                rc8 = set_error(ctx, FF_ERR_OOM, "row-tile allocation failed");
            }
            h->mem[6] = pm;
            h->mem[7] = po;
            struct Slot {
                static void *alloc(void *arg, size_t bytes) {
                    void *p = nullptr;
                    if (hipMalloc(&p, bytes) != hipSuccess) {
                        (void)hipGetLastError();
                        return nullptr;
                    }
                    *(void **)arg = p;
                    return p;
                }
            };
            if (!rc8) rc8 = rt::build_tq_pack(ctx, st, &h->vq, pm, po, pc, Slot::alloc, &h->mem[8]);
            if (pc) {
                (void)hipStreamSynchronize(st);
                (void)hipFree(pc);
            }
        }
        if (!rc8 && hipStreamSynchronize(st) != hipSuccess)
            rc8 = set_error(ctx, FF_ERR_HIP, "row-tile build failed");
        if (rc8) {
            rowtiles_destroy(h);
            return rc8;
        }
        *out = h;
        return FF_OK;
    }
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
    if (!rc) rc = rt::fill(ctx, st, n, ntiles, row_ptr, col, H, M, tptr, entries, tcol, v32, v64);
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
    if (ntiles) *ntiles = rt->hrows ? rt->v8.ntiles : rt->v.ntiles;
    if (entries) *entries = rt->hrows ? rt->v8.entries : rt->v.entries;
    return FF_OK;
}

int spmm_rowtiles(ff_ctx *ctx, const ff_rowtiles *rt, int precision, int m, const void *Y, int64_t ld_y, void *HY,
                  void *MY, int64_t ld_out, int sub) {
    if (!ctx || !rt) return FF_ERR_INVALID_ARG;
    FF_REQUIRE(ctx, Y && HY, "required pointer is NULL");
    if (precision == 2) {
        FF_REQUIRE(ctx, rt->vq.vq != nullptr && !MY, "binary16 blocks need a handle built with precision 6, MY NULL");
        FF_REQUIRE(ctx, rt::tq_ok(m) && ld_y == m && ld_out >= m && ld_out % 4 == 0,
                   "binary16 products take m in {32, 64}, ld_y == m, ld_out >= m and a multiple of 4");
        FF_HIP(ctx, hipSetDevice(ctx->device));
        FF_REQUIRE(ctx, sub >= 0 && sub < rt::kTqSubs, "launch shape %d out of range", sub);
        return rt::spmm_h_tq(ctx, ctx->stream, rt->vq, sub, m, (const uint16_t *)Y, (float *)HY, ld_out);
    }
    FF_REQUIRE(ctx, precision == 0 || precision == 1, "precision must be 0, 1 or 2");
    if (rt->hrows) {
        FF_REQUIRE(ctx, precision == 1 && !MY, "an H-only copy forms H Y alone in FP32 (MY must be NULL)");
        FF_REQUIRE(ctx, (rt->hrows == 8 ? rt::t8_ok(m, ld_y, ld_out) : rt::t16_ok(m, ld_y, ld_out)) && ld_y >= m &&
                            ld_out >= m,
                   "block width %d / leading dimensions not supported by the %d-row kernel", m, rt->hrows);
        FF_REQUIRE(ctx, sub >= 0 && sub < rt::kHSubs, "launch shape %d out of range", sub);
        FF_HIP(ctx, hipSetDevice(ctx->device));
        if (rt->hrows == 16)
            return rt::spmm_h_t16(ctx, ctx->stream, rt->v16, sub, m, (const float *)Y, ld_y, (float *)HY, ld_out,
                                  nullptr, nullptr);
        return rt::spmm_h_t8(ctx, ctx->stream, rt->v8, sub, m, (const float *)Y, ld_y, (float *)HY, ld_out, nullptr,
                             nullptr);
    }
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
