// Device kernels of the blocked LOBPCG eigensolver for H w = lambda M w
// (the generalized eigenproblem that Eq. (15) reduces to).
//
// Block layout: S, HS, MS are row-major [N][3m] arrays holding the search
// space [X | W | P] and its images under H and M. One iteration:
//   resid_kernel   R = HX - MX diag(theta), W = R or diag(H)^-1 R, column norms (FP64)
//   norms_kernel   per-object residuals r_j and convergence / stagnation status
//   spmm_kernel    [HW, MW] = [H, M] W   (the HBM-bound fused product)
//   gram_kernel    S^T HS and S^T MS with MFMA, per-chunk partials in FP64
//   gram_reduce    ordered sum of the partials per object
//   rr_kernel      FP64 Rayleigh-Ritz on the (<= 3m)^2 pencil, one workgroup per object
//   update_kernel  X <- S C, P <- [W P] C_wp (and the same for HS, MS), in place
// Every kernel reads a per-object status word and skips objects that are
// converged, so many independent problems share one launch per stage.
#include "ff_internal.h"

#include <mutex>
#include "k_lobpcg.h"
#include "k_rowtile.h"

#include <algorithm>
#include <chrono>

namespace ff {
namespace lob {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));

__device__ inline int xcd_remap(int b, int nb) {
    // consecutive workgroups are dealt round-robin to the 8 XCDs; give each
    // XCD a contiguous range of logical blocks so its L2 sees neighbouring rows
    const int xcd = b & 7, idx = b >> 3, per = nb >> 3, rem = nb & 7;
    const int start = xcd * per + (xcd < rem ? xcd : rem);
    const int cnt = per + (xcd < rem ? 1 : 0);
    return idx < cnt ? start + idx : b;
}

// ---------------------------------------------------------------------------
// fused SpMM [HY, MY] = [H, M] Y, one wavefront per row
// ---------------------------------------------------------------------------

template <typename T> struct Vec;
template <> struct Vec<float> { typedef float4 type; static constexpr int n = 4; };
template <> struct Vec<double> { typedef double2 type; static constexpr int n = 2; };
__device__ inline float vget(const float4 &a, int i) { return i == 0 ? a.x : i == 1 ? a.y : i == 2 ? a.z : a.w; }
__device__ inline double vget(const double2 &a, int i) { return i == 0 ? a.x : a.y; }
__device__ inline void vset(float4 &a, int i, float v) {
    if (i == 0) a.x = v; else if (i == 1) a.y = v; else if (i == 2) a.z = v; else a.w = v;
}
__device__ inline void vset(double2 &a, int i, double v) {
    if (i == 0) a.x = v; else a.y = v;
}

template <typename T> struct HMPair;
template <> struct HMPair<float> {
    const float2 *hm;
    __device__ inline void get(int64_t e, float &h, float &m) const {
        const unsigned long long u = __builtin_nontemporal_load((const unsigned long long *)hm + e);
        h = __uint_as_float((unsigned)(u & 0xffffffffull));
        m = __uint_as_float((unsigned)(u >> 32));
    }
};
template <> struct HMPair<double> {
    const double *H;
    const double *M;
    __device__ inline void get(int64_t e, double &h, double &m) const {
        h = __builtin_nontemporal_load(H + e);
        m = __builtin_nontemporal_load(M + e);
    }
};

// FP64 accumulators for both precisions: a product of two FP32 numbers is
// exact in FP64, so the FP32 path's only rounding is the final store.
struct Acc4 { double v[4]; };
__device__ inline void acc_zero(Acc4 &a) { a.v[0] = a.v[1] = a.v[2] = a.v[3] = 0.0; }
__device__ inline void acc_fma(Acc4 &a, float h, const float4 &x) {
    const double d = (double)h;
    a.v[0] += d * (double)x.x; a.v[1] += d * (double)x.y; a.v[2] += d * (double)x.z; a.v[3] += d * (double)x.w;
}
__device__ inline void acc_fma(Acc4 &a, double h, const double2 &x) {
    a.v[0] += h * x.x; a.v[1] += h * x.y;
}
__device__ inline void acc_add_shfl(Acc4 &a, int d, int nv) {
    for (int q = 0; q < nv; ++q) a.v[q] += __shfl_xor(a.v[q], d, 64);
}
__device__ inline void acc_store(float *p, const Acc4 &a) {
    *(float4 *)p = make_float4((float)a.v[0], (float)a.v[1], (float)a.v[2], (float)a.v[3]);
}
__device__ inline void acc_store(double *p, const Acc4 &a) { *(double2 *)p = make_double2(a.v[0], a.v[1]); }

// kWaves rows per block, kUnroll independent gathers in flight per lane.
// Lanes are split into groups of G = m / VEC lanes; each group walks every
// NG-th nonzero of the row and the groups are summed at the end.
template <typename T, int kWaves, int kUnroll, bool kXcd>
__global__ void __launch_bounds__(64 * kWaves) spmm_kernel(int64_t nrows, const int64_t *row_ptr, const int32_t *col,
                                                           HMPair<T> hm, const T *Y, int64_t ldy, T *HY, T *MY,
                                                           int64_t ldo, int m, const int *row_obj,
                                                           const int *obj_status) {
    typedef typename Vec<T>::type V;
    constexpr int VN = Vec<T>::n;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int b = kXcd ? xcd_remap(blockIdx.x, gridDim.x) : (int)blockIdx.x;
    const int64_t r = (int64_t)b * kWaves + wv;
    if (r >= nrows) return;
    if (obj_status && obj_status[row_obj[r]] != 0) return;
    const int G = m / VN;
    const int NG = 64 / G;
    const int g = lane / G, c = lane - g * G;
    const bool on = g < NG;
    const int64_t e0 = row_ptr[r], e1 = row_ptr[r + 1];
    Acc4 aH, aM;
    acc_zero(aH);
    acc_zero(aM);
    if (on) {
        int64_t e = e0 + g;
        for (; e + (kUnroll - 1) * NG < e1; e += kUnroll * NG) {
            int32_t j[kUnroll];
            T h[kUnroll], mm[kUnroll];
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
                j[u] = __builtin_nontemporal_load(col + e + u * NG);
                hm.get(e + u * NG, h[u], mm[u]);
            }
            V x[kUnroll];
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) x[u] = *(const V *)(Y + (int64_t)j[u] * ldy + c * VN);
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
                acc_fma(aH, h[u], x[u]);
                acc_fma(aM, mm[u], x[u]);
            }
        }
        for (; e < e1; e += NG) {
            const int32_t j = __builtin_nontemporal_load(col + e);
            T h, mm;
            hm.get(e, h, mm);
            const V x = *(const V *)(Y + (int64_t)j * ldy + c * VN);
            acc_fma(aH, h, x);
            acc_fma(aM, mm, x);
        }
    }
    if ((64 % G) == 0) {
        for (int d = G; d < 64; d <<= 1) {
            acc_add_shfl(aH, d, VN);
            acc_add_shfl(aM, d, VN);
        }
    } else {
        __shared__ double red[kWaves][2][4][64];
        for (int q = 0; q < VN; ++q) {
            red[wv][0][q][lane] = aH.v[q];
            red[wv][1][q][lane] = aM.v[q];
        }
        __builtin_amdgcn_wave_barrier();
        if (g == 0) {
            for (int t = 1; t < NG; ++t)
                for (int q = 0; q < VN; ++q) {
                    aH.v[q] += red[wv][0][q][t * G + c];
                    aM.v[q] += red[wv][1][q][t * G + c];
                }
        }
    }
    if (g == 0) {
        acc_store(HY + r * ldo + c * VN, aH);
        acc_store(MY + r * ldo + c * VN, aM);
    }
}

// Chunked variant: the wave reads 64 (col, h, m) entries of its row with one
// coalesced load per lane, prefetches the next 64 while it works on these,
// hands each entry to the lane group that needs it by cross-lane shuffles and
// keeps kBatch independent gathers of Y rows in flight per lane.
template <typename T, int kWaves, int kBatch, int kOcc>
__global__ void __launch_bounds__(64 * kWaves) __attribute__((amdgpu_waves_per_eu(kOcc, 8)))
spmm_chunk_kernel(int64_t nrows, const int64_t *row_ptr, const int32_t *col, HMPair<T> hm, const T *Y, int64_t ldy,
                  T *HY, T *MY, int64_t ldo, int m, const int *row_obj, const int *obj_status) {
    typedef typename Vec<T>::type V;
    constexpr int VN = Vec<T>::n;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int b = xcd_remap(blockIdx.x, gridDim.x);
    const int64_t r = (int64_t)b * kWaves + wv;
    if (r >= nrows) return;
    if (obj_status && obj_status[row_obj[r]] != 0) return;
    const int G = m / VN;
    const int NG = 64 / G;
    const int g = lane / G, c = lane - g * G;
    const bool on = g < NG;
    const int steps = (64 + NG - 1) / NG;
    const int64_t e0 = row_ptr[r], e1 = row_ptr[r + 1];
    Acc4 aH, aM;
    acc_zero(aH);
    acc_zero(aM);
    int32_t jn = 0;
    T hn = 0, mn = 0;
    if (e0 + lane < e1) {
        jn = __builtin_nontemporal_load(col + e0 + lane);
        hm.get(e0 + lane, hn, mn);
    }
    for (int64_t base = e0; base < e1; base += 64) {
        const int cnt = (int)(e1 - base < 64 ? e1 - base : 64);
        const int32_t jc = jn;
        const T hc = hn, mc = mn;
        jn = 0;
        hn = mn = 0;
        if (base + 64 + lane < e1) {
            jn = __builtin_nontemporal_load(col + base + 64 + lane);
            hm.get(base + 64 + lane, hn, mn);
        }
        for (int s0 = 0; s0 < steps; s0 += kBatch) {
            // issue every gather of the batch first, then fetch the values and accumulate
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
                const int sl = src < 64 ? src : 63;
                const bool ok = on && (s0 + u < steps) && src < cnt;
                const T hv = __shfl(hc, sl, 64), mvv = __shfl(mc, sl, 64);
                acc_fma(aH, ok ? hv : T(0), x[u]);
                acc_fma(aM, ok ? mvv : T(0), x[u]);
            }
        }
    }
    if ((64 % G) == 0) {
        for (int d = G; d < 64; d <<= 1) {
            acc_add_shfl(aH, d, VN);
            acc_add_shfl(aM, d, VN);
        }
    } else {
        __shared__ double red[kWaves][2][4][64];
        for (int q = 0; q < VN; ++q) {
            red[wv][0][q][lane] = aH.v[q];
            red[wv][1][q][lane] = aM.v[q];
        }
        __builtin_amdgcn_wave_barrier();
        if (g == 0) {
            for (int t = 1; t < NG; ++t)
                for (int q = 0; q < VN; ++q) {
                    aH.v[q] += red[wv][0][q][t * G + c];
                    aM.v[q] += red[wv][1][q][t * G + c];
                }
        }
    }
    if (g == 0) {
        acc_store(HY + r * ldo + c * VN, aH);
        acc_store(MY + r * ldo + c * VN, aM);
    }
}

// ---------------------------------------------------------------------------
// Gram products G_H = S^T HS, G_M = S^T MS over the first w columns (MFMA)
// ---------------------------------------------------------------------------
//
// 512 threads: waves 0-3 form S^T HS, waves 4-7 form S^T MS. The 16x16 output
// tiles of a 6x6-tile super block (grid.y walks super blocks) are split into
// four 3x3 groups, one per wave. MFMA 16x16x4: lane l holds A[l%16][l/16] and
// B[l/16][l%16]; the result layout differs between FP32 and FP64 (MfmaAcc::row).

// Result row of accumulator v in lane l: FP32 16x16x4 holds D[4(l/16)+v][l%16],
// FP64 16x16x4 holds D[4v+l/16][l%16] (checked on gfx950).
template <typename T> struct MfmaAcc;
template <> struct MfmaAcc<float> {
    typedef f32x4 type;
    static __device__ inline int row(int lk, int v) { return 4 * lk + v; }
};
template <> struct MfmaAcc<double> {
    typedef f64x4 type;
    static __device__ inline int row(int lk, int v) { return 4 * v + lk; }
};

__device__ inline f32x4 mfma(float a, float b, f32x4 c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
__device__ inline f64x4 mfma(double a, double b, f64x4 c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }

// MT is the arithmetic type: FP32 blocks may run on FP64 MFMA (their products are exact in FP64).
// The block streams its chunk in 16-row sub-blocks: the three 16 x 96 windows
// of S, HS, MS it needs go to LDS with 16-byte loads (double buffered: the
// next sub-block's loads are in flight during the MFMAs), at a row stride that
// puts a fragment read's lanes on distinct banks.
constexpr int kGramTS = 96 + 16;

// the first min(n, VN) elements at p, zeros after them, element by element
template <typename T> __device__ inline typename Vec<T>::type vec_load_partial(const T *p, int n);
template <> __device__ inline float4 vec_load_partial<float>(const float *p, int n) {
    return make_float4(n > 0 ? p[0] : 0.0f, n > 1 ? p[1] : 0.0f, n > 2 ? p[2] : 0.0f, n > 3 ? p[3] : 0.0f);
}
template <> __device__ inline double2 vec_load_partial<double>(const double *p, int n) {
    return make_double2(n > 0 ? p[0] : 0.0, n > 1 ? p[1] : 0.0);
}
template <typename T> constexpr size_t gram_shmem_bytes() { return (size_t)2 * 3 * 16 * kGramTS * sizeof(T); }

// one sub-block of the Gram stream: vector qv of the 3 x 16 x 96 staging area
// (array, row, column vector) into registers, then into LDS buffer b
template <typename T, int kPer>
__device__ inline void gram_stage_load(typename Vec<T>::type *pre, int tid, int64_t rb, int64_t r1, int cs0, int cb0,
                                       int w, const T *S, const T *HS, const T *MS, int64_t ld, int vec_ok) {
    typedef typename Vec<T>::type V;
    constexpr int VN = Vec<T>::n, kWinVec = 96 / VN, kStage = 3 * 16 * kWinVec;
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
        const int qv = tid + u * 512;
        pre[u] = V{};
        if (qv < kStage) {
            const int arr = qv / (16 * kWinVec), rem = qv - arr * (16 * kWinVec);
            const int rr = rem / kWinVec, cv = rem - rr * kWinVec;
            const int col = (arr == 0 ? cs0 : cb0) + cv * VN;
            const int64_t row = rb + rr;
            const T *src = arr == 0 ? S : (arr == 1 ? HS : MS);
            if (row < r1 && col < w) {
                if (vec_ok && col + VN <= w)
                    pre[u] = *(const V *)(src + row * ld + col);
                else                               // unaligned rows or the ragged end of a row
                    pre[u] = vec_load_partial<T>(src + row * ld + col, w - col);
            }
        }
    }
}
template <typename T, int kPer>
__device__ inline void gram_stage_store(const typename Vec<T>::type *pre, int tid, T *buf, int b) {
    typedef typename Vec<T>::type V;
    constexpr int VN = Vec<T>::n, kWinVec = 96 / VN, kStage = 3 * 16 * kWinVec;
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
        const int qv = tid + u * 512;
        if (qv < kStage) {
            const int arr = qv / (16 * kWinVec), rem = qv - arr * (16 * kWinVec);
            const int rr = rem / kWinVec, cv = rem - rr * kWinVec;
            *(V *)(buf + ((size_t)(b * 3 + arr) * 16 + rr) * kGramTS + cv * VN) = pre[u];
        }
    }
}

template <typename T, typename MT>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(2, 2)))
gram_kernel(const GChunk *chunks, const int *obj_status, const int *width, const T *S, const T *HS, const T *MS,
            int64_t ld, int wmax, double *part, int vec_ok) {
    typedef typename MfmaAcc<MT>::type Acc;
    typedef typename Vec<T>::type V;
    constexpr int VN = Vec<T>::n;
    constexpr int kWinVec = 96 / VN;               // vectors per window row
    constexpr int kStage = 3 * 16 * kWinVec;       // vectors per sub-block
    constexpr int kPer = (kStage + 511) / 512;
    const GChunk ch = chunks[blockIdx.x];
    if (obj_status[ch.obj] != 0) return;
    const int w = width[ch.obj];
    const int T16 = (w + 15) >> 4;                 // tiles per dimension
    const int nsup = (T16 + 5) / 6;                // super blocks (96-column windows) per dimension
    const int sy = blockIdx.y / nsup, sx = blockIdx.y - (blockIdx.y / nsup) * nsup;
    if (sy >= nsup) return;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int prod = wv >> 2;                      // 0: H, 1: M
    const int q = wv & 3;
    const int ti0 = (q >> 1) * 3, tj0 = (q & 1) * 3;   // tiles within the windows
    const int cs0 = sy * 96, cb0 = sx * 96;
    const int li = lane & 15, lk = lane >> 4;
    extern __shared__ __align__(16) char smem[];
    T *buf = (T *)smem;                            // [2][3][16][kGramTS]
    const int64_t r0 = ch.r0, r1 = ch.r0 + ch.len;
    V pre[kPer];
    Acc acc[3][3];
    double tot[3][3][4];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            acc[a][c] = Acc{0, 0, 0, 0};
            tot[a][c][0] = tot[a][c][1] = tot[a][c][2] = tot[a][c][3] = 0.0;
        }
    gram_stage_load<T, kPer>(pre, tid, r0, r1, cs0, cb0, w, S, HS, MS, ld, vec_ok);
    gram_stage_store<T, kPer>(pre, tid, buf, 0);
    __syncthreads();
    int b = 0;
    for (int64_t rb = r0; rb < r1; rb += 16) {
        const bool more = rb + 16 < r1;
        if (more) gram_stage_load<T, kPer>(pre, tid, rb + 16, r1, cs0, cb0, w, S, HS, MS, ld, vec_ok);
        const T *Sb = buf + (size_t)(b * 3) * 16 * kGramTS;
        const T *Bb = buf + (size_t)(b * 3 + 1 + prod) * 16 * kGramTS;
#pragma unroll
        for (int k0 = 0; k0 < 16; k0 += 4) {
            const int kr = k0 + lk;
            MT fa[3], fb[3];
#pragma unroll
            for (int t = 0; t < 3; ++t) {
                fa[t] = (MT)Sb[kr * kGramTS + (ti0 + t) * 16 + li];
                fb[t] = (MT)Bb[kr * kGramTS + (tj0 + t) * 16 + li];
            }
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int c = 0; c < 3; ++c) acc[a][c] = mfma(fa[a], fb[c], acc[a][c]);
        }
#pragma unroll
        for (int a = 0; a < 3; ++a)                 // promote to FP64 every 16 rows
#pragma unroll
            for (int c = 0; c < 3; ++c) {
#pragma unroll
                for (int v = 0; v < 4; ++v) tot[a][c][v] += (double)acc[a][c][v];
                acc[a][c] = Acc{0, 0, 0, 0};
            }
        if (more) gram_stage_store<T, kPer>(pre, tid, buf, b ^ 1);
        __syncthreads();
        b ^= 1;
    }
    // write this chunk's partial: part[chunk][prod][i][j]
    double *P = part + ((size_t)blockIdx.x * 2 + prod) * (size_t)wmax * wmax;
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const int tI = sy * 6 + ti0 + a, tJ = sx * 6 + tj0 + c;
            if (tI >= T16 || tJ >= T16) continue;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int i = tI * 16 + MfmaAcc<MT>::row(lk, v), j = tJ * 16 + li;
                if (i < w && j < w) P[(size_t)i * wmax + j] = tot[a][c][v];
            }
        }
}

// G[o][p][i][j] = sum over the object's chunks (ascending) of part[c][p][i][j]
// 256 threads: 16 consecutive outputs x 16 parts; part pp sums the chunks c = pp (mod 16) in ascending
// order, then the 16 part sums are added in order: a fixed order, so the result is deterministic
__global__ void __launch_bounds__(256) gram_reduce_kernel(const int *obj_status, const int *width,
                                                          const int *gfirst, const int *gcount, const double *part,
                                                          int wmax, double *G) {
    const int o = blockIdx.y;
    if (obj_status[o] != 0) return;
    __shared__ double red[16][17];
    const int w = width[o];
    const int q = threadIdx.x & 15, pp = threadIdx.x >> 4;
    const int64_t idx = (int64_t)blockIdx.x * 16 + q;   // over 2 * wmax * wmax
    const int64_t per = (int64_t)wmax * wmax;
    const int i = (int)((idx % per) / wmax), j = (int)(idx % wmax);
    const bool live = idx < 2 * per && i < w && j < w;
    const int c0 = gfirst[o], nc = gcount[o];
    double s = 0.0;
    if (live)
        for (int c = pp; c < nc; c += 16) s += part[(size_t)(c0 + c) * 2 * per + idx];
    red[pp][q] = s;
    __syncthreads();
    if (pp == 0 && live) {
        double t = 0.0;
        for (int u = 0; u < 16; ++u) t += red[u][q];
        G[(size_t)o * 2 * per + idx] = t;
    }
}

// ---------------------------------------------------------------------------
// residuals and the W block
// ---------------------------------------------------------------------------

// Per chunk and column: sum r^2, sum x^2 and, with mdinv, sum r^2 / M_ii (the residual in the
// norm of diag(M)^-1, from which the eigenvalue bounds of norms_kernel are formed); rpart
// holds 3m sums per chunk.
template <typename T>
__global__ void __launch_bounds__(256) resid_kernel(const UChunk *chunks, const int *obj_status, T *S, const T *HS,
                                                    const T *MS, int64_t ld, int m, const double *theta,
                                                    const T *dinv, const double *mdinv, double *rpart,
                                                    float *wpart) {
    // VN consecutive columns per thread (16-byte loads; m is a multiple of 4), rows_per rows per pass
    typedef typename Vec<T>::type V;
    constexpr int VN = Vec<T>::n;
    const UChunk ch = chunks[blockIdx.x];
    if (obj_status[ch.obj] != 0) return;
    const int mv = m / VN;
    const int rows_per = 256 / mv;
    const int t = threadIdx.x;
    const int rr = t / mv, c = (t - (t / mv) * mv) * VN;
    __shared__ double red[3][256 * VN];
    __shared__ float wred[256 * VN];
    double r2[VN], x2[VN], e2[VN], th[VN];
    float wmax[VN];
#pragma unroll
    for (int v = 0; v < VN; ++v) {
        r2[v] = x2[v] = e2[v] = 0.0;
        wmax[v] = 0.f;
    }
    if (rr < rows_per) {
#pragma unroll
        for (int v = 0; v < VN; ++v) th[v] = theta[(size_t)ch.obj * m + c + v];
        for (int64_t r = ch.r0 + rr; r < ch.r0 + ch.len; r += rows_per) {
            const V xs = *(const V *)(S + r * ld + c), hs = *(const V *)(HS + r * ld + c),
                    ms = *(const V *)(MS + r * ld + c);
            const double dv = dinv ? (double)dinv[r] : 1.0;
            const double md = mdinv ? mdinv[r] : 0.0;
            V wv;
#pragma unroll
            for (int v = 0; v < VN; ++v) {
                const double x = (double)vget(xs, v);
                const double R = (double)vget(hs, v) - th[v] * (double)vget(ms, v);
                r2[v] += R * R;
                x2[v] += x * x;
                e2[v] += R * R * md;
                const T w = (T)(dinv ? R * dv : R);
                vset(wv, v, w);
                wmax[v] = fmaxf(wmax[v], fabsf((float)w));
            }
            *(V *)(S + r * ld + m + c) = wv;
        }
    }
    if (rr < rows_per) {
#pragma unroll
        for (int v = 0; v < VN; ++v) {
            red[0][rr * m + c + v] = r2[v];
            red[1][rr * m + c + v] = x2[v];
            red[2][rr * m + c + v] = e2[v];
            wred[rr * m + c + v] = wmax[v];
        }
    }
    __syncthreads();
    if (t < m) {
        double a = 0.0, b = 0.0, e = 0.0;
        float w = 0.f;
        for (int q = 0; q < rows_per; ++q) {
            a += red[0][q * m + t];
            b += red[1][q * m + t];
            e += red[2][q * m + t];
            w = fmaxf(w, wred[q * m + t]);
        }
        rpart[(size_t)blockIdx.x * 3 * m + t] = a;
        rpart[(size_t)blockIdx.x * 3 * m + m + t] = b;
        rpart[(size_t)blockIdx.x * 3 * m + 2 * m + t] = e;
        if (wpart) wpart[(size_t)blockIdx.x * m + t] = w;
    }
}

// r_j = ||R_j|| / ((||H|| + |theta_j| ||M||) ||x_j||); status: 0 active, 1 converged, 2 stagnated.
// 1024 threads: thread (part, q) sums the chunks c = part (mod 16) of output q in
// ascending order, then the 16 parts are added in a fixed order.
//
// With ebound non-NULL, also the a-posteriori bounds of every pair (the residual taken in the
// norm of diag(M)^-1, eta_j^2 = sum_i R_ij^2 / M_ii, standing in for the M^-1 norm of the
// quadratic eigenvalue bound |theta - lambda| <= ||r||^2_{M^-1} / gap and of the Davis-Kahan
// angle bound sin <= ||r||_{M^-1} / gap; the columns are M-orthonormal). For pair j,
// any run C of up to 8 consecutive pairs holding j is a cluster the block form of these bounds
// applies to: eta_C^2 = sum of eta_i^2 over C, gap_C = distance from C to the nearest Ritz value
// outside it (theta_next, the next Ritz value of the last Rayleigh-Ritz step, beyond the block,
// counted no farther than the block's last spacing; unknown = NaN rules the run out), and the
// smallest bound over the runs is kept:
//   ebound_j = min_C eta_C^2 / (gap_C theta_ref), theta_ref = max(|theta_j|, theta_1) (relative
//              error; the constant mode's is relative to theta_1)
//   abound_j = min_C eta_C / gap_C
// With eig_tol > 0 an object converges only when both max_j r_j <= tol and max_j ebound_j <=
// eig_tol over the first k pairs.
__global__ void __launch_bounds__(1024) norms_kernel(int *obj_status, const int *cfirst, const int *ccount,
                                                     const double *rpart, int m, int k, const double *theta,
                                                     const double *norms, double tol, int stall_limit,
                                                     double *res, double *track, const double *theta_next,
                                                     double eig_tol, double angle_tol, double *ebound,
                                                     double *abound) {
    const int o = blockIdx.x;
    if (obj_status[o] != 0) return;
    __shared__ double part[16][192];
    __shared__ double rj[64], eta2[64], th[65], eb[64], ab[64];
    const int q = threadIdx.x & 127, pp = threadIdx.x >> 7;   // 8 parts of 128 outputs
    const int c0 = cfirst[o], nc = ccount[o];
    for (int q2 = q; q2 < 3 * m; q2 += 128)
        for (int pp2 = pp; pp2 < 16; pp2 += 8) {
            double s = 0.0;
            for (int c = pp2; c < nc; c += 16) s += rpart[(size_t)(c0 + c) * 3 * m + q2];
            part[pp2][q2] = s;
        }
    __syncthreads();
    if (threadIdx.x < m) {
        const int c = threadIdx.x;
        double a = 0.0, b = 0.0, e = 0.0;
        for (int t = 0; t < 16; ++t) {
            a += part[t][c];
            b += part[t][m + c];
            e += part[t][2 * m + c];
        }
        const double thc = theta[(size_t)o * m + c];
        double r = sqrt(a) / ((norms[2 * o] + fabs(thc) * norms[2 * o + 1]) * sqrt(b));
        if (!(r == r)) r = INFINITY;
        res[(size_t)o * m + c] = r;
        rj[c] = c < k ? r : 0.0;
        eta2[c] = e;
        th[c] = thc;
    }
    if (threadIdx.x == 0) th[m] = theta_next ? theta_next[o] : NAN;
    __syncthreads();
    if (ebound && threadIdx.x < m) {
        // every run [a, b) of up to kSpan consecutive pairs that holds c is a cluster the block bound
        // applies to; the smallest bound over them is kept (a pair close to a neighbour is bounded
        // together with it instead of by their small distance)
        constexpr int kSpan = 8;
        const int c = threadIdx.x;
        const double ref = fmax(fabs(th[c]), m > 1 ? th[1] : th[m]);
        double best_e = INFINITY, best_a = INFINITY;
        for (int a = c; a >= 0 && a > c - kSpan; --a) {
            double e2 = 0.0;
            for (int j = a; j < c; ++j) e2 += eta2[j];
            for (int b = c + 1; b <= m && b - a <= kSpan; ++b) {
                e2 += eta2[b - 1];
                double gap = a > 0 ? th[a] - th[a - 1] : INFINITY;
                // above the block the next Ritz value is the only estimate of the next eigenvalue, and
                // it lies above it (Ritz values bound eigenvalues from above): the gap to it is taken
                // no wider than the block's last spacing, so that it cannot make the bound small
                const double up = b < m ? th[b] - th[b - 1]
                                        : fmin(th[m] - th[m - 1], m > 1 ? th[m - 1] - th[m - 2] : INFINITY);
                gap = fmin(gap, up);
                if (!(gap > 0.0)) continue;                    // unknown (NaN) or not separated
                best_e = fmin(best_e, e2 / (gap * ref));
                best_a = fmin(best_a, sqrt(e2) / gap);
            }
        }
        if (!(ref > 0.0)) best_e = INFINITY;
        ebound[(size_t)o * m + c] = best_e;
        abound[(size_t)o * m + c] = best_a;
        eb[c] = c < k ? best_e : 0.0;
        ab[c] = c < k ? best_a : 0.0;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double v = 0.0, ve = 0.0, va = 0.0;
        for (int c = 0; c < k; ++c) v = fmax(v, rj[c]);
        if (ebound)
            for (int c = 0; c < k; ++c) {
                ve = fmax(ve, eb[c]);
                va = fmax(va, ab[c]);
            }
        double *tr = track + 2 * o;               // [best max residual, iterations since improvement]
        if (v <= tol && (eig_tol <= 0.0 || (ebound && ve <= eig_tol)) &&
            (angle_tol <= 0.0 || (ebound && va <= angle_tol))) {
            obj_status[o] = 1;
        } else if (stall_limit > 0) {
            if (v < 0.9 * tr[0]) {
                tr[0] = v;
                tr[1] = 0.0;
            } else {
                tr[1] += 1.0;
                if (tr[1] >= stall_limit) obj_status[o] = 2;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// in-place block update: X <- S C, P <- S[:, m:w] C[m:w, :] (and for HS, MS)
// ---------------------------------------------------------------------------
//
// One wavefront owns 16 rows: for each of S, HS, MS it forms X' = S C and
// P' = S C_p' (16 x m each) with MFMA 16x16x4 (C and C_p' staged in LDS, zero
// padded, when they fit). A wave reads its rows completely before writing
// them, and no other wave touches them, so the update is in place.
template <typename T>
__global__ void __launch_bounds__(256) update_kernel(const UChunk *chunks, const int *obj_status, const int *width,
                                                     T *S, T *HS, T *MS, int64_t ld, int m, int wmax,
                                                     const T *C, const T *Cp, int write_p, int c_in_lds) {
    typedef typename MfmaAcc<T>::type Acc;
    const UChunk ch = chunks[blockIdx.x];
    if (obj_status[ch.obj] != 0) return;
    const int w = width[ch.obj];
    const int wpad = (w + 3) & ~3, mpad = (m + 15) & ~15, nct = mpad >> 4;
    extern __shared__ __align__(16) char smem[];
    const T *Co = C + (size_t)ch.obj * wmax * m;
    const T *Cpo = Cp + (size_t)ch.obj * wmax * m;
    // B operands: padded copies in LDS, or the global arrays with bounds checks
    T *Cs = (T *)smem;
    T *Cps = Cs + (size_t)wpad * mpad;
    if (c_in_lds) {
        for (int idx = threadIdx.x; idx < wpad * mpad; idx += 256) {
            const int k = idx / mpad, c = idx - k * mpad;
            const bool in = k < w && c < m;
            Cs[idx] = in ? Co[(size_t)k * m + c] : (T)0;
            Cps[idx] = (in && write_p) ? Cpo[(size_t)k * m + c] : (T)0;
        }
        __syncthreads();
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int li = lane & 15, lk = lane >> 4;
    const int64_t rend = ch.r0 + ch.len;
    for (int64_t rt = ch.r0 + 16 * wv; rt < rend; rt += 64) {
        const int64_t arow = rt + li;
        const bool av = arow < rend;
        for (int a = 0; a < 3; ++a) {
            T *Arr = a == 0 ? S : (a == 1 ? HS : MS);
            Acc ax[4], ap[4];
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                ax[t] = Acc{0, 0, 0, 0};
                ap[t] = Acc{0, 0, 0, 0};
            }
            for (int k0 = 0; k0 < wpad; k0 += 4) {
                const int kk = k0 + lk;
                const T av_ = (av && kk < w) ? Arr[arow * ld + kk] : (T)0;
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    if (t >= nct) break;
                    const int cc = t * 16 + li;
                    T bx, bp;
                    if (c_in_lds) {
                        bx = Cs[kk * mpad + cc];
                        bp = Cps[kk * mpad + cc];
                    } else {
                        const bool in = kk < w && cc < m;
                        bx = in ? Co[(size_t)kk * m + cc] : (T)0;
                        bp = (in && write_p) ? Cpo[(size_t)kk * m + cc] : (T)0;
                    }
                    ax[t] = mfma(av_, bx, ax[t]);
                    if (write_p) ap[t] = mfma(av_, bp, ap[t]);
                }
            }
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                if (t >= nct) break;
                const int c = t * 16 + li;
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int64_t row = rt + MfmaAcc<T>::row(lk, v);
                    if (row >= rend || c >= m) continue;
                    Arr[row * ld + c] = ax[t][v];
                    if (write_p) Arr[row * ld + 2 * m + c] = ap[t][v];
                }
            }
        }
    }
}

// Block update with whole-row fragment loads. MFMA sums over k in any order, so
// the k index of lane group lk at sub-step s of super-step kb is taken as
// kb * 4VK + lk * VK + s (VK = 16 / sizeof(T)): each lane then reads VK
// consecutive entries of its row with one 16-byte load; the loads of the next
// four super-steps are in flight during the MFMAs of these. C and C_p' sit in LDS
// in fragment order ([kb][t][lane][s]), so a lane's VK B values are one 16-byte
// LDS read and a wave's reads cover consecutive addresses.
template <typename T> struct UVec;
template <> struct UVec<float> { typedef f32x4 type; static constexpr int n = 4; };
template <> struct UVec<double> { typedef f64x2 type; static constexpr int n = 2; };

template <typename T> __host__ __device__ inline int upd_nkb(int w) { return (w + 4 * UVec<T>::n - 1) / (4 * UVec<T>::n); }

template <typename T>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4, 8))) update_frag_kernel(const UChunk *chunks, const int *obj_status, const int *width,
                                                          T *S, T *HS, T *MS, int64_t ld, int m, int wmax,
                                                          const T *C, const T *Cp, int write_p) {
    typedef typename MfmaAcc<T>::type Acc;
    typedef typename UVec<T>::type V;
    constexpr int VK = UVec<T>::n, kGrp = sizeof(T) == 8 ? 2 : 4;
    const UChunk ch = chunks[blockIdx.x];
    if (obj_status[ch.obj] != 0) return;
    const int w = width[ch.obj];
    const int nkb = upd_nkb<T>(w), nct = (m + 15) >> 4;
    extern __shared__ __align__(16) char smem[];
    const T *Co = C + (size_t)ch.obj * wmax * m;
    const T *Cpo = Cp + (size_t)ch.obj * wmax * m;
    T *Cf = (T *)smem;
    T *Cpf = Cf + (size_t)nkb * nct * 64 * VK;
    for (int idx = threadIdx.x; idx < nkb * nct * 64 * VK; idx += 256) {
        const int sv = idx % VK, l = (idx / VK) & 63, rest = idx / (64 * VK);
        const int t = rest % nct, kb = rest / nct;
        const int k = kb * 4 * VK + (l >> 4) * VK + sv, c = t * 16 + (l & 15);
        const bool in = k < w && c < m;
        Cf[idx] = in ? Co[(size_t)k * m + c] : (T)0;
        Cpf[idx] = (in && write_p) ? Cpo[(size_t)k * m + c] : (T)0;
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int li = lane & 15, lk = lane >> 4;
    const int64_t rend = ch.r0 + ch.len;
    for (int64_t rt = ch.r0 + 16 * wv; rt < rend; rt += 64) {
        const int64_t arow = rt + li;
        const bool av = arow < rend;
        for (int a = 0; a < 3; ++a) {
            T *Arr = a == 0 ? S : (a == 1 ? HS : MS);
            const T *rowp = Arr + arow * ld;
            // groups of kGrp super-steps; the next group's loads are issued before this group's MFMAs
            auto load_group = [&](int g0, V (&A)[kGrp]) {
#pragma unroll
                for (int u = 0; u < kGrp; ++u) {
                    const int kb = g0 + u, k0 = kb * 4 * VK + lk * VK;
                    V x = V{};
                    if (kb < nkb) {
                        if (av && k0 + VK <= w) {
                            x = *(const V *)(rowp + k0);
                        } else {
#pragma unroll
                            for (int q = 0; q < VK; ++q) x[q] = (av && k0 + q < w) ? rowp[k0 + q] : (T)0;
                        }
                    }
                    A[u] = x;
                }
            };
            Acc ax[4], ap[4];
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                ax[t] = Acc{0, 0, 0, 0};
                ap[t] = Acc{0, 0, 0, 0};
            }
            V cur[kGrp], nxt[kGrp];
            load_group(0, cur);
            for (int g0 = 0; g0 < nkb; g0 += kGrp) {
                load_group(g0 + kGrp, nxt);
#pragma unroll
                for (int u = 0; u < kGrp; ++u) {
                    const int kb = g0 + u;
                    if (kb >= nkb) continue;
#pragma unroll
                    for (int t = 0; t < 4; ++t) {
                        if (t >= nct) continue;
                        const size_t f = ((size_t)(kb * nct + t) * 64 + lane) * VK;
                        const V bx = *(const V *)(Cf + f);
#pragma unroll
                        for (int q = 0; q < VK; ++q) ax[t] = mfma(cur[u][q], bx[q], ax[t]);
                        if (write_p) {
                            const V bp = *(const V *)(Cpf + f);
#pragma unroll
                            for (int q = 0; q < VK; ++q) ap[t] = mfma(cur[u][q], bp[q], ap[t]);
                        }
                    }
                }
#pragma unroll
                for (int u = 0; u < kGrp; ++u) cur[u] = nxt[u];
            }
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                if (t >= nct) break;
                const int c = t * 16 + li;
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int64_t row = rt + MfmaAcc<T>::row(lk, v);
                    if (row >= rend || c >= m) continue;
                    Arr[row * ld + c] = ax[t][v];
                    if (write_p) Arr[row * ld + 2 * m + c] = ap[t][v];
                }
            }
        }
    }
}

constexpr int kRRThreads = 1024;          // stage 1: one workgroup per object
constexpr int kRRWaves = kRRThreads / 64;
constexpr int kRRMax = 192;
constexpr size_t kRRLdsLimit = 156 * 1024;

// Per-object Rayleigh-Ritz scratch in global memory (doubles):
//   A    [wmax^2]  on exit of stage 1 the Householder reflectors (reflector j in
//                  row j, stride ld); the working matrix when it does not fit in LDS
//   B    [wmax^2]  on exit L^-1 (lower triangle, stride ld); working G_M likewise
//   S1, S2 [wmax^2] staging for the two MFMA products
//   sc, dg, eg, tg, evs [wmax each]; kidx [wmax] (kept column -> original),
//   kpos [wmax] (original column -> kept index or -1); meta [16]; Yv [m * wmax]
struct RRScr {
    double *A, *B, *S1, *S2, *sc, *dg, *eg, *tg, *evs, *kidx, *kpos, *meta, *Yv;
};
__host__ __device__ constexpr inline size_t rr_scratch_doubles(int wmax, int m) {
    return (size_t)4 * wmax * wmax + (size_t)7 * wmax + 16 + (size_t)m * wmax;
}
__device__ inline RRScr rr_scr(double *scratch, int o, int wmax, int m) {
    const size_t ww = (size_t)wmax * wmax;
    double *base = scratch + (size_t)o * rr_scratch_doubles(wmax, m);
    RRScr g;
    g.A = base;
    g.B = base + ww;
    g.S1 = base + 2 * ww;
    g.S2 = base + 3 * ww;
    g.sc = base + 4 * ww;
    g.dg = g.sc + wmax;
    g.eg = g.dg + wmax;
    g.tg = g.eg + wmax;
    g.evs = g.tg + wmax;
    g.kidx = g.evs + wmax;
    g.kpos = g.kidx + wmax;
    g.meta = g.kpos + wmax;
    g.Yv = g.meta + 16;
    return g;
}
enum { RR_R = 0, RR_LD, RR_GL, RR_GU, RR_TNORM, RR_PIVMIN };

// stage 1 keeps A and B in LDS when both fit next to its per-column arrays
// (sc, dl, psh, dg, eg, tg and eight partial-sum rows)
constexpr int kRRAux = 14;
inline int rr_use_lds(int wmax) {
    return ((size_t)2 * wmax * wmax + (size_t)kRRAux * wmax) * sizeof(double) <= kRRLdsLimit;
}
inline size_t rr_shmem_bytes(int wmax, int use_lds) {
    return ((use_lds ? (size_t)2 * wmax * wmax : 0) + (size_t)kRRAux * wmax) * sizeof(double);
}
// stage 3 keeps the reflectors in LDS when they fit
inline int rr_vec_lds(int wmax) { return ((size_t)wmax * wmax + (size_t)6 * wmax) * sizeof(double) <= kRRLdsLimit; }
inline size_t rr_vec_shmem_bytes(int wmax, int refl_lds) {
    return ((refl_lds ? (size_t)wmax * wmax : 0) + (size_t)6 * wmax) * sizeof(double);
}

// workgroup barrier that also orders the group's global scratch accesses
__device__ inline void rr_sync() {
    __threadfence_block();
    __syncthreads();
}
// barrier for the working matrices: LDS only, or global scratch
template <bool kLds> __device__ inline void rr_bar() {
    if (!kLds) __threadfence_block();
    __syncthreads();
}

// number of eigenvalues of T (diag dg, offdiag eg) below x
__device__ inline int sturm_count(const double *dg, const double *eg, int r, double x, double pivmin) {
    int cnt = 0;
    double q = dg[0] - x;
    if (fabs(q) < pivmin) q = -pivmin;
    cnt += q < 0.0;
    for (int i = 1; i < r; ++i) {
        q = dg[i] - x - eg[i - 1] * eg[i - 1] / q;
        if (fabs(q) < pivmin) q = -pivmin;
        cnt += q < 0.0;
    }
    return cnt;
}

// Solve (T - lam I) x = b in place (b -> x) with partial pivoting; wk holds 3 r doubles.
__device__ inline void tri_solve(const double *dg, const double *eg, int r, double lam, double tiny, double *x,
                                 double *wk) {
    double *dd = wk, *du = wk + r, *du2 = wk + 2 * r;
    double dcur = dg[0] - lam, ucur = r > 1 ? eg[0] : 0.0;
    double bcur = x[0];
    for (int i = 0; i + 1 < r; ++i) {
        const double ai1 = dg[i + 1] - lam, ei = eg[i], ei1 = (i + 2 < r) ? eg[i + 1] : 0.0;
        const double bnext = x[i + 1];
        double dnext, unext, f, u2, di, ui, bi, bn;
        if (fabs(dcur) >= fabs(ei)) {
            if (dcur == 0.0) dcur = tiny;
            f = ei / dcur;
            di = dcur;
            ui = ucur;
            u2 = 0.0;
            dnext = ai1 - f * ucur;
            unext = ei1;
            bi = bcur;
            bn = bnext - f * bcur;
        } else {                                   // row swap
            f = dcur / ei;
            di = ei;
            ui = ai1;
            u2 = ei1;
            dnext = ucur - f * ai1;
            unext = -f * ei1;
            bi = bnext;
            bn = bcur - f * bnext;
        }
        dd[i] = di;
        du[i] = ui;
        du2[i] = u2;
        x[i] = bi;
        dcur = dnext;
        ucur = unext;
        bcur = bn;
    }
    if (dcur == 0.0) dcur = tiny;
    double x1 = bcur / dcur, x2 = 0.0;
    x[r - 1] = x1;
    for (int i = r - 2; i >= 0; --i) {
        const double xi = (x[i] - du[i] * x1 - du2[i] * x2) / dd[i];
        x[i] = xi;
        x2 = x1;
        x1 = xi;
    }
}

#ifdef FF_RR_TIMING
__device__ unsigned long long rr_clock[16];
#define RR_MARK(i) do { if (blockIdx.x == 0 && threadIdx.x == 0) rr_clock[i] = wall_clock64(); } while (0)
#else
#define RR_MARK(i) do { } while (0)
#endif

// Dst = op(X) op(Y) with op(Z) = Z or Z^T, r x r, stride ld, FP64 MFMA 16x16x4;
// the result goes to dst (a different buffer); entries beyond r are not written.
__device__ inline void rr_gemm(const double *X, const double *Y, int transX, int transY, int r, int ld, double *dst) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int li = lane & 15, lk = lane >> 4;
    const int nt = (r + 15) >> 4;
    for (int tile = wv; tile < nt * nt; tile += kRRWaves) {
        const int ti = tile / nt, tj = tile - (tile / nt) * nt;
        f64x4 acc = {0.0, 0.0, 0.0, 0.0};
        const int row = ti * 16 + li, col = tj * 16 + li;
        for (int k0 = 0; k0 < r; k0 += 4) {
            const int kk = k0 + lk;
            double a = 0.0;
            if (row < r && kk < r) a = transX ? X[(size_t)kk * ld + row] : X[(size_t)row * ld + kk];
            double b = 0.0;
            if (col < r && kk < r) b = transY ? Y[(size_t)col * ld + kk] : Y[(size_t)kk * ld + col];
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int i = ti * 16 + 4 * v + lk, j = tj * 16 + li;   // FP64 result layout
            if (i < r && j < r) dst[(size_t)i * ld + j] = acc[v];
        }
    }
}

// ---------------------------------------------------------------------------
// FP64 Rayleigh-Ritz on the pencil (G_H, G_M) of order w, in four launches
// ---------------------------------------------------------------------------
//
// Stage 1 (rr_tridiag_kernel, one 1024-thread workgroup per object):
//   1. symmetrise, scale both by D^-1/2 with D = diag(G_M)
//   2. Cholesky of the scaled G_M in column order (one barrier per column),
//      dropping a column whose pivot falls to tau or below (a direction
//      already spanned); the X columns come first, so normally only W and P
//      directions are dropped
//   3. compaction to the kept columns, L^-1 in place, A = L^-1 G_H L^-T as two
//      FP64 MFMA products
//   4. Householder reduction of A to tridiagonal T = Q^T A Q (reflector j
//      kept in row j), three barriers per column
// Stage 2 (rr_eig_kernel, one wavefront per wanted eigenvalue): multisection
//   on Sturm counts, 64 points per round.
// Stage 3 (rr_vec_kernel, one wavefront per eigenvalue): inverse iteration
//   with partial pivoting; eigenvalues closer than 1e-9 ||T|| form a cluster
//   that its first wavefront handles in order, orthogonalising each member
//   against the earlier ones; then y -> Q y -> L^-T Q y -> D^-1/2 L^-T Q y = C,
//   theta = Rayleigh quotient on T.
// Stage 4 (rr_post_kernel, one workgroup per column): the P coefficients
//   C_p' = C_p - C (C^T G_M C_p) with C_p = C without its X rows, so that
//   P' = S C_p' is M-orthogonal to X' = S C; FP32 copies for the FP32 update.

// kLds: A and B in LDS (a compile-time choice, so that their accesses are LDS
// instructions rather than generic ones)
template <bool kLds>
__global__ void __launch_bounds__(kRRThreads) rr_tridiag_kernel(int *obj_status, const int *width, const double *G,
                                                                int wmax, int m, double tau, double pmin,
                                                                double *scratch, int *info) {
    constexpr bool use_lds = kLds;
    const int o = blockIdx.x;
    if (obj_status[o] != 0) return;
    const int w = width[o];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    extern __shared__ __align__(16) double sm[];
    const size_t ww = (size_t)wmax * wmax;
    const RRScr g = rr_scr(scratch, o, wmax, m);
    double *A = use_lds ? sm : g.A;
    double *B = use_lds ? sm + ww : g.B;
    double *aux = sm + (use_lds ? 2 * ww : 0);
    double *sc = aux, *dl = aux + wmax, *psh = aux + 2 * wmax, *dg = aux + 3 * wmax, *eg = aux + 4 * wmax;
    double *tg = aux + 5 * wmax, *ppart = aux + 6 * wmax;   // ppart: 8 rows of partial sums
    __shared__ int keep[kRRMax], kidx[kRRMax];
    __shared__ int nkeep, xdrop;
    // partial sums: wave wv takes every 8th inner index (kset) for one 64-wide pass of outputs
    const int kset = wv & 7, opass = wv >> 3;
    const double *GH = G + (size_t)o * 2 * ww;
    const double *GM = GH + ww;
    // Every LDS matrix access below runs along a row (consecutive lanes, consecutive
    // addresses): with a row stride of 96 doubles a column access would put all
    // 64 lanes on one bank.

    RR_MARK(0);
    // 1. load, symmetrise, scale
    for (int j = tid; j < w; j += kRRThreads) {
        const double d = GM[(size_t)j * wmax + j];
        sc[j] = d > 0.0 ? 1.0 / sqrt(d) : 0.0;
    }
    if (tid == 0) xdrop = 0;
    rr_sync();
    for (int i = wv; i < w; i += kRRWaves)
        for (int j = lane; j < w; j += 64) {
            const double s = sc[i] * sc[j];
            A[(size_t)i * wmax + j] = 0.5 * (GH[(size_t)i * wmax + j] + GH[(size_t)j * wmax + i]) * s;
            B[(size_t)i * wmax + j] = 0.5 * (GM[(size_t)i * wmax + j] + GM[(size_t)j * wmax + i]) * s;
        }
    rr_sync();

    RR_MARK(1);
    // 2. Cholesky G_M = U^T U on the upper triangle with dropping. Step j updates
    //    the trailing upper triangle with the unscaled row j (B_il -= B_ji B_jl / piv)
    //    and scales the previous row, which nothing reads any more.
    for (int j = 0; j < w; ++j) {
        const double piv = B[(size_t)j * wmax + j];
        // a P column (j >= 2m) whose squared M-norm is below pmin is dropped as well: its images are
        // implicit updates whose absolute rounding error is set by the X terms, so once P has shrunk to
        // that level the direction is noise to the Rayleigh-Ritz step
        const bool kj = sc[j] > 0.0 && piv > tau && (j < 2 * m || sc[j] * sc[j] * pmin <= 1.0);
        if (tid == 0) {
            keep[j] = kj;
            dl[j] = kj ? sqrt(piv) : 0.0;
            if (!kj && j < m) xdrop = 1;
        }
        if (j > 0 && keep[j - 1]) {
            const double inv = 1.0 / dl[j - 1];
            for (int l = j + tid; l < w; l += kRRThreads) B[(size_t)(j - 1) * wmax + l] *= inv;
        }
        if (kj) {
            const double ip = 1.0 / piv;
            const double *rowj = B + (size_t)j * wmax;
            for (int i = j + 1 + wv; i < w; i += kRRWaves) {
                const double bji = rowj[i] * ip;
                for (int l = i + lane; l < w; l += 64) B[(size_t)i * wmax + l] -= bji * rowj[l];
            }
        }
        rr_bar<kLds>();
    }
    if (tid == 0) {
        int r = 0;
        for (int j = 0; j < w; ++j)
            if (keep[j]) kidx[r++] = j;
        nkeep = r;
        info[o] = r | (xdrop << 16);
    }
    for (int j = tid; j < w; j += kRRThreads)     // diagonal of U
        if (keep[j]) B[(size_t)j * wmax + j] = dl[j];
    rr_sync();
    const int r = nkeep;
    if (r < m) {                                   // basis lost rank: report and leave C untouched
        if (tid == 0) obj_status[o] = 3;
        return;
    }
    const int ld = r < w ? r : wmax;

    RR_MARK(2);
    // 3a. compaction to the kept rows and columns at stride r: a destination
    //     never lies after its source, and each chunk is read before it is written
    if (r < w) {
        const int tot = r * r;
        for (int base = 0; base < tot; base += kRRThreads) {
            const int idx = base + tid;
            double va = 0.0, vb = 0.0;
            if (idx < tot) {
                const int i = idx / r, jj = idx - (idx / r) * r;
                va = A[(size_t)kidx[i] * wmax + kidx[jj]];
                vb = jj >= i ? B[(size_t)kidx[i] * wmax + kidx[jj]] : 0.0;
            }
            rr_sync();
            if (idx < tot) {
                A[idx] = va;
                B[idx] = vb;
            }
            rr_sync();
        }
    }
    // 3b. V = U^-1 in place, rows from the last: with U = [a b^T; 0 U2],
    //     U^-1 = [1/a, -b^T U2^-1 / a; 0, U2^-1]
    //     The sums over t run as eight partial sums (t = kset mod 8) along rows t of V.
    for (int j = r - 1; j >= 0; --j) {
        const double *bj = B + (size_t)j * ld;
        const double d = 1.0 / bj[j];
        for (int l = j + 1 + lane + 64 * opass; l < r; l += 128) {
            double s = 0.0;
            for (int t = j + 1 + kset; t <= l; t += 8) s += bj[t] * B[(size_t)t * ld + l];
            ppart[kset * wmax + l] = s;
        }
        rr_bar<kLds>();
        for (int l = j + 1 + tid; l < r; l += kRRThreads) {
            double s = 0.0;
#pragma unroll
            for (int q = 0; q < 8; ++q) s += ppart[q * wmax + l];
            B[(size_t)j * ld + l] = -d * s;
        }
        if (tid == 0) B[(size_t)j * ld + j] = d;
        rr_bar<kLds>();
    }
    for (int i = wv; i < r; i += kRRWaves)         // zero the strict lower triangle for the products
        for (int j = lane; j < i; j += 64) B[(size_t)i * ld + j] = 0.0;
    rr_sync();
    // 3c. A <- (V^T A) V = L^-1 A L^-T (L = U^T) through the global staging areas, symmetrised
    rr_gemm(B, A, 1, 0, r, ld, g.S1);
    rr_sync();
    rr_gemm(g.S1, B, 0, 0, r, ld, g.S2);
    rr_sync();
    for (int i = wv; i < r; i += kRRWaves)
        for (int j = lane; j < r; j += 64)
            A[(size_t)i * ld + j] = 0.5 * (g.S2[(size_t)i * ld + j] + g.S2[(size_t)j * ld + i]);
    rr_sync();

    RR_MARK(3);
    // 4. Householder tridiagonalisation of the symmetric A. Column j is read as
    //    row j; reflector j, v = [1, x/(x0 - beta)], is written over row j at
    //    step j + 1 (no step reads a row above its own).
    double scale_prev = 0.0, tj_prev = 0.0;
    for (int j = 0; j + 2 < r; ++j) {
        if (j > 0 && tj_prev != 0.0) {
            double *rp = A + (size_t)(j - 1) * ld;
            for (int k = j + tid; k < r; k += kRRThreads) rp[k] = k == j ? 1.0 : rp[k] * scale_prev;
        }
        const double *rowj = A + (size_t)j * ld;
        const double x0 = rowj[j + 1];
        double part = 0.0;                         // every wave forms sigma itself
        for (int i = j + 2 + lane; i < r; i += 64) part += rowj[i] * rowj[i];
#pragma unroll
        for (int dd = 32; dd >= 1; dd >>= 1) part += __shfl_xor(part, dd, 64);
        const double sigma = part;
        double tj = 0.0, beta = x0, scale = 0.0;
        if (sigma > 0.0) {
            const double mu = sqrt(x0 * x0 + sigma);
            beta = x0 <= 0.0 ? mu : -mu;
            tj = (beta - x0) / beta;
            scale = 1.0 / (x0 - beta);
        }
        if (tid == 0) {
            dg[j] = A[(size_t)j * ld + j];
            eg[j] = beta;
            tg[j] = tj;
        }
        scale_prev = scale;
        tj_prev = tj;
        if (tj == 0.0) {                           // uniform: every wave has the same sigma
            rr_bar<kLds>();
            continue;
        }
        // p = tau A v as eight partial sums over k (rows k of the symmetric A, lanes along i)
        for (int i = j + 1 + lane + 64 * opass; i < r; i += 128) {
            double s = 0.0;
            for (int k = j + 1 + kset; k < r; k += 8) s += A[(size_t)k * ld + i] * (k == j + 1 ? 1.0 : rowj[k] * scale);
            ppart[kset * wmax + i] = s;
        }
        rr_bar<kLds>();
        // every wave: p and v on its lanes' columns, then K = tau/2 p^T v
        double pk[3], vk3[3], kp = 0.0;
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const int k = j + 1 + lane + 64 * q;
            pk[q] = 0.0;
            vk3[q] = 0.0;
            if (k < r) {
                double s = 0.0;
#pragma unroll
                for (int u = 0; u < 8; ++u) s += ppart[u * wmax + k];
                pk[q] = tj * s;
                vk3[q] = k == j + 1 ? 1.0 : rowj[k] * scale;
                kp += pk[q] * vk3[q];
            }
        }
#pragma unroll
        for (int dd = 32; dd >= 1; dd >>= 1) kp += __shfl_xor(kp, dd, 64);
        const double K = 0.5 * tj * kp;
        for (int i = j + 1 + wv; i < r; i += kRRWaves) {
            double pi = 0.0;
#pragma unroll
            for (int u = 0; u < 8; ++u) pi += ppart[u * wmax + i];
            const double vi = i == j + 1 ? 1.0 : rowj[i] * scale, wi = tj * pi - K * vi;
            double *ai = A + (size_t)i * ld;
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                const int k = j + 1 + lane + 64 * q;
                if (k < r) ai[k] -= vi * (pk[q] - K * vk3[q]) + wi * vk3[q];
            }
        }
        rr_bar<kLds>();
    }
    if (r >= 3 && tj_prev != 0.0) {                // the last reflector's row
        double *rp = A + (size_t)(r - 3) * ld;
        for (int k = r - 2 + tid; k < r; k += kRRThreads) rp[k] = k == r - 2 ? 1.0 : rp[k] * scale_prev;
    }
    if (tid == 0) {
        if (r >= 2) {
            dg[r - 2] = A[(size_t)(r - 2) * ld + (r - 2)];
            eg[r - 2] = A[(size_t)(r - 2) * ld + (r - 1)];
            tg[r - 2] = 0.0;
        }
        dg[r - 1] = A[(size_t)(r - 1) * ld + (r - 1)];
        tg[r - 1] = 0.0;
        eg[r - 1] = 0.0;
    }
    rr_sync();

    RR_MARK(4);
    // 5. hand over: T, reflectors (rows of A), L^-1 = V^T (row s of L^-1 = column s
    //    of V), column maps and Gershgorin bounds
    for (int idx = tid; idx < r * r; idx += kRRThreads) {
        const int i = idx / r, sidx = idx - (idx / r) * r;
        if (use_lds) g.A[(size_t)i * ld + sidx] = A[(size_t)i * ld + sidx];
        g.S1[(size_t)sidx * ld + i] = B[(size_t)i * ld + sidx];
    }
    for (int i = tid; i < w; i += kRRThreads) {
        g.sc[i] = sc[i];
        g.kpos[i] = -1.0;
    }
    rr_sync();
    for (int idx = tid; idx < r * r; idx += kRRThreads) {
        const int i = idx / r, sidx = idx - (idx / r) * r;
        g.B[(size_t)i * ld + sidx] = g.S1[(size_t)i * ld + sidx];
    }
    for (int i = tid; i < r; i += kRRThreads) {
        g.dg[i] = dg[i];
        g.eg[i] = eg[i];
        g.tg[i] = tg[i];
        g.kidx[i] = (double)kidx[i];
        g.kpos[kidx[i]] = (double)i;
    }
    if (tid == 0) {
        double gl = 0.0, gu = 0.0, maxe2 = 0.0;
        for (int i = 0; i < r; ++i) {
            const double off = (i > 0 ? fabs(eg[i - 1]) : 0.0) + (i + 1 < r ? fabs(eg[i]) : 0.0);
            gl = i == 0 ? dg[i] - off : fmin(gl, dg[i] - off);
            gu = i == 0 ? dg[i] + off : fmax(gu, dg[i] + off);
            if (i + 1 < r) maxe2 = fmax(maxe2, eg[i] * eg[i]);
        }
        const double tnorm = fmax(fabs(gl), fabs(gu));
        const double eps = 2.220446049250313e-16;
        g.meta[RR_R] = r;
        g.meta[RR_LD] = ld;
        g.meta[RR_GL] = gl - (4.0 * eps * tnorm + 1e-300);
        g.meta[RR_GU] = gu + (4.0 * eps * tnorm + 1e-300);
        g.meta[RR_TNORM] = tnorm;
        g.meta[RR_PIVMIN] = 2.2250738585072014e-308 * fmax(1.0, maxe2);
    }
    RR_MARK(5);
}

// stage 2: eigenvalue t of T by multisection (64 Sturm counts per round); the block t = m
// (launched when theta_next is given) finds the next Ritz value beyond the block when the kept
// basis has more than m columns, and otherwise leaves the previous step's value (the X-only
// steps at the start of a phase have none of their own)
__global__ void __launch_bounds__(64) rr_eig_kernel(const int *obj_status, int wmax, int m, double *scratch,
                                                    double *theta_next) {
    const int t = blockIdx.x, o = blockIdx.y, lane = threadIdx.x;
    if (obj_status[o] != 0) return;
    const RRScr g = rr_scr(scratch, o, wmax, m);
    const int r = (int)g.meta[RR_R];
    if (t >= m && r <= m) return;
    __shared__ double dg[kRRMax], eg[kRRMax];
    for (int i = lane; i < r; i += 64) {
        dg[i] = g.dg[i];
        eg[i] = g.eg[i];
    }
    __syncthreads();
    const double eps = 2.220446049250313e-16, pivmin = g.meta[RR_PIVMIN];
    double lo = g.meta[RR_GL], hi = g.meta[RR_GU];
    for (int it = 0; it < 64; ++it) {
        if (hi - lo <= 2.0 * eps * fmax(fabs(lo), fabs(hi)) + pivmin) break;
        const double x = lo + (hi - lo) * (double)(lane + 1) / 65.0;
        const bool above = sturm_count(dg, eg, r, x, pivmin) > t;
        double nlo = above ? lo : x, nhi = above ? x : hi;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            nlo = fmax(nlo, __shfl_xor(nlo, d, 64));
            nhi = fmin(nhi, __shfl_xor(nhi, d, 64));
        }
        lo = nlo;
        hi = nhi;
    }
    if (lane == 0) {
        g.evs[t] = 0.5 * (lo + hi);
        if (t >= m) theta_next[o] = 0.5 * (lo + hi);
    }
}

// stage 3: eigenvector(s) of T for eigenvalue t (its whole cluster when t leads one),
// back-transformed to the coefficients C[:, u] (rows = basis columns, stride m)
template <bool kLds>
__global__ void __launch_bounds__(64) rr_vec_kernel(const int *obj_status, const int *width, int wmax, int m,
                                                    double *scratch, double *C, double *theta) {
    constexpr bool refl_lds = kLds;
    const int t0 = blockIdx.x, o = blockIdx.y, lane = threadIdx.x;
    if (obj_status[o] != 0) return;
    const RRScr g = rr_scr(scratch, o, wmax, m);
    const int w = width[o];
    const int r = (int)g.meta[RR_R], ld = (int)g.meta[RR_LD];
    const double tnorm = g.meta[RR_TNORM];
    const double eps = 2.220446049250313e-16;
    const double ctol = 1e-9 * tnorm, tiny = eps * tnorm + 1e-300;
    const double *evs = g.evs;
    if (t0 > 0 && evs[t0] - evs[t0 - 1] <= ctol) return;   // handled by the cluster's first eigenvalue
    int t1 = t0 + 1;
    while (t1 < m && evs[t1] - evs[t1 - 1] <= ctol) ++t1;
    extern __shared__ __align__(16) double sm[];
    const double *refl = refl_lds ? sm : g.A;
    double *aux = sm + (refl_lds ? (size_t)wmax * wmax : 0);
    double *dg = aux, *eg = aux + wmax, *x = aux + 2 * wmax, *wk = aux + 3 * wmax;
    for (int i = lane; i < r; i += 64) {
        dg[i] = g.dg[i];
        eg[i] = g.eg[i];
    }
    if (refl_lds)
        for (int idx = lane; idx < r * ld; idx += 64) sm[idx] = g.A[idx];
    __syncthreads();
    double *Co = C + (size_t)o * wmax * m;
    for (int u = t0; u < t1; ++u) {
        if (lane == 0) {
            for (int i = 0; i < r; ++i) {
                const unsigned hsh = (unsigned)i * 2654435761u + (unsigned)u * 2246822519u + 12345u;
                x[i] = 1.0 + ((double)((hsh >> 8) & 0xffff) / 65536.0 - 0.5);
            }
            for (int it = 0; it < 3; ++it) {
                tri_solve(dg, eg, r, evs[u], tiny, x, wk);
                for (int q = t0; q < u; ++q) {           // earlier members of the cluster
                    const double *yq = g.Yv + (size_t)q * wmax;
                    double d = 0.0;
                    for (int i = 0; i < r; ++i) d += yq[i] * x[i];
                    for (int i = 0; i < r; ++i) x[i] -= d * yq[i];
                }
                double nx = 0.0;
                for (int i = 0; i < r; ++i) nx += x[i] * x[i];
                const double inv = nx > 0.0 ? 1.0 / sqrt(nx) : 0.0;
                for (int i = 0; i < r; ++i) x[i] *= inv;
            }
            if (t1 - t0 > 1)
                for (int i = 0; i < r; ++i) g.Yv[(size_t)u * wmax + i] = x[i];
        }
        __threadfence_block();
        __syncthreads();
        double y[3], z[3];
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const int i = lane + 64 * q;
            y[q] = i < r ? x[i] : 0.0;
        }
        // Rayleigh quotient on T
        double rq = 0.0;
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const int i = lane + 64 * q;
            if (i < r) {
                double ty = dg[i] * y[q];
                if (i > 0) ty += eg[i - 1] * x[i - 1];
                if (i + 1 < r) ty += eg[i] * x[i + 1];
                rq += y[q] * ty;
            }
        }
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) rq += __shfl_xor(rq, d, 64);
        if (lane == 0) theta[(size_t)o * m + u] = rq;
        // y <- Q y: reflectors applied last to first
        for (int j = r - 3; j >= 0; --j) {
            const double tj = g.tg[j];
            if (tj == 0.0) continue;
            const double *vrow = refl + (size_t)j * ld;
            double sacc = 0.0;
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                const int i = lane + 64 * q;
                if (i > j && i < r) sacc += vrow[i] * y[q];
            }
#pragma unroll
            for (int d = 32; d >= 1; d >>= 1) sacc += __shfl_xor(sacc, d, 64);
            sacc *= tj;
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                const int i = lane + 64 * q;
                if (i > j && i < r) y[q] -= sacc * vrow[i];
            }
        }
        // z = L^-T y: z_i = sum_{s >= i} Linv[s][i] y_s
        z[0] = z[1] = z[2] = 0.0;
        for (int sidx = 0; sidx < r; ++sidx) {
            const double ysrc = sidx < 64 ? y[0] : (sidx < 128 ? y[1] : y[2]);
            const double ys = __shfl(ysrc, sidx & 63, 64);
            const double *Ls = g.B + (size_t)sidx * ld;
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                const int i = lane + 64 * q;
                if (i <= sidx) z[q] += Ls[i] * ys;
            }
        }
        // C column u: D^-1/2 z on the kept basis columns, zero on the dropped ones
        for (int i = lane; i < w; i += 64) {
            const int p = (int)g.kpos[i];
            if (p < 0) Co[(size_t)i * m + u] = 0.0;
        }
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const int i = lane + 64 * q;
            if (i < r) {
                const int c = (int)g.kidx[i];
                Co[(size_t)c * m + u] = g.sc[c] * z[q];
            }
        }
        __syncthreads();
    }
}

// stage 4: column c of C_p' = C_p - C (C^T G_M C_p), and the working-precision copies
template <typename CT>
__global__ void __launch_bounds__(256) rr_post_kernel(const int *obj_status, const int *width, const double *G,
                                                      int wmax, int m, const double *C, CT *Cw, double *Cp,
                                                      CT *Cpw) {
    const int c = blockIdx.x, o = blockIdx.y, tid = threadIdx.x;
    if (obj_status[o] != 0) return;
    const int w = width[o];
    const size_t ww = (size_t)wmax * wmax;
    const double *GM = G + (size_t)o * 2 * ww + ww;
    const double *Co = C + (size_t)o * wmax * m;
    __shared__ double T1[kRRMax], Q[kRRMax];
    for (int i = tid; i < w; i += 256) {
        double acc = 0.0;
        for (int j = m; j < w; ++j) acc += GM[(size_t)i * wmax + j] * Co[(size_t)j * m + c];
        T1[i] = acc;
    }
    __syncthreads();
    for (int a = tid; a < m; a += 256) {
        double acc = 0.0;
        for (int i = 0; i < w; ++i) acc += Co[(size_t)i * m + a] * T1[i];
        Q[a] = acc;
    }
    __syncthreads();
    double *Cpo = Cp + (size_t)o * wmax * m;
    CT *Cpwo = Cpw + (size_t)o * wmax * m;
    CT *Cwo = Cw + (size_t)o * wmax * m;
    for (int i = tid; i < w; i += 256) {
        const size_t idx = (size_t)i * m + c;
        double acc = i >= m ? Co[idx] : 0.0;
        for (int a = 0; a < m; ++a) acc -= Co[(size_t)i * m + a] * Q[a];
        Cpo[idx] = acc;
        Cpwo[idx] = (CT)acc;
        Cwo[idx] = (CT)Co[idx];
    }
}

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------

__global__ void diag_inv_kernel(int64_t n, const int64_t *row_ptr, const int32_t *col, const double *H, double *d64,
                                float *d32) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    double d = 0.0;
    for (int64_t e = row_ptr[r]; e < row_ptr[r + 1]; ++e)
        if (col[e] == r) { d = H[e]; break; }
    const double v = d > 0.0 ? 1.0 / d : 1.0;
    d64[r] = v;
    d32[r] = (float)v;
}

// per-object max row sums of |H| and |M| (norms[2o], norms[2o+1])
__global__ void __launch_bounds__(256) row_norm_kernel(const int64_t *obj_off, const int64_t *row_ptr,
                                                       const double *H, const double *M, double *norms) {
    const int o = blockIdx.x;
    const int64_t a = obj_off[o], b = obj_off[o + 1];
    double mh = 0.0, mm = 0.0;
    for (int64_t r = a + threadIdx.x; r < b; r += blockDim.x) {
        double sh = 0.0, sm = 0.0;
        for (int64_t e = row_ptr[r]; e < row_ptr[r + 1]; ++e) {
            sh += fabs(H[e]);
            sm += fabs(M[e]);
        }
        mh = fmax(mh, sh);
        mm = fmax(mm, sm);
    }
    __shared__ double s[2][256];
    s[0][threadIdx.x] = mh;
    s[1][threadIdx.x] = mm;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) {
            s[0][threadIdx.x] = fmax(s[0][threadIdx.x], s[0][threadIdx.x + st]);
            s[1][threadIdx.x] = fmax(s[1][threadIdx.x], s[1][threadIdx.x + st]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        norms[2 * o] = s[0][0];
        norms[2 * o + 1] = s[1][0];
    }
}

template <typename TD, typename TS>
__global__ void copy_block_kernel(int64_t n, int m, const TS *src, int64_t lds, TD *dst, int64_t ldd) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * m) return;
    const int64_t r = t / m, c = t - r * m;
    dst[r * ldd + c] = (TD)src[r * lds + c];
}

__global__ void set_width_kernel(int n_obj, int *obj_status, int *width, int w, int only_active) {
    const int o = blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= n_obj) return;
    if (only_active && obj_status[o] != 0) return;
    width[o] = w;
}

__global__ void reset_status_kernel(int n_obj, int *obj_status, double *track, int keep_converged) {
    const int o = blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= n_obj) return;
    if (!(keep_converged && obj_status[o] == 1)) obj_status[o] = 0;
    track[2 * o] = INFINITY;
    track[2 * o + 1] = 0.0;
}

// Philox-4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11)
__device__ inline void philox(uint32_t c[4], uint32_t k0, uint32_t k1) {
    for (int rnd = 0; rnd < 10; ++rnd) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
        const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = lo1;
        c[2] = n2;
        c[3] = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

__global__ void philox_block_kernel(int64_t count, uint64_t seed, double *out) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;   // one Philox call per 4 values
    if (4 * g >= count) return;
    uint32_t c[4] = {(uint32_t)g, (uint32_t)((uint64_t)g >> 32), 0u, 0u};
    philox(c, (uint32_t)seed, (uint32_t)(seed >> 32));
    for (int t = 0; t < 4; ++t)
        if (4 * g + t < count) out[4 * g + t] = ldexp((double)c[t], -31) - 1.0;
}

__global__ void philox_raw_kernel(const uint32_t *ctr, const uint32_t *key, uint32_t *out, int count) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= count) return;
    uint32_t c[4] = {ctr[4 * t], ctr[4 * t + 1], ctr[4 * t + 2], ctr[4 * t + 3]};
    philox(c, key[2 * t], key[2 * t + 1]);
    for (int i = 0; i < 4; ++i) out[4 * t + i] = c[i];
}

// sign rule: the entry of largest magnitude of each column is positive (lowest row on ties)
__global__ void __launch_bounds__(256) sign_partial_kernel(int64_t a, int64_t b, int m, const double *X, int64_t ld,
                                                           double *pv, int64_t *pi) {
    // block (c, part): partial argmax of |X[r][c]| over rows a..b
    const int c = blockIdx.y;
    double best = -1.0;
    int64_t bi = INT64_MAX;
    for (int64_t r = a + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < b; r += (int64_t)gridDim.x * blockDim.x) {
        const double v = fabs(X[r * ld + c]);
        if (v > best || (v == best && r < bi)) { best = v; bi = r; }
    }
    __shared__ double sv[256];
    __shared__ int64_t si[256];
    sv[threadIdx.x] = best;
    si[threadIdx.x] = bi;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) {
            const double ov = sv[threadIdx.x + st];
            const int64_t oi = si[threadIdx.x + st];
            if (ov > sv[threadIdx.x] || (ov == sv[threadIdx.x] && oi < si[threadIdx.x])) {
                sv[threadIdx.x] = ov;
                si[threadIdx.x] = oi;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        pv[(size_t)c * gridDim.x + blockIdx.x] = sv[0];
        pi[(size_t)c * gridDim.x + blockIdx.x] = si[0];
    }
}

__global__ void sign_final_kernel(int k, const double *X, int64_t ld, int nparts, const double *pv, const int64_t *pi,
                                  double *sgn) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= k) return;
    double best = -1.0;
    int64_t bi = INT64_MAX;
    for (int p = 0; p < nparts; ++p) {
        const double v = pv[(size_t)c * nparts + p];
        const int64_t i = pi[(size_t)c * nparts + p];
        if (v > best || (v == best && i < bi)) { best = v; bi = i; }
    }
    sgn[c] = (bi != INT64_MAX && X[bi * ld + c] < 0.0) ? -1.0 : 1.0;
}

__global__ void sign_apply_kernel(int64_t a, int64_t b, int k, const double *X, int64_t ld, const double *sgn,
                                  double *W, int64_t ldw) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (b - a) * k) return;
    const int64_t r = a + t / k;
    const int c = (int)(t % k);
    W[r * ldw + c] = sgn[c] * X[r * ld + c];
}

}  // namespace lob
}  // namespace ff

// ===========================================================================
// host side
// ===========================================================================

namespace ff {
namespace lob {

__global__ void __launch_bounds__(256) rownorm_chunk_kernel(const UChunk *chunks, const int64_t *row_ptr,
                                                            const double *H, const double *M, double *part) {
    const UChunk ch = chunks[blockIdx.x];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    double mh = 0.0, mm = 0.0;
    for (int64_t r = ch.r0 + wv; r < ch.r0 + ch.len; r += 4) {
        double sh = 0.0, smv = 0.0;
        for (int64_t e = row_ptr[r] + lane; e < row_ptr[r + 1]; e += 64) {
            sh += fabs(H[e]);
            smv += fabs(M[e]);
        }
        for (int d = 32; d >= 1; d >>= 1) {
            sh += __shfl_xor(sh, d, 64);
            smv += __shfl_xor(smv, d, 64);
        }
        mh = fmax(mh, sh);
        mm = fmax(mm, smv);
    }
    __shared__ double s[2][4];
    if (lane == 0) {
        s[0][wv] = mh;
        s[1][wv] = mm;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = fmax(fmax(s[0][0], s[0][1]), fmax(s[0][2], s[0][3]));
        part[2 * blockIdx.x + 1] = fmax(fmax(s[1][0], s[1][1]), fmax(s[1][2], s[1][3]));
    }
}

__global__ void rownorm_obj_kernel(int n_obj, const int *ufirst, const int *ucount, const double *part, double *norms) {
    const int o = blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= n_obj) return;
    double mh = 0.0, mm = 0.0;
    for (int q = 0; q < ucount[o]; ++q) {
        mh = fmax(mh, part[2 * (ufirst[o] + q)]);
        mm = fmax(mm, part[2 * (ufirst[o] + q) + 1]);
    }
    norms[2 * o] = mh;
    norms[2 * o + 1] = mm;
}

__global__ void diag_inv_bs_kernel(int64_t n, const int64_t *row_ptr, const int32_t *col, const double *H,
                                   double *d64, float *d32) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    int64_t lo = row_ptr[r], hi = row_ptr[r + 1] - 1;
    double d = 0.0;
    while (lo <= hi) {
        const int64_t mid = (lo + hi) >> 1;
        const int32_t c = col[mid];
        if (c == r) { d = H[mid]; break; }
        if (c < r) lo = mid + 1; else hi = mid - 1;
    }
    const double v = d > 0.0 ? 1.0 / d : 1.0;
    d64[r] = v;
    d32[r] = (float)v;
}

// d[r] = 1 / M_rr (1 where the diagonal is not positive)
__global__ void diag_inv_m_kernel(int64_t n, const int64_t *row_ptr, const int32_t *col, const double *M, double *d) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    int64_t lo = row_ptr[r], hi = row_ptr[r + 1] - 1;
    double v = 0.0;
    while (lo <= hi) {
        const int64_t mid = (lo + hi) >> 1;
        const int32_t c = col[mid];
        if (c == r) { v = M[mid]; break; }
        if (c < r) lo = mid + 1; else hi = mid - 1;
    }
    d[r] = v > 0.0 ? 1.0 / v : 1.0;
}

__global__ void fill_f64_kernel(int64_t count, double *a, double v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) a[i] = v;
}

// ---------------------------------------------------------------------------
// Chebyshev-Jacobi preconditioner: z = q(A) D^-1 r with A = D^-1 H, D = diag(H),
// q the Chebyshev semi-iteration polynomial of degree d for A z = D^-1 r on
// [a, b] (b an upper bound of the spectrum of A, a = b / ratio). q(x) > 0 on
// (0, b], so the preconditioner is SPD there. Per object: coef[0] = 1 / theta,
// coef[2s - 1], coef[2s] the step-s factors of dz (rho_s rho_{s-1}) and of r
// (2 rho_s / delta), theta = (a + b) / 2, delta = (b - a) / 2.
// ---------------------------------------------------------------------------

constexpr int kChebCoef = 32;                  // per-object coefficient stride (degree <= 16)
// defaults measured at 10^6 particles, k = 32, over start seeds (mean solve time): degree 8 and
// b / a = 30: 1.54 s, 8 and 1000: 1.22 s, 10 and 500: 0.99 s, 12 and 1000: 0.95 s, 14 and 1000:
// 1.00 s, 16 and 3000: 1.04 s; b / a beyond 1000 changes nothing
constexpr int kChebDefault = 12;               // degree when the caller passes 0
constexpr double kChebRatio = 1000.0;          // b / a when the caller passes 0
constexpr int kChebT8Sub = 1;                  // launch shape of the fused step (fewer registers than the
                                               // H-only product's default with the step's operands live)
// launch shape of the matrix-core Chebyshev step, the super-block pipelined kernel; the product alone
// at 10^6 particles, m = 32 / 64: full K-blocks with eight / four waves per workgroup 0.561 / 0.796 ms,
// zero-free K-blocks with four / two waves 0.510 / 0.781 ms (at six waves per SIMD, 80 registers,
// the four-wave form spilled and took 0.618 ms at m = 32). At m = 64 the single-buffer form (shape
// 13: 108 registers) takes the whole k = 64 solve from 1.403 to 1.395 s; at m = 32 it ties (0.557
// against 0.558 ms per step)
inline int cheb_tq_sub(int m, bool packed) {
    return packed ? (m == 32 ? rt::kTqPacked + 1 : 13) : (m == 32 ? 5 : 6);
}
// the matrix-core steps read the zero-free copy unless precond_values asks for the full K-blocks
constexpr bool kChebPackedDefault = true;

// Gershgorin bound of D^-1/2 H D^-1/2 per row: sum_j |H_ij| / sqrt(H_ii H_jj), one wavefront per row
__global__ void gersh_row_kernel(int64_t n, const int64_t *row_ptr, const int32_t *col, const double *H,
                                 const double *dinv, double *g) {
    const int lane = threadIdx.x & 63;
    const int64_t r = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    if (r >= n) return;
    double s = 0.0;
    for (int64_t e = row_ptr[r] + lane; e < row_ptr[r + 1]; e += 64) s += fabs(H[e]) * sqrt(dinv[col[e]]);
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) s += __shfl_xor(s, d, 64);
    if (lane == 0) g[r] = s * sqrt(dinv[r]);
}

// per chunk: max of g over its rows, and for the 8 power-iteration columns y^T H y and y^T D y
__global__ void __launch_bounds__(256) cheb_chunk_kernel(const GChunk *chunks, const double *g, const double *Y,
                                                         const double *HY, const double *dinv, double *part) {
    const GChunk ch = chunks[blockIdx.x];
    const int t = threadIdx.x;
    const int c = t & 7, rr = t >> 3;              // 32 row lanes x 8 columns
    double gm = 0.0, num = 0.0, den = 0.0;
    for (int64_t r = ch.r0 + rr; r < ch.r0 + ch.len; r += 32) {
        if (Y) {
            const double y = Y[r * 8 + c];
            num += y * HY[r * 8 + c];
            den += y * y / dinv[r];
        }
        if (c == 0) gm = fmax(gm, g[r]);
    }
    __shared__ double red[3][256];
    red[0][t] = gm;
    red[1][t] = num;
    red[2][t] = den;
    __syncthreads();
    if (t < 8) {
        double a = 0.0, b = 0.0, m = 0.0;
        for (int q = 0; q < 32; ++q) {
            m = fmax(m, red[0][q * 8 + t]);
            a += red[1][q * 8 + t];
            b += red[2][q * 8 + t];
        }
        part[(size_t)blockIdx.x * 17 + 1 + t] = a;
        part[(size_t)blockIdx.x * 17 + 9 + t] = b;
        if (t == 0) part[(size_t)blockIdx.x * 17] = m;   // the row maxima live in the c == 0 lanes
    }
}

// per object: sums over its chunks (ascending) -> out[o][17] (Gershgorin max, 8 numerators, 8 denominators)
__global__ void cheb_obj_kernel(int n_obj, const int *gfirst, const int *gcount, const double *part, double *out) {
    const int o = blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= n_obj) return;
    double v[17];
    for (int q = 0; q < 17; ++q) v[q] = 0.0;
    for (int c = gfirst[o]; c < gfirst[o] + gcount[o]; ++c) {
        v[0] = fmax(v[0], part[(size_t)c * 17]);
        for (int q = 1; q < 17; ++q) v[q] += part[(size_t)c * 17 + q];
    }
    for (int q = 0; q < 17; ++q) out[(size_t)o * 17 + q] = v[q];
}

// one power step y <- D^-1 H y / gersh(obj): the factor keeps the block bounded without normalisation
template <typename T>
__global__ void power_step_kernel(int64_t n, const int *row_obj, const double *objv, const T *HY, const T *dinv,
                                  T *Y) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * 8) return;
    const int64_t r = t >> 3;
    Y[t] = (T)((double)dinv[r] * (double)HY[t] / objv[(size_t)row_obj[r] * 17]);
}

template <typename T>
__global__ void to_f64_kernel(int64_t count, const T *a, double *b) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < count) b[t] = (double)a[t];
}
template <typename T>
__global__ void from_f64_kernel(int64_t count, const double *a, T *b) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < count) b[t] = (T)a[t];
}

// z0: R <- W (= D^-1 r, written by resid_kernel), dz = W / theta, W <- dz
template <typename T>
__global__ void cheb_init_kernel(int64_t n, int m, int64_t ld, const int *row_obj, const int *obj_status,
                                 const double *coef, T *S, T *Rb, T *DZ) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * m) return;
    const int64_t r = t / m;
    const int c = (int)(t - r * m);
    const int o = row_obj[r];
    if (obj_status[o] != 0) return;
    T *w = S + r * ld + m + c;
    const double v = (double)*w;
    const double dz = v * coef[(size_t)o * kChebCoef];
    Rb[t] = (T)v;
    DZ[t] = (T)dz;
    *w = (T)dz;
}

// The binary16 recurrence of the matrix-core steps starts from s W per object o and column c,
// s = 1 / max_rows |W[., c]| (1 for a zero column): the preconditioner is linear, so this scales
// column c of its output by s, which leaves the span the Rayleigh-Ritz step works on unchanged,
// and it keeps the iterates inside the binary16 range whatever the residuals' magnitude.
// one wavefront per (column, object): lanes stride the object's chunks, then a butterfly max
__global__ void colmax_obj_kernel(int n_obj, const int *obj_status, const int *cfirst, const int *ccount,
                                  const float *wpart, int m, float *cmax) {
    const int c = blockIdx.x, o = blockIdx.y, lane = threadIdx.x;
    if (o >= n_obj || c >= m || obj_status[o] != 0) return;
    float v = 0.f;
    for (int i = lane; i < ccount[o]; i += 64) v = fmaxf(v, wpart[(size_t)(cfirst[o] + i) * m + c]);
    for (int d = 32; d >= 1; d >>= 1) v = fmaxf(v, __shfl_xor(v, d, 64));
    if (lane == 0) cmax[(size_t)o * m + c] = v;
}

// z0 of the binary16 recurrence: R <- s W, dz = binary16(s W / theta), W <- dz; four columns per
// thread (m is a multiple of 16 on this path)
__global__ void cheb_init_q_kernel(int64_t n, int m, int64_t ld, const int *row_obj, const int *obj_status,
                                   const double *coef, const float *cmax, float *S, float *Rb, _Float16 *DZ) {
    typedef float f32x4_t __attribute__((ext_vector_type(4)));
    typedef _Float16 f16x4_t __attribute__((ext_vector_type(4)));
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int mq = m >> 2;
    if (t >= n * mq) return;
    const int64_t r = t / mq;
    const int c = 4 * (int)(t - r * mq);
    const int o = row_obj[r];
    if (obj_status[o] != 0) return;
    f32x4_t *w = (f32x4_t *)(S + r * ld + m + c);
    const f32x4_t wv = *w;
    const double th = coef[(size_t)o * kChebCoef];
    f32x4_t rv, wo;
    f16x4_t h;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const float mx = cmax[(size_t)o * m + c + q];
        const double v = (double)wv[q] * (mx > 0.f ? 1.0 / (double)mx : 1.0);
        double dz = v * th;
        dz = dz > 65504.0 ? 65504.0 : (dz < -65504.0 ? -65504.0 : dz);
        h[q] = (_Float16)(float)dz;
        rv[q] = (float)v;
        wo[q] = (float)h[q];
    }
    *(f32x4_t *)(Rb + r * m + c) = rv;
    *(f16x4_t *)(DZ + r * m + c) = h;
    *w = wo;
}

// step s: R -= D^-1 H dz, dz = f1 dz + f2 R, W += dz
template <typename T>
__global__ void cheb_step_kernel(int64_t n, int m, int64_t ld, int step, const int *row_obj, const int *obj_status,
                                 const double *coef, const T *dinv, const T *HD, T *S, T *Rb, T *DZ) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * m) return;
    const int64_t r = t / m;
    const int c = (int)(t - r * m);
    const int o = row_obj[r];
    if (obj_status[o] != 0) return;
    const double f1 = coef[(size_t)o * kChebCoef + 2 * step - 1], f2 = coef[(size_t)o * kChebCoef + 2 * step];
    const double rv = (double)Rb[t] - (double)dinv[r] * (double)HD[t];
    const double dz = f1 * (double)DZ[t] + f2 * rv;
    Rb[t] = (T)rv;
    DZ[t] = (T)dz;
    T *w = S + r * ld + m + c;
    *w = (T)((double)*w + dz);
}

__global__ void row_obj_kernel(int64_t N, const int64_t *obj_off, int n_obj, int *row_obj) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= N) return;
    int lo = 0, hi = n_obj - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (obj_off[mid] <= r) lo = mid; else hi = mid - 1;
    }
    row_obj[r] = lo;
}

__global__ void count_iter_kernel(int n_obj, const int *obj_status, int *iters) {
    const int o = blockIdx.x * blockDim.x + threadIdx.x;
    if (o < n_obj && obj_status[o] == 0) iters[o] += 1;
}

static const char *kVariantNames[] = {"waves4_unroll2_xcd", "waves4_unroll4_xcd", "waves8_unroll2_xcd",
                                      "waves4_unroll2_linear", "waves2_unroll4_xcd", "waves8_unroll4_xcd",
                                      "chunk64_waves4_batch8", "chunk64_waves2_batch8", "chunk64_waves8_batch8",
                                      "chunk64_waves4_batch4", "chunk64_waves2_batch8_occ6",
                                      "chunk64_waves4_batch4_occ8", "chunk64_waves2_batch16",
                                      "rowtile4_waves4_batch4", "rowtile4_waves2_batch8",
                                      "rowtile4_waves4_batch4_occ4", "rowtile8_mfma64_waves4_batch8",
                                      "rowtile8_mfma64_waves2_batch8", "rowtile8_mfma64_waves4_batch4_occ6",
                                      "rowtile8_mfma32x64_waves4_batch8", "rowtile8_mfma32x64_waves2_batch8",
                                      "rowtile8_mfma64_pipelined_waves4", "rowtile8_mfma32x64_pipelined_waves4",
                                      "rowtile8_mfma64_pipelined_waves2", "rowtile8_mfma64_zerofree_waves2",
                                      "rowtile8_mfma64_zerofree_waves4", "rowtile8_mfma32c4_pipelined_waves2"};
constexpr int kNumVariants = 27;
constexpr int kZeroFreeBase = 24;              // this one and the next read the zero-free eight-row copy
inline bool zero_free_variant(int v) { return v == kZeroFreeBase || v == kZeroFreeBase + 1; }
constexpr int kRowTileBase = 13;               // variants from here on run on a row-tile copy
constexpr int kRowTile8Base = 16;              // from here on: the eight-row [H, M] copy on MFMA (FP32 blocks)
constexpr int kCsrVariant = 11;                // fastest variant on the CSR itself
constexpr int kDefaultVariant64 = 14;  // fastest untuned FP64 choice on 10^5-10^6-row RKPM matrices (row tiles)
constexpr int kDefaultVariant32 = 23;  // other widths: the pipelined kernel on the FP64 matrix cores (1.31 /
                                       // 1.42 ms at m = 8 / 16 and 10^6 rows against 1.41-1.50 ms unpipelined)
constexpr int kDefaultVariant32m32 = 26;  // at m = 32: the pipelined kernel on the FP32 matrix cores, four
                                          // steps chained before each FP64 addition, two waves per workgroup
                                          // (1.65 ms against 1.72 ms on the FP64 matrix cores and 1.75-1.93
                                          // ms for the others at 10^6 rows)
constexpr int kDefaultVariant32m64 = 26;  // at m = 64 too: 2.22 ms against 3.07 ms for the fastest FP64
                                          // matrix-core form (two waves per workgroup), 3.10-3.47 ms for the rest

inline int rt_spmm(ff_ctx *ctx, hipStream_t st, const rt::RTView &v, int sub, int m, const float *Y, int64_t ldy,
                   float *HY, float *MY, int64_t ldo, const int *row_obj, const int *status) {
    return rt::spmm32(ctx, st, v, sub, m, Y, ldy, HY, MY, ldo, row_obj, status);
}
inline int rt_spmm(ff_ctx *ctx, hipStream_t st, const rt::RTView &v, int sub, int m, const double *Y, int64_t ldy,
                   double *HY, double *MY, int64_t ldo, const int *row_obj, const int *status) {
    return rt::spmm64(ctx, st, v, sub, m, Y, ldy, HY, MY, ldo, row_obj, status);
}

inline int rt_hm8(ff_ctx *ctx, hipStream_t st, const rt::RT8View &v, int sub, int m, const float *Y, int64_t ldy,
                  float *HY, float *MY, int64_t ldo, const int *row_obj, const int *status) {
    return rt::spmm_hm8(ctx, st, v, sub, m, Y, ldy, HY, MY, ldo, row_obj, status);
}
inline int rt_hm8(ff_ctx *ctx, hipStream_t, const rt::RT8View &, int, int, const double *, int64_t, double *,
                  double *, int64_t, const int *, const int *) {
    return set_error(ctx, FF_ERR_INVALID_ARG, "the eight-row MFMA SpMM variants take FP32 blocks only");
}

template <typename T>
int launch_spmm(ff_ctx *ctx, hipStream_t st, int variant, int64_t nrows, const int64_t *row_ptr, const int32_t *col,
                HMPair<T> hm, const T *Y, int64_t ldy, T *HY, T *MY, int64_t ldo, int m, const int *row_obj,
                const int *status, const rt::RTView *rtv, const rt::RT8View *rt8 = nullptr) {
    if (variant >= kRowTile8Base) {
        FF_REQUIRE(ctx, rt8 != nullptr && rt8->vm != nullptr, "eight-row SpMM variant without an eight-row copy");
        return rt_hm8(ctx, st, *rt8, variant - kRowTile8Base, m, Y, ldy, HY, MY, ldo, row_obj, status);
    }
    if (variant >= kRowTileBase) {
        FF_REQUIRE(ctx, rtv != nullptr, "row-tile SpMM variant without a row-tile copy");
        return rt_spmm(ctx, st, *rtv, variant - kRowTileBase, m, Y, ldy, HY, MY, ldo, row_obj, status);
    }
#define FF_SPMM(W, U, X)                                                                                        \
    hipLaunchKernelGGL((spmm_kernel<T, W, U, X>), dim3(grid_for(nrows, W)), dim3(64 * W), 0, st, nrows, row_ptr, \
                       col, hm, Y, ldy, HY, MY, ldo, m, row_obj, status)
#define FF_SPMMC(W, B, O)                                                                                         \
    hipLaunchKernelGGL((spmm_chunk_kernel<T, W, B, O>), dim3(grid_for(nrows, W)), dim3(64 * W), 0, st, nrows,      \
                       row_ptr, col, hm, Y, ldy, HY, MY, ldo, m, row_obj, status)
    switch (variant) {
        case 6: FF_SPMMC(4, 8, 1); break;
        case 7: FF_SPMMC(2, 8, 1); break;
        case 8: FF_SPMMC(8, 8, 1); break;
        case 9: FF_SPMMC(4, 4, 1); break;
        case 10: FF_SPMMC(2, 8, 6); break;
        case 11: FF_SPMMC(4, 4, 8); break;
        case 12: FF_SPMMC(2, 16, 1); break;
        case 1: FF_SPMM(4, 4, true); break;
        case 2: FF_SPMM(8, 2, true); break;
        case 3: FF_SPMM(4, 2, false); break;
        case 4: FF_SPMM(2, 4, true); break;
        case 5: FF_SPMM(8, 4, true); break;
        default: FF_SPMM(4, 2, true); break;
    }
#undef FF_SPMM
#undef FF_SPMMC
    FF_CHECK_LAUNCH(ctx);
    return FF_OK;
}

// HY = H Y alone (the preconditioner and the spectrum estimate): the row-tile
// H-only kernel where the solver runs a row-tile variant, else the fused
// product with MY written to the scratch block MS.
inline int rt_spmm_h(ff_ctx *ctx, hipStream_t st, const rt::RTView &v, int sub, int m, const float *Y, int64_t ldy,
                     float *HY, int64_t ldo, const int *row_obj, const int *status) {
    return rt::spmm_h32(ctx, st, v, sub, m, Y, ldy, HY, ldo, row_obj, status);
}
inline int rt_spmm_h(ff_ctx *ctx, hipStream_t st, const rt::RTView &v, int sub, int m, const double *Y, int64_t ldy,
                     double *HY, int64_t ldo, const int *row_obj, const int *status) {
    return rt::spmm_h64(ctx, st, v, sub, m, Y, ldy, HY, ldo, row_obj, status);
}
inline int rt_cheb_step(ff_ctx *ctx, hipStream_t st, const rt::RTView &v, int sub, int m, const float *DZ, int64_t ld,
                        const int *row_obj, const int *status, const rt::ChebStep<float> &cs) {
    return rt::cheb_step32(ctx, st, v, sub, m, DZ, ld, row_obj, status, cs);
}
inline int rt_cheb_step(ff_ctx *ctx, hipStream_t st, const rt::RTView &v, int sub, int m, const double *DZ, int64_t ld,
                        const int *row_obj, const int *status, const rt::ChebStep<double> &cs) {
    return rt::cheb_step64(ctx, st, v, sub, m, DZ, ld, row_obj, status, cs);
}
template <typename T>
int launch_spmm_h(ff_ctx *ctx, hipStream_t st, int variant, int64_t nrows, const int64_t *row_ptr, const int32_t *col,
                  HMPair<T> hm, const T *Y, int64_t ldy, T *HY, T *MS, int64_t ldo, int m, const int *row_obj,
                  const int *status, const rt::RTView *rtv, const rt::RT8View *rt8 = nullptr) {
    if (variant >= kRowTileBase && variant < kRowTile8Base && rtv &&
        (sizeof(T) == 4 ? rtv->v32 != nullptr : rtv->v64 != nullptr))
        return rt_spmm_h(ctx, st, *rtv, variant - kRowTileBase, m, Y, ldy, HY, ldo, row_obj, status);
    return launch_spmm<T>(ctx, st, variant, nrows, row_ptr, col, hm, Y, ldy, HY, MS, ldo, m, row_obj, status, rtv,
                          rt8);
}

template <typename T> struct Prec;
template <> struct Prec<float> {
    typedef float CT;
    static constexpr int vn = 4;
};
template <> struct Prec<double> {
    typedef double CT;
    static constexpr int vn = 2;
};

struct Solver {
    ff_ctx *ctx = nullptr;
    hipStream_t st = nullptr;
    int n_obj = 0;
    int64_t N = 0;
    std::vector<int64_t> off;
    const int64_t *row_ptr = nullptr;
    const int32_t *col = nullptr;
    const double *H = nullptr, *M = nullptr;
    const float *hm32 = nullptr;
    int m = 0, k = 0, wmax = 0;
    int var32 = 0, var64 = 0;
    rt::RTView rtv;                                // row-tile copy when a row-tile variant is selected
    rt::RT8View rt8;                               // eight-row H-only copy for the FP32 preconditioner
    rt::RT16View rt16;                             // sixteen-row H-only copy (MFMA form), preferred
    rt::RTQView rtq;                               // K-blocked binary16 copy: matrix-core Chebyshev steps
    bool q_on = false;                             // the FP32 preconditioner runs the matrix-core steps
    int tq_sub = 0;                                // their launch shape (the packed ones read the zero-free copy)
    float *wpart = nullptr, *cmax = nullptr;       // [chunks][m], [n_obj][m] column maxima of D^-1 R
    bool jacobi = false;
    int cheb = 0;                                  // Chebyshev-Jacobi degree (0: plain Jacobi or none)
    double *cheb_coef = nullptr;                   // [n_obj][kChebCoef]
    void *cheb_r = nullptr, *cheb_dz = nullptr, *cheb_hd = nullptr, *cheb_md = nullptr;   // [N][m] work blocks
    int *status = nullptr, *width = nullptr, *info = nullptr, *iters = nullptr, *row_obj = nullptr;
    int *ufirst = nullptr, *ucount = nullptr, *gfirst = nullptr, *gcount = nullptr;
    int64_t *obj_off = nullptr;
    double *theta = nullptr, *C = nullptr, *C64w = nullptr, *Cp = nullptr, *Cp64w = nullptr;
    double *G = nullptr, *gpart = nullptr, *rpart = nullptr;
    float *Cp32 = nullptr;
    double *res = nullptr, *track = nullptr, *norms = nullptr, *rrscr = nullptr, *dinv64 = nullptr;
    double *theta_next = nullptr;                  // [n_obj] next Ritz value beyond the block (NaN: unknown)
    double *ebound = nullptr, *abound = nullptr;   // [n_obj][m] eigenvalue and angle bounds of the pairs
    double *mdinv = nullptr;                       // [N] diag(M)^-1 for the bounds
    double eig_tol = 0.0;                          // FP64 phase: also require max ebound <= eig_tol
    double angle_tol = 0.0;                        // and max abound <= angle_tol
    int bounds_on = 0;                             // the residual stage forms the bounds (FP64 phase)
    float *S32 = nullptr;                          // FP32 blocks of the mixed path (its FP64 phase
                                                   // preconditions through them)
    float *C32 = nullptr, *dinv32 = nullptr;
    UChunk *uch = nullptr;
    GChunk *gch = nullptr;
    int nu = 0, ng = 0;
    int refresh32 = 30, refresh64 = 20;
    int total_iters = 0;
    int graph_used = 0;
};

template <typename T> HMPair<T> hm_of(const Solver &s);
template <> HMPair<float> hm_of<float>(const Solver &s) { return HMPair<float>{(const float2 *)s.hm32}; }
template <> HMPair<double> hm_of<double>(const Solver &s) { return HMPair<double>{s.H, s.M}; }
template <typename T> const T *dinv_of(const Solver &s);
template <> const float *dinv_of<float>(const Solver &s) { return s.dinv32; }
template <> const double *dinv_of<double>(const Solver &s) { return s.dinv64; }
template <typename T> typename Prec<T>::CT *cw_of(const Solver &s);
template <> float *cw_of<float>(const Solver &s) { return s.C32; }
template <> double *cw_of<double>(const Solver &s) { return s.C64w; }
template <typename T> typename Prec<T>::CT *cpw_of(const Solver &s);
template <> float *cpw_of<float>(const Solver &s) { return s.Cp32; }
template <> double *cpw_of<double>(const Solver &s) { return s.Cp64w; }

// C and C_p' in LDS for the block update when both padded copies fit in 128 KB
template <typename T> inline int update_c_in_lds(int wmax, int m) {
    return (size_t)2 * ((wmax + 3) & ~3) * ((m + 15) & ~15) * sizeof(T) <= 128 * 1024;
}
template <typename T> inline size_t update_shmem(int wmax, int m) {
    return update_c_in_lds<T>(wmax, m) ? (size_t)2 * ((wmax + 3) & ~3) * ((m + 15) & ~15) * sizeof(T) : 0;
}
// the fragment-order kernel: 16-byte row loads need 16-byte aligned rows (ld = 3m), at most
// four 16-column tiles (m <= 64), and its LDS copies within 128 KB
template <typename T> inline size_t update_frag_shmem(int wmax, int m) {
    return (size_t)2 * upd_nkb<T>(wmax) * 4 * UVec<T>::n * ((m + 15) & ~15) * sizeof(T);
}
template <typename T> inline int update_frag_ok(int wmax, int m) {
    return (3 * (size_t)m * sizeof(T)) % 16 == 0 && m <= 64 && update_frag_shmem<T>(wmax, m) <= 128 * 1024;
}

int set_width(Solver &s, int w, int only_active) {
    hipLaunchKernelGGL(set_width_kernel, dim3(grid_for(s.n_obj, 64)), dim3(64), 0, s.st, s.n_obj, s.status, s.width,
                       w, only_active);
    FF_CHECK_LAUNCH(s.ctx);
    return FF_OK;
}

template <typename T>
int stage_spmm(Solver &s, T *S, T *HS, T *MS, int slot) {
    StageMark mark(s.ctx, s.st, FF_STAGE_SPMM);
    const int64_t ld = 3 * (int64_t)s.m;
    return launch_spmm<T>(s.ctx, s.st, sizeof(T) == 4 ? s.var32 : s.var64, s.N, s.row_ptr, s.col, hm_of<T>(s),
                          S + slot * s.m, ld, HS + slot * s.m, MS + slot * s.m, ld, s.m, s.row_obj, s.status,
                          &s.rtv, &s.rt8);
}

// the four Rayleigh-Ritz stages on every active object (LDS limits set by rr_prepare)
template <typename CT>
int launch_rr(ff_ctx *ctx, hipStream_t st, int n_obj, int *status, const int *width, const double *G, int wmax, int m,
              double tau, double *scratch, double *C, CT *Cw, double *Cp, CT *Cpw, double *theta, int *info,
              double pmin = 0.0, double *theta_next = nullptr) {
    const int lds = rr_use_lds(wmax), vlds = rr_vec_lds(wmax);
    if (lds)
        hipLaunchKernelGGL(rr_tridiag_kernel<true>, dim3(n_obj), dim3(kRRThreads), rr_shmem_bytes(wmax, 1), st, status,
                           width, G, wmax, m, tau, pmin, scratch, info);
    else
        hipLaunchKernelGGL(rr_tridiag_kernel<false>, dim3(n_obj), dim3(kRRThreads), rr_shmem_bytes(wmax, 0), st,
                           status, width, G, wmax, m, tau, pmin, scratch, info);
    hipLaunchKernelGGL(rr_eig_kernel, dim3(theta_next ? m + 1 : m, n_obj), dim3(64), 0, st, status, wmax, m, scratch,
                       theta_next);
    if (vlds)
        hipLaunchKernelGGL(rr_vec_kernel<true>, dim3(m, n_obj), dim3(64), rr_vec_shmem_bytes(wmax, 1), st, status,
                           width, wmax, m, scratch, C, theta);
    else
        hipLaunchKernelGGL(rr_vec_kernel<false>, dim3(m, n_obj), dim3(64), rr_vec_shmem_bytes(wmax, 0), st, status,
                           width, wmax, m, scratch, C, theta);
    hipLaunchKernelGGL(rr_post_kernel<CT>, dim3(m, n_obj), dim3(256), 0, st, status, width, G, wmax, m, C, Cw, Cp,
                       Cpw);
    FF_CHECK_LAUNCH(ctx);
    return FF_OK;
}

// raise the dynamic LDS limits of the Rayleigh-Ritz kernels for blocks of width wmax
int gram_prepare(ff_ctx *ctx) {
    FF_HIP(ctx, hipFuncSetAttribute((const void *)gram_kernel<double, double>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)gram_shmem_bytes<double>()));
    FF_HIP(ctx, hipFuncSetAttribute((const void *)gram_kernel<float, float>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)gram_shmem_bytes<float>()));
    return FF_OK;
}

int rr_prepare(ff_ctx *ctx, int wmax) {
    const int lds = rr_use_lds(wmax), vlds = rr_vec_lds(wmax);
    FF_HIP(ctx, hipFuncSetAttribute(lds ? (const void *)rr_tridiag_kernel<true> : (const void *)rr_tridiag_kernel<false>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)rr_shmem_bytes(wmax, lds)));
    FF_HIP(ctx, hipFuncSetAttribute(vlds ? (const void *)rr_vec_kernel<true> : (const void *)rr_vec_kernel<false>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)rr_vec_shmem_bytes(wmax, vlds)));
    return FF_OK;
}

template <typename T>
int stage_gram_rr(Solver &s, T *S, T *HS, T *MS, double tau) {
    StageMark mark(s.ctx, s.st, FF_STAGE_GRAM);
    const int T16 = (s.wmax + 15) / 16, nsup = (T16 + 5) / 6;
    hipLaunchKernelGGL((gram_kernel<T, T>), dim3(s.ng, nsup * nsup), dim3(512), gram_shmem_bytes<T>(), s.st, s.gch,
                       s.status, s.width, S, HS, MS, (int64_t)3 * s.m, s.wmax, s.gpart, 1);
    FF_CHECK_LAUNCH(s.ctx);
    const int64_t per2 = 2 * (int64_t)s.wmax * s.wmax;
    hipLaunchKernelGGL(gram_reduce_kernel, dim3(grid_for(per2, 16), s.n_obj), dim3(256), 0, s.st, s.status, s.width,
                       s.gfirst, s.gcount, s.gpart, s.wmax, s.G);
    FF_CHECK_LAUNCH(s.ctx);
    mark.end();
    StageMark rr_mark(s.ctx, s.st, FF_STAGE_RR);
    // P columns below an M-norm of 1e-6 (FP32) or 1e-12 (FP64) leave the basis
    return launch_rr<typename Prec<T>::CT>(s.ctx, s.st, s.n_obj, s.status, s.width, s.G, s.wmax, s.m, tau, s.rrscr,
                                           s.C, cw_of<T>(s), s.Cp, cpw_of<T>(s), s.theta, s.info,
                                           sizeof(T) == 4 ? 1e-12 : 1e-24, s.theta_next);
}

template <typename T>
int stage_update(Solver &s, T *S, T *HS, T *MS, int write_p) {
    StageMark mark(s.ctx, s.st, FF_STAGE_UPDATE);
    if (update_frag_ok<T>(s.wmax, s.m)) {
        hipLaunchKernelGGL(update_frag_kernel<T>, dim3(s.nu), dim3(256), update_frag_shmem<T>(s.wmax, s.m), s.st,
                           s.uch, s.status, s.width, S, HS, MS, (int64_t)3 * s.m, s.m, s.wmax,
                           (const T *)cw_of<T>(s), (const T *)cpw_of<T>(s), write_p);
        FF_CHECK_LAUNCH(s.ctx);
        return FF_OK;
    }
    hipLaunchKernelGGL(update_kernel<T>, dim3(s.nu), dim3(256), update_shmem<T>(s.wmax, s.m), s.st, s.uch, s.status,
                       s.width, S, HS, MS, (int64_t)3 * s.m, s.m, s.wmax, (const T *)cw_of<T>(s),
                       (const T *)cpw_of<T>(s), write_p, update_c_in_lds<T>(s.wmax, s.m));
    FF_CHECK_LAUNCH(s.ctx);
    return FF_OK;
}

template <typename T>
int stage_resid(Solver &s, T *S, T *HS, T *MS, double tol, int stall) {
    StageMark mark(s.ctx, s.st, FF_STAGE_RESID);
    const bool bounds = s.bounds_on && sizeof(T) == 8;
    // the chunk maxima of D^-1 R feed the binary16 preconditioner, which the mixed path's FP64 phase uses too
    const bool wmx = s.q_on && (sizeof(T) == 4 || s.S32 != nullptr);
    hipLaunchKernelGGL(resid_kernel<T>, dim3(s.ng), dim3(256), 0, s.st, s.gch, s.status, S, (const T *)HS,
                       (const T *)MS, (int64_t)3 * s.m, s.m, s.theta, s.jacobi ? dinv_of<T>(s) : (const T *)nullptr,
                       bounds ? (const double *)s.mdinv : (const double *)nullptr, s.rpart,
                       wmx ? s.wpart : (float *)nullptr);
    FF_CHECK_LAUNCH(s.ctx);
    hipLaunchKernelGGL(norms_kernel, dim3(s.n_obj), dim3(1024), 0, s.st, s.status, s.gfirst, s.gcount, s.rpart, s.m,
                       s.k, s.theta, s.norms, tol, stall, s.res, s.track, (const double *)s.theta_next,
                       bounds ? s.eig_tol : 0.0, bounds ? s.angle_tol : 0.0, bounds ? s.ebound : (double *)nullptr,
                       bounds ? s.abound : (double *)nullptr);
    FF_CHECK_LAUNCH(s.ctx);
    hipLaunchKernelGGL(count_iter_kernel, dim3(grid_for(s.n_obj, 64)), dim3(64), 0, s.st, s.n_obj, s.status, s.iters);
    FF_CHECK_LAUNCH(s.ctx);
    return FF_OK;
}

// W <- q(D^-1 H) D^-1 R (the resid stage left D^-1 R in W)
template <typename T>
int stage_precond(Solver &s, T *S) {
    if (s.cheb < 2) return FF_OK;
    const int64_t cnt = s.N * s.m;
    const int64_t ld = 3 * (int64_t)s.m;
    if (sizeof(T) == 8 && s.S32 && (s.q_on || s.rt8.vh || s.rt16.vh)) {
        // the mixed path's FP64 phase: the preconditioner is an approximate operator, so it runs the
        // FP32 / binary16 products on an FP32 copy of D^-1 R (the FP32 blocks are free by now) and its
        // output returns to the FP64 W block; residuals, products of the basis, Grams and
        // Rayleigh-Ritz stay FP64
        hipLaunchKernelGGL((copy_block_kernel<float, double>), dim3(grid_for(cnt, 256)), dim3(256), 0, s.st, s.N, s.m,
                           (const double *)(S + s.m), ld, s.S32 + s.m, ld);
        FF_CHECK_LAUNCH(s.ctx);
        const int rc = stage_precond<float>(s, s.S32);
        if (rc) return rc;
        hipLaunchKernelGGL((copy_block_kernel<double, float>), dim3(grid_for(cnt, 256)), dim3(256), 0, s.st, s.N, s.m,
                           (const float *)(s.S32 + s.m), ld, (double *)(S + s.m), ld);
        FF_CHECK_LAUNCH(s.ctx);
        return FF_OK;
    }
    T *Rb = (T *)s.cheb_r, *DZ = (T *)s.cheb_dz, *HD = (T *)s.cheb_hd, *MD = (T *)s.cheb_md;
    if (sizeof(T) == 4 && s.q_on) {
        // binary16 iterate in the DZ buffer (two [N][m] halves), scaled start
        uint16_t *q16[2] = {(uint16_t *)s.cheb_dz, (uint16_t *)s.cheb_dz + s.N * s.m};
        {
            StageMark mark(s.ctx, s.st, FF_STAGE_PRECOND_OTHER);
            hipLaunchKernelGGL(colmax_obj_kernel, dim3(s.m, s.n_obj), dim3(64), 0, s.st, s.n_obj, s.status, s.gfirst,
                               s.gcount, s.wpart, s.m, s.cmax);
            FF_CHECK_LAUNCH(s.ctx);
            hipLaunchKernelGGL(cheb_init_q_kernel, dim3(grid_for(cnt / 4, 256)), dim3(256), 0, s.st, s.N, s.m, ld,
                               s.row_obj, s.status, s.cheb_coef, s.cmax, (float *)S, (float *)Rb, (_Float16 *)q16[0]);
            FF_CHECK_LAUNCH(s.ctx);
        }
        StageMark mark(s.ctx, s.st, FF_STAGE_PRECOND_PRODUCT, s.cheb - 1);
        for (int step = 1; step < s.cheb; ++step) {
            rt::ChebStepQ cs;
            cs.coef = s.cheb_coef;
            cs.stride = kChebCoef;
            cs.step = step;
            cs.dinv = (const float *)dinv_of<T>(s);
            cs.R = (float *)Rb;
            cs.W = (float *)(S + s.m);
            cs.ldw = ld;
            cs.dz_out = q16[step & 1];
            // W gathers two steps' iterates at every even step (and the last one's when it is odd)
            cs.wmode = (step & 1) == 0 ? 2 : (step == s.cheb - 1 ? 1 : 0);
            const int rc = rt::cheb_step_tq(s.ctx, s.st, s.rtq, s.tq_sub, s.m, q16[(step - 1) & 1], s.row_obj,
                                            s.status, cs);
            if (rc) return rc;
        }
        return FF_OK;
    }
    {
        StageMark mark(s.ctx, s.st, FF_STAGE_PRECOND_OTHER);
        hipLaunchKernelGGL(cheb_init_kernel<T>, dim3(grid_for(cnt, 256)), dim3(256), 0, s.st, s.N, s.m, ld,
                           s.row_obj, s.status, s.cheb_coef, S, Rb, DZ);
        FF_CHECK_LAUNCH(s.ctx);
    }
    StageMark mark(s.ctx, s.st, FF_STAGE_PRECOND_PRODUCT, s.cheb - 1);
    const int var = sizeof(T) == 4 ? s.var32 : s.var64;
    if (sizeof(T) == 4 && ((s.rt8.vh && rt::t8_ok(s.m, s.m, s.m)) || s.rt16.vh)) {
        T *buf[2] = {DZ, HD};
        for (int step = 1; step < s.cheb; ++step) {
            rt::ChebStep<float> cs;
            cs.coef = s.cheb_coef;
            cs.stride = kChebCoef;
            cs.step = step;
            cs.dinv = (const float *)dinv_of<T>(s);
            cs.R = (float *)Rb;
            cs.dz_out = (float *)buf[step & 1];
            cs.W = (float *)(S + s.m);
            cs.ldw = ld;
            const int rc = s.rt16.vh ? rt::cheb_step_t16(s.ctx, s.st, s.rt16, 0, s.m,
                                                         (const float *)buf[(step - 1) & 1], s.m, s.row_obj, s.status,
                                                         cs)
                                     : rt::cheb_step_t8(s.ctx, s.st, s.rt8, kChebT8Sub, s.m,
                                                        (const float *)buf[(step - 1) & 1], s.m, s.row_obj, s.status,
                                                        cs);
            if (rc) return rc;
        }
        return FF_OK;
    }
    if (var >= kRowTileBase && (sizeof(T) == 4 ? s.rtv.v32 != nullptr : s.rtv.v64 != nullptr)) {
        // fused: each step's product writes the next DZ into the other buffer
        T *buf[2] = {DZ, HD};
        for (int step = 1; step < s.cheb; ++step) {
            rt::ChebStep<T> cs;
            cs.coef = s.cheb_coef;
            cs.stride = kChebCoef;
            cs.step = step;
            cs.dinv = dinv_of<T>(s);
            cs.R = Rb;
            cs.dz_out = buf[step & 1];
            cs.W = S + s.m;
            cs.ldw = ld;
            const int rc = rt_cheb_step(s.ctx, s.st, s.rtv, var - kRowTileBase, s.m, buf[(step - 1) & 1], s.m,
                                        s.row_obj, s.status, cs);
            if (rc) return rc;
        }
        return FF_OK;
    }
    for (int step = 1; step < s.cheb; ++step) {
        int rc = launch_spmm_h<T>(s.ctx, s.st, var, s.N, s.row_ptr, s.col, hm_of<T>(s),
                                  DZ, s.m, HD, MD, s.m, s.m, s.row_obj, s.status, &s.rtv, &s.rt8);
        if (rc) return rc;
        hipLaunchKernelGGL(cheb_step_kernel<T>, dim3(grid_for(cnt, 256)), dim3(256), 0, s.st, s.N, s.m, ld, step,
                           s.row_obj, s.status, s.cheb_coef, dinv_of<T>(s), HD, S, Rb, DZ);
        FF_CHECK_LAUNCH(s.ctx);
    }
    return FF_OK;
}

// X-only Rayleigh-Ritz: images of X, M-orthonormalise and diagonalise
template <typename T>
int init_block(Solver &s, T *S, T *HS, T *MS, double tau) {
    int rc;
    if ((rc = stage_spmm<T>(s, S, HS, MS, 0))) return rc;
    if ((rc = set_width(s, s.m, 1))) return rc;
    if ((rc = stage_gram_rr<T>(s, S, HS, MS, tau))) return rc;
    if ((rc = stage_update<T>(s, S, HS, MS, 0))) return rc;
    return set_width(s, 2 * s.m, 1);
}

// Chebyshev-Jacobi set-up: per object, the Gershgorin bound g of D^-1/2 H D^-1/2 and
// the largest Rayleigh quotient of D^-1 H after 30 steps of power iteration on 8
// seeded vectors (in the working precision); b = min(1.1 x quotient, g), a = b / ratio.
template <typename T>
int cheb_setup(Solver &s, int degree, double ratio, uint64_t seed, double upper = 0.0, double *b_used = nullptr) {
    ff_ctx *ctx = s.ctx;
    const int64_t N = s.N;
    const int n_obj = s.n_obj;
    const size_t blk = (size_t)N * s.m * sizeof(double);
    s.cheb_r = ws_get(ctx, WS_CHEB0, blk);
    s.cheb_dz = ws_get(ctx, WS_CHEB1, blk);
    s.cheb_hd = ws_get(ctx, WS_CHEB2, blk);
    s.cheb_md = ws_get(ctx, WS_CHEB3, blk);
    double *aux = (double *)ws_get(ctx, WS_CHEB4, ((size_t)n_obj * (kChebCoef + 17) + (size_t)s.ng * 17 + N) *
                                                      sizeof(double));
    if (!s.cheb_r || !s.cheb_dz || !s.cheb_hd || !s.cheb_md || !aux) return FF_ERR_OOM;
    s.cheb_coef = aux;
    double *objv = aux + (size_t)n_obj * kChebCoef, *part = objv + (size_t)n_obj * 17, *grow = part + (size_t)s.ng * 17;
    const int var = sizeof(T) == 4 ? s.var32 : s.var64;
    // Gershgorin bounds
    hipLaunchKernelGGL(gersh_row_kernel, dim3(grid_for(N, 4)), dim3(256), 0, s.st, N, s.row_ptr, s.col, s.H, s.dinv64,
                       grow);
    hipLaunchKernelGGL(cheb_chunk_kernel, dim3(s.ng), dim3(256), 0, s.st, s.gch, grow, (const double *)nullptr,
                       (const double *)nullptr, s.dinv64, part);
    hipLaunchKernelGGL(cheb_obj_kernel, dim3(grid_for(n_obj, 64)), dim3(64), 0, s.st, n_obj, s.gfirst, s.gcount, part,
                       objv);
    FF_CHECK_LAUNCH(ctx);
    // power iteration on 8 columns: Y in cheb_r, HY in cheb_hd, MY in cheb_md (stride 8)
    T *Y = (T *)s.cheb_r, *HY = (T *)s.cheb_hd, *MY = (T *)s.cheb_md;
    double *Yd = (double *)s.cheb_dz;
    hipLaunchKernelGGL(philox_block_kernel, dim3(grid_for((N * 8 + 3) / 4, 256)), dim3(256), 0, s.st, N * 8,
                       seed ^ 0x9e3779b97f4a7c15ull, Yd);
    hipLaunchKernelGGL(from_f64_kernel<T>, dim3(grid_for(N * 8, 256)), dim3(256), 0, s.st, N * 8, (const double *)Yd, Y);
    FF_CHECK_LAUNCH(ctx);
    int rc;
    auto hprod = [&]() -> int {
        if (sizeof(T) == 4 && s.rt16.vh)
            return rt::spmm_h_t16(ctx, s.st, s.rt16, 0, 8, (const float *)Y, 8, (float *)HY, 8, s.row_obj, s.status);
        if (sizeof(T) == 4 && s.rt8.vh)       // the power steps run at m = 8, which the eight-row kernel takes
            return rt::spmm_h_t8(ctx, s.st, s.rt8, 0, 8, (const float *)Y, 8, (float *)HY, 8, s.row_obj, s.status);
        return launch_spmm_h<T>(ctx, s.st, var, N, s.row_ptr, s.col, hm_of<T>(s), Y, 8, HY, MY, 8, 8, s.row_obj,
                                s.status, &s.rtv, &s.rt8);
    };
    for (int it = 0; it < 30; ++it) {
        if ((rc = hprod())) return rc;
        hipLaunchKernelGGL(power_step_kernel<T>, dim3(grid_for(N * 8, 256)), dim3(256), 0, s.st, N, s.row_obj, objv,
                           HY, dinv_of<T>(s), Y);
        FF_CHECK_LAUNCH(ctx);
    }
    if ((rc = hprod())) return rc;
    double *HYd = (double *)s.cheb_md;            // MY is no longer needed
    hipLaunchKernelGGL(to_f64_kernel<T>, dim3(grid_for(N * 8, 256)), dim3(256), 0, s.st, N * 8, (const T *)Y, Yd);
    hipLaunchKernelGGL(to_f64_kernel<T>, dim3(grid_for(N * 8, 256)), dim3(256), 0, s.st, N * 8, (const T *)HY, HYd);
    hipLaunchKernelGGL(cheb_chunk_kernel, dim3(s.ng), dim3(256), 0, s.st, s.gch, grow, (const double *)Yd,
                       (const double *)HYd, s.dinv64, part);
    hipLaunchKernelGGL(cheb_obj_kernel, dim3(grid_for(n_obj, 64)), dim3(64), 0, s.st, n_obj, s.gfirst, s.gcount, part,
                       objv);
    FF_CHECK_LAUNCH(ctx);
    std::vector<double> hv((size_t)n_obj * 17), coef((size_t)n_obj * kChebCoef, 0.0);
    FF_HIP(ctx, hipMemcpyAsync(hv.data(), objv, hv.size() * sizeof(double), hipMemcpyDeviceToHost, s.st));
    FF_HIP(ctx, hipStreamSynchronize(s.st));
    for (int o = 0; o < n_obj; ++o) {
        const double *v = hv.data() + (size_t)o * 17;
        double lam = 0.0;
        for (int j = 0; j < 8; ++j)
            if (v[9 + j] > 0.0) lam = std::max(lam, v[1 + j] / v[9 + j]);
        const double g = v[0] > 0.0 ? v[0] : 1.0;
        const double b = upper > 0.0 ? upper : (lam > 0.0 && lam == lam) ? std::min(1.1 * lam, g) : g;
        if (b_used && o == 0) *b_used = b;
        const double a = b / ratio, theta = 0.5 * (a + b), delta = 0.5 * (b - a), sigma = theta / delta;
        double *c = coef.data() + (size_t)o * kChebCoef;
        c[0] = 1.0 / theta;
        double rho_prev = 1.0 / sigma;
        for (int step = 1; step < degree; ++step) {
            const double rho = 1.0 / (2.0 * sigma - rho_prev);
            c[2 * step - 1] = rho * rho_prev;
            c[2 * step] = 2.0 * rho / delta;
            rho_prev = rho;
        }
        if (ctx->verbose) fprintf(stderr, "[freeform] object %d: Gershgorin %.4g, power estimate %.4g, b %.4g\n", o, g, lam, b);
    }
    FF_HIP(ctx, hipMemcpyAsync(s.cheb_coef, coef.data(), coef.size() * sizeof(double), hipMemcpyHostToDevice, s.st));
    FF_HIP(ctx, hipStreamSynchronize(s.st));
    s.cheb = degree;
    return FF_OK;
}

template <typename T>
int body(Solver &s, T *S, T *HS, T *MS, double tol, int stall, double tau) {
    int rc;
    if ((rc = stage_resid<T>(s, S, HS, MS, tol, stall))) return rc;
    if ((rc = stage_precond<T>(s, S))) return rc;
    if ((rc = stage_spmm<T>(s, S, HS, MS, 1))) return rc;
    if ((rc = stage_gram_rr<T>(s, S, HS, MS, tau))) return rc;
    if ((rc = stage_update<T>(s, S, HS, MS, 1))) return rc;
    return set_width(s, 3 * s.m, 1);
}

// Iterate until every object has left the active state or max_iters is spent.
template <typename T>
int run_phase(Solver &s, T *S, T *HS, T *MS, int max_iters, double tol, int stall, double tau, int check_every,
              int use_graph, int refresh, int *done_iters, int first_check = 0) {
    int it = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int *hstat = (int *)pinned_get(s.ctx, (size_t)s.n_obj * sizeof(int) + 64);
    if (!hstat) return FF_ERR_OOM;
    int rc = FF_OK;
    if (use_graph) {
        if (hipStreamBeginCapture(s.st, hipStreamCaptureModeThreadLocal) != hipSuccess) {
            (void)hipGetLastError();
            use_graph = 0;
        } else {
            rc = body<T>(s, S, HS, MS, tol, stall, tau);
            hipError_t e = hipStreamEndCapture(s.st, &graph);
            if (rc || e != hipSuccess) {
                if (graph) (void)hipGraphDestroy(graph);
                return rc ? rc : set_error(s.ctx, FF_ERR_HIP, "graph capture failed: %s", hipGetErrorString(e));
            }
            e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
            if (e != hipSuccess) {
                (void)hipGraphDestroy(graph);
                return set_error(s.ctx, FF_ERR_HIP, "graph instantiate failed: %s", hipGetErrorString(e));
            }
            s.graph_used = 1;
        }
    }
    while (it < max_iters) {
        const int steps = std::min(it == 0 && first_check > 0 ? first_check : check_every, max_iters - it);
        for (int j = 0; j < steps; ++j) {
            if (refresh > 0 && it > 0 && it % refresh == 0) {
                // recompute the images of X and P so the recurrences do not drift
                if ((rc = stage_spmm<T>(s, S, HS, MS, 0))) break;
                if ((rc = stage_spmm<T>(s, S, HS, MS, 2))) break;
            }
            if (exec) {
                if (hipGraphLaunch(exec, s.st) != hipSuccess) {
                    rc = set_error(s.ctx, FF_ERR_HIP, "graph launch failed");
                    break;
                }
            } else if ((rc = body<T>(s, S, HS, MS, tol, stall, tau))) {
                break;
            }
            ++it;
        }
        if (rc) break;
        if (hipMemcpyAsync(hstat, s.status, (size_t)s.n_obj * sizeof(int), hipMemcpyDeviceToHost, s.st) != hipSuccess ||
            hipStreamSynchronize(s.st) != hipSuccess) {
            rc = set_error(s.ctx, FF_ERR_HIP, "status read failed: %s", hipGetErrorString(hipGetLastError()));
            break;
        }
        bool all = true;
        for (int o = 0; o < s.n_obj; ++o) all = all && hstat[o] != 0;
        if (s.ctx->verbose) {
            std::vector<double> rs((size_t)s.m);
            if (hipMemcpy(rs.data(), s.res, rs.size() * sizeof(double), hipMemcpyDeviceToHost) == hipSuccess) {
                double mx = 0.0;
                int jmax = 0, above = 0;
                for (int j = 0; j < s.k; ++j) {
                    if (rs[j] > mx) {
                        mx = rs[j];
                        jmax = j;
                    }
                    above += rs[j] > tol;
                }
                fprintf(stderr, "[freeform] %s it %d: object 0 max resid %.3e (pair %d, %d above tol) status %d\n",
                        sizeof(T) == 4 ? "fp32" : "fp64", it, mx, jmax, above, hstat[0]);
            }
        }
        if (all) break;
    }
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    *done_iters = it;
    return rc;
}

int reset_status(Solver &s, int keep_converged) {
    hipLaunchKernelGGL(reset_status_kernel, dim3(grid_for(s.n_obj, 64)), dim3(64), 0, s.st, s.n_obj, s.status, s.track,
                       keep_converged);
    FF_CHECK_LAUNCH(s.ctx);
    return FF_OK;
}

template <typename T>
int alloc_blocks(Solver &s, int slot_s, int slot_h, int slot_m, T **S, T **HS, T **MS) {
    const size_t bytes = (size_t)s.N * 3 * s.m * sizeof(T);
    *S = (T *)ws_get(s.ctx, slot_s, bytes);
    *HS = (T *)ws_get(s.ctx, slot_h, bytes);
    *MS = (T *)ws_get(s.ctx, slot_m, bytes);
    if (!*S || !*HS || !*MS) return FF_ERR_OOM;
    return FF_OK;
}

// The preconditioner alone (chebyshev_apply): its input R goes into the X-slot images HX with MX = 0
// and theta = 0, so the residual kernel forms W = D^-1 R and the chunk maxima of |W| exactly as in an
// iteration; then the same preconditioner stage, and W is the output.
struct ChebApply {
    const float *R;
    int64_t ld_r;
    float *Z;
    int64_t ld_z;
    double upper;
    double *upper_used;
};

int cheb_apply_run(Solver &s, const ChebApply &a) {
    float *S32, *HS32, *MS32;
    int rc = alloc_blocks<float>(s, WS_S0, WS_HS0, WS_MS0, &S32, &HS32, &MS32);
    if (rc) return rc;
    const int64_t ld = 3 * (int64_t)s.m, cnt = s.N * ld;
    FF_HIP(s.ctx, hipMemsetAsync(S32, 0, (size_t)cnt * sizeof(float), s.st));
    FF_HIP(s.ctx, hipMemsetAsync(MS32, 0, (size_t)cnt * sizeof(float), s.st));
    hipLaunchKernelGGL((copy_block_kernel<float, float>), dim3(grid_for(s.N * s.m, 256)), dim3(256), 0, s.st, s.N, s.m,
                       a.R, a.ld_r, HS32, ld);
    FF_CHECK_LAUNCH(s.ctx);
    if ((rc = reset_status(s, 0))) return rc;
    s.S32 = S32;
    hipLaunchKernelGGL(resid_kernel<float>, dim3(s.ng), dim3(256), 0, s.st, s.gch, s.status, S32, (const float *)HS32,
                       (const float *)MS32, ld, s.m, s.theta, (const float *)s.dinv32, (const double *)nullptr, s.rpart,
                       s.q_on ? s.wpart : (float *)nullptr);
    FF_CHECK_LAUNCH(s.ctx);
    if ((rc = stage_precond<float>(s, S32))) return rc;
    hipLaunchKernelGGL((copy_block_kernel<float, float>), dim3(grid_for(s.N * s.m, 256)), dim3(256), 0, s.st, s.N, s.m,
                       (const float *)(S32 + s.m), ld, a.Z, a.ld_z);
    FF_CHECK_LAUNCH(s.ctx);
    FF_HIP(s.ctx, hipStreamSynchronize(s.st));
    return FF_OK;
}

int setup(Solver &s, const ff_eig_params *p) {
    ff_ctx *ctx = s.ctx;
    const int n_obj = s.n_obj;
    std::vector<UChunk> u;
    std::vector<GChunk> g;
    std::vector<int> uf(n_obj), uc(n_obj), gf(n_obj), gc(n_obj);
    for (int o = 0; o < n_obj; ++o) {
        uf[o] = (int)u.size();
        for (int64_t r = s.off[o]; r < s.off[o + 1]; r += 256)
            u.push_back(UChunk{r, (int32_t)std::min<int64_t>(256, s.off[o + 1] - r), o});
        uc[o] = (int)u.size() - uf[o];
        gf[o] = (int)g.size();
        for (int64_t r = s.off[o]; r < s.off[o + 1]; r += 2048)
            g.push_back(GChunk{r, (int32_t)std::min<int64_t>(2048, s.off[o + 1] - r), o});
        gc[o] = (int)g.size() - gf[o];
    }
    s.nu = (int)u.size();
    s.ng = (int)g.size();
    s.uch = (UChunk *)ws_get(ctx, WS_CHUNKS, u.size() * sizeof(UChunk));
    s.gch = (GChunk *)ws_get(ctx, WS_GCHUNKS, g.size() * sizeof(GChunk));
    int *ints = (int *)ws_get(ctx, WS_OBJ, (size_t)n_obj * 9 * sizeof(int) + 256);
    s.obj_off = (int64_t *)ws_get(ctx, WS_SIGN, (size_t)(n_obj + 1) * sizeof(int64_t));
    s.row_obj = (int *)ws_get(ctx, WS_TUNE, (size_t)s.N * sizeof(int));
    if (!s.uch || !s.gch || !ints || !s.obj_off || !s.row_obj) return FF_ERR_OOM;
    s.ufirst = ints;
    s.ucount = ints + n_obj;
    s.gfirst = ints + 2 * n_obj;
    s.gcount = ints + 3 * n_obj;
    s.status = ints + 4 * n_obj;
    s.width = ints + 5 * n_obj;
    s.info = ints + 6 * n_obj;
    s.iters = ints + 7 * n_obj;
    FF_HIP(ctx, hipMemcpyAsync(s.uch, u.data(), u.size() * sizeof(UChunk), hipMemcpyHostToDevice, s.st));
    FF_HIP(ctx, hipMemcpyAsync(s.gch, g.data(), g.size() * sizeof(GChunk), hipMemcpyHostToDevice, s.st));
    FF_HIP(ctx, hipMemcpyAsync(s.ufirst, uf.data(), n_obj * sizeof(int), hipMemcpyHostToDevice, s.st));
    FF_HIP(ctx, hipMemcpyAsync(s.ucount, uc.data(), n_obj * sizeof(int), hipMemcpyHostToDevice, s.st));
    FF_HIP(ctx, hipMemcpyAsync(s.gfirst, gf.data(), n_obj * sizeof(int), hipMemcpyHostToDevice, s.st));
    FF_HIP(ctx, hipMemcpyAsync(s.gcount, gc.data(), n_obj * sizeof(int), hipMemcpyHostToDevice, s.st));
    FF_HIP(ctx, hipMemcpyAsync(s.obj_off, s.off.data(), (n_obj + 1) * sizeof(int64_t), hipMemcpyHostToDevice, s.st));
    FF_HIP(ctx, hipMemsetAsync(s.status, 0, (size_t)n_obj * 4 * sizeof(int), s.st));
    // the pageable host vectors above must outlive the copies
    FF_HIP(ctx, hipStreamSynchronize(s.st));
    hipLaunchKernelGGL(row_obj_kernel, dim3(grid_for(s.N, 256)), dim3(256), 0, s.st, s.N, s.obj_off, n_obj, s.row_obj);
    FF_CHECK_LAUNCH(ctx);

    const int m = s.m, wmax = s.wmax;
    s.theta = (double *)ws_get(ctx, WS_THETA, (size_t)n_obj * m * sizeof(double) * 4 + (size_t)n_obj * 5 * sizeof(double));
    s.res = s.theta + (size_t)n_obj * m;
    s.track = s.res + (size_t)n_obj * m;
    s.norms = s.track + 2 * (size_t)n_obj;
    s.theta_next = s.norms + 2 * (size_t)n_obj;
    s.ebound = s.theta_next + (size_t)n_obj;
    s.abound = s.ebound + (size_t)n_obj * m;
    s.C = (double *)ws_get(ctx, WS_C, (size_t)n_obj * wmax * m * sizeof(double) * 4);
    s.C64w = s.C ? s.C + (size_t)n_obj * wmax * m : nullptr;
    s.Cp = s.C ? s.C + (size_t)2 * n_obj * wmax * m : nullptr;
    s.Cp64w = s.C ? s.C + (size_t)3 * n_obj * wmax * m : nullptr;
    s.C32 = (float *)ws_get(ctx, WS_C32, (size_t)n_obj * wmax * m * sizeof(float) * 2);
    s.Cp32 = s.C32 ? s.C32 + (size_t)n_obj * wmax * m : nullptr;
    s.G = (double *)ws_get(ctx, WS_G, (size_t)n_obj * 2 * wmax * wmax * sizeof(double));
    s.gpart = (double *)ws_get(ctx, WS_GPART, (size_t)s.ng * 2 * wmax * wmax * sizeof(double));
    s.rpart = (double *)ws_get(ctx, WS_RPART, (size_t)std::max(s.nu, s.ng) * 3 * std::max(m, 2) * sizeof(double));
    s.rrscr = (double *)ws_get(ctx, WS_RRSCR, (size_t)n_obj * rr_scratch_doubles(wmax, m) * sizeof(double));
    if (!s.theta || !s.C || !s.C32 || !s.G || !s.gpart || !s.rpart || !s.rrscr) return FF_ERR_OOM;
    FF_HIP(ctx, hipMemsetAsync(s.theta, 0, (size_t)n_obj * m * sizeof(double) * 2, s.st));
    // the next Ritz value is unknown (NaN) until a Rayleigh-Ritz step on more than m columns; the
    // bounds are infinite until the FP64 phase forms them
    hipLaunchKernelGGL(fill_f64_kernel, dim3(grid_for(n_obj, 256)), dim3(256), 0, s.st, (int64_t)n_obj, s.theta_next,
                       (double)NAN);
    hipLaunchKernelGGL(fill_f64_kernel, dim3(grid_for((int64_t)n_obj * 2 * m, 256)), dim3(256), 0, s.st,
                       (int64_t)n_obj * 2 * m, s.ebound, (double)INFINITY);
    FF_CHECK_LAUNCH(ctx);
    s.eig_tol = p->eig_tol;
    s.angle_tol = p->angle_tol;
    s.mdinv = (double *)ws_get(ctx, WS_MDINV, (size_t)s.N * sizeof(double));
    if (!s.mdinv) return FF_ERR_OOM;
    hipLaunchKernelGGL(diag_inv_m_kernel, dim3(grid_for(s.N, 256)), dim3(256), 0, s.st, s.N, s.row_ptr, s.col, s.M,
                       s.mdinv);
    FF_CHECK_LAUNCH(ctx);

    // per-object norms of H and M (infinity norm = max absolute row sum)
    hipLaunchKernelGGL(rownorm_chunk_kernel, dim3(s.nu), dim3(256), 0, s.st, s.uch, s.row_ptr, s.H, s.M, s.rpart);
    FF_CHECK_LAUNCH(ctx);
    hipLaunchKernelGGL(rownorm_obj_kernel, dim3(grid_for(n_obj, 64)), dim3(64), 0, s.st, n_obj, s.ufirst, s.ucount,
                       s.rpart, s.norms);
    FF_CHECK_LAUNCH(ctx);
    s.jacobi = p->precond == 1 || p->precond == 2;
    if (s.jacobi) {
        s.dinv64 = (double *)ws_get(ctx, WS_DINV, (size_t)s.N * sizeof(double));
        s.dinv32 = (float *)ws_get(ctx, WS_DINV32, (size_t)s.N * sizeof(float));
        if (!s.dinv64 || !s.dinv32) return FF_ERR_OOM;
        hipLaunchKernelGGL(diag_inv_bs_kernel, dim3(grid_for(s.N, 256)), dim3(256), 0, s.st, s.N, s.row_ptr, s.col, s.H,
                           s.dinv64, s.dinv32);
        FF_CHECK_LAUNCH(ctx);
    }
    FF_HIP(ctx, hipFuncSetAttribute((const void *)update_kernel<double>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)update_shmem<double>(wmax, m)));
    FF_HIP(ctx, hipFuncSetAttribute((const void *)update_kernel<float>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)update_shmem<float>(wmax, m)));
    if (update_frag_ok<double>(wmax, m))
        FF_HIP(ctx, hipFuncSetAttribute((const void *)update_frag_kernel<double>,
                                        hipFuncAttributeMaxDynamicSharedMemorySize,
                                        (int)update_frag_shmem<double>(wmax, m)));
    if (update_frag_ok<float>(wmax, m))
        FF_HIP(ctx, hipFuncSetAttribute((const void *)update_frag_kernel<float>,
                                        hipFuncAttributeMaxDynamicSharedMemorySize,
                                        (int)update_frag_shmem<float>(wmax, m)));
    int rc = gram_prepare(ctx);
    return rc ? rc : rr_prepare(ctx, wmax);
}

std::string tune_key(int64_t n, int64_t nnz, int m, int precision) {
    char buf[128];
    const double per = n > 0 ? (double)nnz / (double)n : 0.0;
    snprintf(buf, sizeof(buf), "n%lld_r%d_m%d_p%d", (long long)n, (int)(per + 0.5), m, precision);
    return buf;
}

int lookup_variant(ff_ctx *ctx, int64_t n, int64_t nnz, int m, int precision) {
    auto it = ctx->tuned.find(tune_key(n, nnz, m, precision));
    if (it != ctx->tuned.end()) return it->second;
    return precision ? (m == 32 ? kDefaultVariant32m32 : m == 64 ? kDefaultVariant32m64 : kDefaultVariant32)
                     : kDefaultVariant64;
}

int solve(ff_ctx *ctx, int n_obj, const int64_t *obj_off, const int64_t *row_ptr, const int32_t *col, const double *H,
          const double *M, const float *hm32, const ff_eig_params *p, const double *X0, double *eigval, double *W,
          double *resid, ff_eig_info *info, const ChebApply *apply = nullptr) {
    auto t_start = std::chrono::steady_clock::now();
    timing_reset(ctx);
    FF_REQUIRE(ctx, p != nullptr && row_ptr && col && H && M && (apply || (eigval && W && resid)),
               "required pointer is NULL");
    FF_REQUIRE(ctx, !apply || (n_obj == 1 && p->precision == 1 && p->precond == 2 && apply->R && apply->Z),
               "the preconditioner alone runs on one object, mixed precision, Chebyshev-Jacobi");
    FF_REQUIRE(ctx, n_obj >= 1 && obj_off, "bad object list");
    FF_REQUIRE(ctx, p->k >= 1, "k must be >= 1");
    FF_REQUIRE(ctx, p->precision == 0 || p->precision == 1, "precision must be 0 or 1");
    FF_REQUIRE(ctx, p->precision == 0 || hm32, "mixed precision needs the FP32 copies (hm32)");
    FF_REQUIRE(ctx, p->tol > 0.0 && p->max_iter >= 0, "bad tolerance or iteration cap");
    FF_REQUIRE(ctx, p->precond >= 0 && p->precond <= 2, "precond must be 0, 1 or 2");
    FF_REQUIRE(ctx, p->precond != 2 || p->precond_degree == 0 || (p->precond_degree >= 2 && p->precond_degree <= 16),
               "Chebyshev degree %d must be 0 (default %d) or in [2, 16]", p->precond_degree, kChebDefault);
    FF_REQUIRE(ctx, p->precond != 2 || p->precond_ratio == 0.0 || (p->precond_ratio > 1.0 && p->precond_ratio <= 1e6),
               "Chebyshev interval ratio %g must be 0 (default %g) or in (1, 1e6]", p->precond_ratio, kChebRatio);
    FF_REQUIRE(ctx, p->eig_tol >= 0.0 && p->eig_tol == p->eig_tol, "eig_tol must be >= 0");
    FF_REQUIRE(ctx, p->angle_tol >= 0.0 && p->angle_tol == p->angle_tol, "angle_tol must be >= 0");
    FF_REQUIRE(ctx, p->precond_values >= 0 && p->precond_values <= 4,
               "precond_values %d must be 0 (default), 1 (FP32), 2 (binary16 H), 3 (binary16 H and iterate) or 4 "
               "(3 without the K-blocks' zeros)",
               p->precond_values);
    int m = p->block > 0 ? p->block : ((p->k + 7) / 8) * 8;
    FF_REQUIRE(ctx, m >= p->k && m % 8 == 0 && m >= 8 && m <= 64, "block %d: needs k <= m <= 64, m multiple of 8", m);
    FF_REQUIRE(ctx,
               p->precision != 1 || p->precond != 2 || (p->precond_values != 3 && p->precond_values != 4) ||
                   rt::tq_ok(m),
               "precond_values %d (binary16 iterate) needs block width 32 or 64 (m = %d)", p->precond_values, m);
    Solver s;
    s.ctx = ctx;
    FF_HIP(ctx, hipSetDevice(ctx->device));
    s.st = ctx->stream;
    int use_graph = p->use_graph;
    if (use_graph && s.st == nullptr) {
        // the null stream cannot be captured: run this call on a private stream
        if (!ctx->graph_stream) FF_HIP(ctx, hipStreamCreateWithFlags(&ctx->graph_stream, hipStreamNonBlocking));
        FF_HIP(ctx, hipStreamSynchronize(nullptr));
        s.st = ctx->graph_stream;
    }
    s.n_obj = n_obj;
    s.off.assign(obj_off, obj_off + n_obj + 1);
    for (int o = 0; o < n_obj; ++o)
        FF_REQUIRE(ctx, s.off[o + 1] - s.off[o] >= m, "object %d has %lld rows, fewer than the block width %d", o,
                   (long long)(s.off[o + 1] - s.off[o]), m);
    FF_REQUIRE(ctx, s.off[0] == 0, "obj_row_off[0] must be 0");
    s.N = s.off[n_obj];
    s.row_ptr = row_ptr;
    s.col = col;
    s.H = H;
    s.M = M;
    s.hm32 = hm32;
    s.m = m;
    s.k = p->k;
    s.wmax = 3 * m;
    if (p->refresh_every > 0) s.refresh32 = s.refresh64 = p->refresh_every;
    int64_t *hnnz = (int64_t *)pinned_get(ctx, 4096);
    if (!hnnz) return FF_ERR_OOM;
    FF_HIP(ctx, hipMemcpyAsync(hnnz, row_ptr + s.N, sizeof(int64_t), hipMemcpyDeviceToHost, s.st));
    FF_HIP(ctx, hipStreamSynchronize(s.st));
    const int64_t nnz = hnnz[0];
    s.var32 = lookup_variant(ctx, s.N, nnz, m, 1);
    s.var64 = lookup_variant(ctx, s.N, nnz, m, 0);
    {
        // the mixed path's FP64 phase is normally the certification alone: it keeps the CSR
        // (kCsrVariant) rather than paying for an FP64 row-tile copy; refining to an eigenvalue or
        // angle bound takes hundreds of FP64 iterations at 10^6 rows, where the copy (tens of ms to
        // build) halves each product (2.9 against 5.9 ms)
        if (p->precision == 1 && s.var64 >= kRowTileBase && p->eig_tol == 0.0 && p->angle_tol == 0.0)
            s.var64 = kCsrVariant;
        // the FP64 blocks never take the eight-row MFMA variants (FP32 only); nor do block widths they lack
        if (s.var64 >= kRowTile8Base) s.var64 = kDefaultVariant64;
        if (s.var32 >= kRowTile8Base && !rt::hm8_ok(m, 3 * (int64_t)m, 3 * (int64_t)m)) s.var32 = kDefaultVariant64;
        const int want32 = p->precision == 1 && s.var32 >= kRowTileBase && s.var32 < kRowTile8Base,
                  want64 = s.var64 >= kRowTileBase;
        if (want32 || want64) {
            int rc0 = rt::build_ws(ctx, s.st, s.N, row_ptr, col, H, M, want32, want64, &s.rtv);
            if (rc0) return rc0;
        }
        if (p->precision == 1 && s.var32 >= kRowTile8Base) {
            // one eight-row copy with H and M serves the fused products and the preconditioner
            int rc0 = rt::build_t8_ws(ctx, s.st, s.N, row_ptr, col, H, &s.rt8, M);
            if (!rc0 && zero_free_variant(s.var32)) rc0 = rt::build_t8z_ws(ctx, s.st, &s.rt8);
            if (rc0) return rc0;
        }
    }
    int rc = setup(s, p);
    if (rc) return rc;
    if (p->precond == 2) {
        const int degree = p->precond_degree > 0 ? p->precond_degree : kChebDefault;
        // the FP32 preconditioner's products run on tiles of eight rows when the block shape allows
        // (the sixteen-row MFMA form measured slower than the eight-row one: 1.38 against 1.23 ms per
        // product at 1M particles, m = 32; it serves the widths the eight-row kernel does not take)
        if (p->precision == 1 && s.var32 >= kRowTileBase && rt::t8_ok(s.m, s.m, s.m)) {
            if (!s.rt8.vh) rc = rt::build_t8_ws(ctx, s.st, s.N, row_ptr, col, H, &s.rt8);
            // H in binary16 for these products: 1.75 value slots per nonzero at 2 bytes instead of 4;
            // with the iterate in binary16 too (block widths 32 and 64) the products run on the matrix
            // cores, otherwise on the FP32 VALU
            const bool q = p->precond_values == 3 || p->precond_values == 4 ||
                           (p->precond_values == 0 && rt::tq_ok(s.m));
            FF_REQUIRE(ctx, !q || rt::tq_ok(s.m), "binary16 iterate needs block width 32 or 64 (m = %d)", s.m);
            if (!rc && q) {
                rc = rt::build_tq(ctx, s.st, s.rt8, &s.rtq);
                // the K-blocks without their zeros (44% of the full blocks' values at 10^6 particles)
                const bool packed = p->precond_values == 4 || (p->precond_values == 0 && kChebPackedDefault);
                if (!rc && packed) rc = rt::build_tq_pack_ws(ctx, s.st, &s.rtq);
                s.tq_sub = cheb_tq_sub(s.m, packed);
                if (ctx->cheb_shape >= 0) {
                    FF_REQUIRE(ctx, ctx->cheb_shape < rt::kTqSubs && (ctx->cheb_shape >= rt::kTqPacked) == packed,
                               "FF_CHEB_SHAPE=%d is not a launch shape of the %s K-blocks", ctx->cheb_shape,
                               packed ? "zero-free" : "full");
                    s.tq_sub = ctx->cheb_shape;
                }
                // the power steps of the interval estimate (eight columns) read the binary16 copy too
                if (!rc) rc = rt::build_t8_half(ctx, s.st, &s.rt8);
                s.wpart = (float *)ws_get(ctx, WS_CHEBQ, ((size_t)s.ng + s.n_obj) * s.m * sizeof(float));
                if (!rc && !s.wpart) rc = FF_ERR_OOM;
                s.cmax = s.wpart + (size_t)s.ng * s.m;
                s.q_on = rc == FF_OK;
            } else if (!rc && p->precond_values != 1) {
                rc = rt::build_t8_half(ctx, s.st, &s.rt8);
            }
            if (rc) return rc;
        } else if (p->precision == 1 && s.var32 >= kRowTileBase && rt::t16_ok(s.m, s.m, s.m)) {
            rc = rt::build_t16_ws(ctx, s.st, s.N, row_ptr, col, H, &s.rt16);
            if (rc) return rc;
        }
        const double ratio = p->precond_ratio > 0.0 ? p->precond_ratio : kChebRatio;
        rc = p->precision == 1 ? cheb_setup<float>(s, degree, ratio, p->seed, apply ? apply->upper : 0.0,
                                                   apply ? apply->upper_used : nullptr)
                               : cheb_setup<double>(s, degree, ratio, p->seed);
        if (rc) return rc;
    }
    if (apply) return cheb_apply_run(s, *apply);
    const int check_every = p->check_every > 0 ? p->check_every : 10;
    const double tau32 = 1e-5, tau64 = 1e-13;
    constexpr int kStall32 = 200;

    double *S64, *HS64, *MS64;
    if ((rc = alloc_blocks<double>(s, WS_D0, WS_HD0, WS_MD0, &S64, &HS64, &MS64))) return rc;
    // starting block in FP64 (given, or Philox uniform [-1, 1))
    double *X0d = nullptr;
    if (X0) {
        X0d = (double *)X0;
    } else {
        X0d = (double *)ws_get(ctx, WS_S1, (size_t)s.N * m * sizeof(double));
        if (!X0d) return FF_ERR_OOM;
        hipLaunchKernelGGL(philox_block_kernel, dim3(grid_for((s.N * m + 3) / 4, 256)), dim3(256), 0, s.st, s.N * m,
                           p->seed, X0d);
        FF_CHECK_LAUNCH(ctx);
    }
    int it32 = 0, it64 = 0;
    std::vector<int> its32((size_t)n_obj, 0);
    if ((rc = reset_status(s, 0))) return rc;
    if (p->precision == 1) {
        float *S32, *HS32, *MS32;
        if ((rc = alloc_blocks<float>(s, WS_S0, WS_HS0, WS_MS0, &S32, &HS32, &MS32))) return rc;
        hipLaunchKernelGGL((copy_block_kernel<float, double>), dim3(grid_for(s.N * m, 256)), dim3(256), 0, s.st, s.N, m,
                           (const double *)X0d, (int64_t)m, S32, (int64_t)3 * m);
        FF_CHECK_LAUNCH(ctx);
        s.S32 = S32;
        if ((rc = init_block<float>(s, S32, HS32, MS32, tau32))) return rc;
        // the FP32 phase ends at tol, or when its residual has not dropped by 10% for kStall32
        // iterations (its rounding floor); the largest residual is not monotone, and bumps
        // lasting tens of iterations occur in exact arithmetic too
        if ((rc = run_phase<float>(s, S32, HS32, MS32, p->max_iter, p->tol, kStall32, tau32, check_every, use_graph,
                                   s.refresh32, &it32)))
            return rc;
        FF_HIP(ctx, hipMemcpyAsync(its32.data(), s.iters, its32.size() * sizeof(int), hipMemcpyDeviceToHost, s.st));
        FF_HIP(ctx, hipMemsetAsync(s.iters, 0, its32.size() * sizeof(int), s.st));
        hipLaunchKernelGGL((copy_block_kernel<double, float>), dim3(grid_for(s.N * m, 256)), dim3(256), 0, s.st, s.N, m,
                           (const float *)S32, (int64_t)3 * m, S64, (int64_t)3 * m);
        FF_CHECK_LAUNCH(ctx);
    } else {
        hipLaunchKernelGGL((copy_block_kernel<double, double>), dim3(grid_for(s.N * m, 256)), dim3(256), 0, s.st, s.N, m,
                           (const double *)X0d, (int64_t)m, S64, (int64_t)3 * m);
        FF_CHECK_LAUNCH(ctx);
    }
    // FP64: Rayleigh-Ritz on X with the FP64 matrices (the certification), then iterate if needed. In the
    // mixed path this phase is timed as one stage, so the per-stage figures describe the FP32 iterations
    // (its passes after every object has converged launch kernels that return at once)
    {
        StageMark phase(ctx, s.st, FF_STAGE_FP64_PHASE);
        TimingMute mute(ctx, p->precision == 1);
        s.bounds_on = 1;                  // the residual stage forms the a-posteriori bounds from here on
        if ((rc = reset_status(s, 0))) return rc;
        if ((rc = init_block<double>(s, S64, HS64, MS64, tau64))) return rc;
        const int left = std::max(0, p->max_iter - it32);
        // after the FP32 phase the first FP64 pass normally certifies every pair: check right after it
        if ((rc = run_phase<double>(s, S64, HS64, MS64, left + 1, p->tol, 0, tau64, check_every, use_graph,
                                    s.refresh64, &it64, p->precision == 1 ? 1 : 0)))
            return rc;
    }
    // outputs: eigenvalues, residuals, bounds, sign-fixed vectors
    std::vector<double> th((size_t)n_obj * m), rs((size_t)n_obj * m), eb((size_t)n_obj * m), ab((size_t)n_obj * m);
    FF_HIP(ctx, hipMemcpyAsync(eb.data(), s.ebound, eb.size() * sizeof(double), hipMemcpyDeviceToHost, s.st));
    FF_HIP(ctx, hipMemcpyAsync(ab.data(), s.abound, ab.size() * sizeof(double), hipMemcpyDeviceToHost, s.st));
    std::vector<int> st((size_t)n_obj), its((size_t)n_obj), inf((size_t)n_obj);
    FF_HIP(ctx, hipMemcpyAsync(th.data(), s.theta, th.size() * sizeof(double), hipMemcpyDeviceToHost, s.st));
    FF_HIP(ctx, hipMemcpyAsync(rs.data(), s.res, rs.size() * sizeof(double), hipMemcpyDeviceToHost, s.st));
    FF_HIP(ctx, hipMemcpyAsync(st.data(), s.status, st.size() * sizeof(int), hipMemcpyDeviceToHost, s.st));
    FF_HIP(ctx, hipMemcpyAsync(its.data(), s.iters, its.size() * sizeof(int), hipMemcpyDeviceToHost, s.st));
    FF_HIP(ctx, hipMemcpyAsync(inf.data(), s.info, inf.size() * sizeof(int), hipMemcpyDeviceToHost, s.st));
    const int nparts = 64;
    double *pv = (double *)ws_get(ctx, WS_RES, (size_t)m * nparts * (sizeof(double) + sizeof(int64_t)) + 64 * 8);
    if (!pv) return FF_ERR_OOM;
    int64_t *pi = (int64_t *)(pv + (size_t)m * nparts);
    double *sgn = (double *)(pi + (size_t)m * nparts);
    for (int o = 0; o < n_obj; ++o) {
        hipLaunchKernelGGL(sign_partial_kernel, dim3(nparts, s.k), dim3(256), 0, s.st, s.off[o], s.off[o + 1], m, S64,
                           (int64_t)3 * m, pv, pi);
        FF_CHECK_LAUNCH(ctx);
        const int64_t rows = s.off[o + 1] - s.off[o];
        hipLaunchKernelGGL(sign_final_kernel, dim3(1), dim3(64), 0, s.st, s.k, S64, (int64_t)3 * m, nparts, pv, pi,
                           sgn);
        FF_CHECK_LAUNCH(ctx);
        hipLaunchKernelGGL(sign_apply_kernel, dim3(grid_for(rows * s.k, 256)), dim3(256), 0, s.st, s.off[o],
                           s.off[o + 1], s.k, S64, (int64_t)3 * m, sgn, W, (int64_t)s.k);
        FF_CHECK_LAUNCH(ctx);
    }
    FF_HIP(ctx, hipStreamSynchronize(s.st));
    bool all_conv = true, broke = false;
    double worst = 0.0;
    ctx->eb_nobj = n_obj;
    ctx->eb_k = s.k;
    ctx->eb_eig.assign((size_t)n_obj * s.k, INFINITY);
    ctx->eb_angle.assign((size_t)n_obj * s.k, INFINITY);
    for (int o = 0; o < n_obj; ++o) {
        double mx = 0.0, mxe = 0.0, mxa = 0.0;
        for (int j = 0; j < s.k; ++j) {
            eigval[(size_t)o * s.k + j] = th[(size_t)o * m + j];
            resid[(size_t)o * s.k + j] = rs[(size_t)o * m + j];
            mx = std::max(mx, rs[(size_t)o * m + j]);
            const double e = eb[(size_t)o * m + j], a = ab[(size_t)o * m + j];
            ctx->eb_eig[(size_t)o * s.k + j] = e;
            ctx->eb_angle[(size_t)o * s.k + j] = a;
            mxe = (e == e) ? std::max(mxe, e) : INFINITY;
            mxa = (a == a) ? std::max(mxa, a) : INFINITY;
        }
        const bool conv = st[o] == 1 && mx <= p->tol;
        all_conv = all_conv && conv;
        broke = broke || st[o] == 3;
        worst = std::max(worst, mx);
        if (info) {
            info[o].iters_fp32 = its32[o];
            info[o].iters_fp64 = its[o];
            info[o].graph = s.graph_used;
            info[o].converged = conv;
            info[o].restarts = (inf[o] >> 16) & 1;
            info[o].max_resid = mx;
            info[o].seconds = 0.0;
            info[o].max_eig_bound = mxe;
            info[o].max_angle_bound = mxa;
            info[o].eig_certified = mxe <= (p->eig_tol > 0.0 ? p->eig_tol : 1e-5) &&
                                    (p->angle_tol <= 0.0 || mxa <= p->angle_tol);
        }
    }
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
    if (info)
        for (int o = 0; o < n_obj; ++o) info[o].seconds = secs;
    timing_collect(ctx);
    ctx->stage_ms[FF_STAGE_TOTAL] = secs * 1e3;
    ctx->stage_launches[FF_STAGE_TOTAL] = 1;
    if (broke && !all_conv) return set_error(ctx, FF_ERR_BREAKDOWN, "Rayleigh-Ritz basis lost rank");
    if (!all_conv)
        return set_error(ctx, FF_ERR_NOT_CONVERGED, "max residual %.3e above tol %.3e after %d + %d iterations", worst,
                         p->tol, it32, it64);
    return FF_OK;
}

}  // namespace lob
}  // namespace ff

using namespace ff;
using namespace ff::lob;

// row i of the dense pencil [H; M] (n x n each, row-major) from the CSR: the row is cleared, then its
// entries are written (one workgroup per row)
__global__ void __launch_bounds__(256) csr_dense_kernel(int64_t n, const int64_t *row_ptr, const int32_t *col,
                                                        const double *H, const double *M, double *G) {
    const int64_t i = blockIdx.x;
    if (i >= n) return;
    double *gh = G + i * n, *gm = G + n * n + i * n;
    for (int64_t j = threadIdx.x; j < n; j += blockDim.x) gh[j] = gm[j] = 0.0;
    __syncthreads();
    for (int64_t e = row_ptr[i] + threadIdx.x; e < row_ptr[i + 1]; e += blockDim.x) {
        gh[col[e]] = H[e];
        gm[col[e]] = M[e];
    }
}

// An object with fewer than five block widths of rows leaves the block iteration no room: its search
// space [X, W, P] is most of the space and the basis loses rank (the oracle's LOBPCG stalls there
// too). When such an object is small enough for the Rayleigh-Ritz kernels (at most 192 rows), its
// start block is the exact lowest m eigenvectors of the dense pencil, Rayleigh-Ritz on the identity
// basis; the iteration then finds them converged and certifies them as any other answer.
constexpr int kDenseStartRows = 192;

extern "C" int eigenmodes(ff_ctx *ctx, int64_t n, const int64_t *row_ptr, const int32_t *col, const double *H,
                          const double *M, const float *hm32, const ff_eig_params *p, const double *X0, double *eigval,
                          double *W, double *resid, ff_eig_info *info) {
    if (!ctx) return FF_ERR_INVALID_ARG;
    FF_REQUIRE(ctx, n > 0, "n must be positive");
    FF_REQUIRE(ctx, p != nullptr, "bad arguments");
    const int64_t off[2] = {0, n};
    const int m = p->block > 0 ? p->block : ((p->k + 7) / 8) * 8;
    if (!X0 && p->k >= 1 && m >= 8 && m <= 64 && m <= n && n < 5 * (int64_t)m && n <= kDenseStartRows && row_ptr &&
        col && H && M) {
        FF_HIP(ctx, hipSetDevice(ctx->device));
        double *G = (double *)ws_get(ctx, WS_DENSE, (size_t)2 * n * n * sizeof(double));
        double *Xd = (double *)ws_get(ctx, WS_DENSE_X, ((size_t)n * m + m) * sizeof(double));
        if (!G || !Xd) return FF_ERR_OOM;
        hipLaunchKernelGGL(csr_dense_kernel, dim3((unsigned)n), dim3(256), 0, ctx->stream, n, row_ptr, col, H, M, G);
        FF_CHECK_LAUNCH(ctx);
        int kept = 0;
        const int rc = rayleigh_ritz(ctx, (int)n, m, G, 1e-13, Xd, Xd + (size_t)n * m, &kept);
        if (rc) return rc;
        return solve(ctx, 1, off, row_ptr, col, H, M, hm32, p, Xd, eigval, W, resid, info);
    }
    return solve(ctx, 1, off, row_ptr, col, H, M, hm32, p, X0, eigval, W, resid, info);
}

extern "C" int eigenmodes_batched(ff_ctx *ctx, int n_obj, const int64_t *obj_row_off, const int64_t *row_ptr,
                                  const int32_t *col, const double *H, const double *M, const float *hm32,
                                  const ff_eig_params *p, const double *X0, double *eigval, double *W, double *resid,
                                  ff_eig_info *info) {
    if (!ctx) return FF_ERR_INVALID_ARG;
    return solve(ctx, n_obj, obj_row_off, row_ptr, col, H, M, hm32, p, X0, eigval, W, resid, info);
}

extern "C" int chebyshev_apply(ff_ctx *ctx, int64_t n, const int64_t *row_ptr, const int32_t *col, const double *H,
                               const double *M, const float *hm32, int m, int degree, double ratio, int values,
                               double upper, const float *R, int64_t ld_r, float *Z, int64_t ld_z,
                               double *upper_used) {
    if (!ctx) return FF_ERR_INVALID_ARG;
    FF_REQUIRE(ctx, n > 0, "n must be positive");
    FF_REQUIRE(ctx, R && Z && hm32, "required pointer is NULL");
    FF_REQUIRE(ctx, m >= 8 && m <= 64 && m % 8 == 0, "block width %d must be a multiple of 8 in [8, 64]", m);
    FF_REQUIRE(ctx, ld_r >= m && ld_z >= m, "leading dimensions must be >= m");
    FF_REQUIRE(ctx, degree >= 2 && degree <= 16, "degree %d must be in [2, 16]", degree);
    FF_REQUIRE(ctx, values >= 1 && values <= 4, "values %d must be 1 .. 4", values);
    FF_REQUIRE(ctx, upper >= 0.0 && std::isfinite(upper), "upper must be finite and >= 0");
    ff_eig_params p;
    memset(&p, 0, sizeof(p));
    p.k = m;
    p.block = m;
    p.precision = 1;
    p.tol = 1e-6;
    p.max_iter = 1;
    p.precond = 2;
    p.precond_degree = degree;
    p.precond_ratio = ratio;
    p.precond_values = values;
    ChebApply a{R, ld_r, Z, ld_z, upper, upper_used};
    const int64_t off[2] = {0, n};
    return solve(ctx, 1, off, row_ptr, col, H, M, hm32, &p, nullptr, nullptr, nullptr, nullptr, nullptr, &a);
}

extern "C" int eig_bounds(ff_ctx *ctx, int n_obj, int k, double *eig_bound, double *angle_bound) {
    if (!ctx) return FF_ERR_INVALID_ARG;
    FF_REQUIRE(ctx, n_obj == ctx->eb_nobj && k == ctx->eb_k && n_obj > 0,
               "n_obj %d, k %d differ from the last eigensolve's (%d, %d)", n_obj, k, ctx->eb_nobj, ctx->eb_k);
    if (eig_bound) memcpy(eig_bound, ctx->eb_eig.data(), ctx->eb_eig.size() * sizeof(double));
    if (angle_bound) memcpy(angle_bound, ctx->eb_angle.data(), ctx->eb_angle.size() * sizeof(double));
    return FF_OK;
}

extern "C" int spmm_hm(ff_ctx *ctx, int64_t n, const int64_t *row_ptr, const int32_t *col, const double *H,
                       const double *M, const float *hm32, int precision, int m, const void *Y, int64_t ld_y, void *HY,
                       void *MY, int64_t ld_out, int variant) {
    if (!ctx) return FF_ERR_INVALID_ARG;
    FF_REQUIRE(ctx, n > 0 && row_ptr && col && Y && HY && MY, "required pointer is NULL");
    FF_REQUIRE(ctx, precision == 0 || precision == 1, "precision must be 0 or 1");
    const int vn = precision ? 4 : 2;
    FF_REQUIRE(ctx, m > 0 && m % vn == 0 && m / vn <= 64, "block width %d not supported", m);
    FF_REQUIRE(ctx, ld_y >= m && ld_out >= m && ld_y % vn == 0 && ld_out % vn == 0, "bad leading dimension");
    FF_HIP(ctx, hipSetDevice(ctx->device));
    int v = variant;
    if (v < 0) {
        int64_t *h = (int64_t *)pinned_get(ctx, 4096);
        if (!h) return FF_ERR_OOM;
        FF_HIP(ctx, hipMemcpyAsync(h, row_ptr + n, sizeof(int64_t), hipMemcpyDeviceToHost, ctx->stream));
        FF_HIP(ctx, hipStreamSynchronize(ctx->stream));
        v = lookup_variant(ctx, n, h[0], m, precision);
    }
    FF_REQUIRE(ctx, v >= 0 && v < kNumVariants, "variant %d out of range", v);
    // a row-tile variant builds its copy of the matrix for this call (rowtiles_build keeps one)
    rt::RTView view;
    rt::RT8View view8;
    if (v >= kRowTile8Base) {
        FF_REQUIRE(ctx, precision == 1, "variant %d (%s) takes FP32 blocks only", v, kVariantNames[v]);
        FF_REQUIRE(ctx, H && M, "row-tile variants need H and M");
        FF_REQUIRE(ctx, rt::hm8_ok(m, ld_y, ld_out), "variant %d takes m in {4, 8, 12, 16, 32, 64}, m = %d", v, m);
        int rc = rt::build_t8_ws(ctx, ctx->stream, n, row_ptr, col, H, &view8, M);
        if (!rc && zero_free_variant(v)) rc = rt::build_t8z_ws(ctx, ctx->stream, &view8);
        if (rc) return rc;
    } else if (v >= kRowTileBase) {
        FF_REQUIRE(ctx, H && M, "row-tile variants need H and M");
        int rc = rt::build_ws(ctx, ctx->stream, n, row_ptr, col, H, M, precision, !precision, &view);
        if (rc) return rc;
    }
    if (precision) {
        FF_REQUIRE(ctx, hm32 != nullptr || v >= kRowTileBase, "hm32 is NULL");
        return launch_spmm<float>(ctx, ctx->stream, v, n, row_ptr, col, HMPair<float>{(const float2 *)hm32},
                                  (const float *)Y, ld_y, (float *)HY, (float *)MY, ld_out, m, nullptr, nullptr,
                                  &view, &view8);
    }
    FF_REQUIRE(ctx, H && M, "H or M is NULL");
    return launch_spmm<double>(ctx, ctx->stream, v, n, row_ptr, col, HMPair<double>{H, M}, (const double *)Y, ld_y,
                               (double *)HY, (double *)MY, ld_out, m, nullptr, nullptr, &view);
}

extern "C" int spmm_variant_count(void) { return kNumVariants; }

extern "C" int spmm_variant_selected(ff_ctx *ctx, int64_t n, int64_t nnz, int m, int precision) {
    if (!ctx) return FF_ERR_INVALID_ARG;
    return lookup_variant(ctx, n, nnz, m, precision);
}

extern "C" const char *spmm_variant_name(int variant) {
    return (variant >= 0 && variant < kNumVariants) ? kVariantNames[variant] : "invalid";
}

extern "C" int spmm_autotune(ff_ctx *ctx, int64_t n, const int64_t *row_ptr, const int32_t *col, const double *H,
                             const double *M, const float *hm32, int precision, int m, const char *cache_path,
                             int *best_variant, double *best_ms) {
    if (!ctx) return FF_ERR_INVALID_ARG;
    FF_REQUIRE(ctx, best_variant && best_ms, "required pointer is NULL");
    FF_REQUIRE(ctx, n > 0 && row_ptr && col && H && M && (precision == 0 || hm32), "bad arguments");
    FF_REQUIRE(ctx, precision == 0 || precision == 1, "precision must be 0 or 1");
    FF_REQUIRE(ctx, m > 0 && m % (precision ? 4 : 2) == 0 && m / (precision ? 4 : 2) <= 64,
               "block width %d not supported", m);
    FF_HIP(ctx, hipSetDevice(ctx->device));
    int64_t *h = (int64_t *)pinned_get(ctx, 4096);
    if (!h) return FF_ERR_OOM;
    FF_HIP(ctx, hipMemcpyAsync(h, row_ptr + n, sizeof(int64_t), hipMemcpyDeviceToHost, ctx->stream));
    FF_HIP(ctx, hipStreamSynchronize(ctx->stream));
    const int64_t nnz = h[0];
    const std::string key = tune_key(n, nnz, m, precision);
    // cached result from the file
    if (cache_path) {
        if (FILE *f = fopen(cache_path, "r")) {
            char line[512];
            while (fgets(line, sizeof(line), f)) {
                char k2[256];
                int v;
                double ms;
                if (sscanf(line, " \"%255[^\"]\": {\"variant\": %d, \"ms\": %lf", k2, &v, &ms) == 3 && key == k2 &&
                    v >= 0 && v < kNumVariants) {
                    ctx->tuned[key] = v;
                    *best_variant = v;
                    *best_ms = ms;
                    fclose(f);
                    return FF_OK;
                }
            }
            fclose(f);
        }
    }
    const size_t esz = precision ? sizeof(float) : sizeof(double);
    char *buf = (char *)ws_get(ctx, WS_MLP7, (size_t)n * m * esz * 3);
    if (!buf) return FF_ERR_OOM;
    FF_HIP(ctx, hipMemsetAsync(buf, 0, (size_t)n * m * esz, ctx->stream));
    hipEvent_t e0, e1;
    FF_HIP(ctx, hipEventCreate(&e0));
    FF_HIP(ctx, hipEventCreate(&e1));
    int best = 0;
    double bms = 1e30;
    rt::RTView view;
    rt::RT8View view8;
    int have_view = 0, have_view8 = 0;
    for (int v = 0; v < kNumVariants; ++v) {
        if (v >= kRowTile8Base && (!precision || !rt::hm8_ok(m, m, m))) continue;
        if (v >= kRowTileBase && v < kRowTile8Base && !have_view) {
            int rc0 = rt::build_ws(ctx, ctx->stream, n, row_ptr, col, H, M, precision, !precision, &view);
            if (rc0) return rc0;
            have_view = 1;
        }
        if (v >= kRowTile8Base && !have_view8) {
            int rc0 = rt::build_t8_ws(ctx, ctx->stream, n, row_ptr, col, H, &view8, M);
            if (!rc0) rc0 = rt::build_t8z_ws(ctx, ctx->stream, &view8);
            if (rc0) return rc0;
            have_view8 = 1;
        }
        auto run = [&]() -> int {
            if (precision)
                return launch_spmm<float>(ctx, ctx->stream, v, n, row_ptr, col,
                                          HMPair<float>{(const float2 *)hm32}, (const float *)buf, m,
                                          (float *)(buf + (size_t)n * m * esz), (float *)(buf + 2 * (size_t)n * m * esz),
                                          m, m, nullptr, nullptr, &view, &view8);
            return launch_spmm<double>(ctx, ctx->stream, v, n, row_ptr, col, HMPair<double>{H, M},
                                       (const double *)buf, m, (double *)(buf + (size_t)n * m * esz),
                                       (double *)(buf + 2 * (size_t)n * m * esz), m, m, nullptr, nullptr, &view);
        };
        int rc = run();
        if (rc) return rc;
        FF_HIP(ctx, hipEventRecord(e0, ctx->stream));
        const int reps = 5;
        for (int r = 0; r < reps; ++r)
            if ((rc = run())) return rc;
        FF_HIP(ctx, hipEventRecord(e1, ctx->stream));
        FF_HIP(ctx, hipEventSynchronize(e1));
        float ms = 0.f;
        FF_HIP(ctx, hipEventElapsedTime(&ms, e0, e1));
        const double per = ms / reps;
        if (ctx->verbose) fprintf(stderr, "[freeform] autotune %s: %.3f ms\n", kVariantNames[v], per);
        if (per < bms) {
            bms = per;
            best = v;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    ctx->tuned[key] = best;
    *best_variant = best;
    *best_ms = bms;
    if (cache_path) {
        std::vector<std::string> keep;
        if (FILE *f = fopen(cache_path, "r")) {
            char line[512];
            while (fgets(line, sizeof(line), f)) {
                char k2[256];
                int v;
                double ms;
                if (sscanf(line, " \"%255[^\"]\": {\"variant\": %d, \"ms\": %lf", k2, &v, &ms) == 3 && key != k2)
                    keep.push_back(line);
            }
            fclose(f);
        }
        if (FILE *f = fopen(cache_path, "w")) {
            fprintf(f, "{\n");
            for (auto &l : keep) {
                std::string t = l;
                while (!t.empty() && (t.back() == '\n' || t.back() == ',' || t.back() == ' ')) t.pop_back();
                fprintf(f, "%s,\n", t.c_str());
            }
            fprintf(f, "  \"%s\": {\"variant\": %d, \"ms\": %.6f, \"name\": \"%s\"}\n}\n", key.c_str(), best, bms,
                    kVariantNames[best]);
            fclose(f);
        }
    }
    return FF_OK;
}

extern "C" int rand_block(ff_ctx *ctx, int64_t n, int m, uint64_t seed, double *out) {
    if (!ctx) return FF_ERR_INVALID_ARG;
    FF_REQUIRE(ctx, n > 0 && m > 0 && out, "bad arguments");
    FF_HIP(ctx, hipSetDevice(ctx->device));
    const int64_t count = n * (int64_t)m;
    hipLaunchKernelGGL(philox_block_kernel, dim3(grid_for((count + 3) / 4, 256)), dim3(256), 0, ctx->stream, count,
                       seed, out);
    FF_CHECK_LAUNCH(ctx);
    return FF_OK;
}

extern "C" int philox4x32_10(ff_ctx *ctx, int count, const uint32_t *ctr, const uint32_t *key, uint32_t *out) {
    if (!ctx) return FF_ERR_INVALID_ARG;
    FF_REQUIRE(ctx, count > 0 && ctr && key && out, "bad arguments");
    FF_HIP(ctx, hipSetDevice(ctx->device));
    hipLaunchKernelGGL(philox_raw_kernel, dim3(grid_for(count, 64)), dim3(64), 0, ctx->stream, ctr, key, out, count);
    FF_CHECK_LAUNCH(ctx);
    return FF_OK;
}

extern "C" int gram_hm(ff_ctx *ctx, int64_t n, int w, int precision, const void *S, const void *HS, const void *MS,
                       int64_t ld, double *G) {
    if (!ctx) return FF_ERR_INVALID_ARG;
    FF_REQUIRE(ctx, n > 0 && w > 0 && w <= 192 && ld >= w && S && HS && MS && G, "bad arguments");
    FF_REQUIRE(ctx, precision == 0 || precision == 1, "precision must be 0 or 1");
    FF_HIP(ctx, hipSetDevice(ctx->device));
    hipStream_t st = ctx->stream;
    std::vector<GChunk> g;
    for (int64_t r = 0; r < n; r += 2048) g.push_back(GChunk{r, (int32_t)std::min<int64_t>(2048, n - r), 0});
    const int ng = (int)g.size();
    GChunk *gch = (GChunk *)ws_get(ctx, WS_GCHUNKS, g.size() * sizeof(GChunk));
    int *ints = (int *)ws_get(ctx, WS_OBJ, 256);
    double *part = (double *)ws_get(ctx, WS_GPART, (size_t)ng * 2 * w * w * sizeof(double));
    if (!gch || !ints || !part) return FF_ERR_OOM;
    int hi[4] = {0, w, 0, ng};   // status, width, gfirst, gcount
    FF_HIP(ctx, hipMemcpyAsync(gch, g.data(), g.size() * sizeof(GChunk), hipMemcpyHostToDevice, st));
    FF_HIP(ctx, hipMemcpyAsync(ints, hi, sizeof(hi), hipMemcpyHostToDevice, st));
    FF_HIP(ctx, hipStreamSynchronize(st));
    const int T16 = (w + 15) / 16, nsup = (T16 + 5) / 6;
    int rc = gram_prepare(ctx);
    if (rc) return rc;
    // 16-byte row loads need 16-byte aligned bases and a leading dimension of whole vectors
    const int vn = precision ? 4 : 2;
    const int vec_ok = ld % vn == 0 && ((uintptr_t)S | (uintptr_t)HS | (uintptr_t)MS) % 16 == 0;
    if (precision)
        hipLaunchKernelGGL((gram_kernel<float, float>), dim3(ng, nsup * nsup), dim3(512), gram_shmem_bytes<float>(), st,
                           gch, ints, ints + 1, (const float *)S, (const float *)HS, (const float *)MS, ld, w, part,
                           vec_ok);
    else
        hipLaunchKernelGGL((gram_kernel<double, double>), dim3(ng, nsup * nsup), dim3(512),
                           gram_shmem_bytes<double>(), st, gch, ints, ints + 1, (const double *)S, (const double *)HS,
                           (const double *)MS, ld, w, part, vec_ok);
    FF_CHECK_LAUNCH(ctx);
    const int64_t per2 = 2 * (int64_t)w * w;
    hipLaunchKernelGGL(gram_reduce_kernel, dim3(grid_for(per2, 16), 1), dim3(256), 0, st, ints, ints + 1, ints + 2,
                       ints + 3, part, w, G);
    FF_CHECK_LAUNCH(ctx);
    FF_HIP(ctx, hipStreamSynchronize(st));
    return FF_OK;
}

namespace ff {
namespace lob {

// Device memory of rayleigh_ritz_noalloc, one copy per GPU for the life of the process: the
// Rayleigh-Ritz work arrays of the largest pencil it takes (order 192, 64 pairs), the three
// coefficient blocks C_w, C_p, C_pw and the status words (1.6 MB). Host code reaches it only
// through the address hipGetSymbolAddress gives for the current device.
constexpr int kNaW = 192, kNaM = 64, kNaDevices = 64;
constexpr size_t kNaRR = rr_scratch_doubles(kNaW, kNaM);
constexpr size_t kNaC = (size_t)3 * kNaW * kNaM;
constexpr size_t kNaDoubles = kNaRR + kNaC + 8;
static __device__ __align__(256) double scratch[kNaDoubles];
static std::mutex na_mu;
static double *na_ptr[kNaDevices] = {};

__global__ void rr_status_init_kernel(int *ints, int w) {
    if (threadIdx.x == 0) {
        ints[0] = 0;      // status: active
        ints[1] = w;      // width
        ints[2] = 0;      // info
    }
}

int noalloc_setup(ff_ctx *ctx) {
    std::lock_guard<std::mutex> lock(na_mu);
    if (ctx->device >= kNaDevices) return FF_OK;      // rayleigh_ritz_noalloc then reports it
    if (na_ptr[ctx->device]) return FF_OK;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
        (void)hipGetLastError();
        return set_error(ctx, FF_ERR_HIP, "hipGetSymbolAddress of the fixed scratch failed on device %d: %s",
                         ctx->device, hipGetErrorString(e));
    }
    na_ptr[ctx->device] = (double *)p;
    return FF_OK;
}

}  // namespace lob
}  // namespace ff

extern "C" int rayleigh_ritz_noalloc(ff_ctx *ctx, int w, int m, const double *G, double tau, double *C,
                                     double *theta, int *kept) {
    if (!ctx) return FF_ERR_INVALID_ARG;
    FF_REQUIRE(ctx, G && C && theta && kept, "required pointer is NULL");
    FF_REQUIRE(ctx, w > 0 && m > 0 && m <= w, "bad order %d or pair count %d", w, m);
    FF_REQUIRE(ctx, w <= kNaW && m <= kNaM,
               "order %d / %d pairs exceed the fixed scratch of rayleigh_ritz_noalloc (order <= %d, pairs <= %d)", w, m,
               kNaW, kNaM);
    double *base = nullptr;
    {
        std::lock_guard<std::mutex> lock(na_mu);
        base = ctx->device < kNaDevices ? na_ptr[ctx->device] : nullptr;
    }
    FF_REQUIRE(ctx, base != nullptr, "no fixed scratch on device %d", ctx->device);
    FF_HIP(ctx, hipSetDevice(ctx->device));
    hipStream_t st = ctx->stream;
    double *scr = base, *cw = base + kNaRR;
    int *ints = (int *)(base + kNaRR + kNaC);
    // the status words start fresh on every call; the work arrays are written before they are read
    hipLaunchKernelGGL(rr_status_init_kernel, dim3(1), dim3(64), 0, st, ints, w);
    FF_CHECK_LAUNCH(ctx);
    int rc = rr_prepare(ctx, w);
    if (!rc) rc = launch_rr<double>(ctx, st, 1, ints, ints + 1, G, w, m, tau, scr, C, cw, cw + (size_t)w * m,
                                    cw + (size_t)2 * w * m, theta, ints + 2);
    if (rc) return rc;
    int h[3];
    FF_HIP(ctx, hipMemcpyAsync(h, ints, sizeof(h), hipMemcpyDeviceToHost, st));
    FF_HIP(ctx, hipStreamSynchronize(st));
    *kept = h[2] & 0xffff;
    if (h[0] == 3) return set_error(ctx, FF_ERR_BREAKDOWN, "only %d of %d columns kept (need %d)", *kept, w, m);
    return FF_OK;
}

extern "C" int rayleigh_ritz(ff_ctx *ctx, int w, int m, const double *G, double tau, double *C, double *theta,
                             int *kept) {
    if (!ctx) return FF_ERR_INVALID_ARG;
    FF_REQUIRE(ctx, w > 0 && w <= 192 && m > 0 && m <= w && m <= 128 && G && C && theta && kept, "bad arguments");
    FF_HIP(ctx, hipSetDevice(ctx->device));
    hipStream_t st = ctx->stream;
    int *ints = (int *)ws_get(ctx, WS_OBJ, 256);
    double *scr = (double *)ws_get(ctx, WS_RRSCR, rr_scratch_doubles(w, m) * sizeof(double));
    double *cw = (double *)ws_get(ctx, WS_C, (size_t)w * m * sizeof(double) * 3);
    if (!ints || !scr || !cw) return FF_ERR_OOM;
    int hi[3] = {0, w, 0};   // status, width, info
    FF_HIP(ctx, hipMemcpyAsync(ints, hi, sizeof(hi), hipMemcpyHostToDevice, st));
    FF_HIP(ctx, hipStreamSynchronize(st));
    int rc = rr_prepare(ctx, w);
    if (!rc) rc = launch_rr<double>(ctx, st, 1, ints, ints + 1, G, w, m, tau, scr, C, cw, cw + (size_t)w * m,
                                    cw + (size_t)2 * w * m, theta, ints + 2);
    if (rc) return rc;
    int h[3];
    FF_HIP(ctx, hipMemcpyAsync(h, ints, sizeof(h), hipMemcpyDeviceToHost, st));
    FF_HIP(ctx, hipStreamSynchronize(st));
    *kept = h[2] & 0xffff;
    if (h[0] == 3) return set_error(ctx, FF_ERR_BREAKDOWN, "only %d of %d columns kept (need %d)", *kept, w, m);
    return FF_OK;
}

#ifdef FF_RR_TIMING
extern "C" int rr_phase_clock(unsigned long long *out16) {
    return hipMemcpyFromSymbol(out16, HIP_SYMBOL(ff::lob::rr_clock), 16 * sizeof(unsigned long long)) == hipSuccess ? 0 : -3;
}
#endif
