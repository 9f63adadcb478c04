// Atomic-free CSR assembly of the weight-space Hessian (Prop. 1) and the RKPM
// mass matrix (Eq. (14)) on gfx950.
//
//   H_kl = sum_i v_i (lambda_i + 4 mu_i) grad phi_k(X_i) . grad phi_l(X_i)
//   M_kl = sum_i v_i [rho_i] phi_k(X_i) phi_l(X_i)
//
// Row k is owned by one wavefront. Its columns are the union of N(i) over the
// quadrature points i with k in N(i). Every such column lies in the 5x5x5
// block of cells around k's cell (k and l are both within one cell of i's
// cell by construction of the lists), i.e. in at most 25 runs of consecutive
// sorted node ids. The wave marks columns in an LDS bitmap over those runs;
// the rank of a bit (prefix popcount) is the entry's slot in the row, so
// columns come out ascending. Values are accumulated in LDS while the wave
// walks i in ascending order, so every entry is the same ordered sum on every
// run, and H_kl and H_lk are the same sum (bitwise symmetry).
//
// Compiled with -ffp-contract=off so each term is rounded exactly as written.
#include "ff_internal.h"

namespace ff {
namespace {

constexpr int kWinMax = 16384;                 // candidate nodes per row window
constexpr int kWinWords = kWinMax / 32;
constexpr size_t kBitmapBytes = (size_t)8 << 30;  // largest store of the symbolic pass's row bitmaps
constexpr int kLdsPerCu = 160 * 1024;
constexpr int kRowMax = 2048;                  // entries per row

struct GridI {
    int64_t d[3];
    int64_t ncell;
};

struct Win {
    int64_t start[25];
    int32_t base[26];
    int32_t nr;
    int32_t pad;
    // the same runs indexed by their (z, y) offset in the 5 x 5 window, (dz + 2) * 5 + (dy + 2):
    // a node's slot follows from its cell's (z, y) without a search
    int64_t s25[25];
    int32_t b25[25];
    int32_t cz, cy;
};

__device__ inline int wave_incl_scan_i32(int v) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        int t = __shfl_up(v, d, 64);
        if (lane >= d) v += t;
    }
    return v;
}

__device__ inline int wave_sum_i32(int v) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
    return v;
}

// Runs of candidate columns for row k; returns the window size (sum of run lengths).
__device__ int64_t build_window(int64_t k, const int64_t *cs, GridI g, Win *win) {
    const int lane = threadIdx.x & 63;
    // last cell c with cs[c] <= k, by a 64-way search (cs is non-decreasing and cs[0] = 0 <= k)
    int64_t lo = 0, hi = g.ncell - 1;
    while (hi - lo >= 64) {
        const int64_t step = (hi - lo + 64) / 64;
        const int64_t probe = lo + lane * step;
        const uint64_t ok = __ballot(probe <= hi && cs[probe] <= k);
        const int last = 63 - __clzll(ok);
        lo += last * step;
        hi = lo + step - 1 < hi ? lo + step - 1 : hi;
    }
    const uint64_t okf = __ballot(lo + lane <= hi && cs[lo + lane] <= k);
    const int64_t c = lo + (63 - __clzll(okf));
    const int64_t cx = c % g.d[0], cy = (c / g.d[0]) % g.d[1], cz = c / (g.d[0] * g.d[1]);
    int64_t start = 0, len = 0;
    if (lane < 25) {
        const int64_t z = cz + lane / 5 - 2, y = cy + lane % 5 - 2;
        if (z >= 0 && z < g.d[2] && y >= 0 && y < g.d[1]) {
            const int64_t x0 = cx >= 2 ? cx - 2 : 0;
            const int64_t x1 = cx + 2 < g.d[0] ? cx + 2 : g.d[0] - 1;
            const int64_t row = (z * g.d[1] + y) * g.d[0];
            start = cs[row + x0];
            len = cs[row + x1 + 1] - start;
        }
    }
    const int64_t lenc = len > (int64_t)kWinMax ? (int64_t)kWinMax + 1 : len;   // keep the scan in int range
    const int incl = wave_incl_scan_i32((int)lenc);
    if (lane < 25) {
        win->s25[lane] = start;
        win->b25[lane] = incl - (int)lenc;
    }
    if (lane == 0) {
        win->cz = (int32_t)cz;
        win->cy = (int32_t)cy;
    }
    const uint64_t mask = __ballot(len > 0);
    const uint64_t below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    if (len > 0) {
        const int pos = __popcll(mask & below);
        win->start[pos] = start;
        win->base[pos] = incl - (int)lenc;
    }
    const int total = __shfl(incl, 63, 64);
    if (lane == 0) {
        const int nr = __popcll(mask);
        win->nr = nr;
        win->base[nr] = total;
    }
    __builtin_amdgcn_wave_barrier();
    return total;
}

// slot of node l in the window, zy = (z << 16) | y of l's cell; -1 outside the 5 x 5 runs
__device__ inline int local_of_zy(int64_t l, uint32_t zy, const Win *w) {
    const int dz = (int)(zy >> 16) - w->cz + 2, dy = (int)(zy & 0xffffu) - w->cy + 2;
    if ((unsigned)dz > 4u || (unsigned)dy > 4u) return -1;
    const int run = dz * 5 + dy;
    return w->b25[run] + (int)(l - w->s25[run]);
}

__device__ inline int64_t global_of(int x, const Win *w) {
    int lo = 0, hi = w->nr - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (w->base[mid] <= x) lo = mid; else hi = mid - 1;
    }
    return w->start[lo] + (int64_t)(x - w->base[lo]);
}

// mark the columns of row k in the bitmap. The row's transpose entries (i, and
// the range of N(i)) are read by the lanes in one pass; the neighbour ids of
// entry j + 1 are requested before entry j is marked.
__device__ inline void mark_row(int64_t k, const int64_t *nt_off, const int2 *nt, const int64_t *off,
                                const int32_t *ids, const uint32_t *zys, const Win *win, uint32_t *bm, int nwords) {
    const int lane = threadIdx.x & 63;
    for (int w = lane; w < nwords; w += 64) bm[w] = 0u;
    __builtin_amdgcn_wave_barrier();
    const int64_t a = nt_off[k], b = nt_off[k + 1];
    const int wend = win->base[win->nr];
    for (int64_t e0 = a; e0 < b; e0 += 64) {
        const int cnt = (int)(b - e0 < 64 ? b - e0 : 64);
        int64_t f0 = 0, f1 = 0;
        if (lane < cnt) {
            const int64_t i = nt[e0 + lane].x;
            f0 = off[i];
            f1 = off[i + 1];
        }
        int32_t idA = -1, idB = -1;
        uint32_t zA = 0, zB = 0;
        {
            const int64_t s0 = __shfl(f0, 0, 64), s1 = __shfl(f1, 0, 64);
            if (s0 + lane < s1) {
                idA = ids[s0 + lane];
                zA = zys[s0 + lane];
            }
        }
        for (int j = 0; j < cnt; j += 2) {
            int64_t s0, s1;
            if (j + 1 < cnt) {
                s0 = __shfl(f0, j + 1, 64);
                s1 = __shfl(f1, j + 1, 64);
                idB = s0 + lane < s1 ? ids[s0 + lane] : -1;
                zB = s0 + lane < s1 ? zys[s0 + lane] : 0u;
            }
            s0 = __shfl(f0, j, 64);
            s1 = __shfl(f1, j, 64);
            for (int64_t f = s0 + lane; f < s1; f += 64) {
                const bool first = f == s0 + lane;
                const int32_t id = first ? idA : ids[f];
                const int x = local_of_zy(id, first ? zA : zys[f], win);
                if (x >= 0 && x < wend) atomicOr(&bm[x >> 5], 1u << (x & 31));
            }
            if (j + 1 >= cnt) break;
            if (j + 2 < cnt) {
                const int64_t t0 = __shfl(f0, j + 2, 64), t1 = __shfl(f1, j + 2, 64);
                idA = t0 + lane < t1 ? ids[t0 + lane] : -1;
                zA = t0 + lane < t1 ? zys[t0 + lane] : 0u;
            }
            s0 = __shfl(f0, j + 1, 64);
            s1 = __shfl(f1, j + 1, 64);
            for (int64_t f = s0 + lane; f < s1; f += 64) {
                const bool first = f == s0 + lane;
                const int32_t id = first ? idB : ids[f];
                const int x = local_of_zy(id, first ? zB : zys[f], win);
                if (x >= 0 && x < wend) atomicOr(&bm[x >> 5], 1u << (x & 31));
            }
        }
    }
    __builtin_amdgcn_wave_barrier();
}

// (z << 16) | y of each node's cell, then of each neighbour entry (aligned with the ids)
__global__ void node_zy_kernel(int64_t ncell, const int64_t *cs, GridI g, uint32_t *zy) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncell) return;
    const uint32_t v = (uint32_t)((c / ((int64_t)g.d[0] * g.d[1])) << 16) | (uint32_t)((c / g.d[0]) % g.d[1]);
    for (int64_t j = cs[c]; j < cs[c + 1]; ++j) zy[j] = v;
}

__global__ void entry_zy_kernel(int64_t total, const int32_t *ids, const uint32_t *node_zy, uint32_t *zy) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < total) zy[e] = node_zy[ids[e]];
}

// ---------------------------------------------------------------------------
// transpose of the neighbour relation: NT(k) = {(i, slot) : N(i)[slot] = k}, i ascending
// ---------------------------------------------------------------------------

__global__ void __launch_bounds__(256) nt_count_kernel(const int32_t *ids, int64_t total, int32_t *cnt) {
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < total) atomicAdd(&cnt[ids[e]], 1);
}

__global__ void __launch_bounds__(256) nt_fill_kernel(const int64_t *off, const int32_t *ids, int64_t q,
                                                      const int64_t *nt_off, int32_t *cursor, int2 *nt) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= q) return;
    const int64_t a = off[i], b = off[i + 1];
    for (int64_t e = a; e < b; ++e) {
        const int32_t k = ids[e];
        const int64_t pos = nt_off[k] + atomicAdd(&cursor[k], 1);
        nt[pos] = make_int2((int)i, (int)(e - a));
    }
}

// NT(k) in ascending i (the i are distinct within a list): one wavefront per
// node copies its list to LDS and writes each entry at its rank; lists longer
// than kSortMax are left to nt_sort_long_kernel.
constexpr int kSortMax = 1024;
__global__ void __launch_bounds__(256) nt_sort_kernel(const int64_t *nt_off, int64_t n, int2 *nt,
                                                      unsigned long long *empty_node) {
    __shared__ int2 buf[4][kSortMax];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t k = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    if (k >= n) return;
    const int64_t a = nt_off[k], b = nt_off[k + 1];
    const int64_t cnt = b - a;
    if (cnt == 0) {
        if (lane == 0) atomicMin(empty_node, (unsigned long long)k);
        return;
    }
    if (cnt > kSortMax) return;
    int2 *bw = buf[wv];
    for (int t = lane; t < cnt; t += 64) bw[t] = nt[a + t];
    __builtin_amdgcn_wave_barrier();
    for (int t = lane; t < cnt; t += 64) {
        const int2 v = bw[t];
        int r = 0;
        for (int u = 0; u < cnt; ++u) r += bw[u].x < v.x;
        nt[a + r] = v;
    }
}

// The lists longer than kSortMax (many quadrature points per node, as with grid integration
// points): one workgroup per node marks its entries' i in an LDS bitmap over the list's range of
// i, and the prefix popcount of the bitmap gives each entry's rank; the sorted list goes to a
// scratch range, then back. A range wider than kLongBits falls back to an insertion sort by one
// thread. Workgroups stride over the nodes.
constexpr int kLongBits = 1 << 17;
constexpr int kLongWords = kLongBits / 32;
__global__ void __launch_bounds__(256) nt_sort_long_kernel(const int64_t *nt_off, int64_t n, int2 *nt, int2 *tmp) {
    __shared__ uint32_t bm[kLongWords];
    __shared__ int32_t pre[kLongWords];
    __shared__ int32_t part[256];
    __shared__ int32_t lo_s, hi_s;
    const int t = threadIdx.x;
    for (int64_t k = blockIdx.x; k < n; k += gridDim.x) {
        const int64_t a = nt_off[k], b = nt_off[k + 1];
        const int64_t cnt = b - a;
        if (cnt <= kSortMax) continue;                 // uniform across the workgroup
        if (t == 0) {
            lo_s = INT32_MAX;
            hi_s = -1;
        }
        __syncthreads();
        int lo = INT32_MAX, hi = -1;
        for (int64_t j = a + t; j < b; j += 256) {
            const int i = nt[j].x;
            lo = i < lo ? i : lo;
            hi = i > hi ? i : hi;
        }
        atomicMin(&lo_s, lo);
        atomicMax(&hi_s, hi);
        __syncthreads();
        const int base = lo_s;
        const int64_t range = (int64_t)hi_s - base + 1;
        if (range > kLongBits) {
            if (t == 0)
                for (int64_t j = a + 1; j < b; ++j) {
                    const int2 v = nt[j];
                    int64_t u = j - 1;
                    while (u >= a && nt[u].x > v.x) {
                        nt[u + 1] = nt[u];
                        --u;
                    }
                    nt[u + 1] = v;
                }
            __syncthreads();
            continue;
        }
        const int nw = (int)((range + 31) >> 5);
        for (int w = t; w < nw; w += 256) bm[w] = 0u;
        __syncthreads();
        for (int64_t j = a + t; j < b; j += 256) {
            const int x = nt[j].x - base;
            atomicOr(&bm[x >> 5], 1u << (x & 31));
        }
        __syncthreads();
        // exclusive prefix of popcounts: each thread a contiguous run of words, then the runs
        const int per = (nw + 255) / 256, w0 = t * per, w1 = w0 + per < nw ? w0 + per : nw;
        int sum = 0;
        for (int w = w0; w < w1; ++w) sum += __popc(bm[w]);
        part[t] = sum;
        __syncthreads();
        for (int d = 1; d < 256; d <<= 1) {
            const int v = t >= d ? part[t - d] : 0;
            __syncthreads();
            part[t] += v;
            __syncthreads();
        }
        int run = part[t] - sum;
        for (int w = w0; w < w1; ++w) {
            pre[w] = run;
            run += __popc(bm[w]);
        }
        __syncthreads();
        for (int64_t j = a + t; j < b; j += 256) {
            const int2 v = nt[j];
            const int x = v.x - base;
            const int r = pre[x >> 5] + __popc(bm[x >> 5] & ((1u << (x & 31)) - 1u));
            tmp[a + r] = v;
        }
        __syncthreads();
        for (int64_t j = a + t; j < b; j += 256) nt[j] = tmp[j];
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// symbolic pass: row lengths
// ---------------------------------------------------------------------------

__global__ void __launch_bounds__(256) sym_kernel(int64_t n, const int64_t *cs, GridI g, const int64_t *nt_off,
                                                  const int2 *nt, const int64_t *off, const int32_t *ids,
                                                  const uint32_t *zys, int32_t *rowlen, int *stats, uint32_t *bm_out) {
    __shared__ Win wins[4];
    __shared__ uint32_t bms[4][kWinWords];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t k = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    if (k >= n) return;
    Win *win = &wins[wv];
    uint32_t *bm = bms[wv];
    const int64_t W = build_window(k, cs, g, win);
    if (W > kWinMax) {
        if (lane == 0) {
            rowlen[k] = 0;
            atomicOr(&stats[0], 1);
        }
        return;
    }
    const int nwords = (int)((W + 31) >> 5);
    mark_row(k, nt_off, nt, off, ids, zys, win, bm, nwords);
    int c = 0;
    for (int w = lane; w < nwords; w += 64) c += __popc(bm[w]);
    if (bm_out)                                    // kept for the numeric pass (row stride kWinWords)
        for (int w = lane; w < nwords; w += 64) bm_out[k * kWinWords + w] = bm[w];
    // maxima over the rows: the atomic only when a plain read shows a smaller value (the maxima only
    // grow, so a stale read costs an atomic, never a missed update); a million contended atomics on
    // one address cost about as much as the pass itself
    if (lane == 0 && nwords > __hip_atomic_load(&stats[2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
        atomicMax(&stats[2], nwords);
    c = wave_sum_i32(c);
    if (lane == 0) {
        rowlen[k] = c;
        if (c > __hip_atomic_load(&stats[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) atomicMax(&stats[1], c);
    }
}

// ---------------------------------------------------------------------------
// numeric pass
// ---------------------------------------------------------------------------

__global__ void __launch_bounds__(256) num_kernel(int64_t n, const int64_t *cs, GridI g, const int64_t *nt_off,
                                                  const int2 *nt, const int64_t *off, const int32_t *ids,
                                                  const uint32_t *zys,
                                                  const double *phi, const double *dphi, const double *vol,
                                                  const double *lam, const double *mu, const double *rho,
                                                  const int32_t *perm, const int64_t *row_ptr, int32_t *col,
                                                  double *H, double *M, float *hm32, int rmax, int per_wave,
                                                  int wwords, const uint32_t *bm_in) {
    extern __shared__ __align__(16) char smem[];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t k = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    if (k >= n) return;
    char *base = smem + (size_t)wv * per_wave;
    double *aH = (double *)base;
    double *aM = aH + rmax;
    Win *win = (Win *)(aM + rmax);
    uint32_t *bm = (uint32_t *)(win + 1);
    int32_t *pre = (int32_t *)(bm + wwords);       // wwords: the largest row window, in bitmap words

    const int64_t W = build_window(k, cs, g, win);
    const int nwords = (int)((W + 31) >> 5);
    if (bm_in) {                                   // the symbolic pass's bitmap of this row
        for (int w = lane; w < nwords; w += 64) bm[w] = bm_in[k * kWinWords + w];
        __builtin_amdgcn_wave_barrier();
    } else {
        mark_row(k, nt_off, nt, off, ids, zys, win, bm, nwords);
    }

    // exclusive prefix of popcounts over the bitmap words
    int carry = 0;
    for (int wb = 0; wb < nwords; wb += 64) {
        const int w = wb + lane;
        const int c = w < nwords ? __popc(bm[w]) : 0;
        const int incl = wave_incl_scan_i32(c);
        if (w < nwords) pre[w] = carry + incl - c;
        carry += __shfl(incl, 63, 64);
    }
    const int len = carry;
    const int64_t rp = row_ptr[k];
    __builtin_amdgcn_wave_barrier();

    if (col) {
        for (int w = lane; w < nwords; w += 64) {
            uint32_t bits = bm[w];
            int r = pre[w];
            while (bits) {
                const int b = __ffs(bits) - 1;
                bits &= bits - 1u;
                col[rp + r] = (int32_t)global_of(w * 32 + b, win);
                ++r;
            }
        }
    }
    for (int t = lane; t < len; t += 64) {
        aH[t] = 0.0;
        aM[t] = 0.0;
    }
    __builtin_amdgcn_wave_barrier();

    // the row's transpose entries: i, the range of N(i), grad phi_k(X_i), phi_k(X_i) and the
    // weights, read by the lanes in one pass; entry j + 1's neighbour data is requested
    // before entry j is accumulated. Entries are accumulated in ascending i, each term as
    // written, so every entry is the same ordered sum on every run.
    const int64_t a = nt_off[k], b = nt_off[k + 1];
    const int wend = win->base[win->nr];
    for (int64_t e0 = a; e0 < b; e0 += 64) {
        const int cnt = (int)(b - e0 < 64 ? b - e0 : 64);
        int64_t f0 = 0, f1 = 0;
        double q0 = 0.0, q1 = 0.0, q2 = 0.0, qp = 0.0, qw = 0.0, qm = 0.0;
        if (lane < cnt) {
            const int2 ent = nt[e0 + lane];
            const int64_t i = ent.x;
            f0 = off[i];
            f1 = off[i + 1];
            const int64_t ek = f0 + ent.y;
            q0 = dphi[3 * ek];
            q1 = dphi[3 * ek + 1];
            q2 = dphi[3 * ek + 2];
            qp = phi[ek];
            const int64_t ii = perm ? (int64_t)perm[i] : i;
            qw = vol[ii] * (lam[ii] + 4.0 * mu[ii]);
            qm = rho ? vol[ii] * rho[ii] : vol[ii];
        }
        // first 128 neighbours of an entry, requested ahead without a branch: lanes past the end of
        // N(i) (never empty: it holds k) load its last neighbour, which accumulate() does not use; the
        // scheduling barriers keep the loads together and their first use in accumulate()
        struct Pre { int32_t id[2]; uint32_t zy[2]; double d0[2], d1[2], d2[2], p[2]; };
        auto fetch = [&](int j, Pre &P) __attribute__((always_inline)) {
            const int64_t s0 = __shfl(f0, j, 64), s1 = __shfl(f1, j, 64);
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int h = 0; h < 2; ++h) {                 // neighbours lane and 64 + lane
                const int64_t f = s0 + 64 * h + lane < s1 ? s0 + 64 * h + lane : s1 - 1;
                P.id[h] = ids[f];
                P.zy[h] = zys[f];
                P.d0[h] = dphi[3 * f];
                P.d1[h] = dphi[3 * f + 1];
                P.d2[h] = dphi[3 * f + 2];
                P.p[h] = phi[f];
            }
            __builtin_amdgcn_sched_barrier(0);
        };
        auto accumulate = [&](int j, const Pre &P) {
            const int64_t s0 = __shfl(f0, j, 64), s1 = __shfl(f1, j, 64);
            const double gk0 = __shfl(q0, j, 64), gk1 = __shfl(q1, j, 64), gk2 = __shfl(q2, j, 64);
            const double pk = __shfl(qp, j, 64), wi = __shfl(qw, j, 64), mi = __shfl(qm, j, 64);
            auto term = [&](int32_t id, uint32_t zy, double d0, double d1, double d2, double pf)
                            __attribute__((always_inline)) {
                const int x = local_of_zy(id, zy, win);
                if (x < 0 || x >= wend) return;
                const uint32_t word = bm[x >> 5];
                const int r = pre[x >> 5] + __popc(word & ((1u << (x & 31)) - 1u));
                const double dot = ((gk0 * d0) + (gk1 * d1)) + (gk2 * d2);
                aH[r] += wi * dot;
                aM[r] += mi * (pk * pf);
            };
#pragma unroll
            for (int h = 0; h < 2; ++h)                  // the first 128, requested ahead
                if (s0 + 64 * h + lane < s1) term(P.id[h], P.zy[h], P.d0[h], P.d1[h], P.d2[h], P.p[h]);
            for (int64_t f = s0 + 128 + lane; f < s1; f += 64)           // the rest of a longer N(i)
                term(ids[f], zys[f], dphi[3 * f], dphi[3 * f + 1], dphi[3 * f + 2], phi[f]);
            __builtin_amdgcn_wave_barrier();
        };
        // entry j + 1's neighbours are requested before entry j is accumulated (the last entry's
        // are requested again at the end rather than behind a branch)
        Pre PA, PB;
        fetch(0, PA);
        for (int j = 0; j < cnt; j += 2) {
            fetch(j + 1 < cnt ? j + 1 : cnt - 1, PB);
            accumulate(j, PA);
            if (j + 1 >= cnt) break;
            fetch(j + 2 < cnt ? j + 2 : cnt - 1, PA);
            accumulate(j + 1, PB);
        }
    }
    for (int t = lane; t < len; t += 64) {
        const double h = aH[t], m = aM[t];
        H[rp + t] = h;
        M[rp + t] = m;
        if (hm32) {
            hm32[2 * (rp + t)] = (float)h;
            hm32[2 * (rp + t) + 1] = (float)m;
        }
    }
}

}  // namespace

int build_transpose(ff_ctx *ctx, hipStream_t st, int64_t n, int64_t q, int64_t total, const int64_t *nbr_off,
                    const int32_t *nbr_id, int64_t *nt_off, int2 *nt, unsigned long long *empty_node) {
    int32_t *cnt = (int32_t *)ws_get(ctx, WS_COUNTS, (size_t)n * sizeof(int32_t));
    int32_t *cursor = (int32_t *)ws_get(ctx, WS_CURSOR, (size_t)n * sizeof(int32_t));
    int2 *tmp = (int2 *)ws_get(ctx, WS_NT_TMP, (size_t)(total > 0 ? total : 1) * sizeof(int2));
    unsigned long long *en = empty_node;
    if (!en) en = (unsigned long long *)ws_get(ctx, WS_FLAG, 64);
    if (!cnt || !cursor || !tmp || !en) return FF_ERR_OOM;
    FF_HIP(ctx, hipMemsetAsync(cnt, 0, (size_t)n * sizeof(int32_t), st));
    FF_HIP(ctx, hipMemsetAsync(cursor, 0, (size_t)n * sizeof(int32_t), st));
    FF_HIP(ctx, hipMemsetAsync(en, 0xff, 8, st));
    if (total > 0) {
        hipLaunchKernelGGL(nt_count_kernel, dim3(grid_for(total, 256)), dim3(256), 0, st, nbr_id, total, cnt);
        FF_CHECK_LAUNCH(ctx);
    }
    int rc = scan_exclusive_i32_to_i64(ctx, cnt, nt_off, n);
    if (rc) return rc;
    hipLaunchKernelGGL(nt_fill_kernel, dim3(grid_for(q, 256)), dim3(256), 0, st, nbr_off, nbr_id, q, nt_off, cursor,
                       nt);
    FF_CHECK_LAUNCH(ctx);
    hipLaunchKernelGGL(nt_sort_kernel, dim3(grid_for(n, 4)), dim3(256), 0, st, nt_off, n, nt, en);
    FF_CHECK_LAUNCH(ctx);
    // the long lists (grid integration points: thousands of points per node)
    hipLaunchKernelGGL(nt_sort_long_kernel, dim3((unsigned)std::min<int64_t>(n, 4096)), dim3(256), 0, st, nt_off, n,
                       nt, tmp);
    FF_CHECK_LAUNCH(ctx);
    return FF_OK;
}

}  // namespace ff

using namespace ff;

extern "C" int assemble_HM(ff_ctx *ctx, int64_t n, int64_t q, const int64_t *nbr_off, const int32_t *nbr_id,
                           const double *phi, const double *dphi, const double *vol, const double *lam,
                           const double *mu, const double *rho, const int32_t *perm, const ff_grid *grid,
                           const int64_t *cell_start, int64_t *row_ptr, int32_t *col, double *H, double *M,
                           float *hm32, int64_t nnz_cap, int64_t *nnz) {
    if (!ctx) return FF_ERR_INVALID_ARG;
    FF_REQUIRE(ctx, n > 0 && q > 0 && n < INT32_MAX && q < INT32_MAX, "bad sizes n=%lld q=%lld", (long long)n,
               (long long)q);
    FF_REQUIRE(ctx, nbr_off && nbr_id && phi && dphi && vol && lam && mu && grid && cell_start && row_ptr && nnz,
               "required pointer is NULL");
    FF_REQUIRE(ctx, (col == nullptr) == (H == nullptr) && (col == nullptr) == (M == nullptr),
               "col, H and M must be all given or all NULL");
    FF_REQUIRE(ctx, grid->n_cells == grid->dims[0] * grid->dims[1] * grid->dims[2] && grid->n_cells > 0,
               "inconsistent grid");
    FF_HIP(ctx, hipSetDevice(ctx->device));
    hipStream_t st = ctx->stream;

    int64_t total = 0;
    int64_t *host = (int64_t *)pinned_get(ctx, 4096);
    if (!host) return FF_ERR_OOM;
    GridI g;
    for (int a = 0; a < 3; ++a) g.d[a] = grid->dims[a];
    g.ncell = grid->n_cells;
    // the sizing call's symbolic state, when this call follows it on the same arrays
    const void *key_ptr[4] = {nbr_off, nbr_id, cell_start, row_ptr};
    const int64_t key_size[5] = {n, q, grid->dims[0], grid->dims[1], grid->dims[2]};
    bool reuse = col != nullptr && ctx->asm_valid;
    for (int i = 0; i < 4 && reuse; ++i) reuse = ctx->asm_ptr[i] == key_ptr[i];
    for (int i = 0; i < 5 && reuse; ++i) reuse = ctx->asm_size[i] == key_size[i];
    ctx->asm_valid = false;
    int64_t *nt_off = (int64_t *)ws_get(ctx, WS_NT_OFF, (size_t)(n + 1) * sizeof(int64_t));
    if (!nt_off) return FF_ERR_OOM;
    int2 *nt = nullptr;
    uint32_t *zys = nullptr;                       // (z << 16) | y of each neighbour entry's cell
    int rowmax = 0, wwords = 0;
    FF_REQUIRE(ctx, grid->dims[1] < 65536 && grid->dims[2] < 65536, "grid of %d x %d x %d cells too large",
               grid->dims[0], grid->dims[1], grid->dims[2]);
    // each row's column bitmap from the symbolic pass, so that the numeric pass need not mark it again
    // (kWinWords words per row; left out beyond kBitmapBytes, where the numeric pass marks it itself)
    uint32_t *bm = nullptr;
    if (reuse) {
        nt = (int2 *)ctx->ws[WS_NT];
        zys = (uint32_t *)ctx->ws[WS_ZYE];
        bm = ctx->asm_bm ? (uint32_t *)ctx->ws[WS_ASM_BM] : nullptr;
        *nnz = ctx->asm_nnz;
        rowmax = ctx->asm_rowmax;
        wwords = ctx->asm_wwords;
        if (nnz_cap < *nnz)
            return set_error(ctx, FF_ERR_CAPACITY, "CSR needs %lld entries, capacity %lld", (long long)*nnz,
                             (long long)nnz_cap);
    } else {
        FF_HIP(ctx, hipMemcpyAsync(host, nbr_off + q, sizeof(int64_t), hipMemcpyDeviceToHost, st));
        FF_HIP(ctx, hipStreamSynchronize(st));
        total = host[0];

        // transpose
        int32_t *cnt = (int32_t *)ws_get(ctx, WS_COUNTS, (size_t)n * sizeof(int32_t));
        int32_t *cursor = (int32_t *)ws_get(ctx, WS_CURSOR, (size_t)n * sizeof(int32_t));
        nt = (int2 *)ws_get(ctx, WS_NT, (size_t)(total > 0 ? total : 1) * sizeof(int2));
        uint32_t *node_zy = (uint32_t *)ws_get(ctx, WS_ZYN, (size_t)n * sizeof(uint32_t));
        zys = (uint32_t *)ws_get(ctx, WS_ZYE, (size_t)(total > 0 ? total : 1) * sizeof(uint32_t));
        if (!node_zy || !zys) return FF_ERR_OOM;
        hipLaunchKernelGGL(node_zy_kernel, dim3(grid_for(g.ncell, 256)), dim3(256), 0, st, (int64_t)g.ncell,
                           cell_start, g, node_zy);
        FF_CHECK_LAUNCH(ctx);
        if (total > 0) {
            hipLaunchKernelGGL(entry_zy_kernel, dim3(grid_for(total, 256)), dim3(256), 0, st, total, nbr_id, node_zy,
                               zys);
            FF_CHECK_LAUNCH(ctx);
        }
        int32_t *rowlen = (int32_t *)ws_get(ctx, WS_ROWLEN, (size_t)n * sizeof(int32_t));
        int *stats = (int *)ws_get(ctx, WS_ASM_FLAG, 64);
        if (!cnt || !cursor || !nt_off || !nt || !rowlen || !stats) return FF_ERR_OOM;
        unsigned long long *empty_node = (unsigned long long *)(stats + 4);
        FF_HIP(ctx, hipMemsetAsync(stats, 0, 16, st));
        int rc = build_transpose(ctx, st, n, q, total, nbr_off, nbr_id, nt_off, nt, empty_node);
        if (rc) return rc;

        const size_t bm_bytes = (size_t)n * kWinWords * sizeof(uint32_t);
        if (bm_bytes <= (ctx->asm_bm_cap >= 0 ? (size_t)ctx->asm_bm_cap : kBitmapBytes)) {
            bm = (uint32_t *)ws_get(ctx, WS_ASM_BM, bm_bytes);
            if (!bm) ctx->last_error.clear();          // without it the numeric pass marks the rows itself
        }
        hipLaunchKernelGGL(sym_kernel, dim3(grid_for(n, 4)), dim3(256), 0, st, n, cell_start, g, nt_off, nt, nbr_off,
                           nbr_id, zys, rowlen, stats, bm);
        FF_CHECK_LAUNCH(ctx);
        rc = scan_exclusive_i32_to_i64(ctx, rowlen, row_ptr, n);
        if (rc) return rc;
        FF_HIP(ctx, hipMemcpyAsync(host, row_ptr + n, sizeof(int64_t), hipMemcpyDeviceToHost, st));
        FF_HIP(ctx, hipMemcpyAsync(host + 1, stats, 16, hipMemcpyDeviceToHost, st));
        FF_HIP(ctx, hipMemcpyAsync(host + 3, empty_node, 8, hipMemcpyDeviceToHost, st));
        FF_HIP(ctx, hipStreamSynchronize(st));
        const int *hs = (const int *)(host + 1);
        const unsigned long long en = (unsigned long long)host[3];
        if (en != ~0ull)
            return set_error(ctx, FF_ERR_INVALID_ARG, "node %llu has no quadrature point in its support", en);
        FF_REQUIRE(ctx, hs[0] == 0, "a row's candidate window exceeds %d nodes; decrease h", kWinMax);
        FF_REQUIRE(ctx, hs[1] <= kRowMax, "a row has %d entries (limit %d); decrease h", hs[1], kRowMax);
        *nnz = host[0];
        rowmax = hs[1];
        wwords = hs[2];
        if (!col) {
            ctx->asm_valid = true;
            for (int i = 0; i < 4; ++i) ctx->asm_ptr[i] = key_ptr[i];
            for (int i = 0; i < 5; ++i) ctx->asm_size[i] = key_size[i];
            ctx->asm_nnz = host[0];
            ctx->asm_rowmax = rowmax;
            ctx->asm_wwords = wwords;
            ctx->asm_bm = bm != nullptr;
            return FF_OK;
        }
        if (nnz_cap < host[0])
            return set_error(ctx, FF_ERR_CAPACITY, "CSR needs %lld entries, capacity %lld", (long long)host[0],
                             (long long)nnz_cap);
    }

    const int rmax = ((rowmax + 63) / 64) * 64;
    // LDS per wave: the row's FP64 accumulators, the window, its bitmap and prefix sized to the largest
    // window; waves per workgroup (4, 2 or 1, at most 64 KiB) for the most waves per CU
    const int per_wave = (int)(((size_t)2 * rmax * sizeof(double) + sizeof(Win) + (size_t)wwords * 8 + 255) & ~255);
    int waves = 1, best = 0;
    for (int w = 4; w >= 1; w >>= 1) {
        if (w * per_wave > 64 * 1024) continue;
        const int per_cu = w * std::min(kLdsPerCu / (w * per_wave), 32 / w);
        if (per_cu > best) best = per_cu, waves = w;
    }
    const size_t shmem = (size_t)waves * per_wave;
    hipLaunchKernelGGL(num_kernel, dim3(grid_for(n, waves)), dim3(64 * waves), shmem, st, n, cell_start, g, nt_off,
                       nt, nbr_off, nbr_id, zys, phi, dphi, vol, lam, mu, rho, perm, row_ptr, col, H, M, hm32,
                       rmax, per_wave, wwords, bm);
    FF_CHECK_LAUNCH(ctx);
    return FF_OK;
}
