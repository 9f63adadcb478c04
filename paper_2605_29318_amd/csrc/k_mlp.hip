// Learned warm start for the eigensolver: an n_in -> 128 -> 128 -> 128 -> k MLP
// with GELU (exact erf form), BF16 weights and activations, FP32 accumulation,
// trained on modes the eigensolver computes, with the subspace loss
//   L = k - tr(A^-1 B E B^T),  A = Y^T D Y,  B = Y^T D T,  E = (T^T D T)^-1
// (D = lumped mass diag(M 1), T = target modes), which is invariant to any
// mixing of the columns of Y or T, and Adam. Not part of the paper.
//
// Parameters are flat FP32 (the master copy) in the order
// [W1 (128 x n_in), b1, W2 (128x128), b2, W3 (128x128), b3, W4 (k x 128), b4],
// each W output-major; a BF16 copy feeds the kernels. The inputs are 11 base
// values per point plus 6 per octave of sine/cosine position encoding.
#include "ff_internal.h"

#include <random>

extern "C" int gram_hm(ff_ctx *ctx, int64_t n, int w, int precision, const void *S, const void *HS, const void *MS,
                       int64_t ld, double *G);

struct ff_mlp {
    ff_ctx *ctx = nullptr;
    int device = 0;
    hipStream_t stream = nullptr;   // the context's stream, kept for destruction
    int k = 0;
    int n_in = 0;
    int P = 0;
    float *p32 = nullptr, *m = nullptr, *v = nullptr, *g = nullptr;
    uint16_t *pb = nullptr;
    int t = 0;
    int64_t cap = 0;
    float *Z[3] = {nullptr, nullptr, nullptr};
    uint16_t *A[3] = {nullptr, nullptr, nullptr};
    float *Y = nullptr, *dY = nullptr, *dZa = nullptr, *dZb = nullptr, *DY = nullptr, *Tf = nullptr, *DT = nullptr;
    float *gpart = nullptr;
    double *small = nullptr;   // Grams and k x k results
};

namespace ff {
namespace mlpk {

constexpr int kH = 128;
constexpr int kBase = 11;          // base inputs per point
constexpr int kMaxFreq = 19;       // 11 + 6 * 19 = 125 <= kH
constexpr int kRowsPerBlock = 32;
constexpr int kWgBlocks = 128;     // blocks that accumulate weight-gradient partials

struct Layout {
    int off_w[4], off_b[4], nin[4], nout[4];
    int total;
};

inline Layout layout(int k, int n_in) {
    Layout L;
    const int nin[4] = {n_in, kH, kH, kH}, nout[4] = {kH, kH, kH, k};
    int o = 0;
    for (int l = 0; l < 4; ++l) {
        L.nin[l] = nin[l];
        L.nout[l] = nout[l];
        L.off_w[l] = o;
        o += nin[l] * nout[l];
        L.off_b[l] = o;
        o += nout[l];
    }
    L.total = o;
    return L;
}

__host__ __device__ inline float bf16_to_f(uint16_t b) {
    union { uint32_t u; float f; } c;
    c.u = (uint32_t)b << 16;
    return c.f;
}

__host__ __device__ inline uint16_t f_to_bf16(float f) {
    union { uint32_t u; float f; } c;
    c.f = f;
    if ((c.u & 0x7f800000u) == 0x7f800000u) return (uint16_t)(c.u >> 16);     // inf / nan
    const uint32_t r = c.u + 0x7fffu + ((c.u >> 16) & 1u);                    // round to nearest even
    return (uint16_t)(r >> 16);
}

__device__ inline float gelu(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }
__device__ inline float gelu_grad(float z) {
    return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) + z * 0.39894228040143268f * expf(-0.5f * z * z);
}

template <typename Tin> __device__ inline float load_in(const Tin *p);
template <> __device__ inline float load_in<float>(const float *p) { return *p; }
template <> __device__ inline float load_in<uint16_t>(const uint16_t *p) { return bf16_to_f(*p); }

// Z = In W^T + b for 32 rows per block; hidden layers store Z (FP32) and GELU(Z) (BF16),
// the output layer stores Y (FP32) and optionally a FP64 copy with leading dimension ldy.
template <typename Tin>
__global__ void __launch_bounds__(256) dense_fwd_kernel(int64_t n, const Tin *in, int nin, const uint16_t *W,
                                                        const float *b, int nout, int act, float *Z, uint16_t *Aout,
                                                        float *Yout, double *Ydbl, int64_t ldy) {
    __shared__ float xs[kRowsPerBlock][kH];
    __shared__ uint16_t ws[kH * kH];                    // transposed: ws[i * nout + o]
    const int64_t r0 = (int64_t)blockIdx.x * kRowsPerBlock;
    for (int idx = threadIdx.x; idx < kRowsPerBlock * nin; idx += 256) {
        const int r = idx / nin, i = idx - (idx / nin) * nin;
        xs[r][i] = (r0 + r < n) ? load_in<Tin>(in + (r0 + r) * nin + i) : 0.0f;
    }
    for (int idx = threadIdx.x; idx < nout * nin; idx += 256) {
        const int o = idx / nin, i = idx - (idx / nin) * nin;
        ws[i * nout + o] = W[idx];
    }
    __syncthreads();
    const int groups = 256 / nout;                       // row groups
    const int o = threadIdx.x % nout, grp = threadIdx.x / nout;
    if (grp >= groups) return;
    const int rows = (kRowsPerBlock + groups - 1) / groups;
    float acc[kRowsPerBlock];
#pragma unroll
    for (int q = 0; q < kRowsPerBlock; ++q) acc[q] = b[o];
    for (int i = 0; i < nin; ++i) {
        const float w = bf16_to_f(ws[i * nout + o]);
#pragma unroll
        for (int q = 0; q < kRowsPerBlock; ++q)
            if (q < rows) acc[q] += xs[min(grp * rows + q, kRowsPerBlock - 1)][i] * w;
    }
#pragma unroll
    for (int q = 0; q < kRowsPerBlock; ++q) {
        if (q >= rows) break;
        const int64_t r = r0 + grp * rows + q;
        if (grp * rows + q >= kRowsPerBlock || r >= n) break;
        if (act) {
            Z[r * nout + o] = acc[q];
            Aout[r * nout + o] = f_to_bf16(gelu(acc[q]));
        } else {
            if (Yout) Yout[r * nout + o] = acc[q];
            if (Ydbl) Ydbl[r * ldy + o] = (double)acc[q];
        }
    }
}

// dZprev = (dZ W) * GELU'(Zprev) for 32 rows per block
__global__ void __launch_bounds__(256) dense_bwd_data_kernel(int64_t n, const float *dZ, int nout, const uint16_t *W,
                                                             int nin, const float *Zprev, float *dZprev) {
    __shared__ float ds[kRowsPerBlock][kH];
    __shared__ uint16_t ws[kH * kH];                    // natural: ws[o * nin + i]
    const int64_t r0 = (int64_t)blockIdx.x * kRowsPerBlock;
    for (int idx = threadIdx.x; idx < kRowsPerBlock * nout; idx += 256) {
        const int r = idx / nout, o = idx - (idx / nout) * nout;
        ds[r][o] = (r0 + r < n) ? dZ[(r0 + r) * nout + o] : 0.0f;
    }
    for (int idx = threadIdx.x; idx < nout * nin; idx += 256) ws[idx] = W[idx];
    __syncthreads();
    const int groups = 256 / nin;
    const int i = threadIdx.x % nin, grp = threadIdx.x / nin;
    if (grp >= groups) return;
    const int rows = (kRowsPerBlock + groups - 1) / groups;
    float acc[kRowsPerBlock];
#pragma unroll
    for (int q = 0; q < kRowsPerBlock; ++q) acc[q] = 0.0f;
    for (int o = 0; o < nout; ++o) {
        const float w = bf16_to_f(ws[o * nin + i]);
#pragma unroll
        for (int q = 0; q < kRowsPerBlock; ++q)
            if (q < rows) acc[q] += ds[min(grp * rows + q, kRowsPerBlock - 1)][o] * w;
    }
#pragma unroll
    for (int q = 0; q < kRowsPerBlock; ++q) {
        if (q >= rows) break;
        const int64_t r = r0 + grp * rows + q;
        if (grp * rows + q >= kRowsPerBlock || r >= n) break;
        dZprev[r * nin + i] = acc[q] * gelu_grad(Zprev[r * nin + i]);
    }
}

// per-block partial weight gradients: gW[o][i] = sum_r dZ[r][o] In[r][i], gb[o] = sum_r dZ[r][o]
template <typename Tin>
__global__ void __launch_bounds__(256) dense_bwd_weight_kernel(int64_t n, const float *dZ, int nout, const Tin *in,
                                                               int nin, float *part, int stride) {
    __shared__ float ds[kRowsPerBlock][kH];
    __shared__ float xs[kRowsPerBlock][kH + 1];
    const int cnt = nout * nin + nout;
    constexpr int kPer = (kH * kH + kH + 255) / 256;
    float acc[kPer];
#pragma unroll
    for (int q = 0; q < kPer; ++q) acc[q] = 0.0f;
    const int64_t rows_per_block = ((n + gridDim.x - 1) / gridDim.x + kRowsPerBlock - 1) / kRowsPerBlock * kRowsPerBlock;
    const int64_t a = (int64_t)blockIdx.x * rows_per_block;
    const int64_t bnd = a + rows_per_block < n ? a + rows_per_block : n;
    for (int64_t r0 = a; r0 < bnd; r0 += kRowsPerBlock) {
        __syncthreads();
        for (int idx = threadIdx.x; idx < kRowsPerBlock * nout; idx += 256) {
            const int r = idx / nout, o = idx - (idx / nout) * nout;
            ds[r][o] = (r0 + r < bnd) ? dZ[(r0 + r) * nout + o] : 0.0f;
        }
        for (int idx = threadIdx.x; idx < kRowsPerBlock * nin; idx += 256) {
            const int r = idx / nin, i = idx - (idx / nin) * nin;
            xs[r][i] = (r0 + r < bnd) ? load_in<Tin>(in + (r0 + r) * nin + i) : 0.0f;
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < kPer; ++q) {
            const int j = threadIdx.x + 256 * q;
            if (j >= cnt) continue;
            float s = 0.0f;
            if (j < nout * nin) {
                const int o = j / nin, i = j - (j / nin) * nin;
                for (int r = 0; r < kRowsPerBlock; ++r) s += ds[r][o] * xs[r][i];
            } else {
                const int o = j - nout * nin;
                for (int r = 0; r < kRowsPerBlock; ++r) s += ds[r][o];
            }
            acc[q] += s;
        }
    }
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
        const int j = threadIdx.x + 256 * q;
        if (j < cnt) part[(size_t)blockIdx.x * stride + j] = acc[q];
    }
}

// g[j] = sum over blocks (ascending) of part[b][j]
__global__ void reduce_part_kernel(int nblk, int cnt, const float *part, int stride, float *g) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= cnt) return;
    float s = 0.0f;
    for (int b = 0; b < nblk; ++b) s += part[(size_t)b * stride + j];
    g[j] = s;
}

__global__ void scale_rows_kernel(int64_t n, int k, const float *Y, const double *T, int64_t ldt, const double *d,
                                  float *DY, float *Tf, float *DT) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * k) return;
    const int64_t r = t / k;
    const int c = (int)(t - r * k);
    const double dr = d[r];
    const double tv = T[r * ldt + c];
    DY[t] = (float)(dr * (double)Y[t]);
    Tf[t] = (float)tv;
    DT[t] = (float)(dr * tv);
}

// Gauss-Jordan inverse of an SPD k x k matrix in LDS (k <= 64), in place; 256 threads
__device__ void gj_inverse(double *Am, double *Inv, int k) {
    const int tid = threadIdx.x;
    for (int idx = tid; idx < k * k; idx += 256) Inv[idx] = (idx / k == idx % k) ? 1.0 : 0.0;
    __syncthreads();
    for (int c = 0; c < k; ++c) {
        const double piv = Am[c * k + c];
        __syncthreads();
        for (int j = tid; j < k; j += 256) {
            Am[c * k + j] /= piv;
            Inv[c * k + j] /= piv;
        }
        __syncthreads();
        for (int idx = tid; idx < k * k; idx += 256) {
            const int r = idx / k, j = idx - (idx / k) * k;
            if (r == c) continue;
            const double f = Am[r * k + c];
            if (j != c) Am[r * k + j] -= f * Am[c * k + j];
            Inv[r * k + j] -= f * Inv[c * k + j];
        }
        __syncthreads();
        for (int r = tid; r < k; r += 256)
            if (r != c) Am[r * k + c] = 0.0;
        __syncthreads();
    }
}

// From A = Y^T D Y, B = Y^T D T (G[0], G[1]) and Cm = T^T D T: the loss and
// G1 = -2 E B^T A^-1, G2 = 2 A^-1 B E B^T A^-1 (E = Cm^-1); one block, k <= 64.
__global__ void __launch_bounds__(256) loss_small_kernel(int k, const double *G, const double *Cg, double *G1,
                                                         double *G2, double *loss) {
    __shared__ double Am[64 * 64], Ai[64 * 64], Cm[64 * 64], Ei[64 * 64];
    double *T1 = Cm;                                     // reused after E is formed
    const int tid = threadIdx.x;
    const int kk = k * k;
    const double *Ag = G, *Bg = G + kk;
    for (int idx = tid; idx < kk; idx += 256) {
        const int r = idx / k, c = idx - (idx / k) * k;
        Am[idx] = 0.5 * (Ag[r * k + c] + Ag[c * k + r]);
        Cm[idx] = 0.5 * (Cg[r * k + c] + Cg[c * k + r]);
    }
    __syncthreads();
    gj_inverse(Am, Ai, k);
    gj_inverse(Cm, Ei, k);
    // T1 = B E ; F = T1 B^T -> stored in Am ; L = k - tr(Ai F)
    for (int idx = tid; idx < kk; idx += 256) {
        const int r = idx / k, c = idx - (idx / k) * k;
        double s = 0.0;
        for (int a = 0; a < k; ++a) s += Bg[r * k + a] * Ei[a * k + c];
        T1[idx] = s;
    }
    __syncthreads();
    for (int idx = tid; idx < kk; idx += 256) {
        const int r = idx / k, c = idx - (idx / k) * k;
        double s = 0.0;
        for (int a = 0; a < k; ++a) s += T1[r * k + a] * Bg[c * k + a];
        Am[idx] = s;                                     // F = B E B^T
    }
    __syncthreads();
    if (tid == 0) {
        double tr = 0.0;
        for (int r = 0; r < k; ++r)
            for (int a = 0; a < k; ++a) tr += Ai[r * k + a] * Am[a * k + r];
        *loss = (double)k - tr;
    }
    // G1 = -2 (B E)^T A^-1 = -2 T1^T Ai ; G2 = 2 Ai F Ai
    for (int idx = tid; idx < kk; idx += 256) {
        const int r = idx / k, c = idx - (idx / k) * k;
        double s = 0.0;
        for (int a = 0; a < k; ++a) s += T1[a * k + r] * Ai[a * k + c];
        G1[idx] = -2.0 * s;
    }
    __syncthreads();
    for (int idx = tid; idx < kk; idx += 256) {
        const int r = idx / k, c = idx - (idx / k) * k;
        double s = 0.0;
        for (int a = 0; a < k; ++a) s += Am[r * k + a] * Ai[a * k + c];
        Ei[idx] = s;                                     // F Ai
    }
    __syncthreads();
    for (int idx = tid; idx < kk; idx += 256) {
        const int r = idx / k, c = idx - (idx / k) * k;
        double s = 0.0;
        for (int a = 0; a < k; ++a) s += Ai[r * k + a] * Ei[a * k + c];
        G2[idx] = 2.0 * s;
    }
}

// dY[r][c] = d_r * sum_a (T[r][a] G1[a][c] + Y[r][a] G2[a][c])
__global__ void dy_kernel(int64_t n, int k, const double *T, int64_t ldt, const float *Y, const double *d,
                          const double *G1, const double *G2, float *dY) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * k) return;
    const int64_t r = t / k;
    const int c = (int)(t - r * k);
    double s = 0.0;
    for (int a = 0; a < k; ++a) s += T[r * ldt + a] * G1[a * k + c] + (double)Y[r * k + a] * G2[a * k + c];
    dY[t] = (float)(d[r] * s);
}

__global__ void adam_kernel(int P, float *p, const float *g, float *m, float *v, float lr, float b1, float b2,
                            float eps, float c1, float c2, uint16_t *pb) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= P) return;
    const float gj = g[j];
    const float mj = b1 * m[j] + (1.0f - b1) * gj;
    const float vj = b2 * v[j] + (1.0f - b2) * gj * gj;
    m[j] = mj;
    v[j] = vj;
    const float pj = p[j] - lr * (mj / c1) / (sqrtf(vj / c2) + eps);
    p[j] = pj;
    pb[j] = f_to_bf16(pj);
}

__global__ void to_bf16_kernel(int P, const float *p, uint16_t *pb) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < P) pb[j] = f_to_bf16(p[j]);
}

// object-wide statistics for the inputs: bbox and the means of two features
__global__ void __launch_bounds__(256) input_stats_kernel(int64_t n, const double *xyz, const float *feat,
                                                          double *part) {
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY}, s4 = 0.0, s5 = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        for (int a = 0; a < 3; ++a) {
            lo[a] = fmin(lo[a], xyz[3 * i + a]);
            hi[a] = fmax(hi[a], xyz[3 * i + a]);
        }
        s4 += feat[8 * i + 4];
        s5 += feat[8 * i + 5];
    }
    __shared__ double sh[8][256];
    for (int a = 0; a < 3; ++a) {
        sh[a][threadIdx.x] = lo[a];
        sh[3 + a][threadIdx.x] = hi[a];
    }
    sh[6][threadIdx.x] = s4;
    sh[7][threadIdx.x] = s5;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) {
            for (int a = 0; a < 3; ++a) {
                sh[a][threadIdx.x] = fmin(sh[a][threadIdx.x], sh[a][threadIdx.x + st]);
                sh[3 + a][threadIdx.x] = fmax(sh[3 + a][threadIdx.x], sh[3 + a][threadIdx.x + st]);
            }
            sh[6][threadIdx.x] += sh[6][threadIdx.x + st];
            sh[7][threadIdx.x] += sh[7][threadIdx.x + st];
        }
        __syncthreads();
    }
    if (threadIdx.x < 8) part[blockIdx.x * 8 + threadIdx.x] = sh[threadIdx.x][0];
}

__global__ void input_map_kernel(int64_t n, const double *xyz, const float *feat, const double *part, int nb,
                                 int n_freq, float *out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double lo[3], hi[3], s4 = 0.0, s5 = 0.0;
    for (int a = 0; a < 3; ++a) {
        lo[a] = part[a];
        hi[a] = part[3 + a];
    }
    for (int b = 0; b < nb; ++b) {
        for (int a = 0; a < 3; ++a) {
            lo[a] = fmin(lo[a], part[b * 8 + a]);
            hi[a] = fmax(hi[a], part[b * 8 + 3 + a]);
        }
        s4 += part[b * 8 + 6];
        s5 += part[b * 8 + 7];
    }
    const double half = 0.5 * fmax(fmax(hi[0] - lo[0], hi[1] - lo[1]), hi[2] - lo[2]);
    float *o = out + (int64_t)(kBase + 6 * n_freq) * i;
    double x[3];
    for (int a = 0; a < 3; ++a) {
        x[a] = (xyz[3 * i + a] - 0.5 * (lo[a] + hi[a])) / half;
        o[a] = (float)x[a];
    }
    // octave l: sin(pi 2^l x_a), then cos(pi 2^l x_a); sinpi/cospi reduce the argument exactly
    double sc = 1.0;
    for (int l = 0; l < n_freq; ++l, sc *= 2.0)
        for (int a = 0; a < 3; ++a) {
            o[kBase + 6 * l + a] = (float)sinpi(sc * x[a]);
            o[kBase + 6 * l + 3 + a] = (float)cospi(sc * x[a]);
        }
    const float *f = feat + 8 * i;
    o[3] = f[0];
    o[4] = f[1];
    o[5] = f[2];
    o[6] = f[3];
    o[7] = (float)(f[4] / (s4 / (double)n));
    o[8] = (float)(f[5] / (s5 / (double)n));
    o[9] = f[6];
    o[10] = f[7];
}

__global__ void row_sum_kernel(int64_t n, const int64_t *row_ptr, const double *M, double *d) {
    const int lane = threadIdx.x & 63;
    const int64_t r = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    if (r >= n) return;
    double s = 0.0;
    for (int64_t e = row_ptr[r] + lane; e < row_ptr[r + 1]; e += 64) s += M[e];
    for (int dd = 32; dd >= 1; dd >>= 1) s += __shfl_xor(s, dd, 64);
    if (lane == 0) d[r] = s;
}

}  // namespace mlpk
}  // namespace ff

using namespace ff;
using namespace ff::mlpk;

namespace {

template <typename T>
int grow(ff_ctx *ctx, T **p, size_t count) {
    if (*p) (void)hipFree(*p);
    *p = nullptr;
    if (hipMalloc((void **)p, count * sizeof(T) + 256) != hipSuccess) {
        (void)hipGetLastError();
        return set_error(ctx, FF_ERR_OOM, "MLP workspace allocation of %zu bytes failed", count * sizeof(T));
    }
    return FF_OK;
}

int ensure_capacity(ff_mlp *mp, int64_t n) {
    if (n <= mp->cap) return FF_OK;
    ff_ctx *ctx = mp->ctx;
    (void)hipStreamSynchronize(ctx->stream);
    int rc = FF_OK;
    for (int l = 0; l < 3 && !rc; ++l) {
        rc = grow(ctx, &mp->Z[l], (size_t)n * kH);
        if (!rc) rc = grow(ctx, &mp->A[l], (size_t)n * kH);
    }
    const size_t nk = (size_t)n * mp->k;
    if (!rc) rc = grow(ctx, &mp->Y, nk);
    if (!rc) rc = grow(ctx, &mp->dY, nk);
    if (!rc) rc = grow(ctx, &mp->DY, nk);
    if (!rc) rc = grow(ctx, &mp->Tf, nk);
    if (!rc) rc = grow(ctx, &mp->DT, nk);
    if (!rc) rc = grow(ctx, &mp->dZa, (size_t)n * kH);
    if (!rc) rc = grow(ctx, &mp->dZb, (size_t)n * kH);
    if (rc) return rc;
    mp->cap = n;
    return FF_OK;
}

int forward_impl(ff_mlp *mp, int64_t n, const float *in, double *Ydbl, int64_t ldy) {
    ff_ctx *ctx = mp->ctx;
    const Layout L = layout(mp->k, mp->n_in);
    const unsigned nb = grid_for(n, kRowsPerBlock);
    hipStream_t st = ctx->stream;
    hipLaunchKernelGGL(dense_fwd_kernel<float>, dim3(nb), dim3(256), 0, st, n, in, mp->n_in, mp->pb + L.off_w[0],
                       mp->p32 + L.off_b[0], kH, 1, mp->Z[0], mp->A[0], (float *)nullptr, (double *)nullptr,
                       (int64_t)0);
    for (int l = 1; l < 3; ++l)
        hipLaunchKernelGGL(dense_fwd_kernel<uint16_t>, dim3(nb), dim3(256), 0, st, n, mp->A[l - 1], kH,
                           mp->pb + L.off_w[l], mp->p32 + L.off_b[l], kH, 1, mp->Z[l], mp->A[l], (float *)nullptr,
                           (double *)nullptr, (int64_t)0);
    hipLaunchKernelGGL(dense_fwd_kernel<uint16_t>, dim3(nb), dim3(256), 0, st, n, mp->A[2], kH, mp->pb + L.off_w[3],
                       mp->p32 + L.off_b[3], mp->k, 0, (float *)nullptr, (uint16_t *)nullptr, mp->Y, Ydbl, ldy);
    FF_CHECK_LAUNCH(ctx);
    return FF_OK;
}

// Column sums of squares of X and R over a chunk of kBlendRows rows: thread t takes column t % m
// (of X for t / m even, of R for t / m odd, so 2m <= 256) and every 256 / (2m)-th row of the
// chunk; partials in a fixed order.
constexpr int kBlendRows = 1024;
__global__ void __launch_bounds__(256) blend_ss_kernel(int64_t n, int m, const double *X, int64_t ldx,
                                                       const double *R, int64_t ldr, double *part) {
    __shared__ double red[256];
    const int t = threadIdx.x, per = 256 / (2 * m);
    const int c = t % m, which = (t / m) & 1, lane_row = t / (2 * m);
    const int64_t r0 = (int64_t)blockIdx.x * kBlendRows;
    const int64_t r1 = r0 + kBlendRows < n ? r0 + kBlendRows : n;
    double acc = 0.0;
    if (lane_row < per)
        for (int64_t r = r0 + lane_row; r < r1; r += per) {
            const double v = which ? R[r * ldr + c] : X[r * ldx + c];
            acc += v * v;
        }
    red[t] = lane_row < per ? acc : 0.0;
    __syncthreads();
    if (t < 2 * m) {
        double sum = 0.0;
        for (int q = 0; q < per; ++q) sum += red[q * 2 * m + t];
        part[(size_t)blockIdx.x * 2 * m + t] = sum;
    }
}

// scale[c] = 1 / rms(X_c), scale[m + c] = w / rms(R_c), chunk partials added in order
__global__ void blend_scale_kernel(int64_t n, int m, int nchunks, const double *part, double w, double *scale) {
    const int t = threadIdx.x;
    if (t >= 2 * m) return;
    double sum = 0.0;
    for (int b = 0; b < nchunks; ++b) sum += part[(size_t)b * 2 * m + t];
    const double rms = sqrt(sum / (double)n);
    const double f = rms > 1e-300 ? 1.0 / rms : 1e300;
    scale[t] = t < m ? f : w * f;
}

__global__ void blend_apply_kernel(int64_t n, int m, double *X, int64_t ldx, const double *R, int64_t ldr,
                                   const double *scale) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n * m) return;
    const int64_t r = i / m;
    const int c = (int)(i - r * m);
    X[r * ldx + c] = X[r * ldx + c] * scale[c] + R[r * ldr + c] * scale[m + c];
}

}  // namespace

extern "C" {

int block_blend(ff_ctx *ctx, int64_t n, int m, double *X, int64_t ldx, const double *R, int64_t ldr, double w) {
    if (!ctx) return FF_ERR_INVALID_ARG;
    FF_REQUIRE(ctx, n > 0 && X && R, "bad arguments");
    FF_REQUIRE(ctx, m >= 1 && m <= 64, "block width %d must be in [1, 64]", m);
    FF_REQUIRE(ctx, ldx >= m && ldr >= m, "leading dimensions must be >= m");
    FF_REQUIRE(ctx, std::isfinite(w) && w >= 0.0, "weight must be finite and >= 0");
    FF_HIP(ctx, hipSetDevice(ctx->device));
    const int nchunks = (int)((n + kBlendRows - 1) / kBlendRows);
    double *part = (double *)ws_get(ctx, WS_BLEND, ((size_t)nchunks + 1) * 2 * m * sizeof(double));
    if (!part) return FF_ERR_OOM;
    double *scale = part + (size_t)nchunks * 2 * m;
    hipStream_t st = ctx->stream;
    hipLaunchKernelGGL(blend_ss_kernel, dim3(nchunks), dim3(256), 0, st, n, m, (const double *)X, ldx, R, ldr, part);
    hipLaunchKernelGGL(blend_scale_kernel, dim3(1), dim3(128), 0, st, n, m, nchunks, (const double *)part, w, scale);
    hipLaunchKernelGGL(blend_apply_kernel, dim3(grid_for(n * m, 256)), dim3(256), 0, st, n, m, X, ldx, R, ldr,
                       (const double *)scale);
    FF_CHECK_LAUNCH(ctx);
    return FF_OK;
}

int mlp_param_count(int k, int n_in) {
    return (k >= 1 && k <= 64 && n_in >= 1 && n_in <= kH) ? layout(k, n_in).total : -1;
}

int mlp_create(ff_ctx *ctx, int k, int n_in, uint64_t seed, ff_mlp **out) {
    if (!ctx || !out) return FF_ERR_INVALID_ARG;
    FF_REQUIRE(ctx, k >= 1 && k <= 64, "MLP output width k = %d must be in [1, 64]", k);
    FF_REQUIRE(ctx, n_in >= 1 && n_in <= kH, "MLP input width %d must be in [1, %d]", n_in, kH);
    FF_HIP(ctx, hipSetDevice(ctx->device));
    ff_mlp *mp = new ff_mlp();
    mp->ctx = ctx;
    mp->device = ctx->device;
    mp->stream = ctx->stream;
    mp->k = k;
    mp->n_in = n_in;
    const Layout L = layout(k, n_in);
    mp->P = L.total;
    int rc = grow(ctx, &mp->p32, L.total);
    if (!rc) rc = grow(ctx, &mp->m, L.total);
    if (!rc) rc = grow(ctx, &mp->v, L.total);
    if (!rc) rc = grow(ctx, &mp->g, L.total);
    if (!rc) rc = grow(ctx, &mp->pb, L.total);
    if (!rc) rc = grow(ctx, &mp->gpart, (size_t)kWgBlocks * (kH * kH + kH));
    if (!rc) rc = grow(ctx, &mp->small, (size_t)8 * 64 * 64 + 16);
    if (rc) {
        mlp_destroy(mp);
        return rc;
    }
    // uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) weights, zero biases
    std::vector<float> h(L.total, 0.0f);
    std::mt19937_64 gen(seed);
    for (int l = 0; l < 4; ++l) {
        const double bound = 1.0 / std::sqrt((double)L.nin[l]);
        std::uniform_real_distribution<double> U(-bound, bound);
        for (int j = 0; j < L.nin[l] * L.nout[l]; ++j) h[L.off_w[l] + j] = (float)U(gen);
    }
    rc = mlp_set_params(mp, h.data());
    if (rc) {
        mlp_destroy(mp);
        return rc;
    }
    *out = mp;
    return FF_OK;
}

void mlp_destroy(ff_mlp *mp) {
    if (!mp) return;
    (void)hipSetDevice(mp->device);
    (void)hipStreamSynchronize(mp->stream);
    void *ptrs[] = {mp->p32, mp->m, mp->v, mp->g, mp->pb, mp->Z[0], mp->Z[1], mp->Z[2], mp->A[0], mp->A[1], mp->A[2],
                    mp->Y, mp->dY, mp->dZa, mp->dZb, mp->DY, mp->Tf, mp->DT, mp->gpart, mp->small};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    delete mp;
}

int mlp_set_params(ff_mlp *mp, const float *host) {
    if (!mp || !host) return FF_ERR_INVALID_ARG;
    ff_ctx *ctx = mp->ctx;
    FF_HIP(ctx, hipMemcpy(mp->p32, host, (size_t)mp->P * sizeof(float), hipMemcpyHostToDevice));
    FF_HIP(ctx, hipMemset(mp->m, 0, (size_t)mp->P * sizeof(float)));
    FF_HIP(ctx, hipMemset(mp->v, 0, (size_t)mp->P * sizeof(float)));
    FF_HIP(ctx, hipMemset(mp->g, 0, (size_t)mp->P * sizeof(float)));
    mp->t = 0;
    hipLaunchKernelGGL(to_bf16_kernel, dim3(grid_for(mp->P, 256)), dim3(256), 0, ctx->stream, mp->P, mp->p32, mp->pb);
    FF_CHECK_LAUNCH(ctx);
    FF_HIP(ctx, hipStreamSynchronize(ctx->stream));
    return FF_OK;
}

int mlp_get_params(ff_mlp *mp, float *host) {
    if (!mp || !host) return FF_ERR_INVALID_ARG;
    FF_HIP(mp->ctx, hipStreamSynchronize(mp->ctx->stream));
    FF_HIP(mp->ctx, hipMemcpy(host, mp->p32, (size_t)mp->P * sizeof(float), hipMemcpyDeviceToHost));
    return FF_OK;
}

int mlp_get_grad(ff_mlp *mp, float *host) {
    if (!mp || !host) return FF_ERR_INVALID_ARG;
    FF_HIP(mp->ctx, hipStreamSynchronize(mp->ctx->stream));
    FF_HIP(mp->ctx, hipMemcpy(host, mp->g, (size_t)mp->P * sizeof(float), hipMemcpyDeviceToHost));
    return FF_OK;
}

int mlp_inputs(ff_ctx *ctx, int64_t n, const double *xyz_sorted, const float *feat, int n_freq, float *in) {
    if (!ctx) return FF_ERR_INVALID_ARG;
    FF_REQUIRE(ctx, n > 0 && xyz_sorted && feat && in, "bad arguments");
    FF_REQUIRE(ctx, n_freq >= 0 && n_freq <= kMaxFreq, "n_freq = %d must be in [0, %d]", n_freq, kMaxFreq);
    FF_HIP(ctx, hipSetDevice(ctx->device));
    const int nb = 256;
    double *part = (double *)ws_get(ctx, WS_MLP0, (size_t)nb * 8 * sizeof(double));
    if (!part) return FF_ERR_OOM;
    hipLaunchKernelGGL(input_stats_kernel, dim3(nb), dim3(256), 0, ctx->stream, n, xyz_sorted, feat, part);
    hipLaunchKernelGGL(input_map_kernel, dim3(grid_for(n, 256)), dim3(256), 0, ctx->stream, n, xyz_sorted, feat, part,
                       nb, n_freq, in);
    FF_CHECK_LAUNCH(ctx);
    return FF_OK;
}

int mlp_forward(ff_mlp *mp, int64_t n, const float *in, double *Y, int64_t ldy) {
    if (!mp) return FF_ERR_INVALID_ARG;
    ff_ctx *ctx = mp->ctx;
    FF_REQUIRE(ctx, n > 0 && in && Y && ldy >= mp->k, "bad arguments");
    FF_HIP(ctx, hipSetDevice(ctx->device));
    int rc = ensure_capacity(mp, n);
    if (rc) return rc;
    return forward_impl(mp, n, in, Y, ldy);
}

int mlp_train_step(ff_mlp *mp, int64_t n, const float *in, const double *T, int64_t ldt, const double *d, float lr,
                   double *loss) {
    if (!mp) return FF_ERR_INVALID_ARG;
    ff_ctx *ctx = mp->ctx;
    const int k = mp->k;
    FF_REQUIRE(ctx, n >= k && in && T && d && ldt >= k, "bad arguments");
    FF_HIP(ctx, hipSetDevice(ctx->device));
    hipStream_t st = ctx->stream;
    int rc = ensure_capacity(mp, n);
    if (!rc) rc = forward_impl(mp, n, in, (double *)nullptr, 0);
    if (rc) return rc;
    // loss and dL/dY
    hipLaunchKernelGGL(scale_rows_kernel, dim3(grid_for(n * k, 256)), dim3(256), 0, st, n, k, mp->Y, T, ldt, d, mp->DY,
                       mp->Tf, mp->DT);
    FF_CHECK_LAUNCH(ctx);
    double *Gab = mp->small, *Gc = mp->small + 2 * 64 * 64, *G1 = Gc + 2 * 64 * 64, *G2 = G1 + 64 * 64;
    double *dloss = G2 + 64 * 64;
    if ((rc = gram_hm(ctx, n, k, 1, mp->Y, mp->DY, mp->DT, k, Gab))) return rc;      // Y^T D Y, Y^T D T
    if ((rc = gram_hm(ctx, n, k, 1, mp->Tf, mp->DT, mp->DT, k, Gc))) return rc;      // T^T D T
    hipLaunchKernelGGL(loss_small_kernel, dim3(1), dim3(256), 0, st, k, Gab, Gc, G1, G2, dloss);
    hipLaunchKernelGGL(dy_kernel, dim3(grid_for(n * k, 256)), dim3(256), 0, st, n, k, T, ldt, mp->Y, d, G1, G2, mp->dY);
    FF_CHECK_LAUNCH(ctx);
    // backward through the layers: weight partials, then data gradients
    const Layout L = layout(k, mp->n_in);
    const unsigned nb = grid_for(n, kRowsPerBlock);
    const int nwb = (int)std::min<int64_t>(kWgBlocks, (n + kRowsPerBlock - 1) / kRowsPerBlock);
    const int stride = kH * kH + kH;
    auto wgrad = [&](int l, const float *dZ, const void *in, bool in_f32) {
        const int nin = L.nin[l], nout = L.nout[l];
        if (in_f32)
            hipLaunchKernelGGL(dense_bwd_weight_kernel<float>, dim3(nwb), dim3(256), 0, st, n, dZ, nout,
                               (const float *)in, nin, mp->gpart, stride);
        else
            hipLaunchKernelGGL(dense_bwd_weight_kernel<uint16_t>, dim3(nwb), dim3(256), 0, st, n, dZ, nout,
                               (const uint16_t *)in, nin, mp->gpart, stride);
        const int cnt = nout * nin + nout;
        hipLaunchKernelGGL(reduce_part_kernel, dim3(grid_for(cnt, 256)), dim3(256), 0, st, nwb, cnt, mp->gpart,
                           stride, mp->g + L.off_w[l]);
    };
    wgrad(3, mp->dY, mp->A[2], false);
    hipLaunchKernelGGL(dense_bwd_data_kernel, dim3(nb), dim3(256), 0, st, n, mp->dY, k, mp->pb + L.off_w[3], kH,
                       mp->Z[2], mp->dZa);
    wgrad(2, mp->dZa, mp->A[1], false);
    hipLaunchKernelGGL(dense_bwd_data_kernel, dim3(nb), dim3(256), 0, st, n, mp->dZa, kH, mp->pb + L.off_w[2], kH,
                       mp->Z[1], mp->dZb);
    wgrad(1, mp->dZb, mp->A[0], false);
    hipLaunchKernelGGL(dense_bwd_data_kernel, dim3(nb), dim3(256), 0, st, n, mp->dZb, kH, mp->pb + L.off_w[1], kH,
                       mp->Z[0], mp->dZa);
    wgrad(0, mp->dZa, in, true);
    FF_CHECK_LAUNCH(ctx);
    mp->t += 1;
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.0f - std::pow(b1, (float)mp->t), c2 = 1.0f - std::pow(b2, (float)mp->t);
    hipLaunchKernelGGL(adam_kernel, dim3(grid_for(mp->P, 256)), dim3(256), 0, st, mp->P, mp->p32, mp->g, mp->m, mp->v,
                       lr, b1, b2, 1e-8f, c1, c2, mp->pb);
    FF_CHECK_LAUNCH(ctx);
    if (loss) {
        FF_HIP(ctx, hipMemcpyAsync(loss, dloss, sizeof(double), hipMemcpyDeviceToHost, st));
        FF_HIP(ctx, hipStreamSynchronize(st));
    }
    return FF_OK;
}

int lumped_mass(ff_ctx *ctx, int64_t n, const int64_t *row_ptr, const double *M, double *d) {
    if (!ctx) return FF_ERR_INVALID_ARG;
    FF_REQUIRE(ctx, n > 0 && row_ptr && M && d, "bad arguments");
    FF_HIP(ctx, hipSetDevice(ctx->device));
    hipLaunchKernelGGL(row_sum_kernel, dim3(grid_for(n, 4)), dim3(256), 0, ctx->stream, n, row_ptr, M, d);
    FF_CHECK_LAUNCH(ctx);
    return FF_OK;
}

}  // extern "C"
