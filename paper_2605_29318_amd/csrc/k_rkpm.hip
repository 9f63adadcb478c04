// RKPM shape functions and gradients (Sec. 3.2, Eq. (7)-(11)) on gfx950.
//
// One wavefront per quadrature point X; lanes stride its neighbour list. Each
// lane accumulates its part of the moment matrix in the shifted, scaled basis
// Ph_k = [1, (p_k - X)/h] (10 unique entries of the symmetric 4x4) and of
// sum_k grad phi~_k Ph_k Ph_k^T (3 x 10), the wave reduces the 40 sums with
// butterfly shuffles, every lane solves the same 4x4 system in FP64, and the
// lanes then write phi_k and grad phi_k for their neighbours (coalesced).
//
//   Mh = sum wt Ph Ph^T,  b = Mh^-1 e1,  phi_k = wt_k Ph_k^T b        (Eq. (7), (9)-(11))
//   d_s Mh = sum d_s wt Ph Ph^T - (e_{s+1} m^T + m e_{s+1}^T)/h,  m = Mh e1
//   d_s b = -Mh^-1 (d_s Mh) b
//   d_s phi_k = d_s wt_k Ph_k^T b - wt_k b_{s+1}/h + wt_k Ph_k^T d_s b
#include "ff_internal.h"

namespace ff {
namespace {

constexpr int kSyms = 10;   // unique entries of a symmetric 4x4: (0,0) (0,1) (0,2) (0,3) (1,1) (1,2) (1,3) (2,2) (2,3) (3,3)

__device__ inline int sym_index(int a, int b) {
    if (a > b) { int t = a; a = b; b = t; }
    // row-major upper triangle
    return a * 4 - (a * (a - 1)) / 2 + (b - a);
}

// cubic B-spline of z = |X - p|/h and its slope divided by z (finite at 0)
__device__ inline void spline(double z, double &w, double &f) {
    if (z <= 0.5) {
        w = 2.0 / 3.0 + z * z * (4.0 * z - 4.0);
        f = 12.0 * z - 8.0;
    } else if (z < 1.0) {
        const double t = 1.0 - z;
        w = (4.0 / 3.0) * (t * t * t);
        f = -4.0 * (t * t) / z;
    } else {
        w = 0.0;
        f = 0.0;
    }
}

// raw weight and gradient factor: grad phi~ = fac * (X - p) / h^2
__device__ inline void raw_kernel(int kind, double d2, double h, double &w, double &fac) {
    if (kind == 1) {
        const double r2 = 0.25 * h * h;    // r = h / 2
        if (d2 < h * h) {
            w = exp(-d2 / r2);
            fac = -2.0 * w * (h * h) / r2;
        } else {
            w = 0.0;
            fac = 0.0;
        }
    } else {
        spline(sqrt(d2) / h, w, fac);
    }
}

__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
    return v;
}

// 4x4 Cholesky; returns false if a pivot is <= 1e-14 * trace
__device__ inline bool chol4(const double A[4][4], double L[4][4]) {
    const double tr = A[0][0] + A[1][1] + A[2][2] + A[3][3];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        double d = A[j][j];
#pragma unroll
        for (int t = 0; t < j; ++t) d -= L[j][t] * L[j][t];
        if (!(d > 1e-14 * tr)) return false;
        L[j][j] = sqrt(d);
        const double inv = 1.0 / L[j][j];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            if (i <= j) { if (i < j) L[i][j] = 0.0; continue; }
            double s = A[i][j];
#pragma unroll
            for (int t = 0; t < j; ++t) s -= L[i][t] * L[j][t];
            L[i][j] = s * inv;
        }
    }
    return true;
}

__device__ inline void chol4_solve(const double L[4][4], const double b[4], double x[4]) {
    double y[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        double s = b[i];
#pragma unroll
        for (int t = 0; t < i; ++t) s -= L[i][t] * y[t];
        y[i] = s / L[i][i];
    }
#pragma unroll
    for (int i = 3; i >= 0; --i) {
        double s = y[i];
#pragma unroll
        for (int t = i + 1; t < 4; ++t) s -= L[t][i] * x[t];
        x[i] = s / L[i][i];
    }
}

// eigenvalues of a symmetric 4x4 by cyclic Jacobi (features only)
__device__ inline void eig4(double A[4][4], double ev[4]) {
    for (int sweep = 0; sweep < 12; ++sweep) {
        double off = 0.0;
        for (int p = 0; p < 4; ++p)
            for (int q = p + 1; q < 4; ++q) off += A[p][q] * A[p][q];
        if (off < 1e-30 * (A[0][0] * A[0][0] + A[1][1] * A[1][1] + A[2][2] * A[2][2] + A[3][3] * A[3][3]))
            break;
        for (int p = 0; p < 4; ++p)
            for (int q = p + 1; q < 4; ++q) {
                if (A[p][q] == 0.0) continue;
                const double tau = (A[q][q] - A[p][p]) / (2.0 * A[p][q]);
                const double t = (tau >= 0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                const double c = 1.0 / sqrt(1.0 + t * t), s = t * c;
                for (int r = 0; r < 4; ++r) {
                    const double ap = A[r][p], aq = A[r][q];
                    A[r][p] = c * ap - s * aq;
                    A[r][q] = s * ap + c * aq;
                }
                for (int r = 0; r < 4; ++r) {
                    const double ap = A[p][r], aq = A[q][r];
                    A[p][r] = c * ap - s * aq;
                    A[q][r] = s * ap + c * aq;
                }
            }
    }
    for (int i = 0; i < 4; ++i) ev[i] = A[i][i];
    for (int i = 1; i < 4; ++i) {
        double v = ev[i];
        int j = i - 1;
        while (j >= 0 && ev[j] > v) { ev[j + 1] = ev[j]; --j; }
        ev[j + 1] = v;
    }
}

__global__ void __launch_bounds__(256) rkpm_kernel(const double *xs, const double *qxyz, int64_t q,
                                                   const int64_t *off, const int32_t *ids, double h, int kind,
                                                   double *phi, double *dphi, float *feat,
                                                   unsigned long long *bad) {
    const int lane = threadIdx.x & 63;
    const int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    if (i >= q) return;
    const double X[3] = {qxyz[3 * i], qxyz[3 * i + 1], qxyz[3 * i + 2]};
    const int64_t e0 = off[i], e1 = off[i + 1];
    const double hinv = 1.0 / h;
    const double hh = h * h;

    // per-lane partial moments: S[0..9] = sum wt Ph Ph^T, G[s][0..9] = sum d_s wt Ph Ph^T
    double S[kSyms], G[3][kSyms], wsq = 0.0;
#pragma unroll
    for (int t = 0; t < kSyms; ++t) { S[t] = 0.0; G[0][t] = G[1][t] = G[2][t] = 0.0; }
    for (int64_t e = e0 + lane; e < e1; e += 64) {
        const int64_t k = ids[e];
        const double r0 = X[0] - xs[3 * k], r1 = X[1] - xs[3 * k + 1], r2 = X[2] - xs[3 * k + 2];
        const double d2 = ((r0 * r0) + (r1 * r1)) + (r2 * r2);
        double w, fac;
        raw_kernel(kind, d2, h, w, fac);
        const double P[4] = {1.0, -r0 * hinv, -r1 * hinv, -r2 * hinv};
        const double g[3] = {fac * r0 / hh, fac * r1 / hh, fac * r2 / hh};
        wsq += w * w;
        int t = 0;
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = a; b < 4; ++b, ++t) {
                const double pp = P[a] * P[b];
                S[t] += w * pp;
                G[0][t] += g[0] * pp;
                G[1][t] += g[1] * pp;
                G[2][t] += g[2] * pp;
            }
    }
#pragma unroll
    for (int t = 0; t < kSyms; ++t) {
        S[t] = wave_sum(S[t]);
        G[0][t] = wave_sum(G[0][t]);
        G[1][t] = wave_sum(G[1][t]);
        G[2][t] = wave_sum(G[2][t]);
    }
    if (feat) wsq = wave_sum(wsq);

    double Mh[4][4], L[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) Mh[a][b] = S[sym_index(a, b)];
    if (!chol4(Mh, L)) {
        if (lane == 0) atomicMin(bad, (unsigned long long)i);
        return;
    }
    const double e1v[4] = {1.0, 0.0, 0.0, 0.0};
    double b[4], db[3][4];
    chol4_solve(L, e1v, b);
#pragma unroll
    for (int s = 0; s < 3; ++s) {
        double dM[4][4];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int c = 0; c < 4; ++c) dM[a][c] = G[s][sym_index(a, c)];
        // the Ph-derivative part: -(e_{s+1} m^T + m e_{s+1}^T)/h with m = Mh e1
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            dM[s + 1][c] -= Mh[c][0] * hinv;
            dM[c][s + 1] -= Mh[c][0] * hinv;
        }
        double t[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) t[a] = dM[a][0] * b[0] + dM[a][1] * b[1] + dM[a][2] * b[2] + dM[a][3] * b[3];
        double x[4];
        chol4_solve(L, t, x);
#pragma unroll
        for (int a = 0; a < 4; ++a) db[s][a] = -x[a];
    }

    for (int64_t e = e0 + lane; e < e1; e += 64) {
        const int64_t k = ids[e];
        const double r0 = X[0] - xs[3 * k], r1 = X[1] - xs[3 * k + 1], r2 = X[2] - xs[3 * k + 2];
        const double d2 = ((r0 * r0) + (r1 * r1)) + (r2 * r2);
        double w, fac;
        raw_kernel(kind, d2, h, w, fac);
        const double P[4] = {1.0, -r0 * hinv, -r1 * hinv, -r2 * hinv};
        const double r[3] = {r0, r1, r2};
        const double Pb = P[0] * b[0] + P[1] * b[1] + P[2] * b[2] + P[3] * b[3];
        phi[e] = w * Pb;
#pragma unroll
        for (int s = 0; s < 3; ++s) {
            const double Pdb = P[0] * db[s][0] + P[1] * db[s][1] + P[2] * db[s][2] + P[3] * db[s][3];
            dphi[3 * e + s] = (fac * r[s] / hh) * Pb - w * b[s + 1] * hinv + w * Pdb;
        }
    }

    if (feat && lane == 0) {
        const double sw = Mh[0][0];
        const double cnt = (double)(e1 - e0);
        double A[4][4];
        for (int a = 0; a < 4; ++a)
            for (int c = 0; c < 4; ++c) A[a][c] = Mh[a][c] / sw;
        double ev[4];
        eig4(A, ev);
        const double mean = sw / cnt;
        const double var = fmax(0.0, wsq / cnt - mean * mean);
        float *f = feat + 8 * i;
        f[0] = (float)ev[0];
        f[1] = (float)ev[1];
        f[2] = (float)ev[2];
        f[3] = (float)ev[3];
        f[4] = (float)cnt;
        f[5] = (float)sw;
        f[6] = (float)(sqrt(Mh[0][1] * Mh[0][1] + Mh[0][2] * Mh[0][2] + Mh[0][3] * Mh[0][3]) / sw);
        f[7] = (float)(sqrt(var) / mean);
    }
}

// Gaussian exp(-s), s = d^2 / r^2, cut at s = c^2 with its tangent there subtracted (value and
// slope vanish at the cut): w = exp(-s) - exp(-c^2) (1 + c^2 - s), grad w = go (X - p) with
// go = 2 (exp(-c^2) - exp(-s)) / r^2; zero beyond the cut.
__device__ inline void gauss_cut(double d2, double rk, double cut, double &w, double &go) {
    const double s = d2 / (rk * rk), c2 = cut * cut;
    if (s < c2) {
        const double e = exp(-s), ec = exp(-c2);
        w = e - ec * (1.0 + c2 - s);
        go = (-e + ec) * 2.0 / (rk * rk);
    } else {
        w = 0.0;
        go = 0.0;
    }
}

// Shape functions on the centres' own Gaussians (radius r_k per node), one wavefront per
// point as rkpm_kernel, for three bases (Sec. 3.2 and its Fig. 3b comparison):
//   kBasis 0  plain RBF               phi_k = w_k
//   kBasis 1  partition-of-unity RBF  phi_k = w_k / sum w
//   kBasis 2  RKPM, linear basis      Eq. (7)-(11) in the shifted basis [1, (p - X)/h]
template <int kBasis>
__global__ void __launch_bounds__(256) rkpm_var_kernel(const double *xs, const double *rnode, const int32_t *perm,
                                                       const double *qxyz, int64_t q, const int64_t *off,
                                                       const int32_t *ids, double h, double cut, double *phi,
                                                       double *dphi, unsigned long long *bad) {
    const int lane = threadIdx.x & 63;
    const int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    if (i >= q) return;
    const double X[3] = {qxyz[3 * i], qxyz[3 * i + 1], qxyz[3 * i + 2]};
    const int64_t e0 = off[i], e1 = off[i + 1];
    const double hinv = 1.0 / h;
    constexpr int NS = kBasis == 2 ? kSyms : 1;
    double S[NS], G[3][NS];
#pragma unroll
    for (int t = 0; t < NS; ++t) { S[t] = 0.0; G[0][t] = G[1][t] = G[2][t] = 0.0; }
    if (kBasis > 0) {
        for (int64_t e = e0 + lane; e < e1; e += 64) {
            const int64_t k = ids[e];
            const double r0 = X[0] - xs[3 * k], r1 = X[1] - xs[3 * k + 1], r2 = X[2] - xs[3 * k + 2];
            const double d2 = ((r0 * r0) + (r1 * r1)) + (r2 * r2);
            double w, go;
            gauss_cut(d2, rnode[perm ? perm[k] : k], cut, w, go);
            const double g[3] = {go * r0, go * r1, go * r2};
            if (kBasis == 1) {
                S[0] += w;
                G[0][0] += g[0];
                G[1][0] += g[1];
                G[2][0] += g[2];
            } else {
                const double P[4] = {1.0, -r0 * hinv, -r1 * hinv, -r2 * hinv};
                int t = 0;
#pragma unroll
                for (int a = 0; a < 4; ++a)
#pragma unroll
                    for (int b = a; b < 4; ++b, ++t) {
                        const double pp = P[a] * P[b];
                        S[t] += w * pp;
                        G[0][t] += g[0] * pp;
                        G[1][t] += g[1] * pp;
                        G[2][t] += g[2] * pp;
                    }
            }
        }
#pragma unroll
        for (int t = 0; t < NS; ++t) {
            S[t] = wave_sum(S[t]);
            G[0][t] = wave_sum(G[0][t]);
            G[1][t] = wave_sum(G[1][t]);
            G[2][t] = wave_sum(G[2][t]);
        }
    }
    double b[4] = {0.0, 0.0, 0.0, 0.0}, db[3][4] = {};
    if (kBasis == 1 && !(S[0] > 0.0)) {
        if (lane == 0) atomicMin(bad, (unsigned long long)i);
        return;
    }
    if (kBasis == 2) {
        double Mh[4][4], L[4][4];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int c = 0; c < 4; ++c) Mh[a][c] = S[kBasis == 2 ? sym_index(a, c) : 0];
        if (!chol4(Mh, L)) {
            if (lane == 0) atomicMin(bad, (unsigned long long)i);
            return;
        }
        const double e1v[4] = {1.0, 0.0, 0.0, 0.0};
        chol4_solve(L, e1v, b);
#pragma unroll
        for (int s = 0; s < 3; ++s) {
            double dM[4][4];
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int c = 0; c < 4; ++c) dM[a][c] = G[s][kBasis == 2 ? sym_index(a, c) : 0];
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                dM[s + 1][c] -= Mh[c][0] * hinv;
                dM[c][s + 1] -= Mh[c][0] * hinv;
            }
            double t[4];
#pragma unroll
            for (int a = 0; a < 4; ++a) t[a] = dM[a][0] * b[0] + dM[a][1] * b[1] + dM[a][2] * b[2] + dM[a][3] * b[3];
            double x[4];
            chol4_solve(L, t, x);
#pragma unroll
            for (int a = 0; a < 4; ++a) db[s][a] = -x[a];
        }
    }
    for (int64_t e = e0 + lane; e < e1; e += 64) {
        const int64_t k = ids[e];
        const double r0 = X[0] - xs[3 * k], r1 = X[1] - xs[3 * k + 1], r2 = X[2] - xs[3 * k + 2];
        const double d2 = ((r0 * r0) + (r1 * r1)) + (r2 * r2);
        double w, go;
        gauss_cut(d2, rnode[perm ? perm[k] : k], cut, w, go);
        const double r[3] = {r0, r1, r2};
        if (kBasis == 0) {
            phi[e] = w;
#pragma unroll
            for (int s = 0; s < 3; ++s) dphi[3 * e + s] = go * r[s];
        } else if (kBasis == 1) {
            const double inv = 1.0 / S[0];
            phi[e] = w * inv;
#pragma unroll
            for (int s = 0; s < 3; ++s) dphi[3 * e + s] = go * r[s] * inv - w * G[s][0] * (inv * inv);
        } else {
            const double P[4] = {1.0, -r0 * hinv, -r1 * hinv, -r2 * hinv};
            const double Pb = P[0] * b[0] + P[1] * b[1] + P[2] * b[2] + P[3] * b[3];
            phi[e] = w * Pb;
#pragma unroll
            for (int s = 0; s < 3; ++s) {
                const double Pdb = P[0] * db[s][0] + P[1] * db[s][1] + P[2] * db[s][2] + P[3] * db[s][3];
                dphi[3 * e + s] = (go * r[s]) * Pb - w * b[s + 1] * hinv + w * Pdb;
            }
        }
    }
}

}  // namespace
}  // namespace ff

using namespace ff;

extern "C" int rkpm_shape_radii(ff_ctx *ctx, int64_t n, const double *xyz_sorted, const double *node_r,
                                const int32_t *perm, int64_t q, const double *qxyz, const int64_t *nbr_off,
                                const int32_t *nbr_id, int64_t nbr_total, double h, double cut, int basis,
                                double *phi, double *dphi, int64_t *bad_index) {
    if (!ctx) return FF_ERR_INVALID_ARG;
    FF_REQUIRE(ctx, n > 0 && q > 0, "empty input");
    FF_REQUIRE(ctx, xyz_sorted && node_r && nbr_off && nbr_id && phi && dphi, "required pointer is NULL");
    FF_REQUIRE(ctx, std::isfinite(h) && h > 0.0, "scale h must be finite and positive");
    FF_REQUIRE(ctx, std::isfinite(cut) && cut > 0.0, "cut must be finite and positive");
    FF_REQUIRE(ctx, basis >= 0 && basis <= 2, "basis must be 0 (RBF), 1 (partition-of-unity RBF) or 2 (RKPM)");
    if (!qxyz) FF_REQUIRE(ctx, q == n, "qxyz == NULL requires q == n");
    (void)nbr_total;
    FF_HIP(ctx, hipSetDevice(ctx->device));
    hipStream_t st = ctx->stream;
    unsigned long long *bad = (unsigned long long *)ws_get(ctx, WS_FLAG, 64);
    unsigned long long *host = (unsigned long long *)pinned_get(ctx, 4096);
    if (!bad || !host) return FF_ERR_OOM;
    FF_HIP(ctx, hipMemsetAsync(bad, 0xff, sizeof(unsigned long long), st));
    const double *Q = qxyz ? qxyz : xyz_sorted;
    const dim3 grid(grid_for(q, 4)), block(256);
    if (basis == 0)
        hipLaunchKernelGGL(rkpm_var_kernel<0>, grid, block, 0, st, xyz_sorted, node_r, perm, Q, q, nbr_off, nbr_id, h,
                           cut, phi, dphi, bad);
    else if (basis == 1)
        hipLaunchKernelGGL(rkpm_var_kernel<1>, grid, block, 0, st, xyz_sorted, node_r, perm, Q, q, nbr_off, nbr_id, h,
                           cut, phi, dphi, bad);
    else
        hipLaunchKernelGGL(rkpm_var_kernel<2>, grid, block, 0, st, xyz_sorted, node_r, perm, Q, q, nbr_off, nbr_id, h,
                           cut, phi, dphi, bad);
    FF_CHECK_LAUNCH(ctx);
    FF_HIP(ctx, hipMemcpyAsync(host, bad, sizeof(unsigned long long), hipMemcpyDeviceToHost, st));
    FF_HIP(ctx, hipStreamSynchronize(st));
    const int64_t b = (host[0] == ~0ull) ? -1 : (int64_t)host[0];
    if (bad_index) *bad_index = b;
    if (b >= 0)
        return set_error(ctx, FF_ERR_SINGULAR_MOMENT, "%s at quadrature point %lld",
                         basis == 2 ? "moment matrix not positive definite" : "kernel sum is zero", (long long)b);
    return FF_OK;
}

extern "C" int rkpm_shape(ff_ctx *ctx, int64_t n, const double *xyz_sorted, int64_t q, const double *qxyz,
                          const int64_t *nbr_off, const int32_t *nbr_id, int64_t nbr_total, double h, int kernel,
                          double *phi, double *dphi, float *feat, int64_t *bad_index) {
    if (!ctx) return FF_ERR_INVALID_ARG;
    FF_REQUIRE(ctx, n > 0 && q > 0, "empty input");
    FF_REQUIRE(ctx, xyz_sorted && nbr_off && nbr_id && phi && dphi, "required pointer is NULL");
    FF_REQUIRE(ctx, std::isfinite(h) && h > 0.0, "support radius h must be finite and positive");
    FF_REQUIRE(ctx, kernel == 0 || kernel == 1, "kernel must be 0 (cubic B-spline) or 1 (Gaussian)");
    if (!qxyz) FF_REQUIRE(ctx, q == n, "qxyz == NULL requires q == n");
    (void)nbr_total;
    FF_HIP(ctx, hipSetDevice(ctx->device));
    hipStream_t st = ctx->stream;
    unsigned long long *bad = (unsigned long long *)ws_get(ctx, WS_FLAG, 64);
    unsigned long long *host = (unsigned long long *)pinned_get(ctx, 4096);
    if (!bad || !host) return FF_ERR_OOM;
    FF_HIP(ctx, hipMemsetAsync(bad, 0xff, sizeof(unsigned long long), st));
    const double *Q = qxyz ? qxyz : xyz_sorted;
    hipLaunchKernelGGL(rkpm_kernel, dim3(grid_for(q, 4)), dim3(256), 0, st, xyz_sorted, Q, q, nbr_off, nbr_id, h,
                       kernel, phi, dphi, feat, bad);
    FF_CHECK_LAUNCH(ctx);
    FF_HIP(ctx, hipMemcpyAsync(host, bad, sizeof(unsigned long long), hipMemcpyDeviceToHost, st));
    FF_HIP(ctx, hipStreamSynchronize(st));
    int64_t b = (host[0] == ~0ull) ? -1 : (int64_t)host[0];
    if (bad_index) *bad_index = b;
    if (b >= 0)
        return set_error(ctx, FF_ERR_SINGULAR_MOMENT,
                         "moment matrix not positive definite at quadrature point %lld", (long long)b);
    return FF_OK;
}
