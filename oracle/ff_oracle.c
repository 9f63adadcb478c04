/*
 * ff_oracle.c - plain, slow, obviously-correct FP64 reference of the
 * subspace-construction path of "FreeForm: Reduced-Order Deformable
 * Simulation from Particle-Based Skinning Eigenmodes" (arXiv 2605.29318).
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product library links, loads or
 * calls this file; only the tests, the smoke check and the CPU baseline leg of
 * the benchmark do. It shares no code, header or table with the GPU path.
 *
 * Build: gcc -O2 -fopenmp -ffp-contract=off -fPIC -shared (no FMA contraction,
 * IEEE division and square root), so that the integer results that floating
 * point decides (cell index, neighbour predicate) are reproducible.
 *
 * Steps and the passages they follow:
 *   orc_grid / orc_bin      uniform cell list (the paper has none; cell size = support radius),
 *                           nodes ordered by cell, then by a Morton code of 4x4x4 sub-cells
 *   orc_neighbors           support of the compact kernel: d^2 < h^2
 *   orc_neighbors_brute     the same predicate by exhaustive search (pin)
 *   orc_rkpm                RKPM shape functions and gradients, Sec. 3.2 Eq. (7)-(11)
 *   orc_transpose           N^T(k) = { i : k in N(i) } with slots
 *   orc_assemble            weight-space Hessian (Prop. 1) and RKPM mass matrix (Eq. (14))
 *   orc_spmm, orc_norm_inf  y = A x and max_i sum_j |A_ij| on a CSR matrix (residual checks)
 *   orc_fps                 farthest point sampling of the kernel centres (Supp. B.1)
 *   orc_radii               each centre's Gaussian radius: distance to its 2nd-nearest centre
 *   orc_neighbors_var       lists with a radius per centre, d^2 < R_k^2 (Supp. B.1)
 *   orc_neighbors_var_brute the same predicate by exhaustive search (pin)
 *   orc_rkpm_var            shape functions on the centres' cut Gaussians for plain RBF,
 *                           partition-of-unity RBF and RKPM (Sec. 3.2, Fig. 3b)
 *
 * Parity status: every function here is pinned by the "not gpu" tests
 * (brute force, reproducing conditions, finite differences of the
 * Neo-Hookean energy, closed forms); see the tests for each pin.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_ERR_ARG (-1)
#define ORC_ERR_SINGULAR (-5)

/* ------------------------------------------------------------------------ */
/* cell grid                                                                 */
/* ------------------------------------------------------------------------ */

/* origin = componentwise minimum of the nodes; dims_a = floor((max_a - o_a)/h) + 1 */
int orc_grid(int64_t n, const double *xyz, double h, double *origin, int64_t *dims)
{
    if (n <= 0 || !(h > 0.0)) return ORC_ERR_ARG;
    for (int a = 0; a < 3; ++a) {
        double lo = xyz[a], hi = xyz[a];
        for (int64_t i = 1; i < n; ++i) {
            double v = xyz[3 * i + a];
            if (v < lo) lo = v;
            if (v > hi) hi = v;
        }
        origin[a] = lo;
        dims[a] = (int64_t)floor((hi - lo) / h) + 1;
    }
    return ORC_OK;
}

/* q_a = min(max(floor((x_a - o_a)/h), 0), D_a - 1), division not reciprocal */
static int64_t cell_coord(double x, double o, double h, int64_t D)
{
    double t = floor((x - o) / h);
    if (t < 0.0) t = 0.0;
    if (t > (double)(D - 1)) t = (double)(D - 1);
    return (int64_t)t;
}

static int64_t cell_of(const double *p, const double *o, double h, const int64_t *D)
{
    int64_t cx = cell_coord(p[0], o[0], h, D[0]);
    int64_t cy = cell_coord(p[1], o[1], h, D[1]);
    int64_t cz = cell_coord(p[2], o[2], h, D[2]);
    return (cz * D[1] + cy) * D[0] + cx;
}

/* sub-cell index of a node inside its cell along one axis: the cell split in 4,
 * s_a = min(max(floor((t_a - q_a) * 4), 0), 3) with t_a = (x_a - o_a)/h and q_a the
 * (clamped) cell coordinate */
static int64_t sub_coord(double x, double o, double h, int64_t D)
{
    double t = (x - o) / h;
    double q = floor(t);
    if (q < 0.0) q = 0.0;
    if (q > (double)(D - 1)) q = (double)(D - 1);
    double s = floor((t - q) * 4.0);
    if (s < 0.0) s = 0.0;
    if (s > 3.0) s = 3.0;
    return (int64_t)s;
}

/* Morton code of the node's sub-cell: the three 2-bit sub-cell indices
 * interleaved, x in the lowest bit of each triple */
static int64_t subcell_code(const double *p, const double *o, double h, const int64_t *D)
{
    int64_t sx = sub_coord(p[0], o[0], h, D[0]);
    int64_t sy = sub_coord(p[1], o[1], h, D[1]);
    int64_t sz = sub_coord(p[2], o[2], h, D[2]);
    int64_t code = 0;
    for (int b = 0; b < 2; ++b)
        code |= (((sx >> b) & 1) << (3 * b)) | (((sy >> b) & 1) << (3 * b + 1)) | (((sz >> b) & 1) << (3 * b + 2));
    return code;
}

/* Stable counting sort of the nodes by (cell id (x fastest), sub-cell code):
 * perm[j] = original index of the j-th node in sorted order,
 * cell_start[c] .. cell_start[c+1]-1 = the sorted nodes of cell c, in ascending
 * sub-cell code, then original index. */
int orc_bin(int64_t n, const double *xyz, double h, const double *origin, const int64_t *dims,
            int32_t *perm, int64_t *cell_start)
{
    int64_t ncell = dims[0] * dims[1] * dims[2];
    int64_t nkey = ncell * 64;
    int64_t *cursor = (int64_t *)calloc((size_t)nkey + 1, sizeof(int64_t));
    int64_t *key = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    if (!cursor || !key) { free(cursor); free(key); return ORC_ERR_ARG; }
    for (int64_t i = 0; i < n; ++i) {
        key[i] = cell_of(xyz + 3 * i, origin, h, dims) * 64 + subcell_code(xyz + 3 * i, origin, h, dims);
        cursor[key[i] + 1] += 1;
    }
    for (int64_t c = 0; c < nkey; ++c) cursor[c + 1] += cursor[c];
    for (int64_t c = 0; c <= ncell; ++c) cell_start[c] = cursor[c * 64];
    for (int64_t i = 0; i < n; ++i) perm[cursor[key[i]]++] = (int32_t)i;
    free(cursor);
    free(key);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* neighbour lists                                                          */
/* ------------------------------------------------------------------------ */

/* d^2 = ((dx*dx) + (dy*dy)) + (dz*dz), dx = X.x - p.x, neighbour iff d^2 < h*h */
static int is_nbr(const double *X, const double *p, double hh)
{
    double dx = X[0] - p[0], dy = X[1] - p[1], dz = X[2] - p[2];
    double d2 = ((dx * dx) + (dy * dy)) + (dz * dz);
    return d2 < hh;
}

static int64_t scan_point(const double *X, const double *xyz_sorted, double h, double hh,
                          const double *origin, const int64_t *dims, const int64_t *cell_start,
                          int32_t *out)
{
    int64_t c[3];
    for (int a = 0; a < 3; ++a) c[a] = cell_coord(X[a], origin[a], h, dims[a]);
    int64_t cnt = 0;
    for (int64_t z = c[2] - 1; z <= c[2] + 1; ++z) {
        if (z < 0 || z >= dims[2]) continue;
        for (int64_t y = c[1] - 1; y <= c[1] + 1; ++y) {
            if (y < 0 || y >= dims[1]) continue;
            for (int64_t x = c[0] - 1; x <= c[0] + 1; ++x) {
                if (x < 0 || x >= dims[0]) continue;
                int64_t cell = (z * dims[1] + y) * dims[0] + x;
                for (int64_t j = cell_start[cell]; j < cell_start[cell + 1]; ++j) {
                    if (is_nbr(X, xyz_sorted + 3 * j, hh)) {
                        if (out) out[cnt] = (int32_t)j;
                        ++cnt;
                    }
                }
            }
        }
    }
    return cnt;
}

/* Two-phase: with nbr_id == NULL only nbr_off is filled. Returns the total. */
int64_t orc_neighbors(int64_t q, const double *qxyz, const double *xyz_sorted, double h,
                      const double *origin, const int64_t *dims, const int64_t *cell_start,
                      int64_t *nbr_off, int32_t *nbr_id)
{
    double hh = h * h;
    if (!nbr_id) {
        int64_t *cnt = nbr_off + 1;
#pragma omp parallel for schedule(dynamic, 256)
        for (int64_t i = 0; i < q; ++i)
            cnt[i] = scan_point(qxyz + 3 * i, xyz_sorted, h, hh, origin, dims, cell_start, NULL);
        nbr_off[0] = 0;
        for (int64_t i = 0; i < q; ++i) nbr_off[i + 1] += nbr_off[i];
        return nbr_off[q];
    }
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < q; ++i)
        scan_point(qxyz + 3 * i, xyz_sorted, h, hh, origin, dims, cell_start, nbr_id + nbr_off[i]);
    return nbr_off[q];
}

/* Exhaustive O(QK) search with the same predicate; nodes visited in ascending order. */
int64_t orc_neighbors_brute(int64_t q, const double *qxyz, int64_t n, const double *xyz_sorted,
                            double h, int64_t *nbr_off, int32_t *nbr_id)
{
    double hh = h * h;
    if (!nbr_id) {
#pragma omp parallel for schedule(dynamic, 64)
        for (int64_t i = 0; i < q; ++i) {
            int64_t c = 0;
            for (int64_t j = 0; j < n; ++j) c += is_nbr(qxyz + 3 * i, xyz_sorted + 3 * j, hh);
            nbr_off[i + 1] = c;
        }
        nbr_off[0] = 0;
        for (int64_t i = 0; i < q; ++i) nbr_off[i + 1] += nbr_off[i];
        return nbr_off[q];
    }
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < q; ++i) {
        int64_t c = nbr_off[i];
        for (int64_t j = 0; j < n; ++j)
            if (is_nbr(qxyz + 3 * i, xyz_sorted + 3 * j, hh)) nbr_id[c++] = (int32_t)j;
    }
    return nbr_off[q];
}

/* ------------------------------------------------------------------------ */
/* kernel (raw weight)                                                       */
/* ------------------------------------------------------------------------ */

/* Cubic B-spline of z = |X - p| / h on [0, 1):
 *   W = 2/3 - 4 z^2 + 4 z^3              for z <= 1/2
 *   W = 4/3 - 4 z + 4 z^2 - (4/3) z^3    for 1/2 < z < 1
 * and W'(z)/z, which stays finite at z = 0:
 *   -8 + 12 z                            for z <= 1/2
 *   -4 (1 - z)^2 / z                     for 1/2 < z < 1          */
static void bspline(double z, double *w, double *dw_over_z)
{
    if (z <= 0.5) {
        *w = 2.0 / 3.0 - 4.0 * z * z + 4.0 * z * z * z;
        *dw_over_z = -8.0 + 12.0 * z;
    } else if (z < 1.0) {
        double t = 1.0 - z;
        *w = 4.0 / 3.0 - 4.0 * z + 4.0 * z * z - (4.0 / 3.0) * z * z * z;
        *dw_over_z = -4.0 * t * t / z;
    } else {
        *w = 0.0;
        *dw_over_z = 0.0;
    }
}

/* Gaussian RBF exp(-d^2/r^2) of Sec. 3.2 with r = h/2, truncated at d = h. */
static void gaussian(double d2, double h, double *w, double *dw_over_z_like)
{
    double r = 0.5 * h;
    double e = exp(-d2 / (r * r));
    *w = e;
    /* gradient factor such that grad = factor * (X - p) / h^2 */
    *dw_over_z_like = -2.0 * e * (h * h) / (r * r);
}

/* ------------------------------------------------------------------------ */
/* 4x4 SPD solve                                                             */
/* ------------------------------------------------------------------------ */

static int chol4(double A[4][4], double L[4][4])
{
    double tr = A[0][0] + A[1][1] + A[2][2] + A[3][3];
    memset(L, 0, sizeof(double) * 16);
    for (int j = 0; j < 4; ++j) {
        double d = A[j][j];
        for (int t = 0; t < j; ++t) d -= L[j][t] * L[j][t];
        if (!(d > 1e-14 * tr)) return 0;
        L[j][j] = sqrt(d);
        for (int i = j + 1; i < 4; ++i) {
            double s = A[i][j];
            for (int t = 0; t < j; ++t) s -= L[i][t] * L[j][t];
            L[i][j] = s / L[j][j];
        }
    }
    return 1;
}

static void chol4_solve(double L[4][4], const double *b, double *x)
{
    double y[4];
    for (int i = 0; i < 4; ++i) {
        double s = b[i];
        for (int t = 0; t < i; ++t) s -= L[i][t] * y[t];
        y[i] = s / L[i][i];
    }
    for (int i = 3; i >= 0; --i) {
        double s = y[i];
        for (int t = i + 1; t < 4; ++t) s -= L[t][i] * x[t];
        x[i] = s / L[i][i];
    }
}

/* ------------------------------------------------------------------------ */
/* RKPM shape functions, Sec. 3.2 Eq. (7)-(11)                              */
/* ------------------------------------------------------------------------ */
/*
 * For quadrature point X and neighbour p_k with raw weight wt_k = phi~_k(X):
 *   Eq. (7)  phi_k = wt_k P(p_k)^T C(X)
 *   Eq. (9)  M(X) C(X) = P(X),   Eq. (10)  M(X) = sum_k wt_k P(p_k) P(p_k)^T
 * evaluated in the shifted, scaled basis Ph_k = [1, (p_k - X)/h] (the same
 * phi in exact arithmetic, better conditioned):
 *   Mh = sum_k wt_k Ph_k Ph_k^T,  b = Mh^{-1} e1,  phi_k = wt_k Ph_k^T b.
 * The gradient is the exact derivative of that expression in X:
 *   d_s Ph_k = -e_{s+1}/h
 *   d_s Mh   = sum_k [ d_s wt_k Ph Ph^T + wt_k (d_s Ph Ph^T + Ph d_s Ph^T) ]
 *   d_s b    = -Mh^{-1} (d_s Mh) b
 *   d_s phi_k = d_s wt_k Ph^T b + wt_k (d_s Ph)^T b + wt_k Ph^T d_s b
 * A moment matrix whose Cholesky pivot falls to 1e-14 tr(Mh) or below is
 * reported as singular with the index of the quadrature point.
 */
int orc_rkpm(int64_t q, const double *qxyz, const double *xyz_sorted, const int64_t *nbr_off,
             const int32_t *nbr_id, double h, int kernel, double *phi, double *dphi,
             int64_t *bad_index)
{
    int64_t bad = -1;
#pragma omp parallel for schedule(dynamic, 128)
    for (int64_t i = 0; i < q; ++i) {
        const double *X = qxyz + 3 * i;
        double Mh[4][4] = {{0}}, dM[3][4][4] = {{{0}}};
        for (int64_t e = nbr_off[i]; e < nbr_off[i + 1]; ++e) {
            const double *p = xyz_sorted + 3 * (int64_t)nbr_id[e];
            double r[3] = {X[0] - p[0], X[1] - p[1], X[2] - p[2]};
            double d2 = ((r[0] * r[0]) + (r[1] * r[1])) + (r[2] * r[2]);
            double wt, f;
            if (kernel == 1) gaussian(d2, h, &wt, &f);
            else bspline(sqrt(d2) / h, &wt, &f);
            double g[3];
            for (int s = 0; s < 3; ++s) g[s] = f * r[s] / (h * h);
            double P[4] = {1.0, -r[0] / h, -r[1] / h, -r[2] / h};
            for (int a = 0; a < 4; ++a)
                for (int b2 = 0; b2 < 4; ++b2) Mh[a][b2] += wt * P[a] * P[b2];
            for (int s = 0; s < 3; ++s) {
                double dP[4] = {0.0, 0.0, 0.0, 0.0};
                dP[s + 1] = -1.0 / h;
                for (int a = 0; a < 4; ++a)
                    for (int b2 = 0; b2 < 4; ++b2)
                        dM[s][a][b2] += g[s] * P[a] * P[b2] + wt * (dP[a] * P[b2] + P[a] * dP[b2]);
            }
        }
        double L[4][4];
        if (!chol4(Mh, L)) {
#pragma omp critical
            { if (bad < 0 || i < bad) bad = i; }
            continue;
        }
        double e1[4] = {1.0, 0.0, 0.0, 0.0}, b[4], db[3][4];
        chol4_solve(L, e1, b);
        for (int s = 0; s < 3; ++s) {
            double t[4];
            for (int a = 0; a < 4; ++a) {
                t[a] = 0.0;
                for (int c = 0; c < 4; ++c) t[a] += dM[s][a][c] * b[c];
            }
            chol4_solve(L, t, db[s]);
            for (int a = 0; a < 4; ++a) db[s][a] = -db[s][a];
        }
        for (int64_t e = nbr_off[i]; e < nbr_off[i + 1]; ++e) {
            const double *p = xyz_sorted + 3 * (int64_t)nbr_id[e];
            double r[3] = {X[0] - p[0], X[1] - p[1], X[2] - p[2]};
            double d2 = ((r[0] * r[0]) + (r[1] * r[1])) + (r[2] * r[2]);
            double wt, f;
            if (kernel == 1) gaussian(d2, h, &wt, &f);
            else bspline(sqrt(d2) / h, &wt, &f);
            double P[4] = {1.0, -r[0] / h, -r[1] / h, -r[2] / h};
            double Pb = 0.0;
            for (int a = 0; a < 4; ++a) Pb += P[a] * b[a];
            phi[e] = wt * Pb;
            for (int s = 0; s < 3; ++s) {
                double gs = f * r[s] / (h * h);
                double Pdb = 0.0;
                for (int a = 0; a < 4; ++a) Pdb += P[a] * db[s][a];
                dphi[3 * e + s] = gs * Pb + wt * (-b[s + 1] / h) + wt * Pdb;
            }
        }
    }
    if (bad_index) *bad_index = bad;
    return bad >= 0 ? ORC_ERR_SINGULAR : ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* transpose of the neighbour relation                                       */
/* ------------------------------------------------------------------------ */

/* NT(k) = { i : k in N(i) } in ascending i, with slot[e] = position of k in N(i). */
int orc_transpose(int64_t n, int64_t q, const int64_t *nbr_off, const int32_t *nbr_id,
                  int64_t *nt_off, int32_t *nt_id, int32_t *nt_slot)
{
    memset(nt_off, 0, (size_t)(n + 1) * sizeof(int64_t));
    for (int64_t e = 0; e < nbr_off[q]; ++e) nt_off[nbr_id[e] + 1] += 1;
    for (int64_t k = 0; k < n; ++k) nt_off[k + 1] += nt_off[k];
    int64_t *cur = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    if (!cur) return ORC_ERR_ARG;
    memcpy(cur, nt_off, (size_t)n * sizeof(int64_t));
    for (int64_t i = 0; i < q; ++i)
        for (int64_t e = nbr_off[i]; e < nbr_off[i + 1]; ++e) {
            int64_t k = nbr_id[e];
            nt_id[cur[k]] = (int32_t)i;
            nt_slot[cur[k]] = (int32_t)(e - nbr_off[i]);
            cur[k] += 1;
        }
    free(cur);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* H_w and the RKPM mass matrix                                              */
/* ------------------------------------------------------------------------ */

static int cmp_i32(const void *a, const void *b)
{
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

/*
 * Prop. 1 with the Monte Carlo quadrature of Supp. C:
 *   (H_w)_kl = sum_i v_i (lambda_i + 4 mu_i) grad phi_k(X_i) . grad phi_l(X_i)
 * and the mass matrix of Eq. (14) with the same quadrature:
 *   M_kl = sum_i v_i [rho_i] phi_k(X_i) phi_l(X_i)
 * The sparsity pattern of row k is the structural union of N(i) over
 * i in NT(k) (numeric zeros kept), columns ascending. Every entry is summed
 * over i in ascending order, starting from 0, with
 *   term = (v_i (lambda_i + 4 mu_i)) * (((gk.x gl.x) + (gk.y gl.y)) + (gk.z gl.z)).
 * Two-phase: with col == NULL only row_ptr is filled. Returns nnz.
 */
int64_t orc_assemble(int64_t n, int64_t q, const int64_t *nbr_off, const int32_t *nbr_id,
                     const double *phi, const double *dphi, const double *vol,
                     const double *lam, const double *mu, const double *rho,
                     const int64_t *nt_off, const int32_t *nt_id, const int32_t *nt_slot,
                     int64_t *row_ptr, int32_t *col, double *H, double *M)
{
    int fill = col != NULL;
    if (!fill) row_ptr[0] = 0;
#pragma omp parallel
    {
        int64_t *mark = (int64_t *)malloc((size_t)n * sizeof(int64_t));
        double *accH = (double *)malloc((size_t)n * sizeof(double));
        double *accM = (double *)malloc((size_t)n * sizeof(double));
        int32_t *cols = (int32_t *)malloc((size_t)n * sizeof(int32_t));
        for (int64_t t = 0; t < n; ++t) mark[t] = -1;
#pragma omp for schedule(dynamic, 64)
        for (int64_t k = 0; k < n; ++k) {
            int64_t len = 0;
            for (int64_t e = nt_off[k]; e < nt_off[k + 1]; ++e) {
                int64_t i = nt_id[e];
                int64_t ek = nbr_off[i] + nt_slot[e];
                double wi = vol[i] * (lam[i] + 4.0 * mu[i]);
                double mi = rho ? vol[i] * rho[i] : vol[i];
                const double *gk = dphi + 3 * ek;
                double pk = phi[ek];
                for (int64_t f = nbr_off[i]; f < nbr_off[i + 1]; ++f) {
                    int32_t l = nbr_id[f];
                    if (mark[l] != k) {
                        mark[l] = k;
                        cols[len++] = l;
                        accH[l] = 0.0;
                        accM[l] = 0.0;
                    }
                    if (fill) {
                        const double *gl = dphi + 3 * f;
                        double dot = ((gk[0] * gl[0]) + (gk[1] * gl[1])) + (gk[2] * gl[2]);
                        accH[l] += wi * dot;
                        accM[l] += mi * (pk * phi[f]);
                    }
                }
            }
            if (!fill) {
                row_ptr[k + 1] = len;
            } else {
                qsort(cols, (size_t)len, sizeof(int32_t), cmp_i32);
                int64_t base = row_ptr[k];
                for (int64_t t = 0; t < len; ++t) {
                    col[base + t] = cols[t];
                    H[base + t] = accH[cols[t]];
                    M[base + t] = accM[cols[t]];
                }
            }
        }
        free(mark);
        free(accH);
        free(accM);
        free(cols);
    }
    if (!fill)
        for (int64_t k = 0; k < n; ++k) row_ptr[k + 1] += row_ptr[k];
    return row_ptr[n];
}

/* ------------------------------------------------------------------------ */
/* CSR products and norms                                                    */
/* ------------------------------------------------------------------------ */

/* Y[n][m] = A X[n][m], row-major blocks */
void orc_spmm(int64_t n, const int64_t *row_ptr, const int32_t *col, const double *val,
              int64_t m, const double *X, double *Y)
{
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t r = 0; r < n; ++r) {
        double *y = Y + r * m;
        for (int64_t c = 0; c < m; ++c) y[c] = 0.0;
        for (int64_t e = row_ptr[r]; e < row_ptr[r + 1]; ++e) {
            const double *x = X + (int64_t)col[e] * m;
            double a = val[e];
            for (int64_t c = 0; c < m; ++c) y[c] += a * x[c];
        }
    }
}

/* max_r sum_e |A_re| */
double orc_norm_inf(int64_t n, const int64_t *row_ptr, const double *val)
{
    double best = 0.0;
    for (int64_t r = 0; r < n; ++r) {
        double s = 0.0;
        for (int64_t e = row_ptr[r]; e < row_ptr[r + 1]; ++e) s += fabs(val[e]);
        if (s > best) best = s;
    }
    return best;
}

/* ------------------------------------------------------------------------ */
/* The paper's own construction (Supp. B.1, "RKPM construction"):            */
/* integration points, farthest-point-sampled centres, a Gaussian kernel     */
/* per centre whose radius is the distance to its 2nd-nearest centre.        */
/* ------------------------------------------------------------------------ */

static double dist2(const double *a, const double *b)
{
    double dx = a[0] - b[0], dy = a[1] - b[1], dz = a[2] - b[2];
    return ((dx * dx) + (dy * dy)) + (dz * dz);
}

/* Farthest point sampling: out[0] = start; out[t] = the point whose squared
 * distance to its nearest already chosen point is largest (ties: lowest
 * index). Requires 1 <= K <= q. */
int orc_fps(int64_t q, const double *xyz, int64_t K, int64_t start, int32_t *out)
{
    if (K < 1 || K > q || start < 0 || start >= q) return ORC_ERR_ARG;
    double *md = (double *)malloc((size_t)q * sizeof(double));
    if (!md) return ORC_ERR_ARG;
    for (int64_t i = 0; i < q; ++i) md[i] = INFINITY;
    int64_t last = start;
    out[0] = (int32_t)start;
    for (int64_t t = 1; t < K; ++t) {
        int64_t best = -1;
        double bv = -1.0;
        for (int64_t i = 0; i < q; ++i) {
            double d = dist2(xyz + 3 * i, xyz + 3 * last);
            if (d < md[i]) md[i] = d;
            if (md[i] > bv) { bv = md[i]; best = i; }
        }
        out[t] = (int32_t)best;
        last = best;
    }
    free(md);
    return ORC_OK;
}

/* Per centre: r_k = distance to the 2nd-nearest other centre (the minimal
 * distance that reaches two other centres), and the support radius
 * R_k = cut * r_k of the truncated kernel. Requires K >= 3. */
int orc_radii(int64_t K, const double *c, double cut, double *r, double *R)
{
    if (K < 3) return ORC_ERR_ARG;
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < K; ++k) {
        double d1 = INFINITY, d2 = INFINITY;            /* two smallest squared distances */
        for (int64_t j = 0; j < K; ++j) {
            if (j == k) continue;
            double d = dist2(c + 3 * k, c + 3 * j);
            if (d < d1) { d2 = d1; d1 = d; }
            else if (d < d2) d2 = d;
        }
        r[k] = sqrt(d2);
        R[k] = cut * r[k];
    }
    return ORC_OK;
}

/* Neighbour lists with a support radius per node: N(X) = { k : d^2 < R_k R_k },
 * over the 27 cells around X of the grid of edge h >= max R_k; ascending. */
static int64_t scan_point_var(const double *X, const double *xyz_sorted, const double *R_sorted, double h,
                              const double *origin, const int64_t *dims, const int64_t *cell_start, int32_t *out)
{
    int64_t c[3];
    for (int a = 0; a < 3; ++a) c[a] = cell_coord(X[a], origin[a], h, dims[a]);
    int64_t cnt = 0;
    for (int64_t z = c[2] - 1; z <= c[2] + 1; ++z) {
        if (z < 0 || z >= dims[2]) continue;
        for (int64_t y = c[1] - 1; y <= c[1] + 1; ++y) {
            if (y < 0 || y >= dims[1]) continue;
            for (int64_t x = c[0] - 1; x <= c[0] + 1; ++x) {
                if (x < 0 || x >= dims[0]) continue;
                int64_t cell = (z * dims[1] + y) * dims[0] + x;
                for (int64_t j = cell_start[cell]; j < cell_start[cell + 1]; ++j) {
                    double Rj = R_sorted[j];
                    if (dist2(X, xyz_sorted + 3 * j) < Rj * Rj) {
                        if (out) out[cnt] = (int32_t)j;
                        ++cnt;
                    }
                }
            }
        }
    }
    return cnt;
}

int64_t orc_neighbors_var(int64_t q, const double *qxyz, const double *xyz_sorted, const double *R_sorted,
                          double h, const double *origin, const int64_t *dims, const int64_t *cell_start,
                          int64_t *nbr_off, int32_t *nbr_id)
{
    if (!nbr_id) {
        int64_t *cnt = nbr_off + 1;
#pragma omp parallel for schedule(dynamic, 256)
        for (int64_t i = 0; i < q; ++i)
            cnt[i] = scan_point_var(qxyz + 3 * i, xyz_sorted, R_sorted, h, origin, dims, cell_start, NULL);
        nbr_off[0] = 0;
        for (int64_t i = 0; i < q; ++i) nbr_off[i + 1] += nbr_off[i];
        return nbr_off[q];
    }
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < q; ++i)
        scan_point_var(qxyz + 3 * i, xyz_sorted, R_sorted, h, origin, dims, cell_start, nbr_id + nbr_off[i]);
    return nbr_off[q];
}

/* the same predicate by exhaustive search (pin) */
int64_t orc_neighbors_var_brute(int64_t q, const double *qxyz, int64_t n, const double *xyz_sorted,
                                const double *R_sorted, int64_t *nbr_off, int32_t *nbr_id)
{
    int64_t tot = 0;
    nbr_off[0] = 0;
    for (int64_t i = 0; i < q; ++i) {
        for (int64_t j = 0; j < n; ++j)
            if (dist2(qxyz + 3 * i, xyz_sorted + 3 * j) < R_sorted[j] * R_sorted[j]) {
                if (nbr_id) nbr_id[tot] = (int32_t)j;
                ++tot;
            }
        nbr_off[i + 1] = tot;
    }
    return tot;
}

/* Gaussian exp(-s), s = d^2/r^2 (Sec. 3.2), cut at s = c^2 with the tangent
 * subtracted so that value and slope vanish there:
 *   w(s) = exp(-s) - exp(-c^2) (1 + c^2 - s),   dw/ds = -exp(-s) + exp(-c^2)   (s < c^2)
 * and 0 beyond; grad_X w = dw/ds * 2 (X - p) / r^2. */
static void gauss_cut(double d2, double rk, double cut, double *w, double *g_over_r)
{
    double s = d2 / (rk * rk), c2 = cut * cut;
    if (s < c2) {
        double e = exp(-s), ec = exp(-c2);
        *w = e - ec * (1.0 + c2 - s);
        *g_over_r = (-e + ec) * 2.0 / (rk * rk);    /* grad = g_over_r * (X - p) */
    } else {
        *w = 0.0;
        *g_over_r = 0.0;
    }
}

/* Shape functions on the centres' kernels with three bases (Sec. 3.2, Fig. 3b):
 *   basis 0  plain RBF:               phi_k = w_k
 *   basis 1  partition-of-unity RBF:  phi_k = w_k / sum_j w_j
 *   basis 2  RKPM, linear basis:      Eq. (7)-(11), evaluated as orc_rkpm in the
 *            shifted basis [1, (p_k - X)/h] with h the given scale
 * with exact gradients. r_sorted[k] is centre k's Gaussian radius. A singular
 * moment matrix (basis 2) or an empty kernel sum (basis 1) reports the point. */
int orc_rkpm_var(int64_t q, const double *qxyz, const double *xyz_sorted, const double *r_sorted,
                 const int64_t *nbr_off, const int32_t *nbr_id, double h, double cut, int basis,
                 double *phi, double *dphi, int64_t *bad_index)
{
    int64_t bad = -1;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < q; ++i) {
        const double *X = qxyz + 3 * i;
        double Mh[4][4] = {{0}}, dM[3][4][4] = {{{0}}}, S = 0.0, dS[3] = {0.0, 0.0, 0.0};
        for (int64_t e = nbr_off[i]; e < nbr_off[i + 1]; ++e) {
            int64_t k = nbr_id[e];
            const double *p = xyz_sorted + 3 * k;
            double rv[3] = {X[0] - p[0], X[1] - p[1], X[2] - p[2]};
            double wt, go;
            gauss_cut(dist2(X, p), r_sorted[k], cut, &wt, &go);
            double g[3] = {go * rv[0], go * rv[1], go * rv[2]};
            S += wt;
            for (int s = 0; s < 3; ++s) dS[s] += g[s];
            if (basis == 2) {
                double P[4] = {1.0, -rv[0] / h, -rv[1] / h, -rv[2] / h};
                for (int a = 0; a < 4; ++a)
                    for (int b2 = 0; b2 < 4; ++b2) Mh[a][b2] += wt * P[a] * P[b2];
                for (int s = 0; s < 3; ++s) {
                    double dP[4] = {0.0, 0.0, 0.0, 0.0};
                    dP[s + 1] = -1.0 / h;
                    for (int a = 0; a < 4; ++a)
                        for (int b2 = 0; b2 < 4; ++b2)
                            dM[s][a][b2] += g[s] * P[a] * P[b2] + wt * (dP[a] * P[b2] + P[a] * dP[b2]);
                }
            }
        }
        double L[4][4], b[4] = {0}, db[3][4] = {{0}};
        int ok = 1;
        if (basis == 2) {
            ok = chol4(Mh, L);
            if (ok) {
                double e1[4] = {1.0, 0.0, 0.0, 0.0};
                chol4_solve(L, e1, b);
                for (int s = 0; s < 3; ++s) {
                    double t[4];
                    for (int a = 0; a < 4; ++a) {
                        t[a] = 0.0;
                        for (int c = 0; c < 4; ++c) t[a] += dM[s][a][c] * b[c];
                    }
                    chol4_solve(L, t, db[s]);
                    for (int a = 0; a < 4; ++a) db[s][a] = -db[s][a];
                }
            }
        } else if (basis == 1) {
            ok = S > 0.0;
        }
        if (!ok) {
#pragma omp critical
            { if (bad < 0 || i < bad) bad = i; }
            continue;
        }
        for (int64_t e = nbr_off[i]; e < nbr_off[i + 1]; ++e) {
            int64_t k = nbr_id[e];
            const double *p = xyz_sorted + 3 * k;
            double rv[3] = {X[0] - p[0], X[1] - p[1], X[2] - p[2]};
            double wt, go;
            gauss_cut(dist2(X, p), r_sorted[k], cut, &wt, &go);
            if (basis == 0) {
                phi[e] = wt;
                for (int s = 0; s < 3; ++s) dphi[3 * e + s] = go * rv[s];
            } else if (basis == 1) {
                phi[e] = wt / S;
                for (int s = 0; s < 3; ++s) dphi[3 * e + s] = go * rv[s] / S - wt * dS[s] / (S * S);
            } else {
                double P[4] = {1.0, -rv[0] / h, -rv[1] / h, -rv[2] / h};
                double Pb = 0.0;
                for (int a = 0; a < 4; ++a) Pb += P[a] * b[a];
                phi[e] = wt * Pb;
                for (int s = 0; s < 3; ++s) {
                    double Pdb = 0.0;
                    for (int a = 0; a < 4; ++a) Pdb += P[a] * db[s][a];
                    dphi[3 * e + s] = go * rv[s] * Pb + wt * (-b[s + 1] / h) + wt * Pdb;
                }
            }
        }
    }
    if (bad_index) *bad_index = bad;
    return bad >= 0 ? ORC_ERR_SINGULAR : ORC_OK;
}
