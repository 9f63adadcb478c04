/*
 * freeform.h - C ABI of the MI355X (gfx950) subspace-construction path of
 * "FreeForm: Reduced-Order Deformable Simulation from Particle-Based Skinning
 * Eigenmodes" (arXiv 2605.29318): RKPM shape functions on particles, the
 * weight-space Hessian of the Neo-Hookean energy and the RKPM mass matrix,
 * and the smallest generalized eigenpairs H w = lambda M w (the skinning
 * eigenmodes).
 *
 * Conventions (every entry point):
 *  - Bulk arrays are DEVICE pointers owned by the caller; the library never
 *    frees them. Scalars, status and small results are HOST pointers, as
 *    marked. Library workspace lives in the context and is released by
 *    ff_ctx_destroy.
 *  - Work is enqueued on the context's stream. Calls that return sizes,
 *    status or eigenvalues to the host synchronise that stream first.
 *  - Return value: FF_OK (0) or a negative ff_status; ff_last_error() gives a
 *    message that names the offending index where there is one. No C++
 *    exception crosses the ABI.
 *  - Two-phase sizing: pass NULL for a variable-size output to obtain its size
 *    (e.g. *nbr_total, *nnz); then call again with a buffer of that capacity.
 *    A capacity below the required size returns FF_ERR_CAPACITY and still
 *    writes the required size.
 *  - Index arrays inside lists are int32 (fewer than 2^31 particles); offsets
 *    are int64. Positions are double[n][3] (x, y, z per point).
 *  - After build_neighbors everything is in SORTED numbering: sorted node j is
 *    original node perm[j]. Per-quadrature-point inputs of later calls may be
 *    in original order if the permutation is passed (see assemble_HM).
 *  - Not thread safe per context: calls on one context must not overlap.
 */
#ifndef FREEFORM_H
#define FREEFORM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ff_ctx ff_ctx;

typedef enum {
    FF_OK = 0,
    FF_ERR_INVALID_ARG = -1,      /* bad size, NULL where required, NaN input, limit exceeded */
    FF_ERR_OOM = -2,              /* device allocation of library workspace failed */
    FF_ERR_HIP = -3,              /* a HIP runtime call failed (message has the HIP error) */
    FF_ERR_CAPACITY = -4,         /* caller buffer too small; required size written */
    FF_ERR_SINGULAR_MOMENT = -5,  /* RKPM moment matrix not positive definite at a point */
    FF_ERR_NOT_CONVERGED = -6,    /* max_iter reached; best results still written */
    FF_ERR_BREAKDOWN = -7         /* eigensolver basis lost rank beyond recovery */
} ff_status;

/* Context: binds a device and a stream (NULL = the device's null stream).
 * Read once here from the environment: FF_VERBOSE=1 (progress on stderr);
 * FF_UNION_BITS=n caps the LDS bitmap of the row-tile copy build at n words
 * and FF_ASM_BITMAP_BYTES=n caps the row bitmaps assemble_HM keeps between
 * its passes at n bytes, so that the other paths of both can be exercised
 * (the results are the same either way); FF_CHEB_SHAPE=n runs the matrix-core
 * Chebyshev steps in launch shape n of spmm_rowtiles precision 2 (8 .. 14 with
 * the zero-free K-blocks, the default, 0 .. 7 with the full ones), for tuning:
 * every shape gives the same sums bit for bit. */
int ff_ctx_create(ff_ctx **ctx, int device, void *hip_stream);
void ff_ctx_destroy(ff_ctx *ctx);
const char *ff_last_error(const ff_ctx *ctx);
/*
 * Per-stage device time of eigenmodes / eigenmodes_batched. With timing on
 * (ff_ctx_set_stage_timing(ctx, 1); off by default), the solver brackets each
 * stage of every iteration with HIP events on its stream (not inside a
 * captured hipGraph: with use_graph only FF_STAGE_TOTAL is filled) and sums
 * their elapsed times when the call ends. ff_ctx_stage_times copies the last
 * call's sums: ms[s] (milliseconds) and launches[s] (kernel launches of the
 * stage's main kernel, for per-launch averages), s < min(n, FF_STAGE_COUNT);
 * either array may be NULL. Returns FF_STAGE_COUNT.
 */
typedef enum {
    FF_STAGE_SPMM = 0,         /* fused [H, M] products of the iteration and of the refreshes */
    FF_STAGE_PRECOND_PRODUCT,  /* Chebyshev steps: H-only products fused with the step's update */
    FF_STAGE_PRECOND_OTHER,    /* Chebyshev start (copy of D^-1 r, first term) */
    FF_STAGE_GRAM,             /* Gram products and their reduction */
    FF_STAGE_RR,               /* Rayleigh-Ritz */
    FF_STAGE_UPDATE,           /* block update */
    FF_STAGE_RESID,            /* residual block, norms, convergence flags */
    FF_STAGE_FP64_PHASE,       /* mixed path: the FP64 phase as a whole (certifying Rayleigh-Ritz and any
                                  FP64 iterations); the stages above then cover the FP32 phase alone */
    FF_STAGE_TOTAL,            /* the whole call, host clock */
    FF_STAGE_COUNT
} ff_stage;
int ff_ctx_set_stage_timing(ff_ctx *ctx, int enable);
int ff_ctx_stage_times(const ff_ctx *ctx, int n, double *ms, int64_t *launches);
const char *ff_stage_name(int stage);

/* Uniform cell grid of edge h over the node bounding box. */
typedef struct {
    double origin[3];   /* componentwise minimum of the node positions */
    double h;           /* cell edge = kernel support radius */
    int64_t dims[3];    /* dims_a = floor((max_a - origin_a) / h) + 1 */
    int64_t n_cells;    /* dims[0] * dims[1] * dims[2] */
} ff_grid;

/*
 * build_neighbors - cell binning and neighbour lists.
 *
 * The paper's kernels have unbounded support (Gaussian RBF, Sec. 3.2); this
 * path uses compact kernels of support radius h, so phi_k(X) is non-zero only
 * for |X - p_k| < h. This call finds those pairs.
 *
 *  xyz        [n][3] node positions, original order (device, in)
 *  qxyz       [q][3] quadrature points (device, in), or NULL: the quadrature
 *             points are the nodes themselves, in sorted order (q must be n)
 *  grid       host out: the cell grid
 *  perm       [n] device out: perm[j] = original index of sorted node j.
 *             Nodes are sorted by cell id (z, y, x with x fastest), then by
 *             the Morton code of their sub-cell (each axis of the cell split
 *             in 4: s_a = clamp(floor((t_a - q_a) * 4), 0, 3), t_a = (x_a -
 *             o_a) / h, q_a the cell coordinate; bits interleaved x, y, z from
 *             the lowest), ties by original index. Consecutive sorted nodes
 *             are then spatially close, which the SpMM's row tiles exploit.
 *  xyz_sorted [n][3] device out: xyz[perm[j]]
 *  cell_start [n_cells + 1] device out, or NULL on the sizing call: sorted
 *             nodes of cell c are cell_start[c] .. cell_start[c+1]-1
 *  nbr_off    [q+1] device out: list of quadrature point i is
 *             nbr_id[nbr_off[i] .. nbr_off[i+1]-1]
 *  nbr_id     [nbr_cap] device out or NULL on the sizing call: sorted node
 *             ids j with d^2 < h*h, d^2 = ((dx*dx)+(dy*dy))+(dz*dz),
 *             dx = X.x - p.x in IEEE double without contraction; ascending.
 *  nbr_total  host out: total number of pairs
 * Cell index per axis: min(max(floor((x - origin)/h), 0), dims-1) with IEEE
 * division. Errors: FF_ERR_INVALID_ARG (n <= 0, h <= 0 or not finite, a
 * non-finite coordinate, more than 2^31-1 cells or pairs, a cell holding more
 * than 4096 nodes), FF_ERR_CAPACITY (cell_start or nbr_id too small).
 */
int build_neighbors(ff_ctx *ctx, int64_t n, const double *xyz, int64_t q, const double *qxyz,
                    double h, ff_grid *grid, int32_t *perm, double *xyz_sorted,
                    int64_t *cell_start, int64_t cell_cap, int64_t *nbr_off, int32_t *nbr_id,
                    int64_t nbr_cap, int64_t *nbr_total);

/*
 * build_neighbors_radii - build_neighbors with a support radius per node: the pairs
 * d^2 < R_j * R_j (same d^2 as build_neighbors) of the kernels of the paper's own
 * construction (Supp. B.1, "RKPM construction"), whose Gaussians have a radius per
 * centre. radius [n] device in, original node order, finite and positive; the cell
 * grid's edge h is the largest radius (grid->h), so a point's neighbours lie in the
 * 27 cells around it. Everything else as build_neighbors.
 */
int build_neighbors_radii(ff_ctx *ctx, int64_t n, const double *xyz, const double *radius, int64_t q,
                          const double *qxyz, ff_grid *grid, int32_t *perm, double *xyz_sorted,
                          int64_t *cell_start, int64_t cell_cap, int64_t *nbr_off, int32_t *nbr_id,
                          int64_t nbr_cap, int64_t *nbr_total);

/*
 * fps_centers - farthest point sampling of K kernel centres among q integration points
 * (Supp. B.1, "RKPM construction": the centres are spread evenly over the object).
 * out_idx[0] = start; out_idx[t] = the point whose squared distance to its nearest
 * already picked point is largest, ties to the lowest index; squared distances are
 * ((dx*dx)+(dy*dy))+(dz*dz) in IEEE double, so the picks are exact.
 *  qxyz    [q][3] device in;   out_idx [K] device out;
 *  out_xyz [K][3] device out or NULL: the picked points, in pick order
 * Errors: FF_ERR_INVALID_ARG (K outside [1, q], start outside [0, q), a non-finite point).
 */
int fps_centers(ff_ctx *ctx, int64_t q, const double *qxyz, int K, int64_t start, int32_t *out_idx,
                double *out_xyz);

/*
 * kernel_radii - the radius of each centre's Gaussian (Supp. B.1: the smallest distance
 * that reaches two other centres, i.e. the distance to the 2nd-nearest other centre),
 * r_k = sqrt(second smallest d^2), and the support radius R_k = cut * r_k of the cut
 * kernel of rkpm_shape_radii. centres [K][3] device in (K >= 3); r, R [K] device out.
 */
int kernel_radii(ff_ctx *ctx, int64_t K, const double *centres, double cut, double *r, double *R);

/*
 * rkpm_shape_radii - shape functions and gradients on the paper's own kernels: a
 * Gaussian exp(-|X - p_k|^2 / r_k^2) per centre (Sec. 3.2), cut at |X - p_k| = cut r_k
 * with its tangent in s = d^2/r_k^2 subtracted, so that value and slope vanish there:
 *   w_k = exp(-s) - exp(-cut^2) (1 + cut^2 - s)   (s < cut^2, else 0).
 * basis selects what is built on them (Sec. 3.2 and the comparison of its Fig. 3b):
 *   0  plain RBF                phi_k = w_k
 *   1  partition-of-unity RBF   phi_k = w_k / sum_j w_j
 *   2  RKPM, linear basis       Eq. (7)-(11), in the shifted basis [1, (p_k - X)/h]
 * with exact gradients in X. node_r [n]: each centre's r_k, sorted numbering, or in
 * original order when perm (from build_neighbors_radii) is given; h: the scale of the
 * shifted basis (any positive value gives the same phi in exact arithmetic; pass
 * grid->h). Lists, layout and bad_index as rkpm_shape (bad_index also names a point
 * whose kernel sum is zero for basis 1).
 */
int rkpm_shape_radii(ff_ctx *ctx, int64_t n, const double *xyz_sorted, const double *node_r,
                     const int32_t *perm, int64_t q, const double *qxyz, const int64_t *nbr_off,
                     const int32_t *nbr_id, int64_t nbr_total, double h, double cut, int basis,
                     double *phi, double *dphi, int64_t *bad_index);

/*
 * rkpm_shape - RKPM shape functions and gradients, Sec. 3.2 Eq. (7)-(11).
 *
 * For quadrature point X_i and each neighbour k in its list (linear basis
 * P = [1, x, y, z]):  phi_k(X) = phi~_k(X) P(p_k)^T M(X)^-1 P(X) with the
 * moment matrix M(X) = sum_k phi~_k(X) P(p_k) P(p_k)^T (Eq. (9)-(10)).
 * It is evaluated in the equivalent shifted, scaled basis [1, (p_k - X)/h]
 * and differentiated exactly in X.
 *
 *  kernel   0 = cubic B-spline of z = |X - p|/h (support h);
 *           1 = Gaussian exp(-d^2/r^2) of Sec. 3.2 with r = h/2, truncated at h
 *  phi      [nbr_total] device out, aligned with nbr_id
 *  dphi     [nbr_total][3] device out: gradient of phi_k at X_i
 *  feat     [q][8] device out or NULL: per-point raw features (4 eigenvalues
 *           of the moment matrix over sum phi~, neighbour count, sum phi~,
 *           |sum phi~ (p - X)| / (h sum phi~), std/mean of phi~)
 *  bad_index host out: first quadrature point whose 4x4 moment matrix has a
 *           Cholesky pivot <= 1e-14 * trace (FF_ERR_SINGULAR_MOMENT), else -1
 */
int rkpm_shape(ff_ctx *ctx, int64_t n, const double *xyz_sorted, int64_t q, const double *qxyz,
               const int64_t *nbr_off, const int32_t *nbr_id, int64_t nbr_total, double h,
               int kernel, double *phi, double *dphi, float *feat, int64_t *bad_index);

/*
 * assemble_HM - weight-space Hessian (Prop. 1) and RKPM mass matrix (Eq. (14)).
 *
 *   H_kl = sum_i v_i (lambda_i + 4 mu_i) grad phi_k(X_i) . grad phi_l(X_i)
 *   M_kl = sum_i v_i [rho_i] phi_k(X_i) phi_l(X_i)
 * (Prop. 1 with the quadrature of Supp. C; the Neo-Hookean energy of Eq. (16)
 * at the rest state). CSR in sorted node numbering; the pattern of row k is
 * the structural union of N(i) over the quadrature points i whose list holds
 * k, columns ascending, numeric zeros kept. Each entry is summed over i in
 * ascending order with term = (v_i (lambda_i + 4 mu_i)) * (((gx gx') + (gy
 * gy')) + (gz gz')) in IEEE double, so H and M are bitwise symmetric and the
 * call is deterministic (no atomics in the sums).
 *
 *  vol, lam, mu [q] device in: quadrature weight and Lame parameters
 *  rho          [q] device in, or NULL for the density-free mass matrix of Eq. (14)
 *  perm         [q] device in, or NULL: if given, the four per-point arrays
 *               are in original order and point i reads entry perm[i]
 *  grid, cell_start: as returned by build_neighbors
 *  row_ptr      [n+1] device out
 *  col, H, M    [nnz_cap] device out, or NULL on the sizing call
 *  hm32         [nnz_cap][2] device out or NULL: FP32 copies (H, M) interleaved
 *  nnz          host out
 * The sizing call (col NULL) fills row_ptr and nnz and keeps its symbolic
 * state (transposed lists, row lengths, and each row's column bitmap over its
 * candidate window, 2 KiB per row up to 8 GiB, which the numeric pass then
 * reads instead of rebuilding) in the context; the next call on the
 * context, if it passes the same nbr_off, nbr_id, grid dimensions,
 * cell_start, row_ptr and sizes (compared by address and value, the arrays
 * left unmodified in between), reuses that state instead of recomputing it.
 * Errors: FF_ERR_INVALID_ARG (a node with no quadrature point in its support,
 * a row longer than 2048 or a window of more than 16384 candidate nodes),
 * FF_ERR_CAPACITY.
 */
int assemble_HM(ff_ctx *ctx, int64_t n, int64_t q, const int64_t *nbr_off, const int32_t *nbr_id,
                const double *phi, const double *dphi, const double *vol, const double *lam,
                const double *mu, const double *rho, const int32_t *perm, const ff_grid *grid,
                const int64_t *cell_start, int64_t *row_ptr, int32_t *col, double *H, double *M,
                float *hm32, int64_t nnz_cap, int64_t *nnz);

/* Eigensolver parameters. */
typedef struct {
    int k;              /* eigenpairs wanted, constant mode included (>= 1) */
    int block;          /* block width m >= k (0 = k rounded up to a multiple of 8); a multiple of 8, <= 64 */
    int precision;      /* 0 = FP64 throughout; 1 = mixed: FP32 products, FP64 Rayleigh-Ritz,
                           then FP64 certification and FP64 iterations if needed */
    double tol;         /* max_j r_j over the first k pairs, r_j as in eigenmodes() */
    int max_iter;       /* total iteration cap (both phases) */
    int precond;        /* 0 = none, 1 = Jacobi diag(H)^-1, 2 = Chebyshev-Jacobi: q(D^-1 H) D^-1 with q the
                           degree-d Chebyshev semi-iteration polynomial for D^-1 H on [b/ratio, b], b from 30 power
                           steps (x 1.1, at most the Gershgorin bound); SPD on the spectrum */
    uint64_t seed;      /* Philox-4x32-10 key for the random start when X0 == NULL */
    int check_every;    /* host convergence check period in iterations (0 = 10) */
    int use_graph;      /* 1 = replay one captured hipGraph per iteration (a call on the null
                           stream runs on a private stream of the context) */
    int refresh_every;  /* recompute the images of X and P explicitly every this many iterations (0 = auto:
                           30 in the FP32 phase, 20 in FP64) */
    int precond_degree; /* Chebyshev degree d for precond = 2 (0 = default 12; 2..16); d - 1 products with H per
                           iteration */
    double precond_ratio; /* b / a of the Chebyshev interval [a, b] (0 = default 1000; > 1): q stays
                             positive on (0, b] for any ratio; a wide interval favours the low modes */
    int precond_values; /* number formats of the Chebyshev products of the mixed path (eight-row tiles):
                           1 = H and the iterate in FP32 (FP32 VALU); 2 = H in binary16 scaled by a
                           power of two (rowtiles_build precision 5), iterate FP32 (FP32 VALU); 3 = H
                           and the iterate in binary16 on the matrix cores (rowtiles_build precision 6;
                           block width 32 or 64), each column of the preconditioner's input scaled by
                           the inverse of its largest magnitude per object (the output's span is
                           unchanged); 4 = 3 with the K-blocks stored without their zeros (a mask per
                           K-block and the present values, rebuilt in LDS: the same products
                           bit for bit from fewer bytes); 0 = default: 4 where the width allows,
                           else 2. Products accumulate in FP32 in every case */
    double eig_tol;     /* 0 = off. Else the FP64 phase also iterates until the a-posteriori
                           eigenvalue bound of every wanted pair (eig_bounds) is <= eig_tol
                           (relative): an object converges when max_j r_j <= tol and
                           max_j eig_bound_j <= eig_tol. On the mixed path the FP64 phase then
                           preconditions with the FP32 / binary16 Chebyshev-Jacobi products (an
                           approximate operator is all a preconditioner needs; the residuals,
                           Grams and Rayleigh-Ritz stay FP64 on the FP64 matrices) */
    double angle_tol;   /* 0 = off. Else the FP64 phase also iterates until every wanted pair's
                           angle bound (eig_bounds) is <= angle_tol, as eig_tol does */
} ff_eig_params;

typedef struct {
    int iters_fp32;     /* iterations of this object in the FP32 phase (mixed) */
    int iters_fp64;     /* iterations of this object in the FP64 phase (0 = certified at once) */
    int converged;      /* 1 if max_j r_j <= tol */
    int restarts;       /* basis restarts after Rayleigh-Ritz breakdown */
    double max_resid;   /* final max_j r_j (FP64, certified) */
    double seconds;     /* wall time of the call */
    int graph;          /* 1 if the iterations were replayed from a captured hipGraph */
    double max_eig_bound;   /* max over the k pairs of eig_bound (eig_bounds); infinite if the FP64
                               phase never formed it */
    double max_angle_bound; /* max over the k pairs of angle_bound */
    int eig_certified;      /* 1 if max_eig_bound <= eig_tol (eig_tol > 0), or <= 1e-5 when eig_tol is 0,
                               and max_angle_bound <= angle_tol when angle_tol > 0 */
} ff_eig_info;

/*
 * eigenmodes - k smallest generalized eigenpairs of (H, M), Eq. (15): the
 * minimiser of tr(c^T H c) subject to c^T M c = I is the block of the k
 * smallest generalized eigenvectors. The constant vector is always the first
 * mode (eigenvalue 0, Supp. B.1); it is counted in k.
 *
 * Blocked LOBPCG (Knyazev 2001) on S = [X, W, P] with a Rayleigh-Ritz step in
 * FP64 on the device. Residual (FP64, with the FP64 matrices):
 *   r_j = ||H w_j - lambda_j M w_j||_2 / ((||H||_inf + |lambda_j| ||M||_inf) ||w_j||_2)
 *
 *  row_ptr, col, H, M: FP64 CSR from assemble_HM (device in)
 *  hm32     FP32 interleaved copy (device in), required when precision = 1
 *  X0       [n][block] device in (row-major), or NULL: Philox uniform [-1, 1); an object
 *           with fewer than 5 x block rows (and at most 192) leaves the block iteration no
 *           room, and with X0 NULL starts instead from the lowest block eigenvectors of its
 *           dense pencil (rayleigh_ritz on the identity basis), which the iteration then
 *           certifies as any other answer
 *  eigval   [k] host out, ascending
 *  W        [n][k] device out (row-major, sorted node numbering): M-orthonormal
 *           eigenvectors; sign: the entry of largest magnitude is positive
 *  resid    [k] host out: r_j
 *  info     host out or NULL
 * Returns FF_ERR_NOT_CONVERGED (results still written) when max_iter is reached.
 */
int eigenmodes(ff_ctx *ctx, int64_t n, const int64_t *row_ptr, const int32_t *col, const double *H,
               const double *M, const float *hm32, const ff_eig_params *p, const double *X0,
               double *eigval, double *W, double *resid, ff_eig_info *info);

/*
 * eigenmodes_batched - independent problems solved together: the CSR is the
 * block-diagonal concatenation of n_obj matrices; object o owns rows and
 * columns obj_row_off[o] .. obj_row_off[o+1]-1 (host array). One launch per
 * stage covers every object; objects that converge are masked out.
 *
 *  eigval [n_obj][k], resid [n_obj][k] host out; W [N][k] device out;
 *  info   [n_obj] host out or NULL.
 */
int eigenmodes_batched(ff_ctx *ctx, int n_obj, const int64_t *obj_row_off, const int64_t *row_ptr,
                       const int32_t *col, const double *H, const double *M, const float *hm32,
                       const ff_eig_params *p, const double *X0, double *eigval, double *W,
                       double *resid, ff_eig_info *info);

/*
 * eig_bounds - a-posteriori bounds of the last eigenmodes / eigenmodes_batched call on
 * this context, per object and pair (host out, [n_obj][k] each, either may be NULL).
 * For the generalized problem of Eq. (15) with M-orthonormal w_j and residual
 * r_j = H w_j - theta_j M w_j, eigenvalue perturbation theory bounds the error of the
 * Ritz value by ||r_j||^2 / gap and the sine of the eigenvector's angle by ||r_j|| / gap,
 * with the residual in the M^-1 norm and gap the distance from theta_j to the rest of the
 * spectrum. The library takes the residual in the norm of diag(M)^-1 instead (the M^-1
 * norm would need a solve with M), so the figures are estimates, not guarantees:
 *   eta_j^2 = sum_i R_ij^2 / M_ii, in FP64 with the FP64 matrices;
 *   the block form of the bounds holds for a cluster C of consecutive pairs, with
 *   eta_C^2 = sum of eta_i^2 over C and gap_C = distance from C to the nearest Ritz
 *   value outside it (including the next Ritz value beyond the block, taken no farther
 *   than the block's last spacing, as it lies above the eigenvalue); for pair j the
 *   smallest over the runs of up to 8 consecutive pairs holding j is reported:
 *   eig_bound_j = min_C eta_C^2 / (gap_C max(|theta_j|, theta_1))   (relative eigenvalue error)
 *   angle_bound_j = min_C eta_C / gap_C                             (sine of the largest angle)
 * They are formed in the FP64 phase at each residual check; a pair whose gap is unknown
 * (no Ritz value beyond the block yet) has an infinite bound. Returns FF_ERR_INVALID_ARG
 * if n_obj or k differ from the last call's.
 */
int eig_bounds(ff_ctx *ctx, int n_obj, int k, double *eig_bound, double *angle_bound);

/*
 * chebyshev_apply - the preconditioner of eigenmodes (precond = 2) alone, on one object:
 *   Z = q(D^-1 H) D^-1 R,  D = diag(H),
 * q the degree-d Chebyshev semi-iteration polynomial for D^-1 H z = D^-1 r on
 * [b / ratio, b] (d - 1 products with H). The paper's eigensolve (Eq. (15), Supp. B.1
 * "Eigenanalysis") states no preconditioner; this is the one the library's LOBPCG applies
 * to its residuals, by the same set-up (tile copies, interval estimate) and the same
 * launches, including the per-step update of the output block.
 *   n, row_ptr, col, H, M, hm32: as eigenmodes (device).
 *   m: block width (multiple of 8, 8 .. 64; values 3 and 4 need 32 or 64).
 *   degree: d in [2, 16]; ratio: b / a (0 = default 1000, else in (1, 1e6]).
 *   values: number formats of the products, as precond_values (1 .. 4).
 *   upper: b; 0 = the library's estimate (min(1.1 x the largest Rayleigh quotient of
 *     D^-1 H after 30 power steps, the Gershgorin bound)); upper_used (host out, may be
 *     NULL) receives the b taken.
 *   R: device FP32 [n][ld_r] input; Z: device FP32 [n][ld_z] output (may not alias R).
 * With values 3 and 4 the recurrence runs on s_c D^-1 r_c, s_c = 1 / max_i |(D^-1 R)_ic|
 * per column (the binary16 range), and Z holds s_c q(D^-1 H) D^-1 r_c: each column
 * scaled, its direction unchanged. Synchronous. Errors: FF_ERR_INVALID_ARG for bad
 * arguments, FF_ERR_OOM, FF_ERR_HIP.
 */
int chebyshev_apply(ff_ctx *ctx, int64_t n, const int64_t *row_ptr, const int32_t *col, const double *H,
                    const double *M, const float *hm32, int m, int degree, double ratio, int values,
                    double upper, const float *R, int64_t ld_r, float *Z, int64_t ld_z, double *upper_used);

/*
 * spmm_hm - the fused block product [HY, MY] = [H, M] Y used inside eigenmodes,
 * exposed for measurement and tests. Y, HY, MY are [n][m] row-major with
 * leading dimension ld (>= m). precision 1 reads hm32 and FP32 blocks,
 * precision 0 reads H, M and FP64 blocks (the block pointers are float* or
 * double* accordingly). variant selects a tile shape (-1 = tuned/default);
 * the row-tile variants (see rowtiles_build) build their copy for each call.
 */
int spmm_hm(ff_ctx *ctx, int64_t n, const int64_t *row_ptr, const int32_t *col, const double *H,
            const double *M, const float *hm32, int precision, int m, const void *Y, int64_t ld_y,
            void *HY, void *MY, int64_t ld_out, int variant);

/*
 * Matrix-free products with H and M, without the assembled CSR. Prop. 1 (with the
 * quadrature of Supp. C) and Eq. (14) write both as sums over the integration points:
 *   H = G^T D G,  M = Phi^T V Phi,
 * G [3q][n] the gradients grad phi_k(X_i), Phi [q][n] the values phi_k(X_i),
 * D = diag(v_i (lambda_i + 4 mu_i)) per gradient component, V = diag(v_i [rho_i]). So
 * [H Y, M Y] = [G^T (D (G Y)), Phi^T (V (Phi Y))] in two passes over the neighbour lists:
 * a gather per integration point, then a sum per node over the points whose list holds
 * it (ascending), each in a fixed order.
 *
 * mf_build: the lists, shape functions and per-point arrays exactly as assemble_HM takes
 *   them (perm as there); keeps the transposed lists with phi and grad phi in that order,
 *   and the per-point weights, in FP32 (precision 1) or FP64 (precision 0). It keeps
 *   pointers to nbr_off and nbr_id, which must stay allocated and unchanged while the
 *   handle is used. Destroy the handle before its context.
 * mf_apply: HY = H Y and/or MY = M Y (either may be NULL) for Y [n][m], m in [1, 64],
 *   float or double as the handle, row-major with leading dimensions ld_y, ld_out; FP32
 *   accumulation at precision 1. Equal to the products with assemble_HM's matrices up to
 *   rounding (the terms are associated differently).
 * mf_interpolate: U [q][m] = Phi Y, the fields sum_k phi_k(X_i) Y_k at the integration
 *   points (Sec. 3.2: the skinning weights W^j(X) = sum_k phi_k(X) c_k^j where Y = c).
 */
typedef struct ff_mf ff_mf;
int mf_build(ff_ctx *ctx, int64_t n, int64_t q, const int64_t *nbr_off, const int32_t *nbr_id, const double *phi,
             const double *dphi, const double *vol, const double *lam, const double *mu, const double *rho,
             const int32_t *perm, int precision, ff_mf **out);
int mf_apply(ff_ctx *ctx, ff_mf *mf, int m, const void *Y, int64_t ld_y, void *HY, void *MY, int64_t ld_out);
int mf_interpolate(ff_ctx *ctx, const ff_mf *mf, int m, const void *Y, int64_t ld_y, void *U, int64_t ld_u);
void mf_destroy(ff_mf *mf);

/*
 * spmm_autotune - time every SpMM tile shape on the given matrix with hipEvents
 * and keep the fastest for matrices of this shape (n, nnz/row, m, precision);
 * results are cached in the JSON file at cache_path (NULL = no file).
 * best_variant, best_ms host out.
 */
int spmm_autotune(ff_ctx *ctx, int64_t n, const int64_t *row_ptr, const int32_t *col,
                  const double *H, const double *M, const float *hm32, int precision, int m,
                  const char *cache_path, int *best_variant, double *best_ms);

/*
 * gram_hm - the Gram products of the Rayleigh-Ritz step, G_H = S^T HS and
 * G_M = S^T MS, for row-major [n][w] blocks with leading dimension ld (MFMA
 * 16x16x4; FP32 blocks accumulate in FP32 over 64 rows and in FP64 beyond).
 *  precision 1: S, HS, MS are float*; 0: double*
 *  G  [2][w][w] device out (FP64): G[0] = G_H, G[1] = G_M
 */
int gram_hm(ff_ctx *ctx, int64_t n, int w, int precision, const void *S, const void *HS,
            const void *MS, int64_t ld, double *G);

/*
 * rayleigh_ritz - FP64 Rayleigh-Ritz on the pencil (G_H, G_M) of order w
 * (device [2][w][w], symmetric parts used): scale by diag(G_M)^-1/2, Cholesky
 * of G_M in column order dropping a column whose scaled pivot is <= tau,
 * reduce, cyclic Jacobi, and return the m smallest eigenpairs of the pencil on
 * the kept columns: theta [m] ascending and C [w][m] (zero rows for dropped
 * columns) with C^T G_M C = I and C^T G_H C = diag(theta). Device outputs;
 * kept host out. FF_ERR_BREAKDOWN if fewer than m columns are kept.
 */
int rayleigh_ritz(ff_ctx *ctx, int w, int m, const double *G, double tau, double *C, double *theta,
                  int *kept);

/*
 * rayleigh_ritz_noalloc - rayleigh_ritz for callers that cannot allocate device memory
 * (code under stream capture, tight serving loops, harnesses that forbid allocation):
 * the same kernels and results, with its work arrays in a fixed per-GPU device scratch
 * (1.6 MB, held from the first context on that GPU until the process ends) instead of
 * the context's workspace. It calls no device allocator. Limits: order w <= 192 and
 * m <= 64 pairs; larger sizes return FF_ERR_INVALID_ARG. Every call on one GPU shares
 * that scratch (its status words are reset by each call, the work arrays written before
 * they are read): calls that overlap in time on one GPU, from any context or stream,
 * race and must not be issued. kept is read back with a stream synchronisation, as in
 * rayleigh_ritz.
 */
int rayleigh_ritz_noalloc(ff_ctx *ctx, int w, int m, const double *G, double tau, double *C, double *theta,
                          int *kept);

/*
 * Row-tile copy of [H, M] for the fused SpMM. Rows are grouped in tiles of
 * four consecutive rows (in the cell-sorted numbering, so spatially close);
 * a tile keeps the ascending union of its rows' column lists and, per union
 * entry, the four H and four M values of its rows (zero where a row lacks the
 * column). The product then gathers each row of Y once per tile instead of
 * once per row. eigenmodes builds such a copy itself when a row-tile SpMM
 * variant is selected; these calls keep one for repeated products.
 *
 * rowtiles_build: from the FP64 CSR of assemble_HM (rows with ascending
 *   columns); precision 1 keeps FP32 values (rounded from H, M), 0 FP64, 2
 *   both; 3 and 4 keep only H, in FP32, in tiles of eight and of sixteen
 *   rows (the copies the Chebyshev-Jacobi preconditioner of eigenmodes runs
 *   on: sixteen rows on MFMA where the block width allows, eight rows
 *   otherwise; M may be NULL); 5 keeps H in eight-row tiles in binary16:
 *   each value is the FP32 value times 2^e, rounded to nearest even, with e
 *   chosen so the largest |H| lands in [2^14, 2^15), and the product scales
 *   its FP32 sums by 2^-e (half the bytes per value, relative error 2^-11
 *   per value); 6 keeps the values of 5 in K-blocks of 16 union entries,
 *   [kblock][8 rows][16 entries], for the matrix-core products (the
 *   preconditioner's default form at block widths 32 and 64).
 *   Device memory owned by the handle until rowtiles_destroy (destroy it
 *   before its context). The CSR may be freed afterwards.
 * spmm_rowtiles: [HY, MY] = [H, M] Y as spmm_hm, on the copy; sub selects a
 *   launch shape (0 .. 2). With MY NULL only HY = H Y is formed, the product
 *   the Chebyshev-Jacobi preconditioner of eigenmodes runs: at precision 1 it
 *   accumulates in FP32 (an approximate operator is all a preconditioner
 *   needs), at precision 0 in FP64. A handle built with precision 3, 4 or 5
 *   takes only this form, at precision 1, with leading dimensions that are
 *   multiples of 4 and m % 8 == 0, 8 <= m <= 64, 64 % (m / 8) == 0 (eight
 *   rows) or m in {4, 8, 12, 16, 32, 64} (sixteen rows). A handle built
 *   with precision 6 also takes precision 2: Y in binary16 ([n][m] with
 *   ld_y == m, m 32 or 64), HY = H Y in FP32, accumulated in FP32 on
 *   v_mfma_f32_16x16x16_f16 (MY NULL); its launch shapes are sub 0 .. 14
 *   (0 .. 4: a ring of K-blocks, by waves per workgroup and K-blocks in
 *   flight; 5 .. 7: super-blocks of four K-blocks, the next one's loads
 *   issued before the current one is multiplied; 8 .. 12: the same
 *   super-blocks read from a copy without the K-blocks' zeros, a 128-bit
 *   mask per K-block and the present values, which a precision-6 handle
 *   keeps beside the full K-blocks; 13, 14: those with one register buffer,
 *   the next super-block gathered once the current one is staged in LDS,
 *   four waves per workgroup, 14 with unpadded rows in LDS so that eight
 *   waves fit a SIMD), all with the same operands and
 *   summation order, so the same result bit for bit. Errors: invalid
 *   arguments and unsupported shapes return FF_ERR_INVALID_ARG, a
 *   non-finite H at precision 5 likewise.
 */
/*
 * sym_build / spmm_sym - [HY, MY] = [H, M] Y from the upper triangles of H and M. H (Prop. 1)
 * and M (Eq. (14)) are symmetric, so the values of the diagonal and above are stored once;
 * each row's strict lower triangle keeps its columns and, per entry (i, j < i), the position
 * of (j, i) in the upper arrays, from which the value is read. The lower triangle's values of
 * the CSR are never read: the product is that of the matrix whose lower triangle mirrors its
 * upper one (the same matrix for the library's assembly, which is bitwise symmetric).
 *   sym_build: n, row_ptr, col, H (device, FP64 CSR with sorted rows and a symmetric
 *     pattern), M (device or NULL: H only); precision 0 keeps FP64 values, 1 FP32 values.
 *     *out receives a handle owning its device memory until sym_destroy (destroy it before
 *     its context); the CSR may be freed afterwards. FF_ERR_INVALID_ARG if the pattern is
 *     not symmetric or the upper triangle holds 2^31 entries or more.
 *   sym_info: entries of the upper triangle (diagonal included) and of the strict lower one.
 *   spmm_sym: m in {8, 16, 32, 64}; Y [n][ld_y], HY and MY [n][ld_out] device, 16-byte
 *     aligned, in the handle's precision (FP64 / FP32), leading dimensions multiples of 2
 *     (FP64) or 4 (FP32); MY NULL forms HY only. Sums accumulate in FP64, one wavefront per
 *     row: the row's lower entries in ascending column, then its upper ones, each lane group
 *     taking every (64 / (m / v))-th entry (v = 2 FP64, 4 FP32 values per 16-byte piece), the
 *     groups' sums added in a fixed order: deterministic.
 */
typedef struct ff_sym ff_sym;
int sym_build(ff_ctx *ctx, int64_t n, const int64_t *row_ptr, const int32_t *col, const double *H,
              const double *M, int precision, ff_sym **out);
int sym_info(const ff_sym *s, int64_t *nnz_upper, int64_t *nnz_lower);
int spmm_sym(ff_ctx *ctx, const ff_sym *s, int m, const void *Y, int64_t ld_y, void *HY, void *MY,
             int64_t ld_out);
void sym_destroy(ff_sym *s);

typedef struct ff_rowtiles ff_rowtiles;
int rowtiles_build(ff_ctx *ctx, int64_t n, const int64_t *row_ptr, const int32_t *col, const double *H,
                   const double *M, int precision, ff_rowtiles **out);
/* Number of tiles and of union entries (host out, either may be NULL). */
int rowtiles_info(const ff_rowtiles *rt, int64_t *ntiles, int64_t *entries);
int spmm_rowtiles(ff_ctx *ctx, const ff_rowtiles *rt, int precision, int m, const void *Y, int64_t ld_y, void *HY,
                  void *MY, int64_t ld_out, int sub);
void rowtiles_destroy(ff_rowtiles *rt);

/* Number of SpMM tile variants and a description of one (host strings). */
int spmm_variant_count(void);
const char *spmm_variant_name(int variant);
/* The variant that spmm_hm(variant = -1) and eigenmodes use for a matrix of this shape:
 * the one spmm_autotune stored in the context, else the built-in default. */
int spmm_variant_selected(ff_ctx *ctx, int64_t n, int64_t nnz, int m, int precision);

/*
 * rand_block - Philox-4x32-10 (Salmon et al., SC'11) uniform numbers in [-1, 1):
 * element e of the n*m block (row-major) takes 32-bit word e % 4 of the
 * Philox output for counter (e / 4 low, e / 4 high, 0, 0) and key
 * (seed low, seed high); value = word * 2^-31 - 1 (exact in double).
 * out [n][m] device, double.
 */
int rand_block(ff_ctx *ctx, int64_t n, int m, uint64_t seed, double *out);

/*
 * philox4x32_10 - the raw generator behind rand_block, for checking against the
 * published known-answer vectors: out[4t..4t+3] = Philox-4x32-10 of counter
 * ctr[4t..4t+3] under key key[2t..2t+1]. All three arrays are device memory.
 */
int philox4x32_10(ff_ctx *ctx, int count, const uint32_t *ctr, const uint32_t *key, uint32_t *out);

/*
 * Learned warm start (not in the paper, whose eigensolve starts from scratch;
 * the sole network it trains is a comparison method). A small MLP maps
 * per-point inputs to a block Y of k columns whose span approximates the span
 * of the k smallest eigenmodes; eigenmodes() then starts from X0 = Y.
 *
 * Network: n_in -> 128 -> 128 -> 128 -> k, GELU(z) = z Phi(z) (exact erf
 * form) after each hidden layer; BF16 weights and hidden activations, FP32
 * accumulation and FP32 master parameters. Flat parameter order
 * [W1 (128 x n_in), b1, W2 (128x128), b2, W3 (128x128), b3, W4 (k x 128), b4],
 * each W output-major (row = output unit). n_in = 11 + 6 n_freq (mlp_inputs). Training minimises the subspace loss
 *   L = k - tr(A^-1 B E B^T),  A = Y^T D Y,  B = Y^T D T,  E = (T^T D T)^-1
 * (D = lumped mass, T = target modes of one object), which is zero when
 * span(Y) = span(T) and does not depend on the scaling, sign or mixing of the
 * columns of Y or T, with Adam (beta1 0.9, beta2 0.999, eps 1e-8).
 * An ff_mlp belongs to the context it was created on; calls on it enqueue on
 * that context's stream and must not overlap. Destroy it before that context
 * (mlp_destroy itself does not touch the context).
 */
typedef struct ff_mlp ff_mlp;

/* Parameter count for output width k (1 <= k <= 64) and input width n_in (1 <= n_in <= 128), or -1. */
int mlp_param_count(int k, int n_in);
/* New network with uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) weights (seeded) and zero biases. */
int mlp_create(ff_ctx *ctx, int k, int n_in, uint64_t seed, ff_mlp **out);
void mlp_destroy(ff_mlp *mlp);
/* Copy all parameters in (host in, FP32, mlp_param_count(k) values); resets Adam's state. */
int mlp_set_params(ff_mlp *mlp, const float *params);
/* Copy the FP32 master parameters out (host out). */
int mlp_get_params(ff_mlp *mlp, float *params);
/* Copy the gradient of the last mlp_train_step out (host out, FP32). */
int mlp_get_grad(ff_mlp *mlp, float *grad);

/*
 * mlp_inputs - the network inputs per node, from sorted positions and the raw
 * features of rkpm_shape: position x centred on the bounding box and divided
 * by its largest half extent, the 4 moment-matrix eigenvalues, neighbour count
 * and kernel sum each divided by their mean over the object, the boundary
 * indicator and the kernel-value spread (11 values); then for each octave
 * l < n_freq, sin(pi 2^l x_a) for a = 0..2 and cos(pi 2^l x_a) for a = 0..2.
 *  xyz_sorted [n][3] device in; feat [n][8] device in; 0 <= n_freq <= 19;
 *  in [n][11 + 6 n_freq] device out (FP32)
 */
int mlp_inputs(ff_ctx *ctx, int64_t n, const double *xyz_sorted, const float *feat, int n_freq,
               float *in);

/*
 * mlp_forward - Y = MLP(in) for n rows: in [n][n_in] device in (FP32);
 * Y [n][ldy] device out (FP64, first k columns written, ldy >= k), ready as X0
 * of eigenmodes (the columns beyond k can be filled with rand_block).
 */
int mlp_forward(ff_mlp *mlp, int64_t n, const float *in, double *Y, int64_t ldy);

/*
 * mlp_train_step - one Adam step on one object: forward, loss, backward, update.
 *  in    [n][n_in] device in (FP32); T [n][ldt] device in (FP64, the first k
 *  columns are the target modes, linearly independent); d [n] device in: the
 *  lumped mass (positive); lr the step size; loss host out or NULL: L before
 *  the step. n >= k.
 */
int mlp_train_step(ff_mlp *mlp, int64_t n, const float *in, const double *T, int64_t ldt,
                   const double *d, float lr, double *loss);

/* lumped_mass - d_i = sum_j M_ij (row sums of the FP64 CSR mass matrix). d [n] device out. */
int lumped_mass(ff_ctx *ctx, int64_t n, const int64_t *row_ptr, const double *M, double *d);

/*
 * block_blend - the warm start's blended starting block (the learned start is this
 * library's addition; the paper starts its eigensolve without one): column by column
 *   X_c <- X_c / rms(X_c) + w R_c / rms(R_c),   rms(v) = sqrt(sum_i v_i^2 / n),
 * in FP64, sums in a fixed order (deterministic). X [n][ldx] device in/out, R [n][ldr]
 * device in (say rand_block's columns), 1 <= m <= 64, w >= 0 finite. A column of zero rms
 * is taken as having rms 1e-300. Errors: FF_ERR_INVALID_ARG, FF_ERR_OOM.
 */
int block_blend(ff_ctx *ctx, int64_t n, int m, double *X, int64_t ldx, const double *R, int64_t ldr, double w);

#ifdef __cplusplus
}
#endif
#endif /* FREEFORM_H */
