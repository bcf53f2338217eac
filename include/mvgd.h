/*
 * mvgd.h -- C ABI of the MI355X (gfx950) implementation of the Modified Virtual Grid Difference
 * (MVGD) discretisation of the Laplace-Beltrami operator on point clouds
 * (M. Wang, S. Leung, H. Zhao, arXiv:1603.04100).
 *
 * Given a point cloud S = {p_i} sampling a d-dimensional manifold in R^n, mvgd_assemble builds,
 * for every point, one row of a sparse matrix L whose entries are the weights of the point and its
 * K nearest neighbours, so that (L U)_i approximates the Laplace-Beltrami operator of U at p_i
 * (Sec. 2, problem statement and the assembled matrix A; Sec. 3.1, the MVGD). mvgd_apply computes
 * y = L x. All work runs in HIP kernels on the device; the host only validates arguments, sizes
 * the buffers and enqueues work.
 *
 * Conventions shared by every entry point:
 *  - Plain pointers and sizes only. Device buffers are device-resident memory (hipMalloc,
 *    hipMallocAsync or a framework allocator); `stream` is a hipStream_t passed as void*, NULL for
 *    the null stream. Work is stream-ordered: a call returns after enqueuing its kernels, except
 *    where stated. The caller keeps inputs alive and unmodified until the stream has finished
 *    the work that reads them.
 *  - No call aborts the process. Every failure is reported by the return code; on failure no
 *    handle is returned and nothing leaks. mvgd_last_error() gives a human-readable reason for the
 *    most recent failure on the calling thread.
 *  - Sign: L approximates +Delta (negative diagonal, rows summing to zero).
 *  - Rows whose neighbourhood is degenerate (spacing h not positive and finite, or a rank-deficient
 *    least-squares design: min |R_kk| < 1e-6 max |R_kk|) keep their columns and get zero values;
 *    they are counted in mvgd_info_t.n_degenerate.
 */
#ifndef MVGD_H
#define MVGD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mvgd_matrix mvgd_matrix; /* opaque; owns the assembled matrix on one device */

typedef enum {
    MVGD_OK = 0,
    MVGD_EINVAL = -1,      /* invalid argument (also: non-finite input coordinates) */
    MVGD_ENOMEM = -2,      /* device or host allocation failed */
    MVGD_EDEVICE = -3,     /* no usable device, or a HIP runtime error */
    MVGD_EUNSUPPORTED = -4 /* valid for the method but not implemented on the GPU path */
} mvgd_status;

typedef enum {
    MVGD_FP64 = 0,       /* points, weights and apply in double */
    MVGD_FP32_MIXED = 1  /* points, weights and apply vectors in float; frame, covariance
                            accumulation, least-squares solves and metric in double */
} mvgd_precision;

enum {
    MVGD_FLAG_LS = 1u << 0,         /* plain least-squares discretisation (Sec. 2): derivatives
                                       of the fitted quadratic at p_i, no centre modification */
    MVGD_FLAG_H_OVERRIDE = 1u << 1, /* use params.h_override as the grid spacing of every row */
    MVGD_FLAG_KEEP_DIAG = 1u << 2,  /* keep per-row h and status bits for mvgd_row_diag */
    MVGD_FLAG_TIME = 1u << 3,       /* record HIP events around the kernel groups of assemble
                                       and apply on the caller's stream (see mvgd_timing) */
    MVGD_FLAG_MLS = 1u << 4,        /* weighted least squares in both fits: weight 1 at p_i and
                                       1/K at every neighbour (the moving-least-squares weights
                                       of the comparison method, Sec. 4); with MVGD_FLAG_LS this
                                       is that method, without it the MVGD rows on those fits */
    MVGD_FLAG_DIVERGENCE = 1u << 5  /* curves only (d = 1), not with MVGD_FLAG_LS: the
                                       divergence form of Eq. divergence instead of Eq. center */
};

typedef struct {
    int32_t n_ambient;  /* n: 3 or 4 for surfaces, 2 or 3 for curves */
    int32_t d_manifold; /* d: 2 (surfaces) or 1 (curves) */
    int32_t k;          /* K nearest neighbours: 5 <= K <= 63 for surfaces, 2 <= K <= 63 for
                           curves, and K < points in every cloud */
    int32_t precision;  /* mvgd_precision */
    uint32_t flags;     /* MVGD_FLAG_* */
    double h_override;  /* > 0, used only with MVGD_FLAG_H_OVERRIDE */
    /* Neighbour-search tuning (performance only: results do not depend on it). 0 selects the
     * built-in default. Values come from the autotuner (paper_1603_04100_amd/autotune.py). */
    float cell_alpha;      /* grid cell edge / estimated K-th neighbour distance (0.6)        */
    float radius_mu;       /* initial search radius / estimated K-th neighbour distance (1.7) */
    float cells_per_point; /* cell-table entries budgeted per point (8)                       */
    int32_t launch;        /* MVGD_LAUNCH_*                                                   */
    int32_t search;        /* MVGD_SEARCH_*                                                   */
} mvgd_params;

enum {
    MVGD_LAUNCH_DEFAULT = 0,
    MVGD_LAUNCH_GRID = 1,      /* one workgroup per 64-point group, XCD-aware order */
    MVGD_LAUNCH_PERSISTENT = 2 /* resident workgroups popping groups from per-XCD queues */
};

enum {
    MVGD_SEARCH_DEFAULT = 0, /* TILE */
    MVGD_SEARCH_GROUP = 1, /* the 64 queries of a group stream their common cell box via LDS */
    MVGD_SEARCH_LANE = 2,  /* every query walks the cells of its own box */
    MVGD_SEARCH_TILE = 3   /* as GROUP, with the 64 x 64 query-candidate squared distances of each
                              staged chunk formed on the matrix cores (FP32 operands from the
                              centred coordinates; the selection stays exact in both precisions) */
};

typedef struct {
    int64_t n_rows;        /* rows = points over all clouds */
    int32_t n_clouds;
    int32_t k;
    int64_t nnz;           /* n_rows * (k + 1) */
    int32_t precision;     /* mvgd_precision */
    int32_t n_ambient;
    int64_t n_degenerate;  /* rows with zero values (see above) */
    int64_t n_slow_knn;    /* rows whose neighbour search took the exhaustive fallback
                              (exact ties or extreme clustering); informational */
    size_t device_bytes;   /* device memory held by the handle */
    int64_t n_subgroups;   /* neighbour-search sub-groups (ranges of 64-point groups) */
    int64_t n_streamed;    /* candidate points streamed through the search, all passes */
    int64_t n_growths;     /* search-radius growths (a sub-group's radius was too small) */
} mvgd_info_t;

/*
 * mvgd_assemble -- build L for one point cloud or a batch of clouds.
 *
 * Method (per point, Sec. 2 and Sec. 3.1): the K nearest neighbours N(i) in ambient Euclidean
 * distance (ties to the smaller index); covariance of N(i) about its barycentre and its
 * eigenvectors (PCA frame, the smallest eigenvalue's vectors are the normals); local coordinates
 * of p_j - p_i; spacing h = 1/4 min over the tangent axes of the coordinate range over N(i)
 * (Eq. DefH); least-squares quadratic fits over {p_i} u N(i) of each normal coordinate
 * (Eq. poly) and of U (Eq. T); metric of the fitted graph (Eq. metric) giving the coefficients of
 * Eq. eqn3; central differences on the virtual grid of spacing h with U_i at the centre node
 * (Eq. centered1 and its higher-dimensional form). Curves (d = 1): one tangent axis, monomials
 * (1, xi, xi^2), h from Eq. DefH, Eq. LB1 with Eq. center, or Eq. divergence with
 * MVGD_FLAG_DIVERGENCE.
 *
 * points        device, row-major [n_total, n_ambient]; float for MVGD_FP32_MIXED, double for
 *               MVGD_FP64. Must be finite (non-finite values give MVGD_EINVAL).
 * n_total       total number of points over all clouds (< 2^31).
 * cloud_offsets HOST array int64[n_clouds + 1], offsets[0] = 0, strictly increasing,
 *               offsets[n_clouds] = n_total; NULL means one cloud. Clouds are independent:
 *               neighbours are searched inside each cloud only.
 * n_clouds      >= 1 (ignored when cloud_offsets is NULL).
 * p             parameters (see mvgd_params).
 * stream        hipStream_t as void*.
 * out           receives the handle on MVGD_OK, NULL otherwise.
 *
 * Synchronisation: the bounding boxes, the cell grids (planned on the device from the boxes)
 * and the binning are enqueued first; the call then waits for `stream` once, so that it can reject
 * non-finite input synchronously before the neighbour search. The search and the stencils are
 * enqueued on `stream` and the call returns without waiting for them. The handle may be used on
 * `stream` at once, or on another stream after the caller has ordered that stream after `stream`.
 */
mvgd_status mvgd_assemble(const void *points, int64_t n_total, const int64_t *cloud_offsets,
                          int32_t n_clouds, const mvgd_params *p, void *stream,
                          mvgd_matrix **out);

/*
 * mvgd_apply -- y = L x (Sec. 2: each row is a linear combination of the point's and its
 * neighbours' values), for nrhs right-hand sides at once.
 *
 * x, y  device, row-major [n_rows, nrhs], element type of the matrix (float for FP32-mixed,
 *       double for FP64); rows are the caller's point order. y is overwritten; x and y must not
 *       overlap. Sums accumulate in double.
 * nrhs  1 <= nrhs <= 64.
 * The handle keeps a staging buffer for the permuted x; calls on the same handle must be ordered
 * (same stream, or ordered by the caller).
 */
mvgd_status mvgd_apply(mvgd_matrix *L, const void *x, void *y, int32_t nrhs, void *stream);

/*
 * mvgd_free -- release the handle and its device memory. Stream-ordered on the stream of the last
 * assemble/apply/export call on this handle; NULL is accepted.
 */
void mvgd_free(mvgd_matrix *L);

/*
 * mvgd_csr -- write L in CSR form into caller-provided device buffers, in the caller's point order
 * (Sec. 2, the assembled matrix): row i holds columns {i} u N(i) in ascending order with their
 * weights, explicit zeros kept. Columns are local to each cloud (0-based within the cloud);
 * row_ptr is global over the batch, row_ptr[i] = i * (K + 1).
 *
 * row_ptr int64[n_rows + 1], col int32[nnz], val float|double[nnz] (matrix element type).
 * Any of the three may be NULL to skip it. Stream-ordered.
 */
mvgd_status mvgd_csr(mvgd_matrix *L, int64_t *row_ptr, int32_t *col, void *val, void *stream);

/*
 * mvgd_row_diag -- per-row diagnostics in the caller's point order, into caller device buffers:
 * h (double[n_rows], the virtual grid spacing of Eq. DefH) and status (uint8[n_rows]: bit 0
 * degenerate, bit 1 exhaustive neighbour-search fallback). Needs MVGD_FLAG_KEEP_DIAG at assembly,
 * otherwise MVGD_EINVAL. Either pointer may be NULL. Stream-ordered.
 */
mvgd_status mvgd_row_diag(mvgd_matrix *L, double *h, uint8_t *status, void *stream);

typedef struct {
    float bin_ms;      /* assemble: bounding boxes, grid plan, cell keys, scan, placement, the
                          one synchronisation */
    float assemble_ms; /* assemble: neighbour search + fit and stencil (search_ms + fit_ms) */
    float apply_ms;    /* last mvgd_apply: permutation of x + ELL SpMV */
    int32_t have_apply;
    float search_ms;   /* assemble: the neighbour-search kernel */
    float fit_ms;      /* assemble: the fit + stencil kernel */
} mvgd_timing_t;

/* mvgd_timing -- device durations measured with HIP events on the stream each call was enqueued
 * on; needs MVGD_FLAG_TIME at assembly, otherwise MVGD_EINVAL. Waits for the handle's last
 * recorded event only (work enqueued on the stream after it is not waited for). */
mvgd_status mvgd_timing(mvgd_matrix *L, mvgd_timing_t *t);

/* mvgd_info -- sizes and counters; waits for the handle's stream (synchronous). */
mvgd_status mvgd_info(mvgd_matrix *L, mvgd_info_t *info);

/*
 * mvgd_row_stats -- sign statistics of the rows of L (Sec. 3.2: the centre modification is
 * meant to give off-diagonal entries the sign opposite to the negative diagonal, so that -L is
 * an M-matrix; plain least-squares rows have entries of mixed sign).
 *
 * Per row, with d the diagonal weight and o_j the off-diagonal weights in ascending column
 * order, each promoted to double: neg_mass = sum_j max(0, -o_j) (one addition per entry, in
 * that order); ratio = neg_mass / |d| (NaN where d == 0; a row summing to zero is diagonally
 * dominant exactly when its ratio is 0); an M-row has d < 0 and every o_j >= 0.
 *
 * ratio  device double[n_rows] in the caller's point order, or NULL.
 * out    host; filled after the work on `stream` has finished (the call waits for it).
 * The mean is over rows with d != 0, reduced in a fixed order (run-to-run reproducible).
 */
typedef struct {
    int64_t n_rows;
    int64_t n_diag_negative;    /* rows with d < 0 */
    int64_t n_m_rows;           /* rows with d < 0 and every off-diagonal weight >= 0 */
    int64_t n_offdiag_negative; /* off-diagonal weights < 0, over all rows */
    int64_t n_zero_diagonal;    /* rows with d == 0 (degenerate rows) */
    double mean_ratio;
    double max_ratio;
} mvgd_row_stats_t;

mvgd_status mvgd_row_stats(mvgd_matrix *L, double *ratio, mvgd_row_stats_t *out, void *stream);

/*
 * mvgd_solve -- iterative solution of (sigma I - L) x = b on the device (Sec. 4: the linear
 * systems of the discretised Laplace-Beltrami equation, e.g. -Delta U = f with sigma = 0, and
 * screened / implicit-diffusion systems with sigma > 0).
 *
 * Methods: BiCGSTAB (L is not symmetric), and damped Jacobi x += omega D^-1 (b - A x) with
 * D = diag(A), the smoother the M-matrix property of the MVGD rows is meant to make convergent.
 * With pin_first = 1 the first point of every cloud gets the identity row x_p = b_p (on closed
 * manifolds L 1 = 0, so sigma = 0 is singular without it; put the wanted value at b_p). A
 * Dirichlet condition on an open surface (Sec. 3.1: the condition is enforced at the boundary
 * points, MVGD rows everywhere else) is the same identity row at every point flagged in
 * `fixed`, with the boundary value in b.
 *
 * b      device, [n_rows] in the caller's order, the matrix dtype.
 * x      device, [n_rows], the matrix dtype; in: initial guess, out: the last iterate.
 * info   host; filled when the call returns (the call waits for `stream`).
 * All iteration vectors and scalars are double and live on the device in the matrix's cell
 * order; the host reads the residual once every check_every iterations. Inner products are
 * reduced in a fixed order, so results are reproducible run to run.
 * BiCGSTAB's recursively updated residual can drift from b - A x over long runs: when it passes
 * the test, the true residual of the iterate is formed, and if that one does not pass, the
 * iteration restarts from the iterate (at most four restarts, within max_iter in all).
 * Returns MVGD_OK also when the iteration does not converge (see info->converged).
 */
enum { MVGD_SOLVE_BICGSTAB = 0, MVGD_SOLVE_JACOBI = 1 };

typedef struct {
    int32_t method;      /* MVGD_SOLVE_* */
    int32_t max_iter;    /* >= 0 */
    double rtol;         /* stop once ||r||_2 <= rtol ||b||_2 (the iteration's own residual) */
    double sigma;        /* A = sigma I - L (finite) */
    double omega;        /* Jacobi damping in (0, 2); 0 selects 2/3 */
    int32_t pin_first;   /* 1: identity row at the first point of every cloud */
    int32_t check_every; /* iterations enqueued between host residual checks; 0 selects 16 */
    const uint8_t *fixed; /* device [n_rows] in the caller's order, nonzero = identity row
                             (Dirichlet points); NULL for none */
} mvgd_solve_params;

typedef struct {
    int32_t iterations;   /* iterations (Jacobi: sweeps) performed */
    int32_t converged;    /* 1: residual test passed (BiCGSTAB: by the true residual of the
                             returned x), 0: max_iter reached or restarts used up, -1: breakdown */
    double rel_residual;  /* ||b - A x||_2 / ||b||_2 of the returned x, recomputed */
} mvgd_solve_info;

mvgd_status mvgd_solve(mvgd_matrix *L, const void *b, void *x, const mvgd_solve_params *p,
                       mvgd_solve_info *info, void *stream);

/*
 * mvgd_assemble_neumann -- L for an open surface in R^3 with the homogeneous Neumann condition,
 * imposed by reflection (Sec. 3.1).
 *
 * The cloud is split into interior points P^I (boundary[i] == 0) and boundary points P^B. An
 * interior point that has a boundary point among its K nearest neighbours (in the whole cloud)
 * gets a ghost point: its mirror image across the boundary, p^R = p - 2 ((p - p^B) . e3) e3, with
 * p^B its closest boundary point (ties to the smaller index) and e3 = e1 x e2 / |e1 x e2| there;
 * e1 is the tangent at p^B of the boundary curve, fitted by quadratic least squares (in the PCA
 * frame of the k_boundary nearest boundary points, p^B included) and e2 the surface normal (the
 * smallest-eigenvalue eigenvector of the covariance of the K nearest points of the whole cloud).
 * All of this is computed in double. MVGD rows (mvgd_assemble) are then built on the augmented
 * cloud P^I u P^R, and every ghost column is folded into its source's column (a zero normal
 * derivative gives the ghost its source's value). Boundary points carry no row.
 *
 * Rows of the returned handle: [0, n_interior) the interior points, in ascending order of their
 * index in `points`; [n_interior, n_interior + n_ghost) the ghosts, whose rows are zero (fix them
 * in mvgd_solve, or solve with sigma != 0). Interior rows reference interior columns only; a
 * column that a fold duplicates is merged into one entry, which leaves a zero entry whose column
 * is the row itself.
 *
 * points      device, [n_total, 3], float (MVGD_FP32_MIXED) or double (MVGD_FP64). One cloud.
 * boundary    device, uint8 [n_total], nonzero = boundary point.
 * k_boundary  boundary points in the curve fit, 3..16 (at most the number of boundary points).
 * p           as for mvgd_assemble, with n_ambient = 3 and d_manifold = 2.
 * ghost_xyz   device double [n_total * 3] or NULL: the ghost points in FP64, row-major, ghost g at
 *             [3g, 3g + 3) (g = its row - n_interior).
 * ghost_src   device int32 [n_total]: the source of ghost g as an interior row.
 * info        host: n_interior and n_ghost.
 * The call waits for `stream` twice (the assembly's own wait, and once to size the ghost set).
 * MVGD_EINVAL when there are fewer boundary points than k_boundary or at most k interior points.
 */
typedef struct {
    int64_t n_interior;
    int64_t n_ghost;
} mvgd_neumann_info;

mvgd_status mvgd_assemble_neumann(const void *points, int64_t n_total, const uint8_t *boundary,
                                  int32_t k_boundary, const mvgd_params *p, void *stream,
                                  mvgd_matrix **out, double *ghost_xyz, int32_t *ghost_src,
                                  mvgd_neumann_info *info);

/*
 * mvgd_eigs -- the nev eigenvalues of -L with the smallest real parts (Sec. 4: -Delta nu = lambda
 * nu; on the unit sphere lambda = l (l + 1) with multiplicity 2 l + 1).
 *
 * Method: Chebyshev-filtered subspace iteration on a block of m vectors (double, the matrix's cell
 * order). Each iteration applies p(A), A = -L, a Chebyshev polynomial of the given degree that is
 * bounded on [a, b] and grows below a (b: the largest absolute row sum of L, a Gershgorin bound;
 * a: the largest Ritz value of the block), with one multi-column ELL product per degree; then
 * orthonormalises the block (Cholesky QR, twice) and takes the eigenvalues of V^T A V (m x m,
 * Hessenberg reduction and the double-shift QR iteration on the host) as Ritz values. L is not
 * symmetric, so Ritz values may come in complex conjugate pairs; both parts are returned.
 * Rows flagged in `fixed` are removed from the operator (the iteration runs on the submatrix of
 * the other rows and columns): Dirichlet points, or the ghost rows of mvgd_assemble_neumann.
 *
 * lambda_re, lambda_im  host [nev], sorted by real part (then imaginary part).
 * info                  host; the call waits for `stream` a few times per iteration.
 * MVGD_EINVAL for parameters out of range or a matrix with at most m rows; MVGD_EDEVICE if the
 * block loses rank or the small QR iteration fails. Returns MVGD_OK also when the iteration
 * stops at max_iter (info->converged = 0).
 */
typedef struct {
    int32_t nev;          /* eigenvalues wanted, 1..64 */
    int32_t block;        /* subspace size m, nev..64; 0 selects min(64, max(nev + 8, 2 nev)) */
    int32_t degree;       /* filter degree per iteration, 0..1000; 0: per iteration
                             2 sqrt((b - a) / (a - a0)) in [8, 500] (a0: the smallest Ritz value
                             or 0), a growth of about e^4 from a to the bottom of the spectrum */
    int32_t max_iter;     /* filter iterations; 0 selects 500 */
    double tol;           /* converged when the nev Ritz values move by at most tol max(1, |lambda|)
                             in two consecutive iterations; 0 selects 1e-10 */
    const uint8_t *fixed; /* device [n_rows] in the caller's order, nonzero = removed; NULL: none */
    uint64_t seed;        /* start block (counter-based random numbers) */
} mvgd_eigs_params;

typedef struct {
    int32_t iterations;
    int32_t converged;     /* 1: the test passed, 0: max_iter reached */
    int32_t block;         /* m used */
    int32_t degree;        /* degree of the last iteration */
    double spectrum_bound; /* b / 1.01 */
    double max_change;     /* the last iteration's largest relative Ritz value change */
} mvgd_eigs_info;

mvgd_status mvgd_eigs(mvgd_matrix *L, const mvgd_eigs_params *p, double *lambda_re,
                      double *lambda_im, mvgd_eigs_info *info, void *stream);

/* mvgd_dense_eigvals -- eigenvalues of a real m x m matrix (host, row-major), the small dense step
 * of mvgd_eigs (Householder reduction to Hessenberg form, then the implicitly double-shifted QR
 * iteration). re, im: host [m], unordered. Host only, no device involved. MVGD_EINVAL on bad
 * arguments or when the iteration does not converge. */
mvgd_status mvgd_dense_eigvals(int32_t m, const double *a, double *re, double *im);

/* mvgd_pool_trim -- device memory of the current device that the library keeps cached. Handles
 * and assembly scratch come from a stream-ordered pool owned by the library, one per device; freed
 * memory stays in the pool for later calls (no fresh mapping per assembly). This call returns the
 * unused part of the current device's pool to the system, keeping at most keep_bytes (0: all of
 * it). Memory of live handles is never released. MVGD_EDEVICE if the pool cannot be created or
 * trimmed. */
mvgd_status mvgd_pool_trim(size_t keep_bytes);

/* Human-readable name of a status code (static string). */
const char *mvgd_status_str(mvgd_status s);

/* Reason for the most recent failure on the calling thread (static thread-local buffer). */
const char *mvgd_last_error(void);

/* Library version as major * 10000 + minor * 100 + patch. */
int32_t mvgd_version(void);

#ifdef __cplusplus
}
#endif

#endif /* MVGD_H */
