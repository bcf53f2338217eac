/*
 * mvgd_oracle.c -- plain FP64 CPU reference of the Modified Virtual Grid Difference (MVGD)
 * discretisation of the Laplace-Beltrami operator on point clouds
 * (M. Wang, S. Leung, H. Zhao, arXiv:1603.04100).
 *
 * TEST INFRASTRUCTURE ONLY. This file is the oracle that the GPU path is checked against. It is
 * called only by tests, by the smoke check and by the benchmark's CPU-baseline leg. It shares no
 * code, header, table or helper with the GPU library, and the GPU library never calls it.
 *
 * Everything is IEEE double, compiled with -ffp-contract=off (no fused multiply-add), one row
 * at a time, in the order the paper states the steps:
 *
 *   O1  K nearest neighbours of p_i, Euclidean in the ambient space (Sec. 2).
 *       key(i,j) = ((d0*d0 + d1*d1) + d2*d2) + d3*d3 with d = p_j - p_i, evaluated left to
 *       right; ties go to the smaller index j; j = i is excluded.
 *   O2  barycentre c_i and covariance C_i over N(i) (Sec. 2), computed from d_j = p_j - p_i.
 *   O3  eigenvectors of C_i by cyclic Jacobi, eigenvalues sorted descending; the first d are the
 *       tangent axes, the rest the normal axes (the smallest one approximates the normal).
 *   O4  local coordinates u_j (tangent) and z_j (normal) of p_j - p_i; origin at p_i.
 *   O5  virtual-grid spacing h = 1/4 min over tangent axes of (max - min) of u over N(i)
 *       (Eq. DefH and its two-dimensional form).
 *   O6  design matrix V over {p_i} u N(i): monomials of degree <= 2 in (u/h) (Sec. 2, the
 *       normal equations A b = U with A_11 = K + 1). Scaling by h is a reparametrisation.
 *   O7  least-squares quadratic fit of every normal coordinate (Eq. poly) by Householder QR.
 *   O8  metric of the fitted graph (Eq. metric) and the coefficients of Eq. eqn3:
 *       Delta U = G11 U_xx + 2 G12 U_xy + G22 U_yy - q . grad U with G = g^-1,
 *       g = I + sum_c grad z_c grad z_c^T, q = sum_c tr(G H_c) G grad z_c (Christoffel terms of
 *       a graph). For d = 1 this is Eq. LB1.
 *   O9  virtual-grid central differences on the LS fit of U with U_i at the centre node
 *       (Eq. centered1 and its higher-dimensional form): U_x = b10, U_xy = b11,
 *       U_xx = 2 b20 + 2 (b00 - U_i)/h^2, U_yy = 2 b02 + 2 (b00 - U_i)/h^2.
 *       So L_i U = ell^T b - tau U_i, tau = 2 (G11 + G22)/h^2,
 *       ell = (tau, -q1, -q2, 2 G11, 2 G12, 2 G22) on b = (b00, b10, b01, b20, b11, b02).
 *       The plain least-squares variant (Sec. 2) uses ell with tau = 0 and no centre term.
 *       Curves (d = 1) also have the divergence form (Eq. divergence): the flux
 *       (1/sqrt g) U_x differenced at +-h/2, with g = 1 + |y'|^2 of the fitted curve.
 *   O10 weights w = V (V^T V)^-1 D ell, D = diag of the h scaling, then w_centre -= tau.
 *       Weighted least squares (the moving-least-squares comparison of Sec. 4, weight 1 at p_i
 *       and w at every neighbour; w = 1/K there): both fits minimise sum_r w_r (residual_r)^2,
 *       i.e. V and the data are scaled row-wise by sqrt(w_r) before the QR, and the row becomes
 *       W V (V^T W V)^-1 D ell. w = 1 is the unweighted fit.
 *   O11 the row: columns {i} u N(i) ascending, explicit zeros kept.
 *   O12 apply: y_i = sum_j L_ij x_j in column order.
 *
 * Degenerate rows (h not positive and finite, or min|R_kk| < 1e-6 max|R_kk| in the QR of V)
 * keep their columns and get all-zero values.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_MAX_N 4
#define ORACLE_MAX_M 6
#define ORACLE_RCOND 1e-6
enum { ODIAG = 64 };

/* --------------------------------------------------------------------------------------- */
/* O1: brute-force k nearest neighbours                                                     */
/* --------------------------------------------------------------------------------------- */
static double knn_key(const double *a, const double *b, int n)
{
    double s = 0.0;
    for (int k = 0; k < n; ++k) {
        double d = b[k] - a[k];
        double sq = d * d;
        s = (k == 0) ? sq : s + sq;
    }
    return s;
}

static int key_less(double ka, int64_t ia, double kb, int64_t ib)
{
    return ka < kb || (ka == kb && ia < ib);
}

/* K nearest of row i, ascending by (key, index). */
static void knn_row(const double *P, int64_t N, int n, int64_t i, int K, int64_t *idx, double *key)
{
    int cnt = 0;
    const double *pi = P + i * n;
    for (int64_t j = 0; j < N; ++j) {
        if (j == i)
            continue;
        double kj = knn_key(pi, P + j * n, n);
        if (cnt == K && !key_less(kj, j, key[K - 1], idx[K - 1]))
            continue;
        int pos = (cnt < K) ? cnt++ : K - 1;
        while (pos > 0 && key_less(kj, j, key[pos - 1], idx[pos - 1])) {
            key[pos] = key[pos - 1];
            idx[pos] = idx[pos - 1];
            --pos;
        }
        key[pos] = kj;
        idx[pos] = j;
    }
}

/* --------------------------------------------------------------------------------------- */
/* O3: cyclic Jacobi eigen-decomposition of a symmetric n x n matrix (n <= 4)               */
/* --------------------------------------------------------------------------------------- */
static void jacobi_eig(int n, double A[ORACLE_MAX_N][ORACLE_MAX_N], double lam[ORACLE_MAX_N],
                       double vec[ORACLE_MAX_N][ORACLE_MAX_N] /* vec[k] = k-th eigenvector */)
{
    double W[ORACLE_MAX_N][ORACLE_MAX_N];
    for (int r = 0; r < n; ++r)
        for (int c = 0; c < n; ++c)
            W[r][c] = (r == c) ? 1.0 : 0.0; /* columns of W are eigenvectors */
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0, diag = 0.0;
        for (int p = 0; p < n; ++p) {
            diag += A[p][p] * A[p][p];
            for (int q = p + 1; q < n; ++q)
                off += A[p][q] * A[p][q];
        }
        if (off == 0.0 || off <= 1e-36 * diag)
            break;
        for (int p = 0; p < n; ++p) {
            for (int q = p + 1; q < n; ++q) {
                if (A[p][q] == 0.0)
                    continue;
                /* rotation annihilating A[p][q] (Golub & Van Loan, symmetric Schur 2x2) */
                double theta = (A[q][q] - A[p][p]) / (2.0 * A[p][q]);
                double t = 1.0 / (fabs(theta) + sqrt(theta * theta + 1.0));
                if (theta < 0.0)
                    t = -t;
                double c = 1.0 / sqrt(t * t + 1.0);
                double s = t * c;
                for (int k = 0; k < n; ++k) { /* A <- A J */
                    double akp = A[k][p], akq = A[k][q];
                    A[k][p] = c * akp - s * akq;
                    A[k][q] = s * akp + c * akq;
                }
                for (int k = 0; k < n; ++k) { /* A <- J^T A */
                    double apk = A[p][k], aqk = A[q][k];
                    A[p][k] = c * apk - s * aqk;
                    A[q][k] = s * apk + c * aqk;
                }
                for (int k = 0; k < n; ++k) { /* W <- W J */
                    double wkp = W[k][p], wkq = W[k][q];
                    W[k][p] = c * wkp - s * wkq;
                    W[k][q] = s * wkp + c * wkq;
                }
            }
        }
    }
    int order[ORACLE_MAX_N];
    for (int k = 0; k < n; ++k)
        order[k] = k;
    for (int a = 0; a < n; ++a) /* selection sort, descending eigenvalue */
        for (int b = a + 1; b < n; ++b)
            if (A[order[b]][order[b]] > A[order[a]][order[a]]) {
                int tmp = order[a];
                order[a] = order[b];
                order[b] = tmp;
            }
    for (int k = 0; k < n; ++k) {
        lam[k] = A[order[k]][order[k]];
        for (int r = 0; r < n; ++r)
            vec[k][r] = W[r][order[k]];
    }
}

/* --------------------------------------------------------------------------------------- */
/* O7/O10: Householder QR of a tall rows x m matrix (row-major), LAPACK-style storage       */
/* --------------------------------------------------------------------------------------- */
typedef struct {
    int rows, m;
    double *a;    /* rows x m: R in the upper triangle, reflector tails below */
    double beta[ORACLE_MAX_M];
    double rdiag[ORACLE_MAX_M];
} qr_t;

static void qr_factor(qr_t *f)
{
    int rows = f->rows, m = f->m;
    double *a = f->a;
    for (int k = 0; k < m; ++k) {
        double x0 = a[k * m + k];
        double tail2 = 0.0;
        for (int r = k + 1; r < rows; ++r)
            tail2 += a[r * m + k] * a[r * m + k];
        double norm = sqrt(x0 * x0 + tail2);
        if (norm == 0.0) {
            f->beta[k] = 0.0;
            f->rdiag[k] = 0.0;
            continue;
        }
        double alpha = (x0 >= 0.0) ? -norm : norm;
        double v0 = x0 - alpha; /* v = x - alpha e1 stored with v0 at the diagonal */
        double vtv = v0 * v0 + tail2;
        f->beta[k] = (vtv > 0.0) ? 2.0 / vtv : 0.0;
        a[k * m + k] = v0;
        /* apply H = I - beta v v^T to the remaining columns */
        for (int c = k + 1; c < m; ++c) {
            double s = 0.0;
            for (int r = k; r < rows; ++r)
                s += a[r * m + k] * a[r * m + c];
            s *= f->beta[k];
            for (int r = k; r < rows; ++r)
                a[r * m + c] -= s * a[r * m + k];
        }
        f->rdiag[k] = alpha;
    }
}

/* y <- H_k y for k = first..last (step dir); reflectors are symmetric, so Q^T and Q only
 * differ in the order of application. */
static void qr_apply_reflector(const qr_t *f, int k, double *y)
{
    int rows = f->rows, m = f->m;
    if (f->beta[k] == 0.0)
        return;
    double s = 0.0;
    for (int r = k; r < rows; ++r)
        s += f->a[r * m + k] * y[r];
    s *= f->beta[k];
    for (int r = k; r < rows; ++r)
        y[r] -= s * f->a[r * m + k];
}

static void qr_apply_qt(const qr_t *f, double *y)
{
    for (int k = 0; k < f->m; ++k)
        qr_apply_reflector(f, k, y);
}

static void qr_apply_q(const qr_t *f, double *y)
{
    for (int k = f->m - 1; k >= 0; --k)
        qr_apply_reflector(f, k, y);
}

static double qr_r(const qr_t *f, int r, int c)
{
    return (r == c) ? f->rdiag[r] : f->a[r * f->m + c];
}

/* solve R x = b (back substitution), in place */
static void qr_solve_r(const qr_t *f, double *b)
{
    for (int r = f->m - 1; r >= 0; --r) {
        double s = b[r];
        for (int c = r + 1; c < f->m; ++c)
            s -= qr_r(f, r, c) * b[c];
        b[r] = s / qr_r(f, r, r);
    }
}

/* solve R^T x = b (forward substitution), in place */
static void qr_solve_rt(const qr_t *f, double *b)
{
    for (int r = 0; r < f->m; ++r) {
        double s = b[r];
        for (int c = 0; c < r; ++c)
            s -= qr_r(f, c, r) * b[c];
        b[r] = s / qr_r(f, r, r);
    }
}

/* --------------------------------------------------------------------------------------- */
/* O8: LB coefficients from the fitted graph                                                */
/* --------------------------------------------------------------------------------------- */
/* a: n_codim blocks of m unscaled coefficients, block c = fit of normal coordinate c.
 * d = 2: a block is (a00, a10, a01, a20, a11, a02).  d = 1: (a0, a1, a2).
 * Outputs G (d x d row-major, inverse metric) and q (d). Returns 0 on success. */
int oracle_lb_coefficients(int d, int n_codim, const double *a, double *G, double *q)
{
    if (d == 2) {
        double g11 = 1.0, g12 = 0.0, g22 = 1.0;
        for (int c = 0; c < n_codim; ++c) {
            const double *ac = a + 6 * c;
            g11 += ac[1] * ac[1];
            g12 += ac[1] * ac[2];
            g22 += ac[2] * ac[2];
        }
        double det = g11 * g22 - g12 * g12;
        double G11 = g22 / det, G12 = -g12 / det, G22 = g11 / det;
        double q1 = 0.0, q2 = 0.0;
        for (int c = 0; c < n_codim; ++c) {
            const double *ac = a + 6 * c;
            double H11 = 2.0 * ac[3], H12 = ac[4], H22 = 2.0 * ac[5];
            double trGH = G11 * H11 + 2.0 * G12 * H12 + G22 * H22;
            double Gz1 = G11 * ac[1] + G12 * ac[2];
            double Gz2 = G12 * ac[1] + G22 * ac[2];
            q1 += trGH * Gz1;
            q2 += trGH * Gz2;
        }
        G[0] = G11; G[1] = G12; G[2] = G12; G[3] = G22;
        q[0] = q1; q[1] = q2;
        return (det > 0.0 && isfinite(det)) ? 0 : -1;
    }
    if (d == 1) {
        double g = 1.0;
        for (int c = 0; c < n_codim; ++c)
            g += a[3 * c + 1] * a[3 * c + 1];
        double Gs = 1.0 / g, qs = 0.0;
        for (int c = 0; c < n_codim; ++c)
            qs += (Gs * 2.0 * a[3 * c + 2]) * (Gs * a[3 * c + 1]);
        G[0] = Gs;
        q[0] = qs;
        return 0;
    }
    return -1;
}

/* --------------------------------------------------------------------------------------- */
/* one MVGD row                                                                             */
/* --------------------------------------------------------------------------------------- */
typedef struct {
    int n, d, K, variant, use_h;
    double h_override;
    double w_nbr; /* least-squares weight of every neighbour (p_i has weight 1) */
} oparams;

/* scratch per thread */
typedef struct {
    int64_t *nbr;
    double *key;
    double *dj;    /* K x n */
    double *V;     /* (K+1) x m */
    double *y;     /* K+1 */
    double *w;     /* K+1 */
} oscratch;

static int cmp_i64(const void *a, const void *b)
{
    int64_t x = *(const int64_t *)a, y = *(const int64_t *)b;
    return (x > y) - (x < y);
}

static void mvgd_row(const double *P, int64_t N, const oparams *pr, int64_t i, oscratch *s,
                     int64_t *cols, double *vals, double *diag)
{
    const int n = pr->n, d = pr->d, K = pr->K, nc = n - d;
    const int m = (d == 2) ? 6 : 3;
    const double *pi = P + i * n;
    double dg[ODIAG];
    memset(dg, 0, sizeof dg);
    int degenerate = 0;

    /* O1 */
    knn_row(P, N, n, i, K, s->nbr, s->key);
    qsort(s->nbr, (size_t)K, sizeof(int64_t), cmp_i64); /* neighbours in ascending index */

    /* O2 */
    double cbar[ORACLE_MAX_N] = {0};
    for (int k = 0; k < K; ++k)
        for (int a = 0; a < n; ++a) {
            double v = P[s->nbr[k] * n + a] - pi[a];
            s->dj[k * n + a] = v;
            cbar[a] += v;
        }
    for (int a = 0; a < n; ++a)
        cbar[a] /= (double)K;
    double C[ORACLE_MAX_N][ORACLE_MAX_N] = {{0}};
    for (int k = 0; k < K; ++k)
        for (int a = 0; a < n; ++a)
            for (int b = 0; b < n; ++b)
                C[a][b] += (s->dj[k * n + a] - cbar[a]) * (s->dj[k * n + b] - cbar[b]);

    /* O3 */
    double lam[ORACLE_MAX_N], E[ORACLE_MAX_N][ORACLE_MAX_N];
    jacobi_eig(n, C, lam, E);

    /* O4, O5 */
    double umin[2] = {INFINITY, INFINITY}, umax[2] = {-INFINITY, -INFINITY};
    double U[64 * 2], Z[64 * 3];
    double *u = (K <= 64) ? U : (double *)malloc(sizeof(double) * 2 * (size_t)K);
    double *z = (K <= 64) ? Z : (double *)malloc(sizeof(double) * 3 * (size_t)K);
    for (int k = 0; k < K; ++k) {
        for (int t = 0; t < d; ++t) {
            double acc = 0.0;
            for (int a = 0; a < n; ++a)
                acc += E[t][a] * s->dj[k * n + a];
            u[k * 2 + t] = acc;
            if (acc < umin[t]) umin[t] = acc;
            if (acc > umax[t]) umax[t] = acc;
        }
        for (int c = 0; c < nc; ++c) {
            double acc = 0.0;
            for (int a = 0; a < n; ++a)
                acc += E[d + c][a] * s->dj[k * n + a];
            z[k * 3 + c] = acc;
        }
    }
    double h = 0.25 * (umax[0] - umin[0]);
    if (d == 2) {
        double h2 = 0.25 * (umax[1] - umin[1]);
        if (h2 < h)
            h = h2;
    }
    if (pr->use_h)
        h = pr->h_override;
    if (!(h > 0.0) || !isfinite(h))
        degenerate = 1;

    double a_unscaled[3 * 6] = {0}, G[4] = {0}, q[2] = {0}, ell[6] = {0}, tau = 0.0;
    qr_t f = {K + 1, m, s->V, {0}, {0}};
    double rmax = 0.0, rmin = INFINITY;
    const double sw = sqrt(pr->w_nbr); /* row scale of the neighbours in the weighted fits */
    if (!degenerate) {
        /* O6 */
        const double ih = 1.0 / h;
        for (int r = 0; r <= K; ++r) {
            double xi = 0.0, eta = 0.0;
            if (r > 0) {
                xi = u[(r - 1) * 2] * ih;
                if (d == 2)
                    eta = u[(r - 1) * 2 + 1] * ih;
            }
            double *row = s->V + (size_t)r * m;
            if (d == 2) {
                row[0] = 1.0; row[1] = xi; row[2] = eta;
                row[3] = xi * xi; row[4] = xi * eta; row[5] = eta * eta;
            } else {
                row[0] = 1.0; row[1] = xi; row[2] = xi * xi;
            }
            if (r > 0 && pr->w_nbr != 1.0)
                for (int t = 0; t < m; ++t)
                    row[t] *= sw;
        }
        qr_factor(&f);
        for (int k = 0; k < m; ++k) {
            double r = fabs(f.rdiag[k]);
            if (r > rmax) rmax = r;
            if (r < rmin) rmin = r;
        }
        if (!(rmin >= ORACLE_RCOND * rmax) || !isfinite(rmax))
            degenerate = 1;
    }
    double scale[6];
    if (d == 2) {
        scale[0] = 1.0; scale[1] = scale[2] = 1.0 / h; scale[3] = scale[4] = scale[5] = 1.0 / (h * h);
    } else {
        scale[0] = 1.0; scale[1] = 1.0 / h; scale[2] = 1.0 / (h * h);
    }
    if (!degenerate) {
        /* O7 */
        for (int c = 0; c < nc; ++c) {
            s->y[0] = 0.0;
            for (int k = 0; k < K; ++k)
                s->y[k + 1] = (pr->w_nbr != 1.0) ? z[k * 3 + c] * sw : z[k * 3 + c];
            qr_apply_qt(&f, s->y);
            qr_solve_r(&f, s->y);
            for (int t = 0; t < m; ++t)
                a_unscaled[c * m + t] = s->y[t] * scale[t];
        }
        /* O8 */
        if (oracle_lb_coefficients(d, nc, a_unscaled, G, q) != 0)
            degenerate = 1;
    }
    if (!degenerate) {
        /* O9 */
        if (d == 2) {
            tau = (pr->variant == 0) ? 2.0 * (G[0] + G[3]) / (h * h) : 0.0;
            ell[0] = tau; ell[1] = -q[0]; ell[2] = -q[1];
            ell[3] = 2.0 * G[0]; ell[4] = 2.0 * G[1]; ell[5] = 2.0 * G[3];
        } else if (pr->variant == 2) {
            /* divergence form (Eq. divergence): with s(x) = sqrt(1 + sum_c y_c'(x)^2) of the
             * fitted curve, a+- = 1 / (h^2 s(0) s(+-h/2)) and
             * L_i U = a+ U(h) + a- U(-h) - (a+ + a-) U_i, U(+-h) = b0 +- b1 h + b2 h^2. */
            double s0 = 1.0, sp = 1.0, sm = 1.0;
            for (int c = 0; c < nc; ++c) {
                const double a1 = a_unscaled[c * m + 1], a2 = a_unscaled[c * m + 2];
                const double dp = a1 + 2.0 * a2 * (0.5 * h), dm = a1 - 2.0 * a2 * (0.5 * h);
                s0 += a1 * a1;
                sp += dp * dp;
                sm += dm * dm;
            }
            s0 = sqrt(s0);
            sp = sqrt(sp);
            sm = sqrt(sm);
            const double ap = 1.0 / (h * h * s0 * sp), am = 1.0 / (h * h * s0 * sm);
            tau = ap + am;
            ell[0] = tau; ell[1] = (ap - am) * h; ell[2] = tau * h * h;
        } else {
            tau = (pr->variant == 0) ? 2.0 * G[0] / (h * h) : 0.0;
            ell[0] = tau; ell[1] = -q[0]; ell[2] = 2.0 * G[0];
        }
        /* O10: w = Q R^-T D ell */
        for (int r = 0; r <= K; ++r)
            s->w[r] = 0.0;
        for (int t = 0; t < m; ++t)
            s->w[t] = ell[t] * scale[t];
        qr_solve_rt(&f, s->w);
        for (int r = m; r <= K; ++r)
            s->w[r] = 0.0;
        qr_apply_q(&f, s->w);
        if (pr->w_nbr != 1.0) /* W V y = W^1/2 (W^1/2 V) y */
            for (int r = 1; r <= K; ++r)
                s->w[r] *= sw;
        s->w[0] -= tau;
    }
    /* O11: merge the centre into the ascending neighbour list */
    int placed = 0, o = 0;
    for (int k = 0; k <= K; ++k) {
        if (!placed && (k == K || i < s->nbr[k])) {
            cols[o] = i;
            vals[o] = degenerate ? 0.0 : s->w[0];
            ++o;
            placed = 1;
        }
        if (k < K) {
            cols[o] = s->nbr[k];
            vals[o] = degenerate ? 0.0 : s->w[k + 1];
            ++o;
        }
    }
    if (diag) {
        dg[0] = h;
        dg[1] = degenerate;
        for (int a = 0; a < n; ++a) {
            dg[2 + a] = lam[a];
            for (int b = 0; b < n; ++b)
                dg[6 + a * 4 + b] = E[a][b];
        }
        for (int t = 0; t < nc * m && t < 18; ++t)
            dg[22 + t] = a_unscaled[t];
        for (int t = 0; t < 4; ++t)
            dg[40 + t] = G[t];
        dg[44] = q[0];
        dg[45] = q[1];
        for (int t = 0; t < 6; ++t)
            dg[46 + t] = ell[t];
        for (int t = 0; t < m; ++t)
            dg[52 + t] = f.rdiag[t];
        dg[58] = tau;
        dg[59] = (rmax > 0.0) ? rmin / rmax : 0.0;
        dg[60] = s->key[K - 1];
        memcpy(diag, dg, sizeof dg);
    }
    if (u != U) free(u);
    if (z != Z) free(z);
}

static int check_common(const double *P, int64_t N, int n, int d, int K)
{
    if (!P || N < 2 || n < 2 || n > ORACLE_MAX_N || (d != 1 && d != 2) || d >= n)
        return -1;
    int m = (d == 2) ? 6 : 3;
    if (K < m - 1 || K > N - 1)
        return -1;
    if (n - d > 3)
        return -1;
    for (int64_t t = 0; t < N * n; ++t)
        if (!isfinite(P[t]))
            return -2;
    return 0;
}

/* --------------------------------------------------------------------------------------- */
/* exported entry points (ctypes)                                                           */
/* --------------------------------------------------------------------------------------- */

/* K nearest neighbours of the listed rows (rows == NULL: all rows), ascending (key, index). */
int oracle_knn(const double *P, int64_t N, int n, int K, const int64_t *rows, int64_t nrows,
               int64_t *out_idx, double *out_key, int nthreads)
{
    if (!P || N < 2 || n < 1 || n > ORACLE_MAX_N || K < 1 || K > N - 1)
        return -1;
    int64_t R = rows ? nrows : N;
#ifdef _OPENMP
    if (nthreads > 0)
        omp_set_num_threads(nthreads);
#pragma omp parallel
#endif
    {
        double *key = (double *)malloc(sizeof(double) * (size_t)K);
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 16)
#endif
        for (int64_t r = 0; r < R; ++r) {
            int64_t i = rows ? rows[r] : r;
            knn_row(P, N, n, i, K, out_idx + r * K, key);
            if (out_key)
                memcpy(out_key + r * K, key, sizeof(double) * (size_t)K);
        }
        free(key);
    }
    return 0;
}

/* MVGD (variant 0), plain LS (variant 1) or, for curves (d = 1), MVGD in the divergence form
 * (variant 2) rows for the listed rows (rows == NULL: all), with
 * least-squares weight w_nbr (> 0) on every neighbour and 1 on p_i (w_nbr = 1: unweighted).
 * out_cols / out_vals: nrows x (K+1), columns ascending. out_diag: nrows x 64 or NULL.
 * Returns 0, -1 on bad arguments, -2 on non-finite coordinates. */
int oracle_rows(const double *P, int64_t N, int n, int d, int K, int variant, int use_h,
                double h_override, double w_nbr, const int64_t *rows, int64_t nrows,
                int64_t *out_cols, double *out_vals, double *out_diag, int nthreads)
{
    int rc = check_common(P, N, n, d, K);
    if (rc)
        return rc;
    if (variant < 0 || variant > 2 || (variant == 2 && d != 1) || !(w_nbr > 0.0) ||
        !isfinite(w_nbr))
        return -1;
    oparams pr = {n, d, K, variant, use_h, h_override, w_nbr};
    int64_t R = rows ? nrows : N;
    const int m = (d == 2) ? 6 : 3;
#ifdef _OPENMP
    if (nthreads > 0)
        omp_set_num_threads(nthreads);
#pragma omp parallel
#endif
    {
        oscratch s;
        s.nbr = (int64_t *)malloc(sizeof(int64_t) * (size_t)K);
        s.key = (double *)malloc(sizeof(double) * (size_t)K);
        s.dj = (double *)malloc(sizeof(double) * (size_t)K * n);
        s.V = (double *)malloc(sizeof(double) * (size_t)(K + 1) * m);
        s.y = (double *)malloc(sizeof(double) * (size_t)(K + 1));
        s.w = (double *)malloc(sizeof(double) * (size_t)(K + 1));
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 16)
#endif
        for (int64_t r = 0; r < R; ++r) {
            int64_t i = rows ? rows[r] : r;
            mvgd_row(P, N, &pr, i, &s, out_cols + r * (K + 1), out_vals + r * (K + 1),
                     out_diag ? out_diag + r * ODIAG : NULL);
        }
        free(s.nbr); free(s.key); free(s.dj); free(s.V); free(s.y); free(s.w);
    }
    return 0;
}

/* O12: y = L x for a CSR matrix, x and y row-major [N, nrhs]. */
int oracle_apply(int64_t N, const int64_t *row_ptr, const int64_t *cols, const double *vals,
                 int nrhs, const double *x, double *y)
{
    for (int64_t i = 0; i < N; ++i)
        for (int r = 0; r < nrhs; ++r) {
            double acc = 0.0;
            for (int64_t t = row_ptr[i]; t < row_ptr[i + 1]; ++t)
                acc += vals[t] * x[cols[t] * nrhs + r];
            y[i * nrhs + r] = acc;
        }
    return 0;
}

int oracle_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
