// solve.hpp -- iterative solution of (sigma I - L) x = b on the assembled matrix.
//
// Everything runs in the matrix's cell order (the sliced-ELL order), in double: b and the initial
// guess are permuted in once, the solution is permuted out once, and every operator application
// is the coalesced ELL product of the apply path. Pinned rows (the first point of every cloud, on
// request, and caller-flagged Dirichlet points) are identity rows, so x_p = b_p there; one per
// cloud removes the constant null vector of L on closed manifolds (L 1 = 0).
//
// Inner products are reduced deterministically: every kernel that produces one writes one
// partial per block (fixed tree over the block), and a single-block kernel adds the partials in
// a fixed order. All scalars of the iteration live in device memory (SolveScalars), so a batch
// of iterations is enqueued without host round trips; once the residual test passes, a device
// flag turns the remaining kernels of the batch into no-ops.
#pragma once

#include "common.hpp"

namespace mvgd {

constexpr int kSolveThreads = 256;
constexpr int kMaxPartials = 3;

struct SolveScalars {
    double rho, rho_prev, alpha, omega, beta;
    double rr;        // squared norm of the current residual
    double bb;        // squared norm of b
    double tol2;      // rtol^2 * bb
    double dot[kMaxPartials];
    int32_t done;     // 1: converged, 2: breakdown (a zero or non-finite denominator)
    int32_t iters;    // iterations completed
};

// sum of the block's partials (kSolveThreads values per slot) in a fixed tree, written by thread 0
template <int NP>
__device__ __forceinline__ void block_partials(double v[NP], double *out /* [NP] */)
{
    __shared__ double sh[NP][kSolveThreads];
#pragma unroll
    for (int j = 0; j < NP; ++j)
        sh[j][threadIdx.x] = v[j];
    __syncthreads();
    for (int w = kSolveThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
#pragma unroll
            for (int j = 0; j < NP; ++j)
                sh[j][threadIdx.x] += sh[j][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0)
#pragma unroll
        for (int j = 0; j < NP; ++j)
            out[j] = sh[j][0];
}

// pinned[s] = 1 for the sorted position of the first caller row of every cloud (if requested)
// and for every row flagged in `fixed` (caller order)
__global__ __launch_bounds__(kSolveThreads) void solve_setup_kernel(
    const int32_t *__restrict__ perm, const CloudGrid *__restrict__ grids, int n_clouds, int64_t n,
    int pin, const uint8_t *__restrict__ fixed, const void *__restrict__ b,
    const void *__restrict__ x0, int is_double, double *__restrict__ bs, double *__restrict__ xs,
    uint8_t *__restrict__ pinned)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n)
        return;
    const int64_t row = perm[s];
    bs[s] = is_double ? ((const double *)b)[row] : (double)((const float *)b)[row];
    xs[s] = is_double ? ((const double *)x0)[row] : (double)((const float *)x0)[row];
    uint8_t pv = 0;
    if (pin) {
        int lo = 0, hi = n_clouds - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (grids[mid].row0 <= row)
                lo = mid;
            else
                hi = mid - 1;
        }
        pv = row == grids[lo].row0;
    }
    if (fixed && fixed[row])
        pv = 1;
    pinned[s] = pv;
}

// (A x)_s for A = sigma I - L, identity on pinned rows
template <typename T>
__device__ __forceinline__ double op_row(const int32_t *__restrict__ col, const T *__restrict__ val,
                                         int64_t s, int64_t ld, int slots, const uint8_t *pinned,
                                         double sigma, const double *__restrict__ x)
{
    if (pinned[s])
        return x[s];
    double acc = 0.0;
    for (int k = 0; k < slots; ++k)
        acc = fma((double)val[(int64_t)k * ld + s], x[col[(int64_t)k * ld + s]], acc);
    return fma(sigma, x[s], -acc);
}

// diagonal of A: sigma - L_ss (slot 0 holds the row's own weight), 1 on pinned rows
template <typename T>
__device__ __forceinline__ double op_diag(const T *__restrict__ val, int64_t s,
                                          const uint8_t *pinned, double sigma)
{
    return pinned[s] ? 1.0 : sigma - (double)val[s];
}

// r = b - A x, rhat = r, p = v = 0; partials: (r, r), (b, b)
template <typename T>
__global__ __launch_bounds__(kSolveThreads) void bicg_init_kernel(
    const int32_t *__restrict__ col, const T *__restrict__ val, int64_t n, int64_t ld, int slots,
    const uint8_t *__restrict__ pinned, double sigma, const double *__restrict__ x,
    const double *__restrict__ b, double *__restrict__ r, double *__restrict__ rhat,
    double *__restrict__ p, double *__restrict__ v, double *__restrict__ part)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double acc[2] = {0.0, 0.0};
    if (s < n) {
        const double rs = b[s] - op_row<T>(col, val, s, ld, slots, pinned, sigma, x);
        r[s] = rs;
        rhat[s] = rs;
        p[s] = 0.0;
        v[s] = 0.0;
        acc[0] = rs * rs;
        acc[1] = b[s] * b[s];
    }
    block_partials<2>(acc, part + 2 * blockIdx.x);
}

// single block: sums of the partials in a fixed order, then the scalar update of `step`
enum SolveStep { kStepInit = 0, kStepRho = 1, kStepAlpha = 2, kStepOmega = 3, kStepJacobi = 4 };

__global__ __launch_bounds__(kSolveThreads) void solve_scalar_kernel(int step, const double *part,
                                                                    int nparts, int np,
                                                                    SolveScalars *sc, double rtol)
{
    if (step != kStepInit && sc->done)
        return;
    double v[kMaxPartials] = {0.0, 0.0, 0.0};
    for (int i = threadIdx.x; i < nparts; i += kSolveThreads)
        for (int j = 0; j < np; ++j)
            v[j] += part[(int64_t)i * np + j];
    double tot[kMaxPartials];
    block_partials<kMaxPartials>(v, tot);
    if (threadIdx.x != 0)
        return;
    auto bad = [](double d) { return !(d != 0.0) || !isfinite(d); };
    switch (step) {
    case kStepInit: // tot = (r.r, b.b)
        sc->rr = tot[0];
        sc->bb = tot[1];
        sc->tol2 = rtol * rtol * tot[1];
        sc->rho = sc->rho_prev = sc->alpha = sc->omega = 1.0;
        sc->beta = 0.0;
        sc->iters = 0;
        sc->done = (tot[0] <= sc->tol2) ? 1 : 0;
        break;
    case kStepAlpha: // tot = (rhat.v)
        if (bad(tot[0])) {
            sc->done = 2;
            sc->alpha = 0.0;
        } else {
            sc->alpha = sc->rho / tot[0];
        }
        break;
    case kStepOmega: // tot = (t.s, t.t); t = 0 means s = 0: x + alpha p is the solution
        if (!isfinite(tot[0]) || !isfinite(tot[1])) {
            sc->done = 2;
            sc->omega = 0.0;
        } else {
            sc->omega = tot[1] > 0.0 ? tot[0] / tot[1] : 0.0;
        }
        break;
    case kStepRho: // tot = (rhat.r, r.r) after the x, r update: next rho and beta, residual test
        sc->iters += 1;
        sc->rr = tot[1];
        if (tot[1] <= sc->tol2) {
            sc->done = 1;
        } else if (bad(tot[0]) || bad(sc->omega) || bad(sc->rho)) {
            sc->done = 2;
        } else {
            sc->beta = (tot[0] / sc->rho) * (sc->alpha / sc->omega);
            sc->rho_prev = sc->rho;
            sc->rho = tot[0];
        }
        break;
    case kStepJacobi: // tot = (r.r) of the residual before the sweep that just ran
        sc->iters += 1;   // sweeps that wrote the next iterate
        sc->rr = tot[0];
        if (!isfinite(tot[0]))
            sc->done = 2;
        else if (tot[0] <= sc->tol2)
            sc->done = 1;
        break;
    }
}

// the first rho = (rhat, r0) = (r0, r0)
__global__ void bicg_first_rho_kernel(SolveScalars *sc)
{
    if (threadIdx.x == 0 && blockIdx.x == 0)
        sc->rho = sc->rr;
}

// p = r + beta (p - omega v)
__global__ __launch_bounds__(kSolveThreads) void bicg_p_kernel(int64_t n, const double *__restrict__ r,
                                                              const double *__restrict__ v,
                                                              double *__restrict__ p,
                                                              const SolveScalars *sc, int first)
{
    if (sc->done)
        return;
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n)
        return;
    if (first)
        p[s] = r[s];
    else
        p[s] = fma(sc->beta, fma(-sc->omega, v[s], p[s]), r[s]);
}

// v = A p; partial (rhat, v)
template <typename T>
__global__ __launch_bounds__(kSolveThreads) void bicg_v_kernel(
    const int32_t *__restrict__ col, const T *__restrict__ val, int64_t n, int64_t ld, int slots,
    const uint8_t *__restrict__ pinned, double sigma, const double *__restrict__ p,
    const double *__restrict__ rhat, double *__restrict__ v, double *__restrict__ part,
    const SolveScalars *sc)
{
    if (sc->done)
        return;
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double acc[1] = {0.0};
    if (s < n) {
        const double vs = op_row<T>(col, val, s, ld, slots, pinned, sigma, p);
        v[s] = vs;
        acc[0] = rhat[s] * vs;
    }
    block_partials<1>(acc, part + blockIdx.x);
}

// s = r - alpha v (written into r's partner buffer)
__global__ __launch_bounds__(kSolveThreads) void bicg_s_kernel(int64_t n, const double *__restrict__ r,
                                                              const double *__restrict__ v,
                                                              double *__restrict__ sv,
                                                              const SolveScalars *sc)
{
    if (sc->done)
        return;
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s < n)
        sv[s] = fma(-sc->alpha, v[s], r[s]);
}

// t = A s; partials (t, s), (t, t)
template <typename T>
__global__ __launch_bounds__(kSolveThreads) void bicg_t_kernel(
    const int32_t *__restrict__ col, const T *__restrict__ val, int64_t n, int64_t ld, int slots,
    const uint8_t *__restrict__ pinned, double sigma, const double *__restrict__ sv,
    double *__restrict__ t, double *__restrict__ part, const SolveScalars *sc)
{
    if (sc->done)
        return;
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double acc[2] = {0.0, 0.0};
    if (s < n) {
        const double ts = op_row<T>(col, val, s, ld, slots, pinned, sigma, sv);
        t[s] = ts;
        acc[0] = ts * sv[s];
        acc[1] = ts * ts;
    }
    block_partials<2>(acc, part + 2 * blockIdx.x);
}

// x += alpha p + omega s; r = s - omega t; partials (rhat, r), (r, r)
__global__ __launch_bounds__(kSolveThreads) void bicg_xr_kernel(
    int64_t n, const double *__restrict__ p, const double *__restrict__ sv,
    const double *__restrict__ t, const double *__restrict__ rhat, double *__restrict__ x,
    double *__restrict__ r, double *__restrict__ part, const SolveScalars *sc)
{
    if (sc->done)
        return;
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double acc[2] = {0.0, 0.0};
    if (s < n) {
        const double a = sc->alpha, w = sc->omega;
        x[s] = fma(w, sv[s], fma(a, p[s], x[s]));
        const double rs = fma(-w, t[s], sv[s]);
        r[s] = rs;
        acc[0] = rhat[s] * rs;
        acc[1] = rs * rs;
    }
    block_partials<2>(acc, part + 2 * blockIdx.x);
}

// damped Jacobi: x_new = x + omega (b - A x) / diag(A); partial (r, r) of the old residual
template <typename T>
__global__ __launch_bounds__(kSolveThreads) void jacobi_kernel(
    const int32_t *__restrict__ col, const T *__restrict__ val, int64_t n, int64_t ld, int slots,
    const uint8_t *__restrict__ pinned, double sigma, double omega, const double *__restrict__ b,
    const double *__restrict__ x, double *__restrict__ xn, double *__restrict__ part,
    const SolveScalars *sc)
{
    if (sc->done)
        return;
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double acc[1] = {0.0};
    if (s < n) {
        const double rs = b[s] - op_row<T>(col, val, s, ld, slots, pinned, sigma, x);
        xn[s] = fma(omega, rs / op_diag<T>(val, s, pinned, sigma), x[s]);
        acc[0] = rs * rs;
    }
    block_partials<1>(acc, part + blockIdx.x);
}

// true residual r = b - A x, partial (r, r)
template <typename T>
__global__ __launch_bounds__(kSolveThreads) void residual_kernel(
    const int32_t *__restrict__ col, const T *__restrict__ val, int64_t n, int64_t ld, int slots,
    const uint8_t *__restrict__ pinned, double sigma, const double *__restrict__ b,
    const double *__restrict__ x, double *__restrict__ part)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double acc[1] = {0.0};
    if (s < n) {
        const double rs = b[s] - op_row<T>(col, val, s, ld, slots, pinned, sigma, x);
        acc[0] = rs * rs;
    }
    block_partials<1>(acc, part + blockIdx.x);
}

// single block: total of one partial slot into *out (fixed order)
__global__ __launch_bounds__(kSolveThreads) void sum_partials_kernel(const double *part, int nparts,
                                                                    double *out)
{
    double v[1] = {0.0};
    for (int i = threadIdx.x; i < nparts; i += kSolveThreads)
        v[0] += part[i];
    double tot[1];
    block_partials<1>(v, tot);
    if (threadIdx.x == 0)
        *out = tot[0];
}

// x (caller order, float or double) from the cell-order solution
__global__ __launch_bounds__(kSolveThreads) void solve_scatter_kernel(
    const int32_t *__restrict__ perm, int64_t n, const double *__restrict__ xs, void *x,
    int is_double)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n)
        return;
    if (is_double)
        ((double *)x)[perm[s]] = xs[s];
    else
        ((float *)x)[perm[s]] = (float)xs[s];
}

} // namespace mvgd
