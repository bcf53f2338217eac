// eigs.hpp -- a few eigenvalues of -L nearest the bottom of its spectrum (Sec. 4: the eigenvalue
// problem -Delta nu = lambda nu on closed surfaces and, with boundary conditions, on open ones).
//
// Chebyshev-filtered subspace iteration on a block of m vectors in the matrix's cell order: the
// filter p(A), A = -L, a Chebyshev polynomial of the first kind that is bounded by 1 on the
// unwanted interval [a, b] and grows fast below a, is applied with the three-term recurrence, one
// multi-column ELL product per degree; the block is then orthonormalised (Cholesky QR, twice) and
// the Rayleigh quotient H = V^T A V (m x m) gives the Ritz values. b bounds the spectrum
// (Gershgorin: the largest absolute row sum), a the largest Ritz value of the previous step.
// Rows flagged in `mask` are removed from the operator: the block is kept zero there, so the
// iteration runs on the submatrix of the other rows and columns (Dirichlet points, ghost rows).
//
// Blocks of vectors are row-major [n][m] (a row's m entries contiguous), so the ELL product
// gathers m contiguous values per neighbour.
#pragma once

#include "common.hpp"

namespace mvgd {

constexpr int kEigMaxBlock = 64;
constexpr int kEigThreads = 256;

// mask[s] = 1 for sorted positions whose caller row is flagged in `fixed` (NULL: none)
__global__ __launch_bounds__(kEigThreads) void eig_mask_kernel(const int32_t *__restrict__ perm,
                                                               int64_t n,
                                                               const uint8_t *__restrict__ fixed,
                                                               uint8_t *__restrict__ mask)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s < n)
        mask[s] = (fixed && fixed[perm[s]]) ? 1 : 0;
}

// counter-based uniform numbers in [-1, 1) (splitmix64 of the seed and the entry), zero on masked
// rows
__global__ __launch_bounds__(kEigThreads) void eig_init_kernel(int64_t n, int m,
                                                               const uint8_t *__restrict__ mask,
                                                               unsigned long long seed,
                                                               double *__restrict__ Y)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * m)
        return;
    unsigned long long z = seed + 0x9e3779b97f4a7c15ull * (unsigned long long)(e + 1);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    z ^= z >> 31;
    const double u = (double)(z >> 11) * (1.0 / 9007199254740992.0); // [0, 1)
    Y[e] = mask[e / m] ? 0.0 : 2.0 * u - 1.0;
}

// Z = a1 A Y + a2 Y + a3 X with A = -L, on unmasked rows (masked rows: 0). Threads: 64 per row
// (lane = column j < m), four rows per block.
template <typename T>
__global__ __launch_bounds__(kEigThreads) void eig_cheb_kernel(
    const int32_t *__restrict__ col, const T *__restrict__ val, int64_t n, int64_t ld, int slots,
    int m, const uint8_t *__restrict__ mask, const double *__restrict__ X,
    const double *__restrict__ Y, double *__restrict__ Z, double a1, double a2, double a3)
{
    const int64_t s = (int64_t)blockIdx.x * (kEigThreads / kWave) + threadIdx.x / kWave;
    const int j = (int)(threadIdx.x % kWave);
    if (s >= n || j >= m)
        return;
    if (mask[s]) {
        Z[s * m + j] = 0.0;
        return;
    }
    double ay = 0.0;
    for (int k = 0; k < slots; ++k) {
        const int64_t c = col[(int64_t)k * ld + s];
        ay = fma((double)val[(int64_t)k * ld + s], Y[c * m + j], ay);
    }
    double z = fma(a2, Y[s * m + j], -a1 * ay);
    if (a3 != 0.0)
        z = fma(a3, X[s * m + j], z);
    Z[s * m + j] = z;
}

// Per-block partials of A^T B (m x m, row-major, entry (i, j) = sum_r A[r][i] B[r][j]) over a
// grid-stride range of rows; part[block][m * m].
__global__ __launch_bounds__(kEigThreads) void eig_gram_kernel(int64_t n, int m,
                                                               const double *__restrict__ A,
                                                               const double *__restrict__ B,
                                                               double *__restrict__ part)
{
    const int mm = m * m;
    double acc[kEigMaxBlock * kEigMaxBlock / kEigThreads];
    const int per = (mm + kEigThreads - 1) / kEigThreads;
    for (int q = 0; q < per; ++q)
        acc[q] = 0.0;
    const int64_t rows_per = (n + gridDim.x - 1) / gridDim.x;
    const int64_t r0 = (int64_t)blockIdx.x * rows_per, r1 = min(n, r0 + rows_per);
    for (int64_t r = r0; r < r1; ++r)
        for (int q = 0; q < per; ++q) {
            const int e = (int)threadIdx.x + q * kEigThreads;
            if (e < mm)
                acc[q] = fma(A[r * m + e / m], B[r * m + e % m], acc[q]);
        }
    for (int q = 0; q < per; ++q) {
        const int e = (int)threadIdx.x + q * kEigThreads;
        if (e < mm)
            part[(int64_t)blockIdx.x * mm + e] = acc[q];
    }
}

// out[e] = sum over blocks of part[block][e], in block order
__global__ __launch_bounds__(kEigThreads) void eig_reduce_kernel(const double *__restrict__ part,
                                                                 int nblk, int mm,
                                                                 double *__restrict__ out)
{
    const int e = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (e >= mm)
        return;
    double s = 0.0;
    for (int b = 0; b < nblk; ++b)
        s += part[(int64_t)b * mm + e];
    out[e] = s;
}

// Q = Y R (R m x m row-major, here the inverse Cholesky factor), 64 threads per row
__global__ __launch_bounds__(kEigThreads) void eig_rmul_kernel(int64_t n, int m,
                                                               const double *__restrict__ Y,
                                                               const double *__restrict__ R,
                                                               double *__restrict__ Q)
{
    const int64_t s = (int64_t)blockIdx.x * (kEigThreads / kWave) + threadIdx.x / kWave;
    const int j = (int)(threadIdx.x % kWave);
    if (s >= n || j >= m)
        return;
    double q = 0.0;
    for (int i = 0; i < m; ++i)
        q = fma(Y[s * m + i], R[i * m + j], q);
    Q[s * m + j] = q;
}

// largest absolute row sum of L over unmasked rows (Gershgorin bound on |lambda|), as an ordered
// encoding for the integer atomic
template <typename T>
__global__ __launch_bounds__(kEigThreads) void eig_gersh_kernel(const T *__restrict__ val,
                                                                int64_t n, int64_t ld, int slots,
                                                                const uint8_t *__restrict__ mask,
                                                                unsigned long long *__restrict__ out)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n || mask[s])
        return;
    double a = 0.0;
    for (int k = 0; k < slots; ++k)
        a += fabs((double)val[(int64_t)k * ld + s]);
    atomicMax(out, ord_encode(a));
}

} // namespace mvgd
