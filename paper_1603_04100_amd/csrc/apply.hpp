// apply.hpp -- y = L x on the sliced-ELL matrix, CSR export and per-row diagnostics.
//
// The handle stores L in cell-sorted order: row s, slot k at [k * ld + s] (slot 0 = the point
// itself), columns as sorted positions. Lanes of a wave own consecutive rows, so every slot
// load is one coalesced 256 B (or 512 B) line, and the gathered x entries of neighbouring rows
// fall in neighbouring sorted positions (L1/L2 hits). x and y stay in the caller's order:
// x is first permuted into sorted order (xs), and results are scattered back through perm.
#pragma once

#include "common.hpp"

namespace mvgd {

template <typename T>
__global__ __launch_bounds__(256) void gather_rows_kernel(const T *__restrict__ x,
                                                          const int32_t *__restrict__ perm,
                                                          T *__restrict__ xs, int64_t n, int nrhs)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * nrhs)
        return;
    const int64_t s = t / nrhs;
    const int r = (int)(t - s * nrhs);
    xs[t] = x[(int64_t)perm[s] * nrhs + r];
}

template <typename T, int R>
__global__ __launch_bounds__(256) void spmv_ell_kernel(const int32_t *__restrict__ col,
                                                       const T *__restrict__ val,
                                                       const T *__restrict__ xs,
                                                       const int32_t *__restrict__ perm,
                                                       T *__restrict__ y, int64_t n, int64_t ld,
                                                       int slots)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n)
        return;
    double acc[R];
#pragma unroll
    for (int r = 0; r < R; ++r)
        acc[r] = 0.0;
    for (int k = 0; k < slots; ++k) {
        const int32_t c = col[(int64_t)k * ld + s];
        const double w = (double)val[(int64_t)k * ld + s];
#pragma unroll
        for (int r = 0; r < R; ++r)
            acc[r] = fma(w, (double)xs[(int64_t)c * R + r], acc[r]);
    }
    const int64_t row = perm[s];
#pragma unroll
    for (int r = 0; r < R; ++r)
        y[row * R + r] = (T)acc[r];
}

// general nrhs (x rows of length nrhs)
template <typename T>
__global__ __launch_bounds__(256) void spmv_ell_any_kernel(const int32_t *__restrict__ col,
                                                           const T *__restrict__ val,
                                                           const T *__restrict__ xs,
                                                           const int32_t *__restrict__ perm,
                                                           T *__restrict__ y, int64_t n, int64_t ld,
                                                           int slots, int nrhs)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * nrhs)
        return;
    const int64_t s = t / nrhs;
    const int r = (int)(t - s * nrhs);
    double acc = 0.0;
    for (int k = 0; k < slots; ++k) {
        const int32_t c = col[(int64_t)k * ld + s];
        acc = fma((double)val[(int64_t)k * ld + s], (double)xs[(int64_t)c * nrhs + r], acc);
    }
    y[(int64_t)perm[s] * nrhs + r] = (T)acc;
}

// CSR in the caller's order: row perm[s] gets columns perm[col] - row0 (local to the cloud),
// sorted ascending with their weights. One thread per row (not on the apply path).
template <typename T>
__global__ __launch_bounds__(64) void export_csr_kernel(const int32_t *__restrict__ col,
                                                        const T *__restrict__ val,
                                                        const int32_t *__restrict__ perm,
                                                        const CloudGrid *__restrict__ grids,
                                                        int n_clouds, int64_t n, int64_t ld,
                                                        int slots, int64_t *__restrict__ row_ptr,
                                                        int32_t *__restrict__ out_col,
                                                        T *__restrict__ out_val)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s == 0 && row_ptr)
        row_ptr[n] = n * slots;
    if (s >= n)
        return;
    const int64_t row = perm[s];
    int lo = 0, hi = n_clouds - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (grids[mid].row0 <= row)
            lo = mid;
        else
            hi = mid - 1;
    }
    const int64_t row0 = grids[lo].row0;
    int32_t c[kMaxK + 1];
    T v[kMaxK + 1];
    for (int k = 0; k < slots; ++k) {
        const int32_t ck = (int32_t)(perm[col[(int64_t)k * ld + s]] - row0);
        const T vk = val[(int64_t)k * ld + s];
        int j = k;
        while (j > 0 && c[j - 1] > ck) {
            c[j] = c[j - 1];
            v[j] = v[j - 1];
            --j;
        }
        c[j] = ck;
        v[j] = vk;
    }
    const int64_t base = row * slots;
    if (row_ptr)
        row_ptr[row] = base;
    for (int k = 0; k < slots; ++k) {
        if (out_col)
            out_col[base + k] = c[k];
        if (out_val)
            out_val[base + k] = v[k];
    }
}

__global__ __launch_bounds__(256) void diag_scatter_kernel(const double *__restrict__ h_s,
                                                           const uint8_t *__restrict__ f_s,
                                                           const int32_t *__restrict__ perm,
                                                           double *__restrict__ h,
                                                           uint8_t *__restrict__ f, int64_t n)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n)
        return;
    const int64_t row = perm[s];
    if (h)
        h[row] = h_s[s];
    if (f)
        f[row] = f_s[s];
}

} // namespace mvgd
