// stats.hpp -- row sign statistics of the assembled matrix (diagonal sign, M-rows, negative
// off-diagonal mass relative to the diagonal), reduced in a fixed order.
//
// row_stats_kernel     block b owns rows [b * rows_per_block, ...): one thread per row at a
//                      time (fixed assignment), per-thread partials, fixed tree over the block
// row_stats_final      one block sums the block partials in a fixed tree
#pragma once

#include "common.hpp"

namespace mvgd {

struct RowStatsPart {
    unsigned long long n_diag_neg, n_m_rows, n_off_neg, n_zero_diag;
    double sum_ratio, max_ratio;
};

constexpr int kStatsThreads = 256;

__device__ __forceinline__ void stats_merge(RowStatsPart &a, const RowStatsPart &b)
{
    a.n_diag_neg += b.n_diag_neg;
    a.n_m_rows += b.n_m_rows;
    a.n_off_neg += b.n_off_neg;
    a.n_zero_diag += b.n_zero_diag;
    a.sum_ratio += b.sum_ratio;
    a.max_ratio = fmax(a.max_ratio, b.max_ratio);
}

// fixed-shape tree over the block's kStatsThreads partials in LDS
__device__ __forceinline__ void stats_block_reduce(RowStatsPart *sh, RowStatsPart mine,
                                                   RowStatsPart *out)
{
    sh[threadIdx.x] = mine;
    __syncthreads();
    for (int w = kStatsThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            RowStatsPart a = sh[threadIdx.x];
            stats_merge(a, sh[threadIdx.x + w]);
            sh[threadIdx.x] = a;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0)
        *out = sh[0];
}

template <typename T>
__global__ __launch_bounds__(kStatsThreads) void row_stats_kernel(
    const T *__restrict__ val, const int32_t *__restrict__ perm, int64_t n, int64_t ld, int slots,
    int64_t rows_per_block, double *__restrict__ ratio_out, RowStatsPart *__restrict__ parts)
{
    __shared__ RowStatsPart sh[kStatsThreads];
    RowStatsPart mine = {0, 0, 0, 0, 0.0, 0.0};
    const int64_t r0 = (int64_t)blockIdx.x * rows_per_block;
    const int64_t r1 = min(n, r0 + rows_per_block);
    for (int64_t s = r0 + threadIdx.x; s < r1; s += kStatsThreads) {
        const double d = (double)val[s]; // slot 0 = the diagonal
        double neg = 0.0;
        unsigned long long off_neg = 0;
        bool nonneg = true;
        for (int k = 1; k < slots; ++k) { // neighbours in ascending column order
            const double o = (double)val[(int64_t)k * ld + s];
            neg += o < 0.0 ? -o : 0.0;
            off_neg += o < 0.0;
            nonneg = nonneg && (o >= 0.0);
        }
        const bool zero = !(d != 0.0);
        const double ratio = zero ? __longlong_as_double(0x7ff8000000000000ll) : neg / fabs(d);
        if (ratio_out)
            ratio_out[perm[s]] = ratio;
        mine.n_diag_neg += d < 0.0;
        mine.n_m_rows += (d < 0.0) && nonneg;
        mine.n_off_neg += off_neg;
        mine.n_zero_diag += zero;
        if (!zero) {
            mine.sum_ratio += ratio;
            mine.max_ratio = fmax(mine.max_ratio, ratio);
        }
    }
    stats_block_reduce(sh, mine, &parts[blockIdx.x]);
}

__global__ __launch_bounds__(kStatsThreads) void row_stats_final_kernel(RowStatsPart *parts,
                                                                        int n_parts)
{
    __shared__ RowStatsPart sh[kStatsThreads];
    RowStatsPart mine = {0, 0, 0, 0, 0.0, 0.0};
    for (int b = threadIdx.x; b < n_parts; b += kStatsThreads)
        stats_merge(mine, parts[b]);
    stats_block_reduce(sh, mine, &parts[n_parts]);
}

} // namespace mvgd
