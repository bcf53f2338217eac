// bin.hpp -- counting sort of the points into Morton-ordered cells (the neighbour-search grid).
//
// bbox_kernel      partial bounding boxes (ambient and projected coordinates) + non-finite counts
// bbox_reduce_kernel  the per-cloud box from the partials
// plan_kernel      per-cloud cell grid and Morton part tables from the bounding boxes
// key_kernel       cell key of every point and its slot inside the cell (atomic count)
// scan_*           exclusive prefix sum of the cell counts -> cell start offsets
// scatter_kernel   cell-sorted copy of the points (padded to 4 components) by the atomic slots
// canon_kernel     canonical order inside every cell (ascending original index), permutation and
//                  its inverse: the cell order is the same on every run
#pragma once

#include "common.hpp"

namespace mvgd {

struct CloudStats {  // ordered-encoded doubles; see ord_encode
    unsigned long long mn[4];   // ambient coordinates
    unsigned long long mx[4];
    unsigned long long pmn[3];  // projected coordinates
    unsigned long long pmx[3];
    unsigned long long nonfinite;
    unsigned long long pad;
};

// Resets the per-cloud statistics, the search counters and the work-queue heads.
__global__ void stats_init_kernel(CloudStats *st, int n_clouds, unsigned long long *counters,
                                  unsigned int *queue)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c < 8) {
        counters[c] = 0;
        queue[c] = 0;
    }
    if (c >= n_clouds)
        return;
    for (int a = 0; a < 4; ++a) {
        st[c].mn[a] = ~0ull;
        st[c].mx[a] = 0ull;
    }
    for (int a = 0; a < 3; ++a) {
        st[c].pmn[a] = ~0ull;
        st[c].pmx[a] = 0ull;
    }
    st[c].nonfinite = 0;
}

// Per-block partial bounding boxes: part[(cloud * gridDim.x + block) * 16 + a], a < 7 the minima
// (ambient, then projected), 7 + a the maxima, 14 the count of non-finite points (as a double).
// bbox_reduce_kernel folds them per cloud (no contended atomics).
template <typename T, int NA>
__global__ __launch_bounds__(256) void bbox_kernel(const T *__restrict__ pts,
                                                   const int64_t *__restrict__ offsets, Proj pr,
                                                   double *__restrict__ part)
{
    const int c = blockIdx.y;
    const int64_t b = offsets[c], e = offsets[c + 1];
    double mn[7], mx[7]; // NA ambient, then 3 projected
#pragma unroll
    for (int a = 0; a < 7; ++a) {
        mn[a] = INFINITY;
        mx[a] = -INFINITY;
    }
    unsigned long long bad = 0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    // four points per trip, their loads issued together
    for (int64_t i0 = b + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i0 < e; i0 += 4 * stride) {
        T xs[4][NA];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t i = i0 + u * stride;
#pragma unroll
            for (int a = 0; a < NA; ++a)
                xs[u][a] = i < e ? pts[i * NA + a] : (T)0;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            if (i0 + u * stride >= e)
                break;
            const T *x = xs[u];
            bool fin = true;
#pragma unroll
            for (int a = 0; a < NA; ++a)
                fin = fin && isfinite((double)x[a]);
            if (!fin) {
                ++bad;
                continue;
            }
#pragma unroll
            for (int a = 0; a < NA; ++a) {
                mn[a] = fmin(mn[a], (double)x[a]);
                mx[a] = fmax(mx[a], (double)x[a]);
            }
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const double pu = (double)project<T, NA>(x, pr, a);
                mn[4 + a] = fmin(mn[4 + a], pu);
                mx[4 + a] = fmax(mx[4 + a], pu);
            }
        }
    }
    __shared__ double smn[4][7], smx[4][7];
    __shared__ unsigned long long sbad[4];
    const int w = threadIdx.x / kWave, l = lane_id();
#pragma unroll
    for (int a = 0; a < 7; ++a) {
        mn[a] = seg_min(mn[a], kWave);
        mx[a] = seg_max(mx[a], kWave);
    }
    bad = wave_sum(bad);
    if (l == 0) {
        for (int a = 0; a < 7; ++a) {
            smn[w][a] = mn[a];
            smx[w][a] = mx[a];
        }
        sbad[w] = bad;
    }
    __syncthreads();
    if (threadIdx.x < 15) {
        const int a = (int)threadIdx.x, nw = blockDim.x / kWave;
        double v;
        if (a < 7) {
            v = smn[0][a];
            for (int k = 1; k < nw; ++k)
                v = fmin(v, smn[k][a]);
        } else if (a < 14) {
            v = smx[0][a - 7];
            for (int k = 1; k < nw; ++k)
                v = fmax(v, smx[k][a - 7]);
        } else {
            unsigned long long tb = 0;
            for (int k = 0; k < nw; ++k)
                tb += sbad[k];
            v = (double)tb;
        }
        part[((int64_t)c * gridDim.x + blockIdx.x) * 16 + a] = v;
    }
}

// One block per cloud: folds the nb partial boxes of the cloud into its statistics.
template <int NA>
__global__ __launch_bounds__(256) void bbox_reduce_kernel(const double *__restrict__ part, int nb,
                                                          CloudStats *st)
{
    const int c = blockIdx.x;
    double mn[7], mx[7], bad = 0.0;
#pragma unroll
    for (int a = 0; a < 7; ++a) {
        mn[a] = INFINITY;
        mx[a] = -INFINITY;
    }
    for (int b = threadIdx.x; b < nb; b += blockDim.x) {
        const double *p = part + ((int64_t)c * nb + b) * 16;
#pragma unroll
        for (int a = 0; a < 7; ++a) {
            mn[a] = fmin(mn[a], p[a]);
            mx[a] = fmax(mx[a], p[7 + a]);
        }
        bad += p[14];
    }
    __shared__ double smn[4][7], smx[4][7], sbad[4];
    const int w = threadIdx.x / kWave, l = lane_id();
#pragma unroll
    for (int a = 0; a < 7; ++a) {
        mn[a] = seg_min(mn[a], kWave);
        mx[a] = seg_max(mx[a], kWave);
    }
    bad = wave_sum(bad);
    if (l == 0) {
        for (int a = 0; a < 7; ++a) {
            smn[w][a] = mn[a];
            smx[w][a] = mx[a];
        }
        sbad[w] = bad;
    }
    __syncthreads();
    if (threadIdx.x != 0)
        return;
    const int nw = blockDim.x / kWave;
    for (int a = 0; a < 7; ++a) {
        if (a >= NA && a < 4)
            continue;
        double lo = smn[0][a], hi = smx[0][a];
        for (int k = 1; k < nw; ++k) {
            lo = fmin(lo, smn[k][a]);
            hi = fmax(hi, smx[k][a]);
        }
        if (lo <= hi) {
            if (a < 4) {
                st[c].mn[a] = ord_encode(lo);
                st[c].mx[a] = ord_encode(hi);
            } else {
                st[c].pmn[a - 4] = ord_encode(lo);
                st[c].pmx[a - 4] = ord_encode(hi);
            }
        }
    }
    double tb = 0.0;
    for (int k = 0; k < nw; ++k)
        tb += sbad[k];
    st[c].nonfinite = (unsigned long long)tb;
}

// The cloud of global row i: the last cloud whose first row is at most i (row offsets off[0..nc]
// ascending; an empty cloud shares its first row with the next one).
__device__ __forceinline__ int cloud_of(const int64_t *__restrict__ off, int nc, int64_t i)
{
    int lo = 0, hi = nc - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (off[mid] <= i)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// Cell key and first-placement slot of every point, one thread per point over all clouds. The
// lanes of a wave take their clouds one at a time (almost always one), so the cloud's grid is
// read with scalar loads.
template <typename T, int NA>
__global__ __launch_bounds__(256) void key_kernel(const T *__restrict__ pts,
                                                  const int64_t *__restrict__ off, int n_clouds,
                                                  int64_t n_total,
                                                  const CloudGrid *__restrict__ grids,
                                                  const uint32_t *__restrict__ parts,
                                                  uint32_t *__restrict__ counts,
                                                  uint32_t *__restrict__ keys,
                                                  uint32_t *__restrict__ slots)
{
    for (int64_t i0 = (int64_t)blockIdx.x * blockDim.x; i0 < n_total;
         i0 += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = i0 + threadIdx.x;
        bool todo = i < n_total;
        const int c = todo ? cloud_of(off, n_clouds, i) : 0;
        T x[NA];
#pragma unroll
        for (int a = 0; a < NA; ++a)
            x[a] = todo ? pts[i * NA + a] : (T)0;
        for (;;) {
            const unsigned long long m = __ballot(todo);
            if (m == 0)
                break;
            const int cu = __builtin_amdgcn_readfirstlane(__shfl(c, __ffsll((long long)m) - 1, kWave));
            if (todo && c == cu) {
                const CloudGrid &g = grids[cu];
                int cc[3];
#pragma unroll
                for (int a = 0; a < 3; ++a)
                    cc[a] = cell_coord<T>(project<T, NA>(x, g.proj, a), g.lo[a], g.inv_cell, g.dim[a]);
                const uint32_t key = (uint32_t)g.cell0 + morton_of(parts, g, cc[0], cc[1], cc[2]);
                keys[i] = key;
                slots[i] = atomicAdd(&counts[key], 1u);
                todo = false;
            }
        }
    }
}

// First placement by the atomic slots (the order inside a cell depends on the race), one thread
// per point over all clouds.
template <typename T>
__global__ __launch_bounds__(256) void scatter_kernel(const T *__restrict__ pts, int n_amb,
                                                      int64_t n_total,
                                                      const uint32_t *__restrict__ cell_start,
                                                      const uint32_t *__restrict__ keys,
                                                      const uint32_t *__restrict__ slots,
                                                      Pt<T> *__restrict__ spts_tmp,
                                                      int32_t *__restrict__ perm_tmp)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t pos = cell_start[keys[i]] + slots[i];
        Pt<T> p;
        for (int a = 0; a < 4; ++a)
            p.v[a] = a < n_amb ? pts[i * n_amb + a] : (T)0;
        spts_tmp[pos] = p;
        perm_tmp[pos] = (int32_t)i;
    }
}

// Canonical order inside every cell: a point's final slot is the number of points of its cell
// with a smaller original index (O(m) per point for a cell of m points; the neighbour search
// already spends O(m) per query on such a cell). The result is the same on every run.
template <typename T>
__global__ __launch_bounds__(256) void canon_kernel(int64_t n_total,
                                                    const uint32_t *__restrict__ cell_start,
                                                    const uint32_t *__restrict__ keys,
                                                    const Pt<T> *__restrict__ spts_tmp,
                                                    const int32_t *__restrict__ perm_tmp,
                                                    Pt<T> *__restrict__ spts,
                                                    int32_t *__restrict__ perm,
                                                    int32_t *__restrict__ iperm)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n_total)
        return;
    const int32_t i = perm_tmp[s];
    const uint32_t key = keys[i];
    const uint32_t st = cell_start[key], en = cell_start[key + 1];
    uint32_t rank = 0;
    for (uint32_t t = st; t < en; ++t)
        rank += perm_tmp[t] < i;
    const int64_t dest = (int64_t)st + rank;
    spts[dest] = spts_tmp[s];
    perm[dest] = i;
    iperm[i] = (int32_t)dest;
}

// ---------------------------------------------------------------------------------------------
// grid planning on the device (one block per cloud), straight from the bounding boxes
// ---------------------------------------------------------------------------------------------
constexpr int kMaxDim = 1024; // cells per projected axis

// Per-cloud layout of the metadata array (int64, host-computed, uploaded once per call):
// [0, n]      row offsets (n + 1 entries)
// then n entries each of: first cell-table entry, cell budget, first 64-point group, first
// Morton part-table entry.
struct PlanArgs {
    const CloudStats *stats;
    const int64_t *meta;
    int32_t n_clouds;
    int32_t n_amb;
    int32_t K;
    int32_t d;             // manifold dimension (1: curves, 2: surfaces)
    double alpha;          // cell edge / estimated K-th neighbour distance
    double mu;             // initial search radius / estimated K-th neighbour distance
    Proj proj;
    CloudGrid *grids;
    uint32_t *parts;
};

__device__ __forceinline__ double ord_decode(unsigned long long u)
{
    const unsigned long long b = (u >> 63) ? (u & 0x7fffffffffffffffull) : ~u;
    return __longlong_as_double((long long)b);
}

// Cell edge from the estimated K-th neighbour distance of a surface sample (the area of a closed
// surface is taken as about half the surface of its projected bounding box) or of a curve sample
// (from an estimated length), coarsened until the
// power-of-two grid fits the cloud's cell budget; Morton part tables interleave the bits of the
// three cell coordinates (axes with fewer bits drop out of the higher levels).
__global__ __launch_bounds__(256) void plan_kernel(PlanArgs a)
{
    const int c = blockIdx.x;
    __shared__ int32_t dim_s[3];
    __shared__ int32_t pos_s[3][16];
    __shared__ int64_t part0_s;
    if (threadIdx.x == 0) {
        const CloudStats st = a.stats[c];
        const int64_t *m = a.meta + a.n_clouds + 1;
        const int64_t row0 = a.meta[c], n = a.meta[c + 1] - a.meta[c];
        const int64_t cell0 = m[c], cap = m[a.n_clouds + c];
        double diam2 = 0.0;
        for (int k = 0; k < a.n_amb; ++k) {
            const double e = ord_decode(st.mx[k]) - ord_decode(st.mn[k]);
            diam2 += e * e;
        }
        double Eb[3], lo[3];
        for (int k = 0; k < 3; ++k) {
            lo[k] = ord_decode(st.pmn[k]);
            Eb[k] = ord_decode(st.pmx[k]) - lo[k];
        }
        const double emax = fmax(fmax(Eb[0], fmax(Eb[1], Eb[2])), 1e-300);
        double Ef[3];
        for (int k = 0; k < 3; ++k)
            Ef[k] = fmax(Eb[k], emax * 1e-3);
        double dk;
        if (a.d == 2) {
            const double area = 0.55 * 2.0 * (Ef[0] * Ef[1] + Ef[1] * Ef[2] + Ef[0] * Ef[2]);
            dk = sqrt((double)a.K * area / (M_PI * (double)n));
        } else { // a closed curve is taken as about 1.6 times the sum of the box edges long
            const double len = 1.6 * (Eb[0] + Eb[1] + Eb[2]);
            dk = (double)a.K * len / (2.0 * (double)n);
        }
        if (!(dk > 0.0 && dk < 1e300)) // extent below the double range, or no finite point
            dk = (emax > 1e-300 && emax < 1e300) ? emax : 1.0;
        double cell = a.alpha * dk;
        int dim[3] = {1, 1, 1};
        bool fits = false;
        for (int it = 0; it < 400 && !fits; ++it) {
            int64_t total = 1;
            bool ok = true;
            for (int k = 0; k < 3; ++k) {
                double cnt = floor(Eb[k] / cell) + 1.0;
                if (!(cnt <= (double)kMaxDim)) {
                    ok = false;
                    cnt = (double)kMaxDim;
                }
                int d = 1;
                while (d < (int)cnt)
                    d <<= 1;
                dim[k] = d;
                total *= d;
            }
            fits = ok && total <= cap;
            if (!fits)
                cell *= 1.26;
        }
        if (!fits) { // a single cell (the search then scans the whole cloud)
            dim[0] = dim[1] = dim[2] = 1;
            cell = fmax(emax, 1e-300);
        }
        CloudGrid g;
        memset(&g, 0, sizeof g);
        g.row0 = row0;
        g.n = n;
        g.cell0 = cell0;
        g.group0 = m[2 * a.n_clouds + c];
        g.part0 = m[3 * a.n_clouds + c];
        g.proj = a.proj;
        for (int k = 0; k < 3; ++k) {
            g.lo[k] = lo[k];
            g.dim[k] = dim[k];
        }
        g.cell = cell;
        g.inv_cell = 1.0 / cell;
        g.diam2 = diam2;
        g.r0 = fmax(a.mu * dk, 0.5 * cell); // positive, so that radius growth reaches the box
        a.grids[c] = g;
        part0_s = g.part0;
        int bits[3], maxb = 0;
        for (int k = 0; k < 3; ++k) {
            bits[k] = 0;
            while ((1 << bits[k]) < dim[k])
                ++bits[k];
            maxb = bits[k] > maxb ? bits[k] : maxb;
        }
        int p = 0;
        for (int l = 0; l < maxb; ++l)
            for (int k = 0; k < 3; ++k)
                if (l < bits[k])
                    pos_s[k][l] = p++;
        for (int k = 0; k < 3; ++k)
            dim_s[k] = dim[k];
    }
    __syncthreads();
    const int total = dim_s[0] + dim_s[1] + dim_s[2];
    for (int t = threadIdx.x; t < total; t += blockDim.x) {
        const int k = t < dim_s[0] ? 0 : (t < dim_s[0] + dim_s[1] ? 1 : 2);
        const int x = t - (k == 0 ? 0 : (k == 1 ? dim_s[0] : dim_s[0] + dim_s[1]));
        uint32_t code = 0;
        for (int l = 0; (1 << l) < dim_s[k]; ++l)
            code |= (uint32_t)((x >> l) & 1) << pos_s[k][l];
        a.parts[part0_s + t] = code;
    }
}

// ---------------------------------------------------------------------------------------------
// exclusive prefix sum of uint32 (three-phase, recursive over block totals)
// ---------------------------------------------------------------------------------------------
constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanThreads * kScanItems;

__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t *total)
{
    __shared__ uint32_t warp_tot[kScanThreads / kWave];
    const int l = lane_id(), w = threadIdx.x / kWave;
    int incl = wave_incl_scan((int)v);
    if (l == kWave - 1)
        warp_tot[w] = (uint32_t)incl;
    __syncthreads();
    uint32_t base = 0, tot = 0;
    for (int k = 0; k < kScanThreads / kWave; ++k) {
        if (k < w)
            base += warp_tot[k];
        tot += warp_tot[k];
    }
    __syncthreads();
    *total = tot;
    return base + (uint32_t)incl - v;
}

__global__ __launch_bounds__(kScanThreads) void scan_tile_kernel(const uint32_t *__restrict__ in,
                                                                 uint32_t *__restrict__ out,
                                                                 uint32_t *__restrict__ tile_sums,
                                                                 int64_t n)
{
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    // a full run of eight: two 16-byte loads / stores (every scanned array starts 256-byte aligned)
    const bool whole = base + kScanItems <= n;
    uint32_t v[kScanItems], s = 0;
    if (whole) {
        const uint4 a = *(const uint4 *)(in + base), b = *(const uint4 *)(in + base + 4);
        v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
        v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
    } else {
        for (int k = 0; k < kScanItems; ++k)
            v[k] = (base + k < n) ? in[base + k] : 0u;
    }
#pragma unroll
    for (int k = 0; k < kScanItems; ++k)
        s += v[k];
    uint32_t tot;
    uint32_t off = block_excl_scan(s, &tot);
    uint32_t o[kScanItems];
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        o[k] = off;
        off += v[k];
    }
    if (whole) {
        *(uint4 *)(out + base) = make_uint4(o[0], o[1], o[2], o[3]);
        *(uint4 *)(out + base + 4) = make_uint4(o[4], o[5], o[6], o[7]);
    } else {
        for (int k = 0; k < kScanItems; ++k)
            if (base + k < n)
                out[base + k] = o[k];
    }
    if (threadIdx.x == 0)
        tile_sums[blockIdx.x] = tot;
}

__global__ __launch_bounds__(kScanThreads) void scan_add_kernel(uint32_t *__restrict__ out,
                                                                const uint32_t *__restrict__ tile_off,
                                                                int64_t n)
{
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    const uint32_t add = tile_off[blockIdx.x];
    for (int k = 4 * threadIdx.x; k < kScanTile; k += 4 * kScanThreads) {
        if (base + k + 4 <= n) {
            uint4 u = *(uint4 *)(out + base + k);
            u.x += add; u.y += add; u.z += add; u.w += add;
            *(uint4 *)(out + base + k) = u;
        } else {
            for (int j = 0; j < 4; ++j)
                if (base + k + j < n)
                    out[base + k + j] += add;
        }
    }
}

// out[n] receives the grand total.
__global__ void scan_total_kernel(const uint32_t *__restrict__ in, uint32_t *__restrict__ out, int64_t n)
{
    if (threadIdx.x == 0 && blockIdx.x == 0)
        out[n] = (n > 0) ? out[n - 1] + in[n - 1] : 0u;
}

} // namespace mvgd
