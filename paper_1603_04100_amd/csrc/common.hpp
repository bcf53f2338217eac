// common.hpp -- shared device-side definitions of the MVGD library (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mvgd {

constexpr int kWave = 64;
constexpr int kMaxK = 63;
constexpr int kBins = 64;              // per-lane histogram bins over the squared distance
constexpr int kBinWords = kBins / 2;   // two 16-bit counters per LDS dword
constexpr int kBndCap = 16;            // boundary candidates resolved exactly per lane
constexpr int kMaxBoxCells = 4096;     // sub-groups are split while their box is larger
constexpr float kRelBand = 4e-6f;      // bound on |f32 distance^2 - exact key| / key (+ margin)

// One cloud's cell grid. Points are binned on three of the ambient coordinates (the three of
// largest extent); cells are numbered in Morton order so that a run of consecutive sorted
// points is spatially compact.
struct CloudGrid {
    int64_t row0;      // first global row (= first sorted position) of the cloud
    int64_t n;         // points in the cloud
    int64_t cell0;     // first entry of the cloud in the global cell table
    int64_t group0;    // first 64-point work group of the cloud
    int64_t part0;     // offset of the cloud's Morton part tables (dim[0]+dim[1]+dim[2] entries)
    double lo[3];      // grid origin along the binning axes
    double inv_cell;   // 1 / cell edge
    double cell;       // cell edge
    double diam2;      // squared diameter of the cloud's bounding box (all ambient axes)
    int32_t dim[3];    // cells per binning axis (powers of two)
    int32_t axis[3];   // ambient coordinate of each binning axis
    int32_t m0;        // initial search margin, in cells
    int32_t pad;
};

// Point storage: coordinates padded to four components.
template <typename T> struct Pt;
template <> struct __attribute__((aligned(16))) Pt<float> {
    float v[4];
};
template <> struct __attribute__((aligned(32))) Pt<double> {
    double v[4];
};

template <typename T>
__device__ __forceinline__ Pt<T> load_pt(const Pt<T> *p, int64_t i)
{
    return p[i];
}

// Cell coordinate along one binning axis. The same expression is used when binning and when
// locating a query, so both see the same cell.
template <typename T>
__device__ __forceinline__ int cell_coord(T x, double lo, double inv, int dim)
{
    T t = (x - (T)lo) * (T)inv;
    int c = (int)floor(t);
    c = c < 0 ? 0 : c;
    return c > dim - 1 ? dim - 1 : c;
}

__device__ __forceinline__ uint32_t morton_of(const uint32_t *parts, const CloudGrid &g, int x, int y,
                                              int z)
{
    const uint32_t *p = parts + g.part0;
    return p[x] | p[g.dim[0] + y] | p[g.dim[0] + g.dim[1] + z];
}

// ---------------------------------------------------------------------------------------------
// wave-level helpers (wave64)
// ---------------------------------------------------------------------------------------------
__device__ __forceinline__ int lane_id()
{
    return (int)__lane_id();
}

template <typename V>
__device__ __forceinline__ V seg_min(V v, int width)
{
    for (int o = 1; o < width; o <<= 1) {
        V w = __shfl_xor(v, o, kWave);
        v = w < v ? w : v;
    }
    return v;
}

template <typename V>
__device__ __forceinline__ V seg_max(V v, int width)
{
    for (int o = 1; o < width; o <<= 1) {
        V w = __shfl_xor(v, o, kWave);
        v = w > v ? w : v;
    }
    return v;
}

template <typename V>
__device__ __forceinline__ V wave_sum(V v)
{
    for (int o = 1; o < kWave; o <<= 1)
        v += __shfl_xor(v, o, kWave);
    return v;
}

// inclusive prefix sum over the wave
__device__ __forceinline__ int wave_incl_scan(int v)
{
    const int l = lane_id();
    for (int o = 1; o < kWave; o <<= 1) {
        int w = __shfl_up(v, o, kWave);
        if (l >= o)
            v += w;
    }
    return v;
}

__device__ __forceinline__ int uniform(int v)
{
    return __builtin_amdgcn_readfirstlane(v);
}

// Ordered encoding of doubles for integer atomics (monotone in the value; NaN excluded by callers).
__device__ __forceinline__ unsigned long long ord_encode(double x)
{
    unsigned long long b = (unsigned long long)__double_as_longlong(x);
    return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}

} // namespace mvgd
