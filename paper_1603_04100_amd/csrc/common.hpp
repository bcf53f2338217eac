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

// Orthonormal projection R^n -> R^3 on which the points are binned (rows of W). For n = 3 it is
// the identity. For n = 4 it is a fixed generic orthonormal 3x4 matrix: binning on three of the
// four coordinates would fold symmetric sheets onto each other (e.g. phi and -phi of a flat
// torus (cos t, sin t, cos p, sin p)), doubling the candidates of every search. Any orthonormal
// projection is 1-Lipschitz, so a cell box of radius R around a query still contains every
// point within distance R of it.
struct Proj {
    double W[3][4];
};

// One cloud's cell grid over the projected coordinates; cells are numbered in Morton order so
// that a run of consecutive sorted points is spatially compact.
struct CloudGrid {
    int64_t row0;      // first global row (= first sorted position) of the cloud
    int64_t n;         // points in the cloud
    int64_t cell0;     // first entry of the cloud in the global cell table
    int64_t group0;    // first 64-point work group of the cloud
    int64_t part0;     // offset of the cloud's Morton part tables (dim[0]+dim[1]+dim[2] entries)
    Proj proj;         // binning projection
    double lo[3];      // grid origin along the projected axes
    double inv_cell;   // 1 / cell edge
    double cell;       // cell edge
    double diam2;      // squared diameter of the cloud's bounding box (all ambient axes)
    double r0;         // initial search radius (real units)
    int32_t dim[3];    // cells per projected axis (powers of two)
    int32_t pad;
};

// projected coordinate a of a point (explicit FMA chain: binning and query lookup evaluate it
// identically)
template <typename T, int NA>
__device__ __forceinline__ T project(const T *x, const Proj &pr, int a)
{
    T u = x[0] * (T)pr.W[a][0];
#pragma unroll
    for (int k = 1; k < NA; ++k)
        u = fma(x[k], (T)pr.W[a][k], u);
    return u;
}

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
    t = t > (T)-1 ? t : (T)-1; // also maps NaN to -1
    t = t < (T)dim ? t : (T)dim;
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
