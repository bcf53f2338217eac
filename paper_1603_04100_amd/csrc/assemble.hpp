// assemble.hpp -- fused per-point MVGD assembly: exact K nearest neighbours, PCA frame,
// quadratic least-squares fits, metric, virtual-grid stencil, sliced-ELL write.
//
// Mapping: one wave (64 lanes) per group of 64 consecutive cell-sorted points; lane = point.
// Because the points are sorted by Morton-ordered cell, a group is spatially compact and all
// of its lanes search the same box of cells: the wave streams the box's points through LDS in
// chunks of 64 (coalesced loads) and every lane reads each staged point as an LDS broadcast.
//
// Exact neighbour selection (the paper's "K nearest neighbours", Sec. 2; ties to the smaller
// index, the exact key being the FP64 sum ((d0^2 + d1^2) + d2^2) + d3^2 without contraction):
//   pass 1  per-lane histogram (64 bins, 16-bit counters in LDS) of the squared distance f over
//           [0, R^2], R the radius the box guarantees; grows the box until every lane counts K.
//   refine  optional second histogram inside the bin holding the K-th neighbour.
//   pass 2  with e = 4e-6 bounding |f - key|/key: f(1+e) < lo(1-e) is surely in (written to the
//           list); f(1-e) <= hi(1+e) is a boundary candidate, re-keyed exactly in FP64.
//   resolve the (K - #sure) smallest boundary candidates by (key, index), ranked in LDS.
//   slow    lanes whose boundary overflows (exact ties, extreme clustering) extract the missing
//           neighbours one at a time by (key, index) over repeated streams.
//
// Fit (per lane, Sec. 2 and Sec. 3.1; surfaces d = 2 and curves d = 1): covariance of N(i)
// about its barycentre accumulated in FP64 from exact differences; cyclic Jacobi in FP64 (frame:
// the d largest eigenvalues are tangent, the rest normal); local coordinates and the spacing
// h = 1/4 min tangent range
// (Eq. DefH); design monomials of (u/h) over {p_i} u N(i); Gram matrix accumulated in FP64;
// Cholesky in FP64; fits of the normal coordinates (Eq. poly); inverse metric G and drift q
// of the fitted graph (Eq. metric, Eq. eqn3); ell = (tau, -q1, -q2, 2G11, 2G12, 2G22),
// tau = 2 (G11 + G22)/h^2 (centre value U_i in the virtual-grid differences, Eq. centered1);
// y = Gram^-1 D ell; w = W V y, w_centre -= tau. W holds the least-squares weights: 1 at p_i
// and w_nbr at every neighbour (1: unweighted; 1/K: the moving-least-squares weights of the
// comparison method in Sec. 4), and the Gram matrix is V^T W V. In FP64 mode the surface fits
// and y each get one refinement step whose residual is formed from V itself (accuracy
// O(kappa(V) u), as a QR).
#pragma once

#include "common.hpp"

namespace mvgd {

struct AsmParams {
    const void *spts;           // Pt<T>[n_total], cell-sorted
    const int32_t *perm;        // sorted position -> global row
    const int32_t *iperm;       // global row -> sorted position
    const uint32_t *cell_start; // global cell table, exclusive prefix (cells + 1)
    const uint32_t *parts;      // Morton part tables
    const CloudGrid *grids;
    int32_t n_clouds;
    int32_t K;
    int64_t n_groups;
    int64_t groups_per_xcd;     // XCD-aware remap of workgroups to groups
    int32_t variant;            // 0 = MVGD, 1 = plain least squares, 2 = divergence form (d=1)
    int32_t use_h;
    double w_nbr;               // least-squares weight of every neighbour (p_i: 1)
    double h_override;
    int64_t ld;                 // sliced-ELL leading dimension
    int64_t n_rows;             // rows over all clouds
    int32_t *ell_col;           // [K+1][ld] sorted positions
    void *ell_val;              // [K+1][ld] weights (T)
    double *row_h;              // optional, sorted order
    uint8_t *row_flags;         // optional, sorted order
    unsigned int *queue;          // [8] per-XCD work-queue counters (persistent launch)
    unsigned long long *counters; // [0] degenerate rows, [1] slow-path rows, [2] internal errors,
                                  // [3] sub-groups, [4] candidates streamed, [5] radius growths
};

// LDS layout of one wave (bytes)
constexpr int kLdsHist = 0;                                 // u32 [kBinWords][64] | f64 [kBndCap][64]
constexpr int kLdsBndPos = kLdsHist + kBndCap * kWave * 8;  // i32 [kBndCap][64] (indices)
constexpr int kLdsSearch = kLdsBndPos + kBndCap * kWave * 4; // group search staging
static_assert(kBinWords * kWave * 4 <= kBndCap * kWave * 8, "histogram must fit the key area");

// Staging of one group / tile stream (S = 0: coordinates of 64 points, their sorted positions
// and original indices; S = 2: the 64 candidates' six augmented operands, positions, indices).
constexpr int kTileStage = 6 * kWave * 4 + 2 * kWave * 4;
__host__ __device__ constexpr int search_stage_bytes(int pt_bytes, int S)
{
    // the tile search's exhaustive fallback streams through the group staging in the same area
    return S == 2 ? (kTileStage > kWave * pt_bytes + 2 * kWave * 4 ? kTileStage
                                                                   : kWave * pt_bytes + 2 * kWave * 4)
                  : kWave * pt_bytes + 2 * kWave * 4;
}

// LDS of one search wave (S: 0 group, 1 lane, 2 tile): histogram / boundary keys and indices,
// plus (group and tile search) the cell ranges, the staging and the sub-group worklist
__host__ __device__ constexpr int search_lds_bytes(int pt_bytes, int S)
{
    return kLdsSearch + (S == 1 ? 0
                                : 2 * kWave * 4 /*cell ranges*/ + search_stage_bytes(pt_bytes, S) +
                                      kWave * 8 /*worklist*/);
}

// LDS of one fit wave: the neighbour list [K][64]
__host__ __device__ constexpr int fit_lds_bytes(int K)
{
    return K * kWave * 4;
}

template <typename T, int NA>
__device__ __forceinline__ double exact_key(const Pt<T> &q, const Pt<T> &c)
{
#pragma clang fp contract(off)
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < NA; ++k) {
        double d = (double)c.v[k] - (double)q.v[k];
        double sq = d * d;
        s = (k == 0) ? sq : s + sq;
    }
    return s;
}

// squared distance used for culling: FP32 for float points, the exact key rounded for doubles
template <typename T, int NA>
__device__ __forceinline__ float cull_dist(const Pt<T> &q, const Pt<T> &c);

template <>
__device__ __forceinline__ float cull_dist<float, 2>(const Pt<float> &q, const Pt<float> &c)
{
    float d0 = c.v[0] - q.v[0], d1 = c.v[1] - q.v[1];
    return fmaf(d1, d1, d0 * d0);
}
template <>
__device__ __forceinline__ float cull_dist<float, 3>(const Pt<float> &q, const Pt<float> &c)
{
    float d0 = c.v[0] - q.v[0], d1 = c.v[1] - q.v[1], d2 = c.v[2] - q.v[2];
    return fmaf(d2, d2, fmaf(d1, d1, d0 * d0));
}
template <>
__device__ __forceinline__ float cull_dist<float, 4>(const Pt<float> &q, const Pt<float> &c)
{
    float d0 = c.v[0] - q.v[0], d1 = c.v[1] - q.v[1], d2 = c.v[2] - q.v[2], d3 = c.v[3] - q.v[3];
    return fmaf(d3, d3, fmaf(d2, d2, fmaf(d1, d1, d0 * d0)));
}
template <>
__device__ __forceinline__ float cull_dist<double, 2>(const Pt<double> &q, const Pt<double> &c)
{
    return (float)exact_key<double, 2>(q, c);
}
template <>
__device__ __forceinline__ float cull_dist<double, 3>(const Pt<double> &q, const Pt<double> &c)
{
    return (float)exact_key<double, 3>(q, c);
}
template <>
__device__ __forceinline__ float cull_dist<double, 4>(const Pt<double> &q, const Pt<double> &c)
{
    return (float)exact_key<double, 4>(q, c);
}

// Stream every point of the cell box [bmin, bmax] of cloud g through LDS, 64 at a time, and call
// The cell of a batch (its lane) that holds stream slot tt < total: the last cell whose first slot
// is at most tt (an empty cell shares its first slot with the next one, so the last such cell is
// never empty). Two levels: the first slots of cells 8, 16, ..., 56 (wave-uniform, p8[1..7]) pick
// a run of eight cells, whose first slots are then read from LDS together.
__device__ __forceinline__ int slot_cell(int tt, const int (&p8)[8], const int32_t *rng_pref)
{
    int c = 0;
#pragma unroll
    for (int i = 1; i < 8; ++i)
        c += p8[i] <= tt ? 1 : 0;
    const int4 a = *(const int4 *)(rng_pref + 8 * c);
    const int4 b = *(const int4 *)(rng_pref + 8 * c + 4);
    const int f = (a.y <= tt ? 1 : 0) + (a.z <= tt ? 1 : 0) + (a.w <= tt ? 1 : 0) +
                  (b.x <= tt ? 1 : 0) + (b.y <= tt ? 1 : 0) + (b.z <= tt ? 1 : 0) +
                  (b.w <= tt ? 1 : 0);
    return 8 * c + f;
}

// visit(f, point, sorted position, original index) on every lane for every point, where f is the
// culling distance of the point to the lane's query (+inf for inactive lanes and for the query
// itself). Staged entries past the end of the stream are sentinels (position -1, coordinates
// 1e30), so the visit loop runs in blocks of four whose LDS reads are issued one block ahead.
template <typename T, int NA, typename F>
__device__ __forceinline__ int stream_box(const AsmParams &P, const CloudGrid &g, const int bmin[3],
                                          const int bmax[3], char *lds_rng, char *lds_stage,
                                          const Pt<T> &qp, int q, bool act, F &&visit)
{
    const int lane = lane_id();
    const Pt<T> *spts = (const Pt<T> *)P.spts;
    int32_t *rng_start = (int32_t *)lds_rng;
    int32_t *rng_pref = rng_start + kWave;
    Pt<T> *st_pt = (Pt<T> *)lds_stage;
    int32_t *st_pos = (int32_t *)(lds_stage + kWave * sizeof(Pt<T>));
    int32_t *st_idx = st_pos + kWave;
    const int nx = uniform(bmax[0] - bmin[0] + 1), ny = uniform(bmax[1] - bmin[1] + 1),
              nz = uniform(bmax[2] - bmin[2] + 1);
    const int bx0 = uniform(bmin[0]), by0 = uniform(bmin[1]), bz0 = uniform(bmin[2]);
    const int nyz = ny * nz, ncells = nx * nyz;
    int streamed = 0;
    for (int cb = 0; cb < ncells; cb += kWave) {
        const int t = cb + lane;
        uint32_t st = 0, cn = 0;
        if (t < ncells) {
            const int x = (int)((uint32_t)t / (uint32_t)nyz);
            const int r = t - x * nyz;
            const int y = (int)((uint32_t)r / (uint32_t)nz);
            const int z = r - y * nz;
            const uint32_t cell = (uint32_t)g.cell0 + morton_of(P.parts, g, bx0 + x, by0 + y, bz0 + z);
            st = P.cell_start[cell];
            cn = P.cell_start[cell + 1] - st;
        }
        const int incl = wave_incl_scan((int)cn);
        const int total = uniform(__shfl(incl, kWave - 1, kWave));
        streamed += total;
        rng_start[lane] = (int32_t)st;
        rng_pref[lane] = incl - (int)cn;
        int p8[8];
#pragma unroll
        for (int i = 0; i < 8; ++i)
            p8[i] = __builtin_amdgcn_readlane(incl - (int)cn, 8 * i);
        __syncthreads();
        for (int sb = 0; sb < total; sb += kWave) {
            const int tt = sb + lane;
            if (tt < total) {
                const int lo = slot_cell(tt, p8, rng_pref);
                const int pos = rng_start[lo] + (tt - rng_pref[lo]);
                st_pt[lane] = spts[pos];
                st_pos[lane] = pos;
                st_idx[lane] = P.perm[pos];
            } else {
                Pt<T> sentinel;
#pragma unroll
                for (int a = 0; a < 4; ++a)
                    sentinel.v[a] = (T)1e30;
                st_pt[lane] = sentinel;
                st_pos[lane] = -1;
                st_idx[lane] = 0x7fffffff;
            }
            __syncthreads();
            const int nst4 = (min(kWave, total - sb) + 3) & ~3;
            Pt<T> c0 = st_pt[0], c1 = st_pt[1], c2 = st_pt[2], c3 = st_pt[3];
            int4 pp = *(const int4 *)(st_pos), ii = *(const int4 *)(st_idx);
            for (int j = 0; j < nst4; j += 4) {
                const int jn = min(j + 4, kWave - 4);
                const Pt<T> n0 = st_pt[jn], n1 = st_pt[jn + 1], n2 = st_pt[jn + 2], n3 = st_pt[jn + 3];
                const int4 np = *(const int4 *)(st_pos + jn), ni = *(const int4 *)(st_idx + jn);
                const float inf = INFINITY;
                const float f0 = (act && pp.x != q) ? cull_dist<T, NA>(qp, c0) : inf;
                const float f1 = (act && pp.y != q) ? cull_dist<T, NA>(qp, c1) : inf;
                const float f2 = (act && pp.z != q) ? cull_dist<T, NA>(qp, c2) : inf;
                const float f3 = (act && pp.w != q) ? cull_dist<T, NA>(qp, c3) : inf;
                visit(f0, c0, pp.x, ii.x);
                visit(f1, c1, pp.y, ii.y);
                visit(f2, c2, pp.z, ii.z);
                visit(f3, c3, pp.w, ii.w);
                c0 = n0; c1 = n1; c2 = n2; c3 = n3;
                pp = np; ii = ni;
            }
            __syncthreads();
        }
    }
    return streamed;
}

// ---------------------------------------------------------------------------------------------
// tile search: squared distances of a 64-query x 64-candidate tile on the matrix cores
// ---------------------------------------------------------------------------------------------
// About a centre c (a query of the sub-group), with q^ = q - c and p^ = p - c formed in the
// points' precision and rounded once to FP32 (float or double points alike),
//   g(q, p) = |q^|^2 + (1 + kTileAdd) |p^|^2 - 2 q^ . p^
// is one dot product of the augmented vectors (-2 q^, 1, |q^|^2) and (p^, (1 + kTileAdd)|p^|^2, 1),
// six terms, formed by three v_mfma_f32_32x32x2f32 per 32 x 32 block. Its error against the
// exact key (FP64, no contraction) obeys |f - key| <= e key + kTileErr (|p^|^2 + |q^|^2) for the
// plain value f (FP32 rounding of the centring, the norms and the six-term sum: below 20 u with
// u = 2^-24); kTileErr = 4e-6 leaves a factor three. The extra kTileAdd |p^|^2 makes g an
// upper-biased estimate whose bounds involve |q^|^2 only:
//   key <= (g + kTileErr |q^|^2) / (1 - e),
//   g   <= key (1 + e + 2 c) + (kTileErr + 2 c) |q^|^2,  c = kTileErr + kTileAdd + u,
// the second from |p^|^2 <= 2 |q^|^2 + 2 key. The selection thresholds below follow from these.
constexpr float kTileErr = 4e-6f;
constexpr float kTileAdd = 8e-6f;
constexpr double kTilePeel = 100.0; // queries of one tile stream lie within sqrt(kTilePeel) r0 of c
constexpr int kTileBins = 32;       // histogram bins per query (32-bit counters)
static_assert((kTileBins + 1) * kWave * 4 <= kLdsSearch, "tile histogram (+ past-cut row) must fit");
constexpr double kTileC = 4e-6 + 8e-6 + 6e-8;
constexpr double kTileU1 = 1.0 + 4e-6 + 2.0 * kTileC; // key coefficient of the upper bound on g
constexpr double kTileU0 = 4e-6 + 2.0 * kTileC;       // |q^|^2 coefficient of the upper bound on g

typedef float floatx16 __attribute__((ext_vector_type(16)));

// Stream every point of the cell box [bmin, bmax] of cloud g through LDS, 64 candidates at a
// time, and call consume(cb, qb, acc) for each of the four 32 x 32 blocks of g(query, candidate):
// in block (cb, qb) lane l holds query 32 qb + l % 32 against the candidates
// 32 cb + 8 (r / 4) + 4 (l / 32) + r % 4 in acc[r], r = 0..15 (the accumulator layout of the
// 32x32x2 instruction). bq[qb][s] are the query operands (augmented component 2 s + l / 32 of query
// 32 qb + l % 32). Staged entries past the end of the stream get g ~ 3e38 (never selected: every
// threshold is at most 1e38) and original index 0x7fffffff.
// Staged sorted positions and original indices are in st_pos / st_idx for the consumer.
template <typename T, int NA, typename F>
__device__ __forceinline__ int stream_tile(const AsmParams &P, const CloudGrid &g, const int bmin[3],
                                           const int bmax[3], char *lds_rng, char *lds_stage,
                                           const T cq[4], const float (&bq)[2][3], int qmask,
                                           F &&consume)
{
    const int lane = lane_id();
    const int hl = lane >> 5, ll = lane & 31;
    const Pt<T> *spts = (const Pt<T> *)P.spts;
    int32_t *rng_start = (int32_t *)lds_rng;
    int32_t *rng_pref = rng_start + kWave;
    float *st_aug = (float *)lds_stage;
    int32_t *st_pos = (int32_t *)(lds_stage + 6 * kWave * 4);
    int32_t *st_idx = st_pos + kWave;
    const int nx = uniform(bmax[0] - bmin[0] + 1), ny = uniform(bmax[1] - bmin[1] + 1),
              nz = uniform(bmax[2] - bmin[2] + 1);
    const int bx0 = uniform(bmin[0]), by0 = uniform(bmin[1]), bz0 = uniform(bmin[2]);
    const int nyz = ny * nz, ncells = nx * nyz;
    // (first sorted position, count) of cell cbase + lane of the box
    auto load_cells = [&](int cbase, uint32_t &st, uint32_t &cn) {
        const int t = cbase + lane;
        st = 0;
        cn = 0;
        if (t < ncells) {
            const int x = (int)((uint32_t)t / (uint32_t)nyz);
            const int r = t - x * nyz;
            const int y = (int)((uint32_t)r / (uint32_t)nz);
            const int z = r - y * nz;
            const uint32_t cell = (uint32_t)g.cell0 + morton_of(P.parts, g, bx0 + x, by0 + y, bz0 + z);
            st = P.cell_start[cell];
            cn = P.cell_start[cell + 1] - st;
        }
    };
    int p8[8]; // first slots of cells 8 i of the current batch
    // the point of stream slot tt of the current cell batch (ranges in LDS), or none
    auto load_point = [&](int tt, int total, Pt<T> &p, int32_t &pos, int32_t &idx) {
        pos = -1;
        idx = 0x7fffffff;
        if (tt < total) {
            const int lo = slot_cell(tt, p8, rng_pref);
            pos = rng_start[lo] + (tt - rng_pref[lo]);
            p = spts[pos];
            idx = P.perm[pos];
        }
    };
    int streamed = 0;
    // The next cell batch and the next chunk of points are loaded while the current chunk is on
    // the matrix cores.
    uint32_t st_n, cn_n;
    load_cells(0, st_n, cn_n);
    for (int cbase = 0; cbase < ncells; cbase += kWave) {
        const uint32_t st = st_n, cn = cn_n;
        if (cbase + kWave < ncells)
            load_cells(cbase + kWave, st_n, cn_n);
        const int incl = wave_incl_scan((int)cn);
        const int total = uniform(__shfl(incl, kWave - 1, kWave));
        streamed += total;
        rng_start[lane] = (int32_t)st;
        rng_pref[lane] = incl - (int)cn;
#pragma unroll
        for (int i = 0; i < 8; ++i)
            p8[i] = __builtin_amdgcn_readlane(incl - (int)cn, 8 * i);
        __syncthreads();
        Pt<T> p_n = {{(T)0, (T)0, (T)0, (T)0}};
        int32_t pos_n, idx_n;
        load_point(lane, total, p_n, pos_n, idx_n);
        for (int sb = 0; sb < total; sb += kWave) {
            float av[6] = {0.f, 0.f, 0.f, 0.f, 3e38f, 1.f};
            if (pos_n >= 0) {
                float np = 0.f;
#pragma unroll
                for (int a = 0; a < 4; ++a) {
                    av[a] = (float)(p_n.v[a] - cq[a]); // centred in T, rounded once to FP32
                    np = fmaf(av[a], av[a], np);
                }
                av[4] = np * (1.f + kTileAdd);
            }
#pragma unroll
            for (int a = 0; a < 6; ++a)
                st_aug[a * kWave + lane] = av[a];
            st_pos[lane] = pos_n;
            st_idx[lane] = idx_n;
            __syncthreads();
            if (sb + kWave < total)
                load_point(sb + kWave + lane, total, p_n, pos_n, idx_n);
            const int nblk = (min(kWave, total - sb) + 31) >> 5;
            for (int cb = 0; cb < nblk; ++cb) {
                const float a0 = st_aug[hl * kWave + 32 * cb + ll];
                const float a1 = st_aug[(2 + hl) * kWave + 32 * cb + ll];
                const float a2 = st_aug[(4 + hl) * kWave + 32 * cb + ll];
                floatx16 acc0 = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f,
                                 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
                if (qmask == 3) {
                    // both query blocks' chains are issued before either is consumed
                    floatx16 acc1 = acc0;
                    acc0 = __builtin_amdgcn_mfma_f32_32x32x2f32(a0, bq[0][0], acc0, 0, 0, 0);
                    acc1 = __builtin_amdgcn_mfma_f32_32x32x2f32(a0, bq[1][0], acc1, 0, 0, 0);
                    acc0 = __builtin_amdgcn_mfma_f32_32x32x2f32(a1, bq[0][1], acc0, 0, 0, 0);
                    acc1 = __builtin_amdgcn_mfma_f32_32x32x2f32(a1, bq[1][1], acc1, 0, 0, 0);
                    acc0 = __builtin_amdgcn_mfma_f32_32x32x2f32(a2, bq[0][2], acc0, 0, 0, 0);
                    acc1 = __builtin_amdgcn_mfma_f32_32x32x2f32(a2, bq[1][2], acc1, 0, 0, 0);
                    consume(cb, 0, acc0);
                    consume(cb, 1, acc1);
                } else if (qmask == 1) { // the second query block holds no active query
                    acc0 = __builtin_amdgcn_mfma_f32_32x32x2f32(a0, bq[0][0], acc0, 0, 0, 0);
                    acc0 = __builtin_amdgcn_mfma_f32_32x32x2f32(a1, bq[0][1], acc0, 0, 0, 0);
                    acc0 = __builtin_amdgcn_mfma_f32_32x32x2f32(a2, bq[0][2], acc0, 0, 0, 0);
                    consume(cb, 0, acc0);
                } else { // the first query block holds no active query
                    acc0 = __builtin_amdgcn_mfma_f32_32x32x2f32(a0, bq[1][0], acc0, 0, 0, 0);
                    acc0 = __builtin_amdgcn_mfma_f32_32x32x2f32(a1, bq[1][1], acc0, 0, 0, 0);
                    acc0 = __builtin_amdgcn_mfma_f32_32x32x2f32(a2, bq[1][2], acc0, 0, 0, 0);
                    consume(cb, 1, acc0);
                }
            }
            __syncthreads();
        }
    }
    return streamed;
}

// float rounded towards -inf / +inf from a double (conservative thresholds); f32_up saturates at
// 1e38, so that a threshold never admits the ~3e38 of a sentinel
__device__ __forceinline__ float f32_down(double x)
{
    float f = (float)x;
    return ((double)f > x) ? nextafterf(f, -INFINITY) : f;
}
__device__ __forceinline__ float f32_up(double x)
{
    float f = (float)x;
    f = ((double)f < x) ? nextafterf(f, INFINITY) : f;
    return fminf(f, 1e38f);
}

// Byte offset of the histogram row of a tile value: row round(x s) clamped to [0, top], times one
// row of 64 lanes. The rounding is that of fma(x, s, 2^23), whose low mantissa bits are the
// integer; shifting by 8 drops the exponent bits and scales the row by kWave * 4 bytes.
static_assert(kWave * 4 == 256, "row stride is 256 bytes");
__device__ __forceinline__ uint32_t tile_bin_offset(float x, float s, float top)
{
    const float y = __builtin_amdgcn_fmed3f(fmaf(x, s, 8388608.f), 8388608.f, 8388608.f + top);
    return (uint32_t)__float_as_uint(y) << 8;
}

// ---------------------------------------------------------------------------------------------
// small dense FP64 kernels (per lane, fully unrolled)
// ---------------------------------------------------------------------------------------------
template <int N>
__device__ __forceinline__ void jacobi_eig(double A[N][N], double W[N][N])
{
#pragma unroll
    for (int r = 0; r < N; ++r)
#pragma unroll
        for (int c = 0; c < N; ++c)
            W[r][c] = (r == c) ? 1.0 : 0.0;
    for (int sweep = 0; sweep < 12; ++sweep) {
        double off = 0.0, dia = 0.0;
#pragma unroll
        for (int p = 0; p < N; ++p) {
            dia += A[p][p] * A[p][p];
#pragma unroll
            for (int q = p + 1; q < N; ++q)
                off += A[p][q] * A[p][q];
        }
        const bool done = !(off > 1e-34 * dia);
        if (__ballot(!done) == 0)
            break;
        // a converged lane takes no further rotation: its result does not depend on how long the
        // other lanes of its wave iterate (the same row gives the same bits in any batch)
        if (done)
            continue;
#pragma unroll
        for (int p = 0; p < N; ++p) {
#pragma unroll
            for (int q = p + 1; q < N; ++q) {
                const double apq = A[p][q];
                double c = 1.0, s = 0.0;
                if (apq != 0.0) {
                    const double theta = (A[q][q] - A[p][p]) / (2.0 * apq);
                    double t = 1.0 / (fabs(theta) + sqrt(fma(theta, theta, 1.0)));
                    t = theta < 0.0 ? -t : t;
                    c = 1.0 / sqrt(fma(t, t, 1.0));
                    s = t * c;
                }
#pragma unroll
                for (int k = 0; k < N; ++k) {
                    const double akp = A[k][p], akq = A[k][q];
                    A[k][p] = c * akp - s * akq;
                    A[k][q] = s * akp + c * akq;
                }
#pragma unroll
                for (int k = 0; k < N; ++k) {
                    const double apk = A[p][k], aqk = A[q][k];
                    A[p][k] = c * apk - s * aqk;
                    A[q][k] = s * apk + c * aqk;
                }
#pragma unroll
                for (int k = 0; k < N; ++k) {
                    const double wkp = W[k][p], wkq = W[k][q];
                    W[k][p] = c * wkp - s * wkq;
                    W[k][q] = s * wkp + c * wkq;
                }
            }
        }
    }
}

// =============================================================================================
// per-lane fit: frame, spacing, least-squares fits, coefficients and the row (d = 1 or 2)
// =============================================================================================
template <int D> struct FitShape {
    static constexpr int M = (D == 2) ? 6 : 3;  // monomials of degree <= 2 in D variables
    static constexpr int NG = M * (M + 1) / 2;  // packed Gram entries
};

// packed upper triangle of an M x M symmetric matrix: index of (i, j), i <= j
template <int M>
__host__ __device__ constexpr int symM(int i, int j)
{
    return i * M - i * (i - 1) / 2 + (j - i);
}

// In-place Cholesky G = L L^T (L(j,i) stored at symM(i,j)). Returns false when a pivot is not
// positive or min L_ii < 1e-6 max L_ii.
template <int M>
__device__ __forceinline__ bool chol_packed(double G[M * (M + 1) / 2], double inv_diag[M])
{
    double dmin = INFINITY, dmax = 0.0;
    bool ok = true;
#pragma unroll
    for (int i = 0; i < M; ++i) {
        double s = G[symM<M>(i, i)];
#pragma unroll
        for (int k = 0; k < i; ++k)
            s -= G[symM<M>(k, i)] * G[symM<M>(k, i)];
        ok = ok && (s > 0.0);
        const double lii = sqrt(s > 0.0 ? s : 0.0);
        G[symM<M>(i, i)] = lii;
        inv_diag[i] = lii > 0.0 ? 1.0 / lii : 0.0;
        dmin = fmin(dmin, lii);
        dmax = fmax(dmax, lii);
#pragma unroll
        for (int j = i + 1; j < M; ++j) {
            double t = G[symM<M>(i, j)];
#pragma unroll
            for (int k = 0; k < i; ++k)
                t -= G[symM<M>(k, j)] * G[symM<M>(k, i)];
            G[symM<M>(i, j)] = t * inv_diag[i];
        }
    }
    return ok && (dmin >= 1e-6 * dmax) && isfinite(dmax);
}

// solve (L L^T) x = b in place
template <int M>
__device__ __forceinline__ void chol_packed_solve(const double L[M * (M + 1) / 2],
                                                  const double inv_diag[M], double b[M])
{
#pragma unroll
    for (int i = 0; i < M; ++i) {
        double s = b[i];
#pragma unroll
        for (int k = 0; k < i; ++k)
            s -= L[symM<M>(k, i)] * b[k];
        b[i] = s * inv_diag[i];
    }
#pragma unroll
    for (int i = M - 1; i >= 0; --i) {
        double s = b[i];
#pragma unroll
        for (int k = i + 1; k < M; ++k)
            s -= L[symM<M>(i, k)] * b[k];
        b[i] = s * inv_diag[i];
    }
}

// design monomials of the scaled local coordinates: (1, xi, eta, xi^2, xi eta, eta^2) for
// surfaces, (1, xi, xi^2) for curves (products formed in T, widened to double)
template <typename T, int D>
__device__ __forceinline__ void monomials(const T u[D], T ih, double m[FitShape<D>::M])
{
    const T xi = u[0] * ih;
    m[0] = 1.0;
    m[1] = (double)xi;
    if constexpr (D == 2) {
        const T eta = u[1] * ih;
        m[2] = (double)eta;
        m[3] = (double)(xi * xi);
        m[4] = (double)(xi * eta);
        m[5] = (double)(eta * eta);
    } else {
        m[2] = (double)(xi * xi);
    }
}

// local coordinates of p_j - p_i: tangent u (D) and normal z (NA - D)
template <typename T, int NA, int D>
__device__ __forceinline__ void local_coords(const Pt<T> &pj, const Pt<T> &qp,
                                             const T tf[D][NA], const T nf[NA - D][NA], T u[D],
                                             T z[NA - D])
{
#pragma unroll
    for (int t = 0; t < D; ++t)
        u[t] = 0;
#pragma unroll
    for (int c = 0; c < NA - D; ++c)
        z[c] = 0;
#pragma unroll
    for (int a = 0; a < NA; ++a) {
        const T d = pj.v[a] - qp.v[a];
#pragma unroll
        for (int t = 0; t < D; ++t)
            u[t] += tf[t][a] * d;
#pragma unroll
        for (int c = 0; c < NA - D; ++c)
            z[c] += nf[c][a] * d;
    }
}

template <typename T, int NA, int D>
__device__ __forceinline__ void fit_row(const AsmParams &P, const Pt<T> *spts,
                                        const int32_t *list, int lane, int q, const Pt<T> &qp,
                                        bool slow_row)
{
    constexpr int NC = NA - D; // normal coordinates
    constexpr int M = FitShape<D>::M;
    constexpr int NG = FitShape<D>::NG;
    const int K = P.K;
    T *val = (T *)P.ell_val;
    double qd[NA];
#pragma unroll
    for (int a = 0; a < NA; ++a)
        qd[a] = (double)qp.v[a];

    // covariance about the barycentre of N(i) (p_i excluded), FP64 from exact differences
    double s1[NA], s2[NA][NA];
#pragma unroll
    for (int a = 0; a < NA; ++a) {
        s1[a] = 0.0;
#pragma unroll
        for (int c = 0; c < NA; ++c)
            s2[a][c] = 0.0;
    }
#pragma unroll 4
    for (int k = 0; k < K; ++k) {
        const Pt<T> pj = spts[list[k * kWave + lane]];
        double dv[NA];
#pragma unroll
        for (int a = 0; a < NA; ++a) {
            dv[a] = (double)pj.v[a] - qd[a];
            s1[a] += dv[a];
        }
#pragma unroll
        for (int a = 0; a < NA; ++a)
#pragma unroll
            for (int c = a; c < NA; ++c)
                s2[a][c] = fma(dv[a], dv[c], s2[a][c]);
    }
    const double invK = 1.0 / (double)K;
    double A[NA][NA], W[NA][NA];
#pragma unroll
    for (int a = 0; a < NA; ++a)
#pragma unroll
        for (int c = a; c < NA; ++c) {
            A[a][c] = s2[a][c] - s1[a] * s1[c] * invK;
            A[c][a] = A[a][c];
        }
    jacobi_eig<NA>(A, W);
    double lam[NA];
    int rank[NA];
#pragma unroll
    for (int a = 0; a < NA; ++a)
        lam[a] = A[a][a];
#pragma unroll
    for (int a = 0; a < NA; ++a) {
        rank[a] = 0;
#pragma unroll
        for (int c = 0; c < NA; ++c)
            rank[a] += (c != a) && (lam[c] > lam[a] || (lam[c] == lam[a] && c < a));
    }
    // frame: the D largest eigenvalues' vectors are tangent, the rest normal
    T tf[D][NA], nf[NC][NA];
    double lam_t[D];
#pragma unroll
    for (int t = 0; t < D; ++t)
        lam_t[t] = 0.0;
#pragma unroll
    for (int a = 0; a < NA; ++a) {
#pragma unroll
        for (int t = 0; t < D; ++t)
            if (rank[a] == t)
                lam_t[t] = lam[a];
#pragma unroll
        for (int r = 0; r < NA; ++r) {
            const T v = (T)W[r][a];
#pragma unroll
            for (int t = 0; t < D; ++t)
                if (rank[a] == t)
                    tf[t][r] = v;
#pragma unroll
            for (int c = 0; c < NC; ++c)
                if (rank[a] == D + c)
                    nf[c][r] = v;
        }
    }

    // local coordinates and the spacing h (Eq. DefH and its two-dimensional form)
    T umin[D], umax[D];
#pragma unroll
    for (int t = 0; t < D; ++t) {
        umin[t] = (T)INFINITY;
        umax[t] = -(T)INFINITY;
    }
#pragma unroll 4
    for (int k = 0; k < K; ++k) {
        T u[D], z[NC];
        local_coords<T, NA, D>(spts[list[k * kWave + lane]], qp, tf, nf, u, z);
#pragma unroll
        for (int t = 0; t < D; ++t) {
            umin[t] = min(umin[t], u[t]);
            umax[t] = max(umax[t], u[t]);
        }
    }
    T range = umax[0] - umin[0];
#pragma unroll
    for (int t = 1; t < D; ++t)
        range = min(range, umax[t] - umin[t]);
    const T hT = (T)0.25 * range;
    double h = P.use_h ? P.h_override : (double)hT;
    bool degenerate = !(h > 0.0) || !isfinite(h);
    const T ih = degenerate ? (T)0 : (T)(1.0 / h);

    // Gram matrix of the design over {p_i} u N(i) and right-hand sides of the surface fits,
    // weighted: V^T W V and V^T W z with W = diag(1, w_nbr, ..., w_nbr)
    const double wn = P.w_nbr;
    double Gm[NG], rz[NC][M];
#pragma unroll
    for (int t = 0; t < NG; ++t)
        Gm[t] = 0.0;
    Gm[0] = 1.0; // centre row (1, 0, ..., 0)
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int t = 0; t < M; ++t)
            rz[c][t] = 0.0;
#pragma unroll 4
    for (int k = 0; k < K; ++k) {
        T u[D], z[NC];
        local_coords<T, NA, D>(spts[list[k * kWave + lane]], qp, tf, nf, u, z);
        double mv[M], wm[M];
        monomials<T, D>(u, ih, mv);
#pragma unroll
        for (int i = 0; i < M; ++i)
            wm[i] = wn * mv[i];
#pragma unroll
        for (int i = 0; i < M; ++i)
#pragma unroll
            for (int j = i; j < M; ++j)
                Gm[symM<M>(i, j)] = fma(wm[i], mv[j], Gm[symM<M>(i, j)]);
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const double zc = (double)z[c];
#pragma unroll
            for (int i = 0; i < M; ++i)
                rz[c][i] = fma(wm[i], zc, rz[c][i]);
        }
    }
    double inv_d[M];
    if (!degenerate)
        degenerate = !chol_packed<M>(Gm, inv_d);

    double y[M], tau = 0.0;
#pragma unroll
    for (int t = 0; t < M; ++t)
        y[t] = 0.0;
    if (!degenerate) {
        const double ihd = 1.0 / h, ih2 = ihd * ihd;
        double scale[M];
        scale[0] = 1.0;
#pragma unroll
        for (int t = 1; t <= D; ++t)
            scale[t] = ihd;
#pragma unroll
        for (int t = D + 1; t < M; ++t)
            scale[t] = ih2;
        // fitted graph of every normal coordinate (Eq. poly), unscaled coefficients
#pragma unroll
        for (int c = 0; c < NC; ++c)
            chol_packed_solve<M>(Gm, inv_d, rz[c]);
        if (sizeof(T) == 8) {
            // one refinement step of the surface fits, residual V^T W (z - V a) formed from V
            double res[NC][M];
#pragma unroll
            for (int c = 0; c < NC; ++c) {
#pragma unroll
                for (int t = 0; t < M; ++t)
                    res[c][t] = 0.0;
                res[c][0] = -rz[c][0]; // centre row e1 with z = 0
            }
#pragma unroll 4
            for (int k = 0; k < K; ++k) {
                T u[D], z[NC];
                local_coords<T, NA, D>(spts[list[k * kWave + lane]], qp, tf, nf, u, z);
                double mv[M];
                monomials<T, D>(u, ih, mv);
#pragma unroll
                for (int c = 0; c < NC; ++c) {
                    double e = (double)z[c];
#pragma unroll
                    for (int t = 0; t < M; ++t)
                        e = fma(-mv[t], rz[c][t], e);
                    e *= wn;
#pragma unroll
                    for (int t = 0; t < M; ++t)
                        res[c][t] = fma(mv[t], e, res[c][t]);
                }
            }
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                chol_packed_solve<M>(Gm, inv_d, res[c]);
#pragma unroll
                for (int t = 0; t < M; ++t)
                    rz[c][t] += res[c][t];
            }
        }
        double ell[M];
        bool ok = true;
        if constexpr (D == 2) {
            // inverse metric (Eq. metric) and the first-order coefficients of Eq. eqn3
            double g11 = 1.0, g12 = 0.0, g22 = 1.0;
            double zx[NC], zy[NC], h11[NC], h12[NC], h22[NC];
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                zx[c] = rz[c][1] * scale[1];
                zy[c] = rz[c][2] * scale[2];
                h11[c] = 2.0 * rz[c][3] * scale[3];
                h12[c] = rz[c][4] * scale[4];
                h22[c] = 2.0 * rz[c][5] * scale[5];
                g11 = fma(zx[c], zx[c], g11);
                g12 = fma(zx[c], zy[c], g12);
                g22 = fma(zy[c], zy[c], g22);
            }
            const double det = g11 * g22 - g12 * g12;
            const double idet = 1.0 / det;
            const double G11 = g22 * idet, G12 = -g12 * idet, G22 = g11 * idet;
            double q1 = 0.0, q2 = 0.0;
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                const double tr = G11 * h11[c] + 2.0 * G12 * h12[c] + G22 * h22[c];
                q1 = fma(tr, G11 * zx[c] + G12 * zy[c], q1);
                q2 = fma(tr, G12 * zx[c] + G22 * zy[c], q2);
            }
            tau = (P.variant == 0) ? 2.0 * (G11 + G22) * ih2 : 0.0;
            ell[0] = tau; ell[1] = -q1; ell[2] = -q2;
            ell[3] = 2.0 * G11; ell[4] = 2.0 * G12; ell[5] = 2.0 * G22;
            ok = det > 0.0;
        } else if (P.variant == 2) {
            // divergence form (Eq. divergence): s(x) = sqrt(1 + sum_c y_c'(x)^2) of the fitted
            // curve, a+- = 1 / (h^2 s(0) s(+-h/2)), L_i U = a+ U(h) + a- U(-h) - (a+ + a-) U_i
            double s0 = 1.0, sp = 1.0, sm = 1.0;
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                const double a1 = rz[c][1] * scale[1], a2 = rz[c][2] * scale[2];
                const double dp = a1 + a2 * h, dm = a1 - a2 * h; // y' at +-h/2
                s0 = fma(a1, a1, s0);
                sp = fma(dp, dp, sp);
                sm = fma(dm, dm, sm);
            }
            const double r0 = sqrt(s0);
            const double ap = ih2 / (r0 * sqrt(sp)), am = ih2 / (r0 * sqrt(sm));
            tau = ap + am;
            ell[0] = tau; ell[1] = (ap - am) * h; ell[2] = tau * h * h;
        } else {
            // Eq. LB1: G = 1 / (1 + |y'|^2), q = sum_c (G y_c'') (G y_c')
            double g = 1.0;
#pragma unroll
            for (int c = 0; c < NC; ++c)
                g = fma(rz[c][1] * scale[1], rz[c][1] * scale[1], g);
            const double G = 1.0 / g;
            double qs = 0.0;
#pragma unroll
            for (int c = 0; c < NC; ++c)
                qs = fma(G * 2.0 * rz[c][2] * scale[2], G * rz[c][1] * scale[1], qs);
            tau = (P.variant == 0) ? 2.0 * G * ih2 : 0.0;
            ell[0] = tau; ell[1] = -qs; ell[2] = 2.0 * G;
        }
        double dl[M];
#pragma unroll
        for (int t = 0; t < M; ++t) {
            dl[t] = ell[t] * scale[t];
            y[t] = dl[t];
        }
        chol_packed_solve<M>(Gm, inv_d, y);
        degenerate = !ok || !isfinite(tau) || !isfinite(y[0]);
        if (sizeof(T) == 8 && !degenerate) {
            // one refinement step on V^T W V y = D ell with the residual formed from V itself
            double res[M];
#pragma unroll
            for (int t = 0; t < M; ++t)
                res[t] = dl[t];
            res[0] -= y[0]; // centre row e1: (V y)_0 = y0
#pragma unroll 4
            for (int k = 0; k < K; ++k) {
                T u[D], z[NC];
                local_coords<T, NA, D>(spts[list[k * kWave + lane]], qp, tf, nf, u, z);
                double mv[M];
                monomials<T, D>(u, ih, mv);
                double w = 0.0;
#pragma unroll
                for (int t = 0; t < M; ++t)
                    w = fma(mv[t], y[t], w);
                w *= wn;
#pragma unroll
                for (int t = 0; t < M; ++t)
                    res[t] = fma(-w, mv[t], res[t]);
            }
            chol_packed_solve<M>(Gm, inv_d, res);
#pragma unroll
            for (int t = 0; t < M; ++t)
                y[t] += res[t];
        }
    }

    // weights w = W V y (centre: y0 - tau) into the sliced ELL, slot 0 = centre
    const int64_t ld = P.ld;
    P.ell_col[q] = q;
    val[q] = degenerate ? (T)0 : (T)(y[0] - tau);
#pragma unroll 4
    for (int k = 0; k < K; ++k) {
        const int pos = list[k * kWave + lane];
        double w = 0.0;
        if (!degenerate) {
            T u[D], z[NC];
            local_coords<T, NA, D>(spts[pos], qp, tf, nf, u, z);
            double mv[M];
            monomials<T, D>(u, ih, mv);
#pragma unroll
            for (int t = 0; t < M; ++t)
                w = fma(mv[t], y[t], w);
            w *= wn;
        }
        P.ell_col[(int64_t)(k + 1) * ld + q] = pos;
        val[(int64_t)(k + 1) * ld + q] = (T)w;
    }
    bool close_pair = false; // tangent eigenvalues within 1e-3 (in-plane frame ill-defined)
    if constexpr (D == 2)
        close_pair = (lam_t[0] - lam_t[1]) < 1e-3 * lam_t[0];
    if (P.row_h)
        P.row_h[q] = h;
    if (P.row_flags)
        P.row_flags[q] = (uint8_t)((degenerate ? 1 : 0) | (slow_row ? 2 : 0) | (close_pair ? 4 : 0));
    const unsigned long long nd = __popcll(__ballot(degenerate));
    if (lane == __ffsll((long long)__ballot(true)) - 1 && nd)
        atomicAdd(&P.counters[0], nd); // slow-path rows are counted by the search
}

// ---------------------------------------------------------------------------------------------
// per-lane search: every lane walks the cells of its own box (no shared staging)
// ---------------------------------------------------------------------------------------------
// Walk every point of the cell box [lo, hi] of this lane's query and call
// visit(f, point, sorted position) on it, f the culling distance (+inf for the query itself).
// Lanes step in lockstep; each step either visits one point or moves to the next cell (x
// fastest; Morton codes are advanced as dilated integers per axis). Returns the points visited.
template <typename T, int NA, typename F>
__device__ __forceinline__ int walk_box(const AsmParams &P, const CloudGrid &g, const int lo[3],
                                        const int hi[3], const Pt<T> &qp, int q, bool act,
                                        F &&visit)
{
    const Pt<T> *spts = (const Pt<T> *)P.spts;
    const uint32_t *px = P.parts + g.part0;
    const uint32_t *py = px + g.dim[0];
    const uint32_t *pz = py + g.dim[1];
    const uint32_t MX = px[g.dim[0] - 1], MY = py[g.dim[1] - 1], MZ = pz[g.dim[2] - 1];
    const uint32_t mx0 = px[lo[0]], my0 = py[lo[1]];
    uint32_t mx = mx0, my = my0, mz = pz[lo[2]];
    int x = lo[0], y = lo[1], z = lo[2];
    uint32_t t = 0, tend = 0;
    bool more = act;
    if (more) {
        const uint32_t cell = (uint32_t)g.cell0 + (mx | my | mz);
        t = P.cell_start[cell];
        tend = P.cell_start[cell + 1];
    }
    int visited = 0;
    while (__ballot(more) != 0) {
        if (more) {
            if (t < tend) {
                const Pt<T> c = spts[t];
                const float f = ((int)t != q) ? cull_dist<T, NA>(qp, c) : INFINITY;
                visit(f, c, (int)t);
                ++t;
                ++visited;
            } else {
                if (x < hi[0]) {
                    ++x;
                    mx = ((mx | ~MX) + 1u) & MX;
                } else {
                    x = lo[0];
                    mx = mx0;
                    if (y < hi[1]) {
                        ++y;
                        my = ((my | ~MY) + 1u) & MY;
                    } else {
                        y = lo[1];
                        my = my0;
                        if (z < hi[2]) {
                            ++z;
                            mz = ((mz | ~MZ) + 1u) & MZ;
                        } else {
                            more = false;
                        }
                    }
                }
                if (more) {
                    const uint32_t cell = (uint32_t)g.cell0 + (mx | my | mz);
                    t = P.cell_start[cell];
                    tend = P.cell_start[cell + 1];
                }
            }
        }
    }
    return visited;
}

// The exact K-nearest selection of the group search, with per-lane boxes: pass 1 (histogram of
// the culling distance over [0, R^2], R grown x1.3 per lane until the lane counts K), optional
// refinement inside the K-th bin, pass 2 (sure neighbours / FP64-keyed boundary band) over the
// box of the lane's own narrowed radius, exact resolution, exhaustive extraction on overflow.
// The list (lst[k * ls], k < K) receives original indices.
template <typename T, int NA>
__device__ __forceinline__ void search_lane(const AsmParams &P, const CloudGrid &g, int lane,
                                            bool valid, int q, const Pt<T> &qp, const T uq[3],
                                            int qidx, uint32_t *hist, double *bndkey,
                                            int32_t *bndpos, int32_t *lst, int64_t ls,
                                            bool &slow_row, int &n_streamed, int &n_grow)
{
    const int K = P.K;
    const float e = kRelBand;
    auto lane_box = [&](double R, int lo_[3], int hi_[3]) {
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
            const double u = (double)uq[ax];
            const double slack = 0.01 * g.cell + 2e-6 * fabs(u);
            lo_[ax] = cell_coord<double>(u - R - slack, g.lo[ax], g.inv_cell, g.dim[ax]);
            hi_[ax] = cell_coord<double>(u + R + slack, g.lo[ax], g.inv_cell, g.dim[ax]);
        }
    };
    // ----- pass 1: histogram; each lane grows its own radius until it counts K ---------------
    double R = g.r0;
    float R2 = 0.f, s0b = 0.f;
    int total = 0;
    int box_lo[3] = {0, 0, 0}, box_hi[3] = {0, 0, 0};
    bool need = valid, all = false;
    for (int grow = 0; __ballot(need) != 0; ++grow) {
        if (need) {
            lane_box(R, box_lo, box_hi);
            all = true;
#pragma unroll
            for (int a = 0; a < 3; ++a)
                all = all && box_lo[a] == 0 && box_hi[a] == g.dim[a] - 1;
            const double R2d = all ? g.diam2 * (1.0 + 1e-5) + 1e-300 : R * R * (1.0 - 1e-5);
            R2 = (float)R2d;
            if (!all)
                R2 = fminf(R2, (float)(R2d * (1.0 - 1e-6)));
            R2 = fmaxf(R2, 1e-30f);
            s0b = (float)kBins / R2;
            for (int w = 0; w < kBinWords; ++w)
                hist[w * kWave + lane] = 0u;
            total = 0;
            if (grow > 0)
                ++n_grow;
        }
        n_streamed += walk_box<T, NA>(P, g, box_lo, box_hi, qp, q, need,
                      [&](float f, const Pt<T> &c, int pos) {
                          if (f <= R2) {
                              ++total;
                              const int bb = max(0, min(kBins - 1, (int)(f * s0b)));
                              atomicAdd(&hist[(bb >> 1) * kWave + lane], 1u << ((bb & 1) * 16));
                          }
                      });
        if (need && total < K && all)
            atomicAdd(&P.counters[2], 1ull); // cannot happen: every cloud has > K points
        need = need && total < K && !all;
        if (need)
            R *= 1.3;
    }
    const bool act = valid;

    // ----- locate the bin of the K-th neighbour ----------------------------------------------
    const bool overflow = total >= 0xffff; // 16-bit counters saturated: exhaustive path
    int below = 0, b0 = kBins - 1, in_b0 = 0;
    {
        int cum = 0;
        bool found = false;
        for (int w = 0; w < kBinWords; ++w) {
            const uint32_t h = hist[w * kWave + lane];
            const int c0 = (int)(h & 0xffffu), c1 = (int)(h >> 16);
            if (!found) {
                if (cum + c0 >= K) {
                    found = true; b0 = 2 * w; below = cum; in_b0 = c0;
                } else if (cum + c0 + c1 >= K) {
                    found = true; b0 = 2 * w + 1; below = cum + c0; in_b0 = c1;
                }
                cum += c0 + c1;
            }
        }
    }
    const float wb = R2 / (float)kBins;
    float lo_f = (float)b0 * wb, hi_f = (b0 == kBins - 1) ? R2 : (float)(b0 + 1) * wb;
    // later passes: the box of this lane's narrowed radius
    int nbox_lo[3] = {0, 0, 0}, nbox_hi[3] = {0, 0, 0};
    {
        const float hmax = overflow ? R2 : hi_f;
        const double rn = sqrt((double)hmax * (1.0 + 4.0 * (double)e)) * (1.0 + 1e-5);
        if (rn < R) {
            lane_box(rn, nbox_lo, nbox_hi);
        } else {
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                nbox_lo[a] = box_lo[a];
                nbox_hi[a] = box_hi[a];
            }
        }
    }
    // ----- optional refinement inside bin b0 -------------------------------------------------
    const bool refine = act && !overflow && in_b0 > kBndCap - 4 && hi_f > lo_f;
    if (__ballot(refine) != 0) {
        const float base_lo = lo_f;
        const float s1 = refine ? (float)kBins / (hi_f - lo_f) : 0.f;
        if (refine)
            for (int w = 0; w < kBinWords; ++w)
                hist[w * kWave + lane] = 0u;
        n_streamed += walk_box<T, NA>(P, g, nbox_lo, nbox_hi, qp, q, refine,
                      [&](float f, const Pt<T> &c, int pos) {
                          if (!(f <= R2) || max(0, min(kBins - 1, (int)(f * s0b))) != b0)
                              return;
                          int sb = (int)((f - base_lo) * s1);
                          sb = sb < 0 ? 0 : (sb > kBins - 1 ? kBins - 1 : sb);
                          atomicAdd(&hist[(sb >> 1) * kWave + lane], 1u << ((sb & 1) * 16));
                      });
        if (refine) {
            int cum = below, b1 = kBins - 1;
            bool found = false;
            for (int w = 0; w < kBinWords; ++w) {
                const uint32_t h = hist[w * kWave + lane];
                const int c0 = (int)(h & 0xffffu), c1 = (int)(h >> 16);
                if (!found) {
                    if (cum + c0 >= K) {
                        found = true; b1 = 2 * w;
                    } else if (cum + c0 + c1 >= K) {
                        found = true; b1 = 2 * w + 1;
                    }
                    cum += c0 + c1;
                }
            }
            const float w1 = (hi_f - base_lo) / (float)kBins;
            const float nlo = base_lo + (float)b1 * w1;
            const float nhi = (b1 == kBins - 1) ? hi_f : base_lo + (float)(b1 + 1) * w1;
            lo_f = nlo;
            hi_f = nhi;
        }
    }
    if (overflow) { // everything within R is a boundary candidate
        lo_f = 0.f;
        hi_f = R2;
    }
    // ----- pass 2: classify ------------------------------------------------------------------
    const float lo_t = lo_f * (1.f - e), hi_t = hi_f * (1.f + e);
    int nin = 0, nb = 0;
    n_streamed += walk_box<T, NA>(P, g, nbox_lo, nbox_hi, qp, q, act,
                  [&](float f, const Pt<T> &c, int pos) {
                      if (f * (1.f + e) < lo_t) {
                          if (nin < K)
                              lst[nin * ls] = P.perm[pos];
                          ++nin;
                      } else if (f * (1.f - e) <= hi_t) {
                          if (nb < kBndCap) {
                              bndkey[nb * kWave + lane] = exact_key<T, NA>(qp, c);
                              bndpos[nb * kWave + lane] = P.perm[pos];
                          }
                          ++nb;
                      }
                  });
    if (act && nin >= K)
        atomicAdd(&P.counters[2], 1ull); // cannot happen (fewer than K below the K-th bin)
    const int r = K - nin;
    const bool slow = act && (nb > kBndCap || nb < r || nin >= K);
    // ----- resolve the boundary by exact (key, index) rank -----------------------------------
    if (act && !slow) {
        for (int bi = 0; bi < nb; ++bi) {
            const double kb = bndkey[bi * kWave + lane];
            const int pb = bndpos[bi * kWave + lane]; // original index
            int rank = 0;
            for (int bj = 0; bj < nb; ++bj) {
                const double kj = bndkey[bj * kWave + lane];
                if (kj < kb || (kj == kb && bndpos[bj * kWave + lane] < pb))
                    ++rank;
            }
            if (rank < r)
                lst[(nin + rank) * ls] = pb;
        }
    }
    // ----- exhaustive extraction for lanes that need it --------------------------------------
    if (__ballot(slow) != 0) {
        const int nin_s = slow ? (nin < K ? nin : 0) : 0;
        const int rr = slow ? K - nin_s : 0;
        const float lo_s = (slow && nin < K) ? lo_t : 0.f;
        const int rmax = seg_max(rr, kWave);
        double last_k = -1.0;
        int last_i = -1;
        for (int sidx = 0; sidx < rmax; ++sidx) {
            double best_k = INFINITY;
            int best_i = 0x7fffffff, best_p = -1;
            const bool want = slow && sidx < rr;
            n_streamed += walk_box<T, NA>(P, g, nbox_lo, nbox_hi, qp, q, want,
                          [&](float f, const Pt<T> &c, int pos) {
                              if (!(f * (1.f - e) <= hi_t) || f * (1.f + e) < lo_s)
                                  return;
                              const double k = exact_key<T, NA>(qp, c);
                              const int idx = P.perm[pos];
                              const bool after = k > last_k || (k == last_k && idx > last_i);
                              const bool better = k < best_k || (k == best_k && idx < best_i);
                              if (after && better) {
                                  best_k = k; best_i = idx; best_p = pos;
                              }
                          });
            if (want) {
                lst[(nin_s + sidx) * ls] = best_p < 0 ? qidx : best_i;
                last_k = best_k;
                last_i = best_i;
                if (best_i == 0x7fffffff)
                    atomicAdd(&P.counters[2], 1ull);
            }
        }
        if (slow)
            slow_row = true;
    }
}

// ---------------------------------------------------------------------------------------------
// the kernel
// ---------------------------------------------------------------------------------------------
template <typename T, int NA, int S>
__device__ __forceinline__ void search_group(const AsmParams &P, const int64_t group, char *lds)
{
    const int lane = lane_id();
    const int K = P.K;
    char *lds_rng = lds + kLdsSearch;
    char *lds_stage = lds_rng + 2 * kWave * 4;
    uint32_t *hist = (uint32_t *)(lds + kLdsHist);
    double *bndkey = (double *)(lds + kLdsHist);
    int32_t *bndpos = (int32_t *)(lds + kLdsBndPos);

    int ci = 0;
    {
        int lo = 0, hi = P.n_clouds - 1;
        while (lo < hi) {
            int mid = (lo + hi + 1) >> 1;
            if (P.grids[mid].group0 <= group)
                lo = mid;
            else
                hi = mid - 1;
        }
        ci = lo;
    }
    const CloudGrid g = P.grids[ci];
    const Pt<T> *spts = (const Pt<T> *)P.spts;
    const int64_t s0 = g.row0 + (group - g.group0) * kWave;
    const int cnt = (int)min((int64_t)kWave, g.row0 + g.n - s0);
    const bool valid = lane < cnt;
    const int q = (int)(s0 + (valid ? lane : 0));
    const Pt<T> qp = spts[q];
    int cc[3];
    T uq[3]; // projected coordinates of the query
    {
        T x[NA];
#pragma unroll
        for (int a = 0; a < NA; ++a)
            x[a] = qp.v[a];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            uq[a] = project<T, NA>(x, g.proj, a);
            cc[a] = cell_coord<T>(uq[a], g.lo[a], g.inv_cell, g.dim[a]);
        }
    }
    // The selection writes original indices straight into the row's ELL column slots 1..K
    // (lst[k * ls]); lanes past the end of the cloud write nothing. (Every slot is written; the
    // fit kernel still range-checks what it reads.)
    const int qidx = P.perm[q];
    int32_t *lst = P.ell_col + P.ld + q;
    const int64_t ls = P.ld;

    bool slow_row = false;
    int n_streamed = 0, n_sub = 0, n_grow = 0;
    if constexpr (S == 1) {
        n_sub = 1;
        search_lane<T, NA>(P, g, lane, valid, q, qp, uq, qidx, hist, bndkey, bndpos, lst, ls,
                           slow_row, n_streamed, n_grow);
    } else {
        // ----- sub-groups: split the wave's points at Morton jumps while that shrinks the boxes ------
        // Consecutive sorted points are compact except where the Morton curve jumps; a group that
        // straddles a jump has a box far larger than either side. A worklist of lane ranges is split
        // at the lane pair whose Morton codes differ in the highest bit, whenever the two halves'
        // boxes hold fewer cells than the whole.
        const uint32_t mc = morton_of(P.parts, g, cc[0], cc[1], cc[2]);
        const uint32_t mnext = __shfl_down(mc, 1, kWave);
        const int hb = (lane + 1 < cnt) ? (32 - (int)__clz((int)(mc ^ mnext))) : -1;
        int2 *work = (int2 *)(lds_stage + search_stage_bytes((int)sizeof(Pt<T>), S));
        // Search box of a lane range for radius R: the range's bounding box in projected coordinates
        // grown by R (plus 1% of a cell, covering rounding in the binning), rounded out to cells.
        // Every point within distance R of a query of the range lies in it.
        // lanes of a range [a, b) that hold a query
        auto lanes = [&](int a, int b) -> uint64_t {
            return __ballot(valid && lane >= a && lane < b);
        };
        auto range_box = [&](uint64_t m, double R, int lo_[3], int hi_[3]) {
            const bool in = (m >> lane) & 1ull;
            int cells = 1;
    #pragma unroll
            for (int ax = 0; ax < 3; ++ax) {
                // minima and maxima are exact in the points' precision (half the shuffles of a
                // double reduction for float points)
                const double umn = (double)seg_min(in ? uq[ax] : (T)INFINITY, kWave);
                const double umx = (double)seg_max(in ? uq[ax] : (T)-INFINITY, kWave);
                const double slack = 0.01 * g.cell + 1e-6 * (fabs(umn) + fabs(umx));
                lo_[ax] = uniform(cell_coord<double>(umn - R - slack, g.lo[ax], g.inv_cell, g.dim[ax]));
                hi_[ax] = uniform(cell_coord<double>(umx + R + slack, g.lo[ax], g.inv_cell, g.dim[ax]));
                cells *= hi_[ax] - lo_[ax] + 1;
            }
            return cells;
        };
        const double r0 = g.r0;
        // split only ranges whose box exceeds twice a single query's box
        const int split_min = (int)fmin(2.0 * pow(2.0 * r0 * g.inv_cell + 2.0, 3.0), 1e9);

        const float e = kRelBand;
        int top = 1;
        if (lane == 0)
            work[0] = make_int2(0, cnt);
        __syncthreads();
        while (top > 0) {
            --top;
            const int ra = uniform(work[top].x), rb = uniform(work[top].y);
            int box_lo[3], box_hi[3];
            const int cells = range_box(lanes(ra, rb), r0, box_lo, box_hi);
            if (rb - ra >= 2 && cells > split_min) {
                const int key = (lane >= ra && lane < rb - 1) ? hb * 64 + (63 - lane) : -1;
                const int sk = uniform(seg_max(key, kWave));
                const int sl = 63 - (sk & 63); // split after lane sl
                int t0[3], t1[3];
                const int c1 = range_box(lanes(ra, sl + 1), r0, t0, t1);
                const int c2 = range_box(lanes(sl + 1, rb), r0, t0, t1);
                if (c1 + c2 < cells) {
                    __syncthreads();
                    if (lane == 0) {
                        work[top] = make_int2(sl + 1, rb);
                        work[top + 1] = make_int2(ra, sl + 1);
                    }
                    __syncthreads();
                    top += 2;
                    continue;
                }
            }
            // Peels: for the tile search, the queries of the range within sqrt(kTilePeel) r0 of a
            // centre query (the first one left), so that |q - c|^2 stays small against the search
            // radius (the error of the tile distances grows with it); where a 2-D sheet crosses
            // another in the binning projection, a range holds queries of both and is searched
            // once per sheet. Other searches take the whole range at once.
            const uint64_t whole = lanes(ra, rb);
            uint64_t todo = whole;
            while (todo != 0) {
                uint64_t peel = todo;
                int c_lane = (int)__ffsll((unsigned long long)todo) - 1;
                if constexpr (S == 2) {
                    float dn = 0.f;
#pragma unroll
                    for (int a = 0; a < 4; ++a) {
                        const float d_ = qp.v[a] - __shfl(qp.v[a], c_lane, kWave);
                        dn = fmaf(d_, d_, dn);
                    }
                    peel = __ballot(((todo >> lane) & 1ull) && (double)dn <= kTilePeel * r0 * r0);
                    peel |= 1ull << c_lane;
                    if (peel != whole) // a later peel, or a part of the range: its own box
                        range_box(peel, r0, box_lo, box_hi);
                }
                todo &= ~peel;
                const bool act = (peel >> lane) & 1ull;
                ++n_sub;
                int nin = 0, nb = 0;  // sure neighbours written, boundary candidates
                int keep_s = 0;       // slow path: sure neighbours it keeps
                float lo_s = 0.f;     // slow path: culling distances below it are kept sure neighbours
                float hi_s = 0.f;     // slow path: culling distances above it are never neighbours
                bool force_slow = false;
                int nbox_lo[3], nbox_hi[3];
                if constexpr (S == 2) {
                    // ===== tile search: g(query, candidate) from the matrix cores =====================
                    // Histograms of 32 bins x 32-bit counters per query: bin b holds the g with
                    // round(g sb) = b (half-integer edges), sb ~ 31.5 / cut of the query's own cut;
                    // values past the cut go to a 33rd, uncounted row (the boundary index area,
                    // unused until pass 2). The bin is read from the bits of fma(g, sb, 2^23).
                    const int hl = lane >> 5, ll = lane & 31;
                    constexpr int NB = kTileBins;
                    // centre: the peel's first query; query operands (-2 q^, 1, |q^|^2)
                    T cq[4];
#pragma unroll
                    for (int a = 0; a < 4; ++a)
                        cq[a] = __shfl(qp.v[a], c_lane, kWave);
                    float qh[4], nq = 0.f;
#pragma unroll
                    for (int a = 0; a < 4; ++a) {
                        qh[a] = (float)(qp.v[a] - cq[a]);
                        nq = fmaf(qh[a], qh[a], nq);
                    }
                    float *qaug = (float *)lds_stage; // the candidate operand area, free between streams
#pragma unroll
                    for (int a = 0; a < 4; ++a)
                        qaug[a * kWave + lane] = -2.f * qh[a];
                    qaug[4 * kWave + lane] = 1.f;
                    qaug[5 * kWave + lane] = nq;
                    __syncthreads();
                    float bq[2][3];
#pragma unroll
                    for (int qb = 0; qb < 2; ++qb)
#pragma unroll
                        for (int s = 0; s < 3; ++s)
                            bq[qb][s] = qaug[(2 * s + hl) * kWave + 32 * qb + ll];
                    __syncthreads();
                    // query blocks (lanes 0..31, 32..63) that hold an active query
                    const uint64_t actm = __ballot(act);
                    const int qmask = ((actm & 0xffffffffull) ? 1 : 0) | ((actm >> 32) ? 2 : 0);
                    const double ed = (double)e, E = (double)kTileErr, nqd = (double)nq;
                    // the pair (query, itself) has g in [0, gself]
                    const double gself = 5.0 * E * nqd;
                    // ----- pass 1: histogram of g; grow the radius until every active lane counts K
                    double R = r0;
                    float cut = 0.f, sb = 0.f;
                    int total = 0;
                    for (int grow = 0;; ++grow) {
                        if (grow > 0) {
                            range_box(peel, R, box_lo, box_hi);
                            ++n_grow;
                        }
                        bool all = true;
#pragma unroll
                        for (int a = 0; a < 3; ++a)
                            all = all && box_lo[a] == 0 && box_hi[a] == g.dim[a] - 1;
                        const double R2d = all ? g.diam2 * (1.0 + 1e-5) + 1e-300 : R * R * (1.0 - 1e-5);
                        // g <= cut implies key <= R2d (inside the box's radius); over the whole grid
                        // every point passes
                        cut = all ? f32_up((R2d * kTileU1 + kTileU0 * nqd) * (1.0 + 1e-6))
                                  : f32_down(R2d * (1.0 - ed) - E * nqd);
                        cut = fmaxf(cut, 1e-30f);
                        // round(g sb) < NB (g sb < NB - 1/2) implies g <= cut
                        sb = act ? f32_up(((double)NB - 0.5) / (double)cut * (1.0 + 1e-6)) : 0.f;
                        for (int w = 0; w < NB; ++w)
                            hist[w * kWave + lane] = 0u;
                        __syncthreads();
                        const float sb0 = __shfl(sb, ll, kWave), sb1 = __shfl(sb, 32 + ll, kWave);
                        n_streamed += stream_tile<T, NA>(P, g, box_lo, box_hi, lds_rng, lds_stage, cq, bq, qmask,
                            [&](int cb, int qb, const floatx16 &acc) {
                                const float s_ = qb ? sb1 : sb0;
                                char *h = (char *)(hist + 32 * qb + ll);
#pragma unroll
                                for (int r = 0; r < 16; ++r)
                                    atomicAdd((uint32_t *)(h + tile_bin_offset(acc[r], s_, (float)NB)), 1u);
                            });
                        __syncthreads();
                        int cntall = 0;
                        for (int w = 0; w < NB; ++w)
                            cntall += (int)hist[w * kWave + lane];
                        total = cntall - 1; // the query itself
                        const bool short_lane = act && total < K;
                        if (__ballot(short_lane) == 0 || all) {
                            if (short_lane)
                                atomicAdd(&P.counters[2], 1ull); // cannot happen: every cloud has > K points
                            break;
                        }
                        R *= 1.3;
                    }
                    // the query itself must sit in bin 0 of its own histogram
                    force_slow = act && !(gself * (double)sb < 0.5);
                    // ----- the bin of the K-th neighbour -------------------------------------------
                    int below = 0, b0 = NB - 1, in_b0 = 0;
                    {
                        int cum = -1; // the query itself, in bin 0
                        bool found = false;
                        for (int w = 0; w < NB; ++w) {
                            const int c0 = (int)hist[w * kWave + lane];
                            if (!found && cum + c0 >= K) {
                                found = true; b0 = w; below = cum; in_b0 = c0;
                            }
                            cum += c0;
                        }
                    }
                    // bin edges in g, widened by the rounding of the edges (absolute 1e-6 cut)
                    const double slack = 1e-6 * (double)cut;
                    const double bw = 1.0 / (double)sb;
                    double lo_e = act ? (b0 == 0 ? -1.0 : ((double)b0 - 0.5) * bw - slack) : -1.0;
                    double hi_e = act ? ((double)b0 + 0.5) * bw + slack : 0.0;
                    {
                        // the K nearest lie within key (hi_e + E |q^|^2) / (1 - e): stream that box
                        const double kb = (hi_e + E * nqd) / (1.0 - ed);
                        const double kmax = seg_max(act ? kb : 0.0, kWave);
                        const double rn = sqrt(kmax) * (1.0 + 1e-5);
                        if (rn < R)
                            range_box(peel, rn, nbox_lo, nbox_hi);
                        else
                            for (int a = 0; a < 3; ++a) {
                                nbox_lo[a] = box_lo[a];
                                nbox_hi[a] = box_hi[a];
                            }
                    }
                    // ----- optional refinement inside bin b0 ----------------------------------------
                    const bool refine = act && in_b0 > kBndCap - 4;
                    if (__ballot(refine) != 0) {
                        // sub-bin c of bin b0: round((g - base_lo) s1) = c, clamped to [0, NB - 1]
                        const double blo = b0 == 0 ? 0.0 : ((double)b0 - 0.5) / (double)sb;
                        const double bhi = ((double)b0 + 0.5) / (double)sb;
                        const float base_lo = refine ? (float)blo : 0.f;
                        const float s1 = refine ? f32_up(((double)NB - 0.5) / (bhi - (double)base_lo)) : 0.f;
                        if (refine && b0 == 0 && !(gself * (double)s1 < 0.5))
                            force_slow = true; // the query itself must sit in sub-bin 0
                        for (int w = 0; w < NB; ++w)
                            hist[w * kWave + lane] = 0u;
                        __syncthreads();
                        const float sq = refine ? sb : 0.f;
                        const float sq0 = __shfl(sq, ll, kWave), sq1 = __shfl(sq, 32 + ll, kWave);
                        const int rb0 = __shfl(b0, ll, kWave), rb1 = __shfl(b0, 32 + ll, kWave);
                        const float bl0 = __shfl(base_lo, ll, kWave), bl1 = __shfl(base_lo, 32 + ll, kWave);
                        const float s10 = __shfl(s1, ll, kWave), s11 = __shfl(s1, 32 + ll, kWave);
                        n_streamed += stream_tile<T, NA>(P, g, nbox_lo, nbox_hi, lds_rng, lds_stage, cq, bq, qmask,
                            [&](int cb, int qb, const floatx16 &acc) {
                                const float s_ = qb ? sq1 : sq0, bl_ = qb ? bl1 : bl0, s1_ = qb ? s11 : s10;
                                const uint32_t own = (uint32_t)(qb ? rb1 : rb0) * kWave * 4;
                                char *h = (char *)(hist + 32 * qb + ll);
#pragma unroll
                                for (int r = 0; r < 16; ++r) {
                                    const float gv = acc[r];
                                    const uint32_t o1 = tile_bin_offset(gv, s_, (float)NB);
                                    const uint32_t o2 = tile_bin_offset(gv - bl_, s1_, (float)(NB - 1));
                                    atomicAdd((uint32_t *)(h + (o1 == own ? o2 : (uint32_t)NB * kWave * 4)), 1u);
                                }
                            });
                        __syncthreads();
                        if (refine) {
                            int cum = below, b1 = NB - 1;
                            bool found = false;
                            for (int w = 0; w < NB; ++w) {
                                const int c0 = (int)hist[w * kWave + lane];
                                if (!found && cum + c0 >= K) {
                                    found = true; b1 = w;
                                }
                                cum += c0;
                            }
                            lo_e = b1 == 0 ? lo_e : (double)base_lo + ((double)b1 - 0.5) / (double)s1 - slack;
                            hi_e = b1 == NB - 1 ? hi_e
                                                : (double)base_lo + ((double)b1 + 0.5) / (double)s1 + slack;
                        }
                    }
                    // ----- pass 2: classify by g ------------------------------------------------------
                    // boundary: every point with key <= kb2 (the K-th neighbour's bound) has g <= hic;
                    // sure: g < loc implies that every point at least as near has g < lo_e, so it was
                    // counted below the K-th neighbour's bin.
                    const double kb2 = (hi_e + E * nqd) / (1.0 - ed);
                    const float hic = act ? f32_up((kb2 * kTileU1 + kTileU0 * nqd) * (1.0 + 1e-6)) : -INFINITY;
                    const double lo_k = ((lo_e - kTileU0 * nqd) / kTileU1) * (1.0 - ed) - E * nqd;
                    const float loc = act ? f32_down(lo_k - 1e-6 * fabs(lo_k)) : -INFINITY;
                    const float hc0 = __shfl(hic, ll, kWave), hc1 = __shfl(hic, 32 + ll, kWave);
                    const float lc0 = __shfl(loc, ll, kWave), lc1 = __shfl(loc, 32 + ll, kWave);
                    const int qi0 = __shfl(qidx, ll, kWave), qi1 = __shfl(qidx, 32 + ll, kWave);
                    const int32_t *st_pos = (const int32_t *)(lds_stage + 6 * kWave * 4);
                    const int32_t *st_idx = st_pos + kWave;
                    // a boundary entry's sorted position waits in the low word of its key slot until
                    // the key is computed after the stream
                    int32_t *bnd_at = (int32_t *)bndkey;
                    // Sure entries take rows 0..K of the query's ELL column in arrival order (row 0
                    // belongs to the row's own entry and is rewritten by the fit). The query itself
                    // takes a row like any sure entry but is not written there; after the stream the
                    // entry of row 0 moves into that row (or, the query not being a sure entry, to the
                    // end of the list), so that rows 1..nin hold the sure neighbours.
                    // Per query block (queries ll and 32 + ll; the two lanes of a query, one per
                    // candidate half, hold the same totals): sure and boundary counts, the row the
                    // query itself took (-1: none) and the entry written to row 0 (-1: none).
                    int cin0 = 0, cin1 = 0, cbd0 = 0, cbd1 = 0;
                    int srow0 = -1, srow1 = -1, rz0 = -1, rz1 = -1;
                    n_streamed += stream_tile<T, NA>(P, g, nbox_lo, nbox_hi, lds_rng, lds_stage, cq, bq, qmask,
                        [&](int cb, int qb, const floatx16 &acc) {
                            const float hc = qb ? hc1 : hc0, lc = qb ? lc1 : lc0;
                            uint32_t mh = 0, ms = 0; // hits (g <= hic) and sure ones (g < loc), bit r
#pragma unroll
                            for (int r = 0; r < 16; ++r) {
                                mh |= (acc[r] <= hc ? 1u : 0u) << r;
                                ms |= (acc[r] < lc ? 1u : 0u) << r;
                            }
                            // (padding entries, g ~ 3e38, never pass hic <= 1e38)
                            if (__ballot(mh != 0) == 0)
                                return;
                            uint32_t mS = mh & ms, mB = mh & ~ms;
                            // slots: the lower candidate half of a block first, then the upper
                            const int c = __popc(mS) | (__popc(mB) << 16);
                            const int pc = __shfl_xor(c, 32, kWave);
                            const int ci0 = qb ? cin1 : cin0, cb0 = qb ? cbd1 : cbd0;
                            int sS = ci0 + (hl ? (pc & 0xffff) : 0);
                            int sB = cb0 + (hl ? (pc >> 16) : 0);
                            const int ci1 = ci0 + (c & 0xffff) + (pc & 0xffff);
                            const int cb1 = cb0 + (c >> 16) + (pc >> 16);
                            if (qb) {
                                cin1 = ci1;
                                cbd1 = cb1;
                            } else {
                                cin0 = ci1;
                                cbd0 = cb1;
                            }
                            const int jb = 32 * qb + ll;
                            const int qi = qb ? qi1 : qi0;
                            int32_t *col = P.ell_col + s0 + jb;
                            int srow = -1, rz = -1;
                            while (mS != 0) {
                                const int r = __builtin_ctz(mS);
                                mS &= mS - 1;
                                const int idx = st_idx[32 * cb + 8 * (r >> 2) + 4 * hl + (r & 3)];
                                if (sS <= K && idx != qi)
                                    col[(int64_t)sS * ls] = idx;
                                srow = idx == qi ? sS : srow;
                                rz = sS == 0 ? idx : rz;
                                ++sS;
                            }
                            if (qb) {
                                srow1 = max(srow1, srow);
                                rz1 = max(rz1, rz);
                            } else {
                                srow0 = max(srow0, srow);
                                rz0 = max(rz0, rz);
                            }
                            while (mB != 0) {
                                const int r = __builtin_ctz(mB);
                                mB &= mB - 1;
                                if (sB < kBndCap) {
                                    const int ci = 32 * cb + 8 * (r >> 2) + 4 * hl + (r & 3);
                                    bnd_at[2 * (sB * kWave + jb)] = st_pos[ci];
                                    bndpos[sB * kWave + jb] = st_idx[ci];
                                }
                                ++sB;
                            }
                        });
                    __syncthreads();
                    {
                        // the other half's records of this lane's query (its block hl)
                        const int psrow = __shfl_xor(hl ? srow0 : srow1, 32, kWave);
                        const int prz = __shfl_xor(hl ? rz0 : rz1, 32, kWave);
                        const int srow = max(hl ? srow1 : srow0, psrow);
                        const int rz = max(hl ? rz1 : rz0, prz);
                        const int nall = hl ? cin1 : cin0;
                        nin = srow >= 0 ? nall - 1 : nall;
                        nb = hl ? cbd1 : cbd0;
                        if (act && nall <= K) {
                            int32_t *col = P.ell_col + s0 + lane;
                            if (srow > 0)
                                col[(int64_t)srow * ls] = rz;
                            else if (srow < 0 && nall > 0)
                                col[(int64_t)nall * ls] = rz;
                        }
                    }
                    // exact keys of the boundary entries (the query itself dropped; two point loads in
                    // flight)
                    if (act && nb <= kBndCap) {
                        int m = 0;
                        for (int bi = 0; bi < nb; ++bi) {
                            const int id = bndpos[bi * kWave + lane];
                            const int at = bnd_at[2 * (bi * kWave + lane)];
                            if (id != qidx) {
                                bndpos[m * kWave + lane] = id;
                                bnd_at[2 * (m * kWave + lane)] = at;
                                ++m;
                            }
                        }
                        nb = m;
                        for (int bi = 0; bi < nb; bi += 2) {
                            const Pt<T> c0 = spts[bnd_at[2 * (bi * kWave + lane)]];
                            const Pt<T> c1 = spts[bnd_at[2 * (min(bi + 1, nb - 1) * kWave + lane)]];
                            bndkey[bi * kWave + lane] = exact_key<T, NA>(qp, c0);
                            if (bi + 1 < nb)
                                bndkey[(bi + 1) * kWave + lane] = exact_key<T, NA>(qp, c1);
                        }
                    }
                    keep_s = 0;
                    lo_s = 0.f;
                    hi_s = f32_up(kb2 * (1.0 + 3.0 * ed));
                } else {
                    // ----- pass 1: histogram; grow the radius until every active lane counts K -----------
                    double R = r0;
                    float R2 = 0.f, s0b = 0.f;
                    int total = 0;
                    for (int grow = 0;; ++grow) {
                        if (grow > 0) {
                            range_box(peel, R, box_lo, box_hi);
                            ++n_grow;
                        }
                        bool all = true;
            #pragma unroll
                        for (int a = 0; a < 3; ++a)
                            all = all && box_lo[a] == 0 && box_hi[a] == g.dim[a] - 1;
                        const double R2d = all ? g.diam2 * (1.0 + 1e-5) + 1e-300 : R * R * (1.0 - 1e-5);
                        R2 = (float)R2d;
                        if (!all)
                            R2 = fminf(R2, (float)(R2d * (1.0 - 1e-6)));
                        R2 = fmaxf(R2, 1e-30f);
                        s0b = (float)kBins / R2;
                        for (int w = 0; w < kBinWords; ++w)
                            hist[w * kWave + lane] = 0u;
                        total = 0;
                        __syncthreads();
                        n_streamed += stream_box<T, NA>(P, g, box_lo, box_hi, lds_rng, lds_stage, qp, q, act,
                                      [&](float f, const Pt<T> &c, int pos, int idx) {
                                          if (f <= R2) {
                                              ++total;
                                              const int bb = max(0, min(kBins - 1, (int)(f * s0b)));
                                              atomicAdd(&hist[(bb >> 1) * kWave + lane], 1u << ((bb & 1) * 16));
                                          }
                                      });
                        const bool short_lane = act && total < K;
                        if (__ballot(short_lane) == 0 || all) {
                            if (short_lane)
                                atomicAdd(&P.counters[2], 1ull); // cannot happen: every cloud has > K points
                            break;
                        }
                        R *= 1.3;
                    }

                    // ----- locate the bin of the K-th neighbour ------------------------------------------
                    const bool overflow = total >= 0xffff; // 16-bit counters saturated: exhaustive path
                    int below = 0, b0 = kBins - 1, in_b0 = 0;
                    {
                        int cum = 0;
                        bool found = false;
                        for (int w = 0; w < kBinWords; ++w) {
                            const uint32_t h = hist[w * kWave + lane];
                            const int c0 = (int)(h & 0xffffu), c1 = (int)(h >> 16);
                            if (!found) {
                                if (cum + c0 >= K) {
                                    found = true; b0 = 2 * w; below = cum; in_b0 = c0;
                                } else if (cum + c0 + c1 >= K) {
                                    found = true; b0 = 2 * w + 1; below = cum + c0; in_b0 = c1;
                                }
                                cum += c0 + c1;
                            }
                        }
                    }
                    const float wb = R2 / (float)kBins;
                    float lo_f = (float)b0 * wb, hi_f = (b0 == kBins - 1) ? R2 : (float)(b0 + 1) * wb;
                    // Later passes only need candidates with f <= hi (times the band): stream the box of the
                    // largest such radius over the range's lanes instead of the pass-1 box.
                    {
                        const float hmax = seg_max(act ? (overflow ? R2 : hi_f) : 0.f, kWave);
                        const double rn = sqrt((double)hmax * (1.0 + 4.0 * (double)e)) * (1.0 + 1e-5);
                        if (rn < R)
                            range_box(peel, rn, nbox_lo, nbox_hi);
                        else
                            for (int a = 0; a < 3; ++a) {
                                nbox_lo[a] = box_lo[a];
                                nbox_hi[a] = box_hi[a];
                            }
                    }
                    // ----- optional refinement inside bin b0 ---------------------------------------------
                    const bool refine = act && !overflow && in_b0 > kBndCap - 4 && hi_f > lo_f;
                    if (__ballot(refine) != 0) {
                        const float base_lo = lo_f;
                        const float s1 = refine ? (float)kBins / (hi_f - lo_f) : 0.f;
                        for (int w = 0; w < kBinWords; ++w)
                            hist[w * kWave + lane] = 0u;
                        __syncthreads();
                        n_streamed += stream_box<T, NA>(P, g, nbox_lo, nbox_hi, lds_rng, lds_stage, qp, q, refine,
                                      [&](float f, const Pt<T> &c, int pos, int idx) {
                                          if (!(f <= R2) || max(0, min(kBins - 1, (int)(f * s0b))) != b0)
                                              return;
                                          int sb = (int)((f - base_lo) * s1);
                                          sb = sb < 0 ? 0 : (sb > kBins - 1 ? kBins - 1 : sb);
                                          atomicAdd(&hist[(sb >> 1) * kWave + lane], 1u << ((sb & 1) * 16));
                                      });
                        if (refine) {
                            int cum = below, b1 = kBins - 1;
                            bool found = false;
                            for (int w = 0; w < kBinWords; ++w) {
                                const uint32_t h = hist[w * kWave + lane];
                                const int c0 = (int)(h & 0xffffu), c1 = (int)(h >> 16);
                                if (!found) {
                                    if (cum + c0 >= K) {
                                        found = true; b1 = 2 * w;
                                    } else if (cum + c0 + c1 >= K) {
                                        found = true; b1 = 2 * w + 1;
                                    }
                                    cum += c0 + c1;
                                }
                            }
                            const float w1 = (hi_f - base_lo) / (float)kBins;
                            const float nlo = base_lo + (float)b1 * w1;
                            const float nhi = (b1 == kBins - 1) ? hi_f : base_lo + (float)(b1 + 1) * w1;
                            lo_f = nlo;
                            hi_f = nhi;
                        }
                    }
                    if (overflow) { // everything within R is a boundary candidate
                        lo_f = 0.f;
                        hi_f = R2;
                    }
                    // ----- pass 2: classify --------------------------------------------------------------
                    const float lo_t = lo_f * (1.f - e), hi_t = hi_f * (1.f + e);
                    n_streamed += stream_box<T, NA>(P, g, nbox_lo, nbox_hi, lds_rng, lds_stage, qp, q, act,
                                  [&](float f, const Pt<T> &c, int pos, int idx) {
                                      if (f * (1.f + e) < lo_t) {
                                          if (nin < K)
                                              lst[nin * ls] = idx;
                                          ++nin;
                                      } else if (f * (1.f - e) <= hi_t) {
                                          if (nb < kBndCap) {
                                              bndkey[nb * kWave + lane] = exact_key<T, NA>(qp, c);
                                              bndpos[nb * kWave + lane] = idx;
                                          }
                                          ++nb;
                                      }
                                  });
                    keep_s = nin < K ? nin : 0;
                    lo_s = nin < K ? lo_t : 0.f;
                    hi_s = hi_t;
                }
                if (act && nin >= K)
                    atomicAdd(&P.counters[2], 1ull); // cannot happen (fewer than K below the K-th bin)
                const int r = K - nin;
                const bool slow = act && (force_slow || nb > kBndCap || nb < r || nin >= K);
                // ----- resolve the boundary by exact (key, index) rank --------------------------------
                // (every key slot is read once into registers; slots past nb are masked)
                if (act && !slow) {
                    double kk[kBndCap];
                    int pp[kBndCap];
#pragma unroll
                    for (int j = 0; j < kBndCap; ++j) {
                        kk[j] = bndkey[j * kWave + lane];
                        pp[j] = bndpos[j * kWave + lane];
                    }
                    for (int bi = 0; bi < nb; ++bi) {
                        const double kb = bndkey[bi * kWave + lane];
                        const int pb = bndpos[bi * kWave + lane]; // original index
                        int rank = 0;
#pragma unroll
                        for (int bj = 0; bj < kBndCap; ++bj)
                            rank += (bj < nb && (kk[bj] < kb || (kk[bj] == kb && pp[bj] < pb))) ? 1 : 0;
                        if (rank < r)
                            lst[(nin + rank) * ls] = pb;
                    }
                }
                // ----- exhaustive extraction for lanes that need it ----------------------------------
                if (__ballot(slow) != 0) {
                    const int nin_s = slow ? keep_s : 0;
                    const int rr = slow ? K - nin_s : 0;
                    const float lo_sl = slow ? lo_s : 0.f;
                    const int rmax = seg_max(rr, kWave);
                    double last_k = -1.0;
                    int last_i = -1;
                    for (int sidx = 0; sidx < rmax; ++sidx) {
                        double best_k = INFINITY;
                        int best_i = 0x7fffffff, best_p = -1;
                        const bool want = slow && sidx < rr;
                        n_streamed += stream_box<T, NA>(P, g, nbox_lo, nbox_hi, lds_rng, lds_stage, qp, q, want,
                                      [&](float f, const Pt<T> &c, int pos, int idx) {
                                          if (!(f * (1.f - e) <= hi_s) || f * (1.f + e) < lo_sl)
                                              return;
                                          const double k = exact_key<T, NA>(qp, c);
                                          const bool after = k > last_k || (k == last_k && idx > last_i);
                                          const bool better = k < best_k || (k == best_k && idx < best_i);
                                          if (after && better) {
                                              best_k = k; best_i = idx; best_p = pos;
                                          }
                                      });
                        if (want) {
                            lst[(nin_s + sidx) * ls] = best_p < 0 ? qidx : best_i;
                            last_k = best_k;
                            last_i = best_i;
                            if (best_i == 0x7fffffff)
                                atomicAdd(&P.counters[2], 1ull);
                        }
                    }
                    if (slow)
                        slow_row = true;
                }
                __syncthreads();
            }
        }
    }

    if (lane == 0) {
        atomicAdd(&P.counters[3], (unsigned long long)n_sub);
        atomicAdd(&P.counters[4], (unsigned long long)n_streamed);
        atomicAdd(&P.counters[5], (unsigned long long)n_grow);
    }
    const unsigned long long ns = __popcll(__ballot(valid && slow_row));
    if (lane == 0 && ns)
        atomicAdd(&P.counters[1], ns);
    if (valid && P.row_flags)
        P.row_flags[q] = slow_row ? 2 : 0;
}

// The search's list of row q (original indices in ELL slots 1..K) in ascending original index,
// mapped to sorted positions, into list[k][lane]: a bitonic network on KP >= K registers (padding
// sorts last), fully unrolled, so every compare-exchange is a min and a max.
template <int KP>
__device__ __forceinline__ void sort_list(const AsmParams &P, int q, int qidx, int lane,
                                          int32_t *list)
{
    const int K = P.K;
    int v[KP];
#pragma unroll
    for (int k = 0; k < KP; ++k) {
        int idx = 0x7fffffff;
        if (k < K) {
            idx = P.ell_col[(int64_t)(k + 1) * P.ld + q];
            idx = (idx >= 0 && (int64_t)idx < P.n_rows) ? idx : qidx;
        }
        v[k] = idx;
    }
#pragma unroll
    for (int size = 2; size <= KP; size <<= 1)
#pragma unroll
        for (int stride = size >> 1; stride > 0; stride >>= 1)
#pragma unroll
            for (int i = 0; i < KP; ++i) {
                const int j = i ^ stride;
                if (j > i) {
                    const int lo = min(v[i], v[j]), hi = max(v[i], v[j]);
                    const bool up = (i & size) == 0;
                    v[i] = up ? lo : hi;
                    v[j] = up ? hi : lo;
                }
            }
#pragma unroll
    for (int k = 0; k < KP; ++k)
        if (k < K)
            list[k * kWave + lane] = P.iperm[v[k]];
}

// Per-lane fit of one row (one wave per 64 consecutive rows in cell order): the neighbour list
// of the search (original indices in ELL slots 1..K) is put in canonical order, ascending
// original index (the order of the rows of V in the paper's normal equations), mapped back to
// sorted positions for local gathers, and fitted (fit_row writes the finished ELL row).
// Occupancy target of the fit kernel (waves per SIMD): float points 4 (128 VGPRs; the R^4 fit
// ~11% faster than the compiler's 148), double points 3 (at 128 VGPRs the FP64 fit spills enough
// to run 40% slower). Measured at 1M points in R^4.
#ifndef MVGD_FIT_WAVES_PER_EU
#define MVGD_FIT_WAVES_PER_EU 4
#endif
#ifndef MVGD_FIT_WAVES_PER_EU_FP64
#define MVGD_FIT_WAVES_PER_EU_FP64 3
#endif
#define MVGD_FIT_ATTR                                                                             \
    __attribute__((amdgpu_waves_per_eu(sizeof(T) == 8 ? MVGD_FIT_WAVES_PER_EU_FP64                \
                                                      : MVGD_FIT_WAVES_PER_EU)))
template <typename T, int NA, int D>
__global__ __launch_bounds__(64) MVGD_FIT_ATTR void fit_kernel(AsmParams P)
{
    extern __shared__ __attribute__((aligned(16))) char lds[];
    int32_t *list = (int32_t *)lds;
    const int lane = lane_id();
    const int64_t q64 = (int64_t)blockIdx.x * kWave + lane;
    if (q64 >= P.n_rows)
        return;
    const int q = (int)q64;
    const int K = P.K;
    const int qidx = P.perm[q];
    if (K <= 8)
        sort_list<8>(P, q, qidx, lane, list);
    else if (K <= 16)
        sort_list<16>(P, q, qidx, lane, list);
    else if (K <= 32)
        sort_list<32>(P, q, qidx, lane, list);
    else
        sort_list<64>(P, q, qidx, lane, list);
    const Pt<T> *spts = (const Pt<T> *)P.spts;
    const bool slow_row = P.row_flags ? (P.row_flags[q] & 2) != 0 : false;
    fit_row<T, NA, D>(P, spts, list, lane, q, spts[q], slow_row);
}

// Occupancy target of the search kernels (waves per SIMD). Left alone, the group search takes
// ~213 VGPRs (2 waves per SIMD); at 3 it fits 168 VGPRs with a small spill and runs ~13% faster at
// 1M points in R^4 (measured). The tile search is held to 2.5 waves per SIMD by its LDS anyway and
// runs ~4% faster with the 256 VGPRs of 2 (measured).
#ifndef MVGD_SEARCH_WAVES_PER_EU
#define MVGD_SEARCH_WAVES_PER_EU 3
#endif
#ifndef MVGD_TILE_WAVES_PER_EU
#define MVGD_TILE_WAVES_PER_EU 2
#endif
#define MVGD_SEARCH_ATTR                                                                          \
    __attribute__((amdgpu_waves_per_eu(S == 2 ? MVGD_TILE_WAVES_PER_EU : MVGD_SEARCH_WAVES_PER_EU)))

// Grid-mapped launch: one workgroup per group, XCD-aware remap (workgroups are dispatched to the
// eight XCDs round-robin, so workgroup b runs on XCD b % 8; consecutive groups, which are
// neighbours in space, go to the same XCD and share its L2).
template <typename T, int NA, int S>
__global__ __launch_bounds__(64) MVGD_SEARCH_ATTR void search_kernel(AsmParams P)
{
    extern __shared__ __attribute__((aligned(16))) char lds[];
    const int64_t b = blockIdx.x;
    const int64_t group = (b & 7) * P.groups_per_xcd + (b >> 3);
    if (group >= P.n_groups)
        return;
    search_group<T, NA, S>(P, group, lds);
}

// Persistent launch: as many workgroups as fit on the device at once; each pops groups from the
// queue of its XCD (queue x owns groups [x * groups_per_xcd, (x + 1) * groups_per_xcd)) and,
// when that queue is empty, steals from the others in turn. Every workgroup exits once all eight
// queues are exhausted. The queue counters must be zero at launch.
template <typename T, int NA, int S>
__global__ __launch_bounds__(64) MVGD_SEARCH_ATTR void search_persistent_kernel(AsmParams P)
{
    extern __shared__ __attribute__((aligned(16))) char lds[];
    const int home = (int)(blockIdx.x & 7);
    for (int v = 0; v < 8; ++v) {
        const int qx = (home + v) & 7;
        const int64_t base = (int64_t)qx * P.groups_per_xcd;
        const int64_t len = min(P.groups_per_xcd, P.n_groups - base);
        if (len <= 0)
            continue;
        for (;;) {
            unsigned int t = 0;
            if (lane_id() == 0)
                t = atomicAdd(&P.queue[qx], 1u);
            t = (unsigned int)uniform((int)t);
            if ((int64_t)t >= len)
                break;
            search_group<T, NA, S>(P, base + t, lds);
            __syncthreads();
        }
    }
}

} // namespace mvgd
