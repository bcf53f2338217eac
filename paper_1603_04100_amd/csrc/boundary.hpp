// boundary.hpp -- the Neumann condition on an open surface by reflection (ghost points).
//
// For an interior point with a boundary point among its K nearest neighbours, a ghost point is
// its mirror image across the boundary: at the closest boundary point p^B the frame is the
// tangent of the boundary curve (quadratic least-squares fit through the k_b nearest boundary
// points), the surface normal (PCA of the K nearest points of the whole cloud) and their cross
// product e3, the normal of the boundary inside the tangent plane; the ghost is
// p - 2 ((p - p^B) . e3) e3 (Sec. 3.1). With a zero normal derivative the ghost carries its
// source's value, so after the assembly on the interior points plus the ghosts every ghost column
// is folded into its source's column.
//
// nm_flag_kernel     interior points with a boundary point among their K nearest neighbours
// nm_frame_kernel    e3 at every boundary point (FP64), one wave per boundary point
// nm_ghost_kernel    closest boundary point (among the K nearest) and mirror image of every
//                    flagged interior point
// nm_fold_kernel     ghost columns -> source columns; ghost rows become zero rows
#pragma once

#include "assemble.hpp"
#include "common.hpp"

namespace mvgd {

// flag[row] = 1 for interior rows with a boundary neighbour (ELL columns are sorted positions)
__global__ __launch_bounds__(256) void nm_flag_kernel(const int32_t *__restrict__ col,
                                                      const int32_t *__restrict__ perm,
                                                      const uint8_t *__restrict__ boundary,
                                                      int64_t n, int64_t ld, int K,
                                                      uint32_t *__restrict__ flag,
                                                      uint32_t *__restrict__ is_interior,
                                                      uint32_t *__restrict__ is_boundary)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n)
        return;
    const int row = perm[s];
    const bool b = boundary[row] != 0;
    bool any = false;
    if (!b)
        for (int k = 1; k <= K; ++k)
            any = any || boundary[perm[col[(int64_t)k * ld + s]]] != 0;
    flag[row] = any ? 1u : 0u;
    is_interior[row] = b ? 0u : 1u;
    is_boundary[row] = b ? 1u : 0u;
}

// list[slot[i]] = i for every i with mask[i] != 0 (slot = exclusive prefix sum of the mask)
__global__ __launch_bounds__(256) void nm_compact_kernel(const uint32_t *__restrict__ mask,
                                                         const uint32_t *__restrict__ slot,
                                                         int64_t n, int32_t *__restrict__ list)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && mask[i])
        list[slot[i]] = (int32_t)i;
}

// inverse of a permutation: ipos[perm[s]] = s
__global__ __launch_bounds__(256) void nm_inverse_kernel(const int32_t *__restrict__ perm, int64_t n,
                                                         int32_t *__restrict__ ipos)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s < n)
        ipos[perm[s]] = (int32_t)s;
}

template <typename T>
__device__ __forceinline__ void nm_load(const T *pts, int64_t i, double p[3])
{
    for (int a = 0; a < 3; ++a)
        p[a] = (double)pts[i * 3 + a];
}

// squared distance, IEEE double left to right, no contraction (as the kNN key)
__device__ __forceinline__ double nm_d2(const double a[3], const double b[3])
{
#pragma clang fp contract(off)
    const double d0 = b[0] - a[0], d1 = b[1] - a[1], d2 = b[2] - a[2];
    return (d0 * d0 + d1 * d1) + d2 * d2;
}

// eigenvectors of a symmetric 3x3 (columns of W), eigenvalues on the diagonal of A
__device__ __forceinline__ void nm_eig3(double A[3][3], double W[3][3])
{
    jacobi_eig<3>(A, W);
}

// e3 at boundary point j (bl[j] = its index in the cloud), one wave per boundary point: the kb
// nearest boundary points are extracted in (squared distance, list index) order, one per round,
// each round a lane-parallel scan of the boundary list and a wave argmin; lane 0 then fits.
template <typename T>
__global__ __launch_bounds__(64) void nm_frame_kernel(const T *__restrict__ pts,
                                                      const int32_t *__restrict__ bl, int64_t nb,
                                                      int kb, const int32_t *__restrict__ col0,
                                                      const int32_t *__restrict__ perm0,
                                                      const int32_t *__restrict__ ipos0,
                                                      int64_t ld0, int K,
                                                      double *__restrict__ e3out)
{
    __shared__ int32_t sel[16];
    const int64_t j = blockIdx.x;
    const int lane = (int)threadIdx.x;
    if (j >= nb)
        return;
    double pj[3];
    nm_load<T>(pts, bl[j], pj);
    double last_k = -1.0;
    int64_t last_t = -1;
    for (int r = 0; r < kb; ++r) {
        double best_k = INFINITY;
        int64_t best_t = INT64_MAX;
        for (int64_t t = lane; t < nb; t += 64) {
            double pt[3];
            nm_load<T>(pts, bl[t], pt);
            const double d = nm_d2(pj, pt);
            const bool after = d > last_k || (d == last_k && t > last_t);
            const bool better = d < best_k || (d == best_k && t < best_t);
            if (after && better) {
                best_k = d;
                best_t = t;
            }
        }
        for (int o = 32; o > 0; o >>= 1) {
            const double ok = __shfl_xor(best_k, o, 64);
            const int64_t ot = __shfl_xor(best_t, o, 64);
            if (ok < best_k || (ok == best_k && ot < best_t)) {
                best_k = ok;
                best_t = ot;
            }
        }
        last_k = best_k;
        last_t = best_t;
        if (lane == 0) // (every round finds one: nb >= kb; the guard keeps an index in range)
            sel[r] = best_t < nb ? (int32_t)best_t : (int32_t)j;
    }
    __syncthreads();
    if (lane != 0)
        return;
    const int cnt = kb;
    const int32_t *bi = sel;
    // PCA of those points: tangent = largest eigenvector, n1, n2 = the others
    double c[3] = {0, 0, 0};
    for (int r = 0; r < cnt; ++r) {
        double q[3];
        nm_load<T>(pts, bl[bi[r]], q);
        for (int a = 0; a < 3; ++a)
            c[a] += q[a];
    }
    for (int a = 0; a < 3; ++a)
        c[a] /= (double)cnt;
    double A[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}}, W[3][3];
    for (int r = 0; r < cnt; ++r) {
        double q[3];
        nm_load<T>(pts, bl[bi[r]], q);
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b)
                A[a][b] += (q[a] - c[a]) * (q[b] - c[b]);
    }
    nm_eig3(A, W);
    int o[3] = {0, 1, 2}; // descending eigenvalues
    for (int a = 0; a < 3; ++a)
        for (int b = a + 1; b < 3; ++b)
            if (A[o[b]][o[b]] > A[o[a]][o[a]]) {
                const int tmp = o[a];
                o[a] = o[b];
                o[b] = tmp;
            }
    double t[3], n1[3], n2[3];
    for (int a = 0; a < 3; ++a) {
        t[a] = W[a][o[0]];
        n1[a] = W[a][o[1]];
        n2[a] = W[a][o[2]];
    }
    // quadratic fits eta(xi), zeta(xi) through the points, in coordinates about p^B_j
    double G[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}}, re[3] = {0, 0, 0}, rz[3] = {0, 0, 0};
    for (int r = 0; r < cnt; ++r) {
        double q[3];
        nm_load<T>(pts, bl[bi[r]], q);
        double d[3] = {q[0] - pj[0], q[1] - pj[1], q[2] - pj[2]};
        const double xi = d[0] * t[0] + d[1] * t[1] + d[2] * t[2];
        const double et = d[0] * n1[0] + d[1] * n1[1] + d[2] * n1[2];
        const double ze = d[0] * n2[0] + d[1] * n2[1] + d[2] * n2[2];
        const double m[3] = {1.0, xi, xi * xi};
        for (int a = 0; a < 3; ++a) {
            for (int b = 0; b < 3; ++b)
                G[a][b] += m[a] * m[b];
            re[a] += m[a] * et;
            rz[a] += m[a] * ze;
        }
    }
    // slopes at xi = 0 from the 3x3 normal equations (Cramer on the symmetric system)
    auto solve3 = [&](const double b[3], double x[3]) {
        const double det = G[0][0] * (G[1][1] * G[2][2] - G[1][2] * G[2][1]) -
                           G[0][1] * (G[1][0] * G[2][2] - G[1][2] * G[2][0]) +
                           G[0][2] * (G[1][0] * G[2][1] - G[1][1] * G[2][0]);
        for (int cidx = 0; cidx < 3; ++cidx) {
            double M[3][3];
            for (int a = 0; a < 3; ++a)
                for (int b2 = 0; b2 < 3; ++b2)
                    M[a][b2] = (b2 == cidx) ? b[a] : G[a][b2];
            x[cidx] = (M[0][0] * (M[1][1] * M[2][2] - M[1][2] * M[2][1]) -
                       M[0][1] * (M[1][0] * M[2][2] - M[1][2] * M[2][0]) +
                       M[0][2] * (M[1][0] * M[2][1] - M[1][1] * M[2][0])) / det;
        }
    };
    double ce[3], cz[3];
    solve3(re, ce);
    solve3(rz, cz);
    double e1[3];
    for (int a = 0; a < 3; ++a)
        e1[a] = t[a] + ce[1] * n1[a] + cz[1] * n2[a];
    double nrm = sqrt(e1[0] * e1[0] + e1[1] * e1[1] + e1[2] * e1[2]);
    for (int a = 0; a < 3; ++a)
        e1[a] /= nrm;
    // surface normal: PCA of the K nearest points of the whole cloud
    const int64_t s = ipos0[bl[j]];
    double m3[3] = {0, 0, 0};
    for (int k = 1; k <= K; ++k) {
        double q[3];
        nm_load<T>(pts, perm0[col0[(int64_t)k * ld0 + s]], q);
        for (int a = 0; a < 3; ++a)
            m3[a] += q[a];
    }
    for (int a = 0; a < 3; ++a)
        m3[a] /= (double)K;
    double C[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}}, V[3][3];
    for (int k = 1; k <= K; ++k) {
        double q[3];
        nm_load<T>(pts, perm0[col0[(int64_t)k * ld0 + s]], q);
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b)
                C[a][b] += (q[a] - m3[a]) * (q[b] - m3[b]);
    }
    nm_eig3(C, V);
    int imin = 0;
    for (int a = 1; a < 3; ++a)
        if (C[a][a] < C[imin][imin])
            imin = a;
    const double e2[3] = {V[0][imin], V[1][imin], V[2][imin]};
    double e3[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2],
                    e1[0] * e2[1] - e1[1] * e2[0]};
    nrm = sqrt(e3[0] * e3[0] + e3[1] * e3[1] + e3[2] * e3[2]);
    for (int a = 0; a < 3; ++a)
        e3out[j * 3 + a] = e3[a] / nrm;
}

// ghost of flagged interior point f: fl[f] = its index in the cloud, irank[i] = its place in the
// interior list, brank[i] = a boundary point's place in the boundary list; aug gets the ghost at
// row n_interior + f. The closest boundary point (ties to the smaller index) is among the point's K
// nearest neighbours: some boundary point is, and every point before it in (key, index) order is too.
template <typename T>
__global__ __launch_bounds__(256) void nm_ghost_kernel(const T *__restrict__ pts,
                                                       const int32_t *__restrict__ fl, int64_t nf,
                                                       const uint8_t *__restrict__ boundary,
                                                       const uint32_t *__restrict__ brank,
                                                       const int32_t *__restrict__ col0,
                                                       const int32_t *__restrict__ perm0,
                                                       const int32_t *__restrict__ ipos0,
                                                       int64_t ld0, int K,
                                                       const double *__restrict__ e3,
                                                       const uint32_t *__restrict__ irank,
                                                       int64_t n_interior, T *__restrict__ aug,
                                                       int32_t *__restrict__ ghost_src,
                                                       double *__restrict__ ghost_xyz)
{
    const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= nf)
        return;
    const int32_t i = fl[f];
    double p[3];
    nm_load<T>(pts, i, p);
    const int64_t s = ipos0[i];
    double best = INFINITY;
    int32_t bc = -1;
    for (int k = 1; k <= K; ++k) {
        const int32_t c = perm0[col0[(int64_t)k * ld0 + s]];
        if (!boundary[c])
            continue;
        double q[3];
        nm_load<T>(pts, c, q);
        const double d = nm_d2(p, q);
        if (d < best || (d == best && c < bc)) {
            best = d;
            bc = c;
        }
    }
    // a flagged point has a boundary neighbour; the guard keeps an index in range regardless
    const int64_t bj = bc >= 0 ? (int64_t)brank[bc] : 0;
    double q[3];
    nm_load<T>(pts, bc >= 0 ? bc : i, q);
    const double *e = e3 + bj * 3;
    const double h = (p[0] - q[0]) * e[0] + (p[1] - q[1]) * e[1] + (p[2] - q[2]) * e[2];
    for (int a = 0; a < 3; ++a) {
        const double g = p[a] - 2.0 * h * e[a];
        aug[(n_interior + f) * 3 + a] = (T)g;
        if (ghost_xyz)
            ghost_xyz[f * 3 + a] = g;
    }
    ghost_src[f] = (int32_t)irank[i];
}

// interior points of the cloud into rows [0, n_interior) of the augmented cloud
template <typename T>
__global__ __launch_bounds__(256) void nm_gather_kernel(const T *__restrict__ pts,
                                                        const int32_t *__restrict__ il,
                                                        int64_t ni, T *__restrict__ aug)
{
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r < ni)
        for (int a = 0; a < 3; ++a)
            aug[r * 3 + a] = pts[(int64_t)il[r] * 3 + a];
}

// fold the ghost columns of the assembled augmented cloud into their sources; ghost rows become
// zero rows (columns: the row itself). A folded column that the row already holds (the source
// itself, or a second ghost of the same source) is merged into that entry, which leaves a zero
// entry in the ghost's slot (column: the row itself), so every nonzero column appears once.
template <typename T>
__global__ __launch_bounds__(256) void nm_fold_kernel(int32_t *__restrict__ col, T *__restrict__ val,
                                                      const int32_t *__restrict__ perm,
                                                      const int32_t *__restrict__ ipos,
                                                      const int32_t *__restrict__ ghost_src,
                                                      int64_t n, int64_t ld, int slots,
                                                      int64_t n_interior)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n)
        return;
    if (perm[s] >= n_interior) {
        for (int k = 0; k < slots; ++k) {
            col[(int64_t)k * ld + s] = (int32_t)s;
            val[(int64_t)k * ld + s] = (T)0;
        }
        return;
    }
    uint64_t ghost = 0; // bit k - 1: slot k held a ghost column (slot 0 is the row itself)
    for (int k = 1; k < slots; ++k) {
        const int32_t a = perm[col[(int64_t)k * ld + s]];
        if (a >= n_interior) {
            col[(int64_t)k * ld + s] = ipos[ghost_src[a - n_interior]];
            ghost |= 1ull << (k - 1);
        }
    }
    for (int k = 1; k < slots; ++k) {
        if (!((ghost >> (k - 1)) & 1))
            continue;
        const int32_t c = col[(int64_t)k * ld + s];
        for (int j = 0; j < slots; ++j) {
            const bool earlier_ghost = j >= 1 && ((ghost >> (j - 1)) & 1) && j < k;
            const bool plain = j == 0 || !((ghost >> (j - 1)) & 1);
            if (j != k && (plain || earlier_ghost) && col[(int64_t)j * ld + s] == c) {
                val[(int64_t)j * ld + s] += val[(int64_t)k * ld + s];
                val[(int64_t)k * ld + s] = (T)0;
                col[(int64_t)k * ld + s] = (int32_t)s;
                break;
            }
        }
    }
}

} // namespace mvgd
