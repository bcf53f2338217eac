// capi.hip -- the C ABI declared in include/mvgd.h: argument checks, cell-grid sizing, device
// memory, and the launch sequence of the assembly and apply kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/mvgd.h"
#include "apply.hpp"
#include "assemble.hpp"
#include "bin.hpp"
#include "boundary.hpp"
#include "common.hpp"
#include "eigs.hpp"
#include "solve.hpp"
#include "stats.hpp"

using namespace mvgd;

namespace {

thread_local char g_err[512] = "";

mvgd_status fail(mvgd_status s, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return s;
}

// Neighbour-search tunables (mvgd_params; 0 selects these defaults).
constexpr double kDefaultCellAlpha = 0.6;
constexpr double kDefaultRadiusMu = 1.7;
constexpr double kDefaultCellsPerPoint = 8.0;

double tunable(float v, double dflt)
{
    return (v > 0.0f && std::isfinite(v)) ? (double)v : dflt;
}

// Allocation with an optional injected failure, to exercise the clean-up paths:
// MVGD_FAIL_ALLOC_AT="<n>[#tag]" makes the n-th device allocation (1-based) counted from the
// first allocation that saw this exact value fail; a new value re-arms the counter.
std::atomic<long> g_alloc_count{0};
std::mutex g_fail_mu;
std::string g_fail_seen;
long g_fail_base = 0;

// The library's own stream-ordered memory pool per device. Its release threshold is unbounded:
// memory freed by mvgd_free and by the end of an assembly stays mapped in the pool for the next
// call (a pool that trims at every synchronisation maps fresh pages on every assembly);
// mvgd_pool_trim hands it back.
constexpr int kMaxDevices = 64;
std::mutex g_pool_mu;
hipMemPool_t g_pool[kMaxDevices] = {};

hipError_t device_pool(hipMemPool_t *out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return e;
    if (dev < 0 || dev >= kMaxDevices)
        return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_pool_mu);
    if (!g_pool[dev]) {
        hipMemPoolProps props;
        memset(&props, 0, sizeof props);
        props.allocType = hipMemAllocationTypePinned;
        props.handleTypes = hipMemHandleTypeNone;
        props.location.type = hipMemLocationTypeDevice;
        props.location.id = dev;
        hipMemPool_t pool = nullptr;
        if ((e = hipMemPoolCreate(&pool, &props)) != hipSuccess)
            return e;
        uint64_t keep = UINT64_MAX;
        if ((e = hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep)) != hipSuccess) {
            (void)hipMemPoolDestroy(pool);
            return e;
        }
        g_pool[dev] = pool;
    }
    *out = g_pool[dev];
    return hipSuccess;
}

hipError_t dev_alloc(void **p, size_t bytes, hipStream_t s)
{
    *p = nullptr;
    const long n = ++g_alloc_count;
    const char *f = getenv("MVGD_FAIL_ALLOC_AT");
    if (f && *f) {
        std::lock_guard<std::mutex> lk(g_fail_mu);
        if (g_fail_seen != f) {
            g_fail_seen = f;
            g_fail_base = n - 1;
        }
        if (atol(f) == n - g_fail_base)
            return hipErrorOutOfMemory;
    }
    if (bytes == 0)
        bytes = 16;
    hipMemPool_t pool = nullptr;
    hipError_t e = device_pool(&pool);
    if (e != hipSuccess)
        return e;
    return hipMallocFromPoolAsync(p, bytes, pool, s);
}

int64_t next_pow2(int64_t v)
{
    int64_t p = 1;
    while (p < v)
        p <<= 1;
    return p;
}

mvgd_status check_launch(const char *what)
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return fail(MVGD_EDEVICE, "%s: %s", what, hipGetErrorString(e));
    return MVGD_OK;
}

bool is_device_pointer(const void *p, int device)
{
    hipPointerAttribute_t attr;
    memset(&attr, 0, sizeof attr);
    hipError_t e = hipPointerGetAttributes(&attr, p);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    if (attr.type != hipMemoryTypeDevice && attr.type != hipMemoryTypeManaged)
        return false;
    return attr.device == device;
}

} // namespace

struct mvgd_matrix {
    int device = 0;
    int precision = 0;
    int K = 0;
    int n_ambient = 0;
    uint32_t flags = 0;
    int64_t n_total = 0;
    int32_t n_clouds = 0;
    int64_t ld = 0;
    hipStream_t stream = nullptr; // stream of the last call on this handle
    void *block = nullptr;        // one device allocation holding every array below but xs
    int32_t *perm = nullptr;
    int32_t *ell_col = nullptr;
    void *ell_val = nullptr;
    CloudGrid *grids = nullptr;
    unsigned long long *counters = nullptr;
    double *row_h = nullptr;
    uint8_t *row_flags = nullptr;
    void *xs = nullptr;
    size_t xs_bytes = 0;
    size_t bytes = 0;
    // MVGD_FLAG_TIME: [0] start, [1] search start, [5] fit start, [2] assembly end, [3, 4] apply
    hipEvent_t ev[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    bool have_apply = false;
};

namespace {

void release(mvgd_matrix *L)
{
    if (!L)
        return;
    void *ptrs[] = {L->block, L->xs};
    for (void *p : ptrs)
        if (p)
            (void)hipFreeAsync(p, L->stream);
    for (hipEvent_t e : L->ev)
        if (e)
            (void)hipEventDestroy(e);
    delete L;
}

// The fixed binning projection (rows orthonormal): identity for n = 2 and 3, a generic 3x4
// matrix for n = 4 (see Proj in common.hpp).
Proj binning_projection(int n_amb)
{
    Proj pr;
    memset(&pr, 0, sizeof pr);
    if (n_amb <= 3) { // identity (n = 2: the third projected coordinate is 0)
        for (int a = 0; a < n_amb; ++a)
            pr.W[a][a] = 1.0;
        return pr;
    }
    static const double W4[3][4] = {
        {-0.5049971086679399, -0.7970289394280843, -0.09843310179405794, 0.3162810687068779},
        {-0.47371621671260017, 0.21177439071878815, -0.7273779116057677, -0.4490722961475343},
        {-0.4950075093018881, 0.01078809292873078, 0.6682902330051771, -0.5551930720529468}};
    memcpy(pr.W, W4, sizeof W4);
    return pr;
}

// Cell-table budget of one cloud (entries): a power of two, at least cells_per_point per point.
int64_t cell_budget(int64_t n, double cpp)
{
    return std::max<int64_t>(512, next_pow2((int64_t)std::ceil(cpp * (double)n)));
}

// Largest dim[0] + dim[1] + dim[2] of a grid with power-of-two dims of at most kMaxDim cells each
// and at most `cap` cells in all (the sum is largest when the dims are as unequal as possible).
int64_t part_bound(int64_t cap)
{
    int64_t left = cap, sum = 0;
    for (int a = 0; a < 3; ++a) {
        const int64_t d = std::max<int64_t>(1, std::min<int64_t>(kMaxDim, left));
        sum += d;
        left = std::max<int64_t>(1, left / d);
    }
    return sum;
}

// Carves 256-byte aligned pieces out of one allocation: a sizing pass (base == nullptr) adds up
// the bytes, a second pass hands out the pointers.
struct Carver {
    char *base = nullptr;
    size_t off = 0;
    template <typename P>
    void take(P *&dst, size_t bytes)
    {
        off = (off + 255) & ~(size_t)255;
        dst = base ? (P *)(base + off) : nullptr;
        off += bytes;
    }
};

// Page-locked staging for the per-call metadata upload and statistics read-back. One buffer per
// host thread, grown on demand and kept for the life of the process. Every assembly call
// synchronises its stream (after the statistics read-back, or before an error return) before it
// returns, so the next call on the same thread never overwrites a buffer a copy still reads.
thread_local void *t_stage = nullptr;
thread_local size_t t_stage_bytes = 0;

void *staging(size_t bytes)
{
    if (t_stage_bytes >= bytes)
        return t_stage;
    if (t_stage)
        (void)hipHostFree(t_stage);
    t_stage = nullptr;
    t_stage_bytes = 0;
    const size_t want = std::max<size_t>(bytes, 64 << 10);
    if (hipHostMalloc(&t_stage, want, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        t_stage = nullptr;
        return nullptr;
    }
    t_stage_bytes = want;
    return t_stage;
}

// Occupancy of the persistent assembly kernel (blocks per CU) per (precision, n, K), queried once.
std::atomic<int> g_occupancy[2][3][3]; // [double][n - 2][search mode]
std::atomic<int> g_n_cu{0};

// Persistent search kernel of a mode (0 group, 1 lane, 2 tile).
template <typename T, int NA>
const void *search_kernel_ptr(int smode)
{
    return smode == 2   ? (const void *)search_persistent_kernel<T, NA, 2>
           : smode == 1 ? (const void *)search_persistent_kernel<T, NA, 1>
                        : (const void *)search_persistent_kernel<T, NA, 0>;
}

template <typename T, int NA>
void launch_search(int smode, bool persistent, unsigned nblk, size_t lds, hipStream_t stream,
                   const AsmParams &ap)
{
    if (smode == 2) {
        if (persistent)
            search_persistent_kernel<T, NA, 2><<<nblk, kWave, lds, stream>>>(ap);
        else
            search_kernel<T, NA, 2><<<nblk, kWave, lds, stream>>>(ap);
        return;
    }
    if (persistent && smode == 1)
        search_persistent_kernel<T, NA, 1><<<nblk, kWave, lds, stream>>>(ap);
    else if (persistent)
        search_persistent_kernel<T, NA, 0><<<nblk, kWave, lds, stream>>>(ap);
    else if (smode == 1)
        search_kernel<T, NA, 1><<<nblk, kWave, lds, stream>>>(ap);
    else
        search_kernel<T, NA, 0><<<nblk, kWave, lds, stream>>>(ap);
}

template <typename T>
mvgd_status assemble_impl(const T *points, int64_t n_total, const std::vector<int64_t> &offs,
                          const mvgd_params &p, hipStream_t stream, mvgd_matrix **out)
{
    const int n_clouds = (int)offs.size() - 1;
    const int n_amb = p.n_ambient;
    const int K = p.k;
    int device = 0;
    if (hipGetDevice(&device) != hipSuccess)
        return fail(MVGD_EDEVICE, "no HIP device");
    if (!is_device_pointer(points, device))
        return fail(MVGD_EINVAL, "points is not device memory of the current device");

    // ---- 1. sizes, all known on the host: cell budgets, groups, part tables -------------------
    // meta: row offsets, then per cloud: first cell entry, cell budget, first group, first part
    const double cpp = tunable(p.cells_per_point, kDefaultCellsPerPoint);
    const size_t n_meta = (size_t)5 * n_clouds + 1;
    std::vector<int64_t> meta(n_meta);
    int64_t cell_total = 0, group_total = 0, part_total = 0, max_n = 0;
    for (int c = 0; c < n_clouds; ++c) {
        const int64_t n = offs[c + 1] - offs[c];
        const int64_t cap = cell_budget(n, cpp);
        meta[n_clouds + 1 + c] = cell_total;
        meta[2 * n_clouds + 1 + c] = cap;
        meta[3 * n_clouds + 1 + c] = group_total;
        meta[4 * n_clouds + 1 + c] = part_total;
        cell_total += cap;
        group_total += (n + kWave - 1) / kWave;
        part_total += part_bound(cap);
        max_n = std::max(max_n, n);
    }
    for (int c = 0; c <= n_clouds; ++c)
        meta[c] = offs[c];
    if (cell_total >= (int64_t)UINT32_MAX - 1)
        return fail(MVGD_EUNSUPPORTED, "cell table too large (%lld cells)", (long long)cell_total);
    std::vector<int64_t> lvl_n; // scan levels over the cell table
    for (int64_t m = cell_total; m > 1; m = (m + kScanTile - 1) / kScanTile)
        lvl_n.push_back(m);
    if (lvl_n.empty())
        lvl_n.push_back(std::max<int64_t>(cell_total, 1));

    mvgd_matrix *L = new (std::nothrow) mvgd_matrix();
    if (!L)
        return fail(MVGD_ENOMEM, "host allocation failed");
    L->device = device;
    L->precision = p.precision;
    L->K = K;
    L->n_ambient = n_amb;
    L->flags = p.flags;
    L->n_total = n_total;
    L->n_clouds = n_clouds;
    L->ld = (n_total + kWave - 1) / kWave * kWave;
    L->stream = stream;
    void *scratch = nullptr;
    bool staged = false; // a copy from/to the staging buffer may be in flight
    struct Guard {
        mvgd_matrix *&L;
        void *&scratch;
        bool &staged;
        hipStream_t s;
        ~Guard()
        {
            if (staged)
                (void)hipStreamSynchronize(s);
            if (scratch)
                (void)hipFreeAsync(scratch, s);
            if (L)
                release(L);
        }
    } guard{L, scratch, staged, stream};

    // ---- 2. two allocations: the handle's arrays and the assembly scratch ----------------------
    const size_t vsz = sizeof(T);
    const bool keep_diag = (p.flags & MVGD_FLAG_KEEP_DIAG) != 0;
    auto carve_handle = [&](Carver &cv) {
        cv.take(L->perm, sizeof(int32_t) * n_total);
        cv.take(L->ell_col, sizeof(int32_t) * (size_t)(K + 1) * L->ld);
        char *val = nullptr;
        cv.take(val, vsz * (size_t)(K + 1) * L->ld);
        L->ell_val = val;
        cv.take(L->grids, sizeof(CloudGrid) * n_clouds);
        cv.take(L->counters, sizeof(unsigned long long) * 8);
        if (keep_diag) {
            cv.take(L->row_h, sizeof(double) * n_total);
            cv.take(L->row_flags, (size_t)n_total);
        }
    };
    int64_t *d_meta;
    CloudStats *d_stats;
    double *d_bpart;
    // bounding boxes: blocks per cloud, each writing a partial box (folded by one block per cloud)
    const int bbx = (int)std::max<int64_t>(
        1, std::min<int64_t>((max_n + 1023) / 1024, std::max<int64_t>(8, 2048 / n_clouds)));
    uint32_t *d_parts, *d_counts, *d_start, *d_keys, *d_slots;
    unsigned int *d_queue;
    int32_t *d_iperm, *d_perm_tmp;
    Pt<T> *d_spts, *d_spts_tmp;
    std::vector<uint32_t *> lvl_sum(lvl_n.size()), lvl_off(lvl_n.size());
    auto carve_scratch = [&](Carver &cv) {
        cv.take(d_meta, sizeof(int64_t) * n_meta);
        cv.take(d_stats, sizeof(CloudStats) * n_clouds);
        cv.take(d_bpart, sizeof(double) * 16 * (size_t)bbx * (size_t)n_clouds);
        cv.take(d_parts, sizeof(uint32_t) * part_total);
        cv.take(d_counts, sizeof(uint32_t) * cell_total);
        cv.take(d_start, sizeof(uint32_t) * (cell_total + 1));
        cv.take(d_keys, sizeof(uint32_t) * n_total);
        cv.take(d_slots, sizeof(uint32_t) * n_total);
        cv.take(d_spts_tmp, sizeof(Pt<T>) * n_total);
        cv.take(d_perm_tmp, sizeof(int32_t) * n_total);
        cv.take(d_spts, sizeof(Pt<T>) * n_total);
        cv.take(d_queue, sizeof(unsigned int) * 8);
        cv.take(d_iperm, sizeof(int32_t) * n_total);
        for (size_t l = 0; l < lvl_n.size(); ++l) {
            const int64_t tiles = (lvl_n[l] + kScanTile - 1) / kScanTile;
            cv.take(lvl_sum[l], sizeof(uint32_t) * tiles);
            cv.take(lvl_off[l], sizeof(uint32_t) * tiles);
        }
    };
    {
        Carver h, t;
        carve_handle(h);
        carve_scratch(t);
        if (dev_alloc(&L->block, h.off, stream) != hipSuccess)
            return fail(MVGD_ENOMEM, "device allocation failed (matrix, %zu bytes)", h.off);
        L->bytes = h.off;
        if (dev_alloc(&scratch, t.off, stream) != hipSuccess)
            return fail(MVGD_ENOMEM, "device allocation failed (assembly scratch, %zu bytes)",
                        t.off);
        h = Carver{(char *)L->block, 0};
        t = Carver{(char *)scratch, 0};
        carve_handle(h);
        carve_scratch(t);
    }
    const size_t meta_bytes = sizeof(int64_t) * n_meta;
    const size_t stats_off = (meta_bytes + 255) & ~(size_t)255;
    char *stage = (char *)staging(stats_off + sizeof(CloudStats) * n_clouds);
    if (!stage)
        return fail(MVGD_ENOMEM, "page-locked staging allocation failed");
    memcpy(stage, meta.data(), meta_bytes);

    if (p.flags & MVGD_FLAG_TIME) {
        for (hipEvent_t &e : L->ev)
            if (hipEventCreate(&e) != hipSuccess)
                return fail(MVGD_EDEVICE, "hipEventCreate failed");
        (void)hipEventRecord(L->ev[0], stream);
    }
    // ---- 3. bounding boxes, grid plan, binning (no host round trip) ----------------------------
    staged = true;
    if (hipMemcpyAsync(d_meta, stage, meta_bytes, hipMemcpyHostToDevice, stream) != hipSuccess)
        return fail(MVGD_EDEVICE, "copy of cloud offsets failed");
    stats_init_kernel<<<(std::max(n_clouds, 8) + 255) / 256, 256, 0, stream>>>(
        d_stats, n_clouds, L->counters, d_queue);
    const Proj proj = binning_projection(n_amb);
    {
        if (n_amb == 2) {
            bbox_kernel<T, 2><<<dim3(bbx, n_clouds), 256, 0, stream>>>(points, d_meta, proj, d_bpart);
            bbox_reduce_kernel<2><<<n_clouds, 256, 0, stream>>>(d_bpart, bbx, d_stats);
        } else if (n_amb == 3) {
            bbox_kernel<T, 3><<<dim3(bbx, n_clouds), 256, 0, stream>>>(points, d_meta, proj, d_bpart);
            bbox_reduce_kernel<3><<<n_clouds, 256, 0, stream>>>(d_bpart, bbx, d_stats);
        } else {
            bbox_kernel<T, 4><<<dim3(bbx, n_clouds), 256, 0, stream>>>(points, d_meta, proj, d_bpart);
            bbox_reduce_kernel<4><<<n_clouds, 256, 0, stream>>>(d_bpart, bbx, d_stats);
        }
    }
    {
        PlanArgs pa;
        memset(&pa, 0, sizeof pa);
        pa.stats = d_stats;
        pa.meta = d_meta;
        pa.n_clouds = n_clouds;
        pa.n_amb = n_amb;
        pa.K = K;
        pa.d = p.d_manifold;
        pa.alpha = tunable(p.cell_alpha, kDefaultCellAlpha);
        pa.mu = tunable(p.radius_mu, kDefaultRadiusMu);
        pa.proj = proj;
        pa.grids = L->grids;
        pa.parts = d_parts;
        plan_kernel<<<n_clouds, 256, 0, stream>>>(pa);
    }
    if (hipMemsetAsync(d_counts, 0, sizeof(uint32_t) * cell_total, stream) != hipSuccess)
        return fail(MVGD_EDEVICE, "clearing the cell counts failed");
    const int bx = (int)std::max<int64_t>(1, std::min<int64_t>(65535, (n_total + 255) / 256));
    if (n_amb == 2)
        key_kernel<T, 2><<<bx, 256, 0, stream>>>(points, d_meta, n_clouds, n_total, L->grids,
                                                  d_parts, d_counts, d_keys, d_slots);
    else if (n_amb == 3)
        key_kernel<T, 3><<<bx, 256, 0, stream>>>(points, d_meta, n_clouds, n_total, L->grids,
                                                  d_parts, d_counts, d_keys, d_slots);
    else
        key_kernel<T, 4><<<bx, 256, 0, stream>>>(points, d_meta, n_clouds, n_total, L->grids,
                                                  d_parts, d_counts, d_keys, d_slots);
    // exclusive scan of the counts, level by level
    {
        const uint32_t *in = d_counts;
        uint32_t *o = d_start;
        for (size_t l = 0; l < lvl_n.size(); ++l) {
            const int64_t tiles = (lvl_n[l] + kScanTile - 1) / kScanTile;
            scan_tile_kernel<<<(unsigned)tiles, kScanThreads, 0, stream>>>(in, o, lvl_sum[l], lvl_n[l]);
            in = lvl_sum[l];
            o = lvl_off[l];
        }
        for (size_t l = lvl_n.size(); l-- > 1;) {
            uint32_t *dst = (l - 1 == 0) ? d_start : lvl_off[l - 2];
            scan_add_kernel<<<(unsigned)((lvl_n[l - 1] + kScanTile - 1) / kScanTile), kScanThreads,
                              0, stream>>>(dst, lvl_off[l - 1], lvl_n[l - 1]);
        }
        scan_total_kernel<<<1, 64, 0, stream>>>(d_counts, d_start, cell_total);
    }
    scatter_kernel<T><<<bx, 256, 0, stream>>>(points, n_amb, n_total, d_start, d_keys, d_slots,
                                               d_spts_tmp, d_perm_tmp);
    canon_kernel<T><<<(unsigned)((n_total + 255) / 256), 256, 0, stream>>>(
        n_total, d_start, d_keys, d_spts_tmp, d_perm_tmp, d_spts, L->perm, d_iperm);
    if (mvgd_status st = check_launch("binning"); st != MVGD_OK)
        return st;

    // ---- 4. the one synchronisation: non-finite coordinates are rejected before the search ----
    CloudStats *hs = (CloudStats *)(stage + stats_off);
    if (hipMemcpyAsync(hs, d_stats, sizeof(CloudStats) * n_clouds, hipMemcpyDeviceToHost,
                       stream) != hipSuccess ||
        hipStreamSynchronize(stream) != hipSuccess)
        return fail(MVGD_EDEVICE, "reading the cloud statistics failed: %s",
                    hipGetErrorString(hipGetLastError()));
    staged = false;
    for (int c = 0; c < n_clouds; ++c)
        if (hs[c].nonfinite)
            return fail(MVGD_EINVAL, "cloud %d has %llu non-finite coordinates", c,
                        (unsigned long long)hs[c].nonfinite);

    // ---- 5. fused neighbour search + fit + stencil ------------------------------------------
    AsmParams ap;
    memset(&ap, 0, sizeof ap);
    ap.spts = d_spts;
    ap.perm = L->perm;
    ap.iperm = d_iperm;
    ap.cell_start = d_start;
    ap.parts = d_parts;
    ap.grids = L->grids;
    ap.n_clouds = n_clouds;
    ap.K = K;
    ap.n_groups = group_total;
    ap.groups_per_xcd = (group_total + 7) / 8;
    ap.variant = (p.flags & MVGD_FLAG_LS) ? 1 : (p.flags & MVGD_FLAG_DIVERGENCE) ? 2 : 0;
    ap.use_h = (p.flags & MVGD_FLAG_H_OVERRIDE) ? 1 : 0;
    ap.h_override = p.h_override;
    ap.w_nbr = (p.flags & MVGD_FLAG_MLS) ? 1.0 / (double)K : 1.0;
    ap.ld = L->ld;
    ap.n_rows = n_total;
    ap.ell_col = L->ell_col;
    ap.ell_val = L->ell_val;
    ap.row_h = L->row_h;
    ap.row_flags = L->row_flags;
    ap.counters = L->counters;
    ap.queue = d_queue;
    const int d = p.d_manifold;
    // search mode: 0 group, 1 lane, 2 tile (the default)
    const int smode = p.search == MVGD_SEARCH_LANE ? 1 : p.search == MVGD_SEARCH_GROUP ? 0 : 2;
    const size_t lds = (size_t)search_lds_bytes((int)sizeof(Pt<T>), smode);
    const bool persistent = p.launch == MVGD_LAUNCH_PERSISTENT;
    unsigned nblk = (unsigned)(ap.groups_per_xcd * 8);
    if (persistent) {
        std::atomic<int> &occ = g_occupancy[sizeof(T) == 8][n_amb - 2][smode];
        int per_cu = occ.load(), n_cu = g_n_cu.load();
        if (per_cu <= 0 || n_cu <= 0) {
            const void *kern = n_amb == 4   ? search_kernel_ptr<T, 4>(smode)
                               : n_amb == 3 ? search_kernel_ptr<T, 3>(smode)
                                            : search_kernel_ptr<T, 2>(smode);
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, kWave, lds) != hipSuccess ||
                hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess)
                return fail(MVGD_EDEVICE, "occupancy query failed");
            per_cu = std::max(per_cu, 1);
            n_cu = std::max(n_cu, 1);
            occ.store(per_cu);
            g_n_cu.store(n_cu);
        }
        const int64_t resident = (int64_t)per_cu * n_cu;
        nblk = (unsigned)std::min<int64_t>((resident + 7) / 8 * 8, ap.groups_per_xcd * 8);
    }
    if (L->ev[1])
        (void)hipEventRecord(L->ev[1], stream);
    // neighbour search: lists of original indices into ELL slots 1..K
    if (n_amb == 4)
        launch_search<T, 4>(smode, persistent, nblk, lds, stream, ap);
    else if (n_amb == 3)
        launch_search<T, 3>(smode, persistent, nblk, lds, stream, ap);
    else
        launch_search<T, 2>(smode, persistent, nblk, lds, stream, ap);
    if (mvgd_status st = check_launch("neighbour search"); st != MVGD_OK)
        return st;
    if (L->ev[5])
        (void)hipEventRecord(L->ev[5], stream);
    // fit and stencil, one wave per 64 rows
    {
        const unsigned fb = (unsigned)((n_total + kWave - 1) / kWave);
        const size_t flds = (size_t)fit_lds_bytes(K);
        if (d == 2 && n_amb == 3)
            fit_kernel<T, 3, 2><<<fb, kWave, flds, stream>>>(ap);
        else if (d == 2)
            fit_kernel<T, 4, 2><<<fb, kWave, flds, stream>>>(ap);
        else if (n_amb == 3)
            fit_kernel<T, 3, 1><<<fb, kWave, flds, stream>>>(ap);
        else
            fit_kernel<T, 2, 1><<<fb, kWave, flds, stream>>>(ap);
    }
    if (mvgd_status st = check_launch("assemble"); st != MVGD_OK)
        return st;
    if (L->ev[2])
        (void)hipEventRecord(L->ev[2], stream);
    *out = L;
    L = nullptr; // ownership passes to the caller; the scratch is freed stream-ordered
    return MVGD_OK;
}

mvgd_status validate(const void *points, int64_t n_total, const int64_t *cloud_offsets,
                     int32_t n_clouds, const mvgd_params *p, mvgd_matrix **out,
                     std::vector<int64_t> &offs)
{
    if (!out)
        return fail(MVGD_EINVAL, "out is NULL");
    *out = nullptr;
    if (!points || !p)
        return fail(MVGD_EINVAL, "points or params is NULL");
    if (p->d_manifold != 1 && p->d_manifold != 2)
        return fail(MVGD_EINVAL, "d_manifold must be 1 or 2 (got %d)", p->d_manifold);
    if (p->d_manifold == 2 && p->n_ambient != 3 && p->n_ambient != 4)
        return fail(MVGD_EINVAL, "surfaces need n_ambient 3 or 4 (got %d)", p->n_ambient);
    if (p->d_manifold == 1 && p->n_ambient != 2 && p->n_ambient != 3)
        return fail(MVGD_EINVAL, "curves need n_ambient 2 or 3 (got %d)", p->n_ambient);
    const int k_min = p->d_manifold == 2 ? 5 : 2; // at least as many points as monomials
    if (p->k < k_min || p->k > kMaxK)
        return fail(MVGD_EINVAL, "k must be in [%d, %d] (got %d)", k_min, kMaxK, p->k);
    if (p->precision != MVGD_FP64 && p->precision != MVGD_FP32_MIXED)
        return fail(MVGD_EINVAL, "unknown precision %d", p->precision);
    if (p->flags & ~(uint32_t)(MVGD_FLAG_LS | MVGD_FLAG_H_OVERRIDE | MVGD_FLAG_KEEP_DIAG |
                             MVGD_FLAG_TIME | MVGD_FLAG_MLS | MVGD_FLAG_DIVERGENCE))
        return fail(MVGD_EINVAL, "unknown flag bits 0x%x", p->flags);
    if ((p->flags & MVGD_FLAG_DIVERGENCE) &&
        (p->d_manifold != 1 || (p->flags & MVGD_FLAG_LS)))
        return fail(MVGD_EINVAL, "the divergence form is for curves (d = 1) and excludes LS");
    if ((p->flags & MVGD_FLAG_H_OVERRIDE) && !(p->h_override > 0.0 && std::isfinite(p->h_override)))
        return fail(MVGD_EINVAL, "h_override must be positive and finite");
    if (p->launch < MVGD_LAUNCH_DEFAULT || p->launch > MVGD_LAUNCH_PERSISTENT)
        return fail(MVGD_EINVAL, "unknown launch mode %d", p->launch);
    if (p->search < MVGD_SEARCH_DEFAULT || p->search > MVGD_SEARCH_TILE)
        return fail(MVGD_EINVAL, "unknown search mode %d", p->search);
    if (p->cell_alpha < 0.0f || p->radius_mu < 0.0f || p->cells_per_point < 0.0f ||
        !std::isfinite(p->cell_alpha) || !std::isfinite(p->radius_mu) ||
        !std::isfinite(p->cells_per_point) || (p->cells_per_point > 0.0f && p->cells_per_point < 0.25f) ||
        p->cells_per_point > 64.0f || (p->radius_mu > 0.0f && p->radius_mu < 0.1f))
        return fail(MVGD_EINVAL, "tuning values out of range");
    if (n_total <= 0 || n_total >= (int64_t(1) << 31))
        return fail(MVGD_EINVAL, "n_total must be in [1, 2^31)");
    if (cloud_offsets) {
        if (n_clouds < 1 || n_clouds > 65535)
            return fail(MVGD_EINVAL, "n_clouds must be in [1, 65535]");
        offs.assign(cloud_offsets, cloud_offsets + n_clouds + 1);
    } else {
        offs = {0, n_total};
    }
    if (offs.front() != 0 || offs.back() != n_total)
        return fail(MVGD_EINVAL, "cloud offsets must start at 0 and end at n_total");
    for (size_t c = 0; c + 1 < offs.size(); ++c)
        if (offs[c + 1] - offs[c] < (int64_t)p->k + 1)
            return fail(MVGD_EINVAL, "cloud %zu has %lld points; needs more than k = %d", c,
                        (long long)(offs[c + 1] - offs[c]), p->k);
    return MVGD_OK;
}

// Exclusive prefix sum of n uint32 into out[0..n] (out[n] = total), stream-ordered; the level
// buffers come from one pool allocation freed stream-ordered.
mvgd_status scan_u32(const uint32_t *in, uint32_t *out, int64_t n, hipStream_t s)
{
    if (n <= 0) {
        scan_total_kernel<<<1, 64, 0, s>>>(in, out, 0);
        return check_launch("scan");
    }
    std::vector<int64_t> lvl_n;
    for (int64_t m = n; m > 1; m = (m + kScanTile - 1) / kScanTile)
        lvl_n.push_back(m);
    if (lvl_n.empty())
        lvl_n.push_back(n);
    std::vector<uint32_t *> lvl_sum(lvl_n.size()), lvl_off(lvl_n.size());
    auto carve = [&](Carver &cv) {
        for (size_t l = 0; l < lvl_n.size(); ++l) {
            const int64_t tiles = (lvl_n[l] + kScanTile - 1) / kScanTile;
            cv.take(lvl_sum[l], sizeof(uint32_t) * tiles);
            cv.take(lvl_off[l], sizeof(uint32_t) * tiles);
        }
    };
    Carver sz;
    carve(sz);
    void *work = nullptr;
    if (dev_alloc(&work, sz.off, s) != hipSuccess)
        return fail(MVGD_ENOMEM, "device allocation failed (scan, %zu bytes)", sz.off);
    Carver cv{(char *)work, 0};
    carve(cv);
    const uint32_t *src = in;
    uint32_t *o = out;
    for (size_t l = 0; l < lvl_n.size(); ++l) {
        const int64_t tiles = (lvl_n[l] + kScanTile - 1) / kScanTile;
        scan_tile_kernel<<<(unsigned)tiles, kScanThreads, 0, s>>>(src, o, lvl_sum[l], lvl_n[l]);
        src = lvl_sum[l];
        o = lvl_off[l];
    }
    for (size_t l = lvl_n.size(); l-- > 1;) {
        uint32_t *dst = (l - 1 == 0) ? out : lvl_off[l - 2];
        scan_add_kernel<<<(unsigned)((lvl_n[l - 1] + kScanTile - 1) / kScanTile), kScanThreads, 0,
                          s>>>(dst, lvl_off[l - 1], lvl_n[l - 1]);
    }
    scan_total_kernel<<<1, 64, 0, s>>>(in, out, n);
    (void)hipFreeAsync(work, s);
    return check_launch("scan");
}

template <typename T>
mvgd_status neumann_impl(const T *points, int64_t n, const uint8_t *boundary, int kb,
                         const mvgd_params &p, hipStream_t s, mvgd_matrix **out,
                         double *ghost_xyz, int32_t *ghost_src, mvgd_neumann_info *info)
{
    const int K = p.k;
    const std::vector<int64_t> whole = {0, n};
    mvgd_matrix *H0 = nullptr;
    if (mvgd_status st = assemble_impl<T>(points, n, whole, p, s, &H0); st != MVGD_OK)
        return st;
    struct Free0 {
        mvgd_matrix *&h;
        ~Free0() { if (h) release(h); }
    } free0{H0};
    // work: flags and their prefix sums, lists, inverse permutation, frames, augmented cloud
    uint32_t *flag, *isi, *isb, *rf, *ri, *rb;
    int32_t *fl, *il, *bl, *ipos0, *ipos1;
    double *e3;
    T *aug;
    auto carve = [&](Carver &cv) {
        for (uint32_t **v : {&flag, &isi, &isb})
            cv.take(*v, sizeof(uint32_t) * (size_t)n);
        for (uint32_t **v : {&rf, &ri, &rb})
            cv.take(*v, sizeof(uint32_t) * (size_t)(n + 1));
        for (int32_t **v : {&fl, &il, &bl, &ipos0})
            cv.take(*v, sizeof(int32_t) * (size_t)n);
        cv.take(ipos1, sizeof(int32_t) * (size_t)(2 * n)); // the augmented cloud: n_i + n_f <= 2n
        cv.take(e3, sizeof(double) * 3 * (size_t)n);
        cv.take(aug, sizeof(T) * 3 * (size_t)(2 * n));
    };
    Carver sz;
    carve(sz);
    void *work = nullptr;
    if (dev_alloc(&work, sz.off, s) != hipSuccess)
        return fail(MVGD_ENOMEM, "device allocation failed (Neumann work, %zu bytes)", sz.off);
    struct FreeW {
        void *w;
        hipStream_t s;
        ~FreeW() { (void)hipFreeAsync(w, s); }
    } freew{work, s};
    Carver cv{(char *)work, 0};
    carve(cv);
    const unsigned nb256 = (unsigned)((n + 255) / 256);
    nm_flag_kernel<<<nb256, 256, 0, s>>>(H0->ell_col, H0->perm, boundary, n, H0->ld, K, flag, isi,
                                         isb);
    for (auto pr : {std::make_pair(isi, ri), std::make_pair(isb, rb), std::make_pair(flag, rf)})
        if (mvgd_status st = scan_u32(pr.first, pr.second, n, s); st != MVGD_OK)
            return st;
    nm_compact_kernel<<<nb256, 256, 0, s>>>(isi, ri, n, il);
    nm_compact_kernel<<<nb256, 256, 0, s>>>(isb, rb, n, bl);
    nm_compact_kernel<<<nb256, 256, 0, s>>>(flag, rf, n, fl);
    nm_inverse_kernel<<<nb256, 256, 0, s>>>(H0->perm, n, ipos0);
    uint32_t tot[3] = {0, 0, 0};
    if (hipMemcpyAsync(&tot[0], ri + n, 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipMemcpyAsync(&tot[1], rb + n, 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipMemcpyAsync(&tot[2], rf + n, 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return fail(MVGD_EDEVICE, "reading the boundary counts failed");
    const int64_t ni = tot[0], nbd = tot[1], nf = tot[2];
    if (nbd < kb)
        return fail(MVGD_EINVAL, "%lld boundary points; k_boundary = %d needs at least as many",
                    (long long)nbd, kb);
    if (ni < K + 1)
        return fail(MVGD_EINVAL, "%lld interior points; needs more than k = %d", (long long)ni, K);
    if (nbd > 0) // one wave per boundary point
        nm_frame_kernel<T><<<(unsigned)nbd, 64, 0, s>>>(points, bl, nbd, kb, H0->ell_col, H0->perm,
                                                        ipos0, H0->ld, K, e3);
    nm_gather_kernel<T><<<(unsigned)((ni + 255) / 256), 256, 0, s>>>(points, il, ni, aug);
    if (nf > 0)
        nm_ghost_kernel<T><<<(unsigned)((nf + 255) / 256), 256, 0, s>>>(
            points, fl, nf, boundary, rb, H0->ell_col, H0->perm, ipos0, H0->ld, K, e3, ri, ni, aug,
            ghost_src, ghost_xyz);
    if (mvgd_status st = check_launch("ghost points"); st != MVGD_OK)
        return st;
    const std::vector<int64_t> whole_aug = {0, ni + nf};
    mvgd_matrix *H = nullptr;
    if (mvgd_status st = assemble_impl<T>(aug, ni + nf, whole_aug, p, s, &H); st != MVGD_OK)
        return st;
    // fold, through the inverse permutation of the augmented assembly
    nm_inverse_kernel<<<(unsigned)((ni + nf + 255) / 256), 256, 0, s>>>(H->perm, ni + nf, ipos1);
    nm_fold_kernel<T><<<(unsigned)((ni + nf + 255) / 256), 256, 0, s>>>(
        H->ell_col, (T *)H->ell_val, H->perm, ipos1, ghost_src, ni + nf, H->ld, K + 1, ni);
    if (mvgd_status st = check_launch("fold"); st != MVGD_OK) {
        release(H);
        return st;
    }
    info->n_interior = ni;
    info->n_ghost = nf;
    *out = H;
    return MVGD_OK;
}

} // namespace

extern "C" {

mvgd_status mvgd_assemble_neumann(const void *points, int64_t n_total, const uint8_t *boundary,
                                  int32_t k_boundary, const mvgd_params *p, void *stream,
                                  mvgd_matrix **out, double *ghost_xyz, int32_t *ghost_src,
                                  mvgd_neumann_info *info)
{
    std::vector<int64_t> offs;
    mvgd_status st = validate(points, n_total, nullptr, 1, p, out, offs);
    if (st != MVGD_OK)
        return st;
    if (!boundary || !ghost_src || !info)
        return fail(MVGD_EINVAL, "boundary, ghost_src or info is NULL");
    if (p->n_ambient != 3 || p->d_manifold != 2)
        return fail(MVGD_EUNSUPPORTED, "the Neumann condition is built for surfaces in R^3");
    if (k_boundary < 3 || k_boundary > 16)
        return fail(MVGD_EINVAL, "k_boundary must be in [3, 16] (got %d)", k_boundary);
    memset(info, 0, sizeof *info);
    int device = 0;
    if (hipGetDevice(&device) != hipSuccess)
        return fail(MVGD_EDEVICE, "no HIP device");
    if (!is_device_pointer(boundary, device) || !is_device_pointer(ghost_src, device) ||
        (ghost_xyz && !is_device_pointer(ghost_xyz, device)))
        return fail(MVGD_EINVAL, "boundary, ghost_src and ghost_xyz must be device memory");
    hipStream_t s = (hipStream_t)stream;
    if (p->precision == MVGD_FP64)
        return neumann_impl<double>((const double *)points, n_total, boundary, k_boundary, *p, s,
                                    out, ghost_xyz, ghost_src, info);
    return neumann_impl<float>((const float *)points, n_total, boundary, k_boundary, *p, s, out,
                               ghost_xyz, ghost_src, info);
}

mvgd_status mvgd_assemble(const void *points, int64_t n_total, const int64_t *cloud_offsets,
                          int32_t n_clouds, const mvgd_params *p, void *stream, mvgd_matrix **out)
{
    std::vector<int64_t> offs;
    mvgd_status st = validate(points, n_total, cloud_offsets, n_clouds, p, out, offs);
    if (st != MVGD_OK)
        return st;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
        (void)hipGetLastError();
        return fail(MVGD_EDEVICE, "no HIP device available");
    }
    hipStream_t s = (hipStream_t)stream;
    if (p->precision == MVGD_FP64)
        return assemble_impl<double>((const double *)points, n_total, offs, *p, s, out);
    return assemble_impl<float>((const float *)points, n_total, offs, *p, s, out);
}

mvgd_status mvgd_apply(mvgd_matrix *L, const void *x, void *y, int32_t nrhs, void *stream)
{
    if (!L || !x || !y)
        return fail(MVGD_EINVAL, "NULL argument");
    if (nrhs < 1 || nrhs > 64)
        return fail(MVGD_EINVAL, "nrhs must be in [1, 64]");
    hipStream_t s = (hipStream_t)stream;
    if (!is_device_pointer(x, L->device) || !is_device_pointer(y, L->device))
        return fail(MVGD_EINVAL, "x and y must be device memory of the matrix's device");
    const size_t vsz = L->precision == MVGD_FP64 ? 8 : 4;
    const size_t need = vsz * (size_t)L->n_total * nrhs;
    {
        const char *xb = (const char *)x, *yb = (const char *)y;
        if (xb < yb + need && yb < xb + need)
            return fail(MVGD_EINVAL, "x and y overlap");
    }
    if (L->xs_bytes < need) {
        if (L->xs)
            (void)hipFreeAsync(L->xs, L->stream);
        L->xs = nullptr;
        L->xs_bytes = 0;
        void *v = nullptr;
        if (dev_alloc(&v, need, s) != hipSuccess)
            return fail(MVGD_ENOMEM, "apply staging allocation failed (%zu bytes)", need);
        L->xs = v;
        L->xs_bytes = need;
    }
    L->stream = s;
    const int64_t n = L->n_total;
    const int slots = L->K + 1;
    const int64_t nt = n * nrhs;
    const unsigned gb = (unsigned)((nt + 255) / 256), rb = (unsigned)((n + 255) / 256);
    auto run = [&](auto tag) {
        using T = decltype(tag);
        const T *xx = (const T *)x;
        T *xs = (T *)L->xs, *yy = (T *)y;
        const T *val = (const T *)L->ell_val;
        gather_rows_kernel<T><<<gb, 256, 0, s>>>(xx, L->perm, xs, n, nrhs);
        switch (nrhs) {
        case 1: spmv_ell_kernel<T, 1><<<rb, 256, 0, s>>>(L->ell_col, val, xs, L->perm, yy, n, L->ld, slots); break;
        case 2: spmv_ell_kernel<T, 2><<<rb, 256, 0, s>>>(L->ell_col, val, xs, L->perm, yy, n, L->ld, slots); break;
        case 4: spmv_ell_kernel<T, 4><<<rb, 256, 0, s>>>(L->ell_col, val, xs, L->perm, yy, n, L->ld, slots); break;
        case 8: spmv_ell_kernel<T, 8><<<rb, 256, 0, s>>>(L->ell_col, val, xs, L->perm, yy, n, L->ld, slots); break;
        default:
            spmv_ell_any_kernel<T><<<gb, 256, 0, s>>>(L->ell_col, val, xs, L->perm, yy, n, L->ld, slots, nrhs);
        }
    };
    if (L->ev[3])
        (void)hipEventRecord(L->ev[3], s);
    if (L->precision == MVGD_FP64)
        run(double());
    else
        run(float());
    if (L->ev[4]) {
        (void)hipEventRecord(L->ev[4], s);
        L->have_apply = true;
    }
    return check_launch("apply");
}

void mvgd_free(mvgd_matrix *L)
{
    release(L);
}

mvgd_status mvgd_csr(mvgd_matrix *L, int64_t *row_ptr, int32_t *col, void *val, void *stream)
{
    if (!L)
        return fail(MVGD_EINVAL, "NULL matrix");
    hipStream_t s = (hipStream_t)stream;
    if ((row_ptr && !is_device_pointer(row_ptr, L->device)) ||
        (col && !is_device_pointer(col, L->device)) || (val && !is_device_pointer(val, L->device)))
        return fail(MVGD_EINVAL, "CSR buffers must be device memory of the matrix's device");
    L->stream = s;
    const int64_t n = L->n_total;
    const unsigned nb = (unsigned)((n + 63) / 64);
    if (L->precision == MVGD_FP64)
        export_csr_kernel<double><<<nb, 64, 0, s>>>(L->ell_col, (const double *)L->ell_val, L->perm,
                                                    L->grids, L->n_clouds, n, L->ld, L->K + 1,
                                                    row_ptr, col, (double *)val);
    else
        export_csr_kernel<float><<<nb, 64, 0, s>>>(L->ell_col, (const float *)L->ell_val, L->perm,
                                                   L->grids, L->n_clouds, n, L->ld, L->K + 1,
                                                   row_ptr, col, (float *)val);
    return check_launch("csr export");
}

mvgd_status mvgd_row_diag(mvgd_matrix *L, double *h, uint8_t *status, void *stream)
{
    if (!L)
        return fail(MVGD_EINVAL, "NULL matrix");
    if (!L->row_h)
        return fail(MVGD_EINVAL, "the matrix was assembled without MVGD_FLAG_KEEP_DIAG");
    if ((h && !is_device_pointer(h, L->device)) || (status && !is_device_pointer(status, L->device)))
        return fail(MVGD_EINVAL, "diagnostic buffers must be device memory of the matrix's device");
    hipStream_t s = (hipStream_t)stream;
    L->stream = s;
    const int64_t n = L->n_total;
    diag_scatter_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(L->row_h, L->row_flags, L->perm,
                                                                   h, status, n);
    return check_launch("row diagnostics");
}

mvgd_status mvgd_info(mvgd_matrix *L, mvgd_info_t *info)
{
    if (!L || !info)
        return fail(MVGD_EINVAL, "NULL argument");
    unsigned long long c[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    if (hipMemcpyAsync(c, L->counters, sizeof c, hipMemcpyDeviceToHost, L->stream) != hipSuccess ||
        hipStreamSynchronize(L->stream) != hipSuccess)
        return fail(MVGD_EDEVICE, "reading counters failed");
    if (c[2])
        return fail(MVGD_EDEVICE, "internal consistency check failed on %llu rows", c[2]);
    memset(info, 0, sizeof *info);
    info->n_rows = L->n_total;
    info->n_clouds = L->n_clouds;
    info->k = L->K;
    info->nnz = L->n_total * (L->K + 1);
    info->precision = L->precision;
    info->n_ambient = L->n_ambient;
    info->n_degenerate = (int64_t)c[0];
    info->n_slow_knn = (int64_t)c[1];
    info->device_bytes = L->bytes + L->xs_bytes;
    info->n_subgroups = (int64_t)c[3];
    info->n_streamed = (int64_t)c[4];
    info->n_growths = (int64_t)c[5];
    return MVGD_OK;
}

mvgd_status mvgd_row_stats(mvgd_matrix *L, double *ratio, mvgd_row_stats_t *out, void *stream)
{
    if (!L || !out)
        return fail(MVGD_EINVAL, "NULL argument");
    hipStream_t s = (hipStream_t)stream;
    if (ratio && !is_device_pointer(ratio, L->device))
        return fail(MVGD_EINVAL, "ratio must be device memory of the matrix's device");
    L->stream = s;
    const int64_t n = L->n_total;
    const int64_t rows_per_block = 4 * kStatsThreads;
    const int n_parts = (int)((n + rows_per_block - 1) / rows_per_block);
    void *v = nullptr;
    if (dev_alloc(&v, sizeof(RowStatsPart) * (size_t)(n_parts + 1), s) != hipSuccess)
        return fail(MVGD_ENOMEM, "device allocation failed (row statistics)");
    RowStatsPart *parts = (RowStatsPart *)v;
    if (L->precision == MVGD_FP64)
        row_stats_kernel<double><<<n_parts, kStatsThreads, 0, s>>>(
            (const double *)L->ell_val, L->perm, n, L->ld, L->K + 1, rows_per_block, ratio, parts);
    else
        row_stats_kernel<float><<<n_parts, kStatsThreads, 0, s>>>(
            (const float *)L->ell_val, L->perm, n, L->ld, L->K + 1, rows_per_block, ratio, parts);
    row_stats_final_kernel<<<1, kStatsThreads, 0, s>>>(parts, n_parts);
    RowStatsPart tot;
    const mvgd_status st = check_launch("row statistics");
    const bool ok = st == MVGD_OK &&
                    hipMemcpyAsync(&tot, parts + n_parts, sizeof tot, hipMemcpyDeviceToHost, s) ==
                        hipSuccess &&
                    hipStreamSynchronize(s) == hipSuccess;
    (void)hipFreeAsync(v, s);
    if (!ok)
        return st != MVGD_OK ? st : fail(MVGD_EDEVICE, "reading the row statistics failed");
    memset(out, 0, sizeof *out);
    out->n_rows = n;
    out->n_diag_negative = (int64_t)tot.n_diag_neg;
    out->n_m_rows = (int64_t)tot.n_m_rows;
    out->n_offdiag_negative = (int64_t)tot.n_off_neg;
    out->n_zero_diagonal = (int64_t)tot.n_zero_diag;
    const int64_t nz = n - (int64_t)tot.n_zero_diag;
    out->mean_ratio = nz > 0 ? tot.sum_ratio / (double)nz : 0.0;
    out->max_ratio = tot.max_ratio;
    return MVGD_OK;
}

} // extern "C"

namespace {

template <typename T>
mvgd_status solve_impl(mvgd_matrix *L, const void *b, void *x, const mvgd_solve_params &p,
                       mvgd_solve_info *info, hipStream_t s)
{
    const int64_t n = L->n_total, ld = L->ld;
    const int slots = L->K + 1;
    const int nb = (int)((n + kSolveThreads - 1) / kSolveThreads);
    const T *val = (const T *)L->ell_val;
    const int32_t *col = L->ell_col;
    const double sigma = p.sigma;
    const int check = p.check_every > 0 ? p.check_every : 16;
    const double omega = p.omega > 0.0 ? p.omega : 2.0 / 3.0;
    const int is_double = sizeof(T) == 8;
    // one allocation: 8 vectors, the partials, the scalars, the pinned-row mask
    double *vb, *vx, *vr, *vrh, *vp, *vv, *vs, *vt, *part;
    SolveScalars *sc;
    uint8_t *pinned;
    auto carve = [&](Carver &cv) {
        for (double **v : {&vb, &vx, &vr, &vrh, &vp, &vv, &vs, &vt})
            cv.take(*v, sizeof(double) * (size_t)n);
        cv.take(part, sizeof(double) * 2 * (size_t)nb);
        cv.take(sc, sizeof(SolveScalars));
        cv.take(pinned, (size_t)n);
    };
    Carver sz;
    carve(sz);
    void *work = nullptr;
    if (dev_alloc(&work, sz.off, s) != hipSuccess)
        return fail(MVGD_ENOMEM, "device allocation failed (solver work, %zu bytes)", sz.off);
    Carver cv{(char *)work, 0};
    carve(cv);
    struct Release {
        void *w;
        hipStream_t s;
        ~Release() { (void)hipFreeAsync(w, s); }
    } release_work{work, s};

    solve_setup_kernel<<<nb, kSolveThreads, 0, s>>>(L->perm, L->grids, L->n_clouds, n, p.pin_first,
                                                    p.fixed, b, x, is_double, vb, vx, pinned);
    bicg_init_kernel<T><<<nb, kSolveThreads, 0, s>>>(col, val, n, ld, slots, pinned, sigma, vx, vb,
                                                     vr, vrh, vp, vv, part);
    solve_scalar_kernel<<<1, kSolveThreads, 0, s>>>(kStepInit, part, nb, 2, sc, p.rtol);
    double *xcur = vx;
    SolveScalars hs;
    memset(&hs, 0, sizeof hs);
    auto read_scalars = [&]() {
        return hipMemcpyAsync(&hs, sc, sizeof hs, hipMemcpyDeviceToHost, s) == hipSuccess &&
               hipStreamSynchronize(s) == hipSuccess;
    };
    int prior_iters = 0; // BiCGSTAB: iterations of the cycles before a restart
    if (p.method == MVGD_SOLVE_BICGSTAB) {
        // The recursively updated residual can drift from b - A x over thousands of iterations.
        // When it passes the test, the true residual is formed; if that one fails, BiCGSTAB restarts
        // from the current iterate (at most kMaxRestarts times).
        constexpr int kMaxRestarts = 4;
        for (int cycle = 0;; ++cycle) {
            const int budget = p.max_iter - prior_iters;
            bicg_first_rho_kernel<<<1, 1, 0, s>>>(sc);
            for (int it = 0; it < budget;) {
                const int batch = std::min(check, budget - it);
                for (int j = 0; j < batch; ++j, ++it) {
                    bicg_p_kernel<<<nb, kSolveThreads, 0, s>>>(n, vr, vv, vp, sc, it == 0);
                    bicg_v_kernel<T><<<nb, kSolveThreads, 0, s>>>(col, val, n, ld, slots, pinned, sigma,
                                                                  vp, vrh, vv, part, sc);
                    solve_scalar_kernel<<<1, kSolveThreads, 0, s>>>(kStepAlpha, part, nb, 1, sc, p.rtol);
                    bicg_s_kernel<<<nb, kSolveThreads, 0, s>>>(n, vr, vv, vs, sc);
                    bicg_t_kernel<T><<<nb, kSolveThreads, 0, s>>>(col, val, n, ld, slots, pinned, sigma,
                                                                  vs, vt, part, sc);
                    solve_scalar_kernel<<<1, kSolveThreads, 0, s>>>(kStepOmega, part, nb, 2, sc, p.rtol);
                    bicg_xr_kernel<<<nb, kSolveThreads, 0, s>>>(n, vp, vs, vt, vrh, vx, vr, part, sc);
                    solve_scalar_kernel<<<1, kSolveThreads, 0, s>>>(kStepRho, part, nb, 2, sc, p.rtol);
                }
                if (mvgd_status st = check_launch("solver"); st != MVGD_OK)
                    return st;
                if (!read_scalars())
                    return fail(MVGD_EDEVICE, "reading the solver state failed");
                if (hs.done)
                    break;
            }
            if (hs.done != 1 || cycle == kMaxRestarts)
                break;
            residual_kernel<T><<<nb, kSolveThreads, 0, s>>>(col, val, n, ld, slots, pinned, sigma, vb,
                                                            vx, part);
            sum_partials_kernel<<<1, kSolveThreads, 0, s>>>(part, nb, &sc->dot[0]);
            if (mvgd_status st = check_launch("solver"); st != MVGD_OK)
                return st;
            if (!read_scalars())
                return fail(MVGD_EDEVICE, "reading the solver state failed");
            if (hs.dot[0] <= hs.tol2 || prior_iters + hs.iters >= p.max_iter)
                break;
            prior_iters += hs.iters;
            bicg_init_kernel<T><<<nb, kSolveThreads, 0, s>>>(col, val, n, ld, slots, pinned, sigma, vx,
                                                             vb, vr, vrh, vp, vv, part);
            solve_scalar_kernel<<<1, kSolveThreads, 0, s>>>(kStepInit, part, nb, 2, sc, p.rtol);
        }
    } else {
        // damped Jacobi, ping-pong between vx and vp
        for (int it = 0; it < p.max_iter;) {
            const int batch = std::min(check, p.max_iter - it);
            for (int j = 0; j < batch; ++j, ++it) {
                const double *xi = (it % 2 == 0) ? vx : vp;
                double *xo = (it % 2 == 0) ? vp : vx;
                jacobi_kernel<T><<<nb, kSolveThreads, 0, s>>>(col, val, n, ld, slots, pinned, sigma,
                                                              omega, vb, xi, xo, part, sc);
                solve_scalar_kernel<<<1, kSolveThreads, 0, s>>>(kStepJacobi, part, nb, 1, sc, p.rtol);
            }
            if (mvgd_status st = check_launch("solver"); st != MVGD_OK)
                return st;
            if (!read_scalars())
                return fail(MVGD_EDEVICE, "reading the solver state failed");
            if (hs.done)
                break;
        }
    }
    if (!read_scalars())
        return fail(MVGD_EDEVICE, "reading the solver state failed");
    if (p.method == MVGD_SOLVE_JACOBI)
        xcur = (hs.iters % 2 == 0) ? vx : vp; // the sweep count fixes the buffer of the last iterate
    // the returned iterate's true residual, and the iterate in the caller's order
    residual_kernel<T><<<nb, kSolveThreads, 0, s>>>(col, val, n, ld, slots, pinned, sigma, vb, xcur,
                                                    part);
    sum_partials_kernel<<<1, kSolveThreads, 0, s>>>(part, nb, &sc->dot[0]);
    solve_scatter_kernel<<<nb, kSolveThreads, 0, s>>>(L->perm, n, xcur, x, is_double);
    if (mvgd_status st = check_launch("solver"); st != MVGD_OK)
        return st;
    if (!read_scalars())
        return fail(MVGD_EDEVICE, "reading the solver state failed");
    info->iterations = prior_iters + hs.iters;
    info->converged = hs.done == 1 ? 1 : hs.done == 2 ? -1 : 0;
    info->rel_residual = hs.bb > 0.0 ? sqrt(hs.dot[0] / hs.bb) : sqrt(hs.dot[0]);
    // BiCGSTAB reports convergence only when the returned iterate's true residual passes
    if (p.method == MVGD_SOLVE_BICGSTAB && info->converged == 1 && !(hs.dot[0] <= hs.tol2))
        info->converged = 0;
    return MVGD_OK;
}

// ---------------------------------------------------------------------------------------------
// small dense helpers on the host (Rayleigh-Ritz of the eigenvalue iteration)
// ---------------------------------------------------------------------------------------------
// Eigenvalues of a real m x m matrix (row-major): Householder reduction to upper Hessenberg form,
// then the implicitly double-shifted QR iteration (Francis) with deflation at negligible
// subdiagonal entries; 1 x 1 blocks give real eigenvalues, 2 x 2 blocks a real pair or a complex
// conjugate pair. Only the active block is transformed (no Schur vectors are kept).
// Returns false if some eigenvalue did not converge within 60 iterations.
bool dense_eigvals(int m, const double *A, double *re, double *im)
{
    std::vector<double> h((size_t)m * m);
    for (int i = 0; i < m * m; ++i)
        h[i] = A[i];
    auto H = [&](int i, int j) -> double & { return h[(size_t)i * m + j]; };
    // Hessenberg reduction
    for (int k = 0; k + 2 < m; ++k) {
        double alpha = 0.0;
        for (int i = k + 1; i < m; ++i)
            alpha += H(i, k) * H(i, k);
        alpha = std::sqrt(alpha);
        if (alpha == 0.0)
            continue;
        if (H(k + 1, k) > 0.0)
            alpha = -alpha;
        std::vector<double> v(m, 0.0);
        v[k + 1] = H(k + 1, k) - alpha;
        for (int i = k + 2; i < m; ++i)
            v[i] = H(i, k);
        double vv = 0.0;
        for (int i = k + 1; i < m; ++i)
            vv += v[i] * v[i];
        if (vv == 0.0)
            continue;
        // H <- (I - 2 v v^T / vv) H (I - 2 v v^T / vv)
        for (int j = 0; j < m; ++j) {
            double d = 0.0;
            for (int i = k + 1; i < m; ++i)
                d += v[i] * H(i, j);
            d *= 2.0 / vv;
            for (int i = k + 1; i < m; ++i)
                H(i, j) -= d * v[i];
        }
        for (int i = 0; i < m; ++i) {
            double d = 0.0;
            for (int j = k + 1; j < m; ++j)
                d += H(i, j) * v[j];
            d *= 2.0 / vv;
            for (int j = k + 1; j < m; ++j)
                H(i, j) -= d * v[j];
        }
        for (int i = k + 2; i < m; ++i)
            H(i, k) = 0.0;
    }
    const double eps = std::numeric_limits<double>::epsilon();
    int hi = m - 1, iter = 0;
    while (hi >= 0) {
        // deflation point: the lowest l with negligible H(l, l - 1)
        int l = hi;
        while (l > 0) {
            const double s = std::fabs(H(l - 1, l - 1)) + std::fabs(H(l, l));
            if (std::fabs(H(l, l - 1)) <= eps * (s == 0.0 ? 1.0 : s))
                break;
            --l;
        }
        if (l == hi) { // 1 x 1 block
            re[hi] = H(hi, hi);
            im[hi] = 0.0;
            --hi;
            iter = 0;
            continue;
        }
        if (l == hi - 1) { // 2 x 2 block: eigenvalues of [[a, b], [c, d]]
            const double a = H(hi - 1, hi - 1), b = H(hi - 1, hi), c = H(hi, hi - 1), d = H(hi, hi);
            const double tr = 0.5 * (a + d), det = a * d - b * c, disc = tr * tr - det;
            if (disc >= 0.0) {
                const double r = std::sqrt(disc);
                const double e1 = tr + (tr >= 0.0 ? r : -r);
                const double e2 = e1 != 0.0 ? det / e1 : tr - (tr >= 0.0 ? r : -r);
                re[hi - 1] = e1;
                re[hi] = e2;
                im[hi - 1] = im[hi] = 0.0;
            } else {
                const double r = std::sqrt(-disc);
                re[hi - 1] = re[hi] = tr;
                im[hi - 1] = r;
                im[hi] = -r;
            }
            hi -= 2;
            iter = 0;
            continue;
        }
        if (++iter > 60)
            return false;
        // double shift from the trailing 2 x 2 block (an exceptional shift every 10th iteration)
        double s = H(hi - 1, hi - 1) + H(hi, hi);
        double t = H(hi - 1, hi - 1) * H(hi, hi) - H(hi - 1, hi) * H(hi, hi - 1);
        if (iter % 10 == 0) {
            const double w = std::fabs(H(hi, hi - 1)) + std::fabs(H(hi - 1, hi - 2));
            s = 1.5 * w;
            t = w * w;
        }
        double x = H(l, l) * H(l, l) + H(l, l + 1) * H(l + 1, l) - s * H(l, l) + t;
        double y = H(l + 1, l) * (H(l, l) + H(l + 1, l + 1) - s);
        double z = H(l + 1, l) * H(l + 2, l + 1);
        for (int k = l; k <= hi - 2; ++k) {
            // reflector P = I - 2 u u^T / (u^T u) with P (x, y, z)^T = (beta, 0, 0)^T
            double nrm = std::sqrt(x * x + y * y + z * z);
            if (nrm != 0.0) {
                const double beta = x > 0.0 ? -nrm : nrm;
                const double u0 = x - beta, u1 = y, u2 = z;
                const double uu = u0 * u0 + u1 * u1 + u2 * u2;
                const int c0 = k > l ? k - 1 : l;
                for (int j = c0; j <= hi; ++j) {
                    const double d = 2.0 * (u0 * H(k, j) + u1 * H(k + 1, j) + u2 * H(k + 2, j)) / uu;
                    H(k, j) -= d * u0;
                    H(k + 1, j) -= d * u1;
                    H(k + 2, j) -= d * u2;
                }
                const int r1 = std::min(k + 3, hi);
                for (int i = l; i <= r1; ++i) {
                    const double d = 2.0 * (H(i, k) * u0 + H(i, k + 1) * u1 + H(i, k + 2) * u2) / uu;
                    H(i, k) -= d * u0;
                    H(i, k + 1) -= d * u1;
                    H(i, k + 2) -= d * u2;
                }
                if (k > l) {
                    H(k + 1, k - 1) = 0.0;
                    H(k + 2, k - 1) = 0.0;
                }
            }
            x = H(k + 1, k);
            y = H(k + 2, k);
            if (k < hi - 2)
                z = H(k + 3, k);
        }
        // final 2-vector reflector on rows / columns hi - 1, hi
        {
            const int k = hi - 1;
            const double nrm = std::sqrt(x * x + y * y);
            if (nrm != 0.0) {
                const double beta = x > 0.0 ? -nrm : nrm;
                const double u0 = x - beta, u1 = y;
                const double uu = u0 * u0 + u1 * u1;
                for (int j = k - 1; j <= hi; ++j) {
                    const double d = 2.0 * (u0 * H(k, j) + u1 * H(k + 1, j)) / uu;
                    H(k, j) -= d * u0;
                    H(k + 1, j) -= d * u1;
                }
                for (int i = l; i <= hi; ++i) {
                    const double d = 2.0 * (H(i, k) * u0 + H(i, k + 1) * u1) / uu;
                    H(i, k) -= d * u0;
                    H(i, k + 1) -= d * u1;
                }
                H(k + 1, k - 1) = 0.0;
            }
        }
    }
    return true;
}

// Cholesky G = R^T R (R upper, row-major) of a symmetric positive definite m x m matrix and the
// inverse of R; false when a pivot is not positive.
bool chol_upper_inverse(int m, const double *G, double *Rinv)
{
    std::vector<double> R((size_t)m * m, 0.0);
    for (int i = 0; i < m; ++i) {
        for (int j = i; j < m; ++j) {
            double s = G[(size_t)i * m + j];
            for (int k = 0; k < i; ++k)
                s -= R[(size_t)k * m + i] * R[(size_t)k * m + j];
            if (j == i) {
                if (!(s > 0.0))
                    return false;
                R[(size_t)i * m + i] = std::sqrt(s);
            } else {
                R[(size_t)i * m + j] = s / R[(size_t)i * m + i];
            }
        }
    }
    // R^-1 by back substitution, column by column
    for (int i = 0; i < m * m; ++i)
        Rinv[i] = 0.0;
    for (int j = 0; j < m; ++j) {
        for (int i = j; i >= 0; --i) {
            double s = (i == j) ? 1.0 : 0.0;
            for (int k = i + 1; k <= j; ++k)
                s -= R[(size_t)i * m + k] * Rinv[(size_t)k * m + j];
            Rinv[(size_t)i * m + j] = s / R[(size_t)i * m + i];
        }
    }
    return true;
}

template <typename T>
mvgd_status eigs_impl(mvgd_matrix *L, const mvgd_eigs_params &p, double *lre, double *lim,
                      mvgd_eigs_info *info, hipStream_t s)
{
    const int64_t n = L->n_total, ld = L->ld;
    const int slots = L->K + 1;
    const T *val = (const T *)L->ell_val;
    const int32_t *col = L->ell_col;
    const int nev = p.nev;
    const int m = p.block > 0 ? p.block : std::min(kEigMaxBlock, std::max(nev + 8, 2 * nev));
    // degree: fixed, or per iteration 2 sqrt((b - a)/(a - a0)) clamped to [8, 500], which makes the
    // filter grow by about e^4 from a down to the bottom of the spectrum
    int degree = p.degree;
    const int max_iter = p.max_iter > 0 ? p.max_iter : 500;
    const double tol = p.tol > 0.0 ? p.tol : 1e-10;
    const int nblk_g = (int)std::min<int64_t>(1024, std::max<int64_t>(1, (n + 255) / 256));
    const size_t blk = (size_t)n * m;
    const int mm = m * m;
    double *V, *X, *Y, *Z, *part, *gout, *rdev;
    uint8_t *mask;
    unsigned long long *gb;
    auto carve = [&](Carver &cv) {
        for (double **v : {&V, &X, &Y, &Z})
            cv.take(*v, sizeof(double) * blk);
        cv.take(part, sizeof(double) * (size_t)nblk_g * mm);
        cv.take(gout, sizeof(double) * mm);
        cv.take(rdev, sizeof(double) * mm);
        cv.take(mask, (size_t)n);
        cv.take(gb, sizeof(unsigned long long));
    };
    Carver sz;
    carve(sz);
    void *work = nullptr;
    if (dev_alloc(&work, sz.off, s) != hipSuccess)
        return fail(MVGD_ENOMEM, "device allocation failed (eigensolver work, %zu bytes)", sz.off);
    struct Release {
        void *w;
        hipStream_t s;
        ~Release() { (void)hipFreeAsync(w, s); }
    } release_work{work, s};
    Carver cv{(char *)work, 0};
    carve(cv);
    const unsigned nb1 = (unsigned)((n + kEigThreads - 1) / kEigThreads);
    const unsigned nbr = (unsigned)((n + (kEigThreads / kWave) - 1) / (kEigThreads / kWave));
    eig_mask_kernel<<<nb1, kEigThreads, 0, s>>>(L->perm, n, p.fixed, mask);
    eig_init_kernel<<<(unsigned)((blk + kEigThreads - 1) / kEigThreads), kEigThreads, 0, s>>>(
        n, m, mask, (unsigned long long)p.seed, Y);
    (void)hipMemsetAsync(gb, 0, sizeof(unsigned long long), s);
    eig_gersh_kernel<T><<<nb1, kEigThreads, 0, s>>>(val, n, ld, slots, mask, gb);
    std::vector<double> G(mm), Rinv(mm), Hh(mm), re(m), im(m);
    unsigned long long gb_host = 0;
    // A^T B on the device, read back into `out`
    auto gram = [&](const double *A, const double *B, std::vector<double> &out) -> bool {
        eig_gram_kernel<<<nblk_g, kEigThreads, 0, s>>>(n, m, A, B, part);
        eig_reduce_kernel<<<(unsigned)((mm + kEigThreads - 1) / kEigThreads), kEigThreads, 0, s>>>(
            part, nblk_g, mm, gout);
        return hipMemcpyAsync(out.data(), gout, sizeof(double) * mm, hipMemcpyDeviceToHost, s) ==
                   hipSuccess &&
               hipStreamSynchronize(s) == hipSuccess;
    };
    // dst = src R^-1 with G = src^T src = R^T R (a diagonal shift if G is not numerically positive)
    auto cholqr = [&](const double *src, double *dst) -> mvgd_status {
        if (!gram(src, src, G))
            return fail(MVGD_EDEVICE, "eigensolver: Gram matrix read-back failed");
        double tr = 0.0;
        for (int i = 0; i < m; ++i)
            tr += G[(size_t)i * m + i];
        bool ok = chol_upper_inverse(m, G.data(), Rinv.data());
        for (int t = 0; !ok && t < 4; ++t) {
            for (int i = 0; i < m; ++i)
                G[(size_t)i * m + i] += 1e-13 * std::pow(100.0, t) * tr;
            ok = chol_upper_inverse(m, G.data(), Rinv.data());
        }
        if (!ok)
            return fail(MVGD_EDEVICE, "eigensolver: the block lost rank (Cholesky QR failed)");
        if (hipMemcpyAsync(rdev, Rinv.data(), sizeof(double) * mm, hipMemcpyHostToDevice, s) !=
            hipSuccess)
            return fail(MVGD_EDEVICE, "eigensolver: upload failed");
        eig_rmul_kernel<<<nbr, kEigThreads, 0, s>>>(n, m, src, rdev, dst);
        return check_launch("eigensolver");
    };
    // V = orthonormal basis of Y (Cholesky QR twice, through X)
    auto orth = [&]() -> mvgd_status {
        if (mvgd_status st = cholqr(Y, X); st != MVGD_OK)
            return st;
        return cholqr(X, V);
    };
    // Ritz values of V^T A V, sorted by real part (then imaginary part)
    std::vector<std::pair<double, double>> ritz(m), prev;
    auto rayleigh_ritz = [&]() -> mvgd_status {
        eig_cheb_kernel<T><<<nbr, kEigThreads, 0, s>>>(col, val, n, ld, slots, m, mask, nullptr, V, Z,
                                                       1.0, 0.0, 0.0);
        if (!gram(V, Z, Hh))
            return fail(MVGD_EDEVICE, "eigensolver: Rayleigh quotient read-back failed");
        if (!dense_eigvals(m, Hh.data(), re.data(), im.data()))
            return fail(MVGD_EDEVICE, "eigensolver: the dense eigenvalue iteration did not converge");
        for (int i = 0; i < m; ++i)
            ritz[i] = {re[i], im[i]};
        std::sort(ritz.begin(), ritz.end());
        return MVGD_OK;
    };
    if (mvgd_status st = orth(); st != MVGD_OK)
        return st;
    if (hipMemcpyAsync(&gb_host, gb, sizeof gb_host, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return fail(MVGD_EDEVICE, "eigensolver: spectrum bound read-back failed");
    // decode the ordered encoding (positive values: the top bit set)
    const double bound = gb_host ? __builtin_bit_cast(double, gb_host & 0x7fffffffffffffffull) : 0.0;
    const double b = 1.01 * bound + 1e-300;
    if (mvgd_status st = rayleigh_ritz(); st != MVGD_OK)
        return st;
    int it = 0, stable = 0;
    double change = INFINITY;
    for (; it < max_iter && stable < 2; ++it) {
        // Chebyshev filter on [a, b], scaled by its value at a0 (Zhou-Saad recurrence)
        // unwanted interval [a, b]: a is the block's largest Ritz value (a lower cut, e.g. halfway
        // into the block, took 1.6 times as many iterations at 200k points on the sphere)
        const double a0 = std::min(ritz[0].first, 0.0);
        double a = ritz[m - 1].first;
        if (!(a > a0) || !(a < b))
            a = 0.5 * (a0 + b);
        const double e = 0.5 * (b - a), c = 0.5 * (b + a);
        const double s1 = e / (a0 - c);
        if (p.degree <= 0)
            degree = (int)std::min(500.0, std::max(8.0, std::ceil(2.0 * std::sqrt((b - a) / std::max(a - a0, 1e-300 * b)))));
        double sg = s1;
        // Y = (s1 / e)(A V - c V)
        eig_cheb_kernel<T><<<nbr, kEigThreads, 0, s>>>(col, val, n, ld, slots, m, mask, nullptr, V, Y,
                                                       s1 / e, -c * s1 / e, 0.0);
        const double *xp = V;
        double *yp = Y, *zp = Z;
        for (int k = 2; k <= degree; ++k) {
            const double sn = 1.0 / (2.0 / s1 - sg);
            eig_cheb_kernel<T><<<nbr, kEigThreads, 0, s>>>(col, val, n, ld, slots, m, mask, xp, yp, zp,
                                                           2.0 * sn / e, -2.0 * sn * c / e, -sg * sn);
            // rotate: x <- y, y <- z, z <- the free buffer
            double *freebuf = (xp == V) ? X : (double *)xp;
            xp = yp;
            yp = zp;
            zp = freebuf;
            sg = sn;
        }
        if (mvgd_status st = check_launch("eigensolver"); st != MVGD_OK)
            return st;
        // the filtered block is in yp: orthonormalise into V (through the other buffers)
        if (yp != Y) {
            if (hipMemcpyAsync(Y, yp, sizeof(double) * blk, hipMemcpyDeviceToDevice, s) != hipSuccess)
                return fail(MVGD_EDEVICE, "eigensolver: copy failed");
        }
        if (mvgd_status st = orth(); st != MVGD_OK)
            return st;
        prev = ritz;
        if (mvgd_status st = rayleigh_ritz(); st != MVGD_OK)
            return st;
        change = 0.0;
        for (int i = 0; i < nev; ++i) {
            const double d = std::hypot(ritz[i].first - prev[i].first, ritz[i].second - prev[i].second);
            const double sc = std::max(1.0, std::hypot(ritz[i].first, ritz[i].second));
            change = std::max(change, d / sc);
        }
        stable = change <= tol ? stable + 1 : 0;
    }
    for (int i = 0; i < nev; ++i) {
        lre[i] = ritz[i].first;
        lim[i] = ritz[i].second;
    }
    info->iterations = it;
    info->converged = stable >= 2 ? 1 : 0;
    info->block = m;
    info->degree = degree;
    info->spectrum_bound = bound;
    info->max_change = change;
    return MVGD_OK;
}

} // namespace

extern "C" {

mvgd_status mvgd_solve(mvgd_matrix *L, const void *b, void *x, const mvgd_solve_params *p,
                       mvgd_solve_info *info, void *stream)
{
    if (!L || !b || !x || !p || !info)
        return fail(MVGD_EINVAL, "NULL argument");
    memset(info, 0, sizeof *info);
    if (p->method != MVGD_SOLVE_BICGSTAB && p->method != MVGD_SOLVE_JACOBI)
        return fail(MVGD_EINVAL, "unknown solver %d", p->method);
    if (p->max_iter < 0 || !(p->rtol >= 0.0) || !std::isfinite(p->rtol) ||
        !std::isfinite(p->sigma) || !(p->omega >= 0.0 && p->omega < 2.0) ||
        (p->pin_first != 0 && p->pin_first != 1) || p->check_every < 0)
        return fail(MVGD_EINVAL, "solver parameters out of range");
    if (!is_device_pointer(b, L->device) || !is_device_pointer(x, L->device) ||
        (p->fixed && !is_device_pointer(p->fixed, L->device)))
        return fail(MVGD_EINVAL, "b, x and fixed must be device memory of the matrix's device");
    hipStream_t s = (hipStream_t)stream;
    L->stream = s;
    if (L->precision == MVGD_FP64)
        return solve_impl<double>(L, b, x, *p, info, s);
    return solve_impl<float>(L, b, x, *p, info, s);
}

mvgd_status mvgd_timing(mvgd_matrix *L, mvgd_timing_t *t)
{
    if (!L || !t)
        return fail(MVGD_EINVAL, "NULL argument");
    if (!L->ev[0])
        return fail(MVGD_EINVAL, "the matrix was assembled without MVGD_FLAG_TIME");
    if (hipEventSynchronize(L->have_apply ? L->ev[4] : L->ev[2]) != hipSuccess)
        return fail(MVGD_EDEVICE, "event synchronisation failed");
    memset(t, 0, sizeof *t);
    if (hipEventElapsedTime(&t->bin_ms, L->ev[0], L->ev[1]) != hipSuccess ||
        hipEventElapsedTime(&t->assemble_ms, L->ev[1], L->ev[2]) != hipSuccess ||
        hipEventElapsedTime(&t->search_ms, L->ev[1], L->ev[5]) != hipSuccess ||
        hipEventElapsedTime(&t->fit_ms, L->ev[5], L->ev[2]) != hipSuccess)
        return fail(MVGD_EDEVICE, "event timing failed");
    if (L->have_apply) {
        if (hipEventElapsedTime(&t->apply_ms, L->ev[3], L->ev[4]) != hipSuccess)
            return fail(MVGD_EDEVICE, "event timing failed");
        t->have_apply = 1;
    }
    return MVGD_OK;
}

mvgd_status mvgd_eigs(mvgd_matrix *L, const mvgd_eigs_params *p, double *lambda_re,
                      double *lambda_im, mvgd_eigs_info *info, void *stream)
{
    if (!L || !p || !lambda_re || !lambda_im || !info)
        return fail(MVGD_EINVAL, "NULL argument");
    if (p->nev < 1 || p->nev > kEigMaxBlock)
        return fail(MVGD_EINVAL, "nev must be in [1, %d] (got %d)", kEigMaxBlock, p->nev);
    if (p->block != 0 && (p->block < p->nev || p->block > kEigMaxBlock))
        return fail(MVGD_EINVAL, "block must be 0 or in [nev, %d] (got %d)", kEigMaxBlock, p->block);
    if (p->degree < 0 || p->degree > 1000 || p->max_iter < 0 || !(p->tol >= 0.0))
        return fail(MVGD_EINVAL, "degree must be in [0, 1000], max_iter >= 0, tol >= 0");
    const int m = p->block > 0 ? p->block : std::min(kEigMaxBlock, std::max(p->nev + 8, 2 * p->nev));
    if (L->n_total <= m)
        return fail(MVGD_EINVAL, "%lld rows; the block of %d vectors needs more",
                    (long long)L->n_total, m);
    memset(info, 0, sizeof *info);
    if (p->fixed && !is_device_pointer(p->fixed, L->device))
        return fail(MVGD_EINVAL, "fixed must be device memory");
    hipStream_t s = (hipStream_t)stream;
    L->stream = s;
    if (L->precision == MVGD_FP64)
        return eigs_impl<double>(L, *p, lambda_re, lambda_im, info, s);
    return eigs_impl<float>(L, *p, lambda_re, lambda_im, info, s);
}

mvgd_status mvgd_dense_eigvals(int32_t m, const double *a, double *re, double *im)
{
    if (m < 1 || !a || !re || !im)
        return fail(MVGD_EINVAL, "m must be positive and the arrays non-NULL");
    if (!dense_eigvals(m, a, re, im))
        return fail(MVGD_EINVAL, "the QR iteration did not converge");
    return MVGD_OK;
}

mvgd_status mvgd_pool_trim(size_t keep_bytes)
{
    hipMemPool_t pool = nullptr;
    if (device_pool(&pool) != hipSuccess || hipMemPoolTrimTo(pool, keep_bytes) != hipSuccess) {
        (void)hipGetLastError();
        return fail(MVGD_EDEVICE, "trimming the device memory pool failed");
    }
    return MVGD_OK;
}

const char *mvgd_status_str(mvgd_status s)
{
    switch (s) {
    case MVGD_OK: return "MVGD_OK";
    case MVGD_EINVAL: return "MVGD_EINVAL";
    case MVGD_ENOMEM: return "MVGD_ENOMEM";
    case MVGD_EDEVICE: return "MVGD_EDEVICE";
    case MVGD_EUNSUPPORTED: return "MVGD_EUNSUPPORTED";
    }
    return "MVGD_UNKNOWN";
}

const char *mvgd_last_error(void)
{
    return g_err;
}

int32_t mvgd_version(void)
{
    return 100; // 0.1.0
}

} // extern "C"
