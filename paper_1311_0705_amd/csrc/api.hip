// C ABI entry points (include/hgrid.h): validation, ownership and dispatch.
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <condition_variable>
#include <mutex>
#include <vector>

#include "common.h"

namespace hg {

int build_grid(const hg_density *dn, const hg_criteria *cr, int tree, hipStream_t s, hg_grid *g);
int build_single_batched(const hg_density *dn, const hg_criteria *cr, int tree, hipStream_t s,
                         hg_grid **out);
int import_structure(int tree, const std::vector<int32_t> &fc, std::vector<uint8_t> &level,
                     std::vector<uint32_t> &coord, std::vector<uint32_t> &geom, int64_t level_begin[64],
                     int *max_level);

static thread_local int g_last_hip = 0;

int set_hip_error(hipError_t e)
{
    g_last_hip = int(e);
    return HG_E_HIP;
}

// Side a power of two; each lower corner an integer multiple of side/2.
int check_domain(const double lo[3], double side)
{
    if (!(side > 0.0) || !isfinite(side)) return HG_E_DOMAIN;
    int e = 0;
    if (frexp(side, &e) != 0.5) return HG_E_DOMAIN;
    if (e < -900 || e > 900) return HG_E_DOMAIN;
    for (int d = 0; d < 3; d++) {
        if (!isfinite(lo[d])) return HG_E_DOMAIN;
        double m = lo[d] / (0.5 * side);
        if (m != floor(m) || fabs(m) > 1e12) return HG_E_DOMAIN;
    }
    return HG_OK;
}

int dalloc(void **p, size_t bytes, hipStream_t s)
{
    static bool pool_ready = false;
    if (!pool_ready) {
        int dev = 0;
        hipMemPool_t pool;
        if (hipGetDevice(&dev) == hipSuccess && hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess) {
            uint64_t keep = UINT64_MAX;
            (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep);
        }
        pool_ready = true;
    }
    *p = nullptr;
    if (bytes == 0) bytes = 256;
    hipError_t e = hipMallocAsync(p, bytes, s);
    if (e == hipErrorOutOfMemory) return HG_E_OOM;
    if (e != hipSuccess) return set_hip_error(e);
    return HG_OK;
}

void dfree(void *p, hipStream_t s)
{
    if (p) (void)hipFreeAsync(p, s);
}

void free_grid_arrays(hg_grid *g)
{
    if (g->block) {
        block_free(g->block, g->block_bytes, g->block_dev);
        return;
    }
    void *ptrs[] = {g->first_child, g->level, g->coord, g->geom, g->S, g->rmin, g->rmax, g->rope,
                    g->leaf_of, g->int_of, g->node_of, g->rho, g->rec32, g->rec64, g->recw,
                    g->child, g->jump, g->table};
    for (void *p : ptrs) dfree(p, nullptr);
}

// Records each path batch needs: the last entry of its offsets.
__global__ void k_batch_totals(const WalkArgs *__restrict__ A, int ng, int64_t *__restrict__ out)
{
    const int i = int(blockIdx.x) * 256 + threadIdx.x;
    if (i < ng) out[i] = A[i].offsets[A[i].n];
}

__global__ void k_reset_status(TraceStatus *st)
{
    st->rechecks = 0;
    st->descents = 0;
    st->bad_dir = 0;
    st->step_guard = 0;
    st->bad_ref = 0;
    st->cap_overflow = 0;
    st->resumed = 0;
    st->next_ray = 0;
    st->done_waves = 0;
}

hg_grid *new_grid(int tree, const double lo[3], double side)
{
    hg_grid *g = (hg_grid *)calloc(1, sizeof(hg_grid));
    if (!g) return nullptr;
    g->tree = tree;
    for (int d = 0; d < 3; d++) g->lo[d] = lo[d];
    g->side = side;
    return g;
}

void destroy(hg_grid *g)
{
    if (!g) return;
    if (!g->borrowed) free_grid_arrays(g);
    free(g);
}

namespace {
bool finite_nonneg(double x) { return x >= 0.0 && !isnan(x); }
}  // namespace

int check_build_args(const hg_density *dn, const hg_criteria *cr, int tree_type)
{
    if (tree_type != HG_OCTREE && tree_type != HG_KDTREE && tree_type != HG_KDGRAD) return HG_E_INVAL;
    int rc = check_domain(dn->lo, dn->side);
    if (rc) return rc;
    const int maxlv = tree_type == HG_OCTREE ? 19 : 57;
    if (cr->max_level < 0 || cr->max_level > maxlv || cr->min_level < 0) return HG_E_INVAL;
    if (cr->n_samples <= 0 || cr->n_samples > (1 << 20)) return HG_E_INVAL;
    if (!(cr->total_mass > 0.0) || !isfinite(cr->total_mass)) return HG_E_INVAL;
    if (isnan(cr->delta_max) || isnan(cr->tau_max) || isnan(cr->q_max)) return HG_E_INVAL;
    if (!finite_nonneg(cr->kappa) || !isfinite(cr->kappa)) return HG_E_INVAL;
    if (dn->n_clumps < 0 || dn->n_clumps > HG_MAX_CLUMPS) return HG_E_INVAL;
    if (dn->n_clumps > 0) {
        if (!dn->clump_c || !dn->clump_sigma || !dn->clump_amp) return HG_E_INVAL;
        if (!(dn->clump_trunc > 0.0) || !isfinite(dn->clump_trunc)) return HG_E_INVAL;
        for (int64_t i = 0; i < dn->n_clumps; i++)
            if (!(dn->clump_sigma[i] > 0.0) || !isfinite(dn->clump_sigma[i])) return HG_E_INVAL;
    }
    if (dn->has_disk && (!(dn->disk_hR > 0.0) || !(dn->disk_hz > 0.0))) return HG_E_INVAL;
    return HG_OK;
}

// Scratch of the one-walk records mode (rows of records, scan temporaries,
// resume entries): one buffer per device, allocated outside the stream-
// ordered pool so that repeated calls neither allocate nor split the pool's
// blocks.  It grows when a call needs more and is kept for later calls; a
// call holds it, under the lock, until its stream has drained.
struct Scratch {
    std::mutex m;
    void *p = nullptr;
    size_t bytes = 0;
};
constexpr int MAX_DEVICES = 64;
static Scratch g_scratch[MAX_DEVICES];

static size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

int scratch_acquire(size_t bytes, Scratch **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e) return set_hip_error(e);
    if (dev < 0 || dev >= MAX_DEVICES) return HG_E_INVAL;
    Scratch &w = g_scratch[dev];
    w.m.lock();
    if (w.bytes < bytes) {
        if (w.p) (void)hipFree(w.p);   // synchronises the device: no call still uses it
        w.p = nullptr;
        w.bytes = 0;
        const size_t grain = size_t(1) << 28;
        const size_t want = (bytes + grain - 1) / grain * grain;
        e = hipMalloc(&w.p, want);
        if (e) {
            (void)hipGetLastError();
            w.p = nullptr;
            w.m.unlock();
            return e == hipErrorOutOfMemory ? HG_E_OOM : set_hip_error(e);
        }
        w.bytes = want;
    }
    *out = &w;
    return HG_OK;
}

void *scratch_ptr(Scratch *w) { return w->p; }

void scratch_release(Scratch *w) { w->m.unlock(); }

int64_t slab_rows(const hg_trace_opts *opts, int64_t n)
{
    const double per = double(4 + (opts->precision == HG_FP64 ? 8 : 4));
    if (n <= 0) return 0;
    if (opts->slab > 0) {
        const int64_t k = (int64_t(opts->slab) + 3) / 4 * 4;
        return double(n) * (double(k) * per + double(sizeof(Resume))) <= SLAB_BUDGET ? k : 0;
    }
    const double fit = (SLAB_BUDGET / double(n) - double(sizeof(Resume))) / per;
    if (fit < double(SLAB_MIN)) return 0;
    return std::min<int64_t>(SLAB_MAX, int64_t(fit) / 4 * 4);
}

// The block cache of block_alloc / block_free.
struct BlockCache {
    std::mutex m;
    std::vector<std::pair<void *, size_t>> blocks;
    size_t bytes = 0;
};
static BlockCache g_blocks[MAX_DEVICES];
constexpr size_t BLOCK_CACHE_COUNT = 4;
constexpr size_t BLOCK_CACHE_BYTES = size_t(16) << 30;

int block_alloc(void **p, size_t bytes, int *dev)
{
    *p = nullptr;
    hipError_t e = hipGetDevice(dev);
    if (e) return set_hip_error(e);
    if (*dev < 0 || *dev >= MAX_DEVICES) return HG_E_INVAL;
    {
        // the smallest cached block that holds bytes without wasting half of it
        BlockCache &c = g_blocks[*dev];
        std::lock_guard<std::mutex> lock(c.m);
        size_t best = c.blocks.size();
        for (size_t i = 0; i < c.blocks.size(); i++) {
            const size_t b = c.blocks[i].second;
            if (b >= bytes && b / 2 <= bytes && (best == c.blocks.size() || b < c.blocks[best].second))
                best = i;
        }
        if (best < c.blocks.size()) {
            *p = c.blocks[best].first;
            c.bytes -= c.blocks[best].second;
            c.blocks.erase(c.blocks.begin() + long(best));
            return HG_OK;
        }
    }
    return dalloc(p, bytes, nullptr);
}

void block_free(void *p, size_t bytes, int dev)
{
    if (!p) return;
    if (dev >= 0 && dev < MAX_DEVICES) {
        BlockCache &c = g_blocks[dev];
        std::lock_guard<std::mutex> lock(c.m);
        if (c.blocks.size() < BLOCK_CACHE_COUNT && c.bytes + bytes <= BLOCK_CACHE_BYTES) {
            c.blocks.emplace_back(p, bytes);
            c.bytes += bytes;
            return;
        }
    }
    dfree(p, nullptr);
}

// Pool of trace status slots per device: blocks of SLOTS_PER_BLOCK slots,
// allocated once and kept until the process ends (a slot is in use only for
// the duration of one call).
struct StatusPool {
    std::mutex m;
    std::vector<TraceStatus *> free_slots;
};
static StatusPool g_status_pool[MAX_DEVICES];
constexpr int SLOTS_PER_BLOCK = 64;
constexpr size_t SLOT_BYTES = 256;
static_assert(sizeof(TraceStatus) <= SLOT_BYTES, "status slot");

int StatusSlot::acquire()
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e) return set_hip_error(e);
    if (dev < 0 || dev >= MAX_DEVICES) return HG_E_INVAL;
    StatusPool &P = g_status_pool[dev];
    std::lock_guard<std::mutex> lock(P.m);
    if (P.free_slots.empty()) {
        void *b = nullptr;
        e = hipMalloc(&b, SLOT_BYTES * SLOTS_PER_BLOCK);
        if (e) {
            (void)hipGetLastError();
            return e == hipErrorOutOfMemory ? HG_E_OOM : set_hip_error(e);
        }
        for (int i = SLOTS_PER_BLOCK - 1; i >= 0; i--)
            P.free_slots.push_back(reinterpret_cast<TraceStatus *>(static_cast<char *>(b) + SLOT_BYTES * size_t(i)));
    }
    p_ = P.free_slots.back();
    P.free_slots.pop_back();
    dev_ = dev;
    return HG_OK;
}

StatusSlot::~StatusSlot()
{
    if (!p_) return;
    StatusPool &P = g_status_pool[dev_];
    std::lock_guard<std::mutex> lock(P.m);
    P.free_slots.push_back(p_);
}

}  // namespace hg

using namespace hg;

extern "C" {

const char *grid_strerror(int code)
{
    switch (code) {
    case HG_OK: return "success";
    case HG_E_INVAL: return "invalid argument";
    case HG_E_DOMAIN: return "domain must be a cube of power-of-two side with corners on half-side multiples";
    case HG_E_DIR: return "direction not a finite unit vector";
    case HG_E_CAPACITY: return "record capacity too small (see needed)";
    case HG_E_OOM: return "device allocation failed";
    case HG_E_LIMIT: return "tree exceeds the library's node limits";
    case HG_E_HIP: return "HIP runtime error";
    case HG_E_STEP: return "path step guard exceeded";
    case HG_E_FORMAT: return "arrays are not a valid breadth-first tree";
    default: return "unknown status";
    }
}

int grid_last_hip_error(void) { return g_last_hip; }

int grid_build(const hg_density *dn, const hg_criteria *cr, int tree_type, void *stream,
               hg_grid_t *out)
{
    if (!dn || !cr || !out) return HG_E_INVAL;
    *out = nullptr;
    int rc = check_build_args(dn, cr, tree_type);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    if (cr->max_nodes > 0 && cr->max_nodes <= MAX_IDS && tree_type != HG_KDGRAD) {
        // a known capacity: the construction without per-level synchronisation
        hg_grid *gb = nullptr;
        rc = build_single_batched(dn, cr, tree_type, s, &gb);
        if (rc) return rc;
        *out = gb;
        return HG_OK;
    }
    hg_grid *g = new_grid(tree_type, dn->lo, dn->side);
    if (!g) return HG_E_OOM;
    rc = build_grid(dn, cr, tree_type, s, g);
    if (rc) {
        (void)hipStreamSynchronize(s);
        destroy(g);
        return rc;
    }
    *out = g;
    return HG_OK;
}

int grid_import(const hg_grid_arrays *a, void *stream, hg_grid_t *out)
{
    if (!a || !out) return HG_E_INVAL;
    *out = nullptr;
    if (a->tree_type != HG_OCTREE && a->tree_type != HG_KDTREE && a->tree_type != HG_KDGRAD) return HG_E_INVAL;
    if (a->n_nodes < 1 || a->n_nodes >= (int64_t(1) << 31) || !a->first_child || !a->rho)
        return HG_E_INVAL;
    if (a->tree_type == HG_KDGRAD && !a->geom) return HG_E_INVAL;
    int rc = check_domain(a->lo, a->side);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    const int64_t n = a->n_nodes;
    std::vector<int32_t> fc((size_t)n);
    std::vector<uint32_t> geom((size_t)n, 0u);
    HG_CHECK(hipMemcpyAsync(fc.data(), a->first_child, size_t(n) * 4, hipMemcpyDeviceToHost, s));
    if (a->tree_type == HG_KDGRAD)
        HG_CHECK(hipMemcpyAsync(geom.data(), a->geom, size_t(n) * 4, hipMemcpyDeviceToHost, s));
    HG_CHECK(hipStreamSynchronize(s));
    std::vector<uint8_t> level;
    std::vector<uint32_t> coord;
    hg_grid *g = new_grid(a->tree_type, a->lo, a->side);
    if (!g) return HG_E_OOM;
    rc = import_structure(a->tree_type, fc, level, coord, geom, g->level_begin, &g->max_level);
    int64_t nl = 0;
    for (int32_t f : fc) nl += f < 0;
    if (!rc && nl != a->n_leaves) rc = HG_E_FORMAT;
    if (rc) {
        destroy(g);
        return rc;
    }
    g->n_nodes = n;
    const size_t N = size_t(n);
    if (dalloc_n(&g->first_child, N, s) || dalloc_n(&g->level, N, s) ||
        dalloc_n(&g->coord, N * 3, s) || dalloc_n(&g->geom, N, s) || dalloc_n(&g->S, N, s) ||
        dalloc_n(&g->rmin, N, s) ||
        dalloc_n(&g->rmax, N, s) || dalloc_n(&g->rope, N * 6, s)) {
        (void)hipStreamSynchronize(s);
        destroy(g);
        return HG_E_OOM;
    }
    hipError_t e = hipSuccess;
    if (!e) e = hipMemcpyAsync(g->first_child, fc.data(), N * 4, hipMemcpyHostToDevice, s);
    if (!e) e = hipMemcpyAsync(g->level, level.data(), N, hipMemcpyHostToDevice, s);
    if (!e) e = hipMemcpyAsync(g->coord, coord.data(), N * 12, hipMemcpyHostToDevice, s);
    if (!e) e = hipMemcpyAsync(g->geom, geom.data(), N * 4, hipMemcpyHostToDevice, s);
    if (!e) e = hipMemsetAsync(g->S, 0, N * 8, s);
    if (!e) e = hipMemsetAsync(g->rmin, 0, N * 8, s);
    if (!e) e = hipMemsetAsync(g->rmax, 0, N * 8, s);
    if (e) {
        destroy(g);
        return set_hip_error(e);
    }
    rc = finalize_layout(g, a->rho, 1, s);
    if (!rc) {
        e = hipStreamSynchronize(s);
        if (e) rc = set_hip_error(e);
    }
    if (rc) {
        (void)hipStreamSynchronize(s);
        destroy(g);
        return rc;
    }
    *out = g;
    return HG_OK;
}

int grid_export(hg_grid_t g, hg_grid_arrays *out)
{
    if (!g || !out) return HG_E_INVAL;
    memset(out, 0, sizeof *out);
    out->tree_type = g->tree;
    out->max_level = g->max_level;
    for (int d = 0; d < 3; d++) out->lo[d] = g->lo[d];
    out->side = g->side;
    out->n_nodes = g->n_nodes;
    out->n_leaves = g->n_leaves;
    out->first_child = g->first_child;
    out->rho = g->rho;
    out->level = g->level;
    out->coord = g->coord;
    out->S = g->S;
    out->rho_min = g->rmin;
    out->rho_max = g->rmax;
    out->leaf_of = g->leaf_of;
    out->node_of = g->node_of;
    out->rope = g->rope;
    out->geom = g->geom;
    return HG_OK;
}

void grid_free(hg_grid_t g) { destroy(g); }

int grid_locate(hg_grid_t g, const double *points, int64_t n, int32_t *leaf_out, void *stream)
{
    if (!g || n < 0) return HG_E_INVAL;
    if (n == 0) return HG_OK;
    if (!points || !leaf_out) return HG_E_INVAL;
    return launch_locate(g, points, n, leaf_out, (hipStream_t)stream);
}

static int check_trace_args(hg_grid_t g, const double *origins, const double *dirs, int64_t n,
                            const hg_trace_opts *opts, const hg_trace_out *out)
{
    if (!g || !opts || !out || n < 0) return HG_E_INVAL;
    if (opts->precision != HG_FP64 && opts->precision != HG_FP32_RECHECK) return HG_E_INVAL;
    if (opts->mode != HG_TAU_ONLY && opts->mode != HG_RECORDS) return HG_E_INVAL;
    if (!isfinite(opts->kappa)) return HG_E_INVAL;
    if (opts->block != 0 && opts->block != 128 && opts->block != 256 && opts->block != 512)
        return HG_E_INVAL;
    if (opts->lds_bytes > 65536 || opts->chunk < 0 || opts->chunk > HG_MAX_CHUNK || opts->refill_min < 0)
        return HG_E_INVAL;
    if (opts->passes < 0 || opts->passes > 2 || opts->slab < 0 || opts->slab > (1 << 20)) return HG_E_INVAL;
    const bool records = opts->mode == HG_RECORDS;
    if (n > 0 && (!origins || !dirs || !out->tau || !out->count)) return HG_E_INVAL;
    if (records && !out->offsets) return HG_E_INVAL;
    if (records && out->capacity > 0 && (!out->leaf || !out->ds)) return HG_E_INVAL;
    if (records && out->capacity < 0) return HG_E_INVAL;
    if (records && ((uintptr_t(out->leaf) | uintptr_t(out->ds)) & 15u)) return HG_E_INVAL;
    return HG_OK;
}

}  // extern "C"

int hg::read_status(const TraceStatus *dev_st, TraceStatus *st, hipStream_t s)
{
    hipError_t e = hipMemcpyAsync(st, dev_st, sizeof *st, hipMemcpyDeviceToHost, s);
    if (!e) e = hipStreamSynchronize(s);
    if (e) return set_hip_error(e);
    if (st->bad_ref) return HG_E_FORMAT;
    if (st->bad_dir) return HG_E_DIR;
    if (st->step_guard) return HG_E_STEP;
    return HG_OK;
}

extern "C" {

int grid_trace_batched(int ng, const hg_grid_t *grids, const double *const *origins,
                       const double *const *dirs, const int64_t *n, const hg_trace_opts *opts,
                       hg_trace_out *outs, void *stream)
{
    if (ng < 1 || !grids || !origins || !dirs || !n || !opts || !outs) return HG_E_INVAL;
    bool any_wide = false;
    for (int i = 0; i < ng; i++) {
        int rc = check_trace_args(grids[i], origins[i], dirs[i], n[i], opts, &outs[i]);
        if (rc) return rc;
        any_wide = any_wide || grids[i]->wide;
    }
    if (any_wide) {
        int first = HG_OK;
        for (int i = 0; i < ng; i++) {
            int rc = grid_trace(grids[i], origins[i], dirs[i], n[i], opts, &outs[i], stream);
            if (rc && !first) first = rc;
        }
        return first;
    }
    hipStream_t s = (hipStream_t)stream;
    const bool records = opts->mode == HG_RECORDS;
    const bool timing = (opts->flags & HG_FLAG_TIMING) != 0;
    const int64_t chunk = opts->chunk > 0 ? opts->chunk : 1024;
    StatusSlot slot;
    {
        const int rc0 = slot.acquire();
        if (rc0) return rc0;
    }
    TraceStatus *const dst = slot.get();
    std::vector<WalkGrid> hG((size_t)ng);
    std::vector<WalkArgs> hA((size_t)ng);
    std::vector<BatchChunk> hC;
    for (int i = 0; i < ng; i++) {
        hG[size_t(i)] = walk_grid(grids[i], opts->precision);
        hA[size_t(i)] = walk_args(grids[i], dst, origins[i], dirs[i], n[i], opts, &outs[i]);
        const int32_t head = int32_t(hC.size());
        for (int64_t a = 0; a < n[i]; a += chunk) hC.push_back(BatchChunk{i, head, a, std::min(n[i], a + chunk)});
        outs[i].needed = 0;
        outs[i].rechecks = 0;
        outs[i].descents = 0;
        for (int t = 0; t < 4; t++) outs[i].kernel_ms[t] = 0.f;
    }
    if (hC.size() > size_t(0x7fffffff)) return HG_E_LIMIT;
    const std::vector<int64_t> hP = chunk_prefix(hC, ng);
    std::vector<int32_t> hcg, hcp;
    {
        std::vector<int> tr((size_t)ng), dm((size_t)ng);
        std::vector<double> sd((size_t)ng);
        for (int i = 0; i < ng; i++) {
            tr[size_t(i)] = hG[size_t(i)].tree;
            dm[size_t(i)] = hG[size_t(i)].dm;
            sd[size_t(i)] = hG[size_t(i)].side;
        }
        grid_classes(tr, dm, sd, hcg, hcp);
    }
    int32_t *dcg = nullptr, *dcp = nullptr;
    WalkGrid *dG = nullptr;
    WalkArgs *dA = nullptr;
    BatchChunk *dC = nullptr;
    int64_t *tmp = nullptr, *dP = nullptr;
    unsigned long long *dctr = nullptr;
    int rc = dalloc_n(&dG, size_t(ng), s);
    if (!rc) rc = dalloc_n(&dA, size_t(ng), s);
    if (!rc) rc = dalloc_n(&dC, std::max<size_t>(hC.size(), 1), s);
    if (!rc) rc = dalloc_n(&dP, hP.size(), s);
    if (!rc) rc = dalloc_n(&dctr, size_t(ng), s);
    if (!rc) rc = dalloc_n(&dcg, hcg.size(), s);
    if (!rc) rc = dalloc_n(&dcp, hcp.size(), s);
    // records: the chunk scan's work space, then one total per grid
    const size_t ctmp = scan_chunks_tmp_elems(int(hC.size()));
    if (!rc && records) rc = dalloc_n(&tmp, ctmp + size_t(ng), s);
    hipEvent_t ev[4] = {};
    if (!rc && timing)
        for (int t = 0; t < 4; t++)
            if (hipEventCreate(&ev[t]) != hipSuccess) rc = HG_E_HIP;
    hipError_t e = hipSuccess;
    if (!rc) e = hipMemcpyAsync(dG, hG.data(), sizeof(WalkGrid) * size_t(ng), hipMemcpyHostToDevice, s);
    if (!rc && !e) e = hipMemcpyAsync(dA, hA.data(), sizeof(WalkArgs) * size_t(ng), hipMemcpyHostToDevice, s);
    if (!rc && !e && !hC.empty())
        e = hipMemcpyAsync(dC, hC.data(), sizeof(BatchChunk) * hC.size(), hipMemcpyHostToDevice, s);
    if (!rc && !e) e = hipMemcpyAsync(dP, hP.data(), sizeof(int64_t) * hP.size(), hipMemcpyHostToDevice, s);
    if (!rc && !e) e = hipMemcpyAsync(dcg, hcg.data(), sizeof(int32_t) * hcg.size(), hipMemcpyHostToDevice, s);
    if (!rc && !e) e = hipMemcpyAsync(dcp, hcp.data(), sizeof(int32_t) * hcp.size(), hipMemcpyHostToDevice, s);
    if (!rc && e) rc = set_hip_error(e);
    const BatchQueue Q{dC, dP, dctr, ng, dcg, dcp, int(hcp.size()) - 1};
    TraceStatus st;
    if (!rc) {
        k_reset_status<<<1, 1, 0, s>>>(dst);
        if (timing) (void)hipEventRecord(ev[0], s);
        rc = launch_batched(dG, dA, Q, opts, WM_COUNT, dst, s);
        if (timing) (void)hipEventRecord(ev[1], s);
    }
    if (!rc) rc = read_status(dst, &st, s);
    if (!rc) {
        outs[0].rechecks = int64_t(st.rechecks);
        outs[0].descents = int64_t(st.descents);
    }
    if (!rc && records) {
        // every grid's offsets in one chunk scan, the totals in one copy
        rc = scan_chunks(dC, int(hC.size()), dA, ng, tmp, s);
        int64_t *dtot = tmp + ctmp;
        if (!rc) {
            k_batch_totals<<<unsigned((ng + 255) / 256), 256, 0, s>>>(dA, ng, dtot);
            e = hipGetLastError();
            if (e) rc = set_hip_error(e);
        }
        std::vector<int64_t> tot((size_t)ng, 0);
        if (!rc) {
            e = hipMemcpyAsync(tot.data(), dtot, sizeof(int64_t) * size_t(ng), hipMemcpyDeviceToHost, s);
            if (e) rc = set_hip_error(e);
        }
        if (!rc) {
            e = hipStreamSynchronize(s);
            if (e) rc = set_hip_error(e);
        }
        bool fits = true;
        for (int i = 0; i < ng && !rc; i++) {
            outs[i].needed = tot[size_t(i)];
            if (tot[size_t(i)] > outs[i].capacity) fits = false;
        }
        if (!rc && !fits) rc = HG_E_CAPACITY;
        if (!rc) {
            if (timing) (void)hipEventRecord(ev[2], s);
            rc = launch_batched(dG, dA, Q, opts, WM_FILL, dst, s);
            if (timing) (void)hipEventRecord(ev[3], s);
        }
        if (!rc) rc = read_status(dst, &st, s);
    }
    if (!rc) {
        e = hipStreamSynchronize(s);
        if (e) rc = set_hip_error(e);
    }
    if (timing && (rc == HG_OK || rc == HG_E_CAPACITY)) {
        (void)hipEventElapsedTime(&outs[0].kernel_ms[0], ev[0], ev[1]);
        if (records && rc == HG_OK) {
            (void)hipEventElapsedTime(&outs[0].kernel_ms[1], ev[1], ev[2]);
            (void)hipEventElapsedTime(&outs[0].kernel_ms[2], ev[2], ev[3]);
            (void)hipEventElapsedTime(&outs[0].kernel_ms[3], ev[0], ev[3]);
        } else {
            outs[0].kernel_ms[3] = outs[0].kernel_ms[0];
        }
    }
    for (int t = 0; t < 4; t++)
        if (ev[t]) (void)hipEventDestroy(ev[t]);
    (void)hipStreamSynchronize(s);
    dfree(dG, s);
    dfree(dA, s);
    dfree(dC, s);
    dfree(dP, s);
    dfree(dctr, s);
    dfree(dcg, s);
    dfree(dcp, s);
    dfree(tmp, s);
    return rc;
}

// Records mode in two walks: a counting walk, the prefix sum of the counts and
// a record-filling walk.  The prefix sum's work space is `tmp`
// (scan_tmp_elems(n) entries) when given, else allocated here.
static int trace_two_pass(hg_grid_t g, TraceStatus *dst, const double *origins, const double *dirs, int64_t n,
                          const hg_trace_opts *opts, hg_trace_out *out, hipStream_t s, hipEvent_t *ev,
                          int64_t *tmp_given = nullptr)
{
    const bool records = opts->mode == HG_RECORDS;
    const bool timing = ev[0] != nullptr;
    k_reset_status<<<1, 1, 0, s>>>(dst);
    if (timing) (void)hipEventRecord(ev[0], s);
    int rc = launch_walk(g, dst, origins, dirs, n, opts, out, WM_COUNT, s, nullptr);
    if (timing) (void)hipEventRecord(ev[1], s);
    TraceStatus st;
    if (!rc) rc = read_status(dst, &st, s);
    if (!rc) {
        out->rechecks = int64_t(st.rechecks);
        out->descents = int64_t(st.descents);
    }
    if (rc || !records) return rc;
    int64_t *tmp = tmp_given;
    if (!tmp) rc = dalloc_n(&tmp, scan_tmp_elems(n), s);
    if (!rc) rc = scan_i32_to_i64(out->count, out->offsets, n, tmp, s);
    if (timing) (void)hipEventRecord(ev[2], s);
    int64_t needed = 0;
    if (!rc) {
        hipError_t e = hipMemcpyAsync(&needed, out->offsets + n, 8, hipMemcpyDeviceToHost, s);
        if (!e) e = hipStreamSynchronize(s);
        if (e) rc = set_hip_error(e);
    }
    if (!rc) {
        out->needed = needed;
        if (needed > out->capacity) rc = HG_E_CAPACITY;
    }
    if (!rc && needed > 0) rc = launch_walk(g, dst, origins, dirs, n, opts, out, WM_FILL, s, nullptr);
    if (timing) (void)hipEventRecord(ev[3], s);
    if (!tmp_given) dfree(tmp, s);
    if (!rc) rc = read_status(dst, &st, s);
    return rc;
}


// Records mode in one walk: tau, counts and each path's first `slab` records
// into a row per path, the prefix sum of the counts, the rows copied into the
// CSR slices, and a record-filling walk that resumes the paths whose records
// did not fit their row at their first record beyond it.  HG_E_OOM (nothing enqueued) when the scratch cannot be had.
static int trace_one_pass(hg_grid_t g, TraceStatus *dst, const double *origins, const double *dirs, int64_t n,
                          int64_t slab, const hg_trace_opts *opts, hg_trace_out *out, hipStream_t s,
                          hipEvent_t *ev)
{
    const bool timing = ev[0] != nullptr;
    const size_t dsz = opts->precision == HG_FP64 ? 8 : 4;
    const size_t b_leaf = align256(size_t(n) * size_t(slab) * 4);
    const size_t b_ds = align256(size_t(n) * size_t(slab) * dsz);
    const size_t b_tmp = align256(scan_tmp_elems(n) * 8);
    const size_t b_res = align256(size_t(n) * sizeof(Resume));
    Scratch *w = nullptr;
    int rc = scratch_acquire(b_leaf + b_ds + b_tmp + b_res + 256, &w);
    if (rc) return rc;
    char *base = static_cast<char *>(scratch_ptr(w));
    int32_t *sleaf = reinterpret_cast<int32_t *>(base);
    void *sds = base + b_leaf;
    int64_t *tmp = reinterpret_cast<int64_t *>(base + b_leaf + b_ds);
    Resume *res = reinterpret_cast<Resume *>(base + b_leaf + b_ds + b_tmp);
    // FP32 records of the persistent slab walk go to rows of (leaf, ds) pairs
    // (the leaf and ds areas together); other walks write the two areas
    const int pmode = opts->persistent < 0 ? 3 : opts->persistent;
    const int pairs = (pmode & 1) && opts->precision != HG_FP64 ? 1 : 0;
    unsigned long long *n_res = reinterpret_cast<unsigned long long *>(base + b_leaf + b_ds + b_tmp + b_res);
    TraceStatus st;
    struct {
        int64_t needed;
        unsigned long long n_res;
    } h = {0, 0};
    if (!rc) {
        k_reset_status<<<1, 1, 0, s>>>(dst);
        hipError_t e = hipMemsetAsync(n_res, 0, sizeof *n_res, s);
        if (e) rc = set_hip_error(e);
    }
    if (!rc) {
        WalkArgs A = walk_args(g, dst, origins, dirs, n, opts, out);
        A.leaf = sleaf;
        A.ds = sds;
        A.slab = slab;
        A.capacity = n * slab;
        A.resume = res;
        A.n_resume = n_res;
        A.pairs = pairs;
        if (timing) (void)hipEventRecord(ev[0], s);
        rc = launch_walk_args(g, A, opts, WM_SLAB, s);
        if (timing) (void)hipEventRecord(ev[1], s);
    }
    if (!rc) rc = scan_i32_to_i64(out->count, out->offsets, n, tmp, s);
    if (timing) (void)hipEventRecord(ev[2], s);
    if (!rc) {
        hipError_t e = hipMemcpyAsync(&h.needed, out->offsets + n, 8, hipMemcpyDeviceToHost, s);
        if (!e) e = hipMemcpyAsync(&h.n_res, n_res, sizeof h.n_res, hipMemcpyDeviceToHost, s);
        if (e) rc = set_hip_error(e);
    }
    if (!rc) rc = read_status(dst, &st, s);   // synchronises
    if (!rc) {
        out->rechecks = int64_t(st.rechecks);
        out->descents = int64_t(st.descents);
        out->needed = h.needed;
        if (h.needed > out->capacity) rc = HG_E_CAPACITY;
    }
    if (!rc) rc = launch_slab_compact(sleaf, sds, slab, opts->precision, pairs, out->count, out->offsets, n,
                                      out->leaf, out->ds, s);
    if (!rc && h.n_res > 0) {
        // the paths past their row, resumed where their row filled up
        WalkArgs F = walk_args(g, dst, origins, dirs, n, opts, out);
        F.resume = res;
        F.n = int64_t(std::min<unsigned long long>(h.n_res, (unsigned long long)n));
        F.slab = slab;
        rc = launch_walk_args(g, F, opts, WM_FILL, s);
    }
    if (timing) (void)hipEventRecord(ev[3], s);
    if (!rc) rc = read_status(dst, &st, s);
    (void)hipStreamSynchronize(s);
    scratch_release(w);
    return rc;
}

int grid_release_scratch(void)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e) return set_hip_error(e);
    if (dev < 0 || dev >= MAX_DEVICES) return HG_E_INVAL;
    {
        BlockCache &c = g_blocks[dev];
        std::lock_guard<std::mutex> lock(c.m);
        for (auto &b : c.blocks) dfree(b.first, nullptr);
        c.blocks.clear();
        c.bytes = 0;
    }
    Scratch &w = g_scratch[dev];
    std::lock_guard<std::mutex> lock(w.m);
    if (w.p) {
        e = hipFree(w.p);
        w.p = nullptr;
        w.bytes = 0;
        if (e) return set_hip_error(e);
    }
    return HG_OK;
}

int grid_trace(hg_grid_t g, const double *origins, const double *dirs, int64_t n,
               const hg_trace_opts *opts, hg_trace_out *out, void *stream)
{
    {
        int rc0 = check_trace_args(g, origins, dirs, n, opts, out);
        if (rc0) return rc0;
    }
    const bool records = opts->mode == HG_RECORDS;
    hipStream_t s = (hipStream_t)stream;
    const bool timing = (opts->flags & HG_FLAG_TIMING) != 0;
    hipEvent_t ev[4] = {};
    for (int i = 0; i < 4; i++) out->kernel_ms[i] = 0.f;
    out->needed = 0;
    out->rechecks = 0;
    out->descents = 0;
    if (timing)
        for (int i = 0; i < 4; i++) HG_CHECK(hipEventCreate(&ev[i]));
    StatusSlot slot;
    int rc = slot.acquire();
    const int64_t slab = slab_rows(opts, n);
    const bool one_pass = records && opts->passes != 2 && slab > 0;
    if (!rc) rc = one_pass ? trace_one_pass(g, slot.get(), origins, dirs, n, slab, opts, out, s, ev) : HG_E_OOM;
    if (rc == HG_E_OOM) rc = trace_two_pass(g, slot.get(), origins, dirs, n, opts, out, s, ev);
    if (timing && (rc == HG_OK || rc == HG_E_CAPACITY)) {
        (void)hipEventSynchronize(ev[1]);
        (void)hipEventElapsedTime(&out->kernel_ms[0], ev[0], ev[1]);
        if (records) {
            (void)hipEventSynchronize(ev[2]);
            (void)hipEventElapsedTime(&out->kernel_ms[1], ev[1], ev[2]);
            if (rc == HG_OK) {
                (void)hipEventSynchronize(ev[3]);
                (void)hipEventElapsedTime(&out->kernel_ms[2], ev[2], ev[3]);
                (void)hipEventElapsedTime(&out->kernel_ms[3], ev[0], ev[3]);
            } else {
                (void)hipEventElapsedTime(&out->kernel_ms[3], ev[0], ev[2]);
            }
        } else {
            out->kernel_ms[3] = out->kernel_ms[0];
        }
    }
    if (timing)
        for (int i = 0; i < 4; i++)
            if (ev[i]) (void)hipEventDestroy(ev[i]);
    return rc;
}

// The early-exit walks: one persistent walk, no records; dst_d / dst_i
// take the per-path double and int32 results.
static int trace_early_exit(hg_grid_t g, const double *origins, const double *dirs, const double *lim,
                            int64_t n, const hg_trace_opts *opts, double *dst_d, int32_t *dst_i, int wm,
                            void *stream)
{
    if (!g || !opts || n < 0) return HG_E_INVAL;
    if (opts->precision != HG_FP64 && opts->precision != HG_FP32_RECHECK) return HG_E_INVAL;
    if (!isfinite(opts->kappa)) return HG_E_INVAL;
    if (opts->block != 0 && opts->block != 128 && opts->block != 256 && opts->block != 512)
        return HG_E_INVAL;
    if (opts->chunk < 0 || opts->chunk > HG_MAX_CHUNK || opts->refill_min < 0) return HG_E_INVAL;
    if (n == 0) return HG_OK;
    if (!origins || !dirs || !lim || !dst_d || !dst_i) return HG_E_INVAL;
    hipStream_t s = (hipStream_t)stream;
    StatusSlot slot;
    int rc = slot.acquire();
    if (rc) return rc;
    TraceStatus *const st = slot.get();
    HG_CHECK(hipMemsetAsync(st, 0, sizeof(TraceStatus), s));
    hg_trace_out out;
    memset(&out, 0, sizeof out);
    out.tau = dst_d;
    out.count = dst_i;
    WalkArgs A = walk_args(g, st, origins, dirs, n, opts, &out);
    A.lim = lim;
    rc = launch_walk_args(g, A, opts, wm, s);
    if (rc) return rc;
    TraceStatus h;
    return read_status(st, &h, s);
}

int grid_trace_segment(hg_grid_t g, const double *origins, const double *dirs, const double *s_max,
                       int64_t n, const hg_trace_opts *opts, double *tau_out, int32_t *count_out,
                       void *stream)
{
    return trace_early_exit(g, origins, dirs, s_max, n, opts, tau_out, count_out, WM_SEG, stream);
}

int grid_trace_interact(hg_grid_t g, const double *origins, const double *dirs, const double *tau_star,
                        int64_t n, const hg_trace_opts *opts, int32_t *leaf_out, double *s_out,
                        void *stream)
{
    return trace_early_exit(g, origins, dirs, tau_star, n, opts, s_out, leaf_out, WM_INT, stream);
}

// grid_trace_noalloc: the scan work space lives in a fixed device array,
// one per GPU the library runs on (held until the process ends); its device
// address is looked up once per device, with that device current.
constexpr size_t NOALLOC_SCRATCH_BYTES = size_t(HG_NOALLOC_SCRATCH_BYTES);
constexpr size_t NOALLOC_STATUS_WORDS = 256 / sizeof(int64_t);   // status words ahead of the scan space
static_assert(NOALLOC_SCRATCH_BYTES % 256 == 0, "scratch size");
static_assert(sizeof(TraceStatus) <= NOALLOC_STATUS_WORDS * sizeof(int64_t), "status in scratch");
static __device__ __align__(256) int64_t scratch[NOALLOC_SCRATCH_BYTES / sizeof(int64_t)];
static std::mutex g_noalloc_m;
static int64_t *g_noalloc_ptr[MAX_DEVICES];

static int noalloc_scratch(int64_t **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e) return set_hip_error(e);
    if (dev < 0 || dev >= MAX_DEVICES) return HG_E_INVAL;
    std::lock_guard<std::mutex> lock(g_noalloc_m);
    if (!g_noalloc_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e || !p) return set_hip_error(e ? e : hipErrorInvalidSymbol);
        g_noalloc_ptr[dev] = static_cast<int64_t *>(p);
    }
    *out = g_noalloc_ptr[dev];
    return HG_OK;
}

int grid_trace_noalloc(hg_grid_t g, const double *origins, const double *dirs, int64_t n,
                       const hg_trace_opts *opts, hg_trace_out *out, void *stream)
{
    {
        int rc0 = check_trace_args(g, origins, dirs, n, opts, out);
        if (rc0) return rc0;
    }
    if ((scan_tmp_elems(n) + NOALLOC_STATUS_WORDS) * sizeof(int64_t) > NOALLOC_SCRATCH_BYTES) return HG_E_LIMIT;
    hipStream_t s = (hipStream_t)stream;
    for (int i = 0; i < 4; i++) out->kernel_ms[i] = 0.f;
    out->needed = 0;
    out->rechecks = 0;
    out->descents = 0;
    int64_t *base = nullptr;
    int rc = noalloc_scratch(&base);
    if (rc) return rc;
    // the call's status words, then the prefix sum's work space
    TraceStatus *st = reinterpret_cast<TraceStatus *>(base);
    int64_t *tmp = base + NOALLOC_STATUS_WORDS;
    hipEvent_t ev[4] = {};   // no timing: HG_FLAG_TIMING is ignored here
    return trace_two_pass(g, st, origins, dirs, n, opts, out, s, ev, tmp);
}

}  // extern "C"
