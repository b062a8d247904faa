// Internal declarations of the gfx950 hierarchical-grid library.
//
// Data layout in HBM (all arrays breadth-first unless noted):
//   node arrays   first_child i32, level u8, coord u32[3], S/rho_min/rho_max f64,
//                 rope i32[6] (node index of each face's rope target),
//                 leaf_of i32, int_of i32 (internal-node rank or -1)
//   walk arrays   per-leaf walk records holding the six encoded rope targets
//                 and the leaf density, so one crossing reads one sector;
//                 child: per internal node the encoded references of its
//                 2 (k-d) or 8 (octree) children, read one per descent step;
//                 jump (k-d): per internal node the references three levels
//                 down, one per side triple, read one per three levels.
// An encoded reference packs  kind (top two bits) | level (6 bits) | id:
// kind 2 = leaf (id = leaf rank), 0 = internal node (id = internal-node rank),
// 1 = "twin", an internal node whose children are all leaves (id = the leaf
// rank of its first child; the others follow it), so a descent resolves it
// without reading the child array; all ones is the null reference.  Compact
// layout: 32-bit references (ids < 2^24) and 32-byte records, one f32 and
// one f64 record array; wide layout (larger trees): 64-bit references and
// one 64-byte record holding both densities.  The cell box of a reference's
// target follows from its level and the integer corner of the node the walk
// comes from.
#pragma once

#include <vector>

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "hgrid.h"

namespace hg {

constexpr int OCT = HG_OCTREE;
constexpr int KD = HG_KDTREE;
constexpr int KDG = HG_KDGRAD;     // k-d tree with per-node split axes
constexpr int KDG_MAX_DEPTH = 19;  // halvings along one axis the cell coordinates allow

constexpr int64_t MAX_IDS = int64_t(1) << 24;       // compact-layout id limit
constexpr int DEPTH_BITS = 20;  // integer box resolution: per-axis depth <= 19

__host__ __device__ inline int axis_depth(int tree, int level, int d)
{
    return tree == OCT ? level : (level + 2 - d) / 3;
}

// Reference encoding for R = uint32_t (compact) or uint64_t (wide).  Wide
// references of a gradient k-d tree also carry the node's halvings along x
// and y (z: the level minus both) and, for internal and twin nodes, its split
// axis (GEO_SHIFT: x in bits 0-5, y in 6-11, axis in 12-13); other trees
// leave those bits zero.
template <typename R>
struct Ref {
    static constexpr int BITS = int(sizeof(R) * 8);
    static constexpr int KIND_SHIFT = BITS - 2;
    static constexpr int LEVEL_SHIFT = BITS == 32 ? 24 : 56;
    static constexpr int ID_BITS = BITS == 32 ? 24 : 40;
    static constexpr int GEO_SHIFT = 40;
    static constexpr R NUL = ~R(0);
    enum { INTERNAL = 0, TWIN = 1, LEAF = 2 };
    __host__ __device__ static R make(int kind, int level, uint64_t id)
    {
        return (R(kind) << KIND_SHIFT) | (R(level) << LEVEL_SHIFT) | R(id);
    }
    // with the per-axis halvings dx, dy and split axis ax (wide references)
    __host__ __device__ static R make_geo(int kind, int level, uint64_t id, int dx, int dy, int ax)
    {
        const uint64_t g = uint64_t(dx) | (uint64_t(dy) << 6) | (uint64_t(ax & 3) << 12);
        return make(kind, level, id) | (BITS == 64 ? R(g << GEO_SHIFT) : R(0));
    }
    __host__ __device__ static int kind(R r) { return int(r >> KIND_SHIFT); }
    __host__ __device__ static bool leaf(R r) { return kind(r) == LEAF; }
    __host__ __device__ static bool twin(R r) { return kind(r) == TWIN; }
    __host__ __device__ static int level(R r) { return int((r >> LEVEL_SHIFT) & R(63)); }
    __host__ __device__ static uint64_t id(R r) { return uint64_t(r & ((R(1) << ID_BITS) - R(1))); }
    // halvings along axis d and the split axis (wide references of a gradient k-d tree)
    __host__ __device__ static int depth(R r, int d)
    {
        const uint64_t g = uint64_t(r) >> (BITS == 64 ? GEO_SHIFT : 0);
        const int dx = int(g & 63u), dy = int((g >> 6) & 63u);
        return d == 0 ? dx : (d == 1 ? dy : level(r) - dx - dy);
    }
    __host__ __device__ static int axis(R r) { return int((uint64_t(r) >> (BITS == 64 ? GEO_SHIFT + 12 : 0)) & 3u); }
};

// Packed geometry of a node (hg_grid::geom): halvings along x, y, z in bytes
// 0-2, split axis in bits 24-25 (3: not split).  Filled for every tree.
__host__ __device__ inline int geom_depth(uint32_t gm, int d) { return int((gm >> (8 * d)) & 255u); }
__host__ __device__ inline int geom_axis(uint32_t gm) { return int((gm >> 24) & 3u); }
__host__ __device__ inline uint32_t geom_make(int dx, int dy, int dz, int ax)
{
    return uint32_t(dx) | (uint32_t(dy) << 8) | (uint32_t(dz) << 16) | (uint32_t(ax & 3) << 24);
}
// Split axis and halvings of node n of a tree (level lv): from the level for
// octrees and cyclic k-d trees, from geom for the gradient k-d tree.
__host__ __device__ inline int node_axis(int tree, int lv, const uint32_t *geom, int64_t n)
{
    return tree == KDG ? geom_axis(geom[n]) : (tree == KD ? lv % 3 : -1);
}
__host__ __device__ inline int node_depth(int tree, int lv, const uint32_t *geom, int64_t n, int d)
{
    return tree == KDG ? geom_depth(geom[n], d) : axis_depth(tree, lv, d);
}

struct alignas(32) LeafRec32 {
    uint32_t rope[6];
    float rho;
    uint32_t pad;
};
struct alignas(32) LeafRec64 {
    uint32_t rope[6];
    double rho;
};
struct alignas(64) LeafRecW {
    uint64_t rope[6];
    double rho64;
    float rho32;
    uint32_t pad;
};
static_assert(sizeof(LeafRec32) == 32, "record size");
static_assert(sizeof(LeafRec64) == 32, "record size");
static_assert(sizeof(LeafRecW) == 64, "record size");

// Density field on the device.  Clumps are found through a uniform binning
// grid whose per-bin lists are sorted by clump index, so the sum over clumps
// in range runs in the same (ascending) order as a plain loop over all clumps.
// A clump as the density loop reads it: centre, (trunc sigma)^2, 2 sigma^2
// and amplitude, the products formed as the loop would form them.
struct alignas(16) ClumpRec {
    double cx, cy, cz, lim2, d2, a;
};

struct Dens {
    double lo[3];
    double side;
    int has_box, has_disk, has_torus, n_clumps;
    double box_lo[3], box_hi[3], box_rho;
    double disk_rho0, disk_hR, disk_hz;
    double torus_R0, torus_a, torus_rho;
    double trunc;
    const double *cc;     // [n][3]
    const double *cs;     // [n]
    const double *ca;     // [n]
    int B;                // bins per axis
    double bin_scale;     // B / side
    const uint32_t *bin_items;  // clump indices, ascending within a bin (bin starts passed apart)
    const ClumpRec *bin_recs;   // the clumps of bin_items, entry for entry
};

// What the walk and locate kernels read.
struct WalkGrid {
    int tree;
    int lg;                        // log2 of the domain side
    double lo[3];
    double side;
    double hi[3];                  // lo + side
    uint64_t root;                 // encoded reference of the root
    uint64_t n_leaves, n_internal; // bounds every reference is checked against
    const void *rec;               // walk records of the precision in use
    const void *child;             // [n_internal][2 or 8] references
    const void *jump;              // k-d: [n_internal][8] references three levels down
                                   // (NULL: a descent reads one level at a time)
    const void *table;             // locate table (NULL: descents start at the root)
    int tdep;                      // its per-axis depth: 2^tdep cells per axis
    int dm;                        // finest per-axis depth of any node: every plane is
                                   // lo + i unit with unit = side 2^-dm, i an integer
    double unit;
    double tw, tscale;             // locate-table cell width and 2^tdep / side
};

// Finest per-axis depth of a tree whose levels go up to max_level.
__host__ __device__ inline int finest_depth(int tree, int max_level)
{
    const int ml = max_level < 0 ? 0 : max_level;
    if (tree == KDG) return ml < KDG_MAX_DEPTH ? ml : KDG_MAX_DEPTH;
    return axis_depth(tree, ml, 0);
}

// Locate table: a uniform grid of 2^tdep cells per axis over the domain; cell
// (i, j, k) (index (i 2^tdep + j) 2^tdep + k) holds the encoded reference of
// the deepest node containing the whole cell: the node at the level where
// every axis has depth tdep (k-d 3 tdep, octree tdep), or the leaf holding the
// cell where the tree is coarser.  A path's first descent starts there.
constexpr int TABLE_MAX_DEPTH = 7;
__host__ __device__ inline int table_level(int tree, int tdep) { return tree == OCT ? tdep : 3 * tdep; }
// Table depth for a tree: about the typical leaf's per-axis depth, at most
// TABLE_MAX_DEPTH and never deeper than the tree's levels allow.
__host__ __device__ inline int table_depth(int tree, int64_t n_leaves, int max_level)
{
    int l2 = 0;
    while ((int64_t(1) << (l2 + 1)) <= n_leaves) l2++;
    int t = (l2 + 1) / 3;
    const int deepest = tree == OCT ? max_level : max_level / 3;
    if (t > deepest) t = deepest;
    if (t > TABLE_MAX_DEPTH) t = TABLE_MAX_DEPTH;
    return t < 0 ? 0 : t;
}

// Status words of one trace call, shared by its kernels (see StatusSlot).
struct TraceStatus {
    unsigned long long rechecks;
    unsigned long long descents;   // child levels descended (walk statistics)
    int bad_dir;
    int step_guard;
    int bad_ref;                   // a reference out of range: the layout is corrupt
    int cap_overflow;              // a grid's records did not fit (batched walk, device check)
    int resumed;                   // a path has more records than its row (set by the batched
                                   // row copy; without one the batched resume walk exits)
    unsigned long long next_ray;   // persistent-kernel work counter (64-bit: it grows by one
                                   // chunk per atomic, the drained wavefronts' included)
    unsigned long long done_waves;
};

// Walk state of a path at its first record beyond its row (one-walk records
// mode), taken on entry to that leaf: the record-filling walk resumes the
// path from here instead of from its origin.
struct Resume {
    double s, p[3];
    uint32_t X[3];                 // the node's lower corner in units of WalkGrid::unit
    int32_t lv;
    uint64_t ref;
    int64_t path;
    int32_t steps, pad;
};

// Per-grid arguments of a walk launch.
struct WalkArgs {
    const double *O;
    const double *K;
    int64_t n;
    double kappa;
    double *tau;
    int32_t *count;
    const int64_t *offsets;
    int32_t *leaf;
    void *ds;
    int64_t capacity;              // record slots behind leaf / ds
    TraceStatus *st;
    int count_rechecks;
    int64_t slab;                  // slab walk: record slots per path row
    Resume *resume;                // slab walk: where paths past their row are saved;
                                   // fill walk: the paths to resume (NULL: walk 0 .. n-1)
    unsigned long long *n_resume;  // slab walk: entries written to resume
    int pairs;                     // persistent slab walk, FP32 records: rows of (leaf, ds32)
                                   // pairs in leaf (ds unused)
    int resume_by_path;            // resume entry i is path i's (no counter): the slab walk
                                   // saves there, the fill walk takes path i if count[i] > slab
    const double *lim;             // WM_SEG: s_max per path; WM_INT: tau* per path
};

// Walk modes (see trace.hip).
enum { WM_COUNT = 0, WM_FILL = 1, WM_SLAB = 2, WM_SEG = 3, WM_INT = 4 };

// One entry of the batched walk's work queue: paths [start, end) of a grid.
// One entry of the batched walk's work table: paths [start, end) of grid
// `grid`; head is the table index of that grid's first chunk (the chunks of a
// grid are contiguous and in path order).
struct BatchChunk {
    int32_t grid;
    int32_t head;
    int64_t start, end;
};

// Work queue of a batched walk: the chunk table (each grid's chunks together,
// grids in order), per grid the prefix of its chunk counts (gpre[ng] = the
// table's length) and a counter of its chunks taken (zeroed by the launch).
struct BatchQueue {
    const BatchChunk *chunks;
    const int64_t *gpre;
    unsigned long long *gctr;
    int ng;
    const int32_t *cgrid;          // the grids class by class (grid_classes)
    const int32_t *cpre;           // [ncls + 1]: class c's grids are cgrid[cpre[c] .. cpre[c+1])
    int ncls;
};

// Classes of a batch's grids: grids of one class (tree type, finest per-axis
// depth, domain side) have the same per-level table.  cgrid lists the grids
// class by class, each class's grids in index order; cpre is the prefix of
// the class sizes.
inline void grid_classes(const std::vector<int> &tree, const std::vector<int> &dm, const std::vector<double> &side,
                         std::vector<int32_t> &cgrid, std::vector<int32_t> &cpre)
{
    const size_t ng = tree.size();
    std::vector<int32_t> cls(ng, -1);
    cgrid.clear();
    cpre.assign(1, 0);
    for (size_t i = 0; i < ng; i++) {
        if (cls[i] >= 0) continue;
        const int32_t c = int32_t(cpre.size()) - 1;
        for (size_t j = i; j < ng; j++) {
            if (cls[j] < 0 && tree[j] == tree[i] && dm[j] == dm[i] && side[j] == side[i]) {
                cls[j] = c;
                cgrid.push_back(int32_t(j));
            }
        }
        cpre.push_back(int32_t(cgrid.size()));
    }
}

// gpre of a chunk table (each grid's chunks together, grids in order).
inline std::vector<int64_t> chunk_prefix(const std::vector<BatchChunk> &table, int ng)
{
    std::vector<int64_t> p(size_t(ng) + 1, 0);
    for (const BatchChunk &c : table) p[size_t(c.grid) + 1]++;
    for (int g = 0; g < ng; g++) p[size_t(g) + 1] += p[size_t(g)];
    return p;
}

}  // namespace hg

// The library's grid object.
struct hg_grid {
    int tree;
    int max_level;
    double lo[3];
    double side;
    int64_t n_nodes, n_leaves, n_internal;
    // breadth-first node arrays
    int32_t *first_child;
    uint8_t *level;
    uint32_t *coord;
    double *S, *rmin, *rmax;
    int32_t *rope;      // [n_nodes][6]
    int32_t *leaf_of;
    int32_t *int_of;
    // leaf arrays
    int32_t *node_of;
    double *rho;
    // walk layout
    int wide;                  // 64-bit references and 64-byte records
    hg::LeafRec32 *rec32;      // compact layout
    hg::LeafRec64 *rec64;      // compact layout
    hg::LeafRecW *recw;        // wide layout
    void *child;               // uint32_t or uint64_t references
    void *jump;                // k-d: three-level jump references (same type), or NULL
    uint32_t *geom;            // per node: halvings per axis and split axis (geom_make), or NULL
    uint64_t root_ref;
    void *table;               // locate table (uint32_t or uint64_t references), or NULL
    int tdep;                  // its per-axis depth
    int64_t level_begin[64];   // first node of each level; level_begin[max_level+1] = n_nodes
    int borrowed;              // arrays belong to a batch
    void *block;               // when set, every array above is carved from it
    size_t block_bytes;        // its size and device (block_free)
    int block_dev;
};

namespace hg {

// ---- host helpers (api.hip) -------------------------------------------------
int set_hip_error(hipError_t e);
#define HG_CHECK(expr)                                           \
    do {                                                         \
        hipError_t e_ = (expr);                                  \
        if (e_ != hipSuccess) return ::hg::set_hip_error(e_);    \
    } while (0)

int check_domain(const double lo[3], double side);
int check_build_args(const hg_density *dn, const hg_criteria *cr, int tree_type);
hg_grid *new_grid(int tree, const double lo[3], double side);
void destroy(hg_grid *g);
void free_grid_arrays(hg_grid *g);

// Stream-ordered device memory from the device's default pool (kept by the
// pool between calls, so repeated builds do not go back to the HIP allocator).
int dalloc(void **p, size_t bytes, hipStream_t s);
void dfree(void *p, hipStream_t s);
template <typename T>
inline int dalloc_n(T **p, size_t n, hipStream_t s)
{
    return dalloc(reinterpret_cast<void **>(p), n * sizeof(T), s);
}

// Blocks of grid and batch arrays: freed blocks are kept (a few per device,
// a bounded total) and handed to later builds that fit them, so repeated
// builds neither allocate nor free.  block_alloc stores the device in *dev;
// block_free takes the block back for that device.
int block_alloc(void **p, size_t bytes, int *dev);
void block_free(void *p, size_t bytes, int dev);

// Several arrays carved from one device block (each piece 256-byte aligned):
// one allocation and one free instead of one per array.
class Carve {
  public:
    template <typename T>
    void add(T **p, size_t n)
    {
        const size_t b = (n * sizeof(T) + 255) & ~size_t(255);
        parts_.push_back(Part{reinterpret_cast<void **>(p), b});
        bytes_ += b;
    }
    size_t bytes() const { return bytes_; }
    // from the block cache (see block_alloc)
    int alloc(void **block, int *dev)
    {
        int rc = block_alloc(block, bytes_, dev);
        if (rc) return rc;
        assign(*block);
        return HG_OK;
    }
    // the pieces of a block of at least bytes() that the caller allocated
    void assign(void *block)
    {
        char *q = static_cast<char *>(block);
        for (const Part &pt : parts_) {
            *pt.p = q;
            q += pt.bytes;
        }
    }

  private:
    struct Part {
        void **p;
        size_t bytes;
    };
    std::vector<Part> parts_;
    size_t bytes_ = 0;
};

// ---- prefix sums (scan.hip) --------------------------------------------------
// out[0..n] = exclusive prefix sum of in[0..n-1] (out[n] = total).  tmp must
// hold scan_tmp_elems(n) int64 values.
size_t scan_tmp_elems(int64_t n);

// Records per path row of the one-walk records mode: opts->slab rounded up to
// a multiple of 4, else as many as keep the rows and resume entries of n
// paths within SLAB_BUDGET bytes (at most SLAB_MAX); 0 when the rows do not
// fit (or, for the library's choice, when fewer than SLAB_MIN would).
constexpr double SLAB_BUDGET = double(int64_t(32) << 30);
constexpr int64_t SLAB_MIN = 256, SLAB_MAX = 2048;
int64_t slab_rows(const hg_trace_opts *opts, int64_t n);

// The records-mode scratch of the current device: one buffer, grown on
// demand and kept for later calls (outside the stream-ordered pool).
// scratch_acquire locks it with at least `bytes` bytes (HG_E_OOM, nothing
// held, when that cannot be had); the holder drains its stream before
// scratch_release.
struct Scratch;
int scratch_acquire(size_t bytes, Scratch **out);
void *scratch_ptr(Scratch *w);
void scratch_release(Scratch *w);
int scan_i32_to_i64(const int32_t *in, int64_t *out, int64_t n, int64_t *tmp, hipStream_t s);
int scan_u8_to_i64(const uint8_t *in, int64_t *out, int64_t n, int64_t *tmp, hipStream_t s);
// The same with the element count read from the device at run time (a fixed
// launch shape, so the call can be captured in a graph); tmp holds
// scan_dev_tmp_elems() values.
size_t scan_dev_tmp_elems();
int scan_u8_to_i64_dev(const uint8_t *in, int64_t *out, const int64_t *n_dev, int64_t *tmp,
                       hipStream_t s);
// Offsets of every grid of a batched walk from its counts, one block per
// chunk of the work table (device copies chunks and args); tmp holds
// scan_chunks_tmp_elems(n_chunks) values.
size_t scan_chunks_tmp_elems(int n_chunks);
int scan_chunks(const BatchChunk *chunks, int n_chunks, const WalkArgs *args, int ng, int64_t *tmp,
                hipStream_t s);

// ---- density (build.hip) -------------------------------------------------------
// Device copies of a density's clump arrays and its clump binning grid.
struct DensStore {
    void *cc = nullptr, *cs = nullptr, *ca = nullptr, *bin_start = nullptr, *bin_items = nullptr;
    void *bin_recs = nullptr;
    double bin_load = 0.0;   // clump records per bin, on average over all bins
};
// Copies the density to the device and bins its clumps (synchronises s once
// when there are clumps).  release_density frees what it allocated.
int prepare_density(const hg_density *dn, hipStream_t s, DensStore *st, Dens *out);
void release_density(DensStore *st, hipStream_t s);

// ---- layout (layout.hip) -----------------------------------------------------
// Given first_child, level and coord for every node (and level_begin), derive
// ropes, leaf / internal numbering, rho32/rho64 walk records and child refs.
// rho_leaf may be NULL, in which case rho = S / n_samples is used.
int finalize_layout(hg_grid *g, const double *rho_leaf, int n_samples, hipStream_t s);

// ---- trace / locate (trace.hip) --------------------------------------------
WalkGrid walk_grid(const hg_grid *g, int precision);

// The status words of one trace call (work counter, error flags, statistics),
// from a per-device pool for the duration of the call, so that calls on one
// grid from several host threads or streams never share them.
class StatusSlot {
  public:
    StatusSlot() = default;
    StatusSlot(const StatusSlot &) = delete;
    StatusSlot &operator=(const StatusSlot &) = delete;
    ~StatusSlot();
    int acquire();
    TraceStatus *get() const { return p_; }

  private:
    TraceStatus *p_ = nullptr;
    int dev_ = -1;
};
// Copy a call's status to the host (synchronises s) and turn its flags into a code.
int read_status(const TraceStatus *dev_st, TraceStatus *host, hipStream_t s);
int launch_walk(const hg_grid *g, TraceStatus *st, const double *o, const double *k, int64_t n,
                const hg_trace_opts *opts, hg_trace_out *out, int wm, hipStream_t s,
                float *ms);
int launch_walk_args(const hg_grid *g, const WalkArgs &A, const hg_trace_opts *opts, int wm,
                     hipStream_t s);
int launch_locate(const hg_grid *g, const double *p, int64_t n, int32_t *leaf, hipStream_t s);
// One-pass records mode: each path's first min(count, slab) records from its
// slab row into its CSR slice (rows of (leaf, ds32) pairs when pairs is set).
int launch_slab_compact(const void *sleaf, const void *sds, int64_t slab, int precision, int pairs,
                        const int32_t *count, const int64_t *offsets, int64_t n, int32_t *leaf, void *ds,
                        hipStream_t s);
WalkArgs walk_args(const hg_grid *g, TraceStatus *st, const double *o, const double *k, int64_t n,
                   const hg_trace_opts *opts, hg_trace_out *out);
// The batched walk in mode wm (WM_COUNT, WM_SLAB or WM_FILL) over queue Q.
int launch_batched(const WalkGrid *grids, const WalkArgs *args, const BatchQueue &Q, const hg_trace_opts *opts,
                   int wm, TraceStatus *st, hipStream_t s);
// One-pass batched records: rows (slab_args[g].leaf / ds) into the CSR slices
// (fill_args[g]) of every chunk's paths (Q's table has at most max_chunks
// entries); grids over capacity are flagged.
int launch_slab_compact_batch(const WalkArgs *slab_args, const WalkArgs *fill_args, const BatchQueue &Q,
                              int max_chunks, int precision, int pairs, TraceStatus *st, hipStream_t s);

}  // namespace hg
