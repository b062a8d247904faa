// Internal declarations of the gfx950 hierarchical-grid library.
//
// Data layout in HBM (all arrays breadth-first unless noted):
//   node arrays   first_child i32, level u8, coord u32[3], S/rho_min/rho_max f64,
//                 rope i32[6] (node index of each face's rope target),
//                 leaf_of i32, int_of i32 (internal-node rank or -1)
//   walk arrays   rec32 / rec64: one 32-byte record per leaf holding the six
//                 encoded rope targets and the leaf density (f32 or f64), so
//                 one crossing reads one 32-byte sector;
//                 child u32: per internal node the encoded references of its
//                 2 (k-d) or 8 (octree) children, read one per descent step.
// An encoded reference packs  leaf flag (bit 31) | level (bits 25..30) | id
// (bits 0..24), id being the leaf rank or the internal-node rank.  It is all
// the walk needs: the cell box of the target follows from the level and from
// the coordinates of the leaf being left.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "hgrid.h"

namespace hg {

constexpr int OCT = HG_OCTREE;
constexpr int KD = HG_KDTREE;

constexpr uint32_t NULL_REF = 0xFFFFFFFFu;
constexpr uint32_t LEAF_BIT = 0x80000000u;
constexpr int LEVEL_SHIFT = 25;
constexpr uint32_t ID_MASK = (1u << 25) - 1u;
constexpr int64_t MAX_IDS = int64_t(1) << 25;
constexpr int DEPTH_BITS = 20;  // integer box resolution: per-axis depth <= 19

__host__ __device__ inline int axis_depth(int tree, int level, int d)
{
    return tree == OCT ? level : (level + 2 - d) / 3;
}

__host__ __device__ inline uint32_t make_ref(bool leaf, int level, uint32_t id)
{
    return (leaf ? LEAF_BIT : 0u) | (uint32_t(level) << LEVEL_SHIFT) | id;
}
__host__ __device__ inline bool ref_is_leaf(uint32_t r) { return (r & LEAF_BIT) != 0u; }
__host__ __device__ inline int ref_level(uint32_t r) { return int((r >> LEVEL_SHIFT) & 63u); }
__host__ __device__ inline uint32_t ref_id(uint32_t r) { return r & ID_MASK; }

struct alignas(32) LeafRec32 {
    uint32_t rope[6];
    float rho;
    uint32_t pad;
};
struct alignas(32) LeafRec64 {
    uint32_t rope[6];
    double rho;
};
static_assert(sizeof(LeafRec32) == 32, "record size");
static_assert(sizeof(LeafRec64) == 32, "record size");

// Density field on the device.  Clumps are found through a uniform binning
// grid whose per-bin lists are sorted by clump index, so the sum over clumps
// in range runs in the same (ascending) order as a plain loop over all clumps.
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
};

// What the walk and locate kernels read.
struct WalkGrid {
    int tree;
    int lg;                        // log2 of the domain side
    double lo[3];
    double side;
    uint32_t root;                 // encoded reference of the root
    uint32_t n_leaves, n_internal; // bounds every reference is checked against
    const LeafRec32 *rec32;
    const LeafRec64 *rec64;
    const uint32_t *child;         // [n_internal][2 or 8]
};

// Scratch for device-side status shared by the trace kernels.
struct TraceStatus {
    unsigned long long rechecks;
    int bad_dir;
    int step_guard;
    int bad_ref;                   // a reference out of range: the layout is corrupt
    unsigned int next_ray;         // persistent-kernel work counter
    unsigned int done_waves;
};

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
    hg::LeafRec32 *rec32;
    hg::LeafRec64 *rec64;
    uint32_t *child;
    uint32_t root_ref;
    hg::TraceStatus *status;   // device scratch
    int64_t level_begin[64];   // first node of each level; level_begin[max_level+1] = n_nodes
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
void free_grid_arrays(hg_grid *g);

// Stream-ordered device memory from the device's default pool (kept by the
// pool between calls, so repeated builds do not go back to the driver).
int dalloc(void **p, size_t bytes, hipStream_t s);
void dfree(void *p, hipStream_t s);
template <typename T>
inline int dalloc_n(T **p, size_t n, hipStream_t s)
{
    return dalloc(reinterpret_cast<void **>(p), n * sizeof(T), s);
}

// ---- prefix sums (scan.hip) --------------------------------------------------
// out[0..n] = exclusive prefix sum of in[0..n-1] (out[n] = total).  tmp must
// hold scan_tmp_elems(n) int64 values.
size_t scan_tmp_elems(int64_t n);
int scan_i32_to_i64(const int32_t *in, int64_t *out, int64_t n, int64_t *tmp, hipStream_t s);
int scan_u8_to_i64(const uint8_t *in, int64_t *out, int64_t n, int64_t *tmp, hipStream_t s);

// ---- layout (layout.hip) -----------------------------------------------------
// Given first_child, level and coord for every node (and level_begin), derive
// ropes, leaf / internal numbering, rho32/rho64 walk records and child refs.
// rho_leaf may be NULL, in which case rho = S / n_samples is used.
int finalize_layout(hg_grid *g, const double *rho_leaf, int n_samples, hipStream_t s);

// ---- trace / locate (trace.hip) --------------------------------------------
WalkGrid walk_grid(const hg_grid *g);
int launch_walk(const hg_grid *g, const double *o, const double *k, int64_t n,
                const hg_trace_opts *opts, hg_trace_out *out, bool fill, hipStream_t s,
                float *ms);
int launch_locate(const hg_grid *g, const double *p, int64_t n, int32_t *leaf, hipStream_t s);

}  // namespace hg
