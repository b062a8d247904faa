/*
 * hgrid.h -- C ABI of the MI355X (gfx950) hierarchical-grid library.
 *
 * Octree and k-d tree dust grids for Monte Carlo radiative transfer
 * (Saftly, Baes & Camps 2014, "Hierarchical octree and k-d tree grids for 3D
 * radiative transfer simulations"): grid construction with per-node density
 * sampling (Sect. 2.2, Eq. 1-3 of Sect. 4), straight-path traversal that
 * returns the ordered crossed leaves, the length ds in each and the optical
 * depth tau = sum kappa rho ds (Sect. 2.3), and point location (Sect. 2.3).
 *
 * Conventions shared by every call:
 *  - Every call returns int: HG_OK (0) or a negative HG_E_* code.  No call
 *    aborts, throws or prints.  grid_strerror() names a code.
 *  - "stream" is a hipStream_t passed as void* (NULL = the null stream).  Work
 *    is enqueued on that stream; calls that must report a data-dependent
 *    status (record counts, direction checks, node counts) synchronise it
 *    before returning, as documented per call.
 *  - Array arguments are DEVICE pointers owned by the caller unless stated
 *    otherwise; the library never frees them.  Grids are owned by the library
 *    and released by grid_free().
 *  - Points and directions are double[n][3] (x, y, z interleaved).
 *  - The domain is a cube [lo, lo+side]^3 with side a power of two and each
 *    lo a multiple of side/2 (e.g. [-1,1]^3), so that every cell boundary is
 *    an exact binary fraction.
 *  - Leaf ids are ranks among the leaves in the breadth-first node list
 *    (the order in which the construction loop of Sect. 2.2 creates them).
 *  - Trees of up to 2^24 leaves and 2^24 internal nodes use a compact walk
 *    layout (32-bit references, 32-byte leaf records); larger trees switch to
 *    64-bit references and 64-byte records automatically.  The environment
 *    variable HGRID_WIDE_REFS=1 forces the wide layout (for testing).
 */
#ifndef HGRID_H
#define HGRID_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define HG_OK          0
#define HG_E_INVAL    -1  /* null pointer, negative count, unknown enum, bad level range */
#define HG_E_DOMAIN   -2  /* domain not a cube of power-of-two side with lo on a half-side multiple */
#define HG_E_DIR      -3  /* a direction is not finite or | |k| - 1 | > 1e-6 */
#define HG_E_CAPACITY -4  /* crossing records do not fit; tau, count, offsets and needed are valid */
#define HG_E_OOM      -5  /* device allocation failed */
#define HG_E_LIMIT    -6  /* tree exceeds 2^31 nodes or criteria.max_nodes */
#define HG_E_HIP      -7  /* HIP runtime error; grid_last_hip_error() gives the hipError_t */
#define HG_E_STEP     -8  /* a path exceeded the step guard (never expected for valid input) */
#define HG_E_FORMAT   -9  /* imported arrays are not a valid breadth-first tree */

/* ---- enums ------------------------------------------------------------- */
#define HG_OCTREE 0        /* regular 8-way split at the node centre (Sect. 2.1) */
#define HG_KDTREE 1        /* 2-way split at the midpoint, axis cycling x,y,z (Sect. 2.2) */
#define HG_KDGRAD 2        /* 2-way split at the midpoint across the axis of strongest density
                              gradient (the orientation option of Sect. 2.2): the gradient along
                              axis d is |rho(x_c + w_d/4 e_d) - rho(x_c - w_d/4 e_d)| / (w_d/2)
                              between the centres of the node's halves; ties (no gradient) go to
                              the axis halved least often, then the lowest; an axis halved 19
                              times is not split again.  Built by grid_build with max_nodes 0 and
                              by grid_import (with split_axis); walked with 64-bit references. */

#define HG_FP64         0  /* every step of the walk in FP64 */
#define HG_FP32_RECHECK 1  /* FP32 exit decision with FP64 re-anchoring and near-tie recheck */

#define HG_TAU_ONLY 0      /* per path: tau and crossing count */
#define HG_RECORDS  1      /* also the ordered (leaf id, ds) records, CSR by path */

#define HG_FLAG_TIMING   1 /* grid_trace: time the walk kernels with HIP events */
#define HG_FLAG_RECHECKS 2 /* grid_trace: count FP64 rechecks (HG_FP32_RECHECK) and descent levels */

#define HG_MAX_CLUMPS (1 << 24)
#define HG_MAX_BATCH  (1 << 16) /* grids per batch (batch_create) */
#define HG_MAX_CHUNK  (1 << 16) /* hg_trace_opts.chunk: largest paths per work-queue atomic */

#define HG_STAGE_BUILD 1   /* batch_run / batch_capture: construct every grid */
#define HG_STAGE_TRACE 2   /* batch_run / batch_capture: trace the bound path batches */
#define HG_STAGE_ALL   3

/* ---- density field ----------------------------------------------------- */
/* The true density rho_t(x) of Sect. 3.2, given as a sum of parametric
 * components (a C ABI cannot take a device callback).  Components are added in
 * the order box, disk, clumps (ascending index), torus:
 *   box    rho = box_rho inside the closed box [box_lo, box_hi], else 0
 *   disk   rho = disk_rho0 exp(-R/disk_hR - |z|/disk_hz), R = sqrt(x^2+y^2)
 *   clumps rho = amp_i exp(-r^2 / (2 sigma_i^2)) for r <= clump_trunc sigma_i
 *   torus  rho = torus_rho where (R - torus_R0)^2 + z^2 <= torus_a^2
 * The clump arrays are HOST pointers (clump_c is double[n][3]); they are
 * copied during grid_build and may be freed afterwards. */
typedef struct {
    double lo[3];
    double side;
    int32_t has_box;
    double box_lo[3], box_hi[3], box_rho;
    int32_t has_disk;
    double disk_rho0, disk_hR, disk_hz;
    int32_t has_torus;
    double torus_R0, torus_a, torus_rho;
    int64_t n_clumps;
    const double *clump_c;
    const double *clump_sigma;
    const double *clump_amp;
    double clump_trunc;
} hg_density;

/* ---- stopping criteria (Sect. 2.2, 4.1, 4.2) ---------------------------- */
/* A node at level l (root = 0) is split when l < min_level, or when
 * l < max_level and any of  delta = M/total_mass > delta_max  (Sect. 2.2),
 * tau = kappa M sqrt(a^2+b^2+c^2)/(abc) > tau_max  (Eq. 2),
 * q = (rho_max - rho_min)/rho_max > q_max  (Eq. 3; q = 0 when rho_max = 0)
 * holds.  M = V/n_samples * sum of rho_t at n_samples random positions in the
 * node (Eq. 1), drawn by a counter-based SplitMix64 generator keyed by seed
 * and the node's level and cell coordinates.  Use tau_max = +inf and
 * q_max >= 1 to switch those criteria off.  max_level <= 19 (octree) or
 * <= 57 (k-d tree).  max_nodes > 0 bounds the node count (else HG_E_LIMIT). */
typedef struct {
    double total_mass, delta_max, tau_max, q_max, kappa;
    int32_t min_level, max_level, n_samples, reserved;
    uint64_t seed;
    int64_t max_nodes;
} hg_criteria;

/* ---- trace options and outputs ----------------------------------------- */
typedef struct {
    int32_t precision;  /* HG_FP64 or HG_FP32_RECHECK */
    int32_t mode;       /* HG_TAU_ONLY or HG_RECORDS */
    double kappa;       /* opacity in tau = sum kappa rho ds */
    int32_t flags;      /* HG_FLAG_* */
    int32_t block;      /* persistent and batched walks: threads per block, 128, 256 or 512;
                           0 = library choice (256) */
    int32_t persistent; /* persistent lane-refill walk for: bit 0 the counting / tau-only walk,
                           bit 1 the record-filling walk (else one thread per path);
                           -1 = library choice */
    int32_t chunk;      /* persistent walk: paths a wavefront takes per atomic (at most
                           HG_MAX_CHUNK), 0 = library choice */
    int32_t refill_min; /* persistent walk: idle lanes that trigger a refill (1..64), 0 = library choice */
    int32_t lds_bytes;  /* unused (kept for the layout of this struct; at most 65536) */
    int32_t passes;     /* grid_trace, records mode: 1 = one walk writing tau, counts and each
                           path's first `slab` records into a per-path row, then a copy into the
                           CSR slices (paths with more records are resumed where their row
                           filled up); 2 = a counting walk, then a record-filling walk; 0 =
                           library choice (1 when the rows of all paths fit in 32 GiB and the
                           scratch can be had, else 2) */
    int32_t slab;       /* records per path row of the one-pass mode (rounded up to a multiple
                           of 4), 0 = library choice (as many as keep the rows of all paths
                           within 32 GiB, at most 2048; two walks below 256) */
} hg_trace_opts;

/* Outputs of grid_trace; every array is a caller-owned device buffer.
 *   tau[n]       double, sum of kappa rho ds along the path
 *   count[n]     int32, number of leaves crossed with ds > 0
 *   offsets[n+1] int64, exclusive prefix sum of count (HG_RECORDS only)
 *   leaf[cap]    int32 leaf ids in path order (HG_RECORDS only)
 *   ds[cap]      double (HG_FP64) or float (HG_FP32_RECHECK) lengths
 *   (leaf and ds must be 16-byte aligned; HG_E_INVAL otherwise)
 * Set by the call: needed (= offsets[n], the total crossings), rechecks and
 * descents (with HG_FLAG_RECHECKS: exit decisions taken again in FP64, and
 * child levels descended from locate-table cells and rope targets, over all
 * paths of the counting / one-pass walk) and kernel_ms[] (with
 * HG_FLAG_TIMING: [0] count or tau-only walk, [1] prefix sum, [2]
 * record-filling walk, [3] whole call). */
typedef struct {
    double *tau;
    int32_t *count;
    int64_t *offsets;
    int32_t *leaf;
    void *ds;
    int64_t capacity;
    int64_t needed;
    int64_t rechecks;
    float kernel_ms[4];
    int64_t descents;
} hg_trace_out;

/* ---- flat grid arrays (the data exchanged with the oracle and the tests) -- */
/* Node arrays follow the breadth-first node list of Sect. 2.2: node 0 is the
 * root; the children of a split node are contiguous (2 for a k-d tree, lower
 * then upper half; 8 for an octree, octant index bx + 2 by + 4 bz) and appear
 * in the order their parents do.  coord[3] is the cell index of the node
 * along each axis at that axis' depth (octree: level; k-d: floor((level+2-d)/3);
 * gradient k-d: the halvings in geom).
 * rope[6] per leaf, faces -x,+x,-y,+y,-z,+z: the node index of the smallest
 * node containing the whole region just across that face (-1 on the domain
 * boundary); its subtree holds the face's neighbor list of Sect. 2.3.
 * geom per node: halvings along x, y, z in bytes 0-2 and the split axis in
 * bits 24-25 (3: a leaf or an octree node).
 * For grid_import only tree_type, lo, side, n_nodes, first_child and rho are
 * read (device pointers), and for HG_KDGRAD geom (the split axes of the
 * internal nodes; its halvings are recomputed); the rest is ignored.  For
 * grid_export every pointer is a borrowed device pointer into the grid,
 * valid until grid_free. */
typedef struct {
    int32_t tree_type;
    int32_t max_level;
    double lo[3];
    double side;
    int64_t n_nodes, n_leaves;
    const int32_t *first_child; /* [n_nodes], -1 for a leaf */
    const double *rho;          /* [n_leaves], grid density of each leaf */
    const uint8_t *level;       /* [n_nodes] */
    const uint32_t *coord;      /* [n_nodes][3] */
    const double *S;            /* [n_nodes] sum of the sampled densities */
    const double *rho_min;      /* [n_nodes] */
    const double *rho_max;      /* [n_nodes] */
    const int32_t *leaf_of;     /* [n_nodes] leaf id or -1 */
    const int32_t *node_of;     /* [n_leaves] */
    const int32_t *rope;        /* [n_nodes][6] rope target of each face (node index, -1: domain face) */
    const uint32_t *geom;       /* [n_nodes] per-axis halvings and split axis (see above) */
} hg_grid_arrays;

typedef struct hg_grid *hg_grid_t;

/* Build a grid (Sect. 2.2: the node list grows breadth-first; each node's mass
 * is the Monte Carlo estimate of Eq. 1 and it is split by the criteria above;
 * leaves are the unsplit nodes).  The construction runs level by level on the
 * GPU.  With criteria.max_nodes = 0 it synchronises the stream once per level
 * to size the next one; with 0 < max_nodes <= 2^24 every array is reserved
 * for max_nodes nodes up front (about 160 bytes per node) and the levels run
 * with their counts kept on the device, synchronising only at the end (the
 * same tree either way).  Leaf density rho = S/n_samples = M/V (Sect. 3.2).
 * On success *out owns the grid.
 * Errors: HG_E_INVAL, HG_E_DOMAIN, HG_E_LIMIT, HG_E_OOM, HG_E_HIP. */
int grid_build(const hg_density *density, const hg_criteria *criteria, int tree_type,
               void *stream, hg_grid_t *out);

/* Trace n straight paths (Sect. 2.3).  origins and dirs are device double[n][3];
 * each direction must be a unit vector.  A path starts at its origin, or at
 * its entry point into the domain when the origin lies outside; a path that
 * misses the domain has count 0 and tau 0.  The walk visits, in order, every
 * leaf the path crosses with positive length and stops where the path leaves
 * the domain.  Records mode (opts->passes 0 or 1) walks once, writing each
 * path's first opts->slab records into a row of a scratch buffer,
 * then takes the prefix sum of the counts into offsets, copies the rows into
 * the caller's leaf / ds slices and resumes the paths whose records overflowed
 * their row from the state the walk saved at their first record beyond it.
 * The scratch (n x slab x (4 + sizeof ds) bytes plus about 90 bytes per path)
 * belongs to the library: one buffer per device, grown on
 * demand and kept for later calls until grid_release_scratch(); calls that
 * share a device take turns on it.  When it would exceed 32 GiB or cannot be
 * allocated, and with opts->passes == 2, records mode runs a counting walk, a
 * prefix sum and a record-filling walk instead (the same results).  If
 * capacity < needed it returns HG_E_CAPACITY with tau, count, offsets and
 * needed valid.  The call synchronises the stream before returning.
 * Errors: HG_E_INVAL, HG_E_DIR, HG_E_CAPACITY, HG_E_STEP, HG_E_HIP. */
int grid_trace(hg_grid_t grid, const double *origins, const double *dirs, int64_t n,
               const hg_trace_opts *opts, hg_trace_out *out, void *stream);

/* For callers that cannot allocate (code under HIP graph capture, serving
 * loops that forbid device allocation): grid_trace without any allocation.
 * Same arguments, results and errors as grid_trace with opts->passes = 2
 * (records mode: a counting walk, the prefix sum of the counts, a
 * record-filling walk); HG_FLAG_TIMING is ignored (kernel_ms stays 0).  The
 * prefix sum's work space is a fixed device array of HG_NOALLOC_SCRATCH_BYTES
 * that every GPU the library runs on holds until the process ends; it allows
 * n <= HG_NOALLOC_MAX_PATHS (larger n: HG_E_LIMIT, nothing enqueued).  All
 * calls on one GPU share that array: calls that overlap on one GPU (several
 * host threads or streams at once) race and must be serialised by the
 * caller.  Synchronises the stream.  Errors: HG_E_INVAL, HG_E_LIMIT, HG_E_DIR,
 * HG_E_CAPACITY, HG_E_STEP, HG_E_HIP. */
#define HG_NOALLOC_SCRATCH_BYTES (512 * 1024)
#define HG_NOALLOC_MAX_PATHS ((int64_t)(HG_NOALLOC_SCRATCH_BYTES / 8 - 1) * 2048)
int grid_trace_noalloc(hg_grid_t grid, const double *origins, const double *dirs, int64_t n,
                       const hg_trace_opts *opts, hg_trace_out *out, void *stream);

/* Free the device memory the library keeps for reuse on the current device:
 * the records-mode scratch of grid_trace (waiting for the calls using it;
 * the next records-mode call allocates it again) and the array blocks of
 * freed grids and batches (up to four blocks, 16 GiB in total, handed to
 * later builds that fit them).  Errors: HG_E_HIP. */
int grid_release_scratch(void);

/* Trace several grids' path batches in one persistent launch per walk pass
 * (Sect. 2.3, as grid_trace).  Entry g traces n[g] paths origins[g] / dirs[g]
 * through grids[g] into outs[g] with the shared options opts.  The device
 * work queue holds chunks of opts->chunk paths (0 = library choice) of one
 * grid each; wavefronts take chunks with one atomic and mix octree and k-d
 * grids freely.  Records mode: one counting launch for the whole batch, a
 * prefix sum per grid, one record-filling launch; HG_E_CAPACITY if any
 * outs[g].capacity < outs[g].needed (all needed are set).  Results equal
 * those of n_grids separate grid_trace calls bit for bit.  The batch's
 * rechecks and kernel times are reported in outs[0].  Grids that need the
 * wide layout are traced one by one.  Synchronises the stream.  Errors as
 * grid_trace. */
int grid_trace_batched(int n_grids, const hg_grid_t *grids, const double *const *origins,
                       const double *const *dirs, const int64_t *n, const hg_trace_opts *opts,
                       hg_trace_out *outs, void *stream);

/* Autotune the launch shape of grid_trace's persistent walk for this grid and
 * workload.  The results of a trace do not depend on the launch shape, only
 * its speed does.  Times the walk of the n paths origins / dirs (device, a
 * representative sample of the workload) with HIP events for candidate
 * shapes -- threads per block, LDS bytes of staged top levels, paths per
 * work-queue atomic and the refill threshold -- by coordinate descent from
 * the library defaults, and writes the fastest into opts->block, lds_bytes,
 * chunk and refill_min (opts->persistent is set to 3; precision, mode and
 * kappa are inputs).  Records mode times the counting plus the filling walk
 * with record buffers the call allocates.  *best_ms (may be NULL) receives
 * the winner's walk time.  Synchronises the stream.  Errors as grid_trace. */
int grid_tune(hg_grid_t grid, const double *origins, const double *dirs, int64_t n,
              hg_trace_opts *opts, float *best_ms, void *stream);

/* ---- consumers of the walk: grid quality (Sect. 3.2), interaction point -- */
/* First quality measure of Sect. 3.2: diff_out[i] = rho_t(x_i) - rho_g(x_i)
 * for the n points (device double[n][3]), rho_t the density model dens
 * (host description, copied; normally the one the grid was built from), rho_g
 * the density of the leaf holding x_i (NaN outside the domain).  Its standard
 * deviation over uniform points is the measure.  Asynchronous except for one
 * synchronisation when dens has clumps.  Errors: HG_E_INVAL, HG_E_DOMAIN,
 * HG_E_OOM, HG_E_HIP. */
int grid_density_diff(hg_grid_t grid, const hg_density *dens, const double *points, int64_t n,
                      double *diff_out, void *stream);

/* Second quality measure of Sect. 3.2, grid side: tau_out[i] = the optical
 * depth of path i from its start up to length s_max[i] (device arrays of n),
 * i.e. the sum of kappa rho ds over its crossings with the last one cut at
 * s_max[i].  records: the outputs of a records-mode grid_trace of these paths
 * on this grid (offsets, leaf, ds; ds of the given precision); paths start at
 * their origins when those lie inside the domain.  Asynchronous.  Errors:
 * HG_E_INVAL, HG_E_HIP. */
int grid_segment_tau(hg_grid_t grid, const hg_trace_out *records, int precision, int64_t n,
                     const double *s_max, double kappa, double *tau_out, void *stream);

/* Second quality measure of Sect. 3.2, true side: tau_out[i] = the integral
 * of kappa rho_t along path i (origins / dirs as traced) up to length
 * s_max[i], by m-node Gauss-Legendre quadrature (1 <= m <= 64) on every piece
 * between consecutive cell boundaries of the path (from records, as above).
 * Synchronises the stream once.  Errors: HG_E_INVAL, HG_E_DOMAIN, HG_E_OOM,
 * HG_E_HIP. */
int grid_true_tau(hg_grid_t grid, const hg_density *dens, const double *origins, const double *dirs,
                  const hg_trace_out *records, int precision, int64_t n, const double *s_max,
                  double kappa, int m, double *tau_out, void *stream);

/* Monte Carlo interaction point along each path: the first crossing where
 * the cumulative optical depth reaches tau_star[i] (e.g. -ln(1 - u) for a
 * uniform u), leaf_out[i] its leaf id and s_out[i] the distance along the
 * path where tau reaches tau_star[i] (tau grows linearly inside a cell); if
 * the whole path stays below, leaf_out[i] = -1 and s_out[i] = its length.
 * records as above; kappa > 0.  Asynchronous.  Errors: HG_E_INVAL,
 * HG_E_HIP. */
int grid_interact(hg_grid_t grid, const hg_trace_out *records, int precision, int64_t n,
                  const double *tau_star, double kappa, int32_t *leaf_out, double *s_out,
                  void *stream);

/* The same two consumers as walks that stop early and write no records: one
 * persistent walk over the paths (exit decisions in opts->precision, tau
 * summed in FP64 from the FP64 leaf densities in both precisions; the leaf
 * sequence and ds are those of grid_trace).  s is the distance along the
 * path from its origin (a part before the domain entry counts).
 *
 * grid_trace_segment (Sect. 3.2, second measure, grid side): tau_out[i] =
 * kappa * sum of rho ds over path i up to length s_max[i] (the leaf holding
 * s = s_max[i] adds its part up to there; the walk stops there), count_out[i]
 * = the leaves with ds > 0 that this part enters.  A NaN s_max counts as 0.
 *
 * grid_trace_interact (Monte Carlo interaction point, Sect. 1 and 2.3):
 * leaf_out[i] = the first leaf where the cumulative optical depth reaches
 * tau_star[i] and s_out[i] the distance where it does (tau grows linearly in
 * the leaf); -1 and the path's whole length when it stays below (paths that
 * miss the domain: -1 and 0).
 *
 * origins, dirs: n x 3 doubles (device), as grid_trace; s_max / tau_star: n
 * doubles (device); outputs: n values each (device, caller-owned).  Of opts
 * only precision, kappa, block, chunk and refill_min are read (the walk is
 * always persistent).  Synchronises the stream once.  Errors: HG_E_INVAL,
 * HG_E_DIR (a direction that is not a unit vector: that path's tau_out or
 * s_out is NaN), HG_E_STEP, HG_E_FORMAT, HG_E_HIP. */
int grid_trace_segment(hg_grid_t grid, const double *origins, const double *dirs, const double *s_max,
                       int64_t n, const hg_trace_opts *opts, double *tau_out, int32_t *count_out,
                       void *stream);
int grid_trace_interact(hg_grid_t grid, const double *origins, const double *dirs, const double *tau_star,
                        int64_t n, const hg_trace_opts *opts, int32_t *leaf_out, double *s_out,
                        void *stream);

/* ---- the optical-depth recipe of Sect. 4.1 ---------------------------- */
/* tau_out[l] (device, n_leaves) = the optical depth of leaf l by Eq. (2) with
 * its sampled mass M = S (V / n_samples) of Eq. (1) (n_samples as in the
 * build).  Asynchronous.  Errors: HG_E_INVAL, HG_E_HIP. */
int grid_leaf_tau(hg_grid_t grid, double kappa, int n_samples, double *tau_out, void *stream);

/* *tau_max (host) = the leaf optical depth at position floor(fraction
 * n_leaves) (0-based, at most n_leaves - 1) of the ascending order, found on
 * the device by radix select.  Synchronises the stream.  Errors: HG_E_INVAL,
 * HG_E_OOM, HG_E_HIP. */
int grid_tau_percentile(hg_grid_t grid, double kappa, int n_samples, double fraction,
                        double *tau_max, void *stream);

/* The recipe of Sect. 4.1: build with criteria minus the optical-depth
 * criterion, take tau_max = grid_tau_percentile(fraction) (0.9 in the paper),
 * build again with criteria and that tau_max; *tau_max receives it.
 * Synchronises the stream.  Errors as grid_build. */
int grid_build_tau_recipe(const hg_density *dens, const hg_criteria *criteria, int tree_type,
                          double fraction, void *stream, hg_grid_t *out, double *tau_max);

/* Leaf containing each point (Sect. 2.3, top-down search).  points is device
 * double[n][3]; leaf_out device int32[n].  Cells are half-open [lo, hi) along
 * each axis except that the domain's upper faces belong to the last cells;
 * points outside the closed domain (or with a NaN coordinate) give -1.
 * Asynchronous.  Errors: HG_E_INVAL, HG_E_HIP. */
int grid_locate(hg_grid_t grid, const double *points, int64_t n, int32_t *leaf_out,
                void *stream);

/* Copy a tree given by its breadth-first first-child array and leaf densities
 * into a new grid (deep copy; levels, cell coordinates and ropes are derived
 * on the GPU).  Used to trace a grid built elsewhere, e.g. by a CPU reference.
 * Synchronises the stream.  Errors: HG_E_INVAL, HG_E_DOMAIN, HG_E_FORMAT,
 * HG_E_LIMIT, HG_E_OOM, HG_E_HIP. */
int grid_import(const hg_grid_arrays *arrays, void *stream, hg_grid_t *out);

/* Fill *out with the grid's counts and borrowed device pointers (see
 * hg_grid_arrays).  Errors: HG_E_INVAL. */
int grid_export(hg_grid_t grid, hg_grid_arrays *out);

/* Release a grid and its device memory (NULL is ignored).  The caller must
 * make sure no work using the grid is still queued. */
void grid_free(hg_grid_t grid);

/* ---- batches: many grids built and traced without host synchronisation -- */
/* A batch holds n_grids grids whose construction (Sect. 2.2 with the
 * criteria of Sect. 4, exactly as grid_build) and path tracing (Sect. 2.3,
 * exactly as grid_trace_batched) are enqueued with launch shapes fixed in
 * advance and every count kept on the device.  batch_run therefore neither
 * allocates nor synchronises, and batch_capture records it into a HIP graph
 * that batch_replay launches again (the build-then-trace pass of a batch with
 * new contents of the bound input buffers, or simply again).  Grids use the
 * compact layout only (node capacity at most 2^24); a k-d grid's arrays
 * include its jump references (about 16 more bytes per node). */
typedef struct hg_batch *hg_batch_t;

/* Reserve a batch: density dens[g] (copied; clumps binned here), criteria
 * crit[g] and tree type tree_types[g] of every grid.  crit[g].max_nodes >= 1
 * is grid g's node capacity: all its device arrays (about 160 bytes per node)
 * are allocated now.  Synchronises the device.  Errors: HG_E_INVAL (as
 * grid_build, or max_nodes < 1, or n_grids outside 1..HG_MAX_BATCH, or a
 * HG_KDGRAD tree),
 * HG_E_DOMAIN, HG_E_LIMIT (max_nodes > 2^24), HG_E_OOM, HG_E_HIP. */
int batch_create(int n_grids, const hg_density *dens, const hg_criteria *crit,
                 const int *tree_types, hg_batch_t *out);

/* Bind the path batches every later trace stage reads: origins[g] / dirs[g]
 * (device, n[g] paths) into outs[g] (caller-owned device buffers, as
 * grid_trace; the pointers are kept, the buffers must outlive their use).
 * opts as grid_trace_batched (chunk = paths per work-queue entry).  Records
 * mode walks the paths once unless opts->passes is 2: each path's first
 * opts->slab records (0: as many as fit 32 GiB, or half the free device memory
 * if less, over all paths, at most 2048)
 * go to a row of its own and a path past its row is saved where the row
 * filled up; the rows are then copied into the CSR slices and the saved paths
 * resume, all on the device.  When fewer than 16 rows per path fit, it walks
 * twice (counting, then filling).  Replaces an earlier binding and drops a
 * captured graph.  Synchronises the device.  Errors: HG_E_INVAL, HG_E_LIMIT,
 * HG_E_OOM, HG_E_HIP. */
int batch_bind(hg_batch_t batch, const double *const *origins, const double *const *dirs,
               const int64_t *n, const hg_trace_opts *opts, hg_trace_out *outs);

/* Enqueue the stages (HG_STAGE_*) on stream: no allocation, no host
 * synchronisation.  The trace stage reads the grids of the last build stage
 * and needs a binding.  Records mode: a grid whose records exceed its
 * capacity gets none written (batch_result reports it).  Errors: HG_E_INVAL,
 * HG_E_HIP. */
int batch_run(hg_batch_t batch, int stages, void *stream);

/* Capture batch_run(batch, stages) on stream (not the legacy default stream)
 * into a graph kept by the batch; batch_replay(batch, stream) launches it.
 * Errors: HG_E_INVAL, HG_E_HIP. */
int batch_capture(hg_batch_t batch, int stages, void *stream);
int batch_replay(hg_batch_t batch, void *stream);

/* Wait for the stream and read the results of the last run or replay:
 * per-grid node and leaf counts (arrays of n_grids, may be NULL) and, when
 * that run included the trace stage, outs[g].needed (records mode) and the
 * recheck count in outs[0].rechecks (with HG_FLAG_RECHECKS).  Returns HG_E_LIMIT if a grid
 * exceeded its node capacity (its tree is incomplete), HG_E_CAPACITY if a
 * grid's records did not fit, else the trace errors of grid_trace. */
int batch_result(hg_batch_t batch, void *stream, int64_t *n_nodes, int64_t *n_leaves,
                 hg_trace_out *outs);

/* A grid handle on grid g of a built batch, for grid_trace, grid_locate and
 * grid_export; it borrows the batch's arrays (valid until the next build
 * stage or batch_free) and is released with grid_free.  Synchronises the
 * device.  Errors: HG_E_INVAL, HG_E_LIMIT (the grid exceeded its capacity),
 * HG_E_OOM, HG_E_HIP. */
int batch_grid(hg_batch_t batch, int g, hg_grid_t *out);

/* Autotune the bound trace of a built batch: times the bound trace stage for
 * candidate threads per block, paths per work-queue entry and refill
 * thresholds (coordinate descent, HIP events) and rebinds the batch with the
 * fastest (which drops a captured graph: tune before batch_capture).  The
 * output buffers are written during the search.  *chosen (may be NULL)
 * receives the winning options, *best_ms (may be NULL) their walk time.
 * Synchronises the stream.  Errors: HG_E_INVAL (no binding), HG_E_LIMIT,
 * HG_E_OOM, HG_E_HIP. */
int batch_tune(hg_batch_t batch, hg_trace_opts *chosen, float *best_ms, void *stream);

/* Release a batch and its device memory (NULL is ignored); synchronises the
 * device.  Grid handles from batch_grid must be freed before. */
void batch_free(hg_batch_t batch);

/* Static description of a status code. */
const char *grid_strerror(int code);

/* hipError_t of the last HG_E_HIP returned on this thread (0 if none). */
int grid_last_hip_error(void);

#ifdef __cplusplus
}
#endif

#endif /* HGRID_H */
