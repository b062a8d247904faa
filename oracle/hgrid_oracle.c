/*
 * hgrid_oracle.c -- plain FP64 CPU oracle for hierarchical octree / k-d tree
 * dust grids (Saftly, Baes & Camps 2014, "Hierarchical octree and k-d tree
 * grids for 3D radiative transfer simulations").
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously correct
 * reference that the GPU library is checked against.  Only the test-suite,
 * the smoke check and the CPU-baseline leg of the benchmark may load it.  It
 * shares no code, header or table with the GPU library.
 *
 * Build with -O2 -ffp-contract=off so that no multiply-add is fused: every
 * floating-point expression below is evaluated exactly as written, left to
 * right.
 *
 * What it computes:
 *   or_build      the node list construction loop of Sect. 2.2 with the
 *                 Monte Carlo node mass of Eq. (1), the mass criterion
 *                 delta = M/M_tot (Sect. 2.2, 4.1), the optical-depth
 *                 criterion of Eq. (2) and the density-dispersion criterion
 *                 q of Eq. (3), plus a maximum subdivision level (Sect. 4.2).
 *                 Trees: octree, k-d tree with cyclic split axes, and the
 *                 k-d variant of Sect. 2.2 that splits each node across the
 *                 axis of strongest density gradient (midpoint planes).
 *   or_equal_mass_plane  the equal-mass split location of Sect. 2.2 for one
 *                 cell and axis (a reading for the scope of that variant; the
 *                 trees above split at the midpoint).
 *   or_locate     top-down search for the leaf containing a point (Sect. 2.3).
 *   or_trace      the ordered list of leaves a straight path crosses, the
 *                 length ds inside each and tau = sum kappa rho ds (Sect. 2.3);
 *                 the next leaf is found by a top-down search from the root.
 *   or_trace_brute  the same list found by intersecting the path with every
 *                 leaf box (no tree traversal at all).
 *   or_neighbors_brute  leaves sharing positive face area with a leaf face
 *                 (the neighbor lists of Sect. 2.3), by testing every leaf.
 *
 * Parity status: every function here is pinned by the CPU tests (closed
 * forms, special cases, brute force, the octree == k-d equivalence of
 * Sect. 2.1 and the published SplitMix64 test vector).
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_OCTREE 0
#define OR_KDTREE 1
#define OR_KDGRAD 2   /* k-d tree, split axis of strongest density gradient */
#define OR_MAX_DEPTH 19   /* per-axis halvings the 19-bit cell coordinates allow */

/* ------------------------------------------------------------------------ */
/* Counter-based random numbers: SplitMix64 (Steele, Lea & Flood 2014).      */
/* ------------------------------------------------------------------------ */

#define GOLDEN_GAMMA 0x9E3779B97F4A7C15ULL

/* One SplitMix64 output for state x: advance by the golden gamma, then the
 * published 64-bit mixing function. */
uint64_t or_splitmix64(uint64_t x)
{
    uint64_t z = x + GOLDEN_GAMMA;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* Sequential SplitMix64 stream (state advanced by gamma per draw); used only
 * to check the generator against its published test vector. */
void or_splitmix64_stream(uint64_t seed, int n, uint64_t *out)
{
    uint64_t s = seed;
    for (int i = 0; i < n; i++) {
        out[i] = or_splitmix64(s);
        s += GOLDEN_GAMMA;
    }
}

/* Node code: level in bits 57..62, integer cell coordinates in 19-bit fields. */
static uint64_t node_code(int level, const uint32_t c[3])
{
    return ((uint64_t)level << 57) | ((uint64_t)c[0] << 38) |
           ((uint64_t)c[1] << 19) | (uint64_t)c[2];
}

/* Uniform double in [0,1) for sample j, axis d of the node with this key. */
static double sample_u(uint64_t key, int j, int d)
{
    uint64_t ctr = (uint64_t)(3 * j + d + 1) * GOLDEN_GAMMA;
    uint64_t r = or_splitmix64(key ^ ctr);
    return (double)(r >> 11) * 0x1.0p-53;
}

/* ------------------------------------------------------------------------ */
/* Density field: sum of components, added in the order box, disk, clumps   */
/* (ascending index), torus.                                                 */
/* ------------------------------------------------------------------------ */

typedef struct {
    int has_box;
    double box_lo[3], box_hi[3], box_rho;
    int has_disk;
    double disk_rho0, disk_hR, disk_hz;
    int has_torus;
    double torus_R0, torus_a, torus_rho;
    int64_t n_clumps;
    const double *clump_c;     /* [n][3] */
    const double *clump_sigma; /* [n]    */
    const double *clump_amp;   /* [n]    */
    double clump_trunc;
} or_density;

static double density_at(const or_density *m, const double x[3])
{
    double rho = 0.0;
    if (m->has_box) {
        if (x[0] >= m->box_lo[0] && x[0] <= m->box_hi[0] &&
            x[1] >= m->box_lo[1] && x[1] <= m->box_hi[1] &&
            x[2] >= m->box_lo[2] && x[2] <= m->box_hi[2])
            rho = rho + m->box_rho;
    }
    if (m->has_disk) {
        double R = sqrt(x[0] * x[0] + x[1] * x[1]);
        double arg = -(R / m->disk_hR) - fabs(x[2]) / m->disk_hz;
        rho = rho + m->disk_rho0 * exp(arg);
    }
    for (int64_t i = 0; i < m->n_clumps; i++) {
        double s = m->clump_sigma[i];
        double lim = m->clump_trunc * s;
        double dx = x[0] - m->clump_c[3 * i + 0];
        double dy = x[1] - m->clump_c[3 * i + 1];
        double dz = x[2] - m->clump_c[3 * i + 2];
        double r2 = dx * dx + dy * dy + dz * dz;
        if (r2 <= lim * lim) {
            double e = r2 / (2.0 * s * s);
            rho = rho + m->clump_amp[i] * exp(-e);
        }
    }
    if (m->has_torus) {
        double R = sqrt(x[0] * x[0] + x[1] * x[1]);
        double dR = R - m->torus_R0;
        if (dR * dR + x[2] * x[2] <= m->torus_a * m->torus_a)
            rho = rho + m->torus_rho;
    }
    return rho;
}

void or_density_eval(const or_density *m, const double *pts, int64_t n, double *out)
{
    for (int64_t i = 0; i < n; i++) out[i] = density_at(m, pts + 3 * i);
}

/* ------------------------------------------------------------------------ */
/* Tree                                                                      */
/* ------------------------------------------------------------------------ */

typedef struct {
    int tree;                 /* OR_OCTREE or OR_KDTREE */
    double lo[3], side;       /* domain cube [lo, lo+side]^3 */
    int n_samples;
    int64_t n_nodes, cap;
    int32_t *first_child;     /* -1 for a leaf; children are contiguous */
    uint8_t *level;
    uint32_t *coord;          /* [n][3], cell index at the per-axis depth */
    uint8_t *dep;             /* [n][3], per-axis depth (halvings along each axis) */
    int8_t *axis;             /* split axis of an internal k-d node, else -1 */
    double *S, *rmin, *rmax;  /* sum, min, max of the sampled densities */
    int64_t n_leaves;
    int32_t *leaf_of;         /* node -> leaf id, -1 for internal nodes */
    int32_t *node_of;         /* leaf -> node */
    double *rho;              /* leaf density */
} or_grid;

/* Number of halvings a node at this level has seen along axis d.  Octree:
 * every level halves every axis.  k-d tree: level l splits axis l mod 3
 * (x, y, z, x, ...; Sect. 2.2), so axis d was halved floor((l+2-d)/3) times.
 * (The gradient k-d tree keeps each node's depths in g->dep.) */
static int axis_depth(int tree, int level, int d)
{
    return tree == OR_OCTREE ? level : (level + 2 - d) / 3;
}

static double cell_width(const or_grid *g, int64_t n, int d)
{
    return ldexp(g->side, -(int)g->dep[3 * n + d]);
}

static void node_box(const or_grid *g, int64_t n, double lo[3], double hi[3])
{
    for (int d = 0; d < 3; d++) {
        double w = cell_width(g, n, d);
        uint32_t c = g->coord[3 * n + d];
        lo[d] = g->lo[d] + (double)c * w;
        hi[d] = g->lo[d] + (double)(c + 1) * w;
    }
}

static int grow(or_grid *g, int64_t need)
{
    if (need <= g->cap) return 0;
    int64_t cap = g->cap ? g->cap : 1024;
    while (cap < need) cap *= 2;
    void *p;
#define RE(field, type, k)                                             \
    p = realloc(g->field, (size_t)cap * (k) * sizeof(type));           \
    if (!p) return -1;                                                 \
    g->field = (type *)p;
    RE(first_child, int32_t, 1)
    RE(level, uint8_t, 1)
    RE(coord, uint32_t, 3)
    RE(dep, uint8_t, 3)
    RE(axis, int8_t, 1)
    RE(S, double, 1)
    RE(rmin, double, 1)
    RE(rmax, double, 1)
#undef RE
    g->cap = cap;
    return 0;
}

void or_free(or_grid *g)
{
    if (!g) return;
    free(g->first_child); free(g->level); free(g->coord); free(g->dep); free(g->axis);
    free(g->S); free(g->rmin); free(g->rmax);
    free(g->leaf_of); free(g->node_of); free(g->rho);
    free(g);
}

/* Leaves are the unsplit nodes, numbered in list order. */
static int number_leaves(or_grid *g)
{
    g->leaf_of = (int32_t *)malloc((size_t)g->n_nodes * sizeof(int32_t));
    if (!g->leaf_of) return -1;
    int64_t nl = 0;
    for (int64_t i = 0; i < g->n_nodes; i++)
        g->leaf_of[i] = g->first_child[i] < 0 ? (int32_t)nl++ : -1;
    g->n_leaves = nl;
    g->node_of = (int32_t *)malloc((size_t)(nl ? nl : 1) * sizeof(int32_t));
    g->rho = (double *)malloc((size_t)(nl ? nl : 1) * sizeof(double));
    if (!g->node_of || !g->rho) return -1;
    for (int64_t i = 0; i < g->n_nodes; i++)
        if (g->leaf_of[i] >= 0) g->node_of[g->leaf_of[i]] = (int32_t)i;
    return 0;
}

/* Random-number key of a node.  A gradient k-d node's depths are mixed into
 * its code: nodes of one level may share coordinates at different depths. */
static uint64_t node_key(uint64_t seed, int tree, int level, const uint32_t c[3], const uint8_t dep[3])
{
    uint64_t code = node_code(level, c);
    if (tree == OR_KDGRAD)
        code ^= or_splitmix64((uint64_t)dep[0] | ((uint64_t)dep[1] << 8) | ((uint64_t)dep[2] << 16));
    return or_splitmix64(seed ^ or_splitmix64(code));
}

/* Eq. (1) sampling of one node: S = sum of rho_t at n_samples positions drawn
 * uniformly in the node, summed in sample order; min and max of the samples. */
static void sample_node(const or_density *m, uint64_t seed, int tree, const double dom_lo[3],
                        double side, int n_samples, int level, const uint32_t c[3], const uint8_t dep[3],
                        double *S, double *mn, double *mx)
{
    double lo[3], w[3];
    for (int d = 0; d < 3; d++) {
        w[d] = ldexp(side, -(int)dep[d]);
        lo[d] = dom_lo[d] + (double)c[d] * w[d];
    }
    uint64_t key = node_key(seed, tree, level, c, dep);
    double s = 0.0, lo_r = INFINITY, hi_r = -INFINITY;
    for (int j = 0; j < n_samples; j++) {
        double x[3];
        for (int d = 0; d < 3; d++) x[d] = lo[d] + sample_u(key, j, d) * w[d];
        double r = density_at(m, x);
        s = s + r;
        if (r < lo_r) lo_r = r;
        if (r > hi_r) hi_r = r;
    }
    *S = s; *mn = lo_r; *mx = hi_r;
}

/* Criteria values of one node (Eq. 1-3). */
typedef struct {
    double M, delta, tau, q;
} or_crit;

static or_crit node_criteria(double S, double mn, double mx, const double w[3],
                             int n_samples, double total_mass, double kappa)
{
    or_crit r;
    double V = w[0] * w[1] * w[2];
    r.M = S * (V / (double)n_samples);                         /* Eq. (1) */
    r.delta = r.M / total_mass;
    double diag = sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
    r.tau = kappa * r.M * diag / (w[0] * w[1] * w[2]);         /* Eq. (2) */
    r.q = mx > 0.0 ? (mx - mn) / mx : 0.0;                     /* Eq. (3) */
    return r;
}

typedef struct {
    double total_mass, delta_max, tau_max, q_max, kappa;
    int min_level, max_level, n_samples;
    uint64_t seed;
} or_criteria;

static int decide_split(const or_criteria *cr, int level, or_crit v)
{
    if (level < cr->min_level) return 1;
    if (level >= cr->max_level) return 0;
    return v.delta > cr->delta_max || v.tau > cr->tau_max || v.q > cr->q_max;
}

/* Split axis of a gradient k-d node (Sect. 2.2, the strongest density
 * gradient).  The gradient along axis d is taken as the central difference
 * |rho_t(x_c + w_d/4 e_d) - rho_t(x_c - w_d/4 e_d)| / (w_d/2) between the
 * centres of the node's two halves across d.  Axes already at
 * OR_MAX_DEPTH are not eligible; ties (a uniform region has no gradient at
 * all) go to the axis with the fewest halvings, then the lowest index, which
 * makes a uniform medium's tree the cyclic one.  Returns -1 if no axis is
 * eligible. */
static int gradient_axis(const or_density *m, const double dom_lo[3], double side, const uint32_t c[3],
                         const uint8_t dep[3])
{
    double xc[3], w[3];
    for (int d = 0; d < 3; d++) {
        w[d] = ldexp(side, -(int)dep[d]);
        xc[d] = dom_lo[d] + (double)c[d] * w[d] + 0.5 * w[d];
    }
    int best = -1;
    double gbest = 0.0;
    for (int d = 0; d < 3; d++) {
        if (dep[d] >= OR_MAX_DEPTH) continue;
        double xp[3] = {xc[0], xc[1], xc[2]}, xm[3] = {xc[0], xc[1], xc[2]};
        xp[d] = xc[d] + 0.25 * w[d];
        xm[d] = xc[d] - 0.25 * w[d];
        double gd = fabs(density_at(m, xp) - density_at(m, xm)) / (0.5 * w[d]);
        if (best < 0 || gd > gbest || (gd == gbest && dep[d] < dep[best])) {
            best = d;
            gbest = gd;
        }
    }
    return best;
}

/* The construction loop of Sect. 2.2: the list starts with the root; one pass
 * over the growing list decides each node and appends the children of every
 * node that is split.  Returns NULL on allocation failure or bad input. */
or_grid *or_build(const or_density *m, const or_criteria *cr, int tree,
                  const double dom_lo[3], double side, int64_t max_nodes)
{
    if (tree != OR_OCTREE && tree != OR_KDTREE && tree != OR_KDGRAD) return NULL;
    if (cr->n_samples <= 0 || cr->max_level < 0) return NULL;
    if (tree == OR_OCTREE && cr->max_level > 19) return NULL;
    if (tree != OR_OCTREE && cr->max_level > 57) return NULL;
    or_grid *g = (or_grid *)calloc(1, sizeof(or_grid));
    if (!g) return NULL;
    g->tree = tree;
    for (int d = 0; d < 3; d++) g->lo[d] = dom_lo[d];
    g->side = side;
    g->n_samples = cr->n_samples;
    if (grow(g, 1)) { or_free(g); return NULL; }
    g->n_nodes = 1;
    g->level[0] = 0;
    g->coord[0] = g->coord[1] = g->coord[2] = 0;
    g->dep[0] = g->dep[1] = g->dep[2] = 0;
    int nchild = tree == OR_OCTREE ? 8 : 2;
    for (int64_t i = 0; i < g->n_nodes; i++) {
        int lv = g->level[i];
        uint32_t c[3] = {g->coord[3 * i], g->coord[3 * i + 1], g->coord[3 * i + 2]};
        uint8_t dp[3] = {g->dep[3 * i], g->dep[3 * i + 1], g->dep[3 * i + 2]};
        sample_node(m, cr->seed, tree, g->lo, side, cr->n_samples, lv, c, dp,
                    &g->S[i], &g->rmin[i], &g->rmax[i]);
        double w[3];
        for (int d = 0; d < 3; d++) w[d] = cell_width(g, i, d);
        or_crit v = node_criteria(g->S[i], g->rmin[i], g->rmax[i], w, cr->n_samples,
                                  cr->total_mass, cr->kappa);
        g->axis[i] = -1;
        int a = tree == OR_KDTREE ? lv % 3 : -1;     /* cyclic orientation */
        if (decide_split(cr, lv, v) && tree == OR_KDGRAD) a = gradient_axis(m, g->lo, side, c, dp);
        if (!decide_split(cr, lv, v) || (tree == OR_KDGRAD && a < 0)) {
            g->first_child[i] = -1;
            continue;
        }
        if (tree != OR_OCTREE) g->axis[i] = (int8_t)a;
        if (max_nodes > 0 && g->n_nodes + nchild > max_nodes) { or_free(g); return NULL; }
        if (grow(g, g->n_nodes + nchild)) { or_free(g); return NULL; }
        int64_t f = g->n_nodes;
        g->first_child[i] = (int32_t)f;
        for (int k = 0; k < nchild; k++) {
            uint32_t cc[3] = {c[0], c[1], c[2]};
            uint8_t cd[3] = {dp[0], dp[1], dp[2]};
            if (tree != OR_OCTREE) {
                cc[a] = 2 * c[a] + (uint32_t)k;  /* lower half, then upper half */
                cd[a] = (uint8_t)(dp[a] + 1);
            } else {
                for (int d = 0; d < 3; d++) {    /* octant k = bx + 2 by + 4 bz */
                    cc[d] = 2 * c[d] + (uint32_t)((k >> d) & 1);
                    cd[d] = (uint8_t)(dp[d] + 1);
                }
            }
            g->level[f + k] = (uint8_t)(lv + 1);
            for (int d = 0; d < 3; d++) {
                g->coord[3 * (f + k) + d] = cc[d];
                g->dep[3 * (f + k) + d] = cd[d];
            }
            g->axis[f + k] = -1;
            g->first_child[f + k] = -1;
        }
        g->n_nodes += nchild;
    }
    if (number_leaves(g)) { or_free(g); return NULL; }
    /* Grid density of a leaf: its uniform density M/V = S/N (Sect. 3.2). */
    for (int64_t l = 0; l < g->n_leaves; l++)
        g->rho[l] = g->S[g->node_of[l]] / (double)cr->n_samples;
    return g;
}

/* Rebuild a grid from a first-child array in list (breadth-first) order; levels
 * and cell coordinates follow from the tree (and, for the gradient k-d tree,
 * from axis[]: the split axis of each internal node).  rho may be NULL (then
 * 0).  The sampled statistics are left at zero.  Returns NULL if the arrays
 * are not a valid tree in list order. */
or_grid *or_import_axes(int tree, const double dom_lo[3], double side, int64_t n_nodes,
                        const int32_t *first_child, const int8_t *axis, const double *rho)
{
    if (n_nodes < 1 || (tree != OR_OCTREE && tree != OR_KDTREE && tree != OR_KDGRAD)) return NULL;
    if (tree == OR_KDGRAD && !axis) return NULL;
    or_grid *g = (or_grid *)calloc(1, sizeof(or_grid));
    if (!g) return NULL;
    g->tree = tree;
    for (int d = 0; d < 3; d++) g->lo[d] = dom_lo[d];
    g->side = side;
    g->n_samples = 1;
    if (grow(g, n_nodes)) { or_free(g); return NULL; }
    g->n_nodes = n_nodes;
    memcpy(g->first_child, first_child, (size_t)n_nodes * sizeof(int32_t));
    memset(g->S, 0, (size_t)n_nodes * sizeof(double));
    memset(g->rmin, 0, (size_t)n_nodes * sizeof(double));
    memset(g->rmax, 0, (size_t)n_nodes * sizeof(double));
    int nchild = tree == OR_OCTREE ? 8 : 2;
    int maxlv = tree == OR_OCTREE ? 19 : 57;
    g->level[0] = 0;
    g->coord[0] = g->coord[1] = g->coord[2] = 0;
    g->dep[0] = g->dep[1] = g->dep[2] = 0;
    for (int64_t i = 0; i < n_nodes; i++) g->axis[i] = -1;
    int64_t expect = 1; /* next child slot in list order */
    for (int64_t i = 0; i < n_nodes; i++) {
        int32_t f = first_child[i];
        if (f < 0) continue;
        if (f != expect || f + nchild > n_nodes || g->level[i] >= maxlv) {
            or_free(g);
            return NULL;
        }
        expect += nchild;
        int lv = g->level[i];
        int a = tree == OR_KDTREE ? lv % 3 : (tree == OR_KDGRAD ? axis[i] : -1);
        if (tree == OR_KDGRAD && (a < 0 || a > 2 || g->dep[3 * i + a] >= OR_MAX_DEPTH)) {
            or_free(g);
            return NULL;
        }
        if (tree != OR_OCTREE) g->axis[i] = (int8_t)a;
        for (int k = 0; k < nchild; k++) {
            uint32_t cc[3] = {g->coord[3 * i], g->coord[3 * i + 1], g->coord[3 * i + 2]};
            uint8_t cd[3] = {g->dep[3 * i], g->dep[3 * i + 1], g->dep[3 * i + 2]};
            if (tree != OR_OCTREE) {
                cc[a] = 2 * cc[a] + (uint32_t)k;
                cd[a] = (uint8_t)(cd[a] + 1);
            } else {
                for (int d = 0; d < 3; d++) {
                    cc[d] = 2 * cc[d] + (uint32_t)((k >> d) & 1);
                    cd[d] = (uint8_t)(cd[d] + 1);
                }
            }
            g->level[f + k] = (uint8_t)(lv + 1);
            for (int d = 0; d < 3; d++) {
                g->coord[3 * (f + k) + d] = cc[d];
                g->dep[3 * (f + k) + d] = cd[d];
            }
        }
    }
    if (expect != n_nodes) { or_free(g); return NULL; }
    if (number_leaves(g)) { or_free(g); return NULL; }
    for (int64_t l = 0; l < g->n_leaves; l++) g->rho[l] = rho ? rho[l] : 0.0;
    return g;
}

or_grid *or_import(int tree, const double dom_lo[3], double side, int64_t n_nodes,
                   const int32_t *first_child, const double *rho)
{
    return or_import_axes(tree, dom_lo, side, n_nodes, first_child, NULL, rho);
}

/* Accessors for the test harness. */
int64_t or_n_nodes(const or_grid *g) { return g->n_nodes; }
int64_t or_n_leaves(const or_grid *g) { return g->n_leaves; }
void or_get_nodes(const or_grid *g, int32_t *first_child, uint8_t *level, uint32_t *coord,
                  double *S, double *rmin, double *rmax, int32_t *leaf_of)
{
    size_t n = (size_t)g->n_nodes;
    if (first_child) memcpy(first_child, g->first_child, n * sizeof(int32_t));
    if (level) memcpy(level, g->level, n);
    if (coord) memcpy(coord, g->coord, n * 3 * sizeof(uint32_t));
    if (S) memcpy(S, g->S, n * sizeof(double));
    if (rmin) memcpy(rmin, g->rmin, n * sizeof(double));
    if (rmax) memcpy(rmax, g->rmax, n * sizeof(double));
    if (leaf_of) memcpy(leaf_of, g->leaf_of, n * sizeof(int32_t));
}
/* Per-node split axes (-1 for leaves and octree nodes) and per-axis depths. */
void or_get_axes(const or_grid *g, int8_t *axis, uint8_t *dep)
{
    size_t n = (size_t)g->n_nodes;
    if (axis) memcpy(axis, g->axis, n);
    if (dep) memcpy(dep, g->dep, 3 * n);
}
void or_get_leaves(const or_grid *g, int32_t *node_of, double *rho)
{
    size_t n = (size_t)g->n_leaves;
    if (node_of) memcpy(node_of, g->node_of, n * sizeof(int32_t));
    if (rho) memcpy(rho, g->rho, n * sizeof(double));
}
void or_set_rho(or_grid *g, const double *rho)
{
    memcpy(g->rho, rho, (size_t)g->n_leaves * sizeof(double));
}
void or_leaf_boxes(const or_grid *g, double *lo, double *hi)
{
    for (int64_t l = 0; l < g->n_leaves; l++)
        node_box(g, g->node_of[l], lo + 3 * l, hi + 3 * l);
}

/* Sampled statistics and criteria of one node given by level and coordinates,
 * without building a tree (for spot checks of large builds; octree and cyclic
 * k-d trees, whose per-axis depths follow from the level). */
void or_sample_node(const or_density *m, const or_criteria *cr, int tree, const double dom_lo[3],
                    double side, int level, const uint32_t c[3], double out[7])
{
    double S, mn, mx, w[3];
    uint8_t dep[3];
    for (int d = 0; d < 3; d++) dep[d] = (uint8_t)axis_depth(tree, level, d);
    sample_node(m, cr->seed, tree, dom_lo, side, cr->n_samples, level, c, dep, &S, &mn, &mx);
    for (int d = 0; d < 3; d++) w[d] = ldexp(side, -(int)dep[d]);
    or_crit v = node_criteria(S, mn, mx, w, cr->n_samples, cr->total_mass, cr->kappa);
    out[0] = S; out[1] = mn; out[2] = mx;
    out[3] = v.delta; out[4] = v.tau; out[5] = v.q;
    out[6] = (double)decide_split(cr, level, v);
}

/* or_sample_node for n nodes in turn (level[i], coord[3i..3i+2]): out[7i..7i+6]
 * as or_sample_node.  One thread; the per-node work of the construction loop,
 * for timing it on a sample of a large tree's nodes. */
void or_sample_nodes(const or_density *m, const or_criteria *cr, int tree, const double dom_lo[3],
                     double side, int64_t n, const uint8_t *level, const uint32_t *coord, double *out)
{
    for (int64_t i = 0; i < n; i++)
        or_sample_node(m, cr, tree, dom_lo, side, level[i], coord + 3 * i, out + 7 * i);
}

/* ------------------------------------------------------------------------ */
/* Point location (Sect. 2.3): descend from the root.                        */
/* ------------------------------------------------------------------------ */

/* Side of a split plane c on axis d for a point x_d.  Off the plane the
 * comparison decides; on the plane the tie code decides (1 = upper). */
typedef struct {
    int use_rules;        /* 0: plain locate (ties go upper)                 */
    int exit_axis;        /* axis of the face just crossed, -1 for none      */
    double k[3];          /* ray direction                                  */
    double old_lo[3], old_hi[3]; /* leaf just left                           */
} tie_rule;

static int upper_side(const tie_rule *t, int d, double x, double c)
{
    if (x > c) return 1;
    if (x < c) return 0;
    if (!t->use_rules) return 1;
    if (d == t->exit_axis) return t->k[d] > 0.0;     /* side the ray moves to */
    if (t->exit_axis >= 0) {
        if (c == t->old_hi[d]) return 0;             /* stay in the old slab */
        if (c == t->old_lo[d]) return 1;
    }
    return !(t->k[d] < 0.0);                         /* by direction, 0 -> upper */
}

static int64_t descend(const or_grid *g, const double x[3], const tie_rule *t)
{
    int64_t n = 0;
    while (g->first_child[n] >= 0) {
        int lv = g->level[n];
        double lo[3], hi[3];
        node_box(g, n, lo, hi);
        int64_t f = g->first_child[n];
        if (g->tree != OR_OCTREE) {
            int a = g->axis[n];
            double mid = g->lo[a] + (double)(2 * g->coord[3 * n + a] + 1) *
                                        ldexp(g->side, -((int)g->dep[3 * n + a] + 1));
            n = f + upper_side(t, a, x[a], mid);
        } else {
            int k = 0;
            for (int d = 0; d < 3; d++) {
                double mid = g->lo[d] + (double)(2 * g->coord[3 * n + d] + 1) *
                                            ldexp(g->side, -(lv + 1));
                k |= upper_side(t, d, x[d], mid) << d;
            }
            n = f + k;
        }
        (void)lo; (void)hi;
    }
    return n;
}

static int inside_closed(const or_grid *g, const double x[3])
{
    for (int d = 0; d < 3; d++) {
        if (!(x[d] >= g->lo[d] && x[d] <= g->lo[d] + g->side)) return 0;
    }
    return 1;
}

/* Leaf id of each point; cells are half-open [lo, hi) except that the upper
 * faces of the domain belong to the last cells; -1 outside the closed domain. */
void or_locate(const or_grid *g, const double *pts, int64_t n, int32_t *out)
{
    tie_rule t;
    memset(&t, 0, sizeof t);
    for (int64_t i = 0; i < n; i++) {
        const double *x = pts + 3 * i;
        out[i] = inside_closed(g, x) ? g->leaf_of[descend(g, x, &t)] : -1;
    }
}

/* ------------------------------------------------------------------------ */
/* Path tracing (Sect. 2.3)                                                  */
/* ------------------------------------------------------------------------ */

/* Clip the ray to the closed domain.  Returns 0 for a miss.  On a hit, s is
 * the path length to the entry point and p the entry point (p0 itself when the
 * origin is inside). */
static int clip_ray(const or_grid *g, const double p0[3], const double k[3],
                    const double inv[3], double *s, double p[3])
{
    if (inside_closed(g, p0)) {
        *s = 0.0;
        for (int d = 0; d < 3; d++) p[d] = p0[d];
        return 1;
    }
    double tn = -INFINITY, tf = INFINITY;
    int ax = -1;
    for (int d = 0; d < 3; d++) {
        double lo = g->lo[d], hi = g->lo[d] + g->side;
        if (k[d] == 0.0) {
            if (p0[d] < lo || p0[d] > hi) return 0;
            continue;
        }
        double t1 = (lo - p0[d]) * inv[d];
        double t2 = (hi - p0[d]) * inv[d];
        double a = t1 < t2 ? t1 : t2;
        double b = t1 < t2 ? t2 : t1;
        if (a > tn) { tn = a; ax = d; }
        if (b < tf) tf = b;
    }
    if (!(tn < tf) || !(tf > 0.0) || ax < 0) return 0;
    *s = tn;
    for (int d = 0; d < 3; d++) {
        double lo = g->lo[d], hi = g->lo[d] + g->side;
        if (d == ax) {
            p[d] = k[d] > 0.0 ? lo : hi;
        } else {
            double v = p0[d] + tn * k[d];
            p[d] = v < lo ? lo : (v > hi ? hi : v);
        }
    }
    return 1;
}

/* Walk one ray.  Writes up to cap records (leaf id, ds) if leaf/ds are given;
 * returns the number of leaves crossed with ds > 0, or -1 if the step guard
 * trips.  tau receives sum kappa rho ds over those leaves, in path order. */
static int64_t walk(const or_grid *g, const double p0[3], const double k[3], double kappa,
                    double *tau, int32_t *leaf, double *ds_out, int64_t cap)
{
    double inv[3], p[3], s;
    for (int d = 0; d < 3; d++) inv[d] = 1.0 / k[d];
    *tau = 0.0;
    if (!clip_ray(g, p0, k, inv, &s, p)) return 0;
    tie_rule t;
    memset(&t, 0, sizeof t);
    t.use_rules = 1;
    t.exit_axis = -1;
    for (int d = 0; d < 3; d++) t.k[d] = k[d];
    int64_t node = descend(g, p, &t);
    int64_t count = 0;
    double tau_acc = 0.0;
    const double dom_hi[3] = {g->lo[0] + g->side, g->lo[1] + g->side, g->lo[2] + g->side};
    for (int64_t step = 0; step < 100000000; step++) {
        double lo[3], hi[3];
        node_box(g, node, lo, hi);
        double tmin = INFINITY;
        int a = -1;
        for (int d = 0; d < 3; d++) {
            double td;
            if (k[d] > 0.0) td = (hi[d] - p[d]) * fabs(inv[d]);
            else if (k[d] < 0.0) td = (p[d] - lo[d]) * fabs(inv[d]);
            else td = INFINITY;
            if (td != td) td = INFINITY;
            if (td < tmin) { tmin = td; a = d; }
        }
        if (a < 0) return -1;
        double ds = tmin;
        int32_t lid = g->leaf_of[node];
        if (ds > 0.0) {
            if (leaf && count < cap) { leaf[count] = lid; ds_out[count] = ds; }
            count++;
            tau_acc = tau_acc + kappa * g->rho[lid] * ds;
        }
        if (k[a] > 0.0 ? hi[a] == dom_hi[a] : lo[a] == g->lo[a]) {
            *tau = tau_acc;
            return count;
        }
        /* Re-anchor the exit point on the crossed face. */
        s = s + ds;
        double q[3];
        for (int d = 0; d < 3; d++) {
            if (d == a) {
                q[d] = k[d] > 0.0 ? hi[d] : lo[d];
            } else {
                double v = p0[d] + s * k[d];
                q[d] = v < lo[d] ? lo[d] : (v > hi[d] ? hi[d] : v);
            }
        }
        t.exit_axis = a;
        for (int d = 0; d < 3; d++) { t.old_lo[d] = lo[d]; t.old_hi[d] = hi[d]; }
        node = descend(g, q, &t);
        for (int d = 0; d < 3; d++) p[d] = q[d];
    }
    return -1;
}

typedef struct {
    const or_grid *g;
    const double *o, *k;
    int64_t lo, hi;
    double kappa;
    double *tau;
    int32_t *count;
    const int64_t *offsets;
    int32_t *leaf;
    double *ds;
    int err;
} trace_job;

static void *trace_worker(void *arg)
{
    trace_job *j = (trace_job *)arg;
    for (int64_t i = j->lo; i < j->hi; i++) {
        int32_t *lf = NULL;
        double *dd = NULL;
        int64_t cap = 0;
        if (j->offsets) {
            lf = j->leaf + j->offsets[i];
            dd = j->ds + j->offsets[i];
            cap = j->offsets[i + 1] - j->offsets[i];
        }
        double tau;
        int64_t c = walk(j->g, j->o + 3 * i, j->k + 3 * i, j->kappa, &tau, lf, dd, cap);
        if (c < 0) { j->err = 1; c = 0; }
        if (j->tau) j->tau[i] = tau;
        if (j->count) j->count[i] = (int32_t)c;
    }
    return NULL;
}

/* Trace n rays on nthreads host threads.  With offsets == NULL only tau and
 * count are produced; with offsets (exclusive prefix sum of count, n+1 values)
 * the records are written to leaf[offsets[i] ...] and ds[...].  Returns 0, or
 * -1 if a walk exceeded its step guard. */
int or_trace(const or_grid *g, const double *origins, const double *dirs, int64_t n,
             double kappa, int nthreads, double *tau, int32_t *count,
             const int64_t *offsets, int32_t *leaf, double *ds)
{
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    if ((int64_t)nthreads > n) nthreads = n > 0 ? (int)n : 1;
    pthread_t th[256];
    trace_job jobs[256];
    int64_t chunk = (n + nthreads - 1) / nthreads;
    for (int t = 0; t < nthreads; t++) {
        trace_job *j = &jobs[t];
        j->g = g; j->o = origins; j->k = dirs; j->kappa = kappa;
        j->lo = t * chunk; j->hi = j->lo + chunk < n ? j->lo + chunk : n;
        j->tau = tau; j->count = count; j->offsets = offsets; j->leaf = leaf; j->ds = ds;
        j->err = 0;
        if (j->lo > j->hi) j->lo = j->hi;
        if (nthreads == 1) trace_worker(j);
        else pthread_create(&th[t], NULL, trace_worker, j);
    }
    int err = 0;
    for (int t = 0; t < nthreads; t++) {
        if (nthreads > 1) pthread_join(th[t], NULL);
        err |= jobs[t].err;
    }
    return err ? -1 : 0;
}

/* ------------------------------------------------------------------------ */
/* Brute force: intersect the path with every leaf box.                      */
/* ------------------------------------------------------------------------ */

typedef struct { double t0, ds; int32_t leaf; } brute_hit;

static int cmp_hit(const void *a, const void *b)
{
    const brute_hit *x = (const brute_hit *)a, *y = (const brute_hit *)b;
    if (x->t0 < y->t0) return -1;
    if (x->t0 > y->t0) return 1;
    return 0;
}

/* For one ray, every leaf whose box the path [s_start, inf) crosses with
 * length > eps, sorted by entry distance.  On an axis where the direction is
 * zero the box is taken half-open [lo, hi) (closed at the domain's upper face)
 * so that a path lying in a split plane belongs to one side only.  Returns the
 * number of hits (all written if <= cap). */
int64_t or_trace_brute(const or_grid *g, const double p0[3], const double k[3], double kappa,
                       double eps, double *tau, int32_t *leaf, double *ds, int64_t cap)
{
    double inv[3], p[3], s0;
    for (int d = 0; d < 3; d++) inv[d] = 1.0 / k[d];
    *tau = 0.0;
    if (!clip_ray(g, p0, k, inv, &s0, p)) return 0;
    brute_hit *h = (brute_hit *)malloc((size_t)(g->n_leaves ? g->n_leaves : 1) * sizeof(brute_hit));
    int64_t nh = 0;
    for (int64_t l = 0; l < g->n_leaves; l++) {
        double lo[3], hi[3];
        node_box(g, g->node_of[l], lo, hi);
        double tn = s0, tf = INFINITY;
        int ok = 1;
        for (int d = 0; d < 3 && ok; d++) {
            if (k[d] == 0.0) {
                int top = hi[d] == g->lo[d] + g->side;
                if (!(p0[d] >= lo[d] && (p0[d] < hi[d] || (top && p0[d] == hi[d])))) ok = 0;
                continue;
            }
            double t1 = (lo[d] - p0[d]) * inv[d];
            double t2 = (hi[d] - p0[d]) * inv[d];
            double a = t1 < t2 ? t1 : t2, b = t1 < t2 ? t2 : t1;
            if (a > tn) tn = a;
            if (b < tf) tf = b;
        }
        if (ok && tf - tn > eps) {
            h[nh].t0 = tn; h[nh].ds = tf - tn; h[nh].leaf = (int32_t)l;
            nh++;
        }
    }
    qsort(h, (size_t)nh, sizeof(brute_hit), cmp_hit);
    double acc = 0.0;
    for (int64_t i = 0; i < nh; i++) {
        if (i < cap) { leaf[i] = h[i].leaf; ds[i] = h[i].ds; }
        acc = acc + kappa * g->rho[h[i].leaf] * h[i].ds;
    }
    *tau = acc;
    free(h);
    return nh;
}

/* Every leaf sharing positive area with face f (f = 2*axis + side, side 1 =
 * upper face) of leaf l.  Exact: boxes are compared in integer units of the
 * finest cell width.  Returns the number found (all written if <= cap). */
int64_t or_neighbors_brute(const or_grid *g, int64_t l, int f, int32_t *out, int64_t cap)
{
    int a = f / 2, up = f % 2;
    int D = g->tree == OR_OCTREE ? 19 : 20;
    int64_t me = g->node_of[l];
    int64_t mlo[3], mhi[3];
    for (int d = 0; d < 3; d++) {
        int sh = D - (int)g->dep[3 * me + d];
        mlo[d] = (int64_t)g->coord[3 * me + d] << sh;
        mhi[d] = (int64_t)(g->coord[3 * me + d] + 1) << sh;
    }
    int64_t nf = 0;
    for (int64_t o = 0; o < g->n_leaves; o++) {
        int64_t n = g->node_of[o];
        int64_t lo[3], hi[3];
        for (int d = 0; d < 3; d++) {
            int sh = D - (int)g->dep[3 * n + d];
            lo[d] = (int64_t)g->coord[3 * n + d] << sh;
            hi[d] = (int64_t)(g->coord[3 * n + d] + 1) << sh;
        }
        if (up ? lo[a] != mhi[a] : hi[a] != mlo[a]) continue;
        int touch = 1;
        for (int d = 0; d < 3; d++) {
            if (d == a) continue;
            int64_t L = lo[d] > mlo[d] ? lo[d] : mlo[d];
            int64_t H = hi[d] < mhi[d] ? hi[d] : mhi[d];
            if (H <= L) touch = 0;
        }
        if (touch) {
            if (nf < cap) out[nf] = (int32_t)o;
            nf++;
        }
    }
    return nf;
}

/* ------------------------------------------------------------------------ */
/* Equal-mass split location (Sect. 2.2, the second location option)        */
/* ------------------------------------------------------------------------ */

/* Mass of the slab [lo[d], x] of a cell across axis d, by the midpoint rule
 * on an m x m x m grid of the slab. */
static double slab_mass(const or_density *den, const double lo[3], const double hi[3], int d, double x, int m)
{
    double a[3] = {lo[0], lo[1], lo[2]}, b[3] = {hi[0], hi[1], hi[2]};
    b[d] = x;
    double h[3];
    for (int e = 0; e < 3; e++) h[e] = (b[e] - a[e]) / (double)m;
    double acc = 0.0;
    for (int i = 0; i < m; i++)
        for (int j = 0; j < m; j++)
            for (int k = 0; k < m; k++) {
                double p[3] = {a[0] + ((double)i + 0.5) * h[0], a[1] + ((double)j + 0.5) * h[1],
                               a[2] + ((double)k + 0.5) * h[2]};
                acc = acc + density_at(den, p);
            }
    return acc * h[0] * h[1] * h[2];
}

/* The plane across axis d that splits the cell [lo, hi] into two parts of
 * equal mass: the cell's mass by the midpoint rule on m^3 points, then
 * bisection (iters halvings of [lo_d, hi_d]) on the mass of the lower slab,
 * each slab integrated the same way.  Returns the midpoint of the final
 * bracket. */
double or_equal_mass_plane(const or_density *den, const double lo[3], const double hi[3], int d, int m,
                           int iters)
{
    const double half = 0.5 * slab_mass(den, lo, hi, d, hi[d], m);
    double a = lo[d], b = hi[d];
    for (int it = 0; it < iters; it++) {
        const double x = 0.5 * (a + b);
        if (slab_mass(den, lo, hi, d, x, m) < half) a = x;
        else b = x;
    }
    return 0.5 * (a + b);
}
