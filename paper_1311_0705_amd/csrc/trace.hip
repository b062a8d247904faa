// Straight-path traversal (Sect. 2.3) and point location on gfx950.
//
// One lane walks one path.  Per crossing the lane
//   1. finds the exit face of its leaf: the face distances Delta_d from the
//      entry point, t_d = Delta_d |1/k_d|, and the lowest axis of the minimum;
//   2. adds kappa rho ds to tau (and in the record modes records (leaf, ds));
//   3. re-anchors the exit point: the crossed face's plane on the exit axis,
//      p0 + s k clamped to the leaf on the others (s = path length so far);
//   4. takes the rope of the exit face from the leaf's 32-byte record (read at
//      the start of the crossing, so the load overlaps the exit decision) and
//      moves its cell to the rope target; a target that is not a leaf is
//      descended with the exit point, one level per step: a "twin" (all
//      children leaves) without a memory access, other nodes by one 4-byte
//      child reference.
// Boxes are never loaded.  A lane carries the integer lower corner of its
// node in units of the grid's finest plane spacing (unit = side 2^-dm) and
// its level; the planes follow exactly as lo + corner * unit, the widths from
// a per-level table in LDS.  Ties on a split plane follow one fixed rule so
// that the result is reproducible to the bit (see tie_upper).
//
// HG_FP32_RECHECK decides the exit face in FP32 from face distances rounded
// from FP64 and rechecks in FP64 when the two smallest FP32 exit distances
// are closer than 1e-5 of the leaf's smallest side; only the chosen axis'
// exit distance (ds) and the re-anchoring are FP64, so the leaf sequence is
// that of the FP64 walk.  tau is then a Kahan-compensated FP32 sum of
// kappa rho32 ds32.
//
// The persistent walks keep lanes busy as paths end: each wavefront prepares
// 64 paths at a time with all its lanes (direction check, inverse direction,
// entry point, locate-table cell) into an LDS queue, and a lane whose path
// ended takes the next prepared one.
#include <math.h>

#include <algorithm>
#include <atomic>
#include <map>
#include <mutex>
#include <tuple>
#include <type_traits>

#include "common.h"

namespace hg {

namespace {

constexpr int TB = 256;
constexpr int64_t STEP_GUARD = int64_t(1) << 26;
constexpr int NLEV = 64;      // levels of the per-level table (references hold 6-bit levels)
constexpr int RING = 64;      // prepared paths per wavefront
constexpr int SG = 8;         // records a lane stages in LDS before its group is written

// Keep a value in registers: a choice among array elements passed through
// this stays a register select instead of being folded into an indexed access,
// which would move the whole array to the stack.
__device__ __forceinline__ double in_reg(double x)
{
    asm volatile("" : "+v"(x));
    return x;
}
__device__ __forceinline__ uint32_t in_reg(uint32_t x)
{
    asm volatile("" : "+v"(x));
    return x;
}

// IEEE min / max of two doubles that are never NaN (or where a NaN operand
// must lose, as for an exit distance): one instruction each, without the
// quieting of operands the compiler adds to fmin / fmax of values it cannot
// prove canonical.
__device__ __forceinline__ double min64(double a, double b)
{
    double r;
    asm("v_min_f64 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
    return r;
}
__device__ __forceinline__ double max64(double a, double b)
{
    double r;
    asm("v_max_f64 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
    return r;
}

// Geometry of the nodes of one level: the widths per axis as doubles (exact
// powers of two) and in units of WalkGrid::unit, the split axis and half
// width a descent uses, and the FP32 recheck threshold (1e-5 of the smallest
// width, which is axis 0's: no axis is finer).  For a k-d jump from this
// level: per axis, the half width of the split among this level and the next
// two that cuts it (jhw) and that split's level offset (byte d of jof).
struct alignas(16) LevelGeo {
    double w[3];
    uint32_t W[3];
    uint32_t hw;
    float guard;
    int32_t axis;
    uint32_t jhw[3];
    uint32_t jof;
};
static_assert(sizeof(LevelGeo) == 64, "level record");

__device__ __forceinline__ LevelGeo make_level(int tree, int dm, double side, int lv)
{
    LevelGeo e;
#pragma unroll
    for (int d = 0; d < 3; d++) {
        const int dep = axis_depth(tree, lv, d);
        const int sh = dm - dep;
        e.W[d] = sh >= 0 && sh < 32 ? 1u << sh : 0u;
        e.w[d] = ldexp(side, -dep);
    }
    e.axis = tree == KD ? lv % 3 : 0;
    const uint32_t W0 = in_reg(e.W[0]), W1 = in_reg(e.W[1]), W2 = in_reg(e.W[2]);
    e.hw = (e.axis == 0 ? W0 : (e.axis == 1 ? W1 : W2)) >> 1;
    e.guard = 1e-5f * float(e.w[0]);
    e.jof = 0;
    e.jhw[0] = e.jhw[1] = e.jhw[2] = 0;
#pragma unroll
    for (int j = 0; j < 3; j++) {
        // k-d level lv + j splits axis (lv + j) mod 3, halving its width there
        const int d = (lv + j) % 3;
        const int sh = dm - axis_depth(tree, lv + j, d) - 1;
        const uint32_t h = tree == KD && sh >= 0 && sh < 32 ? 1u << sh : 0u;
        e.jhw[0] = d == 0 ? h : e.jhw[0];
        e.jhw[1] = d == 1 ? h : e.jhw[1];
        e.jhw[2] = d == 2 ? h : e.jhw[2];
        e.jof |= uint32_t(j) << (8 * d);
    }
    return e;
}

// Fill a level table (all NLEV levels) with the threads [t0, t0 + nt).
__device__ __forceinline__ void fill_levels(LevelGeo *geo, const WalkGrid &G, int t0, int nt)
{
    for (int j = t0; j < NLEV; j += nt) geo[j] = make_level(G.tree, G.dm, G.side, j);
}

// Geometry of a gradient k-d node from its (wide) reference, in the fields
// of a level record: widths from the halvings the reference carries, the
// FP32 recheck threshold from the smallest width, and the split axis with
// its half width.
template <typename R>
__device__ __forceinline__ LevelGeo ref_geo(const WalkGrid &G, R ref)
{
    LevelGeo e;
    double wmin = INFINITY;
#pragma unroll
    for (int d = 0; d < 3; d++) {
        const int dep = Ref<R>::depth(ref, d);
        const int sh = G.dm - dep;
        e.W[d] = sh >= 0 && sh < 32 ? 1u << sh : 0u;
        e.w[d] = ldexp(G.side, -dep);
        wmin = e.w[d] < wmin ? e.w[d] : wmin;
    }
    e.guard = 1e-5f * float(wmin);
    const int a = Ref<R>::axis(ref);
    const int sa = G.dm - Ref<R>::depth(ref, a) - 1;
    e.axis = a;
    e.hw = sa >= 0 && sa < 32 ? 1u << sa : 0u;
    return e;
}

// Halvings along axis d of the node of reference ref at level lv.
template <int TREE, typename R>
__device__ __forceinline__ int ref_depth(R ref, int lv, int d)
{
    return TREE == KDG ? Ref<R>::depth(ref, d) : axis_depth(TREE, lv, d);
}

// A path prepared by its wavefront, waiting in the LDS queue.
struct alignas(16) Prep {
    double ainv[3];     // |1/k|
    double s;           // path length at the start (> 0 when the origin lies outside)
    uint32_t X[3];      // start node: integer lower corner
    uint32_t lvf;       // its level | (clip axis + 1) << 8 (0: origin inside) | force FP64 << 12
    uint64_t ref;       // start node reference
    int32_t idx;        // path index within the launch (resume-entry index for resumed paths)
    int32_t pad;
};
static_assert(sizeof(Prep) == 64, "queue entry");

// Everything a lane carries for one path.
template <int PREC, typename R>
struct Lane {
    using DsT = typename std::conditional<PREC == HG_FP64, double, float>::type;
    double p0[3], k[3], ainv[3];
    float ainv32[3];         // FP32 copies of ainv for the FP32 exit decision
    double s, p[3];          // path length so far and the current entry point
    uint32_t X[3];           // integer lower corner of the current node
    R ref;                   // current node (a leaf when a crossing is due)
    int lv;                  // its level
    int tie;                 // tie context of a pending descent (tie_upper)
    int32_t cnt;             // leaves crossed with ds > 0
    int steps;
    double tau64;
    float tau32, comp32;
    double lim;              // early-exit walks: s_max or tau* (after a hit: its s)
    bool force64;
    int64_t base, room;      // record slice of this path (record modes)
    uint32_t sl[4];          // one-thread walk: the last four records, staged
    DsT sd[4];               // for 16-byte aligned vector stores
};

enum { PATH_WALK = 0, PATH_MISS = 1, PATH_BAD_DIR = 2 };
enum { STEP_GO = 0, STEP_END = 1, STEP_ERR = 2 };
// Walk modes: WM_COUNT (tau and counts; also the tau-only mode), WM_FILL
// (records into the slices given by the offsets of a counting walk),
// WM_SLAB (tau, counts and the first A.slab records of every path into a
// fixed-size row per path, for the one-pass records mode), and the
// early-exit walks, which accumulate tau in FP64 from the FP64 records in
// both precisions: WM_SEG (tau of the first s_max of the path, Sect. 3.2)
// and WM_INT (the leaf and distance where tau reaches tau*, the Monte Carlo
// interaction point of Sect. 1 and 2.3).

__device__ __forceinline__ bool inside_closed(const WalkGrid &G, const double x[3])
{
    bool in = true;
#pragma unroll
    for (int d = 0; d < 3; d++) in = in && (x[d] >= G.lo[d] && x[d] <= G.hi[d]);
    return in;
}

// Coordinate d of the entry point at path length tn through the face of axis ax.
__device__ __forceinline__ double entry_coord(const WalkGrid &G, const double p0[3], const double k[3],
                                              double tn, int ax, int d)
{
    const double lo = G.lo[d], hi = G.hi[d];
    if (d == ax) return k[d] > 0.0 ? lo : hi;
    const double v = p0[d] + tn * k[d];
    return v < lo ? lo : (v > hi ? hi : v);
}

// Start of the path inside the closed domain: the origin itself, or the entry
// point found by the slab test, placed exactly on the entry face.  ax is the
// entry face's axis (-1 for an origin inside).
__device__ __forceinline__ bool clip_ray(const WalkGrid &G, const double p0[3], const double k[3],
                                         const double inv[3], double &s, double p[3], int &ax)
{
    ax = -1;
    if (inside_closed(G, p0)) {
        s = 0.0;
#pragma unroll
        for (int d = 0; d < 3; d++) p[d] = p0[d];
        return true;
    }
    double tn = -INFINITY, tf = INFINITY;
    bool miss = false;
#pragma unroll
    for (int d = 0; d < 3; d++) {
        const double lo = G.lo[d], hi = G.hi[d];
        if (k[d] == 0.0) {
            if (p0[d] < lo || p0[d] > hi) miss = true;
            continue;
        }
        const double t1 = (lo - p0[d]) * inv[d];
        const double t2 = (hi - p0[d]) * inv[d];
        const double a = t1 < t2 ? t1 : t2;
        const double b = t1 < t2 ? t2 : t1;
        if (a > tn) {
            tn = a;
            ax = d;
        }
        if (b < tf) tf = b;
    }
    if (miss || !(tn < tf) || !(tf > 0.0) || ax < 0) return false;
    s = tn;
#pragma unroll
    for (int d = 0; d < 3; d++) p[d] = entry_coord(G, p0, k, tn, ax, d);
    return true;
}


// Node where the first descent toward q starts: the locate-table cell holding
// q (chosen with the descent's rule for a point on a plane with no tie
// context: the upper side unless the direction's component is negative),
// its reference, level and integer corner; the root without a table.  The
// descent from there takes the same decisions as one from the root: every
// plane above the table level is a cell boundary, and the cell is picked by
// exact comparisons with those planes.
template <int TREE, typename R>
__device__ __forceinline__ R start_node(const WalkGrid &G, const double q[3], const double k[3], int &lv,
                                        uint32_t X[3])
{
    if (G.tdep == 0) {
        lv = 0;
#pragma unroll
        for (int d = 0; d < 3; d++) X[d] = 0u;
        return R(G.root);
    }
    const int T = 1 << G.tdep;
    const double wc = G.tw, scale = G.tscale;
    int c[3];
#pragma unroll
    for (int d = 0; d < 3; d++) {
        int i = int(floor((q[d] - G.lo[d]) * scale));
        i = i < 0 ? 0 : (i > T - 1 ? T - 1 : i);
        // (q - lo) may round: settle the cell by exact comparisons with its planes
        if (i > 0 && q[d] < G.lo[d] + double(i) * wc) i--;
        else if (i < T - 1 && q[d] >= G.lo[d] + double(i + 1) * wc) i++;
        if (i > 0 && q[d] == G.lo[d] + double(i) * wc && k[d] < 0.0) i--;
        c[d] = i;
    }
    const R ref = static_cast<const R *>(G.table)[(int64_t(c[0]) * T + c[1]) * T + c[2]];
    lv = Ref<R>::level(ref);
#pragma unroll
    for (int d = 0; d < 3; d++) {
        const int dep = ref_depth<TREE, R>(ref, lv, d);
        X[d] = (uint32_t(c[d]) >> (G.tdep - dep)) << (G.dm - dep);
    }
    return ref;
}

// Side of a split plane on axis d that holds an exit point lying exactly on
// it (off the plane the comparison decides).  tie bit d: the point lies on
// the low face of the leaf just left, bit 3 + d: on its high face (never set
// for the crossed face's axis); such a plane keeps the point inside that
// leaf's slab.  Otherwise the direction decides, a zero component going to the
// upper side (for the crossed axis this is the side the path moves to).
__device__ __forceinline__ bool tie_upper(int tie, double kd, int d)
{
    const bool onlo = (tie >> d) & 1;
    const bool onhi = (tie >> (3 + d)) & 1;
    return onhi ? false : (onlo ? true : !(kd < 0.0));
}

// The sides of three split planes for a point: up[d] from the comparison,
// replaced by tie_upper where the point lies on the plane (eq[d]).  Such
// points are rare, so the rule is applied behind one wavefront-wide test
// instead of being evaluated for every axis of every descent.
__device__ __forceinline__ void tie_sides(int tie, const double k[3], const bool eq[3], bool up[3])
{
    if (__ballot(eq[0] || eq[1] || eq[2])) {
#pragma unroll
        for (int d = 0; d < 3; d++)
            if (eq[d]) up[d] = tie_upper(tie, k[d], d);
    }
}

// The 32-byte record of leaf id (compact layout): six encoded ropes, then the
// density (f32, or the low and high words of the f64 record's density).  An id
// out of range reads record 0: the crossing reports the error.
__device__ __forceinline__ void load_record(const WalkGrid &G, uint64_t id, uint32_t rec[8])
{
    const uint4 *q = static_cast<const uint4 *>(G.rec) + 2 * (id < G.n_leaves ? id : 0);
    const uint4 a = q[0], b = q[1];
    rec[0] = a.x; rec[1] = a.y; rec[2] = a.z; rec[3] = a.w;
    rec[4] = b.x; rec[5] = b.y; rec[6] = b.z; rec[7] = b.w;
}

// True when the node reference may be descended: an internal node or a twin
// inside the arrays, above the format's depth limit.
template <int TREE, typename R>
__device__ __forceinline__ bool descend_ok(const WalkGrid &G, R ref, int lv)
{
    const uint64_t id = Ref<R>::id(ref);
    const int kind = Ref<R>::kind(ref);
    const uint64_t nc = TREE == OCT ? 8 : 2;
    return lv < 62 && ((kind == Ref<R>::INTERNAL && id < G.n_internal) ||
                       (kind == Ref<R>::TWIN && id + nc <= G.n_leaves));
}

// The side of a k-d node's split plane that holds the point L.p (ties by
// tie_upper), with the move of L.X to that child's corner.
template <int PREC, typename R>
__device__ __forceinline__ bool kd_side(const WalkGrid &G, const LevelGeo &g, Lane<PREC, R> &L)
{
    const uint32_t hw = g.hw;
    const int b = g.axis;
    const uint32_t X0 = in_reg(L.X[0]), X1 = in_reg(L.X[1]), X2 = in_reg(L.X[2]);
    const double q0 = in_reg(L.p[0]), q1 = in_reg(L.p[1]), q2 = in_reg(L.p[2]);
    const uint32_t Xb = b == 0 ? X0 : (b == 1 ? X1 : X2);
    const double qb = b == 0 ? q0 : (b == 1 ? q1 : q2);
    const double lob = b == 0 ? G.lo[0] : (b == 1 ? G.lo[1] : G.lo[2]);
    const double c = fma(double(Xb + hw), G.unit, lob);
    bool up = qb > c;
    const bool eq = qb == c;
    if (__ballot(eq)) {
        const double k0 = in_reg(L.k[0]), k1 = in_reg(L.k[1]), k2 = in_reg(L.k[2]);
        const double kb = b == 0 ? k0 : (b == 1 ? k1 : k2);
        if (eq) up = tie_upper(L.tie, kb, b);
    }
    const uint32_t add = up ? hw : 0u;
    L.X[0] = X0 + (b == 0 ? add : 0u);
    L.X[1] = X1 + (b == 1 ? add : 0u);
    L.X[2] = X2 + (b == 2 ? add : 0u);
    return up;
}

// Up to three k-d levels at once through the jump references.  Levels lv,
// lv+1 and lv+2 split the three axes once each, so the sides of all three
// splits follow from the node's corner alone; the jump reference of those
// sides is the node the descent reaches one to three levels down (it stops
// early at a leaf, or at a twin's leaf child), and only the splits above that
// node move the corner.  Returns the levels descended; a reference whose
// level is not one to three below is replaced by the null reference.
template <int PREC, typename R>
__device__ __forceinline__ int kd_jump(const WalkGrid &G, const LevelGeo *geo, Lane<PREC, R> &L)
{
    const uint64_t id = Ref<R>::id(L.ref);
    const int lv = L.lv;
    const LevelGeo &g = geo[lv];
    const uint32_t jof = g.jof;
    uint32_t idx = 0, jo[3], add[3], h[3];
    bool up[3], eq[3];
#pragma unroll
    for (int d = 0; d < 3; d++) {
        h[d] = g.jhw[d];
        jo[d] = (jof >> (8 * d)) & 3u;
        const double c = fma(double(L.X[d] + h[d]), G.unit, G.lo[d]);
        up[d] = L.p[d] > c;
        eq[d] = L.p[d] == c;
    }
    tie_sides(L.tie, L.k, eq, up);
#pragma unroll
    for (int d = 0; d < 3; d++) {
        idx |= (up[d] ? 4u : 0u) >> jo[d];
        add[d] = up[d] ? h[d] : 0u;
    }
    R r = static_cast<const R *>(G.jump)[8 * id + idx];
    int dl = Ref<R>::level(r) - lv;
    const bool ok = (dl >= 1) & (dl <= 3);
    r = ok ? r : Ref<R>::NUL;
    dl = ok ? dl : 0;
#pragma unroll
    for (int d = 0; d < 3; d++) L.X[d] += int(jo[d]) < dl ? add[d] : 0u;
    L.lv = lv + dl;
    L.ref = r;
    return dl;
}

// A descent from the internal or twin node L.ref toward the point L.p: the
// child holding it, with its corner and level.  A twin's children are leaves
// whose ranks follow its own; an internal node's child reference is read from
// the child array, or a k-d node's reference up to three levels down from the
// jump array when the grid has one.  Returns the levels descended.
template <int TREE, int PREC, typename R>
__device__ __forceinline__ int descend_step(const WalkGrid &G, const LevelGeo *geo, Lane<PREC, R> &L)
{
    const bool tw = Ref<R>::twin(L.ref);
    if (TREE == KD && G.jump != nullptr && !tw) return kd_jump<PREC, R>(G, geo, L);
    const uint64_t id = Ref<R>::id(L.ref);
    LevelGeo gk;
    if (TREE == KDG) gk = ref_geo(G, L.ref);   // the node's own axis and half width
    const LevelGeo &g = TREE == KDG ? gk : geo[L.lv];
    const uint32_t hw = g.hw;
    uint32_t slot;
    if (TREE != OCT) {
        slot = kd_side(G, g, L) ? 1u : 0u;
    } else {
        slot = 0;
        bool up[3], eq[3];
#pragma unroll
        for (int d = 0; d < 3; d++) {
            const double c = fma(double(L.X[d] + hw), G.unit, G.lo[d]);
            up[d] = L.p[d] > c;
            eq[d] = L.p[d] == c;
        }
        tie_sides(L.tie, L.k, eq, up);
#pragma unroll
        for (int d = 0; d < 3; d++) {
            slot |= (up[d] ? 1u : 0u) << d;
            L.X[d] += up[d] ? hw : 0u;
        }
    }
    L.lv = L.lv + 1;
    if (tw && TREE == KDG) {
        // the leaf child's halvings: the twin's, one more across its split axis
        const int a = g.axis;
        const int dx = Ref<R>::depth(L.ref, 0) + (a == 0 ? 1 : 0);
        const int dy = Ref<R>::depth(L.ref, 1) + (a == 1 ? 1 : 0);
        L.ref = Ref<R>::make_geo(Ref<R>::LEAF, L.lv, id + slot, dx, dy, 3);
    } else if (tw) {
        L.ref = Ref<R>::make(Ref<R>::LEAF, L.lv, id + slot);
    } else {
        const uint64_t nc = TREE == OCT ? 8 : 2;
        L.ref = static_cast<const R *>(G.child)[nc * id + slot];
    }
    return 1;
}

// Records of the one-thread walk: staged four at a time and written as aligned
// 16-byte vectors once a group of four positions (pos = 4m .. 4m+3 of the
// record arrays, which must be 16-byte aligned) is complete; the partial
// groups at the two ends of a path's slice are written element by element.
template <int PREC>
__device__ __forceinline__ void store_one(const WalkArgs &A, int64_t pos, uint32_t id, double ds)
{
    A.leaf[pos] = int32_t(id);
    if (PREC == HG_FP64) reinterpret_cast<double *>(A.ds)[pos] = ds;
    else reinterpret_cast<float *>(A.ds)[pos] = float(ds);
}

template <int PREC, typename R>
__device__ __forceinline__ void stage_record(const WalkArgs &A, Lane<PREC, R> &L, int64_t pos, uint32_t id,
                                             double ds)
{
    L.sl[0] = L.sl[1]; L.sl[1] = L.sl[2]; L.sl[2] = L.sl[3]; L.sl[3] = id;
    L.sd[0] = L.sd[1]; L.sd[1] = L.sd[2]; L.sd[2] = L.sd[3];
    L.sd[3] = typename Lane<PREC, R>::DsT(ds);
    if ((pos & 3) != 3) return;
    const int64_t g = pos - 3;
    if (g >= L.base) {
        *reinterpret_cast<uint4 *>(A.leaf + g) = make_uint4(L.sl[0], L.sl[1], L.sl[2], L.sl[3]);
        if (PREC == HG_FP64) {
            double2 *d = reinterpret_cast<double2 *>(reinterpret_cast<double *>(A.ds) + g);
            d[0] = make_double2(L.sd[0], L.sd[1]);
            d[1] = make_double2(L.sd[2], L.sd[3]);
        } else {
            *reinterpret_cast<float4 *>(reinterpret_cast<float *>(A.ds) + g) =
                make_float4(L.sd[0], L.sd[1], L.sd[2], L.sd[3]);
        }
    } else {
#pragma unroll
        for (int j = 0; j < 4; j++)
            if (g + j >= L.base) store_one<PREC>(A, g + j, L.sl[j], L.sd[j]);
    }
}

// Write the staged records of an unfinished group at the end of a path.
template <int PREC, typename R>
__device__ __forceinline__ void flush_records(const WalkArgs &A, const Lane<PREC, R> &L)
{
    if (L.cnt == 0) return;
    const int64_t last = L.base + (L.cnt < L.room ? L.cnt : L.room) - 1;
    const int ph = int(last & 3);
    if (ph == 3) return;
#pragma unroll
    for (int j = 0; j < 3; j++) {
        const int64_t pos = last - j;
        if (j <= ph && pos >= L.base) store_one<PREC>(A, pos, L.sl[3 - j], L.sd[3 - j]);
    }
}

// Slab walk: the state on entry to the leaf of the path's first record beyond
// its row, from which the record-filling walk resumes it.  The slab walk
// reaches that point once per path, so the entries never exceed the paths.
// Entries are taken from a counter, or (resume_by_path) entry i is path i's:
// no atomic on one address per overflowing path, which serialises when many
// paths overflow short rows.
template <int PREC, typename R>
__device__ __forceinline__ void save_resume(const WalkArgs &A, int64_t path, const Lane<PREC, R> &L)
{
    if (!A.resume) return;   // a slab walk that only counts (the autotuner's)
    unsigned long long j = (unsigned long long)path;
    if (!A.resume_by_path) {
        j = atomicAdd(A.n_resume, 1ull);
        if (j >= (unsigned long long)A.n) return;
    }
    Resume &S = A.resume[j];
#pragma unroll
    for (int d = 0; d < 3; d++) {
        S.p[d] = L.p[d];
        S.X[d] = L.X[d];
    }
    S.s = L.s;
    S.lv = L.lv;
    S.ref = uint64_t(L.ref);
    S.path = path;
    S.steps = L.steps;
    S.pad = 0;
}

// One crossing of the leaf L.ref: exit face and ds, tau, the record,
// re-anchoring, and the rope target of the exit face (left in L.ref, with its
// level and corner, for the next step).  sl / sd (LSLOT): the lane's record
// slots in LDS, sgm their index mask; else records are staged in registers.
template <int TREE, int PREC, int WM, typename R, bool LSLOT>
__device__ __forceinline__ int cross(const WalkGrid &G, const WalkArgs &A, const LevelGeo *geo,
                                     Lane<PREC, R> &L, int64_t path, unsigned long long &rechecks,
                                     uint32_t *sl, typename Lane<PREC, R>::DsT *sd)
{
    using DsT = typename Lane<PREC, R>::DsT;
    const uint64_t id = Ref<R>::id(L.ref);
    bool err = !(id < G.n_leaves);
    // the record is read first: its load overlaps the exit decision
    uint32_t rec[8];
    if (sizeof(R) == 4) load_record(G, id, rec);
    LevelGeo gk;
    if (TREE == KDG) gk = ref_geo(G, L.ref);   // the leaf's widths from its reference
    const LevelGeo &g = TREE == KDG ? gk : geo[L.lv];
    double lo[3], hi[3], E[3];
    bool kp[3];
#pragma unroll
    for (int d = 0; d < 3; d++) {
        lo[d] = fma(double(L.X[d]), G.unit, G.lo[d]);   // exact: a plane of the grid
        hi[d] = lo[d] + g.w[d];
        kp[d] = L.k[d] > 0.0;
        E[d] = kp[d] ? hi[d] : lo[d];                    // the face the path moves toward
    }
    // exit axis: the lowest axis of the smallest t = |E - p| |1/k| (a zero
    // direction component gives +inf or NaN, which never wins)
    bool a0, a1;
    double ds;
    if (PREC == HG_FP64) {
        double t[3];
#pragma unroll
        for (int d = 0; d < 3; d++) t[d] = fabs(E[d] - L.p[d]) * L.ainv[d];
        const double m = min64(t[0], min64(t[1], t[2]));
        a0 = t[0] == m;
        a1 = !a0 & (t[1] == m);
        ds = m;
    } else {
        double D[3];
        float t32[3];
#pragma unroll
        for (int d = 0; d < 3; d++) {
            D[d] = E[d] - L.p[d];
            t32[d] = fabsf(float(D[d])) * L.ainv32[d];
        }
        const float m1 = fminf(t32[0], fminf(t32[1], t32[2]));
        a0 = t32[0] == m1;
        a1 = !a0 & (t32[1] == m1);
        // near tie: a second exit distance within the guard of the smallest
        const float lim = m1 + g.guard;
        const bool c0 = t32[0] < lim, c1 = t32[1] < lim, c2 = t32[2] < lim;
        const bool recheck = L.force64 | (c0 & c1) | (c0 & c2) | (c1 & c2);
        if (__ballot(recheck)) {
            if (recheck) {
                rechecks++;
                double t[3];
#pragma unroll
                for (int d = 0; d < 3; d++) t[d] = fabs(D[d]) * L.ainv[d];
                const double m = min64(t[0], min64(t[1], t[2]));
                a0 = t[0] == m;
                a1 = !a0 & (t[1] == m);
            }
        }
        // FP64 exit distance of the chosen axis only
        const double D0 = in_reg(D[0]), D1 = in_reg(D[1]), D2 = in_reg(D[2]);
        const double i0 = in_reg(L.ainv[0]), i1 = in_reg(L.ainv[1]), i2 = in_reg(L.ainv[2]);
        const double Da = a0 ? D0 : (a1 ? D1 : D2);
        const double ia = a0 ? i0 : (a1 ? i1 : i2);
        ds = fabs(Da) * ia;
    }
    err = err | !(ds <= 1.0e300);
    const bool a2 = !a0 & !a1;
    const bool up = a0 ? kp[0] : (a1 ? kp[1] : kp[2]);
    // the leaf record: rope of the exit face, density
    R nref;
    float rho32;
    double rho64;
    if (sizeof(R) == 4) {
        const uint32_t r0 = in_reg(rec[0]), r1 = in_reg(rec[1]), r2 = in_reg(rec[2]);
        const uint32_t r3 = in_reg(rec[3]), r4 = in_reg(rec[4]), r5 = in_reg(rec[5]);
        const uint32_t rl = a0 ? r0 : (a1 ? r2 : r4);
        const uint32_t rh = a0 ? r1 : (a1 ? r3 : r5);
        nref = R(up ? rh : rl);
        rho32 = __uint_as_float(rec[6]);
        rho64 = __hiloint2double(int(rec[7]), int(rec[6]));
    } else {
        const char *rec = static_cast<const char *>(G.rec) + (err ? 0 : id) * 64;
        const int face = 2 * (a0 ? 0 : (a1 ? 1 : 2)) + (up ? 1 : 0);
        nref = reinterpret_cast<const R *>(rec)[face];
        rho64 = *reinterpret_cast<const double *>(rec + 48);
        rho32 = *reinterpret_cast<const float *>(rec + 56);
    }
    if (ds > 0.0) {
        if (WM == WM_FILL || WM == WM_SLAB) {
            if (L.cnt < L.room) {
                if (LSLOT) {
                    sl[L.cnt & (SG - 1)] = uint32_t(id);
                    sd[L.cnt & (SG - 1)] = DsT(ds);
                } else {
                    stage_record<PREC, R>(A, L, L.base + L.cnt, uint32_t(id), ds);
                }
            } else if (WM == WM_FILL) {
                err = true;   // the fill walk must repeat the counting walk
            } else if (L.cnt == L.room) {
                // records beyond the row are left to the fill walk, which resumes here
                save_resume<PREC, R>(A, path, L);
            }
        }
        if (PREC != HG_FP64 && WM != WM_FILL && WM != WM_SEG && WM != WM_INT) {
            const float y = float(A.kappa) * rho32 * float(ds) - L.comp32;
            const float t = L.tau32 + y;
            L.comp32 = (t - L.tau32) - y;
            L.tau32 = t;
        }
        if (WM != WM_SEG && WM != WM_INT) L.cnt++;
    }
    // FP64 tau: a zero-length step adds an exact zero
    if (PREC == HG_FP64 && WM != WM_FILL && WM != WM_SEG && WM != WM_INT)
        L.tau64 = L.tau64 + A.kappa * rho64 * ds;
    bool stop = false;
    if (WM == WM_SEG) {
        // the first lim of the path: a leaf entered at s >= lim adds nothing, the
        // leaf holding s = lim adds its part up to there, and the walk stops there
        if ((L.s < L.lim) & (ds > 0.0)) {
            L.tau64 = L.tau64 + A.kappa * rho64 * min64(ds, L.lim - L.s);
            L.cnt++;
        }
        stop = !(L.s + ds < L.lim);
    } else if (WM == WM_INT) {
        // the first leaf where the cumulative tau reaches tau* = lim; tau grows
        // linearly inside it, which places the point
        if (ds > 0.0) {
            const double dt = A.kappa * rho64 * ds;
            if ((L.tau64 + dt >= L.lim) & (dt > 0.0)) {
                L.cnt = int32_t(id);
                L.lim = L.s + (L.lim - L.tau64) / (A.kappa * rho64);
                stop = true;
            } else {
                L.tau64 = L.tau64 + dt;
            }
        }
    }
    // the exit face lies on the domain boundary: its rope is null and the path ends
    const bool end = (nref == Ref<R>::NUL) | stop;
    // re-anchor the exit point on the crossed face
    L.s = L.s + ds;
    double q[3];
    bool hit = false;
#pragma unroll
    for (int d = 0; d < 3; d++) {
        const bool isa = d == 0 ? a0 : (d == 1 ? a1 : a2);
        const double v = L.p0[d] + L.s * L.k[d];
        const double c = min64(max64(v, lo[d]), hi[d]);
        q[d] = isa ? E[d] : c;
        hit = hit | (!isa & ((c == lo[d]) | (c == hi[d])));
    }
    // tie context of the descent from the rope target (rare: an exit point on
    // an edge of the leaf)
    int tie = 0;
    if (__ballot(hit)) {
#pragma unroll
        for (int d = 0; d < 3; d++) {
            const bool isa = d == 0 ? a0 : (d == 1 ? a1 : a2);
            tie |= int(!isa & (q[d] == lo[d])) << d;
            tie |= int(!isa & (q[d] == hi[d])) << (3 + d);
        }
    }
    L.tie = tie;
    // Corner of the rope target: the leaf's corner moved across the exit face
    // and aligned down to the target's cell size.  The target is never finer
    // than the leaf across the face except along the exit axis, where it may
    // be the half of a same-size neighbour touching the face.
    const int nlv = Ref<R>::level(nref);
    LevelGeo gkn;
    if (TREE == KDG) gkn = ref_geo(G, nref);
    const LevelGeo &gn = TREE == KDG ? gkn : geo[nlv];
#pragma unroll
    for (int d = 0; d < 3; d++) {
        const bool isa = d == 0 ? a0 : (d == 1 ? a1 : a2);
        const uint32_t Wn = gn.W[d];
        const uint32_t delta = isa ? (kp[d] ? g.W[d] : 0u - Wn) : 0u;
        L.X[d] = (L.X[d] + delta) & (0u - Wn);
        L.p[d] = q[d];
    }
    L.lv = nlv;
    L.ref = nref;

    return err ? STEP_ERR : (end ? STEP_END : STEP_GO);
}

template <int PREC, int WM, typename R, bool STG>
__device__ __forceinline__ void finish_path(const WalkArgs &A, int64_t i, const Lane<PREC, R> &L)
{
    if (WM == WM_FILL) {
        if (!STG) flush_records<PREC, R>(A, L);
        if (L.cnt != L.room) A.st->step_guard = 1;
        return;
    }
    if (WM == WM_SLAB && !STG) flush_records<PREC, R>(A, L);
    A.count[i] = L.cnt;
    if (WM == WM_INT) A.tau[i] = L.cnt >= 0 ? L.lim : L.s;
    else if (PREC == HG_FP64 || WM == WM_SEG) A.tau[i] = L.tau64;
    else A.tau[i] = double(L.tau32) - double(L.comp32);
}

template <int PREC, int WM>
__device__ __forceinline__ void finish_unwalked(const WalkArgs &A, int64_t i, int why)
{
    if (WM == WM_FILL) return;
    A.count[i] = WM == WM_INT ? -1 : 0;
    if (why == PATH_BAD_DIR) {
        A.tau[i] = __longlong_as_double(0x7ff8000000000000ll);
        A.st->bad_dir = 1;
    } else {
        A.tau[i] = 0.0;
    }
}

// Inverse direction |1/k| and the FP64-decision flag of direction k (the FP32
// exit decision is used only where its error bound holds).
__device__ __forceinline__ void inverse_dir(const double k[3], double ainv[3], bool &force64)
{
    force64 = false;
#pragma unroll
    for (int d = 0; d < 3; d++) {
        ainv[d] = fabs(1.0 / k[d]);
        if (k[d] != 0.0 && !(fabs(k[d]) >= 1e-30)) force64 = true;
    }
}

// Prepare path i: direction check, inverse direction, entry point and the
// node of its first descent.
template <int TREE, typename R>
__device__ __forceinline__ int prep_path(const WalkGrid &G, const WalkArgs &A, int64_t i, Prep &e)
{
    double p0[3], k[3], inv[3], p[3], s;
#pragma unroll
    for (int d = 0; d < 3; d++) {
        p0[d] = A.O[3 * i + d];
        k[d] = A.K[3 * i + d];
    }
    const double nn = k[0] * k[0] + k[1] * k[1] + k[2] * k[2];
    const bool finite = isfinite(k[0]) && isfinite(k[1]) && isfinite(k[2]);
    if (!finite || !(fabs(sqrt(nn) - 1.0) <= 1e-6)) return PATH_BAD_DIR;
    bool f64;
    inverse_dir(k, e.ainv, f64);
#pragma unroll
    for (int d = 0; d < 3; d++) inv[d] = 1.0 / k[d];
    int ax;
    if (!clip_ray(G, p0, k, inv, s, p, ax)) return PATH_MISS;
    int lv;
    e.ref = uint64_t(start_node<TREE, R>(G, p, k, lv, e.X));
    e.s = s;
    e.lvf = uint32_t(lv) | (uint32_t(ax + 1) << 8) | (f64 ? (1u << 12) : 0u);
    e.idx = int32_t(i);
    e.pad = 0;
    return PATH_WALK;
}

// Prepare resume entry j of the record-filling walk.
__device__ __forceinline__ void prep_resume(const WalkArgs &A, int64_t j, Prep &e)
{
    const int64_t i = A.resume[j].path;
    double k[3];
#pragma unroll
    for (int d = 0; d < 3; d++) k[d] = A.K[3 * i + d];
    bool f64;
    inverse_dir(k, e.ainv, f64);
    e.s = 0.0;
    e.X[0] = e.X[1] = e.X[2] = 0u;
    e.lvf = f64 ? (1u << 12) : 0u;
    e.ref = 0;
    e.idx = int32_t(j);
    e.pad = 0;
}

// A lane takes up a prepared path: returns its path index.
template <int WM, int PREC, typename R>
__device__ __forceinline__ int64_t take_path(const WalkGrid &G, const WalkArgs &A, const Prep &e,
                                             Lane<PREC, R> &L)
{
    const bool resumed = WM == WM_FILL && A.resume;
    int64_t i = e.idx;
    if (resumed) {
        const Resume &S = A.resume[e.idx];
        i = S.path;
#pragma unroll
        for (int d = 0; d < 3; d++) {
            L.p[d] = S.p[d];
            L.X[d] = S.X[d];
        }
        L.s = S.s;
        L.ref = R(S.ref);
        L.lv = S.lv;
        L.steps = S.steps;
    }
#pragma unroll
    for (int d = 0; d < 3; d++) {
        L.p0[d] = A.O[3 * i + d];
        L.k[d] = A.K[3 * i + d];
        L.ainv[d] = e.ainv[d];
        L.ainv32[d] = float(e.ainv[d]);
    }
    L.force64 = (e.lvf >> 12) & 1u;
    if (!resumed) {
        const int ax = int((e.lvf >> 8) & 15u) - 1;
        L.s = e.s;
        if (ax < 0) {
#pragma unroll
            for (int d = 0; d < 3; d++) L.p[d] = L.p0[d];
        } else {
#pragma unroll
            for (int d = 0; d < 3; d++) L.p[d] = entry_coord(G, L.p0, L.k, e.s, ax, d);
        }
#pragma unroll
        for (int d = 0; d < 3; d++) L.X[d] = e.X[d];
        L.ref = R(e.ref);
        L.lv = int(e.lvf & 255u);
        L.steps = 0;
    }
    L.tie = 0;
    L.cnt = WM == WM_INT ? -1 : 0;
    L.tau64 = 0.0;
    L.tau32 = 0.f;
    L.comp32 = 0.f;
    if (WM == WM_SEG || WM == WM_INT) L.lim = A.lim[i];
    if (WM == WM_FILL) {
        L.base = A.offsets[i] + (resumed ? A.slab : 0);
        L.room = A.offsets[i + 1] - L.base;
    } else if (WM == WM_SLAB) {
        L.base = i * A.slab;
        L.room = A.slab;
    }
    return i;
}

// One lane per path, the whole walk in one loop.
template <int TREE, int PREC, int WM, typename R>
__global__ void __launch_bounds__(TB) k_walk(WalkGrid G, WalkArgs A)
{
    __shared__ LevelGeo geo[NLEV];
    fill_levels(geo, G, threadIdx.x, TB);
    __syncthreads();
    const int64_t q = int64_t(blockIdx.x) * TB + threadIdx.x;
    if (q >= A.n) return;
    Prep e;
    if (WM == WM_FILL && A.resume) {
        prep_resume(A, q, e);
    } else {
        const int why = prep_path<TREE, R>(G, A, q, e);
        if (why != PATH_WALK) {
            finish_unwalked<PREC, WM>(A, q, why);
            return;
        }
    }
    Lane<PREC, R> L;
    const int64_t i = take_path<WM, PREC, R>(G, A, e, L);
    unsigned long long rechecks = 0;
    uint32_t desc = 0;   // descent levels
    for (;;) {
        if (Ref<R>::leaf(L.ref)) {
            const int r = cross<TREE, PREC, WM, R, false>(G, A, geo, L, i, rechecks, nullptr, nullptr);
            if (r == STEP_ERR || ++L.steps >= STEP_GUARD) {
                A.st->step_guard = 1;
                break;
            }
            if (r == STEP_END) break;
        } else {
            if (!descend_ok<TREE, R>(G, L.ref, L.lv)) {
                A.st->bad_ref = 1;
                break;
            }
            desc += descend_step<TREE, PREC, R>(G, geo, L);
        }
    }
    finish_path<PREC, WM, R, false>(A, i, L);
    if (!(WM == WM_FILL) && A.count_rechecks) {
        if (rechecks) atomicAdd(&A.st->rechecks, rechecks);
        if (desc) atomicAdd(&A.st->descents, (unsigned long long)desc);
    }
}

// Records staged in LDS by the persistent and batched walks (record modes):
// each lane owns SG slots of leaf ids and SG of ds (rows of SG + 1 words
// against bank conflicts).  A lane's group is written out once it holds SG
// records, its row or slice is full or its path ends, by the whole
// wavefront: SG lanes per group, 64 / SG groups per store instruction, so
// that a store covers a few cache lines instead of one line per lane.
constexpr int SP = SG + 1;

// Write the groups of the lanes with nr > 0: records pos .. pos+nr-1 of the
// output come from slots 0 .. nr-1 of that lane (into the rows of (leaf, ds)
// pairs when A.pairs is set).  Wavefront-uniform; wbase is the wavefront's
// first thread in the block.
template <typename DsT>
__device__ __forceinline__ void flush_stage(const WalkArgs &A, const uint32_t *stl, const DsT *stds, int nr,
                                            int64_t pos, int lane, int wbase)
{
    constexpr int PER = 64 / SG;
    uint64_t fm = __ballot(nr > 0);
    if (!fm) return;
    __builtin_amdgcn_wave_barrier();
    const int g = lane / SG, j = lane % SG;
    while (fm) {
        int src = -1;
#pragma unroll
        for (int k = 0; k < PER; k++) {
            const int b = fm ? __builtin_ctzll(fm) : -1;
            if (k == g) src = b;
            fm &= fm - 1;
        }
        const int s = src < 0 ? 0 : src;
        const int rr = __shfl(nr, s, 64);
        const int plo = __shfl(int(uint64_t(pos) & 0xffffffffu), s, 64);
        const int phi = __shfl(int(uint64_t(pos) >> 32), s, 64);
        const int64_t pp = int64_t((uint64_t(uint32_t(phi)) << 32) | uint32_t(plo));
        if (src >= 0 && j < rr) {
            const int t = (wbase + s) * SP + j;
            if (sizeof(DsT) == 4 && A.pairs) {
                reinterpret_cast<uint2 *>(A.leaf)[pp + j] = make_uint2(stl[t], __float_as_uint(float(stds[t])));
            } else {
                A.leaf[pp + j] = int32_t(stl[t]);
                static_cast<DsT *>(A.ds)[pp + j] = stds[t];
            }
        }
    }
}

// The group of LDS-staged records a lane writes out after a step: complete
// (SG records), the row or slice full, or the last records of an ended path.
template <int PREC, typename R>
__device__ __forceinline__ void stage_group(const Lane<PREC, R> &L, bool crossed, int32_t c_before, bool ended,
                                            int &nr, int64_t &pos)
{
    const int64_t c = L.cnt < L.room ? L.cnt : L.room;
    const bool wrote = crossed && L.cnt > c_before && c_before < L.room;
    nr = 0;
    if (wrote && ((c & (SG - 1)) == 0 || c == L.room)) nr = int(((c - 1) & (SG - 1)) + 1);
    else if (ended && c != L.room) nr = int(c & (SG - 1));
    pos = L.base + c - nr;
}

// One step of a busy lane: a crossing if its node is a leaf, then (if the path
// goes on into a node that is not a leaf) one descent level.  Returns true
// when the path ended (or failed); crossed / c_before / bad describe the step
// for the record staging.
template <int TREE, int PREC, int WM, typename R, bool STG>
__device__ __forceinline__ bool walk_step(const WalkGrid &G, const WalkArgs &A, const LevelGeo *geo,
                                          Lane<PREC, R> &L, int64_t ray, unsigned long long &rechecks,
                                          uint32_t &desc, uint32_t *my_l, typename Lane<PREC, R>::DsT *my_d,
                                          bool &crossed, int32_t &c_before, bool &bad)
{
    int r = STEP_GO;
    crossed = false;
    bad = false;
    c_before = L.cnt;
    if (Ref<R>::leaf(L.ref)) {
        r = cross<TREE, PREC, WM, R, STG>(G, A, geo, L, ray, rechecks, my_l, my_d);
        crossed = true;
        if (r == STEP_ERR || ++L.steps >= STEP_GUARD) {
            A.st->step_guard = 1;
            r = STEP_ERR;
        }
    }
    if (r == STEP_GO && !Ref<R>::leaf(L.ref)) {
        if (!descend_ok<TREE, R>(G, L.ref, L.lv)) {
            bad = true;
        } else {
            desc += descend_step<TREE, PREC, R>(G, geo, L);
        }
    }
    return bad || r != STEP_GO;
}

// Fill the wavefront's queue with the prepared paths among [cnext, cnext+64)
// of [cnext, cend) (all lanes take part); paths that miss the domain or have
// an invalid direction are finished here.  Returns the number queued.
template <int TREE, int PREC, int WM, typename R>
__device__ __forceinline__ int fill_queue(const WalkGrid &G, const WalkArgs &A, Prep *ring, int64_t cnext,
                                          int64_t cend, int lane, uint64_t below)
{
    const int64_t i = cnext + lane;
    Prep e;
    bool ok = false;
    if (i < cend) {
        if (WM == WM_FILL && A.resume) {
            // entries by path: only the paths past their row are resumed
            ok = !A.resume_by_path || A.count[i] > A.slab;
            if (ok) prep_resume(A, i, e);
        } else {
            const int why = prep_path<TREE, R>(G, A, i, e);
            ok = why == PATH_WALK;
            if (!ok) finish_unwalked<PREC, WM>(A, i, why);
        }
    }
    const uint64_t okm = __ballot(ok);
    if (ok) ring[__popcll(okm & below)] = e;
    // the entries are read by other lanes of the same wavefront
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    return __popcll(okm);
}

__device__ __forceinline__ unsigned long long readfirstlane64(unsigned long long v)
{
    return (unsigned long long)__builtin_amdgcn_readfirstlane(uint32_t(v)) |
           ((unsigned long long)__builtin_amdgcn_readfirstlane(uint32_t(v >> 32)) << 32);
}

// Chunk sources of the persistent loop (wavefront-uniform; lane 0 takes the
// atomic).  PathCounter: `chunk` paths per atomic on the launch's path counter.
struct PathCounter {
    uint32_t chunk;
    __device__ __forceinline__ bool next(const WalkArgs &A, int lane, int64_t &b, int64_t &e) const
    {
        unsigned long long v = 0;
        if (lane == 0) v = atomicAdd(&A.st->next_ray, (unsigned long long)chunk);
        v = readfirstlane64(v);
        if (v >= (unsigned long long)A.n) return false;
        b = int64_t(v);
        e = std::min<int64_t>(b + chunk, A.n);
        return true;
    }
};

// GridChunks: the chunks of one grid of a batched walk, one per atomic on
// that grid's counter.
struct GridChunks {
    const BatchChunk *chunks;
    unsigned long long *ctr;
    int64_t c0, nq;
    __device__ __forceinline__ bool next(const WalkArgs &, int lane, int64_t &b, int64_t &e) const
    {
        unsigned long long t = 0;
        if (lane == 0) t = atomicAdd(ctr, 1ull);
        t = readfirstlane64(t);
        if (t >= (unsigned long long)nq) return false;
        b = chunks[c0 + int64_t(t)].start;
        e = chunks[c0 + int64_t(t)].end;
        return true;
    }
};

// The persistent loop of one wavefront over one grid: it takes chunks of
// paths from src (starting with [cnext, cend) if not empty), prepares them
// 64 at a time into its LDS queue, and hands queued paths to lanes whose path
// ended once at least refill_min lanes are idle (or none is busy).  Each
// iteration a busy lane crosses its leaf and, if the path goes on into a node
// that is not a leaf, descends.  Returns when src is exhausted and every lane
// is idle.
template <int TREE, int PREC, int WM, typename R, class Src>
__device__ __forceinline__ void persistent_loop(const WalkGrid &G, const WalkArgs &A, const LevelGeo *geo,
                                                Prep *ring, uint32_t *stl, typename Lane<PREC, R>::DsT *stds,
                                                const Src &src, int64_t cnext, int64_t cend, int refill_min,
                                                int lane, int wid, unsigned long long &rechecks, uint32_t &desc)
{
    using DsT = typename Lane<PREC, R>::DsT;
    constexpr bool STG = WM == WM_FILL || WM == WM_SLAB;   // record modes
    uint32_t *my_l = STG ? stl + threadIdx.x * SP : nullptr;
    DsT *my_d = STG ? stds + threadIdx.x * SP : nullptr;
    const uint64_t below = lane ? (~0ull >> (64 - lane)) : 0ull;
    Lane<PREC, R> L;
    int64_t ray = -1;
    bool done = false;
    int rhead = 0, rn = 0;           // the wavefront's queue [rhead, rn)
    bool drained = false;            // src is exhausted
    for (;;) {
        const bool want = ray < 0 && !done;
        const uint64_t wmask = __ballot(want);
        if (wmask) {
            const uint64_t amask = __ballot(ray >= 0);
            const int nwant = __popcll(wmask);
            if (nwant >= refill_min || !amask) {
                while (rhead >= rn && !(drained && cnext >= cend)) {
                    if (cnext >= cend) {
                        if (!src.next(A, lane, cnext, cend)) drained = true;
                        continue;
                    }
                    rn = fill_queue<TREE, PREC, WM, R>(G, A, ring, cnext, cend, lane, below);
                    rhead = 0;
                    cnext = std::min<int64_t>(cnext + 64, cend);
                }
                const int avail = rn - rhead;
                if (want) {
                    const int rank = __popcll(wmask & below);
                    if (rank < avail) ray = take_path<WM, PREC, R>(G, A, ring[rhead + rank], L);
                    else if (drained && cnext >= cend) done = true;
                }
                rhead += std::min(avail, nwant);
            }
        }
        if (!__ballot(ray >= 0) && !__ballot(!done)) break;
        bool fin = false, crossed = false, bad = false;
        int32_t c_before = 0;
        if (ray >= 0)
            fin = walk_step<TREE, PREC, WM, R, STG>(G, A, geo, L, ray, rechecks, desc, my_l, my_d, crossed,
                                                    c_before, bad);
        if (STG) {
            int nr = 0;
            int64_t pos = 0;
            if (ray >= 0 && (crossed || bad)) stage_group<PREC, R>(L, crossed, c_before, fin, nr, pos);
            flush_stage<DsT>(A, stl, stds, nr, pos, lane, wid * 64);
        }
        if (fin) {
            if (bad) A.st->bad_ref = 1;
            finish_path<PREC, WM, R, STG>(A, ray, L);
            ray = -1;
        }
    }
}

// Persistent walk of one grid: every wavefront runs the persistent loop with
// `chunk` paths per atomic on the launch's path counter.
// Five wavefronts per SIMD for the walks without records (their registers
// fit 96 without spilling: more paths in flight hide more load latency); the
// record walks keep the compiler's choice.
template <int TREE, int PREC, int WM, typename R, int BT>
__global__ void __launch_bounds__(BT)
    __attribute__((amdgpu_waves_per_eu(WM == WM_FILL || WM == WM_SLAB ? 1 : 5, 8)))
    k_walk_persistent(WalkGrid G, WalkArgs A, uint32_t chunk, int refill_min)
{
    using DsT = typename Lane<PREC, R>::DsT;
    constexpr bool STG = WM == WM_FILL || WM == WM_SLAB;   // record modes
    constexpr int NW = BT / 64;
    __shared__ LevelGeo geo[NLEV];
    __shared__ Prep ring_all[NW * RING];
    __shared__ uint32_t stl[STG ? BT * SP : 1];
    __shared__ DsT stds[STG ? BT * SP : 1];
    fill_levels(geo, G, threadIdx.x, BT);
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    unsigned long long rechecks = 0;
    uint32_t desc = 0;
    persistent_loop<TREE, PREC, WM, R>(G, A, geo, ring_all + wid * RING, stl, stds, PathCounter{chunk}, 0, 0,
                                       refill_min, lane, wid, rechecks, desc);
    if (!(WM == WM_FILL) && A.count_rechecks) {
        if (rechecks) atomicAdd(&A.st->rechecks, rechecks);
        if (desc) atomicAdd(&A.st->descents, (unsigned long long)desc);
    }
}

// Batched walk over many grids in one persistent launch.  The device work
// queue is a table of chunks (grid, path range), each grid's chunks together
// with a counter per grid, and the grids grouped in classes that share a
// per-level table.  A block works through the classes one at a time (in an
// order rotated by its index) with one level table in LDS: for each class it
// makes the table, then each wavefront starts on a grid of the class spread
// by its index and runs the persistent loop over that grid's chunks, moving
// on to the class's next grid with chunks left once its lanes are idle; the
// block meets at a barrier before the next class's table.  While on a grid a
// wavefront holds the grid's parameters as wavefront-uniform values.
template <int PREC, int WM, int BT>
__device__ __forceinline__ void walk_batched(const WalkGrid *__restrict__ grids, const WalkArgs *__restrict__ args,
                                             const BatchQueue Q, int refill_min, TraceStatus *st, LevelGeo *geo,
                                             Prep *ring_all, uint32_t *stl,
                                             typename Lane<PREC, uint32_t>::DsT *stds)
{
    using R = uint32_t;
    // a resume walk with no path saved past its row has nothing to do
    if (WM == WM_FILL && args[0].resume && args[0].resume_by_path && !st->resumed) return;
    const int lane = threadIdx.x & 63;
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    Prep *ring = ring_all + wid * RING;
    unsigned long long rechecks = 0;
    uint32_t desc = 0;
    bool count_rechecks = false;
    const int64_t gw = int64_t(blockIdx.x) * (BT / 64) + wid, tw = int64_t(gridDim.x) * (BT / 64);
    for (int k = 0; k < Q.ncls; k++) {
        const int c = int((blockIdx.x + unsigned(k)) % unsigned(Q.ncls));
        const int c0g = Q.cpre[c], ncg = Q.cpre[c + 1] - c0g;
        __syncthreads();   // the previous class's walks no longer read the table
        fill_levels(geo, grids[Q.cgrid[c0g]], threadIdx.x, BT);
        __syncthreads();
        int qi = __builtin_amdgcn_readfirstlane(int(gw * ncg / tw));   // the class's grid it takes chunks of
        int tried = 0;   // grids of the class found empty since its last chunk
        for (;;) {
            const int qg = __builtin_amdgcn_readfirstlane(Q.cgrid[c0g + qi]);
            unsigned long long t = 0;
            if (lane == 0) t = atomicAdd(&Q.gctr[qg], 1ull);
            t = readfirstlane64(t);
            const int64_t c0 = Q.gpre[qg], nq = Q.gpre[qg + 1] - c0;
            if (t >= (unsigned long long)nq) {
                if (++tried >= ncg) break;
                qi = qi + 1 == ncg ? 0 : qi + 1;
                continue;
            }
            tried = 0;
            // read through the constant address space, as kernel arguments are:
            // the loads are scalar and may be repeated where registers run short
            const WalkGrid &G = *(const WalkGrid *)(const __attribute__((address_space(4))) WalkGrid *)(grids + qg);
            const WalkArgs &A = *(const WalkArgs *)(const __attribute__((address_space(4))) WalkArgs *)(args + qg);
            // records of a grid that does not fit are not written: its chunks
            // are taken and dropped
            if (WM == WM_FILL && A.offsets[A.n] > A.capacity) {
                if (lane == 0) st->cap_overflow = 1;
                continue;
            }
            count_rechecks = count_rechecks || A.count_rechecks;
            const GridChunks src{Q.chunks, Q.gctr + qg, c0, nq};
            const int64_t b = Q.chunks[c0 + int64_t(t)].start, e = Q.chunks[c0 + int64_t(t)].end;
            if (G.tree == KD)
                persistent_loop<KD, PREC, WM, R>(G, A, geo, ring, stl, stds, src, b, e, refill_min, lane, wid,
                                                 rechecks, desc);
            else
                persistent_loop<OCT, PREC, WM, R>(G, A, geo, ring, stl, stds, src, b, e, refill_min, lane, wid,
                                                  rechecks, desc);
        }
    }
    if (!(WM == WM_FILL) && count_rechecks) {
        if (rechecks) atomicAdd(&st->rechecks, rechecks);
        if (desc) atomicAdd(&st->descents, (unsigned long long)desc);
    }
}

template <int PREC, int BT>
__global__ void __launch_bounds__(BT) __attribute__((amdgpu_waves_per_eu(4)))
    k_walk_batched_count(const WalkGrid *__restrict__ grids, const WalkArgs *__restrict__ args, const BatchQueue Q,
                         int refill_min, TraceStatus *st)
{
    __shared__ LevelGeo geo[NLEV];
    __shared__ Prep ring_all[(BT / 64) * RING];
    walk_batched<PREC, WM_COUNT, BT>(grids, args, Q, refill_min, st, geo, ring_all, nullptr, nullptr);
}

// Record modes of the batched walk: WM_FILL (the chunks' paths, or with
// resume entries in the arguments the paths past their rows) and WM_SLAB
// (the one-pass walk into per-path rows).
template <int PREC, int WM, int BT>
__global__ void __launch_bounds__(BT) __attribute__((amdgpu_waves_per_eu(4)))
    k_walk_batched_rec(const WalkGrid *__restrict__ grids, const WalkArgs *__restrict__ args, const BatchQueue Q,
                       int refill_min, TraceStatus *st)
{
    using DsT = typename Lane<PREC, uint32_t>::DsT;
    __shared__ LevelGeo geo[NLEV];
    __shared__ Prep ring_all[(BT / 64) * RING];
    __shared__ uint32_t stl[BT * SP];
    __shared__ DsT stds[BT * SP];
    walk_batched<PREC, WM, BT>(grids, args, Q, refill_min, st, geo, ring_all, stl, stds);
}

__global__ void k_zero_counters(unsigned long long *__restrict__ c, int n)
{
    for (int i = int(blockIdx.x) * TB + threadIdx.x; i < n; i += int(gridDim.x) * TB) c[i] = 0ull;
}

template <int TREE, typename R>
__global__ void __launch_bounds__(TB) k_locate(WalkGrid G, const double *__restrict__ X, int64_t n,
                                               int32_t *__restrict__ out)
{
    __shared__ LevelGeo geo[NLEV];
    fill_levels(geo, G, threadIdx.x, TB);
    __syncthreads();
    const int64_t i = int64_t(blockIdx.x) * TB + threadIdx.x;
    if (i >= n) return;
    Lane<HG_FP64, R> L;
#pragma unroll
    for (int d = 0; d < 3; d++) {
        L.p[d] = X[3 * i + d];
        L.k[d] = 0.0;
    }
    if (!inside_closed(G, L.p)) {
        out[i] = -1;
        return;
    }
    L.ref = start_node<TREE, R>(G, L.p, L.k, L.lv, L.X);
    L.tie = 0;
    while (!Ref<R>::leaf(L.ref)) {
        if (!descend_ok<TREE, R>(G, L.ref, L.lv)) {
            out[i] = -2;
            return;
        }
        descend_step<TREE, HG_FP64, R>(G, geo, L);
    }
    out[i] = Ref<R>::id(L.ref) < G.n_leaves ? int32_t(Ref<R>::id(L.ref)) : -2;
}

__global__ void k_reset_counter(TraceStatus *st) { st->next_ray = 0ull; }

// One-pass records mode: copy the rows of the slab (each path's first `slab`
// records) into the CSR slices.  A block takes CP consecutive paths, whose
// slices form one contiguous range of the output, and its threads walk that
// range in order (coalesced writes), each finding its path by a binary search
// over the block's offsets in LDS.  Each thread moves CU records per round
// (TB apart), issuing all their loads before any store.  A path with more
// records than its row gets its first `slab` here, the rest from the fill
// walk.
constexpr int CP = 256;
constexpr int CU = 4;

// The copy of the rows of paths [p0, p0 + np) into their CSR slices, by one
// block; off holds offsets[p0 .. p0 + np] (in LDS).  PAIRS: rows of (leaf,
// ds32) pairs in rl, else leaf rows in rl and ds rows in rd.
template <typename DsT, bool PAIRS>
__device__ __forceinline__ void compact_piece(const void *__restrict__ rl, const DsT *__restrict__ rd,
                                              int64_t slab, const int64_t *off, int64_t p0, int np,
                                              int32_t *__restrict__ leaf, DsT *__restrict__ ds)
{
    const int64_t d0 = off[0], d1 = off[np];
    int lo = 0;   // the path of the thread's previous record: the search starts there
    for (int64_t db = d0 + threadIdx.x; db < d1; db += int64_t(CU) * TB) {
        int64_t src[CU];
        bool ok[CU];
#pragma unroll
        for (int u = 0; u < CU; u++) {
            const int64_t d = db + int64_t(u) * TB;
            int hi = np;   // the path q with off[q] <= d < off[q+1]
            while (hi - lo > 1) {
                const int mid = (lo + hi) >> 1;
                if (off[mid] <= d) lo = mid;
                else hi = mid;
            }
            ok[u] = d < d1 && d - off[lo] < slab;
            src[u] = (p0 + lo) * slab + (d - off[lo]);
        }
        int32_t lf[CU];
        DsT dv[CU];
        if (PAIRS) {
            const uint2 *srow = static_cast<const uint2 *>(rl);
#pragma unroll
            for (int u = 0; u < CU; u++) {
                const uint2 v = ok[u] ? srow[src[u]] : make_uint2(0u, 0u);
                lf[u] = int32_t(v.x);
                dv[u] = DsT(__uint_as_float(v.y));
            }
        } else {
            const int32_t *sleaf = static_cast<const int32_t *>(rl);
#pragma unroll
            for (int u = 0; u < CU; u++) {
                lf[u] = ok[u] ? sleaf[src[u]] : 0;
                dv[u] = ok[u] ? rd[src[u]] : DsT(0);
            }
        }
#pragma unroll
        for (int u = 0; u < CU; u++) {
            const int64_t d = db + int64_t(u) * TB;
            if (ok[u]) {
                leaf[d] = lf[u];
                ds[d] = dv[u];
            }
        }
    }
}

// One-pass records mode: copy the rows of the slab (each path's first `slab`
// records) into the CSR slices.  A block takes CP consecutive paths, whose
// slices form one contiguous range of the output, and its threads walk that
// range in order (coalesced writes), each finding its path by a binary search
// over the block's offsets in LDS.  Each thread moves CU records per round
// (TB apart), issuing all their loads before any store.  A path with more
// records than its row gets its first `slab` here, the rest from the fill
// walk.
template <typename DsT, bool PAIRS>
__global__ void __launch_bounds__(TB)
    k_slab_compact(const void *__restrict__ rl, const DsT *__restrict__ rd, int64_t slab,
                   const int64_t *__restrict__ offsets, int64_t n, int32_t *__restrict__ leaf,
                   DsT *__restrict__ ds)
{
    __shared__ int64_t off[CP + 1];
    const int64_t p0 = int64_t(blockIdx.x) * CP;
    const int np = int(n - p0 < CP ? n - p0 : CP);
    for (int j = threadIdx.x; j <= np; j += TB) off[j] = offsets[p0 + j];
    __syncthreads();
    compact_piece<DsT, PAIRS>(rl, rd, slab, off, p0, np, leaf, ds);
}

// The same over the chunks of a batch: grid g's rows are in slab_args[g]
// (leaf / ds), its CSR slices in fill_args[g].  A grid whose records exceed
// its capacity is skipped (and flagged).
template <typename DsT, bool PAIRS>
__global__ void __launch_bounds__(TB)
    k_slab_compact_batch(const WalkArgs *__restrict__ slab_args, const WalkArgs *__restrict__ fill_args,
                         const BatchQueue Q, TraceStatus *st)
{
    __shared__ int64_t off[CP + 1];
    const int64_t n_chunks = Q.gpre[Q.ng];
    bool past = false;   // a path with more records than its row: the resume walk has work
    for (int64_t c = blockIdx.x; c < n_chunks; c += gridDim.x) {
        const BatchChunk ch = Q.chunks[c];
        const WalkArgs &S = slab_args[ch.grid];
        const WalkArgs &F = fill_args[ch.grid];
        if (F.offsets[F.n] > F.capacity) {
            if (threadIdx.x == 0) st->cap_overflow = 1;
            continue;
        }
        for (int64_t p0 = ch.start; p0 < ch.end; p0 += CP) {
            const int np = int(ch.end - p0 < CP ? ch.end - p0 : CP);
            __syncthreads();
            for (int j = threadIdx.x; j <= np; j += TB) off[j] = F.offsets[p0 + j];
            __syncthreads();
            for (int j = threadIdx.x; j < np; j += TB) past = past || off[j + 1] - off[j] > S.slab;
            compact_piece<DsT, PAIRS>(S.leaf, static_cast<const DsT *>(S.ds), S.slab, off, p0, np, F.leaf,
                                      static_cast<DsT *>(F.ds));
        }
    }
    if (__syncthreads_or(past) && threadIdx.x == 0) st->resumed = 1;
}

constexpr int64_t PERSIST_CHUNK = int64_t(1) << 30;
constexpr uint32_t DEFAULT_CHUNK = 256;   // paths per work-queue atomic
constexpr int DEFAULT_REFILL = 4;         // idle lanes that trigger a refill

// Persistent grid size of a kernel: resident blocks per CU at this block size
// and LDS use times the CU count of the current device.  Cached per (device,
// kernel, block size, LDS bytes) under a lock, so concurrent calls from several
// host threads or on several devices each get their own device's figure.
int occupancy_blocks(const void *kern, int bt, size_t lds, unsigned *blocks)
{
    static std::mutex m;
    static std::map<std::tuple<int, const void *, int, size_t>, unsigned> cache;
    int dev = 0;
    HG_CHECK(hipGetDevice(&dev));
    const auto key = std::make_tuple(dev, kern, bt, lds);
    {
        std::lock_guard<std::mutex> lock(m);
        const auto it = cache.find(key);
        if (it != cache.end()) {
            *blocks = it->second;
            return HG_OK;
        }
    }
    int cus = 0, occ = 0;
    HG_CHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    HG_CHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kern, bt, lds));
    const unsigned b = unsigned(std::max(1, cus) * std::max(1, occ));
    {
        std::lock_guard<std::mutex> lock(m);
        cache[key] = b;
    }
    *blocks = b;
    return HG_OK;
}

template <int TREE, int PREC, int WM, typename R, int BT>
int persistent_blocks(size_t lds, unsigned *blocks)
{
    return occupancy_blocks(reinterpret_cast<const void *>(k_walk_persistent<TREE, PREC, WM, R, BT>), BT, lds,
                            blocks);
}

template <int TREE, int PREC, int WM, typename R, int BT>
int launch_persistent(const WalkGrid &G, const WalkArgs &A, const hg_trace_opts *o, hipStream_t s)
{
    unsigned blocks = 0;
    int rc = persistent_blocks<TREE, PREC, WM, R, BT>(0, &blocks);
    if (rc) return rc;
    const uint32_t chunk = o->chunk > 0 ? uint32_t(o->chunk) : DEFAULT_CHUNK;
    const int refill_min = o->refill_min > 0 ? std::min(o->refill_min, 64) : DEFAULT_REFILL;
    for (int64_t start = 0; start < A.n; start += PERSIST_CHUNK) {
        WalkArgs B = A;
        B.n = std::min(PERSIST_CHUNK, A.n - start);
        if (WM == WM_FILL && A.resume) {
            B.resume = A.resume + start;
        } else {
            B.O = A.O + 3 * start;
            B.K = A.K + 3 * start;
            B.tau = A.tau ? A.tau + start : nullptr;
            B.count = A.count ? A.count + start : nullptr;
            B.offsets = A.offsets ? A.offsets + start : nullptr;
            B.lim = A.lim ? A.lim + start : nullptr;
        }
        k_reset_counter<<<1, 1, 0, s>>>(A.st);
        HG_CHECK(hipGetLastError());
        k_walk_persistent<TREE, PREC, WM, R, BT><<<dim3(blocks), dim3(BT), 0, s>>>(G, B, chunk, refill_min);
        HG_CHECK(hipGetLastError());
    }
    return HG_OK;
}

template <int TREE, int PREC, int WM, typename R>
int launch_t(const WalkGrid &G, const WalkArgs &A, int persistent, const hg_trace_opts *o,
             hipStream_t s)
{
    if (A.n == 0) return HG_OK;
    if (!persistent) {
        const int64_t nb = (A.n + TB - 1) / TB;
        k_walk<TREE, PREC, WM, R><<<dim3(unsigned(nb)), dim3(TB), 0, s>>>(G, A);
        HG_CHECK(hipGetLastError());
        return HG_OK;
    }
    switch (o->block) {
    case 128: return launch_persistent<TREE, PREC, WM, R, 128>(G, A, o, s);
    case 512: return launch_persistent<TREE, PREC, WM, R, 512>(G, A, o, s);
    default: return launch_persistent<TREE, PREC, WM, R, 256>(G, A, o, s);
    }
}

template <int TREE, int PREC, typename R>
int dispatch_mode(const WalkGrid &G, const WalkArgs &A, int wm, int persistent, const hg_trace_opts *o,
                  hipStream_t s)
{
    switch (wm) {
    case WM_FILL: return launch_t<TREE, PREC, WM_FILL, R>(G, A, persistent, o, s);
    case WM_SLAB: return launch_t<TREE, PREC, WM_SLAB, R>(G, A, persistent, o, s);
    case WM_SEG: return launch_t<TREE, PREC, WM_SEG, R>(G, A, 1, o, s);
    case WM_INT: return launch_t<TREE, PREC, WM_INT, R>(G, A, 1, o, s);
    default: return launch_t<TREE, PREC, WM_COUNT, R>(G, A, persistent, o, s);
    }
}

template <int TREE, typename R>
int dispatch_walk(const WalkGrid &G, const WalkArgs &A, int prec, int wm, int persistent,
                  const hg_trace_opts *o, hipStream_t s)
{
    if (prec == HG_FP64) return dispatch_mode<TREE, HG_FP64, R>(G, A, wm, persistent, o, s);
    return dispatch_mode<TREE, HG_FP32_RECHECK, R>(G, A, wm, persistent, o, s);
}

template <int PREC, int WM, int BT>
int launch_batched_t(const WalkGrid *grids, const WalkArgs *args, const BatchQueue &Q, int refill_min,
                     TraceStatus *st, hipStream_t s)
{
    const size_t lds = 0;   // the batched walks use static LDS only
    const void *kern = WM == WM_COUNT ? reinterpret_cast<const void *>(k_walk_batched_count<PREC, BT>)
                                      : reinterpret_cast<const void *>(k_walk_batched_rec<PREC, WM, BT>);
    unsigned blocks = 0;
    {
        const int rc = occupancy_blocks(kern, BT, lds, &blocks);
        if (rc) return rc;
    }
    k_zero_counters<<<unsigned((Q.ng + TB - 1) / TB), TB, 0, s>>>(Q.gctr, Q.ng);
    HG_CHECK(hipGetLastError());
    if (WM == WM_COUNT)
        k_walk_batched_count<PREC, BT><<<dim3(blocks), dim3(BT), 0, s>>>(grids, args, Q, refill_min, st);
    else
        k_walk_batched_rec<PREC, WM, BT><<<dim3(blocks), dim3(BT), 0, s>>>(grids, args, Q, refill_min, st);
    HG_CHECK(hipGetLastError());
    return HG_OK;
}

template <int PREC, int WM>
int launch_batched_b(const WalkGrid *grids, const WalkArgs *args, const BatchQueue &Q, int block, int refill_min,
                     TraceStatus *st, hipStream_t s)
{
    switch (block) {
    case 128: return launch_batched_t<PREC, WM, 128>(grids, args, Q, refill_min, st, s);
    case 512: return launch_batched_t<PREC, WM, 512>(grids, args, Q, refill_min, st, s);
    default: return launch_batched_t<PREC, WM, 256>(grids, args, Q, refill_min, st, s);
    }
}

template <int PREC>
int launch_batched_p(const WalkGrid *grids, const WalkArgs *args, const BatchQueue &Q, int wm, int block,
                     int refill_min, TraceStatus *st, hipStream_t s)
{
    switch (wm) {
    case WM_FILL: return launch_batched_b<PREC, WM_FILL>(grids, args, Q, block, refill_min, st, s);
    case WM_SLAB: return launch_batched_b<PREC, WM_SLAB>(grids, args, Q, block, refill_min, st, s);
    default: return launch_batched_b<PREC, WM_COUNT>(grids, args, Q, block, refill_min, st, s);
    }
}

}  // namespace

WalkGrid walk_grid(const hg_grid *g, int precision)
{
    WalkGrid G;
    G.tree = g->tree;
    for (int d = 0; d < 3; d++) G.lo[d] = g->lo[d];
    G.side = g->side;
    int e = 0;
    frexp(g->side, &e);
    G.lg = e - 1;
    for (int d = 0; d < 3; d++) G.hi[d] = g->lo[d] + g->side;
    G.root = g->root_ref;
    G.n_leaves = uint64_t(g->n_leaves);
    G.n_internal = uint64_t(g->n_internal);
    G.rec = g->wide ? static_cast<const void *>(g->recw)
                    : (precision == HG_FP64 ? static_cast<const void *>(g->rec64)
                                            : static_cast<const void *>(g->rec32));
    G.child = g->child;
    G.jump = g->jump;
    G.table = g->table;
    G.tdep = g->table ? g->tdep : 0;
    G.tw = ldexp(g->side, -G.tdep);
    G.tscale = ldexp(1.0, G.tdep) / g->side;
    G.dm = finest_depth(g->tree, g->max_level);
    G.unit = ldexp(g->side, -G.dm);
    return G;
}

int launch_walk_args(const hg_grid *g, const WalkArgs &A, const hg_trace_opts *opts, int wm,
                     hipStream_t s)
{
    // bit 0: persistent counting / tau-only / slab walk, bit 1: persistent fill walk
    const int mode = opts->persistent < 0 ? 3 : opts->persistent;
    const int persistent = wm == WM_FILL ? (mode >> 1) & 1 : mode & 1;
    // the early-exit walks read the FP64 records whatever the exit-decision precision
    const WalkGrid G = walk_grid(g, wm == WM_SEG || wm == WM_INT ? HG_FP64 : opts->precision);
    const int prec = opts->precision;
    if (g->tree == KDG) {
        if (!g->wide) return HG_E_FORMAT;   // its references carry the node geometry
        return dispatch_walk<KDG, uint64_t>(G, A, prec, wm, persistent, opts, s);
    }
    if (g->tree == KD)
        return g->wide ? dispatch_walk<KD, uint64_t>(G, A, prec, wm, persistent, opts, s)
                       : dispatch_walk<KD, uint32_t>(G, A, prec, wm, persistent, opts, s);
    return g->wide ? dispatch_walk<OCT, uint64_t>(G, A, prec, wm, persistent, opts, s)
                   : dispatch_walk<OCT, uint32_t>(G, A, prec, wm, persistent, opts, s);
}

int launch_walk(const hg_grid *g, TraceStatus *st, const double *o, const double *k, int64_t n,
                const hg_trace_opts *opts, hg_trace_out *out, int wm, hipStream_t s, float *ms)
{
    (void)ms;
    return launch_walk_args(g, walk_args(g, st, o, k, n, opts, out), opts, wm, s);
}

WalkArgs walk_args(const hg_grid *g, TraceStatus *st, const double *o, const double *k, int64_t n,
                   const hg_trace_opts *opts, hg_trace_out *out)
{
    WalkArgs A;
    A.O = o;
    A.K = k;
    A.n = n;
    A.kappa = opts->kappa;
    A.tau = out->tau;
    A.count = out->count;
    A.offsets = out->offsets;
    A.leaf = out->leaf;
    A.ds = out->ds;
    A.capacity = out->capacity;
    A.st = st;
    A.count_rechecks = (opts->flags & HG_FLAG_RECHECKS) ? 1 : 0;
    A.slab = 0;
    A.resume = nullptr;
    A.n_resume = nullptr;
    A.pairs = 0;
    A.resume_by_path = 0;
    A.lim = nullptr;
    return A;
}

int launch_batched(const WalkGrid *grids, const WalkArgs *args, const BatchQueue &Q, const hg_trace_opts *opts,
                   int wm, TraceStatus *st, hipStream_t s)
{
    if (Q.ng <= 0) return HG_OK;
    const int refill_min = opts->refill_min > 0 ? std::min(opts->refill_min, 64) : DEFAULT_REFILL;
    if (opts->precision == HG_FP64)
        return launch_batched_p<HG_FP64>(grids, args, Q, wm, opts->block, refill_min, st, s);
    return launch_batched_p<HG_FP32_RECHECK>(grids, args, Q, wm, opts->block, refill_min, st, s);
}

int launch_slab_compact_batch(const WalkArgs *slab_args, const WalkArgs *fill_args, const BatchQueue &Q,
                              int max_chunks, int precision, int pairs, TraceStatus *st, hipStream_t s)
{
    if (max_chunks <= 0) return HG_OK;
    const unsigned blocks = unsigned(std::min(max_chunks, 4096));
    if (pairs && precision != HG_FP64)
        k_slab_compact_batch<float, true><<<blocks, TB, 0, s>>>(slab_args, fill_args, Q, st);
    else if (precision == HG_FP64)
        k_slab_compact_batch<double, false><<<blocks, TB, 0, s>>>(slab_args, fill_args, Q, st);
    else
        k_slab_compact_batch<float, false><<<blocks, TB, 0, s>>>(slab_args, fill_args, Q, st);
    HG_CHECK(hipGetLastError());
    return HG_OK;
}

int launch_slab_compact(const void *sleaf, const void *sds, int64_t slab, int precision, int pairs,
                        const int32_t *count, const int64_t *offsets, int64_t n, int32_t *leaf, void *ds,
                        hipStream_t s)
{
    if (n == 0) return HG_OK;
    const int64_t nb = (n + CP - 1) / CP;
    if (nb > 0x7fffffff) return HG_E_LIMIT;
    const unsigned blocks = unsigned(nb);
    (void)count;
    if (pairs && precision != HG_FP64)
        k_slab_compact<float, true><<<blocks, TB, 0, s>>>(sleaf, nullptr, slab, offsets, n, leaf, (float *)ds);
    else if (precision == HG_FP64)
        k_slab_compact<double, false><<<blocks, TB, 0, s>>>(sleaf, (const double *)sds, slab, offsets, n, leaf,
                                                            (double *)ds);
    else
        k_slab_compact<float, false><<<blocks, TB, 0, s>>>(sleaf, (const float *)sds, slab, offsets, n, leaf,
                                                           (float *)ds);
    HG_CHECK(hipGetLastError());
    return HG_OK;
}

int launch_locate(const hg_grid *g, const double *p, int64_t n, int32_t *leaf, hipStream_t s)
{
    const WalkGrid G = walk_grid(g, HG_FP64);
    const int64_t nb = (n + TB - 1) / TB;
    if (nb == 0) return HG_OK;
    const dim3 grid{unsigned(nb), 1u, 1u}, block{unsigned(TB), 1u, 1u};
    if (g->tree == KDG) {
        if (!g->wide) return HG_E_FORMAT;
        k_locate<KDG, uint64_t><<<grid, block, 0, s>>>(G, p, n, leaf);
    } else if (g->tree == KD) {
        if (g->wide) k_locate<KD, uint64_t><<<grid, block, 0, s>>>(G, p, n, leaf);
        else k_locate<KD, uint32_t><<<grid, block, 0, s>>>(G, p, n, leaf);
    } else {
        if (g->wide) k_locate<OCT, uint64_t><<<grid, block, 0, s>>>(G, p, n, leaf);
        else k_locate<OCT, uint32_t><<<grid, block, 0, s>>>(G, p, n, leaf);
    }
    HG_CHECK(hipGetLastError());
    return HG_OK;
}

}  // namespace hg
