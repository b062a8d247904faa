// Straight-path traversal (Sect. 2.3) and point location on gfx950.
//
// One lane walks one path.  Per crossing the lane
//   1. finds the exit face of its leaf: the face distances Delta_d from the
//      entry point, t_d = Delta_d |1/k_d|, and the lowest axis of the minimum;
//   2. records (leaf, ds) and adds kappa rho ds to tau;
//   3. re-anchors the exit point: the crossed face's plane on the exit axis,
//      p0 + s k clamped to the leaf on the others (s = path length so far);
//   4. reads the rope of the exit face from the leaf's 32-byte record and, if
//      the rope target is not itself a leaf, descends from it with the exit
//      point (one 4-byte child reference per level).
// The leaf's box is never loaded: it follows from the level and the integer
// cell coordinates the lane carries, which the rope target's level and the
// descent update.  Ties on a split plane follow one fixed rule so that the
// result is reproducible to the bit (see upper_side).
//
// HG_FP32_RECHECK computes the exit decision in FP32 from face distances
// rounded from FP64 and rechecks in FP64 when the two smallest FP32 exit
// distances are closer than 1e-5 of the leaf's smallest side; positions, ds
// and the re-anchoring stay in FP64, so the leaf sequence is that of the FP64
// walk.  tau is then a Kahan-compensated FP32 sum of kappa rho32 ds32.
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

// Keeps a value in registers: selecting among values passed through this stays
// a register select instead of being folded into an indexed stack access.
__device__ __forceinline__ double in_reg(double x)
{
    asm volatile("" : "+v"(x));
    return x;
}

// 2^e for a normal exponent.
__device__ __forceinline__ double pow2(int e) { return __hiloint2double((e + 1023) << 20, 0); }

// Tie context of a descent, packed in one register: bits 0-1 the axis of the
// face just crossed (3 = none), bits 2-4 "point on the low face of the leaf
// just left" per axis, bits 5-7 "on its high face".
constexpr int TIE_NONE = 3;

// Direction signs of a path, packed: bit d set if k_d > 0, bit 3+d if k_d < 0.
__device__ __forceinline__ int dir_bits(const double k[3])
{
    int b = 0;
#pragma unroll
    for (int d = 0; d < 3; d++) b |= (int(k[d] > 0.0) << d) | (int(k[d] < 0.0) << (3 + d));
    return b;
}

// Side of a split plane c on axis d that holds the point whose coordinate is
// x.  Off the plane the comparison decides.  On it: the axis of the face just
// crossed goes to the side the path moves to; a plane on the boundary of the
// leaf just left keeps the point inside that leaf's slab; otherwise the
// direction decides, a zero component going to the upper side.
__device__ __forceinline__ int upper_side(double x, double c, int d, int dirb, int tie)
{
    const int kpos = (dirb >> d) & 1;
    const int kneg = (dirb >> (3 + d)) & 1;
    const int onlo = (tie >> (2 + d)) & 1;
    const int onhi = (tie >> (5 + d)) & 1;
    const int on_plane = d == (tie & 3) ? kpos : (onhi ? 0 : (onlo ? 1 : kneg ^ 1));
    return x > c ? 1 : (x < c ? 0 : on_plane);
}

// True when ref may be dereferenced: a leaf or internal id inside the arrays.
template <typename R>
__device__ __forceinline__ bool ref_ok(const WalkGrid &G, R ref)
{
    return ref != Ref<R>::NUL && Ref<R>::id(ref) < (Ref<R>::leaf(ref) ? G.n_leaves : G.n_internal);
}

// Walk-record layout: compact (32-bit references, 32-byte records, separate
// f32 and f64 record arrays) or wide (64-bit references, one 64-byte record).
template <typename R, int PREC>
struct Rec {
    static constexpr int STRIDE = sizeof(R) == 8 ? 64 : 32;
    static constexpr int RHO64 = sizeof(R) == 8 ? 48 : 24;
    static constexpr int RHO32 = sizeof(R) == 8 ? 56 : 24;
};

// Per-axis depth and cell width of a node at level lv.
template <int TREE>
__device__ __forceinline__ void level_geom(int lg, int lv, int dep[3], double w[3])
{
    if (TREE == OCT) {
        const double ww = pow2(lg - lv);
#pragma unroll
        for (int d = 0; d < 3; d++) {
            dep[d] = lv;
            w[d] = ww;
        }
    } else {
        const int q = (lv * 43691) >> 17;  // lv / 3 for 0 <= lv < 64
        const int r = lv - 3 * q;
        dep[0] = q + (r >= 1);
        dep[1] = q + (r >= 2);
        dep[2] = q;
#pragma unroll
        for (int d = 0; d < 3; d++) w[d] = pow2(lg - dep[d]);
    }
}

// One descent step from the internal node ref (level lv, lower corner lo)
// toward the point q: returns the child's reference and moves lo to the
// child's corner.  Split planes are lo + half the node's width (exact: every
// plane is a binary fraction).  Child references of the first lds_n internal
// nodes are read from LDS.
template <int TREE, typename R>
__device__ __forceinline__ R child_of(const WalkGrid &G, const R *lds, uint32_t lds_n, R ref, int &lv,
                                      double lo[3], const double q[3], int dirb, int tie)
{
    const uint64_t id = Ref<R>::id(ref);
    uint64_t slot;
    if (TREE == KD) {
        const int q3 = (lv * 43691) >> 17;  // lv / 3: the split axis b = lv mod 3 has depth lv / 3
        const int b = lv - 3 * q3;
        const double l0 = in_reg(lo[0]), l1 = in_reg(lo[1]), l2 = in_reg(lo[2]);
        const double q0 = in_reg(q[0]), q1 = in_reg(q[1]), q2 = in_reg(q[2]);
        const double lob = b == 0 ? l0 : (b == 1 ? l1 : l2);
        const double qb = b == 0 ? q0 : (b == 1 ? q1 : q2);
        const double mid = lob + pow2(G.lg - q3 - 1);
        const int up = upper_side(qb, mid, b, dirb, tie);
        slot = 2u * id + uint64_t(up);
        const double nlo = up ? mid : lob;
        lo[0] = b == 0 ? nlo : l0;
        lo[1] = b == 1 ? nlo : l1;
        lo[2] = b == 2 ? nlo : l2;
    } else {
        const double wh = pow2(G.lg - lv - 1);
        uint32_t idx = 0;
#pragma unroll
        for (int d = 0; d < 3; d++) {
            const double mid = lo[d] + wh;
            const int up = upper_side(q[d], mid, d, dirb, tie);
            idx |= uint32_t(up) << d;
            lo[d] = up ? mid : lo[d];
        }
        slot = 8u * id + idx;
    }
    lv++;
    return id < lds_n ? lds[slot] : static_cast<const R *>(G.child)[slot];
}

// Descend from ref to the leaf holding q.  Returns the null reference if one is
// out of range or the depth exceeds the format's limit (never for a valid
// layout).
template <int TREE, typename R>
__device__ __forceinline__ R descend(const WalkGrid &G, const R *lds, uint32_t lds_n, R ref, int &lv,
                                     double lo[3], const double q[3], int dirb, int tie)
{
    while (!Ref<R>::leaf(ref)) {
        if (!ref_ok(G, ref) || lv >= 62) return Ref<R>::NUL;
        ref = child_of<TREE, R>(G, lds, lds_n, ref, lv, lo, q, dirb, tie);
    }
    return ref_ok(G, ref) ? ref : Ref<R>::NUL;
}

// Node where the first descent toward q starts: the locate-table cell holding
// q (chosen with the descent's rule for a point on a plane with no tie
// context: the upper side unless the direction's component is negative),
// its reference, level and lower corner; the root without a table.  The
// descent from there takes the same decisions as one from the root: every
// plane above the table level is a cell boundary, and the cell is picked by
// exact comparisons with those planes.
template <int TREE, typename R>
__device__ __forceinline__ R start_node(const WalkGrid &G, const double q[3], int dirb, int &lv, double lo[3])
{
    if (G.tdep == 0) {
        lv = 0;
#pragma unroll
        for (int d = 0; d < 3; d++) lo[d] = G.lo[d];
        return R(G.root);
    }
    const int T = 1 << G.tdep;
    const double wc = pow2(G.lg - G.tdep);
    const double scale = pow2(G.tdep - G.lg);
    int c[3];
#pragma unroll
    for (int d = 0; d < 3; d++) {
        int i = int(floor((q[d] - G.lo[d]) * scale));
        i = i < 0 ? 0 : (i > T - 1 ? T - 1 : i);
        // (q - lo) may round: settle the cell by exact comparisons with its planes
        if (i > 0 && q[d] < G.lo[d] + double(i) * wc) i--;
        else if (i < T - 1 && q[d] >= G.lo[d] + double(i + 1) * wc) i++;
        if (i > 0 && q[d] == G.lo[d] + double(i) * wc && ((dirb >> (3 + d)) & 1)) i--;
        c[d] = i;
    }
    const R ref = static_cast<const R *>(G.table)[(int64_t(c[0]) * T + c[1]) * T + c[2]];
    lv = Ref<R>::level(ref);
    int dep[3];
    double w[3];
    level_geom<TREE>(G.lg, lv, dep, w);
#pragma unroll
    for (int d = 0; d < 3; d++) lo[d] = G.lo[d] + double(c[d] >> (G.tdep - dep[d])) * w[d];
    return ref;
}

__device__ __forceinline__ bool inside_closed(const WalkGrid &G, const double x[3])
{
    bool in = true;
#pragma unroll
    for (int d = 0; d < 3; d++) in = in && (x[d] >= G.lo[d] && x[d] <= G.lo[d] + G.side);
    return in;
}

// Start of the path inside the closed domain: the origin itself, or the entry
// point found by the slab test, placed exactly on the entry face.
__device__ __forceinline__ bool clip_ray(const WalkGrid &G, const double p0[3], const double k[3],
                                const double inv[3], double &s, double p[3])
{
    if (inside_closed(G, p0)) {
        s = 0.0;
#pragma unroll
        for (int d = 0; d < 3; d++) p[d] = p0[d];
        return true;
    }
    double tn = -INFINITY, tf = INFINITY;
    int ax = -1;
    bool miss = false;
#pragma unroll
    for (int d = 0; d < 3; d++) {
        const double lo = G.lo[d], hi = G.lo[d] + G.side;
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
    for (int d = 0; d < 3; d++) {
        const double lo = G.lo[d], hi = G.lo[d] + G.side;
        if (d == ax) {
            p[d] = k[d] > 0.0 ? lo : hi;
        } else {
            const double v = p0[d] + tn * k[d];
            p[d] = v < lo ? lo : (v > hi ? hi : v);
        }
    }
    return true;
}

// Everything a lane carries for one path.
template <int PREC, typename R>
struct Path {
    using DsT = typename std::conditional<PREC == HG_FP64, double, float>::type;
    double p0[3], k[3], ainv[3];
    float ainv32[3];         // FP32 copies of ainv for the FP32 exit decision
    double s, p[3];          // path length so far and the current entry point
    double lo[3];            // lower corner of the current node
    R ref;                   // current node (leaf once the descent ends)
    int lv;                  // its level
    int tie;                 // tie context of the pending descent
    int dirb;                // direction signs (dir_bits)
    int32_t cnt;             // leaves crossed with ds > 0
    int steps;
    double tau64;
    float tau32, comp32;
    bool force64;
    int64_t base, room;      // record slice of this path (fill walk)
    uint32_t sl[4];          // fill walk: last four records, staged for
    DsT sd[4];               // 16-byte aligned vector stores
};

enum { PATH_WALK = 0, PATH_MISS = 1, PATH_BAD_DIR = 2 };
// Walk modes: WM_COUNT (tau and counts; also the tau-only mode), WM_FILL
// (records into the slices given by the offsets of a counting walk),
// WM_SLAB (tau, counts and the first A.slab records of every path into a
// fixed-size row per path, for the one-pass records mode).

template <int TREE, int PREC, int WM, typename R>
__device__ __forceinline__ int init_path(const WalkGrid &G, const WalkArgs &A, int64_t i, Path<PREC, R> &P)
{
    double inv[3];
#pragma unroll
    for (int d = 0; d < 3; d++) {
        P.p0[d] = A.O[3 * i + d];
        P.k[d] = A.K[3 * i + d];
    }
    const double nn = P.k[0] * P.k[0] + P.k[1] * P.k[1] + P.k[2] * P.k[2];
    const bool finite = isfinite(P.k[0]) && isfinite(P.k[1]) && isfinite(P.k[2]);
    if (!finite || !(fabs(sqrt(nn) - 1.0) <= 1e-6)) return PATH_BAD_DIR;
    P.force64 = false;
#pragma unroll
    for (int d = 0; d < 3; d++) {
        inv[d] = 1.0 / P.k[d];
        P.ainv[d] = fabs(inv[d]);
        P.ainv32[d] = float(P.ainv[d]);
        // The FP32 exit decision is used only where its error bound holds.
        if (P.k[d] != 0.0 && !(fabs(P.k[d]) >= 1e-30)) P.force64 = true;
    }
    if (!clip_ray(G, P.p0, P.k, inv, P.s, P.p)) return PATH_MISS;
    P.dirb = dir_bits(P.k);
    P.ref = start_node<TREE, R>(G, P.p, P.dirb, P.lv, P.lo);
    P.tie = TIE_NONE;
    P.cnt = 0;
    P.steps = 0;
    P.tau64 = 0.0;
    P.tau32 = 0.f;
    P.comp32 = 0.f;
    if (WM == WM_FILL) {
        P.base = A.offsets[i];
        P.room = A.offsets[i + 1] - P.base;
    } else if (WM == WM_SLAB) {
        P.base = i * A.slab;
        P.room = A.slab;
    }
    return PATH_WALK;
}

// Fill walk of the one-walk records mode: path S.path continues from the
// state the slab walk saved on entry to the leaf of its first record beyond
// its row; records from there on go to its slice past the first A.slab.
template <int TREE, int PREC, typename R>
__device__ __forceinline__ int64_t resume_path(const WalkArgs &A, const Resume &S, Path<PREC, R> &P)
{
    const int64_t i = S.path;
    P.force64 = false;
#pragma unroll
    for (int d = 0; d < 3; d++) {
        P.p0[d] = A.O[3 * i + d];
        P.k[d] = A.K[3 * i + d];
        P.ainv[d] = fabs(1.0 / P.k[d]);
        P.ainv32[d] = float(P.ainv[d]);
        if (P.k[d] != 0.0 && !(fabs(P.k[d]) >= 1e-30)) P.force64 = true;
        P.p[d] = S.p[d];
        P.lo[d] = S.lo[d];
    }
    P.dirb = dir_bits(P.k);
    P.s = S.s;
    P.ref = R(S.ref);
    P.lv = S.lv;
    P.steps = S.steps;
    P.tie = TIE_NONE;
    P.cnt = 0;
    P.tau64 = 0.0;
    P.tau32 = 0.f;
    P.comp32 = 0.f;
    P.base = A.offsets[i] + A.slab;
    P.room = A.offsets[i + 1] - P.base;
    return i;
}

template <int PREC, typename R>
__device__ __forceinline__ void save_resume(const WalkArgs &A, const Path<PREC, R> &P)
{
    if (!A.resume) return;   // a slab walk that only counts (the autotuner's)
    const unsigned long long j = atomicAdd(A.n_resume, 1ull);
    if (j >= (unsigned long long)A.n) return;   // at most one entry per path: never taken
    Resume &S = A.resume[j];
#pragma unroll
    for (int d = 0; d < 3; d++) {
        S.p[d] = P.p[d];
        S.lo[d] = P.lo[d];
    }
    S.s = P.s;
    S.ref = uint64_t(P.ref);
    S.path = P.base / A.slab;
    S.lv = P.lv;
    S.steps = P.steps;
}

enum { STEP_GO = 0, STEP_END = 1, STEP_ERR = 2 };

// Fill walk: records are staged four at a time and written as aligned 16-byte
// vectors once a group of four positions (pos = 4m .. 4m+3 of the record
// arrays, which must be 16-byte aligned) is complete; the partial groups at
// the two ends of a path's slice are written element by element.
template <int PREC>
__device__ __forceinline__ void store_one(const WalkArgs &A, int64_t pos, uint32_t id, double ds)
{
    A.leaf[pos] = int32_t(id);
    if (PREC == HG_FP64) reinterpret_cast<double *>(A.ds)[pos] = ds;
    else reinterpret_cast<float *>(A.ds)[pos] = float(ds);
}

template <int PREC, typename R>
__device__ __forceinline__ void stage_record(const WalkArgs &A, Path<PREC, R> &P, int64_t pos, uint32_t id,
                                             double ds)
{
    P.sl[0] = P.sl[1]; P.sl[1] = P.sl[2]; P.sl[2] = P.sl[3]; P.sl[3] = id;
    P.sd[0] = P.sd[1]; P.sd[1] = P.sd[2]; P.sd[2] = P.sd[3];
    P.sd[3] = typename Path<PREC, R>::DsT(ds);
    if ((pos & 3) != 3) return;
    const int64_t g = pos - 3;
    if (g >= P.base) {
        *reinterpret_cast<uint4 *>(A.leaf + g) = make_uint4(P.sl[0], P.sl[1], P.sl[2], P.sl[3]);
        if (PREC == HG_FP64) {
            double2 *d = reinterpret_cast<double2 *>(reinterpret_cast<double *>(A.ds) + g);
            d[0] = make_double2(P.sd[0], P.sd[1]);
            d[1] = make_double2(P.sd[2], P.sd[3]);
        } else {
            *reinterpret_cast<float4 *>(reinterpret_cast<float *>(A.ds) + g) =
                make_float4(P.sd[0], P.sd[1], P.sd[2], P.sd[3]);
        }
    } else {
#pragma unroll
        for (int j = 0; j < 4; j++)
            if (g + j >= P.base) store_one<PREC>(A, g + j, P.sl[j], P.sd[j]);
    }
}

// Write the staged records of an unfinished group at the end of a path.
template <int PREC, typename R>
__device__ __forceinline__ void flush_records(const WalkArgs &A, const Path<PREC, R> &P)
{
    if (P.cnt == 0) return;
    const int64_t last = P.base + (P.cnt < P.room ? P.cnt : P.room) - 1;
    const int ph = int(last & 3);
    if (ph == 3) return;
#pragma unroll
    for (int j = 0; j < 3; j++) {
        const int64_t pos = last - j;
        if (j <= ph && pos >= P.base) store_one<PREC>(A, pos, P.sl[3 - j], P.sd[3 - j]);
    }
}

// One crossing of the leaf P.ref: exit face, record / tau, re-anchoring, and
// the rope target of the exit face (left in P.ref for the next descent).  The
// exit face depends only on the cell and the entry point, so it is decided
// before the leaf's record is read; then only the rope of that face and the
// density are loaded.  Written with few branches: the end and error outcomes
// are flags, and the state updates that only matter for a continuing path are
// made unconditionally.
template <int TREE, int PREC, int WM, typename R, bool LSLOT = false>
__device__ __forceinline__ int cross(const WalkGrid &G, const WalkArgs &A, Path<PREC, R> &P,
                                     unsigned long long &rechecks, uint32_t *sl = nullptr,
                                     typename Path<PREC, R>::DsT *sd = nullptr, int sgm = 0)
{
    const bool ok = ref_ok(G, P.ref);
    const uint64_t id = ok ? Ref<R>::id(P.ref) : 0u;
    int dep[3];
    double w[3], hi[3], E[3], t[3];
    int edge = 0;
    const double *lo = P.lo;
    level_geom<TREE>(G.lg, P.lv, dep, w);
#pragma unroll
    for (int d = 0; d < 3; d++) {
        const bool kp = (P.dirb >> d) & 1;
        hi[d] = lo[d] + w[d];
        E[d] = kp ? hi[d] : lo[d];  // the face the path moves toward
        // that face lies on the domain boundary
        edge |= int(kp ? hi[d] == G.hi[d] : lo[d] == G.lo[d]) << d;
        // t = Delta |1/k|; a zero direction component gives +inf or NaN, and
        // neither ever wins the strict comparisons below
        t[d] = fabs(E[d] - P.p[d]) * P.ainv[d];
    }
    int a = -1;
    if (PREC == HG_FP32_RECHECK) {
        // smallest and second smallest exit time in FP32 (NaN counts as +inf);
        // a tie between the two always goes to the FP64 decision below
        float t32[3];
#pragma unroll
        for (int d = 0; d < 3; d++) {
            const float v = float(fabs(E[d] - P.p[d])) * P.ainv32[d];
            t32[d] = v == v ? v : INFINITY;
        }
        const float m1 = fminf(fminf(t32[0], t32[1]), t32[2]);
        const float m2 = __builtin_amdgcn_fmed3f(t32[0], t32[1], t32[2]);
        const int i1 = t32[0] == m1 ? 0 : (t32[1] == m1 ? 1 : 2);
        const float hmin = float(w[0]);  // axis 0 is never coarser than the others
        const bool recheck = P.force64 || !(m2 - m1 >= 1e-5f * hmin);
        rechecks += recheck ? 1u : 0u;
        a = recheck ? -1 : i1;
    }
    if (a < 0) {
        double tmin = INFINITY;
#pragma unroll
        for (int d = 0; d < 3; d++)
            if (t[d] < tmin) {
                tmin = t[d];
                a = d;
            }
    }
    bool err = !ok || a < 0;
    a = a < 0 ? 0 : a;
    const double t0 = in_reg(t[0]), t1 = in_reg(t[1]), t2 = in_reg(t[2]);
    const double ds = a == 0 ? t0 : (a == 1 ? t1 : t2);
    const bool up = (P.dirb >> a) & 1;
    const int face = 2 * a + (up ? 1 : 0);
    // the leaf record: rope of the exit face, density
    const char *rec = static_cast<const char *>(G.rec) + id * Rec<R, PREC>::STRIDE;
    const R nref = reinterpret_cast<const R *>(rec)[face];
    if (ds > 0.0) {
        // LSLOT: records go to the lane's slots sl / sd in LDS (persistent
        // and batched walks), else they are staged in registers
        if (WM == WM_FILL) {
            // the fill walk must repeat the counting walk
            if (P.cnt < P.room) {
                if (LSLOT) {
                    sl[P.cnt & sgm] = uint32_t(id);
                    sd[P.cnt & sgm] = typename Path<PREC, R>::DsT(ds);
                } else {
                    stage_record<PREC, R>(A, P, P.base + P.cnt, uint32_t(id), ds);
                }
            } else {
                err = true;
            }
        } else if (WM == WM_SLAB) {
            // records beyond the row are left to the fill walk, which resumes
            // the path at the first of them
            if (P.cnt < P.room) {
                if (LSLOT) {
                    sl[P.cnt & sgm] = uint32_t(id);
                    sd[P.cnt & sgm] = typename Path<PREC, R>::DsT(ds);
                } else {
                    stage_record<PREC, R>(A, P, P.base + P.cnt, uint32_t(id), ds);
                }
            } else if (P.cnt == P.room) {
                save_resume<PREC, R>(A, P);
            }
        }
        if (WM == WM_FILL) {
        } else if (PREC == HG_FP64) {
            const double rho64 = *reinterpret_cast<const double *>(rec + Rec<R, PREC>::RHO64);
            P.tau64 = P.tau64 + A.kappa * rho64 * ds;
        } else {
            const float rho32 = *reinterpret_cast<const float *>(rec + Rec<R, PREC>::RHO32);
            const float y = float(A.kappa) * rho32 * float(ds) - P.comp32;
            const float tt = P.tau32 + y;
            P.comp32 = (tt - P.tau32) - y;
            P.tau32 = tt;
        }
        P.cnt++;
    }
    // exit face on the domain boundary: the path ends
    const bool end = (edge >> a) & 1;
    // re-anchor the exit point on the crossed face
    P.s = P.s + ds;
    int onlo = 0, onhi = 0;
#pragma unroll
    for (int d = 0; d < 3; d++) {
        const double v = P.p0[d] + P.s * P.k[d];
        const double q = d == a ? E[d] : fmin(fmax(v, lo[d]), hi[d]);
        onlo |= int(q == lo[d]) << d;
        onhi |= int(q == hi[d]) << d;
        P.p[d] = q;
    }
    P.tie = a | (onlo << 2) | (onhi << 5);
    err = err || (!end && nref == Ref<R>::NUL);
    // Lower corner of the rope target: the corner of the leaf, moved across
    // the exit face and aligned down to the target's cell size (exact).  The
    // target is never finer than the leaf across the face; along the exit axis
    // a k-d target may be one level finer (the half of a same-size neighbour
    // touching the face).
    const int nlv = Ref<R>::level(nref);
    int dn[3];
    double wn[3];
    level_geom<TREE>(G.lg, nlv, dn, wn);
    double nlo[3];
#pragma unroll
    for (int d = 0; d < 3; d++) {
        const double x = d != a ? lo[d] : (up ? hi[d] : lo[d] - fmin(w[d], wn[d]));
        const double inv = pow2(dn[d] - G.lg);
        nlo[d] = G.lo[d] + floor((x - G.lo[d]) * inv) * wn[d];
    }
#pragma unroll
    for (int d = 0; d < 3; d++) P.lo[d] = nlo[d];
    P.lv = nlv;
    P.ref = nref;
    return err ? STEP_ERR : (end ? STEP_END : STEP_GO);
}

template <int PREC, int WM, typename R, bool STG = false>
__device__ __forceinline__ void finish_path(const WalkArgs &A, int64_t i, const Path<PREC, R> &P)
{
    if (WM == WM_FILL) {
        if (!STG) flush_records<PREC, R>(A, P);
        if (P.cnt != P.room) A.st->step_guard = 1;
        return;
    }
    if (WM == WM_SLAB && !STG) flush_records<PREC, R>(A, P);
    A.count[i] = P.cnt;
    if (PREC == HG_FP64) A.tau[i] = P.tau64;
    else A.tau[i] = double(P.tau32) - double(P.comp32);
}

template <int PREC, int WM>
__device__ __forceinline__ void finish_unwalked(const WalkArgs &A, int64_t i, int why)
{
    if (WM == WM_FILL) return;
    A.count[i] = 0;
    if (why == PATH_BAD_DIR) {
        A.tau[i] = __longlong_as_double(0x7ff8000000000000ll);
        A.st->bad_dir = 1;
    } else {
        A.tau[i] = 0.0;
    }
}

// One lane per path, the whole walk in one loop.
template <int TREE, int PREC, int WM, typename R>
__global__ void __launch_bounds__(TB) k_walk(WalkGrid G, WalkArgs A)
{
    const int64_t q = int64_t(blockIdx.x) * TB + threadIdx.x;
    if (q >= A.n) return;
    Path<PREC, R> P;
    int64_t i = q;
    int why = PATH_WALK;
    if (WM == WM_FILL && A.resume) i = resume_path<TREE, PREC, R>(A, A.resume[q], P);
    else why = init_path<TREE, PREC, WM, R>(G, A, i, P);
    if (why != PATH_WALK) {
        finish_unwalked<PREC, WM>(A, i, why);
        return;
    }
    unsigned long long rechecks = 0;
    uint32_t desc = 0;   // child levels descended
    for (;;) {
        const int lv0 = P.lv;
        P.ref = descend<TREE, R>(G, nullptr, 0u, P.ref, P.lv, P.lo, P.p, P.dirb, P.tie);
        desc += uint32_t(P.lv - lv0);
        if (P.ref == Ref<R>::NUL) {
            A.st->bad_ref = 1;
            break;
        }
        const int r = cross<TREE, PREC, WM, R>(G, A, P, rechecks);
        if (r == STEP_ERR || ++P.steps >= STEP_GUARD) {
            A.st->step_guard = 1;
            break;
        }
        if (r == STEP_END) break;
    }
    finish_path<PREC, WM, R>(A, i, P);
    if (!(WM == WM_FILL) && A.count_rechecks) {
        if (rechecks) atomicAdd(&A.st->rechecks, rechecks);
        if (desc) atomicAdd(&A.st->descents, (unsigned long long)desc);
    }
}

// Records staged in LDS by the persistent and batched walks (record modes):
// each lane owns SG slots of leaf ids and SG of ds (rows of SG + 1 words
// against bank conflicts).  A lane's group is written out once it holds SG
// records, its row or slice is full or its path ends, by the whole
// wavefront: SG lanes per group,
// 64 / SG groups per store instruction, so that a store covers a few cache
// lines instead of one line per lane.
template <int BT>
struct StageShape {
    static constexpr int SG = BT <= 256 ? 16 : 8;
    static constexpr int SP = SG + 1;
};

// Write the groups of the lanes with nr > 0: records pos .. pos+nr-1 of the
// output come from slots 0 .. nr-1 of that lane (into the rows of (leaf, ds)
// pairs when A.pairs is set).  Wavefront-uniform.
template <int BT, typename DsT>
__device__ __forceinline__ void flush_stage(const WalkArgs &A, const uint32_t *stl, const DsT *stds, int nr,
                                            int64_t pos, int lane)
{
    constexpr int SG = StageShape<BT>::SG, SP = StageShape<BT>::SP, PER = 64 / SG;
    uint64_t fm = __ballot(nr > 0);
    if (!fm) return;
    __builtin_amdgcn_wave_barrier();
    const int g = lane / SG, j = lane % SG;
    const int wbase = int(threadIdx.x) & ~63;
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

// Persistent walk: each wavefront keeps its lanes busy by handing new paths
// to lanes whose path ended.  Refills happen in batches (once at least
// refill_min lanes are idle, or none is busy) from a wavefront-local chunk of
// paths taken with one atomic on the global path counter, so the divergent
// path set-up and the atomic round trip are amortised over many paths.  Each
// iteration a busy lane performs one dependent global access: a descent step
// (the first levels of every descent come from LDS) or a crossing.
// Four wavefronts per SIMD: the record modes would otherwise take a few more
// than 128 VGPRs and run three (the few spills this costs are cheaper).
template <int TREE, int PREC, int WM, typename R, int BT>
__global__ void __launch_bounds__(BT) __attribute__((amdgpu_waves_per_eu(4, 8)))
    k_walk_persistent(WalkGrid G, WalkArgs A, uint32_t lds_n, uint32_t chunk, int refill_min,
                      uint32_t stage_off)
{
    extern __shared__ uint64_t lds_raw[];
    R *lds = reinterpret_cast<R *>(lds_raw);
    const int nc = TREE == OCT ? 8 : 2;
    for (uint32_t j = threadIdx.x; j < lds_n * nc; j += BT) lds[j] = static_cast<const R *>(G.child)[j];
    __syncthreads();
    const int lane = threadIdx.x & 63;
    // record modes: LDS staging of the records (see flush_stage)
    constexpr bool STG = WM != WM_COUNT;
    constexpr int SG = StageShape<BT>::SG, SP = StageShape<BT>::SP;
    using DsT = typename Path<PREC, R>::DsT;
    uint32_t *stl = nullptr, *my_l = nullptr;
    DsT *stds = nullptr, *my_d = nullptr;
    if (STG) {
        char *sb = reinterpret_cast<char *>(lds_raw) + stage_off;
        stl = reinterpret_cast<uint32_t *>(sb);
        stds = reinterpret_cast<DsT *>(sb + size_t(BT) * SP * 4);
        my_l = stl + threadIdx.x * SP;
        my_d = stds + threadIdx.x * SP;
    }
    const uint64_t below = lane ? (~0ull >> (64 - lane)) : 0ull;
    Path<PREC, R> P;
    int64_t ray = -1;
    bool done = false;
    uint32_t cnext = 0, cend = 0;   // wavefront-local chunk [cnext, cend)
    bool drained = false;           // the global counter is exhausted
    unsigned long long rechecks = 0;
    uint32_t desc = 0;   // child levels descended
    for (;;) {
        const bool want = ray < 0 && !done;
        const uint64_t wmask = __ballot(want);
        const uint64_t amask = __ballot(ray >= 0);
        const int nwant = __popcll(wmask);
        if (nwant && (nwant >= refill_min || !amask)) {
            if (cnext >= cend && !drained) {
                unsigned long long b = 0;
                if (lane == 0) b = atomicAdd(&A.st->next_ray, (unsigned long long)chunk);
                // wavefront-uniform from here on
                b = (unsigned long long)__builtin_amdgcn_readfirstlane(uint32_t(b)) |
                    ((unsigned long long)__builtin_amdgcn_readfirstlane(uint32_t(b >> 32)) << 32);
                if (b >= (unsigned long long)A.n) {
                    drained = true;
                    cnext = cend = 0;
                } else {
                    cnext = uint32_t(b);
                    cend = uint32_t(std::min<int64_t>(int64_t(b) + chunk, A.n));
                }
            }
            const uint32_t avail = cend - cnext;
            if (want) {
                const uint32_t rank = uint32_t(__popcll(wmask & below));
                if (rank < avail) {
                    const int64_t q = int64_t(cnext) + rank;
                    int64_t r = q;
                    int why = PATH_WALK;
                    if (WM == WM_FILL && A.resume) r = resume_path<TREE, PREC, R>(A, A.resume[q], P);
                    else why = init_path<TREE, PREC, WM, R>(G, A, r, P);
                    if (why == PATH_WALK) ray = r;
                    else finish_unwalked<PREC, WM>(A, r, why);
                } else if (drained) {
                    done = true;
                }
            }
            cnext += std::min<uint32_t>(avail, uint32_t(nwant));
        }
        if (!amask && !__ballot(ray >= 0)) {
            if (!__ballot(!done)) break;
            continue;
        }
        // One predicate per region (no nesting), so the path state needs no
        // copies at region boundaries.
        bool bad = false, fin = false, crossed = false;
        int32_t c_before = 0;
        if (ray >= 0 && !Ref<R>::leaf(P.ref)) {
            // LDS levels, then at most one global level this iteration
            const int lv0 = P.lv;
            for (;;) {
                if (!ref_ok(G, P.ref) || P.lv >= 62) {
                    P.ref = Ref<R>::NUL;
                    break;
                }
                const bool global = Ref<R>::id(P.ref) >= lds_n;
                P.ref = child_of<TREE, R>(G, lds, lds_n, P.ref, P.lv, P.lo, P.p, P.dirb, P.tie);
                if (global || Ref<R>::leaf(P.ref)) break;
            }
            bad = P.ref == Ref<R>::NUL || (Ref<R>::leaf(P.ref) && !ref_ok(G, P.ref));
            desc += uint32_t(P.lv - lv0);
        }
        if (ray >= 0 && !bad && Ref<R>::leaf(P.ref)) {
            c_before = P.cnt;
            const int r = cross<TREE, PREC, WM, R, STG>(G, A, P, rechecks, my_l, my_d, SG - 1);
            crossed = true;
            const bool guard = r == STEP_ERR || ++P.steps >= STEP_GUARD;
            if (guard) A.st->step_guard = 1;
            fin = guard || r == STEP_END;
        }
        if (STG) {
            // the group to write out this iteration: complete, the row full, or
            // the last records of an ended path
            int nr = 0;
            int64_t pos = 0;
            if (ray >= 0 && (crossed || bad)) {
                const int64_t c = P.cnt < P.room ? P.cnt : P.room;
                const bool wrote = crossed && P.cnt > c_before && c_before < P.room;
                if (wrote && ((c & (SG - 1)) == 0 || c == P.room)) nr = int(((c - 1) & (SG - 1)) + 1);
                else if ((bad || fin) && c != P.room) nr = int(c & (SG - 1));
                pos = P.base + c - nr;
            }
            flush_stage<BT, DsT>(A, stl, stds, nr, pos, lane);
        }
        if (bad || fin) {
            if (bad) A.st->bad_ref = 1;
            finish_path<PREC, WM, R, STG>(A, ray, P);
            ray = -1;
        }
    }
    if (!(WM == WM_FILL) && A.count_rechecks) {
        if (rechecks) atomicAdd(&A.st->rechecks, rechecks);
        if (desc) atomicAdd(&A.st->descents, (unsigned long long)desc);
    }
}

// The group of LDS-staged records a lane writes out after a step: complete
// (SG records), the row or slice full, or the last records of an ended path.
template <int SG, int PREC, typename R>
__device__ __forceinline__ void stage_group(const Path<PREC, R> &P, bool crossed, int32_t c_before,
                                            bool ended, int &nr, int64_t &pos)
{
    const int64_t c = P.cnt < P.room ? P.cnt : P.room;
    const bool wrote = crossed && P.cnt > c_before && c_before < P.room;
    nr = 0;
    if (wrote && ((c & (SG - 1)) == 0 || c == P.room)) nr = int(((c - 1) & (SG - 1)) + 1);
    else if (ended && c != P.room) nr = int(c & (SG - 1));
    pos = P.base + c - nr;
}

// One step of a busy lane in the batched walk: at most one global descent
// level, or one crossing.  Returns false when the path ended (or failed).
// With LDS staging (sl != nullptr) the records go to the lane's slots and
// nr / pos name the group to write out after the step.
template <int TREE, int PREC, int WM, int SG>
__device__ __forceinline__ bool batched_step(const WalkGrid &G, const WalkArgs &A,
                                             Path<PREC, uint32_t> &P, int64_t ray,
                                             unsigned long long &rechecks, uint32_t &desc, uint32_t *sl,
                                             typename Path<PREC, uint32_t>::DsT *sd, int &nr, int64_t &pos)
{
    constexpr bool STG = SG > 0;
    bool crossed = false, ended = false;
    int32_t c_before = 0;
    if (!Ref<uint32_t>::leaf(P.ref)) {
        if (!ref_ok(G, P.ref) || P.lv >= 62) {
            A.st->bad_ref = 1;
            ended = true;
        } else {
            P.ref = child_of<TREE, uint32_t>(G, nullptr, 0u, P.ref, P.lv, P.lo, P.p, P.dirb, P.tie);
            desc++;
            if (Ref<uint32_t>::leaf(P.ref) && !ref_ok(G, P.ref)) {
                A.st->bad_ref = 1;
                ended = true;
            }
        }
    }
    if (!ended && Ref<uint32_t>::leaf(P.ref)) {
        c_before = P.cnt;
        const int r = cross<TREE, PREC, WM, uint32_t, STG>(G, A, P, rechecks, sl, sd, STG ? SG - 1 : 0);
        crossed = true;
        if (r == STEP_ERR || ++P.steps >= STEP_GUARD) {
            A.st->step_guard = 1;
            ended = true;
        } else if (r == STEP_END) {
            ended = true;
        }
    }
    if (STG) stage_group<STG ? SG : 1>(P, crossed, c_before, ended, nr, pos);
    if (ended) finish_path<PREC, WM, uint32_t, STG>(A, ray, P);
    return !ended;
}

// Batched walk over many grids in one persistent launch.  The device work
// queue is a table of chunks (grid, path range); a wavefront takes one chunk
// per atomic and keeps that grid's parameters uniform across its lanes,
// refilling lanes from the chunk.  Before taking up a chunk of another grid it
// lets its lanes finish their paths.  Octree and k-d grids mix freely: the
// tree type is a wavefront-uniform branch.
template <int PREC, int WM, int BT>
__device__ __forceinline__ void walk_batched(const WalkGrid *__restrict__ grids, const WalkArgs *__restrict__ args,
                                             const BatchChunk *__restrict__ chunks, int n_chunks,
                                             int refill_min, TraceStatus *st, char *lds_stage)
{
    const int lane = threadIdx.x & 63;
    // the record-filling walk stages its records in LDS (see flush_stage)
    constexpr bool STG = WM == WM_FILL;
    constexpr int SP = StageShape<BT>::SP;
    using DsT = typename Path<PREC, uint32_t>::DsT;
    uint32_t *stl = nullptr, *my_l = nullptr;
    DsT *stds = nullptr, *my_d = nullptr;
    if (STG) {
        char *sb = lds_stage;
        stl = reinterpret_cast<uint32_t *>(sb);
        stds = reinterpret_cast<DsT *>(sb + size_t(BT) * SP * 4);
        my_l = stl + threadIdx.x * SP;
        my_d = stds + threadIdx.x * SP;
    }
    const uint64_t below = lane ? (~0ull >> (64 - lane)) : 0ull;
    Path<PREC, uint32_t> P;
    int64_t ray = -1;
    bool done = false;
    int gi = -1, pc = -1;
    int64_t cnext = 0, cend = 0;
    bool drained = false;
    WalkGrid G;
    WalkArgs A;
    unsigned long long rechecks = 0;
    uint32_t desc = 0;   // child levels descended
    for (;;) {
        const bool want = ray < 0 && !done;
        const uint64_t wmask = __ballot(want);
        const uint64_t amask = __ballot(ray >= 0);
        const int nwant = __popcll(wmask);
        if (nwant && (nwant >= refill_min || !amask)) {
            if (cnext >= cend) {
                if (pc < 0 && !drained) {
                    int c = 0;
                    if (lane == 0) c = int(std::min<unsigned long long>(atomicAdd(&st->next_ray, 1ull), 0x7fffffffull));
                    c = __builtin_amdgcn_readfirstlane(c);   // wavefront-uniform from here on
                    if (c >= n_chunks) drained = true;
                    else pc = c;
                }
                if (pc >= 0) {
                    const int cg = __builtin_amdgcn_readfirstlane(chunks[pc].grid);
                    if (cg == gi || !amask) {
                        if (cg != gi) {
                            gi = cg;
                            G = grids[gi];
                            A = args[gi];
                        }
                        cnext = chunks[pc].start;
                        cend = chunks[pc].end;
                        pc = -1;
                        // records of a grid that does not fit are not written
                        if ((WM == WM_FILL) && A.offsets[A.n] > A.capacity) {
                            if (lane == 0) st->cap_overflow = 1;
                            cnext = cend;
                        }
                    }
                }
            }
            const int64_t avail = cend - cnext;
            if (want) {
                const int64_t rank = __popcll(wmask & below);
                if (rank < avail) {
                    const int64_t r = cnext + rank;
                    const int why = G.tree == KD ? init_path<KD, PREC, WM, uint32_t>(G, A, r, P)
                                                 : init_path<OCT, PREC, WM, uint32_t>(G, A, r, P);
                    if (why == PATH_WALK) ray = r;
                    else finish_unwalked<PREC, WM>(A, r, why);
                } else if (drained && pc < 0) {
                    done = true;
                }
            }
            cnext += std::min<int64_t>(avail, nwant);
        }
        if (!amask && !__ballot(ray >= 0)) {
            if (!__ballot(!done)) break;
            continue;
        }
        constexpr int SGS = STG ? StageShape<BT>::SG : 0;
        int nr = 0;
        int64_t pos = 0;
        if (ray >= 0) {
            const bool alive =
                G.tree == KD ? batched_step<KD, PREC, WM, SGS>(G, A, P, ray, rechecks, desc, my_l, my_d, nr, pos)
                             : batched_step<OCT, PREC, WM, SGS>(G, A, P, ray, rechecks, desc, my_l, my_d, nr, pos);
            if (!alive) ray = -1;
        }
        // every lane holds the wavefront's current grid, so A is uniform here
        if (STG) flush_stage<BT, DsT>(A, stl, stds, nr, pos, lane);
    }
    if (!(WM == WM_FILL) && A.count_rechecks) {
        if (rechecks) atomicAdd(&st->rechecks, rechecks);
        if (desc) atomicAdd(&st->descents, (unsigned long long)desc);
    }
}

// The batched walks as kernels: the counting walk at four wavefronts per SIMD,
// the record-filling walk at three (it would otherwise take 170 VGPRs and run
// two).
template <int PREC, int BT>
__global__ void __launch_bounds__(BT) __attribute__((amdgpu_waves_per_eu(4, 8)))
    k_walk_batched_count(const WalkGrid *__restrict__ grids, const WalkArgs *__restrict__ args,
                         const BatchChunk *__restrict__ chunks, int n_chunks, int refill_min, TraceStatus *st)
{
    walk_batched<PREC, WM_COUNT, BT>(grids, args, chunks, n_chunks, refill_min, st, nullptr);
}

template <int PREC, int BT>
__global__ void __launch_bounds__(BT) __attribute__((amdgpu_waves_per_eu(3, 8)))
    k_walk_batched_fill(const WalkGrid *__restrict__ grids, const WalkArgs *__restrict__ args,
                        const BatchChunk *__restrict__ chunks, int n_chunks, int refill_min, TraceStatus *st)
{
    extern __shared__ uint64_t lds_raw[];
    walk_batched<PREC, WM_FILL, BT>(grids, args, chunks, n_chunks, refill_min, st,
                                    reinterpret_cast<char *>(lds_raw));
}

template <int TREE, typename R>
__global__ void __launch_bounds__(TB) k_locate(WalkGrid G, const double *__restrict__ X, int64_t n,
                                               int32_t *__restrict__ out)
{
    const int64_t i = int64_t(blockIdx.x) * TB + threadIdx.x;
    if (i >= n) return;
    double x[3];
#pragma unroll
    for (int d = 0; d < 3; d++) x[d] = X[3 * i + d];
    if (!inside_closed(G, x)) {
        out[i] = -1;
        return;
    }
    double lo[3];
    int lv = 0;
    const R start = start_node<TREE, R>(G, x, 0, lv, lo);
    const R r = descend<TREE, R>(G, nullptr, 0u, start, lv, lo, x, 0, TIE_NONE);
    out[i] = r == Ref<R>::NUL ? -2 : int32_t(Ref<R>::id(r));
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

template <typename DsT>
__global__ void __launch_bounds__(TB)
    k_slab_compact(const int32_t *__restrict__ sleaf, const DsT *__restrict__ sds, int64_t slab,
                   const int32_t *__restrict__ count, const int64_t *__restrict__ offsets, int64_t n,
                   int32_t *__restrict__ leaf, DsT *__restrict__ ds)
{
    __shared__ int64_t off[CP + 1];
    const int64_t p0 = int64_t(blockIdx.x) * CP;
    const int np = int(n - p0 < CP ? n - p0 : CP);
    for (int j = threadIdx.x; j <= np; j += TB) off[j] = offsets[p0 + j];
    __syncthreads();
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
#pragma unroll
        for (int u = 0; u < CU; u++) {
            lf[u] = ok[u] ? sleaf[src[u]] : 0;
            dv[u] = ok[u] ? sds[src[u]] : DsT(0);
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

// As k_slab_compact for rows of (leaf, ds32) pairs: one 8-byte load per record.
__global__ void __launch_bounds__(TB)
    k_slab_compact_pairs(const uint2 *__restrict__ srow, int64_t slab, const int64_t *__restrict__ offsets,
                         int64_t n, int32_t *__restrict__ leaf, float *__restrict__ ds)
{
    __shared__ int64_t off[CP + 1];
    const int64_t p0 = int64_t(blockIdx.x) * CP;
    const int np = int(n - p0 < CP ? n - p0 : CP);
    for (int j = threadIdx.x; j <= np; j += TB) off[j] = offsets[p0 + j];
    __syncthreads();
    const int64_t d0 = off[0], d1 = off[np];
    int lo = 0;
    for (int64_t db = d0 + threadIdx.x; db < d1; db += int64_t(CU) * TB) {
        int64_t src[CU];
        bool ok[CU];
#pragma unroll
        for (int u = 0; u < CU; u++) {
            const int64_t d = db + int64_t(u) * TB;
            int hi = np;
            while (hi - lo > 1) {
                const int mid = (lo + hi) >> 1;
                if (off[mid] <= d) lo = mid;
                else hi = mid;
            }
            ok[u] = d < d1 && d - off[lo] < slab;
            src[u] = (p0 + lo) * slab + (d - off[lo]);
        }
        uint2 v[CU];
#pragma unroll
        for (int u = 0; u < CU; u++) v[u] = ok[u] ? srow[src[u]] : make_uint2(0u, 0u);
#pragma unroll
        for (int u = 0; u < CU; u++) {
            const int64_t d = db + int64_t(u) * TB;
            if (ok[u]) {
                leaf[d] = int32_t(v[u].x);
                ds[d] = __uint_as_float(v[u].y);
            }
        }
    }
}

constexpr size_t LDS_BYTES = 16384;          // top-level child references per block
constexpr int64_t PERSIST_CHUNK = int64_t(1) << 30;

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

// LDS a block may allocate on the current device (cached per device).
inline size_t max_block_lds()
{
    constexpr int MAXDEV = 64;
    static std::atomic<size_t> v[MAXDEV];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAXDEV) return 65536;
    size_t r = v[dev].load(std::memory_order_relaxed);
    if (!r) {
        int b = 0;
        r = hipDeviceGetAttribute(&b, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess && b > 0
                ? size_t(b)
                : 65536;
        v[dev].store(r, std::memory_order_relaxed);
    }
    return r;
}

template <int TREE, int PREC, int WM, typename R, int BT>
int launch_persistent(const WalkGrid &G, const WalkArgs &A, const hg_trace_opts *o, hipStream_t s)
{
    const int nc = TREE == OCT ? 8 : 2;
    // record modes stage records in LDS behind the top-level child references
    const size_t stage = WM == WM_COUNT ? 0
                                        : size_t(BT) * StageShape<BT>::SP * (4 + (PREC == HG_FP64 ? 8 : 4));
    const size_t cap = max_block_lds();
    if (stage + 16 > cap) return HG_E_INVAL;
    const size_t want = std::min(o->lds_bytes < 0 ? 0 : (o->lds_bytes == 0 ? LDS_BYTES : size_t(o->lds_bytes)),
                                 cap - stage - 16);
    const uint32_t lds_n = uint32_t(std::min<uint64_t>(G.n_internal, want / (sizeof(R) * size_t(nc))));
    const uint32_t stage_off = uint32_t((size_t(lds_n) * nc * sizeof(R) + 15) & ~size_t(15));
    const size_t lds = stage_off + stage;
    unsigned blocks = 0;
    int rc = persistent_blocks<TREE, PREC, WM, R, BT>(lds, &blocks);
    if (rc) return rc;
    const uint32_t chunk = o->chunk > 0 ? uint32_t(o->chunk) : 128u;
    const int refill_min = o->refill_min > 0 ? std::min(o->refill_min, 64) : 16;
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
        }
        k_reset_counter<<<1, 1, 0, s>>>(A.st);
        HG_CHECK(hipGetLastError());
        k_walk_persistent<TREE, PREC, WM, R, BT><<<dim3(blocks), dim3(BT), lds, s>>>(G, B, lds_n, chunk,
                                                                                         refill_min, stage_off);
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
int launch_batched_t(const WalkGrid *grids, const WalkArgs *args, const BatchChunk *chunks,
                     int n_chunks, int refill_min, TraceStatus *st, hipStream_t s)
{
    const size_t lds = WM == WM_FILL ? size_t(BT) * StageShape<BT>::SP * (4 + (PREC == HG_FP64 ? 8 : 4)) : 0;
    if (lds > max_block_lds()) return HG_E_INVAL;
    const void *kern = WM == WM_FILL ? reinterpret_cast<const void *>(k_walk_batched_fill<PREC, BT>)
                                     : reinterpret_cast<const void *>(k_walk_batched_count<PREC, BT>);
    unsigned blocks = 0;
    {
        const int rc = occupancy_blocks(kern, BT, lds, &blocks);
        if (rc) return rc;
    }
    k_reset_counter<<<1, 1, 0, s>>>(st);
    HG_CHECK(hipGetLastError());
    if (WM == WM_FILL)
        k_walk_batched_fill<PREC, BT><<<dim3(blocks), dim3(BT), lds, s>>>(grids, args, chunks, n_chunks,
                                                                          refill_min, st);
    else
        k_walk_batched_count<PREC, BT><<<dim3(blocks), dim3(BT), 0, s>>>(grids, args, chunks, n_chunks,
                                                                         refill_min, st);
    HG_CHECK(hipGetLastError());
    return HG_OK;
}

template <int PREC, int WM>
int launch_batched_b(const WalkGrid *grids, const WalkArgs *args, const BatchChunk *chunks,
                     int n_chunks, int block, int refill_min, TraceStatus *st, hipStream_t s)
{
    switch (block) {
    case 128: return launch_batched_t<PREC, WM, 128>(grids, args, chunks, n_chunks, refill_min, st, s);
    case 512: return launch_batched_t<PREC, WM, 512>(grids, args, chunks, n_chunks, refill_min, st, s);
    default: return launch_batched_t<PREC, WM, 256>(grids, args, chunks, n_chunks, refill_min, st, s);
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
    G.table = g->table;
    G.tdep = g->table ? g->tdep : 0;
    return G;
}

int launch_walk_args(const hg_grid *g, const WalkArgs &A, const hg_trace_opts *opts, int wm,
                     hipStream_t s)
{
    // bit 0: persistent counting / tau-only / slab walk, bit 1: persistent fill walk
    const int mode = opts->persistent < 0 ? 3 : opts->persistent;
    const int persistent = wm == WM_FILL ? (mode >> 1) & 1 : mode & 1;
    const WalkGrid G = walk_grid(g, opts->precision);
    const int prec = opts->precision;
    if (g->tree == KD)
        return g->wide ? dispatch_walk<KD, uint64_t>(G, A, prec, wm, persistent, opts, s)
                       : dispatch_walk<KD, uint32_t>(G, A, prec, wm, persistent, opts, s);
    return g->wide ? dispatch_walk<OCT, uint64_t>(G, A, prec, wm, persistent, opts, s)
                   : dispatch_walk<OCT, uint32_t>(G, A, prec, wm, persistent, opts, s);
}

int launch_walk(const hg_grid *g, const double *o, const double *k, int64_t n,
                const hg_trace_opts *opts, hg_trace_out *out, int wm, hipStream_t s, float *ms)
{
    (void)ms;
    return launch_walk_args(g, walk_args(g, o, k, n, opts, out), opts, wm, s);
}

WalkArgs walk_args(const hg_grid *g, const double *o, const double *k, int64_t n,
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
    A.st = g->status;
    A.count_rechecks = (opts->flags & HG_FLAG_RECHECKS) ? 1 : 0;
    A.slab = 0;
    A.resume = nullptr;
    A.n_resume = nullptr;
    A.pairs = 0;
    return A;
}

int launch_batched(const WalkGrid *grids, const WalkArgs *args, const BatchChunk *chunks,
                   int n_chunks, const hg_trace_opts *opts, bool fill, TraceStatus *st,
                   hipStream_t s)
{
    const int refill_min = opts->refill_min > 0 ? std::min(opts->refill_min, 64) : 16;
    const int b = opts->block;
    if (opts->precision == HG_FP64)
        return fill ? launch_batched_b<HG_FP64, WM_FILL>(grids, args, chunks, n_chunks, b, refill_min, st, s)
                    : launch_batched_b<HG_FP64, WM_COUNT>(grids, args, chunks, n_chunks, b, refill_min, st, s);
    return fill ? launch_batched_b<HG_FP32_RECHECK, WM_FILL>(grids, args, chunks, n_chunks, b, refill_min, st, s)
                : launch_batched_b<HG_FP32_RECHECK, WM_COUNT>(grids, args, chunks, n_chunks, b, refill_min, st, s);
}

int launch_slab_compact(const void *sleaf, const void *sds, int64_t slab, int precision, int pairs,
                        const int32_t *count, const int64_t *offsets, int64_t n, int32_t *leaf, void *ds,
                        hipStream_t s)
{
    if (n == 0) return HG_OK;
    const int64_t nb = (n + CP - 1) / CP;
    if (nb > 0x7fffffff) return HG_E_LIMIT;
    const unsigned blocks = unsigned(nb);
    if (pairs && precision != HG_FP64)
        k_slab_compact_pairs<<<blocks, TB, 0, s>>>((const uint2 *)sleaf, slab, offsets, n, leaf, (float *)ds);
    else if (precision == HG_FP64)
        k_slab_compact<double><<<blocks, TB, 0, s>>>((const int32_t *)sleaf, (const double *)sds, slab,
                                                     count, offsets, n, leaf, (double *)ds);
    else
        k_slab_compact<float><<<blocks, TB, 0, s>>>((const int32_t *)sleaf, (const float *)sds, slab,
                                                    count, offsets, n, leaf, (float *)ds);
    HG_CHECK(hipGetLastError());
    return HG_OK;
}

int launch_locate(const hg_grid *g, const double *p, int64_t n, int32_t *leaf, hipStream_t s)
{
    const WalkGrid G = walk_grid(g, HG_FP64);
    const int64_t nb = (n + TB - 1) / TB;
    if (nb == 0) return HG_OK;
    const dim3 grid{unsigned(nb), 1u, 1u}, block{unsigned(TB), 1u, 1u};
    if (g->tree == KD) {
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
