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

#include "common.h"

namespace hg {

namespace {

constexpr int TB = 256;
constexpr int64_t STEP_GUARD = int64_t(1) << 26;

// 2^e for a normal exponent.
__device__ inline double pow2(int e) { return __hiloint2double((e + 1023) << 20, 0); }

// Side of a split plane c on axis d that holds the point whose coordinate is
// x.  Off the plane the comparison decides.  On it: the axis of the face just
// crossed goes to the side the path moves to; a plane on the boundary of the
// leaf just left keeps the point inside that leaf's slab; otherwise the
// direction decides, a zero component going to the upper side.  With no face
// crossed (first leaf of a path, point location) olo/ohi are NaN and a = -1.
__device__ inline int upper_side(double x, double c, int d, int a, double kd, double olo,
                                 double ohi)
{
    if (x > c) return 1;
    if (x < c) return 0;
    if (d == a) return kd > 0.0;
    if (c == ohi) return 0;
    if (c == olo) return 1;
    return !(kd < 0.0);
}

// True when ref may be dereferenced: a leaf or internal id inside the arrays.
__device__ inline bool ref_ok(const WalkGrid &G, uint32_t ref)
{
    return ref != NULL_REF && ref_id(ref) < (ref_is_leaf(ref) ? G.n_leaves : G.n_internal);
}

// Descend from the internal node `ref` (level lv, cell coordinates c) to the
// leaf holding q.  Returns NULL_REF if a reference is out of range or the
// depth exceeds the format's limit (never for a valid layout).
template <int TREE>
__device__ inline uint32_t descend(const WalkGrid &G, uint32_t ref, int &lv, uint32_t c[3],
                                   const double q[3], int a, const double k[3],
                                   const double olo[3], const double ohi[3])
{
    while (!ref_is_leaf(ref)) {
        if (!ref_ok(G, ref) || lv >= 62) return NULL_REF;
        const uint32_t id = ref_id(ref);
        if (TREE == KD) {
            const int b = lv % 3;
            uint32_t cb = 0;
            double qb = 0, kb = 0, lob = 0, hib = 0, dlo = 0;
#pragma unroll
            for (int d = 0; d < 3; d++)
                if (d == b) {
                    cb = c[d]; qb = q[d]; kb = k[d]; lob = olo[d]; hib = ohi[d]; dlo = G.lo[d];
                }
            const double mid = dlo + double(2u * cb + 1u) * pow2(G.lg - lv / 3 - 1);
            const int up = upper_side(qb, mid, b, a, kb, lob, hib);
            ref = G.child[2u * id + uint32_t(up)];
#pragma unroll
            for (int d = 0; d < 3; d++)
                if (d == b) c[d] = 2u * cb + uint32_t(up);
        } else {
            const double w = pow2(G.lg - lv - 1);
            int idx = 0;
#pragma unroll
            for (int d = 0; d < 3; d++) {
                const double mid = G.lo[d] + double(2u * c[d] + 1u) * w;
                const int up = upper_side(q[d], mid, d, a, k[d], olo[d], ohi[d]);
                idx |= up << d;
                c[d] = 2u * c[d] + uint32_t(up);
            }
            ref = G.child[8u * id + uint32_t(idx)];
        }
        lv++;
    }
    return ref_ok(G, ref) ? ref : NULL_REF;
}

__device__ inline bool inside_closed(const WalkGrid &G, const double x[3])
{
    bool in = true;
#pragma unroll
    for (int d = 0; d < 3; d++) in = in && (x[d] >= G.lo[d] && x[d] <= G.lo[d] + G.side);
    return in;
}

// Start of the path inside the closed domain: the origin itself, or the entry
// point found by the slab test, placed exactly on the entry face.
__device__ inline bool clip_ray(const WalkGrid &G, const double p0[3], const double k[3],
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

struct LeafData {
    uint32_t rope[6];
    double rho64;
    float rho32;
};

template <int PREC>
__device__ inline LeafData load_leaf(const WalkGrid &G, uint32_t id)
{
    LeafData L;
    if (PREC == HG_FP64) {
        const uint4 *r = reinterpret_cast<const uint4 *>(G.rec64 + id);
        const uint4 a = r[0], b = r[1];
        L.rope[0] = a.x; L.rope[1] = a.y; L.rope[2] = a.z; L.rope[3] = a.w;
        L.rope[4] = b.x; L.rope[5] = b.y;
        L.rho64 = __hiloint2double(int(b.w), int(b.z));
        L.rho32 = 0.f;
    } else {
        const uint4 *r = reinterpret_cast<const uint4 *>(G.rec32 + id);
        const uint4 a = r[0], b = r[1];
        L.rope[0] = a.x; L.rope[1] = a.y; L.rope[2] = a.z; L.rope[3] = a.w;
        L.rope[4] = b.x; L.rope[5] = b.y;
        L.rho32 = __uint_as_float(b.z);
        L.rho64 = 0.0;
    }
    return L;
}

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
    TraceStatus *st;
    int count_rechecks;
};

template <int TREE, int PREC, bool FILL>
__device__ void walk_ray(const WalkGrid &G, const WalkArgs &A, int64_t i)
{
    double p0[3], k[3], inv[3], ainv[3];
#pragma unroll
    for (int d = 0; d < 3; d++) {
        p0[d] = A.O[3 * i + d];
        k[d] = A.K[3 * i + d];
    }
    const double nn = k[0] * k[0] + k[1] * k[1] + k[2] * k[2];
    const bool finite = isfinite(k[0]) && isfinite(k[1]) && isfinite(k[2]);
    if (!finite || !(fabs(sqrt(nn) - 1.0) <= 1e-6)) {
        if (!FILL) {
            A.tau[i] = __longlong_as_double(0x7ff8000000000000ll);
            A.count[i] = 0;
            A.st->bad_dir = 1;
        }
        return;
    }
#pragma unroll
    for (int d = 0; d < 3; d++) {
        inv[d] = 1.0 / k[d];
        ainv[d] = fabs(inv[d]);
    }
    double s, p[3];
    if (!clip_ray(G, p0, k, inv, s, p)) {
        if (!FILL) {
            A.tau[i] = 0.0;
            A.count[i] = 0;
        }
        return;
    }
    // FP32 exit decision is used only where its error bound holds.
    float ainv32[3];
    bool force64 = false;
#pragma unroll
    for (int d = 0; d < 3; d++) {
        ainv32[d] = float(ainv[d]);
        if (k[d] != 0.0 && !(fabs(k[d]) >= 1e-30)) force64 = true;
    }
    const double nanv = __longlong_as_double(0x7ff8000000000000ll);
    double olo[3] = {nanv, nanv, nanv}, ohi[3] = {nanv, nanv, nanv};
    uint32_t c[3] = {0u, 0u, 0u};
    int lv = 0;
    uint32_t ref = descend<TREE>(G, G.root, lv, c, p, -1, k, olo, ohi);
    if (ref == NULL_REF) {
        A.st->bad_ref = 1;
        if (!FILL) {
            A.tau[i] = 0.0;
            A.count[i] = 0;
        }
        return;
    }

    double tau64 = 0.0;
    float tau32 = 0.f, comp32 = 0.f;
    const float kappa32 = float(A.kappa);
    int32_t cnt = 0;
    const int64_t base = FILL ? A.offsets[i] : 0;
    const int64_t room = FILL ? A.offsets[i + 1] - base : 0;
    unsigned long long rechecks = 0;
    for (int64_t step = 0;; step++) {
        if (step >= STEP_GUARD) {
            A.st->step_guard = 1;
            break;
        }
        const uint32_t id = ref_id(ref);
        const LeafData L = load_leaf<PREC>(G, id);
        double lo[3], hi[3], D[3];
        int dep[3];
#pragma unroll
        for (int d = 0; d < 3; d++) {
            dep[d] = axis_depth(TREE, lv, d);
            const double w = pow2(G.lg - dep[d]);
            lo[d] = G.lo[d] + double(c[d]) * w;
            hi[d] = G.lo[d] + double(c[d] + 1u) * w;
            D[d] = k[d] > 0.0 ? hi[d] - p[d] : p[d] - lo[d];
        }
        int a = -1;
        if (PREC == HG_FP32_RECHECK) {
            float m1 = INFINITY, m2 = INFINITY;
            int i1 = -1;
#pragma unroll
            for (int d = 0; d < 3; d++) {
                float t = k[d] == 0.0 ? INFINITY : float(D[d]) * ainv32[d];
                if (t < m1) {
                    m2 = m1;
                    m1 = t;
                    i1 = d;
                } else if (t < m2) {
                    m2 = t;
                }
            }
            const float hmin = float(pow2(G.lg - dep[0]));
            if (force64 || !(m2 - m1 >= 1e-5f * hmin)) {
                rechecks++;
                i1 = -1;
            }
            a = i1;
        }
        if (a < 0) {
            double tmin = INFINITY;
#pragma unroll
            for (int d = 0; d < 3; d++) {
                double t = k[d] == 0.0 ? INFINITY : D[d] * ainv[d];
                if (t != t) t = INFINITY;
                if (t < tmin) {
                    tmin = t;
                    a = d;
                }
            }
        }
        if (a < 0) {
            A.st->step_guard = 1;
            break;
        }
        double Da = 0, ka = 0, aia = 0, loa = 0, hia = 0;
        uint32_t ca = 0;
        int depa = 0;
#pragma unroll
        for (int d = 0; d < 3; d++)
            if (d == a) {
                Da = D[d]; ka = k[d]; aia = ainv[d]; loa = lo[d]; hia = hi[d]; ca = c[d]; depa = dep[d];
            }
        double ds = Da * aia;
        if (ds != ds) ds = INFINITY;
        if (ds > 0.0) {
            if (FILL) {
                if (cnt >= room) {
                    A.st->step_guard = 1;  // the fill walk must repeat the counting walk
                    break;
                }
                const int64_t pos = base + cnt;
                A.leaf[pos] = int32_t(id);
                if (PREC == HG_FP64) reinterpret_cast<double *>(A.ds)[pos] = ds;
                else reinterpret_cast<float *>(A.ds)[pos] = float(ds);
            } else {
                if (PREC == HG_FP64) {
                    tau64 = tau64 + A.kappa * L.rho64 * ds;
                } else {
                    const float y = kappa32 * L.rho32 * float(ds) - comp32;
                    const float t = tau32 + y;
                    comp32 = (t - tau32) - y;
                    tau32 = t;
                }
            }
            cnt++;
        }
        const bool up = ka > 0.0;
        if (up ? (ca + 1u == (1u << depa)) : (ca == 0u)) break;
        // re-anchor the exit point on the crossed face
        s = s + ds;
        double q[3];
#pragma unroll
        for (int d = 0; d < 3; d++) {
            if (d == a) {
                q[d] = up ? hia : loa;
            } else {
                const double v = p0[d] + s * k[d];
                q[d] = v < lo[d] ? lo[d] : (v > hi[d] ? hi[d] : v);
            }
        }
        // rope of the exit face, then descend to the leaf holding the exit point
        const int face = 2 * a + (up ? 1 : 0);
        uint32_t nref = L.rope[0];
#pragma unroll
        for (int f = 1; f < 6; f++)
            if (f == face) nref = L.rope[f];
        // Cell coordinates of the rope target.  It is never finer than the
        // leaf across the face; along the exit axis a k-d target may be one
        // level finer (the half of a same-size neighbour touching the face).
        const int nlv = ref_level(nref);
#pragma unroll
        for (int d = 0; d < 3; d++) {
            const int dn = axis_depth(TREE, nlv, d);
            uint32_t cd = c[d];
            if (d == a) {
                if (dn >= dep[d]) cd = up ? (cd + 1u) << (dn - dep[d]) : (cd << (dn - dep[d])) - 1u;
                else cd = (up ? cd + 1u : cd - 1u) >> (dep[d] - dn);
            } else {
                cd = cd >> (dep[d] - dn);
            }
            c[d] = cd;
        }
        if (nref == NULL_REF) {
            A.st->bad_ref = 1;
            break;
        }
        lv = nlv;
        ref = descend<TREE>(G, nref, lv, c, q, a, k, lo, hi);
        if (ref == NULL_REF) {
            A.st->bad_ref = 1;
            break;
        }
#pragma unroll
        for (int d = 0; d < 3; d++) p[d] = q[d];
    }
    if (!FILL) {
        A.count[i] = cnt;
        if (PREC == HG_FP64) A.tau[i] = tau64;
        else A.tau[i] = double(tau32) - double(comp32);
    }
    if (!FILL && A.count_rechecks && rechecks) atomicAdd(&A.st->rechecks, rechecks);
}

template <int TREE, int PREC, bool FILL>
__global__ void __launch_bounds__(TB) k_walk(WalkGrid G, WalkArgs A)
{
    const int64_t i = int64_t(blockIdx.x) * TB + threadIdx.x;
    if (i < A.n) walk_ray<TREE, PREC, FILL>(G, A, i);
}

template <int TREE>
__global__ void __launch_bounds__(TB) k_locate(WalkGrid G, const double *__restrict__ P, int64_t n,
                                               int32_t *__restrict__ out)
{
    const int64_t i = int64_t(blockIdx.x) * TB + threadIdx.x;
    if (i >= n) return;
    double x[3];
#pragma unroll
    for (int d = 0; d < 3; d++) x[d] = P[3 * i + d];
    if (!inside_closed(G, x)) {
        out[i] = -1;
        return;
    }
    const double nanv = __longlong_as_double(0x7ff8000000000000ll);
    const double z[3] = {0.0, 0.0, 0.0};
    const double nn[3] = {nanv, nanv, nanv};
    uint32_t c[3] = {0u, 0u, 0u};
    int lv = 0;
    const uint32_t r = descend<TREE>(G, G.root, lv, c, x, -1, z, nn, nn);
    out[i] = r == NULL_REF ? -2 : int32_t(ref_id(r));
}

template <int TREE, int PREC, bool FILL>
int launch_t(const WalkGrid &G, const WalkArgs &A, int block, hipStream_t s)
{
    (void)block;
    const int64_t nb = (A.n + TB - 1) / TB;
    if (nb == 0) return HG_OK;
    k_walk<TREE, PREC, FILL><<<dim3(unsigned(nb)), dim3(TB), 0, s>>>(G, A);
    HG_CHECK(hipGetLastError());
    return HG_OK;
}

}  // namespace

WalkGrid walk_grid(const hg_grid *g)
{
    WalkGrid G;
    G.tree = g->tree;
    for (int d = 0; d < 3; d++) G.lo[d] = g->lo[d];
    G.side = g->side;
    int e = 0;
    frexp(g->side, &e);
    G.lg = e - 1;
    G.root = g->root_ref;
    G.n_leaves = uint32_t(g->n_leaves);
    G.n_internal = uint32_t(g->n_internal);
    G.rec32 = g->rec32;
    G.rec64 = g->rec64;
    G.child = g->child;
    return G;
}

int launch_walk(const hg_grid *g, const double *o, const double *k, int64_t n,
                const hg_trace_opts *opts, hg_trace_out *out, bool fill, hipStream_t s, float *ms)
{
    (void)ms;
    const WalkGrid G = walk_grid(g);
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
    A.st = g->status;
    A.count_rechecks = (opts->flags & HG_FLAG_RECHECKS) ? 1 : 0;
    const int prec = opts->precision;
    if (g->tree == KD) {
        if (prec == HG_FP64)
            return fill ? launch_t<KD, HG_FP64, true>(G, A, opts->block, s)
                        : launch_t<KD, HG_FP64, false>(G, A, opts->block, s);
        return fill ? launch_t<KD, HG_FP32_RECHECK, true>(G, A, opts->block, s)
                    : launch_t<KD, HG_FP32_RECHECK, false>(G, A, opts->block, s);
    }
    if (prec == HG_FP64)
        return fill ? launch_t<OCT, HG_FP64, true>(G, A, opts->block, s)
                    : launch_t<OCT, HG_FP64, false>(G, A, opts->block, s);
    return fill ? launch_t<OCT, HG_FP32_RECHECK, true>(G, A, opts->block, s)
                : launch_t<OCT, HG_FP32_RECHECK, false>(G, A, opts->block, s);
}

int launch_locate(const hg_grid *g, const double *p, int64_t n, int32_t *leaf, hipStream_t s)
{
    const WalkGrid G = walk_grid(g);
    const int64_t nb = (n + TB - 1) / TB;
    if (nb == 0) return HG_OK;
    if (g->tree == KD) k_locate<KD><<<dim3(unsigned(nb)), dim3(TB), 0, s>>>(G, p, n, leaf);
    else k_locate<OCT><<<dim3(unsigned(nb)), dim3(TB), 0, s>>>(G, p, n, leaf);
    HG_CHECK(hipGetLastError());
    return HG_OK;
}

}  // namespace hg
