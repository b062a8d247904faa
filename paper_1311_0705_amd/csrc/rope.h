// Face ropes and encoded references of the walk layout, shared by the
// single-grid and the batched builders.
//
// Ropes stand in for the per-wall neighbor lists of Sect. 2.3: a leaf's rope
// through face f is the smallest node that contains the whole region just
// across f.  A child inherits its parent's ropes on the faces it shares with
// the parent, points at its sibling across the new split plane, and every
// rope is then pushed down while a single child of the target still contains
// the face region.
#pragma once

#include "common.h"

namespace hg {

// Integer extent of node n (level `level`) along each axis in units of
// 2^-DEPTH_BITS of the domain side.
__device__ inline void int_extent(int tree, int level, int64_t n, const uint32_t *__restrict__ geom,
                                  const uint32_t c[3], uint32_t lo[3], uint32_t hi[3])
{
#pragma unroll
    for (int d = 0; d < 3; d++) {
        int sh = DEPTH_BITS - node_depth(tree, level, geom, n, d);
        lo[d] = c[d] << sh;
        hi[d] = (c[d] + 1u) << sh;
    }
}

// Push rope target n down while one child of it holds the whole region across
// face (axis a, upper side `up`) of the node with extent [clo, chi).
__device__ inline int32_t push_down(int tree, int32_t n, int a, int up, const uint32_t clo[3],
                             const uint32_t chi[3], const int32_t *__restrict__ fc,
                             const uint8_t *__restrict__ level, const uint32_t *__restrict__ coord,
                             const uint32_t *__restrict__ geom)
{
    if (n < 0) return n;
    for (;;) {
        int32_t f = fc[n];
        if (f < 0) return n;
        int lv = level[n];
        if (tree != OCT) {
            int b = node_axis(tree, lv, geom, n);
            int side;
            if (b == a) {
                side = up ? 0 : 1;   // the half of the target adjacent to the face
            } else {
                uint32_t mid = (2u * coord[3 * n + b] + 1u)
                               << (DEPTH_BITS - node_depth(tree, lv, geom, n, b) - 1);
                if (chi[b] <= mid) side = 0;
                else if (clo[b] >= mid) side = 1;
                else return n;
            }
            n = f + side;
        } else {
            int idx = 0;
#pragma unroll
            for (int d = 0; d < 3; d++) {
                int bit;
                if (d == a) {
                    bit = up ? 0 : 1;
                } else {
                    uint32_t mid = (2u * coord[3 * n + d] + 1u) << (DEPTH_BITS - lv - 1);
                    if (chi[d] <= mid) bit = 0;
                    else if (clo[d] >= mid) bit = 1;
                    else return n;
                }
                idx |= bit << d;
            }
            n = f + idx;
        }
    }
}

// The six ropes of child k of node p (whose own ropes are final), as
// child_rope for every face with the node's loads shared.
__device__ inline void child_ropes(int tree, int64_t p, int k, const int32_t *__restrict__ fc,
                                   const uint8_t *__restrict__ level,
                                   const uint32_t *__restrict__ coord, int32_t *__restrict__ rope,
                                   const uint32_t *__restrict__ geom = nullptr)
{
    const int32_t f = fc[p];
    if (f < 0) return;
    const int lv = level[p];
    const int32_t child = f + k;
    int32_t r[6];
#pragma unroll
    for (int j = 0; j < 6; j++) r[j] = rope[6 * p + j];
    if (tree != OCT) {
        const int a = node_axis(tree, lv, geom, p);
        if (k == 0) r[2 * a + 1] = f + 1;
        else r[2 * a] = f;
    } else {
#pragma unroll
        for (int d = 0; d < 3; d++) {
            if (((k >> d) & 1) == 0) r[2 * d + 1] = f + (k | (1 << d));
            else r[2 * d] = f + (k & ~(1 << d));
        }
    }
    const uint32_t c[3] = {coord[3 * child], coord[3 * child + 1], coord[3 * child + 2]};
    uint32_t clo[3], chi[3];
    int_extent(tree, lv + 1, child, geom, c, clo, chi);
#pragma unroll
    for (int j = 0; j < 6; j++)
        rope[6 * int64_t(child) + j] = push_down(tree, r[j], j / 2, j % 2, clo, chi, fc, level, coord, geom);
}

// Rope of face j (axis j / 2, upper side if j is odd) of child k of node p,
// whose own ropes are final; nothing when p is a leaf.  A face between two
// siblings leads to the sibling, any other face to the parent's rope target;
// either is pushed down to the smallest node that still covers the face.
__device__ inline void child_rope(int tree, int64_t p, int k, int j, const int32_t *__restrict__ fc,
                                  const uint8_t *__restrict__ level, const uint32_t *__restrict__ coord,
                                  int32_t *__restrict__ rope, const uint32_t *__restrict__ geom = nullptr)
{
    const int32_t f = fc[p];
    if (f < 0) return;
    const int lv = level[p];
    const int32_t child = f + k;
    const int d = j / 2, up = j % 2;
    int32_t r;
    if (tree != OCT) {
        const int a = node_axis(tree, lv, geom, p);
        if (d == a && k == 0 && up) r = f + 1;
        else if (d == a && k == 1 && !up) r = f;
        else r = rope[6 * p + j];
    } else {
        const int bit = (k >> d) & 1;
        if (!bit && up) r = f + (k | (1 << d));
        else if (bit && !up) r = f + (k & ~(1 << d));
        else r = rope[6 * p + j];
    }
    const uint32_t c[3] = {coord[3 * child], coord[3 * child + 1], coord[3 * child + 2]};
    uint32_t clo[3], chi[3];
    int_extent(tree, lv + 1, child, geom, c, clo, chi);
    rope[6 * int64_t(child) + j] = push_down(tree, r, d, up, clo, chi, fc, level, coord, geom);
}

// Encoded reference of node n (see Ref) in a tree whose nodes have nc
// children: a leaf, an internal node, or a twin (an internal node whose
// children are all leaves; they are consecutive in the breadth-first list,
// so their leaf ranks are too).
// With geom (a gradient k-d tree, wide references) the reference also
// carries the node's halvings along x and y and its split axis.
template <typename R>
__device__ inline R encode(int32_t n, int nc, const int32_t *__restrict__ fc, const uint8_t *__restrict__ level,
                           const int32_t *__restrict__ leaf_of, const int32_t *__restrict__ int_of,
                           const uint32_t *__restrict__ geom = nullptr)
{
    if (n < 0) return Ref<R>::NUL;
    const int32_t f = fc[n];
    int kind;
    uint64_t id;
    if (f < 0) {
        kind = Ref<R>::LEAF;
        id = uint64_t(uint32_t(leaf_of[n]));
    } else {
        bool all = true;
        for (int k = 0; k < nc; k++) all = all && fc[f + k] < 0;
        kind = all ? Ref<R>::TWIN : Ref<R>::INTERNAL;
        id = all ? uint64_t(uint32_t(leaf_of[f])) : uint64_t(uint32_t(int_of[n]));
    }
    if (!geom) return Ref<R>::make(kind, level[n], id);
    const uint32_t gm = geom[n];
    return Ref<R>::make_geo(kind, level[n], id, geom_depth(gm, 0), geom_depth(gm, 1), geom_axis(gm));
}

// k-d jump reference from internal node i for the side triple c (s0 s1 s2 =
// bits 2 1 0 of c; s_j is the side taken at level(i) + j): the node reached
// by descending at most three levels with those sides: the first leaf met, a
// twin's leaf child when a side is left for it, else the node three levels
// down (internal or twin).
template <typename R>
__device__ inline R jump_ref(int32_t i, int c, const int32_t *__restrict__ fc, const uint8_t *__restrict__ level,
                             const int32_t *__restrict__ leaf_of, const int32_t *__restrict__ int_of)
{
    int32_t m = i;
    R r = Ref<R>::NUL;
    for (int j = 0; j < 3; j++) {
        const int32_t ch = fc[m] + ((c >> (2 - j)) & 1);
        r = encode<R>(ch, 2, fc, level, leaf_of, int_of);
        if (Ref<R>::leaf(r)) break;
        if (Ref<R>::twin(r)) {
            if (j < 2) r = encode<R>(fc[ch] + ((c >> (1 - j)) & 1), 2, fc, level, leaf_of, int_of);
            break;
        }
        m = ch;
    }
    return r;
}

// Grid density of a leaf = M/V = S/N (Sect. 3.2), or the imported value.
__device__ inline double leaf_rho(int64_t l, int32_t n, const double *S, const double *rho_in,
                                  double n_samples)
{
    return rho_in ? rho_in[l] : S[n] / n_samples;
}

// Node holding the whole locate-table cell c (per-axis depth tdep): descend
// from the root by the cell's index bits while the node is internal and its
// split does not cut the cell (the halvings of the split axis are below
// tdep; for the cyclic k-d tree that is below the table level).
__device__ inline int32_t table_node(int tree, int tdep, const uint32_t c[3],
                                     const int32_t *__restrict__ fc, const uint8_t *__restrict__ level,
                                     const uint32_t *__restrict__ geom = nullptr)
{
    const int lt = table_level(tree, tdep);
    int32_t n = 0;
    for (;;) {
        const int32_t f = fc[n];
        const int lv = level[n];
        if (f < 0) return n;
        if (tree != OCT) {
            const int b = node_axis(tree, lv, geom, n);
            const int db = node_depth(tree, lv, geom, n, b);
            if (db >= tdep) return n;
            n = f + int32_t((c[b] >> (tdep - db - 1)) & 1u);
        } else {
            if (lv >= lt) return n;
            int idx = 0;
            for (int d = 0; d < 3; d++) idx |= int((c[d] >> (tdep - lv - 1)) & 1u) << d;
            n = f + idx;
        }
    }
}

}  // namespace hg
