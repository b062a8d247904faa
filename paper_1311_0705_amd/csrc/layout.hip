// Walk layout of a finished tree: face ropes, leaf / internal numbering, the
// 32-byte per-leaf walk records and the encoded child references.
//
// Ropes stand in for the per-wall neighbor lists of Sect. 2.3.  A leaf's rope
// through face f is the smallest node that contains the whole region just
// across f; the leaves of that node's subtree touching f are exactly the
// face's neighbor list, and the walk reaches the right one by descending from
// the rope target with the exit point.  Ropes are derived level by level: a
// child inherits its parent's ropes on the faces it shares with the parent,
// points at its sibling across the new split plane, and every rope is then
// pushed down while a single child of the target still contains the face
// region.
#include <stdlib.h>

#include "common.h"

namespace hg {

namespace {

constexpr int LT = 256;

// Integer extent of a node along each axis in units of 2^-DEPTH_BITS of the
// domain side.
__device__ inline void int_extent(int tree, int level, const uint32_t c[3], uint32_t lo[3],
                                  uint32_t hi[3])
{
#pragma unroll
    for (int d = 0; d < 3; d++) {
        int sh = DEPTH_BITS - axis_depth(tree, level, d);
        lo[d] = c[d] << sh;
        hi[d] = (c[d] + 1u) << sh;
    }
}

// Push rope target n down while one child of it holds the whole region across
// face (axis a, upper side `up`) of the node with extent [clo, chi).
__device__ int32_t push_down(int tree, int32_t n, int a, int up, const uint32_t clo[3],
                             const uint32_t chi[3], const int32_t *__restrict__ fc,
                             const uint8_t *__restrict__ level, const uint32_t *__restrict__ coord)
{
    if (n < 0) return n;
    for (;;) {
        int32_t f = fc[n];
        if (f < 0) return n;
        int lv = level[n];
        if (tree == KD) {
            int b = lv % 3;
            int side;
            if (b == a) {
                side = up ? 0 : 1;   // the half of the target adjacent to the face
            } else {
                uint32_t mid = (2u * coord[3 * n + b] + 1u)
                               << (DEPTH_BITS - axis_depth(KD, lv, b) - 1);
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

// One thread per (node of level l, child slot): the child's six ropes.
__global__ void __launch_bounds__(LT)
    k_child_ropes(int tree, int64_t begin, int64_t count, int nc, const int32_t *__restrict__ fc,
                  const uint8_t *__restrict__ level, const uint32_t *__restrict__ coord,
                  int32_t *__restrict__ rope)
{
    int64_t t = int64_t(blockIdx.x) * LT + threadIdx.x;
    if (t >= count * nc) return;
    int64_t p = begin + t / nc;
    int k = int(t % nc);
    int32_t f = fc[p];
    if (f < 0) return;
    int lv = level[p];
    int32_t child = f + k;
    int32_t r[6];
#pragma unroll
    for (int j = 0; j < 6; j++) r[j] = rope[6 * p + j];
    if (tree == KD) {
        int a = lv % 3;
        if (k == 0) r[2 * a + 1] = f + 1;
        else r[2 * a] = f;
    } else {
#pragma unroll
        for (int d = 0; d < 3; d++) {
            if (((k >> d) & 1) == 0) r[2 * d + 1] = f + (k | (1 << d));
            else r[2 * d] = f + (k & ~(1 << d));
        }
    }
    uint32_t c[3] = {coord[3 * child], coord[3 * child + 1], coord[3 * child + 2]};
    uint32_t clo[3], chi[3];
    int_extent(tree, lv + 1, c, clo, chi);
#pragma unroll
    for (int j = 0; j < 6; j++)
        rope[6 * int64_t(child) + j] = push_down(tree, r[j], j / 2, j % 2, clo, chi, fc, level, coord);
}

__global__ void __launch_bounds__(LT) k_flag_leaves(const int32_t *__restrict__ fc, int64_t n,
                                                    uint8_t *__restrict__ is_leaf)
{
    int64_t i = int64_t(blockIdx.x) * LT + threadIdx.x;
    if (i < n) is_leaf[i] = fc[i] < 0 ? 1 : 0;
}

// Leaf rank = number of leaves before the node; internal rank = the rest.
__global__ void __launch_bounds__(LT)
    k_number(const int32_t *__restrict__ fc, const int64_t *__restrict__ leaf_rank, int64_t n,
             int32_t *__restrict__ leaf_of, int32_t *__restrict__ int_of, int32_t *__restrict__ node_of)
{
    int64_t i = int64_t(blockIdx.x) * LT + threadIdx.x;
    if (i >= n) return;
    int64_t lr = leaf_rank[i];
    if (fc[i] < 0) {
        leaf_of[i] = int32_t(lr);
        int_of[i] = -1;
        node_of[lr] = int32_t(i);
    } else {
        leaf_of[i] = -1;
        int_of[i] = int32_t(i - lr);
    }
}

template <typename R>
__device__ inline R encode(int32_t n, const int32_t *__restrict__ fc, const uint8_t *__restrict__ level,
                           const int32_t *__restrict__ leaf_of, const int32_t *__restrict__ int_of)
{
    if (n < 0) return Ref<R>::NUL;
    const bool leaf = fc[n] < 0;
    return Ref<R>::make(leaf, level[n], uint64_t(uint32_t(leaf ? leaf_of[n] : int_of[n])));
}

// Grid density of a leaf = M/V = S/N (Sect. 3.2), or the imported value.
__device__ inline double leaf_rho(int64_t l, int32_t n, const double *S, const double *rho_in,
                                  double n_samples)
{
    return rho_in ? rho_in[l] : S[n] / n_samples;
}

__global__ void __launch_bounds__(LT)
    k_leaf_records(int64_t n_leaves, const int32_t *__restrict__ node_of,
                   const int32_t *__restrict__ fc, const uint8_t *__restrict__ level,
                   const int32_t *__restrict__ leaf_of, const int32_t *__restrict__ int_of,
                   const int32_t *__restrict__ rope, const double *__restrict__ S,
                   const double *__restrict__ rho_in, double n_samples, double *__restrict__ rho,
                   LeafRec32 *__restrict__ rec32, LeafRec64 *__restrict__ rec64)
{
    int64_t l = int64_t(blockIdx.x) * LT + threadIdx.x;
    if (l >= n_leaves) return;
    const int32_t n = node_of[l];
    const double r = leaf_rho(l, n, S, rho_in, n_samples);
    rho[l] = r;
    LeafRec32 a;
    LeafRec64 b;
#pragma unroll
    for (int j = 0; j < 6; j++) {
        const uint32_t e = encode<uint32_t>(rope[6 * int64_t(n) + j], fc, level, leaf_of, int_of);
        a.rope[j] = e;
        b.rope[j] = e;
    }
    a.rho = float(r);
    a.pad = 0;
    b.rho = r;
    rec32[l] = a;
    rec64[l] = b;
}

__global__ void __launch_bounds__(LT)
    k_leaf_records_wide(int64_t n_leaves, const int32_t *__restrict__ node_of,
                        const int32_t *__restrict__ fc, const uint8_t *__restrict__ level,
                        const int32_t *__restrict__ leaf_of, const int32_t *__restrict__ int_of,
                        const int32_t *__restrict__ rope, const double *__restrict__ S,
                        const double *__restrict__ rho_in, double n_samples,
                        double *__restrict__ rho, LeafRecW *__restrict__ recw)
{
    int64_t l = int64_t(blockIdx.x) * LT + threadIdx.x;
    if (l >= n_leaves) return;
    const int32_t n = node_of[l];
    const double r = leaf_rho(l, n, S, rho_in, n_samples);
    rho[l] = r;
    LeafRecW a;
#pragma unroll
    for (int j = 0; j < 6; j++)
        a.rope[j] = encode<uint64_t>(rope[6 * int64_t(n) + j], fc, level, leaf_of, int_of);
    a.rho64 = r;
    a.rho32 = float(r);
    a.pad = 0;
    recw[l] = a;
}

template <typename R>
__global__ void __launch_bounds__(LT)
    k_child_refs(int64_t n, int nc, const int32_t *__restrict__ fc, const uint8_t *__restrict__ level,
                 const int32_t *__restrict__ leaf_of, const int32_t *__restrict__ int_of,
                 R *__restrict__ child)
{
    int64_t t = int64_t(blockIdx.x) * LT + threadIdx.x;
    if (t >= n * nc) return;
    int64_t i = t / nc;
    int k = int(t % nc);
    int32_t f = fc[i];
    if (f < 0) return;
    child[int64_t(int_of[i]) * nc + k] = encode<R>(f + k, fc, level, leaf_of, int_of);
}

inline unsigned blocks_for(int64_t n) { return unsigned((n + LT - 1) / LT); }

}  // namespace

int finalize_layout(hg_grid *g, const double *rho_leaf, int n_samples, hipStream_t s)
{
    const int64_t N = g->n_nodes;
    const int nc = g->tree == OCT ? 8 : 2;
    // ropes, level by level from the root (whose faces are all domain faces)
    HG_CHECK(hipMemsetAsync(g->rope, 0xFF, size_t(6) * sizeof(int32_t), s));
    for (int l = 0; l < g->max_level; l++) {
        int64_t b = g->level_begin[l], e = g->level_begin[l + 1];
        if (e <= b) continue;
        k_child_ropes<<<blocks_for((e - b) * nc), LT, 0, s>>>(g->tree, b, e - b, nc, g->first_child,
                                                              g->level, g->coord, g->rope);
        HG_CHECK(hipGetLastError());
    }
    // numbering
    uint8_t *flag = nullptr;
    int64_t *rank = nullptr, *tmp = nullptr;
    int rc = dalloc_n(&flag, size_t(N), s);
    if (!rc) rc = dalloc_n(&rank, size_t(N + 1), s);
    if (!rc) rc = dalloc_n(&tmp, scan_tmp_elems(N), s);
    if (rc) {
        dfree(flag, s); dfree(rank, s); dfree(tmp, s);
        return rc;
    }
    k_flag_leaves<<<blocks_for(N), LT, 0, s>>>(g->first_child, N, flag);
    HG_CHECK(hipGetLastError());
    rc = scan_u8_to_i64(flag, rank, N, tmp, s);
    if (rc) return rc;
    int64_t n_leaves = 0;
    HG_CHECK(hipMemcpyAsync(&n_leaves, rank + N, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    HG_CHECK(hipStreamSynchronize(s));
    g->n_leaves = n_leaves;
    g->n_internal = N - n_leaves;
    const char *force = getenv("HGRID_WIDE_REFS");
    g->wide = (n_leaves > MAX_IDS || g->n_internal > MAX_IDS || (force && force[0] == '1')) ? 1 : 0;
    const int64_t L = n_leaves, I = g->n_internal;
    const size_t rsz = g->wide ? 8 : 4;
    int arc = dalloc_n(&g->leaf_of, size_t(N), s);
    if (!arc) arc = dalloc_n(&g->int_of, size_t(N), s);
    if (!arc) arc = dalloc_n(&g->node_of, size_t(L), s);
    if (!arc) arc = dalloc_n(&g->rho, size_t(L), s);
    if (!arc && g->wide) arc = dalloc_n(&g->recw, size_t(L), s);
    if (!arc && !g->wide) arc = dalloc_n(&g->rec32, size_t(L), s);
    if (!arc && !g->wide) arc = dalloc_n(&g->rec64, size_t(L), s);
    if (!arc) arc = dalloc(&g->child, size_t(I > 0 ? I : 1) * nc * rsz, s);
    if (arc) {
        dfree(flag, s); dfree(rank, s); dfree(tmp, s);
        return arc;
    }
    k_number<<<blocks_for(N), LT, 0, s>>>(g->first_child, rank, N, g->leaf_of, g->int_of, g->node_of);
    HG_CHECK(hipGetLastError());
    if (g->wide)
        k_leaf_records_wide<<<blocks_for(L), LT, 0, s>>>(L, g->node_of, g->first_child, g->level,
                                                         g->leaf_of, g->int_of, g->rope, g->S,
                                                         rho_leaf, double(n_samples), g->rho,
                                                         g->recw);
    else
        k_leaf_records<<<blocks_for(L), LT, 0, s>>>(L, g->node_of, g->first_child, g->level,
                                                    g->leaf_of, g->int_of, g->rope, g->S, rho_leaf,
                                                    double(n_samples), g->rho, g->rec32, g->rec64);
    HG_CHECK(hipGetLastError());
    if (I > 0) {
        if (g->wide)
            k_child_refs<uint64_t><<<blocks_for(N * nc), LT, 0, s>>>(
                N, nc, g->first_child, g->level, g->leaf_of, g->int_of, (uint64_t *)g->child);
        else
            k_child_refs<uint32_t><<<blocks_for(N * nc), LT, 0, s>>>(
                N, nc, g->first_child, g->level, g->leaf_of, g->int_of, (uint32_t *)g->child);
        HG_CHECK(hipGetLastError());
    }
    g->root_ref = g->wide ? Ref<uint64_t>::make(I == 0, 0, 0) : Ref<uint32_t>::make(I == 0, 0, 0);
    dfree(flag, s);
    dfree(rank, s);
    dfree(tmp, s);
    HG_CHECK(hipStreamSynchronize(s));
    return HG_OK;
}

}  // namespace hg
