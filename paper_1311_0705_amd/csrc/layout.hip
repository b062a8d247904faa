// Walk layout of a finished tree: face ropes, leaf / internal numbering, the
// 32-byte per-leaf walk records, the encoded child references and, for a k-d
// tree, the three-level jump references.
//
// Ropes stand in for the per-wall neighbor lists of Sect. 2.3: the leaves of
// a rope target's subtree touching the face are exactly that face's neighbor
// list, and the walk reaches the right one by descending from the rope target
// with the exit point.  Ropes are derived level by level from the root.
#include <stdlib.h>

#include "common.h"
#include "rope.h"

namespace hg {

namespace {

constexpr int LT = 256;

// One thread per (node of level l, child slot, face): one rope of the child.
__global__ void __launch_bounds__(LT)
    k_child_ropes(int tree, int64_t begin, int64_t count, int nc, const int32_t *__restrict__ fc,
                  const uint8_t *__restrict__ level, const uint32_t *__restrict__ coord,
                  const uint32_t *__restrict__ geom, int32_t *__restrict__ rope)
{
    const int64_t t = int64_t(blockIdx.x) * LT + threadIdx.x;
    if (t >= count * nc * 6) return;
    const int64_t q = t / 6;   // one thread per (node, child, face)
    child_rope(tree, begin + q / nc, int(q % nc), int(t % 6), fc, level, coord, rope, geom);
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

__global__ void __launch_bounds__(LT)
    k_leaf_records(int64_t n_leaves, int nc, const int32_t *__restrict__ node_of,
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
        const uint32_t e = encode<uint32_t>(rope[6 * int64_t(n) + j], nc, fc, level, leaf_of, int_of);
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
    k_leaf_records_wide(int64_t n_leaves, int nc, const int32_t *__restrict__ node_of,
                        const int32_t *__restrict__ fc, const uint8_t *__restrict__ level,
                        const int32_t *__restrict__ leaf_of, const int32_t *__restrict__ int_of,
                        const int32_t *__restrict__ rope, const double *__restrict__ S,
                        const double *__restrict__ rho_in, double n_samples,
                        double *__restrict__ rho, LeafRecW *__restrict__ recw,
                        const uint32_t *__restrict__ geom)
{
    int64_t l = int64_t(blockIdx.x) * LT + threadIdx.x;
    if (l >= n_leaves) return;
    const int32_t n = node_of[l];
    const double r = leaf_rho(l, n, S, rho_in, n_samples);
    rho[l] = r;
    LeafRecW a;
#pragma unroll
    for (int j = 0; j < 6; j++)
        a.rope[j] = encode<uint64_t>(rope[6 * int64_t(n) + j], nc, fc, level, leaf_of, int_of, geom);
    a.rho64 = r;
    a.rho32 = float(r);
    a.pad = 0;
    recw[l] = a;
}

template <typename R>
__global__ void __launch_bounds__(LT)
    k_child_refs(int64_t n, int nc, const int32_t *__restrict__ fc, const uint8_t *__restrict__ level,
                 const int32_t *__restrict__ leaf_of, const int32_t *__restrict__ int_of,
                 R *__restrict__ child, const uint32_t *__restrict__ geom)
{
    int64_t t = int64_t(blockIdx.x) * LT + threadIdx.x;
    if (t >= n * nc) return;
    int64_t i = t / nc;
    int k = int(t % nc);
    int32_t f = fc[i];
    if (f < 0) return;
    child[int64_t(int_of[i]) * nc + k] = encode<R>(f + k, nc, fc, level, leaf_of, int_of, geom);
}

// k-d jump references: one thread per (node, side triple) (see jump_ref).
template <typename R>
__global__ void __launch_bounds__(LT)
    k_jump_refs(int64_t n, const int32_t *__restrict__ fc, const uint8_t *__restrict__ level,
                const int32_t *__restrict__ leaf_of, const int32_t *__restrict__ int_of, R *__restrict__ jump)
{
    const int64_t t = int64_t(blockIdx.x) * LT + threadIdx.x;
    if (t >= n * 8) return;
    const int64_t i = t >> 3;
    const int c = int(t & 7);
    if (fc[i] < 0) return;
    jump[8 * int64_t(int_of[i]) + c] = jump_ref<R>(int32_t(i), c, fc, level, leaf_of, int_of);
}

template <typename R>
__global__ void __launch_bounds__(LT)
    k_locate_table(int tree, int tdep, int nc, const int32_t *__restrict__ fc, const uint8_t *__restrict__ level,
                   const int32_t *__restrict__ leaf_of, const int32_t *__restrict__ int_of,
                   R *__restrict__ table, const uint32_t *__restrict__ geom)
{
    const int64_t cells = int64_t(1) << (3 * tdep);
    const int64_t t = int64_t(blockIdx.x) * LT + threadIdx.x;
    if (t >= cells) return;
    const uint32_t m = (1u << tdep) - 1u;
    const uint32_t c[3] = {uint32_t(t >> (2 * tdep)) & m, uint32_t(t >> tdep) & m, uint32_t(t) & m};
    table[t] = encode<R>(table_node(tree, tdep, c, fc, level, geom), nc, fc, level, leaf_of, int_of,
                         tree == KDG ? geom : nullptr);
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
        k_child_ropes<<<blocks_for((e - b) * nc * 6), LT, 0, s>>>(g->tree, b, e - b, nc, g->first_child,
                                                              g->level, g->coord, g->geom, g->rope);
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
    // the gradient k-d tree's references carry per-node geometry: wide only
    g->wide = (n_leaves > MAX_IDS || g->n_internal > MAX_IDS || g->tree == KDG || (force && force[0] == '1')) ? 1
                                                                                                              : 0;
    const uint32_t *gk = g->tree == KDG ? g->geom : nullptr;   // geometry carried by references
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
    if (!arc && g->tree == KD && I > 0) arc = dalloc(&g->jump, size_t(I) * 8 * rsz, s);
    if (arc) {
        dfree(flag, s); dfree(rank, s); dfree(tmp, s);
        return arc;
    }
    k_number<<<blocks_for(N), LT, 0, s>>>(g->first_child, rank, N, g->leaf_of, g->int_of, g->node_of);
    HG_CHECK(hipGetLastError());
    if (g->wide)
        k_leaf_records_wide<<<blocks_for(L), LT, 0, s>>>(L, nc, g->node_of, g->first_child, g->level,
                                                         g->leaf_of, g->int_of, g->rope, g->S,
                                                         rho_leaf, double(n_samples), g->rho,
                                                         g->recw, gk);
    else
        k_leaf_records<<<blocks_for(L), LT, 0, s>>>(L, nc, g->node_of, g->first_child, g->level,
                                                    g->leaf_of, g->int_of, g->rope, g->S, rho_leaf,
                                                    double(n_samples), g->rho, g->rec32, g->rec64);
    HG_CHECK(hipGetLastError());
    if (I > 0) {
        if (g->wide)
            k_child_refs<uint64_t><<<blocks_for(N * nc), LT, 0, s>>>(
                N, nc, g->first_child, g->level, g->leaf_of, g->int_of, (uint64_t *)g->child, gk);
        else
            k_child_refs<uint32_t><<<blocks_for(N * nc), LT, 0, s>>>(
                N, nc, g->first_child, g->level, g->leaf_of, g->int_of, (uint32_t *)g->child, nullptr);
        HG_CHECK(hipGetLastError());
        if (g->jump) {
            if (g->wide)
                k_jump_refs<uint64_t><<<blocks_for(N * 8), LT, 0, s>>>(N, g->first_child, g->level, g->leaf_of,
                                                                      g->int_of, (uint64_t *)g->jump);
            else
                k_jump_refs<uint32_t><<<blocks_for(N * 8), LT, 0, s>>>(N, g->first_child, g->level, g->leaf_of,
                                                                      g->int_of, (uint32_t *)g->jump);
            HG_CHECK(hipGetLastError());
        }
    }
    g->root_ref = g->wide ? Ref<uint64_t>::make(I == 0 ? Ref<uint64_t>::LEAF : Ref<uint64_t>::INTERNAL, 0, 0)
                         : Ref<uint32_t>::make(I == 0 ? Ref<uint32_t>::LEAF : Ref<uint32_t>::INTERNAL, 0, 0);
    // locate table
    g->tdep = table_depth(g->tree, L, g->max_level);
    if (g->tdep > 0) {
        const int64_t cells = int64_t(1) << (3 * g->tdep);
        int trc = dalloc(&g->table, size_t(cells) * rsz, s);
        if (trc) {
            dfree(flag, s); dfree(rank, s); dfree(tmp, s);
            return trc;
        }
        if (g->wide)
            k_locate_table<uint64_t><<<blocks_for(cells), LT, 0, s>>>(
                g->tree, g->tdep, nc, g->first_child, g->level, g->leaf_of, g->int_of, (uint64_t *)g->table,
                g->geom);
        else
            k_locate_table<uint32_t><<<blocks_for(cells), LT, 0, s>>>(
                g->tree, g->tdep, nc, g->first_child, g->level, g->leaf_of, g->int_of, (uint32_t *)g->table,
                g->geom);
        HG_CHECK(hipGetLastError());
    }
    dfree(flag, s);
    dfree(rank, s);
    dfree(tmp, s);
    HG_CHECK(hipStreamSynchronize(s));
    return HG_OK;
}

}  // namespace hg
