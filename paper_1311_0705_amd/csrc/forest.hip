// Batched construction and tracing of many grids ("a forest") with every
// launch sized on the host in advance and every count kept on the device, so
// a whole build-then-trace pass has no host synchronisation and can be
// captured in a HIP graph and replayed.
//
// The construction is the same level-synchronous form of the node-list loop
// of Sect. 2.2 as the single-grid builder, run for all grids of the batch at
// once: per level one launch samples every node of that level of every grid
// (Eq. 1-3), one prefix sum over the concatenated split flags gives every
// child its slot in its own grid, one launch appends the children.  Grids are
// told apart by a per-level prefix of their node counts (a binary search per
// work item).  Node arrays are reserved up front from each grid's node
// capacity (criteria.max_nodes); a grid that would exceed it stops growing and
// is reported.  Results are identical to grid_build's, node for node.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "common.h"
#include "rope.h"
#include "sampling.h"

namespace hg {

namespace {

constexpr int FT = 256;
constexpr int LB_N = 66;         // level-begin slots per grid
constexpr int META = LB_N + 4;   // + n_nodes, n_leaves, depth, error
constexpr int M_NODES = LB_N, M_LEAVES = LB_N + 1, M_DEPTH = LB_N + 2, M_ERR = LB_N + 3;
constexpr unsigned FLAT_BLOCKS = 4096;    // grid-stride launches over device-sized ranges
constexpr unsigned SAMPLE_BLOCKS = 2048;  // node sampling: 4 wavefronts of 64 nodes per block
// launch shapes the batch tuner tries
const int BLOCKS[] = {128, 256, 512};
const int BATCH_CHUNKS[] = {128, 256, 512, 1024, 2048, 4096};
const int REFILLS[] = {1, 2, 4, 8, 16};

struct ForestGrid {
    int tree, nc, lg, pad;
    Dens D;
    CritDev C;
    const int64_t *bin_start;
    int64_t cap;
    int32_t *fc;
    uint8_t *level;
    uint32_t *coord;
    double *S, *rmin, *rmax;
    int32_t *rope, *leaf_of, *int_of, *node_of;
    double *rho;
    LeafRec32 *rec32;
    LeafRec64 *rec64;
    uint32_t *child;
    uint32_t *jump;   // k-d jump references (8 per internal node), else NULL
    uint32_t *table;  // locate table, room for 2^(3 tmax) cells
    int tmax, pad2;
    int64_t *meta;  // [META]: level begins, then n_nodes, n_leaves, depth, error
};

// Grid owning flat item t, given the prefix P[0..ng] of per-grid counts.
__device__ inline int owner(const int64_t *__restrict__ P, int ng, int64_t t)
{
    int lo = 0, hi = ng;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (P[mid] <= t) lo = mid;
        else hi = mid;
    }
    return lo;
}

// Exclusive prefix of per-grid values v(i) into P[0..ng] by one block;
// returns the total to every thread.
template <typename F>
__device__ inline int64_t block_prefix(int ng, int64_t *P, F v)
{
    __shared__ int64_t part[FT + 1];
    const int per = (ng + FT - 1) / FT;
    const int a = int(threadIdx.x) * per, b = min(ng, a + per);
    int64_t s = 0;
    for (int i = a; i < b; i++) s += v(i);
    part[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t run = 0;
        for (int j = 0; j < FT; j++) {
            const int64_t x = part[j];
            part[j] = run;
            run += x;
        }
        part[FT] = run;
    }
    __syncthreads();
    int64_t run = part[threadIdx.x];
    for (int i = a; i < b; i++) {
        P[i] = run;
        run += v(i);
    }
    if (threadIdx.x == 0) P[ng] = part[FT];
    return part[FT];
}

__global__ void __launch_bounds__(FT) k_f_init(const ForestGrid *__restrict__ F, int ng)
{
    const int i = int(blockIdx.x) * FT + threadIdx.x;
    if (i >= ng) return;
    const ForestGrid &G = F[i];
    G.fc[0] = -1;
    G.level[0] = 0;
    G.coord[0] = G.coord[1] = G.coord[2] = 0;
    for (int j = 0; j < 6; j++) G.rope[j] = -1;
    G.meta[0] = 0;
    for (int l = 1; l < LB_N; l++) G.meta[l] = 1;
    G.meta[M_NODES] = 0;
    G.meta[M_LEAVES] = 0;
    G.meta[M_DEPTH] = 0;
    G.meta[M_ERR] = 0;
}

// Wavefronts of the sampling of a level with per-grid node counts n(i):
// the lanes per node g for the level's total (sample_group, at least gmin)
// goes to PW[ng+1], and PW[0..ng] is the prefix of the per-grid wavefront
// counts (64/g nodes to a wavefront; a wavefront never spans two grids).
template <typename N>
__device__ inline void sample_waves(int ng, int64_t total, int gmin, int64_t *PW, N n)
{
    const int g = sample_group(total, gmin);
    block_prefix(ng, PW, [&](int i) { return (n(i) * g + 63) / 64; });
    if (threadIdx.x == 0) PW[ng + 1] = g;
}

// P: prefix of the per-grid node counts of level lv; PW: its sampling
// wavefronts (sample_waves).
__global__ void __launch_bounds__(FT) k_f_level_prefix(const ForestGrid *__restrict__ F, int ng, int lv,
                                                       int64_t *P, int64_t *PW, int gmin)
{
    auto count = [&](int i) { return F[i].meta[lv + 1] - F[i].meta[lv]; };
    const int64_t total = block_prefix(ng, P, count);
    __syncthreads();
    sample_waves(ng, total, gmin, PW, count);
}

// G lanes per node of level lv (2 <= G <= 64), over all grids: a wavefront
// takes 64/G consecutive nodes of one grid.
template <int G>
__device__ __forceinline__ void sample_level_group(const ForestGrid *__restrict__ F, int ng, int lv,
                                                   const int64_t *__restrict__ P,
                                                   const int64_t *__restrict__ PW, uint8_t *__restrict__ flag)
{
    const int lane = threadIdx.x & 63;
    const int64_t TW = PW[ng];
    const int64_t nw = int64_t(gridDim.x) * (FT / 64);
    for (int64_t w = (int64_t(blockIdx.x) * FT + threadIdx.x) >> 6; w < TW; w += nw) {
        // the grid is the same for the whole wavefront
        const int i = __builtin_amdgcn_readfirstlane(owner(PW, ng, w));
        const ForestGrid &Gr = F[i];
        const Dens D = Gr.D;
        const CritDev C = Gr.C;
        const int64_t k = (w - PW[i]) * (64 / G) + lane / G;   // rank of the group's node in the level
        if (k < P[i + 1] - P[i]) {
            const int64_t n = Gr.meta[lv] + k;
            const NodeSample r = sample_node_group<G>(Gr.tree, D, C, lv, 0u, Gr.coord[3 * n],
                                                      Gr.coord[3 * n + 1], Gr.coord[3 * n + 2], Gr.bin_start);
            if ((lane & (G - 1)) == 0) {
                Gr.S[n] = r.S;
                Gr.rmin[n] = r.mn;
                Gr.rmax[n] = r.mx;
                flag[P[i] + k] = r.split ? 1 : 0;
            }
        }
    }
}

// One lane per node of level lv: a wavefront takes up to 64 consecutive nodes
// of one grid, whose density and criteria then sit in scalar registers.
__device__ __forceinline__ void sample_level_lane(const ForestGrid *__restrict__ F, int ng, int lv,
                                                  const int64_t *__restrict__ P,
                                                  const int64_t *__restrict__ PW, uint8_t *__restrict__ flag)
{
    const int lane = threadIdx.x & 63;
    const int64_t TW = PW[ng];
    const int64_t nw = int64_t(gridDim.x) * (FT / 64);
    for (int64_t w = (int64_t(blockIdx.x) * FT + threadIdx.x) >> 6; w < TW; w += nw) {
        const int i = __builtin_amdgcn_readfirstlane(owner(PW, ng, w));
        const ForestGrid &G = F[i];
        const Dens D = G.D;
        const CritDev C = G.C;
        const int64_t k = (w - PW[i]) * 64 + lane;   // rank of the lane's node in the level
        if (k < P[i + 1] - P[i]) {
            const int64_t n = G.meta[lv] + k;
            const NodeSample r = sample_node_lane(G.tree, D, C, lv, 0u, G.coord[3 * n], G.coord[3 * n + 1],
                                                  G.coord[3 * n + 2], G.bin_start);
            G.S[n] = r.S;
            G.rmin[n] = r.mn;
            G.rmax[n] = r.mx;
            flag[P[i] + k] = r.split ? 1 : 0;
        }
    }
}

// Node sampling of level lv over all grids, with the lanes per node that the
// level's wavefront prefix was made for (PW[ng+1]; the same for the whole
// launch).
__global__ void __launch_bounds__(FT) k_f_sample(const ForestGrid *__restrict__ F, int ng, int lv,
                                                 const int64_t *__restrict__ P,
                                                 const int64_t *__restrict__ PW, uint8_t *__restrict__ flag)
{
    switch (int(PW[ng + 1])) {
    case 1: sample_level_lane(F, ng, lv, P, PW, flag); break;
    case 2: sample_level_group<2>(F, ng, lv, P, PW, flag); break;
    case 4: sample_level_group<4>(F, ng, lv, P, PW, flag); break;
    case 8: sample_level_group<8>(F, ng, lv, P, PW, flag); break;
    case 16: sample_level_group<16>(F, ng, lv, P, PW, flag); break;
    case 32: sample_level_group<32>(F, ng, lv, P, PW, flag); break;
    default: sample_level_group<64>(F, ng, lv, P, PW, flag); break;
    }
}

// Per grid: the next level's extent, or an error if it would not fit.
// Children of the split nodes of level lv, over all grids.  Each thread
// derives its grid's next-level size from the split-flag prefix (so no
// separate pass has to publish it first); the thread of a grid's first node
// records that size in meta (or the capacity error), and block 0 computes
// the per-grid prefix of the next level's node counts (P_next) and its
// sampling wavefronts (PW; nothing when P_next is null).
__global__ void __launch_bounds__(FT) k_f_append(const ForestGrid *__restrict__ F, int ng, int lv,
                                                 const int64_t *__restrict__ P,
                                                 const uint8_t *__restrict__ flag,
                                                 const int64_t *__restrict__ off, int64_t *P_next,
                                                 int64_t *PW, int gmin)
{
    // the next level's node count of grid i (0 if it would not fit)
    auto next_count = [&](int i) {
        const ForestGrid &G = F[i];
        const int64_t nn = (off[P[i + 1]] - off[P[i]]) * G.nc;
        return G.meta[lv + 1] + nn > G.cap ? int64_t(0) : nn;
    };
    if (P_next && blockIdx.x == 0) {
        const int64_t total = block_prefix(ng, P_next, next_count);
        __syncthreads();
        sample_waves(ng, total, gmin, PW, next_count);
    }
    const int64_t T = P[ng];
    for (int64_t t = int64_t(blockIdx.x) * FT + threadIdx.x; t < T; t += int64_t(gridDim.x) * FT) {
        const int i = owner(P, ng, t);
        const ForestGrid &G = F[i];
        const int64_t nn = (off[P[i + 1]] - off[P[i]]) * G.nc;
        const bool over = G.meta[lv + 1] + nn > G.cap;
        if (t == P[i]) {
            if (over) G.meta[M_ERR] = 1;
            for (int l = lv + 2; l < LB_N; l++) G.meta[l] = G.meta[lv + 1] + (over ? 0 : nn);
        }
        const int64_t n = G.meta[lv] + (t - P[i]);
        if (!flag[t] || over) {
            G.fc[n] = -1;
            continue;
        }
        const int64_t f = G.meta[lv + 1] + (off[t] - off[P[i]]) * G.nc;
        G.fc[n] = int32_t(f);
        const uint32_t c[3] = {G.coord[3 * n], G.coord[3 * n + 1], G.coord[3 * n + 2]};
        for (int k = 0; k < G.nc; k++) {
            uint32_t cc[3];
            uint32_t cgm;
            child_coord(G.tree, level_geom(G.tree, lv), c, k, cc, &cgm);
            const int64_t ch = f + k;
            G.level[ch] = uint8_t(lv + 1);
            G.coord[3 * ch] = cc[0];
            G.coord[3 * ch + 1] = cc[1];
            G.coord[3 * ch + 2] = cc[2];
            G.fc[ch] = -1;
        }
    }
}

// Ropes of the children of level lv's nodes.  A single grid: one thread per
// (node, child, face), so the push-downs of a node's children overlap.  Many
// grids: one thread per node (its children's faces in turn), which keeps the
// search for each item's grid to one per node.
__global__ void __launch_bounds__(FT) k_f_ropes(const ForestGrid *__restrict__ F, int ng, int lv,
                                                const int64_t *__restrict__ P)
{
    if (ng == 1) {
        const ForestGrid &G = F[0];
        const int64_t per = int64_t(G.nc) * 6;
        const int64_t T = P[1] * per;
        for (int64_t t = int64_t(blockIdx.x) * FT + threadIdx.x; t < T; t += int64_t(gridDim.x) * FT) {
            const int64_t tp = t / per;
            const int rem = int(t - tp * per);
            child_rope(G.tree, G.meta[lv] + tp, rem / 6, rem % 6, G.fc, G.level, G.coord, G.rope);
        }
        return;
    }
    const int64_t T = P[ng];
    for (int64_t t = int64_t(blockIdx.x) * FT + threadIdx.x; t < T; t += int64_t(gridDim.x) * FT) {
        const int i = owner(P, ng, t);
        const ForestGrid &G = F[i];
        const int64_t p = G.meta[lv] + (t - P[i]);
        for (int k = 0; k < G.nc; k++) child_ropes(G.tree, p, k, G.fc, G.level, G.coord, G.rope);
    }
}

__global__ void __launch_bounds__(FT) k_f_node_prefix(const ForestGrid *__restrict__ F, int ng,
                                                      int lmax, int64_t *PN)
{
    block_prefix(ng, PN, [&](int i) { return F[i].meta[lmax + 1]; });
    for (int i = threadIdx.x; i < ng; i += FT) {
        const ForestGrid &G = F[i];
        G.meta[M_NODES] = G.meta[lmax + 1];
        int d = 0;
        for (int l = 1; l <= lmax; l++)
            if (G.meta[l + 1] > G.meta[l]) d = l;
        G.meta[M_DEPTH] = d;
    }
}

__global__ void __launch_bounds__(FT) k_f_flag(const ForestGrid *__restrict__ F, int ng,
                                               const int64_t *__restrict__ PN, uint8_t *__restrict__ flag)
{
    const int64_t T = PN[ng];
    for (int64_t t = int64_t(blockIdx.x) * FT + threadIdx.x; t < T; t += int64_t(gridDim.x) * FT) {
        const int i = owner(PN, ng, t);
        flag[t] = F[i].fc[t - PN[i]] < 0 ? 1 : 0;
    }
}

// Leaf rank = leaves before the node in list order; internal rank = the rest.
__global__ void __launch_bounds__(FT) k_f_number(const ForestGrid *__restrict__ F, int ng,
                                                 const int64_t *__restrict__ PN,
                                                 const int64_t *__restrict__ rank)
{
    const int64_t T = PN[ng];
    for (int64_t t = int64_t(blockIdx.x) * FT + threadIdx.x; t < T; t += int64_t(gridDim.x) * FT) {
        const int i = owner(PN, ng, t);
        const ForestGrid &G = F[i];
        const int64_t n = t - PN[i];
        const int64_t lr = rank[t] - rank[PN[i]];
        if (G.fc[n] < 0) {
            G.leaf_of[n] = int32_t(lr);
            G.int_of[n] = -1;
            G.node_of[lr] = int32_t(n);
        } else {
            G.leaf_of[n] = -1;
            G.int_of[n] = int32_t(n - lr);
        }
    }
}

__device__ inline int grid_tdep(const ForestGrid &G, int64_t L)
{
    const int t = table_depth(G.tree, L, int(G.meta[M_DEPTH]));
    return t < G.tmax ? t : G.tmax;
}

// Leaf counts, the leaf and table-cell prefixes and each grid's walk parameters.
__global__ void __launch_bounds__(FT) k_f_leaf_prefix(const ForestGrid *__restrict__ F, int ng,
                                                      const int64_t *__restrict__ PN,
                                                      const int64_t *__restrict__ rank, int64_t *PL,
                                                      int64_t *PT, WalkGrid *__restrict__ w32,
                                                      WalkGrid *__restrict__ w64)
{
    block_prefix(ng, PL, [&](int i) { return rank[PN[i + 1]] - rank[PN[i]]; });
    __syncthreads();
    block_prefix(ng, PT, [&](int i) {
        const int t = grid_tdep(F[i], rank[PN[i + 1]] - rank[PN[i]]);
        return t > 0 ? int64_t(1) << (3 * t) : int64_t(0);
    });
    for (int i = threadIdx.x; i < ng; i += FT) {
        const ForestGrid &G = F[i];
        const int64_t L = rank[PN[i + 1]] - rank[PN[i]];
        const int64_t I = G.meta[M_NODES] - L;
        G.meta[M_LEAVES] = L;
        WalkGrid W;
        W.tree = G.tree;
        W.lg = G.lg;
        for (int d = 0; d < 3; d++) W.lo[d] = G.D.lo[d];
        W.side = G.D.side;
        for (int d = 0; d < 3; d++) W.hi[d] = G.D.lo[d] + G.D.side;
        W.root = Ref<uint32_t>::make(I == 0 ? Ref<uint32_t>::LEAF : Ref<uint32_t>::INTERNAL, 0, 0);
        W.n_leaves = uint64_t(L);
        W.n_internal = uint64_t(I);
        W.child = G.child;
        W.jump = G.jump;
        W.tdep = grid_tdep(G, L);
        W.tw = ldexp(G.D.side, -W.tdep);
        W.tscale = ldexp(1.0, W.tdep) / G.D.side;
        W.table = W.tdep > 0 ? G.table : nullptr;
        W.dm = finest_depth(G.tree, G.C.max_level);
        W.unit = ldexp(G.D.side, -W.dm);
        W.rec = G.rec32;
        w32[i] = W;
        W.rec = G.rec64;
        w64[i] = W;
    }
}

__global__ void __launch_bounds__(FT) k_f_records(const ForestGrid *__restrict__ F, int ng,
                                                  const int64_t *__restrict__ PL)
{
    const int64_t T = PL[ng];
    for (int64_t t = int64_t(blockIdx.x) * FT + threadIdx.x; t < T; t += int64_t(gridDim.x) * FT) {
        const int i = owner(PL, ng, t);
        const ForestGrid &G = F[i];
        const int64_t l = t - PL[i];
        const int32_t n = G.node_of[l];
        const double r = leaf_rho(l, n, G.S, nullptr, double(G.C.n_samples));
        G.rho[l] = r;
        LeafRec32 a;
        LeafRec64 b;
#pragma unroll
        for (int j = 0; j < 6; j++) {
            const uint32_t e = encode<uint32_t>(G.rope[6 * int64_t(n) + j], G.nc, G.fc, G.level, G.leaf_of, G.int_of);
            a.rope[j] = e;
            b.rope[j] = e;
        }
        a.rho = float(r);
        a.pad = 0;
        b.rho = r;
        G.rec32[l] = a;
        G.rec64[l] = b;
    }
}

__global__ void __launch_bounds__(FT) k_f_table(const ForestGrid *__restrict__ F, int ng,
                                                const int64_t *__restrict__ PT,
                                                const WalkGrid *__restrict__ W)
{
    const int64_t T = PT[ng];
    for (int64_t t = int64_t(blockIdx.x) * FT + threadIdx.x; t < T; t += int64_t(gridDim.x) * FT) {
        const int i = owner(PT, ng, t);
        const ForestGrid &G = F[i];
        const int td = W[i].tdep;
        const int64_t cell = t - PT[i];
        const uint32_t m = (1u << td) - 1u;
        const uint32_t c[3] = {uint32_t(cell >> (2 * td)) & m, uint32_t(cell >> td) & m, uint32_t(cell) & m};
        G.table[cell] = encode<uint32_t>(table_node(G.tree, td, c, G.fc, G.level), G.nc, G.fc, G.level,
                                         G.leaf_of, G.int_of);
    }
}

__global__ void __launch_bounds__(FT) k_f_child_refs(const ForestGrid *__restrict__ F, int ng,
                                                     const int64_t *__restrict__ PN)
{
    const int64_t T = PN[ng];
    for (int64_t t = int64_t(blockIdx.x) * FT + threadIdx.x; t < T; t += int64_t(gridDim.x) * FT) {
        const int i = owner(PN, ng, t);
        const ForestGrid &G = F[i];
        const int64_t n = t - PN[i];
        const int32_t f = G.fc[n];
        if (f < 0) continue;
        const int64_t base = int64_t(G.int_of[n]) * G.nc;
        for (int k = 0; k < G.nc; k++)
            G.child[base + k] = encode<uint32_t>(f + k, G.nc, G.fc, G.level, G.leaf_of, G.int_of);
        if (G.jump)
            for (int c = 0; c < 8; c++)
                G.jump[8 * int64_t(G.int_of[n]) + c] =
                    jump_ref<uint32_t>(int32_t(n), c, G.fc, G.level, G.leaf_of, G.int_of);
    }
}

__global__ void k_f_reset_status(TraceStatus *st)
{
    st->rechecks = 0;
    st->descents = 0;
    st->bad_dir = 0;
    st->step_guard = 0;
    st->bad_ref = 0;
    st->cap_overflow = 0;
    st->resumed = 0;
    st->next_ray = 0;
    st->done_waves = 0;
}

__global__ void __launch_bounds__(FT) k_f_totals(const WalkArgs *__restrict__ A, int ng, int64_t *out)
{
    const int i = int(blockIdx.x) * FT + threadIdx.x;
    if (i < ng) out[i] = A[i].offsets[A[i].n];
}

}  // namespace
}  // namespace hg

using namespace hg;

// The library's batch object.
struct hg_batch {
    int ng = 0;
    int lmax = 0;
    std::vector<DensStore> dens;
    std::vector<ForestGrid> hF;
    ForestGrid *dF = nullptr;
    int64_t *meta = nullptr;        // [ng][META]
    int64_t *P = nullptr;           // [(lmax+1)][ng+1]
    int64_t *PN = nullptr, *PL = nullptr, *PT = nullptr;
    int64_t *PW = nullptr;          // [ng+2] sampling wavefronts per grid and lanes per node, current level
    int sample_gmin = 1;            // least lanes per node in sampling (density_group_min over the grids)
    uint8_t *flag = nullptr;        // [sum of capacities]
    int64_t *off = nullptr;         // [sum of capacities + 1]
    int64_t *stmp = nullptr;
    WalkGrid *w32 = nullptr, *w64 = nullptr;
    int32_t *cgrid = nullptr, *cpre = nullptr;   // the grids by level-table class (grid_classes)
    int ncls = 0;
    TraceStatus *status = nullptr;
    void *tmp_block = nullptr;      // the batch-wide arrays above, carved from one block
    size_t tmp_bytes = 0;
    std::vector<void *> arrays;     // one block per grid holding its arrays
    std::vector<size_t> array_bytes;
    int dev = 0;                    // device of the blocks
    // bound trace
    std::vector<WalkArgs> hA;
    bool bound = false;
    hg_trace_opts opts{};
    std::vector<int64_t> n;
    std::vector<hg_trace_out> outs;
    WalkArgs *dA = nullptr;
    BatchChunk *dC = nullptr;
    int64_t *gpre = nullptr;               // [ng + 1] chunks per grid, prefix
    unsigned long long *gctr = nullptr;    // [ng] chunks taken per grid (walk queue counters)
    int n_chunks = 0;
    int64_t *ctmp = nullptr;
    int64_t *totals = nullptr;
    // one-pass records (unless two walks are asked for): the slab walk writes
    // each path's first `slab` records into a row and saves the state of a
    // path past its row; the rows are copied into the CSR slices and the
    // saved paths resume in a filling walk over a device-built chunk table
    bool one_pass = false;
    int64_t slab = 0;
    int pairs = 0;
    WalkArgs *dAs = nullptr;               // slab-walk arguments (rows, resume arrays)
    WalkArgs *dAf = nullptr;               // resume-walk arguments (CSR slices, resume arrays)
    void *op_block = nullptr;              // rows, resume entries, counters, resume chunk table
    // captured graph
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int graph_stages = 0;
    int last_stages = 0;   // stages of the last run or replay (what batch_result reads)
};

namespace {

void free_bound(hg_batch *b)
{
    dfree(b->dA, nullptr);
    dfree(b->dC, nullptr);
    dfree(b->gpre, nullptr);
    dfree(b->gctr, nullptr);
    b->gpre = nullptr;
    b->gctr = nullptr;
    dfree(b->ctmp, nullptr);
    dfree(b->totals, nullptr);
    dfree(b->dAs, nullptr);
    dfree(b->dAf, nullptr);
    dfree(b->op_block, nullptr);
    b->dA = nullptr;
    b->dC = nullptr;
    b->ctmp = nullptr;
    b->totals = nullptr;
    b->dAs = nullptr;
    b->dAf = nullptr;
    b->op_block = nullptr;
    b->one_pass = false;
    b->bound = false;
}

void free_batch(hg_batch *b)
{
    if (!b) return;
    (void)hipDeviceSynchronize();
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    free_bound(b);
    for (auto &d : b->dens) release_density(&d, nullptr);
    for (size_t i = 0; i < b->arrays.size(); i++) block_free(b->arrays[i], b->array_bytes[i], b->dev);
    block_free(b->tmp_block, b->tmp_bytes, b->dev);
    (void)hipDeviceSynchronize();
    delete b;
}

constexpr int64_t BATCH_SLAB_MIN = 16;

// Bytes the rows of a batch may take: the single-grid budget, at most half of
// the device memory free at binding (the rows stay reserved while bound).
double batch_slab_budget()
{
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) return 0.0;
    return std::min(SLAB_BUDGET, 0.5 * double(free_b));
}

// Rows per path of the one-pass batched records mode for n paths in all: the
// caller's slab rounded up to a multiple of 4, else the most that fit the
// budget (at most SLAB_MAX); 0 (two walks) when fewer than BATCH_SLAB_MIN fit.
int64_t batch_slab_rows(const hg_trace_opts *opts, int64_t n, double budget)
{
    const double per = double(4 + (opts->precision == HG_FP64 ? 8 : 4));
    if (n <= 0) return 0;
    if (opts->slab > 0) {
        const int64_t k = (int64_t(opts->slab) + 3) / 4 * 4;
        return double(n) * (double(k) * per + double(sizeof(Resume))) <= budget ? k : 0;
    }
    const double fit = (budget / double(n) - double(sizeof(Resume))) / per;
    if (fit < double(BATCH_SLAB_MIN)) return 0;
    return std::min<int64_t>(SLAB_MAX, int64_t(fit) / 4 * 4);
}

std::vector<BatchChunk> chunk_table(const std::vector<int64_t> &n, int64_t chunk)
{
    std::vector<BatchChunk> hC;
    for (size_t i = 0; i < n.size(); i++) {
        const int32_t head = int32_t(hC.size());
        for (int64_t a = 0; a < n[i]; a += chunk)
            hC.push_back(BatchChunk{int32_t(i), head, a, std::min(n[i], a + chunk)});
    }
    return hC;
}

int enqueue_build(hg_batch *b, hipStream_t s)
{
    const int ng = b->ng;
    const unsigned gb = unsigned((ng + FT - 1) / FT);
    k_f_init<<<gb, FT, 0, s>>>(b->dF, ng);
    HG_CHECK(hipGetLastError());
    const int gmin = b->sample_gmin;
    k_f_level_prefix<<<1, FT, 0, s>>>(b->dF, ng, 0, b->P, b->PW, gmin);
    HG_CHECK(hipGetLastError());
    for (int lv = 0; lv <= b->lmax; lv++) {
        int64_t *P = b->P + size_t(lv) * size_t(ng + 1);
        int64_t *P_next = lv < b->lmax ? P + (ng + 1) : nullptr;
        k_f_sample<<<SAMPLE_BLOCKS, FT, 0, s>>>(b->dF, ng, lv, P, b->PW, b->flag);
        HG_CHECK(hipGetLastError());
        int rc = scan_u8_to_i64_dev(b->flag, b->off, P + ng, b->stmp, s);
        if (rc) return rc;
        k_f_append<<<FLAT_BLOCKS, FT, 0, s>>>(b->dF, ng, lv, P, b->flag, b->off, P_next, b->PW, gmin);
        HG_CHECK(hipGetLastError());
    }
    for (int lv = 0; lv < b->lmax; lv++) {
        k_f_ropes<<<FLAT_BLOCKS, FT, 0, s>>>(b->dF, ng, lv, b->P + size_t(lv) * size_t(ng + 1));
        HG_CHECK(hipGetLastError());
    }
    k_f_node_prefix<<<1, FT, 0, s>>>(b->dF, ng, b->lmax, b->PN);
    HG_CHECK(hipGetLastError());
    k_f_flag<<<FLAT_BLOCKS, FT, 0, s>>>(b->dF, ng, b->PN, b->flag);
    HG_CHECK(hipGetLastError());
    int rc = scan_u8_to_i64_dev(b->flag, b->off, b->PN + ng, b->stmp, s);
    if (rc) return rc;
    k_f_number<<<FLAT_BLOCKS, FT, 0, s>>>(b->dF, ng, b->PN, b->off);
    HG_CHECK(hipGetLastError());
    k_f_leaf_prefix<<<1, FT, 0, s>>>(b->dF, ng, b->PN, b->off, b->PL, b->PT, b->w32, b->w64);
    HG_CHECK(hipGetLastError());
    k_f_table<<<FLAT_BLOCKS, FT, 0, s>>>(b->dF, ng, b->PT, b->w32);
    HG_CHECK(hipGetLastError());
    k_f_records<<<FLAT_BLOCKS, FT, 0, s>>>(b->dF, ng, b->PL);
    HG_CHECK(hipGetLastError());
    k_f_child_refs<<<FLAT_BLOCKS, FT, 0, s>>>(b->dF, ng, b->PN);
    HG_CHECK(hipGetLastError());
    return HG_OK;
}

// The bound trace over chunk table C (nc entries; ctmp: its scan work
// space) with launch options o: one-pass records (slab walk, offsets, row
// copy, resume walk), or the counting walk and, for records, the filling walk.
int trace_pipeline(hg_batch *b, const BatchChunk *C, const int64_t *gpre, int nc, int64_t *ctmp,
                   const hg_trace_opts *o, hipStream_t s)
{
    const WalkGrid *G = b->opts.precision == HG_FP64 ? b->w64 : b->w32;
    const int ng = b->ng;
    const BatchQueue Q{C, gpre, b->gctr, ng, b->cgrid, b->cpre, b->ncls};
    k_f_reset_status<<<1, 1, 0, s>>>(b->status);
    HG_CHECK(hipGetLastError());
    int rc = HG_OK;
    if (b->one_pass) {
        if (nc > 0) rc = launch_batched(G, b->dAs, Q, o, WM_SLAB, b->status, s);
        if (!rc) rc = scan_chunks(C, nc, b->dAf, ng, ctmp, s);
        if (!rc) rc = launch_slab_compact_batch(b->dAs, b->dAf, Q, nc, b->opts.precision, b->pairs, b->status, s);
        if (rc) return rc;
        // the paths past their row (count > slab) resume from their entries
        return nc > 0 ? launch_batched(G, b->dAf, Q, o, WM_FILL, b->status, s) : HG_OK;
    }
    if (nc > 0) rc = launch_batched(G, b->dA, Q, o, WM_COUNT, b->status, s);
    if (rc || b->opts.mode != HG_RECORDS) return rc;
    rc = scan_chunks(C, nc, b->dA, ng, ctmp, s);
    if (rc || nc == 0) return rc;
    return launch_batched(G, b->dA, Q, o, WM_FILL, b->status, s);
}

int enqueue_trace(hg_batch *b, hipStream_t s)
{
    if (!b->bound) return HG_E_INVAL;
    return trace_pipeline(b, b->dC, b->gpre, b->n_chunks, b->ctmp, &b->opts, s);
}

}  // namespace

extern "C" {

int batch_create(int n_grids, const hg_density *dens, const hg_criteria *crit, const int *tree_types,
                 hg_batch_t *out)
{
    if (!out) return HG_E_INVAL;
    *out = nullptr;
    if (n_grids < 1 || n_grids > HG_MAX_BATCH || !dens || !crit || !tree_types) return HG_E_INVAL;
    int lmax = 0;
    int64_t total_cap = 0;
    for (int i = 0; i < n_grids; i++) {
        if (tree_types[i] == HG_KDGRAD) return HG_E_INVAL;   // built by grid_build only
        int rc = check_build_args(&dens[i], &crit[i], tree_types[i]);
        if (rc) return rc;
        if (crit[i].max_nodes < 1) return HG_E_INVAL;
        if (crit[i].max_nodes > MAX_IDS) return HG_E_LIMIT;
        lmax = std::max(lmax, int(crit[i].max_level));
        total_cap += crit[i].max_nodes;
    }
    hg_batch *b = new hg_batch;
    b->ng = n_grids;
    b->lmax = lmax;
    b->dens.resize(size_t(n_grids));
    b->hF.resize(size_t(n_grids));
    int rc = HG_OK;
    for (int i = 0; i < n_grids && !rc; i++) {
        ForestGrid &G = b->hF[size_t(i)];
        memset(&G, 0, sizeof G);
        const hg_criteria &c = crit[i];
        G.tree = tree_types[i];
        G.nc = G.tree == HG_OCTREE ? 8 : 2;
        int e = 0;
        frexp(dens[i].side, &e);
        G.lg = e - 1;
        rc = prepare_density(&dens[i], nullptr, &b->dens[size_t(i)], &G.D);
        if (rc) break;
        b->sample_gmin = std::max(b->sample_gmin,
                                  density_group_min(dens[i].n_clumps, b->dens[size_t(i)].bin_load));
        G.bin_start = (const int64_t *)b->dens[size_t(i)].bin_start;
        G.C = CritDev{c.total_mass, c.delta_max, c.tau_max, c.q_max, c.kappa,
                      c.min_level, c.max_level, c.n_samples, c.seed};
        const size_t cap = size_t(c.max_nodes);
        G.cap = int64_t(cap);
        G.tmax = table_depth(G.tree, int64_t(cap), c.max_level);
        Carve cv;
        cv.add(&G.fc, cap);
        cv.add(&G.level, cap);
        cv.add(&G.coord, 3 * cap);
        cv.add(&G.S, cap);
        cv.add(&G.rmin, cap);
        cv.add(&G.rmax, cap);
        cv.add(&G.rope, 6 * cap);
        cv.add(&G.leaf_of, cap);
        cv.add(&G.int_of, cap);
        cv.add(&G.node_of, cap);
        cv.add(&G.rho, cap);
        cv.add(&G.rec32, cap);
        cv.add(&G.rec64, cap);
        cv.add(&G.child, cap);
        // k-d: eight jump references per internal node (at most cap / 2 of them)
        if (G.tree == HG_KDTREE) cv.add(&G.jump, 4 * cap);
        cv.add(&G.table, size_t(1) << (3 * G.tmax));
        void *blk = nullptr;
        rc = cv.alloc(&blk, &b->dev);
        if (!rc) {
            b->arrays.push_back(blk);
            b->array_bytes.push_back(cv.bytes());
        }
    }
    const size_t ng1 = size_t(n_grids) + 1;
    Carve ct;
    ct.add(&b->meta, size_t(n_grids) * META);
    ct.add(&b->dF, size_t(n_grids));
    ct.add(&b->P, size_t(lmax + 1) * ng1);
    ct.add(&b->PN, ng1);
    ct.add(&b->PL, ng1);
    ct.add(&b->PT, ng1);
    ct.add(&b->PW, ng1 + 1);
    ct.add(&b->flag, size_t(total_cap));
    ct.add(&b->off, size_t(total_cap) + 1);
    ct.add(&b->stmp, scan_dev_tmp_elems());
    ct.add(&b->w32, size_t(n_grids));
    ct.add(&b->w64, size_t(n_grids));
    ct.add(&b->status, 1);
    std::vector<int32_t> hcg, hcp;
    {
        std::vector<int> tr((size_t)n_grids), dm((size_t)n_grids);
        std::vector<double> sd((size_t)n_grids);
        for (int i = 0; i < n_grids; i++) {
            tr[size_t(i)] = tree_types[i];
            dm[size_t(i)] = finest_depth(tree_types[i], crit[i].max_level);
            sd[size_t(i)] = dens[i].side;
        }
        grid_classes(tr, dm, sd, hcg, hcp);
    }
    ct.add(&b->cgrid, hcg.size());
    ct.add(&b->cpre, hcp.size());
    b->ncls = int(hcp.size()) - 1;
    if (!rc) rc = ct.alloc(&b->tmp_block, &b->dev);
    if (!rc) b->tmp_bytes = ct.bytes();
    for (int i = 0; i < n_grids && !rc; i++) b->hF[size_t(i)].meta = b->meta + size_t(i) * META;
    if (!rc) {
        hipError_t e = hipMemcpy(b->dF, b->hF.data(), sizeof(ForestGrid) * size_t(n_grids),
                                 hipMemcpyHostToDevice);
        if (!e) e = hipMemcpy(b->cgrid, hcg.data(), sizeof(int32_t) * hcg.size(), hipMemcpyHostToDevice);
        if (!e) e = hipMemcpy(b->cpre, hcp.data(), sizeof(int32_t) * hcp.size(), hipMemcpyHostToDevice);
        if (!e) e = hipDeviceSynchronize();
        if (e) rc = set_hip_error(e);
    }
    if (rc) {
        free_batch(b);
        return rc;
    }
    *out = b;
    return HG_OK;
}

}  // extern "C"

namespace hg {
namespace {

// One-pass records of a bound batch: rows, resume entries and the argument
// arrays of the slab and resume walks.  Leaves the batch in two-walk mode
// (HG_OK) when the rows would not fit the budget or cannot be allocated.
int bind_one_pass(hg_batch *b, const std::vector<WalkArgs> &hA, const hg_trace_opts *opts)
{
    const int ng = b->ng;
    int64_t total = 0;
    std::vector<int64_t> pre(size_t(ng) + 1, 0);
    for (int g = 0; g < ng; g++) pre[size_t(g) + 1] = pre[size_t(g)] + hA[size_t(g)].n;
    total = pre[size_t(ng)];
    const int64_t slab = batch_slab_rows(opts, total, batch_slab_budget());
    if (slab == 0) return HG_OK;
    const int pairs = opts->precision != HG_FP64 ? 1 : 0;   // FP32 rows of (leaf, ds32) pairs
    const size_t dsz = opts->precision == HG_FP64 ? 8 : 4;
    const size_t rl = size_t(slab) * (pairs ? 8 : 4), rd = pairs ? 0 : size_t(slab) * dsz;
    Carve cv;
    char *rows_l = nullptr, *rows_d = nullptr;
    Resume *res = nullptr;
    cv.add(&rows_l, size_t(total) * rl);
    if (!pairs) cv.add(&rows_d, size_t(total) * rd);
    cv.add(&res, size_t(std::max<int64_t>(total, 1)));
    if (dalloc(&b->op_block, cv.bytes(), nullptr)) return HG_OK;   // two walks instead
    cv.assign(b->op_block);
    std::vector<WalkArgs> hs(hA), hf(hA);
    for (int g = 0; g < ng; g++) {
        WalkArgs &S = hs[size_t(g)], &F = hf[size_t(g)];
        const int64_t p0 = pre[size_t(g)];
        S.leaf = reinterpret_cast<int32_t *>(rows_l + size_t(p0) * rl);
        S.ds = pairs ? nullptr : static_cast<void *>(rows_d + size_t(p0) * rd);
        S.offsets = nullptr;
        S.capacity = S.n * slab;
        S.slab = slab;
        S.resume = res + p0;
        S.n_resume = nullptr;
        S.resume_by_path = 1;
        S.pairs = pairs;
        F.slab = slab;
        F.resume = res + p0;
        F.n_resume = nullptr;
        F.resume_by_path = 1;
        F.pairs = 0;
    }
    int rc = dalloc_n(&b->dAs, size_t(ng), nullptr);
    if (!rc) rc = dalloc_n(&b->dAf, size_t(ng), nullptr);
    if (!rc) {
        hipError_t e = hipMemcpy(b->dAs, hs.data(), sizeof(WalkArgs) * hs.size(), hipMemcpyHostToDevice);
        if (!e) e = hipMemcpy(b->dAf, hf.data(), sizeof(WalkArgs) * hf.size(), hipMemcpyHostToDevice);
        if (!e) e = hipDeviceSynchronize();
        if (e) rc = set_hip_error(e);
    }
    if (rc) return rc;
    b->slab = slab;
    b->pairs = pairs;
    b->one_pass = true;
    return HG_OK;
}

}  // namespace
}  // namespace hg

extern "C" {

int batch_bind(hg_batch_t b, const double *const *origins, const double *const *dirs, const int64_t *n,
               const hg_trace_opts *opts, hg_trace_out *outs)
{
    if (!b || !origins || !dirs || !n || !opts || !outs) return HG_E_INVAL;
    if (opts->precision != HG_FP64 && opts->precision != HG_FP32_RECHECK) return HG_E_INVAL;
    if (opts->mode != HG_TAU_ONLY && opts->mode != HG_RECORDS) return HG_E_INVAL;
    if (!isfinite(opts->kappa)) return HG_E_INVAL;
    if (opts->block != 0 && opts->block != 128 && opts->block != 256 && opts->block != 512)
        return HG_E_INVAL;
    if (opts->chunk < 0 || opts->refill_min < 0) return HG_E_INVAL;
    const bool records = opts->mode == HG_RECORDS;
    for (int i = 0; i < b->ng; i++) {
        const hg_trace_out &o = outs[i];
        if (n[i] < 0) return HG_E_INVAL;
        if (n[i] > 0 && (!origins[i] || !dirs[i] || !o.tau || !o.count)) return HG_E_INVAL;
        if (records && (!o.offsets || o.capacity < 0)) return HG_E_INVAL;
        if (records && o.capacity > 0 && (!o.leaf || !o.ds)) return HG_E_INVAL;
        if (records && ((uintptr_t(o.leaf) | uintptr_t(o.ds)) & 15u)) return HG_E_INVAL;
    }
    if (b->exec) {
        (void)hipGraphExecDestroy(b->exec);
        b->exec = nullptr;
    }
    if (b->graph) {
        (void)hipGraphDestroy(b->graph);
        b->graph = nullptr;
    }
    free_bound(b);
    const int64_t chunk = opts->chunk > 0 ? opts->chunk : 1024;
    std::vector<WalkArgs> hA(size_t(b->ng));
    const std::vector<BatchChunk> hC = chunk_table(std::vector<int64_t>(n, n + b->ng), chunk);
    for (int i = 0; i < b->ng; i++) {
        WalkArgs &A = hA[size_t(i)];
        A.O = origins[i];
        A.K = dirs[i];
        A.n = n[i];
        A.kappa = opts->kappa;
        A.tau = outs[i].tau;
        A.count = outs[i].count;
        A.offsets = records ? outs[i].offsets : nullptr;
        A.leaf = records ? outs[i].leaf : nullptr;
        A.ds = records ? outs[i].ds : nullptr;
        A.capacity = records ? outs[i].capacity : 0;
        A.st = b->status;
        A.count_rechecks = (opts->flags & HG_FLAG_RECHECKS) ? 1 : 0;
        A.slab = 0;
        A.resume = nullptr;
        A.n_resume = nullptr;
        A.pairs = 0;
    }
    if (hC.size() > size_t(0x7fffffff)) return HG_E_LIMIT;
    const std::vector<int64_t> hP = chunk_prefix(hC, b->ng);
    int rc = dalloc_n(&b->dA, size_t(b->ng), nullptr);
    if (!rc) rc = dalloc_n(&b->dC, std::max<size_t>(hC.size(), 1), nullptr);
    if (!rc) rc = dalloc_n(&b->gpre, hP.size(), nullptr);
    if (!rc) rc = dalloc_n(&b->gctr, size_t(b->ng), nullptr);
    if (!rc) rc = dalloc_n(&b->ctmp, scan_chunks_tmp_elems(int(hC.size())), nullptr);
    if (!rc) rc = dalloc_n(&b->totals, size_t(b->ng), nullptr);
    if (!rc) {
        hipError_t e = hipMemcpy(b->dA, hA.data(), sizeof(WalkArgs) * hA.size(), hipMemcpyHostToDevice);
        if (!e && !hC.empty())
            e = hipMemcpy(b->dC, hC.data(), sizeof(BatchChunk) * hC.size(), hipMemcpyHostToDevice);
        if (!e) e = hipMemcpy(b->gpre, hP.data(), sizeof(int64_t) * hP.size(), hipMemcpyHostToDevice);
        if (!e) e = hipDeviceSynchronize();
        if (e) rc = set_hip_error(e);
    }
    if (!rc && records && opts->passes != 2) rc = bind_one_pass(b, hA, opts);
    if (rc) {
        free_bound(b);
        return rc;
    }
    b->opts = *opts;
    b->hA = hA;
    b->n.assign(n, n + b->ng);
    b->outs.assign(outs, outs + b->ng);
    b->n_chunks = int(hC.size());
    b->bound = true;
    b->last_stages &= ~HG_STAGE_TRACE;
    return HG_OK;
}

int batch_run(hg_batch_t b, int stages, void *stream)
{
    if (!b || (stages & ~HG_STAGE_ALL) || !stages) return HG_E_INVAL;
    if ((stages & HG_STAGE_TRACE) && !b->bound) return HG_E_INVAL;
    hipStream_t s = (hipStream_t)stream;
    int rc = HG_OK;
    if (stages & HG_STAGE_BUILD) rc = enqueue_build(b, s);
    if (!rc && (stages & HG_STAGE_TRACE)) rc = enqueue_trace(b, s);
    b->last_stages = rc ? 0 : stages;
    return rc;
}

int batch_capture(hg_batch_t b, int stages, void *stream)
{
    if (!b || (stages & ~HG_STAGE_ALL) || !stages) return HG_E_INVAL;
    if ((stages & HG_STAGE_TRACE) && !b->bound) return HG_E_INVAL;
    hipStream_t s = (hipStream_t)stream;
    if (!s) return HG_E_INVAL;  // the legacy default stream cannot be captured
    if (b->exec) {
        (void)hipGraphExecDestroy(b->exec);
        b->exec = nullptr;
    }
    if (b->graph) {
        (void)hipGraphDestroy(b->graph);
        b->graph = nullptr;
    }
    HG_CHECK(hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed));
    const int before = b->last_stages;
    int rc = batch_run(b, stages, stream);
    b->last_stages = before;   // nothing has run yet
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(s, &g);
    if (rc) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e) return set_hip_error(e);
    e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
    if (e) {
        (void)hipGraphDestroy(g);
        return set_hip_error(e);
    }
    b->graph = g;
    b->graph_stages = stages;
    return HG_OK;
}

int batch_replay(hg_batch_t b, void *stream)
{
    if (!b || !b->exec) return HG_E_INVAL;
    HG_CHECK(hipGraphLaunch(b->exec, (hipStream_t)stream));
    b->last_stages = b->graph_stages;
    return HG_OK;
}

int batch_result(hg_batch_t b, void *stream, int64_t *n_nodes, int64_t *n_leaves, hg_trace_out *outs)
{
    if (!b) return HG_E_INVAL;
    hipStream_t s = (hipStream_t)stream;
    std::vector<int64_t> meta(size_t(b->ng) * META);
    TraceStatus st;
    memset(&st, 0, sizeof st);
    std::vector<int64_t> tot(size_t(b->ng), 0);
    const bool traced = b->bound && (b->last_stages & HG_STAGE_TRACE);
    const bool records = traced && b->opts.mode == HG_RECORDS;
    if (records) {
        k_f_totals<<<unsigned((b->ng + FT - 1) / FT), FT, 0, s>>>(b->dA, b->ng, b->totals);
        HG_CHECK(hipGetLastError());
    }
    HG_CHECK(hipMemcpyAsync(meta.data(), b->meta, sizeof(int64_t) * meta.size(), hipMemcpyDeviceToHost, s));
    HG_CHECK(hipMemcpyAsync(&st, b->status, sizeof st, hipMemcpyDeviceToHost, s));
    if (records)
        HG_CHECK(hipMemcpyAsync(tot.data(), b->totals, sizeof(int64_t) * tot.size(), hipMemcpyDeviceToHost, s));
    HG_CHECK(hipStreamSynchronize(s));
    int rc = HG_OK;
    for (int i = 0; i < b->ng; i++) {
        const int64_t *m = meta.data() + size_t(i) * META;
        if (n_nodes) n_nodes[i] = m[M_NODES];
        if (n_leaves) n_leaves[i] = m[M_LEAVES];
        if (m[M_ERR]) rc = HG_E_LIMIT;
        if (outs && traced) {
            outs[i].needed = records ? tot[size_t(i)] : 0;
            outs[i].rechecks = i == 0 ? int64_t(st.rechecks) : 0;
            outs[i].descents = i == 0 ? int64_t(st.descents) : 0;
            if (records && tot[size_t(i)] > b->outs[size_t(i)].capacity && !rc) rc = HG_E_CAPACITY;
        }
    }
    if (!rc && traced) {
        if (st.bad_ref) rc = HG_E_FORMAT;
        else if (st.bad_dir) rc = HG_E_DIR;
        else if (st.step_guard) rc = HG_E_STEP;
        else if (st.cap_overflow) rc = HG_E_CAPACITY;
    }
    return rc;
}

int batch_grid(hg_batch_t b, int i, hg_grid_t *out)
{
    if (!out) return HG_E_INVAL;
    *out = nullptr;
    if (!b || i < 0 || i >= b->ng) return HG_E_INVAL;
    const ForestGrid &F = b->hF[size_t(i)];
    int64_t m[META];
    HG_CHECK(hipDeviceSynchronize());
    HG_CHECK(hipMemcpy(m, F.meta, sizeof m, hipMemcpyDeviceToHost));
    if (m[M_ERR]) return HG_E_LIMIT;
    WalkGrid W;
    HG_CHECK(hipMemcpy(&W, b->w32 + i, sizeof W, hipMemcpyDeviceToHost));
    hg_grid *g = new_grid(F.tree, F.D.lo, F.D.side);
    if (!g) return HG_E_OOM;
    g->borrowed = 1;
    g->n_nodes = m[M_NODES];
    g->n_leaves = m[M_LEAVES];
    g->n_internal = g->n_nodes - g->n_leaves;
    g->max_level = int(m[M_DEPTH]);
    for (int l = 0; l < 64; l++) g->level_begin[l] = l <= g->max_level + 1 ? m[l] : g->n_nodes;
    g->first_child = F.fc;
    g->level = F.level;
    g->coord = F.coord;
    g->S = F.S;
    g->rmin = F.rmin;
    g->rmax = F.rmax;
    g->rope = F.rope;
    g->leaf_of = F.leaf_of;
    g->int_of = F.int_of;
    g->node_of = F.node_of;
    g->rho = F.rho;
    g->wide = 0;
    g->rec32 = F.rec32;
    g->rec64 = F.rec64;
    g->child = F.child;
    g->jump = F.jump;
    g->root_ref = Ref<uint32_t>::make(g->n_internal == 0 ? Ref<uint32_t>::LEAF : Ref<uint32_t>::INTERNAL, 0, 0);
    g->table = const_cast<void *>(W.table);
    g->tdep = W.tdep;
    *out = g;
    return HG_OK;
}

int batch_tune(hg_batch_t b, hg_trace_opts *chosen, float *best_ms, void *stream)
{
    if (!b || !b->bound) return HG_E_INVAL;
    hipStream_t s = (hipStream_t)stream;
    const int nchunk = int(sizeof BATCH_CHUNKS / sizeof *BATCH_CHUNKS);
    std::vector<std::vector<BatchChunk>> tables;
    size_t most = 1;
    for (int c = 0; c < nchunk; c++) {
        tables.push_back(chunk_table(b->n, BATCH_CHUNKS[c]));
        most = std::max(most, tables.back().size());
    }
    if (most > size_t(0x7fffffff)) return HG_E_LIMIT;
    BatchChunk *dC = nullptr;
    int64_t *ctmp = nullptr, *dP = nullptr;
    const size_t ng1 = size_t(b->ng) + 1;
    std::vector<std::vector<int64_t>> prefixes;
    for (int c = 0; c < nchunk; c++) prefixes.push_back(chunk_prefix(tables[size_t(c)], b->ng));
    int rc = dalloc_n(&dC, most * size_t(nchunk), s);
    if (!rc) rc = dalloc_n(&ctmp, scan_chunks_tmp_elems(int(most)), s);
    if (!rc) rc = dalloc_n(&dP, ng1 * size_t(nchunk), s);
    for (int c = 0; c < nchunk && !rc; c++) {
        hipError_t e = hipMemcpyAsync(dP + size_t(c) * ng1, prefixes[size_t(c)].data(), sizeof(int64_t) * ng1,
                                      hipMemcpyHostToDevice, s);
        if (!e && !tables[size_t(c)].empty())
            e = hipMemcpyAsync(dC + size_t(c) * most, tables[size_t(c)].data(),
                               sizeof(BatchChunk) * tables[size_t(c)].size(), hipMemcpyHostToDevice, s);
        if (e) rc = set_hip_error(e);
    }
    hipEvent_t ev[4] = {};
    for (int i = 0; i < 4 && !rc; i++)
        if (hipEventCreate(&ev[i]) != hipSuccess) rc = HG_E_HIP;
    hg_trace_opts best = b->opts;
    best.block = best.block ? best.block : 256;
    best.refill_min = best.refill_min ? best.refill_min : 4;
    best.chunk = best.chunk ? best.chunk : 1024;
    float best_t = INFINITY;
    auto eval = [&](const hg_trace_opts &c, float *ms) -> int {
        int ci = 0;
        while (ci < nchunk - 1 && BATCH_CHUNKS[ci] != c.chunk) ci++;
        const BatchChunk *C = dC + size_t(ci) * most;
        const int64_t *P = dP + size_t(ci) * ng1;
        const int nc = int(tables[size_t(ci)].size());
        *ms = INFINITY;
        for (int r = 0; r <= 3; r++) {
            HG_CHECK(hipEventRecord(ev[0], s));
            const int rc2 = trace_pipeline(b, C, P, nc, ctmp, &c, s);
            if (rc2) return rc2;
            HG_CHECK(hipEventRecord(ev[1], s));
            HG_CHECK(hipEventSynchronize(ev[1]));
            float t = 0.f;
            HG_CHECK(hipEventElapsedTime(&t, ev[0], ev[1]));
            if (r > 0) *ms = std::min(*ms, t);
        }
        return HG_OK;
    };
    if (!rc) rc = eval(best, &best_t);
    for (int round = 0; round < 2 && !rc; round++) {
        bool moved = false;
        for (int p = 0; p < 3 && !rc; p++) {
            const int *vals = p == 0 ? BLOCKS : (p == 1 ? BATCH_CHUNKS : REFILLS);
            const int nv = p == 0 ? 3 : (p == 1 ? nchunk : 4);
            for (int v = 0; v < nv && !rc; v++) {
                hg_trace_opts c = best;
                int32_t &fld = p == 0 ? c.block : (p == 1 ? c.chunk : c.refill_min);
                if (fld == vals[v]) continue;
                fld = vals[v];
                float ms = 0.f;
                rc = eval(c, &ms);
                if (!rc && ms < 0.99f * best_t) {
                    best = c;
                    best_t = ms;
                    moved = true;
                }
            }
        }
        if (!moved) break;
    }
    for (auto &e : ev)
        if (e) (void)hipEventDestroy(e);
    (void)hipStreamSynchronize(s);
    dfree(dC, s);
    dfree(ctmp, s);
    dfree(dP, s);
    if (rc) return rc;
    // rebind the queue with the winner (a captured graph is dropped)
    std::vector<const double *> o(size_t(b->ng)), k(size_t(b->ng));
    for (int i = 0; i < b->ng; i++) {
        o[size_t(i)] = b->hA[size_t(i)].O;
        k[size_t(i)] = b->hA[size_t(i)].K;
    }
    std::vector<int64_t> n = b->n;
    std::vector<hg_trace_out> outs = b->outs;
    rc = batch_bind(b, o.data(), k.data(), n.data(), &best, outs.data());
    if (!rc && best_ms) *best_ms = best_t;
    if (!rc && chosen) *chosen = best;
    return rc;
}

void batch_free(hg_batch_t b) { free_batch(b); }

}  // extern "C"

namespace hg {

// One grid built by the batch construction (every level count on the device,
// no synchronisation per level) with node capacity cr->max_nodes; the grid
// takes over the batch's arrays.
int build_single_batched(const hg_density *dn, const hg_criteria *cr, int tree, hipStream_t s,
                         hg_grid **out)
{
    *out = nullptr;
    hg_batch_t b = nullptr;
    int rc = batch_create(1, dn, cr, &tree, &b);
    if (rc) return rc;
    rc = batch_run(b, HG_STAGE_BUILD, s);
    if (!rc) rc = batch_result(b, s, nullptr, nullptr, nullptr);
    hg_grid_t g = nullptr;
    if (!rc) rc = batch_grid(b, 0, &g);
    if (!rc) {
        // the grid takes over the block holding its arrays
        g->block = b->arrays[0];
        g->block_bytes = b->array_bytes[0];
        g->block_dev = b->dev;
        b->arrays.clear();
        b->array_bytes.clear();
        g->borrowed = 0;
        *out = g;
    }
    batch_free(b);
    return rc;
}

}  // namespace hg
