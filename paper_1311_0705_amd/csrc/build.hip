// Grid construction on the GPU (Sect. 2.2, Eq. 1-3 of Sect. 4).
//
// The construction loop of the paper walks a growing node list once, deciding
// each node and appending the children of split nodes.  Breadth-first order
// makes that list level-synchronous: the nodes of level l are a contiguous
// slice, and an exclusive prefix sum of their split flags gives every child its
// slot in level l+1 in exactly the order the sequential loop would append it.
// Per level:  k_sample_decide (one lane per node, its Monte Carlo samples in
// order; on levels too small to fill the chip, and for densities with many
// clumps, k_sample_decide_group with 2 to 64 lanes per node: node mass
// of Eq. 1, criteria delta, tau of Eq. 2, q of Eq. 3),
// prefix sum of split flags, k_append (children's level and cell coordinates).
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "common.h"
#include "sampling.h"

namespace hg {

namespace {

constexpr int BT = 256;
// ---- clump binning --------------------------------------------------------

__device__ inline bool clump_bin_range(const Dens &D, uint32_t i, int lo[3], int hi[3])
{
    double R = D.trunc * D.cs[i];
    for (int d = 0; d < 3; d++) {
        double c = D.cc[3 * i + d];
        int a = int(floor((c - R - D.lo[d]) * D.bin_scale)) - 1;
        int b = int(floor((c + R - D.lo[d]) * D.bin_scale)) + 1;
        if (b < 0 || a > D.B - 1) return false;
        lo[d] = a < 0 ? 0 : a;
        hi[d] = b > D.B - 1 ? D.B - 1 : b;
    }
    return true;
}

// Binning: one 64-lane block per clump, its lanes over the clump's bins.
constexpr int BIN_T = 64;

__global__ void __launch_bounds__(BIN_T) k_bin_count(Dens D, int32_t *__restrict__ cnt)
{
    const uint32_t i = blockIdx.x;
    int lo[3], hi[3];
    if (!clump_bin_range(D, i, lo, hi)) return;
    const int ny = hi[1] - lo[1] + 1, nz = hi[2] - lo[2] + 1;
    const int total = (hi[0] - lo[0] + 1) * ny * nz;
    for (int t = threadIdx.x; t < total; t += BIN_T) {
        const int x = lo[0] + t / (ny * nz), y = lo[1] + (t / nz) % ny, z = lo[2] + t % nz;
        atomicAdd(&cnt[(x * D.B + y) * D.B + z], 1);
    }
}

// The clump indices into their bins' slices (in any order; k_bin_sort
// restores ascending order).
__global__ void __launch_bounds__(BIN_T) k_bin_fill(Dens D, const int64_t *__restrict__ start,
                                                    int32_t *__restrict__ cursor,
                                                    uint32_t *__restrict__ items)
{
    const uint32_t i = blockIdx.x;
    int lo[3], hi[3];
    if (!clump_bin_range(D, i, lo, hi)) return;
    const int ny = hi[1] - lo[1] + 1, nz = hi[2] - lo[2] + 1;
    const int total = (hi[0] - lo[0] + 1) * ny * nz;
    for (int t = threadIdx.x; t < total; t += BIN_T) {
        const int x = lo[0] + t / (ny * nz), y = lo[1] + (t / nz) % ny, z = lo[2] + t % nz;
        const int b = (x * D.B + y) * D.B + z;
        const int p = atomicAdd(&cursor[b], 1);
        items[start[b] + p] = i;
    }
}

// Sort each bin's clump list ascending (insertion sort; lists are short).
__global__ void __launch_bounds__(BT) k_bin_sort(int n_bins, const int64_t *__restrict__ start,
                                                 uint32_t *__restrict__ items)
{
    int b = blockIdx.x * BT + threadIdx.x;
    if (b >= n_bins) return;
    int64_t s = start[b], e = start[b + 1];
    for (int64_t i = s + 1; i < e; i++) {
        uint32_t v = items[i];
        int64_t j = i - 1;
        while (j >= s && items[j] > v) {
            items[j + 1] = items[j];
            j--;
        }
        items[j + 1] = v;
    }
}

// Bin list entries as records (ClumpRec) of the clumps they name: (trunc
// sigma)^2 as (trunc sigma)(trunc sigma) and 2 sigma^2 as (2 sigma) sigma, the
// products the density sum compares and divides by.
__global__ void __launch_bounds__(BT) k_bin_recs(Dens D, int64_t items, ClumpRec *__restrict__ recs)
{
    const int64_t j = int64_t(blockIdx.x) * BT + threadIdx.x;
    if (j >= items) return;
    const uint32_t i = D.bin_items[j];
    const double s = D.cs[i];
    const double lim = D.trunc * s;
    ClumpRec r;
    r.cx = D.cc[3 * i + 0];
    r.cy = D.cc[3 * i + 1];
    r.cz = D.cc[3 * i + 2];
    r.lim2 = lim * lim;
    r.d2 = 2.0 * s * s;
    r.a = D.ca[i];
    recs[j] = r;
}

// ---- per-level kernels ------------------------------------------------------

// G lanes per node of the level slice [begin, begin+count).
// The split decision of a node completed by its split axis: a gradient k-d
// node that is split takes the axis of gradient_axis (written into its
// geometry) and stays a leaf when no axis is eligible; other trees keep the
// decision as it is.
__device__ inline bool settle_axis(int tree, const Dens &D, int lv, const uint32_t *c, uint32_t *gm, bool split,
                                   const int64_t *__restrict__ bin_start)
{
    if (tree != KDG || !split) return split;
    const uint32_t g = *gm;
    const uint32_t cc[3] = {c[0], c[1], c[2]};
    double w[3], lo[3];
    node_box(tree, D, lv, g, cc, w, lo);
    const int a = gradient_axis(D, lo, w, g, bin_start);
    if (a < 0) return false;
    *gm = (g & 0xFFFFFFu) | (uint32_t(a) << 24);
    return true;
}

template <int G>
__global__ void __launch_bounds__(BT)
    k_sample_decide_group(int tree, Dens D, CritDev C, int64_t begin, int64_t count,
                          const uint8_t *__restrict__ level, const uint32_t *__restrict__ coord,
                          uint32_t *__restrict__ geom, const int64_t *__restrict__ bin_start,
                          double *__restrict__ S_out, double *__restrict__ mn_out, double *__restrict__ mx_out,
                          uint8_t *__restrict__ split)
{
    const int64_t t = (int64_t(blockIdx.x) * BT + threadIdx.x) / G;
    if (t >= count) return;  // the whole group leaves together
    const int64_t i = begin + t;
    const NodeSample r = sample_node_group<G>(tree, D, C, level[i], geom[i], coord[3 * i], coord[3 * i + 1],
                                              coord[3 * i + 2], bin_start);
    if ((threadIdx.x & (G - 1)) != 0) return;
    S_out[i] = r.S;
    mn_out[i] = r.mn;
    mx_out[i] = r.mx;
    split[t] = settle_axis(tree, D, level[i], coord + 3 * i, geom + i, r.split, bin_start) ? 1 : 0;
}

// One lane per node of the level slice [begin, begin+count).
__global__ void __launch_bounds__(BT)
    k_sample_decide(int tree, Dens D, CritDev C, int64_t begin, int64_t count,
                    const uint8_t *__restrict__ level, const uint32_t *__restrict__ coord,
                    uint32_t *__restrict__ geom, const int64_t *__restrict__ bin_start, double *__restrict__ S_out,
                    double *__restrict__ mn_out, double *__restrict__ mx_out,
                    uint8_t *__restrict__ split)
{
    const int64_t t = int64_t(blockIdx.x) * BT + threadIdx.x;
    if (t >= count) return;
    const int64_t i = begin + t;
    const NodeSample r = sample_node_lane(tree, D, C, level[i], geom[i], coord[3 * i], coord[3 * i + 1],
                                          coord[3 * i + 2], bin_start);
    S_out[i] = r.S;
    mn_out[i] = r.mn;
    mx_out[i] = r.mx;
    split[t] = settle_axis(tree, D, level[i], coord + 3 * i, geom + i, r.split, bin_start) ? 1 : 0;
}

// Children of the split nodes of the level slice, in list order.
__global__ void __launch_bounds__(BT)
    k_append(int tree, int64_t begin, int64_t count, int64_t next, const uint8_t *__restrict__ split,
             const int64_t *__restrict__ off, int32_t *__restrict__ fc, uint8_t *__restrict__ level,
             uint32_t *__restrict__ coord, uint32_t *__restrict__ geom)
{
    int64_t t = int64_t(blockIdx.x) * BT + threadIdx.x;
    if (t >= count) return;
    int64_t i = begin + t;
    if (!split[t]) {
        fc[i] = -1;
        return;
    }
    const int nc = tree == OCT ? 8 : 2;
    int64_t f = next + off[t] * nc;
    fc[i] = int32_t(f);
    int lv = level[i];
    uint32_t c[3] = {coord[3 * i], coord[3 * i + 1], coord[3 * i + 2]};
    for (int k = 0; k < nc; k++) {
        uint32_t cc[3], cgm;
        child_coord(tree, geom[i], c, k, cc, &cgm);
        int64_t ch = f + k;
        level[ch] = uint8_t(lv + 1);
        coord[3 * ch] = cc[0];
        coord[3 * ch + 1] = cc[1];
        coord[3 * ch + 2] = cc[2];
        geom[ch] = tree == KDG ? cgm : level_geom(tree, lv + 1);
        fc[ch] = -1;
    }
}

__global__ void k_init_root(int tree, int32_t *fc, uint8_t *level, uint32_t *coord, uint32_t *geom)
{
    fc[0] = -1;
    level[0] = 0;
    coord[0] = coord[1] = coord[2] = 0;
    geom[0] = tree == KDG ? geom_make(0, 0, 0, 3) : level_geom(tree, 0);
}

inline unsigned nblocks(int64_t n, int per) { return unsigned((n + per - 1) / per); }

template <typename T>
int grow_array(T **p, int64_t old_n, int64_t new_cap, size_t per, hipStream_t s)
{
    T *q = nullptr;
    int rc = dalloc_n(&q, size_t(new_cap) * per, s);
    if (rc) return rc;
    if (*p && old_n > 0)
        HG_CHECK(hipMemcpyAsync(q, *p, size_t(old_n) * per * sizeof(T), hipMemcpyDeviceToDevice, s));
    dfree(*p, s);
    *p = q;
    return HG_OK;
}

int grow_nodes(hg_grid *g, int64_t used, int64_t *cap, int64_t need, hipStream_t s)
{
    if (need <= *cap) return HG_OK;
    int64_t c = *cap ? *cap : 4096;
    while (c < need) c *= 2;
    int rc;
    if ((rc = grow_array(&g->first_child, used, c, 1, s))) return rc;
    if ((rc = grow_array(&g->level, used, c, 1, s))) return rc;
    if ((rc = grow_array(&g->coord, used, c, 3, s))) return rc;
    if ((rc = grow_array(&g->geom, used, c, 1, s))) return rc;
    if ((rc = grow_array(&g->S, used, c, 1, s))) return rc;
    if ((rc = grow_array(&g->rmin, used, c, 1, s))) return rc;
    if ((rc = grow_array(&g->rmax, used, c, 1, s))) return rc;
    *cap = c;
    return HG_OK;
}

// Scratch buffer released on the stream when it goes out of scope.
struct DevBuf {
    void *p = nullptr;
    hipStream_t s = nullptr;
    explicit DevBuf(hipStream_t st) : s(st) {}
    int alloc(size_t bytes)
    {
        dfree(p, s);
        p = nullptr;
        return dalloc(&p, bytes, s);
    }
    ~DevBuf() { dfree(p, s); }
};

}  // namespace

int prepare_density(const hg_density *dn, hipStream_t s, DensStore *st, Dens *out)
{
    Dens D;
    memset(&D, 0, sizeof D);
    *st = DensStore{};
    for (int d = 0; d < 3; d++) D.lo[d] = dn->lo[d];
    D.side = dn->side;
    D.has_box = dn->has_box != 0;
    for (int d = 0; d < 3; d++) {
        D.box_lo[d] = dn->box_lo[d];
        D.box_hi[d] = dn->box_hi[d];
    }
    D.box_rho = dn->box_rho;
    D.has_disk = dn->has_disk != 0;
    D.disk_rho0 = dn->disk_rho0;
    D.disk_hR = dn->disk_hR;
    D.disk_hz = dn->disk_hz;
    D.has_torus = dn->has_torus != 0;
    D.torus_R0 = dn->torus_R0;
    D.torus_a = dn->torus_a;
    D.torus_rho = dn->torus_rho;
    D.trunc = dn->clump_trunc;
    D.n_clumps = int(dn->n_clumps);
    D.B = 1;
    D.bin_scale = 1.0 / dn->side;
    *out = D;
    if (D.n_clumps <= 0) return HG_OK;
    const size_t n = size_t(D.n_clumps);
    int rc = dalloc(&st->cc, n * 24, s);
    if (!rc) rc = dalloc(&st->cs, n * 8, s);
    if (!rc) rc = dalloc(&st->ca, n * 8, s);
    if (rc) return rc;
    HG_CHECK(hipMemcpyAsync(st->cc, dn->clump_c, n * 24, hipMemcpyHostToDevice, s));
    HG_CHECK(hipMemcpyAsync(st->cs, dn->clump_sigma, n * 8, hipMemcpyHostToDevice, s));
    HG_CHECK(hipMemcpyAsync(st->ca, dn->clump_amp, n * 8, hipMemcpyHostToDevice, s));
    D.cc = (const double *)st->cc;
    D.cs = (const double *)st->cs;
    D.ca = (const double *)st->ca;
    // bin width about half the mean truncation radius (a sample then tests
    // about N (w + 2r)^3 / side^3 clumps), at most 256 bins per axis; a
    // quarter of it and at most 512 bins per axis for densities with many
    // clumps, whose crowded bins make the clump tests the sampling cost
    const bool many = int64_t(n) >= WAVE_SAMPLING_CLUMPS;
    double rsum = 0.0;
    for (size_t i = 0; i < n; i++) rsum += dn->clump_trunc * fabs(dn->clump_sigma[i]);
    double rmean = rsum / double(n);
    int B = rmean > 0.0 ? int(std::min(1e6, dn->side / ((many ? 0.25 : 0.5) * rmean))) : 1;
    B = std::max(1, std::min(many ? 512 : 256, B));
    D.B = B;
    D.bin_scale = double(B) / dn->side;
    const int64_t nb = int64_t(B) * B * B;
    DevBuf bcnt(s), btmp(s);
    rc = bcnt.alloc(size_t(nb) * 4);
    if (!rc) rc = dalloc(&st->bin_start, size_t(nb + 1) * 8, s);
    if (!rc) rc = btmp.alloc(scan_tmp_elems(nb) * 8);
    if (rc) return rc;
    HG_CHECK(hipMemsetAsync(bcnt.p, 0, size_t(nb) * 4, s));
    k_bin_count<<<unsigned(D.n_clumps), BIN_T, 0, s>>>(D, (int32_t *)bcnt.p);
    HG_CHECK(hipGetLastError());
    rc = scan_i32_to_i64((const int32_t *)bcnt.p, (int64_t *)st->bin_start, nb, (int64_t *)btmp.p, s);
    if (rc) return rc;
    int64_t items = 0;
    HG_CHECK(hipMemcpyAsync(&items, (int64_t *)st->bin_start + nb, 8, hipMemcpyDeviceToHost, s));
    HG_CHECK(hipStreamSynchronize(s));
    if ((rc = dalloc(&st->bin_items, size_t(items > 0 ? items : 1) * 4, s))) return rc;
    HG_CHECK(hipMemsetAsync(bcnt.p, 0, size_t(nb) * 4, s));
    k_bin_fill<<<unsigned(D.n_clumps), BIN_T, 0, s>>>(D, (const int64_t *)st->bin_start,
                                                     (int32_t *)bcnt.p, (uint32_t *)st->bin_items);
    HG_CHECK(hipGetLastError());
    k_bin_sort<<<nblocks(nb, BT), BT, 0, s>>>(int(nb), (const int64_t *)st->bin_start,
                                              (uint32_t *)st->bin_items);
    HG_CHECK(hipGetLastError());
    D.bin_items = (const uint32_t *)st->bin_items;
    st->bin_load = double(items) / double(nb);
    if ((rc = dalloc(&st->bin_recs, size_t(items > 0 ? items : 1) * sizeof(ClumpRec), s))) return rc;
    if (items > 0) {
        k_bin_recs<<<nblocks(items, BT), BT, 0, s>>>(D, items, (ClumpRec *)st->bin_recs);
        HG_CHECK(hipGetLastError());
    }
    D.bin_recs = (const ClumpRec *)st->bin_recs;
    *out = D;
    return HG_OK;
}

void release_density(DensStore *st, hipStream_t s)
{
    dfree(st->cc, s);
    dfree(st->cs, s);
    dfree(st->ca, s);
    dfree(st->bin_start, s);
    dfree(st->bin_items, s);
    dfree(st->bin_recs, s);
    *st = DensStore{};
}

int build_grid(const hg_density *dn, const hg_criteria *cr, int tree, hipStream_t s, hg_grid *g)
{
    const int nc = tree == OCT ? 8 : 2;
    Dens D;
    DensStore store;
    struct Release {
        DensStore *st;
        hipStream_t s;
        ~Release() { release_density(st, s); }
    } release{&store, s};
    int rc = prepare_density(dn, s, &store, &D);
    if (rc) return rc;
    const int64_t *bin_start = (const int64_t *)store.bin_start;

    CritDev C;
    C.total_mass = cr->total_mass;
    C.delta_max = cr->delta_max;
    C.tau_max = cr->tau_max;
    C.q_max = cr->q_max;
    C.kappa = cr->kappa;
    C.min_level = cr->min_level;
    C.max_level = cr->max_level;
    C.n_samples = cr->n_samples;
    C.seed = cr->seed;

    // ---- level loop ----
    int64_t cap = 0;
    rc = grow_nodes(g, 0, &cap, 4096, s);
    if (rc) return rc;
    k_init_root<<<1, 1, 0, s>>>(tree, g->first_child, g->level, g->coord, g->geom);
    HG_CHECK(hipGetLastError());
    DevBuf split(s), off(s), tmp(s);
    int64_t scap = 0;
    int64_t begin = 0, end = 1;
    int lv = 0;
    g->level_begin[0] = 0;
    const int64_t max_nodes = cr->max_nodes > 0 ? cr->max_nodes : (int64_t(1) << 31) - 16;
    for (;;) {
        const int64_t cnt = end - begin;
        if (cnt > scap) {
            int64_t c = std::max<int64_t>(cnt, 4096);
            while (c < 2 * cnt) c *= 2;
            if ((rc = split.alloc(size_t(c)))) return rc;
            if ((rc = off.alloc(size_t(c + 1) * 8))) return rc;
            if ((rc = tmp.alloc(scan_tmp_elems(c) * 8))) return rc;
            scap = c;
        }
        const int gs = sample_group(cnt, density_group_min(D.n_clumps, store.bin_load));
#define HG_SAMPLE_ARGS tree, D, C, begin, cnt, g->level, g->coord, g->geom, bin_start, g->S, g->rmin, g->rmax, \
                       (uint8_t *)split.p
        switch (gs) {
        case 1: k_sample_decide<<<nblocks(cnt, BT), BT, 0, s>>>(HG_SAMPLE_ARGS); break;
        case 2: k_sample_decide_group<2><<<nblocks(cnt * 2, BT), BT, 0, s>>>(HG_SAMPLE_ARGS); break;
        case 4: k_sample_decide_group<4><<<nblocks(cnt * 4, BT), BT, 0, s>>>(HG_SAMPLE_ARGS); break;
        case 8: k_sample_decide_group<8><<<nblocks(cnt * 8, BT), BT, 0, s>>>(HG_SAMPLE_ARGS); break;
        case 16: k_sample_decide_group<16><<<nblocks(cnt * 16, BT), BT, 0, s>>>(HG_SAMPLE_ARGS); break;
        case 32: k_sample_decide_group<32><<<nblocks(cnt * 32, BT), BT, 0, s>>>(HG_SAMPLE_ARGS); break;
        default: k_sample_decide_group<64><<<nblocks(cnt * 64, BT), BT, 0, s>>>(HG_SAMPLE_ARGS); break;
        }
#undef HG_SAMPLE_ARGS
        HG_CHECK(hipGetLastError());
        rc = scan_u8_to_i64((const uint8_t *)split.p, (int64_t *)off.p, cnt, (int64_t *)tmp.p, s);
        if (rc) return rc;
        int64_t n_split = 0;
        HG_CHECK(hipMemcpyAsync(&n_split, (int64_t *)off.p + cnt, 8, hipMemcpyDeviceToHost, s));
        HG_CHECK(hipStreamSynchronize(s));
        const int64_t n_next = n_split * nc;
        if (n_next == 0) break;
        if (end + n_next > max_nodes) return HG_E_LIMIT;
        if ((rc = grow_nodes(g, end, &cap, end + n_next, s))) return rc;
        k_append<<<nblocks(cnt, BT), BT, 0, s>>>(tree, begin, cnt, end, (const uint8_t *)split.p,
                                                 (const int64_t *)off.p, g->first_child, g->level,
                                                 g->coord, g->geom);
        HG_CHECK(hipGetLastError());
        lv++;
        g->level_begin[lv] = end;
        begin = end;
        end += n_next;
        if (lv > 62) return HG_E_LIMIT;
    }
    g->n_nodes = end;
    g->max_level = lv;
    g->level_begin[lv + 1] = end;
    if ((rc = dalloc_n(&g->rope, size_t(end) * 6, s))) return rc;
    return finalize_layout(g, nullptr, cr->n_samples, s);
}

// Levels, cell coordinates and geometry of an imported breadth-first tree,
// on the host, with the structural checks the node list must satisfy.  For
// a gradient k-d tree geom holds the split axes of the internal nodes on
// entry (bits 24-25); every node's geometry is rewritten.
int import_structure(int tree, const std::vector<int32_t> &fc, std::vector<uint8_t> &level,
                     std::vector<uint32_t> &coord, std::vector<uint32_t> &geom, int64_t level_begin[64],
                     int *max_level)
{
    const int64_t n = int64_t(fc.size());
    const int nc = tree == OCT ? 8 : 2;
    const int maxlv = tree == OCT ? 19 : 57;
    level.assign(size_t(n), 0);
    coord.assign(size_t(n) * 3, 0);
    if (tree != KDG) geom.assign(size_t(n), 0u);
    if (geom.size() != size_t(n)) return HG_E_FORMAT;
    geom[0] = tree == KDG ? geom_make(0, 0, 0, geom_axis(geom[0])) : level_geom(tree, 0);
    int64_t expect = 1;
    for (int64_t i = 0; i < n; i++) {
        int32_t f = fc[size_t(i)];
        const uint32_t gm = geom[size_t(i)];
        if (f < 0) {
            geom[size_t(i)] = (gm & 0xFFFFFFu) | (3u << 24);
            continue;
        }
        if (f != expect || int64_t(f) + nc > n || level[size_t(i)] >= maxlv) return HG_E_FORMAT;
        if (tree == KDG && (geom_axis(gm) > 2 || geom_depth(gm, geom_axis(gm)) >= KDG_MAX_DEPTH))
            return HG_E_FORMAT;
        expect += nc;
        int lv = level[size_t(i)];
        for (int k = 0; k < nc; k++) {
            uint32_t c[3] = {coord[3 * size_t(i)], coord[3 * size_t(i) + 1], coord[3 * size_t(i) + 2]};
            uint32_t cc[3], cgm;
            child_coord(tree, gm, c, k, cc, &cgm);
            size_t ch = size_t(f) + size_t(k);
            level[ch] = uint8_t(lv + 1);
            for (int d = 0; d < 3; d++) coord[3 * ch + d] = cc[d];
            // a gradient node's entry keeps the child's own split axis
            geom[ch] = tree == KDG ? (cgm & 0xFFFFFFu) | (geom[ch] & (3u << 24)) : level_geom(tree, lv + 1);
        }
    }
    if (expect != n) return HG_E_FORMAT;
    int ml = 0;
    for (int64_t i = 0; i < n; i++) {
        int l = level[size_t(i)];
        if (i > 0 && l < level[size_t(i - 1)]) return HG_E_FORMAT;
        if (l > ml) {
            for (int k = ml + 1; k <= l; k++) level_begin[k] = i;
            ml = l;
        }
    }
    level_begin[0] = 0;
    level_begin[ml + 1] = n;
    *max_level = ml;
    return HG_OK;
}

}  // namespace hg
