// Device side of the per-node Monte Carlo sampling (Sect. 2.2 and 4): the
// counter-based sample positions, the density models and the criteria of
// Eq. 1-3, shared by the single-grid and the batched builders.
#pragma once

#include "common.h"

namespace hg {

constexpr uint64_t SPLITMIX_GAMMA = 0x9E3779B97F4A7C15ull;

// Criteria as the kernels read them.
struct CritDev {
    double total_mass, delta_max, tau_max, q_max, kappa;
    int min_level, max_level, n_samples;
    uint64_t seed;
};

// SplitMix64 output for state x (Steele, Lea & Flood 2014): advance by the
// golden gamma, then the published mixing function.
__device__ inline uint64_t splitmix64(uint64_t x)
{
    uint64_t z = x + SPLITMIX_GAMMA;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Node code: level in bits 57.., cell coordinates in 19-bit fields; a
// gradient k-d node's halvings per axis are mixed in (nodes of one level may
// share coordinates at different halvings).
__device__ inline uint64_t node_key(uint64_t seed, int tree, int level, uint32_t gm, uint32_t c0, uint32_t c1,
                                    uint32_t c2)
{
    uint64_t code = (uint64_t(level) << 57) | (uint64_t(c0) << 38) | (uint64_t(c1) << 19) | uint64_t(c2);
    if (tree == KDG) code ^= splitmix64(uint64_t(gm & 0xFFFFFFu));
    return splitmix64(seed ^ splitmix64(code));
}

// Uniform double in [0,1) for sample j, axis d: the draw of counter
// m = 3j + d + 1, given as cg = m gamma (mod 2^64).  The sampling loops carry
// cg and step it by additions of gamma multiples, since a 64-bit product
// costs three quarter-rate 32-bit multiplies per draw.
__device__ inline double sample_unit(uint64_t key, uint64_t cg)
{
    uint64_t r = splitmix64(key ^ cg);
    return double(r >> 11) * 0x1.0p-53;
}

__device__ inline int bin_of(const Dens &D, double x, int d)
{
    int b = int(floor((x - D.lo[d]) * D.bin_scale));
    return b < 0 ? 0 : (b >= D.B ? D.B - 1 : b);
}

// rho_t(x): box, disk, clumps in ascending index, torus -- added in that order.
__device__ inline double density_at(const Dens &D, double x0, double x1, double x2,
                                    const int64_t *__restrict__ bin_start)
{
    double rho = 0.0;
    if (D.has_box) {
        if (x0 >= D.box_lo[0] && x0 <= D.box_hi[0] && x1 >= D.box_lo[1] && x1 <= D.box_hi[1] &&
            x2 >= D.box_lo[2] && x2 <= D.box_hi[2])
            rho = rho + D.box_rho;
    }
    if (D.has_disk) {
        double R = sqrt(x0 * x0 + x1 * x1);
        double arg = -(R / D.disk_hR) - fabs(x2) / D.disk_hz;
        rho = rho + D.disk_rho0 * exp(arg);
    }
    if (D.n_clumps > 0) {
        int b = (bin_of(D, x0, 0) * D.B + bin_of(D, x1, 1)) * D.B + bin_of(D, x2, 2);
        int64_t e = bin_start[b + 1];
        // the bin's clumps in ascending index, each a record read in one go
        // (no dependent load through the clump index)
        for (int64_t j = bin_start[b]; j < e; j++) {
            const ClumpRec c = D.bin_recs[j];
            double dx = x0 - c.cx;
            double dy = x1 - c.cy;
            double dz = x2 - c.cz;
            double r2 = dx * dx + dy * dy + dz * dz;
            if (r2 <= c.lim2) {
                double ee = r2 / c.d2;
                rho = rho + c.a * exp(-ee);
            }
        }
    }
    if (D.has_torus) {
        double R = sqrt(x0 * x0 + x1 * x1);
        double dR = R - D.torus_R0;
        if (dR * dR + x2 * x2 <= D.torus_a * D.torus_a) rho = rho + D.torus_rho;
    }
    return rho;
}

// Optical depth of a node of sides w[3] with sampled sum S over n samples,
// Eq. (2) with the node mass of Eq. (1): kappa M sqrt(a^2+b^2+c^2)/(abc),
// M = S (V/N).
__host__ __device__ inline double node_tau(double kappa, double S, const double w[3], int n_samples)
{
    const double V = w[0] * w[1] * w[2];
    const double M = S * (V / double(n_samples));
    const double diag = sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
    return kappa * M * diag / (w[0] * w[1] * w[2]);
}

struct NodeSample {
    double S, mn, mx;
    bool split;
};

// The criteria of Sect. 2.2 / 4 for a node of sides w with sampled sum S,
// minimum mn and maximum mx: Eq. (1) M = V/N sum rho, delta = M/M_tot;
// Eq. (2) tau = kappa M sqrt(a^2+b^2+c^2)/(abc); Eq. (3) q = (max-min)/max.
__device__ inline NodeSample decide_node(const CritDev &C, int lv, const double w[3], double S, double mn,
                                         double mx)
{
    const double V = w[0] * w[1] * w[2];
    const double M = S * (V / double(C.n_samples));
    const double delta = M / C.total_mass;
    const double tau = node_tau(C.kappa, S, w, C.n_samples);
    const double q = mx > 0.0 ? (mx - mn) / mx : 0.0;
    bool sp;
    if (lv < C.min_level) sp = true;
    else if (lv >= C.max_level) sp = false;
    else sp = delta > C.delta_max || tau > C.tau_max || q > C.q_max;
    return NodeSample{S, mn, mx, sp};
}

__device__ inline void node_box(int tree, const Dens &D, int lv, uint32_t gm, const uint32_t c[3], double w[3],
                                double lo[3])
{
#pragma unroll
    for (int d = 0; d < 3; d++) {
        w[d] = ldexp(D.side, -(tree == KDG ? geom_depth(gm, d) : axis_depth(tree, lv, d)));
        lo[d] = D.lo[d] + double(c[d]) * w[d];
    }
}

// Split axis of a gradient k-d node with box lo + [0, w] and halvings dep[]
// (the orientation option of Sect. 2.2): the axis of the largest central
// difference |rho(x_c + w_d/4 e_d) - rho(x_c - w_d/4 e_d)| / (w_d/2) between
// the centres of the node's halves; ties go to the axis halved least often,
// then the lowest; axes halved KDG_MAX_DEPTH times are not eligible.  -1 if
// none is.
__device__ inline int gradient_axis(const Dens &D, const double lo[3], const double w[3], uint32_t gm,
                                    const int64_t *__restrict__ bin_start)
{
    double xc[3];
#pragma unroll
    for (int d = 0; d < 3; d++) xc[d] = lo[d] + 0.5 * w[d];
    int best = -1, dbest = 0;
    double gbest = 0.0;
    for (int d = 0; d < 3; d++) {
        const int dd = geom_depth(gm, d);
        if (dd >= KDG_MAX_DEPTH) continue;
        double xp[3] = {xc[0], xc[1], xc[2]}, xm[3] = {xc[0], xc[1], xc[2]};
        xp[d] = xc[d] + 0.25 * w[d];
        xm[d] = xc[d] - 0.25 * w[d];
        const double rp = density_at(D, xp[0], xp[1], xp[2], bin_start);
        const double rm = density_at(D, xm[0], xm[1], xm[2], bin_start);
        const double gd = fabs(rp - rm) / (0.5 * w[d]);
        if (best < 0 || gd > gbest || (gd == gbest && dd < dbest)) {
            best = d;
            gbest = gd;
            dbest = dd;
        }
    }
    return best;
}

// One node per lane: samples j = 0 .. N-1 are drawn and summed in order, so
// S is the sequential sum of Eq. (1) with no cross-lane reduction (the lanes
// of a wavefront take different nodes).
__device__ inline NodeSample sample_node_lane(int tree, const Dens &D, const CritDev &C, int lv, uint32_t gm,
                                              uint32_t c0, uint32_t c1, uint32_t c2,
                                              const int64_t *__restrict__ bin_start)
{
    const uint32_t c[3] = {c0, c1, c2};
    double w[3], lo[3];
    node_box(tree, D, lv, gm, c, w, lo);
    const uint64_t key = node_key(C.seed, tree, lv, gm, c0, c1, c2);
    double S = 0.0, mn = INFINITY, mx = -INFINITY;
    uint64_t cg = SPLITMIX_GAMMA;   // counter 3j + 1 of sample j = 0
    for (int j = 0; j < C.n_samples; j++, cg += 3 * SPLITMIX_GAMMA) {
        const double x0 = lo[0] + sample_unit(key, cg) * w[0];
        const double x1 = lo[1] + sample_unit(key, cg + SPLITMIX_GAMMA) * w[1];
        const double x2 = lo[2] + sample_unit(key, cg + 2 * SPLITMIX_GAMMA) * w[2];
        const double r = density_at(D, x0, x1, x2, bin_start);
        S = S + r;
        mn = fmin(mn, r);
        mx = fmax(mx, r);
    }
    return decide_node(C, lv, w, S, mn, mx);
}

__device__ inline double read_lane_f64(double v, int lane)
{
    int lo = __double2loint(v), hi = __double2hiint(v);
    return __hiloint2double(__builtin_amdgcn_readlane(hi, lane), __builtin_amdgcn_readlane(lo, lane));
}

// Value of v in lane j of the caller's group of G lanes (groups are aligned
// in the wavefront; every lane of the group is active).
template <int G>
__device__ inline double group_read_f64(double v, int j)
{
    if (G == 64) return read_lane_f64(v, j);
    return __shfl(v, j, G);
}

// G lanes per node (G a power of two, 2 <= G <= 64; all lanes of a group call
// it with the same node): lane l of the group draws samples l, l+G, ...; each
// lane keeps its own copy of S and adds the G values of a round in sample
// order, so S is the same sequential sum as with one lane per node.  Min and
// max are order-free.  The lanes of a group sample one node and so mostly
// walk the same clump bin, which pays when bins hold many clumps; groups also
// shorten the sequence of samples per lane on levels too small to fill the
// chip.
template <int G>
__device__ inline NodeSample sample_node_group(int tree, const Dens &D, const CritDev &C, int lv, uint32_t gm,
                                               uint32_t c0, uint32_t c1, uint32_t c2,
                                               const int64_t *__restrict__ bin_start)
{
    const int l = threadIdx.x & (G - 1);
    const uint32_t c[3] = {c0, c1, c2};
    double w[3], lo[3];
    node_box(tree, D, lv, gm, c, w, lo);
    const uint64_t key = node_key(C.seed, tree, lv, gm, c0, c1, c2);
    double S = 0.0, mn = INFINITY, mx = -INFINITY;
    uint64_t cg = uint64_t(3 * l + 1) * SPLITMIX_GAMMA;   // counter 3j + 1 of sample j = l
    for (int base = 0; base < C.n_samples; base += G, cg += uint64_t(3 * G) * SPLITMIX_GAMMA) {
        const int j = base + l;
        double r = 0.0;
        if (j < C.n_samples) {
            const double x0 = lo[0] + sample_unit(key, cg) * w[0];
            const double x1 = lo[1] + sample_unit(key, cg + SPLITMIX_GAMMA) * w[1];
            const double x2 = lo[2] + sample_unit(key, cg + 2 * SPLITMIX_GAMMA) * w[2];
            r = density_at(D, x0, x1, x2, bin_start);
            mn = fmin(mn, r);
            mx = fmax(mx, r);
        }
        const int m = min(G, C.n_samples - base);
        for (int jj = 0; jj < m; jj++) S = S + group_read_f64<G>(r, jj);
    }
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) {
        mn = fmin(mn, __shfl_xor(mn, o, 64));
        mx = fmax(mx, __shfl_xor(mx, o, 64));
    }
    return decide_node(C, lv, w, S, mn, mx);
}

// Node sampling with at least 16 lanes per node for densities with at least
// this many clumps (clustered clumps fill bins with many of them; lanes on
// different nodes would then loop over different bins), and with at least 4
// where a clump bin holds at least one clump on average.
constexpr int64_t WAVE_SAMPLING_CLUMPS = 10000;

// Least lanes per node for a density with n_clumps clumps and bin_load
// clump records per bin on average.
inline int density_group_min(int64_t n_clumps, double bin_load)
{
    if (n_clumps >= WAVE_SAMPLING_CLUMPS) return 16;
    return bin_load >= 1.0 ? 4 : 1;
}

// Lanes kept busy by node sampling: eight wavefronts on each of the 1024
// SIMDs of the chip.
constexpr int64_t SAMPLE_LANES = int64_t(1) << 19;

// Lanes per node for a level of n nodes (over all grids sampled together):
// the largest power of two up to 64 with n times it within SAMPLE_LANES (one
// lane per node once the level alone fills the chip), so a small level is
// not a few lanes each drawing all n_samples points in sequence while the
// rest idle; at least gmin (from density_group_min).  Every group size gives
// the same bits.
__host__ __device__ inline int sample_group(int64_t n, int gmin)
{
    int g = 1;
    while (g < 64 && n * (2 * g) <= SAMPLE_LANES) g *= 2;
    return g < gmin ? gmin : g;
}

// Cell coordinates and geometry of child k of a node with geometry gm (k-d:
// across its split axis, lower half first; octree: octant k = bx + 2 by +
// 4 bz).  The child's split axis is left open (3).
__host__ __device__ inline void child_coord(int tree, uint32_t gm, const uint32_t c[3], int k, uint32_t cc[3],
                                            uint32_t *cgm)
{
    cc[0] = c[0];
    cc[1] = c[1];
    cc[2] = c[2];
    int dep[3] = {geom_depth(gm, 0), geom_depth(gm, 1), geom_depth(gm, 2)};
    if (tree != OCT) {
        const int a = geom_axis(gm);
        cc[a] = 2u * c[a] + uint32_t(k);
        dep[a]++;
    } else {
        for (int d = 0; d < 3; d++) {
            cc[d] = 2u * c[d] + uint32_t((k >> d) & 1);
            dep[d]++;
        }
    }
    *cgm = geom_make(dep[0], dep[1], dep[2], 3);
}

// Geometry of a node of an octree or cyclic k-d tree at level lv.
__host__ __device__ inline uint32_t level_geom(int tree, int lv)
{
    return geom_make(axis_depth(tree, lv, 0), axis_depth(tree, lv, 1), axis_depth(tree, lv, 2),
                     tree == KD ? lv % 3 : 3);
}

}  // namespace hg
