// The optical-depth recipe of Sect. 4.1: build with the mass criterion only,
// take the optical depth of every cell (Eq. 2 with the cell's sampled mass),
// set tau_max to the value at position floor(fraction N_cells) of the
// ascending order, build again with both criteria.
//
// The order statistic is found on the device by a most-significant-digit
// radix select over the bit patterns of the (non-negative) optical depths,
// 16 bits per pass: a histogram of the candidates' next digit, then one block
// finds the digit holding the wanted rank and narrows the candidates.
#include <math.h>
#include <string.h>

#include <algorithm>

#include "common.h"
#include "sampling.h"

namespace hg {

namespace {

constexpr int RT = 256;
constexpr int DIGITS = 1 << 16;

struct SelectState {
    unsigned long long prefix, mask;
    long long k;
};

__global__ void __launch_bounds__(RT)
    k_leaf_tau(int tree, double side, const int32_t *__restrict__ node_of, const uint8_t *__restrict__ level,
               const uint32_t *__restrict__ geom, const double *__restrict__ S, double kappa, int n_samples,
               int64_t n, double *__restrict__ out)
{
    const int64_t l = int64_t(blockIdx.x) * RT + threadIdx.x;
    if (l >= n) return;
    const int32_t nd = node_of[l];
    const int lv = level[nd];
    double w[3];
    for (int d = 0; d < 3; d++) w[d] = ldexp(side, -node_depth(tree, lv, geom, nd, d));
    out[l] = node_tau(kappa, S[nd], w, n_samples);
}

__global__ void __launch_bounds__(RT) k_select_init(SelectState *st, long long k, unsigned *hist)
{
    for (int i = threadIdx.x; i < DIGITS; i += RT) hist[i] = 0u;
    if (threadIdx.x == 0) {
        st->prefix = 0ull;
        st->mask = 0ull;
        st->k = k;
    }
}

__global__ void __launch_bounds__(RT)
    k_select_hist(const double *__restrict__ v, int64_t n, const SelectState *__restrict__ st, int shift,
                  unsigned *__restrict__ hist)
{
    const unsigned long long prefix = st->prefix, mask = st->mask;
    for (int64_t i = int64_t(blockIdx.x) * RT + threadIdx.x; i < n; i += int64_t(gridDim.x) * RT) {
        const unsigned long long b = (unsigned long long)__double_as_longlong(v[i]);
        if ((b & mask) == prefix) atomicAdd(&hist[(b >> shift) & 0xFFFFull], 1u);
    }
}

// One block: the digit holding rank k among the candidates; narrows the
// candidates to it and clears the histogram for the next pass.
__global__ void __launch_bounds__(RT) k_select_pick(SelectState *st, int shift, unsigned *hist)
{
    __shared__ long long part[RT];
    __shared__ int found;
    constexpr int PER = DIGITS / RT;
    const int t = threadIdx.x;
    long long sum = 0;
    for (int j = 0; j < PER; j++) sum += hist[t * PER + j];
    part[t] = sum;
    if (t == 0) found = -1;
    __syncthreads();
    if (t == 0) {
        long long run = 0, k = st->k;
        for (int j = 0; j < RT; j++) {
            if (k < run + part[j]) {
                long long r = run;
                for (int q = 0; q < PER; q++) {
                    const long long c = hist[j * PER + q];
                    if (k < r + c) {
                        found = j * PER + q;
                        st->k = k - r;
                        break;
                    }
                    r += c;
                }
                break;
            }
            run += part[j];
        }
        if (found >= 0) {
            st->prefix |= (unsigned long long)found << shift;
            st->mask |= 0xFFFFull << shift;
        }
    }
    __syncthreads();
    for (int j = 0; j < PER; j++) hist[t * PER + j] = 0u;
}

}  // namespace

// k-th smallest (0-based) of v[0..n), found on the device; *out on the host.
int select_kth(const double *v, int64_t n, int64_t k, double *out, hipStream_t s)
{
    SelectState *st = nullptr;
    unsigned *hist = nullptr;
    int rc = dalloc_n(&st, 1, s);
    if (!rc) rc = dalloc_n(&hist, DIGITS, s);
    if (!rc) {
        k_select_init<<<1, RT, 0, s>>>(st, (long long)k, hist);
        const unsigned blocks = unsigned(std::min<int64_t>((n + RT - 1) / RT, 4096));
        for (int shift = 48; shift >= 0 && !rc; shift -= 16) {
            k_select_hist<<<blocks, RT, 0, s>>>(v, n, st, shift, hist);
            k_select_pick<<<1, RT, 0, s>>>(st, shift, hist);
        }
        SelectState h;
        hipError_t e = hipGetLastError();
        if (!e) e = hipMemcpyAsync(&h, st, sizeof h, hipMemcpyDeviceToHost, s);
        if (!e) e = hipStreamSynchronize(s);
        if (e) rc = set_hip_error(e);
        else memcpy(out, &h.prefix, sizeof(double));
    }
    dfree(st, s);
    dfree(hist, s);
    return rc;
}

}  // namespace hg

using namespace hg;

extern "C" {

int grid_leaf_tau(hg_grid_t g, double kappa, int n_samples, double *tau_out, void *stream)
{
    if (!g || !tau_out || n_samples < 1 || !(kappa >= 0.0) || !isfinite(kappa)) return HG_E_INVAL;
    if (g->n_leaves == 0) return HG_OK;
    k_leaf_tau<<<unsigned((g->n_leaves + RT - 1) / RT), RT, 0, (hipStream_t)stream>>>(
        g->tree, g->side, g->node_of, g->level, g->geom, g->S, kappa, n_samples, g->n_leaves, tau_out);
    HG_CHECK(hipGetLastError());
    return HG_OK;
}

int grid_tau_percentile(hg_grid_t g, double kappa, int n_samples, double fraction, double *tau_max,
                        void *stream)
{
    if (!g || !tau_max || !(fraction >= 0.0 && fraction <= 1.0)) return HG_E_INVAL;
    hipStream_t s = (hipStream_t)stream;
    const int64_t n = g->n_leaves;
    int64_t k = int64_t(floor(fraction * double(n)));
    if (k > n - 1) k = n - 1;
    double *tau = nullptr;
    int rc = dalloc_n(&tau, size_t(n), s);
    if (!rc) rc = grid_leaf_tau(g, kappa, n_samples, tau, stream);
    if (!rc) rc = select_kth(tau, n, k, tau_max, s);
    dfree(tau, s);
    return rc;
}

int grid_build_tau_recipe(const hg_density *dn, const hg_criteria *cr, int tree_type, double fraction,
                          void *stream, hg_grid_t *out, double *tau_max)
{
    if (!dn || !cr || !out || !tau_max || !(fraction >= 0.0 && fraction <= 1.0)) return HG_E_INVAL;
    *out = nullptr;
    hg_criteria c1 = *cr;
    c1.tau_max = INFINITY;
    hg_grid_t g1 = nullptr;
    int rc = grid_build(dn, &c1, tree_type, stream, &g1);
    if (rc) return rc;
    rc = grid_tau_percentile(g1, cr->kappa, cr->n_samples, fraction, tau_max, stream);
    (void)hipStreamSynchronize((hipStream_t)stream);
    grid_free(g1);
    if (rc) return rc;
    hg_criteria c2 = *cr;
    c2.tau_max = *tau_max;
    return grid_build(dn, &c2, tree_type, stream, out);
}

}  // extern "C"
