// Consumers of the walk: the grid-quality measures of Sect. 3.2 and the
// Monte Carlo interaction point along a path.
//
// * density difference (first measure of Sect. 3.2): rho_t(x) - rho_g(x) at
//   given points, rho_g being the uniform density of the leaf holding x;
// * grid optical depth of a path up to a length s_max (second measure, grid
//   side): sum of kappa rho ds over its crossings, the last one cut at s_max;
// * true optical depth over the same stretch (second measure, true side):
//   Gauss-Legendre quadrature of kappa rho_t with m nodes on every piece
//   between consecutive cell boundaries of the path;
// * interaction point: the crossing at which the cumulative optical depth
//   first reaches a target tau*, and the distance along the path where it
//   does (tau grows linearly inside a cell).
// The path quantities read the crossing records of a records-mode trace (one
// thread per path over its slice of the records).
#include <math.h>
#include <string.h>

#include <vector>

#include "common.h"
#include "sampling.h"

namespace hg {

namespace {

constexpr int QT = 256;
constexpr int GL_MAX = 64;

inline unsigned qblocks(int64_t n) { return unsigned((n + QT - 1) / QT); }

__global__ void __launch_bounds__(QT)
    k_density_diff(Dens D, const int64_t *__restrict__ bin_start, const double *__restrict__ X,
                   const int32_t *__restrict__ leaf, const double *__restrict__ rho, int64_t n,
                   double *__restrict__ out)
{
    const int64_t i = int64_t(blockIdx.x) * QT + threadIdx.x;
    if (i >= n) return;
    const int32_t l = leaf[i];
    out[i] = l < 0 ? __longlong_as_double(0x7ff8000000000000ll)
                   : density_at(D, X[3 * i], X[3 * i + 1], X[3 * i + 2], bin_start) - rho[l];
}

template <typename DsT>
__global__ void __launch_bounds__(QT)
    k_segment_tau(const int64_t *__restrict__ off, const int32_t *__restrict__ leaf,
                  const DsT *__restrict__ ds, const double *__restrict__ rho,
                  const double *__restrict__ s_max, double kappa, int64_t n, double *__restrict__ out)
{
    const int64_t i = int64_t(blockIdx.x) * QT + threadIdx.x;
    if (i >= n) return;
    const double smax = s_max[i];
    double s = 0.0, t = 0.0;
    for (int64_t j = off[i], e = off[i + 1]; j < e && s < smax; j++) {
        const double d = double(ds[j]);
        const double step = fmin(d, smax - s);
        t = t + kappa * rho[leaf[j]] * step;
        s = s + d;
    }
    out[i] = t;
}

template <typename DsT>
__global__ void __launch_bounds__(QT)
    k_interact(const int64_t *__restrict__ off, const int32_t *__restrict__ leaf,
               const DsT *__restrict__ ds, const double *__restrict__ rho,
               const double *__restrict__ tau_star, double kappa, int64_t n,
               int32_t *__restrict__ leaf_out, double *__restrict__ s_out)
{
    const int64_t i = int64_t(blockIdx.x) * QT + threadIdx.x;
    if (i >= n) return;
    const double ts = tau_star[i];
    double s = 0.0, t = 0.0;
    int32_t hit = -1;
    for (int64_t j = off[i], e = off[i + 1]; j < e; j++) {
        const double d = double(ds[j]);
        const int32_t l = leaf[j];
        const double kr = kappa * rho[l];
        const double dt = kr * d;
        if (dt > 0.0 && t + dt >= ts) {
            hit = l;
            s = s + (ts - t) / kr;
            break;
        }
        t = t + dt;
        s = s + d;
    }
    leaf_out[i] = hit;
    s_out[i] = s;
}

template <typename DsT>
__global__ void __launch_bounds__(QT)
    k_true_tau(Dens D, const int64_t *__restrict__ bin_start, const double *__restrict__ O,
               const double *__restrict__ K, const int64_t *__restrict__ off,
               const DsT *__restrict__ ds, const double *__restrict__ s_max, double kappa,
               const double *__restrict__ xg, const double *__restrict__ wg, int m, int64_t n,
               double *__restrict__ out)
{
    const int64_t i = int64_t(blockIdx.x) * QT + threadIdx.x;
    if (i >= n) return;
    const double o0 = O[3 * i], o1 = O[3 * i + 1], o2 = O[3 * i + 2];
    const double k0 = K[3 * i], k1 = K[3 * i + 1], k2 = K[3 * i + 2];
    const double smax = s_max[i];
    double s = 0.0, t = 0.0;
    for (int64_t j = off[i], e = off[i + 1]; j < e && s < smax; j++) {
        const double d = double(ds[j]);
        const double b = fmin(s + d, smax);
        const double half = 0.5 * (b - s);
        const double mid = 0.5 * (b + s);
        double acc = 0.0;
        for (int q = 0; q < m; q++) {
            const double u = mid + half * xg[q];
            acc = acc + wg[q] * density_at(D, o0 + u * k0, o1 + u * k1, o2 + u * k2, bin_start);
        }
        t = t + kappa * half * acc;
        s = s + d;
    }
    out[i] = t;
}

// Gauss-Legendre nodes (ascending) and weights on [-1, 1]: Newton's method on
// the Legendre polynomial P_m from the asymptotic first guesses, P_m and P_m'
// by the three-term recurrence; w = 2 / ((1 - x^2) P_m'(x)^2).
void gauss_legendre(int m, double *x, double *w)
{
    const double pi = 3.14159265358979323846;
    for (int i = 0; i < (m + 1) / 2; i++) {
        double z = cos(pi * (double(i) + 0.75) / (double(m) + 0.5));
        double dp = 0.0;
        for (int it = 0; it < 100; it++) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= m; k++) {
                const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / double(k);
                p0 = p1;
                p1 = p2;
            }
            dp = double(m) * (z * p1 - p0) / (z * z - 1.0);
            const double dz = p1 / dp;
            z -= dz;
            if (fabs(dz) < 1e-16) break;
        }
        // recompute the derivative at the converged root
        double p0 = 1.0, p1 = z;
        for (int k = 2; k <= m; k++) {
            const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / double(k);
            p0 = p1;
            p1 = p2;
        }
        dp = m == 1 ? 1.0 : double(m) * (z * p1 - p0) / (z * z - 1.0);
        const double wi = 2.0 / ((1.0 - z * z) * dp * dp);
        x[i] = -z;
        x[m - 1 - i] = z;
        w[i] = wi;
        w[m - 1 - i] = wi;
    }
    if (m % 2 == 1) x[m / 2] = 0.0;
}

int check_records(const hg_trace_out *rec, int precision, int64_t n)
{
    if (!rec || n < 0) return HG_E_INVAL;
    if (precision != HG_FP64 && precision != HG_FP32_RECHECK) return HG_E_INVAL;
    if (n > 0 && !rec->offsets) return HG_E_INVAL;
    if (n > 0 && rec->capacity > 0 && (!rec->leaf || !rec->ds)) return HG_E_INVAL;
    return HG_OK;
}

}  // namespace
}  // namespace hg

using namespace hg;

extern "C" {

int grid_density_diff(hg_grid_t g, const hg_density *dn, const double *points, int64_t n,
                      double *diff_out, void *stream)
{
    if (!g || !dn || n < 0) return HG_E_INVAL;
    if (n == 0) return HG_OK;
    if (!points || !diff_out) return HG_E_INVAL;
    int rc = check_domain(dn->lo, dn->side);
    if (rc) return rc;
    if (dn->n_clumps < 0 || dn->n_clumps > HG_MAX_CLUMPS) return HG_E_INVAL;
    if (dn->n_clumps > 0 && (!dn->clump_c || !dn->clump_sigma || !dn->clump_amp)) return HG_E_INVAL;
    hipStream_t s = (hipStream_t)stream;
    Dens D;
    DensStore st;
    int32_t *leaf = nullptr;
    rc = prepare_density(dn, s, &st, &D);
    if (!rc) rc = dalloc_n(&leaf, size_t(n), s);
    if (!rc) rc = launch_locate(g, points, n, leaf, s);
    if (!rc) {
        k_density_diff<<<qblocks(n), QT, 0, s>>>(D, (const int64_t *)st.bin_start, points, leaf, g->rho, n,
                                                 diff_out);
        hipError_t e = hipGetLastError();
        if (e) rc = set_hip_error(e);
    }
    dfree(leaf, s);
    release_density(&st, s);
    return rc;
}

int grid_segment_tau(hg_grid_t g, const hg_trace_out *rec, int precision, int64_t n,
                     const double *s_max, double kappa, double *tau_out, void *stream)
{
    if (!g) return HG_E_INVAL;
    int rc = check_records(rec, precision, n);
    if (rc) return rc;
    if (n == 0) return HG_OK;
    if (!s_max || !tau_out || !isfinite(kappa)) return HG_E_INVAL;
    hipStream_t s = (hipStream_t)stream;
    if (precision == HG_FP64)
        k_segment_tau<double><<<qblocks(n), QT, 0, s>>>(rec->offsets, rec->leaf, (const double *)rec->ds,
                                                        g->rho, s_max, kappa, n, tau_out);
    else
        k_segment_tau<float><<<qblocks(n), QT, 0, s>>>(rec->offsets, rec->leaf, (const float *)rec->ds,
                                                       g->rho, s_max, kappa, n, tau_out);
    HG_CHECK(hipGetLastError());
    return HG_OK;
}

int grid_interact(hg_grid_t g, const hg_trace_out *rec, int precision, int64_t n,
                  const double *tau_star, double kappa, int32_t *leaf_out, double *s_out, void *stream)
{
    if (!g) return HG_E_INVAL;
    int rc = check_records(rec, precision, n);
    if (rc) return rc;
    if (n == 0) return HG_OK;
    if (!tau_star || !leaf_out || !s_out || !(kappa > 0.0) || !isfinite(kappa)) return HG_E_INVAL;
    hipStream_t s = (hipStream_t)stream;
    if (precision == HG_FP64)
        k_interact<double><<<qblocks(n), QT, 0, s>>>(rec->offsets, rec->leaf, (const double *)rec->ds,
                                                     g->rho, tau_star, kappa, n, leaf_out, s_out);
    else
        k_interact<float><<<qblocks(n), QT, 0, s>>>(rec->offsets, rec->leaf, (const float *)rec->ds,
                                                    g->rho, tau_star, kappa, n, leaf_out, s_out);
    HG_CHECK(hipGetLastError());
    return HG_OK;
}

int grid_true_tau(hg_grid_t g, const hg_density *dn, const double *origins, const double *dirs,
                  const hg_trace_out *rec, int precision, int64_t n, const double *s_max, double kappa,
                  int m, double *tau_out, void *stream)
{
    if (!g || !dn) return HG_E_INVAL;
    int rc = check_records(rec, precision, n);
    if (rc) return rc;
    if (m < 1 || m > GL_MAX || !isfinite(kappa)) return HG_E_INVAL;
    if (n == 0) return HG_OK;
    if (!origins || !dirs || !s_max || !tau_out) return HG_E_INVAL;
    if ((rc = check_domain(dn->lo, dn->side))) return rc;
    if (dn->n_clumps < 0 || dn->n_clumps > HG_MAX_CLUMPS) return HG_E_INVAL;
    if (dn->n_clumps > 0 && (!dn->clump_c || !dn->clump_sigma || !dn->clump_amp)) return HG_E_INVAL;
    hipStream_t s = (hipStream_t)stream;
    std::vector<double> hx(size_t(2 * m));
    gauss_legendre(m, hx.data(), hx.data() + m);
    Dens D;
    DensStore st;
    double *gl = nullptr;
    rc = prepare_density(dn, s, &st, &D);
    if (!rc) rc = dalloc_n(&gl, size_t(2 * m), s);
    if (!rc) {
        hipError_t e = hipMemcpyAsync(gl, hx.data(), sizeof(double) * hx.size(), hipMemcpyHostToDevice, s);
        if (!e) e = hipStreamSynchronize(s);   // hx is a host temporary
        if (e) rc = set_hip_error(e);
    }
    if (!rc) {
        if (precision == HG_FP64)
            k_true_tau<double><<<qblocks(n), QT, 0, s>>>(D, (const int64_t *)st.bin_start, origins, dirs,
                                                         rec->offsets, (const double *)rec->ds, s_max, kappa,
                                                         gl, gl + m, m, n, tau_out);
        else
            k_true_tau<float><<<qblocks(n), QT, 0, s>>>(D, (const int64_t *)st.bin_start, origins, dirs,
                                                        rec->offsets, (const float *)rec->ds, s_max, kappa,
                                                        gl, gl + m, m, n, tau_out);
        hipError_t e = hipGetLastError();
        if (e) rc = set_hip_error(e);
    }
    dfree(gl, s);
    release_density(&st, s);
    return rc;
}

}  // extern "C"
