// Autotuner of the walk's launch shape.  The walk's results do not depend on
// the launch shape (every path is walked by one lane with the same
// arithmetic); its speed does: threads per block, the number of paths a
// wavefront takes from the work queue per atomic and the number of idle
// lanes that trigger a refill from its queue of prepared paths.  The tuner
// times candidate shapes on a caller-supplied sample of the workload with HIP
// events and keeps the fastest, by coordinate descent from the defaults.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "common.h"

namespace hg {

namespace {

const int BLOCKS[] = {128, 256, 512};
const int LDS[] = {0};   // lds_bytes: no longer used by the walk
const int CHUNKS[] = {64, 128, 256, 512, 1024};
const int REFILLS[] = {1, 2, 4, 8, 16};

struct Events {
    hipEvent_t e[4] = {};
    int create()
    {
        for (auto &x : e) HG_CHECK(hipEventCreate(&x));
        return HG_OK;
    }
    ~Events()
    {
        for (auto &x : e)
            if (x) (void)hipEventDestroy(x);
    }
};

// Minimum over reps of the walk time (counting walk plus, in records mode,
// the filling walk) of one candidate.
template <typename RunCount, typename RunFill>
int time_candidate(Events &ev, bool records, int reps, hipStream_t s, RunCount count, RunFill fill,
                   float *best)
{
    *best = INFINITY;
    for (int r = 0; r <= reps; r++) {
        HG_CHECK(hipEventRecord(ev.e[0], s));
        int rc = count();
        if (rc) return rc;
        HG_CHECK(hipEventRecord(ev.e[1], s));
        if (records) {
            HG_CHECK(hipEventRecord(ev.e[2], s));
            rc = fill();
            if (rc) return rc;
            HG_CHECK(hipEventRecord(ev.e[3], s));
        }
        HG_CHECK(hipEventSynchronize(records ? ev.e[3] : ev.e[1]));
        float a = 0.f, b = 0.f;
        HG_CHECK(hipEventElapsedTime(&a, ev.e[0], ev.e[1]));
        if (records) HG_CHECK(hipEventElapsedTime(&b, ev.e[2], ev.e[3]));
        if (r > 0) *best = std::min(*best, a + b);  // the first run warms up
    }
    return HG_OK;
}

int status_error(const TraceStatus *dst, hipStream_t s)
{
    TraceStatus st;
    return read_status(dst, &st, s);
}

// Coordinate descent over the parameter lists; eval(cand, &ms) times one.
template <typename Eval>
int descend_params(hg_trace_opts *best, int nparam, const int *const *vals, const int *nvals,
                   int32_t hg_trace_opts::*const *field, Eval eval, float *best_ms)
{
    int rc = eval(*best, best_ms);
    if (rc) return rc;
    for (int round = 0; round < 2; round++) {
        bool moved = false;
        for (int p = 0; p < nparam; p++) {
            for (int v = 0; v < nvals[p]; v++) {
                hg_trace_opts c = *best;
                if (c.*field[p] == vals[p][v]) continue;
                c.*field[p] = vals[p][v];
                float ms = 0.f;
                if ((rc = eval(c, &ms))) return rc;
                if (ms < 0.99f * *best_ms) {
                    *best = c;
                    *best_ms = ms;
                    moved = true;
                }
            }
        }
        if (!moved) break;
    }
    return HG_OK;
}

}  // namespace
}  // namespace hg

using namespace hg;

extern "C" {

int grid_tune(hg_grid_t g, const double *origins, const double *dirs, int64_t n, hg_trace_opts *opts,
              float *best_ms, void *stream)
{
    if (!g || !opts || n < 1 || !origins || !dirs) return HG_E_INVAL;
    if (opts->precision != HG_FP64 && opts->precision != HG_FP32_RECHECK) return HG_E_INVAL;
    if (opts->mode != HG_TAU_ONLY && opts->mode != HG_RECORDS) return HG_E_INVAL;
    if (!isfinite(opts->kappa)) return HG_E_INVAL;
    hipStream_t s = (hipStream_t)stream;
    const bool records = opts->mode == HG_RECORDS;
    hg_trace_opts base = *opts;
    base.persistent = 3;
    base.flags = 0;
    base.block = 256;
    base.lds_bytes = 0;
    base.chunk = 256;
    base.refill_min = 4;
    hg_trace_out out;
    memset(&out, 0, sizeof out);
    int64_t *tmp = nullptr;
    StatusSlot slot;
    int rc = slot.acquire();
    TraceStatus *const dst = slot.get();
    if (!rc) rc = dalloc_n(&out.tau, size_t(n), s);
    if (!rc) rc = dalloc_n(&out.count, size_t(n), s);
    if (!rc) rc = dalloc_n(&out.offsets, size_t(n) + 1, s);
    if (!rc) rc = dalloc_n(&tmp, scan_tmp_elems(n), s);
    int64_t needed = 0;
    // records mode: the one-pass walk (as grid_trace runs it) unless two passes are asked for
    const int64_t slab = slab_rows(opts, n);
    bool slab_mode = records && opts->passes != 2 && slab > 0;
    const size_t dsz = opts->precision == HG_FP64 ? 8 : 4;
    int32_t *sleaf = nullptr;
    void *sds = nullptr;
    Scratch *w = nullptr;
    if (!rc && slab_mode) {
        const size_t b_leaf = (size_t(n) * size_t(slab) * 4 + 255) & ~size_t(255);
        rc = scratch_acquire(b_leaf + size_t(n) * size_t(slab) * dsz, &w);
        if (!rc) {
            sleaf = static_cast<int32_t *>(scratch_ptr(w));
            sds = static_cast<char *>(scratch_ptr(w)) + b_leaf;
        } else if (rc == HG_E_OOM) {
            rc = HG_OK;   // tune the two-walk records mode, as grid_trace would run it
            slab_mode = false;
        }
    }
    if (!rc) {
        hipError_t e = hipMemsetAsync(dst, 0, sizeof(TraceStatus), s);
        if (e) rc = set_hip_error(e);
    }
    if (!rc) rc = launch_walk(g, dst, origins, dirs, n, &base, &out, WM_COUNT, s, nullptr);
    if (!rc) rc = status_error(dst, s);
    if (!rc && records && !slab_mode) {
        rc = scan_i32_to_i64(out.count, out.offsets, n, tmp, s);
        if (!rc) {
            hipError_t e = hipMemcpyAsync(&needed, out.offsets + n, 8, hipMemcpyDeviceToHost, s);
            if (!e) e = hipStreamSynchronize(s);
            if (e) rc = set_hip_error(e);
        }
        const size_t dsz = opts->precision == HG_FP64 ? 8 : 4;
        if (!rc) rc = dalloc_n(&out.leaf, size_t(std::max<int64_t>(needed, 1)), s);
        if (!rc) rc = dalloc(&out.ds, size_t(std::max<int64_t>(needed, 1)) * dsz, s);
        out.capacity = needed;
    }
    Events ev;
    if (!rc) rc = ev.create();
    if (!rc) {
        WalkArgs SA = walk_args(g, dst, origins, dirs, n, &base, &out);
        SA.leaf = sleaf;
        SA.ds = sds;
        SA.slab = slab;
        SA.pairs = opts->precision != HG_FP64 ? 1 : 0;   // as grid_trace's persistent slab walk
        auto eval = [&](const hg_trace_opts &c, float *ms) {
            if (slab_mode)
                return time_candidate(
                    ev, false, 3, s, [&]() { return launch_walk_args(g, SA, &c, WM_SLAB, s); },
                    [&]() { return HG_OK; }, ms);
            return time_candidate(
                ev, records, 3, s,
                [&]() { return launch_walk(g, dst, origins, dirs, n, &c, &out, WM_COUNT, s, nullptr); },
                [&]() { return launch_walk(g, dst, origins, dirs, n, &c, &out, WM_FILL, s, nullptr); }, ms);
        };
        const int *vals[] = {LDS, BLOCKS, CHUNKS, REFILLS};
        const int nvals[] = {int(sizeof LDS / sizeof *LDS), int(sizeof BLOCKS / sizeof *BLOCKS),
                             int(sizeof CHUNKS / sizeof *CHUNKS), int(sizeof REFILLS / sizeof *REFILLS)};
        int32_t hg_trace_opts::*const field[] = {&hg_trace_opts::lds_bytes, &hg_trace_opts::block,
                                                 &hg_trace_opts::chunk, &hg_trace_opts::refill_min};
        float ms = 0.f;
        hg_trace_opts best = base;
        rc = descend_params(&best, 4, vals, nvals, field, eval, &ms);
        if (!rc) rc = status_error(dst, s);
        if (!rc) {
            opts->block = best.block;
            opts->lds_bytes = best.lds_bytes;
            opts->chunk = best.chunk;
            opts->refill_min = best.refill_min;
            opts->persistent = 3;
            if (best_ms) *best_ms = ms;
        }
    }
    (void)hipStreamSynchronize(s);
    dfree(out.tau, s);
    dfree(out.count, s);
    dfree(out.offsets, s);
    dfree(out.leaf, s);
    dfree(out.ds, s);
    dfree(tmp, s);
    if (w) scratch_release(w);
    return rc;
}

}  // extern "C"
