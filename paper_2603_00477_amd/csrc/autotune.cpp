// Model-seeded autotuner: picks (path, T, VALU rows per workgroup) for a plan.
//
// Candidates are every available (path, T <= min(4, steps)) ranked by the
// roofline model's predicted GStencil/s; the best `max_candidates` of them
// are timed on the caller's data (VALU candidates also with 64 and 128 rows
// per workgroup besides the automatic choice).  The fastest configuration is
// applied to the plan and cached per (shape, d, r, dtype, boundary, dims) for
// later plans of the same problem.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "internal.h"

namespace {

using Key = std::tuple<int, int, int, int, int, int64_t, int64_t, int64_t>;
struct Choice {
    int path, T, rows;
    double gst;
};
std::mutex g_mu;
std::map<Key, Choice> g_cache;

Key key_of(const stencil_plan_info_t &i)
{
    return Key(i.shape, i.d, i.r, i.dtype, i.boundary, i.dims[0], i.dims[1], i.dims[2]);
}

struct Cand {
    int path, T, rows;
    double pred;
};

// Switch a plan to (path, T, rows); either order of the first two may be the
// only valid one (each intermediate state must itself be runnable).
int apply(stencil_plan_t plan, int path, int T, int rows)
{
    int rc = stencil_plan_set(plan, STENCIL_OPT_PATH, path);
    if (!rc) rc = stencil_plan_set(plan, STENCIL_OPT_T, T);
    if (rc) {
        rc = stencil_plan_set(plan, STENCIL_OPT_T, T);
        if (!rc) rc = stencil_plan_set(plan, STENCIL_OPT_PATH, path);
    }
    if (!rc) rc = stencil_plan_set(plan, STENCIL_OPT_TILE_ROWS, rows);
    return rc;
}

}  // namespace

using namespace stl;

extern "C" int stencil_plan_autotune(stencil_plan_t plan, const void *in, void *out, int64_t steps,
                                     int max_candidates, void *stream_v, double *best_gst)
{
    if (!plan || !in || !out) return fail(STENCIL_ERR_INVALID_ARG, "stencil_plan_autotune: NULL argument");
    if (steps < 1 || max_candidates < 1)
        return fail(STENCIL_ERR_INVALID_ARG, "stencil_plan_autotune: steps and max_candidates must be >= 1");
    hipStream_t stream = (hipStream_t)stream_v;
    stencil_plan_info_t info;
    stencil_plan_info(plan, &info);
    const Key key = key_of(info);
    {
        std::lock_guard<std::mutex> lk(g_mu);
        auto it = g_cache.find(key);
        if (it != g_cache.end() && it->second.T <= steps) {
            const Choice c = it->second;
            int rc = apply(plan, c.path, c.T, c.rows);
            if (best_gst) *best_gst = c.gst;
            return rc;
        }
    }
    // rank (path, T) by the model
    std::vector<Cand> cands;
    const int Tmax = (int)std::min<int64_t>(4, steps);
    for (int path : {STENCIL_PATH_VALU, STENCIL_PATH_MFMA, STENCIL_PATH_MFMA_SPARSE}) {
        if (info.dtype == STENCIL_F32_BF16X3 && path == STENCIL_PATH_VALU) continue;
        for (int T = 1; T <= Tmax; ++T) {
            stencil_model_in_t mi;
            std::memset(&mi, 0, sizeof mi);
            mi.shape = info.shape;
            mi.d = info.d;
            mi.r = info.r;
            mi.T = T;
            mi.dtype = info.dtype;
            mi.sparse = path == STENCIL_PATH_MFMA_SPARSE;
            stencil_model_out_t mo;
            if (stencil_model_predict(&mi, nullptr, &mo)) continue;
            const double pred = path == STENCIL_PATH_VALU ? mo.gst_valu : mo.gst_mfma;
            cands.push_back({path, T, 0, pred});
        }
    }
    std::stable_sort(cands.begin(), cands.end(), [](const Cand &a, const Cand &b) { return a.pred > b.pred; });
    std::vector<Cand> trial;
    for (const Cand &c : cands) {
        if ((int)trial.size() >= max_candidates) break;
        // skip combinations the library cannot run
        if (apply(plan, c.path, c.T, 0)) continue;
        trial.push_back(c);
        if (c.path == STENCIL_PATH_VALU && info.d == 2) {
            trial.push_back({c.path, c.T, 64, c.pred});
            trial.push_back({c.path, c.T, 128, c.pred});
        }
    }
    if (trial.empty()) return fail(STENCIL_ERR_UNSUPPORTED, "stencil_plan_autotune: no runnable candidate");
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return fail(STENCIL_ERR_HIP, "stencil_plan_autotune: hipEventCreate");
    Choice best{-1, 0, 0, -1.0};
    int rc = STENCIL_OK;
    double npts = 1;
    for (int i = 0; i < info.d; ++i) npts *= (double)info.dims[i];
    for (const Cand &c : trial) {
        rc = apply(plan, c.path, c.T, c.rows);
        if (rc) break;
        // a probe of whole passes: 2 passes (or all steps if fewer)
        const int64_t probe = std::min<int64_t>(steps, 2 * (int64_t)c.T);
        rc = stencil_run(plan, in, out, probe, stream);  // warm-up (uploads operands)
        if (rc) break;
        float ms = 0.f;
        if (hipEventRecord(e0, stream) != hipSuccess) { rc = fail(STENCIL_ERR_HIP, "hipEventRecord"); break; }
        for (int rep = 0; rep < 2 && !rc; ++rep) rc = stencil_run(plan, in, out, probe, stream);
        if (rc) break;
        if (hipEventRecord(e1, stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
            rc = fail(STENCIL_ERR_HIP, "stencil_plan_autotune: event timing");
            break;
        }
        const double gst = npts * (double)probe * 2 / (ms * 1e-3) / 1e9;
        if (gst > best.gst) best = {c.path, c.T, c.rows, gst};
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    rc = apply(plan, best.path, best.T, best.rows);
    if (rc) return rc;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        g_cache[key] = best;
    }
    if (best_gst) *best_gst = best.gst;
    return STENCIL_OK;
}
