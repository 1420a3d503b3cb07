// Plans, weight expansion, composite kernels and the pass driver.
//
// A plan is host state plus lazily allocated device state (scratch grid and
// MFMA operand fragments): everything up to the first run is host-only, so
// argument checking, model results and pass schedules need no GPU.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "internal.h"

namespace stl {

static thread_local std::string g_last_error;

int fail(int code, const std::string &msg)
{
    g_last_error = msg;
    return code;
}

int dtype_bytes(int dtype)
{
    switch (dtype) {
    case STENCIL_F64: return 8;
    case STENCIL_F32: return 4;
    case STENCIL_BF16: return 2;
    case STENCIL_F16: return 2;
    case STENCIL_F32_BF16X3: return 4;
    default: return 0;
    }
}

// Canonical order (paper's patterns: box = full hyper-rectangle of radius r,
// star = points on the coordinate axes):
//   box : row-major over (o_0..o_{d-1}) in [-r, r]^d, last axis fastest
//   star: centre, then axis 0 offsets -r..-1, +1..+r, then axis 1, ...
int pattern_offsets(int shape, int d, int r, std::vector<int> *offs)
{
    if (d < 1 || d > kMaxD || r < 0) return -1;
    std::vector<int> o;
    if (shape == STENCIL_BOX) {
        const int side = 2 * r + 1;
        int total = 1;
        for (int i = 0; i < d; ++i) total *= side;
        o.resize((size_t)total * d);
        for (int idx = 0; idx < total; ++idx) {
            int rem = idx;
            for (int ax = d - 1; ax >= 0; --ax) {
                o[(size_t)idx * d + ax] = rem % side - r;
                rem /= side;
            }
        }
    } else if (shape == STENCIL_STAR) {
        o.assign((size_t)d, 0);
        for (int ax = 0; ax < d; ++ax)
            for (int k = -r; k <= r; ++k) {
                if (k == 0) continue;
                std::vector<int> v((size_t)d, 0);
                v[ax] = k;
                o.insert(o.end(), v.begin(), v.end());
            }
    } else {
        return -1;
    }
    const int K = (int)(o.size() / d);
    if (offs) *offs = std::move(o);
    return K;
}

// T-fold composite: W_{t+1}[q] = sum_o w[o] W_t[q - o]  (two steps of
// u'[x] = sum_o w[o] u[x+o] couple x to x+o+p with weight w[o] w[p]).
void compose_dense(int shape, int d, int r, const double *w, int T, std::vector<double> *out)
{
    std::vector<int> offs;
    const int K = pattern_offsets(shape, d, r, &offs);
    int Rc = r;  // radius of the current composite
    int side = 2 * Rc + 1;
    size_t n = 1;
    for (int i = 0; i < d; ++i) n *= side;
    std::vector<double> cur(n, 0.0);
    auto lin = [&](const int *q, int rad) {
        size_t l = 0;
        for (int i = 0; i < d; ++i) l = l * (2 * rad + 1) + (q[i] + rad);
        return l;
    };
    for (int k = 0; k < K; ++k) cur[lin(&offs[(size_t)k * d], Rc)] += w[k];
    for (int t = 1; t < T; ++t) {
        const int Rn = Rc + r;
        const int sn = 2 * Rn + 1;
        size_t nn = 1;
        for (int i = 0; i < d; ++i) nn *= sn;
        std::vector<double> nxt(nn, 0.0);
        // iterate over the current composite's displacements
        std::vector<int> q(d, -Rc);
        for (size_t idx = 0; idx < cur.size(); ++idx) {
            size_t rem = idx;
            for (int ax = d - 1; ax >= 0; --ax) {
                q[ax] = (int)(rem % (2 * Rc + 1)) - Rc;
                rem /= (2 * Rc + 1);
            }
            const double cv = cur[idx];
            if (cv == 0.0) continue;
            for (int k = 0; k < K; ++k) {
                int p[kMaxD];
                for (int i = 0; i < d; ++i) p[i] = q[i] + offs[(size_t)k * d + i];
                nxt[lin(p, Rn)] += w[k] * cv;
            }
        }
        cur.swap(nxt);
        Rc = Rn;
    }
    *out = std::move(cur);
}

int device_cu_count()
{
    int dev = 0, n = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 256;
    return n > 0 ? n : 256;
}

const KernelEntry *find_kernel(int path, int dtype, int shape, int d, int r, int t)
{
    static const std::vector<const std::vector<KernelEntry> *> tables = all_kernel_tables();
    for (const auto *tab : tables)
        for (const auto &e : *tab)
            if (e.path == path && e.dtype == dtype && e.d == d && (e.shape == shape || e.shape < 0) &&
                (e.r == r || e.r < 0) && (e.t == t || e.t < 0))
                return &e;
    return nullptr;
}

}  // namespace stl

using namespace stl;

namespace {

bool valid_dtype(int dt) { return dt >= STENCIL_F64 && dt <= STENCIL_F32_BF16X3; }

bool has_path(int path, int dtype, int shape, int d, int r, int T)
{
    if (path == STENCIL_PATH_VALU)
        return find_kernel(STENCIL_PATH_VALU, dtype, shape, d, r, T) != nullptr ||
               find_kernel(STENCIL_PATH_VALU, dtype, shape, d, r, 1) != nullptr;
    return find_kernel(path, dtype, shape, d, r, T) != nullptr;
}

// Model results for the plan's (shape, d, r, T, dtype); `sparse`: the matrix
// side on 2:4 structured-sparse instructions (its peak and layout).
void plan_model(stencil_plan_s *p, bool sparse = false)
{
    stencil_model_in_t mi;
    std::memset(&mi, 0, sizeof mi);
    mi.shape = p->shape;
    mi.d = p->d;
    mi.r = p->r;
    mi.T = p->T;
    mi.dtype = p->dtype;
    mi.sparse = sparse ? 1 : 0;
    stencil_model_out_t mo;
    stencil_model_predict(&mi, nullptr, &mo);
    p->K_T = mo.K_T;
    p->alpha = mo.alpha;
    p->S = mo.S;
    p->gamma = mo.gamma;
    p->pred_valu = mo.gst_valu;
    p->pred_mfma = mo.gst_mfma;
    p->pred_winner = mo.winner;
    p->scenario = mo.scenario;
}

int resolve_path(stencil_plan_s *p)
{
    const bool v = has_path(STENCIL_PATH_VALU, p->dtype, p->shape, p->d, p->r, p->T);
    const bool m_built = has_path(STENCIL_PATH_MFMA, p->dtype, p->shape, p->d, p->r, p->T);
    const bool sp_built = has_path(STENCIL_PATH_MFMA_SPARSE, p->dtype, p->shape, p->d, p->r, p->T);
    const bool seq_built = has_path(STENCIL_PATH_MFMA_SEQ, p->dtype, p->shape, p->d, p->r, p->T);
    // a kernel-fused Dirichlet pass needs a VALU kernel of the same depth for
    // its boundary band (launch_fixup)
    const bool band_ok = p->boundary == STENCIL_PERIODIC || p->T == 1 ||
                         find_kernel(STENCIL_PATH_VALU, p->dtype, p->shape, p->d, p->r, p->T) != nullptr;
    const bool m = m_built && band_ok;
    int path = p->path_req;
    if (path == STENCIL_PATH_AUTO) {
        // the compensated mode exists only on the matrix path (its VALU
        // instances serve the Dirichlet band fix-up)
        if (p->dtype == STENCIL_F32_BF16X3) path = STENCIL_PATH_MFMA;
        else path = (p->pred_winner > 0 && m) ? STENCIL_PATH_MFMA : (v ? STENCIL_PATH_VALU : STENCIL_PATH_MFMA);
    }
    if (path == STENCIL_PATH_VALU && !v)
        return fail(STENCIL_ERR_UNSUPPORTED, "VALU path not built for this dtype/shape/d/r");
    if (path == STENCIL_PATH_MFMA && !m_built)
        return fail(STENCIL_ERR_UNSUPPORTED, "MFMA path not built for this dtype/shape/d/r/T");
    if (path == STENCIL_PATH_MFMA_SPARSE && !sp_built)
        return fail(STENCIL_ERR_UNSUPPORTED,
                    "2:4 sparse MFMA path not built for this dtype/shape/d/r/T (bf16/f16, d = 2, r*T <= 7)");
    if (path == STENCIL_PATH_MFMA_SEQ && !seq_built)
        return fail(STENCIL_ERR_UNSUPPORTED,
                    "sequential-step MFMA path not built for this dtype/shape/d/r/T (d = 2, r <= 3, T <= 4)");
    if (is_kernel_fused_path(path) && !band_ok)
        return fail(STENCIL_ERR_UNSUPPORTED,
                    "Dirichlet MFMA plan needs a fused VALU kernel of the same T for its boundary band; "
                    "use a periodic boundary or another T");
    if (p->dtype == STENCIL_F32_BF16X3 && path != STENCIL_PATH_MFMA)
        return fail(STENCIL_ERR_UNSUPPORTED, "bf16x3 is an MFMA-only mode");
    if (is_kernel_fused_path(path) && p->boundary == STENCIL_PERIODIC)
        for (int i = 0; i < p->d; ++i)
            if (p->dims[i] < 2 * (int64_t)p->r * p->T + 1)
                return fail(STENCIL_ERR_INVALID_ARG,
                            "periodic MFMA plan needs every dim >= 2*r*T + 1");
    p->path = path;
    return STENCIL_OK;
}

void free_device(stencil_plan_s *p)
{
    if (p->scratch) (void)hipFree(p->scratch);
    p->scratch = nullptr;
    for (void *f : p->afrag)
        if (f) (void)hipFree(f);
    for (void *f : p->afrag_lo)
        if (f) (void)hipFree(f);
    p->afrag.clear();
    p->afrag_lo.clear();
    p->device = -1;
}

size_t grid_bytes(const stencil_plan_s *p) { return (size_t)p->npts * dtype_bytes(p->dtype); }

// Operand fragments of the plan's path for a pass of t steps (empty for a
// depth the path has no kernel for).
void build_fragments(const stencil_plan_s *p, int t, std::vector<uint8_t> *hi, std::vector<uint8_t> *lo)
{
    hi->clear();
    lo->clear();
    if (!find_kernel(p->path, p->dtype, p->shape, p->d, p->r, t)) return;
    if (p->path == STENCIL_PATH_MFMA_SPARSE)
        mfma_build_sparse_fragments(p->shape, p->r, p->w.data(), t, p->dtype, hi);
    else if (p->path == STENCIL_PATH_MFMA_SEQ)  // the single step's band, whatever the depth
        mfma_build_fragments(p->shape, p->d, p->r, p->w.data(), 1, p->dtype, hi, lo);
    else if (mfma_row_layout(p->dtype, p->d, p->shape, p->r, t))
        mfma_build_row_fragments(p->shape, p->r, p->w.data(), t, p->dtype, hi);
    else
        mfma_build_fragments(p->shape, p->d, p->r, p->w.data(), t, p->dtype, hi, lo);
}

size_t fragment_bytes(const stencil_plan_s *p)
{
    if (!is_mfma_path(p->path)) return 0;
    size_t total = 0;
    for (int t = 1; t <= p->T; ++t) {
        std::vector<uint8_t> hi, lo;
        build_fragments(p, t, &hi, &lo);
        total += hi.size() + lo.size();
    }
    return total;
}

int upload_fragments(stencil_plan_s *p);

// Device state of a plan on the current device: MFMA operands always, the
// ping-pong scratch grid only when a run needs two or more passes.
int ensure_device(stencil_plan_s *p, bool need_scratch)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(STENCIL_ERR_HIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
    if (p->device != dev) {
        free_device(p);
        int rc = upload_fragments(p);
        if (rc) return rc;
        p->device = dev;
    }
    if (need_scratch && !p->scratch) {
        e = hipMalloc(&p->scratch, std::max<size_t>(grid_bytes(p), 256));
        if (e != hipSuccess) {
            p->scratch = nullptr;
            return fail(STENCIL_ERR_OOM, std::string("hipMalloc scratch: ") + hipGetErrorString(e));
        }
        p->scratch_bytes = grid_bytes(p);
    }
    return STENCIL_OK;
}

int upload_fragments(stencil_plan_s *p)
{
    hipError_t e;
    if (is_mfma_path(p->path)) {
        p->afrag.assign(p->T + 1, nullptr);
        p->afrag_lo.assign(p->T + 1, nullptr);
        for (int t = 1; t <= p->T; ++t) {
            std::vector<uint8_t> hi, lo;
            build_fragments(p, t, &hi, &lo);
            for (int part = 0; part < 2; ++part) {
                const std::vector<uint8_t> &v = part ? lo : hi;
                if (v.empty()) continue;
                void *ptr = nullptr;
                e = hipMalloc(&ptr, v.size());
                if (e != hipSuccess) {
                    free_device(p);
                    return fail(STENCIL_ERR_OOM, std::string("hipMalloc fragments: ") + hipGetErrorString(e));
                }
                e = hipMemcpy(ptr, v.data(), v.size(), hipMemcpyHostToDevice);
                if (e != hipSuccess) {
                    (void)hipFree(ptr);
                    free_device(p);
                    return fail(STENCIL_ERR_HIP, std::string("hipMemcpy fragments: ") + hipGetErrorString(e));
                }
                (part ? p->afrag_lo : p->afrag)[t] = ptr;
            }
        }
    }
    return STENCIL_OK;
}

struct PassDesc {
    int path;
    int t;
    const KernelEntry *k;
    bool fixup;  // Dirichlet band of a kernel-fused MFMA pass redone by sequential steps
};

// Passes of a run: floor(steps/T) passes of T steps, then one of steps mod T.
// A depth without a kernel of the plan's path falls back to the VALU path at
// that depth, or to single-step passes.
std::vector<PassDesc> schedule(const stencil_plan_s *p, int64_t steps)
{
    std::vector<int> depths;
    for (int64_t i = 0; i < steps / p->T; ++i) depths.push_back(p->T);
    if (steps % p->T) depths.push_back((int)(steps % p->T));
    std::vector<PassDesc> out;
    for (int t : depths) {
        const KernelEntry *k = find_kernel(p->path, p->dtype, p->shape, p->d, p->r, t);
        int path = p->path;
        if (!k && is_mfma_path(path)) {
            k = find_kernel(STENCIL_PATH_VALU, p->dtype, p->shape, p->d, p->r, t);
            path = STENCIL_PATH_VALU;
        }
        if (k) {
            const bool fix = is_kernel_fused_path(path) && p->boundary == STENCIL_DIRICHLET && t > 1;
            out.push_back({path, t, k, fix});
        } else {
            const KernelEntry *k1 = find_kernel(STENCIL_PATH_VALU, p->dtype, p->shape, p->d, p->r, 1);
            for (int i = 0; i < t; ++i) out.push_back({STENCIL_PATH_VALU, 1, k1, false});
        }
    }
    return out;
}

PassArgs base_args(const stencil_plan_s *p, int t)
{
    PassArgs a;
    std::memset(&a, 0, sizeof a);
    for (int i = 0; i < kMaxD; ++i) {
        a.dims[i] = i < p->d ? p->dims[i] : 1;
        a.region_lo[i] = 0;
        a.region_hi[i] = (int)a.dims[i];
    }
    a.d = p->d;
    a.boundary = p->boundary;
    a.halo = p->halo;
    a.steps = t;
    a.w = p->w.data();
    a.offs = p->offs.data();
    a.K = p->K;
    a.tile_rows = p->tile_rows;
    a.R = p->r * t;
    a.num_cu = device_cu_count();
    return a;
}

// Dirichlet band of a kernel-fused pass: points within r*(t-1) of the
// boundary, recomputed by t sequential steps (VALU) into dst.
hipError_t launch_fixup(const stencil_plan_s *p, int t, const void *src, void *dst, hipStream_t s)
{
    // for bf16x3 this finds the float-storage, FP64-arithmetic VALU variant
    const KernelEntry *k = find_kernel(STENCIL_PATH_VALU, p->dtype, p->shape, p->d, p->r, t);
    if (!k) return hipErrorNotSupported;
    const int band = p->r * (t - 1);
    for (int ax = 0; ax < p->d; ++ax) {
        for (int side = 0; side < 2; ++side) {
            PassArgs a = base_args(p, t);
            a.src = src;
            a.dst = dst;
            // slabs: axis ax restricted to the band; earlier axes exclude their bands
            for (int i = 0; i < ax; ++i) {
                a.region_lo[i] = std::min<int64_t>(band, a.dims[i]);
                a.region_hi[i] = std::max<int64_t>(a.dims[i] - band, a.region_lo[i]);
            }
            const int n = (int)a.dims[ax];
            const int b = std::min(band, n);
            if (side == 0) {
                a.region_lo[ax] = 0;
                a.region_hi[ax] = b;
            } else {
                a.region_lo[ax] = std::max(n - b, b);
                a.region_hi[ax] = n;
            }
            bool empty = false;
            for (int i = 0; i < p->d; ++i) empty |= a.region_hi[i] <= a.region_lo[i];
            if (empty) continue;
            hipError_t e = k->launch(a, s);
            if (e != hipSuccess) return e;
        }
    }
    return hipSuccess;
}

// `scratch` holds the intermediate grid of multi-pass runs (at least one
// grid of the plan's dims and dtype when the schedule has two or more passes).
int run_one(stencil_plan_s *p, const void *in, void *out, int64_t steps, hipStream_t stream,
            void *scratch)
{
    const size_t bytes = grid_bytes(p);
    if (steps == 0) {
        hipError_t e = hipMemcpyAsync(out, in, bytes, hipMemcpyDeviceToDevice, stream);
        if (e != hipSuccess) return fail(STENCIL_ERR_HIP, std::string("hipMemcpyAsync: ") + hipGetErrorString(e));
        return STENCIL_OK;
    }
    std::vector<PassDesc> passes = schedule(p, steps);
    const int P = (int)passes.size();
    const void *src = in;
    for (int i = 0; i < P; ++i) {
        void *dst = ((P - 1 - i) % 2 == 0) ? out : scratch;
        const PassDesc &pd = passes[i];
        if (!pd.k) return fail(STENCIL_ERR_UNSUPPORTED, "no kernel for a pass");
        PassArgs a = base_args(p, pd.t);
        a.src = src;
        a.dst = dst;
        if (is_mfma_path(pd.path)) {
            a.afrag = p->afrag[pd.t];
            a.afrag_lo = p->afrag_lo[pd.t];
        }
        hipError_t e = pd.k->launch(a, stream);
        if (e == hipSuccess && pd.fixup) e = launch_fixup(p, pd.t, src, dst, stream);
        if (e != hipSuccess) return fail(STENCIL_ERR_HIP, std::string("kernel launch: ") + hipGetErrorString(e));
        src = dst;
    }
    return STENCIL_OK;
}

// Batched runs: round j issues pass j of every job that has one.  Passes of
// one round that share a kernel variant go out as one persistent batched
// launch (workgroups pull tiles of all those grids from one list); variants
// without a batched form go out one by one, and the Dirichlet band fix-ups
// of kernel-fused MFMA passes follow the round's launches.  Each job's
// passes stay in stream order and ping-pong exactly as in run_one, so every
// result is bit-identical to running the job alone.
std::mutex g_batch_mu;

int run_batch(int n, const stencil_plan_t *plans, const void *const *ins, void *const *outs,
              const int64_t *steps, hipStream_t stream)
{
    std::lock_guard<std::mutex> lock(g_batch_mu);
    static std::map<int, BatchStaging> stages;
    int dev = 0;
    (void)hipGetDevice(&dev);
    BatchStaging &stage = stages[dev];
    hipError_t e = stage.begin(stream);
    if (e != hipSuccess) return fail(STENCIL_ERR_HIP, std::string("batch staging: ") + hipGetErrorString(e));
    // the slot is marked busy until the stream passes this point, also when a
    // launch below fails after earlier ones were queued
    struct SlotRelease {
        BatchStaging &s;
        hipStream_t st;
        ~SlotRelease() { (void)s.end(st); }
    } release{stage, stream};

    std::vector<std::vector<PassDesc>> sched((size_t)n);
    size_t rounds = 0;
    for (int i = 0; i < n; ++i) {
        if (steps[i] == 0) {
            e = hipMemcpyAsync(outs[i], ins[i], grid_bytes(plans[i]), hipMemcpyDeviceToDevice, stream);
            if (e != hipSuccess) return fail(STENCIL_ERR_HIP, std::string("hipMemcpyAsync: ") + hipGetErrorString(e));
            continue;
        }
        sched[i] = schedule(plans[i], steps[i]);
        rounds = std::max(rounds, sched[i].size());
    }
    std::vector<const void *> src(ins, ins + n);
    struct Fixup {
        stencil_plan_s *p;
        int t;
        const void *src;
        void *dst;
    };
    for (size_t j = 0; j < rounds; ++j) {
        std::map<const KernelEntry *, std::vector<PassArgs>> groups;
        std::vector<Fixup> fixups;  // Dirichlet bands, after the passes they correct
        for (int i = 0; i < n; ++i) {
            const auto &ps = sched[i];
            if (j >= ps.size()) continue;
            stencil_plan_s *p = plans[i];
            const int P = (int)ps.size();
            void *dst = ((P - 1 - (int)j) % 2 == 0) ? outs[i] : p->scratch;
            const PassDesc &pd = ps[j];
            if (!pd.k) return fail(STENCIL_ERR_UNSUPPORTED, "no kernel for a pass");
            PassArgs a = base_args(p, pd.t);
            a.src = src[i];
            a.dst = dst;
            src[i] = dst;
            if (is_mfma_path(pd.path)) {
                a.afrag = p->afrag[pd.t];
                a.afrag_lo = p->afrag_lo[pd.t];
            }
            if (pd.fixup) fixups.push_back({p, pd.t, a.src, dst});
            if (pd.k->launch_batch) {
                groups[pd.k].push_back(a);
                continue;
            }
            e = pd.k->launch(a, stream);
            if (e != hipSuccess) return fail(STENCIL_ERR_HIP, std::string("kernel launch: ") + hipGetErrorString(e));
        }
        for (auto &g : groups) {
            const KernelEntry *k = g.first;
            auto &v = g.second;
            e = v.size() == 1 ? k->launch(v[0], stream)
                              : k->launch_batch(v.data(), (int)v.size(), &stage, stream);
            if (e != hipSuccess) return fail(STENCIL_ERR_HIP, std::string("batched launch: ") + hipGetErrorString(e));
        }
        for (const Fixup &f : fixups) {
            e = launch_fixup(f.p, f.t, f.src, f.dst, stream);
            if (e != hipSuccess) return fail(STENCIL_ERR_HIP, std::string("kernel launch: ") + hipGetErrorString(e));
        }
    }
    return STENCIL_OK;
}

bool overlap(const void *a, const void *b, size_t n)
{
    const uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
    return x < y + n && y < x + n;
}

}  // namespace

namespace stl {

int run_without_allocation(stencil_plan_s *p, const void *in, void *out, int64_t steps,
                           hipStream_t stream, void *scratch, size_t scratch_cap)
{
    if (!p || !in || !out) return fail(STENCIL_ERR_INVALID_ARG, "stencil_run_noalloc: NULL plan or buffer");
    if (steps < 0) return fail(STENCIL_ERR_INVALID_ARG, "stencil_run_noalloc: steps < 0");
    const size_t bytes = grid_bytes(p);
    if (overlap(in, out, bytes)) return fail(STENCIL_ERR_ALIAS, "stencil_run_noalloc: in and out overlap");
    const bool multi = steps > 0 && schedule(p, steps).size() > 1;
    if (multi && bytes > scratch_cap)
        return fail(STENCIL_ERR_INVALID_ARG,
                    "stencil_run_noalloc: the grid (" + std::to_string(bytes) +
                        " bytes) exceeds the static scratch of " + std::to_string(scratch_cap) +
                        " bytes that a run of two or more passes needs");
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(STENCIL_ERR_HIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
    if (p->device != dev) {
        // only the MFMA operand fragments would need device memory
        if (is_mfma_path(p->path))
            return fail(STENCIL_ERR_UNSUPPORTED,
                        "stencil_run_noalloc: this MFMA plan has no operand fragments on the current "
                        "device; run it once with stencil_run there first (that call uploads them)");
        p->device = dev;
    }
    return run_one(p, in, out, steps, stream, scratch);
}

}  // namespace stl

extern "C" const char *stencil_last_error(void) { return g_last_error.c_str(); }

extern "C" int stencil_kernel_available(int path, int dtype, int shape, int d, int r, int T)
{
    if ((path != STENCIL_PATH_VALU && !is_mfma_path(path)) || !valid_dtype(dtype) ||
        (shape != STENCIL_STAR && shape != STENCIL_BOX) || (d != 2 && d != 3) || r < 1 || T < 1)
        return 0;
    return find_kernel(path, dtype, shape, d, r, T) != nullptr ? 1 : 0;
}

extern "C" int stencil_compose(int shape, int d, int r, const double *weights, int T, double *out,
                               int *k_t)
{
    if ((shape != STENCIL_STAR && shape != STENCIL_BOX) || (d != 2 && d != 3) || r < 1 || T < 1 ||
        !weights || !out)
        return fail(STENCIL_ERR_INVALID_ARG, "stencil_compose: invalid arguments");
    std::vector<double> wc;
    compose_dense(shape, d, r, weights, T, &wc);
    std::memcpy(out, wc.data(), wc.size() * sizeof(double));
    if (k_t) {
        // support of the composite for generic weights: compose a positive pattern
        std::vector<int> offs;
        const int K = pattern_offsets(shape, d, r, &offs);
        std::vector<double> ones((size_t)K, 1.0), sup;
        compose_dense(shape, d, r, ones.data(), T, &sup);
        int n = 0;
        for (double v : sup) n += v != 0.0;
        *k_t = n;
    }
    return STENCIL_OK;
}

extern "C" int stencil_plan(stencil_plan_t *plan, int shape, int d, int r, const double *weights,
                            const int64_t *dims, int T, int dtype, int boundary)
{
    if (!plan) return fail(STENCIL_ERR_INVALID_ARG, "stencil_plan: plan is NULL");
    *plan = nullptr;
    if (shape != STENCIL_STAR && shape != STENCIL_BOX)
        return fail(STENCIL_ERR_INVALID_ARG, "stencil_plan: shape must be STAR or BOX");
    if (d != 2 && d != 3) return fail(STENCIL_ERR_INVALID_ARG, "stencil_plan: d must be 2 or 3");
    if (r < 1) return fail(STENCIL_ERR_INVALID_ARG, "stencil_plan: r must be >= 1");
    if (T < 1) return fail(STENCIL_ERR_INVALID_ARG, "stencil_plan: T must be >= 1");
    if (!valid_dtype(dtype)) return fail(STENCIL_ERR_INVALID_ARG, "stencil_plan: unknown dtype");
    if (boundary != STENCIL_DIRICHLET && boundary != STENCIL_PERIODIC)
        return fail(STENCIL_ERR_INVALID_ARG, "stencil_plan: unknown boundary");
    if (!weights || !dims) return fail(STENCIL_ERR_INVALID_ARG, "stencil_plan: NULL weights or dims");
    std::vector<int> offs;
    const int K = pattern_offsets(shape, d, r, &offs);
    if (K > kMaxK) return fail(STENCIL_ERR_UNSUPPORTED, "stencil_plan: pattern too large");
    for (int k = 0; k < K; ++k)
        if (!std::isfinite(weights[k])) return fail(STENCIL_ERR_INVALID_ARG, "stencil_plan: non-finite weight");
    int64_t npts = 1;
    for (int i = 0; i < d; ++i) {
        if (dims[i] < 1) return fail(STENCIL_ERR_INVALID_ARG, "stencil_plan: dims must be >= 1");
        if (dims[i] > (int64_t)1 << 30) return fail(STENCIL_ERR_UNSUPPORTED, "stencil_plan: dim too large");
        npts *= dims[i];
    }
    if (npts > ((int64_t)1 << 40)) return fail(STENCIL_ERR_UNSUPPORTED, "stencil_plan: grid too large");

    stencil_plan_s *p = new (std::nothrow) stencil_plan_s();
    if (!p) return fail(STENCIL_ERR_OOM, "stencil_plan: host allocation");
    p->shape = shape;
    p->d = d;
    p->r = r;
    p->T = T;
    p->dtype = dtype;
    p->boundary = boundary;
    p->path_req = STENCIL_PATH_AUTO;
    for (int i = 0; i < kMaxD; ++i) p->dims[i] = i < d ? dims[i] : 1;
    p->npts = npts;
    p->K = K;
    p->offs = std::move(offs);
    p->w.assign(weights, weights + K);
    p->halo = 0.0;
    p->tile_rows = 0;
    p->device = -1;
    p->scratch = nullptr;
    p->scratch_bytes = 0;
    p->afrag_bytes = 0;
    plan_model(p);
    int rc = resolve_path(p);
    if (rc) {
        delete p;
        return rc;
    }
    p->afrag_bytes = fragment_bytes(p);
    *plan = p;
    return STENCIL_OK;
}

extern "C" int stencil_plan_set(stencil_plan_t p, int option, double value)
{
    if (!p) return fail(STENCIL_ERR_INVALID_ARG, "stencil_plan_set: plan is NULL");
    if (!std::isfinite(value)) return fail(STENCIL_ERR_INVALID_ARG, "stencil_plan_set: non-finite value");
    switch (option) {
    case STENCIL_OPT_HALO_VALUE:
        p->halo = value;
        return STENCIL_OK;
    case STENCIL_OPT_TILE_ROWS:
        if (value < 0 || value > 65536) return fail(STENCIL_ERR_INVALID_ARG, "tile rows out of range");
        p->tile_rows = (int)value;
        return STENCIL_OK;
    case STENCIL_OPT_PATH:
    case STENCIL_OPT_T: {
        const int v = (int)value;
        if ((double)v != value) return fail(STENCIL_ERR_INVALID_ARG, "integer option expected");
        const int old_req = p->path_req, old_path = p->path, old_T = p->T;
        if (option == STENCIL_OPT_PATH) {
            if (v < STENCIL_PATH_AUTO || v > STENCIL_PATH_MFMA_SEQ)
                return fail(STENCIL_ERR_INVALID_ARG, "unknown path");
            p->path_req = v;
        } else {
            if (v < 1) return fail(STENCIL_ERR_INVALID_ARG, "T must be >= 1");
            p->T = v;
        }
        plan_model(p);
        int rc = resolve_path(p);
        if (rc) {
            p->path_req = old_req;
            p->path = old_path;
            p->T = old_T;
            plan_model(p, p->path == STENCIL_PATH_MFMA_SPARSE);
            return rc;
        }
        // model results of the resolved path (the sparse path's peak and layout)
        plan_model(p, p->path == STENCIL_PATH_MFMA_SPARSE);
        free_device(p);
        p->afrag_bytes = fragment_bytes(p);
        return STENCIL_OK;
    }
    default:
        return fail(STENCIL_ERR_INVALID_ARG, "stencil_plan_set: unknown option");
    }
}

extern "C" int stencil_plan_info(stencil_plan_t p, stencil_plan_info_t *out)
{
    if (!p || !out) return fail(STENCIL_ERR_INVALID_ARG, "stencil_plan_info: NULL argument");
    stencil_plan_info_t i;
    std::memset(&i, 0, sizeof i);
    i.shape = p->shape;
    i.d = p->d;
    i.r = p->r;
    i.T = p->T;
    i.dtype = p->dtype;
    i.boundary = p->boundary;
    i.path = p->path;
    for (int k = 0; k < kMaxD; ++k) i.dims[k] = p->dims[k];
    i.K = p->K;
    i.K_T = p->K_T;
    i.alpha = p->alpha;
    i.S = p->S;
    i.gamma = p->gamma;
    i.halo = p->halo;
    i.workspace_bytes = (int64_t)(grid_bytes(p) + p->afrag_bytes);
    i.predicted_gst_valu = p->pred_valu;
    i.predicted_gst_mfma = p->pred_mfma;
    i.predicted_winner = p->pred_winner;
    i.scenario = p->scenario;
    i.tile_rows = p->tile_rows;
    const bool fused = find_kernel(p->path, p->dtype, p->shape, p->d, p->r, p->T) != nullptr ||
                       (is_mfma_path(p->path) &&
                        find_kernel(STENCIL_PATH_VALU, p->dtype, p->shape, p->d, p->r, p->T) != nullptr);
    i.T_fused = fused ? p->T : 1;
    *out = i;
    return STENCIL_OK;
}

extern "C" int stencil_run(stencil_plan_t p, const void *in, void *out, int64_t steps, void *stream)
{
    if (!p || !in || !out) return fail(STENCIL_ERR_INVALID_ARG, "stencil_run: NULL plan or buffer");
    if (steps < 0) return fail(STENCIL_ERR_INVALID_ARG, "stencil_run: steps < 0");
    if (overlap(in, out, grid_bytes(p))) return fail(STENCIL_ERR_ALIAS, "stencil_run: in and out overlap");
    int rc = ensure_device(p, steps > 0 && schedule(p, steps).size() > 1);
    if (rc) return rc;
    return run_one(p, in, out, steps, (hipStream_t)stream, p->scratch);
}

extern "C" int stencil_run_batch(int n, const stencil_plan_t *plans, const void *const *ins,
                                 void *const *outs, const int64_t *steps, void *stream)
{
    if (n < 0) return fail(STENCIL_ERR_INVALID_ARG, "stencil_run_batch: n < 0");
    if (n == 0) return STENCIL_OK;
    if (!plans || !ins || !outs || !steps) return fail(STENCIL_ERR_INVALID_ARG, "stencil_run_batch: NULL array");
    for (int i = 0; i < n; ++i) {
        if (!plans[i] || !ins[i] || !outs[i]) return fail(STENCIL_ERR_INVALID_ARG, "stencil_run_batch: NULL entry");
        if (steps[i] < 0) return fail(STENCIL_ERR_INVALID_ARG, "stencil_run_batch: steps < 0");
        if (overlap(ins[i], outs[i], grid_bytes(plans[i])))
            return fail(STENCIL_ERR_ALIAS, "stencil_run_batch: in and out overlap");
        for (int j = 0; j < i; ++j)
            if (plans[j] == plans[i]) return fail(STENCIL_ERR_INVALID_ARG, "stencil_run_batch: repeated plan");
    }
    for (int i = 0; i < n; ++i) {
        int rc = ensure_device(plans[i], schedule(plans[i], steps[i]).size() > 1);
        if (rc) return rc;
    }
    return run_batch(n, plans, ins, outs, steps, (hipStream_t)stream);
}

extern "C" void stencil_plan_destroy(stencil_plan_t p)
{
    if (!p) return;
    free_device(p);
    delete p;
}
