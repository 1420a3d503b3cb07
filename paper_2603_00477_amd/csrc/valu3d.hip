// VALU path, d = 3, one explicit step per pass, streaming along z (the
// slowest axis).  Passes of T >= 2 fused steps run on the kernel of
// valu3d_fused.hip; the step pipeline below is written for any T, but the
// tile geometry (no skirt, halo staged per thread) is the one-step one.
//
// A workgroup of TX x TY threads owns an in-plane tile of (TY*WY) x (TX*W)
// points (each thread WY rows x W consecutive columns) and streams down a
// segment of planes.  Each thread stages its own points of a plane and a
// share of the plane's R-point halo around the tile (prefetched U planes
// ahead), so every computed point is an output.
// Stage 0 writes input plane k to an LDS plane buffer; stage 1 reads the plane
// written one iteration earlier, scatters it into 2R+1 rotating accumulator
// planes (input plane z adds its in-plane neighbourhood weighted by w[c][.][.]
// to output plane z-c) and emits the completed plane.  One barrier per plane.
//
// Weights: a set of up to 48 dwords lives in scalar registers, up to 64
// dwords is pinned in vector registers.  Boxes with r >= 2 (125 or 343
// weights) run on the one-step kernel of valu3d_box.hip.

#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include "internal.h"
#include "valu_common.h"

namespace stl {
namespace {

template <typename TC, int K>
struct Valu3DArgs {
    const void *src;
    void *dst;
    int n0, n1, n2;
    int oz0, oz1, oy0, oy1, ox0, ox1;
    int BZ, BYv, BXv, nty, ntx, nzs, ntiles;
    int periodic;
    TC h;
    TC w[K];
};

template <typename TS, typename TC, int SHAPE, int R, int T, int W, int WY, int TX, int TY>
struct Valu3DCfg {
    static constexpr int K = SHAPE == STENCIL_BOX ? (2 * R + 1) * (2 * R + 1) * (2 * R + 1) : 6 * R + 1;
    static constexpr int NT = TX * TY;
    static constexpr int PY = TY * WY;                      // extended rows
    static constexpr int PX = TX * W;                       // extended columns
    // The tile stages the input plane's R-point halo (no skirt): staging a
    // halo instead of computing a skirt measured +25-31 % at 512^3.
    static_assert(T == 1, "fused passes run on the fused 3D kernel");
    static constexpr bool HALO = true;
    static constexpr int EY = 0;                            // row skirt
    static constexpr int EX = 0;                            // column skirt
    static constexpr int PADX = ((R + W - 1) / W) * W;      // LDS column pad
    static constexpr int LDX = PX + 2 * PADX;               // LDS row pitch
    static constexpr int LROWS = PY + 2 * R;                // LDS rows (R pad each side)
    static constexpr int PLANE = LROWS * LDX;
    static constexpr int Q = 2 * R + 1;
    static constexpr int U = Q;                             // planes prefetched ahead
    // halo points of a staged plane: rows [-R, PY+R) x columns [-R, PX+R)
    // outside the PY x PX extended tile, NH per thread
    static constexpr int HROW = PX + 2 * R;
    static constexpr int NHALO = 2 * R * HROW + 2 * R * PY;
    static constexpr int NH = HALO ? (NHALO + NT - 1) / NT : 1;
    // 0: scalar registers; 1: pinned vector registers.  Float32 FMAs run ~35 %
    // slower with a scalar-register operand on gfx950, so float32 sets go to
    // vector registers for r <= 2 (+8-13 % measured); at r = 3 the extra
    // registers cost more occupancy than they gain (-17 %), so they stay scalar
    static constexpr int WMODE = (sizeof(TC) * K <= 192 && (sizeof(TC) == 8 || R >= 3)) ? 0 : 1;
    static_assert(sizeof(TC) * K <= 256, "large boxes run on the one-step box kernel");
};

template <int R>
__device__ __forceinline__ int star3_index(int axis, int off)
{
    return 1 + axis * 2 * R + (off < 0 ? off + R : off + R - 1);
}

// One tile (in-plane tile x plane segment) of one pass, run by the whole
// workgroup; `lds` holds T double-buffered planes.
template <typename TS, typename TC, int SHAPE, int R, int T, int W, int WY, int TX, int TY>
__device__ __forceinline__ void valu3d_tile(
    const Valu3DArgs<TC, Valu3DCfg<TS, TC, SHAPE, R, T, W, WY, TX, TY>::K> &a, const int tile,
    TC (&lds)[T][2][Valu3DCfg<TS, TC, SHAPE, R, T, W, WY, TX, TY>::PLANE])
{
    using Cfg = Valu3DCfg<TS, TC, SHAPE, R, T, W, WY, TX, TY>;
    constexpr int K = Cfg::K;
    constexpr int Q = Cfg::Q;
    constexpr int U = Cfg::U;
    constexpr int NT = Cfg::NT;
    constexpr int LDX = Cfg::LDX;
    constexpr int PLANE = Cfg::PLANE;
    constexpr int PADX = Cfg::PADX;
    constexpr int WMODE = Cfg::WMODE;
    using Vec = RawVec<TS, W>;

    const int tid = threadIdx.x;
    const int tx = tid % TX, ty = tid / TX;
    const int tzs = tile / (a.nty * a.ntx);
    const int rem = tile - tzs * (a.nty * a.ntx);
    const int tyi = rem / a.ntx, txi = rem - tyi * a.ntx;
    const int z0 = a.oz0 + tzs * a.BZ;
    const int z1 = min(z0 + a.BZ, a.oz1);
    const int BZe = z1 - z0;
    const int y0 = a.oy0 + tyi * a.BYv;
    const int ye = min(y0 + a.BYv, a.oy1);
    const int x0 = a.ox0 + txi * a.BXv;
    const int xe = min(x0 + a.BXv, a.ox1);
    const int cy0 = y0 - Cfg::EY + ty * WY;  // first row of this thread
    const int cx0 = x0 - Cfg::EX + tx * W;   // first column of this thread

    const TS *src = static_cast<const TS *>(a.src);
    TS *dst = static_cast<TS *>(a.dst);
    const int n0 = a.n0, n1 = a.n1, n2 = a.n2;
    const bool periodic = a.periodic != 0;
    const TC h = a.h;
    const TS hs = to_storage<TS>(h);

    for (int i = tid; i < T * 2 * PLANE; i += NT) (&lds[0][0][0])[i] = TC(0);

    TC wk[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        wk[k] = a.w[k];
        if constexpr (WMODE == 1) asm volatile("" : "+v"(wk[k]));
    }
    auto weight = [&](int k) -> TC { return wk[k]; };

    bool col_in[W], col_store[W];
    int col_src[W];
#pragma unroll
    for (int j = 0; j < W; ++j) {
        const int c = cx0 + j;
        col_in[j] = c >= 0 && c < n2;
        col_src[j] = periodic ? wrap(c, n2) : c;
        col_store[j] = c >= x0 && c < xe;
    }
    bool row_in[WY], row_store[WY];
    int row_src[WY];
#pragma unroll
    for (int i = 0; i < WY; ++i) {
        const int r = cy0 + i;
        row_in[i] = r >= 0 && r < n1;
        row_src[i] = periodic ? wrap(r, n1) : r;
        row_store[i] = r >= y0 && r < ye;
    }
    const bool vec_ok = vec_aligned<TS, W>(src, n2, cx0) && cx0 >= 0 && cx0 + W <= n2;

    const int KTOT = BZe + 2 * R * T + T;
    const int zbase = z0 - R * T;

    TC acc[T][Q][WY][W];
#pragma unroll
    for (int s = 0; s < T; ++s)
#pragma unroll
        for (int q = 0; q < Q; ++q)
#pragma unroll
            for (int i = 0; i < WY; ++i)
#pragma unroll
                for (int j = 0; j < W; ++j) acc[s][q][i][j] = TC(0);

    auto load_plane = [&](int k, Vec *v) {
        const int z = zbase + k;
        const bool zin = z >= 0 && z < n0;
        if (!periodic && !zin) {
#pragma unroll
            for (int i = 0; i < WY; ++i)
#pragma unroll
                for (int j = 0; j < W; ++j) v[i].e[j] = hs;
            return;
        }
        const TS *pl = src + (int64_t)(periodic ? wrap(z, n0) : z) * n1 * n2;
#pragma unroll
        for (int i = 0; i < WY; ++i) {
            if (!periodic && !row_in[i]) {
#pragma unroll
                for (int j = 0; j < W; ++j) v[i].e[j] = hs;
                continue;
            }
            const TS *rowp = pl + (int64_t)row_src[i] * n2;
            if (vec_ok) {
                v[i].load(rowp + cx0);
            } else {
#pragma unroll
                for (int j = 0; j < W; ++j)
                    v[i].e[j] = (periodic || col_in[j]) ? rowp[col_src[j]] : hs;
            }
        }
    };

    Vec ring[U][WY];
#pragma unroll
    for (int u = 0; u < U; ++u)
        if (u < KTOT) load_plane(u, ring[u]);

    // this thread's halo points: LDS offset in a plane (-1: none), source
    // offset in a plane (-1: outside a Dirichlet grid, value h)
    constexpr int NH = Cfg::NH, HROW = Cfg::HROW;
    int h_lds[NH];
    int64_t h_src[NH];
#pragma unroll
    for (int i = 0; i < NH; ++i) {
        h_lds[i] = -1;
        h_src[i] = -1;
        if constexpr (!Cfg::HALO) continue;
        const int e = tid + i * NT;
        int lr = 0, lc = 0;
        if (e < R * HROW) {
            lr = -R + e / HROW;
            lc = -R + e % HROW;
        } else if (e < 2 * R * HROW) {
            lr = Cfg::PY + (e - R * HROW) / HROW;
            lc = -R + (e - R * HROW) % HROW;
        } else {
            const int e3 = e - 2 * R * HROW, m = e3 % (2 * R);
            lr = e3 / (2 * R);
            lc = m < R ? -R + m : Cfg::PX + m - R;
        }
        h_lds[i] = e < Cfg::NHALO ? (R + lr) * LDX + PADX + lc : -1;
        const int gr = y0 - Cfg::EY + lr, gc = x0 - Cfg::EX + lc;
        const bool in = gr >= 0 && gr < n1 && gc >= 0 && gc < n2;
        h_src[i] = periodic ? (int64_t)wrap(gr, n1) * n2 + wrap(gc, n2) : (in ? (int64_t)gr * n2 + gc : -1);
    }
    // halo values of plane k (issued U planes ahead of their use)
    auto load_halo = [&](int k, TS (&hv)[NH]) {
        if constexpr (!Cfg::HALO) return;
        const int z = zbase + k;
        const bool zin = z >= 0 && z < n0;
        const TS *pl = src + (int64_t)(periodic ? wrap(z, n0) : (zin ? z : 0)) * n1 * n2;
#pragma unroll
        for (int i = 0; i < NH; ++i)
            hv[i] = (h_lds[i] >= 0 && h_src[i] >= 0 && (periodic || zin)) ? pl[h_src[i]] : hs;
    };
    TS hring[U][NH];
#pragma unroll
    for (int u = 0; u < U; ++u)
        if (u < KTOT) load_halo(u, hring[u]);
    __syncthreads();

    // LDS position of this thread's first point inside a plane buffer
    const int lpos = (R + ty * WY) * LDX + PADX + tx * W;

    for (int kb = 0; kb < KTOT; kb += U) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int k = kb + u;
            if (k >= KTOT) break;
            const int par = k & 1;
            {
                TC *w0 = &lds[0][par][lpos];
#pragma unroll
                for (int i = 0; i < WY; ++i)
#pragma unroll
                    for (int j = 0; j < W; ++j) w0[i * LDX + j] = to_compute<TC>(ring[u][i].e[j]);
                if constexpr (Cfg::HALO) {
                    TC *h0 = &lds[0][par][0];
#pragma unroll
                    for (int i = 0; i < NH; ++i)
                        if (h_lds[i] >= 0) h0[h_lds[i]] = to_compute<TC>(hring[u][i]);
                    if (k + U < KTOT) load_halo(k + U, hring[u]);
                }
                if (k + U < KTOT) load_plane(k + U, ring[u]);
            }
#pragma unroll
            for (int s = 1; s <= T; ++s) {
                const bool active = k >= s + 2 * R * (s - 1) && k < BZe + 2 * R * T + s;
                const int qc = u % Q;
                if (active) {
                    const TC *rb = &lds[s - 1][par ^ 1][lpos - R * LDX - R];
                    // stream the (WY+2R) x (W+2R) neighbourhood one LDS row at a time
#pragma unroll
                    for (int wi = 0; wi < WY + 2 * R; ++wi) {
                        const bool mid = wi >= R && wi < R + WY;  // row holds an output row
                        TC row[W + 2 * R];
#pragma unroll
                        for (int j = 0; j < W + 2 * R; ++j) {
                            const bool need = SHAPE == STENCIL_BOX || mid || (j >= R && j < R + W);
                            row[j] = need ? rb[wi * LDX + j] : TC(0);
                        }
#pragma unroll
                        for (int c = -R; c <= R; ++c) {
                            const int q = ((u - c + R) % Q + Q) % Q;
#pragma unroll
                            for (int i = 0; i < WY; ++i) {
                                const int ao = wi - i - R;
                                if (ao < -R || ao > R) continue;
                                if constexpr (SHAPE == STENCIL_BOX) {
#pragma unroll
                                    for (int bo = -R; bo <= R; ++bo) {
                                        const TC wv = weight(((c + R) * (2 * R + 1) + (ao + R)) * (2 * R + 1) + (bo + R));
#pragma unroll
                                        for (int j = 0; j < W; ++j)
                                            acc[s - 1][q][i][j] = fma_c(wv, row[j + bo + R], acc[s - 1][q][i][j]);
                                    }
                                } else {
                                    if (c != 0) {
                                        if (ao != 0) continue;  // z arm: centre column only
                                        const TC wv = weight(star3_index<R>(0, c));
#pragma unroll
                                        for (int j = 0; j < W; ++j)
                                            acc[s - 1][q][i][j] = fma_c(wv, row[j + R], acc[s - 1][q][i][j]);
                                    } else if (ao != 0) {  // y arm
                                        const TC wv = weight(star3_index<R>(1, ao));
#pragma unroll
                                        for (int j = 0; j < W; ++j)
                                            acc[s - 1][q][i][j] = fma_c(wv, row[j + R], acc[s - 1][q][i][j]);
                                    } else {  // x arm with the centre
#pragma unroll
                                        for (int bo = -R; bo <= R; ++bo) {
                                            const TC wv = bo == 0 ? weight(0) : weight(star3_index<R>(2, bo));
#pragma unroll
                                            for (int j = 0; j < W; ++j)
                                                acc[s - 1][q][i][j] = fma_c(wv, row[j + bo + R], acc[s - 1][q][i][j]);
                                        }
                                    }
                                }
                            }
                        }
                    }
                    const int zo = zbase + k - s * (1 + R);
                    if (s < T) {
                        TC *wr = &lds[s][par][lpos];
                        const bool zin = zo >= 0 && zo < n0;
#pragma unroll
                        for (int i = 0; i < WY; ++i)
#pragma unroll
                            for (int j = 0; j < W; ++j) {
                                TC v = acc[s - 1][qc][i][j];
                                if (!periodic && !(zin && row_in[i] && col_in[j])) v = h;
                                wr[i * LDX + j] = v;
                            }
                    } else if (zo >= z0 && zo < z1) {
                        TS *pl = dst + (int64_t)zo * n1 * n2;
#pragma unroll
                        for (int i = 0; i < WY; ++i) {
                            if (!row_store[i]) continue;
                            TS *rowp = pl + (int64_t)(cy0 + i) * n2;
                            Vec ov;
                            bool all = vec_ok;
#pragma unroll
                            for (int j = 0; j < W; ++j) {
                                ov.e[j] = to_storage<TS>(acc[s - 1][qc][i][j]);
                                all = all && col_store[j];
                            }
                            if (all) {
                                ov.store(rowp + cx0);
                            } else {
#pragma unroll
                                for (int j = 0; j < W; ++j)
                                    if (col_store[j]) rowp[cx0 + j] = ov.e[j];
                            }
                        }
                    }
                }
#pragma unroll
                for (int i = 0; i < WY; ++i)
#pragma unroll
                    for (int j = 0; j < W; ++j) acc[s - 1][qc][i][j] = TC(0);
            }
            __syncthreads();
        }
    }
}

template <typename TS, typename TC, int SHAPE, int R, int T, int W, int WY, int TX, int TY>
__global__ __launch_bounds__(TX *TY) void valu3d_kernel(
    Valu3DArgs<TC, Valu3DCfg<TS, TC, SHAPE, R, T, W, WY, TX, TY>::K> a)
{
    using Cfg = Valu3DCfg<TS, TC, SHAPE, R, T, W, WY, TX, TY>;
    __shared__ TC lds[T][2][Cfg::PLANE];
    const int tile = xcd_remap(blockIdx.x, gridDim.x);
    if (tile >= a.ntiles) return;
    valu3d_tile<TS, TC, SHAPE, R, T, W, WY, TX, TY>(a, tile, lds);
}

// Persistent batched launch: the workgroups walk one list of tiles spanning
// every job of the batch; workgroup b takes items b + i*gridDim.  tile_start[j]
// is the first item of job j (tile_start[njobs] = total).  The tile body ends
// with a barrier, so the LDS planes are free when the next item starts.
template <typename TS, typename TC, int SHAPE, int R, int T, int W, int WY, int TX, int TY>
__global__ __launch_bounds__(TX *TY) void valu3d_batch_kernel(
    const Valu3DArgs<TC, Valu3DCfg<TS, TC, SHAPE, R, T, W, WY, TX, TY>::K> *__restrict__ jobs,
    const int *__restrict__ tile_start, int njobs)
{
    using Cfg = Valu3DCfg<TS, TC, SHAPE, R, T, W, WY, TX, TY>;
    __shared__ TC lds[T][2][Cfg::PLANE];
    const int total = tile_start[njobs];
    int j = 0;
    for (int item = xcd_remap(blockIdx.x, gridDim.x); item < total; item += gridDim.x) {
        while (j + 1 < njobs && tile_start[j + 1] <= item) ++j;
        const Valu3DArgs<TC, Cfg::K> a = jobs[j];
        valu3d_tile<TS, TC, SHAPE, R, T, W, WY, TX, TY>(a, item - tile_start[j], lds);
    }
}

// Fill the arguments of one pass; returns false when there is nothing to do
// (err then says whether the pass is invalid).
template <typename TS, typename TC, int SHAPE, int R, int T, int W, int WY, int TX, int TY>
bool valu3d_args(const PassArgs &p, Valu3DArgs<TC, Valu3DCfg<TS, TC, SHAPE, R, T, W, WY, TX, TY>::K> *out,
                 hipError_t *err)
{
    using Cfg = Valu3DCfg<TS, TC, SHAPE, R, T, W, WY, TX, TY>;
    *err = hipSuccess;
    Valu3DArgs<TC, Cfg::K> &a = *out;
    a.src = p.src;
    a.dst = p.dst;
    a.n0 = (int)p.dims[0];
    a.n1 = (int)p.dims[1];
    a.n2 = (int)p.dims[2];
    a.oz0 = p.region_lo[0];
    a.oz1 = p.region_hi[0];
    a.oy0 = p.region_lo[1];
    a.oy1 = p.region_hi[1];
    a.ox0 = p.region_lo[2];
    a.ox1 = p.region_hi[2];
    a.periodic = p.boundary == STENCIL_PERIODIC;
    a.h = (TC)p.halo;
    for (int k = 0; k < Cfg::K; ++k) a.w[k] = (TC)p.w[k];
    a.BYv = Cfg::PY - 2 * Cfg::EY;
    a.BXv = Cfg::PX - 2 * Cfg::EX;
    if (a.BYv <= 0 || a.BXv <= 0) {
        *err = hipErrorInvalidValue;
        return false;
    }
    const int D0 = a.oz1 - a.oz0, D1 = a.oy1 - a.oy0, D2 = a.ox1 - a.ox0;
    if (D0 <= 0 || D1 <= 0 || D2 <= 0) return false;
    a.nty = (D1 + a.BYv - 1) / a.BYv;
    a.ntx = (D2 + a.BXv - 1) / a.BXv;
    int BZ = p.tile_rows;
    if (BZ <= 0) {
        const int target = 8 * (p.num_cu > 0 ? p.num_cu : 256);
        const int inplane = a.nty * a.ntx;
        const int segs = (target + inplane - 1) / inplane;
        BZ = (D0 + segs - 1) / segs;
        const int minBZ = 8 * R * T > 32 ? 8 * R * T : 32;
        if (BZ < minBZ) BZ = minBZ;
    }
    a.BZ = BZ;
    a.nzs = (D0 + BZ - 1) / BZ;
    const int64_t nt = (int64_t)a.nzs * a.nty * a.ntx;
    if (nt > (1LL << 30)) {
        *err = hipErrorInvalidValue;
        return false;
    }
    a.ntiles = (int)nt;
    return true;
}

template <typename TS, typename TC, int SHAPE, int R, int T, int W, int WY, int TX, int TY>
hipError_t launch_valu3d_cfg(const PassArgs &p, hipStream_t stream)
{
    using Cfg = Valu3DCfg<TS, TC, SHAPE, R, T, W, WY, TX, TY>;
    Valu3DArgs<TC, Cfg::K> a;
    hipError_t err;
    if (!valu3d_args<TS, TC, SHAPE, R, T, W, WY, TX, TY>(p, &a, &err)) return err;
    hipLaunchKernelGGL((valu3d_kernel<TS, TC, SHAPE, R, T, W, WY, TX, TY>), dim3(a.ntiles),
                       dim3(TX * TY), 0, stream, a);
    return hipGetLastError();
}

// n passes (one per job) of this variant in one persistent launch.
template <typename TS, typename TC, int SHAPE, int R, int T, int W, int WY, int TX, int TY>
hipError_t launch_valu3d_batch_cfg(const PassArgs *ps, int n, BatchStaging *stage, hipStream_t stream)
{
    using Cfg = Valu3DCfg<TS, TC, SHAPE, R, T, W, WY, TX, TY>;
    using Args = Valu3DArgs<TC, Cfg::K>;
    std::vector<Args> jobs;
    std::vector<int> start(1, 0);
    jobs.reserve(n);
    for (int i = 0; i < n; ++i) {
        Args a;
        hipError_t err;
        if (!valu3d_args<TS, TC, SHAPE, R, T, W, WY, TX, TY>(ps[i], &a, &err)) {
            if (err != hipSuccess) return err;
            continue;
        }
        if ((int64_t)start.back() + a.ntiles > (1LL << 30)) return hipErrorInvalidValue;
        jobs.push_back(a);
        start.push_back(start.back() + a.ntiles);
    }
    if (jobs.empty()) return hipSuccess;
    void *djobs = nullptr, *dstart = nullptr;
    hipError_t e = stage_job_table(stage, jobs.data(), jobs.size() * sizeof(Args), start, &djobs, &dstart,
                                   stream);
    if (e != hipSuccess) return e;
    int occ = 0;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &occ, valu3d_batch_kernel<TS, TC, SHAPE, R, T, W, WY, TX, TY>, TX * TY, 0);
    if (e != hipSuccess || occ < 1) occ = 1;
    const int slots = occ * (ps[0].num_cu > 0 ? ps[0].num_cu : 256);
    const int total = start.back();
    hipLaunchKernelGGL((valu3d_batch_kernel<TS, TC, SHAPE, R, T, W, WY, TX, TY>),
                       dim3(total < slots ? total : slots), dim3(TX * TY), 0, stream,
                       static_cast<const Args *>(djobs), static_cast<const int *>(dstart), (int)jobs.size());
    return hipGetLastError();
}

// Tile shapes: float64 2 x 2 points per thread, float32 2 x 4.  r <= 2:
// 32 x 8 threads (wide rows: 64 float64 / 128 float32 columns per tile),
// measured 14-18 % faster than 16 x 16 on 512^3; r = 3 keeps 16 x 16
// (Star-3D3R float32: 371 vs 294 GSt/s).
template <typename TS, int R, int T>
struct Valu3DShape {
    static constexpr int W = sizeof(TS) == 8 ? 2 : (sizeof(TS) == 4 ? 4 : 8);
    static constexpr int WY = 2;
    static constexpr int TX = R <= 2 ? 32 : 16;
    static constexpr int TY = R <= 2 ? 8 : 16;
};

template <typename TS, typename TC, int SHAPE, int R, int T>
hipError_t launch_valu3d(const PassArgs &p, hipStream_t stream)
{
    using S = Valu3DShape<TS, R, T>;
    return launch_valu3d_cfg<TS, TC, SHAPE, R, T, S::W, S::WY, S::TX, S::TY>(p, stream);
}

template <typename TS, typename TC, int SHAPE, int R, int T>
hipError_t launch_valu3d_batch(const PassArgs *ps, int n, BatchStaging *stage, hipStream_t stream)
{
    using S = Valu3DShape<TS, R, T>;
    return launch_valu3d_batch_cfg<TS, TC, SHAPE, R, T, S::W, S::WY, S::TX, S::TY>(ps, n, stage, stream);
}

#define V3(TS, TC, DT, SH, R, T) \
    {STENCIL_PATH_VALU, DT, SH, 3, R, T, &launch_valu3d<TS, TC, SH, R, T>, &launch_valu3d_batch<TS, TC, SH, R, T>}
// One-step passes (T = 1) of every star radius up to 3 and of the 27-point
// box; fused passes (T >= 2) run on the kernel of valu3d_fused.hip.
#define V3_S(TS, TC, DT)                                                                       \
    V3(TS, TC, DT, STENCIL_STAR, 1, 1), V3(TS, TC, DT, STENCIL_STAR, 2, 1), V3(TS, TC, DT, STENCIL_STAR, 3, 1), \
        V3(TS, TC, DT, STENCIL_BOX, 1, 1)

}  // namespace

const std::vector<KernelEntry> &valu3d_kernels()
{
    static const std::vector<KernelEntry> table = {
        V3_S(double, double, STENCIL_F64),
        V3_S(float, float, STENCIL_F32),
    };
    return table;
}

}  // namespace stl
