// VALU path, d = 3, large boxes (r >= 2: 125 or 343 weights), one step per
// pass.  These patterns are compute-bound on MI355X already at T = 1
// (I = K/D >= 15.6 flop/byte in FP64 and >= 31 in FP32, above both ridges),
// so temporal fusion cannot raise their roofline and the kernel spends its
// registers on reuse instead (paper, Sec. "CUDA Core Implementation with
// Temporal Fusion": fusion only pays while the pass is memory-bound).
//
// A workgroup of TX x TY threads owns an output tile of (TY*WY) x (TX*W)
// points and streams down a segment of planes.  Each input plane, with its
// R-point halo, is staged once in LDS (double-buffered; the global loads for
// plane k+1 are in flight while plane k is computed).  Every thread reads its
// (WY+2R) x (W+2R) window row by row and scatters it into 2R+1 accumulator
// planes: input plane z adds w[c][.][.] * window to output plane z - c
// (input-stationary in z, so each input plane is read from LDS once).  After
// plane z the accumulator of output plane z - R is complete: it is stored and
// the accumulators rotate by one plane.
//
// The weights never occupy vector registers: each run of 2R+1 weights
// w[c][a][-R..R] (one "block") is fetched with scalar loads from the
// kernel-argument block just before its FMAs (v_fma takes it as the scalar
// operand).  The fetch of block n+1 is issued before the FMAs of block n
// (software pipelining).  Scalar loads complete out of order, so a wait for
// one waits for all; empty volatile asm statements, which keep their relative
// order, pin the waits: the fetch of block n+1 takes block n's first weight
// as an operand (it follows the wait for block n), and a statement consuming
// block n's results follows its FMAs, so the wait for block n+1 comes after
// them and at most two blocks of weights are live in scalar registers.
//
// Contributions to one output arrive in canonical order (c, then a, then b
// ascending), as in the oracle.

#include <cstddef>
#include <vector>

#include <hip/hip_runtime.h>

#include "internal.h"
#include "valu_common.h"

namespace stl {
namespace {

template <typename TC, int K>
struct Box3Args {
    const void *src;
    void *dst;
    int n0, n1, n2;
    int oz0, oz1, oy0, oy1, ox0, ox1;
    int BZ, nty, ntx, nzs, ntiles;
    int periodic;
    TC h;
    TC w[K];  // canonical order; read through the kernel-argument segment
};

template <typename TS, typename TC, int R, int W, int WY, int TX, int TY>
struct Box3Cfg {
    static constexpr int Q = 2 * R + 1;
    static constexpr int K = Q * Q * Q;
    static constexpr int NT = TX * TY;
    static constexpr int BY = TY * WY;                  // output rows per tile
    static constexpr int BX = TX * W;                   // output columns per tile
    static constexpr int LY = BY + 2 * R;               // staged rows
    static constexpr int LX = BX + 2 * R;               // staged columns
    static constexpr int VE = 16 / sizeof(TC);          // elements per 16-byte LDS read
    static constexpr int LDX = ((LX + VE - 1) / VE) * VE;
    static constexpr int PLANE = LY * LDX;
    static constexpr int NPF = (LY * LX + NT - 1) / NT;  // staged elements per thread
    static constexpr int WIN = W + 2 * R;                // window row length
    static constexpr int WINV = (WIN + VE - 1) / VE;     // 16-byte reads per window row
};

// Weights in the constant address space: loads through it are scalar.
template <typename TC>
using WPtr = const __attribute__((address_space(4))) TC *;

// One tile (in-plane tile x plane segment) of one pass, run by the whole
// workgroup; `wk` points to the K weights of the pass.
template <typename TS, typename TC, int R, int W, int WY, int TX, int TY>
__device__ __forceinline__ void box3_tile(const Box3Args<TC, Box3Cfg<TS, TC, R, W, WY, TX, TY>::K> &a,
                                          WPtr<TC> wk, const int tile,
                                          TC (&lds)[2][Box3Cfg<TS, TC, R, W, WY, TX, TY>::PLANE +
                                                       Box3Cfg<TS, TC, R, W, WY, TX, TY>::VE])
{
    using Cfg = Box3Cfg<TS, TC, R, W, WY, TX, TY>;
    constexpr int Q = Cfg::Q, NT = Cfg::NT, LX = Cfg::LX, LDX = Cfg::LDX, NPF = Cfg::NPF;
    constexpr int VE = Cfg::VE, WINV = Cfg::WINV;

    const int tid = threadIdx.x;
    const int tx = tid % TX, ty = tid / TX;
    const int tzs = tile / (a.nty * a.ntx);
    const int rem = tile - tzs * (a.nty * a.ntx);
    const int tyi = rem / a.ntx, txi = rem - tyi * a.ntx;
    const int z0 = a.oz0 + tzs * a.BZ;
    const int z1 = min(z0 + a.BZ, a.oz1);
    const int y0 = a.oy0 + tyi * Cfg::BY;
    const int x0 = a.ox0 + txi * Cfg::BX;
    const int n0 = a.n0, n1 = a.n1, n2 = a.n2;
    const bool periodic = a.periodic != 0;
    const TC h = a.h;
    // global address space: flat loads would also count against the scalar
    // weight fetches' wait counter
    using GPtr = const __attribute__((address_space(1))) TS *;
    const GPtr src = (GPtr)a.src;
    TS *dst = static_cast<TS *>(a.dst);

    // staging: element e = tid + p*NT of the LY x LX block.  Its in-plane
    // source offset (clamped to 0 where a Dirichlet grid has no point; bit p
    // of `valid` tells) and its LDS slot (a pad slot past the plane for the
    // elements beyond the block) are fixed for the tile, so the per-plane
    // loads and LDS writes run without branches.
    int pf_off[NPF], pf_lds[NPF];
    unsigned valid = 0;
#pragma unroll
    for (int p = 0; p < NPF; ++p) {
        const int e = tid + p * NT;
        const bool inblk = e < Cfg::LY * LX;
        const int ly = inblk ? e / LX : 0, lx = inblk ? e - ly * LX : 0;
        int gy = y0 - R + ly, gx = x0 - R + lx;
        bool in = inblk;
        if (periodic) {
            gy = wrap(gy, n1);
            gx = wrap(gx, n2);
        } else {
            in = in && gy >= 0 && gy < n1 && gx >= 0 && gx < n2;
        }
        pf_lds[p] = inblk ? ly * LDX + lx : Cfg::PLANE;
        pf_off[p] = in ? gy * n2 + gx : 0;
        valid |= (in ? 1u : 0u) << p;
    }
    TC pf[NPF];
    auto fetch = [&](int z) {
        const bool zin = periodic || (z >= 0 && z < n0);
        const GPtr pl = src + (int64_t)(periodic ? wrap(z, n0) : (zin ? z : 0)) * n1 * n2;
#pragma unroll
        for (int p = 0; p < NPF; ++p) {
            const TC v = to_compute<TC>(pl[pf_off[p]]);
            pf[p] = (zin && ((valid >> p) & 1u)) ? v : h;
        }
    };
    auto stage = [&](int buf) {
#pragma unroll
        for (int p = 0; p < NPF; ++p) lds[buf][pf_lds[p]] = pf[p];
    };

    TC acc[Q][WY][W];
#pragma unroll
    for (int m = 0; m < Q; ++m)
#pragma unroll
        for (int i = 0; i < WY; ++i)
#pragma unroll
            for (int j = 0; j < W; ++j) acc[m][i][j] = TC(0);

    const int zb = z0 - R;               // first input plane
    const int nk = (z1 - z0) + 2 * R;    // input planes of the segment
    fetch(zb);
    stage(0);
    __syncthreads();
    const int wpos = ty * WY * LDX + tx * W;  // window origin in a staged plane

    for (int k = 0; k < nk; ++k) {
        const int buf = k & 1;
        if (k + 1 < nk) fetch(zb + k + 1);
        auto load_row = [&](TC *row, int wi) {
            const TC *rp = &lds[buf][wpos + wi * LDX];
#pragma unroll
            for (int v = 0; v < WINV; ++v) {
                RawVec<TC, VE> t;
                t.load(rp + v * VE);
#pragma unroll
                for (int e = 0; e < VE; ++e) row[v * VE + e] = t.e[e];
            }
        };
        // blocks n = 0 .. Q*Q-1 in order (a = n / Q, c = n % Q - R): the
        // weights of block n+1 are fetched while block n runs
        // Scalar loads complete out of order, so any wait for one waits for all:
        // the fetch of block n+1 takes block n's first weight as an operand,
        // which puts it after the wait for block n's weights (and it then runs
        // under block n's FMAs).
        // The ordering dependency goes through the base pointer, so each
        // block's offset stays a compile-time immediate of its scalar loads
        // (an opaque offset cost scalar address arithmetic per block:
        // Box-3D2R 512^3 f32 / f64 250 -> 258, 155 -> 162 GSt/s without it).
        auto fetch_w = [&](int n, TC *wv, TC after) {
            const int wrow = ((n % Q) * Q + n / Q) * Q;  // canonical index of w[c][a][-R]
            WPtr<TC> p = wk;
            if constexpr (sizeof(TC) == 4 && R == 2) asm volatile("" : "+s"(p) : "v"(after));  // W(n)
            else asm volatile("" : "+s"(p) : "s"(after));
#pragma unroll
            for (int b = 0; b < Q; ++b) {
                wv[b] = p[wrow + b];
                // float32 r = 2: FMAs run faster on vector-register operands (one
                // move each, +15 %); r = 3 keeps them scalar (the moves' registers
                // cost a wave of occupancy, -9 %)
                if constexpr (sizeof(TC) == 4 && R == 2) asm volatile("" : "+v"(wv[b]));
            }
        };
        TC wcur[Q], wnxt[Q];
        fetch_w(0, wcur, TC(0));
        TC rr[WY][WINV * VE];  // window rows a .. a+WY-1 (row a+i serves output row i)
#pragma unroll
        for (int n = 0; n < Q * Q; ++n) {
            const int a = n / Q, c = n % Q - R;
            if (n == 0) {
#pragma unroll
                for (int i = 0; i < WY; ++i) load_row(rr[i], i);
            } else if (c == -R) {
#pragma unroll
                for (int i = 0; i + 1 < WY; ++i)
#pragma unroll
                    for (int e = 0; e < WINV * VE; ++e) rr[i][e] = rr[i + 1][e];
                load_row(rr[WY - 1], a + WY - 1);
            }
            if (n + 1 < Q * Q) fetch_w(n + 1, wnxt, wcur[0]);
            const int m = R - c;  // accumulator plane of output z - c
#pragma unroll
            for (int i = 0; i < WY; ++i)
#pragma unroll
                for (int b = 0; b < Q; ++b)
#pragma unroll
                    for (int j = 0; j < W; ++j) acc[m][i][j] = fma_c(wcur[b], rr[i][j + b], acc[m][i][j]);
            // E(n): block n's results exist before W(n+2), whose operand
            // needs block n+1's weights: the wait for them follows block n
#pragma unroll
            for (int i = 0; i < WY; ++i)
#pragma unroll
                for (int j = 0; j < W; ++j) asm volatile("" ::"v"(acc[m][i][j]));
#pragma unroll
            for (int b = 0; b < Q; ++b) wcur[b] = wnxt[b];
        }
        // accumulator plane 0 is output plane zb + k - R
        const int zo = zb + k - R;
        if (zo >= z0 && zo < z1) {
            TS *pl = dst + (int64_t)zo * n1 * n2;
#pragma unroll
            for (int i = 0; i < WY; ++i) {
                const int y = y0 + ty * WY + i;
                if (y >= a.oy1) continue;
                TS *rowp = pl + (int64_t)y * n2;
                const int xb = x0 + tx * W;
                RawVec<TS, W> ov;
#pragma unroll
                for (int j = 0; j < W; ++j) ov.e[j] = to_storage<TS>(acc[0][i][j]);
                if (xb + W <= a.ox1 && vec_aligned<TS, W>(dst, n2, xb)) {
                    ov.store(rowp + xb);
                } else {
#pragma unroll
                    for (int j = 0; j < W; ++j)
                        if (xb + j < a.ox1) rowp[xb + j] = ov.e[j];
                }
            }
        }
#pragma unroll
        for (int m = 0; m + 1 < Q; ++m)
#pragma unroll
            for (int i = 0; i < WY; ++i)
#pragma unroll
                for (int j = 0; j < W; ++j) acc[m][i][j] = acc[m + 1][i][j];
#pragma unroll
        for (int i = 0; i < WY; ++i)
#pragma unroll
            for (int j = 0; j < W; ++j) acc[Q - 1][i][j] = TC(0);
        if (k + 1 < nk) stage(buf ^ 1);
        __syncthreads();
    }
}

template <typename TS, typename TC, int R, int W, int WY, int TX, int TY>
__global__ __launch_bounds__(TX *TY) void valu3d_box_kernel(
    Box3Args<TC, Box3Cfg<TS, TC, R, W, WY, TX, TY>::K> a)
{
    using Cfg = Box3Cfg<TS, TC, R, W, WY, TX, TY>;
    using Args = Box3Args<TC, Cfg::K>;
    __shared__ __align__(16) TC lds[2][Cfg::PLANE + Cfg::VE];  // + VE: pad slot of the staging
    const int tile = xcd_remap(blockIdx.x, gridDim.x);
    if (tile >= a.ntiles) return;
    const WPtr<TC> wk = (WPtr<TC>)((const __attribute__((address_space(4))) char *)
                                       __builtin_amdgcn_kernarg_segment_ptr() +
                                   offsetof(Args, w));
    box3_tile<TS, TC, R, W, WY, TX, TY>(a, wk, tile, lds);
}

// Persistent batched launch over the tiles of several jobs (see the 3D
// kernel of valu3d.hip); each job's weights are scalar-loaded from the job
// table, which the kernel only reads.
template <typename TS, typename TC, int R, int W, int WY, int TX, int TY>
__global__ __launch_bounds__(TX *TY) void valu3d_box_batch_kernel(
    const Box3Args<TC, Box3Cfg<TS, TC, R, W, WY, TX, TY>::K> *__restrict__ jobs,
    const int *__restrict__ tile_start, int njobs)
{
    using Cfg = Box3Cfg<TS, TC, R, W, WY, TX, TY>;
    using Args = Box3Args<TC, Cfg::K>;
    __shared__ __align__(16) TC lds[2][Cfg::PLANE + Cfg::VE];
    const int total = tile_start[njobs];
    int j = 0;
    for (int item = xcd_remap(blockIdx.x, gridDim.x); item < total; item += gridDim.x) {
        while (j + 1 < njobs && tile_start[j + 1] <= item) ++j;
        const Args a = jobs[j];
        const WPtr<TC> wk = (WPtr<TC>)((const __attribute__((address_space(4))) char *)(jobs + j) +
                                       offsetof(Args, w));
        box3_tile<TS, TC, R, W, WY, TX, TY>(a, wk, item - tile_start[j], lds);
    }
}

template <typename TS, typename TC, int R, int W, int WY, int TX, int TY>
bool box3_args(const PassArgs &p, Box3Args<TC, Box3Cfg<TS, TC, R, W, WY, TX, TY>::K> *out, hipError_t *err)
{
    using Cfg = Box3Cfg<TS, TC, R, W, WY, TX, TY>;
    *err = hipSuccess;
    if (p.K != Cfg::K || p.steps != 1) {
        *err = hipErrorInvalidValue;
        return false;
    }
    Box3Args<TC, Cfg::K> &a = *out;
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
    const int D0 = a.oz1 - a.oz0, D1 = a.oy1 - a.oy0, D2 = a.ox1 - a.ox0;
    if (D0 <= 0 || D1 <= 0 || D2 <= 0) return false;
    if ((int64_t)a.n1 * a.n2 > (1LL << 31) - 1) {  // in-plane offsets are int
        *err = hipErrorInvalidValue;
        return false;
    }
    a.nty = (D1 + Cfg::BY - 1) / Cfg::BY;
    a.ntx = (D2 + Cfg::BX - 1) / Cfg::BX;
    int BZ = p.tile_rows;
    if (BZ <= 0) {
        // about one resident set of workgroups, segments no shorter than 4R
        // planes (the 2R halo planes of a segment cost (BZ + 2R) / BZ)
        const int target = 4 * (p.num_cu > 0 ? p.num_cu : 256);
        const int inplane = a.nty * a.ntx;
        const int segs = (target + inplane - 1) / inplane;
        BZ = (D0 + segs - 1) / segs;
        if (BZ < 4 * R) BZ = 4 * R;
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

template <typename TS, typename TC, int R, int W, int WY, int TX, int TY>
hipError_t launch_box3_cfg(const PassArgs &p, hipStream_t stream)
{
    using Cfg = Box3Cfg<TS, TC, R, W, WY, TX, TY>;
    static_assert(sizeof(Box3Args<TC, Cfg::K>) <= 4096, "weights exceed the kernel-argument block");
    Box3Args<TC, Cfg::K> a;
    hipError_t err;
    if (!box3_args<TS, TC, R, W, WY, TX, TY>(p, &a, &err)) return err;
    hipLaunchKernelGGL((valu3d_box_kernel<TS, TC, R, W, WY, TX, TY>), dim3(a.ntiles), dim3(TX * TY), 0,
                       stream, a);
    return hipGetLastError();
}

template <typename TS, typename TC, int R, int W, int WY, int TX, int TY>
hipError_t launch_box3_batch_cfg(const PassArgs *ps, int n, BatchStaging *stage, hipStream_t stream)
{
    using Cfg = Box3Cfg<TS, TC, R, W, WY, TX, TY>;
    using Args = Box3Args<TC, Cfg::K>;
    std::vector<Args> jobs;
    std::vector<int> start(1, 0);
    jobs.reserve(n);
    for (int i = 0; i < n; ++i) {
        Args a;
        hipError_t err;
        if (!box3_args<TS, TC, R, W, WY, TX, TY>(ps[i], &a, &err)) {
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
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, valu3d_box_batch_kernel<TS, TC, R, W, WY, TX, TY>,
                                                     TX * TY, 0);
    if (e != hipSuccess || occ < 1) occ = 1;
    const int slots = occ * (ps[0].num_cu > 0 ? ps[0].num_cu : 256);
    const int total = start.back();
    hipLaunchKernelGGL((valu3d_box_batch_kernel<TS, TC, R, W, WY, TX, TY>), dim3(total < slots ? total : slots),
                       dim3(TX * TY), 0, stream, static_cast<const Args *>(djobs),
                       static_cast<const int *>(dstart), (int)jobs.size());
    return hipGetLastError();
}

// Tiles: 16 columns of threads with one 16-byte vector each (float32 4
// points, float64 2) and one row per thread; 16 thread rows for r = 3, 32 for
// r = 2.  Measured on 384^3 / 512^3 periodic grids against 2-row threads,
// 3-row threads and 8 x 32 / 32 x 8 thread tiles: the one-row threads need
// 70-96 VGPRs and keep 5-7 waves per SIMD, which hides the LDS and
// scalar-load latencies best (5-15 % faster).
template <typename TS, typename TC, int R>
hipError_t launch_box3(const PassArgs &p, hipStream_t stream)
{
    constexpr int W = sizeof(TC) == 8 ? 2 : 4;
    return launch_box3_cfg<TS, TC, R, W, 1, 16, (R >= 3 ? 16 : 32)>(p, stream);
}

template <typename TS, typename TC, int R>
hipError_t launch_box3_batch(const PassArgs *ps, int n, BatchStaging *stage, hipStream_t stream)
{
    constexpr int W = sizeof(TC) == 8 ? 2 : 4;
    return launch_box3_batch_cfg<TS, TC, R, W, 1, 16, (R >= 3 ? 16 : 32)>(ps, n, stage, stream);
}

#define B3(TS, TC, DT, R) \
    {STENCIL_PATH_VALU, DT, STENCIL_BOX, 3, R, 1, &launch_box3<TS, TC, R>, &launch_box3_batch<TS, TC, R>}

}  // namespace

const std::vector<KernelEntry> &valu3d_box_kernels()
{
    static const std::vector<KernelEntry> table = {
        B3(double, double, STENCIL_F64, 2), B3(double, double, STENCIL_F64, 3),
        B3(float, float, STENCIL_F32, 2),   B3(float, float, STENCIL_F32, 3),
    };
    return table;
}

}  // namespace stl
