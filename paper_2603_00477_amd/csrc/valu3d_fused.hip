// VALU path, d = 3, T >= 2 explicit steps fused per pass (temporal fusion,
// paper Sec. "CUDA Core Implementation with Temporal Fusion": the intermediate
// fields of the T steps stay on chip, so a pass moves one field in and one out
// while its arithmetic grows with T, Eq. 8).
//
// A workgroup streams down a segment of z planes.  In each plane it computes
// step 1 on a layout of L1 x M1 points (each thread WY rows x W consecutive
// columns) and steps 2..T on the same layout; only the layout shrunk by
// R (T - 1) per side is exact after T steps, and that is the output tile.
//
// Input staging is cooperative and separate from the compute layout: all
// threads copy the layout plus its R-point halo, as whole aligned vectors, from
// HBM into the step-0 LDS plane, a prefetched plane at a time.  The step-1
// region therefore needs no skirt of its own, and the redundant ring is
// R (T - 1) wide rather than R T.
//
// The z pipeline is the one of the one-step 3D kernel: step s reads the plane
// step s-1 wrote one iteration earlier, scatters it into 2R+1 rotating
// accumulator planes (input plane z adds its in-plane neighbourhood weighted
// by w[c][.][.] to output plane z-c) and emits the completed plane, either to
// its own LDS plane (s < T) or to HBM (s = T).  One barrier per plane.
//
// Every LDS plane has the same geometry: row 0 is layout row -R, column OX is
// layout column 0, where OX >= R is chosen so that LDS column 0 sits on a
// vector boundary of the grid row whenever the output tile does.

#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <type_traits>

#include "internal.h"
#include "valu_common.h"

namespace stl {
namespace {

template <typename TC, int K>
struct Fused3DArgs {
    const void *src;
    void *dst;
    int n0, n1, n2;
    int oz0, oz1, oy0, oy1, ox0, ox1;
    int BZ, nty, ntx, nzs, ntiles;
    int periodic;
    TC h;
    TC w[K];
};

// value of v in lane (lane - 1) (PREV) or (lane + 1) of the same 16-lane
// row; the row's first (PREV) or last lane receives `edge`
template <bool PREV>
__device__ __forceinline__ float lane_row_shift(float v, float edge)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(edge), __float_as_int(v), PREV ? 0x111 : 0x101,
                                                      0xF, 0xF, false));
}

template <typename TS, typename TC, int SHAPE, int R, int T, int W, int WY, int TX, int TY>
struct Fused3DCfg {
    static constexpr int K = SHAPE == STENCIL_BOX ? (2 * R + 1) * (2 * R + 1) * (2 * R + 1) : 6 * R + 1;
    static constexpr int NT = TX * TY;
    static constexpr int L1 = TY * WY;                      // layout rows
    static constexpr int M1 = TX * W;                       // layout columns
    static constexpr int SK = R * (T - 1);                  // exact margin around the output tile
    static constexpr int SKL = ((SK + W - 1) / W) * W;      // left margin, whole vectors
    static constexpr int BY = L1 - 2 * SK;                  // output tile rows
    static constexpr int BX = ((M1 - SKL - SK) / W) * W;    // output tile columns (whole vectors)
    static constexpr int OX = ((R + W - 1) / W) * W;        // LDS column of layout column 0
    static constexpr int NV = (OX + M1 + R + W - 1) / W;    // staged vectors per row
    static constexpr int LDX = NV * W;                      // LDS row pitch
    static constexpr int LR = L1 + 2 * R;                   // LDS rows
    static constexpr int PLANE = LR * LDX;
    static constexpr int NSV = LR * NV;                     // staged vectors per plane
    static constexpr int NS = (NSV + NT - 1) / NT;          // ... per thread
    static constexpr int Q = 2 * R + 1;
    // 0: weights in scalar registers; 1: pinned in vector registers (float32
    // FMAs with a scalar operand issue slower on gfx950)
    static constexpr int WMODE = (sizeof(TC) * K <= 192 && (sizeof(TC) == 8 || R >= 3)) ? 0 : 1;
    static_assert(BY > 0 && BX > 0, "layout narrower than the fused margin");
    static_assert(sizeof(TC) * K <= 256, "large boxes run on the one-step box kernel");
};

// W consecutive compute-type values to LDS at an address that is a multiple
// of the vector (LDS rows hold whole vectors).
template <typename TC, int W>
__device__ __forceinline__ void store_lds_vec(const RawVec<TC, W> &o, TC *d)
{
    if constexpr (sizeof(TC) * W == 16 || sizeof(TC) * W == 8)
        o.store(static_cast<TC *>(__builtin_assume_aligned(d, sizeof(TC) * W)));
    else
#pragma unroll
        for (int j = 0; j < W; ++j) d[j] = o.e[j];
}

template <int R>
__device__ __forceinline__ int star3f_index(int axis, int off)
{
    return 1 + axis * 2 * R + (off < 0 ? off + R : off + R - 1);
}

template <typename TS, typename TC, int SHAPE, int R, int T, int W, int WY, int TX, int TY, bool FAST>
__device__ __forceinline__ void fused3d_tile(
    const Fused3DArgs<TC, Fused3DCfg<TS, TC, SHAPE, R, T, W, WY, TX, TY>::K> &a, const int tile,
    TC (&lds)[T][2][Fused3DCfg<TS, TC, SHAPE, R, T, W, WY, TX, TY>::PLANE])
{
    using Cfg = Fused3DCfg<TS, TC, SHAPE, R, T, W, WY, TX, TY>;
    constexpr int K = Cfg::K, Q = Cfg::Q, NT = Cfg::NT, LDX = Cfg::LDX, PLANE = Cfg::PLANE;
    constexpr int NS = Cfg::NS, NV = Cfg::NV, SK = Cfg::SK, SKL = Cfg::SKL, OX = Cfg::OX;
    using Vec = RawVec<TS, W>;

    const int tid = threadIdx.x;
    const int tx = tid % TX, ty = tid / TX;
    const int tzs = tile / (a.nty * a.ntx);
    const int rem = tile - tzs * (a.nty * a.ntx);
    const int tyi = rem / a.ntx, txi = rem - tyi * a.ntx;
    const int z0 = a.oz0 + tzs * a.BZ;
    const int z1 = min(z0 + a.BZ, a.oz1);
    const int BZe = z1 - z0;
    const int y0 = a.oy0 + tyi * Cfg::BY;
    const int ye = min(y0 + Cfg::BY, a.oy1);
    const int x0 = a.ox0 + txi * Cfg::BX;
    const int xe = min(x0 + Cfg::BX, a.ox1);
    const int cy0 = y0 - SK + ty * WY;  // grid row of this thread's first point
    const int cx0 = x0 - SKL + tx * W;  // grid column of this thread's first point
    const int sy0 = y0 - SK - R;        // grid row of LDS row 0
    const int sx0 = x0 - SKL - OX;      // grid column of LDS column 0 (a vector boundary when x0 is)

    const TS *src = static_cast<const TS *>(a.src);
    TS *dst = static_cast<TS *>(a.dst);
    const int n0 = a.n0, n1 = a.n1, n2 = a.n2;
    const bool periodic = a.periodic != 0;
    const TC h = a.h;

    for (int i = tid; i < T * 2 * PLANE; i += NT) (&lds[0][0][0])[i] = TC(0);

    TC wk[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        wk[k] = a.w[k];
        if constexpr (Cfg::WMODE == 1) asm volatile("" : "+v"(wk[k]));
    }

    bool col_in[W], col_store[W];
#pragma unroll
    for (int j = 0; j < W; ++j) {
        const int c = cx0 + j;
        col_in[j] = c >= 0 && c < n2;
        col_store[j] = c >= x0 && c < xe;
    }
    bool row_in[WY], row_store[WY];
#pragma unroll
    for (int i = 0; i < WY; ++i) {
        const int r = cy0 + i;
        row_in[i] = r >= 0 && r < n1;
        row_store[i] = r >= y0 && r < ye;
    }

    // Fast staging: rows of whole aligned vectors (grid row a multiple of the
    // vector, tile on a vector boundary).  Every staged vector then lies
    // wholly inside or wholly outside the grid: periodic ones wrap by whole
    // vectors, Dirichlet ones outside are h.  Each thread loads its vectors
    // unconditionally (entries past the plane repeat the last vector; those
    // outside a Dirichlet grid load a valid dummy) and selects h at the LDS
    // write, so staging has no per-vector branch and the prefetched loads are
    // waited for once per 2R+1 planes.  Other tiles (rows not a whole number
    // of vectors, unaligned sub-regions) stage element by element.
    constexpr bool fast = FAST;
    int s_lds[NS], s_row[NS], s_col[NS];
    bool s_h[NS], s_ok[NS];
#pragma unroll
    for (int i = 0; i < NS; ++i) {
        const int e0 = tid + i * NT;
        s_ok[i] = e0 < Cfg::NSV;
        const int e = s_ok[i] ? e0 : Cfg::NSV - 1;
        const int row = e / NV, v = e - (e / NV) * NV;
        const int gy = sy0 + row, gc = sx0 + v * W;
        s_lds[i] = row * LDX + v * W;
        if (periodic) {
            s_row[i] = wrap(gy, n1);
            s_col[i] = fast ? wrap(gc, n2) : gc;
            s_h[i] = false;
        } else {
            const bool rin = gy >= 0 && gy < n1;
            const bool cin = gc >= 0 && gc + W <= n2;
            s_row[i] = rin ? gy : -1;
            s_col[i] = gc;
            s_h[i] = !rin || !cin;  // fast path: the whole vector is h
            if (fast && s_h[i]) {    // valid dummy source
                s_row[i] = 0;
                s_col[i] = 0;
            }
        }
    }
    const int KTOT = BZe + 2 * R * T + T;
    const int zbase = z0 - R * T;
    auto plane_ptr = [&](int k) -> const TS * {
        const int z = zbase + k;
        return src + (int64_t)(periodic ? wrap(z, n0) : min(max(z, 0), n0 - 1)) * n1 * n2;
    };
    auto plane_in = [&](int k) -> bool {
        const int z = zbase + k;
        return periodic || (z >= 0 && z < n0);
    };

    const bool dst_vec = vec_aligned<TS, W>(dst, n2, x0);
    // LDS offset of this thread's first point inside a plane
    const int lpos = (R + ty * WY) * LDX + OX + tx * W;
    // Window edges from the neighbouring lane.  Each lane's single-element
    // reads of the r columns left and right of its vector all fall in banks
    // of one residue mod 4 (the row pitch keeps the vectors aligned), a 4-way
    // conflict.  With rows of 16 threads (one DPP row each) the edges are
    // the neighbours' own elements: a row shift by one lane, the first and
    // last lanes of the row taking the LDS value instead; the other lanes
    // read a dummy element of their own vector, spread over the banks.
    // Measured on 512^3 float32: Box-3D1R T = 2 / 3 600 -> 651, 642 -> 726,
    // Star-3D3R T = 2 518 -> 553 GSt/s; Star-3D2R 5-10 % slower (stars need
    // edges on their middle rows only), Star-3D1R unchanged.
    constexpr bool XDPP = TX == 16 && R <= W && sizeof(TC) == 4 && (SHAPE == STENCIL_BOX || R >= 3);
    const int dj = R + ((tx + ty) & (W - 1));

    {
        auto load_plane = [&](int k, Vec (&v)[NS]) {
            if constexpr (FAST) {
                const TS *pl = plane_ptr(k);
#pragma unroll
                for (int i = 0; i < NS; ++i) v[i].load(pl + (int64_t)s_row[i] * n2 + s_col[i]);
            }
        };
        auto stage_plane = [&](int k, const Vec (&v)[NS], TC *w0) {
            const bool zin = plane_in(k);
            if constexpr (FAST) {
#pragma unroll
                for (int i = 0; i < NS; ++i) {
                    RawVec<TC, W> o;
#pragma unroll
                    for (int j = 0; j < W; ++j) o.e[j] = (s_h[i] || !zin) ? h : to_compute<TC>(v[i].e[j]);
                    store_lds_vec(o, w0 + s_lds[i]);
                }
            } else {
                const TS *pl = plane_ptr(k);
#pragma unroll
                for (int i = 0; i < NS; ++i) {
                    if (!s_ok[i]) continue;
                    TC *d = w0 + s_lds[i];
                    const TS *rowp = pl + (int64_t)(s_row[i] < 0 ? 0 : s_row[i]) * n2;
#pragma unroll
                    for (int j = 0; j < W; ++j) {
                        const int c = s_col[i] + j;
                        const bool in = zin && s_row[i] >= 0 && c >= 0 && c < n2;
                        d[j] = periodic ? to_compute<TC>(rowp[wrap(c, n2)]) : (in ? to_compute<TC>(rowp[c]) : h);
                    }
                }
            }
        };

        TC acc[T][Q][WY][W];
#pragma unroll
        for (int s = 0; s < T; ++s)
#pragma unroll
            for (int q = 0; q < Q; ++q)
#pragma unroll
                for (int i = 0; i < WY; ++i)
#pragma unroll
                    for (int j = 0; j < W; ++j) acc[s][q][i][j] = TC(0);

        // prefetch of the next plane (one plane ahead: the plane's compute
        // covers the load latency, and a deeper ring costs registers)
        Vec ring[NS];
        load_plane(0, ring);
        __syncthreads();

        for (int kb = 0; kb < KTOT; kb += Q) {
#pragma unroll
            for (int u = 0; u < Q; ++u) {
                const int k = kb + u;
                if (k >= KTOT) break;
                const int par = k & 1;
                {
                    stage_plane(k, ring, &lds[0][par][0]);
                    // keep the refill of the ring behind the writes that drain it
                    __builtin_amdgcn_sched_barrier(0);
                    if (k + 1 < KTOT) load_plane(k + 1, ring);
                }
#pragma unroll
                for (int s = 1; s <= T; ++s) {
                    const bool active = k >= s + 2 * R * (s - 1) && k < BZe + 2 * R * T + s;
                    const int qc = u % Q;
                    if (active) {
                        const TC *rb = &lds[s - 1][par ^ 1][lpos - R * LDX - R];
#pragma unroll
                        for (int wi = 0; wi < WY + 2 * R; ++wi) {
                            const bool mid = wi >= R && wi < R + WY;
                            TC row[W + 2 * R];
                            if constexpr (XDPP) {
#pragma unroll
                                for (int j = 0; j < W; ++j) row[R + j] = rb[wi * LDX + R + j];
#pragma unroll
                                for (int j = 0; j < R; ++j) {
                                    row[j] = TC(0);
                                    row[R + W + j] = TC(0);
                                }
                                if (SHAPE == STENCIL_BOX || mid) {
#pragma unroll
                                    for (int m = 0; m < R; ++m) {
                                        const TC lt = rb[wi * LDX + (tx == 0 ? m : dj)];
                                        const TC rt = rb[wi * LDX + (tx == TX - 1 ? R + W + m : dj)];
                                        row[m] = lane_row_shift<true>(row[W + m], lt);
                                        row[R + W + m] = lane_row_shift<false>(row[R + m], rt);
                                    }
                                }
                            } else {
#pragma unroll
                                for (int j = 0; j < W + 2 * R; ++j) {
                                    const bool need = SHAPE == STENCIL_BOX || mid || (j >= R && j < R + W);
                                    row[j] = need ? rb[wi * LDX + j] : TC(0);
                                }
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
                                            const TC wv = wk[((c + R) * (2 * R + 1) + (ao + R)) * (2 * R + 1) + (bo + R)];
#pragma unroll
                                            for (int j = 0; j < W; ++j)
                                                acc[s - 1][q][i][j] = fma_c(wv, row[j + bo + R], acc[s - 1][q][i][j]);
                                        }
                                    } else {
                                        if (c != 0) {
                                            if (ao != 0) continue;  // z arm: own column only
                                            const TC wv = wk[star3f_index<R>(0, c)];
#pragma unroll
                                            for (int j = 0; j < W; ++j)
                                                acc[s - 1][q][i][j] = fma_c(wv, row[j + R], acc[s - 1][q][i][j]);
                                        } else if (ao != 0) {  // y arm
                                            const TC wv = wk[star3f_index<R>(1, ao)];
#pragma unroll
                                            for (int j = 0; j < W; ++j)
                                                acc[s - 1][q][i][j] = fma_c(wv, row[j + R], acc[s - 1][q][i][j]);
                                        } else {  // x arm with the centre
#pragma unroll
                                            for (int bo = -R; bo <= R; ++bo) {
                                                const TC wv = bo == 0 ? wk[0] : wk[star3f_index<R>(2, bo)];
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
                            for (int i = 0; i < WY; ++i) {
                                RawVec<TC, W> o;
#pragma unroll
                                for (int j = 0; j < W; ++j) {
                                    TC v = acc[s - 1][qc][i][j];
                                    if (!periodic && !(zin && row_in[i] && col_in[j])) v = h;
                                    o.e[j] = v;
                                }
                                store_lds_vec(o, wr + i * LDX);
                            }
                        } else if (zo >= z0 && zo < z1) {
                            TS *pl = dst + (int64_t)zo * n1 * n2;
#pragma unroll
                            for (int i = 0; i < WY; ++i) {
                                if (!row_store[i]) continue;
                                TS *rowp = pl + (int64_t)(cy0 + i) * n2 + cx0;
                                Vec ov;
                                bool all = dst_vec;
#pragma unroll
                                for (int j = 0; j < W; ++j) {
                                    ov.e[j] = to_storage<TS>(acc[s - 1][qc][i][j]);
                                    all = all && col_store[j];
                                }
                                if (all) {
                                    ov.store(rowp);
                                } else {
#pragma unroll
                                    for (int j = 0; j < W; ++j)
                                        if (col_store[j]) rowp[j] = ov.e[j];
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
}

// Whether a tile takes the fast staging path: rows of whole aligned vectors
// and a tile starting on a vector boundary.
template <typename TS, int W, typename A>
__device__ __forceinline__ bool fused3d_fast(const A &a, int tile, int BX)
{
    const int rem = tile % (a.nty * a.ntx);
    const int x0 = a.ox0 + (rem % a.ntx) * BX;
    return vec_aligned<TS, W>(a.src, a.n2, 0) && (x0 % W) == 0;
}

template <typename TS, typename TC, int SHAPE, int R, int T, int W, int WY, int TX, int TY>
__global__ __launch_bounds__(TX *TY) void fused3d_kernel(
    Fused3DArgs<TC, Fused3DCfg<TS, TC, SHAPE, R, T, W, WY, TX, TY>::K> a)
{
    using Cfg = Fused3DCfg<TS, TC, SHAPE, R, T, W, WY, TX, TY>;
    __shared__ __attribute__((aligned(16))) TC lds[T][2][Cfg::PLANE];
    const int tile = xcd_remap(blockIdx.x, gridDim.x);
    if (tile >= a.ntiles) return;
    if (fused3d_fast<TS, W>(a, tile, Cfg::BX))
        fused3d_tile<TS, TC, SHAPE, R, T, W, WY, TX, TY, true>(a, tile, lds);
    else
        fused3d_tile<TS, TC, SHAPE, R, T, W, WY, TX, TY, false>(a, tile, lds);
}

// Persistent batched launch over the tiles of every job of the batch (see the
// one-step 3D kernel); the tile body ends with a barrier.
template <typename TS, typename TC, int SHAPE, int R, int T, int W, int WY, int TX, int TY>
__global__ __launch_bounds__(TX *TY) void fused3d_batch_kernel(
    const Fused3DArgs<TC, Fused3DCfg<TS, TC, SHAPE, R, T, W, WY, TX, TY>::K> *__restrict__ jobs,
    const int *__restrict__ tile_start, int njobs)
{
    using Cfg = Fused3DCfg<TS, TC, SHAPE, R, T, W, WY, TX, TY>;
    __shared__ __attribute__((aligned(16))) TC lds[T][2][Cfg::PLANE];
    const int total = tile_start[njobs];
    int j = 0;
    for (int item = xcd_remap(blockIdx.x, gridDim.x); item < total; item += gridDim.x) {
        while (j + 1 < njobs && tile_start[j + 1] <= item) ++j;
        const Fused3DArgs<TC, Cfg::K> a = jobs[j];
        const int tile = item - tile_start[j];
        if (fused3d_fast<TS, W>(a, tile, Cfg::BX))
            fused3d_tile<TS, TC, SHAPE, R, T, W, WY, TX, TY, true>(a, tile, lds);
        else
            fused3d_tile<TS, TC, SHAPE, R, T, W, WY, TX, TY, false>(a, tile, lds);
    }
}

// Segment length along z: the number of segments maximises (share of the
// resident slots the last round keeps busy) x (share of staged planes that
// are outputs, BZ / (BZ + 2 R T)), with segments of at least max(8 R T, 32)
// planes (or the whole grid): shorter ones restage and recompute their
// 2 R T + T lead-in planes too often, which a batched launch of many small
// grids does not need to fill the GPU.
inline int fused3d_segments(int D0, int inplane, int slots, int R, int T)
{
    const int minBZ = 8 * R * T > 32 ? 8 * R * T : 32;
    int best = 1;
    double best_score = -1.0;
    for (int segs = 1; segs <= 256 && segs <= D0; ++segs) {
        const int BZ = (D0 + segs - 1) / segs;
        if (segs > 1 && BZ < minBZ) break;
        const int nzs = (D0 + BZ - 1) / BZ;
        const int64_t items = (int64_t)nzs * inplane;
        const int64_t rounds = (items + slots - 1) / slots;
        const double balance = (double)items / (double)(rounds * slots);
        const double zeff = (double)BZ / (double)(BZ + 2 * R * T);
        const double score = balance * zeff;
        if (score > best_score + 1e-9) {
            best_score = score;
            best = segs;
        }
    }
    return best;
}

template <typename TS, typename TC, int SHAPE, int R, int T, int W, int WY, int TX, int TY>
bool fused3d_args(const PassArgs &p, int slots,
                  Fused3DArgs<TC, Fused3DCfg<TS, TC, SHAPE, R, T, W, WY, TX, TY>::K> *out, hipError_t *err)
{
    using Cfg = Fused3DCfg<TS, TC, SHAPE, R, T, W, WY, TX, TY>;
    *err = hipSuccess;
    Fused3DArgs<TC, Cfg::K> &a = *out;
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
    a.nty = (D1 + Cfg::BY - 1) / Cfg::BY;
    a.ntx = (D2 + Cfg::BX - 1) / Cfg::BX;
    int BZ = p.tile_rows;
    if (BZ <= 0) {
        const int segs = fused3d_segments(D0, a.nty * a.ntx, slots, R, T);
        BZ = (D0 + segs - 1) / segs;
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

// resident workgroups per CU x CUs
template <typename K>
int fused3d_slots(K kernel, int threads, int num_cu)
{
    int occ = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kernel, threads, 0) != hipSuccess || occ < 1) occ = 1;
    return occ * (num_cu > 0 ? num_cu : 256);
}

template <typename TS, typename TC, int SHAPE, int R, int T, int W, int WY, int TX, int TY>
hipError_t launch_fused3d_cfg(const PassArgs &p, hipStream_t stream)
{
    using Cfg = Fused3DCfg<TS, TC, SHAPE, R, T, W, WY, TX, TY>;
    static const int slots = fused3d_slots(fused3d_kernel<TS, TC, SHAPE, R, T, W, WY, TX, TY>, TX * TY,
                                           p.num_cu);
    Fused3DArgs<TC, Cfg::K> a;
    hipError_t err;
    if (!fused3d_args<TS, TC, SHAPE, R, T, W, WY, TX, TY>(p, slots, &a, &err)) return err;
    hipLaunchKernelGGL((fused3d_kernel<TS, TC, SHAPE, R, T, W, WY, TX, TY>), dim3(a.ntiles), dim3(TX * TY), 0,
                       stream, a);
    return hipGetLastError();
}

template <typename TS, typename TC, int SHAPE, int R, int T, int W, int WY, int TX, int TY>
hipError_t launch_fused3d_batch_cfg(const PassArgs *ps, int n, BatchStaging *stage, hipStream_t stream)
{
    using Cfg = Fused3DCfg<TS, TC, SHAPE, R, T, W, WY, TX, TY>;
    using Args = Fused3DArgs<TC, Cfg::K>;
    static const int slots = fused3d_slots(fused3d_batch_kernel<TS, TC, SHAPE, R, T, W, WY, TX, TY>,
                                           TX * TY, ps[0].num_cu);
    std::vector<Args> jobs;
    std::vector<int> start(1, 0);
    jobs.reserve(n);
    for (int i = 0; i < n; ++i) {
        Args a;
        hipError_t err;
        if (!fused3d_args<TS, TC, SHAPE, R, T, W, WY, TX, TY>(ps[i], slots, &a, &err)) {
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
    const int total = start.back();
    hipLaunchKernelGGL((fused3d_batch_kernel<TS, TC, SHAPE, R, T, W, WY, TX, TY>),
                       dim3(total < slots ? total : slots), dim3(TX * TY), 0, stream,
                       static_cast<const Args *>(djobs), static_cast<const int *>(dstart), (int)jobs.size());
    return hipGetLastError();
}

// Thread layouts: W consecutive columns per thread (float64 2, float32 4), 2
// rows per thread.  Stars take 16 x 32 threads (a 64-row layout: the skirt is
// a smaller share of it); measured on 512^3 against 16 x 16, Star-3D2R float32
// T = 3 runs at 959 vs 517 GSt/s and Star-3D3R float64 T = 2 at 323 vs 281.
// The 27-point box takes a 32-row x 64-column layout: 16 x 16 threads in
// float32 (Box-3D1R T = 2: 601 vs 574 GSt/s with 32 thread rows; two resident
// workgroups per CU matter more than a smaller skirt), 32 x 16 in float64
// (406 vs 374 against 16 x 16: 512 columns take 9 output tiles of 60 instead
// of 19 of 28).
template <typename TS, int SHAPE, int R, int T>
struct Fused3DShape {
    static constexpr int W = sizeof(TS) == 8 ? 2 : 4;
    static constexpr int WY = 2;
    static constexpr int TX = SHAPE == STENCIL_STAR ? 16 : 64 / W;
    static constexpr int TY = SHAPE == STENCIL_STAR ? 32 : 16;
};

template <typename TS, typename TC, int SHAPE, int R, int T>
hipError_t launch_fused3d(const PassArgs &p, hipStream_t stream)
{
    using S = Fused3DShape<TS, SHAPE, R, T>;
    return launch_fused3d_cfg<TS, TC, SHAPE, R, T, S::W, S::WY, S::TX, S::TY>(p, stream);
}

template <typename TS, typename TC, int SHAPE, int R, int T>
hipError_t launch_fused3d_batch(const PassArgs *ps, int n, BatchStaging *stage, hipStream_t stream)
{
    using S = Fused3DShape<TS, SHAPE, R, T>;
    return launch_fused3d_batch_cfg<TS, TC, SHAPE, R, T, S::W, S::WY, S::TX, S::TY>(ps, n, stage, stream);
}

#define F3(TS, TC, DT, SH, R, T) \
    {STENCIL_PATH_VALU, DT, SH, 3, R, T, &launch_fused3d<TS, TC, SH, R, T>, &launch_fused3d_batch<TS, TC, SH, R, T>}
#define F3_S(TS, TC, DT)                                                                                  \
    F3(TS, TC, DT, STENCIL_STAR, 1, 2), F3(TS, TC, DT, STENCIL_STAR, 1, 3), F3(TS, TC, DT, STENCIL_STAR, 2, 2), \
        F3(TS, TC, DT, STENCIL_STAR, 2, 3), F3(TS, TC, DT, STENCIL_STAR, 3, 2), F3(TS, TC, DT, STENCIL_BOX, 1, 2), \
        F3(TS, TC, DT, STENCIL_BOX, 1, 3)

}  // namespace

const std::vector<KernelEntry> &valu3d_fused_kernels()
{
    static const std::vector<KernelEntry> table = {
        F3_S(double, double, STENCIL_F64),
        F3_S(float, float, STENCIL_F32),
    };
    return table;
}

}  // namespace stl
