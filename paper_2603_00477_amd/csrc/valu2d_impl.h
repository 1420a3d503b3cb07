// VALU path, d = 2: T explicit steps fused per pass (temporal fusion on the
// vector units; paper, Sec. "CUDA Core Implementation with Temporal Fusion":
// C grows by t, M stays 2D per point because intermediates stay on chip).
//
// Work decomposition
//   Every wave is independent: it owns a column band of 64*W columns (each
//   lane W consecutive columns) and streams down a segment of rows.  Of the
//   band, E = roundup(R*T, W) columns on each side are the skirt that later
//   steps consume; the valid output width is BX = 64W - 2E.  There is no LDS
//   and no barrier: neighbour columns come from cross-lane permutes (DPP
//   rotates for float64 with four columns per lane).
//
// Step pipeline
//   Stage 0 takes input row k (prefetched P rows ahead into registers).
//   Stage s = 1..T consumes the row stage s-1 produced one iteration earlier,
//   as a (W + 2R)-column window assembled by permutes at the end of that
//   iteration (so the permute latency overlaps the next row's arithmetic).
//   It scatters the window into 2R+1 rotating accumulator rows per lane
//   column (input-stationary: input row i adds w[a][.] to output row i-a) and
//   emits the completed output row i-R: to the next stage, or to HBM for
//   stage T.  Contributions to an output arrive in canonical order (kernel
//   row a ascending, column b ascending).
//
// Boundaries
//   Dirichlet: every field, intermediate ones included, is h outside the grid
//   (rows and columns outside are forced to h after each stage).  Periodic:
//   loads wrap; intermediate values in the skirt are then the periodic images.
//
// The kernel writes an arbitrary output rectangle [oy0,oy1) x [ox0,ox1), used
// both for whole grids and for the Dirichlet boundary band of the MFMA path.

#pragma once

#include <cstddef>

#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include "internal.h"
#include "valu_common.h"

namespace stl {

// Geometry of one pass of one grid: output box, tiling and boundary.
template <typename TC>
struct Valu2DJob {
    const void *src;
    void *dst;
    int n0, n1;
    int oy0, oy1, ox0, ox1;
    int BX, BY, nbands, nsegs;
    int nwg;  // workgroup items: ceil(nbands / waves) band groups x nsegs segments
    int periodic;
    TC h;
};

template <typename TC, int K>
struct Valu2DArgs {
    Valu2DJob<TC> g;
    TC w[K];
};

constexpr int kValu2DWaves = 4;  // waves per workgroup (independent bands)

template <typename TS, typename TC, int SHAPE, int R, int T, int W>
struct Valu2DCfg {
    static constexpr int K = SHAPE == STENCIL_BOX ? (2 * R + 1) * (2 * R + 1) : 4 * R + 1;
    static constexpr int NCW = 64 * W;                     // columns per wave
    static constexpr int E = ((R * T + W - 1) / W) * W;    // skirt per side
    static constexpr int Q = 2 * R + 1;
    // rows prefetched ahead: a multiple of Q, at least 4
    static constexpr int U = Q * ((4 + Q - 1) / Q);
    // input rows in flight: U for small Q; for r = 7 (Q = 15, compute-bound,
    // 225 or 29 FMAs per input value) 3 rows, a divisor of U, so the ring
    // slot of row k is k mod P at compile time and 48 VGPRs stay free
    // 32-byte lanes (float64 at T = 2) prefetch one row: their rows take
    // twice the arithmetic, and the registers go to the wider accumulators
    static constexpr int P = sizeof(TS) * W > 16 ? 1
                             : (U <= 8 ? U : (U % 3 == 0 ? 3 : (U % 4 == 0 ? 4 : (U % 5 == 0 ? 5 : U))));
    // Boxes whose weights exceed 48 dwords (float64 r >= 2, float32 r = 3)
    // fused over T >= 3 steps keep them out of the vector registers: stored
    // column-major (w[b][a]), each column of 2R+1 is scalar-loaded just before
    // its FMAs.  That frees 49-98 VGPRs for the T stages' accumulators
    // (Box-2D3R float64 T = 4: 232 instead of 340 registers, no spills, +30 %
    // measured).  Float64 at T = 1 streams them too (Box-2D3R: 88 instead of
    // 236 VGPRs; +9 % measured at 10240^2, equal at 8192^2).  Float32 at T = 2
    // keeps them pinned in VGPRs (632 vs 478 GSt/s measured) unless they need
    // more than 128 dwords (r = 7: 225 weights).  Float64 at T = 2 runs
    // 32-byte lanes, which stream them too: each weight then serves four
    // columns, and the freed registers hold the wider accumulators at two
    // waves per SIMD.
    static constexpr bool WPTR = SHAPE == STENCIL_BOX && sizeof(TC) * K > 192 &&
                                 (T >= 3 || sizeof(TC) == 8 || sizeof(TC) * K > 512);
    // Streamed weights at T >= 3: each column is fetched once per input row
    // and serves every stage (columns outer, stages inner) instead of once
    // per stage.  Measured on 8192^2: Box-2D2R float64 T = 4 476 -> 570,
    // Box-2D3R float32 T = 3/4 498/501 -> 532/556, float64 302 -> 317
    // GSt/s; at T = 2 the per-stage order is as fast or faster (Box-2D3R
    // float64 353 vs 344).
    static constexpr bool WCOL = WPTR && T >= 3;
};

// Weights in constant memory (scalar loads).
template <typename TC>
using ConstPtr = const __attribute__((address_space(4))) TC *;

// Weight order the kernels expect: canonical, or column-major for WPTR boxes.
template <typename Cfg, int R>
__host__ __device__ constexpr int weight_slot(int k)
{
    if constexpr (Cfg::WPTR) {
        const int a = k / (2 * R + 1), b = k % (2 * R + 1);
        return b * (2 * R + 1) + a;
    } else {
        return k;
    }
}

template <int SHAPE, int R>
__device__ __forceinline__ int star_axis_index(int axis, int off)
{
    // canonical star order: centre, axis0 -R..-1,+1..+R, axis1 ...
    return 1 + axis * 2 * R + (off < 0 ? off + R : off + R - 1);
}

// value of `v` in lane (addr / 4) mod 64 (ds_bpermute: LDS crossbar, no storage)
__device__ __forceinline__ float lane_read(float v, int addr)
{
    return __int_as_float(__builtin_amdgcn_ds_bpermute(addr, __float_as_int(v)));
}
__device__ __forceinline__ double lane_read(double v, int addr)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_ds_bpermute(addr, (int)(b & 0xffffffffLL));
    const int hi = __builtin_amdgcn_ds_bpermute(addr, (int)(b >> 32));
    return __longlong_as_double(((long long)(unsigned)lo) | ((long long)hi << 32));
}

// value of `v` in lane (lane - 1) mod 64 (PREV) or (lane + 1) mod 64: a
// whole-wave DPP rotate by one lane (vector-ALU moves; no LDS access, so no
// lgkmcnt wait shared with the scalar weight loads)
template <bool PREV>
__device__ __forceinline__ double lane_rotate(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffLL), PREV ? 0x13C : 0x134, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), PREV ? 0x13C : 0x134, 0xF, 0xF, false);
    return __longlong_as_double(((long long)(unsigned)lo) | ((long long)hi << 32));
}

// win[j] = column lane*W - R + j of the wave's row, from the lanes' own W
// values (edge lanes receive wrapped values; those columns lie in the skirt).
// Float64 with four columns per lane (R <= W: every window column comes from
// the lane itself or a direct neighbour) rotates instead of permuting
// (Box-2D3R T = 2 8192^2: 366 -> 371 GSt/s); float32 and 16-bit storage
// measured 3-7 % slower with rotates.
template <typename TC, int W, int R>
__device__ __forceinline__ void assemble_window(const TC (&own)[W], TC (&win)[W + 2 * R], int lane)
{
#pragma unroll
    for (int j = 0; j < W; ++j) win[R + j] = own[j];
    if constexpr (sizeof(TC) == 8 && W == 4 && R <= W) {
#pragma unroll
        for (int m = 1; m <= R; ++m) win[R - m] = lane_rotate<true>(own[W - m]);
#pragma unroll
        for (int m = 0; m < R; ++m) win[R + W + m] = lane_rotate<false>(own[m]);
        return;
    }
#pragma unroll
    for (int m = 1; m <= R; ++m) {  // column lane*W - m
        const int dl = -((m + W - 1) / W);
        const int je = -m - dl * W;
        win[R - m] = lane_read(own[je], (lane + dl) * 4);
    }
#pragma unroll
    for (int m = 0; m < R; ++m) {  // column lane*W + W + m
        const int t = W + m;
        win[R + W + m] = lane_read(own[t % W], (lane + t / W) * 4);
    }
}

// One tile (column band x row segment) of one pass, run by one wave.
// FAST: the grid rows are whole aligned vectors and the output box starts on
// a vector boundary, so every lane's W columns lie wholly inside or wholly
// outside the grid.  Row loads are then one unconditional vector load per
// row (periodic lanes and rows wrap by whole vectors; Dirichlet ones outside
// the grid load a valid dummy and take h when the row is consumed); with no
// other write to the prefetch ring, the compiler waits only for the row being
// consumed and the loads of the next rows stay in flight.
template <typename TS, typename TC, int SHAPE, int R, int T, int W, bool FAST>
__device__ __forceinline__ void valu2d_tile(const Valu2DJob<TC> &a,
                                            const TC (&wk)[Valu2DCfg<TS, TC, SHAPE, R, T, W>::WPTR
                                                               ? 1
                                                               : Valu2DCfg<TS, TC, SHAPE, R, T, W>::K],
                                            ConstPtr<TC> wp, int band, int seg, int lane)
{
    using Cfg = Valu2DCfg<TS, TC, SHAPE, R, T, W>;
    constexpr int Q = Cfg::Q;
    constexpr int U = Cfg::U;
    using Vec = RawVec<TS, W>;

    const int x0 = a.ox0 + band * a.BX;
    const int y0 = a.oy0 + seg * a.BY;
    const int y1 = min(y0 + a.BY, a.oy1);
    const int BYe = y1 - y0;
    const int xe = min(x0 + a.BX, a.ox1);
    const int cb = x0 - Cfg::E + lane * W;  // first column owned by this lane

    const TS *src = static_cast<const TS *>(a.src);
    TS *dst = static_cast<TS *>(a.dst);
    const int n0 = a.n0, n1 = a.n1;
    const bool periodic = a.periodic != 0;
    const TC h = a.h;

    bool col_in[W];
    int col_src[W];
    bool col_store[W];
#pragma unroll
    for (int j = 0; j < W; ++j) {
        const int c = cb + j;
        col_in[j] = c >= 0 && c < n1;
        col_src[j] = periodic ? wrap(c, n1) : c;
        col_store[j] = c >= x0 && c < xe;
    }
    const bool vec_ok = vec_aligned<TS, W>(src, n1, cb) && cb >= 0 && cb + W <= n1;
    // output stores: the whole vector, or (lanes at the band's ragged edge)
    // element by element; the element path is skipped by a wave-uniform
    // branch when no lane of the wave needs it
    bool st_all = vec_ok, st_any = false;
#pragma unroll
    for (int j = 0; j < W; ++j) {
        st_all = st_all && col_store[j];
        st_any = st_any || col_store[j];
    }
    const bool st_part_wave = __ballot(st_any && !st_all) != 0;
    const TS hs = to_storage<TS>(h);

    const int KTOT = BYe + 2 * R * T + T;
    const int ybase = y0 - R * T;

    // accumulators: T stages x Q rotating rows x W columns
    TC acc[T][Q][W];
#pragma unroll
    for (int s = 0; s < T; ++s)
#pragma unroll
        for (int q = 0; q < Q; ++q)
#pragma unroll
            for (int j = 0; j < W; ++j) acc[s][q][j] = TC(0);
    // input windows of stages 1..T (the previous iteration's rows)
    TC wins[T][W + 2 * R];
#pragma unroll
    for (int s = 0; s < T; ++s)
#pragma unroll
        for (int j = 0; j < W + 2 * R; ++j) wins[s][j] = TC(0);

    // fast path: the lane's source column (wrapped, or a valid dummy) and
    // whether its vector lies outside a Dirichlet grid
    int f_col = cb;
    bool f_h = false;
    if constexpr (FAST) {
        if (periodic) {
            f_col = wrap(cb, n1);
        } else {
            const bool in = cb >= 0 && cb + W <= n1;
            f_h = !in;
            f_col = in ? cb : 0;
        }
    }
    auto load_row = [&](int k, Vec &v) {
        const int i = ybase + k;
        if constexpr (FAST) {
            const int ri = periodic ? wrap(i, n0) : min(max(i, 0), n0 - 1);
            v.load(src + (int64_t)ri * n1 + f_col);
            return;
        }
        const bool row_in = i >= 0 && i < n0;
        if (!periodic && !row_in) {
#pragma unroll
            for (int j = 0; j < W; ++j) v.e[j] = hs;
            return;
        }
        const int ri = periodic ? wrap(i, n0) : i;
        const TS *rowp = src + (int64_t)ri * n1;
        if (vec_ok) {
            v.load(rowp + cb);
        } else {
#pragma unroll
            for (int j = 0; j < W; ++j)
                v.e[j] = (periodic || col_in[j]) ? rowp[col_src[j]] : hs;
        }
    };

    constexpr int P = Cfg::P;
    Vec ring[P];
#pragma unroll
    for (int u = 0; u < P; ++u)
        if (u < KTOT) load_row(u, ring[u]);

    // WPTR: weight column b (2R+1 values) of the block being computed and of
    // the next one.  Scalar loads complete out of order, so any wait for one
    // waits for all: the fetch of the next column takes the current column's
    // first weight as an operand, which puts it after the wait for the
    // current column, and an empty volatile asm statement on the current
    // block's accumulators after its FMAs keeps the next wait behind them
    // (volatile asm statements keep their order), so each fetch overlaps a
    // whole block of FMAs and at most two columns are live.
    // float32: FMAs run faster on vector-register operands (one move per
    // weight).  For r >= 5 a column moves to vector registers when it becomes
    // current, after the previous block's FMAs, so its scalar loads complete
    // under them (moving at the fetch waits for each load at once and
    // serialises them: Box-2D7R 129 -> 135 GSt/s); for r = 3 moving at the
    // fetch measured as fast or slightly faster.
    constexpr bool LATE_MOVE = sizeof(TC) == 4 && R >= 5;
    TC wcur[Q], wnxt[Q];
    // The ordering dependency goes through the base pointer, so the column
    // offsets stay compile-time immediates of the scalar loads (an opaque
    // offset cost five scalar instructions of address arithmetic per column:
    // Box-2D3R float64 T = 2 370 -> 378 GSt/s without them).
    auto fetch_col = [&](int b, TC *dstw, TC after) {
        ConstPtr<TC> p = wp;
        if constexpr (sizeof(TC) == 4) asm volatile("" : "+s"(p) : "v"(after));
        else asm volatile("" : "+s"(p) : "s"(after));
#pragma unroll
        for (int e = 0; e < Q; ++e) {
            dstw[e] = p[b * Q + e];
            if constexpr (sizeof(TC) == 4 && !LATE_MOVE) asm volatile("" : "+v"(dstw[e]));
        }
    };
    auto to_vgpr = [&](TC *wv) {
        if constexpr (LATE_MOVE)
#pragma unroll
            for (int e = 0; e < Q; ++e) asm volatile("" : "+v"(wv[e]));
    };
    if constexpr (Cfg::WPTR) {
        fetch_col(0, wcur, TC(0));
        to_vgpr(wcur);
    }

    for (int kb = 0; kb < KTOT; kb += U) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int k = kb + u;
            if (k >= KTOT) break;
            // Stages run from T down to 1 so that the window each one produces
            // for the next stage can be assembled at once (its consumer has
            // already used the previous window this iteration); the permute
            // latency then hides behind the lower stages' arithmetic.
            if constexpr (Cfg::WCOL) {
#pragma unroll
                for (int bo = -R; bo <= R; ++bo) {
                    fetch_col(bo + R < 2 * R ? bo + R + 1 : 0, wnxt, wcur[0]);
#pragma unroll
                    for (int s = T; s >= 1; --s) {
                        const bool active = k >= s + 2 * R * (s - 1) && k < BYe + 2 * R * T + s;
                        if (!active) continue;
                        const TC *win = wins[s - 1];
#pragma unroll
                        for (int ao = -R; ao <= R; ++ao) {
                            const int q = ((u - ao + R) % Q + Q) % Q;
#pragma unroll
                            for (int j = 0; j < W; ++j)
                                acc[s - 1][q][j] = fma_c(wcur[ao + R], win[j + bo + R], acc[s - 1][q][j]);
                        }
                    }
                    // this column's FMAs complete before the wait for the next
                    // column's weights
#pragma unroll
                    for (int s = 0; s < T; ++s)
#pragma unroll
                        for (int q = 0; q < Q; ++q)
#pragma unroll
                            for (int j = 0; j < W; ++j) asm volatile("" ::"v"(acc[s][q][j]));
#pragma unroll
                    for (int e = 0; e < Q; ++e) wcur[e] = wnxt[e];
                    to_vgpr(wcur);
                }
            }
#pragma unroll
            for (int s = T; s >= 1; --s) {
                const bool active = k >= s + 2 * R * (s - 1) && k < BYe + 2 * R * T + s;
                const int qc = u % Q;  // slot completing at this iteration
                TC outv[W];
#pragma unroll
                for (int j = 0; j < W; ++j) outv[j] = TC(0);
                if (active) {
                    const TC *win = wins[s - 1];
                    if constexpr (Cfg::WCOL) {
                        // accumulated above, all stages per weight column
                    } else if constexpr (Cfg::WPTR) {
#pragma unroll
                        for (int bo = -R; bo <= R; ++bo) {
                            fetch_col(bo + R < 2 * R ? bo + R + 1 : 0, wnxt, wcur[0]);
#pragma unroll
                            for (int ao = -R; ao <= R; ++ao) {
                                const int q = ((u - ao + R) % Q + Q) % Q;
#pragma unroll
                                for (int j = 0; j < W; ++j)
                                    acc[s - 1][q][j] = fma_c(wcur[ao + R], win[j + bo + R], acc[s - 1][q][j]);
                            }
                            // this column's FMAs complete before the wait for the
                            // next column's weights (which the fetch after next
                            // needs), so that fetch runs under all of them
#pragma unroll
                            for (int q = 0; q < Q; ++q)
#pragma unroll
                                for (int j = 0; j < W; ++j) asm volatile("" ::"v"(acc[s - 1][q][j]));
#pragma unroll
                            for (int e = 0; e < Q; ++e) wcur[e] = wnxt[e];
                            to_vgpr(wcur);
                        }
                    } else {
#pragma unroll
                        for (int bo = -R; bo <= R; ++bo) {
#pragma unroll
                            for (int ao = -R; ao <= R; ++ao) {
                                const int q = ((u - ao + R) % Q + Q) % Q;
                                if constexpr (SHAPE == STENCIL_BOX) {
                                    const TC wv = wk[(ao + R) * (2 * R + 1) + (bo + R)];
#pragma unroll
                                    for (int j = 0; j < W; ++j)
                                        acc[s - 1][q][j] = fma_c(wv, win[j + bo + R], acc[s - 1][q][j]);
                                } else if (ao != 0 && bo == 0) {
                                    const TC wv = wk[star_axis_index<SHAPE, R>(0, ao)];
#pragma unroll
                                    for (int j = 0; j < W; ++j)
                                        acc[s - 1][q][j] = fma_c(wv, win[j + R], acc[s - 1][q][j]);
                                } else if (ao == 0) {
                                    const TC wv = bo == 0 ? wk[0] : wk[star_axis_index<SHAPE, R>(1, bo)];
#pragma unroll
                                    for (int j = 0; j < W; ++j)
                                        acc[s - 1][q][j] = fma_c(wv, win[j + bo + R], acc[s - 1][q][j]);
                                }
                            }
                        }
                    }
                    // the completed row
                    const int yo = ybase + k - s * (1 + R);  // row completed by stage s
#pragma unroll
                    for (int j = 0; j < W; ++j) outv[j] = acc[s - 1][qc][j];
                    if (s < T) {
                        if (!periodic) {
                            const bool row_in = yo >= 0 && yo < n0;
#pragma unroll
                            for (int j = 0; j < W; ++j)
                                if (!(row_in && col_in[j])) outv[j] = h;
                        }
                    } else if (yo >= y0 && yo < y1) {
                        TS *rowp = dst + (int64_t)yo * n1;
                        Vec ov;
#pragma unroll
                        for (int j = 0; j < W; ++j) ov.e[j] = to_storage<TS>(outv[j]);
                        if (st_all) ov.store(rowp + cb);
                        if (st_part_wave && !st_all) {
#pragma unroll
                            for (int j = 0; j < W; ++j)
                                if (col_store[j]) rowp[cb + j] = ov.e[j];
                        }
                    }
                }
#pragma unroll
                for (int j = 0; j < W; ++j) acc[s - 1][qc][j] = TC(0);
                // window of this stage's row for stage s+1 at the next iteration
                if (s < T) assemble_window<TC, W, R>(outv, wins[s], lane);
            }
            // ---- stage 0: input row (window for stage 1), prefetch P rows ahead
            {
                TC inrow[W];
                if constexpr (FAST) {
                    const int i = ybase + k;
                    const bool hrow = f_h || (!periodic && (i < 0 || i >= n0));
#pragma unroll
                    for (int j = 0; j < W; ++j) inrow[j] = hrow ? h : to_compute<TC>(ring[u % P].e[j]);
                } else {
#pragma unroll
                    for (int j = 0; j < W; ++j) inrow[j] = to_compute<TC>(ring[u % P].e[j]);
                }
                // keep the refill of this ring slot behind the reads that drain it
                __builtin_amdgcn_sched_barrier(0);
                if (k + P < KTOT) load_row(k + P, ring[u % P]);
                assemble_window<TC, W, R>(inrow, wins[0], lane);
            }
        }
    }
}

// Load the weights.  Float32 weights go to vector registers: a v_fma_f32 with a
// scalar-register operand measured ~35 % slower on gfx950 than with vector
// operands only (61-68 vs 92-97 TFLOP/s in FMA chains; float64 shows no such
// difference).  Float64 sets up to ~48 dwords stay in scalar registers; larger
// ones (49 float64 box weights) are pinned in vector registers, otherwise the
// compiler spills them to vector lanes and pays a readlane per use.
// The float64 Star-2D7R set (29 weights) stays in scalar registers: pinned in
// vector registers beside its 15 accumulator rows per stage it needs all 256.
template <typename TC, int K, bool SCALAR64 = false, typename SrcT>
__device__ __forceinline__ void load_weights(TC (&wk)[K], const SrcT *w)
{
#pragma unroll
    for (int k = 0; k < K; ++k) {
        wk[k] = w[k];
        if constexpr (sizeof(TC) == 4 || (sizeof(TC) * K > 192 && !SCALAR64)) asm volatile("" : "+v"(wk[k]));
    }
}

// Whether a job's tiles take the fast row loads (see valu2d_tile).
template <typename TS, int W, typename TC>
__device__ __forceinline__ bool valu2d_fast(const Valu2DJob<TC> &g)
{
    return vec_aligned<TS, W>(g.src, g.n1, 0) && (g.ox0 % W) == 0;
}

template <typename TS, typename TC, int SHAPE, int R, int T, int W>
__global__ __launch_bounds__(64 * kValu2DWaves) void valu2d_kernel(
    Valu2DArgs<TC, Valu2DCfg<TS, TC, SHAPE, R, T, W>::K> a)
{
    using Cfg = Valu2DCfg<TS, TC, SHAPE, R, T, W>;
    // The waves of a workgroup take adjacent bands of one row segment (their
    // skirt columns are read together); XCD-aware order: the workgroups
    // resident on one XCD take consecutive segments of a band group (which
    // share halo rows in that XCD's L2).
    const int g = xcd_remap(blockIdx.x, gridDim.x);
    if (g >= a.g.nwg) return;
    const int band = (g / a.g.nsegs) * kValu2DWaves + (int)(threadIdx.x >> 6);
    if (band >= a.g.nbands) return;
    TC wk[Cfg::WPTR ? 1 : Cfg::K];
    ConstPtr<TC> wp = nullptr;
    if constexpr (Cfg::WPTR) {
        // the argument block is the first entry of the kernel-argument segment
        using Args = Valu2DArgs<TC, Cfg::K>;
        wp = (ConstPtr<TC>)((const __attribute__((address_space(4))) char *)
                                __builtin_amdgcn_kernarg_segment_ptr() +
                            offsetof(Args, w));
        wk[0] = TC(0);
    } else {
        load_weights<TC, Cfg::K, SHAPE == STENCIL_STAR && R == 7>(wk, a.w);
    }
    if (valu2d_fast<TS, W>(a.g))
        valu2d_tile<TS, TC, SHAPE, R, T, W, true>(a.g, wk, wp, band, g % a.g.nsegs, threadIdx.x & 63);
    else
        valu2d_tile<TS, TC, SHAPE, R, T, W, false>(a.g, wk, wp, band, g % a.g.nsegs, threadIdx.x & 63);
}

// One job of a batched launch: geometry plus weights.
template <typename TC, int K>
struct Valu2DBatchJob {
    Valu2DJob<TC> g;
    TC w[K];
};

// Persistent batched launch: the workgroups walk one list of (job, band
// group x segment) items spanning every job of the batch (jobs of uneven
// sizes); workgroup b takes items b + i*gridDim.  tile_start[j] is the first
// item of job j (tile_start[njobs] = total).
template <typename TS, typename TC, int SHAPE, int R, int T, int W>
__global__ __launch_bounds__(64 * kValu2DWaves) void valu2d_batch_kernel(
    const Valu2DBatchJob<TC, Valu2DCfg<TS, TC, SHAPE, R, T, W>::K> *jobs,
    const int *tile_start, int njobs)
{
    using Cfg = Valu2DCfg<TS, TC, SHAPE, R, T, W>;
    const int total = tile_start[njobs];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    int j = 0;
    for (int item = xcd_remap(blockIdx.x, gridDim.x); item < total; item += gridDim.x) {
        while (j + 1 < njobs && tile_start[j + 1] <= item) ++j;
        const Valu2DJob<TC> g = jobs[j].g;
        const int local = item - tile_start[j];
        const int band = (local / g.nsegs) * kValu2DWaves + wave;
        if (band >= g.nbands) continue;
        TC wk[Cfg::WPTR ? 1 : Cfg::K];
        ConstPtr<TC> wp = nullptr;
        if constexpr (Cfg::WPTR) {
            wp = (ConstPtr<TC>)(jobs[j].w);  // the job table is read-only in the kernel
            wk[0] = TC(0);
        } else {
            load_weights<TC, Cfg::K, SHAPE == STENCIL_STAR && R == 7>(wk, jobs[j].w);
        }
        if (valu2d_fast<TS, W>(g))
            valu2d_tile<TS, TC, SHAPE, R, T, W, true>(g, wk, wp, band, local % g.nsegs, lane);
        else
            valu2d_tile<TS, TC, SHAPE, R, T, W, false>(g, wk, wp, band, local % g.nsegs, lane);
    }
}

// Columns per lane: one 16-byte vector, except float64 at T = 2, which takes
// two (256-column bands: the 2E-column skirt is half the share of the band;
// Box-2D3R 8192^2: 368 vs 345 GSt/s, Star-2D3R: 580 vs 528).  At T = 1 and
// T >= 3 the 2-column lanes measured faster (occupancy), except for the
// compute-bound float64 r = 7 passes, whose 8-column skirt is then half the
// share of the band (10240^2 T = 1: Star-2D7R 260 -> 297, Box-2D7R 95 -> 101
// GSt/s; memory-bound r <= 3 one-step passes 3-10 % slower with 4 columns).
template <typename TS, int R, int T>
struct Valu2DShape {
    static constexpr int W = (sizeof(TS) == 8 && (T == 2 || (T == 1 && R >= 7)))
                                 ? 4
                                 : (16 / sizeof(TS) > 8 ? 8 : 16 / sizeof(TS));
};

// Fill the geometry of one pass; returns false when there is nothing to do.
template <typename TS, typename TC, int SHAPE, int R, int T>
bool valu2d_geometry(const PassArgs &p, Valu2DJob<TC> *g, hipError_t *err)
{
    using S = Valu2DShape<TS, R, T>;
    using Cfg = Valu2DCfg<TS, TC, SHAPE, R, T, S::W>;
    *err = hipSuccess;
    g->src = p.src;
    g->dst = p.dst;
    g->n0 = (int)p.dims[0];
    g->n1 = (int)p.dims[1];
    g->oy0 = p.region_lo[0];
    g->oy1 = p.region_hi[0];
    g->ox0 = p.region_lo[1];
    g->ox1 = p.region_hi[1];
    g->periodic = p.boundary == STENCIL_PERIODIC;
    g->h = (TC)p.halo;
    g->BX = Cfg::NCW - 2 * Cfg::E;
    if (g->BX <= 0) {
        *err = hipErrorInvalidValue;
        return false;
    }
    const int W_out = g->ox1 - g->ox0, H_out = g->oy1 - g->oy0;
    if (W_out <= 0 || H_out <= 0) return false;
    g->nbands = (W_out + g->BX - 1) / g->BX;
    // rows per wave: the wave count is a whole number of waves of the resident
    // slots (waves per CU x CUs), as few rounds as keep segments long enough to
    // amortise the 2rT + T pipeline rows
    int BY = p.tile_rows;
    if (BY <= 0) {
        const int slots = (p.num_cu > 0 ? p.num_cu : 256) * (p.slots_per_cu > 0 ? p.slots_per_cu : 8);
        const int minBY = 16 * (2 * R * T + T) > 64 ? 16 * (2 * R * T + T) : 64;
        const int groups = (g->nbands + kValu2DWaves - 1) / kValu2DWaves;
        int segs = 1;
        for (int rounds = 1; rounds <= 64; ++rounds) {
            segs = (rounds * slots) / (groups * kValu2DWaves);
            if (segs < 1) segs = 1;
            if ((H_out + segs - 1) / segs <= 4 * minBY) break;
        }
        BY = (H_out + segs - 1) / segs;
        if (BY < 16) BY = 16;
    }
    g->BY = BY;
    g->nsegs = (H_out + BY - 1) / BY;
    g->nwg = ((g->nbands + kValu2DWaves - 1) / kValu2DWaves) * g->nsegs;
    return true;
}

template <typename TS, typename TC, int SHAPE, int R, int T>
hipError_t launch_valu2d(const PassArgs &p, hipStream_t stream)
{
    using S = Valu2DShape<TS, R, T>;
    using Cfg = Valu2DCfg<TS, TC, SHAPE, R, T, S::W>;
    Valu2DArgs<TC, Cfg::K> a;
    hipError_t err;
    static const int occ = [] {  // resident waves per CU of this instance
        int o = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&o, valu2d_kernel<TS, TC, SHAPE, R, T, S::W>,
                                                         64 * kValu2DWaves, 0) != hipSuccess || o < 1)
            o = 2;
        return o * kValu2DWaves;
    }();
    PassArgs q = p;
    q.slots_per_cu = occ;
    if (!valu2d_geometry<TS, TC, SHAPE, R, T>(q, &a.g, &err)) return err;
    for (int k = 0; k < Cfg::K; ++k) a.w[weight_slot<Cfg, R>(k)] = (TC)p.w[k];
    const int grid = a.g.nwg;
    hipLaunchKernelGGL((valu2d_kernel<TS, TC, SHAPE, R, T, S::W>), dim3(grid), dim3(64 * kValu2DWaves), 0,
                       stream, a);
    return hipGetLastError();
}

// Batched form: n passes (one per job) of the same variant in one launch.
template <typename TS, typename TC, int SHAPE, int R, int T>
hipError_t launch_valu2d_batch(const PassArgs *ps, int n, BatchStaging *stage, hipStream_t stream)
{
    using S = Valu2DShape<TS, R, T>;
    using Cfg = Valu2DCfg<TS, TC, SHAPE, R, T, S::W>;
    using Job = Valu2DBatchJob<TC, Cfg::K>;
    std::vector<Job> jobs;
    std::vector<int> start(1, 0);
    jobs.reserve(n);
    for (int i = 0; i < n; ++i) {
        Job j;
        hipError_t err;
        if (!valu2d_geometry<TS, TC, SHAPE, R, T>(ps[i], &j.g, &err)) {
            if (err != hipSuccess) return err;
            continue;
        }
        for (int k = 0; k < Cfg::K; ++k) j.w[weight_slot<Cfg, R>(k)] = (TC)ps[i].w[k];
        jobs.push_back(j);
        start.push_back(start.back() + j.g.nwg);
    }
    if (jobs.empty()) return hipSuccess;
    const int nj = (int)jobs.size();
    void *djobs = nullptr, *dstart = nullptr;
    hipError_t e = stage_job_table(stage, jobs.data(), jobs.size() * sizeof(Job), start, &djobs, &dstart, stream);
    if (e != hipSuccess) return e;
    const int total_wg = start.back();
    int occ = 0;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &occ, valu2d_batch_kernel<TS, TC, SHAPE, R, T, S::W>, 64 * kValu2DWaves, 0);
    if (e != hipSuccess || occ < 1) occ = 1;
    const int slots = occ * (ps[0].num_cu > 0 ? ps[0].num_cu : 256);
    const int grid = total_wg < slots ? total_wg : slots;
    hipLaunchKernelGGL((valu2d_batch_kernel<TS, TC, SHAPE, R, T, S::W>), dim3(grid),
                       dim3(64 * kValu2DWaves), 0, stream, static_cast<const Job *>(djobs),
                       static_cast<const int *>(dstart), nj);
    return hipGetLastError();
}

#define V2(TS, TC, DT, SH, R, T) \
    {STENCIL_PATH_VALU, DT, SH, 2, R, T, &launch_valu2d<TS, TC, SH, R, T>, \
     &launch_valu2d_batch<TS, TC, SH, R, T>}
#define V2_T(TS, TC, DT, SH, R) \
    V2(TS, TC, DT, SH, R, 1), V2(TS, TC, DT, SH, R, 2), V2(TS, TC, DT, SH, R, 3), V2(TS, TC, DT, SH, R, 4)
#define V2_R(TS, TC, DT, SH) V2_T(TS, TC, DT, SH, 1), V2_T(TS, TC, DT, SH, 2), V2_T(TS, TC, DT, SH, 3)
#define V2_S(TS, TC, DT) V2_R(TS, TC, DT, STENCIL_STAR), V2_R(TS, TC, DT, STENCIL_BOX)

}  // namespace stl
