// MFMA path, d = 2: the T-step composite kernel applied once per pass as
// banded Toeplitz products on the matrix cores (kernel fusion; paper, Sec.
// "Tensor Core Implementation with Kernel Fusion": executed work (alpha/S)
// t C, memory traffic unchanged).
//
// Workgroup: NW waves side by side; wave w owns V stacked 16 x 16 output
// tiles (16V rows x 16 columns).  The input block the workgroup needs
// ((16V + 2R) x (16 NW + 2R) points, halo included, boundary rule applied) is
// staged once in LDS in the operand type.  For every kernel column b the wave
// loads that column's A fragments (lane-ordered on the host, L2-resident; the
// 16-bit kernels copy the whole fragment table to LDS with the input block
// when it fits in 24 KiB) and issues one MFMA per (tile, structurally non-zero
// k-block).  With KDIM = 4
// (f64/f32) a B fragment of rows 4q..4q+3 serves every stacked tile whose
// k-block lands on it.  With KDIM = 32 (bf16/f16) the LDS block is stored
// column-major so each lane's 8 consecutive rows are one 16-byte read.
//
// Compensated mode (float32 storage): data split x = x_hi + x_lo and weights
// w = w_hi + w_lo into bf16; three products hi*hi + hi*lo + lo*hi per term,
// accumulated in float32.
#pragma once

#include <type_traits>

#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include "internal.h"
#include "mfma_layout.h"
#include "valu_common.h"

namespace stl {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef _Float16 v8h __attribute__((ext_vector_type(8)));

template <int DT>
struct MfmaTypes;
template <>
struct MfmaTypes<STENCIL_F64> {
    using TS = double;   // storage
    using OP = double;   // operand element
    using FR = double;   // operand fragment (per lane)
    using ACC = v4d;
    static constexpr int KDIM = 4;
    static constexpr bool X3 = false;
    // f64 16x16x4: register e of lane l holds D[4e + l/16][l % 16]
    static constexpr bool D_ROW_INTERLEAVED = true;
};
template <>
struct MfmaTypes<STENCIL_F32> {
    using TS = float;
    using OP = float;
    using FR = float;
    using ACC = v4f;
    static constexpr int KDIM = 4;
    static constexpr bool X3 = false;
    // register e of lane l holds D[4 (l/16) + e][l % 16]
    static constexpr bool D_ROW_INTERLEAVED = false;
};
template <>
struct MfmaTypes<STENCIL_BF16> {
    using TS = __hip_bfloat16;
    using OP = __bf16;
    using FR = v8bf;
    using ACC = v4f;
    static constexpr int KDIM = 32;
    static constexpr bool X3 = false;
    // register e of lane l holds D[4 (l/16) + e][l % 16]
    static constexpr bool D_ROW_INTERLEAVED = false;
};
template <>
struct MfmaTypes<STENCIL_F16> {
    using TS = __half;
    using OP = _Float16;
    using FR = v8h;
    using ACC = v4f;
    static constexpr int KDIM = 32;
    static constexpr bool X3 = false;
    // register e of lane l holds D[4 (l/16) + e][l % 16]
    static constexpr bool D_ROW_INTERLEAVED = false;
};
template <>
struct MfmaTypes<STENCIL_F32_BF16X3> {
    using TS = float;
    using OP = __bf16;
    using FR = v8bf;
    using ACC = v4f;
    static constexpr int KDIM = 32;
    static constexpr bool X3 = true;
    // register e of lane l holds D[4 (l/16) + e][l % 16]
    static constexpr bool D_ROW_INTERLEAVED = false;
};

__device__ __forceinline__ v4d mfma16(double a, double b, v4d c)
{
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ v4f mfma16(float a, float b, v4f c)
{
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ v4f mfma16(v8bf a, v8bf b, v4f c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ v4f mfma16(v8h a, v8h b, v4f c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
}

typedef __bf16 v16bf __attribute__((ext_vector_type(16)));
typedef _Float16 v16h __attribute__((ext_vector_type(16)));

// 2:4 structured-sparse 16x16x64: `a` holds two of every four k positions of
// lane l's row (positions in `idx`, 2 bits each), `b` 16 dense k values.
__device__ __forceinline__ v4f smfma16(v8bf a, v16bf b, v4f c, int idx)
{
    return __builtin_amdgcn_smfmac_f32_16x16x64_bf16(a, b, c, idx, 0, 0);
}
__device__ __forceinline__ v4f smfma16(v8h a, v16h b, v4f c, int idx)
{
    return __builtin_amdgcn_smfmac_f32_16x16x64_f16(a, b, c, idx, 0, 0);
}
template <typename FR>
using SparseB = typename std::conditional<std::is_same<FR, v8bf>::value, v16bf, v16h>::type;

// storage value -> compute float/double
template <typename TS>
__device__ __forceinline__ auto load_val(TS v)
{
    if constexpr (sizeof(TS) == 2) return to_compute<float>(v);
    else return v;
}

template <typename OP, typename X>
__device__ __forceinline__ OP to_op(X v)
{
    if constexpr (sizeof(OP) == 2) return (OP)(float)v;  // round to nearest even
    else return (OP)v;
}

struct Mfma2DArgs {
    const void *src;
    void *dst;
    const void *afrag;
    const void *afrag_lo;
    int n0, n1;
    int ntr, ntc, ntiles;
    int periodic;
    double h;
};

template <int DT, int SHAPE, int r, int T, int V, int NW, bool SP = false>
struct Mfma2DCfg {
    using MT = MfmaTypes<DT>;
    static constexpr int KDIM = MT::KDIM;
    static constexpr int KPL = KDIM / 4;
    static constexpr int R = r * T;
    static constexpr int TR = 16 * V;          // output rows per workgroup
    static constexpr int TCOL = 16 * NW;       // output columns per workgroup
    static constexpr int LRD = TR + 2 * R;     // data rows staged
    static constexpr int LC = TCOL + 2 * R;    // data columns staged
    static constexpr int KKH = band_kk_hi(SHAPE, r, T, 0, 0, KDIM);
    static constexpr int LRK = 16 * (V - 1) + KDIM * (KKH + 1);  // rows an operand may touch
    static constexpr int LR0 = LRD > LRK ? LRD : LRK;
    // column-major blocks (16-bit operands): the column pitch in 16-byte
    // units is 2 mod 4 for the dense kernels and odd for the 2:4 sparse one
    // (measured against the other parity: compensated bf16x3 Box-2D2R T = 4
    // 16384^2 1186 -> 1229, bf16 Box-2D3R T = 4 8192^2 1390 -> 1443 GSt/s;
    // the sparse kernel 23-32 % slower with 2 mod 4)
    static constexpr int LR8 = ((LR0 + 7) / 8) * 8;
    static constexpr int LR = KDIM == 4 ? LR8
                              : SP      ? LR8 + ((LR8 / 8) % 2 == 0 ? 8 : 0)
                                        : LR8 + 8 * ((2 - (LR8 / 8) % 4 + 4) % 4);
    // row-major pitch (KDIM = 4) padded off multiples of the bank count
    static constexpr int LCP = LC + ((LC % 32) == 0 ? 1 : 0);
    static constexpr int LDS_ELEMS = KDIM == 4 ? LR * LCP : LC * LR;
};

// Non-empty kernel columns of the composite, in order, and the depth of the
// A-fragment prefetch of the float64/float32 kernels: operand fragments of
// the next PF columns are in flight while a column's MFMAs run, within a
// register budget of 64 VGPRs.  The 16-bit kernels load a column's fragments
// at the column (measured faster: they need the occupancy more).
template <int SHAPE, int r, int T, int KDIM, int FRW>
struct BandCols {
    static constexpr int R = r * T;
    static constexpr int count()
    {
        int n = 0;
        for (int b = -R; b <= R; ++b) n += band_amax(SHAPE, r, T, 0, b) >= 0;
        return n;
    }
    static constexpr int col(int j)
    {
        int n = 0;
        for (int b = -R; b <= R; ++b)
            if (band_amax(SHAPE, r, T, 0, b) >= 0) {
                if (n == j) return b;
                ++n;
            }
        return 0;
    }
    static constexpr int N = count();
    static constexpr int NB = band_nblk(SHAPE, r, T, 0, 0, KDIM);  // k-blocks of the widest column
    static constexpr int PF0 = 64 / (NB * FRW);
    static constexpr int PF = PF0 < 2 ? 2 : (PF0 > N ? N : PF0);
};

// One 16V x 16NW output tile of one pass, run by the whole workgroup.  SP:
// 2:4 structured-sparse instructions, one per pair of kernel columns (16-bit
// operands, composite radius <= 7; layout in mfma_layout.h).
template <int DT, int SHAPE, int r, int T, int V, int NW, bool SP = false>
__device__ __forceinline__ void mfma2d_tile(const Mfma2DArgs &a, const int tile)
{
    using Cfg = Mfma2DCfg<DT, SHAPE, r, T, V, NW, SP>;
    using MT = typename Cfg::MT;
    using TS = typename MT::TS;
    using OP = typename MT::OP;
    using FR = typename MT::FR;
    using ACC = typename MT::ACC;
    constexpr int KDIM = Cfg::KDIM, R = Cfg::R;
    constexpr int LR = Cfg::LR, LRD = Cfg::LRD, LC = Cfg::LC, LCP = Cfg::LCP;
    constexpr int NT = 64 * NW;
    constexpr bool X3 = MT::X3;

    __shared__ __attribute__((aligned(16))) OP lhi[Cfg::LDS_ELEMS];
    __shared__ __attribute__((aligned(16))) OP llo[X3 ? Cfg::LDS_ELEMS : 1];
    // 16-bit operands: the whole A fragment table (NFRAG fragments of 64
    // lanes) is copied to LDS with the input block when it fits in 24 KiB,
    // so the column loop reads A from LDS instead of from L2
    constexpr int NFRAG = band_total_frags(SHAPE, r, T, KDIM, 2);
    constexpr int NAF = NFRAG * (X3 ? 2 : 1);
    constexpr bool ALDS = KDIM != 4 && NAF <= 24 && !SP;
    static_assert(!SP || (KDIM == 32 && !X3 && R <= sparse_max_radius()), "sparse layout: 16-bit, R <= 7");
    using FRS = typename MT::FR;
    __shared__ __attribute__((aligned(16))) FRS lA[ALDS ? NAF * 64 : 1];

    const int tid = threadIdx.x;
    const int tr = tile / a.ntc, tcn = tile - tr * a.ntc;
    const int r0 = tr * Cfg::TR, c0 = tcn * Cfg::TCOL;
    const int n0 = a.n0, n1 = a.n1;
    const bool periodic = a.periodic != 0;
    const TS *src = static_cast<const TS *>(a.src);

    // ---- A fragments of the first PF columns: in flight during the staging
    const int lane = tid & 63, wave = tid >> 6;
    const FR *afr = static_cast<const FR *>(a.afrag);
    const FR *afr_lo = static_cast<const FR *>(a.afrag_lo);
    using Cols = BandCols<SHAPE, r, T, KDIM, (sizeof(FR) + 3) / 4 * (X3 ? 2 : 1)>;
    constexpr int NBMAX = Cols::NB, PF = KDIM == 4 ? Cols::PF : 1;
    FR Ar[PF][NBMAX], Alr[X3 ? PF : 1][X3 ? NBMAX : 1];
    auto load_col = [&](int j, int slot) {
        const int b = Cols::col(j);
        const int klo = band_kk_lo(SHAPE, r, T, 0, b, KDIM);
        const int khi = band_kk_hi(SHAPE, r, T, 0, b, KDIM);
        const int off = band_frag_offset(SHAPE, r, T, 0, b, KDIM, 2);
#pragma unroll
        for (int i = 0; i < NBMAX; ++i)
            if (i <= khi - klo) {
                if constexpr (ALDS) {
                    Ar[slot][i] = lA[(off + i) * 64 + lane];
                    if constexpr (X3) Alr[slot][i] = lA[(NFRAG + off + i) * 64 + lane];
                } else {
                    Ar[slot][i] = afr[(off + i) * 64 + lane];
                    if constexpr (X3) Alr[slot][i] = afr_lo[(off + i) * 64 + lane];
                }
            }
    };
    if constexpr (KDIM == 4)
#pragma unroll
        for (int j = 0; j < PF; ++j) load_col(j, j);
    // sparse: compressed weights and positions of every column pair, in
    // flight during the staging (at most 8 pairs: 40 VGPRs)
    constexpr int NP = SP ? sparse_pairs(SHAPE, r, T) : 1;
    FR Asp[NP];
    int Isp[NP];
    if constexpr (SP) {
        const int *aidx = reinterpret_cast<const int *>(afr + NP * 64);
#pragma unroll
        for (int pi = 0; pi < NP; ++pi) {
            Asp[pi] = afr[pi * 64 + lane];
            Isp[pi] = aidx[pi * 64 + lane];
        }
    }
    // A table for the LDS copy: loads in flight during the staging
    constexpr int NAT = ALDS ? (NAF * 64 + NT - 1) / NT : 1;
    FR ta[NAT];
    if constexpr (ALDS) {
#pragma unroll
        for (int i = 0; i < NAT; ++i) {
            const int e = tid + i * NT;
            if (e < NAF * 64) ta[i] = e < NFRAG * 64 ? afr[e] : afr_lo[e - NFRAG * 64];
        }
    }

    // ---- 16-bit operands (bf16/f16 storage, or float storage split into
    // bf16 hi/lo), interior tile: rows are read in aligned chunks of four
    // elements (one 8- or 16-byte load each) and scattered into the
    // column-major block; one wait per batch of chunks.
    bool staged = false;
    if constexpr (KDIM != 4) {
        using Chunk = typename std::conditional<sizeof(TS) == 2, uint2, uint4>::type;
        constexpr int NCH = (LC + 3 + 3) / 4;  // chunks per row (start aligned down by up to 3)
        // Chunk-to-lane map.  Row-major (lanes on consecutive chunks of a row:
        // one contiguous segment per load) makes the column-major LDS writes
        // of one instruction land 4 columns apart, on a few banks (measured:
        // 69 % of LDS cycles in bank conflicts, Box-2D2R bf16 T = 4).  Blocks
        // of 16 rows x 4 chunks (lane = row + 16 chunk) write 16 consecutive
        // rows of 4 columns whose pitch is an odd number of 16-byte units:
        // disjoint bank groups.  Measured on 16384^2: blocks are faster for
        // the compensated split (two blocks written, +7-19 %) and for
        // composite radii R >= 6 (+5-10 %); row-major is faster below
        // (up to 15 % at T = 1), where staging latency rather than LDS
        // throughput dominates.
        constexpr bool SBLK = X3 || R >= 6;
        constexpr int NRB = (LRD + 15) / 16, NCB = (NCH + 3) / 4, NBLK = NRB * NCB;
        constexpr int NE4 = SBLK ? (NBLK + NW - 1) / NW : (LRD * NCH + NT - 1) / NT;  // chunks per thread
        constexpr int CB = NE4 < 8 ? NE4 : 8;
        const int swv = tid >> 6, srr = tid & 15, scc = (tid >> 4) & 3;
        auto chunk_at = [&](int it, int &row, int &ch) {
            if constexpr (SBLK) {
                const int blk = swv + NW * it;
                const int rb = blk % NRB, cb = blk / NRB;
                row = 16 * rb + srr;
                ch = 4 * cb + scc;
                return it < NE4 && blk < NBLK && row < LRD && ch < NCH;
            } else {
                const int e = tid + it * NT;
                row = e / NCH;
                ch = e - row * NCH;
                return it < NE4 && e < LRD * NCH;
            }
        };
        const int cs = (c0 - R) & ~3;
        const int lead = (c0 - R) - cs;
        const bool fast = r0 - R >= 0 && r0 - R + LRD <= n0 && c0 - R >= 0 && cs + 4 * NCH <= n1 &&
                          (n1 % 4) == 0 && (reinterpret_cast<uintptr_t>(src) % sizeof(Chunk)) == 0;
        if (fast) {
            uint16_t *l16 = reinterpret_cast<uint16_t *>(lhi);
            uint16_t *l16lo = reinterpret_cast<uint16_t *>(llo);
#pragma unroll
            for (int e0 = 0; e0 < NE4; e0 += CB) {
                Chunk v[CB];
#pragma unroll
                for (int i = 0; i < CB; ++i) {
                    int row, ch;
                    if (chunk_at(e0 + i, row, ch))
                        v[i] = *reinterpret_cast<const Chunk *>(src + (int64_t)(r0 - R + row) * n1 + cs + 4 * ch);
                }
#pragma unroll
                for (int i = 0; i < CB; ++i) {
                    int row, ch;
                    if (!chunk_at(e0 + i, row, ch)) continue;
                    uint16_t hi4[4], lo4[4];
                    if constexpr (sizeof(TS) == 2) {
                        hi4[0] = (uint16_t)(v[i].x & 0xffff);
                        hi4[1] = (uint16_t)(v[i].x >> 16);
                        hi4[2] = (uint16_t)(v[i].y & 0xffff);
                        hi4[3] = (uint16_t)(v[i].y >> 16);
                    } else {  // compensated: x = hi + lo in bf16, hi rounded to nearest even
                        const uint32_t u[4] = {v[i].x, v[i].y, v[i].z, v[i].w};
#pragma unroll
                        for (int j = 0; j < 4; ++j) {
                            const float f = __uint_as_float(u[j]);
                            const OP h = (OP)f;
                            const OP l = (OP)(f - (float)h);
                            hi4[j] = __builtin_bit_cast(uint16_t, h);
                            lo4[j] = __builtin_bit_cast(uint16_t, l);
                        }
                    }
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        const int col = 4 * ch + j - lead;
                        if (col >= 0 && col < LC) {
                            l16[col * LR + row] = hi4[j];
                            if constexpr (X3) l16lo[col * LR + row] = lo4[j];
                        }
                    }
                }
            }
            // rows past the data rows: zeros for the last k-blocks
            for (int e = tid; e < (LR - LRD) * LC; e += NT) {
                const int row = LRD + e / LC, col = e - (e / LC) * LC;
                l16[col * LR + row] = 0;
                if constexpr (X3) l16lo[col * LR + row] = 0;
            }
            staged = true;
        }
    }
    // ---- float64/float32 operands, interior tile: rows are read in aligned
    // 16-byte chunks (2 or 4 elements) and written to the row-major block.
    if constexpr (KDIM == 4) {
        constexpr int EPC = 16 / (int)sizeof(TS);       // elements per chunk
        constexpr int NCH = (LC + 2 * (EPC - 1)) / EPC;  // chunks per row (start aligned down)
        constexpr int NE4 = (LRD * NCH + NT - 1) / NT;
        constexpr int CB = NE4 < 8 ? NE4 : 8;
        const int cs = (c0 - R) & ~(EPC - 1);
        const int lead = (c0 - R) - cs;
        const bool fast = r0 - R >= 0 && r0 - R + LRD <= n0 && c0 - R >= 0 && cs + EPC * NCH <= n1 &&
                          (n1 % EPC) == 0 && (reinterpret_cast<uintptr_t>(src) % 16) == 0;
        if (fast) {
#pragma unroll
            for (int e0 = 0; e0 < NE4; e0 += CB) {
                RawVec<TS, EPC> v[CB];
#pragma unroll
                for (int i = 0; i < CB; ++i) {
                    const int e = tid + (e0 + i) * NT;
                    const int row = e / NCH, ch = e - (e / NCH) * NCH;
                    if (e0 + i < NE4 && e < LRD * NCH)
                        v[i].load(src + (int64_t)(r0 - R + row) * n1 + cs + EPC * ch);
                }
#pragma unroll
                for (int i = 0; i < CB; ++i) {
                    const int e = tid + (e0 + i) * NT;
                    if (e0 + i >= NE4 || e >= LRD * NCH) break;
                    const int row = e / NCH, ch = e - (e / NCH) * NCH;
#pragma unroll
                    for (int j = 0; j < EPC; ++j) {
                        const int col = EPC * ch + j - lead;
                        if (col >= 0 && col < LC) lhi[row * LCP + col] = (OP)v[i].e[j];
                    }
                }
            }
            // rows past the data rows: zeros for the last k-blocks
            for (int e = tid; e < (LR - LRD) * LC; e += NT) {
                const int row = LRD + e / LC, col = e - (e / LC) * LC;
                lhi[row * LCP + col] = OP(0);
            }
            staged = true;
        }
    }
    if (!staged) {
        // ---- stage the input block (boundary rule applied) in LDS.  A thread's
        // loads are issued in batches of CH before the batch's LDS writes (one
        // wait per batch rather than one memory latency per element): the whole
        // block for 32/64-bit data; 8 elements for 16-bit data, whose kernels
        // need the occupancy more than the fewer waits.
        constexpr int NE = (LR * LC + NT - 1) / NT;  // elements per thread
        constexpr int CH = sizeof(TS) == 2 ? (NE < 8 ? NE : 8) : NE;
        using SV = decltype(load_val(TS{}));
#pragma unroll
        for (int c0e = 0; c0e < NE; c0e += CH) {
            SV vals[CH];
#pragma unroll
            for (int i = 0; i < CH; ++i) {
                const int idx = tid + (c0e + i) * NT;
                const int row = idx / LC, col = idx - (idx / LC) * LC;
                vals[i] = SV(a.h);
                if (c0e + i < NE && idx < LR * LC && row < LRD) {
                    int gr = r0 - R + row, gc = c0 - R + col;
                    const bool in = gr >= 0 && gr < n0 && gc >= 0 && gc < n1;
                    // points past n + R only feed outputs of a partial tile that
                    // are not stored; the rest lie in [-R, n + R), where one fold
                    // wraps (periodic plans have every dim >= 2R + 1)
                    const bool used = gr < n0 + R && gc < n1 + R;
                    if (in || (periodic && used)) {
                        gr = wrap1(gr, n0);
                        gc = wrap1(gc, n1);
                        vals[i] = load_val(src[(int64_t)gr * n1 + gc]);
                    }
                } else {
                    vals[i] = SV(0);  // rows past the data rows: zeros for the last k-blocks
                }
            }
#pragma unroll
            for (int i = 0; i < CH; ++i) {
                const int idx = tid + (c0e + i) * NT;
                if (c0e + i >= NE || idx >= LR * LC) break;
                const int row = idx / LC, col = idx - (idx / LC) * LC;
                const int li = KDIM == 4 ? row * LCP + col : col * LR + row;
                if constexpr (sizeof(OP) == 8 || sizeof(OP) == 4) {
                    lhi[li] = (OP)vals[i];
                } else if constexpr (X3) {
                    const float vf = (float)vals[i];
                    const OP hi = (OP)vf;
                    lhi[li] = hi;
                    llo[li] = (OP)(vf - (float)hi);
                } else {
                    lhi[li] = (OP)(float)vals[i];
                }
            }
        }
    }
    if constexpr (ALDS) {
#pragma unroll
        for (int i = 0; i < NAT; ++i) {
            const int e = tid + i * NT;
            if (e < NAF * 64) lA[e] = ta[i];
        }
    }
    __syncthreads();

    const int lg = lane >> 4, ln = lane & 15;
    const int wc0 = 16 * wave;
    ACC acc[V];
#pragma unroll
    for (int v = 0; v < V; ++v) acc[v] = ACC{};

    if constexpr (SP) {
        // pair (b0, b1): lane (lg, ln) supplies rows 4lg..4lg+3 and
        // 4lg+16..4lg+19 of both columns' 32-row blocks, interleaved two rows
        // at a time: k positions 8lg..8lg+7 (column b0) and 32+8lg..32+8lg+7
        // (column b1) of the instruction's dense k
#pragma unroll
        for (int pi = 0; pi < NP; ++pi) {
            const int b0 = Cols::col(2 * pi);
            const int b1 = 2 * pi + 1 < Cols::N ? Cols::col(2 * pi + 1) : b0;
            const int col0 = wc0 + ln + b0 + R, col1 = wc0 + ln + b1 + R;
#pragma unroll
            for (int v = 0; v < V; ++v) {
                const int row = 16 * v + 4 * lg;
                const uint2 x0 = *reinterpret_cast<const uint2 *>(&lhi[col0 * LR + row]);
                const uint2 x1 = *reinterpret_cast<const uint2 *>(&lhi[col0 * LR + row + 16]);
                const uint2 y0 = *reinterpret_cast<const uint2 *>(&lhi[col1 * LR + row]);
                const uint2 y1 = *reinterpret_cast<const uint2 *>(&lhi[col1 * LR + row + 16]);
                typedef unsigned v8u __attribute__((ext_vector_type(8)));
                const v8u Bw = {x0.x, x1.x, x0.y, x1.y, y0.x, y1.x, y0.y, y1.y};
                acc[v] = smfma16(Asp[pi], __builtin_bit_cast(SparseB<FR>, Bw), acc[v], Isp[pi]);
            }
        }
    }
#pragma unroll
    for (int j = 0; j < (SP ? 0 : Cols::N); ++j) {
        const int b = Cols::col(j);
        const int klo = band_kk_lo(SHAPE, r, T, 0, b, KDIM);
        const int khi = band_kk_hi(SHAPE, r, T, 0, b, KDIM);
        const int slot = j % PF;
        if constexpr (KDIM != 4) load_col(j, 0);
        const FR(&A)[NBMAX] = Ar[slot];
        const int col = wc0 + ln + b + R;
        if constexpr (KDIM == 4) {
#pragma unroll
            for (int q = 0; q < NBMAX + 4 * (V - 1) + 4; ++q) {
                const int qq = klo + q;
                if (qq > khi + 4 * (V - 1)) break;
                const FR B = lhi[(4 * qq + lg) * LCP + col];
#pragma unroll
                for (int v = 0; v < V; ++v) {
                    const int kk = qq - 4 * v;
                    if (kk >= klo && kk <= khi) acc[v] = mfma16(A[kk - klo], B, acc[v]);
                }
            }
        } else {
#pragma unroll
            for (int v = 0; v < V; ++v)
#pragma unroll
                for (int i = 0; i < NBMAX; ++i) {
                    if (i > khi - klo) break;
                    const int row = 16 * v + KDIM * (klo + i) + 8 * lg;
                    const FR B = *reinterpret_cast<const FR *>(&lhi[col * LR + row]);
                    acc[v] = mfma16(A[i], B, acc[v]);
                    if constexpr (X3) {
                        const FR Bl = *reinterpret_cast<const FR *>(&llo[col * LR + row]);
                        acc[v] = mfma16(A[i], Bl, acc[v]);
                        acc[v] = mfma16(Alr[slot][i], B, acc[v]);
                    }
                }
        }
        if constexpr (KDIM == 4)
            if (j + PF < Cols::N) load_col(j + PF, slot);  // refill the slot just used
    }

    // ---- store the stacked tiles (output register layout per instruction)
    TS *dst = static_cast<TS *>(a.dst);
    const int gc = c0 + wc0 + ln;
    if (gc < n1) {
#pragma unroll
        for (int v = 0; v < V; ++v)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int gr = r0 + 16 * v + (MT::D_ROW_INTERLEAVED ? 4 * e + lg : 4 * lg + e);
                if (gr < n0) dst[(int64_t)gr * n1 + gc] = to_storage<TS>(acc[v][e]);
            }
    }
}

// 16-bit operands, row layout (mfma_layout.h): 16V x 16NW output tiles.
// The input block is staged row-major (16-byte loads and LDS writes, no
// transposition); for every composite row a and k-block the wave issues one
// MFMA per stacked tile with the weight band as operand A and 8 consecutive
// columns of one data row per lane as operand B; the transposed 16 x 16
// results give each lane 4 consecutive output columns of one row.
template <int DT, int SHAPE, int r, int T, int V, int NW>
struct RowsCfg {
    using MT = MfmaTypes<DT>;
    using TS = typename MT::TS;
    using OP = typename MT::OP;
    using FR = typename MT::FR;
    using ACC = typename MT::ACC;
    static_assert(MT::KDIM == 32 && !MT::X3, "16-bit operands");
    static constexpr int R = r * T, DL = rows_delta(R);
    static constexpr int TR = 16 * V, TC = 16 * NW, NT = 64 * NW;
    static constexpr int LRD = TR + 2 * R;                                  // frame rows
    static constexpr int NKB0 = rows_nblk(SHAPE, r, T, 0) + rows_kk_lo(SHAPE, r, T, 0);  // widest row's k extent
    static constexpr int KMAX = 16 * (NW - 1) + 32 * NKB0;                  // frame columns read
    static constexpr int LCD = TC + 2 * R + DL;                             // frame columns holding data
    static constexpr int LCF = ((KMAX > LCD ? KMAX : LCD) + 7) / 8 * 8;     // staged columns
    // row pitch in 16-byte units: 2 mod 4 for eight-wave tiles, which makes
    // the operand-B reads conflict-free (measured on 16384^2: bf16 Box-2D2R
    // T = 4 2766 -> 2968, Star-2D2R T = 4 2839 -> 3075 GSt/s against an odd
    // pitch); odd for four-wave tiles (1-2 % faster there than the others)
    static constexpr int PIT = NW == 8 ? LCF + 8 * ((2 - (LCF / 8) % 4 + 4) % 4)
                                       : ((LCF / 8) % 2 ? LCF : LCF + 8);
    static constexpr int NFRAG = rows_total_frags(SHAPE, r, T);
    static constexpr bool ALDS = NFRAG <= 24;
    static constexpr int NCH = LCF / 8;                                     // 16-byte chunks per frame row
    static constexpr int NE = (LRD * NCH + NT - 1) / NT;                    // chunks per thread
    // a 16-byte chunk as a plain vector type (a struct with unions would be
    // kept in scratch memory when it lives across a loop iteration)
    typedef unsigned int Chunk __attribute__((ext_vector_type(4)));

    // frame origin in the grid (column a multiple of 8)
    __device__ __forceinline__ static int fr0(const Mfma2DArgs &a, int tile) { return (tile / a.ntc) * TR - R; }
    __device__ __forceinline__ static int fc0(const Mfma2DArgs &a, int tile) { return (tile % a.ntc) * TC - R - DL; }
    // interior tile: the frame lies inside the grid, rows of whole 16-byte units
    __device__ __forceinline__ static bool fast(const Mfma2DArgs &a, int tile)
    {
        const int f0 = fr0(a, tile), g0 = fc0(a, tile);
        return f0 >= 0 && f0 + LRD <= a.n0 && g0 >= 0 && g0 + LCF <= a.n1 && (a.n1 % 8) == 0 &&
               (reinterpret_cast<uintptr_t>(a.src) % 16) == 0;
    }
    // issue the frame loads of an interior tile, chunks i = 0..NE-1 of this
    // thread; clamped indices: every lane loads (in bounds), so the loads
    // stay in flight together
    __device__ __forceinline__ static void issue(const Mfma2DArgs &a, int tile, Chunk (&v)[NE], int tid)
    {
        const TS *src = static_cast<const TS *>(a.src);
        const int f0 = fr0(a, tile), g0 = fc0(a, tile), n1 = a.n1;
#pragma unroll
        for (int i = 0; i < NE; ++i) {
            const int e = tid + i * NT;
            const int ec = e < LRD * NCH ? e : LRD * NCH - 1;
            const int rowc = ec / NCH, chc = ec - rowc * NCH;
            v[i] = *reinterpret_cast<const Chunk *>(src + (int64_t)(f0 + rowc) * n1 + g0 + 8 * chc);
        }
    }
    __device__ __forceinline__ static void write(const Chunk (&v)[NE], OP *lb, int tid)
    {
#pragma unroll
        for (int i = 0; i < NE; ++i) {
            const int e = tid + i * NT;
            const int row = e / NCH, ch = e - row * NCH;
            if (e < LRD * NCH) *reinterpret_cast<Chunk *>(&lb[row * PIT + 8 * ch]) = v[i];
        }
    }
    // edge tiles: element by element with the boundary rule; columns past
    // the data (read only against zero weights) get zeros
    __device__ __forceinline__ static void stage_slow(const Mfma2DArgs &a, int tile, OP *lb, int tid)
    {
        const TS *src = static_cast<const TS *>(a.src);
        const int f0 = fr0(a, tile), g0 = fc0(a, tile), n0 = a.n0, n1 = a.n1;
        const bool periodic = a.periodic != 0;
        for (int e = tid; e < LRD * LCF; e += NT) {
            const int row = e / LCF, col = e - row * LCF;
            int gr = f0 + row, gc = g0 + col;
            OP v = OP(0);
            if (col < LCD) {
                const bool in = gr >= 0 && gr < n0 && gc >= 0 && gc < n1;
                v = to_op<OP>(a.h);
                if (in || periodic) {
                    gr = wrap(gr, n0);
                    gc = wrap(gc, n1);
                    v = to_op<OP>(load_val(src[(int64_t)gr * n1 + gc]));
                }
            }
            lb[row * PIT + col] = v;
        }
    }
    // MFMAs over the staged frame and the store of the tile
    __device__ __forceinline__ static void compute_store(const Mfma2DArgs &a, int tile, const OP *lb, const FR *lA, int tid)
    {
        const int lane = tid & 63, wave = tid >> 6;
        const int lg = lane >> 4, ln = lane & 15;
        const FR *afr = static_cast<const FR *>(a.afrag);
        ACC acc[V];
#pragma unroll
        for (int v = 0; v < V; ++v) acc[v] = ACC{};
        const int colw = 16 * wave + 8 * lg;
#pragma unroll
        for (int ar = -R; ar <= R; ++ar) {
            if (band_amax(SHAPE, r, T, 0, ar) < 0) continue;
            const int klo = rows_kk_lo(SHAPE, r, T, ar), nb = rows_nblk(SHAPE, r, T, ar);
            const int off = rows_frag_offset(SHAPE, r, T, ar);
#pragma unroll
            for (int ib = 0; ib < nb; ++ib) {
                const FR A = ALDS ? lA[(off + ib) * 64 + lane] : afr[(off + ib) * 64 + lane];
                const int col = colw + 32 * (klo + ib);
#pragma unroll
                for (int v = 0; v < V; ++v) {
                    const FR B = *reinterpret_cast<const FR *>(&lb[(16 * v + ln + ar + R) * PIT + col]);
                    acc[v] = mfma16(A, B, acc[v]);
                }
            }
        }
        // lane (lg, ln) holds row r0 + 16 v + ln, columns 4 lg .. 4 lg + 3
        TS *dst = static_cast<TS *>(a.dst);
        const int n0 = a.n0, n1 = a.n1;
        const int r0 = (tile / a.ntc) * TR, c0 = (tile % a.ntc) * TC;
        const int gc = c0 + 16 * wave + 4 * lg;
        const bool vec = gc + 4 <= n1 && (n1 % 4) == 0 && (reinterpret_cast<uintptr_t>(dst) % 8) == 0;
#pragma unroll
        for (int v = 0; v < V; ++v) {
            const int gr = r0 + 16 * v + ln;
            if (gr >= n0 || gc >= n1) continue;
            TS *p = dst + (int64_t)gr * n1 + gc;
            if (vec) {
                RawVec<TS, 4> ov;
#pragma unroll
                for (int e = 0; e < 4; ++e) ov.e[e] = to_storage<TS>(acc[v][e]);
                ov.store(p);
            } else {
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    if (gc + e < n1) p[e] = to_storage<TS>(acc[v][e]);
            }
        }
    }
};

// One tile per workgroup (a persistent grid of occupancy x CUs workgroups, each
// prefetching its next tile's frame under the current tile's MFMAs, measured
// 2x slower on 16384^2: the dispatcher balances tiles over CUs better).
template <int DT, int SHAPE, int r, int T, int V, int NW>
__device__ __forceinline__ void mfma2d_rows_tile(const Mfma2DArgs &a, const int tile)
{
    using C = RowsCfg<DT, SHAPE, r, T, V, NW>;
    using FR = typename C::FR;
    using OP = typename C::OP;
    constexpr int NFRAG = C::NFRAG, NT = C::NT;
    __shared__ __attribute__((aligned(16))) OP lb[C::LRD * C::PIT];
    __shared__ __attribute__((aligned(16))) FR lA[C::ALDS ? NFRAG * 64 : 1];
    const int tid = threadIdx.x;
    const FR *afr = static_cast<const FR *>(a.afrag);

    // A table: loads in flight during the staging
    constexpr int NAT = C::ALDS ? (NFRAG * 64 + NT - 1) / NT : 1;
    FR ta[NAT];
    if constexpr (C::ALDS) {
#pragma unroll
        for (int i = 0; i < NAT; ++i) {
            const int e = tid + i * NT;
            if (e < NFRAG * 64) ta[i] = afr[e];
        }
    }
    if (C::fast(a, tile)) {
        typename C::Chunk v[C::NE];
        C::issue(a, tile, v, tid);
        C::write(v, lb, tid);
    } else {
        C::stage_slow(a, tile, lb, tid);
    }
    if constexpr (C::ALDS) {
#pragma unroll
        for (int i = 0; i < NAT; ++i) {
            const int e = tid + i * NT;
            if (e < NFRAG * 64) lA[e] = ta[i];
        }
    }
    __syncthreads();
    C::compute_store(a, tile, lb, lA, tid);
}

// The 16-bit dense kernels use the row layout when its operand table fits
// LDS (measured on 16384^2 against the column layout: Box-2D2R bf16 T = 4
// +5 %, T = 1 +2 %; Box-2D3R bf16 T = 4, 50 fragments read from L2, -41 %);
// float64/float32, the compensated mode and the sparse instructions use the
// column layout.  Must agree with mfma_row_layout() (operand upload).
template <int DT, int SHAPE, int r, int T, bool SP>
constexpr bool use_rows()
{
    return MfmaTypes<DT>::KDIM == 32 && !MfmaTypes<DT>::X3 && !SP && rows_total_frags(SHAPE, r, T) <= 24;
}

template <int DT, int SHAPE, int r, int T, int V, int NW, bool SP>
__global__ __launch_bounds__(64 * NW) void mfma2d_kernel(Mfma2DArgs a)
{
    const int tile = xcd_remap(blockIdx.x, gridDim.x);
    if (tile >= a.ntiles) return;
    if constexpr (use_rows<DT, SHAPE, r, T, SP>())
        mfma2d_rows_tile<DT, SHAPE, r, T, V, NW>(a, tile);
    else
        mfma2d_tile<DT, SHAPE, r, T, V, NW, SP>(a, tile);
}

// Persistent batched launch over the tiles of several jobs: workgroup b takes
// items b + i*gridDim of one list; tile_start[j] is the first item of job j
// (tile_start[njobs] = total).  A barrier between items keeps the next
// item's staging from overwriting LDS blocks still being read.
template <int DT, int SHAPE, int r, int T, int V, int NW, bool SP>
__global__ __launch_bounds__(64 * NW) void mfma2d_batch_kernel(const Mfma2DArgs *__restrict__ jobs,
                                                             const int *__restrict__ tile_start, int njobs)
{
    const int total = tile_start[njobs];
    int j = 0;
    for (int item = xcd_remap(blockIdx.x, gridDim.x); item < total; item += gridDim.x) {
        while (j + 1 < njobs && tile_start[j + 1] <= item) ++j;
        const Mfma2DArgs a = jobs[j];
        if constexpr (use_rows<DT, SHAPE, r, T, SP>())
            mfma2d_rows_tile<DT, SHAPE, r, T, V, NW>(a, item - tile_start[j]);
        else
            mfma2d_tile<DT, SHAPE, r, T, V, NW, SP>(a, item - tile_start[j]);
        __syncthreads();
    }
}

// 16-bit operands: eight waves side by side (64 x 128 workgroup tiles,
// a smaller halo share).  With the conflict-free row pitch of these tiles
// they measured faster at every depth on 16384^2 (bf16 Box-2D2R T = 1 / 2 /
// 4: 856 -> 949, 1644 -> 1814, 2766 -> 2978 GSt/s; Box-2D1R T = 1 848 ->
// 987); with an odd pitch, small composite radii had been up to 12 % slower
// with eight.  The compensated mode's column-layout tiles gain too (bf16x3
// Box-2D2R T = 2 / 4: 886 -> 974, 1211 -> 1272 GSt/s).  Dense (not 2:4
// sparse) 16-bit
// passes with r <= 2 and composite radius 2-4 stack six tiles per wave (96 x
// 128: fewer halo rows per output row; +0.5-3 % measured, e.g. Star-2D2R
// T = 2 1806 -> 1858, Box-2D1R T = 4 3610 -> 3696 GSt/s); Box-2D3R T = 1
// was 8 % slower with six.
template <int DT, int r, int T, bool SP = false>
struct Mfma2DShape {
    static constexpr int V =
        (MfmaTypes<DT>::KDIM == 32 && !MfmaTypes<DT>::X3 && !SP && r <= 2 && r * T >= 2 && r * T <= 4) ? 6 : 4;
    static constexpr int NW = MfmaTypes<DT>::KDIM == 32 ? 8 : 4;
};

template <int DT, int SHAPE, int r, int T, bool SP = false>
bool mfma2d_args(const PassArgs &p, Mfma2DArgs *out)
{
    constexpr int V = Mfma2DShape<DT, r, T, SP>::V, NW = Mfma2DShape<DT, r, T, SP>::NW;
    using Cfg = Mfma2DCfg<DT, SHAPE, r, T, V, NW>;
    if (p.steps != T || !p.afrag) return false;
    if (MfmaTypes<DT>::X3 && !p.afrag_lo) return false;
    Mfma2DArgs &a = *out;
    a.src = p.src;
    a.dst = p.dst;
    a.afrag = p.afrag;
    a.afrag_lo = p.afrag_lo;
    a.n0 = (int)p.dims[0];
    a.n1 = (int)p.dims[1];
    a.periodic = p.boundary == STENCIL_PERIODIC;
    a.h = p.halo;
    a.ntr = (a.n0 + Cfg::TR - 1) / Cfg::TR;
    a.ntc = (a.n1 + Cfg::TCOL - 1) / Cfg::TCOL;
    a.ntiles = a.ntr * a.ntc;
    return true;
}

template <int DT, int SHAPE, int r, int T, bool SP = false>
hipError_t launch_mfma2d(const PassArgs &p, hipStream_t stream)
{
    constexpr int V = Mfma2DShape<DT, r, T, SP>::V, NW = Mfma2DShape<DT, r, T, SP>::NW;
    Mfma2DArgs a;
    if (!mfma2d_args<DT, SHAPE, r, T, SP>(p, &a)) return hipErrorInvalidValue;
    if (a.ntiles <= 0) return hipSuccess;
    hipLaunchKernelGGL((mfma2d_kernel<DT, SHAPE, r, T, V, NW, SP>), dim3(a.ntiles), dim3(64 * NW), 0, stream,
                       a);
    return hipGetLastError();
}

// n passes (one per job) of this variant in one persistent launch.
template <int DT, int SHAPE, int r, int T, bool SP = false>
hipError_t launch_mfma2d_batch(const PassArgs *ps, int n, BatchStaging *stage, hipStream_t stream)
{
    constexpr int V = Mfma2DShape<DT, r, T, SP>::V, NW = Mfma2DShape<DT, r, T, SP>::NW;
    std::vector<Mfma2DArgs> jobs;
    std::vector<int> start(1, 0);
    jobs.reserve(n);
    for (int i = 0; i < n; ++i) {
        Mfma2DArgs a;
        if (!mfma2d_args<DT, SHAPE, r, T, SP>(ps[i], &a)) return hipErrorInvalidValue;
        if (a.ntiles <= 0) continue;
        if ((int64_t)start.back() + a.ntiles > (1LL << 30)) return hipErrorInvalidValue;
        jobs.push_back(a);
        start.push_back(start.back() + a.ntiles);
    }
    if (jobs.empty()) return hipSuccess;
    void *djobs = nullptr, *dstart = nullptr;
    hipError_t e = stage_job_table(stage, jobs.data(), jobs.size() * sizeof(Mfma2DArgs), start, &djobs,
                                   &dstart, stream);
    if (e != hipSuccess) return e;
    int occ = 0;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, mfma2d_batch_kernel<DT, SHAPE, r, T, V, NW, SP>,
                                                     64 * NW, 0);
    if (e != hipSuccess || occ < 1) occ = 1;
    const int slots = occ * (ps[0].num_cu > 0 ? ps[0].num_cu : 256);
    const int total = start.back();
    hipLaunchKernelGGL((mfma2d_batch_kernel<DT, SHAPE, r, T, V, NW, SP>), dim3(total < slots ? total : slots),
                       dim3(64 * NW), 0, stream, static_cast<const Mfma2DArgs *>(djobs),
                       static_cast<const int *>(dstart), (int)jobs.size());
    return hipGetLastError();
}

#define M2(DT, SH, R, T) \
    {STENCIL_PATH_MFMA, DT, SH, 2, R, T, &launch_mfma2d<DT, SH, R, T>, &launch_mfma2d_batch<DT, SH, R, T>}
#define M2_T(DT, SH, R) M2(DT, SH, R, 1), M2(DT, SH, R, 2), M2(DT, SH, R, 3), M2(DT, SH, R, 4)
#define M2_R(DT, SH) M2_T(DT, SH, 1), M2_T(DT, SH, 2), M2_T(DT, SH, 3)
#define M2_S(DT) M2_R(DT, STENCIL_STAR), M2_R(DT, STENCIL_BOX)

// 2:4 structured-sparse instances (composite radius <= 7)
#define M2SP(DT, SH, R, T)                                                                  \
    {STENCIL_PATH_MFMA_SPARSE, DT, SH, 2, R, T, &launch_mfma2d<DT, SH, R, T, true>,         \
     &launch_mfma2d_batch<DT, SH, R, T, true>}
#define M2SP_S(DT, SH)                                                                      \
    M2SP(DT, SH, 1, 1), M2SP(DT, SH, 1, 2), M2SP(DT, SH, 1, 3), M2SP(DT, SH, 1, 4),           \
        M2SP(DT, SH, 1, 7), M2SP(DT, SH, 2, 1), M2SP(DT, SH, 2, 2), M2SP(DT, SH, 2, 3),       \
        M2SP(DT, SH, 3, 1), M2SP(DT, SH, 3, 2)

}  // namespace stl
