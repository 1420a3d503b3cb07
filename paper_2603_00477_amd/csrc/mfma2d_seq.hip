// MFMA path with sequential-step fusion (alpha = 1), d = 2.
//
// Kernel fusion applies the T-step composite once per pass and pays its
// redundancy alpha = K_T / (T K) (paper, Sec. "Handling Stencils with Small
// Radius", which contrasts it with fusing T sequential steps).  This kernel
// fuses the T steps sequentially instead: a workgroup stages its 64 x 64
// (or 32 x 32) output tile's input block with a halo of r T points in LDS, then runs T
// single-step band products (the composite of one step, radius r) on the
// matrix cores, each step computing the block shrunk by r per side from the
// previous step's block, which stays in LDS.  No step multiplies a composite
// weight, so alpha = 1; the price is the halo each step recomputes (the
// step regions are rounded up to whole 16 x 16 MFMA tiles), which the model
// reports beside the kernel-fused layout's (stencil_model_predict, C_mfma_seq).
// Intermediate fields are exactly those of T separate steps (Dirichlet: h
// outside the grid after every step), so Dirichlet passes need no boundary
// band fix-up.  Intermediate values are rounded to the operand type between
// steps (16-bit modes: once per step, float64 / float32: exact).

#include "mfma2d_impl.h"

namespace stl {
namespace {

template <int DT, int SHAPE, int r, int T, int TL>
struct SeqCfg {
    using MT = MfmaTypes<DT>;
    static constexpr int KDIM = MT::KDIM;
    static constexpr int TILE = TL;                 // output tile side
    static constexpr int H = r * T;                 // halo of the input block
    static constexpr int KP = seq_kp(r, KDIM);      // band length per column
    static constexpr int NW = 4;                    // waves per workgroup
    static constexpr int start(int s) { return seq_start(r, s, KDIM); }
    static constexpr int size(int s) { return seq_size(TILE, r, T, s, KDIM); }
    // float64/float32 frames row-major, 16-bit ones column-major (a lane's
    // 8 consecutive rows of one column are one 16-byte read)
    static constexpr bool COLMAJOR = KDIM == 32;
    static constexpr int PITCH = seq_pitch(TILE, r, T, KDIM);
    static constexpr int NLDS = seq_frame_elems(TILE, r, T, KDIM);
    static constexpr int NFRAG = band_total_frags(SHAPE, r, 1, KDIM, 2);
    __host__ __device__ static constexpr int at(int row, int col) { return COLMAJOR ? col * PITCH + row : row * PITCH + col; }
};

template <int DT, int SHAPE, int r, int T, int TL>
__global__ __launch_bounds__(256) void mfma2d_seq_kernel(Mfma2DArgs a)
{
    using Cfg = SeqCfg<DT, SHAPE, r, T, TL>;
    using MT = typename Cfg::MT;
    using TS = typename MT::TS;
    using OP = typename MT::OP;
    using FR = typename MT::FR;
    using ACC = typename MT::ACC;
    constexpr int KDIM = Cfg::KDIM, TILE = Cfg::TILE, H = Cfg::H, NT = 64 * Cfg::NW;

    __shared__ __attribute__((aligned(16))) OP buf[2][Cfg::NLDS];
    __shared__ __attribute__((aligned(16))) FR lA[Cfg::NFRAG * 64];

    const int tile = xcd_remap(blockIdx.x, gridDim.x);
    if (tile >= a.ntiles) return;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int r0 = (tile / a.ntc) * TILE, c0 = (tile % a.ntc) * TILE;
    const int n0 = a.n0, n1 = a.n1;
    const bool periodic = a.periodic != 0;
    const TS *src = static_cast<const TS *>(a.src);
    TS *dst = static_cast<TS *>(a.dst);
    const FR *afr = static_cast<const FR *>(a.afrag);

    // zero frame (reads past a step's region see finite values), operand
    // fragments of the single step to LDS
    for (int i = tid; i < 2 * Cfg::NLDS; i += NT) (&buf[0][0])[i] = OP(0);
    for (int i = tid; i < Cfg::NFRAG * 64; i += NT) lA[i] = afr[i];
    __syncthreads();
    // input block: frame (fr, fc) <-> grid (r0 - H + fr, c0 - H + fc)
    constexpr int IB = TILE + 2 * H;
    for (int e = tid; e < IB * IB; e += NT) {
        const int fr = e / IB, fc = e - fr * IB;
        int gr = r0 - H + fr, gc = c0 - H + fc;
        const bool in = gr >= 0 && gr < n0 && gc >= 0 && gc < n1;
        OP v = to_op<OP>(a.h);
        if (in || periodic) {
            gr = wrap(gr, n0);
            gc = wrap(gc, n1);
            v = to_op<OP>(load_val(src[(int64_t)gr * n1 + gc]));
        }
        buf[0][Cfg::at(fr, fc)] = v;
    }
    __syncthreads();

    const int lg = lane >> 4, ln = lane & 15;
#pragma unroll
    for (int s = 1; s <= T; ++s) {
        const OP *in = buf[(s - 1) & 1];
        OP *out = buf[s & 1];
        const int fs = Cfg::start(s), nb = Cfg::size(s) / 16;
        for (int blk = wave; blk < nb * nb; blk += Cfg::NW) {
            const int f0 = fs + 16 * (blk / nb), g0 = fs + 16 * (blk % nb);
            ACC acc = ACC{};
#pragma unroll
            for (int b = -r; b <= r; ++b) {
                if (band_amax(SHAPE, r, 1, 0, b) < 0) continue;
                const int klo = band_kk_lo(SHAPE, r, 1, 0, b, KDIM);
                const int khi = band_kk_hi(SHAPE, r, 1, 0, b, KDIM);
                const int off = band_frag_offset(SHAPE, r, 1, 0, b, KDIM, 2);
#pragma unroll
                for (int kk = klo; kk <= khi; ++kk) {
                    const FR A = lA[(off + kk - klo) * 64 + lane];
                    const int col = g0 + ln + b;
                    if constexpr (KDIM == 4) {
                        const FR B = in[Cfg::at(f0 - r + 4 * kk + lg, col)];
                        acc = mfma16(A, B, acc);
                    } else {
                        const FR B = *reinterpret_cast<const FR *>(&in[Cfg::at(f0 - r + 32 * kk + 8 * lg, col)]);
                        acc = mfma16(A, B, acc);
                    }
                }
            }
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int dr = MT::D_ROW_INTERLEAVED ? 4 * e + lg : 4 * lg + e;
                const int fr = f0 + dr, fc = g0 + ln;
                const int gr = r0 - H + fr, gc = c0 - H + fc;
                if (s < T) {
                    const bool in_grid = gr >= 0 && gr < n0 && gc >= 0 && gc < n1;
                    out[Cfg::at(fr, fc)] = (periodic || in_grid) ? to_op<OP>(acc[e]) : to_op<OP>(a.h);
                } else if (fr >= H && fc >= H && fr - H < TILE && fc - H < TILE && gr < n0 && gc < n1) {
                    dst[(int64_t)gr * n1 + gc] = to_storage<TS>(acc[e]);
                }
            }
        }
        __syncthreads();
    }
}

template <int DT, int SHAPE, int r, int T>
hipError_t launch_mfma2d_seq(const PassArgs &p, hipStream_t stream)
{
    constexpr int KDIM = MfmaTypes<DT>::KDIM;
    constexpr int EB = (int)sizeof(typename MfmaTypes<DT>::OP);
    constexpr int TL = seq_tile(SHAPE, r, T, KDIM, EB);
    using Cfg = SeqCfg<DT, SHAPE, r, T, TL>;
    static_assert(seq_lds_bytes(SHAPE, TL, r, T, KDIM, EB) <= 160 * 1024, "frames exceed LDS");
    if (p.steps != T || !p.afrag) return hipErrorInvalidValue;
    Mfma2DArgs a;
    a.src = p.src;
    a.dst = p.dst;
    a.afrag = p.afrag;
    a.afrag_lo = nullptr;
    a.n0 = (int)p.dims[0];
    a.n1 = (int)p.dims[1];
    a.periodic = p.boundary == STENCIL_PERIODIC;
    a.h = p.halo;
    a.ntr = (a.n0 + Cfg::TILE - 1) / Cfg::TILE;
    a.ntc = (a.n1 + Cfg::TILE - 1) / Cfg::TILE;
    a.ntiles = a.ntr * a.ntc;
    if (a.ntiles <= 0) return hipSuccess;
    hipLaunchKernelGGL((mfma2d_seq_kernel<DT, SHAPE, r, T, TL>), dim3(a.ntiles), dim3(256), 0, stream, a);
    return hipGetLastError();
}

#define MS(DT, SH, R, T) {STENCIL_PATH_MFMA_SEQ, DT, SH, 2, R, T, &launch_mfma2d_seq<DT, SH, R, T>, nullptr}
#define MS_T(DT, SH, R) MS(DT, SH, R, 1), MS(DT, SH, R, 2), MS(DT, SH, R, 3), MS(DT, SH, R, 4)
#define MS_S(DT) MS_T(DT, STENCIL_BOX, 1), MS_T(DT, STENCIL_BOX, 2), MS_T(DT, STENCIL_BOX, 3), \
    MS_T(DT, STENCIL_STAR, 1), MS_T(DT, STENCIL_STAR, 2), MS_T(DT, STENCIL_STAR, 3)

}  // namespace

const std::vector<KernelEntry> &mfma2d_table_seq()
{
    static const std::vector<KernelEntry> table = {MS_S(STENCIL_F64), MS_S(STENCIL_F32), MS_S(STENCIL_BF16),
                                                   MS_S(STENCIL_F16)};
    return table;
}

}  // namespace stl
