// Roofline model of the two paths and the MFMA operand layout's sparsity.
//
// Paper, Sec. "Performance Formulation":
//   roofline                P = min(PP, BB * I),  I = C / M
//   original problem        C = 2K flops, M = 2D bytes per point
//   temporal fusion (VALU)  C = t * 2K, M = 2D      -> I = tK / D
//   kernel fusion (MFMA)    executed C = (alpha / S) t 2K, M = 2D,
//                           useful throughput = (S / alpha) * min(PP, BB I)
//   redundancy              alpha = K_t / (t K)
// Sec. "Performance Comparative Analysis": speed-up ratio of the two, four
// scenarios by which side of its ridge each path sits, sweet spot
// alpha < S PP_TC / PP_CU when both are compute-bound.  Sec. "Further
// Acceleration with Sparse Hardware": sparse units keep I and raise PP.
//
// This library adds gamma (products per useful multiply-add: 3 for the
// compensated bf16 hi/lo split, 1 otherwise), which scales executed MFMA work
// exactly like alpha / S does.

#include <cmath>
#include <cstring>
#include <vector>

#include "internal.h"
#include "mfma_layout.h"

namespace stl {

static int64_t ipow(int64_t b, int e)
{
    int64_t v = 1;
    while (e-- > 0) v *= b;
    return v;
}

static int ceil_div(int a, int b) { return (a + b - 1) / b; }

// Support of the t-fold composed pattern (non-zero displacements).
static int64_t fused_points(int shape, int d, int r, int t)
{
    if (shape == STENCIL_BOX) return ipow(2 * (int64_t)r * t + 1, d);
    // star: displacements x with sum_i ceil(|x_i| / r) <= t
    const int R = r * t;
    int64_t n = 0;
    if (d == 2) {
        for (int a = -R; a <= R; ++a)
            for (int b = -R; b <= R; ++b)
                if (ceil_div(std::abs(a), r) + ceil_div(std::abs(b), r) <= t) ++n;
    } else {
        for (int c = -R; c <= R; ++c)
            for (int a = -R; a <= R; ++a)
                for (int b = -R; b <= R; ++b)
                    if (ceil_div(std::abs(c), r) + ceil_div(std::abs(a), r) +
                            ceil_div(std::abs(b), r) <= t)
                        ++n;
    }
    return n;
}

static int64_t single_points(int shape, int d, int r)
{
    return shape == STENCIL_BOX ? ipow(2 * r + 1, d) : 2 * d * r + 1;
}

static int mfma_k(int dtype)
{
    switch (dtype) {
    case STENCIL_F64: return 4;   // v_mfma_f64_16x16x4_f64
    case STENCIL_F32: return 4;   // v_mfma_f32_16x16x4_f32
    default: return 32;           // v_mfma_f32_16x16x32_{bf16,f16}
    }
}

MfmaLayout mfma_layout(int shape, int d, int r, int steps, int dtype)
{
    MfmaLayout L;
    L.R = r * steps;
    L.kdim = mfma_k(dtype);
    L.Kp = ceil_div(16 + 2 * L.R, L.kdim) * L.kdim;
    L.nblk = L.Kp / L.kdim;
    const double KT = (double)fused_points(shape, d, r, steps);
    // MACs issued per output point: KDIM per structurally non-zero k-block of
    // every column band (see mfma_layout.h)
    double executed = (double)band_total_frags(shape, r, steps, L.kdim, d) * L.kdim;
    if (mfma_row_layout(dtype, d, shape, r, steps))  // 16-bit row layout: per k-block of each row
        executed = (double)rows_total_frags(shape, r, steps) * L.kdim;
    L.S = KT / executed;
    return L;
}

// Skirt recomputation of the VALU kernels' fused tiles: executed / useful
// FMAs.  2D: a wave's band of 64 W columns (W = 16-byte vector) keeps
// 64 W - 2 E outputs, E = r T rounded up to W.  3D: an in-plane tile of
// (TY WY) x (TX W) points keeps (TY WY - 2 EY) x (TX W - 2 EX), EY = r T for
// fused passes (one-step passes stage their halo: no skirt); the thread tiles
// are those the 3D launcher picks.
static double valu_halo_factor(int shape, int d, int r, int T, int dtype)
{
    const int D = dtype_bytes(dtype);
    const int W16 = 16 / D > 8 ? 8 : 16 / D;
    // columns per lane of the 2D kernel: one 16-byte vector, two for float64
    // at T = 2 and for float64 r = 7 at T = 1
    const int W = (d == 2 && D == 8 && (T == 2 || (T == 1 && r >= 7))) ? 2 * W16 : W16;
    if (d == 2) {
        const int E = (r * T + W - 1) / W * W;
        return (64.0 * W) / (64.0 * W - 2.0 * E);
    }
    if (T == 1) return 1.0;
    // fused 3D passes: every step computes the L1 x M1 layout (2 rows x W
    // columns per thread; stars 16 x 32 threads, boxes 32 rows x 64 columns);
    // the input halo is staged, so the output tile is the layout less
    // r (T - 1) per side, the left margin rounded up to a whole vector
    const int L1 = 2 * (shape == STENCIL_STAR ? 32 : 16), M1 = shape == STENCIL_STAR ? 16 * W : 64;
    const int SK = r * (T - 1), SKL = (SK + W - 1) / W * W;
    const int BY = L1 - 2 * SK, BX = (M1 - SKL - SK) / W * W;
    if (BY <= 0 || BX <= 0) return 0.0;
    return (double)L1 * M1 / ((double)BY * BX);
}

// Executed flops per point per pass of sequential-step MFMA fusion: each of
// the T steps runs the single step's band product (every structurally
// non-zero k-block of every column) on (size(s) / 16)^2 16 x 16 tiles of a
// tile x tile output tile.
static double mfma_seq_flops(int shape, int r, int T, int dtype)
{
    const int kdim = mfma_k(dtype);
    const int eb = dtype == STENCIL_F64 ? 8 : (dtype == STENCIL_F32 ? 4 : 2);
    const int tile = seq_tile(shape, r, T, kdim, eb);
    const double per_block = 2.0 * 16 * 16 * kdim * band_total_frags(shape, r, 1, kdim, 2);
    double blocks = 0;
    for (int s = 1; s <= T; ++s) {
        const double nb = seq_size(tile, r, T, s, kdim) / 16;
        blocks += nb * nb;
    }
    return blocks * per_block / ((double)tile * tile);
}

}  // namespace stl

using namespace stl;

extern "C" int stencil_hw_default(int dtype, stencil_hw_t *out)
{
    if (!out) return fail(STENCIL_ERR_INVALID_ARG, "stencil_hw_default: out is NULL");
    stencil_hw_t h;
    h.BB = 8.0e12;  // HBM3E
    switch (dtype) {
    case STENCIL_F64:
        h.PP_valu = 78.6e12;   // FP64 vector
        h.PP_mfma = 78.6e12;   // FP64 matrix
        h.PP_mfma_sparse = 78.6e12;
        break;
    case STENCIL_F32:
        h.PP_valu = 157.3e12;  // FP32 vector (scalar v_fma_f32 issues at twice the FP64 rate)
        h.PP_mfma = 157.3e12;  // FP32 matrix
        h.PP_mfma_sparse = 157.3e12;
        break;
    case STENCIL_BF16:
    case STENCIL_F16:
    case STENCIL_F32_BF16X3:
        h.PP_valu = 157.3e12;  // FP32 arithmetic on the vector path
        h.PP_mfma = 2516.6e12; // dense BF16/FP16 matrix
        h.PP_mfma_sparse = 5033.2e12;
        break;
    default:
        return fail(STENCIL_ERR_INVALID_ARG, "stencil_hw_default: unknown dtype");
    }
    *out = h;
    return STENCIL_OK;
}

extern "C" double stencil_mfma_sparsity(int shape, int d, int r, int T, int dtype)
{
    if ((shape != STENCIL_STAR && shape != STENCIL_BOX) || (d != 2 && d != 3) || r < 1 || T < 1 ||
        dtype < STENCIL_F64 || dtype > STENCIL_F32_BF16X3)
        return -1.0;
    return mfma_layout(shape, d, r, T, dtype).S;
}

extern "C" int stencil_model_predict(const stencil_model_in_t *in, const stencil_hw_t *hw,
                                     stencil_model_out_t *out)
{
    if (!in || !out) return fail(STENCIL_ERR_INVALID_ARG, "stencil_model_predict: NULL argument");
    if ((in->shape != STENCIL_STAR && in->shape != STENCIL_BOX) || (in->d != 2 && in->d != 3) ||
        in->r < 1 || in->T < 1 || in->dtype < STENCIL_F64 || in->dtype > STENCIL_F32_BF16X3)
        return fail(STENCIL_ERR_INVALID_ARG, "stencil_model_predict: invalid shape/d/r/T/dtype");
    stencil_hw_t H;
    if (hw) {
        H = *hw;
    } else {
        int rc = stencil_hw_default(in->dtype, &H);
        if (rc) return rc;
    }
    if (!(H.BB > 0) || !(H.PP_valu > 0) || !(H.PP_mfma > 0))
        return fail(STENCIL_ERR_INVALID_ARG, "stencil_model_predict: non-positive ceilings");
    stencil_model_out_t o;
    std::memset(&o, 0, sizeof o);
    const int T = in->T;
    o.K = (int)single_points(in->shape, in->d, in->r);
    o.K_T = (int)fused_points(in->shape, in->d, in->r, T);
    o.D = dtype_bytes(in->dtype);
    o.alpha = in->alpha > 0 ? in->alpha : (double)o.K_T / ((double)T * o.K);
    if (in->S > 0) {
        o.S = in->S;
    } else if (in->sparse && in->d == 2 && mfma_k(in->dtype) == 32 && in->dtype != STENCIL_F32_BF16X3 &&
               in->r * T <= sparse_max_radius()) {
        // 2:4 layout: one 16x16x64 instruction (64 dense-equivalent MACs per
        // output point, counted against the sparse peak) per column pair
        o.S = (double)o.K_T / (64.0 * sparse_pairs(in->shape, in->r, T));
    } else {
        o.S = mfma_layout(in->shape, in->d, in->r, T, in->dtype).S;
    }
    o.gamma = in->dtype == STENCIL_F32_BF16X3 ? 3.0 : 1.0;
    const double PPm = in->sparse ? H.PP_mfma_sparse : H.PP_mfma;
    o.C_valu = 2.0 * o.K * T;
    o.C_mfma = o.gamma * (o.alpha / o.S) * o.C_valu;
    o.M = 2.0 * o.D;
    o.I_valu = o.C_valu / o.M;
    o.I_mfma = o.C_mfma / o.M;
    o.ridge_valu = H.PP_valu / H.BB;
    o.ridge_mfma = PPm / H.BB;
    o.P_valu = std::fmin(H.PP_valu, H.BB * o.I_valu);
    o.P_mfma_raw = std::fmin(PPm, H.BB * o.I_mfma);
    o.P_mfma = o.P_mfma_raw * o.S / (o.gamma * o.alpha);
    o.gst_valu = o.P_valu / (2.0 * o.K) / 1e9;
    o.gst_mfma = o.P_mfma / (2.0 * o.K) / 1e9;
    o.ratio = o.gst_mfma / o.gst_valu;
    const bool cu_cb = o.I_valu > o.ridge_valu;
    const bool tc_cb = o.I_mfma > o.ridge_mfma;
    o.scenario = !cu_cb ? (!tc_cb ? 1 : 2) : (!tc_cb ? 3 : 4);
    o.sweet_spot = o.gamma * o.alpha < o.S * PPm / H.PP_valu;
    o.winner = o.ratio < 0.87 ? -1 : (o.ratio > 1.15 ? 1 : 0);
    o.halo_valu = valu_halo_factor(in->shape, in->d, in->r, T, in->dtype);
    if (in->d == 2 && in->dtype != STENCIL_F32_BF16X3) {
        o.C_mfma_seq = mfma_seq_flops(in->shape, in->r, T, in->dtype);
        const double useful = o.C_valu;  // 2 K T per point per pass
        const double P_raw = std::fmin(H.PP_mfma, H.BB * o.C_mfma_seq / o.M);
        o.gst_mfma_seq = P_raw * useful / o.C_mfma_seq / (2.0 * o.K) / 1e9;
    }
    *out = o;
    return STENCIL_OK;
}
