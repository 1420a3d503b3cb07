// Band layout of the MFMA path (shared by the kernels and the host code that
// builds their weight operands).
//
// The composite kernel of `t` fused steps (radius R = r t) is applied as a sum
// over kernel columns b of banded Toeplitz products (the "decomposing"
// transformation: one partial product per kernel vector, then accumulation):
//
//   out[16x16 tile] += A_b[16 x Kp] . X_b[Kp x 16],
//   A_b[m][k] = w_t[k - m - R][b]  (zero outside |k - m - R| <= amax(b)),
//   X_b[k][n] = u[tile_row - R + k][tile_col + n + b].
//
// In 3D the same holds per (plane offset c, column b) pair.  Along k only the
// blocks of KDIM rows that hold a structural non-zero of column b are issued:
// rows k in [R - amax, R + amax + 15].  For a box amax = R for every column;
// for a star composite amax(b) = r (t - ceil(|b| / r)) (its support is
// {x : sum_i ceil(|x_i| / r) <= t}); in 3D the column (c, b) has
// amax = r (t - ceil(|c|/r) - ceil(|b|/r)) and is skipped when negative.
#pragma once

namespace stl {

__host__ __device__ constexpr int cdiv(int a, int b) { return (a + b - 1) / b; }
__host__ __device__ constexpr int iabs(int a) { return a < 0 ? -a : a; }

// Largest |row offset| with a non-zero in column (c, b) of the composite, or
// -1 when the column is empty.  d = 2 uses c = 0.
__host__ __device__ constexpr int band_amax(int shape, int r, int t, int c, int b)
{
    if (shape == 1 /* box */) return r * t;
    const int left = t - cdiv(iabs(c), r) - cdiv(iabs(b), r);
    return left < 0 ? -1 : r * left;
}

__host__ __device__ constexpr int band_kk_lo(int shape, int r, int t, int c, int b, int kdim)
{
    return (r * t - band_amax(shape, r, t, c, b)) / kdim;
}

__host__ __device__ constexpr int band_kk_hi(int shape, int r, int t, int c, int b, int kdim)
{
    return (r * t + band_amax(shape, r, t, c, b) + 15) / kdim;
}

__host__ __device__ constexpr int band_nblk(int shape, int r, int t, int c, int b, int kdim)
{
    return band_amax(shape, r, t, c, b) < 0 ? 0
                                            : band_kk_hi(shape, r, t, c, b, kdim) -
                                                  band_kk_lo(shape, r, t, c, b, kdim) + 1;
}

// Fragments stored before column (c, b) in the operand array (columns ordered
// c-major, then b, each from -R to R).  d = 2 passes c = 0 and cmin = 0.
__host__ __device__ constexpr int band_frag_offset(int shape, int r, int t, int c, int b, int kdim,
                                                   int d)
{
    const int R = r * t;
    int off = 0;
    for (int cc = (d == 3 ? -R : 0); cc <= (d == 3 ? R : 0); ++cc)
        for (int bb = -R; bb <= R; ++bb) {
            if (cc == c && bb == b) return off;
            off += band_nblk(shape, r, t, cc, bb, kdim);
        }
    return off;
}

__host__ __device__ constexpr int band_total_frags(int shape, int r, int t, int kdim, int d)
{
    const int R = r * t;
    int off = 0;
    for (int cc = (d == 3 ? -R : 0); cc <= (d == 3 ? R : 0); ++cc)
        for (int bb = -R; bb <= R; ++bb) off += band_nblk(shape, r, t, cc, bb, kdim);
    return off;
}

// k of the MFMA instruction for a storage dtype (STENCIL_* codes).
__host__ __device__ constexpr int mfma_kdim(int dtype) { return dtype <= 1 ? 4 : 32; }

}  // namespace stl
