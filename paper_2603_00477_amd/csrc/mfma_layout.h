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

// Row layout of the 16-bit matrix path (d = 2): the composite is applied as a
// sum over its rows a of products D' = A_a B_a in which the 16 x 16 output
// tile appears transposed (D'[i][j] = out[row m0 + j][col c + i]):
//   A_a[i][k] = w_t[a][k - R - delta - i]   (band of the composite's row a),
//   B_a[k][j] = u[m0 + j + a][c - R - delta + k],
// so operand B is 8 consecutive columns of one data row per lane (a 16-byte
// read of a row-major block) and each lane's outputs are 4 consecutive
// columns of one row.  delta = (-R) mod 8 aligns the data window to 8
// columns.  Row a has non-zeros for |b| <= amax(a) (band_amax with the axes
// exchanged), so its k-blocks run from (R + delta - amax) / 32 to
// (R + delta + amax + 15) / 32.
__host__ __device__ constexpr int rows_delta(int R) { return (8 - R % 8) % 8; }
__host__ __device__ constexpr int rows_kk_lo(int shape, int r, int t, int a)
{
    return (r * t + rows_delta(r * t) - band_amax(shape, r, t, 0, a)) / 32;
}
__host__ __device__ constexpr int rows_kk_hi(int shape, int r, int t, int a)
{
    return (r * t + rows_delta(r * t) + band_amax(shape, r, t, 0, a) + 15) / 32;
}
__host__ __device__ constexpr int rows_nblk(int shape, int r, int t, int a)
{
    return band_amax(shape, r, t, 0, a) < 0 ? 0 : rows_kk_hi(shape, r, t, a) - rows_kk_lo(shape, r, t, a) + 1;
}
// Fragments stored before row a (rows ordered -R .. R).
__host__ __device__ constexpr int rows_frag_offset(int shape, int r, int t, int a)
{
    int off = 0;
    for (int aa = -r * t; aa < a; ++aa) off += rows_nblk(shape, r, t, aa);
    return off;
}
__host__ __device__ constexpr int rows_total_frags(int shape, int r, int t)
{
    return rows_frag_offset(shape, r, t, r * t + 1);
}

// 2:4 structured-sparse layout (d = 2, 16-bit operands, composite radius
// R <= 7).  One v_smfmac_f32_16x16x64 covers two non-empty kernel columns
// (b, b') of a 16-row output tile: its 64 dense k positions are 16 groups of
// four; group h < 8 holds rows {2h, 2h+1, 2h+16, 2h+17} of column b's
// 32-row data block, group 8 + h the same rows of column b'.  A band of at
// most 15 rows never covers two rows of a group 15 or more apart, so every
// group holds at most two non-zero weights, as the instruction requires.
// Columns pair in order; an odd last column pairs with itself, its second
// half weighted zero.
__host__ __device__ constexpr int sparse_max_radius() { return 7; }

__host__ __device__ constexpr int band_ncols(int shape, int r, int t)
{
    int n = 0;
    for (int b = -r * t; b <= r * t; ++b) n += band_amax(shape, r, t, 0, b) >= 0 ? 1 : 0;
    return n;
}

__host__ __device__ constexpr int sparse_pairs(int shape, int r, int t) { return (band_ncols(shape, r, t) + 1) / 2; }

// Row of the 32-row data block held at position e (0..3) of group h (0..7).
__host__ __device__ constexpr int sparse_group_row(int h, int e) { return 2 * h + (e & 1) + 16 * (e >> 1); }

// Sequential-step fusion (d = 2): step s (1..t) of a pass computes frame
// rows and columns [seq_start, seq_start + seq_size) of a tile x tile output
// tile's frame (the input block with its halo of r t points on each side):
// the points later steps need, [r s, tile + 2 r t - r s), widened to whole
// 16 x 16 MFMA tiles; with 32-row operand blocks (16-bit) a block starts at
// a row = r (mod 8) so that its 8-row operand chunks are 16-byte aligned.
__host__ __device__ constexpr int seq_start(int r, int s, int kdim) { return kdim == 32 ? r + 8 * ((r * (s - 1)) / 8) : r * s; }
__host__ __device__ constexpr int seq_size(int tile, int r, int t, int s, int kdim)
{
    return ((tile + 2 * r * t - r * s - seq_start(r, s, kdim) + 15) / 16) * 16;
}
__host__ __device__ constexpr int seq_kp(int r, int kdim) { return ((16 + 2 * r + kdim - 1) / kdim) * kdim; }
// Frame extent holding every operand read: step s reads rows f0 - r ..
// f0 - r + kp - 1 and columns g0 - r .. g0 + 15 + r of its blocks.
__host__ __device__ constexpr int seq_frame_rows(int tile, int r, int t, int kdim)
{
    int m = tile + 2 * r * t;
    for (int s = 1; s <= t; ++s) {
        const int e = seq_start(r, s, kdim) + seq_size(tile, r, t, s, kdim) - 16 - r + seq_kp(r, kdim);
        m = m > e ? m : e;
    }
    return m;
}
__host__ __device__ constexpr int seq_frame_cols(int tile, int r, int t, int kdim)
{
    int m = tile + 2 * r * t;
    for (int s = 1; s <= t; ++s) {
        const int e = seq_start(r, s, kdim) + seq_size(tile, r, t, s, kdim) + r;
        m = m > e ? m : e;
    }
    return m;
}
// Row pitch (row-major frames, 4-deep operands) and column pitch
// (column-major frames, 32-deep operands: an odd number of 16-byte units).
__host__ __device__ constexpr int seq_pitch(int tile, int r, int t, int kdim)
{
    if (kdim == 32) {
        const int u = (seq_frame_rows(tile, r, t, kdim) + 7) / 8;
        return (u % 2 ? u : u + 1) * 8;
    }
    const int c = seq_frame_cols(tile, r, t, kdim);
    return c + (c % 32 == 0 ? 1 : 0);
}
__host__ __device__ constexpr int seq_frame_elems(int tile, int r, int t, int kdim)
{
    return kdim == 32 ? seq_frame_cols(tile, r, t, kdim) * seq_pitch(tile, r, t, kdim)
                      : seq_frame_rows(tile, r, t, kdim) * seq_pitch(tile, r, t, kdim);
}
// LDS bytes: two frames plus the single step's operand fragments.
__host__ __device__ constexpr int seq_lds_bytes(int shape, int tile, int r, int t, int kdim, int elem_bytes)
{
    return 2 * seq_frame_elems(tile, r, t, kdim) * elem_bytes +
           band_total_frags(shape, r, 1, kdim, 2) * 64 * (kdim / 4) * elem_bytes;
}
// 64 x 64 output tiles, or 32 x 32 where two 64-tile frames would not fit.
__host__ __device__ constexpr int seq_tile(int shape, int r, int t, int kdim, int elem_bytes)
{
    return seq_lds_bytes(shape, 64, r, t, kdim, elem_bytes) <= 150 * 1024 ? 64 : 32;
}

// k of the MFMA instruction for a storage dtype (STENCIL_* codes).
__host__ __device__ constexpr int mfma_kdim(int dtype) { return dtype <= 1 ? 4 : 32; }

}  // namespace stl
