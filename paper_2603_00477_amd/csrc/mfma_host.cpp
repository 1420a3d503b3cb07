// Host construction of the MFMA path's weight operands.
//
// For every structurally non-zero (column, k-block) of the band layout the
// 64 lanes' A-operand elements are written in the order the matrix
// instruction consumes them: lane l holds A[m = l % 16][k = kk*KDIM +
// (l / 16)*KPL + e], e < KPL = KDIM / 4.  Values come from the composite
// kernel of `steps` fused steps, composed in float64 and rounded once to the
// operand type (round to nearest even).  The compensated mode stores
// hi = bf16(w) and lo = bf16(w - hi).

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

#include "internal.h"
#include "mfma_layout.h"

namespace stl {
namespace {

// Round a double to `bits` significant bits, ties to even.
double round_bits(double x, int bits)
{
    if (x == 0.0 || !std::isfinite(x)) return x;
    int e = 0;
    std::frexp(x, &e);
    const double scale = std::ldexp(1.0, bits - e);
    return std::nearbyint(x * scale) / scale;
}

uint16_t bf16_bits(double x)
{
    const float f = (float)round_bits(x, 8);  // exact in float
    uint32_t u;
    std::memcpy(&u, &f, 4);
    return (uint16_t)(u >> 16);
}

double bf16_value(uint16_t b)
{
    uint32_t u = (uint32_t)b << 16;
    float f;
    std::memcpy(&f, &u, 4);
    return f;
}

uint16_t f16_bits(double x)
{
    const _Float16 h = (_Float16)(float)round_bits(x, 11);
    uint16_t b;
    std::memcpy(&b, &h, 2);
    return b;
}

template <typename T>
void put(std::vector<uint8_t> *v, size_t idx, T val)
{
    std::memcpy(v->data() + idx * sizeof(T), &val, sizeof(T));
}

}  // namespace

void mfma_build_fragments(int shape, int d, int r, const double *w, int steps, int dtype,
                          std::vector<uint8_t> *hi, std::vector<uint8_t> *lo)
{
    hi->clear();
    lo->clear();
    const int kdim = mfma_kdim(dtype);
    const int kpl = kdim / 4;
    const int R = r * steps;
    const int side = 2 * R + 1;
    std::vector<double> wc;
    compose_dense(shape, d, r, w, steps, &wc);
    const int nfrag = band_total_frags(shape, r, steps, kdim, d);
    const size_t nel = (size_t)nfrag * 64 * kpl;
    const int esize = dtype == STENCIL_F64 ? 8 : (dtype == STENCIL_F32 ? 4 : 2);
    hi->assign(nel * esize, 0);
    if (dtype == STENCIL_F32_BF16X3) lo->assign(nel * 2, 0);
    size_t frag = 0;
    for (int c = (d == 3 ? -R : 0); c <= (d == 3 ? R : 0); ++c) {
        for (int b = -R; b <= R; ++b) {
            const int nb = band_nblk(shape, r, steps, c, b, kdim);
            const int klo = band_kk_lo(shape, r, steps, c, b, kdim);
            for (int i = 0; i < nb; ++i, ++frag) {
                const int kk = klo + i;
                for (int l = 0; l < 64; ++l) {
                    for (int e = 0; e < kpl; ++e) {
                        const int m = l % 16;
                        const int k = kk * kdim + (l / 16) * kpl + e;
                        const int a = k - m - R;
                        double v = 0.0;
                        if (a >= -R && a <= R) {
                            size_t idx = (size_t)(a + R) * side + (b + R);
                            if (d == 3) idx += (size_t)(c + R) * side * side;
                            v = wc[idx];
                        }
                        const size_t el = (frag * 64 + l) * kpl + e;
                        switch (dtype) {
                        case STENCIL_F64: put<double>(hi, el, v); break;
                        case STENCIL_F32: put<float>(hi, el, (float)v); break;
                        case STENCIL_BF16: put<uint16_t>(hi, el, bf16_bits(v)); break;
                        case STENCIL_F16: put<uint16_t>(hi, el, f16_bits(v)); break;
                        case STENCIL_F32_BF16X3: {
                            const uint16_t h = bf16_bits(v);
                            put<uint16_t>(hi, el, h);
                            put<uint16_t>(lo, el, bf16_bits(v - bf16_value(h)));
                            break;
                        }
                        default: break;
                        }
                    }
                }
            }
        }
    }
}

void mfma_build_row_fragments(int shape, int r, const double *w, int steps, int dtype,
                              std::vector<uint8_t> *out)
{
    // Per non-empty k-block of each composite row a (rows -R .. R): 64 lanes
    // x 8 weights; lane l holds A_a[i = l % 16][k = 32 kk + 8 (l / 16) + e].
    out->clear();
    const int R = r * steps;
    const int side = 2 * R + 1;
    const int dl = rows_delta(R);
    std::vector<double> wc;
    compose_dense(shape, 2, r, w, steps, &wc);
    out->assign((size_t)rows_total_frags(shape, r, steps) * 64 * 8 * 2, 0);
    size_t frag = 0;
    for (int a = -R; a <= R; ++a) {
        const int nb = rows_nblk(shape, r, steps, a);
        const int klo = rows_kk_lo(shape, r, steps, a);
        for (int ib = 0; ib < nb; ++ib, ++frag) {
            for (int l = 0; l < 64; ++l) {
                const int i = l % 16, q = l / 16;
                for (int e = 0; e < 8; ++e) {
                    const int k = 32 * (klo + ib) + 8 * q + e;
                    const int b = k - R - dl - i;  // column offset of the weight
                    const double v = (b >= -R && b <= R) ? wc[(size_t)(a + R) * side + (b + R)] : 0.0;
                    const uint16_t bits = dtype == STENCIL_F16 ? f16_bits(v) : bf16_bits(v);
                    std::memcpy(out->data() + ((frag * 64 + l) * 8 + e) * 2, &bits, 2);
                }
            }
        }
    }
}

void mfma_build_sparse_fragments(int shape, int r, const double *w, int steps, int dtype,
                                 std::vector<uint8_t> *out)
{
    // Per column pair: 64 lanes x 8 compressed 16-bit weights, then 64 lanes
    // x one int32 of 2-bit positions.  Lane l holds output row m = l % 16 and
    // groups g = 4 (l / 16) + j / 2 (j = 0..7; groups 0-7 column b, 8-15
    // column b'); value j's position within its group is bits 2j..2j+1.
    out->clear();
    const int R = r * steps;
    const int side = 2 * R + 1;
    std::vector<double> wc;
    compose_dense(shape, 2, r, w, steps, &wc);
    std::vector<int> cols;
    for (int b = -R; b <= R; ++b)
        if (band_amax(shape, r, steps, 0, b) >= 0) cols.push_back(b);
    const int np = (int)(cols.size() + 1) / 2;
    out->assign((size_t)np * 64 * (16 + 4), 0);
    uint8_t *vals = out->data();
    uint8_t *idxs = out->data() + (size_t)np * 64 * 16;
    for (int pi = 0; pi < np; ++pi) {
        const int cb[2] = {cols[2 * pi], 2 * pi + 1 < (int)cols.size() ? cols[2 * pi + 1] : cols[2 * pi]};
        const bool second_empty = 2 * pi + 1 >= (int)cols.size();
        for (int l = 0; l < 64; ++l) {
            const int m = l % 16, q = l / 16;
            uint32_t idx = 0;
            for (int gg = 0; gg < 4; ++gg) {
                const int g = 4 * q + gg;
                const int half = g / 8, h = g % 8;
                const int b = cb[half];
                double v[4];
                for (int e = 0; e < 4; ++e) {
                    const int a = sparse_group_row(h, e) - m - R;  // row offset of the weight
                    v[e] = 0.0;
                    if (!(half == 1 && second_empty) && a >= -R && a <= R)
                        v[e] = wc[(size_t)(a + R) * side + (b + R)];
                }
                // the (at most two) non-zero positions, padded with zero
                // weights at free positions, in ascending order
                int pos[2], n = 0;
                for (int e = 0; e < 4 && n < 2; ++e)
                    if (v[e] != 0.0) pos[n++] = e;
                for (int e = 0; e < 4 && n < 2; ++e)
                    if (v[e] == 0.0 && (n == 0 || pos[0] != e)) pos[n++] = e;
                if (pos[0] > pos[1]) std::swap(pos[0], pos[1]);
                for (int s = 0; s < 2; ++s) {
                    const int j = 2 * gg + s;
                    const double x = v[pos[s]];
                    const uint16_t bits = dtype == STENCIL_F16 ? f16_bits(x) : bf16_bits(x);
                    std::memcpy(vals + ((size_t)(pi * 64 + l) * 8 + j) * 2, &bits, 2);
                    idx |= (uint32_t)pos[s] << (2 * j);
                }
            }
            std::memcpy(idxs + (size_t)(pi * 64 + l) * 4, &idx, 4);
        }
    }
}

}  // namespace stl
