// Host construction of the MFMA path's weight operands.
//
// For every structurally non-zero (column, k-block) of the band layout the
// 64 lanes' A-operand elements are written in the order the matrix
// instruction consumes them: lane l holds A[m = l % 16][k = kk*KDIM +
// (l / 16)*KPL + e], e < KPL = KDIM / 4.  Values come from the composite
// kernel of `steps` fused steps, composed in float64 and rounded once to the
// operand type (round to nearest even).  The compensated mode stores
// hi = bf16(w) and lo = bf16(w - hi).

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

}  // namespace stl
