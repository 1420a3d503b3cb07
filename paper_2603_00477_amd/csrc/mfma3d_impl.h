// MFMA path, d = 3: the T-step composite kernel applied once per pass as
// banded Toeplitz products, one per non-zero (plane offset c, column b) pair:
//   out[z][16x16 tile] += A_{c,b}[16 x Kp] . X_{c,b}[Kp x 16],
//   A_{c,b}[m][k] = w_t[c][k - m - R][b],  X_{c,b}[k][n] = u[z+c][y0-R+k][x0+n+b].
//
// A workgroup (NW waves side by side, one 16 x 16 tile each) owns a 16 x 16NW
// in-plane tile and streams a segment of output planes.  Input planes pass
// through an LDS ring of 2R+1 plane tiles (halo included, boundary rule
// applied); the plane for the next iteration is fetched into registers while
// the current one is used.  Output plane z reads ring slots z-R .. z+R.
#pragma once

#include "mfma2d_impl.h"

namespace stl {

struct Mfma3DArgs {
    const void *src;
    void *dst;
    const void *afrag;
    const void *afrag_lo;
    int n0, n1, n2;
    int BZ, nty, ntx, nzs, ntiles;
    int periodic;
    double h;
};

template <int DT, int SHAPE, int r, int T, int NW>
struct Mfma3DCfg {
    using MT = MfmaTypes<DT>;
    static constexpr int KDIM = MT::KDIM;
    static constexpr int R = r * T;
    static constexpr int Q = 2 * R + 1;
    static constexpr int TY = 16, TXC = 16 * NW;  // output tile
    static constexpr int LRD = TY + 2 * R;         // data rows per plane
    static constexpr int LC = TXC + 2 * R;         // data columns per plane
    static constexpr int KKH = band_kk_hi(SHAPE, r, T, 0, 0, KDIM);
    static constexpr int LRK = KDIM * (KKH + 1);
    static constexpr int LR0 = LRD > LRK ? LRD : LRK;
    static constexpr int LR = ((LR0 + 7) / 8) * 8;
    static constexpr int LCP = LC + ((LC % 32) == 0 ? 1 : 0);
    static constexpr int PLANE = KDIM == 4 ? LR * LCP : LC * LR;  // elements per ring slot
    static constexpr int NT = 64 * NW;
    static constexpr int PER_THREAD = (LRD * LC + NT - 1) / NT;   // data elements a thread stages
};

template <int DT, int SHAPE, int r, int T, int NW>
__global__ __launch_bounds__(64 * NW) void mfma3d_kernel(Mfma3DArgs a)
{
    using Cfg = Mfma3DCfg<DT, SHAPE, r, T, NW>;
    using MT = typename Cfg::MT;
    using TS = typename MT::TS;
    using OP = typename MT::OP;
    using FR = typename MT::FR;
    using ACC = typename MT::ACC;
    constexpr int KDIM = Cfg::KDIM, R = Cfg::R, Q = Cfg::Q;
    constexpr int LR = Cfg::LR, LRD = Cfg::LRD, LC = Cfg::LC, LCP = Cfg::LCP;
    constexpr int PLANE = Cfg::PLANE, NT = Cfg::NT, PT = Cfg::PER_THREAD;
    constexpr bool X3 = MT::X3;
    using SV = decltype(load_val(TS{}));  // staged value type (float or double)

    __shared__ __attribute__((aligned(16))) OP ring[Q * PLANE];
    __shared__ __attribute__((aligned(16))) OP ring_lo[X3 ? Q * PLANE : 1];

    const int tid = threadIdx.x;
    const int tile = xcd_remap(blockIdx.x, gridDim.x);
    if (tile >= a.ntiles) return;
    const int tzs = tile / (a.nty * a.ntx);
    const int rem = tile - tzs * (a.nty * a.ntx);
    const int tyi = rem / a.ntx, txi = rem - tyi * a.ntx;
    const int y0 = tyi * Cfg::TY, x0 = txi * Cfg::TXC;
    const int z0 = tzs * a.BZ;
    const int z1 = min(z0 + a.BZ, a.n0);
    const int n0 = a.n0, n1 = a.n1, n2 = a.n2;
    const bool periodic = a.periodic != 0;
    const TS *src = static_cast<const TS *>(a.src);
    TS *dst = static_cast<TS *>(a.dst);

    // zero the ring once: rows beyond the data rows are read by the last
    // k-blocks and must hold zeros
    for (int i = tid; i < Q * PLANE; i += NT) {
        ring[i] = OP(0);
        if constexpr (X3) ring_lo[i] = OP(0);
    }

    // this thread's staging slots: element e = tid + i*NT of the LRD x LC block
    auto fetch = [&](int z, SV (&v)[PT]) {
        const bool zin = z >= 0 && z < n0;
        const int zz = periodic ? wrap1(z, n0) : z;  // every dim >= 2R + 1: one fold suffices
#pragma unroll
        for (int i = 0; i < PT; ++i) {
            const int e = tid + i * NT;
            v[i] = SV(a.h);
            if (e >= LRD * LC) continue;
            const int row = e / LC, col = e - (e / LC) * LC;
            int gy = y0 - R + row, gx = x0 - R + col;
            const bool in = zin && gy >= 0 && gy < n1 && gx >= 0 && gx < n2;
            // points past n + R feed only unstored outputs of partial tiles;
            // the rest lie in [-R, n + R), where one fold wraps
            const bool used = gy < n1 + R && gx < n2 + R;
            if (in || (periodic && used)) {
                gy = wrap1(gy, n1);
                gx = wrap1(gx, n2);
                v[i] = load_val(src[((int64_t)zz * n1 + gy) * n2 + gx]);
            }
        }
    };
    auto stash = [&](int slot, const SV (&v)[PT]) {
        OP *pl = ring + slot * PLANE;
#pragma unroll
        for (int i = 0; i < PT; ++i) {
            const int e = tid + i * NT;
            if (e >= LRD * LC) continue;
            const int row = e / LC, col = e - (e / LC) * LC;
            const int li = KDIM == 4 ? row * LCP + col : col * LR + row;
            if constexpr (X3) {
                const float f = (float)v[i];
                const OP hi = (OP)f;
                pl[li] = hi;
                ring_lo[slot * PLANE + li] = (OP)(f - (float)hi);
            } else {
                pl[li] = (OP)v[i];
            }
        }
    };

    const int lane = tid & 63, wave = tid >> 6;
    const int lg = lane >> 4, ln = lane & 15;
    const int wc0 = 16 * wave;
    const FR *afr = static_cast<const FR *>(a.afrag);
    const FR *afr_lo = static_cast<const FR *>(a.afrag_lo);

    const int KTOT = (z1 - z0) + 2 * R;
    SV nxt[PT];
    fetch(z0 - R, nxt);
    __syncthreads();  // ring zeroed
    for (int k = 0; k < KTOT; ++k) {
        stash(k % Q, nxt);
        if (k + 1 < KTOT) fetch(z0 - R + k + 1, nxt);
        __syncthreads();
        if (k >= 2 * R) {
            const int zo = z0 + k - 2 * R;
            ACC acc = ACC{};
#pragma unroll
            for (int c = -R; c <= R; ++c) {
                // keep the operand loads of plane offset c after those of c-1
                // (bounds their live ranges in the fully unrolled loop)
                asm volatile("" ::: "memory");
                const int slot = (k - R + c) % Q;
                const OP *pl = ring + slot * PLANE;
                const OP *pl_lo = ring_lo + (X3 ? slot * PLANE : 0);
#pragma unroll
                for (int b = -R; b <= R; ++b) {
                    const int amax = band_amax(SHAPE, r, T, c, b);
                    if (amax < 0) continue;
                    // opaque per-column operand base: stops the ~K_T per-lane
                    // fragment addresses from being hoisted out of the plane loop
                    const FR *ab = afr + lane;
                    const FR *ab_lo = afr_lo + lane;
                    asm volatile("" : "+v"(ab), "+v"(ab_lo)::"memory");
                    const int klo = band_kk_lo(SHAPE, r, T, c, b, KDIM);
                    const int khi = band_kk_hi(SHAPE, r, T, c, b, KDIM);
                    const int off = band_frag_offset(SHAPE, r, T, c, b, KDIM, 3);
                    const int col = wc0 + ln + b + R;
#pragma unroll
                    for (int kk = klo; kk <= khi; ++kk) {
                        const FR A = ab[(off + kk - klo) * 64];
                        FR B;
                        if constexpr (KDIM == 4) {
                            B = pl[(4 * kk + lg) * LCP + col];
                        } else {
                            B = *reinterpret_cast<const FR *>(&pl[col * LR + KDIM * kk + 8 * lg]);
                        }
                        acc = mfma16(A, B, acc);
                        if constexpr (X3) {
                            const FR Al = ab_lo[(off + kk - klo) * 64];
                            const FR Bl = *reinterpret_cast<const FR *>(&pl_lo[col * LR + KDIM * kk + 8 * lg]);
                            acc = mfma16(A, Bl, acc);
                            acc = mfma16(Al, B, acc);
                        }
                    }
                }
            }
            const int gx = x0 + wc0 + ln;
            if (gx < n2) {
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int gy = y0 + (MT::D_ROW_INTERLEAVED ? 4 * e + lg : 4 * lg + e);
                    if (gy < n1) dst[((int64_t)zo * n1 + gy) * n2 + gx] = to_storage<TS>(acc[e]);
                }
            }
        }
        __syncthreads();  // slot (k+1) % Q is overwritten next iteration
    }
}

template <int DT, int SHAPE, int r, int T>
struct Mfma3DShape {
    // four 16-column waves unless the plane ring would not fit in LDS
    static constexpr int bytes4 = Mfma3DCfg<DT, SHAPE, r, T, 4>::Q * Mfma3DCfg<DT, SHAPE, r, T, 4>::PLANE *
                                  (int)sizeof(typename MfmaTypes<DT>::OP) * (MfmaTypes<DT>::X3 ? 2 : 1);
    static constexpr int NW = bytes4 <= 144 * 1024 ? 4 : 2;
};

template <int DT, int SHAPE, int r, int T>
hipError_t launch_mfma3d(const PassArgs &p, hipStream_t stream)
{
    constexpr int NW = Mfma3DShape<DT, SHAPE, r, T>::NW;
    using Cfg = Mfma3DCfg<DT, SHAPE, r, T, NW>;
    if (p.steps != T || !p.afrag) return hipErrorInvalidValue;
    if (MfmaTypes<DT>::X3 && !p.afrag_lo) return hipErrorInvalidValue;
    Mfma3DArgs a;
    a.src = p.src;
    a.dst = p.dst;
    a.afrag = p.afrag;
    a.afrag_lo = p.afrag_lo;
    a.n0 = (int)p.dims[0];
    a.n1 = (int)p.dims[1];
    a.n2 = (int)p.dims[2];
    a.periodic = p.boundary == STENCIL_PERIODIC;
    a.h = p.halo;
    a.nty = (a.n1 + Cfg::TY - 1) / Cfg::TY;
    a.ntx = (a.n2 + Cfg::TXC - 1) / Cfg::TXC;
    const int inplane = a.nty * a.ntx;
    const int target = 4 * (p.num_cu > 0 ? p.num_cu : 256);
    const int segs = (target + inplane - 1) / inplane;
    int BZ = (a.n0 + segs - 1) / segs;
    if (BZ < 4 * Cfg::R) BZ = 4 * Cfg::R;
    if (BZ < 8) BZ = 8;
    a.BZ = BZ;
    a.nzs = (a.n0 + BZ - 1) / BZ;
    const int64_t nt = (int64_t)a.nzs * inplane;
    if (nt > (1LL << 30)) return hipErrorInvalidValue;
    a.ntiles = (int)nt;
    hipLaunchKernelGGL((mfma3d_kernel<DT, SHAPE, r, T, NW>), dim3(a.ntiles), dim3(64 * NW), 0, stream, a);
    return hipGetLastError();
}

#define M3(DT, SH, R, T) {STENCIL_PATH_MFMA, DT, SH, 3, R, T, &launch_mfma3d<DT, SH, R, T>, nullptr}
// combinations whose Dirichlet band fix-up has a fused VALU kernel
#define M3_S(DT)                                                                            \
    M3(DT, STENCIL_STAR, 1, 1), M3(DT, STENCIL_STAR, 1, 2), M3(DT, STENCIL_STAR, 1, 3),     \
        M3(DT, STENCIL_STAR, 2, 1), M3(DT, STENCIL_STAR, 2, 2), M3(DT, STENCIL_STAR, 2, 3), \
        M3(DT, STENCIL_BOX, 1, 1), M3(DT, STENCIL_BOX, 1, 2), M3(DT, STENCIL_BOX, 1, 3)

}  // namespace stl
