// Device helpers shared by the vector-unit kernels.
#pragma once

#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <cstdint>

namespace stl {

// Number of XCDs of the chip: consecutive workgroup ids are dealt round-robin
// to the XCDs, each of which has its own L2.
constexpr int kNumXcd = 8;

// Map a workgroup id to a tile id so that the workgroups resident on one XCD
// process a contiguous run of tiles (neighbouring tiles share halo lines in
// that XCD's L2).  Bijective on [0, nb).
__device__ __forceinline__ int xcd_remap(int bid, int nb)
{
    const int per = nb / kNumXcd;
    if (bid >= per * kNumXcd) return bid;
    return (bid % kNumXcd) * per + bid / kNumXcd;
}

__device__ __forceinline__ int wrap(int i, int n)
{
    int m = i % n;
    return m < 0 ? m + n : m;
}

// wrap for -n <= i < 2n (a halo no wider than the grid): no division
__device__ __forceinline__ int wrap1(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

__device__ __forceinline__ double fma_c(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fma_c(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

template <typename TS> __device__ __forceinline__ TS to_storage(double v);
template <typename TS> __device__ __forceinline__ TS to_storage(float v);
template <> __device__ __forceinline__ double to_storage<double>(double v) { return v; }
template <> __device__ __forceinline__ float to_storage<float>(double v) { return (float)v; }
template <> __device__ __forceinline__ float to_storage<float>(float v) { return v; }
template <> __device__ __forceinline__ double to_storage<double>(float v) { return (double)v; }
template <> __device__ __forceinline__ __hip_bfloat16 to_storage<__hip_bfloat16>(float v) { return __float2bfloat16(v); }
template <> __device__ __forceinline__ __hip_bfloat16 to_storage<__hip_bfloat16>(double v) { return __float2bfloat16((float)v); }
template <> __device__ __forceinline__ __half to_storage<__half>(float v) { return __float2half(v); }
template <> __device__ __forceinline__ __half to_storage<__half>(double v) { return __float2half((float)v); }

template <typename TC> __device__ __forceinline__ TC to_compute(double v) { return (TC)v; }
template <typename TC> __device__ __forceinline__ TC to_compute(float v) { return (TC)v; }
template <typename TC> __device__ __forceinline__ TC to_compute(__hip_bfloat16 v) { return (TC)__bfloat162float(v); }
template <typename TC> __device__ __forceinline__ TC to_compute(__half v) { return (TC)__half2float(v); }

// W consecutive storage elements moved with 16-byte accesses when aligned
// (one, or two for 32 bytes).
template <typename TS, int W>
struct RawVec {
    TS e[W];
    __device__ __forceinline__ void load(const TS *p)
    {
        static_assert(sizeof(TS) * W == 32 || sizeof(TS) * W == 16 || sizeof(TS) * W == 8 || sizeof(TS) * W == 4,
                      "vector width");
        if constexpr (sizeof(TS) * W == 32) {
            const uint4 v0 = reinterpret_cast<const uint4 *>(p)[0];
            const uint4 v1 = reinterpret_cast<const uint4 *>(p)[1];
            __builtin_memcpy(e, &v0, 16);
            __builtin_memcpy(reinterpret_cast<char *>(e) + 16, &v1, 16);
        } else if constexpr (sizeof(TS) * W == 16) {
            const uint4 v = *reinterpret_cast<const uint4 *>(p);
            __builtin_memcpy(e, &v, 16);
        } else if constexpr (sizeof(TS) * W == 8) {
            const uint2 v = *reinterpret_cast<const uint2 *>(p);
            __builtin_memcpy(e, &v, 8);
        } else {
            const uint32_t v = *reinterpret_cast<const uint32_t *>(p);
            __builtin_memcpy(e, &v, 4);
        }
    }
    __device__ __forceinline__ void store(TS *p) const
    {
        if constexpr (sizeof(TS) * W == 32) {
            uint4 v0, v1;
            __builtin_memcpy(&v0, e, 16);
            __builtin_memcpy(&v1, reinterpret_cast<const char *>(e) + 16, 16);
            reinterpret_cast<uint4 *>(p)[0] = v0;
            reinterpret_cast<uint4 *>(p)[1] = v1;
        } else if constexpr (sizeof(TS) * W == 16) {
            uint4 v;
            __builtin_memcpy(&v, e, 16);
            *reinterpret_cast<uint4 *>(p) = v;
        } else if constexpr (sizeof(TS) * W == 8) {
            uint2 v;
            __builtin_memcpy(&v, e, 8);
            *reinterpret_cast<uint2 *>(p) = v;
        } else {
            uint32_t v;
            __builtin_memcpy(&v, e, 4);
            *reinterpret_cast<uint32_t *>(p) = v;
        }
    }
};

// True when the W elements starting at column cb of every row are one aligned
// vector: base aligned, row pitch a multiple of the vector, cb a multiple of W.
template <typename TS, int W>
__device__ __forceinline__ bool vec_aligned(const void *base, int n1, int cb)
{
    const int m = ((cb % W) + W) % W;
    return ((reinterpret_cast<uintptr_t>(base) % (sizeof(TS) * W)) == 0) &&
           ((int64_t(n1) * sizeof(TS)) % (sizeof(TS) * W) == 0) && m == 0;
}

}  // namespace stl
