// Device helpers shared by the HIP sources of libf2m: exact EUC_2D
// rounding, the GDP step, the hash finaliser and wave-level reductions.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace f2m {

// nint(sqrt(D)) exactly: the k with (2k-1)^2 <= 4D < (2k+1)^2 (TSPLIB
// EUC_2D rounding).  sqrtf gives k within one; the loops make it exact.
__device__ __forceinline__ int64_t nint_sqrt(int64_t D)
{
    const float f = sqrtf((float)D);
    int64_t k = (int64_t)(f + 0.5f);
    const int64_t d4 = 4 * D;
    while ((2 * k + 1) * (2 * k + 1) <= d4) ++k;
    while (k > 0 && (2 * k - 1) * (2 * k - 1) > d4) --k;
    return k;
}

// dLam = sign(s) * floor((|s| + 2) / 4)
__device__ __forceinline__ int64_t gdp_step(int64_t s)
{
    if (s > 0) return (s + 2) >> 2;
    if (s < 0) return -((-s + 2) >> 2);
    return 0;
}

// SplitMix64 output finaliser (Steele, Lea, Flood 2014)
__device__ __forceinline__ uint64_t mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

template <typename T>
__device__ __forceinline__ T wave_sum(T x)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    return x;
}

template <typename T>
__device__ __forceinline__ T wave_max(T x)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const T y = __shfl_xor(x, o, 64);
        x = y > x ? y : x;
    }
    return x;
}

template <typename T>
__device__ __forceinline__ T wave_min(T x)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const T y = __shfl_xor(x, o, 64);
        x = y < x ? y : x;
    }
    return x;
}

// Orders the LDS accesses of one wave (no other wave takes part).
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

}  // namespace f2m
