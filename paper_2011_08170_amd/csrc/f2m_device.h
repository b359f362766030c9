// Device helpers shared by the HIP sources of libf2m: exact EUC_2D
// rounding, the GDP step, the hash finaliser and wave-level reductions.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace f2m {

// nint(sqrt(D)) exactly: the k with (2k-1)^2 <= 4D < (2k+1)^2 (TSPLIB
// EUC_2D rounding), for 0 <= D < 2^42 (coordinate spans below 2^20 give
// D < 2^41), from an FP32 value Df of D with relative error at most 2^-23.
// The hardware square root is within one ulp, so sqrt(Df) is within
// 2^-23 + 2^-24 + 2^-46 relative of sqrt(D) < 2^21, i.e. within 0.4; adding
// 1/2 in FP32 rounds by at most 1/8, so trunc(sqrt(Df) + 1/2) is within one
// of k, and one integer test each way makes it exact (from k - 1 the upward
// test fires and the downward one does not; from k + 1 only the downward
// one fires).
__device__ __forceinline__ int64_t nint_sqrt_f(int64_t D, float Df)
{
    int64_t k = (int32_t)(__builtin_amdgcn_sqrtf(Df) + 0.5f);
    const int64_t d4 = 4 * D;
    k += (2 * k + 1) * (2 * k + 1) <= d4 ? 1 : 0;
    k -= (k > 0 && (2 * k - 1) * (2 * k - 1) > d4) ? 1 : 0;
    return k;
}

// the same from D alone (the conversion rounds once: relative error 2^-24)
__device__ __forceinline__ int64_t nint_sqrt(int64_t D)
{
    return nint_sqrt_f(D, (float)D);
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
