// Precision conversions shared by the pack, gather and reduce kernels.
// All conversions round to nearest even; FP64 -> BF16 goes through FP32.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace hm {

__host__ __device__ inline uint16_t f32_to_bf16_bits(float f)
{
    uint32_t u;
    __builtin_memcpy(&u, &f, 4);
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__host__ __device__ inline float bf16_bits_to_f32(uint16_t h)
{
    uint32_t u = (uint32_t)h << 16;
    float f;
    __builtin_memcpy(&f, &u, 4);
    return f;
}

template <class T>
__host__ __device__ inline T cvt(double v);
template <>
__host__ __device__ inline double cvt<double>(double v) { return v; }
template <>
__host__ __device__ inline float cvt<float>(double v) { return (float)v; }
template <>
__host__ __device__ inline uint16_t cvt<uint16_t>(double v) { return f32_to_bf16_bits((float)v); }

}  // namespace hm
