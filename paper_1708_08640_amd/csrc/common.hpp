// Shared device helpers for the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define S3_DEV __device__ __forceinline__

namespace s3 {

constexpr int kWave = 64;

template <typename T> S3_DEV T fmaT(T a, T b, T c) { return __builtin_fma(a, b, c); }
template <> S3_DEV float fmaT<float>(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// bf16 <-> f32, round to nearest even (finite inputs; NaN kept quiet).
S3_DEV uint16_t f32_to_bf16_rne(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u) {  // inf / nan
        return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
    }
    uint32_t lsb = (u >> 16) & 1u;
    u += 0x7fffu + lsb;
    return (uint16_t)(u >> 16);
}
S3_DEV float bf16_to_f32(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }

// full-wave butterfly sum in a fixed order (deterministic for a given input)
template <typename T> S3_DEV T wave_sum(T v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

}  // namespace s3
