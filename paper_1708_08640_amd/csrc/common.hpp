// Shared device helpers for the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define S3_DEV __device__ __forceinline__

namespace s3 {

constexpr int kWave = 64;

template <typename T> S3_DEV T fmaT(T a, T b, T c) { return __builtin_fma(a, b, c); }
template <> S3_DEV float fmaT<float>(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// full-wave butterfly sum in a fixed order (deterministic for a given input)
template <typename T> S3_DEV T wave_sum(T v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

}  // namespace s3
