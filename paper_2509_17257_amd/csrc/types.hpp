// Element types of the stored operator and the coupling-matrix storage layout.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace h2x {

// bfloat16 held as raw bits.  Conversion from FP64: round to FP32 (nearest
// even), then to bfloat16 (nearest even); NaN stays NaN.
struct bf16_t {
    uint16_t b;
};

template <typename T>
__host__ __device__ inline T from_double(double v);

template <>
__host__ __device__ inline double from_double<double>(double v) { return v; }
template <>
__host__ __device__ inline float from_double<float>(double v) { return (float)v; }
// FP32 -> bfloat16 bits, round to nearest even; NaN stays NaN
__host__ __device__ inline uint16_t bf16_bits(float f) {
    uint32_t u = __builtin_bit_cast(uint32_t, f);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return (uint16_t)((u >> 16) | 0x40);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

template <>
__host__ __device__ inline bf16_t from_double<bf16_t>(double v) {
    return bf16_t{bf16_bits((float)v)};
}

__host__ __device__ inline float to_float(double v) { return (float)v; }
__host__ __device__ inline float to_float(float v) { return v; }
__host__ __device__ inline float to_float(bf16_t v) { return __builtin_bit_cast(float, (uint32_t)v.b << 16); }
__host__ __device__ inline double to_double(double v) { return v; }
__host__ __device__ inline double to_double(float v) { return v; }
__host__ __device__ inline double to_double(bf16_t v) { return (double)to_float(v); }

// Coupling matrices: layout 0 is row-major k x k; layouts 2 (FP32) and 3 (BF16),
// for k = 64, put the 16 bytes one lane of the low-precision matrix-core kernels
// reads for one (16-row tile, k-chunk) next to each other, 64 lanes in order.  Layout 1 (k a multiple of
// 16) is the operand order of the FP64 matrix-core coupling kernel: for each
// 16-row tile I and each pair of 4-column steps, the 64 lanes of a wave read
// 2 consecutive doubles each (one 16-byte load per lane).  Within a tile
// (I, kk2), lane l = 16 * q + r holds S[16 I + r, 8 kk2 + 4 h + q] at slot h.
__host__ __device__ inline int64_t s_index(int swz, int k, int nu, int mu) {
    if (swz == 0) return (int64_t)nu * k + mu;
    const int I = nu >> 4, r = nu & 15;
    if (swz == 2) {  // FP32: lane 16 g + r holds S[16 I + r, 16 a + 4 g + h], h = 0..3
        const int a = mu >> 4, g = (mu >> 2) & 3, h = mu & 3;
        return (((int64_t)I * (k >> 4) + a) * 64 + 16 * g + r) * 4 + h;
    }
    if (swz == 3) {  // BF16: lane 16 g + r holds S[16 I + r, 32 c + 8 g + e], e = 0..7
        const int c = mu >> 5, g = (mu >> 3) & 3, e = mu & 7;
        return (((int64_t)I * (k >> 5) + c) * 64 + 16 * g + r) * 8 + e;
    }
    const int kk2 = mu >> 3, h = (mu >> 2) & 1, q = mu & 3;
    const int lane = 16 * q + r;
    const int tiles_k2 = k >> 3;
    return (((int64_t)I * tiles_k2 + kk2) * 64 + lane) * 2 + h;
}

}  // namespace h2x
