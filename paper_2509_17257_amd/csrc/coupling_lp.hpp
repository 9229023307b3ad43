// Matrix-core coupling kernels for the low-precision operators (k = 64; k <= 32 below):
//   y_t = sum_{(t,s) in C_t, admissible} S_b x_s     for every row cluster t,
// S_b stored in FP32 or BF16, x-hat and y-hat in FP32, FP32 accumulation.
//
// Same organisation as the FP64 kernel: one work-group (4 waves) per row
// cluster and slab of 16*NJ columns, wave w owns rows 16w..16w+15, S_b streamed
// from HBM one block ahead in the lane order of the MFMA operand (layouts 2 and
// 3 of s_index: one 16-byte load per lane per k-chunk), x_s staged in LDS
// (double-buffered).  Output layout of both 16x16 MFMAs: register q of lane l
// holds row 4 (l / 16) + q, column l % 16.
//
// FP32: v_mfma_f32_16x16x4f32, lane (r, g) takes columns 16a + 4g + h of S_b in
//       k-step 4a + h (h = 0..3), so one float4 load serves four k-steps.
// BF16: v_mfma_f32_16x16x32_bf16, lane (r, g) takes columns 32c + 8g .. + 7 in
//       k-chunk c; x_s comes from a copy of x-hat rounded to BF16 (nearest even; the
//       rounding of the right-hand factor, done once per cluster instead of once per
//       block, and half the bytes of each x_s read) and is kept transposed in LDS so
//       that each lane reads its 8 values at once.
#pragma once

#include <type_traits>

#include "device.hpp"
#include "types.hpp"

namespace h2x {

typedef float flt4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

template <int NJ>
__global__ __launch_bounds__(256) void k_coupling_mfma_f32(int64_t m, int32_t C, int32_t rows_per_xcd,
                                                           const int32_t *__restrict__ order,
                                                           const int64_t *__restrict__ adm_ptr,
                                                           const int32_t *__restrict__ adm_col,
                                                           const float *__restrict__ S, const float *__restrict__ xh,
                                                           float *__restrict__ yh, int64_t ldh, Skip skip) {
    // x_s in LDS, two layouts.  64 columns (TR): transposed (column c of x_s is LDS row c,
    // pitch K + 4 floats), so a lane reads the four rows 16 a + 4 g .. + 3 of its column, the
    // operands of four k-steps, with one 16-byte load (16 lanes of consecutive columns on
    // disjoint banks).  Fewer columns: row-major with pitch MC + 4 floats (the four row groups
    // of one read, rows 4 apart, on disjoint banks), which measured faster there.
    constexpr int K = 64, MC = 16 * NJ, LDX = MC + 4, LDT = K + 4;
    constexpr bool TR = NJ == 4;
    __shared__ __align__(16) float xs[2][TR ? MC * LDT : K * LDX];
    // the column slabs of one row cluster are consecutive work-groups of one XCD, so S_b
    // comes from HBM once and from that XCD's L2 for the other slabs
    const int nslab = (int)((m + MC - 1) / MC), qx = blockIdx.x >> 3;
    const int slot = (blockIdx.x & 7) * rows_per_xcd + qx / nslab;
    if (slot >= C) return;
    const int32_t t = order[slot];
    if (skip(t)) return;
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    const int lr = lane & 15, g = lane >> 4;
    const int64_t j0 = (int64_t)(qx % nslab) * MC;
    const int mc = (int)min<int64_t>(MC, m - j0);
    const int64_t b0 = adm_ptr[t], b1 = adm_ptr[t + 1];

    flt4 acc[NJ];
#pragma unroll
    for (int J = 0; J < NJ; ++J) acc[J] = flt4{0.f, 0.f, 0.f, 0.f};

    if (b1 > b0) {
        // TR: thread = column xc = tid % MC and the XPT consecutive rows from xr0 (global loads
        // read whole row segments, LDS stores are 16 bytes); otherwise element e = tid + 256 u
        // is (row e / MC, column e % MC)
        constexpr int XPT = (K * MC) / 256;
        const int xc = tid % MC, xr0 = (tid / MC) * XPT;
        float xv[XPT];
        auto load_x = [&](int32_t s) {
            if constexpr (TR) {
                const float *src = xh + ((int64_t)s * K + xr0) * ldh + j0 + (xc < mc ? xc : 0);
#pragma unroll
                for (int u = 0; u < XPT; ++u) xv[u] = src[(int64_t)u * ldh];  // columns past mc: zeroed when stored
            } else {
                const float *src = xh + (int64_t)s * K * ldh + j0;
#pragma unroll
                for (int u = 0; u < XPT; ++u) {
                    const int e = tid + 256 * u, r = e / MC, c = e % MC;
                    xv[u] = src[(int64_t)r * ldh + (c < mc ? c : 0)];  // columns past mc: zeroed when stored
                }
            }
        };
        auto store_x = [&](int buf) {
            if constexpr (TR) {
                float *dst = &xs[buf][xc * LDT + xr0];
#pragma unroll
                for (int q = 0; q < XPT / 4; ++q)
                    *(flt4 *)(dst + 4 * q) = xc < mc ? flt4{xv[4 * q], xv[4 * q + 1], xv[4 * q + 2], xv[4 * q + 3]}
                                                     : flt4{0.f, 0.f, 0.f, 0.f};
            } else {
#pragma unroll
                for (int u = 0; u < XPT; ++u) {
                    const int e = tid + 256 * u, r = e / MC, c = e % MC;
                    xs[buf][r * LDX + c] = c < mc ? xv[u] : 0.f;
                }
            }
        };
        flt4 sa[4], sn[4];
        auto load_s = [&](int64_t b, flt4 *dst) {
            const __amdgpu_buffer_rsrc_t rs = buf_rsrc(S + b * K * K, K * K * 4);
#pragma unroll
            for (int a = 0; a < 4; ++a)
                dst[a] = __builtin_bit_cast(flt4, buf_ld16<kBufNT>(rs, 16u * (w * 4 * 64 + a * 64 + lane)));
        };

        // the same order of products per accumulator in both layouts
        auto multiply = [&](int buf) {
            const float *xb = xs[buf];
            if constexpr (TR) {
#pragma unroll
                for (int a = 0; a < 4; ++a)
#pragma unroll
                    for (int J = 0; J < NJ; ++J) {
                        // rows 16 a + 4 g + h (h = 0..3) of column 16 J + lr: k-steps 4 a + h
                        const flt4 bv = *(const flt4 *)(xb + (16 * J + lr) * LDT + 16 * a + 4 * g);
#pragma unroll
                        for (int h = 0; h < 4; ++h)
                            acc[J] = __builtin_amdgcn_mfma_f32_16x16x4f32(sa[a][h], bv[h], acc[J], 0, 0, 0);
                    }
            } else {
#pragma unroll
                for (int a = 0; a < 4; ++a)
#pragma unroll
                    for (int h = 0; h < 4; ++h) {
                        const int krow = 16 * a + 4 * g + h;
#pragma unroll
                        for (int J = 0; J < NJ; ++J)
                            acc[J] = __builtin_amdgcn_mfma_f32_16x16x4f32(sa[a][h], xb[krow * LDX + 16 * J + lr],
                                                                           acc[J], 0, 0, 0);
                    }
            }
        };

        load_x(adm_col[b0]);
        load_s(b0, sa);
        store_x(0);
        __syncthreads();
        // unconditional loads and a peeled last block: the compiler's wait counters stay
        // exact, so the MFMAs never wait for the block being prefetched
        for (int64_t b = b0; b + 1 < b1; ++b) {
            const int buf = (int)((b - b0) & 1);
            load_x(adm_col[b + 1]);
            load_s(b + 1, sn);
            multiply(buf);
            store_x(buf ^ 1);
#pragma unroll
            for (int a = 0; a < 4; ++a) sa[a] = sn[a];
            __syncthreads();
        }
        multiply((int)((b1 - 1 - b0) & 1));
    }
#pragma unroll
    for (int J = 0; J < NJ; ++J) {
        const int col = 16 * J + lr;
        if (col < mc)
#pragma unroll
            for (int q = 0; q < 4; ++q) yh[((int64_t)t * K + 16 * w + 4 * g + q) * ldh + j0 + col] = acc[J][q];
    }
}

template <int NJ>
__global__ __launch_bounds__(256) void k_coupling_mfma_bf16(int64_t m, int32_t C, int32_t rows_per_xcd,
                                                            const int32_t *__restrict__ order,
                                                            const int64_t *__restrict__ adm_ptr,
                                                            const int32_t *__restrict__ adm_col,
                                                            const bf16_t *__restrict__ S,
                                                            const uint16_t *__restrict__ xb, float *__restrict__ yh,
                                                            int64_t ldh, Skip skip) {
    constexpr int K = 64, MC = 16 * NJ;
    constexpr int LDT = K + 8;  // LDS row (one column of x_s) in bf16 units, padded against bank conflicts
    __shared__ __align__(16) uint16_t xs[2][MC * LDT];
    // the column slabs of one row cluster are consecutive work-groups of one XCD, so S_b
    // comes from HBM once and from that XCD's L2 for the other slabs
    const int nslab = (int)((m + MC - 1) / MC), qx = blockIdx.x >> 3;
    const int slot = (blockIdx.x & 7) * rows_per_xcd + qx / nslab;
    if (slot >= C) return;
    const int32_t t = order[slot];
    if (skip(t)) return;
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    const int lr = lane & 15, g = lane >> 4;
    const int64_t j0 = (int64_t)(qx % nslab) * MC;
    const int mc = (int)min<int64_t>(MC, m - j0);
    const int64_t b0 = adm_ptr[t], b1 = adm_ptr[t + 1];

    flt4 acc[NJ];
#pragma unroll
    for (int J = 0; J < NJ; ++J) acc[J] = flt4{0.f, 0.f, 0.f, 0.f};

    if (b1 > b0) {
        // MC dividing 256: thread = column xc = tid % MC of x_s and the XPT consecutive rows
        // from xr0; each global load instruction reads whole row segments (lanes over
        // columns), and the rows go to LDS as 16-byte (8-byte for XPT = 4) stores:
        // consecutive lanes write LDS rows 144 bytes apart, on disjoint banks.  Otherwise
        // (MC = 48) element e = tid + 256 u is (row e / MC, column e % MC), stored one by one.
        constexpr bool VEC = 256 % MC == 0;
        constexpr int XPT = (K * MC) / 256, CH = XPT % 8 == 0 ? 8 : 4;
        static_assert(!VEC || XPT % CH == 0, "rows per thread");
        const int xc = tid % MC, xr0 = (tid / MC) * XPT;
        uint16_t xv[XPT];
        auto load_x = [&](int32_t s) {  // x-hat already rounded to BF16 (k_pack_bf16)
            if constexpr (VEC) {
                const uint16_t *src = xb + ((int64_t)s * K + xr0) * ldh + j0 + (xc < mc ? xc : 0);
#pragma unroll
                for (int u = 0; u < XPT; ++u) xv[u] = src[(int64_t)u * ldh];  // columns past mc: zeroed when stored
            } else {
                const uint16_t *src = xb + (int64_t)s * K * ldh + j0;
#pragma unroll
                for (int u = 0; u < XPT; ++u) {
                    const int e = tid + 256 * u, r = e / MC, c = e % MC;
                    xv[u] = src[(int64_t)r * ldh + (c < mc ? c : 0)];
                }
            }
        };
        auto store_x = [&](int buf) {  // transposed: column c of x_s is LDS row c
            if constexpr (VEC) {
                uint16_t *dst = &xs[buf][xc * LDT + xr0];
#pragma unroll
                for (int q = 0; q < XPT / CH; ++q) {
                    uint32_t d[CH / 2];
#pragma unroll
                    for (int i = 0; i < CH / 2; ++i)
                        d[i] = xc < mc ? (uint32_t)xv[CH * q + 2 * i] | ((uint32_t)xv[CH * q + 2 * i + 1] << 16) : 0u;
                    if constexpr (CH == 8)
                        *(u32x4 *)(dst + CH * q) = u32x4{d[0], d[1], d[2], d[3]};
                    else
                        *(u32x2 *)(dst + CH * q) = u32x2{d[0], d[1]};
                }
            } else {
#pragma unroll
                for (int u = 0; u < XPT; ++u) {
                    const int e = tid + 256 * u, r = e / MC, c = e % MC;
                    xs[buf][c * LDT + r] = c < mc ? xv[u] : (uint16_t)0;
                }
            }
        };
        u32x4 sa[2], sn[2];
        auto load_s = [&](int64_t b, u32x4 *dst) {
            const __amdgpu_buffer_rsrc_t rs = buf_rsrc(S + b * K * K, K * K * 2);
#pragma unroll
            for (int c = 0; c < 2; ++c) dst[c] = buf_ld16<kBufNT>(rs, 16u * (w * 2 * 64 + c * 64 + lane));
        };

        auto multiply = [&](int buf) {
            const uint16_t *xb = xs[buf];
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                const bf16x8 av = __builtin_bit_cast(bf16x8, sa[c]);
#pragma unroll
                for (int J = 0; J < NJ; ++J) {
                    const u32x4 bb = *(const u32x4 *)(xb + (16 * J + lr) * LDT + 32 * c + 8 * g);
                    acc[J] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, __builtin_bit_cast(bf16x8, bb), acc[J], 0,
                                                                      0, 0);
                }
            }
        };

        load_x(adm_col[b0]);
        load_s(b0, sa);
        store_x(0);
        __syncthreads();
        // unconditional loads and a peeled last block, as in the FP32 kernel
        for (int64_t b = b0; b + 1 < b1; ++b) {
            const int buf = (int)((b - b0) & 1);
            load_x(adm_col[b + 1]);
            load_s(b + 1, sn);
            multiply(buf);
            store_x(buf ^ 1);
            sa[0] = sn[0];
            sa[1] = sn[1];
            __syncthreads();
        }
        multiply((int)((b1 - 1 - b0) & 1));
    }
#pragma unroll
    for (int J = 0; J < NJ; ++J) {
        const int col = 16 * J + lr;
        if (col < mc)
#pragma unroll
            for (int q = 0; q < 4; ++q) yh[((int64_t)t * K + 16 * w + 4 * g + q) * ldh + j0 + col] = acc[J][q];
    }
}

// Low-precision coupling for k <= 32 (S_b row-major in FP32 or BF16, x-hat and y-hat in
// FP32, x_s rounded to the storage type, FP32 accumulation on v_mfma_f32_16x16x4f32).
// A work-group of 2 waves owns one row cluster t and a slab of 16*NJ columns; wave w
// owns rows 16w..16w+15 of y_t (rows past k are zero in the operand and never
// written).  Lane (r, g), g = lane / 16, takes
// columns 16a + 4g + h of S_b in k-step 4a + h (h = 0..3), so its four S values of a
// group of k-steps are adjacent in memory; x_s is staged in LDS (double-buffered) and
// read with the same permutation.  A lane past the last column reads column 0 and
// multiplies a zero row of x_s.  S_b is streamed one block ahead; the last block is
// peeled off the loop so that every load is unconditional.
template <int NJ, typename T>
__global__ __launch_bounds__(128) void k_coupling_small_lp(int k, int64_t m, int32_t C, int32_t rows_per_xcd,
                                                           const int32_t *__restrict__ order,
                                                           const int64_t *__restrict__ adm_ptr,
                                                           const int32_t *__restrict__ adm_col,
                                                           const T *__restrict__ S, const float *__restrict__ xh,
                                                           float *__restrict__ yh, int64_t ldh, Skip skip) {
    // LDS row pitch MC + 4 floats: the four row groups of one read (rows 4 apart) on disjoint banks
    constexpr int MC = 16 * NJ, LDX = MC + 4;
    __shared__ float xs[2][32 * LDX];
    const int nslab = (int)((m + MC - 1) / MC), qx = blockIdx.x >> 3;
    const int slot = (blockIdx.x & 7) * rows_per_xcd + qx / nslab;
    if (slot >= C) return;
    const int32_t t = order[slot];
    if (skip(t)) return;
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    const int lr = lane & 15, g = lane >> 4;
    const int64_t j0 = (int64_t)(qx % nslab) * MC;
    const int mc = (int)min<int64_t>(MC, m - j0);
    const int64_t b0 = adm_ptr[t], b1 = adm_ptr[t + 1];
    const int na = (k + 15) >> 4;  // groups of four k-steps (16 columns of S each)
    const int nu = 16 * w + lr;    // row of S_b held by this lane
    const bool row_ok = nu < k;

    flt4 acc[NJ];
#pragma unroll
    for (int J = 0; J < NJ; ++J) acc[J] = flt4{0.f, 0.f, 0.f, 0.f};

    if (b1 > b0) {
        constexpr int XPT = (32 * MC) / 128;  // x_s elements per thread (4 * NJ)
        float xv[XPT];
        auto load_x = [&](int32_t s) {
            const float *src = xh + (int64_t)s * k * ldh + j0;
#pragma unroll
            for (int u = 0; u < XPT; ++u) {
                const int e = tid + 128 * u, r = e / MC, c = e % MC;
                xv[u] = src[(r < k && c < mc) ? (int64_t)r * ldh + c : 0];  // zeroed when stored
            }
        };
        // the right-hand factor is rounded to the storage type (BF16: nearest even) as staged
        auto store_x = [&](int buf) {
#pragma unroll
            for (int u = 0; u < XPT; ++u) {
                const int e = tid + 128 * u, r = e / MC, c = e % MC;
                float v = xv[u];
                if constexpr (std::is_same<T, bf16_t>::value) v = to_float(bf16_t{bf16_bits(v)});
                xs[buf][r * LDX + c] = (r < k && c < mc) ? v : 0.f;
            }
        };
        float sa[2][4], sn[2][4];
        auto load_s = [&](int64_t b, float (*dst)[4]) {
            const T *src = S + b * k * k + (int64_t)(row_ok ? nu : 0) * k;
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int h = 0; h < 4; ++h) {
                    const int mu = 16 * a + 4 * g + h;
                    dst[a][h] = to_float(src[(row_ok && mu < k) ? mu : 0]);
                }
        };
        auto multiply = [&](int buf) {
            const float *xb = xs[buf];
#pragma unroll
            for (int a = 0; a < 2; ++a) {
                if (a < na) {
#pragma unroll
                    for (int h = 0; h < 4; ++h) {
                        const int krow = 16 * a + 4 * g + h;
#pragma unroll
                        for (int J = 0; J < NJ; ++J)
                            acc[J] = __builtin_amdgcn_mfma_f32_16x16x4f32(sa[a][h], xb[krow * LDX + 16 * J + lr],
                                                                          acc[J], 0, 0, 0);
                    }
                }
            }
        };

        load_x(adm_col[b0]);
        load_s(b0, sa);
        store_x(0);
        __syncthreads();
        for (int64_t b = b0; b + 1 < b1; ++b) {
            const int buf = (int)((b - b0) & 1);
            load_x(adm_col[b + 1]);
            load_s(b + 1, sn);
            multiply(buf);
            store_x(buf ^ 1);
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int h = 0; h < 4; ++h) sa[a][h] = sn[a][h];
            __syncthreads();
        }
        multiply((int)((b1 - 1 - b0) & 1));
    }
    // output layout of v_mfma_f32_16x16x4f32: register q of lane l holds row 4 (l / 16) + q,
    // column l % 16
#pragma unroll
    for (int J = 0; J < NJ; ++J) {
        const int col = 16 * J + lr;
        if (col < mc) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int row = 16 * w + 4 * g + q;
                if (row < k) yh[((int64_t)t * k + row) * ldh + j0 + col] = acc[J][q];
            }
        }
    }
}

// Launches the low-precision matrix-core coupling when the layout supports it.
// xb: x-hat rounded to BF16 in the layout of xh (BF16 storage with k = 64; else unused)
template <typename T>
bool launch_coupling_lp(const DevMat &dm, int64_t m, const float *xh, const uint16_t *xb, float *yh, int64_t ldh,
                        hipStream_t st, Skip skip, int nj_force) {
    const bool f32 = std::is_same<T, float>::value;
    if (!dm.cpl_order) return false;
    const int nj = nj_force ? nj_force : (int)std::min<int64_t>(4, (m + 15) / 16);
    const int32_t rpx = (dm.C + 7) / 8;
    const dim3 grid((unsigned)(8 * rpx * ((m + 16 * nj - 1) / (16 * nj))));
    if (dm.k <= 32) {
        if (dm.swz != 0) return false;
        auto go = [&](auto NJc) {
            constexpr int NJ = decltype(NJc)::value;
            hipLaunchKernelGGL((k_coupling_small_lp<NJ, T>), grid, dim3(128), 0, st, dm.k, m, dm.C, rpx,
                               dm.cpl_order, dm.adm_ptr, dm.adm_col, (const T *)dm.S, xh, yh, ldh, skip);
        };
        switch (nj) {
            case 1: go(std::integral_constant<int, 1>{}); break;
            case 2: go(std::integral_constant<int, 2>{}); break;
            case 3: go(std::integral_constant<int, 3>{}); break;
            default: go(std::integral_constant<int, 4>{}); break;
        }
        return true;
    }
    if (dm.k != 64 || dm.swz != (f32 ? 2 : 3)) return false;
    auto go = [&](auto NJc) {
        constexpr int NJ = decltype(NJc)::value;
        if constexpr (std::is_same<T, float>::value)
            hipLaunchKernelGGL(k_coupling_mfma_f32<NJ>, grid, dim3(256), 0, st, m, dm.C, rpx, dm.cpl_order,
                               dm.adm_ptr, dm.adm_col, (const float *)dm.S, xh, yh, ldh, skip);
        else
            hipLaunchKernelGGL(k_coupling_mfma_bf16<NJ>, grid, dim3(256), 0, st, m, dm.C, rpx, dm.cpl_order,
                               dm.adm_ptr, dm.adm_col, (const bf16_t *)dm.S, xb, yh, ldh, skip);
    };
    switch (nj) {
        case 1: go(std::integral_constant<int, 1>{}); break;
        case 2: go(std::integral_constant<int, 2>{}); break;
        case 3: go(std::integral_constant<int, 3>{}); break;
        default: go(std::integral_constant<int, 4>{}); break;
    }
    return true;
}

}  // namespace h2x
