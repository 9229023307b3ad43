// Matrix-core transfer passes and forward leaf transform for the low-precision operators
// (k = 64 or k <= 32):
// E stored in FP32 or BF16, x-hat and y-hat in FP32, the right-hand factor rounded
// to the storage type, FP32 accumulation on v_mfma_f32_16x16x4f32.
//   upward:   x_t = E_{t0}^T x_{t0} + E_{t1}^T x_{t1}   (inner clusters of one depth)
//   downward: y_c += E_c y_{parent(c)}                 (clusters of one depth)
//
// One work-group of 4 waves per (cluster, slab of 16 NJT columns: 32, or 64 for the downward
// pass at k = 64 when m > 32); wave w owns rows
// 16w..16w+15 of the result (a wave whose rows all lie past k has nothing to do).
// Both operands go straight from memory into registers in the lane order of the
// instruction (lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16] of a 4-long
// contraction step): upward, 16 lanes read 16 consecutive entries of a row of E_s
// and of x_s; downward, 16 lanes read 16 rows of E_c (one 64-byte line of each row
// serves four steps).  All KS steps of a term are loaded at once from clamped
// addresses; contraction indices past k multiply zeros of B.  Output layout: register
// q of lane l holds row 4 (l / 16) + q, column l % 16.
#pragma once

#include <type_traits>

#include "device.hpp"
#include "types.hpp"

namespace h2x {
namespace tlp {

typedef float flt4 __attribute__((ext_vector_type(4)));
constexpr int kCols = 32;  // columns per work-group (two 16-column tiles)

template <typename T>
__device__ inline float round_to(float v) {
    if constexpr (std::is_same<T, bf16_t>::value) return to_float(bf16_t{bf16_bits(v)});
    return v;
}

// acc[J] += A B over one term: A row r of the tile = arow(r, a), B = x[a][j0 + 16J + lr],
// contraction a = 0 .. k-1 in KS steps of 4; NJT 16-column tiles
template <int KS, typename T, int NJT = 2, typename FA>
__device__ inline void term(int k, int lr, int g, FA arow, const float *__restrict__ xs, int64_t ldh, int mc,
                            flt4 (&acc)[NJT]) {
    float av[KS], bv[KS][NJT];
#pragma unroll
    for (int st = 0; st < KS; ++st) {
        const int a = min(4 * st + g, k - 1);
        av[st] = to_float(*arow(a));
#pragma unroll
        for (int J = 0; J < NJT; ++J) bv[st][J] = xs[(int64_t)a * ldh + min(16 * J + lr, mc - 1)];
    }
#pragma unroll
    for (int st = 0; st < KS; ++st) {
        const bool in = 4 * st + g < k;
#pragma unroll
        for (int J = 0; J < NJT; ++J) {
            const float b = in ? round_to<T>(bv[st][J]) : 0.f;
            acc[J] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[st], b, acc[J], 0, 0, 0);
        }
    }
}

template <int KS, typename T, int NJT = 2>
__global__ __launch_bounds__(256) void k_up_lp(int k, int64_t m, const int32_t *__restrict__ list,
                                               const int32_t *__restrict__ son0, const int32_t *__restrict__ son1,
                                               const T *__restrict__ E, float *__restrict__ xh, int64_t ldh) {
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, lr = lane & 15, g = lane >> 4;
    if (16 * w >= k) return;
    const int32_t t = list[blockIdx.x];
    const int64_t j0 = (int64_t)blockIdx.y * 16 * NJT;
    const int mc = (int)min<int64_t>(16 * NJT, m - j0);
    const int nu = min(16 * w + lr, k - 1);  // row of x_t (column of E_s) this lane supplies
    flt4 acc[NJT];
#pragma unroll
    for (int J = 0; J < NJT; ++J) acc[J] = flt4{0.f, 0.f, 0.f, 0.f};
    const int32_t sons[2] = {son0[t], son1[t]};
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int32_t s = sons[q];
        const T *Es = E + (int64_t)s * k * k;
        term<KS, T, NJT>(k, lr, g, [&](int a) { return Es + (int64_t)a * k + nu; }, xh + (int64_t)s * k * ldh + j0,
                         ldh, mc, acc);
    }
#pragma unroll
    for (int J = 0; J < NJT; ++J) {
        const int col = 16 * J + lr;
        if (col < mc)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = 16 * w + 4 * g + r;
                if (row < k) xh[((int64_t)t * k + row) * ldh + j0 + col] = acc[J][r];
            }
    }
}

template <int KS, typename T, int NJT = 2>
__global__ __launch_bounds__(256) void k_down_lp(int k, int64_t m, const int32_t *__restrict__ list,
                                                 const int32_t *__restrict__ parent, const T *__restrict__ E,
                                                 float *__restrict__ yh, int64_t ldh) {
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, lr = lane & 15, g = lane >> 4;
    if (16 * w >= k) return;
    const int32_t c = list[blockIdx.x];
    const int32_t par = parent[c];
    const int64_t j0 = (int64_t)blockIdx.y * 16 * NJT;
    const int mc = (int)min<int64_t>(16 * NJT, m - j0);
    const int ra = min(16 * w + lr, k - 1);  // row of E_c this lane supplies
    const T *Ec = E + (int64_t)c * k * k + (int64_t)ra * k;
    flt4 acc[NJT];
#pragma unroll
    for (int J = 0; J < NJT; ++J) acc[J] = flt4{0.f, 0.f, 0.f, 0.f};
    term<KS, T, NJT>(k, lr, g, [&](int nu) { return Ec + nu; }, yh + (int64_t)par * k * ldh + j0, ldh, mc, acc);
#pragma unroll
    for (int J = 0; J < NJT; ++J) {
        const int col = 16 * J + lr;
        if (col < mc)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = 16 * w + 4 * g + r;
                if (row < k) yh[((int64_t)c * k + row) * ldh + j0 + col] += acc[J][r];
            }
    }
}

// Forward leaf transform x_t = V_t^T X|_t for every leaf t, X from the FP32 tree-ordered
// copy (rounded to the storage type as it is used), the points of the leaf in chunks of 64
template <typename T>
__global__ __launch_bounds__(256) void k_fwd_leaf_lp(int k, int64_t m, const int32_t *__restrict__ leaves,
                                                     const int32_t *__restrict__ first,
                                                     const int32_t *__restrict__ size, const T *__restrict__ V,
                                                     const float *__restrict__ Xt, int64_t ldxt,
                                                     float *__restrict__ xh, int64_t ldh) {
    constexpr int KS = 16;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, lr = lane & 15, g = lane >> 4;
    if (16 * w >= k) return;
    const int32_t t = leaves[blockIdx.x];
    const int64_t j0 = (int64_t)blockIdx.y * kCols;
    const int mc = (int)min<int64_t>(kCols, m - j0);
    const int64_t r0 = first[t];
    const int nt = size[t];
    const int nu = min(16 * w + lr, k - 1);  // row of x_t (column of V) this lane supplies
    flt4 acc[2] = {flt4{0.f, 0.f, 0.f, 0.f}, flt4{0.f, 0.f, 0.f, 0.f}};
    for (int i0 = 0; i0 < nt; i0 += 4 * KS) {
        const T *Vc = V + (r0 + i0) * k + nu;
        term<KS, T>(min(4 * KS, nt - i0), lr, g, [&](int i) { return Vc + (int64_t)i * k; },
                    Xt + (r0 + i0) * ldxt + j0, ldxt, mc, acc);
    }
#pragma unroll
    for (int J = 0; J < 2; ++J) {
        const int col = 16 * J + lr;
        if (col < mc)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = 16 * w + 4 * g + r;
                if (row < k) xh[((int64_t)t * k + row) * ldh + j0 + col] = acc[J][r];
            }
    }
}

}  // namespace tlp
}  // namespace h2x
