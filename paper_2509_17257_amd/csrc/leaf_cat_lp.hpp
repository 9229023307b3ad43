// Leaf stage of the FP32 / BF16 operators as one contraction per leaf (FP32 matrix cores):
//
//   Y|_t = beta Y|_t + alpha (V_t y_t + sum_{(t,s) near} N_ts X|_s)
//
// the organisation of the FP64 form in leaf_cat.hpp with v_mfma_f32_16x16x4f32: the
// transposed near blocks of a leaf (FP32, rows padded to an even length) and its transposed
// basis (FP32 or BF16) form one matrix of sum |s| + k rows, contracted in rounds of 16 rows
// against rows of the FP32 tree-ordered copy of X (through the per-leaf table of near rows in
// LDS) or of y_t; FP32 sums.  With a BF16 basis, y_t is rounded to BF16 where it meets V_t
// (both factors of a product in the storage type).  Only the end of each segment is padded (to
// 16 rows) and the rows of the leaf come in 16-row tiles.
//
// Lane layout of v_mfma_f32_16x16x4f32 (A: 16 x 4, B: 4 x 16, D: 16 x 16): lane l holds
// A[l % 16][l / 16], B[l / 16][l % 16] and D rows 4 (l / 16) + q, column l % 16 (q = 0..3).
// Here A = X^T (a lane loads two neighbouring columns with one 8-byte load, which feed an
// "even" and an "odd" column tile) and B = N^T (one 4-byte load per row tile and k-step).
#pragma once

#include "leaf_cat.hpp"
#include "leaf_lp.hpp"

namespace h2x {
namespace lp {

template <int NP>
struct CatRoundLp {
    flt2 a[NP][4];  // [column half p][k-step u]: columns 32p + 2 (l % 16) + {0, 1}
    float b[2][4];  // [row tile of the wave][k-step u]: row 16 I + l % 16
    int ok[4];      // k-row of step u inside its segment
};

__device__ inline float ld1(const float *p) { return *p; }
__device__ inline float ld1(const bf16_t *p) { return __builtin_bit_cast(float, (uint32_t)p->b << 16); }

struct LeafCatLpArgs {
    int k;
    int64_t m;
    int32_t L;
    const int32_t *order;  // launch order of the leaves (leaf indices)
    const int32_t *leaves, *first, *size;
    const int64_t *perm;
    const void *Vt;  // transposed leaf bases, FP32 or BF16
    const int64_t *vt_off;
    const float *yh;
    int64_t ldh;
    const int64_t *near_ptr;
    const int32_t *near_col;
    const int64_t *near_off;
    const float *Nt, *Xt;
    int64_t ldxt;
    double alpha, beta;
    double *Y;
    int64_t ldy;
    int tree_order, round_y;
    Skip skip;
};

template <int NP>
constexpr size_t leaf_cat_lp_red_bytes() { return sizeof(float) * 64 * (32 * NP + 1); }

// one (leaf, column slab) per work-group, mapped to XCDs as in the FP64 form (slot & 7 is the
// XCD, whose leaves form one contiguous eighth of the launch order; the slabs of one leaf are
// consecutive slots of one XCD).  Dynamic LDS: the near-row table.
template <int NP, typename TV>
__global__ __launch_bounds__(256, 2) void k_leaf_cat_lp(LeafCatLpArgs a) {
    constexpr int MC = 32 * NP, LDR = MC + 1;
    __shared__ float red[64 * LDR];
    extern __shared__ int32_t xrow[];
    const int64_t slot = blockIdx.x;
    const int32_t per_xcd = (a.L + 7) / 8;
    const int nslab = (int)((a.m + MC - 1) / MC);
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63, lr = lane & 15,
              lq = lane >> 4;
    const int64_t qx = slot >> 3;
    const int32_t pos = (int32_t)((slot & 7) * per_xcd + qx / nslab);
    if (pos >= a.L) return;
    const int32_t l = a.order[pos];
    const int32_t t = a.leaves[l];
    if (a.skip(t)) return;
    const int k = a.k;
    const int nt = a.size[t];
    const int64_t nt2 = pad_rows(nt), r0 = a.first[t];
    const int64_t j0 = (qx % nslab) * MC;
    const int mc = (int)min<int64_t>(MC, a.m - j0);
    const int64_t q0 = a.near_ptr[l];
    const int nnear = (int)(a.near_ptr[l + 1] - q0);
    const int32_t rn =
        nnear > 0 ? mfma::cat_build_rows(xrow, q0, nnear, nt2, a.near_col, a.near_off, a.first, a.size) : 0;
    const float *nb = nnear > 0 ? a.Nt + a.near_off[q0] : a.Nt;
    const TV *vb = (const TV *)a.Vt + a.vt_off[l];
    const int RN = (rn + 15) >> 4, RT = RN + ((k + 15) >> 4);
    const int xc = (mc - 1) & ~1;  // last even column offset of the slab
    // two row tiles per wave: a 64-row chunk of more than two tiles is two row groups of two
    // waves (k-groups), otherwise one row group of all four waves
    for (int i0 = 0; i0 < nt; i0 += 64) {
        const int ic = min(64, nt - i0);
        const int ntile = (ic + 15) >> 4;
        const int G = ntile > 2 ? 2 : 4;       // waves per row group (k-groups)
        const int wr = w / G, g = w - wr * G;  // row group, k-group (wave-uniform)
        const int tl0 = 2 * wr;                // first row tile of the wave
        const bool t0 = tl0 < ntile, t1 = tl0 + 1 < ntile;
        const int row_a = i0 + min(16 * tl0 + lr, ic - 1), row_b = i0 + min(16 * tl0 + 16 + lr, ic - 1);

        flt4v acc[2 * NP][2];
#pragma unroll
        for (int J = 0; J < 2 * NP; ++J) acc[J][0] = acc[J][1] = flt4v{0.f, 0.f, 0.f, 0.f};

        // round r (clamped to the wave's rounds) -> registers; both branches issue the same
        // number of loads from clamped in-range addresses, so the wait counts stay exact.  The
        // near-field operands come through buffer resources (32-bit byte offsets; the host
        // takes this form only while X is below 4 GiB).
        auto load = [&](int r, CatRoundLp<NP> &R) {
            if (r < RN) {
                const int c0 = 16 * r;
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int c = c0 + 4 * u + lq, cc = min(c, rn - 1);
                    R.ok[u] = c < rn;
                    const __amdgpu_buffer_rsrc_t rx = buf_rsrc(a.Xt + j0, 0xFFFFFFFFu);
                    const uint32_t xo = (uint32_t)(xrow[cc] * a.ldxt);
#pragma unroll
                    for (int p = 0; p < NP; ++p)
                        R.a[p][u] = __builtin_bit_cast(flt2, buf_ld8<0>(rx, 4u * (xo + min(32 * p + 2 * lr, xc))));
                    const __amdgpu_buffer_rsrc_t rb = buf_rsrc(nb, 0xFFFFFFFFu);
                    R.b[0][u] = buf_ld4f<0>(rb, 4u * (uint32_t)(cc * nt2 + row_a));
                    R.b[1][u] = buf_ld4f<0>(rb, 4u * (uint32_t)(cc * nt2 + row_b));
                }
            } else {
                const int c0 = 16 * (r - RN);
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int c = c0 + 4 * u + lq, cc = min(c, k - 1);
                    R.ok[u] = c < k;
                    const float *ar = a.yh + ((int64_t)t * k + cc) * a.ldh + j0;
#pragma unroll
                    for (int p = 0; p < NP; ++p) R.a[p][u] = ld2(ar + min(32 * p + 2 * lr, xc));
                    R.b[0][u] = ld1(vb + (int64_t)cc * nt2 + row_a);
                    R.b[1][u] = ld1(vb + (int64_t)cc * nt2 + row_b);
                }
            }
        };
        auto multiply = [&](const CatRoundLp<NP> &R, bool basis) {
            const bool rnd = a.round_y && basis;
#pragma unroll
            for (int u = 0; u < 4; ++u) {
#pragma unroll
                for (int p = 0; p < NP; ++p) {
                    flt2 v = R.ok[u] ? R.a[p][u] : flt2{0.f, 0.f};
                    if (rnd) v = flt2{round_bf16(v.x), round_bf16(v.y)};
#pragma unroll
                    for (int hj = 0; hj < 2; ++hj) {
                        if (t0)
                            acc[2 * p + hj][0] =
                                __builtin_amdgcn_mfma_f32_16x16x4f32(v[hj], R.b[0][u], acc[2 * p + hj][0], 0, 0, 0);
                        if (t1)
                            acc[2 * p + hj][1] =
                                __builtin_amdgcn_mfma_f32_16x16x4f32(v[hj], R.b[1][u], acc[2 * p + hj][1], 0, 0, 0);
                    }
                }
            }
        };

        if (g < RT) {
            const int last = g + ((RT - 1 - g) / G) * G;  // the wave's last round
            CatRoundLp<NP> s0, s1, s2;
            int r = g;
            load(r, s0);
            load(min(r + G, last), s1);
            // three register sets in turn; a set is loaded two rounds ahead of its use
            for (;;) {
                load(min(r + 2 * G, last), s2);
                multiply(s0, r >= RN);
                r += G;
                if (r > last) break;
                load(min(r + 2 * G, last), s0);
                multiply(s1, r >= RN);
                r += G;
                if (r > last) break;
                load(min(r + 2 * G, last), s1);
                multiply(s2, r >= RN);
                r += G;
                if (r > last) break;
            }
        }
        // partial tiles of the G waves of each row group, added in wave order.  Lane l,
        // register q of acc[2p + hj][I] -> column 32p + 2 (4 (l / 16) + q) + hj, row
        // 16 (tl0 + I) + l % 16.
        for (int gg = 0; gg < G; ++gg) {
            if (g == gg)
#pragma unroll
                for (int J = 0; J < 2 * NP; ++J)
#pragma unroll
                    for (int I = 0; I < 2; ++I)
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            const int col = 32 * (J >> 1) + 2 * (4 * lq + q) + (J & 1);
                            const int row = 16 * (tl0 + I) + lr;
                            float *cell = &red[row * LDR + col];
                            *cell = (gg == 0) ? acc[J][I][q] : *cell + acc[J][I][q];
                        }
            __syncthreads();
        }
        for (int x = threadIdx.x; x < ic * MC; x += 256) {
            const int i = x / MC, j = x - i * MC;
            if (j < mc) {
                int64_t row = r0 + i0 + i;
                if (!a.tree_order) row = a.perm[row];
                double *y = &a.Y[row * a.ldy + j0 + j];
                const double v = a.alpha * (double)red[i * LDR + j];
                *y = (a.beta == 0.0) ? v : a.beta * *y + v;
            }
        }
        __syncthreads();
    }
}

}  // namespace lp
}  // namespace h2x
