// Matrix-core leaf stage for the low-precision operators (k = 64 or k <= 32): near field in
// FP32, leaf basis in FP32 or BF16, FP32 accumulation (v_mfma_f32_16x16x4f32):
//   Y|_t = beta Y|_t + alpha (V_t y_t + sum_s N_ts X|_s).
// X arrives as an FP32 copy in tree order.  With a BF16 basis, y_t is rounded to
// BF16 before it multiplies V_t (both factors of a product in the storage type;
// a product of two BF16 values is exact in FP32).
//
// Organisation as in the FP64 leaf kernel: transposed orientation Y_t^T = X_s^T
// N_ts^T, near-field blocks stored transposed with rows padded to an even length,
// one 8-byte load per lane feeds an "even" and an "odd" tile, the 4 waves of a
// work-group share the leaf's terms round-robin and their partial tiles are
// added in LDS in wave order.  Output layout of the FP32 MFMA: register q of
// lane l holds row 4 (l / 16) + q (here: a column of Y), column l % 16 (a row).
#pragma once

#include "device.hpp"
#include "types.hpp"

namespace h2x {
namespace lp {

typedef float flt2 __attribute__((ext_vector_type(2)));
typedef float flt4v __attribute__((ext_vector_type(4)));

__device__ inline flt2 ld2(const float *p) { return *(const flt2 *)p; }
__device__ inline flt2 ld2(const bf16_t *p) {
    const uint32_t u = *(const uint32_t *)p;
    return flt2{__builtin_bit_cast(float, u << 16), __builtin_bit_cast(float, u & 0xffff0000u)};
}
__device__ inline float round_bf16(float v) { return __builtin_bit_cast(float, (uint32_t)bf16_bits(v) << 16); }

template <int NP>
struct Round {
    flt2 b[2][4];   // [row half g][k-step u]: rows 32g + 2 lr + {0, 1}
    flt2 a[NP][4];  // [column half p][k-step u]: columns 32p + 2 lr + {0, 1}
    int kb, kl;     // first k-step of the round and the item's length
    bool basis;     // the round belongs to the basis term
};

template <int NP, typename TV>
__global__ __launch_bounds__(256, 2) void k_leaf_lp(int k, int64_t m, int32_t L, const int32_t *__restrict__ leaves,
                                                    const int32_t *__restrict__ first, const int32_t *__restrict__ size,
                                                    const int64_t *__restrict__ perm, const TV *__restrict__ Vt,
                                                    const int64_t *__restrict__ vt_off, const float *__restrict__ yh,
                                                    int64_t ldh, const int64_t *__restrict__ near_ptr,
                                                    const int32_t *__restrict__ near_col,
                                                    const int64_t *__restrict__ near_off,
                                                    const float *__restrict__ Nt, const float *__restrict__ Xt,
                                                    int64_t ldxt, double alpha, double beta, double *__restrict__ Y,
                                                    int64_t ldy, int tree_order, int round_y, Skip skip) {
    constexpr int MC = 32 * NP, LDR = MC + 1;
    __shared__ float red[64 * LDR];
    // one (leaf, column slab) per work-group; the slabs of one leaf are consecutive
    // work-groups of one XCD, so its near blocks come from HBM once
    const int32_t per_xcd = (L + 7) / 8;
    const int nslab = (int)((m + MC - 1) / MC);
    const int64_t qx = blockIdx.x >> 3;
    const int32_t l = (int32_t)((blockIdx.x & 7) * per_xcd + qx / nslab);
    if (l >= L) return;
    const int32_t t = leaves[l];
    if (skip(t)) return;
    const int nt = size[t];
    const int64_t nt2 = pad_rows(nt);
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63, lr = lane & 15,
                  lq = lane >> 4;  // w is wave-uniform: item loops stay scalar
    const int64_t r0 = first[t];
    const int64_t j0 = (qx % nslab) * MC;
    const int mc = (int)min<int64_t>(MC, m - j0);
    const int64_t q0 = near_ptr[l], vt0 = vt_off[l];
    // items: the basis term, then the near blocks
    const int nnear = (int)(near_ptr[l + 1] - q0);
    const int nitems = nnear + 1;
    // near-block metadata staged once (beyond kMeta: read directly)
    constexpr int kMeta = 160;
    __shared__ int64_t m_off[kMeta], m_first[kMeta];
    __shared__ int32_t m_size[kMeta];
    for (int x = threadIdx.x; x < min(nnear, kMeta); x += 256) {
        const int32_t s = near_col[q0 + x];
        m_off[x] = near_off[q0 + x];
        m_first[x] = first[s];
        m_size[x] = size[s];
    }
    __syncthreads();
    auto near_meta = [&](int x, int64_t &off, int64_t &fs, int &ks) {
        if (x < kMeta) {
            off = m_off[x];
            fs = m_first[x];
            ks = m_size[x];
        } else {
            // relaxed atomic loads: the compiler cannot fold this path and the LDS path
            // into one load through a generic pointer
            const int32_t s = __hip_atomic_load(near_col + q0 + x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            off = __hip_atomic_load(near_off + q0 + x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            fs = __hip_atomic_load(first + s, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            ks = __hip_atomic_load(size + s, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    };

    for (int i0 = 0; i0 < nt; i0 += 64) {
        const int ic = min(64, nt - i0);
        const int nhalf = (ic + 31) >> 5;
        flt4v acc[2 * NP][4];
#pragma unroll
        for (int J = 0; J < 2 * NP; ++J)
#pragma unroll
            for (int I = 0; I < 4; ++I) acc[J][I] = flt4v{0.f, 0.f, 0.f, 0.f};

        // unconditional loads from clamped addresses, the k-mask (and the BF16 rounding
        // of y_t) applied once a round's loads are in, and the last round peeled off: the
        // MFMAs of a round never wait for the next round's loads (as in the FP64 kernel)
        const int xr = (ic - 1) & ~1, xc = (mc - 1) & ~1;
        auto load = [&](int e, int kb, Round<NP> &R) {
            R.kb = kb;
            R.basis = e == 0;
            if (e == 0) {  // wave-uniform: both paths issue the same loads
                const TV *bb = Vt + vt0 + i0;                   // V_t^T[nu][i]
                const float *ab = yh + (int64_t)t * k * ldh + j0;  // y_t[nu][j]
                R.kl = k;
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int c = min(kb + 4 * u + lq, k - 1);
#pragma unroll
                    for (int g = 0; g < 2; ++g) R.b[g][u] = ld2(bb + c * nt2 + min(32 * g + 2 * lr, xr));
#pragma unroll
                    for (int p = 0; p < NP; ++p) R.a[p][u] = ld2(ab + c * ldh + min(32 * p + 2 * lr, xc));
                }
            } else {
                int64_t off, fs;
                int kl;
                near_meta(e - 1, off, fs, kl);
                const float *bb = Nt + off + i0;       // N_ts^T[c][i]
                const float *ab = Xt + fs * ldxt + j0;  // X_s[c][j]
                R.kl = kl;
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int c = min(kb + 4 * u + lq, kl - 1);
#pragma unroll
                    for (int g = 0; g < 2; ++g) R.b[g][u] = ld2(bb + c * nt2 + min(32 * g + 2 * lr, xr));
#pragma unroll
                    for (int p = 0; p < NP; ++p) R.a[p][u] = ld2(ab + c * ldxt + min(32 * p + 2 * lr, xc));
                }
            }
        };
        auto klen = [&](int e) {
            if (e == 0) return k;
            int64_t off, fs;
            int ks;
            near_meta(e - 1, off, fs, ks);
            return ks;
        };
        auto mask = [&](Round<NP> &R) {
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const bool cok = R.kb + 4 * u + lq < R.kl;
#pragma unroll
                for (int p = 0; p < NP; ++p) {
                    flt2 v = cok ? R.a[p][u] : flt2{0.f, 0.f};
                    if (round_y && R.basis) v = flt2{round_bf16(v.x), round_bf16(v.y)};
                    R.a[p][u] = v;
                }
            }
        };
        auto multiply = [&](const Round<NP> &R) {
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int g = 0; g < 2; ++g)
                    if (g < nhalf)
#pragma unroll
                        for (int h = 0; h < 2; ++h)
#pragma unroll
                            for (int p = 0; p < NP; ++p)
#pragma unroll
                                for (int hj = 0; hj < 2; ++hj)
                                    acc[2 * p + hj][2 * g + h] = __builtin_amdgcn_mfma_f32_16x16x4f32(
                                        R.a[p][u][hj], R.b[g][u][h], acc[2 * p + hj][2 * g + h], 0, 0, 0);
        };

        int e = w;
        if (e < nitems) {
            Round<NP> cur, nxt;
            int kb = 0, len = klen(e);
            load(e, kb, cur);
            mask(cur);
            for (;;) {
                int en = e, kbn = kb + 16, lenn = len;
                if (kbn >= len) {
                    en = e + 4;
                    kbn = 0;
                    if (en < nitems) lenn = klen(en);
                }
                if (en >= nitems) break;
                load(en, kbn, nxt);
                multiply(cur);
                cur = nxt;
                mask(cur);
                e = en;
                kb = kbn;
                len = lenn;
            }
            multiply(cur);
        }
        // tile (J = 2p + hj, I = 2g + h): register q of lane l -> column 32p + 2 (4 (l / 16) + q) + hj,
        // row 32g + 2 (l % 16) + h
        for (int ww = 0; ww < 4; ++ww) {
            if (w == ww)
#pragma unroll
                for (int J = 0; J < 2 * NP; ++J)
#pragma unroll
                    for (int I = 0; I < 4; ++I)
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            const int col = 32 * (J >> 1) + 2 * (4 * lq + q) + (J & 1);
                            const int row = 32 * (I >> 1) + 2 * lr + (I & 1);
                            float *cell = &red[row * LDR + col];
                            *cell = (ww == 0) ? acc[J][I][q] : *cell + acc[J][I][q];
                        }
            __syncthreads();
        }
        for (int x = threadIdx.x; x < ic * MC; x += 256) {
            const int i = x / MC, j = x % MC;
            if (j < mc) {
                int64_t row = r0 + i0 + i;
                if (!tree_order) row = perm[row];
                double *y = &Y[row * ldy + j0 + j];
                const double v = alpha * (double)red[i * LDR + j];
                *y = (beta == 0.0) ? v : beta * *y + v;
            }
        }
        __syncthreads();
    }
}

// rows of X into tree order as FP32 (nearest) with an even leading dimension, zero padding; one
// wave per row (256 threads: rows 4 blockIdx.x .. 4 blockIdx.x + 3), lane j takes columns j + 64 s
__global__ __launch_bounds__(256) void k_gather_f32(int64_t n, int64_t m, const int64_t *__restrict__ perm,
                                                    const double *__restrict__ X, int64_t ldx,
                                                    float *__restrict__ Xt, int64_t ldt) {
    const int64_t i = 4 * (int64_t)blockIdx.x + (threadIdx.x >> 6);
    if (i >= n) return;
    const double *xr = X + (perm ? perm[i] : i) * ldx;
    float *tr = Xt + i * ldt;
    for (int64_t j = threadIdx.x & 63; j < ldt; j += 64) tr[j] = j < m ? (float)xr[j] : 0.f;
}

}  // namespace lp
}  // namespace h2x
