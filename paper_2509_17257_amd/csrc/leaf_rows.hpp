// Leaf stage with the rows split over the waves (FP64 operator in the matrix-core
// layout, k = 64 or k <= 32):
//   Y|_t = beta Y|_t + alpha (V_t y_t + sum_s N_ts X|_s)        for every leaf t.
//
// Organised like the coupling kernel: one work-group per leaf (and slab of 16*NJ
// columns), wave w owns rows 16w..16w+15 of the leaf (in 64-row chunks for larger
// leaves), and the terms of the sum are items: the basis term (A = V_t from its
// transposed copy, B = y_t) and the near blocks (A = N_ts from the transposed
// storage, B = X|_s, tree-ordered X).  For every item the work-group stages B
// (contraction rows x 16*NJ columns, zero rows up to a multiple of 4, double-buffered)
// in LDS, and each wave streams its 16 rows of A from HBM into registers one item
// ahead (8-byte loads, 16 lanes over 16 consecutive rows of a transposed row).  A
// wave whose rows all lie past the leaf skips the matrix cores, and no partial
// sums cross waves, so there is no reduction in LDS.  The contraction is padded to
// 4, not to a 16-step round.  Contractions longer than 64 (leaves above 64 points)
// are split into 64-long sub-items.
//
// Complex operator (n_plane > 0): every near block is two items, its real plane on
// X and its imaginary plane on J X (column pairs (re, im) -> (-im, re), applied
// while X is staged).
#pragma once

#include "device.hpp"

namespace h2x {
namespace mfma {

typedef double dbl4 __attribute__((ext_vector_type(4)));

template <int NJ>
__global__ __launch_bounds__(256) void k_leaf_rows(int k, int64_t m, int32_t L, const int32_t *__restrict__ leaves,
                                                   const int32_t *__restrict__ first, const int32_t *__restrict__ size,
                                                   const int64_t *__restrict__ perm, const double *__restrict__ Vt,
                                                   const int64_t *__restrict__ vt_off, const double *__restrict__ yh,
                                                   int64_t ldh, const int64_t *__restrict__ near_ptr,
                                                   const int32_t *__restrict__ near_col,
                                                   const int64_t *__restrict__ near_off,
                                                   const double *__restrict__ Nt, const double *__restrict__ Xt,
                                                   int64_t ldxt, double alpha, double beta, double *__restrict__ Y,
                                                   int64_t ldy, int tree_order, int basis, int near, Skip skip,
                                                   int64_t n_plane) {
    constexpr int MC = 16 * NJ, LDB = MC + 1, KC = 64;  // sub-item contraction length
    constexpr int BPT = KC * MC / 256;                  // staged B values per thread
    __shared__ double bs[2][KC * LDB];
    constexpr int kMeta = 160;
    __shared__ int64_t m_off[kMeta], m_first[kMeta];
    __shared__ int32_t m_size[kMeta];

    const int32_t per_xcd = (L + 7) / 8;
    const int nslab = (int)((m + MC - 1) / MC);
    const int64_t qx = blockIdx.x >> 3;
    const int32_t l = (int32_t)((blockIdx.x & 7) * per_xcd + qx / nslab);
    if (l >= L) return;
    const int32_t t = leaves[l];
    if (skip(t)) return;
    const int tid = threadIdx.x, lane = tid & 63, lr = lane & 15, lq = lane >> 4;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int nt = size[t];
    const int64_t nt2 = nt + (nt & 1), r0 = first[t];
    const int64_t j0 = (qx % nslab) * MC;
    const int mc = (int)min<int64_t>(MC, m - j0);
    const int64_t q0 = near_ptr[l], vt0 = basis ? vt_off[l] : 0;
    const int nnear = near ? (int)(near_ptr[l + 1] - q0) : 0;
    const int cpx = n_plane > 0 ? 1 : 0;
    const int nitems = (basis ? 1 : 0) + (nnear << cpx);

    for (int x = tid; x < min(nnear, kMeta); x += 256) {
        const int32_t s = near_col[q0 + x];
        m_off[x] = near_off[q0 + x];
        m_first[x] = first[s];
        m_size[x] = size[s];
    }
    __syncthreads();
    // item e -> (A base, B base, B leading dimension, contraction length, plane)
    struct Item {
        const double *a, *b;
        int64_t ldb;
        int len, plane;
    };
    auto item = [&](int e) {
        Item it;
        if (basis && e == 0) {
            it.a = Vt + vt0;                          // V_t^T[nu][i]
            it.b = yh + (int64_t)t * k * ldh + j0;  // y_t[nu][j]
            it.ldb = ldh;
            it.len = k;
            it.plane = 0;
            return it;
        }
        const int e2 = e - (basis ? 1 : 0), q = e2 >> cpx;
        it.plane = e2 & cpx;
        int64_t off, fs;
        if (q < kMeta) {
            off = m_off[q];
            fs = m_first[q];
            it.len = m_size[q];
        } else {
            // relaxed atomic loads: the compiler cannot fold this path and the LDS path
            // into one load through a generic pointer
            const int32_t s = __hip_atomic_load(near_col + q0 + q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            off = __hip_atomic_load(near_off + q0 + q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            fs = __hip_atomic_load(first + s, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            it.len = __hip_atomic_load(size + s, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        it.a = Nt + off + (it.plane ? n_plane : 0);  // N_ts^T[c][i]
        it.b = Xt + fs * ldxt + j0;                   // X_s[c][j]
        it.ldb = ldxt;
        return it;
    };

    for (int i0 = 0; i0 < nt; i0 += 64) {
        const int ic = min(64, nt - i0);
        const bool active = 16 * w < ic;                  // wave-uniform
        const int rowa = i0 + min(16 * w + lr, ic - 1);  // this lane's A row (clamped)
        dbl4 acc[NJ];
#pragma unroll
        for (int J = 0; J < NJ; ++J) acc[J] = dbl4{0.0, 0.0, 0.0, 0.0};

        // sub-item (e, c0): contraction rows c0..c0+63 of item e
        double av[16], an[16], bv[BPT];
        auto load = [&](const Item &it, int c0, double *a) {
            const int kl = min(KC, it.len - c0);
#pragma unroll
            for (int kk = 0; kk < 16; ++kk) {
                const int c = c0 + min(4 * kk + lq, kl - 1);
                a[kk] = it.a[(int64_t)c * nt2 + rowa];
            }
#pragma unroll
            for (int u = 0; u < BPT; ++u) {
                const int ee = tid + 256 * u, r = ee / MC, col = ee % MC;
                // rows past the sub-item and columns past the slab: zeroed when stored; the
                // imaginary plane takes the partner column (J)
                bv[u] = it.b[(int64_t)(c0 + min(r, kl - 1)) * it.ldb + ((col < mc ? col : 0) ^ it.plane)];
            }
        };
        auto store = [&](const Item &it, int c0, int buf) {
            const int kl = min(KC, it.len - c0);
#pragma unroll
            for (int u = 0; u < BPT; ++u) {
                const int ee = tid + 256 * u, r = ee / MC, col = ee % MC;
                const double v = (it.plane & ~col & 1) ? -bv[u] : bv[u];
                bs[buf][r * LDB + col] = (r < kl && col < mc) ? v : 0.0;
            }
        };
        auto multiply = [&](const double *a, int nk, int buf) {
            if (!active) return;
            const double *bb = bs[buf] + lq * LDB + lr;
#pragma unroll
            for (int kk = 0; kk < 16; ++kk)
                if (kk < nk)
#pragma unroll
                    for (int J = 0; J < NJ; ++J)
                        acc[J] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[kk], bb[4 * kk * LDB + 16 * J], acc[J], 0,
                                                                       0, 0);
        };

        if (nitems > 0) {
            int e = 0, c0 = 0, buf = 0;
            Item cur = item(0);
            load(cur, c0, av);
            store(cur, c0, 0);
            __syncthreads();
            // the last sub-item is peeled off so that every load of the loop is unconditional
            for (;;) {
                int en = e, cn = c0 + KC;
                if (cn >= cur.len) {
                    en = e + 1;
                    cn = 0;
                }
                const int nk = (min(KC, cur.len - c0) + 3) >> 2;
                if (en >= nitems) {
                    multiply(av, nk, buf);
                    break;
                }
                const Item nxt = en == e ? cur : item(en);
                load(nxt, cn, an);
                multiply(av, nk, buf);
                store(nxt, cn, buf ^ 1);
#pragma unroll
                for (int kk = 0; kk < 16; ++kk) av[kk] = an[kk];
                __syncthreads();
                e = en;
                c0 = cn;
                cur = nxt;
                buf ^= 1;
            }
        }
        // D layout of the 16x16x4 f64 MFMA: lane l, register r -> row l / 16 + 4 r, column l % 16
        if (active)
#pragma unroll
            for (int J = 0; J < NJ; ++J) {
                const int col = 16 * J + lr;
                if (col < mc)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int i = 16 * w + lq + 4 * r;
                        if (i < ic) {
                            int64_t row = r0 + i0 + i;
                            if (!tree_order) row = perm[row];
                            double *y = &Y[row * ldy + j0 + col];
                            const double v = alpha * acc[J][r];
                            *y = (beta == 0.0) ? v : beta * *y + v;
                        }
                    }
            }
        __syncthreads();  // the next row chunk restages the LDS buffers
    }
}

}  // namespace mfma
}  // namespace h2x
