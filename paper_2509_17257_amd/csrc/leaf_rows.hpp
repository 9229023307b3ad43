// Leaf stage with the rows split over independent waves (FP64 operator in the
// matrix-core layout, k = 64 or k <= 32):
//   Y|_t = beta Y|_t + alpha (V_t y_t + sum_s N_ts X|_s)        for every leaf t.
//
// One wave (one work-group) per (leaf, band of 32 rows, slab of 32 * NP columns); a
// leaf above 64 points takes its bands 0, 2, 4, ... in the wave of grid row 0 and 1,
// 3, ... in that of grid row 1.  The terms of the sum are items: the basis term
// (A = V_t from its transposed copy, B = y_t) and the near blocks (A = N_ts from the
// transposed storage, B = X|_s, tree-ordered X).  The wave streams them in rounds of
// KR contraction steps, both operands straight from memory into registers one round
// ahead: A as two 16-row strips (8-byte loads, 16 lanes over 16 consecutive rows of
// a transposed row), B as column pairs (16-byte loads), so that one 16x16x4 f64
// matrix-core product takes the even and one the odd columns of a pair.  A strip past
// the leaf is skipped (a band of one strip has its own code); every load is issued
// unconditionally from a clamped address, so the wait counters stay exact, and the
// k-rows of B past the item are zeroed where they are used.  No operand goes through
// LDS and no wave waits for another; rows are padded to 16 (a 32-row half in the
// wave-per-term form), the contraction to a 16-long round in both.
//
// Complex operator (n_plane > 0): every near block is two items, its real plane on
// X and its imaginary plane on J X (column pairs (re, im) -> (-im, re), applied to
// the B registers).
#pragma once

#include <type_traits>

#include "device.hpp"

namespace h2x {
namespace mfma {

typedef double dbl4 __attribute__((ext_vector_type(4)));
typedef double dbl2v __attribute__((ext_vector_type(2)));

template <int NP>
__global__ __launch_bounds__(64) void k_leaf_rows(int k, int64_t m, int32_t L, const int32_t *__restrict__ leaves,
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
    constexpr int MC = 32 * NP;             // columns per wave
    constexpr int NU = 4;                   // 4-long contraction steps per round
    constexpr int KR = 4 * NU;              // contraction length of a round
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
    const int nt = size[t];
    if (32 * (int)blockIdx.y >= nt) return;
    const int lane = threadIdx.x, lr = lane & 15, lq = lane >> 4;
    const int64_t nt2 = pad_rows(nt), r0 = first[t];
    const int64_t j0 = (qx % nslab) * MC;
    const int mc = (int)min<int64_t>(MC, m - j0);
    const int xc = (mc - 1) & ~1;  // last even column offset of the slab
    const int64_t q0 = near_ptr[l], vt0 = basis ? vt_off[l] : 0;
    const int nnear = near ? (int)(near_ptr[l + 1] - q0) : 0;
    const int cpx = n_plane > 0 ? 1 : 0;
    const int nitems = (basis ? 1 : 0) + (nnear << cpx);

    // the near blocks' offsets, row ranges and sizes, staged once so that moving to the
    // next item costs no dependent global loads (beyond kMeta: read directly)
    // and the number of rounds of all items (a plane doubles a near block's rounds)
    int nr = 0;
    for (int x = lane; x < nnear; x += 64) {
        const int32_t s = near_col[q0 + x];
        const int ks = size[s];
        if (x < kMeta) {
            m_off[x] = near_off[q0 + x];
            m_first[x] = first[s];
            m_size[x] = ks;
        }
        nr += ((ks + KR - 1) / KR) << cpx;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) nr += __shfl_xor(nr, o);
    const int nrounds = nr + (basis ? (k + KR - 1) / KR : 0);
    __syncthreads();

    struct Item {
        const double *a, *b;
        int64_t ldb;
        int len, jx;
    };
    auto item = [&](int e) {
        Item it;
        if (basis && e == 0) {
            it.a = Vt + vt0;                          // V_t^T[nu][i]
            it.b = yh + (int64_t)t * k * ldh + j0;  // y_t[nu][j]
            it.ldb = ldh;
            it.len = k;
            it.jx = 0;
            return it;
        }
        const int e2 = e - (basis ? 1 : 0), q = e2 >> cpx;
        it.jx = e2 & cpx;
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
        it.a = Nt + off + (it.jx ? n_plane : 0);  // N_ts^T[c][i]
        it.b = Xt + fs * ldxt + j0;                 // X_s[c][j]
        it.ldb = ldxt;
        return it;
    };

    // one band of rows b0 .. b0 + 16 NS - 1 (NS 16-row strips inside the leaf)
    auto band = [&](int b0, auto NSc) {
        constexpr int NS = decltype(NSc)::value;
        struct Round {
            double a[NS][NU];
            dbl2v b[NU][NP];
            int kl, jx;
        };
        int ra[NS];
#pragma unroll
        for (int s = 0; s < NS; ++s) ra[s] = b0 + min(16 * s + lr, nt - 1 - b0);
        dbl4 acc[NS][2 * NP];
#pragma unroll
        for (int s = 0; s < NS; ++s)
#pragma unroll
            for (int J = 0; J < 2 * NP; ++J) acc[s][J] = dbl4{0.0, 0.0, 0.0, 0.0};

        auto load = [&](const Item &it, int k0, Round &R) {
            R.kl = it.len - k0;
            R.jx = it.jx;
#pragma unroll
            for (int u = 0; u < NU; ++u) {
                const int64_t c = min(k0 + 4 * u + lq, it.len - 1);
#pragma unroll
                for (int s = 0; s < NS; ++s) R.a[s][u] = it.a[c * nt2 + ra[s]];
#pragma unroll
                for (int p = 0; p < NP; ++p)
                    R.b[u][p] = *(const dbl2v *)(it.b + c * it.ldb + min(32 * p + 2 * lr, xc));
            }
        };
        // every step of a round goes through the matrix cores (the k-rows of B past the item
        // are zero), so that no branch splits the accumulator chains
        auto multiply = [&](const Round &R) {
#pragma unroll
            for (int u = 0; u < NU; ++u) {
                const bool cok = 4 * u + lq < R.kl;
#pragma unroll
                for (int p = 0; p < NP; ++p) {
                    dbl2v v = cok ? R.b[u][p] : dbl2v{0.0, 0.0};
                    if (R.jx) v = dbl2v{-v.y, v.x};
#pragma unroll
                    for (int s = 0; s < NS; ++s)
#pragma unroll
                        for (int hj = 0; hj < 2; ++hj)
                            acc[s][2 * p + hj] =
                                __builtin_amdgcn_mfma_f64_16x16x4f64(R.a[s][u], v[hj], acc[s][2 * p + hj], 0, 0, 0);
                }
            }
        };

        // rounds in item order; past the last item a round is empty (kl = 0: B zero) and
        // reloads the last item's addresses.  The loop takes two rounds per pass with the
        // two register sets alternating, so that it has a single exit, the accumulators
        // stay in place and waiting for a round's loads comes only when it is multiplied.
        if (nitems > 0) {
            int e = 0, k0 = 0;
            Item cur = item(0);
            auto load_next = [&](Round &R) {
                load(cur, k0, R);
                if (e >= nitems) R.kl = 0;
                k0 += KR;
                if (k0 >= cur.len && e < nitems) {
                    ++e;
                    k0 = 0;
                    if (e < nitems) cur = item(e);
                    else k0 = cur.len - 1;
                }
            };
            Round rx, ry;
            load_next(rx);
            for (int r = 0; r < nrounds; r += 2) {
                load_next(ry);
                __builtin_amdgcn_sched_barrier(0);
                multiply(rx);
                load_next(rx);
                __builtin_amdgcn_sched_barrier(0);
                multiply(ry);
            }
        }
        // D layout of the 16x16x4 f64 MFMA: lane l, register r -> row l / 16 + 4 r, column
        // l % 16, here column pair 2 (l % 16) + hj of the 32-column group p.  With beta != 0
        // the old values are read first, all at once, from clamped addresses.
        auto yptr = [&](int s, int J, int r) {
            const int i = min(b0 + 16 * s + lq + 4 * r, nt - 1);
            const int col = min(32 * (J >> 1) + 2 * lr + (J & 1), mc - 1);
            int64_t row = r0 + i;
            if (!tree_order) row = perm[row];
            return &Y[row * ldy + j0 + col];
        };
        double old[NS][2 * NP][4];
        if (beta != 0.0) {
#pragma unroll
            for (int s = 0; s < NS; ++s)
#pragma unroll
                for (int J = 0; J < 2 * NP; ++J)
#pragma unroll
                    for (int r = 0; r < 4; ++r) old[s][J][r] = *yptr(s, J, r);
        }
#pragma unroll
        for (int s = 0; s < NS; ++s)
#pragma unroll
            for (int J = 0; J < 2 * NP; ++J)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const double v = alpha * acc[s][J][r];
                    if (b0 + 16 * s + lq + 4 * r < nt && 32 * (J >> 1) + 2 * lr + (J & 1) < mc)
                        *yptr(s, J, r) = (beta == 0.0) ? v : beta * old[s][J][r] + v;
                }
    };

    for (int b0 = 32 * (int)blockIdx.y; b0 < nt; b0 += 64) {
        if (nt - b0 > 16) band(b0, std::integral_constant<int, 2>{});
        else band(b0, std::integral_constant<int, 1>{});
    }
}

}  // namespace mfma
}  // namespace h2x
