// Matrix-core (MFMA) coupling kernels for the FP64 operator (k = 64 below; a
// small-rank variant for k <= 32 further down):
//   y_t = sum_{(t,s) in C_t, admissible} S_b x_s     for every row cluster t.
//
// One work-group (4 waves) owns one row cluster t and a slab of up to 64
// columns; wave w owns rows 16w..16w+15 of y_t.  For each block of the list,
// the work-group stages x_s (64 x 16*NJ) in LDS (double-buffered, next block
// loaded while the current one is multiplied) and each wave streams its
// 16 x 64 slice of S_b straight from HBM into registers (one 16-byte load per
// lane per pair of k-steps; S is stored in that operand order, see s_index),
// also one block ahead.  v_mfma_f64_16x16x4f64 accumulates in registers; y_t
// is written once.  No atomics: each row cluster has exactly one owner.
//
// Work-groups are mapped to rows so that each XCD (work-groups are dealt to
// the 8 XCDs round-robin) gets one contiguous eighth of the rows in tree
// order: neighbouring row clusters share most column clusters, so their x_s
// reads hit the XCD's L2.  Within an eighth, longer lists go first.
#pragma once

#include <algorithm>
#include <type_traits>

#include "device.hpp"

namespace h2x {

typedef double dbl4 __attribute__((ext_vector_type(4)));

constexpr int kMfmaK = 64;

template <int NJ>
__global__ __launch_bounds__(256) void k_coupling_mfma_f64(int64_t m, int32_t C, int32_t rows_per_xcd,
                                                           const int32_t *__restrict__ order,
                                                           const int64_t *__restrict__ adm_ptr,
                                                           const int32_t *__restrict__ adm_col,
                                                           const double *__restrict__ S,
                                                           const double *__restrict__ xh, double *__restrict__ yh,
                                                           int64_t ldh, Skip skip, int jpass) {
    constexpr int MC = 16 * NJ;   // columns per work-group
    constexpr int LDX = MC + 1;   // padded LDS row
    // 64 columns (TR): x_s transposed in LDS (column c is LDS row c, pitch 66 doubles) with the
    // rows of each group of eight in the order of the S operand pairs (row 8 a + 4 h + l at
    // position 8 a + 2 l + h), so one 16-byte read gives a lane the operands of both k-steps of
    // a pair; narrower slabs keep the row-major tile, which measured faster there
    constexpr bool TR = NJ == 4;
    constexpr int LDT = kMfmaK + 2;
    __shared__ __align__(16) double xs[2][TR ? MC * LDT : kMfmaK * LDX];
    // the column slabs of one row cluster are consecutive work-groups of one XCD, so S_b
    // comes from HBM once and from that XCD's L2 for the other slabs
    const int nslab = (int)((m + MC - 1) / MC), qx = blockIdx.x >> 3;
    const int slot = (blockIdx.x & 7) * rows_per_xcd + qx / nslab;
    if (slot >= C) return;
    const int32_t t = order[slot];
    if (skip(t)) return;
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    const int lr = lane & 15, lq = lane >> 4;
    const int64_t j0 = (int64_t)(qx % nslab) * MC;
    const int mc = (int)min<int64_t>(MC, m - j0);
    const int64_t b0 = adm_ptr[t], b1 = adm_ptr[t + 1];

    dbl4 acc[NJ];
#pragma unroll
    for (int J = 0; J < NJ; ++J) acc[J] = dbl4{0.0, 0.0, 0.0, 0.0};

    if (b1 > b0) {
        // x_s staging: element e = row * MC + col, MC * 64 elements over 256 threads
        // TR: thread = column xc = tid % MC and the XPT (16) consecutive rows from xr0; else
        // element e = tid + 256 u is (row e / MC, column e % MC)
        constexpr int XPT = (kMfmaK * MC) / 256;  // elements per thread (4 * NJ)
        const int xc = tid % MC, xr0 = (tid / MC) * XPT;
        double xv[XPT];
        // jpass: column c takes its partner c ^ 1 (J x = (-im, re) per complex column); columns
        // past mc are zeroed when stored
        auto load_x = [&](int32_t s) {
            if constexpr (TR) {
                const double *src = xh + ((int64_t)s * kMfmaK + xr0) * ldh + j0 + ((xc < mc ? xc : 0) ^ jpass);
#pragma unroll
                for (int u = 0; u < XPT; ++u) xv[u] = src[(int64_t)u * ldh];
            } else {
                const double *src = xh + (int64_t)s * kMfmaK * ldh + j0;
#pragma unroll
                for (int u = 0; u < XPT; ++u) {
                    const int e = tid + 256 * u, r = e / MC, c = e % MC;
                    xv[u] = src[(int64_t)r * ldh + ((c < mc ? c : 0) ^ jpass)];
                }
            }
        };
        typedef double dbl2 __attribute__((ext_vector_type(2)));
        auto store_x = [&](int buf) {
            if constexpr (TR) {
                const bool neg = jpass & ~xc & 1;
                double *dst = &xs[buf][xc * LDT + xr0];
#pragma unroll
                for (int a8 = 0; a8 < XPT / 8; ++a8)
#pragma unroll
                    for (int l = 0; l < 4; ++l) {
                        const double v0 = neg ? -xv[8 * a8 + l] : xv[8 * a8 + l];
                        const double v1 = neg ? -xv[8 * a8 + 4 + l] : xv[8 * a8 + 4 + l];
                        *(dbl2 *)(dst + 8 * a8 + 2 * l) = xc < mc ? dbl2{v0, v1} : dbl2{0.0, 0.0};
                    }
            } else {
#pragma unroll
                for (int u = 0; u < XPT; ++u) {
                    const int e = tid + 256 * u, r = e / MC, c = e % MC;
                    const double v = (jpass & ~c & 1) ? -xv[u] : xv[u];
                    xs[buf][r * LDX + c] = c < mc ? v : 0.0;
                }
            }
        };
        dbl2 sa[8], sn[8];
        auto load_s = [&](int64_t b, dbl2 *dst) {
            // S_b (32 KB) through a buffer resource: streaming loads at 32-bit offsets
            const __amdgpu_buffer_rsrc_t rs = buf_rsrc(S + b * kMfmaK * kMfmaK, kMfmaK * kMfmaK * 8);
#pragma unroll
            for (int kk2 = 0; kk2 < 8; ++kk2)
                dst[kk2] = __builtin_bit_cast(dbl2, buf_ld16<kBufNT>(rs, 16u * (w * 8 * 64 + kk2 * 64 + lane)));
        };

        // the same order of products per accumulator in both layouts
        auto multiply = [&](int buf) {
            const double *xb = xs[buf];
#pragma unroll
            for (int kk2 = 0; kk2 < 8; ++kk2) {
                if constexpr (TR) {
                    dbl2 bq[NJ];  // rows 8 kk2 + lq and 8 kk2 + 4 + lq of column 16 J + lr
#pragma unroll
                    for (int J = 0; J < NJ; ++J) bq[J] = *(const dbl2 *)(xb + (16 * J + lr) * LDT + 8 * kk2 + 2 * lq);
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        const double a = h ? sa[kk2].y : sa[kk2].x;
#pragma unroll
                        for (int J = 0; J < NJ; ++J)
                            acc[J] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, h ? bq[J].y : bq[J].x, acc[J], 0, 0, 0);
                    }
                } else {
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        const double a = h ? sa[kk2].y : sa[kk2].x;
                        const int krow = 4 * (2 * kk2 + h) + lq;
#pragma unroll
                        for (int J = 0; J < NJ; ++J) {
                            const double bv = xb[krow * LDX + 16 * J + lr];
                            acc[J] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bv, acc[J], 0, 0, 0);
                        }
                    }
                }
            }
        };

        load_x(adm_col[b0]);
        load_s(b0, sa);
        store_x(0);
        __syncthreads();
        // every load of the loop is unconditional (bounds handled by clamped addresses and
        // selects) and the last block is peeled off, so the compiler's wait counters are
        // exact: the MFMAs wait only for the current block, never for the prefetch
        for (int64_t b = b0; b + 1 < b1; ++b) {
            const int buf = (int)((b - b0) & 1);
            load_x(adm_col[b + 1]);
            load_s(b + 1, sn);
            multiply(buf);
            store_x(buf ^ 1);
#pragma unroll
            for (int kk2 = 0; kk2 < 8; ++kk2) sa[kk2] = sn[kk2];
            __syncthreads();
        }
        multiply((int)((b1 - 1 - b0) & 1));
    }
    // D layout of the 16x16x4 f64 MFMA: lane l, register r -> row l / 16 + 4 r, column l % 16
#pragma unroll
    for (int J = 0; J < NJ; ++J) {
        const int col = 16 * J + lr;
        if (col < mc) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = 16 * w + lq + 4 * r;
                double *y = &yh[((int64_t)t * kMfmaK + row) * ldh + j0 + col];
                *y = jpass ? *y + acc[J][r] : acc[J][r];  // the second pass adds
            }
        }
    }
}

// Coupling for small ranks (k <= 32, row-major k x k coupling matrices).  One
// work-group of 2 waves owns one row cluster t and a slab of 16*NJ columns;
// wave w owns rows 16w..16w+15 of y_t (rows past k are zero in the operand and
// never written).  The k-steps of the 16x16x4 MFMA are permuted so that a lane
// owns two neighbouring columns of S_b per pair of k-steps: lane (r, g), g =
// lane / 16, takes columns 8q + 2g and 8q + 2g + 1 in k-steps 2q and 2q + 1, so
// its two S values are adjacent in memory; x_s (staged in LDS, three buffers) is
// read with the same permutation.  x_s and S_b are loaded two blocks ahead: a block's
// x_s carries as many bytes as its S_b here and mostly misses the L2, so one block of
// lead left its latency exposed.
// Work-groups are mapped to rows by XCD eighths as in the k = 64 kernel.
template <int NJ>
__global__ __launch_bounds__(128) void k_coupling_mfma_small(int k, int64_t m, int32_t C, int32_t rows_per_xcd,
                                                             const int32_t *__restrict__ order,
                                                             const int64_t *__restrict__ adm_ptr,
                                                             const int32_t *__restrict__ adm_col,
                                                             const double *__restrict__ S,
                                                             const double *__restrict__ xh, double *__restrict__ yh,
                                                             int64_t ldh, Skip skip, int jpass) {
    constexpr int MC = 16 * NJ;
    constexpr int LDX = MC + 1;
    __shared__ double xs[3][32 * LDX];
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
    const int nq = (k + 7) >> 3;          // pairs of k-steps (8 columns of S each)
    const int nu = 16 * w + lr;           // row of S_b held by this lane
    const bool row_ok = nu < k;

    dbl4 acc[NJ];
#pragma unroll
    for (int J = 0; J < NJ; ++J) acc[J] = dbl4{0.0, 0.0, 0.0, 0.0};

    if (b1 > b0) {
        constexpr int XPT = (32 * MC) / 128;  // x_s elements per thread (4 * NJ)
        double xv[XPT], xw[XPT];
        auto load_x = [&](int32_t s, double (&xv)[XPT]) {
            const double *src = xh + (int64_t)s * k * ldh + j0;
#pragma unroll
            for (int u = 0; u < XPT; ++u) {
                const int e = tid + 128 * u, r = e / MC, c = e % MC;
                xv[u] = src[(r < k && c < mc) ? (int64_t)r * ldh + (c ^ jpass) : 0];  // zeroed when stored
            }
        };
        auto store_x = [&](int buf, const double (&xv)[XPT]) {
#pragma unroll
            for (int u = 0; u < XPT; ++u) {
                const int e = tid + 128 * u, r = e / MC, c = e % MC;
                const double v = (jpass & ~c & 1) ? -xv[u] : xv[u];
                xs[buf][r * LDX + c] = (r < k && c < mc) ? v : 0.0;
            }
        };
        double sa[4][2], sn[4][2];
        auto load_s = [&](int64_t b, double (*dst)[2]) {
            const double *src = S + b * k * k + (int64_t)(row_ok ? nu : 0) * k;
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    // a lane past the last column reads column 0 instead: it multiplies a zero
                    // row of x_s, and rows past k are never written
                    const int mu = 8 * q + 2 * g + h;
                    dst[q][h] = __builtin_nontemporal_load(src + (row_ok && mu < k ? mu : 0));
                }
        };

        auto multiply = [&](int buf) {
            const double *xb = xs[buf];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                if (q < nq) {
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        const int krow = 8 * q + 2 * g + h;
#pragma unroll
                        for (int J = 0; J < NJ; ++J) {
                            const double bv = xb[krow * LDX + 16 * J + lr];
                            acc[J] = __builtin_amdgcn_mfma_f64_16x16x4f64(sa[q][h], bv, acc[J], 0, 0, 0);
                        }
                    }
                }
            }
        };

        // two blocks ahead: x_(b+2) is loaded while block b is multiplied and stored one step
        // later (register sets xv / xw swap roles), S_(b+2) is loaded at the end of step b;
        // three LDS buffers; every load unconditional from clamped block indices
        load_x(adm_col[b0], xv);
        load_s(b0, sa);
        store_x(0, xv);
        load_x(adm_col[min(b0 + 1, b1 - 1)], xv);
        load_s(min(b0 + 1, b1 - 1), sn);
        __syncthreads();
        int64_t b = b0;
        int cur = 0;
        auto step = [&](double (&xa)[XPT], double (&xn)[XPT]) {
            const int nxt = cur == 2 ? 0 : cur + 1;
            load_x(adm_col[min(b + 2, b1 - 1)], xn);
            multiply(cur);
            store_x(nxt, xa);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                sa[q][0] = sn[q][0];
                sa[q][1] = sn[q][1];
            }
            load_s(min(b + 2, b1 - 1), sn);
            __syncthreads();
            ++b;
            cur = nxt;
        };
        for (;;) {
            if (b + 1 >= b1) break;
            step(xv, xw);
            if (b + 1 >= b1) break;
            step(xw, xv);
        }
        multiply(cur);
    }
#pragma unroll
    for (int J = 0; J < NJ; ++J) {
        const int col = 16 * J + lr;
        if (col < mc) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = 16 * w + g + 4 * r;
                if (row < k) {
                    double *y = &yh[((int64_t)t * k + row) * ldh + j0 + col];
                    *y = jpass ? *y + acc[J][r] : acc[J][r];
                }
            }
        }
    }
}

// Launches the matrix-core coupling stage when the operator's layout supports
// it; returns false (launching nothing) otherwise.
template <typename T, typename Acc>
bool launch_coupling_fast(const DevMat &dm, int64_t m, const Acc *xh, Acc *yh, int64_t ldh, hipStream_t st,
                          Skip skip, int nj_force, int jpass = 0, int32_t nrows = -1, const int32_t *rows = nullptr,
                          size_t keep_lds = 0) {
    if constexpr (!std::is_same<T, double>::value || !std::is_same<Acc, double>::value) {
        return false;
    } else {
        if (!dm.mc || !dm.cpl_order) return false;
        // all rows in cpl_order, or the part (nrows, rows) of them
        const int32_t C = rows ? nrows : dm.C;
        const int32_t *order = rows ? rows : dm.cpl_order;
        if (C <= 0) return true;
        const int nj = nj_force ? nj_force : (int)std::min<int64_t>(4, (m + 15) / 16);
        const int mcols = 16 * nj;
        const int32_t rpx = (C + 7) / 8;
        const dim3 grid((unsigned)(8 * rpx * ((m + mcols - 1) / mcols)));
        // jpass (complex operator): the imaginary plane of S on J x-hat, added to y-hat
        const double *S = (const double *)dm.S + (jpass ? dm.s_plane : 0);
        if (dm.k <= 32) {
            auto go = [&](auto NJc) {
                constexpr int NJ = decltype(NJc)::value;
                hipLaunchKernelGGL(k_coupling_mfma_small<NJ>, grid, dim3(128), 0, st, dm.k, m, C, rpx,
                                   order, dm.adm_ptr, dm.adm_col, S, xh, yh, ldh, skip, jpass);
            };
            switch (nj) {
                case 1: go(std::integral_constant<int, 1>{}); break;
                case 2: go(std::integral_constant<int, 2>{}); break;
                case 3: go(std::integral_constant<int, 3>{}); break;
                default: go(std::integral_constant<int, 4>{}); break;
            }
            return true;
        }
        if (dm.swz != 1 || dm.k != kMfmaK) return false;
        // keep_lds > 0: each work-group also takes unused dynamic LDS, so that a CU holds at
        // most two of them and keep_lds bytes stay free for a work-group of another launch
        // (the work-groups of a long launch must not take every slot of the chip)
        auto dyn_lds = [&](const void *fn) -> size_t {
            if (!keep_lds) return 0;
            hipFuncAttributes a{};
            int dev = 0, per_cu = 0;
            if (hipFuncGetAttributes(&a, fn) != hipSuccess || hipGetDevice(&dev) != hipSuccess ||
                hipDeviceGetAttribute(&per_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) !=
                    hipSuccess || (size_t)per_cu <= keep_lds)
                return 0;
            const size_t target = (((size_t)per_cu - keep_lds) / 2) & ~(size_t)255;
            return target > a.sharedSizeBytes ? target - a.sharedSizeBytes : 0;
        };
        auto go = [&](auto NJc) {
            constexpr int NJ = decltype(NJc)::value;
            const size_t dyn = dyn_lds((const void *)k_coupling_mfma_f64<NJ>);
            hipLaunchKernelGGL(k_coupling_mfma_f64<NJ>, grid, dim3(256), dyn, st, m, C, rpx, order, dm.adm_ptr,
                               dm.adm_col, S, xh, yh, ldh, skip, jpass);
        };
        switch (nj) {
            case 1: go(std::integral_constant<int, 1>{}); break;
            case 2: go(std::integral_constant<int, 2>{}); break;
            case 3: go(std::integral_constant<int, 3>{}); break;
            default: go(std::integral_constant<int, 4>{}); break;
        }
        return true;
    }
}

}  // namespace h2x
