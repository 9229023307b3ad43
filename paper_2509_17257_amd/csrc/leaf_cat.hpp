// Leaf stage of the FP64 operator as one contraction per leaf (matrix cores).
//
//   Y|_t = beta Y|_t + alpha (V_t y_t + sum_{(t,s) near} N_ts X|_s)
//
// computed in the transposed orientation Y_t^T = [X_s1^T ... X_sq^T y_t^T] [N_ts1^T; ...; N_tsq^T; V_t^T]:
// the near blocks of a leaf are stored transposed one after another with the same row
// length |t| (padded to even), so the near field of leaf t is one matrix of R_t = sum |s|
// rows, and the transposed leaf basis adds k rows.  The contraction runs over these rows in
// rounds of 16 (four 4-long matrix-core steps); the right operand of a row is the row of X
// of its point (a per-leaf table in LDS maps near rows to tree positions) or the row of
// y_t.  Only the end of each segment is padded (to 16 rows), and the rows of the leaf come
// in 16-row tiles, so a leaf of 43 points and 1100 near rows costs 48 x 1104 instead of
// 64 x 1152 terms per column.
//
// Work-group: 4 waves for one (leaf, slab of 32 * NP columns).  A wave holds at most two
// 16-row tiles: leaves of up to 32 rows are one row group and the 4 waves split the rounds
// (wave w takes rounds w, w + 4, ...); larger leaves are two row groups of two tiles, each
// split over 2 waves.  The partial tiles of the waves of a row group are added in LDS in
// wave order (a fixed order: the result is reproducible).  Three register sets keep two
// rounds of loads in flight behind the matrix-core work of the current one; every load is
// issued unconditionally from a clamped in-range address (a round past the wave's last
// re-reads that round, which the cache serves) so that the compiler's wait counts stay
// exact, and rows past a segment are zeroed where they are used.
//
// Lane layout of v_mfma_f64_16x16x4f64 (A: 16 x 4, B: 4 x 16, D: 16 x 16): lane l holds
// A[l % 16][l / 16], B[l / 16][l % 16] and D rows l / 16 + 4 r, column l % 16 (r = 0..3).
// Here A = X^T (M over columns of X: a lane loads two neighbouring columns with one 16-byte
// load, which feed an "even" and an "odd" column tile), B = N^T (N over rows of the leaf).
#pragma once

#include "device.hpp"
#include "stages_mfma.hpp"

namespace h2x {
namespace mfma {

typedef double dbl4c __attribute__((ext_vector_type(4)));
typedef double dbl2c __attribute__((ext_vector_type(2)));

template <int NP>
struct CatRound {
    dbl2c a[NP][4];  // [column half p][k-step u]: columns 32p + 2 (l % 16) + {0, 1}
    double b[2][4];  // [row tile of the wave][k-step u]: row 16 I + l % 16
    int ok[4];       // k-row of step u inside its segment
};

// registers of one round of a wave that takes one 32-column half and three row tiles
struct CatHalf {
    dbl2c a[4];      // [k-step u]: columns 32 (w >> 1) + 2 (l % 16) + {0, 1}
    double b[3][4];  // [row tile][k-step u]
    int ok[4];
};

// rows of the near field of one leaf, as a table of tree positions in LDS (built from the
// blocks' offsets: block q starts at near row (off_q - off_q0) / |t|_even)
__device__ inline int32_t cat_build_rows(int32_t *xrow, int64_t q0, int nnear, int64_t nt2,
                                         const int32_t *__restrict__ near_col, const int64_t *__restrict__ near_off,
                                         const int32_t *__restrict__ first, const int32_t *__restrict__ size) {
    __shared__ int32_t rn;
    const int64_t base = near_off[q0];
    if (threadIdx.x == 0) rn = 0;
    __syncthreads();
    for (int x = threadIdx.x; x < nnear; x += blockDim.x) {
        const int32_t s = near_col[q0 + x];
        const int32_t off = (int32_t)((near_off[q0 + x] - base) / nt2), fs = first[s], ks = size[s];
        for (int c = 0; c < ks; ++c) xrow[off + c] = fs + c;
        if (x == nnear - 1) rn = off + ks;
    }
    __syncthreads();
    return rn;
}

// the leaf stage's arguments (one struct, shared by the kernels that run leaf work)
struct LeafCatArgs {
    int k;
    int64_t m;
    int32_t L;
    const int32_t *order;  // launch order of the leaves (leaf indices)
    const int32_t *leaves, *first, *size;
    const int64_t *perm;
    const double *Vt;
    const int64_t *vt_off;
    const double *yh;
    int64_t ldh;
    const int64_t *near_ptr;
    const int32_t *near_col;
    const int64_t *near_off;
    const double *Nt, *Xt;
    int64_t ldxt;
    double alpha, beta;
    double *Y;
    int64_t ldy;
    int tree_order, basis, near;
    Skip skip;
};

// LDS of the leaf work: the partial-tile buffer, then the near-row table
template <int NP>
constexpr size_t leaf_cat_red_bytes() { return sizeof(double) * 64 * (32 * NP + 1); }

// one (leaf, column slab) slot: slot & 7 is the XCD, whose leaves form one contiguous
// eighth (taken in the order of a.order: the most work first); the slabs of one leaf are
// consecutive slots of one XCD, so its near blocks come from HBM once.  red: 64 x (32 NP + 1) doubles of LDS; xrow: the near-row table.
template <int NP>
__device__ inline void leaf_cat_slot(int64_t slot, const LeafCatArgs &a, double *red, int32_t *xrow) {
    constexpr int MC = 32 * NP, LDR = MC + 1;
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
    const int nnear = a.near ? (int)(a.near_ptr[l + 1] - q0) : 0;
    const int32_t rn = nnear > 0 ? cat_build_rows(xrow, q0, nnear, nt2, a.near_col, a.near_off, a.first, a.size) : 0;
    const double *nb = nnear > 0 ? a.Nt + a.near_off[q0] : a.Nt;
    const double *vb = a.Vt + a.vt_off[l];
    const int RN = (rn + 15) >> 4, RB = a.basis ? (k + 15) >> 4 : 0, RT = RN + RB;
    const int xc = (mc - 1) & ~1;  // last even column offset of the slab

    for (int i0 = 0; i0 < nt; i0 += 64) {
        const int ic = min(64, nt - i0);
        const int ntile = (ic + 15) >> 4;
        if (NP == 2 && ntile == 3) {
            // 64 columns, 33-48 rows: wave w takes the column half w >> 1 and the k-group w & 1
            // for all three row tiles, so every wave has the same matrix-core work and each X
            // row is loaded once (two row groups would give one wave pair a single tile and
            // load the X rows twice); the same rounds per k-group and the same order of adds
            // as the row groups, so the result is the same bit for bit
            const int ch = w >> 1, g = w & 1;
            int rw[3];
#pragma unroll
            for (int I = 0; I < 3; ++I) rw[I] = i0 + min(16 * I + lr, ic - 1);
            dbl4c acc[2][3];
#pragma unroll
            for (int hj = 0; hj < 2; ++hj)
#pragma unroll
                for (int I = 0; I < 3; ++I) acc[hj][I] = dbl4c{0.0, 0.0, 0.0, 0.0};
            auto load = [&](int r, CatHalf &R) {
                const bool nr = r < RN;
                const double *ab = nr ? a.Xt + j0 : a.yh + (int64_t)t * k * a.ldh + j0;
                const int64_t lda = nr ? a.ldxt : a.ldh;
                const double *bb = nr ? nb : vb;
                const int c0 = nr ? 16 * r : 16 * (r - RN), lim = nr ? rn : k;
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int c = c0 + 4 * u + lq, cc = min(c, lim - 1);
                    R.ok[u] = c < lim;
                    const int64_t arow = nr ? (int64_t)xrow[cc] : (int64_t)cc;
                    R.a[u] = __builtin_bit_cast(
                        dbl2c, buf_ld16<0>(buf_rsrc(ab, 0xFFFFFFFFu),
                                           8u * (uint32_t)(arow * lda + min(32 * ch + 2 * lr, xc))));
#pragma unroll
                    for (int I = 0; I < 3; ++I) R.b[I][u] = bb[(int64_t)cc * nt2 + rw[I]];
                }
            };
            auto multiply = [&](CatHalf &R) {
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const dbl2c v = R.ok[u] ? R.a[u] : dbl2c{0.0, 0.0};
#pragma unroll
                    for (int hj = 0; hj < 2; ++hj)
#pragma unroll
                        for (int I = 0; I < 3; ++I)
                            acc[hj][I] = __builtin_amdgcn_mfma_f64_16x16x4f64(v[hj], R.b[I][u], acc[hj][I], 0, 0, 0);
                }
            };
            if (g < RT) {
                const int last = g + ((RT - 1 - g) / 2) * 2;
                CatHalf s0, s1;  // two register sets in turn: one round of loads in flight
                int r = g;
                load(r, s0);
                for (;;) {
                    load(min(r + 2, last), s1);
                    multiply(s0);
                    r += 2;
                    if (r > last) break;
                    load(min(r + 2, last), s0);
                    multiply(s1);
                    r += 2;
                    if (r > last) break;
                }
            }
            for (int gg = 0; gg < 2; ++gg) {
                if (g == gg)
#pragma unroll
                    for (int hj = 0; hj < 2; ++hj)
#pragma unroll
                        for (int I = 0; I < 3; ++I)
#pragma unroll
                            for (int q = 0; q < 4; ++q) {
                                const int col = 32 * ch + 2 * (lq + 4 * q) + hj;
                                double *cell = &red[(16 * I + lr) * LDR + col];
                                *cell = (gg == 0) ? acc[hj][I][q] : *cell + acc[hj][I][q];
                            }
                __syncthreads();
            }
        } else {
            const int G = ntile > 2 ? 2 : 4;          // waves per row group (k-groups)
            const int wr = w / G, g = w - wr * G;     // row group, k-group (wave-uniform)
            const int tl0 = 2 * wr;                   // first row tile of the wave
            const bool t0 = tl0 < ntile, t1 = tl0 + 1 < ntile;
            const int row_a = i0 + min(16 * tl0 + lr, ic - 1), row_b = i0 + min(16 * tl0 + 16 + lr, ic - 1);

            dbl4c acc[2 * NP][2];
    #pragma unroll
            for (int J = 0; J < 2 * NP; ++J) acc[J][0] = acc[J][1] = dbl4c{0.0, 0.0, 0.0, 0.0};

            // round r (clamped to the wave's rounds) -> registers
            auto load = [&](int r, CatRound<NP> &R) {
                const bool nr = r < RN;
                const double *ab;
                int64_t lda;
                const double *bb;
                int c0, lim;
                if (nr) {
                    c0 = 16 * r;
                    lim = rn;
                    bb = nb;
                    lda = a.ldxt;
                    ab = a.Xt + j0;
                } else {
                    c0 = 16 * (r - RN);
                    lim = k;
                    bb = vb;
                    lda = a.ldh;
                    ab = a.yh + (int64_t)t * k * a.ldh + j0;
                }
    #pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int c = c0 + 4 * u + lq, cc = min(c, lim - 1);
                    R.ok[u] = c < lim;
                    const int64_t arow = nr ? (int64_t)xrow[cc] : (int64_t)cc;
    #pragma unroll
                    for (int p = 0; p < NP; ++p)
                        R.a[p][u] = __builtin_bit_cast(
                            dbl2c, buf_ld16<0>(buf_rsrc(ab, 0xFFFFFFFFu),
                                               8u * (uint32_t)(arow * lda + min(32 * p + 2 * lr, xc))));
                    R.b[0][u] = bb[(int64_t)cc * nt2 + row_a];
                    R.b[1][u] = bb[(int64_t)cc * nt2 + row_b];
                }
            };
            auto multiply = [&](CatRound<NP> &R) {
    #pragma unroll
                for (int u = 0; u < 4; ++u) {
    #pragma unroll
                    for (int p = 0; p < NP; ++p) {
                        const dbl2c v = R.ok[u] ? R.a[p][u] : dbl2c{0.0, 0.0};
    #pragma unroll
                        for (int hj = 0; hj < 2; ++hj) {
                            if (t0)
                                acc[2 * p + hj][0] =
                                    __builtin_amdgcn_mfma_f64_16x16x4f64(v[hj], R.b[0][u], acc[2 * p + hj][0], 0, 0, 0);
                            if (t1)
                                acc[2 * p + hj][1] =
                                    __builtin_amdgcn_mfma_f64_16x16x4f64(v[hj], R.b[1][u], acc[2 * p + hj][1], 0, 0, 0);
                        }
                    }
                }
            };

            if (g < RT) {
                const int last = g + ((RT - 1 - g) / G) * G;  // the wave's last round
                CatRound<NP> s0, s1, s2;
                int r = g;
                load(r, s0);
                load(min(r + G, last), s1);
                // three register sets in turn; a set is loaded two rounds ahead of its use
                for (;;) {
                    load(min(r + 2 * G, last), s2);
                    multiply(s0);
                    r += G;
                    if (r > last) break;
                    load(min(r + 2 * G, last), s0);
                    multiply(s1);
                    r += G;
                    if (r > last) break;
                    load(min(r + 2 * G, last), s1);
                    multiply(s2);
                    r += G;
                    if (r > last) break;
                }
            }
            // partial tiles of the G waves of each row group, added in wave order.  Lane l,
            // register q of acc[2p + hj][I] -> column 32p + 2 (l / 16 + 4 q) + hj, row
            // 16 (tl0 + I) + l % 16.
            for (int gg = 0; gg < G; ++gg) {
                if (g == gg)
    #pragma unroll
                    for (int J = 0; J < 2 * NP; ++J)
    #pragma unroll
                        for (int I = 0; I < 2; ++I)
    #pragma unroll
                            for (int q = 0; q < 4; ++q) {
                                const int col = 32 * (J >> 1) + 2 * (lq + 4 * q) + (J & 1);
                                const int row = 16 * (tl0 + I) + lr;
                                double *cell = &red[row * LDR + col];
                                *cell = (gg == 0) ? acc[J][I][q] : *cell + acc[J][I][q];
                            }
                __syncthreads();
            }
        }
        for (int x = threadIdx.x; x < ic * MC; x += 256) {
            const int i = x / MC, j = x - i * MC;
            if (j < mc) {
                int64_t row = r0 + i0 + i;
                if (!a.tree_order) row = a.perm[row];
                double *y = &a.Y[row * a.ldy + j0 + j];
                const double v = a.alpha * red[i * LDR + j];
                *y = (a.beta == 0.0) ? v : a.beta * *y + v;
            }
        }
        __syncthreads();
    }
}

// ---- the near-field term of d ell ----
//
// sum over leaves t of <dY|_t, sum_{(t,s) near} G_ts X|_s> with G_ts[i][c] =
// dg/dell(x_i, x_c) = (r / ell^2) exp(-r / ell) = (r / ell^2) N_ts[i][c] for the exponential
// kernel (the shift on the diagonal sits where r = 0): the near-field contraction of the leaf
// stage with the stored N scaled by r / ell^2 (r from the points, tree order).  Same slots,
// near-row table, row groups and rounds as leaf_cat_slot; returns the work-group's partial
// sum of the dot product (the same value in every thread).
struct DellArgs {
    const double *pts;  // n x 3, tree order
    double inv_ell, inv_ell2;
    const double *dYt;  // n x ldt, tree order
    int64_t ldt;
};

template <int NP>
struct DellRound {
    dbl2c a[NP][4];
    double c[4][3];  // coordinates of the near row's point of each k-step
    double n[2][4];  // the stored near-field entries (row tile of the wave, k-step)
    int ok[4];
};

template <int NP>
__device__ inline double leaf_dell_slot(int64_t slot, const LeafCatArgs &a, const DellArgs &d, double *red,
                                        int32_t *xrow) {
    constexpr int MC = 32 * NP, LDR = MC + 1;
    __shared__ double part_red[256];
    const int32_t per_xcd = (a.L + 7) / 8;
    const int nslab = (int)((a.m + MC - 1) / MC);
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63, lr = lane & 15,
              lq = lane >> 4;
    const int64_t qx = slot >> 3;
    const int32_t pos = (int32_t)((slot & 7) * per_xcd + qx / nslab);
    if (pos >= a.L) return 0.0;
    const int32_t l = a.order[pos];
    const int32_t t = a.leaves[l];
    const int nt = a.size[t];
    const int64_t nt2 = pad_rows(nt), r0 = a.first[t];
    const int64_t j0 = (qx % nslab) * MC;
    const int mc = (int)min<int64_t>(MC, a.m - j0);
    const int64_t q0 = a.near_ptr[l];
    const int nnear = (int)(a.near_ptr[l + 1] - q0);
    const int32_t rn = nnear > 0 ? cat_build_rows(xrow, q0, nnear, nt2, a.near_col, a.near_off, a.first, a.size) : 0;
    const int RT = (rn + 15) >> 4;
    const double *nb = nnear > 0 ? a.Nt + a.near_off[q0] : a.Nt;
    const int xc = (mc - 1) & ~1;
    double mine = 0.0;

    for (int i0 = 0; i0 < nt; i0 += 64) {
        const int ic = min(64, nt - i0);
        const int ntile = (ic + 15) >> 4;
        const int G = ntile > 2 ? 2 : 4;
        const int wr = w / G, g = w - wr * G;
        const int tl0 = 2 * wr;
        const bool t0 = tl0 < ntile, t1 = tl0 + 1 < ntile;
        const int64_t pa = r0 + i0 + min(16 * tl0 + lr, ic - 1), pb = r0 + i0 + min(16 * tl0 + 16 + lr, ic - 1);
        const double ax = d.pts[3 * pa], ay = d.pts[3 * pa + 1], az = d.pts[3 * pa + 2];
        const double bx = d.pts[3 * pb], by = d.pts[3 * pb + 1], bz = d.pts[3 * pb + 2];

        dbl4c acc[2 * NP][2];
#pragma unroll
        for (int J = 0; J < 2 * NP; ++J) acc[J][0] = acc[J][1] = dbl4c{0.0, 0.0, 0.0, 0.0};

        auto load = [&](int r, DellRound<NP> &R) {
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int c = 16 * r + 4 * u + lq, cc = min(c, rn - 1);
                R.ok[u] = c < rn;
                const int64_t xr = xrow[cc];
#pragma unroll
                for (int p = 0; p < NP; ++p)
                    R.a[p][u] = *(const dbl2c *)(a.Xt + j0 + xr * a.ldxt + min(32 * p + 2 * lr, xc));
#pragma unroll
                for (int q = 0; q < 3; ++q) R.c[u][q] = d.pts[3 * xr + q];
                R.n[0][u] = nb[(int64_t)cc * nt2 + (pa - r0)];
                R.n[1][u] = nb[(int64_t)cc * nt2 + (pb - r0)];
            }
        };
        auto gval = [&](double x, double y, double z, const double *c, double nv) {
            const double dx = x - c[0], dy = y - c[1], dz = z - c[2];
            const double r = sqrt(dx * dx + dy * dy + dz * dz);
            return (r * d.inv_ell2) * nv;
        };
        auto multiply = [&](DellRound<NP> &R) {
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const double g0 = t0 ? gval(ax, ay, az, R.c[u], R.n[0][u]) : 0.0;
                const double g1 = t1 ? gval(bx, by, bz, R.c[u], R.n[1][u]) : 0.0;
#pragma unroll
                for (int p = 0; p < NP; ++p) {
                    const dbl2c v = R.ok[u] ? R.a[p][u] : dbl2c{0.0, 0.0};
#pragma unroll
                    for (int hj = 0; hj < 2; ++hj) {
                        if (t0)
                            acc[2 * p + hj][0] =
                                __builtin_amdgcn_mfma_f64_16x16x4f64(v[hj], g0, acc[2 * p + hj][0], 0, 0, 0);
                        if (t1)
                            acc[2 * p + hj][1] =
                                __builtin_amdgcn_mfma_f64_16x16x4f64(v[hj], g1, acc[2 * p + hj][1], 0, 0, 0);
                    }
                }
            }
        };
        if (g < RT) {
            const int last = g + ((RT - 1 - g) / G) * G;
            DellRound<NP> s0, s1, s2;
            int r = g;
            load(r, s0);
            load(min(r + G, last), s1);
            for (;;) {
                load(min(r + 2 * G, last), s2);
                multiply(s0);
                r += G;
                if (r > last) break;
                load(min(r + 2 * G, last), s0);
                multiply(s1);
                r += G;
                if (r > last) break;
                load(min(r + 2 * G, last), s1);
                multiply(s2);
                r += G;
                if (r > last) break;
            }
        }
        for (int gg = 0; gg < G; ++gg) {
            if (g == gg)
#pragma unroll
                for (int J = 0; J < 2 * NP; ++J)
#pragma unroll
                    for (int I = 0; I < 2; ++I)
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            const int col = 32 * (J >> 1) + 2 * (lq + 4 * q) + (J & 1);
                            const int row = 16 * (tl0 + I) + lr;
                            double *cell = &red[row * LDR + col];
                            *cell = (gg == 0) ? acc[J][I][q] : *cell + acc[J][I][q];
                        }
            __syncthreads();
        }
        // <dY|_t, G X> over the chunk's rows and the slab's columns
        for (int x = threadIdx.x; x < ic * MC; x += 256) {
            const int i = x / MC, j = x - i * MC;
            if (j < mc) mine += red[i * LDR + j] * d.dYt[(r0 + i0 + i) * d.ldt + j0 + j];
        }
        __syncthreads();
    }
    // the work-group's sum in a fixed order
    part_red[threadIdx.x] = mine;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) part_red[threadIdx.x] += part_red[threadIdx.x + h];
        __syncthreads();
    }
    const double tot = part_red[0];
    __syncthreads();
    return tot;
}

// near-field term of d ell: one slot per work-group, part[blockIdx.x] = its partial sum
template <int NP>
__global__ __launch_bounds__(256, 2) void k_dell_near(LeafCatArgs a, DellArgs d, double *__restrict__ part) {
    __shared__ double red[64 * (32 * NP + 1)];
    extern __shared__ int32_t xrow[];
    const double tot = leaf_dell_slot<NP>(blockIdx.x, a, d, red, xrow);
    if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

// the leaf stage over slots [slot0, slot1): dynamic LDS = the near-row table
template <int NP>
__global__ __launch_bounds__(256, NP == 1 ? 3 : 2) void k_leaf_cat(LeafCatArgs a, int64_t slot0, int64_t slot1) {
    __shared__ double red[64 * (32 * NP + 1)];
    extern __shared__ int32_t xrow[];
    for (int64_t slot = slot0 + blockIdx.x; slot < slot1; slot += gridDim.x) leaf_cat_slot<NP>(slot, a, red, xrow);
}

// A transfer level with a share of the near field beside it: work-groups [0, items) run the
// level (item i: list entry i / gy, column slab i % gy), work-group items + lead + s runs
// leaf slot slot0 + s with near = 1, basis = 0 (the near field needs only X); the `lead`
// idle work-groups put slot s on XCD s % 8 (work-groups are dealt to the XCDs in turn), as
// in the leaf stage's own launch.  The level's chain of dependent launches then overlaps
// streaming near-field work.  Dynamic LDS: the larger of the level's operand tiles and the
// leaf work's buffers.
template <int NJ, int NP, int UP>
__global__ __launch_bounds__(256, 2) void k_level_near(int64_t items, int gy, int64_t m, const int32_t *__restrict__ list,
                                                       const int32_t *__restrict__ aux, const double *__restrict__ E,
                                                       double *__restrict__ hat, int64_t ldh, Skip skip,
                                                       LeafCatArgs a, int64_t slot0, int lead) {
    extern __shared__ double lds[];
    const int64_t b = blockIdx.x;
    if (b < items) {
        const int i = (int)(b / gy), by = (int)(b - (int64_t)i * gy);
        if (UP)
            up64_item<NJ>(i, by, m, list, aux, E, hat, ldh, skip, lds);
        else
            down64_item<NJ>(i, by, m, list, aux, E, hat, ldh, skip, lds);
    } else if (b >= items + lead) {
        leaf_cat_slot<NP>(slot0 + (b - items - lead), a, lds, (int32_t *)(lds + 64 * (32 * NP + 1)));
    }
}

}  // namespace mfma
}  // namespace h2x
