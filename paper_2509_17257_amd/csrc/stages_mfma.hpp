// Matrix-core (MFMA) kernels for the FP64 operator with rank k <= 64: forward
// leaf transform, upward and downward transfer passes, and the leaf stage
// (near field and leaf basis).  Each work-group (4 waves) computes one output
// tile of 64 rows x 16*NJ columns; wave w owns rows 16w..16w+15 (waves whose
// rows all lie beyond k skip the multiplications).  Operands are
// staged through LDS with coalesced global loads (a near-field block is one
// contiguous |t| x |s| array), then v_mfma_f64_16x16x4f64 accumulates in
// registers.  Contraction lengths are padded to a multiple of 4 with zeros in
// LDS, rows beyond the block are never written back.
#pragma once

#include "device.hpp"

namespace h2x {
namespace mfma {

typedef double dbl4 __attribute__((ext_vector_type(4)));

constexpr int K = 64;     // largest rank handled by these kernels
constexpr int LDA = K + 1;  // padded LDS row of the left operand

template <int NJ>
struct Smem {  // operand tiles of one work-group
    static constexpr int MC = 16 * NJ;
    static constexpr int LDB = MC + 1;
    double a[64 * LDA];
    double b[64 * LDB];
};

// index split e -> (e / d, e % d) for e < 4096, d <= 64, via a float reciprocal:
// (e + 0.5) / d is at least 0.5 / d away from an integer, far above the error
__device__ inline void split(int e, int d, float inv_d, int &q, int &r) {
    q = (int)((e + 0.5f) * inv_d);
    r = e - q * d;
}

// One term A B of a sum accumulated into a 64 x 16*NJ tile.
// A: arows x acols row-major at a (row stride lda); trans == false puts
// A[i][c] at LDS row i (contraction over c), trans == true puts it at LDS row c
// (contraction over i).  B: contraction-length rows, row r at
// b + row(r) * ldb with row(r) = perm ? perm[brow0 + r] : brow0 + r.
struct Term {
    const double *a;
    int64_t lda;
    int arows, acols;
    bool trans;
    const double *b;
    int64_t ldb;
    const int64_t *perm;
    int64_t brow0;
    __device__ int klen() const { return trans ? arows : acols; }
};

template <int NJ>
struct Regs {
    double a[16];
    double b[4 * NJ];
};

// global -> registers: all loads of a term issued back to back, none in a branch
// (an element past the term reads an in-range neighbour and is replaced by zero
// when stored), so that the loads of several terms can be in flight together.
// A term has at least one row and one column.
template <int NJ>
__device__ inline void load_term(const Term &d, int mc, Regs<NJ> &R) {
    constexpr int MC = 16 * NJ;
    const int tid = threadIdx.x, total = d.arows * d.acols;
    const float inv = 1.0f / (float)d.acols;
#pragma unroll
    for (int u = 0; u < 16; ++u) {
        int i, c;
        split(min(tid + 256 * u, total - 1), d.acols, inv, i, c);
        R.a[u] = d.a[(int64_t)i * d.lda + c];
    }
    const int kl = d.klen();
#pragma unroll
    for (int u = 0; u < 4 * NJ; ++u) {
        const int e = tid + 256 * u, r = min(e / MC, kl - 1), c = min(e % MC, mc - 1);
        const int64_t g = d.perm ? d.perm[d.brow0 + r] : d.brow0 + r;
        R.b[u] = d.b[g * d.ldb + c];
    }
}

// registers -> LDS.  The right operand tile is rewritten in full (zeros past the
// contraction length and past the last column), so stale left-operand padding
// only ever meets zeros; the tiles are cleared once per kernel wherever padding
// exists so that it is finite.
template <int NJ>
__device__ inline void store_term(const Term &d, int mc, const Regs<NJ> &R, Smem<NJ> &sm) {
    constexpr int MC = 16 * NJ, LDB = MC + 1;
    const int tid = threadIdx.x, total = d.arows * d.acols;
    const float inv = 1.0f / (float)d.acols;
#pragma unroll
    for (int u = 0; u < 16; ++u) {
        const int e = tid + 256 * u;
        if (e < total) {
            int i, c;
            split(e, d.acols, inv, i, c);
            if (d.trans) sm.a[c * LDA + i] = R.a[u];
            else sm.a[i * LDA + c] = R.a[u];
        }
    }
    const int kl = d.klen();
#pragma unroll
    for (int u = 0; u < 4 * NJ; ++u) {
        const int e = tid + 256 * u, r = e / MC, c = e % MC;
        sm.b[r * LDB + c] = (r < kl && c < mc) ? R.b[u] : 0.0;
    }
}

template <int NJ>
__device__ inline void clear(Smem<NJ> &sm) {
    constexpr int NA = 64 * LDA, NB = 64 * Smem<NJ>::LDB;
    for (int e = threadIdx.x; e < NA; e += 256) sm.a[e] = 0.0;
    for (int e = threadIdx.x; e < NB; e += 256) sm.b[e] = 0.0;
    __syncthreads();
}

template <int NJ>
__device__ inline void mma(const double *As, const double *Bs, int kpad, int rows, dbl4 *acc) {
    constexpr int LDB = 16 * NJ + 1;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (16 * w >= rows) return;  // wave-uniform: no output row of this wave exists
    const int lr = lane & 15, lq = lane >> 4;
    const double *arow = As + (16 * w + lr) * LDA + lq;
    const double *bcol = Bs + lq * LDB + lr;
    for (int kk = 0; kk < kpad; kk += 4) {
        const double a = arow[kk];
#pragma unroll
        for (int J = 0; J < NJ; ++J) acc[J] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bcol[kk * LDB + 16 * J], acc[J], 0, 0, 0);
    }
}

template <int NJ>
__device__ inline void zero(dbl4 *acc) {
#pragma unroll
    for (int J = 0; J < NJ; ++J) acc[J] = dbl4{0.0, 0.0, 0.0, 0.0};
}

__device__ inline int dkpad4(int v) { return (v + 3) & ~3; }

// acc += sum_{q < nq} A_q B_q; the next term's global loads are in flight while
// the matrix cores work on the current one.  A term with no columns adds nothing.
template <int NJ, typename F>
__device__ inline void accumulate(Smem<NJ> &sm, dbl4 *acc, int nq, int mc, int rows, F term) {
    if (nq <= 0) return;
    Regs<NJ> R;
    Term d = term(0);
    load_term<NJ>(d, mc, R);
    for (int q = 0; q < nq; ++q) {
        store_term<NJ>(d, mc, R, sm);
        __syncthreads();
        const int kp = dkpad4(d.klen());
        if (q + 1 < nq) {
            d = term(q + 1);
            load_term<NJ>(d, mc, R);
        }
        mma<NJ>(sm.a, sm.b, kp, rows, acc);
        __syncthreads();
    }
}

// result element (lane, J, r) -> (row, col) of the 64 x 16*NJ tile
__device__ inline int out_row(int r) { return 16 * (threadIdx.x >> 6) + ((threadIdx.x & 63) >> 4) + 4 * r; }
__device__ inline int out_col(int J) { return 16 * J + (threadIdx.x & 15); }

// x_t = V_t^T X|_t for each leaf t
template <int NJ>
__global__ __launch_bounds__(256) void k_fwd_leaf(int k, int64_t m, const int32_t *__restrict__ leaves,
                                                  const int32_t *__restrict__ first, const int32_t *__restrict__ size,
                                                  const int64_t *__restrict__ perm, const double *__restrict__ V,
                                                  const double *__restrict__ X, int64_t ldx, int tree_order,
                                                  double *__restrict__ xh, int64_t ldh, Skip skip) {
    __shared__ Smem<NJ> sm;
    const int32_t t = leaves[blockIdx.x];
    if (skip(t)) return;
    const int64_t j0 = (int64_t)blockIdx.y * Smem<NJ>::MC;
    const int mc = (int)min<int64_t>(Smem<NJ>::MC, m - j0);
    const int64_t r0 = first[t];
    const int nt = size[t];
    clear<NJ>(sm);
    dbl4 acc[NJ];
    zero<NJ>(acc);
    const int64_t *pm = tree_order ? nullptr : perm;
    accumulate<NJ>(sm, acc, (nt + 63) / 64, mc, k, [&](int q) {
        const int i0 = 64 * q;
        return Term{V + (r0 + i0) * k, k, min(64, nt - i0), k, true, X + j0, ldx, pm, r0 + i0};
    });
#pragma unroll
    for (int J = 0; J < NJ; ++J)
        if (out_col(J) < mc)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                if (out_row(r) < k) xh[((int64_t)t * k + out_row(r)) * ldh + j0 + out_col(J)] = acc[J][r];
}

// x_t = E_{t0}^T x_{t0} + E_{t1}^T x_{t1} for the inner clusters in `list`;
// son[2 i], son[2 i + 1] are the sons of list[i].  Both terms are loaded at once.
template <int NJ>
__global__ __launch_bounds__(256) void k_up(int k, int64_t m, const int32_t *__restrict__ list,
                                            const int32_t *__restrict__ son, const double *__restrict__ E,
                                            double *__restrict__ xh, int64_t ldh, Skip skip) {
    __shared__ Smem<NJ> sm;
    const int32_t t = list[blockIdx.x], s0 = son[2 * blockIdx.x], s1 = son[2 * blockIdx.x + 1];
    if (skip(t)) return;
    const int64_t j0 = (int64_t)blockIdx.y * Smem<NJ>::MC;
    const int mc = (int)min<int64_t>(Smem<NJ>::MC, m - j0);
    auto term = [&](int32_t sn) {
        return Term{E + (int64_t)sn * k * k, k, k, k, true, xh + j0, ldh, nullptr, (int64_t)sn * k};
    };
    const Term d0 = term(s0), d1 = term(s1);
    Regs<NJ> R0, R1;
    load_term<NJ>(d0, mc, R0);
    load_term<NJ>(d1, mc, R1);
    if (k < K) clear<NJ>(sm);  // padding rows and columns of the k x k tiles
    dbl4 acc[NJ];
    zero<NJ>(acc);
    const int kp = dkpad4(k);
    store_term<NJ>(d0, mc, R0, sm);
    __syncthreads();
    mma<NJ>(sm.a, sm.b, kp, k, acc);
    __syncthreads();
    store_term<NJ>(d1, mc, R1, sm);
    __syncthreads();
    mma<NJ>(sm.a, sm.b, kp, k, acc);
#pragma unroll
    for (int J = 0; J < NJ; ++J)
        if (out_col(J) < mc)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                if (out_row(r) < k) xh[((int64_t)t * k + out_row(r)) * ldh + j0 + out_col(J)] = acc[J][r];
}

// Forward leaf transform and upward transfer pass in one launch: the work-group
// of leaf t computes x_t = V_t^T X|_t, then walks up the tree.  At each parent
// the work-group that finishes second (a device-scope counter per parent and
// column slab; the results are published with device-scope fences before the
// count) computes x_p = E_{s0}^T x_{s0} + E_{s1}^T x_{s1}; the first one stops.
// Clusters above min_depth are not needed.  No work-group ever waits for
// another.  cnt (clusters x column slabs) must be zero on entry.
template <int NJ>
__global__ __launch_bounds__(256) void k_fwd_up(int k, int64_t m, int32_t L, const int32_t *__restrict__ leaves,
                                                const int32_t *__restrict__ first, const int32_t *__restrict__ size,
                                                const double *__restrict__ V, const double *__restrict__ Xt,
                                                int64_t ldxt, const int32_t *__restrict__ parent,
                                                const int32_t *__restrict__ son0, const int32_t *__restrict__ son1,
                                                const int32_t *__restrict__ depth, int min_depth,
                                                const double *__restrict__ E, double *__restrict__ xh, int64_t ldh,
                                                int32_t *__restrict__ cnt, Skip skip) {
    __shared__ Smem<NJ> sm;
    __shared__ int order;
    const int32_t per_xcd = (L + 7) / 8;
    const int32_t l = (blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
    if (l >= L) return;
    const int32_t t = leaves[l];
    if (skip(t)) return;
    const int64_t j0 = (int64_t)blockIdx.y * Smem<NJ>::MC;
    const int mc = (int)min<int64_t>(Smem<NJ>::MC, m - j0);
    const int64_t r0 = first[t];
    const int nt = size[t];
    clear<NJ>(sm);
    dbl4 acc[NJ];
    zero<NJ>(acc);
    accumulate<NJ>(sm, acc, (nt + 63) / 64, mc, k, [&](int q) {
        const int i0 = 64 * q;
        return Term{V + (r0 + i0) * k, k, min(64, nt - i0), k, true, Xt + j0, ldxt, nullptr, r0 + i0};
    });
    auto write = [&](int32_t c) {
#pragma unroll
        for (int J = 0; J < NJ; ++J)
            if (out_col(J) < mc)
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    if (out_row(r) < k) xh[((int64_t)c * k + out_row(r)) * ldh + j0 + out_col(J)] = acc[J][r];
    };
    write(t);
    for (int32_t c = t;;) {
        const int32_t p = parent[c];
        if (p < 0 || depth[p] < min_depth) break;
        __threadfence();  // publish x_c before counting it
        __syncthreads();
        if (threadIdx.x == 0) order = atomicAdd(&cnt[(int64_t)p * gridDim.y + blockIdx.y], 1);
        __syncthreads();
        if (order == 0) break;  // the sibling is not done yet; its work-group continues
        __threadfence();        // see the sibling's x before reading it
        zero<NJ>(acc);
        const int32_t s0 = son0[p], s1 = son1[p];
        accumulate<NJ>(sm, acc, 2, mc, k, [&](int q) {
            const int32_t sn = q ? s1 : s0;
            return Term{E + (int64_t)sn * k * k, k, k, k, true, xh + j0, ldh, nullptr, (int64_t)sn * k};
        });
        write(p);
        c = p;
    }
}

static __global__ void k_zero_i32(int64_t count, int32_t *__restrict__ p) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < count) p[e] = 0;
}

// y_c += E_c y_parent(c) for the clusters in `list`; par[i] is the parent of list[i]
template <int NJ>
__global__ __launch_bounds__(256) void k_down(int k, int64_t m, const int32_t *__restrict__ list,
                                              const int32_t *__restrict__ par, const double *__restrict__ E,
                                              double *__restrict__ yh, int64_t ldh, Skip skip) {
    __shared__ Smem<NJ> sm;
    const int32_t c = list[blockIdx.x], p = par[blockIdx.x];
    if (skip(c)) return;
    const int64_t j0 = (int64_t)blockIdx.y * Smem<NJ>::MC;
    const int mc = (int)min<int64_t>(Smem<NJ>::MC, m - j0);
    const Term d{E + (int64_t)c * k * k, k, k, k, false, yh + j0, ldh, nullptr, (int64_t)p * k};
    Regs<NJ> R;
    load_term<NJ>(d, mc, R);
    if (k < K) clear<NJ>(sm);  // padding rows and columns of the k x k tile
    dbl4 acc[NJ];
    zero<NJ>(acc);
    store_term<NJ>(d, mc, R, sm);
    __syncthreads();
    mma<NJ>(sm.a, sm.b, dkpad4(k), k, acc);
#pragma unroll
    for (int J = 0; J < NJ; ++J)
        if (out_col(J) < mc)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                if (out_row(r) < k) yh[((int64_t)c * k + out_row(r)) * ldh + j0 + out_col(J)] += acc[J][r];
}

// Transfer passes for rank k = 64 with the transfer matrices straight from memory as the
// matrix-core left operand: wave w holds rows 16w..16w+15 of E_s^T (upward) or E_s
// (downward) in registers, 16 k-steps of one 8-byte load per lane (upward: 16 lanes over
// 16 consecutive entries of a row of E_s; downward: 16 rows of E_s, their 128-byte lines
// shared by four k-steps through the L1), so that only the right operand (x-hat or y-hat
// rows, 64 x 16*NJ) goes through LDS, both upward terms at once behind one barrier.  The
// k-steps and terms are summed in the order of k_up / k_down.
//   upward:   x_t = E_{s0}^T x_{s0} + E_{s1}^T x_{s1}   (list, son as for k_up)
//   downward: y_c += E_c y_{par(c)}                    (list, par as for k_down)
// by: the column slab; bs: NT x 64 x (16 NJ + 1) doubles of LDS
template <int NJ, int NT, int TR>
__device__ inline void transfer_rows(const double *const *Ea, const int64_t *brow, int64_t m,
                                     const double *__restrict__ hat_in, int64_t ldh, dbl4 *acc, int by, double *bs) {
    constexpr int MC = 16 * NJ, LDB = MC + 1, XPT = 64 * MC / 256;
    const int tid = threadIdx.x, lane = tid & 63, lr = lane & 15, lq = lane >> 4;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int64_t j0 = (int64_t)by * MC;
    const int mc = (int)min<int64_t>(MC, m - j0);
    double a[NT][16], bv[NT][XPT];
#pragma unroll
    for (int q = 0; q < NT; ++q) {
#pragma unroll
        for (int kk = 0; kk < 16; ++kk)
            a[q][kk] = TR ? Ea[q][(4 * kk + lq) * 64 + 16 * w + lr] : Ea[q][(16 * w + lr) * 64 + 4 * kk + lq];
#pragma unroll
        for (int u = 0; u < XPT; ++u) {
            const int e = tid + 256 * u, r = e / MC, c = e % MC;
            bv[q][u] = hat_in[(brow[q] + r) * ldh + j0 + min(c, mc - 1)];  // columns past mc: zeroed when stored
        }
    }
#pragma unroll
    for (int q = 0; q < NT; ++q)
#pragma unroll
        for (int u = 0; u < XPT; ++u) {
            const int e = tid + 256 * u, r = e / MC, c = e % MC;
            bs[q * 64 * LDB + r * LDB + c] = c < mc ? bv[q][u] : 0.0;
        }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NT; ++q)
#pragma unroll
        for (int kk = 0; kk < 16; ++kk)
#pragma unroll
            for (int J = 0; J < NJ; ++J)
                acc[J] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[q][kk], bs[q * 64 * LDB + (4 * kk + lq) * LDB + 16 * J + lr],
                                                              acc[J], 0, 0, 0);
}

// one upward item: x_t = E_{s0}^T x_{s0} + E_{s1}^T x_{s1} for list entry i, column slab by
template <int NJ>
__device__ inline void up64_item(int i, int by, int64_t m, const int32_t *__restrict__ list,
                                 const int32_t *__restrict__ son, const double *__restrict__ E, double *__restrict__ xh,
                                 int64_t ldh, Skip skip, double *bs) {
    const int32_t t = list[i], s0 = son[2 * i], s1 = son[2 * i + 1];
    if (skip(t)) return;
    const double *Ea[2] = {E + (int64_t)s0 * 4096, E + (int64_t)s1 * 4096};
    const int64_t brow[2] = {(int64_t)s0 * 64, (int64_t)s1 * 64};
    dbl4 acc[NJ];
    zero<NJ>(acc);
    transfer_rows<NJ, 2, 1>(Ea, brow, m, xh, ldh, acc, by, bs);
    const int64_t j0 = (int64_t)by * 16 * NJ;
    const int mc = (int)min<int64_t>(16 * NJ, m - j0);
#pragma unroll
    for (int J = 0; J < NJ; ++J)
        if (out_col(J) < mc)
#pragma unroll
            for (int r = 0; r < 4; ++r) xh[((int64_t)t * 64 + out_row(r)) * ldh + j0 + out_col(J)] = acc[J][r];
}

// one downward item: y_c += E_c y_par for list entry i, column slab by
template <int NJ>
__device__ inline void down64_item(int i, int by, int64_t m, const int32_t *__restrict__ list,
                                   const int32_t *__restrict__ par, const double *__restrict__ E,
                                   double *__restrict__ yh, int64_t ldh, Skip skip, double *bs) {
    const int32_t c = list[i], p = par[i];
    if (skip(c)) return;
    const double *Ea[1] = {E + (int64_t)c * 4096};
    const int64_t brow[1] = {(int64_t)p * 64};
    dbl4 acc[NJ];
    zero<NJ>(acc);
    transfer_rows<NJ, 1, 0>(Ea, brow, m, yh, ldh, acc, by, bs);
    const int64_t j0 = (int64_t)by * 16 * NJ;
    const int mc = (int)min<int64_t>(16 * NJ, m - j0);
#pragma unroll
    for (int J = 0; J < NJ; ++J)
        if (out_col(J) < mc)
#pragma unroll
            for (int r = 0; r < 4; ++r) yh[((int64_t)c * 64 + out_row(r)) * ldh + j0 + out_col(J)] += acc[J][r];
}

template <int NJ>
__global__ __launch_bounds__(256) void k_up64(int64_t m, const int32_t *__restrict__ list,
                                              const int32_t *__restrict__ son, const double *__restrict__ E,
                                              double *__restrict__ xh, int64_t ldh, Skip skip) {
    __shared__ double bs[2 * 64 * (16 * NJ + 1)];
    up64_item<NJ>(blockIdx.x, blockIdx.y, m, list, son, E, xh, ldh, skip, bs);
}

template <int NJ>
__global__ __launch_bounds__(256) void k_down64(int64_t m, const int32_t *__restrict__ list,
                                                const int32_t *__restrict__ par, const double *__restrict__ E,
                                                double *__restrict__ yh, int64_t ldh, Skip skip) {
    __shared__ double bs[64 * (16 * NJ + 1)];
    down64_item<NJ>(blockIdx.x, blockIdx.y, m, list, par, E, yh, ldh, skip, bs);
}

// Forward leaf transform for rank 64, x_t = V_t^T X|_t, with V_t^T straight into the
// matrix-core registers (wave w: rows 16w..16w+15 of x_t, 16 lanes over 16 consecutive
// entries of a row of V) and the rows of X|_t (tree order) through LDS, in chunks of 64
// points; rows past the leaf are zero in LDS.  Summed in the order of k_fwd_leaf.
template <int NJ>
__global__ __launch_bounds__(256) void k_fwd_leaf64(int64_t m, const int32_t *__restrict__ leaves,
                                                    const int32_t *__restrict__ first, const int32_t *__restrict__ size,
                                                    const double *__restrict__ V, const double *__restrict__ Xt,
                                                    int64_t ldxt, double *__restrict__ xh, int64_t ldh, Skip skip) {
    constexpr int MC = 16 * NJ, LDB = MC + 1, XPT = 64 * MC / 256;
    __shared__ double bs[64 * LDB];
    const int32_t t = leaves[blockIdx.x];
    if (skip(t)) return;
    const int tid = threadIdx.x, lane = tid & 63, lr = lane & 15, lq = lane >> 4;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int64_t j0 = (int64_t)blockIdx.y * MC;
    const int mc = (int)min<int64_t>(MC, m - j0);
    const int64_t r0 = first[t];
    const int nt = size[t];
    dbl4 acc[NJ];
    zero<NJ>(acc);
    for (int i0 = 0; i0 < nt; i0 += 64) {
        const int ic = min(64, nt - i0);
        double a[16], bv[XPT];
#pragma unroll
        for (int kk = 0; kk < 16; ++kk) a[kk] = V[(r0 + i0 + min(4 * kk + lq, ic - 1)) * 64 + 16 * w + lr];
#pragma unroll
        for (int u = 0; u < XPT; ++u) {
            const int e = tid + 256 * u, r = e / MC, c = e % MC;
            bv[u] = Xt[(r0 + i0 + min(r, ic - 1)) * ldxt + j0 + min(c, mc - 1)];
        }
        if (i0 > 0) __syncthreads();  // the previous chunk's products have read bs
#pragma unroll
        for (int u = 0; u < XPT; ++u) {
            const int e = tid + 256 * u, r = e / MC, c = e % MC;
            bs[r * LDB + c] = (r < ic && c < mc) ? bv[u] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < 16; ++kk)
#pragma unroll
            for (int J = 0; J < NJ; ++J)
                acc[J] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[kk], bs[(4 * kk + lq) * LDB + 16 * J + lr], acc[J], 0,
                                                              0, 0);
    }
#pragma unroll
    for (int J = 0; J < NJ; ++J)
        if (out_col(J) < mc)
#pragma unroll
            for (int r = 0; r < 4; ++r) xh[((int64_t)t * 64 + out_row(r)) * ldh + j0 + out_col(J)] = acc[J][r];
}

// Forward leaf transform for ranks up to 32 in the form of k_fwd_leaf64: two waves (rows
// 16w..16w+15 of x_t; rows past k are zero in the operand and never written) load V_t^T
// straight into the matrix-core registers and the rows of X|_t (tree order) go through LDS
// in chunks of 64 points.
template <int NJ>
__global__ __launch_bounds__(128) void k_fwd_leaf_small(int k, int64_t m, const int32_t *__restrict__ leaves,
                                                        const int32_t *__restrict__ first,
                                                        const int32_t *__restrict__ size, const double *__restrict__ V,
                                                        const double *__restrict__ Xt, int64_t ldxt,
                                                        double *__restrict__ xh, int64_t ldh, Skip skip) {
    constexpr int MC = 16 * NJ, LDB = MC + 1, XPT = 64 * MC / 128;
    __shared__ double bs[64 * LDB];
    const int32_t t = leaves[blockIdx.x];
    if (skip(t)) return;
    const int tid = threadIdx.x, lane = tid & 63, lr = lane & 15, lq = lane >> 4;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int64_t j0 = (int64_t)blockIdx.y * MC;
    const int mc = (int)min<int64_t>(MC, m - j0);
    const int64_t r0 = first[t];
    const int nt = size[t];
    const int nu = 16 * w + lr;  // row of x_t (column of V) this lane supplies
    const bool nu_ok = nu < k;
    dbl4 acc[NJ];
    zero<NJ>(acc);
    for (int i0 = 0; i0 < nt; i0 += 64) {
        const int ic = min(64, nt - i0);
        double a[16], bv[XPT];
#pragma unroll
        for (int kk = 0; kk < 16; ++kk) a[kk] = V[(r0 + i0 + min(4 * kk + lq, ic - 1)) * k + (nu_ok ? nu : 0)];
#pragma unroll
        for (int u = 0; u < XPT; ++u) {
            const int e = tid + 128 * u, r = e / MC, c = e % MC;
            bv[u] = Xt[(r0 + i0 + min(r, ic - 1)) * ldxt + j0 + min(c, mc - 1)];
        }
        if (i0 > 0) __syncthreads();  // the previous chunk's products have read bs
#pragma unroll
        for (int u = 0; u < XPT; ++u) {
            const int e = tid + 128 * u, r = e / MC, c = e % MC;
            bs[r * LDB + c] = (r < ic && c < mc) ? bv[u] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < 16; ++kk)
#pragma unroll
            for (int J = 0; J < NJ; ++J)
                acc[J] = __builtin_amdgcn_mfma_f64_16x16x4f64(nu_ok ? a[kk] : 0.0,
                                                              bs[(4 * kk + lq) * LDB + 16 * J + lr], acc[J], 0, 0, 0);
    }
#pragma unroll
    for (int J = 0; J < NJ; ++J)
        if (out_col(J) < mc)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                if (out_row(r) < k) xh[((int64_t)t * k + out_row(r)) * ldh + j0 + out_col(J)] = acc[J][r];
}

// Leaf stage in the transposed orientation Y_t^T = X_s^T N_ts^T: the
// matrix-core M dimension runs over columns of X, N over rows of the leaf.
// Near-field blocks are stored transposed (|s| rows of length |t| padded to
// even), and the leaf basis also has a transposed copy (k rows of length |t|
// padded to even).  Every operand load is then 16 bytes per lane: a lane
// holds two neighbouring rows (or columns), so one load feeds the "even" and
// the "odd" 16-row (16-column) tile.  Tile (J = 2p + hj, I = 2g + h) holds
// columns 32p + 2m' + hj and rows 32g + 2n' + h, m', n' = 0..15.
// The 4 waves of a work-group split the leaf's terms (the basis term V_t y_t
// and the near blocks, dealt round-robin) and each computes all 64 rows x
// 32*NP columns of its partial sum, in rounds of four k-steps with the next
// round's loads in flight during the current round's MFMAs.  The four partial
// tiles are then added in LDS in wave order (fixed, so the result is
// reproducible).  Leaves are dealt to XCDs in contiguous eighths so that
// neighbouring leaves, which share near-field partners, read the same rows of
// X through one L2.
//   Y|_t = beta Y|_t + alpha (basis ? V_t y_t : 0) + alpha (near ? sum_s N_ts X|_s : 0)
typedef double dbl2 __attribute__((ext_vector_type(2)));

template <int NP>
struct Round {
    dbl2 b[2][4];   // [row half g][k-step u]: rows 32g + 2 lr + {0, 1}
    dbl2 a[NP][4];  // [column half p][k-step u]: columns 32p + 2 lr + {0, 1}
    int kb, kl;     // first k-step of the round and the item's length
    int jx;         // apply J to the left operand (imaginary plane of a complex near block)
};

__device__ inline dbl2 ld2(const double *p) { return *(const dbl2 *)p; }

template <int NP>
__global__ __launch_bounds__(256, NP == 1 ? 2 : 1) void k_leaf_direct(int k, int64_t m, int32_t L, const int32_t *__restrict__ leaves,
                                                     const int32_t *__restrict__ first,
                                                     const int32_t *__restrict__ size,
                                                     const int64_t *__restrict__ perm, const double *__restrict__ Vt,
                                                     const int64_t *__restrict__ vt_off,
                                                     const double *__restrict__ yh, int64_t ldh,
                                                     const int64_t *__restrict__ near_ptr,
                                                     const int32_t *__restrict__ near_col,
                                                     const int64_t *__restrict__ near_off,
                                                     const double *__restrict__ Nt, const double *__restrict__ Xt,
                                                     int64_t ldxt, double alpha, double beta, double *__restrict__ Y,
                                                     int64_t ldy, int tree_order, int basis, int near, Skip skip,
                                                     int64_t n_plane) {
    constexpr int MC = 32 * NP, LDR = MC + 1;
    __shared__ double red[64 * LDR];
    const int32_t per_xcd = (L + 7) / 8;
    const int nslab = (int)((m + MC - 1) / MC);
    // one (leaf, column slab) per work-group, or (a capped grid) a grid-stride loop over
    // them; a slot keeps its XCD because the grid is a multiple of 8, and the slabs of one
    // leaf are consecutive slots of one XCD, so its near blocks come from HBM once
    for (int64_t slot = blockIdx.x; slot < (int64_t)8 * per_xcd * nslab; slot += gridDim.x) {
        const int64_t qx = slot >> 3;
        const int32_t l = (int32_t)((slot & 7) * per_xcd + qx / nslab);
        if (l >= L) continue;
        const int32_t t = leaves[l];
        if (skip(t)) continue;
        const int nt = size[t];
        const int64_t nt2 = pad_rows(nt);
        const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63, lr = lane & 15,
                  lq = lane >> 4;  // w is wave-uniform: item loops stay scalar
        const int64_t r0 = first[t];
        const int64_t j0 = (qx % nslab) * MC;
        const int mc = (int)min<int64_t>(MC, m - j0);
        const int64_t q0 = near_ptr[l], vt0 = basis ? vt_off[l] : 0;
        // items: nb parts of the basis term (k-ranges of ceil(k / nb)), then the near
        // blocks; without near blocks the basis term is split over the 4 waves
        const int nb = basis ? (near ? 1 : 4) : 0;
        const int kbase = (k + max(nb, 1) - 1) / max(nb, 1);
        const int nnear = near ? (int)(near_ptr[l + 1] - q0) : 0;
        // complex operator (n_plane > 0): every near block is two items, its real plane on X
        // and its imaginary plane on J X (column pairs (re, im) -> (-im, re))
        const int cpx = n_plane > 0 ? 1 : 0;
        const int nitems = (nnear << cpx) + nb;
        // the near blocks' offsets, column ranges and sizes, staged once so that moving
        // to the next item costs no dependent global loads (beyond kMeta: read directly)
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
            const int nhalf = (ic + 31) >> 5;  // 32-row halves present (wave-uniform)
            dbl4 acc[2 * NP][4];
    #pragma unroll
            for (int J = 0; J < 2 * NP; ++J)
    #pragma unroll
                for (int I = 0; I < 4; ++I) acc[J][I] = dbl4{0.0, 0.0, 0.0, 0.0};

            // item e, k-steps kb..kb+15 -> registers.  Right operand: rows (k) of a
            // transposed block with row stride nt2; left operand: rows (k) of X or y_t.
            // Every load is issued unconditionally from a clamped address (rows past the
            // tile, columns past the slab and k past the item read in-range neighbours), so
            // the compiler's wait counters stay exact and the MFMAs of a round never wait
            // for the next round's loads; the left operand's k-rows past the item are
            // zeroed where they are used.  Rows and columns past the tile are never stored.
            const int xr = (ic - 1) & ~1, xc = (mc - 1) & ~1;  // last even row / column offset
            auto load = [&](int e, int kb, Round<NP> &R) {
                const double *bb, *ab;
                int64_t lda;
                int kl;
                if (e < nb) {
                    bb = Vt + vt0 + (int64_t)e * kbase * nt2 + i0;   // V_t^T[nu][i]
                    ab = yh + ((int64_t)t * k + e * kbase) * ldh + j0; // y_t[nu][j]
                    lda = ldh;
                    kl = min(kbase, k - e * kbase);
                } else {
                    int64_t off, fs;
                    const int q = (e - nb) >> cpx, plane = (e - nb) & cpx;
                    near_meta(q, off, fs, kl);
                    bb = Nt + off + (plane ? n_plane : 0) + i0;  // N_ts^T[c][i]
                    ab = Xt + fs * ldxt + j0;                     // X_s[c][j]
                    lda = ldxt;
                    R.jx = plane;
                }
                if (e < nb) R.jx = 0;
                R.kb = kb;
                R.kl = kl;
    #pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int c = min(kb + 4 * u + lq, kl - 1);
    #pragma unroll
                    for (int g = 0; g < 2; ++g) R.b[g][u] = ld2(bb + c * nt2 + min(32 * g + 2 * lr, xr));
    #pragma unroll
                    for (int p = 0; p < NP; ++p) R.a[p][u] = ld2(ab + c * lda + min(32 * p + 2 * lr, xc));
                }
            };
            auto klen = [&](int e) {
                if (e < nb) return min(kbase, k - e * kbase);
                int64_t off, fs;
                int ks;
                near_meta((e - nb) >> cpx, off, fs, ks);
                return ks;
            };
            // zero the left operand's k-rows past the item, and apply J for an imaginary
            // plane (once the round's loads are in)
            auto mask = [&](Round<NP> &R) {
    #pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const bool cok = R.kb + 4 * u + lq < R.kl;
    #pragma unroll
                    for (int p = 0; p < NP; ++p) {
                        dbl2 v = cok ? R.a[p][u] : dbl2{0.0, 0.0};
                        if (R.jx) v = dbl2{-v.y, v.x};
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
                                        acc[2 * p + hj][2 * g + h] = __builtin_amdgcn_mfma_f64_16x16x4f64(
                                            R.a[p][u][hj], R.b[g][u][h], acc[2 * p + hj][2 * g + h], 0, 0, 0);
            };

            int e = w;
            if (e < nitems) {
                Round<NP> cur, nxt;
                int kb = 0, len = klen(e);
                load(e, kb, cur);
                mask(cur);
                // the last round is peeled off, so that every round of the loop loads the next
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
            // partial tiles of the 4 waves, added in wave order.  Lane l, register r of
            // tile (J = 2p + hj, I = 2g + h) -> column 32p + 2 (l / 16 + 4 r) + hj,
            // row 32g + 2 (l % 16) + h.
            for (int ww = 0; ww < 4; ++ww) {
                if (w == ww)
    #pragma unroll
                    for (int J = 0; J < 2 * NP; ++J)
    #pragma unroll
                        for (int I = 0; I < 4; ++I)
    #pragma unroll
                            for (int r = 0; r < 4; ++r) {
                                const int col = 32 * (J >> 1) + 2 * (lq + 4 * r) + (J & 1);
                                const int row = 32 * (I >> 1) + 2 * lr + (I & 1);
                                double *cell = &red[row * LDR + col];
                                *cell = (ww == 0) ? acc[J][I][r] : *cell + acc[J][I][r];
                            }
                __syncthreads();
            }
            for (int x = threadIdx.x; x < ic * MC; x += 256) {
                const int i = x / MC, j = x % MC;
                if (j < mc) {
                    int64_t row = r0 + i0 + i;
                    if (!tree_order) row = perm[row];
                    double *y = &Y[row * ldy + j0 + j];
                    const double v = alpha * red[i * LDR + j];
                    *y = (beta == 0.0) ? v : beta * *y + v;
                }
            }
            __syncthreads();
        }
    }
}

// rows of X into tree order with an even leading dimension: Xt[i] = X[perm[i]] (zero padding).
// One thread per pair of columns, written with one 16-byte store (Xt 16-byte aligned, ldt
// even); launch over n * ldt / 2 threads.
static __global__ void k_gather(int64_t n, int64_t m, const int64_t *__restrict__ perm, const double *__restrict__ X,
                         int64_t ldx, double *__restrict__ Xt, int64_t ldt) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x, half = ldt >> 1;
    if (e >= n * half) return;
    const int64_t i = e / half, j = 2 * (e - i * half);
    const double *src = X + (perm ? perm[i] : i) * ldx;
    const dbl2 v = {j < m ? src[j] : 0.0, j + 1 < m ? src[j + 1] : 0.0};
    *(dbl2 *)(Xt + i * ldt + j) = v;
}

}  // namespace mfma
}  // namespace h2x
