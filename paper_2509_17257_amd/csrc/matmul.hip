// H^2 x X (Algorithm "H2_mvm" in its matrix form, section 4):
//   forward transformation  x_s = V_s^T X|_s at leaves, x_t = sum_{t'} E_{t'}^T x_{t'} upwards
//   multiplication phase    y_t = sum_{(t,s) in C_t, admissible} S_b x_s   for every cluster t
//   backward transformation y_{t'} += E_{t'} y_t downwards,
//                            Y|_t = beta Y|_t + alpha (V_t y_t + sum_{(t,s) near} N_b X|_s) at leaves
// Ownership follows the paper's race-free rules: a parent sums its sons (no two
// writers of x_t), each row cluster owns its list and its rows of Y (no two
// writers of y_t or Y|_t).  No floating-point atomics: results are
// bitwise reproducible run to run.
//
// Every stage is a batch of small GEMMs.  This file holds the generic kernels
// (any rank k, any leaf size, any m): 256 threads stage 64 x 64 operand tiles
// and 64 x 32 column tiles in LDS, each thread accumulates 8 outputs.
#include <functional>
#include <type_traits>

#include "device.hpp"
#include "coupling_lp.hpp"
#include "leaf_cat.hpp"
#include "leaf_cat_lp.hpp"
#include "leaf_lp.hpp"
#include "leaf_rows.hpp"
#include "matmul_mfma.hpp"
#include "stages_mfma.hpp"
#include "transfer_kron.hpp"
#include "transfer_lp.hpp"
#include "types.hpp"

namespace h2x {

namespace {

constexpr int TR = 64;  // output rows / contraction chunk per tile
constexpr int TC = 32;  // columns of X per work-group (grid.y)

// out[i] = x[i] rounded to BF16 (nearest even), as raw bits, four entries per thread
// (cnt4 = count / 4; both buffers 16-byte aligned)
__global__ void k_pack_bf16(int64_t cnt4, const float4 *__restrict__ x, uint2 *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < cnt4) {
        const float4 v = x[i];
        out[i] = uint2{(uint32_t)bf16_bits(v.x) | ((uint32_t)bf16_bits(v.y) << 16),
                       (uint32_t)bf16_bits(v.z) | ((uint32_t)bf16_bits(v.w) << 16)};
    }
}
// transfer levels of the FP64 operators with p = 3 and 4 through the Kronecker factors of E
// (kron::) instead of the dense transfer matrices on the matrix cores (mfma::k_up64 / k_down64,
// mfma::k_up / k_down)
constexpr bool kKronTransfer = true;
// levels with fewer work-groups than this (clusters x column slabs) take 16-column slabs:
// more work-groups with half the work each shorten a level that is one wave of work-groups
constexpr int64_t kNarrowLevel = 256;
// forward leaf transform for k <= 32 with V_t^T straight into the matrix-core registers
constexpr bool kSmallFwdLeaf = true;

template <typename T, typename Acc>
__device__ inline Acc ld_op(const T *p) { return (Acc)to_double(*p); }

// operand rounding of a right-hand factor to the storage precision T
template <typename T, typename Acc>
__device__ inline Acc round_op(double v) { return (Acc)to_double(from_double<T>(v)); }

template <typename Acc>
__device__ inline void tile_fma(Acc acc[8], const Acc (*As)[TR + 1], const Acc (*Bs)[TC], int kc, int rg, int j) {
    for (int c = 0; c < kc; ++c) {
        const Acc b = Bs[c][j];
#pragma unroll
        for (int q = 0; q < 8; ++q) acc[q] += As[rg + 8 * q][c] * b;
    }
}

// x_t = V_t^T X|_t for each leaf t
template <typename T, typename Acc>
__global__ __launch_bounds__(256) void k_fwd_leaf(int k, int64_t m, const int32_t *__restrict__ leaves,
                                                  const int32_t *__restrict__ first, const int32_t *__restrict__ size,
                                                  const int64_t *__restrict__ perm, const T *__restrict__ V,
                                                  const double *__restrict__ X, int64_t ldx, int tree_order,
                                                  Acc *__restrict__ xh, int64_t ldh) {
    __shared__ Acc As[TR][TR + 1];
    __shared__ Acc Bs[TR][TC];
    const int32_t t = leaves[blockIdx.x];
    const int64_t j0 = (int64_t)blockIdx.y * TC;
    const int mc = (int)min<int64_t>(TC, m - j0);
    const int tid = threadIdx.x, rg = tid >> 5, j = tid & 31;
    const int64_t r0 = first[t];
    const int nt = size[t];
    for (int n0 = 0; n0 < k; n0 += TR) {
        Acc acc[8] = {};
        for (int i0 = 0; i0 < nt; i0 += TR) {
            const int ic = min(TR, nt - i0);
            for (int e = tid; e < TR * TR; e += 256) {
                const int i = e / TR, nu = e % TR;
                As[nu][i] = (i < ic && n0 + nu < k) ? ld_op<T, Acc>(&V[(r0 + i0 + i) * k + n0 + nu]) : Acc(0);
            }
            for (int e = tid; e < TR * TC; e += 256) {
                const int i = e / TC, jj = e % TC;
                Acc v = 0;
                if (i < ic && jj < mc) {
                    int64_t row = r0 + i0 + i;
                    if (!tree_order) row = perm[row];
                    v = round_op<T, Acc>(X[row * ldx + j0 + jj]);
                }
                Bs[i][jj] = v;
            }
            __syncthreads();
            tile_fma(acc, As, Bs, ic, rg, j);
            __syncthreads();
        }
        if (j < mc)
            for (int q = 0; q < 8; ++q) {
                const int nu = n0 + rg + 8 * q;
                if (nu < k) xh[((int64_t)t * k + nu) * ldh + j0 + j] = acc[q];
            }
    }
}

// x_t = E_{t0}^T x_{t0} + E_{t1}^T x_{t1} for the inner clusters of one depth
template <typename T, typename Acc>
__global__ __launch_bounds__(256) void k_up(int k, int64_t m, const int32_t *__restrict__ list,
                                            const int32_t *__restrict__ son0, const int32_t *__restrict__ son1,
                                            const T *__restrict__ E, Acc *__restrict__ xh, int64_t ldh) {
    __shared__ Acc As[TR][TR + 1];
    __shared__ Acc Bs[TR][TC];
    const int32_t t = list[blockIdx.x];
    const int64_t j0 = (int64_t)blockIdx.y * TC;
    const int mc = (int)min<int64_t>(TC, m - j0);
    const int tid = threadIdx.x, rg = tid >> 5, j = tid & 31;
    const int32_t sons[2] = {son0[t], son1[t]};
    for (int n0 = 0; n0 < k; n0 += TR) {
        Acc acc[8] = {};
        for (int q2 = 0; q2 < 2; ++q2) {
            const int32_t s = sons[q2];
            const T *Es = E + (int64_t)s * k * k;
            for (int a0 = 0; a0 < k; a0 += TR) {
                const int ac = min(TR, k - a0);
                for (int e = tid; e < TR * TR; e += 256) {
                    const int a = e / TR, nu = e % TR;
                    As[nu][a] = (a < ac && n0 + nu < k) ? ld_op<T, Acc>(&Es[(int64_t)(a0 + a) * k + n0 + nu]) : Acc(0);
                }
                for (int e = tid; e < TR * TC; e += 256) {
                    const int a = e / TC, jj = e % TC;
                    Bs[a][jj] = (a < ac && jj < mc)
                                    ? round_op<T, Acc>((double)xh[((int64_t)s * k + a0 + a) * ldh + j0 + jj])
                                    : Acc(0);
                }
                __syncthreads();
                tile_fma(acc, As, Bs, ac, rg, j);
                __syncthreads();
            }
        }
        if (j < mc)
            for (int q = 0; q < 8; ++q) {
                const int nu = n0 + rg + 8 * q;
                if (nu < k) xh[((int64_t)t * k + nu) * ldh + j0 + j] = acc[q];
            }
    }
}

// y_t = sum over the admissible blocks of row cluster t of S_b x_s (every cluster)
template <typename T, typename Acc>
__global__ __launch_bounds__(256) void k_coupling(int k, int64_t m, const int64_t *__restrict__ adm_ptr,
                                                  const int32_t *__restrict__ adm_col, const T *__restrict__ S,
                                                  int swz, const Acc *__restrict__ xh, Acc *__restrict__ yh,
                                                  int64_t ldh) {
    __shared__ Acc As[TR][TR + 1];
    __shared__ Acc Bs[TR][TC];
    const int32_t t = blockIdx.x;
    const int64_t j0 = (int64_t)blockIdx.y * TC;
    const int mc = (int)min<int64_t>(TC, m - j0);
    const int tid = threadIdx.x, rg = tid >> 5, j = tid & 31;
    const int64_t b0 = adm_ptr[t], b1 = adm_ptr[t + 1];
    for (int n0 = 0; n0 < k; n0 += TR) {
        Acc acc[8] = {};
        for (int64_t b = b0; b < b1; ++b) {
            const int32_t s = adm_col[b];
            const T *Sb = S + b * k * k;
            for (int u0 = 0; u0 < k; u0 += TR) {
                const int uc = min(TR, k - u0);
                for (int e = tid; e < TR * TR; e += 256) {
                    const int nu = e / TR, mu = e % TR;
                    As[nu][mu] = (mu < uc && n0 + nu < k) ? ld_op<T, Acc>(&Sb[s_index(swz, k, n0 + nu, u0 + mu)]) : Acc(0);
                }
                for (int e = tid; e < TR * TC; e += 256) {
                    const int mu = e / TC, jj = e % TC;
                    Bs[mu][jj] = (mu < uc && jj < mc)
                                     ? round_op<T, Acc>((double)xh[((int64_t)s * k + u0 + mu) * ldh + j0 + jj])
                                     : Acc(0);
                }
                __syncthreads();
                tile_fma(acc, As, Bs, uc, rg, j);
                __syncthreads();
            }
        }
        if (j < mc)
            for (int q = 0; q < 8; ++q) {
                const int nu = n0 + rg + 8 * q;
                if (nu < k) yh[((int64_t)t * k + nu) * ldh + j0 + j] = acc[q];
            }
    }
}

// y_c += E_c y_parent(c) for the clusters of one depth >= 1
template <typename T, typename Acc>
__global__ __launch_bounds__(256) void k_down(int k, int64_t m, const int32_t *__restrict__ list,
                                              const int32_t *__restrict__ parent, const T *__restrict__ E,
                                              Acc *__restrict__ yh, int64_t ldh) {
    __shared__ Acc As[TR][TR + 1];
    __shared__ Acc Bs[TR][TC];
    const int32_t c = list[blockIdx.x];
    const int32_t par = parent[c];
    const int64_t j0 = (int64_t)blockIdx.y * TC;
    const int mc = (int)min<int64_t>(TC, m - j0);
    const int tid = threadIdx.x, rg = tid >> 5, j = tid & 31;
    const T *Ec = E + (int64_t)c * k * k;
    for (int a0 = 0; a0 < k; a0 += TR) {
        Acc acc[8] = {};
        for (int u0 = 0; u0 < k; u0 += TR) {
            const int uc = min(TR, k - u0);
            for (int e = tid; e < TR * TR; e += 256) {
                const int a = e / TR, nu = e % TR;
                As[a][nu] = (nu < uc && a0 + a < k) ? ld_op<T, Acc>(&Ec[(int64_t)(a0 + a) * k + u0 + nu]) : Acc(0);
            }
            for (int e = tid; e < TR * TC; e += 256) {
                const int nu = e / TC, jj = e % TC;
                Bs[nu][jj] = (nu < uc && jj < mc)
                                 ? round_op<T, Acc>((double)yh[((int64_t)par * k + u0 + nu) * ldh + j0 + jj])
                                 : Acc(0);
            }
            __syncthreads();
            tile_fma(acc, As, Bs, uc, rg, j);
            __syncthreads();
        }
        if (j < mc)
            for (int q = 0; q < 8; ++q) {
                const int a = a0 + rg + 8 * q;
                if (a < k) yh[((int64_t)c * k + a) * ldh + j0 + j] += acc[q];
            }
    }
}

// Y|_t = beta Y|_t + alpha (V_t y_t + sum_{near (t,s)} N_b X|_s) for each leaf t
template <typename T, typename TN, typename Acc>
__global__ __launch_bounds__(256) void k_leaf_near(int k, int64_t m, const int32_t *__restrict__ leaves,
                                                   const int32_t *__restrict__ first, const int32_t *__restrict__ size,
                                                   const int64_t *__restrict__ perm, const T *__restrict__ V,
                                                   const Acc *__restrict__ yh, int64_t ldh,
                                                   const int64_t *__restrict__ near_ptr,
                                                   const int32_t *__restrict__ near_col,
                                                   const int64_t *__restrict__ near_off, const TN *__restrict__ N,
                                                   const double *__restrict__ X, int64_t ldx, double alpha,
                                                   double beta, double *__restrict__ Y, int64_t ldy, int tree_order,
                                                   int near_t) {
    __shared__ Acc As[TR][TR + 1];
    __shared__ Acc Bs[TR][TC];
    const int32_t l = blockIdx.x;
    const int32_t t = leaves[l];
    const int64_t j0 = (int64_t)blockIdx.y * TC;
    const int mc = (int)min<int64_t>(TC, m - j0);
    const int tid = threadIdx.x, rg = tid >> 5, j = tid & 31;
    const int64_t r0 = first[t];
    const int nt = size[t];
    for (int i0 = 0; i0 < nt; i0 += TR) {
        const int ic = min(TR, nt - i0);
        Acc acc[8] = {};
        for (int u0 = 0; u0 < k; u0 += TR) {
            const int uc = min(TR, k - u0);
            for (int e = tid; e < TR * TR; e += 256) {
                const int i = e / TR, nu = e % TR;
                As[i][nu] = (i < ic && nu < uc) ? ld_op<T, Acc>(&V[(r0 + i0 + i) * k + u0 + nu]) : Acc(0);
            }
            for (int e = tid; e < TR * TC; e += 256) {
                const int nu = e / TC, jj = e % TC;
                Bs[nu][jj] = (nu < uc && jj < mc)
                                 ? round_op<T, Acc>((double)yh[((int64_t)t * k + u0 + nu) * ldh + j0 + jj])
                                 : Acc(0);
            }
            __syncthreads();
            tile_fma(acc, As, Bs, uc, rg, j);
            __syncthreads();
        }
        for (int64_t q = near_ptr[l]; q < near_ptr[l + 1]; ++q) {
            const int32_t s = near_col[q];
            const int ns = size[s];
            const int64_t fs = first[s];
            const TN *Nb = N + near_off[q];
            for (int c0 = 0; c0 < ns; c0 += TR) {
                const int cc = min(TR, ns - c0);
                for (int e = tid; e < TR * TR; e += 256) {
                    const int i = e / TR, c = e % TR;
                    const int64_t o = near_t ? (int64_t)(c0 + c) * pad_rows(nt) + i0 + i : (int64_t)(i0 + i) * ns + c0 + c;
                    As[i][c] = (i < ic && c < cc) ? ld_op<TN, Acc>(&Nb[o]) : Acc(0);
                }
                for (int e = tid; e < TR * TC; e += 256) {
                    const int c = e / TC, jj = e % TC;
                    Acc v = 0;
                    if (c < cc && jj < mc) {
                        int64_t row = fs + c0 + c;
                        if (!tree_order) row = perm[row];
                        v = round_op<TN, Acc>(X[row * ldx + j0 + jj]);
                    }
                    Bs[c][jj] = v;
                }
                __syncthreads();
                tile_fma(acc, As, Bs, cc, rg, j);
                __syncthreads();
            }
        }
        if (j < mc)
            for (int q = 0; q < 8; ++q) {
                const int i = rg + 8 * q;
                if (i < ic) {
                    int64_t row = r0 + i0 + i;
                    if (!tree_order) row = perm[row];
                    double *y = &Y[row * ldy + j0 + j];
                    const double v = alpha * (double)acc[q];
                    *y = (beta == 0.0) ? v : beta * *y + v;
                }
            }
    }
}

inline int64_t even_ld(int64_t m) { return m + (m & 1); }

// All five stages on the matrix cores (FP64 operator, k = 64 or k <= 32).
template <int NJ>
void matmul_mfma_f64(const DevMat &dm, const TuneCfg &cfg, int64_t m, double alpha, const double *X, int64_t ldx,
                     double beta, double *Y, int64_t ldy, int to, double *xh, double *yh, int64_t ldh, double *xt_ws,
                     hipStream_t st, const std::function<void(int)> &mark, hipEvent_t *ev, const int32_t *skip) {
    const Plan &P = *dm.plan;
    const unsigned gy = (unsigned)((m + 16 * NJ - 1) / (16 * NJ));
    // leaf stage: 32 or 64 columns per work-group
    const int NP = cfg.np_leaf ? cfg.np_leaf : (m > 32 ? 2 : 1);
    const double *V = (const double *)dm.V, *E = (const double *)dm.E;
    mark(0);
    // the leaf stage reads X in tree order, 16 bytes per lane: copy it unless it already is
    const double *Xt = X;
    int64_t ldxt = ldx;
    if (!to || (ldx & 1) || ((uintptr_t)X & 15)) {
        ldxt = even_ld(m);
        const int64_t cnt = dm.n * ldxt;
        hipLaunchKernelGGL(mfma::k_gather, dim3((unsigned)((cnt / 2 + 255) / 256)), dim3(256), 0, st, dm.n, m,
                           to ? nullptr : dm.perm, X, ldx, xt_ws, ldxt);
        Xt = xt_ws;
    }
    const Skip sk{skip, dm.sys_of};
    // rank 64: the basis and transfer matrices go straight into the matrix-core registers
    const bool t64 = dm.k == mfma::K;
    auto fwd_leaf = [&]() {
        if (t64)
            hipLaunchKernelGGL(mfma::k_fwd_leaf64<NJ>, dim3(dm.L, gy), dim3(256), 0, st, m, dm.leaves, dm.first,
                               dm.size, V, Xt, ldxt, xh, ldh, sk);
        else if (kSmallFwdLeaf)
            hipLaunchKernelGGL(mfma::k_fwd_leaf_small<NJ>, dim3(dm.L, gy), dim3(128), 0, st, dm.k, m, dm.leaves,
                               dm.first, dm.size, V, Xt, ldxt, xh, ldh, sk);
        else
            hipLaunchKernelGGL(mfma::k_fwd_leaf<NJ>, dim3(dm.L, gy), dim3(256), 0, st, dm.k, m, dm.leaves, dm.first,
                               dm.size, dm.perm, V, Xt, ldxt, 1, xh, ldh, sk);
    };
    const unsigned gl = (unsigned)((m + 32 * NP - 1) / (32 * NP));
    // leaf stage: one contraction per leaf (built-in where its LDS table of near rows fits),
    // a 64-row tile per wave and term, or the rows split over the waves
    const size_t cat_lds = sizeof(int32_t) * (size_t)std::max(1, dm.max_near_rows);
    // (it reads the rows of X through a buffer resource: 32-bit byte offsets)
    const bool cat_ok = !dm.cplx && cat_lds + sizeof(double) * 64 * (32 * NP + 1) + 64 <= 65536 &&
                        sizeof(double) * (size_t)dm.n * (size_t)ldxt < ((size_t)1 << 32);
    const int kind = cfg.leaf_kind == 0 ? (cat_ok ? 3 : 1) : (cfg.leaf_kind == 3 && !cat_ok ? 1 : cfg.leaf_kind);
    const bool rows = kind == 2;
    const int64_t cat_slots = (int64_t)8 * ((dm.L + 7) / 8) * gl;
    auto cat_args = [&](double b, int basis, int near) {
        return mfma::LeafCatArgs{dm.k, m, dm.L, dm.leaf_order, dm.leaves, dm.first, dm.size, dm.perm, (const double *)dm.Vt,
                                 dm.vt_off, yh, ldh, dm.near_ptr, dm.near_col, dm.near_off, (const double *)dm.N, Xt,
                                 ldxt, alpha, b, Y, ldy, to, basis, near, sk};
    };
    auto leaf = [&](hipStream_t s, double b, int basis, int near, unsigned cap) {
        if (kind == 3) {
            const unsigned gx = (unsigned)(cap ? std::min<int64_t>(cat_slots, cap) : cat_slots);
            if (NP == 2)
                hipLaunchKernelGGL(mfma::k_leaf_cat<2>, dim3(gx), dim3(256), cat_lds, s, cat_args(b, basis, near),
                                   (int64_t)0, cat_slots);
            else
                hipLaunchKernelGGL(mfma::k_leaf_cat<1>, dim3(gx), dim3(256), cat_lds, s, cat_args(b, basis, near),
                                   (int64_t)0, cat_slots);
            return;
        }
        if (rows) {
            const dim3 grid(8 * ((dm.L + 7) / 8) * gl, 2);
            if (NP == 2)
                hipLaunchKernelGGL(mfma::k_leaf_rows<2>, grid, dim3(64), 0, s, dm.k, m, dm.L, dm.leaves, dm.first,
                                   dm.size, dm.perm, (const double *)dm.Vt, dm.vt_off, yh, ldh, dm.near_ptr,
                                   dm.near_col, dm.near_off, (const double *)dm.N, Xt, ldxt, alpha, b, Y, ldy, to,
                                   basis, near, sk, dm.n_plane);
            else
                hipLaunchKernelGGL(mfma::k_leaf_rows<1>, grid, dim3(64), 0, s, dm.k, m, dm.L, dm.leaves, dm.first,
                                   dm.size, dm.perm, (const double *)dm.Vt, dm.vt_off, yh, ldh, dm.near_ptr,
                                   dm.near_col, dm.near_off, (const double *)dm.N, Xt, ldxt, alpha, b, Y, ldy, to,
                                   basis, near, sk, dm.n_plane);
            return;
        }
        unsigned gx = 8 * ((dm.L + 7) / 8) * gl;
        if (cap) gx = std::min(gx, cap);
        if (NP == 2)
            hipLaunchKernelGGL(mfma::k_leaf_direct<2>, dim3(gx), dim3(256), 0, s, dm.k, m,
                               dm.L, dm.leaves, dm.first, dm.size, dm.perm, (const double *)dm.Vt, dm.vt_off, yh, ldh,
                               dm.near_ptr, dm.near_col, dm.near_off, (const double *)dm.N, Xt, ldxt, alpha, b, Y,
                               ldy, to, basis, near, sk, dm.n_plane);
        else
            hipLaunchKernelGGL(mfma::k_leaf_direct<1>, dim3(gx), dim3(256), 0, s, dm.k, m,
                               dm.L, dm.leaves, dm.first, dm.size, dm.perm, (const double *)dm.Vt, dm.vt_off, yh, ldh,
                               dm.near_ptr, dm.near_col, dm.near_off, (const double *)dm.N, Xt, ldxt, alpha, b, Y,
                               ldy, to, basis, near, sk, dm.n_plane);
    };
    // near field on the operator's second stream while the transfer passes and the
    // coupling run here (it needs only X); the basis term joins it at the end.  Its
    // grid is capped so that it leaves room on the chip for the transfer chain:
    // overlap 1: 256 work-groups, 3: 128, 4: 512; 0 (the built-in rule) and 2: off
    const bool ov = dm.side && dm.n_near > 0 && (cfg.overlap == 1 || cfg.overlap == 3 || cfg.overlap == 4);
    if (ov) {
        const unsigned cap = cfg.overlap == 3 ? 128u : (cfg.overlap == 4 ? 512u : 256u);
        (void)hipEventRecord(dm.ev_fork, st);
        (void)hipStreamWaitEvent(dm.side, dm.ev_fork, 0);
        leaf(dm.side, beta, 0, 1, cap);
        (void)hipEventRecord(dm.ev_join, dm.side);
    }
    // overlap 6: the near field in two halves on the operator's second stream, each beside a
    // latency-bound stretch of this stream: the first half (the first leaf_half positions of
    // every XCD eighth of the leaf order, about half of the near entries) beside the forward
    // leaf transform and the upward pass, the second beside the downward pass.  Its
    // work-groups take enough LDS that a CU holds at most three of them and keeps room for a
    // transfer work-group.  The basis term follows the downward pass (not with per-stage
    // timing or the fused upward pass).
    const bool halves = kind == 3 && t64 && dm.side && dm.n_near > 0 && cfg.overlap == 6 && !ev &&
                        cfg.fuse_up != 1 && dm.leaf_half > 0;
    // coupling of the deep rows on the second stream beside the upper transfer levels, the
    // coupling of the other rows and the upper downward levels (not with per-stage timing,
    // the concurrent near field or the fused upward pass)
    const bool split = (cfg.split == 1 || cfg.split == 3) && dm.split_depth > 0 && dm.side && !ov && !halves && !ev &&
                       cfg.fuse_up != 1;
    // near field in shares beside the transfer levels (the leaf form with one contraction per
    // leaf, rank 64): each level launch also runs a share of the near-field slots, so that
    // the levels' chain of dependent launches overlaps streaming work; the basis term
    // follows the downward pass.  overlap 5 only (measured slower: a leaf's work-group runs
    // for tens of microseconds, so every level launch lasts as long as its slowest leaf)
    int n_levels = 0;
    for (int d = dm.depth_max - 1; d >= P.adm_depth; --d) n_levels += P.lvl_inner_ptr[d + 1] > P.lvl_inner_ptr[d];
    for (int d = std::max(1, P.adm_depth + 1); d <= dm.depth_max; ++d) n_levels += P.lvl_ptr[d + 1] > P.lvl_ptr[d];
    const size_t lvl_lds = std::max(sizeof(double) * 2 * 64 * (16 * NJ + 1),
                                    sizeof(double) * 64 * (32 * NP + 1) + cat_lds);
    const bool inter = kind == 3 && t64 && dm.n_near > 0 && n_levels > 0 && !ov && !split && cfg.fuse_up != 1 &&
                       cfg.overlap == 5 && lvl_lds <= 65536;
    const int64_t share = n_levels > 0 ? (cat_slots + n_levels - 1) / n_levels : 0;
    int64_t next_slot = 0;
    auto level_near = [&](bool up, int32_t b, int32_t e) {
        const int64_t s0 = next_slot, s1 = std::min(cat_slots, next_slot + share);
        next_slot = s1;
        const int64_t items = (int64_t)(e - b) * gy;
        const int lead = (int)(((s0 - items) % 8 + 8) % 8);
        const dim3 grid((unsigned)(items + lead + (s1 - s0)));
        const mfma::LeafCatArgs a = cat_args(beta, 0, 1);
        const int32_t *list = up ? dm.lvl_inner + b : dm.lvl_all + b;
        const int32_t *aux = up ? dm.up_son + 2 * b : dm.dn_par + b;
        double *hat = up ? xh : yh;
        if (up) {
            if (NP == 2)
                hipLaunchKernelGGL((mfma::k_level_near<NJ, 2, 1>), grid, dim3(256), lvl_lds, st, items, (int)gy, m,
                                   list, aux, E, hat, ldh, sk, a, s0, lead);
            else
                hipLaunchKernelGGL((mfma::k_level_near<NJ, 1, 1>), grid, dim3(256), lvl_lds, st, items, (int)gy, m,
                                   list, aux, E, hat, ldh, sk, a, s0, lead);
        } else {
            if (NP == 2)
                hipLaunchKernelGGL((mfma::k_level_near<NJ, 2, 0>), grid, dim3(256), lvl_lds, st, items, (int)gy, m,
                                   list, aux, E, hat, ldh, sk, a, s0, lead);
            else
                hipLaunchKernelGGL((mfma::k_level_near<NJ, 1, 0>), grid, dim3(256), lvl_lds, st, items, (int)gy, m,
                                   list, aux, E, hat, ldh, sk, a, s0, lead);
        }
    };
    auto up_levels = [&](int dhi, int dlo) {  // upward levels dhi down to dlo
        for (int d = dhi; d >= dlo; --d) {
            const int32_t b = P.lvl_inner_ptr[d], e = P.lvl_inner_ptr[d + 1];
            if (e <= b) continue;
            if (inter)
                level_near(true, b, e);
            else if (t64 && kKronTransfer && NJ > 1 && (int64_t)(e - b) * gy < kNarrowLevel)
                hipLaunchKernelGGL((kron::k_up<4, 16>), dim3(e - b, (unsigned)((m + 15) / 16)), dim3(256), 0, st, m,
                                   dm.lvl_inner + b, dm.up_son + 2 * b, dm.E1, xh, ldh, sk);
            else if (t64 && kKronTransfer)
                hipLaunchKernelGGL((kron::k_up<4, 16 * NJ>), dim3(e - b, gy), dim3(256), 0, st, m, dm.lvl_inner + b,
                                   dm.up_son + 2 * b, dm.E1, xh, ldh, sk);
            else if (t64)
                hipLaunchKernelGGL(mfma::k_up64<NJ>, dim3(e - b, gy), dim3(256), 0, st, m, dm.lvl_inner + b,
                                   dm.up_son + 2 * b, E, xh, ldh, sk);
            else if (dm.p == 3 && kKronTransfer)
                hipLaunchKernelGGL((kron::k_up<3, 16 * NJ>), dim3(e - b, gy), dim3(256), 0, st, m, dm.lvl_inner + b,
                                   dm.up_son + 2 * b, dm.E1, xh, ldh, sk);
            else
                hipLaunchKernelGGL(mfma::k_up<NJ>, dim3(e - b, gy), dim3(256), 0, st, dm.k, m, dm.lvl_inner + b,
                                   dm.up_son + 2 * b, E, xh, ldh, sk);
        }
    };
    auto down_levels = [&](int dlo, int dhi) {  // downward levels (son depths) dlo up to dhi
        for (int d = dlo; d <= dhi; ++d) {
            const int32_t b = P.lvl_ptr[d], e = P.lvl_ptr[d + 1];
            if (e <= b) continue;
            if (inter)
                level_near(false, b, e);
            else if (t64 && kKronTransfer && NJ > 1 && (int64_t)(e - b) * gy < kNarrowLevel)
                hipLaunchKernelGGL((kron::k_down<4, 16>), dim3(e - b, (unsigned)((m + 15) / 16)), dim3(256), 0, st, m,
                                   dm.lvl_all + b, dm.dn_par + b, dm.E1, yh, ldh, sk);
            else if (t64 && kKronTransfer)
                hipLaunchKernelGGL((kron::k_down<4, 16 * NJ>), dim3(e - b, gy), dim3(256), 0, st, m, dm.lvl_all + b,
                                   dm.dn_par + b, dm.E1, yh, ldh, sk);
            else if (t64)
                hipLaunchKernelGGL(mfma::k_down64<NJ>, dim3(e - b, gy), dim3(256), 0, st, m, dm.lvl_all + b,
                                   dm.dn_par + b, E, yh, ldh, sk);
            else if (dm.p == 3 && kKronTransfer)
                hipLaunchKernelGGL((kron::k_down<3, 16 * NJ>), dim3(e - b, gy), dim3(256), 0, st, m, dm.lvl_all + b,
                                   dm.dn_par + b, dm.E1, yh, ldh, sk);
            else
                hipLaunchKernelGGL(mfma::k_down<NJ>, dim3(e - b, gy), dim3(256), 0, st, dm.k, m, dm.lvl_all + b,
                                   dm.dn_par + b, E, yh, ldh, sk);
        }
    };
    // complex operator: y-hat += S_im (J x-hat), so that y-hat = (S_re + i S_im) x-hat per complex column
    auto coupling = [&](hipStream_t s, int32_t nrows, const int32_t *rows, size_t keep) {
        launch_coupling_fast<double, double>(dm, m, xh, yh, ldh, s, sk, cfg.nj_coupling, 0, nrows, rows, keep);
        if (dm.cplx)
            launch_coupling_fast<double, double>(dm, m, xh, yh, ldh, s, sk, cfg.nj_coupling, 1, nrows, rows, keep);
    };
    const int dlo = std::max(1, P.adm_depth + 1);
    if (halves) {
        // dynamic LDS of the near work-groups: more than a quarter of a CU's LDS (at most
        // three per CU), and small enough that three of them and an upward work-group fit
        size_t dyn = cat_lds;
        {
            hipFuncAttributes fa{}, fu{};
            int dev = 0, per_cu = 0;
            const void *fl = NP == 2 ? (const void *)mfma::k_leaf_cat<2> : (const void *)mfma::k_leaf_cat<1>;
            if (hipFuncGetAttributes(&fa, fl) == hipSuccess &&
                hipFuncGetAttributes(&fu, kKronTransfer ? (const void *)kron::k_up<4, 16 * NJ>
                                                        : (const void *)mfma::k_up64<NJ>) == hipSuccess &&
                hipGetDevice(&dev) == hipSuccess &&
                hipDeviceGetAttribute(&per_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) ==
                    hipSuccess) {
                const size_t lo = (((size_t)per_cu / 4 + 1024) + 511) & ~(size_t)511;
                const size_t hi = (size_t)per_cu > fu.sharedSizeBytes ? ((size_t)per_cu - fu.sharedSizeBytes) / 3 : 0;
                if (lo <= hi && lo <= 65536 && lo > fa.sharedSizeBytes + cat_lds) dyn = lo - fa.sharedSizeBytes;
            }
        }
        auto near_part = [&](int64_t s0, int64_t s1) {
            if (s1 <= s0) return;
            if (NP == 2)
                hipLaunchKernelGGL(mfma::k_leaf_cat<2>, dim3((unsigned)(s1 - s0)), dim3(256), dyn, dm.side,
                                   cat_args(beta, 0, 1), s0, s1);
            else
                hipLaunchKernelGGL(mfma::k_leaf_cat<1>, dim3((unsigned)(s1 - s0)), dim3(256), dyn, dm.side,
                                   cat_args(beta, 0, 1), s0, s1);
        };
        // slots below sA: the first leaf_half positions of every eighth (a multiple of 8, so
        // slot s still runs on XCD s % 8)
        const int64_t sA = std::min<int64_t>(cat_slots, (int64_t)8 * dm.leaf_half * gl);
        (void)hipEventRecord(dm.ev_fork, st);
        (void)hipStreamWaitEvent(dm.side, dm.ev_fork, 0);
        near_part(0, sA);
        fwd_leaf();
        up_levels(dm.depth_max - 1, P.adm_depth);
        coupling(st, -1, nullptr, 0);
        (void)hipEventRecord(dm.ev_fork, st);
        (void)hipStreamWaitEvent(dm.side, dm.ev_fork, 0);
        near_part(sA, cat_slots);
        (void)hipEventRecord(dm.ev_join, dm.side);
        down_levels(dlo, dm.depth_max);
        (void)hipStreamWaitEvent(st, dm.ev_join, 0);
        leaf(st, 1.0, 1, 0, 0);  // the near field is in Y already (beta applied there)
        return;
    }
    if (split) {
        fwd_leaf();
        const int D = dm.split_depth;
        up_levels(dm.depth_max - 1, D);
        (void)hipEventRecord(dm.ev_fork, st);
        (void)hipStreamWaitEvent(dm.side, dm.ev_fork, 0);
        // split 1: the deep coupling leaves room on every CU for a work-group of the transfer
        // passes (their LDS); split 3: no reserve
        size_t keep = 0;
        if (cfg.split == 1) {
            hipFuncAttributes a{}, b{};
            const void *fu = t64 ? (kKronTransfer ? (const void *)kron::k_up<4, 16 * NJ> : (const void *)mfma::k_up64<NJ>)
                             : (dm.p == 3 && kKronTransfer ? (const void *)kron::k_up<3, 16 * NJ>
                                                           : (const void *)mfma::k_up<NJ>);
            const void *fd = t64 ? (kKronTransfer ? (const void *)kron::k_down<4, 16 * NJ> : (const void *)mfma::k_down64<NJ>)
                             : (dm.p == 3 && kKronTransfer ? (const void *)kron::k_down<3, 16 * NJ>
                                                           : (const void *)mfma::k_down<NJ>);
            if (hipFuncGetAttributes(&a, fu) == hipSuccess && hipFuncGetAttributes(&b, fd) == hipSuccess)
                keep = std::max(a.sharedSizeBytes, b.sharedSizeBytes);
        }
        coupling(dm.side, dm.n_deep, dm.cpl_deep, keep);
        (void)hipEventRecord(dm.ev_join, dm.side);
        up_levels(D - 1, P.adm_depth);
        coupling(st, dm.n_shallow, dm.cpl_shallow, 0);
        down_levels(dlo, D - 1);
        (void)hipStreamWaitEvent(st, dm.ev_join, 0);
        down_levels(std::max(dlo, D), dm.depth_max);
        leaf(st, beta, 1, 1, 0);
        return;
    }
    if (cfg.fuse_up == 1) {
        // one launch: leaves, then each parent by the work-group that finishes its second son
        // (slower than level-by-level launches on this chip: every device-scope fence writes
        // back the XCD's L2, so the built-in rule keeps it off)
        int32_t *cnt = (int32_t *)(xt_ws + dm.n * even_ld(m));
        const int64_t nc = (int64_t)dm.C * gy;
        hipLaunchKernelGGL(mfma::k_zero_i32, dim3((unsigned)((nc + 255) / 256)), dim3(256), 0, st, nc, cnt);
        hipLaunchKernelGGL(mfma::k_fwd_up<NJ>, dim3(8 * ((dm.L + 7) / 8), gy), dim3(256), 0, st, dm.k, m, dm.L,
                           dm.leaves, dm.first, dm.size, V, Xt, ldxt, dm.parent, dm.son0, dm.son1, dm.depth,
                           P.adm_depth, E, xh, ldh, cnt, sk);
        mark(1);
    } else {
        fwd_leaf();
        mark(1);
        up_levels(dm.depth_max - 1, P.adm_depth);
    }
    mark(2);
    coupling(st, -1, nullptr, 0);
    mark(3);
    down_levels(dlo, dm.depth_max);
    mark(4);
    // Y = beta Y + alpha (V y-hat + N X)
    if (ov) {
        (void)hipStreamWaitEvent(st, dm.ev_join, 0);
        leaf(st, 1.0, 1, 0, 0);
    } else if (inter) {
        leaf(st, 1.0, 1, 0, 0);  // the near field is in Y already (beta applied there)
    } else {
        leaf(st, beta, 1, 1, 0);
    }
    mark(5);
    if (ev) (void)hipEventRecord(ev[6], st);
}

template <typename Acc>
size_t hat_bytes(const DevMat &dm, int64_t m) {
    return align_up(sizeof(Acc) * (size_t)dm.C * dm.k * (size_t)even_ld(m));
}

template <typename T, typename TN, typename Acc>
hipError_t matmul_typed(const DevMat &dm, const TuneCfg &cfg, int64_t m, double alpha, const double *X, int64_t ldx,
                        double beta, double *Y, int64_t ldy, bool tree_order, char *ws, hipStream_t st, hipEvent_t *ev,
                        const int32_t *skip) {
    auto mark = [&](int i) {
        if (ev) (void)hipEventRecord(ev[i], st);
    };
    const Plan &P = *dm.plan;
    // low-precision operator in the matrix-core layout (k = 64 or k <= 32): FP32
    // matrix-core coupling and leaf stage, generic transfer passes
    const bool lpmc = !std::is_same<T, double>::value && dm.near_t && (dm.k == 64 || dm.k <= 32);
    const int64_t ldh = (dm.mc || lpmc) ? even_ld(m) : m;
    Acc *xh = (Acc *)ws;
    Acc *yh = (Acc *)(ws + hat_bytes<Acc>(dm, m));
    const unsigned gy = (unsigned)((m + TC - 1) / TC);
    const int to = tree_order ? 1 : 0;
    const T *V = (const T *)dm.V, *E = (const T *)dm.E, *S = (const T *)dm.S;
    (void)skip;  // only the matrix-core path leaves stopped systems out

    if constexpr (std::is_same<T, double>::value && std::is_same<Acc, double>::value) {
        if (dm.mc) {
            const std::function<void(int)> mk = mark;
            double *xt = (double *)(ws + 2 * hat_bytes<Acc>(dm, m));
            switch (cfg.nj_transfer ? (int)cfg.nj_transfer : (int)std::min<int64_t>(4, (m + 15) / 16)) {
                case 1: matmul_mfma_f64<1>(dm, cfg, m, alpha, X, ldx, beta, Y, ldy, to, xh, yh, ldh, xt, st, mk, ev, skip); break;
                case 2: matmul_mfma_f64<2>(dm, cfg, m, alpha, X, ldx, beta, Y, ldy, to, xh, yh, ldh, xt, st, mk, ev, skip); break;
                case 3: matmul_mfma_f64<3>(dm, cfg, m, alpha, X, ldx, beta, Y, ldy, to, xh, yh, ldh, xt, st, mk, ev, skip); break;
                default: matmul_mfma_f64<4>(dm, cfg, m, alpha, X, ldx, beta, Y, ldy, to, xh, yh, ldh, xt, st, mk, ev, skip); break;
            }
            return hipGetLastError();
        }
    }

    mark(0);
    bool fwd_done = false;
    if constexpr (std::is_same<Acc, float>::value && !std::is_same<T, double>::value) {
        if (lpmc) {
            // the FP32 tree-ordered copy of X serves the forward leaf transform and the leaf stage
            float *xt = (float *)(ws + 2 * hat_bytes<Acc>(dm, m));
            const int64_t ldxt = even_ld(m);
            hipLaunchKernelGGL(lp::k_gather_f32, dim3((unsigned)((dm.n + 3) / 4)), dim3(256), 0, st, dm.n, m,
                               to ? nullptr : dm.perm, X, ldx, xt, ldxt);
            if (dm.L > 0)
                hipLaunchKernelGGL((tlp::k_fwd_leaf_lp<T>), dim3(dm.L, gy), dim3(256), 0, st, dm.k, m, dm.leaves,
                                   dm.first, dm.size, V, (const float *)xt, ldxt, xh, ldh);
            fwd_done = true;
        }
    }
    if (!fwd_done)
        hipLaunchKernelGGL((k_fwd_leaf<T, Acc>), dim3(dm.L, gy), dim3(256), 0, st, dm.k, m, dm.leaves, dm.first,
                           dm.size, dm.perm, V, X, ldx, to, xh, ldh);
    mark(1);
    // transfer passes of the low-precision matrix-core layout on the FP32 matrix cores
    // (4-long contraction steps: 16 for k = 64, 8 for k <= 32)
    // downward, rank 64 with more than 32 columns: 64 columns per work-group, so that E_c is
    // read once (measured at m = 64: 0.42 -> 0.37 ms per product; the upward pass was slower
    // that way, 0.20 -> 0.23 ms, and keeps 32)
    const unsigned g64 = (unsigned)((m + 63) / 64);
    auto up_lp = [&](int32_t b, int32_t e) {
        if constexpr (std::is_same<Acc, float>::value && !std::is_same<T, double>::value) {
            if (dm.k == 64)
                hipLaunchKernelGGL((tlp::k_up_lp<16, T>), dim3(e - b, gy), dim3(256), 0, st, dm.k, m,
                                   dm.lvl_inner + b, dm.son0, dm.son1, E, xh, ldh);
            else
                hipLaunchKernelGGL((tlp::k_up_lp<8, T>), dim3(e - b, gy), dim3(256), 0, st, dm.k, m,
                                   dm.lvl_inner + b, dm.son0, dm.son1, E, xh, ldh);
            return true;
        }
        return false;
    };
    auto down_lp = [&](int32_t b, int32_t e) {
        if constexpr (std::is_same<Acc, float>::value && !std::is_same<T, double>::value) {
            if (dm.k == 64 && m > 32)
                hipLaunchKernelGGL((tlp::k_down_lp<16, T, 4>), dim3(e - b, g64), dim3(256), 0, st, dm.k, m,
                                   dm.lvl_all + b, dm.parent, E, yh, ldh);
            else if (dm.k == 64)
                hipLaunchKernelGGL((tlp::k_down_lp<16, T>), dim3(e - b, gy), dim3(256), 0, st, dm.k, m,
                                   dm.lvl_all + b, dm.parent, E, yh, ldh);
            else
                hipLaunchKernelGGL((tlp::k_down_lp<8, T>), dim3(e - b, gy), dim3(256), 0, st, dm.k, m,
                                   dm.lvl_all + b, dm.parent, E, yh, ldh);
            return true;
        }
        return false;
    };
    for (int d = dm.depth_max - 1; d >= P.adm_depth; --d) {
        const int32_t b = P.lvl_inner_ptr[d], e = P.lvl_inner_ptr[d + 1];
        if (e > b && !(lpmc && up_lp(b, e)))
            hipLaunchKernelGGL((k_up<T, Acc>), dim3(e - b, gy), dim3(256), 0, st, dm.k, m, dm.lvl_inner + b, dm.son0,
                               dm.son1, E, xh, ldh);
    }
    mark(2);
    bool fast = launch_coupling_fast<T, Acc>(dm, m, xh, yh, ldh, st, Skip{}, 0);
    if constexpr (std::is_same<Acc, float>::value && !std::is_same<T, double>::value)
        if (!fast) {
            // BF16, k = 64: x-hat rounded to BF16 once per cluster for the coupling
            uint16_t *xb = nullptr;
            if (std::is_same<T, bf16_t>::value && lpmc && dm.k == 64) {
                xb = (uint16_t *)(ws + 2 * hat_bytes<Acc>(dm, m) + align_up(sizeof(float) * (size_t)dm.n * even_ld(m)));
                const int64_t cnt4 = (int64_t)dm.C * dm.k * ldh / 4;  // k = 64: a multiple of 4
                hipLaunchKernelGGL(k_pack_bf16, dim3((unsigned)((cnt4 + 255) / 256)), dim3(256), 0, st, cnt4,
                                   (const float4 *)xh, (uint2 *)xb);
            }
            fast = launch_coupling_lp<T>(dm, m, xh, xb, yh, ldh, st, Skip{skip, dm.sys_of}, cfg.nj_coupling);
        }
    if (!fast)
        hipLaunchKernelGGL((k_coupling<T, Acc>), dim3(dm.C, gy), dim3(256), 0, st, dm.k, m, dm.adm_ptr, dm.adm_col, S,
                           dm.swz, xh, yh, ldh);
    mark(3);
    for (int d = std::max(1, P.adm_depth + 1); d <= dm.depth_max; ++d) {
        const int32_t b = P.lvl_ptr[d], e = P.lvl_ptr[d + 1];
        if (e > b && !(lpmc && down_lp(b, e)))
            hipLaunchKernelGGL((k_down<T, Acc>), dim3(e - b, gy), dim3(256), 0, st, dm.k, m, dm.lvl_all + b, dm.parent,
                               E, yh, ldh);
    }
    mark(4);
    if constexpr (std::is_same<Acc, float>::value && !std::is_same<T, double>::value && std::is_same<TN, float>::value) {
        if (lpmc) {
            float *xt = (float *)(ws + 2 * hat_bytes<Acc>(dm, m));  // gathered before the forward transform
            const int64_t ldxt = even_ld(m);
            const Skip sk{skip, dm.sys_of};
            const int rb = std::is_same<T, bf16_t>::value ? 1 : 0;
            const unsigned gl8 = 8 * ((dm.L + 7) / 8);
            const int NPl = cfg.np_leaf ? cfg.np_leaf : (m > 32 ? 2 : 1);
            // one contraction per leaf (built-in where its table of near rows fits in LDS;
            // leaf_kind 3 or 0), else a 64-row tile per wave and term (leaf_kind 1 or 2)
            const size_t cat_lds = sizeof(int32_t) * (size_t)std::max(1, dm.max_near_rows);
            const size_t red = NPl == 2 ? lp::leaf_cat_lp_red_bytes<2>() : lp::leaf_cat_lp_red_bytes<1>();
            // (it reads the rows of X through a buffer resource: 32-bit byte offsets)
            const bool cat_ok = !dm.cplx && cat_lds + red + 64 <= 65536 &&
                                sizeof(float) * (size_t)dm.n * (size_t)ldxt < ((size_t)1 << 32);
            if (cat_ok && (cfg.leaf_kind == 0 || cfg.leaf_kind == 3)) {
                const lp::LeafCatLpArgs a{dm.k, m, dm.L, dm.leaf_order, dm.leaves, dm.first, dm.size, dm.perm,
                                          dm.Vt, dm.vt_off, yh, ldh, dm.near_ptr, dm.near_col, dm.near_off,
                                          (const float *)dm.N, xt, ldxt, alpha, beta, Y, ldy, to, rb, sk};
                const unsigned grid = gl8 * (unsigned)((m + 32 * NPl - 1) / (32 * NPl));
                if (NPl == 2)
                    hipLaunchKernelGGL((lp::k_leaf_cat_lp<2, T>), dim3(grid), dim3(256), cat_lds, st, a);
                else
                    hipLaunchKernelGGL((lp::k_leaf_cat_lp<1, T>), dim3(grid), dim3(256), cat_lds, st, a);
            } else if (NPl == 2)
                hipLaunchKernelGGL((lp::k_leaf_lp<2, T>), dim3(gl8 * (unsigned)((m + 63) / 64)), dim3(256), 0, st,
                                   dm.k, m, dm.L, dm.leaves, dm.first, dm.size, dm.perm, (const T *)dm.Vt, dm.vt_off,
                                   yh, ldh, dm.near_ptr, dm.near_col, dm.near_off, (const float *)dm.N, xt, ldxt,
                                   alpha, beta, Y, ldy, to, rb, sk);
            else
                hipLaunchKernelGGL((lp::k_leaf_lp<1, T>), dim3(gl8 * (unsigned)((m + 31) / 32)), dim3(256), 0, st,
                                   dm.k, m, dm.L, dm.leaves, dm.first, dm.size, dm.perm, (const T *)dm.Vt, dm.vt_off,
                                   yh, ldh, dm.near_ptr, dm.near_col, dm.near_off, (const float *)dm.N, xt, ldxt,
                                   alpha, beta, Y, ldy, to, rb, sk);
            mark(5);
            if (ev) (void)hipEventRecord(ev[6], st);
            return hipGetLastError();
        }
    }
    hipLaunchKernelGGL((k_leaf_near<T, TN, Acc>), dim3(dm.L, gy), dim3(256), 0, st, dm.k, m, dm.leaves, dm.first,
                       dm.size, dm.perm, V, yh, ldh, dm.near_ptr, dm.near_col, dm.near_off, (const TN *)dm.N, X, ldx,
                       alpha, beta, Y, ldy, to, dm.near_t);
    mark(5);
    if (ev) (void)hipEventRecord(ev[6], st);
    return hipGetLastError();
}

}  // namespace

hipError_t run_forward_transform(const DevMat &dm, int64_t m, const double *X, int64_t ldx, bool tree_order,
                                 double *xh, int64_t ldh, double *xt_ws, hipStream_t st) {
    const Plan &P = *dm.plan;
    const double *V = (const double *)dm.V, *E = (const double *)dm.E;
    if (dm.mc) {
        const double *Xt = X;
        int64_t ldxt = ldx;
        if (!tree_order || (ldx & 1) || ((uintptr_t)X & 15)) {
            ldxt = even_ld(m);
            const int64_t cnt = dm.n * ldxt;
            hipLaunchKernelGGL(mfma::k_gather, dim3((unsigned)((cnt / 2 + 255) / 256)), dim3(256), 0, st, dm.n, m,
                               tree_order ? nullptr : dm.perm, X, ldx, xt_ws, ldxt);
            Xt = xt_ws;
        }
        const int nj = (int)std::min<int64_t>(4, (m + 15) / 16);
        const unsigned gy = (unsigned)((m + 16 * nj - 1) / (16 * nj));
        auto launch = [&](auto NJc) {
            constexpr int NJ = decltype(NJc)::value;
            hipLaunchKernelGGL(mfma::k_fwd_leaf<NJ>, dim3(dm.L, gy), dim3(256), 0, st, dm.k, m, dm.leaves, dm.first,
                               dm.size, dm.perm, V, Xt, ldxt, 1, xh, ldh, Skip{});
            for (int d = dm.depth_max - 1; d >= P.adm_depth; --d) {
                const int32_t b = P.lvl_inner_ptr[d], e = P.lvl_inner_ptr[d + 1];
                if (e > b && dm.k == 64 && kKronTransfer)
                    hipLaunchKernelGGL((kron::k_up<4, 16 * NJ>), dim3(e - b, gy), dim3(256), 0, st, m, dm.lvl_inner + b,
                                       dm.up_son + 2 * b, dm.E1, xh, ldh, Skip{});
                else if (e > b && dm.p == 3 && kKronTransfer)
                    hipLaunchKernelGGL((kron::k_up<3, 16 * NJ>), dim3(e - b, gy), dim3(256), 0, st, m, dm.lvl_inner + b,
                                       dm.up_son + 2 * b, dm.E1, xh, ldh, Skip{});
                else if (e > b)
                    hipLaunchKernelGGL(mfma::k_up<NJ>, dim3(e - b, gy), dim3(256), 0, st, dm.k, m, dm.lvl_inner + b,
                                       dm.up_son + 2 * b, E, xh, ldh, Skip{});
            }
        };
        switch (nj) {
            case 1: launch(std::integral_constant<int, 1>{}); break;
            case 2: launch(std::integral_constant<int, 2>{}); break;
            case 3: launch(std::integral_constant<int, 3>{}); break;
            default: launch(std::integral_constant<int, 4>{}); break;
        }
        return hipGetLastError();
    }
    const unsigned gy = (unsigned)((m + TC - 1) / TC);
    hipLaunchKernelGGL((k_fwd_leaf<double, double>), dim3(dm.L, gy), dim3(256), 0, st, dm.k, m, dm.leaves, dm.first,
                       dm.size, dm.perm, V, X, ldx, tree_order ? 1 : 0, xh, ldh);
    for (int d = dm.depth_max - 1; d >= P.adm_depth; --d) {
        const int32_t b = P.lvl_inner_ptr[d], e = P.lvl_inner_ptr[d + 1];
        if (e > b)
            hipLaunchKernelGGL((k_up<double, double>), dim3(e - b, gy), dim3(256), 0, st, dm.k, m, dm.lvl_inner + b,
                               dm.son0, dm.son1, E, xh, ldh);
    }
    return hipGetLastError();
}

hipError_t run_down_pass(const DevMat &dm, int64_t m, double *yh, int64_t ldh, hipStream_t st) {
    const Plan &P = *dm.plan;
    const double *E = (const double *)dm.E;
    if (dm.mc) {
        const int nj = (int)std::min<int64_t>(4, (m + 15) / 16);
        const unsigned gy = (unsigned)((m + 16 * nj - 1) / (16 * nj));
        auto go = [&](auto NJc) {
            constexpr int NJ = decltype(NJc)::value;
            for (int d = std::max(1, P.adm_depth + 1); d <= dm.depth_max; ++d) {
                const int32_t b = P.lvl_ptr[d], e = P.lvl_ptr[d + 1];
                if (e > b && dm.k == 64 && kKronTransfer)
                    hipLaunchKernelGGL((kron::k_down<4, 16 * NJ>), dim3(e - b, gy), dim3(256), 0, st, m, dm.lvl_all + b,
                                       dm.dn_par + b, dm.E1, yh, ldh, Skip{});
                else if (e > b && dm.p == 3 && kKronTransfer)
                    hipLaunchKernelGGL((kron::k_down<3, 16 * NJ>), dim3(e - b, gy), dim3(256), 0, st, m, dm.lvl_all + b,
                                       dm.dn_par + b, dm.E1, yh, ldh, Skip{});
                else if (e > b)
                    hipLaunchKernelGGL(mfma::k_down<NJ>, dim3(e - b, gy), dim3(256), 0, st, dm.k, m, dm.lvl_all + b,
                                       dm.dn_par + b, E, yh, ldh, Skip{});
            }
        };
        switch (nj) {
            case 1: go(std::integral_constant<int, 1>{}); break;
            case 2: go(std::integral_constant<int, 2>{}); break;
            case 3: go(std::integral_constant<int, 3>{}); break;
            default: go(std::integral_constant<int, 4>{}); break;
        }
        return hipGetLastError();
    }
    const unsigned gy = (unsigned)((m + TC - 1) / TC);
    for (int d = std::max(1, P.adm_depth + 1); d <= dm.depth_max; ++d) {
        const int32_t b = P.lvl_ptr[d], e = P.lvl_ptr[d + 1];
        if (e > b)
            hipLaunchKernelGGL((k_down<double, double>), dim3(e - b, gy), dim3(256), 0, st, dm.k, m, dm.lvl_all + b,
                               dm.parent, E, yh, ldh);
    }
    return hipGetLastError();
}

size_t matmul_ws_bytes(const DevMat &dm, int64_t m) {
    // x-hat, y-hat, and the tree-ordered copy of X used by the matrix-core path
    // (FP64: plus the per-parent counters of the fused upward pass, clusters x column slabs)
    if (dm.storage == H2X_F64)
        return 2 * hat_bytes<double>(dm, m) + align_up(sizeof(double) * (size_t)dm.n * even_ld(m)) +
               align_up(sizeof(int32_t) * (size_t)dm.C * (size_t)((m + 15) / 16));
    // low precision: x-hat, y-hat, and the FP32 tree-ordered copy of X of the matrix-core leaf stage;
    // BF16 with k = 64: and the BF16 copy of x-hat that the coupling reads
    const bool xb = dm.storage == H2X_BF16 && dm.near_t && dm.k == 64;
    return 2 * hat_bytes<float>(dm, m) + (dm.near_t ? align_up(sizeof(float) * (size_t)dm.n * even_ld(m)) : 0) +
           (xb ? align_up(sizeof(uint16_t) * (size_t)dm.C * dm.k * (size_t)even_ld(m)) : 0);
}

hipError_t run_matmul_cfg(const DevMat &dm, const TuneCfg &cfg, int64_t m, double alpha, const double *X, int64_t ldx,
                          double beta, double *Y, int64_t ldy, bool tree_order, char *ws, hipStream_t st,
                          hipEvent_t *ev, const int32_t *skip) {
    switch (dm.storage) {
        case H2X_F64:
            return matmul_typed<double, double, double>(dm, cfg, m, alpha, X, ldx, beta, Y, ldy, tree_order, ws, st,
                                                        ev, skip);
        case H2X_F32:
            return matmul_typed<float, float, float>(dm, cfg, m, alpha, X, ldx, beta, Y, ldy, tree_order, ws, st, ev,
                                                     skip);
        default:
            return matmul_typed<bf16_t, float, float>(dm, cfg, m, alpha, X, ldx, beta, Y, ldy, tree_order, ws, st, ev,
                                                      skip);
    }
}

hipError_t run_matmul(const DevMat &dm, int64_t m, double alpha, const double *X, int64_t ldx, double beta, double *Y,
                      int64_t ldy, bool tree_order, char *ws, hipStream_t st, hipEvent_t *ev, const int32_t *skip) {
    return run_matmul_cfg(dm, dm.tuned[tune_bucket(m)], m, alpha, X, ldx, beta, Y, ldy, tree_order, ws, st, ev, skip);
}

}  // namespace h2x
