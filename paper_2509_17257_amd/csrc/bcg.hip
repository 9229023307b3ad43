// Block CG over one shared block Krylov space (O'Leary's block CG, which the
// paper cites as the variant that enriches the Krylov space), FP64 throughout:
//   Q = A P,  G = P^T Q,  Lambda = G^{-1} P^T R,  X += P Lambda,  R -= Q Lambda,
//   Psi = -G^{-1} Q^T R,  P = orth(R + P Psi).
// The search block P is kept orthonormal by Cholesky QR applied twice; the
// first pass pivots on the largest remaining column norm and drops directions
// whose remaining norm falls below 1e-6 of the largest (deflation), so the
// m x m Gram matrices stay positive definite when columns become dependent.
// Dropped columns of P are zero; all m x m work uses the active index set.
//
// Tall-skinny products (U^T V, U C) stream the n x m blocks once; the m x m
// factorizations run in one work-group.  Gram matrices are reduced in two
// fixed-order passes, so the solve is bitwise reproducible.  The host reads the
// convergence state after every iteration.
#include <cmath>
#include <vector>

#include "device.hpp"

namespace h2x {

namespace {

constexpr int kMaxM = 64;      // block size limit of this variant
constexpr double kDrop = 1e-6; // deflation threshold (relative column norm)

struct BcgState {
    int32_t rank, all_conv, iter, breakdown;
    int32_t stop, pad;  // stop: set at the start of an iteration that must not run
    int32_t active[kMaxM];
    int32_t piv[kMaxM];
    int32_t conv[kMaxM];
    int32_t first_conv[kMaxM];
    double bnorm[kMaxM];
    double rnorm[kMaxM];
};

// part[(pair * nblk + blk) * m * m + a * m + b] = sum over the block's rows of U[i][a] V[i][b],
// on the FP64 matrix cores: U^T V as a contraction over the block's rows, A = U^T (16 lanes
// over 16 consecutive columns of a row of U) and B = V (likewise), both straight from
// memory.  Wave w takes the 4-row steps w, w + 4, ... of the block; rows past the block are
// zero in U; the four waves' tiles are added in LDS in wave order.  MT = ceil(m / 16) tiles
// per dimension.
typedef double dbl4 __attribute__((ext_vector_type(4)));

template <int MT>
__global__ __launch_bounds__(256) void k_gram_mfma(int64_t n, int m, int nblk, const double *__restrict__ U0,
                                                   const double *__restrict__ V0, const double *__restrict__ U1,
                                                   const double *__restrict__ V1, double *__restrict__ part,
                                                   const int32_t *stop) {
    if (stop && *stop) return;
    __shared__ double red[kMaxM * kMaxM];
    const int tid = threadIdx.x, lane = tid & 63, lr = lane & 15, lq = lane >> 4;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int mm = m * m;
    const int64_t rows = (n + nblk - 1) / nblk;
    const int64_t r0 = (int64_t)blockIdx.x * rows, r1 = min(n, r0 + rows);
    const int nstep = r1 > r0 ? (int)((r1 - r0 + 3) >> 2) : 0;
    for (int q = 0; q < (U1 ? 2 : 1); ++q) {
        const double *U = q ? U1 : U0, *V = q ? V1 : V0;
        dbl4 acc[MT][MT];
#pragma unroll
        for (int I = 0; I < MT; ++I)
#pragma unroll
            for (int J = 0; J < MT; ++J) acc[I][J] = dbl4{0.0, 0.0, 0.0, 0.0};
        // NS steps of the wave per round, all their loads issued before the first product
        // (steps past the block read a clamped row and multiply zeros); the steps are added in
        // the same order as one at a time
        constexpr int NS = 4;
        for (int st0 = w; st0 < nstep; st0 += 4 * NS) {
            double a[NS][MT], b[NS][MT];
            bool in[NS];
#pragma unroll
            for (int ss = 0; ss < NS; ++ss) {
                const int64_t i = r0 + 4 * (st0 + 4 * ss) + lq;
                in[ss] = i < r1;
                const int64_t ic = in[ss] ? i : r1 - 1;
#pragma unroll
                for (int I = 0; I < MT; ++I) {
                    const int c = min(16 * I + lr, m - 1);
                    a[ss][I] = U[ic * m + c];
                    b[ss][I] = V[ic * m + c];
                }
            }
#pragma unroll
            for (int ss = 0; ss < NS; ++ss)
#pragma unroll
                for (int I = 0; I < MT; ++I) {
                    const double av = in[ss] ? a[ss][I] : 0.0;
#pragma unroll
                    for (int J = 0; J < MT; ++J)
                        acc[I][J] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, b[ss][J], acc[I][J], 0, 0, 0);
                }
        }
        // D layout of the 16x16x4 f64 MFMA: lane l, register r -> row l / 16 + 4 r, column l % 16
        for (int ww = 0; ww < 4; ++ww) {
            if (w == ww)
#pragma unroll
                for (int I = 0; I < MT; ++I)
#pragma unroll
                    for (int J = 0; J < MT; ++J)
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            const int a = 16 * I + lq + 4 * r, b = 16 * J + lr;
                            if (a < m && b < m) {
                                double *cell = &red[a * m + b];
                                *cell = ww == 0 ? acc[I][J][r] : *cell + acc[I][J][r];
                            }
                        }
            __syncthreads();
        }
        for (int e = tid; e < mm; e += 256) part[((int64_t)q * nblk + blockIdx.x) * mm + e] = red[e];
        __syncthreads();
    }
}

// G_q[e] = sum over blocks of the partial sums, in a fixed order: eight neighbouring lanes
// share an entry, lane s adds the blocks of its eighth of the range in block order (all its
// loads in flight at once, clamped addresses; past the end: exact zeros), and the eight
// sums are then added in lane order
constexpr int kGramSplit = 8;
__global__ void k_gram_sum(int m, int nblk, const double *__restrict__ part, double *__restrict__ G0,
                           double *__restrict__ G1, const int32_t *stop) {
    if (stop && *stop) return;
    const int mm = m * m;
    const int gtid = blockIdx.x * blockDim.x + threadIdx.x;
    const int e = gtid / kGramSplit, sp = gtid % kGramSplit;
    const int q = blockIdx.y;
    constexpr int U = 32;  // blocks per lane (nblk <= 256)
    const int per = (nblk + kGramSplit - 1) / kGramSplit, b0 = sp * per;
    const double *p = part + (int64_t)q * nblk * mm + min(e, mm - 1);
    double v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = p[(int64_t)min(b0 + u, nblk - 1) * mm];
    double s = 0.0;
#pragma unroll
    for (int u = 0; u < U; ++u) s += (u < per && b0 + u < nblk) ? v[u] : 0.0;
    double t = 0.0;
#pragma unroll
    for (int k = 0; k < kGramSplit; ++k) t += __shfl(s, (threadIdx.x & ~(kGramSplit - 1)) + k);
    if (sp == 0 && e < mm) (q ? G1 : G0)[e] = t;
}

// out = beta Yin + alpha U C  (n x m blocks, C m x m; Yin may alias out, beta == 0 ignores it).
// A work-group takes 2048 / MT rows (MT = m rounded up to 16): their rows of U are staged
// in LDS with coalesced loads, and thread (rg, b) keeps column b of C in registers and forms
// out[i][b] = sum_a U[i][a] C[a][b] (a in order) for rows i = rg, rg + 256 / m, ...
// Work-groups with blockIdx.y = 1 form the second product (U2, Yin2, out2, alpha2) with the
// same C and beta.
template <int MT>
__global__ __launch_bounds__(256) void k_tsmm(int64_t n, int m, const double *__restrict__ U,
                                              const double *__restrict__ Cm, const double *Yin, double *out,
                                              double alpha, double beta, const double *__restrict__ U2,
                                              const double *Yin2, double *out2, double alpha2, const int32_t *stop) {
    if (stop && *stop) return;
    if (blockIdx.y == 1) {
        U = U2;
        Yin = Yin2;
        out = out2;
        alpha = alpha2;
    }
    constexpr int RW = 2048 / MT;  // rows per work-group
    __shared__ __align__(16) double su[RW][MT];
    const int tid = threadIdx.x;
    const int64_t r0 = (int64_t)blockIdx.x * RW;
    const int rows = (int)min<int64_t>(RW, n - r0);
    const double *ut = U + r0 * m;
    for (int e = tid; e < rows * m; e += 256) su[e / m][e % m] = ut[e];
    const int b = tid % m, rg = tid / m, ng = 256 / m;
    double c[MT];
#pragma unroll
    for (int a = 0; a < MT; ++a) c[a] = (a < m && rg < ng) ? Cm[a * m + b] : 0.0;
    // rows per thread: at most NR, as 256 / m >= 256 / MT; their old values are loaded
    // before the barrier (clamped addresses)
    constexpr int NR = (RW + 256 / MT - 1) / (256 / MT);
    double yv[NR];
#pragma unroll
    for (int t = 0; t < NR; ++t)
        yv[t] = (beta != 0.0 && rg < ng) ? Yin[(r0 + min(rg + t * ng, rows - 1)) * m + b] : 0.0;
    __syncthreads();
    if (rg >= ng) return;
#pragma unroll
    for (int t = 0; t < NR; ++t) {
        const int i = rg + t * ng;
        if (i >= rows) break;
        double s = 0.0;
#pragma unroll
        for (int a = 0; a < MT; a += 2) {
            const double2 u2 = *(const double2 *)&su[i][a];
            if (a < m) s += u2.x * c[a];
            if (a + 1 < m) s += u2.y * c[a + 1];
        }
        out[(r0 + i) * m + b] = (beta == 0.0) ? alpha * s : beta * yv[t] + alpha * s;
    }
}

// ---- m x m steps: right-looking, four waves, one barrier per step ----
//
// Wave w takes the rows congruent to w modulo 4 and lane j the column j of the step's
// update, so a step is one pass of independent multiply-adds over the trailing part; a value
// that the step reads (the pivot column, the pivot row) is scaled where it is read and
// written back scaled in the next step, which no longer reads it.  kMaxM >= m, so a column
// index is a lane index.

// C = sign * G^{-1} F on the active index set (Cholesky of G restricted to it);
// inactive rows of C are zero.  Sets breakdown if G is not positive definite there.  The
// factor is stored in Lc (lower triangle, row stride m, diagonal included); with reuse the
// factor stored by the previous call (same G, same active set) is taken instead.
__global__ __launch_bounds__(256) void k_bcg_solve(int m, const double *__restrict__ G, const double *__restrict__ F,
                                                   double *__restrict__ Cm, double sign, BcgState *st,
                                                   double *__restrict__ Lc, int reuse, const int32_t *stop) {
    if (stop && *stop) return;
    __shared__ double L[kMaxM][kMaxM + 1], Y[kMaxM][kMaxM + 1];
    __shared__ double inv[kMaxM], dgv[kMaxM];
    __shared__ int idx[kMaxM], pos[kMaxM];
    __shared__ int r, bad;
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    if (w == 0) {
        const bool a = lane < m && st->active[lane] != 0;
        const unsigned long long am = __ballot(a);
        const int p = __popcll(am & ((1ull << lane) - 1ull));
        if (a) idx[p] = lane;
        pos[lane] = a ? p : -1;
        if (lane == 0) {
            r = __popcll(am);
            bad = 0;
        }
    }
    __syncthreads();
    const int rr = r;
    // G on the active set (or the stored factor) and the rows of F on it
    for (int i = w; i < rr; i += 4) {
        if (lane < rr) L[i][lane] = reuse ? (lane <= i ? Lc[i * m + lane] : 0.0) : G[idx[i] * m + idx[lane]];
        if (lane < m) Y[i][lane] = F[idx[i] * m + lane];
    }
    __syncthreads();
    if (!reuse) {
        // right-looking Cholesky: step k updates the trailing lower triangle with the scaled
        // column k and finalises column k - 1
        for (int k = 0; k < rr; ++k) {
            const double v = L[k][k];
            const double dk = sqrt(v > 0.0 ? v : 1.0), ik = 1.0 / dk;
            if (k > 0 && w == 0) {  // column k - 1, which this step no longer reads
                if (lane == k - 1) L[k - 1][k - 1] = dgv[k - 1];
                else if (lane >= k && lane < rr) L[lane][k - 1] *= inv[k - 1];
            }
            const double sj = lane > k && lane < rr ? L[lane][k] * ik : 0.0;
            for (int i = k + 1 + w; i < rr; i += 4) {
                const double si = L[i][k] * ik;
                if (lane > k && lane <= i) L[i][lane] -= si * sj;
            }
            if (tid == 0) {
                inv[k] = ik;
                dgv[k] = dk;
                if (!(v > 0.0)) bad = 1;
            }
            __syncthreads();
        }
        if (rr > 0 && tid == 0) L[rr - 1][rr - 1] = dgv[rr - 1];
        if (tid == 0 && bad) st->breakdown = 1;
        __syncthreads();
        for (int i = w; i < rr; i += 4)
            if (lane <= i) Lc[i * m + lane] = L[i][lane];
    } else {
        for (int k = tid; k < rr; k += 256) inv[k] = 1.0 / L[k][k];
        __syncthreads();
    }
    // forward substitution L Z = Y, then back substitution L^T X = Z, one column per lane;
    // row q is scaled by 1 / L[q][q] where it is read and written back scaled one step later
    for (int q = 0; q < rr; ++q) {
        if (lane < m) {
            if (q > 0 && w == 0) Y[q - 1][lane] *= inv[q - 1];
            const double yq = Y[q][lane] * inv[q];
            for (int a = q + 1 + w; a < rr; a += 4) Y[a][lane] -= L[a][q] * yq;
        }
        __syncthreads();
    }
    if (rr > 0 && w == 0 && lane < m) Y[rr - 1][lane] *= inv[rr - 1];
    __syncthreads();
    for (int a = rr - 1; a >= 0; --a) {
        if (lane < m) {
            if (a < rr - 1 && w == 0) Y[a + 1][lane] *= inv[a + 1];
            const double xa = Y[a][lane] * inv[a];
            for (int q = w; q < a; q += 4) Y[q][lane] -= L[a][q] * xa;
        }
        __syncthreads();
    }
    if (rr > 0 && w == 0 && lane < m) Y[0][lane] *= inv[0];
    __syncthreads();
    if (lane < m)
        for (int j = w; j < m; j += 4) Cm[(int64_t)j * m + lane] = pos[j] >= 0 ? sign * Y[pos[j]][lane] : 0.0;
}

// M = T^{-1} scattered to M[piv[a]][piv[q]] (all other entries zero) for the upper-triangular
// T of a Cholesky-QR pass in pivot order (T[a][c] = tf(a, c) for a < c, diagonal dg): back
// substitution on the identity, one column per lane, row a scaled where it is read.
template <typename TF>
__device__ inline void tinv_scatter(int m, int r, TF tf, const double *dg, const int *piv, double *M,
                                    double (*Z)[kMaxM + 1], double *invd) {
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    for (int e = tid; e < m * m; e += 256) M[e] = 0.0;
    for (int a = w; a < r; a += 4)
        if (lane < r) Z[a][lane] = a == lane ? 1.0 : 0.0;
    for (int a = tid; a < r; a += 256) invd[a] = 1.0 / dg[a];
    __syncthreads();
    for (int a = r - 1; a >= 0; --a) {
        if (lane < r) {
            if (a < r - 1 && w == 0) Z[a + 1][lane] *= invd[a + 1];
            const double xa = Z[a][lane] * invd[a];
            for (int c = w; c < a; c += 4) Z[c][lane] -= tf(c, a) * xa;
        }
        __syncthreads();
    }
    if (r > 0 && w == 0 && lane < r) Z[0][lane] *= invd[0];
    __syncthreads();
    if (lane < r)
        for (int a = w; a <= lane; a += 4) M[(int64_t)piv[a] * m + piv[lane]] = Z[a][lane];
}

// first Cholesky-QR pass: pivoted Cholesky of W = Z^T Z with deflation, right-looking on the
// Schur complement S (kept in place of W): the pivot of step k is the first column, in column
// order, of largest remaining diagonal among those not yet taken (a NaN in the first
// candidate stays chosen); a remaining diagonal at or below kDrop^2 of the largest diagonal
// entry of W ends the factorization.  Row k of the factor: lv[k][j] = S[j][b] / sqrt(S[b][b]).
__global__ __launch_bounds__(256) void k_bcg_orth1(int m, const double *__restrict__ W, double *__restrict__ M,
                                                   BcgState *st, const int32_t *gate) {
    if (gate && *gate) return;
    __shared__ double S[kMaxM][kMaxM + 1], lv[kMaxM][kMaxM + 1];
    __shared__ double dg[kMaxM], invd[kMaxM];
    __shared__ int piv[kMaxM], act[kMaxM];
    __shared__ int rank, best;
    __shared__ double dmax;
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    for (int i = w; i < m; i += 4)
        if (lane < m) S[i][lane] = W[i * m + lane];
    if (tid < kMaxM) act[tid] = 0;
    __syncthreads();
    if (w == 0) {
        // largest diagonal entry (fmax ignores NaN: any order gives the value of a scan from 0)
        double d = lane < m ? S[lane][lane] : 0.0;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) d = fmax(d, __shfl_xor(d, o));
        if (lane == 0) {
            dmax = fmax(0.0, d);
            rank = 0;
        }
    }
    __syncthreads();
    for (int k = 0; k < m; ++k) {
        if (w == 0) {
            const bool cand = lane < m && !act[lane];
            const double d = cand ? S[lane][lane] : 0.0;
            const unsigned long long cm = __ballot(cand);
            int b = -1;
            if (cm != 0) {
                const int j0 = __ffsll(cm) - 1;
                if (isnan(S[j0][j0])) {
                    b = j0;
                } else {
                    // the largest value among the candidates that are numbers, then the first
                    // lane that holds it (at least one candidate is a number here)
                    const bool ok = cand && !isnan(d);
                    double v = ok ? d : -INFINITY;
#pragma unroll
                    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
                    b = __ffsll(__ballot(ok && d == v)) - 1;
                }
            }
            if (lane == 0) {
                if (b < 0 || !(dmax > 0.0) || !(S[b][b] > kDrop * kDrop * dmax)) {
                    best = -1;
                } else {
                    best = b;
                    act[b] = 1;
                    piv[k] = b;
                    dg[k] = sqrt(S[b][b]);
                    rank = k + 1;
                }
            }
        }
        __syncthreads();
        const int b = best;
        if (b < 0) break;
        // row k of the factor, then the Schur complement of the columns not yet taken
        const double ik = 1.0 / dg[k];
        const bool free_j = lane < m && !act[lane];
        const double sj = free_j ? S[lane][b] * ik : 0.0;
        if (w == 0 && lane < m) lv[k][lane] = lane == b ? dg[k] : sj;
        for (int i = w; i < m; i += 4)
            if (free_j && !act[i]) S[i][lane] -= (S[i][b] * ik) * sj;
        __syncthreads();
    }
    const int r = rank;
    tinv_scatter(
        m, r, [&](int a, int c) { return lv[a][piv[c]]; }, dg, piv, M, S, invd);
    if (tid == 0) st->rank = r;
    if (tid < m) {
        st->active[tid] = act[tid];
        st->piv[tid] = tid < r ? piv[tid] : -1;
    }
}

// second Cholesky-QR pass: plain Cholesky of W2 = P1^T P1 on the kept columns in pivot order
// (right-looking, as in k_bcg_solve); T = L^T.
__global__ __launch_bounds__(256) void k_bcg_orth2(int m, const double *__restrict__ W, double *__restrict__ M,
                                                   const BcgState *st, const int32_t *stop) {
    if (stop && *stop) return;
    __shared__ double L[kMaxM][kMaxM + 1], Z[kMaxM][kMaxM + 1];
    __shared__ double dg[kMaxM], inv[kMaxM];
    __shared__ int piv[kMaxM];
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63, r = st->rank;
    if (tid < r) piv[tid] = st->piv[tid];
    __syncthreads();
    for (int i = w; i < r; i += 4)
        if (lane < r) L[i][lane] = W[piv[i] * m + piv[lane]];
    __syncthreads();
    for (int k = 0; k < r; ++k) {
        const double v = L[k][k];
        const double dk = sqrt(v > 0.0 ? v : 0.0), ik = 1.0 / dk;
        if (k > 0 && w == 0 && lane >= k && lane < r) L[lane][k - 1] *= inv[k - 1];
        const double sj = lane > k && lane < r ? L[lane][k] * ik : 0.0;
        for (int i = k + 1 + w; i < r; i += 4) {
            const double si = L[i][k] * ik;
            if (lane > k && lane <= i) L[i][lane] -= si * sj;
        }
        if (tid == 0) {
            inv[k] = ik;
            dg[k] = dk;
        }
        __syncthreads();
    }
    tinv_scatter(
        m, r, [&](int a, int c) { return L[c][a]; }, dg, piv, M, Z, inv);
}

// convergence from the diagonal of R^T R
__global__ void k_bcg_conv(int m, const double *__restrict__ RR, double rtol, BcgState *st, int init,
                           const int32_t *stop) {
    if (stop && *stop) return;
    __shared__ int notconv;
    if (threadIdx.x == 0) notconv = 0;
    __syncthreads();
    const int it = init ? 0 : st->iter + 1;
    for (int j = threadIdx.x; j < m; j += blockDim.x) {
        const double rn = sqrt(RR[j * m + j]);
        st->rnorm[j] = rn;
        const int c = rn <= rtol * st->bnorm[j];
        st->conv[j] = c;
        if (init) st->first_conv[j] = c ? 0 : -1;
        else if (c && st->first_conv[j] < 0) st->first_conv[j] = it;
        if (!c) atomicOr(&notconv, 1);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        st->iter = it;
        st->all_conv = notconv ? 0 : 1;
        if (init) st->breakdown = 0;
    }
}

__global__ void k_bcg_bnorm(int m, const double *__restrict__ BB, BcgState *st) {
    for (int j = threadIdx.x; j < m; j += blockDim.x) st->bnorm[j] = sqrt(BB[j * m + j]);
}

// start of an iteration: it must not run once every column has converged, after a
// breakdown, without search directions or after max_iter iterations (the host takes the same
// decision from the state it reads after queueing the iteration)
__global__ void k_bcg_gate(BcgState *st, int32_t max_iter) {
    st->stop = (st->breakdown || st->all_conv || st->iter >= max_iter || st->rank == 0) ? 1 : 0;
}

__global__ void k_copy_rows(int64_t n, int64_t m, const int64_t *__restrict__ perm, const double *__restrict__ src,
                            int64_t lds, double *__restrict__ dst, int scatter) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * m) return;
    const int64_t i = e / m, j = e % m;
    if (scatter) dst[perm[i] * lds + j] = src[e];
    else dst[e] = src[perm[i] * lds + j];
}

struct BcgWs {
    double *Bt, *Xt, *R, *P, *Q, *Z, *P1, *part, *G, *F, *C, *Wm, *RR, *M, *Lc;
    BcgState *st;
    char *mm;
    int nblk;
    size_t bytes;
};

BcgWs bcg_layout(const DevMat &dm, int64_t m, char *base) {
    BcgWs w{};
    size_t off = 0;
    auto carve = [&](size_t bytes) {
        off = align_up(off);
        char *p = base ? base + off : nullptr;
        off += bytes;
        return p;
    };
    const size_t nm = (size_t)dm.n * m * sizeof(double), mm = (size_t)m * m * sizeof(double);
    w.nblk = (int)std::min<int64_t>(256, std::max<int64_t>(1, (dm.n + 255) / 256));
    for (double **p : {&w.Bt, &w.Xt, &w.R, &w.P, &w.Q, &w.Z, &w.P1}) *p = (double *)carve(nm);
    w.part = (double *)carve(2 * (size_t)w.nblk * mm);
    for (double **p : {&w.G, &w.F, &w.C, &w.Wm, &w.RR, &w.M, &w.Lc}) *p = (double *)carve(mm);
    w.st = (BcgState *)carve(sizeof(BcgState));
    w.mm = carve(matmul_ws_bytes(dm, m));
    w.bytes = align_up(off);
    return w;
}

}  // namespace

size_t bcg_ws_bytes(const DevMat &dm, int64_t m) { return bcg_layout(dm, m, nullptr).bytes; }

h2x_status run_block_cg_shared(const DevMat &dm, const h2x_cg_params &prm, int64_t m, const double *B, int64_t ldb,
                               double *X, int64_t ldx, char *ws, size_t ws_bytes, h2x_cg_info *info,
                               hipStream_t st) {
    if (m > kMaxM) {
        set_error("h2x_block_cg: the shared-space variant supports m <= 64");
        return H2X_EINVAL;
    }
    BcgWs w = bcg_layout(dm, m, ws);
    if (ws_bytes < w.bytes) {
        set_error("h2x_block_cg: workspace too small");
        return H2X_ENOMEM;
    }
    const int64_t n = dm.n, nm = n * m;
    const int mi = (int)m;
    const unsigned g1 = (unsigned)((nm + 255) / 256);
    const int mt = 16 * ((mi + 15) / 16), rpw = 2048 / mt;
    const unsigned gt = (unsigned)((n + rpw - 1) / rpw);
    const dim3 gs((unsigned)((m * m * kGramSplit + 255) / 256), 2);
    auto fail = [&](hipError_t e) {
        set_error(std::string("h2x_block_cg: ") + hipGetErrorString(e));
        return H2X_EHIP;
    };
    // sp: the stop flag of the state inside the iteration loop (null before it)
    const int32_t *sp = nullptr;
    auto gram2 = [&](const double *U0, const double *V0, const double *U1, const double *V1, double *G0,
                     double *G1) {
        switch ((mi + 15) / 16) {
            case 1: hipLaunchKernelGGL(k_gram_mfma<1>, dim3(w.nblk), dim3(256), 0, st, n, mi, w.nblk, U0, V0, U1, V1, w.part, sp); break;
            case 2: hipLaunchKernelGGL(k_gram_mfma<2>, dim3(w.nblk), dim3(256), 0, st, n, mi, w.nblk, U0, V0, U1, V1, w.part, sp); break;
            case 3: hipLaunchKernelGGL(k_gram_mfma<3>, dim3(w.nblk), dim3(256), 0, st, n, mi, w.nblk, U0, V0, U1, V1, w.part, sp); break;
            default: hipLaunchKernelGGL(k_gram_mfma<4>, dim3(w.nblk), dim3(256), 0, st, n, mi, w.nblk, U0, V0, U1, V1, w.part, sp); break;
        }
        hipLaunchKernelGGL(k_gram_sum, dim3(gs.x, U1 ? 2 : 1), dim3(256), 0, st, mi, w.nblk, (const double *)w.part,
                           G0, G1, sp);
    };
    // out = beta Yin + alpha U C, and with U2 also out2 = beta Yin2 + alpha2 U2 C in the same launch
    auto tsmm = [&](const double *U, const double *Cm, const double *Yin, double *out, double alpha, double beta,
                    const double *U2 = nullptr, const double *Yin2 = nullptr, double *out2 = nullptr,
                    double alpha2 = 0.0) {
        const dim3 g(gt, U2 ? 2 : 1);
        switch (mt) {
            case 16: hipLaunchKernelGGL(k_tsmm<16>, g, dim3(256), 0, st, n, mi, U, Cm, Yin, out, alpha, beta, U2, Yin2, out2, alpha2, sp); break;
            case 32: hipLaunchKernelGGL(k_tsmm<32>, g, dim3(256), 0, st, n, mi, U, Cm, Yin, out, alpha, beta, U2, Yin2, out2, alpha2, sp); break;
            case 48: hipLaunchKernelGGL(k_tsmm<48>, g, dim3(256), 0, st, n, mi, U, Cm, Yin, out, alpha, beta, U2, Yin2, out2, alpha2, sp); break;
            default: hipLaunchKernelGGL(k_tsmm<64>, g, dim3(256), 0, st, n, mi, U, Cm, Yin, out, alpha, beta, U2, Yin2, out2, alpha2, sp); break;
        }
    };
    // the second solve of an iteration has the same G and active set: it takes the factor
    auto solve = [&](double sign, int reuse) {
        hipLaunchKernelGGL(k_bcg_solve, dim3(1), dim3(256), 0, st, mi, (const double *)w.G, (const double *)w.F, w.C,
                           sign, w.st, w.Lc, reuse, sp);
    };
    auto orth = [&](const double *Zs) {
        gram2(Zs, Zs, nullptr, nullptr, w.Wm, nullptr);
        hipLaunchKernelGGL(k_bcg_orth1, dim3(1), dim3(256), 0, st, mi, (const double *)w.Wm, w.M, w.st, sp);
        tsmm(Zs, w.M, nullptr, w.P1, 1.0, 0.0);
        gram2(w.P1, w.P1, nullptr, nullptr, w.Wm, nullptr);
        hipLaunchKernelGGL(k_bcg_orth2, dim3(1), dim3(256), 0, st, mi, (const double *)w.Wm, w.M,
                           (const BcgState *)w.st, sp);
        tsmm(w.P1, w.M, nullptr, w.P, 1.0, 0.0);
    };

    hipLaunchKernelGGL(k_copy_rows, dim3(g1), dim3(256), 0, st, n, m, dm.perm, B, ldb, w.Bt, 0);
    hipLaunchKernelGGL(k_copy_rows, dim3(g1), dim3(256), 0, st, n, m, dm.perm, (const double *)X, ldx, w.Xt, 0);
    hipError_t e = hipMemcpyAsync(w.R, w.Bt, nm * sizeof(double), hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess) e = run_matmul(dm, m, -1.0, w.Xt, m, 1.0, w.R, m, true, w.mm, st);
    if (e != hipSuccess) return fail(e);
    gram2(w.Bt, w.Bt, w.R, w.R, w.G, w.RR);
    hipLaunchKernelGGL(k_bcg_bnorm, dim3(1), dim3(64), 0, st, mi, (const double *)w.G, w.st);
    hipLaunchKernelGGL(k_bcg_conv, dim3(1), dim3(64), 0, st, mi, (const double *)w.RR, prm.rtol, w.st, 1,
                       (const int32_t *)nullptr);
    orth(w.R);

    // two pinned host copies of the state: the host reads the state after iteration it while
    // iteration it + 1 is already queued, so the device does not idle at each decision
    struct HostCopies {
        BcgState *p = nullptr;
        hipEvent_t ev[2] = {nullptr, nullptr};
        ~HostCopies() {
            for (hipEvent_t x : ev)
                if (x) (void)hipEventDestroy(x);
            if (p) (void)hipHostFree(p);
        }
    } hc;
    e = hipHostMalloc((void **)&hc.p, 2 * sizeof(BcgState), hipHostMallocDefault);
    for (int q = 0; q < 2 && e == hipSuccess; ++q) e = hipEventCreateWithFlags(&hc.ev[q], hipEventDisableTiming);
    auto snapshot = [&](int slot) {
        hipError_t r = hipMemcpyAsync(&hc.p[slot], w.st, sizeof(BcgState), hipMemcpyDeviceToHost, st);
        return r == hipSuccess ? hipEventRecord(hc.ev[slot], st) : r;
    };
    if (e == hipSuccess) e = snapshot(0);
    if (e != hipSuccess) return fail(e);

    sp = &w.st->stop;
    int32_t status = H2X_OK;
    for (int32_t it = 0;; ++it) {
        // iteration it + 1; its kernels return at once when the gate stops it, which happens
        // exactly when the host stops below
        hipLaunchKernelGGL(k_bcg_gate, dim3(1), dim3(1), 0, st, w.st, prm.max_iter);
        e = run_matmul(dm, m, 1.0, w.P, m, 0.0, w.Q, m, true, w.mm, st, nullptr, sp);
        if (e != hipSuccess) return fail(e);
        gram2(w.P, w.Q, w.P, w.R, w.G, w.F);  // G = P^T A P, F = P^T R
        solve(1.0, 0);
        tsmm(w.P, w.C, w.Xt, w.Xt, 1.0, 1.0,  // X += P Lambda
             w.Q, w.R, w.R, -1.0);            // R -= Q Lambda
        gram2(w.Q, w.R, w.R, w.R, w.F, w.RR);   // F = (A P)^T R, RR = R^T R
        hipLaunchKernelGGL(k_bcg_conv, dim3(1), dim3(64), 0, st, mi, (const double *)w.RR, prm.rtol, w.st, 0, sp);
        solve(-1.0, 1);
        tsmm(w.P, w.C, w.R, w.Z, 1.0, 1.0);     // Z = R + P Psi
        orth(w.Z);
        e = snapshot((it + 1) & 1);
        // the state after iteration it
        if (e == hipSuccess) e = hipEventSynchronize(hc.ev[it & 1]);
        if (e != hipSuccess) return fail(e);
        const BcgState &hs = hc.p[it & 1];
        if (hs.breakdown) {
            status = H2X_EBREAKDOWN;
            break;
        }
        if (hs.all_conv) break;
        if (it >= prm.max_iter || hs.rank == 0) {
            status = H2X_ENOCONV;
            break;
        }
    }
    hipLaunchKernelGGL(k_copy_rows, dim3(g1), dim3(256), 0, st, n, m, dm.perm, (const double *)w.Xt, ldx, X, 1);
    BcgState hs{};
    e = hipMemcpyAsync(&hs, w.st, sizeof(BcgState), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return fail(e);
    if (info) {
        info->iters = hs.iter;
        info->status = status;
        info->outer_iters = 0;
        if (info->sys_iters) info->sys_iters[0] = hs.iter;
        for (int64_t j = 0; j < m; ++j) {
            const double bn = hs.bnorm[j], rn = hs.rnorm[j];
            if (info->col_relres) info->col_relres[j] = bn > 0 ? rn / bn : rn;
            if (info->col_iters) info->col_iters[j] = hs.first_conv[j] >= 0 ? hs.first_conv[j] : hs.iter;
            if (info->col_status) info->col_status[j] = hs.conv[j] ? 0 : (status == H2X_EBREAKDOWN ? 1 : 2);
        }
    }
    return H2X_OK;
}

}  // namespace h2x
