// Matrix-core kernels of the adjoint product Y = beta Y + alpha A^T X (FP64
// operator in the matrix-core layout, k = 64 or k <= 32).
//
// Both kernels accumulate a 64-row x 16*NJ-column tile per work-group (wave w
// owns rows 16w..16w+15) as a sum of terms A_q B_q, where each term's left factor
// (up to 64 x 64) and right factor (up to 64 x 16*NJ) are staged through LDS: the
// next term is loaded into registers with coalesced loads while the matrix cores
// work on the current one, then written to LDS between two barriers.
//
// k_coupling_adj_mfma: one work-group per column cluster s, terms = the
//   admissible blocks b = (t, s) of its column list, A = S_b^T (staged from the
//   stored operand order of S_b, transposed), B = x_t; writes y_s.
// k_leaf_adj_mfma: one work-group per leaf s (and 64-row chunk of it), terms =
//   the basis term (A = V_s, B = y_s) and the near blocks (t, s) of its column
//   list (A = N_ts^T, which is exactly the stored transposed near block, B = X|_t
//   from the tree-ordered copy of X); writes Y|_s = beta Y|_s + alpha sum.
#pragma once

#include "device.hpp"
#include "types.hpp"

namespace h2x {
namespace adj {

typedef double dbl4 __attribute__((ext_vector_type(4)));

constexpr int LDA = 65;  // LDS row of the left factor

template <int NJ>
struct Tiles {
    static constexpr int MC = 16 * NJ, LDB = MC + 1;
    double a[64 * LDA];
    double b[2][64 * LDB];
};

// acc += A B over kpad (multiple of 4) contraction steps; waves whose rows all lie
// at or beyond `rows` skip the multiplications
template <int NJ>
__device__ inline void mma(const double *As, const double *Bs, int kpad, int rows, dbl4 *acc) {
    constexpr int LDB = 16 * NJ + 1;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, lr = lane & 15, g = lane >> 4;
    if (16 * w >= rows) return;
    const double *arow = As + (16 * w + lr) * LDA + g;
    const double *bcol = Bs + g * LDB + lr;
    for (int kk = 0; kk < kpad; kk += 4) {
        const double a = arow[kk];
#pragma unroll
        for (int J = 0; J < NJ; ++J)
            acc[J] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bcol[kk * LDB + 16 * J], acc[J], 0, 0, 0);
    }
}

// storage index e of a k x k coupling matrix -> (nu, mu) (inverse of s_index, layouts 0 and 1)
__device__ inline void s_coords(int swz, int k, int e, int &nu, int &mu) {
    if (swz == 0) {
        nu = e / k;
        mu = e - nu * k;
        return;
    }
    const int h = e & 1, lane = (e >> 1) & 63, rest = e >> 7, k8 = k >> 3;
    const int kk2 = rest % k8, I = rest / k8;
    nu = 16 * I + (lane & 15);
    mu = 8 * kk2 + 4 * h + (lane >> 4);
}

template <int NJ>
__global__ __launch_bounds__(256) void k_coupling_adj_mfma(int k, int swz, int64_t m, int32_t C,
                                                           const int64_t *__restrict__ cptr,
                                                           const int64_t *__restrict__ cblk,
                                                           const int32_t *__restrict__ adm_row,
                                                           const double *__restrict__ S,
                                                           const double *__restrict__ xh, double *__restrict__ yh,
                                                           int64_t ldh) {
    constexpr int MC = 16 * NJ, LDB = MC + 1, XPT = 64 * MC / 256;
    __shared__ Tiles<NJ> sm;
    const int32_t per_xcd = (C + 7) / 8;
    const int32_t s = (blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
    if (s >= C) return;
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63, lr = lane & 15, g = lane >> 4;
    const int64_t j0 = (int64_t)blockIdx.y * MC;
    const int mc = (int)min<int64_t>(MC, m - j0);
    const int kk = k * k, kpad = (k + 3) & ~3;
    const int64_t q0 = cptr[s], q1 = cptr[s + 1];
    dbl4 acc[NJ];
#pragma unroll
    for (int J = 0; J < NJ; ++J) acc[J] = dbl4{0.0, 0.0, 0.0, 0.0};
    if (q1 > q0) {
        for (int e = tid; e < 64 * LDA; e += 256) sm.a[e] = 0.0;  // padding rows and columns stay zero
        double sv[16], xv[XPT];
        auto load = [&](int64_t q) {
            const int64_t b = cblk[q];
            const double *Sb = S + b * kk;
#pragma unroll
            for (int u = 0; u < 16; ++u) {
                const int e = tid + 256 * u;
                sv[u] = e < kk ? __builtin_nontemporal_load(Sb + e) : 0.0;
            }
            const double *src = xh + (int64_t)adm_row[b] * k * ldh + j0;
#pragma unroll
            for (int u = 0; u < XPT; ++u) {
                const int e = tid + 256 * u, r = e / MC, c = e % MC;
                xv[u] = (r < k && c < mc) ? src[(int64_t)r * ldh + c] : 0.0;
            }
        };
        auto store = [&](int buf) {
#pragma unroll
            for (int u = 0; u < 16; ++u) {
                const int e = tid + 256 * u;
                if (e < kk) {
                    int nu, mu;
                    s_coords(swz, k, e, nu, mu);
                    sm.a[mu * LDA + nu] = sv[u];  // A = S_b^T
                }
            }
#pragma unroll
            for (int u = 0; u < XPT; ++u) {
                const int e = tid + 256 * u, r = e / MC, c = e % MC;
                sm.b[buf][r * LDB + c] = xv[u];
            }
        };
        __syncthreads();
        load(q0);
        store(0);
        __syncthreads();
        for (int64_t q = q0; q < q1; ++q) {
            const int buf = (int)((q - q0) & 1);
            const bool more = q + 1 < q1;
            if (more) load(q + 1);
            mma<NJ>(sm.a, sm.b[buf], kpad, k, acc);
            __syncthreads();
            if (more) store(buf ^ 1);
            __syncthreads();
        }
    }
#pragma unroll
    for (int J = 0; J < NJ; ++J) {
        const int col = 16 * J + lr;
        if (col < mc)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = 16 * w + g + 4 * r;
                if (row < k) yh[((int64_t)s * k + row) * ldh + j0 + col] = acc[J][r];
            }
    }
}

template <int NJ>
__global__ __launch_bounds__(256) void k_leaf_adj_mfma(int k, int64_t m, int32_t L, const int32_t *__restrict__ leaves,
                                                       const int32_t *__restrict__ first,
                                                       const int32_t *__restrict__ size,
                                                       const int64_t *__restrict__ perm, const double *__restrict__ V,
                                                       const double *__restrict__ yh, int64_t ldh,
                                                       const int64_t *__restrict__ ncptr,
                                                       const int64_t *__restrict__ ncblk,
                                                       const int32_t *__restrict__ near_row,
                                                       const int64_t *__restrict__ near_off,
                                                       const double *__restrict__ Nt, const double *__restrict__ Xt,
                                                       int64_t ldxt, double alpha, double beta,
                                                       double *__restrict__ Y, int64_t ldy) {
    constexpr int MC = 16 * NJ, LDB = MC + 1, XPT = 64 * MC / 256;
    __shared__ Tiles<NJ> sm;
    const int32_t per_xcd = (L + 7) / 8;
    const int32_t l = (blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
    if (l >= L) return;
    const int32_t s = leaves[l];
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63, lr = lane & 15, g = lane >> 4;
    const int64_t j0 = (int64_t)blockIdx.y * MC;
    const int mc = (int)min<int64_t>(MC, m - j0);
    const int ns = size[s];
    const int64_t fs = first[s];
    const int64_t q0 = ncptr[l];
    const int nitems = (int)(ncptr[l + 1] - q0) + 1;
    for (int c0 = 0; c0 < ns; c0 += 64) {
        const int cc = min(64, ns - c0);
        dbl4 acc[NJ];
#pragma unroll
        for (int J = 0; J < NJ; ++J) acc[J] = dbl4{0.0, 0.0, 0.0, 0.0};
        double av[16], xv[XPT];
        // term e, contraction chunk ch (64 wide): A (cc x K rows of this chunk), B (K x 16*NJ);
        // returns the chunk's contraction length, ktot receives the term's
        auto load = [&](int e, int ch, int &ktot) {
            const double *A, *Bm;
            int64_t lda, ldb;
            if (e == 0) {  // basis term: A = V_s rows, B = y_s
                A = V + (fs + c0) * k;
                lda = k;
                ktot = k;
                Bm = yh + (int64_t)s * k * ldh + j0;
                ldb = ldh;
            } else {  // near block (t, s): A = N_ts^T rows, B = X|_t
                const int64_t q = ncblk[q0 + e - 1];
                const int32_t t = near_row[q];
                const int nt = size[t];
                A = Nt + near_off[q] + (int64_t)c0 * pad_rows(nt);
                lda = pad_rows(nt);
                ktot = nt;
                Bm = Xt + (int64_t)first[t] * ldxt + j0;
                ldb = ldxt;
            }
            const int kc0 = 64 * ch, Kc = min(64, ktot - kc0);
            A += kc0;
            Bm += (int64_t)kc0 * ldb;
#pragma unroll
            for (int u = 0; u < 16; ++u) {
                const int e2 = tid + 256 * u, r = e2 >> 6, c = e2 & 63;
                av[u] = (r < cc && c < Kc) ? A[(int64_t)r * lda + c] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < XPT; ++u) {
                const int e2 = tid + 256 * u, r = e2 / MC, c = e2 % MC;
                xv[u] = (r < Kc && c < mc) ? Bm[(int64_t)r * ldb + c] : 0.0;
            }
            return Kc;
        };
        auto store = [&](int buf) {
#pragma unroll
            for (int u = 0; u < 16; ++u) {
                const int e2 = tid + 256 * u, r = e2 >> 6, c = e2 & 63;
                sm.a[r * LDA + c] = av[u];
            }
#pragma unroll
            for (int u = 0; u < XPT; ++u) {
                const int e2 = tid + 256 * u, r = e2 / MC, c = e2 % MC;
                sm.b[buf][r * LDB + c] = xv[u];
            }
        };
        __syncthreads();
        int e = 0, ch = 0, ktot = 0;
        int klen = load(0, 0, ktot);
        store(0);
        __syncthreads();
        for (int it = 0;; ++it) {
            const int buf = it & 1;
            int en = e, chn = ch + 1;
            if (64 * chn >= ktot) {
                en = e + 1;
                chn = 0;
            }
            const bool more = en < nitems;
            int ktot_next = 0, klen_next = 0;
            if (more) klen_next = load(en, chn, ktot_next);
            mma<NJ>(sm.a, sm.b[buf], (klen + 3) & ~3, cc, acc);
            __syncthreads();
            if (more) store(buf ^ 1);
            __syncthreads();
            if (!more) break;
            e = en;
            ch = chn;
            ktot = ktot_next;
            klen = klen_next;
        }
#pragma unroll
        for (int J = 0; J < NJ; ++J) {
            const int col = 16 * J + lr;
            if (col < mc)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int row = 16 * w + g + 4 * r;
                    if (row < cc) {
                        double *y = &Y[perm[fs + c0 + row] * ldy + j0 + col];
                        const double v = alpha * acc[J][r];
                        *y = (beta == 0.0) ? v : beta * *y + v;
                    }
                }
        }
    }
}


// ---- gradients: 64 x 64 tiles D = A B^T with the contraction over the m columns ----
//
// A: arows x m (row stride lda), B: brows x m (row stride ldb), both in FP64;
// staged through LDS in chunks of CW columns (16, 32 or 64: the tiles are sized to the
// chunk, so a small m leaves room for more work-groups per CU).  Wave w owns rows
// 16w..16w+15 of D, acc[J] columns 16J..16J+15; register r of lane l holds row
// 16w + l/16 + 4r, column 16J + l%16.
template <int CW>
struct GradTiles {
    static constexpr int LD = CW + 1;
    double a[64 * LD];
    double b[64 * LD];
};

template <int CW>
__device__ inline void outer_tile(GradTiles<CW> &sm, const double *A, int64_t lda, int arows, const double *B,
                                  int64_t ldb, int brows, int64_t m, dbl4 *acc) {
    constexpr int LD = GradTiles<CW>::LD, EPT = 64 * CW / 256;  // elements per thread
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63, lr = lane & 15, g = lane >> 4;
#pragma unroll
    for (int J = 0; J < 4; ++J) acc[J] = dbl4{0.0, 0.0, 0.0, 0.0};
    for (int64_t j0 = 0; j0 < m; j0 += CW) {
        const int mc = (int)min<int64_t>(CW, m - j0);
        double av[EPT], bv[EPT];
#pragma unroll
        for (int u = 0; u < EPT; ++u) {
            const int e = tid + 256 * u, r = e / CW, c = e % CW;
            av[u] = (r < arows && c < mc) ? A[(int64_t)r * lda + j0 + c] : 0.0;
            bv[u] = (r < brows && c < mc) ? B[(int64_t)r * ldb + j0 + c] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < EPT; ++u) {
            const int e = tid + 256 * u, r = e / CW, c = e % CW;
            sm.a[r * LD + c] = av[u];
            sm.b[r * LD + c] = bv[u];
        }
        __syncthreads();
        if (16 * w < arows) {
            const double *arow = sm.a + (16 * w + lr) * LD + g;
            const int kpad = (mc + 3) & ~3;
            for (int kk = 0; kk < kpad; kk += 4) {
                const double a = arow[kk];
#pragma unroll
                for (int J = 0; J < 4; ++J)
                    acc[J] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, sm.b[(16 * J + lr) * LD + kk + g], acc[J], 0, 0, 0);
            }
        }
    }
}

// d g / d ell = (r / ell^2) exp(-r / ell) between two points staged in LDS
__device__ inline double dg_dell_mc(double inv_ell, double inv_ell2, const double *a, const double *b) {
    const double dx = a[0] - b[0], dy = a[1] - b[1], dz = a[2] - b[2];
    const double r = sqrt(dx * dx + dy * dy + dz * dz);
    return (r * inv_ell2) * exp(-r * inv_ell);
}

// coordinates of up to 64 points (3 doubles each) into LDS
__device__ inline void stage_points(double (*dst)[3], const double *src, int count) {
    for (int e = threadIdx.x; e < 3 * 64; e += blockDim.x) {
        const int i = e / 3, d = e - 3 * i;
        dst[i][d] = i < count ? src[3 * i + d] : 0.0;
    }
}

// sum over the work-group of one value per thread, in a fixed order
__device__ inline double block_sum(double v) {
    __shared__ double red[256];
    red[threadIdx.x] = v;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
}

// one admissible block per work-group: D = scale * dyhat_t xhat_s^T (k x k, k <= 64); dS_b = D
// if requested (row-major); part[b] = sum of (dg/dell)(xi_t,nu, xi_s,mu) D[nu][mu] (0 unless
// want_dell)
template <int CW>
__global__ __launch_bounds__(256) void k_grad_S_mfma(int k, int64_t m, const int32_t *__restrict__ adm_row,
                                                     const int32_t *__restrict__ adm_col,
                                                     const double *__restrict__ nodes, int kernel, double ell,
                                                     const double *__restrict__ dh, const double *__restrict__ xh,
                                                     int64_t ldh, double scale, int want_dell,
                                                     double *__restrict__ dS, double *__restrict__ part) {
    __shared__ GradTiles<CW> sm;
    __shared__ double pt[64][3], ps[64][3];
    const int64_t b = blockIdx.x;
    const int32_t t = adm_row[b], s = adm_col[b];
    const bool exp_kernel = kernel == H2X_KERNEL_EXP && want_dell;
    if (exp_kernel) {
        stage_points(pt, nodes + (int64_t)t * k * 3, k);
        stage_points(ps, nodes + (int64_t)s * k * 3, k);
    }
    dbl4 acc[4];
    outer_tile(sm, dh + (int64_t)t * k * ldh, ldh, k, xh + (int64_t)s * k * ldh, ldh, k, m, acc);
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63, lr = lane & 15, g = lane >> 4;
    const double inv_ell = 1.0 / ell, inv_ell2 = inv_ell * inv_ell;
    double gsum = 0.0;
#pragma unroll
    for (int J = 0; J < 4; ++J) {
        const int mu = 16 * J + lr;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int nu = 16 * w + g + 4 * r;
            if (nu < k && mu < k) {
                const double d = scale * acc[J][r];
                if (dS) dS[b * k * k + nu * k + mu] = d;
                if (exp_kernel) gsum += dg_dell_mc(inv_ell, inv_ell2, pt[nu], ps[mu]) * d;
            }
        }
    }
    if (want_dell) {  // work-group-uniform: the sum and its barriers only when d ell is wanted
        const double tot = block_sum(gsum);
        if (tid == 0) part[b] = tot;
    }
}

// one near-field block per work-group: D = scale * dY|_t X|_s^T (tree-ordered dY, X); dN_b = D
// (row-major |t| x |s|) if requested; part[q] = sum of (dg/dell)(x_i, x_j) D[i][j] (0 unless
// want_dell)
template <int CW>
__global__ __launch_bounds__(256) void k_grad_N_mfma(int64_t m, const int32_t *__restrict__ near_row,
                                                     const int32_t *__restrict__ near_col,
                                                     const int64_t *__restrict__ near_off_rm,
                                                     const int32_t *__restrict__ first,
                                                     const int32_t *__restrict__ size,
                                                     const double *__restrict__ pts, int kernel, double ell,
                                                     const double *__restrict__ dYt, const double *__restrict__ Xt,
                                                     int64_t ldt, double scale, int want_dell,
                                                     double *__restrict__ dN, double *__restrict__ part) {
    __shared__ GradTiles<CW> sm;
    __shared__ double pt[64][3], ps[64][3];
    const int64_t q = blockIdx.x;
    const int32_t t = near_row[q], s = near_col[q];
    const int nt = size[t], ns = size[s];
    const int64_t ft = first[t], fs = first[s];
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63, lr = lane & 15, g = lane >> 4;
    const bool exp_kernel = kernel == H2X_KERNEL_EXP && want_dell;
    const double inv_ell = 1.0 / ell, inv_ell2 = inv_ell * inv_ell;
    double gsum = 0.0;
    for (int i0 = 0; i0 < nt; i0 += 64)
        for (int c0 = 0; c0 < ns; c0 += 64) {
            const int ic = min(64, nt - i0), cc = min(64, ns - c0);
            if (exp_kernel) {
                stage_points(pt, pts + 3 * (ft + i0), ic);
                stage_points(ps, pts + 3 * (fs + c0), cc);
            }
            dbl4 acc[4];
            outer_tile(sm, dYt + (ft + i0) * ldt, ldt, ic, Xt + (fs + c0) * ldt, ldt, cc, m, acc);
#pragma unroll
            for (int J = 0; J < 4; ++J) {
                const int c = 16 * J + lr;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int i = 16 * w + g + 4 * r;
                    if (i < ic && c < cc) {
                        const double d = scale * acc[J][r];
                        if (dN) dN[near_off_rm[q] + (int64_t)(i0 + i) * ns + c0 + c] = d;
                        if (exp_kernel) gsum += dg_dell_mc(inv_ell, inv_ell2, pt[i], ps[c]) * d;
                    }
                }
            }
            __syncthreads();  // the staged points of this tile are read before the next overwrites them
        }
    if (want_dell) {
        const double tot = block_sum(gsum);
        if (tid == 0) part[q] = tot;
    }
}

// ---- d ell without the per-block tiles (rank 64) ----
//
// The coupling term of d ell is sum_t <dyhat_t, sum_{(t,s) in C_t} G_b xhat_s> with
// G_b[nu][mu] = dg/dell(xi_t,nu, xi_s,mu) = (r / ell^2) S_b[nu][mu] for the exponential kernel
// (r the distance of the two interpolation nodes): the coupling product with G_b in place of
// S_b.  One work-group per row cluster and slab of 16 NJ columns, as in the coupling kernel;
// each lane streams its operand entries of S_b (row 16 w + l % 16, columns 4 k + l / 16) in
// the stored operand order and scales them by r / ell^2 (the row's node in registers, the
// column cluster's nodes staged in LDS with x-hat_s, double-buffered), so no k x k tile of D
// is stored.  The work-group's partial sum of the dot product with dyhat_t goes to
// part[slot] (a fixed order); the sums are added in a fixed order afterwards.
template <int NJ>
__global__ __launch_bounds__(256) void k_dell_coupling(int64_t m, int32_t C, int32_t rows_per_xcd,
                                                       const int32_t *__restrict__ order,
                                                       const int64_t *__restrict__ adm_ptr,
                                                       const int32_t *__restrict__ adm_col,
                                                       const double *__restrict__ nodes, double inv_ell2,
                                                       const double *__restrict__ S,
                                                       const double *__restrict__ xh,
                                                       const double *__restrict__ dh, int64_t ldh,
                                                       double *__restrict__ part) {
    constexpr int MC = 16 * NJ, LDX = MC + 1;
    __shared__ double xs[2][64 * LDX];
    __shared__ double ns[2][64 * 3];
    const int nslab = (int)((m + MC - 1) / MC), qx = blockIdx.x >> 3;
    const int slot = (blockIdx.x & 7) * rows_per_xcd + qx / nslab;
    double mine = 0.0;
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63, lr = lane & 15, lq = lane >> 4;
    if (slot < C) {
        const int32_t t = order[slot];
        const int64_t j0 = (int64_t)(qx % nslab) * MC;
        const int mc = (int)min<int64_t>(MC, m - j0);
        const int64_t b0 = adm_ptr[t], b1 = adm_ptr[t + 1];
        // the lane's row node xi_t,nu, nu = 16 w + l % 16
        const double *nt = nodes + ((int64_t)t * 64 + 16 * w + lr) * 3;
        const double px = nt[0], py = nt[1], pz = nt[2];
        dbl4 acc[NJ];
#pragma unroll
        for (int J = 0; J < NJ; ++J) acc[J] = dbl4{0.0, 0.0, 0.0, 0.0};
        if (b1 > b0) {
            constexpr int XPT = (64 * MC) / 256;
            double xv[XPT], nv;
            auto load = [&](int32_t s) {
                const double *src = xh + (int64_t)s * 64 * ldh + j0;
#pragma unroll
                for (int u = 0; u < XPT; ++u) {
                    const int e = tid + 256 * u, r = e / MC, c = e % MC;
                    xv[u] = src[(int64_t)r * ldh + (c < mc ? c : 0)];
                }
                nv = nodes[(int64_t)s * 64 * 3 + min(tid, 191)];
            };
            auto store = [&](int buf) {
#pragma unroll
                for (int u = 0; u < XPT; ++u) {
                    const int e = tid + 256 * u, r = e / MC, c = e % MC;
                    xs[buf][r * LDX + c] = c < mc ? xv[u] : 0.0;
                }
                if (tid < 192) ns[buf][tid] = nv;
            };
            // S_b in the coupling's operand order: lane l holds S[16 w + l % 16][4 kk + l / 16]
            // for k-steps kk = 2 q, 2 q + 1 as one 16-byte pair (q = 0..7)
            typedef double dbl2 __attribute__((ext_vector_type(2)));
            dbl2 sa[8], sn[8];
            auto load_s = [&](int64_t b, dbl2 *dst) {
                const __amdgpu_buffer_rsrc_t rs = buf_rsrc(S + b * 64 * 64, 64 * 64 * 8);
#pragma unroll
                for (int q = 0; q < 8; ++q)
                    dst[q] = __builtin_bit_cast(dbl2, buf_ld16<kBufNT>(rs, 16u * (w * 8 * 64 + q * 64 + lane)));
            };
            auto multiply = [&](int buf) {
                const double *xb = xs[buf], *nb = ns[buf];
#pragma unroll
                for (int kk = 0; kk < 16; ++kk) {
                    const int mu = 4 * kk + lq;
                    const double dx = px - nb[3 * mu], dy = py - nb[3 * mu + 1], dz = pz - nb[3 * mu + 2];
                    const double r = sqrt(dx * dx + dy * dy + dz * dz);
                    const double a = (r * inv_ell2) * ((kk & 1) ? sa[kk >> 1].y : sa[kk >> 1].x);
#pragma unroll
                    for (int J = 0; J < NJ; ++J)
                        acc[J] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, xb[mu * LDX + 16 * J + lr], acc[J], 0, 0, 0);
                }
            };
            load(adm_col[b0]);
            load_s(b0, sa);
            store(0);
            __syncthreads();
            // every load is unconditional and the last block is peeled off, as in the coupling
            for (int64_t b = b0; b + 1 < b1; ++b) {
                const int buf = (int)((b - b0) & 1);
                load(adm_col[b + 1]);
                load_s(b + 1, sn);
                multiply(buf);
                store(buf ^ 1);
#pragma unroll
                for (int q = 0; q < 8; ++q) sa[q] = sn[q];
                __syncthreads();
            }
            multiply((int)((b1 - 1 - b0) & 1));
        }
        // <dyhat_t, y'_t> over the slab: lane l, register r -> row 16 w + l / 16 + 4 r, column 16 J + l % 16
#pragma unroll
        for (int J = 0; J < NJ; ++J) {
            const int col = 16 * J + lr;
            if (col < mc)
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    mine += acc[J][r] * dh[((int64_t)t * 64 + 16 * w + lq + 4 * r) * ldh + j0 + col];
        }
    }
    const double tot = block_sum(mine);
    if (tid == 0) part[blockIdx.x] = tot;
}

}  // namespace adj
}  // namespace h2x
