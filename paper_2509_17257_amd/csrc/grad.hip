// Differentiation of the H^2 product (FP64 operators).
//
// Adjoint product Y = beta Y + alpha A^T X: the forward transformation of X,
// then for every column cluster s its column list (every admissible block
// (t, s): y_s += S_b^T x_t), the downward transfer pass, and per leaf s the
// basis term plus every near-field block (t, s) of its column list,
// Y|_s += N_ts^T X|_t.  Each column cluster owns its output, as each row
// cluster does in the product.
//
// Gradients of L = <dY, A X> (sum over all entries):
//   dS_b = dyhat_t xhat_s^T     (xhat, dyhat: forward transformations of X, dY)
//   dN_b = dY|_t X|_s^T
//   dell = sum_b <dS_b / dell, dS_b> + sum_b <dN_b / dell, dN_b>,
//          dg/dell = (r / ell^2) exp(-r / ell), evaluated where it is needed.
// Per-block partial sums of dell are reduced in a fixed order.
#include <cmath>
#include <type_traits>

#include "adjoint_mfma.hpp"
#include "device.hpp"
#include "leaf_cat.hpp"
#include "types.hpp"

namespace h2x {

namespace {

constexpr int TR = 64;  // tile of the transposed coupling / near kernels
constexpr int TC = 32;

__device__ inline double dg_dell(int kernel, double ell, const double *a, const double *b) {
    if (kernel != H2X_KERNEL_EXP) return 0.0;
    const double dx = a[0] - b[0], dy = a[1] - b[1], dz = a[2] - b[2];
    const double r = sqrt(dx * dx + dy * dy + dz * dz);
    return (r / (ell * ell)) * exp(-r / ell);
}

__device__ inline void tile_fma(double acc[8], const double (*As)[TR + 1], const double (*Bs)[TC], int kc, int rg,
                                int j) {
    for (int c = 0; c < kc; ++c) {
        const double b = Bs[c][j];
#pragma unroll
        for (int q = 0; q < 8; ++q) acc[q] += As[rg + 8 * q][c] * b;
    }
}

// y_s = sum over the column list of s of S_b^T x_{t(b)}  (every cluster s)
__global__ __launch_bounds__(256) void k_coupling_adj(int k, int64_t m, const int64_t *__restrict__ cptr,
                                                      const int64_t *__restrict__ cblk,
                                                      const int32_t *__restrict__ adm_row,
                                                      const double *__restrict__ S, int swz,
                                                      const double *__restrict__ xh, double *__restrict__ yh,
                                                      int64_t ldh) {
    __shared__ double As[TR][TR + 1];
    __shared__ double Bs[TR][TC];
    const int32_t s = blockIdx.x;
    const int64_t j0 = (int64_t)blockIdx.y * TC;
    const int mc = (int)min<int64_t>(TC, m - j0);
    const int tid = threadIdx.x, rg = tid >> 5, j = tid & 31;
    for (int n0 = 0; n0 < k; n0 += TR) {
        double acc[8] = {};
        for (int64_t q = cptr[s]; q < cptr[s + 1]; ++q) {
            const int64_t b = cblk[q];
            const int32_t t = adm_row[b];
            const double *Sb = S + b * k * k;
            for (int u0 = 0; u0 < k; u0 += TR) {
                const int uc = min(TR, k - u0);
                // As[mu][nu] = S_b[nu][mu]
                for (int e = tid; e < TR * TR; e += 256) {
                    const int mu = e / TR, nu = e % TR;
                    As[mu][nu] = (nu < uc && n0 + mu < k) ? Sb[s_index(swz, k, u0 + nu, n0 + mu)] : 0.0;
                }
                for (int e = tid; e < TR * TC; e += 256) {
                    const int nu = e / TC, jj = e % TC;
                    Bs[nu][jj] = (nu < uc && jj < mc) ? xh[((int64_t)t * k + u0 + nu) * ldh + j0 + jj] : 0.0;
                }
                __syncthreads();
                tile_fma(acc, As, Bs, uc, rg, j);
                __syncthreads();
            }
        }
        if (j < mc)
            for (int q = 0; q < 8; ++q) {
                const int mu = n0 + rg + 8 * q;
                if (mu < k) yh[((int64_t)s * k + mu) * ldh + j0 + j] = acc[q];
            }
    }
}

// Y|_s = beta Y|_s + alpha (V_s y_s + sum over the near column list of s of N_ts^T X|_t)
__global__ __launch_bounds__(256) void k_leaf_near_adj(int k, int64_t m, const int32_t *__restrict__ leaves,
                                                       const int32_t *__restrict__ first,
                                                       const int32_t *__restrict__ size,
                                                       const int64_t *__restrict__ perm, const double *__restrict__ V,
                                                       const double *__restrict__ yh, int64_t ldh,
                                                       const int64_t *__restrict__ ncptr,
                                                       const int64_t *__restrict__ ncblk,
                                                       const int32_t *__restrict__ near_row,
                                                       const int64_t *__restrict__ near_off, int near_t,
                                                       const double *__restrict__ N, const double *__restrict__ X,
                                                       int64_t ldx, double alpha, double beta,
                                                       double *__restrict__ Y, int64_t ldy) {
    __shared__ double As[TR][TR + 1];
    __shared__ double Bs[TR][TC];
    const int32_t l = blockIdx.x;
    const int32_t s = leaves[l];
    const int64_t j0 = (int64_t)blockIdx.y * TC;
    const int mc = (int)min<int64_t>(TC, m - j0);
    const int tid = threadIdx.x, rg = tid >> 5, j = tid & 31;
    const int64_t r0 = first[s];
    const int ns = size[s];
    for (int c0 = 0; c0 < ns; c0 += TR) {
        const int cc = min(TR, ns - c0);
        double acc[8] = {};
        for (int u0 = 0; u0 < k; u0 += TR) {
            const int uc = min(TR, k - u0);
            for (int e = tid; e < TR * TR; e += 256) {
                const int c = e / TR, nu = e % TR;
                As[c][nu] = (c < cc && nu < uc) ? V[(r0 + c0 + c) * k + u0 + nu] : 0.0;
            }
            for (int e = tid; e < TR * TC; e += 256) {
                const int nu = e / TC, jj = e % TC;
                Bs[nu][jj] = (nu < uc && jj < mc) ? yh[((int64_t)s * k + u0 + nu) * ldh + j0 + jj] : 0.0;
            }
            __syncthreads();
            tile_fma(acc, As, Bs, uc, rg, j);
            __syncthreads();
        }
        for (int64_t q = ncptr[l]; q < ncptr[l + 1]; ++q) {
            const int64_t b = ncblk[q];
            const int32_t t = near_row[b];
            const int nt = size[t];
            const int64_t nt2 = pad_rows(nt), ft = first[t];
            const double *Nb = N + near_off[b];
            for (int i0 = 0; i0 < nt; i0 += TR) {
                const int ic = min(TR, nt - i0);
                // As[c][i] = N_ts[i][c]
                for (int e = tid; e < TR * TR; e += 256) {
                    const int c = e / TR, i = e % TR;
                    double v = 0.0;
                    if (c < cc && i < ic) {
                        const int64_t o = near_t ? (int64_t)(c0 + c) * nt2 + i0 + i : (int64_t)(i0 + i) * ns + c0 + c;
                        v = Nb[o];
                    }
                    As[c][i] = v;
                }
                for (int e = tid; e < TR * TC; e += 256) {
                    const int i = e / TC, jj = e % TC;
                    Bs[i][jj] = (i < ic && jj < mc) ? X[perm[ft + i0 + i] * ldx + j0 + jj] : 0.0;
                }
                __syncthreads();
                tile_fma(acc, As, Bs, ic, rg, j);
                __syncthreads();
            }
        }
        if (j < mc)
            for (int q = 0; q < 8; ++q) {
                const int c = rg + 8 * q;
                if (c < cc) {
                    double *y = &Y[perm[r0 + c0 + c] * ldy + j0 + j];
                    const double v = alpha * acc[q];
                    *y = (beta == 0.0) ? v : beta * *y + v;
                }
            }
    }
}

// one admissible block per work-group: D = scale * dyhat_t xhat_s^T (k x k, k <= 64);
// dS_b = D if requested; part[b] = sum of (dg/dell) * D in a fixed order (0 unless want_dell)
__global__ __launch_bounds__(256) void k_grad_S(int k, int64_t m, const int32_t *__restrict__ adm_row,
                                                const int32_t *__restrict__ adm_col,
                                                const double *__restrict__ nodes, int kernel, double ell,
                                                const double *__restrict__ dh, const double *__restrict__ xh,
                                                int64_t ldh, double scale, int want_dell, double *__restrict__ dS,
                                                double *__restrict__ part) {
    __shared__ double sd[64][65], sx[64][65];
    __shared__ double red[256];
    const int64_t b = blockIdx.x;
    const int32_t t = adm_row[b], s = adm_col[b];
    const int tid = threadIdx.x, kk = k * k;
    double acc[16] = {};
    for (int64_t j0 = 0; j0 < m; j0 += 64) {
        const int mc = (int)min<int64_t>(64, m - j0);
        for (int e = tid; e < k * 64; e += 256) {
            const int nu = e / 64, jj = e % 64;
            sd[nu][jj] = jj < mc ? dh[((int64_t)t * k + nu) * ldh + j0 + jj] : 0.0;
            sx[nu][jj] = jj < mc ? xh[((int64_t)s * k + nu) * ldh + j0 + jj] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int e = tid + 256 * u;
            if (e < kk) {
                const int nu = e / k, mu = e % k;
                double a = acc[u];
                for (int jj = 0; jj < mc; ++jj) a += sd[nu][jj] * sx[mu][jj];
                acc[u] = a;
            }
        }
        __syncthreads();
    }
    double g = 0.0;
#pragma unroll
    for (int u = 0; u < 16; ++u) {
        const int e = tid + 256 * u;
        if (e < kk) {
            const int nu = e / k, mu = e % k;
            const double d = scale * acc[u];
            if (dS) dS[b * kk + e] = d;
            if (want_dell)
                g += dg_dell(kernel, ell, &nodes[((int64_t)t * k + nu) * 3], &nodes[((int64_t)s * k + mu) * 3]) * d;
        }
    }
    red[tid] = g;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (tid < w) red[tid] += red[tid + w];
        __syncthreads();
    }
    if (tid == 0) part[b] = red[0];
}

// one near-field block per work-group: D = scale * dY|_t X|_s^T (tree-ordered dY, X);
// dN_b = D (row-major |t| x |s|) if requested; part[q] = sum of (dg/dell) * D (0 unless want_dell)
__global__ __launch_bounds__(256) void k_grad_N(int64_t m, const int32_t *__restrict__ near_row,
                                                const int32_t *__restrict__ near_col,
                                                const int64_t *__restrict__ near_off_rm,
                                                const int32_t *__restrict__ first, const int32_t *__restrict__ size,
                                                const double *__restrict__ pts, int kernel, double ell,
                                                const double *__restrict__ dYt, const double *__restrict__ Xt,
                                                int64_t ldt, double scale, int want_dell, double *__restrict__ dN,
                                                double *__restrict__ part) {
    __shared__ double sd[64][33], sx[64][33];
    __shared__ double red[256];
    const int64_t q = blockIdx.x;
    const int32_t t = near_row[q], s = near_col[q];
    const int nt = size[t], ns = size[s];
    const int64_t ft = first[t], fs = first[s];
    const int tid = threadIdx.x;
    double g = 0.0;
    for (int i0 = 0; i0 < nt; i0 += 64)
        for (int c0 = 0; c0 < ns; c0 += 64) {
            const int ic = min(64, nt - i0), cc = min(64, ns - c0);
            double acc[16] = {};
            for (int64_t j0 = 0; j0 < m; j0 += 32) {
                const int mc = (int)min<int64_t>(32, m - j0);
                for (int e = tid; e < 64 * 32; e += 256) {
                    const int r = e / 32, jj = e % 32;
                    sd[r][jj] = (r < ic && jj < mc) ? dYt[(ft + i0 + r) * ldt + j0 + jj] : 0.0;
                    sx[r][jj] = (r < cc && jj < mc) ? Xt[(fs + c0 + r) * ldt + j0 + jj] : 0.0;
                }
                __syncthreads();
#pragma unroll
                for (int u = 0; u < 16; ++u) {
                    const int e = tid + 256 * u, i = e / 64, c = e % 64;
                    double a = acc[u];
                    for (int jj = 0; jj < mc; ++jj) a += sd[i][jj] * sx[c][jj];
                    acc[u] = a;
                }
                __syncthreads();
            }
#pragma unroll
            for (int u = 0; u < 16; ++u) {
                const int e = tid + 256 * u, i = e / 64, c = e % 64;
                if (i < ic && c < cc) {
                    const double d = scale * acc[u];
                    if (dN) dN[near_off_rm[q] + (int64_t)(i0 + i) * ns + c0 + c] = d;
                    if (want_dell) g += dg_dell(kernel, ell, &pts[3 * (ft + i0 + i)], &pts[3 * (fs + c0 + c)]) * d;
                }
            }
        }
    red[tid] = g;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (tid < w) red[tid] += red[tid + w];
        __syncthreads();
    }
    if (tid == 0) part[q] = red[0];
}

// dell = sum of the per-block partial sums, in a fixed order: work-group g adds
// entries [g * chunk, (g + 1) * chunk) into out[g] (one work-group: the total)
__global__ void k_sum_fixed(int64_t count, int64_t chunk, const double *__restrict__ part, double *__restrict__ out) {
    __shared__ double red[256];
    const int64_t a = (int64_t)blockIdx.x * chunk, b = min(count, a + chunk);
    double s = 0.0;
    for (int64_t i = a + threadIdx.x; i < b; i += 256) s += part[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[blockIdx.x] = red[0];
}

constexpr int64_t kSumChunk = 2048;

__global__ void k_gather_even(int64_t n, int64_t m, const int64_t *__restrict__ perm, const double *__restrict__ X,
                              int64_t ldx, double *__restrict__ Xt, int64_t ldt) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * ldt) return;
    const int64_t i = e / ldt, j = e % ldt;
    Xt[e] = j < m ? X[perm[i] * ldx + j] : 0.0;
}

// coupling matrices read back row-major (undoing the matrix-core layout)
__global__ void k_read_S(int k, int swz, const double *__restrict__ S, double *__restrict__ out) {
    const int64_t b = blockIdx.x, kk = (int64_t)k * k;
    for (int e = threadIdx.x; e < kk; e += blockDim.x) out[b * kk + e] = S[b * kk + s_index(swz, k, e / k, e % k)];
}

__global__ void k_write_S(int k, int swz, const double *__restrict__ in, double *__restrict__ S) {
    const int64_t b = blockIdx.x, kk = (int64_t)k * k;
    for (int e = threadIdx.x; e < kk; e += blockDim.x) S[b * kk + s_index(swz, k, e / k, e % k)] = in[b * kk + e];
}

int64_t even(int64_t m) { return m + (m & 1); }

struct GradWs {
    double *xh, *dh, *Xt, *dYt, *part, *part2, *xt_ws;
    size_t bytes;
};

// d ell alone on the rank-64 matrix-core path: the coupling term as the coupling product with
// dg/dell in place of S (one partial sum per work-group), the near-field term as the leaf
// stage's near contraction with dg/dell in place of N
struct DellShape {
    int nj, np;
    int64_t cpl_groups, near_slots;
    size_t near_lds;
    bool ok;
};

DellShape dell_shape(const DevMat &dm, int64_t m) {
    DellShape d{};
    d.nj = (int)std::min<int64_t>(4, (m + 15) / 16);
    d.np = 1;  // 32 columns per work-group (64 would not fit the registers of the near kernel)
    d.cpl_groups = (int64_t)8 * ((dm.C + 7) / 8) * ((m + 16 * d.nj - 1) / (16 * d.nj));
    d.near_slots = (int64_t)8 * ((dm.L + 7) / 8) * ((m + 32 * d.np - 1) / (32 * d.np));
    d.near_lds = sizeof(int32_t) * (size_t)std::max(1, dm.max_near_rows);
    d.ok = dm.mc && dm.k == 64 && dm.swz == 1 && !dm.cplx && dm.cpl_order &&
           d.near_lds + sizeof(double) * (64 * (32 * d.np + 1) + 256) + 64 <= 65536;
    return d;
}

GradWs grad_layout(const DevMat &dm, int64_t m, char *base) {
    GradWs w{};
    size_t off = 0;
    auto carve = [&](size_t bytes) {
        off = align_up(off);
        char *p = base ? base + off : nullptr;
        off += bytes;
        return (double *)p;
    };
    const size_t hat = (size_t)dm.C * dm.k * even(m) * sizeof(double), nm = (size_t)dm.n * even(m) * sizeof(double);
    w.xh = carve(hat);
    w.dh = carve(hat);
    w.Xt = carve(nm);
    w.dYt = carve(nm);
    w.xt_ws = carve(nm);
    const DellShape ds = dell_shape(dm, m);
    const int64_t np = std::max<int64_t>(dm.n_adm + dm.n_near, ds.cpl_groups + ds.near_slots) + 1;
    w.part = carve((size_t)np * sizeof(double));
    w.part2 = carve((size_t)(np / kSumChunk + 2) * sizeof(double));
    w.bytes = align_up(off);
    return w;
}

}  // namespace

size_t grad_ws_bytes(const DevMat &dm, int64_t m) { return grad_layout(dm, m, nullptr).bytes; }

hipError_t run_read_coupling(const DevMat &dm, double *out, hipStream_t st) {
    if (dm.n_adm > 0)
        hipLaunchKernelGGL(k_read_S, dim3((unsigned)dm.n_adm), dim3(256), 0, st, dm.k, dm.swz, (const double *)dm.S,
                           out);
    return hipGetLastError();
}

hipError_t run_write_coupling(const DevMat &dm, const double *in, hipStream_t st) {
    if (dm.n_adm > 0)
        hipLaunchKernelGGL(k_write_S, dim3((unsigned)dm.n_adm), dim3(256), 0, st, dm.k, dm.swz, in, (double *)dm.S);
    return hipGetLastError();
}

size_t adjoint_ws_bytes(const DevMat &dm, int64_t m) {
    return 2 * align_up((size_t)dm.C * dm.k * even(m) * sizeof(double)) +
           align_up((size_t)dm.n * even(m) * sizeof(double));
}

hipError_t run_matmul_adjoint(const DevMat &dm, int64_t m, double alpha, const double *X, int64_t ldx, double beta,
                              double *Y, int64_t ldy, char *ws, hipStream_t st) {
    // workspace: x-hat, y-hat (even leading dimension) and a tree-ordered copy of X
    const int64_t ldh = even(m);
    const size_t hat = align_up((size_t)dm.C * dm.k * ldh * sizeof(double));
    double *xh = (double *)ws, *yh = (double *)(ws + hat), *xt = (double *)(ws + 2 * hat);
    hipError_t e = run_forward_transform(dm, m, X, ldx, false, xh, ldh, xt, st);
    if (e != hipSuccess) return e;
    if (dm.mc) {
        // matrix-core path: the forward transformation left X in tree order in xt (leading dimension ldh)
        const int nj = (int)std::min<int64_t>(4, (m + 15) / 16);
        const unsigned gy = (unsigned)((m + 16 * nj - 1) / (16 * nj));
        auto go = [&](auto NJc) {
            constexpr int NJ = decltype(NJc)::value;
            hipLaunchKernelGGL(adj::k_coupling_adj_mfma<NJ>, dim3(8 * ((dm.C + 7) / 8), gy), dim3(256), 0, st, dm.k,
                               dm.swz, m, dm.C, dm.adm_cptr, dm.adm_cblk, dm.adm_row, (const double *)dm.S,
                               (const double *)xh, yh, ldh);
            hipError_t ee = run_down_pass(dm, m, yh, ldh, st);
            if (ee != hipSuccess) return ee;
            hipLaunchKernelGGL(adj::k_leaf_adj_mfma<NJ>, dim3(8 * ((dm.L + 7) / 8), gy), dim3(256), 0, st, dm.k, m,
                               dm.L, dm.leaves, dm.first, dm.size, dm.perm, (const double *)dm.V,
                               (const double *)yh, ldh, dm.near_cptr, dm.near_cblk, dm.near_row, dm.near_off,
                               (const double *)dm.N, (const double *)xt, ldh, alpha, beta, Y, ldy);
            return hipGetLastError();
        };
        switch (nj) {
            case 1: return go(std::integral_constant<int, 1>{});
            case 2: return go(std::integral_constant<int, 2>{});
            case 3: return go(std::integral_constant<int, 3>{});
            default: return go(std::integral_constant<int, 4>{});
        }
    }
    const unsigned gy = (unsigned)((m + TC - 1) / TC);
    hipLaunchKernelGGL(k_coupling_adj, dim3(dm.C, gy), dim3(256), 0, st, dm.k, m, dm.adm_cptr, dm.adm_cblk,
                       dm.adm_row, (const double *)dm.S, dm.swz, (const double *)xh, yh, ldh);
    e = run_down_pass(dm, m, yh, ldh, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_leaf_near_adj, dim3(dm.L, gy), dim3(256), 0, st, dm.k, m, dm.leaves, dm.first, dm.size,
                       dm.perm, (const double *)dm.V, (const double *)yh, ldh, dm.near_cptr, dm.near_cblk,
                       dm.near_row, dm.near_off, dm.near_t, (const double *)dm.N, X, ldx, alpha, beta, Y, ldy);
    return hipGetLastError();
}

__global__ void k_fill0(int64_t count, double *__restrict__ p) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < count) p[e] = 0.0;
}

__global__ void k_scale1(double *__restrict__ v, double s) { v[0] *= s; }

// d ell alone: the fused kernels above, then one fixed-order sum of their partial sums
hipError_t run_dell_fused(const DevMat &dm, const DellShape &ds, int64_t m, const double *X, int64_t ldx,
                          const double *dY, int64_t lddy, double *dell, double scale, int cpl, int nr, GradWs &w,
                          hipStream_t st) {
    const int64_t ldh = even(m);
    hipError_t e = hipSuccess;
    double *pc = w.part, *pn = w.part + ds.cpl_groups;
    const int64_t cnt = ds.cpl_groups + ds.near_slots;
    if (cpl) {
        e = run_forward_transform(dm, m, X, ldx, false, w.xh, ldh, w.xt_ws, st);
        if (e == hipSuccess) e = run_forward_transform(dm, m, dY, lddy, false, w.dh, ldh, w.xt_ws, st);
        if (e != hipSuccess) return e;
        const int32_t rpx = (dm.C + 7) / 8;
        const double ie = 1.0 / dm.ell;
        auto go = [&](auto NJc) {
            constexpr int NJ = decltype(NJc)::value;
            hipLaunchKernelGGL(adj::k_dell_coupling<NJ>, dim3((unsigned)ds.cpl_groups), dim3(256), 0, st, m, dm.C, rpx,
                               dm.cpl_order, dm.adm_ptr, dm.adm_col, dm.nodes, ie * ie, (const double *)dm.S,
                               (const double *)w.xh, (const double *)w.dh, ldh, pc);
        };
        switch (ds.nj) {
            case 1: go(std::integral_constant<int, 1>{}); break;
            case 2: go(std::integral_constant<int, 2>{}); break;
            case 3: go(std::integral_constant<int, 3>{}); break;
            default: go(std::integral_constant<int, 4>{}); break;
        }
    } else {
        hipLaunchKernelGGL(k_fill0, dim3((unsigned)((ds.cpl_groups + 255) / 256)), dim3(256), 0, st, ds.cpl_groups, pc);
    }
    if (nr) {
        const int64_t cg = dm.n * ldh;
        hipLaunchKernelGGL(k_gather_even, dim3((unsigned)((cg + 255) / 256)), dim3(256), 0, st, dm.n, m, dm.perm, X,
                           ldx, w.Xt, ldh);
        hipLaunchKernelGGL(k_gather_even, dim3((unsigned)((cg + 255) / 256)), dim3(256), 0, st, dm.n, m, dm.perm, dY,
                           lddy, w.dYt, ldh);
        const mfma::LeafCatArgs a{dm.k, m, dm.L, dm.leaf_order, dm.leaves, dm.first, dm.size, dm.perm, (const double *)dm.Vt,
                                  dm.vt_off, nullptr, 0, dm.near_ptr, dm.near_col, dm.near_off, (const double *)dm.N,
                                  w.Xt, ldh, 1.0, 0.0, nullptr, 0, 1, 0, 1, Skip{}};
        const double ie = 1.0 / dm.ell;
        const mfma::DellArgs d{dm.pts, ie, ie * ie, w.dYt, ldh};
        hipLaunchKernelGGL(mfma::k_dell_near<1>, dim3((unsigned)ds.near_slots), dim3(256), ds.near_lds, st, a, d, pn);
    } else {
        hipLaunchKernelGGL(k_fill0, dim3((unsigned)((ds.near_slots + 255) / 256)), dim3(256), 0, st, ds.near_slots, pn);
    }
    const int64_t ng = (cnt + kSumChunk - 1) / kSumChunk;
    if (ng > 1) {
        hipLaunchKernelGGL(k_sum_fixed, dim3((unsigned)ng), dim3(256), 0, st, cnt, kSumChunk, (const double *)w.part,
                           w.part2);
        hipLaunchKernelGGL(k_sum_fixed, dim3(1), dim3(256), 0, st, ng, ng, (const double *)w.part2, dell);
    } else {
        hipLaunchKernelGGL(k_sum_fixed, dim3(1), dim3(256), 0, st, cnt, cnt + 1, (const double *)w.part, dell);
    }
    if (scale != 1.0) hipLaunchKernelGGL(k_scale1, dim3(1), dim3(1), 0, st, dell, scale);
    return hipGetLastError();
}

hipError_t run_grad(const DevMat &dm, int64_t m, const double *X, int64_t ldx, const double *dY, int64_t lddy,
                    double *dS, double *dN, double *dell, double scale, int32_t dell_terms, char *ws,
                    hipStream_t st) {
    GradWs w = grad_layout(dm, m, ws);
    const int64_t ldh = even(m);
    hipError_t e = hipSuccess;
    const int cpl = dell && (dell_terms & H2X_DELL_COUPLING) ? 1 : 0, nr = dell && (dell_terms & H2X_DELL_NEAR) ? 1 : 0;
    // d ell on the rank-64 exponential operator: its own fused kernels (after the block
    // gradients, which then skip their d ell terms)
    const DellShape ds = dell_shape(dm, m);
    const bool fused = dell && ds.ok && dm.kernel == H2X_KERNEL_EXP && dm.n_adm + dm.n_near > 0;
    if (fused && !dS && !dN) return run_dell_fused(dm, ds, m, X, ldx, dY, lddy, dell, scale, cpl, nr, w, st);
    const int cpl_b = fused ? 0 : cpl, nr_b = fused ? 0 : nr;  // d ell terms of the block-gradient kernels
    // the partial sums of dell's terms that are not wanted are zero
    if (dell && !fused && !cpl && dm.n_adm > 0)
        hipLaunchKernelGGL(k_fill0, dim3((unsigned)((dm.n_adm + 255) / 256)), dim3(256), 0, st, dm.n_adm, w.part);
    if (dell && !fused && !nr && dm.n_near > 0)
        hipLaunchKernelGGL(k_fill0, dim3((unsigned)((dm.n_near + 255) / 256)), dim3(256), 0, st, dm.n_near,
                           w.part + dm.n_adm);
    if (dS || cpl_b) {
        e = run_forward_transform(dm, m, X, ldx, false, w.xh, ldh, w.xt_ws, st);
        if (e == hipSuccess) e = run_forward_transform(dm, m, dY, lddy, false, w.dh, ldh, w.xt_ws, st);
        if (e != hipSuccess) return e;
        if (dm.n_adm > 0) {
            if (dm.mc) {
                // LDS tiles sized to the column chunk (16, 32 or 64 columns)
                auto go = [&](auto CWc) {
                    hipLaunchKernelGGL(adj::k_grad_S_mfma<decltype(CWc)::value>, dim3((unsigned)dm.n_adm), dim3(256), 0,
                                       st, dm.k, m, dm.adm_row, dm.adm_col, dm.nodes, dm.kernel, dm.ell,
                                       (const double *)w.dh, (const double *)w.xh, ldh, scale, cpl_b, dS, w.part);
                };
                if (m <= 16) go(std::integral_constant<int, 16>{});
                else if (m <= 32) go(std::integral_constant<int, 32>{});
                else go(std::integral_constant<int, 64>{});
            } else
                hipLaunchKernelGGL(k_grad_S, dim3((unsigned)dm.n_adm), dim3(256), 0, st, dm.k, m, dm.adm_row,
                                   dm.adm_col, dm.nodes, dm.kernel, dm.ell, (const double *)w.dh,
                                   (const double *)w.xh, ldh, scale, cpl_b, dS, w.part);
        }
    }
    if (dN || nr_b) {
        const int64_t cnt = dm.n * ldh;
        hipLaunchKernelGGL(k_gather_even, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, st, dm.n, m, dm.perm, X,
                           ldx, w.Xt, ldh);
        hipLaunchKernelGGL(k_gather_even, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, st, dm.n, m, dm.perm, dY,
                           lddy, w.dYt, ldh);
        if (dm.n_near > 0) {
            if (dm.mc) {
                auto go = [&](auto CWc) {
                    hipLaunchKernelGGL(adj::k_grad_N_mfma<decltype(CWc)::value>, dim3((unsigned)dm.n_near), dim3(256), 0,
                                       st, m, dm.near_row, dm.near_col, dm.near_off_rm, dm.first, dm.size, dm.pts,
                                       dm.kernel, dm.ell, (const double *)w.dYt, (const double *)w.Xt, ldh, scale, nr_b,
                                       dN, w.part + dm.n_adm);
                };
                if (m <= 16) go(std::integral_constant<int, 16>{});
                else if (m <= 32) go(std::integral_constant<int, 32>{});
                else go(std::integral_constant<int, 64>{});
            } else
                hipLaunchKernelGGL(k_grad_N, dim3((unsigned)dm.n_near), dim3(256), 0, st, m, dm.near_row,
                                   dm.near_col, dm.near_off_rm, dm.first, dm.size, dm.pts, dm.kernel, dm.ell,
                                   (const double *)w.dYt, (const double *)w.Xt, ldh, scale, nr_b, dN,
                                   w.part + dm.n_adm);
        }
    }
    if (fused) return run_dell_fused(dm, ds, m, X, ldx, dY, lddy, dell, scale, cpl, nr, w, st);
    if (dell) {
        const int64_t cnt = dm.n_adm + dm.n_near, ng = (cnt + kSumChunk - 1) / kSumChunk;
        if (ng > 1) {
            hipLaunchKernelGGL(k_sum_fixed, dim3((unsigned)ng), dim3(256), 0, st, cnt, kSumChunk,
                               (const double *)w.part, w.part2);
            hipLaunchKernelGGL(k_sum_fixed, dim3(1), dim3(256), 0, st, ng, ng, (const double *)w.part2, dell);
        } else {
            hipLaunchKernelGGL(k_sum_fixed, dim3(1), dim3(256), 0, st, cnt, cnt + 1, (const double *)w.part, dell);
        }
    }
    return hipGetLastError();
}

}  // namespace h2x
