// Block CG (section 5.1): m independent CG iterations that share one H^2 x P
// product per iteration; step sizes per column,
//   beta_i = <p_i, a_i>, alpha_i = <p_i, r_i> / beta_i,
//   x_i += alpha_i p_i,  r_i -= alpha_i a_i,
//   gamma_i = <a_i, r_i> / beta_i,  p_i = r_i - gamma_i p_i,
// until every column satisfies ||r_i|| <= rtol ||b_i||.
//
// The iteration runs in tree order (rows permuted once on entry and once on
// exit) so the products need no gathers.  Dot products are reduced in two
// fixed-order passes (per-row-block partial sums, then one work-group), so the
// solve is bitwise reproducible.  Convergence is decided on the device; the
// host reads one flag every check_every iterations, and the CG kernels of an
// iteration that starts after convergence do nothing.
#include <cmath>
#include <vector>

#include "device.hpp"

namespace h2x {

namespace {

constexpr int kDotCols = 32;  // columns per work-group in the dot kernels

struct CgState {
    int32_t all_conv, skip, iter, pad;
};

struct CgCols {  // per-column arrays, m entries each
    double *bnorm, *rr, *beta, *alpha, *gamma;
    int32_t *frozen, *conv, *first_conv, *status, *act;
};

__global__ void k_gather_rows(int64_t n, int64_t m, const int64_t *__restrict__ perm, const double *__restrict__ src,
                              int64_t lds, double *__restrict__ dst, int64_t ldd) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * m) return;
    const int64_t i = e / m, j = e % m;
    dst[i * ldd + j] = src[perm[i] * lds + j];
}

__global__ void k_scatter_rows(int64_t n, int64_t m, const int64_t *__restrict__ perm, const double *__restrict__ src,
                               int64_t lds, double *__restrict__ dst, int64_t ldd) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * m) return;
    const int64_t i = e / m, j = e % m;
    dst[perm[i] * ldd + j] = src[i * lds + j];
}

__global__ void k_copy(int64_t count, const double *__restrict__ src, double *__restrict__ dst) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < count) dst[e] = src[e];
}

// Partial sums of up to two column-wise dot products over one block of rows:
// part[(pair * nblk + blk) * m + j].  Row ownership is fixed, the reduction
// order too.
__device__ inline void block_dots(int64_t n, int64_t m, int nblk, const double *u0, const double *v0,
                                  const double *u1, const double *v1, double *part) {
    __shared__ double red[2][8][kDotCols];
    const int tid = threadIdx.x, rg = tid >> 5, jl = tid & 31;
    const int64_t j = (int64_t)blockIdx.y * kDotCols + jl;
    const int64_t rows = (n + nblk - 1) / nblk;
    const int64_t r0 = (int64_t)blockIdx.x * rows, r1 = min(n, r0 + rows);
    double s0 = 0.0, s1 = 0.0;
    if (j < m)
        for (int64_t i = r0 + rg; i < r1; i += 8) {
            s0 += u0[i * m + j] * v0[i * m + j];
            if (u1) s1 += u1[i * m + j] * v1[i * m + j];
        }
    red[0][rg][jl] = s0;
    red[1][rg][jl] = s1;
    __syncthreads();
    if (rg == 0 && j < m) {
        double a = 0.0, b = 0.0;
        for (int g = 0; g < 8; ++g) { a += red[0][g][jl]; b += red[1][g][jl]; }
        part[(int64_t)blockIdx.x * m + j] = a;
        if (u1) part[((int64_t)nblk + blockIdx.x) * m + j] = b;
    }
}

__global__ __launch_bounds__(256) void k_dots(int64_t n, int64_t m, int nblk, const double *u0, const double *v0,
                                              const double *u1, const double *v1, double *part,
                                              const CgState *state) {
    if (state && state->skip) return;
    block_dots(n, m, nblk, u0, v0, u1, v1, part);
}

__device__ inline double sum_part(const double *part, int pair, int nblk, int64_t m, int64_t j) {
    double s = 0.0;
    for (int b = 0; b < nblk; ++b) s += part[((int64_t)pair * nblk + b) * m + j];
    return s;
}

// initial norms: pairs (B, B) and (R, R)
__global__ void k_cg_init(int64_t m, int nblk, const double *part, double rtol, CgState *state, CgCols cols) {
    __shared__ int notconv;
    if (threadIdx.x == 0) notconv = 0;
    __syncthreads();
    for (int64_t j = threadIdx.x; j < m; j += blockDim.x) {
        const double bb = sum_part(part, 0, nblk, m, j), rr = sum_part(part, 1, nblk, m, j);
        cols.bnorm[j] = sqrt(bb);
        cols.rr[j] = rr;
        const int c = sqrt(rr) <= rtol * sqrt(bb);
        cols.conv[j] = c;
        cols.first_conv[j] = c ? 0 : -1;
        cols.frozen[j] = 0;
        cols.status[j] = 0;
        cols.act[j] = 0;
        if (!c) atomicOr(&notconv, 1);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        state->all_conv = notconv ? 0 : 1;
        state->skip = 0;
        state->iter = 0;
    }
}

// pairs (P, AP) and (P, R): beta_i, alpha_i, breakdown detection
__global__ void k_cg_alpha(int64_t m, int nblk, const double *part, int freeze_converged, CgState *state,
                           CgCols cols) {
    const int skip = state->all_conv;
    __syncthreads();
    if (threadIdx.x == 0) state->skip = skip;
    if (skip) return;
    for (int64_t j = threadIdx.x; j < m; j += blockDim.x) {
        const double beta = sum_part(part, 0, nblk, m, j), rho = sum_part(part, 1, nblk, m, j);
        // an exactly zero residual is an exact solution: nothing to update
        int act = !cols.frozen[j] && !(freeze_converged && cols.conv[j]) && cols.rr[j] > 0.0;
        double alpha = 0.0;
        if (act) {
            alpha = rho / beta;
            if (!(beta > 0.0) || !isfinite(alpha)) {
                cols.frozen[j] = 1;
                cols.status[j] = 1;
                act = 0;
                alpha = 0.0;
            }
        }
        cols.beta[j] = beta;
        cols.alpha[j] = alpha;
        cols.act[j] = act;
    }
}

// x += alpha p, r -= alpha a for active columns; then partial sums of <a, r>, <r, r>
__global__ __launch_bounds__(256) void k_cg_update_xr(int64_t n, int64_t m, int nblk, double *X, double *R,
                                                      const double *P, const double *AP, double *part,
                                                      const CgState *state, CgCols cols) {
    if (state->skip) return;
    const int tid = threadIdx.x, rg = tid >> 5, jl = tid & 31;
    const int64_t j = (int64_t)blockIdx.y * kDotCols + jl;
    const int64_t rows = (n + nblk - 1) / nblk;
    const int64_t r0 = (int64_t)blockIdx.x * rows, r1 = min(n, r0 + rows);
    if (j < m && cols.act[j]) {
        const double a = cols.alpha[j];
        for (int64_t i = r0 + rg; i < r1; i += 8) {
            X[i * m + j] += a * P[i * m + j];
            R[i * m + j] -= a * AP[i * m + j];
        }
    }
    // each thread re-reads only the rows it just wrote, so no barrier is needed
    block_dots(n, m, nblk, AP, R, R, R, part);
}

// gamma_i, convergence test, iteration count
__global__ void k_cg_gamma(int64_t m, int nblk, const double *part, double rtol, CgState *state, CgCols cols) {
    if (state->skip) return;
    __shared__ int notconv;
    if (threadIdx.x == 0) notconv = 0;
    __syncthreads();
    const int it = state->iter + 1;
    for (int64_t j = threadIdx.x; j < m; j += blockDim.x) {
        const double ar = sum_part(part, 0, nblk, m, j), rr = sum_part(part, 1, nblk, m, j);
        cols.gamma[j] = cols.act[j] ? ar / cols.beta[j] : 0.0;
        cols.rr[j] = rr;
        const int c = sqrt(rr) <= rtol * cols.bnorm[j];
        cols.conv[j] = c;
        if (c && cols.first_conv[j] < 0) cols.first_conv[j] = it;
        if (!c && !cols.frozen[j]) atomicOr(&notconv, 1);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        state->iter = it;
        state->all_conv = notconv ? 0 : 1;
    }
}

// p = r - gamma p for active columns
__global__ void k_cg_update_p(int64_t n, int64_t m, const double *R, double *P, const CgState *state, CgCols cols) {
    if (state->skip) return;
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * m) return;
    const int64_t j = e % m;
    if (cols.act[j]) P[e] = R[e] - cols.gamma[j] * P[e];
}

struct CgWs {
    double *Bt, *Xt, *R, *P, *AP, *part;
    CgState *state;
    CgCols cols;
    char *mm;
    int nblk;
    size_t bytes;
};

CgWs cg_layout(const DevMat &dm, int64_t m, char *base) {
    CgWs w{};
    size_t off = 0;
    auto carve = [&](size_t bytes) {
        off = align_up(off);
        char *p = base ? base + off : nullptr;
        off += bytes;
        return p;
    };
    const size_t nm = (size_t)dm.n * m * sizeof(double);
    w.nblk = (int)std::min<int64_t>(1024, std::max<int64_t>(1, (dm.n + 63) / 64));
    w.Bt = (double *)carve(nm);
    w.Xt = (double *)carve(nm);
    w.R = (double *)carve(nm);
    w.P = (double *)carve(nm);
    w.AP = (double *)carve(nm);
    w.part = (double *)carve(2 * (size_t)w.nblk * m * sizeof(double));
    w.state = (CgState *)carve(sizeof(CgState));
    double **dcols[5] = {&w.cols.bnorm, &w.cols.rr, &w.cols.beta, &w.cols.alpha, &w.cols.gamma};
    for (auto d : dcols) *d = (double *)carve(m * sizeof(double));
    int32_t **icols[5] = {&w.cols.frozen, &w.cols.conv, &w.cols.first_conv, &w.cols.status, &w.cols.act};
    for (auto d : icols) *d = (int32_t *)carve(m * sizeof(int32_t));
    w.mm = carve(matmul_ws_bytes(dm, m));
    w.bytes = align_up(off);
    return w;
}

// R = B (leading dimensions ldb -> m)
__global__ void k_copy_ld(int64_t n, int64_t m, const double *__restrict__ src, int64_t lds, double *__restrict__ dst,
                          int64_t ldd) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * m) return;
    const int64_t i = e / m, j = e % m;
    dst[i * ldd + j] = src[i * lds + j];
}

// X += D
__global__ void k_axpy_ld(int64_t n, int64_t m, const double *__restrict__ D, double *__restrict__ X, int64_t ldx) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * m) return;
    const int64_t i = e / m, j = e % m;
    X[i * ldx + j] += D[e];
}

__global__ void k_zero(int64_t count, double *__restrict__ p) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < count) p[e] = 0.0;
}

// squared column norms of two n x m blocks, in a fixed order: out[0..m) and out[m..2m)
__global__ void k_sum_parts(int64_t m, int nblk, const double *part, double *out) {
    for (int64_t j = threadIdx.x; j < m; j += blockDim.x) {
        out[j] = sum_part(part, 0, nblk, m, j);
        out[m + j] = sum_part(part, 1, nblk, m, j);
    }
}

struct RefineWs {
    double *B, *R, *D, *part, *norms;
    char *mm, *cg;
    int nblk;
    size_t bytes;
};

RefineWs refine_layout(const DevMat &hi, const DevMat &lo, int64_t m, char *base) {
    RefineWs w{};
    size_t off = 0;
    auto carve = [&](size_t bytes) {
        off = align_up(off);
        char *p = base ? base + off : nullptr;
        off += bytes;
        return p;
    };
    const size_t nm = (size_t)hi.n * m * sizeof(double);
    w.nblk = (int)std::min<int64_t>(1024, std::max<int64_t>(1, (hi.n + 63) / 64));
    w.B = (double *)carve(nm);
    w.R = (double *)carve(nm);
    w.D = (double *)carve(nm);
    w.part = (double *)carve(2 * (size_t)w.nblk * m * sizeof(double));
    w.norms = (double *)carve(2 * m * sizeof(double));
    w.mm = carve(matmul_ws_bytes(hi, m));
    w.cg = carve(cg_layout(lo, m, nullptr).bytes);
    w.bytes = align_up(off);
    return w;
}

}  // namespace

size_t cg_ws_bytes(const DevMat &dm, int64_t m) { return cg_layout(dm, m, nullptr).bytes; }

size_t refine_ws_bytes(const DevMat &hi, const DevMat &lo, int64_t m) { return refine_layout(hi, lo, m, nullptr).bytes; }

h2x_status run_refine(const DevMat &hi, const DevMat &lo, const h2x_cg_params &inner, double rtol, int32_t max_outer,
                      int64_t m, const double *B, int64_t ldb, double *X, int64_t ldx, char *ws, size_t ws_bytes,
                      h2x_cg_info *info, hipStream_t st) {
    RefineWs w = refine_layout(hi, lo, m, ws);
    if (ws_bytes < w.bytes) {
        set_error("h2x_block_cg_refine: workspace too small");
        return H2X_ENOMEM;
    }
    const int64_t n = hi.n, nm = n * m;
    const unsigned g1 = (unsigned)((nm + 255) / 256);
    const dim3 gd(w.nblk, (unsigned)((m + kDotCols - 1) / kDotCols));
    auto fail = [&](hipError_t e) {
        set_error(std::string("h2x_block_cg_refine: ") + hipGetErrorString(e));
        return H2X_EHIP;
    };
    hipLaunchKernelGGL(k_copy_ld, dim3(g1), dim3(256), 0, st, n, m, B, ldb, w.B, m);
    std::vector<double> norms(2 * m);
    int32_t outer = 0, inner_total = 0, status = H2X_OK, stalls = 0;
    double prev = HUGE_VAL;
    for (;;) {
        // R = B - A X in FP64; squared norms of R and B
        hipLaunchKernelGGL(k_copy, dim3(g1), dim3(256), 0, st, nm, (const double *)w.B, w.R);
        hipError_t e = run_matmul(hi, m, -1.0, X, ldx, 1.0, w.R, m, false, w.mm, st);
        if (e != hipSuccess) return fail(e);
        hipLaunchKernelGGL(k_dots, gd, dim3(256), 0, st, n, m, w.nblk, w.R, w.R, w.B, w.B, w.part,
                           (const CgState *)nullptr);
        hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(256), 0, st, m, w.nblk, w.part, w.norms);
        e = hipMemcpyAsync(norms.data(), w.norms, 2 * m * sizeof(double), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) return fail(e);
        bool done = true;
        double worst = 0.0;
        for (int64_t j = 0; j < m; ++j) {
            const double bn = std::sqrt(norms[m + j]), rn = std::sqrt(norms[j]);
            if (rn > rtol * bn) done = false;
            worst = std::max(worst, bn > 0 ? rn / bn : rn);
        }
        // a step that does not halve the worst relative residual is a stall; two stalls stop
        if (worst > 0.5 * prev) ++stalls;
        prev = worst;
        if (done) break;
        if (outer >= max_outer || stalls >= 2) {
            status = H2X_ENOCONV;
            break;
        }
        // A_lo D = R by block CG, then X += D
        hipLaunchKernelGGL(k_zero, dim3(g1), dim3(256), 0, st, nm, w.D);
        h2x_cg_info ii{};
        h2x_status s = run_block_cg(lo, inner, m, w.R, m, w.D, m, w.cg, cg_layout(lo, m, nullptr).bytes, &ii, st);
        if (s != H2X_OK) return s;
        inner_total += ii.iters;
        hipLaunchKernelGGL(k_axpy_ld, dim3(g1), dim3(256), 0, st, n, m, w.D, X, ldx);
        ++outer;
    }
    if (info) {
        info->iters = inner_total;
        info->outer_iters = outer;
        info->status = status;
        for (int64_t j = 0; j < m; ++j) {
            const double rn = std::sqrt(norms[j]), bn = std::sqrt(norms[m + j]);
            const double rel = bn > 0 ? rn / bn : rn;
            if (info->col_relres) info->col_relres[j] = rel;
            if (info->col_iters) info->col_iters[j] = inner_total;
            if (info->col_status) info->col_status[j] = rel <= rtol ? 0 : 2;
        }
    }
    return H2X_OK;
}

h2x_status run_block_cg(const DevMat &dm, const h2x_cg_params &prm, int64_t m, const double *B, int64_t ldb,
                        double *X, int64_t ldx, char *ws, size_t ws_bytes, h2x_cg_info *info, hipStream_t st) {
    CgWs w = cg_layout(dm, m, ws);
    if (ws_bytes < w.bytes) {
        set_error("h2x_block_cg: workspace too small");
        return H2X_ENOMEM;
    }
    const int64_t n = dm.n, nm = n * m;
    const unsigned g1 = (unsigned)((nm + 255) / 256);
    const dim3 gd(w.nblk, (unsigned)((m + kDotCols - 1) / kDotCols));
    auto fail = [&](hipError_t e) {
        set_error(std::string("h2x_block_cg: ") + hipGetErrorString(e));
        return H2X_EHIP;
    };

    hipLaunchKernelGGL(k_gather_rows, dim3(g1), dim3(256), 0, st, n, m, dm.perm, B, ldb, w.Bt, m);
    hipLaunchKernelGGL(k_gather_rows, dim3(g1), dim3(256), 0, st, n, m, dm.perm, (const double *)X, ldx, w.Xt, m);
    // R = B - A X0, P = R
    hipLaunchKernelGGL(k_copy, dim3(g1), dim3(256), 0, st, nm, w.Bt, w.R);
    hipError_t e = run_matmul(dm, m, -1.0, w.Xt, m, 1.0, w.R, m, true, w.mm, st);
    if (e != hipSuccess) return fail(e);
    hipLaunchKernelGGL(k_copy, dim3(g1), dim3(256), 0, st, nm, w.R, w.P);
    hipLaunchKernelGGL(k_dots, gd, dim3(256), 0, st, n, m, w.nblk, w.Bt, w.Bt, w.R, w.R, w.part,
                       (const CgState *)nullptr);
    hipLaunchKernelGGL(k_cg_init, dim3(1), dim3(256), 0, st, m, w.nblk, w.part, prm.rtol, w.state, w.cols);

    const int check = prm.check_every > 0 ? prm.check_every : 1;
    CgState hs{};
    for (int32_t it = 0;; ++it) {
        if (it % check == 0 || it >= prm.max_iter) {
            e = hipMemcpyAsync(&hs, w.state, sizeof(CgState), hipMemcpyDeviceToHost, st);
            if (e == hipSuccess) e = hipStreamSynchronize(st);
            if (e != hipSuccess) return fail(e);
            if (hs.all_conv || it >= prm.max_iter) break;
        }
        e = run_matmul(dm, m, 1.0, w.P, m, 0.0, w.AP, m, true, w.mm, st);
        if (e != hipSuccess) return fail(e);
        hipLaunchKernelGGL(k_dots, gd, dim3(256), 0, st, n, m, w.nblk, w.P, w.AP, w.P, w.R, w.part,
                           (const CgState *)nullptr);
        hipLaunchKernelGGL(k_cg_alpha, dim3(1), dim3(256), 0, st, m, w.nblk, w.part, prm.freeze_converged, w.state,
                           w.cols);
        hipLaunchKernelGGL(k_cg_update_xr, gd, dim3(256), 0, st, n, m, w.nblk, w.Xt, w.R, w.P, w.AP, w.part,
                           (const CgState *)w.state, w.cols);
        hipLaunchKernelGGL(k_cg_gamma, dim3(1), dim3(256), 0, st, m, w.nblk, w.part, prm.rtol, w.state, w.cols);
        hipLaunchKernelGGL(k_cg_update_p, dim3(g1), dim3(256), 0, st, n, m, w.R, w.P, (const CgState *)w.state,
                           w.cols);
    }
    hipLaunchKernelGGL(k_scatter_rows, dim3(g1), dim3(256), 0, st, n, m, dm.perm, w.Xt, m, X, ldx);
    std::vector<double> rr(m), bn(m);
    std::vector<int32_t> fc(m), stt(m), fr(m), cv(m);
    e = hipMemcpyAsync(&hs, w.state, sizeof(CgState), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipMemcpyAsync(rr.data(), w.cols.rr, m * sizeof(double), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipMemcpyAsync(bn.data(), w.cols.bnorm, m * sizeof(double), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipMemcpyAsync(fc.data(), w.cols.first_conv, m * 4, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipMemcpyAsync(stt.data(), w.cols.status, m * 4, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipMemcpyAsync(cv.data(), w.cols.conv, m * 4, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return fail(e);
    int32_t status = H2X_OK;
    for (int64_t j = 0; j < m; ++j) {
        if (stt[j] == 0 && !cv[j]) stt[j] = 2;
        if (stt[j] == 1) status = H2X_EBREAKDOWN;
        else if (stt[j] == 2 && status == H2X_OK) status = H2X_ENOCONV;
    }
    if (info) {
        info->iters = hs.iter;
        info->status = status;
        info->outer_iters = 0;
        for (int64_t j = 0; j < m; ++j) {
            if (info->col_relres) info->col_relres[j] = bn[j] > 0 ? std::sqrt(rr[j]) / bn[j] : std::sqrt(rr[j]);
            if (info->col_iters) info->col_iters[j] = fc[j] >= 0 ? fc[j] : hs.iter;
            if (info->col_status) info->col_status[j] = stt[j];
        }
    }
    return H2X_OK;
}

}  // namespace h2x
