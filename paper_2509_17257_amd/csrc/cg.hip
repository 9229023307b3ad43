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
constexpr int kScalarThreads = 1024;  // threads of the per-system scalar kernels

struct CgState {
    int32_t all_conv, skip, iter, pad;
};

struct CgCols {  // per (system, column) arrays, nseg * m entries each, system-major
    double *bnorm, *rr, *beta, *alpha, *gamma;
    double *best;  // smallest squared true residual norm seen (mixed precision)
    int32_t *frozen, *conv, *first_conv, *status, *act;
    int32_t *keep;  // column whose current iterate is to be kept as the best (mixed precision)
};

// Dot-product blocks: block b covers rows [blk_r0[b], blk_r0[b + 1]) of system
// blk_seg[b]; system s owns blocks [seg_blk[s], seg_blk[s + 1]).  A system stops
// (seg_done) once all its columns have converged or broken down.
struct Segs {
    const int64_t *blk_r0;
    const int32_t *blk_seg, *seg_blk;
    int32_t *seg_done, *seg_iters;
    int32_t nseg;
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

// Row-block kernels: thread (rg, jl) of a 256-thread work-group takes column
// blockIdx.y * kDotCols + jl and the rows r0 + rg, r0 + rg + 8, ... of its row
// block.  The rows are visited eight at a time, all their loads issued first from
// clamped addresses, then used in row order (a row past the end is skipped).
constexpr int kRowStep = 8;

// Second stage of the partial sums: the eight row groups' sums of column j added
// in group order, part[(pair * nblk + blockIdx.x) * m + j].
__device__ inline void store_dots(double s0, double s1, int64_t m, int nblk, bool two, double *part) {
    __shared__ double red[2][8][kDotCols];
    const int tid = threadIdx.x, rg = tid >> 5, jl = tid & 31;
    const int64_t j = (int64_t)blockIdx.y * kDotCols + jl;
    red[0][rg][jl] = s0;
    red[1][rg][jl] = s1;
    __syncthreads();
    if (rg == 0 && j < m) {
        double a = 0.0, b = 0.0;
        for (int g = 0; g < 8; ++g) { a += red[0][g][jl]; b += red[1][g][jl]; }
        part[(int64_t)blockIdx.x * m + j] = a;
        if (two) part[((int64_t)nblk + blockIdx.x) * m + j] = b;
    }
}

// Partial sums of up to two column-wise dot products over rows [r0, r1), each in
// row order (fixed row ownership and reduction order).
__device__ inline void block_dots(int64_t r0, int64_t r1, int64_t m, int nblk, const double *u0, const double *v0,
                                  const double *u1, const double *v1, double *part) {
    const int tid = threadIdx.x, rg = tid >> 5, jl = tid & 31;
    const int64_t j = (int64_t)blockIdx.y * kDotCols + jl;
    const bool two = u1 != nullptr;
    double s0 = 0.0, s1 = 0.0;
    if (j < m && r1 > r0)
        for (int64_t i0 = r0 + rg; i0 < r1; i0 += 8 * kRowStep) {
            double a[kRowStep], b[kRowStep], c[kRowStep], d[kRowStep];
#pragma unroll
            for (int u = 0; u < kRowStep; ++u) {
                const int64_t i = min(i0 + 8 * u, r1 - 1);
                a[u] = u0[i * m + j];
                b[u] = v0[i * m + j];
                if (two) {
                    c[u] = u1[i * m + j];
                    d[u] = v1[i * m + j];
                }
            }
#pragma unroll
            for (int u = 0; u < kRowStep; ++u)
                if (i0 + 8 * u < r1) {
                    s0 += a[u] * b[u];
                    if (two) s1 += c[u] * d[u];
                }
        }
    store_dots(s0, s1, m, nblk, two, part);
}

// rows split evenly over nblk blocks (one system)
__global__ __launch_bounds__(256) void k_dots(int64_t n, int64_t m, int nblk, const double *u0, const double *v0,
                                              const double *u1, const double *v1, double *part) {
    const int64_t rows = (n + nblk - 1) / nblk;
    const int64_t r0 = (int64_t)blockIdx.x * rows;
    block_dots(r0, min(n, r0 + rows), m, nblk, u0, v0, u1, v1, part);
}

// rows split by the system tables
__global__ __launch_bounds__(256) void k_sdots(int64_t m, int nblk, Segs sg, const double *u0, const double *v0,
                                               const double *u1, const double *v1, double *part,
                                               const CgState *state) {
    if (state && state->skip) return;
    block_dots(sg.blk_r0[blockIdx.x], sg.blk_r0[blockIdx.x + 1], m, nblk, u0, v0, u1, v1, part);
}

__device__ inline double sum_part(const double *part, int pair, int nblk, int64_t m, int64_t j) {
    double s = 0.0;
    for (int b = 0; b < nblk; ++b) s += part[((int64_t)pair * nblk + b) * m + j];
    return s;
}

// The per-column scalar work runs with one work-group per system.  Column sums
// of the two partial-sum pairs over the system's blocks are formed in a fixed
// order: thread (r, j) adds blocks r, r + R, ... of column j, then the R partial
// sums are added in order of r.  fn(j, e, s0, s1) handles entry e = s * m + j
// and returns whether the column is still open (not converged, not broken down).
template <typename F>
__device__ inline bool for_columns(int64_t m, int nblk, const double *part, const Segs &sg, int s, F fn) {
    __shared__ double red[2][kScalarThreads];
    __shared__ int open;
    const int tid = threadIdx.x;
    const int mm = (int)min<int64_t>(m, kScalarThreads), R = kScalarThreads / mm;
    const int r = tid / mm, jl = tid % mm;
    const int b0 = sg.seg_blk[s], b1 = sg.seg_blk[s + 1];
    if (tid == 0) open = 0;
    for (int64_t jc = 0; jc < m; jc += mm) {
        const int64_t j = jc + jl;
        double a = 0.0, c = 0.0;
        // eight blocks per step, their loads issued together (clamped addresses) and added in
        // block order (a block past the end adds an exact zero): the sums keep their order
        if (r < R && j < m && b1 > b0)
            for (int bb = b0 + r; bb < b1; bb += 8 * R) {
                double va[8], vc[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int64_t b = min(bb + u * R, b1 - 1);
                    va[u] = part[b * m + j];
                    vc[u] = part[((int64_t)nblk + b) * m + j];
                }
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const bool in = bb + u * R < b1;
                    a += in ? va[u] : 0.0;
                    c += in ? vc[u] : 0.0;
                }
            }
        red[0][tid] = a;
        red[1][tid] = c;
        __syncthreads();
        if (tid < mm && j < m) {
            double s0 = 0.0, s1 = 0.0;
            for (int q = 0; q < R; ++q) {
                s0 += red[0][q * mm + tid];
                s1 += red[1][q * mm + tid];
            }
            if (fn(j, (int64_t)s * m + j, s0, s1)) atomicOr(&open, 1);
        }
        __syncthreads();
    }
    return open != 0;
}

// initial norms: pairs (B, B) and (R, R); one work-group per system
__global__ __launch_bounds__(kScalarThreads) void k_cg_init(int64_t m, int nblk, const double *part, double rtol, CgCols cols, Segs sg) {
    const int s = blockIdx.x;
    const bool open = for_columns(m, nblk, part, sg, s, [&](int64_t, int64_t e, double bb, double rr) {
        cols.bnorm[e] = sqrt(bb);
        cols.rr[e] = rr;
        const int c = sqrt(rr) <= rtol * sqrt(bb);
        cols.conv[e] = c;
        cols.first_conv[e] = c ? 0 : -1;
        cols.frozen[e] = 0;
        cols.status[e] = 0;
        cols.act[e] = 0;
        cols.alpha[e] = 0.0;
        cols.gamma[e] = 0.0;
        cols.best[e] = HUGE_VAL;
        cols.keep[e] = 0;
        return !c;
    });
    if (threadIdx.x == 0) {
        sg.seg_done[s] = open ? 0 : 1;
        sg.seg_iters[s] = 0;
    }
}

// every system done -> stop; counts the iteration (init: starts at 0)
__global__ void k_cg_state(int init, CgState *state, Segs sg) {
    __shared__ int open;
    if (!init && state->skip) return;
    if (threadIdx.x == 0) open = 0;
    __syncthreads();
    for (int s = threadIdx.x; s < sg.nseg; s += blockDim.x)
        if (!sg.seg_done[s]) atomicOr(&open, 1);
    __syncthreads();
    if (threadIdx.x == 0) {
        state->all_conv = open ? 0 : 1;
        if (init) {
            state->iter = 0;
            state->skip = 0;
        } else {
            state->iter += 1;
        }
    }
}

// pairs (P, AP) and (P, R): beta, alpha, breakdown detection; one work-group per system
__global__ __launch_bounds__(kScalarThreads) void k_cg_alpha(int64_t m, int nblk, const double *part, int freeze_converged, CgState *state,
                           CgCols cols, Segs sg) {
    const int skip = state->all_conv;
    if (blockIdx.x == 0 && threadIdx.x == 0) state->skip = skip;
    if (skip) return;
    const int s = blockIdx.x;
    const int done = sg.seg_done[s];
    for_columns(m, nblk, part, sg, s, [&](int64_t, int64_t e, double beta, double rho) {
        // an exactly zero residual is an exact solution: nothing to update
        int act = !done && !cols.frozen[e] && !(freeze_converged && cols.conv[e]) && cols.rr[e] > 0.0;
        double alpha = 0.0;
        if (act) {
            alpha = rho / beta;
            if (!(beta > 0.0) || !isfinite(alpha)) {
                cols.frozen[e] = 1;
                cols.status[e] = 1;
                act = 0;
                alpha = 0.0;
            }
        }
        cols.beta[e] = beta;
        cols.alpha[e] = alpha;
        cols.act[e] = act;
        return false;
    });
}

// x += alpha p, r -= alpha a for active columns; then partial sums of <a, r>, <r, r>
__global__ __launch_bounds__(256) void k_cg_update_xr(int64_t m, int nblk, Segs sg, double *X, double *R,
                                                      const double *P, const double *AP, double *part,
                                                      const CgState *state, CgCols cols) {
    if (state->skip) return;
    const int tid = threadIdx.x, rg = tid >> 5, jl = tid & 31;
    const int64_t j = (int64_t)blockIdx.y * kDotCols + jl;
    const int64_t r0 = sg.blk_r0[blockIdx.x], r1 = sg.blk_r0[blockIdx.x + 1];
    const int64_t e = (int64_t)sg.blk_seg[blockIdx.x] * m + j;
    // x += alpha p, r -= alpha Ap on open columns, then the partial sums of Ap . r
    // and r . r from the new r held in registers
    double s0 = 0.0, s1 = 0.0;
    if (j < m && r1 > r0) {
        const bool act = cols.act[e] != 0;
        const double a = act ? cols.alpha[e] : 0.0;
        for (int64_t i0 = r0 + rg; i0 < r1; i0 += 8 * kRowStep) {
            double xv[kRowStep], pv[kRowStep], rv[kRowStep], av[kRowStep];
#pragma unroll
            for (int u = 0; u < kRowStep; ++u) {
                const int64_t i = min(i0 + 8 * u, r1 - 1);
                rv[u] = R[i * m + j];
                av[u] = AP[i * m + j];
                if (act) {
                    xv[u] = X[i * m + j];
                    pv[u] = P[i * m + j];
                }
            }
#pragma unroll
            for (int u = 0; u < kRowStep; ++u) {
                const int64_t i = i0 + 8 * u;
                if (i < r1) {
                    double rn = rv[u];
                    if (act) {
                        X[i * m + j] = xv[u] + a * pv[u];
                        rn = rv[u] - a * av[u];
                        R[i * m + j] = rn;
                    }
                    s0 += av[u] * rn;
                    s1 += rn * rn;
                }
            }
        }
    }
    store_dots(s0, s1, m, nblk, true, part);
}

// gamma, convergence test; one work-group per system
__global__ __launch_bounds__(kScalarThreads) void k_cg_gamma(int64_t m, int nblk, const double *part, double rtol, const CgState *state, CgCols cols,
                           Segs sg) {
    if (state->skip) return;
    const int s = blockIdx.x;
    if (sg.seg_done[s]) return;  // uniform over the work-group
    const int it = state->iter + 1;
    const bool open = for_columns(m, nblk, part, sg, s, [&](int64_t, int64_t e, double ar, double rr) {
        cols.gamma[e] = cols.act[e] ? ar / cols.beta[e] : 0.0;
        cols.rr[e] = rr;
        const int c = sqrt(rr) <= rtol * cols.bnorm[e];
        cols.conv[e] = c;
        if (c && cols.first_conv[e] < 0) cols.first_conv[e] = it;
        return !c && !cols.frozen[e];
    });
    if (threadIdx.x == 0 && !open) {
        sg.seg_done[s] = 1;
        sg.seg_iters[s] = it;
    }
}

// p = r - gamma p for active columns
__global__ __launch_bounds__(256) void k_cg_update_p(int64_t m, Segs sg, const double *R, double *P,
                                                     const CgState *state, CgCols cols) {
    if (state->skip) return;
    const int tid = threadIdx.x, rg = tid >> 5, jl = tid & 31;
    const int64_t j = (int64_t)blockIdx.y * kDotCols + jl;
    const int64_t e = (int64_t)sg.blk_seg[blockIdx.x] * m + j;
    if (j >= m || !cols.act[e]) return;
    const double g = cols.gamma[e];
    for (int64_t i = sg.blk_r0[blockIdx.x] + rg; i < sg.blk_r0[blockIdx.x + 1]; i += 8)
        P[i * m + j] = R[i * m + j] - g * P[i * m + j];
}

// Residual replacement (mixed precision, one system): after every iteration the
// largest residual norm since the last replacement is tracked per column, and a
// replacement is requested (state->pad) once an open column's recursive residual
// has dropped below delta times that maximum.
__global__ void k_rel_track(int64_t m, double delta, CgState *state, CgCols cols, double *rmax) {
    __shared__ int want;
    if (state->skip) return;
    if (threadIdx.x == 0) want = 0;
    __syncthreads();
    for (int64_t j = threadIdx.x; j < m; j += blockDim.x) {
        if (cols.conv[j] || cols.frozen[j]) continue;
        const double rn = sqrt(cols.rr[j]);
        rmax[j] = fmax(rmax[j], rn);
        if (rn < delta * rmax[j]) atomicOr(&want, 1);
    }
    __syncthreads();
    if (threadIdx.x == 0 && want) state->pad = 1;
}

// The residual R was just recomputed as B - A X with the FP64 operator; the
// first pair of part holds its squared column norms (the second pair is not
// used).  Recursive norms, maxima and convergence restart from the true
// residual; the system stops when every column has converged (or broken down).
__global__ __launch_bounds__(kScalarThreads) void k_rel_replace(int64_t m, int nblk, const double *part, double rtol, CgState *state, CgCols cols,
                              Segs sg, double *rmax) {
    const bool open = for_columns(m, nblk, part, sg, 0, [&](int64_t, int64_t e, double rr, double) {
        cols.rr[e] = rr;
        // the best iterate so far: a strictly smaller true residual
        const int better = rr < cols.best[e];
        cols.keep[e] = better;
        if (better) cols.best[e] = rr;
        rmax[e] = sqrt(rr);
        const int c = sqrt(rr) <= rtol * cols.bnorm[e];
        cols.conv[e] = c;
        if (c && cols.first_conv[e] < 0) cols.first_conv[e] = state->iter;
        return !c && !cols.frozen[e];
    });
    if (threadIdx.x == 0) {
        sg.seg_done[0] = open ? 0 : 1;
        sg.seg_iters[0] = state->iter;
        state->all_conv = open ? 0 : 1;
        state->skip = 0;
        state->pad = 0;
    }
}

// Columns of X (n x m, leading dimension m) flagged in keep -> the same columns of Xb.
__global__ void k_keep_cols(int64_t n, int64_t m, const int32_t *__restrict__ keep, const double *__restrict__ X,
                            double *__restrict__ Xb) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * m) return;
    if (keep[e % m]) Xb[e] = X[e];
}

// End of a mixed-precision solve (the residual was just recomputed): a column whose best
// true residual is smaller than its current one gets its best iterate back (keep = 1)
// and the best residual; convergence follows the returned iterate.
__global__ void k_best_final(int64_t m, double rtol, CgCols cols) {
    for (int64_t j = threadIdx.x; j < m; j += blockDim.x) {
        const int back = cols.best[j] < cols.rr[j];
        cols.keep[j] = back;
        if (back) cols.rr[j] = cols.best[j];
        cols.conv[j] = sqrt(cols.rr[j]) <= rtol * cols.bnorm[j];
    }
}

// Rows of the concatenated systems: operator j owns rows [row0[j], row0[j] + n_j)
// (its own original or tree order); its systems follow in order.
struct Layout {
    std::vector<int64_t> row0;
    std::vector<int32_t> seg0;  // first system of each operator
    std::vector<int64_t> blk_r0;
    std::vector<int32_t> blk_seg, seg_blk;
    int64_t n = 0;
    int32_t nseg = 0, nblk = 0;
    size_t mm_bytes = 0;
};

Layout make_layout(const DevMat *const *mats, int32_t nmat, int64_t m) {
    Layout L;
    L.seg_blk.push_back(0);
    for (int32_t q = 0; q < nmat; ++q) {
        const DevMat &dm = *mats[q];
        const Plan &P = *dm.plan;
        L.row0.push_back(L.n);
        L.seg0.push_back(L.nseg);
        for (int32_t s = 0; s < P.nsys(); ++s) {
            const int64_t a = L.n + P.sys_row[s], ns = P.sys_row[s + 1] - P.sys_row[s];
            const int64_t nb = std::min<int64_t>(1024, std::max<int64_t>(1, (ns + 63) / 64));
            const int64_t rows = (ns + nb - 1) / nb;
            for (int64_t b = 0; b < nb; ++b) {
                L.blk_r0.push_back(a + std::min(ns, b * rows));
                L.blk_seg.push_back(L.nseg);
            }
            ++L.nseg;
            L.seg_blk.push_back((int32_t)L.blk_seg.size());
        }
        L.n += dm.n;
        L.mm_bytes = std::max(L.mm_bytes, matmul_ws_bytes(dm, m));
    }
    L.blk_r0.push_back(L.n);
    L.nblk = (int32_t)L.blk_seg.size();
    return L;
}

struct CgWs {
    double *Bt, *Xt, *R, *P, *AP, *part, *rmax, *Xb;
    CgState *state;
    CgCols cols;
    int64_t *blk_r0;
    int32_t *blk_seg, *seg_blk, *seg_done, *seg_iters;
    char *mm;
    size_t bytes;
};

// keep_best: mixed precision, with room for the best iterate (tree order)
CgWs cg_layout(const Layout &L, int64_t m, char *base, bool keep_best = false) {
    CgWs w{};
    size_t off = 0;
    auto carve = [&](size_t bytes) {
        off = align_up(off);
        char *p = base ? base + off : nullptr;
        off += bytes;
        return p;
    };
    const size_t nm = (size_t)L.n * m * sizeof(double), sm = (size_t)L.nseg * m;
    w.Bt = (double *)carve(nm);
    w.Xt = (double *)carve(nm);
    w.R = (double *)carve(nm);
    w.P = (double *)carve(nm);
    w.AP = (double *)carve(nm);
    w.Xb = keep_best ? (double *)carve(nm) : nullptr;
    w.part = (double *)carve(2 * (size_t)L.nblk * m * sizeof(double));
    w.rmax = (double *)carve(sm * sizeof(double));
    w.state = (CgState *)carve(sizeof(CgState));
    double **dcols[6] = {&w.cols.bnorm, &w.cols.rr, &w.cols.beta, &w.cols.alpha, &w.cols.gamma, &w.cols.best};
    for (auto d : dcols) *d = (double *)carve(sm * sizeof(double));
    int32_t **icols[6] = {&w.cols.frozen, &w.cols.conv, &w.cols.first_conv, &w.cols.status, &w.cols.act,
                          &w.cols.keep};
    for (auto d : icols) *d = (int32_t *)carve(sm * sizeof(int32_t));
    w.blk_r0 = (int64_t *)carve((L.nblk + 1) * sizeof(int64_t));
    w.blk_seg = (int32_t *)carve(L.nblk * sizeof(int32_t));
    w.seg_blk = (int32_t *)carve((L.nseg + 1) * sizeof(int32_t));
    w.seg_done = (int32_t *)carve(L.nseg * sizeof(int32_t));
    w.seg_iters = (int32_t *)carve(L.nseg * sizeof(int32_t));
    w.mm = carve(L.mm_bytes);
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

// columns flagged in keep: X (leading dimension ldx) -> Xb (leading dimension m) when
// to_best, Xb -> X otherwise
__global__ void k_copy_cols_ld(int64_t n, int64_t m, const int32_t *__restrict__ keep, double *__restrict__ X,
                               int64_t ldx, double *__restrict__ Xb, int to_best) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * m) return;
    const int64_t i = e / m, j = e % m;
    if (!keep[j]) return;
    if (to_best) Xb[e] = X[i * ldx + j];
    else X[i * ldx + j] = Xb[e];
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
    double *B, *R, *D, *part, *norms, *Xb;
    int32_t *keep;
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
    w.Xb = (double *)carve(nm);
    w.part = (double *)carve(2 * (size_t)w.nblk * m * sizeof(double));
    w.norms = (double *)carve(2 * m * sizeof(double));
    w.keep = (int32_t *)carve(m * sizeof(int32_t));
    w.mm = carve(matmul_ws_bytes(hi, m));
    w.cg = carve(cg_ws_bytes(lo, m));
    w.bytes = align_up(off);
    return w;
}

}  // namespace

size_t cg_batch_ws_bytes(const DevMat *const *mats, int32_t nmat, int64_t m) {
    return cg_layout(make_layout(mats, nmat, m), m, nullptr).bytes;
}

size_t cg_ws_bytes(const DevMat &dm, int64_t m) {
    const DevMat *p = &dm;
    return cg_batch_ws_bytes(&p, 1, m);
}

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
    std::vector<double> norms(2 * m), best(m, HUGE_VAL);
    std::vector<int32_t> keep(m);
    // columns flagged in keep: X -> Xb (to_best) or Xb -> X
    auto copy_cols = [&](bool to_best) {
        hipError_t e = hipMemcpyAsync(w.keep, keep.data(), m * sizeof(int32_t), hipMemcpyHostToDevice, st);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_copy_cols_ld, dim3(g1), dim3(256), 0, st, n, m, (const int32_t *)w.keep, X, ldx, w.Xb,
                           to_best ? 1 : 0);
        return hipGetLastError();
    };
    int32_t outer = 0, inner_total = 0, stalls = 0;
    double prev = HUGE_VAL;
    for (;;) {
        // R = B - A X in FP64; squared norms of R and B
        hipLaunchKernelGGL(k_copy, dim3(g1), dim3(256), 0, st, nm, (const double *)w.B, w.R);
        hipError_t e = run_matmul(hi, m, -1.0, X, ldx, 1.0, w.R, m, false, w.mm, st);
        if (e != hipSuccess) return fail(e);
        hipLaunchKernelGGL(k_dots, gd, dim3(256), 0, st, n, m, w.nblk, w.R, w.R, w.B, w.B, w.part);
        hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(256), 0, st, m, w.nblk, w.part, w.norms);
        e = hipMemcpyAsync(norms.data(), w.norms, 2 * m * sizeof(double), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) return fail(e);
        bool done = true, better = false;
        double worst = 0.0;
        for (int64_t j = 0; j < m; ++j) {
            const double bn = std::sqrt(norms[m + j]), rn = std::sqrt(norms[j]);
            if (rn > rtol * bn) done = false;
            worst = std::max(worst, bn > 0 ? rn / bn : rn);
            // the best outer iterate of every column (smallest true residual) is kept
            keep[j] = norms[j] < best[j];
            if (keep[j]) {
                best[j] = norms[j];
                better = true;
            }
        }
        if (better && (e = copy_cols(true)) != hipSuccess) return fail(e);
        // a step that does not halve the worst relative residual is a stall; two stalls stop
        if (worst > 0.5 * prev) ++stalls;
        prev = worst;
        if (done || outer >= max_outer || stalls >= 2) break;
        // A_lo D = R by block CG, then X += D
        hipLaunchKernelGGL(k_zero, dim3(g1), dim3(256), 0, st, nm, w.D);
        h2x_cg_info ii{};
        h2x_status s = run_block_cg(lo, inner, m, w.R, m, w.D, m, w.cg, cg_ws_bytes(lo, m), &ii, st);
        if (s != H2X_OK) return s;
        inner_total += ii.iters;
        hipLaunchKernelGGL(k_axpy_ld, dim3(g1), dim3(256), 0, st, n, m, w.D, X, ldx);
        ++outer;
    }
    // every column returns its best outer iterate
    bool back = false;
    for (int64_t j = 0; j < m; ++j) {
        keep[j] = best[j] < norms[j];
        if (keep[j]) {
            norms[j] = best[j];
            back = true;
        }
    }
    if (back) {
        hipError_t e = copy_cols(false);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) return fail(e);
    }
    int32_t status = H2X_OK;
    for (int64_t j = 0; j < m; ++j) {
        const double rn = std::sqrt(norms[j]), bn = std::sqrt(norms[m + j]);
        if (!((bn > 0 ? rn / bn : rn) <= rtol)) status = H2X_ENOCONV;
    }
    if (info) {
        info->iters = inner_total;
        info->outer_iters = outer;
        info->status = status;
        if (info->sys_iters) info->sys_iters[0] = inner_total;
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

h2x_status run_block_cg_batch(const DevMat *const *mats, int32_t nmat, const h2x_cg_params &prm, int64_t m,
                              const double *B, int64_t ldb, double *X, int64_t ldx, char *ws, size_t ws_bytes,
                              h2x_cg_info *info, hipStream_t st, const DevMat *hi, double delta) {
    Layout L = make_layout(mats, nmat, m);
    if (hi) L.mm_bytes = std::max(L.mm_bytes, matmul_ws_bytes(*hi, m));
    CgWs w = cg_layout(L, m, ws, hi != nullptr);
    if (ws_bytes < w.bytes) {
        set_error("h2x_block_cg: workspace too small");
        return H2X_ENOMEM;
    }
    const int64_t n = L.n, nm = n * m;
    const unsigned g1 = (unsigned)((nm + 255) / 256);
    const int nblk = L.nblk;
    const dim3 gd(nblk, (unsigned)((m + kDotCols - 1) / kDotCols));
    const Segs sg{w.blk_r0, w.blk_seg, w.seg_blk, w.seg_done, w.seg_iters, L.nseg};
    hipStream_t cs = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipEvent_t ev = nullptr;
    auto cleanup = [&]() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (ev) (void)hipEventDestroy(ev);
        if (cs) (void)hipStreamDestroy(cs);
        exec = nullptr;
        graph = nullptr;
        ev = nullptr;
        cs = nullptr;
    };
    auto fail = [&](hipError_t e) {
        cleanup();
        set_error(std::string("h2x_block_cg: ") + hipGetErrorString(e));
        return H2X_EHIP;
    };
    hipError_t e = hipMemcpyAsync(w.blk_r0, L.blk_r0.data(), L.blk_r0.size() * sizeof(int64_t),
                                  hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(w.blk_seg, L.blk_seg.data(), L.blk_seg.size() * sizeof(int32_t), hipMemcpyHostToDevice,
                           st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(w.seg_blk, L.seg_blk.data(), L.seg_blk.size() * sizeof(int32_t), hipMemcpyHostToDevice,
                           st);
    if (e != hipSuccess) return fail(e);

    // the product of one iteration, operator by operator on its own rows; with
    // skip, the clusters of systems that have stopped are left out
    auto product = [&](const double *Pv, double *APv, double alpha, double beta, bool skip, hipStream_t s) {
        for (int32_t q = 0; q < nmat; ++q) {
            const int64_t r = L.row0[q] * m;
            hipError_t ee = run_matmul(*mats[q], m, alpha, Pv + r, m, beta, APv + r, m, true, w.mm, s, nullptr,
                                       skip ? w.seg_done + L.seg0[q] : nullptr);
            if (ee != hipSuccess) return ee;
        }
        return hipSuccess;
    };
    auto iteration = [&](hipStream_t s) {
        hipError_t ee = product(w.P, w.AP, 1.0, 0.0, true, s);
        if (ee != hipSuccess) return ee;
        hipLaunchKernelGGL(k_sdots, gd, dim3(256), 0, s, m, nblk, sg, w.P, w.AP, w.P, w.R, w.part,
                           (const CgState *)w.state);
        hipLaunchKernelGGL(k_cg_alpha, dim3(L.nseg), dim3(kScalarThreads), 0, s, m, nblk, w.part, prm.freeze_converged,
                           w.state, w.cols, sg);
        hipLaunchKernelGGL(k_cg_update_xr, gd, dim3(256), 0, s, m, nblk, sg, w.Xt, w.R, w.P, w.AP, w.part,
                           (const CgState *)w.state, w.cols);
        hipLaunchKernelGGL(k_cg_gamma, dim3(L.nseg), dim3(kScalarThreads), 0, s, m, nblk, w.part, prm.rtol,
                           (const CgState *)w.state, w.cols, sg);
        hipLaunchKernelGGL(k_cg_state, dim3(1), dim3(256), 0, s, 0, w.state, sg);
        hipLaunchKernelGGL(k_cg_update_p, gd, dim3(256), 0, s, m, sg, w.R, w.P, (const CgState *)w.state, w.cols);
        if (hi) hipLaunchKernelGGL(k_rel_track, dim3(1), dim3(256), 0, s, m, delta, w.state, w.cols, w.rmax);
        return hipGetLastError();
    };
    // mixed precision: R = B - A X with the FP64 operator, recursive quantities restart from it
    auto replace = [&](hipStream_t s) {
        hipLaunchKernelGGL(k_copy, dim3(g1), dim3(256), 0, s, nm, (const double *)w.Bt, w.R);
        hipError_t ee = run_matmul(*hi, m, -1.0, w.Xt, m, 1.0, w.R, m, true, w.mm, s);
        if (ee != hipSuccess) return ee;
        hipLaunchKernelGGL(k_sdots, gd, dim3(256), 0, s, m, nblk, sg, w.R, w.R, (const double *)nullptr,
                           (const double *)nullptr, w.part, (const CgState *)nullptr);
        hipLaunchKernelGGL(k_rel_replace, dim3(1), dim3(kScalarThreads), 0, s, m, nblk, (const double *)w.part, prm.rtol,
                           w.state, w.cols, sg, w.rmax);
        hipLaunchKernelGGL(k_keep_cols, dim3(g1), dim3(256), 0, s, n, m, (const int32_t *)w.cols.keep,
                           (const double *)w.Xt, w.Xb);
        return hipGetLastError();
    };

    for (int32_t q = 0; q < nmat; ++q) {
        const DevMat &dm = *mats[q];
        const int64_t r = L.row0[q];
        const unsigned gq = (unsigned)((dm.n * m + 255) / 256);
        hipLaunchKernelGGL(k_gather_rows, dim3(gq), dim3(256), 0, st, dm.n, m, dm.perm, B + r * ldb, ldb,
                           w.Bt + r * m, m);
        hipLaunchKernelGGL(k_gather_rows, dim3(gq), dim3(256), 0, st, dm.n, m, dm.perm, (const double *)X + r * ldx,
                           ldx, w.Xt + r * m, m);
    }
    // R = B - A X0 (with the FP64 operator in mixed precision), P = R
    hipLaunchKernelGGL(k_copy, dim3(g1), dim3(256), 0, st, nm, w.Bt, w.R);
    e = hi ? run_matmul(*hi, m, -1.0, w.Xt, m, 1.0, w.R, m, true, w.mm, st) : product(w.Xt, w.R, -1.0, 1.0, false, st);
    if (e != hipSuccess) return fail(e);
    hipLaunchKernelGGL(k_copy, dim3(g1), dim3(256), 0, st, nm, w.R, w.P);
    hipLaunchKernelGGL(k_sdots, gd, dim3(256), 0, st, m, nblk, sg, w.Bt, w.Bt, w.R, w.R, w.part,
                       (const CgState *)nullptr);
    hipLaunchKernelGGL(k_cg_init, dim3(L.nseg), dim3(kScalarThreads), 0, st, m, nblk, w.part, prm.rtol, w.cols, sg);
    hipLaunchKernelGGL(k_cg_state, dim3(1), dim3(256), 0, st, 1, w.state, sg);
    if (hi) {
        hipLaunchKernelGGL(k_sdots, gd, dim3(256), 0, st, m, nblk, sg, w.R, w.R, (const double *)nullptr,
                           (const double *)nullptr, w.part, (const CgState *)nullptr);
        hipLaunchKernelGGL(k_rel_replace, dim3(1), dim3(kScalarThreads), 0, st, m, nblk, (const double *)w.part, prm.rtol,
                           w.state, w.cols, sg, w.rmax);
        hipLaunchKernelGGL(k_keep_cols, dim3(g1), dim3(256), 0, st, n, m, (const int32_t *)w.cols.keep,
                           (const double *)w.Xt, w.Xb);
    }

    const int check = prm.check_every > 0 ? prm.check_every : 1;
    hipStream_t run = st;
    if (prm.graph) {
        // check_every iterations captured once into one graph on a private stream
        // (the caller's stream may be the null stream, which cannot be captured)
        e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventRecord(ev, st);
        if (e == hipSuccess) e = hipStreamWaitEvent(cs, ev, 0);
        if (e == hipSuccess) e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return fail(e);
        for (int c = 0; c < check && e == hipSuccess; ++c) e = iteration(cs);
        hipError_t e2 = hipStreamEndCapture(cs, &graph);
        if (e == hipSuccess) e = e2;
        if (e == hipSuccess) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        if (e != hipSuccess) return fail(e);
        run = cs;
    }
    CgState hs{};
    int32_t replaced = 0, rep_it = 0;
    auto read_state = [&]() {
        hipError_t ee = hipMemcpyAsync(&hs, w.state, sizeof(CgState), hipMemcpyDeviceToHost, run);
        if (ee == hipSuccess) ee = hipStreamSynchronize(run);
        return ee;
    };
    for (int32_t it = 0;;) {
        e = read_state();
        if (e != hipSuccess) return fail(e);
        // mixed precision: replace the residual when asked, and before stopping
        if (hi && it != rep_it && (hs.pad || hs.all_conv || it >= prm.max_iter)) {
            e = replace(run);
            if (e == hipSuccess) e = read_state();
            if (e != hipSuccess) return fail(e);
            ++replaced;
            rep_it = it;
        }
        if (hs.all_conv || it >= prm.max_iter) break;
        if (exec && it + check <= prm.max_iter) {
            e = hipGraphLaunch(exec, run);
            it += check;
        } else {
            const int steps = (int)std::min<int64_t>(check, prm.max_iter - it);
            for (int c = 0; c < steps && e == hipSuccess; ++c) e = iteration(run);
            it += steps;
        }
        if (e != hipSuccess) return fail(e);
    }
    if (run != st) {
        e = hipStreamSynchronize(run);
        if (e != hipSuccess) return fail(e);
    }
    if (hi) {
        // every column returns its iterate with the smallest recomputed true residual
        hipLaunchKernelGGL(k_best_final, dim3(1), dim3(256), 0, st, m, prm.rtol, w.cols);
        hipLaunchKernelGGL(k_keep_cols, dim3(g1), dim3(256), 0, st, n, m, (const int32_t *)w.cols.keep,
                           (const double *)w.Xb, w.Xt);
    }
    for (int32_t q = 0; q < nmat; ++q) {
        const DevMat &dm = *mats[q];
        const int64_t r = L.row0[q];
        const unsigned gq = (unsigned)((dm.n * m + 255) / 256);
        hipLaunchKernelGGL(k_scatter_rows, dim3(gq), dim3(256), 0, st, dm.n, m, dm.perm, w.Xt + r * m, m,
                           X + r * ldx, ldx);
    }
    const size_t sm = (size_t)L.nseg * m;
    std::vector<double> rr(sm), bn(sm);
    std::vector<int32_t> fc(sm), stt(sm), cv(sm), si(L.nseg), sd(L.nseg);
    e = hipMemcpyAsync(&hs, w.state, sizeof(CgState), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipMemcpyAsync(rr.data(), w.cols.rr, sm * sizeof(double), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipMemcpyAsync(bn.data(), w.cols.bnorm, sm * sizeof(double), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipMemcpyAsync(fc.data(), w.cols.first_conv, sm * 4, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipMemcpyAsync(stt.data(), w.cols.status, sm * 4, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipMemcpyAsync(cv.data(), w.cols.conv, sm * 4, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipMemcpyAsync(si.data(), w.seg_iters, L.nseg * 4, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipMemcpyAsync(sd.data(), w.seg_done, L.nseg * 4, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return fail(e);
    cleanup();
    int32_t status = H2X_OK;
    for (size_t j = 0; j < sm; ++j) {
        if (stt[j] == 0 && !cv[j]) stt[j] = 2;
        if (stt[j] == 1) status = H2X_EBREAKDOWN;
        else if (stt[j] == 2 && status == H2X_OK) status = H2X_ENOCONV;
    }
    if (info) {
        info->iters = hs.iter;
        info->status = status;
        info->outer_iters = replaced;
        for (size_t j = 0; j < sm; ++j) {
            const int32_t cap = sd[j / m] ? si[j / m] : hs.iter;
            if (info->col_relres) info->col_relres[j] = bn[j] > 0 ? std::sqrt(rr[j]) / bn[j] : std::sqrt(rr[j]);
            if (info->col_iters) info->col_iters[j] = fc[j] >= 0 ? fc[j] : cap;
            if (info->col_status) info->col_status[j] = stt[j];
        }
        if (info->sys_iters)
            for (int32_t s = 0; s < L.nseg; ++s) info->sys_iters[s] = sd[s] ? si[s] : hs.iter;
    }
    return H2X_OK;
}

h2x_status run_block_cg(const DevMat &dm, const h2x_cg_params &prm, int64_t m, const double *B, int64_t ldb,
                        double *X, int64_t ldx, char *ws, size_t ws_bytes, h2x_cg_info *info, hipStream_t st) {
    const DevMat *p = &dm;
    return run_block_cg_batch(&p, 1, prm, m, B, ldb, X, ldx, ws, ws_bytes, info, st, nullptr, 0.0);
}

size_t mixed_ws_bytes(const DevMat &hi, const DevMat &lo, int64_t m) {
    const DevMat *p = &lo;
    Layout L = make_layout(&p, 1, m);
    L.mm_bytes = std::max(L.mm_bytes, matmul_ws_bytes(hi, m));
    return cg_layout(L, m, nullptr, true).bytes;
}

h2x_status run_block_cg_mixed(const DevMat &hi, const DevMat &lo, const h2x_cg_params &prm, double delta, int64_t m,
                              const double *B, int64_t ldb, double *X, int64_t ldx, char *ws, size_t ws_bytes,
                              h2x_cg_info *info, hipStream_t st) {
    const DevMat *p = &lo;
    return run_block_cg_batch(&p, 1, prm, m, B, ldb, X, ldx, ws, ws_bytes, info, st, &hi, delta);
}

}  // namespace h2x
