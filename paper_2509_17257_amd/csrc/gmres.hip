// Block GMRES(ell) without a preconditioner (section 5.2, block form of the
// generalized minimal residual method with M = I): m independent GMRES
// processes that share one H^2 x Q product per Arnoldi step.  Per column i and
// cycle: r = b - A x, rhat = ||r|| e_0, q_0 = r / ||r||; step k: a = A q_k,
// h[j][k] = <q_j, a> for j <= k (classical Gram-Schmidt: all projections taken
// from the same a), a -= sum_j q_j h[j][k], h[k+1][k] = ||a||, q_{k+1} =
// a / h[k+1][k]; the earlier Givens rotations are applied to column k of h and a
// new one zeroes h[k+1][k] (applied to h and rhat).  A column closes once
// |rhat[k+1]| <= rtol ||b_i|| (a vanishing direction gives rhat[k+1] = 0); a zero
// pivot is a breakdown and that step is not used.  At the end of a cycle every
// column solves R y = rhat with its own number of steps and sets x += V y; the
// next cycle restarts from the improved x.
//
// The iteration runs in tree order on packed n x m blocks (ld = m): B, X and the
// basis q_0..q_ell.  Dot products and norms are reduced in two fixed-order
// passes (per row block, then per column), so the solve is bitwise
// reproducible.  The Hessenberg columns, rotations and rhat of every column stay
// on the device; once no column is open the remaining kernels of the cycle and
// the products (through the per-system skip flag) do nothing, and the host reads
// that flag every check_every steps.
//
// The kernels are templates on the field: double for a real operator, a complex
// pair for the complex (Helmholtz) operator.  Over C the inner product is
// <u, v> = u^H v and the rotations are G = [c s; -conj(s) c] with c real: for
// (u, w), w = h[k+1][k] >= 0, rho = sqrt(|u|^2 + w^2), c = |u| / rho and
// s = (u / |u|) w / rho (c = 0, s = 1 when u = 0), so G (u, w) = (rho u / |u|, 0).
// Over R the rotation keeps the sign in c: c = u / rho, s = w / rho, G (u, w) = (rho, 0).
// A complex column occupies two real columns (real, imaginary part) of the
// n x m blocks, so the product and the row permutations work on real columns.
#include <cmath>
#include <vector>

#include "device.hpp"

namespace h2x {

namespace {

constexpr int kCols = 32;    // columns per work-group in the row-block kernels
constexpr int kRowGroups = 8;  // 256 threads = 8 row groups x 32 columns
constexpr int kRowsPerBlk = 128;
constexpr int kRowsPerThread = kRowsPerBlk / kRowGroups;

struct cpx {  // complex double: real part x, imaginary part y
    double x, y;
};

// field operations: conjugated product (conj(a) b), product, difference, |a|^2, ...
__device__ inline double f_zero(double) { return 0.0; }
__device__ inline cpx f_zero(cpx) { return cpx{0.0, 0.0}; }
__device__ inline double f_of(double, double v) { return v; }
__device__ inline cpx f_of(cpx, double v) { return cpx{v, 0.0}; }
__device__ inline double f_add(double a, double b) { return a + b; }
__device__ inline cpx f_add(cpx a, cpx b) { return cpx{a.x + b.x, a.y + b.y}; }
__device__ inline double f_sub(double a, double b) { return a - b; }
__device__ inline cpx f_sub(cpx a, cpx b) { return cpx{a.x - b.x, a.y - b.y}; }
__device__ inline double f_mul(double a, double b) { return a * b; }
__device__ inline cpx f_mul(cpx a, cpx b) { return cpx{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }
__device__ inline double f_cmul(double a, double b) { return a * b; }
__device__ inline cpx f_cmul(cpx a, cpx b) { return cpx{a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x}; }
__device__ inline double f_conj(double a) { return a; }
__device__ inline cpx f_conj(cpx a) { return cpx{a.x, -a.y}; }
__device__ inline double f_scale(double a, double s) { return a * s; }
__device__ inline cpx f_scale(cpx a, double s) { return cpx{a.x * s, a.y * s}; }
__device__ inline double f_abs2(double a) { return a * a; }
__device__ inline double f_abs2(cpx a) { return a.x * a.x + a.y * a.y; }
__device__ inline double f_abs(double a) { return fabs(a); }
__device__ inline double f_abs(cpx a) { return hypot(a.x, a.y); }
__device__ inline double f_div(double a, double b) { return a / b; }
__device__ inline cpx f_div(cpx a, cpx b) {
    const double d = b.x * b.x + b.y * b.y;
    return cpx{(a.x * b.x + a.y * b.y) / d, (a.y * b.x - a.x * b.y) / d};
}
__device__ inline double f_shfl_xor(double v, int d) { return __shfl_xor(v, d, 64); }
__device__ inline cpx f_shfl_xor(cpx v, int d) { return cpx{__shfl_xor(v.x, d, 64), __shfl_xor(v.y, d, 64)}; }

// The rotation that zeroes w under u: c, s and the new diagonal entry.  Returns false
// for a zero pivot (u = w = 0).
__device__ inline bool givens(double u, double w, double &c, double &s, double &r) {
    const double rho = hypot(u, w);
    if (rho == 0.0) return false;
    c = u / rho;
    s = w / rho;
    r = rho;
    return true;
}
__device__ inline bool givens(cpx u, double w, double &c, cpx &s, cpx &r) {
    const double au = hypot(u.x, u.y), rho = sqrt(au * au + w * w);
    if (rho == 0.0) return false;
    if (au == 0.0) {
        c = 0.0;
        s = cpx{1.0, 0.0};
    } else {
        c = au / rho;
        s = cpx{u.x / au * (w / rho), u.y / au * (w / rho)};
    }
    r = f_add(f_scale(u, c), f_scale(s, w));
    return true;
}

struct GmState {
    int32_t done;   // no column open: the rest of the cycle is skipped (first member: the skip flag)
    int32_t steps;  // Arnoldi steps run
    int32_t pad[2];
};

template <typename T>
struct GmCols {  // per-column data, m columns of the field
    double *bn;   // ||b_i||
    T *H;         // (ell + 1) x ell per column, row-major
    double *cs;   // rotations: c, ell per column
    T *sn;        //            s, ell per column
    T *rh;        // rhat, ell + 1 per column
    T *y;         // least-squares coefficients, ell per column
    double *inv;  // scale of the new basis vector (0 for a closed column)
    double *est;  // |rhat[k_i]| / ||b_i|| after the column's last cycle
    double *nrm2; // squared column norms of the latest norm pass
    int32_t *open, *done, *kc, *iters, *status;
};

// part[(j * nblk + blk) * m + c] = sum over the rows of block blk of conj(Q_j[r][c]) a[r][c];
// projection j = blockIdx.z (0..k)
template <typename T>
__global__ __launch_bounds__(256) void k_gm_dots(int64_t n, int64_t m, const T *__restrict__ Q,
                                                 const T *__restrict__ a, T *__restrict__ part,
                                                 const GmState *__restrict__ st) {
    if (st->done) return;
    __shared__ T red[kRowGroups][kCols];
    const int tid = threadIdx.x, rg = tid / kCols, jl = tid % kCols;
    const int64_t blk = blockIdx.x, nblk = gridDim.x, c = (int64_t)blockIdx.y * kCols + jl, j = blockIdx.z;
    const int64_t r0 = blk * kRowsPerBlk, r1 = min(n, r0 + kRowsPerBlk);
    const T *q = Q + j * n * m;
    // every load unconditional from a clamped address; out-of-range terms add an exact zero
    T s = f_zero(T{});
    const int64_t cc = min(c, m - 1);
    T qv[kRowsPerThread], av[kRowsPerThread];
#pragma unroll
    for (int u = 0; u < kRowsPerThread; ++u) {
        const int64_t r = min(r0 + rg + kRowGroups * u, r1 - 1);
        qv[u] = q[r * m + cc];
        av[u] = a[r * m + cc];
    }
#pragma unroll
    for (int u = 0; u < kRowsPerThread; ++u) {
        const int64_t r = r0 + rg + kRowGroups * u;
        if (c < m && r < r1) s = f_add(s, f_cmul(qv[u], av[u]));
    }
    red[rg][jl] = s;
    __syncthreads();
    if (rg == 0 && c < m) {
        T t = f_zero(T{});
        for (int g = 0; g < kRowGroups; ++g) t = f_add(t, red[g][jl]);
        part[(j * nblk + blk) * m + c] = t;
    }
}

// Sum of the nblk partials part[(b * stride) + off] in a fixed order by one wave:
// lane l adds b = l, l + 64, ... in turn, then a fixed butterfly; lane 0's value is
// the result (the same on every run).
template <typename T>
__device__ inline T wave_sum(const T *__restrict__ part, int64_t nblk, int64_t stride, int64_t off) {
    const int lane = threadIdx.x & 63;
    T v = f_zero(T{});
    for (int64_t b = lane; b < nblk; b += 64) v = f_add(v, part[b * stride + off]);
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v = f_add(v, f_shfl_xor(v, d));
    return v;
}

// H[c][j][k] = sum over row blocks of part, open columns only; one wave per (j, c)
template <typename T>
__global__ __launch_bounds__(256) void k_gm_hcol(int64_t m, int64_t nblk, int k, int ell,
                                                 const T *__restrict__ part, GmCols<T> cl,
                                                 const GmState *__restrict__ st) {
    if (st->done) return;
    const int64_t e = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    if (e >= (int64_t)(k + 1) * m) return;
    const int64_t j = e / m, c = e % m;
    if (!cl.open[c]) return;
    const T s = wave_sum(part + j * nblk * m, nblk, m, c);
    if ((threadIdx.x & 63) == 0) cl.H[(c * (ell + 1) + j) * ell + k] = s;
}

// nrm2[c] = sum over row blocks of part2 (squared norms); one wave per column
template <typename T>
__global__ __launch_bounds__(256) void k_gm_colsum(int64_t m, int64_t nblk, const double *__restrict__ part2,
                                                   GmCols<T> cl, const GmState *__restrict__ st, int always) {
    if (!always && st->done) return;
    const int64_t c = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    if (c >= m) return;
    const double s = wave_sum(part2, nblk, m, c);
    if ((threadIdx.x & 63) == 0) cl.nrm2[c] = s;
}

// a -= sum_{j <= k} Q_j h[j][k] on the open columns (k < 0: no subtraction, every
// column), then the partial sums of |a|^2: part2[blk * m + c]
template <typename T>
__global__ __launch_bounds__(256) void k_gm_update(int64_t n, int64_t m, int k, int ell, const T *__restrict__ Q,
                                                   T *__restrict__ a, GmCols<T> cl, double *__restrict__ part2,
                                                   const GmState *__restrict__ st) {
    if (k >= 0 && st->done) return;
    __shared__ double red[kRowGroups][kCols];
    const int tid = threadIdx.x, rg = tid / kCols, jl = tid % kCols;
    const int64_t blk = blockIdx.x, c = (int64_t)blockIdx.y * kCols + jl;
    const int64_t r0 = blk * kRowsPerBlk, r1 = min(n, r0 + kRowsPerBlk);
    const bool sub = k >= 0 && c < m && cl.open[c];
    T av[kRowsPerThread];
#pragma unroll
    for (int u = 0; u < kRowsPerThread; ++u) {
        const int64_t r = r0 + rg + kRowGroups * u;
        av[u] = (c < m && r < r1) ? a[r * m + c] : f_zero(T{});
    }
    if (sub) {
        // rows past the block read the block's last row (every load unconditional, so the
        // loads of the next basis vectors are in flight during the current one's updates);
        // their values are never stored or counted.  JU basis vectors per pass, each
        // subtracted in order j = 0, 1, ..., k as in the plain loop.
        constexpr int JU = sizeof(T) > sizeof(double) ? 2 : 4;
        int64_t ro[kRowsPerThread];
#pragma unroll
        for (int u = 0; u < kRowsPerThread; ++u) ro[u] = min(r0 + rg + kRowGroups * u, r1 - 1) * m + c;
        for (int j0 = 0; j0 <= k; j0 += JU) {
            T qv[JU][kRowsPerThread], h[JU];
#pragma unroll
            for (int jj = 0; jj < JU; ++jj) {
                const int j = min(j0 + jj, k);
                const T *q = Q + (int64_t)j * n * m;
                h[jj] = cl.H[(c * (ell + 1) + j) * ell + k];
#pragma unroll
                for (int u = 0; u < kRowsPerThread; ++u) qv[jj][u] = q[ro[u]];
            }
#pragma unroll
            for (int jj = 0; jj < JU; ++jj)
                if (j0 + jj <= k)
#pragma unroll
                    for (int u = 0; u < kRowsPerThread; ++u) av[u] = f_sub(av[u], f_mul(qv[jj][u], h[jj]));
        }
    }
    double s = 0.0;
#pragma unroll
    for (int u = 0; u < kRowsPerThread; ++u) {
        const int64_t r = r0 + rg + kRowGroups * u;
        if (c < m && r < r1) {
            s += f_abs2(av[u]);
            if (sub) a[r * m + c] = av[u];
        }
    }
    red[rg][jl] = s;
    __syncthreads();
    if (rg == 0 && c < m) {
        double t = 0.0;
        for (int g = 0; g < kRowGroups; ++g) t += red[g][jl];
        part2[blk * m + c] = t;
    }
}

// One work-group: ||b_i|| (nrm2 holds the squared norms of B) and the per-column
// state before the first cycle.
template <typename T>
__global__ void k_gm_init(int64_t m, GmCols<T> cl, GmState *st) {
    for (int64_t c = threadIdx.x; c < m; c += blockDim.x) {
        cl.bn[c] = sqrt(cl.nrm2[c]);
        cl.done[c] = 0;
        cl.open[c] = 0;
        cl.kc[c] = 0;
        cl.iters[c] = 0;
        cl.status[c] = 2;
        cl.est[c] = 0.0;
    }
    if (threadIdx.x == 0) {
        st->done = 0;
        st->steps = 0;
    }
}

// One work-group, start of a cycle: nrm2 holds the squared norms of r = b - A x.
// Columns within the bound are done; the others open with rhat = ||r|| e_0.
template <typename T>
__global__ void k_gm_start(int64_t m, int ell, double rtol, GmCols<T> cl, GmState *st) {
    __shared__ int any;
    if (threadIdx.x == 0) any = 0;
    __syncthreads();
    for (int64_t c = threadIdx.x; c < m; c += blockDim.x) {
        cl.open[c] = 0;
        cl.kc[c] = 0;
        cl.inv[c] = 0.0;
        if (cl.done[c]) continue;
        const double beta = sqrt(cl.nrm2[c]);
        if (beta <= rtol * cl.bn[c]) {
            cl.done[c] = 1;
            cl.status[c] = 0;
            continue;
        }
        cl.open[c] = 1;
        T *rh = cl.rh + c * (ell + 1);
        rh[0] = f_of(T{}, beta);
        for (int r = 1; r <= ell; ++r) rh[r] = f_zero(T{});
        cl.inv[c] = 1.0 / beta;
        any = 1;  // every writer stores the same value
    }
    __syncthreads();
    if (threadIdx.x == 0) st->done = any ? 0 : 1;
}

// One work-group, end of step k: h[k+1][k] = ||a|| (nrm2: squared norms of a),
// rotations, rhat, closing.
template <typename T>
__global__ void k_gm_rotate(int64_t m, int k, int ell, double rtol, GmCols<T> cl, GmState *st) {
    if (st->done) return;
    __shared__ int any;
    if (threadIdx.x == 0) any = 0;
    __syncthreads();
    for (int64_t c = threadIdx.x; c < m; c += blockDim.x) {
        if (!cl.open[c]) {
            cl.inv[c] = 0.0;
            continue;
        }
        T *H = cl.H + c * (ell + 1) * ell, *sn = cl.sn + c * ell, *rh = cl.rh + c * (ell + 1);
        double *cs = cl.cs + c * ell;
        const double hn = sqrt(cl.nrm2[c]);
        H[(k + 1) * ell + k] = f_of(T{}, hn);
        for (int j = 0; j < k; ++j) {
            const T u = H[j * ell + k], w = H[(j + 1) * ell + k];
            H[j * ell + k] = f_add(f_scale(u, cs[j]), f_mul(sn[j], w));
            H[(j + 1) * ell + k] = f_sub(f_scale(w, cs[j]), f_mul(f_conj(sn[j]), u));
        }
        double cc;
        T ss, rnew;
        if (!givens(H[k * ell + k], hn, cc, ss, rnew)) {  // zero pivot: the step is not used
            cl.open[c] = 0;
            cl.done[c] = 1;
            cl.status[c] = 1;
            cl.inv[c] = 0.0;
            continue;
        }
        cs[k] = cc;
        sn[k] = ss;
        H[k * ell + k] = rnew;
        H[(k + 1) * ell + k] = f_zero(T{});
        const T r0 = rh[k];
        rh[k] = f_scale(r0, cc);
        rh[k + 1] = f_scale(f_mul(f_conj(ss), r0), -1.0);
        cl.kc[c] = k + 1;
        cl.iters[c] += 1;
        if (f_abs(rh[k + 1]) <= rtol * cl.bn[c] || hn == 0.0) {
            cl.open[c] = 0;
            cl.inv[c] = 0.0;
        } else {
            cl.inv[c] = 1.0 / hn;
            any = 1;
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        st->steps += 1;
        if (!any) st->done = 1;
    }
}

// q[r][c] *= inv[c] (0 for closed columns); `comps` doubles per element (1 real, 2 complex)
__global__ void k_gm_scale(int64_t count, int64_t m, int comps, double *__restrict__ q, const double *__restrict__ inv,
                           const GmState *st, int always) {
    if (!always && st->done) return;
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < count) q[e] *= inv[(e / comps) % m];
}

// One work-group, end of a cycle: back substitution R y = rhat with k_i steps
template <typename T>
__global__ void k_gm_solve(int64_t m, int ell, GmCols<T> cl) {
    for (int64_t c = threadIdx.x; c < m; c += blockDim.x) {
        const int kk = cl.kc[c];
        if (kk == 0) continue;
        const T *H = cl.H + c * (ell + 1) * ell, *rh = cl.rh + c * (ell + 1);
        T *y = cl.y + c * ell;
        for (int r = kk - 1; r >= 0; --r) {
            T s = rh[r];
            for (int q = r + 1; q < kk; ++q) s = f_sub(s, f_mul(H[r * ell + q], y[q]));
            y[r] = f_div(s, H[r * ell + r]);
        }
        cl.est[c] = cl.bn[c] > 0.0 ? f_abs(rh[kk]) / cl.bn[c] : 0.0;
    }
}

// x[r][c] += sum_{j < k_c} Q_j[r][c] y[c][j]
template <typename T>
__global__ void k_gm_xupdate(int64_t n, int64_t m, int ell, const T *__restrict__ Q, GmCols<T> cl,
                             T *__restrict__ X) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * m) return;
    const int64_t c = e % m;
    const int kk = cl.kc[c];
    if (kk == 0) return;
    const T *y = cl.y + c * ell;
    T x = X[e];
    for (int j = 0; j < kk; ++j) x = f_add(x, f_mul(Q[(int64_t)j * n * m + e], y[j]));
    X[e] = x;
}

// rows into (scatter = 0) or out of (scatter = 1) tree order; m real columns
__global__ void k_gm_rows(int64_t n, int64_t m, const int64_t *__restrict__ perm, const double *__restrict__ src,
                          int64_t lds, double *__restrict__ dst, int64_t ldd, int scatter) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * m) return;
    const int64_t i = e / m, j = e % m;
    if (scatter) dst[perm[i] * ldd + j] = src[i * lds + j];
    else dst[i * ldd + j] = src[perm[i] * lds + j];
}

template <typename T>
struct Ws {
    T *Bt, *Xt, *Q, *part;
    double *part2;
    GmCols<T> cl;
    GmState *st;
    char *mm;
};

int64_t host_nblocks(int64_t n) { return (n + kRowsPerBlk - 1) / kRowsPerBlk; }

// bytes for m real columns (a complex column takes two, and the complex layout fits)
size_t small_bytes(int64_t m, int ell) {
    const size_t per_col = (size_t)(ell + 1) * ell + 2 * (size_t)ell + (ell + 1) + ell + 4;
    return align_up(sizeof(double) * per_col * m) + align_up(sizeof(int32_t) * 5 * m) + align_up(sizeof(GmState));
}

// mf columns of the field T
template <typename T>
Ws<T> carve_ws(int64_t n, int64_t mf, int ell, char *ws) {
    const int64_t nblk = host_nblocks(n);
    Ws<T> w;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char *p = ws + off;
        off += align_up(bytes);
        return p;
    };
    w.Bt = (T *)take(sizeof(T) * n * mf);
    w.Xt = (T *)take(sizeof(T) * n * mf);
    w.Q = (T *)take(sizeof(T) * n * mf * (ell + 1));
    w.part = (T *)take(sizeof(T) * nblk * mf * (ell + 1));
    w.part2 = (double *)take(sizeof(double) * nblk * mf);
    char *d = take(sizeof(T) * mf * ((size_t)(ell + 1) * ell + ell + (ell + 1) + ell) +
                   sizeof(double) * mf * ((size_t)ell + 4));
    auto next_t = [&](size_t cnt) {
        T *p = (T *)d;
        d += sizeof(T) * cnt;
        return p;
    };
    auto next_d = [&](size_t cnt) {
        double *p = (double *)d;
        d += sizeof(double) * cnt;
        return p;
    };
    w.cl.H = next_t(mf * (ell + 1) * ell);
    w.cl.sn = next_t(mf * ell);
    w.cl.rh = next_t(mf * (ell + 1));
    w.cl.y = next_t(mf * ell);
    w.cl.cs = next_d(mf * ell);
    w.cl.bn = next_d(mf);
    w.cl.inv = next_d(mf);
    w.cl.est = next_d(mf);
    w.cl.nrm2 = next_d(mf);
    int32_t *ip = (int32_t *)take(sizeof(int32_t) * 5 * mf);
    w.cl.open = ip;
    w.cl.done = ip + mf;
    w.cl.kc = ip + 2 * mf;
    w.cl.iters = ip + 3 * mf;
    w.cl.status = ip + 4 * mf;
    w.st = (GmState *)take(sizeof(GmState));
    w.mm = ws + off;
    return w;
}

// m real columns (mf = m / comps columns of the field)
template <typename T>
h2x_status run_gmres_impl(const DevMat &dm, const h2x_gmres_params &prm, int64_t m, const double *B, int64_t ldb,
                          double *X, int64_t ldx, char *ws, h2x_gmres_info *info, hipStream_t st) {
    constexpr int comps = sizeof(T) / sizeof(double);
    const int ell = prm.restart;
    const int64_t n = dm.n, mf = m / comps, nm = n * m, nblk = host_nblocks(n);
    Ws<T> w = carve_ws<T>(n, mf, ell, ws);
    double *Qd = (double *)w.Q, *Btd = (double *)w.Bt, *Xtd = (double *)w.Xt;
    const dim3 g_el((unsigned)((nm + 255) / 256)), g_elf((unsigned)((n * mf + 255) / 256)), b256(256);
    const dim3 g_rb((unsigned)nblk, (unsigned)((mf + kCols - 1) / kCols));
    const dim3 g_col((unsigned)((mf + 3) / 4));  // one wave per column
    const int check = prm.check_every > 0 ? prm.check_every : 1;
    hipError_t e = hipSuccess;
    auto sync_state = [&](GmState &h) {
        if (e == hipSuccess) e = hipMemcpyAsync(&h, w.st, sizeof(GmState), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
    };

    // tree order: B~ = B[perm], X~ = X0[perm]; ||b_i||
    hipLaunchKernelGGL(k_gm_rows, g_el, b256, 0, st, n, m, dm.perm, B, ldb, Btd, m, 0);
    hipLaunchKernelGGL(k_gm_rows, g_el, b256, 0, st, n, m, dm.perm, X, ldx, Xtd, m, 0);
    hipLaunchKernelGGL(k_gm_update<T>, g_rb, b256, 0, st, n, mf, -1, ell, (const T *)nullptr, w.Bt, w.cl, w.part2,
                       (const GmState *)w.st);
    hipLaunchKernelGGL(k_gm_colsum<T>, g_col, b256, 0, st, mf, nblk, w.part2, w.cl, (const GmState *)w.st, 1);
    hipLaunchKernelGGL(k_gm_init<T>, dim3(1), b256, 0, st, mf, w.cl, w.st);
    e = hipGetLastError();

    GmState hs{};
    int64_t steps_known = 0;  // Arnoldi steps run, as of the last state read
    int32_t cycles = 0;
    for (;;) {
        // r = b - A x into q_0, its norms, the cycle's start, q_0 = r / ||r||
        if (e == hipSuccess) e = hipMemcpyAsync(Qd, Btd, sizeof(double) * nm, hipMemcpyDeviceToDevice, st);
        if (e == hipSuccess) e = run_matmul(dm, m, -1.0, Xtd, m, 1.0, Qd, m, true, w.mm, st);
        if (e != hipSuccess) break;
        hipLaunchKernelGGL(k_gm_update<T>, g_rb, b256, 0, st, n, mf, -1, ell, (const T *)nullptr, w.Q, w.cl,
                           w.part2, (const GmState *)w.st);
        hipLaunchKernelGGL(k_gm_colsum<T>, g_col, b256, 0, st, mf, nblk, w.part2, w.cl, (const GmState *)w.st, 1);
        hipLaunchKernelGGL(k_gm_start<T>, dim3(1), b256, 0, st, mf, ell, prm.rtol, w.cl, w.st);
        hipLaunchKernelGGL(k_gm_scale, g_el, b256, 0, st, nm, mf, comps, Qd, (const double *)w.cl.inv,
                           (const GmState *)w.st, 1);
        e = hipGetLastError();
        sync_state(hs);
        if (e != hipSuccess) break;
        steps_known = hs.steps;
        if (hs.done || steps_known >= prm.max_iter) break;
        ++cycles;
        // Arnoldi steps; the host looks at the state every `check` steps
        int64_t launched = 0;  // steps launched since the last state read
        for (int k = 0; k < ell; ++k) {
            if (steps_known + launched >= prm.max_iter) break;
            double *qk = Qd + (int64_t)k * nm, *q1 = qk + nm;
            e = run_matmul(dm, m, 1.0, qk, m, 0.0, q1, m, true, w.mm, st, nullptr, (const int32_t *)w.st);
            if (e != hipSuccess) break;
            hipLaunchKernelGGL(k_gm_dots<T>, dim3(g_rb.x, g_rb.y, (unsigned)(k + 1)), b256, 0, st, n, mf, w.Q,
                               (const T *)q1, w.part, (const GmState *)w.st);
            hipLaunchKernelGGL(k_gm_hcol<T>, dim3((unsigned)(((int64_t)(k + 1) * mf + 3) / 4)), b256, 0, st, mf, nblk,
                               k, ell, (const T *)w.part, w.cl, (const GmState *)w.st);
            hipLaunchKernelGGL(k_gm_update<T>, g_rb, b256, 0, st, n, mf, k, ell, (const T *)w.Q, (T *)q1, w.cl,
                               w.part2, (const GmState *)w.st);
            hipLaunchKernelGGL(k_gm_colsum<T>, g_col, b256, 0, st, mf, nblk, w.part2, w.cl, (const GmState *)w.st, 0);
            hipLaunchKernelGGL(k_gm_rotate<T>, dim3(1), b256, 0, st, mf, k, ell, prm.rtol, w.cl, w.st);
            hipLaunchKernelGGL(k_gm_scale, g_el, b256, 0, st, nm, mf, comps, q1, (const double *)w.cl.inv,
                               (const GmState *)w.st, 0);
            e = hipGetLastError();
            if (e != hipSuccess) break;
            ++launched;
            if (launched % check == 0 || k + 1 == ell) {
                sync_state(hs);
                if (e != hipSuccess) break;
                steps_known = hs.steps;
                launched = 0;
                if (hs.done) break;
            }
        }
        if (e != hipSuccess) break;
        // x += V y with each column's own number of steps
        hipLaunchKernelGGL(k_gm_solve<T>, dim3(1), b256, 0, st, mf, ell, w.cl);
        hipLaunchKernelGGL(k_gm_xupdate<T>, g_elf, b256, 0, st, n, mf, ell, (const T *)w.Q, w.cl, w.Xt);
        e = hipGetLastError();
        if (e == hipSuccess && launched > 0) sync_state(hs);
        if (e != hipSuccess) break;
        steps_known = hs.steps;
    }
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_gm_rows, g_el, b256, 0, st, n, m, dm.perm, Xtd, m, X, ldx, 1);
        e = hipGetLastError();
    }
    std::vector<int32_t> iters(mf), status(mf);
    std::vector<double> est(mf);
    if (e == hipSuccess) e = hipMemcpyAsync(iters.data(), w.cl.iters, sizeof(int32_t) * mf, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipMemcpyAsync(status.data(), w.cl.status, sizeof(int32_t) * mf, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipMemcpyAsync(est.data(), w.cl.est, sizeof(double) * mf, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipMemcpyAsync(&hs, w.st, sizeof(GmState), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        set_error(std::string("h2x_block_gmres: ") + hipGetErrorString(e));
        return H2X_EHIP;
    }
    if (info) {
        info->iters = hs.steps;
        info->cycles = cycles;
        int broke = 0, open = 0;
        for (int64_t c = 0; c < mf; ++c) {
            broke |= status[c] == 1;
            open |= status[c] == 2;
            if (info->col_iters) info->col_iters[c] = iters[c];
            if (info->col_status) info->col_status[c] = status[c];
            if (info->col_res) info->col_res[c] = est[c];
        }
        info->status = broke ? H2X_EBREAKDOWN : (open ? H2X_ENOCONV : H2X_OK);
    }
    return H2X_OK;
}

}  // namespace

size_t gmres_ws_bytes(const DevMat &dm, int64_t m, int ell) {
    const int64_t n = dm.n, nblk = host_nblocks(n);
    return align_up(sizeof(double) * n * m) * 2 + align_up(sizeof(double) * n * m * (ell + 1)) +
           align_up(sizeof(double) * nblk * m * (ell + 1)) + align_up(sizeof(double) * nblk * m) +
           small_bytes(m, ell) + matmul_ws_bytes(dm, m);
}

h2x_status run_block_gmres(const DevMat &dm, const h2x_gmres_params &prm, int64_t m, const double *B, int64_t ldb,
                           double *X, int64_t ldx, char *ws, size_t ws_bytes, h2x_gmres_info *info, hipStream_t st) {
    if (ws_bytes < gmres_ws_bytes(dm, m, prm.restart)) {
        set_error("h2x_block_gmres: workspace too small");
        return H2X_ENOMEM;
    }
    if (dm.cplx) return run_gmres_impl<cpx>(dm, prm, m, B, ldb, X, ldx, ws, info, st);
    return run_gmres_impl<double>(dm, prm, m, B, ldb, X, ldx, ws, info, st);
}

}  // namespace h2x
