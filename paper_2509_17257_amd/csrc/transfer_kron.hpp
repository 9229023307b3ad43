// Transfer passes of the FP64 operator with p = 4 (k = 64) through the tensor structure of
// the transfer matrices.  The interpolation nodes of a cluster form a 4 x 4 x 4 Chebyshev grid
// on its axis-parallel box and the Lagrange polynomials are products of one-dimensional ones,
// so the transfer matrix of a son c (the father's polynomials at the son's nodes) is the
// Kronecker product of three 4 x 4 matrices:
//
//   E_c[a, nu] = F_c^0[a0, nu0] F_c^1[a1, nu1] F_c^2[a2, nu2],   a = a0 + 4 a1 + 16 a2,
//
// F_c^d[i, j] = the father's j-th Lagrange polynomial on axis d at the son's i-th node on that
// axis (stored as 48 doubles per cluster, [d][4 i + j]).  The upward step x_t = sum_c E_c^T x_c
// and the downward step y_c += E_c y_t then take three passes of 4-term sums over the 64
// entries of a column (768 multiply-adds instead of 4096) and read 48 factors instead of the
// 4096 entries of E_c.
//
// One work-group of 256 threads per (cluster, slab of MC columns): the input columns go to LDS
// (64 rows of MC + 1 doubles per block); a pass maps each 4-entry pencil along its axis to a
// thread, which overwrites it in place (pencils are disjoint: no barrier inside a pass);
// consecutive threads take consecutive columns, so LDS rows are read without bank conflicts.
// The last pass reads LDS and writes (upward) or adds to (downward) the output in HBM.
#pragma once

#include "device.hpp"

namespace h2x {
namespace kron {

constexpr int kK = 64;

// rows of the 4-entry pencil o (0..15: the two digits other than axis d, in increasing
// order) along axis d: base + stride * l, l = 0..3
__device__ inline int pencil_base(int d, int o) {
    return d == 0 ? 4 * o : (d == 1 ? (o & 3) + 16 * (o >> 2) : o);
}
__device__ inline int axis_stride(int d) { return d == 0 ? 1 : (d == 1 ? 4 : 16); }

// v' = M v on every pencil along axis d of NQ blocks in LDS; M = (F^d)^T (TR, upward) or F^d
template <int MC, int NQ, bool TR>
__device__ inline void pass(double *buf, const double *fs, int d) {
    constexpr int LD = MC + 1;
    const int st = axis_stride(d);
#pragma unroll
    for (int u = 0; u < NQ * 16 * MC / 256; ++u) {
        const int idx = threadIdx.x + 256 * u, j = idx % MC, pen = idx / MC, q = pen >> 4;
        double *col = buf + (q * kK + pencil_base(d, pen & 15)) * LD + j;
        const double *F = fs + q * 48 + 16 * d;
        double v[4], o[4];
#pragma unroll
        for (int l = 0; l < 4; ++l) v[l] = col[st * l * LD];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            double s = 0.0;
#pragma unroll
            for (int l = 0; l < 4; ++l) s += (TR ? F[4 * l + i] : F[4 * i + l]) * v[l];
            o[i] = s;
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) col[st * i * LD] = o[i];
    }
}

// x_t = E_{s0}^T x_{s0} + E_{s1}^T x_{s1} for the clusters list[i] with sons son[2 i], son[2 i + 1]
template <int MC>
__global__ __launch_bounds__(256) void k_up(int64_t m, const int32_t *__restrict__ list,
                                            const int32_t *__restrict__ son, const double *__restrict__ F1,
                                            double *__restrict__ xh, int64_t ldh, Skip skip) {
    constexpr int LD = MC + 1;
    __shared__ double buf[2 * kK * LD];
    __shared__ double fs[2 * 48];
    const int32_t t = list[blockIdx.x];
    if (skip(t)) return;
    const int32_t sc[2] = {son[2 * blockIdx.x], son[2 * blockIdx.x + 1]};
    const int64_t j0 = (int64_t)blockIdx.y * MC;
    const int mc = (int)min<int64_t>(MC, m - j0);
    if (threadIdx.x < 96) fs[threadIdx.x] = F1[(int64_t)sc[threadIdx.x / 48] * 48 + threadIdx.x % 48];
#pragma unroll
    for (int u = 0; u < 2 * kK * MC / 256; ++u) {
        const int idx = threadIdx.x + 256 * u, j = idx % MC, r = (idx / MC) % kK, q = idx / (MC * kK);
        buf[(q * kK + r) * LD + j] = xh[((int64_t)sc[q] * kK + r) * ldh + j0 + min(j, mc - 1)];
    }
    __syncthreads();
    pass<MC, 2, true>(buf, fs, 0);
    __syncthreads();
    pass<MC, 2, true>(buf, fs, 1);
    __syncthreads();
    // axis 2 and the sum over the two sons
#pragma unroll
    for (int u = 0; u < 16 * MC / 256; ++u) {
        const int idx = threadIdx.x + 256 * u, j = idx % MC, o = idx / MC;
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const double *F = fs + q * 48 + 32;
            double v[4];
#pragma unroll
            for (int l = 0; l < 4; ++l) v[l] = buf[(q * kK + o + 16 * l) * LD + j];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int l = 0; l < 4; ++l) acc[i] += F[4 * l + i] * v[l];
        }
        if (j < mc)
#pragma unroll
            for (int i = 0; i < 4; ++i) xh[((int64_t)t * kK + o + 16 * i) * ldh + j0 + j] = acc[i];
    }
}

// y_c += E_c y_{par} for the clusters list[i] with fathers par[i]
template <int MC>
__global__ __launch_bounds__(256) void k_down(int64_t m, const int32_t *__restrict__ list,
                                              const int32_t *__restrict__ par, const double *__restrict__ F1,
                                              double *__restrict__ yh, int64_t ldh, Skip skip) {
    constexpr int LD = MC + 1;
    __shared__ double buf[kK * LD];
    __shared__ double fs[48];
    const int32_t c = list[blockIdx.x], p = par[blockIdx.x];
    if (skip(c)) return;
    const int64_t j0 = (int64_t)blockIdx.y * MC;
    const int mc = (int)min<int64_t>(MC, m - j0);
    if (threadIdx.x < 48) fs[threadIdx.x] = F1[(int64_t)c * 48 + threadIdx.x];
#pragma unroll
    for (int u = 0; u < kK * MC / 256; ++u) {
        const int idx = threadIdx.x + 256 * u, j = idx % MC, r = idx / MC;
        buf[r * LD + j] = yh[((int64_t)p * kK + r) * ldh + j0 + min(j, mc - 1)];
    }
    __syncthreads();
    pass<MC, 1, false>(buf, fs, 0);
    __syncthreads();
    pass<MC, 1, false>(buf, fs, 1);
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 16 * MC / 256; ++u) {
        const int idx = threadIdx.x + 256 * u, j = idx % MC, o = idx / MC;
        const double *F = fs + 32;
        double v[4];
#pragma unroll
        for (int l = 0; l < 4; ++l) v[l] = buf[(o + 16 * l) * LD + j];
        if (j < mc)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                double s = 0.0;
#pragma unroll
                for (int l = 0; l < 4; ++l) s += F[4 * i + l] * v[l];
                yh[((int64_t)c * kK + o + 16 * i) * ldh + j0 + j] += s;
            }
    }
}

}  // namespace kron
}  // namespace h2x
