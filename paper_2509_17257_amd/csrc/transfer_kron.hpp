// Transfer passes of the FP64 operator through the tensor structure of the transfer matrices
// (Chebyshev order P = 3 or 4, rank k = P^3).  The interpolation nodes of a cluster form a
// P x P x P Chebyshev grid on its axis-parallel box and the Lagrange polynomials are products
// of one-dimensional ones, so the transfer matrix of a son c (the father's polynomials at the
// son's nodes) is the Kronecker product of three P x P matrices:
//
//   E_c[a, nu] = F_c^0[a0, nu0] F_c^1[a1, nu1] F_c^2[a2, nu2],   a = a0 + P a1 + P^2 a2,
//
// F_c^d[i, j] = the father's j-th Lagrange polynomial on axis d at the son's i-th node on that
// axis (stored as 3 P^2 doubles per cluster, [d][P i + j]).  The upward step
// x_t = sum_c E_c^T x_c and the downward step y_c += E_c y_t then take three passes of P-term
// sums over the k entries of a column (3 P^4 multiply-adds instead of P^6: 768 instead of 4096
// at P = 4) and read 3 P^2 factors instead of the k^2 entries of E_c.
//
// One work-group of 256 threads per (cluster, slab of MC columns): the input columns go to LDS
// (k rows of MC + 1 doubles per block); a pass maps each P-entry pencil along its axis to a
// thread, which overwrites it in place (pencils are disjoint: no barrier inside a pass);
// consecutive threads take consecutive columns, so LDS rows are read without bank conflicts.
// The last pass reads LDS and writes (upward) or adds to (downward) the output in HBM.
#pragma once

#include "device.hpp"

namespace h2x {
namespace kron {

// rows of the P-entry pencil o (0..P^2-1: the two digits other than axis d, the lower one
// first) along axis d: base + stride * l, l = 0..P-1
template <int P>
__device__ inline int pencil_base(int d, int o) {
    return d == 0 ? P * o : (d == 1 ? (o % P) + P * P * (o / P) : o);
}
template <int P>
__device__ inline int axis_stride(int d) { return d == 0 ? 1 : (d == 1 ? P : P * P); }

// v' = M v on every pencil along axis d of NQ blocks in LDS; M = (F^d)^T (TR, upward) or F^d
template <int P, int MC, int NQ, bool TR>
__device__ inline void pass(double *buf, const double *fs, int d) {
    constexpr int K = P * P * P, LD = MC + 1, NPEN = NQ * P * P * MC;
    const int st = axis_stride<P>(d);
#pragma unroll
    for (int u = 0; u < (NPEN + 255) / 256; ++u) {
        const int idx = threadIdx.x + 256 * u;
        if (NPEN % 256 != 0 && idx >= NPEN) break;
        const int j = idx % MC, pen = idx / MC, q = pen / (P * P);
        double *col = buf + (q * K + pencil_base<P>(d, pen % (P * P))) * LD + j;
        const double *F = fs + q * 3 * P * P + P * P * d;
        double v[P], o[P];
#pragma unroll
        for (int l = 0; l < P; ++l) v[l] = col[st * l * LD];
#pragma unroll
        for (int i = 0; i < P; ++i) {
            double s = 0.0;
#pragma unroll
            for (int l = 0; l < P; ++l) s += (TR ? F[P * l + i] : F[P * i + l]) * v[l];
            o[i] = s;
        }
#pragma unroll
        for (int i = 0; i < P; ++i) col[st * i * LD] = o[i];
    }
}

// x_t = E_{s0}^T x_{s0} + E_{s1}^T x_{s1} for the clusters list[i] with sons son[2 i], son[2 i + 1]
template <int P, int MC>
__global__ __launch_bounds__(256) void k_up(int64_t m, const int32_t *__restrict__ list,
                                            const int32_t *__restrict__ son, const double *__restrict__ F1,
                                            double *__restrict__ xh, int64_t ldh, Skip skip) {
    constexpr int K = P * P * P, LD = MC + 1, NF = 3 * P * P, NIN = 2 * K * MC, NOUT = P * P * MC;
    __shared__ double buf[2 * K * LD];
    __shared__ double fs[2 * NF];
    const int32_t t = list[blockIdx.x];
    if (skip(t)) return;
    const int32_t sc[2] = {son[2 * blockIdx.x], son[2 * blockIdx.x + 1]};
    const int64_t j0 = (int64_t)blockIdx.y * MC;
    const int mc = (int)min<int64_t>(MC, m - j0);
    if (threadIdx.x < 2 * NF) fs[threadIdx.x] = F1[(int64_t)sc[threadIdx.x / NF] * NF + threadIdx.x % NF];
#pragma unroll
    for (int u = 0; u < (NIN + 255) / 256; ++u) {
        const int idx = threadIdx.x + 256 * u;
        if (NIN % 256 != 0 && idx >= NIN) break;
        const int j = idx % MC, r = (idx / MC) % K, q = idx / (MC * K);
        buf[(q * K + r) * LD + j] = xh[((int64_t)sc[q] * K + r) * ldh + j0 + min(j, mc - 1)];
    }
    __syncthreads();
    pass<P, MC, 2, true>(buf, fs, 0);
    __syncthreads();
    pass<P, MC, 2, true>(buf, fs, 1);
    __syncthreads();
    // axis 2 and the sum over the two sons
#pragma unroll
    for (int u = 0; u < (NOUT + 255) / 256; ++u) {
        const int idx = threadIdx.x + 256 * u;
        if (NOUT % 256 != 0 && idx >= NOUT) break;
        const int j = idx % MC, o = idx / MC;
        double acc[P];
#pragma unroll
        for (int i = 0; i < P; ++i) acc[i] = 0.0;
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const double *F = fs + q * NF + 2 * P * P;
            double v[P];
#pragma unroll
            for (int l = 0; l < P; ++l) v[l] = buf[(q * K + o + P * P * l) * LD + j];
#pragma unroll
            for (int i = 0; i < P; ++i)
#pragma unroll
                for (int l = 0; l < P; ++l) acc[i] += F[P * l + i] * v[l];
        }
        if (j < mc)
#pragma unroll
            for (int i = 0; i < P; ++i) xh[((int64_t)t * K + o + P * P * i) * ldh + j0 + j] = acc[i];
    }
}

// y_c += E_c y_{par} for the clusters list[i] with fathers par[i]
template <int P, int MC>
__global__ __launch_bounds__(256) void k_down(int64_t m, const int32_t *__restrict__ list,
                                              const int32_t *__restrict__ par, const double *__restrict__ F1,
                                              double *__restrict__ yh, int64_t ldh, Skip skip) {
    constexpr int K = P * P * P, LD = MC + 1, NF = 3 * P * P, NIN = K * MC, NOUT = P * P * MC;
    __shared__ double buf[K * LD];
    __shared__ double fs[NF];
    const int32_t c = list[blockIdx.x], p = par[blockIdx.x];
    if (skip(c)) return;
    const int64_t j0 = (int64_t)blockIdx.y * MC;
    const int mc = (int)min<int64_t>(MC, m - j0);
    if (threadIdx.x < NF) fs[threadIdx.x] = F1[(int64_t)c * NF + threadIdx.x];
#pragma unroll
    for (int u = 0; u < (NIN + 255) / 256; ++u) {
        const int idx = threadIdx.x + 256 * u;
        if (NIN % 256 != 0 && idx >= NIN) break;
        const int j = idx % MC, r = idx / MC;
        buf[r * LD + j] = yh[((int64_t)p * K + r) * ldh + j0 + min(j, mc - 1)];
    }
    __syncthreads();
    pass<P, MC, 1, false>(buf, fs, 0);
    __syncthreads();
    pass<P, MC, 1, false>(buf, fs, 1);
    __syncthreads();
#pragma unroll
    for (int u = 0; u < (NOUT + 255) / 256; ++u) {
        const int idx = threadIdx.x + 256 * u;
        if (NOUT % 256 != 0 && idx >= NOUT) break;
        const int j = idx % MC, o = idx / MC;
        const double *F = fs + 2 * P * P;
        double v[P];
#pragma unroll
        for (int l = 0; l < P; ++l) v[l] = buf[(o + P * P * l) * LD + j];
        if (j < mc)
#pragma unroll
            for (int i = 0; i < P; ++i) {
                double s = 0.0;
#pragma unroll
                for (int l = 0; l < P; ++l) s += F[P * i + l] * v[l];
                yh[((int64_t)c * K + o + P * P * i) * ldh + j0 + j] += s;
            }
    }
}

}  // namespace kron
}  // namespace h2x
