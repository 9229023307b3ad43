// Device-side construction of the H^2 representation (section 2): Chebyshev
// tensor nodes per cluster, leaf matrices V_t, transfer matrices E_t, coupling
// matrices S_b of the admissible leaves and dense near-field blocks.  The
// operator can be tens of GB (coupling matrices dominate), so it is generated
// where it is used, directly into the caller's workspace.
#include <cmath>

#include "device.hpp"
#include "types.hpp"

namespace h2x {

namespace {

template <typename T>
T *carve(size_t &off, char *base, size_t count) {
    off = align_up(off);
    T *ptr = base ? (T *)(base + off) : nullptr;
    off += count * sizeof(T);
    return ptr;
}

__device__ inline double kernel_g(int kernel, double ell, const double *a, const double *b) {
    if (kernel == H2X_KERNEL_EXP) {
        double dx = a[0] - b[0], dy = a[1] - b[1], dz = a[2] - b[2];
        return exp(-sqrt(dx * dx + dy * dy + dz * dz) / ell);
    }
    if (kernel == H2X_KERNEL_POLY) {
        double d = 1.0 + a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
        return d * d;
    }
    return 1.0;
}

// complex Helmholtz kernel with equal quadrature weights: exp(i kappa r) / (n r),
// kappa = ell; coinciding points give 0
__device__ inline void kernel_gc(double ell, double npts, const double *a, const double *b, double &re, double &im) {
    const double dx = a[0] - b[0], dy = a[1] - b[1], dz = a[2] - b[2];
    const double r = sqrt(dx * dx + dy * dy + dz * dz);
    if (r == 0.0) {
        re = im = 0.0;
        return;
    }
    const double f = 1.0 / (npts * r);
    re = cos(ell * r) * f;
    im = sin(ell * r) * f;
}

// one-dimensional Lagrange polynomial j of the nodes nd[0..p) at x
__device__ inline double lagrange1(const double *nd, int p, int j, double x) {
    double v = 1.0, xj = nd[j];
    for (int i = 0; i < p; ++i) {
        if (i == j) continue;
        v *= (x - nd[i]) / (xj - nd[i]);
    }
    return v;
}

// tensor nodes: nu = jx + p*jy + p^2*jz, first-kind Chebyshev points of the box
__global__ void k_nodes(int32_t C, int p, const double *__restrict__ box, double *__restrict__ nodes) {
    const int k = p * p * p;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)C * k) return;
    const int32_t c = (int32_t)(idx / k);
    const int nu = (int)(idx % k);
    const int jj[3] = {nu % p, (nu / p) % p, nu / (p * p)};
    for (int d = 0; d < 3; ++d) {
        double lo = box[6 * c + d], hi = box[6 * c + 3 + d];
        double ctr = 0.5 * (lo + hi), half = 0.5 * (hi - lo);
        nodes[idx * 3 + d] = ctr + half * cos((2.0 * jj[d] + 1.0) * M_PI / (2.0 * p));
    }
}

__device__ inline void nodes1d(const double *nodes, int32_t c, int p, int d, double *nd) {
    const int k = p * p * p;
    const int stride = d == 0 ? 1 : (d == 1 ? p : p * p);
    for (int j = 0; j < p; ++j) nd[j] = nodes[((int64_t)c * k + (int64_t)j * stride) * 3 + d];
}

// V_t[i, nu] = L_{t,jx}(x_i) L_{t,jy}(y_i) L_{t,jz}(z_i) for the leaf t (one block per leaf)
template <typename T>
__global__ void k_fill_V(int p, const int32_t *__restrict__ leaves, const int32_t *__restrict__ first,
                         const int32_t *__restrict__ size, const double *__restrict__ pts,
                         const double *__restrict__ nodes, T *__restrict__ V, T *__restrict__ Vt,
                         const int64_t *__restrict__ vt_off) {
    const int k = p * p * p;
    const int32_t t = leaves[blockIdx.x];
    __shared__ double nd[3][16];
    if (threadIdx.x < 3 * p) {
        int d = threadIdx.x / p, j = threadIdx.x % p;
        const int stride = d == 0 ? 1 : (d == 1 ? p : p * p);
        nd[d][j] = nodes[((int64_t)t * k + (int64_t)j * stride) * 3 + d];
    }
    __syncthreads();
    const int64_t rows = size[t];
    for (int64_t e = threadIdx.x; e < rows * k; e += blockDim.x) {
        const int64_t i = first[t] + e / k;
        const int nu = (int)(e % k);
        const double *x = &pts[3 * i];
        double v = lagrange1(nd[0], p, nu % p, x[0]) * lagrange1(nd[1], p, (nu / p) % p, x[1]) *
                   lagrange1(nd[2], p, nu / (p * p), x[2]);
        V[i * k + nu] = from_double<T>(v);
        if (Vt) {
            // transposed copy: k x nt2 (rows padded to pad_rows(|t|), padding zero)
            const int64_t nt2 = pad_rows(rows), il = i - first[t];
            T *vt = Vt + vt_off[blockIdx.x];
            vt[nu * nt2 + il] = from_double<T>(v);
            if (il == rows - 1)
                for (int64_t z = rows; z < nt2; ++z) vt[nu * nt2 + z] = from_double<T>(0.0);
        }
    }
}

// E_c[a, nu] = L_{parent(c), nu}(xi_{c, a}) (one block per non-root cluster)
template <typename T>
__global__ void k_fill_E(int p, const int32_t *__restrict__ parent, const double *__restrict__ nodes,
                         T *__restrict__ E) {
    const int k = p * p * p;
    const int32_t c = blockIdx.x + 1;  // the root has no transfer matrix
    const int32_t par = parent[c];
    if (par < 0) {  // the root of a later system of a merged plan: zeros
        for (int e = threadIdx.x; e < k * k; e += blockDim.x) E[(int64_t)c * k * k + e] = from_double<T>(0.0);
        return;
    }
    __shared__ double nd[3][16];
    if (threadIdx.x < 3 * p) {
        int d = threadIdx.x / p, j = threadIdx.x % p;
        const int stride = d == 0 ? 1 : (d == 1 ? p : p * p);
        nd[d][j] = nodes[((int64_t)par * k + (int64_t)j * stride) * 3 + d];
    }
    __syncthreads();
    for (int e = threadIdx.x; e < k * k; e += blockDim.x) {
        const int a = e / k, nu = e % k;
        const double *x = &nodes[((int64_t)c * k + a) * 3];
        double v = lagrange1(nd[0], p, nu % p, x[0]) * lagrange1(nd[1], p, (nu / p) % p, x[1]) *
                   lagrange1(nd[2], p, nu / (p * p), x[2]);
        E[(int64_t)c * k * k + e] = from_double<T>(v);
    }
}

// one-dimensional factors of the transfer matrices: F1[c][d][p i + j] = the father's j-th
// Lagrange polynomial on axis d at the son's i-th node on axis d, so that E_c[a, nu] =
// F1[c][0][a0, nu0] F1[c][1][a1, nu1] F1[c][2][a2, nu2] (digits a = a0 + p a1 + p^2 a2); the
// entries of a root (of every system of a merged plan) are zero
__global__ void k_fill_E1(int32_t C, int p, const int32_t *__restrict__ parent, const double *__restrict__ nodes,
                          double *__restrict__ F1) {
    const int per = 3 * p * p;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)C * per) return;
    const int32_t c = (int32_t)(idx / per);
    const int e = (int)(idx % per), d = e / (p * p), i = (e / p) % p, j = e % p;
    if (parent[c] < 0) {
        F1[idx] = 0.0;
        return;
    }
    double ndp[16], ndc[16];
    nodes1d(nodes, parent[c], p, d, ndp);
    nodes1d(nodes, c, p, d, ndc);
    F1[idx] = lagrange1(ndp, p, j, ndc[i]);
}

// S_b[nu, mu] = g(xi_{t,nu}, xi_{s,mu}), stored in the layout the coupling kernel reads
// (complex kernel: real part into S, imaginary part into S + s_plane)
template <typename T>
__global__ void k_fill_S(int k, int kernel, double ell, double npts, const int32_t *__restrict__ adm_row,
                         const int32_t *__restrict__ adm_col, const double *__restrict__ nodes,
                         T *__restrict__ S, int swz, int64_t s_plane) {
    const int64_t b = blockIdx.x;
    const int32_t t = adm_row[b], s = adm_col[b];
    for (int e = threadIdx.x; e < k * k; e += blockDim.x) {
        const int nu = e / k, mu = e % k;
        const double *xa = &nodes[((int64_t)t * k + nu) * 3], *xb = &nodes[((int64_t)s * k + mu) * 3];
        const int64_t at = b * k * k + s_index(swz, k, nu, mu);
        if (kernel == H2X_KERNEL_HELMHOLTZ) {
            double re, im;
            kernel_gc(ell, npts, xa, xb, re, im);
            S[at] = from_double<T>(re);
            S[at + s_plane] = from_double<T>(im);
        } else {
            S[at] = from_double<T>(kernel_g(kernel, ell, xa, xb));
        }
    }
}

// N_(t,s)[i, j] = g(x_i, x_j) + shift [i == j], row-major |t| x |s|, or stored
// transposed when trans != 0: |s| rows of length pad_rows(|t|), padding zero
// (complex kernel: real part into N, imaginary part into N + n_plane)
template <typename TN>
__global__ void k_fill_N(int kernel, double ell, double shift, double npts, const int32_t *__restrict__ near_row,
                         const int32_t *__restrict__ near_col, const int64_t *__restrict__ near_off,
                         const int32_t *__restrict__ first, const int32_t *__restrict__ size,
                         const double *__restrict__ pts, TN *__restrict__ N, int trans, int64_t n_plane) {
    const int64_t q = blockIdx.x;
    const int32_t t = near_row[q], s = near_col[q];
    const int64_t nt = size[t], ns = size[s], ft = first[t], fs = first[s];
    TN *Nb = N + near_off[q];
    const int64_t nt2 = pad_rows(nt);
    const bool cplx = kernel == H2X_KERNEL_HELMHOLTZ;
    for (int64_t e = threadIdx.x; e < nt * ns; e += blockDim.x) {
        const int64_t il = e / ns, jl = e % ns, i = ft + il, j = fs + jl;
        const int64_t at = trans ? jl * nt2 + il : e;
        if (cplx) {
            double re, im;
            kernel_gc(ell, npts, &pts[3 * i], &pts[3 * j], re, im);
            if (i == j) re += shift;
            Nb[at] = (TN)re;
            Nb[at + n_plane] = (TN)im;
        } else {
            double v = kernel_g(kernel, ell, &pts[3 * i], &pts[3 * j]);
            if (i == j) v += shift;
            Nb[at] = (TN)v;
        }
    }
    if (trans)
        for (int64_t e = threadIdx.x; e < (nt2 - nt) * ns; e += blockDim.x) {
            const int64_t at = (e / (nt2 - nt)) * nt2 + nt + e % (nt2 - nt);
            Nb[at] = (TN)0;
            if (cplx) Nb[at + n_plane] = (TN)0;
        }
}

// coupling matrices and near field, system by system (each with its own kernel
// parameters; a one-system operator uses the operator's current ones)
template <typename T, typename TN>
hipError_t fill_SN(const DevMat &dm, hipStream_t st) {
    const Plan &P = *dm.plan;
    const int32_t ns = P.nsys();
    for (int32_t i = 0; i < ns; ++i) {
        const int kernel = ns == 1 ? dm.kernel : (int)P.sys_prm[i].kernel;
        const double ell = ns == 1 ? dm.ell : P.sys_prm[i].ell, shift = ns == 1 ? dm.shift : P.sys_prm[i].shift;
        const int64_t a = P.sys_adm[i], na = P.sys_adm[i + 1] - a;
        const int64_t q = P.sys_near[i], nq = P.sys_near[i + 1] - q;
        const double npts = (double)(P.sys_row[i + 1] - P.sys_row[i]);  // points of system i
        if (na > 0)
            hipLaunchKernelGGL(k_fill_S<T>, dim3((unsigned)na), dim3(256), 0, st, dm.k, kernel, ell, npts,
                               dm.adm_row + a, dm.adm_col + a, dm.nodes, (T *)dm.S + a * dm.k * dm.k, s_swizzled(dm),
                               dm.s_plane);
        if (nq > 0)
            hipLaunchKernelGGL(k_fill_N<TN>, dim3((unsigned)nq), dim3(256), 0, st, kernel, ell, shift, npts,
                               dm.near_row + q, dm.near_col + q, dm.near_off + q, dm.first, dm.size, dm.pts,
                               (TN *)dm.N, dm.near_t, dm.n_plane);
    }
    return hipGetLastError();
}

template <typename T, typename TN>
hipError_t fill_typed(const DevMat &dm, hipStream_t st) {
    const int64_t ck = (int64_t)dm.C * dm.k;
    hipLaunchKernelGGL(k_nodes, dim3((unsigned)((ck + 255) / 256)), dim3(256), 0, st, dm.C, dm.p, dm.box, dm.nodes);
    if (dm.L > 0)
        hipLaunchKernelGGL(k_fill_V<T>, dim3(dm.L), dim3(256), 0, st, dm.p, dm.leaves, dm.first, dm.size, dm.pts,
                           dm.nodes, (T *)dm.V, (T *)dm.Vt, dm.vt_off);
    if (dm.C > 1) {
        hipLaunchKernelGGL(k_fill_E<T>, dim3(dm.C - 1), dim3(256), 0, st, dm.p, dm.parent, dm.nodes, (T *)dm.E);
        const int64_t nf = (int64_t)dm.C * 3 * dm.p * dm.p;
        hipLaunchKernelGGL(k_fill_E1, dim3((unsigned)((nf + 255) / 256)), dim3(256), 0, st, dm.C, dm.p, dm.parent,
                           dm.nodes, dm.E1);
    }
    return fill_SN<T, TN>(dm, st);
}

template <typename T, typename TN>
hipError_t refill_typed(const DevMat &dm, hipStream_t st) {
    return fill_SN<T, TN>(dm, st);
}

}  // namespace

hipError_t refill_ell(DevMat &dm, double ell, hipStream_t st) {
    dm.ell = ell;
    switch (dm.storage) {
        case H2X_F64: return refill_typed<double, double>(dm, st);
        case H2X_F32: return refill_typed<float, float>(dm, st);
        default: return refill_typed<bf16_t, float>(dm, st);
    }
}

size_t mat_layout(const Plan &P, h2x_prec storage, DevMat *dm, char *base) {
    size_t cur = 0;
    const int32_t C = P.C, L = (int32_t)P.leaves.size(), k = P.k;
    const int64_t n = P.n, na = (int64_t)P.adm_col.size(), nn = (int64_t)P.near_col.size();
    DevMat d;
    d.n = n; d.C = C; d.L = L; d.k = k; d.p = P.p; d.depth_max = P.depth_max; d.max_leaf = P.max_leaf;
    d.max_near_rows = P.max_near_rows;
    d.leaf_half = P.leaf_half;
    d.n_adm = na; d.n_near = nn; d.near_entries = P.near_entries; d.storage = storage;
    d.kernel = P.prm.kernel; d.ell = P.prm.ell; d.shift = P.prm.shift; d.plan = &P;
    d.swz = k != 64 ? 0 : (storage == H2X_F64 ? 1 : (storage == H2X_F32 ? 2 : 3));
    // matrix-core layout (transposed near field, transposed leaf bases): FP64, k = 64 or k <= 32
    d.mc = (storage == H2X_F64 && (k == 64 || k <= 32)) ? 1 : 0;
    // low-precision operators with k = 64 use the same transposed near field (FP32) and leaf bases
    d.near_t = (d.mc || (storage != H2X_F64 && (k == 64 || k <= 32))) ? 1 : 0;
    d.first = carve<int32_t>(cur, base, C);
    d.size = carve<int32_t>(cur, base, C);
    d.parent = carve<int32_t>(cur, base, C);
    d.son0 = carve<int32_t>(cur, base, C);
    d.son1 = carve<int32_t>(cur, base, C);
    d.leaves = carve<int32_t>(cur, base, L);
    d.lvl_all = carve<int32_t>(cur, base, C);
    d.lvl_inner = carve<int32_t>(cur, base, P.lvl_inner.size() + 1);
    d.up_son = carve<int32_t>(cur, base, 2 * P.lvl_inner.size() + 1);
    d.dn_par = carve<int32_t>(cur, base, C);
    d.adm_ptr = carve<int64_t>(cur, base, C + 1);
    d.adm_col = carve<int32_t>(cur, base, na + 1);
    d.adm_row = carve<int32_t>(cur, base, na + 1);
    d.cpl_order = carve<int32_t>(cur, base, C);
    d.leaf_order = carve<int32_t>(cur, base, L);
    d.split_depth = P.split_depth;
    d.n_deep = (int32_t)P.cpl_deep.size();
    d.n_shallow = (int32_t)P.cpl_shallow.size();
    d.cpl_deep = carve<int32_t>(cur, base, d.n_deep + 1);
    d.cpl_shallow = carve<int32_t>(cur, base, d.n_shallow + 1);
    d.near_ptr = carve<int64_t>(cur, base, L + 1);
    d.near_col = carve<int32_t>(cur, base, nn + 1);
    d.near_row = carve<int32_t>(cur, base, nn + 1);
    d.near_off = carve<int64_t>(cur, base, nn + 1);
    d.vt_off = carve<int64_t>(cur, base, L + 1);
    d.near_off_rm = carve<int64_t>(cur, base, nn + 1);
    d.adm_cptr = carve<int64_t>(cur, base, C + 1);
    d.adm_cblk = carve<int64_t>(cur, base, na + 1);
    d.near_cptr = carve<int64_t>(cur, base, L + 1);
    d.near_cblk = carve<int64_t>(cur, base, nn + 1);
    d.sys_of = carve<int32_t>(cur, base, C);
    d.depth = carve<int32_t>(cur, base, C);
    d.perm = carve<int64_t>(cur, base, n);
    d.pts = carve<double>(cur, base, 3 * n);
    d.box = carve<double>(cur, base, 6 * (size_t)C);
    d.nodes = carve<double>(cur, base, 3 * (size_t)C * k);
    const size_t es = storage == H2X_F64 ? 8 : (storage == H2X_F32 ? 4 : 2);
    const size_t ens = storage == H2X_F64 ? 8 : 4;
    d.V = carve<char>(cur, base, es * (size_t)n * k);
    d.E = carve<char>(cur, base, es * (size_t)C * k * k);
    d.E1 = carve<double>(cur, base, 3 * (size_t)C * P.p * P.p);
    // complex kernel: a real and an imaginary plane of S and N (V and E stay real)
    d.cplx = (P.nsys() == 1 && P.prm.kernel == H2X_KERNEL_HELMHOLTZ) ? 1 : 0;
    const int planes = d.cplx ? 2 : 1;
    const int64_t nstored = d.near_t ? P.near_entries_t : P.near_entries;
    d.s_plane = d.cplx ? na * k * k : 0;
    d.n_plane = d.cplx ? nstored : 0;
    d.S = carve<char>(cur, base, es * planes * (size_t)(na ? na : 1) * k * k);
    d.N = carve<char>(cur, base, ens * planes * (size_t)(nstored ? nstored : 1) + 16);
    d.Vt = d.near_t ? carve<char>(cur, base, es * (size_t)P.vt_entries) : nullptr;
    if (dm) *dm = d;
    return align_up(cur);
}

hipError_t launch_fill(const DevMat &dm, hipStream_t st) {
    switch (dm.storage) {
        case H2X_F64: return fill_typed<double, double>(dm, st);
        case H2X_F32: return fill_typed<float, float>(dm, st);
        default: return fill_typed<bf16_t, float>(dm, st);
    }
}

}  // namespace h2x
