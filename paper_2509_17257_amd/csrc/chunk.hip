// Right-hand-side chunking (section 5, the remarks on the memory footprint of
// block CG and block GMRES): the solvers' auxiliary storage grows linearly in the
// number of right-hand sides m -- block CG keeps O(6 n m) numbers, block GMRES
// O(n (ell + 1) m) -- so for a large m the columns are solved in chunks of at most
// m_chunk.  The chunk size is chosen from the device memory the caller grants and
// from the measured time of one product per column count (the product dominates
// every iteration): among the candidate sizes whose workspace fits, the one with
// the least predicted time ceil(m / c) * t(c).  The iteration count of a chunk is
// that of its slowest column, which does not depend on how the columns are grouped,
// so the product time is the quantity that decides.
#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "device.hpp"

namespace h2x {

namespace {

// deterministic right-hand sides for the timing runs
__global__ void k_times_pattern(int64_t count, double *__restrict__ X) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < count) X[e] = (double)((e * 40503ll) % 1999 - 999) * 1e-3;
}

}  // namespace

size_t solve_ws_bytes(const DevMat &dm, int32_t solver, int64_t m, int32_t restart) {
    if (m < 1) return 0;
    if (solver == H2X_SOLVER_CG) return std::max(cg_ws_bytes(dm, m), bcg_ws_bytes(dm, m));
    if (solver == H2X_SOLVER_GMRES && restart >= 1) return gmres_ws_bytes(dm, m, restart);
    return 0;
}

h2x_status choose_chunk(const DevMat &dm, int32_t solver, int32_t restart, int64_t m, size_t mem_bytes, int32_t ncand,
                        const int64_t *cand, const double *ms, int64_t *m_chunk) {
    auto fits = [&](int64_t c) { return solve_ws_bytes(dm, solver, c, restart) <= mem_bytes; };
    if (!fits(1)) {
        set_error("h2x_choose_chunk: the workspace of one column exceeds the memory budget");
        return H2X_ENOMEM;
    }
    // the largest chunk that fits (the workspace does not decrease with the column count)
    int64_t lo = 1, hi = m;
    while (lo < hi) {
        const int64_t mid = lo + (hi - lo + 1) / 2;
        if (fits(mid)) lo = mid;
        else hi = mid - 1;
    }
    const int64_t cmax = lo;
    int64_t best = -1;
    double best_t = HUGE_VAL;
    for (int32_t i = 0; ms && i < ncand; ++i) {
        const int64_t c = std::min<int64_t>(cand[i], m);
        if (c < 1 || c > cmax || !(ms[i] > 0.0)) continue;
        const double t = (double)((m + c - 1) / c) * ms[i];
        if (t < best_t || (t == best_t && c > best)) {
            best_t = t;
            best = c;
        }
    }
    *m_chunk = best > 0 ? best : cmax;
    return H2X_OK;
}

size_t product_times_ws_bytes(const DevMat &dm, int32_t ncand, const int64_t *cand) {
    size_t need = 0;
    for (int32_t i = 0; i < ncand; ++i)
        if (cand[i] >= 1)
            need = std::max(need, 2 * align_up(sizeof(double) * (size_t)dm.n * (size_t)cand[i]) +
                                      matmul_ws_bytes(dm, cand[i]));
    return need;
}

h2x_status run_product_times(const DevMat &dm, int32_t ncand, const int64_t *cand, int32_t reps, char *ws,
                             size_t ws_bytes, hipStream_t st, double *ms) {
    if (ws_bytes < product_times_ws_bytes(dm, ncand, cand)) {
        set_error("h2x_product_times: workspace too small");
        return H2X_ENOMEM;
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    for (int32_t i = 0; i < ncand && e == hipSuccess; ++i) {
        const int64_t m = cand[i], cnt = dm.n * m;
        double *X = (double *)ws, *Y = (double *)(ws + align_up(sizeof(double) * cnt));
        char *mm = ws + 2 * align_up(sizeof(double) * cnt);
        hipLaunchKernelGGL(k_times_pattern, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, st, cnt, X);
        e = run_matmul(dm, m, 1.0, X, m, 0.0, Y, m, false, mm, st);  // untimed first run
        if (e == hipSuccess) e = hipEventRecord(e0, st);
        for (int32_t r = 0; r < reps && e == hipSuccess; ++r) e = run_matmul(dm, m, 1.0, X, m, 0.0, Y, m, false, mm, st);
        if (e == hipSuccess) e = hipEventRecord(e1, st);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float t = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
        ms[i] = e == hipSuccess ? (double)t / reps : 0.0;
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (e != hipSuccess) {
        set_error(std::string("h2x_product_times: ") + hipGetErrorString(e));
        return H2X_EHIP;
    }
    return H2X_OK;
}

namespace {

int worse(int a, int b) { return a != H2X_OK ? a : b; }

}  // namespace

h2x_status run_cg_chunked(const DevMat &dm, const h2x_cg_params &prm, int64_t m, int64_t mc, const double *B,
                          int64_t ldb, double *X, int64_t ldx, char *ws, size_t ws_bytes, h2x_cg_info *info,
                          hipStream_t st) {
    int32_t iters = 0, outer = 0, status = H2X_OK;
    for (int64_t c0 = 0; c0 < m; c0 += mc) {
        const int64_t cm = std::min(mc, m - c0);
        h2x_cg_info sub{};
        int32_t sys = 0;
        if (info) {
            sub.col_relres = info->col_relres ? info->col_relres + c0 : nullptr;
            sub.col_iters = info->col_iters ? info->col_iters + c0 : nullptr;
            sub.col_status = info->col_status ? info->col_status + c0 : nullptr;
            sub.sys_iters = &sys;
        }
        const h2x_status r = prm.variant == H2X_CG_SHARED
                                 ? run_block_cg_shared(dm, prm, cm, B + c0, ldb, X + c0, ldx, ws, ws_bytes,
                                                       info ? &sub : nullptr, st)
                                 : run_block_cg(dm, prm, cm, B + c0, ldb, X + c0, ldx, ws, ws_bytes,
                                                info ? &sub : nullptr, st);
        if (r != H2X_OK) return r;
        iters = std::max(iters, sub.iters);
        outer = std::max(outer, sub.outer_iters);
        status = worse(status, sub.status);
    }
    if (info) {
        info->iters = iters;
        info->outer_iters = outer;
        info->status = status;
        if (info->sys_iters) info->sys_iters[0] = iters;
    }
    return H2X_OK;
}

h2x_status run_gmres_chunked(const DevMat &dm, const h2x_gmres_params &prm, int64_t m, int64_t mc, const double *B,
                             int64_t ldb, double *X, int64_t ldx, char *ws, size_t ws_bytes, h2x_gmres_info *info,
                             hipStream_t st) {
    int32_t iters = 0, cycles = 0, status = H2X_OK;
    for (int64_t c0 = 0; c0 < m; c0 += mc) {
        const int64_t cm = std::min(mc, m - c0);
        h2x_gmres_info sub{};
        const int64_t ci = dm.cplx ? c0 / 2 : c0;  // info entries are per complex column
        if (info) {
            sub.col_res = info->col_res ? info->col_res + ci : nullptr;
            sub.col_iters = info->col_iters ? info->col_iters + ci : nullptr;
            sub.col_status = info->col_status ? info->col_status + ci : nullptr;
        }
        const h2x_status r =
            run_block_gmres(dm, prm, cm, B + c0, ldb, X + c0, ldx, ws, ws_bytes, info ? &sub : nullptr, st);
        if (r != H2X_OK) return r;
        iters = std::max(iters, sub.iters);
        cycles = std::max(cycles, sub.cycles);
        status = worse(status, sub.status);
    }
    if (info) {
        info->iters = iters;
        info->cycles = cycles;
        info->status = status;
    }
    return H2X_OK;
}

}  // namespace h2x
