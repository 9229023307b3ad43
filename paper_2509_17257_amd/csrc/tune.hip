// Autotuner of the matrix-core tile shapes.  For one operator and one column
// count m it times the product with each candidate tile width per stage (HIP
// events around every stage), keeps the fastest per stage, and stores the
// choice in the operator's table for m's bucket; later products with a column
// count in that bucket use it.  Candidates: 16-column tiles per work-group of
// the forward leaf and transfer passes (1 .. ceil(m / 16), at most 4), of the
// coupling (same range), the leaf stage (a 64-row tile per wave and term, or a wave
// per 32-row band, with 1 or 2 32-column tiles),
// whether the near field runs on a second stream concurrently with the transfer
// passes, and whether the coupling of the deep rows runs on it beside the upper
// transfer levels (whole-product times decide the last and the final choice).
#include <cmath>
#include <string>
#include <vector>

#include "device.hpp"

namespace h2x {

namespace {

// deterministic right-hand sides for the timing runs
__global__ void k_pattern(int64_t count, double *__restrict__ X) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < count) X[e] = (double)((e * 2654435761ll) % 2001 - 1000) * 1e-3;
}

}  // namespace

size_t autotune_ws_bytes(const DevMat &dm, int64_t m) {
    return 2 * align_up((size_t)dm.n * m * sizeof(double)) + matmul_ws_bytes(dm, m);
}

h2x_status run_autotune(DevMat &dm, int64_t m, char *ws, size_t ws_bytes, hipStream_t st, h2x_tune_info *info) {
    if (ws_bytes < autotune_ws_bytes(dm, m)) {
        set_error("h2x_mat_autotune: workspace too small");
        return H2X_ENOMEM;
    }
    const size_t nm = align_up((size_t)dm.n * m * sizeof(double));
    double *X = (double *)ws, *Y = (double *)(ws + nm);
    char *mm = ws + 2 * nm;
    hipEvent_t ev[7] = {};
    hipError_t e = hipSuccess;
    for (int i = 0; i < 7 && e == hipSuccess; ++i) e = hipEventCreate(&ev[i]);
    auto done = [&](hipError_t err) {
        for (auto &x : ev)
            if (x) (void)hipEventDestroy(x);
        if (err != hipSuccess) {
            set_error(std::string("h2x_mat_autotune: ") + hipGetErrorString(err));
            return H2X_EHIP;
        }
        return H2X_OK;
    };
    if (e != hipSuccess) return done(e);
    const int64_t cnt = dm.n * m;
    hipLaunchKernelGGL(k_pattern, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, st, cnt, X);

    constexpr int reps = 3;
    // mean per-stage times of the product with tile choices c (one untimed run first)
    auto time_cfg = [&](const TuneCfg &c, double *stage) {
        hipError_t r = run_matmul_cfg(dm, c, m, 1.0, X, m, 0.0, Y, m, false, mm, st, nullptr, nullptr);
        for (int i = 0; i < 5; ++i) stage[i] = 0.0;
        for (int q = 0; q < reps && r == hipSuccess; ++q) {
            r = run_matmul_cfg(dm, c, m, 1.0, X, m, 0.0, Y, m, false, mm, st, ev, nullptr);
            if (r == hipSuccess) r = hipEventSynchronize(ev[6]);
            for (int i = 0; i < 5 && r == hipSuccess; ++i) {
                float ms = 0.f;
                r = hipEventElapsedTime(&ms, ev[i], ev[i + 1]);
                stage[i] += ms / reps;
            }
        }
        return r;
    };
    auto total = [](const double *s) { return s[0] + s[1] + s[2] + s[3] + s[4]; };

    const int b = tune_bucket(m);
    const int max_nj = (int)std::min<int64_t>(4, (m + 15) / 16);
    double s0[5];
    dm.tuned[b] = TuneCfg{};
    e = time_cfg(TuneCfg{}, s0);
    if (e != hipSuccess) return done(e);
    TuneCfg best{};
    double best_t = HUGE_VAL, best_c = HUGE_VAL, best_l = HUGE_VAL;
    for (int nj = 1; nj <= max_nj && e == hipSuccess; ++nj) {
        double s[5];
        TuneCfg c{};
        c.nj_transfer = (int8_t)nj;
        e = time_cfg(c, s);
        const double tt = s[0] + s[1] + s[3];  // forward leaf, forward and backward transfer passes
        if (e == hipSuccess && tt < best_t) {
            best_t = tt;
            best.nj_transfer = (int8_t)nj;
        }
        c = TuneCfg{};
        c.nj_coupling = (int8_t)nj;
        if (e == hipSuccess) e = time_cfg(c, s);
        if (e == hipSuccess && s[2] < best_c) {
            best_c = s[2];
            best.nj_coupling = (int8_t)nj;
        }
    }
    // leaf stage: a 64-row tile per wave and term, a wave per 32-row band (FP64 matrix-core
    // path) or one contraction per leaf (matrix-core paths), with 32 * np columns per wave
    for (int kind = 1; kind <= (dm.mc ? 3 : 1) && e == hipSuccess; ++kind)
        for (int np = 1; np <= (m > 32 ? 2 : 1) && e == hipSuccess; ++np) {
            double s[5];
            TuneCfg c{};
            c.np_leaf = (int8_t)np;
            c.leaf_kind = (int8_t)kind;
            e = time_cfg(c, s);
            // the whole product decides (the forms' placements of the near field differ)
            if (e == hipSuccess && total(s) < best_l) {
                best_l = total(s);
                best.np_leaf = (int8_t)np;
                best.leaf_kind = (int8_t)kind;
            }
        }
    if (e != hipSuccess) return done(e);
    // forward leaf and upward pass fused into one launch or level by level
    if (dm.mc) {
        double sf[5], ss[5];
        TuneCfg c = best;
        c.fuse_up = 1;
        e = time_cfg(c, sf);
        c.fuse_up = 2;
        if (e == hipSuccess) e = time_cfg(c, ss);
        if (e != hipSuccess) return done(e);
        best.fuse_up = (sf[0] + sf[1] <= ss[0] + ss[1]) ? 1 : 2;
    }
    // near field concurrent with the transfer passes (it changes the time of several
    // stages, so the whole product decides)
    if (dm.side) {
        double best_o = HUGE_VAL;
        for (int o : {1, 2, 3, 4, 5}) {
            double so[5];
            TuneCfg c = best;
            c.overlap = (int8_t)o;
            e = time_cfg(c, so);
            if (e != hipSuccess) return done(e);
            if (total(so) < best_o) {
                best_o = total(so);
                best.overlap = (int8_t)o;
            }
        }
    }
    // mean time of the whole product, events around the call only (the split schedule
    // and the stage events exclude each other)
    auto time_whole = [&](const TuneCfg &c, double &ms) {
        hipError_t r = run_matmul_cfg(dm, c, m, 1.0, X, m, 0.0, Y, m, false, mm, st, nullptr, nullptr);
        if (r == hipSuccess) r = hipEventRecord(ev[0], st);
        for (int q = 0; q < reps && r == hipSuccess; ++q)
            r = run_matmul_cfg(dm, c, m, 1.0, X, m, 0.0, Y, m, false, mm, st, nullptr, nullptr);
        if (r == hipSuccess) r = hipEventRecord(ev[6], st);
        if (r == hipSuccess) r = hipEventSynchronize(ev[6]);
        float t = 0.f;
        if (r == hipSuccess) r = hipEventElapsedTime(&t, ev[0], ev[6]);
        ms = (double)t / reps;
        return r;
    };
    // the near field in two halves beside the transfer passes (whole products decide, as the
    // stage events exclude it); kept when it wins by 1 %
    double w_best = 0.0, w0 = 0.0;
    if (dm.side && dm.mc && best.fuse_up != 1) {
        TuneCfg c = best;
        c.overlap = 6;
        double w6 = 0.0, wb = 0.0;
        e = time_whole(best, wb);
        if (e == hipSuccess) e = time_whole(c, w6);
        if (e != hipSuccess) return done(e);
        if (w6 * 1.01 < wb) best.overlap = 6;
    }
    // coupling of the deep rows beside the upper transfer levels, on or off
    if (dm.side && dm.split_depth > 0 && best.fuse_up != 1 &&
        !(best.overlap == 1 || best.overlap == 3 || best.overlap == 4 || best.overlap == 6)) {
        // the second stream and its events cost something on every product: the split has
        // to win by 1 % over the single launch
        double w_min = HUGE_VAL;
        for (int sp : {2, 1, 3}) {
            TuneCfg c = best;
            c.split = (int8_t)sp;
            double w = 0.0;
            e = time_whole(c, w);
            if (e != hipSuccess) return done(e);
            if (sp != 2) w *= 1.01;
            if (w < w_min) {
                w_min = w;
                best.split = (int8_t)sp;
            }
        }
    }
    e = time_whole(best, w_best);
    if (e == hipSuccess) e = time_whole(TuneCfg{}, w0);
    if (e != hipSuccess) return done(e);
    // keep the default when the combination is not faster
    const bool use = w_best < w0;
    dm.tuned[b] = use ? best : TuneCfg{};
    if (info) {
        info->nj_transfer = dm.tuned[b].nj_transfer;
        info->nj_coupling = dm.tuned[b].nj_coupling;
        info->np_leaf = dm.tuned[b].np_leaf;
        info->overlap = dm.tuned[b].overlap;
        info->fuse_up = dm.tuned[b].fuse_up;
        info->leaf_kind = dm.tuned[b].leaf_kind;
        info->split = dm.tuned[b].split;
        info->ms_default = w0;
        info->ms_tuned = use ? w_best : w0;
    }
    return done(hipSuccess);
}

}  // namespace h2x
