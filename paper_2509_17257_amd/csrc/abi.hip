// C ABI entry points: argument validation, workspace layout, dispatch.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "device.hpp"

namespace h2x {

static thread_local std::string g_err;

void set_error(const std::string &msg) { g_err = msg; }

}  // namespace h2x

using namespace h2x;

namespace {

h2x_status fail(h2x_status s, const std::string &msg) {
    set_error(msg);
    return s;
}

h2x_status hip_fail(const char *where, hipError_t e) {
    return fail(H2X_EHIP, std::string(where) + ": " + hipGetErrorString(e));
}

bool aligned(const void *p) { return ((uintptr_t)p % kAlign) == 0; }

// complex operators: products take column pairs; CG (which needs a Hermitian positive
// definite operator), the adjoint, gradients, coupling access and batching are real only
h2x_status refuse_complex(const h2x_mat *A, const char *what) {
    if (A && A->dm.cplx) return fail(H2X_EUNSUPPORTED, std::string(what) + ": not for a complex operator");
    return H2X_OK;
}

h2x_status need_pairs(const h2x_mat *A, int64_t m, const char *what) {
    if (A && A->dm.cplx && (m & 1))
        return fail(H2X_EINVAL, std::string(what) + ": a complex operator takes an even number of real columns "
                                                    "(real and imaginary part of each complex column)");
    return H2X_OK;
}

template <typename T>
hipError_t upload(T *dst, const std::vector<T> &src, hipStream_t st) {
    if (src.empty()) return hipSuccess;
    return hipMemcpyAsync(dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice, st);
}

}  // namespace

extern "C" {

const char *h2x_last_error(void) { return g_err.c_str(); }
const char *h2x_version(void) { return "h2x 0.1 gfx950"; }

h2x_status h2x_plan_create(const double *pts, int64_t n, const h2x_params *prm, h2x_plan **out) {
    if (!out) return fail(H2X_EINVAL, "h2x_plan_create: out is NULL");
    *out = nullptr;
    if (!pts || !prm) return fail(H2X_EINVAL, "h2x_plan_create: NULL argument");
    if (n < 1 || n > (int64_t)1 << 30) return fail(H2X_EINVAL, "h2x_plan_create: n must be in [1, 2^30]");
    if (prm->cheb_order < 1 || prm->cheb_order > 8)
        return fail(H2X_EINVAL, "h2x_plan_create: cheb_order must be in [1, 8]");
    if (prm->leaf_size < 1) return fail(H2X_EINVAL, "h2x_plan_create: leaf_size must be >= 1");
    if (!(prm->eta > 0.0)) return fail(H2X_EINVAL, "h2x_plan_create: eta must be > 0");
    if (prm->kernel < H2X_KERNEL_EXP || prm->kernel > H2X_KERNEL_HELMHOLTZ)
        return fail(H2X_EINVAL, "h2x_plan_create: unknown kernel");
    if (prm->kernel == H2X_KERNEL_EXP && !(prm->ell > 0.0))
        return fail(H2X_EINVAL, "h2x_plan_create: ell must be > 0");
    if (prm->kernel == H2X_KERNEL_HELMHOLTZ && !(prm->ell >= 0.0 && std::isfinite(prm->ell)))
        return fail(H2X_EINVAL, "h2x_plan_create: the wavenumber (ell) must be finite and >= 0");
    for (int64_t i = 0; i < 3 * n; ++i)
        if (!std::isfinite(pts[i])) return fail(H2X_EINVAL, "h2x_plan_create: non-finite point coordinate");
    std::string err;
    Plan *P = build_plan(pts, n, *prm, err);
    if (!P) return fail(H2X_EINVAL, "h2x_plan_create: " + err);
    *out = new h2x_plan{P};
    return H2X_OK;
}

void h2x_plan_destroy(h2x_plan *plan) {
    if (!plan) return;
    delete plan->p;
    delete plan;
}

h2x_status h2x_plan_merge(const h2x_plan *const *plans, int32_t count, h2x_plan **out) {
    if (!out) return fail(H2X_EINVAL, "h2x_plan_merge: out is NULL");
    *out = nullptr;
    if (!plans || count < 1) return fail(H2X_EINVAL, "h2x_plan_merge: need count >= 1 plans");
    std::vector<const Plan *> parts;
    for (int32_t i = 0; i < count; ++i) {
        if (!plans[i]) return fail(H2X_EINVAL, "h2x_plan_merge: NULL plan");
        if (plans[i]->p->prm.kernel == H2X_KERNEL_HELMHOLTZ)
            return fail(H2X_EUNSUPPORTED, "h2x_plan_merge: complex (Helmholtz) plans are not batched");
        parts.push_back(plans[i]->p);
    }
    std::string err;
    Plan *P = merge_plans(parts, err);
    if (!P) return fail(H2X_EINVAL, "h2x_plan_merge: " + err);
    *out = new h2x_plan{P};
    return H2X_OK;
}

h2x_status h2x_plan_systems(const h2x_plan *plan, int32_t *count, int64_t *row_offsets) {
    if (!plan || !count) return fail(H2X_EINVAL, "h2x_plan_systems: NULL argument");
    const Plan &P = *plan->p;
    *count = P.nsys();
    if (row_offsets)
        for (int32_t i = 0; i <= P.nsys(); ++i) row_offsets[i] = P.sys_row[i];
    return H2X_OK;
}

h2x_status h2x_plan_stats(const h2x_plan *plan, h2x_stats *out) {
    if (!plan || !out) return fail(H2X_EINVAL, "h2x_plan_stats: NULL argument");
    const Plan &P = *plan->p;
    std::memset(out, 0, sizeof(*out));
    out->n = P.n;
    out->clusters = P.C;
    out->leaves = (int64_t)P.leaves.size();
    out->n_adm = (int64_t)P.adm_col.size();
    out->n_near = (int64_t)P.near_col.size();
    out->near_entries = P.near_entries;
    out->depth = P.depth_max;
    out->k = P.k;
    const int64_t ent = P.n * P.k + (int64_t)(P.C - 1) * P.k * P.k + out->n_adm * P.k * P.k;
    out->bytes_operator[H2X_F64] = 8 * ent;
    out->bytes_operator[H2X_F32] = 4 * ent;
    out->bytes_operator[H2X_BF16] = 2 * ent;
    out->bytes_near = 8 * P.near_entries;
    out->adm_depth = P.adm_depth;
    out->split_depth = P.split_depth;
    for (int32_t t : P.cpl_deep) out->deep_blocks += P.adm_ptr[t + 1] - P.adm_ptr[t];
    return H2X_OK;
}

h2x_status h2x_plan_perm(const h2x_plan *plan, int64_t *perm) {
    if (!plan || !perm) return fail(H2X_EINVAL, "h2x_plan_perm: NULL argument");
    std::memcpy(perm, plan->p->perm.data(), sizeof(int64_t) * plan->p->n);
    return H2X_OK;
}

h2x_status h2x_plan_clusters(const h2x_plan *plan, int64_t *first, int64_t *size, int64_t *parent, int64_t *son0,
                             int64_t *son1, int64_t *depth) {
    if (!plan) return fail(H2X_EINVAL, "h2x_plan_clusters: NULL plan");
    const Plan &P = *plan->p;
    for (int32_t c = 0; c < P.C; ++c) {
        if (first) first[c] = P.first[c];
        if (size) size[c] = P.size[c];
        if (parent) parent[c] = P.parent[c];
        if (son0) son0[c] = P.son0[c];
        if (son1) son1[c] = P.son1[c];
        if (depth) depth[c] = P.depth[c];
    }
    return H2X_OK;
}

h2x_status h2x_plan_blocks(const h2x_plan *plan, int64_t *adm_t, int64_t *adm_s, int64_t *near_t, int64_t *near_s) {
    if (!plan) return fail(H2X_EINVAL, "h2x_plan_blocks: NULL plan");
    const Plan &P = *plan->p;
    for (int32_t t = 0; t < P.C; ++t)
        for (int64_t b = P.adm_ptr[t]; b < P.adm_ptr[t + 1]; ++b) {
            if (adm_t) adm_t[b] = t;
            if (adm_s) adm_s[b] = P.adm_col[b];
        }
    for (size_t l = 0; l < P.leaves.size(); ++l)
        for (int64_t q = P.near_ptr[l]; q < P.near_ptr[l + 1]; ++q) {
            if (near_t) near_t[q] = P.leaves[l];
            if (near_s) near_s[q] = P.near_col[q];
        }
    return H2X_OK;
}

size_t h2x_mat_workspace_bytes(const h2x_plan *plan, h2x_prec storage) {
    if (!plan || storage < H2X_F64 || storage > H2X_BF16) return 0;
    return mat_layout(*plan->p, storage, nullptr, nullptr);
}

h2x_status h2x_mat_create(const h2x_plan *plan, h2x_prec storage, void *dev_ws, size_t ws_bytes, void *hip_stream,
                          h2x_mat **out) {
    if (!out) return fail(H2X_EINVAL, "h2x_mat_create: out is NULL");
    *out = nullptr;
    if (!plan || !dev_ws) return fail(H2X_EINVAL, "h2x_mat_create: NULL argument");
    if (storage < H2X_F64 || storage > H2X_BF16) return fail(H2X_EINVAL, "h2x_mat_create: bad storage precision");
    if (!aligned(dev_ws)) return fail(H2X_EINVAL, "h2x_mat_create: workspace not 256-byte aligned");
    const Plan &P = *plan->p;
    if (P.prm.kernel == H2X_KERNEL_HELMHOLTZ && (storage != H2X_F64 || !(P.k == 64 || P.k <= 32)))
        return fail(H2X_EUNSUPPORTED, "h2x_mat_create: the complex kernel needs FP64 storage and k = 64 or k <= 32");
    const size_t need = mat_layout(P, storage, nullptr, nullptr);
    if (ws_bytes < need) return fail(H2X_ENOMEM, "h2x_mat_create: workspace too small");
    auto *M = new h2x_mat{};
    M->plan = plan;
    M->ws_bytes = need;
    mat_layout(P, storage, &M->dm, (char *)dev_ws);
    DevMat &d = M->dm;
    hipStream_t st = (hipStream_t)hip_stream;

    std::vector<int32_t> adm_row(P.adm_col.size()), near_row(P.near_col.size());
    for (int32_t t = 0; t < P.C; ++t)
        for (int64_t b = P.adm_ptr[t]; b < P.adm_ptr[t + 1]; ++b) adm_row[b] = t;
    for (size_t l = 0; l < P.leaves.size(); ++l)
        for (int64_t q = P.near_ptr[l]; q < P.near_ptr[l + 1]; ++q) near_row[q] = P.leaves[l];

    hipError_t e = hipSuccess;
    auto up = [&](auto *dst, const auto &src) {
        if (e == hipSuccess) e = upload(dst, src, st);
    };
    up(d.first, P.first);
    up(d.size, P.size);
    up(d.parent, P.parent);
    up(d.son0, P.son0);
    up(d.son1, P.son1);
    up(d.leaves, P.leaves);
    up(d.lvl_all, P.lvl_all);
    up(d.lvl_inner, P.lvl_inner);
    std::vector<int32_t> up_son(2 * P.lvl_inner.size()), dn_par(P.C);
    for (size_t i = 0; i < P.lvl_inner.size(); ++i) {
        up_son[2 * i] = P.son0[P.lvl_inner[i]];
        up_son[2 * i + 1] = P.son1[P.lvl_inner[i]];
    }
    for (int32_t i = 0; i < P.C; ++i) dn_par[i] = P.parent[P.lvl_all[i]];
    up(d.up_son, up_son);
    up(d.dn_par, dn_par);
    up(d.adm_ptr, P.adm_ptr);
    up(d.adm_col, P.adm_col);
    up(d.adm_row, adm_row);
    up(d.cpl_order, P.cpl_order);
    up(d.leaf_order, P.leaf_order);
    up(d.cpl_deep, P.cpl_deep);
    up(d.cpl_shallow, P.cpl_shallow);
    up(d.near_ptr, P.near_ptr);
    up(d.near_col, P.near_col);
    up(d.near_row, near_row);
    up(d.near_off, d.near_t ? P.near_off_t : P.near_off);
    up(d.vt_off, P.vt_off);
    up(d.near_off_rm, P.near_off);
    up(d.adm_cptr, P.adm_cptr);
    up(d.adm_cblk, P.adm_cblk);
    up(d.near_cptr, P.near_cptr);
    up(d.near_cblk, P.near_cblk);
    std::vector<int32_t> sys_of(P.C);
    for (int32_t i = 0; i < P.nsys(); ++i)
        for (int64_t c = P.sys_C[i]; c < P.sys_C[i + 1]; ++c) sys_of[c] = i;
    up(d.sys_of, sys_of);
    up(d.depth, P.depth);
    up(d.perm, P.perm);
    up(d.pts, P.pts_tree);
    up(d.box, P.box);
    if (e == hipSuccess) e = launch_fill(d, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    // second stream (default priority) for the near field of the matrix-core path
    if (e == hipSuccess && d.mc && d.n_near > 0) {
        e = hipStreamCreateWithFlags(&d.side, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&d.ev_fork, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&d.ev_join, hipEventDisableTiming);
    }
    if (e != hipSuccess) {
        h2x_mat_destroy(M);
        return hip_fail("h2x_mat_create", e);
    }
    *out = M;
    return H2X_OK;
}

void h2x_mat_destroy(h2x_mat *mat) {
    if (!mat) return;
    if (mat->dm.side) {
        (void)hipStreamSynchronize(mat->dm.side);
        (void)hipStreamDestroy(mat->dm.side);
    }
    if (mat->dm.ev_fork) (void)hipEventDestroy(mat->dm.ev_fork);
    if (mat->dm.ev_join) (void)hipEventDestroy(mat->dm.ev_join);
    delete mat;
}

size_t h2x_matmul_workspace_bytes(const h2x_mat *A, int64_t m) {
    if (!A || m < 1) return 0;
    return matmul_ws_bytes(A->dm, m);
}

}  // extern "C"

namespace {

h2x_status validate_matmul(const char *who, const h2x_mat *A, int64_t m, const double *X, int64_t ldx, const double *Y,
                           int64_t ldy, int32_t flags, void *dev_ws, size_t ws_bytes) {
    const std::string w(who);
    if (!A || !X || !Y || !dev_ws) return fail(H2X_EINVAL, w + ": NULL argument");
    if (m < 1 || ldx < m || ldy < m) return fail(H2X_EINVAL, w + ": need m >= 1, ldx >= m, ldy >= m");
    if (flags & ~H2X_TREE_ORDER) return fail(H2X_EINVAL, w + ": unknown flags");
    if (!aligned(dev_ws)) return fail(H2X_EINVAL, w + ": workspace not 256-byte aligned");
    if (ws_bytes < matmul_ws_bytes(A->dm, m)) return fail(H2X_ENOMEM, w + ": workspace too small");
    const int64_t n = A->dm.n;
    const char *x0 = (const char *)X, *x1 = (const char *)(X + (n - 1) * ldx + m);
    const char *y0 = (const char *)Y, *y1 = (const char *)(Y + (n - 1) * ldy + m);
    if (x0 < y1 && y0 < x1) return fail(H2X_EINVAL, w + ": X and Y overlap");
    return H2X_OK;
}

}  // namespace

extern "C" {

h2x_status h2x_matmul(const h2x_mat *A, int64_t m, double alpha, const double *X, int64_t ldx, double beta, double *Y,
                      int64_t ldy, int32_t flags, void *dev_ws, size_t ws_bytes, void *hip_stream) {
    if (h2x_status r = need_pairs(A, m, "h2x_matmul")) return r;
    h2x_status s = validate_matmul("h2x_matmul", A, m, X, ldx, Y, ldy, flags, dev_ws, ws_bytes);
    if (s != H2X_OK) return s;
    hipError_t e = run_matmul(A->dm, m, alpha, X, ldx, beta, Y, ldy, (flags & H2X_TREE_ORDER) != 0, (char *)dev_ws,
                              (hipStream_t)hip_stream);
    if (e != hipSuccess) return hip_fail("h2x_matmul", e);
    return H2X_OK;
}

h2x_status h2x_matmul_timed(const h2x_mat *A, int64_t m, double alpha, const double *X, int64_t ldx, double beta,
                            double *Y, int64_t ldy, int32_t flags, void *dev_ws, size_t ws_bytes, void *hip_stream,
                            double *stage_ms) {
    if (h2x_status r = need_pairs(A, m, "h2x_matmul_timed")) return r;
    if (!stage_ms) return fail(H2X_EINVAL, "h2x_matmul_timed: stage_ms is NULL");
    h2x_status s = validate_matmul("h2x_matmul_timed", A, m, X, ldx, Y, ldy, flags, dev_ws, ws_bytes);
    if (s != H2X_OK) return s;
    hipEvent_t ev[7] = {};
    hipError_t e = hipSuccess;
    for (int i = 0; i < 7 && e == hipSuccess; ++i) e = hipEventCreate(&ev[i]);
    hipStream_t st = (hipStream_t)hip_stream;
    if (e == hipSuccess)
        e = run_matmul(A->dm, m, alpha, X, ldx, beta, Y, ldy, (flags & H2X_TREE_ORDER) != 0, (char *)dev_ws, st, ev);
    if (e == hipSuccess) e = hipEventSynchronize(ev[5]);
    if (e == hipSuccess) e = hipEventSynchronize(ev[6]);
    for (int i = 0; i < 5 && e == hipSuccess; ++i) {
        float ms = 0.f;
        e = hipEventElapsedTime(&ms, ev[i], ev[i + 1]);
        stage_ms[i] = ms;
    }
    for (auto &x : ev)
        if (x) (void)hipEventDestroy(x);
    if (e != hipSuccess) return hip_fail("h2x_matmul_timed", e);
    return H2X_OK;
}

}  // extern "C"

struct h2x_timer {
    int32_t slots = 0;
    std::vector<hipEvent_t> ev;  // slots x 7
};

extern "C" {

h2x_status h2x_timer_create(int32_t slots, h2x_timer **out) {
    if (!out) return fail(H2X_EINVAL, "h2x_timer_create: out is NULL");
    *out = nullptr;
    if (slots < 1) return fail(H2X_EINVAL, "h2x_timer_create: need slots >= 1");
    auto *t = new h2x_timer{};
    t->slots = slots;
    t->ev.assign((size_t)slots * 7, nullptr);
    hipError_t e = hipSuccess;
    for (auto &x : t->ev)
        if (e == hipSuccess) e = hipEventCreate(&x);
    if (e != hipSuccess) {
        h2x_timer_destroy(t);
        return hip_fail("h2x_timer_create", e);
    }
    *out = t;
    return H2X_OK;
}

void h2x_timer_destroy(h2x_timer *timer) {
    if (!timer) return;
    for (auto &x : timer->ev)
        if (x) (void)hipEventDestroy(x);
    delete timer;
}

h2x_status h2x_matmul_marked(const h2x_mat *A, int64_t m, double alpha, const double *X, int64_t ldx, double beta,
                             double *Y, int64_t ldy, int32_t flags, void *dev_ws, size_t ws_bytes, void *hip_stream,
                             h2x_timer *timer, int32_t slot) {
    if (h2x_status r = need_pairs(A, m, "h2x_matmul_marked")) return r;
    if (!timer || slot < 0 || slot >= timer->slots) return fail(H2X_EINVAL, "h2x_matmul_marked: bad timer or slot");
    h2x_status s = validate_matmul("h2x_matmul_marked", A, m, X, ldx, Y, ldy, flags, dev_ws, ws_bytes);
    if (s != H2X_OK) return s;
    const hipError_t e = run_matmul(A->dm, m, alpha, X, ldx, beta, Y, ldy, (flags & H2X_TREE_ORDER) != 0,
                                    (char *)dev_ws, (hipStream_t)hip_stream, timer->ev.data() + (size_t)7 * slot);
    if (e != hipSuccess) return hip_fail("h2x_matmul_marked", e);
    return H2X_OK;
}

h2x_status h2x_timer_read(const h2x_timer *timer, int32_t slot, double *stage_ms) {
    if (!timer || !stage_ms || slot < 0 || slot >= timer->slots)
        return fail(H2X_EINVAL, "h2x_timer_read: bad timer, slot or output");
    hipEvent_t *ev = const_cast<hipEvent_t *>(timer->ev.data()) + (size_t)7 * slot;
    hipError_t e = hipEventSynchronize(ev[6]);
    for (int i = 0; i < H2X_NUM_STAGES && e == hipSuccess; ++i) {
        float ms = 0.f;
        e = hipEventElapsedTime(&ms, ev[i], ev[i + 1]);
        stage_ms[i] = ms;
    }
    if (e != hipSuccess) return hip_fail("h2x_timer_read", e);
    return H2X_OK;
}

size_t h2x_block_cg_workspace_bytes(const h2x_mat *A, int64_t m) {
    if (!A || m < 1) return 0;
    return std::max(cg_ws_bytes(A->dm, m), bcg_ws_bytes(A->dm, m));
}

h2x_status h2x_block_cg(const h2x_mat *A, const h2x_cg_params *prm, int64_t m, const double *B, int64_t ldb,
                        double *X, int64_t ldx, void *dev_ws, size_t ws_bytes, h2x_cg_info *info, void *hip_stream) {
    if (h2x_status r = refuse_complex(A, "h2x_block_cg")) return r;
    if (!A || !prm || !B || !X || !dev_ws) return fail(H2X_EINVAL, "h2x_block_cg: NULL argument");
    if (m < 1 || ldb < m || ldx < m) return fail(H2X_EINVAL, "h2x_block_cg: need m >= 1, ldb >= m, ldx >= m");
    if (!(prm->rtol >= 0.0) || prm->max_iter < 0) return fail(H2X_EINVAL, "h2x_block_cg: bad rtol or max_iter");
    if (!aligned(dev_ws)) return fail(H2X_EINVAL, "h2x_block_cg: workspace not 256-byte aligned");
    if (prm->variant == H2X_CG_SHARED && A->dm.plan->nsys() > 1)
        return fail(H2X_EUNSUPPORTED, "h2x_block_cg: the shared-space variant is not for merged plans");
    if (prm->variant == H2X_CG_SHARED)
        return run_block_cg_shared(A->dm, *prm, m, B, ldb, X, ldx, (char *)dev_ws, ws_bytes, info,
                                   (hipStream_t)hip_stream);
    if (prm->variant != H2X_CG_INDEPENDENT) return fail(H2X_EINVAL, "h2x_block_cg: unknown variant");
    return run_block_cg(A->dm, *prm, m, B, ldb, X, ldx, (char *)dev_ws, ws_bytes, info, (hipStream_t)hip_stream);
}

size_t h2x_block_gmres_workspace_bytes(const h2x_mat *A, int64_t m, int32_t restart) {
    if (!A || m < 1 || restart < 1) return 0;
    return gmres_ws_bytes(A->dm, m, restart);
}

h2x_status h2x_block_gmres(const h2x_mat *A, const h2x_gmres_params *prm, int64_t m, const double *B, int64_t ldb,
                           double *X, int64_t ldx, void *dev_ws, size_t ws_bytes, h2x_gmres_info *info,
                           void *hip_stream) {
    if (h2x_status r = need_pairs(A, m, "h2x_block_gmres")) return r;
    if (!A || !prm || !B || !X || !dev_ws) return fail(H2X_EINVAL, "h2x_block_gmres: NULL argument");
    if (m < 1 || ldb < m || ldx < m) return fail(H2X_EINVAL, "h2x_block_gmres: need m >= 1, ldb >= m, ldx >= m");
    if (!(prm->rtol >= 0.0) || prm->restart < 1 || prm->max_iter < 0 || prm->check_every < 1)
        return fail(H2X_EINVAL, "h2x_block_gmres: need rtol >= 0, restart >= 1, max_iter >= 0, check_every >= 1");
    if (A->dm.plan->nsys() > 1) return fail(H2X_EUNSUPPORTED, "h2x_block_gmres: not for merged plans");
    if (!aligned(dev_ws)) return fail(H2X_EINVAL, "h2x_block_gmres: workspace not 256-byte aligned");
    if (ws_bytes < gmres_ws_bytes(A->dm, m, prm->restart))
        return fail(H2X_ENOMEM, "h2x_block_gmres: workspace too small");
    return run_block_gmres(A->dm, *prm, m, B, ldb, X, ldx, (char *)dev_ws, ws_bytes, info, (hipStream_t)hip_stream);
}

size_t h2x_solve_workspace_bytes(const h2x_plan *plan, h2x_prec storage, int32_t solver, int64_t m, int32_t restart) {
    if (!plan || storage < H2X_F64 || storage > H2X_BF16 || m < 1) return 0;
    DevMat dm;
    mat_layout(*plan->p, storage, &dm, nullptr);  // sizes only: no device memory behind it
    return solve_ws_bytes(dm, solver, m, restart);
}

h2x_status h2x_choose_chunk(const h2x_plan *plan, h2x_prec storage, int32_t solver, int32_t restart, int64_t m,
                            size_t mem_bytes, int32_t ncand, const int64_t *cand_m, const double *cand_ms,
                            int64_t *m_chunk) {
    if (!plan || !m_chunk) return fail(H2X_EINVAL, "h2x_choose_chunk: NULL argument");
    if (storage < H2X_F64 || storage > H2X_BF16 || m < 1 || ncand < 0 || (ncand > 0 && cand_ms && !cand_m))
        return fail(H2X_EINVAL, "h2x_choose_chunk: bad storage, m or candidates");
    if (solver != H2X_SOLVER_CG && !(solver == H2X_SOLVER_GMRES && restart >= 1))
        return fail(H2X_EINVAL, "h2x_choose_chunk: unknown solver or restart < 1");
    DevMat dm;
    mat_layout(*plan->p, storage, &dm, nullptr);
    return choose_chunk(dm, solver, restart, m, mem_bytes, ncand, cand_m, cand_ms, m_chunk);
}

size_t h2x_product_times_workspace_bytes(const h2x_mat *A, int32_t ncand, const int64_t *cand_m) {
    if (!A || ncand < 1 || !cand_m) return 0;
    return product_times_ws_bytes(A->dm, ncand, cand_m);
}

h2x_status h2x_product_times(const h2x_mat *A, int32_t ncand, const int64_t *cand_m, int32_t reps, void *dev_ws,
                             size_t ws_bytes, void *hip_stream, double *ms) {
    for (int32_t i = 0; A && cand_m && i < ncand; ++i)
        if (h2x_status r = need_pairs(A, cand_m[i], "h2x_product_times")) return r;
    if (!A || !cand_m || !ms || !dev_ws) return fail(H2X_EINVAL, "h2x_product_times: NULL argument");
    if (ncand < 1 || reps < 1) return fail(H2X_EINVAL, "h2x_product_times: need ncand >= 1 and reps >= 1");
    for (int32_t i = 0; i < ncand; ++i)
        if (cand_m[i] < 1) return fail(H2X_EINVAL, "h2x_product_times: column counts must be >= 1");
    if (!aligned(dev_ws)) return fail(H2X_EINVAL, "h2x_product_times: workspace not 256-byte aligned");
    return run_product_times(A->dm, ncand, cand_m, reps, (char *)dev_ws, ws_bytes, (hipStream_t)hip_stream, ms);
}

h2x_status h2x_block_cg_chunked(const h2x_mat *A, const h2x_cg_params *prm, int64_t m, int64_t m_chunk,
                                const double *B, int64_t ldb, double *X, int64_t ldx, void *dev_ws, size_t ws_bytes,
                                h2x_cg_info *info, void *hip_stream) {
    if (h2x_status r = refuse_complex(A, "h2x_block_cg_chunked")) return r;
    if (!A || !prm || !B || !X || !dev_ws) return fail(H2X_EINVAL, "h2x_block_cg_chunked: NULL argument");
    if (m < 1 || m_chunk < 1 || ldb < m || ldx < m)
        return fail(H2X_EINVAL, "h2x_block_cg_chunked: need m >= 1, m_chunk >= 1, ldb >= m, ldx >= m");
    if (!(prm->rtol >= 0.0) || prm->max_iter < 0) return fail(H2X_EINVAL, "h2x_block_cg_chunked: bad rtol or max_iter");
    if (prm->variant != H2X_CG_INDEPENDENT && prm->variant != H2X_CG_SHARED)
        return fail(H2X_EINVAL, "h2x_block_cg_chunked: unknown variant");
    if (A->dm.plan->nsys() > 1) return fail(H2X_EUNSUPPORTED, "h2x_block_cg_chunked: not for merged plans");
    if (!aligned(dev_ws)) return fail(H2X_EINVAL, "h2x_block_cg_chunked: workspace not 256-byte aligned");
    const int64_t mc = std::min(m_chunk, m);
    if (ws_bytes < solve_ws_bytes(A->dm, H2X_SOLVER_CG, mc, 0))
        return fail(H2X_ENOMEM, "h2x_block_cg_chunked: workspace too small for m_chunk columns");
    return run_cg_chunked(A->dm, *prm, m, mc, B, ldb, X, ldx, (char *)dev_ws, ws_bytes, info, (hipStream_t)hip_stream);
}

h2x_status h2x_block_gmres_chunked(const h2x_mat *A, const h2x_gmres_params *prm, int64_t m, int64_t m_chunk,
                                   const double *B, int64_t ldb, double *X, int64_t ldx, void *dev_ws,
                                   size_t ws_bytes, h2x_gmres_info *info, void *hip_stream) {
    if (h2x_status r = need_pairs(A, m, "h2x_block_gmres_chunked")) return r;
    if (h2x_status r = need_pairs(A, m_chunk, "h2x_block_gmres_chunked")) return r;
    if (!A || !prm || !B || !X || !dev_ws) return fail(H2X_EINVAL, "h2x_block_gmres_chunked: NULL argument");
    if (m < 1 || m_chunk < 1 || ldb < m || ldx < m)
        return fail(H2X_EINVAL, "h2x_block_gmres_chunked: need m >= 1, m_chunk >= 1, ldb >= m, ldx >= m");
    if (!(prm->rtol >= 0.0) || prm->restart < 1 || prm->max_iter < 0 || prm->check_every < 1)
        return fail(H2X_EINVAL, "h2x_block_gmres_chunked: bad rtol, restart, max_iter or check_every");
    if (A->dm.plan->nsys() > 1) return fail(H2X_EUNSUPPORTED, "h2x_block_gmres_chunked: not for merged plans");
    if (!aligned(dev_ws)) return fail(H2X_EINVAL, "h2x_block_gmres_chunked: workspace not 256-byte aligned");
    const int64_t mc = std::min(m_chunk, m);
    if (ws_bytes < gmres_ws_bytes(A->dm, mc, prm->restart))
        return fail(H2X_ENOMEM, "h2x_block_gmres_chunked: workspace too small for m_chunk columns");
    return run_gmres_chunked(A->dm, *prm, m, mc, B, ldb, X, ldx, (char *)dev_ws, ws_bytes, info,
                             (hipStream_t)hip_stream);
}

size_t h2x_block_cg_mixed_workspace_bytes(const h2x_mat *A, const h2x_mat *A_lo, int64_t m) {
    if (!A || !A_lo || m < 1) return 0;
    return mixed_ws_bytes(A->dm, A_lo->dm, m);
}

h2x_status h2x_block_cg_mixed(const h2x_mat *A, const h2x_mat *A_lo, const h2x_cg_params *prm, double delta,
                              int64_t m, const double *B, int64_t ldb, double *X, int64_t ldx, void *dev_ws,
                              size_t ws_bytes, h2x_cg_info *info, void *hip_stream) {
    if (h2x_status r = refuse_complex(A, "h2x_block_cg_mixed")) return r;
    if (h2x_status r = refuse_complex(A_lo, "h2x_block_cg_mixed")) return r;
    if (!A || !A_lo || !prm || !B || !X || !dev_ws) return fail(H2X_EINVAL, "h2x_block_cg_mixed: NULL argument");
    if (A->plan != A_lo->plan) return fail(H2X_EINVAL, "h2x_block_cg_mixed: A and A_lo must share one plan");
    if (A->dm.storage != H2X_F64) return fail(H2X_EINVAL, "h2x_block_cg_mixed: A must be stored in FP64");
    if (A->dm.plan->nsys() > 1) return fail(H2X_EUNSUPPORTED, "h2x_block_cg_mixed: not for merged plans");
    if (m < 1 || ldb < m || ldx < m) return fail(H2X_EINVAL, "h2x_block_cg_mixed: need m >= 1, ldb >= m, ldx >= m");
    if (!(prm->rtol >= 0.0) || prm->max_iter < 0 || !(delta > 0.0 && delta < 1.0))
        return fail(H2X_EINVAL, "h2x_block_cg_mixed: bad rtol, max_iter or delta");
    if (prm->variant != H2X_CG_INDEPENDENT)
        return fail(H2X_EUNSUPPORTED, "h2x_block_cg_mixed: only the independent variant");
    if (!aligned(dev_ws)) return fail(H2X_EINVAL, "h2x_block_cg_mixed: workspace not 256-byte aligned");
    if (ws_bytes < mixed_ws_bytes(A->dm, A_lo->dm, m)) return fail(H2X_ENOMEM, "h2x_block_cg_mixed: workspace too small");
    return run_block_cg_mixed(A->dm, A_lo->dm, *prm, delta, m, B, ldb, X, ldx, (char *)dev_ws, ws_bytes, info,
                              (hipStream_t)hip_stream);
}

size_t h2x_mat_autotune_workspace_bytes(const h2x_mat *A, int64_t m) {
    if (!A || m < 1) return 0;
    return autotune_ws_bytes(A->dm, m);
}

h2x_status h2x_mat_autotune(h2x_mat *A, int64_t m, void *dev_ws, size_t ws_bytes, void *hip_stream,
                            h2x_tune_info *info) {
    if (h2x_status r = need_pairs(A, m, "h2x_mat_autotune")) return r;
    if (!A || !dev_ws) return fail(H2X_EINVAL, "h2x_mat_autotune: NULL argument");
    if (m < 1) return fail(H2X_EINVAL, "h2x_mat_autotune: need m >= 1");
    if (!aligned(dev_ws)) return fail(H2X_EINVAL, "h2x_mat_autotune: workspace not 256-byte aligned");
    return run_autotune(A->dm, m, (char *)dev_ws, ws_bytes, (hipStream_t)hip_stream, info);
}

h2x_status h2x_mat_set_tune(h2x_mat *A, int64_t m, const h2x_tune_info *cfg) {
    if (!A || !cfg) return fail(H2X_EINVAL, "h2x_mat_set_tune: NULL argument");
    if (m < 1) return fail(H2X_EINVAL, "h2x_mat_set_tune: need m >= 1");
    auto in = [](int32_t v, int32_t hi) { return v >= 0 && v <= hi; };
    if (!in(cfg->nj_transfer, 4) || !in(cfg->nj_coupling, 4) || !in(cfg->np_leaf, 2) ||
        !in(cfg->overlap, 6) || !in(cfg->fuse_up, 2) || !in(cfg->leaf_kind, 3) || !in(cfg->split, 3))
        return fail(H2X_EINVAL, "h2x_mat_set_tune: a shape field is out of range");
    TuneCfg c{};
    c.nj_transfer = (int8_t)cfg->nj_transfer;
    c.nj_coupling = (int8_t)cfg->nj_coupling;
    c.np_leaf = (int8_t)cfg->np_leaf;
    c.overlap = (int8_t)cfg->overlap;
    c.fuse_up = (int8_t)cfg->fuse_up;
    c.leaf_kind = (int8_t)cfg->leaf_kind;
    c.split = (int8_t)cfg->split;
    A->dm.tuned[tune_bucket(m)] = c;
    return H2X_OK;
}

h2x_status h2x_mat_get_tune(const h2x_mat *A, int64_t m, h2x_tune_info *cfg) {
    if (!A || !cfg) return fail(H2X_EINVAL, "h2x_mat_get_tune: NULL argument");
    if (m < 1) return fail(H2X_EINVAL, "h2x_mat_get_tune: need m >= 1");
    const TuneCfg &c = A->dm.tuned[tune_bucket(m)];
    *cfg = h2x_tune_info{};
    cfg->nj_transfer = c.nj_transfer;
    cfg->nj_coupling = c.nj_coupling;
    cfg->np_leaf = c.np_leaf;
    cfg->overlap = c.overlap;
    cfg->fuse_up = c.fuse_up;
    cfg->leaf_kind = c.leaf_kind;
    cfg->split = c.split;
    return H2X_OK;
}

h2x_status h2x_batch_create(const h2x_mat *const *mats, int32_t count, h2x_batch **out) {
    for (int32_t i = 0; mats && i < count; ++i)
        if (h2x_status r = refuse_complex(mats[i], "h2x_batch_create")) return r;
    if (!out) return fail(H2X_EINVAL, "h2x_batch_create: out is NULL");
    *out = nullptr;
    if (!mats || count < 1) return fail(H2X_EINVAL, "h2x_batch_create: need count >= 1 operators");
    auto *b = new h2x_batch{};
    for (int32_t i = 0; i < count; ++i) {
        if (!mats[i]) {
            delete b;
            return fail(H2X_EINVAL, "h2x_batch_create: NULL operator");
        }
        b->mats.push_back(mats[i]);
        b->dms.push_back(&mats[i]->dm);
    }
    *out = b;
    return H2X_OK;
}

void h2x_batch_destroy(h2x_batch *batch) { delete batch; }

size_t h2x_batch_matmul_workspace_bytes(const h2x_batch *batch, int64_t m) {
    if (!batch || m < 1) return 0;
    size_t b = 0;
    for (auto *d : batch->dms) b = std::max(b, matmul_ws_bytes(*d, m));
    return b;
}

h2x_status h2x_batch_matmul(const h2x_batch *batch, int64_t m, double alpha, const double *X, int64_t ldx,
                            double beta, double *Y, int64_t ldy, int32_t flags, void *dev_ws, size_t ws_bytes,
                            void *hip_stream) {
    if (!batch || !X || !Y || !dev_ws) return fail(H2X_EINVAL, "h2x_batch_matmul: NULL argument");
    if (m < 1 || ldx < m || ldy < m) return fail(H2X_EINVAL, "h2x_batch_matmul: need m >= 1, ldx >= m, ldy >= m");
    if (flags & ~H2X_TREE_ORDER) return fail(H2X_EINVAL, "h2x_batch_matmul: unknown flags");
    if (!aligned(dev_ws)) return fail(H2X_EINVAL, "h2x_batch_matmul: workspace not 256-byte aligned");
    if (ws_bytes < h2x_batch_matmul_workspace_bytes(batch, m))
        return fail(H2X_ENOMEM, "h2x_batch_matmul: workspace too small");
    int64_t n = 0;
    for (auto *d : batch->dms) n += d->n;
    const char *x0 = (const char *)X, *x1 = (const char *)(X + (n - 1) * ldx + m);
    const char *y0 = (const char *)Y, *y1 = (const char *)(Y + (n - 1) * ldy + m);
    if (x0 < y1 && y0 < x1) return fail(H2X_EINVAL, "h2x_batch_matmul: X and Y overlap");
    int64_t r = 0;
    for (auto *d : batch->dms) {
        hipError_t e = run_matmul(*d, m, alpha, X + r * ldx, ldx, beta, Y + r * ldy, ldy, (flags & H2X_TREE_ORDER) != 0,
                                  (char *)dev_ws, (hipStream_t)hip_stream);
        if (e != hipSuccess) return hip_fail("h2x_batch_matmul", e);
        r += d->n;
    }
    return H2X_OK;
}

size_t h2x_batch_block_cg_workspace_bytes(const h2x_batch *batch, int64_t m) {
    if (!batch || m < 1) return 0;
    return cg_batch_ws_bytes(batch->dms.data(), (int32_t)batch->dms.size(), m);
}

h2x_status h2x_batch_block_cg(const h2x_batch *batch, const h2x_cg_params *prm, int64_t m, const double *B,
                              int64_t ldb, double *X, int64_t ldx, void *dev_ws, size_t ws_bytes, h2x_cg_info *info,
                              void *hip_stream) {
    if (!batch || !prm || !B || !X || !dev_ws) return fail(H2X_EINVAL, "h2x_batch_block_cg: NULL argument");
    if (m < 1 || ldb < m || ldx < m) return fail(H2X_EINVAL, "h2x_batch_block_cg: need m >= 1, ldb >= m, ldx >= m");
    if (!(prm->rtol >= 0.0) || prm->max_iter < 0) return fail(H2X_EINVAL, "h2x_batch_block_cg: bad rtol or max_iter");
    if (prm->variant != H2X_CG_INDEPENDENT)
        return fail(H2X_EUNSUPPORTED, "h2x_batch_block_cg: only the independent variant");
    if (!aligned(dev_ws)) return fail(H2X_EINVAL, "h2x_batch_block_cg: workspace not 256-byte aligned");
    return run_block_cg_batch(batch->dms.data(), (int32_t)batch->dms.size(), *prm, m, B, ldb, X, ldx, (char *)dev_ws,
                              ws_bytes, info, (hipStream_t)hip_stream);
}

size_t h2x_matmul_adjoint_workspace_bytes(const h2x_mat *A, int64_t m) {
    if (!A || m < 1) return 0;
    return adjoint_ws_bytes(A->dm, m);
}

size_t h2x_grad_workspace_bytes(const h2x_mat *A, int64_t m) {
    if (!A || m < 1) return 0;
    return grad_ws_bytes(A->dm, m);
}

h2x_status h2x_matmul_adjoint(const h2x_mat *A, int64_t m, double alpha, const double *X, int64_t ldx, double beta,
                              double *Y, int64_t ldy, void *dev_ws, size_t ws_bytes, void *hip_stream) {
    if (h2x_status r = refuse_complex(A, "h2x_matmul_adjoint")) return r;
    if (!A || !X || !Y || !dev_ws) return fail(H2X_EINVAL, "h2x_matmul_adjoint: NULL argument");
    if (A->dm.storage != H2X_F64 || A->dm.k > 64)
        return fail(H2X_EUNSUPPORTED, "h2x_matmul_adjoint: FP64 operators with k <= 64 only");
    if (m < 1 || ldx < m || ldy < m) return fail(H2X_EINVAL, "h2x_matmul_adjoint: need m >= 1, ldx >= m, ldy >= m");
    if (!aligned(dev_ws)) return fail(H2X_EINVAL, "h2x_matmul_adjoint: workspace not 256-byte aligned");
    if (ws_bytes < adjoint_ws_bytes(A->dm, m)) return fail(H2X_ENOMEM, "h2x_matmul_adjoint: workspace too small");
    const int64_t n = A->dm.n;
    const char *x0 = (const char *)X, *x1 = (const char *)(X + (n - 1) * ldx + m);
    const char *y0 = (const char *)Y, *y1 = (const char *)(Y + (n - 1) * ldy + m);
    if (x0 < y1 && y0 < x1) return fail(H2X_EINVAL, "h2x_matmul_adjoint: X and Y overlap");
    hipError_t e = run_matmul_adjoint(A->dm, m, alpha, X, ldx, beta, Y, ldy, (char *)dev_ws, (hipStream_t)hip_stream);
    if (e != hipSuccess) return hip_fail("h2x_matmul_adjoint", e);
    return H2X_OK;
}

h2x_status h2x_grad(const h2x_mat *A, int64_t m, const double *X, int64_t ldx, const double *dY, int64_t lddy,
                    double *dS, double *dN, double *dell, double scale, int32_t dell_terms, void *dev_ws,
                    size_t ws_bytes, void *hip_stream) {
    if (h2x_status r = refuse_complex(A, "h2x_grad")) return r;
    if (!A || !X || !dY || !dev_ws) return fail(H2X_EINVAL, "h2x_grad: NULL argument");
    if (A->dm.storage != H2X_F64 || A->dm.k > 64)
        return fail(H2X_EUNSUPPORTED, "h2x_grad: FP64 operators with k <= 64 only");
    if (A->dm.plan->nsys() > 1) return fail(H2X_EUNSUPPORTED, "h2x_grad: not for merged plans");
    if (m < 1 || ldx < m || lddy < m) return fail(H2X_EINVAL, "h2x_grad: need m >= 1, ldx >= m, lddy >= m");
    if (!aligned(dev_ws)) return fail(H2X_EINVAL, "h2x_grad: workspace not 256-byte aligned");
    if (ws_bytes < grad_ws_bytes(A->dm, m)) return fail(H2X_ENOMEM, "h2x_grad: workspace too small");
    if (dell_terms & ~(H2X_DELL_COUPLING | H2X_DELL_NEAR)) return fail(H2X_EINVAL, "h2x_grad: unknown dell_terms");
    if (!std::isfinite(scale)) return fail(H2X_EINVAL, "h2x_grad: scale must be finite");
    if (!dS && !dN && !dell) return H2X_OK;
    hipError_t e = run_grad(A->dm, m, X, ldx, dY, lddy, dS, dN, dell, scale, dell_terms, (char *)dev_ws,
                            (hipStream_t)hip_stream);
    if (e != hipSuccess) return hip_fail("h2x_grad", e);
    return H2X_OK;
}

h2x_status h2x_mat_set_ell(h2x_mat *A, double ell, void *hip_stream) {
    if (!A) return fail(H2X_EINVAL, "h2x_mat_set_ell: NULL operator");
    if (!(ell > 0.0) || !std::isfinite(ell)) return fail(H2X_EINVAL, "h2x_mat_set_ell: ell must be finite and > 0");
    if (A->dm.plan->nsys() > 1) return fail(H2X_EUNSUPPORTED, "h2x_mat_set_ell: not for merged plans");
    hipStream_t st = (hipStream_t)hip_stream;
    hipError_t e = refill_ell(A->dm, ell, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail("h2x_mat_set_ell", e);
    return H2X_OK;
}

h2x_status h2x_mat_coupling(const h2x_mat *A, double *out, void *hip_stream) {
    if (h2x_status r = refuse_complex(A, "h2x_mat_coupling")) return r;
    if (!A || !out) return fail(H2X_EINVAL, "h2x_mat_coupling: NULL argument");
    if (A->dm.storage != H2X_F64) return fail(H2X_EUNSUPPORTED, "h2x_mat_coupling: FP64 operators only");
    hipError_t e = run_read_coupling(A->dm, out, (hipStream_t)hip_stream);
    if (e != hipSuccess) return hip_fail("h2x_mat_coupling", e);
    return H2X_OK;
}

h2x_status h2x_mat_set_coupling(h2x_mat *A, const double *in, void *hip_stream) {
    if (h2x_status r = refuse_complex(A, "h2x_mat_set_coupling")) return r;
    if (!A || !in) return fail(H2X_EINVAL, "h2x_mat_set_coupling: NULL argument");
    if (A->dm.storage != H2X_F64) return fail(H2X_EUNSUPPORTED, "h2x_mat_set_coupling: FP64 operators only");
    hipError_t e = run_write_coupling(A->dm, in, (hipStream_t)hip_stream);
    if (e != hipSuccess) return hip_fail("h2x_mat_set_coupling", e);
    return H2X_OK;
}

size_t h2x_block_cg_refine_workspace_bytes(const h2x_mat *A, const h2x_mat *A_lo, int64_t m) {
    if (!A || !A_lo || m < 1) return 0;
    return refine_ws_bytes(A->dm, A_lo->dm, m);
}

h2x_status h2x_block_cg_refine(const h2x_mat *A, const h2x_mat *A_lo, const h2x_cg_params *inner, double rtol,
                               int32_t max_outer, int64_t m, const double *B, int64_t ldb, double *X, int64_t ldx,
                               void *dev_ws, size_t ws_bytes, h2x_cg_info *info, void *hip_stream) {
    if (h2x_status r = refuse_complex(A, "h2x_block_cg_refine")) return r;
    if (h2x_status r = refuse_complex(A_lo, "h2x_block_cg_refine")) return r;
    if (!A || !A_lo || !inner || !B || !X || !dev_ws) return fail(H2X_EINVAL, "h2x_block_cg_refine: NULL argument");
    if (A->plan != A_lo->plan) return fail(H2X_EINVAL, "h2x_block_cg_refine: A and A_lo must share one plan");
    if (A->dm.storage != H2X_F64) return fail(H2X_EINVAL, "h2x_block_cg_refine: A must be stored in FP64");
    if (A->dm.plan->nsys() > 1) return fail(H2X_EUNSUPPORTED, "h2x_block_cg_refine: not for merged plans");
    if (m < 1 || ldb < m || ldx < m) return fail(H2X_EINVAL, "h2x_block_cg_refine: need m >= 1, ldb >= m, ldx >= m");
    if (!(rtol >= 0.0) || max_outer < 0 || !(inner->rtol >= 0.0) || inner->max_iter < 0)
        return fail(H2X_EINVAL, "h2x_block_cg_refine: bad tolerance or iteration limit");
    if (!aligned(dev_ws)) return fail(H2X_EINVAL, "h2x_block_cg_refine: workspace not 256-byte aligned");
    return run_refine(A->dm, A_lo->dm, *inner, rtol, max_outer, m, B, ldb, X, ldx, (char *)dev_ws, ws_bytes, info,
                      (hipStream_t)hip_stream);
}

}  // extern "C"
