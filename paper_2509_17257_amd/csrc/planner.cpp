// Host planner: cluster tree, block tree and row-cluster lists (section 2 and
// Algorithm "prepare_addeval" of section 3), laid out as flat CSR arrays for the
// device.  Iterative (explicit stacks) so deep trees cannot overflow the call
// stack.  Built with -ffp-contract=off: the admissibility test compares
// floating-point distances, and its outcome must not depend on FMA contraction.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "plan.hpp"

namespace h2x {

namespace {

struct Pending {
    int64_t first, size;
    int32_t parent, depth;
    int which;  // 0: first son of parent, 1: second son
};

double box_diam(const double *lo, const double *hi) {
    double s = 0.0;
    for (int d = 0; d < 3; ++d) {
        double e = hi[d] - lo[d];
        s += e * e;
    }
    return std::sqrt(s);
}

double box_dist(const double *lo_t, const double *hi_t, const double *lo_s, const double *hi_s) {
    double s = 0.0;
    for (int d = 0; d < 3; ++d) {
        double g = std::max(0.0, std::max(lo_s[d] - hi_t[d], lo_t[d] - hi_s[d]));
        s += g * g;
    }
    return std::sqrt(s);
}

// launch order of coupling rows (ascending cluster ids): 8 contiguous eighths (one per
// XCD), longest list first within each
void xcd_order(const Plan &P, std::vector<int32_t> &rows) {
    const int32_t R = (int32_t)rows.size(), rpx = (R + 7) / 8;
    for (int32_t x = 0; x < 8; ++x) {
        const int32_t lo = std::min(R, x * rpx), hi = std::min(R, (x + 1) * rpx);
        std::stable_sort(rows.begin() + lo, rows.begin() + hi, [&](int32_t a, int32_t b) {
            return P.adm_ptr[a + 1] - P.adm_ptr[a] > P.adm_ptr[b + 1] - P.adm_ptr[b];
        });
    }
}

void coupling_order(Plan &P) {
    const int32_t C = P.C;
    P.cpl_order.resize(C);
    for (int32_t c = 0; c < C; ++c) P.cpl_order[c] = c;
    xcd_order(P, P.cpl_order);

    // deep / shallow split: the deepest split depth D whose deep part still holds at least
    // 60 % of the admissible blocks, so that its coupling outlasts the upper transfer levels,
    // the coupling of the other rows and the upper downward levels running beside it
    const int64_t total = P.adm_ptr[C];
    std::vector<int32_t> ready(C, 1 << 30);  // shallowest inner cluster of the list
    for (int32_t t = 0; t < C; ++t)
        for (int64_t b = P.adm_ptr[t]; b < P.adm_ptr[t + 1]; ++b) {
            const int32_t s = P.adm_col[b];
            if (P.son0[s] >= 0) ready[t] = std::min(ready[t], P.depth[s]);
        }
    auto deep = [&](int32_t t, int32_t D) { return P.depth[t] >= D && ready[t] >= D; };
    P.split_depth = 0;
    for (int32_t D = P.depth_max; D > P.adm_depth + 1 && total > 0; --D) {
        int64_t nb = 0;
        for (int32_t t = 0; t < C; ++t)
            if (deep(t, D)) nb += P.adm_ptr[t + 1] - P.adm_ptr[t];
        if (10 * nb >= 6 * total) {
            P.split_depth = D;
            break;
        }
    }
    P.cpl_deep.clear();
    P.cpl_shallow.clear();
    if (P.split_depth > 0) {
        for (int32_t t = 0; t < C; ++t) (deep(t, P.split_depth) ? P.cpl_deep : P.cpl_shallow).push_back(t);
        xcd_order(P, P.cpl_deep);
        xcd_order(P, P.cpl_shallow);
    }
}

// leaf order of the leaf stage: the work of a leaf is its rounds of 16 contraction rows
// (near rows and the k basis rows) per wave, over 4 waves for leaves of up to 32 points and
// 2 waves per 32-row group above, for each 64-row chunk of the leaf
void leaf_order(Plan &P) {
    const int32_t L = (int32_t)P.leaves.size(), lpx = (L + 7) / 8;
    std::vector<int64_t> work(L);
    for (int32_t l = 0; l < L; ++l) {
        int64_t rows = 0;
        for (int64_t q = P.near_ptr[l]; q < P.near_ptr[l + 1]; ++q) rows += P.size[P.near_col[q]];
        const int32_t nt = P.size[P.leaves[l]];
        int64_t w = 0;
        for (int32_t i0 = 0; i0 < nt; i0 += 64) {
            const int32_t ntile = (std::min(64, nt - i0) + 15) / 16;
            const int64_t rounds = (rows + 15) / 16 + (P.k + 15) / 16;
            w += (rounds + (ntile > 2 ? 1 : 3)) / (ntile > 2 ? 2 : 4);
        }
        work[l] = w;
    }
    P.leaf_order.resize(L);
    for (int32_t l = 0; l < L; ++l) P.leaf_order[l] = l;
    for (int32_t x = 0; x < 8; ++x) {
        const int32_t lo = std::min(L, x * lpx), hi = std::min(L, (x + 1) * lpx);
        std::stable_sort(P.leaf_order.begin() + lo, P.leaf_order.begin() + hi,
                         [&](int32_t a, int32_t b) { return work[a] > work[b]; });
    }
    // the first q positions of every eighth hold about half of the near-field entries
    std::vector<int64_t> ent(L, 0);
    int64_t total = 0;
    for (int32_t l = 0; l < L; ++l) {
        const int32_t nt = P.size[P.leaves[l]];
        for (int64_t q = P.near_ptr[l]; q < P.near_ptr[l + 1]; ++q) ent[l] += (int64_t)P.size[P.near_col[q]] * nt;
        total += ent[l];
    }
    int64_t cum = 0;
    P.leaf_half = 0;
    for (int32_t q = 0; q < lpx && 2 * cum < total; ++q) {
        for (int32_t x = 0; x < 8; ++x)
            if (x * lpx + q < L) cum += ent[P.leaf_order[x * lpx + q]];
        P.leaf_half = q + 1;
    }
}

}  // namespace

Plan *build_plan(const double *pts, int64_t n, const h2x_params &prm, std::string &err) {
    auto *P = new Plan();
    P->n = n;
    P->prm = prm;
    P->p = prm.cheb_order;
    P->k = prm.cheb_order * prm.cheb_order * prm.cheb_order;
    P->perm.resize(n);
    for (int64_t i = 0; i < n; ++i) P->perm[i] = i;

    // tight boxes while building; interpolation boxes derived afterwards
    std::vector<double> tlo, thi;
    const int64_t cap = 2 * n;
    P->first.reserve(cap);

    std::vector<Pending> stack;
    stack.push_back({0, n, -1, 0, 0});
    while (!stack.empty()) {
        Pending q = stack.back();
        stack.pop_back();
        const int32_t id = P->C++;
        P->first.push_back((int32_t)q.first);
        P->size.push_back((int32_t)q.size);
        P->parent.push_back(q.parent);
        P->son0.push_back(-1);
        P->son1.push_back(-1);
        P->depth.push_back(q.depth);
        if (q.parent >= 0) (q.which == 0 ? P->son0 : P->son1)[q.parent] = id;
        P->depth_max = std::max(P->depth_max, q.depth);

        double lo[3], hi[3];
        for (int d = 0; d < 3; ++d) lo[d] = hi[d] = pts[3 * P->perm[q.first] + d];
        for (int64_t i = q.first + 1; i < q.first + q.size; ++i)
            for (int d = 0; d < 3; ++d) {
                double v = pts[3 * P->perm[i] + d];
                lo[d] = std::min(lo[d], v);
                hi[d] = std::max(hi[d], v);
            }
        for (int d = 0; d < 3; ++d) { tlo.push_back(lo[d]); thi.push_back(hi[d]); }

        if (q.size <= prm.leaf_size) continue;
        int dim = 0;
        for (int d = 1; d < 3; ++d)
            if (hi[d] - lo[d] > hi[dim] - lo[dim]) dim = d;
        if (hi[dim] - lo[dim] == 0.0) continue;
        const double mid = 0.5 * (lo[dim] + hi[dim]);
        auto b = P->perm.begin() + q.first;
        auto cut = std::stable_partition(b, b + q.size, [&](int64_t g) { return pts[3 * g + dim] < mid; });
        const int64_t n0 = cut - b;
        if (n0 == 0 || n0 == q.size) continue;
        // second son pushed first so the first son's subtree is numbered next (pre-order)
        stack.push_back({q.first + n0, q.size - n0, id, q.depth + 1, 1});
        stack.push_back({q.first, n0, id, q.depth + 1, 0});
    }
    const int32_t C = P->C;

    // interpolation boxes: tight box, widened to 1e-10 where it is flatter than that
    const double tau = 1e-10;
    P->box.resize((size_t)C * 6);
    for (int32_t c = 0; c < C; ++c)
        for (int d = 0; d < 3; ++d) {
            double lo = tlo[3 * c + d], hi = thi[3 * c + d];
            if (hi - lo < tau) {
                double ctr = 0.5 * (lo + hi);
                lo = ctr - 0.5 * tau;
                hi = ctr + 0.5 * tau;
            }
            P->box[6 * c + d] = lo;
            P->box[6 * c + 3 + d] = hi;
        }

    P->pts_tree.resize((size_t)n * 3);
    for (int64_t i = 0; i < n; ++i)
        for (int d = 0; d < 3; ++d) P->pts_tree[3 * i + d] = pts[3 * P->perm[i] + d];

    P->leaf_index.assign(C, -1);
    for (int32_t c = 0; c < C; ++c)
        if (P->son0[c] < 0) {
            P->leaf_index[c] = (int32_t)P->leaves.size();
            P->leaves.push_back(c);
            P->max_leaf = std::max(P->max_leaf, P->size[c]);
        }

    // clusters by depth
    const int32_t D = P->depth_max + 1;
    P->lvl_ptr.assign(D + 1, 0);
    P->lvl_inner_ptr.assign(D + 1, 0);
    for (int32_t c = 0; c < C; ++c) {
        P->lvl_ptr[P->depth[c] + 1]++;
        if (P->son0[c] >= 0) P->lvl_inner_ptr[P->depth[c] + 1]++;
    }
    for (int32_t d = 0; d < D; ++d) {
        P->lvl_ptr[d + 1] += P->lvl_ptr[d];
        P->lvl_inner_ptr[d + 1] += P->lvl_inner_ptr[d];
    }
    P->lvl_all.resize(C);
    P->lvl_inner.resize(P->lvl_inner_ptr[D]);
    {
        std::vector<int32_t> fa(P->lvl_ptr.begin(), P->lvl_ptr.end() - 1);
        std::vector<int32_t> fi(P->lvl_inner_ptr.begin(), P->lvl_inner_ptr.end() - 1);
        for (int32_t c = 0; c < C; ++c) {
            P->lvl_all[fa[P->depth[c]]++] = c;
            if (P->son0[c] >= 0) P->lvl_inner[fi[P->depth[c]]++] = c;
        }
    }

    // block tree: depth-first with an explicit stack; children pushed in reverse
    // so leaves are emitted in pre-order
    std::vector<std::pair<int32_t, int32_t>> bstack;
    std::vector<std::pair<int32_t, int32_t>> adm, near;
    bstack.push_back({0, 0});
    auto tl = [&](int32_t c) { return &tlo[3 * c]; };
    auto th = [&](int32_t c) { return &thi[3 * c]; };
    while (!bstack.empty()) {
        auto [t, s] = bstack.back();
        bstack.pop_back();
        const double dist = box_dist(tl(t), th(t), tl(s), th(s));
        if (dist > 0.0) {
            const double dm = std::max(box_diam(tl(t), th(t)), box_diam(tl(s), th(s)));
            if (dm <= prm.eta * dist) { adm.push_back({t, s}); continue; }
        }
        const bool lt = P->son0[t] < 0, ls = P->son0[s] < 0;
        if (lt && ls) { near.push_back({t, s}); continue; }
        if (lt) {
            bstack.push_back({t, P->son1[s]});
            bstack.push_back({t, P->son0[s]});
        } else if (ls) {
            bstack.push_back({P->son1[t], s});
            bstack.push_back({P->son0[t], s});
        } else {
            bstack.push_back({P->son1[t], P->son1[s]});
            bstack.push_back({P->son1[t], P->son0[s]});
            bstack.push_back({P->son0[t], P->son1[s]});
            bstack.push_back({P->son0[t], P->son0[s]});
        }
    }

    // CSR by row cluster; a stable counting sort keeps block pre-order in a row
    P->adm_ptr.assign(C + 1, 0);
    for (auto &b : adm) P->adm_ptr[b.first + 1]++;
    for (int32_t c = 0; c < C; ++c) P->adm_ptr[c + 1] += P->adm_ptr[c];
    P->adm_col.resize(adm.size());
    {
        std::vector<int64_t> f(P->adm_ptr.begin(), P->adm_ptr.end() - 1);
        for (auto &b : adm) P->adm_col[f[b.first]++] = b.second;
    }
    const int32_t L = (int32_t)P->leaves.size();
    P->near_ptr.assign(L + 1, 0);
    for (auto &b : near) P->near_ptr[P->leaf_index[b.first] + 1]++;
    for (int32_t l = 0; l < L; ++l) P->near_ptr[l + 1] += P->near_ptr[l];
    P->near_col.resize(near.size());
    P->near_off.resize(near.size());
    {
        std::vector<int64_t> f(P->near_ptr.begin(), P->near_ptr.end() - 1);
        for (auto &b : near) P->near_col[f[P->leaf_index[b.first]]++] = b.second;
    }
    int64_t off = 0;
    for (int32_t l = 0; l < L; ++l) {
        const int32_t t = P->leaves[l];
        for (int64_t q = P->near_ptr[l]; q < P->near_ptr[l + 1]; ++q) {
            P->near_off[q] = off;
            off += (int64_t)P->size[t] * P->size[P->near_col[q]];
        }
    }
    P->near_entries = off;
    // column lists (stable: row order within a column)
    P->adm_cptr.assign(C + 1, 0);
    for (int32_t s = 0; s < (int32_t)P->adm_col.size(); ++s) P->adm_cptr[P->adm_col[s] + 1]++;
    for (int32_t c = 0; c < C; ++c) P->adm_cptr[c + 1] += P->adm_cptr[c];
    P->adm_cblk.resize(P->adm_col.size());
    {
        std::vector<int64_t> f(P->adm_cptr.begin(), P->adm_cptr.end() - 1);
        for (int64_t b = 0; b < (int64_t)P->adm_col.size(); ++b) P->adm_cblk[f[P->adm_col[b]]++] = b;
    }
    P->near_cptr.assign(L + 1, 0);
    for (size_t q = 0; q < near.size(); ++q) P->near_cptr[P->leaf_index[P->near_col[q]] + 1]++;
    for (int32_t l = 0; l < L; ++l) P->near_cptr[l + 1] += P->near_cptr[l];
    P->near_cblk.resize(near.size());
    {
        std::vector<int64_t> f(P->near_cptr.begin(), P->near_cptr.end() - 1);
        for (int64_t q = 0; q < (int64_t)near.size(); ++q) P->near_cblk[f[P->leaf_index[P->near_col[q]]]++] = q;
    }
    P->adm_depth = P->depth_max + 1;
    for (auto &b : adm) P->adm_depth = std::min(P->adm_depth, std::min(P->depth[b.first], P->depth[b.second]));
    P->near_off_t.resize(near.size());
    P->vt_off.resize(L);
    off = 0;
    int64_t voff = 0;
    for (int32_t l = 0; l < L; ++l) {
        const int32_t t = P->leaves[l];
        const int64_t nt2 = pad_rows(P->size[t]);
        P->vt_off[l] = voff;
        voff += (int64_t)P->k * nt2;
        int32_t rows = 0;
        for (int64_t q = P->near_ptr[l]; q < P->near_ptr[l + 1]; ++q) {
            P->near_off_t[q] = off;
            off += nt2 * P->size[P->near_col[q]];
            rows += P->size[P->near_col[q]];
        }
        P->max_near_rows = std::max(P->max_near_rows, rows);
    }
    P->near_entries_t = off;
    P->vt_entries = voff;

    coupling_order(*P);
    leaf_order(*P);
    P->sys_prm.assign(1, prm);
    P->sys_row = {0, n};
    P->sys_C = {0, (int64_t)C};
    P->sys_adm = {0, (int64_t)P->adm_col.size()};
    P->sys_near = {0, (int64_t)P->near_col.size()};
    (void)err;
    return P;
}

Plan *merge_plans(const std::vector<const Plan *> &parts, std::string &err) {
    if (parts.empty()) {
        err = "no plans to merge";
        return nullptr;
    }
    for (const Plan *q : parts)
        if (q->p != parts[0]->p) {
            err = "all merged plans must have the same Chebyshev order";
            return nullptr;
        }
    auto *P = new Plan();
    P->prm = parts[0]->prm;
    P->p = parts[0]->p;
    P->k = parts[0]->k;
    P->depth_max = 0;
    P->adm_depth = 1 << 30;
    for (const Plan *q : parts) {
        P->depth_max = std::max(P->depth_max, q->depth_max);
        P->adm_depth = std::min(P->adm_depth, q->adm_depth);
        P->max_leaf = std::max(P->max_leaf, q->max_leaf);
        P->max_near_rows = std::max(P->max_near_rows, q->max_near_rows);
    }
    P->sys_row.push_back(0);
    P->sys_C.push_back(0);
    P->sys_adm.push_back(0);
    P->sys_near.push_back(0);
    P->adm_ptr.push_back(0);
    P->near_ptr.push_back(0);
    P->adm_cptr.push_back(0);
    P->near_cptr.push_back(0);
    int64_t n0 = 0, c0 = 0, l0 = 0, a0 = 0, q0 = 0, e0 = 0, et0 = 0, v0 = 0;
    for (const Plan *q : parts) {
        const int32_t cs = (int32_t)c0;
        auto sh = [cs](int32_t c) { return c < 0 ? c : c + cs; };
        for (int64_t i = 0; i < q->n; ++i) P->perm.push_back(n0 + q->perm[i]);
        P->pts_tree.insert(P->pts_tree.end(), q->pts_tree.begin(), q->pts_tree.end());
        for (int32_t c = 0; c < q->C; ++c) {
            P->first.push_back((int32_t)(q->first[c] + n0));
            P->size.push_back(q->size[c]);
            P->parent.push_back(sh(q->parent[c]));
            P->son0.push_back(sh(q->son0[c]));
            P->son1.push_back(sh(q->son1[c]));
            P->depth.push_back(q->depth[c]);
            P->leaf_index.push_back(q->leaf_index[c] < 0 ? -1 : (int32_t)(q->leaf_index[c] + l0));
        }
        P->box.insert(P->box.end(), q->box.begin(), q->box.end());
        for (int32_t t : q->leaves) P->leaves.push_back(t + cs);
        for (int32_t c = 0; c < q->C; ++c) P->adm_ptr.push_back(q->adm_ptr[c + 1] + a0);
        for (int32_t s : q->adm_col) P->adm_col.push_back(s + cs);
        for (int32_t c = 0; c < q->C; ++c) P->adm_cptr.push_back(q->adm_cptr[c + 1] + a0);
        for (int64_t b : q->adm_cblk) P->adm_cblk.push_back(b + a0);
        const int32_t L = (int32_t)q->leaves.size();
        for (int32_t l = 0; l < L; ++l) {
            P->near_ptr.push_back(q->near_ptr[l + 1] + q0);
            P->near_cptr.push_back(q->near_cptr[l + 1] + q0);
            P->vt_off.push_back(q->vt_off[l] + v0);
        }
        for (size_t b = 0; b < q->near_col.size(); ++b) {
            P->near_col.push_back(q->near_col[b] + cs);
            P->near_off.push_back(q->near_off[b] + e0);
            P->near_off_t.push_back(q->near_off_t[b] + et0);
            P->near_cblk.push_back(q->near_cblk[b] + q0);
        }
        for (size_t i = 0; i < q->sys_prm.size(); ++i) {
            P->sys_prm.push_back(q->sys_prm[i]);
            P->sys_row.push_back(q->sys_row[i + 1] + n0);
            P->sys_C.push_back(q->sys_C[i + 1] + c0);
            P->sys_adm.push_back(q->sys_adm[i + 1] + a0);
            P->sys_near.push_back(q->sys_near[i + 1] + q0);
        }
        n0 += q->n;
        c0 += q->C;
        l0 += L;
        a0 += (int64_t)q->adm_col.size();
        q0 += (int64_t)q->near_col.size();
        e0 += q->near_entries;
        et0 += q->near_entries_t;
        v0 += q->vt_entries;
    }
    if (c0 >= (int64_t)1 << 31 || n0 >= (int64_t)1 << 31) {
        err = "merged plan too large";
        delete P;
        return nullptr;
    }
    P->n = n0;
    P->C = (int32_t)c0;
    P->near_entries = e0;
    P->near_entries_t = et0;
    P->vt_entries = v0;
    // per-level lists: level d of every system, systems in order
    const int32_t D = P->depth_max + 1;
    P->lvl_ptr.assign(D + 1, 0);
    P->lvl_inner_ptr.assign(D + 1, 0);
    for (int d = 0; d < D; ++d) {
        int64_t cc = 0;
        for (const Plan *q : parts) {
            if (d <= q->depth_max) {
                for (int32_t i = q->lvl_ptr[d]; i < q->lvl_ptr[d + 1]; ++i)
                    P->lvl_all.push_back(q->lvl_all[i] + (int32_t)cc);
                for (int32_t i = q->lvl_inner_ptr[d]; i < q->lvl_inner_ptr[d + 1]; ++i)
                    P->lvl_inner.push_back(q->lvl_inner[i] + (int32_t)cc);
            }
            cc += q->C;
        }
        P->lvl_ptr[d + 1] = (int32_t)P->lvl_all.size();
        P->lvl_inner_ptr[d + 1] = (int32_t)P->lvl_inner.size();
    }
    coupling_order(*P);
    leaf_order(*P);
    return P;
}

}  // namespace h2x
