// Host code under AddressSanitizer and UndefinedBehaviorSanitizer (built and run by
// tests/test_sanitize_host.py): the library's planner (cluster tree, block tree, lists,
// coupling and leaf launch orders, merged plans) and the oracle's products, solvers and
// gradients on small random problems.  Exit status 0 and no sanitizer report is a pass.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <random>
#include <string>
#include <vector>

#include "../paper_2509_17257_amd/csrc/plan.hpp"

namespace h2x {
void set_error(const std::string &) {}
}  // namespace h2x

extern "C" {
typedef struct orc_h2 orc_h2;
orc_h2 *orc_build(const double *pts, int64_t n, int kernel, double ell, double shift, double eta, int leaf, int p);
void orc_free(orc_h2 *h);
void orc_info(const orc_h2 *h, int64_t *info);
void orc_matmul(const orc_h2 *h, int64_t m, double alpha, const double *X, double beta, double *Y);
void orc_matmul_lowp(const orc_h2 *h, int prec, int64_t m, double alpha, const double *X, double beta, double *Y);
void orc_matmul_adjoint(const orc_h2 *h, int64_t m, double alpha, const double *X, double beta, double *Y);
void orc_grad(const orc_h2 *h, int64_t m, const double *X, const double *dY, double *dS, double *dN, double *dell);
int64_t orc_block_cg(const orc_h2 *h, int64_t m, const double *B, double *X, double rtol, int64_t max_iter,
                     int freeze_converged, int64_t *col_iters, int32_t *status);
int64_t orc_block_cg_shared(const orc_h2 *h, int64_t m, const double *B, double *X, double rtol, int64_t max_iter,
                            double drop, int64_t *rank_min, int32_t *status);
int64_t orc_refine_cg(const orc_h2 *h, int prec, int64_t m, const double *B, double *X, double rtol,
                      double inner_rtol, int64_t max_outer, int64_t max_inner, int64_t *inner_total,
                      double *col_relres, int32_t *status);
int64_t orc_block_cg_mixed(const orc_h2 *h, int prec, int64_t m, const double *B, double *X, double rtol,
                           double delta, int64_t max_iter, int64_t check, int64_t *replacements, double *col_relres,
                           int32_t *status);
int64_t orc_block_gmres(const orc_h2 *h, int64_t m, const double *B, double *X, double rtol, int64_t ell,
                        int64_t max_iter, int64_t *col_iters, int32_t *status, double *res_est, int64_t *cycles);
}

static int fails = 0;
#define CHECK(c)                                                           \
    do {                                                                   \
        if (!(c)) {                                                        \
            std::fprintf(stderr, "check failed line %d: %s\n", __LINE__, #c); \
            ++fails;                                                       \
        }                                                                  \
    } while (0)

int main() {
    std::mt19937_64 rng(12345);
    std::normal_distribution<double> nd;
    std::uniform_real_distribution<double> ud;
    std::vector<const h2x::Plan *> parts;
    struct Case {
        int64_t n;
        int leaf, p, sphere;
        double eta;
    } cases[] = {{700, 32, 3, 1, 1.0}, {900, 64, 4, 0, 1.0}, {300, 16, 2, 1, 1.5}, {1, 8, 3, 0, 1.0}, {64, 64, 4, 1, 1.0}};
    for (const Case &c : cases) {
        std::vector<double> pts(3 * c.n);
        for (int64_t i = 0; i < c.n; ++i) {
            double v[3], s = 0.0;
            for (double &x : v) {
                x = c.sphere ? nd(rng) : ud(rng);
                s += x * x;
            }
            for (int d = 0; d < 3; ++d) pts[3 * i + d] = c.sphere ? v[d] / std::sqrt(s) : v[d];
        }
        h2x_params prm{H2X_KERNEL_EXP, 0.5, 1.0, c.eta, c.leaf, c.p};
        std::string err;
        h2x::Plan *P = h2x::build_plan(pts.data(), c.n, prm, err);
        CHECK(P != nullptr);
        if (!P) continue;
        CHECK((int64_t)P->perm.size() == c.n && (int32_t)P->cpl_order.size() == P->C);
        CHECK(P->leaf_order.size() == P->leaves.size());
        parts.push_back(P);

        orc_h2 *o = orc_build(pts.data(), c.n, 0, 0.5, 1.0, c.eta, c.leaf, c.p);
        CHECK(o != nullptr);
        if (!o) continue;
        int64_t info[16] = {};
        orc_info(o, info);
        CHECK(info[1] == P->C && info[3] == (int64_t)P->adm_col.size() && info[4] == (int64_t)P->near_col.size());
        const int64_t m = 3, n = c.n, nm = n * m;
        std::vector<double> X(nm), Y(nm), B(nm), dY(nm), Z(nm, 0.0);
        for (double &x : X) x = nd(rng);
        for (double &x : dY) x = nd(rng);
        B = X;
        orc_matmul(o, m, 1.0, X.data(), 0.0, Y.data());
        orc_matmul_lowp(o, 2, m, 1.0, X.data(), 0.5, Y.data());
        orc_matmul_adjoint(o, m, 1.0, X.data(), 0.0, Y.data());
        std::vector<double> dS((size_t)info[3] * info[7] * info[7] + 1), dN((size_t)info[5] + 1);
        double dell = 0.0;
        orc_grad(o, m, X.data(), dY.data(), dS.data(), dN.data(), &dell);
        CHECK(std::isfinite(dell));
        std::vector<int64_t> ci(m);
        std::vector<int32_t> st(m);
        std::vector<double> rel(m), est(m);
        int32_t s1 = 0;
        int64_t r1 = 0, tot = 0, cyc = 0;
        Z.assign(nm, 0.0);
        orc_block_cg(o, m, B.data(), Z.data(), 1e-8, 500, 0, ci.data(), st.data());
        Z.assign(nm, 0.0);
        orc_block_cg_shared(o, m, B.data(), Z.data(), 1e-8, 500, 1e-6, &r1, st.data());
        Z.assign(nm, 0.0);
        orc_refine_cg(o, 1, m, B.data(), Z.data(), 1e-10, 1e-5, 6, 500, &tot, rel.data(), &s1);
        Z.assign(nm, 0.0);
        orc_block_cg_mixed(o, 2, m, B.data(), Z.data(), 1e-10, 0.1, 300, 4, &r1, rel.data(), &s1);
        Z.assign(nm, 0.0);
        orc_block_gmres(o, m, B.data(), Z.data(), 1e-8, 10, 200, ci.data(), st.data(), est.data(), &cyc);
        orc_free(o);
    }
    // the merged plan of the plans with one Chebyshev order (p = 3)
    std::vector<const h2x::Plan *> same;
    for (const h2x::Plan *P : parts)
        if (P->p == 3) same.push_back(P);
    std::string err;
    h2x::Plan *M = h2x::merge_plans(same, err);
    CHECK(M != nullptr);
    if (M) {
        CHECK(M->nsys() == (int32_t)same.size() && M->leaf_order.size() == M->leaves.size());
        delete M;
    }
    for (const h2x::Plan *P : parts) delete P;
    std::printf("sanitized host run: %d failed checks\n", fails);
    return fails ? 1 : 0;
}
