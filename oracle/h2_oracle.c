/*
 * Independent FP64 CPU oracle for the H^2-matrix x block-of-vectors product and
 * block CG ("On efficient block Krylov solvers for H^2-matrices", arXiv 2509.17257).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or call
 * this file; only the tests, the smoke check and the CPU-baseline leg of the
 * benchmark do.  It shares no code, header, table or helper with the HIP path.
 *
 * Plain and slow on purpose: recursion where the paper recurses, plain loops for
 * every small matrix product, FP64 everywhere (except the explicitly emulated
 * low-precision operator), OpenMP only where the paper itself runs "parfor".
 * Build: gcc -O2 -fopenmp -ffp-contract=off -shared -fPIC (see oracle/build.py).
 *
 * Readings of the paper where it is silent (each is also listed in the design
 * notes): binary bounding-box bisection at the box midpoint of the widest
 * dimension; leaf when |t| <= leaf size; tight boxes for diam/dist, equality is
 * admissible, dist 0 never is; first-kind Chebyshev tensor interpolation with
 * nu = jx + p*jy + p^2*jz; W == V (real symmetric kernel); the shift sits in the
 * diagonal near-field blocks; lists C_t are processed for every cluster t.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { ORC_KERNEL_EXP = 0, ORC_KERNEL_POLY = 1, ORC_KERNEL_CONST = 2, ORC_KERNEL_HELMHOLTZ = 3 };

typedef struct {
    /* problem (section 2: index set I = J, points as the supports Omega_i) */
    int64_t n;
    double *pts; /* n x 3, original order */
    int kernel;
    double ell, shift, eta;
    int leaf, p, k;

    /* cluster tree T_I (Definition "Cluster tree"), clusters numbered in pre-order */
    int64_t C;
    int64_t *first, *size, *son0, *son1, *parent, *depth;
    double *blo, *bhi;   /* tight bounding boxes, C x 3 */
    double *ilo, *ihi;   /* interpolation boxes, C x 3 */
    double *nodes;       /* Chebyshev tensor nodes, C x k x 3 */
    int64_t *perm;       /* tree position -> original index */

    /* leaves of the block tree T_{IxJ} (Definition "Block tree"), in pre-order */
    int64_t nb, bcap;
    int64_t *bt, *bs;
    int *badm;
    int64_t n_adm, n_near, near_entries;
    int64_t *boff;       /* offset of each leaf block's matrix in S (adm) or N (near) */

    /* lists C_t of prepare_addeval (Algorithm "prepare_addeval") */
    int64_t *list_ptr;   /* C + 1 */
    int64_t *list_blk;   /* nb, block ids grouped by row cluster, in block pre-order */

    /* H^2 representation */
    double *V;           /* n x k, leaf matrices, rows in tree order */
    double *E;           /* C x k x k, transfer matrices (root's entry unused) */
    double *S;           /* n_adm x k x k coupling matrices */
    double *N;           /* near_entries, near-field blocks row-major |t| x |s| */
    /* complex kernel (Helmholtz): imaginary parts of S and N; V and E stay real */
    int cplx;
    double *Si, *Ni;
} orc_h2;

/* ------------------------------------------------------------------------ */
/* kernel function g and its derivative in ell                               */

static double orc_dist3(const double *a, const double *b) {
    double dx = a[0] - b[0], dy = a[1] - b[1], dz = a[2] - b[2];
    return sqrt(dx * dx + dy * dy + dz * dz);
}

static double orc_g(const orc_h2 *h, const double *a, const double *b) {
    if (h->kernel == ORC_KERNEL_EXP) return exp(-orc_dist3(a, b) / h->ell);
    if (h->kernel == ORC_KERNEL_POLY) {
        double d = 1.0 + a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
        return d * d;
    }
    return 1.0;
}

/* Helmholtz single-layer kernel with equal quadrature weights (the unit sphere's area
 * 4 pi over n points): g(x, y) = (4 pi / n) exp(i kappa r) / (4 pi r) = exp(i kappa r) / (n r),
 * kappa held in ell; coinciding points (the self-interaction) contribute 0 (the shift is
 * added on the diagonal) */
static void orc_gc(const orc_h2 *h, const double *a, const double *b, double *re, double *im) {
    const double r = orc_dist3(a, b);
    if (r == 0.0) {
        *re = *im = 0.0;
        return;
    }
    const double f = 1.0 / ((double)h->n * r);
    *re = cos(h->ell * r) * f;
    *im = sin(h->ell * r) * f;
}

/* d g / d ell for the exponential kernel: (r / ell^2) exp(-r / ell); 0 otherwise */
static double orc_dg(const orc_h2 *h, const double *a, const double *b) {
    if (h->kernel != ORC_KERNEL_EXP) return 0.0;
    double r = orc_dist3(a, b);
    return (r / (h->ell * h->ell)) * exp(-r / h->ell);
}

/* ------------------------------------------------------------------------ */
/* cluster tree: recursive binary bisection                                  */

static void orc_tight_box(orc_h2 *h, int64_t c) {
    for (int d = 0; d < 3; ++d) {
        double lo = h->pts[3 * h->perm[h->first[c]] + d], hi = lo;
        for (int64_t i = 1; i < h->size[c]; ++i) {
            double v = h->pts[3 * h->perm[h->first[c] + i] + d];
            if (v < lo) lo = v;
            if (v > hi) hi = v;
        }
        h->blo[3 * c + d] = lo;
        h->bhi[3 * c + d] = hi;
    }
}

static int64_t orc_build_cluster(orc_h2 *h, int64_t first, int64_t size, int64_t parent,
                                 int64_t depth, int64_t *tmp) {
    int64_t c = h->C++;
    h->first[c] = first;
    h->size[c] = size;
    h->parent[c] = parent;
    h->depth[c] = depth;
    h->son0[c] = h->son1[c] = -1;
    orc_tight_box(h, c);
    if (size <= h->leaf) return c;
    int dstar = 0;
    double ext = h->bhi[3 * c] - h->blo[3 * c];
    for (int d = 1; d < 3; ++d) {
        double e = h->bhi[3 * c + d] - h->blo[3 * c + d];
        if (e > ext) { ext = e; dstar = d; }
    }
    if (ext == 0.0) return c; /* all points coincide */
    double mid = 0.5 * (h->blo[3 * c + dstar] + h->bhi[3 * c + dstar]);
    /* stable partition: points strictly below mid first, then the rest */
    int64_t n0 = 0, n1 = 0;
    for (int64_t i = 0; i < size; ++i) {
        int64_t g = h->perm[first + i];
        if (h->pts[3 * g + dstar] < mid) h->perm[first + n0++] = g;
        else tmp[n1++] = g;
    }
    for (int64_t i = 0; i < n1; ++i) h->perm[first + n0 + i] = tmp[i];
    if (n0 == 0 || n1 == 0) return c; /* degenerate split: keep as leaf */
    h->son0[c] = orc_build_cluster(h, first, n0, c, depth + 1, tmp);
    h->son1[c] = orc_build_cluster(h, first + n0, n1, c, depth + 1, tmp);
    return c;
}

/* ------------------------------------------------------------------------ */
/* block tree with the standard admissibility condition                       */

static double orc_diam(const orc_h2 *h, int64_t c) {
    double s = 0.0;
    for (int d = 0; d < 3; ++d) {
        double e = h->bhi[3 * c + d] - h->blo[3 * c + d];
        s += e * e;
    }
    return sqrt(s);
}

static double orc_dist(const orc_h2 *h, int64_t t, int64_t s) {
    double acc = 0.0;
    for (int d = 0; d < 3; ++d) {
        double g = 0.0;
        double a = h->blo[3 * s + d] - h->bhi[3 * t + d];
        double b = h->blo[3 * t + d] - h->bhi[3 * s + d];
        if (a > g) g = a;
        if (b > g) g = b;
        acc += g * g;
    }
    return sqrt(acc);
}

static int orc_admissible(const orc_h2 *h, int64_t t, int64_t s) {
    double dist = orc_dist(h, t, s);
    if (!(dist > 0.0)) return 0;
    double dt = orc_diam(h, t), ds = orc_diam(h, s);
    double dm = dt > ds ? dt : ds;
    return dm <= h->eta * dist;
}

static void orc_add_block(orc_h2 *h, int64_t t, int64_t s, int adm) {
    if (h->nb == h->bcap) {
        h->bcap = h->bcap ? 2 * h->bcap : 1024;
        h->bt = realloc(h->bt, sizeof(int64_t) * h->bcap);
        h->bs = realloc(h->bs, sizeof(int64_t) * h->bcap);
        h->badm = realloc(h->badm, sizeof(int) * h->bcap);
    }
    h->bt[h->nb] = t;
    h->bs[h->nb] = s;
    h->badm[h->nb] = adm;
    h->nb++;
}

static int orc_is_leaf(const orc_h2 *h, int64_t c) { return h->son0[c] < 0; }

static void orc_build_blocks(orc_h2 *h, int64_t t, int64_t s) {
    if (orc_admissible(h, t, s)) { orc_add_block(h, t, s, 1); return; }
    int lt = orc_is_leaf(h, t), ls = orc_is_leaf(h, s);
    if (lt && ls) { orc_add_block(h, t, s, 0); return; }
    if (lt) {
        orc_build_blocks(h, t, h->son0[s]);
        orc_build_blocks(h, t, h->son1[s]);
    } else if (ls) {
        orc_build_blocks(h, h->son0[t], s);
        orc_build_blocks(h, h->son1[t], s);
    } else {
        orc_build_blocks(h, h->son0[t], h->son0[s]);
        orc_build_blocks(h, h->son0[t], h->son1[s]);
        orc_build_blocks(h, h->son1[t], h->son0[s]);
        orc_build_blocks(h, h->son1[t], h->son1[s]);
    }
}

/* ------------------------------------------------------------------------ */
/* Chebyshev interpolation: nodes, Lagrange polynomials, V, E, S, N           */

#define ORC_TAU 1e-10

static void orc_interp_boxes_and_nodes(orc_h2 *h) {
    const int p = h->p, k = h->k;
    const double pi = acos(-1.0);
    for (int64_t c = 0; c < h->C; ++c) {
        double nd[3][16];
        for (int d = 0; d < 3; ++d) {
            double lo = h->blo[3 * c + d], hi = h->bhi[3 * c + d];
            if (hi - lo < ORC_TAU) {
                double ctr = 0.5 * (lo + hi);
                lo = ctr - 0.5 * ORC_TAU;
                hi = ctr + 0.5 * ORC_TAU;
            }
            h->ilo[3 * c + d] = lo;
            h->ihi[3 * c + d] = hi;
            double ctr = 0.5 * (lo + hi), half = 0.5 * (hi - lo);
            for (int j = 0; j < p; ++j) nd[d][j] = ctr + half * cos((2.0 * j + 1.0) * pi / (2.0 * p));
        }
        for (int jz = 0; jz < p; ++jz)
            for (int jy = 0; jy < p; ++jy)
                for (int jx = 0; jx < p; ++jx) {
                    int nu = jx + p * jy + p * p * jz;
                    double *o = &h->nodes[((size_t)c * k + nu) * 3];
                    o[0] = nd[0][jx];
                    o[1] = nd[1][jy];
                    o[2] = nd[2][jz];
                }
    }
}

/* one-dimensional Chebyshev node j of cluster c in dimension d */
static double orc_node1(const orc_h2 *h, int64_t c, int d, int j) {
    int p = h->p;
    int nu = (d == 0) ? j : (d == 1 ? p * j : p * p * j);
    return h->nodes[((size_t)c * h->k + nu) * 3 + d];
}

/* L_{c,j}(x) in dimension d: prod_{i != j} (x - xi_i) / (xi_j - xi_i) */
static double orc_lagrange(const orc_h2 *h, int64_t c, int d, int j, double x) {
    double v = 1.0, xj = orc_node1(h, c, d, j);
    for (int i = 0; i < h->p; ++i) {
        if (i == j) continue;
        double xi = orc_node1(h, c, d, i);
        v *= (x - xi) / (xj - xi);
    }
    return v;
}

/* tensor Lagrange polynomial nu of cluster c at the point x */
static double orc_lagrange3(const orc_h2 *h, int64_t c, int nu, const double *x) {
    int p = h->p;
    int jx = nu % p, jy = (nu / p) % p, jz = nu / (p * p);
    return orc_lagrange(h, c, 0, jx, x[0]) * orc_lagrange(h, c, 1, jy, x[1]) *
           orc_lagrange(h, c, 2, jz, x[2]);
}

static void orc_fill_matrices(orc_h2 *h) {
    const int k = h->k;
    /* leaf matrices V_t[i, nu] = L_{t,nu}(x_i) */
    for (int64_t c = 0; c < h->C; ++c) {
        if (!orc_is_leaf(h, c)) continue;
        for (int64_t i = 0; i < h->size[c]; ++i) {
            int64_t row = h->first[c] + i;
            const double *x = &h->pts[3 * h->perm[row]];
            for (int nu = 0; nu < k; ++nu) h->V[row * k + nu] = orc_lagrange3(h, c, nu, x);
        }
    }
    /* transfer matrices E_{t'}[nu', nu] = L_{t,nu}(xi_{t',nu'}) for t' in sons(t) */
    for (int64_t c = 0; c < h->C; ++c) {
        int64_t par = h->parent[c];
        if (par < 0) continue;
        for (int a = 0; a < k; ++a) {
            const double *xi = &h->nodes[((size_t)c * k + a) * 3];
            for (int nu = 0; nu < k; ++nu) h->E[((size_t)c * k + a) * k + nu] = orc_lagrange3(h, par, nu, xi);
        }
    }
    /* coupling and near-field blocks */
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t b = 0; b < h->nb; ++b) {
        int64_t t = h->bt[b], s = h->bs[b];
        if (h->badm[b] && h->cplx) {
            double *Sb = &h->S[h->boff[b]], *Sib = &h->Si[h->boff[b]];
            for (int nu = 0; nu < k; ++nu)
                for (int mu = 0; mu < k; ++mu)
                    orc_gc(h, &h->nodes[((size_t)t * k + nu) * 3], &h->nodes[((size_t)s * k + mu) * 3],
                           &Sb[nu * k + mu], &Sib[nu * k + mu]);
        } else if (h->badm[b]) {
            double *Sb = &h->S[h->boff[b]];
            for (int nu = 0; nu < k; ++nu)
                for (int mu = 0; mu < k; ++mu)
                    Sb[nu * k + mu] = orc_g(h, &h->nodes[((size_t)t * k + nu) * 3], &h->nodes[((size_t)s * k + mu) * 3]);
        } else if (h->cplx) {
            double *Nb = &h->N[h->boff[b]], *Nib = &h->Ni[h->boff[b]];
            for (int64_t i = 0; i < h->size[t]; ++i)
                for (int64_t j = 0; j < h->size[s]; ++j) {
                    int64_t gi = h->perm[h->first[t] + i], gj = h->perm[h->first[s] + j];
                    double re, im;
                    orc_gc(h, &h->pts[3 * gi], &h->pts[3 * gj], &re, &im);
                    if (gi == gj) re += h->shift;
                    Nb[i * h->size[s] + j] = re;
                    Nib[i * h->size[s] + j] = im;
                }
        } else {
            double *Nb = &h->N[h->boff[b]];
            for (int64_t i = 0; i < h->size[t]; ++i)
                for (int64_t j = 0; j < h->size[s]; ++j) {
                    int64_t gi = h->perm[h->first[t] + i], gj = h->perm[h->first[s] + j];
                    double v = orc_g(h, &h->pts[3 * gi], &h->pts[3 * gj]);
                    if (gi == gj) v += h->shift;
                    Nb[i * h->size[s] + j] = v;
                }
        }
    }
}

/* ------------------------------------------------------------------------ */
/* construction                                                             */

orc_h2 *orc_build(const double *pts, int64_t n, int kernel, double ell, double shift, double eta,
                  int leaf, int p) {
    if (n <= 0 || p < 1 || p > 16 || leaf < 1) return NULL;
    orc_h2 *h = calloc(1, sizeof(orc_h2));
    h->n = n;
    h->kernel = kernel;
    h->ell = ell;
    h->shift = shift;
    h->eta = eta;
    h->leaf = leaf;
    h->p = p;
    h->k = p * p * p;
    h->pts = malloc(sizeof(double) * 3 * n);
    memcpy(h->pts, pts, sizeof(double) * 3 * n);
    int64_t cap = 2 * n;
    h->first = malloc(sizeof(int64_t) * cap);
    h->size = malloc(sizeof(int64_t) * cap);
    h->son0 = malloc(sizeof(int64_t) * cap);
    h->son1 = malloc(sizeof(int64_t) * cap);
    h->parent = malloc(sizeof(int64_t) * cap);
    h->depth = malloc(sizeof(int64_t) * cap);
    h->blo = malloc(sizeof(double) * 3 * cap);
    h->bhi = malloc(sizeof(double) * 3 * cap);
    h->perm = malloc(sizeof(int64_t) * n);
    for (int64_t i = 0; i < n; ++i) h->perm[i] = i;
    int64_t *tmp = malloc(sizeof(int64_t) * n);
    orc_build_cluster(h, 0, n, -1, 0, tmp);
    free(tmp);

    orc_build_blocks(h, 0, 0);

    /* matrix offsets of the leaf blocks */
    h->boff = malloc(sizeof(int64_t) * (h->nb ? h->nb : 1));
    int64_t so = 0, no = 0;
    for (int64_t b = 0; b < h->nb; ++b) {
        if (h->badm[b]) { h->boff[b] = so; so += (int64_t)h->k * h->k; h->n_adm++; }
        else { h->boff[b] = no; no += h->size[h->bt[b]] * h->size[h->bs[b]]; h->n_near++; }
    }
    h->near_entries = no;

    /* prepare_addeval: each leaf block goes to the list of its row cluster */
    h->list_ptr = calloc(h->C + 1, sizeof(int64_t));
    h->list_blk = malloc(sizeof(int64_t) * (h->nb ? h->nb : 1));
    for (int64_t b = 0; b < h->nb; ++b) h->list_ptr[h->bt[b] + 1]++;
    for (int64_t c = 0; c < h->C; ++c) h->list_ptr[c + 1] += h->list_ptr[c];
    int64_t *fill = calloc((size_t)h->C + 1, sizeof(int64_t));
    for (int64_t b = 0; b < h->nb; ++b) {
        int64_t t = h->bt[b];
        h->list_blk[h->list_ptr[t] + fill[t]++] = b;
    }
    free(fill);

    h->ilo = malloc(sizeof(double) * 3 * h->C);
    h->ihi = malloc(sizeof(double) * 3 * h->C);
    h->nodes = malloc(sizeof(double) * 3 * h->C * h->k);
    orc_interp_boxes_and_nodes(h);

    h->V = malloc(sizeof(double) * n * h->k);
    h->E = calloc((size_t)h->C * h->k * h->k, sizeof(double));
    h->S = malloc(sizeof(double) * (so ? so : 1));
    h->N = malloc(sizeof(double) * (no ? no : 1));
    h->cplx = h->kernel == ORC_KERNEL_HELMHOLTZ;
    h->Si = h->cplx ? malloc(sizeof(double) * (so ? so : 1)) : NULL;
    h->Ni = h->cplx ? malloc(sizeof(double) * (no ? no : 1)) : NULL;
    orc_fill_matrices(h);
    return h;
}

void orc_free(orc_h2 *h) {
    if (!h) return;
    free(h->pts); free(h->first); free(h->size); free(h->son0); free(h->son1);
    free(h->parent); free(h->depth); free(h->blo); free(h->bhi); free(h->ilo); free(h->ihi);
    free(h->nodes); free(h->perm); free(h->bt); free(h->bs); free(h->badm); free(h->boff);
    free(h->list_ptr); free(h->list_blk); free(h->V); free(h->E); free(h->S); free(h->N);
    free(h->Si); free(h->Ni);
    free(h);
}

/* info[0..9] = n, C, leaves, n_adm, n_near, near_entries, max depth, k, p, n blocks */
void orc_info(const orc_h2 *h, int64_t *info) {
    int64_t leaves = 0, dmax = 0;
    for (int64_t c = 0; c < h->C; ++c) {
        if (orc_is_leaf(h, c)) leaves++;
        if (h->depth[c] > dmax) dmax = h->depth[c];
    }
    info[0] = h->n; info[1] = h->C; info[2] = leaves; info[3] = h->n_adm; info[4] = h->n_near;
    info[5] = h->near_entries; info[6] = dmax; info[7] = h->k; info[8] = h->p; info[9] = h->nb;
}

void orc_get_tree(const orc_h2 *h, int64_t *perm, int64_t *first, int64_t *size, int64_t *son0,
                  int64_t *son1, int64_t *parent, int64_t *depth, double *blo, double *bhi,
                  double *ilo, double *ihi) {
    memcpy(perm, h->perm, sizeof(int64_t) * h->n);
    memcpy(first, h->first, sizeof(int64_t) * h->C);
    memcpy(size, h->size, sizeof(int64_t) * h->C);
    memcpy(son0, h->son0, sizeof(int64_t) * h->C);
    memcpy(son1, h->son1, sizeof(int64_t) * h->C);
    memcpy(parent, h->parent, sizeof(int64_t) * h->C);
    memcpy(depth, h->depth, sizeof(int64_t) * h->C);
    memcpy(blo, h->blo, sizeof(double) * 3 * h->C);
    memcpy(bhi, h->bhi, sizeof(double) * 3 * h->C);
    memcpy(ilo, h->ilo, sizeof(double) * 3 * h->C);
    memcpy(ihi, h->ihi, sizeof(double) * 3 * h->C);
}

void orc_get_blocks(const orc_h2 *h, int64_t *bt, int64_t *bs, int32_t *badm, int64_t *boff) {
    for (int64_t b = 0; b < h->nb; ++b) {
        bt[b] = h->bt[b]; bs[b] = h->bs[b]; badm[b] = h->badm[b]; boff[b] = h->boff[b];
    }
}

void orc_get_lists(const orc_h2 *h, int64_t *list_ptr, int64_t *list_blk) {
    memcpy(list_ptr, h->list_ptr, sizeof(int64_t) * (h->C + 1));
    memcpy(list_blk, h->list_blk, sizeof(int64_t) * h->nb);
}

void orc_get_nodes(const orc_h2 *h, double *nodes) { memcpy(nodes, h->nodes, sizeof(double) * 3 * h->C * h->k); }
void orc_get_V(const orc_h2 *h, double *V) { memcpy(V, h->V, sizeof(double) * h->n * h->k); }
void orc_get_E(const orc_h2 *h, double *E) { memcpy(E, h->E, sizeof(double) * h->C * h->k * h->k); }
void orc_get_S(const orc_h2 *h, double *S) { memcpy(S, h->S, sizeof(double) * h->n_adm * h->k * h->k); }
void orc_get_N(const orc_h2 *h, double *N) { memcpy(N, h->N, sizeof(double) * h->near_entries); }

/* Direct Lagrange evaluation of the basis of ANY cluster c (leaf or not) at the
 * points of c, in tree order: out is |c| x k.  Used to pin nestedness. */
void orc_basis_direct(const orc_h2 *h, int64_t c, double *out) {
    for (int64_t i = 0; i < h->size[c]; ++i) {
        const double *x = &h->pts[3 * h->perm[h->first[c] + i]];
        for (int nu = 0; nu < h->k; ++nu) out[i * h->k + nu] = orc_lagrange3(h, c, nu, x);
    }
}

/* Replace the stored matrices (used by tests that perturb S or inject a mistake). */
void orc_set_S(orc_h2 *h, const double *S) { memcpy(h->S, S, sizeof(double) * h->n_adm * h->k * h->k); }
void orc_set_N(orc_h2 *h, const double *N) { memcpy(h->N, N, sizeof(double) * h->near_entries); }
void orc_set_E(orc_h2 *h, const double *E) { memcpy(h->E, E, sizeof(double) * h->C * h->k * h->k); }

/* Re-evaluate S and N for a new length scale ell (same tree and bases). */
void orc_set_ell(orc_h2 *h, double ell) {
    h->ell = ell;
    orc_fill_matrices(h);
}

/* ------------------------------------------------------------------------ */
/* H^2 x X: forward transformation, list-wise multiplication phase, backward  */
/* X, Y are n x m row-major in ORIGINAL point order.                          */

typedef struct {
    const orc_h2 *h;
    int64_t m;
    const double *X;
    double *xh, *yh; /* C x k x m */
} orc_mm;

/* Forward: leaf x_s = W_s^* x|_s ; inner x_s = sum_{s' in sons} E_{s'}^* x_{s'} */
static void orc_forward(orc_mm *w, int64_t s) {
    const orc_h2 *h = w->h;
    const int k = h->k;
    const int64_t m = w->m;
    double *xs = &w->xh[(size_t)s * k * m];
    if (orc_is_leaf(h, s)) {
        for (int nu = 0; nu < k; ++nu)
            for (int64_t j = 0; j < m; ++j) {
                double acc = 0.0;
                for (int64_t i = 0; i < h->size[s]; ++i) {
                    int64_t row = h->first[s] + i;
                    acc += h->V[row * k + nu] * w->X[h->perm[row] * m + j];
                }
                xs[nu * m + j] = acc;
            }
        return;
    }
    int64_t sons[2] = {h->son0[s], h->son1[s]};
    /* sons in parallel (P_Forward), then the parent sums sequentially */
    for (int q = 0; q < 2; ++q) orc_forward(w, sons[q]);
    for (int q = 0; q < 2; ++q) {
        const double *E = &h->E[(size_t)sons[q] * k * k];
        const double *xq = &w->xh[(size_t)sons[q] * k * m];
        for (int nu = 0; nu < k; ++nu)
            for (int64_t j = 0; j < m; ++j) {
                double acc = 0.0;
                for (int a = 0; a < k; ++a) acc += E[a * k + nu] * xq[a * m + j];
                xs[nu * m + j] += acc;
            }
    }
}

/* Backward: inner y_{t'} += E_{t'} y_t then recurse ; leaf y|_t += V_t y_t */
static void orc_backward(const orc_mm *w, int64_t t, double *Y) {
    const orc_h2 *h = w->h;
    const int k = h->k;
    const int64_t m = w->m;
    double *yt = &w->yh[(size_t)t * k * m];
    if (orc_is_leaf(h, t)) {
        for (int64_t i = 0; i < h->size[t]; ++i) {
            int64_t row = h->first[t] + i;
            double *yrow = &Y[h->perm[row] * m];
            for (int64_t j = 0; j < m; ++j) {
                double acc = 0.0;
                for (int nu = 0; nu < k; ++nu) acc += h->V[row * k + nu] * yt[nu * m + j];
                yrow[j] += acc;
            }
        }
        return;
    }
    int64_t sons[2] = {h->son0[t], h->son1[t]};
    for (int q = 0; q < 2; ++q) {
        const double *E = &h->E[(size_t)sons[q] * k * k];
        double *yq = &w->yh[(size_t)sons[q] * k * m];
        for (int a = 0; a < k; ++a)
            for (int64_t j = 0; j < m; ++j) {
                double acc = 0.0;
                for (int nu = 0; nu < k; ++nu) acc += E[a * k + nu] * yt[nu * m + j];
                yq[a * m + j] += acc;
            }
        orc_backward(w, sons[q], Y);
    }
}

/* Complex kernel: column pairs (2j, 2j + 1) of X, x-hat, y-hat and Y hold the real and
 * imaginary part of complex column j; S_b = S + i Si and N_b = N + i Ni are complex, the
 * bases real.  One leaf block of list_addeval in complex arithmetic. */
static void orc_block_addeval_c(const orc_mm *w, int64_t t, int64_t b, double alpha, double *Y) {
    const orc_h2 *h = w->h;
    const int k = h->k;
    const int64_t m = w->m, mc = m / 2, s = h->bs[b];
    if (h->badm[b]) {
        const double *Sr = &h->S[h->boff[b]], *Si = &h->Si[h->boff[b]];
        const double *xs = &w->xh[(size_t)s * k * m];
        double *yt = &w->yh[(size_t)t * k * m];
        for (int nu = 0; nu < k; ++nu)
            for (int64_t j = 0; j < mc; ++j) {
                double complex acc = 0.0;
                for (int mu = 0; mu < k; ++mu)
                    acc += (Sr[nu * k + mu] + I * Si[nu * k + mu]) * (xs[mu * m + 2 * j] + I * xs[mu * m + 2 * j + 1]);
                yt[nu * m + 2 * j] += alpha * creal(acc);
                yt[nu * m + 2 * j + 1] += alpha * cimag(acc);
            }
    } else {
        const double *Nr = &h->N[h->boff[b]], *Ni = &h->Ni[h->boff[b]];
        const int64_t ns = h->size[s];
        for (int64_t i = 0; i < h->size[t]; ++i) {
            double *yrow = &Y[h->perm[h->first[t] + i] * m];
            for (int64_t j = 0; j < mc; ++j) {
                double complex acc = 0.0;
                for (int64_t c = 0; c < ns; ++c) {
                    const double *x = &w->X[h->perm[h->first[s] + c] * m + 2 * j];
                    acc += (Nr[i * ns + c] + I * Ni[i * ns + c]) * (x[0] + I * x[1]);
                }
                yrow[2 * j] += alpha * creal(acc);
                yrow[2 * j + 1] += alpha * cimag(acc);
            }
        }
    }
}

/* list_addeval for one row cluster t: admissible -> y_t += alpha S_b x_s,
 * inadmissible -> y|_t += alpha G|_{t x s} x|_s.  Owns y_t and the rows of t. */
static void orc_list_addeval(const orc_mm *w, int64_t t, double alpha, double *Y) {
    const orc_h2 *h = w->h;
    const int k = h->k;
    const int64_t m = w->m;
    for (int64_t q = h->list_ptr[t]; q < h->list_ptr[t + 1]; ++q) {
        int64_t b = h->list_blk[q], s = h->bs[b];
        if (h->cplx) {
            orc_block_addeval_c(w, t, b, alpha, Y);
            continue;
        }
        if (h->badm[b]) {
            const double *Sb = &h->S[h->boff[b]];
            const double *xs = &w->xh[(size_t)s * k * m];
            double *yt = &w->yh[(size_t)t * k * m];
            for (int nu = 0; nu < k; ++nu)
                for (int64_t j = 0; j < m; ++j) {
                    double acc = 0.0;
                    for (int mu = 0; mu < k; ++mu) acc += Sb[nu * k + mu] * xs[mu * m + j];
                    yt[nu * m + j] += alpha * acc;
                }
        } else {
            const double *Nb = &h->N[h->boff[b]];
            int64_t ns = h->size[s];
            for (int64_t i = 0; i < h->size[t]; ++i) {
                double *yrow = &Y[h->perm[h->first[t] + i] * m];
                for (int64_t j = 0; j < m; ++j) {
                    double acc = 0.0;
                    for (int64_t c = 0; c < ns; ++c) acc += Nb[i * ns + c] * w->X[h->perm[h->first[s] + c] * m + j];
                    yrow[j] += alpha * acc;
                }
            }
        }
    }
}

/* Y|_t += V_t y_t for the nested bases, top-down over the tree as index loops: clusters are
 * numbered in pre-order, so a parent comes before its sons and y_t is complete when its turn
 * comes (y_{t'} += E_{t'} y_t for the sons, then V_t y_t at the leaves).  Every entry receives
 * the same terms in the same order as in orc_backward's recursion. */
static void orc_backward_loops(const orc_mm *w, double *Y) {
    const orc_h2 *h = w->h;
    const int k = h->k;
    const int64_t m = w->m;
    for (int64_t t = 0; t < h->C; ++t) {
        if (orc_is_leaf(h, t)) continue;
        const double *yt = &w->yh[(size_t)t * k * m];
        int64_t sons[2] = {h->son0[t], h->son1[t]};
        for (int q = 0; q < 2; ++q) {
            const double *E = &h->E[(size_t)sons[q] * k * k];
            double *yq = &w->yh[(size_t)sons[q] * k * m];
            for (int a = 0; a < k; ++a)
                for (int64_t j = 0; j < m; ++j) {
                    double acc = 0.0;
                    for (int nu = 0; nu < k; ++nu) acc += E[a * k + nu] * yt[nu * m + j];
                    yq[a * m + j] += acc;
                }
        }
    }
    for (int64_t t = 0; t < h->C; ++t) {
        if (!orc_is_leaf(h, t)) continue;
        const double *yt = &w->yh[(size_t)t * k * m];
        for (int64_t i = 0; i < h->size[t]; ++i) {
            int64_t row = h->first[t] + i;
            double *yrow = &Y[h->perm[row] * m];
            for (int64_t j = 0; j < m; ++j) {
                double acc = 0.0;
                for (int nu = 0; nu < k; ++nu) acc += h->V[row * k + nu] * yt[nu * m + j];
                yrow[j] += acc;
            }
        }
    }
}

/* Y <- beta Y + alpha A_H2 X from the definition of the H^2 matrix (section 2):
 * A_H2 = sum over admissible leaves (t, s) of V_t S_ts V_s^T + sum over the inadmissible ones
 * of G|_{t x s}, with nested bases V_t|_{t'} = V_{t'} E_{t'}.  As index loops over the
 * pre-ordered clusters: x_s = V_s^T X|_s (leaves directly, inner clusters from their sons),
 * y_t = sum_s S_ts x_s and the near blocks for every cluster t, then Y|_t += V_t y_t pushed
 * down through the nested bases. */
void orc_matmul(const orc_h2 *h, int64_t m, double alpha, const double *X, double beta, double *Y) {
    orc_mm w;
    w.h = h;
    w.m = m;
    w.X = X;
    size_t cw = (size_t)h->C * h->k * m;
    w.xh = calloc(cw ? cw : 1, sizeof(double));
    w.yh = calloc(cw ? cw : 1, sizeof(double));
    for (int64_t i = 0; i < h->n * m; ++i) Y[i] = (beta == 0.0) ? 0.0 : beta * Y[i];

    /* x_s = V_s^T X|_s at the leaves (independent of each other) */
    {
        const int k = h->k;
#pragma omp parallel for schedule(dynamic, 4)
        for (int64_t s = 0; s < h->C; ++s) {
            if (!orc_is_leaf(h, s)) continue;
            double *xs = &w.xh[(size_t)s * k * m];
            for (int nu = 0; nu < k; ++nu)
                for (int64_t j = 0; j < m; ++j) {
                    double acc = 0.0;
                    for (int64_t i = 0; i < h->size[s]; ++i) {
                        int64_t row = h->first[s] + i;
                        acc += h->V[row * k + nu] * X[h->perm[row] * m + j];
                    }
                    xs[nu * m + j] = acc;
                }
        }
    }
    /* x_s = sum over sons s' of E_{s'}^T x_{s'} for inner clusters */
    {
        /* sons before parents: clusters are in pre-order, so iterate from the back */
        const int k = h->k;
        for (int64_t s = h->C - 1; s >= 0; --s) {
            if (orc_is_leaf(h, s)) continue;
            double *xs = &w.xh[(size_t)s * k * m];
            int64_t sons[2] = {h->son0[s], h->son1[s]};
            for (int q = 0; q < 2; ++q) {
                const double *E = &h->E[(size_t)sons[q] * k * k];
                const double *xq = &w.xh[(size_t)sons[q] * k * m];
                for (int nu = 0; nu < k; ++nu)
                    for (int64_t j = 0; j < m; ++j) {
                        double acc = 0.0;
                        for (int a = 0; a < k; ++a) acc += E[a * k + nu] * xq[a * m + j];
                        xs[nu * m + j] += acc;
                    }
            }
        }
    }
    /* y_t = sum over admissible (t, s) of S_ts x_s and Y|_t += G|_{t x s} X|_s for the
     * inadmissible ones: every cluster owns y_t and its rows, clusters in parallel */
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t t = 0; t < h->C; ++t) orc_list_addeval(&w, t, alpha, Y);
    /* Y|_t += V_t y_t through the nested bases */
    orc_backward_loops(&w, Y);
    free(w.xh);
    free(w.yh);
}

/* The same product with the forward and backward transformations as recursions over the
 * cluster tree (the paper's sequential form, section 3); orc_matmul must equal it bitwise. */
void orc_matmul_recursive(const orc_h2 *h, int64_t m, double alpha, const double *X, double beta, double *Y) {
    orc_mm w;
    w.h = h;
    w.m = m;
    w.X = X;
    size_t cw = (size_t)h->C * h->k * m;
    w.xh = calloc(cw ? cw : 1, sizeof(double));
    w.yh = calloc(cw ? cw : 1, sizeof(double));
    for (int64_t i = 0; i < h->n * m; ++i) Y[i] = (beta == 0.0) ? 0.0 : beta * Y[i];
    orc_forward(&w, 0);
    for (int64_t t = 0; t < h->C; ++t) orc_list_addeval(&w, t, alpha, Y);
    orc_backward(&w, 0, Y);
    free(w.xh);
    free(w.yh);
}

/* Forward transform only: xh (C x k x m) of X (n x m, original order). */
void orc_forward_transform(const orc_h2 *h, int64_t m, const double *X, double *xh) {
    orc_mm w;
    w.h = h;
    w.m = m;
    w.X = X;
    w.xh = xh;
    w.yh = NULL;
    memset(xh, 0, sizeof(double) * h->C * h->k * m);
    orc_forward(&w, 0);
}

/* ------------------------------------------------------------------------ */
/* Low-precision operator (emulated).  V, E, S are rounded to the storage type
 * (prec 1: FP32, 2: bfloat16), the near field to FP32; every small product
 * rounds its right-hand factor to the same type (X at the forward leaf
 * product, x-hat where it meets E and S, y-hat where it meets E and V; X to
 * FP32 where it meets the near field) and every sum is an FP32 sum.
 * bfloat16 rounding: the FP64 value is rounded to FP32 (nearest even), then
 * the FP32 value to bfloat16 (nearest even on the upper 16 bits).            */

static float orc_round_bf16(float f) {
    uint32_t u;
    memcpy(&u, &f, 4);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) { u |= 0x00400000u; }
    else u = u + 0x7fffu + ((u >> 16) & 1u);
    u &= 0xffff0000u;
    float r;
    memcpy(&r, &u, 4);
    return r;
}

/* exported for the rounding pin: bfloat16 rounding of FP32 values */
void orc_round_bf16_array(const float *in, float *out, int64_t count) {
    for (int64_t i = 0; i < count; ++i) out[i] = orc_round_bf16(in[i]);
}

/* round an FP64 value to the storage type, returned as FP32 */
static float orc_q(int prec, double v) {
    float f = (float)v;
    return prec == 2 ? orc_round_bf16(f) : f;
}

/* Rounding points of the emulation that a test can switch off one at a time
 * (planted slips, to show that the hand-worked golden product catches each):
 * bit 0  X not rounded to the storage type at the forward leaf product
 * bit 1  x-hat of a son not rounded where it meets E (forward transfer)
 * bit 2  x-hat not rounded where it meets S (coupling)
 * bit 3  y-hat of a parent not rounded where it meets E (backward transfer)
 * bit 4  y-hat not rounded where it meets V (leaf basis term)
 * bit 5  X rounded to the storage type (not to FP32) where it meets the near field
 * bit 6  sums carried in FP64 instead of FP32
 * The library's arithmetic is omit = 0. */
#define ORC_OMIT_X_LEAF 1
#define ORC_OMIT_XH_TRANSFER 2
#define ORC_OMIT_XH_COUPLING 4
#define ORC_OMIT_YH_TRANSFER 8
#define ORC_OMIT_YH_LEAF 16
#define ORC_ROUND_X_NEAR 32
#define ORC_FP64_SUMS 64

/* a right-hand factor: rounded to the storage type unless that rounding point is omitted */
static double orc_rh(int prec, int omit, int bit, double v) { return (omit & bit) ? v : (double)orc_q(prec, v); }

/* one FP32 product or sum (FP64 when the planted slip asks for it); through FP64 this is
 * exactly the FP32 operation, since FP64 carries more than twice FP32's precision */
static double orc_f32(int omit, double v) { return (omit & ORC_FP64_SUMS) ? v : (double)(float)v; }

static void orc_matmul_lowp_omit(const orc_h2 *h, int prec, int64_t m, double alpha, const double *X, double beta,
                                 double *Y, int omit) {
    const int k = h->k;
    const int64_t n = h->n;
    size_t cw = (size_t)h->C * k * m;
    double *xh = calloc(cw ? cw : 1, sizeof(double)), *yh = calloc(cw ? cw : 1, sizeof(double));
    for (int64_t i = 0; i < n * m; ++i) Y[i] = (beta == 0.0) ? 0.0 : beta * Y[i];
#define LP_TERM(a, b) orc_f32(omit, (a) * (b))
    /* forward: leaves, then transfers bottom-up */
    for (int64_t s = 0; s < h->C; ++s) {
        if (!orc_is_leaf(h, s)) continue;
        for (int nu = 0; nu < k; ++nu)
            for (int64_t j = 0; j < m; ++j) {
                double a = 0.0;
                for (int64_t i = 0; i < h->size[s]; ++i) {
                    int64_t row = h->first[s] + i;
                    a = orc_f32(omit, a + LP_TERM((double)orc_q(prec, h->V[row * k + nu]),
                                                  orc_rh(prec, omit, ORC_OMIT_X_LEAF, (double)(float)X[h->perm[row] * m + j])));
                }
                xh[((size_t)s * k + nu) * m + j] = a;
            }
    }
    for (int64_t s = h->C - 1; s >= 0; --s) {
        if (orc_is_leaf(h, s)) continue;
        int64_t sons[2] = {h->son0[s], h->son1[s]};
        for (int nu = 0; nu < k; ++nu)
            for (int64_t j = 0; j < m; ++j) {
                double a = 0.0;
                for (int q = 0; q < 2; ++q) {
                    const double *E = &h->E[(size_t)sons[q] * k * k];
                    for (int b = 0; b < k; ++b)
                        a = orc_f32(omit, a + LP_TERM((double)orc_q(prec, E[b * k + nu]),
                                                      orc_rh(prec, omit, ORC_OMIT_XH_TRANSFER,
                                                             xh[((size_t)sons[q] * k + b) * m + j])));
                }
                xh[((size_t)s * k + nu) * m + j] = a;
            }
    }
    /* multiplication phase, every cluster's list */
    for (int64_t t = 0; t < h->C; ++t)
        for (int nu = 0; nu < k; ++nu)
            for (int64_t j = 0; j < m; ++j) {
                double a = 0.0;
                for (int64_t q = h->list_ptr[t]; q < h->list_ptr[t + 1]; ++q) {
                    int64_t b = h->list_blk[q], s = h->bs[b];
                    if (!h->badm[b]) continue;
                    const double *Sb = &h->S[h->boff[b]];
                    for (int mu = 0; mu < k; ++mu)
                        a = orc_f32(omit, a + LP_TERM((double)orc_q(prec, Sb[nu * k + mu]),
                                                      orc_rh(prec, omit, ORC_OMIT_XH_COUPLING,
                                                             xh[((size_t)s * k + mu) * m + j])));
                }
                yh[((size_t)t * k + nu) * m + j] = a;
            }
    /* backward transfers top-down (pre-order visits parents first) */
    for (int64_t c = 1; c < h->C; ++c) {
        int64_t par = h->parent[c];
        const double *E = &h->E[(size_t)c * k * k];
        for (int b = 0; b < k; ++b)
            for (int64_t j = 0; j < m; ++j) {
                double a = 0.0;
                for (int nu = 0; nu < k; ++nu)
                    a = orc_f32(omit, a + LP_TERM((double)orc_q(prec, E[b * k + nu]),
                                                  orc_rh(prec, omit, ORC_OMIT_YH_TRANSFER, yh[((size_t)par * k + nu) * m + j])));
                yh[((size_t)c * k + b) * m + j] = orc_f32(omit, yh[((size_t)c * k + b) * m + j] + a);
            }
    }
    /* leaves: basis and near field, accumulated together in FP32 */
    for (int64_t t = 0; t < h->C; ++t) {
        if (!orc_is_leaf(h, t)) continue;
        for (int64_t i = 0; i < h->size[t]; ++i) {
            int64_t row = h->first[t] + i;
            for (int64_t j = 0; j < m; ++j) {
                double a = 0.0;
                for (int nu = 0; nu < k; ++nu)
                    a = orc_f32(omit, a + LP_TERM((double)orc_q(prec, h->V[row * k + nu]),
                                                  orc_rh(prec, omit, ORC_OMIT_YH_LEAF, yh[((size_t)t * k + nu) * m + j])));
                for (int64_t q = h->list_ptr[t]; q < h->list_ptr[t + 1]; ++q) {
                    int64_t b = h->list_blk[q], s = h->bs[b];
                    if (h->badm[b]) continue;
                    const double *Nb = &h->N[h->boff[b]];
                    int64_t ns = h->size[s];
                    for (int64_t c = 0; c < ns; ++c) {
                        const double x = X[h->perm[h->first[s] + c] * m + j];
                        const double xr = (omit & ORC_ROUND_X_NEAR) ? (double)orc_q(prec, x) : (double)(float)x;
                        a = orc_f32(omit, a + LP_TERM((double)(float)Nb[i * ns + c], xr));
                    }
                }
                Y[h->perm[row] * m + j] += alpha * a;
            }
        }
    }
#undef LP_TERM
    free(xh); free(yh);
}

void orc_matmul_lowp(const orc_h2 *h, int prec, int64_t m, double alpha, const double *X, double beta, double *Y) {
    orc_matmul_lowp_omit(h, prec, m, alpha, X, beta, Y, 0);
}

/* the emulation with some of its rounding points switched off (test infrastructure: planted slips) */
void orc_matmul_lowp_planted(const orc_h2 *h, int prec, int64_t m, double alpha, const double *X, double beta,
                             double *Y, int omit) {
    orc_matmul_lowp_omit(h, prec, m, alpha, X, beta, Y, omit);
}

/* Mixed-precision solve: FP64 iterative refinement around block CG with the
 * low-precision operator.  Outer step: R = B - A X with the FP64 operator; stop
 * when every column has ||R_i|| <= rtol ||B_i||; otherwise solve A_lo D = R by
 * block CG (FP64 vectors and dot products) to inner_rtol and set X += D.  A step
 * that does not halve the worst column's relative residual is a stall; the
 * refinement stops after two (the low-precision operator is then too far from A).
 * Every column returns the outer iterate with the smallest FP64 true residual
 * (a refinement that diverges returns its best iterate, at worst X0).
 * Returns the number of outer steps; *inner_total receives the inner iterations;
 * col_relres (m entries, may be NULL) the true relative residual of each returned
 * column; *status 0 when every column met rtol, 5 otherwise. */
int64_t orc_refine_cg(const orc_h2 *h, int prec, int64_t m, const double *B, double *X, double rtol,
                      double inner_rtol, int64_t max_outer, int64_t max_inner, int64_t *inner_total,
                      double *col_relres, int32_t *status);

/* ------------------------------------------------------------------------ */
/* Differentiation.                                                          */
/* Adjoint product Y <- beta Y + alpha A^T X: the forward transformation of X,  */
/* then for every column cluster s the blocks (t, s) of its column list:       */
/* admissible y_s += alpha S_b^T x_t, inadmissible y|_s += alpha G|_{t x s}^T x|_t, */
/* then the backward transformation (W == V).                                 */
void orc_matmul_adjoint(const orc_h2 *h, int64_t m, double alpha, const double *X, double beta, double *Y) {
    const int k = h->k;
    size_t cw = (size_t)h->C * k * m;
    orc_mm w;
    w.h = h;
    w.m = m;
    w.X = X;
    w.xh = calloc(cw ? cw : 1, sizeof(double));
    w.yh = calloc(cw ? cw : 1, sizeof(double));
    for (int64_t i = 0; i < h->n * m; ++i) Y[i] = (beta == 0.0) ? 0.0 : beta * Y[i];
    orc_forward(&w, 0);
    /* column lists: every leaf block grouped by its column cluster, block order */
    int64_t *cptr = calloc(h->C + 1, sizeof(int64_t)), *cblk = malloc(sizeof(int64_t) * (h->nb ? h->nb : 1));
    for (int64_t b = 0; b < h->nb; ++b) cptr[h->bs[b] + 1]++;
    for (int64_t c = 0; c < h->C; ++c) cptr[c + 1] += cptr[c];
    int64_t *fill = calloc(h->C + 1, sizeof(int64_t));
    for (int64_t b = 0; b < h->nb; ++b) cblk[cptr[h->bs[b]] + fill[h->bs[b]]++] = b;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t s = 0; s < h->C; ++s)
        for (int64_t q = cptr[s]; q < cptr[s + 1]; ++q) {
            int64_t b = cblk[q], t = h->bt[b];
            if (h->badm[b]) {
                const double *Sb = &h->S[h->boff[b]];
                const double *xt = &w.xh[(size_t)t * k * m];
                double *ys = &w.yh[(size_t)s * k * m];
                for (int mu = 0; mu < k; ++mu)
                    for (int64_t j = 0; j < m; ++j) {
                        double acc = 0.0;
                        for (int nu = 0; nu < k; ++nu) acc += Sb[nu * k + mu] * xt[nu * m + j];
                        ys[mu * m + j] += alpha * acc;
                    }
            } else {
                const double *Nb = &h->N[h->boff[b]];
                int64_t nt = h->size[t], ns = h->size[s];
                for (int64_t c = 0; c < ns; ++c) {
                    double *yrow = &Y[h->perm[h->first[s] + c] * m];
                    for (int64_t j = 0; j < m; ++j) {
                        double acc = 0.0;
                        for (int64_t i = 0; i < nt; ++i) acc += Nb[i * ns + c] * X[h->perm[h->first[t] + i] * m + j];
                        yrow[j] += alpha * acc;
                    }
                }
            }
        }
    orc_backward_loops(&w, Y);
    free(cptr); free(cblk); free(fill); free(w.xh); free(w.yh);
}

/* Gradients of L = <dY, A X> (sum over all entries):
 *   dS_b = dyhat_t xhat_s^T  (k x k) for every admissible block, xhat / dyhat the
 *          forward transforms of X and dY;
 *   dN_b = dY|_t X|_s^T      (|t| x |s|) for every near-field block;
 *   dell = sum_b <dS_b/dell, dS_b> + sum_b <dN_b/dell, dN_b>, with
 *          dg/dell = (r / ell^2) exp(-r / ell) at the Chebyshev nodes / points
 *          (V and E do not depend on ell).
 * dS / dN (nullable) are laid out like S / N; dell (nullable) receives the scalar. */
void orc_grad(const orc_h2 *h, int64_t m, const double *X, const double *dY, double *dS, double *dN, double *dell) {
    const int k = h->k;
    size_t cw = (size_t)h->C * k * m;
    double *xh = calloc(cw ? cw : 1, sizeof(double)), *dh = calloc(cw ? cw : 1, sizeof(double));
    orc_forward_transform(h, m, X, xh);
    orc_forward_transform(h, m, dY, dh);
    double total = 0.0;
    for (int64_t b = 0; b < h->nb; ++b) {
        int64_t t = h->bt[b], s = h->bs[b];
        if (h->badm[b]) {
            for (int nu = 0; nu < k; ++nu)
                for (int mu = 0; mu < k; ++mu) {
                    double acc = 0.0;
                    for (int64_t j = 0; j < m; ++j) acc += dh[((size_t)t * k + nu) * m + j] * xh[((size_t)s * k + mu) * m + j];
                    if (dS) dS[h->boff[b] + nu * k + mu] = acc;
                    total += orc_dg(h, &h->nodes[((size_t)t * k + nu) * 3], &h->nodes[((size_t)s * k + mu) * 3]) * acc;
                }
        } else {
            int64_t nt = h->size[t], ns = h->size[s];
            for (int64_t i = 0; i < nt; ++i)
                for (int64_t c = 0; c < ns; ++c) {
                    int64_t gi = h->perm[h->first[t] + i], gj = h->perm[h->first[s] + c];
                    double acc = 0.0;
                    for (int64_t j = 0; j < m; ++j) acc += dY[gi * m + j] * X[gj * m + j];
                    if (dN) dN[h->boff[b] + i * ns + c] = acc;
                    total += orc_dg(h, &h->pts[3 * gi], &h->pts[3 * gj]) * acc;
                }
        }
    }
    if (dell) *dell = total;
    free(xh); free(dh);
}

/* ------------------------------------------------------------------------ */
/* Dense assembly of A_H2 from its definition (n x n, original order)         */

/* full cluster basis V_t (|t| x k): leaf matrix, or [V_{t0} E_{t0}; V_{t1} E_{t1}] */
static void orc_basis_full(const orc_h2 *h, int64_t t, double *out) {
    const int k = h->k;
    if (orc_is_leaf(h, t)) {
        memcpy(out, &h->V[h->first[t] * k], sizeof(double) * h->size[t] * k);
        return;
    }
    int64_t sons[2] = {h->son0[t], h->son1[t]};
    int64_t row0 = 0;
    for (int q = 0; q < 2; ++q) {
        int64_t sq = sons[q];
        double *Vq = malloc(sizeof(double) * h->size[sq] * k);
        orc_basis_full(h, sq, Vq);
        const double *E = &h->E[(size_t)sq * k * k];
        for (int64_t i = 0; i < h->size[sq]; ++i)
            for (int nu = 0; nu < k; ++nu) {
                double acc = 0.0;
                for (int a = 0; a < k; ++a) acc += Vq[i * k + a] * E[a * k + nu];
                out[(row0 + i) * k + nu] = acc;
            }
        row0 += h->size[sq];
        free(Vq);
    }
}

void orc_dense(const orc_h2 *h, double *A) {
    const int k = h->k;
    const int64_t n = h->n;
    memset(A, 0, sizeof(double) * n * n);
    for (int64_t b = 0; b < h->nb; ++b) {
        int64_t t = h->bt[b], s = h->bs[b], nt = h->size[t], ns = h->size[s];
        if (h->badm[b]) {
            double *Vt = malloc(sizeof(double) * nt * k), *Vs = malloc(sizeof(double) * ns * k);
            double *VS = malloc(sizeof(double) * nt * k);
            orc_basis_full(h, t, Vt);
            orc_basis_full(h, s, Vs);
            const double *Sb = &h->S[h->boff[b]];
            for (int64_t i = 0; i < nt; ++i)
                for (int mu = 0; mu < k; ++mu) {
                    double acc = 0.0;
                    for (int nu = 0; nu < k; ++nu) acc += Vt[i * k + nu] * Sb[nu * k + mu];
                    VS[i * k + mu] = acc;
                }
            for (int64_t i = 0; i < nt; ++i)
                for (int64_t j = 0; j < ns; ++j) {
                    double acc = 0.0;
                    for (int mu = 0; mu < k; ++mu) acc += VS[i * k + mu] * Vs[j * k + mu];
                    A[h->perm[h->first[t] + i] * n + h->perm[h->first[s] + j]] = acc;
                }
            free(Vt); free(Vs); free(VS);
        } else {
            const double *Nb = &h->N[h->boff[b]];
            for (int64_t i = 0; i < nt; ++i)
                for (int64_t j = 0; j < ns; ++j)
                    A[h->perm[h->first[t] + i] * n + h->perm[h->first[s] + j]] = Nb[i * ns + j];
        }
    }
}

/* Dense complex H^2 matrix of the Helmholtz kernel, assembled as orc_dense does (full
 * bases V_t S_b V_s^T per admissible block, N_b per near block) with S_b = S + i Si and
 * N_b = N + i Ni; A is n x n complex, entry (i, j) at A[2 (i n + j)] (real), + 1 (imaginary). */
void orc_dense_complex(const orc_h2 *h, double *A) {
    const int k = h->k;
    const int64_t n = h->n;
    memset(A, 0, sizeof(double) * 2 * n * n);
    for (int64_t b = 0; b < h->nb; ++b) {
        int64_t t = h->bt[b], s = h->bs[b], nt = h->size[t], ns = h->size[s];
        if (h->badm[b]) {
            double *Vt = malloc(sizeof(double) * nt * k), *Vs = malloc(sizeof(double) * ns * k);
            double complex *VS = malloc(sizeof(double complex) * nt * k);
            orc_basis_full(h, t, Vt);
            orc_basis_full(h, s, Vs);
            const double *Sr = &h->S[h->boff[b]], *Si = &h->Si[h->boff[b]];
            for (int64_t i = 0; i < nt; ++i)
                for (int mu = 0; mu < k; ++mu) {
                    double complex acc = 0.0;
                    for (int nu = 0; nu < k; ++nu) acc += Vt[i * k + nu] * (Sr[nu * k + mu] + I * Si[nu * k + mu]);
                    VS[i * k + mu] = acc;
                }
            for (int64_t i = 0; i < nt; ++i)
                for (int64_t j = 0; j < ns; ++j) {
                    double complex acc = 0.0;
                    for (int mu = 0; mu < k; ++mu) acc += VS[i * k + mu] * Vs[j * k + mu];
                    const int64_t e = h->perm[h->first[t] + i] * n + h->perm[h->first[s] + j];
                    A[2 * e] = creal(acc);
                    A[2 * e + 1] = cimag(acc);
                }
            free(Vt); free(Vs); free(VS);
        } else {
            const double *Nr = &h->N[h->boff[b]], *Ni = &h->Ni[h->boff[b]];
            for (int64_t i = 0; i < nt; ++i)
                for (int64_t j = 0; j < ns; ++j) {
                    const int64_t e = h->perm[h->first[t] + i] * n + h->perm[h->first[s] + j];
                    A[2 * e] = Nr[i * ns + j];
                    A[2 * e + 1] = Ni[i * ns + j];
                }
        }
    }
}

int orc_is_complex(const orc_h2 *h) { return h->cplx; }

/* Dense derivative d A_H2 / d ell (same structure: V, E fixed; S and N depend on ell). */
void orc_dense_dell(const orc_h2 *h, double *A) {
    const int k = h->k;
    const int64_t n = h->n;
    memset(A, 0, sizeof(double) * n * n);
    double *dS = malloc(sizeof(double) * k * k);
    for (int64_t b = 0; b < h->nb; ++b) {
        int64_t t = h->bt[b], s = h->bs[b], nt = h->size[t], ns = h->size[s];
        if (h->badm[b]) {
            for (int nu = 0; nu < k; ++nu)
                for (int mu = 0; mu < k; ++mu)
                    dS[nu * k + mu] = orc_dg(h, &h->nodes[((size_t)t * k + nu) * 3], &h->nodes[((size_t)s * k + mu) * 3]);
            double *Vt = malloc(sizeof(double) * nt * k), *Vs = malloc(sizeof(double) * ns * k);
            orc_basis_full(h, t, Vt);
            orc_basis_full(h, s, Vs);
            for (int64_t i = 0; i < nt; ++i)
                for (int64_t j = 0; j < ns; ++j) {
                    double acc = 0.0;
                    for (int nu = 0; nu < k; ++nu) {
                        double inner = 0.0;
                        for (int mu = 0; mu < k; ++mu) inner += dS[nu * k + mu] * Vs[j * k + mu];
                        acc += Vt[i * k + nu] * inner;
                    }
                    A[h->perm[h->first[t] + i] * n + h->perm[h->first[s] + j]] = acc;
                }
            free(Vt); free(Vs);
        } else {
            for (int64_t i = 0; i < nt; ++i)
                for (int64_t j = 0; j < ns; ++j) {
                    int64_t gi = h->perm[h->first[t] + i], gj = h->perm[h->first[s] + j];
                    A[gi * n + gj] = orc_dg(h, &h->pts[3 * gi], &h->pts[3 * gj]);
                }
        }
    }
    free(dS);
}

/* ------------------------------------------------------------------------ */
/* Conjugate gradients                                                      */

static double orc_dot_col(int64_t n, int64_t m, const double *u, const double *v, int64_t j) {
    double acc = 0.0;
    for (int64_t i = 0; i < n; ++i) acc += u[i * m + j] * v[i * m + j];
    return acc;
}

/*
 * Block CG with m independent systems (the paper's block CG: one H^2 x P product
 * per iteration, per-column step sizes, stop when every column has converged).
 * X holds X0 on entry and the iterate on exit.  Stopping rule per column:
 * ||r_i|| <= rtol ||b_i||.  A column whose beta_i <= 0 or non-finite is frozen.
 * freeze_converged != 0 stops updating columns once they have converged.
 * Returns the number of iterations; col_iters[i] = the iteration at which column
 * i first met the tolerance (what a single-RHS CG would run); status[i]: 0 ok,
 * 1 breakdown (frozen), 2 not converged within max_iter.
 */
typedef void (*orc_op_fn)(const orc_h2 *h, int prec, int64_t m, double alpha, const double *X, double beta, double *Y);

static void orc_op_f64(const orc_h2 *h, int prec, int64_t m, double alpha, const double *X, double beta, double *Y) {
    (void)prec;
    orc_matmul(h, m, alpha, X, beta, Y);
}

static int64_t orc_block_cg_op(const orc_h2 *h, orc_op_fn op, int prec, int64_t m, const double *B, double *X,
                               double rtol, int64_t max_iter, int freeze_converged, int64_t *col_iters,
                               int32_t *status);

int64_t orc_block_cg(const orc_h2 *h, int64_t m, const double *B, double *X, double rtol,
                     int64_t max_iter, int freeze_converged, int64_t *col_iters, int32_t *status) {
    return orc_block_cg_op(h, orc_op_f64, 0, m, B, X, rtol, max_iter, freeze_converged, col_iters, status);
}

static int64_t orc_block_cg_op(const orc_h2 *h, orc_op_fn op, int prec, int64_t m, const double *B, double *X,
                               double rtol, int64_t max_iter, int freeze_converged, int64_t *col_iters,
                               int32_t *status) {
    const int64_t n = h->n;
    double *R = malloc(sizeof(double) * n * m), *P = malloc(sizeof(double) * n * m);
    double *Ap = malloc(sizeof(double) * n * m);
    double *bn = malloc(sizeof(double) * m);
    int *frozen = calloc(m, sizeof(int)), *seen = calloc(m, sizeof(int));
    int x0_zero = 1;
    for (int64_t i = 0; i < n * m; ++i) if (X[i] != 0.0) { x0_zero = 0; break; }
    if (x0_zero) memcpy(R, B, sizeof(double) * n * m);
    else {
        op(h, prec, m, 1.0, X, 0.0, R);
        for (int64_t i = 0; i < n * m; ++i) R[i] = B[i] - R[i];
    }
    memcpy(P, R, sizeof(double) * n * m);
    for (int64_t j = 0; j < m; ++j) {
        bn[j] = sqrt(orc_dot_col(n, m, B, B, j));
        col_iters[j] = 0;
        status[j] = 0;
    }
    int64_t it = 0;
    for (;;) {
        int all = 1;
        int *conv = malloc(sizeof(int) * m);
        for (int64_t j = 0; j < m; ++j) {
            double rn = sqrt(orc_dot_col(n, m, R, R, j));
            conv[j] = (rn <= rtol * bn[j]);
            if (conv[j] && !seen[j]) { seen[j] = 1; col_iters[j] = it; }
            if (!conv[j] && !frozen[j]) all = 0;
        }
        if (all || it >= max_iter) {
            for (int64_t j = 0; j < m; ++j) {
                if (!conv[j] && !frozen[j]) status[j] = 2;
                if (!seen[j]) col_iters[j] = it;
            }
            free(conv);
            break;
        }
        op(h, prec, m, 1.0, P, 0.0, Ap);
        for (int64_t j = 0; j < m; ++j) {
            if (frozen[j] || (freeze_converged && conv[j])) continue;
            /* an exactly zero residual is an exact solution: nothing to update (the
             * step size would be 0/0) */
            if (orc_dot_col(n, m, R, R, j) == 0.0) continue;
            double beta = orc_dot_col(n, m, P, Ap, j);
            double alpha = orc_dot_col(n, m, P, R, j) / beta;
            if (!(beta > 0.0) || !isfinite(alpha)) { frozen[j] = 1; status[j] = 1; continue; }
            for (int64_t i = 0; i < n; ++i) {
                X[i * m + j] += alpha * P[i * m + j];
                R[i * m + j] -= alpha * Ap[i * m + j];
            }
            double gamma = orc_dot_col(n, m, Ap, R, j) / beta;
            for (int64_t i = 0; i < n; ++i) P[i * m + j] = R[i * m + j] - gamma * P[i * m + j];
        }
        free(conv);
        it++;
    }
    free(R); free(P); free(Ap); free(bn); free(frozen); free(seen);
    return it;
}

static void orc_op_lowp(const orc_h2 *h, int prec, int64_t m, double alpha, const double *X, double beta, double *Y) {
    orc_matmul_lowp(h, prec, m, alpha, X, beta, Y);
}

int64_t orc_block_cg_lowp(const orc_h2 *h, int prec, int64_t m, const double *B, double *X, double rtol,
                          int64_t max_iter, int64_t *col_iters, int32_t *status) {
    return orc_block_cg_op(h, orc_op_lowp, prec, m, B, X, rtol, max_iter, 0, col_iters, status);
}

/* Keep, per column, the iterate with the smallest true residual norm seen so far:
 * rn[j] is the residual norm of the current X; columns that improve on best[j] are
 * copied to Xb.  orc_best_restore puts the best columns back into X. */
static void orc_best_track(int64_t n, int64_t m, const double *X, const double *rn, double *best, double *Xb) {
    for (int64_t j = 0; j < m; ++j) {
        if (!(rn[j] < best[j])) continue;
        best[j] = rn[j];
        for (int64_t i = 0; i < n; ++i) Xb[i * m + j] = X[i * m + j];
    }
}

static void orc_best_restore(int64_t n, int64_t m, double *X, double *rn, const double *best, const double *Xb) {
    for (int64_t j = 0; j < m; ++j) {
        if (!(best[j] < rn[j])) continue;
        rn[j] = best[j];
        for (int64_t i = 0; i < n; ++i) X[i * m + j] = Xb[i * m + j];
    }
}

/*
 * Mixed precision in one CG run by residual replacement (van der Vorst and Ye,
 * 2000): the iterations are the block CG above with the emulated low-precision
 * operator; the recursive residual of every column is watched, and when an open
 * column's norm has dropped below delta times its largest value since the last
 * replacement -- or every column looks converged -- the residual is recomputed
 * as B - A X with the FP64 operator and the iteration continues from it with
 * the same search directions.  The decision is taken every `check` iterations
 * (the GPU reads its state at that cadence); iterations after every column has
 * converged and before the next check do nothing.  Stops when every column meets
 * rtol on a recomputed residual (or is broken down, or max_iter is reached).
 * Every column returns the iterate with the smallest true residual among the
 * recomputed ones (X0 included), so a run that breaks down or diverges returns
 * its best iterate.  Returns the iterations performed; *replacements receives
 * the number of recomputations, col_relres (m entries, may be NULL) the true
 * relative residual of each returned column, *status 0 (all met rtol), 4 (a
 * column broke down) or 5 (not converged).
 */
int64_t orc_block_cg_mixed(const orc_h2 *h, int prec, int64_t m, const double *B, double *X, double rtol,
                           double delta, int64_t max_iter, int64_t check, int64_t *replacements,
                           double *col_relres, int32_t *status) {
    const int64_t n = h->n;
    double *R = malloc(sizeof(double) * n * m), *P = malloc(sizeof(double) * n * m);
    double *Ap = malloc(sizeof(double) * n * m);
    double *bn = malloc(sizeof(double) * m), *rmax = malloc(sizeof(double) * m);
    int *frozen = calloc(m, sizeof(int)), *conv = calloc(m, sizeof(int));
    double *Xb = malloc(sizeof(double) * n * m), *best = malloc(sizeof(double) * m);
    if (check < 1) check = 1;
    /* true residual and the quantities that restart from it; the best iterate so far */
    #define ORC_REPLACE()                                                        \
        do {                                                                     \
            memcpy(R, B, sizeof(double) * n * m);                                \
            orc_matmul(h, m, -1.0, X, 1.0, R);                                   \
            for (int64_t j = 0; j < m; ++j) {                                    \
                rmax[j] = sqrt(orc_dot_col(n, m, R, R, j));                      \
                conv[j] = rmax[j] <= rtol * bn[j];                               \
            }                                                                    \
            orc_best_track(n, m, X, rmax, best, Xb);                             \
        } while (0)
    for (int64_t j = 0; j < m; ++j) {
        bn[j] = sqrt(orc_dot_col(n, m, B, B, j));
        best[j] = INFINITY;
    }
    ORC_REPLACE();
    memcpy(P, R, sizeof(double) * n * m);
    int64_t it = 0, done_iters = 0, rep = 0, last_rep = 0;
    int want = 0;
    for (;;) {
        if (it % check == 0 || it >= max_iter) {
            int all = 1;
            for (int64_t j = 0; j < m; ++j) if (!conv[j] && !frozen[j]) all = 0;
            if (it != last_rep && (want || all || it >= max_iter)) {
                ORC_REPLACE();
                want = 0;
                ++rep;
                last_rep = it;
                all = 1;
                for (int64_t j = 0; j < m; ++j) if (!conv[j] && !frozen[j]) all = 0;
            }
            if (all || it >= max_iter) break;
        }
        int all = 1;
        for (int64_t j = 0; j < m; ++j) if (!conv[j] && !frozen[j]) all = 0;
        if (!all) {
            orc_op_lowp(h, prec, m, 1.0, P, 0.0, Ap);
            for (int64_t j = 0; j < m; ++j) {
                if (frozen[j]) continue;
                if (orc_dot_col(n, m, R, R, j) == 0.0) continue;
                double beta = orc_dot_col(n, m, P, Ap, j);
                double alpha = orc_dot_col(n, m, P, R, j) / beta;
                if (!(beta > 0.0) || !isfinite(alpha)) { frozen[j] = 1; continue; }
                for (int64_t i = 0; i < n; ++i) {
                    X[i * m + j] += alpha * P[i * m + j];
                    R[i * m + j] -= alpha * Ap[i * m + j];
                }
                double gamma = orc_dot_col(n, m, Ap, R, j) / beta;
                for (int64_t i = 0; i < n; ++i) P[i * m + j] = R[i * m + j] - gamma * P[i * m + j];
            }
            for (int64_t j = 0; j < m; ++j) {
                double rn = sqrt(orc_dot_col(n, m, R, R, j));
                conv[j] = rn <= rtol * bn[j];
                if (conv[j] || frozen[j]) continue;
                if (rn > rmax[j]) rmax[j] = rn;
                if (rn < delta * rmax[j]) want = 1;
            }
            ++done_iters;
        }
        ++it;
    }
    #undef ORC_REPLACE
    /* the loop ends on a recomputed residual: rmax holds the true residual norms of X;
     * the status describes the returned columns (a breakdown is reported as such) */
    orc_best_restore(n, m, X, rmax, best, Xb);
    int st = 0;
    for (int64_t j = 0; j < m; ++j) {
        if (frozen[j]) st = 4;
        else if (!(rmax[j] <= rtol * bn[j]) && st == 0) st = 5;
    }
    if (col_relres)
        for (int64_t j = 0; j < m; ++j) col_relres[j] = bn[j] > 0.0 ? rmax[j] / bn[j] : rmax[j];
    if (status) *status = st;
    *replacements = rep;
    free(R); free(P); free(Ap); free(bn); free(rmax); free(frozen); free(conv); free(Xb); free(best);
    return done_iters;
}

int64_t orc_refine_cg(const orc_h2 *h, int prec, int64_t m, const double *B, double *X, double rtol,
                      double inner_rtol, int64_t max_outer, int64_t max_inner, int64_t *inner_total,
                      double *col_relres, int32_t *status) {
    const int64_t n = h->n;
    double *R = malloc(sizeof(double) * n * m), *D = malloc(sizeof(double) * n * m);
    double *Xb = malloc(sizeof(double) * n * m), *rn = malloc(sizeof(double) * m);
    double *best = malloc(sizeof(double) * m), *bn = malloc(sizeof(double) * m);
    int64_t *ci = malloc(sizeof(int64_t) * m);
    int32_t *st = malloc(sizeof(int32_t) * m);
    for (int64_t j = 0; j < m; ++j) {
        bn[j] = sqrt(orc_dot_col(n, m, B, B, j));
        best[j] = INFINITY;
    }
    *inner_total = 0;
    int64_t outer = 0, stalls = 0;
    int done = 0;
    double prev = INFINITY;
    for (;;) {
        memcpy(R, B, sizeof(double) * n * m);
        orc_matmul(h, m, -1.0, X, 1.0, R);
        done = 1;
        double worst = 0.0;
        for (int64_t j = 0; j < m; ++j) {
            rn[j] = sqrt(orc_dot_col(n, m, R, R, j));
            double rel = bn[j] > 0.0 ? rn[j] / bn[j] : rn[j];
            if (rel > rtol) done = 0;
            if (rel > worst) worst = rel;
        }
        orc_best_track(n, m, X, rn, best, Xb);
        /* a step that does not halve the worst relative residual is a stall; two stalls stop */
        if (worst > 0.5 * prev) stalls++;
        prev = worst;
        if (done || outer >= max_outer || stalls >= 2) break;
        memset(D, 0, sizeof(double) * n * m);
        *inner_total += orc_block_cg_op(h, orc_op_lowp, prec, m, R, D, inner_rtol, max_inner, 0, ci, st);
        for (int64_t i = 0; i < n * m; ++i) X[i] += D[i];
        outer++;
    }
    orc_best_restore(n, m, X, rn, best, Xb);
    done = 1;
    for (int64_t j = 0; j < m; ++j) {
        const double rel = bn[j] > 0.0 ? rn[j] / bn[j] : rn[j];
        if (col_relres) col_relres[j] = rel;
        if (!(rel <= rtol)) done = 0;
    }
    if (status) *status = done ? 0 : 5;
    free(R); free(D); free(Xb); free(rn); free(best); free(bn); free(ci); free(st);
    return outer;
}

/* ------------------------------------------------------------------------ */
/* Block CG with one shared block Krylov space (O'Leary's block CG, cited by  */
/* the paper as the alternative that enriches the Krylov space).  The search  */
/* block is kept orthonormal; directions that become linearly dependent are  */
/* dropped (deflation), so the m x m Gram matrices stay positive definite.    */

/* G = U^T V for n x m blocks (m x m, row-major) */
static void orc_gram(int64_t n, int64_t m, const double *U, const double *V, double *G) {
    for (int64_t a = 0; a < m; ++a)
        for (int64_t b = 0; b < m; ++b) {
            double acc = 0.0;
            for (int64_t i = 0; i < n; ++i) acc += U[i * m + a] * V[i * m + b];
            G[a * m + b] = acc;
        }
}

/* Y += sign * U C for an n x m block U and an m x m matrix C */
static void orc_block_axpy(int64_t n, int64_t m, double sign, const double *U, const double *C, double *Y) {
    for (int64_t i = 0; i < n; ++i)
        for (int64_t b = 0; b < m; ++b) {
            double acc = 0.0;
            for (int64_t a = 0; a < m; ++a) acc += U[i * m + a] * C[a * m + b];
            Y[i * m + b] += sign * acc;
        }
}

/* Orthonormalise the columns of Z (n x m) into P: pivoted Cholesky of W = Z^T Z
 * picks the columns in order of decreasing remaining norm and stops when the
 * remaining squared norm is below drop^2 times the largest initial one; the kept
 * columns give P = Z_kept L^{-T}; a second Cholesky QR of the kept block (no
 * pivoting, no dropping) restores FP64 orthogonality.  Dropped columns of P are
 * zero; active[j] marks kept columns.  Returns the rank.
 * lv[q * m + j] is the factor entry of column j at pivot step q, dg[q] its diagonal. */
static void orc_apply_inv_lt(int64_t n, int64_t m, int64_t rank, const int64_t *piv, const double *lv,
                             const double *dg, const double *T, double *P) {
    memset(P, 0, sizeof(double) * n * m);
    for (int64_t q = 0; q < rank; ++q) {
        int64_t c = piv[q];
        for (int64_t i = 0; i < n; ++i) {
            double v = T[i * m + c];
            for (int64_t r = 0; r < q; ++r) v -= P[i * m + piv[r]] * lv[r * m + c];
            P[i * m + c] = v / dg[q];
        }
    }
}

static int64_t orc_orth(int64_t n, int64_t m, const double *Z, double *P, int *active, double drop) {
    double *W = malloc(sizeof(double) * m * m), *lv = calloc(m * m, sizeof(double));
    double *dg = calloc(m, sizeof(double)), *d = malloc(sizeof(double) * m);
    double *T = malloc(sizeof(double) * n * m);
    int64_t *piv = malloc(sizeof(int64_t) * m);
    /* pass 1: pivoted Cholesky of Z^T Z with dropping */
    orc_gram(n, m, Z, Z, W);
    double dmax = 0.0;
    for (int64_t j = 0; j < m; ++j) {
        d[j] = W[j * m + j];
        active[j] = 0;
        if (d[j] > dmax) dmax = d[j];
    }
    int64_t rank = 0;
    while (rank < m) {
        int64_t best = -1;
        for (int64_t j = 0; j < m; ++j)
            if (!active[j] && (best < 0 || d[j] > d[best])) best = j;
        if (!(dmax > 0.0) || !(d[best] > drop * drop * dmax)) break;
        active[best] = 1;
        piv[rank] = best;
        dg[rank] = sqrt(d[best]);
        for (int64_t j = 0; j < m; ++j) {
            if (active[j]) continue;
            double v = W[j * m + best];
            for (int64_t q = 0; q < rank; ++q) v -= lv[q * m + j] * lv[q * m + best];
            lv[rank * m + j] = v / dg[rank];
            d[j] -= lv[rank * m + j] * lv[rank * m + j];
        }
        rank++;
    }
    orc_apply_inv_lt(n, m, rank, piv, lv, dg, Z, P);
    /* pass 2: Cholesky QR of the kept block, same pivot order */
    memcpy(T, P, sizeof(double) * n * m);
    orc_gram(n, m, T, T, W);
    memset(lv, 0, sizeof(double) * m * m);
    for (int64_t q = 0; q < rank; ++q) {
        int64_t c = piv[q];
        double v = W[c * m + c];
        for (int64_t r = 0; r < q; ++r) v -= lv[r * m + c] * lv[r * m + c];
        dg[q] = sqrt(v > 0.0 ? v : 0.0);
        for (int64_t q2 = q + 1; q2 < rank; ++q2) {
            int64_t c2 = piv[q2];
            double u = W[c2 * m + c];
            for (int64_t r = 0; r < q; ++r) u -= lv[r * m + c2] * lv[r * m + c];
            lv[q * m + c2] = u / dg[q];
        }
    }
    orc_apply_inv_lt(n, m, rank, piv, lv, dg, T, P);
    free(W); free(lv); free(dg); free(d); free(T); free(piv);
    return rank;
}

/* Solve G C = F for the active indices (G symmetric positive definite on them),
 * C and F m x m; inactive rows of C are zero.  Returns 0, or 1 if G is not
 * positive definite on the active set. */
static int orc_spd_solve(int64_t m, const int *active, const double *G, const double *F, double *C) {
    int64_t r = 0, *idx = malloc(sizeof(int64_t) * m);
    for (int64_t j = 0; j < m; ++j) if (active[j]) idx[r++] = j;
    double *L = calloc(r > 0 ? r * r : 1, sizeof(double));
    int bad = 0;
    for (int64_t a = 0; a < r && !bad; ++a) {
        double v = G[idx[a] * m + idx[a]];
        for (int64_t q = 0; q < a; ++q) v -= L[a * r + q] * L[a * r + q];
        if (!(v > 0.0)) { bad = 1; break; }
        L[a * r + a] = sqrt(v);
        for (int64_t b = a + 1; b < r; ++b) {
            double u = G[idx[b] * m + idx[a]];
            for (int64_t q = 0; q < a; ++q) u -= L[b * r + q] * L[a * r + q];
            L[b * r + a] = u / L[a * r + a];
        }
    }
    memset(C, 0, sizeof(double) * m * m);
    if (!bad)
        for (int64_t col = 0; col < m; ++col) {
            double *y = malloc(sizeof(double) * (r ? r : 1));
            for (int64_t a = 0; a < r; ++a) {  /* L y = F[idx, col] */
                double v = F[idx[a] * m + col];
                for (int64_t q = 0; q < a; ++q) v -= L[a * r + q] * y[q];
                y[a] = v / L[a * r + a];
            }
            for (int64_t a = r - 1; a >= 0; --a) {  /* L^T c = y */
                double v = y[a];
                for (int64_t q = a + 1; q < r; ++q) v -= L[q * r + a] * C[idx[q] * m + col];
                C[idx[a] * m + col] = v / L[a * r + a];
            }
            free(y);
        }
    free(L); free(idx);
    return bad;
}

/* Returns the number of iterations; *rank_min receives the smallest rank of the
 * search block; status[j]: 0 converged, 2 not converged, 1 breakdown. */
int64_t orc_block_cg_shared(const orc_h2 *h, int64_t m, const double *B, double *X, double rtol, int64_t max_iter,
                            double drop, int64_t *rank_min, int32_t *status) {
    const int64_t n = h->n;
    double *R = malloc(sizeof(double) * n * m), *P = malloc(sizeof(double) * n * m);
    double *Q = malloc(sizeof(double) * n * m), *Z = malloc(sizeof(double) * n * m);
    double *G = malloc(sizeof(double) * m * m), *F = malloc(sizeof(double) * m * m);
    double *Lam = malloc(sizeof(double) * m * m), *bn = malloc(sizeof(double) * m);
    int *active = malloc(sizeof(int) * m);
    orc_matmul(h, m, 1.0, X, 0.0, R);
    for (int64_t i = 0; i < n * m; ++i) R[i] = B[i] - R[i];
    for (int64_t j = 0; j < m; ++j) { bn[j] = sqrt(orc_dot_col(n, m, B, B, j)); status[j] = 0; }
    *rank_min = orc_orth(n, m, R, P, active, drop);
    int64_t it = 0;
    int broke = 0;
    for (;;) {
        int all = 1;
        for (int64_t j = 0; j < m; ++j)
            if (sqrt(orc_dot_col(n, m, R, R, j)) > rtol * bn[j]) all = 0;
        if (all || it >= max_iter) break;
        orc_matmul(h, m, 1.0, P, 0.0, Q);
        orc_gram(n, m, P, Q, G);          /* G = P^T A P */
        orc_gram(n, m, P, R, F);          /* F = P^T R   */
        if (orc_spd_solve(m, active, G, F, Lam)) { broke = 1; break; }
        orc_block_axpy(n, m, 1.0, P, Lam, X);
        orc_block_axpy(n, m, -1.0, Q, Lam, R);
        orc_gram(n, m, Q, R, F);          /* F = (A P)^T R */
        if (orc_spd_solve(m, active, G, F, Lam)) { broke = 1; break; }
        memcpy(Z, R, sizeof(double) * n * m);
        orc_block_axpy(n, m, -1.0, P, Lam, Z);  /* Z = R + P Psi, Psi = -G^{-1} (A P)^T R */
        int64_t r = orc_orth(n, m, Z, P, active, drop);
        if (r < *rank_min) *rank_min = r;
        it++;
    }
    for (int64_t j = 0; j < m; ++j)
        if (sqrt(orc_dot_col(n, m, R, R, j)) > rtol * bn[j]) status[j] = broke ? 1 : 2;
    free(R); free(P); free(Q); free(Z); free(G); free(F); free(Lam); free(bn); free(active);
    return it;
}

/* The paper's single-RHS CG (relative stopping rule), for the per-column pin. */
int64_t orc_cg1(const orc_h2 *h, const double *b, double *x, double rtol, int64_t max_iter) {
    const int64_t n = h->n;
    double *r = malloc(sizeof(double) * n), *p = malloc(sizeof(double) * n), *a = malloc(sizeof(double) * n);
    int x0_zero = 1;
    for (int64_t i = 0; i < n; ++i) if (x[i] != 0.0) { x0_zero = 0; break; }
    if (x0_zero) memcpy(r, b, sizeof(double) * n);
    else {
        orc_matmul(h, 1, 1.0, x, 0.0, r);
        for (int64_t i = 0; i < n; ++i) r[i] = b[i] - r[i];
    }
    memcpy(p, r, sizeof(double) * n);
    double bn = sqrt(orc_dot_col(n, 1, b, b, 0));
    int64_t it = 0;
    while (sqrt(orc_dot_col(n, 1, r, r, 0)) > rtol * bn && it < max_iter) {
        orc_matmul(h, 1, 1.0, p, 0.0, a);
        double beta = orc_dot_col(n, 1, p, a, 0);
        double alpha = orc_dot_col(n, 1, p, r, 0) / beta;
        if (!(beta > 0.0) || !isfinite(alpha)) break;
        for (int64_t i = 0; i < n; ++i) { x[i] += alpha * p[i]; r[i] -= alpha * a[i]; }
        double gamma = orc_dot_col(n, 1, a, r, 0) / beta;
        for (int64_t i = 0; i < n; ++i) p[i] = r[i] - gamma * p[i];
        it++;
    }
    free(r); free(p); free(a);
    return it;
}

int orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_threads(int t) {
#ifdef _OPENMP
    if (t > 0) omp_set_num_threads(t);
#else
    (void)t;
#endif
}

/* ------------------------------------------------------------------------ */
/* Block GMRES(ell)                                                         */

/*
 * Block GMRES with restarts and no preconditioner (section 5.2, the block form of
 * the generalized minimal residual method with M = I): m independent GMRES
 * processes that share one H^2 x Q product per Arnoldi step.  X holds X0 on entry
 * and the iterate on exit.
 *
 * One cycle, for every column i that has not met ||b_i - A x_i|| <= rtol ||b_i||:
 *   r = b - A x, beta = ||r||, rhat = beta e_0, q_0 = r / beta;
 *   step k (while k < ell and some column is open):
 *     a = A q_k                                    (one product for all columns)
 *     h[j][k] = <q_j, a>, j = 0..k                (classical Gram-Schmidt: every
 *     a = a - sum_j q_j h[j][k]                    projection taken from the same a)
 *     h[k+1][k] = ||a||, q_{k+1} = a / h[k+1][k]
 *     the earlier rotations G_0..G_{k-1} applied to column k of h, then the
 *     rotation G_k that zeroes h[k+1][k], applied to h and to rhat.
 *   A column closes once |rhat[k+1]| <= rtol ||b_i|| (a vanishing new direction
 *   gives rhat[k+1] = 0); a zero pivot (h[k][k] = h[k+1][k] = 0) is a breakdown and
 *   the step is not used.  At the end of the cycle each column solves R y = rhat
 *   with its own number of steps k_i (R the rotated upper triangle of h) and sets
 *   x += sum_{j < k_i} q_j y_j.
 * Cycles repeat until every column meets the bound or max_iter Arnoldi steps have
 * run (counted once per step, whatever the number of open columns).
 * Returns the number of Arnoldi steps; col_iters[i]: steps in which column i was
 * open; status[i]: 0 converged, 1 breakdown, 2 not converged; res_est[i]:
 * |rhat[k_i]| / ||b_i|| at the end of the column's last cycle (the GMRES estimate
 * of its relative residual); *cycles: number of cycles.
 */
int64_t orc_block_gmres(const orc_h2 *h, int64_t m, const double *B, double *X, double rtol, int64_t ell,
                        int64_t max_iter, int64_t *col_iters, int32_t *status, double *res_est, int64_t *cycles) {
    const int64_t n = h->n;
    double *Q = malloc(sizeof(double) * (ell + 1) * n * m);  /* basis blocks q_0..q_ell, n x m each */
    double *R = malloc(sizeof(double) * n * m), *Aq = malloc(sizeof(double) * n * m);
    double *H = malloc(sizeof(double) * m * (ell + 1) * ell);  /* column i: (ell + 1) x ell, row-major */
    double *cs = malloc(sizeof(double) * m * ell), *sn = malloc(sizeof(double) * m * ell);
    double *rh = malloc(sizeof(double) * m * (ell + 1)), *y = malloc(sizeof(double) * ell);
    double *bn = malloc(sizeof(double) * m);
    int64_t *kc = malloc(sizeof(int64_t) * m);
    int *open = malloc(sizeof(int) * m), *done = calloc(m, sizeof(int));
#define HH(i, r, c) H[((i) * (ell + 1) + (r)) * ell + (c)]
#define QQ(j) (Q + (int64_t)(j) * n * m)
    for (int64_t i = 0; i < m; ++i) {
        bn[i] = sqrt(orc_dot_col(n, m, B, B, i));
        col_iters[i] = 0;
        status[i] = 2;
        res_est[i] = 0.0;
    }
    int64_t it = 0, cyc = 0;
    for (;;) {
        /* residual of the current iterate; columns already within the bound are done */
        orc_matmul(h, m, 1.0, X, 0.0, R);
        for (int64_t e = 0; e < n * m; ++e) R[e] = B[e] - R[e];
        int any = 0;
        for (int64_t i = 0; i < m; ++i) {
            open[i] = 0;
            kc[i] = 0;
            if (done[i]) continue;
            const double beta = sqrt(orc_dot_col(n, m, R, R, i));
            if (beta <= rtol * bn[i]) {
                done[i] = 1;
                status[i] = 0;
                continue;
            }
            open[i] = 1;
            any = 1;
            for (int64_t r = 0; r <= ell; ++r) rh[i * (ell + 1) + r] = 0.0;
            rh[i * (ell + 1)] = beta;
            for (int64_t v = 0; v < n; ++v) QQ(0)[v * m + i] = R[v * m + i] / beta;
        }
        if (!any || it >= max_iter) break;
        /* columns that are not open carry zero basis vectors */
        for (int64_t i = 0; i < m; ++i)
            if (!open[i])
                for (int64_t v = 0; v < n; ++v) QQ(0)[v * m + i] = 0.0;
        cyc++;
        for (int64_t k = 0; k < ell && it < max_iter; ++k) {
            int still = 0;
            for (int64_t i = 0; i < m; ++i) still |= open[i];
            if (!still) break;
            orc_matmul(h, m, 1.0, QQ(k), 0.0, Aq);
            it++;
            for (int64_t i = 0; i < m; ++i) {
                double *q1 = QQ(k + 1);
                if (!open[i]) {
                    for (int64_t v = 0; v < n; ++v) q1[v * m + i] = 0.0;
                    continue;
                }
                /* classical Gram-Schmidt against q_0..q_k */
                for (int64_t j = 0; j <= k; ++j) HH(i, j, k) = orc_dot_col(n, m, QQ(j), Aq, i);
                for (int64_t v = 0; v < n; ++v) {
                    double a = Aq[v * m + i];
                    for (int64_t j = 0; j <= k; ++j) a -= QQ(j)[v * m + i] * HH(i, j, k);
                    Aq[v * m + i] = a;
                }
                const double hn = sqrt(orc_dot_col(n, m, Aq, Aq, i));
                HH(i, k + 1, k) = hn;
                /* earlier rotations on the new column */
                for (int64_t j = 0; j < k; ++j) {
                    const double c = cs[i * ell + j], s = sn[i * ell + j];
                    const double u = HH(i, j, k), w = HH(i, j + 1, k);
                    HH(i, j, k) = c * u + s * w;
                    HH(i, j + 1, k) = -s * u + c * w;
                }
                /* new rotation: (h[k][k], h[k+1][k]) -> (rho, 0) */
                const double u = HH(i, k, k), w = HH(i, k + 1, k);
                const double rho = hypot(u, w);
                if (rho == 0.0) {  /* singular projected matrix: the step is not used */
                    open[i] = 0;
                    done[i] = 1;
                    status[i] = 1;
                    for (int64_t v = 0; v < n; ++v) q1[v * m + i] = 0.0;
                    continue;
                }
                const double c = u / rho, s = w / rho;
                cs[i * ell + k] = c;
                sn[i * ell + k] = s;
                HH(i, k, k) = rho;
                HH(i, k + 1, k) = 0.0;
                const double r0 = rh[i * (ell + 1) + k];
                rh[i * (ell + 1) + k] = c * r0;
                rh[i * (ell + 1) + k + 1] = -s * r0;
                kc[i] = k + 1;
                col_iters[i]++;
                if (fabs(rh[i * (ell + 1) + k + 1]) <= rtol * bn[i] || hn == 0.0) {
                    open[i] = 0;
                    for (int64_t v = 0; v < n; ++v) q1[v * m + i] = 0.0;
                } else {
                    for (int64_t v = 0; v < n; ++v) q1[v * m + i] = Aq[v * m + i] / hn;
                }
            }
        }
        /* least-squares solution of the cycle: R y = rhat, then x += V y */
        for (int64_t i = 0; i < m; ++i) {
            const int64_t kk = kc[i];
            if (kk == 0) continue;
            for (int64_t r = kk - 1; r >= 0; --r) {
                double s = rh[i * (ell + 1) + r];
                for (int64_t c = r + 1; c < kk; ++c) s -= HH(i, r, c) * y[c];
                y[r] = s / HH(i, r, r);
            }
            for (int64_t v = 0; v < n; ++v) {
                double a = X[v * m + i];
                for (int64_t j = 0; j < kk; ++j) a += QQ(j)[v * m + i] * y[j];
                X[v * m + i] = a;
            }
            res_est[i] = bn[i] > 0.0 ? fabs(rh[i * (ell + 1) + kk]) / bn[i] : 0.0;
        }
    }
#undef HH
#undef QQ
    *cycles = cyc;
    free(Q); free(R); free(Aq); free(H); free(cs); free(sn); free(rh); free(y); free(bn); free(kc);
    free(open); free(done);
    return it;
}

/*
 * Block GMRES(ell) over the complex numbers (section 5.2 with K = C): the same
 * cycle as orc_block_gmres with the complex inner product <u, v> = u^H v, complex
 * Hessenberg entries and complex Givens rotations G = [c s; -conj(s) c] with c real:
 * for (u, w), w = h[k+1][k] >= 0, rho = sqrt(|u|^2 + w^2), c = |u| / rho,
 * s = (u / |u|) w / rho (c = 0, s = 1 when u = 0), so that G (u, w) = (rho u / |u|, 0).
 * B and X hold m complex columns as n x 2m real arrays (column pairs real, imaginary);
 * the operator must use the complex kernel.  Outputs as orc_block_gmres, per complex
 * column.
 */
int64_t orc_block_gmres_c(const orc_h2 *h, int64_t m, const double *B, double *X, double rtol, int64_t ell,
                          int64_t max_iter, int64_t *col_iters, int32_t *status, double *res_est, int64_t *cycles) {
    const int64_t n = h->n, mr = 2 * m;
    double complex *Q = malloc(sizeof(double complex) * (ell + 1) * n * m);
    double complex *a = malloc(sizeof(double complex) * n * m);
    double *R = malloc(sizeof(double) * n * mr), *Xr = malloc(sizeof(double) * n * mr);
    double complex *H = malloc(sizeof(double complex) * m * (ell + 1) * ell);
    double *cs = malloc(sizeof(double) * m * ell);
    double complex *sn = malloc(sizeof(double complex) * m * ell);
    double complex *rh = malloc(sizeof(double complex) * m * (ell + 1)), *y = malloc(sizeof(double complex) * ell);
    double *bn = malloc(sizeof(double) * m);
    int64_t *kc = malloc(sizeof(int64_t) * m);
    int *open = malloc(sizeof(int) * m), *done = calloc(m, sizeof(int));
#define HH(i, r, c) H[((i) * (ell + 1) + (r)) * ell + (c)]
#define QQ(j) (Q + (int64_t)(j) * n * m)
#define CX(A, v, i) ((A)[(v) * mr + 2 * (i)] + I * (A)[(v) * mr + 2 * (i) + 1])
    for (int64_t i = 0; i < m; ++i) {
        double s2 = 0.0;
        for (int64_t v = 0; v < n; ++v) {
            const double complex z = CX(B, v, i);
            s2 += creal(z) * creal(z) + cimag(z) * cimag(z);
        }
        bn[i] = sqrt(s2);
        col_iters[i] = 0;
        status[i] = 2;
        res_est[i] = 0.0;
    }
    int64_t it = 0, cyc = 0;
    for (;;) {
        orc_matmul(h, mr, 1.0, X, 0.0, R);
        for (int64_t e = 0; e < n * mr; ++e) R[e] = B[e] - R[e];
        int any = 0;
        for (int64_t i = 0; i < m; ++i) {
            open[i] = 0;
            kc[i] = 0;
            if (done[i]) continue;
            double s2 = 0.0;
            for (int64_t v = 0; v < n; ++v) {
                const double complex z = CX(R, v, i);
                s2 += creal(z) * creal(z) + cimag(z) * cimag(z);
            }
            const double beta = sqrt(s2);
            if (beta <= rtol * bn[i]) {
                done[i] = 1;
                status[i] = 0;
                continue;
            }
            open[i] = 1;
            any = 1;
            for (int64_t r = 0; r <= ell; ++r) rh[i * (ell + 1) + r] = 0.0;
            rh[i * (ell + 1)] = beta;
            for (int64_t v = 0; v < n; ++v) QQ(0)[v * m + i] = CX(R, v, i) / beta;
        }
        if (!any || it >= max_iter) break;
        for (int64_t i = 0; i < m; ++i)
            if (!open[i])
                for (int64_t v = 0; v < n; ++v) QQ(0)[v * m + i] = 0.0;
        cyc++;
        for (int64_t k = 0; k < ell && it < max_iter; ++k) {
            int still = 0;
            for (int64_t i = 0; i < m; ++i) still |= open[i];
            if (!still) break;
            /* a = A q_k (the real product on the interleaved column pairs) */
            for (int64_t v = 0; v < n; ++v)
                for (int64_t i = 0; i < m; ++i) {
                    Xr[v * mr + 2 * i] = creal(QQ(k)[v * m + i]);
                    Xr[v * mr + 2 * i + 1] = cimag(QQ(k)[v * m + i]);
                }
            orc_matmul(h, mr, 1.0, Xr, 0.0, R);
            for (int64_t v = 0; v < n; ++v)
                for (int64_t i = 0; i < m; ++i) a[v * m + i] = CX(R, v, i);
            it++;
            for (int64_t i = 0; i < m; ++i) {
                double complex *q1 = QQ(k + 1);
                if (!open[i]) {
                    for (int64_t v = 0; v < n; ++v) q1[v * m + i] = 0.0;
                    continue;
                }
                for (int64_t j = 0; j <= k; ++j) {
                    double complex d = 0.0;
                    for (int64_t v = 0; v < n; ++v) d += conj(QQ(j)[v * m + i]) * a[v * m + i];
                    HH(i, j, k) = d;
                }
                double s2 = 0.0;
                for (int64_t v = 0; v < n; ++v) {
                    double complex z = a[v * m + i];
                    for (int64_t j = 0; j <= k; ++j) z -= QQ(j)[v * m + i] * HH(i, j, k);
                    a[v * m + i] = z;
                    s2 += creal(z) * creal(z) + cimag(z) * cimag(z);
                }
                const double hn = sqrt(s2);
                HH(i, k + 1, k) = hn;
                for (int64_t j = 0; j < k; ++j) {
                    const double c = cs[i * ell + j];
                    const double complex sj = sn[i * ell + j];
                    const double complex u = HH(i, j, k), w = HH(i, j + 1, k);
                    HH(i, j, k) = c * u + sj * w;
                    HH(i, j + 1, k) = -conj(sj) * u + c * w;
                }
                const double complex u = HH(i, k, k);
                const double au = cabs(u), rho = sqrt(au * au + hn * hn);
                if (rho == 0.0) {
                    open[i] = 0;
                    done[i] = 1;
                    status[i] = 1;
                    for (int64_t v = 0; v < n; ++v) q1[v * m + i] = 0.0;
                    continue;
                }
                double c;
                double complex sk;
                if (au == 0.0) {
                    c = 0.0;
                    sk = 1.0;
                } else {
                    c = au / rho;
                    sk = (u / au) * (hn / rho);
                }
                cs[i * ell + k] = c;
                sn[i * ell + k] = sk;
                HH(i, k, k) = c * u + sk * hn;
                HH(i, k + 1, k) = 0.0;
                const double complex r0 = rh[i * (ell + 1) + k];
                rh[i * (ell + 1) + k] = c * r0;
                rh[i * (ell + 1) + k + 1] = -conj(sk) * r0;
                kc[i] = k + 1;
                col_iters[i]++;
                if (cabs(rh[i * (ell + 1) + k + 1]) <= rtol * bn[i] || hn == 0.0) {
                    open[i] = 0;
                    for (int64_t v = 0; v < n; ++v) q1[v * m + i] = 0.0;
                } else {
                    for (int64_t v = 0; v < n; ++v) q1[v * m + i] = a[v * m + i] / hn;
                }
            }
        }
        for (int64_t i = 0; i < m; ++i) {
            const int64_t kk = kc[i];
            if (kk == 0) continue;
            for (int64_t r = kk - 1; r >= 0; --r) {
                double complex acc = rh[i * (ell + 1) + r];
                for (int64_t c = r + 1; c < kk; ++c) acc -= HH(i, r, c) * y[c];
                y[r] = acc / HH(i, r, r);
            }
            for (int64_t v = 0; v < n; ++v) {
                double complex z = CX(X, v, i);
                for (int64_t j = 0; j < kk; ++j) z += QQ(j)[v * m + i] * y[j];
                X[v * mr + 2 * i] = creal(z);
                X[v * mr + 2 * i + 1] = cimag(z);
            }
            res_est[i] = bn[i] > 0.0 ? cabs(rh[i * (ell + 1) + kk]) / bn[i] : 0.0;
        }
    }
#undef HH
#undef QQ
#undef CX
    *cycles = cyc;
    free(Q); free(a); free(R); free(Xr); free(H); free(cs); free(sn); free(rh); free(y); free(bn); free(kc);
    free(open); free(done);
    return it;
}
