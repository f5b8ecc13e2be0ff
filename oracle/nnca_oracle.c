/*
 * nnca_oracle.c -- plain FP64 CPU oracle for the NNCA-based H2 matrix-vector
 * product (Gujjula & Ambikasaran, "A new Nested Cross Approximation").
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
 * baseline of the benchmark load this library.  It shares no code, header,
 * table or helper with the GPU library; the two are written separately from
 * the paper and from the readings listed in the design notes.
 *
 * What it computes, in the paper's order:
 *   - the uniform 2^d tree (Sec. 2.1) over the bounding cube of the points;
 *   - the admissibility condition (Sec. 2.2, eq. for max diam <= eta dist),
 *     neighbours N(B) and interaction lists IL(B) (Table 1, Fig. 1);
 *   - partially pivoted ACA with the stopping rule of Sec. 2.2.1;
 *   - the single bottom-up pivot traversal of Sec. 2.3.2 (steps 1 and 2),
 *     symmetric case of Sec. 5 (P = Q, one ACA per cell);
 *   - the transfer operators as by-products of the ACA (Remark in Sec. 2.3.2,
 *     the nested bases of Sec. 2.3.1);
 *   - the H2 matrix-vector product of Sec. 4 (upward, transverse, downward
 *     passes and the near field);
 *   - the dense direct sum, the plain definition A_ij = K(p_i, p_j);
 *   - the general case P != Q (Sec. 2.1, 2.3): one tree over both sets, the
 *     incoming and the outgoing ACA of every cell, the rectangular product
 *     and its transpose, and the rectangular direct sum.
 *
 * Everything is FP64, sequential inside a cell, with OpenMP only over the
 * independent cells of one tree level.  Floating-point expressions are written
 * without fused multiply-add (build with -ffp-contract=off) so that the order
 * of every rounding is the one written here.
 *
 * parity unpinned: nothing.  Every function below has a pin in tests/.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <stdio.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#include "nnca_oracle.h"

/* ------------------------------------------------------------------------- */
/* Kernel functions                                                           */
/* ------------------------------------------------------------------------- */

/* Natural logarithm from IEEE operations only (project-defined so that the
 * CPU and the GPU evaluate the 2D kernel identically):
 *   x = m 2^e with m in (sqrt(1/2), sqrt(2)];  log m = 2 atanh(s),
 *   s = (m-1)/(m+1);  atanh(s)/s = sum_{n=0}^{12} s^{2n}/(2n+1) by Horner;
 *   log x = e ln2 + 2 s P(s^2).                                              */
double orc_log(double x)
{
    int e;
    double m = frexp(x, &e);          /* x = m 2^e, m in [0.5, 1) */
    m = m * 2.0;                      /* m in [1, 2) */
    e = e - 1;
    if (m > 0x1.6a09e667f3bcdp+0) {   /* m > sqrt(2) */
        m = m * 0.5;
        e = e + 1;
    }
    double s = (m - 1.0) / (m + 1.0);
    double z = s * s;
    double p = 1.0 / 25.0;
    p = p * z + 1.0 / 23.0;
    p = p * z + 1.0 / 21.0;
    p = p * z + 1.0 / 19.0;
    p = p * z + 1.0 / 17.0;
    p = p * z + 1.0 / 15.0;
    p = p * z + 1.0 / 13.0;
    p = p * z + 1.0 / 11.0;
    p = p * z + 1.0 / 9.0;
    p = p * z + 1.0 / 7.0;
    p = p * z + 1.0 / 5.0;
    p = p * z + 1.0 / 3.0;
    p = p * z + 1.0;
    return (double)e * 0x1.62e42fefa39efp-1 + (2.0 * s) * p;
}

/* exp(x) for x <= 0 from IEEE operations only: x = n ln2 + r, |r| <= ln2/2,
 * with ln2 split into a 32-bit head (so n*head is exact) and a tail;
 * exp(r) by the Taylor polynomial of degree 13 in Horner form; scale 2^n.   */
double orc_exp(double x)
{
    if (x < -745.5) return 0.0;
    if (x > 709.0) return INFINITY;
    double n = floor(x * 0x1.71547652b82fep+0 + 0.5);
    double r = (x - n * 0x1.62e42fee00000p-1) - n * 0x1.a39ef35793c76p-33;
    double p = 1.0 / 6227020800.0;            /* 1/13! */
    p = p * r + 1.0 / 479001600.0;            /* 1/12! */
    p = p * r + 1.0 / 39916800.0;
    p = p * r + 1.0 / 3628800.0;
    p = p * r + 1.0 / 362880.0;
    p = p * r + 1.0 / 40320.0;
    p = p * r + 1.0 / 5040.0;
    p = p * r + 1.0 / 720.0;
    p = p * r + 1.0 / 120.0;
    p = p * r + 1.0 / 24.0;
    p = p * r + 1.0 / 6.0;
    p = p * r + 1.0 / 2.0;
    p = p * r + 1.0;
    p = p * r + 1.0;
    return ldexp(p, (int)n);
}

/* Squared distance, written out axis by axis: ((dx dx + dy dy) + dz dz). */
static double dist2(const double *a, const double *b, int d)
{
    double dx = a[0] - b[0];
    double s = dx * dx;
    for (int q = 1; q < d; q++) {
        double dq = a[q] - b[q];
        s = s + dq * dq;
    }
    return s;
}

/* The kernel K(x, y) used inside the method (build and apply).
 * 1/r and log r are set to zero at r = 0 ("zero on the diagonal");
 * the Gaussian exp(-r^2/h^2) and exp(-r/h) are 1 there.  ORC_K_POLY2 = (1 + x.y)^2 is a
 * test kernel of known rank used only to pin the ACA.                       */
static double kern(int kind, double hparam, const double *a, const double *b, int d)
{
    switch (kind) {
    case ORC_K_INV_R: {
        double d2 = dist2(a, b, d);
        return d2 == 0.0 ? 0.0 : 1.0 / sqrt(d2);
    }
    case ORC_K_LOG_R: {
        double d2 = dist2(a, b, d);
        return d2 == 0.0 ? 0.0 : 0.5 * orc_log(d2);
    }
    case ORC_K_GAUSS: {
        double d2 = dist2(a, b, d);
        return orc_exp(-(d2 / (hparam * hparam)));
    }
    case ORC_K_EXP_R: {     /* Exp. 6 ("Matern"): exp(-r/h), 1 at r = 0; hparam = h */
        double d2 = dist2(a, b, d);
        return orc_exp(-(sqrt(d2) / hparam));
    }
    case ORC_K_INV_REG: {   /* Exp. 1-4: r/a for r < a, a/r for r >= a; hparam = a */
        double d2 = dist2(a, b, d);
        if (d2 == 0.0) return 0.0;
        return d2 >= hparam * hparam ? hparam / sqrt(d2) : sqrt(d2) / hparam;
    }
    case ORC_K_LOG_REG: {   /* Exp. 1-2: r (log r - 1)/(a (log a - 1)) for r < a, log r / log a else */
        double d2 = dist2(a, b, d);
        if (d2 == 0.0) return 0.0;
        double la = orc_log(hparam);
        return d2 >= hparam * hparam ? (0.5 * orc_log(d2)) / la
                                     : (sqrt(d2) * (0.5 * orc_log(d2) - 1.0)) / (hparam * (la - 1.0));
    }
    case ORC_K_POLY2: {
        double s = 1.0;
        for (int q = 0; q < d; q++) s = s + a[q] * b[q];
        return s * s;
    }
    }
    return NAN;
}

/* The kernel in its textbook form with the C library's functions; used only
 * by the direct sum, which is the plain definition of A x.                   */
static double kern_ref(int kind, double hparam, const double *a, const double *b, int d)
{
    double d2 = 0.0;
    for (int q = 0; q < d; q++) d2 += (a[q] - b[q]) * (a[q] - b[q]);
    switch (kind) {
    case ORC_K_INV_R: return d2 == 0.0 ? 0.0 : 1.0 / sqrt(d2);
    case ORC_K_LOG_R: return d2 == 0.0 ? 0.0 : log(sqrt(d2));
    case ORC_K_GAUSS: return exp(-d2 / (hparam * hparam));
    case ORC_K_EXP_R: return exp(-sqrt(d2) / hparam);
    case ORC_K_INV_REG: {
        double r = sqrt(d2), a0 = hparam;
        if (r == 0.0) return 0.0;
        return r < a0 ? r / a0 : a0 / r;
    }
    case ORC_K_LOG_REG: {
        double r = sqrt(d2), a0 = hparam;
        if (r == 0.0) return 0.0;
        return r < a0 ? r * (log(r) - 1.0) / (a0 * (log(a0) - 1.0)) : log(r) / log(a0);
    }
    case ORC_K_POLY2: {
        double s = 1.0;
        for (int q = 0; q < d; q++) s += a[q] * b[q];
        return s * s;
    }
    }
    return NAN;
}

double orc_kernel_eval(int kind, double hparam, const double *a, const double *b, int d)
{
    return kern(kind, hparam, a, b, d);
}

/* ------------------------------------------------------------------------- */
/* Direct sum y_i = sum_j K(p_i, p_j) x_j  (Neumaier-compensated, FP64)       */
/* ------------------------------------------------------------------------- */

void orc_direct(const double *pts, int64_t n, int d, int kind, double hparam,
                const double *x, int64_t nrhs, const int64_t *rows, int64_t nrows,
                double *y)
{
    int64_t nr = rows ? nrows : n;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t r = 0; r < nr; r++) {
        int64_t i = rows ? rows[r] : r;
        for (int64_t c = 0; c < nrhs; c++) {
            double sum = 0.0, comp = 0.0;
            for (int64_t j = 0; j < n; j++) {
                double t = kern_ref(kind, hparam, pts + i * d, pts + j * d, d) * x[c * n + j];
                double s2 = sum + t;
                if (fabs(sum) >= fabs(t)) comp += (sum - s2) + t;
                else comp += (t - s2) + sum;
                sum = s2;
            }
            y[c * nr + r] = sum + comp;
        }
    }
}

/* ------------------------------------------------------------------------- */
/* Tree (Sec. 2.1) and lists (Sec. 2.2, Table 1)                              */
/* ------------------------------------------------------------------------- */

typedef struct {
    int64_t ncell;
    uint64_t *key;          /* Morton prefix of the cell, ascending           */
    int64_t *coord;         /* ncell x d integer coordinates at this level    */
    int64_t *first, *count; /* range of sorted positions                      */
    int64_t *parent;        /* cell index one level up (-1 at the root)       */
    int64_t *child_first, *child_count; /* range of cell indices one level down */
    int64_t *nb_ptr, *nb;   /* N(B): same-level non-admissible cells, incl. B */
    int64_t *il_ptr, *il;   /* IL(B): children of N(parent) admissible to B   */
} olevel;

struct orc_tree {
    int d, nu, kmax, kappa;
    int64_t n;
    int64_t split;          /* general case: original indices < split are the
                               targets P, the rest the sources Q; -1 if P = Q */
    int64_t eta_num, eta_den;
    double lo[3], L;
    double *pts;            /* n x d, in sorted order                        */
    int64_t *order;         /* order[pos] = original index of sorted pos     */
    uint64_t *key;          /* Morton key at level kmax, per sorted position */
    olevel *lev;            /* levels 0..kappa                               */
};

typedef struct { uint64_t key; int64_t idx; } keyidx;

static int cmp_keyidx(const void *a, const void *b)
{
    const keyidx *x = (const keyidx *)a, *y = (const keyidx *)b;
    if (x->key < y->key) return -1;
    if (x->key > y->key) return 1;
    return (x->idx < y->idx) ? -1 : (x->idx > y->idx);
}

/* Admissibility of two same-level cells with integer coordinates a, b
 * (Sec. 2.2): max(diam) <= eta dist.  Both cells are cubes of side h, so
 * diam = h sqrt(d) and dist = h sqrt(sum_q g_q^2) with g_q the number of
 * whole cells between them along axis q.  Squared, with eta^2 = num/den:
 *   d * den <= num * sum_q g_q^2   (exact integer test).                   */
static int admissible(const int64_t *a, const int64_t *b, int d, int64_t num, int64_t den)
{
    int64_t s = 0;
    for (int q = 0; q < d; q++) {
        int64_t g = llabs(a[q] - b[q]) - 1;
        if (g < 0) g = 0;
        s += g * g;
    }
    return (int64_t)d * den <= num * s;
}

static uint64_t morton(const int64_t *c, int d, int bits)
{
    uint64_t k = 0;
    for (int b = 0; b < bits; b++)
        for (int q = 0; q < d; q++)
            k |= (uint64_t)((c[q] >> b) & 1) << (d * b + q);
    return k;
}

static int64_t find_cell(const olevel *lv, uint64_t key)
{
    int64_t lo = 0, hi = lv->ncell - 1;
    while (lo <= hi) {
        int64_t mid = (lo + hi) / 2;
        if (lv->key[mid] == key) return mid;
        if (lv->key[mid] < key) lo = mid + 1; else hi = mid - 1;
    }
    return -1;
}

static int cmp_i64(const void *a, const void *b)
{
    int64_t x = *(const int64_t *)a, y = *(const int64_t *)b;
    return (x > y) - (x < y);
}

/* All same-level cells whose offset along each axis is at most R. */
static int64_t box_cells(const orc_tree *T, int l, const int64_t *c, int R, int64_t *out)
{
    int d = T->d;
    int64_t side = (int64_t)1 << l;
    int64_t cnt = 0;
    int64_t off[3] = {-R, -R, -R};
    for (;;) {
        int64_t cc[3];
        int ok = 1;
        for (int q = 0; q < d; q++) {
            cc[q] = c[q] + off[q];
            if (cc[q] < 0 || cc[q] >= side) ok = 0;
        }
        if (ok) {
            int64_t id = find_cell(&T->lev[l], morton(cc, d, l));
            if (id >= 0) out[cnt++] = id;
        }
        int q = 0;
        while (q < d && ++off[q] > R) { off[q] = -R; q++; }
        if (q == d) break;
    }
    return cnt;
}

static orc_tree *tree_build(const double *pts, int64_t n, int d, int leaf_size,
                            int64_t eta_num, int64_t eta_den, int64_t split)
{
    if (n < 1 || (d != 2 && d != 3) || leaf_size < 1 || eta_num < 1 || eta_den < 1) return NULL;
    orc_tree *T = (orc_tree *)calloc(1, sizeof(orc_tree));
    T->d = d; T->n = n; T->nu = leaf_size; T->split = split;
    T->eta_num = eta_num; T->eta_den = eta_den;
    T->kmax = 60 / d;

    /* Domain D (Sec. 2.1): the cube anchored at the per-axis minimum whose
     * side is the largest extent.                                          */
    double hi[3];
    for (int q = 0; q < d; q++) { T->lo[q] = pts[q]; hi[q] = pts[q]; }
    for (int64_t i = 0; i < n; i++)
        for (int q = 0; q < d; q++) {
            if (pts[i * d + q] < T->lo[q]) T->lo[q] = pts[i * d + q];
            if (pts[i * d + q] > hi[q]) hi[q] = pts[i * d + q];
        }
    T->L = 0.0;
    for (int q = 0; q < d; q++) if (hi[q] - T->lo[q] > T->L) T->L = hi[q] - T->lo[q];

    /* Finest integer coordinates and Morton keys. */
    keyidx *ki = (keyidx *)malloc(sizeof(keyidx) * n);
    int64_t side = (int64_t)1 << T->kmax;
    for (int64_t i = 0; i < n; i++) {
        int64_t c[3] = {0, 0, 0};
        if (T->L > 0.0)
            for (int q = 0; q < d; q++) {
                double u = (pts[i * d + q] - T->lo[q]) / T->L;
                int64_t v = (int64_t)floor(u * (double)side);
                c[q] = v < side - 1 ? v : side - 1;
            }
        ki[i].key = morton(c, d, T->kmax);
        ki[i].idx = i;
    }
    qsort(ki, n, sizeof(keyidx), cmp_keyidx);
    T->order = (int64_t *)malloc(sizeof(int64_t) * n);
    T->key = (uint64_t *)malloc(sizeof(uint64_t) * n);
    T->pts = (double *)malloc(sizeof(double) * n * d);
    for (int64_t p = 0; p < n; p++) {
        T->order[p] = ki[p].idx;
        T->key[p] = ki[p].key;
        for (int q = 0; q < d; q++) T->pts[p * d + q] = pts[ki[p].idx * d + q];
    }
    free(ki);

    /* Depth (Sec. 2.1): the first level at which no cell holds more than nu
     * points of P and no more than nu points of Q (capped at kmax; all points
     * identical => a single leaf).  With P = Q the two counts are one.      */
    T->kappa = T->kmax;
    if (T->L == 0.0) T->kappa = 0;
    else
        for (int l = 0; l <= T->kmax; l++) {
            int shift = d * (T->kmax - l);
            int64_t runp = 0, runq = 0, maxrun = 0;
            for (int64_t p = 0; p < n; p++) {
                if (p > 0 && (T->key[p] >> shift) != (T->key[p - 1] >> shift)) runp = runq = 0;
                if (split < 0 || T->order[p] < split) runp++;
                else runq++;
                if (runp > maxrun) maxrun = runp;
                if (runq > maxrun) maxrun = runq;
            }
            if (maxrun <= leaf_size) { T->kappa = l; break; }
        }

    /* Cells of every level: the distinct key prefixes, in ascending order. */
    T->lev = (olevel *)calloc((size_t)(T->kappa >= 0 ? T->kappa + 1 : 1), sizeof(olevel));
    for (int l = 0; l <= T->kappa; l++) {
        olevel *lv = &T->lev[l];
        int shift = d * (T->kmax - l);
        int64_t nc = 0;
        for (int64_t p = 0; p < n; p++)
            if (p == 0 || (T->key[p] >> shift) != (T->key[p - 1] >> shift)) nc++;
        lv->ncell = nc;
        lv->key = (uint64_t *)malloc(sizeof(uint64_t) * nc);
        lv->coord = (int64_t *)malloc(sizeof(int64_t) * nc * d);
        lv->first = (int64_t *)malloc(sizeof(int64_t) * nc);
        lv->count = (int64_t *)calloc(nc, sizeof(int64_t));
        int64_t c = -1;
        for (int64_t p = 0; p < n; p++) {
            if (p == 0 || (T->key[p] >> shift) != (T->key[p - 1] >> shift)) {
                c++;
                lv->key[c] = T->key[p] >> shift;
                lv->first[c] = p;
                /* integer coordinates: de-interleave the prefix */
                for (int q = 0; q < d; q++) {
                    int64_t v = 0;
                    for (int b = 0; b < l; b++) v |= (int64_t)((lv->key[c] >> (d * b + q)) & 1) << b;
                    lv->coord[c * d + q] = v;
                }
            }
            lv->count[c]++;
        }
    }
    /* parent / children links */
    for (int l = 0; l <= T->kappa; l++) {
        olevel *lv = &T->lev[l];
        lv->parent = (int64_t *)malloc(sizeof(int64_t) * lv->ncell);
        lv->child_first = (int64_t *)malloc(sizeof(int64_t) * lv->ncell);
        lv->child_count = (int64_t *)calloc(lv->ncell, sizeof(int64_t));
        for (int64_t c = 0; c < lv->ncell; c++) {
            lv->parent[c] = l == 0 ? -1 : find_cell(&T->lev[l - 1], lv->key[c] >> d);
            lv->child_first[c] = -1;
        }
    }
    for (int l = 1; l <= T->kappa; l++) {
        olevel *lv = &T->lev[l];
        for (int64_t c = 0; c < lv->ncell; c++) {
            olevel *pv = &T->lev[l - 1];
            int64_t p = lv->parent[c];
            if (pv->child_first[p] < 0) pv->child_first[p] = c;
            pv->child_count[p]++;
        }
    }

    /* Neighbours N(B) at every level and interaction lists IL(B).  Cells that
     * are not admissible are at most R cells away along every axis, with
     * R = 1 + ceil(sqrt(d den / num)); every candidate is tested exactly.  */
    int R = 1 + (int)ceil(sqrt((double)d * (double)eta_den / (double)eta_num));
    int64_t boxmax = 1;
    for (int q = 0; q < d; q++) boxmax *= (2 * R + 1);
    int64_t ilmax = boxmax * ((int64_t)1 << d);
    for (int l = 0; l <= T->kappa; l++) {
        olevel *lv = &T->lev[l];
        lv->nb_ptr = (int64_t *)calloc(lv->ncell + 1, sizeof(int64_t));
        lv->il_ptr = (int64_t *)calloc(lv->ncell + 1, sizeof(int64_t));
        int64_t *nbtmp = (int64_t *)malloc(sizeof(int64_t) * lv->ncell * boxmax);
        int64_t *iltmp = (int64_t *)malloc(sizeof(int64_t) * lv->ncell * ilmax);
        int64_t *nbcnt = (int64_t *)calloc(lv->ncell, sizeof(int64_t));
        int64_t *ilcnt = (int64_t *)calloc(lv->ncell, sizeof(int64_t));
#pragma omp parallel for schedule(dynamic, 64)
        for (int64_t c = 0; c < lv->ncell; c++) {
            int64_t *box = (int64_t *)malloc(sizeof(int64_t) * boxmax);
            int64_t nb = box_cells(T, l, lv->coord + c * d, R, box);
            int64_t k = 0;
            for (int64_t e = 0; e < nb; e++)
                if (!admissible(lv->coord + c * d, lv->coord + box[e] * d, d, eta_num, eta_den))
                    nbtmp[c * boxmax + k++] = box[e];
            qsort(nbtmp + c * boxmax, k, sizeof(int64_t), cmp_i64);
            nbcnt[c] = k;
            k = 0;
            if (l >= 1) {
                const olevel *pv = &T->lev[l - 1];
                int64_t p = lv->parent[c];
                int64_t np = box_cells(T, l - 1, pv->coord + p * d, R, box);
                for (int64_t e = 0; e < np; e++) {
                    int64_t pn = box[e];
                    if (admissible(pv->coord + p * d, pv->coord + pn * d, d, eta_num, eta_den)) continue;
                    for (int64_t ch = pv->child_first[pn]; ch < pv->child_first[pn] + pv->child_count[pn]; ch++)
                        if (admissible(lv->coord + c * d, lv->coord + ch * d, d, eta_num, eta_den))
                            iltmp[c * ilmax + k++] = ch;
                }
                qsort(iltmp + c * ilmax, k, sizeof(int64_t), cmp_i64);
            }
            ilcnt[c] = k;
            free(box);
        }
        for (int64_t c = 0; c < lv->ncell; c++) {
            lv->nb_ptr[c + 1] = lv->nb_ptr[c] + nbcnt[c];
            lv->il_ptr[c + 1] = lv->il_ptr[c] + ilcnt[c];
        }
        lv->nb = (int64_t *)malloc(sizeof(int64_t) * (lv->nb_ptr[lv->ncell] + 1));
        lv->il = (int64_t *)malloc(sizeof(int64_t) * (lv->il_ptr[lv->ncell] + 1));
        for (int64_t c = 0; c < lv->ncell; c++) {
            memcpy(lv->nb + lv->nb_ptr[c], nbtmp + c * boxmax, sizeof(int64_t) * nbcnt[c]);
            memcpy(lv->il + lv->il_ptr[c], iltmp + c * ilmax, sizeof(int64_t) * ilcnt[c]);
        }
        free(nbtmp); free(iltmp); free(nbcnt); free(ilcnt);
    }
    return T;
}

orc_tree *orc_tree_build(const double *pts, int64_t n, int d, int leaf_size,
                         int64_t eta_num, int64_t eta_den)
{
    return tree_build(pts, n, d, leaf_size, eta_num, eta_den, -1);
}

/* The tree of the general case (Sec. 2.1): one tree over the union of the
 * targets P (np points) and the sources Q (nq points); a point of the union
 * has original index i < np for p_i and np + j for q_j.                      */
orc_tree *orc_tree_build2(const double *P, int64_t np, const double *Q, int64_t nq, int d, int leaf_size,
                          int64_t eta_num, int64_t eta_den)
{
    if (np < 1 || nq < 1 || (d != 2 && d != 3)) return NULL;
    double *Z = (double *)malloc(sizeof(double) * (np + nq) * d);
    memcpy(Z, P, sizeof(double) * np * d);
    memcpy(Z + np * d, Q, sizeof(double) * nq * d);
    orc_tree *T = tree_build(Z, np + nq, d, leaf_size, eta_num, eta_den, np);
    free(Z);
    return T;
}

void orc_tree_free(orc_tree *T)
{
    if (!T) return;
    for (int l = 0; l <= T->kappa; l++) {
        olevel *lv = &T->lev[l];
        free(lv->key); free(lv->coord); free(lv->first); free(lv->count);
        free(lv->parent); free(lv->child_first); free(lv->child_count);
        free(lv->nb_ptr); free(lv->nb); free(lv->il_ptr); free(lv->il);
    }
    free(T->lev); free(T->pts); free(T->order); free(T->key); free(T);
}

int orc_tree_kappa(const orc_tree *T) { return T->kappa; }
int64_t orc_tree_ncell(const orc_tree *T, int l) { return (l < 0 || l > T->kappa) ? -1 : T->lev[l].ncell; }
void orc_tree_domain(const orc_tree *T, double *lo, double *L)
{
    for (int q = 0; q < T->d; q++) lo[q] = T->lo[q];
    *L = T->L;
}
void orc_tree_order(const orc_tree *T, int64_t *order) { memcpy(order, T->order, sizeof(int64_t) * T->n); }

void orc_tree_cells(const orc_tree *T, int l, uint64_t *key, int64_t *coord, int64_t *first,
                    int64_t *count, int64_t *parent)
{
    const olevel *lv = &T->lev[l];
    if (key) memcpy(key, lv->key, sizeof(uint64_t) * lv->ncell);
    if (coord) memcpy(coord, lv->coord, sizeof(int64_t) * lv->ncell * T->d);
    if (first) memcpy(first, lv->first, sizeof(int64_t) * lv->ncell);
    if (count) memcpy(count, lv->count, sizeof(int64_t) * lv->ncell);
    if (parent) memcpy(parent, lv->parent, sizeof(int64_t) * lv->ncell);
}

/* which = 0: neighbours N(B); which = 1: interaction lists IL(B).
 * With ptr == NULL only the total length is returned.                       */
int64_t orc_tree_lists(const orc_tree *T, int l, int which, int64_t *ptr, int64_t *idx)
{
    const olevel *lv = &T->lev[l];
    const int64_t *p = which ? lv->il_ptr : lv->nb_ptr;
    const int64_t *v = which ? lv->il : lv->nb;
    if (ptr) {
        memcpy(ptr, p, sizeof(int64_t) * (lv->ncell + 1));
        memcpy(idx, v, sizeof(int64_t) * p[lv->ncell]);
    }
    return p[lv->ncell];
}

/* ------------------------------------------------------------------------- */
/* Partially pivoted ACA (Sec. 2.2.1)                                         */
/* ------------------------------------------------------------------------- */

/* Dot product with a fixed summation shape: 256 partial sums (element e goes
 * to partial e mod 256, accumulated in ascending e), then a pairwise tree
 * p[t] += p[t+s] for s = 128, 64, ..., 1.  The shape is part of the method's
 * definition here so that every implementation rounds identically.          */
static double dot256(const double *a, const double *b, int64_t n)
{
    double p[256];
    for (int t = 0; t < 256; t++) p[t] = 0.0;
    for (int64_t e = 0; e < n; e++) p[e % 256] = p[e % 256] + a[e] * b[e];
    for (int s = 128; s >= 1; s /= 2)
        for (int t = 0; t < s; t++) p[t] = p[t] + p[t + s];
    return p[0];
}

/* ACA of the m x n block A(r, c) = K(P[rows[r]], P[cols[c]]) with tolerance
 * tol.  On return: k crosses, rowpos[0..k) and colpos[0..k) (pivot positions
 * in selection order), U (m x kcap, column l at U + l m) holding u_1..u_k.
 * V (kcap x n) is scratch.  kcap = min(m, n).
 *
 * Step k (1-based):
 * With swap = 1 the block is the transpose, A(r, c) = K(P[cols[c]], P[rows[r]]).
 *
 *   1. residual of row i_k:  R(c) = K(i_k, c) - sum_{l<k} u_l(i_k) v_l(c);
 *   2. j_k = argmax over unused columns of |R(c)|, ties to the smallest c;
 *      if that maximum is 0 the row is marked used without a cross and the
 *      smallest unused row is tried next;
 *   3. v_k = R / R(j_k);  entries at used columns are exactly zero;
 *   4. u_k(r) = K(r, j_k) - sum_{l<k} v_l(j_k) u_l(r); exactly zero at rows
 *      already used as pivots;
 *   5. ||A^(k)||_F^2 = (||A^(k-1)||_F^2 + 2 sum_{l<k} (u_k.u_l)(v_l.v_k))
 *                      + ||u_k||^2 ||v_k||^2   (clamped at 0);
 *   6. stop if ||u_k|| ||v_k|| <= tol ||A^(k)||_F (the k-th cross is kept),
 *      or if k = min(m, n);
 *   7. i_{k+1} = argmax over unused rows of |u_k(r)|, ties to the smallest r. */
static int64_t aca_core(const double *P, int d, int kind, double hparam,
                        const int64_t *rows, int64_t m, const int64_t *cols, int64_t n,
                        double tol, int64_t *rowpos, int64_t *colpos, double *U, double *V, int swap)
{
    int64_t kcap = m < n ? m : n;
    char *rused = (char *)calloc(m, 1);
    char *cused = (char *)calloc(n, 1);
    double *R = (double *)malloc(sizeof(double) * (n > 0 ? n : 1));
    double *uu = (double *)malloc(sizeof(double) * (kcap + 1));
    double *vv = (double *)malloc(sizeof(double) * (kcap + 1));
    double nrm2 = 0.0;
    int64_t k = 0, i = 0;
    while (k < kcap) {
        const double *pi = P + rows[i] * d;
        for (int64_t c = 0; c < n; c++) {
            double r = swap ? kern(kind, hparam, P + cols[c] * d, pi, d) : kern(kind, hparam, pi, P + cols[c] * d, d);
            for (int64_t l = 0; l < k; l++) r = r - U[l * m + i] * V[l * n + c];
            R[c] = r;
        }
        int64_t jk = -1;
        double best = 0.0;
        for (int64_t c = 0; c < n; c++)
            if (!cused[c] && fabs(R[c]) > best) { best = fabs(R[c]); jk = c; }
        if (jk < 0) {
            rused[i] = 1;
            i = -1;
            for (int64_t r = 0; r < m; r++) if (!rused[r]) { i = r; break; }
            if (i < 0) break;
            continue;
        }
        double piv = R[jk];
        double *vk = V + k * n;
        for (int64_t c = 0; c < n; c++) vk[c] = cused[c] ? 0.0 : R[c] / piv;
        double *uk = U + k * m;
        const double *pj = P + cols[jk] * d;
        for (int64_t r = 0; r < m; r++) {
            if (rused[r]) { uk[r] = 0.0; continue; }
            double u = swap ? kern(kind, hparam, pj, P + rows[r] * d, d) : kern(kind, hparam, P + rows[r] * d, pj, d);
            for (int64_t l = 0; l < k; l++) u = u - V[l * n + jk] * U[l * m + r];
            uk[r] = u;
        }
        rused[i] = 1;
        cused[jk] = 1;
        rowpos[k] = i;
        colpos[k] = jk;
        double ukk = dot256(uk, uk, m);
        double vkk = dot256(vk, vk, n);
        double s = 0.0;
        for (int64_t l = 0; l < k; l++) {
            uu[l] = dot256(uk, U + l * m, m);
            vv[l] = dot256(V + l * n, vk, n);
            s = s + uu[l] * vv[l];
        }
        nrm2 = (nrm2 + 2.0 * s) + ukk * vkk;
        if (nrm2 < 0.0) nrm2 = 0.0;
        k++;
        if (sqrt(ukk) * sqrt(vkk) <= tol * sqrt(nrm2)) break;
        if (k >= kcap) break;
        i = -1;
        best = -1.0;
        for (int64_t r = 0; r < m; r++)
            if (!rused[r] && fabs(uk[r]) > best) { best = fabs(uk[r]); i = r; }
        if (i < 0) break;
    }
    free(rused); free(cused); free(R); free(uu); free(vv);
    return k;
}

/* Transfer operator from the ACA by-products (Remark in Sec. 2.3.2):
 *   C = A(rows, J) A(I, J)^{-1} = U L^{-1},  L = U(I, :) lower triangular.
 * Rows that are pivots give the identity rows exactly.  For any other row r
 * the equation X L = U(r, :) is solved from the last column to the first:
 *   X(c) = (U(r, c) - sum_{l = c+1}^{k-1} X(l) L(l, c)) / L(c, c).
 * C is m x k, row-major.                                                      */
static void transfer_from_aca(int64_t m, int64_t k, const int64_t *rowpos, const double *U, double *C)
{
    int64_t *pivof = (int64_t *)malloc(sizeof(int64_t) * (m > 0 ? m : 1));
    for (int64_t r = 0; r < m; r++) pivof[r] = -1;
    for (int64_t q = 0; q < k; q++) pivof[rowpos[q]] = q;
    for (int64_t r = 0; r < m; r++) {
        double *x = C + r * k;
        if (pivof[r] >= 0) {
            for (int64_t c = 0; c < k; c++) x[c] = 0.0;
            x[pivof[r]] = 1.0;
            continue;
        }
        for (int64_t c = k - 1; c >= 0; c--) {
            double acc = U[c * m + r];
            for (int64_t l = c + 1; l < k; l++) acc = acc - x[l] * U[c * m + rowpos[l]];
            x[c] = acc / U[c * m + rowpos[c]];
        }
    }
    free(pivof);
}

int64_t orc_aca_block(const double *prow, int64_t m, const double *pcol, int64_t n, int d,
                      int kind, double hparam, double tol,
                      int64_t *rowpos, int64_t *colpos, double *U, double *V, double *C)
{
    double *P = (double *)malloc(sizeof(double) * (m + n) * d + 8);
    int64_t *rows = (int64_t *)malloc(sizeof(int64_t) * (m + 1));
    int64_t *cols = (int64_t *)malloc(sizeof(int64_t) * (n + 1));
    memcpy(P, prow, sizeof(double) * m * d);
    memcpy(P + m * d, pcol, sizeof(double) * n * d);
    for (int64_t r = 0; r < m; r++) rows[r] = r;
    for (int64_t c = 0; c < n; c++) cols[c] = m + c;
    int64_t k = aca_core(P, d, kind, hparam, rows, m, cols, n, tol, rowpos, colpos, U, V, 0);
    if (C) transfer_from_aca(m, k, rowpos, U, C);
    free(P); free(rows); free(cols);
    return k;
}

/* ------------------------------------------------------------------------- */
/* NNCA pivots and operators: bottom-up traversal (Sec. 2.3.2), symmetric     */
/* case (Sec. 5): t^{B,o} := s^{B,i}, s^{B,o} := t^{B,i}, one ACA per cell.   */
/* ------------------------------------------------------------------------- */

typedef struct {
    int done;
    int passthrough;
    int64_t m, n, k;
    int64_t *tt;        /* candidate rows t~^{B,i} (sorted positions), m    */
    int64_t *piv;       /* t^{B,i} (sorted positions), selection order, k   */
    int64_t *rowpos;    /* positions of the pivots inside tt, k             */
    int64_t *colpos;    /* positions of s^{B,i} inside s~^{B,i}, k          */
    int64_t *colpts;    /* s^{B,i} (sorted positions), k                    */
    double *C;          /* m x k transfer operator (U_B or stacked C_{B_c B}) */
} ocell;

struct orc_h2 {
    orc_tree *T;
    int kind;
    double hparam, tol;
    int policy;         /* 0: literal ACA; 1: pass-through when s~ has fewer columns than rows */
    int lmin;           /* coarsest level carrying pivots (kappa+1 if none) */
    ocell **cell;       /* levels 0..kappa */
};

orc_h2 *orc_h2_new(orc_tree *T, int kind, double hparam, double tol, int policy)
{
    orc_h2 *H = (orc_h2 *)calloc(1, sizeof(orc_h2));
    H->T = T; H->kind = kind; H->hparam = hparam; H->tol = tol; H->policy = policy;
    H->cell = (ocell **)calloc(T->kappa + 1, sizeof(ocell *));
    for (int l = 0; l <= T->kappa; l++) H->cell[l] = (ocell *)calloc(T->lev[l].ncell, sizeof(ocell));
    /* Levels coarser than the first one with a non-empty interaction list
     * carry no far field (Table 1; Fig. 1 shows an empty list at level 1).  */
    H->lmin = T->kappa + 1;
    for (int l = 1; l <= T->kappa; l++)
        if (T->lev[l].il_ptr[T->lev[l].ncell] > 0) { H->lmin = l; break; }
    return H;
}

int orc_h2_lmin(const orc_h2 *H) { return H->lmin; }

/* Step 1 and step 2 of Sec. 2.3.2 for one cell; the children and the
 * children of the interaction list must already be done.                    */
static void cell_pivots(orc_h2 *H, int l, int64_t b)
{
    orc_tree *T = H->T;
    const olevel *lv = &T->lev[l];
    ocell *cb = &H->cell[l][b];
    int64_t m = 0, n = 0;
    /* t~^{B,i}: the cell's points at a leaf; else the children's t^{B_c,i}. */
    if (l == T->kappa) {
        m = lv->count[b];
        cb->tt = (int64_t *)malloc(sizeof(int64_t) * (m + 1));
        for (int64_t r = 0; r < m; r++) cb->tt[r] = lv->first[b] + r;
    } else {
        for (int64_t c = lv->child_first[b]; c < lv->child_first[b] + lv->child_count[b]; c++)
            m += H->cell[l + 1][c].k;
        cb->tt = (int64_t *)malloc(sizeof(int64_t) * (m + 1));
        m = 0;
        for (int64_t c = lv->child_first[b]; c < lv->child_first[b] + lv->child_count[b]; c++)
            for (int64_t q = 0; q < H->cell[l + 1][c].k; q++) cb->tt[m++] = H->cell[l + 1][c].piv[q];
    }
    /* s~^{B,i}: points of the interaction list at a leaf; else the pivots
     * s^{B'',o} = t^{B'',i} of the children B'' of every B' in IL(B).       */
    int64_t *ss = NULL;
    for (int pass = 0; pass < 2; pass++) {
        n = 0;
        for (int64_t e = lv->il_ptr[b]; e < lv->il_ptr[b + 1]; e++) {
            int64_t bp = lv->il[e];
            if (l == T->kappa) {
                for (int64_t r = 0; r < lv->count[bp]; r++) {
                    if (pass) ss[n] = lv->first[bp] + r;
                    n++;
                }
            } else {
                for (int64_t c = lv->child_first[bp]; c < lv->child_first[bp] + lv->child_count[bp]; c++)
                    for (int64_t q = 0; q < H->cell[l + 1][c].k; q++) {
                        if (pass) ss[n] = H->cell[l + 1][c].piv[q];
                        n++;
                    }
            }
        }
        if (!pass) ss = (int64_t *)malloc(sizeof(int64_t) * (n + 1));
    }
    cb->m = m;
    cb->n = n;
    if (n == 0 || (H->policy == 1 && n < m)) {
        /* nothing to compress against: every candidate row is kept and the
         * operator is the identity                                          */
        cb->passthrough = 1;
        cb->k = m;
        cb->piv = (int64_t *)malloc(sizeof(int64_t) * (m + 1));
        cb->rowpos = (int64_t *)malloc(sizeof(int64_t) * (m + 1));
        cb->colpos = (int64_t *)malloc(sizeof(int64_t) * 1);
        cb->colpts = (int64_t *)malloc(sizeof(int64_t) * 1);
        cb->C = (double *)calloc(m * m + 1, sizeof(double));
        for (int64_t r = 0; r < m; r++) {
            cb->piv[r] = cb->tt[r];
            cb->rowpos[r] = r;
            cb->C[r * m + r] = 1.0;
        }
    } else {
        int64_t kcap = m < n ? m : n;
        double *U = (double *)malloc(sizeof(double) * m * kcap);
        double *V = (double *)malloc(sizeof(double) * kcap * n);
        int64_t *rp = (int64_t *)malloc(sizeof(int64_t) * kcap);
        int64_t *cp = (int64_t *)malloc(sizeof(int64_t) * kcap);
        int64_t k = aca_core(T->pts, T->d, H->kind, H->hparam, cb->tt, m, ss, n, H->tol, rp, cp, U, V, 0);
        cb->k = k;
        cb->rowpos = rp;
        cb->colpos = cp;
        cb->piv = (int64_t *)malloc(sizeof(int64_t) * (k + 1));
        cb->colpts = (int64_t *)malloc(sizeof(int64_t) * (k + 1));
        for (int64_t q = 0; q < k; q++) {
            cb->piv[q] = cb->tt[rp[q]];
            cb->colpts[q] = ss[cp[q]];
        }
        cb->C = (double *)malloc(sizeof(double) * (m * k + 1));
        transfer_from_aca(m, k, rp, U, cb->C);
        free(U); free(V);
    }
    free(ss);
    cb->done = 1;
}

/* Compute the pivots of the listed cells of level l (and, first, of every
 * cell they depend on), or of all cells at all levels when ncells < 0.      */
int orc_h2_build(orc_h2 *H, int l, const int64_t *cells, int64_t ncells)
{
    orc_tree *T = H->T;
    if (H->lmin > T->kappa) return 0;
    char **need = (char **)calloc(T->kappa + 1, sizeof(char *));
    for (int q = 0; q <= T->kappa; q++) need[q] = (char *)calloc(T->lev[q].ncell + 1, 1);
    if (ncells < 0) {
        for (int q = H->lmin; q <= T->kappa; q++) memset(need[q], 1, T->lev[q].ncell);
    } else {
        if (l < H->lmin || l > T->kappa) goto done;
        for (int64_t e = 0; e < ncells; e++) need[l][cells[e]] = 1;
        for (int q = l; q < T->kappa; q++) {
            const olevel *lv = &T->lev[q];
            for (int64_t b = 0; b < lv->ncell; b++) {
                if (!need[q][b]) continue;
                for (int64_t c = lv->child_first[b]; c < lv->child_first[b] + lv->child_count[b]; c++)
                    need[q + 1][c] = 1;
                for (int64_t e = lv->il_ptr[b]; e < lv->il_ptr[b + 1]; e++) {
                    int64_t bp = lv->il[e];
                    for (int64_t c = lv->child_first[bp]; c < lv->child_first[bp] + lv->child_count[bp]; c++)
                        need[q + 1][c] = 1;
                }
            }
        }
    }
    for (int q = T->kappa; q >= H->lmin; q--) {
        int64_t nc = T->lev[q].ncell;
#pragma omp parallel for schedule(dynamic, 1)
        for (int64_t b = 0; b < nc; b++)
            if (need[q][b] && !H->cell[q][b].done) cell_pivots(H, q, b);
    }
done:
    for (int q = 0; q <= T->kappa; q++) free(need[q]);
    free(need);
    return 0;
}

void orc_h2_free(orc_h2 *H)
{
    if (!H) return;
    for (int l = 0; l <= H->T->kappa; l++) {
        for (int64_t b = 0; b < H->T->lev[l].ncell; b++) {
            ocell *c = &H->cell[l][b];
            free(c->tt); free(c->piv); free(c->rowpos); free(c->colpos); free(c->colpts); free(c->C);
        }
        free(H->cell[l]);
    }
    free(H->cell);
    free(H);
}

/* Per-cell results: m, n, k, passthrough flag; piv (original indices, k),
 * colpts (original indices, k), tt (original indices, m), C (m x k).        */
int orc_h2_cell(const orc_h2 *H, int l, int64_t b, int64_t *mnk, int64_t *piv, int64_t *colpts,
                int64_t *tt, double *C)
{
    const ocell *c = &H->cell[l][b];
    if (!c->done) return -1;
    if (mnk) { mnk[0] = c->m; mnk[1] = c->n; mnk[2] = c->k; mnk[3] = c->passthrough; }
    const int64_t *ord = H->T->order;
    if (piv) for (int64_t q = 0; q < c->k; q++) piv[q] = ord[c->piv[q]];
    if (colpts && !c->passthrough) for (int64_t q = 0; q < c->k; q++) colpts[q] = ord[c->colpts[q]];
    if (tt) for (int64_t q = 0; q < c->m; q++) tt[q] = ord[c->tt[q]];
    if (C) memcpy(C, c->C, sizeof(double) * c->m * c->k);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* H2 matrix-vector product (Sec. 4), symmetric case                          */
/* ------------------------------------------------------------------------- */

/* y = A~ x for nrhs columns (column-major, original point order).
 * For the symmetric kernels of Sec. 5 the transposed product A~^T x runs the
 * same passes with every block transposed; K(x,y) = K(y,x) makes each block
 * its own transpose, so `adjoint` only changes the order of the loops.      */
void orc_h2_matvec(const orc_h2 *H, const double *x, double *y, int64_t nrhs, int adjoint)
{
    const orc_tree *T = H->T;
    int d = T->d;
    int64_t n = T->n;
    int kap = T->kappa;
    double *xs = (double *)malloc(sizeof(double) * n);
    double *ys = (double *)malloc(sizeof(double) * n);
    double **w = (double **)calloc(kap + 1, sizeof(double *));
    double **u = (double **)calloc(kap + 1, sizeof(double *));
    int64_t **off = (int64_t **)calloc(kap + 1, sizeof(int64_t *));
    for (int l = H->lmin; l <= kap; l++) {
        int64_t nc = T->lev[l].ncell;
        off[l] = (int64_t *)malloc(sizeof(int64_t) * (nc + 1));
        off[l][0] = 0;
        for (int64_t b = 0; b < nc; b++) off[l][b + 1] = off[l][b] + H->cell[l][b].k;
        w[l] = (double *)calloc(off[l][nc] + 1, sizeof(double));
        u[l] = (double *)calloc(off[l][nc] + 1, sizeof(double));
    }
    for (int64_t col = 0; col < nrhs; col++) {
        for (int64_t p = 0; p < n; p++) xs[p] = x[col * n + T->order[p]];
        for (int l = H->lmin; l <= kap; l++) {
            memset(w[l], 0, sizeof(double) * (off[l][T->lev[l].ncell] + 1));
            memset(u[l], 0, sizeof(double) * (off[l][T->lev[l].ncell] + 1));
        }
        /* Upward pass: leaf w^{B,o} = V_B^T x^B with V_B = U_B; then
         * w^{B,o} = sum_c T_{B B_c} w^{B_c,o} with T_{B B_c} = C_{B_c B}^T.
         * For the stacked operator C_B (rows = children's pivots in order)
         * this is w^{B,o} = C_B^T [w^{B_1,o}; ...; w^{B_2^d,o}].             */
        for (int l = kap; l >= H->lmin; l--) {
            const olevel *lv = &T->lev[l];
#pragma omp parallel for schedule(dynamic, 16)
            for (int64_t b = 0; b < lv->ncell; b++) {
                const ocell *cb = &H->cell[l][b];
                double *xt = (double *)malloc(sizeof(double) * (cb->m + 1));
                if (l == kap) {
                    for (int64_t r = 0; r < cb->m; r++) xt[r] = xs[cb->tt[r]];
                } else {
                    int64_t r = 0;
                    for (int64_t c = lv->child_first[b]; c < lv->child_first[b] + lv->child_count[b]; c++)
                        for (int64_t q = off[l + 1][c]; q < off[l + 1][c + 1]; q++) xt[r++] = w[l + 1][q];
                }
                double *wb = w[l] + off[l][b];
                for (int64_t q = 0; q < cb->k; q++) {
                    double s = 0.0;
                    for (int64_t r = 0; r < cb->m; r++) s += cb->C[r * cb->k + q] * xt[r];
                    wb[q] = s;
                }
                free(xt);
            }
        }
        /* Transverse pass: u^{B,i} = sum_{B' in IL(B)} S_{B,B'} w^{B',o},
         * S_{B,B'} = A(t^{B,i}, s^{B',o}) = K(t^{B,i}, t^{B',i}).            */
        for (int l = H->lmin; l <= kap; l++) {
            const olevel *lv = &T->lev[l];
#pragma omp parallel for schedule(dynamic, 16)
            for (int64_t b = 0; b < lv->ncell; b++) {
                const ocell *cb = &H->cell[l][b];
                double *ub = u[l] + off[l][b];
                for (int64_t e = lv->il_ptr[b]; e < lv->il_ptr[b + 1]; e++) {
                    int64_t bp = lv->il[e];
                    const ocell *cp = &H->cell[l][bp];
                    const double *wp = w[l] + off[l][bp];
                    for (int64_t i = 0; i < cb->k; i++) {
                        double s = 0.0;
                        for (int64_t j = 0; j < cp->k; j++) {
                            const double *a = T->pts + cb->piv[i] * d, *bb = T->pts + cp->piv[j] * d;
                            double kij = adjoint ? kern(H->kind, H->hparam, bb, a, d)
                                                 : kern(H->kind, H->hparam, a, bb, d);
                            s += kij * wp[j];
                        }
                        ub[i] += s;
                    }
                }
            }
        }
        /* Downward pass: u^{B_c,i} += C_{B_c B} u^{B,i}, i.e. the stacked
         * C_B u^{B,i} split among the children.                             */
        for (int l = H->lmin; l < kap; l++) {
            const olevel *lv = &T->lev[l];
#pragma omp parallel for schedule(dynamic, 16)
            for (int64_t b = 0; b < lv->ncell; b++) {
                const ocell *cb = &H->cell[l][b];
                const double *ub = u[l] + off[l][b];
                int64_t r = 0;
                for (int64_t c = lv->child_first[b]; c < lv->child_first[b] + lv->child_count[b]; c++)
                    for (int64_t q = off[l + 1][c]; q < off[l + 1][c + 1]; q++, r++) {
                        double s = 0.0;
                        for (int64_t j = 0; j < cb->k; j++) s += cb->C[r * cb->k + j] * ub[j];
                        u[l + 1][q] += s;
                    }
            }
        }
        /* Leaves: u^B = U_B u^{B,i} plus the near field
         * sum_{B' in N(B)} A(t^B, s^{B'}) w^{B'}.                            */
        const olevel *lf = &T->lev[kap];
#pragma omp parallel for schedule(dynamic, 16)
        for (int64_t b = 0; b < lf->ncell; b++) {
            for (int64_t r = 0; r < lf->count[b]; r++) {
                int64_t p = lf->first[b] + r;
                double s = 0.0;
                if (kap >= H->lmin) {
                    const ocell *cb = &H->cell[kap][b];
                    const double *ub = u[kap] + off[kap][b];
                    for (int64_t j = 0; j < cb->k; j++) s += cb->C[r * cb->k + j] * ub[j];
                }
                for (int64_t e = lf->nb_ptr[b]; e < lf->nb_ptr[b + 1]; e++) {
                    int64_t bp = lf->nb[e];
                    for (int64_t q = lf->first[bp]; q < lf->first[bp] + lf->count[bp]; q++) {
                        const double *a = T->pts + p * d, *bb = T->pts + q * d;
                        double kij = adjoint ? kern(H->kind, H->hparam, bb, a, d)
                                             : kern(H->kind, H->hparam, a, bb, d);
                        s += kij * xs[q];
                    }
                }
                ys[p] = s;
            }
        }
        for (int64_t p = 0; p < n; p++) y[col * n + T->order[p]] = ys[p];
    }
    for (int l = H->lmin; l <= kap; l++) { free(w[l]); free(u[l]); free(off[l]); }
    free(w); free(u); free(off); free(xs); free(ys);
}

/* Number of kernel interactions one matvec evaluates per right-hand side
 * (Sec. 4: the transverse pass applies S_{B,B'} = K(t^{B,i}, t^{B',i}), a
 * k_B x k_B' block, for every B' in IL(B); the near field a |t^B| x |t^B'|
 * block for every B' in N(B) of a leaf):
 *   out[0] = transverse total, out[1] = near field,
 *   out[2 + l] = transverse pairs of level l for l = 0..kappa (0 above lmin). */
void orc_h2_interactions(const orc_h2 *H, int64_t *out)
{
    const orc_tree *T = H->T;
    out[0] = out[1] = 0;
    for (int l = 0; l <= T->kappa; l++) out[2 + l] = 0;
    for (int l = H->lmin; l <= T->kappa; l++) {
        const olevel *lv = &T->lev[l];
        for (int64_t b = 0; b < lv->ncell; b++)
            for (int64_t e = lv->il_ptr[b]; e < lv->il_ptr[b + 1]; e++)
                out[2 + l] += H->cell[l][b].k * H->cell[l][lv->il[e]].k;
        out[0] += out[2 + l];
    }
    const olevel *lf = &T->lev[T->kappa];
    for (int64_t b = 0; b < lf->ncell; b++)
        for (int64_t e = lf->nb_ptr[b]; e < lf->nb_ptr[b + 1]; e++)
            out[1] += lf->count[b] * lf->count[lf->nb[e]];
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_num_threads(int k)
{
#ifdef _OPENMP
    if (k > 0) omp_set_num_threads(k);
#else
    (void)k;
#endif
}

/* ------------------------------------------------------------------------- */
/* Derivative with respect to the Gaussian length scale, pivots frozen        */
/* ------------------------------------------------------------------------- */
/* For K(r) = exp(-r^2/h^2) every block of the H2 form depends on h.  With the
 * index sets t^{B,i}, s^{B,i} held fixed, an ACA cell's operator is the plain
 * definition  C_B(h) = K_h(t~, J) K_h(I, J)^{-1}  (I = t^{B,i} inside t~,
 * J = s^{B,i}; Remark in Sec. 2.3.2), the M2L blocks are K_h(t^{B,i}, t^{B',i})
 * and the near field is K_h itself (Sec. 4).  Pass-through cells keep the
 * identity.  dK/dh = (2 r^2 / h^3) K.                                        */

/* Gaussian elimination with partial pivoting (row interchanges, the largest
 * |entry| of the column below the diagonal; ties to the first), solving
 * A X = B for k x k row-major A and k x nrhs row-major B in place.
 * Returns -1 on an exactly zero pivot.                                        */
static int solve_gepp(int64_t k, double *A, double *B, int64_t nrhs)
{
    for (int64_t p = 0; p < k; p++) {
        int64_t best = p;
        for (int64_t r = p + 1; r < k; r++)
            if (fabs(A[r * k + p]) > fabs(A[best * k + p])) best = r;
        if (A[best * k + p] == 0.0) return -1;
        if (best != p) {
            for (int64_t c = 0; c < k; c++) {
                double t = A[p * k + c]; A[p * k + c] = A[best * k + c]; A[best * k + c] = t;
            }
            for (int64_t c = 0; c < nrhs; c++) {
                double t = B[p * nrhs + c]; B[p * nrhs + c] = B[best * nrhs + c]; B[best * nrhs + c] = t;
            }
        }
        for (int64_t r = p + 1; r < k; r++) {
            double f = A[r * k + p] / A[p * k + p];
            for (int64_t c = p; c < k; c++) A[r * k + c] -= f * A[p * k + c];
            for (int64_t c = 0; c < nrhs; c++) B[r * nrhs + c] -= f * B[p * nrhs + c];
        }
    }
    for (int64_t p = k - 1; p >= 0; p--)
        for (int64_t c = 0; c < nrhs; c++) {
            double s = B[p * nrhs + c];
            for (int64_t q = p + 1; q < k; q++) s -= A[p * k + q] * B[q * nrhs + c];
            B[p * nrhs + c] = s / A[p * k + p];
        }
    return 0;
}

/* X (m x k, row-major) = R K(I, J)^{-1} for the ACA cell cb at length scale
 * h, R m x k row-major.  Solved as K(I, J)^T X^T = R^T.                     */
static int right_solve_kij(const orc_tree *T, const ocell *cb, double h, const double *R, double *X)
{
    int64_t m = cb->m, k = cb->k;
    int d = T->d;
    double *At = (double *)malloc(sizeof(double) * (k * k + 1));
    double *Bt = (double *)malloc(sizeof(double) * (k * m + 1));
    for (int64_t a = 0; a < k; a++)
        for (int64_t b = 0; b < k; b++)   /* At[b][a] = K(I_a, J_b) */
            At[b * k + a] = kern(ORC_K_GAUSS, h, T->pts + cb->piv[a] * d, T->pts + cb->colpts[b] * d, d);
    for (int64_t r = 0; r < m; r++)
        for (int64_t q = 0; q < k; q++) Bt[q * m + r] = R[r * k + q];
    int rc = solve_gepp(k, At, Bt, m);
    for (int64_t r = 0; r < m; r++)
        for (int64_t q = 0; q < k; q++) X[r * k + q] = Bt[q * m + r];
    free(At); free(Bt);
    return rc;
}

static double dkern_dh(double h, const double *a, const double *b, int d)
{
    double d2 = dist2(a, b, d);
    return (2.0 * d2 / (h * h * h)) * kern(ORC_K_GAUSS, h, a, b, d);
}

/* A copy of H whose operators are re-evaluated at length scale hnew with the
 * pivots of H (Gaussian kernel only).  Shares H's tree.  NULL on a zero pivot. */
orc_h2 *orc_h2_frozen(const orc_h2 *H, double hnew)
{
    const orc_tree *T = H->T;
    if (H->kind != ORC_K_GAUSS) return NULL;
    orc_h2 *F = orc_h2_new(H->T, H->kind, hnew, H->tol, H->policy);
    int bad = 0;
    for (int l = H->lmin; l <= T->kappa; l++) {
        int64_t nc = T->lev[l].ncell;
#pragma omp parallel for schedule(dynamic, 4) reduction(|| : bad)
        for (int64_t b = 0; b < nc; b++) {
            const ocell *s = &H->cell[l][b];
            ocell *c = &F->cell[l][b];
            if (!s->done) continue;
            *c = *s;
            int64_t m = s->m, k = s->k;
            c->tt = (int64_t *)malloc(sizeof(int64_t) * (m + 1));
            c->piv = (int64_t *)malloc(sizeof(int64_t) * (k + 1));
            c->rowpos = (int64_t *)malloc(sizeof(int64_t) * (k + 1));
            c->colpos = (int64_t *)malloc(sizeof(int64_t) * (k + 1));
            c->colpts = (int64_t *)malloc(sizeof(int64_t) * (k + 1));
            c->C = (double *)malloc(sizeof(double) * (m * k + 1));
            memcpy(c->tt, s->tt, sizeof(int64_t) * m);
            memcpy(c->piv, s->piv, sizeof(int64_t) * k);
            memcpy(c->rowpos, s->rowpos, sizeof(int64_t) * k);
            if (!s->passthrough) {
                memcpy(c->colpos, s->colpos, sizeof(int64_t) * k);
                memcpy(c->colpts, s->colpts, sizeof(int64_t) * k);
            }
            if (s->passthrough || k == 0) {
                memcpy(c->C, s->C, sizeof(double) * m * k);
                continue;
            }
            double *R = (double *)malloc(sizeof(double) * (m * k + 1));
            for (int64_t r = 0; r < m; r++)
                for (int64_t q = 0; q < k; q++)
                    R[r * k + q] = kern(ORC_K_GAUSS, hnew, T->pts + s->tt[r] * T->d, T->pts + s->colpts[q] * T->d, T->d);
            if (right_solve_kij(T, s, hnew, R, c->C)) bad = 1;
            free(R);
        }
    }
    if (bad) { orc_h2_free(F); return NULL; }
    return F;
}

/* g^T (dA~/dh) x for one column (original point order), by forward-mode
 * differentiation of each step of the matvec of Sec. 4 with the pivots
 * frozen:
 *   dC_B   = (dK(t~, J) - C_B dK(I, J)) K(I, J)^{-1}      (ACA cells; 0 else)
 *   up:      w = C^T x~,            dw = dC^T x~ + C^T dx~
 *   across:  u = sum K w',          du = sum (dK w' + K dw')
 *   down:    u_c += C u,            du_c += dC u + C du
 *   leaves:  y = C u + N x,         dy = dC u + C du + dN x
 * and the result is g . dy.  `parts` selects terms for tests: bit 0 near
 * field, bit 1 the M2L blocks, bit 2 the transfer operators (7 = all).
 * Returns NaN for a kernel other than the Gaussian or on a zero pivot.       */
double orc_h2_grad_h(const orc_h2 *H, const double *x, const double *g, int parts)
{
    const orc_tree *T = H->T;
    if (H->kind != ORC_K_GAUSS) return NAN;
    const int d = T->d, kap = T->kappa;
    const int64_t n = T->n;
    const double h = H->hparam;
    const int pn = parts & 1, pm = (parts >> 1) & 1, pt = (parts >> 2) & 1;
    double *xs = (double *)malloc(sizeof(double) * (n + 1));
    double *dy = (double *)calloc(n + 1, sizeof(double));
    for (int64_t p = 0; p < n; p++) xs[p] = x[T->order[p]];
    double **w = (double **)calloc(kap + 1, sizeof(double *));
    double **dw = (double **)calloc(kap + 1, sizeof(double *));
    double **u = (double **)calloc(kap + 1, sizeof(double *));
    double **du = (double **)calloc(kap + 1, sizeof(double *));
    double ***dC = (double ***)calloc(kap + 1, sizeof(double **));
    int64_t **off = (int64_t **)calloc(kap + 1, sizeof(int64_t *));
    int bad = 0;
    for (int l = H->lmin; l <= kap; l++) {
        int64_t nc = T->lev[l].ncell;
        off[l] = (int64_t *)malloc(sizeof(int64_t) * (nc + 1));
        off[l][0] = 0;
        for (int64_t b = 0; b < nc; b++) off[l][b + 1] = off[l][b] + H->cell[l][b].k;
        w[l] = (double *)calloc(off[l][nc] + 1, sizeof(double));
        dw[l] = (double *)calloc(off[l][nc] + 1, sizeof(double));
        u[l] = (double *)calloc(off[l][nc] + 1, sizeof(double));
        du[l] = (double *)calloc(off[l][nc] + 1, sizeof(double));
        dC[l] = (double **)calloc(nc, sizeof(double *));
        /* dC_B, dense m x k (all zero for pass-through cells) */
#pragma omp parallel for schedule(dynamic, 4) reduction(|| : bad)
        for (int64_t b = 0; b < nc; b++) {
            const ocell *cb = &H->cell[l][b];
            int64_t m = cb->m, k = cb->k;
            dC[l][b] = (double *)calloc(m * k + 1, sizeof(double));
            if (cb->passthrough || k == 0 || !pt) continue;
            double *R = (double *)malloc(sizeof(double) * (m * k + 1));
            for (int64_t r = 0; r < m; r++)
                for (int64_t q = 0; q < k; q++) {
                    double s = dkern_dh(h, T->pts + cb->tt[r] * d, T->pts + cb->colpts[q] * d, d);
                    for (int64_t a = 0; a < k; a++)
                        s -= cb->C[r * k + a] * dkern_dh(h, T->pts + cb->piv[a] * d, T->pts + cb->colpts[q] * d, d);
                    R[r * k + q] = s;
                }
            if (right_solve_kij(T, cb, h, R, dC[l][b])) bad = 1;
            free(R);
        }
    }
    /* upward pass with its tangent */
    for (int l = kap; l >= H->lmin; l--) {
        const olevel *lv = &T->lev[l];
#pragma omp parallel for schedule(dynamic, 16)
        for (int64_t b = 0; b < lv->ncell; b++) {
            const ocell *cb = &H->cell[l][b];
            double *xt = (double *)calloc(cb->m + 1, sizeof(double));
            double *dxt = (double *)calloc(cb->m + 1, sizeof(double));
            if (l == kap) {
                for (int64_t r = 0; r < cb->m; r++) xt[r] = xs[cb->tt[r]];
            } else {
                int64_t r = 0;
                for (int64_t c = lv->child_first[b]; c < lv->child_first[b] + lv->child_count[b]; c++)
                    for (int64_t q = off[l + 1][c]; q < off[l + 1][c + 1]; q++, r++) {
                        xt[r] = w[l + 1][q];
                        dxt[r] = dw[l + 1][q];
                    }
            }
            for (int64_t q = 0; q < cb->k; q++) {
                double s = 0.0, ds = 0.0;
                for (int64_t r = 0; r < cb->m; r++) {
                    s += cb->C[r * cb->k + q] * xt[r];
                    ds += dC[l][b][r * cb->k + q] * xt[r] + cb->C[r * cb->k + q] * dxt[r];
                }
                w[l][off[l][b] + q] = s;
                dw[l][off[l][b] + q] = ds;
            }
            free(xt); free(dxt);
        }
    }
    /* transverse pass with its tangent */
    for (int l = H->lmin; l <= kap; l++) {
        const olevel *lv = &T->lev[l];
#pragma omp parallel for schedule(dynamic, 16)
        for (int64_t b = 0; b < lv->ncell; b++) {
            const ocell *cb = &H->cell[l][b];
            for (int64_t e = lv->il_ptr[b]; e < lv->il_ptr[b + 1]; e++) {
                int64_t bp = lv->il[e];
                const ocell *cp = &H->cell[l][bp];
                for (int64_t i = 0; i < cb->k; i++) {
                    double s = 0.0, ds = 0.0;
                    for (int64_t j = 0; j < cp->k; j++) {
                        const double *a = T->pts + cb->piv[i] * d, *bb = T->pts + cp->piv[j] * d;
                        double kij = kern(ORC_K_GAUSS, h, a, bb, d);
                        double wj = w[l][off[l][bp] + j], dwj = dw[l][off[l][bp] + j];
                        s += kij * wj;
                        ds += (pm ? dkern_dh(h, a, bb, d) * wj : 0.0) + kij * dwj;
                    }
                    u[l][off[l][b] + i] += s;
                    du[l][off[l][b] + i] += ds;
                }
            }
        }
    }
    /* downward pass with its tangent */
    for (int l = H->lmin; l < kap; l++) {
        const olevel *lv = &T->lev[l];
#pragma omp parallel for schedule(dynamic, 16)
        for (int64_t b = 0; b < lv->ncell; b++) {
            const ocell *cb = &H->cell[l][b];
            const double *ub = u[l] + off[l][b], *dub = du[l] + off[l][b];
            int64_t r = 0;
            for (int64_t c = lv->child_first[b]; c < lv->child_first[b] + lv->child_count[b]; c++)
                for (int64_t q = off[l + 1][c]; q < off[l + 1][c + 1]; q++, r++) {
                    double s = 0.0, ds = 0.0;
                    for (int64_t j = 0; j < cb->k; j++) {
                        s += cb->C[r * cb->k + j] * ub[j];
                        ds += dC[l][b][r * cb->k + j] * ub[j] + cb->C[r * cb->k + j] * dub[j];
                    }
                    u[l + 1][q] += s;
                    du[l + 1][q] += ds;
                }
        }
    }
    /* leaves: far field tangent plus the derivative of the near field */
    const olevel *lf = &T->lev[kap];
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t b = 0; b < lf->ncell; b++) {
        for (int64_t r = 0; r < lf->count[b]; r++) {
            int64_t p = lf->first[b] + r;
            double ds = 0.0;
            if (kap >= H->lmin) {
                const ocell *cb = &H->cell[kap][b];
                const double *ub = u[kap] + off[kap][b], *dub = du[kap] + off[kap][b];
                for (int64_t j = 0; j < cb->k; j++)
                    ds += dC[kap][b][r * cb->k + j] * ub[j] + cb->C[r * cb->k + j] * dub[j];
            }
            if (pn)
                for (int64_t e = lf->nb_ptr[b]; e < lf->nb_ptr[b + 1]; e++) {
                    int64_t bp = lf->nb[e];
                    for (int64_t q = lf->first[bp]; q < lf->first[bp] + lf->count[bp]; q++)
                        ds += dkern_dh(h, T->pts + p * d, T->pts + q * d, d) * xs[q];
                }
            dy[p] = ds;
        }
    }
    double sum = 0.0, comp = 0.0;
    for (int64_t p = 0; p < n; p++) {
        double t = g[T->order[p]] * dy[p];
        double s2 = sum + t;
        if (fabs(sum) >= fabs(t)) comp += (sum - s2) + t;
        else comp += (t - s2) + sum;
        sum = s2;
    }
    for (int l = H->lmin; l <= kap; l++) {
        for (int64_t b = 0; b < T->lev[l].ncell; b++) free(dC[l][b]);
        free(dC[l]); free(w[l]); free(dw[l]); free(u[l]); free(du[l]); free(off[l]);
    }
    free(dC); free(w); free(dw); free(u); free(du); free(off); free(xs); free(dy);
    return bad ? NAN : sum + comp;
}

/* The plain definition of the derivative of the dense form:
 *   g^T (dA/dh) x = sum_ij g_i x_j (2 r_ij^2 / h^3) exp(-r_ij^2 / h^2),
 * C library exp, Neumaier-compensated sums.                                 */
double orc_dense_grad_h(const double *pts, int64_t n, int d, double h, const double *x, const double *g)
{
    double *row = (double *)malloc(sizeof(double) * (n + 1));
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n; i++) {
        double sum = 0.0, comp = 0.0;
        for (int64_t j = 0; j < n; j++) {
            double d2 = 0.0;
            for (int q = 0; q < d; q++) d2 += (pts[i * d + q] - pts[j * d + q]) * (pts[i * d + q] - pts[j * d + q]);
            double t = (2.0 * d2 / (h * h * h)) * exp(-d2 / (h * h)) * x[j];
            double s2 = sum + t;
            if (fabs(sum) >= fabs(t)) comp += (sum - s2) + t;
            else comp += (t - s2) + sum;
            sum = s2;
        }
        row[i] = g[i] * (sum + comp);
    }
    double sum = 0.0, comp = 0.0;
    for (int64_t i = 0; i < n; i++) {
        double t = row[i];
        double s2 = sum + t;
        if (fabs(sum) >= fabs(t)) comp += (sum - s2) + t;
        else comp += (t - s2) + sum;
        sum = s2;
    }
    free(row);
    return sum + comp;
}

/* ------------------------------------------------------------------------- */
/* General case P != Q (Sec. 2.3): two ACAs per cell                          */
/* ------------------------------------------------------------------------- */

/* Every cell carries two halves.  Half 0 (incoming) compresses
 * A(t~^{B,i}, s~^{B,i}): rows are the cell's own targets (a leaf's t^B, else
 * the children's t^{B_c,i}), columns the sources of the interaction-list
 * region (a leaf: s^{B'} for B' in IL(B); else the outgoing pivots s^{B'',o}
 * of the children of every B' in IL(B)).  Its row pivots are t^{B,i}, its
 * column pivots s^{B,i}, and C = U~ L^{-1} is U_B (leaf) or the stacked
 * C_{B_c B} (Sec. 2.3.1).
 *
 * Half 1 (outgoing) compresses A(t~^{B,o}, s~^{B,o}) with rows t~^{B,o} (the
 * targets of the interaction-list region: a leaf's t^{B'}, else the incoming
 * pivots t^{B'',i} of the IL cells' children) and columns s~^{B,o} (a leaf's
 * s^B, else the children's s^{B_c,o}).  The ACA runs on the transposed block,
 * its first pivot taken among the cell's own sources, so that its row pivots
 * are s^{B,o} and its column pivots t^{B,o}; then
 *   C = U~ L^{-1} = A(s~^{B,o}, t^{B,o}) A(s^{B,o}, t^{B,o})^{-1}
 * (entries read as K(p, q)) is the transpose of
 *   A(t^{B,o}, s^{B,o})^{-1} A(t^{B,o}, s~^{B,o}),
 * i.e. V_B at a leaf and the stacked T_{B B_c}^T above (Sec. 2.3.1).  With
 * P = Q and a symmetric kernel the two halves are the same ACA, which is the
 * one-ACA symmetric case of Sec. 5 (t^{B,o} = s^{B,i}, s^{B,o} = t^{B,i}).
 * Pass-through cells (empty far-field candidates, or fewer candidate columns
 * than rows under policy 1) keep every row with the identity operator.      */

struct orc_g2 {
    orc_tree *T;
    int kind;
    double hparam, tol;
    int policy, lmin;
    ocell **half[2];    /* [0] incoming, [1] outgoing; levels 0..kappa       */
};

static int is_target(const orc_tree *T, int64_t pos) { return T->order[pos] < T->split; }

orc_g2 *orc_g2_new(orc_tree *T, int kind, double hparam, double tol, int policy)
{
    if (T->split < 0) return NULL;
    orc_g2 *G = (orc_g2 *)calloc(1, sizeof(orc_g2));
    G->T = T; G->kind = kind; G->hparam = hparam; G->tol = tol; G->policy = policy;
    for (int h = 0; h < 2; h++) {
        G->half[h] = (ocell **)calloc(T->kappa + 1, sizeof(ocell *));
        for (int l = 0; l <= T->kappa; l++) G->half[h][l] = (ocell *)calloc(T->lev[l].ncell, sizeof(ocell));
    }
    G->lmin = T->kappa + 1;
    for (int l = 1; l <= T->kappa; l++)
        if (T->lev[l].il_ptr[T->lev[l].ncell] > 0) { G->lmin = l; break; }
    return G;
}

int orc_g2_lmin(const orc_g2 *G) { return G->lmin; }

/* Positions of a leaf cell's own points of one class: targets for half 0,
 * sources for half 1 (want_target = 1 - h).  With out == NULL only counts.  */
static int64_t class_positions(const orc_tree *T, const olevel *lv, int64_t b, int want_target, int64_t *out)
{
    int64_t k = 0;
    for (int64_t r = 0; r < lv->count[b]; r++) {
        int64_t pos = lv->first[b] + r;
        if (is_target(T, pos) == want_target) {
            if (out) out[k] = pos;
            k++;
        }
    }
    return k;
}

/* Candidates of Sec. 2.3.2 step 1 for half h of cell b at level l. */
static int64_t g2_rows(const orc_g2 *G, int h, int l, int64_t b, int64_t *out)
{
    const orc_tree *T = G->T;
    const olevel *lv = &T->lev[l];
    if (l == T->kappa) return class_positions(T, lv, b, 1 - h, out);
    int64_t m = 0;
    for (int64_t c = lv->child_first[b]; c < lv->child_first[b] + lv->child_count[b]; c++) {
        const ocell *cc = &G->half[h][l + 1][c];
        if (out) memcpy(out + m, cc->piv, sizeof(int64_t) * cc->k);
        m += cc->k;
    }
    return m;
}
static int64_t g2_cols(const orc_g2 *G, int h, int l, int64_t b, int64_t *out)
{
    const orc_tree *T = G->T;
    const olevel *lv = &T->lev[l];
    int64_t n = 0;
    for (int64_t e = lv->il_ptr[b]; e < lv->il_ptr[b + 1]; e++) {
        int64_t bp = lv->il[e];
        if (l == T->kappa) {
            n += class_positions(T, lv, bp, h, out ? out + n : NULL);
        } else {
            /* half 0 takes the IL children's outgoing pivots s^{B'',o},
             * half 1 their incoming pivots t^{B'',i}                        */
            for (int64_t c = lv->child_first[bp]; c < lv->child_first[bp] + lv->child_count[bp]; c++) {
                const ocell *cc = &G->half[1 - h][l + 1][c];
                if (out) memcpy(out + n, cc->piv, sizeof(int64_t) * cc->k);
                n += cc->k;
            }
        }
    }
    return n;
}

static void g2_half_pivots(orc_g2 *G, int h, int l, int64_t b)
{
    orc_tree *T = G->T;
    ocell *cb = &G->half[h][l][b];
    int64_t m = g2_rows(G, h, l, b, NULL);
    int64_t n = g2_cols(G, h, l, b, NULL);
    cb->tt = (int64_t *)malloc(sizeof(int64_t) * (m + 1));
    int64_t *ss = (int64_t *)malloc(sizeof(int64_t) * (n + 1));
    g2_rows(G, h, l, b, cb->tt);
    g2_cols(G, h, l, b, ss);
    cb->m = m;
    cb->n = n;
    if (n == 0 || (G->policy == 1 && n < m)) {
        cb->passthrough = 1;
        cb->k = m;
        cb->piv = (int64_t *)malloc(sizeof(int64_t) * (m + 1));
        cb->rowpos = (int64_t *)malloc(sizeof(int64_t) * (m + 1));
        cb->colpos = (int64_t *)malloc(sizeof(int64_t) * 1);
        cb->colpts = (int64_t *)malloc(sizeof(int64_t) * 1);
        cb->C = (double *)calloc(m * m + 1, sizeof(double));
        for (int64_t r = 0; r < m; r++) {
            cb->piv[r] = cb->tt[r];
            cb->rowpos[r] = r;
            cb->C[r * m + r] = 1.0;
        }
    } else {
        int64_t kcap = m < n ? m : n;
        double *U = (double *)malloc(sizeof(double) * (m * kcap + 1));
        double *V = (double *)malloc(sizeof(double) * (kcap * n + 1));
        int64_t *rp = (int64_t *)malloc(sizeof(int64_t) * (kcap + 1));
        int64_t *cp = (int64_t *)malloc(sizeof(int64_t) * (kcap + 1));
        int64_t k = aca_core(T->pts, T->d, G->kind, G->hparam, cb->tt, m, ss, n, G->tol, rp, cp, U, V, h);
        cb->k = k;
        cb->rowpos = rp;
        cb->colpos = cp;
        cb->piv = (int64_t *)malloc(sizeof(int64_t) * (k + 1));
        cb->colpts = (int64_t *)malloc(sizeof(int64_t) * (k + 1));
        for (int64_t q = 0; q < k; q++) {
            cb->piv[q] = cb->tt[rp[q]];
            cb->colpts[q] = ss[cp[q]];
        }
        cb->C = (double *)malloc(sizeof(double) * (m * k + 1));
        transfer_from_aca(m, k, rp, U, cb->C);
        free(U); free(V);
    }
    free(ss);
    cb->done = 1;
}

/* Both halves of every cell, one reverse level-order traversal (Sec. 2.3.2). */
int orc_g2_build(orc_g2 *G)
{
    orc_tree *T = G->T;
    for (int l = T->kappa; l >= G->lmin; l--) {
        int64_t nc = T->lev[l].ncell;
#pragma omp parallel for schedule(dynamic, 1)
        for (int64_t e = 0; e < 2 * nc; e++) g2_half_pivots(G, (int)(e % 2), l, e / 2);
    }
    return 0;
}

void orc_g2_free(orc_g2 *G)
{
    if (!G) return;
    for (int h = 0; h < 2; h++) {
        for (int l = 0; l <= G->T->kappa; l++) {
            for (int64_t b = 0; b < G->T->lev[l].ncell; b++) {
                ocell *c = &G->half[h][l][b];
                free(c->tt); free(c->piv); free(c->rowpos); free(c->colpos); free(c->colpts); free(c->C);
            }
            free(G->half[h][l]);
        }
        free(G->half[h]);
    }
    free(G);
}

/* Index of a union point inside its own set: p_i -> i, q_j -> j. */
static int64_t own_index(const orc_tree *T, int64_t pos)
{
    int64_t z = T->order[pos];
    return z < T->split ? z : z - T->split;
}

/* Half h of a cell: m, n, k, pass-through flag; piv (k row pivots), colpts
 * (k column pivots), tt (m candidate rows), as indices into P or Q (half 0:
 * piv and tt in P, colpts in Q; half 1 the other way round); C (m x k).      */
int orc_g2_cell(const orc_g2 *G, int h, int l, int64_t b, int64_t *mnk, int64_t *piv, int64_t *colpts,
                int64_t *tt, double *C)
{
    if (h < 0 || h > 1 || l < 0 || l > G->T->kappa || b < 0 || b >= G->T->lev[l].ncell) return -1;
    const ocell *c = &G->half[h][l][b];
    if (!c->done) return -1;
    if (mnk) { mnk[0] = c->m; mnk[1] = c->n; mnk[2] = c->k; mnk[3] = c->passthrough; }
    if (piv) for (int64_t q = 0; q < c->k; q++) piv[q] = own_index(G->T, c->piv[q]);
    if (colpts && !c->passthrough) for (int64_t q = 0; q < c->k; q++) colpts[q] = own_index(G->T, c->colpts[q]);
    if (tt) for (int64_t q = 0; q < c->m; q++) tt[q] = own_index(G->T, c->tt[q]);
    if (C) memcpy(C, c->C, sizeof(double) * c->m * c->k);
    return 0;
}

/* y = A~ x (adjoint = 0: x has nq entries per column, y np) or y = A~^T x
 * (adjoint = 1: x has np entries, y nq), column-major, original order.
 * A~ = sum over admissible pairs of U_X S_{X,Y} V_Y^T plus the near field
 * (Sec. 3-4):
 *   upward    w^{B,o} = V_B^T x^B at a leaf, sum_c T_{B B_c} w^{B_c,o} above;
 *   transverse u^{B,i} = sum_{B' in IL(B)} S_{B,B'} w^{B',o},
 *              S_{B,B'} = A(t^{B,i}, s^{B',o});
 *   downward  u^{B_c,i} += C_{B_c B} u^{B,i};
 *   leaves    y^B = U_B u^{B,i} + sum_{B' in N(B)} A(t^B, s^{B'}) x^{B'}.
 * The transposed product runs the same passes with the halves exchanged:
 * up with U^T and C^T, S^T across, down with T^T and V.                     */
void orc_g2_matvec(const orc_g2 *G, const double *x, double *y, int64_t nrhs, int adjoint)
{
    const orc_tree *T = G->T;
    int d = T->d, kap = T->kappa;
    int64_t n = T->n, np = T->split, nq = T->n - T->split;
    int64_t nin = adjoint ? np : nq, nout = adjoint ? nq : np;
    const int sh = adjoint ? 0 : 1;   /* half gathered on the way up      */
    const int dh = 1 - sh;            /* half scattered on the way down    */
    ocell *const *S = G->half[sh];
    ocell *const *D = G->half[dh];
    double *xs = (double *)calloc(n, sizeof(double));
    double *ys = (double *)calloc(n, sizeof(double));
    double **w = (double **)calloc(kap + 1, sizeof(double *));
    double **u = (double **)calloc(kap + 1, sizeof(double *));
    int64_t **offs = (int64_t **)calloc(kap + 1, sizeof(int64_t *));
    int64_t **offd = (int64_t **)calloc(kap + 1, sizeof(int64_t *));
    for (int l = G->lmin; l <= kap; l++) {
        int64_t nc = T->lev[l].ncell;
        offs[l] = (int64_t *)malloc(sizeof(int64_t) * (nc + 1));
        offd[l] = (int64_t *)malloc(sizeof(int64_t) * (nc + 1));
        offs[l][0] = offd[l][0] = 0;
        for (int64_t b = 0; b < nc; b++) {
            offs[l][b + 1] = offs[l][b] + S[l][b].k;
            offd[l][b + 1] = offd[l][b] + D[l][b].k;
        }
        w[l] = (double *)calloc(offs[l][nc] + 1, sizeof(double));
        u[l] = (double *)calloc(offd[l][nc] + 1, sizeof(double));
    }
    for (int64_t col = 0; col < nrhs; col++) {
        for (int64_t p = 0; p < n; p++) {
            int64_t z = T->order[p];
            int inp = adjoint ? (z < np) : (z >= np);
            xs[p] = inp ? x[col * nin + (adjoint ? z : z - np)] : 0.0;
        }
        for (int l = G->lmin; l <= kap; l++) {
            memset(w[l], 0, sizeof(double) * (offs[l][T->lev[l].ncell] + 1));
            memset(u[l], 0, sizeof(double) * (offd[l][T->lev[l].ncell] + 1));
        }
        /* upward pass with the gathered half's operators (C^T times the
         * stacked input: x at a leaf, the children's w above)               */
        for (int l = kap; l >= G->lmin; l--) {
            const olevel *lv = &T->lev[l];
#pragma omp parallel for schedule(dynamic, 16)
            for (int64_t b = 0; b < lv->ncell; b++) {
                const ocell *cb = &S[l][b];
                double *xt = (double *)malloc(sizeof(double) * (cb->m + 1));
                if (l == kap) {
                    for (int64_t r = 0; r < cb->m; r++) xt[r] = xs[cb->tt[r]];
                } else {
                    int64_t r = 0;
                    for (int64_t c = lv->child_first[b]; c < lv->child_first[b] + lv->child_count[b]; c++)
                        for (int64_t q = offs[l + 1][c]; q < offs[l + 1][c + 1]; q++) xt[r++] = w[l + 1][q];
                }
                double *wb = w[l] + offs[l][b];
                for (int64_t q = 0; q < cb->k; q++) {
                    double s = 0.0;
                    for (int64_t r = 0; r < cb->m; r++) s += cb->C[r * cb->k + q] * xt[r];
                    wb[q] = s;
                }
                free(xt);
            }
        }
        /* transverse pass: K between the scattered half's pivots of B and
         * the gathered half's pivots of B' in IL(B), entries K(p, q)       */
        for (int l = G->lmin; l <= kap; l++) {
            const olevel *lv = &T->lev[l];
#pragma omp parallel for schedule(dynamic, 16)
            for (int64_t b = 0; b < lv->ncell; b++) {
                const ocell *cb = &D[l][b];
                double *ub = u[l] + offd[l][b];
                for (int64_t e = lv->il_ptr[b]; e < lv->il_ptr[b + 1]; e++) {
                    int64_t bp = lv->il[e];
                    const ocell *cp = &S[l][bp];
                    const double *wp = w[l] + offs[l][bp];
                    for (int64_t i = 0; i < cb->k; i++) {
                        double s = 0.0;
                        for (int64_t j = 0; j < cp->k; j++) {
                            const double *a = T->pts + cb->piv[i] * d, *bb = T->pts + cp->piv[j] * d;
                            double kij = adjoint ? kern(G->kind, G->hparam, bb, a, d)
                                                 : kern(G->kind, G->hparam, a, bb, d);
                            s += kij * wp[j];
                        }
                        ub[i] += s;
                    }
                }
            }
        }
        /* downward pass with the scattered half's operators */
        for (int l = G->lmin; l < kap; l++) {
            const olevel *lv = &T->lev[l];
#pragma omp parallel for schedule(dynamic, 16)
            for (int64_t b = 0; b < lv->ncell; b++) {
                const ocell *cb = &D[l][b];
                const double *ub = u[l] + offd[l][b];
                int64_t r = 0;
                for (int64_t c = lv->child_first[b]; c < lv->child_first[b] + lv->child_count[b]; c++)
                    for (int64_t q = offd[l + 1][c]; q < offd[l + 1][c + 1]; q++, r++) {
                        double s = 0.0;
                        for (int64_t j = 0; j < cb->k; j++) s += cb->C[r * cb->k + j] * ub[j];
                        u[l + 1][q] += s;
                    }
            }
        }
        /* leaves: the scattered half's basis times u, plus the near field
         * over the input points of the neighbours                           */
        const olevel *lf = &T->lev[kap];
#pragma omp parallel for schedule(dynamic, 16)
        for (int64_t b = 0; b < lf->ncell; b++) {
            int64_t mo = class_positions(T, lf, b, adjoint ? 0 : 1, NULL);
            int64_t *rows = (int64_t *)malloc(sizeof(int64_t) * (mo + 1));
            class_positions(T, lf, b, adjoint ? 0 : 1, rows);
            for (int64_t r = 0; r < mo; r++) {
                int64_t p = rows[r];
                double s = 0.0;
                if (kap >= G->lmin) {
                    const ocell *cb = &D[kap][b];
                    const double *ub = u[kap] + offd[kap][b];
                    for (int64_t j = 0; j < cb->k; j++) s += cb->C[r * cb->k + j] * ub[j];
                }
                for (int64_t e = lf->nb_ptr[b]; e < lf->nb_ptr[b + 1]; e++) {
                    int64_t bp = lf->nb[e];
                    for (int64_t q = lf->first[bp]; q < lf->first[bp] + lf->count[bp]; q++) {
                        if (is_target(T, q) == !adjoint) continue;   /* only input points */
                        const double *a = T->pts + p * d, *bb = T->pts + q * d;
                        double kij = adjoint ? kern(G->kind, G->hparam, bb, a, d)
                                             : kern(G->kind, G->hparam, a, bb, d);
                        s += kij * xs[q];
                    }
                }
                ys[p] = s;
            }
            free(rows);
        }
        for (int64_t p = 0; p < n; p++) {
            int64_t z = T->order[p];
            int outp = adjoint ? (z >= np) : (z < np);
            if (outp) y[col * nout + (adjoint ? z - np : z)] = ys[p];
        }
    }
    for (int l = G->lmin; l <= kap; l++) { free(w[l]); free(u[l]); free(offs[l]); free(offd[l]); }
    free(w); free(u); free(offs); free(offd); free(xs); free(ys);
}

/* Kernel interactions of one product column: out[0] transverse total
 * (k^{B,i} x k^{B',o} for every B' in IL(B)), out[1] near field
 * (|t^B| x |s^{B'}| for every B' in N(B) of a leaf), out[2 + l] per level.  */
void orc_g2_interactions(const orc_g2 *G, int64_t *out)
{
    const orc_tree *T = G->T;
    out[0] = out[1] = 0;
    for (int l = 0; l <= T->kappa; l++) out[2 + l] = 0;
    for (int l = G->lmin; l <= T->kappa; l++) {
        const olevel *lv = &T->lev[l];
        for (int64_t b = 0; b < lv->ncell; b++)
            for (int64_t e = lv->il_ptr[b]; e < lv->il_ptr[b + 1]; e++)
                out[2 + l] += G->half[0][l][b].k * G->half[1][l][lv->il[e]].k;
        out[0] += out[2 + l];
    }
    const olevel *lf = &T->lev[T->kappa];
    for (int64_t b = 0; b < lf->ncell; b++)
        for (int64_t e = lf->nb_ptr[b]; e < lf->nb_ptr[b + 1]; e++)
            out[1] += class_positions(T, lf, b, 1, NULL) * class_positions(T, lf, lf->nb[e], 0, NULL);
}

/* Dense sum of the general case, y_i = sum_j K(p_i, q_j) x_j, Neumaier-
 * compensated, with the textbook kernel (K = 0 at r = 0 for log and 1/r).   */
void orc_direct2(const double *P, int64_t np, const double *Q, int64_t nq, int d, int kind, double hparam,
                 const double *x, int64_t nrhs, const int64_t *rows, int64_t nrows, double *y)
{
    int64_t nr = rows ? nrows : np;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t r = 0; r < nr; r++) {
        int64_t i = rows ? rows[r] : r;
        for (int64_t c = 0; c < nrhs; c++) {
            double sum = 0.0, comp = 0.0;
            for (int64_t j = 0; j < nq; j++) {
                double t = kern_ref(kind, hparam, P + i * d, Q + j * d, d) * x[c * nq + j];
                double s2 = sum + t;
                if (fabs(sum) >= fabs(t)) comp += (sum - s2) + t;
                else comp += (t - s2) + sum;
                sum = s2;
            }
            y[c * nr + r] = sum + comp;
        }
    }
}
