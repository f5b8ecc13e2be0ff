/*
 * nnca_oracle.h -- declarations of the plain FP64 CPU oracle (test
 * infrastructure only; see nnca_oracle.c).  Points are n x d row-major FP64
 * in the caller's (original) order; every index returned is an original
 * point index unless stated otherwise.
 */
#ifndef NNCA_ORACLE_H
#define NNCA_ORACLE_H
#include <stdint.h>

enum { ORC_K_LOG_R = 1, ORC_K_INV_R = 2, ORC_K_GAUSS = 3, ORC_K_LOG_REG = 4, ORC_K_INV_REG = 5, ORC_K_EXP_R = 6, ORC_K_POLY2 = 99 };

typedef struct orc_tree orc_tree;
typedef struct orc_h2 orc_h2;

double orc_log(double x);
double orc_exp(double x);
double orc_kernel_eval(int kind, double hparam, const double *a, const double *b, int d);

void orc_direct(const double *pts, int64_t n, int d, int kind, double hparam,
                const double *x, int64_t nrhs, const int64_t *rows, int64_t nrows, double *y);

orc_tree *orc_tree_build(const double *pts, int64_t n, int d, int leaf_size,
                         int64_t eta_num, int64_t eta_den);
void orc_tree_free(orc_tree *T);
int orc_tree_kappa(const orc_tree *T);
int64_t orc_tree_ncell(const orc_tree *T, int l);
void orc_tree_domain(const orc_tree *T, double *lo, double *L);
void orc_tree_order(const orc_tree *T, int64_t *order);
void orc_tree_cells(const orc_tree *T, int l, uint64_t *key, int64_t *coord, int64_t *first,
                    int64_t *count, int64_t *parent);
int64_t orc_tree_lists(const orc_tree *T, int l, int which, int64_t *ptr, int64_t *idx);

int64_t orc_aca_block(const double *prow, int64_t m, const double *pcol, int64_t n, int d,
                      int kind, double hparam, double tol,
                      int64_t *rowpos, int64_t *colpos, double *U, double *V, double *C);

orc_h2 *orc_h2_new(orc_tree *T, int kind, double hparam, double tol, int policy);
int orc_h2_lmin(const orc_h2 *H);
int orc_h2_build(orc_h2 *H, int l, const int64_t *cells, int64_t ncells);
void orc_h2_free(orc_h2 *H);
int orc_h2_cell(const orc_h2 *H, int l, int64_t b, int64_t *mnk, int64_t *piv, int64_t *colpts,
                int64_t *tt, double *C);
void orc_h2_matvec(const orc_h2 *H, const double *x, double *y, int64_t nrhs, int adjoint);
void orc_h2_interactions(const orc_h2 *H, int64_t *out);
void orc_set_num_threads(int k);
orc_h2 *orc_h2_frozen(const orc_h2 *H, double hnew);
double orc_h2_grad_h(const orc_h2 *H, const double *x, const double *g, int parts);
double orc_dense_grad_h(const double *pts, int64_t n, int d, double h, const double *x, const double *g);
int orc_num_threads(void);

/* general case P != Q (targets P, sources Q) */
typedef struct orc_g2 orc_g2;
orc_tree *orc_tree_build2(const double *P, int64_t np, const double *Q, int64_t nq, int d, int leaf_size,
                          int64_t eta_num, int64_t eta_den);
orc_g2 *orc_g2_new(orc_tree *T, int kind, double hparam, double tol, int policy);
int orc_g2_lmin(const orc_g2 *G);
int orc_g2_build(orc_g2 *G);
void orc_g2_free(orc_g2 *G);
int orc_g2_cell(const orc_g2 *G, int h, int l, int64_t b, int64_t *mnk, int64_t *piv, int64_t *colpts,
                int64_t *tt, double *C);
void orc_g2_matvec(const orc_g2 *G, const double *x, double *y, int64_t nrhs, int adjoint);
void orc_g2_interactions(const orc_g2 *G, int64_t *out);
void orc_direct2(const double *P, int64_t np, const double *Q, int64_t nq, int d, int kind, double hparam,
                 const double *x, int64_t nrhs, const int64_t *rows, int64_t nrows, double *y);

#endif
