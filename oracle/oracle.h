/*
 * Plain FP64 CPU oracle for the mollified nonlocal finite-element assembly of
 * Aulisa, Capodaglio, Chierici, D'Elia, "Efficient quadrature rules for finite
 * element discretizations of nonlocal equations" (arXiv 2101.08825).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark load this library.  The GPU library never
 * links, includes or calls it, and it shares no code, header or table with it.
 *
 * Conventions: arrays are row-major and 0-based; element connectivity is int32,
 * counts int64, all physical data double.  Simplices (triangles, tets; P1 or P2
 * Lagrange) and quadrilaterals / hexahedra (Q1 or serendipity, multilinear
 * geometry).
 */
#ifndef NLQ_ORACLE_H
#define NLQ_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int32_t dim;
    int64_t n_nodes;
    int64_t n_elems;
    const double *coords;   /* [n_nodes][dim] */
    const int32_t *conn;    /* [n_elems][nodes per element] */
    int32_t order;          /* 1: P1 (dim+1 vertices); 2: P2 Lagrange, the vertices then the
                               edge midpoints in the order (0,1),(0,2),(1,2) [2D],
                               (0,1),(0,2),(0,3),(1,2),(1,3),(2,3) [3D]; straight sides */
    int32_t shape;          /* 0: simplices; 1: quadrilaterals / hexahedra on [0,1]^N with
                               the corners in tensor order (corner c at (c&1, c>>1&1,
                               c>>2&1)), order 1 = Q1, order 2 = serendipity (then the
                               edge midpoints by position, see or_box_basis) */
} or_mesh;

typedef struct {
    double delta, eps;
    double scale;           /* > 0: kernel constant; 0: the paper's normalisation */
    int32_t kernel;         /* 0: eta = 1; 1: eta = exp(-d^2/delta^2) */
    int32_t lmin, lmax;     /* Algorithm 1 levels, 1 <= lmin <= lmax */
    int32_t form;           /* 0: four-term integrand; 1: 2*(A21 + A22), adaptive outer
                               integral; 2: the same with the adaptive rule on the
                               inner integral (rows of the refined element) */
    int32_t min_l2;         /* 0: the J^ref test with the L_inf box gap of eq. (mindist);
                               1: with the Euclidean box gap (ablation, see or_boxgap_l2);
                               2: the Euclidean gap to the box of the inner element's
                                  quadrature points (ablation, see run_outer) */
} or_params;

double or_xi(double r);
double or_mu(double d, double delta, double eps);
double or_kernel_constant(int32_t dim, int32_t kernel, double delta, double eps);
int32_t or_rule(int32_t dim, double *bary, double *w);
void or_children(int32_t dim, const double *v, double *child);
double or_aprxmax(int32_t dim, const double *lo1, const double *hi1,
                  const double *lo2, const double *hi2);
double or_aprxmin(int32_t dim, const double *lo1, const double *hi1,
                  const double *lo2, const double *hi2);
double or_boxgap_l2(int32_t dim, const double *lo1, const double *hi1,
                    const double *lo2, const double *hi2);
double or_elem_measure(const or_mesh *m, int64_t e);
/* quadrilaterals / hexahedra: the 3^N Gauss-Legendre rule on [0,1]^N (points
 * [nq][dim], weights summing to 1; returns nq), the basis at a reference point
 * (Q1: 2^N values; serendipity: 8 or 20), the 2^N children [2^N][2^N][dim] of a
 * box given by its corners [2^N][dim] */
int32_t or_box_rule(int32_t dim, double *xi, double *w);
void or_box_basis(int32_t dim, int32_t order, const double *xi, double *phi);
void or_box_children(int32_t dim, const double *P, double *child);

int64_t or_pairs(const or_mesh *m, double thr, int32_t nthreads,
                 int64_t *offsets, int32_t *m_out);
int64_t or_pairs_of(const or_mesh *m, double thr, int64_t l, int32_t *m_out);

int64_t or_pattern(const or_mesh *m, const int64_t *pair_off, const int32_t *pair_m,
                   int64_t *row_ptr, int32_t *col);

int32_t or_pair_block(const or_mesh *m, const or_params *p, int64_t l, int64_t mm,
                      double *E, int64_t *leaves, int64_t *evals);

int32_t or_assemble(const or_mesh *m, const or_params *p, int32_t nthreads,
                    const int64_t *pair_off, const int32_t *pair_m,
                    int64_t n_sel, const int64_t *sel,
                    const int64_t *row_ptr, const int32_t *col, double *val,
                    int64_t *leaves, int64_t *evals);

void or_leaf_counts(const or_mesh *m, const or_params *p, int32_t nthreads, int64_t n_sel,
                    const int64_t *sel, int64_t *leaves);
double or_outer_blocks(const or_mesh *m, const or_params *p, int32_t nthreads, int64_t n_sel,
                       const int64_t *sel, int64_t *leaves, int64_t *evals);
int64_t or_rows(const or_mesh *m, const or_params *p, double thr, int32_t nthreads,
                int64_t n_rows, const int64_t *rows,
                int64_t *row_len, int32_t *cols, double *vals);

void or_load(const or_mesh *m, const double *f_nodal, const uint8_t *constrained,
             double *F);
void or_lift(int64_t n, const int64_t *row_ptr, const int32_t *col, const double *val,
             const uint8_t *constrained, const double *g, const double *F, double *Ft);
int32_t or_cg(int64_t n, const int64_t *row_ptr, const int32_t *col, const double *val,
              const uint8_t *constrained, const double *rhs, double rtol, int32_t maxit,
              double *w, double *relres);
int32_t or_lu_solve(int64_t n, const int64_t *row_ptr, const int32_t *col, const double *val,
                    const uint8_t *constrained, const double *rhs, double *w);
int32_t or_cholesky_solve(int64_t n, const int64_t *row_ptr, const int32_t *col,
                          const double *val, const uint8_t *constrained,
                          const double *rhs, double *w);

#ifdef __cplusplus
}
#endif
#endif
