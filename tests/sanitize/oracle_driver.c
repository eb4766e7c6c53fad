/* Runs the oracle end to end on tiny 2D and 3D Kuhn meshes; built with the
 * host address and undefined-behaviour sanitizers by tests/test_oracle_sanitize.py.
 * Exit status 0 when every step returns normally and the four-term matrix has
 * zero row sums to round-off. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../../oracle/oracle.h"

static int run(int dim, int n, int K, int lmax, int form)
{
    const int nv = dim + 1;
    int64_t nn = 1, ncell = 1;
    for (int k = 0; k < dim; ++k) {
        nn *= n + 1;
        ncell *= n;
    }
    const int64_t ne = ncell * (dim == 2 ? 2 : 6);
    double *coords = malloc(sizeof(double) * nn * dim);
    int32_t *conn = malloc(sizeof(int32_t) * ne * nv);
    uint8_t *cst = malloc(nn);
    for (int64_t id = 0; id < nn; ++id) {
        int64_t r = id;
        int interior = 1;
        for (int k = 0; k < dim; ++k) {
            const int64_t i = r % (n + 1);
            r /= n + 1;
            coords[id * dim + k] = (double)i / n;
            if (i < K || i > n - K) interior = 0;
        }
        cst[id] = interior ? 0 : 1;
    }
    static const int perm3[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
    static const int perm2[2][2] = {{0, 1}, {1, 0}};
    int64_t e = 0;
    for (int64_t c = 0; c < ncell; ++c) {
        int idx[3] = {0, 0, 0};
        int64_t r = c;
        for (int k = 0; k < dim; ++k) {
            idx[k] = (int)(r % n);
            r /= n;
        }
        const int np = dim == 2 ? 2 : 6;
        for (int q = 0; q < np; ++q) {
            int cur[3] = {idx[0], idx[1], idx[2]};
            for (int v = 0; v < nv; ++v) {
                if (v > 0) cur[dim == 2 ? perm2[q][v - 1] : perm3[q][v - 1]] += 1;
                int64_t id = 0, stride = 1;
                for (int k = 0; k < dim; ++k) {
                    id += cur[k] * stride;
                    stride *= n + 1;
                }
                conn[e * nv + v] = (int32_t)id;
            }
            ++e;
        }
    }
    or_mesh m = {dim, nn, ne, coords, conn};
    const double h = 1.0 / n, delta = K * h;
    or_params p = {delta, delta / 8, 0.0, 0, 1, lmax, form};
    int64_t *off = malloc(sizeof(int64_t) * (ne + 1));
    const int64_t np = or_pairs(&m, delta + p.eps, 2, off, NULL);
    int32_t *pm = malloc(sizeof(int32_t) * (np > 0 ? np : 1));
    or_pairs(&m, delta + p.eps, 2, off, pm);
    int64_t *rp = malloc(sizeof(int64_t) * (nn + 1));
    const int64_t nnz = or_pattern(&m, off, pm, rp, NULL);
    int32_t *col = malloc(sizeof(int32_t) * nnz);
    or_pattern(&m, off, pm, rp, col);
    double *val = calloc(nnz, sizeof(double));
    int64_t leaves[16] = {0}, evals[2] = {0, 0};
    if (or_assemble(&m, &p, 2, off, pm, 0, NULL, rp, col, val, leaves, evals) != 0) return 1;
    double worst = 0.0;
    for (int64_t i = 0; i < nn && form == 0; ++i) {
        double s = 0.0, a = 0.0;
        for (int64_t q = rp[i]; q < rp[i + 1]; ++q) {
            s += val[q];
            a += fabs(val[q]);
        }
        if (a > 0.0 && fabs(s) / a > worst) worst = fabs(s) / a;
    }
    double *f = malloc(sizeof(double) * nn), *g = malloc(sizeof(double) * nn);
    double *F = calloc(nn, sizeof(double)), *Ft = calloc(nn, sizeof(double));
    double *w = calloc(nn, sizeof(double)), *w2 = calloc(nn, sizeof(double));
    for (int64_t i = 0; i < nn; ++i) {
        f[i] = -2.0;
        g[i] = coords[i * dim] * coords[i * dim];
    }
    or_load(&m, f, cst, F);
    or_lift(nn, rp, col, val, cst, g, F, Ft);
    double relres = 0.0;
    if (form == 0) {
        if (or_cg(nn, rp, col, val, cst, Ft, 1e-12, 10000, w, &relres) < 0) return 2;
        if (or_cholesky_solve(nn, rp, col, val, cst, Ft, w2) != 0) return 3;
    }
    double E[64];
    int64_t lv[16] = {0}, ev[2] = {0, 0};
    if (np > 0 && or_pair_block(&m, &p, 0, pm[off[0]], E, lv, ev) != 0) return 4;
    int64_t rows[2] = {0, nn - 1}, rl[2];
    const int64_t tot = or_rows(&m, &p, delta + p.eps, 2, 2, rows, rl, NULL, NULL);
    int32_t *rc = malloc(sizeof(int32_t) * (tot > 0 ? tot : 1));
    double *rv = malloc(sizeof(double) * (tot > 0 ? tot : 1));
    or_rows(&m, &p, delta + p.eps, 2, 2, rows, rl, rc, rv);
    printf("dim %d n %d K %d lmax %d form %d: pairs %lld nnz %lld evals %lld row-sum %.2e relres %.1e\n", dim, n,
           K, lmax, form, (long long)np, (long long)nnz, (long long)evals[0], worst, relres);
    free(coords); free(conn); free(cst); free(off); free(pm); free(rp); free(col); free(val);
    free(f); free(g); free(F); free(Ft); free(w); free(w2); free(rc); free(rv);
    return worst < 1e-12 ? 0 : 5;
}

int main(void)
{
    int rc = 0;
    rc |= run(2, 6, 2, 3, 0);
    rc |= run(2, 5, 1, 2, 1);
    rc |= run(3, 3, 1, 2, 0);
    return rc;
}
