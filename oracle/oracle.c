/*
 * Plain FP64 CPU oracle for the mollified nonlocal finite-element assembly
 * (arXiv 2101.08825).  TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check
 * and the CPU-baseline leg of the benchmark are its only users; the GPU library
 * shares no code with it.
 *
 * The oracle follows the paper step by step, in its order and notation:
 *   - mollifier mu_{delta,eps} and xi                Section 3, eq. (mollifier)
 *   - kernel constants C_{delta,eps}                 Section 6 (constants paragraph)
 *   - element-split stiffness entry with the full
 *     four-term integrand                            Section 4, eq. (Aij-support2)
 *   - the paper's own two-term form 2*A21 + 2*A22    Section 5, Corollary + eqs. J21Nr, J22Nr
 *   - neighbour set J_l and bbox min distance        Section 5, eq. (k_l), Section 5.1 eq. (mindist)
 *   - Algorithm 1 (adaptive outer quadrature)        Section 5, Algorithm 1
 *   - approximate max / min distance                 Section 5.1, eqs. (maxdist), (mindist)
 *   - volume constraint and lifting                  Section 2, eqs. (poisson), (weak-homo)
 *
 * Readings where the paper is garbled (stated again at each use):
 *   R1 the argument of xi is (delta - |x-y|)/eps, so mu is 1 at the inner band
 *      edge and 0 at the outer edge (as printed it is discontinuous there);
 *   R2 the discrete A12 / A21 carry the minus sign of their continuous definitions;
 *   R3 the lifting enters the right-hand side with a minus sign;
 *   R4 kappa = 1 in the constants C_delta.
 *
 * No FMA contraction: build with -ffp-contract=off so that every bbox distance is
 * evaluated as written.
 */
#include "oracle.h"

#include <math.h>
#include <pthread.h>
#include <stdlib.h>
#include <string.h>

#define OR_PI 3.14159265358979323846
#define MAXQ 27   /* quadrature points per element: 27 for the 3x3x3 hexahedron rule */
#define MAXV 8    /* geometric vertices: 8 for a hexahedron */

/* ---------------------------------------------------------------- mollifier */

/* xi(r) = (128 + 315 r - 420 r^3 + 378 r^5 - 180 r^7 + 35 r^9) / 256,
 * Section 3, eq. (mollifier). */
/* The same degree-9 polynomial as printed, (128 + 315 r - 420 r^3 + 378 r^5
 * - 180 r^7 + 35 r^9) / 256, evaluated in factored form so that it keeps its
 * relative accuracy where it is small: xi' = (315/256)(1 - r^2)^4 makes r = -1 a
 * zero of order five, and with s = 1 - |r|
 *   xi(-|r|) = s^5 (1008 - 1680 s + 1080 s^2 - 315 s^3 + 35 s^4) / 256,
 *   xi(|r|)  = 1 - xi(-|r|)   (xi - 1/2 is odd).
 * (Expanded, the printed form cancels to an absolute error of ~1e-16 near
 * r = -1, where xi ~ (1 + r)^5.) */
double or_xi(double r)
{
    double s = 1.0 - fabs(r);
    double s5 = s * s * s * s * s;
    double w = s5 * (1008.0 - 1680.0 * s + 1080.0 * s * s - 315.0 * s * s * s + 35.0 * s * s * s * s) / 256.0;
    return r < 0.0 ? w : 1.0 - w;
}

/* mu_{delta,eps}(d): 1 below delta-eps, xi in the band (reading R1), 0 above
 * delta+eps.  Section 3, eq. (mollifier); band edges inclusive as printed. */
double or_mu(double d, double delta, double eps)
{
    if (d < delta - eps) return 1.0;
    if (d > delta + eps) return 0.0;
    return or_xi((delta - d) / eps);
}

static double eta(int kernel, double d, double delta)
{
    if (kernel == 0) return 1.0;
    return exp(-(d * d) / (delta * delta));
}

/* Gauss-Legendre nodes and weights on [-1,1] by Newton on P_n. */
static void gauss_legendre(int n, double *x, double *w)
{
    for (int i = 0; i < n; ++i) {
        double z = cos(OR_PI * (i + 0.75) / (n + 0.5));
        double dp = 0.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; ++k) {
                double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            dp = n * (z * p1 - p0) / (z * z - 1.0);
            double dz = p1 / dp;
            z -= dz;
            if (fabs(dz) < 1e-16) break;
        }
        {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; ++k) {
                double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            dp = n * (z * p1 - p0) / (z * z - 1.0);
        }
        x[i] = z;
        w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

/* Kernel constant.
 * eta = 1: C_{delta,eps} of Section 6 (constants paragraph), kappa = 1 (R4).
 * Gaussian eta: the constant c with c * omega_N * int_0^{delta+eps}
 * rho^{N+1} eta(rho) mu(rho) drho = N, i.e. L_eps u = Laplacian u for quadratic u
 * (the same normalisation that fixes C_{delta,eps}); the radial integral uses 40
 * Gauss-Legendre points on [0, delta-eps] and 40 on [delta-eps, delta+eps]. */
double or_kernel_constant(int32_t dim, int32_t kernel, double delta, double eps)
{
    if (kernel == 0) {
        double q = eps / delta;
        if (dim == 2) {
            double cd = 4.0 / (OR_PI * pow(delta, 4));
            return cd / (1.0 + (6.0 / 11.0) * q * q + (3.0 / 143.0) * pow(q, 4));
        }
        double cd = 15.0 / (4.0 * OR_PI * pow(delta, 5));
        return cd / (1.0 + (10.0 / 11.0) * q * q + (15.0 / 143.0) * pow(q, 4));
    }
    double gx[40], gw[40];
    gauss_legendre(40, gx, gw);
    double omega = (dim == 2) ? 2.0 * OR_PI : 4.0 * OR_PI;
    double edges[3] = {0.0, delta - eps, delta + eps};
    double integral = 0.0;
    for (int piece = 0; piece < 2; ++piece) {
        double a = edges[piece], b = edges[piece + 1];
        for (int i = 0; i < 40; ++i) {
            double rho = 0.5 * (a + b) + 0.5 * (b - a) * gx[i];
            double wt = 0.5 * (b - a) * gw[i];
            integral += wt * pow(rho, dim + 1) * eta(1, rho, delta) * or_mu(rho, delta, eps);
        }
    }
    return dim / (omega * integral);
}

/* ------------------------------------------------------------ quadrature */

/* Quadrature on the reference simplex, barycentric points, weights summing to 1
 * (they are multiplied by the element measure).
 * Triangles: the 7-point degree-5 rule named in Section 6 ("Dunavant 7-point").
 *   order: centroid; (1-2a, a, a) rotated; (1-2b, b, b) rotated.
 * Tetrahedra: Keast's 15-point degree-5 rule (positive weights).
 *   order: centroid; four points with one coordinate 0 and the rest 1/3;
 *   four with one coordinate 8/11 and the rest 1/11; six with two coordinates
 *   c = (13 - sqrt(91))/52 and two 1/2 - c, pairs (i,j) in lexicographic order. */
int32_t or_rule(int32_t dim, double *bary, double *w)
{
    if (dim == 2) {
        double s15 = sqrt(15.0);
        double a = (6.0 - s15) / 21.0, b = (6.0 + s15) / 21.0;
        double wa = (155.0 - s15) / 1200.0, wb = (155.0 + s15) / 1200.0;
        int q = 0;
        bary[0] = bary[1] = bary[2] = 1.0 / 3.0;
        w[q++] = 9.0 / 40.0;
        for (int k = 0; k < 3; ++k, ++q) {
            for (int j = 0; j < 3; ++j) bary[3 * q + j] = (j == k) ? 1.0 - 2.0 * a : a;
            w[q] = wa;
        }
        for (int k = 0; k < 3; ++k, ++q) {
            for (int j = 0; j < 3; ++j) bary[3 * q + j] = (j == k) ? 1.0 - 2.0 * b : b;
            w[q] = wb;
        }
        return 7;
    }
    const double w0 = 0.1817020685825350548382618;
    const double w1 = 0.03616071428571428571428571;
    const double w2 = 0.06987149451617381646536165;
    const double w3 = 0.06569484936831875607385811;
    double c = (13.0 - sqrt(91.0)) / 52.0, d = 0.5 - c;
    int q = 0;
    for (int j = 0; j < 4; ++j) bary[j] = 0.25;
    w[q++] = w0;
    for (int k = 0; k < 4; ++k, ++q) {
        for (int j = 0; j < 4; ++j) bary[4 * q + j] = (j == k) ? 0.0 : 1.0 / 3.0;
        w[q] = w1;
    }
    for (int k = 0; k < 4; ++k, ++q) {
        for (int j = 0; j < 4; ++j) bary[4 * q + j] = (j == k) ? 8.0 / 11.0 : 1.0 / 11.0;
        w[q] = w2;
    }
    for (int i = 0; i < 4; ++i)
        for (int j = i + 1; j < 4; ++j, ++q) {
            for (int k = 0; k < 4; ++k) bary[4 * q + k] = (k == i || k == j) ? c : d;
            w[q] = w3;
        }
    return 15;
}

/* ------------------------------------------------------------ refinement */

/* Midpoint refinement of a simplex into 2^N children (Section 5: "split E_l
 * into 2^N sub-elements using the midpoint rule").  Triangles: the three corner
 * triangles and the middle one.  Tetrahedra (not specified by the paper, which
 * refines hexahedra): four corner tets and the inner octahedron cut along the
 * m02-m13 diagonal.  Midpoints are (a + b) * 0.5 in FP64.  `ncomp` components
 * per vertex (physical coordinates, or barycentric coordinates w.r.t. the root). */
static const int TRI_CHILD[4][3] = {{0, 3, 4}, {3, 1, 5}, {4, 5, 2}, {3, 4, 5}};
/* points: v0 v1 v2 m01 m02 m12 */
static const int TET_CHILD[8][4] = {{0, 4, 5, 6}, {4, 1, 7, 8}, {5, 7, 2, 9}, {6, 8, 9, 3},
                                    {4, 5, 6, 8}, {4, 5, 7, 8}, {5, 6, 8, 9}, {5, 7, 8, 9}};
/* points: v0 v1 v2 v3 m01 m02 m03 m12 m13 m23 */

static void children_n(int dim, int ncomp, const double *v, double *child)
{
    double pts[10][4];
    int nv = dim + 1;
    for (int i = 0; i < nv; ++i)
        for (int k = 0; k < ncomp; ++k) pts[i][k] = v[i * ncomp + k];
    int np = nv;
    for (int i = 0; i < nv; ++i)
        for (int j = i + 1; j < nv; ++j, ++np)
            for (int k = 0; k < ncomp; ++k) pts[np][k] = (pts[i][k] + pts[j][k]) * 0.5;
    int nchild = 1 << dim;
    for (int c = 0; c < nchild; ++c)
        for (int i = 0; i < nv; ++i) {
            int src = (dim == 2) ? TRI_CHILD[c][i] : TET_CHILD[c][i];
            for (int k = 0; k < ncomp; ++k) child[(c * nv + i) * ncomp + k] = pts[src][k];
        }
}

void or_children(int32_t dim, const double *v, double *child)
{
    children_n(dim, dim, v, child);
}

/* ------------------------------------------------------------ quadrilaterals, hexahedra */

/* Tensor-product elements (Section 4 allows quadrilaterals and hexahedra; Section 6
 * integrates them with the 3x3 and 3x3x3 Gauss-Legendre product rules).  The
 * reference element is [0,1]^N.  Corner c (c = c_0 + 2 c_1 + 4 c_2, "tensor
 * order") sits at the reference point (c_0, c_1, c_2), and the element map is the
 * multilinear interpolation of the corners,
 *   F(xi) = sum_c N_c(xi) P_c,   N_c(xi) = prod_k (c_k ? xi_k : 1 - xi_k).
 * Linear elements (Q1) have the corners as nodes.  Quadratic ones are the
 * serendipity elements (8-node quadrilateral, 20-node hexahedron: the node counts
 * of the paper's Section 6 meshes, 35 -> 93 and 175 -> 605 unknowns): the corners,
 * then the edge midpoints, each node named by its position t in half-units
 * (t_k in {0,1,2}; an edge midpoint has exactly one odd t_k), edge midpoints in
 * increasing t_0 + 3 t_1 + 9 t_2. */

/* 3^N Gauss-Legendre product rule on [0,1]^N: point q = i_0 + 3 i_1 + 9 i_2 at
 * ((1 + z_{i_0})/2, ...), weight prod_k w_{i_k}/2 (the weights sum to 1), with
 * the closed-form 3-point nodes z = -sqrt(3/5), 0, sqrt(3/5) and weights 5/9,
 * 8/9, 5/9 */
static int box_rule(int dim, double *xi, double *w)
{
    const double r = sqrt(3.0 / 5.0);
    const double z[3] = {-r, 0.0, r}, wz[3] = {5.0 / 9.0, 8.0 / 9.0, 5.0 / 9.0};
    int nq = dim == 2 ? 9 : 27;
    for (int q = 0; q < nq; ++q) {
        int i[3] = {q % 3, (q / 3) % 3, q / 9};
        double ww = 1.0;
        for (int k = 0; k < dim; ++k) {
            xi[q * dim + k] = (1.0 + z[i[k]]) / 2.0;
            ww *= wz[i[k]] / 2.0;
        }
        w[q] = ww;
    }
    return nq;
}

int32_t or_box_rule(int32_t dim, double *xi, double *w)
{
    return box_rule(dim, xi, w);
}

/* multilinear weights N_c(xi), products taken over k = 0..N-1 in order */
static void box_corner_weights(int dim, const double *xi, double *N)
{
    for (int c = 0; c < (1 << dim); ++c) {
        double p = 1.0;
        for (int k = 0; k < dim; ++k) p = p * (((c >> k) & 1) ? xi[k] : 1.0 - xi[k]);
        N[c] = p;
    }
}

/* x = F(xi): products N_c(xi) * P_c[k] rounded, then added in corner order */
static void box_map(int dim, const double *P, const double *xi, double *x)
{
    double N[8];
    box_corner_weights(dim, xi, N);
    for (int k = 0; k < dim; ++k) {
        double sum = 0.0;
        for (int c = 0; c < (1 << dim); ++c) sum = sum + N[c] * P[c * dim + k];
        x[k] = sum;
    }
}

/* |det dF/dxi| at xi */
static double box_jacdet(int dim, const double *P, const double *xi)
{
    double J[3][3];
    for (int k = 0; k < dim; ++k)
        for (int i = 0; i < dim; ++i) {
            double sum = 0.0;
            for (int c = 0; c < (1 << dim); ++c) {
                /* d N_c / d xi_i */
                double p = 1.0;
                for (int j = 0; j < dim; ++j) {
                    int cj = (c >> j) & 1;
                    if (j == i) p *= cj ? 1.0 : -1.0;
                    else p *= cj ? xi[j] : 1.0 - xi[j];
                }
                sum += p * P[c * dim + k];
            }
            J[k][i] = sum;
        }
    double det;
    if (dim == 2) {
        det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
    } else {
        det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
              J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
              J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
    }
    return fabs(det);
}

/* node positions in half-units, in node order */
static int box_nodes(int dim, int order, int t[20][3])
{
    int n = 0;
    for (int c = 0; c < (1 << dim); ++c, ++n)
        for (int k = 0; k < 3; ++k) t[n][k] = k < dim ? 2 * ((c >> k) & 1) : 0;
    if (order != 2) return n;
    int n3 = dim == 2 ? 9 : 27;
    for (int q = 0; q < n3; ++q) {
        int tt[3] = {q % 3, (q / 3) % 3, q / 9}, odd = 0;
        for (int k = 0; k < dim; ++k) odd += tt[k] == 1;
        if (odd != 1) continue;
        for (int k = 0; k < 3; ++k) t[n][k] = tt[k];
        ++n;
    }
    return n;
}

/* Basis functions at reference point xi.  Q1: N_c.  Serendipity, with
 * zeta = 2 xi - 1 and the node at p = t - 1 in {-1,0,1}^N:
 *   corner:           prod_k (1 + zeta_k p_k)/2 * (sum_k zeta_k p_k - (N - 1)),
 *   midpoint (p_j=0): (1 - zeta_j^2) prod_{k != j} (1 + zeta_k p_k)/2. */
static void box_basis(int dim, int order, const double *xi, double *phi)
{
    if (order != 2) {
        box_corner_weights(dim, xi, phi);
        return;
    }
    int t[20][3];
    int nb = box_nodes(dim, order, t);
    double zeta[3];
    for (int k = 0; k < dim; ++k) zeta[k] = 2.0 * xi[k] - 1.0;
    for (int a = 0; a < nb; ++a) {
        int j = -1;
        double prod = 1.0, sum = 0.0;
        for (int k = 0; k < dim; ++k) {
            int p = t[a][k] - 1;
            if (p == 0) {
                j = k;
                continue;
            }
            prod *= (1.0 + zeta[k] * p) / 2.0;
            sum += zeta[k] * p;
        }
        phi[a] = j < 0 ? prod * (sum - (dim - 1)) : (1.0 - zeta[j] * zeta[j]) * prod;
    }
}

void or_box_basis(int32_t dim, int32_t order, const double *xi, double *phi)
{
    box_basis(dim, order, xi, phi);
}

/* Midpoint refinement of a quadrilateral or hexahedron into 2^N children
 * (Section 5: "split E_l into 2^N sub-elements using the midpoint rule").  The
 * 3^N lattice Q[t], t in {0,1,2}^N, holds the corners at even t; the other points
 * are formed axis by axis: for k = 0, 1, 2 every point with t_k = 1 and even t_j
 * (j > k) is (Q[t_k = 0] + Q[t_k = 2]) * 0.5, so edge midpoints come first, then
 * face and cell centres as midpoints of earlier midpoints.  Child i (i_k in {0,1})
 * has corner c at Q[i + c]. */
static void box_children(int dim, const double *P, double *child)
{
    double Q[27][3];
    int n3 = dim == 2 ? 9 : 27;
    for (int q = 0; q < n3; ++q) {
        int t[3] = {q % 3, (q / 3) % 3, q / 9}, even = 1;
        for (int k = 0; k < dim; ++k) even = even && t[k] != 1;
        if (!even) continue;
        int c = 0;
        for (int k = 0; k < dim; ++k) c |= (t[k] / 2) << k;
        for (int k = 0; k < dim; ++k) Q[q][k] = P[c * dim + k];
    }
    const int stride[3] = {1, 3, 9};
    for (int ax = 0; ax < dim; ++ax)
        for (int q = 0; q < n3; ++q) {
            int t[3] = {q % 3, (q / 3) % 3, q / 9}, ok = t[ax] == 1;
            for (int j = ax + 1; j < dim; ++j) ok = ok && t[j] != 1;
            if (!ok) continue;
            for (int k = 0; k < dim; ++k)
                Q[q][k] = (Q[q - stride[ax]][k] + Q[q + stride[ax]][k]) * 0.5;
        }
    for (int i = 0; i < (1 << dim); ++i)
        for (int c = 0; c < (1 << dim); ++c) {
            int q = 0;
            for (int k = 0; k < dim; ++k) q += (((i >> k) & 1) + ((c >> k) & 1)) * stride[k];
            for (int k = 0; k < dim; ++k) child[(i * (1 << dim) + c) * dim + k] = Q[q][k];
        }
}

void or_box_children(int32_t dim, const double *P, double *child)
{
    box_children(dim, P, child);
}

/* ------------------------------------------------------------ distances */

/* Section 5.1, eq. (maxdist): sqrt(sum_k max(d1_k^2, d2_k^2)),
 * d1 = x_min - y_max, d2 = y_min - x_max. */
double or_aprxmax(int32_t dim, const double *lo1, const double *hi1,
                  const double *lo2, const double *hi2)
{
    double s = 0.0;
    for (int k = 0; k < dim; ++k) {
        double d1 = lo1[k] - hi2[k];
        double d2 = lo2[k] - hi1[k];
        double a = d1 * d1, b = d2 * d2;
        s = s + (a > b ? a : b);
    }
    return sqrt(s);
}

/* Section 5.1, eq. (mindist): max_k max(0, d1_k, d2_k). */
double or_aprxmin(int32_t dim, const double *lo1, const double *hi1,
                  const double *lo2, const double *hi2)
{
    double r = 0.0;
    for (int k = 0; k < dim; ++k) {
        double d1 = lo1[k] - hi2[k];
        double d2 = lo2[k] - hi1[k];
        if (d1 > r) r = d1;
        if (d2 > r) r = d2;
    }
    return r;
}

/* Euclidean distance of two boxes, sqrt(sum_k max(0, d1_k, d2_k)^2).  Not the
 * paper's test (Section 5.1 uses the L_inf form above): an ablation of Algorithm
 * 1's J^ref test.  Every point of a sub-element lies in its box and every inner
 * point in the inner element's box, so when this distance is at least delta + eps
 * every point pair is beyond the kernel's support and the sub-element would only
 * contribute zeros: dropping it leaves the integrals unchanged, with fewer leaves. */
double or_boxgap_l2(int32_t dim, const double *lo1, const double *hi1,
                    const double *lo2, const double *hi2)
{
    double s = 0.0;
    for (int k = 0; k < dim; ++k) {
        double g = 0.0;
        double d1 = lo1[k] - hi2[k];
        double d2 = lo2[k] - hi1[k];
        if (d1 > g) g = d1;
        if (d2 > g) g = d2;
        s = s + g * g;
    }
    return sqrt(s);
}

static void bbox_of(int dim, int nv, const double *v, double *lo, double *hi)
{
    for (int k = 0; k < dim; ++k) {
        lo[k] = v[k];
        hi[k] = v[k];
    }
    for (int i = 1; i < nv; ++i)
        for (int k = 0; k < dim; ++k) {
            double x = v[i * dim + k];
            if (x < lo[k]) lo[k] = x;
            if (x > hi[k]) hi[k] = x;
        }
}

static int nodes_of(const or_mesh *m);
static double box_jacdet(int dim, const double *P, const double *xi);
static int box_rule(int dim, double *xi, double *w);

/* geometric vertices: a simplex's dim+1, a quadrilateral's or hexahedron's 2^dim
 * corners (the first nodes of the element either way) */
static int geo_vertices(const or_mesh *m)
{
    return m->shape ? 1 << m->dim : m->dim + 1;
}

static void elem_vertices(const or_mesh *m, int64_t e, double *v)
{
    int nv = geo_vertices(m), nb = nodes_of(m);
    for (int i = 0; i < nv; ++i) {
        int64_t node = m->conn[e * nb + i];
        for (int k = 0; k < m->dim; ++k) v[i * m->dim + k] = m->coords[node * m->dim + k];
    }
}

/* |E| = |det J| / N! for a simplex; for a quadrilateral or hexahedron the
 * integral of |det J| of its multilinear map over [0,1]^N by the 3^N Gauss rule
 * (exact: |det J| has degree <= N-1 in each variable) */
double or_elem_measure(const or_mesh *m, int64_t e)
{
    double v[MAXV * 3];
    elem_vertices(m, e, v);
    if (m->shape) {
        double xi[MAXQ * 3], w[MAXQ];
        int nq = box_rule(m->dim, xi, w);
        double s = 0.0;
        for (int q = 0; q < nq; ++q) s += w[q] * box_jacdet(m->dim, v, xi + q * m->dim);
        return s;
    }
    if (m->dim == 2) {
        double ax = v[2] - v[0], ay = v[3] - v[1];
        double bx = v[4] - v[0], by = v[5] - v[1];
        return fabs(ax * by - ay * bx) / 2.0;
    }
    double a[3], b[3], c[3];
    for (int k = 0; k < 3; ++k) {
        a[k] = v[3 + k] - v[k];
        b[k] = v[6 + k] - v[k];
        c[k] = v[9 + k] - v[k];
    }
    double det = a[0] * (b[1] * c[2] - b[2] * c[1]) - a[1] * (b[0] * c[2] - b[2] * c[0]) +
                 a[2] * (b[0] * c[1] - b[1] * c[0]);
    return fabs(det) / 6.0;
}

/* ------------------------------------------------------------ pair list */

typedef struct {
    const or_mesh *m;
    double thr;
    const double *lo, *hi;
    int64_t l0, l1;
    int64_t *counts;
    const int64_t *offsets;
    int32_t *m_out;
} pair_job;

/* J_l = {m : aprx min dist(E_l, E_m) < delta + eps}: the complement of K_l of
 * Section 5, eq. (k_l), with the bbox min distance in place of the L-infinity
 * distance as Section 5.1 states. */
static int64_t pairs_one(const or_mesh *m, const double *lo, const double *hi, double thr,
                         int64_t l, int32_t *out)
{
    int dim = m->dim;
    int64_t cnt = 0;
    for (int64_t e = 0; e < m->n_elems; ++e) {
        double d = or_aprxmin(dim, lo + l * dim, hi + l * dim, lo + e * dim, hi + e * dim);
        if (d < thr) {
            if (out) out[cnt] = (int32_t)e;
            ++cnt;
        }
    }
    return cnt;
}

static void *pair_worker(void *arg)
{
    pair_job *j = (pair_job *)arg;
    for (int64_t l = j->l0; l < j->l1; ++l) {
        if (j->m_out)
            pairs_one(j->m, j->lo, j->hi, j->thr, l, j->m_out + j->offsets[l]);
        else
            j->counts[l] = pairs_one(j->m, j->lo, j->hi, j->thr, l, NULL);
    }
    return NULL;
}

static void all_bboxes(const or_mesh *m, double *lo, double *hi)
{
    double v[MAXV * 3];
    for (int64_t e = 0; e < m->n_elems; ++e) {
        elem_vertices(m, e, v);
        bbox_of(m->dim, geo_vertices(m), v, lo + e * m->dim, hi + e * m->dim);
    }
}

static void run_threads(int nthreads, void *(*fn)(void *), void *jobs, size_t job_size)
{
    pthread_t th[256];
    if (nthreads > 256) nthreads = 256;
    for (int t = 0; t < nthreads; ++t) pthread_create(&th[t], NULL, fn, (char *)jobs + t * job_size);
    for (int t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
}

/* Brute force over all element pairs.  With m_out == NULL the offsets array
 * (n_elems+1) is filled and the pair count returned; otherwise m_out is filled
 * using those offsets (each J_l in ascending m). */
int64_t or_pairs(const or_mesh *m, double thr, int32_t nthreads, int64_t *offsets,
                 int32_t *m_out)
{
    int64_t ne = m->n_elems;
    double *lo = (double *)malloc(sizeof(double) * ne * m->dim);
    double *hi = (double *)malloc(sizeof(double) * ne * m->dim);
    all_bboxes(m, lo, hi);
    if (nthreads < 1) nthreads = 1;
    pair_job jobs[256];
    if (nthreads > 256) nthreads = 256;
    int64_t *counts = NULL;
    if (!m_out) counts = (int64_t *)calloc(ne, sizeof(int64_t));
    for (int t = 0; t < nthreads; ++t) {
        jobs[t].m = m;
        jobs[t].thr = thr;
        jobs[t].lo = lo;
        jobs[t].hi = hi;
        jobs[t].l0 = ne * t / nthreads;
        jobs[t].l1 = ne * (t + 1) / nthreads;
        jobs[t].counts = counts;
        jobs[t].offsets = offsets;
        jobs[t].m_out = m_out;
    }
    run_threads(nthreads, pair_worker, jobs, sizeof(pair_job));
    int64_t total;
    if (!m_out) {
        offsets[0] = 0;
        for (int64_t l = 0; l < ne; ++l) offsets[l + 1] = offsets[l] + counts[l];
        total = offsets[ne];
        free(counts);
    } else {
        total = offsets[ne];
    }
    free(lo);
    free(hi);
    return total;
}

int64_t or_pairs_of(const or_mesh *m, double thr, int64_t l, int32_t *m_out)
{
    int64_t ne = m->n_elems;
    double *lo = (double *)malloc(sizeof(double) * ne * m->dim);
    double *hi = (double *)malloc(sizeof(double) * ne * m->dim);
    all_bboxes(m, lo, hi);
    int64_t c = pairs_one(m, lo, hi, thr, l, m_out);
    free(lo);
    free(hi);
    return c;
}

/* ------------------------------------------------------------ adjacency */

typedef struct {
    int64_t *off;
    int64_t *items;
} adjacency;

static adjacency node_elements(const or_mesh *m)
{
    adjacency a;
    int nv = nodes_of(m);
    a.off = (int64_t *)calloc(m->n_nodes + 1, sizeof(int64_t));
    for (int64_t e = 0; e < m->n_elems; ++e)
        for (int i = 0; i < nv; ++i) a.off[m->conn[e * nv + i] + 1]++;
    for (int64_t n = 0; n < m->n_nodes; ++n) a.off[n + 1] += a.off[n];
    int64_t *fill = (int64_t *)calloc(m->n_nodes, sizeof(int64_t));
    a.items = (int64_t *)malloc(sizeof(int64_t) * (a.off[m->n_nodes] + 1));
    for (int64_t e = 0; e < m->n_elems; ++e)
        for (int i = 0; i < nv; ++i) {
            int64_t n = m->conn[e * nv + i];
            a.items[a.off[n] + fill[n]++] = e;
        }
    free(fill);
    return a;
}

/* transpose of the pair list: for each inner element, its outer elements */
static adjacency pairs_transpose(int64_t ne, const int64_t *off, const int32_t *pm)
{
    adjacency a;
    a.off = (int64_t *)calloc(ne + 1, sizeof(int64_t));
    for (int64_t l = 0; l < ne; ++l)
        for (int64_t p = off[l]; p < off[l + 1]; ++p) a.off[pm[p] + 1]++;
    for (int64_t e = 0; e < ne; ++e) a.off[e + 1] += a.off[e];
    int64_t *fill = (int64_t *)calloc((size_t)(ne > 0 ? ne : 1), sizeof(int64_t));
    a.items = (int64_t *)malloc(sizeof(int64_t) * (a.off[ne] + 1));
    for (int64_t l = 0; l < ne; ++l)
        for (int64_t p = off[l]; p < off[l + 1]; ++p) {
            int64_t e = pm[p];
            a.items[a.off[e] + fill[e]++] = l;
        }
    free(fill);
    return a;
}

static int cmp_i32(const void *a, const void *b)
{
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

/* Column set of row i: every node j that shares a paired (l, m) with i, i.e.
 * i and j both in nodes(l) u nodes(m) -- the entries touched by the integrand
 * of eq. (Aij-support2).  Pairs with i in the outer element come from J_e for
 * e containing i, pairs with i in the inner element from the transposed list. */
static int64_t row_columns(const or_mesh *m, const adjacency *ne_adj, const int64_t *off,
                           const int32_t *pm, const adjacency *tr, int64_t i, int32_t *mark,
                           int32_t *buf)
{
    int nv = nodes_of(m);
    int64_t cnt = 0;
#define ADD_ELEM_NODES(E_)                                   \
    do {                                                     \
        for (int q_ = 0; q_ < nv; ++q_) {                    \
            int32_t j_ = m->conn[(E_) * nv + q_];            \
            if (mark[j_] != (int32_t)i) {                    \
                mark[j_] = (int32_t)i;                       \
                buf[cnt++] = j_;                             \
            }                                                \
        }                                                    \
    } while (0)
    for (int64_t t = ne_adj->off[i]; t < ne_adj->off[i + 1]; ++t) {
        int64_t e = ne_adj->items[t];
        ADD_ELEM_NODES(e);
        for (int64_t p = off[e]; p < off[e + 1]; ++p) ADD_ELEM_NODES((int64_t)pm[p]);
        for (int64_t p = tr->off[e]; p < tr->off[e + 1]; ++p) ADD_ELEM_NODES(tr->items[p]);
    }
#undef ADD_ELEM_NODES
    qsort(buf, (size_t)cnt, sizeof(int32_t), cmp_i32);
    return cnt;
}

/* Structural CSR pattern of the stiffness matrix (all rows, including the
 * constrained ones).  col == NULL: fill row_ptr and return nnz. */
int64_t or_pattern(const or_mesh *m, const int64_t *pair_off, const int32_t *pair_m,
                   int64_t *row_ptr, int32_t *col)
{
    adjacency na = node_elements(m);
    adjacency tr = pairs_transpose(m->n_elems, pair_off, pair_m);
    int32_t *mark = (int32_t *)malloc(sizeof(int32_t) * m->n_nodes);
    for (int64_t n = 0; n < m->n_nodes; ++n) mark[n] = -1;
    int32_t *buf = (int32_t *)malloc(sizeof(int32_t) * m->n_nodes);
    if (!col) row_ptr[0] = 0;
    for (int64_t i = 0; i < m->n_nodes; ++i) {
        int64_t c = row_columns(m, &na, pair_off, pair_m, &tr, i, mark, buf);
        if (!col)
            row_ptr[i + 1] = row_ptr[i] + c;
        else
            memcpy(col + row_ptr[i], buf, sizeof(int32_t) * c);
    }
    int64_t nnz = row_ptr[m->n_nodes];
    free(mark);
    free(buf);
    free(na.off);
    free(na.items);
    free(tr.off);
    free(tr.items);
    return nnz;
}

/* ------------------------------------------------------------ Algorithm 1 */

typedef struct {
    const or_mesh *mesh;
    const or_params *p;
    int dim, nv, nq;
    int nb;              /* nodes per element (the basis functions of one element) */
    int shape;           /* 0: simplices; 1: quadrilaterals / hexahedra */
    double bary[MAXQ * MAXV], w[MAXQ];   /* simplices: barycentric points; boxes: the
                                            reference points xi in [0,1]^N */
    double P_l[MAXV * 3];                /* boxes: the corners of the root element l */
    double C, dme, dpe;
    int64_t l;
    double meas_l;
    const int32_t *J;    /* inner element ids, indexed by position */
    double *E;           /* per position: (2nv)^2 extended block */
    double *jlo, *jhi;   /* bounding boxes of the inner elements, by position */
    double *qlo, *qhi;   /* boxes the J^ref test measures the gap to (min_l2 = 2:
                            those of the inner quadrature points; else jlo, jhi) */
    int64_t *leaves;     /* per level */
    int64_t evals[2];    /* all kernel evaluations, evaluations inside the band */
    int count_only;      /* 1: Integration() only counts its (sub-element, m) leaves */
} alg_ctx;

/* nodes per element: P1 the dim+1 vertices, P2 also the edge midpoints; Q1 the
 * 2^dim corners, serendipity also the edge midpoints (8 and 20) */
static int nodes_of(const or_mesh *m)
{
    if (m->shape) return m->order == 2 ? (m->dim == 2 ? 8 : 20) : 1 << m->dim;
    return m->order == 2 ? (m->dim + 1) * (m->dim + 2) / 2 : m->dim + 1;
}

/* Lagrange basis of the element at barycentric coordinates lam (nv = dim+1):
 * P1 lam_i; P2 lam_i (2 lam_i - 1) at the vertices and 4 lam_i lam_j at the edge
 * midpoints, edges (i < j) in lexicographic order. */
static void basis(int order, int nv, const double *lam, double *phi)
{
    if (order != 2) {
        for (int i = 0; i < nv; ++i) phi[i] = lam[i];
        return;
    }
    for (int i = 0; i < nv; ++i) phi[i] = lam[i] * (2.0 * lam[i] - 1.0);
    int k = nv;
    for (int i = 0; i < nv; ++i)
        for (int j = i + 1; j < nv; ++j) phi[k++] = 4.0 * lam[i] * lam[j];
}

#define MAXB 20   /* nodes per element, 20-node hexahedron */

/* The double Gauss loop over outer points (x_a, weight Wa_a, basis values phx_a)
 * and inner points (y_b, Wb_b, phy_b) of one (sub-element, m) leaf, added to
 * the pair's extended block E.  With z = [phi^l(x_a); -phi^m(y_b)] the
 * four-term integrand (phi_i(x)-phi_i(y))(phi_j(x)-phi_j(y)) of eq.
 * (Aij-support2) is g z z^T in the extended index space [nodes(l), nodes(m)];
 * the two-term form is 2 A21 + 2 A22 (Corollary), whose rows are those of the
 * inner test function (reading R2 restores A21's minus sign); form 2 puts the
 * rows on the outer element (see integration()). */
static void point_pairs(alg_ctx *c, double *E, int nq, double (*x)[3], const double *Wa,
                        double (*phx)[MAXB], double (*y)[3], const double *Wb, double (*phy)[MAXB])
{
    int dim = c->dim, nb = c->nb, ne2 = 2 * nb;
    for (int a = 0; a < nq; ++a) {
        for (int b = 0; b < nq; ++b) {
            double d2 = 0.0;
            for (int k = 0; k < dim; ++k) d2 += (x[a][k] - y[b][k]) * (x[a][k] - y[b][k]);
            double d = sqrt(d2);
            double g = c->C * eta(c->p->kernel, d, c->p->delta) *
                       or_mu(d, c->p->delta, c->p->eps) * Wa[a] * Wb[b];
            c->evals[0]++;
            if (d >= c->dme && d <= c->dpe) c->evals[1]++;
            double z[2 * MAXB];
            for (int i = 0; i < nb; ++i) {
                z[i] = phx[a][i];
                z[nb + i] = -phy[b][i];
            }
            if (c->p->form == 0) {
                for (int P = 0; P < ne2; ++P)
                    for (int Q = 0; Q < ne2; ++Q) E[P * ne2 + Q] += g * z[P] * z[Q];
            } else if (c->p->form == 1) {
                for (int bb = 0; bb < nb; ++bb)
                    for (int Q = 0; Q < ne2; ++Q)
                        E[(nb + bb) * ne2 + Q] += 2.0 * g * phy[b][bb] * (-z[Q]);
            } else {
                for (int aa = 0; aa < nb; ++aa)
                    for (int Q = 0; Q < ne2; ++Q) E[aa * ne2 + Q] += 2.0 * g * phx[a][aa] * z[Q];
            }
        }
    }
}

/* Integration(E_s, J'): the double Gauss loop of eqs. (J21Nr)/(J22Nr) over the
 * outer sub-element s (level `level`) and every whole inner element m in J'.
 * The outer weights are w_a |E_l| 2^{-N(level-1)} (midpoint children have equal
 * measure); the inner weights w_b |E_m|.  With z = [phi^l(x_a); -phi^m(y_b)] the
 * four-term integrand (phi_i(x)-phi_i(y))(phi_j(x)-phi_j(y)) of eq.
 * (Aij-support2) is g z z^T in the extended index space [nodes(l), nodes(m)];
 * the two-term form is 2 A21 + 2 A22 (Corollary), whose rows are those of the
 * inner test function (reading R2 restores A21's minus sign).
 * Form 2 is the same two-term formula with the adaptive rule on the INNER
 * integral instead (Section 5: the choice of the adaptive side is empirical):
 * the test function's element is the refined one and the other element gets
 * its Gauss rule.  Here every element is refined against its J_l, so form 2
 * puts the rows on the refined (outer) element l: 2 g phi^l_i(x) (phi_Q(x) -
 * phi_Q(y)).  Summed over the pair list, which holds (l, m) and (m, l) alike,
 * this is the assembly with the inner integral adaptive and the outer one by
 * Gauss rule, relabelled. */
static void integration(alg_ctx *c, int level, const double *V, const double *Lam,
                        const int *Jpos, int nJ)
{
    if (c->count_only) {
        c->leaves[level] += nJ;
        return;
    }
    int dim = c->dim, nv = c->nv, nq = c->nq, nb = c->nb, ne2 = 2 * nb;
    double ws = ldexp(c->meas_l, -dim * (level - 1));
    double x[MAXQ][3], lam[MAXQ][MAXV], phx[MAXQ][MAXB], phy[MAXQ][MAXB], Wa[MAXQ];
    for (int a = 0; a < nq; ++a) {
        for (int k = 0; k < dim; ++k) {
            double s = 0.0;
            for (int v = 0; v < nv; ++v) s += c->bary[a * nv + v] * V[v * dim + k];
            x[a][k] = s;
        }
        for (int i = 0; i < nv; ++i) {
            double s = 0.0;
            for (int v = 0; v < nv; ++v) s += c->bary[a * nv + v] * Lam[v * nv + i];
            lam[a][i] = s;
        }
        basis(c->mesh->order, nv, lam[a], phx[a]);
        basis(c->mesh->order, nv, c->bary + a * nv, phy[a]);
        Wa[a] = c->w[a] * ws;
    }
    for (int t = 0; t < nJ; ++t) {
        int pos = Jpos[t];
        int64_t mm = c->J[pos];
        double Vm[MAXV * 3];
        elem_vertices(c->mesh, mm, Vm);
        double meas_m = or_elem_measure(c->mesh, mm);
        double y[MAXQ][3], Wb[MAXQ];
        for (int b = 0; b < nq; ++b) {
            for (int k = 0; k < dim; ++k) {
                double s = 0.0;
                for (int v = 0; v < nv; ++v) s += c->bary[b * nv + v] * Vm[v * dim + k];
                y[b][k] = s;
            }
            Wb[b] = c->w[b] * meas_m;
        }
        point_pairs(c, c->E + (size_t)pos * ne2 * ne2, nq, x, Wa, phx, y, Wb, phy);
        c->leaves[level]++;
    }
}

/* Integration(E_s, J') for quadrilaterals and hexahedra: the sub-element s of
 * level `level` is the reference box xi0 + [0, h]^N, h = 2^{1-level}, of the root
 * element l.  Its points are the images F_l(xi0 + h g_a) of the 3^N Gauss points
 * g_a, with weights w_a h^N |det F_l'| there (the composite rule mapped by l's
 * multilinear map), and l's basis is evaluated at xi0 + h g_a.  Inner element m:
 * y_b = F_m(g_b), weights w_b |det F_m'(g_b)|. */
static void integration_box(alg_ctx *c, int level, const double *xi0, const int *Jpos, int nJ)
{
    if (c->count_only) {
        c->leaves[level] += nJ;
        return;
    }
    int dim = c->dim, nq = c->nq, nb = c->nb, ne2 = 2 * nb;
    double h = ldexp(1.0, 1 - level), hN = ldexp(1.0, -dim * (level - 1));
    double x[MAXQ][3], phx[MAXQ][MAXB], phy[MAXQ][MAXB], Wa[MAXQ];
    for (int a = 0; a < nq; ++a) {
        double xi[3];
        for (int k = 0; k < dim; ++k) xi[k] = xi0[k] + h * c->bary[a * dim + k];
        box_map(dim, c->P_l, xi, x[a]);
        box_basis(dim, c->mesh->order, xi, phx[a]);
        box_basis(dim, c->mesh->order, c->bary + a * dim, phy[a]);
        Wa[a] = c->w[a] * hN * box_jacdet(dim, c->P_l, xi);
    }
    for (int t = 0; t < nJ; ++t) {
        int pos = Jpos[t];
        double Pm[MAXV * 3];
        elem_vertices(c->mesh, c->J[pos], Pm);
        double y[MAXQ][3], Wb[MAXQ];
        for (int b = 0; b < nq; ++b) {
            box_map(dim, Pm, c->bary + b * dim, y[b]);
            Wb[b] = c->w[b] * box_jacdet(dim, Pm, c->bary + b * dim);
        }
        point_pairs(c, c->E + (size_t)pos * ne2 * ne2, nq, x, Wa, phx, y, Wb, phy);
        c->leaves[level]++;
    }
}

/* Algorithm 1, AdaptiveIntegration(L_min, L_max, L_cur, E_l, J_l).  V holds
 * the physical vertices of the current (sub-)element, Lam their barycentric
 * coordinates with respect to the root element l. */
static void adaptive(alg_ctx *c, int lcur, const double *V, const double *Lam, const int *Jpos,
                     int nJ)
{
    int dim = c->dim, nv = c->nv;
    int lmin = c->p->lmin, lmax = c->p->lmax;
    if (lcur < lmin) {
        double CV[8 * MAXV * 3], CL[8 * MAXV * MAXV];
        children_n(dim, dim, V, CV);
        children_n(dim, nv, Lam, CL);
        for (int ch = 0; ch < (1 << dim); ++ch)
            adaptive(c, lcur + 1, CV + ch * nv * dim, CL + ch * nv * nv, Jpos, nJ);
        return;
    }
    if (lcur == lmax) {
        integration(c, lcur, V, Lam, Jpos, nJ);
        return;
    }
    double lo[3], hi[3];
    bbox_of(dim, nv, V, lo, hi);
    int *Jint = (int *)malloc(sizeof(int) * (nJ + 1));
    int *Jref = (int *)malloc(sizeof(int) * (nJ + 1));
    int nint = 0, nref = 0;
    for (int t = 0; t < nJ; ++t) {
        const double *lo2 = c->jlo + Jpos[t] * dim, *hi2 = c->jhi + Jpos[t] * dim;
        const double *glo = c->qlo + Jpos[t] * dim, *ghi = c->qhi + Jpos[t] * dim;
        if (or_aprxmax(dim, lo, hi, lo2, hi2) < c->dme)
            Jint[nint++] = Jpos[t];
        else if ((c->p->min_l2 ? or_boxgap_l2(dim, lo, hi, glo, ghi) : or_aprxmin(dim, lo, hi, lo2, hi2)) < c->dpe)
            Jref[nref++] = Jpos[t];
    }
    if (nint > 0) integration(c, lcur, V, Lam, Jint, nint);
    if (nref > 0) {
        double CV[8 * MAXV * 3], CL[8 * MAXV * MAXV];
        children_n(dim, dim, V, CV);
        children_n(dim, nv, Lam, CL);
        for (int ch = 0; ch < (1 << dim); ++ch)
            adaptive(c, lcur + 1, CV + ch * nv * dim, CL + ch * nv * nv, Jref, nref);
    }
    free(Jint);
    free(Jref);
}

/* Algorithm 1 for quadrilaterals and hexahedra: P holds the physical corners of
 * the current sub-element (formed by box_children from the root's), xi0 its
 * reference origin in the root element, h = 2^{1-lcur} its reference size. */
static void adaptive_box(alg_ctx *c, int lcur, const double *P, const double *xi0, const int *Jpos,
                         int nJ)
{
    int dim = c->dim, nc = 1 << dim;
    int lmin = c->p->lmin, lmax = c->p->lmax;
    double CP[8 * 8 * 3];
    if (lcur < lmin) {
        box_children(dim, P, CP);
        for (int ch = 0; ch < nc; ++ch) {
            double cxi[3];
            for (int k = 0; k < dim; ++k) cxi[k] = xi0[k] + (((ch >> k) & 1) ? ldexp(1.0, -lcur) : 0.0);
            adaptive_box(c, lcur + 1, CP + ch * nc * dim, cxi, Jpos, nJ);
        }
        return;
    }
    if (lcur == lmax) {
        integration_box(c, lcur, xi0, Jpos, nJ);
        return;
    }
    double lo[3], hi[3];
    bbox_of(dim, nc, P, lo, hi);
    int *Jint = (int *)malloc(sizeof(int) * (nJ + 1));
    int *Jref = (int *)malloc(sizeof(int) * (nJ + 1));
    int nint = 0, nref = 0;
    for (int t = 0; t < nJ; ++t) {
        const double *lo2 = c->jlo + Jpos[t] * dim, *hi2 = c->jhi + Jpos[t] * dim;
        const double *glo = c->qlo + Jpos[t] * dim, *ghi = c->qhi + Jpos[t] * dim;
        if (or_aprxmax(dim, lo, hi, lo2, hi2) < c->dme)
            Jint[nint++] = Jpos[t];
        else if ((c->p->min_l2 ? or_boxgap_l2(dim, lo, hi, glo, ghi) : or_aprxmin(dim, lo, hi, lo2, hi2)) < c->dpe)
            Jref[nref++] = Jpos[t];
    }
    if (nint > 0) integration_box(c, lcur, xi0, Jint, nint);
    if (nref > 0) {
        box_children(dim, P, CP);
        for (int ch = 0; ch < nc; ++ch) {
            double cxi[3];
            for (int k = 0; k < dim; ++k) cxi[k] = xi0[k] + (((ch >> k) & 1) ? ldexp(1.0, -lcur) : 0.0);
            adaptive_box(c, lcur + 1, CP + ch * nc * dim, cxi, Jref, nref);
        }
    }
    free(Jint);
    free(Jref);
}

static void ctx_init(alg_ctx *c, const or_mesh *m, const or_params *p, int64_t *leaves)
{
    memset(c, 0, sizeof(*c));
    c->mesh = m;
    c->p = p;
    c->dim = m->dim;
    c->shape = m->shape;
    c->nv = geo_vertices(m);
    c->nq = m->shape ? box_rule(m->dim, c->bary, c->w) : or_rule(m->dim, c->bary, c->w);
    c->nb = nodes_of(m);
    c->C = (p->scale > 0.0) ? p->scale : or_kernel_constant(m->dim, p->kernel, p->delta, p->eps);
    c->dme = p->delta - p->eps;
    c->dpe = p->delta + p->eps;
    c->leaves = leaves;
}

/* run Algorithm 1 for outer element l against the inner list J (n entries);
 * the per-position extended blocks go to E */
static void run_outer(alg_ctx *c, int64_t l, const int32_t *J, int n, double *E)
{
    int nv = c->nv, dim = c->dim;
    c->l = l;
    c->meas_l = or_elem_measure(c->mesh, l);
    c->J = J;
    c->E = E;
    memset(E, 0, sizeof(double) * (size_t)n * (2 * c->nb) * (2 * c->nb));
    double V[MAXV * 3], Lam[MAXV * MAXV];
    c->jlo = (double *)malloc(sizeof(double) * (size_t)(n + 1) * dim);
    c->jhi = (double *)malloc(sizeof(double) * (size_t)(n + 1) * dim);
    for (int t = 0; t < n; ++t) {
        elem_vertices(c->mesh, J[t], V);
        bbox_of(dim, nv, V, c->jlo + t * dim, c->jhi + t * dim);
    }
    c->qlo = c->jlo;
    c->qhi = c->jhi;
    if (c->p->min_l2 == 2) {
        /* The box of the inner quadrature points y_b, formed exactly as
         * integration() forms them: no outer point of a sub-element whose box is
         * at least delta + eps from this box has a y_b within the kernel's
         * support, so dropping it again removes only zero contributions (a
         * tighter test than the inner element's own box, of our own) */
        c->qlo = (double *)malloc(sizeof(double) * (size_t)(n + 1) * dim);
        c->qhi = (double *)malloc(sizeof(double) * (size_t)(n + 1) * dim);
        for (int t = 0; t < n; ++t) {
            elem_vertices(c->mesh, J[t], V);
            for (int k = 0; k < dim; ++k) {
                double a = 0.0, b = 0.0;
                for (int q = 0; q < c->nq; ++q) {
                    double s = 0.0;
                    if (c->shape) {
                        double y[3];
                        box_map(dim, V, c->bary + q * dim, y);
                        s = y[k];
                    } else {
                        for (int v = 0; v < nv; ++v) s += c->bary[q * nv + v] * V[v * dim + k];
                    }
                    if (q == 0 || s < a) a = s;
                    if (q == 0 || s > b) b = s;
                }
                c->qlo[t * dim + k] = a;
                c->qhi[t * dim + k] = b;
            }
        }
    }
    elem_vertices(c->mesh, l, V);
    int *Jpos = (int *)malloc(sizeof(int) * (n + 1));
    for (int t = 0; t < n; ++t) Jpos[t] = t;
    if (c->shape) {
        const double xi0[3] = {0.0, 0.0, 0.0};
        memcpy(c->P_l, V, sizeof(double) * nv * dim);
        adaptive_box(c, 1, V, xi0, Jpos, n);
    } else {
        for (int i = 0; i < nv; ++i)
            for (int j = 0; j < nv; ++j) Lam[i * nv + j] = (i == j) ? 1.0 : 0.0;
        adaptive(c, 1, V, Lam, Jpos, n);
    }
    free(Jpos);
    if (c->qlo != c->jlo) {
        free(c->qlo);
        free(c->qhi);
    }
    free(c->jlo);
    free(c->jhi);
}

/* Extended block of one ordered pair (l, m), Algorithm 1 run with J = {m}.
 * E is (2N+2)x(2N+2), index space [local nodes of l, local nodes of m]. */
int32_t or_pair_block(const or_mesh *m, const or_params *p, int64_t l, int64_t mm, double *E,
                      int64_t *leaves, int64_t *evals)
{
    alg_ctx c;
    ctx_init(&c, m, p, leaves);
    int32_t J = (int32_t)mm;
    run_outer(&c, l, &J, 1, E);
    if (evals) {
        evals[0] += c.evals[0];
        evals[1] += c.evals[1];
    }
    return 0;
}

static int64_t find_col(const int64_t *row_ptr, const int32_t *col, int64_t r, int32_t c)
{
    int64_t lo = row_ptr[r], hi = row_ptr[r + 1] - 1;
    while (lo <= hi) {
        int64_t mid = (lo + hi) / 2;
        if (col[mid] == c) return mid;
        if (col[mid] < c) lo = mid + 1; else hi = mid - 1;
    }
    return -1;
}

typedef struct {
    const or_mesh *m;
    const or_params *p;
    const int64_t *pair_off;
    const int32_t *pair_m;
    const int64_t *list;
    int64_t i0, i1;
    const int64_t *row_ptr;
    const int32_t *col;
    double *val;
    int64_t leaves[16];
    int64_t evals[2];
    int32_t status;
} asm_job;

static void *asm_worker(void *arg)
{
    asm_job *j = (asm_job *)arg;
    const or_mesh *m = j->m;
    int nv = nodes_of(m), ne2 = 2 * nv;
    alg_ctx c;
    ctx_init(&c, m, j->p, j->leaves);
    int64_t maxn = 0;
    for (int64_t t = j->i0; t < j->i1; ++t) {
        int64_t l = j->list ? j->list[t] : t;
        int64_t n = j->pair_off[l + 1] - j->pair_off[l];
        if (n > maxn) maxn = n;
    }
    double *E = (double *)malloc(sizeof(double) * (size_t)(maxn + 1) * ne2 * ne2);
    for (int64_t t = j->i0; t < j->i1; ++t) {
        int64_t l = j->list ? j->list[t] : t;
        int64_t b = j->pair_off[l];
        int n = (int)(j->pair_off[l + 1] - b);
        run_outer(&c, l, j->pair_m + b, n, E);
        for (int pos = 0; pos < n; ++pos) {
            int64_t mm = j->pair_m[b + pos];
            const double *Ep = E + (size_t)pos * ne2 * ne2;
            for (int P = 0; P < ne2; ++P) {
                int32_t r = (P < nv) ? m->conn[l * nv + P] : m->conn[mm * nv + P - nv];
                for (int Q = 0; Q < ne2; ++Q) {
                    int32_t cc = (Q < nv) ? m->conn[l * nv + Q] : m->conn[mm * nv + Q - nv];
                    int64_t at = find_col(j->row_ptr, j->col, r, cc);
                    if (at < 0) {
                        j->status = -1;
                        continue;
                    }
                    j->val[at] += Ep[P * ne2 + Q];
                }
            }
        }
    }
    j->evals[0] = c.evals[0];
    j->evals[1] = c.evals[1];
    free(E);
    return NULL;
}

/* Global assembly: Algorithm 1 per outer element l with J = J_l, pair blocks
 * scattered into the given CSR pattern.  sel (n_sel entries) restricts the outer
 * elements; sel == NULL means all.  Outer elements are split into contiguous
 * blocks per thread; per-thread value arrays are summed in thread order. */
int32_t or_assemble(const or_mesh *m, const or_params *p, int32_t nthreads,
                    const int64_t *pair_off, const int32_t *pair_m, int64_t n_sel,
                    const int64_t *sel, const int64_t *row_ptr, const int32_t *col,
                    double *val, int64_t *leaves, int64_t *evals)
{
    int64_t ne = m->n_elems, nnz = row_ptr[m->n_nodes];
    int64_t cnt = sel ? n_sel : ne;
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 64) nthreads = 64;
    asm_job *jobs = (asm_job *)calloc(nthreads, sizeof(asm_job));
    for (int t = 0; t < nthreads; ++t) {
        asm_job *j = &jobs[t];
        j->m = m;
        j->p = p;
        j->pair_off = pair_off;
        j->pair_m = pair_m;
        j->list = sel;
        j->i0 = cnt * t / nthreads;
        j->i1 = cnt * (t + 1) / nthreads;
        j->row_ptr = row_ptr;
        j->col = col;
        j->val = (double *)calloc((size_t)nnz, sizeof(double));
    }
    run_threads(nthreads, asm_worker, jobs, sizeof(asm_job));
    int32_t status = 0;
    for (int64_t k = 0; k < nnz; ++k) val[k] = 0.0;
    for (int t = 0; t < nthreads; ++t) {
        for (int64_t k = 0; k < nnz; ++k) val[k] += jobs[t].val[k];
        if (leaves)
            for (int lv = 0; lv <= p->lmax && lv < 16; ++lv) leaves[lv] += jobs[t].leaves[lv];
        if (evals) {
            evals[0] += jobs[t].evals[0];
            evals[1] += jobs[t].evals[1];
        }
        if (jobs[t].status) status = jobs[t].status;
        free(jobs[t].val);
    }
    free(jobs);
    return status;
}

/* ------------------------------------------------------------ leaf counts */

typedef struct {
    const or_mesh *m;
    const or_params *p;
    const double *lo, *hi;
    const int64_t *sel;
    int64_t i0, i1;
    int evaluate;        /* 1: Integration() evaluated, 0: leaves counted only */
    int64_t leaves[16];
    int64_t evals[2];
    double checksum;     /* sum of the blocks' entries (keeps the work observable) */
} count_job;

static void *count_worker(void *arg)
{
    count_job *j = (count_job *)arg;
    const or_mesh *m = j->m;
    int ne2 = 2 * nodes_of(m);
    alg_ctx c;
    ctx_init(&c, m, j->p, j->leaves);
    c.count_only = !j->evaluate;
    int32_t *J = (int32_t *)malloc(sizeof(int32_t) * (size_t)(m->n_elems + 1));
    for (int64_t t = j->i0; t < j->i1; ++t) {
        int64_t l = j->sel[t];
        int64_t n = pairs_one(m, j->lo, j->hi, j->p->delta + j->p->eps, l, J);
        double *E = (double *)malloc(sizeof(double) * (size_t)(n + 1) * ne2 * ne2);
        run_outer(&c, l, J, (int)n, E);
        if (j->evaluate)
            for (int64_t k = 0; k < n * ne2 * ne2; ++k) j->checksum += E[k];
        free(E);
    }
    j->evals[0] = c.evals[0];
    j->evals[1] = c.evals[1];
    free(J);
    return NULL;
}

/* Algorithm 1 for the outer elements sel[0..n_sel), each with its brute-force
 * J_l, in nthreads threads: leaves per level (and evaluations) summed.  With
 * evaluate == 0 the leaves are counted without evaluating them (the counts a
 * full assembly of those elements gives, at the cost of the traversal alone). */
static double outer_runs(const or_mesh *m, const or_params *p, int32_t nthreads, int64_t n_sel,
                         const int64_t *sel, int evaluate, int64_t *leaves, int64_t *evals)
{
    int64_t ne = m->n_elems;
    double *lo = (double *)malloc(sizeof(double) * ne * m->dim);
    double *hi = (double *)malloc(sizeof(double) * ne * m->dim);
    all_bboxes(m, lo, hi);
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 64) nthreads = 64;
    count_job *jobs = (count_job *)calloc(nthreads, sizeof(count_job));
    for (int t = 0; t < nthreads; ++t) {
        jobs[t].m = m;
        jobs[t].p = p;
        jobs[t].lo = lo;
        jobs[t].hi = hi;
        jobs[t].sel = sel;
        jobs[t].i0 = n_sel * t / nthreads;
        jobs[t].i1 = n_sel * (t + 1) / nthreads;
        jobs[t].evaluate = evaluate;
    }
    run_threads(nthreads, count_worker, jobs, sizeof(count_job));
    double checksum = 0.0;
    for (int t = 0; t < nthreads; ++t) {
        if (leaves)
            for (int lv = 0; lv < 16; ++lv) leaves[lv] += jobs[t].leaves[lv];
        if (evals) {
            evals[0] += jobs[t].evals[0];
            evals[1] += jobs[t].evals[1];
        }
        checksum += jobs[t].checksum;
    }
    free(jobs);
    free(lo);
    free(hi);
    return checksum;
}

void or_leaf_counts(const or_mesh *m, const or_params *p, int32_t nthreads, int64_t n_sel,
                    const int64_t *sel, int64_t *leaves)
{
    outer_runs(m, p, nthreads, n_sel, sel, 0, leaves, NULL);
}

/* Algorithm 1 with every Integration() evaluated for the outer elements
 * sel[0..n_sel) (each with its brute-force J_l), blocks discarded: the oracle's
 * assembly work without the global matrix (timed as the CPU baseline).
 * Returns the sum of all block entries. */
double or_outer_blocks(const or_mesh *m, const or_params *p, int32_t nthreads, int64_t n_sel,
                       const int64_t *sel, int64_t *leaves, int64_t *evals)
{
    return outer_runs(m, p, nthreads, n_sel, sel, 1, leaves, evals);
}

/* ------------------------------------------------------------ sampled rows */

typedef struct {
    int64_t l, m;
} pair_key;

static int cmp_pair(const void *a, const void *b)
{
    const pair_key *x = (const pair_key *)a, *y = (const pair_key *)b;
    if (x->l != y->l) return (x->l > y->l) - (x->l < y->l);
    return (x->m > y->m) - (x->m < y->m);
}

typedef struct {
    const or_mesh *m;
    const or_params *p;
    const pair_key *pairs;
    int64_t i0, i1;
    int64_t n_rows;
    const int64_t *rows;
    const int64_t *row_off;   /* offsets into the output entries */
    const int64_t *row_len;
    const int32_t *cols;
    double *acc;              /* per-thread accumulator over the output entries */
} rows_job;

static void *rows_worker(void *arg)
{
    rows_job *j = (rows_job *)arg;
    const or_mesh *m = j->m;
    int nv = nodes_of(m), ne2 = 2 * nv;
    double E[4 * MAXB * MAXB];
    int64_t leaves[16] = {0};
    for (int64_t t = j->i0; t < j->i1; ++t) {
        int64_t l = j->pairs[t].l, mm = j->pairs[t].m;
        or_pair_block(m, j->p, l, mm, E, leaves, NULL);
        for (int P = 0; P < ne2; ++P) {
            int32_t r = (P < nv) ? m->conn[l * nv + P] : m->conn[mm * nv + P - nv];
            for (int64_t k = 0; k < j->n_rows; ++k) {
                if (j->rows[k] != r) continue;
                for (int Q = 0; Q < ne2; ++Q) {
                    int32_t cc = (Q < nv) ? m->conn[l * nv + Q] : m->conn[mm * nv + Q - nv];
                    const int32_t *cs = j->cols + j->row_off[k];
                    int64_t lo = 0, hi = j->row_len[k] - 1, at = -1;
                    while (lo <= hi) {
                        int64_t mid = (lo + hi) / 2;
                        if (cs[mid] == cc) { at = mid; break; }
                        if (cs[mid] < cc) lo = mid + 1; else hi = mid - 1;
                    }
                    if (at >= 0) j->acc[j->row_off[k] + at] += E[P * ne2 + Q];
                }
            }
        }
    }
    return NULL;
}

/* Pattern and values of selected rows, from every ordered pair (l, m) whose
 * node set touches the row, each pair integrated by Algorithm 1 with J = {m}.
 * cols == NULL: fill row_len and return the total entry count.  vals == NULL:
 * pattern only.  J_e is found by brute force against every element. */
int64_t or_rows(const or_mesh *m, const or_params *p, double thr, int32_t nthreads,
                int64_t n_rows, const int64_t *rows, int64_t *row_len, int32_t *cols,
                double *vals)
{
    int64_t ne = m->n_elems;
    int nv = nodes_of(m);
    double *lo = (double *)malloc(sizeof(double) * ne * m->dim);
    double *hi = (double *)malloc(sizeof(double) * ne * m->dim);
    all_bboxes(m, lo, hi);
    adjacency na = node_elements(m);
    int32_t *buf = (int32_t *)malloc(sizeof(int32_t) * (m->n_nodes + 1));   /* one row's columns */
    /* pairs touching the rows: (e, x) with e containing the row node, x in J_e,
     * and (x, e) with e in J_x (found by the same brute-force test, from x's side) */
    int64_t cap = 1024, np = 0;
    pair_key *pk = (pair_key *)malloc(sizeof(pair_key) * cap);
    for (int64_t k = 0; k < n_rows; ++k) {
        int64_t i = rows[k];
        for (int64_t t = na.off[i]; t < na.off[i + 1]; ++t) {
            int64_t e = na.items[t];
            for (int64_t x = 0; x < ne; ++x) {
                int out = or_aprxmin(m->dim, lo + e * m->dim, hi + e * m->dim, lo + x * m->dim,
                                     hi + x * m->dim) < thr;
                int in = or_aprxmin(m->dim, lo + x * m->dim, hi + x * m->dim, lo + e * m->dim,
                                    hi + e * m->dim) < thr;
                if (np + 2 > cap) {
                    cap *= 2;
                    pk = (pair_key *)realloc(pk, sizeof(pair_key) * cap);
                }
                if (out) { pk[np].l = e; pk[np].m = x; ++np; }
                if (in) { pk[np].l = x; pk[np].m = e; ++np; }
            }
        }
    }
    qsort(pk, (size_t)np, sizeof(pair_key), cmp_pair);
    int64_t nu = 0;
    for (int64_t t = 0; t < np; ++t)
        if (nu == 0 || cmp_pair(&pk[nu - 1], &pk[t]) != 0) pk[nu++] = pk[t];
    /* per-row column sets from the touching pairs */
    int32_t *mark = (int32_t *)malloc(sizeof(int32_t) * m->n_nodes);
    int64_t total = 0;
    int64_t *row_off = (int64_t *)malloc(sizeof(int64_t) * (n_rows + 1));
    for (int64_t k = 0; k < n_rows; ++k) {
        int64_t i = rows[k];
        for (int64_t n = 0; n < m->n_nodes; ++n) mark[n] = -1;
        int64_t cnt = 0;
        for (int64_t t = 0; t < nu; ++t) {
            int64_t l = pk[t].l, mm = pk[t].m;
            int touches = 0;
            for (int q = 0; q < nv; ++q)
                if (m->conn[l * nv + q] == i || m->conn[mm * nv + q] == i) touches = 1;
            if (!touches) continue;
            for (int q = 0; q < nv; ++q) {
                int32_t a = m->conn[l * nv + q], b = m->conn[mm * nv + q];
                if (mark[a] != (int32_t)k) { mark[a] = (int32_t)k; buf[cnt++] = a; }
                if (mark[b] != (int32_t)k) { mark[b] = (int32_t)k; buf[cnt++] = b; }
            }
        }
        qsort(buf, (size_t)cnt, sizeof(int32_t), cmp_i32);
        row_off[k] = total;
        if (cols) memcpy(cols + total, buf, sizeof(int32_t) * cnt);
        row_len[k] = cnt;
        total += cnt;
    }
    row_off[n_rows] = total;
    if (cols && vals) {
        if (nthreads < 1) nthreads = 1;
        if (nthreads > 64) nthreads = 64;
        rows_job *jobs = (rows_job *)calloc(nthreads, sizeof(rows_job));
        for (int t = 0; t < nthreads; ++t) {
            rows_job *j = &jobs[t];
            j->m = m;
            j->p = p;
            j->pairs = pk;
            j->i0 = nu * t / nthreads;
            j->i1 = nu * (t + 1) / nthreads;
            j->n_rows = n_rows;
            j->rows = rows;
            j->row_off = row_off;
            j->row_len = row_len;
            j->cols = cols;
            j->acc = (double *)calloc((size_t)(total + 1), sizeof(double));
        }
        run_threads(nthreads, rows_worker, jobs, sizeof(rows_job));
        for (int64_t k = 0; k < total; ++k) vals[k] = 0.0;
        for (int t = 0; t < nthreads; ++t) {
            for (int64_t k = 0; k < total; ++k) vals[k] += jobs[t].acc[k];
            free(jobs[t].acc);
        }
        free(jobs);
    }
    free(row_off);
    free(mark);
    free(pk);
    free(buf);
    free(na.off);
    free(na.items);
    free(lo);
    free(hi);
    return total;
}

/* ------------------------------------------------------------ load, lifting, solve */

/* F_i = int_Omega f_h phi_i for free nodes i (Section 2, eq. (A-F)); f_h is the
 * interpolant of the nodal f in the element's space.  Simplices (P1, P2): the
 * degree-5 rule integrates f_h phi_i exactly for P1 and for P2 with f_h of
 * degree <= 3 (every configuration has constant f).  Quadrilaterals and
 * hexahedra (Q1, serendipity): the 3^N Gauss rule with the weights
 * w_q |det F'(xi_q)|, exact for affine elements. */
void or_load(const or_mesh *m, const double *f_nodal, const uint8_t *constrained, double *F)
{
    int nv = geo_vertices(m), nb = nodes_of(m), dim = m->dim;
    double bary[MAXQ * MAXV], w[MAXQ], phi[MAXQ][MAXB];
    int nq;
    if (m->shape) {
        nq = box_rule(dim, bary, w);
        for (int q = 0; q < nq; ++q) box_basis(dim, m->order, bary + q * dim, phi[q]);
    } else {
        nq = or_rule(dim, bary, w);
        for (int q = 0; q < nq; ++q) basis(m->order, nv, bary + q * nv, phi[q]);
    }
    for (int64_t n = 0; n < m->n_nodes; ++n) F[n] = 0.0;
    for (int64_t e = 0; e < m->n_elems; ++e) {
        double meas = or_elem_measure(m, e);
        /* per-point weights: w_q |E| (simplices), w_q |det F_e'(xi_q)| (boxes) */
        double W[MAXQ], P[MAXV * 3];
        if (m->shape) elem_vertices(m, e, P);
        for (int q = 0; q < nq; ++q) W[q] = m->shape ? w[q] * box_jacdet(dim, P, bary + q * dim) : w[q] * meas;
        for (int a = 0; a < nb; ++a) {
            int32_t node = m->conn[e * nb + a];
            if (constrained[node]) continue;
            double s = 0.0;
            for (int q = 0; q < nq; ++q) {
                double fq = 0.0;
                for (int j = 0; j < nb; ++j) fq += f_nodal[m->conn[e * nb + j]] * phi[q][j];
                s += W[q] * fq * phi[q][a];
            }
            F[node] += s;
        }
    }
}

/* F~_i = F_i - sum_{j in Gamma} A_ij g_j for free i, 0 on Gamma: the lifting of
 * Section 2, eq. (weak-homo), with the sign that linearity fixes (reading R3). */
void or_lift(int64_t n, const int64_t *row_ptr, const int32_t *col, const double *val,
             const uint8_t *constrained, const double *g, const double *F, double *Ft)
{
    for (int64_t i = 0; i < n; ++i) {
        if (constrained[i]) {
            Ft[i] = 0.0;
            continue;
        }
        double s = F[i];
        for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k)
            if (constrained[col[k]]) s -= val[k] * g[col[k]];
        Ft[i] = s;
    }
}

static void spmv_free(int64_t n, const int64_t *row_ptr, const int32_t *col, const double *val,
                      const uint8_t *constrained, const double *x, double *y)
{
    for (int64_t i = 0; i < n; ++i) {
        if (constrained[i]) {
            y[i] = 0.0;
            continue;
        }
        double s = 0.0;
        for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k)
            if (!constrained[col[k]]) s += val[k] * x[col[k]];
        y[i] = s;
    }
}

/* Jacobi-preconditioned conjugate gradients on A_{Omega,Omega} w = rhs_Omega
 * (the paper leaves its PETSc solver unstated); w = 0 on Gamma. */
int32_t or_cg(int64_t n, const int64_t *row_ptr, const int32_t *col, const double *val,
              const uint8_t *constrained, const double *rhs, double rtol, int32_t maxit,
              double *w, double *relres)
{
    double *r = (double *)calloc(n, sizeof(double));
    double *z = (double *)calloc(n, sizeof(double));
    double *p = (double *)calloc(n, sizeof(double));
    double *q = (double *)calloc(n, sizeof(double));
    double *dinv = (double *)calloc(n, sizeof(double));
    for (int64_t i = 0; i < n; ++i) {
        w[i] = 0.0;
        if (constrained[i]) continue;
        for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k)
            if (col[k] == i) dinv[i] = 1.0 / val[k];
    }
    double bnorm = 0.0;
    for (int64_t i = 0; i < n; ++i)
        if (!constrained[i]) bnorm += rhs[i] * rhs[i];
    bnorm = sqrt(bnorm);
    for (int64_t i = 0; i < n; ++i) {
        r[i] = constrained[i] ? 0.0 : rhs[i];
        z[i] = dinv[i] * r[i];
        p[i] = z[i];
    }
    double rz = 0.0;
    for (int64_t i = 0; i < n; ++i) rz += r[i] * z[i];
    int32_t it = 0;
    double rn = bnorm;
    if (bnorm == 0.0) {
        *relres = 0.0;
        goto done;
    }
    for (it = 0; it < maxit; ++it) {
        spmv_free(n, row_ptr, col, val, constrained, p, q);
        double pq = 0.0;
        for (int64_t i = 0; i < n; ++i) pq += p[i] * q[i];
        double alpha = rz / pq;
        rn = 0.0;
        for (int64_t i = 0; i < n; ++i) {
            w[i] += alpha * p[i];
            r[i] -= alpha * q[i];
            rn += r[i] * r[i];
        }
        rn = sqrt(rn);
        if (rn <= rtol * bnorm) {
            ++it;
            break;
        }
        double rz2 = 0.0;
        for (int64_t i = 0; i < n; ++i) {
            z[i] = dinv[i] * r[i];
            rz2 += r[i] * z[i];
        }
        double beta = rz2 / rz;
        rz = rz2;
        for (int64_t i = 0; i < n; ++i) p[i] = z[i] + beta * p[i];
    }
    *relres = rn / bnorm;
done:
    free(r);
    free(z);
    free(p);
    free(q);
    free(dinv);
    return it;
}

/* Dense Gaussian elimination with partial pivoting on the free block (for the
 * two-term forms, whose matrices are not symmetric); same arguments as
 * or_cholesky_solve.  Returns 0, -1 (too large) or -2 (singular). */
int32_t or_lu_solve(int64_t n, const int64_t *row_ptr, const int32_t *col, const double *val,
                    const uint8_t *constrained, const double *rhs, double *w)
{
    int64_t *map = (int64_t *)malloc(sizeof(int64_t) * n);
    int64_t nf = 0;
    for (int64_t i = 0; i < n; ++i) map[i] = constrained[i] ? -1 : nf++;
    if (nf > 6000) {
        free(map);
        return -1;
    }
    double *M = (double *)calloc((size_t)(nf * nf + 1), sizeof(double));
    double *b = (double *)calloc((size_t)(nf + 1), sizeof(double));
    for (int64_t i = 0; i < n; ++i) {
        if (map[i] < 0) continue;
        b[map[i]] = rhs[i];
        for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k)
            if (map[col[k]] >= 0) M[map[i] * nf + map[col[k]]] = val[k];
    }
    int32_t st = 0;
    for (int64_t c = 0; c < nf && st == 0; ++c) {
        int64_t piv = c;
        for (int64_t r = c + 1; r < nf; ++r)
            if (fabs(M[r * nf + c]) > fabs(M[piv * nf + c])) piv = r;
        if (M[piv * nf + c] == 0.0) {
            st = -2;
            break;
        }
        if (piv != c) {
            for (int64_t k = 0; k < nf; ++k) {
                double t = M[c * nf + k];
                M[c * nf + k] = M[piv * nf + k];
                M[piv * nf + k] = t;
            }
            double t = b[c];
            b[c] = b[piv];
            b[piv] = t;
        }
        for (int64_t r = c + 1; r < nf; ++r) {
            double f = M[r * nf + c] / M[c * nf + c];
            if (f == 0.0) continue;
            for (int64_t k = c; k < nf; ++k) M[r * nf + k] -= f * M[c * nf + k];
            b[r] -= f * b[c];
        }
    }
    if (st == 0) {
        for (int64_t r = nf - 1; r >= 0; --r) {
            double t = b[r];
            for (int64_t k = r + 1; k < nf; ++k) t -= M[r * nf + k] * b[k];
            b[r] = t / M[r * nf + r];
        }
        for (int64_t i = 0; i < n; ++i) w[i] = map[i] >= 0 ? b[map[i]] : 0.0;
    }
    free(M);
    free(b);
    free(map);
    return st;
}

/* Dense Cholesky solve of A_{Omega,Omega} w = rhs_Omega (small systems only). */
int32_t or_cholesky_solve(int64_t n, const int64_t *row_ptr, const int32_t *col,
                          const double *val, const uint8_t *constrained, const double *rhs,
                          double *w)
{
    int64_t *map = (int64_t *)malloc(sizeof(int64_t) * n);
    int64_t nf = 0;
    for (int64_t i = 0; i < n; ++i) map[i] = constrained[i] ? -1 : nf++;
    if (nf > 6000) {
        free(map);
        return -1;
    }
    double *L = (double *)calloc((size_t)(nf * nf + 1), sizeof(double));
    double *b = (double *)calloc((size_t)(nf + 1), sizeof(double));
    for (int64_t i = 0; i < n; ++i) {
        if (map[i] < 0) continue;
        b[map[i]] = rhs[i];
        for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k)
            if (map[col[k]] >= 0) L[map[i] * nf + map[col[k]]] = val[k];
    }
    for (int64_t j = 0; j < nf; ++j) {
        double s = L[j * nf + j];
        for (int64_t k = 0; k < j; ++k) s -= L[j * nf + k] * L[j * nf + k];
        if (s <= 0.0) {
            free(L);
            free(b);
            free(map);
            return -2;
        }
        double d = sqrt(s);
        L[j * nf + j] = d;
        for (int64_t i = j + 1; i < nf; ++i) {
            double t = L[i * nf + j];
            for (int64_t k = 0; k < j; ++k) t -= L[i * nf + k] * L[j * nf + k];
            L[i * nf + j] = t / d;
        }
    }
    for (int64_t i = 0; i < nf; ++i) {
        double t = b[i];
        for (int64_t k = 0; k < i; ++k) t -= L[i * nf + k] * b[k];
        b[i] = t / L[i * nf + i];
    }
    for (int64_t i = nf - 1; i >= 0; --i) {
        double t = b[i];
        for (int64_t k = i + 1; k < nf; ++k) t -= L[k * nf + i] * b[k];
        b[i] = t / L[i * nf + i];
    }
    for (int64_t i = 0; i < n; ++i) w[i] = (map[i] >= 0) ? b[map[i]] : 0.0;
    free(L);
    free(b);
    free(map);
    return 0;
}
