// Quadrilaterals and hexahedra: tensor-product elements on the reference box
// [0,1]^N (Section 4 allows them in the triangulation; Section 6 integrates
// them with the 3x3 and 3x3x3 Gauss-Legendre product rules).
//
//   * corners in tensor order: corner c = c0 + 2 c1 + 4 c2 sits at the reference
//     point (c0, c1, c2); the element map is their multilinear interpolation
//     F(xi) = sum_c N_c(xi) P_c, N_c(xi) = prod_k (c_k ? xi_k : 1 - xi_k);
//   * order 1 = Q1 (the corners are the nodes), order 2 = serendipity (8 / 20
//     nodes: the corners, then the edge midpoints in increasing t0 + 3 t1 + 9 t2
//     of their position t in half units);
//   * midpoint refinement into 2^N children, formed by halving the box along
//     axis 0, then 1, then 2 (each halving takes the midpoints (a + b) * 0.5 of
//     the corner pairs along that axis), so a child's corners are exactly the
//     points of the parent's 3^N midpoint lattice formed axis by axis.
//
// The integration contracts each pair's kernel values against the monomials
// xi^e of the products phi_I phi_J of two basis functions (e = a + b, a and b
// in the element's space): 9 / 27 rows for Q1, 22 / 90 for serendipity.  The
// host maps those rows to the basis functions and their products
// (make_box_tables).
#pragma once

#include <hip/hip_runtime.h>

namespace nlq {

__host__ __device__ constexpr int box_corner_count(int dim) { return 1 << dim; }
__host__ __device__ constexpr int box_node_count(int dim, int order)
{
    return order == 2 ? (dim == 2 ? 8 : 20) : 1 << dim;
}
__host__ __device__ constexpr int box_nq(int dim) { return dim == 2 ? 9 : 27; }

// xi^e in the element's space: Q1 every e_k <= 1; serendipity every e_k <= 2
// with at most one e_k = 2 (superlinear degree <= 2)
__host__ __device__ constexpr bool box_in_space(int order, int dim, const int *e)
{
    int twos = 0;
    for (int k = 0; k < dim; ++k) {
        if (e[k] < 0 || e[k] > order) return false;
        twos += e[k] == 2;
    }
    return twos <= 1;
}

// e = a + b with a, b in the space (a runs over the space; b = e - a)
__host__ __device__ constexpr bool box_is_product(int order, int dim, const int *e)
{
    for (int q = 0; q < 27; ++q) {
        int a[3] = {q % 3, (q / 3) % 3, q / 9}, b[3] = {0, 0, 0};
        bool ok = true;
        for (int k = 0; k < 3; ++k) {
            if (k >= dim) {
                if (a[k] != 0) ok = false;
                continue;
            }
            b[k] = e[k] - a[k];
        }
        if (ok && box_in_space(order, dim, a) && box_in_space(order, dim, b)) return true;
    }
    return false;
}

// the product monomials, in increasing e0 + 5 e1 + 25 e2 (e_k <= 4)
template <int DIM, int ORD> struct BoxMono {
    static constexpr int count()
    {
        int n = 0;
        for (int q = 0; q < (DIM == 2 ? 25 : 125); ++q) {
            int e[3] = {q % 5, (q / 5) % 5, q / 25};
            if (box_is_product(ORD, DIM, e)) ++n;
        }
        return n;
    }
    static constexpr int N = count();
    int e[N][DIM];
    constexpr BoxMono() : e{}
    {
        int n = 0;
        for (int q = 0; q < (DIM == 2 ? 25 : 125); ++q) {
            int x[3] = {q % 5, (q / 5) % 5, q / 25};
            if (!box_is_product(ORD, DIM, x)) continue;
            for (int k = 0; k < DIM; ++k) e[n][k] = x[k];
            ++n;
        }
    }
};

// 3-point Gauss-Legendre nodes on [0,1] from the closed form (1 + z)/2,
// z = -sqrt(3/5), 0, sqrt(3/5), and their weights (5/9, 8/9, 5/9)/2
__host__ __device__ inline double box_gauss_node(int i)
{
    const double r = sqrt(3.0 / 5.0);
    const double z = i == 0 ? -r : (i == 1 ? 0.0 : r);
    return (1.0 + z) / 2.0;
}
__host__ __device__ inline double box_gauss_weight(int i) { return (i == 1 ? 8.0 / 9.0 : 5.0 / 9.0) / 2.0; }

// ---------------------------------------------------------------- geometry
#if defined(__HIP__)

template <int DIM> struct BoxVerts {
    double v[1 << DIM][DIM];
};

// multilinear weights N_c(xi), products over k in order, rounded as written
template <int DIM> __device__ __forceinline__ void box_corner_weights(const double *xi, double *N)
{
#pragma unroll
    for (int c = 0; c < (1 << DIM); ++c) {
        double p = 1.0;
#pragma unroll
        for (int k = 0; k < DIM; ++k) p = __dmul_rn(p, ((c >> k) & 1) ? xi[k] : __dsub_rn(1.0, xi[k]));
        N[c] = p;
    }
}

// |det dF/dxi| at xi of the box with corners P (dN_c/dxi_i as products)
template <int DIM> __device__ __forceinline__ double box_jacdet(const BoxVerts<DIM> &P, const double *xi)
{
    double J[DIM][DIM];
#pragma unroll
    for (int k = 0; k < DIM; ++k)
#pragma unroll
        for (int i = 0; i < DIM; ++i) {
            double sum = 0.0;
#pragma unroll
            for (int c = 0; c < (1 << DIM); ++c) {
                double p = 1.0;
#pragma unroll
                for (int j = 0; j < DIM; ++j) {
                    const int cj = (c >> j) & 1;
                    p *= j == i ? (cj ? 1.0 : -1.0) : (cj ? xi[j] : 1.0 - xi[j]);
                }
                sum = fma(p, P.v[c][k], sum);
            }
            J[k][i] = sum;
        }
    double det;
    if constexpr (DIM == 2) {
        det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
    } else {
        det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) - J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
              J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
    }
    return fabs(det);
}

// child c of a box: halve along axis 0, then 1, then 2; along axis k every
// corner pair (bit k clear / set) becomes (lo, m) for c_k = 0 or (m, hi) for
// c_k = 1, m = (lo + hi) * 0.5 rounded as written
template <int DIM> __device__ __forceinline__ BoxVerts<DIM> box_child_of(const BoxVerts<DIM> &S, int c)
{
    BoxVerts<DIM> B = S;
#pragma unroll
    for (int ax = 0; ax < DIM; ++ax) {
        const bool hi_half = ((c >> ax) & 1) != 0;
#pragma unroll
        for (int q = 0; q < (1 << DIM); ++q) {
            if ((q >> ax) & 1) continue;
            const int q1 = q | (1 << ax);
#pragma unroll
            for (int k = 0; k < DIM; ++k) {
                const double m = __dmul_rn(__dadd_rn(B.v[q][k], B.v[q1][k]), 0.5);
                if (hi_half) B.v[q][k] = m;
                else B.v[q1][k] = m;
            }
        }
    }
    return B;
}

#endif  // __HIP__

}  // namespace nlq
