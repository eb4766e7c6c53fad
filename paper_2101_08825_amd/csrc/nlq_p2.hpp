// Quadratic (P2) Lagrange elements: the integration's contraction rows for them.
//
// A P2 element has the dim+1 vertices and the edge midpoints as nodes (edges
// (i, j), i < j, in lexicographic order); its basis in the barycentric
// coordinates lambda is lambda_i (2 lambda_i - 1) at vertex i and
// 4 lambda_i lambda_j at edge (i, j).  The per-pair blocks of eq.
// (Aij-support2) need, over the outer points x_a of the leaves,
//   sum_a w_a phi_I(x_a) g_ab           (B_lm),
//   sum_a w_a g_ab                      (B_mm, through the inner basis),
//   sum_a w_a phi_I(x_a) phi_J(x_a) g_ab   (B_ll),
// all of which are linear combinations of the sums over the homogeneous
// monomials of degree 4 in lambda (sum lambda = 1 raises every lower degree to
// 4): 15 monomials in 2D, 35 in 3D.  The kernels accumulate those monomial rows
// and the epilogue maps them to the rows it needs with a table built on the
// host (make_p2_map).
#pragma once

#include <hip/hip_runtime.h>

namespace nlq {

__host__ __device__ constexpr int p2_nodes(int dim) { return (dim + 1) * (dim + 2) / 2; }
__host__ __device__ constexpr int p2_monomials(int dim) { return dim == 2 ? 15 : 35; }

// exponents of monomial k (degree 4 in nv = dim + 1 variables), in the order of
// a lexicographically decreasing exponent vector: (4,0,..), (3,1,0,..), ...
template <int NV> struct Mono4 {
    static constexpr int N = NV == 3 ? 15 : 35;
    int e[N][NV];
    constexpr Mono4() : e{}
    {
        int k = 0;
        int c[NV] = {};
        c[0] = 4;
        for (;;) {
            for (int v = 0; v < NV; ++v) e[k][v] = c[v];
            ++k;
            // next composition of 4 into NV parts, lexicographically decreasing
            int j = NV - 2;
            while (j >= 0 && c[j] == 0) --j;
            if (j < 0) break;
            c[j] -= 1;
            int rest = 0;
            for (int v = j + 1; v < NV; ++v) rest += c[v];
            for (int v = j + 1; v < NV; ++v) c[v] = 0;
            c[j + 1] = rest + 1;
        }
    }
};

}  // namespace nlq
