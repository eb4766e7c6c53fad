// Midpoint refinement of a simplex into 2^N children (Algorithm 1, Section 5:
// "split E_l into 2^N sub-elements using the midpoint rule").  Every child
// vertex is either a parent vertex or the midpoint (V_i + V_j) * 0.5 of a parent
// edge; the table lists, for each child and each of its vertices, the parent
// vertex pair (i, j), with i == j for a parent vertex.
//  triangles: the three corner triangles, then the middle one;
//  tetrahedra (the paper refines hexahedra and leaves tets open): the four
//  corner tets, then the inner octahedron cut along its m02-m13 diagonal.
// For Kuhn simplices the children are the Kuhn simplices of the half-size cubes.
#pragma once

#include <hip/hip_runtime.h>

namespace nlq {

struct ChildTable {
    // [child][vertex] -> packed (i << 4) | j
    static constexpr unsigned char tri[4][3] = {
        {0x00, 0x01, 0x02}, {0x01, 0x11, 0x12}, {0x02, 0x12, 0x22}, {0x01, 0x02, 0x12}};
    static constexpr unsigned char tet[8][4] = {
        {0x00, 0x01, 0x02, 0x03}, {0x01, 0x11, 0x12, 0x13}, {0x02, 0x12, 0x22, 0x23},
        {0x03, 0x13, 0x23, 0x33}, {0x01, 0x02, 0x03, 0x13}, {0x01, 0x02, 0x12, 0x13},
        {0x02, 0x03, 0x13, 0x23}, {0x02, 0x12, 0x13, 0x23}};
};

__host__ __device__ inline unsigned char child_src(int dim, int child, int vertex)
{
    return dim == 2 ? ChildTable::tri[child][vertex] : ChildTable::tet[child][vertex];
}

// Child `ch` of the simplex with vertices V[nv][ncomp] (row-major), written to
// out[nv][ncomp].
inline void refine_child(int dim, int ncomp, const double *V, int ch, double *out)
{
    const int nv = dim + 1;
    for (int v = 0; v < nv; ++v) {
        const unsigned char s = child_src(dim, ch, v);
        const int i = s >> 4, j = s & 15;
        for (int k = 0; k < ncomp; ++k)
            out[v * ncomp + k] = (i == j) ? V[i * ncomp + k] : (V[i * ncomp + k] + V[j * ncomp + k]) * 0.5;
    }
}

}  // namespace nlq
