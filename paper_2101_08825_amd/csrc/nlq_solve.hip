// Load vector, lifting and the FP64 conjugate-gradient solve of the volume-
// constrained system (Section 2, eqs. (poisson), (A-F), (weak-homo)).
//   F_i  = int_Omega f_h phi_i   (f_h the P1 interpolant of the nodal f)
//   F~_i = F_i - sum_{j in Gamma} A_ij g_j   for free i (lifting, minus sign)
//   A_{Omega,Omega} w = F~_Omega by Jacobi-preconditioned CG; u = w (free), g (Gamma)
#include <cmath>
#include <cstdlib>
#include <mutex>
#include <string>
#include <vector>

#include "nlq_device.hpp"
#include "nlq_box.hpp"
#include "nlq_internal.hpp"

namespace nlq {

namespace {

// Lagrange basis of order ORD at barycentric point lam: P1 lambda_i; P2
// lambda_i (2 lambda_i - 1) at the vertices, 4 lambda_i lambda_j at the edges
// (i < j, lexicographic)
template <int DIM, int ORD>
__device__ __forceinline__ void lagrange_basis(const double *lam, double *phi)
{
    constexpr int NV = DIM + 1;
    if constexpr (ORD == 1) {
#pragma unroll
        for (int i = 0; i < NV; ++i) phi[i] = lam[i];
    } else {
#pragma unroll
        for (int i = 0; i < NV; ++i) phi[i] = lam[i] * (2.0 * lam[i] - 1.0);
        int k = NV;
#pragma unroll
        for (int i = 0; i < NV; ++i)
#pragma unroll
            for (int j = i + 1; j < NV; ++j) phi[k++] = 4.0 * lam[i] * lam[j];
    }
}

// F_i += sum_q w_q |T| f_h(x_q) phi_i(x_q) over the elements T containing i, with
// f_h the interpolant of the nodal f in the element's space (P1 or P2)
template <int DIM, int ORD = 1>
__global__ void k_load(int64_t ne, const int32_t *__restrict__ conn, const double *__restrict__ meas,
                       const double *__restrict__ rule, const double *__restrict__ f,
                       const uint8_t *__restrict__ constrained, double *__restrict__ F)
{
    constexpr int NV = DIM + 1, NQ = DIM == 2 ? 7 : 15;
    constexpr int NB = ORD == 1 ? NV : NV * (NV + 1) / 2;
    const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= ne) return;
    const double *bary = rule;
    const double *w = rule + NQ * NV;
    double fv[NB];
    int32_t id[NB];
#pragma unroll
    for (int v = 0; v < NB; ++v) {
        id[v] = conn[e * NB + v];
        fv[v] = f[id[v]];
    }
    const double me = meas[e];
    double s[NB];
#pragma unroll
    for (int a = 0; a < NB; ++a) s[a] = 0.0;
    for (int q = 0; q < NQ; ++q) {
        double phi[NB];
        lagrange_basis<DIM, ORD>(bary + q * NV, phi);
        double fq = 0.0;
#pragma unroll
        for (int v = 0; v < NB; ++v) fq += fv[v] * phi[v];
#pragma unroll
        for (int a = 0; a < NB; ++a) s[a] += w[q] * fq * phi[a];
    }
#pragma unroll
    for (int a = 0; a < NB; ++a)
        if (!constrained[id[a]]) unsafeAtomicAdd(&F[id[a]], s[a] * me);
}

// Quadrilaterals / hexahedra: F_i += sum_q w_q |det F_e'(g_q)| f_h(g_q) phi_i(g_q)
// with the 3^DIM Gauss rule and the basis values at its points (psi [NB][QS])
template <int DIM, int NB>
__global__ void k_load_box(int64_t ne, const int32_t *__restrict__ conn, const double *__restrict__ vert,
                           const double *__restrict__ rule, const double *__restrict__ psi,
                           const double *__restrict__ f, const uint8_t *__restrict__ constrained,
                           double *__restrict__ F)
{
    constexpr int NQ = DIM == 2 ? 9 : 27, QS = DIM == 2 ? 16 : 32, NC = 1 << DIM;
    const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= ne) return;
    BoxVerts<DIM> P;
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int k = 0; k < DIM; ++k) P.v[c][k] = vert[(c * DIM + k) * ne + e];
    double fv[NB];
    int32_t id[NB];
#pragma unroll
    for (int v = 0; v < NB; ++v) {
        id[v] = conn[e * NB + v];
        fv[v] = f[id[v]];
    }
    double s[NB];
#pragma unroll
    for (int a = 0; a < NB; ++a) s[a] = 0.0;
    for (int q = 0; q < NQ; ++q) {
        const double wq = rule[NQ * DIM + q] * box_jacdet<DIM>(P, rule + q * DIM);
        double fq = 0.0;
#pragma unroll
        for (int v = 0; v < NB; ++v) fq += fv[v] * psi[v * QS + q];
#pragma unroll
        for (int a = 0; a < NB; ++a) s[a] += wq * fq * psi[a * QS + q];
    }
#pragma unroll
    for (int a = 0; a < NB; ++a)
        if (!constrained[id[a]]) unsafeAtomicAdd(&F[id[a]], s[a]);
}

// The same load vector summed per node over its elements in ascending order
// (deterministic mode: no atomics, so F is the same bit for bit every time).
template <int DIM>
__global__ void k_load_ordered(int64_t nn, const int64_t *__restrict__ n2e_off, const int32_t *__restrict__ n2e,
                               const int32_t *__restrict__ conn, const double *__restrict__ meas,
                               const double *__restrict__ rule, const double *__restrict__ f,
                               const uint8_t *__restrict__ constrained, double *__restrict__ F)
{
    constexpr int NV = DIM + 1, NQ = DIM == 2 ? 7 : 15;
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= nn) return;
    const double *bary = rule;
    const double *w = rule + NQ * NV;
    double acc = 0.0;
    if (!constrained[i]) {
        for (int64_t q0 = n2e_off[i]; q0 < n2e_off[i + 1]; ++q0) {
            const int64_t e = n2e[q0];
            double fv[NV];
            int a = 0;
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                const int32_t id = conn[e * NV + v];
                fv[v] = f[id];
                if (id == i) a = v;
            }
            double s = 0.0;
            for (int q = 0; q < NQ; ++q) {
                double fq = 0.0;
#pragma unroll
                for (int v = 0; v < NV; ++v) fq += fv[v] * bary[q * NV + v];
                s += w[q] * fq * bary[q * NV + a];
            }
            acc += s * meas[e];
        }
    }
    F[i] = acc;
}

// one wave per row: F~_i = F_i - sum_{j in Gamma} A_ij g_j (free i), 0 on Gamma
__global__ void __launch_bounds__(256)
k_lift(int64_t n, const int64_t *__restrict__ row_ptr, const int32_t *__restrict__ col,
       const double *__restrict__ val, const uint8_t *__restrict__ constrained,
       const double *__restrict__ g, const double *__restrict__ F, double *__restrict__ Ft)
{
    const int64_t i = static_cast<int64_t>(blockIdx.x) * (blockDim.x / kWave) + threadIdx.x / kWave;
    if (i >= n) return;
    double s = 0.0;
    if (!constrained[i])
        for (int64_t k = row_ptr[i] + lane_id(); k < row_ptr[i + 1]; k += kWave) {
            const int32_t j = col[k];
            if (constrained[j]) s += val[k] * g[j];
        }
    s = wave_sum(s);
    if (lane_id() == 0) Ft[i] = constrained[i] ? 0.0 : F[i] - s;
}

// ---- CG pieces -------------------------------------------------------------

constexpr int kCgThreads = 256;

struct CgScalars {
    double rz, rz_new, pq, rr, alpha, beta, bnorm2;
};

constexpr int kSpmvThreads = 1024;
constexpr int kRowLanes = 16;                               // lanes per matrix row
constexpr int kSpmvRows = kSpmvThreads / kRowLanes;         // rows per block

// Fixed-order sum of nb block partials by one wave (lane l adds partials l,
// l + 64, ..., then a butterfly across the lanes), every lane getting the
// result: the consumers of a reduction compute it themselves, each wave alike
// and without a barrier, instead of a reduction kernel and a scalar kernel in
// between.
__device__ double wave_total(const double *__restrict__ v, int64_t nb)
{
    double s = 0.0;
    for (int64_t b = lane_id(); b < nb; b += kWave) s += v[b];
    return wave_sum(s);
}

// The search direction and its product at once: p = z + beta p_old with beta =
// (new r.z) / (old r.z) from the update's partials (beta = 0 on the first
// iteration, where p_old = z), formed on the fly wherever the product reads it
// and stored by the wave of its row into p_new (p is double-buffered, so no
// row reads a value another row has already replaced); q = A_ff p on free rows
// (0 on Gamma); partial sums of p.q per block (64 rows, 16 lanes each).
__global__ void __launch_bounds__(kSpmvThreads)
k_spmv_dot(int64_t n, const int64_t *__restrict__ row_ptr, const int32_t *__restrict__ col,
           const double *__restrict__ val, const uint8_t *__restrict__ constrained,
           const double *__restrict__ rz_new_part, const double *__restrict__ rz_old_part, int64_t nb,
           int first, const double *__restrict__ z, const double *__restrict__ p_old,
           double *__restrict__ p_new, double *__restrict__ q, double *__restrict__ partial)
{
    __shared__ double red[kSpmvRows];
    double beta = 0.0;
    if (!first) {
        const double rz_new = wave_total(rz_new_part, nb);
        const double rz_old = wave_total(rz_old_part, nb);
        beta = rz_old != 0.0 ? rz_new / rz_old : 0.0;
    }
    const int rl = threadIdx.x % kRowLanes;
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kSpmvRows + threadIdx.x / kRowLanes;
    double s = 0.0;
    bool live = i < n && !constrained[i];
    if (live)
        for (int64_t k = row_ptr[i] + rl; k < row_ptr[i + 1]; k += kRowLanes) {
            const int32_t j = col[k];
            if (!constrained[j]) s += val[k] * fma(beta, p_old[j], z[j]);
        }
    // sum over the row's 16 lanes (a butterfly within each 16-lane group)
    for (int o = kRowLanes / 2; o > 0; o >>= 1) s += __shfl_xor(s, o, kWave);
    double contrib = 0.0;
    if (i < n && rl == 0) {
        const double pi = fma(beta, p_old[i], z[i]);
        p_new[i] = pi;
        q[i] = live ? s : 0.0;
        contrib = live ? s * pi : 0.0;
    }
    if (rl == 0) red[threadIdx.x / kRowLanes] = contrib;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int r = 0; r < kSpmvRows; ++r) t += red[r];
        partial[blockIdx.x] = t;
    }
}

// fixed-order reduction of the block partials (one block): out = sum partial
__global__ void __launch_bounds__(kCgThreads)
k_reduce(int64_t nb, const double *__restrict__ partial, double *__restrict__ out, int nvals)
{
    __shared__ double red[kCgThreads / kWave];
    for (int v = 0; v < nvals; ++v) {
        double s = 0.0;
        for (int64_t b = threadIdx.x; b < nb; b += kCgThreads) s += partial[v * nb + b];
        s = wave_sum(s);
        if (lane_id() == 0) red[threadIdx.x / kWave] = s;
        __syncthreads();
        if (threadIdx.x == 0) {
            double t = 0.0;
            for (int r = 0; r < kCgThreads / kWave; ++r) t += red[r];
            out[v] = t;
        }
        __syncthreads();
    }
}

// alpha = r.z / p.q from the partials of the last update (or the start) and of
// the SpMV; w += alpha p; r -= alpha q; z = D^-1 r; partials of the new r.z
// and of r.r
__global__ void __launch_bounds__(kCgThreads)
k_update(int64_t n, CgScalars *__restrict__ sc, const double *__restrict__ rz_part,
         const double *__restrict__ pq_part, int64_t nb_rows, const double *__restrict__ dinv,
         const double *__restrict__ p, const double *__restrict__ q, double *__restrict__ w,
         double *__restrict__ r, double *__restrict__ z, double *__restrict__ rz_next,
         double *__restrict__ rr_part, int64_t nb)
{
    __shared__ double red[2][kCgThreads / kWave];
    const double rz_old = wave_total(rz_part, nb);
    const double pq = wave_total(pq_part, nb_rows);
    const double a = pq != 0.0 ? rz_old / pq : 0.0;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        sc->pq = pq;
        sc->alpha = a;
    }
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kCgThreads + threadIdx.x;
    double rz = 0.0, rr = 0.0;
    if (i < n) {
        w[i] += a * p[i];
        const double ri = r[i] - a * q[i];
        r[i] = ri;
        const double zi = dinv[i] * ri;
        z[i] = zi;
        rz = ri * zi;
        rr = ri * ri;
    }
    rz = wave_sum(rz);
    rr = wave_sum(rr);
    if (lane_id() == 0) {
        red[0][threadIdx.x / kWave] = rz;
        red[1][threadIdx.x / kWave] = rr;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = 0.0, b = 0.0;
        for (int k = 0; k < kCgThreads / kWave; ++k) {
            a += red[0][k];
            b += red[1][k];
        }
        rz_next[blockIdx.x] = a;
        rr_part[blockIdx.x] = b;
    }
}

// r = F~ (free), z = D^-1 r, p = z, w = 0; dinv from the diagonal; partials r.z, r.r
__global__ void __launch_bounds__(kCgThreads)
k_cg_init(int64_t n, const int64_t *__restrict__ row_ptr, const int32_t *__restrict__ col,
          const double *__restrict__ val, const uint8_t *__restrict__ constrained,
          const double *__restrict__ b, double *__restrict__ dinv, double *__restrict__ w,
          double *__restrict__ r, double *__restrict__ z, double *__restrict__ p,
          double *__restrict__ partial, int64_t nb)
{
    __shared__ double red[2][kCgThreads / kWave];
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kCgThreads + threadIdx.x;
    double rz = 0.0, rr = 0.0;
    if (i < n) {
        double d = 0.0;
        const bool fr = !constrained[i];
        if (fr) {
            int64_t a0 = row_ptr[i], a1 = row_ptr[i + 1] - 1;
            while (a0 <= a1) {
                const int64_t mid = (a0 + a1) >> 1;
                const int32_t c = col[mid];
                if (c == i) { d = val[mid]; break; }
                if (c < i) a0 = mid + 1; else a1 = mid - 1;
            }
        }
        const double di = (fr && d != 0.0) ? 1.0 / d : 0.0;
        dinv[i] = di;
        const double ri = fr ? b[i] : 0.0;
        w[i] = 0.0;
        r[i] = ri;
        z[i] = di * ri;
        p[i] = di * ri;
        rz = ri * di * ri;
        rr = ri * ri;
    }
    rz = wave_sum(rz);
    rr = wave_sum(rr);
    if (lane_id() == 0) {
        red[0][threadIdx.x / kWave] = rz;
        red[1][threadIdx.x / kWave] = rr;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = 0.0, c = 0.0;
        for (int k = 0; k < kCgThreads / kWave; ++k) {
            a += red[0][k];
            c += red[1][k];
        }
        partial[blockIdx.x] = a;
        partial[nb + blockIdx.x] = c;
    }
}

// ---- BiCGSTAB pieces (the two-term forms: A is not symmetric) -------------

// y = A x on the free block: y_i = sum_{j free} A_ij x_j for free i, 0 on Gamma;
// one thread per row
__global__ void __launch_bounds__(256) k_spmv_free(int64_t n, const int64_t *__restrict__ row_ptr,
                                                   const int32_t *__restrict__ col,
                                                   const double *__restrict__ val,
                                                   const uint8_t *__restrict__ cst,
                                                   const double *__restrict__ x, double *__restrict__ y)
{
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double s = 0.0;
    if (!cst[i])
        for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
            const int32_t j = col[k];
            if (!cst[j]) s = fma(val[k], x[j], s);
        }
    y[i] = s;
}

// block partials of a.b and c.d (c may be null), a fixed order within a block
__global__ void __launch_bounds__(kCgThreads) k_dot2(int64_t n, const double *__restrict__ a,
                                                      const double *__restrict__ b,
                                                      const double *__restrict__ c,
                                                      const double *__restrict__ d, double *__restrict__ part)
{
    __shared__ double red[2][kCgThreads / kWave];
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    double x = i < n ? a[i] * b[i] : 0.0;
    double y = (c && i < n) ? c[i] * d[i] : 0.0;
    x = wave_sum(x);
    y = wave_sum(y);
    if (lane_id() == 0) {
        red[0][threadIdx.x / kWave] = x;
        red[1][threadIdx.x / kWave] = y;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double sx = 0.0, sy = 0.0;
        for (int w = 0; w < kCgThreads / kWave; ++w) {
            sx += red[0][w];
            sy += red[1][w];
        }
        part[2 * blockIdx.x] = sx;
        part[2 * blockIdx.x + 1] = sy;
    }
}

// p = r + beta (p - omega v), y = D^{-1} p   (free rows; 0 on Gamma)
__global__ void __launch_bounds__(256) k_bicg_p(int64_t n, const uint8_t *__restrict__ cst,
                                                const double *__restrict__ dinv, const double *__restrict__ r,
                                                const double *__restrict__ v, double beta, double omega,
                                                double *__restrict__ p, double *__restrict__ y)
{
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double pi = cst[i] ? 0.0 : r[i] + beta * (p[i] - omega * v[i]);
    p[i] = pi;
    y[i] = dinv[i] * pi;
}

// s = r - alpha v, z = D^{-1} s
__global__ void __launch_bounds__(256) k_bicg_s(int64_t n, const double *__restrict__ dinv,
                                                const double *__restrict__ r, const double *__restrict__ v,
                                                double alpha, double *__restrict__ s, double *__restrict__ z)
{
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double si = r[i] - alpha * v[i];
    s[i] = si;
    z[i] = dinv[i] * si;
}

// x += alpha y + omega z, r = s - omega t
__global__ void __launch_bounds__(256) k_bicg_x(int64_t n, const double *__restrict__ y,
                                                const double *__restrict__ z, const double *__restrict__ s,
                                                const double *__restrict__ t, double alpha, double omega,
                                                double *__restrict__ x, double *__restrict__ r)
{
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    x[i] += alpha * y[i] + omega * z[i];
    r[i] = s[i] - omega * t[i];
}

__global__ void k_compose_u(int64_t n, const uint8_t *__restrict__ constrained,
                            const double *__restrict__ w, const double *__restrict__ g,
                            double *__restrict__ u)
{
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) u[i] = constrained[i] ? g[i] : w[i];
}

}  // namespace

void launch_load_lift(System &s, hipStream_t st, const double *f_dev, const double *g_dev)
{
    const Mesh &m = *s.mesh;
    const Tables &T = s.ctx->get_tables(m.dim, s.p.lmax);
    const int64_t n = m.n_nodes, ne = m.n_elems;
    if (s.F.empty()) s.F.alloc(s.ctx, sizeof(double) * n);
    if (s.Ft.empty()) s.Ft.alloc(s.ctx, sizeof(double) * n);
    NLQ_HIP(hipMemsetAsync(s.F.as<void>(), 0, sizeof(double) * n, st));
    dim3 g1((ne + 255) / 256), b1(256);
    if (s.p.deterministic && !s.n2e_off.empty() && n > 0) {
        const dim3 gn((n + 255) / 256);
        if (m.dim == 2)
            hipLaunchKernelGGL(k_load_ordered<2>, gn, b1, 0, st, n, s.n2e_off.as<int64_t>(), s.n2e.as<int32_t>(),
                               m.conn.as<int32_t>(), s.meas.as<double>(), T.rule.as<double>(), f_dev,
                               m.constrained.as<uint8_t>(), s.F.as<double>());
        else
            hipLaunchKernelGGL(k_load_ordered<3>, gn, b1, 0, st, n, s.n2e_off.as<int64_t>(), s.n2e.as<int32_t>(),
                               m.conn.as<int32_t>(), s.meas.as<double>(), T.rule.as<double>(), f_dev,
                               m.constrained.as<uint8_t>(), s.F.as<double>());
    } else if (ne == 0) {
    } else if (m.shape == 1) {
        auto kern = m.dim == 2 ? (m.order == 2 ? k_load_box<2, 8> : k_load_box<2, 4>)
                               : (m.order == 2 ? k_load_box<3, 20> : k_load_box<3, 8>);
        hipLaunchKernelGGL(kern, g1, b1, 0, st, ne, m.conn.as<int32_t>(), s.vert.as<double>(),
                           T.boxrule.as<double>(), T.boxpsi[m.order - 1].as<double>(), f_dev,
                           m.constrained.as<uint8_t>(), s.F.as<double>());
    } else {
        auto kern = m.dim == 2 ? (m.order == 2 ? k_load<2, 2> : k_load<2, 1>)
                               : (m.order == 2 ? k_load<3, 2> : k_load<3, 1>);
        hipLaunchKernelGGL(kern, g1, b1, 0, st, ne, m.conn.as<int32_t>(), s.meas.as<double>(), T.rule.as<double>(),
                           f_dev, m.constrained.as<uint8_t>(), s.F.as<double>());
    }
    NLQ_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_lift, dim3((n + 3) / 4), dim3(256), 0, st, n, s.row_ptr.as<int64_t>(),
                       s.col.as<int32_t>(), s.val.as<double>(), m.constrained.as<uint8_t>(), g_dev,
                       s.F.as<double>(), s.Ft.as<double>());
    NLQ_CHECK_LAUNCH();
}

namespace {

// device vectors of one CG solve
struct CgBuffers {
    double *dinv, *w, *r, *z, *p, *p2, *q;
    double *partial;   // block partials: r.z in two slots, r.r, p.q
    CgScalars *sc;
};

int64_t cg_nb_rows(int64_t n) { return (n + kSpmvRows - 1) / kSpmvRows; }
int64_t cg_nb_vec(int64_t n) { return (n + kCgThreads - 1) / kCgThreads; }

// Jacobi CG on the free rows into b; u = w (free), g (Gamma) into u_dst.
// graph: replay blocks of 8 iterations as a HIP graph (else plain launches, in
// the same order and with the same results).
int cg_run(System &s, hipStream_t st, double rtol, int maxit, double *relres, int *converged, const CgBuffers &b,
           bool graph, double *u_dst)
{
    const Mesh &m = *s.mesh;
    const int64_t n = m.n_nodes;
    double *const pbuf[2] = {b.p, b.p2};
    const int64_t nb_rows = cg_nb_rows(n);
    const int64_t nb_vec = cg_nb_vec(n);
    double *const rz_slot[2] = {b.partial, b.partial + nb_vec};
    double *const rr_part = b.partial + 2 * nb_vec;
    double *const pq_part = b.partial + 3 * nb_vec;
    CgScalars *sc = b.sc;
    NLQ_HIP(hipMemsetAsync(sc, 0, sizeof(CgScalars), st));
    const uint8_t *cst = m.constrained.as<uint8_t>();
    hipLaunchKernelGGL(k_cg_init, dim3(nb_vec), dim3(kCgThreads), 0, st, n, s.row_ptr.as<int64_t>(),
                       s.col.as<int32_t>(), s.val.as<double>(), cst, s.Ft.as<double>(), b.dinv, b.w, b.r, b.z,
                       b.p, b.partial, nb_vec);
    NLQ_CHECK_LAUNCH();
    // rz -> sc->rz, rr -> sc->rz_new (temporarily)
    hipLaunchKernelGGL(k_reduce, dim3(1), dim3(kCgThreads), 0, st, nb_vec, b.partial, &sc->rz, 2);
    NLQ_CHECK_LAUNCH();
    CgScalars h{};
    NLQ_HIP(hipMemcpyAsync(&h, sc, sizeof(CgScalars), hipMemcpyDeviceToHost, st));
    NLQ_HIP(hipStreamSynchronize(st));
    const double bnorm = std::sqrt(h.rz_new);
    int it = 0;
    *converged = 0;
    double rn = bnorm;
    if (bnorm == 0.0) {
        *converged = 1;
        *relres = 0.0;
    } else {
        const int check = 8;
        // CG iteration k: 2 kernels, no host work.  Its parity selects the r.z
        // slots (the update writes the next r.z where the product has just read
        // the previous one) and the p buffers (p_old -> p_new).
        auto iteration = [&](int k) {
            const int par = k & 1;
            hipLaunchKernelGGL(k_spmv_dot, dim3(nb_rows), dim3(kSpmvThreads), 0, st, n, s.row_ptr.as<int64_t>(),
                               s.col.as<int32_t>(), s.val.as<double>(), cst, rz_slot[par], rz_slot[1 - par],
                               nb_vec, k == 0 ? 1 : 0, b.z, pbuf[par], pbuf[1 - par], b.q, pq_part);
            hipLaunchKernelGGL(k_update, dim3(nb_vec), dim3(kCgThreads), 0, st, n, sc, rz_slot[par], pq_part,
                               nb_rows, b.dinv, pbuf[1 - par], b.q, b.w, b.r, b.z, rz_slot[1 - par], rr_part, nb_vec);
        };
        // r.r of the last update, for the host's residual check
        auto residual = [&]() {
            hipLaunchKernelGGL(k_reduce, dim3(1), dim3(kCgThreads), 0, st, nb_vec, rr_part, &sc->rr, 1);
        };
        // The residual is checked after iteration 0 and then after every 8
        // iterations.  Iterations 1..8 (the first iteration's kernels differ)
        // and the check's reduction are captured once as a HIP graph (kernels
        // only: no memset or copy inside) and replayed for every later block of
        // 8, whose parities are the same; without the graph the same launches
        // run one by one, in the same order.
        hipGraphExec_t exec = nullptr;
        if (graph && maxit >= 2 * check) {
            hipGraph_t gr = nullptr;
            NLQ_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
            for (int k = 1; k <= check; ++k) iteration(k);
            residual();
            const hipError_t e_end = hipStreamEndCapture(st, &gr);
            if (e_end != hipSuccess) fail(NLQ_EDEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(e_end));
            const hipError_t e_inst = hipGraphInstantiate(&exec, gr, nullptr, nullptr, 0);
            (void)hipGraphDestroy(gr);
            if (e_inst != hipSuccess) fail(NLQ_EDEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e_inst));
        }
        for (it = 0; it < maxit;) {
            if (it == 0) {
                iteration(0);
                residual();
                it = 1;
            } else if (exec && maxit - it >= check) {
                NLQ_HIP(hipGraphLaunch(exec, st));
                it += check;
            } else {
                for (int k = 0; k < check && it < maxit; ++k, ++it) iteration(it);
                residual();
            }
            NLQ_CHECK_LAUNCH();
            NLQ_HIP(hipMemcpyAsync(&h, sc, sizeof(CgScalars), hipMemcpyDeviceToHost, st));
            NLQ_HIP(hipStreamSynchronize(st));
            rn = std::sqrt(h.rr);
            if (rn <= rtol * bnorm) {
                *converged = 1;
                break;
            }
        }
        if (exec) (void)hipGraphExecDestroy(exec);
        *relres = rn / bnorm;
    }
    hipLaunchKernelGGL(k_compose_u, dim3(nb_vec), dim3(kCgThreads), 0, st, n, cst, b.w, s.g.as<double>(), u_dst);
    NLQ_CHECK_LAUNCH();
    NLQ_HIP(hipStreamSynchronize(st));
    return it;
}

// ---- scratch of the allocation-free solve (nlq_solve_noalloc) -------------
// A file-scope device array: every GPU the library runs on holds its own copy
// until the process ends.  Host code never uses its name as an address: the
// device address is taken once per device with hipGetSymbolAddress (the
// context's creation, that device current) and kept here.
constexpr size_t kScratchBytes = size_t(16) << 20;
__device__ __align__(256) char scratch[kScratchBytes];
std::mutex g_scratch_mu;
void *g_scratch_ptr[64] = {};

size_t al256(size_t x) { return (x + 255) & ~size_t(255); }

// bytes of the CG vectors, partials and scalars for n nodes, carved as below
size_t cg_scratch_bytes(int64_t n)
{
    const size_t vec = al256(sizeof(double) * static_cast<size_t>(n));
    const size_t part = al256(sizeof(double) * static_cast<size_t>(3 * cg_nb_vec(n) + cg_nb_rows(n)));
    return 7 * vec + part + al256(sizeof(CgScalars));
}

}  // namespace

// Returns the iteration count; the solution (u = w on free nodes, g on Gamma)
// is left in s.u.  The host checks the residual every 8 iterations.
int cg_solve(System &s, hipStream_t st, double rtol, int maxit, double *relres, int *converged)
{
    const int64_t n = s.mesh->n_nodes;
    if (s.u.empty()) s.u.alloc(s.ctx, sizeof(double) * n);
    DevBuf dinv(s.ctx, sizeof(double) * n, st), w(s.ctx, sizeof(double) * n, st),
        r(s.ctx, sizeof(double) * n, st), z(s.ctx, sizeof(double) * n, st), p(s.ctx, sizeof(double) * n, st),
        p2(s.ctx, sizeof(double) * n, st), q(s.ctx, sizeof(double) * n, st);
    DevBuf partial(s.ctx, sizeof(double) * (3 * cg_nb_vec(n) + cg_nb_rows(n)), st);
    DevBuf scal(s.ctx, sizeof(CgScalars), st);
    const CgBuffers b{dinv.as<double>(), w.as<double>(), r.as<double>(), z.as<double>(), p.as<double>(),
                      p2.as<double>(), q.as<double>(), partial.as<double>(), scal.as<CgScalars>()};
    const char *env = std::getenv("NLQ_CG_GRAPH");
    return cg_run(s, st, rtol, maxit, relres, converged, b, !(env && env[0] == '0'), s.u.as<double>());
}

// Jacobi-preconditioned BiCGSTAB on A_{Omega,Omega} w = F~_Omega for the
// two-term forms (A not symmetric, so CG does not apply); the same stopping rule
// as the CG (||r||_2 <= rtol ||F~||_2, checked every iteration); u into s.u.
int bicgstab_solve(System &s, hipStream_t st, double rtol, int maxit, double *relres, int *converged)
{
    const Mesh &m = *s.mesh;
    const int64_t n = m.n_nodes;
    if (s.u.empty()) s.u.alloc(s.ctx, sizeof(double) * n);
    const int64_t nb_vec = cg_nb_vec(n);
    DevBuf dinv(s.ctx, sizeof(double) * n, st), x(s.ctx, sizeof(double) * n, st), r(s.ctx, sizeof(double) * n, st),
        rh(s.ctx, sizeof(double) * n, st), p(s.ctx, sizeof(double) * n, st), v(s.ctx, sizeof(double) * n, st),
        y(s.ctx, sizeof(double) * n, st), sv(s.ctx, sizeof(double) * n, st), z(s.ctx, sizeof(double) * n, st),
        t(s.ctx, sizeof(double) * n, st), part(s.ctx, sizeof(double) * 2 * nb_vec, st);
    const uint8_t *cst = m.constrained.as<uint8_t>();
    std::vector<double> hp(2 * nb_vec);
    auto dot2 = [&](const double *a, const double *b, const double *c, const double *d, double *o0, double *o1) {
        hipLaunchKernelGGL(k_dot2, dim3(nb_vec), dim3(kCgThreads), 0, st, n, a, b, c, d, part.as<double>());
        NLQ_CHECK_LAUNCH();
        NLQ_HIP(hipMemcpyAsync(hp.data(), part.as<void>(), sizeof(double) * 2 * nb_vec, hipMemcpyDeviceToHost, st));
        NLQ_HIP(hipStreamSynchronize(st));
        double a0 = 0.0, a1 = 0.0;
        for (int64_t k = 0; k < nb_vec; ++k) {
            a0 += hp[2 * k];
            a1 += hp[2 * k + 1];
        }
        *o0 = a0;
        if (o1) *o1 = a1;
    };
    // the CG's initialisation gives D^{-1}, x = 0, r = F~ (free rows); its
    // other outputs are overwritten below
    hipLaunchKernelGGL(k_cg_init, dim3(nb_vec), dim3(kCgThreads), 0, st, n, s.row_ptr.as<int64_t>(),
                       s.col.as<int32_t>(), s.val.as<double>(), cst, s.Ft.as<double>(), dinv.as<double>(),
                       x.as<double>(), r.as<double>(), z.as<double>(), p.as<double>(), part.as<double>(), nb_vec);
    NLQ_CHECK_LAUNCH();
    NLQ_HIP(hipMemcpyAsync(rh.as<void>(), r.as<void>(), sizeof(double) * n, hipMemcpyDeviceToDevice, st));
    NLQ_HIP(hipMemsetAsync(p.as<void>(), 0, sizeof(double) * n, st));
    NLQ_HIP(hipMemsetAsync(v.as<void>(), 0, sizeof(double) * n, st));
    double bb = 0.0;
    dot2(r.as<double>(), r.as<double>(), nullptr, nullptr, &bb, nullptr);
    const double bnorm = std::sqrt(bb);
    *converged = 0;
    int it = 0;
    double rn = bnorm;
    const dim3 g((n + 255) / 256), b(256);
    if (bnorm == 0.0) {
        *converged = 1;
    } else {
        double rho = 1.0, alpha = 1.0, omega = 1.0;
        for (it = 0; it < maxit; ++it) {
            double rho_new = 0.0;
            dot2(rh.as<double>(), r.as<double>(), nullptr, nullptr, &rho_new, nullptr);
            if (rho_new == 0.0) break;
            const double beta = it == 0 ? 0.0 : (rho_new / rho) * (alpha / omega);
            hipLaunchKernelGGL(k_bicg_p, g, b, 0, st, n, cst, dinv.as<double>(), r.as<double>(), v.as<double>(), beta,
                               omega, p.as<double>(), y.as<double>());
            hipLaunchKernelGGL(k_spmv_free, g, b, 0, st, n, s.row_ptr.as<int64_t>(), s.col.as<int32_t>(),
                               s.val.as<double>(), cst, y.as<double>(), v.as<double>());
            NLQ_CHECK_LAUNCH();
            double rv = 0.0;
            dot2(rh.as<double>(), v.as<double>(), nullptr, nullptr, &rv, nullptr);
            if (rv == 0.0) break;
            alpha = rho_new / rv;
            hipLaunchKernelGGL(k_bicg_s, g, b, 0, st, n, dinv.as<double>(), r.as<double>(), v.as<double>(), alpha,
                               sv.as<double>(), z.as<double>());
            hipLaunchKernelGGL(k_spmv_free, g, b, 0, st, n, s.row_ptr.as<int64_t>(), s.col.as<int32_t>(),
                               s.val.as<double>(), cst, z.as<double>(), t.as<double>());
            NLQ_CHECK_LAUNCH();
            double ts = 0.0, tt = 0.0;
            dot2(t.as<double>(), sv.as<double>(), t.as<double>(), t.as<double>(), &ts, &tt);
            omega = tt > 0.0 ? ts / tt : 0.0;
            hipLaunchKernelGGL(k_bicg_x, g, b, 0, st, n, y.as<double>(), z.as<double>(), sv.as<double>(),
                               t.as<double>(), alpha, omega, x.as<double>(), r.as<double>());
            NLQ_CHECK_LAUNCH();
            double rr = 0.0;
            dot2(r.as<double>(), r.as<double>(), nullptr, nullptr, &rr, nullptr);
            rn = std::sqrt(rr);
            rho = rho_new;
            if (rn <= rtol * bnorm) {
                *converged = 1;
                ++it;
                break;
            }
            if (omega == 0.0) break;
        }
    }
    *relres = bnorm > 0.0 ? rn / bnorm : 0.0;
    hipLaunchKernelGGL(k_compose_u, dim3(nb_vec), dim3(kCgThreads), 0, st, n, cst, x.as<double>(),
                       s.g.as<double>(), s.u.as<double>());
    NLQ_CHECK_LAUNCH();
    NLQ_HIP(hipStreamSynchronize(st));
    return it;
}

void noalloc_scratch_init(int device)
{
    if (device < 0 || device >= 64) fail(NLQ_EINVAL, "device id beyond the scratch table");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[device]) return;
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) fail(NLQ_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[device] = ptr;
}

size_t noalloc_scratch_limit() { return kScratchBytes; }

int cg_solve_noalloc(System &s, hipStream_t st, double rtol, int maxit, double *relres, int *converged,
                     double *u_dev)
{
    const int64_t n = s.mesh->n_nodes;
    const size_t need = cg_scratch_bytes(n);
    if (need > kScratchBytes)
        fail(NLQ_EINVAL, "nlq_solve_noalloc: " + std::to_string(n) + " nodes need " + std::to_string(need) +
                             " bytes of scratch, more than its " + std::to_string(kScratchBytes));
    char *base = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        base = static_cast<char *>(g_scratch_ptr[s.ctx->device]);
    }
    if (!base) fail(NLQ_EDEVICE, "scratch of this device not set up (context creation takes its address)");
    const size_t vec = al256(sizeof(double) * static_cast<size_t>(n));
    double *v[7];
    for (int k = 0; k < 7; ++k) v[k] = reinterpret_cast<double *>(base + k * vec);
    double *partial = reinterpret_cast<double *>(base + 7 * vec);
    CgScalars *sc = reinterpret_cast<CgScalars *>(
        base + 7 * vec + al256(sizeof(double) * static_cast<size_t>(3 * cg_nb_vec(n) + cg_nb_rows(n))));
    const CgBuffers b{v[0], v[1], v[2], v[3], v[4], v[5], v[6], partial, sc};
    return cg_run(s, st, rtol, maxit, relres, converged, b, false, u_dev);
}

}  // namespace nlq
