// Hot path of the assembly: for every ordered pair (l, m) of the pair list,
// Algorithm 1 (Section 5) refines the outer element l by midpoints, classifying
// each sub-element s against the whole inner element m with the bbox distances
// of Section 5.1; every settled (s, m) is integrated with the degree-5 rule on s
// and on m, and the four-term integrand of eq. (Aij-support2) (or the two-term
// form of the Corollary) is accumulated into the pair's blocks.
//
// Work decomposition (one GPU, persistent launch):
//   * a workgroup of kWaves waves takes work items (an outer element l, or a
//     part of its pair list) from a global counter, stages the CSR rows of l's
//     nodes in LDS, and its waves take the pairs (l, m), m in J_l, from an LDS
//     counter;
//   * a wave walks the refinement tree of its pair depth first with a bounded
//     stack in LDS, up to 64 sub-elements a pass: lanes classify them in FP64
//     (every rounding as written, so the leaf set is reproducible bit for bit),
//     wave ballots + prefix counts push the refined ones' children and append
//     the leaves to a leaf buffer;
//   * the pair's leaves are integrated in batches of 64 outer points staged in
//     LDS (the table loads of the next batch are issued before the current
//     batch runs):
//       plain  (FP64): each lane owns one inner point and a slice of the batch,
//                      evaluates gamma_eps in FP64 and accumulates
//                      H_ib = sum_a P_i(a) g_ab, Q_kb = sum_a P_k(a) g_ab in FP64
//                      (3D P2 and box elements: the same sums on the FP64
//                      matrix cores, v_mfma_f64_16x16x4f64);
//       mixed  (FP32): anchor-relative FP32 coordinates, gamma_eps in FP32 and the
//                      contraction H = P^T G on the matrix cores
//                      (v_mfma_f32_16x16x4f32), flushed to FP64 every two batches;
//     with P_i(a) = w_a 2^{-N(lev-1)} lambda_i(x_a) (rows i < N+1) and
//     P_k(a) = w_a 2^{-N(lev-1)} lambda_i lambda_j (k = off-diagonal pair i < j);
//   * FP64 epilogue: S = C |E_l| |E_m|,
//       B_lm[i][j] = -S sum_b H_ib w_b psi_j(y_b)
//       B_mm[i][j] =  S sum_b w_b psi_i psi_j sum_i' H_i'b
//       B_ll[i][j] =  S sum_b Q_(ij)b w_b  (i != j),
//       B_ll[i][i] =  S sum_b (H_ib - sum_{j != i} Q_(ij)b) w_b
//     (partition of unity: lambda_i^2 = lambda_i - sum_{j != i} lambda_i lambda_j),
//     one output per lane as a dot product over b with a constant row;
//   * accumulation (FP64): SYM4 blocks are symmetric and B_ml = B_lm^T, so the
//     launch builds a half matrix R with A = R + R^T: B_lm goes to (l_i, m_j)
//     through the LDS-cached row of l_i (or its sampled columns), the upper triangles of B_mm (per pair)
//     and B_ll (per outer element, summed in LDS) go to a per-element array;
//     a fold pass adds that array to R and a last pass forms R + R^T in place,
//     which makes A symmetric bit for bit.  The two-term form writes its
//     entries where they belong and skips the last pass.
#include <algorithm>
#include <cmath>
#include <type_traits>

#include "nlq_box.hpp"
#include "nlq_device.hpp"
#include "nlq_internal.hpp"
#include "nlq_p2.hpp"
#include "nlq_refine.hpp"

namespace nlq {

namespace {

constexpr int kWaves = 4;
constexpr int kThreads = kWaves * kWave;
// leaf buffer entries per wave (a launch parameter; at least one wave's pushes)
constexpr int kLeafCapMin = 64, kLeafCapMax = 512;
constexpr int kBatch = 64;
// waves per SIMD requested from the register allocator: variant 0 (the default:
// 5 in 2D, 4 for the 3D FP32 path, 3 for the 3D FP64 path) and variant 1 -- one
// wave more for the 2D FP32 path (fewer registers, more latency hiding), one
// fewer for the others (more registers, fewer spills); the autotuner picks per
// workload
template <int DIM, int PREC, int OCC> constexpr int waves_per_eu()
{
    constexpr int base = DIM == 2 ? 5 : (PREC == 1 ? 4 : 3);
    return base + (OCC ? ((DIM == 2 && PREC == 1) ? 1 : -1) : 0);
}

template <int DIM> struct Shape {
    static constexpr int NV = DIM + 1;
    static constexpr int NQ = DIM == 2 ? 7 : 15;
    static constexpr int NCH = 1 << DIM;
    static constexpr int NOFF = NV * (NV - 1) / 2;
    static constexpr int NR = NV + NOFF;
};

// What the element order changes: nodes per element NB, contraction rows NR
// (P1: lambda_i and lambda_i lambda_j; P2: the quartic monomials of nlq_p2.hpp),
// upper-triangle slots NU of a diagonal block, per-pair outputs NOUT
// (B_lm, then the upper triangles of B_mm and B_ll).
template <int DIM, int ORD> struct OShape {
    static constexpr int NV = DIM + 1;
    static constexpr int NB = ORD == 1 ? NV : p2_nodes(DIM);
    static constexpr int NR = ORD == 1 ? Shape<DIM>::NR : p2_monomials(DIM);
    static constexpr int NU = NB * (NB + 1) / 2;
    static constexpr int NOUT = NB * NB + 2 * NU;
    // P2 epilogue rows mapped from the monomial rows (make_p2_map)
    static constexpr int NRX = NU + NB + 1;
};

struct AsmArgs {
    int64_t ne;
    const int64_t *pair_off;
    const int32_t *pair_m;
    const double *vert;   // [nv*dim][ne]
    const double *lo;     // [dim][ne]
    const double *hi;
    const double *dlo;    // [dim][ne] boxes the refine test measures the gap to:
    const double *dhi;    // lo, hi, or the quadrature-point boxes (min_dist_l2 = 2)
    const double *qlo;    // [dim][ne] boxes of the elements' quadrature points
    const double *qhi;    // (the zero test of the children at L_max)
    const double *meas;
    const int32_t *conn;
    const int64_t *row_ptr;
    const int32_t *col;
    const int32_t *tmap;
    const int32_t *elpos;
    double *val;
    int nb;               // nodes per element (conn stride): dim + 1 (P1), (dim+1)(dim+2)/2 (P2),
                          // 2^dim (Q1), 8 / 20 (serendipity)
    const double *p2map;  // P2: [NRX][NR] map from the monomial rows to the epilogue rows
    const double *boxrule;   // boxes: the 3^dim rule, [nq][dim] points then [nq] weights
    const double *boxpsi;    // boxes: [nb][qs] basis at the rule points
    const double *boxphi;    // boxes: [nb][nr] basis functions over the product monomials
    const double *boxprod;   // boxes: [nu][nr] products of two basis functions
    const double *lam64;  // [sub][nq][nv]
    const float *pt32;    // rows of the FP32 contraction per point (see the tables)
    int pt32_zero;        // its zero row
    double *pb;           // deterministic mode: per-pair outputs [pair - pb_base][NV^2 + 2 NR], else null
    double dpe_sq;        // s* of delta + eps for the Euclidean box gap
    int min_l2;           // J^ref test with the Euclidean box gap (ablation): 1 to the
                          // inner element's box, 2 to its quadrature points' box
    int64_t pb_base;
    const double *rule;   // [nq][nv] barycentric points, then [nq] weights
    double delta, eps, dme, dpe, dme2, dpe2, C;
    double inv_eps, inv_delta2;   // 1 / eps, 1 / delta^2
    double dme_sq;        // s* with (sqrt(s) < delta - eps) <=> (s < s*), s >= 0
    double *dmm;          // [ne][NU] upper-triangle diagonal-block sums per element
    float f_inv_eps, f_delta_over_eps, f_inv_delta2;
    float f_dme2, f_dpe2;  // (delta - eps)^2, (delta + eps)^2 in FP32: the band test of a tile register
    int lmin, lmax, form;
    int split;            // work items per outer element (pair list cut in equal parts)
    int capl;             // traversal stack entries of this system (see make_args)
    int rowcap;           // LDS row cache this system would like
    AsmCounters *counters;
    int64_t n_explicit;
    const int32_t *ex_l;
    const int32_t *ex_m;
    double *ex_out;
};

// Per-system arguments are read from device memory through the constant
// address space, so that every field is a scalar load of a uniform address.
typedef const __attribute__((address_space(4))) AsmArgs CArgs;

// One launch integrates segments of outer elements [seg_lo, seg_lo + n) of one
// or more systems (same dim, precision and kernel).  Every outer element of a
// system is cut into `split` work items (equal parts of its pair list), so a
// segment holds n * split items; work item w of the flat counter lies in the
// segment k with seg_start[k] <= w < seg_start[k+1].
constexpr int kMaxSeg = 32;
// largest part of one J_l handled as one work item (a workgroup's unit of work)
constexpr int64_t kPairsPerItem = 512;
// logical capacity of a wave's traversal stack (entries): a tuning parameter
constexpr int kStackCapMin = 64, kStackCapMax = 1024;
struct LaunchArgs {
    const AsmArgs *sys;
    const int32_t *seg_sys;
    const int64_t *seg_lo;
    const int64_t *seg_start;   // [nseg + 1]
    int nseg;
    int capl;                   // LDS layout: traversal stack entries per wave
    int rowcap;                 // LDS layout: cached CSR row capacity
    int leafcap;                // LDS layout: leaf buffer entries per wave
    unsigned int *counter;
};

__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <class T> __device__ __forceinline__ T bcast0(T v) { return __shfl(v, 0, kWave); }

__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// -------------------------------------------------------------- mollifier

// xi of Section 3, eq. (mollifier), the degree-9 polynomial
// (128 + 315 r - 420 r^3 + 378 r^5 - 180 r^7 + 35 r^9) / 256 at r = (delta - d) / eps
// (1 at the inner band edge, 0 at the outer), in the factored form that keeps its
// relative accuracy where it is small (see xi32 below): with s = 1 - |r|,
// xi(-|r|) = s^5 Q(s) and xi(|r|) = 1 - xi(-|r|).
__device__ __forceinline__ double xi64(double r)
{
    const double sgn = copysign(1.0, r);
    const double t = 0.5 - fabs(r);
    const double ss = sgn - r;    // sgn * s
    double q = 35.0 / 256.0;
    q = fma(q, t, -245.0 / 256.0);
    q = fma(q, t, 660.0 / 256.0);
    q = fma(q, t, -3275.0 / 1024.0);
    q = fma(q, t, 6413.0 / 4096.0);
    const double s2 = ss * ss;
    return fma(-(s2 * s2), ss * q, fma(sgn, 0.5, 0.5));
}

// xi in FP32 with relative accuracy where it is small.  xi' = (315/256)(1 - r^2)^4
// has zeros of order four at r = -1 and r = 1, so xi has a zero of order five at
// r = -1 and, with sigma = 1 - |r|,
//   xi(-|r|) = sigma^5 Q(sigma),  Q(sigma) = (1008 - 1680 sigma + 1080 sigma^2
//                                            - 315 sigma^3 + 35 sigma^4) / 256,
// and xi(|r|) = 1 - xi(-|r|) (xi - 1/2 is odd).  Q is evaluated by Horner in
// t = sigma - 1/2 = 1/2 - |r| (coefficients exact in FP32), which keeps its
// cancellation small on [0, 1]: |error| <= 1.8e-7 everywhere and <= 5e-7
// relative, down to xi = 0 at the outer band edge (the plain Horner form in r,
// 1/2 + r p(r^2), carries an absolute error of ~1e-7 there, where xi ~ (1+r)^5).
// At |r| = 1 sigma is 0, so the clamped plateau and outside give exactly 1 and 0.
// The two sides are one expression: with g = sign(r) (+1 at r = +0) and
// m = (1 + g) / 2, xi = m - g sigma^5 Q, where g sigma = g - r is formed exactly as
// sigma would be; both sides then round as 1 - sigma^5 Q (one multiply-add) and
// sigma^5 Q (one multiply) would, without a compare and a select.
__device__ __forceinline__ float xi32(float r)
{
    const float sgn = copysignf(1.0f, r);
    const float t = 0.5f - fabsf(r);
    const float ss = sgn - r;    // sgn * sigma
    float q = 35.0f / 256.0f;
    q = fmaf(q, t, -245.0f / 256.0f);
    q = fmaf(q, t, 660.0f / 256.0f);
    q = fmaf(q, t, -3275.0f / 1024.0f);
    q = fmaf(q, t, 6413.0f / 4096.0f);
    const float s2 = ss * ss;
    return fmaf(-(s2 * s2), ss * q, fmaf(sgn, 0.5f, 0.5f));
}

// The constants of the FP64 kernel evaluation, copied into vector registers once
// per batch: read through the argument block inside the loops, their scalar
// loads would share a wait counter with the LDS loads of the next step's
// operands and hold those back.
struct Band64 {
    double delta, inv_eps, dme2, dpe2, inv_delta2;
};
__device__ __forceinline__ double in_vgpr64(double x)
{
    double r;
    asm("v_mov_b64 %0, %1" : "=v"(r) : "v"(x));
    return r;
}
__device__ __forceinline__ Band64 band64(const CArgs &A)
{
    return Band64{in_vgpr64(A.delta), in_vgpr64(A.inv_eps), in_vgpr64(A.dme2), in_vgpr64(A.dpe2),
                  in_vgpr64(A.inv_delta2)};
}

// Square root of a squared distance inside the band (a normal FP64 number far
// from 0 and from overflow, so no rescaling is needed): Goldschmidt's iteration
// from the hardware reciprocal square root estimate y ~ 1/sqrt(x), with g -> sqrt(x)
// and h -> 1/(2 sqrt(x)) refined together, then two Newton corrections of g
// through the residual x - g^2.
__device__ __forceinline__ double sqrt_band(double x)
{
    const double y = __builtin_amdgcn_rsq(x);
    double g = x * y, h = 0.5 * y;
    const double r = fma(-h, g, 0.5);
    g = fma(g, r, g);
    h = fma(h, r, h);
    double e = fma(-g, g, x);
    g = fma(e, h, g);
    e = fma(-g, g, x);
    return fma(e, h, g);
}

// gamma_eps / C at squared distance d2: eta * mu (FP64), without branches.  d2 is
// clamped into the band's range [dme2, dpe2] before the square root, the band
// coordinate r = (delta - d) / eps (as (delta - d) * (1 / eps)) to [-1, 1], where
// xi is exactly 1 and 0; the plateau and the outside are then selected on d2
// itself (dme2 and dpe2 are (delta -+ eps)^2 moved outwards by a relative 1e-12,
// so a d2 between either pair of values gives the clamped r of its side).
template <int ETA> __device__ __forceinline__ double kernel64(const Band64 &K, double d2)
{
    const double d = sqrt_band(fmin(fmax(d2, K.dme2), K.dpe2));
    const double xi = xi64(fmin(fmax((K.delta - d) * K.inv_eps, -1.0), 1.0));
    double mu = d2 < K.dme2 ? 1.0 : (d2 > K.dpe2 ? 0.0 : xi);
    if (ETA == NLQ_ETA_GAUSS) mu *= exp(-d2 * K.inv_delta2);
    return mu;
}

// mu at distance d (FP32), without branches: the band coordinate
// r = (delta - d) / eps is clamped to [-1, 1], where the factored form of xi
// gives exactly 0 and 1 (s = 1 - |r| is 0 there), so the plateau and the
// outside need no separate case.  Every evaluation costs the same, but a wave
// no longer diverges between the three cases (a leaf that straddles the band
// nearly always holds all three).
// doe = delta / eps, held in a vector register by the caller (a multiply-add
// reads at most one scalar register, and 1 / eps is the other operand).
__device__ __forceinline__ float mu32(CArgs &A, float d, float doe)
{
    return xi32(__builtin_amdgcn_fmed3f(fmaf(-d, A.f_inv_eps, doe), -1.0f, 1.0f));
}

// a wave-uniform value copied into a vector register, so that the compiler does
// not re-copy it from its scalar register inside a loop
__device__ __forceinline__ float in_vgpr(float x)
{
    float r;
    asm("v_mov_b32 %0, %1" : "=v"(r) : "v"(x));
    return r;
}

// gamma_eps / C at squared distance d2 >= 0 (FP32; sqrt to ~1 ulp)
template <int ETA> __device__ __forceinline__ float kernel32(CArgs &A, float d2, float doe)
{
    float g = mu32(A, __builtin_amdgcn_sqrtf(d2), doe);
    if (ETA == NLQ_ETA_GAUSS) g *= __expf(-d2 * A.f_inv_delta2);
    return g;
}

// gamma_eps / C of the 64 squared distances one register holds across the wave
// (one per lane), with the band test taken once per register: when no lane's
// distance is in the band, mu is a step (1 on the plateau, 0 beyond) and the
// square root and xi are skipped for the whole register (a wave-uniform
// branch).  Both sides of the branch give the same values up to the band edges,
// where xi is within (1e-7)^5 of 1 or 0 in FP32.  FP64 here, FP32 below.
template <int ETA> __device__ __forceinline__ double kernel64_reg(const Band64 &K, double d2)
{
    const bool plateau = d2 < K.dme2;
    const bool band = !plateau && d2 <= K.dpe2;
    if (__builtin_amdgcn_ballot_w64(band)) return kernel64<ETA>(K, d2);
    if (ETA == NLQ_ETA_GAUSS) return plateau ? exp(-d2 * K.inv_delta2) : 0.0;
    return plateau ? 1.0 : 0.0;
}

template <int ETA> __device__ __forceinline__ float kernel32_reg(CArgs &A, float d2, float doe)
{
    const bool plateau = d2 < A.f_dme2;
    const bool band = !plateau && d2 <= A.f_dpe2;
    if (__builtin_amdgcn_ballot_w64(band)) return kernel32<ETA>(A, d2, doe);
    float g = plateau ? 1.0f : 0.0f;
    if (ETA == NLQ_ETA_GAUSS) g = plateau ? __expf(-d2 * A.f_inv_delta2) : 0.0f;
    return g;
}

// -------------------------------------------------------------- geometry

template <int DIM> struct Simplex {
    double v[DIM + 1][DIM];
};

// Child c of a tetrahedron by the midpoint rule: child vertex v is (V_i + V_j)
// * 0.5, rounded as written, for the pair (i, j) of the child table (i == j: the
// vertex itself, exactly, as (x + x) * 0.5 = x).  The two parent vertices are
// picked by selects on i and j, unpacked two bits per child from constants, so
// only the parent and the child are live (forming all ten points first held
// sixty more registers).
__device__ __forceinline__ Simplex<3> tet_child_of(const Simplex<3> &S, int c)
{
    Simplex<3> out;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        unsigned pi = 0, pj = 0;
#pragma unroll
        for (int cc = 0; cc < 8; ++cc) {
            pi |= static_cast<unsigned>(child_src(3, cc, v) >> 4) << (2 * cc);
            pj |= static_cast<unsigned>(child_src(3, cc, v) & 15) << (2 * cc);
        }
        const int i = static_cast<int>((pi >> (2 * c)) & 3u), j = static_cast<int>((pj >> (2 * c)) & 3u);
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const double x = i == 0 ? S.v[0][k] : (i == 1 ? S.v[1][k] : (i == 2 ? S.v[2][k] : S.v[3][k]));
            const double y = j == 0 ? S.v[0][k] : (j == 1 ? S.v[1][k] : (j == 2 ? S.v[2][k] : S.v[3][k]));
            out.v[v][k] = __dmul_rn(__dadd_rn(x, y), 0.5);
        }
    }
    return out;
}

// child `c` of S by the midpoint rule, (V_i + V_j) * 0.5 rounded as written.
// Triangles: every edge midpoint is formed once and the child's vertices are
// chosen by select chains on c, so all table indices are compile-time
// constants and the simplex stays in registers.
template <int DIM>
__device__ __forceinline__ Simplex<DIM> child_of(const Simplex<DIM> &S, int c)
{
    if constexpr (DIM == 3) {
        return tet_child_of(S, c);
    } else {
        constexpr int NV = DIM + 1;
        double M[NV][NV][DIM];
#pragma unroll
        for (int i = 0; i < NV; ++i)
#pragma unroll
            for (int j = 0; j < NV; ++j)
#pragma unroll
                for (int k = 0; k < DIM; ++k)
                    M[i][j][k] = (i == j) ? S.v[i][k]
                                          : (i < j ? __dmul_rn(__dadd_rn(S.v[i][k], S.v[j][k]), 0.5) : 0.0);
        // the triangle table (corner children, then the middle one) as two-bit
        // select trees with its repeated entries merged: 7 selects per
        // coordinate instead of 9
        Simplex<DIM> out;
        const bool b0 = (c & 1) != 0, b1 = (c & 2) != 0;
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            out.v[0][k] = b0 ? M[0][1][k] : (b1 ? M[0][2][k] : M[0][0][k]);
            out.v[1][k] = b1 ? (b0 ? M[0][2][k] : M[1][2][k]) : (b0 ? M[1][1][k] : M[0][1][k]);
            out.v[2][k] = b0 ? M[1][2][k] : (b1 ? M[2][2][k] : M[0][2][k]);
        }
        return out;
    }
}

// first index of level lev in the sub-element tables (level 1 = the element at
// 0; children of local index i at local NCH i + c): (NCH^(lev-1) - 1) / (NCH - 1)
template <int DIM> __device__ __forceinline__ int level_offset(int lev)
{
    constexpr int NCH = 1 << DIM;
    return ((1 << (DIM * (lev - 1))) - 1) / (NCH - 1);
}

// The geometry of an element by shape: a simplex (DIM + 1 vertices, midpoint
// children of child_of) or a box (2^DIM corners in tensor order, children of
// box_child_of).
template <int DIM, int SHP> struct Geo {
    using type = Simplex<DIM>;
    static constexpr int NV = DIM + 1;
};
template <int DIM> struct Geo<DIM, 1> {
    using type = BoxVerts<DIM>;
    static constexpr int NV = 1 << DIM;
};
template <int DIM, int SHP>
__device__ __forceinline__ typename Geo<DIM, SHP>::type geo_child_of(const typename Geo<DIM, SHP>::type &S, int c)
{
    if constexpr (SHP == 1) return box_child_of<DIM>(S, c);
    else return child_of<DIM>(S, c);
}

// Children of a box whose contributions are all exact zeros (as zero_children
// below): each child formed by box_child_of, its box against the quadrature
// points' box.
template <int DIM>
__device__ __forceinline__ uint32_t zero_children_box(CArgs &A, const BoxVerts<DIM> &S, const double *qlo,
                                                      const double *qhi)
{
    uint32_t z = 0;
#pragma unroll 1
    for (int c = 0; c < (1 << DIM); ++c) {
        const BoxVerts<DIM> B = box_child_of<DIM>(S, c);
        double acc = 0.0;
#pragma unroll
        for (int k = 0; k < DIM; ++k) {
            double lo = B.v[0][k], hi = B.v[0][k];
#pragma unroll
            for (int v = 1; v < (1 << DIM); ++v) {
                lo = fmin(lo, B.v[v][k]);
                hi = fmax(hi, B.v[v][k]);
            }
            const double g = fmax(0.0, fmax(__dsub_rn(lo, qhi[k]), __dsub_rn(qlo[k], hi)));
            acc = __dadd_rn(acc, __dmul_rn(g, g));
        }
        z |= acc >= A.dpe_sq ? (1u << c) : 0u;
    }
    return z;
}

// Children of a sub-element whose contributions are all exact zeros: bit c of
// the result is set when child c's box lies at Euclidean distance >= delta + eps
// from the box of the inner element's quadrature points (every point pair of
// the child then lies beyond the kernel's support, so Integration(child, m) adds
// zeros).  Only children at L_max are tested: Algorithm 1 integrates them all,
// and skipping such a child changes no value.  Child vertices are the parent's
// vertices and edge midpoints, (V_i + V_j) * 0.5 rounded as written; each
// coordinate is formed once and every child box updated from it.
template <int DIM>
__device__ __forceinline__ uint32_t zero_children(CArgs &A, const Simplex<DIM> &S, const double *qlo,
                                                  const double *qhi)
{
    constexpr int NV = DIM + 1, NCH = 1 << DIM;
    double acc[NCH];
#pragma unroll
    for (int c = 0; c < NCH; ++c) acc[c] = 0.0;
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
        double P[NV][NV];
#pragma unroll
        for (int i = 0; i < NV; ++i)
#pragma unroll
            for (int j = i; j < NV; ++j)
                P[i][j] = i == j ? S.v[i][k] : __dmul_rn(__dadd_rn(S.v[i][k], S.v[j][k]), 0.5);
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
            double lo = 0.0, hi = 0.0;
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                const int src = child_src(DIM, c, v);
                const double x = P[src >> 4][src & 15];
                lo = v == 0 ? x : fmin(lo, x);
                hi = v == 0 ? x : fmax(hi, x);
            }
            const double g = fmax(0.0, fmax(__dsub_rn(lo, qhi[k]), __dsub_rn(qlo[k], hi)));
            acc[c] = __dadd_rn(acc[c], __dmul_rn(g, g));
        }
    }
    uint32_t z = 0;
#pragma unroll
    for (int c = 0; c < NCH; ++c) z |= acc[c] >= A.dpe_sq ? (1u << c) : 0u;
    return z;
}

// 0 = drop, 1 = integrate now (J^int), 2 = refine (J^ref): Algorithm 1.
// The sub-element's vertices are formed by the midpoint recursion from the
// root, or from its ancestor at level min(lev, memo_lev) whose vertices the
// memo holds (formed by the same recursion; memo_lev < 2: no memo).  For a
// refined sub-element one level above L_max, *zero receives the children whose
// integrals are all zeros (zero_children); otherwise it is left alone.
template <int DIM, int SHP = 0>
__device__ __forceinline__ int classify(CArgs &A, const typename Geo<DIM, SHP>::type root, const double *memo,
                                        int memo_lev, int lev, uint32_t local, const double *mlo,
                                        const double *mhi, const double *dlo, const double *dhi,
                                        const double *qlo, const double *qhi, uint32_t *zero)
{
    constexpr int NCH = 1 << DIM, NV = Geo<DIM, SHP>::NV;
    typename Geo<DIM, SHP>::type S = root;
    int d = lev - 2;   // digits of `local` below the start node
    if (lev >= 2 && memo_lev >= 2) {
        const int la = lev < memo_lev ? lev : memo_lev;
        const int idx = level_offset<DIM>(la) - 1 + static_cast<int>(local >> (DIM * (lev - la)));
        const double *src = memo + idx * NV * DIM;
#pragma unroll
        for (int v = 0; v < NV; ++v)
#pragma unroll
            for (int k = 0; k < DIM; ++k) S.v[v][k] = src[v * DIM + k];
        d = lev - la - 1;
    }
    for (; d >= 0; --d) {
        const int c = (local >> (DIM * d)) & (NCH - 1);
        S = geo_child_of<DIM, SHP>(S, c);
    }
    double slo[DIM], shi[DIM];
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
        double a = S.v[0][k], b = S.v[0][k];
#pragma unroll
        for (int v = 1; v < NV; ++v) {
            a = fmin(a, S.v[v][k]);
            b = fmax(b, S.v[v][k]);
        }
        slo[k] = a;
        shi[k] = b;
    }
    if (aprx_max_sq<DIM>(slo, shi, mlo, mhi) < A.dme_sq) return 1;
    if (A.min_l2 ? box_gap_sq<DIM>(slo, shi, dlo, dhi) < A.dpe_sq : aprx_min_dist<DIM>(slo, shi, mlo, mhi) < A.dpe) {
        if (lev + 1 == A.lmax) {
            if constexpr (SHP == 1) *zero = zero_children_box<DIM>(A, S, qlo, qhi);
            else *zero = zero_children<DIM>(A, S, qlo, qhi);
        }
        return 2;
    }
    return 0;
}

// row of the off-diagonal product lambda_a lambda_c (a < c) among the P rows
template <int NV> __host__ __device__ constexpr int offrow(int a, int c)
{
    return NV + a * NV - (a * (a + 1)) / 2 + (c - a - 1);
}

// -------------------------------------------------------------- integrators

// Leaf entries: (level << 24) | global sub-element index.
__device__ __forceinline__ uint32_t leaf_entry(int lev, int sub)
{
    return (static_cast<uint32_t>(lev) << 24) | static_cast<uint32_t>(sub);
}

// FP64 plain: lane = (k, b): b = inner point (lane % NYP), k = batch slice
template <int DIM, int ETA, int ORD = 1> struct PlainAcc {
    struct S : Shape<DIM> {
        static constexpr int NR = OShape<DIM, ORD>::NR;   // contraction rows of the order
    };
    static constexpr int NYP = DIM == 2 ? 8 : 16;
    static constexpr int K = kWave / NYP;
    // points per batch: 32 for P2 tetrahedra (35 rows a point), so that two
    // workgroups' staging fits the LDS of a CU beside the row caches
    static constexpr int kPoints = DIM == 3 && ORD == 2 ? 32 : kBatch;
    static constexpr int kStageBytes = kPoints * (DIM + S::NR) * 8;
    struct In {
        double lam[S::NV];
        double w;
    };
    double acc[S::NR];
    double yh[DIM];   // inner point relative to the anchor
    bool active;
    __device__ void set_rule(const double *) {}   // the points come from the barycentric tables
    __device__ void init(const double *y, int lane, char *)
    {
#pragma unroll
        for (int r = 0; r < S::NR; ++r) acc[r] = 0.0;
#pragma unroll
        for (int k = 0; k < DIM; ++k) yh[k] = y[k];
        active = (lane % NYP) < S::NQ;
    }
    __device__ static In fetch(CArgs &A, bool valid, int sub, int a, int lev, float, double wa)
    {
        In in;
        if (valid) {
            const double *lam = A.lam64 + (sub * S::NQ + a) * S::NV;
#pragma unroll
            for (int i = 0; i < S::NV; ++i) in.lam[i] = lam[i];
            in.w = ldexp(wa, -DIM * (lev - 1));
        } else {
#pragma unroll
            for (int i = 0; i < S::NV; ++i) in.lam[i] = 0.0;
            in.w = 0.0;
        }
        return in;
    }
    template <class Edge> __device__ static void stage(char *work, int t, const In &in, const Edge &E)
    {
        double *sx = reinterpret_cast<double *>(work);
        double *sp = sx + kPoints * DIM;
#pragma unroll
        for (int k = 0; k < DIM; ++k) {
            double s = 0.0;
#pragma unroll
            for (int i = 1; i <= DIM; ++i) s = fma(in.lam[i], E.e[i - 1][k], s);
            sx[t * DIM + k] = s;
        }
        if constexpr (ORD == 1) {
#pragma unroll
            for (int i = 0; i < S::NV; ++i) sp[t * S::NR + i] = in.w * in.lam[i];
#pragma unroll
            for (int i = 0; i < S::NV; ++i)
#pragma unroll
                for (int j = i + 1; j < S::NV; ++j)
                    sp[t * S::NR + offrow<S::NV>(i, j)] = in.w * in.lam[i] * in.lam[j];
        } else {
            // P2: w times the quartic monomials of lambda, in Mono4's order
            constexpr Mono4<S::NV> mono{};
            double pw[S::NV][5];
#pragma unroll
            for (int v = 0; v < S::NV; ++v) {
                pw[v][0] = 1.0;
#pragma unroll
                for (int q = 1; q <= 4; ++q) pw[v][q] = pw[v][q - 1] * in.lam[v];
            }
#pragma unroll
            for (int k = 0; k < S::NR; ++k) {
                double x = in.w;
#pragma unroll
                for (int v = 0; v < S::NV; ++v) x *= pw[v][mono.e[k][v]];
                sp[t * S::NR + k] = x;
            }
        }
    }
    __device__ void run(CArgs &A, const char *work, int npts)
    {
        const Band64 KB = band64(A);
        const double *sx = reinterpret_cast<const double *>(work);
        const double *sp = sx + kPoints * DIM;
        const int k0 = lane_id() / NYP;
        if (!active) return;
        for (int p = k0; p < npts; p += K) {
            double d2 = 0.0;
#pragma unroll
            for (int k = 0; k < DIM; ++k) {
                const double dx = sx[p * DIM + k] - yh[k];
                d2 = fma(dx, dx, d2);
            }
            const double g = kernel64_reg<ETA>(KB, d2);
#pragma unroll
            for (int r = 0; r < S::NR; ++r) acc[r] = fma(sp[p * S::NR + r], g, acc[r]);
        }
    }
    // totals H/Q for inner point b -> out[r*16 + b]
    __device__ void finish(double *out, double *)
    {
#pragma unroll
        for (int r = 0; r < S::NR; ++r) {
            double v = acc[r];
            for (int o = NYP; o < kWave; o <<= 1) v += __shfl_xor(v, o, kWave);
            acc[r] = v;
        }
        const int b = lane_id() % NYP;
        if (lane_id() < NYP && b < S::NQ) {
#pragma unroll
            for (int r = 0; r < S::NR; ++r) out[r * 16 + b] = acc[r];
        }
    }
};

// Sizes of a box element of order ORD: NB nodes, NU upper-triangle slots, NOUT
// per-pair outputs, NR product-monomial rows, NQ rule points, QS the stride of
// the per-inner-point rows (a power of two >= NQ).
template <int DIM, int ORD> struct BoxShape {
    static constexpr int NB = box_node_count(DIM, ORD);
    static constexpr int NU = NB * (NB + 1) / 2;
    static constexpr int NOUT = NB * NB + 2 * NU;
    static constexpr int NR = BoxMono<DIM, ORD>::N;
    static constexpr int NQ = box_nq(DIM);
    static constexpr int QS = DIM == 2 ? 16 : 32;
};

// The frame of the outer box l for its points: the corner differences
// D_c = P_c - P_0 (c >= 1), so that x(xi) - P_0 = sum_{c >= 1} N_c(xi) D_c and
// dx/dxi_i = sum_{c >= 1} dN_c/dxi_i D_c, and 1/|E_l|.
template <int DIM> struct BoxFrame {
    double d[(1 << DIM) - 1][DIM];
    double inv_meas;
};

// FP64 accumulator of box elements.  Lane = (b, k): b = inner point (lane %
// QS), k = group.  A leaf point a of sub-box `sub` at level lev is the root
// reference point xi = (X + g_a) 2^{1-lev}, X the sub-box's integer origin
// (the base-2^DIM digits of its local index, one bit per axis and level), g_a
// the rule point; staging maps it through the root's multilinear map and
// weighs it with w_a 2^{-DIM(lev-1)} |det F_l'(xi)| / |E_l|, then forms the
// NR product monomials xi^e.  The groups split the points (K slices), or, for
// the 90 rows of the 20-node hexahedron, the rows (each group all points, half
// of the rows, so that the accumulators fit the registers; its batches hold 32
// points to fit the staging in LDS).
template <int DIM, int ETA, int ORD> struct BoxAcc {
    using BS = BoxShape<DIM, ORD>;
    static constexpr int NR = BS::NR, NQ = BS::NQ, NYP = BS::QS;
    static constexpr int K = kWave / NYP;
    static constexpr bool ROWS = NR > 48;
    static constexpr int NRL = ROWS ? (NR + K - 1) / K : NR;
    static constexpr int kPoints = ROWS ? 32 : 64;
    static constexpr int kStageBytes = kPoints * (DIM + NR) * 8;
    static constexpr int NCH = 1 << DIM;
    struct In {
        double xi[DIM];
        double w;
    };
    double acc[NRL];
    double yh[DIM];
    bool active;
    int grp;
    const double *g;   // rule points [NQ][DIM] (LDS)
    __device__ void init(const double *y, int lane, char *)
    {
#pragma unroll
        for (int r = 0; r < NRL; ++r) acc[r] = 0.0;
#pragma unroll
        for (int k = 0; k < DIM; ++k) yh[k] = y[k];
        active = (lane % NYP) < NQ;
        grp = lane / NYP;
    }
    __device__ void set_rule(const double *rule) { g = rule; }
    __device__ In fetch(CArgs &A, bool valid, int sub, int a, int lev, float, double wa) const
    {
        In in;
        if (valid) {
            const int local = sub - level_offset<DIM>(lev);
            int X[DIM];
#pragma unroll
            for (int k = 0; k < DIM; ++k) X[k] = 0;
            for (int d = 0; d < lev - 1; ++d) {
                const int c = (local >> (DIM * d)) & (NCH - 1);
#pragma unroll
                for (int k = 0; k < DIM; ++k) X[k] |= ((c >> k) & 1) << d;
            }
#pragma unroll
            for (int k = 0; k < DIM; ++k)
                in.xi[k] = ldexp(__dadd_rn(static_cast<double>(X[k]), g[a * DIM + k]), 1 - lev);
            in.w = ldexp(wa, -DIM * (lev - 1));
        } else {
#pragma unroll
            for (int k = 0; k < DIM; ++k) in.xi[k] = 0.0;
            in.w = 0.0;
        }
        return in;
    }
    __device__ static void stage(char *work, int t, const In &in, const BoxFrame<DIM> &F)
    {
        double *sx = reinterpret_cast<double *>(work);
        double *sp = sx + kPoints * DIM;
        double x[DIM], J[DIM][DIM];
#pragma unroll
        for (int k = 0; k < DIM; ++k) {
            x[k] = 0.0;
#pragma unroll
            for (int i = 0; i < DIM; ++i) J[k][i] = 0.0;
        }
#pragma unroll
        for (int c = 1; c < NCH; ++c) {
            double N = 1.0, dN[DIM];
#pragma unroll
            for (int i = 0; i < DIM; ++i) dN[i] = 1.0;
#pragma unroll
            for (int j = 0; j < DIM; ++j) {
                const bool cj = ((c >> j) & 1) != 0;
                const double f = cj ? in.xi[j] : 1.0 - in.xi[j];
                N *= f;
#pragma unroll
                for (int i = 0; i < DIM; ++i) dN[i] *= i == j ? (cj ? 1.0 : -1.0) : f;
            }
#pragma unroll
            for (int k = 0; k < DIM; ++k) {
                x[k] = fma(N, F.d[c - 1][k], x[k]);
#pragma unroll
                for (int i = 0; i < DIM; ++i) J[k][i] = fma(dN[i], F.d[c - 1][k], J[k][i]);
            }
        }
        double det;
        if constexpr (DIM == 2) {
            det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
        } else {
            det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) - J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                  J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
        }
        const double w = in.w * fabs(det) * F.inv_meas;
#pragma unroll
        for (int k = 0; k < DIM; ++k) sx[t * DIM + k] = x[k];
        double pw[DIM][5];
#pragma unroll
        for (int k = 0; k < DIM; ++k) {
            pw[k][0] = 1.0;
#pragma unroll
            for (int q = 1; q <= 4; ++q) pw[k][q] = pw[k][q - 1] * in.xi[k];
        }
        constexpr BoxMono<DIM, ORD> mono{};
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            double v = w;
#pragma unroll
            for (int k = 0; k < DIM; ++k) v *= pw[k][mono.e[r][k]];
            sp[t * NR + r] = v;
        }
    }
    __device__ void run(CArgs &A, const char *work, int npts)
    {
        const Band64 KB = band64(A);
        const double *sx = reinterpret_cast<const double *>(work);
        const double *sp = sx + kPoints * DIM;
        if (!active) return;
        const int p0 = ROWS ? 0 : grp, dp = ROWS ? 1 : K;
        for (int p = p0; p < npts; p += dp) {
            double d2 = 0.0;
#pragma unroll
            for (int k = 0; k < DIM; ++k) {
                const double dx = sx[p * DIM + k] - yh[k];
                d2 = fma(dx, dx, d2);
            }
            const double gv = kernel64_reg<ETA>(KB, d2);
            if constexpr (ROWS) {
#pragma unroll
                for (int r = 0; r < NRL; ++r) {
                    const int rr = grp * NRL + r;
                    if (rr < NR) acc[r] = fma(sp[p * NR + rr], gv, acc[r]);
                }
            } else {
#pragma unroll
                for (int r = 0; r < NR; ++r) acc[r] = fma(sp[p * NR + r], gv, acc[r]);
            }
        }
    }
    // totals for inner point b, times jm = |det F_m'(g_b)| / |E_m| -> out[r*QS + b]
    __device__ void finish(double *out, double jm)
    {
        const int b = lane_id() % NYP;
        if constexpr (ROWS) {
            if (b < NQ) {
#pragma unroll
                for (int r = 0; r < NRL; ++r) {
                    const int rr = grp * NRL + r;
                    if (rr < NR) out[rr * NYP + b] = acc[r] * jm;
                }
            }
        } else {
#pragma unroll
            for (int r = 0; r < NR; ++r) {
                double v = acc[r];
                for (int o = NYP; o < kWave; o <<= 1) v += __shfl_xor(v, o, kWave);
                acc[r] = v;
            }
            if (lane_id() < NYP && b < NQ) {
#pragma unroll
                for (int r = 0; r < NR; ++r) out[r * NYP + b] = acc[r] * jm;
            }
        }
    }
};

typedef double doublex4 __attribute__((ext_vector_type(4)));

// FP64 accumulator with the contraction on the matrix cores
// (v_mfma_f64_16x16x4f64): the staging of Base (PlainAcc or BoxAcc: FP64
// coordinates and NR rows per point), then per step of 4 staged points every
// lane evaluates gamma for one (point k, inner point j) pair, lane j + 16k --
// the B operand G[k][j] -- and the A operand P[i][k] (row 16t + i of point k,
// lane i + 16k) is read from the staged rows; D[i][j] += sum_k P[i][k] G[k][j]
// for every 16-row tile t and 16-column tile c of the inner points.  Distances
// and gamma stay on the vector ALU in FP64; the NR multiply-adds per
// evaluation move to the matrix cores.  The FP64 instruction's D[i][j] is held
// in lane j + 16 (i % 4), register i / 4 (unlike the FP32 16x16x4 one: lane
// j + 16 (i / 4), register i % 4).
template <class Base, int DIM, int ETA, int NR, int NQ, int NYPV, int BATCH> struct Mfma64 {
    static constexpr int NRT = (NR + 15) / 16, NCT = (NQ + 15) / 16;
    static constexpr int NYP = NYPV;   // lane period of the inner points given to init
    static constexpr int kStageBytes = Base::kStageBytes;
    using In = typename Base::In;
    Base base;
    doublex4 acc[NRT][NCT];
    double yc[NCT][DIM];   // inner points of this lane's columns j and 16 + j
    bool colv[NCT];
    __device__ void init(const double *y, int lane, char *work)
    {
#pragma unroll
        for (int t = 0; t < NRT; ++t)
#pragma unroll
            for (int c = 0; c < NCT; ++c) acc[t][c] = doublex4{0.0, 0.0, 0.0, 0.0};
        const int x = lane & 15;
#pragma unroll
        for (int c = 0; c < NCT; ++c) {
            // the lane holding inner point 16c + x (period NYP >= 16 * NCT)
#pragma unroll
            for (int d = 0; d < DIM; ++d) yc[c][d] = __shfl(y[d], 16 * c + x, kWave);
            colv[c] = 16 * c + x < NQ;
        }
    }
    __device__ void set_rule(const double *g) { base.set_rule(g); }
    __device__ In fetch(CArgs &A, bool valid, int sub, int a, int lev, float w32, double wa) const
    {
        return base.fetch(A, valid, sub, a, lev, w32, wa);
    }
    template <class Frame> __device__ static void stage(char *work, int t, const In &in, const Frame &F)
    {
        Base::stage(work, t, in, F);
    }
    // Step p0 takes the outer points p0 + k (k = lane / 16).  Its operands are read
    // without conditions (a lane past npts, or a row past NR, reads point 0 / row 0
    // of the batch, which is always staged, and its value is masked to 0), and
    // the next step's are loaded before this step's kernel values and MFMAs, so
    // the LDS latency overlaps them.
    __device__ void load(const double *sx, const double *sp, int p0, int npts, double *xp, double *a) const
    {
        const int lane = lane_id(), x = lane & 15, k = lane >> 4;
        const int p = p0 + k < npts ? p0 + k : 0;
#pragma unroll
        for (int d = 0; d < DIM; ++d) xp[d] = sx[p * DIM + d];
#pragma unroll
        for (int t = 0; t < NRT; ++t) {
            const int r = 16 * t + x;
            a[t] = sp[p * NR + (r < NR ? r : 0)];
        }
    }
    __device__ void run(CArgs &A, const char *work, int npts)
    {
        const Band64 KB = band64(A);
        const double *sx = reinterpret_cast<const double *>(work);
        const double *sp = sx + BATCH * DIM;
        const int lane = lane_id(), x = lane & 15, k = lane >> 4;
        double xp[DIM], a[NRT];
        load(sx, sp, 0, npts, xp, a);
        for (int p0 = 0; p0 < npts; p0 += 4) {
            const bool pv = p0 + k < npts;
            double xn[DIM], an[NRT];
#pragma unroll
            for (int d = 0; d < DIM; ++d) xn[d] = xp[d];
#pragma unroll
            for (int t = 0; t < NRT; ++t) an[t] = a[t];
            if (p0 + 4 < npts) load(sx, sp, p0 + 4, npts, xn, an);
            double b[NCT];
#pragma unroll
            for (int c = 0; c < NCT; ++c) {
                double d2 = 0.0;
#pragma unroll
                for (int d = 0; d < DIM; ++d) {
                    const double dx = xp[d] - yc[c][d];
                    d2 = fma(dx, dx, d2);
                }
                const double gv = kernel64_reg<ETA>(KB, d2);
                b[c] = pv && colv[c] ? gv : 0.0;
            }
#pragma unroll
            for (int t = 0; t < NRT; ++t) {
                const double at = pv && 16 * t + x < NR ? a[t] : 0.0;
#pragma unroll
                for (int c = 0; c < NCT; ++c) acc[t][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(at, b[c], acc[t][c], 0, 0, 0);
            }
#pragma unroll
            for (int d = 0; d < DIM; ++d) xp[d] = xn[d];
#pragma unroll
            for (int t = 0; t < NRT; ++t) a[t] = an[t];
        }
    }
    // rows -> out[r * QS + b] (QS = the epilogue's row stride), times the inner
    // point's factor jm (held by lane b: period NYP)
    template <int QS> __device__ void finish_rows(double *out, double jm)
    {
        const int lane = lane_id(), x = lane & 15, q = lane >> 4;
#pragma unroll
        for (int c = 0; c < NCT; ++c) {
            const double f = __shfl(jm, 16 * c + x, kWave);
#pragma unroll
            for (int t = 0; t < NRT; ++t)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int row = 16 * t + 4 * r + q, col = 16 * c + x;
                    if (row < NR && col < NQ) out[row * QS + col] = acc[t][c][r] * f;
                }
        }
    }
    // simplices: the epilogue's stride 16 (the tile argument is unused)
    __device__ void finish(double *out, double *) { finish_rows<16>(out, 1.0); }
    // boxes: stride 16 (2D) / 32 (3D), times |det F_m'| / |E_m|
    __device__ void finish(double *out, double jm) { finish_rows<(DIM == 2 ? 16 : 32)>(out, jm); }
};

typedef float floatx4 __attribute__((ext_vector_type(4)));

// The FP32 matrix-core sums of a pair are added to its FP64 totals every this
// many batches of 64 outer points (and at the pair's end): each FP32 sum holds
// at most 64 (2D) or 128 (3D) positive products per entry.
constexpr int kFlushBatches = 2;

// FP32 mixed path with distances on the vector ALU (2D, where it is faster
// than the variant below): v_mfma_f32_16x16x4f32, A = P (rows x 4 points),
// B = G (4 points x 16 inner points).  Operand layout: A[i][k] and B[k][j] live
// in lane i + 16k (resp. j + 16k); D[i][j] in lane j + 16*(i/4), register i%4.
// 8 points per step as two independent 8x8 diagonal blocks: lanes with column
// < 8 use point set 0, columns >= 8 set 1.
// Staging layout: 2 floats of coordinates and 8 floats of rows per point (the
// 6 P rows, then lambda_1, lambda_2, read only by A rows >= 6, which feed rows
// of D that are never used); the padding inner column gets a coordinate far
// outside the horizon, so gamma is 0 there.
template <int DIM, int ETA> struct MixedAccDirect {
    static_assert(DIM == 2, "the vector-ALU distance variant is the 2D accumulator");
    using S = Shape<DIM>;
    static constexpr int PPS = 8;                  // points per MFMA step
    static constexpr int STEPS = kBatch / PPS;
    static constexpr int XS = 2;
    static constexpr int PS = 8;
    static constexpr int kStageBytes = kBatch * (XS + PS) * 4;
    // one point: its row of the precomputed table (P rows, lambda_1, lambda_2)
    struct In {
        floatx4 r0, r1;
    };
    double dacc[4];
    floatx4 facc;   // FP32 sums of the batches since the last flush
    int nb;         // batches since the last flush (wave-uniform)
    float yh[2];
    float doe;   // delta / eps (vector register)
    int sub;     // inner point (and P row) handled by this lane
    int poff;    // point offset within a step
    __device__ void init(const double *y, int lane, char *)
    {
        const int n = lane & 15;
        const int k = lane >> 4;
        sub = n & 7;
        poff = 4 * (n >> 3) + k;
#pragma unroll
        for (int r = 0; r < 4; ++r) dacc[r] = 0.0;
        facc = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
        nb = 0;
        const bool colv = sub < S::NQ;
        yh[0] = colv ? static_cast<float>(y[0]) : 1.0e18f;
        yh[1] = colv ? static_cast<float>(y[1]) : 1.0e18f;
    }
    __device__ void set_column(CArgs &A, const double *, bool) { doe = in_vgpr(A.f_delta_over_eps); }
    // the table row of point a of sub-element sub; lanes without a point read
    // the zero row at the end
    __device__ static In fetch(CArgs &A, bool valid, int sub, int a, int, float, double)
    {
        const int row = valid ? sub * S::NQ + a : A.pt32_zero;
        const floatx4 *t = reinterpret_cast<const floatx4 *>(A.pt32 + static_cast<int64_t>(row) * 8);
        return In{t[0], t[1]};
    }
    // point t of the batch: anchor-relative coordinates and the table row
    template <class Edge> __device__ static void stage(char *work, int t, const In &in, const Edge &E)
    {
        float *sx = reinterpret_cast<float *>(work);
        float *sp = sx + kBatch * XS;
        const float l1 = in.r1[2], l2 = in.r1[3];
        const float x0 = fmaf(l2, E.e[1][0], l1 * E.e[0][0]);
        const float x1 = fmaf(l2, E.e[1][1], l1 * E.e[0][1]);
        *reinterpret_cast<float2 *>(sx + t * XS) = make_float2(x0, x1);
        *reinterpret_cast<floatx4 *>(sp + t * PS) = in.r0;
        *reinterpret_cast<floatx4 *>(sp + t * PS + 4) = in.r1;
    }
    __device__ void run(CArgs &A, const char *work, int npts)
    {
        const float *sx = reinterpret_cast<const float *>(work) + poff * XS;
        const float *sp = reinterpret_cast<const float *>(work) + kBatch * XS + poff * PS + sub;
        floatx4 acc = facc;
        const int steps = (npts + PPS - 1) / PPS;
        // each step's operands are read one step ahead, so that their LDS latency
        // passes under the previous step's vector work
        float a_next = sp[0];
        float2 x_next = *reinterpret_cast<const float2 *>(sx);
#pragma unroll
        for (int t = 0; t < STEPS; ++t) {
            if (t >= steps) break;
            const float a = a_next;
            const float2 x = x_next;
            if (t + 1 < STEPS) {
                a_next = sp[(t + 1) * PPS * PS];
                x_next = *reinterpret_cast<const float2 *>(sx + (t + 1) * PPS * XS);
            }
            const float dx = x.x - yh[0], dy = x.y - yh[1];
            const float d2 = fmaf(dx, dx, dy * dy);
            const float g = kernel32_reg<ETA>(A, d2, doe);
            acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a, g, acc, 0, 0, 0);
        }
        facc = acc;
        if (++nb == kFlushBatches) flush();
    }
    // FP32 partial sums into the FP64 totals (every kFlushBatches batches and
    // at the end of the pair)
    __device__ void flush()
    {
#pragma unroll
        for (int r = 0; r < 4; ++r) dacc[r] += static_cast<double>(facc[r]);
        facc = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
        nb = 0;
    }
    // D[i][j] (FP64) -> H/Q totals out[r*16 + b]; out may be the tile itself: each
    // lane reads its own slot and a slot of rows 8..15, which nobody writes
    __device__ void finish(double *out, double *tile)
    {
        flush();
        const int l = lane_id();
        const int j = l & 15, ib = 4 * (l >> 4);
#pragma unroll
        for (int r = 0; r < 4; ++r) tile[(ib + r) * 16 + j] = dacc[r];
        wave_sync();
        // padding columns hold gamma = 0, so their totals are 0 as well
        for (int t = l; t < S::NR * 8; t += kWave) {
            const int r = t / 8, b = t % 8;
            out[r * 16 + b] = tile[r * 16 + b] + tile[(r + 8) * 16 + (b + 8)];
        }
    }
};

// FP32 mixed path, both products on the matrix cores (3D; v_mfma_f32_16x16x4f32;
// operand layout: A[i][k] in lane i + 16k, B[k][j] in lane j + 16k, C and D
// [i][j] in lane j + 16(i/4), register i%4):
//  * distances: D = |x_i|^2 - 2 x_i . y_j + |y_j|^2 for 16 outer points i x 16
//    columns j, K = (x, y, z, |x|^2) . (-2y, 1) and C = |y_j|^2; 15 inner
//    points + 1 padding column;
//  * gamma_eps of the four distances a lane holds (its rows 4g..4g+3);
//  * contraction H = P^T G: register r of the distance tile is exactly the B
//    operand of step r (K index k <-> row 4k + r), A = the P rows of those
//    points.
// Rows >= NR of D (A rows beyond the P rows read neighbouring staged values)
// are never used; the padding column gets |y|^2 huge, so gamma is 0 there.
template <int DIM, int ETA> struct MixedAccMfma {
    static_assert(DIM == 3, "the matrix-core distance variant is the 3D accumulator");
    using S = Shape<DIM>;
    static constexpr int XS = 4;                            // x, y, z, |x|^2 per point
    static constexpr int PS = S::NR;
    static constexpr int kXBytes = kBatch * XS * 4;
    // the P rows come first, so that the contraction operands of a batch's first two
    // tiles are read at the instruction's own offsets, without an address add
    static constexpr int kPBytes = kBatch * PS * 4;
    static constexpr int kStageBytes = kXBytes + kPBytes;
    // one point: its row of the precomputed table (P0..P9, lambda_1..lambda_3; the
    // row's last three floats are padding and not loaded: registers loaded but
    // never read are reused while the load is in flight, which makes the wave
    // wait for it)
    struct In {
        floatx4 r0, r1, r2;
        float l3;
    };
    double dacc[4];
    floatx4 facc;    // FP32 sums of the batches since the last flush
    int nb;          // batches since the last flush (wave-uniform)
    float bop;       // B operand of the distance MFMA
    float yb2;       // |y_j|^2 of this lane's column (huge for a padding column: gamma 0)
    float doe;       // delta / eps (vector register)
    int arow, acol;  // A operand: row i and K index k of this lane
    int col;         // column j (C / D layout)
    __device__ void init(const double *y, int lane, char *)
    {
        arow = lane & 15;
        acol = lane >> 4;
        col = lane & 15;
#pragma unroll
        for (int r = 0; r < 4; ++r) dacc[r] = 0.0;
        facc = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
        nb = 0;
        (void)y;
    }
    // inner point of this lane's column (anchor-relative, FP64), set once per pair
    __device__ void set_column(CArgs &A, const double *yb, bool valid)
    {
        doe = in_vgpr(A.f_delta_over_eps);
        double q = 0.0;
#pragma unroll
        for (int k = 0; k < DIM; ++k) q += yb[k] * yb[k];
        yb2 = valid ? static_cast<float>(q) : 1.0e30f;
        bop = acol < 3 ? (valid ? static_cast<float>(-2.0 * yb[acol]) : 0.0f) : 1.0f;
    }
    // the table row of point a of sub-element sub; lanes without a point read
    // the zero row at the end
    __device__ static In fetch(CArgs &A, bool valid, int sub, int a, int, float, double)
    {
        const int row = valid ? sub * S::NQ + a : A.pt32_zero;
        const floatx4 *t = reinterpret_cast<const floatx4 *>(A.pt32 + static_cast<int64_t>(row) * 16);
        return In{t[0], t[1], t[2], reinterpret_cast<const float *>(t)[12]};
    }
    // point t of the batch: anchor-relative coordinates, |x|^2 and the P rows
    template <class Edge> __device__ static void stage(char *work, int t, const In &in, const Edge &E)
    {
        float *sx = reinterpret_cast<float *>(work + kPBytes);
        float *sp = reinterpret_cast<float *>(work);
        const float l1 = in.r2[2], l2 = in.r2[3], l3 = in.l3;
        float x[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) x[k] = fmaf(l3, E.e[2][k], fmaf(l2, E.e[1][k], l1 * E.e[0][k]));
        const float n2 = fmaf(x[2], x[2], fmaf(x[1], x[1], x[0] * x[0]));
        *reinterpret_cast<float4 *>(sx + t * XS) = make_float4(x[0], x[1], x[2], n2);
        // 10 rows: t * 10 floats is a multiple of 8 bytes
        float2 *dst = reinterpret_cast<float2 *>(sp + t * PS);
        dst[0] = make_float2(in.r0[0], in.r0[1]);
        dst[1] = make_float2(in.r0[2], in.r0[3]);
        dst[2] = make_float2(in.r1[0], in.r1[1]);
        dst[3] = make_float2(in.r1[2], in.r1[3]);
        dst[4] = make_float2(in.r2[0], in.r2[1]);
    }
    // gamma_eps / C of tile value v = |x|^2 - 2 x.y + |y|^2 = |x - y|^2.  The
    // band test and the plateau take v as it is (a slightly negative v from the
    // cancellation of nearly equal points lies on the plateau); the band path
    // takes |v| (a source modifier of the square root), which for such a v is a
    // distance far inside the plateau as well.
    __device__ __forceinline__ float gamma(CArgs &A, float v) const
    {
        const bool plateau = v < A.f_dme2;
        const bool band = !plateau && v <= A.f_dpe2;
        const float d2 = fabsf(v);
        if (__builtin_amdgcn_ballot_w64(band)) return kernel32<ETA>(A, d2, doe);
        float g = plateau ? 1.0f : 0.0f;
        if (ETA == NLQ_ETA_GAUSS) g = plateau ? __expf(-d2 * A.f_inv_delta2) : 0.0f;
        return g;
    }
    __device__ void run(CArgs &A, const char *work, int npts)
    {
        const float *sx = reinterpret_cast<const float *>(work + kPBytes);
        const float *sp = reinterpret_cast<const float *>(work);
        floatx4 acc = facc;
        const int tiles = (npts + 15) / 16;
        // the distance operand of the next tile is read one tile ahead
        float a_next = sx[arow * XS + acol];
#pragma unroll
        for (int ss = 0; ss < kBatch / 16; ++ss) {
            if (ss >= tiles) break;
            const int p0 = ss * 16;
            const float a_d = a_next;
            if (ss + 1 < kBatch / 16) a_next = sx[(p0 + 16 + arow) * XS + acol];
            // C = |y_j|^2 in every row: the tile is |x_i - y_j|^2 directly
            const floatx4 v = __builtin_amdgcn_mfma_f32_16x16x4f32(a_d, bop, floatx4{yb2, yb2, yb2, yb2}, 0, 0, 0);
            // the contraction's A operands, read before the mollifier so that the LDS
            // latency passes under its vector work
            float a4[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) a4[r] = sp[(p0 + 4 * acol + r) * PS + arow];
            // a register whose 64 distances all lie beyond delta + eps has gamma = 0
            // everywhere: its contraction step would add exact zeros and is skipped.
            // The mask is the wave's ordered v <= (delta + eps)^2 comparison (LLVM
            // predicate 5, FCMP_OLE), the same comparison as the band test's, which
            // the compiler then shares (a ballot of the boolean was re-materialised
            // through two vector instructions for one of the four registers).
            float g[4];
            unsigned long long inside[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                inside[r] = __builtin_amdgcn_fcmpf(v[r], A.f_dpe2, 5);
                g[r] = gamma(A, v[r]);
            }
#pragma unroll
            for (int r = 0; r < 4; ++r)
                if (inside[r]) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a4[r], g[r], acc, 0, 0, 0);
        }
        facc = acc;
        if (++nb == kFlushBatches) flush();
    }
    __device__ void flush()
    {
#pragma unroll
        for (int r = 0; r < 4; ++r) dacc[r] += static_cast<double>(facc[r]);
        facc = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
        nb = 0;
    }
    // D[i][j] (FP64) -> H/Q totals out[r*16 + b]; out may be the tile itself
    // (each lane reads back its own slots)
    __device__ void finish(double *out, double *tile)
    {
        flush();
        const int l = lane_id();
        const int j = l & 15, ib = 4 * (l >> 4);
#pragma unroll
        for (int r = 0; r < 4; ++r) tile[(ib + r) * 16 + j] = dacc[r];
        wave_sync();
        // the padding column holds gamma = 0, so its totals are 0 as well
        for (int t = l; t < S::NR * 16; t += kWave) out[t] = tile[t];
    }
};

// the FP32 accumulator of each dimension (measured: distances on the vector ALU
// are faster in 2D, on the matrix cores in 3D)
template <int DIM, int ETA>
using MixedAcc = typename std::conditional<DIM == 2, MixedAccDirect<DIM, ETA>, MixedAccMfma<DIM, ETA>>::type;

// per-wave LDS: staging, then the epilogue's H/Q rows and MFMA tile | leaves | stack
template <int DIM, int PREC, int ORD = 1, int SHP = 0> struct WaveMem {
    using S = Shape<DIM>;
    using O = OShape<DIM, ORD>;
    using BS = BoxShape<DIM, ORD>;
    static constexpr int kStageBytes =
        SHP == 1 ? BoxAcc<DIM, 0, ORD>::kStageBytes
                 : (PREC == 0 ? PlainAcc<DIM, 0, ORD>::kStageBytes : MixedAcc<DIM, 0>::kStageBytes);
    // P1: H/Q rows + column sums + diagonal rows; P2: the monomial rows, then the
    // rows mapped from them; boxes: the monomial rows, the basis-function rows and
    // the weighted row sums
    static constexpr int kEpiRows = ORD == 1 ? S::NR + 1 + S::NV : O::NR + O::NRX;
    static constexpr int kBoxEpiBytes = (BS::NR + BS::NB + (BS::NR + BS::QS - 1) / BS::QS) * BS::QS * 8;
    // the mixed path's 16 x 16 MFMA tile is written in place of the H/Q rows
    static constexpr int kEpiBytes = SHP == 1 ? kBoxEpiBytes : (PREC == 1 && kEpiRows < 16 ? 16 : kEpiRows) * 16 * 8;
    // the epilogue runs after the pair's last batch: it shares the staging area
    static constexpr int kWorkBytes = kStageBytes > kEpiBytes ? kStageBytes : kEpiBytes;
    // vertices of the sub-elements of levels 2..kMemoLevel (FP64), formed once per
    // pair (2D only: in 3D it measured 1% faster at L_max 4 but 3% slower at
    // L_max 3, where it is not even used)
    static constexpr int kMemoLevel = DIM == 2 ? 3 : 1;
    static constexpr int kMemoCount = DIM == 2 ? 4 + 16 : 0;
    static constexpr int kMemoBytes = kMemoCount * Geo<DIM, SHP>::NV * DIM * 8;
    __host__ __device__ static int bytes(int capl, int leafcap)
    {
        return (kWorkBytes + leafcap * 4 + kMemoBytes + capl * 4 + 15) & ~15;
    }
};

// binary search of column c in the sorted list cols[0..n)
__device__ __forceinline__ int64_t search(const int32_t *cols, int64_t n, int32_t c)
{
    int64_t a = 0, b = n - 1;
    while (a <= b) {
        const int64_t mid = (a + b) >> 1;
        const int32_t v = cols[mid];
        if (v == c) return mid;
        if (v < c) a = mid + 1; else b = mid - 1;
    }
    return -1;
}

// CSR rows of the outer element's nodes, cached in LDS by the workgroup as 16-bit
// offsets from the row's first column when the row fits (length <= rowcap and
// column span < 65536); otherwise searched in the global row
struct RowCache {
    const uint16_t *c16[20];   // LDS copy, or nullptr (one row per node of l: up to 20, the serendipity hexahedron)
    const int32_t *cols[20];   // the global row
    int32_t first[20];
    int64_t base[20];
    int64_t len[20];
    // a row that does not fit keeps every step-th column (int32) in its LDS area
    // instead: the search narrows to one block of `step` columns there, then
    // searches that block in the global row (0 samples: the whole global row)
    const int32_t *samp[20];
    int step[20];
    int nsamp[20];
};

// int32 samples that fit in a row's LDS area of rowcap 16-bit entries, after
// aligning its start to 4 bytes
__host__ __device__ constexpr int row_sample_cap(int rowcap) { return (rowcap - 1) / 2; }

// position of column c in cached row r, or -1 (a cached row holds at most
// rowcap < 2^16 entries, so the lower-bound search runs in 32-bit arithmetic)
__device__ __forceinline__ int64_t row_find(const RowCache *rc, int r, int32_t c)
{
    const uint16_t *q = rc->c16[r];
    if (!q) {
        const int ns = rc->nsamp[r];
        if (ns == 0) return search(rc->cols[r], rc->len[r], c);
        const int32_t *sm = rc->samp[r];
        if (c < sm[0]) return -1;
        // k = the last sample <= c (sm[0] is the row's first column)
        int lo = 0, n = ns;
        while (n > 0) {
            const int half = n >> 1;
            if (sm[lo + half] <= c) {
                lo += half + 1;
                n -= half + 1;
            } else {
                n = half;
            }
        }
        const int64_t b0 = static_cast<int64_t>(lo - 1) * rc->step[r];
        const int64_t blen = rc->len[r] - b0 < rc->step[r] ? rc->len[r] - b0 : rc->step[r];
        const int64_t at = search(rc->cols[r] + b0, blen, c);
        return at < 0 ? -1 : b0 + at;
    }
    const int32_t d = c - rc->first[r];
    if (d < 0 || d > 65535) return -1;
    const int len = static_cast<int>(rc->len[r]);
    int lo = 0, n = len;
    while (n > 0) {
        const int half = n >> 1;
        if (static_cast<int32_t>(q[lo + half]) < d) {
            lo += half + 1;
            n -= half + 1;
        } else {
            n = half;
        }
    }
    return lo < len && static_cast<int32_t>(q[lo]) == d ? lo : -1;
}

template <int DIM, class Real> struct Edges {
    Real e[DIM][DIM];
};

// -------------------------------------------------------------- epilogue tables

// Output kinds of the per-pair epilogue: B_lm entries, upper-triangle entries of
// B_mm and of B_ll.
constexpr int kOutNone = 0, kOutLM = 1, kOutMM = 2, kOutLL = 3;

// (i, j), i <= j, of upper-triangle slot u of an N x N block: u < N is the
// diagonal (u, u), the others follow (i, j), i < j, in lexicographic order (the
// numbering of the product rows lambda_i lambda_j for P1 elements)
template <int N> __host__ __device__ constexpr void pair_of(int u, int &i, int &j)
{
    i = j = u;
    for (int a = 0; a < N; ++a)
        for (int c = a + 1; c < N; ++c)
            if (offrow<N>(a, c) == u) {
                i = a;
                j = c;
            }
}

// Epilogue descriptor of one output: kind | x-row << 2 | t-row << 9 | i << 16 | j << 20 | u << 24
__host__ __device__ constexpr int epi_desc(int kind, int xr, int tr, int i, int j, int u)
{
    return kind | (xr << 2) | (tr << 9) | (i << 16) | (j << 20) | (u << 24);
}

// Constant rows (FP64, stride 16) over the inner points b, with psi the NB basis
// functions of the inner element:
//   0..NB-1          w_b psi_j(y_b)                  (B_lm)
//   NB..NB+NU-1      w_b psi_i(y_b) psi_j(y_b), i<=j  (B_mm, slot u)
//   NB+NU            w_b                             (B_ll)
// and one descriptor per output o < NOUT (B_lm, then the B_mm and B_ll slots).
// x-rows index the rows after the contraction.  P1: 0..NR-1 the totals H_i and
// Q_ij, NR the column sums sum_i H_i, NR+1+i the rows H_i - sum_{q != i} Q_iq
// (lambda_i^2 through the partition of unity).  P2: 0..NR-1 the monomial totals,
// NR + k the k-th row of make_p2_map's image (phi_I phi_J, then
// phi_I (sum lambda)^2, then (sum lambda)^4).
template <int DIM, int ORD>
__device__ void epilogue_tables(const double *s_rule, double *s_T, int *s_desc)
{
    using O = OShape<DIM, ORD>;
    constexpr int NV = O::NV, NQ = Shape<DIM>::NQ, NR = O::NR, NB = O::NB, NU = O::NU;
    constexpr int NPASS = (O::NOUT + kWave - 1) / kWave;
    const double *bary = s_rule;
    const double *wq = s_rule + NQ * NV;
    // inner basis function I at point b
    auto psi = [&](int I, int b) {
        const double *lb = bary + b * NV;
        if (ORD == 1) return lb[I];
        if (I < NV) return lb[I] * (2.0 * lb[I] - 1.0);
        int a, c;
        pair_of<NV>(I, a, c);
        return 4.0 * lb[a] * lb[c];
    };
    for (int t = threadIdx.x; t < (NB + NU + 1) * 16; t += kThreads) {
        const int row = t >> 4, b = t & 15;
        double v = 0.0;
        if (b < NQ) {
            if (row < NB) {
                v = wq[b] * psi(row, b);
            } else if (row < NB + NU) {
                int i, j;
                pair_of<NB>(row - NB, i, j);
                v = wq[b] * psi(i, b) * psi(j, b);
            } else {
                v = wq[b];
            }
        }
        s_T[t] = v;
    }
    for (int o = threadIdx.x; o < NPASS * kWave; o += kThreads) {
        int kind = kOutNone, xr = 0, tr = 0, i = 0, j = 0, u = 0;
        if (o < NB * NB) {
            kind = kOutLM;
            i = o / NB;
            j = o % NB;
            xr = ORD == 1 ? i : NR + NU + i;
            tr = j;
        } else if (o < NB * NB + NU) {
            kind = kOutMM;
            u = o - NB * NB;
            pair_of<NB>(u, i, j);
            xr = ORD == 1 ? NR : NR + NU + NB;
            tr = NB + u;
        } else if (o < NB * NB + 2 * NU) {
            kind = kOutLL;
            u = o - NB * NB - NU;
            pair_of<NB>(u, i, j);
            xr = ORD == 1 ? (u < NV ? NR + 1 + u : u) : NR + u;
            tr = NB + NU;
        }
        s_desc[o] = epi_desc(kind, xr, tr, i, j, u);
    }
}

// P1: rows NR (sum_i H_i) and NR+1+i (H_i - sum_{q != i} Q_iq) of the per-pair totals
template <int DIM> __device__ __forceinline__ void extend_rows(double *HQ)
{
    using S = Shape<DIM>;
    constexpr int NV = S::NV, NR = S::NR;
    constexpr int BW = S::NQ <= 8 ? 8 : 16;
    for (int t = lane_id(); t < (1 + NV) * BW; t += kWave) {
        const int q = t / BW, b = t % BW;
        double v;
        if (q == 0) {
            v = HQ[b];
#pragma unroll
            for (int r = 1; r < NV; ++r) v += HQ[r * 16 + b];
        } else {
            const int i = q - 1;
            v = HQ[i * 16 + b];
#pragma unroll
            for (int c = 0; c < NV; ++c)
                if (c != i) v -= HQ[offrow<NV>(i < c ? i : c, i < c ? c : i) * 16 + b];
        }
        HQ[(NR + q) * 16 + b] = v;
    }
}

// P2: rows NR + k = sum_r map[k][r] * (monomial total r), k < NRX
template <int DIM> __device__ __forceinline__ void map_rows(double *HQ, const float *map)
{
    using O = OShape<DIM, 2>;
    constexpr int BW = Shape<DIM>::NQ <= 8 ? 8 : 16;
    for (int t = lane_id(); t < O::NRX * BW; t += kWave) {
        const int k = t / BW, b = t % BW;
        const float *mk = map + k * O::NR;
        double v = 0.0;
#pragma unroll
        for (int r = 0; r < O::NR; ++r) v = fma(static_cast<double>(mk[r]), HQ[r * 16 + b], v);
        HQ[(O::NR + k) * 16 + b] = v;
    }
}

// Boxes: the rows after the contraction.  HQ rows r < NR hold, per inner point
// b, sum_a w_a xi_a^{e_r} g_ab (times |det F_m'(g_b)| / |E_m|).  Then
//   PHI[I][b] = sum_r phi_I[r] HQ[r][b]   (the outer basis function phi_I),
//   R1[r]     = sum_b w_b HQ[r][b]        (the rows summed against the inner weights).
template <int DIM, int ORD> __device__ __forceinline__ void box_rows(const double *phi, double *HQ, const double *wq)
{
    using BS = BoxShape<DIM, ORD>;
    constexpr int NR = BS::NR, NB = BS::NB, NQ = BS::NQ, QS = BS::QS;
    double *PHI = HQ + NR * QS, *R1 = PHI + NB * QS;
    for (int t = lane_id(); t < NB * NQ; t += kWave) {
        const int I = t / NQ, b = t - I * NQ;
        const double *ph = phi + I * NR;
        double v = 0.0;
        for (int r = 0; r < NR; ++r) v = fma(ph[r], HQ[r * QS + b], v);
        PHI[I * QS + b] = v;
    }
    for (int r = lane_id(); r < NR; r += kWave) {
        double v = 0.0;
#pragma unroll
        for (int b = 0; b < NQ; ++b) v = fma(wq[b], HQ[r * QS + b], v);
        R1[r] = v;
    }
}

// Boxes: one per-pair output before the factor +-C |E_l| |E_m| (psi = the inner
// basis at the rule points, [NB][QS]):
//   B_lm[i][j] = sum_b w_b psi_j(b) PHI[i][b]
//   B_mm[u]    = sum_b w_b psi_i(b) psi_j(b) HQ[0][b]   (row 0: the monomial 1)
//   B_ll[u]    = sum_r prod_u[r] R1[r]
template <int DIM, int ORD>
__device__ __forceinline__ double box_output(CArgs &A, const double *HQ, const double *psi, const double *wq,
                                             int kind, int i, int j, int u)
{
    using BS = BoxShape<DIM, ORD>;
    constexpr int NR = BS::NR, NB = BS::NB, NQ = BS::NQ, QS = BS::QS;
    const double *PHI = HQ + NR * QS, *R1 = PHI + NB * QS;
    double v = 0.0;
    if (kind == kOutLM) {
#pragma unroll
        for (int b = 0; b < NQ; ++b) v = fma(wq[b] * psi[j * QS + b], PHI[i * QS + b], v);
    } else if (kind == kOutMM) {
#pragma unroll
        for (int b = 0; b < NQ; ++b) v = fma(wq[b] * psi[i * QS + b] * psi[j * QS + b], HQ[b], v);
    } else if (kind == kOutLL) {
        const double *pr = A.boxprod + u * NR;
        for (int r = 0; r < NR; ++r) v = fma(pr[r], R1[r], v);
    }
    return v;
}

// Boxes: the basis at the rule points into LDS and one descriptor per output
// (B_lm, then the B_mm and B_ll slots): kind | i << 2 | j << 7 | u << 12
template <int DIM, int ORD> __device__ void box_epilogue_tables(CArgs &A0, double *s_psi, int *s_desc)
{
    using BS = BoxShape<DIM, ORD>;
    constexpr int NB = BS::NB, NU = BS::NU, NPASS = (BS::NOUT + kWave - 1) / kWave;
    for (int t = threadIdx.x; t < NB * BS::QS; t += kThreads) s_psi[t] = A0.boxpsi[t];
    // then the outer basis over the product monomials, [NB][NR] (box_rows)
    for (int t = threadIdx.x; t < NB * BS::NR; t += kThreads) s_psi[NB * BS::QS + t] = A0.boxphi[t];
    for (int o = threadIdx.x; o < NPASS * kWave; o += kThreads) {
        int kind = kOutNone, i = 0, j = 0, u = 0;
        if (o < NB * NB) {
            kind = kOutLM;
            i = o / NB;
            j = o % NB;
        } else if (o < NB * NB + NU) {
            kind = kOutMM;
            u = o - NB * NB;
            pair_of<NB>(u, i, j);
        } else if (o < NB * NB + 2 * NU) {
            kind = kOutLL;
            u = o - NB * NB - NU;
            pair_of<NB>(u, i, j);
        }
        s_desc[o] = kind | (i << 2) | (j << 7) | (u << 12);   // i, j < 32, u < 2^19
    }
}

// -------------------------------------------------------------- one pair

template <int DIM, int PREC, int ETA, int ORD, int SHP = 0>
__device__ __forceinline__ void process_pair(CArgs &A, int l, int m, int64_t pidx, char *wmem,
                             const double *s_rule, const float *s_w32, const double *s_T, const int *s_desc,
                             const float *s_map, double *s_bll, const RowCache *rc, double *ex_block,
                             unsigned long long *s_leaf, int leafcap)
{
    using S = Shape<DIM>;
    using O = OShape<DIM, ORD>;
    using BS = BoxShape<DIM, ORD>;
    using GV = typename Geo<DIM, SHP>::type;
    constexpr int NV = S::NV, NCH = S::NCH, NVG = Geo<DIM, SHP>::NV;
    // rule points (stride RS: barycentric for simplices, reference coordinates for boxes)
    constexpr int NQ = SHP == 1 ? BS::NQ : S::NQ, RS = SHP == 1 ? DIM : NV;
    constexpr int NB = SHP == 1 ? BS::NB : O::NB, NU = SHP == 1 ? BS::NU : O::NU;
    constexpr int NOUT = SHP == 1 ? BS::NOUT : O::NOUT;
    constexpr int BATCH = SHP == 1 ? BoxAcc<DIM, ETA, ORD>::kPoints : (PREC == 0 ? PlainAcc<DIM, ETA, ORD>::kPoints : kBatch);
    // FP64: the contraction on the matrix cores (Mfma64) for the 3D elements with
    // many rows (P2 tetrahedra: 35, hexahedra: 27 / 90); measured slower for P1
    // tetrahedra (10 rows: one FP64 MFMA per 64 evaluations takes longer than the
    // ten vector multiply-adds) and no faster in 2D (7 or 9 of a tile's 16 columns
    // carry inner points)
    constexpr bool kMfma64 = PREC == 0 && DIM == 3 && (ORD == 2 || SHP == 1);
    using Base64 = typename std::conditional<SHP == 1, BoxAcc<DIM, ETA, ORD>, PlainAcc<DIM, ETA, ORD>>::type;
    constexpr int BNR = SHP == 1 ? BS::NR : O::NR;
    // lane period of the inner points handed to the accumulator
    constexpr int YS = SHP == 1 ? BS::QS : (kMfma64 ? 16 : (PREC == 0 ? PlainAcc<DIM, ETA>::NYP : (DIM == 2 ? 8 : 16)));
    using Acc64 = typename std::conditional<kMfma64, Mfma64<Base64, DIM, ETA, BNR, NQ, YS, BATCH>, Base64>::type;
    using Acc = typename std::conditional<PREC == 0, Acc64, MixedAcc<DIM, ETA>>::type;
    using Real = typename std::conditional<PREC == 0, double, float>::type;
    using WM = WaveMem<DIM, PREC, ORD, SHP>;
    const int lane = lane_id();
    const int64_t ne = A.ne;
    l = uniform(l);
    m = uniform(m);
    char *work = wmem;
    double *HQ = reinterpret_cast<double *>(wmem);   // [rows][16], after the last batch
    double *tile = HQ;                               // 16 x 16 (mixed), in place
    uint32_t *leafbuf = reinterpret_cast<uint32_t *>(wmem + WM::kWorkBytes);
    double *memo = reinterpret_cast<double *>(leafbuf + leafcap);     // WM::kMemoCount simplices
    uint32_t *stack = reinterpret_cast<uint32_t *>(reinterpret_cast<char *>(memo) + WM::kMemoBytes);   // A.capl

    // geometry of l (root simplex) and m: wave-uniform, read through the scalar
    // cache into scalar registers (read-only tables), which keeps them out of
    // the vector register budget
    typedef const __attribute__((address_space(4))) double cdouble;
    const cdouble *cvert = (const cdouble *)(A.vert);
    const cdouble *clo = (const cdouble *)(A.lo);
    const cdouble *chi = (const cdouble *)(A.hi);
    GV root;
#pragma unroll
    for (int v = 0; v < NVG; ++v)
#pragma unroll
        for (int k = 0; k < DIM; ++k) root.v[v][k] = cvert[(v * DIM + k) * ne + l];
    const cdouble *cdlo = (const cdouble *)(A.dlo);
    const cdouble *cdhi = (const cdouble *)(A.dhi);
    const cdouble *cqlo = (const cdouble *)(A.qlo);
    const cdouble *cqhi = (const cdouble *)(A.qhi);
    double mlo[DIM], mhi[DIM], dlo[DIM], dhi[DIM], qlo[DIM], qhi[DIM];
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
        mlo[k] = clo[k * ne + m];
        mhi[k] = chi[k * ne + m];
        dlo[k] = cdlo[k * ne + m];
        dhi[k] = cdhi[k * ne + m];
        qlo[k] = cqlo[k * ne + m];
        qhi[k] = cqhi[k * ne + m];
    }
    const double *bary = s_rule;
    const double *wq = s_rule + NQ * RS;
    // P1 simplices: node m_j of the epilogue's B_lm lane (lane = i * NV + j), read early
    constexpr bool kP1 = ORD == 1 && SHP == 0;
    const int32_t mj1 = kP1 ? A.conn[static_cast<int64_t>(m) * NV + lane % NV] : 0;

    // inner point of this lane, relative to the anchor v0(l)
    const int bsel = lane % YS;
    const int bq = bsel < NQ ? bsel : 0;
    double y[DIM];
    double jm = 1.0;   // boxes: |det F_m'(g_b)| / |E_m|
    if constexpr (SHP == 1) {
        BoxVerts<DIM> Pm;
#pragma unroll
        for (int c = 0; c < NVG; ++c)
#pragma unroll
            for (int k = 0; k < DIM; ++k) Pm.v[c][k] = cvert[(c * DIM + k) * ne + m];
        double N[1 << DIM];
        box_corner_weights<DIM>(bary + bq * DIM, N);
#pragma unroll
        for (int k = 0; k < DIM; ++k) {
            double s = 0.0;
#pragma unroll
            for (int c = 0; c < NVG; ++c) s = fma(N[c], Pm.v[c][k], s);
            y[k] = s - root.v[0][k];
        }
        jm = box_jacdet<DIM>(Pm, bary + bq * DIM) / A.meas[m];
    } else {
#pragma unroll
        for (int k = 0; k < DIM; ++k) {
            double s = 0.0;
#pragma unroll
            for (int v = 0; v < NV; ++v) s = fma(bary[bq * NV + v], cvert[(v * DIM + k) * ne + m], s);
            y[k] = s - root.v[0][k];
        }
    }
    // the outer element's frame: the edges v_i - v_0 of a simplex, or a box's
    // corner differences and 1/|E_l|
    typename std::conditional<SHP == 1, BoxFrame<DIM>, Edges<DIM, Real>>::type E;
    if constexpr (SHP == 1) {
#pragma unroll
        for (int c = 1; c < NVG; ++c)
#pragma unroll
            for (int k = 0; k < DIM; ++k) E.d[c - 1][k] = root.v[c][k] - root.v[0][k];
        E.inv_meas = 1.0 / A.meas[l];
    } else {
#pragma unroll
        for (int i = 1; i <= DIM; ++i)
#pragma unroll
            for (int k = 0; k < DIM; ++k) E.e[i - 1][k] = static_cast<Real>(root.v[i][k] - root.v[0][k]);
    }

    Acc acc;
    acc.init(y, lane, work);
    if constexpr (SHP == 1) acc.set_rule(bary);
    if constexpr (PREC == 1) acc.set_column(A, y, bsel < NQ);

    // integrate the leaves in leafbuf[0..nleaf)
    auto integrate = [&](int nleaf) {
        const int total = nleaf * NQ;
        auto fetch = [&](int p0) {
            const int p = p0 + lane;
            const bool valid = p < total && lane < BATCH;
            int a = 0, lev = 1, sub = 0;
            if (valid) {
                const int q = p / NQ;
                a = p - q * NQ;
                const uint32_t ent = leafbuf[q];
                lev = static_cast<int>(ent >> 24);
                sub = static_cast<int>(ent & 0xFFFFFFu);
            }
            return acc.fetch(A, valid, sub, a, lev, SHP == 1 ? 0.0f : s_w32[a], wq[a]);
        };
        auto in = fetch(0);
        for (int p0 = 0; p0 < total; p0 += BATCH) {
            wave_sync();
            if (lane < BATCH) Acc::stage(work, lane, in, E);
            wave_sync();
            if (p0 + BATCH < total) in = fetch(p0 + BATCH);
            acc.run(A, work, total - p0 < BATCH ? total - p0 : BATCH);
        }
    };

    // ---- Algorithm 1 (per pair: J = {m}), depth first in batches ------------
    // A per-wave stack holds the sub-elements still to classify as
    // (level << 24) | local index.  A pass pops up to 64 from the top (fewer when
    // the stack is near its capacity, so that the children always fit), sends
    // the J^int members to the leaf buffer, pushes the children of the J^ref
    // members, and sends the children of members one level above L_max straight
    // to the leaf buffer (Algorithm 1 integrates everything at L_max).  Leaves
    // are integrated when the buffer fills and once at the end, so batches stay
    // full across levels.
    int nleaf = 0;
    bool any_leaf = false;   // wave-uniform
    auto push_leaf = [&](bool take, uint32_t ent) {
        const unsigned long long mask = wave_ballot(take);
        const int c = __popcll(mask);
        if (c == 0) return;
        any_leaf = true;
        if (nleaf + c > leafcap) {
            integrate(nleaf);
            nleaf = 0;
        }
        wave_sync();
        if (take) leafbuf[nleaf + lanes_below(mask)] = ent;
        nleaf += c;
        wave_sync();
    };
    uint32_t *stk = stack;
    const int lmax = A.lmax, lmin = A.lmin;
    const int cap = A.capl - NCH * (lmax + 1) - kWave;   // logical capacity (see make_args)
    // memo of the vertices of levels 2..memo_lev, formed when the first of them
    // is classified; only levels below L_max are classified, and a memo pays off
    // only if some classified level lies below it (its own levels save what
    // forming it costs)
    const int memo_lev = WM::kMemoLevel < 2 ? 0 : (WM::kMemoLevel < lmax - 2 ? WM::kMemoLevel : lmax - 2);
    bool memo_ready = memo_lev < 2;
    auto build_memo = [&]() {
        // lane t < NCH: level 2, local t; then level 3, local t - NCH
        const int count = memo_lev == 2 ? NCH : WM::kMemoCount;
        if (lane < count) {
            const int tlev = lane < NCH ? 2 : 3;
            const int tloc = lane < NCH ? lane : lane - NCH;
            GV T = root;
            for (int d = tlev - 2; d >= 0; --d) T = geo_child_of<DIM, SHP>(T, (tloc >> (DIM * d)) & (NCH - 1));
            double *dst = memo + lane * NVG * DIM;
#pragma unroll
            for (int v = 0; v < NVG; ++v)
#pragma unroll
                for (int k = 0; k < DIM; ++k) dst[v * DIM + k] = T.v[v][k];
        }
        wave_sync();
        memo_ready = true;
    };
    int n = 0;
    // the actions of one classified window: J^int members to the leaf buffer;
    // children of J^ref members one level above L_max straight to the leaf
    // buffer, the others' children to the stack when `expand`.  False if the
    // stack would overflow (the pop rule below prevents it).
    auto act = [&](int lev, uint32_t local, int cls, uint32_t zmask, bool expand) {
        if (cls == 1 && s_leaf) atomicAdd(&s_leaf[lev], 1ull);
        push_leaf(cls == 1, cls == 1 ? leaf_entry(lev, level_offset<DIM>(lev) + static_cast<int>(local)) : 0u);
        const bool to_leaves = cls == 2 && lev + 1 == lmax;
        const bool to_stack = cls == 2 && lev + 1 < lmax && expand;
        const unsigned long long mpush = wave_ballot(to_stack);
        const unsigned long long mleaf = wave_ballot(to_leaves);
        if (n + static_cast<int>(__popcll(mpush)) * NCH + static_cast<int>(__popcll(mleaf)) > A.capl) {
            // never write past the stack
            if (lane == 0) atomicOr(&A.counters->error, kErrStack);
            return false;
        }
        if (to_stack) {
            const uint32_t base = (static_cast<uint32_t>(lev + 1) << 24) | (local * NCH);
            const int at = n + lanes_below(mpush) * NCH;
#pragma unroll
            for (int c = 0; c < NCH; ++c) stk[at + c] = base + c;
        }
        n += static_cast<int>(__popcll(mpush)) * NCH;
        if (mleaf) {
            // parents above the pushed region (with their zero-children masks in
            // the top byte: local indices are below 2^24), then their children
            // packed across lanes; a child whose integrals are all zeros is
            // counted as Algorithm 1's leaf but not integrated
            if (to_leaves) stk[n + lanes_below(mleaf)] = (zmask << 24) | local;
            wave_sync();
            const int nl = __popcll(mleaf) * NCH;
            const int offn = level_offset<DIM>(lmax);
            int nzero = 0;
            for (int i0 = 0; i0 < nl; i0 += kWave) {
                const int i = i0 + lane;
                const bool take = i < nl;
                const uint32_t e = take ? stk[n + i / NCH] : 0u;
                const int c = i % NCH;
                const bool live = take && ((e >> (24 + c)) & 1u) == 0u;
                nzero += __popcll(wave_ballot(take && !live));
                const int sub = live ? offn + static_cast<int>((e & 0xFFFFFFu) * NCH + c) : 0;
                push_leaf(live, leaf_entry(lmax, sub));
            }
            if (lane == 0 && s_leaf) {
                atomicAdd(&s_leaf[lmax], static_cast<unsigned long long>(nl));
                if (nzero) atomicAdd(&s_leaf[0], static_cast<unsigned long long>(nzero));
            }
        }
        wave_sync();
        return true;
    };
    // The top of the tree without the stack: the root is classified by every lane
    // alike; if it is refined, levels 2..sl (NCH [+ NCH^2] nodes, a lane each, in
    // the memo's lane order) are classified in one pass instead of one pop per
    // level, a node counting only if its level-2 ancestor was refined too -- the
    // same leaf set as the pops give.
    constexpr int kTopLevels = DIM == 2 ? 3 : 2;
    const int sl = kTopLevels < lmax - 1 ? kTopLevels : lmax - 1;
    bool ok = true;
    if (sl >= 2) {
        uint32_t z0 = 0u;
        const int rc = 1 < lmin ? 2 : classify<DIM, SHP>(A, root, memo, memo_lev, 1, 0u, mlo, mhi, dlo, dhi, qlo, qhi, &z0);
        if (rc == 2) {
            const int ntop = sl == 2 ? NCH : NCH + NCH * NCH;
            const bool valid = lane < ntop;
            const int lev = lane < NCH ? 2 : 3;
            const uint32_t local = static_cast<uint32_t>(lane < NCH ? lane : lane - NCH);
            if (!memo_ready) build_memo();
            int cls = 0;
            uint32_t zm = 0u;
            if (valid)
                cls = lev < lmin ? 2 : classify<DIM, SHP>(A, root, memo, memo_lev, lev, local, mlo, mhi, dlo, dhi, qlo, qhi, &zm);
            // the parent of level-3 node `local` is level-2 node local / NCH, in that lane
            const unsigned long long ref = wave_ballot(valid && cls == 2);
            const bool reach = lev == 2 || ((ref >> (local >> DIM)) & 1ull) != 0;
            ok = act(lev, local, valid && reach ? cls : 0, zm, lev == sl);
        } else {
            ok = act(1, 0u, lane == 0 ? rc : 0, z0, false);
        }
    } else {
        n = 1;
        if (lane == 0) stk[0] = 1u << 24;
        wave_sync();
    }
    while (ok && n > 0) {
        // pop the largest top window whose refinable members (level < L_max - 1:
        // the only ones that push) fit: NCH * pushers - k <= cap - n, at least 1
        const int w = n < kWave ? n : kWave;
        int k = 1;
        {
            const uint32_t e = lane < w ? stk[n - 1 - lane] : 0u;
            const bool pusher = lane < w && static_cast<int>(e >> 24) < lmax - 1;
            const unsigned long long pm = wave_ballot(pusher);
            const unsigned long long upto = lane == 63 ? ~0ull : ((2ull << lane) - 1ull);
            const int kk = lane + 1;
            // signed: __popcll returns an unsigned count, and cap - n may be negative
            const int pushers = static_cast<int>(__popcll(pm & upto));
            const bool ok = lane < w && NCH * pushers - kk <= cap - n;
            const unsigned long long okm = wave_ballot(ok);
            if (okm) k = 64 - __clzll(okm);
        }
        n -= k;
        const bool valid = lane < k;
        const uint32_t ent = valid ? stk[n + lane] : 0u;
        wave_sync();
        const int lev = static_cast<int>(ent >> 24);
        const uint32_t local = ent & 0xFFFFFFu;
        if (!memo_ready && wave_ballot(valid && lev >= 2)) build_memo();
        int cls = 0;
        uint32_t zm = 0u;
        if (valid) {
            if (lev == lmax) cls = 1;                 // the root when L_max = 1
            else if (lev < lmin) cls = 2;
            else cls = classify<DIM, SHP>(A, root, memo, memo_lev, lev, local, mlo, mhi, dlo, dhi, qlo, qhi, &zm);
        }
        ok = act(lev, local, cls, zm, true);
    }
    if (nleaf > 0) integrate(nleaf);
    // a pair without leaves (every sub-element dropped) has zero blocks: nothing to
    // add (the explicit and deterministic outputs are still written)
    if (!any_leaf && !ex_block && !A.pb) return;

    // ---- epilogue (FP64) ----------------------------------------------------
    wave_sync();
    if constexpr (SHP == 1) {
        acc.finish(HQ, jm);
        wave_sync();
        box_rows<DIM, ORD>(s_T + NB * BS::QS, HQ, wq);
    } else {
        acc.finish(HQ, tile);
        wave_sync();
        if constexpr (ORD == 1) extend_rows<DIM>(HQ);
        else map_rows<DIM>(HQ, s_map);
    }
    wave_sync();
    const double Sc = A.C * A.meas[l] * A.meas[m];
    const bool four = A.form == NLQ_FORM_SYM4;
    // the two-term form with the adaptive rule on the inner integral: rows of the
    // refined (outer) element, 2 B_ll and 2 B_lm (see the oracle's form 2)
    const bool inner = A.form == NLQ_FORM_PAPER2_INNER;
    constexpr int NPASS = (NOUT + kWave - 1) / kWave;
    // Boxes accumulated into the CSR matrix: B_ll = sum_r prod_u[r] R1[r] is linear in
    // the weighted row sums R1, so the pair adds its scaled R1 to the outer
    // element's sums (in s_bll; NR <= NU) and the work item forms B_ll from them
    // once (k_integrate); explicit blocks form B_ll per pair
    const bool box_r1 = SHP == 1 && !ex_block && !A.pb;
    if constexpr (SHP == 1) {
        if (box_r1 && (four || inner)) {
            const double *R1 = HQ + BS::NR * BS::QS + BS::NB * BS::QS;
            const double f = inner ? 2.0 * Sc : Sc;
            for (int r = lane; r < BS::NR; r += kWave) atomicAdd(&s_bll[r], f * R1[r]);
        }
    }
    const int npass = box_r1 ? (NB * NB + NU + kWave - 1) / kWave : NPASS;
    for (int pass = 0; pass < npass; ++pass) {
        const int o = pass * kWave + lane;
        const int desc = s_desc[o];
        const int kind = desc & 3;
        if (box_r1 && kind == kOutLL) continue;
        int i, j, u;
        double v = 0.0;
        if constexpr (SHP == 1) {
            i = (desc >> 2) & 31;
            j = (desc >> 7) & 31;
            u = desc >> 12;
            v = box_output<DIM, ORD>(A, HQ, s_T, wq, kind, i, j, u);
        } else {
            // every output is a dot product over the inner points b of one row
            // after the contraction with one constant row of s_T; the descriptor
            // names both
            const int xr = (desc >> 2) & 127, tr = (desc >> 9) & 127;
            i = (desc >> 16) & 15;
            j = (desc >> 20) & 15;
            u = (desc >> 24) & 63;
            const double *x = HQ + xr * 16;
            const double *tt = s_T + tr * 16;
#pragma unroll
            for (int b = 0; b < NQ; ++b) v = fma(x[b], tt[b], v);
        }
        v *= kind == kOutLM ? -Sc : Sc;
        if (ex_block) {
            constexpr int N2 = 2 * NB;
            if (kind == kOutLM) {
                ex_block[i * N2 + NB + j] = four ? v : (inner ? 2.0 * v : 0.0);
                ex_block[(NB + j) * N2 + i] = four ? v : (inner ? 0.0 : 2.0 * v);
            } else if (kind == kOutMM) {
                ex_block[(NB + i) * N2 + NB + j] = four ? v : (inner ? 0.0 : 2.0 * v);
                ex_block[(NB + j) * N2 + NB + i] = four ? v : (inner ? 0.0 : 2.0 * v);
            } else if (kind == kOutLL) {
                ex_block[i * N2 + j] = four ? v : (inner ? 2.0 * v : 0.0);
                ex_block[j * N2 + i] = four ? v : (inner ? 2.0 * v : 0.0);
            }
            continue;
        }
        if (A.pb) {
            // deterministic mode: the outputs of pair pidx, in descriptor order, are
            // summed later in a fixed order
            if (kind != kOutNone) A.pb[(pidx - A.pb_base) * NOUT + o] = v;
            continue;
        }
        if (kind == kOutLM) {
            // B_lm at (l_i, m_j) through the cached row of l_i.  SYM4 adds it to the
            // half matrix R (A = R + R^T afterwards); the two-term form puts 2 B_lm^T
            // at (m_j, l_i) directly, its adaptive-inner variant 2 B_lm at (l_i, m_j).
            const int32_t mj = kP1 ? mj1 : A.conn[static_cast<int64_t>(m) * NB + j];
            const int64_t at = row_find(rc, i, mj);
            if (at >= 0) {
                const int64_t pos = rc->base[i] + at;
                if (four) unsafeAtomicAdd(&A.val[pos], v);
                else if (inner) unsafeAtomicAdd(&A.val[pos], 2.0 * v);
                else unsafeAtomicAdd(&A.val[A.tmap[pos]], 2.0 * v);
            } else {
                // (l_i, m_j) outside the pattern: the pair list and the pattern disagree
                atomicOr(&A.counters->error, kErrPattern);
            }
        } else if (kind == kOutMM) {
            if (!inner) unsafeAtomicAdd(&A.dmm[static_cast<int64_t>(m) * NU + u], four ? v : 2.0 * v);
        } else if (kind == kOutLL) {
            if (four) atomicAdd(&s_bll[u], v);
            else if (inner) atomicAdd(&s_bll[u], 2.0 * v);
        }
    }
}

// -------------------------------------------------------------- kernels

// Occupancy hint: more waves per SIMD cover LDS and table latency at the cost of
// registers (5 waves in 2D, 4 for the 3D FP32 path and 3 for the 3D FP64 path
// were fastest on the 2D 128^2 and 3D 8^3 cases; see waves_per_eu).  P2 and box
// elements: 2 waves per SIMD, 1 for hexahedra, so that their wider rows, frames
// and accumulators stay in registers instead of spilling.
template <int DIM, int PREC, int OCC, int ORD, int SHP> constexpr int kernel_waves()
{
    return SHP == 1 && DIM == 3 ? 1 : (SHP == 1 || ORD == 2 ? 2 : waves_per_eu<DIM, PREC, OCC>());
}

template <int DIM, int PREC, int ETA, int OCC, int ORD, int SHP = 0>
__global__ void __launch_bounds__(kThreads)
    __attribute__((amdgpu_waves_per_eu(kernel_waves<DIM, PREC, OCC, ORD, SHP>())))
k_integrate(LaunchArgs L)
{
    using S = Shape<DIM>;
    using O = OShape<DIM, ORD>;
    using BS = BoxShape<DIM, ORD>;
    using WM = WaveMem<DIM, PREC, ORD, SHP>;
    constexpr int NV = S::NV, RS = SHP == 1 ? DIM : NV, NQ = SHP == 1 ? BS::NQ : S::NQ;
    constexpr int NB = SHP == 1 ? BS::NB : O::NB, NU = SHP == 1 ? BS::NU : O::NU;
    constexpr int NOUT = SHP == 1 ? BS::NOUT : O::NOUT;
    extern __shared__ __align__(16) char smem[];
    __shared__ double s_rule[NQ * RS + NQ];
    __shared__ float s_w32[16];
    // simplices: the constant rows of epilogue_tables; boxes: the inner basis [NB][QS], then the outer basis [NB][NR]
    __shared__ __align__(16) double s_T[SHP == 1 ? NB * (BS::QS + BS::NR) : (NB + NU + 1) * 16];
    __shared__ int s_desc[(NOUT + kWave - 1) / kWave * kWave];
    // the P2 row map: small integers, exact in FP32 (checked where it is built)
    __shared__ float s_map[ORD == 1 || SHP == 1 ? 1 : O::NRX * O::NR];
    __shared__ double s_bll[NU];
    static_assert(SHP != 1 || BS::NR <= NU, "a box's weighted row sums are summed in s_bll");
    __shared__ int64_t s_seg[kMaxSeg + 1];
    __shared__ int64_t s_item;
    __shared__ int s_sys;
    __shared__ int s_part;
    __shared__ int s_next;
    __shared__ unsigned long long s_leaf[10];
    __shared__ RowCache s_rc;
    const int wid = threadIdx.x / kWave;
    char *wmem = smem + wid * WM::bytes(L.capl, L.leafcap);
    uint16_t *rows_lds = reinterpret_cast<uint16_t *>(smem + kWaves * WM::bytes(L.capl, L.leafcap));
    // the quadrature rule (and the P2 map) depends on the dimension only: every
    // system of the launch shares it
    CArgs &A0 = *(CArgs *)(L.sys);
    const double *rule0 = SHP == 1 ? A0.boxrule : A0.rule;
    for (int t = threadIdx.x; t < NQ * RS + NQ; t += kThreads) s_rule[t] = rule0[t];
    if constexpr (ORD == 2 && SHP == 0)
        for (int t = threadIdx.x; t < O::NRX * O::NR; t += kThreads) s_map[t] = static_cast<float>(A0.p2map[t]);
    if (SHP == 0 && threadIdx.x < NQ) s_w32[threadIdx.x] = static_cast<float>(A0.rule[NQ * NV + threadIdx.x]);
    for (int t = threadIdx.x; t <= L.nseg; t += kThreads) s_seg[t] = L.seg_start[t];
    __syncthreads();
    if constexpr (SHP == 1) box_epilogue_tables<DIM, ORD>(A0, s_T, s_desc);
    else epilogue_tables<DIM, ORD>(s_rule, s_T, s_desc);
    const int64_t total = s_seg[L.nseg];
    for (;;) {
        if (threadIdx.x == 0) {
            const int64_t w = atomicAdd(L.counter, 1u);
            int64_t item = -1;
            int sys = 0, part = 0;
            if (w < total) {
                int lo = 0, hi = L.nseg - 1;   // last segment with s_seg[k] <= w
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (s_seg[mid] <= w) lo = mid; else hi = mid - 1;
                }
                sys = L.seg_sys[lo];
                const int split = L.sys[sys].split;
                const int64_t i = w - s_seg[lo];
                item = L.seg_lo[lo] + i / split;
                part = static_cast<int>(i % split);
            }
            s_item = item;
            s_sys = sys;
            s_part = part;
        }
        if (threadIdx.x < NU) s_bll[threadIdx.x] = 0.0;
        if (threadIdx.x < 10) s_leaf[threadIdx.x] = 0ull;
        __syncthreads();
        const int64_t l = s_item;
        if (l < 0) break;
        CArgs &A = *(CArgs *)(L.sys + __builtin_amdgcn_readfirstlane(s_sys));
        // stage the CSR rows of l's nodes
        if (threadIdx.x < NB) {
            const int32_t node = A.conn[l * NB + threadIdx.x];
            const int64_t b = A.row_ptr[node], len = A.row_ptr[node + 1] - b;
            const int32_t first = len > 0 ? A.col[b] : 0;
            const bool fits = len <= L.rowcap && (len == 0 || A.col[b + len - 1] - first <= 65535);
            s_rc.base[threadIdx.x] = b;
            s_rc.len[threadIdx.x] = len;
            s_rc.first[threadIdx.x] = first;
            s_rc.cols[threadIdx.x] = A.col + b;
            s_rc.c16[threadIdx.x] = fits ? rows_lds + threadIdx.x * L.rowcap : nullptr;
            const int scap = row_sample_cap(L.rowcap);
            int step = 0, ns = 0;
            if (!fits && scap > 0) {
                step = static_cast<int>((len + scap - 1) / scap);
                ns = static_cast<int>((len + step - 1) / step);
            }
            const uintptr_t area = reinterpret_cast<uintptr_t>(rows_lds + threadIdx.x * L.rowcap);
            s_rc.samp[threadIdx.x] = reinterpret_cast<const int32_t *>((area + 3) & ~static_cast<uintptr_t>(3));
            s_rc.step[threadIdx.x] = step;
            s_rc.nsamp[threadIdx.x] = ns;
        }
        __syncthreads();
        for (int r = 0; r < NB; ++r) {
            uint16_t *dst = const_cast<uint16_t *>(s_rc.c16[r]);
            if (dst) {
                for (int64_t k = threadIdx.x; k < s_rc.len[r]; k += kThreads)
                    dst[k] = static_cast<uint16_t>(A.col[s_rc.base[r] + k] - s_rc.first[r]);
            } else {
                int32_t *sm = const_cast<int32_t *>(s_rc.samp[r]);
                for (int k = threadIdx.x; k < s_rc.nsamp[r]; k += kThreads)
                    sm[k] = A.col[s_rc.base[r] + static_cast<int64_t>(k) * s_rc.step[r]];
            }
        }
        __syncthreads();
        const int64_t b0 = A.pair_off[l];
        const int nJ = static_cast<int>(A.pair_off[l + 1] - b0);
        // this item's part of J_l
        const int chunk = (nJ + A.split - 1) / A.split;
        const int p_lo = min(nJ, s_part * chunk), p_hi = min(nJ, p_lo + chunk);
        if (threadIdx.x == 0) s_next = p_lo;
        __syncthreads();
        for (;;) {
            int p = 0;
            if (lane_id() == 0) p = atomicAdd(&s_next, 1);
            p = bcast0(p);
            if (p >= p_hi) break;
            const int32_t m = A.pair_m[b0 + p];
            process_pair<DIM, PREC, ETA, ORD, SHP>(A, static_cast<int>(l), m, b0 + p, wmem, s_rule, s_w32, s_T,
                                                   s_desc, s_map, s_bll, &s_rc, nullptr, s_leaf, L.leafcap);
        }
        __syncthreads();
        // B_ll of l (upper triangle; doubled for the adaptive-inner two-term form)
        // joins the diagonal-block sums of l; boxes form it here from the summed
        // weighted row sums
        if (A.form != NLQ_FORM_PAPER2 && !A.pb && threadIdx.x < NU) {
            double v = s_bll[threadIdx.x];
            if constexpr (SHP == 1) {
                const double *pr = A.boxprod + threadIdx.x * BS::NR;
                v = 0.0;
                for (int r = 0; r < BS::NR; ++r) v = fma(pr[r], s_bll[r], v);
            }
            unsafeAtomicAdd(&A.dmm[l * NU + threadIdx.x], v);
        }
        if (threadIdx.x >= 1 && threadIdx.x <= A.lmax && s_leaf[threadIdx.x])
            atomicAdd(&A.counters->leaf[threadIdx.x], s_leaf[threadIdx.x]);
        if (threadIdx.x == 0 && s_leaf[0]) atomicAdd(&A.counters->zero_leaves, s_leaf[0]);
        if (threadIdx.x == 0 && p_hi > p_lo)
            atomicAdd(&A.counters->pairs_done, static_cast<unsigned long long>(p_hi - p_lo));
        __syncthreads();
    }
}

// explicit pairs of system 0: every wave takes pairs from the counter and
// writes the extended block [2N+2][2N+2] of each
template <int DIM, int PREC, int ETA, int ORD, int SHP = 0>
__global__ void __launch_bounds__(kThreads)
k_pair_blocks(LaunchArgs L)
{
    using S = Shape<DIM>;
    using O = OShape<DIM, ORD>;
    using BS = BoxShape<DIM, ORD>;
    constexpr int NV = S::NV, RS = SHP == 1 ? DIM : NV, NQ = SHP == 1 ? BS::NQ : S::NQ;
    constexpr int NB = SHP == 1 ? BS::NB : O::NB, NU = SHP == 1 ? BS::NU : O::NU;
    constexpr int NOUT = SHP == 1 ? BS::NOUT : O::NOUT;
    extern __shared__ __align__(16) char smem[];
    __shared__ double s_rule[NQ * RS + NQ];
    __shared__ float s_w32[16];
    __shared__ __align__(16) double s_T[SHP == 1 ? NB * (BS::QS + BS::NR) : (NB + NU + 1) * 16];
    __shared__ int s_desc[(NOUT + kWave - 1) / kWave * kWave];
    // the P2 row map: small integers, exact in FP32 (checked where it is built)
    __shared__ float s_map[ORD == 1 || SHP == 1 ? 1 : O::NRX * O::NR];
    CArgs &A = *(CArgs *)(L.sys);
    const int wid = threadIdx.x / kWave;
    char *wmem = smem + wid * WaveMem<DIM, PREC, ORD, SHP>::bytes(L.capl, L.leafcap);
    const double *rule0 = SHP == 1 ? A.boxrule : A.rule;
    for (int t = threadIdx.x; t < NQ * RS + NQ; t += kThreads) s_rule[t] = rule0[t];
    if (SHP == 0 && threadIdx.x < NQ) s_w32[threadIdx.x] = static_cast<float>(A.rule[NQ * NV + threadIdx.x]);
    if constexpr (ORD == 2 && SHP == 0)
        for (int t = threadIdx.x; t < O::NRX * O::NR; t += kThreads) s_map[t] = static_cast<float>(A.p2map[t]);
    __syncthreads();
    if constexpr (SHP == 1) box_epilogue_tables<DIM, ORD>(A, s_T, s_desc);
    else epilogue_tables<DIM, ORD>(s_rule, s_T, s_desc);
    __syncthreads();
    for (;;) {
        unsigned int it = 0;
        if (lane_id() == 0) it = atomicAdd(L.counter, 1u);
        it = bcast0(it);
        if (it >= A.n_explicit) break;
        double *blk = A.ex_out + static_cast<int64_t>(it) * (2 * NB) * (2 * NB);
        for (int t = lane_id(); t < 4 * NB * NB; t += kWave) blk[t] = 0.0;
        wave_sync();
        process_pair<DIM, PREC, ETA, ORD, SHP>(A, A.ex_l[it], A.ex_m[it], -1, wmem, s_rule, s_w32, s_T, s_desc,
                                               s_map, nullptr, nullptr, blk, nullptr, L.leafcap);
    }
}

// Diagonal blocks into the CSR values: slot u = (i, j), i <= j, of element e goes
// to (e_i, e_j).  SYM4 halves the diagonal slots, so that R + R^T restores every
// symmetric block; the two-term form adds both triangles directly.
template <int NB>
__global__ void __launch_bounds__(256) k_fold_diag(int64_t ne, const double *dmm, const int32_t *elpos,
                                                  double *val, int four)
{
    constexpr int NU = NB * (NB + 1) / 2;
    const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= ne * NU) return;
    const int64_t e = t / NU;
    const int u = static_cast<int>(t - e * NU);
    int i, j;
    pair_of<NB>(u, i, j);
    const double d = dmm[t];
    const int32_t *ep = elpos + e * NB * NB;
    if (four) {
        unsafeAtomicAdd(&val[ep[i * NB + j]], i == j ? 0.5 * d : d);
    } else {
        unsafeAtomicAdd(&val[ep[i * NB + j]], d);
        if (i != j) unsafeAtomicAdd(&val[ep[j * NB + i]], d);
    }
}

// A = R + R^T in place: the entry p and its transpose t are written by the
// thread of min(p, t) only, diagonal entries are doubled.
__global__ void __launch_bounds__(256) k_symmetrize(int64_t nnz, const int32_t *tmap, double *val)
{
    const int64_t p = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (p >= nnz) return;
    const int64_t t = tmap[p];
    if (p < t) {
        const double s = val[p] + val[t];
        val[p] = s;
        val[t] = s;
    } else if (p == t) {
        val[p] = 2.0 * val[p];
    }
}

// workgroups per CU of one launch and its dynamic LDS bytes
// LDS of a workgroup: static tables plus the dynamic per-wave areas and cached
// CSR rows within 160 KiB
constexpr int kLdsBytes = 160 * 1024;

// the cached CSR row capacity that fits the LDS next to the per-wave areas
// (rows longer than that are searched in global memory)
template <int DIM, int PREC, int ETA, int OCC, int ORD, int SHP>
int fit_rowcap(int capl, int rowcap, int leafcap)
{
    auto kern = k_integrate<DIM, PREC, ETA, OCC, ORD, SHP>;
    hipFuncAttributes fa{};
    NLQ_HIP(hipFuncGetAttributes(&fa, reinterpret_cast<const void *>(kern)));
    const int nb = SHP == 1 ? BoxShape<DIM, ORD>::NB : OShape<DIM, ORD>::NB;
    const int fixed = static_cast<int>(fa.sharedSizeBytes) + 16 + kWaves * WaveMem<DIM, PREC, ORD, SHP>::bytes(capl, leafcap);
    // the LDS share of one workgroup when a CU holds as many as its registers
    // allow (one wave per SIMD each); if that leaves under 64 entries a row, one
    // workgroup takes the whole LDS instead (rows that do not fit are searched
    // through their sampled columns, see RowCache)
    int room = kLdsBytes / kernel_waves<DIM, PREC, OCC, ORD, SHP>() - fixed;
    if (room / (2 * nb) - 8 < 64) room = kLdsBytes - fixed;
    const int fit = room / (2 * nb) - 8;
    return std::max(1, std::min(rowcap, fit));
}

template <int DIM, int PREC, int ETA, int OCC, int ORD, int SHP = 0>
int occupancy(int capl, int rowcap, int leafcap, bool explicit_mode, int *lds_out)
{
    const int per_wave = WaveMem<DIM, PREC, ORD, SHP>::bytes(capl, leafcap);
    const int nb = SHP == 1 ? BoxShape<DIM, ORD>::NB : OShape<DIM, ORD>::NB;
    const int lds = kWaves * per_wave + (explicit_mode ? 0 : ((nb * rowcap * 2 + 15) & ~15));
    auto kern = explicit_mode ? k_pair_blocks<DIM, PREC, ETA, ORD, SHP> : k_integrate<DIM, PREC, ETA, OCC, ORD, SHP>;
    {
        hipFuncAttributes fa{};
        NLQ_HIP(hipFuncGetAttributes(&fa, reinterpret_cast<const void *>(kern)));
        if (lds + static_cast<int>(fa.sharedSizeBytes) > kLdsBytes)
            fail(NLQ_EINVAL, "lmax too large for the per-wave refinement lists");
    }
    NLQ_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                hipFuncAttributeMaxDynamicSharedMemorySize, lds));
    int per_cu = 0;
    NLQ_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, kThreads, lds));
    if (lds_out) *lds_out = lds;
    return per_cu < 1 ? 1 : per_cu;
}

template <int DIM, int PREC, int ETA, int OCC, int ORD = 1, int SHP = 0>
void launch_one(Ctx *ctx, const LaunchArgs &L0, int64_t items, hipStream_t st, bool explicit_mode,
                int wg_per_cu, hipEvent_t e0, hipEvent_t e1)
{
    LaunchArgs L = L0;
    if (!explicit_mode) L.rowcap = fit_rowcap<DIM, PREC, ETA, OCC, ORD, SHP>(L.capl, L.rowcap, L.leafcap);
    int lds = 0;
    int per_cu = occupancy<DIM, PREC, ETA, OCC, ORD, SHP>(L.capl, L.rowcap, L.leafcap, explicit_mode, &lds);
    if (wg_per_cu > 0 && wg_per_cu < per_cu) per_cu = wg_per_cu;
    auto kern = explicit_mode ? k_pair_blocks<DIM, PREC, ETA, ORD, SHP> : k_integrate<DIM, PREC, ETA, OCC, ORD, SHP>;
    int64_t grid = static_cast<int64_t>(ctx->n_cu) * per_cu;
    if (grid > items) grid = items;
    if (grid < 1) grid = 1;
    if (e0) NLQ_HIP(hipEventRecord(e0, st));
    hipLaunchKernelGGL(kern, dim3(static_cast<unsigned>(grid)), dim3(kThreads), lds, st, L);
    NLQ_CHECK_LAUNCH();
    if (e1) NLQ_HIP(hipEventRecord(e1, st));
}

// one template instance per (dim, precision, kernel, register variant)
template <int DIM, int PREC>
void launch_var(Ctx *ctx, int kernel, const TuneConfig &c, const LaunchArgs &L, int64_t items, hipStream_t st,
                bool ex, hipEvent_t e0, hipEvent_t e1)
{
    const bool gauss = kernel == NLQ_ETA_GAUSS;
    if (c.occ == 0) {
        if (gauss) launch_one<DIM, PREC, NLQ_ETA_GAUSS, 0>(ctx, L, items, st, ex, c.wg_per_cu, e0, e1);
        else launch_one<DIM, PREC, NLQ_ETA_CONST, 0>(ctx, L, items, st, ex, c.wg_per_cu, e0, e1);
    } else {
        if (gauss) launch_one<DIM, PREC, NLQ_ETA_GAUSS, 1>(ctx, L, items, st, ex, c.wg_per_cu, e0, e1);
        else launch_one<DIM, PREC, NLQ_ETA_CONST, 1>(ctx, L, items, st, ex, c.wg_per_cu, e0, e1);
    }
}

void dispatch(Ctx *ctx, const System &s, const TuneConfig &c, const LaunchArgs &L, int64_t items, hipStream_t st,
              bool ex, hipEvent_t e0, hipEvent_t e1)
{
    const int dim = s.mesh->dim;
    if (s.mesh->shape == 1) {
        // quadrilaterals / hexahedra: FP64 plain path only, one register variant
        if (s.p.precision != NLQ_FP64_PLAIN) fail(NLQ_EINVAL, "box elements take the FP64 plain path");
        const bool g = s.p.kernel == NLQ_ETA_GAUSS;
        const int wpc = c.wg_per_cu;
        const bool q2 = s.mesh->order == 2;
        if (dim == 2) {
            if (q2) {
                if (g) launch_one<2, 0, NLQ_ETA_GAUSS, 0, 2, 1>(ctx, L, items, st, ex, wpc, e0, e1);
                else launch_one<2, 0, NLQ_ETA_CONST, 0, 2, 1>(ctx, L, items, st, ex, wpc, e0, e1);
            } else {
                if (g) launch_one<2, 0, NLQ_ETA_GAUSS, 0, 1, 1>(ctx, L, items, st, ex, wpc, e0, e1);
                else launch_one<2, 0, NLQ_ETA_CONST, 0, 1, 1>(ctx, L, items, st, ex, wpc, e0, e1);
            }
        } else {
            if (q2) {
                if (g) launch_one<3, 0, NLQ_ETA_GAUSS, 0, 2, 1>(ctx, L, items, st, ex, wpc, e0, e1);
                else launch_one<3, 0, NLQ_ETA_CONST, 0, 2, 1>(ctx, L, items, st, ex, wpc, e0, e1);
            } else {
                if (g) launch_one<3, 0, NLQ_ETA_GAUSS, 0, 1, 1>(ctx, L, items, st, ex, wpc, e0, e1);
                else launch_one<3, 0, NLQ_ETA_CONST, 0, 1, 1>(ctx, L, items, st, ex, wpc, e0, e1);
            }
        }
        return;
    }
    if (s.mesh->order == 2) {
        // P2 elements: FP64 plain path only, one register variant
        if (s.p.precision != NLQ_FP64_PLAIN) fail(NLQ_EINVAL, "P2 elements take the FP64 plain path");
        const bool g = s.p.kernel == NLQ_ETA_GAUSS;
        const int wpc = c.wg_per_cu;
        if (dim == 2) {
            if (g) launch_one<2, 0, NLQ_ETA_GAUSS, 0, 2>(ctx, L, items, st, ex, wpc, e0, e1);
            else launch_one<2, 0, NLQ_ETA_CONST, 0, 2>(ctx, L, items, st, ex, wpc, e0, e1);
        } else {
            if (g) launch_one<3, 0, NLQ_ETA_GAUSS, 0, 2>(ctx, L, items, st, ex, wpc, e0, e1);
            else launch_one<3, 0, NLQ_ETA_CONST, 0, 2>(ctx, L, items, st, ex, wpc, e0, e1);
        }
        return;
    }
    if (dim == 2) {
        if (s.p.precision == NLQ_FP64_PLAIN) launch_var<2, 0>(ctx, s.p.kernel, c, L, items, st, ex, e0, e1);
        else launch_var<2, 1>(ctx, s.p.kernel, c, L, items, st, ex, e0, e1);
    } else {
        if (s.p.precision == NLQ_FP64_PLAIN) launch_var<3, 0>(ctx, s.p.kernel, c, L, items, st, ex, e0, e1);
        else launch_var<3, 1>(ctx, s.p.kernel, c, L, items, st, ex, e0, e1);
    }
}

template <int DIM, int PREC>
int occupancy_of(int kernel, int occ, int capl, int rowcap, int leafcap, int order, int shape)
{
    const bool g = kernel == NLQ_ETA_GAUSS;
    if (shape == 1) {
        if (PREC != 0) fail(NLQ_EINVAL, "box elements take the FP64 plain path");
        if (order == 2) {
            rowcap = g ? fit_rowcap<DIM, 0, 1, 0, 2, 1>(capl, rowcap, leafcap)
                       : fit_rowcap<DIM, 0, 0, 0, 2, 1>(capl, rowcap, leafcap);
            return g ? occupancy<DIM, 0, 1, 0, 2, 1>(capl, rowcap, leafcap, false, nullptr)
                     : occupancy<DIM, 0, 0, 0, 2, 1>(capl, rowcap, leafcap, false, nullptr);
        }
        rowcap = g ? fit_rowcap<DIM, 0, 1, 0, 1, 1>(capl, rowcap, leafcap)
                   : fit_rowcap<DIM, 0, 0, 0, 1, 1>(capl, rowcap, leafcap);
        return g ? occupancy<DIM, 0, 1, 0, 1, 1>(capl, rowcap, leafcap, false, nullptr)
                 : occupancy<DIM, 0, 0, 0, 1, 1>(capl, rowcap, leafcap, false, nullptr);
    }
    if (order == 2) {
        if (PREC != 0) fail(NLQ_EINVAL, "P2 elements take the FP64 plain path");
        return g ? occupancy<DIM, 0, 1, 0, 2>(capl, rowcap, leafcap, false, nullptr)
                 : occupancy<DIM, 0, 0, 0, 2>(capl, rowcap, leafcap, false, nullptr);
    }
    if (occ == 0) return g ? occupancy<DIM, PREC, 1, 0, 1>(capl, rowcap, leafcap, false, nullptr)
                           : occupancy<DIM, PREC, 0, 0, 1>(capl, rowcap, leafcap, false, nullptr);
    return g ? occupancy<DIM, PREC, 1, 1, 1>(capl, rowcap, leafcap, false, nullptr)
             : occupancy<DIM, PREC, 0, 1, 1>(capl, rowcap, leafcap, false, nullptr);
}

// leaf buffer entries per wave of a system's configuration
int leaf_cap_of(const System &s)
{
    const int c = s.cfg.leaf_cap;
    if (c < kLeafCapMin || c > kLeafCapMax) fail(NLQ_EINVAL, "leaf buffer capacity out of range");
    return c;
}

// work items per outer element of a system
int split_of(const System &s)
{
    const int64_t ppi = s.cfg.pairs_per_item > 0 ? s.cfg.pairs_per_item : kPairsPerItem;
    return static_cast<int>(std::max<int64_t>(1, (s.max_pairs + ppi - 1) / ppi));
}

// smallest s >= 0 with fl(sqrt(s)) >= t (t > 0; sqrt correctly rounded)
double sqrt_threshold(double t)
{
    double x = t * t;
    while (x > 0.0 && std::sqrt(x) >= t) x = std::nextafter(x, 0.0);
    while (std::sqrt(x) < t) x = std::nextafter(x, HUGE_VAL);
    return x;
}

AsmArgs make_args(const System &s, const Tables &T)
{
    const Mesh &m = *s.mesh;
    if (T.n_sub * T.nq * T.nv >= (int64_t(1) << 31) || T.n_sub >= (1 << 24))
        fail(NLQ_EINVAL, "refinement table too large");
    AsmArgs A{};
    A.ne = m.n_elems;
    A.pair_off = s.pair_off.as<int64_t>();
    A.pair_m = s.pair_m.as<int32_t>();
    A.vert = s.vert.as<double>();
    A.lo = s.lo.as<double>();
    A.hi = s.hi.as<double>();
    A.dlo = s.p.min_dist_l2 == 2 ? s.qlo.as<double>() : A.lo;
    A.dhi = s.p.min_dist_l2 == 2 ? s.qhi.as<double>() : A.hi;
    A.qlo = s.qlo.as<double>();
    A.qhi = s.qhi.as<double>();
    A.meas = s.meas.as<double>();
    A.conn = m.conn.as<int32_t>();
    A.nb = m.nb;
    A.p2map = T.p2map.as<double>();
    A.boxrule = T.boxrule.as<double>();
    A.boxpsi = T.boxpsi[m.order - 1].as<double>();
    A.boxphi = T.boxphi[m.order - 1].as<double>();
    A.boxprod = T.boxprod[m.order - 1].as<double>();
    A.row_ptr = s.row_ptr.as<int64_t>();
    A.col = s.col.as<int32_t>();
    A.tmap = s.tmap.as<int32_t>();
    A.elpos = s.elpos.as<int32_t>();
    A.val = s.val.as<double>();
    A.lam64 = T.lam64.as<double>();
    A.pt32 = T.pt32.as<float>();
    A.pt32_zero = static_cast<int>(T.n_sub * T.nq);
    A.rule = T.rule.as<double>();
    // the kernel indexes the sub-element tables by the closed form of the level offsets
    const int nch = 1 << m.dim;
    for (int q = 1; q <= s.p.lmax; ++q) {
        int64_t pw = 1;
        for (int r = 1; r < q; ++r) pw *= nch;
        if (T.lvl_off[q] != (pw - 1) / (nch - 1)) fail(NLQ_EDEVICE, "sub-element table layout mismatch");
    }
    A.delta = s.p.delta;
    A.eps = s.p.eps;
    A.dme = s.p.delta - s.p.eps;
    A.dpe = s.p.delta + s.p.eps;
    A.dme_sq = sqrt_threshold(A.dme);
    A.dpe_sq = sqrt_threshold(A.dpe);
    A.min_l2 = s.p.min_dist_l2;
    A.dmm = s.dmm.as<double>();
    A.dme2 = A.dme * A.dme * (1.0 - 1e-12);
    A.dpe2 = A.dpe * A.dpe * (1.0 + 1e-12);
    A.C = s.C;
    A.inv_eps = 1.0 / s.p.eps;
    A.inv_delta2 = 1.0 / (s.p.delta * s.p.delta);
    A.f_inv_eps = static_cast<float>(1.0 / s.p.eps);
    A.f_delta_over_eps = static_cast<float>(s.p.delta / s.p.eps);
    A.f_inv_delta2 = static_cast<float>(1.0 / (s.p.delta * s.p.delta));
    A.f_dme2 = static_cast<float>(A.dme * A.dme);
    A.f_dpe2 = static_cast<float>(A.dpe * A.dpe);
    A.lmin = s.p.lmin;
    A.lmax = s.p.lmax;
    A.form = s.p.form;
    // traversal stack: the tuned logical capacity, plus what forced
    // single pops can add beyond it (NCH - 1 per level), plus one pass of
    // parents whose children go straight to the leaf buffer
    const int stack_cap = s.cfg.stack_cap;
    if (stack_cap < kStackCapMin || stack_cap > kStackCapMax) fail(NLQ_EINVAL, "stack capacity out of range");
    A.capl = stack_cap + (1 << m.dim) * (s.p.lmax + 1) + 64;
    // LDS row cache: as long as the longest row, at most 2048 entries per row
    A.rowcap = static_cast<int>(std::min<int64_t>(std::max<int64_t>(s.max_row, 1), 2048));
    A.counters = s.counters.as<AsmCounters>();
    A.split = split_of(s);
    A.pb = s.det_pb;
    A.pb_base = s.det_pb_base;
    return A;
}

// Argument block in device memory: counter | AsmArgs[nsys] | seg_sys | seg_lo | seg_start
struct BlockLayout {
    size_t off_args, off_sys, off_lo, off_start, bytes;
    BlockLayout(int nsys, int nseg)
    {
        auto al = [](size_t x) { return (x + 15) & ~size_t(15); };
        off_args = 16;
        off_sys = al(off_args + sizeof(AsmArgs) * nsys);
        off_lo = al(off_sys + sizeof(int32_t) * nseg);
        off_start = al(off_lo + sizeof(int64_t) * nseg);
        bytes = al(off_start + sizeof(int64_t) * (nseg + 1));
    }
};

}  // namespace

void LaunchBlock::ensure(Ctx *ctx, size_t bytes)
{
    if (bytes <= cap) return;
    if (host) (void)hipHostFree(host);
    host = nullptr;
    cap = 0;
    dev.alloc(ctx, bytes);
    NLQ_HIP(hipHostMalloc(&host, bytes, hipHostMallocDefault));
    cap = bytes;
}

LaunchBlock::~LaunchBlock()
{
    if (host) (void)hipHostFree(host);
}

void launch_integrate_jobs(Ctx *ctx, LaunchBlock &lb, const std::vector<IntegrateJob> &jobs, hipStream_t st,
                           hipEvent_t e0, hipEvent_t e1)
{
    if (jobs.empty()) return;
    if (static_cast<int>(jobs.size()) > kMaxSeg) fail(NLQ_EINVAL, "too many segments in one launch");
    const System &s0 = *jobs[0].s;
    std::vector<const System *> systems;
    std::vector<int32_t> seg_sys;
    std::vector<int64_t> seg_lo, seg_start{0};
    for (const auto &j : jobs) {
        const System &s = *j.s;
        if (s.mesh->dim != s0.mesh->dim || s.p.precision != s0.p.precision || s.p.kernel != s0.p.kernel ||
            s.mesh->order != s0.mesh->order || s.mesh->shape != s0.mesh->shape)
            fail(NLQ_EINVAL, "one launch takes systems of one dimension, element type, precision and kernel");
        if (s.p.deterministic && (!s.det_pb || jobs.size() != 1))
            fail(NLQ_EINVAL, "a deterministic system is integrated by itself (nlq_assemble)");
        if (j.lo < 0 || j.hi > s.mesh->n_elems || j.lo > j.hi) fail(NLQ_EINVAL, "bad outer-element range");
        int k = 0;
        while (k < static_cast<int>(systems.size()) && systems[k] != &s) ++k;
        if (k == static_cast<int>(systems.size())) systems.push_back(&s);
        seg_sys.push_back(k);
        seg_lo.push_back(j.lo);
        seg_start.push_back(seg_start.back() + (j.hi - j.lo) * split_of(s));
    }
    const int64_t items = seg_start.back();
    if (items >= (int64_t(1) << 32) - 1) fail(NLQ_EINVAL, "too many outer elements in one launch");
    const BlockLayout B(static_cast<int>(systems.size()), static_cast<int>(jobs.size()));
    lb.ensure(ctx, B.bytes);
    char *h = static_cast<char *>(lb.host);
    std::memset(h, 0, B.bytes);
    int capl = 1, rowcap = 1, leafcap = kLeafCapMin;
    for (size_t k = 0; k < systems.size(); ++k) {
        const System &s = *systems[k];
        const AsmArgs A = make_args(s, ctx->get_tables(s.mesh->dim, s.p.lmax));
        capl = std::max(capl, A.capl);
        rowcap = std::max(rowcap, A.rowcap);
        leafcap = std::max(leafcap, leaf_cap_of(s));
        std::memcpy(h + B.off_args + k * sizeof(AsmArgs), &A, sizeof(AsmArgs));
    }
    std::memcpy(h + B.off_sys, seg_sys.data(), sizeof(int32_t) * seg_sys.size());
    std::memcpy(h + B.off_lo, seg_lo.data(), sizeof(int64_t) * seg_lo.size());
    std::memcpy(h + B.off_start, seg_start.data(), sizeof(int64_t) * seg_start.size());
    // a system whose first outer element is in this launch starts from zero
    for (const auto &j : jobs) {
        if (j.lo != 0) continue;
        const System &s = *j.s;
        NLQ_HIP(hipMemsetAsync(s.counters.as<void>(), 0, sizeof(AsmCounters), st));
        NLQ_HIP(hipMemsetAsync(s.val.as<void>(), 0, sizeof(double) * s.nnz, st));
        const int64_t nu = static_cast<int64_t>(s.mesh->nb) * (s.mesh->nb + 1) / 2;
        NLQ_HIP(hipMemsetAsync(s.dmm.as<void>(), 0, sizeof(double) * s.mesh->n_elems * nu, st));
    }
    NLQ_HIP(hipMemcpyAsync(lb.dev.as<void>(), h, B.bytes, hipMemcpyHostToDevice, st));
    char *d = lb.dev.as<char>();
    LaunchArgs L{};
    L.sys = reinterpret_cast<const AsmArgs *>(d + B.off_args);
    L.seg_sys = reinterpret_cast<const int32_t *>(d + B.off_sys);
    L.seg_lo = reinterpret_cast<const int64_t *>(d + B.off_lo);
    L.seg_start = reinterpret_cast<const int64_t *>(d + B.off_start);
    L.nseg = static_cast<int>(jobs.size());
    L.capl = capl;
    L.rowcap = rowcap;
    L.leafcap = leafcap;
    L.counter = reinterpret_cast<unsigned int *>(d);
    if (items > 0) dispatch(ctx, s0, s0.cfg, L, items, st, false, e0, e1);
    // systems whose last outer element is in this launch: diagonal blocks and R + R^T
    // (in deterministic mode the fixed-order sums do both)
    for (const auto &j : jobs) {
        const System &s = *j.s;
        if (j.hi != s.mesh->n_elems || s.det_pb) continue;
        const int nb = s.mesh->nb;
        const int four = s.p.form == NLQ_FORM_SYM4;
        const int64_t nf = s.mesh->n_elems * (static_cast<int64_t>(nb) * (nb + 1) / 2);
        const double *dmm = s.dmm.as<double>();
        const int32_t *elpos = s.elpos.as<int32_t>();
        double *val = s.val.as<double>();
        if (nf > 0) {
            const unsigned gf = static_cast<unsigned>((nf + 255) / 256);
            auto kern = nb == 3    ? k_fold_diag<3>
                        : nb == 4  ? k_fold_diag<4>
                        : nb == 6  ? k_fold_diag<6>
                        : nb == 8  ? k_fold_diag<8>
                        : nb == 10 ? k_fold_diag<10> : k_fold_diag<20>;
            hipLaunchKernelGGL(kern, dim3(gf), dim3(256), 0, st, s.mesh->n_elems, dmm, elpos, val, four);
            NLQ_CHECK_LAUNCH();
        }
        if (four && s.nnz > 0) {
            hipLaunchKernelGGL(k_symmetrize, dim3(static_cast<unsigned>((s.nnz + 255) / 256)), dim3(256), 0, st,
                               s.nnz, s.tmap.as<int32_t>(), val);
            NLQ_CHECK_LAUNCH();
        }
    }
}

int64_t integrate_slots(Ctx *ctx, const System &s)
{
    const AsmArgs A = make_args(s, ctx->get_tables(s.mesh->dim, s.p.lmax));
    const bool plain = s.p.precision == NLQ_FP64_PLAIN;
    int per_cu;
    const int ord = s.mesh->order, shp = s.mesh->shape, lc = leaf_cap_of(s);
    if (s.mesh->dim == 2)
        per_cu = plain ? occupancy_of<2, 0>(s.p.kernel, s.cfg.occ, A.capl, A.rowcap, lc, ord, shp)
                       : occupancy_of<2, 1>(s.p.kernel, s.cfg.occ, A.capl, A.rowcap, lc, ord, shp);
    else
        per_cu = plain ? occupancy_of<3, 0>(s.p.kernel, s.cfg.occ, A.capl, A.rowcap, lc, ord, shp)
                       : occupancy_of<3, 1>(s.p.kernel, s.cfg.occ, A.capl, A.rowcap, lc, ord, shp);
    if (s.cfg.wg_per_cu > 0 && s.cfg.wg_per_cu < per_cu) per_cu = s.cfg.wg_per_cu;
    return static_cast<int64_t>(ctx->n_cu) * per_cu;
}

int integrate_split(const System &s) { return split_of(s); }

void launch_symmetrize(const System &s, hipStream_t st)
{
    if (s.nnz <= 0) return;
    hipLaunchKernelGGL(k_symmetrize, dim3(static_cast<unsigned>((s.nnz + 255) / 256)), dim3(256), 0, st, s.nnz,
                       s.tmap.as<int32_t>(), s.val.as<double>());
    NLQ_CHECK_LAUNCH();
}

void launch_integrate(System &s, hipStream_t st, hipEvent_t e0, hipEvent_t e1)
{
    if (s.p.deterministic) integrate_deterministic(s, st, e0, e1);
    else launch_integrate_jobs(s.ctx, s.launch, {IntegrateJob{&s, 0, s.mesh->n_elems}}, st, e0, e1);
}

void launch_pair_blocks(System &s, hipStream_t st, int64_t n, const int32_t *ex_l, const int32_t *ex_m,
                        double *ex_out)
{
    AsmArgs A = make_args(s, s.ctx->get_tables(s.mesh->dim, s.p.lmax));
    A.n_explicit = n;
    A.ex_l = ex_l;
    A.ex_m = ex_m;
    A.ex_out = ex_out;
    const BlockLayout B(1, 1);
    s.launch.ensure(s.ctx, B.bytes);
    char *h = static_cast<char *>(s.launch.host);
    std::memset(h, 0, B.bytes);
    std::memcpy(h + B.off_args, &A, sizeof(AsmArgs));
    NLQ_HIP(hipMemcpyAsync(s.launch.dev.as<void>(), h, B.bytes, hipMemcpyHostToDevice, st));
    char *d = s.launch.dev.as<char>();
    LaunchArgs L{};
    L.sys = reinterpret_cast<const AsmArgs *>(d + B.off_args);
    L.nseg = 1;
    L.capl = A.capl;
    L.rowcap = A.rowcap;
    L.leafcap = leaf_cap_of(s);
    L.counter = reinterpret_cast<unsigned int *>(d);
    if (n > 0) dispatch(s.ctx, s, TuneConfig{}, L, n, st, true, nullptr, nullptr);
}

}  // namespace nlq
