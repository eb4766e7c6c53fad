// Setup kernels of the assembly: element tables, the pair list J_l and the
// structural CSR pattern, plus a device exclusive scan and the box-mesh builder.
#include <algorithm>
#include <climits>
#include <cmath>

#include "nlq_device.hpp"
#include "nlq_box.hpp"
#include "nlq_internal.hpp"

namespace nlq {

// ---------------------------------------------------------------- scan

namespace {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 4;
constexpr int kScanTile = kScanThreads * kScanItems;

__global__ void __launch_bounds__(kScanThreads)
k_scan_tiles(const int64_t *in, int64_t *out, int64_t *tile_sums, int64_t n)
{
    __shared__ int64_t warp_tot[kScanThreads / kWave];
    const int64_t base = static_cast<int64_t>(blockIdx.x) * kScanTile;
    int64_t v[kScanItems];
    int64_t acc = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        int64_t idx = base + threadIdx.x * kScanItems + i;
        v[i] = idx < n ? in[idx] : 0;
        acc += v[i];
    }
    int64_t incl = wave_incl_scan(acc);
    const int w = threadIdx.x / kWave;
    if (lane_id() == kWave - 1) warp_tot[w] = incl;
    __syncthreads();
    int64_t wave_off = 0;
    for (int j = 0; j < w; ++j) wave_off += warp_tot[j];
    int64_t run = wave_off + incl - acc;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        int64_t idx = base + threadIdx.x * kScanItems + i;
        if (idx < n) out[idx] = run;
        run += v[i];
    }
    if (threadIdx.x == kScanThreads - 1) tile_sums[blockIdx.x] = wave_off + incl;
}

__global__ void k_add_tile_offsets(int64_t *out, const int64_t *tile_off, int64_t n)
{
    int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx < n) out[idx] += tile_off[idx / kScanTile];
}

}  // namespace

// out[i] = sum_{j<i} in[j] for i < n (in and out may alias only if equal).
void exclusive_scan_i64(Ctx *ctx, const int64_t *in, int64_t *out, int64_t n, hipStream_t st)
{
    if (n <= 0) return;
    const int64_t tiles = (n + kScanTile - 1) / kScanTile;
    DevBuf sums(ctx, sizeof(int64_t) * tiles, st);
    hipLaunchKernelGGL(k_scan_tiles, dim3(tiles), dim3(kScanThreads), 0, st, in, out,
                       sums.as<int64_t>(), n);
    NLQ_CHECK_LAUNCH();
    if (tiles > 1) {
        DevBuf offs(ctx, sizeof(int64_t) * tiles, st);
        exclusive_scan_i64(ctx, sums.as<int64_t>(), offs.as<int64_t>(), tiles, st);
        hipLaunchKernelGGL(k_add_tile_offsets, dim3((n + 255) / 256), dim3(256), 0, st, out,
                           offs.as<int64_t>(), n);
        NLQ_CHECK_LAUNCH();
        NLQ_HIP(hipStreamSynchronize(st));  // keep the temporaries alive until done
    } else {
        NLQ_HIP(hipStreamSynchronize(st));
    }
}

// ---------------------------------------------------------------- element tables

namespace {

template <int DIM>
__global__ void k_elem_tables(int64_t ne, int nb, const double *__restrict__ coords,
                              const int32_t *__restrict__ conn, double *__restrict__ vert,
                              double *__restrict__ lo, double *__restrict__ hi,
                              double *__restrict__ meas)
{
    constexpr int NV = DIM + 1;
    const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= ne) return;
    double V[NV][DIM];
    // the vertices are the first NV of the element's nb nodes (P1 or P2)
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        const int64_t node = conn[e * nb + v];
#pragma unroll
        for (int k = 0; k < DIM; ++k) {
            V[v][k] = coords[node * DIM + k];
            vert[(v * DIM + k) * ne + e] = V[v][k];
        }
    }
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
        double a = V[0][k], b = V[0][k];
#pragma unroll
        for (int v = 1; v < NV; ++v) {
            a = fmin(a, V[v][k]);
            b = fmax(b, V[v][k]);
        }
        lo[k * ne + e] = a;
        hi[k * ne + e] = b;
    }
    double det;
    if (DIM == 2) {
        det = (V[1][0] - V[0][0]) * (V[2][1] - V[0][1]) - (V[1][1] - V[0][1]) * (V[2][0] - V[0][0]);
        meas[e] = fabs(det) * 0.5;
    } else {
        double a[3], b[3], c[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            a[k] = V[1][k] - V[0][k];
            b[k] = V[2][k] - V[0][k];
            c[k] = V[3 % NV][k % DIM] - V[0][k % DIM];
        }
        det = a[0] * (b[1] * c[2] - b[2] * c[1]) - a[1] * (b[0] * c[2] - b[2] * c[0]) +
              a[2] * (b[0] * c[1] - b[1] * c[0]);
        meas[e] = fabs(det) / 6.0;
    }
}

// Box of each element's quadrature points y_b = sum_v bary_bv V_v, formed as
// the oracle and the integration's inner points form them in FP64: products
// rounded, then added in vertex order (no fused multiply-add), so that the box
// holds every such point exactly.  Used by the zero test of the children at
// L_max and by the refine test of min_dist_l2 = 2.
template <int DIM>
__global__ void k_quad_boxes(int64_t ne, int nq, const double *__restrict__ vert,
                             const double *__restrict__ bary, double *__restrict__ qlo,
                             double *__restrict__ qhi)
{
#pragma clang fp contract(off)
    constexpr int NV = DIM + 1;
    const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= ne) return;
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
        double a = 0.0, b = 0.0;
        for (int q = 0; q < nq; ++q) {
            double y = 0.0;
#pragma unroll
            for (int v = 0; v < NV; ++v) y = y + bary[q * NV + v] * vert[(v * DIM + k) * ne + e];
            a = q == 0 ? y : fmin(a, y);
            b = q == 0 ? y : fmax(b, y);
        }
        qlo[k * ne + e] = a;
        qhi[k * ne + e] = b;
    }
}

// Quadrilaterals / hexahedra: the 2^DIM corners (SoA), their box (a multilinear
// map takes its extremes at the corners) and the measure, the integral of
// |det F'| by the 3^DIM Gauss rule (exact: degree <= DIM - 1 per variable).
template <int DIM>
__global__ void k_elem_tables_box(int64_t ne, int nb, const double *__restrict__ coords,
                                  const int32_t *__restrict__ conn, double *__restrict__ vert,
                                  double *__restrict__ lo, double *__restrict__ hi, double *__restrict__ meas)
{
    constexpr int NC = 1 << DIM;
    const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= ne) return;
    BoxVerts<DIM> P;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        const int64_t node = conn[e * nb + c];
#pragma unroll
        for (int k = 0; k < DIM; ++k) {
            P.v[c][k] = coords[node * DIM + k];
            vert[(c * DIM + k) * ne + e] = P.v[c][k];
        }
    }
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
        double a = P.v[0][k], b = P.v[0][k];
#pragma unroll
        for (int c = 1; c < NC; ++c) {
            a = fmin(a, P.v[c][k]);
            b = fmax(b, P.v[c][k]);
        }
        lo[k * ne + e] = a;
        hi[k * ne + e] = b;
    }
    double m = 0.0;
    for (int q = 0; q < box_nq(DIM); ++q) {
        const int i[3] = {q % 3, (q / 3) % 3, q / 9};
        double xi[DIM], w = 1.0;
#pragma unroll
        for (int k = 0; k < DIM; ++k) {
            xi[k] = box_gauss_node(i[k]);
            w *= box_gauss_weight(i[k]);
        }
        m = fma(w, box_jacdet<DIM>(P, xi), m);
    }
    meas[e] = m;
}

// Box of each box element's quadrature points y_b = F(g_b), formed as the
// oracle forms them: the multilinear weights rounded as written, then the
// products N_c P_c rounded and added in corner order (no fused multiply-add).
template <int DIM>
__global__ void k_quad_boxes_box(int64_t ne, const double *__restrict__ vert, double *__restrict__ qlo,
                                 double *__restrict__ qhi)
{
    constexpr int NC = 1 << DIM;
    const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= ne) return;
    double a[DIM], b[DIM];
    for (int q = 0; q < box_nq(DIM); ++q) {
        const int i[3] = {q % 3, (q / 3) % 3, q / 9};
        double xi[DIM], N[NC];
#pragma unroll
        for (int k = 0; k < DIM; ++k) xi[k] = box_gauss_node(i[k]);
        box_corner_weights<DIM>(xi, N);
#pragma unroll
        for (int k = 0; k < DIM; ++k) {
            double y = 0.0;
#pragma unroll
            for (int c = 0; c < NC; ++c) y = __dadd_rn(y, __dmul_rn(N[c], vert[(c * DIM + k) * ne + e]));
            a[k] = q == 0 ? y : fmin(a[k], y);
            b[k] = q == 0 ? y : fmax(b[k], y);
        }
    }
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
        qlo[k * ne + e] = a[k];
        qhi[k * ne + e] = b[k];
    }
}

}  // namespace

void launch_elem_tables(System &s, hipStream_t st)
{
    const Mesh &m = *s.mesh;
    const int64_t ne = m.n_elems;
    const int nv = m.ngeo;
    s.vert.alloc(s.ctx, sizeof(double) * ne * nv * m.dim);
    s.lo.alloc(s.ctx, sizeof(double) * ne * m.dim);
    s.hi.alloc(s.ctx, sizeof(double) * ne * m.dim);
    s.meas.alloc(s.ctx, sizeof(double) * ne);
    s.qlo.alloc(s.ctx, sizeof(double) * ne * m.dim);
    s.qhi.alloc(s.ctx, sizeof(double) * ne * m.dim);
    dim3 grid((ne + 255) / 256), block(256);
    if (m.shape == 1) {
        auto kt = m.dim == 2 ? k_elem_tables_box<2> : k_elem_tables_box<3>;
        hipLaunchKernelGGL(kt, grid, block, 0, st, ne, m.nb, m.coords.as<double>(), m.conn.as<int32_t>(),
                           s.vert.as<double>(), s.lo.as<double>(), s.hi.as<double>(), s.meas.as<double>());
        NLQ_CHECK_LAUNCH();
        auto kq = m.dim == 2 ? k_quad_boxes_box<2> : k_quad_boxes_box<3>;
        hipLaunchKernelGGL(kq, grid, block, 0, st, ne, s.vert.as<double>(), s.qlo.as<double>(), s.qhi.as<double>());
        NLQ_CHECK_LAUNCH();
        return;
    }
    if (m.dim == 2)
        hipLaunchKernelGGL(k_elem_tables<2>, grid, block, 0, st, ne, m.nb, m.coords.as<double>(),
                           m.conn.as<int32_t>(), s.vert.as<double>(), s.lo.as<double>(),
                           s.hi.as<double>(), s.meas.as<double>());
    else
        hipLaunchKernelGGL(k_elem_tables<3>, grid, block, 0, st, ne, m.nb, m.coords.as<double>(),
                           m.conn.as<int32_t>(), s.vert.as<double>(), s.lo.as<double>(),
                           s.hi.as<double>(), s.meas.as<double>());
    NLQ_CHECK_LAUNCH();
    {
        const Tables &T = s.ctx->get_tables(m.dim, s.p.lmax);
        if (m.dim == 2)
            hipLaunchKernelGGL(k_quad_boxes<2>, grid, block, 0, st, ne, T.nq, s.vert.as<double>(),
                               T.rule.as<double>(), s.qlo.as<double>(), s.qhi.as<double>());
        else
            hipLaunchKernelGGL(k_quad_boxes<3>, grid, block, 0, st, ne, T.nq, s.vert.as<double>(),
                               T.rule.as<double>(), s.qlo.as<double>(), s.qhi.as<double>());
        NLQ_CHECK_LAUNCH();
    }
}

// ---------------------------------------------------------------- pair list

namespace {

struct BinGrid {
    double gmin[3];
    double size[3];
    int nb[3];
};

template <int DIM>
__device__ __forceinline__ int bin_coord(const BinGrid &g, int k, double x)
{
    double t = floor((x - g.gmin[k]) / g.size[k]);
    int b = t < 0.0 ? 0 : (t > g.nb[k] - 1 ? g.nb[k] - 1 : static_cast<int>(t));
    return b;
}

template <int DIM>
__global__ void k_bin_count(int64_t ne, const double *__restrict__ lo, BinGrid g,
                            int64_t *__restrict__ bin_cnt, int32_t *__restrict__ bin_of)
{
    const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= ne) return;
    int64_t b = 0, mul = 1;
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
        b += mul * bin_coord<DIM>(g, k, lo[k * ne + e]);
        mul *= g.nb[k];
    }
    bin_of[e] = static_cast<int32_t>(b);
    atomicAdd(reinterpret_cast<unsigned long long *>(&bin_cnt[b]), 1ull);
}

__global__ void k_bin_fill(int64_t ne, const int32_t *__restrict__ bin_of,
                           const int64_t *__restrict__ bin_off, int64_t *__restrict__ cursor,
                           int32_t *__restrict__ items)
{
    const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= ne) return;
    const int b = bin_of[e];
    const int64_t at = atomicAdd(reinterpret_cast<unsigned long long *>(&cursor[b]), 1ull);
    items[bin_off[b] + at] = static_cast<int32_t>(e);
}

constexpr int kPairCap = 8192;  // largest |J_l| handled (per-wave LDS list)

// bitonic sort of buf[0..n2) (n2 a power of two) by one wave
__device__ void wave_bitonic_sort(int32_t *buf, int n2)
{
    for (int k = 2; k <= n2; k <<= 1)
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = lane_id(); i < n2; i += kWave) {
                const int ixj = i ^ j;
                if (ixj > i) {
                    int32_t a = buf[i], b = buf[ixj];
                    const bool up = (i & k) == 0;
                    if ((a > b) == up) {
                        buf[i] = b;
                        buf[ixj] = a;
                    }
                }
            }
            __syncthreads();
        }
}

// One single-wave workgroup per outer element l.  J_l = {m : aprx min dist
// (bbox_l, bbox_m) < delta + eps} (Section 5, eq. (k_l) with eq. (mindist)),
// candidates from the uniform bins whose lower-corner range can hold such m.
// count mode (m_out == nullptr): counts[l] = |J_l|, err[0] = 1 when a list
// exceeds kPairCap (the longest list comes from k_count_max); fill mode: J_l ascending, sorted in a dynamic
// LDS list of `cap` entries (a power of two >= max |J_l|), so that the count
// pass needs no LDS and the fill pass only what the longest list needs (LDS
// bounds how many of these one-wave workgroups a CU holds).
template <int DIM>
__global__ void __launch_bounds__(kWave)
k_pairs(int64_t ne, const double *__restrict__ lo, const double *__restrict__ hi, BinGrid g,
        double thr, double reach_lo0, double reach_lo1, double reach_lo2,
        const int64_t *__restrict__ bin_off, const int32_t *__restrict__ items,
        int64_t *__restrict__ counts, const int64_t *__restrict__ offsets,
        int32_t *__restrict__ m_out, int cap, int *__restrict__ err)
{
    extern __shared__ int32_t buf[];
    const int64_t l = blockIdx.x;
    if (l >= ne) return;
    double llo[DIM], lhi[DIM];
    const double reach[3] = {reach_lo0, reach_lo1, reach_lo2};
    int b0[3] = {0, 0, 0}, b1[3] = {0, 0, 0};
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
        llo[k] = lo[k * ne + l];
        lhi[k] = hi[k * ne + l];
        b0[k] = bin_coord<DIM>(g, k, llo[k] - thr - reach[k]);
        b1[k] = bin_coord<DIM>(g, k, lhi[k] + thr);
    }
    int count = 0;
    // the bins x = b0..b1 of one row (y, z) are consecutive in the bin order, so
    // their items form one range: the wave walks it 64 items at a time
    for (int z = b0[2]; z <= b1[2]; ++z)
        for (int y = b0[1]; y <= b1[1]; ++y) {
            const int64_t row = static_cast<int64_t>(g.nb[0]) * (y + static_cast<int64_t>(g.nb[1]) * z);
            const int64_t s0 = bin_off[row + b0[0]], s1 = bin_off[row + b1[0] + 1];
            for (int64_t i = s0; i < s1; i += kWave) {
                const int64_t it = i + lane_id();
                bool take = false;
                int32_t mm = 0;
                if (it < s1) {
                    mm = items[it];
                    double mlo[DIM], mhi[DIM];
#pragma unroll
                    for (int k = 0; k < DIM; ++k) {
                        mlo[k] = lo[k * ne + mm];
                        mhi[k] = hi[k * ne + mm];
                    }
                    take = aprx_min_dist<DIM>(llo, lhi, mlo, mhi) < thr;
                }
                const unsigned long long mask = wave_ballot(take);
                if (m_out && take) {
                    const int at = count + lanes_below(mask);
                    if (at < cap) buf[at] = mm;
                }
                count += __popcll(mask);
            }
        }
    if (!m_out) {
        if (lane_id() == 0) {
            counts[l] = count;
            if (count > kPairCap) atomicOr(err, 1);
        }
        return;
    }
    if (count > cap) return;
    int n2 = 1;
    while (n2 < count) n2 <<= 1;
    for (int i = count + lane_id(); i < n2; i += kWave) buf[i] = INT_MAX;
    __syncthreads();
    wave_bitonic_sort(buf, n2);
    const int64_t base = offsets[l];
    for (int i = lane_id(); i < count; i += kWave) m_out[base + i] = buf[i];
}

// err[1] = max counts[0..n) by one block, without atomics (a same-address atomic
// from every workgroup of the count pass serialised it: 50 ms for 83k tets)
__global__ void __launch_bounds__(1024) k_count_max(int64_t n, const int64_t *__restrict__ counts, int *err)
{
    __shared__ int64_t red[1024 / kWave];
    int64_t v = 0;
    for (int64_t i = threadIdx.x; i < n; i += 1024) v = counts[i] > v ? counts[i] : v;
    v = wave_max(v);
    if (lane_id() == 0) red[threadIdx.x / kWave] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t m = 0;
        for (int r = 0; r < 1024 / kWave; ++r) m = red[r] > m ? red[r] : m;
        err[1] = static_cast<int>(m < INT_MAX ? m : INT_MAX);
    }
}

}  // namespace

void build_pairs(System &s, hipStream_t st)
{
    const Mesh &m = *s.mesh;
    const int dim = m.dim;
    const int64_t ne = m.n_elems;
    const double thr = s.p.delta + s.p.eps;
    BinGrid g{};
    int64_t nbins = 1;
    for (int k = 0; k < 3; ++k) {
        g.gmin[k] = 0.0;
        g.size[k] = 1.0;
        g.nb[k] = 1;
    }
    // bins of ~2 (3D) / ~4 (2D) element extents, at least a quarter of the horizon
    const double mult = (dim == 2) ? 4.0 : 2.0;
    for (int k = 0; k < dim; ++k) {
        double ext = std::max(m.ext_max[k], 1e-300);
        double size = std::max(mult * ext, 0.25 * thr);
        double span = m.gmax[k] - m.gmin[k];
        int nb = static_cast<int>(std::min(std::ceil(span / size) + 1.0, 4096.0));
        if (nb < 1) nb = 1;
        g.gmin[k] = m.gmin[k];
        g.size[k] = size;
        g.nb[k] = nb;
        nbins *= nb;
    }
    DevBuf bin_cnt(s.ctx, sizeof(int64_t) * (nbins + 1), st);
    DevBuf bin_off(s.ctx, sizeof(int64_t) * (nbins + 1), st);
    DevBuf cursor(s.ctx, sizeof(int64_t) * (nbins + 1), st);
    DevBuf bin_of(s.ctx, sizeof(int32_t) * ne, st);
    DevBuf items(s.ctx, sizeof(int32_t) * ne, st);
    DevBuf err(s.ctx, 2 * sizeof(int), st);
    NLQ_HIP(hipMemsetAsync(bin_cnt.as<void>(), 0, sizeof(int64_t) * (nbins + 1), st));
    NLQ_HIP(hipMemsetAsync(cursor.as<void>(), 0, sizeof(int64_t) * (nbins + 1), st));
    NLQ_HIP(hipMemsetAsync(err.as<void>(), 0, 2 * sizeof(int), st));
    dim3 g1((ne + 255) / 256), b1(256);
    if (dim == 2)
        hipLaunchKernelGGL(k_bin_count<2>, g1, b1, 0, st, ne, s.lo.as<double>(), g,
                           bin_cnt.as<int64_t>(), bin_of.as<int32_t>());
    else
        hipLaunchKernelGGL(k_bin_count<3>, g1, b1, 0, st, ne, s.lo.as<double>(), g,
                           bin_cnt.as<int64_t>(), bin_of.as<int32_t>());
    NLQ_CHECK_LAUNCH();
    exclusive_scan_i64(s.ctx, bin_cnt.as<int64_t>(), bin_off.as<int64_t>(), nbins + 1, st);
    hipLaunchKernelGGL(k_bin_fill, g1, b1, 0, st, ne, bin_of.as<int32_t>(),
                       bin_off.as<int64_t>(), cursor.as<int64_t>(), items.as<int32_t>());
    NLQ_CHECK_LAUNCH();

    DevBuf counts(s.ctx, sizeof(int64_t) * (ne + 1), st);
    NLQ_HIP(hipMemsetAsync(counts.as<void>(), 0, sizeof(int64_t) * (ne + 1), st));
    s.pair_off.alloc(s.ctx, sizeof(int64_t) * (ne + 1));
    const double r0 = m.ext_max[0], r1 = dim > 1 ? m.ext_max[1] : 0.0, r2 = dim > 2 ? m.ext_max[2] : 0.0;
    auto launch = [&](int32_t *m_out, int cap) {
        const size_t lds = m_out ? sizeof(int32_t) * static_cast<size_t>(cap) : 0;
        if (dim == 2)
            hipLaunchKernelGGL(k_pairs<2>, dim3(ne), dim3(kWave), lds, st, ne, s.lo.as<double>(),
                               s.hi.as<double>(), g, thr, r0, r1, r2, bin_off.as<int64_t>(),
                               items.as<int32_t>(), counts.as<int64_t>(),
                               s.pair_off.as<int64_t>(), m_out, cap, err.as<int>());
        else
            hipLaunchKernelGGL(k_pairs<3>, dim3(ne), dim3(kWave), lds, st, ne, s.lo.as<double>(),
                               s.hi.as<double>(), g, thr, r0, r1, r2, bin_off.as<int64_t>(),
                               items.as<int32_t>(), counts.as<int64_t>(),
                               s.pair_off.as<int64_t>(), m_out, cap, err.as<int>());
        NLQ_CHECK_LAUNCH();
    };
    launch(nullptr, 0);
    hipLaunchKernelGGL(k_count_max, dim3(1), dim3(1024), 0, st, ne, counts.as<int64_t>(), err.as<int>());
    NLQ_CHECK_LAUNCH();
    int herr[2] = {0, 0};
    NLQ_HIP(hipMemcpyAsync(herr, err.as<void>(), 2 * sizeof(int), hipMemcpyDeviceToHost, st));
    exclusive_scan_i64(s.ctx, counts.as<int64_t>(), s.pair_off.as<int64_t>(), ne + 1, st);
    NLQ_HIP(hipMemcpyAsync(&s.n_pairs, s.pair_off.as<int64_t>() + ne, sizeof(int64_t),
                           hipMemcpyDeviceToHost, st));
    NLQ_HIP(hipStreamSynchronize(st));
    if (herr[0]) fail(NLQ_EINVAL, "an element has more than 8192 neighbours within delta+eps");
    s.max_pairs = herr[1];
    s.pair_m.alloc(s.ctx, sizeof(int32_t) * std::max<int64_t>(s.n_pairs, 1));
    int cap = kWave;
    while (cap < s.max_pairs) cap <<= 1;
    launch(s.pair_m.as<int32_t>(), cap);
    NLQ_HIP(hipStreamSynchronize(st));
}

// ---------------------------------------------------------------- pattern

namespace {

constexpr int kBitmapWords = 4096;            // 131072 node ids per neighbourhood window

__global__ void k_node_elem_count(int64_t ne, int nv, const int32_t *__restrict__ conn,
                                  int64_t *__restrict__ cnt)
{
    const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= ne * nv) return;
    atomicAdd(reinterpret_cast<unsigned long long *>(&cnt[conn[t]]), 1ull);
}

__global__ void k_node_elem_fill(int64_t ne, int nv, const int32_t *__restrict__ conn,
                                 const int64_t *__restrict__ off, int64_t *__restrict__ cursor,
                                 int32_t *__restrict__ items)
{
    const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= ne * nv) return;
    const int32_t node = conn[t];
    const int64_t at = atomicAdd(reinterpret_cast<unsigned long long *>(&cursor[node]), 1ull);
    items[off[node] + at] = static_cast<int32_t>(t / nv);
}

// Set-union of node ids by one single-wave workgroup through an LDS bitmap over
// [lo_id, lo_id + 32*kBitmapWords).  Emits the sorted union (or its size).
struct BitmapUnion {
    unsigned int *words;
    int nwords;
    int32_t base;
    __device__ void clear()
    {
        for (int i = lane_id(); i < nwords; i += kWave) words[i] = 0u;
        __syncthreads();
    }
    __device__ void insert(int32_t id)
    {
        const int32_t r = id - base;
        atomicOr(&words[r >> 5], 1u << (r & 31));
    }
    // total count; if out != nullptr also writes the sorted ids
    __device__ int64_t emit(int32_t *out)
    {
        __syncthreads();
        int64_t run = 0;
        for (int w0 = 0; w0 < nwords; w0 += kWave) {
            const int w = w0 + lane_id();
            const unsigned int bits = w < nwords ? words[w] : 0u;
            const int c = __popc(bits);
            const int incl = wave_incl_scan(c);
            if (out) {
                int64_t at = run + incl - c;
                unsigned int b = bits;
                while (b) {
                    const int bit = __ffs(b) - 1;
                    out[at++] = base + (w << 5) + bit;
                    b &= b - 1;
                }
            }
            run += __shfl(incl, kWave - 1, kWave);
        }
        return run;
    }
};

// N(e) = sorted union of the nodes of every m in J_e.
template <int NV>
__global__ void __launch_bounds__(kWave)
k_elem_nbhd(int64_t ne, const int32_t *__restrict__ conn, const int64_t *__restrict__ pair_off,
            const int32_t *__restrict__ pair_m, int64_t *__restrict__ counts,
            const int64_t *__restrict__ offsets, int32_t *__restrict__ out, int *__restrict__ err)
{
    __shared__ unsigned int words[kBitmapWords];
    const int64_t e = blockIdx.x;
    if (e >= ne) return;
    const int64_t p0 = pair_off[e], p1 = pair_off[e + 1];
    int32_t mn = INT_MAX, mx = INT_MIN;
    for (int64_t p = p0 + lane_id(); p < p1; p += kWave) {
        const int32_t mm = pair_m[p];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const int32_t id = conn[static_cast<int64_t>(mm) * NV + v];
            mn = min(mn, id);
            mx = max(mx, id);
        }
    }
    mn = wave_min(mn);
    mx = wave_max(mx);
    const int64_t range = static_cast<int64_t>(mx) - mn + 1;
    if (range > 32ll * kBitmapWords) {
        if (lane_id() == 0) atomicOr(err, 2);
        return;
    }
    BitmapUnion u{words, static_cast<int>((range + 31) / 32), mn};
    u.clear();
    for (int64_t p = p0 + lane_id(); p < p1; p += kWave) {
        const int32_t mm = pair_m[p];
#pragma unroll
        for (int v = 0; v < NV; ++v) u.insert(conn[static_cast<int64_t>(mm) * NV + v]);
    }
    const int64_t c = u.emit(out ? out + offsets[e] : nullptr);
    if (!out && lane_id() == 0) counts[e] = c;
}

// row(i) = union over elements e containing i of N(e): every node j with i, j in
// nodes(l) u nodes(m) for some pair (l, m) (the pair list is symmetric and holds
// (e, e), so pairs with i in the inner element are covered too).
__global__ void __launch_bounds__(kWave)
k_rows(int64_t n_nodes, const int64_t *__restrict__ ne_off, const int32_t *__restrict__ ne_items,
       const int64_t *__restrict__ nb_off, const int32_t *__restrict__ nb,
       int64_t *__restrict__ counts, const int64_t *__restrict__ row_ptr,
       int32_t *__restrict__ col, int *__restrict__ err)
{
    __shared__ unsigned int words[kBitmapWords];
    const int64_t i = blockIdx.x;
    if (i >= n_nodes) return;
    const int64_t a0 = ne_off[i], a1 = ne_off[i + 1];
    int32_t mn = INT_MAX, mx = INT_MIN;
    for (int64_t a = a0; a < a1; ++a) {
        const int32_t e = ne_items[a];
        const int64_t q0 = nb_off[e], q1 = nb_off[e + 1];
        if (q1 > q0) {
            mn = min(mn, nb[q0]);
            mx = max(mx, nb[q1 - 1]);
        }
    }
    if (a1 == a0) {
        if (!col && lane_id() == 0) counts[i] = 0;
        return;
    }
    const int64_t range = static_cast<int64_t>(mx) - mn + 1;
    if (range > 32ll * kBitmapWords) {
        if (lane_id() == 0) atomicOr(err, 4);
        return;
    }
    BitmapUnion u{words, static_cast<int>((range + 31) / 32), mn};
    u.clear();
    for (int64_t a = a0; a < a1; ++a) {
        const int32_t e = ne_items[a];
        for (int64_t q = nb_off[e] + lane_id(); q < nb_off[e + 1]; q += kWave) u.insert(nb[q]);
    }
    const int64_t c = u.emit(col ? col + row_ptr[i] : nullptr);
    if (!col && lane_id() == 0) counts[i] = c;
}

__device__ __forceinline__ int64_t find_in_row(const int64_t *row_ptr, const int32_t *col,
                                               int64_t r, int32_t c)
{
    int64_t a = row_ptr[r], b = row_ptr[r + 1] - 1;
    while (a <= b) {
        const int64_t mid = (a + b) >> 1;
        const int32_t v = col[mid];
        if (v == c) return mid;
        if (v < c) a = mid + 1; else b = mid - 1;
    }
    return -1;
}

// tmap[k] = position of (j, i) for the entry k = (i, j)
__global__ void __launch_bounds__(kWave)
k_transpose_map(int64_t n, const int64_t *__restrict__ row_ptr, const int32_t *__restrict__ col,
                int32_t *__restrict__ tmap, int *__restrict__ err)
{
    const int64_t i = blockIdx.x;
    if (i >= n) return;
    for (int64_t k = row_ptr[i] + lane_id(); k < row_ptr[i + 1]; k += kWave) {
        const int64_t t = find_in_row(row_ptr, col, col[k], static_cast<int32_t>(i));
        if (t < 0) atomicOr(err, 8);
        tmap[k] = static_cast<int32_t>(t);
    }
}

template <int NV>
__global__ void k_elem_block_pos(int64_t ne, const int32_t *__restrict__ conn,
                                 const int64_t *__restrict__ row_ptr, const int32_t *__restrict__ col,
                                 int32_t *__restrict__ elpos, int *__restrict__ err)
{
    const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= ne * NV * NV) return;
    const int64_t e = t / (NV * NV);
    const int a = static_cast<int>((t / NV) % NV), b = static_cast<int>(t % NV);
    const int64_t pos = find_in_row(row_ptr, col, conn[e * NV + a], conn[e * NV + b]);
    if (pos < 0) atomicOr(err, 16);
    elpos[t] = static_cast<int32_t>(pos);
}

}  // namespace

void build_pattern(System &s, hipStream_t st)
{
    const Mesh &m = *s.mesh;
    const int nv = m.nb;   // nodes per element (P1 or P2)
    const int64_t ne = m.n_elems, nn = m.n_nodes;
    DevBuf err(s.ctx, sizeof(int), st);
    NLQ_HIP(hipMemsetAsync(err.as<void>(), 0, sizeof(int), st));
    // node -> elements
    DevBuf ne_cnt(s.ctx, sizeof(int64_t) * (nn + 1), st);
    DevBuf ne_off(s.ctx, sizeof(int64_t) * (nn + 1), st);
    DevBuf ne_cur(s.ctx, sizeof(int64_t) * (nn + 1), st);
    DevBuf ne_items(s.ctx, sizeof(int32_t) * ne * nv, st);
    NLQ_HIP(hipMemsetAsync(ne_cnt.as<void>(), 0, sizeof(int64_t) * (nn + 1), st));
    NLQ_HIP(hipMemsetAsync(ne_cur.as<void>(), 0, sizeof(int64_t) * (nn + 1), st));
    dim3 g1((ne * nv + 255) / 256), b1(256);
    hipLaunchKernelGGL(k_node_elem_count, g1, b1, 0, st, ne, nv, m.conn.as<int32_t>(),
                       ne_cnt.as<int64_t>());
    NLQ_CHECK_LAUNCH();
    exclusive_scan_i64(s.ctx, ne_cnt.as<int64_t>(), ne_off.as<int64_t>(), nn + 1, st);
    hipLaunchKernelGGL(k_node_elem_fill, g1, b1, 0, st, ne, nv, m.conn.as<int32_t>(),
                       ne_off.as<int64_t>(), ne_cur.as<int64_t>(), ne_items.as<int32_t>());
    NLQ_CHECK_LAUNCH();
    // element neighbourhoods
    DevBuf nb_cnt(s.ctx, sizeof(int64_t) * (ne + 1), st);
    DevBuf nb_off(s.ctx, sizeof(int64_t) * (ne + 1), st);
    NLQ_HIP(hipMemsetAsync(nb_cnt.as<void>(), 0, sizeof(int64_t) * (ne + 1), st));
    auto nbhd = [&](int32_t *out) {
        auto kern = nv == 3 ? k_elem_nbhd<3>
                  : nv == 4 ? k_elem_nbhd<4>
                  : nv == 6 ? k_elem_nbhd<6>
                  : nv == 8 ? k_elem_nbhd<8>
                  : nv == 10 ? k_elem_nbhd<10> : k_elem_nbhd<20>;
        hipLaunchKernelGGL(kern, dim3(ne), dim3(kWave), 0, st, ne, m.conn.as<int32_t>(), s.pair_off.as<int64_t>(),
                           s.pair_m.as<int32_t>(), nb_cnt.as<int64_t>(), nb_off.as<int64_t>(), out, err.as<int>());
        NLQ_CHECK_LAUNCH();
    };
    nbhd(nullptr);
    exclusive_scan_i64(s.ctx, nb_cnt.as<int64_t>(), nb_off.as<int64_t>(), ne + 1, st);
    int64_t nb_total = 0;
    NLQ_HIP(hipMemcpyAsync(&nb_total, nb_off.as<int64_t>() + ne, sizeof(int64_t),
                           hipMemcpyDeviceToHost, st));
    NLQ_HIP(hipStreamSynchronize(st));
    DevBuf nb(s.ctx, sizeof(int32_t) * std::max<int64_t>(nb_total, 1), st);
    nbhd(nb.as<int32_t>());
    // rows
    DevBuf row_cnt(s.ctx, sizeof(int64_t) * (nn + 1), st);
    NLQ_HIP(hipMemsetAsync(row_cnt.as<void>(), 0, sizeof(int64_t) * (nn + 1), st));
    s.row_ptr.alloc(s.ctx, sizeof(int64_t) * (nn + 1));
    hipLaunchKernelGGL(k_rows, dim3(nn), dim3(kWave), 0, st, nn, ne_off.as<int64_t>(),
                       ne_items.as<int32_t>(), nb_off.as<int64_t>(), nb.as<int32_t>(),
                       row_cnt.as<int64_t>(), s.row_ptr.as<int64_t>(), nullptr, err.as<int>());
    NLQ_CHECK_LAUNCH();
    exclusive_scan_i64(s.ctx, row_cnt.as<int64_t>(), s.row_ptr.as<int64_t>(), nn + 1, st);
    NLQ_HIP(hipMemcpyAsync(&s.nnz, s.row_ptr.as<int64_t>() + nn, sizeof(int64_t),
                           hipMemcpyDeviceToHost, st));
    {
        std::vector<int64_t> cnt(nn);
        NLQ_HIP(hipMemcpyAsync(cnt.data(), row_cnt.as<void>(), sizeof(int64_t) * nn,
                               hipMemcpyDeviceToHost, st));
        NLQ_HIP(hipStreamSynchronize(st));
        s.max_row = nn > 0 ? *std::max_element(cnt.begin(), cnt.end()) : 0;
    }
    if (s.nnz > INT32_MAX) fail(NLQ_EINVAL, "more than 2^31 stored entries");
    s.col.alloc(s.ctx, sizeof(int32_t) * std::max<int64_t>(s.nnz, 1));
    hipLaunchKernelGGL(k_rows, dim3(nn), dim3(kWave), 0, st, nn, ne_off.as<int64_t>(),
                       ne_items.as<int32_t>(), nb_off.as<int64_t>(), nb.as<int32_t>(),
                       row_cnt.as<int64_t>(), s.row_ptr.as<int64_t>(), s.col.as<int32_t>(),
                       err.as<int>());
    NLQ_CHECK_LAUNCH();
    // transpose map and element blocks
    s.tmap.alloc(s.ctx, sizeof(int32_t) * std::max<int64_t>(s.nnz, 1));
    hipLaunchKernelGGL(k_transpose_map, dim3(nn), dim3(kWave), 0, st, nn,
                       s.row_ptr.as<int64_t>(), s.col.as<int32_t>(), s.tmap.as<int32_t>(),
                       err.as<int>());
    NLQ_CHECK_LAUNCH();
    s.elpos.alloc(s.ctx, sizeof(int32_t) * ne * nv * nv);
    dim3 g2((ne * nv * nv + 255) / 256);
    {
        auto kern = nv == 3 ? k_elem_block_pos<3>
                  : nv == 4 ? k_elem_block_pos<4>
                  : nv == 6 ? k_elem_block_pos<6>
                  : nv == 8 ? k_elem_block_pos<8>
                  : nv == 10 ? k_elem_block_pos<10> : k_elem_block_pos<20>;
        hipLaunchKernelGGL(kern, g2, b1, 0, st, ne, m.conn.as<int32_t>(), s.row_ptr.as<int64_t>(),
                           s.col.as<int32_t>(), s.elpos.as<int32_t>(), err.as<int>());
    }
    NLQ_CHECK_LAUNCH();
    int herr = 0;
    NLQ_HIP(hipMemcpyAsync(&herr, err.as<void>(), sizeof(int), hipMemcpyDeviceToHost, st));
    NLQ_HIP(hipStreamSynchronize(st));
    if (herr & 6) fail(NLQ_EINVAL, "node-id window of a neighbourhood exceeds 131072 (renumber the mesh)");
    if (herr) fail(NLQ_EDEVICE, "internal error: pattern is not symmetric");
}

// ---------------------------------------------------------------- box mesh

namespace {

__global__ void k_box_nodes(int dim, int n, int k_gamma, int64_t nn, double *coords,
                            uint8_t *constrained)
{
    const int64_t id = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (id >= nn) return;
    int64_t r = id;
    uint8_t c = 0;
    for (int k = 0; k < dim; ++k) {
        const int i = static_cast<int>(r % (n + 1));
        r /= (n + 1);
        coords[id * dim + k] = static_cast<double>(i) / static_cast<double>(n);
        if (i <= k_gamma || i >= n - k_gamma) c = 1;
    }
    constrained[id] = c;
}

__global__ void k_box_elems(int dim, int n, int64_t ne, int32_t *conn)
{
    const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= ne) return;
    const int nperm = dim == 2 ? 2 : 6;
    const int p = static_cast<int>(e % nperm);
    int64_t cell = e / nperm;
    // permutations of {0..dim-1} in lexicographic order
    const int perm2[2][2] = {{0, 1}, {1, 0}};
    const int perm3[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
    int c[3] = {0, 0, 0};
    for (int k = 0; k < dim; ++k) {
        c[k] = static_cast<int>(cell % n);
        cell /= n;
    }
    const int64_t nn1 = n + 1;
    auto node = [&](const int *v) {
        int64_t id = v[0];
        if (dim > 1) id += nn1 * v[1];
        if (dim > 2) id += nn1 * nn1 * v[2];
        return static_cast<int32_t>(id);
    };
    int v[3] = {c[0], c[1], c[2]};
    conn[e * (dim + 1)] = node(v);
    for (int k = 0; k < dim; ++k) {
        const int ax = dim == 2 ? perm2[p][k] : perm3[p][k];
        v[ax] += 1;
        conn[e * (dim + 1) + k + 1] = node(v);
    }
}

}  // namespace

void launch_box_mesh(int dim, int n, int k_gamma, double *coords, int32_t *conn,
                     uint8_t *constrained, hipStream_t st)
{
    int64_t nn = 1, ne = 1;
    for (int k = 0; k < dim; ++k) {
        nn *= (n + 1);
        ne *= n;
    }
    ne *= (dim == 2 ? 2 : 6);
    hipLaunchKernelGGL(k_box_nodes, dim3((nn + 255) / 256), dim3(256), 0, st, dim, n, k_gamma, nn,
                       coords, constrained);
    NLQ_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_box_elems, dim3((ne + 255) / 256), dim3(256), 0, st, dim, n, ne, conn);
    NLQ_CHECK_LAUNCH();
}

}  // namespace nlq
