// Deterministic (fixed-order) accumulation of the assembled matrix.
//
// In this mode the integration kernel writes the outputs of every pair (the
// entries of B_lm, and the upper triangles of B_mm and B_ll, in the order of
// the epilogue's descriptors) to a pair-indexed buffer instead of adding them
// atomically.  The kernels here then form every sum in a fixed order, so the
// matrix is the same bit for bit from run to run, whatever the order in which
// work items ran or which other systems shared their launches:
//  * E_l: the B_lm of outer element l in the rows of l's nodes (aligned with
//    their CSR rows), summed over l's pairs in pair-list order;
//  * Dll[e]: B_ll of e's pairs in pair-list order; Dmm[e]: B_mm of the pairs
//    (l, e), l ascending (the pair relation is symmetric, so these l are J_e);
//  * entry (r, c): the sum over the elements l of node r, ascending, of E_l at
//    (r, c), then over the elements e holding r and c, ascending, of their
//    diagonal-block sums; then A = R + R^T (four-term form) as in the atomic
//    path.  The two-term form takes 2 B_lm^T and the full 2 B_mm blocks.
// Pairs are integrated in slabs of outer elements whose outputs fit one
// buffer; the sums above do not depend on the slab boundaries.
#include <algorithm>
#include <cstdlib>
#include <vector>

#include "nlq_device.hpp"
#include "nlq_internal.hpp"

namespace nlq {

namespace {

constexpr int64_t kDetSlabPairs = int64_t(8) << 20;   // pairs per slab (outputs: 1.3 GB in 2D, 2.3 GB in 3D)

__device__ __forceinline__ int64_t find_sorted(const int32_t *a, int64_t n, int32_t v)
{
    int64_t lo = 0, hi = n - 1;
    while (lo <= hi) {
        const int64_t mid = (lo + hi) >> 1;
        const int32_t x = a[mid];
        if (x == v) return mid;
        if (x < v) lo = mid + 1; else hi = mid - 1;
    }
    return -1;
}

// first index with a[k] >= v
__device__ __forceinline__ int64_t lower_bound_i32(const int32_t *a, int64_t n, int32_t v)
{
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (a[mid] < v) lo = mid + 1; else hi = mid;
    }
    return lo;
}

template <int NV> __device__ __forceinline__ int upper_slot(int i, int j)
{
    // slot of (i, j), i <= j: the diagonal first, then the products in row order
    if (i == j) return i;
    return NV + i * NV - (i * (i + 1)) / 2 + (j - i - 1);
}

template <int NV> __device__ __forceinline__ int local_of(const int32_t *conn, int64_t e, int32_t node)
{
    int k = -1;
#pragma unroll
    for (int v = 0; v < NV; ++v)
        if (conn[e * NV + v] == node) k = v;
    return k;
}

__global__ void k_n2e_count(int64_t n, const int32_t *conn, int64_t *cnt)
{
    const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t < n) atomicAdd(reinterpret_cast<unsigned long long *>(&cnt[conn[t]]), 1ull);
}

__global__ void k_n2e_fill(int64_t n, int nv, const int32_t *conn, const int64_t *off, int64_t *cur,
                           int32_t *items)
{
    const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const int32_t node = conn[t];
    const int64_t at = atomicAdd(reinterpret_cast<unsigned long long *>(&cur[node]), 1ull);
    items[off[node] + at] = static_cast<int32_t>(t / nv);
}

// each node's element list in ascending order (lists are short: insertion sort)
__global__ void k_n2e_sort(int64_t nn, const int64_t *off, int32_t *items)
{
    const int64_t r = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (r >= nn) return;
    int32_t *a = items + off[r];
    const int64_t n = off[r + 1] - off[r];
    for (int64_t i = 1; i < n; ++i) {
        const int32_t x = a[i];
        int64_t j = i - 1;
        while (j >= 0 && a[j] > x) {
            a[j + 1] = a[j];
            --j;
        }
        a[j + 1] = x;
    }
}

// entries of E_l: the lengths of the rows of l's nodes
template <int NV>
__global__ void k_elem_rowlen(int64_t ne, const int32_t *conn, const int64_t *row_ptr, int64_t *len)
{
    const int64_t l = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (l >= ne) return;
    int64_t s = 0;
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        const int32_t node = conn[l * NV + i];
        s += row_ptr[node + 1] - row_ptr[node];
    }
    len[l] = s;
}

// E_l and Dll[l] of the outer elements l of one slab, one wave each; the rows
// are summed in LDS, pairs in pair-list order (G pairs' positions and values
// are fetched at once, then added one pair after another).
template <int DIM>
__global__ void __launch_bounds__(kWave)
k_det_elem(int64_t lo, const int64_t *pair_off, const int32_t *pair_m, const int32_t *conn, const int64_t *row_ptr,
           const int32_t *col, const int64_t *eoff, const double *pb, int64_t pb_base, double *E, double *Dll,
           int *err)
{
    constexpr int NV = DIM + 1, NR = NV * (NV + 1) / 2, NO = NV * NV + 2 * NR, NLM = NV * NV;
    constexpr int G = kWave / NLM;   // pairs per round: 7 (2D), 4 (3D)
    extern __shared__ double rows[];
    const int64_t l = lo + blockIdx.x;
    const int lane = lane_id();
    int64_t rb[NV], rl[NV], ro[NV];
    int64_t tot = 0;
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        const int32_t node = conn[l * NV + i];
        rb[i] = row_ptr[node];
        rl[i] = row_ptr[node + 1] - rb[i];
        ro[i] = tot;
        tot += rl[i];
    }
    for (int64_t k = lane; k < tot; k += kWave) rows[k] = 0.0;
    __syncthreads();
    const int64_t p0 = pair_off[l], np = pair_off[l + 1] - p0;
    const int g = lane / NLM, o = lane % NLM;
    const int i = o / NV, j = o % NV;
    int64_t rbi = rb[0], rli = rl[0], roi = ro[0];
#pragma unroll
    for (int q = 1; q < NV; ++q)
        if (i == q) {
            rbi = rb[q];
            rli = rl[q];
            roi = ro[q];
        }
    for (int64_t q0 = 0; q0 < np; q0 += G) {
        int64_t at = -1;
        double v = 0.0;
        if (g < G && q0 + g < np) {
            const int64_t p = p0 + q0 + g;
            const int32_t mj = conn[static_cast<int64_t>(pair_m[p]) * NV + j];
            const int64_t k = find_sorted(col + rbi, rli, mj);
            if (k < 0) atomicOr(err, 1);
            else at = roi + k;
            v = pb[(p - pb_base) * NO + o];
        }
        for (int gg = 0; gg < G; ++gg) {
            if (g == gg && at >= 0) rows[at] += v;
            __syncthreads();
        }
    }
    // B_ll: lane u sums slot u over the pairs in order
    if (lane < NR) {
        double s = 0.0;
        for (int64_t q = 0; q < np; ++q) s += pb[(p0 + q - pb_base) * NO + NLM + NR + lane];
        Dll[l * NR + lane] = s;
    }
    for (int64_t k = lane; k < tot; k += kWave) E[eoff[l] + k] = rows[k];
}

// Dmm[e] += B_mm of the pairs (l, e), l in [lo, hi) ascending; one wave per e
template <int DIM>
__global__ void __launch_bounds__(kWave)
k_det_mm(int64_t lo, int64_t hi, const int64_t *pair_off, const int32_t *pair_m, const double *pb,
         int64_t pb_base, double *Dmm, int *err)
{
    constexpr int NV = DIM + 1, NR = NV * (NV + 1) / 2, NO = NV * NV + 2 * NR, NLM = NV * NV;
    const int64_t e = blockIdx.x;
    const int lane = lane_id();
    const int64_t a0 = pair_off[e], n = pair_off[e + 1] - a0;
    const int64_t qa = lower_bound_i32(pair_m + a0, n, static_cast<int32_t>(lo));
    const int64_t qb = lower_bound_i32(pair_m + a0, n, static_cast<int32_t>(hi));
    double acc = lane < NR ? Dmm[e * NR + lane] : 0.0;
    for (int64_t q0 = qa; q0 < qb; q0 += kWave) {
        int64_t pl = -1;
        if (q0 + lane < qb) {
            const int32_t l = pair_m[a0 + q0 + lane];
            const int64_t b = pair_off[l];
            const int64_t k = find_sorted(pair_m + b, pair_off[l + 1] - b, static_cast<int32_t>(e));
            if (k < 0) atomicOr(err, 2);
            else pl = b + k;
        }
        const int cnt = static_cast<int>(qb - q0 < kWave ? qb - q0 : kWave);
        for (int t = 0; t < cnt; ++t) {
            const int64_t pt = __shfl(pl, t, kWave);
            if (lane < NR && pt >= 0) acc += pb[(pt - pb_base) * NO + NLM + lane];
        }
    }
    if (lane < NR) Dmm[e * NR + lane] = acc;
}

// every stored entry of row r in a fixed order; one wave per row
template <int DIM>
__global__ void __launch_bounds__(kWave)
k_det_gather(int64_t nn, const int64_t *row_ptr, const int32_t *col, const int32_t *tmap, const int64_t *n2e_off,
             const int32_t *n2e, const int32_t *conn, const int64_t *eoff, const double *E, const double *Dll,
             const double *Dmm, int four, double *val)
{
    constexpr int NV = DIM + 1, NR = NV * (NV + 1) / 2;
    const int64_t r = blockIdx.x;
    const int lane = lane_id();
    const int64_t rb = row_ptr[r], len = row_ptr[r + 1] - rb;
    const int64_t e0 = n2e_off[r], ne_r = n2e_off[r + 1] - e0;
    // offset of row x within E_l: the rows of l's nodes before x
    auto row_off = [&](int64_t l, int32_t x) {
        int64_t s = 0;
        for (int v = 0; v < NV; ++v) {
            const int32_t node = conn[l * NV + v];
            if (node == x) break;
            s += row_ptr[node + 1] - row_ptr[node];
        }
        return s;
    };
    for (int64_t k = lane; k < len; k += kWave) {
        const int64_t pos = rb + k;
        const int32_t c = col[pos];
        double v = 0.0;
        if (four) {
            for (int64_t q = 0; q < ne_r; ++q) {
                const int64_t l = n2e[e0 + q];
                v += E[eoff[l] + row_off(l, static_cast<int32_t>(r)) + k];
            }
            for (int64_t q = 0; q < ne_r; ++q) {
                const int64_t e = n2e[e0 + q];
                const int i = local_of<NV>(conn, e, static_cast<int32_t>(r));
                const int j = local_of<NV>(conn, e, c);
                if (j < 0 || i > j) continue;
                const int u = upper_slot<NV>(i, j);
                const double d = Dll[e * NR + u] + Dmm[e * NR + u];
                v += i == j ? 0.5 * d : d;
            }
        } else {
            // 2 B_lm^T: the entry (c, r) of the l-rows, then the full 2 B_mm blocks
            const int64_t t = tmap[pos];
            const int64_t kc = t - row_ptr[c];
            const int64_t c0 = n2e_off[c], ne_c = n2e_off[c + 1] - c0;
            for (int64_t q = 0; q < ne_c; ++q) {
                const int64_t l = n2e[c0 + q];
                v += 2.0 * E[eoff[l] + row_off(l, c) + kc];
            }
            for (int64_t q = 0; q < ne_r; ++q) {
                const int64_t e = n2e[e0 + q];
                const int i = local_of<NV>(conn, e, static_cast<int32_t>(r));
                const int j = local_of<NV>(conn, e, c);
                if (j < 0) continue;
                v += 2.0 * Dmm[e * NR + upper_slot<NV>(i < j ? i : j, i < j ? j : i)];
            }
        }
        val[pos] = v;
    }
    (void)nn;
}

// node -> elements (ascending) and the E_l offsets of a system, once; built in
// local buffers and kept only when all of them exist (an allocation failure
// leaves the system without them, to be built on the next call)
void det_tables(System &s, hipStream_t st)
{
    if (!s.eoff.empty()) return;
    const Mesh &M = *s.mesh;
    const int nv = M.dim + 1;
    const int64_t ne = M.n_elems, nn = M.n_nodes, nc = ne * nv;
    DevBuf cnt(s.ctx, sizeof(int64_t) * (nn + 1), st), cur(s.ctx, sizeof(int64_t) * (nn + 1), st);
    NLQ_HIP(hipMemsetAsync(cnt.as<void>(), 0, sizeof(int64_t) * (nn + 1), st));
    NLQ_HIP(hipMemsetAsync(cur.as<void>(), 0, sizeof(int64_t) * (nn + 1), st));
    DevBuf n2e_off(s.ctx, sizeof(int64_t) * (nn + 1)), n2e(s.ctx, sizeof(int32_t) * std::max<int64_t>(nc, 1));
    const dim3 b(256);
    if (nc > 0) {
        hipLaunchKernelGGL(k_n2e_count, dim3((nc + 255) / 256), b, 0, st, nc, M.conn.as<int32_t>(), cnt.as<int64_t>());
        NLQ_CHECK_LAUNCH();
    }
    exclusive_scan_i64(s.ctx, cnt.as<int64_t>(), n2e_off.as<int64_t>(), nn + 1, st);
    if (nc > 0) {
        hipLaunchKernelGGL(k_n2e_fill, dim3((nc + 255) / 256), b, 0, st, nc, nv, M.conn.as<int32_t>(),
                           n2e_off.as<int64_t>(), cur.as<int64_t>(), n2e.as<int32_t>());
        NLQ_CHECK_LAUNCH();
    }
    if (nn > 0) {
        hipLaunchKernelGGL(k_n2e_sort, dim3((nn + 255) / 256), b, 0, st, nn, n2e_off.as<int64_t>(),
                           n2e.as<int32_t>());
        NLQ_CHECK_LAUNCH();
    }
    DevBuf len(s.ctx, sizeof(int64_t) * (ne + 1), st);
    NLQ_HIP(hipMemsetAsync(len.as<void>(), 0, sizeof(int64_t) * (ne + 1), st));
    if (ne > 0) {
        if (nv == 3)
            hipLaunchKernelGGL(k_elem_rowlen<3>, dim3((ne + 255) / 256), b, 0, st, ne, M.conn.as<int32_t>(),
                               s.row_ptr.as<int64_t>(), len.as<int64_t>());
        else
            hipLaunchKernelGGL(k_elem_rowlen<4>, dim3((ne + 255) / 256), b, 0, st, ne, M.conn.as<int32_t>(),
                               s.row_ptr.as<int64_t>(), len.as<int64_t>());
        NLQ_CHECK_LAUNCH();
    }
    DevBuf eoff(s.ctx, sizeof(int64_t) * (ne + 1));
    exclusive_scan_i64(s.ctx, len.as<int64_t>(), eoff.as<int64_t>(), ne + 1, st);
    NLQ_HIP(hipStreamSynchronize(st));
    s.n2e_off = std::move(n2e_off);
    s.n2e = std::move(n2e);
    s.eoff = std::move(eoff);
}

template <int DIM>
void det_slab_kernels(System &s, int64_t lo, int64_t hi, const double *pb, int64_t base, double *E, double *Dll,
                      double *Dmm, int *err, int lds, hipStream_t st)
{
    const Mesh &M = *s.mesh;
    if (hi > lo) {
        hipLaunchKernelGGL(k_det_elem<DIM>, dim3(static_cast<unsigned>(hi - lo)), dim3(kWave), lds, st, lo,
                           s.pair_off.as<int64_t>(), s.pair_m.as<int32_t>(), M.conn.as<int32_t>(),
                           s.row_ptr.as<int64_t>(), s.col.as<int32_t>(), s.eoff.as<int64_t>(), pb, base, E, Dll, err);
        NLQ_CHECK_LAUNCH();
    }
    hipLaunchKernelGGL(k_det_mm<DIM>, dim3(static_cast<unsigned>(M.n_elems)), dim3(kWave), 0, st, lo, hi,
                       s.pair_off.as<int64_t>(), s.pair_m.as<int32_t>(), pb, base, Dmm, err);
    NLQ_CHECK_LAUNCH();
}

// clears the slab pointer of a system however the assembly ends
struct SlabGuard {
    System &s;
    ~SlabGuard() { s.det_pb = nullptr; }
};

}  // namespace

void integrate_deterministic(System &s, hipStream_t st, hipEvent_t e0, hipEvent_t e1)
{
    const Mesh &M = *s.mesh;
    const int dim = M.dim, nv = dim + 1, nr = nv * (nv + 1) / 2, no = nv * nv + 2 * nr;
    const int64_t ne = M.n_elems, nn = M.n_nodes;
    if (e0) NLQ_HIP(hipEventRecord(e0, st));
    det_tables(s, st);
    // the rows of one element in LDS
    const int64_t lds = static_cast<int64_t>(nv) * std::max<int64_t>(s.max_row, 1) * 8;
    if (lds > 150 * 1024) fail(NLQ_EINVAL, "deterministic mode: the rows of an element exceed the LDS");
    int64_t e_total = 0;
    NLQ_HIP(hipMemcpyAsync(&e_total, s.eoff.as<int64_t>() + ne, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    std::vector<int64_t> off(ne + 1);
    NLQ_HIP(hipMemcpyAsync(off.data(), s.pair_off.as<void>(), sizeof(int64_t) * (ne + 1), hipMemcpyDeviceToHost, st));
    NLQ_HIP(hipStreamSynchronize(st));
    DevBuf E(s.ctx, sizeof(double) * std::max<int64_t>(e_total, 1), st);
    DevBuf Dll(s.ctx, sizeof(double) * std::max<int64_t>(ne * nr, 1), st);
    DevBuf Dmm(s.ctx, sizeof(double) * std::max<int64_t>(ne * nr, 1), st);
    DevBuf err(s.ctx, sizeof(int), st);
    NLQ_HIP(hipMemsetAsync(Dmm.as<void>(), 0, sizeof(double) * std::max<int64_t>(ne * nr, 1), st));
    NLQ_HIP(hipMemsetAsync(err.as<void>(), 0, sizeof(int), st));
    // NLQ_DET_SLAB_PAIRS overrides the slab size (tests use it to cut many slabs)
    int64_t slab = kDetSlabPairs;
    if (const char *env = std::getenv("NLQ_DET_SLAB_PAIRS")) slab = std::max<int64_t>(1, std::atoll(env));
    const int64_t cap = std::max(s.max_pairs, std::min(s.n_pairs, slab));
    DevBuf pb(s.ctx, sizeof(double) * no * std::max<int64_t>(cap, 1), st);
    if (dim == 2)
        NLQ_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(k_det_elem<2>),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds)));
    else
        NLQ_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(k_det_elem<3>),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds)));
    SlabGuard guard{s};
    int64_t lo = 0;
    do {
        // the largest slab from lo whose pairs fit the buffer (at least one element)
        int64_t hi = std::upper_bound(off.begin() + lo + 1, off.end(), off[lo] + cap) - off.begin() - 1;
        hi = std::min(std::max(hi, lo + 1), ne);
        s.det_pb = pb.as<double>();
        s.det_pb_base = off[lo];
        launch_integrate_jobs(s.ctx, s.launch, {IntegrateJob{&s, lo, hi}}, st);
        if (dim == 2)
            det_slab_kernels<2>(s, lo, hi, pb.as<double>(), off[lo], E.as<double>(), Dll.as<double>(),
                                Dmm.as<double>(), err.as<int>(), static_cast<int>(lds), st);
        else
            det_slab_kernels<3>(s, lo, hi, pb.as<double>(), off[lo], E.as<double>(), Dll.as<double>(),
                                Dmm.as<double>(), err.as<int>(), static_cast<int>(lds), st);
        // the next slab rewrites the pinned argument block this one was copied from
        NLQ_HIP(hipStreamSynchronize(st));
        lo = hi;
    } while (lo < ne);
    s.det_pb = nullptr;
    const int four = s.p.form == NLQ_FORM_SYM4;
    if (nn > 0) {
        if (dim == 2)
            hipLaunchKernelGGL(k_det_gather<2>, dim3(static_cast<unsigned>(nn)), dim3(kWave), 0, st, nn,
                               s.row_ptr.as<int64_t>(), s.col.as<int32_t>(), s.tmap.as<int32_t>(),
                               s.n2e_off.as<int64_t>(), s.n2e.as<int32_t>(), M.conn.as<int32_t>(),
                               s.eoff.as<int64_t>(), E.as<double>(), Dll.as<double>(), Dmm.as<double>(), four,
                               s.val.as<double>());
        else
            hipLaunchKernelGGL(k_det_gather<3>, dim3(static_cast<unsigned>(nn)), dim3(kWave), 0, st, nn,
                               s.row_ptr.as<int64_t>(), s.col.as<int32_t>(), s.tmap.as<int32_t>(),
                               s.n2e_off.as<int64_t>(), s.n2e.as<int32_t>(), M.conn.as<int32_t>(),
                               s.eoff.as<int64_t>(), E.as<double>(), Dll.as<double>(), Dmm.as<double>(), four,
                               s.val.as<double>());
        NLQ_CHECK_LAUNCH();
    }
    if (four) launch_symmetrize(s, st);
    if (e1) NLQ_HIP(hipEventRecord(e1, st));
    int herr = 0;
    NLQ_HIP(hipMemcpyAsync(&herr, err.as<void>(), sizeof(int), hipMemcpyDeviceToHost, st));
    NLQ_HIP(hipStreamSynchronize(st));
    if (herr) fail(NLQ_EDEVICE, "internal error: deterministic sums found a pair or entry missing from the pattern");
}

}  // namespace nlq
