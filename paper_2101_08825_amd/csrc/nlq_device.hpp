// Device helpers shared by the library's kernels (wave64, gfx950).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace nlq {

constexpr int kWave = 64;

__device__ __forceinline__ int lane_id() { return static_cast<int>(__lane_id()); }

// number of set bits of `mask` below this lane
__device__ __forceinline__ int lanes_below(unsigned long long mask)
{
    return __popcll(mask & ((1ull << lane_id()) - 1ull));
}

__device__ __forceinline__ unsigned long long wave_ballot(bool p) { return __ballot(p); }

template <class T> __device__ __forceinline__ T wave_sum(T v)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

template <class T> __device__ __forceinline__ T wave_max(T v)
{
    for (int o = 32; o > 0; o >>= 1) {
        T w = __shfl_xor(v, o, kWave);
        v = w > v ? w : v;
    }
    return v;
}

template <class T> __device__ __forceinline__ T wave_min(T v)
{
    for (int o = 32; o > 0; o >>= 1) {
        T w = __shfl_xor(v, o, kWave);
        v = w < v ? w : v;
    }
    return v;
}

// inclusive prefix sum across the wave
template <class T> __device__ __forceinline__ T wave_incl_scan(T v)
{
    const int l = lane_id();
    for (int o = 1; o < kWave; o <<= 1) {
        T w = __shfl_up(v, o, kWave);
        if (l >= o) v += w;
    }
    return v;
}

// Approximate bbox distances of Section 5.1 in FP64 with every operation
// rounded as written (no contraction), so that the classification of Algorithm
// 1 is reproducible bit for bit.
//   aprx max = sqrt(sum_k max(d1_k^2, d2_k^2)),  aprx min = max_k max(0, d1_k, d2_k),
//   d1 = x_min - y_max, d2 = y_min - x_max.
// The square of aprx max is returned without the root: the caller compares it
// with the exact threshold s* = min{s : fl(sqrt(s)) >= t}, which decides
// fl(sqrt(s)) < t identically because the rounded root is monotone.  fmax
// (one instruction) picks the same value as a comparison for the finite
// operands here; the two differ only in the sign of a zero, which no later
// comparison sees.
template <int DIM>
__device__ __forceinline__ double aprx_max_sq(const double *lo1, const double *hi1,
                                              const double *lo2, const double *hi2)
{
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
        double d1 = __dsub_rn(lo1[k], hi2[k]);
        double d2 = __dsub_rn(lo2[k], hi1[k]);
        s = __dadd_rn(s, fmax(__dmul_rn(d1, d1), __dmul_rn(d2, d2)));
    }
    return s;
}

// Squared Euclidean distance of two boxes, sum_k max(0, d1_k, d2_k)^2, rounded
// as written (an ablation of the J^ref test; the paper's is aprx min below):
// compared with s* = min{s : fl(sqrt(s)) >= delta + eps}.
template <int DIM>
__device__ __forceinline__ double box_gap_sq(const double *lo1, const double *hi1, const double *lo2,
                                             const double *hi2)
{
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
        const double g = fmax(0.0, fmax(__dsub_rn(lo1[k], hi2[k]), __dsub_rn(lo2[k], hi1[k])));
        s = __dadd_rn(s, __dmul_rn(g, g));
    }
    return s;
}

template <int DIM>
__device__ __forceinline__ double aprx_min_dist(const double *lo1, const double *hi1,
                                                const double *lo2, const double *hi2)
{
    double r = 0.0;
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
        double d1 = __dsub_rn(lo1[k], hi2[k]);
        double d2 = __dsub_rn(lo2[k], hi1[k]);
        r = fmax(r, fmax(d1, d2));
    }
    return r;
}

}  // namespace nlq
