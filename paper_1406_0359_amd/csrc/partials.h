// Fixed-order sums of partial-sum buffers inside one 256-thread workgroup.  Kernels in
// different source files that derive the same solver scalar from the same partials (the CG
// step length, for one) use these, so every one of them sees the identical value.
#pragma once

#include "common.h"

namespace purify {

constexpr int PART_THREADS = 256;   // block size of every kernel that calls these

// acc <- acc + part[i] (or fmax) over i = threadIdx.x + k PART_THREADS, k = 0, 1, ... in that
// order, four loads in flight at a time (the loop otherwise waits on each load in turn)
template <bool MAX>
__device__ __forceinline__ double strided_fold(const double* __restrict__ part, int count, double acc) {
    constexpr int S = PART_THREADS;
    for (int i0 = threadIdx.x; i0 < count; i0 += 4 * S) {
        double v[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) v[k] = i0 + k * S < count ? part[i0 + k * S] : 0.0;
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (i0 + k * S < count) acc = MAX ? fmax(acc, v[k]) : acc + v[k];
    }
    return acc;
}

// Two partial-sum buffers in one pass; every thread receives both totals.
__device__ __forceinline__ void sum_partials2(const double* __restrict__ pa, int na, const double* __restrict__ pb,
                                              int nb, double& ta, double& tb) {
    __shared__ double red3[2][PART_THREADS / 64];
    double a = strided_fold<false>(pa, na, 0.0);
    double b = strided_fold<false>(pb, nb, 0.0);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        a += __shfl_xor(a, o);
        b += __shfl_xor(b, o);
    }
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) {
        red3[0][w] = a;
        red3[1][w] = b;
    }
    __syncthreads();
    ta = 0;
    tb = 0;
#pragma unroll
    for (int i = 0; i < PART_THREADS / 64; ++i) {
        ta += red3[0][i];
        tb += red3[1][i];
    }
    __syncthreads();
}

// CG step length alpha = rho / <p, q> from their partial sums (0 when rho == 0: the early
// stop), in the precision the update x += alpha p is applied in
template <typename T>
__device__ __forceinline__ T cg_alpha(const double* rho_part, int rho_count, const double* pq_part, int pq_count) {
    double rho, pq;
    sum_partials2(rho_part, rho_count, pq_part, pq_count, rho, pq);
    return (T)(rho == 0.0 ? 0.0 : rho / pq);
}

}  // namespace purify
