// G and G^T of the measurement operator Phi = G F Z S (NUFFT, Section 4): Kaiser-Bessel
// interpolation between the K x K oversampled grid and M continuous visibilities.
//
// Each visibility m has grid coordinates kappa_m = omega_m K / (2 pi) and, per axis, J taps
// k = k0 .. k0+J-1 with k0 = floor(kappa - J/2) + 1 and weights psi(kappa - k).  The plan
// stores k0 mod K (packed, two 16-bit fields) and the fractional offset f = kappa - k0 -
// (J/2 - 1) in [0, 1), so the tap offsets are t_a = f + (J/2 - 1) - a.
//
// Degridding (G, a gather) runs one thread per visibility in tile-sorted order, so a
// wavefront reads neighbouring grid cells.  Gridding (G^T, a scatter) is owner-computes:
// one workgroup per T x T grid tile accumulates, in LDS, every contribution that lands in
// its tile -- from its own visibilities and from the neighbours' visibilities whose
// footprint spills across the tile edge -- then writes the tile once.  No global atomics,
// no halo buffers.  The plan sorts each tile's visibilities by spill class
// [none | +k1 | +k1 and +k2 | +k2] so every neighbour's spill set is one contiguous range.
#include "common.h"

namespace purify {

namespace {

template <typename T, int J>
__global__ void __launch_bounds__(256)
k_degrid(const cpx<T>* __restrict__ grid, cpx<T>* __restrict__ y, const int32_t* __restrict__ perm,
         const int32_t* __restrict__ base, const T* __restrict__ frac, int M, int K, T scale,
         KBSeries<T> kb) {
    const int m = blockIdx.x * 256 + threadIdx.x;
    if (m >= M) return;
    const int b = base[m];
    const int k1 = b & 0xFFFF, k2 = (b >> 16) & 0xFFFF;
    const T f1 = frac[2 * m], f2 = frac[2 * m + 1];
    T wa[J], wb[J];
#pragma unroll
    for (int a = 0; a < J; ++a) {
        wa[a] = kb_eval(kb, f1 + (kb.tap0 - (T)a));
        wb[a] = kb_eval(kb, f2 + (kb.tap0 - (T)a));
    }
    const int mask = K - 1;
    T ax = 0, ay = 0;
#pragma unroll
    for (int bb = 0; bb < J; ++bb) {
        const cpx<T>* row = grid + (size_t)((k2 + bb) & mask) * K;
        T rx = 0, ry = 0;
#pragma unroll
        for (int a = 0; a < J; ++a) {
            const cpx<T> g = row[(k1 + a) & mask];
            rx += wa[a] * g.x;
            ry += wa[a] * g.y;
        }
        ax += wb[bb] * rx;
        ay += wb[bb] * ry;
    }
    y[perm ? perm[m] : m] = mk<T>(scale * ax, scale * ay);
}

// Generic-J variant (J <= 16) for the less common kernel widths.
template <typename T>
__global__ void __launch_bounds__(256)
k_degrid_any(const cpx<T>* __restrict__ grid, cpx<T>* __restrict__ y, const int32_t* __restrict__ perm,
             const int32_t* __restrict__ base, const T* __restrict__ frac, int M, int K, T scale,
             KBSeries<T> kb, int J) {
    const int m = blockIdx.x * 256 + threadIdx.x;
    if (m >= M) return;
    const int b = base[m];
    const int k1 = b & 0xFFFF, k2 = (b >> 16) & 0xFFFF;
    const T f1 = frac[2 * m], f2 = frac[2 * m + 1];
    T wa[16], wb[16];
    for (int a = 0; a < J; ++a) {
        wa[a] = kb_eval(kb, f1 + (kb.tap0 - (T)a));
        wb[a] = kb_eval(kb, f2 + (kb.tap0 - (T)a));
    }
    const int mask = K - 1;
    T ax = 0, ay = 0;
    for (int bb = 0; bb < J; ++bb) {
        const cpx<T>* row = grid + (size_t)((k2 + bb) & mask) * K;
        T rx = 0, ry = 0;
        for (int a = 0; a < J; ++a) {
            const cpx<T> g = row[(k1 + a) & mask];
            rx += wa[a] * g.x;
            ry += wa[a] * g.y;
        }
        ax += wb[bb] * rx;
        ay += wb[bb] * ry;
    }
    y[perm ? perm[m] : m] = mk<T>(scale * ax, scale * ay);
}

template <typename T, int J, int TT>
__device__ __forceinline__ void grid_range(const cpx<T>* __restrict__ y, const int32_t* __restrict__ perm,
                                           const int32_t* __restrict__ base, const T* __restrict__ frac,
                                           int start, int end, int K, int t1o, int t2o,
                                           const KBSeries<T>& kb, int Jr, T* acc_re, T* acc_im) {
    constexpr int JJ = J > 0 ? J : 16;
    const int mask = K - 1;
    const int Jn = J > 0 ? J : Jr;
    for (int idx = start + (int)threadIdx.x; idx < end; idx += (int)blockDim.x) {
        const int b = base[idx];
        const int k1 = b & 0xFFFF, k2 = (b >> 16) & 0xFFFF;
        const T f1 = frac[2 * idx], f2 = frac[2 * idx + 1];
        const cpx<T> v = y[perm ? perm[idx] : idx];
        T wa[JJ];
#pragma unroll
        for (int a = 0; a < JJ; ++a)
            if (a < Jn) wa[a] = kb_eval(kb, f1 + (kb.tap0 - (T)a));
#pragma unroll
        for (int bb = 0; bb < JJ; ++bb) {
            if (bb >= Jn) break;
            const int c2 = ((k2 + bb) & mask) - t2o;
            if ((unsigned)c2 >= (unsigned)TT) continue;
            const T wbv = kb_eval(kb, f2 + (kb.tap0 - (T)bb));
            const T vx = wbv * v.x, vy = wbv * v.y;
#pragma unroll
            for (int a = 0; a < JJ; ++a) {
                if (a >= Jn) break;
                const int c1 = ((k1 + a) & mask) - t1o;
                if ((unsigned)c1 < (unsigned)TT) {
                    atomicAdd(&acc_re[c2 * TT + c1], wa[a] * vx);
                    atomicAdd(&acc_im[c2 * TT + c1], wa[a] * vy);
                }
            }
        }
    }
}

template <typename T, int J, int TT>
__global__ void __launch_bounds__(256)
k_grid(const cpx<T>* __restrict__ y, const int32_t* __restrict__ perm, const int32_t* __restrict__ base,
       const T* __restrict__ frac, const int32_t* __restrict__ off, cpx<T>* __restrict__ grid, int K,
       int nT, KBSeries<T> kb, int Jr) {
    __shared__ T acc_re[TT * TT];
    __shared__ T acc_im[TT * TT];
    const int tile = blockIdx.x;
    const int t1 = tile % nT, t2 = tile / nT;
    for (int i = threadIdx.x; i < TT * TT; i += blockDim.x) {
        acc_re[i] = 0;
        acc_im[i] = 0;
    }
    __syncthreads();
    const int t1m = (t1 + nT - 1) % nT, t2m = (t2 + nT - 1) % nT;
    const int L = t2 * nT + t1m, U = t2m * nT + t1, Dg = t2m * nT + t1m;
    const int t1o = t1 * TT, t2o = t2 * TT;
    // own visibilities (every spill class), then the three neighbours' spill sets
    grid_range<T, J, TT>(y, perm, base, frac, off[4 * tile], off[4 * tile + 4], K, t1o, t2o, kb, Jr, acc_re, acc_im);
    grid_range<T, J, TT>(y, perm, base, frac, off[4 * L + 1], off[4 * L + 3], K, t1o, t2o, kb, Jr, acc_re, acc_im);
    grid_range<T, J, TT>(y, perm, base, frac, off[4 * U + 2], off[4 * U + 4], K, t1o, t2o, kb, Jr, acc_re, acc_im);
    grid_range<T, J, TT>(y, perm, base, frac, off[4 * Dg + 2], off[4 * Dg + 3], K, t1o, t2o, kb, Jr, acc_re, acc_im);
    __syncthreads();
    for (int i = threadIdx.x; i < TT * TT; i += blockDim.x) {
        const int r = i / TT, c = i % TT;
        grid[(size_t)(t2o + r) * K + t1o + c] = mk<T>(acc_re[i], acc_im[i]);
    }
}

template <typename T>
const KBSeries<T>& kb_of(const Plan& P);
template <>
const KBSeries<float>& kb_of<float>(const Plan& P) { return P.kb32; }
template <>
const KBSeries<double>& kb_of<double>(const Plan& P) { return P.kb64; }

template <typename T, int TT>
void grid_tt(const Plan& P, const cpx<T>* y, const int32_t* perm, cpx<T>* grid, hipStream_t s) {
    const dim3 g(P.nT * P.nT), b(256);
    const T* fr = (const T*)P.frac;
    const KBSeries<T>& kb = kb_of<T>(P);
    switch (P.J) {
        case 4: hipLaunchKernelGGL((k_grid<T, 4, TT>), g, b, 0, s, y, perm, P.base, fr, P.tileoff, grid, P.K, P.nT, kb, 4); break;
        case 6: hipLaunchKernelGGL((k_grid<T, 6, TT>), g, b, 0, s, y, perm, P.base, fr, P.tileoff, grid, P.K, P.nT, kb, 6); break;
        case 8: hipLaunchKernelGGL((k_grid<T, 8, TT>), g, b, 0, s, y, perm, P.base, fr, P.tileoff, grid, P.K, P.nT, kb, 8); break;
        default: hipLaunchKernelGGL((k_grid<T, 0, TT>), g, b, 0, s, y, perm, P.base, fr, P.tileoff, grid, P.K, P.nT, kb, P.J); break;
    }
}

}  // namespace

template <typename T>
void launch_degrid(const Plan& P, const cpx<T>* grid, cpx<T>* y, const int32_t* perm, double scale,
                   hipStream_t s) {
    const int M = (int)P.M;
    const dim3 g((M + 255) / 256), b(256);
    const T* fr = (const T*)P.frac;
    const KBSeries<T>& kb = kb_of<T>(P);
    switch (P.J) {
        case 4: hipLaunchKernelGGL((k_degrid<T, 4>), g, b, 0, s, grid, y, perm, P.base, fr, M, P.K, (T)scale, kb); break;
        case 6: hipLaunchKernelGGL((k_degrid<T, 6>), g, b, 0, s, grid, y, perm, P.base, fr, M, P.K, (T)scale, kb); break;
        case 8: hipLaunchKernelGGL((k_degrid<T, 8>), g, b, 0, s, grid, y, perm, P.base, fr, M, P.K, (T)scale, kb); break;
        default: hipLaunchKernelGGL((k_degrid_any<T>), g, b, 0, s, grid, y, perm, P.base, fr, M, P.K, (T)scale, kb, P.J); break;
    }
}

template <typename T>
void launch_grid(const Plan& P, const cpx<T>* y, const int32_t* perm, cpx<T>* grid, hipStream_t s) {
    if (P.TT == 16) grid_tt<T, 16>(P, y, perm, grid, s);
    else grid_tt<T, 32>(P, y, perm, grid, s);
}

template void launch_degrid<float>(const Plan&, const cpx<float>*, cpx<float>*, const int32_t*, double, hipStream_t);
template void launch_degrid<double>(const Plan&, const cpx<double>*, cpx<double>*, const int32_t*, double, hipStream_t);
template void launch_grid<float>(const Plan&, const cpx<float>*, const int32_t*, cpx<float>*, hipStream_t);
template void launch_grid<double>(const Plan&, const cpx<double>*, const int32_t*, cpx<double>*, hipStream_t);

}  // namespace purify
