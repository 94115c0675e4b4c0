// SARA dictionary Psi / Psi^dagger (Section 2.2): Dirac basis plus Daubechies Db1..Db8
// wavelet bases, each scaled by 1/sqrt(q) so that Psi Psi^dagger = I (tight frame, as
// used in Section 3).
//
// Each wavelet basis is an L-level periodised orthonormal 2D DWT in Mallat layout.  One level
// on an axis of even length Ls:  a[i] = sum_k h[k] x[(2i+k) mod Ls],  d[i] = sum_k g[k] x[...]
// with g[k] = (-1)^k h[2N-1-k]; a level filters axis 1 then axis 0 of the top-left Ls x Ls
// block and the next level recurses on its LL quarter.  Synthesis is the exact transpose.
//
// All wavelet bases run in the same launch (blockIdx.z = basis); a level is two separable
// passes through a per-basis temporary so no launch reads what it writes.  The finest
// synthesis pass sums every basis (and the Dirac block) and writes the image once.
#include "common.h"

namespace purify {

namespace {

struct WavArgs {
    int n, q, nwav;
    int block[MAX_WAV];   // alpha block of each wavelet basis
    int flen[MAX_WAV];    // filter length 2N
    int dirac_block;      // -1 if no Dirac basis
};

// filters layout: [basis][0..15] = h, [basis][16..31] = g
template <typename T>
__global__ void __launch_bounds__(256)
k_dwt_rows_fwd(const cpx<T>* __restrict__ src, int src_stride_basis, cpx<T>* __restrict__ wt,
               const T* __restrict__ filt, WavArgs A, int Ls, T scale) {
    const int i = blockIdx.z;
    const int idx = blockIdx.x * 256 + threadIdx.x;
    if (idx >= Ls * Ls) return;
    const int n = A.n;
    const int r = idx / Ls, o = idx % Ls;
    const int half = Ls >> 1;
    const bool hi = o >= half;
    const int oi = hi ? o - half : o;
    const T* f = filt + i * 2 * MAX_TAPS + (hi ? MAX_TAPS : 0);
    const cpx<T>* s = src + (size_t)A.block[i] * src_stride_basis + (size_t)r * n;
    if (src_stride_basis == 0) s = src + (size_t)r * n;
    const int F = A.flen[i];
    T ax = 0, ay = 0;
    int pos = (2 * oi) % Ls;
    for (int k = 0; k < F; ++k) {
        const cpx<T> v = s[pos];
        ax += f[k] * v.x;
        ay += f[k] * v.y;
        if (++pos == Ls) pos = 0;
    }
    wt[(size_t)i * n * n + (size_t)r * n + o] = mk<T>(scale * ax, scale * ay);
}

template <typename T>
__global__ void __launch_bounds__(256)
k_dwt_cols_fwd(const cpx<T>* __restrict__ wt, cpx<T>* __restrict__ alpha, const T* __restrict__ filt,
               WavArgs A, int Ls) {
    const int i = blockIdx.z;
    const int idx = blockIdx.x * 256 + threadIdx.x;
    if (idx >= Ls * Ls) return;
    const int n = A.n;
    const int o = idx / Ls, c = idx % Ls;
    const int half = Ls >> 1;
    const bool hi = o >= half;
    const int oi = hi ? o - half : o;
    const T* f = filt + i * 2 * MAX_TAPS + (hi ? MAX_TAPS : 0);
    const cpx<T>* s = wt + (size_t)i * n * n + c;
    const int F = A.flen[i];
    T ax = 0, ay = 0;
    int pos = (2 * oi) % Ls;
    for (int k = 0; k < F; ++k) {
        const cpx<T> v = s[(size_t)pos * n];
        ax += f[k] * v.x;
        ay += f[k] * v.y;
        if (++pos == Ls) pos = 0;
    }
    alpha[(size_t)A.block[i] * n * n + (size_t)o * n + c] = mk<T>(ax, ay);
}

__device__ __forceinline__ int pmod(int a, int m) {
    int r = a % m;
    return r < 0 ? r + m : r;
}

// Transpose of the axis-0 analysis of one level: rows [0, half) of the block are the
// lowpass (LL from `ll` when given, the rest from alpha), rows [half, Ls) the highpass.
template <typename T>
__global__ void __launch_bounds__(256)
k_dwt_cols_inv(const cpx<T>* __restrict__ alpha, const cpx<T>* __restrict__ ll, cpx<T>* __restrict__ wt,
               const T* __restrict__ filt, WavArgs A, int Ls) {
    const int i = blockIdx.z;
    const int idx = blockIdx.x * 256 + threadIdx.x;
    if (idx >= Ls * Ls) return;
    const int n = A.n;
    const size_t N = (size_t)n * n;
    const int m = idx / Ls, c = idx % Ls;
    const int half = Ls >> 1;
    const T* h = filt + i * 2 * MAX_TAPS;
    const T* g = h + MAX_TAPS;
    const cpx<T>* al = alpha + (size_t)A.block[i] * N;
    const cpx<T>* lo = (ll && c < half) ? ll + (size_t)i * N : al;
    const int F = A.flen[i];
    T ax = 0, ay = 0;
    for (int k = m & 1; k < F; k += 2) {
        const int ii = pmod((m - k) / 2, half);
        const cpx<T> a = lo[(size_t)ii * n + c];
        const cpx<T> d = al[(size_t)(half + ii) * n + c];
        ax += h[k] * a.x + g[k] * d.x;
        ay += h[k] * a.y + g[k] * d.y;
    }
    wt[(size_t)i * N + (size_t)m * n + c] = mk<T>(ax, ay);
}

// Transpose of the axis-1 analysis; writes the basis' LL for the next finer level.
template <typename T>
__global__ void __launch_bounds__(256)
k_dwt_rows_inv(const cpx<T>* __restrict__ wt, cpx<T>* __restrict__ out, const T* __restrict__ filt,
               WavArgs A, int Ls) {
    const int i = blockIdx.z;
    const int idx = blockIdx.x * 256 + threadIdx.x;
    if (idx >= Ls * Ls) return;
    const int n = A.n;
    const size_t N = (size_t)n * n;
    const int r = idx / Ls, m = idx % Ls;
    const int half = Ls >> 1;
    const T* h = filt + i * 2 * MAX_TAPS;
    const T* g = h + MAX_TAPS;
    const cpx<T>* s = wt + (size_t)i * N + (size_t)r * n;
    const int F = A.flen[i];
    T ax = 0, ay = 0;
    for (int k = m & 1; k < F; k += 2) {
        const int ii = pmod((m - k) / 2, half);
        const cpx<T> a = s[ii];
        const cpx<T> d = s[half + ii];
        ax += h[k] * a.x + g[k] * d.x;
        ay += h[k] * a.y + g[k] * d.y;
    }
    out[(size_t)i * N + (size_t)r * n + m] = mk<T>(ax, ay);
}

// Finest synthesis level: axis-1 transpose for every basis, summed with the Dirac block,
// scaled by 1/sqrt(q), written to the image.
template <typename T>
__global__ void __launch_bounds__(256)
k_dwt_rows_inv_sum(const cpx<T>* __restrict__ wt, const cpx<T>* __restrict__ alpha, cpx<T>* __restrict__ x,
                   const T* __restrict__ filt, WavArgs A, T scale) {
    const int n = A.n;
    const size_t N = (size_t)n * n;
    const int idx = blockIdx.x * 256 + threadIdx.x;
    if (idx >= (int)N) return;
    const int r = idx / n, m = idx % n;
    const int half = n >> 1;
    T ax = 0, ay = 0;
    if (A.dirac_block >= 0) {
        const cpx<T> v = alpha[(size_t)A.dirac_block * N + idx];
        ax = v.x;
        ay = v.y;
    }
    for (int i = 0; i < A.nwav; ++i) {
        const T* h = filt + i * 2 * MAX_TAPS;
        const T* g = h + MAX_TAPS;
        const cpx<T>* s = wt + (size_t)i * N + (size_t)r * n;
        const int F = A.flen[i];
        for (int k = m & 1; k < F; k += 2) {
            const int ii = pmod((m - k) / 2, half);
            const cpx<T> a = s[ii];
            const cpx<T> d = s[half + ii];
            ax += h[k] * a.x + g[k] * d.x;
            ay += h[k] * a.y + g[k] * d.y;
        }
    }
    x[idx] = mk<T>(scale * ax, scale * ay);
}

template <typename T>
__global__ void __launch_bounds__(256)
k_scale_copy_c(const cpx<T>* __restrict__ src, cpx<T>* __restrict__ dst, T scale, int64_t count) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < count) dst[i] = scale * src[i];
}

WavArgs wav_args(const Plan& P) {
    WavArgs A{};
    A.n = P.n;
    A.q = P.q;
    A.nwav = P.nwav;
    for (int i = 0; i < P.nwav; ++i) {
        A.block[i] = P.wav_block[i];
        A.flen[i] = 2 * P.wav_N[i];
    }
    A.dirac_block = P.has_dirac ? 0 : -1;
    return A;
}

}  // namespace

template <typename T>
void launch_psi_adj(const Plan& P, const cpx<T>* x, cpx<T>* alpha, hipStream_t s) {
    const WavArgs A = wav_args(P);
    const T scale = (T)(1.0 / std::sqrt((double)P.q));
    const int64_t N = P.N;
    if (P.has_dirac)
        hipLaunchKernelGGL(k_scale_copy_c<T>, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, x,
                           alpha, scale, N);
    if (P.nwav == 0) return;
    const T* filt = (const T*)P.filters;
    cpx<T>* wt = (cpx<T>*)P.wt;
    for (int lev = 0; lev < P.levels; ++lev) {
        const int Ls = P.n >> lev;
        const dim3 g((Ls * Ls + 255) / 256, 1, P.nwav);
        if (lev == 0)
            hipLaunchKernelGGL(k_dwt_rows_fwd<T>, g, dim3(256), 0, s, x, 0, wt, filt, A, Ls, scale);
        else
            hipLaunchKernelGGL(k_dwt_rows_fwd<T>, g, dim3(256), 0, s, (const cpx<T>*)alpha,
                               (int)N, wt, filt, A, Ls, (T)1);
        hipLaunchKernelGGL(k_dwt_cols_fwd<T>, g, dim3(256), 0, s, (const cpx<T>*)wt, alpha, filt, A, Ls);
    }
}

template <typename T>
void launch_psi(const Plan& P, const cpx<T>* alpha, cpx<T>* x, hipStream_t s) {
    const WavArgs A = wav_args(P);
    const T scale = (T)(1.0 / std::sqrt((double)P.q));
    const int64_t N = P.N;
    if (P.nwav == 0) {
        hipLaunchKernelGGL(k_scale_copy_c<T>, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s,
                           alpha, x, scale, N);
        return;
    }
    const T* filt = (const T*)P.filters;
    cpx<T>* wt = (cpx<T>*)P.wt;
    cpx<T>* ll = (cpx<T>*)P.ws2;
    for (int lev = P.levels - 1; lev >= 0; --lev) {
        const int Ls = P.n >> lev;
        const dim3 g((Ls * Ls + 255) / 256, 1, P.nwav);
        const cpx<T>* llsrc = (lev == P.levels - 1) ? nullptr : ll;
        hipLaunchKernelGGL(k_dwt_cols_inv<T>, g, dim3(256), 0, s, alpha, llsrc, wt, filt, A, Ls);
        if (lev > 0)
            hipLaunchKernelGGL(k_dwt_rows_inv<T>, g, dim3(256), 0, s, (const cpx<T>*)wt, ll, filt, A, Ls);
        else
            hipLaunchKernelGGL(k_dwt_rows_inv_sum<T>, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s,
                               (const cpx<T>*)wt, alpha, x, filt, A, scale);
    }
}

template void launch_psi_adj<float>(const Plan&, const cpx<float>*, cpx<float>*, hipStream_t);
template void launch_psi_adj<double>(const Plan&, const cpx<double>*, cpx<double>*, hipStream_t);
template void launch_psi<float>(const Plan&, const cpx<float>*, cpx<float>*, hipStream_t);
template void launch_psi<double>(const Plan&, const cpx<double>*, cpx<double>*, hipStream_t);

}  // namespace purify
