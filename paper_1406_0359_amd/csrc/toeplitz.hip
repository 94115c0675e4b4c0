// Stored normal operator (Section 3): Phi^dagger Phi of the Fourier model is the convolution
// of the image with the point-spread function h(d) = sum_m exp(+i omega_m . d), |d| < n per
// axis, so the global update's conjugate-gradient steps can use
//     T = Z^T F^dagger diag(c_hat) F Z,   c_hat = Re F c / K^2,
// with c the K x K circulant embedding of h (c[d mod K] = h(d), |d| < n; 0 where d = n).
// h is taken from the plan's own Phi^dagger, one n x n quadrant of d at a time:
//     h(p + s) = (Phi^dagger v_s)_p,  v_s,m = exp(i omega_m . s),  s in {-n/2, n/2}^2,
// and F c = sum_s exp(-2 pi i k . s / K) (F Z h_s)(k), F Z without S.  Taking the real part
// keeps the Hermitian part of c, so T stays Hermitian for the conjugate gradient.
#include "common.h"

namespace purify {

namespace {

// v_m = exp(i omega_m . s) in sorted order, from the plan's coordinates
// kappa = k0 + f + (J/2 - 1) (k0 mod K: exp(2 pi i kappa s / K) is K-periodic in kappa)
template <typename T>
__global__ void __launch_bounds__(256)
k_modulate(const int32_t* __restrict__ base, const T* __restrict__ frac, int64_t M, int K, double hj,
           int s1, int s2, cpx<T>* __restrict__ v) {
    const int64_t m = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (m >= M) return;
    const int b = base[m];
    const double k1 = (double)(b & 0xFFFF) + (double)frac[2 * m] + hj;
    const double k2 = (double)((b >> 16) & 0xFFFF) + (double)frac[2 * m + 1] + hj;
    // phase / pi = 2 (kappa_1 s_1 + kappa_2 s_2) / K
    const double t = 2.0 * (k1 * s1 + k2 * s2) / (double)K;
    double sn, cs;
    sincospi(t, &sn, &cs);
    v[m] = mk<T>((T)cs, (T)sn);
}

// zero image row 0 and/or column 0 (the offsets d = -n of the quadrants with s = -n/2)
template <typename T>
__global__ void __launch_bounds__(256) k_zero_edge(cpx<T>* __restrict__ x, int n, int zr, int zc) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    if (zr) x[i] = mk<T>(0, 0);
    if (zc) x[(size_t)i * n] = mk<T>(0, 0);
}

// chat[k] (+)= Re(exp(-2 pi i k . s / K) H[k]) / K^2 for s = (sig1, sig2) n/2:
// the phase is (-i)^e with e = (sig1 k1 + sig2 k2) mod 4.  chat is stored by groups of W
// columns, the layout the column stage reads (element (k1, k2) at ((k2 / W) K + k1) W + k2 mod W).
template <typename T>
__global__ void __launch_bounds__(256)
k_chat_accum(const cpx<T>* __restrict__ H, int K, int sig1, int sig2, int first, double scale, int W,
             T* __restrict__ chat) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= (int64_t)K * K) return;
    const int k1 = (int)(i / K), k2 = (int)(i % K);
    const int e = ((sig1 * k1 + sig2 * k2) % 4 + 4) % 4;
    const cpx<T> h = H[i];
    const T re = e == 0 ? h.x : (e == 1 ? h.y : (e == 2 ? -h.x : -h.y));
    const T add = (T)scale * re;
    const size_t o = ((size_t)(k2 / W) * K + k1) * W + k2 % W;
    chat[o] = first ? add : chat[o] + add;
}

}  // namespace

template <typename T>
void launch_modulate(const Plan& P, int s1, int s2, cpx<T>* v, hipStream_t s) {
    const unsigned b = (unsigned)((P.M + 255) / 256);
    hipLaunchKernelGGL(k_modulate<T>, dim3(b), dim3(256), 0, s, P.base, (const T*)P.frac, P.M, P.K,
                       0.5 * P.J - 1.0, s1, s2, v);
}
template <typename T>
void launch_zero_edge(cpx<T>* x, int n, bool row, bool col, hipStream_t s) {
    hipLaunchKernelGGL(k_zero_edge<T>, dim3((n + 255) / 256), dim3(256), 0, s, x, n, (int)row, (int)col);
}
template <typename T>
void launch_chat_accum(const Plan& P, const cpx<T>* H, int sig1, int sig2, bool first, hipStream_t s) {
    const int64_t KK = (int64_t)P.K * P.K;
    hipLaunchKernelGGL(k_chat_accum<T>, dim3((unsigned)((KK + 255) / 256)), dim3(256), 0, s, H, P.K, sig1, sig2,
                       (int)first, 1.0 / (double)KK, fft_toep_group<T>(P), (T*)P.chat);
}

#define PURIFY_INST_TOEP(T)                                                                     \
    template void launch_modulate<T>(const Plan&, int, int, cpx<T>*, hipStream_t);              \
    template void launch_zero_edge<T>(cpx<T>*, int, bool, bool, hipStream_t);                   \
    template void launch_chat_accum<T>(const Plan&, const cpx<T>*, int, int, bool, hipStream_t);
PURIFY_INST_TOEP(float)
PURIFY_INST_TOEP(double)

}  // namespace purify
