// Total-variation prior (the TV problem of Section 5) as f1 of SDMM with L1 = I: the proximity
// operator prox_{gamma TV_w}(u) by Chambolle's dual projection algorithm,
//     g = grad(div p - u / gamma),   p <- (p + tau g) / (1 + tau |g| / w),   tau = 1/8,
// from p = 0 for a fixed number of steps, then r1 = u - gamma div p.  grad: forward
// differences, zero on the last row / column; div = -grad^T; |g|^2 = |g1|^2 + |g2|^2.
//
// One step is one launch over 16 x 16 pixel tiles: the tile's p (with a one-pixel halo) goes
// to LDS, div p - u / gamma is formed on the tile plus one row and one column, and its
// gradient updates the tile's p into the other buffer of a ping-pong pair.  p stays zero on
// the last row (p1) and column (p2), where g is zero, so div needs no boundary cases.
#include "common.h"

namespace purify {

namespace {

constexpr int TVT = 16;          // tile side (256 threads)
constexpr double TV_TAU = 0.125;

// |a|^2 + |b|^2 of two complex numbers, in T
template <typename T>
__device__ __forceinline__ T mag2(cpx<T> a, cpx<T> b) {
    return a.x * a.x + a.y * a.y + b.x * b.x + b.y * b.y;
}

// u = x_hat + z1
template <typename T>
__global__ void __launch_bounds__(256)
k_tv_u(const cpx<T>* __restrict__ xh, const cpx<T>* __restrict__ z1, cpx<T>* __restrict__ u, int64_t N) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < N) u[i] = xh[i] + z1[i];
}

// One dual projection step.  first: p_in is zero (not read).
template <typename T>
__global__ void __launch_bounds__(TVT * TVT)
k_tv_step(const cpx<T>* __restrict__ u, const cpx<T>* __restrict__ p1i, const cpx<T>* __restrict__ p2i,
          cpx<T>* __restrict__ p1o, cpx<T>* __restrict__ p2o, const double* __restrict__ w, T inv_gamma,
          int n, int first) {
    __shared__ cpx<T> s1[TVT + 2][TVT + 2];   // p1 on rows i0-1 .. i0+16, cols j0-1 .. j0+16
    __shared__ cpx<T> s2[TVT + 2][TVT + 2];
    __shared__ cpx<T> sw[TVT + 1][TVT + 1];   // div p - u / gamma on rows i0 .. i0+16
    const int tiles = n / TVT;
    const int i0 = (blockIdx.x / tiles) * TVT, j0 = (blockIdx.x % tiles) * TVT;
    const cpx<T> zero = mk<T>(0, 0);
    for (int e = threadIdx.x; e < (TVT + 2) * (TVT + 2); e += TVT * TVT) {
        const int a = e / (TVT + 2), b = e % (TVT + 2);
        const int i = i0 - 1 + a, j = j0 - 1 + b;
        const bool in = !first && i >= 0 && i < n && j >= 0 && j < n;
        s1[a][b] = in ? p1i[(size_t)i * n + j] : zero;
        s2[a][b] = in ? p2i[(size_t)i * n + j] : zero;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < (TVT + 1) * (TVT + 1); e += TVT * TVT) {
        const int a = e / (TVT + 1), b = e % (TVT + 1);
        const int i = i0 + a, j = j0 + b;
        cpx<T> v = zero;
        if (i < n && j < n) {
            const cpx<T> d = (s1[a + 1][b + 1] - s1[a][b + 1]) + (s2[a + 1][b + 1] - s2[a + 1][b]);
            v = d - inv_gamma * u[(size_t)i * n + j];
        }
        sw[a][b] = v;
    }
    __syncthreads();
    const int ty = threadIdx.x / TVT, tx = threadIdx.x % TVT;
    const int i = i0 + ty, j = j0 + tx;
    const cpx<T> g1 = i < n - 1 ? sw[ty + 1][tx] - sw[ty][tx] : zero;
    const cpx<T> g2 = j < n - 1 ? sw[ty][tx + 1] - sw[ty][tx] : zero;
    const T mag = sqrt(mag2(g1, g2));
    const size_t o = (size_t)i * n + j;
    const T den = (T)1 + ((T)TV_TAU * mag) / (T)(w ? w[o] : 1.0);
    const cpx<T> q1 = s1[ty + 1][tx + 1] + (T)TV_TAU * g1;
    const cpx<T> q2 = s2[ty + 1][tx + 1] + (T)TV_TAU * g2;
    p1o[o] = mk<T>(q1.x / den, q1.y / den);
    p2o[o] = mk<T>(q2.x / den, q2.y / den);
}

// r1 = u - gamma div p ; z1 = u - r1 ; x1 = r1 - z1 ; partial sum_ij w_ij |(grad x_hat)_ij|
// (the objective TV_w(x_hat), before the update)
template <typename T>
__global__ void __launch_bounds__(256)
k_tv_final(const cpx<T>* __restrict__ xh, const cpx<T>* __restrict__ u, const cpx<T>* __restrict__ p1,
           const cpx<T>* __restrict__ p2, T gamma, cpx<T>* __restrict__ z1, cpx<T>* __restrict__ x1,
           const double* __restrict__ w, int n, double* part) {
    __shared__ double red[4];
    const int64_t N = (int64_t)n * n;
    double acc = 0;
    for (int64_t o = (int64_t)blockIdx.x * 256 + threadIdx.x; o < N; o += (int64_t)gridDim.x * 256) {
        const int i = (int)(o / n), j = (int)(o % n);
        const cpx<T> zero = mk<T>(0, 0);
        const cpx<T> d = (p1[o] - (i > 0 ? p1[o - n] : zero)) + (p2[o] - (j > 0 ? p2[o - 1] : zero));
        const cpx<T> uu = u[o];
        const cpx<T> r1 = uu - gamma * d;
        const cpx<T> z = uu - r1;
        z1[o] = z;
        x1[o] = r1 - z;
        const cpx<T> x = xh[o];
        const cpx<T> g1 = i < n - 1 ? xh[o + n] - x : zero;
        const cpx<T> g2 = j < n - 1 ? xh[o + 1] - x : zero;
        const double m = sqrt((double)g1.x * g1.x + (double)g1.y * g1.y + (double)g2.x * g2.x +
                              (double)g2.y * g2.y);
        acc += w ? w[o] * m : m;
    }
#pragma unroll
    for (int s = 32; s > 0; s >>= 1) acc += __shfl_xor(acc, s);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

// |(grad v)_ij| into a complex vector (real part; the statistics and weights of reweighted TV
// read it like dictionary coefficients) and/or its partial maxima (the default gamma)
template <typename T>
__global__ void __launch_bounds__(256)
k_grad_mag(const cpx<T>* __restrict__ v, int n, cpx<T>* __restrict__ out, double* part_max) {
    __shared__ double red[4];
    const int64_t N = (int64_t)n * n;
    double mx = 0;
    for (int64_t o = (int64_t)blockIdx.x * 256 + threadIdx.x; o < N; o += (int64_t)gridDim.x * 256) {
        const int i = (int)(o / n), j = (int)(o % n);
        const cpx<T> zero = mk<T>(0, 0);
        const cpx<T> x = v[o];
        const cpx<T> g1 = i < n - 1 ? v[o + n] - x : zero;
        const cpx<T> g2 = j < n - 1 ? v[o + 1] - x : zero;
        const double m = sqrt((double)g1.x * g1.x + (double)g1.y * g1.y + (double)g2.x * g2.x +
                              (double)g2.y * g2.y);
        if (out) out[o] = mk<T>((T)m, (T)0);
        mx = fmax(mx, m);
    }
#pragma unroll
    for (int s = 32; s > 0; s >>= 1) mx = fmax(mx, __shfl_xor(mx, s));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
    __syncthreads();
    if (threadIdx.x == 0 && part_max) part_max[blockIdx.x] = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
}

int tv_blocks(int64_t N) {
    const int64_t b = (N + 255) / 256;
    return (int)(b < 1024 ? b : 1024);
}

}  // namespace

template <typename T>
void launch_tv_step(const Plan& P, const cpx<T>* u, int k, const double* w, double gamma, hipStream_t s) {
    const int64_t N = P.N;
    cpx<T>* pa = (cpx<T>*)P.tvp;   // ping-pong dual fields: (p1, p2) of A then of B
    cpx<T>* pb = pa + 2 * N;
    cpx<T>* out = (k % 2 == 0) ? pa : pb;
    const cpx<T>* in = (k % 2 == 0) ? pb : pa;
    const int tiles = (P.n / TVT) * (P.n / TVT);
    hipLaunchKernelGGL(k_tv_step<T>, dim3(tiles), dim3(TVT * TVT), 0, s, u, in, in + N, out, out + N, w,
                       (T)(1.0 / gamma), P.n, k == 0 ? 1 : 0);
}

template <typename T>
void launch_tv_prox(const Plan& P, const cpx<T>* xh, cpx<T>* z1, cpx<T>* x1, cpx<T>* u, const double* w,
                    double gamma, int iters, double* part, int* nparts, hipStream_t s) {
    const int n = P.n;
    const int64_t N = P.N;
    cpx<T>* pa = (cpx<T>*)P.tvp;
    cpx<T>* pb = pa + 2 * N;
    hipLaunchKernelGGL(k_tv_u<T>, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, xh, z1, u, N);
    for (int k = 0; k < iters; ++k) launch_tv_step<T>(P, u, k, w, gamma, s);
    const cpx<T>* fin = ((iters - 1) % 2 == 0) ? pa : pb;
    const int nb = tv_blocks(N);
    hipLaunchKernelGGL(k_tv_final<T>, dim3(nb), dim3(256), 0, s, xh, (const cpx<T>*)u, fin, fin + N, (T)gamma, z1,
                       x1, w, n, part);
    *nparts = nb;
}

template <typename T>
int launch_grad_mag(const Plan& P, const cpx<T>* v, cpx<T>* out, double* part_max, hipStream_t s) {
    const int nb = tv_blocks(P.N);
    hipLaunchKernelGGL(k_grad_mag<T>, dim3(nb), dim3(256), 0, s, v, P.n, out, part_max);
    return nb;
}

#define PURIFY_INST_TV(T)                                                                                   \
    template void launch_tv_prox<T>(const Plan&, const cpx<T>*, cpx<T>*, cpx<T>*, cpx<T>*, const double*,    \
                                    double, int, double*, int*, hipStream_t);                               \
    template int launch_grad_mag<T>(const Plan&, const cpx<T>*, cpx<T>*, double*, hipStream_t);             \
    template void launch_tv_step<T>(const Plan&, const cpx<T>*, int, const double*, double, hipStream_t);
PURIFY_INST_TV(float)
PURIFY_INST_TV(double)

}  // namespace purify
