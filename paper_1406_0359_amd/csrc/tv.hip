// Total-variation prior (the TV problem of Section 5) as f1 of SDMM with L1 = I: the proximity
// operator prox_{gamma TV_w}(u) by Chambolle's dual projection algorithm,
//     g = grad(div p - u / gamma),   p <- (p + tau g) / (1 + tau |g| / w),   tau = 1/8,
// from p = 0 for a fixed number of steps, then r1 = u - gamma div p.  grad: forward
// differences, zero on the last row / column; div = -grad^T; |g|^2 = |g1|^2 + |g2|^2.
//
// Four steps run in one launch over 16 x 16 pixel tiles: the tile's p and u with a four-pixel
// halo go to LDS, and each step forms div p - u / gamma and its gradient there, updating p in
// place; the tile's p is written to the other buffer of a ping-pong pair.  p stays zero on
// the last row (p1) and column (p2), where g is zero, and outside the image, so div needs no
// boundary cases.
#include "common.h"

namespace purify {

namespace {

constexpr int TVT = 16;          // tile side (256 threads)
constexpr double TV_TAU = 0.125;
constexpr int TV_KS = 4;         // dual projection steps per launch (halo width)

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

// Several dual projection steps in one launch: a 16 x 16 output tile with a halo of KS pixels
// (one step depends on the dual field one pixel away), so the tile's (16 + 2 KS)^2 region of
// p and u is loaded once, KS steps run in LDS (the valid part shrinking by one pixel a step),
// and the tile's p is written.  Pixels outside the image keep p = 0; every in-image pixel
// runs the arithmetic of k_tv_step, so the results are the same.
template <typename T, int KS>
__global__ void __launch_bounds__(TVT * TVT)
k_tv_steps(const cpx<T>* __restrict__ u, const cpx<T>* __restrict__ p1i, const cpx<T>* __restrict__ p2i,
           cpx<T>* __restrict__ p1o, cpx<T>* __restrict__ p2o, const double* __restrict__ w, T inv_gamma,
           int n, int first, int steps) {
    constexpr int RS = TVT + 2 * KS;
    __shared__ cpx<T> s1[RS][RS], s2[RS][RS], su[RS][RS], sw[RS][RS];
    const int tiles = n / TVT;
    const int i0 = (blockIdx.x / tiles) * TVT - KS, j0 = (blockIdx.x % tiles) * TVT - KS;   // region origin
    const cpx<T> zero = mk<T>(0, 0);
    for (int e = threadIdx.x; e < RS * RS; e += TVT * TVT) {
        const int a = e / RS, b = e % RS;
        const int i = i0 + a, j = j0 + b;
        const bool img = i >= 0 && i < n && j >= 0 && j < n;
        const size_t o = (size_t)(img ? i : 0) * n + (img ? j : 0);
        s1[a][b] = img && !first ? p1i[o] : zero;
        s2[a][b] = img && !first ? p2i[o] : zero;
        su[a][b] = img ? u[o] : zero;
    }
    __syncthreads();
    for (int st = 0; st < steps; ++st) {
        // W = div p - u / gamma where its inputs (one pixel up and left) are in the region
        for (int e = threadIdx.x; e < RS * RS; e += TVT * TVT) {
            const int a = e / RS, b = e % RS;
            if (a >= 1 && b >= 1) {
                const cpx<T> d = (s1[a][b] - s1[a - 1][b]) + (s2[a][b] - s2[a][b - 1]);
                sw[a][b] = d - inv_gamma * su[a][b];
            }
        }
        __syncthreads();
        // p <- (p + tau g) / (1 + tau |g| / w) with g the forward gradient of W (in place: a
        // pixel's update reads only its own p)
        for (int e = threadIdx.x; e < RS * RS; e += TVT * TVT) {
            const int a = e / RS, b = e % RS;
            const int i = i0 + a, j = j0 + b;
            if (a >= 1 && b >= 1 && a < RS - 1 && b < RS - 1 && i >= 0 && i < n && j >= 0 && j < n) {
                const cpx<T> g1 = i < n - 1 ? sw[a + 1][b] - sw[a][b] : zero;
                const cpx<T> g2 = j < n - 1 ? sw[a][b + 1] - sw[a][b] : zero;
                const T mag = sqrt(mag2(g1, g2));
                const T den = (T)1 + ((T)TV_TAU * mag) / (T)(w ? w[(size_t)i * n + j] : 1.0);
                const cpx<T> q1 = s1[a][b] + (T)TV_TAU * g1;
                const cpx<T> q2 = s2[a][b] + (T)TV_TAU * g2;
                s1[a][b] = mk<T>(q1.x / den, q1.y / den);
                s2[a][b] = mk<T>(q2.x / den, q2.y / den);
            }
        }
        __syncthreads();
    }
    const int ty = threadIdx.x / TVT, tx = threadIdx.x % TVT;
    const size_t o = (size_t)(i0 + KS + ty) * n + (j0 + KS + tx);
    p1o[o] = s1[KS + ty][KS + tx];
    p2o[o] = s2[KS + ty][KS + tx];
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

// launch k of the dual projection (TV_KS steps from the pair written by launch k - 1; k = 0
// starts from p = 0)
template <typename T>
void launch_tv_step(const Plan& P, const cpx<T>* u, int k, const double* w, double gamma, hipStream_t s) {
    const int64_t N = P.N;
    cpx<T>* pa = (cpx<T>*)P.tvp;   // ping-pong dual fields: (p1, p2) of A then of B
    cpx<T>* pb = pa + 2 * N;
    cpx<T>* out = (k % 2 == 0) ? pa : pb;
    const cpx<T>* in = (k % 2 == 0) ? pb : pa;
    const int tiles = (P.n / TVT) * (P.n / TVT);
    hipLaunchKernelGGL((k_tv_steps<T, TV_KS>), dim3(tiles), dim3(TVT * TVT), 0, s, u, in, in + N, out, out + N, w,
                       (T)(1.0 / gamma), P.n, k == 0 ? 1 : 0, TV_KS);
}

template <typename T>
void launch_tv_prox(const Plan& P, const cpx<T>* xh, cpx<T>* z1, cpx<T>* x1, cpx<T>* u, const double* w,
                    double gamma, int iters, double* part, int* nparts, hipStream_t s) {
    const int n = P.n;
    const int64_t N = P.N;
    cpx<T>* pa = (cpx<T>*)P.tvp;
    cpx<T>* pb = pa + 2 * N;
    hipLaunchKernelGGL(k_tv_u<T>, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, xh, z1, u, N);
    // TV_KS steps a launch, ping-pong between the pairs A and B (the last launch's output pair
    // holds the final field)
    const int tiles = (n / TVT) * (n / TVT);
    int launches = 0;
    for (int k = 0; k < iters; k += TV_KS, ++launches) {
        cpx<T>* out = (launches % 2 == 0) ? pa : pb;
        const cpx<T>* in = (launches % 2 == 0) ? pb : pa;
        const int steps = iters - k < TV_KS ? iters - k : TV_KS;
        hipLaunchKernelGGL((k_tv_steps<T, TV_KS>), dim3(tiles), dim3(TVT * TVT), 0, s, (const cpx<T>*)u, in, in + N,
                           out, out + N, w, (T)(1.0 / gamma), n, k == 0 ? 1 : 0, steps);
    }
    const cpx<T>* fin = ((launches - 1) % 2 == 0) ? pa : pb;
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
