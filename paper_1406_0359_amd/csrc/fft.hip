// F and F^dagger of the measurement operator Phi = G F Z S (NUFFT, Section 4), fused with
// S (deapodisation) and Z (zero padding / cropping).
//
// One axis of F Z acting on n pixels p = j - n/2 and producing K = 2n frequencies is
//     (D v)[k] = sum_j v_j exp(-2 pi i k (j - n/2) / K).
// Splitting the output by parity, k = 2k' + r (r = 0, 1):
//     (D v)[2k' + r] = (-1)^k' i^r FFT_n( v_j exp(-pi i r j / n) )[k'],
// so each line costs two n-point FFTs and the n zero rows of the padded grid are never
// read.  The adjoint (K -> n) splits the input by parity instead:
//     (D^dag u)[j] = IFFT_n((-1)^k' u_2k')[j] + (-i) exp(pi i j / n) IFFT_n((-1)^k' u_2k'+1)[j].
//
// Passes (image x is n x n row-major, the grid is K x K stored [k2][k1]):
//   rows_fwd : x rows  --(S, D along axis 1)-->  tmp[k2][j1]    (K x n)
//   cols_fwd : tmp rows --(D along axis 0)-->    grid[k2][k1]   (K x K)
//   cols_adj : grid rows --(D^dag along k1)-->   tmp[k2][j1]
//   rows_adj : tmp columns --(D^dag along k2, S)--> x rows (+ fused CG epilogue)
// Every transform is a self-sorting Stockham FFT (radix 4, one radix-2 pass when log2 n is
// odd) on lines held in LDS; twiddles come from an FP64-accurate table.
#include "common.h"

namespace purify {

namespace {

constexpr int LDS_PAD = 1;   // one complex of padding per LDS line (transposed accesses)

template <typename T, bool INV>
__device__ __forceinline__ cpx<T> twid(const cpx<T>* __restrict__ tw, int idx) {
    cpx<T> w = tw[idx];
    if (INV) w.y = -w.y;
    return w;
}

// In-LDS Stockham FFT of NLINES lines of N = 2^LOGN points (line stride ls), NT threads.
// Data in natural order on entry and on exit; forward sign exp(-2 pi i), INV = conjugate.
template <typename T, int LOGN, int NLINES, int NT, bool INV>
__device__ __forceinline__ void lds_fft(cpx<T>* buf, int ls, const cpx<T>* __restrict__ tw, int tid) {
    constexpr int N = 1 << LOGN;
    constexpr int NR4 = LOGN / 2;
    constexpr bool HAS_R2 = (LOGN & 1) != 0;
    constexpr int Q = N / 4;
    constexpr int BF = NLINES * Q;
    constexpr int E = (BF + NT - 1) / NT;
#pragma unroll
    for (int s = 0; s < NR4; ++s) {
        const int Ns = 1 << (2 * s);
        const int tws = N >> (2 * s + 2);
        cpx<T> v[E][4];
        int gb[E];
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int g = tid + e * NT;
            gb[e] = g;
            if (g < BF) {
                const int line = g / Q, j = g % Q;
                const cpx<T>* src = buf + line * ls + j;
#pragma unroll
                for (int r = 0; r < 4; ++r) v[e][r] = src[r * Q];
            }
        }
        __syncthreads();
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int g = gb[e];
            if (g < BF) {
                const int line = g / Q, j = g % Q;
                const int k = j & (Ns - 1);
                if (s > 0) {
                    v[e][1] = v[e][1] * twid<T, INV>(tw, k * tws);
                    v[e][2] = v[e][2] * twid<T, INV>(tw, 2 * k * tws);
                    v[e][3] = v[e][3] * twid<T, INV>(tw, 3 * k * tws);
                }
                const cpx<T> s02 = v[e][0] + v[e][2], d02 = v[e][0] - v[e][2];
                const cpx<T> s13 = v[e][1] + v[e][3], d13 = v[e][1] - v[e][3];
                cpx<T>* dst = buf + line * ls + ((j - k) << 2) + k;
                dst[0] = s02 + s13;
                dst[2 * Ns] = s02 - s13;
                if (INV) {
                    dst[Ns] = d02 + mul_i(d13);
                    dst[3 * Ns] = d02 + mul_mi(d13);
                } else {
                    dst[Ns] = d02 + mul_mi(d13);
                    dst[3 * Ns] = d02 + mul_i(d13);
                }
            }
        }
        __syncthreads();
    }
    if (HAS_R2) {
        constexpr int H = N / 2;
        constexpr int BF2 = NLINES * H;
        constexpr int E2 = (BF2 + NT - 1) / NT;
        cpx<T> a[E2], b[E2];
#pragma unroll
        for (int e = 0; e < E2; ++e) {
            const int g = tid + e * NT;
            if (g < BF2) {
                const int line = g / H, j = g % H;
                a[e] = buf[line * ls + j];
                b[e] = buf[line * ls + j + H];
            }
        }
        __syncthreads();
#pragma unroll
        for (int e = 0; e < E2; ++e) {
            const int g = tid + e * NT;
            if (g < BF2) {
                const int line = g / H, j = g % H;
                const cpx<T> bt = b[e] * twid<T, INV>(tw, j);
                buf[line * ls + j] = a[e] + bt;
                buf[line * ls + j + H] = a[e] - bt;
            }
        }
        __syncthreads();
    }
}

// Rows (image lines) per workgroup for the row passes, and columns per workgroup for the
// column passes.  Two LDS lines (parities) per image line.
template <typename T>
constexpr int rows_per_wg(int logn) {
    const int N = 1 << logn;
    const int es = 2 * sizeof(T);
    int b_lds = 65536 / (2 * N * es);
    int b_occ = N / 256;
    int b = b_lds < b_occ ? b_lds : b_occ;
    if (b < 1) b = 1;
    int b_min = 128 / N;       // keep at least one wavefront of butterflies
    if (b < b_min) b = b_min;
    return b;
}
constexpr int cols_per_wg(int logn) {
    const int N = 1 << logn;
    int c = 128 / N;
    return c < 1 ? 1 : c;
}
constexpr int threads_for(int lines, int logn) {
    int bf = lines * (1 << logn) / 4;
    return bf < 64 ? 64 : (bf > 256 ? 256 : bf);
}

template <typename T, int LOGN, int B>
__global__ void __launch_bounds__(threads_for(2 * B, LOGN))
k_fft_rows_fwd(const cpx<T>* __restrict__ x, cpx<T>* __restrict__ tmp, const T* __restrict__ deap,
               const cpx<T>* __restrict__ tw, const cpx<T>* __restrict__ tw2) {
    constexpr int N = 1 << LOGN;
    constexpr int NT = threads_for(2 * B, LOGN);
    constexpr int LS = N + LDS_PAD;
    extern __shared__ unsigned char smem_raw[];
    cpx<T>* buf = reinterpret_cast<cpx<T>*>(smem_raw);
    const int tid = threadIdx.x;
    const int row0 = blockIdx.x * B;
    for (int idx = tid; idx < B * N; idx += NT) {
        const int b = idx / N, j = idx % N;
        const T s = deap[row0 + b] * deap[j];
        const cpx<T> v = s * x[(size_t)(row0 + b) * N + j];
        buf[(2 * b) * LS + j] = v;
        buf[(2 * b + 1) * LS + j] = v * tw2[j];
    }
    __syncthreads();
    lds_fft<T, LOGN, 2 * B, NT, false>(buf, LS, tw, tid);
    for (int idx = tid; idx < 2 * N * B; idx += NT) {
        const int b = idx % B, k2 = idx / B;
        const int r = k2 & 1, kp = k2 >> 1;
        cpx<T> v = buf[(2 * b + r) * LS + kp];
        if (kp & 1) v = mk<T>(-v.x, -v.y);
        if (r) v = mul_i(v);
        tmp[(size_t)k2 * N + row0 + b] = v;
    }
}

template <typename T, int LOGN, int C>
__global__ void __launch_bounds__(threads_for(2 * C, LOGN))
k_fft_cols_fwd(const cpx<T>* __restrict__ tmp, cpx<T>* __restrict__ grid,
               const cpx<T>* __restrict__ tw, const cpx<T>* __restrict__ tw2) {
    constexpr int N = 1 << LOGN;
    constexpr int K = 2 * N;
    constexpr int NT = threads_for(2 * C, LOGN);
    constexpr int LS = N + LDS_PAD;
    extern __shared__ unsigned char smem_raw[];
    cpx<T>* buf = reinterpret_cast<cpx<T>*>(smem_raw);
    const int tid = threadIdx.x;
    const int col0 = blockIdx.x * C;
    for (int idx = tid; idx < C * N; idx += NT) {
        const int c = idx / N, j = idx % N;
        const cpx<T> v = tmp[(size_t)(col0 + c) * N + j];
        buf[(2 * c) * LS + j] = v;
        buf[(2 * c + 1) * LS + j] = v * tw2[j];
    }
    __syncthreads();
    lds_fft<T, LOGN, 2 * C, NT, false>(buf, LS, tw, tid);
    for (int idx = tid; idx < C * K; idx += NT) {
        const int c = idx / K, k1 = idx % K;
        const int r = k1 & 1, kp = k1 >> 1;
        cpx<T> v = buf[(2 * c + r) * LS + kp];
        if (kp & 1) v = mk<T>(-v.x, -v.y);
        if (r) v = mul_i(v);
        grid[(size_t)(col0 + c) * K + k1] = v;
    }
}

template <typename T, int LOGN, int C>
__global__ void __launch_bounds__(threads_for(2 * C, LOGN))
k_fft_cols_adj(const cpx<T>* __restrict__ grid, cpx<T>* __restrict__ tmp,
               const cpx<T>* __restrict__ tw, const cpx<T>* __restrict__ tw2) {
    constexpr int N = 1 << LOGN;
    constexpr int K = 2 * N;
    constexpr int NT = threads_for(2 * C, LOGN);
    constexpr int LS = N + LDS_PAD;
    extern __shared__ unsigned char smem_raw[];
    cpx<T>* buf = reinterpret_cast<cpx<T>*>(smem_raw);
    const int tid = threadIdx.x;
    const int col0 = blockIdx.x * C;
    for (int idx = tid; idx < C * K; idx += NT) {
        const int c = idx / K, k1 = idx % K;
        const int r = k1 & 1, kp = k1 >> 1;
        cpx<T> v = grid[(size_t)(col0 + c) * K + k1];
        if (kp & 1) v = mk<T>(-v.x, -v.y);
        buf[(2 * c + r) * LS + kp] = v;
    }
    __syncthreads();
    lds_fft<T, LOGN, 2 * C, NT, true>(buf, LS, tw, tid);
    for (int idx = tid; idx < C * N; idx += NT) {
        const int c = idx / N, j = idx % N;
        const cpx<T> a = buf[(2 * c) * LS + j];
        const cpx<T> b = buf[(2 * c + 1) * LS + j];
        // a + (-i) exp(pi i j / n) b,  exp(pi i j/n) = conj(tw2[j])
        const cpx<T> t = mulc(b, tw2[j]);
        tmp[(size_t)(col0 + c) * N + j] = a + mul_mi(t);
    }
}

__device__ __forceinline__ double block_sum_256(double v, double* red) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) red[w] = v;
    __syncthreads();
    double t = 0;
    if (threadIdx.x == 0) {
        const int nw = (blockDim.x + 63) >> 6;
        for (int i = 0; i < nw; ++i) t += red[i];
    }
    return t;
}

template <typename T, int LOGN, int B>
__global__ void __launch_bounds__(threads_for(2 * B, LOGN))
k_fft_rows_adj(const cpx<T>* __restrict__ tmp, cpx<T>* __restrict__ x, const T* __restrict__ deap,
               const cpx<T>* __restrict__ tw, const cpx<T>* __restrict__ tw2, T c1,
               const cpx<T>* __restrict__ v, T c2, double* __restrict__ dot_part) {
    constexpr int N = 1 << LOGN;
    constexpr int K = 2 * N;
    constexpr int NT = threads_for(2 * B, LOGN);
    constexpr int LS = N + LDS_PAD;
    extern __shared__ unsigned char smem_raw[];
    cpx<T>* buf = reinterpret_cast<cpx<T>*>(smem_raw);
    __shared__ double red[8];
    const int tid = threadIdx.x;
    const int row0 = blockIdx.x * B;
    for (int idx = tid; idx < B * K; idx += NT) {
        const int b = idx % B, k2 = idx / B;
        const int r = k2 & 1, kp = k2 >> 1;
        cpx<T> u = tmp[(size_t)k2 * N + row0 + b];
        if (kp & 1) u = mk<T>(-u.x, -u.y);
        buf[(2 * b + r) * LS + kp] = u;
    }
    __syncthreads();
    lds_fft<T, LOGN, 2 * B, NT, true>(buf, LS, tw, tid);
    double acc = 0.0;
    for (int idx = tid; idx < B * N; idx += NT) {
        const int b = idx / N, j = idx % N;
        const cpx<T> a = buf[(2 * b) * LS + j];
        const cpx<T> bb = buf[(2 * b + 1) * LS + j];
        const cpx<T> t = a + mul_mi(mulc(bb, tw2[j]));
        const T s = c1 * deap[row0 + b] * deap[j];
        cpx<T> o = s * t;
        const size_t off = (size_t)(row0 + b) * N + j;
        if (v) {
            const cpx<T> vv = v[off];
            o = o + c2 * vv;
            if (dot_part) acc += (double)vv.x * (double)o.x + (double)vv.y * (double)o.y;
        }
        x[off] = o;
    }
    if (dot_part) {
        const double tot = block_sum_256(acc, red);
        if (tid == 0) dot_part[blockIdx.x] = tot;
    }
}

template <typename F>
void set_lds_limit(F* f, size_t bytes) {
    if (bytes > 65536) (void)hipFuncSetAttribute(reinterpret_cast<const void*>(f),
                                                 hipFuncAttributeMaxDynamicSharedMemorySize,
                                                 (int)bytes);
}

template <typename T, int LOGN>
void rows_fwd_impl(const Plan& P, const cpx<T>* x, cpx<T>* tmp, hipStream_t s) {
    constexpr int B = rows_per_wg<T>(LOGN);
    constexpr int NT = threads_for(2 * B, LOGN);
    constexpr int N = 1 << LOGN;
    const size_t lds = (size_t)2 * B * (N + LDS_PAD) * sizeof(cpx<T>);
    auto f = k_fft_rows_fwd<T, LOGN, B>;
    set_lds_limit(f, lds);
    hipLaunchKernelGGL(f, dim3(N / B), dim3(NT), lds, s, x, tmp, (const T*)P.deap,
                       (const cpx<T>*)P.tw, (const cpx<T>*)P.tw2);
}
template <typename T, int LOGN>
void cols_fwd_impl(const Plan& P, const cpx<T>* tmp, cpx<T>* grid, hipStream_t s) {
    constexpr int C = cols_per_wg(LOGN);
    constexpr int NT = threads_for(2 * C, LOGN);
    constexpr int N = 1 << LOGN;
    const size_t lds = (size_t)2 * C * (N + LDS_PAD) * sizeof(cpx<T>);
    auto f = k_fft_cols_fwd<T, LOGN, C>;
    set_lds_limit(f, lds);
    hipLaunchKernelGGL(f, dim3(2 * N / C), dim3(NT), lds, s, tmp, grid, (const cpx<T>*)P.tw,
                       (const cpx<T>*)P.tw2);
}
template <typename T, int LOGN>
void cols_adj_impl(const Plan& P, const cpx<T>* grid, cpx<T>* tmp, hipStream_t s) {
    constexpr int C = cols_per_wg(LOGN);
    constexpr int NT = threads_for(2 * C, LOGN);
    constexpr int N = 1 << LOGN;
    const size_t lds = (size_t)2 * C * (N + LDS_PAD) * sizeof(cpx<T>);
    auto f = k_fft_cols_adj<T, LOGN, C>;
    set_lds_limit(f, lds);
    hipLaunchKernelGGL(f, dim3(2 * N / C), dim3(NT), lds, s, grid, tmp, (const cpx<T>*)P.tw,
                       (const cpx<T>*)P.tw2);
}
template <typename T, int LOGN>
void rows_adj_impl(const Plan& P, const cpx<T>* tmp, cpx<T>* x, double c1, const cpx<T>* v,
                   double c2, double* dot_part, hipStream_t s) {
    constexpr int B = rows_per_wg<T>(LOGN);
    constexpr int NT = threads_for(2 * B, LOGN);
    constexpr int N = 1 << LOGN;
    const size_t lds = (size_t)2 * B * (N + LDS_PAD) * sizeof(cpx<T>);
    auto f = k_fft_rows_adj<T, LOGN, B>;
    set_lds_limit(f, lds);
    hipLaunchKernelGGL(f, dim3(N / B), dim3(NT), lds, s, tmp, x, (const T*)P.deap,
                       (const cpx<T>*)P.tw, (const cpx<T>*)P.tw2, (T)c1, v, (T)c2, dot_part);
}

int ilog2(int n) {
    int l = 0;
    while ((1 << l) < n) ++l;
    return l;
}

#define PURIFY_LOGN_DISPATCH(LOGN_VAR, CALL)          \
    switch (LOGN_VAR) {                               \
        case 4: { constexpr int L_ = 4; CALL; } break;  \
        case 5: { constexpr int L_ = 5; CALL; } break;  \
        case 6: { constexpr int L_ = 6; CALL; } break;  \
        case 7: { constexpr int L_ = 7; CALL; } break;  \
        case 8: { constexpr int L_ = 8; CALL; } break;  \
        case 9: { constexpr int L_ = 9; CALL; } break;  \
        case 10: { constexpr int L_ = 10; CALL; } break; \
        case 11: { constexpr int L_ = 11; CALL; } break; \
        case 12: { constexpr int L_ = 12; CALL; } break; \
        default: break;                               \
    }

}  // namespace

template <typename T>
void launch_fft_rows_fwd(const Plan& P, const cpx<T>* x, cpx<T>* tmp, hipStream_t s) {
    PURIFY_LOGN_DISPATCH(ilog2(P.n), (rows_fwd_impl<T, L_>(P, x, tmp, s)));
}
template <typename T>
void launch_fft_cols_fwd(const Plan& P, const cpx<T>* tmp, cpx<T>* grid, hipStream_t s) {
    PURIFY_LOGN_DISPATCH(ilog2(P.n), (cols_fwd_impl<T, L_>(P, tmp, grid, s)));
}
template <typename T>
void launch_fft_cols_adj(const Plan& P, const cpx<T>* grid, cpx<T>* tmp, hipStream_t s) {
    PURIFY_LOGN_DISPATCH(ilog2(P.n), (cols_adj_impl<T, L_>(P, grid, tmp, s)));
}
template <typename T>
void launch_fft_rows_adj(const Plan& P, const cpx<T>* tmp, cpx<T>* x, double c1, const cpx<T>* v,
                         double c2, double* dot_part, hipStream_t s) {
    PURIFY_LOGN_DISPATCH(ilog2(P.n), (rows_adj_impl<T, L_>(P, tmp, x, c1, v, c2, dot_part, s)));
}
template <typename T>
int fft_rows_adj_blocks(const Plan& P) {
    int r = 0;
    PURIFY_LOGN_DISPATCH(ilog2(P.n), (r = (1 << L_) / rows_per_wg<T>(L_)));
    return r;
}

template void launch_fft_rows_fwd<float>(const Plan&, const cpx<float>*, cpx<float>*, hipStream_t);
template void launch_fft_rows_fwd<double>(const Plan&, const cpx<double>*, cpx<double>*, hipStream_t);
template void launch_fft_cols_fwd<float>(const Plan&, const cpx<float>*, cpx<float>*, hipStream_t);
template void launch_fft_cols_fwd<double>(const Plan&, const cpx<double>*, cpx<double>*, hipStream_t);
template void launch_fft_cols_adj<float>(const Plan&, const cpx<float>*, cpx<float>*, hipStream_t);
template void launch_fft_cols_adj<double>(const Plan&, const cpx<double>*, cpx<double>*, hipStream_t);
template void launch_fft_rows_adj<float>(const Plan&, const cpx<float>*, cpx<float>*, double,
                                         const cpx<float>*, double, double*, hipStream_t);
template void launch_fft_rows_adj<double>(const Plan&, const cpx<double>*, cpx<double>*, double,
                                          const cpx<double>*, double, double*, hipStream_t);
template int fft_rows_adj_blocks<float>(const Plan&);
template int fft_rows_adj_blocks<double>(const Plan&);

}  // namespace purify
