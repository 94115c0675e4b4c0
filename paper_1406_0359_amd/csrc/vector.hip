// Vector kernels of SDMM (Algorithm 1): the three proximity steps with their dual updates
// (eq. (7) applied to the functions of eq. (6)), the conjugate-gradient updates of the
// global step, and deterministic FP64 reductions.
//
// Reductions are two-stage and fixed-order: each workgroup of a grid-stride kernel writes
// one FP64 partial (wavefront shuffle tree, then waves in order), and a single-workgroup
// finalize kernel sums the partials in a fixed pattern and derives the solver scalars
// (CG alpha / beta, the l2-ball scale, ...) on the device.  No float atomics, so the FP64
// path is bitwise reproducible.
#include "common.h"
#include "partials.h"

namespace purify {

namespace {

constexpr int RED_BLOCKS = 1024;   // grid size of every reducing vector kernel
constexpr int VT = 256;
static_assert(VT == PART_THREADS, "partial sums assume the vector kernels' block size");

__device__ __forceinline__ double block_sum(double v) {
    __shared__ double red[VT / 64];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) red[w] = v;
    __syncthreads();
    double t = 0;
    if (threadIdx.x == 0)
        for (int i = 0; i < VT / 64; ++i) t += red[i];
    __syncthreads();
    return t;
}

__device__ __forceinline__ double block_max(double v) {
    __shared__ double red[VT / 64];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) red[w] = v;
    __syncthreads();
    double t = 0;
    if (threadIdx.x == 0)
        for (int i = 0; i < VT / 64; ++i) t = fmax(t, red[i]);
    __syncthreads();
    return t;
}

// Every workgroup of a consumer kernel re-sums a partial-sum buffer in the same fixed
// order, so all of them see the identical scalar (no finalize launch, still deterministic).
__device__ __forceinline__ double sum_partials(const double* __restrict__ part, int count) {
    __shared__ double red2[VT / 64];
    double acc = strided_fold<false>(part, count, 0.0);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) red2[w] = acc;
    __syncthreads();
    double t = 0;
#pragma unroll
    for (int i = 0; i < VT / 64; ++i) t += red2[i];
    __syncthreads();
    return t;
}

int red_blocks(int64_t n) {
    int64_t b = (n + VT - 1) / VT;
    return (int)(b < RED_BLOCKS ? (b < 1 ? 1 : b) : RED_BLOCKS);
}
unsigned ew_blocks(int64_t n) { return (unsigned)((n + VT - 1) / VT); }

#define GRID_STRIDE(i, n) \
    for (int64_t i = (int64_t)blockIdx.x * VT + threadIdx.x; i < (n); i += (int64_t)gridDim.x * VT)

// Grid-stride loop over [0, n) that takes U of a thread's elements at a time: ld(i) for all
// of them first, so their loads are in flight together, then op(i, loaded) in index order --
// the order of GRID_STRIDE, so sums come out bit for bit the same.  (A reducing kernel's grid
// is RED_BLOCKS workgroups, four per CU: one element at a time keeps too few loads in flight
// to stream at HBM rate.)
template <int U, typename Ld, typename Op>
__device__ __forceinline__ void grid_stride_batched(int64_t n, Ld ld, Op op) {
    const int64_t S = (int64_t)gridDim.x * VT;
    for (int64_t i0 = (int64_t)blockIdx.x * VT + threadIdx.x; i0 < n; i0 += U * S) {
        decltype(ld(i0)) v[U];
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (i0 + u * S < n) v[u] = ld(i0 + u * S);
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (i0 + u * S < n) op(i0 + u * S, v[u]);
    }
}

template <typename T>
__global__ void __launch_bounds__(VT) k_fill(cpx<T>* v, cpx<T> val, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * VT + threadIdx.x;
    if (i < n) v[i] = val;
}

template <typename T>
__global__ void __launch_bounds__(VT) k_norm2(const cpx<T>* __restrict__ v, int64_t n, double* part) {
    double acc = 0;
    grid_stride_batched<4>(n, [&](int64_t i) { return v[i]; }, [&](int64_t, cpx<T> a) {
        acc += (double)a.x * a.x + (double)a.y * a.y;
    });
    const double t = block_sum(acc);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
}

template <typename T>
__global__ void __launch_bounds__(VT) k_maxabs(const cpx<T>* __restrict__ v, int64_t n, double* part) {
    double acc = 0;
    grid_stride_batched<4>(n, [&](int64_t i) { return v[i]; }, [&](int64_t, cpx<T> a) {
        acc = fmax(acc, sqrt((double)a.x * a.x + (double)a.y * a.y));
    });
    const double t = block_max(acc);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
}

__global__ void __launch_bounds__(VT)
k_finalize(const double* __restrict__ part, int count, double* sc, int slot, int op, double arg,
           double* hist, int hist_index) {
    double acc = 0;
    if (op == FIN_MAX) {
        acc = block_max(strided_fold<true>(part, count, acc));
    } else {
        acc = block_sum(strided_fold<false>(part, count, acc));
    }
    if (threadIdx.x != 0) return;
    const bool bad = !(acc == acc) || acc == INFINITY;
    if (bad) sc[SL_NONFINITE] = 1.0;
    switch (op) {
        case FIN_STORE:
        case FIN_MAX: sc[slot] = acc; break;
        case FIN_CG_ALPHA: {
            sc[SL_PQ] = acc;
            const double rho = sc[SL_RHO];
            sc[SL_ALPHA] = rho == 0.0 ? 0.0 : rho / acc;
        } break;
        case FIN_CG_BETA: {
            const double rho = sc[SL_RHO];
            sc[SL_BETA] = rho == 0.0 ? 0.0 : acc / rho;
            sc[SL_RHO] = acc;
        } break;
        case FIN_LAMBDA: {
            const double l = sqrt(acc);
            sc[SL_LAMBDA] = l;
            sc[SL_INVLAMBDA] = l > 0.0 ? 1.0 / l : 0.0;
        } break;
        case FIN_BALL: {
            sc[SL_D2] = acc;
            const double nd = sqrt(acc);
            sc[SL_BALL] = (nd == 0.0 || arg >= nd) ? 1.0 : arg / nd;
        } break;
        case FIN_HIST_OBJ:
        case FIN_HIST_OBJ_END: {
            sc[SL_OBJ] = acc;
            const int row = (int)sc[SL_ITER] % hist_index;
            if (hist) hist[2 * row] = acc;
            if (op == FIN_HIST_OBJ_END) sc[SL_ITER] += 1.0;
        } break;
        case FIN_HIST_RES: {
            sc[SL_RES2] = acc;
            const int row = (int)sc[SL_ITER] % hist_index;
            if (hist) hist[2 * row + 1] = sqrt(acc);
        } break;
        default: break;
    }
}

// The CG's last update: alpha = rho / Re<p, q> from the partial sums of both (rho == 0:
// alpha = 0, the early stop); x += alpha p.  The residual is not updated: the next global
// update starts again from r = b - A x.
template <typename T>
__global__ void __launch_bounds__(VT)
k_cg_x(cpx<T>* __restrict__ x, const cpx<T>* __restrict__ p, const double* __restrict__ rho_part, int rho_count,
       const double* __restrict__ pq_part, int pq_count, int64_t n) {
    // first element's operands are loaded before the partial sums are read (both in flight)
    const int64_t i0 = (int64_t)blockIdx.x * VT + threadIdx.x;
    cpx<T> x0, p0;
    if (i0 < n) {
        x0 = x[i0];
        p0 = p[i0];
    }
    const T alpha = cg_alpha<T>(rho_part, rho_count, pq_part, pq_count);
    GRID_STRIDE(i, n) {
        const bool first = i == i0;
        x[i] = (first ? x0 : x[i]) + alpha * (first ? p0 : p[i]);
    }
}

// i = 1 of Algorithm 1: u = v1 + z1 ; r1 = soft(u, gamma w) ; z1 = u - r1 ; v1 <- r1 - z1 ;
// partial sum_j w_j |v1_j| (objective ||W Psi^dag x_hat||_1, before the update).
template <typename T>
__global__ void __launch_bounds__(VT)
k_prox_l1(cpx<T>* __restrict__ v1, cpx<T>* __restrict__ z1, const double* __restrict__ w, double gamma,
          int64_t n, double* part) {
    double acc = 0;
    struct In {
        cpx<T> v, z;
        double w;
    };
    grid_stride_batched<4>(
        n, [&](int64_t i) { return In{v1[i], z1[i], w ? w[i] : 1.0}; },
        [&](int64_t i, const In& a) {
            const cpx<T> v = a.v;
            const double wi = a.w;
            acc += wi * sqrt((double)v.x * v.x + (double)v.y * v.y);
            const cpx<T> u = v + a.z;
            const T mag = sqrt(u.x * u.x + u.y * u.y);
            const T thr = (T)(gamma * wi);
            const T s = mag > thr ? (T)1 - thr / mag : (T)0;
            const cpx<T> r1 = s * u;
            const cpx<T> z = u - r1;
            z1[i] = z;
            v1[i] = r1 - z;
        });
    const double t = block_sum(acc);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// i = 2: u = x_hat + z2 ; r2 = max(Re u, 0) ; z2 = u - r2 ; x2 = r2 - z2
template <typename T>
__global__ void __launch_bounds__(VT)
k_prox_pos(const cpx<T>* __restrict__ xh, cpx<T>* __restrict__ z2, cpx<T>* __restrict__ x2, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * VT + threadIdx.x;
    if (i >= n) return;
    const cpx<T> u = xh[i] + z2[i];
    const cpx<T> r2 = mk<T>(u.x > 0 ? u.x : (T)0, (T)0);
    const cpx<T> z = u - r2;
    z2[i] = z;
    x2[i] = r2 - z;
}

// i = 3, pass 1: partial ||v3 + z3 - y~||^2 and ||y~ - v3||^2
template <typename T>
__global__ void __launch_bounds__(VT)
k_ball_part(const cpx<T>* __restrict__ v3, const cpx<T>* __restrict__ z3, const cpx<T>* __restrict__ yt,
            int64_t n, double* part_d, double* part_res) {
    double ad = 0, ar = 0;
    struct In {
        cpx<T> v, y, z;
    };
    grid_stride_batched<4>(
        n, [&](int64_t i) { return In{v3[i], yt[i], z3[i]}; },
        [&](int64_t, const In& a) {
            const cpx<T> d = a.v + a.z - a.y;
            ad += (double)d.x * d.x + (double)d.y * d.y;
            const double rx = (double)a.y.x - a.v.x, ry = (double)a.y.y - a.v.y;
            ar += rx * rx + ry * ry;
        });
    const double td = block_sum(ad);
    const double tr = block_sum(ar);
    if (threadIdx.x == 0) {
        part_d[blockIdx.x] = td;
        part_res[blockIdx.x] = tr;
    }
}

// i = 3, pass 2: s = min(1, eps~ / ||v3 + z3 - y~||) from the partial sums;
// u = v3 + z3 ; r3 = y~ + (u - y~) s ; z3 = u - r3 ; v3 <- r3 - z3 (diff: v3 <- r3 - z3 - v3,
// the change from the incoming Phi~ x_hat).  Workgroup 0 also records ||u - y~||^2, the
// residual ||y~ - v3||^2 and its history row.
template <typename T>
__global__ void __launch_bounds__(VT)
k_prox_ball(cpx<T>* __restrict__ v3, cpx<T>* __restrict__ z3, const cpx<T>* __restrict__ yt,
            const double* __restrict__ part_d, const double* __restrict__ part_res, int count,
            double eps, double* sc, double* hist, int hist_cap, int64_t n, int diff) {
    // first element's operands are loaded before the partial sums are read (both in flight)
    const int64_t i0 = (int64_t)blockIdx.x * VT + threadIdx.x;
    cpx<T> y0, v0, z0;
    if (i0 < n) {
        y0 = yt[i0];
        v0 = v3[i0];
        z0 = z3[i0];
    }
    const double d2 = sum_partials(part_d, count);
    const double nd = sqrt(d2);
    const T s = (T)((nd == 0.0 || eps >= nd) ? 1.0 : eps / nd);
    if (blockIdx.x == 0) {
        const double res2 = sum_partials(part_res, count);
        if (threadIdx.x == 0) {
            sc[SL_D2] = d2;
            sc[SL_RES2] = res2;
            if (!(d2 == d2) || !(res2 == res2) || d2 == INFINITY || res2 == INFINITY) sc[SL_NONFINITE] = 1.0;
            if (hist) hist[2 * ((int)sc[SL_ITER] % hist_cap) + 1] = sqrt(res2);
        }
    }
    GRID_STRIDE(i, n) {
        const cpx<T> y = i == i0 ? y0 : yt[i];
        const cpx<T> v = i == i0 ? v0 : v3[i];
        const cpx<T> u = v + (i == i0 ? z0 : z3[i]);
        const cpx<T> r3 = y + s * (u - y);
        const cpx<T> z = u - r3;
        z3[i] = z;
        v3[i] = diff ? (r3 - z) - v : r3 - z;
    }
}

// Power iteration: v = w / ||w|| with ||w||^2 from the partial sums; workgroup 0 records
// lambda = ||w|| (so nu = sqrt(lambda) after the last step).
template <typename T>
__global__ void __launch_bounds__(VT)
k_power_normalise(cpx<T>* __restrict__ v, const cpx<T>* __restrict__ w, const double* __restrict__ part,
                  int count, double* sc, int64_t n) {
    const double l = sqrt(sum_partials(part, count));
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        sc[SL_LAMBDA] = l;
        if (!(l == l) || l == INFINITY) sc[SL_NONFINITE] = 1.0;
    }
    const T inv = (T)(l > 0.0 ? 1.0 / l : 0.0);
    GRID_STRIDE(i, n) v[i] = inv * w[i];
}

template <typename T>
__global__ void __launch_bounds__(VT)
k_permute_scale(const cpx<T>* __restrict__ yu, const int32_t* __restrict__ perm, T scale,
                cpx<T>* __restrict__ ys, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * VT + threadIdx.x;
    if (i < n) ys[i] = scale * yu[perm[i]];
}

template <typename T>
__global__ void __launch_bounds__(VT)
k_scale_by_slot(cpx<T>* __restrict__ dst, const cpx<T>* __restrict__ src, const double* __restrict__ sc,
                int slot, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * VT + threadIdx.x;
    if (i < n) dst[i] = (T)sc[slot] * src[i];
}

// Visibility blocks, pass 1: workgroup c sums over bperm[first, end) of its chunk (one block's
// visibilities) ||v3 + z3 - y~||^2 and ||y~ - v3||^2
template <typename T>
__global__ void __launch_bounds__(VT)
k_ball_part_blk(const cpx<T>* __restrict__ v3, const cpx<T>* __restrict__ z3, const cpx<T>* __restrict__ yt,
                const int32_t* __restrict__ bperm, const int32_t* __restrict__ chunks, double* part_d,
                double* part_res) {
    const int a = chunks[2 * blockIdx.x], b = chunks[2 * blockIdx.x + 1];
    double ad = 0, ar = 0;
    for (int j = a + (int)threadIdx.x; j < b; j += VT) {
        const int m = bperm[j];
        const cpx<T> v = v3[m], y = yt[m];
        const cpx<T> d = v + z3[m] - y;
        ad += (double)d.x * d.x + (double)d.y * d.y;
        const double rx = (double)y.x - v.x, ry = (double)y.y - v.y;
        ar += rx * rx + ry * ry;
    }
    const double td = block_sum(ad);
    const double tr = block_sum(ar);
    if (threadIdx.x == 0) {
        part_d[blockIdx.x] = td;
        part_res[blockIdx.x] = tr;
    }
}

// pass 2 (one workgroup): thread i sums block i's chunk partials in order; scale_i =
// min(1, eps~_i / ||u_i - y~_i||); thread 0 then records, over the blocks in order, the total
// residual ||y~ - Phi~ x||^2 (and its history row) and max_i ||y~_i - v3_i|| / eps~_i
__global__ void __launch_bounds__(1024)
k_ball_fin_blk(const double* __restrict__ part_d, const double* __restrict__ part_res,
               const int32_t* __restrict__ chunk_off, const double* __restrict__ eps, int R, double* scale,
               double* sc, double* hist, int hist_cap) {
    __shared__ double res_b[MAX_BLOCKS];
    __shared__ int bad;
    if (threadIdx.x == 0) bad = 0;
    __syncthreads();
    for (int i = threadIdx.x; i < R; i += blockDim.x) {
        double d2 = 0, r2 = 0;
        for (int c = chunk_off[i]; c < chunk_off[i + 1]; ++c) {
            d2 += part_d[c];
            r2 += part_res[c];
        }
        const double nd = sqrt(d2);
        scale[i] = (nd == 0.0 || eps[i] >= nd) ? 1.0 : eps[i] / nd;
        res_b[i] = r2;
        if (!(d2 == d2) || !(r2 == r2) || d2 == INFINITY || r2 == INFINITY) bad = 1;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    double tot = 0, ratio = 0;
    for (int i = 0; i < R; ++i) {
        tot += res_b[i];
        const double r = sqrt(res_b[i]);
        const double q = eps[i] > 0.0 ? r / eps[i] : (r > 0.0 ? INFINITY : 0.0);
        ratio = fmax(ratio, q);
    }
    sc[SL_RES2] = tot;
    sc[SL_BLK_RATIO] = ratio;
    if (bad) sc[SL_NONFINITE] = 1.0;
    if (hist) hist[2 * ((int)sc[SL_ITER] % hist_cap) + 1] = sqrt(tot);
}

// pass 3: u = v3 + z3 ; r3 = y~ + s_b (u - y~) with b the visibility's block ; z3 = u - r3 ;
// v3 <- r3 - z3
template <typename T>
__global__ void __launch_bounds__(VT)
k_prox_ball_blk(cpx<T>* __restrict__ v3, cpx<T>* __restrict__ z3, const cpx<T>* __restrict__ yt,
                const int32_t* __restrict__ bid, const double* __restrict__ scale, int64_t n, int diff) {
    const int64_t i = (int64_t)blockIdx.x * VT + threadIdx.x;
    if (i >= n) return;
    const T s = (T)scale[bid[i]];
    const cpx<T> y = yt[i];
    const cpx<T> v = v3[i];
    const cpx<T> u = v + z3[i];
    const cpx<T> r3 = y + s * (u - y);
    const cpx<T> z = u - r3;
    z3[i] = z;
    v3[i] = diff ? (r3 - z) - v : r3 - z;
}

// a -= b
template <typename T>
__global__ void __launch_bounds__(VT)
k_sub(cpx<T>* __restrict__ a, const cpx<T>* __restrict__ b, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * VT + threadIdx.x;
    if (i < n) a[i] = a[i] - b[i];
}

// Reweighting statistics: partial sums of Re and Im (the mean of the coefficients)
template <typename T>
__global__ void __launch_bounds__(VT)
k_sum(const cpx<T>* __restrict__ v, int64_t n, double* part_re, double* part_im) {
    double ar = 0, ai = 0;
    GRID_STRIDE(i, n) {
        const cpx<T> a = v[i];
        ar += (double)a.x;
        ai += (double)a.y;
    }
    const double tr = block_sum(ar);
    const double ti = block_sum(ai);
    if (threadIdx.x == 0) {
        part_re[blockIdx.x] = tr;
        part_im[blockIdx.x] = ti;
    }
}

// partial sums of |v_j - mean|^2 (second pass of the standard deviation)
template <typename T>
__global__ void __launch_bounds__(VT)
k_dev2(const cpx<T>* __restrict__ v, int64_t n, const double* __restrict__ sc, int slot_re, int slot_im,
       double* part) {
    const double mr = sc[slot_re] / (double)n, mi = sc[slot_im] / (double)n;
    double acc = 0;
    GRID_STRIDE(i, n) {
        const cpx<T> a = v[i];
        const double dr = (double)a.x - mr, di = (double)a.y - mi;
        acc += dr * dr + di * di;
    }
    const double t = block_sum(acc);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// w_j = delta / (delta + |a_j|): delta times the slope of log(delta + s) at s = |a_j|
template <typename T>
__global__ void __launch_bounds__(VT)
k_reweight(const cpx<T>* __restrict__ a, int64_t n, double delta, double* __restrict__ w) {
    const int64_t i = (int64_t)blockIdx.x * VT + threadIdx.x;
    if (i >= n) return;
    const cpx<T> v = a[i];
    const double den = delta + sqrt((double)v.x * v.x + (double)v.y * v.y);
    w[i] = den > 0.0 ? delta / den : 1.0;
}

// partial sums of ||a - b||^2 and ||b||^2 (relative variation between successive solves)
template <typename T>
__global__ void __launch_bounds__(VT)
k_diff2(const cpx<T>* __restrict__ a, const cpx<T>* __restrict__ b, int64_t n, double* part_d,
        double* part_b) {
    double ad = 0, ab = 0;
    GRID_STRIDE(i, n) {
        const cpx<T> u = a[i], v = b[i];
        const double dr = (double)u.x - v.x, di = (double)u.y - v.y;
        ad += dr * dr + di * di;
        ab += (double)v.x * v.x + (double)v.y * v.y;
    }
    const double td = block_sum(ad);
    const double tb = block_sum(ab);
    if (threadIdx.x == 0) {
        part_d[blockIdx.x] = td;
        part_b[blockIdx.x] = tb;
    }
}

}  // namespace

template <typename T>
void launch_fill(cpx<T>* v, cpx<T> val, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_fill<T>, dim3(ew_blocks(n)), dim3(VT), 0, s, v, val, n);
}
template <typename T>
int launch_norm2_part(const cpx<T>* v, int64_t n, double* part, hipStream_t s) {
    const int b = red_blocks(n);
    hipLaunchKernelGGL(k_norm2<T>, dim3(b), dim3(VT), 0, s, v, n, part);
    return b;
}
template <typename T>
int launch_maxabs_part(const cpx<T>* v, int64_t n, double* part, hipStream_t s) {
    const int b = red_blocks(n);
    hipLaunchKernelGGL(k_maxabs<T>, dim3(b), dim3(VT), 0, s, v, n, part);
    return b;
}
void launch_finalize(const double* part, int count, double* sc, int slot, int op, double arg,
                     double* hist, int hist_index, hipStream_t s) {
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(VT), 0, s, part, count, sc, slot, op, arg, hist,
                       hist_index);
}
template <typename T>
void launch_cg_x(cpx<T>* x, const cpx<T>* p, const double* rho_part, int rho_count, const double* pq_part,
                 int pq_count, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_cg_x<T>, dim3(red_blocks(n)), dim3(VT), 0, s, x, p, rho_part, rho_count, pq_part,
                       pq_count, n);
}
template <typename T>
int launch_prox_l1(cpx<T>* v1, cpx<T>* z1, const double* w, double gamma, int64_t n, double* part,
                   hipStream_t s) {
    const int b = red_blocks(n);
    hipLaunchKernelGGL(k_prox_l1<T>, dim3(b), dim3(VT), 0, s, v1, z1, w, gamma, n, part);
    return b;
}
template <typename T>
void launch_prox_pos(const cpx<T>* xh, cpx<T>* z2, cpx<T>* x2, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_prox_pos<T>, dim3(ew_blocks(n)), dim3(VT), 0, s, xh, z2, x2, n);
}
template <typename T>
int launch_ball_part(const cpx<T>* v3, const cpx<T>* z3, const cpx<T>* yt, int64_t n, double* part_d,
                     double* part_res, hipStream_t s) {
    const int b = red_blocks(n);
    hipLaunchKernelGGL(k_ball_part<T>, dim3(b), dim3(VT), 0, s, v3, z3, yt, n, part_d, part_res);
    return b;
}
template <typename T>
void launch_prox_ball(cpx<T>* v3, cpx<T>* z3, const cpx<T>* yt, const double* part_d,
                      const double* part_res, int count, double eps, double* sc, double* hist,
                      int hist_cap, int64_t n, bool diff, hipStream_t s) {
    hipLaunchKernelGGL(k_prox_ball<T>, dim3(red_blocks(n)), dim3(VT), 0, s, v3, z3, yt, part_d, part_res,
                       count, eps, sc, hist, hist_cap, n, diff ? 1 : 0);
}
template <typename T>
void launch_power_normalise(cpx<T>* v, const cpx<T>* w, const double* part, int count, double* sc,
                            int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_power_normalise<T>, dim3(red_blocks(n)), dim3(VT), 0, s, v, w, part, count, sc, n);
}
template <typename T>
void launch_permute_scale(const cpx<T>* y_user, const int32_t* perm, double scale, cpx<T>* y_sorted,
                          int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_permute_scale<T>, dim3(ew_blocks(n)), dim3(VT), 0, s, y_user, perm, (T)scale,
                       y_sorted, n);
}
template <typename T>
void launch_scale_by_slot(cpx<T>* dst, const cpx<T>* src, const double* sc, int slot, int64_t n,
                          hipStream_t s) {
    hipLaunchKernelGGL(k_scale_by_slot<T>, dim3(ew_blocks(n)), dim3(VT), 0, s, dst, src, sc, slot, n);
}

template <typename T>
void launch_ball_part_blk(const cpx<T>* v3, const cpx<T>* z3, const cpx<T>* yt, const int32_t* bperm,
                          const int32_t* chunks, int nchunks, double* part_d, double* part_res, hipStream_t s) {
    hipLaunchKernelGGL(k_ball_part_blk<T>, dim3(nchunks), dim3(VT), 0, s, v3, z3, yt, bperm, chunks, part_d,
                       part_res);
}
void launch_ball_fin_blk(const double* part_d, const double* part_res, const int32_t* chunk_off,
                         const double* eps, int R, double* scale, double* sc, double* hist, int hist_cap,
                         hipStream_t s) {
    hipLaunchKernelGGL(k_ball_fin_blk, dim3(1), dim3(1024), 0, s, part_d, part_res, chunk_off, eps, R, scale, sc,
                       hist, hist_cap);
}
template <typename T>
void launch_prox_ball_blk(cpx<T>* v3, cpx<T>* z3, const cpx<T>* yt, const int32_t* bid, const double* scale,
                          int64_t n, bool diff, hipStream_t s) {
    hipLaunchKernelGGL(k_prox_ball_blk<T>, dim3(ew_blocks(n)), dim3(VT), 0, s, v3, z3, yt, bid, scale, n,
                       diff ? 1 : 0);
}
template <typename T>
void launch_sub(cpx<T>* a, const cpx<T>* b, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_sub<T>, dim3(ew_blocks(n)), dim3(VT), 0, s, a, b, n);
}
template <typename T>
int launch_sum_part(const cpx<T>* v, int64_t n, double* part_re, double* part_im, hipStream_t s) {
    const int b = red_blocks(n);
    hipLaunchKernelGGL(k_sum<T>, dim3(b), dim3(VT), 0, s, v, n, part_re, part_im);
    return b;
}
template <typename T>
int launch_dev2_part(const cpx<T>* v, int64_t n, const double* sc, int slot_re, int slot_im, double* part,
                     hipStream_t s) {
    const int b = red_blocks(n);
    hipLaunchKernelGGL(k_dev2<T>, dim3(b), dim3(VT), 0, s, v, n, sc, slot_re, slot_im, part);
    return b;
}
template <typename T>
void launch_reweight(const cpx<T>* a, int64_t n, double delta, double* w, hipStream_t s) {
    hipLaunchKernelGGL(k_reweight<T>, dim3(ew_blocks(n)), dim3(VT), 0, s, a, n, delta, w);
}
template <typename T>
int launch_diff2_part(const cpx<T>* a, const cpx<T>* b, int64_t n, double* part_d, double* part_b,
                      hipStream_t s) {
    const int nb = red_blocks(n);
    hipLaunchKernelGGL(k_diff2<T>, dim3(nb), dim3(VT), 0, s, a, b, n, part_d, part_b);
    return nb;
}

#define PURIFY_INST_VEC(T)                                                                              \
    template void launch_fill<T>(cpx<T>*, cpx<T>, int64_t, hipStream_t);                                \
    template int launch_norm2_part<T>(const cpx<T>*, int64_t, double*, hipStream_t);                     \
    template int launch_maxabs_part<T>(const cpx<T>*, int64_t, double*, hipStream_t);                    \
    template void launch_cg_x<T>(cpx<T>*, const cpx<T>*, const double*, int, const double*, int, int64_t, \
                                 hipStream_t);                                                           \
    template void launch_power_normalise<T>(cpx<T>*, const cpx<T>*, const double*, int, double*, int64_t, \
                                            hipStream_t);                                                \
    template int launch_prox_l1<T>(cpx<T>*, cpx<T>*, const double*, double, int64_t, double*, hipStream_t); \
    template void launch_prox_pos<T>(const cpx<T>*, cpx<T>*, cpx<T>*, int64_t, hipStream_t);            \
    template int launch_ball_part<T>(const cpx<T>*, const cpx<T>*, const cpx<T>*, int64_t, double*,      \
                                     double*, hipStream_t);                                              \
    template void launch_prox_ball<T>(cpx<T>*, cpx<T>*, const cpx<T>*, const double*, const double*, int,  \
                                      double, double*, double*, int, int64_t, bool, hipStream_t);       \
    template void launch_permute_scale<T>(const cpx<T>*, const int32_t*, double, cpx<T>*, int64_t,       \
                                          hipStream_t);                                                  \
    template void launch_scale_by_slot<T>(cpx<T>*, const cpx<T>*, const double*, int, int64_t, hipStream_t); \
    template void launch_ball_part_blk<T>(const cpx<T>*, const cpx<T>*, const cpx<T>*, const int32_t*,      \
                                          const int32_t*, int, double*, double*, hipStream_t);            \
    template void launch_prox_ball_blk<T>(cpx<T>*, cpx<T>*, const cpx<T>*, const int32_t*, const double*,  \
                                          int64_t, bool, hipStream_t);                                    \
    template void launch_sub<T>(cpx<T>*, const cpx<T>*, int64_t, hipStream_t);                           \
    template int launch_sum_part<T>(const cpx<T>*, int64_t, double*, double*, hipStream_t);               \
    template int launch_dev2_part<T>(const cpx<T>*, int64_t, const double*, int, int, double*, hipStream_t); \
    template void launch_reweight<T>(const cpx<T>*, int64_t, double, double*, hipStream_t);               \
    template int launch_diff2_part<T>(const cpx<T>*, const cpx<T>*, int64_t, double*, double*, hipStream_t);

PURIFY_INST_VEC(float)
PURIFY_INST_VEC(double)

}  // namespace purify
