// SARA dictionary Psi / Psi^dagger (Section 2.2): Dirac basis plus Daubechies Db1..Db8
// wavelet bases, each scaled by 1/sqrt(q) so that Psi Psi^dagger = I (tight frame, as
// used in Section 3).
//
// Each wavelet basis is an L-level periodised orthonormal 2D DWT in Mallat layout.  One level
// on an axis of even length Ls:  a[i] = sum_k h[k] x[(2i+k) mod Ls],  d[i] = sum_k g[k] x[...]
// with g[k] = (-1)^k h[2N-1-k]; a level filters axis 1 then axis 0 of the top-left Ls x Ls
// block and the next level recurses on its LL quarter.  Synthesis is the exact transpose.
//
// All wavelet bases run in the same launch; a level is one launch of 2D tiles (both axes
// through LDS).  The finest synthesis level sums every basis (and the Dirac block) per
// output tile and writes the image once.
#include "common.h"
#include "partials.h"

namespace purify {

namespace {

struct WavArgs {
    int n, q, nwav;
    int block[MAX_WAV];   // alpha block of each wavelet basis
    int flen[MAX_WAV];    // filter length 2N
    int dirac_block;      // -1 if no Dirac basis
};

// filters layout: [basis][0..15] = h, [basis][16..31] = g.  Kernels stage a basis' taps in
// LDS (lanes index them by output parity, which a register array cannot serve).

__device__ __forceinline__ float fma_(float a, float b, float c) { return fmaf(a, b, c); }
__device__ __forceinline__ double fma_(double a, double b, double c) { return fma(a, b, c); }

// Row and column of a flattened tile index: i / d and i mod d for 0 <= i < 2^20 and
// 1 <= d < 2^12 (every tile and window index here) from a float reciprocal taken once.  The
// float quotient is within 1/4 of i / d, so its truncation is off by at most one, which one
// remainder test corrects; a few instructions instead of an integer division, in kernels
// whose arithmetic, not memory, sets their time.
struct SmallDiv {
    int d;
    float rd;
    __device__ explicit SmallDiv(int d_) : d(d_), rd(__builtin_amdgcn_rcpf((float)d_)) {}   // 1-ulp reciprocal
    __device__ __forceinline__ int quot(int i, int& rem) const {
        int q = (int)((float)i * rd);
        int r = i - q * d;
        if (r >= d) {
            ++q;
            r -= d;
        } else if (r < 0) {
            --q;
            r += d;
        }
        rem = r;
        return q;
    }
};

// Global-to-LDS staging of `count` elements (element i read by ld(i) and stored by st(i, v),
// count <= MAXE NTH): a thread issues the loads of all its elements before storing any, so
// they are in flight together rather than one memory latency after another.
template <typename V, int MAXE, int NTH, typename Ld, typename St>
__device__ __forceinline__ void stage_batched(int count, int tid, Ld ld, St st) {
    V v[MAXE];
#pragma unroll
    for (int k = 0; k < MAXE; ++k) {
        const int i = tid + k * NTH;
        if (i < count) v[k] = ld(i);
    }
#pragma unroll
    for (int k = 0; k < MAXE; ++k) {
        const int i = tid + k * NTH;
        if (i < count) st(i, v[k]);
    }
}

// Every level is one launch of 2D tiles over all bases, both axes through LDS.  Each thread
// computes output pairs that read the same inputs: the lowpass and highpass coefficient at
// one position (analysis), or the even and odd sample from one window of coefficients
// (synthesis), so every LDS read feeds two outputs.
constexpr int AP = 16;                      // analysis tile: outputs per axis per subband (max)
constexpr int AR = 2 * AP + MAX_TAPS - 2;   // analysis tile: input rows/cols needed (max, even)
constexpr int SP = 32;                      // synthesis tile: outputs per axis (max)
constexpr int SC = SP / 2 + MAX_TAPS / 2 - 1;   // synthesis window per axis per subband (max)

// One analysis level on a tile: coefficients at positions [ap ti1, ap ti1 + ap) x
// [ap ti2, ...) of all four subbands of the Ls x Ls block (ap = min(AP, Ls/2)), from the
// (2 ap + F - 2)^2 input window starting at (2 ap ti1, 2 ap ti2) (periodic).  Axis 1 is
// filtered first, then axis 0.  Window rows are stored even samples first, then odd, so
// lanes with consecutive outputs read consecutive LDS words.  src: the image (level 0,
// shared by all bases, times `scale`; src_bstride = 0) or the previous level's LL blocks
// (compact slots).  Detail subbands go to the alpha block; the LL subband goes to `llout`
// (compact slots of (n/2)^2 per basis, row stride Ls/2), or into the alpha block at the
// coarsest level (llout == null), so no launch reads what it writes.  blockIdx.z == nwav
// copies the image into the Dirac block instead.
// XHAT (finest level only): the image is x + a p with a the CG step length from xa's partial
// sums, formed as the window is read.
template <typename T, bool XHAT>
__global__ void __launch_bounds__(256)
k_wav_fwd_level(const cpx<T>* __restrict__ src, size_t src_bstride, int src_ld, cpx<T>* __restrict__ alpha,
                cpx<T>* __restrict__ llout, const T* __restrict__ filt, WavArgs A, int Ls, T scale,
                XhatArgs<T> xa) {
    constexpr int IS = AR + 1, MS = 2 * AP + 1;
    __shared__ cpx<T> in[AR * IS];
    __shared__ cpx<T> mid[AR * MS];
    __shared__ T tp[2 * MAX_TAPS];
    const int n = A.n;
    const size_t N = (size_t)n * n;
    const int half = Ls >> 1;
    const int ap = half < AP ? half : AP;
    const int tiles = half / ap;
    const int ti1 = blockIdx.x / tiles, ti2 = blockIdx.x % tiles;
    const int r0 = 2 * ap * ti1, c0 = 2 * ap * ti2;
    const int z = blockIdx.z;
    T xs = 0;
    if constexpr (XHAT) xs = cg_alpha<T>(xa.rho_part, xa.rho_count, xa.pq_part, xa.pq_count);
    // image element at offset o (x + a p with XHAT)
    auto img = [&](size_t o) {
        if constexpr (XHAT) return src[o] + xs * xa.p[o];
        else return src[o];
    };
    if (z == A.nwav) {
        cpx<T>* d = alpha + (size_t)A.dirac_block * N;
        const SmallDiv d2a(2 * ap);
        auto at = [&](int i) {
            int c;
            const int r = d2a.quot(i, c);
            return (size_t)(r0 + r) * n + c0 + c;
        };
        stage_batched<cpx<T>, 4 * AP * AP / 256, 256>(
            4 * ap * ap, threadIdx.x, [&](int i) { return img(at(i)); },
            [&](int i, cpx<T> v) { d[at(i)] = scale * v; });
        return;
    }
    const size_t blk = (size_t)A.block[z] * N;
    const cpx<T>* s = src + (size_t)z * src_bstride;
    const int F = A.flen[z];
    const int R = 2 * ap + F - 2, RH = R >> 1;
    const SmallDiv dR(R), da(ap), d2a(2 * ap);
    // the taps and the window (R <= AR) are loaded together, then stored to LDS
    const T tap = threadIdx.x < 2 * MAX_TAPS ? filt[z * 2 * MAX_TAPS + threadIdx.x] : (T)0;
    stage_batched<cpx<T>, (AR * AR + 255) / 256, 256>(
        R * R, threadIdx.x,
        [&](int i) {
            int b;
            const int a = dR.quot(i, b);
            const size_t o = (size_t)((r0 + a) & (Ls - 1)) * src_ld + ((c0 + b) & (Ls - 1));
            if constexpr (XHAT) return img(o);
            else return s[o];
        },
        [&](int i, cpx<T> v) {
            int b;
            const int a = dR.quot(i, b);
            in[a * IS + (b & 1) * RH + (b >> 1)] = v;
        });
    if (threadIdx.x < 2 * MAX_TAPS) tp[threadIdx.x] = tap;
    __syncthreads();
    // axis 1: window row a, position oi -> mid[a][oi] (low), mid[a][ap + oi] (high)
    for (int i = threadIdx.x; i < R * ap; i += 256) {
        int oi;
        const int a = da.quot(i, oi);
        const cpx<T>* row = in + a * IS + oi;
        T lx = 0, ly = 0, hx = 0, hy = 0;
#pragma unroll
        for (int k = 0; k < MAX_TAPS; ++k) {
            if (k >= F) break;
            const cpx<T> v = row[(k & 1) * RH + (k >> 1)];
            const T h = tp[k], g = tp[MAX_TAPS + k];
            lx += h * v.x;
            ly += h * v.y;
            hx += g * v.x;
            hy += g * v.y;
        }
        mid[a * MS + oi] = mk<T>(lx, ly);
        mid[a * MS + ap + oi] = mk<T>(hx, hy);
    }
    __syncthreads();
    // axis 0: position oi, column o1 (low | high along axis 1) -> both axis-0 subbands
    for (int i = threadIdx.x; i < 2 * ap * ap; i += 256) {
        int o1;
        const int oi = d2a.quot(i, o1);
        const cpx<T>* col = mid + 2 * oi * MS + o1;
        T lx = 0, ly = 0, hx = 0, hy = 0;
#pragma unroll
        for (int k = 0; k < MAX_TAPS; ++k) {
            if (k >= F) break;
            const cpx<T> v = col[k * MS];
            const T h = tp[k], g = tp[MAX_TAPS + k];
            lx += h * v.x;
            ly += h * v.y;
            hx += g * v.x;
            hy += g * v.y;
        }
        const int row = ap * ti1 + oi;
        const int cl = (o1 >= ap ? half + o1 - ap : o1) + ap * ti2;
        if (o1 < ap && llout) llout[(size_t)z * (N / 4) + (size_t)row * half + cl] = mk<T>(scale * lx, scale * ly);
        else alpha[blk + (size_t)row * n + cl] = mk<T>(scale * lx, scale * ly);
        alpha[blk + (size_t)(half + row) * n + cl] = mk<T>(scale * hx, scale * hy);
    }
}

// The finest analysis level of every basis at once: all bases read the same image window,
// so a workgroup loads the (2 AP + Fmax - 2)^2 window of its tile once (polyphase rows, as
// above) and runs each basis' two axis passes on it in turn, instead of each basis' own
// workgroup re-reading the image.  The Dirac block is the scaled tile of the image.
template <typename T>
__global__ void __launch_bounds__(256)
k_wav_fwd_level0_all(const cpx<T>* __restrict__ x, cpx<T>* __restrict__ alpha, cpx<T>* __restrict__ llout,
                     const T* __restrict__ filt, WavArgs A, T scale, int Fmax) {
    constexpr int IS = AR + 1, MS = 2 * AP + 1;
    __shared__ cpx<T> in[AR * IS];
    __shared__ cpx<T> mid[AR * MS];
    __shared__ T tp[MAX_WAV][2 * MAX_TAPS];
    const int n = A.n, Ls = n;
    const size_t N = (size_t)n * n;
    const int half = Ls >> 1;
    const int tiles = half / AP;
    const int ti1 = blockIdx.x / tiles, ti2 = blockIdx.x % tiles;
    const int r0 = 2 * AP * ti1, c0 = 2 * AP * ti2;
    const int R = 2 * AP + Fmax - 2, RH = R >> 1;
    const SmallDiv dR(R);
    // the taps of every basis (at most 256 values) and the window are loaded together
    const T tap = threadIdx.x < A.nwav * 2 * MAX_TAPS ? filt[threadIdx.x] : (T)0;
    stage_batched<cpx<T>, (AR * AR + 255) / 256, 256>(
        R * R, threadIdx.x,
        [&](int i) {
            int b;
            const int a = dR.quot(i, b);
            return x[(size_t)((r0 + a) & (Ls - 1)) * n + ((c0 + b) & (Ls - 1))];
        },
        [&](int i, cpx<T> v) {
            int b;
            const int a = dR.quot(i, b);
            in[a * IS + (b & 1) * RH + (b >> 1)] = v;
        });
    if (threadIdx.x < A.nwav * 2 * MAX_TAPS) tp[threadIdx.x / (2 * MAX_TAPS)][threadIdx.x % (2 * MAX_TAPS)] = tap;
    if (A.dirac_block >= 0) {
        cpx<T>* d = alpha + (size_t)A.dirac_block * N;
        auto at = [&](int i) { return (size_t)(r0 + i / (2 * AP)) * n + c0 + i % (2 * AP); };
        stage_batched<cpx<T>, 4 * AP * AP / 256, 256>(
            4 * AP * AP, threadIdx.x, [&](int i) { return x[at(i)]; },
            [&](int i, cpx<T> v) { d[at(i)] = scale * v; });
    }
    __syncthreads();
    for (int z = 0; z < A.nwav; ++z) {
        const size_t blk = (size_t)A.block[z] * N;
        const int F = A.flen[z];
        const int Rz = 2 * AP + F - 2;   // this basis uses the window's first Rz rows / cols
        const T* h = tp[z];
        const T* g = h + MAX_TAPS;
        for (int i = threadIdx.x; i < Rz * AP; i += 256) {
            const int a = i / AP, oi = i - a * AP;
            const cpx<T>* row = in + a * IS + oi;
            T lx = 0, ly = 0, hx = 0, hy = 0;
#pragma unroll
            for (int k = 0; k < MAX_TAPS; ++k) {
                if (k >= F) break;
                const cpx<T> v = row[(k & 1) * RH + (k >> 1)];
                lx += h[k] * v.x;
                ly += h[k] * v.y;
                hx += g[k] * v.x;
                hy += g[k] * v.y;
            }
            mid[a * MS + oi] = mk<T>(lx, ly);
            mid[a * MS + AP + oi] = mk<T>(hx, hy);
        }
        __syncthreads();
        for (int i = threadIdx.x; i < 2 * AP * AP; i += 256) {
            const int oi = i / (2 * AP), o1 = i - oi * (2 * AP);
            const cpx<T>* col = mid + 2 * oi * MS + o1;
            T lx = 0, ly = 0, hx = 0, hy = 0;
#pragma unroll
            for (int k = 0; k < MAX_TAPS; ++k) {
                if (k >= F) break;
                const cpx<T> v = col[k * MS];
                lx += h[k] * v.x;
                ly += h[k] * v.y;
                hx += g[k] * v.x;
                hy += g[k] * v.y;
            }
            const int row = AP * ti1 + oi;
            const int cl = (o1 >= AP ? half + o1 - AP : o1) + AP * ti2;
            if (o1 < AP && llout) llout[(size_t)z * (N / 4) + (size_t)row * half + cl] = mk<T>(scale * lx, scale * ly);
            else alpha[blk + (size_t)row * n + cl] = mk<T>(scale * lx, scale * ly);
            alpha[blk + (size_t)(half + row) * n + cl] = mk<T>(scale * hx, scale * hy);
        }
        __syncthreads();
    }
}

// Synthesis of one level on a po x po output tile (po = min(SP, Ls)) of one basis: the
// window of the four subbands the tile reaches (po/2 + F/2 - 1 positions per axis per
// subband, periodic) goes into `in`, axis 0 is undone into `mid`, then axis 1; the thread's
// outputs (pairs of adjacent samples along axis 1) are returned through `emit`.
// Window layout: rows [0, C) lowpass and [C, 2C) highpass along axis 0, columns likewise.
// synth_tile loads the window and runs synth_axis0 and synth_axis1; the finest-level kernel
// that prefetches the next basis uses synth_load (the window into registers) and
// synth_store (registers into `in`) instead.
template <typename T, int NTH, int CMAX>
struct SynthWin {
    static constexpr int WS = 2 * CMAX + 1;   // LDS row stride of `in` and `mid`
    static constexpr int E = (4 * CMAX * CMAX + NTH - 1) / NTH;   // window elements a thread
    cpx<T> v[E];
    T tap;
};

template <typename T, int NTH, int CMAX>
__device__ __forceinline__ void synth_load(SynthWin<T, NTH, CMAX>& w, const cpx<T>* __restrict__ alpha, size_t blk,
                                           const cpx<T>* __restrict__ lls, int lld, int n, int half, int po,
                                           int m0, int m1, int F, const T* __restrict__ ftaps, int tid) {
    const int C = po / 2 + F / 2 - 1;
    const SmallDiv d2c(2 * C);
    const int s0 = m0 / 2 - F / 2 + 1, s1 = m1 / 2 - F / 2 + 1;   // first window index
    w.tap = tid < 2 * MAX_TAPS ? ftaps[tid] : (T)0;
#pragma unroll
    for (int k = 0; k < SynthWin<T, NTH, CMAX>::E; ++k) {
        const int i = tid + k * NTH;
        if (i < 4 * C * C) {
            int v;
            const int u = d2c.quot(i, v);
            const bool h0 = u >= C, h1 = v >= C;
            const int i0 = (s0 + (h0 ? u - C : u)) & (half - 1), i1 = (s1 + (h1 ? v - C : v)) & (half - 1);
            w.v[k] = (!h0 && !h1) ? lls[(size_t)i0 * lld + i1]
                                  : alpha[blk + (size_t)(i0 + (h0 ? half : 0)) * n + i1 + (h1 ? half : 0)];
        }
    }
}

template <typename T, int NTH, int CMAX>
__device__ __forceinline__ void synth_store(const SynthWin<T, NTH, CMAX>& w, int po, int F, T* tp, cpx<T>* in,
                                            int tid) {
    constexpr int WS = SynthWin<T, NTH, CMAX>::WS;
    const int C = po / 2 + F / 2 - 1;
    const SmallDiv d2c(2 * C);
#pragma unroll
    for (int k = 0; k < SynthWin<T, NTH, CMAX>::E; ++k) {
        const int i = tid + k * NTH;
        if (i < 4 * C * C) {
            int v;
            const int u = d2c.quot(i, v);
            in[u * WS + v] = w.v[k];
        }
    }
    if (tid < 2 * MAX_TAPS) tp[tid] = w.tap;
}

// undo axis 0: output rows 2j, 2j+1 (j = m0/2 + jr) for every window column v
template <typename T, int NTH, int CMAX>
__device__ __forceinline__ void synth_axis0(int po, int F, const T* tp, const cpx<T>* in, cpx<T>* mid, int tid) {
    constexpr int WS = SynthWin<T, NTH, CMAX>::WS;
    const int C = po / 2 + F / 2 - 1;
    const int hp = po / 2;
    const SmallDiv d2c(2 * C);
    for (int i = tid; i < hp * 2 * C; i += NTH) {
        int v;
        const int jr = d2c.quot(i, v);
        T ex = 0, ey = 0, ox = 0, oy = 0;
#pragma unroll
        for (int t = 0; t < MAX_TAPS / 2; ++t) {
            if (2 * t >= F) break;
            const int u = jr + F / 2 - 1 - t;   // window row of index j - t
            const cpx<T> lo = in[u * WS + v], hv = in[(C + u) * WS + v];
            const T he = tp[2 * t], ge = tp[MAX_TAPS + 2 * t];
            const T ho = tp[2 * t + 1], go = tp[MAX_TAPS + 2 * t + 1];
            // one fused multiply-add a product (the sum of the pair first costs a multiply,
            // an FMA and an add)
            ex = fma_(he, lo.x, ex);
            ex = fma_(ge, hv.x, ex);
            ey = fma_(he, lo.y, ey);
            ey = fma_(ge, hv.y, ey);
            ox = fma_(ho, lo.x, ox);
            ox = fma_(go, hv.x, ox);
            oy = fma_(ho, lo.y, oy);
            oy = fma_(go, hv.y, oy);
        }
        mid[(2 * jr) * WS + v] = mk<T>(ex, ey);
        mid[(2 * jr + 1) * WS + v] = mk<T>(ox, oy);
    }
}

// undo axis 1: row r, output columns 2j, 2j+1 (a thread's k-th pair is i = tid + k NTH;
// the unrolled k is a compile-time index for the caller's accumulators)
template <typename T, int NTH, int CMAX, typename Emit>
__device__ __forceinline__ void synth_axis1(int po, int F, const T* tp, const cpx<T>* mid, int tid, Emit emit) {
    constexpr int WS = SynthWin<T, NTH, CMAX>::WS;
    const int C = po / 2 + F / 2 - 1;
    const int hp = po / 2;
    constexpr int PMAX = CMAX - MAX_TAPS / 2 + 1;          // largest po / 2
    constexpr int KMAX = (2 * PMAX * PMAX + NTH - 1) / NTH;
    const SmallDiv dh(hp);
#pragma unroll
    for (int k = 0; k < KMAX; ++k) {
        const int i = tid + k * NTH;
        if (i >= po * hp) break;
        int jc;
        const int r = dh.quot(i, jc);
        T ex = 0, ey = 0, ox = 0, oy = 0;
#pragma unroll
        for (int t = 0; t < MAX_TAPS / 2; ++t) {
            if (2 * t >= F) break;
            const int v = jc + F / 2 - 1 - t;
            const cpx<T> lo = mid[r * WS + v], hv = mid[r * WS + C + v];
            const T he = tp[2 * t], ge = tp[MAX_TAPS + 2 * t];
            const T ho = tp[2 * t + 1], go = tp[MAX_TAPS + 2 * t + 1];
            // one fused multiply-add a product (the sum of the pair first costs a multiply,
            // an FMA and an add)
            ex = fma_(he, lo.x, ex);
            ex = fma_(ge, hv.x, ex);
            ey = fma_(he, lo.y, ey);
            ey = fma_(ge, hv.y, ey);
            ox = fma_(ho, lo.x, ox);
            ox = fma_(go, hv.x, ox);
            oy = fma_(ho, lo.y, oy);
            oy = fma_(go, hv.y, oy);
        }
        emit(k, r, 2 * jc, mk<T>(ex, ey), mk<T>(ox, oy));
    }
}

template <typename T, int NTH, int CMAX, typename Emit>
__device__ __forceinline__ void synth_tile(const cpx<T>* __restrict__ alpha, size_t blk, const cpx<T>* __restrict__ lls,
                                          int lld, int n, int half, int po, int m0, int m1, int F,
                                          const T* __restrict__ ftaps, T* tp, cpx<T>* in, cpx<T>* mid, int tid,
                                          Emit emit) {
    constexpr int WS = SynthWin<T, NTH, CMAX>::WS;
    const int C = po / 2 + F / 2 - 1;
    const SmallDiv d2c(2 * C);
    const int s0 = m0 / 2 - F / 2 + 1, s1 = m1 / 2 - F / 2 + 1;   // first window index
    // the basis' taps (ftaps, into tp) and the window (C <= CMAX) are loaded together, then
    // stored to LDS
    const T tap = tid < 2 * MAX_TAPS ? ftaps[tid] : (T)0;
    stage_batched<cpx<T>, (4 * CMAX * CMAX + NTH - 1) / NTH, NTH>(
        4 * C * C, tid,
        [&](int i) {
            int v;
            const int u = d2c.quot(i, v);
            const bool h0 = u >= C, h1 = v >= C;
            const int i0 = (s0 + (h0 ? u - C : u)) & (half - 1), i1 = (s1 + (h1 ? v - C : v)) & (half - 1);
            return (!h0 && !h1) ? lls[(size_t)i0 * lld + i1]
                                : alpha[blk + (size_t)(i0 + (h0 ? half : 0)) * n + i1 + (h1 ? half : 0)];
        },
        [&](int i, cpx<T> val) {
            int v;
            const int u = d2c.quot(i, v);
            in[u * WS + v] = val;
        });
    if (tid < 2 * MAX_TAPS) tp[tid] = tap;
    __syncthreads();
    synth_axis0<T, NTH, CMAX>(po, F, tp, in, mid, tid);
    __syncthreads();
    synth_axis1<T, NTH, CMAX>(po, F, tp, mid, tid, emit);
}

// One synthesis level (output side Ls, level >= 1) for every basis (blockIdx.z): the
// coarser LL comes from `llin` (compact slots of (n/2)^2 per basis) or, at the coarsest
// level, from the alpha block; the result goes to `out` (compact slots, row stride Ls).
template <typename T>
__global__ void __launch_bounds__(256)
k_wav_inv_level(const cpx<T>* __restrict__ alpha, const cpx<T>* __restrict__ llin, int ll_from_alpha,
                cpx<T>* __restrict__ out, const T* __restrict__ filt, WavArgs A, int Ls) {
    constexpr int WS = 2 * SC + 1;
    __shared__ cpx<T> in[2 * SC * WS];
    __shared__ cpx<T> mid[SP * WS];
    __shared__ T tp[2 * MAX_TAPS];
    const int n = A.n;
    const size_t N = (size_t)n * n;
    const int half = Ls >> 1;
    const int po = Ls < SP ? Ls : SP;
    const int tiles = Ls / po;
    const int m0 = po * (blockIdx.x / tiles), m1 = po * (blockIdx.x % tiles);
    const int z = blockIdx.z;
    const size_t blk = (size_t)A.block[z] * N;
    const cpx<T>* lls = ll_from_alpha ? alpha + blk : llin + (size_t)z * (N / 4);
    const int lld = ll_from_alpha ? n : half;
    cpx<T>* o = out + (size_t)z * (N / 4);
    synth_tile<T, 256, SC>(alpha, blk, lls, lld, n, half, po, m0, m1, A.flen[z], filt + z * 2 * MAX_TAPS, tp, in,
                           mid, (int)threadIdx.x,
                       [&](int, int r, int c, cpx<T> e, cpx<T> od) {
                           o[(size_t)(m0 + r) * Ls + m1 + c] = e;
                           o[(size_t)(m0 + r) * Ls + m1 + c + 1] = od;
                       });
}

// Finest synthesis level: an FP x FP image tile sums every basis plus the Dirac block, times
// `scale`.  NSLOT groups of 256 threads synthesise different bases concurrently and their
// partial sums are added in slot order (a fixed order: deterministic).
template <typename T, int FP, int NSLOT>
__global__ void __launch_bounds__(256 * NSLOT)
k_wav_inv_final(const cpx<T>* __restrict__ alpha, const cpx<T>* __restrict__ llin, int ll_from_alpha,
                cpx<T>* __restrict__ x, const T* __restrict__ filt, WavArgs A, T scale) {
    constexpr int CF = FP / 2 + MAX_TAPS / 2 - 1;
    constexpr int WS = 2 * CF + 1;
    constexpr int PAIRS = (FP * FP / 2 + 255) / 256;   // output pairs per thread
    __shared__ cpx<T> in[NSLOT][2 * CF * WS];
    __shared__ cpx<T> mid[NSLOT][FP * WS];
    __shared__ T tp[NSLOT][2 * MAX_TAPS];
    __shared__ cpx<T> part[NSLOT][FP * FP];
    const int n = A.n;
    const size_t N = (size_t)n * n;
    const int half = n >> 1;
    const int tiles = n / FP;
    const int m0 = FP * (blockIdx.x / tiles), m1 = FP * (blockIdx.x % tiles);
    const int slot = threadIdx.x >> 8, tid = threadIdx.x & 255;
    // thread tid owns the output pairs i = tid + 256 k: row i / (FP/2), columns 2 (i % (FP/2)) + {0, 1}
    cpx<T> acc0[PAIRS], acc1[PAIRS];
#pragma unroll
    for (int k = 0; k < PAIRS; ++k) acc0[k] = acc1[k] = mk<T>(0, 0);
    const int rounds = (A.nwav + NSLOT - 1) / NSLOT;
    for (int rd = 0; rd < rounds; ++rd) {
        const int z = rd * NSLOT + slot;
        const bool active = z < A.nwav;
        const int zz = active ? z : 0;
        const size_t blk = (size_t)A.block[zz] * N;
        const cpx<T>* lls = ll_from_alpha ? alpha + blk : llin + (size_t)zz * (N / 4);
        const int lld = ll_from_alpha ? n : half;
        if (rd > 0) __syncthreads();
        // inactive slots run on basis 0 and discard the result (keeps the barriers uniform)
        synth_tile<T, 256, CF>(alpha, blk, lls, lld, n, half, FP, m0, m1, A.flen[zz], filt + zz * 2 * MAX_TAPS,
                               tp[slot], in[slot], mid[slot], tid, [&](int k, int, int, cpx<T> e, cpx<T> od) {
                                   if (active) {
                                       acc0[k].x += e.x;
                                       acc0[k].y += e.y;
                                       acc1[k].x += od.x;
                                       acc1[k].y += od.y;
                                   }
                               });
    }
#pragma unroll
    for (int k = 0; k < PAIRS; ++k) {
        const int i = tid + 256 * k;
        if (i < FP * FP / 2) {
            const int r = i / (FP / 2), c = 2 * (i % (FP / 2));
            part[slot][r * FP + c] = acc0[k];
            part[slot][r * FP + c + 1] = acc1[k];
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < FP * FP; i += 256 * NSLOT) {
        const int r = i / FP, c = i % FP;
        const size_t o = (size_t)(m0 + r) * n + m1 + c;
        T sx = 0, sy = 0;
        if (A.dirac_block >= 0) {
            const cpx<T> d = alpha[(size_t)A.dirac_block * N + o];
            sx = d.x;
            sy = d.y;
        }
#pragma unroll
        for (int sl = 0; sl < NSLOT; ++sl) {
            sx += part[sl][i].x;
            sy += part[sl][i].y;
        }
        x[o] = mk<T>(scale * sx, scale * sy);
    }
}

// Finest synthesis level, one basis at a time per 256-thread workgroup, with the next basis'
// window loaded into registers while the current one is filtered: it is stored to `in` as
// soon as axis 0 of the current basis has read `in` (the taps are double-buffered), so its
// load latency hides behind the filtering.  Same arithmetic, in the same basis order, as
// k_wav_inv_final with one slot.
template <typename T, int FP>
__global__ void __launch_bounds__(256)
k_wav_inv_final_pipe(const cpx<T>* __restrict__ alpha, const cpx<T>* __restrict__ llin, int ll_from_alpha,
                     cpx<T>* __restrict__ x, const T* __restrict__ filt, WavArgs A, T scale) {
    constexpr int CF = FP / 2 + MAX_TAPS / 2 - 1;
    constexpr int WS = 2 * CF + 1;
    constexpr int PAIRS = (FP * FP / 2 + 255) / 256;   // output pairs per thread
    __shared__ cpx<T> in[2 * CF * WS];
    __shared__ cpx<T> mid[FP * WS];
    __shared__ T tp[2][2 * MAX_TAPS];
    const int n = A.n;
    const size_t N = (size_t)n * n;
    const int half = n >> 1;
    const int tiles = n / FP;
    const int m0 = FP * (blockIdx.x / tiles), m1 = FP * (blockIdx.x % tiles);
    const int tid = threadIdx.x;
    const int lld = ll_from_alpha ? n : half;
    auto blk_of = [&](int z) { return (size_t)A.block[z] * N; };
    auto lls_of = [&](int z) { return ll_from_alpha ? alpha + blk_of(z) : llin + (size_t)z * (N / 4); };
    cpx<T> acc0[PAIRS], acc1[PAIRS];
#pragma unroll
    for (int k = 0; k < PAIRS; ++k) acc0[k] = acc1[k] = mk<T>(0, 0);
    SynthWin<T, 256, CF> w;
    synth_load<T, 256, CF>(w, alpha, blk_of(0), lls_of(0), lld, n, half, FP, m0, m1, A.flen[0], filt, tid);
    synth_store<T, 256, CF>(w, FP, A.flen[0], tp[0], in, tid);
    __syncthreads();
    for (int z = 0; z < A.nwav; ++z) {
        const int F = A.flen[z];
        const bool more = z + 1 < A.nwav;
        if (more)
            synth_load<T, 256, CF>(w, alpha, blk_of(z + 1), lls_of(z + 1), lld, n, half, FP, m0, m1, A.flen[z + 1],
                                   filt + (z + 1) * 2 * MAX_TAPS, tid);
        synth_axis0<T, 256, CF>(FP, F, tp[z & 1], in, mid, tid);
        __syncthreads();
        if (more) synth_store<T, 256, CF>(w, FP, A.flen[z + 1], tp[(z + 1) & 1], in, tid);
        synth_axis1<T, 256, CF>(FP, F, tp[z & 1], mid, tid, [&](int k, int, int, cpx<T> e, cpx<T> od) {
            acc0[k].x += e.x;
            acc0[k].y += e.y;
            acc1[k].x += od.x;
            acc1[k].y += od.y;
        });
        __syncthreads();
    }
    // each thread adds the Dirac block to its own output pairs and writes them
#pragma unroll
    for (int k = 0; k < PAIRS; ++k) {
        const int i = tid + 256 * k;
        if (i < FP * FP / 2) {
            const int r = i / (FP / 2), c = 2 * (i % (FP / 2));
            const size_t o = (size_t)(m0 + r) * n + m1 + c;
            cpx<T> e = acc0[k], od = acc1[k];
            if (A.dirac_block >= 0) {
                const cpx<T>* d = alpha + (size_t)A.dirac_block * N + o;
                e = e + d[0];
                od = od + d[1];
            }
            x[o] = scale * e;
            x[o + 1] = scale * od;
        }
    }
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

// The finest level goes through k_wav_fwd_level (which can form x + alpha p) unless the
// image is large enough for the one-pass kernel of all bases.
bool psi_adj_takes_xhat(const Plan& P) {
    if (P.nwav == 0) return false;
    const int ap = std::min(AP, P.n / 2), tiles = (P.n / 2) / ap;
    return !(ap == AP && tiles * tiles >= 1024);
}

template <typename T>
void launch_psi_adj(const Plan& P, const cpx<T>* x, cpx<T>* alpha, hipStream_t s, const XhatArgs<T>* xa,
                    hipEvent_t first_done) {
    if (xa && !psi_adj_takes_xhat(P)) return;   // callers check psi_adj_takes_xhat first
    const WavArgs A = wav_args(P);
    const T scale = (T)(1.0 / std::sqrt((double)P.q));
    const int64_t N = P.N;
    if (P.nwav == 0) {
        hipLaunchKernelGGL(k_scale_copy_c<T>, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, x,
                           alpha, scale, N);
        return;
    }
    const T* filt = (const T*)P.filters;
    const int ztot = P.nwav + (P.has_dirac ? 1 : 0);
    // LL ping-pong buffers, one (n/2)^2 slot per basis each
    cpx<T>* llb[2] = {(cpx<T>*)P.ws2, (cpx<T>*)P.ws2 + (size_t)P.nwav * (N / 4)};
    for (int lev = 0; lev < P.levels; ++lev) {
        const int Ls = P.n >> lev;
        const int half = Ls / 2, ap = std::min(AP, half);
        const int tiles = half / ap;
        const dim3 g(tiles * tiles, 1, lev == 0 ? ztot : P.nwav);
        cpx<T>* llout = lev + 1 < P.levels ? llb[lev & 1] : nullptr;
        // large images: one pass over the image for all bases (small ones need the bases'
        // separate workgroups to fill the device)
        if (lev == 0 && ap == AP && tiles * tiles >= 1024) {
            int Fmax = 2;
            for (int i = 0; i < P.nwav; ++i) Fmax = std::max(Fmax, A.flen[i]);
            hipLaunchKernelGGL(k_wav_fwd_level0_all<T>, dim3(tiles * tiles), dim3(256), 0, s, x, alpha, llout,
                               filt, A, scale, Fmax);
        } else if (lev == 0 && xa) {
            hipLaunchKernelGGL((k_wav_fwd_level<T, true>), g, dim3(256), 0, s, x, (size_t)0, P.n, alpha, llout,
                               filt, A, Ls, scale, *xa);
        } else if (lev == 0) {
            hipLaunchKernelGGL((k_wav_fwd_level<T, false>), g, dim3(256), 0, s, x, (size_t)0, P.n, alpha, llout,
                               filt, A, Ls, scale, XhatArgs<T>{});
        } else {
            hipLaunchKernelGGL((k_wav_fwd_level<T, false>), g, dim3(256), 0, s, (const cpx<T>*)llb[(lev - 1) & 1],
                               (size_t)(N / 4), Ls, alpha, llout, filt, A, Ls, (T)1, XhatArgs<T>{});
        }
        if (lev == 0 && first_done) (void)hipEventRecord(first_done, s);
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
    // LL ping-pong buffers, one (n/2)^2 slot per basis each
    cpx<T>* llb[2] = {(cpx<T>*)P.ws2, (cpx<T>*)P.ws2 + (size_t)P.nwav * (N / 4)};
    int cur = -1;   // buffer holding the current LL, -1: the alpha block (coarsest level)
    for (int lev = P.levels - 1; lev >= 1; --lev) {
        const int Ls = P.n >> lev;
        const int po = std::min(SP, Ls);
        const int tiles = Ls / po;
        const int dst = cur == 0 ? 1 : 0;
        const cpx<T>* in = cur < 0 ? alpha : llb[cur];
        hipLaunchKernelGGL(k_wav_inv_level<T>, dim3(tiles * tiles, 1, P.nwav), dim3(256), 0, s, alpha, in,
                           cur < 0 ? 1 : 0, llb[dst], filt, A, Ls);
        cur = dst;
    }
    const cpx<T>* in = cur < 0 ? alpha : llb[cur];
    // FP32 on large images: 32 x 32 tiles (half the window overhead of 16 x 16), one basis
    // at a time per 256-thread workgroup with the next basis' window prefetched, so five
    // workgroups share a CU's LDS and loads overlap filtering (4096^2: 1321 -> 950 us for the
    // whole synthesis against four bases at a time in one 1024-thread workgroup)
    if constexpr (sizeof(T) == 4) {
        if (P.n >= 512) {
            const int tiles = P.n / 32;
            hipLaunchKernelGGL((k_wav_inv_final_pipe<T, 32>), dim3(tiles * tiles), dim3(256), 0, s, alpha, in,
                               cur < 0 ? 1 : 0, x, filt, A, scale);
            return;
        }
    }
    const int tiles = P.n / 16;
    hipLaunchKernelGGL((k_wav_inv_final<T, 16, 4>), dim3(tiles * tiles), dim3(1024), 0, s, alpha, in,
                       cur < 0 ? 1 : 0, x, filt, A, scale);
}

template void launch_psi_adj<float>(const Plan&, const cpx<float>*, cpx<float>*, hipStream_t,
                                    const XhatArgs<float>*, hipEvent_t);
template void launch_psi_adj<double>(const Plan&, const cpx<double>*, cpx<double>*, hipStream_t,
                                     const XhatArgs<double>*, hipEvent_t);
template void launch_psi<float>(const Plan&, const cpx<float>*, cpx<float>*, hipStream_t);
template void launch_psi<double>(const Plan&, const cpx<double>*, cpx<double>*, hipStream_t);

}  // namespace purify
