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


// Runtime-J variant of kb_weights (J <= 16), for the less common kernel widths.
template <typename T>
__device__ __noinline__ void kb_weights_any(const T* __restrict__ c, T f, T* w, int J) {
    constexpr int NC = KBDeg<T>::value + 1;
    const T x = f - (T)0.5;
#pragma unroll 1
    for (int a = 0; a < J; ++a) {
        T acc = c[a * NC + NC - 1];
#pragma unroll
        for (int k = NC - 2; k >= 0; --k) acc = acc * x + c[a * NC + k];
        w[a] = acc;
    }
}

// FP64 plans store every visibility's 2J tap weights (computed once at plan time) and the
// kernels read them; FP32 plans evaluate the per-tap polynomials on the fly (an FP64 table
// of 18 coefficients per tap does not fit in registers, and reading 16 B per tap weight
// from a cache-resident table is cheaper than re-evaluating it).
template <typename T, int J>
__device__ __forceinline__ void visibility_weights(const T* __restrict__ wtab, const T* __restrict__ kbc,
                                                   int idx, cpx<T> f, T* wa, T* wb, int Jr);

template <typename T, int J>
__device__ __forceinline__ void tap_weights(const T* __restrict__ c, T f, T* w, int Jr) {
    if constexpr (J > 0) kb_weights<T, J>(c, f, w);
    else kb_weights_any<T>(c, f, w, Jr);
}

template <typename T, int J>
__device__ __forceinline__ void visibility_weights(const T* __restrict__ wtab, const T* __restrict__ kbc,
                                                   int idx, cpx<T> f, T* wa, T* wb, int Jr) {
    if constexpr (sizeof(T) == 8) {
        const int Jn = J > 0 ? J : Jr;
        const T* w = wtab + (size_t)idx * 2 * Jn;
        if constexpr (J > 0) {
#pragma unroll
            for (int a = 0; a < J; ++a) {
                wa[a] = w[a];
                wb[a] = w[J + a];
            }
        } else {
            for (int a = 0; a < Jn; ++a) {
                wa[a] = w[a];
                wb[a] = w[Jn + a];
            }
        }
    } else {
        tap_weights<T, J>(kbc, f.x, wa, Jr);
        tap_weights<T, J>(kbc, f.y, wb, Jr);
    }
}

// sum_a wa[a] sum_b wb[b] G[k1 + a][k2 + b] (cyclic), the J x J gather of one visibility
template <typename T, int J>
__device__ __forceinline__ cpx<T> interpolate(const cpx<T>* __restrict__ grid, int k1, int k2, const T* wa,
                                              const T* wb, int K, int Jr) {
    constexpr int JJ = J > 0 ? J : KB_MAX_J;
    constexpr int UNR = J > 0 ? J : 1;
    const int Jn = J > 0 ? J : Jr;
    const int mask = K - 1;
    T ax = 0, ay = 0;
#pragma unroll UNR
    for (int a = 0; a < JJ; ++a) {
        if (a >= Jn) break;
        const cpx<T>* row = grid + (size_t)((k1 + a) & mask) * K;
        T rx = 0, ry = 0;
#pragma unroll UNR
        for (int bb = 0; bb < JJ; ++bb) {
            if (bb >= Jn) break;
            const cpx<T> g = row[(k2 + bb) & mask];
            rx += wb[bb] * g.x;
            ry += wb[bb] * g.y;
        }
        ax += wa[a] * rx;
        ay += wa[a] * ry;
    }
    return mk<T>(ax, ay);
}

// G: one thread per visibility (tile-sorted order), J x J gather from the row-major grid
// G[k1][k2].  J = 0: runtime Jr.
template <typename T, int J>
__global__ void __launch_bounds__(256)
k_degrid(const cpx<T>* __restrict__ grid, cpx<T>* __restrict__ y, const int32_t* __restrict__ perm,
         const int32_t* __restrict__ base, const T* __restrict__ frac, const T* __restrict__ kbc,
         const T* __restrict__ wtab, int M, int K, T scale, int Jr, const int32_t* __restrict__ chunks) {
    constexpr int JJ = J > 0 ? J : KB_MAX_J;
    int m;
    if (chunks) {   // strip-ordered chunk {first, count} of this workgroup
        if ((int)threadIdx.x >= chunks[2 * blockIdx.x + 1]) return;
        m = chunks[2 * blockIdx.x] + threadIdx.x;
    } else {
        m = blockIdx.x * 256 + threadIdx.x;
        if (m >= M) return;
    }
    const int b = base[m];
    const int k1 = b & 0xFFFF, k2 = (b >> 16) & 0xFFFF;
    const cpx<T> f = reinterpret_cast<const cpx<T>*>(frac)[m];
    T wa[JJ], wb[JJ];
    visibility_weights<T, J>(wtab, kbc, m, f, wa, wb, Jr);
    const cpx<T> v = interpolate<T, J>(grid, k1, k2, wa, wb, K, Jr);
    y[perm ? perm[m] : m] = mk<T>(scale * v.x, scale * v.y);
}

// G by tiles: one work unit of the gridding work list (a tile, or part of a heavy one) per
// workgroup; the unit's own visibilities (its shares of the tile's interior and spilling
// ranges; spill-ins belong to other tiles) interpolate from the (TT + J - 1)^2 window of the
// grid that holds all their footprints, staged once in LDS (FP64 with global_load_lds).  Each
// visibility is handled once; the strip-ordered work list keeps a unit on the XCD whose L2
// holds its grid columns.
template <typename T, int J, int TT, int NT>
__global__ void __launch_bounds__(NT)
k_degrid_tiles(const cpx<T>* __restrict__ grid, cpx<T>* __restrict__ y, const int32_t* __restrict__ perm,
               const int32_t* __restrict__ base, const T* __restrict__ frac, const T* __restrict__ kbc,
               const T* __restrict__ wtab, const int32_t* __restrict__ work, int K, int nT, T scale, int Jr) {
    constexpr int JJ = J > 0 ? J : KB_MAX_J;
    constexpr int UNR = J > 0 ? J : 1;
    constexpr int WS = TT + JJ - 1;
    constexpr int WPT = (WS * WS + NT - 1) / NT;
    constexpr bool DMA = sizeof(T) == 8;
    __shared__ cpx<T> win[WPT * NT];
    const int32_t* w = work + GRID_REC * blockIdx.x;
    const int tile = w[0];
    if (tile < 0) return;
    const int s0 = w[4], n0 = w[5] - w[4], s1 = w[6], total = n0 + (w[7] - w[6]);
    if (total == 0) return;
    const int t1o = (tile % nT) * TT, t2o = (tile / nT) * TT;
    const int mask = K - 1;
    const int Jn = J > 0 ? J : Jr;
    if constexpr (DMA) {
#pragma unroll
        for (int k = 0; k < WPT; ++k) {
            const int i = threadIdx.x + k * NT;
            if (i < WS * WS) {
                const cpx<T>* src = grid + (size_t)((t1o + i / WS) & mask) * K + ((t2o + i % WS) & mask);
                __builtin_amdgcn_global_load_lds(
                    (const void*)src, (__attribute__((address_space(3))) void*)(win + (threadIdx.x & ~63u) + k * NT),
                    16, 0, 0);
            }
        }
    } else {
        // WB of a thread's window elements are loaded before any is stored to LDS, so their
        // loads are in flight together
        constexpr int WB = WPT < 10 ? WPT : 10;
#pragma unroll
        for (int k0 = 0; k0 < WPT; k0 += WB) {
            cpx<T> t[WB];
#pragma unroll
            for (int kk = 0; kk < WB; ++kk) {
                const int i = threadIdx.x + (k0 + kk) * NT;
                if (k0 + kk < WPT && i < WS * WS)
                    t[kk] = grid[(size_t)((t1o + i / WS) & mask) * K + ((t2o + i % WS) & mask)];
            }
#pragma unroll
            for (int kk = 0; kk < WB; ++kk) {
                const int i = threadIdx.x + (k0 + kk) * NT;
                if (k0 + kk < WPT && i < WS * WS) win[i] = t[kk];
            }
        }
    }
    __syncthreads();
    for (int j = threadIdx.x; j < total; j += NT) {
        const int idx = j < n0 ? s0 + j : s1 + (j - n0);
        const int bk = base[idx];
        const cpx<T> f = reinterpret_cast<const cpx<T>*>(frac)[idx];
        T wa[JJ], wb[JJ];
        visibility_weights<T, J>(wtab, kbc, idx, f, wa, wb, Jr);
        const cpx<T>* w0 = win + (((bk & 0xFFFF) - t1o) & mask) * WS + ((((bk >> 16) & 0xFFFF) - t2o) & mask);
        T ax = 0, ay = 0;
        auto tap_row = [&](int a) {
            const cpx<T>* row = w0 + a * WS;
            T rx = 0, ry = 0;
#pragma unroll UNR
            for (int bb = 0; bb < JJ; ++bb) {
                if (bb >= Jn) break;
                const cpx<T> g = row[bb];
                rx += wb[bb] * g.x;
                ry += wb[bb] * g.y;
            }
            ax += wa[a] * rx;
            ay += wa[a] * ry;
        };
        // FP64 and J = 8: two rows at a time, so the window reads of all J rows are not all
        // held in registers at once (158 -> 65 VGPRs at J = 8, four workgroups a CU instead
        // of three: 4096^2 G 233 -> 220 us; FP64 256^2 4.0 -> 3.4 us); FP32 with J <= 6 keeps
        // the fully unrolled form (1024^2 G 26.8 against 30.0 us)
        if constexpr (sizeof(T) == 8 || J == 8) {
#pragma unroll 2
            for (int a = 0; a < JJ; ++a) {
                if (a >= Jn) break;
                tap_row(a);
            }
        } else {
#pragma unroll UNR
            for (int a = 0; a < JJ; ++a) {
                if (a >= Jn) break;
                tap_row(a);
            }
        }
        y[perm ? perm[idx] : idx] = mk<T>(scale * ax, scale * ay);
    }
}

// Gridding accumulates in LDS with integer atomics on a fixed-point representation:
// contributions are scaled by an exact power of two per tile and rounded to int32 (FP32
// path) or int64 (FP64 path).  Integer addition is associative, so the result does not
// depend on the order in which lanes and waves add (bit-reproducible gridding), and LDS
// integer atomics run at full rate.  The scale is chosen from the tile's largest |y| and
// the plan's bound on how many visibilities cover one cell of the tile, so no sum can
// overflow:  |cell| <= cover * max|y| * max psi^2 <= 2^(bits-2) quanta, and no single
// contribution reaches 2^(CBITS-1) quanta.  A contribution w * v is rounded to an integer
// by one fused multiply-add onto 1.5 * 2^(mantissa bits): the sum then lies in a binade
// whose unit is one quantum, so its low mantissa bits hold round(w v) in two's complement.
template <typename T> struct FixedAcc;
template <> struct FixedAcc<float> {
    using I = int;
    static constexpr int BITS = 30;   // bound on a cell sum, in quanta
    static constexpr int CBITS = 22;  // bound on one contribution, in quanta
    static __device__ __forceinline__ I conv_mul(float a, float b) {
        return __float_as_int(fmaf(a, b, 12582912.0f)) - 0x4B400000;
    }
};
template <> struct FixedAcc<double> {
    using I = long long;
    static constexpr int BITS = 62;
    static constexpr int CBITS = 51;
    static __device__ __forceinline__ I conv_mul(double a, double b) {
        return __double_as_longlong(fma(a, b, 6755399441055744.0)) - 0x4338000000000000LL;
    }
};

template <typename T>
__device__ __forceinline__ void lds_add(typename FixedAcc<T>::I* p, typename FixedAcc<T>::I v) {
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// FP32 path: the real and imaginary int32 sums of a cell share one 64-bit word, real part
// in the high half, so one 64-bit LDS atomic adds both.  Addition mod 2^64 gives
// word = R 2^32 + I exactly; as |I| < 2^31 (the scale bound above), the low half read as
// int32 is I, and (word - I) / 2^32 read as int32 is R.
__device__ __forceinline__ unsigned long long pack_pair(int re, int im) {
    return ((unsigned long long)(unsigned)re << 32) + (unsigned long long)(long long)im;
}
__device__ __forceinline__ void unpack_pair(unsigned long long w, int& re, int& im) {
    im = (int)(unsigned)w;
    re = (int)(unsigned)((w - (unsigned long long)(long long)im) >> 32);
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    return v;
}

// G^T: one work unit per workgroup.  A unit is a TT x TT tile, or one part of a heavy tile
// whose visibility list was split over several workgroups.  Its visibility passes (its share
// of the tile's own visibilities and of the three neighbours' spill-ins) form one item list;
// each thread takes a contiguous chunk (so the lanes of a wave add to different cells) and
// loads CHR items at a time -- coordinates, weights and values -- before adding any, so the
// loads of a chunk overlap.  Contributions accumulate in LDS in fixed point (integer
// atomics: the sum does not depend on the order of the adds) on the tile plus a margin of
// J - 1 cells on every side: every item's J x J footprint lies inside that padded tile, so
// the scatter adds all J^2 taps at fixed offsets from one base address with no bounds
// tests (taps that fall in the margin belong to neighbouring tiles and are discarded).  A
// whole tile is written to the grid; a part stores its integer partial tile and scale
// exponent in its own slot, and k_grid_merge sums the parts of each split tile in part
// order.  The real and imaginary parts accumulate in separate planes, so the lanes of one
// add instruction spread over all LDS banks.
//
// GTG: the unit's visibility values are not read from y but interpolated from the grid
// `gin` (the same J x J gather as G), so one launch applies G^T G (gin and grid distinct).
//
// Coordinates relative to the tile: r0 = ((k1 - t1o + J - 1) mod K) - (J - 1) lies in
// [-(J - 1), TT) for the unit's items (own items start inside the tile, spill-ins at most
// J - 1 cells before it); this needs K >= TT + J - 1, which the plan guarantees.
template <typename T, int J, int TT, int NT, int CHR, bool GTG>
__global__ void __launch_bounds__(NT)
k_grid(const cpx<T>* __restrict__ y, const cpx<T>* __restrict__ gin, const int32_t* __restrict__ perm, const int32_t* __restrict__ base,
       const T* __restrict__ frac, const T* __restrict__ kbc, const T* __restrict__ wtab,
       const int32_t* __restrict__ work, typename FixedAcc<T>::I* __restrict__ partial,
       int32_t* __restrict__ pexp, cpx<T>* __restrict__ grid, int K, int nT, int Jr) {
    using Acc = FixedAcc<T>;
    constexpr int JJ = J > 0 ? J : KB_MAX_J;
    constexpr int UNR = J > 0 ? J : 1;
    constexpr int JM = JJ - 1;           // margin of the padded accumulator tile
    constexpr int WA = TT + 2 * JM;      // padded accumulator side
    // GTG: window of gin covering every footprint of the unit's visibilities (own and
    // spill-in), rows/cols [tile origin - (J-1), tile end + J - 1)
    constexpr int WS = TT + 2 * (JJ - 1);
    constexpr int WPT = (WS * WS + NT - 1) / NT;
    // FP64: the window goes straight from global memory to LDS (global_load_lds, one 16-byte
    // element per lane at consecutive LDS slots of the wave), keeping it out of registers
    constexpr bool DMA = GTG && sizeof(T) == 8;
    // FP32: one 64-bit word per cell holding both parts; FP64: a real and an imaginary plane
    constexpr bool PACK = sizeof(T) == 4;
    __shared__ __attribute__((aligned(8))) typename Acc::I acc[2 * WA * WA];
    unsigned long long* accp = reinterpret_cast<unsigned long long*>(acc);
    __shared__ double red[NT / 64];
    __shared__ cpx<T> win[GTG ? WPT * NT : 1];
    const int32_t* w = work + GRID_REC * blockIdx.x;
    const int tile = w[0], slot = w[1], cover = w[2], total = w[3];
    if (tile < 0) return;   // padding unit of the strip-ordered work list
    int rs[5], cum[6];
    cum[0] = 0;
#pragma unroll
    for (int r = 0; r < 5; ++r) {
        rs[r] = w[4 + 2 * r];
        cum[r + 1] = cum[r] + w[5 + 2 * r] - rs[r];
    }
    const int t1o = (tile % nT) * TT, t2o = (tile / nT) * TT;
    const int mask = K - 1;
    const int Jn = J > 0 ? J : Jr;
    if (total == 0 && slot < 0) {   // no visibility reaches the tile
        for (int i = threadIdx.x; i < TT * TT; i += NT)
            grid[(size_t)(t1o + i / TT) * K + t2o + i % TT] = mk<T>(0, 0);
        return;
    }
    for (int i = threadIdx.x; i < 2 * WA * WA; i += NT) acc[i] = 0;
    const int ch = (total + NT - 1) / NT;
    const int j0 = (int)threadIdx.x * ch;
    auto item = [&](int j) {
        int idx = rs[0] + j;
#pragma unroll
        for (int r = 1; r < 5; ++r)
            if (j >= cum[r]) idx = rs[r] + (j - cum[r]);
        return idx;
    };
    const int wo1 = (t1o - (Jn - 1)) & mask, wo2 = (t2o - (Jn - 1)) & mask;   // window origin
    cpx<T> wreg[GTG && !DMA ? WPT : 1];
    if constexpr (GTG) {
#pragma unroll
        for (int k = 0; k < WPT; ++k) {
            const int i = threadIdx.x + k * NT;
            if (i < WS * WS) {
                const cpx<T>* src = gin + (size_t)((wo1 + i / WS) & mask) * K + ((wo2 + i % WS) & mask);
                if constexpr (DMA)
                    __builtin_amdgcn_global_load_lds(
                        (const void*)src,
                        (__attribute__((address_space(3))) void*)(win + (threadIdx.x & ~63u) + k * NT), 16, 0, 0);
                else
                    wreg[k] = *src;
            }
        }
    }
    bool staged = false;
#define PURIFY_STAGE_WINDOW()                                  \
    do {                                                       \
        if constexpr (!DMA) {                                  \
            _Pragma("unroll") for (int k = 0; k < WPT; ++k) {  \
                const int i = threadIdx.x + k * NT;            \
                if (i < WS * WS) win[i] = wreg[k];             \
            }                                                  \
        }                                                      \
        __syncthreads();                                       \
        staged = true;                                         \
    } while (0)
    // the visibility value: y (gridding) or the J x J interpolation from the window (G^T G,
    // same arithmetic order as the G kernel); the footprint's first window cell is
    // ((k - wo) mod K) on each axis and the taps follow at fixed offsets
    auto value = [&](int idx, int bk, const T* wa, const T* wb) {
        if constexpr (GTG) {
            const cpx<T>* w0 = win + (((bk & 0xFFFF) - wo1) & mask) * WS + ((((bk >> 16) & 0xFFFF) - wo2) & mask);
            T ax = 0, ay = 0;
#pragma unroll UNR
            for (int a = 0; a < JJ; ++a) {
                if (a >= Jn) break;
                T rx = 0, ry = 0;
#pragma unroll UNR
                for (int bb = 0; bb < JJ; ++bb) {
                    if (bb >= Jn) break;
                    const cpx<T> g = w0[a * WS + bb];
                    rx += wb[bb] * g.x;
                    ry += wb[bb] * g.y;
                }
                ax += wa[a] * rx;
                ay += wa[a] * ry;
            }
            return mk<T>(ax, ay);
        } else {
            return y[perm ? perm[idx] : idx];
        }
    };
    // largest component magnitude of the values over the unit's items (a separate pass only
    // when a thread's chunk does not fit in one batch)
    double ym = 0.0;
    if constexpr (GTG) {
        if (ch > CHR) PURIFY_STAGE_WINDOW();
    }
    if (ch > CHR) {
        for (int s = 0; s < ch; ++s) {
            const int j = j0 + s;
            if (j < total) {
                const int idx = item(j);
                cpx<T> v;
                if constexpr (GTG) {
                    T wa[JJ], wb[JJ];
                    visibility_weights<T, J>(wtab, kbc, idx, reinterpret_cast<const cpx<T>*>(frac)[idx], wa, wb, Jr);
                    v = value(idx, base[idx], wa, wb);
                } else {
                    v = value(idx, 0, nullptr, nullptr);
                }
                ym = fmax(ym, fmax(fabs((double)v.x), fabs((double)v.y)));
            }
        }
    }
    T inv_q = 0;
    int e = 0;
    bool any = false;
    for (int s0 = 0; s0 < ch; s0 += CHR) {
        int bk[CHR];
        cpx<T> vv[CHR];
        T wa[CHR][JJ], wb[CHR][JJ];
        bool ok[CHR];
#pragma unroll
        for (int c = 0; c < CHR; ++c) {
            const int j = j0 + s0 + c;
            ok[c] = s0 + c < ch && j < total;
            if (ok[c]) {
                const int idx = item(j);
                bk[c] = base[idx];
                const cpx<T> f = reinterpret_cast<const cpx<T>*>(frac)[idx];
                visibility_weights<T, J>(wtab, kbc, idx, f, wa[c], wb[c], Jr);
                if constexpr (!GTG) vv[c] = value(idx, bk[c], wa[c], wb[c]);
            }
        }
        if constexpr (GTG) {
            // the window's loads were issued before this batch's coordinate and weight loads
            if (!staged) PURIFY_STAGE_WINDOW();
#pragma unroll
            for (int c = 0; c < CHR; ++c)
                if (ok[c]) vv[c] = value(0, bk[c], wa[c], wb[c]);
        }
        if (ch <= CHR) {
#pragma unroll
            for (int c = 0; c < CHR; ++c)
                if (ok[c]) ym = fmax(ym, fmax(fabs((double)vv[c].x), fabs((double)vv[c].y)));
        }
        if (s0 == 0) {
            ym = wave_max(ym);
            if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = ym;
            __syncthreads();
            ym = 0.0;
#pragma unroll
            for (int wv = 0; wv < NT / 64; ++wv) ym = fmax(ym, red[wv]);
            // quantum q = 2^e with 2 * cover * max|y| <= 2^BITS q (at most `cover`
            // visibilities add to one cell, each by at most max|y|, psi <= 1, factor 2
            // margin) and 2 * max|y| <= 2^CBITS q (one contribution)
            const double bound = 2.0 * (double)cover * ym;
            any = bound > 0.0;
            e = any ? max(ilogb(bound) + 1 - Acc::BITS, ilogb(2.0 * ym) + 1 - Acc::CBITS) : 0;
            inv_q = (T)ldexp(1.0, -e);
        }
        if (!any) break;
#pragma unroll
        for (int c = 0; c < CHR; ++c) {
            if (!ok[c]) continue;
            const int r0 = (((bk[c] & 0xFFFF) - t1o + JM) & mask) - JM;
            const int c0 = ((((bk[c] >> 16) & 0xFFFF) - t2o + JM) & mask) - JM;
            typename Acc::I* ap = acc + (r0 + JM) * WA + (c0 + JM);
#pragma unroll UNR
            for (int a = 0; a < JJ; ++a) {
                if (a >= Jn) break;
                const T sc = wa[c][a] * inv_q;
                const T vx = sc * vv[c].x, vy = sc * vv[c].y;
#pragma unroll UNR
                for (int bb = 0; bb < JJ; ++bb) {
                    if (bb >= Jn) break;
                    if constexpr (PACK) {
                        __hip_atomic_fetch_add(accp + (ap - acc) + a * WA + bb,
                                               pack_pair((int)Acc::conv_mul(wb[c][bb], vx),
                                                         (int)Acc::conv_mul(wb[c][bb], vy)),
                                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                    } else {
                        lds_add<T>(ap + a * WA + bb, Acc::conv_mul(wb[c][bb], vx));
                        lds_add<T>(ap + WA * WA + a * WA + bb, Acc::conv_mul(wb[c][bb], vy));
                    }
                }
            }
        }
    }
    __syncthreads();
    // the cell sums (real, imaginary) of padded-tile cell pi
    auto cell = [&](int pi, typename Acc::I& re, typename Acc::I& im) {
        if constexpr (PACK) {
            int a, b;
            unpack_pair(accp[pi], a, b);
            re = a;
            im = b;
        } else {
            re = acc[pi];
            im = acc[WA * WA + pi];
        }
    };
    if (slot < 0) {
        const T q = (T)ldexp(1.0, e);
        // grids of 8192^2 and more (512 MB in FP32, twice the last-level cache) are written
        // with streaming stores, so they do not push out what the next launches reuse
        const bool stream = K >= 8192;
        for (int i = threadIdx.x; i < TT * TT; i += NT) {
            const int r = i / TT, c = i % TT;
            typename Acc::I re, im;
            cell((r + JM) * WA + c + JM, re, im);
            cpx<T>* o = grid + (size_t)(t1o + r) * K + t2o + c;
            if (stream) {
                __builtin_nontemporal_store(q * (T)re, &o->x);
                __builtin_nontemporal_store(q * (T)im, &o->y);
            } else {
                *o = mk<T>(q * (T)re, q * (T)im);
            }
        }
        return;
    }
    typename Acc::I* pt = partial + (size_t)slot * 2 * TT * TT;
    for (int i = threadIdx.x; i < TT * TT; i += NT) {
        const int r = i / TT, c = i % TT;
        typename Acc::I re, im;
        cell((r + JM) * WA + c + JM, re, im);
        pt[2 * i] = re;
        pt[2 * i + 1] = im;
    }
    if (threadIdx.x == 0) pexp[slot] = e;
}

#undef PURIFY_STAGE_WINDOW

// Sum of the partial tiles of each split tile (one workgroup per split tile), in part order
// and in double, then written to the grid.
template <typename T, int TT>
__global__ void __launch_bounds__(256)
k_grid_merge(const int32_t* __restrict__ merge, const typename FixedAcc<T>::I* __restrict__ partial,
             const int32_t* __restrict__ pexp, cpx<T>* __restrict__ grid, int K, int nT) {
    const int tile = merge[3 * blockIdx.x], parts = merge[3 * blockIdx.x + 1];
    const int slot0 = merge[3 * blockIdx.x + 2];
    const int t1o = (tile % nT) * TT, t2o = (tile / nT) * TT;
    using I = typename FixedAcc<T>::I;
    constexpr int EPT = (TT * TT + 255) / 256;   // cells a thread
    constexpr int PB = 4;                          // parts whose loads are in flight together
    double sr[EPT], si[EPT];
#pragma unroll
    for (int k = 0; k < EPT; ++k) sr[k] = si[k] = 0.0;
    for (int p0 = 0; p0 < parts; p0 += PB) {
        // a batch of parts is loaded before any is added; the sums still run in part order
        I vr[PB][EPT], vi[PB][EPT];
        int ex[PB];
#pragma unroll
        for (int b = 0; b < PB; ++b) {
            if (p0 + b < parts) {
                ex[b] = pexp[slot0 + p0 + b];
                const I* pt = partial + (size_t)(slot0 + p0 + b) * 2 * TT * TT;
#pragma unroll
                for (int k = 0; k < EPT; ++k) {
                    const int i = threadIdx.x + k * 256;
                    if (i < TT * TT) {
                        vr[b][k] = pt[2 * i];
                        vi[b][k] = pt[2 * i + 1];
                    }
                }
            }
        }
#pragma unroll
        for (int b = 0; b < PB; ++b) {
            if (p0 + b < parts) {
#pragma unroll
                for (int k = 0; k < EPT; ++k) {
                    if (threadIdx.x + k * 256 < TT * TT) {
                        sr[k] += ldexp((double)vr[b][k], ex[b]);
                        si[k] += ldexp((double)vi[b][k], ex[b]);
                    }
                }
            }
        }
    }
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
        const int i = threadIdx.x + k * 256;
        if (i < TT * TT) {
            const int r = i / TT, c = i % TT;
            grid[(size_t)(t1o + r) * K + t2o + c] = mk<T>((T)sr[k], (T)si[k]);
        }
    }
}

template <typename T, int TT, int NT, bool GTG>
void grid_tt(const Plan& P, const cpx<T>* y, const cpx<T>* gin, const int32_t* perm, cpx<T>* grid, hipStream_t s) {
    const dim3 g(P.nwork), b(NT);
    using I = typename FixedAcc<T>::I;
    // items per batch (register budget).  FP32 gridding of y: one, for occupancy (a unit whose
    // threads hold more items reads y once more for the scale); FP32 G^T G: four, since
    // there the scale's extra pass would interpolate every value twice
    constexpr int C = sizeof(T) == 8 ? 2 : (GTG ? 4 : 1);
    I* scr = (I*)P.gscratch;
    const T* fr = (const T*)P.frac;
    const T* kbc = (const T*)P.kbpoly;
    const T* wt = (const T*)P.wtab;
    switch (P.J) {
        case 4: hipLaunchKernelGGL((k_grid<T, 4, TT, NT, C, GTG>), g, b, 0, s, y, gin, perm, P.base, fr, kbc, wt, P.gwork, scr, P.gexp, grid, P.K, P.nT, 4); break;
        case 6: hipLaunchKernelGGL((k_grid<T, 6, TT, NT, C, GTG>), g, b, 0, s, y, gin, perm, P.base, fr, kbc, wt, P.gwork, scr, P.gexp, grid, P.K, P.nT, 6); break;
        case 8: hipLaunchKernelGGL((k_grid<T, 8, TT, NT, C, GTG>), g, b, 0, s, y, gin, perm, P.base, fr, kbc, wt, P.gwork, scr, P.gexp, grid, P.K, P.nT, 8); break;
        default: hipLaunchKernelGGL((k_grid<T, 0, TT, NT, 1, GTG>), g, b, 0, s, y, gin, perm, P.base, fr, kbc, wt, P.gwork, scr, P.gexp, grid, P.K, P.nT, P.J); break;
    }
    if (P.nmerge > 0)
        hipLaunchKernelGGL((k_grid_merge<T, TT>), dim3(P.nmerge), dim3(256), 0, s, P.gmerge, scr, P.gexp, grid, P.K, P.nT);
}

}  // namespace

template <typename T, int TT>
void degrid_tiles_tt(const Plan& P, const cpx<T>* grid, cpx<T>* y, const int32_t* perm, double scale,
                     hipStream_t s) {
    // tiles of side TD: the gridding work units (TD = TT) or the plan's degridding records
    const bool own = P.TD > P.TT;
    const int32_t* work = own ? P.dwork : P.gwork;
    const int nT = own ? P.nTD : P.nT;
    const dim3 g(own ? P.ndwork : P.nwork), b(256);
    const T* fr = (const T*)P.frac;
    const T* kbc = (const T*)P.kbpoly;
    const T* wt = (const T*)P.wtab;
    switch (P.J) {
        case 4: hipLaunchKernelGGL((k_degrid_tiles<T, 4, TT, 256>), g, b, 0, s, grid, y, perm, P.base, fr, kbc, wt, work, P.K, nT, (T)scale, 4); break;
        case 6: hipLaunchKernelGGL((k_degrid_tiles<T, 6, TT, 256>), g, b, 0, s, grid, y, perm, P.base, fr, kbc, wt, work, P.K, nT, (T)scale, 6); break;
        case 8: hipLaunchKernelGGL((k_degrid_tiles<T, 8, TT, 256>), g, b, 0, s, grid, y, perm, P.base, fr, kbc, wt, work, P.K, nT, (T)scale, 8); break;
        default: hipLaunchKernelGGL((k_degrid_tiles<T, 0, TT, 256>), g, b, 0, s, grid, y, perm, P.base, fr, kbc, wt, work, P.K, nT, (T)scale, P.J); break;
    }
}

template <typename T>
void launch_degrid(const Plan& P, const cpx<T>* grid, cpx<T>* y, const int32_t* perm, double scale,
                   hipStream_t s) {
    if (P.degrid_tiles) {
        if (P.TD == 16) degrid_tiles_tt<T, 16>(P, grid, y, perm, scale, s);
        else if constexpr (sizeof(T) == 4) {   // 64 x 64 windows: FP32 only (LDS)
            if (P.TD == 64) degrid_tiles_tt<T, 64>(P, grid, y, perm, scale, s);
            else degrid_tiles_tt<T, 32>(P, grid, y, perm, scale, s);
        } else degrid_tiles_tt<T, 32>(P, grid, y, perm, scale, s);
        return;
    }
    const int M = (int)P.M;
    const int32_t* ch = P.ndchunk > 0 ? P.dchunk : nullptr;
    const dim3 g(ch ? P.ndchunk : (M + 255) / 256), b(256);
    const T* fr = (const T*)P.frac;
    const T* kbc = (const T*)P.kbpoly;
    switch (P.J) {
        case 4: hipLaunchKernelGGL((k_degrid<T, 4>), g, b, 0, s, grid, y, perm, P.base, fr, kbc, (const T*)P.wtab, M, P.K, (T)scale, 4, ch); break;
        case 6: hipLaunchKernelGGL((k_degrid<T, 6>), g, b, 0, s, grid, y, perm, P.base, fr, kbc, (const T*)P.wtab, M, P.K, (T)scale, 6, ch); break;
        case 8: hipLaunchKernelGGL((k_degrid<T, 8>), g, b, 0, s, grid, y, perm, P.base, fr, kbc, (const T*)P.wtab, M, P.K, (T)scale, 8, ch); break;
        default: hipLaunchKernelGGL((k_degrid<T, 0>), g, b, 0, s, grid, y, perm, P.base, fr, kbc, (const T*)P.wtab, M, P.K, (T)scale, P.J, ch); break;
    }
}

template <typename T>
void launch_grid(const Plan& P, const cpx<T>* y, const int32_t* perm, cpx<T>* grid, hipStream_t s) {
    // FP32 32 x 32 tiles: 128 threads a unit (more units a CU; most units hold far fewer
    // visibilities than threads: 4096^2 G^T 503 -> 469 us, 1024^2 68.6 -> 64.0 us against 256)
    if (P.TT == 16) grid_tt<T, 16, 256, false>(P, y, nullptr, perm, grid, s);
    else grid_tt<T, 32, sizeof(T) == 4 ? 128 : 256, false>(P, y, nullptr, perm, grid, s);
}

template <typename T>
void launch_gtg(const Plan& P, const cpx<T>* gin, cpx<T>* gout, hipStream_t s) {
    if (sizeof(T) == 4 && P.K >= 2048) {
        // FP32 grids from 2048 x 2048: G into the plan's visibility buffer, then G^T from it
        // (the 64 x 64 degridding windows carry less halo than the fused launch's, and the
        // one-item gridding batches in 128-thread units keep more units on a CU: 1024^2
        // 97.8 -> 90.1 us, 4096^2 897 -> 737 us)
        launch_degrid<T>(P, gin, (cpx<T>*)P.vis, nullptr, 1.0, s);
        launch_grid<T>(P, (const cpx<T>*)P.vis, nullptr, gout, s);
        return;
    }
    if (P.TT == 16) grid_tt<T, 16, 256, true>(P, nullptr, gin, nullptr, gout, s);
    else grid_tt<T, 32, 256, true>(P, nullptr, gin, nullptr, gout, s);
}

template void launch_degrid<float>(const Plan&, const cpx<float>*, cpx<float>*, const int32_t*, double, hipStream_t);
template void launch_degrid<double>(const Plan&, const cpx<double>*, cpx<double>*, const int32_t*, double, hipStream_t);
template void launch_grid<float>(const Plan&, const cpx<float>*, const int32_t*, cpx<float>*, hipStream_t);
template void launch_grid<double>(const Plan&, const cpx<double>*, const int32_t*, cpx<double>*, hipStream_t);
template void launch_gtg<float>(const Plan&, const cpx<float>*, cpx<float>*, hipStream_t);
template void launch_gtg<double>(const Plan&, const cpx<double>*, cpx<double>*, hipStream_t);

}  // namespace purify
