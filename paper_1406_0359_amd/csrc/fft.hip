// F and F^dagger of the measurement operator Phi = G F Z S (NUFFT, Section 4), fused with
// S (deapodisation) and Z (zero padding / cropping).
//
// One axis of F Z maps n pixels p = j - n/2 to K = 2n frequencies:
//     (D v)[k] = sum_j v_j exp(-2 pi i k (j - n/2) / K).
// Splitting the output by parity, k = 2k' + r (r = 0, 1):
//     (D v)[2k' + r] = (-1)^k' i^r FFT_n( v_j exp(-pi i r j / n) )[k'],
// so each line costs two n-point FFTs and the zero half of the padded line is never
// touched.  The adjoint (K -> n) splits the input by parity instead:
//     (D^dag u)[j] = IFFT_n((-1)^k' u_2k')[j] + (-i) exp(pi i j / n) IFFT_n((-1)^k' u_2k'+1)[j].
//
// Layouts (row-major): image x[j1][j2] (n x n), intermediate tmp[j1][k2] (n x K), grid
// G[k1][k2] (K x K).  Passes:
//   rows_fwd : each image row j1      -> tmp row j1     (S, D along axis 1)
//   cols_fwd : each tmp column k2     -> G column k2    (D along axis 0)
//   cols_adj : each G column k2       -> tmp column k2  (D^dag along axis 0)
//   rows_adj : each tmp row j1        -> image row j1   (D^dag along axis 1, S, epilogue)
// Row passes read and write whole rows; column passes handle C adjacent columns per
// workgroup so every global access is a contiguous run of C elements.  The two parities of
// a line run on separate thread groups; the adjoint combines them through LDS.
//
// Each n-point transform is a self-sorting (Stockham) FFT with large radices (8..32) held in
// registers: one thread owns n/RMAX butterflies of each pass, runs the radix-R DFT in
// registers (unrolled, compile-time roots of unity), and passes exchange data through one
// LDS line buffer.  n = 1024 is two radix-32 passes: a single LDS round trip.  Inter-pass
// twiddles come from an FP64-accurate table staged in LDS.
#include <map>
#include <mutex>
#include <type_traits>

#include "common.h"

namespace purify {

namespace {

// ---------------------------------------------------------------------------------------
// Compile-time roots of unity: cos and sin of 2 pi k / L, by octant reduction and Taylor
// series of the reduced angle (|phi| < pi/4).
struct CS {
    double c, s;
};
constexpr double taylor_sin(double x) {
    double term = x, sum = x;
    for (int k = 1; k < 14; ++k) {
        term *= -x * x / ((2.0 * k) * (2.0 * k + 1.0));
        sum += term;
    }
    return sum;
}
constexpr double taylor_cos(double x) {
    double term = 1.0, sum = 1.0;
    for (int k = 1; k < 14; ++k) {
        term *= -x * x / ((2.0 * k - 1.0) * (2.0 * k));
        sum += term;
    }
    return sum;
}
constexpr CS root(int k, int L) {
    // angle = 2 pi k / L = (pi / 4) * (8k / L); split 8k = q L + r
    const long long num = 8LL * (k % L);
    const int q = (int)(num / L);
    const double frac = (double)(num % L) / (double)L;   // in [0, 1)
    const double pi4 = 0.78539816339744830961566084581987572;
    // angle = q pi/4 + phi, phi = frac pi/4; use the nearest octant boundary
    double phi = frac * pi4;
    int oct = q;
    if (frac > 0.5) {
        phi = (frac - 1.0) * pi4;
        oct = q + 1;
    }
    const double c0 = taylor_cos(phi), s0 = taylor_sin(phi);
    const double h = 0.70710678118654752440084436210484904;
    double c = 0, s = 0;
    switch (oct & 7) {
        case 0: c = c0; s = s0; break;
        case 1: c = h * (c0 - s0); s = h * (c0 + s0); break;
        case 2: c = -s0; s = c0; break;
        case 3: c = -h * (c0 + s0); s = h * (c0 - s0); break;
        case 4: c = -c0; s = -s0; break;
        case 5: c = h * (s0 - c0); s = -h * (c0 + s0); break;
        case 6: c = s0; s = -c0; break;
        default: c = h * (c0 + s0); s = h * (s0 - c0); break;
    }
    return CS{c, s};
}
template <int L>
struct Roots {
    CS w[L > 0 ? L : 1];
    constexpr Roots() : w() {
        for (int k = 0; k < L; ++k) w[k] = root(k, L);
    }
};

constexpr int bitrev(int i, int R) {
    int r = 0;
    for (int b = 1; b < R; b <<= 1) {
        r = (r << 1) | (i & 1);
        i >>= 1;
    }
    return r;
}

// v[st+k] <- a+b ; v[st+k+H] <- (a-b) w^k  for every radix-2 DIF stage of an R-point DFT.
template <typename T, int R, int LEN, bool INV>
__device__ __forceinline__ void dif_stages(cpx<T>* v) {
    if constexpr (LEN >= 2) {
        constexpr int H = LEN / 2;
        constexpr Roots<LEN> tab{};
#pragma unroll
        for (int st = 0; st < R; st += LEN) {
#pragma unroll
            for (int k = 0; k < H; ++k) {
                const cpx<T> a = v[st + k], b = v[st + k + H];
                v[st + k] = a + b;
                const cpx<T> d = a - b;
                if (k == 0) {
                    v[st + k + H] = d;
                } else if (4 * k == LEN) {
                    v[st + k + H] = INV ? mul_i(d) : mul_mi(d);
                } else {
                    const T c = (T)tab.w[k].c;
                    const T s = INV ? (T)tab.w[k].s : -(T)tab.w[k].s;
                    v[st + k + H] = mk<T>(d.x * c - d.y * s, d.x * s + d.y * c);
                }
            }
        }
        dif_stages<T, R, LEN / 2, INV>(v);
    }
}

// In-register R-point DFT: natural order in, natural order out (forward exp(-2 pi i),
// INV = conjugate).
template <typename T, int R, bool INV>
__device__ __forceinline__ void reg_dft(cpx<T>* v) {
    dif_stages<T, R, R, INV>(v);
    cpx<T> t[R];
#pragma unroll
    for (int i = 0; i < R; ++i) t[i] = v[i];
#pragma unroll
    for (int i = 0; i < R; ++i) v[i] = t[bitrev(i, R)];
}

// ---------------------------------------------------------------------------------------
// Radix plans: product of the radices is n; RMAX elements live in registers per thread.
// AX = 0: row passes, AX = 1: column passes (which reuse the row plan unless listed).  The
// row passes of the small and mid sizes have few rows (n of them), so they are latency-bound
// and use more, shorter threads (radix-4 passes); measured per size.
template <typename T, int LOGN, int AX>
struct Radices : Radices<T, LOGN, 0> {};
#define PURIFY_RADICES_AX4(TY, LG, AX, NP_, R0, R1, R2, R3)   \
    template <>                                               \
    struct Radices<TY, LG, AX> {                              \
        static constexpr int NP = NP_;                        \
        static constexpr int r[4] = {R0, R1, R2, R3};         \
    };
#define PURIFY_RADICES_AX(TY, LG, AX, NP_, R0, R1, R2) PURIFY_RADICES_AX4(TY, LG, AX, NP_, R0, R1, R2, 1)
#define PURIFY_RADICES(TY, LG, NP_, R0, R1, R2) PURIFY_RADICES_AX(TY, LG, 0, NP_, R0, R1, R2)
PURIFY_RADICES(float, 4, 1, 16, 1, 1)
PURIFY_RADICES(float, 5, 1, 32, 1, 1)
PURIFY_RADICES(float, 6, 2, 8, 8, 1)
PURIFY_RADICES_AX4(float, 7, 0, 4, 4, 4, 4, 2)
PURIFY_RADICES_AX(float, 7, 1, 3, 8, 4, 4)
PURIFY_RADICES_AX4(float, 8, 0, 4, 4, 4, 4, 4)
PURIFY_RADICES_AX(float, 8, 1, 3, 8, 8, 4)
PURIFY_RADICES(float, 9, 3, 8, 8, 8)
// n = 1024 FP32: rows in four passes (128 threads per line), columns in three
PURIFY_RADICES_AX4(float, 10, 0, 4, 4, 8, 8, 4)
PURIFY_RADICES_AX(float, 10, 1, 3, 8, 8, 16)
PURIFY_RADICES(float, 11, 3, 32, 16, 4)
// n = 4096 FP32: rows and columns in four radix-8 passes (512 threads per line); the long
// column passes then hold half as many values a thread (126 instead of 256 VGPRs), so a CU
// runs 16 waves of them instead of 8 (forward 556 -> 460 us, adjoint 480 -> 451 us against
// three radix-16 passes)
PURIFY_RADICES_AX4(float, 12, 0, 4, 8, 8, 8, 8)
PURIFY_RADICES(double, 4, 1, 16, 1, 1)
PURIFY_RADICES(double, 5, 2, 16, 2, 1)
PURIFY_RADICES(double, 6, 2, 8, 8, 1)
PURIFY_RADICES_AX4(double, 7, 0, 4, 4, 4, 4, 2)
PURIFY_RADICES_AX(double, 7, 1, 3, 8, 4, 4)
// n = 256 FP64: four radix-4 passes (64 threads per line) for rows and columns; measured 3.7
// against 5.1 us for 8 x 8 x 4 on the 256 rows of a pass
PURIFY_RADICES_AX4(double, 8, 0, 4, 4, 4, 4, 4)
PURIFY_RADICES_AX4(double, 8, 1, 4, 4, 4, 4, 4)
PURIFY_RADICES(double, 9, 3, 8, 8, 8)
PURIFY_RADICES(double, 10, 3, 16, 16, 4)
PURIFY_RADICES(double, 11, 3, 16, 16, 8)
PURIFY_RADICES(double, 12, 3, 16, 16, 16)

// Long FP32 columns (n >= 4096) keep one pad element after every 8 of a line buffer.  A
// Stockham pass writes its first outputs 8 elements apart (64 bytes: every lane of a wave on
// the same two of LDS's banks) and its second in runs of 8 that repeat every 512 bytes; with
// the pad the strides become 9 elements and runs 72 apart, which spread over all banks.
// Every stride of these plans is a multiple of 8, so a padded address is still a per-thread
// base plus a compile-time offset.
template <typename T, int LOGN, int AX>
constexpr bool pad_lines() { return AX == 1 && sizeof(T) == 4 && LOGN >= 12; }

template <typename T, int LOGN, int AX>
struct Plan1D {
    using Rd = Radices<T, LOGN, AX>;
    static constexpr int N = 1 << LOGN;
    static constexpr int NP = Rd::NP;
    static constexpr int R0 = Rd::r[0];
    static constexpr int RL = Rd::r[NP - 1];
    static constexpr int RMAX01 = Rd::r[0] > Rd::r[1] ? Rd::r[0] : Rd::r[1];
    static constexpr int RMAX23 = Rd::r[2] > Rd::r[3] ? Rd::r[2] : Rd::r[3];
    static constexpr int RMAX = RMAX01 > RMAX23 ? RMAX01 : RMAX23;
    static constexpr int TL = N / RMAX;          // threads per line
    static constexpr bool PAD = pad_lines<T, LOGN, AX>();
    static constexpr int LS = PAD ? N + N / 8 : N + 1;   // LDS line stride (padding)
    static_assert(!PAD || TL % 8 == 0, "padded lines need thread counts in multiples of 8");
    // LDS offset of line position p, and the LDS distance of a position distance d (a
    // multiple of 8 in padded lines)
    __device__ static __forceinline__ int at(int p) { return PAD ? p + (p >> 3) : p; }
    static constexpr int span(int d) { return PAD ? d + d / 8 : d; }
    static constexpr int at_c(int p) { return PAD ? p + p / 8 : p; }
    // register slot i on entry holds position in_pos(tl, i); on exit out_pos(tl, i)
    __device__ static __forceinline__ int in_pos(int tl, int i) {
        return tl + (i / R0) * TL + (i % R0) * (N / R0);
    }
    __device__ static __forceinline__ int out_pos(int tl, int i) {
        return tl + (i / RL) * TL + (i % RL) * (N / RL);
    }
    // LDS offsets of in_pos and out_pos
    __device__ static __forceinline__ int in_at(int tl, int i) {
        static_assert(!PAD || (N / R0) % 8 == 0, "padded lines");
        return at(tl) + span((i / R0) * TL + (i % R0) * (N / R0));
    }
    __device__ static __forceinline__ int out_at(int tl, int i) {
        static_assert(!PAD || (N / RL) % 8 == 0, "padded lines");
        return at(tl) + span((i / RL) * TL + (i % RL) * (N / RL));
    }
};

// FP32 lines of 4096 and more take their inter-pass twiddles from two short tables,
// W[m] = W[(m >> LB) 2^LB] W[m mod 2^LB] (2^LB + n / 2^LB entries instead of n; one more
// rounding, well inside FP32 accuracy), so a workgroup's LDS is little more than its line
// buffers and two workgroups fit on a CU.
template <typename T, int LOGN>
constexpr bool twiddles_split() { return sizeof(T) == 4 && LOGN >= 12; }
template <typename T, int LOGN>
constexpr int split_lb() { return (LOGN + 1) / 2; }
// twiddle W[m] = exp(-2 pi i m / n) from the staged table
template <typename T, int LOGN>
__device__ __forceinline__ cpx<T> tw_get(const cpx<T>* W, int m) {
    if constexpr (twiddles_split<T, LOGN>()) {
        constexpr int LB = split_lb<T, LOGN>(), L = 1 << LB;
        return W[L + (m >> LB)] * W[m & (L - 1)];
    } else {
        return W[m];
    }
}

template <typename T, int LOGN, int AX, int P, bool INV>
__device__ __forceinline__ void fft_pass(cpx<T>* v, cpx<T>* line, int tl, const cpx<T>* W) {
    using PL = Plan1D<T, LOGN, AX>;
    using Rd = Radices<T, LOGN, AX>;
    constexpr int N = PL::N;
    constexpr int R = Rd::r[P];
    constexpr int NB = PL::RMAX / R;   // butterflies per thread in this pass
    constexpr int NS = P == 0 ? 1 : (P == 1 ? Rd::r[0] : (P == 2 ? Rd::r[0] * Rd::r[1] : Rd::r[0] * Rd::r[1] * Rd::r[2]));
    static_assert(!PL::PAD || ((N / R) % 8 == 0 && (NS % 8 == 0 || (NS == 1 && R % 8 == 0))), "padded lines");
    if constexpr (P > 0) {
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const int j = PL::at(tl) + PL::span(b * PL::TL);
#pragma unroll
            for (int r = 0; r < R; ++r) v[b * R + r] = line[j + r * PL::span(N / R)];
        }
        __syncthreads();
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const int j = tl + b * PL::TL;
            const int k = j % NS;
#pragma unroll
            for (int r = 1; r < R; ++r) {
                cpx<T> w = tw_get<T, LOGN>(W, r * k * (N / (NS * R)));
                if (INV) w.y = -w.y;
                v[b * R + r] = v[b * R + r] * w;
            }
        }
    }
#pragma unroll
    for (int b = 0; b < NB; ++b) reg_dft<T, R, INV>(v + b * R);
    if constexpr (P < Rd::NP - 1) {
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const int j = tl + b * PL::TL;
            const int k = j % NS;
            const int o = PL::at((j - k) * R + k);
#pragma unroll
            for (int t = 0; t < R; ++t) line[o + (NS == 1 ? PL::at_c(t) : PL::span(t * NS))] = v[b * R + t];
        }
        __syncthreads();
    }
}

// Run every pass on this thread's registers; `line` is this line's LDS buffer.
template <typename T, int LOGN, int AX, bool INV>
__device__ __forceinline__ void line_fft(cpx<T>* v, cpx<T>* line, int tl, const cpx<T>* W) {
    using Rd = Radices<T, LOGN, AX>;
    fft_pass<T, LOGN, AX, 0, INV>(v, line, tl, W);
    if constexpr (Rd::NP > 1) fft_pass<T, LOGN, AX, 1, INV>(v, line, tl, W);
    if constexpr (Rd::NP > 2) fft_pass<T, LOGN, AX, 2, INV>(v, line, tl, W);
    if constexpr (Rd::NP > 3) fft_pass<T, LOGN, AX, 3, INV>(v, line, tl, W);
}

template <typename T>
__device__ __forceinline__ cpx<T> neg(cpx<T> a) { return mk<T>(-a.x, -a.y); }

// Workgroups are dispatched round-robin over the 8 XCDs (each with its own L2).  Column
// passes read and write runs of C columns, so neighbouring column groups share cache
// lines: give each XCD a contiguous range of column groups.
__device__ __forceinline__ int xcd_block() {
    const int nb = gridDim.x, b = blockIdx.x;
    if (nb % 8 != 0) return b;
    return (b % 8) * (nb / 8) + b / 8;
}

// Column group of this workgroup when the grid's gridding tiles are strips of `sg` column
// groups: workgroup b runs on XCD b % 8 and takes the strips congruent to b % 8 (mod 8), the
// same strips whose tiles the gridding kernel runs on that XCD, so the grid stays in that
// XCD's L2 between the column passes and the gridding.  sg = 0: xcd_block().
__device__ __forceinline__ int strip_block(int sg) {
    if (sg <= 0) return xcd_block();
    const int e = blockIdx.x % 8, k = blockIdx.x / 8;
    return (e + 8 * (k / sg)) * sg + k % sg;
}

// Workgroup shapes.  Each n-point line transform uses TL threads; the two output parities of
// a line are separate thread groups.  Row passes: B rows per workgroup (64-128 threads).
// Column passes: C adjacent columns (contiguous runs of C elements), at most 1024 threads,
// at least ~256 workgroups, and LDS (2C lines + twiddle table) within 160 KB.
template <typename T, int LOGN>
constexpr int rows_per_wg() {
    constexpr int tl = Plan1D<T, LOGN, 0>::TL;
    int b = 64 / (2 * tl);
    if (b < 1) b = 1;
    if (b > (1 << LOGN)) b = 1 << LOGN;
    return b;
}
template <typename T, int LOGN>
constexpr bool twiddles_in_lds() {
    constexpr int N = 1 << LOGN;
    return twiddles_split<T, LOGN>() || (size_t)(N + 2 * (N + 1)) * 2 * sizeof(T) <= 160 * 1024;
}
template <typename T, int LOGN>
constexpr int table_elems() {
    if constexpr (twiddles_split<T, LOGN>()) return (1 << split_lb<T, LOGN>()) + (1 << (LOGN - split_lb<T, LOGN>()));
    else return twiddles_in_lds<T, LOGN>() ? (1 << LOGN) : 0;
}
template <typename T, int LOGN>
constexpr int cols_per_wg() {
    constexpr int N = 1 << LOGN;
    constexpr int tl = Plan1D<T, LOGN, 1>::TL;
    int c = 512 / tl;
    if (c > (4 * N) / 256) c = (4 * N) / 256;
    if (c > 8) c = 8;
    if (c < 1) c = 1;
    const int tab = table_elems<T, LOGN>();
    while (c > 1 && (size_t)(tab + 2 * c * (N + 1)) * 2 * sizeof(T) > 160 * 1024) c >>= 1;
    return c;
}

// Long columns (a workgroup's LDS holds only one column's two parity lines, or FP32 lines of
// 4096 and more) run the kernels that keep CR adjacent columns per thread in registers.
template <typename T, int LOGN>
constexpr bool long_cols() { return LOGN >= 11 && (cols_per_wg<T, LOGN>() == 1 || twiddles_split<T, LOGN>()); }
template <typename T, int LOGN>
constexpr int long_cols_cr() { return sizeof(T) == 8 || Plan1D<T, LOGN, 1>::RMAX >= 16 ? 2 : 4; }
// Column groups of the stored operator's spectrum: element (k1, k2) at
// ((k2 / W) K + k1) W + k2 mod W.  Long FP32 columns (two a thread in registers; four, with the
// spectrum's loads, spilled at the 128-register limit of the 1024-thread workgroup) store each
// workgroup's K x 2 block contiguously, so it reads one run instead of 8 bytes from each of K
// rows (4096^2 column stage 907 -> 672 us); elsewhere W = K, the row-major grid, which the
// multi-column workgroups read in runs of C values (a blocked layout there measured slower).
template <typename T, int LOGN>
constexpr bool toep_mc() { return sizeof(T) == 4 && long_cols<T, LOGN>(); }
template <typename T, int LOGN>
constexpr int toep_group() { return toep_mc<T, LOGN>() ? 2 : 2 << LOGN; }
// workgroups of a long-column kernel that can share a CU: two of 512 threads or fewer (16
// waves at up to 128 VGPRs) if their twiddle table and two line buffers fit twice in LDS
template <typename T, int LOGN>
constexpr int mc_wgs_per_cu() {
    constexpr size_t lines = (size_t)(table_elems<T, LOGN>() + 2 * Plan1D<T, LOGN, 1>::LS) * sizeof(cpx<T>);
    return 2 * Plan1D<T, LOGN, 1>::TL <= 512 && 2 * lines <= 160 * 1024 ? 2 : 1;
}
// The long-column kernels keep the n parity twiddles exp(-pi i j / n) in LDS beside their two
// line buffers where they fit: staged at the start (all loads in flight at once), then read
// for every column from LDS instead of from global memory once each column's data is in.
template <typename T, int LOGN>
constexpr bool mc_tw2_in_lds() {
    return (size_t)(table_elems<T, LOGN>() + 2 * Plan1D<T, LOGN, 1>::LS + (1 << LOGN)) * sizeof(cpx<T>) <=
           160 * 1024 / mc_wgs_per_cu<T, LOGN>();
}
// waves per SIMD the register allocation of a long-column kernel must allow
template <typename T, int LOGN>
constexpr int mc_waves_per_eu() {
    constexpr int w = mc_wgs_per_cu<T, LOGN>() * 2 * Plan1D<T, LOGN, 1>::TL / 256;
    return w < 1 ? 1 : w;
}
template <typename T, int LOGN>
constexpr size_t mc_lds_bytes() {
    return (size_t)(table_elems<T, LOGN>() + 2 * Plan1D<T, LOGN, 1>::LS + (mc_tw2_in_lds<T, LOGN>() ? (1 << LOGN) : 0)) *
           sizeof(cpx<T>);
}
// stage tw2 after the two line buffers (a workgroup of 2 TL threads); returns where to read it
template <typename T, int LOGN>
__device__ __forceinline__ const cpx<T>* mc_stage_tw2(cpx<T>* lines, const cpx<T>* __restrict__ tw2) {
    using PL = Plan1D<T, LOGN, 1>;
    if constexpr (mc_tw2_in_lds<T, LOGN>()) {
        constexpr int NQ = PL::RMAX / 2;
        cpx<T>* t2l = lines + 2 * PL::LS;
        cpx<T> t[NQ];
#pragma unroll
        for (int k = 0; k < NQ; ++k) t[k] = tw2[threadIdx.x + k * 2 * PL::TL];
#pragma unroll
        for (int k = 0; k < NQ; ++k) t2l[threadIdx.x + k * 2 * PL::TL] = t[k];
        return t2l;
    } else {
        return tw2;
    }
}

template <typename T, int LOGN>
__device__ __forceinline__ const cpx<T>* stage_twiddles(cpx<T>* Wl, const cpx<T>* __restrict__ tw) {
    if constexpr (twiddles_split<T, LOGN>()) {
        constexpr int LB = split_lb<T, LOGN>(), L = 1 << LB;
        for (int i = threadIdx.x; i < table_elems<T, LOGN>(); i += blockDim.x)
            Wl[i] = i < L ? tw[i] : tw[(size_t)(i - L) << LB];
        return Wl;
    } else if constexpr (twiddles_in_lds<T, LOGN>()) {
        for (int i = threadIdx.x; i < (1 << LOGN); i += blockDim.x) Wl[i] = tw[i];
        return Wl;
    } else {
        return tw;
    }
}

// ---------------------------------------------------------------------------------------
// Sums of two partial-sum buffers by one workgroup of any size, in one pass and in a fixed
// order (thread-strided, then across lanes, then across waves in wave order), so every
// workgroup gets the identical values; red holds 32 doubles.
__device__ __forceinline__ void sum_parts2_dyn(const double* __restrict__ pa, int na, const double* __restrict__ pb,
                                               int nb, double* red, double& ta, double& tb) {
    // four loads of each buffer in flight at a time, added in the thread-strided order
    double a = 0, b = 0;
    const int st = blockDim.x;
    for (int i0 = threadIdx.x; i0 < na || i0 < nb; i0 += 4 * st) {
        double va[4], vb[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int i = i0 + k * st;
            va[k] = i < na ? pa[i] : 0.0;
            vb[k] = i < nb ? pb[i] : 0.0;
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int i = i0 + k * st;
            if (i < na) a += va[k];
            if (i < nb) b += vb[k];
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        a += __shfl_xor(a, o);
        b += __shfl_xor(b, o);
    }
    if ((threadIdx.x & 63) == 0) {
        red[threadIdx.x >> 6] = a;
        red[16 + (threadIdx.x >> 6)] = b;
    }
    __syncthreads();
    ta = 0;
    tb = 0;
    const int nw = (blockDim.x + 63) >> 6;
    for (int i = 0; i < nw; ++i) {
        ta += red[i];
        tb += red[16 + i];
    }
    __syncthreads();
}

// Block sum of one value per thread (result in thread 0), any block size.
__device__ __forceinline__ double block_sum_dyn(double v, double* red) {
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

// Block sums of three values per thread (results in thread 0), any block size up to 1024;
// red holds 48 doubles.
__device__ __forceinline__ void block_sum3_dyn(double a, double b, double c, double* red, double& ta, double& tb,
                                               double& tc) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        a += __shfl_xor(a, o);
        b += __shfl_xor(b, o);
        c += __shfl_xor(c, o);
    }
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) {
        red[w] = a;
        red[16 + w] = b;
        red[32 + w] = c;
    }
    __syncthreads();
    ta = tb = tc = 0;
    if (threadIdx.x == 0) {
        const int nw = (blockDim.x + 63) >> 6;
        for (int i = 0; i < nw; ++i) {
            ta += red[i];
            tb += red[16 + i];
            tc += red[32 + i];
        }
    }
}

// Conjugate-gradient step folded into the row pass (used from the second step on), with the
// previous step's q = A p and the partial sums of rho = ||r||^2, <p, q>, <r, q> and ||q||^2:
// alpha = rho / <p, q>; x += alpha p; r -= alpha q; the new rho, ||r - alpha q||^2 =
// rho - 2 alpha <r, q> + alpha^2 ||q||^2, gives beta = rho_new / rho before any new residual is
// summed, so the new direction p = r + beta p is formed here too.  x, r and p are written back,
// the row transform is taken of the new p, and the partial ||r||^2 of the row block is written
// (the next step's rho, summed exactly).
template <typename T>
struct CgXr {
    cpx<T>* x = nullptr;
    cpx<T>* r = nullptr;
    cpx<T>* p = nullptr;
    const cpx<T>* q = nullptr;
    const double* rho_part = nullptr;
    int rho_count = 0;
    const double* pq_part = nullptr;
    int pq_count = 0;               // also the count of rq_part and qq_part
    const double* rq_part = nullptr;
    const double* qq_part = nullptr;
    double* rho_new_part = nullptr;
};

// Dot products of the adjoint row pass of a CG step besides <p, q>: <r, q> and ||q||^2 (the
// next row pass's beta)
template <typename T>
struct CgDots {
    const cpx<T>* r = nullptr;      // null: none
    double* rq_part = nullptr;
    double* qq_part = nullptr;
};

// A row's K outputs after its two parity transforms: position 2k' + r holds (-1)^k' i^r
// times parity r's value k'.  FP32 rows of 4096 and more pass through the line buffers first
// (both parity groups have read their last pass's inputs before that pass's barrier), so each
// thread stores both parities of a position as one 16-byte store and a wave's stores are one
// contiguous run; written straight from registers, the two parity groups' 8-byte stores
// interleave at a 16-byte stride.  These stores are streaming (non-temporal): the row
// transforms of a padded grid this large (256 MB at 8192^2) do not stay in the last-level
// cache for the column pass anyway, and written around it the row pass runs about 10% faster.
template <typename T, int LOGN>
constexpr bool rows_pair_store() { return sizeof(T) == 4 && LOGN >= 12; }
typedef float f4_nt __attribute__((ext_vector_type(4)));

template <typename T, int LOGN>
__device__ __forceinline__ void store_row_fwd(const cpx<T>* v, cpx<T>* lines, cpx<T>* outr, int tl, int r) {
    using PL = Plan1D<T, LOGN, 0>;
    if constexpr (rows_pair_store<T, LOGN>()) {
        static_assert(PL::NP > 1, "the last pass's barrier orders these writes after its reads");
        cpx<T>* line = lines + r * PL::LS;
#pragma unroll
        for (int i = 0; i < PL::RMAX; ++i) {
            const int kp = PL::out_pos(tl, i);
            cpx<T> o = (kp & 1) ? neg(v[i]) : v[i];
            if (r) o = mul_i(o);
            line[PL::out_at(tl, i)] = o;
        }
        __syncthreads();
        const int t = r * PL::TL + tl;
#pragma unroll
        for (int m = 0; m < PL::RMAX / 2; ++m) {
            const int a = PL::at(t) + PL::span(m * 2 * PL::TL);
            const cpx<T> e = lines[a], o = lines[PL::LS + a];
            const f4_nt q4 = {e.x, e.y, o.x, o.y};
            __builtin_nontemporal_store(q4, reinterpret_cast<f4_nt*>(outr + 2 * (t + m * 2 * PL::TL)));
        }
    } else {
#pragma unroll
        for (int i = 0; i < PL::RMAX; ++i) {
            const int kp = PL::out_pos(tl, i);
            cpx<T> o = (kp & 1) ? neg(v[i]) : v[i];
            if (r) o = mul_i(o);
            outr[2 * kp + r] = o;
        }
    }
}

// rows_fwd: thread (b, r, tl), line 2b + r; tmp[row][2k' + r] = (-1)^k' i^r FFT(s x tw2^r)[k']
template <typename T, int LOGN, int B>
__global__ void __launch_bounds__((2 * B * Plan1D<T, LOGN, 0>::TL))
k_fft_rows_fwd(const cpx<T>* __restrict__ x, cpx<T>* __restrict__ tmp, const T* __restrict__ deap,
               const cpx<T>* __restrict__ tw, const cpx<T>* __restrict__ tw2) {
    using PL = Plan1D<T, LOGN, 0>;
    constexpr int N = PL::N, K = 2 * N;
    extern __shared__ unsigned char smem_raw[];
    cpx<T>* base = reinterpret_cast<cpx<T>*>(smem_raw);
    const cpx<T>* W = stage_twiddles<T, LOGN>(base, tw);
    const int tl = threadIdx.x % PL::TL, r = (threadIdx.x / PL::TL) & 1, lr = threadIdx.x / (2 * PL::TL);
    cpx<T>* line = base + table_elems<T, LOGN>() + (2 * lr + r) * PL::LS;
    const int row = blockIdx.x * B + lr;
    const T srow = deap[row];
    const cpx<T>* xr = x + (size_t)row * N;
    cpx<T>* outr = tmp + (size_t)row * K;
    // short lines: S and the parity twiddles are read before the barrier too
    constexpr bool PRE = PL::RMAX <= 8 && 2 * B * PL::TL <= 512;   // register budget
    // one row a workgroup: group 0 alone loads the row and hands S x to group 1 through
    // group 1's line buffer
    constexpr bool SHARE = B == 1;
    cpx<T> v[PL::RMAX];
    if (!SHARE || r == 0) {
#pragma unroll
        for (int i = 0; i < PL::RMAX; ++i) v[i] = xr[PL::in_pos(tl, i)];
    }
    T dq[PRE ? PL::RMAX : 1];
    cpx<T> t2[PRE ? PL::RMAX : 1];
    if constexpr (PRE) {
#pragma unroll
        for (int i = 0; i < PL::RMAX; ++i) {
            const int p = PL::in_pos(tl, i);
            dq[i] = deap[p];
            t2[i] = r ? tw2[p] : mk<T>(1, 0);
        }
    }
    if constexpr (SHARE) {
        cpx<T>* line1 = line + (1 - r) * PL::LS;
        if (r == 0) {
#pragma unroll
            for (int i = 0; i < PL::RMAX; ++i) {
                v[i] = (srow * (PRE ? dq[i] : deap[PL::in_pos(tl, i)])) * v[i];
                line1[PL::in_at(tl, i)] = v[i];
            }
        }
        __syncthreads();   // also: the twiddle table is staged
        if (r == 1) {
#pragma unroll
            for (int i = 0; i < PL::RMAX; ++i) v[i] = line[PL::in_at(tl, i)] * (PRE ? t2[i] : tw2[PL::in_pos(tl, i)]);
        }
    }
    __syncthreads();   // the twiddle table is staged (one row a workgroup: group 1 has read its buffer)
    if constexpr (!SHARE) {
#pragma unroll
        for (int i = 0; i < PL::RMAX; ++i) {
            const int p = PL::in_pos(tl, i);
            cpx<T> a;
            if constexpr (PRE) {
                a = (srow * dq[i]) * v[i];
                if (r) a = a * t2[i];
            } else {
                a = (srow * deap[p]) * v[i];
                if (r) a = a * tw2[p];
            }
            v[i] = a;
        }
    }
    line_fft<T, LOGN, 0, false>(v, line, tl, W);
    store_row_fwd<T, LOGN>(v, line - r * PL::LS, outr, tl, r);
}

// CG set-up folded into the first step's row pass: r = p = x1 + x2 + x3 - q0 (q0 may be
// null), partial ||r||^2 per workgroup, and p's row transform.
template <typename T>
struct CgInit {
    const cpx<T>* x1 = nullptr;
    const cpx<T>* x2 = nullptr;
    const cpx<T>* x3 = nullptr;
    const cpx<T>* q0 = nullptr;
    cpx<T>* r = nullptr;
    cpx<T>* p = nullptr;
    double* rho_part = nullptr;
};

template <typename T, int LOGN, int B>
__global__ void __launch_bounds__((2 * B * Plan1D<T, LOGN, 0>::TL))
k_fft_rows_init(cpx<T>* __restrict__ tmp, const T* __restrict__ deap, const cpx<T>* __restrict__ tw,
                const cpx<T>* __restrict__ tw2, CgInit<T> ci) {
    using PL = Plan1D<T, LOGN, 0>;
    constexpr int N = PL::N, K = 2 * N;
    extern __shared__ unsigned char smem_raw[];
    cpx<T>* base = reinterpret_cast<cpx<T>*>(smem_raw);
    __shared__ double red[16];
    const cpx<T>* W = stage_twiddles<T, LOGN>(base, tw);
    const int tl = threadIdx.x % PL::TL, r = (threadIdx.x / PL::TL) & 1, lr = threadIdx.x / (2 * PL::TL);
    cpx<T>* line = base + table_elems<T, LOGN>() + (2 * lr + r) * PL::LS;
    const int row = blockIdx.x * B + lr;
    const T srow = deap[row];
    const size_t ro = (size_t)row * N;
    cpx<T>* outr = tmp + (size_t)row * K;
    // one row a workgroup: group 0 alone loads the row and hands S r to group 1 through
    // group 1's line buffer; otherwise both parity groups load the whole row
    constexpr bool SHARE = B == 1;
    cpx<T> v[PL::RMAX];
    double acc = 0;
    if (!SHARE || r == 0) {
#pragma unroll
        for (int i = 0; i < PL::RMAX; ++i) {
            const int p = PL::in_pos(tl, i);
            cpx<T> b = ci.x1[ro + p] + ci.x2[ro + p] + ci.x3[ro + p];
            if (ci.q0) b = b - ci.q0[ro + p];
            v[i] = b;
            acc += (double)b.x * b.x + (double)b.y * b.y;
        }
    }
    // group 0 writes r and p and counts ||r||^2
    if (r == 0) {
#pragma unroll
        for (int i = 0; i < PL::RMAX; ++i) {
            const int p = PL::in_pos(tl, i);
            ci.r[ro + p] = v[i];
            ci.p[ro + p] = v[i];
        }
    }
    const double tot = block_sum_dyn(r == 0 ? acc : 0.0, red);   // also orders the twiddle staging
    if (threadIdx.x == 0) ci.rho_part[blockIdx.x] = tot;
    if constexpr (SHARE) {
        cpx<T>* line1 = line + (1 - r) * PL::LS;
        if (r == 0) {
#pragma unroll
            for (int i = 0; i < PL::RMAX; ++i) {
                v[i] = (srow * deap[PL::in_pos(tl, i)]) * v[i];
                line1[PL::in_at(tl, i)] = v[i];
            }
        }
        __syncthreads();
        if (r == 1) {
#pragma unroll
            for (int i = 0; i < PL::RMAX; ++i) v[i] = line[PL::in_at(tl, i)] * tw2[PL::in_pos(tl, i)];
        }
        __syncthreads();   // group 1 has read its buffer before the first pass rewrites it
    } else {
#pragma unroll
        for (int i = 0; i < PL::RMAX; ++i) {
            const int p = PL::in_pos(tl, i);
            cpx<T> a = (srow * deap[p]) * v[i];
            if (r) a = a * tw2[p];
            v[i] = a;
        }
    }
    line_fft<T, LOGN, 0, false>(v, line, tl, W);
    store_row_fwd<T, LOGN>(v, line - r * PL::LS, outr, tl, r);
}

// rows pass of a CG step from the second on (see CgXr): loads x, r, p, q of the row, then
// the partial sums; updates x, r and p, transforms the new p.
template <typename T, int LOGN, int B>
__global__ void __launch_bounds__((2 * B * Plan1D<T, LOGN, 0>::TL))
k_fft_rows_xr(cpx<T>* __restrict__ tmp, const T* __restrict__ deap, const cpx<T>* __restrict__ tw,
              const cpx<T>* __restrict__ tw2, CgXr<T> cg) {
    using PL = Plan1D<T, LOGN, 0>;
    constexpr int N = PL::N, K = 2 * N;
    extern __shared__ unsigned char smem_raw[];
    cpx<T>* base = reinterpret_cast<cpx<T>*>(smem_raw);
    __shared__ double red[32];
    const cpx<T>* W = stage_twiddles<T, LOGN>(base, tw);
    const int tl = threadIdx.x % PL::TL, r = (threadIdx.x / PL::TL) & 1, lr = threadIdx.x / (2 * PL::TL);
    cpx<T>* line = base + table_elems<T, LOGN>() + (2 * lr + r) * PL::LS;
    const int row = blockIdx.x * B + lr;
    const T srow = deap[row];
    const size_t ro = (size_t)row * N;
    cpx<T>* outr = tmp + (size_t)row * K;
    // the row's loads are issued before the partial sums are read, so both are in flight
    // (x only by parity group 0, which writes the row back)
    // One row a workgroup: parity group 0 alone loads and updates the row and hands the new
    // direction to group 1 through group 1's line buffer
    constexpr bool PRE = PL::RMAX <= 8 && 2 * B * PL::TL <= 512;   // register budget
    constexpr bool SHARE = B == 1;
    cpx<T> xv[PL::RMAX], rv[PL::RMAX], pv[PL::RMAX], qv[PL::RMAX];
    if (!SHARE || r == 0) {
#pragma unroll
        for (int i = 0; i < PL::RMAX; ++i) {
            const int p = PL::in_pos(tl, i);
            rv[i] = cg.r[ro + p];
            pv[i] = cg.p[ro + p];
            qv[i] = cg.q[ro + p];
        }
    }
    if (r == 0) {
#pragma unroll
        for (int i = 0; i < PL::RMAX; ++i) xv[i] = cg.x[ro + PL::in_pos(tl, i)];
    }
    // short lines: the transform's S and parity twiddles are read here too
    T dq[PRE ? PL::RMAX : 1];
    cpx<T> t2[PRE ? PL::RMAX : 1];
    if constexpr (PRE) {
#pragma unroll
        for (int i = 0; i < PL::RMAX; ++i) {
            const int p = PL::in_pos(tl, i);
            dq[i] = deap[p];
            t2[i] = r ? tw2[p] : mk<T>(1, 0);
        }
    }
    double rho, pq, rq, qq;
    sum_parts2_dyn(cg.rho_part, cg.rho_count, cg.pq_part, cg.pq_count, red, rho, pq);
    sum_parts2_dyn(cg.rq_part, cg.pq_count, cg.qq_part, cg.pq_count, red, rq, qq);
    const double al = rho == 0.0 ? 0.0 : rho / pq;
    const double rn = rho - 2.0 * al * rq + al * al * qq;
    const T alpha = (T)al, beta = (T)(rho == 0.0 || !(rn > 0.0) ? 0.0 : rn / rho);
    double acc = 0;
    if (!SHARE || r == 0) {
#pragma unroll
        for (int i = 0; i < PL::RMAX; ++i) {
            if (r == 0) xv[i] = xv[i] + alpha * pv[i];
            rv[i] = rv[i] - alpha * qv[i];
            acc += (double)rv[i].x * rv[i].x + (double)rv[i].y * rv[i].y;
            pv[i] = rv[i] + beta * pv[i];
        }
    }
    // both parity groups hold the whole row; group 0 writes it back once all have read it
    if constexpr (!SHARE) __syncthreads();
    if (r == 0) {
#pragma unroll
        for (int i = 0; i < PL::RMAX; ++i) {
            const int p = PL::in_pos(tl, i);
            // streaming stores: x, r and p are next read several launches later, so they
            // should not push the row transforms this pass writes out of the caches
            __builtin_nontemporal_store(xv[i].x, &cg.x[ro + p].x);
            __builtin_nontemporal_store(xv[i].y, &cg.x[ro + p].y);
            __builtin_nontemporal_store(rv[i].x, &cg.r[ro + p].x);
            __builtin_nontemporal_store(rv[i].y, &cg.r[ro + p].y);
            __builtin_nontemporal_store(pv[i].x, &cg.p[ro + p].x);
            __builtin_nontemporal_store(pv[i].y, &cg.p[ro + p].y);
        }
    }
    const double tot = block_sum_dyn(r == 0 ? acc : 0.0, red);
    if (threadIdx.x == 0) cg.rho_new_part[blockIdx.x] = tot;
    if constexpr (SHARE) {
        // group 0: S p into its registers and into group 1's line buffer; group 1 then
        // applies its parity twiddles; a barrier before the first pass rewrites the buffer
        cpx<T>* line1 = line + (1 - r) * PL::LS;
        if (r == 0) {
#pragma unroll
            for (int i = 0; i < PL::RMAX; ++i) {
                const int p = PL::in_pos(tl, i);
                pv[i] = (srow * (PRE ? dq[i] : deap[p])) * pv[i];
                line1[PL::in_at(tl, i)] = pv[i];
            }
        }
        __syncthreads();
        if (r == 1) {
#pragma unroll
            for (int i = 0; i < PL::RMAX; ++i) pv[i] = line[PL::in_at(tl, i)] * (PRE ? t2[i] : tw2[PL::in_pos(tl, i)]);
        }
        __syncthreads();
    } else {
#pragma unroll
        for (int i = 0; i < PL::RMAX; ++i) {
            const int p = PL::in_pos(tl, i);
            cpx<T> a;
            if constexpr (PRE) {
                a = (srow * dq[i]) * pv[i];
                if (r) a = a * t2[i];
            } else {
                a = (srow * deap[p]) * pv[i];
                if (r) a = a * tw2[p];
            }
            pv[i] = a;
        }
    }
    line_fft<T, LOGN, 0, false>(pv, line, tl, W);
    store_row_fwd<T, LOGN>(pv, line - r * PL::LS, outr, tl, r);
}

// cols_fwd: thread (c, r, tl) with c fastest (coalesced runs of C columns)
template <typename T, int LOGN, int C>
__global__ void __launch_bounds__((2 * C * Plan1D<T, LOGN, 1>::TL))
k_fft_cols_fwd(const cpx<T>* __restrict__ tmp, cpx<T>* __restrict__ grid, const cpx<T>* __restrict__ tw,
               const cpx<T>* __restrict__ tw2, int sg) {
    using PL = Plan1D<T, LOGN, 1>;
    constexpr int N = PL::N, K = 2 * N;
    extern __shared__ unsigned char smem_raw[];
    cpx<T>* base = reinterpret_cast<cpx<T>*>(smem_raw);
    const cpx<T>* W = stage_twiddles<T, LOGN>(base, tw);
    const int c = threadIdx.x % C, r = (threadIdx.x / C) & 1, tl = threadIdx.x / (2 * C);
    cpx<T>* line = base + table_elems<T, LOGN>() + (2 * c + r) * PL::LS;
    const int col = strip_block(sg) * C + c;
    __syncthreads();
    cpx<T> v[PL::RMAX];
#pragma unroll
    for (int i = 0; i < PL::RMAX; ++i) v[i] = tmp[(size_t)PL::in_pos(tl, i) * K + col];
    constexpr bool PRE = PL::RMAX <= 8 && 2 * C * PL::TL <= 512;   // register budget
    cpx<T> t2[PRE ? PL::RMAX : 1];
    if constexpr (PRE) {
#pragma unroll
        for (int i = 0; i < PL::RMAX; ++i) t2[i] = r ? tw2[PL::in_pos(tl, i)] : mk<T>(1, 0);
    }
#pragma unroll
    for (int i = 0; i < PL::RMAX; ++i) {
        if constexpr (PRE) {
            if (r) v[i] = v[i] * t2[i];
        } else {
            if (r) v[i] = v[i] * tw2[PL::in_pos(tl, i)];
        }
    }
    line_fft<T, LOGN, 1, false>(v, line, tl, W);
#pragma unroll
    for (int i = 0; i < PL::RMAX; ++i) {
        const int kp = PL::out_pos(tl, i);
        cpx<T> o = (kp & 1) ? neg(v[i]) : v[i];
        if (r) o = mul_i(o);
        grid[(size_t)(2 * kp + r) * K + col] = o;
    }
}

// Column passes for long columns, where a workgroup's LDS holds only the two parity lines
// of one column: each thread keeps CR adjacent columns in registers, so every row access is
// one contiguous run of CR elements, and the workgroup transforms the columns one after
// another through the same two line buffers.
template <typename T, int LOGN, int CR>
__global__ void __launch_bounds__((2 * Plan1D<T, LOGN, 1>::TL)) __attribute__((amdgpu_waves_per_eu(mc_waves_per_eu<T, LOGN>())))
k_fft_cols_fwd_mc(const cpx<T>* __restrict__ tmp, cpx<T>* __restrict__ grid, const cpx<T>* __restrict__ tw,
                  const cpx<T>* __restrict__ tw2, int sg) {
    using PL = Plan1D<T, LOGN, 1>;
    constexpr int N = PL::N, K = 2 * N;
    extern __shared__ unsigned char smem_raw[];
    cpx<T>* base = reinterpret_cast<cpx<T>*>(smem_raw);
    const cpx<T>* W = stage_twiddles<T, LOGN>(base, tw);
    const int r = threadIdx.x / PL::TL, tl = threadIdx.x % PL::TL;
    cpx<T>* line = base + table_elems<T, LOGN>() + r * PL::LS;
    const int col0 = strip_block(sg) * CR;
    const cpx<T>* T2 = mc_stage_tw2<T, LOGN>(base + table_elems<T, LOGN>(), tw2);
    __syncthreads();
    cpx<T> v[CR][PL::RMAX];
#pragma unroll
    for (int i = 0; i < PL::RMAX; ++i) {
        const size_t ro = (size_t)PL::in_pos(tl, i) * K + col0;
#pragma unroll
        for (int cc = 0; cc < CR; ++cc) v[cc][i] = tmp[ro + cc];
    }
    if (r) {
#pragma unroll
        for (int i = 0; i < PL::RMAX; ++i) {
            const cpx<T> t = T2[PL::in_pos(tl, i)];
#pragma unroll
            for (int cc = 0; cc < CR; ++cc) v[cc][i] = v[cc][i] * t;
        }
    }
    // each transform's last pass reads the line before a barrier, so the next column may
    // overwrite it
#pragma unroll
    for (int cc = 0; cc < CR; ++cc) line_fft<T, LOGN, 1, false>(v[cc], line, tl, W);
#pragma unroll
    for (int i = 0; i < PL::RMAX; ++i) {
        const int kp = PL::out_pos(tl, i);
        const size_t ro = (size_t)(2 * kp + r) * K + col0;
#pragma unroll
        for (int cc = 0; cc < CR; ++cc) {
            cpx<T> o = (kp & 1) ? neg(v[cc][i]) : v[cc][i];
            if (r) o = mul_i(o);
            grid[ro + cc] = o;
        }
    }
}

template <typename T, int LOGN, int CR>
__global__ void __launch_bounds__((2 * Plan1D<T, LOGN, 1>::TL)) __attribute__((amdgpu_waves_per_eu(mc_waves_per_eu<T, LOGN>())))
k_fft_cols_adj_mc(const cpx<T>* __restrict__ grid, cpx<T>* __restrict__ tmp, const cpx<T>* __restrict__ tw,
                  const cpx<T>* __restrict__ tw2, int sg) {
    using PL = Plan1D<T, LOGN, 1>;
    constexpr int N = PL::N, K = 2 * N;
    extern __shared__ unsigned char smem_raw[];
    cpx<T>* base = reinterpret_cast<cpx<T>*>(smem_raw);
    const cpx<T>* W = stage_twiddles<T, LOGN>(base, tw);
    const int r = threadIdx.x / PL::TL, tl = threadIdx.x % PL::TL;
    cpx<T>* lines = base + table_elems<T, LOGN>();
    cpx<T>* line = lines + r * PL::LS;
    const int col0 = strip_block(sg) * CR;
    constexpr int NQ = PL::RMAX / 2;
    const cpx<T>* T2 = mc_stage_tw2<T, LOGN>(lines, tw2);
    __syncthreads();
    // The (-1)^k' factor of the input is left out: it shifts each transform by n/2, so the
    // combine reads position j + n/2 (mod n) of the lines instead.  The loads then have no
    // use before the transforms and are all in flight together.
    static_assert(PL::RMAX % 4 == 0, "the n/2 shift is a whole number of combine slots");
    cpx<T> v[CR][PL::RMAX];
#pragma unroll
    for (int i = 0; i < PL::RMAX; ++i) {
        const size_t ro = (size_t)(2 * PL::in_pos(tl, i) + r) * K + col0;
#pragma unroll
        for (int cc = 0; cc < CR; ++cc) v[cc][i] = grid[ro + cc];
    }
    cpx<T> res[CR][NQ];
#pragma unroll
    for (int cc = 0; cc < CR; ++cc) {
        line_fft<T, LOGN, 1, true>(v[cc], line, tl, W);
        __syncthreads();
#pragma unroll
        for (int i = 0; i < PL::RMAX; ++i) line[PL::out_at(tl, i)] = v[cc][i];
        __syncthreads();
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const int a = PL::at(r + 2 * tl) + PL::span(((q + NQ / 2) % NQ) * 2 * PL::TL);
            res[cc][q] = lines[a] + mul_mi(mulc(lines[PL::LS + a], T2[r + 2 * tl + q * 2 * PL::TL]));
        }
        __syncthreads();   // the next column reuses the lines
    }
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const int j = r + 2 * tl + q * 2 * PL::TL;
#pragma unroll
        for (int cc = 0; cc < CR; ++cc) tmp[(size_t)j * K + col0 + cc] = res[cc][q];
    }
}

// cols_adj: parity lines transformed in parallel, results meet in LDS, then
// tmp[j][col] = A[j] + (-i) exp(pi i j / n) B[j]
template <typename T, int LOGN, int C>
__global__ void __launch_bounds__((2 * C * Plan1D<T, LOGN, 1>::TL))
k_fft_cols_adj(const cpx<T>* __restrict__ grid, cpx<T>* __restrict__ tmp, const cpx<T>* __restrict__ tw,
               const cpx<T>* __restrict__ tw2, int sg) {
    using PL = Plan1D<T, LOGN, 1>;
    constexpr int N = PL::N, K = 2 * N;
    extern __shared__ unsigned char smem_raw[];
    cpx<T>* base = reinterpret_cast<cpx<T>*>(smem_raw);
    const cpx<T>* W = stage_twiddles<T, LOGN>(base, tw);
    const int c = threadIdx.x % C, r = (threadIdx.x / C) & 1, tl = threadIdx.x / (2 * C);
    cpx<T>* lines = base + table_elems<T, LOGN>();
    cpx<T>* line = lines + (2 * c + r) * PL::LS;
    const int col = strip_block(sg) * C + c;
    __syncthreads();
    cpx<T> v[PL::RMAX];
#pragma unroll
    for (int i = 0; i < PL::RMAX; ++i) {
        const int kp = PL::in_pos(tl, i);
        const cpx<T> u = grid[(size_t)(2 * kp + r) * K + col];
        v[i] = (kp & 1) ? neg(u) : u;
    }
    // short lines: the combine's twiddles are read before the transform
    constexpr int NQ = PL::RMAX / 2;
    constexpr bool PRE = PL::RMAX <= 8 && 2 * C * PL::TL <= 512;   // register budget
    cpx<T> tj[PRE ? NQ : 1];
    if constexpr (PRE) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) tj[q] = tw2[r + 2 * tl + q * 2 * PL::TL];
    }
    line_fft<T, LOGN, 1, true>(v, line, tl, W);
    __syncthreads();
#pragma unroll
    for (int i = 0; i < PL::RMAX; ++i) line[PL::out_at(tl, i)] = v[i];
    __syncthreads();
    const cpx<T>* la = lines + (2 * c) * PL::LS;
    const cpx<T>* lb = la + PL::LS;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const int j = r + 2 * tl + q * 2 * PL::TL, a = PL::at(r + 2 * tl) + PL::span(q * 2 * PL::TL);
        if constexpr (PRE) tmp[(size_t)j * K + col] = la[a] + mul_mi(mulc(lb[a], tj[q]));
        else tmp[(size_t)j * K + col] = la[a] + mul_mi(mulc(lb[a], tw2[j]));
    }
}

// Column stage of the stored normal operator T = Z^T F^dagger diag(c_hat) F Z (the Toeplitz
// form of Phi^dagger Phi, Section 3): per column k2 of tmp, the forward transform along axis 0
// (n -> K, parity-split as in cols_fwd), the product with the real spectrum c_hat[k1][k2],
// and the adjoint transform (K -> n, as in cols_adj), in place.  Between the two transforms
// the spectrum goes through the line buffer, from the forward pass's output order to the
// adjoint pass's input order; the (-1)^k' factors of the two cancel.
template <typename T, int LOGN, int C>
__global__ void __launch_bounds__((2 * C * Plan1D<T, LOGN, 1>::TL))
k_fft_cols_toep(const cpx<T>* in, cpx<T>* out, const T* __restrict__ chat, const cpx<T>* __restrict__ tw,
                const cpx<T>* __restrict__ tw2, int sg) {
    using PL = Plan1D<T, LOGN, 1>;
    constexpr int N = PL::N, K = 2 * N;
    extern __shared__ unsigned char smem_raw[];
    cpx<T>* base = reinterpret_cast<cpx<T>*>(smem_raw);
    const cpx<T>* W = stage_twiddles<T, LOGN>(base, tw);
    const int c = threadIdx.x % C, r = (threadIdx.x / C) & 1, tl = threadIdx.x / (2 * C);
    cpx<T>* lines = base + table_elems<T, LOGN>();
    cpx<T>* line = lines + (2 * c + r) * PL::LS;
    const int col = strip_block(sg) * C + c;
    __syncthreads();
    cpx<T> v[PL::RMAX];
#pragma unroll
    for (int i = 0; i < PL::RMAX; ++i) v[i] = in[(size_t)PL::in_pos(tl, i) * K + col];
#pragma unroll
    for (int i = 0; i < PL::RMAX; ++i) {
        if (r) v[i] = v[i] * tw2[PL::in_pos(tl, i)];
    }
    line_fft<T, LOGN, 1, false>(v, line, tl, W);
    // frequency k1 = 2k' + r holds (-1)^k' i^r v; the adjoint reads (-1)^k' times its input
#pragma unroll
    for (int i = 0; i < PL::RMAX; ++i) {
        const int kp = PL::out_pos(tl, i);
        cpx<T> o = chat[(size_t)(2 * kp + r) * K + col] * v[i];
        v[i] = r ? mul_i(o) : o;
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < PL::RMAX; ++i) line[PL::out_at(tl, i)] = v[i];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < PL::RMAX; ++i) v[i] = line[PL::in_at(tl, i)];
    __syncthreads();
    line_fft<T, LOGN, 1, true>(v, line, tl, W);
    __syncthreads();
#pragma unroll
    for (int i = 0; i < PL::RMAX; ++i) line[PL::out_at(tl, i)] = v[i];
    __syncthreads();
    const cpx<T>* la = lines + (2 * c) * PL::LS;
    const cpx<T>* lb = la + PL::LS;
#pragma unroll
    for (int q = 0; q < PL::RMAX / 2; ++q) {
        const int j = r + 2 * tl + q * 2 * PL::TL, a = PL::at(r + 2 * tl) + PL::span(q * 2 * PL::TL);
        out[(size_t)j * K + col] = la[a] + mul_mi(mulc(lb[a], tw2[j]));
    }
}


// The stored normal operator's column stage for long columns: each thread keeps CR adjacent
// columns in registers (32-byte runs of a row, as in k_fft_cols_fwd_mc) and the workgroup
// takes them one after another through the same two line buffers, each column with the same
// arithmetic as k_fft_cols_toep; a column's adjoint output replaces its input in registers and
// all CR columns are written at the end (in place is safe: every read precedes every write).
template <typename T, int LOGN, int CR>
__global__ void __launch_bounds__((2 * Plan1D<T, LOGN, 1>::TL)) __attribute__((amdgpu_waves_per_eu(mc_waves_per_eu<T, LOGN>())))
k_fft_cols_toep_mc(const cpx<T>* in, cpx<T>* out, const T* __restrict__ chat, const cpx<T>* __restrict__ tw,
                   const cpx<T>* __restrict__ tw2, int sg) {
    using PL = Plan1D<T, LOGN, 1>;
    constexpr int N = PL::N, K = 2 * N;
    extern __shared__ unsigned char smem_raw[];
    cpx<T>* base = reinterpret_cast<cpx<T>*>(smem_raw);
    const cpx<T>* W = stage_twiddles<T, LOGN>(base, tw);
    const int r = threadIdx.x / PL::TL, tl = threadIdx.x % PL::TL;
    cpx<T>* lines = base + table_elems<T, LOGN>();
    cpx<T>* line = lines + r * PL::LS;
    const int col0 = strip_block(sg) * CR;
    const cpx<T>* T2 = mc_stage_tw2<T, LOGN>(lines, tw2);
    __syncthreads();
    cpx<T> v[CR][PL::RMAX];
#pragma unroll
    for (int i = 0; i < PL::RMAX; ++i) {
        const size_t ro = (size_t)PL::in_pos(tl, i) * K + col0;
#pragma unroll
        for (int cc = 0; cc < CR; ++cc) v[cc][i] = in[ro + cc];
    }
    if (r) {
#pragma unroll
        for (int i = 0; i < PL::RMAX; ++i) {
            const cpx<T> t = T2[PL::in_pos(tl, i)];
#pragma unroll
            for (int cc = 0; cc < CR; ++cc) v[cc][i] = v[cc][i] * t;
        }
    }
#pragma unroll
    for (int cc = 0; cc < CR; ++cc) {
        line_fft<T, LOGN, 1, false>(v[cc], line, tl, W);
        // frequency k1 = 2k' + r holds (-1)^k' i^r v; the adjoint reads (-1)^k' times its input
#pragma unroll
        for (int i = 0; i < PL::RMAX; ++i) {
            const int kp = PL::out_pos(tl, i);
            cpx<T> o = chat[((size_t)(col0 / CR) * K + 2 * kp + r) * CR + cc] * v[cc][i];
            v[cc][i] = r ? mul_i(o) : o;
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < PL::RMAX; ++i) line[PL::out_at(tl, i)] = v[cc][i];
        __syncthreads();
#pragma unroll
        for (int i = 0; i < PL::RMAX; ++i) v[cc][i] = line[PL::in_at(tl, i)];
        __syncthreads();
        line_fft<T, LOGN, 1, true>(v[cc], line, tl, W);
        __syncthreads();
#pragma unroll
        for (int i = 0; i < PL::RMAX; ++i) line[PL::out_at(tl, i)] = v[cc][i];
        __syncthreads();
#pragma unroll
        for (int q = 0; q < PL::RMAX / 2; ++q) {
            const int j = r + 2 * tl + q * 2 * PL::TL, a = PL::at(r + 2 * tl) + PL::span(q * 2 * PL::TL);
            v[cc][q] = lines[a] + mul_mi(mulc(lines[PL::LS + a], T2[j]));
        }
        __syncthreads();   // the next column reuses the lines
    }
#pragma unroll
    for (int q = 0; q < PL::RMAX / 2; ++q) {
        const int j = r + 2 * tl + q * 2 * PL::TL;
#pragma unroll
        for (int cc = 0; cc < CR; ++cc) out[(size_t)j * K + col0 + cc] = v[cc][q];
    }
}

// rows_adj: thread (b, tl, r) with r fastest; parity lines in parallel, combined in LDS;
// x[row][j] = c1 s_row s_j (A[j] + (-i) exp(pi i j/n) B[j]) + c2 v, partial Re<v, x>
template <typename T, int LOGN, int B>
__global__ void __launch_bounds__((2 * B * Plan1D<T, LOGN, 0>::TL))
k_fft_rows_adj(const cpx<T>* __restrict__ tmp, cpx<T>* __restrict__ x, const T* __restrict__ deap,
               const cpx<T>* __restrict__ tw, const cpx<T>* __restrict__ tw2, T c1,
               const cpx<T>* __restrict__ vin, T c2, double* __restrict__ dot_part, CgDots<T> dots) {
    using PL = Plan1D<T, LOGN, 0>;
    constexpr int N = PL::N, K = 2 * N;
    extern __shared__ unsigned char smem_raw[];
    cpx<T>* base = reinterpret_cast<cpx<T>*>(smem_raw);
    __shared__ double red[48];
    const cpx<T>* W = stage_twiddles<T, LOGN>(base, tw);
    const int r = threadIdx.x & 1, tl = (threadIdx.x >> 1) % PL::TL, lr = threadIdx.x / (2 * PL::TL);
    cpx<T>* lines = base + table_elems<T, LOGN>() + (2 * lr) * PL::LS;
    cpx<T>* line = lines + r * PL::LS;
    const int row = blockIdx.x * B + lr;
    const cpx<T>* inr = tmp + (size_t)row * K;
    __syncthreads();
    cpx<T> v[PL::RMAX];
#pragma unroll
    for (int i = 0; i < PL::RMAX; ++i) {
        const int kp = PL::in_pos(tl, i);
        const cpx<T> u = inr[2 * kp + r];
        v[i] = (kp & 1) ? neg(u) : u;
    }
    // The epilogue's operands (v, and r of the CG dot products) are read before the
    // transform, so their loads overlap the input's (short lines; long lines read them in the
    // epilogue).
    constexpr int NQ = PL::RMAX / 2;
    constexpr bool PRE = PL::RMAX <= 8 && 2 * B * PL::TL <= 512;   // register budget
    cpx<T> pv[PRE ? NQ : 1], pr[PRE ? NQ : 1], tj[PRE ? NQ : 1];
    T dj[PRE ? NQ : 1];
    if constexpr (PRE) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const int j = r + 2 * tl + q * 2 * PL::TL;
            const size_t off = (size_t)row * N + j;
            if (vin) pv[q] = vin[off];
            if (dots.r) pr[q] = dots.r[off];
            tj[q] = tw2[j];
            dj[q] = deap[j];
        }
    }
    line_fft<T, LOGN, 0, true>(v, line, tl, W);
    __syncthreads();
#pragma unroll
    for (int i = 0; i < PL::RMAX; ++i) line[PL::out_at(tl, i)] = v[i];
    __syncthreads();
    const T srow = c1 * deap[row];
    double acc = 0.0, arq = 0.0, aqq = 0.0;
    // the epilogue, one straight-line copy per operand set (long lines: its operands are
    // loaded first, all before the first store, so they are in flight together)
    auto epilogue = [&](auto has_v, auto has_r) {
        constexpr bool HV = decltype(has_v)::value, HR = decltype(has_r)::value;
        cpx<T> ev[PRE ? 1 : NQ], er[PRE ? 1 : NQ], et[PRE ? 1 : NQ];
        T ed[PRE ? 1 : NQ];
        if constexpr (!PRE) {
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                const int j = r + 2 * tl + q * 2 * PL::TL;
                const size_t off = (size_t)row * N + j;
                if constexpr (HV) ev[q] = vin[off];
                if constexpr (HR) er[q] = dots.r[off];
                et[q] = tw2[j];
                ed[q] = deap[j];
            }
        }
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const int j = r + 2 * tl + q * 2 * PL::TL, a = PL::at(r + 2 * tl) + PL::span(q * 2 * PL::TL);
            cpx<T> o;
            if constexpr (PRE) {
                const cpx<T> t = lines[a] + mul_mi(mulc(lines[PL::LS + a], tj[q]));
                o = (srow * dj[q]) * t;
            } else {
                const cpx<T> t = lines[a] + mul_mi(mulc(lines[PL::LS + a], et[q]));
                o = (srow * ed[q]) * t;
            }
            if constexpr (HV) {
                const cpx<T> vv = PRE ? pv[q] : ev[PRE ? 0 : q];
                o = o + c2 * vv;
                acc += (double)vv.x * (double)o.x + (double)vv.y * (double)o.y;
            }
            if constexpr (HR) {
                const cpx<T> rr = PRE ? pr[q] : er[PRE ? 0 : q];
                arq += (double)rr.x * (double)o.x + (double)rr.y * (double)o.y;
                aqq += (double)o.x * (double)o.x + (double)o.y * (double)o.y;
            }
            __builtin_nontemporal_store(o.x, &x[(size_t)row * N + j].x);   // streaming, as in the
            __builtin_nontemporal_store(o.y, &x[(size_t)row * N + j].y);   // CG row pass
        }
    };
    if (vin && dots.r) epilogue(std::true_type{}, std::true_type{});
    else if (vin) epilogue(std::true_type{}, std::false_type{});
    else epilogue(std::false_type{}, std::false_type{});
    if (dots.r) {
        double t0, t1, t2;
        block_sum3_dyn(acc, arq, aqq, red, t0, t1, t2);
        if (threadIdx.x == 0) {
            dot_part[blockIdx.x] = t0;
            dots.rq_part[blockIdx.x] = t1;
            dots.qq_part[blockIdx.x] = t2;
        }
    } else if (dot_part) {
        const double tot = block_sum_dyn(acc, red);
        if (threadIdx.x == 0) dot_part[blockIdx.x] = tot;
    }
}

// Column groups per gridding-tile strip when the plan's work list is strip-ordered (see
// strip_block), else 0.
int strip_groups(const Plan& P, int C) {
    return (P.strip_xcd && P.TT % C == 0) ? P.TT / C : 0;
}

// Raises a kernel's dynamic LDS limit above 64 KB once per process (per kernel and size),
// under a lock: solves on several host threads (the server) then never change a kernel's
// attribute while another thread launches or captures it at a size it already allows.
std::mutex g_lds_mu;
std::map<const void*, size_t> g_lds_set;

template <typename F>
void set_lds_limit(F* f, size_t bytes) {
    if (bytes <= 65536) return;
    const void* k = reinterpret_cast<const void*>(f);
    std::lock_guard<std::mutex> lk(g_lds_mu);
    auto it = g_lds_set.find(k);
    if (it != g_lds_set.end() && it->second >= bytes) return;
    if (hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) == hipSuccess)
        g_lds_set[k] = bytes;
}

template <typename T, int LOGN, int AX>
constexpr size_t lds_bytes(int lines) {
    using PL = Plan1D<T, LOGN, AX>;
    return (size_t)(table_elems<T, LOGN>() + lines * PL::LS) * sizeof(cpx<T>);
}

template <typename T, int LOGN>
void rows_fwd_impl(const Plan& P, const cpx<T>* x, cpx<T>* tmp, const T* deap, hipStream_t s) {
    constexpr int B = rows_per_wg<T, LOGN>();
    constexpr int NT = 2 * B * Plan1D<T, LOGN, 0>::TL;
    constexpr int N = 1 << LOGN;
    const size_t lds = lds_bytes<T, LOGN, 0>(2 * B);
    auto f = k_fft_rows_fwd<T, LOGN, B>;
    set_lds_limit(f, lds);
    hipLaunchKernelGGL(f, dim3(N / B), dim3(NT), lds, s, x, tmp, deap, (const cpx<T>*)P.tw,
                       (const cpx<T>*)P.tw2);
}
template <typename T, int LOGN>
void rows_xr_impl(const Plan& P, cpx<T>* tmp, CgXr<T> cg, const T* deap, hipStream_t s) {
    constexpr int B = rows_per_wg<T, LOGN>();
    constexpr int NT = 2 * B * Plan1D<T, LOGN, 0>::TL;
    constexpr int N = 1 << LOGN;
    const size_t lds = lds_bytes<T, LOGN, 0>(2 * B);
    auto f = k_fft_rows_xr<T, LOGN, B>;
    set_lds_limit(f, lds);
    hipLaunchKernelGGL(f, dim3(N / B), dim3(NT), lds, s, tmp, deap, (const cpx<T>*)P.tw, (const cpx<T>*)P.tw2, cg);
}
template <typename T, int LOGN>
void rows_init_impl(const Plan& P, cpx<T>* tmp, CgInit<T> ci, const T* deap, hipStream_t s) {
    constexpr int B = rows_per_wg<T, LOGN>();
    constexpr int NT = 2 * B * Plan1D<T, LOGN, 0>::TL;
    constexpr int N = 1 << LOGN;
    const size_t lds = lds_bytes<T, LOGN, 0>(2 * B);
    auto f = k_fft_rows_init<T, LOGN, B>;
    set_lds_limit(f, lds);
    hipLaunchKernelGGL(f, dim3(N / B), dim3(NT), lds, s, tmp, deap, (const cpx<T>*)P.tw, (const cpx<T>*)P.tw2, ci);
}
template <typename T, int LOGN>
void cols_fwd_impl(const Plan& P, const cpx<T>* tmp, cpx<T>* grid, hipStream_t s) {
    constexpr int C = cols_per_wg<T, LOGN>();
    constexpr int NT = 2 * C * Plan1D<T, LOGN, 1>::TL;
    constexpr int N = 1 << LOGN;
    const size_t lds = lds_bytes<T, LOGN, 1>(2 * C);
    if constexpr (long_cols<T, LOGN>()) {   // long columns: CR columns per thread in registers
        constexpr int CR = long_cols_cr<T, LOGN>();
        const size_t lds1 = mc_lds_bytes<T, LOGN>();
        // each XCD takes one contiguous range of column groups (sg = 0), so the groups that
        // share 128-byte lines run on one L2 at about the same time (the adjoint 559 -> 506 us
        // at n = 4096 against the gridding-strip order)
        auto f = k_fft_cols_fwd_mc<T, LOGN, CR>;
        set_lds_limit(f, lds1);
        hipLaunchKernelGGL(f, dim3(2 * N / CR), dim3(2 * Plan1D<T, LOGN, 1>::TL), lds1, s, tmp, grid,
                           (const cpx<T>*)P.tw, (const cpx<T>*)P.tw2, 0);
        return;
    }
    auto f = k_fft_cols_fwd<T, LOGN, C>;
    set_lds_limit(f, lds);
    hipLaunchKernelGGL(f, dim3(2 * N / C), dim3(NT), lds, s, tmp, grid, (const cpx<T>*)P.tw,
                       (const cpx<T>*)P.tw2, strip_groups(P, C));
}
template <typename T, int LOGN>
void cols_adj_impl(const Plan& P, const cpx<T>* grid, cpx<T>* tmp, hipStream_t s) {
    constexpr int C = cols_per_wg<T, LOGN>();
    constexpr int NT = 2 * C * Plan1D<T, LOGN, 1>::TL;
    constexpr int N = 1 << LOGN;
    const size_t lds = lds_bytes<T, LOGN, 1>(2 * C);
    if constexpr (long_cols<T, LOGN>()) {
        constexpr int CR = long_cols_cr<T, LOGN>();
        const size_t lds1 = mc_lds_bytes<T, LOGN>();
        auto f = k_fft_cols_adj_mc<T, LOGN, CR>;
        set_lds_limit(f, lds1);
        hipLaunchKernelGGL(f, dim3(2 * N / CR), dim3(2 * Plan1D<T, LOGN, 1>::TL), lds1, s, grid, tmp,
                           (const cpx<T>*)P.tw, (const cpx<T>*)P.tw2, 0);
        return;
    }
    auto f = k_fft_cols_adj<T, LOGN, C>;
    set_lds_limit(f, lds);
    hipLaunchKernelGGL(f, dim3(2 * N / C), dim3(NT), lds, s, grid, tmp, (const cpx<T>*)P.tw,
                       (const cpx<T>*)P.tw2, strip_groups(P, C));
}
template <typename T, int LOGN>
void cols_toep_impl(const Plan& P, const cpx<T>* in, cpx<T>* out, hipStream_t s) {
    constexpr int C = cols_per_wg<T, LOGN>();
    constexpr int NT = 2 * C * Plan1D<T, LOGN, 1>::TL;
    constexpr int N = 1 << LOGN;
    const size_t lds = lds_bytes<T, LOGN, 1>(2 * C);
    if constexpr (toep_mc<T, LOGN>()) {
        constexpr int CR = toep_group<T, LOGN>();   // columns per thread, in registers
        const size_t lds1 = mc_lds_bytes<T, LOGN>();
        auto f = k_fft_cols_toep_mc<T, LOGN, CR>;
        set_lds_limit(f, lds1);
        hipLaunchKernelGGL(f, dim3(2 * N / CR), dim3(2 * Plan1D<T, LOGN, 1>::TL), lds1, s, in, out,
                           (const T*)P.chat, (const cpx<T>*)P.tw, (const cpx<T>*)P.tw2, 0);
        return;
    }
    auto f = k_fft_cols_toep<T, LOGN, C>;
    set_lds_limit(f, lds);
    hipLaunchKernelGGL(f, dim3(2 * N / C), dim3(NT), lds, s, in, out, (const T*)P.chat, (const cpx<T>*)P.tw,
                       (const cpx<T>*)P.tw2, strip_groups(P, C));
}
template <typename T, int LOGN>
void rows_adj_impl(const Plan& P, const cpx<T>* tmp, cpx<T>* x, double c1, const cpx<T>* v,
                   double c2, double* dot_part, const T* deap, CgDots<T> dots, hipStream_t s) {
    constexpr int B = rows_per_wg<T, LOGN>();
    constexpr int NT = 2 * B * Plan1D<T, LOGN, 0>::TL;
    constexpr int N = 1 << LOGN;
    const size_t lds = lds_bytes<T, LOGN, 0>(2 * B);
    auto f = k_fft_rows_adj<T, LOGN, B>;
    set_lds_limit(f, lds);
    hipLaunchKernelGGL(f, dim3(N / B), dim3(NT), lds, s, tmp, x, deap, (const cpx<T>*)P.tw,
                       (const cpx<T>*)P.tw2, (T)c1, v, (T)c2, dot_part, dots);
}

int ilog2(int n) {
    int l = 0;
    while ((1 << l) < n) ++l;
    return l;
}

#define PURIFY_LOGN_DISPATCH(LOGN_VAR, CALL)            \
    switch (LOGN_VAR) {                                 \
        case 4: { constexpr int L_ = 4; CALL; } break;  \
        case 5: { constexpr int L_ = 5; CALL; } break;  \
        case 6: { constexpr int L_ = 6; CALL; } break;  \
        case 7: { constexpr int L_ = 7; CALL; } break;  \
        case 8: { constexpr int L_ = 8; CALL; } break;  \
        case 9: { constexpr int L_ = 9; CALL; } break;  \
        case 10: { constexpr int L_ = 10; CALL; } break; \
        case 11: { constexpr int L_ = 11; CALL; } break; \
        case 12: { constexpr int L_ = 12; CALL; } break; \
        default: break;                                 \
    }

}  // namespace

template <typename T>
void launch_fft_rows_fwd(const Plan& P, const cpx<T>* x, cpx<T>* tmp, hipStream_t s, const void* deap) {
    const T* dp = (const T*)(deap ? deap : P.deap);
    PURIFY_LOGN_DISPATCH(ilog2(P.n), (rows_fwd_impl<T, L_>(P, x, tmp, dp, s)));
}
template <typename T>
int launch_fft_rows_init(const Plan& P, const cpx<T>* x1, const cpx<T>* x2, const cpx<T>* x3, const cpx<T>* q0,
                         cpx<T>* r, cpx<T>* p, double* rho_part, cpx<T>* tmp, hipStream_t s, const void* deap) {
    CgInit<T> ci;
    ci.x1 = x1;
    ci.x2 = x2;
    ci.x3 = x3;
    ci.q0 = q0;
    ci.r = r;
    ci.p = p;
    ci.rho_part = rho_part;
    const T* dp = (const T*)(deap ? deap : P.deap);
    int blocks = 0;
    PURIFY_LOGN_DISPATCH(ilog2(P.n), (rows_init_impl<T, L_>(P, tmp, ci, dp, s), blocks = (1 << L_) / rows_per_wg<T, L_>()));
    return blocks;
}
template <typename T>
void launch_fft_cols_fwd(const Plan& P, const cpx<T>* tmp, cpx<T>* grid, hipStream_t s) {
    PURIFY_LOGN_DISPATCH(ilog2(P.n), (cols_fwd_impl<T, L_>(P, tmp, grid, s)));
}
template <typename T>
int launch_fft_rows_xr(const Plan& P, cpx<T>* x, cpx<T>* r, cpx<T>* p, const cpx<T>* q, const double* rho_part,
                       int rho_count, const double* pq_part, const double* rq_part, const double* qq_part,
                       int dot_count, double* rho_new_part, cpx<T>* tmp, hipStream_t s, const void* deap) {
    const T* dp = (const T*)(deap ? deap : P.deap);
    CgXr<T> cg;
    cg.x = x;
    cg.r = r;
    cg.p = p;
    cg.q = q;
    cg.rho_part = rho_part;
    cg.rho_count = rho_count;
    cg.pq_part = pq_part;
    cg.pq_count = dot_count;
    cg.rq_part = rq_part;
    cg.qq_part = qq_part;
    cg.rho_new_part = rho_new_part;
    int blocks = 0;
    PURIFY_LOGN_DISPATCH(ilog2(P.n), (rows_xr_impl<T, L_>(P, tmp, cg, dp, s), blocks = (1 << L_) / rows_per_wg<T, L_>()));
    return blocks;
}
template <typename T>
void launch_fft_rows_adj_cg(const Plan& P, const cpx<T>* tmp, cpx<T>* q, double c1, const cpx<T>* p, double c2,
                            double* pq_part, const cpx<T>* r, double* rq_part, double* qq_part, hipStream_t s,
                            const void* deap) {
    const T* dp = (const T*)(deap ? deap : P.deap);
    CgDots<T> dots;
    dots.r = r;
    dots.rq_part = rq_part;
    dots.qq_part = qq_part;
    PURIFY_LOGN_DISPATCH(ilog2(P.n), (rows_adj_impl<T, L_>(P, tmp, q, c1, p, c2, pq_part, dp, dots, s)));
}
template <typename T>
void launch_fft_cols_adj(const Plan& P, const cpx<T>* grid, cpx<T>* tmp, hipStream_t s) {
    PURIFY_LOGN_DISPATCH(ilog2(P.n), (cols_adj_impl<T, L_>(P, grid, tmp, s)));
}
template <typename T>
void launch_fft_cols_toep(const Plan& P, cpx<T>* tmp, hipStream_t s, const cpx<T>* in) {
    PURIFY_LOGN_DISPATCH(ilog2(P.n), (cols_toep_impl<T, L_>(P, in ? in : tmp, tmp, s)));
}
template <typename T>
void launch_fft_rows_adj(const Plan& P, const cpx<T>* tmp, cpx<T>* x, double c1, const cpx<T>* v,
                         double c2, double* dot_part, hipStream_t s, const void* deap) {
    const T* dp = (const T*)(deap ? deap : P.deap);
    PURIFY_LOGN_DISPATCH(ilog2(P.n), (rows_adj_impl<T, L_>(P, tmp, x, c1, v, c2, dot_part, dp, CgDots<T>{}, s)));
}
template <typename T>
int fft_toep_group(const Plan& P) {
    int w = 0;
    PURIFY_LOGN_DISPATCH(ilog2(P.n), (w = toep_group<T, L_>()));
    return w;
}
template <typename T>
int fft_rows_adj_blocks(const Plan& P) {
    int r = 0;
    PURIFY_LOGN_DISPATCH(ilog2(P.n), (r = (1 << L_) / rows_per_wg<T, L_>()));
    return r;
}

template void launch_fft_rows_fwd<float>(const Plan&, const cpx<float>*, cpx<float>*, hipStream_t, const void*);
template void launch_fft_rows_fwd<double>(const Plan&, const cpx<double>*, cpx<double>*, hipStream_t, const void*);
template int launch_fft_rows_init<float>(const Plan&, const cpx<float>*, const cpx<float>*, const cpx<float>*,
                                         const cpx<float>*, cpx<float>*, cpx<float>*, double*, cpx<float>*,
                                         hipStream_t, const void*);
template int launch_fft_rows_init<double>(const Plan&, const cpx<double>*, const cpx<double>*, const cpx<double>*,
                                          const cpx<double>*, cpx<double>*, cpx<double>*, double*, cpx<double>*,
                                          hipStream_t, const void*);
template void launch_fft_cols_fwd<float>(const Plan&, const cpx<float>*, cpx<float>*, hipStream_t);
template void launch_fft_cols_fwd<double>(const Plan&, const cpx<double>*, cpx<double>*, hipStream_t);
template void launch_fft_cols_adj<float>(const Plan&, const cpx<float>*, cpx<float>*, hipStream_t);
template void launch_fft_cols_adj<double>(const Plan&, const cpx<double>*, cpx<double>*, hipStream_t);
template int launch_fft_rows_xr<float>(const Plan&, cpx<float>*, cpx<float>*, cpx<float>*, const cpx<float>*,
                                       const double*, int, const double*, const double*, const double*, int, double*,
                                       cpx<float>*, hipStream_t, const void*);
template int launch_fft_rows_xr<double>(const Plan&, cpx<double>*, cpx<double>*, cpx<double>*, const cpx<double>*,
                                        const double*, int, const double*, const double*, const double*, int, double*,
                                        cpx<double>*, hipStream_t, const void*);
template void launch_fft_rows_adj_cg<float>(const Plan&, const cpx<float>*, cpx<float>*, double, const cpx<float>*,
                                            double, double*, const cpx<float>*, double*, double*, hipStream_t,
                                            const void*);
template void launch_fft_rows_adj_cg<double>(const Plan&, const cpx<double>*, cpx<double>*, double, const cpx<double>*,
                                             double, double*, const cpx<double>*, double*, double*, hipStream_t,
                                             const void*);
template void launch_fft_cols_toep<float>(const Plan&, cpx<float>*, hipStream_t, const cpx<float>*);
template void launch_fft_cols_toep<double>(const Plan&, cpx<double>*, hipStream_t, const cpx<double>*);
template void launch_fft_rows_adj<float>(const Plan&, const cpx<float>*, cpx<float>*, double,
                                         const cpx<float>*, double, double*, hipStream_t, const void*);
template void launch_fft_rows_adj<double>(const Plan&, const cpx<double>*, cpx<double>*, double,
                                          const cpx<double>*, double, double*, hipStream_t, const void*);
template int fft_toep_group<float>(const Plan&);
template int fft_toep_group<double>(const Plan&);
template int fft_rows_adj_blocks<float>(const Plan&);
template int fft_rows_adj_blocks<double>(const Plan&);

}  // namespace purify
