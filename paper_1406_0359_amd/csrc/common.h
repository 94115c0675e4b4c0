// Internal declarations shared by the host runtime and the HIP kernels of libpurify.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>

#include "../../include/purify.h"

namespace purify {

struct SolverStreams;   // solver_rt.h

// ---------------------------------------------------------------------------------------
// Complex numbers: interleaved (re, im), 8- or 16-byte aligned so loads are single vector
// instructions.
template <typename T>
struct alignas(2 * sizeof(T)) cpx {
    T x, y;
};

template <typename T> __host__ __device__ __forceinline__ cpx<T> mk(T a, T b) { return {a, b}; }
template <typename T> __host__ __device__ __forceinline__ cpx<T> operator+(cpx<T> a, cpx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T> __host__ __device__ __forceinline__ cpx<T> operator-(cpx<T> a, cpx<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T> __host__ __device__ __forceinline__ cpx<T> operator*(cpx<T> a, cpx<T> b) {
    return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename T> __host__ __device__ __forceinline__ cpx<T> operator*(T s, cpx<T> a) { return {s * a.x, s * a.y}; }
template <typename T> __host__ __device__ __forceinline__ cpx<T> conjg(cpx<T> a) { return {a.x, -a.y}; }
// a * conj(b)
template <typename T> __host__ __device__ __forceinline__ cpx<T> mulc(cpx<T> a, cpx<T> b) {
    return {a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y};
}
// multiply by i and by -i
template <typename T> __host__ __device__ __forceinline__ cpx<T> mul_i(cpx<T> a) { return {-a.y, a.x}; }
template <typename T> __host__ __device__ __forceinline__ cpx<T> mul_mi(cpx<T> a) { return {a.y, -a.x}; }

// ---------------------------------------------------------------------------------------
// Kaiser-Bessel kernel psi(t) = I0(beta sqrt(1 - (2t/J)^2)) / I0(beta), |t| <= J/2.
// A visibility's J taps per axis sit at t_a = f + (J/2 - 1) - a with f in [0, 1), so tap a
// only ever evaluates psi on one unit interval.  The plan fits, per tap, a polynomial of
// fixed degree in x = f - 1/2 (Chebyshev interpolation in long double, converted to
// monomials), checked against the Bessel series to 1e-14 (FP64) / 1e-8 (FP32) absolute.
// Evaluating all J taps together is J independent Horner chains with uniform coefficients.
template <typename T> struct KBDeg;
template <> struct KBDeg<double> { static constexpr int value = 17; };
template <> struct KBDeg<float> { static constexpr int value = 9; };
constexpr int KB_MAX_J = 16;
constexpr int KB_MAX_COEF = KB_MAX_J * 18;

// w[a] = psi(f + J/2 - 1 - a), a < J;  c: [a][k] coefficients, k = 0..DEG (device memory)
template <typename T, int J>
__device__ __forceinline__ void kb_weights(const T* __restrict__ c, T f, T* w) {
    constexpr int NC = KBDeg<T>::value + 1;
    const T x = f - (T)0.5;
#pragma unroll
    for (int a = 0; a < J; ++a) w[a] = c[a * NC + NC - 1];
#pragma unroll
    for (int k = NC - 2; k >= 0; --k) {
#pragma unroll
        for (int a = 0; a < J; ++a) w[a] = w[a] * x + c[a * NC + k];
    }
}

// Daubechies filter bank for the wavelet passes: up to 8 bases, 16 taps each.
constexpr int MAX_WAV = 8;
constexpr int MAX_TAPS = 16;

// ---------------------------------------------------------------------------------------
// Scalar slots (doubles) of the solver, in device memory.
enum Slot : int {
    SL_RHO = 0, SL_PQ, SL_ALPHA, SL_BETA, SL_RHONEW,
    SL_OBJ, SL_RES2, SL_D2, SL_BALL, SL_LAMBDA, SL_INVLAMBDA, SL_MAXABS, SL_NONFINITE, SL_ITER,
    SL_RW_A, SL_RW_B, SL_RW_C,   // reweighting statistics (sums of the reweighting kernels)
    SL_BLK_RATIO,                // visibility blocks: max_i ||y~_i - Phi~_i x|| / eps~_i
    SL_COUNT = 32
};

constexpr int MAX_PARTIALS = 8192;   // per partial-sum buffer
// Visibility blocks (eqs. (4)-(5)): at most MAX_BLOCKS data blocks; their ball projections
// reduce over chunks of each block's visibilities (at most BLK_CHUNKS chunks of at least 256)
constexpr int MAX_BLOCKS = 1024;
constexpr int BLK_CHUNKS = 4096 + MAX_BLOCKS;
constexpr int GRID_UNIT = 1024;      // smallest gridding work unit (visibility passes)
constexpr int GRID_REC = 16;         // ints per gridding work-unit record
constexpr int NUM_PARTIAL_BUFS = 10;

// ---------------------------------------------------------------------------------------
// Plan: host handle with device pointers into the caller's workspace.
struct Plan {
    // descriptor
    int n = 0, K = 0, J = 0, levels = 0, precision = 0;
    int64_t M = 0;
    double beta = 0;
    uint32_t dict_mask = 0;
    int q = 0;                 // number of bases
    bool has_dirac = false;
    int nwav = 0;              // wavelet bases
    int wav_N[MAX_WAV] = {};   // Daubechies order of each wavelet basis (dictionary order)
    int wav_block[MAX_WAV] = {};  // alpha block index of each wavelet basis
    int TT = 32, nT = 0;       // gridding tile side and tiles per axis
    int grid_threads = 256;    // gridding workgroup size (256 or 1024)
    int max_tile_load = 0;     // most visibilities one gridding workgroup handles
    int64_t D = 0, N = 0;
    size_t elem = 0;           // bytes per complex element
    double kb_i0beta = 0;      // I0(beta)
    double kb_fit_err = 0;     // max |polynomial - psi| found when the plan was built
    double filt[MAX_WAV][MAX_TAPS] = {};

    // device buffers (carved from the workspace)
    char* ws = nullptr;
    size_t ws_bytes = 0;
    int32_t* base = nullptr;     // M: packed first taps (k0_1 | k0_2 << 16), sorted order
    void* frac = nullptr;        // 2M reals: fractional offsets, sorted order
    int32_t* perm = nullptr;     // M: sorted position -> caller index
    int32_t* tileoff = nullptr;  // 4 nT^2 + 1 class offsets
    int32_t* tilecover = nullptr;  // nT^2: max number of visibilities covering one cell of the tile
    int32_t* gwork = nullptr;    // gridding work-unit records, GRID_REC ints each
    int nwork = 0;
    bool strip_xcd = false;      // work unit w handles a tile of strip t2 with t2 % 8 == w % 8
    int32_t* dchunk = nullptr;   // degridding: {first visibility, count} per workgroup (strip order)
    int ndchunk = 0, dchunk_cap = 0;   // 0 workgroups listed: plain 256-visibility blocks
    bool degrid_tiles = false;   // G by tiles with an LDS window of the grid (else per visibility)
    int TD = 32, nTD = 0;        // degridding tile side (TT or 2 TT) and tiles per axis
    int32_t* dwork = nullptr;    // TD > TT: degridding records {tile, -, -, -, s0, e0, s1, e1, ...}
    int ndwork = 0, dwork_cap = 0;
    int dunit = 0;               // visibilities per degridding record before a tile is split
    int grid_unit = 0;           // visibility passes per gridding work unit before a split
    int32_t* gmerge = nullptr;   // split tiles {tile, parts, first partial slot}
    int nmerge = 0, gmerge_cap = 0;
    void* gscratch = nullptr;    // split tiles: one integer partial tile per part
    int32_t* gexp = nullptr;     // split tiles: scale exponent of each partial tile
    int gslots = 0;
    void* deap = nullptr;        // n reals
    void* tw = nullptr;          // n complex: exp(-2 pi i t / n)
    void* tw2 = nullptr;         // n complex: exp(-pi i t / n)
    void* filters = nullptr;     // MAX_WAV * 2 * MAX_TAPS reals (h then g)
    void* kbpoly = nullptr;      // J * (KBDeg + 1) reals: per-tap polynomial coefficients
    void* wtab = nullptr;        // FP64 plans: M x 2J tap weights (sorted order), else null
    void* grid = nullptr;        // K x K complex, row-major G[k1][k2]
    void* grid2 = nullptr;       // K x K complex: G^T G output of the normal operator
    void* tmp = nullptr;         // n x K complex, layout [j1][k2]
    void* unit = nullptr;        // n reals, all 1 (row passes without S)
    void* chat = nullptr;        // K x K reals: spectrum of the stored normal operator, / K^2
    bool chat_ready = false;     // chat computed (on the first call that needs it)
    double* part = nullptr;      // NUM_PARTIAL_BUFS * MAX_PARTIALS
    double* sc = nullptr;        // SL_COUNT scalars
    double* hist = nullptr;      // 2 * hist_cap doubles
    int hist_cap = 0;
    // solver state
    void *xh = nullptr, *x1 = nullptr, *x2 = nullptr, *x3 = nullptr;
    void *r = nullptr, *p = nullptr, *qv = nullptr;
    void *z2 = nullptr, *ytil = nullptr, *z3 = nullptr, *v3 = nullptr;
    void *z1 = nullptr, *v1 = nullptr;
    void *wt = nullptr;          // wavelet temp: nwav * N complex
    void *ws2 = nullptr;         // wavelet LL temp: nwav * N/4 complex (x2 ping-pong)
    void *vis = nullptr;         // M complex scratch (visibility-space temp)
    void *tvp = nullptr;         // TV prior: two dual fields (p1, p2) of N complex, ping-pong
    // visibility blocks of the current solve (R > 1)
    int32_t* bid = nullptr;      // M: block of each sorted visibility
    int32_t* bperm = nullptr;    // M: sorted positions grouped by block (ascending within a block)
    int32_t* bchunk = nullptr;   // BLK_CHUNKS x {first, end} ranges of bperm, block by block
    int32_t* bchunk_off = nullptr;  // MAX_BLOCKS + 1: first chunk of each block
    double* beps = nullptr;      // MAX_BLOCKS: eps_i / nu
    double* bscale = nullptr;    // MAX_BLOCKS: ball scale of each block (this iteration)
    // streams and events the solver runs on (the plan's own, or a server slot's)
    SolverStreams* ss = nullptr;
};

// ---------------------------------------------------------------------------------------
// Kernel launchers (defined in the .hip files, instantiated for float and double).
// deap: per-pixel factors of S (n reals of the plan's type); null = the plan's
// deapodisation, the plan's `unit` table = no S (the stored normal operator)
template <typename T> void launch_fft_rows_fwd(const Plan& P, const cpx<T>* x, cpx<T>* tmp, hipStream_t s,
                                               const void* deap = nullptr);
template <typename T> void launch_fft_cols_fwd(const Plan& P, const cpx<T>* tmp, cpx<T>* grid, hipStream_t s);
template <typename T> void launch_fft_cols_adj(const Plan& P, const cpx<T>* grid, cpx<T>* tmp, hipStream_t s);
// first CG step's row pass with the CG set-up folded in: r = p = x1 + x2 + x3 - q0 (q0 may be
// null), partial ||r||^2 per workgroup into rho_part (count returned), row transform of p
// into tmp
template <typename T> int launch_fft_rows_init(const Plan& P, const cpx<T>* x1, const cpx<T>* x2,
                                               const cpx<T>* x3, const cpx<T>* q0, cpx<T>* r, cpx<T>* p,
                                               double* rho_part, cpx<T>* tmp, hipStream_t s,
                                               const void* deap = nullptr);
// CG step from the second on (exact or stored operator): row pass with alpha = rho / <p, q>,
// x += alpha p, r -= alpha q, beta = (rho - 2 alpha <r, q> + alpha^2 ||q||^2) / rho,
// p = r + beta p (partial sums of rho, <p, q>, <r, q>, ||q||^2 given; the last three dot_count
// of them), partial ||r||^2 per row block (returns their count), row transform of p into tmp
template <typename T> int launch_fft_rows_xr(const Plan& P, cpx<T>* x, cpx<T>* r, cpx<T>* p, const cpx<T>* q,
                                             const double* rho_part, int rho_count, const double* pq_part,
                                             const double* rq_part, const double* qq_part, int dot_count,
                                             double* rho_new_part, cpx<T>* tmp, hipStream_t s,
                                             const void* deap = nullptr);
// adjoint row pass of a CG step: q = c1 (S Z^T F^dag rows)(tmp) + c2 p, partials <p, q>, <r, q>
// and ||q||^2 per row block
template <typename T> void launch_fft_rows_adj_cg(const Plan& P, const cpx<T>* tmp, cpx<T>* q, double c1,
                                                  const cpx<T>* p, double c2, double* pq_part, const cpx<T>* r,
                                                  double* rq_part, double* qq_part, hipStream_t s,
                                                  const void* deap = nullptr);
// column stage of the stored normal operator: forward transform, times chat, adjoint, into tmp
// (input `in`, default tmp itself)
template <typename T> void launch_fft_cols_toep(const Plan& P, cpx<T>* tmp, hipStream_t s, const cpx<T>* in = nullptr);
// x = c1 * (S Z^T F^dag rows)(tmp) + c2 * v   (v may be null); optional partial Re<v, x>
template <typename T> void launch_fft_rows_adj(const Plan& P, const cpx<T>* tmp, cpx<T>* x, double c1,
                                               const cpx<T>* v, double c2, double* dot_part,
                                               hipStream_t s, const void* deap = nullptr);
template <typename T> int fft_rows_adj_blocks(const Plan& P);
// width W of the column groups by which the stored operator's spectrum is laid out
// (element (k1, k2) at ((k2 / W) K + k1) W + k2 mod W; W = K is the row-major grid)
template <typename T> int fft_toep_group(const Plan& P);

// G: y[perm ? perm[m] : m] = scale * sum psi psi grid
template <typename T> void launch_degrid(const Plan& P, const cpx<T>* grid, cpx<T>* y, const int32_t* perm,
                                         double scale, hipStream_t s);
// G^T: grid = sum psi psi y[perm ? perm[m] : m]
template <typename T> void launch_grid(const Plan& P, const cpx<T>* y, const int32_t* perm, cpx<T>* grid,
                                       hipStream_t s);
// gout = G^T G gin (visibility values interpolated from gin and gridded in one launch)
template <typename T> void launch_gtg(const Plan& P, const cpx<T>* gin, cpx<T>* gout, hipStream_t s);

// The CG's last update folded into the analysis: with XhatArgs, Psi^dag is taken of
// x + alpha p, alpha = rho / <p, q> from the partial sums (the value the CG update kernel
// derives from them), and `first_done` (if given) is recorded after the finest level, the
// only one that reads x and p.  Only plans for which psi_adj_takes_xhat holds accept it.
template <typename T>
struct XhatArgs {
    const cpx<T>* p = nullptr;
    const double* rho_part = nullptr;
    int rho_count = 0;
    const double* pq_part = nullptr;
    int pq_count = 0;
};
bool psi_adj_takes_xhat(const Plan& P);
template <typename T> void launch_psi_adj(const Plan& P, const cpx<T>* x, cpx<T>* alpha, hipStream_t s,
                                          const XhatArgs<T>* xa = nullptr, hipEvent_t first_done = nullptr);
template <typename T> void launch_psi(const Plan& P, const cpx<T>* alpha, cpx<T>* x, hipStream_t s);

// Vector kernels (vector.hip)
template <typename T> void launch_fill(cpx<T>* v, cpx<T> val, int64_t n, hipStream_t s);
// partial sums of |v|^2 (into part), grid-stride; returns number of partials
template <typename T> int launch_norm2_part(const cpx<T>* v, int64_t n, double* part, hipStream_t s);
template <typename T> int launch_maxabs_part(const cpx<T>* v, int64_t n, double* part, hipStream_t s);
// finalize: sum (or max) partials into slot, then apply op
enum FinalOp : int {
    FIN_STORE = 0,        // sc[slot] = sum
    FIN_CG_ALPHA = 1,     // sc[PQ] = sum; sc[ALPHA] = rho == 0 ? 0 : rho / pq
    FIN_CG_BETA = 2,      // rn = sum; sc[BETA] = rho == 0 ? 0 : rn / rho; sc[RHO] = rn
    FIN_LAMBDA = 3,       // sc[LAMBDA] = sqrt(sum); sc[INVLAMBDA] = 1/that (0 if 0)
    FIN_MAX = 4,          // sc[slot] = max
    FIN_BALL = 5,         // sc[D2] = sum; sc[BALL] = min(1, eps / sqrt(sum)) (1 if 0)
    FIN_HIST_OBJ = 6,     // sc[OBJ] = sum; hist[2*it] = sum, it = sc[ITER] mod hist_index
    FIN_HIST_RES = 7,     // sc[RES2] = sum; hist[2*it+1] = sqrt(sum)
    FIN_HIST_OBJ_END = 8  // as FIN_HIST_OBJ, then sc[ITER] += 1 (the end of an SDMM iteration)
};
// For FIN_HIST_*, hist_index is the history capacity and the row is sc[SL_ITER] mod it.
void launch_finalize(const double* part, int count, double* sc, int slot, int op, double arg,
                     double* hist, int hist_index, hipStream_t s);

// the CG's last update x += alpha p, alpha = rho / <p, q> summed from partials in the kernel
template <typename T> void launch_cg_x(cpx<T>* x, const cpx<T>* p, const double* rho_part, int rho_count,
                                       const double* pq_part, int pq_count, int64_t n, hipStream_t s);
// p = r + (rho_new / rho) p, both from partials
// power-iteration normalisation v = w / ||w|| (||w||^2 from partials), sc[LAMBDA] = ||w||
template <typename T> void launch_power_normalise(cpx<T>* v, const cpx<T>* w, const double* part,
                                                  int count, double* sc, int64_t n, hipStream_t s);
template <typename T> int launch_prox_l1(cpx<T>* v1, cpx<T>* z1, const double* w, double gamma,
                                         int64_t n, double* part, hipStream_t s);
template <typename T> void launch_prox_pos(const cpx<T>* xh, cpx<T>* z2, cpx<T>* x2, int64_t n,
                                           hipStream_t s);
template <typename T> int launch_ball_part(const cpx<T>* v3, const cpx<T>* z3, const cpx<T>* yt,
                                           int64_t n, double* part_d, double* part_res,
                                           hipStream_t s);
template <typename T> void launch_prox_ball(cpx<T>* v3, cpx<T>* z3, const cpx<T>* yt, const double* part_d,
                                            const double* part_res, int count, double eps, double* sc,
                                            double* hist, int hist_cap, int64_t n, bool diff, hipStream_t s);
template <typename T> void launch_permute_scale(const cpx<T>* y_user, const int32_t* perm, double scale,
                                                cpx<T>* y_sorted, int64_t n, hipStream_t s);
template <typename T> void launch_scale_by_slot(cpx<T>* dst, const cpx<T>* src, const double* sc,
                                                int slot, int64_t n, hipStream_t s);
// Stored normal operator: v_m = exp(i omega_m . s) (sorted order); zero row / column 0 of an
// n x n image; chat (+)= Re(exp(-2 pi i k . s / K) H) / K^2 for s = (sig1, sig2) n / 2
template <typename T> void launch_modulate(const Plan& P, int s1, int s2, cpx<T>* v, hipStream_t s);
template <typename T> void launch_zero_edge(cpx<T>* x, int n, bool row, bool col, hipStream_t s);
template <typename T> void launch_chat_accum(const Plan& P, const cpx<T>* H, int sig1, int sig2, bool first,
                                             hipStream_t s);
// Visibility blocks: chunk partials of ||v3 + z3 - y~||^2 and ||y~ - v3||^2 over bperm ranges;
// per-block finalize (scale, residual, max ratio, history); elementwise projection by block
template <typename T> void launch_ball_part_blk(const cpx<T>* v3, const cpx<T>* z3, const cpx<T>* yt,
                                                const int32_t* bperm, const int32_t* chunks, int nchunks,
                                                double* part_d, double* part_res, hipStream_t s);
void launch_ball_fin_blk(const double* part_d, const double* part_res, const int32_t* chunk_off,
                         const double* eps, int R, double* scale, double* sc, double* hist, int hist_cap,
                         hipStream_t s);
template <typename T> void launch_prox_ball_blk(cpx<T>* v3, cpx<T>* z3, const cpx<T>* yt, const int32_t* bid,
                                                const double* scale, int64_t n, bool diff, hipStream_t s);
// a -= b
template <typename T> void launch_sub(cpx<T>* a, const cpx<T>* b, int64_t n, hipStream_t s);
// TV prior, branch i = 1: u = x_hat + z1 (into u), `iters` dual projection steps, then
// r1 = u - gamma div p, z1 = u - r1, x1 = r1 - z1, objective partials TV_w(x_hat) (count in *nparts)
template <typename T> void launch_tv_prox(const Plan& P, const cpx<T>* xh, cpx<T>* z1, cpx<T>* x1, cpx<T>* u,
                                          const double* w, double gamma, int iters, double* part, int* nparts,
                                          hipStream_t s);
// launch k of the dual projection (four steps; k = 0 starts from p = 0) on the plan's
// ping-pong dual fields
template <typename T> void launch_tv_step(const Plan& P, const cpx<T>* u, int k, const double* w, double gamma,
                                          hipStream_t s);
// |grad v| (into out's real parts, if out) and partial maxima (if part_max); returns the count
template <typename T> int launch_grad_mag(const Plan& P, const cpx<T>* v, cpx<T>* out, double* part_max,
                                          hipStream_t s);
// Reweighting (SARA): partials of sum Re v and sum Im v
template <typename T> int launch_sum_part(const cpx<T>* v, int64_t n, double* part_re, double* part_im,
                                          hipStream_t s);
// partials of sum |v_j - mean|^2, mean = (sc[slot_re] + i sc[slot_im]) / n
template <typename T> int launch_dev2_part(const cpx<T>* v, int64_t n, const double* sc, int slot_re,
                                           int slot_im, double* part, hipStream_t s);
// w_j = delta / (delta + |a_j|) (1 where that denominator is 0)
template <typename T> void launch_reweight(const cpx<T>* a, int64_t n, double delta, double* w, hipStream_t s);
// partials of ||a - b||^2 and ||b||^2
template <typename T> int launch_diff2_part(const cpx<T>* a, const cpx<T>* b, int64_t n, double* part_d,
                                            double* part_b, hipStream_t s);

// error helper
void set_error(const std::string& msg);

// Host-side plan construction (plan.cpp)
struct DescCheck {
    bool ok = false;
    std::string why;
};
DescCheck check_desc(const purify_plan_desc* d);
size_t layout(Plan& P, const purify_plan_desc* d, char* ws);
purify_status build_plan(Plan& P, const purify_plan_desc* d, hipStream_t s);
long double kb_i0(long double x);
// per-tap polynomial coefficients (J x (deg+1), row a = tap), returns max abs fit error
double kb_fit(int J, double beta, int deg, long double* coef);
double kb_eval_fit(const long double* coef, int J, int deg, double t);
double kb_hat(double nu, int J, double beta, long double i0b);
int daubechies(int N, double* h_out);

}  // namespace purify

#define PURIFY_HIP(expr)                                                                   \
    do {                                                                                   \
        hipError_t _e = (expr);                                                            \
        if (_e != hipSuccess) {                                                            \
            ::purify::set_error(std::string(#expr) + ": " + hipGetErrorString(_e));        \
            return PURIFY_E_DEVICE;                                                        \
        }                                                                                  \
    } while (0)

#include "solver_rt.h"

// The plan struct handle type of the C ABI.  `own` holds the plan's solver streams, created
// on its first solve unless P.ss points elsewhere (a server slot's).
struct purify_plan {
    purify::Plan P;
    purify::SolverStreams own;
};
