/*
 * purify.h -- C ABI of libpurify.so, the MI355X (gfx950) SDMM radio-interferometric imaging
 * hot path of PURIFY (Carrillo, McEwen & Wiaux, "PURIFY: a new algorithmic framework for
 * next-generation radio-interferometric imaging").
 *
 * Problem (Section 2, eqs. (2)-(3)): recover an n x n image x >= 0 from M visibilities
 * y = Phi x + noise by   minimise ||W Psi^dagger x||_1  subject to  ||y - Phi x||_2 <= eps,
 * solved with SDMM (Section 3, eq. (6), Algorithm 1).
 *
 * Conventions shared by every call
 * --------------------------------
 * - Complex vectors are interleaved (re, im) pairs of the plan's precision: double for
 *   PURIFY_FP64, float for PURIFY_FP32 (layout of std::complex / torch.complex128 /
 *   torch.complex64).  Images are n x n row-major; axis 0 (rows, index j1) pairs with
 *   omega_1, axis 1 with omega_2; pixel coordinate p = j - n/2.
 * - Vectors passed to compute calls are DEVICE pointers owned by the caller.  The library
 *   never allocates device memory: every plan-owned buffer is carved out of the caller's
 *   workspace (the one exception, purify_phi_noalloc's fixed array, is part of the library's
 *   code object).  Host pointers are marked "host".
 * - `stream` is a hipStream_t passed as void* (NULL = the default stream).  Compute calls
 *   enqueue on it and return without synchronising, except purify_plan_create and
 *   purify_sdmm_solve, which return once their work is complete.
 * - Calls return a purify_status and never throw.  On error, purify_last_error() returns a
 *   thread-local message.  Calls on one plan must not overlap (they share the plan's
 *   scratch buffers); different plans are independent.
 */
#ifndef PURIFY_H
#define PURIFY_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PURIFY_OK = 0,
    PURIFY_E_INVALID = 1,    /* bad argument (sizes, null pointers, non-finite uv, ...) */
    PURIFY_E_WORKSPACE = 2,  /* workspace missing or smaller than purify_plan_workspace_bytes */
    PURIFY_E_DEVICE = 3,     /* a HIP runtime error; see purify_last_error() */
    PURIFY_E_NONFINITE = 4   /* SDMM produced a NaN/Inf objective or residual */
} purify_status;

typedef enum {
    PURIFY_FP64 = 0,  /* all arithmetic in double */
    PURIFY_FP32 = 1   /* operators and prox in float; reductions, norms, CG scalars and the
                         stopping tests in double */
} purify_precision;

/* Dictionary bits: bit 0 = Dirac basis, bit b (1..8) = Daubechies Db-b wavelet basis
 * (Section 2.2: SARA = Dirac + Db1..Db8 = 0x1FF; BPDb8 = 1u << 8; BP = 1u). */
#define PURIFY_DICT_SARA 0x1FFu

typedef struct {
    int32_t n;           /* image side; power of two, 16 <= n <= 4096, divisible by 2^levels */
    int32_t oversample;  /* grid oversampling factor; must be 2 (K = 2n) */
    int32_t J;           /* Kaiser-Bessel taps per axis, 2..16 */
    double beta;         /* Kaiser-Bessel shape; <= 0 selects 2.34 * J */
    int64_t M;           /* number of visibilities, 1 <= M < 2^31 */
    const double* uv;    /* host, M x 2 row-major: (omega_1, omega_2) in radians per pixel.
                            Any finite value; wrapped into [-pi, pi) (exact: the model is
                            2 pi periodic in omega).  Read only during plan creation. */
    uint32_t dict_mask;  /* bases of Psi, see PURIFY_DICT_SARA; nonzero */
    int32_t levels;      /* wavelet levels, 1..8 */
    int32_t precision;   /* purify_precision */
} purify_plan_desc;

typedef struct purify_plan purify_plan;

/* Device workspace a plan needs (bytes), or 0 if the descriptor is invalid.  Host only. */
size_t purify_plan_workspace_bytes(const purify_plan_desc* desc);

/* Dictionary size D = q * n * n for the descriptor (q = number of bases), or 0 if invalid. */
int64_t purify_plan_dict_size(const purify_plan_desc* desc);

/* Build a plan (Section 4 measurement operator, continuous visibilities): wraps and bins
 * the uv points on the host (grid coordinates kappa = omega K / 2 pi in double, split into
 * an integer first tap and a fractional offset), sorts them by grid tile, computes the
 * deapodisation, FFT twiddles, Kaiser-Bessel per-tap polynomials and Daubechies filters, and uploads
 * them into `workspace` (device, >= purify_plan_workspace_bytes(desc) bytes, 256-byte
 * aligned, owned by the caller and kept alive until purify_plan_destroy).  Synchronous on
 * `stream`.  *out receives a host handle. */
purify_status purify_plan_create(const purify_plan_desc* desc, void* workspace, size_t bytes,
                                 void* stream, purify_plan** out);

/* Release the host handle.  The workspace stays owned by the caller. */
void purify_plan_destroy(purify_plan* plan);

/* y = Phi x = G F Z S x (Section 4; Phi of eq. (2)).  x: device, N = n*n complex.
 * y: device, M complex in the caller's uv order. */
purify_status purify_phi(const purify_plan* plan, const void* x, void* y, void* stream);

/* y = Phi x as purify_phi, for callers that cannot allocate device memory or touch the plan's
 * workspace (code under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): the row-transformed image and the oversampled grid live in a fixed 48 MiB array
 * of library device memory, one per device, held until the process ends, instead of the
 * plan's workspace.  The call allocates nothing and calls no allocating routine; the array's
 * device address is looked up once per device (the first call with that device current).
 * Same kernels and same result as purify_phi.  n x K + K x K complex values must fit in the
 * array (n <= 1024 in FP32, n <= 512 in FP64); larger plans get PURIFY_E_INVALID.  Every call
 * on a device shares its array: calls that overlap on one device (other streams, other host
 * threads) race and must be serialised by the caller. */
purify_status purify_phi_noalloc(const purify_plan* plan, const void* x, void* y, void* stream);

/* x = Phi^dagger y = S Z^T F^dagger G^T y (the exact adjoint of purify_phi). */
purify_status purify_phi_adj(const purify_plan* plan, const void* y, void* x, void* stream);

/* x = Psi alpha = (1/sqrt q) sum_b W_b^T alpha_b (Section 2.2).  alpha: device, D complex
 * laid out as q blocks of n x n in dictionary order [Dirac, Db1, ..., Db8] restricted to
 * dict_mask, each wavelet block in Mallat layout. */
purify_status purify_psi(const purify_plan* plan, const void* alpha, void* x, void* stream);

/* alpha = Psi^dagger x = (1/sqrt q) [x; W_1 x; ...] (Section 2.2), layout as purify_psi. */
purify_status purify_psi_adj(const purify_plan* plan, const void* x, void* alpha, void* stream);

/* purify_sdmm_params.flags: enqueue every kernel eagerly instead of replaying one captured
 * HIP graph per SDMM iteration (same kernels, same results; for debugging and tests). */
#define PURIFY_SDMM_NO_GRAPH 1
/* purify_sdmm_params.flags: x_out holds the starting point x_hat(0) on entry (Algorithm 1,
 * step 1 with a given x_hat(0): z_i = 0, x_i = L_i^dagger L_i x_hat(0)); without it
 * x_hat(0) = 0.  x_out then receives the result as usual. */
#define PURIFY_SDMM_WARM_START 2
/* purify_sdmm_params.flags: the global update's conjugate gradient applies the stored
 * (Toeplitz) form of Phi^dagger Phi instead of Phi and Phi^dagger (Section 3 suggests
 * precomputing that composite operator; see purify_phi_normal).  It differs from the
 * NUFFT's Phi^dagger Phi by the NUFFT's own error; nu, the proximity steps and the
 * data-fidelity branch still apply Phi and Phi^dagger. */
#define PURIFY_SDMM_TOEPLITZ 4
/* purify_sdmm_params.flags: the prior is the total variation of the image (the TV problem of
 * Section 5: minimise sum_ij w_ij |(grad x)_ij| subject to the data constraint(s) and x >= 0)
 * instead of ||W Psi^dagger x||_1.  f1 = TV with L1 = I, so the global update is unchanged;
 * its proximity operator runs tv_iter steps of Chambolle's dual projection algorithm (step
 * 1/8, from a zero dual field; forward differences, zero on the last row and column).
 * weights, if given, are N per-pixel doubles; the default gamma is
 * 1e-3 max_ij |(grad Phi~^dagger y~)_ij|; the objective is TV_w(x_hat). */
#define PURIFY_SDMM_TV 8

typedef struct {
    double epsilon;       /* l2 bound of eq. (2) on ||y - Phi x||, unnormalised units */
    double gamma;         /* SDMM step gamma (Algorithm 1); <= 0: 1e-3 max|Psi^dag Phi~^dag y~| */
    double nu;            /* ||Phi||_2 used to normalise Phi; <= 0: power iteration */
    double xi;            /* halting: relative objective variation bound (Section 3) */
    double slack;         /* halting: accept ||y~ - Phi~ x|| <= eps~ (1 + slack) */
    int32_t max_iter;     /* T_max (Algorithm 1), >= 1 */
    int32_t cg_iter;      /* conjugate-gradient steps per global update, >= 1 */
    int32_t check_every;  /* halting test period in iterations (>= 1) when halting != 0 */
    int32_t halting;      /* 0: run exactly max_iter iterations; 1: Section 3 stopping rule */
    int32_t nu_iter;      /* power-iteration count when nu <= 0 (e.g. 100) */
    int32_t flags;        /* PURIFY_SDMM_* bits; 0 = defaults */
    const double* weights; /* device, D doubles (diagonal W of eq. (3)), or NULL for W = I;
                              N doubles (per-pixel TV weights) with PURIFY_SDMM_TV */
    double* history;      /* host, 2 * max_iter doubles or NULL: per iteration the objective
                             ||W Psi^dag x_hat||_1 and the residual ||y~ - Phi~ x_hat|| */
    int32_t nblocks;      /* R: 0 or 1 = one data constraint with `epsilon`; 2..1024 = the data
                             split into R blocks (eqs. (4)-(5)), one l2 constraint each, S = R + 2
                             functions; `epsilon` is then unused */
    const int64_t* block_offsets;  /* host, R + 1 (R >= 2): block i holds the visibilities
                             [off[i], off[i+1]) of the caller's uv order; off[0] = 0, off[R] = M,
                             strictly increasing */
    const double* block_eps;       /* host, R (R >= 2): eps_i >= 0, unnormalised */
    int32_t tv_iter;      /* PURIFY_SDMM_TV: dual projection steps per proximity operator, >= 1 */
} purify_sdmm_params;

typedef struct {
    int32_t iterations;   /* iterations run */
    int32_t converged;    /* 1 if the stopping rule fired */
    double objective;     /* last ||W Psi^dagger x_hat||_1 */
    double residual;      /* last ||y - Phi x_hat||_2 in unnormalised units */
    double nu;            /* operator norm used */
    double gamma;         /* gamma used */
} purify_sdmm_info;

/* SDMM (Algorithm 1) for eq. (3) with R = 1: f1 = ||W .||_1 on Psi^dagger x, f2 = positive
 * orthant, f3 = l2 ball of radius epsilon about y on Phi x (with nblocks = R >= 2: f_{i+2} =
 * l2 ball of radius eps_i about y_i on Phi_i x, projected block by block; the halting rule
 * then asks every block's residual to be within eps_i (1 + slack)).  The global update solves
 * (Phi~^dagger Phi~ + 2 I) x = sum_i x_i by cg_iter warm-started conjugate-gradient steps
 * (Section 3), with Phi~ = Phi / nu.  y: device, M complex in uv order.  x_out: device, N
 * complex; receives x_hat (the image is its real part).  Uses the plan's solver state, so
 * one solve per plan at a time.  Internally the solve runs on two library-created streams
 * ordered after `stream`'s prior work (branch i = 1 of Algorithm 1 overlaps branches 2-3),
 * replaying one captured HIP graph per iteration.  Returns after the last iteration
 * (synchronous). */
purify_status purify_sdmm_solve(purify_plan* plan, const void* y, const purify_sdmm_params* params,
                                void* x_out, purify_sdmm_info* info, void* stream);

/* purify_phi_normal modes. */
#define PURIFY_NORMAL_TOEPLITZ 1

/* out = Phi^dagger Phi x (x, out: device, N complex; both n x n).  mode 0: through the
 * NUFFT, exactly the operator of the CG update (the interpolation and gridding of G^T G fused
 * in one launch; on FP32 grids of 2048 x 2048 and more, G then G^T as two launches).  mode PURIFY_NORMAL_TOEPLITZ: the stored form
 * T = Z^T F^dagger diag(c_hat) F Z, a convolution with the point-spread function
 * h(d) = sum_m exp(i omega_m . d) on the 2n x 2n circulant embedding, with c_hat the real
 * part of its spectrum / K^2 (so T is Hermitian).  h comes from the plan's Phi^dagger applied
 * to modulated unit visibilities (four n x n quadrants of d), so T matches the NUDFT normal
 * operator to the NUFFT's accuracy.  c_hat is computed on the first call that needs it
 * (that call is synchronous) and kept in the plan workspace; later calls only enqueue. */
purify_status purify_phi_normal(purify_plan* plan, const void* x, void* out, int32_t mode, void* stream);

/* Reweighted l1 (SARA, Section 2.2): a sequence of weighted-l1 problems, each weight roughly
 * the inverse magnitude of the previous solution's coefficient.  Solve 0 uses params->weights
 * (NULL: W = I); solve k >= 1 uses w_j = delta_k / (delta_k + |(Psi^dagger x(k-1))_j|), is warm
 * started from x(k-1) (PURIFY_SDMM_WARM_START) and reuses solve 0's nu and gamma.
 * delta_1 = max(delta0, delta_min), delta0 <= 0 meaning the standard deviation of the
 * coefficients Psi^dagger x(0); delta_{k+1} = max(decay delta_k, delta_min), delta_min < 0
 * meaning sigma / nu with sigma = epsilon / sqrt(M + 2 sqrt(M)) (the noise level of the
 * chi-square bound epsilon; with visibility blocks, the largest eps_i / sqrt(M_i + 2 sqrt(M_i))).  The loop ends after solve k when
 * ||x(k) - x(k-1)|| / ||x(k-1)|| < rel_var, or after `reweights` weighted solves. */
typedef struct {
    double delta0;      /* <= 0: standard deviation of Psi^dagger x(0) */
    double decay;       /* 0 < decay <= 1 */
    double delta_min;   /* floor on delta; < 0: sigma / nu as above */
    double rel_var;     /* relative-variation stopping bound, >= 0 (0: run every reweight) */
    int32_t reweights;  /* weighted solves after solve 0, >= 0 */
} purify_reweight_params;

typedef struct {
    int32_t solves;            /* SDMM solves run, solve 0 included */
    int32_t total_iterations;  /* SDMM iterations over all solves */
    double delta;              /* delta of the last weighted solve (0 if none ran) */
    double rel_var;            /* relative variation after the last weighted solve (-1 if none) */
} purify_reweight_info;

/* Reweighted SDMM.  y: device, M complex in uv order.  params: as for purify_sdmm_solve
 * (flags apply to every solve; PURIFY_SDMM_WARM_START also to solve 0; history, if given,
 * keeps the rows of the last solve).  weights: device, D doubles owned by the caller
 * (purify_plan_dict_size), overwritten with each solve's weights (may be params->weights);
 * may be NULL when rw->reweights = 0.  x_io: device, N complex; x(0) on entry when
 * PURIFY_SDMM_WARM_START is set; receives the last solution.  info: the last solve's.
 * With PURIFY_SDMM_TV (reweighted TV) the coefficients are the gradient magnitudes
 * |(grad x)_ij| and weights holds N doubles.
 * Synchronous, one call per plan at a time. */
purify_status purify_sdmm_reweighted(purify_plan* plan, const void* y, const purify_sdmm_params* params,
                                     const purify_reweight_params* rw, double* weights, void* x_io,
                                     purify_sdmm_info* info, purify_reweight_info* rw_info, void* stream);

/* Kernel stages that purify_time_stage can time (one launch = one application). */
typedef enum {
    PURIFY_STAGE_FFT_ROWS = 0,     /* S Z + row transforms of Phi            (n x n -> K x n) */
    PURIFY_STAGE_FFT_COLS = 1,     /* column transforms of Phi               (K x n -> K x K) */
    PURIFY_STAGE_DEGRID = 2,       /* G: Kaiser-Bessel interpolation          (K x K -> M)     */
    PURIFY_STAGE_GRID = 3,         /* G^T: tiled gridding                     (M -> K x K)     */
    PURIFY_STAGE_IFFT_COLS = 4,    /* column transforms of Phi^dagger         (K x K -> K x n) */
    PURIFY_STAGE_IFFT_ROWS = 5,    /* row transforms + Z^T S of Phi^dagger    (K x n -> n x n) */
    PURIFY_STAGE_PHI = 6,          /* whole Phi                                                */
    PURIFY_STAGE_PHI_ADJ = 7,      /* whole Phi^dagger                                         */
    PURIFY_STAGE_PSI_ADJ = 8,      /* whole Psi^dagger                                         */
    PURIFY_STAGE_PSI = 9,          /* whole Psi                                                */
    PURIFY_STAGE_GTG = 10,         /* G^T G in one launch (interpolate + grid), as in the
                                      normal operator Phi^dagger Phi of the CG update  (K x K -> K x K) */
    PURIFY_STAGE_TOEP_COLS = 11,   /* column stage of the stored normal operator (transform,
                                      spectrum, adjoint transform, in place)          (n x K -> n x K) */
    PURIFY_STAGE_TOEP_NORMAL = 12, /* whole stored normal operator T x                (n x n -> n x n) */
    PURIFY_STAGE_TV_STEP = 13      /* one launch of the TV prox's dual projection: four steps
                                      (reads the dual fields and an image, writes the dual
                                      fields)                                         (n x n -> n x n) */
} purify_stage;

/* Time `reps` back-to-back launches of one stage on the plan's internal buffers (their
 * contents are whatever the last call left; inputs are not validated) with HIP events
 * recorded on `stream`; *ms_per_launch receives the average.  Synchronous. */
purify_status purify_time_stage(purify_plan* plan, int32_t stage, int32_t reps, void* stream,
                                double* ms_per_launch);

/* ---------------------------------------------------------------------------------------
 * Serving form: a persistent request loop that runs the SDMM solves of independent imaging
 * requests (any size and visibility count the plan accepts) concurrently on the current
 * device.  The caller owns one device arena (the HBM budget); each admitted request gets a
 * block of it (plan workspace + visibilities + image, purify_plan_workspace_bytes + M + N
 * complex, 256-byte aligned) until its result is on the host.  Up to max_active requests
 * run at once, each on its own stream with its own graph-replayed iteration, so their
 * kernels overlap on the device; waiting requests are admitted as slots and arena memory
 * free up (oldest first; a later request that fits may overtake a waiting one at most
 * 2 * max_active times).  A served result is identical to purify_sdmm_solve of the same
 * request on its own.  Calls are thread-safe.
 * ------------------------------------------------------------------------------------- */
typedef struct purify_server purify_server;

typedef struct {
    void* arena;          /* device, 256-byte aligned, owned by the caller, kept alive until
                             purify_server_destroy returns */
    size_t arena_bytes;   /* HBM budget: requests whose block exceeds it are rejected */
    int32_t max_active;   /* requests solved at once (worker slots, one stream each), 1..64 */
} purify_server_desc;

/* Start the server's worker slots on the current device. */
purify_status purify_server_create(const purify_server_desc* desc, purify_server** out);

/* Queue one solve.  desc: as for purify_plan_create (desc->uv host, M x 2, copied).  y: host,
 * M complex of desc->precision in uv order (copied).  params: as for purify_sdmm_solve, with
 * history and weights NULL and nblocks <= 1.  *ticket identifies the request.  Returns at once. */
purify_status purify_server_submit(purify_server* server, const purify_plan_desc* desc, const void* y,
                                   const purify_sdmm_params* params, int64_t* ticket);

/* State of a request: 0 waiting, 1 running, 2 done, -1 unknown ticket. */
int32_t purify_server_poll(purify_server* server, int64_t ticket);

/* Block until the request is done, then release it.  x: host, N complex of the request's
 * precision (or NULL); info as for purify_sdmm_solve (or NULL); timings: host, 3 doubles or
 * NULL: milliseconds waiting for admission, running (plan creation, solve, result
 * download), and from submission to the result on the host.  Returns the solve's status.
 * A ticket is collected once: an unknown or already collected ticket, or a second thread
 * waiting on the same ticket, gets PURIFY_E_INVALID. */
purify_status purify_server_wait(purify_server* server, int64_t ticket, void* x, purify_sdmm_info* info,
                                 double* timings);

/* Finish every queued request, stop the workers and free the server (uncollected results
 * are dropped).  The arena may be freed afterwards. */
void purify_server_destroy(purify_server* server);

/* Host-side introspection (no GPU needed). */
/* Daubechies Db-b lowpass filter the library uses (extremal phase, sum h = sqrt 2), computed
 * by its own spectral factorisation.  Writes min(2b, cap) doubles to h (host); returns 2b,
 * or -1 if b is not in 1..8. */
int32_t purify_daubechies_filter(int32_t b, double* h, int32_t cap);
/* Kaiser-Bessel kernel psi(t) (I0(beta sqrt(1-(2t/J)^2)) / I0(beta), 0 outside |t| <= J/2)
 * as evaluated by the kernels' series, in double, for `count` host values t -> out. */
int32_t purify_kb_kernel(int32_t J, double beta, int32_t count, const double* t, double* out);
/* Deapodisation factors s_j = 1 / psi_hat((j - n/2)/K), j < n (host, n doubles). */
int32_t purify_deapodisation(int32_t n, int32_t K, int32_t J, double beta, double* out);

const char* purify_status_string(purify_status status);
const char* purify_last_error(void);
/* Library version string. */
const char* purify_version(void);

#ifdef __cplusplus
}
#endif

#endif /* PURIFY_H */
