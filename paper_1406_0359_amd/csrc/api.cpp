// C ABI of libpurify (declared in include/purify.h) and the SDMM driver (Algorithm 1).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "common.h"

namespace purify {

namespace {
thread_local std::string g_last_error;

template <typename T>
struct Ops {
    const Plan& P;
    hipStream_t s;
    using C = cpx<T>;

    // y = scale * G F Z S x ; y in user order when perm is given, else in sorted order
    void phi(const C* x, C* y, double scale, const int32_t* perm) const {
        launch_fft_rows_fwd<T>(P, x, (C*)P.tmp, s);
        phi_tail(y, scale, perm);
    }
    void phi_tail(C* y, double scale, const int32_t* perm) const {
        launch_fft_cols_fwd<T>(P, (const C*)P.tmp, (C*)P.grid, s);
        launch_degrid<T>(P, (const C*)P.grid, y, perm, scale, s);
    }
    // x = c1 * S Z^T F^dag G^T y + c2 * v  (partial Re<v, x> into dot when given)
    void phi_adj(const C* y, const int32_t* perm, C* x, double c1, const C* v, double c2,
                 double* dot) const {
        launch_grid<T>(P, y, perm, (C*)P.grid, s);
        launch_fft_cols_adj<T>(P, (const C*)P.grid, (C*)P.tmp, s);
        launch_fft_rows_adj<T>(P, (const C*)P.tmp, x, c1, v, c2, dot, s);
    }
    // q = (Phi~^dag Phi~ + 2 I) v, Phi~ = Phi / nu
    // (G^T G fused: the visibilities of Phi v are interpolated inside the gridding launch)
    void apply_A(const C* v, C* q, double inv_nu2, double* dot) const {
        launch_fft_rows_fwd<T>(P, v, (C*)P.tmp, s);
        normal_tail(v, q, inv_nu2, 2.0, dot);
    }
    // q = Phi^dag Phi v
    void normal(const C* v, C* q) const {
        launch_fft_rows_fwd<T>(P, v, (C*)P.tmp, s);
        normal_tail(nullptr, q, 1.0, 0.0, nullptr);
    }
    // first CG step: the set-up r = p = x1 + x2 + x3 - q0 (partial ||r||^2 into rho, count
    // returned) in the row pass, then q = A p with the partial sums of <p, q>, <r, q> and
    // ||q||^2 (dots[0..2]) for the next step
    int apply_A_first(const C* x1, const C* x2, const C* x3, const C* q0, C* r, C* p, C* q, double inv_nu2,
                      double* rho, double* const* dots) const {
        const int nb = launch_fft_rows_init<T>(P, x1, x2, x3, q0, r, p, rho, (C*)P.tmp, s);
        launch_fft_cols_fwd<T>(P, (const C*)P.tmp, (C*)P.grid, s);
        launch_gtg<T>(P, (const C*)P.grid, (C*)P.grid2, s);
        launch_fft_cols_adj<T>(P, (const C*)P.grid2, (C*)P.tmp, s);
        launch_fft_rows_adj_cg<T>(P, (const C*)P.tmp, q, inv_nu2, p, 2.0, dots[0], r, dots[1], dots[2], s);
        return nb;
    }
    // a later CG step: the row pass applies the previous step's update (x += alpha p,
    // r -= alpha q, p = r + beta p, partial ||r||^2 into rho_new) and transforms the new p;
    // then q = A p with its dot products, as in the first step.  Returns the count of rho_new's
    // partials.
    int apply_A_step(C* x, C* r, C* p, C* q, const double* rho, int rho_count, double* const* dots, int dot_count,
                     double* rho_new, double inv_nu2) const {
        const int nr = launch_fft_rows_xr<T>(P, x, r, p, q, rho, rho_count, dots[0], dots[1], dots[2], dot_count,
                                             rho_new, (C*)P.tmp, s);
        launch_fft_cols_fwd<T>(P, (const C*)P.tmp, (C*)P.grid, s);
        launch_gtg<T>(P, (const C*)P.grid, (C*)P.grid2, s);
        launch_fft_cols_adj<T>(P, (const C*)P.grid2, (C*)P.tmp, s);
        launch_fft_rows_adj_cg<T>(P, (const C*)P.tmp, q, inv_nu2, p, 2.0, dots[0], r, dots[1], dots[2], s);
        return nr;
    }
    // q = c1 T v + c2 v with T the stored (Toeplitz) form of Phi^dag Phi (chat ready)
    void toep_A(const C* v, C* q, double c1, double c2, double* dot) const {
        launch_fft_rows_fwd<T>(P, v, (C*)P.tmp, s, P.unit);
        launch_fft_cols_toep<T>(P, (C*)P.tmp, s);
        launch_fft_rows_adj<T>(P, (const C*)P.tmp, q, c1, v, c2, dot, s, P.unit);
    }
    // CG with T, as apply_A_first / apply_A_step: q = c1 T p + 2 p
    int toep_A_first(const C* x1, const C* x2, const C* x3, const C* q0, C* r, C* p, C* q, double c1,
                     double* rho, double* const* dots) const {
        const int nb = launch_fft_rows_init<T>(P, x1, x2, x3, q0, r, p, rho, (C*)P.tmp, s, P.unit);
        launch_fft_cols_toep<T>(P, (C*)P.tmp, s);
        launch_fft_rows_adj_cg<T>(P, (const C*)P.tmp, q, c1, p, 2.0, dots[0], r, dots[1], dots[2], s, P.unit);
        return nb;
    }
    int toep_A_step(C* x, C* r, C* p, C* q, const double* rho, int rho_count, double* const* dots, int dot_count,
                    double* rho_new, double c1) const {
        const int nr = launch_fft_rows_xr<T>(P, x, r, p, q, rho, rho_count, dots[0], dots[1], dots[2], dot_count,
                                             rho_new, (C*)P.tmp, s, P.unit);
        launch_fft_cols_toep<T>(P, (C*)P.tmp, s);
        launch_fft_rows_adj_cg<T>(P, (const C*)P.tmp, q, c1, p, 2.0, dots[0], r, dots[1], dots[2], s, P.unit);
        return nr;
    }
    // after the row pass of v: q = c1 Phi^dag Phi v + c2 v
    void normal_tail(const C* v, C* q, double c1, double c2, double* dot) const {
        launch_fft_cols_fwd<T>(P, (const C*)P.tmp, (C*)P.grid, s);
        launch_gtg<T>(P, (const C*)P.grid, (C*)P.grid2, s);
        launch_fft_cols_adj<T>(P, (const C*)P.grid2, (C*)P.tmp, s);
        launch_fft_rows_adj<T>(P, (const C*)P.tmp, q, c1, v, c2, dot, s);
    }
};

double* part_buf(const Plan& P, int k) { return P.part + (size_t)k * MAX_PARTIALS; }

// Spectrum of the stored normal operator, computed once per plan (first use): for each
// quadrant shift s in {-n/2, n/2}^2, h_s = Phi^dagger v_s (v_s,m = exp(i omega_m . s)) holds
// h(p + s); the offsets d = -n are zeroed; chat += Re(exp(-2 pi i k . s / K) F Z h_s) / K^2.
// Uses the plan's visibility, grid and image scratch; synchronous on s.
template <typename T>
purify_status ensure_chat(Plan& P, hipStream_t s) {
    if (P.chat_ready) return PURIFY_OK;
    using C = cpx<T>;
    const int h = P.n / 2;
    const int sig[4][2] = {{-1, -1}, {-1, 1}, {1, -1}, {1, 1}};
    for (int q = 0; q < 4; ++q) {
        launch_modulate<T>(P, sig[q][0] * h, sig[q][1] * h, (C*)P.vis, s);
        launch_grid<T>(P, (const C*)P.vis, nullptr, (C*)P.grid, s);
        launch_fft_cols_adj<T>(P, (const C*)P.grid, (C*)P.tmp, s);
        launch_fft_rows_adj<T>(P, (const C*)P.tmp, (C*)P.qv, 1.0, nullptr, 0.0, nullptr, s);
        launch_zero_edge<T>((C*)P.qv, P.n, sig[q][0] < 0, sig[q][1] < 0, s);
        launch_fft_rows_fwd<T>(P, (const C*)P.qv, (C*)P.tmp, s, P.unit);
        launch_fft_cols_fwd<T>(P, (const C*)P.tmp, (C*)P.grid, s);
        launch_chat_accum<T>(P, (const C*)P.grid, sig[q][0], sig[q][1], q == 0, s);
    }
    PURIFY_HIP(hipGetLastError());
    PURIFY_HIP(hipStreamSynchronize(s));
    P.chat_ready = true;
    return PURIFY_OK;
}

template <typename T>
struct Sdmm {
    using C = cpx<T>;
    Plan& P;
    const purify_sdmm_params* prm;
    double inv_nu = 1, inv_nu2 = 1, eps_t = 0, gamma = 0;
    bool toep = false;   // CG operator from the stored normal operator (PURIFY_SDMM_TOEPLITZ)
    int nblk = 0, nchunks = 0;   // visibility blocks (R >= 2) and their reduction chunks
    bool tv = false;             // f1 = total variation with L1 = I (PURIFY_SDMM_TV)

    double* part(int k) const { return part_buf(P, k); }

    // q = A v = Phi~^dag Phi~ v + 2 v (or its stored form), partial <v, q> into dot
    void A(const Ops<T>& op, const C* v, C* q, double* dot) const {
        if (toep) op.toep_A(v, q, inv_nu2, 2.0, dot);
        else op.apply_A(v, q, inv_nu2, dot);
    }

    // One power-iteration step: v <- Phi^dag Phi v / ||Phi^dag Phi v||, lambda in sc.
    void enqueue_power_step(hipStream_t s) const {
        const Ops<T> op{P, s};
        C* v = (C*)P.p;
        C* w = (C*)P.qv;
        op.normal(v, w);
        const int nb = launch_norm2_part<T>(w, P.N, part(6), s);
        launch_power_normalise<T>(v, w, part(6), nb, P.sc, P.N, s);
    }

    // One SDMM iteration (Algorithm 1, steps 5-9).  Branch i = 1 runs on s2 between the
    // fork and join events; CG and branches i = 2, 3 run on s.  Scalars (CG alpha and beta,
    // the l2-ball scale) are summed from partial-sum buffers inside the kernels that use
    // them; rho alternates between buffers 0 and 1, <p, Ap> uses buffer 2.
    void enqueue_iteration(hipStream_t s, hipStream_t s2, hipEvent_t fork, hipEvent_t join, hipEvent_t hat) const {
        const Ops<T> op{P, s};
        const int64_t N = P.N, M = P.M, D = P.D;
        double* sc = P.sc;
        C* xh = (C*)P.xh;
        C *x1 = (C*)P.x1, *x2 = (C*)P.x2, *x3 = (C*)P.x3;
        C *r = (C*)P.r, *p = (C*)P.p, *q = (C*)P.qv;
        C *z1 = (C*)P.z1, *v1 = (C*)P.v1, *z2 = (C*)P.z2, *z3 = (C*)P.z3, *v3 = (C*)P.v3;
        const C* yt = (const C*)P.ytil;
        const int rows_blocks = fft_rows_adj_blocks<T>(P);
        // Global update (step 5): CG on (Phi~^dag Phi~ + 2I) x = x1 + x2 + x3, warm started
        // at x_hat, so r = x1 + x2 + x3 - A x_hat.  With the NUFFT operator, x3 already holds
        // x3 - A x_hat (branch i = 3 below); with the stored operator, q = A x_hat was formed
        // at the end of the previous iteration (or by enqueue_prologue) beside branch i = 1.
        // rho of step c (the residual norm before step c's update) is in buffer c & 1,
        // <p, A p> in buffer 2, <r, A p> and ||A p||^2 in buffers 8 and 9
        // step 0: the set-up r = p = x1 + x2 + x3 (- q) folded into its row pass, then q = A p;
        // step c > 0: step c - 1's update and the new direction p = r + beta p folded into the
        // row pass (beta from ||r - alpha q||^2 expanded in those dot products, so it is known
        // before the new residual is summed), then q = A p (Ops::apply_A_step); then the last
        // step's update
        double* const dots[3] = {part(2), part(8), part(9)};   // <p, q>, <r, q>, ||q||^2
        int rho_count = toep ? op.toep_A_first(x1, x2, x3, q, r, p, q, inv_nu2, part(0), dots)
                             : op.apply_A_first(x1, x2, x3, nullptr, r, p, q, inv_nu2, part(0), dots);
        for (int c = 1; c < prm->cg_iter; ++c) {
            if (toep)
                rho_count = op.toep_A_step(xh, r, p, q, part((c - 1) & 1), rho_count, dots, rows_blocks, part(c & 1),
                                           inv_nu2);
            else
                rho_count = op.apply_A_step(xh, r, p, q, part((c - 1) & 1), rho_count, dots, rows_blocks, part(c & 1),
                                            inv_nu2);
        }
        const int cl = prm->cg_iter;
        // i = 1 (on s2): l1 prior on Psi^dag x_hat.  With the NUFFT operator branch i = 1 is
        // the longer one, so where the analysis can form x_hat = x + alpha p itself it forks
        // before the CG's last update, and the update (which writes x_hat over x) waits only
        // for the finest analysis level, the one launch that reads x and p.  With the stored
        // operator the main stream also forms the next A x_hat and is the longer branch, so
        // it does not wait.
        // The objective's partial sums (part 3, nb1 of them) are summed on the main stream
        // after the join, by the kernel that ends the iteration, off this branch's chain.
        int nb1 = 0;
        if (!tv && !toep && psi_adj_takes_xhat(P)) {
            (void)hipEventRecord(fork, s);
            (void)hipStreamWaitEvent(s2, fork, 0);
            const XhatArgs<T> xa{p, part((cl - 1) & 1), rho_count, part(2), rows_blocks};
            launch_psi_adj<T>(P, xh, v1, s2, &xa, hat);
            (void)hipStreamWaitEvent(s, hat, 0);
            launch_cg_x<T>(xh, p, part((cl - 1) & 1), rho_count, part(2), rows_blocks, N, s);
            nb1 = launch_prox_l1<T>(v1, z1, prm->weights, gamma, D, part(3), s2);
            launch_psi<T>(P, v1, x1, s2);
        } else {
            launch_cg_x<T>(xh, p, part((cl - 1) & 1), rho_count, part(2), rows_blocks, N, s);
            (void)hipEventRecord(fork, s);
            (void)hipStreamWaitEvent(s2, fork, 0);
            if (tv) {   // TV prior: prox on u = x_hat + z1 (in v1), x1 = r1 - z1
                launch_tv_prox<T>(P, xh, z1, x1, v1, prm->weights, gamma, prm->tv_iter, part(3), &nb1, s2);
            } else {
                launch_psi_adj<T>(P, xh, v1, s2);
                nb1 = launch_prox_l1<T>(v1, z1, prm->weights, gamma, D, part(3), s2);
                launch_psi<T>(P, v1, x1, s2);
            }
        }
        (void)hipEventRecord(join, s2);
        // i = 2: positivity
        launch_prox_pos<T>(xh, z2, x2, N, s);
        // i = 3: l2 ball about y~ on Phi~ x_hat.  x3 = Phi~^dag (r3 - z3); with the NUFFT
        // operator the next CG's A x_hat = Phi~^dag (Phi~ x_hat) + 2 x_hat is folded in by
        // linearity: the projection leaves r3 - z3 - Phi~ x_hat in v3 and the adjoint's
        // epilogue subtracts 2 x_hat, so x3 <- x3 - A x_hat costs no operator of its own.
        const bool fold = !toep;
        op.phi(xh, v3, inv_nu, nullptr);
        if (nblk > 1) {   // R balls: chunk sums, per-block scales, projection by block
            launch_ball_part_blk<T>(v3, z3, yt, P.bperm, P.bchunk, nchunks, part(4), part(5), s);
            launch_ball_fin_blk(part(4), part(5), P.bchunk_off, P.beps, nblk, P.bscale, sc, P.hist, P.hist_cap, s);
            launch_prox_ball_blk<T>(v3, z3, yt, P.bid, P.bscale, M, fold, s);
        } else {
            const int nb3 = launch_ball_part<T>(v3, z3, yt, M, part(4), part(5), s);
            launch_prox_ball<T>(v3, z3, yt, part(4), part(5), nb3, eps_t, sc, P.hist, P.hist_cap, M, fold, s);
        }
        if (fold) {
            op.phi_adj(v3, nullptr, x3, inv_nu, xh, -2.0, nullptr);
        } else {
            op.phi_adj(v3, nullptr, x3, inv_nu, nullptr, 0.0, nullptr);
            // the next iteration's warm-start product A x_hat with the stored operator needs
            // only x_hat: it runs here, overlapping branch i = 1 on the other stream
            A(op, xh, q, nullptr);
        }
        (void)hipStreamWaitEvent(s, join, 0);
        launch_finalize(part(3), nb1, sc, SL_OBJ, FIN_HIST_OBJ_END, 0, P.hist, P.hist_cap, s);
    }

    // The first iteration's warm start: q = A x_hat, and with the NUFFT operator
    // x3 <- x3 - q (the form every later iteration's branch i = 3 leaves in x3).
    void enqueue_prologue(hipStream_t s) const {
        const Ops<T> op{P, s};
        A(op, (const C*)P.xh, (C*)P.qv, nullptr);
        if (!toep) launch_sub<T>((C*)P.x3, (const C*)P.qv, P.N, s);
    }
};

// Tables of the visibility blocks for one solve: the block of each sorted visibility, the
// sorted positions grouped by block, chunks of at least 256 of them per reduction workgroup
// (at most BLK_CHUNKS in all) and eps_i / nu.  Host work like the plan's binning; synchronous.
purify_status setup_blocks(const Plan& P, const purify_sdmm_params* prm, double nu, hipStream_t s,
                           int* nchunks_out) {
    const int R = prm->nblocks;
    const int64_t M = P.M;
    const int64_t* off = prm->block_offsets;
    std::vector<int32_t> perm((size_t)M), ublk((size_t)M), bid((size_t)M), bperm((size_t)M);
    PURIFY_HIP(hipMemcpyAsync(perm.data(), P.perm, (size_t)M * 4, hipMemcpyDeviceToHost, s));
    PURIFY_HIP(hipStreamSynchronize(s));
    for (int i = 0; i < R; ++i)
        for (int64_t u = off[i]; u < off[i + 1]; ++u) ublk[(size_t)u] = i;
    std::vector<int64_t> start((size_t)R + 1, 0);
    for (int64_t m = 0; m < M; ++m) {
        bid[(size_t)m] = ublk[(size_t)perm[(size_t)m]];
        ++start[(size_t)bid[(size_t)m] + 1];
    }
    for (int i = 0; i < R; ++i) start[(size_t)i + 1] += start[(size_t)i];
    std::vector<int64_t> fill(start.begin(), start.end() - 1);
    for (int64_t m = 0; m < M; ++m) bperm[(size_t)fill[(size_t)bid[(size_t)m]]++] = (int32_t)m;
    const int64_t per = 256 * 4096;
    const int64_t CH = 256 * std::max<int64_t>(1, (M + per - 1) / per);
    std::vector<int32_t> chunks, coff((size_t)R + 1, 0);
    for (int i = 0; i < R; ++i) {
        coff[(size_t)i] = (int32_t)(chunks.size() / 2);
        for (int64_t a = start[(size_t)i]; a < start[(size_t)i + 1]; a += CH) {
            chunks.push_back((int32_t)a);
            chunks.push_back((int32_t)std::min(a + CH, start[(size_t)i + 1]));
        }
    }
    const int nch = (int)(chunks.size() / 2);
    coff[(size_t)R] = nch;
    if (nch > BLK_CHUNKS) {
        set_error("too many block reduction chunks");
        return PURIFY_E_INVALID;
    }
    std::vector<double> eps((size_t)R);
    for (int i = 0; i < R; ++i) eps[(size_t)i] = prm->block_eps[i] / nu;
    PURIFY_HIP(hipMemcpyAsync(P.bid, bid.data(), (size_t)M * 4, hipMemcpyHostToDevice, s));
    PURIFY_HIP(hipMemcpyAsync(P.bperm, bperm.data(), (size_t)M * 4, hipMemcpyHostToDevice, s));
    PURIFY_HIP(hipMemcpyAsync(P.bchunk, chunks.data(), chunks.size() * 4, hipMemcpyHostToDevice, s));
    PURIFY_HIP(hipMemcpyAsync(P.bchunk_off, coff.data(), coff.size() * 4, hipMemcpyHostToDevice, s));
    PURIFY_HIP(hipMemcpyAsync(P.beps, eps.data(), eps.size() * sizeof(double), hipMemcpyHostToDevice, s));
    PURIFY_HIP(hipStreamSynchronize(s));
    *nchunks_out = nch;
    return PURIFY_OK;
}

// Check the block description of a solve (R <= 1 needs nothing) and the TV step count.
bool blocks_valid(const purify_sdmm_params* prm, int64_t M) {
    if ((prm->flags & PURIFY_SDMM_TV) && prm->tv_iter < 1) return false;
    if (prm->nblocks <= 1) return true;
    if (prm->nblocks > MAX_BLOCKS || !prm->block_offsets || !prm->block_eps) return false;
    const int64_t* off = prm->block_offsets;
    if (off[0] != 0 || off[prm->nblocks] != M) return false;
    for (int i = 0; i < prm->nblocks; ++i) {
        if (off[i + 1] <= off[i]) return false;
        if (!(prm->block_eps[i] >= 0) || !std::isfinite(prm->block_eps[i])) return false;
    }
    return true;
}

// x_in: x_hat(0) (device, N complex) or null for x_hat(0) = 0; x_out: receives x_hat, or null
// to leave it in the plan's x_hat buffer only (x_in and x_out may be the same vector).
template <typename T>
purify_status sdmm_impl(Plan& P, const void* y_user, const purify_sdmm_params* prm, const void* x_in,
                        void* x_out, purify_sdmm_info* info, hipStream_t s) {
    using C = cpx<T>;
    const int64_t N = P.N, M = P.M, D = P.D;
    const C zero = mk<T>(0, 0);
    double* sc = P.sc;
    const bool use_graph = (prm->flags & PURIFY_SDMM_NO_GRAPH) == 0;
    Sdmm<T> S{P, prm};
    if (!P.ss) {
        set_error("plan has no solver streams");
        return PURIFY_E_INVALID;
    }
    {
        const purify_status st = solver_streams_init(*P.ss);
        if (st != PURIFY_OK) return st;
    }
    SolverStreams& R = *P.ss;
    SolveGraphs G(&R);   // drains R's streams before its graphs go, also on error returns
    hipStream_t cs = R.cs;

    // the solver's streams start after the caller's prior work on s
    PURIFY_HIP(hipEventRecord(R.entry, s));
    PURIFY_HIP(hipStreamWaitEvent(cs, R.entry, 0));
    S.toep = (prm->flags & PURIFY_SDMM_TOEPLITZ) != 0;
    S.tv = (prm->flags & PURIFY_SDMM_TV) != 0;
    if (S.toep) {
        const purify_status st = ensure_chat<T>(P, cs);
        if (st != PURIFY_OK) return st;
    }
    const Ops<T> opc{P, cs};
    PURIFY_HIP(hipMemsetAsync(sc, 0, SL_COUNT * sizeof(double), cs));

    // Operator norm nu = ||Phi||_2 by power iteration on Phi^dag Phi from the all-ones image.
    double nu = prm->nu;
    if (!(nu > 0)) {
        launch_fill<T>((C*)P.p, mk<T>((T)(1.0 / std::sqrt((double)N)), 0), N, cs);
        if (use_graph && prm->nu_iter > 1) {
            {
                std::lock_guard<std::mutex> lk(graph_mutex());
                PURIFY_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed));
                S.enqueue_power_step(cs);
                const purify_status st = end_capture(G, 0, cs);
                if (st != PURIFY_OK) return st;
            }
            for (int it = 0; it < prm->nu_iter; ++it) PURIFY_HIP(hipGraphLaunch(G.x[0], cs));
        } else {
            for (int it = 0; it < prm->nu_iter; ++it) S.enqueue_power_step(cs);
        }
        double lam = 0;
        PURIFY_HIP(hipMemcpyAsync(&lam, sc + SL_LAMBDA, sizeof(double), hipMemcpyDeviceToHost, cs));
        PURIFY_HIP(hipStreamSynchronize(cs));
        nu = std::sqrt(lam);
        if (!(nu > 0) || !std::isfinite(nu)) {
            set_error("operator norm is zero or not finite");
            return PURIFY_E_NONFINITE;
        }
    }
    S.inv_nu = 1.0 / nu;
    S.inv_nu2 = S.inv_nu * S.inv_nu;
    S.eps_t = prm->epsilon * S.inv_nu;
    if (prm->nblocks > 1) {
        const purify_status st = setup_blocks(P, prm, nu, cs, &S.nchunks);
        if (st != PURIFY_OK) return st;
        S.nblk = prm->nblocks;
    }

    // y~ = y / nu in solver (tile-sorted) order
    launch_permute_scale<T>((const C*)y_user, P.perm, S.inv_nu, (C*)P.ytil, M, cs);

    // gamma = 1e-3 max |Psi^dag Phi~^dag y~| (TV prior: max |grad Phi~^dag y~|) unless given
    double gamma = prm->gamma;
    if (!(gamma > 0)) {
        opc.phi_adj((const C*)P.ytil, nullptr, (C*)P.p, S.inv_nu, nullptr, 0.0, nullptr);
        int nb = 0;
        if (S.tv) {
            nb = launch_grad_mag<T>(P, (const C*)P.p, nullptr, part_buf(P, 7), cs);
        } else {
            launch_psi_adj<T>(P, (const C*)P.p, (C*)P.v1, cs);
            nb = launch_maxabs_part<T>((const C*)P.v1, D, part_buf(P, 7), cs);
        }
        launch_finalize(part_buf(P, 7), nb, sc, SL_MAXABS, FIN_MAX, 0, nullptr, 0, cs);
        double mx = 0;
        PURIFY_HIP(hipMemcpyAsync(&mx, sc + SL_MAXABS, sizeof(double), hipMemcpyDeviceToHost, cs));
        PURIFY_HIP(hipStreamSynchronize(cs));
        gamma = 1e-3 * mx;
        if (!(gamma > 0)) gamma = 1e-12;
    }
    S.gamma = gamma;

    // Algorithm 1 initialisation: z_i = 0, r_i = L_i x_hat(0), x_i = L_i^dag r_i; with
    // x_hat(0) = 0 every x_i is 0, else x1 = Psi Psi^dag x_hat, x2 = x_hat, x3 = Phi~^dag Phi~ x_hat.
    if (x_in) {
        PURIFY_HIP(hipMemcpyAsync(P.xh, x_in, (size_t)N * sizeof(C), hipMemcpyDeviceToDevice, cs));
        if (S.tv) {   // L1 = I
            PURIFY_HIP(hipMemcpyAsync(P.x1, P.xh, (size_t)N * sizeof(C), hipMemcpyDeviceToDevice, cs));
        } else {
            launch_psi_adj<T>(P, (const C*)P.xh, (C*)P.v1, cs);
            launch_psi<T>(P, (const C*)P.v1, (C*)P.x1, cs);
        }
        PURIFY_HIP(hipMemcpyAsync(P.x2, P.xh, (size_t)N * sizeof(C), hipMemcpyDeviceToDevice, cs));
        launch_fft_rows_fwd<T>(P, (const C*)P.xh, (C*)P.tmp, cs);
        opc.normal_tail(nullptr, (C*)P.x3, S.inv_nu2, 0.0, nullptr);
        launch_fill<T>((C*)P.z2, zero, N, cs);
    } else {
        for (void* v : {P.xh, P.x1, P.x2, P.x3, P.z2}) launch_fill<T>((C*)v, zero, N, cs);
    }
    launch_fill<T>((C*)P.z1, zero, D, cs);
    launch_fill<T>((C*)P.z3, zero, M, cs);
    PURIFY_HIP(hipMemsetAsync(sc, 0, SL_COUNT * sizeof(double), cs));
    S.enqueue_prologue(cs);

    if (use_graph) {
        std::lock_guard<std::mutex> lk(graph_mutex());
        PURIFY_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed));
        S.enqueue_iteration(cs, R.cs2, R.fork, R.join, R.hat);
        const purify_status st = end_capture(G, 1, cs);
        if (st != PURIFY_OK) return st;
    }
    const int T_max = prm->max_iter;
    const int check = prm->check_every > 0 ? prm->check_every : 1;
    int it_done = 0;
    bool converged = false;
    for (int t = 0; t < T_max; ++t) {
        if (use_graph) PURIFY_HIP(hipGraphLaunch(G.x[1], cs));
        else S.enqueue_iteration(cs, R.cs2, R.fork, R.join, R.hat);
        it_done = t + 1;
        if (prm->halting && t >= 1 && ((t + 1) % check == 0 || t + 1 == T_max)) {
            double h[5] = {0, 0, 0, 0, 0};
            const int hi = t % P.hist_cap, hp = (t - 1) % P.hist_cap;
            PURIFY_HIP(hipMemcpyAsync(h, P.hist + 2 * hp, 2 * sizeof(double), hipMemcpyDeviceToHost, cs));
            PURIFY_HIP(hipMemcpyAsync(h + 2, P.hist + 2 * hi, 2 * sizeof(double), hipMemcpyDeviceToHost, cs));
            if (S.nblk > 1)
                PURIFY_HIP(hipMemcpyAsync(h + 4, sc + SL_BLK_RATIO, sizeof(double), hipMemcpyDeviceToHost, cs));
            PURIFY_HIP(hipStreamSynchronize(cs));
            const double f = h[2], fp = h[0], res = h[3];
            if (!std::isfinite(f) || !std::isfinite(res)) break;
            // every data constraint within its bound (one ball, or each block's)
            const bool feasible = S.nblk > 1 ? h[4] <= 1.0 + prm->slack : res <= S.eps_t * (1.0 + prm->slack);
            if (f > 0 && std::fabs(f - fp) / f < prm->xi && feasible) {
                converged = true;
                break;
            }
        }
    }
    if (x_out) PURIFY_HIP(hipMemcpyAsync(x_out, P.xh, (size_t)N * sizeof(C), hipMemcpyDeviceToDevice, cs));
    double scal[SL_COUNT];
    PURIFY_HIP(hipMemcpyAsync(scal, sc, sizeof(scal), hipMemcpyDeviceToHost, cs));
    if (prm->history) {
        const int cnt = it_done < P.hist_cap ? it_done : P.hist_cap;
        PURIFY_HIP(hipMemcpyAsync(prm->history, P.hist, (size_t)2 * cnt * sizeof(double),
                                  hipMemcpyDeviceToHost, cs));
    }
    // cs has drained (branch i = 1 joins it inside every iteration), so the caller's later
    // work on s, enqueued after this call returns, is ordered after the solve
    PURIFY_HIP(hipStreamSynchronize(cs));
    if (info) {
        info->iterations = it_done;
        info->converged = converged ? 1 : 0;
        info->objective = scal[SL_OBJ];
        info->residual = std::sqrt(scal[SL_RES2]) * nu;
        info->nu = nu;
        info->gamma = gamma;
    }
    if (scal[SL_NONFINITE] != 0.0 || !std::isfinite(scal[SL_OBJ]) || !std::isfinite(scal[SL_RES2])) {
        set_error("non-finite objective or residual in SDMM");
        return PURIFY_E_NONFINITE;
    }
    return PURIFY_OK;
}

// Reweighted l1 (SARA, Section 2.2): solve 0 with the caller's W, then weighted solves with
// w_j = delta / (delta + |(Psi^dag x_prev)_j|), each warm started from the previous x_hat
// with the nu and gamma of solve 0.  delta_1 = max(delta0 or the standard deviation of
// Psi^dag x(0), delta_min), then delta <- max(decay delta, delta_min); stop when the relative
// variation ||x(k) - x(k-1)|| / ||x(k-1)|| drops below rel_var.  Statistics are summed by
// the reduction kernels; the host only reads the resulting scalars between solves.
template <typename T>
purify_status reweighted_impl(Plan& P, const void* y, const purify_sdmm_params* prm,
                              const purify_reweight_params* rw, double* weights, void* x_io,
                              purify_sdmm_info* info, purify_reweight_info* rinfo, hipStream_t s) {
    using C = cpx<T>;
    const int64_t N = P.N, M = P.M;
    purify_sdmm_info inf{};
    purify_reweight_info out{};
    out.solves = 1;
    out.rel_var = -1.0;
    const bool warm0 = (prm->flags & PURIFY_SDMM_WARM_START) != 0;
    purify_status st = sdmm_impl<T>(P, y, prm, warm0 ? x_io : nullptr, x_io, &inf, s);
    out.total_iterations = inf.iterations;
    if (st == PURIFY_OK && rw->reweights > 0) {
        purify_sdmm_params pk = *prm;
        pk.nu = inf.nu;
        pk.gamma = inf.gamma;
        pk.weights = weights;
        pk.flags = prm->flags | PURIFY_SDMM_WARM_START;
        // noise level behind the chi-square bound(s): eps = sigma sqrt(M + 2 sqrt M) per constraint
        double sigma = prm->epsilon / std::sqrt((double)M + 2.0 * std::sqrt((double)M));
        if (prm->nblocks > 1) {
            sigma = 0;
            for (int i = 0; i < prm->nblocks; ++i) {
                const double m = (double)(prm->block_offsets[i + 1] - prm->block_offsets[i]);
                sigma = std::max(sigma, prm->block_eps[i] / std::sqrt(m + 2.0 * std::sqrt(m)));
            }
        }
        const double floor = rw->delta_min >= 0 ? rw->delta_min : sigma / inf.nu;
        double* sc = P.sc;
        // coefficients: Psi^dag x, or |grad x| for the TV prior (N of them)
        const bool tv = (prm->flags & PURIFY_SDMM_TV) != 0;
        const int64_t D = tv ? N : P.D;
        auto coefficients = [&]() {
            if (tv) launch_grad_mag<T>(P, (const C*)x_io, (C*)P.v1, nullptr, s);
            else launch_psi_adj<T>(P, (const C*)x_io, (C*)P.v1, s);
        };
        coefficients();
        double delta = rw->delta0;
        if (!(delta > 0)) {   // standard deviation of the coefficients, two passes
            const int nb = launch_sum_part<T>((const C*)P.v1, D, part_buf(P, 0), part_buf(P, 1), s);
            launch_finalize(part_buf(P, 0), nb, sc, SL_RW_A, FIN_STORE, 0.0, nullptr, 0, s);
            launch_finalize(part_buf(P, 1), nb, sc, SL_RW_B, FIN_STORE, 0.0, nullptr, 0, s);
            const int nb2 = launch_dev2_part<T>((const C*)P.v1, D, sc, SL_RW_A, SL_RW_B, part_buf(P, 2), s);
            launch_finalize(part_buf(P, 2), nb2, sc, SL_RW_C, FIN_STORE, 0.0, nullptr, 0, s);
            double dev2 = 0;
            PURIFY_HIP(hipMemcpyAsync(&dev2, sc + SL_RW_C, sizeof(double), hipMemcpyDeviceToHost, s));
            PURIFY_HIP(hipStreamSynchronize(s));
            delta = std::sqrt(dev2 / (double)D);
        }
        delta = std::max(delta, floor);
        for (int k = 1; k <= rw->reweights; ++k) {
            launch_reweight<T>((const C*)P.v1, D, delta, weights, s);
            st = sdmm_impl<T>(P, y, &pk, x_io, nullptr, &inf, s);
            ++out.solves;
            out.total_iterations += inf.iterations;
            out.delta = delta;
            if (st != PURIFY_OK) break;
            const int nb = launch_diff2_part<T>((const C*)P.xh, (const C*)x_io, N, part_buf(P, 0),
                                                part_buf(P, 1), s);
            launch_finalize(part_buf(P, 0), nb, sc, SL_RW_A, FIN_STORE, 0.0, nullptr, 0, s);
            launch_finalize(part_buf(P, 1), nb, sc, SL_RW_B, FIN_STORE, 0.0, nullptr, 0, s);
            double ab[2] = {0, 0};
            static_assert(SL_RW_B == SL_RW_A + 1, "adjacent slots");
            PURIFY_HIP(hipMemcpyAsync(ab, sc + SL_RW_A, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
            PURIFY_HIP(hipMemcpyAsync(x_io, P.xh, (size_t)N * sizeof(C), hipMemcpyDeviceToDevice, s));
            PURIFY_HIP(hipStreamSynchronize(s));
            const double d = std::sqrt(ab[0]), o = std::sqrt(ab[1]);
            const double rv = o > 0 ? d / o : (d == 0 ? 0.0 : INFINITY);
            out.rel_var = rv;
            if (rv < rw->rel_var) break;
            delta = std::max(rw->decay * delta, floor);
            coefficients();
        }
    }
    if (info) *info = inf;
    if (rinfo) *rinfo = out;
    return st;
}

template <typename T>
void run_stage(const Plan& P, int stage, hipStream_t s) {
    using C = cpx<T>;
    const Ops<T> op{P, s};
    switch (stage) {
        case PURIFY_STAGE_FFT_ROWS: launch_fft_rows_fwd<T>(P, (const C*)P.xh, (C*)P.tmp, s); break;
        case PURIFY_STAGE_FFT_COLS: launch_fft_cols_fwd<T>(P, (const C*)P.tmp, (C*)P.grid, s); break;
        case PURIFY_STAGE_DEGRID: launch_degrid<T>(P, (const C*)P.grid, (C*)P.vis, nullptr, 1.0, s); break;
        case PURIFY_STAGE_GRID: launch_grid<T>(P, (const C*)P.vis, nullptr, (C*)P.grid, s); break;
        case PURIFY_STAGE_GTG: launch_gtg<T>(P, (const C*)P.grid, (C*)P.grid2, s); break;
        case PURIFY_STAGE_IFFT_COLS: launch_fft_cols_adj<T>(P, (const C*)P.grid, (C*)P.tmp, s); break;
        case PURIFY_STAGE_IFFT_ROWS:
            launch_fft_rows_adj<T>(P, (const C*)P.tmp, (C*)P.qv, 1.0, nullptr, 0.0, nullptr, s);
            break;
        case PURIFY_STAGE_PHI: op.phi((const C*)P.xh, (C*)P.vis, 1.0, nullptr); break;
        case PURIFY_STAGE_PHI_ADJ: op.phi_adj((const C*)P.vis, nullptr, (C*)P.qv, 1.0, nullptr, 0.0, nullptr); break;
        case PURIFY_STAGE_PSI_ADJ: launch_psi_adj<T>(P, (const C*)P.xh, (C*)P.v1, s); break;
        case PURIFY_STAGE_PSI: launch_psi<T>(P, (const C*)P.v1, (C*)P.qv, s); break;
        case PURIFY_STAGE_TOEP_COLS: launch_fft_cols_toep<T>(P, (C*)P.tmp, s); break;
        case PURIFY_STAGE_TOEP_NORMAL: op.toep_A((const C*)P.xh, (C*)P.qv, 1.0, 0.0, nullptr); break;
        case PURIFY_STAGE_TV_STEP: launch_tv_step<T>(P, (const C*)P.xh, 1, nullptr, 1.0, s); break;
        default: break;
    }
}

bool f64(const Plan& P) { return P.precision == PURIFY_FP64; }

}  // namespace

void set_error(const std::string& msg) { g_last_error = msg; }

}  // namespace purify

using namespace purify;

#define CHECK_PLAN(pl)                                   \
    do {                                                 \
        if (!(pl)) {                                     \
            set_error("null plan");                      \
            return PURIFY_E_INVALID;                     \
        }                                                \
    } while (0)

#define CHECK_LAUNCH()                                                           \
    do {                                                                         \
        hipError_t _e = hipGetLastError();                                       \
        if (_e != hipSuccess) {                                                  \
            set_error(std::string("kernel launch: ") + hipGetErrorString(_e));   \
            return PURIFY_E_DEVICE;                                              \
        }                                                                        \
    } while (0)

extern "C" {

size_t purify_plan_workspace_bytes(const purify_plan_desc* desc) {
    const DescCheck c = check_desc(desc);
    if (!c.ok) {
        set_error(c.why);
        return 0;
    }
    Plan P;
    return layout(P, desc, nullptr);
}

int64_t purify_plan_dict_size(const purify_plan_desc* desc) {
    const DescCheck c = check_desc(desc);
    if (!c.ok) {
        set_error(c.why);
        return 0;
    }
    Plan P;
    layout(P, desc, nullptr);
    return P.D;
}

purify_status purify_plan_create(const purify_plan_desc* desc, void* workspace, size_t bytes,
                                 void* stream, purify_plan** out) {
    if (!out) {
        set_error("null output pointer");
        return PURIFY_E_INVALID;
    }
    *out = nullptr;
    const DescCheck c = check_desc(desc);
    if (!c.ok) {
        set_error(c.why);
        return PURIFY_E_INVALID;
    }
    if (!desc->uv) {
        set_error("null uv");
        return PURIFY_E_INVALID;
    }
    purify_plan* h = new (std::nothrow) purify_plan();
    if (!h) {
        set_error("host allocation failed");
        return PURIFY_E_INVALID;
    }
    Plan& P = h->P;
    const size_t need = layout(P, desc, nullptr);
    if (!workspace || bytes < need || (reinterpret_cast<uintptr_t>(workspace) & 255u)) {
        set_error("workspace missing, unaligned or smaller than " + std::to_string(need) + " bytes");
        delete h;
        return PURIFY_E_WORKSPACE;
    }
    layout(P, desc, (char*)workspace);
    P.ss = &h->own;
    P.ws = (char*)workspace;
    P.ws_bytes = bytes;
    const purify_status st = build_plan(P, desc, (hipStream_t)stream);
    if (st != PURIFY_OK) {
        delete h;
        return st;
    }
    *out = h;
    return PURIFY_OK;
}

void purify_plan_destroy(purify_plan* plan) {
    if (!plan) return;
    solver_streams_release(plan->own);
    delete plan;
}

purify_status purify_phi(const purify_plan* plan, const void* x, void* y, void* stream) {
    CHECK_PLAN(plan);
    if (!x || !y) {
        set_error("null vector");
        return PURIFY_E_INVALID;
    }
    const Plan& P = plan->P;
    hipStream_t s = (hipStream_t)stream;
    if (f64(P)) Ops<double>{P, s}.phi((const cpx<double>*)x, (cpx<double>*)y, 1.0, P.perm);
    else Ops<float>{P, s}.phi((const cpx<float>*)x, (cpx<float>*)y, 1.0, P.perm);
    CHECK_LAUNCH();
    return PURIFY_OK;
}

purify_status purify_phi_adj(const purify_plan* plan, const void* y, void* x, void* stream) {
    CHECK_PLAN(plan);
    if (!x || !y) {
        set_error("null vector");
        return PURIFY_E_INVALID;
    }
    const Plan& P = plan->P;
    hipStream_t s = (hipStream_t)stream;
    if (f64(P)) Ops<double>{P, s}.phi_adj((const cpx<double>*)y, P.perm, (cpx<double>*)x, 1.0, nullptr, 0.0, nullptr);
    else Ops<float>{P, s}.phi_adj((const cpx<float>*)y, P.perm, (cpx<float>*)x, 1.0, nullptr, 0.0, nullptr);
    CHECK_LAUNCH();
    return PURIFY_OK;
}

purify_status purify_psi(const purify_plan* plan, const void* alpha, void* x, void* stream) {
    CHECK_PLAN(plan);
    if (!x || !alpha) {
        set_error("null vector");
        return PURIFY_E_INVALID;
    }
    const Plan& P = plan->P;
    hipStream_t s = (hipStream_t)stream;
    if (f64(P)) launch_psi<double>(P, (const cpx<double>*)alpha, (cpx<double>*)x, s);
    else launch_psi<float>(P, (const cpx<float>*)alpha, (cpx<float>*)x, s);
    CHECK_LAUNCH();
    return PURIFY_OK;
}

purify_status purify_psi_adj(const purify_plan* plan, const void* x, void* alpha, void* stream) {
    CHECK_PLAN(plan);
    if (!x || !alpha) {
        set_error("null vector");
        return PURIFY_E_INVALID;
    }
    const Plan& P = plan->P;
    hipStream_t s = (hipStream_t)stream;
    if (f64(P)) launch_psi_adj<double>(P, (const cpx<double>*)x, (cpx<double>*)alpha, s);
    else launch_psi_adj<float>(P, (const cpx<float>*)x, (cpx<float>*)alpha, s);
    CHECK_LAUNCH();
    return PURIFY_OK;
}

purify_status purify_sdmm_solve(purify_plan* plan, const void* y, const purify_sdmm_params* params,
                                void* x_out, purify_sdmm_info* info, void* stream) {
    CHECK_PLAN(plan);
    if (!y || !params || !x_out) {
        set_error("null argument");
        return PURIFY_E_INVALID;
    }
    if (params->max_iter < 1 || params->cg_iter < 1 || !(params->epsilon >= 0) ||
        (params->nu <= 0 && params->nu_iter < 1)) {
        set_error("invalid SDMM parameters (max_iter, cg_iter >= 1; epsilon >= 0; nu_iter >= 1 when nu <= 0)");
        return PURIFY_E_INVALID;
    }
    Plan& P = plan->P;
    if (!blocks_valid(params, P.M)) {
        set_error("invalid visibility blocks (2 <= R <= 1024, offsets 0 .. M strictly increasing, eps_i >= 0) "
                  "or TV step count (tv_iter >= 1)");
        return PURIFY_E_INVALID;
    }
    hipStream_t s = (hipStream_t)stream;
    const void* x_in = (params->flags & PURIFY_SDMM_WARM_START) ? x_out : nullptr;
    purify_status st = f64(P) ? sdmm_impl<double>(P, y, params, x_in, x_out, info, s)
                              : sdmm_impl<float>(P, y, params, x_in, x_out, info, s);
    if (st == PURIFY_OK) CHECK_LAUNCH();
    return st;
}

purify_status purify_sdmm_reweighted(purify_plan* plan, const void* y, const purify_sdmm_params* params,
                                     const purify_reweight_params* rw, double* weights, void* x_io,
                                     purify_sdmm_info* info, purify_reweight_info* rw_info, void* stream) {
    CHECK_PLAN(plan);
    if (!y || !params || !rw || !x_io || (rw->reweights > 0 && !weights)) {
        set_error("null argument");
        return PURIFY_E_INVALID;
    }
    if (params->max_iter < 1 || params->cg_iter < 1 || !(params->epsilon >= 0) ||
        (params->nu <= 0 && params->nu_iter < 1)) {
        set_error("invalid SDMM parameters (max_iter, cg_iter >= 1; epsilon >= 0; nu_iter >= 1 when nu <= 0)");
        return PURIFY_E_INVALID;
    }
    if (rw->reweights < 0 || !(rw->decay > 0 && rw->decay <= 1) || !std::isfinite(rw->delta0) ||
        !std::isfinite(rw->delta_min) || !(rw->rel_var >= 0)) {
        set_error("invalid reweighting parameters (reweights >= 0, 0 < decay <= 1, finite deltas, rel_var >= 0)");
        return PURIFY_E_INVALID;
    }
    Plan& P = plan->P;
    if (!blocks_valid(params, P.M)) {
        set_error("invalid visibility blocks (2 <= R <= 1024, offsets 0 .. M strictly increasing, eps_i >= 0) "
                  "or TV step count (tv_iter >= 1)");
        return PURIFY_E_INVALID;
    }
    hipStream_t s = (hipStream_t)stream;
    purify_status st = f64(P) ? reweighted_impl<double>(P, y, params, rw, weights, x_io, info, rw_info, s)
                              : reweighted_impl<float>(P, y, params, rw, weights, x_io, info, rw_info, s);
    if (st == PURIFY_OK) CHECK_LAUNCH();
    return st;
}

purify_status purify_phi_normal(purify_plan* plan, const void* x, void* out, int32_t mode, void* stream) {
    CHECK_PLAN(plan);
    if (!x || !out || (mode != 0 && mode != PURIFY_NORMAL_TOEPLITZ)) {
        set_error("null vector or unknown mode");
        return PURIFY_E_INVALID;
    }
    Plan& P = plan->P;
    hipStream_t s = (hipStream_t)stream;
    if (mode == PURIFY_NORMAL_TOEPLITZ) {
        const purify_status st = f64(P) ? ensure_chat<double>(P, s) : ensure_chat<float>(P, s);
        if (st != PURIFY_OK) return st;
        if (f64(P)) Ops<double>{P, s}.toep_A((const cpx<double>*)x, (cpx<double>*)out, 1.0, 0.0, nullptr);
        else Ops<float>{P, s}.toep_A((const cpx<float>*)x, (cpx<float>*)out, 1.0, 0.0, nullptr);
    } else {
        if (f64(P)) Ops<double>{P, s}.normal((const cpx<double>*)x, (cpx<double>*)out);
        else Ops<float>{P, s}.normal((const cpx<float>*)x, (cpx<float>*)out);
    }
    CHECK_LAUNCH();
    return PURIFY_OK;
}

purify_status purify_time_stage(purify_plan* plan, int32_t stage, int32_t reps, void* stream,
                                double* ms_per_launch) {
    CHECK_PLAN(plan);
    if (stage < 0 || stage > PURIFY_STAGE_TV_STEP || reps < 1 || !ms_per_launch) {
        set_error("invalid stage or reps");
        return PURIFY_E_INVALID;
    }
    Plan& P = plan->P;
    hipStream_t s = (hipStream_t)stream;
    if (stage == PURIFY_STAGE_TOEP_COLS || stage == PURIFY_STAGE_TOEP_NORMAL) {
        const purify_status st = f64(P) ? ensure_chat<double>(P, s) : ensure_chat<float>(P, s);
        if (st != PURIFY_OK) return st;
    }
    hipEvent_t e0, e1;
    PURIFY_HIP(hipEventCreate(&e0));
    PURIFY_HIP(hipEventCreate(&e1));
    PURIFY_HIP(hipEventRecord(e0, s));
    for (int i = 0; i < reps; ++i) {
        if (f64(P)) run_stage<double>(P, stage, s);
        else run_stage<float>(P, stage, s);
    }
    PURIFY_HIP(hipEventRecord(e1, s));
    PURIFY_HIP(hipEventSynchronize(e1));
    float ms = 0;
    PURIFY_HIP(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *ms_per_launch = (double)ms / reps;
    CHECK_LAUNCH();
    return PURIFY_OK;
}

int32_t purify_daubechies_filter(int32_t b, double* h, int32_t cap) {
    double tmp[2 * 8];
    const int F = daubechies(b, tmp);
    if (F < 0) return -1;
    for (int i = 0; i < F && i < cap; ++i) h[i] = tmp[i];
    return F;
}

int32_t purify_kb_kernel(int32_t J, double beta, int32_t count, const double* t, double* out) {
    if (J < 2 || J > 16 || count < 0 || (count > 0 && (!t || !out))) return -1;
    if (!(beta > 0)) beta = 2.34 * J;
    const int deg = KBDeg<double>::value;
    std::vector<long double> c((size_t)J * (deg + 1));
    kb_fit(J, beta, deg, c.data());
    for (int i = 0; i < count; ++i) out[i] = kb_eval_fit(c.data(), J, deg, t[i]);
    return count;
}

int32_t purify_deapodisation(int32_t n, int32_t K, int32_t J, double beta, double* out) {
    if (n < 1 || K < 1 || J < 2 || J > 16 || !out) return -1;
    if (!(beta > 0)) beta = 2.34 * J;
    const long double i0b = kb_i0((long double)beta);
    for (int j = 0; j < n; ++j) out[j] = 1.0 / kb_hat((double)(j - n / 2) / K, J, beta, i0b);
    return n;
}

const char* purify_status_string(purify_status status) {
    switch (status) {
        case PURIFY_OK: return "ok";
        case PURIFY_E_INVALID: return "invalid argument";
        case PURIFY_E_WORKSPACE: return "workspace too small or missing";
        case PURIFY_E_DEVICE: return "HIP device error";
        case PURIFY_E_NONFINITE: return "non-finite value in the solver";
        default: return "unknown status";
    }
}

const char* purify_last_error(void) { return g_last_error.c_str(); }

const char* purify_version(void) { return "purify-mi355x 0.1.0 (gfx950)"; }

}  // extern "C"
