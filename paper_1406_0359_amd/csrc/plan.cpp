// Plan construction for libpurify: host-side set-up of the measurement operator and the
// dictionary (Section 4 NUFFT; Section 2.2 SARA), and the layout of the caller's workspace.
//
// Everything here runs once per plan on the host in long double / double:
//  * Kaiser-Bessel series coefficients and I0(beta);
//  * deapodisation s_j = 1 / psi_hat((j - n/2) / K);
//  * FFT twiddle tables exp(-2 pi i t / n) and exp(-pi i t / n);
//  * Daubechies Db1..Db8 extremal-phase filters by spectral factorisation (own root finder);
//  * uv wrapping, grid coordinates kappa = omega K / (2 pi), first taps and fractions, and a
//    stable counting sort of the visibilities by (grid tile, spill class).
#include <algorithm>
#include <atomic>
#include <cmath>
#include <complex>
#include <cstring>
#include <mutex>
#include <thread>
#include <vector>

#include "common.h"

namespace purify {

namespace {

constexpr long double PI_L = 3.141592653589793238462643383279502884L;
constexpr int HIST_CAP = 65536;

long double i0_series(long double x) {
    // I0(x) = sum_k (x^2/4)^k / (k!)^2, all terms positive
    const long double w = x * x / 4.0L;
    long double term = 1.0L, sum = 1.0L;
    for (int k = 1; k < 400; ++k) {
        term *= w / ((long double)k * k);
        sum += term;
        if (term < sum * 1e-22L) break;
    }
    return sum;
}

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

bool is_pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

}  // namespace

// ---------------------------------------------------------------------------------------
long double kb_i0(long double x) { return i0_series(x); }

namespace {
long double psi_ld(long double t, int J, long double beta, long double i0b) {
    const long double u = 1.0L - (2.0L * t / J) * (2.0L * t / J);
    if (u < 0) return 0.0L;
    return i0_series(beta * sqrtl(u)) / i0b;
}
}  // namespace

// Per-tap polynomial fit of psi on each tap's unit interval: tap a covers
// t = x + 1/2 + (J/2 - 1) - a, x in [-1/2, 1/2].  Chebyshev interpolation at deg+1 nodes
// (long double), converted to monomials in x.  Returns the max abs error of the double
// Horner evaluation against the Bessel series over a fine grid.
double kb_fit(int J, double beta, int deg, long double* coef) {
    const long double i0b = i0_series((long double)beta);
    const long double h = 0.5L * J - 1.0L;
    const int nc = deg + 1;
    std::vector<long double> vals(nc), b(nc), tj(nc), tjm(nc), tjp(nc), mono(nc);
    for (int a = 0; a < J; ++a) {
        for (int i = 0; i < nc; ++i) {
            const long double y = cosl(PI_L * (i + 0.5L) / nc);     // node in [-1, 1]
            vals[i] = psi_ld(0.5L * y + 0.5L + h - a, J, beta, i0b);
        }
        for (int j = 0; j < nc; ++j) {
            long double acc = 0;
            for (int i = 0; i < nc; ++i) acc += vals[i] * cosl(PI_L * j * (i + 0.5L) / nc);
            b[j] = acc * 2.0L / nc;
        }
        b[0] *= 0.5L;
        // sum_j b_j T_j(y), y = 2x, as monomials in y
        std::fill(mono.begin(), mono.end(), 0.0L);
        std::fill(tjm.begin(), tjm.end(), 0.0L);
        std::fill(tj.begin(), tj.end(), 0.0L);
        tjm[0] = 1.0L;            // T_0
        if (nc > 1) tj[1] = 1.0L; // T_1
        for (int k = 0; k < nc; ++k) mono[k] += b[0] * tjm[k];
        for (int j = 1; j < nc; ++j) {
            for (int k = 0; k < nc; ++k) mono[k] += b[j] * tj[k];
            // T_{j+1} = 2 y T_j - T_{j-1}
            std::fill(tjp.begin(), tjp.end(), 0.0L);
            for (int k = 0; k + 1 < nc; ++k) tjp[k + 1] = 2.0L * tj[k];
            for (int k = 0; k < nc; ++k) tjp[k] -= tjm[k];
            tjm.swap(tj);
            tj.swap(tjp);
        }
        long double p2 = 1.0L;
        for (int k = 0; k < nc; ++k) {
            coef[a * nc + k] = mono[k] * p2;   // y^k = 2^k x^k
            p2 *= 2.0L;
        }
    }
    double err = 0;
    const int S = 2001;
    for (int a = 0; a < J; ++a)
        for (int i = 0; i < S; ++i) {
            const double x = -0.5 + (double)i / (S - 1);
            double acc = (double)coef[a * nc + nc - 1];
            for (int k = nc - 2; k >= 0; --k) acc = acc * x + (double)coef[a * nc + k];
            const double ref = (double)psi_ld((long double)x + 0.5L + h - a, J, beta, i0b);
            err = std::max(err, std::fabs(acc - ref));
        }
    return err;
}

// Evaluate the fitted psi at any t in [-J/2, J/2) (0 outside), as the kernels do in FP64.
double kb_eval_fit(const long double* coef, int J, int deg, double t) {
    const double h = 0.5 * J - 1.0;
    const int a = (int)std::ceil(h - t);
    if (a < 0 || a >= J) return 0.0;
    const double x = t - h + a - 0.5;
    const int nc = deg + 1;
    double acc = (double)coef[a * nc + nc - 1];
    for (int k = nc - 2; k >= 0; --k) acc = acc * x + (double)coef[a * nc + k];
    return acc;
}

double kb_hat(double nu, int J, double beta, long double i0b) {
    const long double z2 = (long double)beta * beta - powl(PI_L * J * nu, 2);
    long double v;
    if (z2 > 0) {
        const long double z = sqrtl(z2);
        v = J * sinhl(z) / z;
    } else if (z2 < 0) {
        const long double z = sqrtl(-z2);
        v = J * sinl(z) / z;
    } else {
        v = J;
    }
    return (double)(v / i0b);
}

// ---------------------------------------------------------------------------------------
// Daubechies filters.  |H(w)|^2 = 2 cos^{2N}(w/2) P(sin^2(w/2)) with
// P(y) = sum_{k<N} C(N-1+k, k) y^k.  Roots of P by the Weierstrass (Durand-Kerner)
// iteration in long double, polished by Newton; each root y gives the pair z, 1/z of
// z^2 - (2 - 4y) z + 1 = 0 and the one inside the unit circle is kept (extremal phase).
// h = coefficients of (z + 1)^N prod (z - z_r), highest power first, scaled to sum sqrt 2.
int daubechies_compute(int N, double* h_out) {
    typedef std::complex<long double> C;
    if (N < 1 || N > 8) return -1;
    std::vector<long double> pc(N);
    for (int k = 0; k < N; ++k) {
        long double b = 1.0L;   // C(N-1+k, k)
        for (int j = 1; j <= k; ++j) b = b * (N - 1 + j) / j;
        pc[k] = b;
    }
    const int deg = N - 1;
    std::vector<C> roots;
    if (deg > 0) {
        auto peval = [&](C y) {
            C acc = pc[deg];
            for (int k = deg - 1; k >= 0; --k) acc = acc * y + pc[k];
            return acc;
        };
        auto dpeval = [&](C y) {
            C acc = (long double)deg * pc[deg];
            for (int k = deg - 1; k >= 1; --k) acc = acc * y + (long double)k * pc[k];
            return acc;
        };
        roots.resize(deg);
        C seed(0.4L, 0.9L), cur(1.0L, 0.0L);
        for (int i = 0; i < deg; ++i) {
            cur *= seed;
            roots[i] = cur;
        }
        for (int it = 0; it < 2000; ++it) {
            long double change = 0;
            for (int i = 0; i < deg; ++i) {
                C den = pc[deg];
                for (int j = 0; j < deg; ++j)
                    if (j != i) den *= (roots[i] - roots[j]);
                const C d = peval(roots[i]) / den;
                roots[i] -= d;
                change = std::max(change, std::abs(d));
            }
            if (change < 1e-30L) break;
        }
        for (int i = 0; i < deg; ++i)
            for (int it = 0; it < 4; ++it) roots[i] -= peval(roots[i]) / dpeval(roots[i]);
    }
    std::vector<C> poly(1, C(1.0L, 0.0L));
    auto mul_lin = [&](C a) {   // poly *= (z - a), highest power first
        std::vector<C> out(poly.size() + 1, C(0, 0));
        for (size_t i = 0; i < poly.size(); ++i) {
            out[i] += poly[i];
            out[i + 1] -= a * poly[i];
        }
        poly.swap(out);
    };
    for (int i = 0; i < N; ++i) mul_lin(C(-1.0L, 0.0L));
    for (const C& y : roots) {
        const C b = 2.0L - 4.0L * y;
        const C disc = std::sqrt(b * b - 4.0L);
        const C z1 = (b + disc) / 2.0L, z2 = (b - disc) / 2.0L;
        mul_lin(std::abs(z1) < 1.0L ? z1 : z2);
    }
    long double sum = 0;
    for (const C& c : poly) sum += c.real();
    const long double scale = sqrtl(2.0L) / sum;
    for (int i = 0; i < 2 * N; ++i) h_out[i] = (double)(poly[i].real() * scale);
    return 2 * N;
}

// ---------------------------------------------------------------------------------------
DescCheck check_desc(const purify_plan_desc* d) {
    DescCheck c;
    if (!d) { c.why = "null descriptor"; return c; }
    if (!is_pow2(d->n) || d->n < 16 || d->n > 4096) { c.why = "n must be a power of two in [16, 4096]"; return c; }
    if (d->oversample != 2) { c.why = "oversample must be 2"; return c; }
    if (d->J < 2 || d->J > 16) { c.why = "J must be in [2, 16]"; return c; }
    if (d->M < 1 || d->M >= (int64_t)1 << 31) { c.why = "M must be in [1, 2^31)"; return c; }
    if ((d->dict_mask & 0x1FFu) == 0 || (d->dict_mask & ~0x1FFu)) { c.why = "dict_mask must be a nonzero subset of 0x1FF"; return c; }
    if (d->levels < 1 || d->levels > 8) { c.why = "levels must be in [1, 8]"; return c; }
    if (d->n % (1 << d->levels) != 0 || (d->n >> d->levels) < 1) { c.why = "n must be divisible by 2^levels"; return c; }
    if (d->precision != PURIFY_FP64 && d->precision != PURIFY_FP32) { c.why = "unknown precision"; return c; }
    c.ok = true;
    return c;
}

// Fill the descriptor-derived fields and carve the workspace (ws may be null: sizing only).
size_t layout(Plan& P, const purify_plan_desc* d, char* ws) {
    P.n = d->n;
    P.K = 2 * d->n;
    P.J = d->J;
    P.M = d->M;
    P.levels = d->levels;
    P.precision = d->precision;
    P.beta = d->beta > 0 ? d->beta : 2.34 * d->J;
    P.dict_mask = d->dict_mask & 0x1FFu;
    P.has_dirac = (P.dict_mask & 1u) != 0;
    P.q = 0;
    P.nwav = 0;
    for (int b = 0; b < 9; ++b)
        if (P.dict_mask >> b & 1u) {
            if (b > 0) {
                P.wav_N[P.nwav] = b;
                P.wav_block[P.nwav] = P.q;
                ++P.nwav;
            }
            ++P.q;
        }
    P.N = (int64_t)P.n * P.n;
    P.D = (int64_t)P.q * P.N;
    // 16 x 16 tiles up to K = 1024 (more, lighter workgroups for small grids), else 32 x 32
    P.TT = P.K > 1024 ? 32 : 16;
    P.nT = P.K / P.TT;   // >= 2, so K >= TT + KB_MAX_J - 1: a footprint never wraps onto its own tile
    // Degridding reads no neighbour's visibilities and adds nothing, so it takes larger tiles
    // where its LDS window fits: FP32 plans from K = 2048 degrid by 64 x 64 tiles, each the
    // union of 2 x 2 gridding tiles (smaller halo per visibility)
    P.TD = (P.precision == PURIFY_FP32 && P.K >= 2048) ? 2 * P.TT : P.TT;
    P.nTD = P.K / P.TD;
    const size_t es = P.precision == PURIFY_FP64 ? sizeof(double) : sizeof(float);
    const size_t ce = 2 * es;
    P.elem = ce;
    const size_t M = (size_t)P.M, N = (size_t)P.N, D = (size_t)P.D, K = (size_t)P.K;

    size_t off = 0;
    auto carve = [&](size_t bytes) -> void* {
        off = align256(off);
        void* p = ws ? (void*)(ws + off) : nullptr;
        off += bytes;
        return p;
    };
    P.base = (int32_t*)carve(M * 4);
    P.frac = carve(2 * M * es);
    P.perm = (int32_t*)carve(M * 4);
    P.tileoff = (int32_t*)carve(((size_t)4 * P.nT * P.nT + 1) * 4);
    P.tilecover = (int32_t*)carve((size_t)P.nT * P.nT * 4);
    // Gridding work units: a tile whose visibility list (own + spill-ins) exceeds
    // the unit U is split over several workgroups, each writing a private partial tile that a
    // second kernel sums.  A visibility is in at most four tiles' lists, so a split tile
    // (load > U) has parts = ceil(load / U) < 2 load / U, the parts of all split tiles number
    // below 8M / U and split tiles below 4M / U.
    // The unit grows with M / tiles so that the partial tiles never exceed four grids.
    {
        const size_t tiles = (size_t)P.nT * P.nT;
        P.grid_unit = (int)std::max<int64_t>(GRID_UNIT, (2 * (int64_t)M + (int64_t)tiles - 1) / (int64_t)tiles);
        const size_t parts_max = (size_t)(8 * M / P.grid_unit) + 1;
        const size_t split_max = std::min(tiles, (size_t)(4 * M / P.grid_unit) + 1);
        P.gslots = (int)parts_max;
        P.gmerge_cap = (int)split_max;
        P.gwork = (int32_t*)carve((tiles + parts_max) * GRID_REC * sizeof(int32_t));
        P.gmerge = (int32_t*)carve(split_max * 3 * sizeof(int32_t));
        const size_t ib = P.precision == PURIFY_FP64 ? 8 : 4;
        P.gscratch = carve(parts_max * 2 * (size_t)P.TT * P.TT * ib);
        P.gexp = (int32_t*)carve(parts_max * sizeof(int32_t));
        // degridding records: sum over tiles of ceil(load / dunit) <= tiles + M / dunit <= 1.5
        // tiles parts, room for strip padding up to twice the tiles
        const size_t dtiles = (size_t)P.nTD * P.nTD;
        P.dunit = (int)std::max<int64_t>(GRID_UNIT, (2 * (int64_t)M + (int64_t)dtiles - 1) / (int64_t)dtiles);
        P.dwork_cap = (int)(2 * dtiles + (size_t)(M / P.dunit) + 8);
        P.dwork = P.TD > P.TT ? (int32_t*)carve((size_t)P.dwork_cap * GRID_REC * sizeof(int32_t)) : nullptr;
        // degridding chunk table: at most twice the blocks of a plain launch plus one partial
        // chunk per strip and padding (larger strip-ordered tables fall back to plain blocks)
        P.dchunk_cap = (int)std::min<int64_t>((int64_t)2 * ((M + 255) / 256) + P.nT + 64, INT32_MAX / 2);
        P.dchunk = (int32_t*)carve((size_t)P.dchunk_cap * 2 * sizeof(int32_t));
    }
    P.deap = carve(P.n * es);
    P.tw = carve(P.n * ce);
    P.tw2 = carve(P.n * ce);
    P.filters = carve((size_t)MAX_WAV * 2 * MAX_TAPS * es);
    P.kbpoly = carve((size_t)KB_MAX_COEF * es);
    P.grid = carve(K * K * ce);
    P.grid2 = carve(K * K * ce);
    P.tmp = carve(K * P.n * ce);
    P.unit = carve(P.n * es);
    P.chat = carve(K * K * es);
    P.part = (double*)carve((size_t)NUM_PARTIAL_BUFS * MAX_PARTIALS * sizeof(double));
    P.sc = (double*)carve(SL_COUNT * sizeof(double));
    P.hist_cap = HIST_CAP;
    P.hist = (double*)carve((size_t)2 * HIST_CAP * sizeof(double));
    P.xh = carve(N * ce);
    P.x1 = carve(N * ce);
    P.x2 = carve(N * ce);
    P.x3 = carve(N * ce);
    P.r = carve(N * ce);
    P.p = carve(N * ce);
    P.qv = carve(N * ce);
    P.z2 = carve(N * ce);
    P.ytil = carve(M * ce);
    P.z3 = carve(M * ce);
    P.v3 = carve(M * ce);
    P.vis = carve(M * ce);
    P.tvp = carve(4 * N * ce);
    P.bid = (int32_t*)carve(M * 4);
    P.bperm = (int32_t*)carve(M * 4);
    P.bchunk = (int32_t*)carve((size_t)BLK_CHUNKS * 2 * 4);
    P.bchunk_off = (int32_t*)carve((size_t)(MAX_BLOCKS + 1) * 4);
    P.beps = (double*)carve((size_t)MAX_BLOCKS * sizeof(double));
    P.bscale = (double*)carve((size_t)MAX_BLOCKS * sizeof(double));
    P.z1 = carve(D * ce);
    P.v1 = carve(D * ce);
    // FP64: every visibility's 2J tap weights, computed once (degridding and gridding read
    // them instead of evaluating the polynomials).
    P.wtab = P.precision == PURIFY_FP64 ? carve(M * 2 * (size_t)P.J * sizeof(double)) : nullptr;
    const size_t nw = P.nwav > 0 ? (size_t)P.nwav : 1;
    P.wt = carve(nw * N * ce);
    P.ws2 = carve(nw * N * ce);
    return align256(off);
}

// ---------------------------------------------------------------------------------------
// The Kaiser-Bessel fit (with its verification against the Bessel series) and the Daubechies
// factorisations depend only on (J, beta, degree) and the filter order, and cost milliseconds
// in long double; they are computed once per process and shared by later plans (the server
// creates plans on several threads, hence the lock).
namespace {
struct KbFit {
    int J, deg;
    double beta, err;
    std::vector<long double> coef;
};
std::mutex g_table_mu;
std::vector<KbFit> g_kb_fits;
std::vector<std::vector<double>> g_daub(9);
}  // namespace

double kb_fit_cached(int J, double beta, int deg, long double* coef) {
    std::lock_guard<std::mutex> lk(g_table_mu);
    for (const KbFit& f : g_kb_fits)
        if (f.J == J && f.deg == deg && f.beta == beta) {
            std::copy(f.coef.begin(), f.coef.end(), coef);
            return f.err;
        }
    KbFit f{J, deg, beta, 0.0, std::vector<long double>((size_t)J * (deg + 1))};
    f.err = kb_fit(J, beta, deg, f.coef.data());
    std::copy(f.coef.begin(), f.coef.end(), coef);
    g_kb_fits.push_back(std::move(f));
    return g_kb_fits.back().err;
}

int daubechies(int N, double* h_out) {
    if (N < 1 || N > 8) return daubechies_compute(N, h_out);
    std::lock_guard<std::mutex> lk(g_table_mu);
    std::vector<double>& h = g_daub[(size_t)N];
    if (h.empty()) {
        double tmp[2 * 8];
        const int F = daubechies_compute(N, tmp);
        if (F < 0) return F;
        h.assign(tmp, tmp + F);
    }
    std::copy(h.begin(), h.end(), h_out);
    return (int)h.size();
}

// f(begin, end) over [0, n) split into contiguous ranges of at least `grain` items, on up to
// eight host threads (the calling thread takes the first range); serial where a thread
// cannot be started.  Each item must be independent of the others.
template <typename F>
void host_parallel(int64_t n, int64_t grain, F f) {
    const int64_t hw = std::max<int64_t>(1, (int64_t)std::thread::hardware_concurrency());
    const int64_t T = std::min<int64_t>(std::min<int64_t>(hw, 8), (n + grain - 1) / grain);
    if (T <= 1) {
        f((int64_t)0, n);
        return;
    }
    std::vector<std::thread> th;
    int64_t done = T;   // ranges [done, T) run on this thread if a thread cannot be started
    for (int64_t t = 1; t < T; ++t) {
        try {
            th.emplace_back(f, n * t / T, n * (t + 1) / T);
        } catch (...) {
            done = t;
            break;
        }
    }
    f((int64_t)0, n / T);
    for (int64_t t = done; t < T; ++t) f(n * t / T, n * (t + 1) / T);
    for (auto& x : th) x.join();
}

// ---------------------------------------------------------------------------------------
// Host-side plan tables and visibility binning; uploads into the workspace.
purify_status build_plan(Plan& P, const purify_plan_desc* d, hipStream_t s) {
    const int n = P.n, K = P.K, J = P.J, TT = P.TT, nT = P.nT;
    const int64_t M = P.M;
    const bool f64 = P.precision == PURIFY_FP64;

    // Kaiser-Bessel per-tap polynomials.
    const long double i0b = i0_series((long double)P.beta);
    P.kb_i0beta = (double)i0b;
    const int deg = f64 ? KBDeg<double>::value : KBDeg<float>::value;
    std::vector<long double> kbc((size_t)J * (deg + 1));
    P.kb_fit_err = kb_fit_cached(J, P.beta, deg, kbc.data());
    const double fit_tol = f64 ? 1e-13 : 1e-7;
    if (!(P.kb_fit_err <= fit_tol)) {
        set_error("Kaiser-Bessel polynomial fit error " + std::to_string(P.kb_fit_err) +
                  " exceeds tolerance for this J/beta");
        return PURIFY_E_INVALID;
    }
    std::vector<double> kbd(kbc.begin(), kbc.end());

    // Deapodisation and twiddles.
    std::vector<double> deap(n);
    for (int j = 0; j < n; ++j) deap[j] = 1.0 / kb_hat((double)(j - n / 2) / K, J, P.beta, i0b);
    std::vector<double> tw(2 * n), tw2(2 * n);
    for (int t = 0; t < n; ++t) {
        const long double a = 2.0L * PI_L * t / n;
        tw[2 * t] = (double)cosl(a);
        tw[2 * t + 1] = (double)-sinl(a);
        const long double b = PI_L * t / n;
        tw2[2 * t] = (double)cosl(b);
        tw2[2 * t + 1] = (double)-sinl(b);
    }
    // Filters: [basis][h(16) | g(16)], g[k] = (-1)^k h[F-1-k].
    std::vector<double> filt((size_t)MAX_WAV * 2 * MAX_TAPS, 0.0);
    for (int i = 0; i < P.nwav; ++i) {
        double h[MAX_TAPS] = {};
        const int F = daubechies(P.wav_N[i], h);
        for (int k = 0; k < F; ++k) {
            P.filt[i][k] = h[k];
            filt[(size_t)i * 2 * MAX_TAPS + k] = h[k];
            filt[(size_t)i * 2 * MAX_TAPS + MAX_TAPS + k] = ((k & 1) ? -1.0 : 1.0) * h[F - 1 - k];
        }
    }

    // Visibility binning: first tap, fractions and bucket key of each visibility (ranges of
    // visibilities on host threads), then a counting sort by key.
    std::vector<int32_t> base(M), key(M);
    std::vector<double> fr(2 * M);
    const double twopi = 2.0 * M_PI;
    const int nkeys = 4 * nT * nT;
    static const int rank_of_class[4] = {0, 1, 3, 2};
    std::atomic<bool> bad_uv{false};
    host_parallel(M, 16384, [&](int64_t m0, int64_t m1) {
        for (int64_t m = m0; m < m1; ++m) {
            int k0m[2];
            for (int ax = 0; ax < 2; ++ax) {
                double w = d->uv[2 * m + ax];
                if (!std::isfinite(w)) {
                    bad_uv.store(true, std::memory_order_relaxed);
                    w = 0.0;
                }
                if (w < -M_PI || w >= M_PI) {
                    w = std::fmod(w + M_PI, twopi);
                    if (w < 0) w += twopi;
                    w -= M_PI;
                    if (w >= M_PI) w -= twopi;
                }
                const double kap = (w * K) / (2.0 * M_PI);
                const double k0 = std::floor(kap - 0.5 * J) + 1.0;
                fr[2 * m + ax] = kap - k0 - (0.5 * J - 1.0);
                int km = (int)((int64_t)k0 % K);
                if (km < 0) km += K;
                k0m[ax] = km;
            }
            base[m] = k0m[0] | (k0m[1] << 16);
            const int t1 = k0m[0] / TT, t2 = k0m[1] / TT;
            const int s1 = (k0m[0] % TT) + J - 1 >= TT, s2 = (k0m[1] % TT) + J - 1 >= TT;
            key[m] = (t2 * nT + t1) * 4 + rank_of_class[s1 + 2 * s2];
        }
    });
    if (bad_uv.load()) {
        set_error("non-finite uv coordinate");
        return PURIFY_E_INVALID;
    }
    std::vector<int64_t> cnt(nkeys + 1, 0);
    for (int64_t m = 0; m < M; ++m) ++cnt[key[m] + 1];
    for (int k = 0; k < nkeys; ++k) cnt[k + 1] += cnt[k];
    std::vector<int32_t> off(nkeys + 1);
    for (int k = 0; k <= nkeys; ++k) off[k] = (int32_t)cnt[k];
    // Order: by (tile, spill class), then by first-tap cell inside each bucket (row-major),
    // ties in caller order.  Neighbouring visibilities then share grid cache lines.  A
    // bucket arrives in caller order, so sorting by (cell, index) is the stable order; the
    // buckets are sorted on host threads.
    std::vector<int32_t> order(M);
    {
        std::vector<int64_t> pos(cnt.begin(), cnt.end() - 1);
        for (int64_t m = 0; m < M; ++m) order[pos[key[m]]++] = (int32_t)m;
        host_parallel(nkeys, M < 65536 ? nkeys : 64, [&](int64_t k0, int64_t k1) {
            for (int64_t k = k0; k < k1; ++k) {
                auto b0 = order.begin() + off[k], b1 = order.begin() + off[k + 1];
                if (b1 - b0 > 1)
                    std::sort(b0, b1, [&](int32_t a, int32_t b) {
                        const int ca = ((base[a] & 0xFFFF) << 16) | ((base[a] >> 16) & 0xFFFF);
                        const int cb = ((base[b] & 0xFFFF) << 16) | ((base[b] >> 16) & 0xFFFF);
                        return ca < cb || (ca == cb && a < b);
                    });
            }
        });
    }
    std::vector<int32_t> perm(M), sbase(M);
    std::vector<double> sfr(2 * M);
    host_parallel(M, 65536, [&](int64_t p0, int64_t p1) {
        for (int64_t p = p0; p < p1; ++p) {
            const int32_t m = order[p];
            perm[p] = m;
            sbase[p] = base[m];
            sfr[2 * p] = fr[2 * m];
            sfr[2 * p + 1] = fr[2 * m + 1];
        }
    });

    // Heaviest gridding workgroup: own visibilities plus the spill-ins from three neighbours.
    P.max_tile_load = 0;
    for (int t2 = 0; t2 < nT; ++t2)
        for (int t1 = 0; t1 < nT; ++t1) {
            const int t = t2 * nT + t1;
            const int L = t2 * nT + (t1 + nT - 1) % nT, U = ((t2 + nT - 1) % nT) * nT + t1;
            const int Dg = ((t2 + nT - 1) % nT) * nT + (t1 + nT - 1) % nT;
            const int load = (off[4 * t + 4] - off[4 * t]) + (off[4 * L + 3] - off[4 * L + 1]) +
                             (off[4 * U + 4] - off[4 * U + 2]) + (off[4 * Dg + 3] - off[4 * Dg + 2]);
            P.max_tile_load = std::max(P.max_tile_load, load);
        }
    P.grid_threads = 256;
    // Per-tile bound on the number of visibilities that add to one cell (gridding scale):
    // count first taps per cell, sum over the J x J window of first taps that reach each
    // cell (cyclic), and take the maximum over each tile.  The window sums slide along both
    // axes (integer sums: the same values as summing each window), with the axis-1 sums of
    // the J rows in the current axis-2 window held in a ring.
    std::vector<int32_t> cover((size_t)nT * nT, 0);
    {
        std::vector<int32_t> cnt((size_t)K * K, 0);
        for (int64_t m = 0; m < M; ++m) {
            const int k1 = base[m] & 0xFFFF, k2 = (base[m] >> 16) & 0xFFFF;
            ++cnt[(size_t)k2 * K + k1];
        }
        // r[k1] = sum_{a < J} cnt[k2][(k1 - a) mod K]
        auto row_sums = [&](int k2, int32_t* r) {
            const int32_t* c = &cnt[(size_t)k2 * K];
            int32_t acc = 0;
            for (int a = 0; a < J; ++a) acc += c[(K - a) & (K - 1)];
            r[0] = acc;
            for (int k1 = 1; k1 < K; ++k1) {
                acc += c[k1] - c[(k1 - J + K) & (K - 1)];
                r[k1] = acc;
            }
        };
        // ring slot (k2 + J) mod J holds row k2's sums; S[k1] = sum_{b < J} r[(k2 - b) mod K][k1]
        std::vector<int32_t> ring((size_t)J * K), S((size_t)K, 0);
        for (int b = J - 1; b >= 0; --b) {
            int32_t* r = &ring[(size_t)((J - b) % J) * K];
            row_sums((K - b) & (K - 1), r);
            for (int k1 = 0; k1 < K; ++k1) S[k1] += r[k1];
        }
        for (int k2 = 0; k2 < K; ++k2) {
            if (k2 > 0) {
                int32_t* r = &ring[(size_t)(k2 % J) * K];   // row k2 - J, leaving the window
                for (int k1 = 0; k1 < K; ++k1) S[k1] -= r[k1];
                row_sums(k2, r);
                for (int k1 = 0; k1 < K; ++k1) S[k1] += r[k1];
            }
            int32_t* cv = &cover[(size_t)(k2 / TT) * nT];
            for (int t1 = 0; t1 < nT; ++t1) {
                int32_t mx = cv[t1];
                for (int k1 = t1 * TT; k1 < (t1 + 1) * TT; ++k1) mx = std::max(mx, S[k1]);
                cv[t1] = mx;
            }
        }
    }

    // Work list: heavy tiles first (their parts start earliest), then the rest.  One record
    // of GRID_REC ints per work unit: {tile, partial slot or -1, cover, visibility passes,
    // then [start, end) of its share of the tile's five visibility ranges: own interior, own
    // spilling, and the left, upper and diagonal neighbours' spill-ins}.  Merge list: one
    // entry {tile, parts, first partial slot} per split tile.
    std::vector<int32_t> work, merge;
    {
        std::vector<std::pair<int, int>> load_tile;   // (load, tile)
        auto ranges = [&](int t, int* s, int* e) {
            const int t1 = t % nT, t2 = t / nT;
            const int L = t2 * nT + (t1 + nT - 1) % nT, U = ((t2 + nT - 1) % nT) * nT + t1;
            const int Dg = ((t2 + nT - 1) % nT) * nT + (t1 + nT - 1) % nT;
            s[0] = off[4 * t];      e[0] = off[4 * t + 1];
            s[1] = off[4 * t + 1];  e[1] = off[4 * t + 4];
            s[2] = off[4 * L + 1];  e[2] = off[4 * L + 3];
            s[3] = off[4 * U + 2];  e[3] = off[4 * U + 4];
            s[4] = off[4 * Dg + 2]; e[4] = off[4 * Dg + 3];
        };
        for (int t = 0; t < nT * nT; ++t) {
            int s[5], e[5], load = 0;
            ranges(t, s, e);
            for (int r = 0; r < 5; ++r) load += e[r] - s[r];
            load_tile.push_back({load, t});
        }
        std::stable_sort(load_tile.begin(), load_tile.end(),
                         [](const std::pair<int, int>& a, const std::pair<int, int>& b) { return a.first > b.first; });
        int slot = 0;
        for (const auto& lt : load_tile) {
            const int t = lt.second;
            const int parts = std::max(1, (lt.first + P.grid_unit - 1) / P.grid_unit);
            int s[5], e[5];
            ranges(t, s, e);
            for (int q = 0; q < parts; ++q) {
                int32_t rec[GRID_REC] = {};
                rec[0] = t;
                rec[1] = parts > 1 ? slot + q : -1;
                rec[2] = cover[t];
                int total = 0;
                for (int r = 0; r < 5; ++r) {
                    // part q of parts takes [s + len q / parts, s + len (q + 1) / parts)
                    const int64_t len = e[r] - s[r];
                    rec[4 + 2 * r] = s[r] + (int)(len * q / parts);
                    rec[5 + 2 * r] = s[r] + (int)(len * (q + 1) / parts);
                    total += rec[5 + 2 * r] - rec[4 + 2 * r];
                }
                rec[3] = total;
                work.insert(work.end(), rec, rec + GRID_REC);
            }
            if (parts > 1) {
                merge.push_back(t);
                merge.push_back(parts);
                merge.push_back(slot);
                slot += parts;
            }
        }
        const size_t work_cap = (size_t)nT * nT + (size_t)P.gslots;
        if (slot > P.gslots || (int)(merge.size() / 3) > P.gmerge_cap || work.size() / GRID_REC > work_cap) {
            set_error("internal: gridding work list exceeds its bound");
            return PURIFY_E_INVALID;
        }
        // Strip order: workgroups are dispatched round-robin over the 8 XCDs, so unit w runs on
        // XCD w % 8.  Give unit w a tile of a strip t2 = w (mod 8) (each XCD's units keep the
        // heaviest-first order, empty units pad the shorter lists), matching the column FFT
        // passes' strip_block mapping: the grid columns a tile reads and writes stay in one
        // XCD's L2.  Kept only if the padding fits the work list's capacity.
        P.strip_xcd = false;
        if (nT % 8 == 0) {
            std::vector<std::vector<int32_t>> q(8);
            for (size_t u = 0; u < work.size() / GRID_REC; ++u) {
                const int32_t* rec = &work[u * GRID_REC];
                const int e = (rec[0] / nT) % 8;
                q[e].insert(q[e].end(), rec, rec + GRID_REC);
            }
            size_t longest = 0;
            for (const auto& v : q) longest = std::max(longest, v.size() / GRID_REC);
            if (8 * longest <= work_cap) {
                std::vector<int32_t> ord;
                ord.reserve(8 * longest * GRID_REC);
                for (size_t k = 0; k < longest; ++k)
                    for (int e = 0; e < 8; ++e) {
                        if (k < q[e].size() / GRID_REC) {
                            ord.insert(ord.end(), q[e].begin() + k * GRID_REC, q[e].begin() + (k + 1) * GRID_REC);
                        } else {
                            int32_t empty[GRID_REC] = {};
                            empty[0] = -1;   // no tile: the workgroup exits at once
                            ord.insert(ord.end(), empty, empty + GRID_REC);
                        }
                    }
                work.swap(ord);
                P.strip_xcd = true;
            }
        }
        P.nwork = (int)(work.size() / GRID_REC);
        P.nmerge = (int)(merge.size() / 3);
    }
    // Degridding tiles of side TD = 2 TT: tile (d1, d2) is gridding tiles (2 d1 + i, 2 d2 + j),
    // i, j in {0, 1}; the two with j = 0 are adjacent in the sorted order (keys ascend with
    // t = t2 nT + t1), and so are the two with j = 1, so its visibilities are two contiguous
    // ranges.  A tile with more than dunit visibilities is split into parts (each part a
    // slice of the two ranges); heavy tiles come first, then the list is strip-ordered like
    // the gridding work list (record w holds a tile of strip d2 = w (mod 8)) when the padding
    // fits.
    std::vector<int32_t> dwork;
    if (P.TD > TT) {
        const int nTD = P.nTD;
        std::vector<std::pair<int, int>> load_tile;   // (load, tile)
        auto dranges = [&](int t, int* s, int* e) {
            const int d1 = t % nTD, d2 = t / nTD;
            for (int j = 0; j < 2; ++j) {
                const int g = (2 * d2 + j) * nT + 2 * d1;
                s[j] = off[4 * g];
                e[j] = off[4 * (g + 2)];
            }
        };
        for (int t = 0; t < nTD * nTD; ++t) {
            int s[2], e[2];
            dranges(t, s, e);
            load_tile.push_back({(e[0] - s[0]) + (e[1] - s[1]), t});
        }
        std::stable_sort(load_tile.begin(), load_tile.end(),
                         [](const std::pair<int, int>& a, const std::pair<int, int>& b) { return a.first > b.first; });
        std::vector<int32_t> list;
        for (const auto& lt : load_tile) {
            const int t = lt.second, L = lt.first;
            const int parts = std::max(1, (L + P.dunit - 1) / P.dunit);
            int s[2], e[2];
            dranges(t, s, e);
            const int n0 = e[0] - s[0];
            for (int q = 0; q < parts; ++q) {
                // slice [a, b) of the two ranges laid end to end
                const int a = (int)((int64_t)L * q / parts), b = (int)((int64_t)L * (q + 1) / parts);
                int32_t rec[GRID_REC] = {};
                rec[0] = t;
                rec[4] = s[0] + std::min(a, n0);
                rec[5] = s[0] + std::min(b, n0);
                rec[6] = s[1] + std::max(a, n0) - n0;
                rec[7] = s[1] + std::max(b, n0) - n0;
                list.insert(list.end(), rec, rec + GRID_REC);
            }
        }
        const size_t nrec = list.size() / GRID_REC;
        if (nrec > (size_t)P.dwork_cap) {
            set_error("internal: degridding work list exceeds its bound");
            return PURIFY_E_INVALID;
        }
        dwork.swap(list);
        if (nTD % 8 == 0) {
            std::vector<std::vector<int32_t>> q(8);
            for (size_t u = 0; u < nrec; ++u) {
                const int32_t* rec = &dwork[u * GRID_REC];
                const int e = (rec[0] / nTD) % 8;
                q[e].insert(q[e].end(), rec, rec + GRID_REC);
            }
            size_t longest = 0;
            for (const auto& v : q) longest = std::max(longest, v.size() / GRID_REC);
            if (8 * longest <= (size_t)P.dwork_cap) {
                std::vector<int32_t> ord;
                ord.reserve(8 * longest * GRID_REC);
                for (size_t k = 0; k < longest; ++k)
                    for (int e = 0; e < 8; ++e) {
                        if (k < q[e].size() / GRID_REC) {
                            ord.insert(ord.end(), q[e].begin() + k * GRID_REC, q[e].begin() + (k + 1) * GRID_REC);
                        } else {
                            int32_t empty[GRID_REC] = {};
                            empty[0] = -1;   // no tile: the workgroup exits at once
                            ord.insert(ord.end(), empty, empty + GRID_REC);
                        }
                    }
                dwork.swap(ord);
            }
        }
        P.ndwork = (int)(dwork.size() / GRID_REC);
    }
    // G by tiles (k_degrid_tiles) when the tiles' grid windows, (TD + J - 1)^2 cells each,
    // add up to at most half the J^2 taps the visibilities gather (dense coverage); sparse
    // coverage keeps one thread per visibility gathering straight from the grid.
    {
        const std::vector<int32_t>& dl = P.TD > TT ? dwork : work;
        int64_t busy = 0;
        for (size_t u = 0; u < dl.size() / GRID_REC; ++u) {
            const int32_t* rec = &dl[u * GRID_REC];
            if (rec[0] >= 0 && (rec[5] - rec[4]) + (rec[7] - rec[6]) > 0) ++busy;
        }
        const int64_t ws = P.TD + J - 1;
        P.degrid_tiles = busy * ws * ws * 2 <= (int64_t)M * J * J;
    }
    // Degridding in the same strip order: workgroup b (XCD b % 8) takes up to 256 visibilities
    // of a strip t2 = b (mod 8), so it reads the grid columns the column FFT pass left in its
    // XCD's L2.  Strip t2 holds the visibilities of tiles t2 * nT .. t2 * nT + nT - 1.
    std::vector<int32_t> dch;
    P.ndchunk = 0;
    if (nT % 8 == 0) {
        std::vector<std::vector<int32_t>> q(8);
        for (int s2 = 0; s2 < nT; ++s2) {
            const int a0 = off[4 * (s2 * nT)], a1 = off[4 * ((s2 + 1) * nT)];
            for (int a = a0; a < a1; a += 256) {
                q[s2 % 8].push_back(a);
                q[s2 % 8].push_back(std::min(256, a1 - a));
            }
        }
        size_t longest = 0;
        for (const auto& v : q) longest = std::max(longest, v.size() / 2);
        if (8 * longest <= (size_t)P.dchunk_cap) {
            for (size_t k = 0; k < longest; ++k)
                for (int e = 0; e < 8; ++e) {
                    if (k < q[e].size() / 2) {
                        dch.push_back(q[e][2 * k]);
                        dch.push_back(q[e][2 * k + 1]);
                    } else {
                        dch.push_back(0);
                        dch.push_back(0);
                    }
                }
            P.ndchunk = (int)(dch.size() / 2);
        }
    }

    // FP64 tap weights in sorted order: w[p][a] = psi(f1 + J/2 - 1 - a), w[p][J + a] likewise
    // for axis 2, from the same per-tap polynomials the FP32 kernels evaluate.
    std::vector<double> wt;
    if (f64) {
        wt.resize((size_t)M * 2 * J);
        const int nc = deg + 1;
        // Horner per weight; the 2J weights of a visibility advance together (independent
        // chains), each with the same operations in the same order as one at a time; ranges
        // of visibilities on several host threads
        host_parallel(M, 4096, [&](int64_t q0, int64_t q1) {
            for (int64_t q = q0; q < q1; ++q) {
                double acc[2 * KB_MAX_J];
                const double x0 = sfr[2 * q] - 0.5, x1 = sfr[2 * q + 1] - 0.5;
                for (int a = 0; a < J; ++a) acc[a] = acc[J + a] = kbd[(size_t)a * nc + nc - 1];
                for (int k = nc - 2; k >= 0; --k)
                    for (int a = 0; a < J; ++a) {
                        const double c = kbd[(size_t)a * nc + k];
                        acc[a] = acc[a] * x0 + c;
                        acc[J + a] = acc[J + a] * x1 + c;
                    }
                std::copy(acc, acc + 2 * J, wt.begin() + (ptrdiff_t)((size_t)q * 2 * J));
            }
        });
    }

    // Upload (pageable host memory; synchronous at the end).
    auto up = [&](void* dst, const void* src, size_t bytes) -> hipError_t {
        return hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s);
    };
    std::vector<float> f32buf;
    auto up_real = [&](void* dst, const std::vector<double>& v) -> hipError_t {
        if (f64) return up(dst, v.data(), v.size() * sizeof(double));
        f32buf.assign(v.begin(), v.end());
        hipError_t e = up(dst, f32buf.data(), f32buf.size() * sizeof(float));
        if (e != hipSuccess) return e;
        return hipStreamSynchronize(s);   // f32buf is reused
    };
    PURIFY_HIP(up(P.base, sbase.data(), M * 4));
    PURIFY_HIP(up(P.perm, perm.data(), M * 4));
    PURIFY_HIP(up(P.tileoff, off.data(), off.size() * 4));
    PURIFY_HIP(up(P.tilecover, cover.data(), cover.size() * 4));
    PURIFY_HIP(up(P.gwork, work.data(), work.size() * sizeof(int32_t)));
    if (!dwork.empty()) PURIFY_HIP(up(P.dwork, dwork.data(), dwork.size() * sizeof(int32_t)));
    if (!dch.empty()) PURIFY_HIP(up(P.dchunk, dch.data(), dch.size() * sizeof(int32_t)));
    if (!merge.empty()) PURIFY_HIP(up(P.gmerge, merge.data(), merge.size() * sizeof(int32_t)));
    PURIFY_HIP(up_real(P.frac, sfr));
    PURIFY_HIP(up_real(P.deap, deap));
    const std::vector<double> ones((size_t)n, 1.0);   // lives until the final synchronisation
    PURIFY_HIP(up_real(P.unit, ones));
    PURIFY_HIP(up_real(P.tw, tw));
    PURIFY_HIP(up_real(P.tw2, tw2));
    PURIFY_HIP(up_real(P.filters, filt));
    PURIFY_HIP(up_real(P.kbpoly, kbd));
    if (f64) PURIFY_HIP(up(P.wtab, wt.data(), wt.size() * sizeof(double)));
    PURIFY_HIP(hipMemsetAsync(P.sc, 0, SL_COUNT * sizeof(double), s));
    PURIFY_HIP(hipStreamSynchronize(s));
    return PURIFY_OK;
}

}  // namespace purify
