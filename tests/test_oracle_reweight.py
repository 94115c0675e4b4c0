"""Pins of the reweighted-l1 oracle (SARA reweighting, Section 2.2) against properties that do
not come from the oracle itself: the weights as slopes of the log-sum penalty (finite
differences and the tangent-line majorant), the descent of that penalty over reweights (the
majorise-minimise property), the reduction to the unweighted warm-started solve when delta
is huge, and the chi-square noise floor."""
import math

import numpy as np

from oracle.nufft import Nufft
from oracle.reweight import noise_floor, relative_variation, reweight, reweighted_sdmm
from oracle.sara import Sara
from oracle.sdmm import sdmm
from paper_1406_0359_amd import synth


def _tiny_problem(n=8, M=48, mask=0x3, L=2, seed=21, isnr=30.0):
    rng = np.random.default_rng(seed)
    uv = synth.uv_coverage(M, 2 * n, rng)
    op = Nufft(n, uv, 6)
    x = synth.blob_image(n, 3, rng)
    y0 = op.phi(x)
    sigma = np.linalg.norm(y0) / math.sqrt(M) * 10 ** (-isnr / 20)
    y = y0 + sigma * synth.unit_complex_noise(M, rng)
    return op, Sara(n, mask, L), x, y, synth.chi2_epsilon(sigma, M), sigma


def test_weights_are_delta_times_log_penalty_slope():
    rng = np.random.default_rng(3)
    alpha = rng.standard_normal(200) * np.exp(rng.uniform(-6, 3, 200)) + 1j * rng.standard_normal(200)
    for delta in (1e-3, 0.37, 25.0):
        w = reweight(alpha, delta)
        s0 = np.abs(alpha)
        h = 1e-6 * (delta + s0)
        slope = (np.log(delta + s0 + h) - np.log(delta + s0 - h)) / (2 * h)
        assert np.max(np.abs(w - delta * slope)) < 1e-8
        # tangent line of the concave log(delta + s) lies above it everywhere
        s = np.abs(rng.standard_normal(200)) * 10
        assert np.all(np.log(delta + s) <= np.log(delta + s0) + (w / delta) * (s - s0) + 1e-12)
    assert np.array_equal(reweight(np.zeros(4), 0.0), np.ones(4))


def test_noise_floor_is_sigma_over_nu():
    for sigma, M, nu in ((1.7, 400, 3.0), (0.02, 19661, 251.5)):
        assert abs(noise_floor(synth.chi2_epsilon(sigma, M), M, nu) - sigma / nu) < 1e-15 * sigma / nu


def test_relative_variation_edge_cases():
    a = np.array([3.0, 4.0])
    assert relative_variation(a, a) == 0.0
    assert relative_variation(np.zeros(2), np.zeros(2)) == 0.0
    assert relative_variation(a, np.zeros(2)) == math.inf
    assert relative_variation(2 * a, a) == 1.0


def test_huge_delta_reduces_to_unweighted_warm_start():
    op, sa, x, y, eps, _ = _tiny_problem()
    kw = dict(iters=60, cg_iters=10)
    r = reweighted_sdmm(op.phi, op.phi_adj, sa.psi, sa.psi_adj, y, eps, (8, 8), reweights=1,
                        delta0=1e300, decay=1.0, rel_var=0.0, **kw)
    r0 = sdmm(op.phi, op.phi_adj, sa.psi, sa.psi_adj, y, eps, (8, 8), **kw)
    r1 = sdmm(op.phi, op.phi_adj, sa.psi, sa.psi_adj, y, eps, (8, 8), x0=r0.x, nu=r0.nu,
              gamma=r0.gamma, **kw)
    assert np.all(r.weights == 1.0)
    assert np.array_equal(r.solves[0].x, r0.x)
    assert np.array_equal(r.x, r1.x)
    assert r.solves[1].objective == r1.objective


def test_warm_start_from_zero_equals_cold_start():
    op, sa, x, y, eps, _ = _tiny_problem(seed=7)
    a = sdmm(op.phi, op.phi_adj, sa.psi, sa.psi_adj, y, eps, (8, 8), iters=30)
    b = sdmm(op.phi, op.phi_adj, sa.psi, sa.psi_adj, y, eps, (8, 8), iters=30, x0=np.zeros((8, 8)))
    assert np.array_equal(a.x, b.x)


def test_log_sum_penalty_descends_over_reweights():
    # majorise-minimise: with delta fixed, solving each weighted problem exactly cannot raise
    # sum_j log(delta + |(Psi^dag x)_j|) over the feasible set; SDMM run long is close to exact
    op, sa, x, y, eps, _ = _tiny_problem(n=8, M=40, mask=0x3, L=1, seed=12)
    delta = 0.05 * float(np.max(np.abs(sa.psi_adj(x))))
    r = reweighted_sdmm(op.phi, op.phi_adj, sa.psi, sa.psi_adj, y, eps, (8, 8), reweights=3,
                        delta0=delta, decay=1.0, rel_var=0.0, iters=3000, gamma=0.05)
    g = [float(np.sum(np.log(delta + np.abs(sa.psi_adj(np.real(s.x)))))) for s in r.solves]
    for k in range(1, len(g)):
        assert g[k] <= g[k - 1] + 1e-6 * abs(g[k - 1])
    for s in r.solves:
        assert np.linalg.norm(y - op.phi(np.real(s.x))) <= eps * (1 + 1e-3)


def test_stops_when_relative_variation_is_small():
    op, sa, x, y, eps, sigma = _tiny_problem(seed=5)
    r = reweighted_sdmm(op.phi, op.phi_adj, sa.psi, sa.psi_adj, y, eps, (8, 8), reweights=4,
                        rel_var=1e9, iters=40)
    assert len(r.solves) == 2 and len(r.rel_vars) == 1
    full = reweighted_sdmm(op.phi, op.phi_adj, sa.psi, sa.psi_adj, y, eps, (8, 8), reweights=3,
                           rel_var=0.0, iters=40, decay=0.5)
    assert len(full.solves) == 4
    # delta halves each time down to the noise floor sigma / nu
    floor = noise_floor(eps, y.size, full.solves[0].nu)
    d0 = max(float(np.std(sa.psi_adj(full.solves[0].x))), floor)
    assert full.deltas == [d0, max(0.5 * d0, floor), max(0.25 * d0, floor)]


def test_reweighted_tv_huge_delta_reduces_to_warm_tv_solve():
    op, sa, x, y, eps, _ = _tiny_problem(seed=9)
    kw = dict(iters=30, tv_iters=20)
    r = reweighted_sdmm(op.phi, op.phi_adj, None, None, y, eps, (8, 8), reweights=1, delta0=1e300,
                        decay=1.0, rel_var=0.0, **kw)
    r0 = sdmm(op.phi, op.phi_adj, None, None, y, eps, (8, 8), **kw)
    r1 = sdmm(op.phi, op.phi_adj, None, None, y, eps, (8, 8), x0=r0.x, nu=r0.nu, gamma=r0.gamma,
              weights=np.ones((8, 8)), **kw)
    assert np.all(r.weights == 1.0) and r.weights.shape == (8, 8)
    assert np.array_equal(r.x, r1.x)
