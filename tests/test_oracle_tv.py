"""Pins of the total-variation oracle (the TV prior of Section 5): the divergence as the
negative adjoint of the gradient, the gradient's norm bound behind the step tau = 1/8, the
Chambolle prox against a brute-force convex minimisation (plain and weighted), dual
feasibility, and SDMM with the TV prior against feasibility at convergence and a brute-force
constrained minimisation."""
import math

import numpy as np
import pytest
from scipy import optimize

from oracle.nufft import Nufft
from oracle.sdmm import sdmm
from oracle.tv import div, grad, prox_tv, tv_norm
from paper_1406_0359_amd import synth


def _c(shape, seed):
    r = np.random.default_rng(seed)
    return r.standard_normal(shape) + 1j * r.standard_normal(shape)


def test_divergence_is_minus_gradient_adjoint():
    for n in (2, 3, 7, 16):
        x, p1, p2 = _c((n, n), 1), _c((n, n), 2), _c((n, n), 3)
        g1, g2 = grad(x)
        lhs = np.vdot(g1, p1) + np.vdot(g2, p2)
        rhs = -np.vdot(x, div(p1, p2))
        assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_gradient_norm_bound():
    n = 64
    v = _c((n, n), 4)
    for _ in range(3000):
        v = -div(*grad(v))
        lam = np.linalg.norm(v)
        v /= lam
    assert 7.9 < lam < 8.0


def _dual_value(u, gamma, w):
    """Brute-force dual of min_x |x - u|^2 / 2 + gamma sum w |grad x|: maximise
    |u|^2 / 2 - |u - gamma div p|^2 / 2 over |p_ij| <= w_ij (a smooth problem with convex
    quadratic constraints, solved by SLSQP); by duality its value is the prox's optimum."""
    n = u.shape[0]
    N = n * n

    def obj(z):
        d = u - gamma * div(z[:N].reshape(n, n), z[N:].reshape(n, n)).real
        return 0.5 * np.sum(d * d)

    cons = dict(type="ineq", fun=lambda z: (w ** 2).ravel() - z[:N] ** 2 - z[N:] ** 2)
    sol = optimize.minimize(obj, np.zeros(2 * N), method="SLSQP", constraints=[cons],
                            options=dict(maxiter=5000, ftol=1e-16))
    return 0.5 * np.sum(u * u) - sol.fun


@pytest.mark.parametrize("weighted", [False, True])
def test_prox_tv_matches_brute_force(weighted):
    rng = np.random.default_rng(5)
    n, gamma = 4, 0.3
    u = rng.standard_normal((n, n))
    w = rng.uniform(0.3, 1.5, (n, n)) if weighted else np.ones((n, n))
    x = prox_tv(u, gamma, 20000, w if weighted else None)
    f = 0.5 * np.sum(np.abs(x - u) ** 2) + gamma * tv_norm(x, w)
    d = _dual_value(u, gamma, w)
    # weak duality f >= d always; the gap certifies that x is the minimiser
    assert -1e-9 * f <= f - d <= 1e-7 * f
    assert np.max(np.abs(x.imag)) < 1e-14


def test_dual_field_stays_feasible_and_constants_are_fixed():
    u = _c((12, 12), 6)
    w = np.random.default_rng(7).uniform(0.2, 2.0, (12, 12))
    for it in (1, 5, 40):
        _, (p1, p2) = prox_tv(u, 0.5, it, w, return_dual=True)
        assert np.all(np.sqrt(np.abs(p1) ** 2 + np.abs(p2) ** 2) <= w * (1 + 1e-12))
    c = np.full((9, 9), 2.5 - 1.0j)
    assert np.allclose(prox_tv(c, 3.0, 50), c, atol=1e-14)


def _tiny(n=8, M=48, seed=21, isnr=30.0):
    rng = np.random.default_rng(seed)
    uv = synth.uv_coverage(M, 2 * n, rng)
    op = Nufft(n, uv, 6)
    x = synth.blob_image(n, 3, rng)
    y0 = op.phi(x)
    sigma = np.linalg.norm(y0) / math.sqrt(M) * 10 ** (-isnr / 20)
    y = y0 + sigma * synth.unit_complex_noise(M, rng)
    return op, x, y, synth.chi2_epsilon(sigma, M)


def test_tv_sdmm_constraints_at_convergence():
    op, x, y, eps = _tiny(n=16, M=160, seed=4)
    r = sdmm(op.phi, op.phi_adj, None, None, y, eps, (16, 16), iters=2000, tv_iters=50)
    xr = np.real(r.x)
    assert np.linalg.norm(y - op.phi(xr)) <= eps * (1 + 1e-3)
    assert xr.min() >= -1e-6 * xr.max()


@pytest.mark.slow
def test_tv_sdmm_matches_slsqp_brute_force():
    n = 4
    op, x, y, eps = _tiny(n=n, M=10, seed=8)
    N = n * n
    Phi = np.stack([op.phi(np.eye(N)[k].reshape(n, n)) for k in range(N)], axis=1)
    r = sdmm(op.phi, op.phi_adj, None, None, y, eps, (n, n), iters=4000, gamma=0.05, tv_iters=300)
    f_sdmm = tv_norm(np.real(r.x))

    def unpack(z):
        return z[:N].reshape(n, n), z[N:].reshape(n, n)

    def cone(z):
        xx, t = unpack(z)
        g1, g2 = grad(xx)
        return (t ** 2 - np.abs(g1) ** 2 - np.abs(g2) ** 2).ravel()
    cons = [dict(type="ineq", fun=cone),
            dict(type="ineq", fun=lambda z: eps ** 2 - np.sum(np.abs(y - Phi @ z[:N]) ** 2))]
    z0 = np.concatenate([np.real(r.x).ravel(), np.ones(N)])
    sol = optimize.minimize(lambda z: z[N:].sum(), z0, method="SLSQP", constraints=cons,
                            bounds=[(0, None)] * N + [(0, None)] * N,
                            options=dict(maxiter=3000, ftol=1e-15))
    assert np.linalg.norm(y - Phi @ np.real(r.x).ravel()) <= eps * (1 + 1e-3)
    assert abs(f_sdmm - sol.fun) <= 1e-5 * sol.fun
