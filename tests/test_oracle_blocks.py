"""Pins of the visibility-block form of the oracle (eqs. (4)-(5): R data blocks, S = R + 2):
the product-of-balls projection against the projection inequality, a single block against the
plain solve, every block's constraint at convergence, and a brute-force constrained
minimisation with two blocks."""
import math

import numpy as np
import pytest
from scipy import optimize

from oracle.nufft import Nufft
from oracle.prox import project_l2_ball, project_l2_balls
from oracle.sara import Sara
from oracle.sdmm import sdmm
from paper_1406_0359_amd import synth


def test_product_projection_inequality_and_single_block():
    rng = np.random.default_rng(1)
    M, offs, eps = 90, [0, 20, 55, 90], [0.7, 2.0, 0.1]
    y = rng.standard_normal(M) + 1j * rng.standard_normal(M)
    for _ in range(10):
        u = y + 2 * (rng.standard_normal(M) + 1j * rng.standard_normal(M))
        p = project_l2_balls(u, y, offs, eps)
        for i in range(3):
            assert np.linalg.norm(p[offs[i]:offs[i + 1]] - y[offs[i]:offs[i + 1]]) <= eps[i] * (1 + 1e-12)
        assert np.allclose(project_l2_balls(p, y, offs, eps), p)
        for _ in range(20):   # <u - P u, v - P u> <= 0 for every v in the product set
            v = y.copy()
            for i in range(3):
                d = rng.standard_normal(offs[i + 1] - offs[i]) + 1j * rng.standard_normal(offs[i + 1] - offs[i])
                v[offs[i]:offs[i + 1]] += d / np.linalg.norm(d) * eps[i] * rng.uniform(0, 1)
            assert np.vdot(u - p, v - p).real <= 1e-10
    u = y + rng.standard_normal(M)
    assert np.array_equal(project_l2_balls(u, y, [0, M], [1.3]), project_l2_ball(u, y, 1.3))


def _tiny(n=8, M=48, mask=0x3, L=2, seed=21, isnr=30.0):
    rng = np.random.default_rng(seed)
    uv = synth.uv_coverage(M, 2 * n, rng)
    op = Nufft(n, uv, 6)
    x = synth.blob_image(n, 3, rng)
    y0 = op.phi(x)
    sigma = np.linalg.norm(y0) / math.sqrt(M) * 10 ** (-isnr / 20)
    y = y0 + sigma * synth.unit_complex_noise(M, rng)
    return op, Sara(n, mask, L), x, y, sigma


def test_single_block_equals_plain_solve():
    op, sa, x, y, sigma = _tiny()
    eps = synth.chi2_epsilon(sigma, y.size)
    a = sdmm(op.phi, op.phi_adj, sa.psi, sa.psi_adj, y, eps, (8, 8), iters=40)
    b = sdmm(op.phi, op.phi_adj, sa.psi, sa.psi_adj, y, 0.0, (8, 8), iters=40,
             blocks=([0, y.size], [eps]))
    assert np.array_equal(a.x, b.x)
    assert a.residual == b.residual


def test_every_block_constraint_holds_at_convergence():
    op, sa, x, y, sigma = _tiny(n=16, M=160, mask=0x1FF, L=2, seed=4)
    offs = [0, 40, 100, 160]
    eps = [synth.chi2_epsilon(sigma, offs[i + 1] - offs[i]) for i in range(3)]
    r = sdmm(op.phi, op.phi_adj, sa.psi, sa.psi_adj, y, 0.0, (16, 16), iters=3000, blocks=(offs, eps))
    xr = np.real(r.x)
    v = op.phi(xr)
    for i in range(3):
        a, b = offs[i], offs[i + 1]
        assert np.linalg.norm(y[a:b] - v[a:b]) <= eps[i] * (1 + 1e-3)
    assert xr.min() >= -1e-6 * xr.max()


@pytest.mark.slow
def test_two_blocks_match_slsqp_brute_force():
    n = 4
    op, sa, x, y, sigma = _tiny(n=n, M=12, mask=0x3, L=1, seed=8)
    offs = [0, 5, 12]
    eps = [synth.chi2_epsilon(sigma, 5), 0.5 * synth.chi2_epsilon(sigma, 7)]
    N = n * n
    Phi = np.stack([op.phi(np.eye(N)[k].reshape(n, n)) for k in range(N)], axis=1)
    Psit = np.stack([sa.psi_adj(np.eye(N)[k].reshape(n, n)).ravel() for k in range(N)], axis=1).real
    D = Psit.shape[0]
    r = sdmm(op.phi, op.phi_adj, sa.psi, sa.psi_adj, y, 0.0, (n, n), iters=6000, gamma=0.1,
             blocks=(offs, eps))
    f_sdmm = np.sum(np.abs(Psit @ np.real(r.x).ravel()))

    def obj(z):
        return z[N:].sum()
    cons = [dict(type="ineq", fun=lambda z: z[N:] - Psit @ z[:N]),
            dict(type="ineq", fun=lambda z: z[N:] + Psit @ z[:N])]
    for i in range(2):
        a, b, e = offs[i], offs[i + 1], eps[i]
        cons.append(dict(type="ineq", fun=lambda z, a=a, b=b, e=e:
                         e ** 2 - np.sum(np.abs(y[a:b] - Phi[a:b] @ z[:N]) ** 2)))
    z0 = np.concatenate([np.real(r.x).ravel(), np.abs(Psit @ np.real(r.x).ravel()) + 1e-3])
    bounds = [(0, None)] * N + [(None, None)] * D
    sol = optimize.minimize(obj, z0, method="SLSQP", constraints=cons, bounds=bounds,
                            options=dict(maxiter=3000, ftol=1e-14))
    for i in range(2):
        a, b = offs[i], offs[i + 1]
        assert np.linalg.norm(y[a:b] - Phi[a:b] @ np.real(r.x).ravel()) <= eps[i] * (1 + 1e-3)
    assert abs(f_sdmm - sol.fun) <= 1e-6 * sol.fun
