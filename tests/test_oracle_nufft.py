"""Pins for the oracle's measurement operator (Section 2.1, Section 4 NUFFT).

* direct NUDFT brute force on tiny inputs (the target model the NUFFT approximates);
* closed form of the Kaiser-Bessel Fourier transform against numerical quadrature;
* the adjoint identity <Phi x, y> = <x, Phi^dagger y> (Phi^dagger is coded separately:
  transposed sparse matrix and inverse FFT);
* F against the explicit DFT matrix on a tiny grid;
* special case: a single-pixel image gives a pure phase ramp exp(-i omega.p).
"""
import numpy as np
import pytest
from scipy import integrate, special

from oracle.kaiser_bessel import deapodisation, default_beta, kb_ft, kb_kernel
from oracle.nufft import Nufft, first_tap, grid_coordinates, nudft


@pytest.mark.parametrize("n,J,tol", [(8, 6, 3e-5), (16, 6, 3e-5), (32, 6, 3e-5),
                                     (16, 8, 3e-7), (32, 8, 3e-7)])
def test_nufft_matches_direct_nudft(n, J, tol):
    rng = np.random.default_rng(100 + n + J)
    uv = rng.uniform(-np.pi, np.pi, (200, 2))
    x = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    op = Nufft(n, uv, J)
    y = op.phi(x)
    ref = nudft(x, uv)
    assert np.linalg.norm(y - ref) / np.linalg.norm(ref) < tol


def test_nudft_is_the_textbook_sum():
    # nudft on a 2x2 image, written out term by term
    x = np.array([[1.0, 2.0], [3.0, 4.0j]])
    uv = np.array([[0.3, -1.1], [2.0, 0.5]])
    p = [-1, 0]
    ref = [sum(x[a, b] * np.exp(-1j * (w[0] * p[a] + w[1] * p[b]))
               for a in range(2) for b in range(2)) for w in uv]
    assert np.allclose(nudft(x, uv), ref, rtol=0, atol=1e-14)


@pytest.mark.parametrize("J", [4, 6, 8])
def test_kb_ft_closed_form_vs_quadrature(J):
    beta = default_beta(J)
    for nu in [0.0, 0.05, 0.13, 0.25]:
        re = integrate.quad(lambda t: kb_kernel(np.array([t]), J, beta)[0] * np.cos(2 * np.pi * nu * t),
                            -J / 2, J / 2, epsabs=1e-14, epsrel=1e-13, limit=200)[0]
        assert abs(re - kb_ft(np.array([nu]), J, beta)[0]) <= 1e-12 * abs(re)


def test_kb_kernel_values():
    J, beta = 6, default_beta(6)
    assert kb_kernel(np.array([0.0]), J, beta)[0] == pytest.approx(1.0, abs=1e-15)
    assert kb_kernel(np.array([3.0]), J, beta)[0] == pytest.approx(1.0 / special.i0(beta), rel=1e-14)
    assert kb_kernel(np.array([3.0001, -3.5]), J, beta).tolist() == [0.0, 0.0]
    t = np.linspace(-3, 3, 41)
    assert np.allclose(kb_kernel(t, J, beta), kb_kernel(-t, J, beta), rtol=0, atol=0)


def test_first_tap_rule():
    J = 6
    kap = np.array([0.0, 0.5, -0.5, 2.999999, 3.0, -7.25])
    k0 = first_tap(kap, J)
    for kv, k in zip(kap, k0):
        t = kv - (k + np.arange(J))
        assert np.all(t <= J / 2) and np.all(t > -J / 2 - 1e-12)
        assert t[0] < J / 2 and t[-1] >= -J / 2


def test_adjoint_identity():
    rng = np.random.default_rng(7)
    n = 32
    uv = rng.normal(0, np.pi / 4, (500, 2))
    op = Nufft(n, uv, 6)
    x = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    y = rng.standard_normal(500) + 1j * rng.standard_normal(500)
    lhs = np.vdot(op.phi(x), y)
    rhs = np.vdot(x, op.phi_adj(y))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_fft_factor_against_dft_matrix():
    # With a Dirac at the centre pixel (p = 0), Z S x puts s0^2 at grid node (0,0) only;
    # F then gives a constant grid, and y_m = s0^2 sum_k psi psi.  Check F on a random
    # grid against the explicit DFT matrix instead, through phi with a 1-tap identity-like G.
    K = 8
    rng = np.random.default_rng(3)
    g = rng.standard_normal((K, K)) + 1j * rng.standard_normal((K, K))
    k = np.arange(K)
    Fm = np.exp(-2j * np.pi * np.outer(k, k) / K)
    import scipy.fft
    assert np.allclose(scipy.fft.fft2(g), Fm @ g @ Fm.T, rtol=0, atol=1e-12)
    assert np.allclose(scipy.fft.ifft2(g) * K * K, Fm.conj().T @ g @ Fm.conj(), rtol=0, atol=1e-12)


def test_single_pixel_is_phase_ramp():
    n, J = 16, 8
    rng = np.random.default_rng(11)
    uv = rng.uniform(-np.pi, np.pi, (100, 2))
    op = Nufft(n, uv, J)
    for (j1, j2) in [(8, 8), (0, 15), (3, 11)]:
        x = np.zeros((n, n)); x[j1, j2] = 1.0
        ref = np.exp(-1j * (uv[:, 0] * (j1 - n // 2) + uv[:, 1] * (j2 - n // 2)))
        assert np.max(np.abs(op.phi(x) - ref)) < 3e-6


def test_deapodisation_symmetry_and_centre():
    n, K, J = 64, 128, 6
    beta = default_beta(J)
    s = deapodisation(n, K, J, beta)
    assert s[n // 2] == pytest.approx(1.0 / kb_ft(np.array([0.0]), J, beta)[0], rel=1e-15)
    assert np.allclose(s[1:], s[1:][::-1], rtol=1e-14)


def test_grid_coordinates_formula():
    uv = np.array([[np.pi / 2, -np.pi]])
    kap = grid_coordinates(uv, 128)
    assert kap.tolist() == [[32.0, -64.0]]


def test_nudft_adjoint_at_pixels_is_the_adjoint_of_nudft():
    # <nudft(x), y> = <x, adjoint(y)> over all pixels of a small image
    from oracle.nufft import nudft, nudft_adjoint_at
    rng = np.random.default_rng(31)
    n, M = 6, 25
    uv = rng.uniform(-np.pi, np.pi, (M, 2))
    x = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    y = rng.standard_normal(M) + 1j * rng.standard_normal(M)
    pix = [(a, b) for a in range(n) for b in range(n)]
    xa = nudft_adjoint_at(y, uv, n, pix).reshape(n, n)
    lhs = np.vdot(nudft(x, uv), y)
    rhs = np.vdot(x, xa)
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)
