"""Pins of the Toeplitz (PSF) form of Phi^dagger Phi (Section 3, precomputed composite
operator): the PSF-convolution equals the dense NUDFT normal matrix built by brute force,
the FFT circulant embedding equals the direct double sum, the PSF is Hermitian with
h(0) = M, and the NUFFT normal operator agrees with it to the NUFFT's accuracy."""
import numpy as np

from oracle.nufft import Nufft, nudft
from oracle.sara import Sara
from oracle.sdmm import sdmm
from oracle.toeplitz import psf, toeplitz_normal, toeplitz_normal_direct
from paper_1406_0359_amd import synth


def _uv(M, n, seed):
    return synth.uv_coverage(M, 2 * n, np.random.default_rng(seed))


def test_psf_convolution_is_the_nudft_normal_matrix():
    n, M = 8, 60
    uv = _uv(M, n, 1)
    N = n * n
    A = np.stack([nudft(np.eye(N)[k].reshape(n, n), uv) for k in range(N)], axis=1)   # M x N
    rng = np.random.default_rng(2)
    x = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    ref = (A.conj().T @ (A @ x.ravel())).reshape(n, n)
    h = psf(uv, n)
    assert np.linalg.norm(toeplitz_normal_direct(h, x) - ref) < 1e-12 * np.linalg.norm(ref)
    assert np.linalg.norm(toeplitz_normal(h, x) - ref) < 1e-12 * np.linalg.norm(ref)


def test_fft_embedding_equals_direct_sum_for_any_kernel():
    n = 6
    rng = np.random.default_rng(4)
    h = rng.standard_normal((2 * n, 2 * n)) + 1j * rng.standard_normal((2 * n, 2 * n))
    x = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    d = toeplitz_normal_direct(h, x)
    assert np.linalg.norm(toeplitz_normal(h, x) - d) < 1e-13 * np.linalg.norm(d)


def test_psf_hermitian_and_centre():
    n, M = 16, 300
    h = psf(_uv(M, n, 3), n)
    i = np.arange(1, 2 * n)                     # d = -(n-1) .. n-1
    assert np.max(np.abs(h[np.ix_(i, i)] - np.conj(h[np.ix_(i[::-1], i[::-1])]))) < 1e-11
    assert abs(h[n, n] - M) < 1e-12 * M


def test_nufft_normal_agrees_with_psf_to_nufft_accuracy():
    n, M = 32, 2000
    uv = _uv(M, n, 5)
    rng = np.random.default_rng(6)
    x = rng.standard_normal((n, n))
    t = toeplitz_normal(psf(uv, n), x)
    g = Nufft(n, uv, 6).normal(x)
    assert np.linalg.norm(g - t) / np.linalg.norm(t) < 1e-4


def test_sdmm_with_stored_normal_equals_plain_sdmm():
    n, M = 8, 48
    uv = _uv(M, n, 7)
    op = Nufft(n, uv, 6)
    sa = Sara(n, 0x3, 2)
    rng = np.random.default_rng(8)
    x = synth.blob_image(n, 3, rng)
    y = op.phi(x)
    eps = 0.01 * np.linalg.norm(y)
    a = sdmm(op.phi, op.phi_adj, sa.psi, sa.psi_adj, y, eps, (n, n), iters=40)
    b = sdmm(op.phi, op.phi_adj, sa.psi, sa.psi_adj, y, eps, (n, n), iters=40,
             normal=lambda v: op.phi_adj(op.phi(v)))
    assert np.linalg.norm(a.x - b.x) < 1e-12 * np.linalg.norm(a.x)
