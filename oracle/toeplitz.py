"""Precomputed normal operator Phi^dagger Phi as a Toeplitz (PSF) operator: oracle, FP64.
Test infrastructure only.

Section 3 notes that the global update's composite operator Phi^dagger Phi can be computed
once and stored, so the conjugate-gradient steps need not apply Phi and Phi^dagger.  For the
Fourier model y_m = sum_p x_p exp(-i omega_m . p) (pixel coordinates p = j - n/2), the
normal operator is a convolution on the image grid:

    (Phi^dagger Phi x)_p = sum_q h(p - q) x_q,    h(d) = sum_m exp(+i omega_m . d),

with d in [-(n-1), n-1] on each axis; h is Hermitian, h(-d) = conj h(d), and h(0) = M.  This
module holds that exact definition (the point-spread function h by direct sums) and the
operator itself, by circulant embedding on the 2n x 2n grid: c[d mod 2n] = h(d) for
|d| < n on both axes, 0 on the row and column d = n, and T x = crop(ifft2(fft2(c) fft2(pad
x))), a cyclic convolution that equals the linear one on the n x n image because
|p - q| < n.  The FFT is a library step; a direct double sum pins it on tiny inputs.
"""
import numpy as np
import scipy.fft


def psf(uv: np.ndarray, n: int) -> np.ndarray:
    """h(d) for d in [-n, n)^2 as a (2n, 2n) array indexed [d1 + n, d2 + n] (direct sums
    over the M frequencies, factorised per axis)."""
    uv = np.asarray(uv, dtype=np.float64)
    d = np.arange(-n, n, dtype=np.float64)
    e1 = np.exp(1j * np.outer(uv[:, 0], d))     # M x 2n
    e2 = np.exp(1j * np.outer(uv[:, 1], d))
    return e1.T @ e2


def circulant_embedding(h: np.ndarray) -> np.ndarray:
    """c on the K x K grid (K = 2n): c[d1 mod K, d2 mod K] = h(d1, d2) for |d| < n, 0 where
    d1 = n or d2 = n (never used by the cropped product)."""
    K = h.shape[0]
    n = K // 2
    c = np.zeros((K, K), dtype=np.complex128)
    idx = np.arange(-(n - 1), n)
    c[np.ix_(idx % K, idx % K)] = h[np.ix_(idx + n, idx + n)]
    return c


def toeplitz_normal(h: np.ndarray, x: np.ndarray) -> np.ndarray:
    """(T x)_p = sum_q h(p - q) x_q for an n x n image x (h from psf(uv, n))."""
    K = h.shape[0]
    n = K // 2
    c = circulant_embedding(h)
    xp = np.zeros((K, K), dtype=np.complex128)
    ix = (np.arange(n) - n // 2) % K                # pixel p = j - n/2 placed at p mod K
    xp[np.ix_(ix, ix)] = x
    y = scipy.fft.ifft2(scipy.fft.fft2(c) * scipy.fft.fft2(xp))
    return y[np.ix_(ix, ix)]


def toeplitz_normal_direct(h: np.ndarray, x: np.ndarray) -> np.ndarray:
    """The same product as a direct double sum (tiny n only)."""
    K = h.shape[0]
    n = K // 2
    out = np.zeros((n, n), dtype=np.complex128)
    for a1 in range(n):
        for a2 in range(n):
            # d = p - q = a - b for pixel indices a (output) and b (input)
            d1 = a1 - np.arange(n)[:, None] + n
            d2 = a2 - np.arange(n)[None, :] + n
            out[a1, a2] = np.sum(h[d1, d2] * x)
    return out
