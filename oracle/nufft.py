"""Measurement operator Phi = G F Z S and its adjoint (oracle, FP64).

Section 2.1: visibilities are Fourier measurements of the image at M continuous spatial
frequencies, y = Phi x + n.  Section 4: PURIFY implements Phi as a non-uniform FFT.  The
conventions taken (the paper defers them to its companion paper):

* pixel coordinates p = j - n/2 on each axis (j = 0..n-1), axis 0 pairs with omega_1;
* target model (direct NUDFT):  y_m ~ sum_p x_p exp(-i (omega_m1 p_1 + omega_m2 p_2));
* S: multiply by s_p1 s_p2, the Kaiser-Bessel deapodisation;
* Z: place s_p x_p at grid node (p_1 mod K, p_2 mod K) of a K x K grid, K = 2n, zeros
  elsewhere;
* F: unnormalised forward 2D DFT, exp(-2 pi i k.a / K) (scipy.fft.fft2);
* G: kappa_m = omega_m K / (2 pi); per axis taps k = k0 .. k0+J-1 with
  k0 = floor(kappa - J/2) + 1; weight psi(kappa_1 - k_1) psi(kappa_2 - k_2) on grid node
  (k_1 mod K, k_2 mod K).  Built as a scipy.sparse CSR matrix (M x K^2, J^2 entries a row).
* Phi^dagger = S Z^T F^dagger G^T, where F^dagger = K^2 ifft2 is the conjugate transpose of
  F (not its inverse) and G^T is the transpose of the real matrix G.
"""
import math
import os

import numpy as np
import scipy.fft
import scipy.sparse as sp

from .kaiser_bessel import default_beta, deapodisation, kb_kernel

# scipy.fft splits a 2D transform into independent 1D transforms over its threads, so the
# thread count changes the run time, not the result.
FFT_WORKERS = os.cpu_count() or 1


def grid_coordinates(uv: np.ndarray, K: int) -> np.ndarray:
    """kappa = omega K / (2 pi), FP64, evaluated as (omega * K) / (2 pi)."""
    return (np.asarray(uv, dtype=np.float64) * K) / (2.0 * math.pi)


def first_tap(kappa: np.ndarray, J: int) -> np.ndarray:
    """k0 = floor(kappa - J/2) + 1 (ties at |kappa - k| = J/2 resolve to this rule)."""
    return np.floor(kappa - J / 2.0).astype(np.int64) + 1


class Nufft:
    """Phi and Phi^dagger for an n x n image and M frequencies ``uv`` (M x 2, radians)."""

    def __init__(self, n: int, uv: np.ndarray, J: int = 6, beta: float = None,
                 oversample: int = 2):
        self.n = n
        self.K = K = oversample * n
        self.J = J
        self.beta = default_beta(J) if beta is None else beta
        self.uv = np.asarray(uv, dtype=np.float64)
        self.M = M = self.uv.shape[0]
        s = deapodisation(n, K, J, self.beta)
        self.s2 = np.outer(s, s)
        p = np.arange(n) - n // 2
        self.rows = p % K          # grid index of each pixel, both axes
        kap = grid_coordinates(self.uv, K)
        k0 = first_tap(kap, J)
        taps = np.arange(J)
        k1 = k0[:, 0:1] + taps[None, :]                       # M x J
        k2 = k0[:, 1:2] + taps[None, :]
        w1 = kb_kernel(kap[:, 0:1] - k1, J, self.beta)        # M x J
        w2 = kb_kernel(kap[:, 1:2] - k2, J, self.beta)
        col = ((k1 % K)[:, :, None] * K + (k2 % K)[:, None, :]).reshape(M, J * J)
        val = (w1[:, :, None] * w2[:, None, :]).reshape(M, J * J)
        rowi = np.repeat(np.arange(M), J * J)
        self.G = sp.csr_matrix((val.ravel(), (rowi, col.ravel())), shape=(M, K * K))
        self.GT = self.G.T.tocsr()

    # --- the four factors -------------------------------------------------------------
    def zero_pad(self, x):
        g = np.zeros((self.K, self.K), dtype=np.complex128)
        g[np.ix_(self.rows, self.rows)] = x
        return g

    def crop(self, g):
        return g[np.ix_(self.rows, self.rows)]

    def phi(self, x: np.ndarray) -> np.ndarray:
        """y = G F Z S x."""
        x = np.asarray(x, dtype=np.complex128).reshape(self.n, self.n)
        g = self.zero_pad(self.s2 * x)
        ghat = scipy.fft.fft2(g, workers=FFT_WORKERS)
        return self.G @ ghat.ravel()

    def phi_adj(self, y: np.ndarray) -> np.ndarray:
        """x = S Z^T F^dagger G^T y."""
        y = np.asarray(y, dtype=np.complex128)
        ghat = (self.GT @ y).reshape(self.K, self.K)
        g = scipy.fft.ifft2(ghat, workers=FFT_WORKERS) * (self.K * self.K)
        return self.s2 * self.crop(g)

    def normal(self, x: np.ndarray) -> np.ndarray:
        return self.phi_adj(self.phi(x))


def nudft(x: np.ndarray, uv: np.ndarray) -> np.ndarray:
    """Direct non-uniform DFT, y_m = sum_p x_p exp(-i omega_m . p), p = j - n/2.
    O(M N); for tiny problems only."""
    n = x.shape[0]
    p = np.arange(n, dtype=np.float64) - n // 2
    e1 = np.exp(-1j * np.outer(uv[:, 0], p))    # M x n
    e2 = np.exp(-1j * np.outer(uv[:, 1], p))
    return np.einsum("ma,ab,mb->m", e1, np.asarray(x, dtype=np.complex128), e2)


def nudft_adjoint_at(y: np.ndarray, uv: np.ndarray, n: int, pixels) -> np.ndarray:
    """Direct adjoint NUDFT at selected pixels: x_p = sum_m y_m exp(+i omega_m . p), with
    p = (j1 - n/2, j2 - n/2) for each (j1, j2) in `pixels`.  O(M) per pixel."""
    j = np.asarray(pixels, dtype=np.float64).reshape(-1, 2) - n // 2
    ph = np.outer(uv[:, 0], j[:, 0]) + np.outer(uv[:, 1], j[:, 1])      # M x P
    return np.asarray(y, dtype=np.complex128) @ np.exp(1j * ph)
