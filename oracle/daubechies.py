"""Daubechies orthonormal wavelet filters (oracle, FP64).

Section 2.2: the SARA dictionary concatenates the Dirac basis and the first eight
orthonormal Daubechies wavelet bases, Db1-Db8.  Db-N has N vanishing moments and a
lowpass filter h of length 2N.  Reading taken (the paper names the bases only): the
extremal-phase (minimum-phase) filters, obtained by spectral factorisation

    |H(w)|^2 = 2 cos^{2N}(w/2) P(sin^2(w/2)),  P(y) = sum_{k<N} C(N-1+k, k) y^k,

keeping the roots of the factor Q(z) inside the unit circle, normalised so sum h = sqrt 2.
The highpass is g[k] = (-1)^k h[2N-1-k].  Closed forms: Db1 = [1, 1]/sqrt 2;
Db2 = [1+sqrt3, 3+sqrt3, 3-sqrt3, 1-sqrt3] / (4 sqrt 2).
"""
from math import comb, sqrt

import numpy as np


def daubechies_lowpass(N: int) -> np.ndarray:
    """Extremal-phase Daubechies lowpass filter with N vanishing moments (length 2N)."""
    if N < 1:
        raise ValueError("N >= 1")
    # Roots of P(y) (polynomial in y = sin^2(w/2)); numpy.roots wants highest power first.
    pc = [comb(N - 1 + k, k) for k in range(N)]
    yroots = np.roots(pc[::-1]) if N > 1 else np.array([])
    # y = (2 - z - 1/z)/4  =>  z^2 - (2 - 4y) z + 1 = 0; keep the root inside the circle.
    zr = []
    for y in yroots:
        b = 2.0 - 4.0 * y
        disc = np.sqrt(b * b - 4.0 + 0j)
        z1, z2 = (b + disc) / 2.0, (b - disc) / 2.0
        zr.append(z1 if abs(z1) < 1.0 else z2)
    poly = np.array([1.0 + 0j])
    for _ in range(N):
        poly = np.convolve(poly, [1.0, 1.0])          # (z + 1)^N
    for z in zr:
        poly = np.convolve(poly, [1.0, -z])            # (z - z_r)
    h = np.real(poly)
    return h * (sqrt(2.0) / h.sum())


def highpass_from_lowpass(h: np.ndarray) -> np.ndarray:
    L = len(h)
    k = np.arange(L)
    return ((-1.0) ** k) * h[::-1]
