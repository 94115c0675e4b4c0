"""Periodised multi-level 2D DWT and the SARA dictionary (oracle, FP64).

Section 2.2: Psi = [Psi_1, ..., Psi_q] concatenates q orthonormal bases, here the Dirac
basis and Daubechies Db1-Db8.  Section 3 uses Psi Psi^dagger = I, which holds for a
concatenation of q orthonormal bases once each is scaled by 1/sqrt(q) (the tight-frame
reading taken here).

Each wavelet basis W_b is an L-level periodised orthonormal 2D DWT:

  one level on an axis of length Ls (even):  a[i] = sum_k h[k] x[(2i + k) mod Ls]
                                              d[i] = sum_k g[k] x[(2i + k) mod Ls]
  output along the axis is [a | d]; a level applies axis 1, then axis 0, to the
  top-left Ls x Ls block; the next level recurses on the top-left (LL) quarter
  (Mallat layout).

Psi^dagger x = (1/sqrt q) [x (Dirac), W_1 x, ..., W_8 x] restricted to the selected bases;
Psi alpha = (1/sqrt q) sum_b W_b^T alpha_b.  The synthesis here is written as the literal
transpose of the analysis (scatter-add), not as an inverse formula.
"""
import numpy as np

from .daubechies import daubechies_lowpass, highpass_from_lowpass

DIRAC = 0


def basis_list(dict_mask: int):
    """Selected bases in dictionary order: 0 = Dirac, b = Db-b (b = 1..8)."""
    return [b for b in range(9) if dict_mask >> b & 1]


def _analysis_axis(X, h, g, axis):
    Ls = X.shape[axis]
    half = Ls // 2
    i2 = 2 * np.arange(half)
    a = np.zeros_like(np.take(X, np.arange(half), axis=axis))
    d = np.zeros_like(a)
    for k in range(len(h)):
        sl = np.take(X, (i2 + k) % Ls, axis=axis)
        a = a + h[k] * sl
        d = d + g[k] * sl
    return np.concatenate([a, d], axis=axis)


def _synthesis_axis(Y, h, g, axis):
    """Transpose of _analysis_axis: scatter each coefficient back along its filter taps."""
    Ls = Y.shape[axis]
    half = Ls // 2
    a = np.take(Y, np.arange(half), axis=axis)
    d = np.take(Y, np.arange(half, Ls), axis=axis)
    X = np.zeros_like(Y)
    i2 = 2 * np.arange(half)
    Xm = np.moveaxis(X, axis, 0)
    am = np.moveaxis(a, axis, 0)
    dm = np.moveaxis(d, axis, 0)
    for k in range(len(h)):
        np.add.at(Xm, (i2 + k) % Ls, h[k] * am + g[k] * dm)
    return X


def dwt2(x: np.ndarray, h: np.ndarray, levels: int) -> np.ndarray:
    """Forward L-level periodised 2D DWT (Mallat layout)."""
    g = highpass_from_lowpass(h)
    out = np.array(x, dtype=np.result_type(x, np.float64), copy=True)
    n = out.shape[0]
    for lev in range(levels):
        Ls = n >> lev
        blk = out[:Ls, :Ls]
        blk = _analysis_axis(blk, h, g, axis=1)
        blk = _analysis_axis(blk, h, g, axis=0)
        out[:Ls, :Ls] = blk
    return out


def dwt2_adjoint(c: np.ndarray, h: np.ndarray, levels: int) -> np.ndarray:
    """Transpose of dwt2 (equal to its inverse, the basis being orthonormal)."""
    g = highpass_from_lowpass(h)
    out = np.array(c, dtype=np.result_type(c, np.float64), copy=True)
    n = out.shape[0]
    for lev in reversed(range(levels)):
        Ls = n >> lev
        blk = out[:Ls, :Ls]
        blk = _synthesis_axis(blk, h, g, axis=0)
        blk = _synthesis_axis(blk, h, g, axis=1)
        out[:Ls, :Ls] = blk
    return out


class Sara:
    """Psi and Psi^dagger for n x n images, dictionary ``dict_mask``, ``levels`` levels."""

    def __init__(self, n: int, dict_mask: int = 0x1FF, levels: int = 4):
        if n % (1 << levels):
            raise ValueError("n must be divisible by 2^levels")
        self.n = n
        self.levels = levels
        self.bases = basis_list(dict_mask)
        self.q = len(self.bases)
        self.scale = 1.0 / np.sqrt(self.q)
        self.filters = {b: daubechies_lowpass(b) for b in self.bases if b != DIRAC}

    @property
    def D(self):
        return self.q * self.n * self.n

    def psi_adj(self, x: np.ndarray) -> np.ndarray:
        """alpha = Psi^dagger x, shape (q, n, n)."""
        x = np.asarray(x).reshape(self.n, self.n)
        out = []
        for b in self.bases:
            if b == DIRAC:
                out.append(self.scale * x.astype(np.result_type(x, np.float64)))
            else:
                out.append(self.scale * dwt2(x, self.filters[b], self.levels))
        return np.stack(out)

    def psi(self, alpha: np.ndarray) -> np.ndarray:
        """x = Psi alpha for alpha of shape (q, n, n)."""
        alpha = np.asarray(alpha).reshape(self.q, self.n, self.n)
        x = np.zeros((self.n, self.n), dtype=np.result_type(alpha, np.float64))
        for i, b in enumerate(self.bases):
            if b == DIRAC:
                x = x + alpha[i]
            else:
                x = x + dwt2_adjoint(alpha[i], self.filters[b], self.levels)
        return self.scale * x
