"""Total-variation prior (the TV and RWTV problems of Section 5): oracle, FP64.  Test
infrastructure only.

The TV problem replaces the analysis l1 term of eq. (3) by the (weighted) isotropic total
variation of the image, keeping positivity and the l2 data constraint:

    minimise  sum_ij w_ij |(grad x)_ij|   subject to  ||y - Phi x|| <= eps,  x >= 0.

In SDMM (Algorithm 1) this is f1 = TV with L1 = I, so sum_i L_i^dagger L_i is still
Phi^dagger Phi + 2 I and only branch i = 1 changes: r1 = prox_{gamma TV}(x_hat + z1).  The
paper does not print the TV proximity operator; this module takes Chambolle's dual projection
algorithm (J. Math. Imaging Vis. 20, 2004), with these readings shared by the GPU library:

* discrete gradient by forward differences, zero on the last row / column;
  divergence div = -grad^T (backward differences with the matching boundary rows);
* |g_ij| = sqrt(|g1_ij|^2 + |g2_ij|^2) with complex moduli (the image is iterated in C^N);
* weighted TV: the dual field is bounded by |p_ij| <= w_ij (w = 1: plain TV);
* prox_{gamma TV}(u) = u - gamma div p, p from `iters` steps of
      g = grad(div p - u / gamma),   p <- (p + tau g) / (1 + tau |g| / w)
  started at p = 0, with tau = 1/8 (Chambolle's bound, ||grad||^2 <= 8); a fixed step count
  (no data-dependent stop) so every solve runs the same arithmetic;
* gamma = 1e-3 max_ij |(grad Phi~^dagger y~)_ij| unless given (the l1 rule with grad in
  place of Psi^dagger).
"""
import numpy as np

TAU = 0.125


def grad(x: np.ndarray):
    """Forward differences (g1 along axis 0, g2 along axis 1), zero on the last row / column."""
    x = np.asarray(x, dtype=np.complex128)
    g1 = np.zeros_like(x)
    g2 = np.zeros_like(x)
    g1[:-1, :] = x[1:, :] - x[:-1, :]
    g2[:, :-1] = x[:, 1:] - x[:, :-1]
    return g1, g2


def div(p1: np.ndarray, p2: np.ndarray) -> np.ndarray:
    """div = -grad^T: backward differences, first row p1[0], last row -p1[n-2] (and so on)."""
    d = np.zeros_like(p1, dtype=np.complex128)
    d[0, :] += p1[0, :]
    d[1:-1, :] += p1[1:-1, :] - p1[:-2, :]
    d[-1, :] -= p1[-2, :]
    d[:, 0] += p2[:, 0]
    d[:, 1:-1] += p2[:, 1:-1] - p2[:, :-2]
    d[:, -1] -= p2[:, -2]
    return d


def tv_norm(x: np.ndarray, w=None) -> float:
    g1, g2 = grad(x)
    mag = np.sqrt(np.abs(g1) ** 2 + np.abs(g2) ** 2)
    return float(np.sum(mag if w is None else w * mag))


def prox_tv(u: np.ndarray, gamma: float, iters: int, w=None, return_dual: bool = False):
    """prox_{gamma TV_w}(u) by `iters` steps of Chambolle's dual projection algorithm."""
    u = np.asarray(u, dtype=np.complex128)
    wt = np.ones(u.shape) if w is None else np.asarray(w, dtype=np.float64)
    p1 = np.zeros_like(u)
    p2 = np.zeros_like(u)
    for _ in range(iters):
        g1, g2 = grad(div(p1, p2) - u / gamma)
        mag = np.sqrt(np.abs(g1) ** 2 + np.abs(g2) ** 2)
        den = 1.0 + TAU * mag / wt
        p1 = (p1 + TAU * g1) / den
        p2 = (p2 + TAU * g2) / den
    x = u - gamma * div(p1, p2)
    return (x, (p1, p2)) if return_dual else x
