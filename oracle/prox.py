"""Proximity operators (oracle, FP64).

Eq. (7) defines prox_f(x) = argmin_z f(z) + ||x - z||^2 / 2.  Eq. (6) splits the problem
into f1 = ||W .||_1 (on Psi^dagger x), f2 = indicator of the positive orthant, and
f3 = indicator of the l2 ball B(y, eps) (on Phi x).  Their proximity operators in closed form:

* prox_{gamma ||W.||_1}(u)_j = u_j max(0, 1 - gamma w_j / |u_j|)   (complex soft threshold;
  0 where u_j = 0);
* prox of the positive-orthant indicator: Re(u) clipped at 0, imaginary part 0 (x is
  iterated in C^N, positivity means x in R_+^N, a subset of C^N);
* prox of the l2-ball indicator: y + (u - y) min(1, eps / ||u - y||)  (u itself when
  ||u - y|| = 0);
* with the data split into R blocks (eqs. (4)-(5)), the constraint set is the product of the
  blocks' balls B(y_i, eps_i) and its projection acts block by block.
"""
import numpy as np


def soft_threshold(u: np.ndarray, thr) -> np.ndarray:
    u = np.asarray(u, dtype=np.complex128)
    mag = np.abs(u)
    scale = np.zeros_like(mag)
    nz = mag > 0
    thr = np.broadcast_to(np.asarray(thr, dtype=np.float64), mag.shape)
    scale[nz] = np.maximum(0.0, 1.0 - thr[nz] / mag[nz])
    return u * scale


def project_positive(u: np.ndarray) -> np.ndarray:
    return np.maximum(np.real(u), 0.0).astype(np.complex128)


def project_l2_ball(u: np.ndarray, y: np.ndarray, eps: float) -> np.ndarray:
    d = np.asarray(u, dtype=np.complex128) - y
    nd = np.linalg.norm(d)
    if nd == 0.0:
        return np.array(u, dtype=np.complex128)
    return y + d * min(1.0, eps / nd)


def project_l2_balls(u: np.ndarray, y: np.ndarray, offsets, eps) -> np.ndarray:
    """Projection onto the product of the balls B(y_i, eps_i), block i = [offsets[i],
    offsets[i + 1]) of the visibility vector."""
    out = np.array(u, dtype=np.complex128)
    for i in range(len(eps)):
        a, b = offsets[i], offsets[i + 1]
        out[a:b] = project_l2_ball(u[a:b], y[a:b], eps[i])
    return out
