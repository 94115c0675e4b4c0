"""Reweighted l1 minimisation (SARA, Section 2.2): oracle, FP64.  Test infrastructure only.

SARA replaces the l0 prior ||Psi^dagger x||_0 by a sequence of weighted-l1 problems (eq. (3)
with a diagonal W of positive weights), each weight roughly the inverse magnitude of the
matching coefficient of the previous solution.  The paper fixes the scheme but not its
constants (they are those of the SARA paper, not reproduced here), so this module takes
these readings, shared with the GPU library:

* solve 0 is the problem with the given W (W = I by default: BPSA for the SARA dictionary);
* the weights of solve k >= 1 are w_j = delta_k / (delta_k + |alpha_j|) with
  alpha = Psi^dagger x^(k-1) (w_j = 1 where delta_k + |alpha_j| = 0).  This is the
  majorise-minimise step for the log-sum penalty sum_j log(delta + |alpha_j|): the weight is
  delta times the slope of log(delta + s) at s = |alpha_j|;
* delta_1 = max(delta0, delta_min), delta0 given or else the standard deviation of the
  coefficients alpha = Psi^dagger x^(0); delta_{k+1} = max(decay * delta_k, delta_min), with
  delta_min given or else sigma~ = sigma / nu, sigma = eps / sqrt(M + 2 sqrt(M)) (the noise
  level behind the chi-square bound eps, in the units of the normalised problem; with
  visibility blocks, the largest of the blocks' sigma_i = eps_i / sqrt(M_i + 2 sqrt(M_i)));
* solve k >= 1 is SDMM warm started from x^(k-1), with the nu and gamma of solve 0;
* stop after solve k when ||x^(k) - x^(k-1)|| / ||x^(k-1)|| < rel_var (0 when both are zero,
  infinite when only x^(k-1) is), or when k = reweights;
* reweighted TV (RWTV, Section 5): the same loop with the TV prior, the coefficients being the
  gradient magnitudes |(grad x)_ij| and the weights per pixel.
"""
import math
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

from .sdmm import SdmmResult, sdmm
from .tv import grad


def reweight(alpha: np.ndarray, delta: float) -> np.ndarray:
    """w_j = delta / (delta + |alpha_j|), 1 where the denominator is 0."""
    a = np.abs(np.asarray(alpha, dtype=np.complex128))
    den = delta + a
    out = np.ones_like(a)
    nz = den > 0
    out[nz] = delta / den[nz]
    return out


def noise_floor(epsilon: float, M: int, nu: float) -> float:
    """sigma / nu with sigma = eps / sqrt(M + 2 sqrt(M))."""
    return epsilon / math.sqrt(M + 2.0 * math.sqrt(M)) / nu


def relative_variation(x_new: np.ndarray, x_old: np.ndarray) -> float:
    d = float(np.linalg.norm(np.ravel(x_new - x_old)))
    o = float(np.linalg.norm(np.ravel(x_old)))
    if o == 0.0:
        return 0.0 if d == 0.0 else math.inf
    return d / o


@dataclass
class ReweightResult:
    x: np.ndarray
    solves: List[SdmmResult] = field(default_factory=list)
    deltas: List[float] = field(default_factory=list)        # delta of solves 1, 2, ...
    rel_vars: List[float] = field(default_factory=list)      # after solves 1, 2, ...
    weights: Optional[np.ndarray] = None                     # those of the last solve


def reweighted_sdmm(phi, phi_adj, psi, psi_adj, y, epsilon, shape, reweights: int = 5,
                    delta0: Optional[float] = None, decay: float = 0.1,
                    delta_min: Optional[float] = None, rel_var: float = 1e-3,
                    weights=None, **sdmm_kwargs) -> ReweightResult:
    """Solve 0 with `weights` (None: W = I), then up to `reweights` weighted solves."""
    r0 = sdmm(phi, phi_adj, psi, psi_adj, y, epsilon, shape, weights=weights, **sdmm_kwargs)
    out = ReweightResult(x=r0.x, solves=[r0], weights=weights)
    kw = dict(sdmm_kwargs)
    kw["nu"], kw["gamma"] = r0.nu, r0.gamma
    if delta_min is not None and delta_min >= 0:
        floor = delta_min
    elif sdmm_kwargs.get("blocks") is not None:
        offs, eps_b = sdmm_kwargs["blocks"]
        floor = max(noise_floor(e, offs[i + 1] - offs[i], r0.nu) for i, e in enumerate(eps_b))
    else:
        floor = noise_floor(epsilon, np.size(y), r0.nu)
    if sdmm_kwargs.get("tv_iters") is not None:
        # reweighted TV: the coefficients are the gradient magnitudes |(grad x)_ij|
        def coefficients(v):
            g1, g2 = grad(v)
            return np.sqrt(np.abs(g1) ** 2 + np.abs(g2) ** 2).astype(np.complex128)
    else:
        coefficients = psi_adj
    x = r0.x
    alpha = coefficients(x)
    delta = float(np.std(alpha)) if delta0 is None or delta0 <= 0 else delta0
    delta = max(delta, floor)
    for _ in range(reweights):
        w = reweight(alpha, delta)
        rk = sdmm(phi, phi_adj, psi, psi_adj, y, epsilon, shape, weights=w, x0=x, **kw)
        rv = relative_variation(rk.x, x)
        out.solves.append(rk)
        out.deltas.append(delta)
        out.rel_vars.append(rv)
        out.weights = w
        x = rk.x
        if rv < rel_var:
            break
        delta = max(decay * delta, floor)
        alpha = coefficients(x)
    out.x = x
    return out
