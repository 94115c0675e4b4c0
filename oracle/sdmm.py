"""SDMM for the constrained, weighted-l1, analysis problem with positivity (oracle, FP64).

Problem, eqs. (3) and (6) with R = 1: minimise ||W Psi^dagger x||_1 subject to x >= 0 and
||y - Phi x||_2 <= eps, written as f1(L1 x) + f2(L2 x) + f3(L3 x) with L1 = Psi^dagger,
L2 = I, L3 = Phi.  Algorithm 1 (SDMM):

  init  gamma > 0, x_hat = 0, z_i = 0, r_i = L_i x_hat, x_i = L_i^dagger r_i   (so x_i = 0)
  loop  x_hat = (sum_i L_i^dagger L_i)^-1 sum_i x_i                    (global update)
        for each i:  r_i = prox_{gamma f_i}(L_i x_hat + z_i)
                     z_i = z_i + L_i x_hat - r_i
                     x_i = L_i^dagger (r_i - z_i)
        stop on the halting test

Section 3: sum_i L_i^dagger L_i = Phi^dagger Phi + Psi Psi^dagger + I = Phi^dagger Phi + 2I
(Psi a tight frame), and the global update is solved by conjugate gradient.  The halting
test: relative variation of the objective below xi and ||y - Phi x_hat|| <= eps.

Readings taken where the paper is silent:
* Phi is normalised by nu = ||Phi||_2 (power iteration on Phi^dagger Phi from the all-ones
  image, fixed count): Phi~ = Phi/nu, y~ = y/nu, eps~ = eps/nu.  The constraint set is
  unchanged; the iteration path is not.
* gamma = 1e-3 max_j |(Psi^dagger Phi~^dagger y~)_j| unless given.
* CG: warm start from the previous x_hat, exactly ``cg_iters`` steps, no preconditioner,
  stop early only when <r, r> = 0.
* objective f_t = ||W Psi^dagger x_hat||_1; halting uses eps~ (1 + slack).
"""
from dataclasses import dataclass, field
from typing import Callable, List, Optional

import numpy as np

from .prox import project_l2_ball, project_l2_balls, project_positive, soft_threshold
from .tv import grad, prox_tv, tv_norm


def operator_norm(normal: Callable[[np.ndarray], np.ndarray], shape, iters: int = 100):
    """nu = sqrt(largest eigenvalue of Phi^dagger Phi) by the power method, starting from
    the normalised all-ones image; returns (nu, last Rayleigh-free estimate lambda)."""
    v = np.ones(shape, dtype=np.complex128)
    v /= np.linalg.norm(v)
    lam = 0.0
    for _ in range(iters):
        w = normal(v)
        lam = np.linalg.norm(w)
        v = w / lam
    return float(np.sqrt(lam)), float(lam)


def conjugate_gradient(apply_A, b, x0, iters: int):
    """Textbook CG on the Hermitian positive definite A, warm started at x0."""
    x = np.array(x0, dtype=np.complex128, copy=True)
    r = b - apply_A(x)
    p = r.copy()
    rho = np.vdot(r, r).real
    for _ in range(iters):
        if rho == 0.0:
            break
        q = apply_A(p)
        alpha = rho / np.vdot(p, q).real
        x = x + alpha * p
        r = r - alpha * q
        rho_new = np.vdot(r, r).real
        p = r + (rho_new / rho) * p
        rho = rho_new
    return x


def halting_due(t: int, check_every: int, iters: int) -> bool:
    """Whether the stopping test runs after iteration t (1-based) when it is checked every
    ``check_every`` iterations: from the second iteration on (the first has no predecessor
    to compare with), at multiples of ``check_every`` and after the last iteration."""
    k = max(1, int(check_every))
    return t >= 2 and (t % k == 0 or t == iters)


def constraints_met(residuals, bounds, slack: float) -> bool:
    """Data-fidelity half of the stopping rule (Section 3): every block's residual
    ||y_i - Phi_i x_hat|| is within its bound eps_i, relaxed by the factor (1 + slack)."""
    return all(r <= e * (1.0 + slack) for r, e in zip(residuals, bounds))


def halting_test(f_prev: float, f: float, feasible: bool, xi: float) -> bool:
    """Stopping rule of Section 3 (Algorithm 1's halting criteria): stop when the relative
    variation of the objective between successive solutions, |f_t - f_{t-1}| / f_t, is
    below xi AND the data constraints hold (``feasible``).  Both conditions are required;
    a zero (or non-positive, or non-finite) current objective never stops."""
    if f_prev is None or not (f > 0) or not np.isfinite(f) or not np.isfinite(f_prev):
        return False
    return bool(abs(f - f_prev) / f < xi) and bool(feasible)


@dataclass
class SdmmResult:
    x: np.ndarray
    iterations: int
    nu: float
    gamma: float
    objective: List[float] = field(default_factory=list)
    residual: List[float] = field(default_factory=list)
    converged: bool = False


def sdmm(phi, phi_adj, psi, psi_adj, y, epsilon, shape, iters: int = 300,
         cg_iters: int = 10, gamma: Optional[float] = None, nu: Optional[float] = None,
         weights=None, halting: bool = False, xi: float = 1e-4, slack: float = 1e-3,
         nu_iters: int = 100, x0=None, normal=None, blocks=None, tv_iters=None,
         check_every: int = 1) -> SdmmResult:
    """Run SDMM (Algorithm 1, R = 1, S = 3) and return x_hat (complex; the image is Re).
    normal: a stored form of Phi^dagger Phi for the global update's conjugate-gradient
    operator (Section 3), e.g. the Toeplitz operator of oracle.toeplitz; None applies Phi
    and Phi^dagger.  nu, the proximity steps and x_i = L_i^dagger L_i x_hat(0) always use Phi.
    blocks: (offsets, eps_list) splitting the visibilities into R blocks, block i =
    [offsets[i], offsets[i + 1]) with bound eps_list[i] (eqs. (4)-(5), S = R + 2 functions);
    `epsilon` is then unused.  Since Phi^dagger of the stacked vector is sum_i Phi_i^dagger,
    the R data branches together are one projection onto the product of balls followed by one
    Phi^dagger; halting asks every block's residual to be within its bound.
    tv_iters: f1 = the (weighted) total variation with L1 = I instead of the l1 term
    (oracle.tv: prox by that many dual projection steps; weights per pixel; objective TV(x_hat);
    default gamma 1e-3 max |grad Phi~^dagger y~|).  psi and psi_adj are then unused.
    halting: stop after iteration t when halting_due(t, check_every, iters) and
    halting_test(f_{t-1}, f_t, constraints_met(...), xi); f_{t-1} is always the previous
    iteration's objective (successive solutions), whatever the test period."""
    if nu is None or nu <= 0:
        nu, _ = operator_norm(lambda v: phi_adj(phi(v)), shape, nu_iters)
    yt = np.asarray(y, dtype=np.complex128) / nu
    et = epsilon / nu
    if blocks is not None:
        offsets = [int(o) for o in blocks[0]]
        ets = [float(e) / nu for e in blocks[1]]
    P = lambda v: phi(v) / nu
    Pt = lambda v: phi_adj(v) / nu
    if gamma is None or gamma <= 0:
        if tv_iters is None:
            gamma = 1e-3 * float(np.max(np.abs(psi_adj(Pt(yt)))))
        else:
            g1, g2 = grad(Pt(yt))
            gamma = 1e-3 * float(np.max(np.sqrt(np.abs(g1) ** 2 + np.abs(g2) ** 2)))
    if normal is None:
        A = lambda v: Pt(P(v)) + 2.0 * v
    else:
        A = lambda v: normal(v) / (nu * nu) + 2.0 * v

    xh = np.zeros(shape, dtype=np.complex128) if x0 is None else np.array(x0, np.complex128)
    v1 = psi_adj(xh) if tv_iters is None else xh.copy()
    z1 = np.zeros_like(v1, dtype=np.complex128)
    z2 = np.zeros(shape, dtype=np.complex128)
    z3 = np.zeros(yt.shape, dtype=np.complex128)
    x1 = (psi(v1) if tv_iters is None else v1).astype(np.complex128)   # L_1^dagger L_1 x_hat(0)
    x2 = xh.copy()
    x3 = Pt(P(xh))
    w = 1.0 if weights is None else np.asarray(weights, dtype=np.float64).reshape(v1.shape)

    res = SdmmResult(x=xh, iterations=0, nu=nu, gamma=gamma)
    f_prev = None
    for t in range(1, iters + 1):
        xh = conjugate_gradient(A, x1 + x2 + x3, xh, cg_iters)
        if tv_iters is None:
            # i = 1: l1 term on Psi^dagger x
            v1 = psi_adj(xh)
            u = v1 + z1
            r1 = soft_threshold(u, gamma * w)
            z1 = u - r1
            x1 = psi(r1 - z1)
        else:
            # i = 1: total variation on x (L1 = I)
            u = xh + z1
            r1 = prox_tv(u, gamma, tv_iters, None if weights is None else w)
            z1 = u - r1
            x1 = r1 - z1
        # i = 2: positivity
        u = xh + z2
        r2 = project_positive(u)
        z2 = u - r2
        x2 = r2 - z2
        # i = 3: data fidelity l2 ball
        v3 = P(xh)
        u = v3 + z3
        r3 = project_l2_ball(u, yt, et) if blocks is None else project_l2_balls(u, yt, offsets, ets)
        z3 = u - r3
        x3 = Pt(r3 - z3)

        f = float(np.sum(w * np.abs(v1))) if tv_iters is None else tv_norm(xh, None if weights is None else w)
        resid = float(np.linalg.norm(yt - v3))
        res.objective.append(f)
        res.residual.append(resid)
        res.iterations = t
        if halting and halting_due(t, check_every, iters):
            if blocks is None:
                feasible = constraints_met([resid], [et], slack)
            else:
                feasible = constraints_met(
                    [np.linalg.norm(yt[a:b] - v3[a:b]) for a, b in zip(offsets[:-1], offsets[1:])], ets, slack)
            if halting_test(f_prev, f, feasible, xi):
                res.converged = True
                break
        f_prev = f
    res.x = xh
    return res
