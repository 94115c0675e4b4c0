"""Kaiser-Bessel interpolation kernel (oracle, FP64).

The paper's measurement operator is a non-uniform FFT (Section 4, citing Greengard & Lee
and the companion paper for details).  Its interpolation kernel is Kaiser-Bessel with J
taps per axis on a 2x oversampled grid and shape beta = 2.34 J.

    psi(t)      = I0(beta sqrt(1 - (2t/J)^2)) / I0(beta)            for |t| <= J/2, else 0
    psi_hat(nu) = J sinh(sqrt(beta^2 - (pi J nu)^2))
                  / (sqrt(beta^2 - (pi J nu)^2) I0(beta))              (continuous FT)

The deapodisation (the S of Phi = G F Z S) divides by psi_hat at each pixel's frequency.
"""
import numpy as np
from scipy import special


def default_beta(J: int) -> float:
    return 2.34 * J


def kb_kernel(t, J: int, beta: float):
    """psi(t) in grid units; zero outside |t| <= J/2."""
    t = np.asarray(t, dtype=np.float64)
    arg = 1.0 - (2.0 * t / J) ** 2
    inside = arg >= 0.0
    out = np.zeros_like(t)
    out[inside] = special.i0(beta * np.sqrt(arg[inside])) / special.i0(beta)
    return out


def kb_ft(nu, J: int, beta: float):
    """Continuous Fourier transform of psi at frequency nu (cycles per grid unit)."""
    nu = np.asarray(nu, dtype=np.float64)
    z2 = beta ** 2 - (np.pi * J * nu) ** 2
    out = np.empty_like(nu)
    pos = z2 > 0
    z = np.sqrt(z2[pos])
    out[pos] = J * np.sinh(z) / z
    zn = np.sqrt(-z2[~pos])
    # sinh(i z)/(i z) = sin z / z; z = 0 limit is 1.
    with np.errstate(invalid="ignore", divide="ignore"):
        out[~pos] = np.where(zn > 0, J * np.sin(zn) / np.where(zn > 0, zn, 1.0), J)
    return out / special.i0(beta)


def deapodisation(n: int, K: int, J: int, beta: float) -> np.ndarray:
    """1D deapodisation factors s_j = 1 / psi_hat(p / K), p = j - n/2 (pixel centring).
    The 2D factor is the outer product s_j1 * s_j2."""
    p = np.arange(n, dtype=np.float64) - n // 2
    return 1.0 / kb_ft(p / K, J, beta)
