"""Seeded synthetic inputs shaped like the paper's experiments (Section 4).

The paper images the 256x256 30Dor field from continuous visibilities drawn from a
variable-density profile (denser at low spatial frequency), with the (0,0) Fourier
component suppressed and complex Gaussian noise at a fixed input SNR.  The field itself is
not available, so sums of Gaussian blobs stand in for it.

This module only draws random numbers and lays them out.  It contains none of the
method's arithmetic: the measurement operator is passed in by the caller wherever the
noise level needs ||Phi x||.  Both the CPU oracle tests and the GPU path use it.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Callable, Optional

import numpy as np

SEED_BASE = 14060359


@dataclass(frozen=True)
class Workload:
    """One problem size.  ``name`` is descriptive; sizes follow the paper's experiments."""
    name: str
    n: int                      # image side (N = n*n pixels)
    M: int                      # number of visibilities
    J: int = 6                  # Kaiser-Bessel support (taps per axis)
    dict_mask: int = 0x1FF      # bit0 Dirac, bit b = Daubechies-b
    levels: int = 4
    iters: int = 300
    cg_iters: int = 10
    blobs: int = 40
    uniform_frac: float = 0.0   # fraction of uv drawn uniformly instead of Gaussian
    isnr_db: float = 30.0
    index: int = 0              # seed slot
    precision: str = "fp64"
    diffuse: bool = False       # add a 1/f^2 Gaussian random field (large image)


# Sizes: 64^2 Db8 CPU case; 256^2 SARA FP64 case; 1024^2 SARA FP32 case (M = 2N, 10% uniform);
# 4096^2 large single solve (J = 8, 5 levels).
WORKLOADS = {
    "small64": Workload("small64", n=64, M=2048, J=6, dict_mask=1 << 8, levels=4, iters=200,
                        blobs=20, index=0),
    "sara256": Workload("sara256", n=256, M=19661, J=6, dict_mask=0x1FF, levels=4, iters=300,
                        blobs=40, index=1),
    "sara1024": Workload("sara1024", n=1024, M=2097152, J=6, dict_mask=0x1FF, levels=4,
                         iters=300, blobs=40, uniform_frac=209715 / 2097152, index=2,
                         precision="fp32"),
    "sara4096": Workload("sara4096", n=4096, M=10_000_000, J=8, dict_mask=0x1FF, levels=5,
                         iters=100, blobs=512, index=4, precision="fp32", diffuse=True),
}


def rng_for(index: int, stream: int) -> np.random.Generator:
    """Seeded generator: stream 0 image, 1 uv, 2 noise."""
    return np.random.default_rng(SEED_BASE + 100 * index + stream)


def blob_image(n: int, blobs: int, rng: np.random.Generator) -> np.ndarray:
    """Real nonnegative n x n image: sum of Gaussian blobs with uniform centres, widths
    1-6 px and lognormal(0, 1) amplitudes."""
    c = rng.uniform(0.0, n, size=(blobs, 2))
    s = rng.uniform(1.0, 6.0, size=blobs)
    a = rng.lognormal(0.0, 1.0, size=blobs)
    j = np.arange(n, dtype=np.float64)
    # separable blobs: sum_b a_b g0_b g1_b^T as one (n x blobs)(blobs x n) product
    g0 = np.exp(-((j[None, :] - c[:, 0:1]) ** 2) / (2 * s[:, None] ** 2))
    g1 = np.exp(-((j[None, :] - c[:, 1:2]) ** 2) / (2 * s[:, None] ** 2))
    return np.maximum((g0 * a[:, None]).T @ g1, 0.0)


def diffuse_field(n: int, rng: np.random.Generator, scale: float) -> np.ndarray:
    """1/f^2 Gaussian random field (power ~ 1/|k|^2, amplitude ~ 1/|k|), zero mean,
    standard deviation ``scale``."""
    w = rng.standard_normal((n, n))
    k = np.fft.fftfreq(n)
    kk = np.sqrt(k[:, None] ** 2 + k[None, :] ** 2)
    amp = np.zeros_like(kk)
    amp[kk > 0] = 1.0 / kk[kk > 0]
    f = np.real(np.fft.ifft2(np.fft.fft2(w) * amp))
    f -= f.mean()
    return f * (scale / f.std())


def uv_coverage(M: int, K: int, rng: np.random.Generator, uniform_frac: float = 0.0,
                sigma: float = math.pi / 4) -> np.ndarray:
    """M x 2 continuous frequencies in [-pi, pi)^2 (radians per pixel).

    Variable density: isotropic Gaussian (std ``sigma`` per axis) truncated to the square
    by rejection; optionally a fraction drawn uniformly.  A sample whose nearest node of the
    K x K oversampled grid is (0, 0) is rejected, which suppresses the zero frequency.
    """
    n_uni = int(round(M * uniform_frac))
    n_gau = M - n_uni
    out = []

    def draw(count, gen):
        got = np.empty((0, 2))
        while got.shape[0] < count:
            need = count - got.shape[0]
            cand = gen(int(need * 1.3) + 16)
            ok = np.all((cand >= -math.pi) & (cand < math.pi), axis=1)
            kap = cand * K / (2 * math.pi)
            ok &= ~np.all(np.abs(kap) < 0.5, axis=1)
            got = np.concatenate([got, cand[ok]])
        return got[:count]

    if n_gau:
        out.append(draw(n_gau, lambda m: rng.normal(0.0, sigma, size=(m, 2))))
    if n_uni:
        out.append(draw(n_uni, lambda m: rng.uniform(-math.pi, math.pi, size=(m, 2))))
    uv = np.concatenate(out) if len(out) > 1 else out[0]
    if n_uni and n_gau:
        uv = uv[rng.permutation(M)]
    return np.ascontiguousarray(uv, dtype=np.float64)


def unit_complex_noise(M: int, rng: np.random.Generator) -> np.ndarray:
    """(a + i b)/sqrt(2) with a, b ~ N(0, 1): unit-variance complex Gaussian draws."""
    return (rng.standard_normal(M) + 1j * rng.standard_normal(M)) / math.sqrt(2.0)


def chi2_epsilon(sigma: float, M: int) -> float:
    """l2 bound on complex noise of per-component variance sigma^2/2: mean plus two standard
    deviations of the chi-square law of ||n||^2 / (sigma^2 / 2) with 2M degrees of freedom."""
    return sigma * math.sqrt(M + 2.0 * math.sqrt(M))


@dataclass
class Problem:
    workload: Workload
    x_true: np.ndarray          # n x n real
    uv: np.ndarray              # M x 2 float64
    noise_unit: np.ndarray      # M complex, unit variance
    y: Optional[np.ndarray] = None
    sigma: float = 0.0
    epsilon: float = 0.0
    extra: dict = field(default_factory=dict)


def make_inputs(w: Workload, M: Optional[int] = None, n: Optional[int] = None) -> Problem:
    """Image, uv coverage and unit noise draws for a workload (optionally resized)."""
    n = n or w.n
    M = M or w.M
    K = 2 * n
    img = blob_image(n, w.blobs, rng_for(w.index, 0))
    if w.diffuse:
        r = rng_for(w.index, 0)
        amp = float(np.mean(r.lognormal(0.0, 1.0, size=w.blobs)))
        img = np.clip(img + diffuse_field(n, r, 0.1 * amp), 0.0, None)
    uv = uv_coverage(M, K, rng_for(w.index, 1), w.uniform_frac)
    nz = unit_complex_noise(M, rng_for(w.index, 2))
    return Problem(w, img, uv, nz)


def add_noise(p: Problem, y0: np.ndarray, isnr_db: Optional[float] = None) -> Problem:
    """y = y0 + sigma * noise with sigma = ||y0|| / sqrt(M) * 10^(-ISNR/20); epsilon from the
    chi-square bound.  ``y0`` is the noiseless visibility vector computed by the caller's
    measurement operator."""
    isnr = p.workload.isnr_db if isnr_db is None else isnr_db
    M = y0.shape[0]
    sigma = float(np.linalg.norm(y0)) / math.sqrt(M) * 10.0 ** (-isnr / 20.0)
    p.y = y0 + sigma * p.noise_unit
    p.sigma = sigma
    p.epsilon = chi2_epsilon(sigma, M)
    return p


def make_problem(w: Workload, phi: Callable[[np.ndarray, np.ndarray], np.ndarray],
                 M: Optional[int] = None, n: Optional[int] = None) -> Problem:
    """Full problem: ``phi(x_true, uv)`` must return the noiseless visibilities."""
    p = make_inputs(w, M=M, n=n)
    return add_noise(p, phi(p.x_true, p.uv))


def snr_db(x_true: np.ndarray, x_hat: np.ndarray) -> float:
    """Reconstruction SNR in dB: 20 log10(||x|| / ||x - Re x_hat||)."""
    x_true = np.asarray(x_true, dtype=np.float64)
    err = x_true - np.real(np.asarray(x_hat))
    return 20.0 * math.log10(np.linalg.norm(x_true) / np.linalg.norm(err))


# Serving stream: solves of mixed sizes in the ratio 8:4:2:1 (shuffled), M/N ~ U[0.2, 2] and
# input SNR ~ U[20, 40] dB per request, Poisson arrivals.
SERVING_SIZES = (128, 256, 512, 1024)
SERVING_MIX = (8, 4, 2, 1)
SERVING_INDEX = 3


def serving_counts(count: int) -> list:
    """Requests per size for a stream of ``count``: the 8:4:2:1 shares by largest remainder
    (512 -> 273/137/68/34)."""
    tot = sum(SERVING_MIX)
    exact = [count * m / tot for m in SERVING_MIX]
    per = [int(e) for e in exact]
    order = sorted(range(len(per)), key=lambda i: -(exact[i] - per[i]))
    for i in order[: count - sum(per)]:
        per[i] += 1
    return per


def serving_requests(count: int) -> list:
    """``count`` requests (Problem, noise not yet added: the caller's operator gives the
    noiseless visibilities; the request's ISNR is in ``extra['isnr_db']``)."""
    rng = rng_for(SERVING_INDEX, 0)
    sizes = np.repeat(np.array(SERVING_SIZES), serving_counts(count))
    rng.shuffle(sizes)
    out = []
    for i, n in enumerate(sizes.tolist()):
        r = np.random.default_rng(SEED_BASE + 100 * SERVING_INDEX + 10 + i)
        M = int(round(r.uniform(0.2, 2.0) * n * n))
        isnr = float(r.uniform(20.0, 40.0))
        w = Workload(f"serve{i}", n=n, M=M, J=6, dict_mask=0x1FF, levels=4, iters=300, blobs=40,
                     isnr_db=isnr, index=SERVING_INDEX, precision="fp32")
        img = blob_image(n, w.blobs, r)
        uv = uv_coverage(M, 2 * n, r, 0.0)
        nz = unit_complex_noise(M, r)
        out.append(Problem(w, img, uv, nz, extra={"isnr_db": isnr}))
    return out


BACKGROUND_INDEX = 5


def background_requests(count: int, n: int = 256) -> list:
    """``count`` requests of one size (the background stream beside the large single solve):
    M/N ~ U[0.2, 2], ISNR ~ U[20, 40] dB, SARA, as the serving stream; noise not yet added."""
    out = []
    for i in range(count):
        r = np.random.default_rng(SEED_BASE + 100 * BACKGROUND_INDEX + 10 + i)
        M = int(round(r.uniform(0.2, 2.0) * n * n))
        isnr = float(r.uniform(20.0, 40.0))
        w = Workload(f"bg{i}", n=n, M=M, J=6, dict_mask=0x1FF, levels=4, iters=300, blobs=40,
                     isnr_db=isnr, index=BACKGROUND_INDEX, precision="fp32")
        img = blob_image(n, w.blobs, r)
        uv = uv_coverage(M, 2 * n, r, 0.0)
        nz = unit_complex_noise(M, r)
        out.append(Problem(w, img, uv, nz, extra={"isnr_db": isnr}))
    return out


def poisson_arrivals(count: int, rate: float, index: int = SERVING_INDEX) -> np.ndarray:
    """Arrival times (seconds from the first) of a Poisson stream of ``rate`` per second."""
    gaps = rng_for(index, 1).exponential(1.0 / rate, size=count)
    gaps[0] = 0.0
    return np.cumsum(gaps)
