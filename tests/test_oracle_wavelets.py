"""Pins for the oracle's Daubechies filters, periodised DWT and SARA dictionary (Section 2.2).

* closed forms Db1 (Haar) and Db2;
* filter invariants: sum h = sqrt 2, double-shift orthonormality, N vanishing moments of
  the highpass, extremal (minimum) phase;
* a hand-computed one-level Haar transform of a 4x4 image;
* vanishing moments seen through the DWT: polynomial rows give zero interior details;
* orthonormality of each W_b, Psi Psi^dagger = I (tight frame, Section 3), adjoint identity.
"""
import math

import numpy as np
import pytest

from oracle.daubechies import daubechies_lowpass, highpass_from_lowpass
from oracle.sara import Sara, dwt2, dwt2_adjoint


def test_db1_db2_closed_forms():
    assert np.allclose(daubechies_lowpass(1), [1 / math.sqrt(2)] * 2, rtol=0, atol=1e-15)
    s3 = math.sqrt(3)
    ref = np.array([1 + s3, 3 + s3, 3 - s3, 1 - s3]) / (4 * math.sqrt(2))
    assert np.allclose(daubechies_lowpass(2), ref, rtol=0, atol=1e-15)


@pytest.mark.parametrize("N", range(1, 9))
def test_filter_invariants(N):
    h = daubechies_lowpass(N)
    g = highpass_from_lowpass(h)
    assert len(h) == 2 * N
    assert h.sum() == pytest.approx(math.sqrt(2), abs=1e-14)
    for m in range(N):
        dot = sum(h[k] * h[k + 2 * m] for k in range(2 * N - 2 * m))
        assert dot == pytest.approx(1.0 if m == 0 else 0.0, abs=5e-15)
        cross = sum(h[k] * g[k + 2 * m] for k in range(2 * N - 2 * m))
        assert cross == pytest.approx(0.0, abs=5e-15)
    k = np.arange(2 * N, dtype=np.float64)
    for j in range(N):
        mom = np.sum(g * k ** j) / max(1.0, np.sum(np.abs(g) * k ** j))
        assert abs(mom) < 1e-12
    # extremal phase: all zeros of H other than z = -1 lie inside the unit circle
    # (divide out the N-fold zero at z = -1 exactly first: roots of a multiple zero are
    # ill-conditioned)
    q = h.copy()
    for _ in range(N):
        q, rem = np.polydiv(q, [1.0, 1.0])
        assert np.max(np.abs(rem)) < 1e-12
    if len(q) > 1:
        assert np.all(np.abs(np.roots(q)) < 1.0)


def test_haar_one_level_by_hand():
    x = np.arange(16, dtype=float).reshape(4, 4)
    c = dwt2(x, daubechies_lowpass(1), 1)
    # axis 1 then axis 0, each [sum, difference]/sqrt2 of pairs (a[i] from x[2i], x[2i+1];
    # g = [h1, -h0] gives d = (x[2i] - x[2i+1])/sqrt2)
    ll = np.array([[x[0:2, 0:2].sum(), x[0:2, 2:4].sum()], [x[2:4, 0:2].sum(), x[2:4, 2:4].sum()]]) / 2
    assert np.allclose(c[:2, :2], ll)
    # horizontal detail (axis-1 high, axis-0 low): (x[., 2i] - x[., 2i+1]) summed over row pairs
    hd = np.array([[(x[0:2, 0] - x[0:2, 1]).sum(), (x[0:2, 2] - x[0:2, 3]).sum()],
                   [(x[2:4, 0] - x[2:4, 1]).sum(), (x[2:4, 2] - x[2:4, 3]).sum()]]) / 2
    assert np.allclose(c[:2, 2:], hd)
    vd = np.array([[(x[0, 0:2] - x[1, 0:2]).sum(), (x[0, 2:4] - x[1, 2:4]).sum()],
                   [(x[2, 0:2] - x[3, 0:2]).sum(), (x[2, 2:4] - x[3, 2:4]).sum()]]) / 2
    assert np.allclose(c[2:, :2], vd)


@pytest.mark.parametrize("N", [2, 4, 8])
def test_vanishing_moments_through_dwt(N):
    n = 64
    j = np.arange(n, dtype=float)
    x = np.tile(0.5 + 0.01 * j + (N > 2) * 1e-4 * j ** 2, (n, 1))   # rows are polynomials
    c = dwt2(x, daubechies_lowpass(N), 1)
    F = 2 * N
    interior = [i for i in range(n // 2) if 2 * i + F - 1 < n]      # taps do not wrap
    d = c[: n // 2, n // 2:][:, interior]
    assert np.max(np.abs(d)) < 1e-11


def test_constant_image_goes_to_coarsest_ll():
    n, L = 32, 3
    c = dwt2(np.full((n, n), 3.0), daubechies_lowpass(5), L)
    m = n >> L
    assert np.allclose(c[:m, :m], 3.0 * 2 ** L)
    c[:m, :m] = 0
    assert np.max(np.abs(c)) < 1e-12


@pytest.mark.parametrize("N,n,L", [(1, 16, 4), (3, 32, 2), (8, 64, 4), (8, 16, 3), (6, 8, 2)])
def test_dwt_orthonormal(N, n, L):
    rng = np.random.default_rng(N * 100 + n)
    x = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    h = daubechies_lowpass(N)
    c = dwt2(x, h, L)
    assert np.linalg.norm(c) == pytest.approx(np.linalg.norm(x), rel=1e-13)
    assert np.allclose(dwt2_adjoint(c, h, L), x, rtol=0, atol=1e-12)
    y = rng.standard_normal((n, n))
    assert np.vdot(c, y) == pytest.approx(np.vdot(x, dwt2_adjoint(y, h, L)), rel=1e-12)


@pytest.mark.parametrize("mask", [0x1FF, 1 << 8, 0x3, 0x101])
def test_sara_tight_frame(mask):
    n, L = 64, 4
    sa = Sara(n, mask, L)
    rng = np.random.default_rng(mask)
    x = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    a = sa.psi_adj(x)
    assert a.shape == (sa.q, n, n)
    assert np.allclose(sa.psi(a), x, rtol=0, atol=1e-12)
    assert np.linalg.norm(a) == pytest.approx(np.linalg.norm(x), rel=1e-13)
    b = rng.standard_normal(a.shape) + 1j * rng.standard_normal(a.shape)
    assert np.vdot(a, b) == pytest.approx(np.vdot(x, sa.psi(b)), rel=1e-12)


def test_sara_block_order_and_scale():
    n = 16
    sa = Sara(n, 0x1FF, 2)
    x = np.random.default_rng(0).standard_normal((n, n))
    a = sa.psi_adj(x)
    assert np.allclose(a[0], x / 3.0)
    assert np.allclose(a[8], dwt2(x, daubechies_lowpass(8), 2) / 3.0)
