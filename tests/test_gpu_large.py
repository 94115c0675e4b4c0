"""Φ and Φ† at the large-image sizes, where the column passes keep several columns per
thread in registers (2n-point oversampled columns too long for more than one per workgroup
in LDS): n = 4096 in FP32 (the 4096^2 workload's shape, J = 6 and 8) and n = 2048 in FP64.

The oracle computes sampled outputs one by one (direct NUDFT sums at a few visibilities and
pixels); the NUFFT differs from the NUDFT by its approximation error (~1e-5 relative for
J = 6, far less for J = 8) plus FP32 rounding, so sampled values are held to 1e-4 of the
largest sampled magnitude.  The adjoint identity holds to rounding: 1e-5 (FP32), 1e-12
(FP64).

The whole outputs are also compared with the oracle's NUFFT, element by element, where its
sparse interpolation matrix fits in host memory: the 1024 x 1024 precision-form shape with its
full coverage (M = 2N = 2 097 152, 10% uniform) in FP32, n = 2048 in FP64 and n = 4096 with
J = 8 (10^6 visibilities) in FP32, each with the normal operator Phi^dagger Phi as well.  Bounds: FP64 relative l2 <= 1e-12 and element-wise
<= 1e-11 of the largest value; FP32 relative l2 and element-wise <= 1e-5."""
import numpy as np
import pytest

from gpu_cases import DEV, max_rel, rand_complex, rel_l2, to_np, uv_case
from oracle.nufft import Nufft, nudft, nudft_adjoint_at
from paper_1406_0359_amd import synth

torch = pytest.importorskip("torch")
from paper_1406_0359_amd import purify  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n,J,prec", [(4096, 6, "fp32"), (4096, 8, "fp32"), (2048, 6, "fp64")])
def test_large_phi_and_adjoint_sampled_against_nudft(n, J, prec):
    M = 20000
    uv = uv_case(M, n, 41 + J, 0.1)
    plan = purify.Plan(n, uv, J=J, dict_mask=0x100, levels=4, precision=prec, device=DEV)
    rng = np.random.default_rng(7)
    x = np.zeros((n, n))
    for _ in range(60):   # a few bright points and a smooth background keep |y| well spread
        x[rng.integers(0, n), rng.integers(0, n)] = rng.uniform(0.5, 2.0)
    x += 0.01
    y = to_np(plan.phi(plan.as_vec(x)))
    idx = rng.choice(M, 12, replace=False)
    ref = nudft(x, uv[idx])
    assert np.max(np.abs(y[idx] - ref)) < 1e-4 * np.max(np.abs(ref))
    v = rand_complex(M, 9)
    xa = to_np(plan.phi_adj(plan.as_vec(v)))
    pix = [(int(a), int(b)) for a, b in rng.integers(0, n, (12, 2))]
    refa = nudft_adjoint_at(v, uv, n, pix)
    got = np.array([xa[a, b] for a, b in pix])
    assert np.max(np.abs(got - refa)) < 1e-4 * np.max(np.abs(refa))
    lhs = np.vdot(y, v)
    rhs = np.vdot(x, xa)
    assert abs(lhs - rhs) < (1e-5 if prec == "fp32" else 1e-12) * abs(lhs)


@pytest.mark.parametrize("n,M,J,uf,prec", [
    (1024, 2097152, 6, 209715 / 2097152, "fp32"),   # the 1024^2 precision-form coverage
    (2048, 200000, 6, 0.1, "fp64"),
    (4096, 1000000, 8, 0.1, "fp32"),
])
def test_large_phi_and_adjoint_elementwise_against_oracle(n, M, J, uf, prec):
    uv = synth.uv_coverage(M, 2 * n, np.random.default_rng(500 + n), uf)
    op = Nufft(n, uv, J)
    plan = purify.Plan(n, uv, J=J, dict_mask=0x100, levels=4, precision=prec, device=DEV)
    x = rand_complex((n, n), 31)
    v = rand_complex(M, 32)
    ref_y = op.phi(x)
    got_y = to_np(plan.phi(plan.as_vec(x)))
    ref_x = op.phi_adj(v)
    got_x = to_np(plan.phi_adj(plan.as_vec(v)))
    # the normal operator as the CG update applies it (G^T G fused in one launch, or G then
    # G^T on FP32 grids from 2048^2) against the oracle's Phi^dagger (Phi x)
    ref_n = op.phi_adj(ref_y)
    got_n = to_np(plan.normal(plan.as_vec(x)))
    if prec == "fp64":
        assert rel_l2(got_y, ref_y) < 1e-12 and max_rel(got_y, ref_y) < 1e-11
        assert rel_l2(got_x, ref_x) < 1e-12 and max_rel(got_x, ref_x) < 1e-11
        assert rel_l2(got_n, ref_n) < 1e-12 and max_rel(got_n, ref_n) < 1e-11
    else:
        assert rel_l2(got_y, ref_y) < 1e-5 and max_rel(got_y, ref_y) < 1e-5
        assert rel_l2(got_x, ref_x) < 1e-5 and max_rel(got_x, ref_x) < 1e-5
        assert rel_l2(got_n, ref_n) < 1e-5 and max_rel(got_n, ref_n) < 1e-5
