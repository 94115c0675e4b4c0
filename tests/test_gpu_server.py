"""Serving form through the C ABI: mixed-size requests solved concurrently from one arena.

A served result must equal the same request solved alone (the kernels are deterministic and
solves share no state), whatever else runs beside it and whatever the arena budget forces
(serialised admission); an FP32 served solve must reconstruct within 0.05 dB of the FP64
solve of the same request.
"""
import numpy as np
import pytest

from gpu_cases import DEV
from oracle.nufft import Nufft
from paper_1406_0359_amd import synth

torch = pytest.importorskip("torch")
from paper_1406_0359_amd import purify  # noqa: E402

pytestmark = pytest.mark.gpu

# Concurrent worker slots (max_active >= 2) run solves' HIP work from several host threads at
# once.  With the solver streams created once per slot and graph building serialised, a server
# test run and two bench streams (30 and 512 requests) passed, and a later 512-request bench
# stream still ended in a host segmentation fault whose cause is not shown; the tests that run
# that path stay skipped until it is.
CONCURRENT_SKIP = pytest.mark.skip(reason="concurrent server workers: host segmentation fault in a bench "
                                          "serving stream, cause not yet shown")

PARAMS = dict(max_iter=40, cg_iter=10, halting=True, xi=1e-4, slack=1e-3, check_every=10, nu_iter=50)


def _request(n, M, seed):
    w = synth.WORKLOADS["small64"]
    p = synth.make_inputs(w, M=M, n=n)
    rng = np.random.default_rng(1000 + seed)
    # a different coverage and noise draw per request
    p.uv = synth.uv_coverage(M, 2 * n, rng, 0.0)
    return synth.add_noise(p, Nufft(n, p.uv, w.J).phi(p.x_true))


def _alone(p, n, precision):
    plan = purify.Plan(n, p.uv, J=6, dict_mask=purify.DICT_SARA, levels=3, precision=precision, device=DEV)
    r = plan.sdmm(plan.as_vec(p.y), p.epsilon, **PARAMS)
    return r.x.cpu().numpy(), r


def _submit(srv, p, n, precision):
    return srv.submit(n, p.uv, p.y, p.epsilon, dict_mask=purify.DICT_SARA, levels=3, precision=precision,
                      **PARAMS)


@CONCURRENT_SKIP
def test_served_results_equal_solo_results_in_a_mix():
    reqs = [(64, 1200, 0, "fp32"), (128, 3000, 1, "fp32"), (64, 2500, 2, "fp64"), (128, 6000, 3, "fp32"),
            (32, 400, 4, "fp32"), (64, 800, 5, "fp64")]
    probs = [_request(n, M, s) for n, M, s, _ in reqs]
    srv = purify.Server(512 << 20, max_active=3, device=DEV)
    tickets = [_submit(srv, p, n, prec) for p, (n, _, _, prec) in zip(probs, reqs)]
    served = [srv.wait(t) for t in tickets]
    srv.close()
    for p, (n, _, _, prec), s in zip(probs, reqs, served):
        x, r = _alone(p, n, prec)
        assert s.iterations == r.iterations
        assert np.array_equal(s.x, x)
        assert s.latency_ms >= s.run_ms > 0


@CONCURRENT_SKIP
def test_small_arena_serialises_admission_with_the_same_results():
    reqs = [(64, 1500, 10), (64, 1800, 11), (64, 1200, 12)]
    probs = [_request(n, M, s) for n, M, s in reqs]
    need = max(purify.workspace_bytes(n, M, levels=3, precision=purify.FP32) for n, M, _ in reqs)
    srv = purify.Server(need + (8 << 20), max_active=3, device=DEV)   # room for one at a time
    tickets = [_submit(srv, p, n, "fp32") for p, (n, _, _) in zip(probs, reqs)]
    served = [srv.wait(t) for t in tickets]
    srv.close()
    for p, (n, _, _), s in zip(probs, reqs, served):
        x, _ = _alone(p, n, "fp32")
        assert np.array_equal(s.x, x)
    # one request at a time: the later ones waited for the earlier ones' blocks
    assert served[2].queue_ms > 0.0


def test_oversized_request_is_rejected():
    p = _request(64, 1000, 20)
    srv = purify.Server(1 << 20, max_active=1, device=DEV)
    with pytest.raises(purify.PurifyError):
        _submit(srv, p, 64, "fp32")
    srv.close()


@CONCURRENT_SKIP
def test_served_fp32_snr_within_005db_of_fp64_solve():
    p = _request(128, 5000, 30)
    srv = purify.Server(256 << 20, max_active=2, device=DEV)
    t32 = srv.submit(128, p.uv, p.y, p.epsilon, levels=3, precision="fp32", max_iter=300, halting=True,
                     check_every=10)
    t64 = srv.submit(128, p.uv, p.y, p.epsilon, levels=3, precision="fp64", max_iter=300, halting=True,
                     check_every=10)
    s32, s64 = srv.wait(t32), srv.wait(t64)
    srv.close()
    assert abs(synth.snr_db(p.x_true, s32.x) - synth.snr_db(p.x_true, s64.x)) < 0.05


@CONCURRENT_SKIP
def test_served_stored_operator_solve_equals_solo():
    # the stored (Toeplitz) normal operator in the served CG: its spectrum is built inside the
    # worker's solve, and the result equals the same request solved alone
    p = _request(64, 1500, 40)
    srv = purify.Server(256 << 20, max_active=2, device=DEV)
    kw = dict(dict_mask=purify.DICT_SARA, levels=3, precision="fp32", **PARAMS)
    t1 = srv.submit(64, p.uv, p.y, p.epsilon, toeplitz=True, **kw)
    t2 = srv.submit(64, p.uv, p.y, p.epsilon, **kw)
    s1, s2 = srv.wait(t1), srv.wait(t2)
    srv.close()
    plan = purify.Plan(64, p.uv, J=6, dict_mask=purify.DICT_SARA, levels=3, precision="fp32", device=DEV)
    r = plan.sdmm(plan.as_vec(p.y), p.epsilon, toeplitz=True, **PARAMS)
    assert s1.iterations == r.iterations
    assert np.array_equal(s1.x, r.x.cpu().numpy())
    assert abs(synth.snr_db(p.x_true, s1.x) - synth.snr_db(p.x_true, s2.x)) < 0.05
