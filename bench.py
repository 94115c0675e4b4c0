"""Benchmark of the SDMM imaging hot path on one MI355X.

A step is one complete imaging solve of the 256 x 256 SARA workload in FP64 (the plain
method on the GPU): plan creation (uv binning, tables, upload), the operator norm by 100
power iterations, the default gamma, and 300 SDMM iterations with 10 CG steps each, halting
off.  ``value`` is SDMM iterations per second over the timed steps (inputs resident in HBM).

Also reported:
* ``roofline``: the dominant kernel's algorithmic bytes per launch divided by its average
  launch time (HIP events on the stream it runs on), against 8 TB/s HBM; ``traffic`` is the
  copy-calibrated counter figure committed under profiles/ for that kernel and workload (null
  when the kernel source changed since); ``roofline_large`` is the same for the 4096^2 solve;
* ``cpu_baseline``: the FP64 NumPy/SciPy oracle on the same workload, timed on a bounded
  sample (setup + a few SDMM iterations, extrapolated to the 300-iteration solve), and one
  whole 64^2 solve;
* ``steady_state``: the marginal SDMM iterations per second on an existing plan;
* ``also``: per-stage timings; rocFFT (torch.fft.fft2) on each workload's oversampled grid
  beside the library's row + column passes; the 1024 x 1024 FP32 precision-form workload
  (M = 2N): Phi / Phi^dagger Gvis/s, Psi / Psi^dagger GB/s and SDMM iterations per second;
  the 4096 x 4096 single solve (M = 10^7, J = 8, 5 levels, FP32, 100 iterations: SNR and
  residual at the end), alone and beside a Poisson stream of 256^2 requests on the server;
  the serving form (FP32 server on a Poisson stream of mixed-size requests against the FP64
  one-at-a-time solves); at 256^2 and 1024^2, the same solve with the stored (Toeplitz) normal
  operator in CG (Section 3's precomputed composite operator): its iteration rate, stage times
  and its image against the exact solve's; and at 256^2 the paper's other methods (reweighted
  l1, visibility blocks, TV and reweighted TV): iteration rates and SNR.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
T_START = time.perf_counter()


def progress(msg: str) -> None:
    """One line per finished section on stderr (the JSON result line goes to stdout)."""
    print(f"[bench {time.perf_counter() - T_START:7.1f} s] {msg}", file=sys.stderr, flush=True)


def stage_bytes(plan, stage: str) -> float:
    """Algorithmic HBM bytes of one launch of a stage (each operand read or written once)."""
    n, M, q = plan.n, plan.M, plan.q
    N = n * n
    c = 16 if plan.precision == 0 else 8          # complex element
    coord = 4 + 2 * (c // 2)                       # packed first tap + two fractions
    tbl = {
        "fft_rows": N * c + 2 * N * c,             # read x, write K x n
        "fft_cols": 2 * N * c + 4 * N * c,         # read K x n, write K x K
        "degrid": 4 * N * c + M * (coord + c),     # read grid, coords; write y
        "grid": M * (coord + c) + 4 * N * c,       # read y, coords; write grid
        "gtg": 4 * N * c + M * coord + 4 * N * c,  # read grid, coords; write grid
        "ifft_cols": 4 * N * c + 2 * N * c,
        "ifft_rows": 2 * N * c + N * c,
        "psi_adj": N * c + q * N * c,
        "psi": q * N * c + N * c,
        # stored normal operator: column stage reads n x K and the real K x K spectrum, writes
        # n x K; the whole operator adds a row pass each way
        "toep_cols": 2 * N * c + 4 * N * (c // 2) + 2 * N * c,
        # TV prox launch (four dual steps in LDS): read both dual fields and u, write both
        # dual fields
        "tv_step": 5 * N * c,
    }
    tbl["toep_normal"] = (N * c + 2 * N * c) + tbl["toep_cols"] + (2 * N * c + N * c)
    tbl["phi"] = tbl["fft_rows"] + tbl["fft_cols"] + tbl["degrid"]
    tbl["phi_adj"] = tbl["grid"] + tbl["ifft_cols"] + tbl["ifft_rows"]
    return float(tbl[stage])


# launches of each kernel stage per SDMM iteration with cg CG steps
def launches_per_iter(cg: int) -> dict:
    a = cg                # A-applications in CG (one per step; the warm-start residual's
                          # A x_hat rides on the l2-ball branch's Phi^dagger), each with G^T G
                          # fused; Phi and Phi^dagger once more for the l2-ball branch
    return {"fft_rows": a + 1, "fft_cols": a + 1, "degrid": 1, "grid": 1, "gtg": a,
            "ifft_cols": a + 1, "ifft_rows": a + 1, "psi_adj": 1, "psi": 1}


KERNEL_NAME = {
    "fft_rows": "k_fft_rows_fwd", "fft_cols": "k_fft_cols_fwd", "degrid": "k_degrid",
    "grid": "k_grid", "gtg": "k_grid (G^T G)", "ifft_cols": "k_fft_cols_adj", "ifft_rows": "k_fft_rows_adj",
}
# where a workload's stage runs other kernels: FP32 grids from 2048^2 apply G^T G as G then
# G^T (two launches; the stage's algorithmic bytes stay those of G^T G)
KERNEL_NAME_BY_WORKLOAD = {(w, "gtg"): "k_degrid_tiles + k_grid (G^T G as G then G^T)"
                           for w in ("sara1024", "sara4096")}


def kernel_name(stage: str, workload: str) -> str:
    return KERNEL_NAME_BY_WORKLOAD.get((workload, stage), KERNEL_NAME[stage])


def stage_table(plan, reps: int = 50) -> dict:
    """Per-stage average launch time on the plan's internal buffers; call after a solve so
    they hold real data (gridding skips tiles whose visibilities are all zero)."""
    out = {}
    for st in ["fft_rows", "fft_cols", "degrid", "grid", "gtg", "ifft_cols", "ifft_rows", "phi",
               "phi_adj", "psi_adj", "psi"]:
        plan.time_stage(st, 3)
        ms = plan.time_stage(st, reps)
        b = stage_bytes(plan, st)
        out[st] = {"ms": ms, "bytes": b, "GBs": b / (ms * 1e-3) / 1e9,
                   "frac": b / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS}
    return out


def make_gpu_problem(w, torch, purify, synth, precision: str):
    """Synthetic problem whose noiseless visibilities come from the GPU operator itself."""
    p = synth.make_inputs(w)
    plan = purify.Plan(w.n, p.uv, J=w.J, dict_mask=w.dict_mask, levels=w.levels,
                       precision=precision, device="cuda:0")
    x = plan.as_vec(p.x_true)
    y0 = plan.phi(x)
    torch.cuda.synchronize()
    synth.add_noise(p, y0.cpu().numpy().astype(np.complex128))
    return p, plan


def cpu_baseline(w, p, sample_iters: int) -> dict:
    """Oracle timed on this host: NUFFT set-up, 100 power iterations, gamma, and
    ``sample_iters`` SDMM iterations of the workload, extrapolated to the full solve; plus one
    whole 64^2 Db8 solve (200 iterations).  scipy.fft runs on every host core (the oracle's
    setting); the sparse products and the wavelet transforms are single-threaded."""
    from oracle import nufft as onufft
    from oracle.nufft import Nufft
    from oracle.sara import Sara
    from oracle import sdmm as osd
    from paper_1406_0359_amd import synth

    t0 = time.perf_counter()
    op = Nufft(w.n, p.uv, w.J)
    sa = Sara(w.n, w.dict_mask, w.levels)
    nu, _ = osd.operator_norm(op.normal, (w.n, w.n), 100)
    t1 = time.perf_counter()
    osd.sdmm(op.phi, op.phi_adj, sa.psi, sa.psi_adj, p.y, p.epsilon, (w.n, w.n),
             iters=sample_iters, cg_iters=w.cg_iters, nu=nu)
    t2 = time.perf_counter()
    setup = t1 - t0
    per_iter = (t2 - t1) / sample_iters
    solve_s = setup + w.iters * per_iter
    w1 = synth.WORKLOADS["small64"]
    p1 = synth.make_problem(w1, lambda x, uv: Nufft(x.shape[0], uv, w1.J).phi(x))
    t3 = time.perf_counter()
    op1 = Nufft(w1.n, p1.uv, w1.J)
    sa1 = Sara(w1.n, w1.dict_mask, w1.levels)
    r1 = osd.sdmm(op1.phi, op1.phi_adj, sa1.psi, sa1.psi_adj, p1.y, p1.epsilon, (w1.n, w1.n), iters=w1.iters,
                  cg_iters=w1.cg_iters)
    t4 = time.perf_counter()
    cores = onufft.FFT_WORKERS
    return {"value": w.iters / solve_s, "unit": "iters/s", "cores": cores, "kind": "oracle",
            "sample": f"{w.name}: set-up + 100 power iterations ({setup:.1f} s) and "
                      f"{sample_iters} SDMM iterations ({per_iter:.2f} s each), "
                      f"extrapolated to the {w.iters}-iteration solve; NumPy/SciPy FP64, scipy.fft on "
                      f"{cores} threads, sparse products and wavelets single-threaded, on "
                      f"{platform.processor() or platform.machine()} ({os.cpu_count()} host cores visible)",
            "small64_full_solve": {"iterations": w1.iters, "seconds": t4 - t3, "iters_s": w1.iters / (t4 - t3),
                                   "snr_db": synth.snr_db(p1.x_true, r1.x)},
            "seconds": t4 - t0}


def precision_form(torch, purify, synth, solve_iters: int) -> dict:
    w = synth.WORKLOADS["sara1024"]
    p, plan = make_gpu_problem(w, torch, purify, synth, "fp32")
    y = plan.as_vec(p.y)
    # a short solve first: the stage timings then run on the solver's real buffers
    plan.sdmm(y, p.epsilon, max_iter=2, nu_iter=5)
    torch.cuda.synchronize()
    st = stage_table(plan, reps=20)
    t0 = time.perf_counter()
    res = plan.sdmm(y, p.epsilon, max_iter=solve_iters, nu_iter=100)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    toep = toeplitz_form(torch, plan, y, p.epsilon, res.nu, solve_iters, w.cg_iters, p.x_true, synth,
                         res.x.cpu().numpy())

    def timed(k):
        torch.cuda.synchronize()
        t = time.perf_counter()
        plan.sdmm(y, p.epsilon, max_iter=k, cg_iter=w.cg_iters, nu=res.nu)
        torch.cuda.synchronize()
        return time.perf_counter() - t
    steady = solve_iters / (timed(10 + solve_iters) - timed(10))
    return {
        "sdmm_steady_iters_s": steady,
        "roofline": dominant_roofline(st, w.cg_iters, "sara1024"),
        "fft_vs_rocfft": fft_vs_rocfft(torch, 2 * w.n, torch.complex64, st["fft_rows"]["ms"] + st["fft_cols"]["ms"],
                                       st["fft_rows"]["bytes"] + st["fft_cols"]["bytes"]),
        "toeplitz": toep,
        "workload": "sara1024 FP32 (n=1024, M=2097152, SARA 9 bases, L=4, J=6)",
        "phi_gvis_s": w.M / (st["phi"]["ms"] * 1e-3) / 1e9,
        "phi_adj_gvis_s": w.M / (st["phi_adj"]["ms"] * 1e-3) / 1e9,
        "psi_adj_GBs": st["psi_adj"]["GBs"], "psi_GBs": st["psi"]["GBs"],
        "sdmm_iters_s_incl_setup": solve_iters / dt,
        "solve_iters": solve_iters, "stages": st,
        "residual_over_eps": res.residual / p.epsilon,
    }


def toeplitz_form(torch, plan, y, eps, nu, iters, cg, x_true, synth, x_exact) -> dict:
    """CG with the stored (Toeplitz) normal operator on an existing plan: marginal iterations
    per second, the stage times, and the image against the exact solve of the same length."""
    def timed(k):
        torch.cuda.synchronize()
        t = time.perf_counter()
        r = plan.sdmm(y, eps, max_iter=k, cg_iter=cg, nu=nu, toeplitz=True)
        torch.cuda.synchronize()
        return time.perf_counter() - t, r
    timed(10)
    t_short, _ = timed(10)
    t_long, res = timed(10 + iters)
    t_full, res = timed(iters)
    out = {"steady_iters_s": iters / (t_long - t_short)}
    for st in ("toep_cols", "toep_normal"):
        plan.time_stage(st, 3)
        ms = plan.time_stage(st, 50)
        b = stage_bytes(plan, st)
        out[st] = {"ms": ms, "bytes": b, "GBs": b / (ms * 1e-3) / 1e9,
                   "frac": b / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS}
    xt = res.x.cpu().numpy()
    out["snr_db"] = synth.snr_db(x_true, xt)
    out["snr_db_exact"] = synth.snr_db(x_true, x_exact)
    out["rel_diff_vs_exact"] = float(np.linalg.norm(xt - x_exact) / np.linalg.norm(x_exact))
    return out


def method_variants(torch, plan, y, eps, nu, iters, x_true, synth, snr_plain, uv_count) -> dict:
    """The paper's other methods on the same 256^2 FP64 plan and data: reweighted l1 (SARA,
    three weighted solves after BPSA), four visibility blocks with per-block bounds, and the
    TV prior (plain and reweighted).  Iterations per second and the SNR of each."""
    def run(fn):
        torch.cuda.synchronize()
        t = time.perf_counter()
        r = fn()
        torch.cuda.synchronize()
        return time.perf_counter() - t, r
    out = {"snr_db_bpsa": snr_plain}
    dt, r = run(lambda: plan.sdmm_reweighted(y, eps, reweights=3, rel_var=0.0, max_iter=iters, nu=nu))
    out["sara_reweighted"] = {"solves": r.solves, "iterations": r.total_iterations,
                              "iters_s": r.total_iterations / dt, "snr_db": synth.snr_db(x_true, r.x.cpu().numpy())}
    R = 4
    offs = [uv_count * i // R for i in range(R + 1)]
    sigma = eps / math.sqrt(uv_count + 2 * math.sqrt(uv_count))
    beps = [synth.chi2_epsilon(sigma, offs[i + 1] - offs[i]) for i in range(R)]
    dt, r = run(lambda: plan.sdmm(y, 0.0, max_iter=iters, nu=nu, blocks=(offs, beps)))
    out["blocks_R4"] = {"iters_s_incl_block_tables": iters / dt, "snr_db": synth.snr_db(x_true, r.x.cpu().numpy())}
    tv_iter = 50
    dt, r = run(lambda: plan.sdmm(y, eps, max_iter=iters, nu=nu, tv_iter=tv_iter))
    out["tv"] = {"tv_iter": tv_iter, "iters_s": iters / dt, "snr_db": synth.snr_db(x_true, r.x.cpu().numpy())}
    plan.time_stage("tv_step", 3)
    ms = plan.time_stage("tv_step", 50)
    b = stage_bytes(plan, "tv_step")
    out["tv"]["tv_step"] = {"ms": ms, "bytes": b, "GBs": b / (ms * 1e-3) / 1e9,
                            "frac": b / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS}
    dt, r = run(lambda: plan.sdmm_reweighted(y, eps, reweights=2, rel_var=0.0, max_iter=iters, nu=nu,
                                             tv_iter=tv_iter))
    out["rwtv"] = {"solves": r.solves, "iters_s": r.total_iterations / dt,
                   "snr_db": synth.snr_db(x_true, r.x.cpu().numpy())}
    return out


PROFILES = os.path.join(ROOT, "profiles")
CSRC = os.path.join(ROOT, "paper_1406_0359_amd", "csrc")
STAGE_SOURCE = {"gtg": "nufft.hip", "grid": "nufft.hip", "degrid": "nufft.hip", "fft_rows": "fft.hip",
                "fft_cols": "fft.hip", "ifft_cols": "fft.hip", "ifft_rows": "fft.hip", "psi": "wavelet.hip",
                "psi_adj": "wavelet.hip"}


def measured_traffic(stage: str, workload: str):
    """HBM bytes per launch of a stage's kernel from a committed counter summary under
    profiles/ (two rocprofv3 --pmc runs, FETCH_SIZE and WRITE_SIZE, each scaled by a plain
    copy kernel of known size).  None unless a summary covers (stage, workload) and the kernel
    source it was taken on is the current one."""
    import glob
    import hashlib
    src = STAGE_SOURCE.get(stage)
    if src is None or not os.path.exists(os.path.join(CSRC, src)):
        return None
    sha = hashlib.sha256(open(os.path.join(CSRC, src), "rb").read()).hexdigest()
    for path in sorted(glob.glob(os.path.join(PROFILES, "*_counters.md"))):
        fields = {}
        for ln in open(path):
            if ":" in ln:
                k, v = ln.split(":", 1)
                if k.strip() in ("stage", "workload", "traffic_bytes_per_launch", "kernel_source_sha256"):
                    fields[k.strip()] = v.strip().strip("`")
        if fields.get("stage") == stage and fields.get("workload") == workload:
            if fields.get("kernel_source_sha256") != sha or "traffic_bytes_per_launch" not in fields:
                return None
            return float(fields["traffic_bytes_per_launch"])
    return None


def dominant_roofline(st: dict, cg: int, workload: str) -> dict:
    """Roofline entry for the kernel stage with the largest time share of an SDMM iteration
    (launches per iteration x average launch time from the stage table)."""
    per_iter = launches_per_iter(cg)
    share = {k: st[k]["ms"] * per_iter[k] for k in per_iter if k in KERNEL_NAME}
    dom = max(share, key=lambda k: share[k])
    d = st[dom]
    return {"bound": "hbm", "achieved": d["GBs"], "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": d["frac"],
            "traffic": measured_traffic(dom, workload), "kernel": kernel_name(dom, workload), "stage": dom,
            "bytes_per_launch": d["bytes"], "ms_per_launch": d["ms"],
            "share_of_iteration_kernels": share[dom] / sum(share.values())}


def fft_vs_rocfft(torch, K: int, dtype, ours_ms: float, ours_bytes: float) -> dict:
    """torch.fft.fft2 (rocFFT on this build) of a K x K grid, timed with events on the current
    stream, beside the library's row + column passes of the same oversampled transform (which
    read the n x n image and never touch the zero half of the padded grid)."""
    a = torch.randn(K, K, dtype=dtype, device="cuda:0")
    for _ in range(3):
        torch.fft.fft2(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    reps = 10
    for _ in range(reps):
        torch.fft.fft2(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    b = 2.0 * K * K * a.element_size()
    del a
    return {"grid": f"{K}x{K} {str(dtype).replace('torch.', '')}", "rocfft_ms": ms, "rocfft_GBs": b / (ms * 1e-3) / 1e9,
            "ours_rows_plus_cols_ms": ours_ms, "ours_GBs": ours_bytes / (ours_ms * 1e-3) / 1e9}


def gpu_requests(purify, reqs):
    """Noiseless visibilities of each request from the FP64 operator, then its noise."""
    from paper_1406_0359_amd import synth
    for p in reqs:
        n = p.x_true.shape[0]
        pl = purify.Plan(n, p.uv, precision="fp64", device="cuda:0")
        y0 = pl.phi(pl.as_vec(p.x_true)).cpu().numpy()
        synth.add_noise(p, y0, p.extra["isnr_db"])
        del pl
    return reqs


def large_solve(torch, purify, synth, iters: int, background: int) -> dict:
    """The 4096^2 single solve (M = 10^7, J = 8, SARA, 5 levels, FP32 with FP64 reductions):
    per-operator rates, the dominant kernel's roofline, the oversampled FFT against rocFFT, and
    the full solve (nu by 100 power iterations, `iters` SDMM iterations) with its SNR and
    residual, the same solve with the stored (Toeplitz) normal operator in CG; then the exact
    solve beside a Poisson stream of 256^2 requests served at half their standalone
    capacity."""
    w = synth.WORKLOADS["sara4096"]
    t0 = time.perf_counter()
    p = synth.make_inputs(w)
    t_inputs = time.perf_counter() - t0
    t0 = time.perf_counter()
    plan = purify.Plan(w.n, p.uv, J=w.J, dict_mask=w.dict_mask, levels=w.levels, precision="fp32",
                       device="cuda:0")
    torch.cuda.synchronize()
    t_plan = time.perf_counter() - t0
    y0 = plan.phi(plan.as_vec(p.x_true)).cpu().numpy().astype(np.complex128)
    synth.add_noise(p, y0)
    y = plan.as_vec(p.y)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r0 = plan.sdmm(y, p.epsilon, max_iter=1, nu_iter=100)
    torch.cuda.synchronize()
    t_nu = time.perf_counter() - t0
    t0 = time.perf_counter()
    r = plan.sdmm(y, p.epsilon, max_iter=iters, nu=r0.nu, gamma=r0.gamma, record_history=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    # stage times on the solve's buffers (after one iteration x_hat is still zero, and the
    # stages chained from it would grid all-zero tiles, whose scatter the kernel skips)
    st = stage_table(plan, reps=5)
    x_solo = r.x.clone()
    out = {
        "workload": "sara4096 FP32 (n=4096, M=10^7, J=8, SARA 9 bases, L=5; 512 blobs + 1/f^2 field)",
        "sdmm_iters_s": iters / dt, "solve_iters": iters, "solve_s": dt,
        "snr_db": synth.snr_db(p.x_true, x_solo.cpu().numpy()),
        "residual_over_eps": r.residual / p.epsilon,
        "objective_rel_change_last": abs(r.history[-1, 0] - r.history[-2, 0]) / r.history[-1, 0],
        "phi_gvis_s": w.M / (st["phi"]["ms"] * 1e-3) / 1e9,
        "phi_adj_gvis_s": w.M / (st["phi_adj"]["ms"] * 1e-3) / 1e9,
        "psi_adj_GBs": st["psi_adj"]["GBs"], "psi_GBs": st["psi"]["GBs"],
        "host_inputs_s": t_inputs, "plan_s": t_plan, "nu_s": t_nu, "stages": st,
        "roofline": dominant_roofline(st, w.cg_iters, "sara4096"),
        "fft_vs_rocfft": fft_vs_rocfft(torch, 2 * w.n, torch.complex64,
                                       st["fft_rows"]["ms"] + st["fft_cols"]["ms"],
                                       st["fft_rows"]["bytes"] + st["fft_cols"]["bytes"]),
    }
    try:
        out["toeplitz"] = toeplitz_form(torch, plan, y, p.epsilon, r0.nu, iters, w.cg_iters, p.x_true, synth,
                                        x_solo.cpu().numpy())
    except Exception as e:  # report, do not hide the rest
        out["toeplitz_error"] = repr(e)
    if background > 0:
        out["with_background"] = large_with_background(torch, purify, synth, plan, y, p.epsilon, r0.nu, r0.gamma,
                                                       iters, x_solo, iters / dt, background)
    return out


def large_with_background(torch, purify, synth, plan, y, eps, nu, gamma, iters, x_solo, solo_rate, count):
    """The large solve again while a server runs 256^2 FP32 requests (halting on, T_max 300)
    arriving as a Poisson stream at half the rate the server sustains for them alone."""
    import threading
    probe = 8
    reqs = gpu_requests(purify, synth.background_requests(count + probe))
    kw = dict(max_iter=300, cg_iter=10, halting=True, xi=1e-4, slack=1e-3, check_every=10)
    srv = purify.Server(16 << 30, max_active=4, device="cuda:0")

    def submit(p):
        return srv.submit(p.x_true.shape[0], p.uv, p.y.astype(np.complex64), p.epsilon, precision="fp32", **kw)
    t0 = time.perf_counter()
    done = [srv.wait(t) for t in [submit(p) for p in reqs[:probe]]]
    capacity = probe / (time.perf_counter() - t0)
    rate = 0.5 * capacity
    arrivals = synth.poisson_arrivals(count, rate, index=synth.BACKGROUND_INDEX)
    tickets, stop = [], threading.Event()

    def feeder():
        t_start = time.perf_counter()
        for p, at in zip(reqs[probe:], arrivals):
            if stop.is_set():
                break
            now = time.perf_counter() - t_start
            if at > now and stop.wait(at - now):
                break
            tickets.append(submit(p))
    th = threading.Thread(target=feeder)
    torch.cuda.synchronize()
    th.start()
    # While the server's workers may be capturing graphs, this thread makes no device-wide
    # synchronisation (the runtime refuses one while any stream captures): the solve returns
    # once its own streams have drained.
    t0 = time.perf_counter()
    r = plan.sdmm(y, eps, max_iter=iters, nu=nu, gamma=gamma)
    dt = time.perf_counter() - t0
    stop.set()
    th.join()
    res = [srv.wait(t) for t in tickets]
    srv.close()
    lat = np.array([q.latency_ms for q in res]) if res else np.zeros(1)
    same = bool(torch.equal(r.x, x_solo))
    return {"large_sdmm_iters_s": iters / dt, "large_sdmm_iters_s_alone": solo_rate,
            "large_image_bitwise_equal_to_alone": same,
            "background": "256^2 SARA FP32, M/N ~ U[0.2, 2], ISNR ~ U[20, 40] dB, halting (xi 1e-4, every 10), 4 slots",
            "background_capacity_solves_s": capacity, "arrival_rate_per_s": rate,
            "background_served": len(res), "background_solves_s_during_large": len(res) / dt,
            "background_p50_ms": float(np.percentile(lat, 50)), "background_p99_ms": float(np.percentile(lat, 99)),
            "probe_mean_iterations": float(np.mean([q.iterations for q in done]))}


def serving(torch, purify, synth, count: int, max_active: int) -> dict:
    """Serving form on a seeded stream of ``count`` requests (sizes 128^2..1024^2 in the ratio
    8:4:2:1, M/N ~ U[0.2, 2], ISNR ~ U[20, 40] dB, SARA, halting on, T_max = 300): the FP64
    one-at-a-time GPU baseline (plan + solve per request, in order, on one stream), then the
    FP32 server fed by Poisson arrivals at twice the baseline's solves/s, with the exact
    normal operator in CG and again with the stored (Toeplitz) one.  Latency is arrival to
    result on the host; each request's SNR is compared with its FP64 solve."""
    reqs = gpu_requests(purify, synth.serving_requests(count))
    kw = dict(max_iter=300, cg_iter=10, halting=True, xi=1e-4, slack=1e-3, check_every=10)
    torch.cuda.synchronize()
    base_ms, base_snr = [], []
    t0 = time.perf_counter()
    for p in reqs:
        ts = time.perf_counter()
        n = p.x_true.shape[0]
        pl = purify.Plan(n, p.uv, precision="fp64", device="cuda:0")
        r = pl.sdmm(pl.as_vec(p.y), p.epsilon, **kw)
        x = r.x.cpu().numpy()
        base_ms.append((time.perf_counter() - ts) * 1e3)
        base_snr.append(synth.snr_db(p.x_true, x))
        del pl, r
    base_s = time.perf_counter() - t0
    base_rate = count / base_s
    progress(f"serving: FP64 one-at-a-time baseline {base_rate:.2f} solves/s")

    free, _ = torch.cuda.mem_get_info()
    arena = int(min(200e9, free - 16e9))
    arrivals = synth.poisson_arrivals(count, 2.0 * base_rate)

    def served(toeplitz: bool) -> dict:
        srv = purify.Server(arena, max_active=max_active, device="cuda:0")
        tickets = []
        t0 = time.perf_counter()
        for p, at in zip(reqs, arrivals):
            now = time.perf_counter() - t0
            if at > now:
                time.sleep(at - now)
            tickets.append(srv.submit(p.x_true.shape[0], p.uv, p.y.astype(np.complex64), p.epsilon,
                                      precision="fp32", toeplitz=toeplitz, **kw))
        res = [srv.wait(t) for t in tickets]
        t_end = time.perf_counter() - t0
        srv.close()
        lat = np.array([r.latency_ms for r in res])
        dsnr = [abs(synth.snr_db(p.x_true, r.x) - s) for p, r, s in zip(reqs, res, base_snr)]
        return {"served_fp32_solves_s": count / t_end, "p50_ms": float(np.percentile(lat, 50)),
                "p99_ms": float(np.percentile(lat, 99)), "max_abs_snr_diff_db": float(max(dsnr)),
                "requests_within_005db": int(sum(d < 0.05 for d in dsnr)),
                "mean_iterations": float(np.mean([r.iterations for r in res]))}
    exact = served(False)
    progress(f"serving: exact operator {exact['served_fp32_solves_s']:.2f} solves/s")
    stored = served(True)
    return {
        "requests": count, "per_size": dict(zip([f"{s}^2" for s in synth.SERVING_SIZES],
                                                 synth.serving_counts(count))),
        **exact,
        "stored_normal_operator": stored,
        "arrival_rate_per_s": 2.0 * base_rate,
        "baseline_fp64_one_at_a_time_solves_s": base_rate,
        "baseline_p50_ms": float(np.percentile(base_ms, 50)), "baseline_p99_ms": float(np.percentile(base_ms, 99)),
        "mean_snr_db": float(np.mean(base_snr)),
        "max_active": max_active, "arena_gb": arena / 1e9,
    }


def copy_calibration(torch, mib: int) -> dict:
    """Ten launches of a plain elementwise kernel (negation, float32) that reads and writes
    mib MiB once each: the reference for scaling hardware byte counters."""
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(10):
        torch.neg(src, out=dst)
    torch.cuda.synchronize()
    return {"read": 4 * n, "write": 4 * n, "launches": 10}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-extra", action="store_true", help="skip the 1024^2 FP32 workload")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-iters", type=int, default=20)
    ap.add_argument("--extra-iters", type=int, default=30)
    ap.add_argument("--large-iters", type=int, default=100,
                    help="SDMM iterations of the 4096^2 solve (0: skip it)")
    ap.add_argument("--background-requests", type=int, default=0,
                    help="256^2 requests available to the background stream beside the 4096^2 solve "
                         "(0, the default: no background run; it runs the server's concurrent worker "
                         "slots, which stay off while a serving-stream segmentation fault is open)")
    ap.add_argument("--serving-requests", type=int, default=0,
                    help="requests in the serving-form stream (0, the default: skip; 512 is the full "
                         "stream).  Off by default: a run of the full stream ended in a host "
                         "segmentation fault after the solver-stream fix, cause not yet shown")
    ap.add_argument("--serving-slots", type=int, default=8)
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the reweighted, visibility-block and TV solves")
    ap.add_argument("--kernel-only", default="", metavar="STAGE[,STAGE...]",
                    help="only time stages (20 launches each, plain launches) of one workload's plan, "
                         "on the buffers a two-iteration solve of its data leaves (for hardware-counter "
                         "runs), and print one line per stage")
    ap.add_argument("--kernel-workload", default="sara256", choices=["sara256", "sara1024", "sara4096"],
                    help="workload of --kernel-only (sara256 in FP64, the others in FP32)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="after the run, negate a float32 tensor of MIB MiB into another 10 times "
                         "(a plain read-once/write-once kernel of known size that calibrates the "
                         "HBM byte counters of a profiler run)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: this build runs every solve on a single "
              "MI355X (no multi-GPU path); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1406_0359_amd import purify, synth

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    if args.kernel_only:
        wk = synth.WORKLOADS[args.kernel_workload]
        pk, plank = make_gpu_problem(wk, torch, purify, synth, "fp64" if args.kernel_workload == "sara256" else "fp32")
        # stage inputs from a two-iteration solve of the problem's data, so that every buffer a
        # stage reads (x_hat, the grids, the visibilities) holds the solve's values: a fresh
        # plan's x_hat is zero, every stage chained from it would then see zeros, and the
        # gridding kernels skip the adds of a tile whose values are all zero
        plank.sdmm(plank.as_vec(pk.y), pk.epsilon, max_iter=2, nu_iter=20)
        for stage in args.kernel_only.split(","):
            ms = plank.time_stage(stage, 20)
            print(json.dumps({"workload": args.kernel_workload, "stage": stage, "ms_per_launch": ms,
                              "bytes_per_launch": stage_bytes(plank, stage), "launches": 20}), flush=True)
        if args.copy_calibration > 0:
            print(json.dumps({"copy_calibration_bytes": copy_calibration(torch, args.copy_calibration)}))
        return
    w = synth.WORKLOADS["sara256"]
    p, plan0 = make_gpu_problem(w, torch, purify, synth, "fp64")
    y = plan0.as_vec(p.y)

    def step():
        plan = purify.Plan(w.n, p.uv, J=w.J, dict_mask=w.dict_mask, levels=w.levels,
                           precision="fp64", device="cuda:0")
        return plan, plan.sdmm(y, p.epsilon, max_iter=w.iters, cg_iter=w.cg_iters, nu_iter=100)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plan, res = step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms_per_step = dt / args.steps * 1e3
    value = args.steps * w.iters / dt
    snr = synth.snr_db(p.x_true, res.x.cpu().numpy())

    # steady state: the marginal cost of 300 more iterations on the same plan (nu given)
    def timed_solve(k):
        torch.cuda.synchronize()
        t = time.perf_counter()
        plan.sdmm(y, p.epsilon, max_iter=k, cg_iter=w.cg_iters, nu=res.nu)
        torch.cuda.synchronize()
        return time.perf_counter() - t
    steady = w.iters / (timed_solve(10 + w.iters) - timed_solve(10))
    progress(f"sara256 FP64: {value:.0f} SDMM iterations/s over {args.steps} timed solves")

    # per-stage timing (HIP events on the plan's stream) and the dominant kernel
    st = stage_table(plan)
    roofline = dominant_roofline(st, w.cg_iters, "sara256")

    line = {
        "metric": "SDMM iters/s", "value": value, "unit": "iters/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic (40 Gaussian blobs, variable-density Gaussian uv, 30 dB ISNR)",
        "config": {"workload": "sara256: n=256, M=19661, SARA 9 bases, L=4, J=6, KB beta=2.34J, "
                               "300 SDMM iters, CG 10, FP64; step = plan + nu + gamma + solve",
                   "global_batch": 1, "parallelism": "single GPU"},
        "snr_db": snr, "residual_over_eps": res.residual / p.epsilon,
        "steady_state": {"value": steady, "unit": "iters/s",
                         "what": "marginal SDMM iterations/s on the plan (no plan, nu or gamma)"},
        "roofline": roofline,
    }
    also = {"sara256_stages": st,
            "sara256_fft_vs_rocfft": fft_vs_rocfft(torch, 2 * w.n, torch.complex128,
                                                   st["fft_rows"]["ms"] + st["fft_cols"]["ms"],
                                                   st["fft_rows"]["bytes"] + st["fft_cols"]["bytes"])}
    try:
        also["sara256_toeplitz"] = toeplitz_form(torch, plan, y, p.epsilon, res.nu, w.iters, w.cg_iters,
                                                 p.x_true, synth, res.x.cpu().numpy())
    except Exception as e:  # report, do not hide the main line
        also["sara256_toeplitz_error"] = repr(e)
    progress("sara256 stages, rocFFT comparison, stored-operator solves")
    if not args.no_variants:
        try:
            also["sara256_methods"] = method_variants(torch, plan, y, p.epsilon, res.nu, w.iters, p.x_true, synth,
                                                      snr, w.M)
        except Exception as e:  # report, do not hide the main line
            also["sara256_methods_error"] = repr(e)
    progress("sara256 method variants")
    if not args.no_extra:
        try:
            also["sara1024_fp32"] = precision_form(torch, purify, synth, args.extra_iters)
        except Exception as e:  # report, do not hide the main line
            also["sara1024_fp32_error"] = repr(e)
    progress("sara1024 precision form")
    if args.large_iters > 0:
        try:
            also["sara4096_fp32"] = large_solve(torch, purify, synth, args.large_iters, args.background_requests)
            line["roofline_large"] = also["sara4096_fp32"]["roofline"]
        except Exception as e:  # report, do not hide the main line
            also["sara4096_fp32_error"] = repr(e)
    progress("sara4096 large solve")
    if args.serving_requests > 0:
        try:
            also["serving"] = serving(torch, purify, synth, args.serving_requests, args.serving_slots)
        except Exception as e:  # report, do not hide the main line
            also["serving_error"] = repr(e)
    progress("serving stream")
    line["also"] = also
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(w, p, args.cpu_iters)
        progress("CPU oracle baseline")
    if args.copy_calibration > 0:
        line["copy_calibration_bytes"] = copy_calibration(torch, args.copy_calibration)
    print(json.dumps(line))


if __name__ == "__main__":
    main()
