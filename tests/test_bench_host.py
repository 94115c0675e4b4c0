"""Host logic of bench.py (no GPU): algorithmic byte counts, the dominant-kernel roofline entry,
and the lookup of committed counter summaries (a figure is reported only for the kernel source
it was measured on)."""
import os

import pytest

import bench


class _Plan:
    def __init__(self, n, M, q, precision):
        self.n, self.M, self.q, self.precision = n, M, q, precision


def test_stage_bytes_match_the_stated_accounting():
    # 256^2 FP64 SARA: G^T G reads and writes the K x K grid once and the packed coordinates once
    p = _Plan(256, 19661, 9, 0)
    N, c = 256 * 256, 16
    assert bench.stage_bytes(p, "gtg") == 4 * N * c + 19661 * 20 + 4 * N * c == 8781828
    # Phi = 104 N + 20 M in FP32 units, twice the values in FP64: (3 + 6 + 4) N c + M (20 + 16)
    assert bench.stage_bytes(p, "phi") == 13 * N * c + 19661 * (20 + 16)
    # 4096^2 FP32, M = 10^7: the column pass reads n x K and writes K x K complex64
    q = _Plan(4096, 10_000_000, 9, 1)
    assert bench.stage_bytes(q, "fft_cols") == 6 * 4096 * 4096 * 8 == 805306368
    assert bench.stage_bytes(q, "psi") == 10 * 4096 * 4096 * 8


def test_dominant_roofline_picks_the_largest_share():
    st = {k: {"ms": 0.1, "bytes": 1e9, "GBs": 1000.0, "frac": 0.125}
          for k in ["fft_rows", "fft_cols", "degrid", "grid", "gtg", "ifft_cols", "ifft_rows", "psi_adj", "psi"]}
    st["gtg"]["ms"] = 0.5          # 10 launches an iteration: share 5.0
    st["fft_cols"]["ms"] = 0.6     # 11 launches: share 6.6 -> dominant
    r = bench.dominant_roofline(st, 10, "no-such-workload")
    assert r["stage"] == "fft_cols" and r["kernel"] == "k_fft_cols_fwd"
    assert r["traffic"] is None
    assert r["bound"] == "hbm" and r["peak"] == 8000.0 and r["unit"] == "GB/s"
    # on FP32 grids from 2048^2 the G^T G stage is two launches, named as such
    st["gtg"]["ms"] = 0.7
    r = bench.dominant_roofline(st, 10, "sara4096")
    assert r["stage"] == "gtg" and r["kernel"].startswith("k_degrid_tiles + k_grid")


def test_counter_summaries_are_used_only_for_the_current_kernel_source(tmp_path, monkeypatch):
    src = tmp_path / "csrc"
    src.mkdir()
    (src / "nufft.hip").write_text("kernel source v1\n")
    (src / "fft.hip").write_text("another kernel source\n")
    import hashlib
    sha = hashlib.sha256(b"kernel source v1\n").hexdigest()
    prof = tmp_path / "profiles"
    prof.mkdir()
    (prof / "x_counters.md").write_text(f"stage: gtg\nworkload: w1\ntraffic_bytes_per_launch: 12345\n"
                                        f"kernel_source_sha256: `{sha}`\n")
    monkeypatch.setattr(bench, "CSRC", str(src))
    monkeypatch.setattr(bench, "PROFILES", str(prof))
    assert bench.measured_traffic("gtg", "w1") == 12345.0
    assert bench.measured_traffic("gtg", "w2") is None
    assert bench.measured_traffic("fft_cols", "w1") is None
    (src / "nufft.hip").write_text("kernel source v2\n")
    assert bench.measured_traffic("gtg", "w1") is None


def test_committed_summaries_name_their_stage_and_workload():
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    names = [f for f in os.listdir(os.path.join(root, "profiles")) if f.endswith("_counters.md")]
    assert names
    for f in names:
        text = open(os.path.join(root, "profiles", f)).read()
        for key in ("stage:", "workload:", "traffic_bytes_per_launch:", "kernel_source_sha256:"):
            assert key in text, (f, key)


def test_more_than_one_gpu_is_refused():
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(os.path.dirname(bench.__file__), "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr
