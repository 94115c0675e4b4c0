"""The serving loop and plan creation under host sanitizers (no GPU).

server.cpp and plan.cpp are compiled with g++ together with tests/host_harness, which puts
host stand-ins in place of the HIP runtime and the solve, and runs a stream of mixed-size,
mixed-precision requests on eight worker slots.  ThreadSanitizer checks for unsynchronised
shared host state between the workers (and between the host threads that bin each plan's
visibilities); AddressSanitizer with UBSan checks buffer bounds and undefined behaviour in
the same code.  Every request's result must come back intact."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1406_0359_amd", "csrc")
HARNESS = os.path.join(ROOT, "tests", "host_harness", "server_plan_stub.cpp")
HIP_INCLUDE = "/opt/rocm/include"


@pytest.mark.parametrize("san", ["thread", "address,undefined"])
def test_server_and_plan_host_code_under_sanitizers(san, tmp_path):
    gxx = shutil.which("g++")
    if gxx is None or not os.path.isdir(HIP_INCLUDE):
        pytest.skip("needs g++ and the HIP headers")
    flags = ["-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=" + san,
             "-D__HIP_PLATFORM_AMD__", "-I" + HIP_INCLUDE, "-w"]
    exe = str(tmp_path / "harness")
    srcs = [os.path.join(CSRC, "plan.cpp"), os.path.join(CSRC, "server.cpp"), os.path.join(CSRC, "solver_rt.cpp"),
            HARNESS]
    r = subprocess.run([gxx, *flags, *srcs, "-o", exe, "-lpthread"], capture_output=True, text=True,
                       timeout=600)
    if r.returncode != 0 and any(lib in r.stderr for lib in ("libtsan", "libasan", "libubsan")):
        pytest.skip("sanitizer runtime not available: " + r.stderr[-300:])
    assert r.returncode == 0, r.stderr[-3000:]
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1 exitcode=66",
               ASAN_OPTIONS="detect_leaks=1 exitcode=66", UBSAN_OPTIONS="halt_on_error=1 print_stacktrace=1")
    r = subprocess.run([exe, "24", "8"], capture_output=True, text=True, timeout=600, env=env)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "Sanitizer" not in out and "runtime error" not in out, out[-4000:]
    assert "done 24 requests, 0 bad" in out
