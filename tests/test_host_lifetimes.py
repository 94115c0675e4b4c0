"""The solver's HIP object lifetimes on the CPU (no GPU).

The library's host code (plan.cpp, api.cpp, solver_rt.cpp, server.cpp) is compiled with g++
beside tests/host_harness/solver_lifetimes.cpp, whose stand-ins for the HIP runtime track
every stream, event and graph, and beside kernel-launcher stubs generated here from the
declarations in common.h (each marks its stream busy, and records the event a launcher is
given, as the real one does).  Direct solves (graph and eager, reweighted, every stage timed, more solves, on three plans
created and destroyed one after another in FP64 and FP32) and a server stream of mixed
requests on eight worker slots then run the real solve sequence;
the run fails on any unsafe use: an event destroyed while a stream waits on it, a stream or a
launched graph destroyed with work pending, a call on a destroyed object, or two threads
capturing or instantiating graphs at once.  The same run under ThreadSanitizer checks the
host code of concurrent solves for data races."""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1406_0359_amd", "csrc")
HARNESS = os.path.join(ROOT, "tests", "host_harness", "solver_lifetimes.cpp")
HIP_INCLUDE = "/opt/rocm/include"

SPECIAL = {
    # the power iteration's norm and the largest coefficient feed nu and gamma on the host
    "launch_power_normalise": "sc[SL_LAMBDA] = 4.0;",
    "launch_finalize": "if (op == FIN_MAX) sc[slot] = 1.0;",
}


def _strip_defaults(params: str) -> str:
    return re.sub(r"\s*=\s*[^,()]+(?=[,)]|$)", "", params)


def launcher_stubs() -> str:
    """No-op definitions (and float/double instantiations) of every kernel launcher that
    common.h declares."""
    src = open(os.path.join(CSRC, "common.h")).read()
    src = re.sub(r"//[^\n]*", "", src)
    out = ['#include "common.h"', "void harness_kernel(hipStream_t s);", "namespace purify {"]
    pat = re.compile(r"(template\s*<typename T>\s*)?\b(void|int|bool)\s+(launch_\w+|fft_rows_adj_blocks|"
                     r"psi_adj_takes_xhat)\s*\(([^;{]*?)\)\s*;", re.S)
    seen = set()
    for m in pat.finditer(src):
        tmpl, ret, name, params = m.group(1), m.group(2), m.group(3), " ".join(m.group(4).split())
        if name in seen:
            continue
        seen.add(name)
        params = _strip_defaults(params)
        body = []
        sm = re.search(r"hipStream_t\s+(\w+)", params)
        if sm:
            body.append(f"harness_kernel({sm.group(1)});")
        for ev in re.findall(r"hipEvent_t\s+(\w+)", params):
            body.append(f"if ({ev}) (void)hipEventRecord({ev}, {sm.group(1)});")
        body.append(SPECIAL.get(name, ""))
        if name == "psi_adj_takes_xhat":
            body.append("return P.nwav > 0 && P.n < 1024;")
        elif ret != "void":
            body.append("return 1;")
        head = f"{tmpl or ''}{ret} {name}({params})"
        out.append(head + " { " + " ".join(b for b in body if b) + " }")
        if tmpl:
            for t in ("float", "double"):
                inst = re.sub(r"\bT\b", t, params)
                out.append(f"template {ret} {name}<{t}>({inst});")
    out.append("}  // namespace purify")
    assert len(seen) >= 40, sorted(seen)
    return "\n".join(out) + "\n"


def _build(tmp_path, extra):
    gxx = shutil.which("g++")
    if gxx is None or not os.path.isdir(HIP_INCLUDE):
        pytest.skip("needs g++ and the HIP headers")
    stubs = tmp_path / "launch_stubs.cpp"
    stubs.write_text(launcher_stubs())
    exe = str(tmp_path / "lifetimes")
    srcs = [os.path.join(CSRC, f) for f in ("plan.cpp", "api.cpp", "solver_rt.cpp", "server.cpp")]
    flags = ["-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-D__HIP_PLATFORM_AMD__",
             "-I" + HIP_INCLUDE, "-I" + CSRC, "-w", *extra]
    r = subprocess.run([gxx, *flags, *srcs, str(stubs), HARNESS, "-o", exe, "-lpthread"], capture_output=True,
                       text=True, timeout=900)
    if r.returncode != 0 and any(lib in r.stderr for lib in ("libtsan", "libasan", "libubsan")):
        pytest.skip("sanitizer runtime not available: " + r.stderr[-300:])
    assert r.returncode == 0, r.stderr[-3000:]
    return exe


@pytest.mark.parametrize("san", ["", "thread"])
def test_solver_object_lifetimes(san, tmp_path):
    exe = _build(tmp_path, ["-fsanitize=" + san] if san else [])
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1 exitcode=66")
    r = subprocess.run([exe, "32", "8"], capture_output=True, text=True, timeout=900, env=env)
    out = r.stdout + r.stderr
    assert "MISUSE" not in out, out[-4000:]
    assert "Sanitizer" not in out, out[-4000:]
    assert r.returncode == 0, out[-4000:]
    assert "done 32 requests, 0 bad, 0 misuses" in out
