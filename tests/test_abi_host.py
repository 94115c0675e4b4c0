"""Host-only checks of libpurify.so (no GPU needed): the library loads, exports every
function include/purify.h declares, validates plan descriptors, and its host-side math
(Daubechies spectral factorisation, Kaiser-Bessel series, deapodisation) agrees with the
oracle's independent implementations."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle.daubechies import daubechies_lowpass
from oracle.kaiser_bessel import deapodisation as oracle_deap
from oracle.kaiser_bessel import default_beta, kb_kernel as oracle_kb
from paper_1406_0359_amd import purify

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "purify.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(purify_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = purify.load_library()
    names = declared_functions()
    assert len(names) >= 15
    for name in names:
        assert hasattr(lib, name), name
    assert b"gfx950" in lib.purify_version()


@pytest.mark.parametrize("b", range(1, 9))
def test_library_filters_match_oracle(b):
    h = purify.daubechies_filter(b)
    ref = daubechies_lowpass(b)
    assert h.shape == ref.shape
    assert np.max(np.abs(h - ref)) < 2e-14


def test_library_filter_invariants_in_long_double():
    for b in range(1, 9):
        h = purify.daubechies_filter(b)
        assert abs(h.sum() - np.sqrt(2)) < 1e-15
        assert abs((h * h).sum() - 1) < 1e-15


@pytest.mark.parametrize("J", [2, 4, 5, 6, 8, 12, 16])
def test_library_kb_polynomials_match_oracle(J):
    # the kernels evaluate psi by per-tap polynomials in the fractional offset; the FP64
    # fit must agree with the Bessel-function definition to 1e-13 (psi(0) = 1)
    t = np.concatenate([np.linspace(-J / 2, J / 2, 4001)[:-1], [-J / 2, 0.0, 1e-12 - J / 2]])
    got = purify.kb_kernel(J, t)
    ref = oracle_kb(t, J, default_beta(J))
    assert np.max(np.abs(got - ref)) < 1e-13
    assert purify.kb_kernel(J, np.array([J / 2 + 1e-9, -J / 2 - 1e-9]))[0] == 0.0


@pytest.mark.parametrize("n,J", [(64, 6), (256, 6), (1024, 8)])
def test_library_deapodisation_matches_oracle(n, J):
    got = purify.deapodisation(n, 2 * n, J)
    ref = oracle_deap(n, 2 * n, J, default_beta(J))
    assert np.max(np.abs(got / ref - 1)) < 1e-13


def test_workspace_sizing_and_validation():
    ok = purify.workspace_bytes(256, 19661, 6, 0x1FF, 4, purify.FP64)
    assert ok > 0
    f32 = purify.workspace_bytes(256, 19661, 6, 0x1FF, 4, purify.FP32)
    assert 0 < f32 < ok
    assert purify.workspace_bytes(100, 100) == 0            # n not a power of two
    assert "power of two" in purify.last_error()
    assert purify.workspace_bytes(64, 100, J=17) == 0       # J out of range
    assert purify.workspace_bytes(64, 100, levels=7) == 0   # 64 not divisible by 2^7
    assert purify.workspace_bytes(64, 100, dict_mask=0) == 0
    assert purify.workspace_bytes(64, 0) == 0


def test_plan_create_rejects_small_workspace_without_touching_device():
    lib = purify.load_library()
    uv = np.zeros((10, 2))
    d = purify._desc(64, uv, 6, 0.0, 0x1FF, 4, purify.FP64)
    h = ctypes.c_void_p()
    st = lib.purify_plan_create(ctypes.byref(d), None, 0, None, ctypes.byref(h))
    assert st == 2 and not h.value
    st = lib.purify_plan_create(ctypes.byref(d), None, 1 << 40, None, None)
    assert st == 1
    assert lib.purify_status_string(2) == b"workspace too small or missing"


def test_binding_structs_match_the_c_header(tmp_path):
    # the ctypes mirrors of the C ABI's structs: same size and field offsets as the header
    import subprocess
    structs = {
        "purify_plan_desc": purify.PlanDesc, "purify_sdmm_params": purify.SdmmParams,
        "purify_sdmm_info": purify.SdmmInfo, "purify_server_desc": purify.ServerDesc,
        "purify_reweight_params": purify.ReweightParams, "purify_reweight_info": purify.ReweightInfo,
    }
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "purify.h"', 'int main(void) {']
    for cname, py in structs.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            lines.append(f'printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l}
    for cname, py in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for fname, _ in py._fields_:
            assert got[(cname, fname)] == getattr(py, fname).offset, (cname, fname)
