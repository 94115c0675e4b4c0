"""Every kernel writes inside the buffers it is given.

The plan's workspace and every caller vector sit between guard zones filled with a byte
pattern; after each group of calls (every stage on its own, the operators, solves with and
without graphs, the stored normal operator, the TV prior, visibility blocks, reweighting) the
guards must be unchanged.  An out-of-bounds write past the end (or before the start) of a
workspace or vector would land in a guard and fail here instead of corrupting a neighbouring
allocation or the runtime's own device memory.  Shapes: the 64^2 Db8 case with a ragged
visibility count, and the 256^2 (FP64), 1024^2 and 4096^2 (FP32) workloads."""
import numpy as np
import pytest

from gpu_cases import DEV
from paper_1406_0359_amd import synth

torch = pytest.importorskip("torch")
from paper_1406_0359_amd import purify  # noqa: E402

pytestmark = pytest.mark.gpu

PAT = 0xA5
WS_GUARD = 16 << 20
VEC_GUARD = 1 << 20


class Guarded:
    """A device region of ``nbytes`` between two guard zones of ``guard`` bytes."""

    def __init__(self, nbytes: int, guard: int):
        self.nbytes, self.guard = nbytes, guard
        self.buf = torch.full((nbytes + 2 * guard,), PAT, dtype=torch.uint8, device=DEV)
        self.inner = self.buf[guard:guard + nbytes]

    def vec(self, dtype, *shape):
        return self.inner.view(dtype).reshape(*shape)

    def intact(self) -> bool:
        torch.cuda.synchronize()
        g = self.guard
        return bool((self.buf[:g] == PAT).all()) and bool((self.buf[g + self.nbytes:] == PAT).all())


CASES = [
    ("small64", 2051, "fp64"),
    ("sara256", None, "fp64"),
    ("sara1024", None, "fp32"),
    ("sara4096", None, "fp32"),
]


@pytest.mark.parametrize("name,M,prec", CASES, ids=[c[0] for c in CASES])
def test_writes_stay_inside_workspace_and_vectors(name, M, prec):
    w = synth.WORKLOADS[name]
    p = synth.make_inputs(w, M=M)
    M = p.uv.shape[0]
    ws_bytes = purify.workspace_bytes(w.n, M, J=w.J, dict_mask=w.dict_mask, levels=w.levels,
                                      precision=purify.FP64 if prec == "fp64" else purify.FP32)
    ws = Guarded(ws_bytes, WS_GUARD)
    plan = purify.Plan(w.n, p.uv, J=w.J, dict_mask=w.dict_mask, levels=w.levels, precision=prec,
                       device=DEV, workspace=ws.inner)
    assert ws.intact(), "plan creation"
    cd = plan.cdtype
    es = 16 if cd == torch.complex128 else 8
    N, D = w.n * w.n, plan.D

    def gvec(count, *shape):
        g = Guarded(count * es, VEC_GUARD)
        return g, g.vec(cd, *shape)

    x = plan.as_vec(p.x_true)
    gy, y = gvec(M, M)
    plan.phi(x, out=y)
    gx, xa = gvec(N, w.n, w.n)
    plan.phi_adj(y, out=xa)
    ga, al = gvec(D, plan.q, w.n, w.n)
    plan.psi_adj(x, out=al)
    gs, xs = gvec(N, w.n, w.n)
    plan.psi(al, out=xs)
    gn, xn = gvec(N, w.n, w.n)
    plan.normal(x, out=xn)
    gt, xt = gvec(N, w.n, w.n)
    plan.normal(x, toeplitz=True, out=xt)
    for g, what in ((gy, "phi"), (gx, "phi_adj"), (ga, "psi_adj"), (gs, "psi"), (gn, "normal"),
                    (gt, "normal (stored operator)")):
        assert g.intact(), what
    assert ws.intact(), "operators"

    for st in purify.STAGES:
        plan.time_stage(st, 1)
        assert ws.intact(), f"stage {st}"

    synth.add_noise(p, y.cpu().numpy().astype(np.complex128))
    yv = plan.as_vec(p.y)
    small = w.n <= 256
    runs = [dict(graph=True), dict(graph=False), dict(toeplitz=True)]
    if small:
        runs += [dict(tv_iter=5), dict(blocks=([0, M // 3, M], [p.epsilon / 2, p.epsilon / 2]))]
    for kw in runs:
        go, xo = gvec(N, w.n, w.n)
        plan.sdmm(yv, p.epsilon, max_iter=3, nu_iter=5, cg_iter=3, out=xo, **kw)
        assert go.intact(), f"sdmm {kw}"
        assert ws.intact(), f"sdmm {kw}"
    if small:
        go, xo = gvec(N, w.n, w.n)
        plan.sdmm_reweighted(yv, p.epsilon, reweights=2, max_iter=3, nu_iter=5, cg_iter=3, out=xo)
        assert go.intact(), "reweighted"
        assert ws.intact(), "reweighted"
    del plan
    torch.cuda.synchronize()


def test_guard_detects_a_write_past_the_end():
    """The check itself: a write one element past a guarded vector is seen."""
    g = Guarded(1024, VEC_GUARD)
    g.buf[VEC_GUARD + 1024] = 0
    assert not g.intact()
