"""ctypes binding over libpurify.so (the C ABI declared in include/purify.h).

This module only marshals arguments: every step of Phi, Phi^dagger, Psi, Psi^dagger and
SDMM runs in the library's HIP kernels.  PyTorch supplies device memory (the plan workspace
and the vectors) and the current HIP stream.  If the library is missing the first call
raises; there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "lib", "libpurify.so")

FP64, FP32 = 0, 1
DICT_SARA = 0x1FF
SDMM_NO_GRAPH = 1
SDMM_WARM_START = 2
SDMM_TOEPLITZ = 4
SDMM_TV = 8
NORMAL_TOEPLITZ = 1

STAGES = {
    "fft_rows": 0, "fft_cols": 1, "degrid": 2, "grid": 3, "ifft_cols": 4, "ifft_rows": 5,
    "phi": 6, "phi_adj": 7, "psi_adj": 8, "psi": 9, "gtg": 10, "toep_cols": 11, "toep_normal": 12, "tv_step": 13,
}

_STATUS = {0: "ok", 1: "invalid argument", 2: "workspace", 3: "device error", 4: "non-finite"}


class PurifyError(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__(f"{what}: {_STATUS.get(status, status)} ({last_error()})")
        self.status = status


class PlanDesc(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int32), ("oversample", ctypes.c_int32), ("J", ctypes.c_int32),
        ("beta", ctypes.c_double), ("M", ctypes.c_int64), ("uv", ctypes.POINTER(ctypes.c_double)),
        ("dict_mask", ctypes.c_uint32), ("levels", ctypes.c_int32), ("precision", ctypes.c_int32),
    ]


class SdmmParams(ctypes.Structure):
    _fields_ = [
        ("epsilon", ctypes.c_double), ("gamma", ctypes.c_double), ("nu", ctypes.c_double),
        ("xi", ctypes.c_double), ("slack", ctypes.c_double),
        ("max_iter", ctypes.c_int32), ("cg_iter", ctypes.c_int32), ("check_every", ctypes.c_int32),
        ("halting", ctypes.c_int32), ("nu_iter", ctypes.c_int32), ("flags", ctypes.c_int32),
        ("weights", ctypes.c_void_p), ("history", ctypes.POINTER(ctypes.c_double)),
        ("nblocks", ctypes.c_int32), ("block_offsets", ctypes.POINTER(ctypes.c_int64)),
        ("block_eps", ctypes.POINTER(ctypes.c_double)), ("tv_iter", ctypes.c_int32),
    ]


class SdmmInfo(ctypes.Structure):
    _fields_ = [
        ("iterations", ctypes.c_int32), ("converged", ctypes.c_int32),
        ("objective", ctypes.c_double), ("residual", ctypes.c_double),
        ("nu", ctypes.c_double), ("gamma", ctypes.c_double),
    ]


class ReweightParams(ctypes.Structure):
    _fields_ = [
        ("delta0", ctypes.c_double), ("decay", ctypes.c_double), ("delta_min", ctypes.c_double),
        ("rel_var", ctypes.c_double), ("reweights", ctypes.c_int32),
    ]


class ReweightInfo(ctypes.Structure):
    _fields_ = [
        ("solves", ctypes.c_int32), ("total_iterations", ctypes.c_int32),
        ("delta", ctypes.c_double), ("rel_var", ctypes.c_double),
    ]


class ServerDesc(ctypes.Structure):
    _fields_ = [("arena", ctypes.c_void_p), ("arena_bytes", ctypes.c_size_t), ("max_active", ctypes.c_int32)]


_lib = None


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libpurify.so (raises OSError if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise OSError(f"libpurify.so not found at {path}; run paper_1406_0359_amd.build")
    lib = ctypes.CDLL(path)
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    pdesc = ctypes.POINTER(PlanDesc)
    sig = {
        "purify_plan_workspace_bytes": (ctypes.c_size_t, [pdesc]),
        "purify_plan_dict_size": (i64, [pdesc]),
        "purify_plan_create": (i32, [pdesc, vp, ctypes.c_size_t, vp, ctypes.POINTER(vp)]),
        "purify_plan_destroy": (None, [vp]),
        "purify_phi": (i32, [vp, vp, vp, vp]),
        "purify_phi_noalloc": (i32, [vp, vp, vp, vp]),
        "purify_phi_adj": (i32, [vp, vp, vp, vp]),
        "purify_psi": (i32, [vp, vp, vp, vp]),
        "purify_psi_adj": (i32, [vp, vp, vp, vp]),
        "purify_sdmm_solve": (i32, [vp, vp, ctypes.POINTER(SdmmParams), vp,
                                    ctypes.POINTER(SdmmInfo), vp]),
        "purify_sdmm_reweighted": (i32, [vp, vp, ctypes.POINTER(SdmmParams), ctypes.POINTER(ReweightParams),
                                         vp, vp, ctypes.POINTER(SdmmInfo), ctypes.POINTER(ReweightInfo), vp]),
        "purify_phi_normal": (i32, [vp, vp, vp, i32, vp]),
        "purify_time_stage": (i32, [vp, i32, i32, vp, ctypes.POINTER(dbl)]),
        "purify_daubechies_filter": (i32, [i32, ctypes.POINTER(dbl), i32]),
        "purify_kb_kernel": (i32, [i32, dbl, i32, ctypes.POINTER(dbl), ctypes.POINTER(dbl)]),
        "purify_deapodisation": (i32, [i32, i32, i32, dbl, ctypes.POINTER(dbl)]),
        "purify_server_create": (i32, [ctypes.POINTER(ServerDesc), ctypes.POINTER(vp)]),
        "purify_server_submit": (i32, [vp, pdesc, vp, ctypes.POINTER(SdmmParams), ctypes.POINTER(i64)]),
        "purify_server_poll": (i32, [vp, i64]),
        "purify_server_wait": (i32, [vp, i64, vp, ctypes.POINTER(SdmmInfo), ctypes.POINTER(dbl)]),
        "purify_server_destroy": (None, [vp]),
        "purify_status_string": (ctypes.c_char_p, [i32]),
        "purify_last_error": (ctypes.c_char_p, []),
        "purify_version": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def last_error() -> str:
    if _lib is None:
        return ""
    return _lib.purify_last_error().decode()


def _check(status: int, what: str):
    if status != 0:
        raise PurifyError(status, what)


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


# --- host-only queries -------------------------------------------------------------------
def daubechies_filter(b: int) -> np.ndarray:
    lib = load_library()
    h = np.zeros(16)
    F = lib.purify_daubechies_filter(b, _dptr(h), 16)
    if F < 0:
        raise ValueError("b must be in 1..8")
    return h[:F].copy()


def kb_kernel(J: int, t, beta: float = 0.0) -> np.ndarray:
    lib = load_library()
    t = np.ascontiguousarray(t, dtype=np.float64).ravel()
    out = np.zeros_like(t)
    if lib.purify_kb_kernel(J, beta, t.size, _dptr(t), _dptr(out)) < 0:
        raise ValueError("bad kb arguments")
    return out


def deapodisation(n: int, K: int, J: int, beta: float = 0.0) -> np.ndarray:
    lib = load_library()
    out = np.zeros(n)
    if lib.purify_deapodisation(n, K, J, beta, _dptr(out)) < 0:
        raise ValueError("bad deapodisation arguments")
    return out


def _desc(n, uv, J, beta, dict_mask, levels, precision):
    d = PlanDesc()
    d.n, d.oversample, d.J, d.beta = n, 2, J, beta
    d.M = uv.shape[0]
    d.uv = _dptr(uv)
    d.dict_mask, d.levels, d.precision = dict_mask, levels, precision
    return d


def workspace_bytes(n: int, M: int, J: int = 6, dict_mask: int = DICT_SARA, levels: int = 4,
                    precision: int = FP64) -> int:
    lib = load_library()
    uv = np.zeros((1, 2))
    d = _desc(n, uv, J, 0.0, dict_mask, levels, precision)
    d.M = M
    return int(lib.purify_plan_workspace_bytes(ctypes.byref(d)))


@dataclass
class SolveResult:
    x: "object"                  # torch complex tensor (n, n); the image is x.real
    iterations: int
    converged: bool
    objective: float
    residual: float
    nu: float
    gamma: float
    history: Optional[np.ndarray]


@dataclass
class ReweightResult:
    x: "object"                  # torch complex tensor (n, n): the last solve's x_hat
    weights: "object"            # torch float64 (D,): the last weighted solve's weights
    solves: int                  # SDMM solves, solve 0 included
    total_iterations: int
    delta: float                 # delta of the last weighted solve
    rel_var: float               # relative variation after it (-1 if none ran)
    last: SolveResult            # info of the last solve


class Plan:
    """A measurement operator / dictionary / solver plan on one GPU.

    ``uv`` is an (M, 2) float64 host array of frequencies in radians per pixel.  The plan's
    workspace is a torch uint8 tensor on ``device`` (allocated here, or the caller's
    ``workspace`` of at least ``purify_plan_workspace_bytes``); vectors are torch complex
    tensors of the plan's precision (complex128 for fp64, complex64 for fp32) on the same
    device.
    """

    def __init__(self, n: int, uv, J: int = 6, beta: float = 0.0, dict_mask: int = DICT_SARA,
                 levels: int = 4, precision: str = "fp64", device="cuda:0", workspace=None):
        import torch
        self.lib = load_library()
        self.torch = torch
        self.device = torch.device(device)
        self.n, self.J, self.levels, self.dict_mask = n, J, levels, dict_mask
        self.precision = FP64 if precision in ("fp64", FP64) else FP32
        self.cdtype = torch.complex128 if self.precision == FP64 else torch.complex64
        self.uv = np.ascontiguousarray(uv, dtype=np.float64).reshape(-1, 2)
        self.M = self.uv.shape[0]
        d = _desc(n, self.uv, J, beta, dict_mask, levels, self.precision)
        self.ws_bytes = int(self.lib.purify_plan_workspace_bytes(ctypes.byref(d)))
        if self.ws_bytes == 0:
            raise PurifyError(1, "purify_plan_workspace_bytes")
        self.D = int(self.lib.purify_plan_dict_size(ctypes.byref(d)))
        self.q = self.D // (n * n)
        if workspace is None:
            workspace = torch.empty(self.ws_bytes, dtype=torch.uint8, device=self.device)
        elif (not isinstance(workspace, torch.Tensor) or workspace.device != self.device
              or workspace.dtype != torch.uint8 or not workspace.is_contiguous()
              or workspace.numel() < self.ws_bytes or workspace.data_ptr() % 256):
            raise ValueError(f"workspace must be a contiguous, 256-byte aligned uint8 tensor on "
                             f"{self.device} of at least {self.ws_bytes} bytes")
        self.workspace = workspace
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _check(self.lib.purify_plan_create(ctypes.byref(d), self.workspace.data_ptr(),
                                               self.ws_bytes, self._stream(), ctypes.byref(h)),
                   "purify_plan_create")
        self.handle = h

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value:
            self.lib.purify_plan_destroy(h)
            self.handle = None

    # --- helpers ------------------------------------------------------------------------
    def _stream(self):
        return self.torch.cuda.current_stream(self.device).cuda_stream

    def _vec(self, t, count: int, name: str):
        if not isinstance(t, self.torch.Tensor) or t.device != self.device:
            raise ValueError(f"{name} must be a torch tensor on {self.device}")
        if t.dtype != self.cdtype or not t.is_contiguous() or t.numel() != count:
            raise ValueError(f"{name} must be contiguous {self.cdtype} with {count} elements")
        return t.data_ptr()

    def empty(self, *shape):
        return self.torch.empty(*shape, dtype=self.cdtype, device=self.device)

    def as_vec(self, a):
        """Copy host data (numpy / torch) to a contiguous device vector of the plan's type."""
        t = self.torch.as_tensor(np.asarray(a)) if not isinstance(a, self.torch.Tensor) else a
        return t.to(device=self.device, dtype=self.cdtype).contiguous()

    # --- operators ----------------------------------------------------------------------
    def phi(self, x, out=None):
        """y = Phi x (x: n x n, y: M in uv order)."""
        y = self.empty(self.M) if out is None else out
        _check(self.lib.purify_phi(self.handle, self._vec(x, self.n * self.n, "x"),
                                   self._vec(y, self.M, "y"), self._stream()), "purify_phi")
        return y

    def phi_noalloc(self, x, out=None):
        """y = Phi x through purify_phi_noalloc (intermediates in the library's fixed device
        array instead of the plan workspace; n <= 1024 FP32, n <= 512 FP64)."""
        y = self.empty(self.M) if out is None else out
        _check(self.lib.purify_phi_noalloc(self.handle, self._vec(x, self.n * self.n, "x"),
                                           self._vec(y, self.M, "y"), self._stream()), "purify_phi_noalloc")
        return y

    def phi_adj(self, y, out=None):
        x = self.empty(self.n, self.n) if out is None else out
        _check(self.lib.purify_phi_adj(self.handle, self._vec(y, self.M, "y"),
                                       self._vec(x, self.n * self.n, "x"), self._stream()),
               "purify_phi_adj")
        return x

    def psi(self, alpha, out=None):
        x = self.empty(self.n, self.n) if out is None else out
        _check(self.lib.purify_psi(self.handle, self._vec(alpha, self.D, "alpha"),
                                   self._vec(x, self.n * self.n, "x"), self._stream()),
               "purify_psi")
        return x

    def psi_adj(self, x, out=None):
        a = self.empty(self.q, self.n, self.n) if out is None else out
        _check(self.lib.purify_psi_adj(self.handle, self._vec(x, self.n * self.n, "x"),
                                       self._vec(a, self.D, "alpha"), self._stream()),
               "purify_psi_adj")
        return a

    def normal(self, x, toeplitz: bool = False, out=None):
        """Phi^dagger Phi x through the NUFFT (fused G^T G), or its stored Toeplitz form."""
        o = self.empty(self.n, self.n) if out is None else out
        _check(self.lib.purify_phi_normal(self.handle, self._vec(x, self.n * self.n, "x"),
                                          self._vec(o, self.n * self.n, "out"),
                                          NORMAL_TOEPLITZ if toeplitz else 0, self._stream()),
               "purify_phi_normal")
        return o

    def _params(self, epsilon, max_iter, cg_iter, gamma, nu, nu_iter, halting, xi, slack,
                check_every, weights, graph, warm, hist, toeplitz=False, blocks=None, tv_iter=None):
        p = SdmmParams()
        if tv_iter is not None:
            p.tv_iter = int(tv_iter)
        if blocks is not None:
            # visibility blocks (offsets into the uv order, R + 1 of them; eps_i per block);
            # the arrays stay referenced by the parameter object for the call
            offs = np.ascontiguousarray(blocks[0], dtype=np.int64)
            eps_b = np.ascontiguousarray(blocks[1], dtype=np.float64)
            if offs.size != eps_b.size + 1:
                raise ValueError("blocks: R + 1 offsets and R bounds")
            if eps_b.size == 1:          # one block: the plain constraint
                epsilon = float(eps_b[0])
            else:
                p._keep = (offs, eps_b)
                p.nblocks = eps_b.size
                p.block_offsets = offs.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
                p.block_eps = _dptr(eps_b)
        p.epsilon, p.gamma, p.nu, p.xi, p.slack = epsilon, gamma, nu, xi, slack
        p.max_iter, p.cg_iter, p.check_every = max_iter, cg_iter, check_every
        p.halting, p.nu_iter = int(bool(halting)), nu_iter
        p.flags = ((0 if graph else SDMM_NO_GRAPH) | (SDMM_WARM_START if warm else 0)
                   | (SDMM_TOEPLITZ if toeplitz else 0) | (SDMM_TV if tv_iter is not None else 0))
        if weights is not None:
            p.weights = self._weights(weights, self.n * self.n if tv_iter is not None else self.D)
        p.history = _dptr(hist) if hist is not None else None
        return p

    def _weights(self, w, count):
        if (not isinstance(w, self.torch.Tensor) or w.dtype != self.torch.float64 or w.numel() != count
                or w.device != self.device or not w.is_contiguous()):
            raise ValueError(f"weights must be a contiguous float64 device tensor of {count} elements")
        return w.data_ptr()

    def _start(self, x0, out):
        x = self.empty(self.n, self.n) if out is None else out
        if x0 is not None:
            x.copy_(self.as_vec(x0).reshape(x.shape))
        return x

    def sdmm(self, y, epsilon: float, max_iter: int = 300, cg_iter: int = 10,
             gamma: float = 0.0, nu: float = 0.0, nu_iter: int = 100, halting: bool = False,
             xi: float = 1e-4, slack: float = 1e-3, check_every: int = 10, weights=None,
             record_history: bool = False, graph: bool = True, x0=None, toeplitz: bool = False,
             blocks=None, tv_iter=None, out=None) -> SolveResult:
        """SDMM (Algorithm 1) for eq. (3); returns x_hat and solver info.
        x0: starting point x_hat(0) (default 0).  toeplitz: CG with the stored normal operator.
        blocks: (offsets, eps_list) for R >= 2 visibility blocks (eqs. (4)-(5)); epsilon unused.
        tv_iter: TV prior (Section 5) with that many dual projection steps per prox; weights are
        then per pixel."""
        x = self._start(x0, out)
        hist = np.zeros(2 * max_iter) if record_history else None
        p = self._params(epsilon, max_iter, cg_iter, gamma, nu, nu_iter, halting, xi, slack, check_every,
                         weights, graph, x0 is not None, hist, toeplitz, blocks, tv_iter)
        info = SdmmInfo()
        _check(self.lib.purify_sdmm_solve(self.handle, self._vec(y, self.M, "y"), ctypes.byref(p),
                                          self._vec(x, self.n * self.n, "x"), ctypes.byref(info),
                                          self._stream()), "purify_sdmm_solve")
        if hist is not None:
            hist = hist[: 2 * info.iterations].reshape(-1, 2)
        return SolveResult(x, info.iterations, bool(info.converged), info.objective,
                           info.residual, info.nu, info.gamma, hist)

    def sdmm_reweighted(self, y, epsilon: float, reweights: int = 5, delta0: float = 0.0,
                        decay: float = 0.1, delta_min: float = -1.0, rel_var: float = 1e-3,
                        max_iter: int = 300, cg_iter: int = 10, gamma: float = 0.0, nu: float = 0.0,
                        nu_iter: int = 100, halting: bool = False, xi: float = 1e-4, slack: float = 1e-3,
                        check_every: int = 10, weights=None, graph: bool = True, x0=None,
                        toeplitz: bool = False, blocks=None, tv_iter=None, out=None) -> "ReweightResult":
        """Reweighted l1 (SARA): solve 0 with `weights` (None: W = I), then up to `reweights`
        weighted solves (purify_sdmm_reweighted)."""
        x = self._start(x0, out)
        count = self.n * self.n if tv_iter is not None else self.D
        w = self.torch.empty(count, dtype=self.torch.float64, device=self.device)
        p = self._params(epsilon, max_iter, cg_iter, gamma, nu, nu_iter, halting, xi, slack, check_every,
                         weights, graph, x0 is not None, None, toeplitz, blocks, tv_iter)
        rw = ReweightParams()
        rw.delta0, rw.decay, rw.delta_min, rw.rel_var, rw.reweights = delta0, decay, delta_min, rel_var, reweights
        info, rinfo = SdmmInfo(), ReweightInfo()
        _check(self.lib.purify_sdmm_reweighted(self.handle, self._vec(y, self.M, "y"), ctypes.byref(p),
                                               ctypes.byref(rw), w.data_ptr(),
                                               self._vec(x, self.n * self.n, "x"), ctypes.byref(info),
                                               ctypes.byref(rinfo), self._stream()),
               "purify_sdmm_reweighted")
        return ReweightResult(x, w, rinfo.solves, rinfo.total_iterations, rinfo.delta, rinfo.rel_var,
                              SolveResult(x, info.iterations, bool(info.converged), info.objective,
                                          info.residual, info.nu, info.gamma, None))

    def time_stage(self, stage: str, reps: int = 20) -> float:
        """Average milliseconds per launch of one stage (HIP events on the current stream)."""
        ms = ctypes.c_double()
        _check(self.lib.purify_time_stage(self.handle, STAGES[stage], reps, self._stream(),
                                          ctypes.byref(ms)), "purify_time_stage")
        return ms.value


@dataclass
class ServedResult:
    x: np.ndarray                # host complex (n, n); the image is x.real
    iterations: int
    converged: bool
    objective: float
    residual: float
    nu: float
    gamma: float
    queue_ms: float              # submission -> admission
    run_ms: float                # admission -> result on the host (plan, solve, download)
    latency_ms: float            # submission -> result on the host


class Server:
    """Serving form: solves of independent requests (mixed sizes) run concurrently on one GPU.

    The HBM budget is one device arena (a torch uint8 tensor of ``arena_bytes``) from which
    every admitted request gets its plan workspace, visibilities and image; ``max_active``
    requests run at once, each on its own stream.  ``submit`` returns a ticket at once;
    ``wait`` blocks until that request's image is on the host.
    """

    def __init__(self, arena_bytes: int, max_active: int = 4, device="cuda:0"):
        import torch
        self.lib = load_library()
        self.torch = torch
        self.device = torch.device(device)
        self.arena = torch.empty(int(arena_bytes), dtype=torch.uint8, device=self.device)
        d = ServerDesc()
        d.arena, d.arena_bytes, d.max_active = self.arena.data_ptr(), int(arena_bytes), max_active
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _check(self.lib.purify_server_create(ctypes.byref(d), ctypes.byref(h)), "purify_server_create")
        self.handle = h
        self._meta = {}

    def submit(self, n: int, uv, y, epsilon: float, J: int = 6, dict_mask: int = DICT_SARA,
               levels: int = 4, precision: str = "fp32", max_iter: int = 300, cg_iter: int = 10,
               halting: bool = True, xi: float = 1e-4, slack: float = 1e-3, check_every: int = 10,
               nu: float = 0.0, nu_iter: int = 100, gamma: float = 0.0, graph: bool = True,
               toeplitz: bool = False) -> int:
        """Queue one solve (host uv and visibilities are copied); returns its ticket.
        toeplitz: the global update's CG applies the stored (Toeplitz) normal operator."""
        prec = FP64 if precision in ("fp64", FP64) else FP32
        uv = np.ascontiguousarray(uv, dtype=np.float64).reshape(-1, 2)
        yh = np.ascontiguousarray(y, dtype=np.complex128 if prec == FP64 else np.complex64).ravel()
        if yh.size != uv.shape[0]:
            raise ValueError("y must have one value per uv point")
        d = _desc(n, uv, J, 0.0, dict_mask, levels, prec)
        p = SdmmParams()
        p.epsilon, p.gamma, p.nu, p.xi, p.slack = epsilon, gamma, nu, xi, slack
        p.max_iter, p.cg_iter, p.check_every = max_iter, cg_iter, check_every
        p.halting, p.nu_iter = int(bool(halting)), nu_iter
        p.flags = (0 if graph else SDMM_NO_GRAPH) | (SDMM_TOEPLITZ if toeplitz else 0)
        t = ctypes.c_int64()
        _check(self.lib.purify_server_submit(self.handle, ctypes.byref(d), yh.ctypes.data, ctypes.byref(p),
                                             ctypes.byref(t)), "purify_server_submit")
        self._meta[t.value] = (n, prec)
        return t.value

    def poll(self, ticket: int) -> int:
        return int(self.lib.purify_server_poll(self.handle, ticket))

    def wait(self, ticket: int) -> ServedResult:
        n, prec = self._meta.pop(ticket)
        x = np.zeros((n, n), dtype=np.complex128 if prec == FP64 else np.complex64)
        info = SdmmInfo()
        tm = np.zeros(3)
        _check(self.lib.purify_server_wait(self.handle, ticket, x.ctypes.data, ctypes.byref(info), _dptr(tm)),
               "purify_server_wait")
        return ServedResult(x, info.iterations, bool(info.converged), info.objective, info.residual,
                            info.nu, info.gamma, float(tm[0]), float(tm[1]), float(tm[2]))

    def close(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value:
            self.lib.purify_server_destroy(h)
            self.handle = None

    def __del__(self):
        self.close()
