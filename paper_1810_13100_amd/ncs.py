"""Python binding of the NCS C ABI (``include/ncs.h``).

Argument marshalling only: every step of the method runs in the HIP library
``libncs.so``.  PyTorch supplies device memory and the current stream.  There
is no fallback; if the library is missing or the device is not a GPU the calls
raise.
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libncs.so")

NCS_OK = 0
NCS_NOT_CONVERGED = 1
NCS_ERR_INVALID_ARG = -1
NCS_ERR_HIP = -2
NCS_ERR_OOM = -3
NCS_ERR_NONFINITE = -4
NCS_ERR_DIVERGED = -5

NCS_F32 = 0
NCS_F64 = 1
METHOD_NCS = 0
METHOD_PDHG = 1
METHOD_ADMM_CG = 2
DATA_QUADRATIC = 0
DATA_POISSON = 1
TV_ANISO = 0
TV_ISO = 1
BEAM_PARALLEL = 0
BEAM_FAN = 1

_STATUS_NAMES = {
    NCS_OK: "NCS_OK", NCS_NOT_CONVERGED: "NCS_NOT_CONVERGED",
    NCS_ERR_INVALID_ARG: "NCS_ERR_INVALID_ARG", NCS_ERR_HIP: "NCS_ERR_HIP",
    NCS_ERR_OOM: "NCS_ERR_OOM", NCS_ERR_NONFINITE: "NCS_ERR_NONFINITE",
    NCS_ERR_DIVERGED: "NCS_ERR_DIVERGED",
}

EXPORTED = [
    "ncs_setup", "ncs_set_init", "ncs_set_x", "ncs_iterate", "ncs_solve", "ncs_get_objectives",
    "ncs_get_iteration", "ncs_get_x", "ncs_get_u", "ncs_get_v", "ncs_get_t", "ncs_get_state", "ncs_set_state",
    "ncs_forward", "ncs_forward_noalloc", "ncs_adjoint", "ncs_apply_minv", "ncs_objective", "ncs_prefilter", "ncs_fbp", "ncs_get_eigenvalues",
    "ncs_time_phases", "ncs_get_info", "ncs_destroy", "ncs_last_error",
    "ncs_batch_setup", "ncs_batch_set_init", "ncs_batch_solve", "ncs_batch_slice", "ncs_batch_destroy",
]
PHASES = ["backproject", "fft_rows", "fft_cols_multiplier", "fft_rows_inv_update",
          "project_dataprox_tv", "objective_reduce"]


class NcsError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{_STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class _Geometry(ctypes.Structure):
    _fields_ = [("n_side", ctypes.c_int32), ("n_angles", ctypes.c_int32), ("n_bins", ctypes.c_int32),
                ("beam", ctypes.c_int32), ("source_radius", ctypes.c_double)]


class _Params(ctypes.Structure):
    _fields_ = [
        ("alpha", ctypes.c_double), ("beta", ctypes.c_double), ("gamma", ctypes.c_double),
        ("lambda_", ctypes.c_double), ("c_r", ctypes.c_double), ("mu_dc", ctypes.c_double),
        ("data_term", ctypes.c_int32), ("tv_term", ctypes.c_int32),
        ("check_every", ctypes.c_int32), ("diverge_checks", ctypes.c_int32),
        ("projector", ctypes.c_int32), ("graph_chunk", ctypes.c_int32),
        ("dual_ramp", ctypes.c_double), ("backprojector", ctypes.c_int32), ("method", ctypes.c_int32),
        ("cg_iters", ctypes.c_int32), ("cg_precondition", ctypes.c_int32), ("positivity", ctypes.c_int32),
        ("probes", ctypes.c_int32),
    ]


class _Info(ctypes.Structure):
    _fields_ = [("nnz", ctypes.c_int64), ("c_r", ctypes.c_double), ("mu_dc", ctypes.c_double),
                ("norm_e1_sq", ctypes.c_double), ("projector", ctypes.c_int32), ("backprojector", ctypes.c_int32),
                ("projector_ms", ctypes.c_double * 3), ("backprojector_ms", ctypes.c_double * 3)]


_lib = None


def load_library() -> ctypes.CDLL:
    """Load libncs.so (torch is imported first so both share one HIP runtime)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() first")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double
    pi32, pdbl, psz = ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_size_t)
    sigs = {
        "ncs_setup": ([ctypes.POINTER(_Geometry), ctypes.POINTER(_Params), i32, vp, vp, vp,
                       ctypes.POINTER(vp)], i32),
        "ncs_set_init": ([vp, vp, i32], i32),
        "ncs_set_x": ([vp, vp], i32),
        "ncs_iterate": ([vp, i32, pdbl], i32),
        "ncs_solve": ([vp, i32, dbl, dbl, pi32, pdbl], i32),
        "ncs_get_objectives": ([vp, i32, i32, pdbl], i32),
        "ncs_get_iteration": ([vp, pi32], i32),
        "ncs_get_x": ([vp, vp], i32),
        "ncs_get_u": ([vp, vp], i32),
        "ncs_get_v": ([vp, vp], i32),
        "ncs_get_t": ([vp, vp], i32),
        "ncs_get_state": ([vp, vp, psz], i32),
        "ncs_set_state": ([vp, vp, ctypes.c_size_t], i32),
        "ncs_forward": ([vp, vp, vp], i32),
        "ncs_forward_noalloc": ([ctypes.POINTER(_Geometry), vp, vp, vp], i32),
        "ncs_adjoint": ([vp, vp, vp], i32),
        "ncs_apply_minv": ([vp, vp, vp], i32),
        "ncs_prefilter": ([vp, vp, vp], i32),
        "ncs_fbp": ([vp, vp, vp], i32),
        "ncs_objective": ([vp, vp, pdbl], i32),
        "ncs_get_eigenvalues": ([vp, pdbl], i32),
        "ncs_time_phases": ([vp, i32, pdbl], i32),
        "ncs_get_info": ([vp, ctypes.POINTER(_Info)], i32),
        "ncs_destroy": ([vp], None),
        "ncs_batch_setup": ([i32, ctypes.POINTER(_Geometry), ctypes.POINTER(_Params), i32,
                             ctypes.POINTER(vp), ctypes.POINTER(vp), vp, ctypes.POINTER(vp)], i32),
        "ncs_batch_set_init": ([vp, ctypes.POINTER(vp), i32], i32),
        "ncs_batch_solve": ([vp, i32, pdbl, pi32, pdbl], i32),
        "ncs_batch_slice": ([vp, i32, ctypes.POINTER(vp)], i32),
        "ncs_batch_destroy": ([vp], None),
        "ncs_last_error": ([], ctypes.c_char_p),
    }
    for name, (args, res) in sigs.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def _check(status: int, allow=(NCS_OK,)) -> int:
    if status in allow:
        return status
    msg = load_library().ncs_last_error().decode(errors="replace")
    raise NcsError(status, msg)


def forward_noalloc(geom: "Geometry", x: torch.Tensor, y: torch.Tensor) -> torch.Tensor:
    """y = E x through ncs_forward_noalloc: no handle, and the library allocates
    nothing (its workspace is a fixed device array).  x: N*N float32, y:
    N_theta*N_s float32, both on the current device; runs on torch's current
    stream."""
    lib = load_library()
    if x.dtype != torch.float32 or y.dtype != torch.float32 or not x.is_cuda or not y.is_cuda:
        raise ValueError("forward_noalloc takes float32 device tensors")
    if x.numel() != geom.n_side * geom.n_side or y.numel() != geom.n_angles * geom.n_bins:
        raise ValueError("forward_noalloc: x must hold N*N values and y N_theta*N_s")
    if not (x.is_contiguous() and y.is_contiguous()):
        raise ValueError("forward_noalloc: x and y must be contiguous")
    g = geom._c()
    stream = torch.cuda.current_stream(x.device).cuda_stream
    _check(lib.ncs_forward_noalloc(ctypes.byref(g), x.data_ptr(), y.data_ptr(), stream))
    return y


@dataclass
class Geometry:
    n_side: int
    n_angles: int             # parallel angles over [0, pi), or fan source positions over a full turn
    n_bins: int
    beam: int = BEAM_PARALLEL
    source_radius: float = 0.0  # fan: source distance from the image centre, in pixels

    def _c(self) -> "_Geometry":
        return _Geometry(self.n_side, self.n_angles, self.n_bins, self.beam, self.source_radius)

    @property
    def n(self) -> int:
        return self.n_side * self.n_side

    @property
    def m(self) -> int:
        return self.n_angles * self.n_bins


@dataclass
class Params:
    alpha: float
    beta: float
    gamma: float
    lam: float
    c_r: float = 0.0
    mu_dc: float = 0.0
    data_term: int = DATA_QUADRATIC
    tv_term: int = TV_ANISO
    check_every: int = 50
    diverge_checks: int = 0
    projector: int = 0        # 0: autotune at setup, 1: LDS-staged, 2: direct, 3: ray pairs
    graph_chunk: int = 0      # 0: graphs of up to 32 iterations, < 0: no graphs
    dual_ramp: float = 0.0    # TV-dual ramp width of the warm start (0: sign)
    backprojector: int = 0    # 0: autotune at setup, 1: LDS-staged windows, 2: direct, 3: 2x2 per lane
                              # with 16-byte windows
    method: int = 0           # METHOD_NCS, METHOD_PDHG (M = gamma I) or METHOD_ADMM_CG
    cg_iters: int = 0         # ADMM-CG: CG steps per linear solve (0: 10)
    cg_precondition: int = 1  # ADMM-CG: precondition CG with alpha M^+
    positivity: int = 0       # 1: constrain x >= 0 (a third dual block t; NCS and PDHG)
    probes: int = 0           # > 0: E^T E's multiplier from this many probes (eq. H-fan); 0: analytic
                              # (parallel) or 16 probes (fan)


def _ptr(t: torch.Tensor | None) -> int | None:
    return None if t is None else t.data_ptr()


class Solver:
    """One NCS problem instance on the current CUDA (HIP) device."""

    def __init__(self, geom: Geometry, params: Params, b: torch.Tensor | None = None,
                 bg: torch.Tensor | None = None, dtype: torch.dtype = torch.float32):
        if dtype not in (torch.float32, torch.float64):
            raise ValueError("dtype must be torch.float32 or torch.float64")
        if not torch.cuda.is_available():
            raise RuntimeError("the NCS library needs a GPU; none is visible")
        self.lib = load_library()
        self.geom = geom
        self.params = params
        self.dtype = dtype
        self.device = torch.device("cuda", torch.cuda.current_device())
        self._b = self._sino(b, "b") if b is not None else None
        self._bg = self._sino(bg, "bg") if bg is not None else None
        g = geom._c()
        p = _Params(params.alpha, params.beta, params.gamma, params.lam, params.c_r, params.mu_dc,
                    params.data_term, params.tv_term, params.check_every, params.diverge_checks,
                    params.projector, params.graph_chunk, params.dual_ramp, params.backprojector, params.method,
                    params.cg_iters, params.cg_precondition, params.positivity, params.probes)
        self.stream = torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        _check(self.lib.ncs_setup(ctypes.byref(g), ctypes.byref(p),
                                  NCS_F64 if dtype == torch.float64 else NCS_F32,
                                  _ptr(self._b), _ptr(self._bg), self.stream.cuda_stream, ctypes.byref(h)))
        self.h = h

    # -- argument checks ---------------------------------------------------
    def _dev(self, t: torch.Tensor, numel: int, name: str) -> torch.Tensor:
        if not isinstance(t, torch.Tensor) or t.device != self.device:
            raise ValueError(f"{name} must be a tensor on {self.device}")
        if t.dtype != self.dtype:
            raise ValueError(f"{name} must have dtype {self.dtype}")
        if t.numel() != numel:
            raise ValueError(f"{name} must have {numel} elements (got {t.numel()})")
        if not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous")
        return t

    def _sino(self, t, name):
        return self._dev(t, self.geom.m, name)

    def _img(self, t, name):
        return self._dev(t, self.geom.n, name)

    # -- state -------------------------------------------------------------
    def set_init(self, x0: torch.Tensor | None = None, dual_from_x0: bool = False) -> None:
        x0p = _ptr(self._img(x0, "x0")) if x0 is not None else None
        self._x0_keep = x0
        _check(self.lib.ncs_set_init(self.h, x0p, int(dual_from_x0)))

    def set_x(self, x: torch.Tensor) -> None:
        """Replace the iterate (E x recomputed); duals and iteration count are kept."""
        self._x_keep = self._img(x, "x")
        _check(self.lib.ncs_set_x(self.h, self._x_keep.data_ptr()))

    def iterate(self, k: int, record: bool = False) -> np.ndarray | None:
        if record:
            obj = np.empty(k, dtype=np.float64)
            _check(self.lib.ncs_iterate(self.h, k, obj.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
            return obj
        _check(self.lib.ncs_iterate(self.h, k, None))
        return None

    def solve(self, max_iters: int, f_target: float = math.nan,
              fp_residual_tol: float = 0.0) -> tuple[int, int, float]:
        """Returns (status, iterations run, last objective); status is NCS_OK or NCS_NOT_CONVERGED.
        fp_residual_tol > 0 also stops at a host check once |x^k - x^{k-1}| <= tol |x^k|."""
        it = ctypes.c_int32()
        f = ctypes.c_double()
        st = _check(self.lib.ncs_solve(self.h, max_iters, f_target, fp_residual_tol, ctypes.byref(it),
                                       ctypes.byref(f)),
                    allow=(NCS_OK, NCS_NOT_CONVERGED))
        return st, it.value, f.value

    def objectives(self, first: int, count: int) -> np.ndarray:
        out = np.empty(count, dtype=np.float64)
        _check(self.lib.ncs_get_objectives(self.h, first, count,
                                           out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return out

    def iteration(self) -> int:
        it = ctypes.c_int32()
        _check(self.lib.ncs_get_iteration(self.h, ctypes.byref(it)))
        return it.value

    def x(self) -> torch.Tensor:
        out = torch.empty(self.geom.n, dtype=self.dtype, device=self.device)
        _check(self.lib.ncs_get_x(self.h, out.data_ptr()))
        return out

    def u(self) -> torch.Tensor:
        out = torch.empty(self.geom.m, dtype=self.dtype, device=self.device)
        _check(self.lib.ncs_get_u(self.h, out.data_ptr()))
        return out

    def v(self) -> torch.Tensor:
        out = torch.empty(2 * self.geom.n, dtype=self.dtype, device=self.device)
        _check(self.lib.ncs_get_v(self.h, out.data_ptr()))
        return out

    def t(self) -> torch.Tensor:
        """The positivity dual t (params.positivity = 1 only)."""
        out = torch.empty(self.geom.n, dtype=self.dtype, device=self.device)
        _check(self.lib.ncs_get_t(self.h, out.data_ptr()))
        return out

    def get_state(self) -> bytes:
        n = ctypes.c_size_t()
        _check(self.lib.ncs_get_state(self.h, None, ctypes.byref(n)))
        buf = ctypes.create_string_buffer(n.value)
        _check(self.lib.ncs_get_state(self.h, buf, ctypes.byref(n)))
        return buf.raw[: n.value]

    def set_state(self, blob: bytes) -> None:
        buf = ctypes.create_string_buffer(blob, len(blob))
        _check(self.lib.ncs_set_state(self.h, buf, len(blob)))

    # -- operators ---------------------------------------------------------
    def forward(self, x: torch.Tensor) -> torch.Tensor:
        y = torch.empty(self.geom.m, dtype=self.dtype, device=self.device)
        _check(self.lib.ncs_forward(self.h, self._img(x, "x").data_ptr(), y.data_ptr()))
        return y

    def adjoint(self, y: torch.Tensor) -> torch.Tensor:
        x = torch.empty(self.geom.n, dtype=self.dtype, device=self.device)
        _check(self.lib.ncs_adjoint(self.h, self._sino(y, "y").data_ptr(), x.data_ptr()))
        return x

    def apply_minv(self, w: torch.Tensor) -> torch.Tensor:
        out = torch.empty(self.geom.n, dtype=self.dtype, device=self.device)
        _check(self.lib.ncs_apply_minv(self.h, self._img(w, "w").data_ptr(), out.data_ptr()))
        return out

    def prefilter(self, y: torch.Tensor) -> torch.Tensor:
        """alpha M^+ E^T y: the filtered backprojection that feeds the warm-start network."""
        out = torch.empty(self.geom.n, dtype=self.dtype, device=self.device)
        _check(self.lib.ncs_prefilter(self.h, self._sino(y, "y").data_ptr(), out.data_ptr()))
        return out

    def fbp(self, y: torch.Tensor) -> torch.Tensor:
        """Filtered backprojection (pi / N_theta) E^T (h * y) with the Shepp-Logan filter."""
        out = torch.empty(self.geom.n, dtype=self.dtype, device=self.device)
        _check(self.lib.ncs_fbp(self.h, self._sino(y, "y").data_ptr(), out.data_ptr()))
        return out

    def objective(self, x: torch.Tensor) -> float:
        f = ctypes.c_double()
        _check(self.lib.ncs_objective(self.h, self._img(x, "x").data_ptr(), ctypes.byref(f)))
        return f.value

    def time_phases(self, iters: int) -> dict:
        """Mean ms per iteration of each kernel, timed with HIP events (advances the state)."""
        ms = np.zeros(len(PHASES), dtype=np.float64)
        _check(self.lib.ncs_time_phases(self.h, iters, ms.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return dict(zip(PHASES, ms.tolist()))

    def info(self) -> dict:
        inf = _Info()
        _check(self.lib.ncs_get_info(self.h, ctypes.byref(inf)))
        return {"nnz": inf.nnz, "c_r": inf.c_r, "mu_dc": inf.mu_dc, "norm_e1_sq": inf.norm_e1_sq,
                "projector": inf.projector, "projector_ms": list(inf.projector_ms),
                "backprojector": inf.backprojector, "backprojector_ms": list(inf.backprojector_ms)}

    def eigenvalues(self) -> np.ndarray:
        mu = np.empty(self.geom.n, dtype=np.float64)
        _check(self.lib.ncs_get_eigenvalues(self.h, mu.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return mu.reshape(self.geom.n_side, self.geom.n_side)

    def close(self) -> None:
        if getattr(self, "h", None) is not None and self.h.value:
            self.lib.ncs_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class _SliceView(Solver):
    """A slice of a Batch: the Solver interface on a handle the batch owns."""

    def __init__(self, batch: "Batch", i: int, geom: Geometry, params: Params):
        self.lib = batch.lib
        self.geom = geom
        self.params = params
        self.dtype = batch.dtype
        self.device = batch.device
        self._b = batch._b[i]
        self._bg = None
        self.stream = batch.stream
        h = ctypes.c_void_p()
        _check(self.lib.ncs_batch_slice(batch.h, i, ctypes.byref(h)))
        self.h = h

    def close(self) -> None:   # owned by the batch
        self.h = ctypes.c_void_p()


class Batch:
    """Many independent slices of uneven size solved by shared launches."""

    def __init__(self, geoms: list, params: list, bs: list, bgs: list | None = None,
                 dtype: torch.dtype = torch.float32):
        if not torch.cuda.is_available():
            raise RuntimeError("the NCS library needs a GPU; none is visible")
        n = len(geoms)
        if not (n == len(params) == len(bs)) or n == 0:
            raise ValueError("geoms, params and bs must have the same non-zero length")
        self.lib = load_library()
        self.dtype = dtype
        self.device = torch.device("cuda", torch.cuda.current_device())
        self.geoms, self.params = list(geoms), list(params)
        for g, b in zip(geoms, bs):
            if b.device != self.device or b.dtype != dtype or b.numel() != g.m or not b.is_contiguous():
                raise ValueError("each b must be a contiguous tensor of n_angles*n_bins elements on the device")
        self._b = list(bs)
        self._bg = list(bgs) if bgs is not None else None
        G = (_Geometry * n)(*[g._c() for g in geoms])
        P = (_Params * n)(*[_Params(p.alpha, p.beta, p.gamma, p.lam, p.c_r, p.mu_dc, p.data_term, p.tv_term,
                                    p.check_every, p.diverge_checks, p.projector, p.graph_chunk, p.dual_ramp,
                                    p.backprojector, p.method, p.cg_iters, p.cg_precondition, p.positivity,
                                    p.probes)
                              for p in params])
        B = (ctypes.c_void_p * n)(*[b.data_ptr() for b in bs])
        BG = None
        if bgs is not None:
            BG = (ctypes.c_void_p * n)(*[None if t is None else t.data_ptr() for t in bgs])
        self.stream = torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        _check(self.lib.ncs_batch_setup(n, G, P, NCS_F64 if dtype == torch.float64 else NCS_F32, B, BG,
                                        self.stream.cuda_stream, ctypes.byref(h)))
        self.h = h
        self.n = n

    def set_init(self, x0s: list | None = None, dual_from_x0: bool = False) -> None:
        arr = None
        if x0s is not None:
            self._x0_keep = list(x0s)
            arr = (ctypes.c_void_p * self.n)(*[None if t is None else t.data_ptr() for t in x0s])
        _check(self.lib.ncs_batch_set_init(self.h, arr, int(dual_from_x0)))

    def solve(self, max_iters: int, f_targets=None):
        """Returns (status, iterations per slice, last objective per slice)."""
        ft = None
        if f_targets is not None:
            ft = np.ascontiguousarray(f_targets, dtype=np.float64)
        it = np.zeros(self.n, dtype=np.int32)
        f = np.zeros(self.n, dtype=np.float64)
        st = _check(self.lib.ncs_batch_solve(
            self.h, max_iters, None if ft is None else ft.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
            it.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), f.ctypes.data_as(ctypes.POINTER(ctypes.c_double))),
            allow=(NCS_OK, NCS_NOT_CONVERGED))
        return st, it, f

    def slice(self, i: int) -> Solver:
        return _SliceView(self, i, self.geoms[i], self.params[i])

    def close(self) -> None:
        if getattr(self, "h", None) is not None and self.h.value:
            self.lib.ncs_batch_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
