"""Python binding of the cone-beam C ABI (``include/ncs_cone.h``).

Argument marshalling only: every step runs in the HIP library ``libncs.so``.
PyTorch supplies device memory and the current stream.  There is no fallback.
"""
from __future__ import annotations

import ctypes
import math
from dataclasses import dataclass

import numpy as np
import torch

from .ncs import METHOD_NCS, NCS_F32, NCS_F64, _check, load_library

EXPORTED = [
    "ncs_cone_setup", "ncs_cone_set_init", "ncs_cone_iterate", "ncs_cone_get_x", "ncs_cone_get_u",
    "ncs_cone_get_v", "ncs_cone_get_t", "ncs_cone_forward", "ncs_cone_adjoint", "ncs_cone_apply_minv",
    "ncs_cone_get_eigenvalues", "ncs_cone_get_info", "ncs_cone_time_phases", "ncs_cone_destroy",
    "ncs_cone_get_state", "ncs_cone_set_state",
]
PHASES = ["backproject", "dft_update", "project_dataprox", "tv_dual", "objective_reduce"]


class _ConeGeometry(ctypes.Structure):
    _fields_ = [("n_side", ctypes.c_int32), ("n_slices", ctypes.c_int32), ("n_views", ctypes.c_int32),
                ("n_bins", ctypes.c_int32), ("n_rows", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("source_radius", ctypes.c_double)]


class _ConeParams(ctypes.Structure):
    _fields_ = [("alpha", ctypes.c_double), ("beta", ctypes.c_double), ("gamma", ctypes.c_double),
                ("lambda_", ctypes.c_double), ("mu_dc", ctypes.c_double), ("method", ctypes.c_int32),
                ("probes", ctypes.c_int32), ("positivity", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class _ConeInfo(ctypes.Structure):
    _fields_ = [("nnz", ctypes.c_int64), ("norm_e1_sq", ctypes.c_double), ("mu_dc", ctypes.c_double),
                ("bin_window", ctypes.c_int32)]


_bound = False


def _lib() -> ctypes.CDLL:
    global _bound
    lib = load_library()
    if _bound:
        return lib
    vp, i32, pdbl = ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_double)
    sigs = {
        "ncs_cone_setup": ([ctypes.POINTER(_ConeGeometry), ctypes.POINTER(_ConeParams), i32, vp, vp,
                            ctypes.POINTER(vp)], i32),
        "ncs_cone_set_init": ([vp, vp], i32),
        "ncs_cone_iterate": ([vp, i32, pdbl], i32),
        "ncs_cone_get_x": ([vp, vp], i32),
        "ncs_cone_get_u": ([vp, vp], i32),
        "ncs_cone_get_v": ([vp, vp], i32),
        "ncs_cone_get_t": ([vp, vp], i32),
        "ncs_cone_forward": ([vp, vp, vp], i32),
        "ncs_cone_adjoint": ([vp, vp, vp], i32),
        "ncs_cone_apply_minv": ([vp, vp, vp], i32),
        "ncs_cone_get_eigenvalues": ([vp, pdbl], i32),
        "ncs_cone_get_info": ([vp, ctypes.POINTER(_ConeInfo)], i32),
        "ncs_cone_time_phases": ([vp, i32, pdbl], i32),
        "ncs_cone_destroy": ([vp], None),
        "ncs_cone_get_state": ([vp, vp, ctypes.POINTER(ctypes.c_size_t)], i32),
        "ncs_cone_set_state": ([vp, vp, ctypes.c_size_t], i32),
    }
    for name, (args, res) in sigs.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _bound = True
    return lib


@dataclass
class ConeGeometry:
    n_side: int
    n_slices: int
    n_views: int              # source positions over a full turn
    n_bins: int               # detector columns (equi-angular)
    n_rows: int               # detector rows (equal slope steps)
    source_radius: float      # in voxels

    def _c(self) -> _ConeGeometry:
        return _ConeGeometry(self.n_side, self.n_slices, self.n_views, self.n_bins, self.n_rows, 0,
                             self.source_radius)

    @property
    def n(self) -> int:
        return self.n_side * self.n_side * self.n_slices

    @property
    def m(self) -> int:
        return self.n_views * self.n_rows * self.n_bins


@dataclass
class ConeParams:
    alpha: float
    beta: float
    gamma: float
    lam: float
    mu_dc: float = 0.0        # <= 0: gamma + alpha |E 1|^2 / n
    method: int = METHOD_NCS  # METHOD_NCS or METHOD_PDHG
    probes: int = 0           # probes of eq. (H-fan); 0: 16
    positivity: int = 0       # 1: constrain x >= 0 (a dual t)


class ConeSolver:
    """One cone-beam NCS (or PDHG) problem on the current CUDA (HIP) device."""

    def __init__(self, geom: ConeGeometry, params: ConeParams, b: torch.Tensor | None = None,
                 dtype: torch.dtype = torch.float32):
        if dtype not in (torch.float32, torch.float64):
            raise ValueError("dtype must be torch.float32 or torch.float64")
        if not torch.cuda.is_available():
            raise RuntimeError("the NCS library needs a GPU; none is visible")
        self.lib = _lib()
        self.geom, self.params, self.dtype = geom, params, dtype
        self.device = torch.device("cuda", torch.cuda.current_device())
        self._b = self._dev(b, geom.m, "b") if b is not None else None
        g = geom._c()
        p = _ConeParams(params.alpha, params.beta, params.gamma, params.lam, params.mu_dc, params.method,
                        params.probes, params.positivity, 0)
        self.stream = torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        _check(self.lib.ncs_cone_setup(ctypes.byref(g), ctypes.byref(p), NCS_F64 if dtype == torch.float64 else NCS_F32,
                                       None if self._b is None else self._b.data_ptr(), self.stream.cuda_stream,
                                       ctypes.byref(h)))
        self.h = h

    def _dev(self, t: torch.Tensor, numel: int, name: str) -> torch.Tensor:
        if not isinstance(t, torch.Tensor) or t.device != self.device:
            raise ValueError(f"{name} must be a tensor on {self.device}")
        if t.dtype != self.dtype:
            raise ValueError(f"{name} must have dtype {self.dtype}")
        if t.numel() != numel or not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous with {numel} elements")
        return t

    def set_init(self, x0: torch.Tensor | None = None) -> None:
        self._x0_keep = None if x0 is None else self._dev(x0, self.geom.n, "x0")
        _check(self.lib.ncs_cone_set_init(self.h, None if x0 is None else self._x0_keep.data_ptr()))

    def iterate(self, k: int, record: bool = False) -> np.ndarray | None:
        if record:
            obj = np.empty(k, dtype=np.float64)
            _check(self.lib.ncs_cone_iterate(self.h, k, obj.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
            return obj
        _check(self.lib.ncs_cone_iterate(self.h, k, None))
        return None

    def _get(self, fn, numel: int) -> torch.Tensor:
        out = torch.empty(numel, dtype=self.dtype, device=self.device)
        _check(fn(self.h, out.data_ptr()))
        return out

    def x(self) -> torch.Tensor:
        return self._get(self.lib.ncs_cone_get_x, self.geom.n)

    def u(self) -> torch.Tensor:
        return self._get(self.lib.ncs_cone_get_u, self.geom.m)

    def v(self) -> torch.Tensor:
        return self._get(self.lib.ncs_cone_get_v, 3 * self.geom.n)

    def t(self) -> torch.Tensor:
        """The positivity dual t (params.positivity = 1 only)."""
        return self._get(self.lib.ncs_cone_get_t, self.geom.n)

    def get_state(self) -> bytes:
        n = ctypes.c_size_t()
        _check(self.lib.ncs_cone_get_state(self.h, None, ctypes.byref(n)))
        buf = ctypes.create_string_buffer(n.value)
        _check(self.lib.ncs_cone_get_state(self.h, buf, ctypes.byref(n)))
        return buf.raw[: n.value]

    def set_state(self, blob: bytes) -> None:
        buf = ctypes.create_string_buffer(blob, len(blob))
        _check(self.lib.ncs_cone_set_state(self.h, buf, len(blob)))

    def forward(self, x: torch.Tensor) -> torch.Tensor:
        y = torch.empty(self.geom.m, dtype=self.dtype, device=self.device)
        _check(self.lib.ncs_cone_forward(self.h, self._dev(x, self.geom.n, "x").data_ptr(), y.data_ptr()))
        return y

    def adjoint(self, y: torch.Tensor) -> torch.Tensor:
        x = torch.empty(self.geom.n, dtype=self.dtype, device=self.device)
        _check(self.lib.ncs_cone_adjoint(self.h, self._dev(y, self.geom.m, "y").data_ptr(), x.data_ptr()))
        return x

    def apply_minv(self, w: torch.Tensor) -> torch.Tensor:
        out = torch.empty(self.geom.n, dtype=self.dtype, device=self.device)
        _check(self.lib.ncs_cone_apply_minv(self.h, self._dev(w, self.geom.n, "w").data_ptr(), out.data_ptr()))
        return out

    def eigenvalues(self) -> np.ndarray:
        g = self.geom
        mu = np.empty(g.n, dtype=np.float64)
        _check(self.lib.ncs_cone_get_eigenvalues(self.h, mu.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return mu.reshape(g.n_slices, g.n_side, g.n_side)

    def info(self) -> dict:
        inf = _ConeInfo()
        _check(self.lib.ncs_cone_get_info(self.h, ctypes.byref(inf)))
        return {k: getattr(inf, k) for k, _ in _ConeInfo._fields_}

    def time_phases(self, iters: int = 20) -> dict:
        ms = np.zeros(5, dtype=np.float64)
        _check(self.lib.ncs_cone_time_phases(self.h, iters, ms.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return dict(zip(PHASES, ms.tolist()))

    def close(self) -> None:
        if getattr(self, "h", None) is not None and self.h.value:
            self.lib.ncs_cone_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def default_gamma(geom: ConeGeometry, alpha: float) -> float:
    """gamma = alpha N_v N / (2 pi): the fan beam's choice, the scale of E^T E's
    multiplier at the lowest frequencies per unit length of the rays."""
    return alpha * geom.n_views * geom.n_side / (2.0 * math.pi)
