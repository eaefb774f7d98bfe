"""Python binding of the warm-start network ABI (``include/ncs_cnn.h``).

Argument marshalling only: the convolutions, gradients, loss and Adam run in
the HIP library ``libncs.so``.  There is no fallback.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from .ncs import NcsError, _check, load_library

N_PARAMS = 37601
CHANNELS = 32
LAYERS = [(1, 32), (32, 32), (32, 32), (32, 32), (32, 32), (32, 1)]

CONV_RELU_BF16 = 0
CONV_RESID_F32 = 1
CONV_MASK_BF16 = 2
CONV_F32 = 3

EXPORTED = [
    "ncs_cnn_create", "ncs_cnn_set_params", "ncs_cnn_get_params", "ncs_cnn_forward", "ncs_cnn_gradient",
    "ncs_cnn_adam_step", "ncs_cnn_train_step", "ncs_cnn_last_loss", "ncs_cnn_destroy",
    "ncs_conv3x3_bf16", "ncs_conv3x3_wgrad_bf16", "ncs_to_bf16",
]

_bound = False


def _lib() -> ctypes.CDLL:
    global _bound
    lib = load_library()
    if not _bound:
        vp, i32, i64, f32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_float
        pdbl = ctypes.POINTER(ctypes.c_double)
        sigs = {
            "ncs_cnn_create": ([i32, i32, i32, vp, ctypes.POINTER(vp)], i32),
            "ncs_cnn_set_params": ([vp, vp], i32),
            "ncs_cnn_get_params": ([vp, vp], i32),
            "ncs_cnn_forward": ([vp, vp, vp, i32, i32, i32], i32),
            "ncs_cnn_gradient": ([vp, vp, vp, i32, i32, i32, pdbl, vp], i32),
            "ncs_cnn_adam_step": ([vp, f32, f32, f32, f32], i32),
            "ncs_cnn_train_step": ([vp, vp, vp, i32, i32, i32, f32, pdbl], i32),
            "ncs_cnn_last_loss": ([vp, pdbl], i32),
            "ncs_cnn_destroy": ([vp], None),
            "ncs_conv3x3_bf16": ([vp, vp, vp, vp, vp, vp, i32, i32, i32, i32, i32, i32, vp], i32),
            "ncs_conv3x3_wgrad_bf16": ([vp, vp, i32, i32, i32, i32, i32, vp, vp], i32),
            "ncs_to_bf16": ([vp, vp, i64, vp], i32),
        }
        for name, (args, res) in sigs.items():
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = res
        _bound = True
    return lib


def _dev_tensor(t: torch.Tensor, dtype: torch.dtype, numel: int, what: str) -> torch.Tensor:
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != dtype or not t.is_contiguous() \
            or t.numel() != numel:
        raise ValueError(f"{what} must be a contiguous {dtype} device tensor of {numel} elements")
    return t


def _ptr(t):
    return None if t is None else t.data_ptr()


class WarmStartNet:
    """The residual network x0 = z + N(z) with its training step."""

    def __init__(self, max_batch: int, max_height: int, max_width: int | None = None):
        if not torch.cuda.is_available():
            raise RuntimeError("the warm-start network needs a GPU; none is visible")
        self.lib = _lib()
        self.device = torch.device("cuda", torch.cuda.current_device())
        self.stream = torch.cuda.current_stream(self.device)
        self.max_batch, self.max_h = max_batch, max_height
        self.max_w = max_height if max_width is None else max_width
        h = ctypes.c_void_p()
        _check(self.lib.ncs_cnn_create(max_batch, self.max_h, self.max_w, self.stream.cuda_stream, ctypes.byref(h)))
        self.h = h

    def set_params(self, theta) -> None:
        a = np.ascontiguousarray(np.asarray(theta, dtype=np.float32).ravel())
        if a.size != N_PARAMS:
            raise ValueError(f"need {N_PARAMS} parameters, got {a.size}")
        _check(self.lib.ncs_cnn_set_params(self.h, a.ctypes.data))

    def params(self) -> np.ndarray:
        a = np.empty(N_PARAMS, dtype=np.float32)
        _check(self.lib.ncs_cnn_get_params(self.h, a.ctypes.data))
        return a

    def _batch(self, z: torch.Tensor):
        if z.dim() == 2:
            z = z.unsqueeze(0)
        if z.dim() != 3:
            raise ValueError("images must be [batch, height, width] or [height, width]")
        return z, z.shape[0], z.shape[1], z.shape[2]

    def forward(self, z: torch.Tensor) -> torch.Tensor:
        z3, B, H, W = self._batch(z)
        _dev_tensor(z3, torch.float32, B * H * W, "z")
        x0 = torch.empty_like(z3)
        _check(self.lib.ncs_cnn_forward(self.h, z3.data_ptr(), x0.data_ptr(), B, H, W))
        return x0.reshape(z.shape)

    def gradient(self, z: torch.Tensor, target: torch.Tensor):
        """(loss, gradient as a float32 numpy vector); the gradient also stays on the device."""
        z3, B, H, W = self._batch(z)
        _dev_tensor(z3, torch.float32, B * H * W, "z")
        _dev_tensor(target, torch.float32, B * H * W, "target")
        loss = ctypes.c_double()
        g = np.empty(N_PARAMS, dtype=np.float32)
        _check(self.lib.ncs_cnn_gradient(self.h, z3.data_ptr(), target.data_ptr(), B, H, W, ctypes.byref(loss),
                                         g.ctypes.data))
        return loss.value, g

    def adam_step(self, lr: float, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8) -> None:
        _check(self.lib.ncs_cnn_adam_step(self.h, lr, beta1, beta2, eps))

    def train_step(self, z: torch.Tensor, target: torch.Tensor, lr: float, want_loss: bool = False):
        z3, B, H, W = self._batch(z)
        _dev_tensor(z3, torch.float32, B * H * W, "z")
        _dev_tensor(target, torch.float32, B * H * W, "target")
        loss = ctypes.c_double()
        _check(self.lib.ncs_cnn_train_step(self.h, z3.data_ptr(), target.data_ptr(), B, H, W, lr,
                                           ctypes.byref(loss) if want_loss else None))
        return loss.value if want_loss else None

    def last_loss(self) -> float:
        loss = ctypes.c_double()
        _check(self.lib.ncs_cnn_last_loss(self.h, ctypes.byref(loss)))
        return loss.value

    def close(self) -> None:
        if getattr(self, "h", None) is not None and self.h.value:
            self.lib.ncs_cnn_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def conv3x3_bf16(x: torch.Tensor, w: torch.Tensor, bias: torch.Tensor | None, epilogue: int,
                 mask: torch.Tensor | None = None, resid: torch.Tensor | None = None) -> torch.Tensor:
    """One layer: x bfloat16 NHWC [B, H, W, c_in], w bfloat16 [9, c_out, c_in]."""
    lib = _lib()
    B, H, W, cin = x.shape
    cout = w.shape[1]
    if x.dtype != torch.bfloat16 or w.dtype != torch.bfloat16 or not x.is_contiguous() or not w.is_contiguous():
        raise ValueError("x and w must be contiguous bfloat16 tensors")
    if tuple(w.shape) != (9, cout, cin):
        raise ValueError("w must be [9, c_out, c_in]")
    if epilogue in (CONV_RELU_BF16, CONV_MASK_BF16):
        out = torch.empty((B, H, W, cout), dtype=torch.bfloat16, device=x.device)
    elif epilogue == CONV_RESID_F32:
        out = torch.empty((B, H, W), dtype=torch.float32, device=x.device)
    else:
        out = torch.empty((B, H, W, cout), dtype=torch.float32, device=x.device)
    st = torch.cuda.current_stream(x.device).cuda_stream
    _check(lib.ncs_conv3x3_bf16(x.data_ptr(), w.data_ptr(), _ptr(bias), _ptr(mask), _ptr(resid), out.data_ptr(),
                                B, H, W, cin, cout, epilogue, st))
    return out


def conv3x3_wgrad_bf16(x: torch.Tensor, dz: torch.Tensor) -> torch.Tensor:
    """Weight and bias gradient: float [9 c_out c_in + c_out]."""
    lib = _lib()
    B, H, W, cin = x.shape
    cout = dz.shape[3]
    if x.dtype != torch.bfloat16 or dz.dtype != torch.bfloat16 or not x.is_contiguous() or not dz.is_contiguous():
        raise ValueError("x and dz must be contiguous bfloat16 tensors")
    if tuple(dz.shape[:3]) != (B, H, W):
        raise ValueError("x and dz must share batch, height and width")
    g = torch.empty(9 * cout * cin + cout, dtype=torch.float32, device=x.device)
    st = torch.cuda.current_stream(x.device).cuda_stream
    _check(lib.ncs_conv3x3_wgrad_bf16(x.data_ptr(), dz.data_ptr(), B, H, W, cin, cout, g.data_ptr(), st))
    return g


def to_bf16(x: torch.Tensor) -> torch.Tensor:
    lib = _lib()
    if x.dtype != torch.float32 or not x.is_contiguous() or not x.is_cuda:
        raise ValueError("x must be a contiguous float32 device tensor")
    out = torch.empty(x.shape, dtype=torch.bfloat16, device=x.device)
    _check(lib.ncs_to_bf16(x.data_ptr(), out.data_ptr(), x.numel(), torch.cuda.current_stream(x.device).cuda_stream))
    return out


__all__ = ["WarmStartNet", "conv3x3_bf16", "conv3x3_wgrad_bf16", "to_bf16", "N_PARAMS", "LAYERS", "NcsError"]
