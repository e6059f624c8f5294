"""Python side of the warm-start network (include/adr_cnn.h): argument
marshalling only; the convolutions, loss, gradients and Adam run in the
library's HIP kernels."""
import ctypes

import numpy as np

from . import _lib


def param_count():
    return int(_lib.load().adr_cnn_param_count())


def _torch():
    import torch
    return torch


def _stream_handle(stream):
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _dev(t, dtype, shape, name):
    torch = _torch()
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == dtype):
        raise TypeError("%s must be a CUDA %s tensor" % (name, dtype))
    if tuple(t.shape) != tuple(shape) or not t.is_contiguous():
        raise ValueError("%s must be contiguous with shape %s (got %s)" % (name, tuple(shape), tuple(t.shape)))
    return ctypes.c_void_p(t.data_ptr())


class WarmStartNet:
    """Six-layer 3x3 convolutional network on (ny+2) x (nx+2) node grids."""

    def __init__(self, height, width, max_batch, stream=None):
        self.H, self.W, self.max_batch = int(height), int(width), int(max_batch)
        self._h = ctypes.c_void_p()
        _lib.check(_lib.load().adr_cnn_create(self.H, self.W, self.max_batch, _stream_handle(stream),
                                              ctypes.byref(self._h)))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            try:
                _lib.load().adr_cnn_destroy(h)
            except (AttributeError, TypeError):   # interpreter shutdown
                pass
            self._h = None

    def close(self):
        self.__del__()

    def set_params(self, params):
        p = np.ascontiguousarray(params, dtype=np.float32).ravel()
        if p.size != param_count():
            raise ValueError("expected %d parameters (got %d)" % (param_count(), p.size))
        _lib.check(_lib.load().adr_cnn_set_params(self._h, p.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))

    def get_params(self):
        p = np.zeros(param_count(), dtype=np.float32)
        _lib.check(_lib.load().adr_cnn_get_params(self._h, p.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))
        return p

    def _in(self, x):
        torch = _torch()
        return _dev(x, torch.bfloat16, (x.shape[0], self.H, self.W, 32), "input")

    def forward(self, x, out=None):
        """x: bfloat16 [B, H, W, 32] -> float32 [B, H, W]."""
        torch = _torch()
        B = int(x.shape[0])
        u = out if out is not None else torch.empty((B, self.H, self.W), dtype=torch.float32, device="cuda")
        _lib.check(_lib.load().adr_cnn_forward(self._h, self._in(x), B, _dev(u, torch.float32, (B, self.H, self.W),
                                                                               "out")))
        return u

    def gradient(self, x, target, want_u=False):
        """Loss, packed gradient (float32 numpy) and optionally the output."""
        torch = _torch()
        B = int(x.shape[0])
        tp = _dev(target, torch.float32, (B, self.H - 2, self.W - 2), "target")
        g = np.zeros(param_count(), dtype=np.float32)
        loss = ctypes.c_double(0.0)
        u = torch.empty((B, self.H, self.W), dtype=torch.float32, device="cuda") if want_u else None
        up = None if u is None else ctypes.c_void_p(u.data_ptr())
        _lib.check(_lib.load().adr_cnn_gradient(self._h, self._in(x), tp, B, up,
                                                g.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                                ctypes.byref(loss)))
        return (loss.value, g, u) if want_u else (loss.value, g)

    def adam(self, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        _lib.check(_lib.load().adr_cnn_adam(self._h, float(lr), float(beta1), float(beta2), float(eps)))

    def train_step(self, x, target, lr=1e-3):
        torch = _torch()
        B = int(x.shape[0])
        tp = _dev(target, torch.float32, (B, self.H - 2, self.W - 2), "target")
        loss = ctypes.c_double(0.0)
        _lib.check(_lib.load().adr_cnn_train_step(self._h, self._in(x), tp, B, float(lr), ctypes.byref(loss)))
        return loss.value
