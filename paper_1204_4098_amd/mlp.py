"""ctypes binding of the sigma-surrogate network (C ABI in include/lbm_mlp.h).

Argument marshalling only; the forward pass, back-propagation and Adam run in
the library's HIP kernels.  PyTorch holds the device workspace and batches.
"""
from __future__ import annotations

import ctypes as C
import math

import numpy as np
import torch

from .lbm import LbmError, _check, lib as _lib_lbm

NPARAMS = 4546


class mlp_norm(C.Structure):
    _fields_ = [("in_mean", C.c_float * 3), ("in_std", C.c_float * 3),
                ("out_mean", C.c_float * 2), ("out_std", C.c_float * 2)]


_SIGS = {
    "mlp_workspace_bytes": (C.c_int, [C.c_int32, C.POINTER(C.c_size_t)]),
    "mlp_init": (C.c_int, [C.c_void_p, C.POINTER(mlp_norm), C.c_int32, C.c_void_p, C.c_size_t,
                           C.c_void_p, C.POINTER(C.c_void_p)]),
    "mlp_set_params": (C.c_int, [C.c_void_p, C.c_void_p]),
    "mlp_get_params": (C.c_int, [C.c_void_p, C.c_void_p]),
    "mlp_set_norm": (C.c_int, [C.c_void_p, C.POINTER(mlp_norm)]),
    "mlp_forward": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32]),
    "mlp_gradient": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p]),
    "mlp_adam": (C.c_int, [C.c_void_p, C.c_void_p, C.c_float, C.c_float, C.c_float, C.c_float]),
    "mlp_train_step": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_float, C.c_void_p]),
    "mlp_destroy": (C.c_int, [C.c_void_p]),
}
_ready = False


def lib():
    global _ready
    L = _lib_lbm()
    if not _ready:
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _ready = True
    return L


def make_norm(in_mean, in_std, out_mean, out_std) -> mlp_norm:
    n = mlp_norm()
    n.in_mean[:] = [float(v) for v in in_mean]
    n.in_std[:] = [float(v) for v in in_std]
    n.out_mean[:] = [float(v) for v in out_mean]
    n.out_std[:] = [float(v) for v in out_std]
    return n


def _dev(a, cols, device):
    t = torch.as_tensor(np.ascontiguousarray(a, dtype=np.float32), device=device)
    if t.ndim != 2 or t.shape[1] != cols:
        raise ValueError(f"expected an (n, {cols}) array")
    return t.contiguous()


class Mlp:
    """The surrogate network on the GPU (an mlp_ctx and its workspace)."""

    def __init__(self, params, norm: mlp_norm, max_batch: int, device="cuda:0", stream=None):
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.Stream(device=self.device)
        self.norm = norm
        self.max_batch = int(max_batch)
        n = C.c_size_t()
        _check(lib().mlp_workspace_bytes(self.max_batch, C.byref(n)), "mlp_workspace_bytes")
        self.workspace = torch.empty(n.value, dtype=torch.uint8, device=self.device)
        self.grad = torch.empty(NPARAMS, dtype=torch.float32, device=self.device)
        self.loss = torch.zeros(1, dtype=torch.float32, device=self.device)
        p = np.ascontiguousarray(params, dtype=np.float32)
        assert p.size == NPARAMS
        torch.cuda.synchronize(self.device)
        h = C.c_void_p()
        _check(lib().mlp_init(p.ctypes.data, C.byref(norm), self.max_batch, self.workspace.data_ptr(),
                              self.workspace.numel(), self.stream.cuda_stream, C.byref(h)), "mlp_init")
        self.ctx = h

    def params(self) -> np.ndarray:
        out = np.empty(NPARAMS, dtype=np.float32)
        _check(lib().mlp_get_params(self.ctx, out.ctypes.data), "mlp_get_params")
        return out

    def set_params(self, params):
        p = np.ascontiguousarray(params, dtype=np.float32)
        _check(lib().mlp_set_params(self.ctx, p.ctypes.data), "mlp_set_params")

    def forward(self, X) -> np.ndarray:
        Xd = X if isinstance(X, torch.Tensor) else _dev(X, 3, self.device)
        B = Xd.shape[0]
        Y = torch.empty((B, 2), dtype=torch.float32, device=self.device)
        torch.cuda.current_stream(self.device).synchronize()
        _check(lib().mlp_forward(self.ctx, Xd.data_ptr(), Y.data_ptr(), B), "mlp_forward")
        self.stream.synchronize()
        return Y.cpu().numpy()

    def gradient(self, X, T):
        Xd, Td = _dev(X, 3, self.device), _dev(T, 2, self.device)
        torch.cuda.current_stream(self.device).synchronize()
        _check(lib().mlp_gradient(self.ctx, Xd.data_ptr(), Td.data_ptr(), Xd.shape[0], self.grad.data_ptr(),
                                  self.loss.data_ptr()), "mlp_gradient")
        self.stream.synchronize()
        return float(self.loss.cpu()[0]), self.grad.cpu().numpy()

    def adam(self, grad, lr, beta1=0.9, beta2=0.999, eps=1e-8):
        g = torch.as_tensor(np.ascontiguousarray(grad, dtype=np.float32), device=self.device)
        torch.cuda.current_stream(self.device).synchronize()
        _check(lib().mlp_adam(self.ctx, g.data_ptr(), lr, beta1, beta2, eps), "mlp_adam")
        self.stream.synchronize()

    def train(self, X, T, steps: int, lr: float, batch: int, seed: int = 0, log_every: int = 0,
              cosine: bool = True):
        """Minibatch Adam on device-resident data (learning rate decayed by a half
        cosine when `cosine`); returns the loss history (sampled)."""
        Xd, Td = _dev(X, 3, self.device), _dev(T, 2, self.device)
        n = Xd.shape[0]
        batch = min(batch, n, self.max_batch)
        g = torch.Generator(device="cpu").manual_seed(seed)
        hist = []
        torch.cuda.current_stream(self.device).synchronize()
        nb = max(1, n // batch)
        perm = None
        for s in range(steps):
            k = s % nb
            with torch.cuda.stream(self.stream):
                if k == 0:
                    # each epoch's permutation is copied on the training stream, so
                    # the minibatch gathers below are ordered after the copy
                    perm = torch.randperm(n, generator=g).to(self.device)
                idx = perm[k * batch:(k + 1) * batch]
                xb = Xd.index_select(0, idx).contiguous()
                tb = Td.index_select(0, idx).contiguous()
                lr_s = lr * 0.5 * (1.0 + math.cos(math.pi * s / steps)) if cosine else lr
                _check(lib().mlp_train_step(self.ctx, xb.data_ptr(), tb.data_ptr(), xb.shape[0], lr_s,
                                            self.loss.data_ptr()), "mlp_train_step")
            if log_every and (s % log_every == 0 or s == steps - 1):
                self.stream.synchronize()
                hist.append((s, float(self.loss.cpu()[0])))
        self.stream.synchronize()
        return hist

    def close(self):
        if getattr(self, "ctx", None):
            lib().mlp_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
