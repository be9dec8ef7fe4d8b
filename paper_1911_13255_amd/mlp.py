"""ctypes binding of the surrogate network (include/mrsph_mlp.h).

Argument marshalling only: every forward, error and update pass runs in the
library's HIP kernels; torch provides device memory and the stream.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import sph

HIDDEN = 128


def _bind(L):
    if getattr(L, "_mlp_bound", False):
        return L
    vp = C.c_void_p
    L.mlp_arena_bytes.restype = C.c_size_t
    L.mlp_arena_bytes.argtypes = [C.c_int, C.c_int, C.c_int]
    L.mlp_init.argtypes = [C.c_int, C.c_int, C.c_int, vp, C.c_size_t, vp, C.POINTER(vp)]
    L.mlp_param_count.restype = C.c_size_t
    L.mlp_param_count.argtypes = [vp]
    for name in ("mlp_set_params", "mlp_get_params", "mlp_get_grads"):
        getattr(L, name).argtypes = [vp, C.POINTER(C.c_float), C.c_size_t]
    L.mlp_forward.argtypes = [vp, vp, vp, C.c_int]
    L.mlp_backward.argtypes = [vp, vp, vp, C.c_int, C.POINTER(C.c_double)]
    L.mlp_adam.argtypes = [vp, C.c_float, C.c_float, C.c_float, C.c_float]
    L.mlp_train_step.argtypes = [vp, vp, vp, C.c_int, C.c_float, C.c_float, C.c_float, C.c_float,
                                 C.POINTER(C.c_double)]
    L.mlp_sync.argtypes = [vp]
    L.mlp_destroy.argtypes = [vp]
    L.mlp_destroy.restype = None
    L._mlp_bound = True
    return L


def layer_shapes(in_dim: int, out_dim: int):
    return [(in_dim, HIDDEN), (HIDDEN, HIDDEN), (HIDDEN, HIDDEN), (HIDDEN, out_dim)]


def flatten(params) -> np.ndarray:
    """[(W1, b1), ..., (W4, b4)] -> FP32 vector in the library's order."""
    return np.concatenate([np.concatenate([np.asarray(W, np.float32).reshape(-1), np.asarray(b, np.float32)])
                           for W, b in params]).astype(np.float32)


def unflatten(vec, in_dim: int, out_dim: int):
    out, o = [], 0
    for k, n in layer_shapes(in_dim, out_dim):
        W = vec[o:o + k * n].reshape(k, n)
        o += k * n
        b = vec[o:o + n]
        o += n
        out.append((W.copy(), b.copy()))
    return out


class Network:
    """The in_dim -> 128 -> 128 -> 128 -> out_dim SiLU network on one GPU."""

    def __init__(self, in_dim: int, out_dim: int, max_rows: int, device: int = 0, stream=None):
        import torch

        self.L = _bind(sph.lib())
        self.in_dim, self.out_dim, self.max_rows = int(in_dim), int(out_dim), int(max_rows)
        nbytes = self.L.mlp_arena_bytes(self.in_dim, self.out_dim, self.max_rows)
        if nbytes == 0:
            raise sph.SphError(sph.SPH_E_ARG, "invalid network sizes")
        self.device = torch.device("cuda", device)
        with torch.cuda.device(self.device):
            self.stream = stream if stream is not None else torch.cuda.Stream(device=self.device)
            self.arena = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        torch.cuda.synchronize(self.device)
        ctx = C.c_void_p()
        rc = self.L.mlp_init(self.in_dim, self.out_dim, self.max_rows, C.c_void_p(self.arena.data_ptr()),
                             nbytes + 256, C.c_void_p(self.stream.cuda_stream), C.byref(ctx))
        if rc != sph.SPH_OK:
            raise sph.SphError(rc, "mlp_init failed")
        self.ctx = ctx
        self.n = int(self.L.mlp_param_count(ctx))

    def _check(self, rc):
        if rc != sph.SPH_OK:
            raise sph.SphError(rc, "network call failed")

    # The library works on its own stream: it waits for torch's current
    # stream before a call (inputs written there) and torch's current stream
    # waits for it afterwards (outputs read there).
    def _enter(self):
        import torch

        self.stream.wait_stream(torch.cuda.current_stream(self.device))

    def _leave(self):
        import torch

        torch.cuda.current_stream(self.device).wait_stream(self.stream)

    def _rows(self, x):
        import torch

        assert x.is_cuda and x.dtype == torch.float32 and x.is_contiguous()
        rows = x.shape[0]
        if not 1 <= rows <= self.max_rows:
            raise sph.SphError(sph.SPH_E_ARG, f"rows {rows} outside [1, {self.max_rows}]")
        return rows

    def set_params(self, params):
        vec = flatten(params)
        assert vec.size == self.n
        self._check(self.L.mlp_set_params(self.ctx, vec.ctypes.data_as(C.POINTER(C.c_float)), self.n))

    def _get(self, fn):
        vec = np.empty(self.n, np.float32)
        self._check(fn(self.ctx, vec.ctypes.data_as(C.POINTER(C.c_float)), self.n))
        return unflatten(vec, self.in_dim, self.out_dim)

    def get_params(self):
        return self._get(self.L.mlp_get_params)

    def grads(self):
        return self._get(self.L.mlp_get_grads)

    def forward(self, x, out=None):
        import torch

        rows = self._rows(x)
        y = out if out is not None else torch.empty((rows, self.out_dim), dtype=torch.float32, device=x.device)
        self._enter()
        self._check(self.L.mlp_forward(self.ctx, C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr()), rows))
        self._leave()
        return y

    def backward(self, x, t, want_loss: bool = True):
        rows = self._rows(x)
        assert t.shape == (rows, self.out_dim) and t.is_contiguous()
        loss = C.c_double(0.0)
        self._enter()
        self._check(self.L.mlp_backward(self.ctx, C.c_void_p(x.data_ptr()), C.c_void_p(t.data_ptr()), rows,
                                        C.byref(loss) if want_loss else None))
        self._leave()
        return loss.value if want_loss else None

    def adam(self, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self._check(self.L.mlp_adam(self.ctx, lr, b1, b2, eps))

    def train_step(self, x, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8, want_loss: bool = False):
        rows = self._rows(x)
        loss = C.c_double(0.0)
        self._enter()
        self._check(self.L.mlp_train_step(self.ctx, C.c_void_p(x.data_ptr()), C.c_void_p(t.data_ptr()), rows, lr,
                                          b1, b2, eps, C.byref(loss) if want_loss else None))
        self._leave()
        return loss.value if want_loss else None

    def sync(self):
        self._check(self.L.mlp_sync(self.ctx))

    def close(self):
        if getattr(self, "ctx", None):
            self.L.mlp_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
