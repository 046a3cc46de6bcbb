"""Thin ctypes binding of the surrogate network's C-ABI (``include/alelb_mlp.h``).

Argument marshalling only: the forward and backward passes (BF16 matrix-core
products with FP32 accumulation), the loss gradient and Adam run in the HIP
kernels of ``libalelb.so``.  There is no CPU fallback.
"""

from __future__ import annotations

import ctypes as C

import numpy as np

from . import alelb

SYMBOLS = ["ale_mlp_create", "ale_mlp_destroy", "ale_mlp_info", "ale_mlp_set_params", "ale_mlp_get_params",
           "ale_mlp_forward", "ale_mlp_gradients", "ale_mlp_train_step", "ale_mlp_train_steps",
           "ale_mlp_gemm_bf16"]

_done = False


def load():
    global _done
    lib = alelb.load()
    if not _done:
        vp, i32, i64, f32 = C.c_void_p, C.c_int32, C.c_int64, C.c_float
        sig = {
            "ale_mlp_create": [vp, i32, i32, vp, C.POINTER(vp)],
            "ale_mlp_info": [vp, vp, i32],
            "ale_mlp_set_params": [vp, vp, i64],
            "ale_mlp_get_params": [vp, vp, i64],
            "ale_mlp_forward": [vp, vp, i32, vp, i32],
            "ale_mlp_gradients": [vp, vp, vp, i32, vp, vp, i32],
            "ale_mlp_train_step": [vp, vp, vp, i32, f32, f32, f32, f32, vp, i32],
            "ale_mlp_train_steps": [vp, vp, vp, i32, i32, vp, f32, f32, f32, vp, i32],
            "ale_mlp_gemm_bf16": [vp, vp, vp, i32, i32, i32],
        }
        for name, args in sig.items():
            f = getattr(lib, name)
            f.argtypes = args
            f.restype = i32
        lib.ale_mlp_destroy.argtypes = [vp]
        lib.ale_mlp_destroy.restype = None
        _done = True
    return lib


def _p(a):
    return a.ctypes.data_as(C.c_void_p)


def _check(code):
    if code != 0:
        raise alelb.AleLbError(code, load().ale_lb_last_error().decode())


class MLP:
    """Fully connected network (tanh hidden layers, linear output) on the GPU."""

    def __init__(self, widths, max_batch: int, stream=None):
        lib = load()
        self.widths = [int(w) for w in widths]
        self.max_batch = int(max_batch)
        w = np.asarray(self.widths, dtype=np.int32)
        h = C.c_void_p()
        if stream is None:
            stream = alelb.current_stream()
        _check(lib.ale_mlp_create(_p(w), len(self.widths), self.max_batch, stream, C.byref(h)))
        self.h = h
        out = np.zeros(2, dtype=np.int64)
        _check(lib.ale_mlp_info(self.h, _p(out), 2))
        self.n_params = int(out[0])

    def close(self):
        if getattr(self, "h", None):
            load().ale_mlp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:  # interpreter teardown: the library may already be gone
            pass

    def set_params(self, params):
        p = np.ascontiguousarray(params, dtype=np.float32)
        _check(load().ale_mlp_set_params(self.h, _p(p), p.size))

    def params(self) -> np.ndarray:
        p = np.empty(self.n_params, dtype=np.float32)
        _check(load().ale_mlp_get_params(self.h, _p(p), p.size))
        return p

    def forward(self, x) -> np.ndarray:
        x = np.ascontiguousarray(x, dtype=np.float32)
        y = np.empty((x.shape[0], self.widths[-1]), dtype=np.float32)
        _check(load().ale_mlp_forward(self.h, _p(x), x.shape[0], _p(y), 0))
        return y

    def gradients(self, x, t):
        x = np.ascontiguousarray(x, dtype=np.float32)
        t = np.ascontiguousarray(t, dtype=np.float32)
        g = np.empty(self.n_params, dtype=np.float32)
        loss = C.c_double(0.0)
        _check(load().ale_mlp_gradients(self.h, _p(x), _p(t), x.shape[0], _p(g), C.byref(loss), 0))
        return loss.value, g

    def train_step(self, x, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8) -> float:
        x = np.ascontiguousarray(x, dtype=np.float32)
        t = np.ascontiguousarray(t, dtype=np.float32)
        loss = C.c_double(0.0)
        _check(load().ale_mlp_train_step(self.h, _p(x), _p(t), x.shape[0], lr, beta1, beta2, eps,
                                         C.byref(loss), 0))
        return loss.value

    def train_step_device(self, x_ptr: int, t_ptr: int, batch: int, lr=1e-3, beta1=0.9, beta2=0.999,
                          eps=1e-8) -> float:
        loss = C.c_double(0.0)
        _check(load().ale_mlp_train_step(self.h, C.c_void_p(x_ptr), C.c_void_p(t_ptr), int(batch), lr, beta1,
                                         beta2, eps, C.byref(loss), 1))
        return loss.value

    def train_steps(self, x, t, lrs, beta1=0.9, beta2=0.999, eps=1e-8, on_device=False, batch=None) -> np.ndarray:
        """len(lrs) Adam steps on one batch without a host synchronization per
        step; returns the loss before each step.  With on_device, x and t are
        device pointers and batch gives the row count."""
        lrs = np.ascontiguousarray(lrs, dtype=np.float32)
        losses = np.empty(lrs.shape[0])
        if on_device:
            xp, tp, n = C.c_void_p(x), C.c_void_p(t), int(batch)
        else:
            x = np.ascontiguousarray(x, dtype=np.float32)
            t = np.ascontiguousarray(t, dtype=np.float32)
            xp, tp, n = _p(x), _p(t), x.shape[0]
        _check(load().ale_mlp_train_steps(self.h, xp, tp, n, lrs.shape[0], _p(lrs), beta1, beta2, eps,
                                          _p(losses), 1 if on_device else 0))
        return losses


def gemm_bf16(a_bits_ptr: int, b_bits_ptr: int, c_ptr: int, M: int, N: int, K: int):
    """C [M][N] = A [M][K] B [K][N] on device pointers (BF16 bit patterns in, FP32 out)."""
    _check(load().ale_mlp_gemm_bf16(C.c_void_p(a_bits_ptr), C.c_void_p(b_bits_ptr), C.c_void_p(c_ptr),
                                    int(M), int(N), int(K)))


def ale_mlp_create(widths, max_batch, stream=None) -> MLP:
    return MLP(widths, max_batch, stream)
