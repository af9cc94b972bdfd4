"""Thin Python binding of the closure-network C ABI (include/mlp.h).

Argument marshalling only: forward, backward, loss, Adam, windows and the
closure map all run in the HIP library.  torch provides device memory.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from ._lib import check, lib

NPARAM = 43408
ROWS = 64


def init_params(seed=0):
    """Initial FP32 parameter vector: normal weights scaled by 1/sqrt(fan-in)
    (x sqrt(2) before the GELU layers), zero biases, zero padding rows and
    columns; the last layer starts small so the closure starts near
    (nu_eff, drag) = (nu, (1 - eps) log 2)."""
    rng = np.random.default_rng(seed)
    p = np.zeros(NPARAM, np.float32)
    o = 0
    for k, n, used_k, used_n, gain in ((64, 128, 33, 128, 2.0), (128, 128, 128, 128, 2.0),
                                       (128, 128, 128, 128, 2.0), (128, 16, 128, 2, 0.1)):
        w = np.zeros((k, n), np.float32)
        w[:used_k, :used_n] = rng.standard_normal((used_k, used_n)) * np.sqrt(gain / used_k)
        p[o:o + k * n] = w.ravel()
        o += k * n + n  # weights, then the (zero) biases
    assert o == NPARAM
    return p


def _p(t):
    return C.c_void_p(t.data_ptr())


class ClosureNet:
    def __init__(self, params=None, device="cuda", stream=None):
        self.dev = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.dev)
        p = np.zeros(NPARAM, np.float32) if params is None else np.asarray(params, np.float32)
        assert p.shape == (NPARAM,)
        self.params = torch.from_numpy(p.copy()).to(self.dev)
        self.pbf = torch.empty(2 * NPARAM, dtype=torch.bfloat16, device=self.dev)
        self.m = torch.zeros(NPARAM, dtype=torch.float32, device=self.dev)
        self.v = torch.zeros(NPARAM, dtype=torch.float32, device=self.dev)
        self.grad = torch.zeros(NPARAM, dtype=torch.float32, device=self.dev)
        self.t = 0
        self._ws = None
        self._wsB = 0
        check(lib.mlp_pack_bf16(_p(self.params), _p(self.pbf), C.c_void_p(self.stream.cuda_stream)), "mlp_pack_bf16")

    @property
    def s(self):
        return C.c_void_p(self.stream.cuda_stream)

    def set_params(self, p):
        self.params.copy_(torch.as_tensor(np.asarray(p, np.float32)))
        torch.cuda.synchronize(self.dev)
        check(lib.mlp_pack_bf16(_p(self.params), _p(self.pbf), self.s), "mlp_pack_bf16")

    def workspace(self, B):
        if self._ws is None or self._wsB < B:
            n = C.c_int64()
            check(lib.mlp_workspace_bytes(B, C.byref(n)), "mlp_workspace_bytes")
            self._ws = torch.empty(n.value, dtype=torch.uint8, device=self.dev)
            self._wsB = B
        return self._ws

    def forward(self, x_bf16, train=False):
        B = x_bf16.shape[0]
        y = torch.empty((B, 16), dtype=torch.float32, device=self.dev)
        ws = _p(self.workspace(B)) if train else None
        check(lib.mlp_forward(_p(self.params), _p(self.pbf), _p(x_bf16), B, _p(y), ws, self.s), "mlp_forward")
        return y

    def backward(self, x_bf16, dy, want_dx=False):
        B = x_bf16.shape[0]
        dx = torch.empty((B, 64), dtype=torch.float32, device=self.dev) if want_dx else None
        check(lib.mlp_backward(_p(self.params), _p(self.pbf), _p(x_bf16), _p(self.workspace(B)), _p(dy), B,
                               _p(self.grad), None if dx is None else _p(dx), self.s), "mlp_backward")
        return self.grad, dx

    def loss(self, y, target, mask, mask_sum):
        B = y.shape[0]
        dy = torch.empty_like(y)
        part = torch.empty((B + 255) // 256, dtype=torch.float64, device=self.dev)
        L = C.c_double()
        check(lib.mlp_loss(_p(y), _p(target), _p(mask), B, float(mask_sum), _p(dy), _p(part), C.byref(L), self.s),
              "mlp_loss")
        return L.value, dy

    def adam(self, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.t += 1
        check(lib.mlp_adam_step(_p(self.params), _p(self.pbf), _p(self.m), _p(self.v), _p(self.grad), lr, b1, b2, eps,
                                self.t, self.s), "mlp_adam_step")

    def train_step(self, x_bf16, target, mask, mask_sum, lr=1e-3):
        y = self.forward(x_bf16, train=True)
        L, dy = self.loss(y, target, mask, mask_sum)
        self.backward(x_bf16, dy)
        self.adam(lr)
        return L

    def profile_loss(self, y, eps, u_target, nprof, nz, nu, G, weight=1.0, dy=None):
        """Loss of nprof profiles through the steady gray column; dL/dy goes
        to rows [0, nprof*nz) of dy (allocated like y if None).  Returns
        (per-profile losses as numpy, dy)."""
        if dy is None:
            dy = torch.zeros_like(y)
        e = torch.as_tensor(np.ascontiguousarray(eps, np.float64) if isinstance(eps, np.ndarray) else eps,
                            dtype=torch.float64, device=self.dev).contiguous()
        t = torch.as_tensor(np.ascontiguousarray(u_target, np.float64) if isinstance(u_target, np.ndarray)
                            else u_target, dtype=torch.float64, device=self.dev).contiguous()
        assert y.shape[0] >= nprof * nz and e.numel() == nprof * nz and t.numel() == nprof * nz
        loss = torch.empty(nprof, dtype=torch.float64, device=self.dev)
        check(lib.mlp_profile_loss(_p(y), _p(e), _p(t), nprof, nz, nu, G, weight, _p(dy), _p(loss), self.s),
              "mlp_profile_loss")
        return loss.cpu().numpy(), dy

    def windows(self, eps_cols):
        """eps_cols: (ncols, nz) FP64 numpy -> BF16 inputs (rows padded to 64)."""
        eps_cols = np.atleast_2d(np.ascontiguousarray(eps_cols, dtype=np.float64))
        ncols, nz = eps_cols.shape
        n = ncols * nz
        npad = (n + ROWS - 1) // ROWS * ROWS
        e = torch.from_numpy(eps_cols).to(self.dev)
        x = torch.zeros((npad, 64), dtype=torch.bfloat16, device=self.dev)
        check(lib.mlp_windows(_p(e), ncols, nz, _p(x), self.s), "mlp_windows")
        return x, n

    def closure(self, eps_cols, nu):
        """(nu_eff, drag) arrays shaped like eps_cols, computed on the GPU."""
        eps_cols = np.atleast_2d(eps_cols)
        x, n = self.windows(eps_cols)
        y = self.forward(x)
        nue = torch.empty(n, dtype=torch.float64, device=self.dev)
        drag = torch.empty(n, dtype=torch.float64, device=self.dev)
        e = torch.from_numpy(np.ascontiguousarray(eps_cols, dtype=np.float64).ravel()).to(self.dev)
        check(lib.mlp_closure(_p(y), _p(e), n, nu, _p(nue), _p(drag), self.s), "mlp_closure")
        return nue.cpu().numpy().reshape(eps_cols.shape), drag.cpu().numpy().reshape(eps_cols.shape)
