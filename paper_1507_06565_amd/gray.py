"""Thin Python binding of the gray-column C ABI (include/gray.h).

Argument marshalling only; the model runs in the HIP library.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from ._lib import check, lib


def _arr(a, ncols, nz):
    a = np.ascontiguousarray(np.broadcast_to(np.asarray(a, dtype=np.float64), (ncols, nz)))
    return a


class GrayColumns:
    """ncols independent 1 x 1 x nz columns; eps, nu_eff, drag: (ncols, nz)."""

    def __init__(self, eps, nu_eff, drag, G=(0.0, 0.0, 0.0), walls=True, lid=None, magic_lambda=3.0 / 16.0,
                 rho0=1.0, device="cuda", stream=None, precision=64):
        eps = np.atleast_2d(np.asarray(eps, dtype=np.float64))
        self.ncols, self.nz = eps.shape
        self._eps = _arr(eps, self.ncols, self.nz)
        self._nue = _arr(nu_eff, self.ncols, self.nz)
        self._drag = _arr(drag, self.ncols, self.nz)
        nb = C.c_int64()
        check(lib.gray_required_bytes(self.ncols, self.nz, C.byref(nb)), "gray_required_bytes")
        self.buf = torch.empty(nb.value, dtype=torch.uint8, device=device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.buf.device)
        g = np.asarray(G, dtype=np.float64)
        lw = None if lid is None else np.asarray(lid, dtype=np.float64)
        ptr = C.c_void_p()
        check(lib.gray_init(self.ncols, self.nz, int(bool(walls)), self._eps.ctypes.data, self._nue.ctypes.data,
                            self._drag.ctypes.data, magic_lambda, rho0, g.ctypes.data,
                            None if lw is None else lw.ctypes.data, C.c_void_p(self.buf.data_ptr()), nb.value,
                            C.c_void_p(self.stream.cuda_stream), C.byref(ptr)), "gray_init")
        self.ptr = ptr
        if precision != 64:
            self.set_precision(precision)

    def set_precision(self, bits):
        """Working precision of the kernel, 64 (default) or 32 bits (gray_set_precision)."""
        check(lib.gray_set_precision(self.ptr, int(bits)), "gray_set_precision")

    def __del__(self, _destroy=lib.gray_destroy):
        if getattr(self, "ptr", None):
            _destroy(self.ptr)
            self.ptr = None

    def set_cells(self, eps, nu_eff, drag):
        self._eps = _arr(eps, self.ncols, self.nz)
        self._nue = _arr(nu_eff, self.ncols, self.nz)
        self._drag = _arr(drag, self.ncols, self.nz)
        check(lib.gray_set_cells(self.ptr, self._eps.ctypes.data, self._nue.ctypes.data, self._drag.ctypes.data),
              "gray_set_cells")

    def set_forchheimer(self, phi):
        """Per-cell Forchheimer coefficients eps F_eps / sqrt(K) (None: off)."""
        if phi is None:
            check(lib.gray_set_forchheimer(self.ptr, None), "gray_set_forchheimer")
            return
        self._phi = _arr(phi, self.ncols, self.nz)
        check(lib.gray_set_forchheimer(self.ptr, self._phi.ctypes.data), "gray_set_forchheimer")

    def reset(self):
        check(lib.gray_reset(self.ptr), "gray_reset")

    def run(self, nsteps):
        check(lib.gray_run(self.ptr, int(nsteps)), "gray_run")

    def run_to_steady(self, rel_tol=1e-7, check_every=100, max_steps=2_000_000):
        out = np.zeros(self.ncols, np.int64)
        check(lib.gray_run_to_steady(self.ptr, rel_tol, check_every, max_steps, out.ctypes.data), "gray_run_to_steady")
        return out

    def profile(self, col=0):
        u = np.zeros((self.nz, 3))
        check(lib.gray_profile(self.ptr, col, u.ctypes.data), "gray_profile")
        return u
