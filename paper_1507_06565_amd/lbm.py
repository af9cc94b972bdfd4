"""Thin Python binding of the pore-scale C ABI (include/lbm.h).

Argument marshalling only: every step of the computation runs in the HIP
library.  torch provides the caller-owned device buffer and the stream.
"""
from __future__ import annotations

import ctypes as C
import dataclasses

import numpy as np
import torch

from ._lib import DomainDesc, LbmError, Params, Sphere, check, lib  # noqa: F401

BC = {"sbb": 0, "cli": 1, "bouzidi": 2}
COLLISION = {"bgk": 0, "trt": 1}
LAYOUT = {"twogrid": 0, "aa": 1, "brick": 2}
LAYOUT_NAME = {v: k for k, v in LAYOUT.items()}


def _desc(dom, keep):
    s = np.ascontiguousarray(np.asarray(dom.spheres, dtype=np.float64).reshape(-1, 4))
    keep.append(s)
    d = DomainDesc()
    d.nx, d.ny, d.nz = dom.nx, dom.ny, dom.nz
    d.periodic[:] = [int(v) for v in dom.periodic]
    d.wall_lo[:] = [int(v) for v in dom.wall_lo]
    d.wall_hi[:] = [int(v) for v in dom.wall_hi]
    d.wall_hi_velocity[:] = [float(v) for v in dom.wall_hi_velocity]
    d.spheres = s.ctypes.data if len(s) else None
    d.n_spheres = len(s)
    d.bc = BC[dom.bc]
    return d


def make_params(p) -> Params:
    q = Params()
    q.collision = COLLISION[p.collision]
    q.tau_plus = p.tau_plus
    q.magic_lambda = p.magic_lambda
    q.rho0 = p.rho0
    q.force[:] = [float(v) for v in p.force]
    q.layout = LAYOUT[p.layout]
    return q


class Geometry:
    """Owns an lbm_geometry*; built from workloads.Domain objects."""

    def __init__(self, domains):
        if not isinstance(domains, (list, tuple)):
            domains = [domains]
        keep = []
        arr = (DomainDesc * len(domains))(*[_desc(d, keep) for d in domains])
        ptr = C.c_void_p()
        check(lib.lbm_geometry_build(arr, len(domains), C.byref(ptr)), "lbm_geometry_build")
        self.ptr = ptr
        self.domains = list(domains)

    def __del__(self, _free=lib.lbm_geometry_free):
        if getattr(self, "ptr", None):
            _free(self.ptr)
            self.ptr = None

    def flags(self, dom=0):
        d = self.domains[dom]
        f = np.zeros((d.nz, d.ny, d.nx), np.uint8)
        check(lib.lbm_geometry_flags(self.ptr, dom, f.ctypes.data), "lbm_geometry_flags")
        return f

    def links(self, dom=0):
        n = C.c_int64(0)
        check(lib.lbm_geometry_links(self.ptr, dom, C.byref(n), None, None, None), "lbm_geometry_links")
        cell = np.zeros(n.value, np.int64)
        k = np.zeros(n.value, np.int8)
        q = np.zeros(n.value)
        check(lib.lbm_geometry_links(self.ptr, dom, C.byref(n), cell.ctypes.data, k.ctypes.data, q.ctypes.data),
              "lbm_geometry_links")
        return cell, k, q

    def info(self, dom=0):
        nd, nf, nl = C.c_int32(), C.c_int64(), C.c_int64()
        check(lib.lbm_geometry_info(self.ptr, dom, C.byref(nd), C.byref(nf), C.byref(nl)), "lbm_geometry_info")
        return nd.value, nf.value, nl.value


def required_bytes(geo: Geometry, params) -> int:
    b = C.c_int64()
    check(lib.lbm_required_bytes(geo.ptr, C.byref(make_params(params)), C.byref(b)), "lbm_required_bytes")
    return b.value


def autotune_layout(geo: Geometry, params, steps_per_trial=10, device="cuda", stream=None):
    """The fastest layout for this geometry and physics (lbm_autotune_layout),
    as (name, ms per step).  A choice cached in this process returns at once;
    otherwise a scratch buffer of lbm_autotune_layout_bytes is allocated for
    the trials and released."""
    q = make_params(dataclasses.replace(params, layout="twogrid"))
    s = stream if stream is not None else torch.cuda.current_stream(device)
    lay, ms = C.c_int32(), C.c_double()
    if lib.lbm_autotune_layout(geo.ptr, C.byref(q), None, 0, C.c_void_p(s.cuda_stream), steps_per_trial,
                               C.byref(lay), C.byref(ms)) == 0:
        return LAYOUT_NAME[lay.value], ms.value
    b = C.c_int64()
    check(lib.lbm_autotune_layout_bytes(geo.ptr, C.byref(q), C.byref(b)), "lbm_autotune_layout_bytes")
    buf = torch.empty(b.value, dtype=torch.uint8, device=s.device)
    check(lib.lbm_autotune_layout(geo.ptr, C.byref(q), C.c_void_p(buf.data_ptr()), b.value,
                                  C.c_void_p(s.cuda_stream), steps_per_trial, C.byref(lay), C.byref(ms)),
          "lbm_autotune_layout")
    del buf
    return LAYOUT_NAME[lay.value], ms.value


def tuning_export():
    """The autotuners' cached choices as text (lbm_tuning_export)."""
    n = C.c_int64()
    check(lib.lbm_tuning_export(None, 0, C.byref(n)), "lbm_tuning_export")
    buf = C.create_string_buffer(n.value + 1)
    check(lib.lbm_tuning_export(buf, n.value + 1, C.byref(n)), "lbm_tuning_export")
    return buf.value.decode()


def tuning_import(text):
    """Add cached choices from text written by tuning_export (lbm_tuning_import)."""
    check(lib.lbm_tuning_import(text.encode()), "lbm_tuning_import")


def save_tuning(path):
    with open(path, "w") as f:
        f.write(tuning_export())


def load_tuning(path):
    with open(path) as f:
        tuning_import(f.read())


def stream_probe(nbricks, grouped=False, passes=20, device="cuda", stream=None):
    """Milliseconds per pass of lbm_stream_probe: the brick sweep's population
    bytes for nbricks bricks (19 x 64 FP32 per brick read and written once),
    in the sweep's layout or grouped per brick; allocates the two buffers."""
    s = stream if stream is not None else torch.cuda.current_stream(device)
    n = int(nbricks) * 64 * 19
    a = torch.zeros(n, dtype=torch.float32, device=s.device)
    b = torch.empty_like(a)
    ms = C.c_double()
    check(lib.lbm_stream_probe(C.c_void_p(a.data_ptr()), C.c_void_p(b.data_ptr()), int(nbricks), int(bool(grouped)),
                               int(passes), C.c_void_p(s.cuda_stream), C.byref(ms)), "lbm_stream_probe")
    return ms.value


class Context:
    """Owns an lbm_ctx* and the torch tensor that backs its device memory.
    params.layout == "auto" picks the layout with autotune_layout first."""

    def __init__(self, geo: Geometry, params, device="cuda", stream=None, buffer=None):
        if params.layout == "auto":
            params = dataclasses.replace(params, layout=autotune_layout(geo, params, device=device,
                                                                         stream=stream)[0])
        nbytes = required_bytes(geo, params)
        if buffer is None:
            buffer = torch.empty(nbytes, dtype=torch.uint8, device=device)
        if buffer.numel() * buffer.element_size() < nbytes:
            raise ValueError("device buffer too small")
        self.buf = buffer
        self.stream = stream if stream is not None else torch.cuda.current_stream(buffer.device)
        self.params = params
        self.domains = geo.domains
        ptr = C.c_void_p()
        check(lib.lbm_init(geo.ptr, C.byref(make_params(params)), C.c_void_p(buffer.data_ptr()), nbytes,
                           C.c_void_p(self.stream.cuda_stream), C.byref(ptr)), "lbm_init")
        self.ptr = ptr
        self.nbytes = nbytes

    def __del__(self, _destroy=lib.lbm_destroy):
        if getattr(self, "ptr", None):
            _destroy(self.ptr)
            self.ptr = None

    # --- stepping
    def step(self, n=1):
        check(lib.lbm_step(self.ptr, int(n)), "lbm_step")

    def run_to_steady(self, rel_tol=1e-7, check_every=100, max_steps=2_000_000):
        nd = len(self.domains)
        out = np.zeros(nd, np.int64)
        check(lib.lbm_run_to_steady(self.ptr, rel_tol, check_every, max_steps, out.ctypes.data),
              "lbm_run_to_steady")
        return out

    def steps_done(self):
        s = C.c_int64()
        check(lib.lbm_steps_done(self.ptr, C.byref(s)), "lbm_steps_done")
        return s.value

    # --- results
    def average_profile(self, dom=0, axis=2, comp=0):
        d = self.domains[dom]
        n = (d.nx, d.ny, d.nz)[axis]
        sup, intr, por = np.zeros(n), np.zeros(n), np.zeros(n)
        check(lib.lbm_average_profile(self.ptr, dom, axis, comp, sup.ctypes.data, intr.ctypes.data,
                                      por.ctypes.data), "lbm_average_profile")
        return sup, intr, por

    def permeability(self, dom=0, flow_axis=0, z0=None, z1=None):
        d = self.domains[dom]
        z0 = 0 if z0 is None else z0
        z1 = d.nz if z1 is None else z1
        k = C.c_double()
        check(lib.lbm_permeability(self.ptr, dom, flow_axis, z0, z1, C.byref(k)), "lbm_permeability")
        return k.value

    def fields(self, dom=0):
        """(rho[nz, ny, nx], u[3, nz, ny, nx]) in FP64, 0 in solid cells."""
        d = self.domains[dom]
        rho = np.zeros((d.nz, d.ny, d.nx))
        u = np.zeros((3, d.nz, d.ny, d.nx))
        check(lib.lbm_fields(self.ptr, dom, rho.ctypes.data, u.ctypes.data), "lbm_fields")
        return rho, u

    def totals(self, dom=0):
        m = C.c_double()
        j = np.zeros(3)
        check(lib.lbm_totals(self.ptr, dom, C.byref(m), j.ctypes.data), "lbm_totals")
        return m.value, j

    # --- checkpoint
    def save(self) -> bytes:
        n = C.c_int64()
        check(lib.lbm_state_bytes(self.ptr, C.byref(n)), "lbm_state_bytes")
        buf = np.zeros(n.value, np.uint8)
        check(lib.lbm_save(self.ptr, buf.ctypes.data, n.value), "lbm_save")
        return buf

    def load(self, image):
        image = np.ascontiguousarray(image, dtype=np.uint8)
        check(lib.lbm_load(self.ptr, image.ctypes.data, image.size), "lbm_load")

    # --- launch configuration
    def set_launch(self, block, flags=1):
        """flags (lbm_set_launch): 1 = XCD-contiguous tiles, 2 = non-temporal
        aligned streams, 4 / 8 = two / four cells per thread."""
        check(lib.lbm_set_launch(self.ptr, block, flags), "lbm_set_launch")

    def get_launch(self):
        b, r = C.c_int32(), C.c_int32()
        check(lib.lbm_get_launch(self.ptr, C.byref(b), C.byref(r)), "lbm_get_launch")
        return b.value, r.value

    def batch_set_launch(self, block, workgroups_per_domain):
        """AA batches: workgroups stepping one domain together (1..64); brick
        batches: cells per thread (1, 2 or 4)."""
        check(lib.lbm_batch_set_launch(self.ptr, block, workgroups_per_domain), "lbm_batch_set_launch")

    def batch_get_launch(self):
        b, w = C.c_int32(), C.c_int32()
        check(lib.lbm_batch_get_launch(self.ptr, C.byref(b), C.byref(w)), "lbm_batch_get_launch")
        return b.value, w.value

    def autotune(self, steps_per_trial=20):
        check(lib.lbm_autotune(self.ptr, steps_per_trial), "lbm_autotune")
        return self.get_launch() if len(self.domains) == 1 else self.batch_get_launch()
