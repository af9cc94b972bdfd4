"""ctypes loader of libmi355lbm.so (built in-tree by csrc/build.py).

torch is imported first so that the HIP runtime it loads is the one the
library binds to (both use the soname libamdhip64.so.7).  There is no CPU
fallback: if the library is missing, importing this module raises.
"""
import ctypes as C
import os

import torch  # noqa: F401  (loads the HIP runtime shared with the library)

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmi355lbm.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1507_06565_amd.csrc.build` "
                      "(or __graft_entry__.build()); there is no fallback path")

lib = C.CDLL(LIB_PATH)


class Sphere(C.Structure):
    _fields_ = [("cx", C.c_double), ("cy", C.c_double), ("cz", C.c_double), ("r", C.c_double)]


class DomainDesc(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("periodic", C.c_int32 * 3), ("wall_lo", C.c_int32 * 3), ("wall_hi", C.c_int32 * 3),
                ("wall_hi_velocity", C.c_double * 3), ("spheres", C.c_void_p), ("n_spheres", C.c_int64),
                ("bc", C.c_int32)]


class Params(C.Structure):
    _fields_ = [("collision", C.c_int32), ("tau_plus", C.c_double), ("magic_lambda", C.c_double),
                ("rho0", C.c_double), ("force", C.c_double * 3), ("layout", C.c_int32)]


P = C.POINTER
vp = C.c_void_p
i32, i64, f64 = C.c_int32, C.c_int64, C.c_double

_sig = {
    "lbm_last_error": ([], C.c_char_p),
    "lbm_geometry_build": ([P(DomainDesc), i32, P(vp)], i32),
    "lbm_geometry_flags": ([vp, i32, vp], i32),
    "lbm_geometry_links": ([vp, i32, P(i64), vp, vp, vp], i32),
    "lbm_geometry_info": ([vp, i32, P(i32), P(i64), P(i64)], i32),
    "lbm_geometry_free": ([vp], None),
    "lbm_required_bytes": ([vp, P(Params), P(i64)], i32),
    "lbm_init": ([vp, P(Params), vp, i64, vp, P(vp)], i32),
    "lbm_step": ([vp, i64], i32),
    "lbm_run_to_steady": ([vp, f64, i64, i64, vp], i32),
    "lbm_average_profile": ([vp, i32, i32, i32, vp, vp, vp], i32),
    "lbm_permeability": ([vp, i32, i32, i32, i32, P(f64)], i32),
    "lbm_fields": ([vp, i32, vp, vp], i32),
    "lbm_totals": ([vp, i32, P(f64), vp], i32),
    "lbm_state_bytes": ([vp, P(i64)], i32),
    "lbm_save": ([vp, vp, i64], i32),
    "lbm_load": ([vp, vp, i64], i32),
    "lbm_steps_done": ([vp, P(i64)], i32),
    "lbm_set_launch": ([vp, i32, i32], i32),
    "lbm_get_launch": ([vp, P(i32), P(i32)], i32),
    "lbm_autotune": ([vp, i32], i32),
    "lbm_autotune_layout_bytes": ([vp, P(Params), P(i64)], i32),
    "lbm_autotune_layout": ([vp, P(Params), vp, i64, vp, i32, P(i32), P(f64)], i32),
    "lbm_stream_probe": ([vp, vp, i64, i32, i32, vp, P(f64)], i32),
    "lbm_tuning_export": ([C.c_char_p, i64, P(i64)], i32),
    "lbm_tuning_import": ([C.c_char_p], i32),
    "lbm_batch_set_launch": ([vp, i32, i32], i32),
    "lbm_batch_get_launch": ([vp, P(i32), P(i32)], i32),
    "lbm_destroy": ([vp], None),
    # gray columns (include/gray.h)
    "gray_required_bytes": ([i32, i32, P(i64)], i32),
    "gray_init": ([i32, i32, i32, vp, vp, vp, f64, f64, vp, vp, vp, i64, vp, P(vp)], i32),
    "gray_set_cells": ([vp, vp, vp, vp], i32),
    "gray_reset": ([vp], i32),
    "gray_run": ([vp, i64], i32),
    "gray_run_to_steady": ([vp, f64, i64, i64, vp], i32),
    "gray_set_precision": ([vp, i32], i32),
    "gray_profile": ([vp, i32, vp], i32),
    "gray_destroy": ([vp], None),
    # closure network (include/mlp.h)
    "mlp_workspace_bytes": ([i64, P(i64)], i32),
    "mlp_pack_bf16": ([vp, vp, vp], i32),
    "mlp_forward": ([vp, vp, vp, i64, vp, vp, vp], i32),
    "mlp_backward": ([vp, vp, vp, vp, vp, i64, vp, vp, vp], i32),
    "mlp_loss": ([vp, vp, vp, i64, f64, vp, vp, P(f64), vp], i32),
    "mlp_loss_noalloc": ([vp, vp, vp, i64, f64, vp, P(f64), vp], i32),
    "mlp_adam_step": ([vp, vp, vp, vp, vp, f64, f64, f64, f64, i64, vp], i32),
    "mlp_windows": ([vp, i32, i32, vp, vp], i32),
    "mlp_closure": ([vp, vp, i64, f64, vp, vp, vp], i32),
    "gray_set_forchheimer": ([vp, vp], i32),
    "mlp_profile_loss": ([vp, vp, vp, i32, i32, f64, f64, f64, vp, vp, vp], i32),
}

EXPORTS = []
for _name, (_args, _res) in _sig.items():
    _f = getattr(lib, _name)
    _f.argtypes = _args
    _f.restype = _res
    EXPORTS.append(_name)


def register(name, args, res):
    f = getattr(lib, name)
    f.argtypes = args
    f.restype = res
    EXPORTS.append(name)
    return f


class LbmError(RuntimeError):
    def __init__(self, status, where):
        msg = lib.lbm_last_error().decode(errors="replace")
        super().__init__(f"{where} failed with status {status}: {msg}")
        self.status = status


def check(status, where):
    if status != 0:
        raise LbmError(status, where)
    return status
