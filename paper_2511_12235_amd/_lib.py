"""ctypes binding of ``libsm.so`` (the C ABI in ``include/sm.h``).

Argument marshalling only: every computation happens in the HIP library.
The library is built in-tree by ``paper_2511_12235_amd/build.py``; importing
this module never falls back to anything else when it is missing.
"""
from __future__ import annotations

import ctypes as C
import math
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsm.so")

SM_OK, SM_EINVAL, SM_ENOMEM, SM_EDEVICE, SM_EUNSUPPORTED, SM_ERANGE = range(6)
SM_FP32, SM_FP64 = 0, 1

EXPORTED = ("sm_plan_create", "sm_plan_destroy", "sm_plan_sizes", "sm_plan_launch_shape",
            "sm_workspace_size",
            "sm_plan_record_bytes", "sm_plan_keep_records",
            "sm_forward", "sm_back", "sm_apply_noalloc", "sm_line_forward", "sm_line_back",
            "sm_weights_csr", "sm_stored_count", "sm_stored_fill", "sm_stored_apply",
            "sm_footprints", "sm_solver_workspace_size", "sm_power_norm",
            "sm_cgls", "sm_nag", "sm_line_power_norm", "sm_line_nag", "sm_timing_enable", "sm_timing_read",
            "sm_status_str", "sm_last_error")

SM_SOLVER_CGLS, SM_SOLVER_NAG, SM_SOLVER_POWER = range(3)
SM_LINE_LENGTH, SM_LINE_MEASURE = range(2)
SM_LINE_MAX_K = 64
SM_NOALLOC_SCRATCH_BYTES = 128 << 20  # include/sm.h

# sm_kernel ids (timing)
KERNELS = ("records", "forward", "adjoint", "prefix", "transpose")


class SmKernelTime(C.Structure):
    """Mirror of ``sm_kernel_time`` in include/sm.h."""
    _fields_ = [("launches", C.c_int64), ("ms", C.c_double)]


class SmGeometry(C.Structure):
    """Mirror of ``sm_geometry`` in include/sm.h."""
    _fields_ = [
        ("dim", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
        ("a", C.c_double), ("b", C.c_double), ("c", C.c_double),
        ("x0", C.c_double), ("y0", C.c_double), ("z0", C.c_double),
        ("n_p", C.c_int32), ("reserved0", C.c_int32),
        ("phi", C.POINTER(C.c_double)), ("trig", C.POINTER(C.c_double)),
        ("s", C.c_double), ("d", C.c_double),
        ("det_ny", C.c_int32), ("det_nz", C.c_int32),
        ("dy", C.c_double), ("dz", C.c_double),
        ("det_y0", C.c_double), ("det_z0", C.c_double),
    ]


class SmError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str):
        super().__init__("%s failed (%s): %s" % (where, _STATUS.get(status, status), msg))
        self.status = status


_STATUS = {SM_OK: "ok", SM_EINVAL: "invalid argument", SM_ENOMEM: "out of memory",
           SM_EDEVICE: "device error", SM_EUNSUPPORTED: "unsupported", SM_ERANGE: "buffer too small"}

_lib = None


def lib():
    """Load libsm.so; raises if it has not been built (no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libsm.so is not built; run paper_2511_12235_amd/build.py "
                              "(or __graft_entry__.build())")
        L = C.CDLL(LIB_PATH)
        vp, i64p, i32p = C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_int32)
        L.sm_plan_create.restype = C.c_int
        L.sm_plan_create.argtypes = [C.POINTER(SmGeometry), C.c_int, C.POINTER(vp)]
        L.sm_plan_destroy.restype = C.c_int
        L.sm_plan_destroy.argtypes = [vp]
        L.sm_plan_sizes.restype = C.c_int
        L.sm_plan_sizes.argtypes = [vp, i64p, i64p]
        L.sm_plan_launch_shape.restype = C.c_int
        L.sm_plan_launch_shape.argtypes = [vp, i32p, i32p]
        L.sm_workspace_size.restype = C.c_int
        L.sm_plan_record_bytes.restype = C.c_int
        L.sm_plan_record_bytes.argtypes = [vp, i64p]
        L.sm_plan_keep_records.restype = C.c_int
        L.sm_plan_keep_records.argtypes = [vp, C.c_int64, vp]
        L.sm_workspace_size.argtypes = [vp, C.c_int32, i64p]
        L.sm_forward.restype = C.c_int
        L.sm_forward.argtypes = [vp, vp, vp, C.c_int32, vp, C.c_int64, vp]
        L.sm_back.restype = C.c_int
        L.sm_back.argtypes = [vp, vp, vp, C.c_int32, vp, C.c_int64, vp]
        L.sm_apply_noalloc.restype = C.c_int
        L.sm_apply_noalloc.argtypes = [vp, C.c_int32, vp, vp, C.c_int32, vp]
        L.sm_line_forward.restype = C.c_int
        L.sm_line_forward.argtypes = [vp, C.c_int32, C.c_int, vp, vp, C.c_int32, vp]
        L.sm_line_back.restype = C.c_int
        L.sm_line_back.argtypes = [vp, C.c_int32, C.c_int, vp, vp, C.c_int32, vp]
        L.sm_weights_csr.restype = C.c_int
        L.sm_weights_csr.argtypes = [vp, C.c_int, i64p, i64p, i32p, vp]
        L.sm_stored_count.restype = C.c_int
        L.sm_stored_count.argtypes = [vp, C.c_int32, i64p]
        L.sm_stored_fill.restype = C.c_int
        L.sm_stored_fill.argtypes = [vp, C.c_int32, C.c_int, C.c_int64, vp, vp, vp, vp]
        L.sm_stored_apply.restype = C.c_int
        L.sm_stored_apply.argtypes = [C.c_int64, vp, vp, vp, C.c_int, vp, vp, C.c_int32, C.c_int64,
                                      C.c_int64, vp]
        L.sm_footprints.restype = C.c_int
        L.sm_footprints.argtypes = [vp, C.c_int32, i32p]
        dp = C.POINTER(C.c_double)
        L.sm_solver_workspace_size.restype = C.c_int
        L.sm_solver_workspace_size.argtypes = [vp, C.c_int, C.c_int32, i64p]
        L.sm_power_norm.restype = C.c_int
        L.sm_power_norm.argtypes = [vp, vp, C.c_int32, vp, vp, C.c_int64, vp]
        L.sm_cgls.restype = C.c_int
        L.sm_cgls.argtypes = [vp, vp, vp, C.c_int32, C.c_int32, C.c_double, C.c_double, vp, vp,
                              C.c_int64, vp]
        L.sm_nag.restype = C.c_int
        L.sm_nag.argtypes = [vp, vp, vp, C.c_int32, C.c_int32, C.c_double, C.c_double, vp, vp, vp,
                             C.c_int64, vp]
        L.sm_line_power_norm.restype = C.c_int
        L.sm_line_power_norm.argtypes = [vp, C.c_int32, C.c_int, vp, C.c_int32, vp, vp, C.c_int64, vp]
        L.sm_line_nag.restype = C.c_int
        L.sm_line_nag.argtypes = [vp, C.c_int32, C.c_int, vp, vp, C.c_int32, C.c_int32, C.c_double,
                                  C.c_double, vp, vp, vp, C.c_int64, vp]
        L.sm_timing_enable.restype = C.c_int
        L.sm_timing_enable.argtypes = [vp, C.c_int32]
        L.sm_timing_read.restype = C.c_int
        L.sm_timing_read.argtypes = [vp, C.POINTER(SmKernelTime)]
        L.sm_status_str.restype = C.c_char_p
        L.sm_status_str.argtypes = [C.c_int]
        L.sm_last_error.restype = C.c_char_p
        L.sm_last_error.argtypes = []
        _lib = L
    return _lib


def check(status: int, where: str):
    if status != SM_OK:
        raise SmError(status, where, lib().sm_last_error().decode(errors="replace"))


def make_geometry_struct(g, keep: list) -> SmGeometry:
    """Fill an ``SmGeometry`` from a geometry object (the attributes of
    ``workloads.Geometry``).  Arrays referenced by the struct are appended
    to ``keep`` so they outlive the call."""
    import numpy as np
    phi = np.ascontiguousarray(np.asarray(g.phi, dtype=np.float64))
    keep.append(phi)
    trig_p = C.POINTER(C.c_double)()
    if getattr(g, "trig", None) is not None:
        trig = np.ascontiguousarray(np.asarray(g.trig, dtype=np.float64).reshape(-1))
        keep.append(trig)
        trig_p = trig.ctypes.data_as(C.POINTER(C.c_double))
    nan = math.nan
    return SmGeometry(
        dim=g.dim, nx=g.nx, ny=g.ny, nz=g.nz, a=g.a, b=g.b, c=g.c,
        x0=nan if g.x0 is None else g.x0, y0=nan if g.y0 is None else g.y0,
        z0=nan if g.z0 is None else g.z0, n_p=len(phi), reserved0=0,
        phi=phi.ctypes.data_as(C.POINTER(C.c_double)), trig=trig_p,
        s=g.s, d=g.d, det_ny=g.det_ny, det_nz=g.det_nz, dy=g.dy, dz=g.dz,
        det_y0=nan if g.det_y0 is None else g.det_y0,
        det_z0=nan if g.det_z0 is None else g.det_z0)
