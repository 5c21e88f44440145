"""Python front end of the FP64 CPU oracle (test infrastructure only).

Only the test suite, the smoke check and the CPU-baseline leg of the
benchmark import this module.  It loads ``oracle/_build/libsm_oracle.so``
(compiled from ``sm_oracle.c`` by ``oracle/build.py``) and never touches the
HIP library.

Every function takes a geometry object with the attributes of
``paper_2511_12235_amd.workloads.Geometry`` (duck-typed; this module does not
import the product package).  W_ij is the exact measure of voxel j inside the
beam of detector element i (Sec. I, eq. "ip" and the consistency definition),
computed by clipping in ``sm_oracle.c``.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build

_LIB = None


class _Geom(C.Structure):
    _fields_ = [
        ("dim", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
        ("a", C.c_double), ("b", C.c_double), ("c", C.c_double),
        ("x0", C.c_double), ("y0", C.c_double), ("z0", C.c_double),
        ("n_p", C.c_int32), ("pad0", C.c_int32),
        ("phi", C.POINTER(C.c_double)), ("trig", C.POINTER(C.c_double)),
        ("s", C.c_double), ("d", C.c_double),
        ("det_ny", C.c_int32), ("det_nz", C.c_int32),
        ("dy", C.c_double), ("dz", C.c_double),
        ("det_y0", C.c_double), ("det_z0", C.c_double),
    ]


def lib():
    """Load (building first if needed) the oracle shared library."""
    global _LIB
    if _LIB is None:
        path = _build.LIB
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_build.SRC):
            _build.build()
        L = C.CDLL(path)
        dp, ip32, ip64 = C.POINTER(C.c_double), C.POINTER(C.c_int32), C.POINTER(C.c_int64)
        G = C.POINTER(_Geom)
        L.orc_clip_rect.restype = C.c_double
        L.orc_clip_rect.argtypes = [C.c_double, C.c_double, dp, C.c_int]
        L.orc_clip_box.restype = C.c_double
        L.orc_clip_box.argtypes = [C.c_double, C.c_double, C.c_double, dp, C.c_int]
        L.orc_validate.restype = C.c_int
        L.orc_validate.argtypes = [G]
        L.orc_footprints.restype = C.c_int
        L.orc_footprints.argtypes = [G, C.c_int, ip32]
        L.orc_cell_measure.restype = C.c_double
        L.orc_cell_measure.argtypes = [G] + [C.c_int] * 6
        L.orc_ray_gridbox.restype = C.c_double
        L.orc_ray_gridbox.argtypes = [G, C.c_int, C.c_int, C.c_int]
        L.orc_ray_gridbox_view.restype = None
        L.orc_ray_gridbox_view.argtypes = [G, C.c_int, dp]
        L.orc_count.restype = C.c_int64
        L.orc_count.argtypes = [G, C.c_int, C.c_int, C.c_double, ip64]
        L.orc_fill.restype = C.c_int
        L.orc_fill.argtypes = [G, C.c_int, C.c_int, C.c_double, ip64, ip64, ip32, dp]
        L.orc_forward.restype = C.c_int
        L.orc_forward.argtypes = [G, dp, ip32, C.c_int, C.c_double, dp]
        L.orc_back.restype = C.c_int
        L.orc_back.argtypes = [G, dp, ip64, C.c_int64, C.c_double, dp]
        L.orc_forward_rays.restype = C.c_int
        L.orc_forward_rays.argtypes = [G, dp, ip64, C.c_int64, C.c_double, dp]
        L.orc_num_threads.restype = C.c_int
        _LIB = L
    return _LIB


def _ptr(a, ctype=C.c_double):
    return a.ctypes.data_as(C.POINTER(ctype))


class _Bound:
    """Keeps the numpy buffers referenced by a ``_Geom`` alive."""

    def __init__(self, g):
        self.phi = np.ascontiguousarray(np.asarray(g.phi, dtype=np.float64))
        self.trig = None
        if getattr(g, "trig", None) is not None:
            self.trig = np.ascontiguousarray(np.asarray(g.trig, dtype=np.float64).reshape(-1))
        self.s = _Geom(
            dim=g.dim, nx=g.nx, ny=g.ny, nz=g.nz, a=g.a, b=g.b, c=g.c,
            x0=g.x0, y0=g.y0, z0=g.z0, n_p=len(self.phi), pad0=0,
            phi=_ptr(self.phi),
            trig=_ptr(self.trig) if self.trig is not None else C.POINTER(C.c_double)(),
            s=g.s, d=g.d, det_ny=g.det_ny, det_nz=g.det_nz, dy=g.dy, dz=g.dz,
            det_y0=g.det_y0, det_z0=g.det_z0)

    @property
    def ref(self):
        return C.byref(self.s)


def default_tau(g) -> float:
    """Entries at or below 1e-12 of the voxel measure count as exact zeros
    (rounding residue of clips that only touch a face or an edge)."""
    return 1e-12 * g.a * g.b * (g.c if g.dim == 3 else 1.0)


def num_threads() -> int:
    return int(lib().orc_num_threads())


def validate(g) -> bool:
    return lib().orc_validate(_Bound(g).ref) == 0


def clip_rect(hx, hy, planes) -> float:
    """Area of [-hx,hx]x[-hy,hy] where every row (alpha, bx, by) of
    ``planes`` satisfies alpha + bx*x + by*y >= 0."""
    p = np.ascontiguousarray(np.asarray(planes, dtype=np.float64).reshape(-1, 3))
    return float(lib().orc_clip_rect(hx, hy, _ptr(p), len(p)))


def clip_box(hx, hy, hz, planes) -> float:
    """Volume of the centred box where alpha + b.q >= 0 for every row
    (alpha, bx, by, bz) of ``planes``."""
    p = np.ascontiguousarray(np.asarray(planes, dtype=np.float64).reshape(-1, 4))
    return float(lib().orc_clip_box(hx, hy, hz, _ptr(p), len(p)))


def footprints(g, view: int) -> np.ndarray:
    """int32 array [nz, ny, nx, 4]: first/last detector column, first/last
    row of every voxel's footprint in one view (first > last when empty)."""
    out = np.empty((g.nz, g.ny, g.nx, 4), dtype=np.int32)
    b = _Bound(g)
    if lib().orc_footprints(b.ref, int(view), _ptr(out, C.c_int32)) != 0:
        raise ValueError("invalid geometry: source inside or behind the grid")
    return out


def cell_measure(g, view, ix, iy, iz, k, r) -> float:
    """Exact measure of voxel (ix, iy, iz) inside element (k, r), one view."""
    return float(lib().orc_cell_measure(_Bound(g).ref, int(view), int(ix), int(iy),
                                         int(iz), int(k), int(r)))


def ray_gridbox(g, view, k, r) -> float:
    """Exact measure of the whole grid box inside element (k, r)."""
    return float(lib().orc_ray_gridbox(_Bound(g).ref, int(view), int(k), int(r)))


def ray_gridbox_view(g, view) -> np.ndarray:
    """ray_gridbox of every element of one view -> array [det_nz, det_ny]."""
    out = np.empty((g.det_nz, g.det_ny), dtype=np.float64)
    lib().orc_ray_gridbox_view(_Bound(g).ref, int(view), _ptr(out))
    return out


def triplets(g, views=None, tau=None):
    """Kept entries (W > tau) as (rows int64, cols int32, vals float64),
    sorted by (row, col)."""
    L = lib()
    b = _Bound(g)
    tau = default_tau(g) if tau is None else float(tau)
    if views is None:
        views = (0, g.n_p)
    v0, v1 = int(views[0]), int(views[1])
    counts = np.zeros(v1 - v0, dtype=np.int64)
    tot = L.orc_count(b.ref, v0, v1, tau, _ptr(counts, C.c_int64))
    if tot < 0:
        raise ValueError("invalid geometry: source inside or behind the grid")
    rows = np.empty(tot, dtype=np.int64)
    cols = np.empty(tot, dtype=np.int32)
    vals = np.empty(tot, dtype=np.float64)
    if L.orc_fill(b.ref, v0, v1, tau, _ptr(counts, C.c_int64), _ptr(rows, C.c_int64),
                  _ptr(cols, C.c_int32), _ptr(vals)) != 0:
        raise MemoryError("orc_fill")
    order = np.lexsort((cols, rows))
    return rows[order], cols[order], vals[order]


def count(g, views=None, tau=None) -> int:
    """Number of kept entries (W > tau) of the views [v0, v1) (all by default)."""
    L = lib()
    b = _Bound(g)
    tau = default_tau(g) if tau is None else float(tau)
    v0, v1 = (0, g.n_p) if views is None else (int(views[0]), int(views[1]))
    counts = np.zeros(max(v1 - v0, 1), dtype=np.int64)
    tot = L.orc_count(b.ref, v0, v1, tau, _ptr(counts, C.c_int64))
    if tot < 0:
        raise ValueError("invalid geometry: source inside or behind the grid")
    return int(tot)


def matrix(g, tau=None):
    """The full system matrix as a scipy CSR matrix (small problems)."""
    import scipy.sparse as sp
    rows, cols, vals = triplets(g, tau=tau)
    return sp.csr_matrix((vals, (rows, cols)), shape=(g.n_rays, g.n_vox))


def forward(g, x, views=None, tau=None) -> np.ndarray:
    """y = W x in FP64 for the listed views -> array [len(views), det_nz, det_ny]."""
    L = lib()
    b = _Bound(g)
    tau = default_tau(g) if tau is None else float(tau)
    x = np.ascontiguousarray(np.asarray(x, dtype=np.float64).reshape(-1))
    if x.size != g.n_vox:
        raise ValueError("x has the wrong size")
    views = np.arange(g.n_p) if views is None else np.asarray(views)
    views = np.ascontiguousarray(views.astype(np.int32))
    y = np.empty((len(views), g.det_nz, g.det_ny), dtype=np.float64)
    if L.orc_forward(b.ref, _ptr(x), _ptr(views, C.c_int32), len(views), tau, _ptr(y)) != 0:
        raise ValueError("invalid geometry: source inside or behind the grid")
    return y


def back(g, y, voxels=None, tau=None) -> np.ndarray:
    """x_j = sum_i W_ij y_i in FP64 for the listed linear voxel indices
    (all voxels when ``voxels`` is None, returned as [nz, ny, nx])."""
    L = lib()
    b = _Bound(g)
    tau = default_tau(g) if tau is None else float(tau)
    y = np.ascontiguousarray(np.asarray(y, dtype=np.float64).reshape(-1))
    if y.size != g.n_rays:
        raise ValueError("y has the wrong size")
    full = voxels is None
    vox = np.arange(g.n_vox, dtype=np.int64) if full else np.asarray(voxels, dtype=np.int64)
    vox = np.ascontiguousarray(vox)
    x = np.empty(len(vox), dtype=np.float64)
    if L.orc_back(b.ref, _ptr(y), _ptr(vox, C.c_int64), len(vox), tau, _ptr(x)) != 0:
        raise ValueError("invalid geometry: source inside or behind the grid")
    return x.reshape(g.vol_shape) if full else x


def forward_rays(g, x, rays, tau=None) -> np.ndarray:
    """y_i for the listed linear ray indices (brute force over all voxels)."""
    L = lib()
    b = _Bound(g)
    tau = default_tau(g) if tau is None else float(tau)
    x = np.ascontiguousarray(np.asarray(x, dtype=np.float64).reshape(-1))
    if x.size != g.n_vox:
        raise ValueError("x has the wrong size")
    rays = np.ascontiguousarray(np.asarray(rays, dtype=np.int64))
    y = np.empty(len(rays), dtype=np.float64)
    if L.orc_forward_rays(b.ref, _ptr(x), _ptr(rays, C.c_int64), len(rays), tau, _ptr(y)) != 0:
        raise ValueError("invalid geometry: source inside or behind the grid")
    return y
