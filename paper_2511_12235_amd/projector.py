"""Torch front end of the HIP system-matrix library.

``SystemMatrix`` owns one plan (include/sm.h) and applies W (forward
projection, Sec. III of arXiv 2511.12235) and W^T (its exact adjoint) to
device tensors through the C ABI.  Tensors are validated here; all
arithmetic runs in the library's kernels on the caller's current HIP stream.
``Projection`` wraps the pair as a ``torch.autograd.Function``: W is linear,
so the backward of y = W x is W^T applied to the incoming gradient.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _lib


def _dtype_of(precision: str):
    if precision == "fp32":
        return torch.float32, _lib.SM_FP32
    if precision == "fp64":
        return torch.float64, _lib.SM_FP64
    raise ValueError("precision must be 'fp32' or 'fp64'")


class SystemMatrix:
    """Matrix-free exact system matrix W for one scan geometry.

    ``geometry`` has the attributes of ``workloads.Geometry``.  Volumes are
    tensors of shape (nz, ny, nx) or (B, nz, ny, nx), sinograms (n_p, det_nz,
    det_ny) or (B, n_p, det_nz, det_ny), on the plan's device, contiguous, in
    the plan's dtype.
    """

    def __init__(self, geometry, precision: str = "fp32", device=None):
        self.geometry = geometry
        self.precision = precision
        self.dtype, prec = _dtype_of(precision)
        dev = torch.device("cuda", torch.cuda.current_device() if device is None else
                           torch.device(device).index or 0)
        self.device = dev
        L = _lib.lib()
        keep = []
        gs = _lib.make_geometry_struct(geometry, keep)
        plan = C.c_void_p()
        with torch.cuda.device(dev):
            _lib.check(L.sm_plan_create(C.byref(gs), prec, C.byref(plan)), "sm_plan_create")
        self._plan = plan
        nv, nr = C.c_int64(), C.c_int64()
        _lib.check(L.sm_plan_sizes(plan, C.byref(nv), C.byref(nr)), "sm_plan_sizes")
        self.n_vox, self.n_rays = nv.value, nr.value
        self.vol_shape = (geometry.nz, geometry.ny, geometry.nx)
        self.sino_shape = (geometry.n_p, geometry.det_nz, geometry.det_ny)

    # ------------------------------------------------------------------ utils
    def close(self):
        if getattr(self, "_plan", None):
            _lib.lib().sm_plan_destroy(self._plan)
            self._plan = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, t: torch.Tensor, shape, name: str) -> int:
        if not isinstance(t, torch.Tensor):
            raise TypeError("%s must be a torch.Tensor" % name)
        if t.device != self.device:
            raise ValueError("%s is on %s, the plan on %s" % (name, t.device, self.device))
        if t.dtype != self.dtype:
            raise TypeError("%s has dtype %s, the plan needs %s" % (name, t.dtype, self.dtype))
        if not t.is_contiguous():
            raise ValueError("%s must be contiguous" % name)
        if tuple(t.shape) == tuple(shape):
            return 1
        if t.dim() == len(shape) + 1 and tuple(t.shape[1:]) == tuple(shape):
            return t.shape[0]
        raise ValueError("%s has shape %s, expected %s or (B, *%s)" % (name, tuple(t.shape), shape, shape))

    def record_bytes(self) -> int:
        """Bytes of the strip records of every view (sm_plan_record_bytes)."""
        n = C.c_int64()
        _lib.check(_lib.lib().sm_plan_record_bytes(self._plan, C.byref(n)), "sm_plan_record_bytes")
        return n.value

    def keep_records(self, max_bytes: int | None = None) -> None:
        """Keep the strip records of every view on the device between calls
        (sm_plan_keep_records); max_bytes = 0 releases them.  Workspaces sized
        before this call stay large enough."""
        n = self.record_bytes() if max_bytes is None else int(max_bytes)
        st = torch.cuda.current_stream(self.device).cuda_stream
        with torch.cuda.device(self.device):
            _lib.check(_lib.lib().sm_plan_keep_records(self._plan, n, st), "sm_plan_keep_records")

    def launch_shape(self) -> tuple[int, int]:
        """(views per record chunk, adjoint view runs per chunk) of the 3D
        operators (sm_plan_launch_shape); (n_p, 1) in 2D."""
        v, r = C.c_int32(), C.c_int32()
        _lib.check(_lib.lib().sm_plan_launch_shape(self._plan, C.byref(v), C.byref(r)),
                   "sm_plan_launch_shape")
        return v.value, r.value

    def workspace_bytes(self, batch: int = 1) -> int:
        n = C.c_int64()
        _lib.check(_lib.lib().sm_workspace_size(self._plan, int(batch), C.byref(n)), "sm_workspace_size")
        return n.value

    def workspace(self, batch: int = 1) -> torch.Tensor:
        return torch.empty(max(self.workspace_bytes(batch), 1), dtype=torch.uint8, device=self.device)

    # -------------------------------------------------------------- operators
    def forward(self, x: torch.Tensor, out: torch.Tensor | None = None,
                ws: torch.Tensor | None = None) -> torch.Tensor:
        """y = W x on the current stream."""
        B = self._check(x, self.vol_shape, "x")
        batched = x.dim() == 4
        shape = ((B,) if batched else ()) + self.sino_shape
        if out is None:
            out = torch.empty(shape, dtype=self.dtype, device=self.device)
        elif self._check(out, self.sino_shape, "out") != B:
            raise ValueError("out batch does not match x")
        if ws is None:
            ws = self.workspace(B)
        st = torch.cuda.current_stream(self.device).cuda_stream
        _lib.check(_lib.lib().sm_forward(self._plan, x.data_ptr(), out.data_ptr(), B, ws.data_ptr(),
                                         ws.numel(), st), "sm_forward")
        return out

    def back(self, y: torch.Tensor, out: torch.Tensor | None = None,
             ws: torch.Tensor | None = None) -> torch.Tensor:
        """x = W^T y on the current stream."""
        B = self._check(y, self.sino_shape, "y")
        batched = y.dim() == 4
        shape = ((B,) if batched else ()) + self.vol_shape
        if out is None:
            out = torch.empty(shape, dtype=self.dtype, device=self.device)
        elif self._check(out, self.vol_shape, "out") != B:
            raise ValueError("out batch does not match y")
        if ws is None:
            ws = self.workspace(B)
        st = torch.cuda.current_stream(self.device).cuda_stream
        _lib.check(_lib.lib().sm_back(self._plan, y.data_ptr(), out.data_ptr(), B, ws.data_ptr(),
                                      ws.numel(), st), "sm_back")
        return out

    __matmul__ = forward

    def apply_noalloc(self, inp: torch.Tensor, adjoint: bool, out: torch.Tensor) -> torch.Tensor:
        """W inp (adjoint=False) or W^T inp (adjoint=True) into `out` through
        sm_apply_noalloc: no workspace and no allocation, the library's static
        scratch array instead (calls on one device must not overlap)."""
        src, dst = (self.sino_shape, self.vol_shape) if adjoint else (self.vol_shape, self.sino_shape)
        B = self._check(inp, src, "input")
        if self._check(out, dst, "out") != B or out.dim() != inp.dim():
            raise ValueError("out batch does not match the input")
        st = torch.cuda.current_stream(self.device).cuda_stream
        _lib.check(_lib.lib().sm_apply_noalloc(self._plan, 1 if adjoint else 0, inp.data_ptr(),
                                               out.data_ptr(), B, st), "sm_apply_noalloc")
        return out

    # ------------------------------------------------- line-based comparison
    @staticmethod
    def _line_weight(weight: str) -> int:
        if weight == "length":
            return _lib.SM_LINE_LENGTH
        if weight == "measure":
            return _lib.SM_LINE_MEASURE
        raise ValueError("weight must be 'length' or 'measure'")

    def line_forward(self, x: torch.Tensor, k: int = 1, weight: str = "length",
                     out: torch.Tensor | None = None) -> torch.Tensor:
        """y = W_line x: the line-based model with k (k x k in 3D) lines per
        detector element (sm_line_forward), on the current stream."""
        B = self._check(x, self.vol_shape, "x")
        shape = ((B,) if x.dim() == 4 else ()) + self.sino_shape
        if out is None:
            out = torch.empty(shape, dtype=self.dtype, device=self.device)
        elif self._check(out, self.sino_shape, "out") != B:
            raise ValueError("out batch does not match x")
        st = torch.cuda.current_stream(self.device).cuda_stream
        _lib.check(_lib.lib().sm_line_forward(self._plan, int(k), self._line_weight(weight), x.data_ptr(),
                                              out.data_ptr(), B, st), "sm_line_forward")
        return out

    def line_back(self, y: torch.Tensor, k: int = 1, weight: str = "length",
                  out: torch.Tensor | None = None) -> torch.Tensor:
        """x = W_line^T y (sm_line_back), the transpose of line_forward."""
        B = self._check(y, self.sino_shape, "y")
        shape = ((B,) if y.dim() == 4 else ()) + self.vol_shape
        if out is None:
            out = torch.empty(shape, dtype=self.dtype, device=self.device)
        elif self._check(out, self.vol_shape, "out") != B:
            raise ValueError("out batch does not match y")
        st = torch.cuda.current_stream(self.device).cuda_stream
        _lib.check(_lib.lib().sm_line_back(self._plan, int(k), self._line_weight(weight), y.data_ptr(),
                                           out.data_ptr(), B, st), "sm_line_back")
        return out

    # ---------------------------------------------------------------- solvers
    def solver_workspace(self, solver: int, batch: int = 1) -> torch.Tensor:
        n = C.c_int64()
        _lib.check(_lib.lib().sm_solver_workspace_size(self._plan, int(solver), int(batch), C.byref(n)),
                   "sm_solver_workspace_size")
        return torch.empty(max(n.value, 1), dtype=torch.uint8, device=self.device)

    def power_norm(self, v0: torch.Tensor, iters: int = 100, out: torch.Tensor | None = None,
                   ws: torch.Tensor | None = None, line=None) -> torch.Tensor:
        """||W||_2 by power iteration from the start volume v0 (sm_power_norm);
        returns a one-element float64 device tensor (no synchronisation).
        line=(k, weight) iterates the line-based model instead
        (sm_line_power_norm)."""
        if self._check(v0, self.vol_shape, "v0") != 1 or v0.dim() != 3:
            raise ValueError("v0 must be one volume")
        if out is None:
            out = torch.empty(1, dtype=torch.float64, device=self.device)
        if ws is None:
            ws = self.solver_workspace(_lib.SM_SOLVER_POWER, 1)
        st = torch.cuda.current_stream(self.device).cuda_stream
        if line is None:
            _lib.check(_lib.lib().sm_power_norm(self._plan, v0.data_ptr(), int(iters), out.data_ptr(),
                                                ws.data_ptr(), ws.numel(), st), "sm_power_norm")
        else:
            k, weight = line
            _lib.check(_lib.lib().sm_line_power_norm(self._plan, int(k), self._line_weight(weight),
                                                     v0.data_ptr(), int(iters), out.data_ptr(),
                                                     ws.data_ptr(), ws.numel(), st), "sm_line_power_norm")
        return out

    def _solve_args(self, y, x0, iters, hist_rows):
        B = self._check(y, self.sino_shape, "y")
        shape = ((B,) if y.dim() == 4 else ()) + self.vol_shape
        if x0 is None:
            x = torch.zeros(shape, dtype=self.dtype, device=self.device)
        else:
            if self._check(x0, self.vol_shape, "x0") != B:
                raise ValueError("x0 batch does not match y")
            x = x0.clone()
        hist = torch.empty((hist_rows(iters), B), dtype=torch.float64, device=self.device)
        return B, x, hist

    def cgls(self, y: torch.Tensor, iters: int, lam: float = 0.0, wscale: float = 1.0,
             x0: torch.Tensor | None = None, ws: torch.Tensor | None = None):
        """CGLS for 1/2 |s W x - y|^2 + lam/2 |x|^2 (sm_cgls).  Returns
        (x, hist) with hist[k] = |grad F(x_k)|^2, k = 0..iters."""
        B, x, hist = self._solve_args(y, x0, iters, lambda n: n + 1)
        if ws is None:
            ws = self.solver_workspace(_lib.SM_SOLVER_CGLS, B)
        st = torch.cuda.current_stream(self.device).cuda_stream
        _lib.check(_lib.lib().sm_cgls(self._plan, y.data_ptr(), x.data_ptr(), B, int(iters), float(lam),
                                      float(wscale), hist.data_ptr(), ws.data_ptr(), ws.numel(), st),
                   "sm_cgls")
        return x, hist

    def nag(self, y: torch.Tensor, iters: int, norm: torch.Tensor, lam: float = 0.0,
            wscale: float = 1.0, x0: torch.Tensor | None = None, ws: torch.Tensor | None = None,
            line=None):
        """Nesterov / FISTA for the same objective with step 1/(s^2 norm^2 + lam)
        (sm_nag); norm is a one-element float64 device tensor such as
        power_norm() returns.  Returns (x, hist), hist[k] = |grad F(z_k)|^2.
        line=(k, weight) solves with the line-based model (sm_line_nag)."""
        B, x, hist = self._solve_args(y, x0, iters, lambda n: max(n, 1))
        if not (isinstance(norm, torch.Tensor) and norm.dtype == torch.float64 and norm.device == self.device):
            raise TypeError("norm must be a float64 tensor on the plan's device")
        if ws is None:
            ws = self.solver_workspace(_lib.SM_SOLVER_NAG, B)
        st = torch.cuda.current_stream(self.device).cuda_stream
        if line is None:
            _lib.check(_lib.lib().sm_nag(self._plan, y.data_ptr(), x.data_ptr(), B, int(iters), float(lam),
                                         float(wscale), norm.data_ptr(), hist.data_ptr(), ws.data_ptr(),
                                         ws.numel(), st), "sm_nag")
        else:
            k, weight = line
            _lib.check(_lib.lib().sm_line_nag(self._plan, int(k), self._line_weight(weight), y.data_ptr(),
                                              x.data_ptr(), B, int(iters), float(lam), float(wscale),
                                              norm.data_ptr(), hist.data_ptr(), ws.data_ptr(), ws.numel(),
                                              st), "sm_line_nag")
        return x, hist[:iters]

    # ----------------------------------------------------------------- timing
    def timing(self, enable: bool = True):
        """Switch per-kernel event timing on or off (sm_timing_enable)."""
        with torch.cuda.device(self.device):
            _lib.check(_lib.lib().sm_timing_enable(self._plan, 1 if enable else 0), "sm_timing_enable")

    def read_timing(self) -> dict:
        """{kernel: (launches, ms)} since the last read (sm_timing_read)."""
        arr = (_lib.SmKernelTime * len(_lib.KERNELS))()
        with torch.cuda.device(self.device):
            _lib.check(_lib.lib().sm_timing_read(self._plan, arr), "sm_timing_read")
        return {name: (int(arr[i].launches), float(arr[i].ms)) for i, name in enumerate(_lib.KERNELS)}

    def weights_csr(self, values: str | None = None):
        """(row_ptr int64 [M+1], col_idx int32 [nnz], values [nnz]) on the host;
        the pattern is decided in FP64 (entries <= 1e-12 voxel measure drop)."""
        vprec = self.precision if values is None else values
        vdt, vcode = (np.float32, _lib.SM_FP32) if vprec == "fp32" else (np.float64, _lib.SM_FP64)
        L = _lib.lib()
        nnz = C.c_int64(0)
        with torch.cuda.device(self.device):
            _lib.check(L.sm_weights_csr(self._plan, vcode, C.byref(nnz), None, None, None),
                       "sm_weights_csr")
            row_ptr = np.empty(self.n_rays + 1, dtype=np.int64)
            cols = np.empty(max(nnz.value, 1), dtype=np.int32)
            vals = np.empty(max(nnz.value, 1), dtype=vdt)
            _lib.check(L.sm_weights_csr(self._plan, vcode, C.byref(nnz),
                                        row_ptr.ctypes.data_as(C.POINTER(C.c_int64)),
                                        cols.ctypes.data_as(C.POINTER(C.c_int32)),
                                        vals.ctypes.data_as(C.c_void_p)), "sm_weights_csr")
        n = nnz.value
        return row_ptr, cols[:n], vals[:n]

    def footprints(self, view: int) -> np.ndarray:
        """int32 [nz, ny, nx, 4] footprint boxes of one view."""
        out = np.empty(self.vol_shape + (4,), dtype=np.int32)
        with torch.cuda.device(self.device):
            _lib.check(_lib.lib().sm_footprints(self._plan, int(view),
                                                out.ctypes.data_as(C.POINTER(C.c_int32))),
                       "sm_footprints")
        return out


class Projection(torch.autograd.Function):
    """y = W x with dL/dx = W^T dL/dy."""

    @staticmethod
    def forward(ctx, x, A: SystemMatrix):
        ctx.A = A
        return A.forward(x.contiguous())

    @staticmethod
    def backward(ctx, gy):
        return ctx.A.back(gy.contiguous()), None


def project(x: torch.Tensor, A: SystemMatrix) -> torch.Tensor:
    return Projection.apply(x, A)


class StoredMatrix:
    """Stored-W mode: W and W^T of a plan as device CSR arrays
    (sm_stored_fill), applied by sparse matrix-vector products
    (sm_stored_apply).  For problems whose matrix fits in device memory; the
    arrays take about (4 + value bytes) per entry and per orientation."""

    def __init__(self, A: SystemMatrix, values: str | None = None):
        self.A = A
        self.values = values or A.precision
        self.dtype, self._vp = _dtype_of(self.values)
        L = _lib.lib()
        n = C.c_int64()
        with torch.cuda.device(A.device):
            _lib.check(L.sm_stored_count(A._plan, 0, C.byref(n)), "sm_stored_count")
        self.nnz = n.value
        self.W = self._fill(0, A.n_rays)
        self.Wt = self._fill(1, A.n_vox)

    def _fill(self, transposed: int, rows: int):
        dev = self.A.device
        ptr = torch.empty(rows + 1, dtype=torch.int64, device=dev)
        col = torch.empty(max(self.nnz, 1), dtype=torch.int32, device=dev)
        val = torch.empty(max(self.nnz, 1), dtype=self.dtype, device=dev)
        st = torch.cuda.current_stream(dev).cuda_stream
        _lib.check(_lib.lib().sm_stored_fill(self.A._plan, transposed, self._vp, self.nnz, ptr.data_ptr(),
                                             col.data_ptr(), val.data_ptr(), st), "sm_stored_fill")
        return ptr, col, val

    def _apply(self, M, x: torch.Tensor, rows: int, cols: int, out_shape) -> torch.Tensor:
        if x.device != self.A.device or x.dtype != self.dtype or not x.is_contiguous():
            raise ValueError("input must be a contiguous %s tensor on %s" % (self.dtype, self.A.device))
        B = x.numel() // cols
        if B * cols != x.numel():
            raise ValueError("input size is not a multiple of %d" % cols)
        y = torch.empty((B,) + out_shape if x.numel() != cols else out_shape, dtype=self.dtype,
                        device=self.A.device)
        ptr, col, val = M
        st = torch.cuda.current_stream(self.A.device).cuda_stream
        _lib.check(_lib.lib().sm_stored_apply(rows, ptr.data_ptr(), col.data_ptr(), val.data_ptr(), self._vp,
                                              x.data_ptr(), y.data_ptr(), B, cols, rows, st),
                   "sm_stored_apply")
        return y

    def forward(self, x: torch.Tensor) -> torch.Tensor:
        """y = W x (volume(s) in, sinogram(s) out)."""
        return self._apply(self.W, x, self.A.n_rays, self.A.n_vox, self.A.sino_shape)

    def back(self, y: torch.Tensor) -> torch.Tensor:
        """x = W^T y."""
        return self._apply(self.Wt, y, self.A.n_vox, self.A.n_rays, self.A.vol_shape)
