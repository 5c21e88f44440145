"""Edge cases of the 3D operators through the C ABI: rejected geometries and
arguments (with the status the header promises), a grid the beam misses, one
voxel and one detector element, the largest row and column counts a plan
accepts (1024 detector rows, 1024 voxels per column), a column taller than one
workgroup of the adjoint's first shape (nz = 300), a one-voxel slab, and the
batch limit.  Parity bars as in test_gpu_parity.py (FP64 1e-12, FP32 1e-5
relative L2 against the oracle's matrix)."""
import ctypes as C

import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2511_12235_amd import _lib
from paper_2511_12235_amd import workloads as wl
from paper_2511_12235_amd.projector import SystemMatrix

from _errlog import record

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
TOL = {"fp64": 1e-12, "fp32": 1e-5}


def _rel(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _t(a, prec):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV, torch.float64 if prec == "fp64" else torch.float32)


def _say(*msg):
    print("[case]", *msg, flush=True)


def _status(geometry, prec="fp32"):
    keep = []
    gs = _lib.make_geometry_struct(geometry, keep)
    plan = C.c_void_p()
    st = _lib.lib().sm_plan_create(C.byref(gs), _lib.SM_FP32 if prec == "fp32" else _lib.SM_FP64, C.byref(plan))
    if st == _lib.SM_OK:
        _lib.lib().sm_plan_destroy(plan)
    return st


def _small(**kw):
    base = dict(dim=3, n=(6, 5, 4), pitch=(1.0, 1.0, 1.0), n_p=3, s=30.0, d=20.0, det=(8, 6),
                det_pitch=(1.2, 1.2))
    base.update(kw)
    return wl.make_geometry(base["dim"], base["n"], base["pitch"], base["n_p"], base["s"], base["d"],
                            base["det"], base["det_pitch"], corner=base.get("corner"),
                            det_corner=base.get("det_corner"), phi=base.get("phi"))


def test_plan_rejects_bad_geometry():
    _say("bad geometries")
    assert _status(_small()) == _lib.SM_OK
    assert _status(_small(det=(8, 1025), det_pitch=(1.2, 0.01))) == _lib.SM_EUNSUPPORTED
    assert _status(_small(n=(2, 2, 1025), pitch=(1.0, 1.0, 0.01))) == _lib.SM_EUNSUPPORTED
    assert _status(_small(pitch=(1.0, 0.0, 1.0))) == _lib.SM_EINVAL
    assert _status(_small(det_pitch=(-1.0, 1.0))) == _lib.SM_EINVAL
    assert _status(_small(s=2.0)) == _lib.SM_EINVAL  # source inside the grid
    assert _status(_small(phi=[0.0, float("nan"), 1.0])) == _lib.SM_EINVAL
    assert _status(_small(corner=(float("inf"), 0.0, 0.0))) == _lib.SM_EINVAL


def test_apply_rejects_bad_arguments():
    _say("bad arguments")
    A = SystemMatrix(_small(), "fp32", device=DEV)
    L = _lib.lib()
    x = torch.zeros(A.vol_shape, device=DEV)
    y = torch.zeros(A.sino_shape, device=DEV)
    ws = A.workspace(1)
    n = ws.numel()
    assert L.sm_forward(A._plan, None, y.data_ptr(), 1, ws.data_ptr(), n, None) == _lib.SM_EINVAL
    assert L.sm_forward(A._plan, x.data_ptr(), y.data_ptr(), 0, ws.data_ptr(), n, None) == _lib.SM_EINVAL
    assert L.sm_forward(A._plan, x.data_ptr(), y.data_ptr(), 1, ws.data_ptr(), n - 1, None) == _lib.SM_EINVAL
    assert L.sm_back(A._plan, y.data_ptr(), x.data_ptr(), 1, None, 0, None) == _lib.SM_EINVAL
    assert L.sm_forward(None, x.data_ptr(), y.data_ptr(), 1, ws.data_ptr(), n, None) == _lib.SM_EINVAL
    # the error leaves the outputs untouched and the plan usable
    torch.cuda.synchronize()
    assert not y.any()
    A.forward(torch.ones(A.vol_shape, device=DEV), out=y, ws=ws)
    assert y.abs().sum() > 0


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_grid_outside_the_beam(prec):
    """A grid in front of the source but far to the side of the fan (u about
    60 against a detector half-width of 4.8): every weight is zero."""
    _say("outside", prec)
    g = _small(corner=(-3.0, 40.0, -2.0), n_p=1, phi=[0.0])
    W = O.matrix(g)
    assert W.nnz == 0
    A = SystemMatrix(g, prec, device=DEV)
    assert not A.forward(_t(wl.uniform(g.vol_shape, 1) + 1.0, prec)).any()
    assert not A.back(_t(wl.uniform(g.sino_shape, 2) + 1.0, prec)).any()


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_one_voxel_one_element(prec):
    _say("1x1x1", prec)
    g = _small(n=(1, 1, 1), pitch=(2.0, 2.0, 2.0), n_p=1, det=(1, 1), det_pitch=(1.5, 1.5), phi=[0.3])
    W = O.matrix(g)
    A = SystemMatrix(g, prec, device=DEV)
    yg = A.forward(_t(np.full(g.vol_shape, 2.0), prec)).double().cpu().numpy()
    assert W.nnz == 1
    assert record("forward, one voxel one element, %s" % prec, yg, W @ np.full(g.n_vox, 2.0), TOL[prec])[0] <= TOL[prec]
    xg = A.back(_t(np.full(g.sino_shape, 3.0), prec)).double().cpu().numpy()
    assert record("adjoint, one voxel one element, %s" % prec, xg, W.T @ np.full(g.n_rays, 3.0), TOL[prec])[0] <= TOL[prec]


CASES = {
    # 1024 detector rows (the largest an FP32 plan takes): the forward's widest
    # workgroup; FP64 plans stage 1.5x the bytes per row and stop near 830 rows
    "rows1024": dict(n=(5, 4, 30), pitch=(1.0, 1.0, 1.0), n_p=2, s=40.0, d=20.0, det=(7, 1024),
                     det_pitch=(1.3, 0.06)),
    "rows768": dict(n=(5, 4, 30), pitch=(1.0, 1.0, 1.0), n_p=2, s=40.0, d=20.0, det=(7, 768),
                    det_pitch=(1.3, 0.08)),
    # 1024 voxels per column (the largest a plan takes): the adjoint's widest workgroup
    "nz1024": dict(n=(3, 3, 1024), pitch=(1.0, 1.0, 0.03), n_p=2, s=40.0, d=20.0, det=(6, 40),
                   det_pitch=(1.2, 1.0)),
    # a column of 300 voxels: five waves, the last one partly idle
    "nz300": dict(n=(4, 3, 300), pitch=(1.0, 1.0, 0.1), n_p=3, s=40.0, d=20.0, det=(7, 50),
                  det_pitch=(1.2, 1.0)),
    # a slab one voxel thick
    "nz1": dict(n=(9, 8, 1), pitch=(1.0, 1.0, 1.5), n_p=4, s=30.0, d=20.0, det=(14, 5),
                det_pitch=(1.1, 0.9)),
}


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_extreme_shapes_match_oracle(name, prec):
    _say("extreme", name, prec)
    g = _small(**CASES[name])
    if name == "rows1024" and prec == "fp64":
        assert _status(g, prec) == _lib.SM_EUNSUPPORTED
        return
    W = O.matrix(g)
    A = SystemMatrix(g, prec, device=DEV)
    x = wl.uniform(g.vol_shape, 3) + 0.5
    y = wl.uniform(g.sino_shape, 4)
    assert record("forward, edge shape %s, %s" % (name, prec), A.forward(_t(x, prec)).cpu().numpy(), W @ x.ravel(),
                  TOL[prec])[0] <= TOL[prec]
    assert record("adjoint, edge shape %s, %s" % (name, prec), A.back(_t(y, prec)).cpu().numpy(), W.T @ y.ravel(),
                  TOL[prec])[0] <= TOL[prec]


def test_batch_limit():
    """ny * batch above 65535 is refused (SM_EUNSUPPORTED), not launched."""
    _say("batch limit")
    g = _small(n=(4, 64, 1), pitch=(1.0, 1.0, 1.0), det=(8, 2), n_p=1)
    A = SystemMatrix(g, "fp32", device=DEV)
    B = 65535 // 64 + 1
    x = torch.zeros((B,) + A.vol_shape, device=DEV)
    y = torch.zeros((B,) + A.sino_shape, device=DEV)
    ws = A.workspace(B)
    st = _lib.lib().sm_forward(A._plan, x.data_ptr(), y.data_ptr(), B, ws.data_ptr(), ws.numel(), None)
    assert st == _lib.SM_EUNSUPPORTED
    A.forward(x[: B - 1], out=y[: B - 1], ws=ws)  # the largest accepted batch runs
    torch.cuda.synchronize()
