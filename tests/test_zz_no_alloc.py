"""sm_apply_noalloc: the operators without a workspace, on the library's
static scratch array, against sm_forward / sm_back through the C ABI.

Two calls in a row share the array: a 128^3 scan with two volumes, then a
smaller 64^3 scan with one, so the second call runs over what the first left
in the array.  The forward is bitwise sm_forward's (each detector column's
sums do not depend on how views are chunked); the adjoint may chunk views
and split view runs differently, so it is held to the parity bars (relative
L2 1e-5 in FP32, 1e-12 in FP64) and every comparison logs its error.
"""
import numpy as np
import pytest
import torch

from paper_2511_12235_amd import _lib
from paper_2511_12235_amd import workloads as wl
from paper_2511_12235_amd.projector import SystemMatrix

from _errlog import record

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
TOL = {"fp64": 1e-12, "fp32": 1e-5}


def _say(*msg):
    print("[case]", *msg, flush=True)


def _t(a, prec):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV, torch.float64 if prec == "fp64" else torch.float32)


def _both(A, x, y, prec, name):
    """noalloc against the workspace entry points, forward and adjoint."""
    B = x.shape[0] if x.dim() == 4 else 1
    yn = torch.full(((B,) if x.dim() == 4 else ()) + A.sino_shape, float("nan"), dtype=A.dtype, device=DEV)
    xn = torch.full(((B,) if y.dim() == 4 else ()) + A.vol_shape, float("nan"), dtype=A.dtype, device=DEV)
    A.apply_noalloc(x, False, yn)
    A.apply_noalloc(y, True, xn)
    yr = A.forward(x)
    xr = A.back(y)
    torch.cuda.synchronize()
    assert torch.equal(yn, yr), name + ": forward differs from sm_forward"
    xn64, xr64 = xn.double().cpu().numpy(), xr.double().cpu().numpy()
    assert np.isfinite(xn64).all()
    rel, _ = record("noalloc adjoint vs sm_back, %s" % name, xn64, xr64, TOL[prec])
    assert rel <= TOL[prec], name


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_two_calls_second_smaller(prec):
    big = wl.c2_cone128()
    small = wl.scaled(big, (64, 64, 64), (96, 64), 90)
    _say("noalloc", prec, "128^3 batch 2, then 64^3 batch 1")
    A = SystemMatrix(big, prec, device=DEV)
    X = np.stack([wl.ellipse_phantom(big, 10, seed=3 + i) for i in range(2)])
    Y = np.stack([wl.uniform(big.sino_shape, 20 + i) for i in range(2)])
    _both(A, _t(X, prec), _t(Y, prec), prec, "128^3 B=2 %s" % prec)
    S = SystemMatrix(small, prec, device=DEV)
    x = wl.ellipse_phantom(small, 8, seed=5)
    y = wl.uniform(small.sino_shape, 6)
    _both(S, _t(x, prec), _t(y, prec), prec, "64^3 B=1 %s (after 128^3)" % prec)


def test_kept_records_and_2d():
    g = wl.scaled(wl.c2_cone128(), (64, 64, 48), (96, 64), 60)
    _say("noalloc with kept records; 2D")
    A = SystemMatrix(g, "fp32", device=DEV)
    A.keep_records()
    _both(A, _t(wl.ellipse_phantom(g, 6, seed=9), "fp32"), _t(wl.uniform(g.sino_shape, 10), "fp32"), "fp32",
          "64x64x48 kept records")
    g2 = wl.c1_fan2d()
    A2 = SystemMatrix(g2, "fp64", device=DEV)
    _both(A2, _t(wl.ellipse_phantom(g2, 5, seed=1), "fp64"), _t(wl.uniform(g2.sino_shape, 2), "fp64"), "fp64",
          "2D fan 64^2")


def test_one_256_volume():
    """One 256^3 FP32 volume fits (its voxel columns, 64 MiB, beside about one
    view of strip records): records rebuilt one chunk at a time."""
    g = wl.c3_cone256()
    _say("noalloc 256^3 fp32, one volume")
    A = SystemMatrix(g, "fp32", device=DEV)
    x = wl.ellipse_phantom(g, 10, seed=2)
    y = wl.uniform(g.sino_shape, 8)
    _both(A, _t(x, "fp32"), _t(y, "fp32"), "fp32", "256^3 B=1 fp32")


def test_rejects_what_does_not_fit():
    """Three 256^3 volumes need about 200 MB of column buffers: SM_ERANGE,
    nothing launched, and the message names the sizes."""
    g = wl.c3_cone256()
    _say("noalloc rejection 256^3 batch 3")
    A = SystemMatrix(g, "fp32", device=DEV)
    x = torch.zeros((3,) + A.vol_shape, dtype=A.dtype, device=DEV)
    y = torch.zeros((3,) + A.sino_shape, dtype=A.dtype, device=DEV)
    with pytest.raises(_lib.SmError) as ei:
        A.apply_noalloc(x, False, y)
    assert ei.value.status == _lib.SM_ERANGE
    assert "static scratch" in str(ei.value)
    st = _lib.lib().sm_apply_noalloc(A._plan, 2, x.data_ptr(), y.data_ptr(), 3, None)  # neither direction
    assert st == _lib.SM_EINVAL
