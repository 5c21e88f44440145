"""Parity of the HIP line-based projector (sm_line_forward / sm_line_back,
through the C ABI) with the FP64 line oracle (oracle/lines.py).

Bars: FP64 plans within 1e-12 relative L2 of the oracle, FP32 plans within
1e-5 (sums run in FP64 either way); dot-product test at 1e-13 (FP64); batched
calls bitwise equal to single ones.  Small geometries are compared in full,
the 256^3 scan on sampled detector elements and voxels that the oracle
computes one by one.
"""
import numpy as np
import pytest
import torch

from oracle import lines as LN
from oracle import solvers as SV
from paper_2511_12235_amd import workloads as wl
from paper_2511_12235_amd.projector import SystemMatrix

from _errlog import record

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
TOL = {"fp64": 1e-12, "fp32": 1e-5}
AXIS_TRIG = np.array([[1.0, 0.0], [0.0, 1.0], [-1.0, 0.0], [0.0, -1.0], [np.cos(0.7), np.sin(0.7)]])


def _rel(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _t(a, prec):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV, torch.float64 if prec == "fp64" else torch.float32)


def _say(*msg):
    print("[case]", *msg, flush=True)


def geometries():
    g = {}
    g["fan"] = wl.make_geometry(2, (13, 11), (1.0, 1.2), 7, 30.0, 20.0, (15,), (1.3,))
    g["fan_offset"] = wl.make_geometry(2, (9, 12), (0.8, 1.1), 5, 26.0, 14.0, (17,), (1.1,),
                                       corner=(-3.0, -7.0, -0.5), det_corner=(-11.0, -0.5))
    g["cone"] = wl.make_geometry(3, (10, 9, 8), (1.0, 1.1, 0.9), 6, 30.0, 20.0, (14, 12), (1.1, 1.0))
    # exact axis views, odd detector counts: lines along x and y, lines in the
    # z = 0 plane (a voxel face for even nz), and lines in the y = 0 face
    g["cone_axis"] = wl.make_geometry(3, (8, 8, 8), (1.0, 1.0, 1.0), len(AXIS_TRIG), 20.0, 15.0, (9, 7),
                                      (1.2, 1.3), trig=AXIS_TRIG,
                                      phi=np.arctan2(AXIS_TRIG[:, 1], AXIS_TRIG[:, 0]))
    g["cone_aniso_offset"] = wl.make_geometry(3, (7, 9, 12), (0.7, 1.3, 0.45), 4, 35.0, 25.0, (13, 21),
                                              (0.9, 0.5), det_corner=(-5.0, -6.0),
                                              corner=(-3.0, -6.0, -2.0))
    return g


GEOMS = geometries()
_MATS = {}


def _W(name, k, weight):
    key = (name, k, weight)
    if key not in _MATS:
        _MATS[key] = LN.matrix(GEOMS[name], k, weight)
    return _MATS[key]


@pytest.mark.parametrize("name", list(GEOMS))
@pytest.mark.parametrize("k", [1, 3])
@pytest.mark.parametrize("weight", ["length", "measure"])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_line_matches_oracle(name, k, weight, prec):
    g = GEOMS[name]
    _say("line", name, k, weight, prec)
    W = _W(name, k, weight)
    A = SystemMatrix(g, prec, device=DEV)
    x = wl.ellipse_phantom(g, 4, seed=3) + 0.1 * wl.uniform(g.vol_shape, 4)
    y = wl.uniform(g.sino_shape, 5)
    yg = A.line_forward(_t(x, prec), k, weight).cpu().numpy()
    xg = A.line_back(_t(y, prec), k, weight).cpu().numpy()
    assert record("line forward k=%d %s, %s %s" % (k, weight, name, prec), yg, W @ x.ravel(), TOL[prec])[0] <= TOL[prec]
    assert record("line adjoint k=%d %s, %s %s" % (k, weight, name, prec), xg, W.T @ y.ravel(),
                  TOL[prec])[0] <= TOL[prec]


@pytest.mark.parametrize("name", ["fan", "cone", "cone_axis"])
@pytest.mark.parametrize("weight", ["length", "measure"])
def test_line_dot_product(name, weight):
    g = GEOMS[name]
    _say("line dot", name, weight)
    A = SystemMatrix(g, "fp64", device=DEV)
    x = wl.random_unit(g.vol_shape, 11)
    y = wl.random_unit(g.sino_shape, 12)
    Wx = A.line_forward(_t(x, "fp64"), 2, weight).cpu().numpy()
    Wty = A.line_back(_t(y, "fp64"), 2, weight).cpu().numpy()
    lhs, rhs = float(np.vdot(Wx, y)), float(np.vdot(x, Wty))
    assert abs(lhs - rhs) <= 1e-13 * np.linalg.norm(Wx) * np.linalg.norm(y)


@pytest.mark.parametrize("name", ["fan", "cone"])
def test_line_batched_equals_single(name):
    g = GEOMS[name]
    _say("line batch", name)
    A = SystemMatrix(g, "fp32", device=DEV)
    X = np.stack([wl.ellipse_phantom(g, 3, seed=30 + i) for i in range(5)])
    Y = np.stack([wl.uniform(g.sino_shape, 40 + i) for i in range(5)])
    yb = A.line_forward(_t(X, "fp32"), 2, "length").cpu().numpy()
    xb = A.line_back(_t(Y, "fp32"), 2, "measure").cpu().numpy()
    for i in range(5):
        assert np.array_equal(yb[i], A.line_forward(_t(X[i], "fp32"), 2, "length").cpu().numpy())
        assert np.array_equal(xb[i], A.line_back(_t(Y[i], "fp32"), 2, "measure").cpu().numpy())


@pytest.mark.parametrize("name", ["fan", "cone"])
def test_line_measure_tends_to_consistent_matrix(name):
    """The measure weighting is the midpoint rule of the exact element measure:
    at k = 32 (2D) / 16 (3D) W_line x is close to the consistent W x of
    sm_forward, and closer than at k = 2."""
    g = GEOMS[name]
    _say("line limit", name)
    A = SystemMatrix(g, "fp64", device=DEV)
    x = _t(wl.ellipse_phantom(g, 4, seed=8) + 0.2, "fp64")
    ref = A.forward(x).cpu().numpy()
    k_hi = 32 if g.dim == 2 else 16
    e_lo = _rel(A.line_forward(x, 2, "measure").cpu().numpy(), ref)
    e_hi = _rel(A.line_forward(x, k_hi, "measure").cpu().numpy(), ref)
    assert e_hi < e_lo / 16 and e_hi < 1e-3


def test_line_rejects_bad_arguments():
    A = SystemMatrix(GEOMS["fan"], "fp32", device=DEV)
    x = torch.zeros(A.vol_shape, device=DEV)
    for k in (0, 65):
        with pytest.raises(RuntimeError):
            A.line_forward(x, k, "length")
    with pytest.raises(ValueError):
        A.line_forward(x, 1, "area")


def test_line_full_size_sampled():
    """256^3 scan, k = 1, in FP32: sampled detector elements and voxels
    against the oracle, and the dot-product test of the whole pair."""
    g = wl.c3_cone256()
    _say("line full size")
    rng = np.random.default_rng(13)
    A = SystemMatrix(g, "fp32", device=DEV)
    x = wl.ellipse_phantom(g, 10, seed=2) + 0.05 * wl.uniform(g.vol_shape, 15)
    y = A.line_forward(_t(x, "fp32"), 1, "length").cpu().numpy()
    els = [(int(rng.integers(g.n_p)), int(rng.integers(g.det_nz)), int(rng.integers(g.det_ny)))
           for _ in range(5)]
    els.append((0, g.det_nz // 2, g.det_ny // 2))
    yo = LN.forward_rows(g, 1, "length", x, els)
    assert record("line forward rays, c3 fp32", [y[v, r, m] for v, r, m in els], yo, 1e-5)[0] <= 1e-5
    ys = wl.uniform(g.sino_shape, 14)
    xb = A.line_back(_t(ys, "fp32"), 1, "measure").cpu().numpy().ravel()
    # voxels of the central half of the grid (the corners lie outside the cone)
    q = rng.integers(g.nx // 4, 3 * g.nx // 4, size=(4, 3))
    vox = (q[:, 0] * g.ny + q[:, 1]) * g.nx + q[:, 2]
    xo = LN.back_voxels(g, 1, "measure", ys, vox)
    assert record("line adjoint voxels, c3 fp32", xb[vox], xo, 1e-5)[0] <= 1e-5
    yw = A.line_forward(_t(x, "fp32"), 1, "measure").double().cpu().numpy()
    lhs, rhs = float(np.vdot(yw, ys)), float(np.vdot(x, xb))
    assert abs(lhs - rhs) <= 1e-6 * abs(lhs)


@pytest.mark.parametrize("weight", ["length", "measure"])
def test_line_solvers_match_oracle(weight):
    """sm_line_power_norm and sm_line_nag against the oracle's power iteration
    and NAG run on the oracle's line matrix."""
    g = GEOMS["fan"]
    k = 3
    _say("line solvers", weight)
    W = _W("fan", k, weight)
    A = SystemMatrix(g, "fp64", device=DEV)
    v0 = wl.uniform(g.vol_shape, 21)
    norm = A.power_norm(_t(v0, "fp64"), 50, line=(k, weight))
    ref = SV.power_norm(W, v0.ravel(), 50)
    assert abs(norm.item() - ref) <= 1e-12 * ref
    u = wl.ellipse_phantom(g, 3, seed=22).ravel()
    p = (W @ u) / ref + 1e-4 * np.random.default_rng(23).normal(size=g.n_rays)
    x, hist = A.nag(_t(p.reshape(g.sino_shape), "fp64"), 60, norm, lam=1e-4, wscale=1.0 / ref,
                    line=(k, weight))
    x_ref, h_ref = SV.nag(W, p, np.zeros(g.n_vox), 60, ref, lam=1e-4, s=1.0 / ref)
    assert _rel(x.cpu().numpy(), x_ref) <= 1e-10
    assert _rel(hist.cpu().numpy()[:, 0], h_ref) <= 1e-8
