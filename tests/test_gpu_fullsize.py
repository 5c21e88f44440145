"""Full-size parity in the launch configuration the benchmark times.

The 128^3 (180 views) and 256^3 (360 views) cone-beam workloads, FP32 and
FP64 plans, through the C ABI.  The oracle cannot assemble W at these sizes,
so it computes sampled outputs one by one (brute-force ray sums, per-voxel
adjoint sums) and the checks below reach every launch path:
  - rays on the first and last view of every record chunk (the strip records
    are rebuilt per chunk of views);
  - the adjoint with y restricted to the views of one adjoint run (each run
    of each chunk sums into its own partial volume), sampled voxels;
  - four volumes per call (the two-by-two-pixel batched adjoint and the
    four-volume forward), bitwise equal to single calls and sampled against
    the oracle;
  - the consistency invariants of Sec. I at every voxel and every ray of one
    view per chunk: W^T 1 = N_p |voxel| where a voxel's shadow stays on the
    detector in every view, and W 1 = the measure of the grid box inside each
    element's beam (one clip per element);
  - the dot-product test of the adjoint pair (Sec. IV footnote).
Every comparison logs its measured error (tests/_errlog.py).
"""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2511_12235_amd import workloads as wl
from paper_2511_12235_amd.projector import SystemMatrix

from _errlog import note, record

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
TOL = {"fp64": 1e-12, "fp32": 1e-5}
# W^T 1 at always-lit voxels: FP64 at the FP64 bar; FP32 sums about 4 strip
# volumes per view over the 360 views of the 256^3 scan (72 per adjoint run,
# 15 partial volumes), whose recursive-summation bound is ~(72 + 15) 2^-24
DOT = {"fp64": 1e-12, "fp32": 1e-6}
INV = {"fp64": 1e-12, "fp32": 6e-6}
CASES = [("c2", "fp32"), ("c2", "fp64"), ("c3", "fp32"), ("c3", "fp64")]


def _say(*msg):
    print("[case]", *msg, flush=True)


def _geom(cfg):
    return wl.c2_cone128() if cfg == "c2" else wl.c3_cone256()


def _seed(cfg):
    return 1 if cfg == "c2" else 2


def _t(a, prec):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV, torch.float64 if prec == "fp64" else torch.float32)


def _chunks(g, V):
    return [(v0, min(v0 + V, g.n_p)) for v0 in range(0, g.n_p, V)]


def _ray(g, view, r, k):
    return (view * g.det_nz + r) * g.det_ny + k


@pytest.mark.parametrize("cfg,prec", CASES)
def test_forward_every_chunk(cfg, prec):
    g = _geom(cfg)
    A = SystemMatrix(g, prec, device=DEV)
    V, runs = A.launch_shape()
    chunks = _chunks(g, V)
    _say("full-size forward", cfg, prec, "chunks", len(chunks), "views per chunk", V)
    assert len(chunks) >= 1 and (cfg != "c3" or len(chunks) > 1)
    # the ellipsoids leave much of the detector dark; a faint uniform background
    # makes every ray that meets the grid carry a nonzero sum
    x = wl.ellipse_phantom(g, 10, seed=_seed(cfg)) + wl.uniform(g.vol_shape, 7, 0.0, 1e-3)
    y = A.forward(_t(x, prec)).double().cpu().numpy().ravel()
    rng = np.random.default_rng(11)
    rays, owner = [], []
    for c, (v0, v1) in enumerate(chunks):
        for view in sorted({v0, v1 - 1}):
            rays.append(_ray(g, view, g.det_nz // 2, g.det_ny // 2))
            for _ in range(2):
                rays.append(_ray(g, view, int(rng.integers(g.det_nz)), int(rng.integers(g.det_ny))))
            owner += [c] * 3
    rays, owner = np.asarray(rays, dtype=np.int64), np.asarray(owner)
    yo = O.forward_rays(g, x, rays)
    assert np.count_nonzero(yo) > len(rays) // 2
    rel, _ = record("forward rays, chunk-edge views, %s %s" % (cfg, prec), y[rays], yo, TOL[prec])
    assert rel <= TOL[prec]
    for c in range(len(chunks)):  # each chunk on its own
        sel = owner == c
        assert np.linalg.norm(y[rays[sel]] - yo[sel]) <= TOL[prec] * np.linalg.norm(yo[sel]), c


@pytest.mark.parametrize("cfg,prec", CASES)
def test_adjoint_every_run(cfg, prec):
    g = _geom(cfg)
    A = SystemMatrix(g, prec, device=DEV)
    V, runs = A.launch_shape()
    _say("full-size adjoint runs", cfg, prec, "views per chunk", V, "runs", runs)
    ws = A.workspace(1)
    ys = wl.uniform(g.sino_shape, 9)
    rng = np.random.default_rng(12)
    got, ref = [], []
    for v0, v1 in _chunks(g, V):
        n = v1 - v0
        for gr in range(runs):
            a, b = v0 + n * gr // runs, v0 + n * (gr + 1) // runs
            if b <= a:
                continue
            ym = np.zeros_like(ys)
            ym[a:b] = ys[a:b]
            xb = A.back(_t(ym, prec), ws=ws).double().cpu().numpy().ravel()
            vox = rng.choice(g.n_vox, size=6, replace=False)
            xo = O.back(g, ym, vox)
            assert np.count_nonzero(xo) >= 3, (a, b)
            assert np.linalg.norm(xb[vox] - xo) <= TOL[prec] * np.linalg.norm(xo), (a, b)
            got.append(xb[vox])
            ref.append(xo)
    record("adjoint voxels, every run of every chunk, %s %s" % (cfg, prec), np.concatenate(got),
           np.concatenate(ref), TOL[prec])


def test_batch4_256():
    """Four volumes per call at 256^3 (the four-volume forward and the
    two-by-two-pixel adjoint): bitwise the single-volume results, and sampled
    outputs of two of the volumes against the oracle."""
    g = wl.c3_cone256()
    _say("full-size batch of 4", "c3 fp32")
    A = SystemMatrix(g, "fp32", device=DEV)
    V, _ = A.launch_shape()
    X = np.stack([wl.ellipse_phantom(g, 10, seed=2 + i) + wl.uniform(g.vol_shape, 40 + i, 0.0, 1e-3)
                  for i in range(4)])
    Y = np.stack([wl.uniform(g.sino_shape, 30 + i) for i in range(4)])
    Xt, Yt = _t(X, "fp32"), _t(Y, "fp32")
    yb = A.forward(Xt)
    xb = A.back(Yt)
    ws = A.workspace(1)
    for i in range(4):
        assert torch.equal(yb[i], A.forward(Xt[i], ws=ws)), i
        assert torch.equal(xb[i], A.back(Yt[i], ws=ws)), i
    rng = np.random.default_rng(13)
    rays = np.asarray([_ray(g, v, int(rng.integers(g.det_nz)), int(rng.integers(g.det_ny)))
                       for v0, v1 in _chunks(g, V) for v in (v0, v1 - 1)], dtype=np.int64)
    y3 = yb[3].double().cpu().numpy().ravel()
    yo = O.forward_rays(g, X[3], rays)
    assert np.count_nonzero(yo) > len(rays) // 2
    rel, _ = record("forward rays, batch of 4, volume 3, c3 fp32", y3[rays], yo, TOL["fp32"])
    assert rel <= TOL["fp32"]
    vox = rng.choice(g.n_vox, size=24, replace=False)
    x2 = xb[2].double().cpu().numpy().ravel()
    rel, _ = record("adjoint voxels, batch of 4, volume 2, c3 fp32", x2[vox], O.back(g, Y[2], vox), TOL["fp32"])
    assert rel <= TOL["fp32"]


def _always_lit(g):
    """Voxels whose shadow lies on the detector in every view: with rho the
    largest distance of a top-view corner from the rotation axis, every view
    has depth l >= s - rho and |t| <= rho, so |u| <= D rho / (s - rho) and
    |v| <= D max|z| / (s - rho)."""
    D = g.s + g.d
    xs = g.x0 + np.arange(g.nx + 1) * g.a
    ys = g.y0 + np.arange(g.ny + 1) * g.b
    zs = g.z0 + np.arange(g.nz + 1) * g.c
    rx = np.maximum(np.abs(xs[:-1]), np.abs(xs[1:]))
    ry = np.maximum(np.abs(ys[:-1]), np.abs(ys[1:]))
    rho = np.sqrt(rx[None, :] ** 2 + ry[:, None] ** 2)          # [ny, nx]
    zmax = np.maximum(np.abs(zs[:-1]), np.abs(zs[1:]))          # [nz]
    umax = D * rho / (g.s - rho)
    vmax = D * zmax[:, None, None] / (g.s - rho)[None]
    u_ok = (umax < -g.det_y0) & (umax < g.det_y0 + g.det_ny * g.dy)
    v_ok = (vmax < -g.det_z0) & (vmax < g.det_z0 + g.det_nz * g.dz)
    return u_ok[None] & v_ok


@pytest.mark.parametrize("cfg,prec", CASES)
def test_consistency_invariants(cfg, prec):
    g = _geom(cfg)
    A = SystemMatrix(g, prec, device=DEV)
    V, _ = A.launch_shape()
    _say("full-size invariants", cfg, prec)
    dt = A.dtype
    ws = A.workspace(1)
    # W^T 1 = N_p |voxel| on always-lit voxels, element-wise
    xb = A.back(torch.ones(A.sino_shape, dtype=dt, device=DEV), ws=ws).double().cpu().numpy()
    mask = _always_lit(g)
    assert mask.sum() > 0.3 * g.n_vox
    ref = g.n_p * g.a * g.b * g.c
    err = np.abs(xb[mask] - ref) / ref
    note("W^T 1 = N_p|voxel|, %d always-lit voxels, %s %s" % (mask.sum(), cfg, prec), float(err.max()),
         float(err.max()), int(mask.sum()), INV[prec], kind="max_rel")
    assert err.max() <= INV[prec]
    # W 1 against the grid-box clip, every ray of the first view of each chunk
    y1 = A.forward(torch.ones(A.vol_shape, dtype=dt, device=DEV), ws=ws).double().cpu().numpy()
    got, exp = [], []
    for v0, _ in _chunks(g, V):
        gb = O.ray_gridbox_view(g, v0)
        assert np.linalg.norm(y1[v0] - gb) <= TOL[prec] * np.linalg.norm(gb), v0
        got.append(y1[v0].ravel())
        exp.append(gb.ravel())
    record("W 1 = grid-box clip, all rays of %d views, %s %s" % (len(got), cfg, prec), np.concatenate(got),
           np.concatenate(exp), TOL[prec])
    # dot-product test of the pair (Sec. IV footnote: adjoint mismatch)
    x = wl.random_unit(g.vol_shape, 5)
    y = wl.random_unit(g.sino_shape, 6)
    Wx = A.forward(_t(x, prec), ws=ws).double().cpu().numpy()
    Wty = A.back(_t(y, prec), ws=ws).double().cpu().numpy()
    lhs, rhs = float(np.vdot(Wx, y)), float(np.vdot(x, Wty))
    mis = abs(lhs - rhs) / (np.linalg.norm(Wx) * np.linalg.norm(y))
    note("dot test <Wx,y> vs <x,W^T y>, %s %s" % (cfg, prec), mis, mis, 1, DOT[prec], kind="dot")
    assert mis <= DOT[prec]
