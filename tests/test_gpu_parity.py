"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Bars: FP64 plans within 1e-12 relative L2 of the oracle, FP32 plans within
1e-5; footprint boxes and the CSR pattern bit-exact; dot-product test at
1e-12 (FP64) / 1e-6 (FP32).  Small geometries are compared in full; the
256^3 and 128^3 cone-beam workloads are compared on sampled rays and voxels
that the oracle computes one by one, plus the row-sum invariant.
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


def _t(a, prec):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV, torch.float64 if prec == "fp64" else torch.float32)


def _say(*msg):
    print("[case]", *msg, flush=True)


DEG_TRIG = np.array([[1.0, 0.0], [0.0, 1.0], [-1.0, 0.0], [0.0, -1.0],
                     [np.cos(1e-9), np.sin(1e-9)], [np.cos(np.pi / 2 + 1e-7), np.sin(np.pi / 2 + 1e-7)],
                     [np.cos(np.pi / 4), np.sin(np.pi / 4)], [np.cos(2.2), np.sin(2.2)]])


def geometries():
    g = {}
    g["c1_fan64"] = wl.c1_fan2d()
    g["fan_odd"] = wl.make_geometry(2, (37, 29), (1.1, 0.9), 23, 80.0, 60.0, (51,), (1.7,),
                                    det_corner=(-40.0, 0.0))
    g["cone_small"] = wl.scaled(wl.c2_cone128(), (26, 22, 20), (30, 26), 12)
    g["cone_degenerate"] = wl.make_geometry(3, (12, 11, 10), (1.0, 1.0, 1.0), len(DEG_TRIG), 40.0, 30.0,
                                            (20, 18), (1.2, 1.1), trig=DEG_TRIG,
                                            phi=np.arctan2(DEG_TRIG[:, 1], DEG_TRIG[:, 0]))
    g["cone_aniso_offset"] = wl.make_geometry(3, (17, 13, 70), (0.7, 1.3, 0.45), 9, 35.0, 25.0,
                                              (29, 83), (0.9, 0.5),
                                              det_corner=(-11.0, -20.0), corner=(-5.0, -9.0, -14.0))
    # tall voxels under fine detector rows: up to 19 rows per voxel and view
    g["cone_many_rows"] = wl.make_geometry(3, (10, 9, 6), (1.0, 1.1, 2.5), 7, 30.0, 30.0,
                                           (24, 60), (1.0, 0.35))
    # short scan: 9 seeded angles in [0.3, 0.3 + pi + fan angle), not equidistant
    fan = 2.0 * np.arctan(12.0 / 60.0)
    phi = np.sort(np.random.default_rng(41).uniform(0.3, 0.3 + np.pi + fan, 9))
    g["cone_short_scan"] = wl.make_geometry(3, (14, 12, 9), (1.0, 1.0, 1.0), len(phi), 40.0, 35.0,
                                            (30, 20), (1.1, 1.3), phi=phi)
    return g


GEOMS = geometries()
SMALL = list(GEOMS)


@pytest.fixture(scope="module")
def oracle_mats():
    return {}


def _W(name, cache):
    if name not in cache:
        cache[name] = O.matrix(GEOMS[name])
    return cache[name]


@pytest.mark.parametrize("name", SMALL)
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_forward_adjoint_match_oracle(name, prec, oracle_mats):
    g = GEOMS[name]
    _say("forward/adjoint", name, prec)
    W = _W(name, oracle_mats)
    A = SystemMatrix(g, prec, device=DEV)
    x = wl.ellipse_phantom(g, 5, seed=0) + 0.1 * wl.uniform(g.vol_shape, 1)
    y = wl.uniform(g.sino_shape, 2)
    yg = A.forward(_t(x, prec)).cpu().numpy()
    xg = A.back(_t(y, prec)).cpu().numpy()
    torch.cuda.synchronize()
    assert record("forward W x, %s %s" % (name, prec), yg, W @ x.ravel(), TOL[prec])[0] <= TOL[prec]
    assert record("adjoint W^T y, %s %s" % (name, prec), xg, W.T @ y.ravel(), TOL[prec])[0] <= TOL[prec]


@pytest.mark.parametrize("name", SMALL)
def test_csr_pattern_and_values(name, oracle_mats):
    g = GEOMS[name]
    _say("csr", name)
    W = _W(name, oracle_mats)
    A = SystemMatrix(g, "fp64", device=DEV)
    rp, ci, va = A.weights_csr("fp64")
    assert np.array_equal(rp, W.indptr.astype(np.int64))
    assert np.array_equal(ci, W.indices.astype(np.int32))
    assert record("CSR values, %s fp64" % name, va, W.data, 1e-12)[0] <= 1e-12
    rp32, ci32, va32 = A.weights_csr("fp32")
    assert np.array_equal(rp32, rp) and np.array_equal(ci32, ci)
    assert record("CSR values, %s fp32" % name, va32, W.data, 1e-5)[0] <= 1e-5


@pytest.mark.parametrize("name", ["c1_fan64", "cone_small", "cone_degenerate", "cone_aniso_offset",
                                  "cone_short_scan"])
def test_footprints_bit_exact(name):
    g = GEOMS[name]
    _say("footprints", name)
    A = SystemMatrix(g, "fp32", device=DEV)
    for v in sorted({0, 1, g.n_p // 2, g.n_p - 1}):
        assert np.array_equal(A.footprints(v), O.footprints(g, v)), v


@pytest.mark.parametrize("name", ["fan_odd", "cone_small", "cone_aniso_offset", "cone_many_rows"])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_dot_product(name, prec):
    g = GEOMS[name]
    _say("dot", name, prec)
    A = SystemMatrix(g, prec, device=DEV)
    x = wl.random_unit(g.vol_shape, 5)
    y = wl.random_unit(g.sino_shape, 6)
    Wx = A.forward(_t(x, prec)).double().cpu().numpy()
    Wty = A.back(_t(y, prec)).double().cpu().numpy()
    lhs, rhs = float(np.vdot(Wx, y)), float(np.vdot(x, Wty))
    bound = 1e-12 if prec == "fp64" else 1e-6
    mis = abs(lhs - rhs) / (np.linalg.norm(Wx) * np.linalg.norm(y))
    note("dot test, %s %s" % (name, prec), mis, mis, 1, bound, kind="dot")
    assert mis <= bound


@pytest.mark.parametrize("name", ["fan_odd", "cone_small"])
@pytest.mark.parametrize("batch", [3, 8, 11])
def test_batched_equals_single(name, batch):
    g = GEOMS[name]
    _say("batch", name, batch)
    A = SystemMatrix(g, "fp32", device=DEV)
    X = np.stack([wl.ellipse_phantom(g, 4, seed=10 + i) for i in range(batch)])
    Y = np.stack([wl.uniform(g.sino_shape, 20 + i) for i in range(batch)])
    yb = A.forward(_t(X, "fp32")).cpu().numpy()
    xb = A.back(_t(Y, "fp32")).cpu().numpy()
    for i in range(batch):
        assert np.array_equal(yb[i], A.forward(_t(X[i], "fp32")).cpu().numpy())
        assert np.array_equal(xb[i], A.back(_t(Y[i], "fp32")).cpu().numpy())


@pytest.mark.parametrize("name", ["cone_small", "cone_many_rows", "cone_aniso_offset"])
def test_fp32_forward_magnitudes(name, oracle_mats):
    """The FP32 forward sums its straddle terms on a fixed-point grid set by
    max|x| of each volume: the relative error must not depend on the scale of
    x, volumes of very different scale share a batch, zero stays zero and a
    non-finite voxel makes (only) its own volume's measurements NaN."""
    g = GEOMS[name]
    _say("fp32 magnitudes", name)
    W = _W(name, oracle_mats)
    A = SystemMatrix(g, "fp32", device=DEV)
    x = wl.ellipse_phantom(g, 5, seed=7) + 0.1 * wl.uniform(g.vol_shape, 8)
    for s in (1e-30, 1e-8, 1e8, 1e30):
        yg = A.forward(_t(x * s, "fp32")).double().cpu().numpy()
        assert record("forward, x scaled by %.0e, %s fp32" % (s, name), yg, W @ (x * s).ravel(),
                      TOL["fp32"])[0] <= TOL["fp32"], s
    X = np.stack([x * 1e-20, x, x * 1e20, np.zeros_like(x)])
    yb = A.forward(_t(X, "fp32")).cpu().numpy()
    for i in range(len(X)):
        assert np.array_equal(yb[i], A.forward(_t(X[i], "fp32")).cpu().numpy()), i
    assert not yb[3].any()
    Xn = np.stack([x, x.copy()])
    Xn[1].flat[Xn[1].size // 2] = np.nan
    yn = A.forward(_t(Xn, "fp32")).cpu().numpy()
    assert np.array_equal(yn[0], yb[1])
    assert np.isnan(yn[1]).all()


@pytest.mark.parametrize("name", ["cone_small", "cone_aniso_offset", "cone_many_rows"])
@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_kept_records_bitwise(name, prec):
    """sm_plan_keep_records: the same bits with the records kept in the plan
    as with the records rebuilt per call, for single and batched calls;
    a budget below the record size is refused and changes nothing; the
    workspace shrinks by the records while they are kept."""
    g = GEOMS[name]
    _say("kept records", name, prec)
    A = SystemMatrix(g, prec, device=DEV)
    X = np.stack([wl.ellipse_phantom(g, 4, seed=50 + i) for i in range(3)])
    Y = np.stack([wl.uniform(g.sino_shape, 60 + i) for i in range(3)])
    Xt, Yt = _t(X, prec), _t(Y, prec)
    ref = (A.forward(Xt[0]), A.back(Yt[0]), A.forward(Xt), A.back(Yt))
    ws_before = A.workspace_bytes(3)
    nbytes = A.record_bytes()
    assert nbytes > 0
    with pytest.raises(RuntimeError):
        A.keep_records(nbytes - 1)
    assert A.workspace_bytes(3) == ws_before
    A.keep_records()
    assert A.workspace_bytes(3) < ws_before
    got = (A.forward(Xt[0]), A.back(Yt[0]), A.forward(Xt), A.back(Yt))
    for a, b in zip(got, ref):
        assert torch.equal(a, b)
    A.keep_records(0)
    assert A.workspace_bytes(3) == ws_before
    assert torch.equal(A.forward(Xt[0]), ref[0])


def test_deterministic_repeat():
    g = GEOMS["cone_small"]
    _say("determinism")
    A = SystemMatrix(g, "fp32", device=DEV)
    x = _t(wl.ellipse_phantom(g, 5, seed=3), "fp32")
    y = _t(wl.uniform(g.sino_shape, 4), "fp32")
    assert torch.equal(A.forward(x), A.forward(x))
    assert torch.equal(A.back(y), A.back(y))


@pytest.mark.parametrize("which", ["c2_cone128", "c3_cone256"])
def test_full_size_sampled(which):
    """Full-size workloads in the launch configuration the benchmark times:
    sampled rays (brute force in the oracle), sampled voxels, and the row
    sums W 1 against one clip of the whole grid box per ray."""
    g = getattr(wl, which)()
    _say("full size", which)
    rng = np.random.default_rng(7)
    A = SystemMatrix(g, "fp32", device=DEV)
    x = wl.ellipse_phantom(g, 10, seed=1 if which == "c2_cone128" else 2)
    y = A.forward(_t(x, "fp32")).cpu().numpy().ravel()
    n_rays = 24 if which == "c3_cone256" else 48
    rays = rng.choice(g.n_rays, size=n_rays, replace=False)
    # rays near the central row and on the degenerate views are included
    views = np.array([0, g.n_p // 4, g.n_p // 2])
    extra = (views * g.det_nz + g.det_nz // 2) * g.det_ny + g.det_ny // 2
    rays = np.concatenate([rays, extra])
    yo = O.forward_rays(g, x, rays)
    assert record("forward rays, random, %s fp32" % which, y[rays], yo, 1e-5)[0] <= 1e-5
    # row sums of W against the grid-box clip
    ones = A.forward(torch.ones(g.vol_shape, device=DEV)).cpu().numpy().ravel()
    gb = []
    for i in rays[:16]:
        v, rem = divmod(int(i), g.det_nz * g.det_ny)
        r, k = divmod(rem, g.det_ny)
        gb.append(O.ray_gridbox(g, v, k, r))
    assert record("W 1 = grid-box clip, 16 rays, %s fp32" % which, ones[rays[:16]], gb, 1e-5)[0] <= 1e-5
    # adjoint on sampled voxels
    ys = wl.uniform(g.sino_shape, 9)
    xb = A.back(_t(ys, "fp32")).cpu().numpy().ravel()
    vox = rng.choice(g.n_vox, size=48, replace=False)
    xo = O.back(g, ys, vox)
    assert record("adjoint voxels, random, %s fp32" % which, xb[vox], xo, 1e-5)[0] <= 1e-5


def test_nnz_count_beyond_2pow32_work_items():
    """The pair count of the 256^3 scan (n_p * n_vox ~ 6e9 > 2^32) equals
    the sum of the counts of four 90-view scans, and its per-voxel-view
    density matches the oracle's count on one view of the central slab."""
    import ctypes as C
    from paper_2511_12235_amd import _lib
    g = wl.c3_cone256()
    _say("nnz count", g.n_p * g.n_vox)

    def count(geom):
        A = SystemMatrix(geom, "fp32", device=DEV)
        n = C.c_int64(0)
        _lib.check(_lib.lib().sm_weights_csr(A._plan, _lib.SM_FP32, C.byref(n), None, None, None), "count")
        return n.value

    total = count(g)
    parts = sum(count(g.with_(phi=g.phi[q::4].copy())) for q in range(4))
    assert total == parts
    slab = wl.make_geometry(3, (g.nx, g.ny, 16), (g.a, g.b, g.c), 1, g.s, g.d, (g.det_ny, g.det_nz),
                            (g.dy, g.dz), phi=g.phi[45:46])
    rows, _, _ = O.triplets(slab)
    assert count(slab) == len(rows)


def test_kernel_timing_counts_dispatches():
    """sm_timing_*: one timed interval per dispatch, none while disabled,
    and reading clears the record."""
    from paper_2511_12235_amd import _lib
    g = GEOMS["cone_small"]
    _say("kernel timing")
    A = SystemMatrix(g, "fp32", device=DEV)
    x = _t(wl.ellipse_phantom(g, 5, seed=3), "fp32")
    ws = A.workspace(1)
    with pytest.raises(_lib.SmError):
        A.read_timing()
    A.timing(True)
    y = A.forward(x, ws=ws)
    A.back(y, ws=ws)
    t = A.read_timing()
    assert t["prefix"][0] == 1 and t["transpose"][0] == 1
    assert t["forward"][0] >= 1 and t["forward"][0] == t["adjoint"][0]
    assert t["records"][0] == 2 * t["forward"][0]
    assert all(ms > 0.0 for _, ms in t.values())
    assert all(n == 0 for n, _ in A.read_timing().values())
    A.timing(False)
    A.forward(x, ws=ws)
    with pytest.raises(_lib.SmError):
        A.read_timing()
