"""Pins of the line-based oracle (oracle/lines.py) against facts fixed outside
it: hand-computed path lengths of an axis-parallel line, the half-open rule
for a line lying in a voxel face, path lengths by dense sampling of the line,
the per-voxel pieces tiling the line's chord through the grid box, and the
convergence of the "measure" weighting to the exact clipping oracle's W as k
grows (the area/volume matrix of Sec. I, computed by an unrelated method).
"""
import types

import numpy as np
import pytest

from oracle import lines as LN
from oracle import oracle as O
from paper_2511_12235_amd import workloads as wl


def _axis_line_geometry(ny):
    # phi = 0, three detector elements of pitch 1 centred on the axis: the
    # middle element's single sub-line (k = 1) is the line u = 0, i.e. y = 0
    return wl.make_geometry(2, (5, ny), (1.0, 1.0), 1, 10.0, 10.0, (3,), (1.0,), phi=[0.0])


def test_axis_parallel_line_hand_values():
    g = _axis_line_geometry(5)
    L = LN.row(g, 1, "length", 0, 0, 1).reshape(g.vol_shape)[0]
    expect = np.zeros((5, 5))
    expect[2, :] = 1.0  # y = 0 is the middle of row 2; every pixel is crossed over its width a = 1
    np.testing.assert_allclose(L, expect, rtol=0, atol=1e-14)
    # measure weighting: x(alpha) = s - alpha D with D = 20, so pixel ix is
    # crossed for alpha in [(10 - X_{ix+1}) / 20, (10 - X_ix) / 20], X_ix = ix - 2.5;
    # its weight is dy D (alpha_1^2 - alpha_0^2) / 2 with dy = 1
    Q = LN.row(g, 1, "measure", 0, 0, 1).reshape(g.vol_shape)[0]
    for ix in range(5):
        a0, a1 = (10 - (ix - 1.5)) / 20.0, (10 - (ix - 2.5)) / 20.0
        a0, a1 = min(a0, a1), max(a0, a1)
        assert Q[2, ix] == pytest.approx(20.0 * (a1 ** 2 - a0 ** 2) / 2.0, rel=1e-14)
    assert Q.sum() == pytest.approx(10.0 * (0.625 ** 2 - 0.375 ** 2), rel=1e-14)


def test_line_in_a_face_counted_once():
    g = _axis_line_geometry(4)  # y = 0 is the face between rows 1 and 2
    L = LN.row(g, 1, "length", 0, 0, 1).reshape(g.vol_shape)[0]
    assert L[2].sum() == pytest.approx(5.0, rel=1e-14)  # half-open rule: the row with lo <= 0 < hi
    assert L[1].sum() == 0.0 and L[0].sum() == 0.0 and L[3].sum() == 0.0


def test_path_length_by_dense_sampling():
    rng = np.random.default_rng(5)
    for trial in range(30):
        lo = rng.uniform(-2, 2, 3)
        h = rng.uniform(0.3, 2.0, 3)
        box = types.SimpleNamespace(dim=3, nx=1, ny=1, nz=1, a=h[0], b=h[1], c=h[2],
                                    x0=lo[0], y0=lo[1], z0=lo[2], vol_shape=(1, 1, 1))
        S = rng.uniform(-8, 8, 3)
        target = lo + h * rng.uniform(0.2, 0.8, 3)  # aim through the box
        d = target - S
        a_in, a_out = LN.box_intervals(box, S, d)
        n = 400000
        alpha = (np.arange(n) + 0.5) * (3.0 / n)
        p = S[None, :] + alpha[:, None] * d[None, :]
        inside = np.all((p >= lo) & (p <= lo + h), axis=1)
        est = inside.sum() * (3.0 / n) * np.linalg.norm(d)
        got = (a_out.item() - a_in.item()) * np.linalg.norm(d)
        assert abs(got - est) <= 2 * (3.0 / n) * np.linalg.norm(d) + 1e-12, trial


@pytest.mark.parametrize("dim", [2, 3])
def test_pieces_tile_the_grid_chord(dim):
    if dim == 2:
        g = wl.make_geometry(2, (9, 7), (1.1, 0.8), 5, 30.0, 20.0, (13,), (1.2,))
    else:
        g = wl.make_geometry(3, (7, 6, 5), (1.0, 1.2, 0.9), 4, 30.0, 20.0, (11, 9), (1.1, 1.0))
    k = 3
    for view in range(g.n_p):
        for my in range(g.det_ny):
            for s in range(k):
                mz, t = (g.det_nz // 2, 1) if dim == 3 else (0, 0)
                S, d, _, _ = LN.sub_line(g, view, my, s, k, mz, t)
                lo, hi = LN.box_intervals(g, S, d)
                hit = lo < hi
                A0, A1 = LN.grid_interval(g, S, d)
                assert np.sum((hi - lo)[hit]) == pytest.approx(A1 - A0, rel=1e-12, abs=1e-14)
                assert np.sum((hi ** 3 - lo ** 3)[hit]) == pytest.approx(A1 ** 3 - A0 ** 3, rel=1e-12, abs=1e-14)
                # pieces are disjoint: sorted by entry, each starts where the previous ends
                order = np.argsort(lo[hit])
                a, b = lo[hit][order], hi[hit][order]
                np.testing.assert_allclose(a[1:], b[:-1], rtol=1e-12, atol=1e-14)


def _rel_fro(A, B):
    D = (A - B).tocsr()
    return float(np.sqrt(D.multiply(D).sum()) / np.sqrt(B.multiply(B).sum()))


def test_measure_weighting_converges_to_exact_area_2d():
    g = wl.make_geometry(2, (10, 8), (1.0, 1.2), 5, 25.0, 20.0, (9,), (1.5,))
    W = O.matrix(g)
    e = {k: _rel_fro(LN.matrix(g, k, "measure"), W) for k in (2, 8, 32)}
    assert e[8] < e[2] / 8 and e[32] < e[8] / 8  # midpoint rule: O(k^-2)
    assert e[32] < 2e-3


def test_measure_weighting_converges_to_exact_volume_3d():
    g = wl.make_geometry(3, (5, 4, 3), (1.0, 1.1, 0.9), 3, 25.0, 20.0, (6, 5), (1.4, 1.3))
    W = O.matrix(g)
    e = {k: _rel_fro(LN.matrix(g, k, "measure"), W) for k in (2, 8, 32)}
    # midpoint rule in (u, v); on this small grid still short of the k^-2 regime
    assert e[8] < e[2] / 4 and e[32] < e[8] / 8
    assert e[32] < 5e-3


def test_length_weighting_is_the_mean_of_sub_line_lengths():
    g = wl.make_geometry(2, (6, 5), (1.0, 1.0), 3, 25.0, 20.0, (7,), (1.3,))
    k = 4
    for view in range(g.n_p):
        for my in range(g.det_ny):
            r = LN.row(g, k, "length", view, 0, my)
            total = 0.0
            for s in range(k):
                S, d, _, _ = LN.sub_line(g, view, my, s, k)
                A0, A1 = LN.grid_interval(g, S, d)
                total += (A1 - A0) * np.linalg.norm(d) / k
            assert r.sum() == pytest.approx(total, rel=1e-12, abs=1e-14)


@pytest.mark.parametrize("dim", [2, 3])
def test_column_view_equals_matrix_columns(dim):
    """The per-voxel form (vectorised over sub-lines) and the per-line form
    (vectorised over voxels) give the same matrix."""
    if dim == 2:
        g = wl.make_geometry(2, (6, 5), (1.0, 1.2), 3, 25.0, 20.0, (7,), (1.3,))
    else:
        g = wl.make_geometry(3, (4, 3, 3), (1.0, 1.1, 0.9), 2, 25.0, 20.0, (6, 5), (1.4, 1.3))
    k = 3
    for weight in LN.WEIGHTS:
        W = LN.matrix(g, k, weight).toarray()
        for j in range(g.n_vox):
            iz, rem = divmod(j, g.ny * g.nx)
            iy, ix = divmod(rem, g.nx)
            col = np.concatenate([LN.column(g, k, weight, v, ix, iy, iz).ravel() for v in range(g.n_p)])
            np.testing.assert_allclose(col, W[:, j], rtol=1e-12, atol=1e-14)
