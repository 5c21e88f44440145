"""Line-based system matrix with k lines per detector element -- FP64 CPU
oracle (test infrastructure only: the test suite, the smoke check and the
CPU-baseline leg of the benchmark use it; the HIP library never does).

This is the comparison model of Sec. IV: instead of the measure of a voxel
inside a detector element's beam, the element is sampled by k (2D) or k x k
(3D) lines from the source, and the weights of the lines are averaged (the
complexity experiment of Sec. IV, "2D complexity", raises k to approach the
area-based matrix).

Sub-lines.  Detector element m (column m_y, row m_z) is sampled at the cell
midpoints of a k-fold subdivision:
    u = det_y0 + (m_y + (s + 1/2) / k) dy,   v = det_z0 + (m_z + (t + 1/2) / k) dz.
In the view's frame (depth l along the central ray, lateral t, height z;
the scanner geometry of Sec. III-A) the sub-line's points are
(l, t, z) = alpha (D, u, v), alpha >= 0, alpha = 1 on the detector, and in
world coordinates x = (s - l) cos(phi) - t sin(phi), y = (s - l) sin(phi) +
t cos(phi).  Voxel j is the closed box of Sec. III-A; the line is inside it for
alpha in [alpha_in, alpha_out] (slab method).  Along an axis the line runs
parallel to, the half-open condition lo <= S_axis < hi decides (so a line in a
voxel face belongs to exactly one of the two voxels).

Weights (one term per sub-line and voxel, alpha_in < alpha_out):
  "length":  the mean over the element's sub-lines of the path length
             R (alpha_out - alpha_in), R = |(D, u, v)| -- the classical
             line model whose averages the paper uses;
  "measure": the midpoint rule over the element of its exact measure written
             in line coordinates.  With (l, t, z) -> (l, u, v) having
             Jacobian (l / D)^(dim - 1) and l = alpha D,
                 2D: area   = int du int (l/D) dl     -> (dy/k) D (alpha_out^2 - alpha_in^2) / 2,
                 3D: volume = int du dv int (l/D)^2 dl -> (dy dz/k^2) D (alpha_out^3 - alpha_in^3) / 3
             per sub-line.  As k grows it tends to the exact W of the
             consistent model (Sec. I); the plain average of lengths does
             not (it weights depth differently), which is the saturation
             the paper observes in its complexity experiment.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

WEIGHTS = ("length", "measure")


def _trig(g, view):
    if g.trig is not None:
        return float(g.trig[view][0]), float(g.trig[view][1])
    return float(np.cos(g.phi[view])), float(np.sin(g.phi[view]))


def sub_line(g, view, m_y, s, k, m_z=0, t=0):
    """Source S and direction d of sub-line (s, t) of element (m_y, m_z);
    the detector point is S + d."""
    cp, sn = _trig(g, view)
    D = g.s + g.d
    u = g.det_y0 + (m_y + (s + 0.5) / k) * g.dy
    v = g.det_z0 + (m_z + (t + 0.5) / k) * g.dz if g.dim == 3 else 0.0
    S = np.array([g.s * cp, g.s * sn, 0.0])
    # x(alpha) = (s - alpha D) cos - alpha u sin, y(alpha) = (s - alpha D) sin + alpha u cos
    d = np.array([-D * cp - u * sn, -D * sn + u * cp, v])
    return S, d, u, v


def box_intervals(g, S, d):
    """[alpha_in, alpha_out] of the line S + alpha d (alpha >= 0) inside every
    voxel box, as two arrays of shape vol_shape (empty where in >= out)."""
    lo = np.zeros(g.vol_shape)
    hi = np.full(g.vol_shape, np.inf)
    axes = [(0, g.x0, g.a, g.nx, (1, 1, g.nx)), (1, g.y0, g.b, g.ny, (1, g.ny, 1))]
    if g.dim == 3:
        axes.append((2, g.z0, g.c, g.nz, (g.nz, 1, 1)))
    for ax, o, h, n, shape in axes:
        edges_lo = o + np.arange(n) * h
        edges_hi = o + (np.arange(n) + 1) * h
        if d[ax] != 0.0:
            a1 = (edges_lo - S[ax]) / d[ax]
            a2 = (edges_hi - S[ax]) / d[ax]
            lo = np.maximum(lo, np.minimum(a1, a2).reshape(shape))
            hi = np.minimum(hi, np.maximum(a1, a2).reshape(shape))
        else:
            inside = (edges_lo <= S[ax]) & (S[ax] < edges_hi)
            hi = np.where(inside.reshape(shape), hi, -np.inf)
    return lo, hi


def sub_line_weights(g, view, m_y, s, k, weight, m_z=0, t=0):
    """Weights of one sub-line against every voxel (flat, length n_vox),
    already divided by the sub-line count where the weighting averages."""
    S, d, u, v = sub_line(g, view, m_y, s, k, m_z, t)
    lo, hi = box_intervals(g, S, d)
    hit = lo < hi
    a0 = np.where(hit, lo, 0.0)
    a1 = np.where(hit, hi, 0.0)
    D = g.s + g.d
    if weight == "length":
        R = float(np.sqrt(d @ d))
        w = R * (a1 - a0) / (k ** (g.dim - 1))
    elif weight == "measure":
        if g.dim == 2:
            w = (g.dy / k) * D * (a1 ** 2 - a0 ** 2) / 2.0
        else:
            w = (g.dy * g.dz / k ** 2) * D * (a1 ** 3 - a0 ** 3) / 3.0
    else:
        raise ValueError("weight must be 'length' or 'measure'")
    return np.where(hit, w, 0.0).ravel()


def _subs(g, k):
    return [(s, t) for t in range(k if g.dim == 3 else 1) for s in range(k)]


def row(g, k, weight, view, m_z, m_y):
    """Row of detector element (view, m_z, m_y): flat array of n_vox weights."""
    acc = np.zeros(g.n_vox)
    for s, t in _subs(g, k):
        acc += sub_line_weights(g, view, m_y, s, k, weight, m_z, t)
    return acc


def matrix(g, k, weight):
    """The whole line-based matrix as CSR (rows: (view, m_z, m_y); columns:
    (iz, iy, ix)); entries with positive weight only."""
    rows, cols, vals = [], [], []
    for view in range(g.n_p):
        for mz in range(g.det_nz):
            for my in range(g.det_ny):
                r = row(g, k, weight, view, mz, my)
                nz = np.nonzero(r > 0.0)[0]
                i = (view * g.det_nz + mz) * g.det_ny + my
                rows.append(np.full(nz.size, i))
                cols.append(nz)
                vals.append(r[nz])
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(g.n_rays, g.n_vox))


def forward_rows(g, k, weight, x, rays):
    """(W_line x) at the listed (view, m_z, m_y) elements, one row at a time."""
    xf = np.asarray(x, dtype=np.float64).ravel()
    return np.array([row(g, k, weight, v, mz, my) @ xf for v, mz, my in rays])


def column(g, k, weight, view, ix, iy, iz=0):
    """Weights of voxel (ix, iy, iz) for every detector element of one view,
    shape (det_nz, det_ny): the same definition, vectorised over the view's
    sub-lines instead of the voxels."""
    cp, sn = _trig(g, view)
    D = g.s + g.d
    gu = np.arange(g.det_ny * k)
    u = g.det_y0 + (gu // k + (gu % k + 0.5) / k) * g.dy
    if g.dim == 3:
        gv = np.arange(g.det_nz * k)
        v = g.det_z0 + (gv // k + (gv % k + 0.5) / k) * g.dz
    else:
        v = np.zeros(1)
    U, V = np.meshgrid(u, v)  # (rows, columns) of sub-lines
    S = (g.s * cp, g.s * sn, 0.0)
    d = (-D * cp - U * sn, -D * sn + U * cp, V)
    lo = np.zeros(U.shape)
    hi = np.full(U.shape, np.inf)
    axes = [(0, g.x0 + ix * g.a, g.x0 + (ix + 1) * g.a), (1, g.y0 + iy * g.b, g.y0 + (iy + 1) * g.b)]
    if g.dim == 3:
        axes.append((2, g.z0 + iz * g.c, g.z0 + (iz + 1) * g.c))
    for ax, e0, e1 in axes:
        da = d[ax]
        par = da == 0.0
        with np.errstate(divide="ignore", invalid="ignore"):
            a1 = (e0 - S[ax]) / da
            a2 = (e1 - S[ax]) / da
        inside = (e0 <= S[ax]) & (S[ax] < e1)
        lo = np.where(par, lo, np.maximum(lo, np.minimum(a1, a2)))
        hi = np.where(par, np.where(inside, hi, -np.inf), np.minimum(hi, np.maximum(a1, a2)))
    hit = lo < hi
    a0 = np.where(hit, lo, 0.0)
    a1 = np.where(hit, hi, 0.0)
    if weight == "length":
        R = np.sqrt(d[0] ** 2 + d[1] ** 2 + d[2] ** 2)
        w = R * (a1 - a0) / (k ** (g.dim - 1))
    elif weight == "measure":
        if g.dim == 2:
            w = (g.dy / k) * D * (a1 ** 2 - a0 ** 2) / 2.0
        else:
            w = (g.dy * g.dz / k ** 2) * D * (a1 ** 3 - a0 ** 3) / 3.0
    else:
        raise ValueError("weight must be 'length' or 'measure'")
    w = np.where(hit, w, 0.0)
    kv = k if g.dim == 3 else 1
    return w.reshape(g.det_nz, kv, g.det_ny, k).sum(axis=(1, 3))


def back_voxels(g, k, weight, y, voxels):
    """(W_line^T y) at the listed flat voxel indices, one voxel at a time."""
    yv = np.asarray(y, dtype=np.float64).reshape(g.sino_shape)
    out = []
    for j in voxels:
        iz, rem = divmod(int(j), g.ny * g.nx)
        iy, ix = divmod(rem, g.nx)
        out.append(sum(float(np.sum(column(g, k, weight, v, ix, iy, iz) * yv[v])) for v in range(g.n_p)))
    return np.array(out)


def grid_interval(g, S, d):
    """[alpha_in, alpha_out] of the line inside the whole grid box (one box,
    the same slab rule); used to check that the per-voxel pieces tile it."""
    lo, hi = 0.0, np.inf
    axes = [(0, g.x0, g.a * g.nx), (1, g.y0, g.b * g.ny)]
    if g.dim == 3:
        axes.append((2, g.z0, g.c * g.nz))
    for ax, o, span in axes:
        if d[ax] != 0.0:
            a1, a2 = (o - S[ax]) / d[ax], (o + span - S[ax]) / d[ax]
            lo, hi = max(lo, min(a1, a2)), min(hi, max(a1, a2))
        elif not (o <= S[ax] < o + span):
            return 0.0, 0.0
    return (lo, hi) if lo < hi else (0.0, 0.0)
