"""Seeded synthetic inputs: scanner geometries, phantoms and measurement noise.

This module only *describes* problems; it holds none of the projector's
arithmetic.  Both the HIP path and the test oracle take their inputs from
here, so it imports neither of them.

Geometry conventions (Sec. III-A and the appendix "Fundamental relations" of
arXiv 2511.12235): the source sits at (s cos(phi), s sin(phi), 0) and rotates
counter-clockwise about +z; the flat detector is perpendicular to the central
ray at distance d beyond the origin; detector corners lie on a grid of pitch
(dy, dz).  The paper puts voxel vertices at multiples of (a, b, c) and the
first detector corner at a multiple of (dy, dz); here both grids get an
explicit first corner so that centred grids with any element count can be
described.  The defaults centre both grids on the rotation axis.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional, Sequence

import numpy as np


@dataclasses.dataclass(frozen=True)
class Geometry:
    """Fan-beam (dim=2) or circular cone-beam (dim=3) flat-detector scan.

    Names follow the paper: voxel side lengths ``a, b, c``; source-origin
    distance ``s``; origin-detector distance ``d``; detector element side
    lengths ``dy, dz``; ``n_p`` projection angles ``phi``.  ``det_ny`` and
    ``det_nz`` count detector columns (along the in-plane detector axis) and
    rows (along z).  In 2D ``nz == det_nz == 1`` and ``c``/``dz`` are unused.
    """

    dim: int
    nx: int
    ny: int
    nz: int
    a: float
    b: float
    c: float
    x0: float
    y0: float
    z0: float
    phi: np.ndarray
    s: float
    d: float
    det_ny: int
    det_nz: int
    dy: float
    dz: float
    det_y0: float
    det_z0: float
    trig: Optional[np.ndarray] = None

    @property
    def n_p(self) -> int:
        return int(len(self.phi))

    @property
    def n_vox(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def n_rays(self) -> int:
        return self.n_p * self.det_nz * self.det_ny

    @property
    def vol_shape(self):
        return (self.nz, self.ny, self.nx)

    @property
    def sino_shape(self):
        return (self.n_p, self.det_nz, self.det_ny)

    @property
    def voxel_measure(self) -> float:
        return self.a * self.b * (self.c if self.dim == 3 else 1.0)

    def with_(self, **kw) -> "Geometry":
        return dataclasses.replace(self, **kw)


def make_geometry(dim: int, n: Sequence[int], pitch: Sequence[float], n_p: int,
                  s: float, d: float, det: Sequence[int], det_pitch: Sequence[float],
                  phi: Optional[Sequence[float]] = None,
                  corner: Optional[Sequence[float]] = None,
                  det_corner: Optional[Sequence[float]] = None,
                  trig: Optional[np.ndarray] = None) -> Geometry:
    """Build a geometry; grids default to being centred on the origin.

    ``n``/``pitch`` are (nx, ny[, nz]) / (a, b[, c]); ``det``/``det_pitch``
    are (det_ny[, det_nz]) / (dy[, dz]).  Angles default to
    phi_k = 2 pi k / n_p (equidistant in [0, 2 pi), as in Sec. IV).
    """
    if dim == 2:
        nx, ny = n[:2]
        nz = 1
        a, b = pitch[:2]
        c = 1.0
        det_ny, det_nz = det[0], 1
        dy, dz = det_pitch[0], 1.0
    else:
        nx, ny, nz = n
        a, b, c = pitch
        det_ny, det_nz = det
        dy, dz = det_pitch
    if corner is None:
        corner = (-nx * a / 2.0, -ny * b / 2.0, -nz * c / 2.0 if dim == 3 else -0.5)
    if det_corner is None:
        det_corner = (-det_ny * dy / 2.0, -det_nz * dz / 2.0 if dim == 3 else -0.5)
    if phi is None:
        phi = 2.0 * np.pi * np.arange(n_p, dtype=np.float64) / n_p
    phi = np.ascontiguousarray(np.asarray(phi, dtype=np.float64))
    if len(phi) != n_p:
        raise ValueError("len(phi) != n_p")
    if trig is not None:
        trig = np.ascontiguousarray(np.asarray(trig, dtype=np.float64).reshape(n_p, 2))
    return Geometry(dim=dim, nx=int(nx), ny=int(ny), nz=int(nz), a=float(a), b=float(b),
                    c=float(c), x0=float(corner[0]), y0=float(corner[1]), z0=float(corner[2]),
                    phi=phi, s=float(s), d=float(d), det_ny=int(det_ny), det_nz=int(det_nz),
                    dy=float(dy), dz=float(dz), det_y0=float(det_corner[0]),
                    det_z0=float(det_corner[1]), trig=trig)


# --------------------------------------------------------------------------
# named workloads
# --------------------------------------------------------------------------

def c1_fan2d() -> Geometry:
    """2D fan beam: 64x64 pixels of 1 mm, 90 views over 360 deg, 96 detector
    elements of 1 mm, source-isocentre 500 mm, source-detector 1000 mm."""
    return make_geometry(2, (64, 64), (1.0, 1.0), 90, 500.0, 500.0, (96,), (1.0,))


def c2_cone128() -> Geometry:
    """3D cone beam: 128^3 voxels of 1 mm, 180 views, 192x128 detector of
    1.5 mm elements, SID 600 mm, SDD 1200 mm."""
    return make_geometry(3, (128, 128, 128), (1.0, 1.0, 1.0), 180, 600.0, 600.0,
                         (192, 128), (1.5, 1.5))


def c3_cone256() -> Geometry:
    """3D cone beam: 256^3 voxels of 0.8 mm, 360 views, 384x256 detector of
    1.2 mm elements, SID 800 mm, SDD 1400 mm."""
    return make_geometry(3, (256, 256, 256), (0.8, 0.8, 0.8), 360, 800.0, 600.0,
                         (384, 256), (1.2, 1.2))


def c4_batch128() -> Geometry:
    """Differentiable batch geometry: 128^3 voxels, 120 views, 160x128
    detector.  Pitch and distances are not given for this workload; the
    128^3 cone-beam values (1 mm, 1.5 mm, 600/1200 mm) are used."""
    return make_geometry(3, (128, 128, 128), (1.0, 1.0, 1.0), 120, 600.0, 600.0,
                         (160, 128), (1.5, 1.5))


def serving_geometry(kind: str, n_p: int = 360) -> Geometry:
    """Request geometries of the serving mix: 2D 256^2 (360 views, 384 cells
    of 1.5 mm at the 2D source distances) and 3D 64^3 / 128^3 (1 mm voxels,
    1.5 mm cells, 600/1200 mm) or 256^3 (as the 256^3 workload), with
    detector cells = 1.5 x grid size."""
    if kind == "2d256":
        return make_geometry(2, (256, 256), (1.0, 1.0), 360, 500.0, 500.0, (384,), (1.5,))
    if kind == "3d64":
        return make_geometry(3, (64, 64, 64), (1.0, 1.0, 1.0), n_p, 600.0, 600.0,
                             (96, 96), (1.5, 1.5))
    if kind == "3d128":
        return make_geometry(3, (128, 128, 128), (1.0, 1.0, 1.0), n_p, 600.0, 600.0,
                             (192, 192), (1.5, 1.5))
    if kind == "3d256":
        return make_geometry(3, (256, 256, 256), (0.8, 0.8, 0.8), n_p, 800.0, 600.0,
                             (384, 384), (1.2, 1.2))
    raise ValueError(kind)


def scaled(g: Geometry, n: Sequence[int], det: Sequence[int], n_p: int) -> Geometry:
    """Same scanner with a smaller grid/detector/view count and the same
    field of view (pitches scaled so the grid and detector keep their size)."""
    if g.dim == 2:
        a = g.a * g.nx / n[0]
        b = g.b * g.ny / n[1]
        dy = g.dy * g.det_ny / det[0]
        return make_geometry(2, n, (a, b), n_p, g.s, g.d, det, (dy,))
    a = g.a * g.nx / n[0]
    b = g.b * g.ny / n[1]
    c = g.c * g.nz / n[2]
    dy = g.dy * g.det_ny / det[0]
    dz = g.dz * g.det_nz / det[1]
    return make_geometry(3, n, (a, b, c), n_p, g.s, g.d, det, (dy, dz))


# --------------------------------------------------------------------------
# phantoms
# --------------------------------------------------------------------------

def _voxel_centres(g: Geometry):
    xc = g.x0 + (np.arange(g.nx) + 0.5) * g.a
    yc = g.y0 + (np.arange(g.ny) + 0.5) * g.b
    zc = g.z0 + (np.arange(g.nz) + 0.5) * g.c
    return xc, yc, zc


def ellipse_phantom(g: Geometry, n_shapes: int, seed: int,
                    mu_max: float = 0.02) -> np.ndarray:
    """Sum of random ellipses (2D) or ellipsoids (3D), FP64, shape
    ``g.vol_shape``.  Centres are U(-0.5, 0.5) x half field of view per axis,
    semi-axes U(0.1, 0.45) x half field of view, orientation U(0, pi) in 2D or
    a random rotation (QR of a Gaussian matrix, signs fixed) in 3D,
    attenuation U(0, mu_max) per mm.  A voxel takes the sum of the
    attenuations of the shapes that contain its centre."""
    rng = np.random.default_rng(seed)
    xc, yc, zc = _voxel_centres(g)
    half = np.array([g.nx * g.a, g.ny * g.b, g.nz * g.c]) / 2.0
    mid = np.array([g.x0, g.y0, g.z0]) + half
    out = np.zeros(g.vol_shape, dtype=np.float64)
    if g.dim == 2:
        X, Y = np.meshgrid(xc, yc, indexing="xy")
        for _ in range(n_shapes):
            cen = mid[:2] + rng.uniform(-0.5, 0.5, 2) * half[:2]
            ax = rng.uniform(0.1, 0.45, 2) * half[:2]
            th = rng.uniform(0.0, np.pi)
            mu = rng.uniform(0.0, mu_max)
            dx, dy = X - cen[0], Y - cen[1]
            p = (dx * np.cos(th) + dy * np.sin(th)) / ax[0]
            q = (-dx * np.sin(th) + dy * np.cos(th)) / ax[1]
            out[0] += mu * (p * p + q * q <= 1.0)
        return out
    Z, Y, X = np.meshgrid(zc, yc, xc, indexing="ij")
    for _ in range(n_shapes):
        cen = mid + rng.uniform(-0.5, 0.5, 3) * half
        ax = rng.uniform(0.1, 0.45, 3) * half
        q_, r_ = np.linalg.qr(rng.standard_normal((3, 3)))
        R = q_ * np.sign(np.diag(r_))
        mu = rng.uniform(0.0, mu_max)
        P = np.stack([X - cen[0], Y - cen[1], Z - cen[2]], axis=-1) @ R
        inside = ((P / ax) ** 2).sum(axis=-1) <= 1.0
        out += mu * inside
    return out


def poisson_sinogram(y_clean: np.ndarray, g: Geometry, photons: float,
                     seed: int) -> np.ndarray:
    """Poisson counting noise on a projection of measures (mm^2 or mm^3).

    The projector returns beam-integrated attenuation, i.e. a line integral
    times the beam cross-section.  The cross-section at the isocentre
    A_iso = dy * s / D (2D) or dy * dz * (s / D)^2 (3D) turns it into a line
    integral q = y / A_iso; counts are N ~ Poisson(photons * exp(-q)) and the
    noisy measurement is A_iso * (-log(max(N, 1) / photons)).
    """
    rng = np.random.default_rng(seed)
    D = g.s + g.d
    if g.dim == 2:
        a_iso = g.dy * g.s / D
    else:
        a_iso = g.dy * g.dz * (g.s / D) ** 2
    q = np.asarray(y_clean, dtype=np.float64) / a_iso
    n = rng.poisson(photons * np.exp(-q))
    return a_iso * (-np.log(np.maximum(n, 1) / photons))


def random_unit(shape, seed: int) -> np.ndarray:
    """Gaussian vector normalised to unit Euclidean norm (FP64)."""
    v = np.random.default_rng(seed).standard_normal(shape)
    return v / np.linalg.norm(v)


def uniform(shape, seed: int, lo: float = 0.0, hi: float = 1.0) -> np.ndarray:
    return np.random.default_rng(seed).uniform(lo, hi, size=shape)
