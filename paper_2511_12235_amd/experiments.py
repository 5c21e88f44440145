"""The paper's synthetic checkerboard reconstructions (Sec. IV, "Synthetic
Data" of the 2D and the 3D case), run on the GPU operators.

Each run: a checkerboard of 4 blocks per axis (values 0 and 1), the
projection data p = W u / ||W|| + noise with Gaussian noise of standard
deviation sigma = 1e-4, the spectral norm ||W|| from 100 power iterations,
and Nesterov's accelerated gradient on
    F(u) = 1/2 |W u / ||W|| - p|^2 + lambda/2 |u|^2,   lambda = 1e-4,
from u = 0 for 1000 iterations (2D) or 500 (3D).  The scan: 60 views
equidistant in [0, 2 pi), 60 detector elements (60 x 60 in 3D) of 0.75,
source-origin and origin-detector distance 250 (Sec. IV; the distances are
garbled in the text and read as s = d = 250).

The paper leaves the pixel size at the larger resolutions open ("a = b = 1"
while N grows).  Two readings are offered:
  "fov"  -- the image side stays 16 units, so the pixel is 16 / N (every
            voxel stays inside the beam; 64^2 unknowns exceed the 60 x 60
            data: the underdetermined regime the paper describes);
  "unit" -- the pixel stays 1, so the image grows to N units and its outer
            part leaves the field of view (22.5 units at the centre).
The paper stops NAG once |grad F|^2 < 1e-9 (or at the iteration budget).
Here the whole budget runs once, which gives the gradient at every
extrapolated point; the first k at which it falls below the bound is the
stop, and the solve is repeated for exactly k iterations (deterministic, so
the same trajectory) to give the iterate at the stop.  Both MSEs are
reported.

The MSE the paper prints for its area/volume-based reconstructions
(Sec. IV, figures "2D-checkerboard" and "3D-checkerboard-slices") are
listed beside ours as context only: the noise draw, the pixel size and the
solver details are not fully given.
"""
from __future__ import annotations

import json
import sys
from typing import Optional

import numpy as np
import torch

from . import workloads as wl
from .projector import SystemMatrix

# printed MSE of the area/volume-based reconstructions (Sec. IV figures)
PAPER_MSE = {2: {16: 0.06, 32: 0.08, 48: 0.08, 64: 0.08},
             3: {16: 0.035, 32: 0.081, 48: 0.11, 64: 0.13}}
N_VIEWS, N_DET, DET_PITCH, DIST = 60, 60, 0.75, 250.0
SIGMA, LAM, POWER_ITERS = 1e-4, 1e-4, 100
ITERS = {2: 1000, 3: 500}
STOP = 1e-9


def geometry(dim: int, n: int, reading: str = "fov") -> wl.Geometry:
    """Checkerboard scan of an n^dim grid (see the module text for the readings)."""
    if reading not in ("fov", "unit"):
        raise ValueError("reading must be 'fov' or 'unit'")
    pitch = 16.0 / n if reading == "fov" else 1.0
    if dim == 2:
        return wl.make_geometry(2, (n, n), (pitch, pitch), N_VIEWS, DIST, DIST, (N_DET,), (DET_PITCH,))
    return wl.make_geometry(3, (n, n, n), (pitch, pitch, pitch), N_VIEWS, DIST, DIST,
                            (N_DET, N_DET), (DET_PITCH, DET_PITCH))


def checkerboard(g: wl.Geometry, blocks: int = 4) -> np.ndarray:
    """0/1 checkerboard with `blocks` blocks per axis, shape g.vol_shape."""
    def idx(n):
        return (np.arange(n) * blocks) // n
    ix, iy = idx(g.nx), idx(g.ny)
    if g.dim == 2:
        return ((iy[:, None] + ix[None, :]) % 2).astype(np.float64).reshape(g.vol_shape)
    iz = idx(g.nz)
    return ((iz[:, None, None] + iy[None, :, None] + ix[None, None, :]) % 2).astype(np.float64)


def noise(g: wl.Geometry, seed: int) -> np.ndarray:
    """The measurement noise, N(0, sigma^2) per detector element."""
    return np.random.default_rng(seed).normal(0.0, SIGMA, size=g.sino_shape)


def start_vector(g: wl.Geometry, seed: int) -> np.ndarray:
    """Random start of the power iteration."""
    return wl.uniform(g.vol_shape, seed)


def run(dim: int, n: int, reading: str = "fov", precision: str = "fp64", seed: int = 0,
        device: Optional[str] = None, iters: Optional[int] = None) -> dict:
    """One checkerboard reconstruction on the GPU; returns its figures."""
    dev = torch.device(device or "cuda:0")
    g = geometry(dim, n, reading)
    A = SystemMatrix(g, precision, device=dev)
    dt = A.dtype
    u = checkerboard(g)
    v0 = torch.from_numpy(start_vector(g, seed + 1)).to(dev, dt)
    norm = A.power_norm(v0, POWER_ITERS)
    nv = float(norm.item())
    ut = torch.from_numpy(u).to(dev, dt)
    p = A.forward(ut) / nv + torch.from_numpy(noise(g, seed + 2)).to(dev, dt)
    k = iters if iters is not None else ITERS[dim]
    x, hist = A.nag(p, k, norm, lam=LAM, wscale=1.0 / nv)
    xs = x.double().cpu().numpy()
    h = hist.cpu().numpy()[:, 0]
    below = np.nonzero(h < STOP)[0]
    k_stop = int(below[0]) if below.size else k
    xk = xs
    if k_stop < k:
        xk = A.nag(p, k_stop, norm, lam=LAM, wscale=1.0 / nv)[0].double().cpu().numpy()
    return {"dim": dim, "n": n, "reading": reading, "precision": precision,
            "pitch": g.a, "norm": nv, "iters": k, "stop_iter": k_stop,
            "grad2_last": float(h[-1]),
            "mse": float(np.mean((xs - u) ** 2)),
            "mse_at_stop": float(np.mean((xk - u) ** 2)),
            "paper_mse": PAPER_MSE[dim].get(n),
            "x": xs}


def main(argv=None) -> None:
    import argparse
    ap = argparse.ArgumentParser(description="checkerboard reconstructions of Sec. IV")
    ap.add_argument("--dims", default="2,3")
    ap.add_argument("--sizes", default="16,32,48,64")
    ap.add_argument("--readings", default="fov,unit")
    ap.add_argument("--precision", default="fp64")
    args = ap.parse_args(argv)
    for dim in [int(v) for v in args.dims.split(",")]:
        for reading in args.readings.split(","):
            for n in [int(v) for v in args.sizes.split(",")]:
                r = run(dim, n, reading, args.precision)
                r.pop("x")
                print(json.dumps(r), flush=True)


if __name__ == "__main__":
    main(sys.argv[1:])
