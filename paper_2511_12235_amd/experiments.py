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

``complexity`` is the paper's 2D complexity comparison (Sec. IV, figure
"complexity"): a 40 x 40 phantom, data p = W u / ||W|| + noise (sigma =
1e-4) from the consistent (area) model, reconstructed by NAG with lambda in
{1e-5, 1e-4} using the area matrix and the line-based model with k = 1, 2,
4, ... lines per detector element ("length": averaged path lengths, the
paper's comparison; "measure": the midpoint rule of the element's area),
each operator normalised by its own spectral norm.  Reported per run: the
MSE to the phantom at the paper's stopping rule, the iterations, the solve
time and the time of one forward + adjoint pair.  The paper's phantom is a
Shepp-Logan head; a seeded random-ellipse phantom of the same size stands in.
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


COMPLEXITY_LAMS = (1e-5, 1e-4)
COMPLEXITY_KS = (1, 2, 4, 8, 16, 32, 64)


def complexity_phantom(g, seed: int = 0) -> np.ndarray:
    """Seeded ellipse phantom scaled to [0, 1] (stand-in for Shepp-Logan)."""
    u = wl.ellipse_phantom(g, 8, seed=seed)
    u = u - u.min()
    return u / max(float(u.max()), 1e-300)


def _time_pair(A, x, y, line, reps: int = 20) -> float:
    """Milliseconds of one forward + adjoint pair (events on the current stream)."""
    f = (lambda: (A.forward(x), A.back(y))) if line is None else \
        (lambda: (A.line_forward(x, line[0], line[1]), A.line_back(y, line[0], line[1])))
    f()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        f()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def complexity(n: int = 40, reading: str = "fov", lams=COMPLEXITY_LAMS, ks=COMPLEXITY_KS,
               weights=("length", "measure"), seed: int = 0, device: Optional[str] = None):
    """The complexity comparison; yields one dict per (model, k, lambda)."""
    import time
    dev = torch.device(device or "cuda:0")
    g = geometry(2, n, reading)
    A = SystemMatrix(g, "fp64", device=dev)
    u = complexity_phantom(g, seed)
    ut = torch.from_numpy(u).to(dev, torch.float64)
    v0 = torch.from_numpy(start_vector(g, seed + 1)).to(dev, torch.float64)
    nv = float(A.power_norm(v0, POWER_ITERS).item())
    p = A.forward(ut) / nv + torch.from_numpy(noise(g, seed + 2)).to(dev, torch.float64)
    models = [("area", 0, None)] + [("line-" + w, k, (k, w)) for w in weights for k in ks]
    ysino = torch.ones(g.sino_shape, dtype=torch.float64, device=dev)
    for name, k, line in models:
        norm = A.power_norm(v0, POWER_ITERS, line=line)
        nm = float(norm.item())
        pair_ms = _time_pair(A, ut, ysino, line)
        for lam in lams:
            x, hist = A.nag(p, ITERS[2], norm, lam=lam, wscale=1.0 / nm, line=line)
            h = hist.cpu().numpy()[:, 0]
            below = np.nonzero(h < STOP)[0]
            k_stop = int(below[0]) if below.size else ITERS[2]
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            xs, _ = A.nag(p, k_stop, norm, lam=lam, wscale=1.0 / nm, line=line)
            torch.cuda.synchronize()
            solve_s = time.perf_counter() - t0
            xk = xs.double().cpu().numpy()
            yield {"model": name, "k": k, "lambda": lam, "norm": nm, "stop_iter": k_stop,
                   "mse": float(np.mean((xk - u) ** 2)), "solve_ms": 1e3 * solve_s,
                   "pair_ms": pair_ms}


def main(argv=None) -> None:
    import argparse
    ap = argparse.ArgumentParser(description="checkerboard reconstructions of Sec. IV")
    ap.add_argument("--dims", default="2,3")
    ap.add_argument("--sizes", default="16,32,48,64")
    ap.add_argument("--readings", default="fov,unit")
    ap.add_argument("--precision", default="fp64")
    ap.add_argument("--complexity", action="store_true",
                    help="run the 2D complexity comparison (area vs line-based) instead")
    args = ap.parse_args(argv)
    if args.complexity:
        for r in complexity():
            print(json.dumps(r), flush=True)
        return
    for dim in [int(v) for v in args.dims.split(",")]:
        for reading in args.readings.split(","):
            for n in [int(v) for v in args.sizes.split(",")]:
                r = run(dim, n, reading, args.precision)
                r.pop("x")
                print(json.dumps(r), flush=True)


if __name__ == "__main__":
    main(sys.argv[1:])
