"""Throughput of the exact cone-beam projector pair W x + W^T y on one MI355X.

Workload: 256^3 voxels of 0.8 mm, 360 views over 360 deg, 384 x 256 flat
detector of 1.2 mm cells, source-isocentre 800 mm, source-detector 1400 mm,
FP32 values with FP64 geometry; input = seeded random-ellipsoid phantom
(10 ellipsoids).  One step = one forward projection plus one adjoint of the
whole volume/sinogram, inputs resident in HBM.  The metric counts exact
nonzero voxel-detector pairs (W_ij > 1e-12 voxel volume) per second:
value = 2 nnz / (t_forward + t_adjoint).

Prints one JSON line (see the contract in the design doc).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
# VALU issue rate with packed FP32 disabled: 256 CU x 4 SIMD x 16 lanes x 2.4 GHz
VALU_PEAK_LANE_OPS = 256 * 4 * 16 * 2.4e9


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp64"])
    ap.add_argument("--config", default="c3", choices=["c2", "c3"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-views", type=int, default=16)
    return ap.parse_args()


def cpu_baseline(g, n_views):
    """The FP64 oracle timed on a bounded sample of the same scanner: the
    central 16-slice slab (nx x ny x 16 voxels), n_views views spread over
    the scan, forward only (the adjoint visits the same pairs)."""
    import numpy as np
    from oracle import oracle as O
    from paper_2511_12235_amd import workloads as wl
    slab = wl.make_geometry(3, (g.nx, g.ny, 16), (g.a, g.b, g.c), g.n_p, g.s, g.d,
                            (g.det_ny, g.det_nz), (g.dy, g.dz), phi=g.phi)
    x = wl.ellipse_phantom(slab, 10, seed=2)
    views = np.linspace(0, g.n_p - 1, n_views).round().astype(np.int32)
    counts = np.zeros(1, dtype=np.int64)
    nnz = 0
    for v in views:
        rows, cols, vals = O.triplets(slab, views=(int(v), int(v) + 1))
        nnz += len(vals)
    t0 = time.perf_counter()
    O.forward(slab, x, views=views)
    dt = time.perf_counter() - t0
    return {"value": nnz / dt, "unit": "pairs/s", "cores": O.num_threads(), "kind": "oracle",
            "sample": "FP64 clipping oracle, forward W x on the central 16-slice slab "
                      "(%dx%dx16 voxels) of the 256^3 scanner, %d of %d views, %d pairs in %.1f s"
                      % (g.nx, g.ny, n_views, g.n_p, nnz, dt)}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only (this build has no multi-GPU path); "
              "got --gpus %d" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    from paper_2511_12235_amd import workloads as wl
    from paper_2511_12235_amd.projector import SystemMatrix

    g = wl.c3_cone256() if args.config == "c3" else wl.c2_cone128()
    dev = torch.device("cuda:0")
    A = SystemMatrix(g, args.precision, device=dev)
    dt = A.dtype
    x = torch.from_numpy(wl.ellipse_phantom(g, 10, seed=2)).to(dev, dt)
    ws = A.workspace(1)
    y = torch.empty(A.sino_shape, dtype=dt, device=dev)
    xb = torch.empty(A.vol_shape, dtype=dt, device=dev)

    # exact number of nonzero pairs (FP64 pattern), counted on the GPU
    import ctypes as C
    from paper_2511_12235_amd import _lib
    nnz = C.c_int64(0)
    t0 = time.perf_counter()
    _lib.check(_lib.lib().sm_weights_csr(A._plan, _lib.SM_FP32, C.byref(nnz), None, None, None),
               "sm_weights_csr(count)")
    count_s = time.perf_counter() - t0
    nnz = nnz.value

    stream = torch.cuda.current_stream(dev)
    for _ in range(args.warmup):
        A.forward(x, out=y, ws=ws)
        A.back(y, out=xb, ws=ws)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True),
           torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    for e0, e1, e2 in ev:
        e0.record(stream)
        A.forward(x, out=y, ws=ws)
        e1.record(stream)
        A.back(y, out=xb, ws=ws)
        e2.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    t_f = np.array([a.elapsed_time(b) for a, b, _ in ev]) / 1e3
    t_b = np.array([b.elapsed_time(c) for _, b, c in ev]) / 1e3
    step = t_f + t_b
    value = 2.0 * nnz / float(np.mean(step))
    eff_bw = value * 8.0 / 1e9  # GB/s a stored FP32+int32 CSR matrix would stream
    res = {
        "metric": "Wx+W^Ty voxel-detector pairs/s at 256^3 (% HBM roofline); p50/p99 solve latency",
        "value": value,
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": float(np.mean(step)) * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.precision == "fp32" else "f64",
        "data": "synthetic",
        "config": {"workload": "cone-beam %d^3 voxels, %d views, %dx%d detector, forward + adjoint"
                               % (g.nx, g.n_p, g.det_ny, g.det_nz),
                   "nnz_pairs": nnz, "ms_forward": float(np.mean(t_f)) * 1e3,
                   "ms_adjoint": float(np.mean(t_b)) * 1e3, "nnz_count_s": count_s,
                   "wall_s": wall,
                   "pct_hbm_roofline_effective": 100.0 * eff_bw / HBM_PEAK_GBS},
    }
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(g, args.cpu_views)
    print(json.dumps(res))


if __name__ == "__main__":
    main()
