"""Throughput of the exact cone-beam projector pair W x + W^T y on one MI355X.

Workload: 256^3 voxels of 0.8 mm, 360 views over 360 deg, 384 x 256 flat
detector of 1.2 mm cells, source-isocentre 800 mm, source-detector 1400 mm,
FP32 values with FP64 geometry; input = seeded random-ellipsoid phantom
(10 ellipsoids).  One step = one forward projection plus one adjoint of the
whole volume/sinogram, inputs resident in HBM.  The metric counts exact
nonzero voxel-detector pairs (W_ij > 1e-12 voxel volume) per second:
value = 2 nnz / (t_forward + t_adjoint).

Prints one JSON line.  Besides the throughput it carries
  roofline     -- the dominant kernel (largest summed launch time, timed with
                  HIP events on the launch stream through sm_timing_*):
                  algorithmic FP operations per launch / mean launch time,
                  against the vector-ALU peak; traffic = HBM bytes per launch
                  from the committed counter summary, null when the kernel
                  sources changed since it was taken;
  cpu_baseline -- the FP64 clipping oracle on a bounded sample.

Extra modes (no GPU) turn rocprofv3 CSV output into the text summaries kept
under profiles/:
  --digest-stats KERNEL_STATS_CSV --out FILE --command "..."
  --digest-counters FETCH_CSV WRITE_CSV --kernel NAME --copy-mib N --out FILE --command "..."
  --digest-valu COUNTER_CSV --out FILE --command "..."
A further GPU mode times the stored-W path (device CSR of W and W^T, sparse
products) against the matrix-free operators on the 128^3 scan:
  --stored [--config c2]
and one the line-based comparison model (k lines per detector element,
sm_line_forward / sm_line_back) against the exact operators:
  --line [--line-ks 1,2] [--config c3]
"""
import argparse
import csv
import glob
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
# Vector ALU peak: 256 CUs x 4 SIMDs x 16 lanes x 2 flop per FMA x 2.4 GHz =
# 78.6 TFLOP/s.  That is the FP64 rate and the FP32 rate without packed-FP32
# instructions, which this library's build disables.
ALU_PEAK_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
# Algorithmic FP operations per nonzero pair: one evaluation of the
# cumulative column volume K on its piecewise branch (21 flop) plus the
# pair's multiply-add (2 flop).
FLOP_PER_PAIR = 23
KERNEL_SYMBOL = {"forward": "fwd3d_kernel", "adjoint": "back3d_kernel",
                 "records": "rec_kernel", "prefix": "columns_kernel",
                 "transpose": "from_columns_kernel"}
KERNEL_SYMBOL_2D = {"forward": "fwd2d_kernel", "adjoint": "back2d_kernel"}


def _geometry(config):
    from paper_2511_12235_amd import workloads as wl
    return CONFIGS[config](wl)


CONFIGS = {"c1": lambda wl: wl.c1_fan2d(), "c2": lambda wl: wl.c2_cone128(), "c3": lambda wl: wl.c3_cone256(),
           "c4": lambda wl: wl.c4_batch128(), "fan256": lambda wl: wl.serving_geometry("2d256")}


def _describe(g):
    if g.dim == 2:
        return "fan-beam %d^2 pixels, %d views, %d detector cells" % (g.nx, g.n_p, g.det_ny)
    return "cone-beam %d^3 voxels, %d views, %dx%d detector" % (g.nx, g.n_p, g.det_ny, g.det_nz)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp64"])
    ap.add_argument("--config", default="c3", choices=sorted(CONFIGS),
                    help="c3: the 256^3 headline workload; c2: 128^3, 180 views; c4: 128^3, 120 views; "
                         "c1: 2D fan 64^2, 90 views; fan256: 2D fan 256^2, 360 views (serving size)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--stored", action="store_true",
                    help="time the stored-W mode beside the matrix-free operators instead")
    ap.add_argument("--cpu-views", type=int, default=0,
                    help="views in the oracle sample (default: one per oracle thread)")
    ap.add_argument("--batch", type=int, default=1,
                    help="volumes per call (the weights are evaluated once for all of them)")
    ap.add_argument("--keep-records", action="store_true",
                    help="keep the strip records of every view in the plan (sm_plan_keep_records) "
                         "instead of rebuilding them in every call")
    ap.add_argument("--line", action="store_true",
                    help="time the line-based model (k lines per element) beside the exact operators")
    ap.add_argument("--line-ks", default="1,2")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="before timing, run one plain device copy of this many MiB "
                         "(reference for HBM counters)")
    ap.add_argument("--digest-stats", metavar="CSV")
    ap.add_argument("--digest-counters", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"))
    ap.add_argument("--digest-valu", metavar="CSV")
    ap.add_argument("--kernel", default="back3d_kernel")
    ap.add_argument("--nnz", type=int, default=0,
                    help="nonzero pairs of the profiled operator (--digest-valu: lane instructions per pair)")
    ap.add_argument("--out")
    ap.add_argument("--command", default="")
    return ap.parse_args()


# ----------------------------------------------------------------- profiles
def sources_digest():
    """sha256 over the HIP sources and build flags of the library."""
    h = hashlib.sha256()
    pkg = os.path.join(ROOT, "paper_2511_12235_amd")
    files = sorted(glob.glob(os.path.join(pkg, "csrc", "*"))) + [os.path.join(pkg, "build.py")]
    for f in files:
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def counters_file(config, precision, kernel):
    return os.path.join(ROOT, "profiles", "%s_%s_%s_hbm_counters.txt"
                        % (kernel, {"c3": "cone256", "c2": "cone128"}.get(config, config), precision))


def read_summary(path):
    vals = {}
    if not os.path.exists(path):
        return vals
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                vals[k.strip()] = v.strip()
    return vals


def traffic_per_launch(config, precision, kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary, or
    None when there is none or the library sources changed since."""
    s = read_summary(counters_file(config, precision, kernel))
    if not s or s.get("sources_sha256") != sources_digest():
        return None
    try:
        return float(s["hbm_bytes_per_dispatch"])
    except (KeyError, ValueError):
        return None


def _rows(path):
    with open(path, newline="") as fh:
        return list(csv.DictReader(fh))


def digest_stats(args):
    rows = _rows(args.digest_stats)
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    lines = ["# rocprofv3 --kernel-trace --stats summary", "command: %s" % args.command, "",
             "%-60s %7s %12s %12s %7s" % ("kernel", "calls", "avg_ms", "total_ms", "pct")]
    for r in rows:
        name = r["Name"]
        short = name.replace("(anonymous namespace)::", "").split("(")[0].replace("void ", "")
        lines.append("%-60s %7s %12.4f %12.3f %7.2f" % (short[:60], r["Calls"], float(r["AverageNs"]) / 1e6,
                                                       float(r["TotalDurationNs"]) / 1e6,
                                                       float(r["Percentage"])))
    _write(args.out, lines)


def _per_dispatch(rows, counter, match):
    vals = [float(r["Counter_Value"]) for r in rows
            if r["Counter_Name"] == counter and match(r["Kernel_Name"])]
    return vals


def digest_counters(args):
    fetch_rows, write_rows = _rows(args.digest_counters[0]), _rows(args.digest_counters[1])
    is_k = lambda n: args.kernel in n
    is_copy = lambda n: "copyBuffer" in n or ("copy" in n.lower() and args.kernel not in n)
    fk = _per_dispatch(fetch_rows, "FETCH_SIZE", is_k)
    wk = _per_dispatch(write_rows, "WRITE_SIZE", is_k)
    fc = max(_per_dispatch(fetch_rows, "FETCH_SIZE", is_copy) or [0.0])
    wc = max(_per_dispatch(write_rows, "WRITE_SIZE", is_copy) or [0.0])
    if not fk or not wk or fc <= 0 or wc <= 0:
        sys.exit("digest: kernel or copy dispatches missing from the counter files")
    copy_kib = args.copy_mib * 1024.0
    ff, wf = copy_kib / fc, copy_kib / wc
    fetch = sum(fk) / len(fk)
    write = sum(wk) / len(wk)
    hbm = (fetch * ff + write * wf) * 1024.0
    lines = ["# HBM traffic of %s from two rocprofv3 --pmc passes" % args.kernel,
             "command: %s" % args.command,
             "kernel: %s" % args.kernel,
             "dispatches: %d" % len(fk),
             "fetch_kib_per_dispatch: %.1f" % fetch,
             "write_kib_per_dispatch: %.1f" % write,
             "copy_mib: %d" % args.copy_mib,
             "copy_fetch_kib: %.1f" % fc,
             "copy_write_kib: %.1f" % wc,
             "fetch_scale: %.5f" % ff,
             "write_scale: %.5f" % wf,
             "hbm_bytes_per_dispatch: %.0f" % hbm,
             "sources_sha256: %s" % sources_digest()]
    _write(args.out, lines)


def digest_valu(args):
    """Vector-instruction issue of the 3D kernels from one rocprofv3 --pmc pass
    (SQ_INSTS_VALU, SQ_WAVES): a wave64 VALU instruction occupies its SIMD for
    4 cycles, so issue-bound time = insts x 4 / (1024 SIMDs x 2.4 GHz).  With
    --nnz (the operator's nonzero pairs, which one direction's launches cover
    once) it also reports VALU lane-instructions (64 per wave instruction) per
    pair."""
    rows = _rows(args.digest_valu)
    lines = ["# VALU issue of the 3D kernels from one rocprofv3 --pmc pass",
             "command: %s" % args.command,
             "issue_fraction = SQ_INSTS_VALU x 4 cycles / (1024 SIMDs x 2.4 GHz x duration)",
             "lane_insts_per_pair = 64 x SQ_INSTS_VALU summed over the launches / nnz"
             + (" (nnz = %d)" % args.nnz if args.nnz else " (no --nnz given)"), "",
             "%-16s %5s %12s %16s %12s %9s %10s" % ("kernel", "calls", "avg_ms", "valu_per_call", "waves", "issue",
                                                     "lane/pair")]
    for short in ("fwd3d_kernel", "back3d_kernel", "rec_kernel"):
        disp = {}
        for r in rows:
            if short not in r["Kernel_Name"]:
                continue
            d = disp.setdefault(r["Dispatch_Id"], {"t": (float(r["End_Timestamp"]) - float(r["Start_Timestamp"])) * 1e-9})
            d[r["Counter_Name"]] = float(r["Counter_Value"])
        if not disp:
            continue
        n = len(disp)
        t = sum(d["t"] for d in disp.values()) / n
        v = sum(d.get("SQ_INSTS_VALU", 0.0) for d in disp.values()) / n
        w = sum(d.get("SQ_WAVES", 0.0) for d in disp.values()) / n
        issue = v * 4.0 / (1024 * 2.4e9 * t) if t > 0 else 0.0
        # the record kernel runs once per direction and chunk: half its
        # launches cover the pairs once
        per_pair = 64.0 * v * (n / 2 if short == "rec_kernel" else n) / args.nnz if args.nnz else float("nan")
        lines.append("%-16s %5d %12.4f %16.4g %12.4g %9.3f %10.2f" % (short, n, t * 1e3, v, w, issue, per_pair))
    _write(args.out, lines)


def _write(path, lines):
    text = "\n".join(lines) + "\n"
    if path:
        os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
        with open(path, "w") as fh:
            fh.write(text)
    print(text, end="")


# ------------------------------------------------------------- CPU baseline
def cpu_baseline(g, n_views):
    """The FP64 oracle timed on a bounded sample of the same scanner: the
    central 16-slice slab (nx x ny x 16 voxels) seen from n_views views spread
    over the scan (one per oracle thread by default), forward W x only (the
    adjoint visits the same pairs).  Pairs are counted by the oracle outside
    the timed call."""
    import numpy as np
    from oracle import oracle as O
    from paper_2511_12235_amd import workloads as wl
    threads = O.num_threads()
    n_views = n_views if n_views > 0 else threads
    views = np.linspace(0, g.n_p - 1, n_views).round().astype(np.int64)
    sample = wl.make_geometry(3, (g.nx, g.ny, 16), (g.a, g.b, g.c), n_views, g.s, g.d,
                              (g.det_ny, g.det_nz), (g.dy, g.dz), phi=np.asarray(g.phi)[views])
    x = wl.ellipse_phantom(sample, 10, seed=2)
    t0 = time.perf_counter()
    O.forward(sample, x)
    dt = time.perf_counter() - t0
    nnz = O.count(sample)
    return {"value": nnz / dt, "unit": "pairs/s", "cores": min(threads, n_views), "kind": "oracle",
            "sample": "FP64 clipping oracle, forward W x on the central 16-slice slab "
                      "(%dx%dx16 voxels) of the %dx%dx%d scan, %d of its %d views, %d pairs in %.1f s"
                      % (g.nx, g.ny, g.nx, g.ny, g.nz, n_views, g.n_p, nnz, dt)}


# ------------------------------------------------------------- stored W
def stored_bench(args):
    """Stored-W mode against the matrix-free operators on one scan: build
    time of the device CSR pair, mean time of W x and W^T y by sparse
    products and by the matrix-free kernels, and the bytes each product
    streams (values + column indices + row offsets + input + output)."""
    import numpy as np
    import torch

    from paper_2511_12235_amd import workloads as wl
    from paper_2511_12235_amd.projector import StoredMatrix, SystemMatrix

    g = _geometry(args.config)
    dev = torch.device("cuda:0")
    A = SystemMatrix(g, args.precision, device=dev)
    dt = A.dtype
    x = torch.from_numpy(wl.ellipse_phantom(g, 10, seed=2)).to(dev, dt)
    yin = torch.from_numpy(wl.uniform(g.sino_shape, 3)).to(dev, dt)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    S = StoredMatrix(A)
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0
    ws = A.workspace(1)
    stream = torch.cuda.current_stream(dev)

    def timed(fn, reps):
        for _ in range(max(args.warmup, 1)):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            out = fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps, out

    reps = max(args.steps, 3)
    ms_sf, ys = timed(lambda: S.forward(x), reps)
    ms_sb, xs = timed(lambda: S.back(yin), reps)
    ms_mf, ym = timed(lambda: A.forward(x, ws=ws), reps)
    ms_mb, xm = timed(lambda: A.back(yin, ws=ws), reps)
    vb = 8 if args.precision == "fp64" else 4
    nnz = S.nnz
    b_fwd = nnz * (4 + vb) + 8 * (A.n_rays + 1) + vb * (A.n_vox + A.n_rays)
    b_back = nnz * (4 + vb) + 8 * (A.n_vox + 1) + vb * (A.n_vox + A.n_rays)
    rel = lambda a, b: float(torch.linalg.norm((a - b).double()) / torch.linalg.norm(b.double()))
    res = {"mode": "stored-W vs matrix-free", "config": {"workload": _describe(g)},
           "precision": args.precision, "nnz": nnz, "stored_bytes": 2 * nnz * (4 + vb),
           "build_s": build_s,
           "ms_forward": {"stored": ms_sf, "matrix_free": ms_mf},
           "ms_adjoint": {"stored": ms_sb, "matrix_free": ms_mb},
           "pairs_per_s": {"stored": 2 * nnz / ((ms_sf + ms_sb) / 1e3),
                           "matrix_free": 2 * nnz / ((ms_mf + ms_mb) / 1e3)},
           "stored_GBps": {"forward": b_fwd / ms_sf / 1e6, "adjoint": b_back / ms_sb / 1e6},
           "stored_vs_matrix_free_rel_l2": {"forward": rel(ys, ym), "adjoint": rel(xs, xm)}}
    print(json.dumps(res), flush=True)


def line_bench(args):
    """Line-based model against the exact operators on one scan: mean time
    of W_line x and W_line^T y for each k and weighting, the sub-lines per
    second of the forward and the voxel-views per second of the adjoint."""
    import torch

    from paper_2511_12235_amd import workloads as wl
    from paper_2511_12235_amd.projector import SystemMatrix

    g = _geometry(args.config)
    dev = torch.device("cuda:0")
    A = SystemMatrix(g, args.precision, device=dev)
    dt = A.dtype
    x = torch.from_numpy(wl.ellipse_phantom(g, 10, seed=2)).to(dev, dt)
    yin = torch.from_numpy(wl.uniform(g.sino_shape, 3)).to(dev, dt)
    ws = A.workspace(1)
    stream = torch.cuda.current_stream(dev)

    def timed(fn, reps):
        for _ in range(max(args.warmup, 1)):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    reps = max(args.steps, 3)
    rows = []
    for k in [int(v) for v in args.line_ks.split(",")]:
        for w in ("length", "measure"):
            mf = timed(lambda: A.line_forward(x, k, w), reps)
            mb = timed(lambda: A.line_back(yin, k, w), reps)
            sub = A.n_rays * k ** (g.dim - 1)
            rows.append({"k": k, "weight": w, "ms_forward": mf, "ms_adjoint": mb,
                         "sub_lines_per_s": sub / (mf / 1e3),
                         "voxel_views_per_s": A.n_vox * g.n_p / (mb / 1e3)})
            print("line k=%d %s: forward %.2f ms, adjoint %.2f ms" % (k, w, mf, mb), file=sys.stderr, flush=True)
    area = {"ms_forward": timed(lambda: A.forward(x, ws=ws), reps),
            "ms_adjoint": timed(lambda: A.back(yin, ws=ws), reps)}
    res = {"mode": "line-based vs exact", "config": {"workload": _describe(g)},
           "precision": args.precision, "line": rows, "exact": area}
    print(json.dumps(res), flush=True)


# -------------------------------------------------------------------- bench
def main():
    args = parse()
    if args.digest_stats:
        return digest_stats(args)
    if args.digest_valu:
        return digest_valu(args)
    if args.digest_counters:
        return digest_counters(args)
    if args.line:
        return line_bench(args)
    if args.stored:
        return stored_bench(args)
    if args.gpus != 1:
        print("bench.py runs on one GPU only (this library has no multi-GPU path); "
              "got --gpus %d" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import ctypes as C

    import numpy as np
    import torch

    from paper_2511_12235_amd import _lib
    from paper_2511_12235_amd import workloads as wl
    from paper_2511_12235_amd.projector import SystemMatrix

    g = _geometry(args.config)
    dev = torch.device("cuda:0")
    A = SystemMatrix(g, args.precision, device=dev)
    dt = A.dtype
    B = max(int(args.batch), 1)
    x = torch.from_numpy(wl.ellipse_phantom(g, 10, seed=2)).to(dev, dt)
    if B > 1:
        x = torch.stack([x] + [torch.from_numpy(wl.ellipse_phantom(g, 10, seed=2 + i)).to(dev, dt)
                               for i in range(1, B)])
    keep_s = None
    if args.keep_records:  # geometry-only tables, built once before the timed region
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        A.keep_records()
        keep_s = time.perf_counter() - t0
    ws = A.workspace(B)
    lead = (B,) if B > 1 else ()
    y = torch.empty(lead + A.sino_shape, dtype=dt, device=dev)
    xb = torch.empty(lead + A.vol_shape, dtype=dt, device=dev)

    # exact number of nonzero pairs (FP64 pattern), counted on the GPU
    nnz = C.c_int64(0)
    t0 = time.perf_counter()
    _lib.check(_lib.lib().sm_weights_csr(A._plan, _lib.SM_FP32, C.byref(nnz), None, None, None),
               "sm_weights_csr(count)")
    count_s = time.perf_counter() - t0
    nnz = nnz.value

    if args.copy_mib > 0:  # plain copy of known size: reference for the HBM counters
        n = args.copy_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    stream = torch.cuda.current_stream(dev)
    for _ in range(args.warmup):
        A.forward(x, out=y, ws=ws)
        A.back(y, out=xb, ws=ws)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True),
           torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    A.timing(True)
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
    kt = A.read_timing()
    A.timing(False)
    t_f = np.array([a.elapsed_time(b) for a, b, _ in ev]) / 1e3
    t_b = np.array([b.elapsed_time(c) for _, b, c in ev]) / 1e3
    step = t_f + t_b
    value = 2.0 * nnz * B / float(np.mean(step))
    eff_bw = value * 8.0 / 1e9  # GB/s a stored FP32+int32 CSR matrix would stream

    # dominant kernel: largest summed launch time in the timed region
    dom = max(("forward", "adjoint", "records", "prefix", "transpose"), key=lambda k: kt[k][1])
    launches, ms = kt[dom]
    ms_launch = ms / max(launches, 1)
    pairs_per_launch = nnz * B * args.steps / max(launches, 1) if dom in ("forward", "adjoint") else 0.0
    achieved = FLOP_PER_PAIR * pairs_per_launch / (ms_launch / 1e3) / 1e12 if ms_launch > 0 else 0.0
    symbol = (KERNEL_SYMBOL_2D if g.dim == 2 else KERNEL_SYMBOL)[dom]
    # the counter summaries were taken on single-volume launches
    traffic = traffic_per_launch(args.config, args.precision, symbol) if B == 1 and g.dim == 3 else None
    roofline = {"bound": "alu", "achieved": achieved, "peak": ALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / ALU_PEAK_TFLOPS, "traffic": traffic,
                "kernel": symbol, "ms_per_launch": ms_launch,
                "pairs_per_launch": pairs_per_launch, "flop_per_pair": FLOP_PER_PAIR}
    if g.dim == 2:  # the 23 flop per pair count is the 3D K evaluation's
        roofline = {"kernel": symbol, "ms_per_launch": ms_launch, "pairs_per_launch": pairs_per_launch}

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
        "config": {"workload": _describe(g) + ", forward + adjoint" + (", %d volumes per call" % B if B > 1 else ""),
                   "nnz_pairs": nnz, "ms_forward": float(np.mean(t_f)) * 1e3,
                   "ms_adjoint": float(np.mean(t_b)) * 1e3, "nnz_count_s": count_s,
                   "wall_s": wall,
                   "kernel_ms": {k: round(v[1] / args.steps, 3) for k, v in kt.items()},
                   "launch_shape": dict(zip(("views_per_chunk", "adjoint_runs"), A.launch_shape())),
                   "pct_hbm_roofline_effective": 100.0 * eff_bw / HBM_PEAK_GBS,
                   "records": ("kept in the plan: %.1f GB built once in %.2f s" % (A.record_bytes() / 1e9, keep_s)
                               if args.keep_records else "rebuilt in every call")},
        "roofline": roofline,
    }
    if not args.no_cpu_baseline and g.dim == 3:
        res["cpu_baseline"] = cpu_baseline(g, args.cpu_views)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
