"""Continuous-batching server for projection and reconstruction requests.

A request is (geometry, kind, input): kind "forward" projects a volume,
kind "cg" runs CGLS for a fixed number of iterations on a sinogram.  Inputs
are resident on the device when a request arrives.  The server

* keeps one plan per geometry (plans are immutable and shared by streams);
  with a record budget, a new plan also keeps its strip records on the
  device (sm_plan_keep_records) while the budget lasts, so that its calls
  skip rebuilding them and its workspace shrinks by them;
* owns a few HIP streams ("slots"); a waiting request is admitted as soon
  as a slot is free and its device footprint fits the HBM budget next to the
  requests already running (first come, first served);
* batches: requests waiting with the same geometry, kind and iteration count
  are admitted together (up to `max_batch`) and run as one batched call,
  which evaluates every weight once for all of them;
* enqueues the whole request (sm_forward, or sm_cgls with its scalars on the
  device) on its slot's stream without waiting, so requests on different
  slots overlap on the GPU, and retires them by polling completion events.

Results do not depend on what else runs: the library's kernels reduce in a
fixed order and a batched call returns bitwise the single-call results.

`run_sequential` is the baseline: one request at a time, in arrival order, on
one stream.  Both report per-request latency (arrival to observed
completion), p50/p99 and throughput.
"""
from __future__ import annotations

import dataclasses
import math
import time
import zlib
from typing import Dict, List, Optional, Sequence

import numpy as np
import torch

from . import _lib
from .projector import SystemMatrix


@dataclasses.dataclass
class Request:
    rid: int
    key: str                 # geometry name (plans are cached by it)
    geometry: object
    kind: str                # "forward" or "cg"
    data: torch.Tensor       # device input: volume (forward) or sinogram (cg)
    arrival: float           # seconds after the start of the run
    iters: int = 10
    lam: float = 0.0
    result: Optional[torch.Tensor] = None
    t_admit: float = math.nan
    t_done: float = math.nan


@dataclasses.dataclass
class _Launch:
    reqs: List[Request]
    slot: int
    footprint: int
    done: torch.cuda.Event
    keep: list


def percentile(v: Sequence[float], q: float) -> float:
    return float(np.percentile(np.asarray(v, dtype=np.float64), q)) if len(v) else math.nan


class Server:
    def __init__(self, device=None, hbm_budget: int = 2 << 30, slots: int = 4, max_batch: int = 8,
                 precision: str = "fp32", keep_results: bool = False, record_budget: int = 0):
        self.device = torch.device(device or "cuda:0")
        self.budget = int(hbm_budget)
        self.record_budget = int(record_budget)  # HBM for kept records, outside the request budget
        self.record_used = 0
        self.max_batch = int(max_batch)
        self.precision = precision
        self.keep_results = keep_results
        self.streams = [torch.cuda.Stream(self.device) for _ in range(slots)]
        self.plans: Dict[str, SystemMatrix] = {}
        self.stats = {"max_in_flight_bytes": 0, "max_concurrent": 0, "launches": 0, "batched": 0}

    # ------------------------------------------------------------------ plans
    def plan(self, key: str, geometry) -> SystemMatrix:
        if key not in self.plans:
            A = SystemMatrix(geometry, self.precision, device=self.device)
            nb = A.record_bytes()
            if 0 < nb <= self.record_budget - self.record_used:
                A.keep_records(nb)
                self.record_used += nb
            self.plans[key] = A
        return self.plans[key]

    def footprint(self, r: Request, batch: int) -> int:
        """Device bytes a launch of `batch` such requests holds while it runs:
        outputs, the library workspace and, for batch > 1, the stacked copy of
        the inputs (each input itself is already resident)."""
        A = self.plan(r.key, r.geometry)
        es = 8 if self.precision == "fp64" else 4
        if r.kind == "forward":
            stacked = batch * A.n_vox * es if batch > 1 else 0
            return A.workspace_bytes(batch) + batch * A.n_rays * es + stacked
        n = C_int64()
        _lib.check(_lib.lib().sm_solver_workspace_size(A._plan, _lib.SM_SOLVER_CGLS, batch, n.ref()),
                   "sm_solver_workspace_size")
        stacked = batch * A.n_rays * es if batch > 1 else 0
        return n.value + batch * (A.n_vox * es + (r.iters + 1) * 8) + stacked

    # ---------------------------------------------------------------- launch
    def _launch(self, reqs: List[Request], slot: int, footprint: int, now: float) -> _Launch:
        r0 = reqs[0]
        A = self.plan(r0.key, r0.geometry)
        B = len(reqs)
        st = self.streams[slot]
        st.wait_stream(torch.cuda.current_stream(self.device))  # inputs were made there
        keep = []
        with torch.cuda.stream(st):
            x = reqs[0].data.unsqueeze(0) if B == 1 else torch.stack([r.data for r in reqs])
            if r0.kind == "forward":
                out = A.forward(x.contiguous())
            else:
                out, hist = A.cgls(x.contiguous(), r0.iters, lam=r0.lam)
                keep.append(hist)
            keep += [x, out]
            ev = torch.cuda.Event()
            ev.record(st)
        for i, r in enumerate(reqs):
            r.t_admit = now
            r.result = out[i]
        self.stats["launches"] += 1
        self.stats["batched"] += B > 1
        return _Launch(reqs, slot, footprint, ev, keep)

    def prepare(self, requests: List[Request]):
        """Create the plans and run every distinct request type once (untimed),
        so that neither plan creation nor first-call costs enter latencies."""
        seen = set()
        for r in requests:
            k = (r.key, r.kind, r.iters)
            if k in seen:
                continue
            seen.add(k)
            A = self.plan(r.key, r.geometry)
            if r.kind == "forward":
                A.forward(r.data)
            else:
                A.cgls(r.data, r.iters, lam=r.lam)
        torch.cuda.synchronize(self.device)

    # ------------------------------------------------------------------- run
    def run(self, requests: List[Request], progress: int = 0) -> List[Request]:
        """Serve `requests` (sorted by arrival) in real time; with progress > 0
        print a line every `progress` completed requests."""
        pending = sorted(requests, key=lambda r: r.arrival)
        waiting: List[Request] = []
        active: List[_Launch] = []
        free = list(range(len(self.streams)))
        used = 0
        i = 0
        done = 0
        torch.cuda.synchronize(self.device)
        t0 = time.perf_counter()
        while i < len(pending) or waiting or active:
            now = time.perf_counter() - t0
            while i < len(pending) and pending[i].arrival <= now:
                waiting.append(pending[i])
                i += 1
            progressed = False
            # retire finished launches
            for L in list(active):
                if L.done.query():
                    for r in L.reqs:
                        r.t_done = now
                        if not self.keep_results:
                            r.result = None
                        done += 1
                        if progress and done % progress == 0:
                            print("[serve] %d/%d done at %.1f s" % (done, len(pending), now), flush=True)
                    active.remove(L)
                    free.append(L.slot)
                    used -= L.footprint
                    progressed = True
            # admit in arrival order while a slot and memory are free
            while waiting and free:
                head = waiting[0]
                group = [r for r in waiting if r.key == head.key and r.kind == head.kind
                         and r.iters == head.iters][: self.max_batch]
                fp = self.footprint(head, len(group))
                while len(group) > 1 and used + fp > self.budget:
                    group = group[:-1]
                    fp = self.footprint(head, len(group))
                if used + fp > self.budget and active:
                    break  # wait for memory to free up
                for r in group:
                    waiting.remove(r)
                slot = free.pop(0)
                active.append(self._launch(group, slot, fp, now))
                used += fp
                self.stats["max_in_flight_bytes"] = max(self.stats["max_in_flight_bytes"], used)
                self.stats["max_concurrent"] = max(self.stats["max_concurrent"], len(active))
                progressed = True
            if not progressed:
                if i < len(pending) and not waiting and not active:
                    time.sleep(max(0.0, min(pending[i].arrival - now, 0.002)))
                else:
                    time.sleep(0.0002)
        return requests

    def run_sequential(self, requests: List[Request], progress: int = 0) -> List[Request]:
        """Baseline: one request at a time in arrival order on one stream."""
        st = self.streams[0]
        torch.cuda.synchronize(self.device)
        t0 = time.perf_counter()
        for n, r in enumerate(sorted(requests, key=lambda q: q.arrival)):
            if progress and n and n % progress == 0:
                print("[sequential] %d/%d done at %.1f s" % (n, len(requests), time.perf_counter() - t0),
                      flush=True)
            now = time.perf_counter() - t0
            if r.arrival > now:
                time.sleep(r.arrival - now)
            r.t_admit = time.perf_counter() - t0
            A = self.plan(r.key, r.geometry)
            st.wait_stream(torch.cuda.current_stream(self.device))
            with torch.cuda.stream(st):
                if r.kind == "forward":
                    out = A.forward(r.data)
                else:
                    out, _ = A.cgls(r.data, r.iters, lam=r.lam)
            st.synchronize()
            r.t_done = time.perf_counter() - t0
            r.result = out if self.keep_results else None
        return requests


class C_int64:
    """Small helper: an int64 output argument for the ctypes calls."""

    def __init__(self):
        import ctypes
        self._v = ctypes.c_int64(0)

    def ref(self):
        import ctypes
        return ctypes.byref(self._v)

    @property
    def value(self) -> int:
        return int(self._v.value)


def summarize(requests: List[Request]) -> dict:
    lat = [r.t_done - r.arrival for r in requests]
    span = max(r.t_done for r in requests) - min(r.arrival for r in requests)
    return {"requests": len(requests), "p50_s": percentile(lat, 50), "p99_s": percentile(lat, 99),
            "mean_s": float(np.mean(lat)), "throughput_rps": len(requests) / span, "makespan_s": span}


# ------------------------------------------------------------------ workload
# (geometry name, kind, weight).  The weights were set from measured service
# times of one request alone on an MI355X (FP32, mean over 90/180/360 views):
# 2D 256^2 forward 0.4 ms / CG-10 11 ms; 64^3 1.6 ms / 42 ms; 128^3 8.7 ms /
# 208 ms; 256^3 73 ms / 1.37 s.  With these weights the mean service time is
# about 38 ms, an offered load of 0.75 for the sequential baseline at 20
# requests/s.
MIX = (
    ("2d256", "forward", 0.22), ("2d256", "cg", 0.18),
    ("3d64", "forward", 0.22), ("3d64", "cg", 0.15),
    ("3d128", "forward", 0.12), ("3d128", "cg", 0.05),
    ("3d256", "forward", 0.05), ("3d256", "cg", 0.01),
)


def make_requests(n: int, rate: float, seed: int, device, mix=MIX, iters: int = 10,
                  precision: str = "fp32", geometry=None, views=(90, 180, 360)) -> List[Request]:
    """Poisson arrivals at `rate` per second of requests drawn from `mix`;
    3D requests draw their view count from `views`.  `geometry(name, n_p)`
    builds a request geometry (default: the serving geometries of
    workloads.py).  Inputs are seeded uniform random volumes / sinograms
    generated on the device, one per (geometry, kind), shared read-only by
    the requests that use it."""
    from . import workloads as wl
    geometry = geometry or wl.serving_geometry
    rng = np.random.default_rng(seed)
    names = [m[0] for m in mix]
    kinds_ = [m[1] for m in mix]
    w = np.array([m[2] for m in mix], dtype=np.float64)
    w /= w.sum()
    t = 0.0
    dt = torch.float64 if precision == "fp64" else torch.float32
    inputs: Dict[tuple, torch.Tensor] = {}
    geoms: Dict[str, object] = {}
    out = []
    gen = torch.Generator(device=device)
    for rid in range(n):
        t += rng.exponential(1.0 / rate)
        j = int(rng.choice(len(mix), p=w))
        name, kind = names[j], kinds_[j]
        n_p = 360 if name.startswith("2d") else int(rng.choice(list(views)))
        key = "%s/%d" % (name, n_p)
        if key not in geoms:
            geoms[key] = geometry(name, n_p)
        g = geoms[key]
        if (key, kind) not in inputs:
            gen.manual_seed(zlib.crc32(("%s|%s|%d" % (key, kind, seed)).encode()))
            shape = g.vol_shape if kind == "forward" else g.sino_shape
            inputs[(key, kind)] = torch.rand(shape, generator=gen, device=device, dtype=dt)
        out.append(Request(rid, key, g, kind, inputs[(key, kind)], t, iters=iters))
    return out


def service_times(device, mix=MIX, views=(90, 180, 360), iters: int = 10, precision: str = "fp32",
                  record_budget: int = 0) -> dict:
    """Time one request of every (geometry, kind, views) type alone (after a
    warm-up call): the per-type service times the mix weights are set from."""
    from . import workloads as wl
    srv = Server(device, precision=precision, record_budget=record_budget)
    out = {}
    for name, kind, _ in mix:
        for n_p in ((360,) if name.startswith("2d") else views):
            g = wl.serving_geometry(name, n_p)
            key = "%s/%d" % (name, n_p)
            A = srv.plan(key, g)
            shape = g.vol_shape if kind == "forward" else g.sino_shape
            dt = torch.float64 if precision == "fp64" else torch.float32
            x = torch.rand(shape, device=srv.device, dtype=dt)
            run = (lambda: A.forward(x)) if kind == "forward" else (lambda: A.cgls(x, iters))
            run()
            torch.cuda.synchronize(srv.device)
            t = time.perf_counter()
            run()
            torch.cuda.synchronize(srv.device)
            out["%s/%s" % (key, kind)] = time.perf_counter() - t
            del x
    return out


def offered_load(times: dict, rate: float, mix=MIX, views=(90, 180, 360)) -> float:
    """Mean service time of the mix times the arrival rate (sequential load)."""
    w = np.array([m[2] for m in mix], dtype=np.float64)
    w /= w.sum()
    mean = 0.0
    for (name, kind, _), wi in zip(mix, w):
        vs = (360,) if name.startswith("2d") else views
        mean += wi * np.mean([times["%s/%d/%s" % (name, v, kind)] for v in vs])
    return mean * rate


def main(argv=None):
    import argparse
    import json
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--requests", type=int, default=1000)
    ap.add_argument("--rate", type=float, default=20.0)
    ap.add_argument("--budget-gib", type=float, default=2.0)
    ap.add_argument("--slots", type=int, default=4)
    ap.add_argument("--record-budget-gib", type=float, default=0.0,
                    help="HBM for strip records kept in the plans (outside the request budget)")
    ap.add_argument("--seed", type=int, default=7)
    ap.add_argument("--service-times", action="store_true")
    args = ap.parse_args(argv)
    dev = torch.device("cuda:0")
    rb = int(args.record_budget_gib * (1 << 30))
    if args.service_times:
        t = service_times(dev, record_budget=rb)
        print(json.dumps({"service_s": t, "offered_load_at_rate": offered_load(t, args.rate),
                          "rate": args.rate}), flush=True)
        return
    res = {"rate": args.rate, "budget_gib": args.budget_gib, "slots": args.slots,
           "record_budget_gib": args.record_budget_gib, "mix": [list(m) for m in MIX]}
    srv = Server(dev, hbm_budget=int(args.budget_gib * (1 << 30)), slots=args.slots, record_budget=rb)
    reqs = make_requests(args.requests, args.rate, args.seed, dev)
    srv.prepare(reqs)
    srv.run(reqs, progress=100)
    res["continuous"] = summarize(reqs)
    res["stats"] = dict(srv.stats)
    res["stats"]["records_kept_bytes"] = srv.record_used
    seq = make_requests(args.requests, args.rate, args.seed, dev)
    srv.run_sequential(seq, progress=100)
    res["sequential"] = summarize(seq)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
