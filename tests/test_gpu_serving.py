"""Continuous-batching server: every result in the mix equals the same
request served alone (bitwise: the kernels reduce in a fixed order and a
batched call returns the single-call results), admission never exceeds the
HBM budget, and requests do overlap and batch."""
import dataclasses

import pytest
import torch

from paper_2511_12235_amd import serve
from paper_2511_12235_amd import workloads as wl

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def tiny_geometry(name, n_p):
    if name == "2d":
        return wl.make_geometry(2, (48, 48), (1.0, 1.0), 60, 200.0, 200.0, (72,), (1.5,))
    if name == "3d32":
        return wl.make_geometry(3, (32, 32, 32), (1.0, 1.0, 1.0), n_p, 300.0, 300.0, (48, 48), (1.5, 1.5))
    if name == "3d48":
        return wl.make_geometry(3, (48, 48, 40), (1.0, 1.0, 1.0), n_p, 300.0, 300.0, (72, 64), (1.5, 1.5))
    raise ValueError(name)


MIX = (("2d", "forward", 1.0), ("2d", "cg", 1.0), ("3d32", "forward", 2.0), ("3d32", "cg", 1.0),
       ("3d48", "forward", 1.0), ("3d48", "cg", 1.0))


def test_results_equal_alone_and_in_the_mix():
    print("[case] serving mix", flush=True)
    reqs = serve.make_requests(48, 500.0, 3, torch.device(DEV), mix=MIX, iters=5,
                               geometry=tiny_geometry, views=(30, 60))
    # a burst of same-geometry requests waiting together at the first
    # admission, so that one batched launch is certain whatever the timing
    g = tiny_geometry("3d32", 30)
    ys = [torch.rand(g.sino_shape, generator=torch.Generator(device=DEV).manual_seed(40 + i),
                     device=DEV) for i in range(5)]
    reqs += [serve.Request(100 + i, "3d32/burst", g, "cg", ys[i], 0.0, iters=5) for i in range(5)]
    probe = serve.Server(DEV)
    probe.prepare(reqs)
    biggest = max(probe.footprint(r, 1) for r in reqs)
    budget = int(2.5 * biggest)
    srv = serve.Server(DEV, hbm_budget=budget, slots=4, keep_results=True)
    srv.plans = probe.plans
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated(DEV)
    torch.cuda.reset_peak_memory_stats(DEV)
    srv.run(reqs)
    torch.cuda.synchronize()
    # device memory the run allocated beyond what it keeps (the results and
    # the CG histories of finished launches) stays within the admission budget
    peak = torch.cuda.max_memory_allocated(DEV) - base
    kept = sum(r.result.numel() * r.result.element_size() for r in reqs) + 8 * sum(
        (r.iters + 1) for r in reqs if r.kind == "cg")
    print("[serve] peak allocation %d bytes, budget %d, kept %d" % (peak, budget, kept), flush=True)
    assert peak <= budget + kept + (4 << 20)
    alone = [dataclasses.replace(r, result=None) for r in reqs]
    srv.run_sequential(alone)
    for a, b in zip(reqs, alone):
        assert a.result.shape == b.result.shape
        assert torch.equal(a.result, b.result), (a.rid, a.key, a.kind)
    st = srv.stats
    print("[serve] stats", st, serve.summarize(reqs), serve.summarize(alone), flush=True)
    assert st["max_in_flight_bytes"] <= budget
    assert st["max_concurrent"] >= 2
    assert st["batched"] >= 1
    assert all(r.t_done >= r.arrival for r in reqs)


def test_kept_records_change_no_result():
    """Plans that keep their strip records (record budget) serve the same bits."""
    print("[case] serving kept records", flush=True)
    reqs = serve.make_requests(16, 500.0, 5, torch.device(DEV), mix=MIX, iters=4,
                               geometry=tiny_geometry, views=(30, 60))
    plain = serve.Server(DEV, keep_results=True)
    plain.prepare(reqs)
    plain.run_sequential(reqs)
    kept = serve.Server(DEV, keep_results=True, record_budget=1 << 34)
    again = [dataclasses.replace(r, result=None) for r in reqs]
    kept.prepare(again)
    kept.run(again)
    assert kept.record_used > 0
    assert kept.record_used == sum(A.record_bytes() for A in kept.plans.values())
    for a, b in zip(reqs, again):
        assert torch.equal(a.result, b.result), (a.rid, a.key, a.kind)
