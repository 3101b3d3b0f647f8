"""Serving loop: scheduling logic on the CPU with a fake executor; on the GPU, results of
every request are bitwise the same alone and in the concurrent mix."""
import numpy as np
import pytest

from paper_2210_11122_amd import serve

COST = {"a": 1e-6, "b": 4e-6}
BPE = {"a": 1000, "b": 4000}


def fake(fail=None):
    return serve.FakeExecutor(COST, BPE, fail=fail)


def test_all_requests_complete_in_fifo_admission_order():
    reqs = serve.poisson_requests(200, 2000.0, ["a", "b"], size_range=(10, 1000), seed=3)
    sch = serve.Scheduler(fake(), n_slots=3, hbm_budget=10_000_000)
    done = sch.run(reqs)
    assert sorted(c.req.rid for c in done) == list(range(200))
    assert all(c.ok for c in done)
    admits = sorted(done, key=lambda c: (c.t_admit, c.req.rid))
    assert [c.req.rid for c in admits] == sorted(c.req.rid for c in admits)
    for c in done:
        assert c.t_admit >= c.req.arrival and c.t_done >= c.t_admit


def test_slots_and_budget_never_exceeded_and_work_overlaps():
    class Watch(serve.FakeExecutor):
        def __init__(self, *a, **k):
            super().__init__(*a, **k)
            self.active, self.peak = {}, 0

    ex = Watch(COST, BPE)
    budget = 3_000_000
    sch = serve.Scheduler(ex, n_slots=4, hbm_budget=budget)
    orig_admit = sch._admit

    def admit():
        orig_admit()
        assert len(sch.running) <= 4
        assert sch.used <= budget

    sch._admit = admit
    reqs = [r._replace(arrival=0.0) for r in serve.poisson_requests(50, 1.0, ["a", "b"], (100, 600), seed=5)]
    done = sch.run(reqs)
    assert all(c.ok for c in done)
    assert sch.max_in_flight > 1   # requests overlap on the device


def test_admission_waits_for_memory():
    """a large head request waits until enough memory is released; nothing overtakes it"""
    reqs = [serve.Request(0, "b", 500, 0, 0.0), serve.Request(1, "b", 500, 0, 0.0),
            serve.Request(2, "a", 10, 0, 0.0)]
    sch = serve.Scheduler(fake(), n_slots=4, hbm_budget=2_500_000)
    done = {c.req.rid: c for c in sch.run(reqs)}
    assert done[1].t_admit >= done[0].t_done       # waited for request 0's memory
    assert done[2].t_admit >= done[1].t_admit      # FIFO: no overtaking


def test_oversize_request_fails_alone():
    reqs = [serve.Request(0, "a", 100, 0, 0.0), serve.Request(1, "b", 10**6, 0, 0.0),
            serve.Request(2, "a", 100, 0, 0.0)]
    done = {c.req.rid: c for c in serve.Scheduler(fake(), 2, 1_000_000).run(reqs)}
    assert done[0].ok and done[2].ok
    assert not done[1].ok and "exceeds" in done[1].error


def test_failed_launch_frees_its_slot():
    reqs = [serve.Request(i, "a", 100, 0, 0.0) for i in range(6)]
    done = {c.req.rid: c for c in serve.Scheduler(fake(fail={2, 3}), 1, 10**9).run(reqs)}
    assert [done[i].ok for i in range(6)] == [True, True, False, False, True, True]
    assert "injected" in done[2].error


def test_latency_statistics():
    reqs = serve.poisson_requests(100, 100.0, ["a"], (100, 100), seed=9)
    done = serve.Scheduler(fake(), 2, 10**9).run(reqs)
    st = serve.latency_stats(done)
    # each request takes exactly 1e-4 s and the load is light: latency = service time
    assert st["n"] == 100 and abs(st["p50_ms"] - 0.1) < 1e-9 and st["p99_ms"] >= st["p50_ms"]


@pytest.mark.gpu
def test_alone_equals_mix_bitwise():
    import torch
    procs = ["gg_tt", "gg_ttg", "gg_ttgg"]
    ex = serve.GpuExecutor(procs, n_slots=4)
    reqs = serve.poisson_requests(24, 1e6, procs, size_range=(256, 4096), seed=11)
    alone = {k: v.cpu().numpy() for k, v in serve.run_alone(ex, reqs).items()}
    mix = serve.Scheduler(ex, 4, 8 << 30).run([r._replace(arrival=0.0) for r in reqs], keep_results=True)
    torch.cuda.synchronize()
    assert len(mix) == 24 and all(c.ok for c in mix)
    for c in mix:
        assert np.array_equal(c.result.cpu().numpy(), alone[c.req.rid]), c.req
