"""Serving loop: scheduling logic on the CPU with a fake executor (simulated clock); on the GPU,
every request's result is bitwise the same in the concurrent mix as in one me_sigma call over the
whole request, and the server's device memory stays within its budget."""
import numpy as np
import pytest

from paper_2210_11122_amd import serve

COST = {"a": 1e-6, "b": 4e-6, "L": 2e-5}
BPE = {"a": 1000, "b": 4000, "L": 2000}


def fake(fail=None, item=None, n_large=1):
    return serve.FakeExecutor(COST, BPE, item_events=item or {"L": 256}, large=("L",), n_large_slots=n_large,
                              fail=fail)


def test_split_items():
    assert serve.split_items(100, 4096) == [(0, 100)]
    assert serve.split_items(4097, 4096) == [(0, 2112), (2112, 1985)]
    assert serve.split_items(3 * 4096, 4096) == [(0, 4096), (4096, 4096), (8192, 4096)]
    for n in (1, 63, 64, 65, 8191, 12345):
        it = serve.split_items(n, 4096)
        assert sum(k for _, k in it) == n and all(k <= 4096 for _, k in it)
        assert all(a == sum(k for _, k in it[:i]) for i, (a, _) in enumerate(it))


def test_arena_first_fit_and_coalescing():
    a = serve.Arena(10 * 256)
    x = [a.alloc(256) for _ in range(10)]
    assert x == [256 * i for i in range(10)] and a.alloc(1) is None
    for i in (1, 2, 3):
        a.release(x[i], 256)
    assert a.alloc(3 * 256) == 256          # three neighbours coalesced
    a.release(256, 3 * 256)
    for i in (0, 4, 5, 6, 7, 8, 9):
        a.release(x[i], 256)
    assert a.free == [(0, 10 * 256)] and a.used == 0


def test_all_requests_complete_and_admission_in_arrival_order():
    reqs = serve.poisson_requests(200, 2000.0, ["a", "b"], size_range=(10, 1000), seed=3)
    sch = serve.Scheduler(fake(), n_slots=3, arena_bytes=10_000_000)
    done = sch.run(reqs)
    assert sorted(c.req.rid for c in done) == list(range(200))
    assert all(c.ok for c in done)
    admits = sorted(done, key=lambda c: (c.t_admit, c.req.rid))
    assert [c.req.rid for c in admits] == sorted(c.req.rid for c in admits)
    for c in done:
        assert c.req.arrival <= c.t_admit <= c.t_start <= c.t_done


def test_items_cover_every_event_once():
    """requests cut into items on several slots: every event written once, by the right request"""
    reqs = [r._replace(arrival=0.0) for r in serve.poisson_requests(30, 1.0, ["a", "L"], (10, 1500), seed=4)]
    done = serve.Scheduler(fake(n_large=2), n_slots=4, arena_bytes=10**9).run(reqs, keep_results=True)
    assert all(c.ok for c in done)
    for c in done:
        assert np.array_equal(c.result, c.req.rid * 1e6 + np.arange(c.req.n_evt))


def test_slots_and_arena_never_exceeded_and_work_overlaps():
    ex = fake(n_large=2)
    budget = 3_000_000
    sch = serve.Scheduler(ex, n_slots=4, arena_bytes=budget)
    orig = sch._dispatch

    def dispatch():
        orig()
        assert len(sch.running) <= 4
        assert sch.arena.used <= budget

    sch._dispatch = dispatch
    reqs = [r._replace(arrival=0.0) for r in serve.poisson_requests(50, 1.0, ["a", "b", "L"], (100, 600), seed=5)]
    done = sch.run(reqs)
    assert all(c.ok for c in done)
    assert sch.max_busy_slots > 1 and sch.max_in_flight > 1   # requests overlap on the device
    assert sch.arena.used == 0 and sch.arena.free == [(0, budget)]


def test_large_process_runs_on_its_slots_only():
    ex = fake(n_large=2)
    reqs = [r._replace(arrival=0.0) for r in serve.poisson_requests(40, 1.0, ["a", "L"], (100, 2000), seed=6)]
    serve.Scheduler(ex, n_slots=4, arena_bytes=10**9).run(reqs)
    assert {s for p, s in ex.slot_log if p == "L"} <= {0, 1}
    assert {s for p, s in ex.slot_log if p == "a"} & {2, 3}


def test_admission_waits_for_memory():
    """a large head request waits until enough memory is released; nothing overtakes it"""
    reqs = [serve.Request(0, "b", 500, 0, 0.0), serve.Request(1, "b", 500, 0, 0.0),
            serve.Request(2, "a", 10, 0, 0.0)]
    sch = serve.Scheduler(fake(), n_slots=4, arena_bytes=2_500_000)
    done = {c.req.rid: c for c in sch.run(reqs)}
    assert done[1].t_admit >= done[0].t_done       # waited for request 0's memory
    assert done[2].t_admit >= done[1].t_admit      # arrival order: no overtaking at admission
    assert sch.waited_for_memory == 1 and done[1].waited_for_memory


def test_small_requests_overtake_a_large_one():
    """a large request that arrived first runs item by item; small requests arriving while it
    runs take the free slots first and finish long before it"""
    reqs = [serve.Request(0, "L", 8 * 256, 0, 0.0)] + \
        [serve.Request(i, "a", 100, 0, 1e-4 * i) for i in range(1, 20)]
    done = {c.req.rid: c for c in serve.Scheduler(fake(), n_slots=2, arena_bytes=10**9, aging=1.0).run(reqs)}
    assert all(c.ok for c in done.values())
    for i in range(1, 20):
        assert done[i].t_done - done[i].req.arrival < 3 * COST["L"] * 256   # at most an item's wait
    assert done[0].t_done > max(done[i].t_done for i in range(1, 20))


def test_aging_lets_a_large_request_through_a_stream_of_small_ones():
    """small requests saturate both slots for a long time; the large one still completes, about
    its own work after arrival plus what aging lets small requests take first"""
    reqs = [serve.Request(0, "L", 4 * 256, 0, 0.0)] + \
        [serve.Request(i, "a", 1000, 0, 5e-4 * (i - 1)) for i in range(1, 2000)]
    done = {c.req.rid: c for c in serve.Scheduler(fake(), n_slots=2, arena_bytes=10**9, aging=1.0).run(reqs)}
    big = done[0]
    last_small = max(c.t_done for c in done.values() if c.req.rid > 0)
    assert big.ok and big.t_done < 0.25 * last_small
    assert big.t_done - big.req.arrival < 3 * COST["L"] * 4 * 256


def test_oversize_request_fails_alone():
    reqs = [serve.Request(0, "a", 100, 0, 0.0), serve.Request(1, "b", 10**6, 0, 0.0),
            serve.Request(2, "a", 100, 0, 0.0)]
    done = {c.req.rid: c for c in serve.Scheduler(fake(), 2, 1_000_000).run(reqs)}
    assert done[0].ok and done[2].ok
    assert not done[1].ok and "exceeds" in done[1].error


def test_failed_launch_frees_its_slot_and_memory():
    reqs = [serve.Request(i, "a", 100, 0, 0.0) for i in range(6)]
    sch = serve.Scheduler(fake(fail={2, 3}), 1, 10**9)
    done = {c.req.rid: c for c in sch.run(reqs)}
    assert [done[i].ok for i in range(6)] == [True, True, False, False, True, True]
    assert "injected" in done[2].error
    assert sch.arena.used == 0 and not sch.running


def test_latency_statistics():
    reqs = serve.poisson_requests(100, 100.0, ["a"], (100, 100), seed=9)
    done = serve.Scheduler(fake(), 2, 10**9).run(reqs)
    st = serve.latency_stats(done)
    # each request takes exactly 1e-4 s and the load is light: latency = service time
    assert st["n"] == 100 and abs(st["p50_ms"] - 0.1) < 1e-9 and st["p99_ms"] >= st["p50_ms"]
    assert set(serve.latency_by_process(done)) == {"a"}


@pytest.mark.gpu
@pytest.mark.parametrize("precision", ["fp64", "mixed_fp16"])
def test_alone_equals_mix_bitwise(precision):
    """the four QCD processes in the concurrent mix (gg_ttggg requests of one to three chunks,
    cut into chunk-sized items) against one me_sigma call per request (gg_ttggg requests of
    several chunks then run on the library's two internal streams): bitwise equal; the server's
    device memory stays within its budget"""
    import torch
    procs = ["gg_tt", "gg_ttg", "gg_ttgg", "gg_ttggg"]
    print(f"case serving mix {precision}", flush=True)
    budget = 24 << 30
    ex = serve.GpuExecutor(procs, n_slots=4, precision=precision, hbm_budget=budget, n_large_slots=1)
    chunk = ex.handles["gg_ttggg"].info["chunk_events"]
    reqs = serve.poisson_requests(24, 1e6, procs, size_range=(256, 65536), seed=11)
    big = iter([chunk + 1, 300, 2 * chunk + 5, 3 * chunk, 4096])
    reqs = [r._replace(n_evt=next(big, 500)) if r.process == "gg_ttggg" else r for r in reqs]
    assert sum(r.process == "gg_ttggg" and r.n_evt > chunk for r in reqs) >= 2
    mix = serve.Scheduler(ex, 4, ex.arena_bytes).run([r._replace(arrival=0.0) for r in reqs], keep_results=True)
    torch.cuda.synchronize()
    mem = ex.memory_report()
    print(f"serving mix {precision}: scratch {mem['reserved_scratch_bytes'] / 2**30:.2f} GiB, arena "
          f"{mem['request_arena_bytes'] / 2**30:.2f} GiB, device peak {mem['device_used_peak_bytes'] / 2**30:.2f} GiB "
          f"of {budget / 2**30:.0f} GiB", flush=True)
    assert mem["device_used_peak_bytes"] <= budget
    alone = serve.run_alone(ex, reqs)
    assert len(mix) == 24 and all(c.ok for c in mix)
    for c in mix:
        assert np.array_equal(c.result, alone[c.req.rid]), (c.req, np.max(np.abs(c.result / alone[c.req.rid] - 1)))
