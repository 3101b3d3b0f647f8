"""Serving loop: matrix-element requests of mixed processes and sizes, admitted continuously and
run concurrently on HIP streams.

Requests arrive as an MC integrator's channels issue them (here: a Poisson process).  The server
keeps one library handle per process resident (colour matrices, helicity masks and couplings on
the device) and S slots, each a HIP stream.  Its device memory is fixed when it starts, so that
a budget bounds what it holds:
  * the library's scratch for every (process, slot) pair, reserved at start (me_reserve_scratch),
    and what the runtime allocates for the kernels' first launches, measured at start;
  * one request arena, the rest of the budget, from which each admitted request takes the bytes
    of its momenta and output (first fit).
A request is admitted, in arrival order, as soon as its footprint fits in the arena.  An admitted
request is cut into work items of at most one chunk of events (gg_ttggg: the library's 4096-event
chunk; the other processes: the whole request).  Whenever a slot is free it takes the next item
of the admitted request with the least remaining work, less `aging` times the time the request
has waited, so small requests overtake large ones while no request waits for ever.  Items of the
processes with the largest scratch (gg_ttggg) may run on the first `n_large_slots` slots only,
which bounds the scratch reserved for them.  Each item makes its events with the library's RAMBO
(counter-based, so an item's events are those of the whole request) and evaluates them with one
me_sigma call: every event's result is bitwise that of one me_sigma call over the whole request.
Completion is polled through HIP events; latency = completion - arrival on the host monotonic
clock.

The scheduling logic is independent of the executor: ``GpuExecutor`` runs the library on the GPU,
``FakeExecutor`` (tests on the CPU) completes an item after a time proportional to its cost, so
admission, priorities, slot limits and failure handling are checked without a GPU.
"""
import collections
import time

import numpy as np

Request = collections.namedtuple("Request", "rid process n_evt seed arrival")


def poisson_requests(n, rate_hz, processes, size_range=(256, 65536), seed=1, t0=0.0):
    """n requests: exponential inter-arrival times (rate_hz), uniform process, batch size
    uniform integer in size_range, per-request RAMBO seed."""
    rng = np.random.default_rng(seed)
    t = t0
    out = []
    for i in range(n):
        t += rng.exponential(1.0 / rate_hz)
        proc = processes[int(rng.integers(len(processes)))]
        size = int(rng.integers(size_range[0], size_range[1] + 1))
        out.append(Request(i, proc, size, 1000 + i, t))
    return out


def split_items(n, item):
    """[(evt0, n_i)]: n events in equal pieces of at most `item` (multiples of 64 but the last)"""
    k = -(-n // item)
    step = -(-(-(-n // k)) // 64) * 64
    return [(a, min(step, n - a)) for a in range(0, n, step)]


class Arena:
    """First-fit allocation of byte ranges in one buffer, offsets aligned to `align`."""

    def __init__(self, size, align=256):
        self.size, self.align = size, align
        self.free = [(0, size)]   # sorted, coalesced (offset, length)
        self.used = 0

    def _round(self, n):
        return -(-n // self.align) * self.align

    def alloc(self, n):
        n = self._round(n)
        for i, (o, ln) in enumerate(self.free):
            if ln >= n:
                if ln == n:
                    del self.free[i]
                else:
                    self.free[i] = (o + n, ln - n)
                self.used += n
                return o
        return None

    def release(self, off, n):
        n = self._round(n)
        self.used -= n
        fr = self.free
        i = 0
        while i < len(fr) and fr[i][0] < off:
            i += 1
        fr.insert(i, (off, n))
        if i + 1 < len(fr) and fr[i][0] + fr[i][1] == fr[i + 1][0]:
            fr[i] = (fr[i][0], fr[i][1] + fr[i + 1][1])
            del fr[i + 1]
        if i > 0 and fr[i - 1][0] + fr[i - 1][1] == fr[i][0]:
            fr[i - 1] = (fr[i - 1][0], fr[i - 1][1] + fr[i][1])
            del fr[i]


class Completed:
    __slots__ = ("req", "t_admit", "t_start", "t_done", "ok", "error", "result", "waited_for_memory")

    def __init__(self, req):
        self.req = req
        self.t_admit = self.t_start = self.t_done = None
        self.ok, self.error, self.result, self.waited_for_memory = None, None, None, False


class _Job:
    __slots__ = ("c", "off", "fp", "items", "running", "cost_left", "binding")


class Scheduler:
    """Admission (arena), priorities and completion bookkeeping over an executor with `n_slots`
    slots and a request arena of `arena_bytes`."""

    def __init__(self, executor, n_slots, arena_bytes, aging=1.0):
        self.ex = executor
        self.n_slots = n_slots
        self.arena = Arena(arena_bytes)
        self.aging = aging
        self.free_slots = set(range(n_slots))
        self.waiting = collections.deque()
        self.jobs = []           # admitted, not yet complete
        self.running = {}        # slot -> (token, job, n_evt)
        self.done = []
        self.max_in_flight = 0   # admitted requests at once
        self.max_busy_slots = 0
        self.waited_for_memory = 0

    def submit(self, req):
        c = Completed(req)
        fp = self.ex.footprint(req)
        if fp > self.arena.size:
            c.ok, c.t_done = False, self.ex.now()
            c.error = f"footprint {fp} B exceeds the request arena of {self.arena.size} B"
            self.done.append(c)
            return
        self.waiting.append(c)

    def _admit(self):
        while self.waiting:
            c = self.waiting[0]
            fp = self.ex.footprint(c.req)
            off = self.arena.alloc(fp)
            if off is None:
                if not c.waited_for_memory:
                    c.waited_for_memory = True
                    self.waited_for_memory += 1
                break   # arrival order: the head waits for memory; later requests do not overtake it
            self.waiting.popleft()
            j = _Job()
            j.c, j.off, j.fp, j.running = c, off, fp, 0
            j.items = collections.deque(self.ex.items(c.req))
            j.cost_left = sum(self.ex.cost(c.req, n) for _, n in j.items)
            j.binding = self.ex.bind(c.req, off)
            c.t_admit = self.ex.now()
            self.jobs.append(j)
            self.max_in_flight = max(self.max_in_flight, len(self.jobs))

    def _dispatch(self):
        now = self.ex.now()
        # the highest slots first: the lower ones are those the large processes may use
        for slot in sorted(self.free_slots, reverse=True):
            best, key = None, None
            for j in self.jobs:
                if j.items and j.c.error is None and self.ex.slot_allowed(j.c.req.process, slot):
                    k = j.cost_left - self.aging * (now - j.c.req.arrival)
                    if key is None or k < key:
                        best, key = j, k
            if best is None:
                continue
            evt0, n = best.items.popleft()
            best.cost_left -= self.ex.cost(best.c.req, n)
            try:
                tok = self.ex.launch(best.binding, best.c.req, evt0, n, slot)
            except Exception as e:   # a failed launch fails its request; the slot stays free
                best.c.error = str(e)
                best.items.clear()
                self._maybe_complete(best)
                continue
            if best.c.t_start is None:
                best.c.t_start = now
            best.running += 1
            self.free_slots.discard(slot)
            self.running[slot] = (tok, best, n)
        self.max_busy_slots = max(self.max_busy_slots, len(self.running))

    def _maybe_complete(self, j, keep_results=False):
        if j.items or j.running:
            return
        c = j.c
        c.t_done = self.ex.now()
        c.ok = c.error is None
        if c.ok and keep_results:
            c.result = self.ex.result(j.binding, c.req)
        self.ex.unbind(j.binding)
        self.arena.release(j.off, j.fp)
        self.jobs.remove(j)
        self.done.append(c)

    def _poll(self, keep_results):
        for slot in list(self.running):
            tok, j, _ = self.running[slot]
            st = self.ex.poll(tok)
            if st is None:
                continue
            del self.running[slot]
            self.free_slots.add(slot)
            j.running -= 1
            if st is not True:
                j.c.error = str(st)
                j.items.clear()
            self._maybe_complete(j, keep_results)

    def run(self, requests, keep_results=False, progress=None, progress_every=20.0):
        """Drive the requests (arrival times relative to the start) to completion; returns the
        list of Completed.  progress(elapsed, done, total) is called every progress_every seconds
        of the executor's clock."""
        reqs = sorted(requests, key=lambda r: r.arrival)
        t0 = self.ex.now()
        next_report = progress_every
        i = 0
        while i < len(reqs) or self.waiting or self.jobs:
            now = self.ex.now() - t0
            if progress is not None and now >= next_report:
                progress(now, len(self.done), len(reqs))
                next_report += progress_every
            while i < len(reqs) and reqs[i].arrival <= now:
                r = reqs[i]
                self.submit(r._replace(arrival=t0 + r.arrival))
                i += 1
            self._poll(keep_results)
            self._admit()
            self._dispatch()
            self.ex.idle(reqs[i].arrival - now if i < len(reqs) else None, bool(self.running))
        return self.done


def latency_stats(done):
    lat = np.array([c.t_done - c.req.arrival for c in done if c.ok])
    if len(lat) == 0:
        return {"n": 0}
    return {"n": int(len(lat)), "p50_ms": float(np.quantile(lat, 0.5) * 1e3),
            "p99_ms": float(np.quantile(lat, 0.99) * 1e3), "mean_ms": float(lat.mean() * 1e3),
            "max_ms": float(lat.max() * 1e3)}


def latency_by_process(done):
    out = {}
    for p in sorted({c.req.process for c in done}):
        out[p] = latency_stats([c for c in done if c.req.process == p])
    return out


# ----------------------------------------------------------------------------------------
# executors


class FakeExecutor:
    """CPU stand-in: an item of n events of a process runs for cost[process] * n seconds of
    simulated time on its slot (slots run concurrently; simulated clock, no sleeping).  The
    'result' of event e of request r is r * 1e6 + e, written by the item that covers it."""

    def __init__(self, cost_per_event, bytes_per_event, item_events=None, large=(), n_large_slots=1, fail=None):
        self.cpe = cost_per_event
        self.bpe = bytes_per_event
        self.item_events = item_events or {}
        self.large = set(large)
        self.n_large = n_large_slots
        self.fail = fail or set()
        self.t = 0.0
        self.finish = {}
        self.slot_log = []    # (process, slot) of every launched item

    def now(self):
        return self.t

    def footprint(self, req):
        return self.bpe[req.process] * req.n_evt

    def items(self, req):
        return split_items(req.n_evt, self.item_events.get(req.process, req.n_evt))

    def cost(self, req, n):
        return self.cpe[req.process] * n

    def slot_allowed(self, process, slot):
        return process not in self.large or slot < self.n_large

    def bind(self, req, off):
        return {"out": np.full(req.n_evt, np.nan), "off": off}

    def unbind(self, binding):
        pass

    def launch(self, binding, req, evt0, n, slot):
        if req.rid in self.fail:
            raise RuntimeError(f"injected failure of request {req.rid}")
        tok = (req.rid, evt0, slot)
        self.finish[tok] = self.t + self.cpe[req.process] * n
        binding["out"][evt0:evt0 + n] = req.rid * 1e6 + np.arange(evt0, evt0 + n)
        self.slot_log.append((req.process, slot))
        return tok

    def poll(self, tok):
        if self.t >= self.finish[tok]:
            del self.finish[tok]
            return True
        return None

    def result(self, binding, req):
        return binding["out"].copy()

    def idle(self, until_next_arrival, busy):
        nxt = [f for f in self.finish.values() if f > self.t]
        cands = ([min(nxt)] if nxt and busy else []) + \
            ([self.t + until_next_arrival] if until_next_arrival is not None else [])
        self.t = max(self.t, min(cands)) if cands else self.t + 1e-6


class GpuExecutor:
    """Runs the library on one HIP stream per slot within a device-memory budget: the handles'
    tables, the scratch reserved for every (process, slot) pair, the runtime's memory for the
    kernels (measured after a warm-up), and a request arena that takes the rest.  Momenta of an
    item are made on its slot's stream by the library's RAMBO from the request's seed (in a
    deployment they would come from the integrator)."""

    def __init__(self, processes, n_slots, precision="fp64", hbm_budget=32 << 30, large=("gg_ttggg",),
                 n_large_slots=2, max_request_events=65536, sqrt_s=None, params=None, arena_bytes=None):
        import torch
        from .binding import Process
        self.torch = torch
        params = params or {}
        self.handles = {p: Process(p, precision=precision, **params) for p in processes}
        self.streams = [torch.cuda.Stream() for _ in range(n_slots)]
        # baseline: the process with the library loaded and the handles made (their tables are
        # charged to the budget below; the library's static array is not the server's), and
        # nothing left in torch's cache
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        free0, total = torch.cuda.mem_get_info()
        self.used0 = total - free0
        self.sqrt_s = sqrt_s or {p: (500.0 if p.startswith("ee") else 1500.0) for p in processes}
        self.large = set(large)
        self.n_large = max(1, min(n_large_slots, n_slots))
        self.max_request_events = max_request_events
        # items: one chunk of the library where a request would span several (the processes with
        # segment kernels, whose chunks are small), else the whole request
        self.item_events = {}
        for p, h in self.handles.items():
            ce = h.info["chunk_events"]
            self.item_events[p] = ce if h.info["n_partial_slots"] > 0 else max(ce, max_request_events)
        for p, h in self.handles.items():
            for s, st in enumerate(self.streams):
                if self.slot_allowed(p, s):
                    h.reserve_scratch(min(self.item_events[p], max_request_events), stream=st)
        self.scratch_bytes = sum(h.scratch_bytes() for h in self.handles.values())
        self.table_bytes = sum(h.info["bytes_resident"] for h in self.handles.values())
        # one item-sized call of every process on every slot it may use: the kernels' first launches
        # make the runtime allocate what they need beside the library's buffers (code objects, each
        # hardware queue's backing store for register spills), measured here and charged to the
        # budget; the timed calls on slot 0 give each process's seconds per event
        self.sec_per_event = self._warm_up()
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        free1, _ = torch.cuda.mem_get_info()
        self.fixed_bytes = (total - free1) - self.used0 + self.table_bytes
        # a given arena size sets the budget to what is measured plus the arena
        if arena_bytes is not None:
            hbm_budget = self.fixed_bytes + arena_bytes
        self.budget = hbm_budget
        self.budget_derived = arena_bytes is not None
        self.arena_bytes = (hbm_budget - self.fixed_bytes) // (2 << 20) * (2 << 20)
        biggest = max(self.footprint(Request(0, p, max_request_events, 0, 0.0)) for p in processes)
        if self.arena_bytes < biggest:
            raise ValueError(f"HBM budget {hbm_budget} B leaves {self.arena_bytes} B for requests after "
                             f"{self.fixed_bytes} B of scratch, tables and runtime memory; the largest request "
                             f"needs {biggest} B")
        self.arena = torch.empty(self.arena_bytes, dtype=torch.uint8, device="cuda")
        torch.cuda.synchronize()
        self.peak_used = 0
        self.track_memory()

    def _warm_up(self):
        torch = self.torch
        out = {}
        for p, h in self.handles.items():
            n = min(self.item_events[p], self.max_request_events)
            x = h.rambo(1, self.sqrt_s[p], n)
            y = torch.empty(n, dtype=torch.float64, device="cuda")
            torch.cuda.synchronize()
            for s, st in enumerate(self.streams):
                if not self.slot_allowed(p, s):
                    continue
                h.sigma(x, out=y, stream=st)
                st.synchronize()
                if s == 0:
                    t = time.perf_counter()
                    h.sigma(x, out=y, stream=st)
                    st.synchronize()
                    out[p] = (time.perf_counter() - t) / n
            del x, y
        return out

    # device memory held beyond what the process held before the executor existed
    def track_memory(self):
        free, total = self.torch.cuda.mem_get_info()
        self.peak_used = max(self.peak_used, total - free - self.used0)
        return self.peak_used

    def memory_report(self):
        return {"budget_bytes": self.budget, "budget_from_arena_size": self.budget_derived,
                "reserved_scratch_bytes": self.scratch_bytes,
                "handle_table_bytes": self.table_bytes,
                "runtime_bytes": self.fixed_bytes - self.scratch_bytes - self.table_bytes,
                "request_arena_bytes": self.arena_bytes,
                "device_used_peak_bytes": self.track_memory() + self.table_bytes,
                "device_used_peak_note": "hipMemGetInfo: device memory in use above the process's use once the "
                                         "library was loaded and the handles made, plus the handles' tables; "
                                         "highest value seen at admissions"}

    def now(self):
        return time.perf_counter()

    def _layout(self, req):
        npar = self.handles[req.process].n_par
        mom = -(-(req.n_evt * npar * 32) // 256) * 256
        return mom, req.n_evt * 8

    def footprint(self, req):
        mom, out = self._layout(req)
        return mom + out

    def items(self, req):
        return split_items(req.n_evt, self.item_events[req.process])

    def cost(self, req, n):
        return self.sec_per_event[req.process] * n

    def slot_allowed(self, process, slot):
        return process not in self.large or slot < self.n_large

    def bind(self, req, off):
        torch = self.torch
        mom, out = self._layout(req)
        h = self.handles[req.process]
        x = self.arena[off:off + req.n_evt * h.n_par * 32].view(torch.float64).view(req.n_evt, h.n_par, 4)
        y = self.arena[off + mom:off + mom + out].view(torch.float64)
        self.track_memory()
        return (x, y)

    def unbind(self, binding):
        pass

    def launch(self, binding, req, evt0, n, slot):
        torch = self.torch
        h = self.handles[req.process]
        st = self.streams[slot]
        x, y = binding
        xs, ys = x[evt0:evt0 + n], y[evt0:evt0 + n]
        h.rambo(req.seed, self.sqrt_s[req.process], n, evt0=evt0, out=xs, stream=st)
        h.sigma(xs, out=ys, stream=st)
        ev = torch.cuda.Event()
        ev.record(st)
        return ev

    def poll(self, ev):
        return True if ev.query() else None

    def result(self, binding, req):
        return binding[1].cpu().numpy()

    def idle(self, until_next_arrival, busy):
        # short spin: completions are polled, the device keeps working meanwhile
        if until_next_arrival is not None and until_next_arrival > 0 and not busy:
            time.sleep(min(until_next_arrival, 1e-3))


def run_alone(executor, requests):
    """each request alone, as one me_sigma call over all its events (the library's own chunking,
    and its two internal streams where a request spans several gg_ttggg chunks): results by
    request id"""
    torch = executor.torch
    out = {}
    for r in requests:
        h = executor.handles[r.process]
        x = h.rambo(r.seed, executor.sqrt_s[r.process], r.n_evt)
        out[r.rid] = h.sigma(x).cpu().numpy()
        del x
    torch.cuda.synchronize()
    return out


# Default memory of the serving benchmark.  Without gg_ttggg: a request arena of 96 MiB (about 15
# requests of the mean size), small enough that bursts wait for memory, on top of what the server
# measures it holds (scratch, tables, runtime memory for the kernels, about 1 GB); with gg_ttggg: a
# budget of 32 GiB, of which two slots' scratch for its 4096-event chunks (about 14.5 GB each in
# FP64) comes first.
SERVING_ARENA_SMALL = 96 << 20
SERVING_BUDGET_LARGE = 32 << 30


def bench_serving(duration_s=10.0, processes=("gg_tt", "gg_ttg", "gg_ttgg"), n_slots=4, hbm_budget=None,
                  loads=(0.5, 0.9), log=print):
    """Measure the saturated mix throughput, then run Poisson arrivals at the given fractions of
    it; report p50/p99 latency (overall and per process), throughput, and device memory against
    the budget."""
    import torch
    arena = None
    if hbm_budget is None:
        if "gg_ttggg" in processes:
            hbm_budget = SERVING_BUDGET_LARGE
        else:
            arena = SERVING_ARENA_SMALL
    ex = GpuExecutor(list(processes), n_slots, hbm_budget=hbm_budget, arena_bytes=arena)
    hbm_budget = ex.budget
    m = ex.memory_report()
    log(f"serving: budget {hbm_budget / 2**20:.0f} MiB = scratch {m['reserved_scratch_bytes'] / 2**20:.0f} MiB + "
        f"runtime {m['runtime_bytes'] / 2**20:.0f} MiB + tables {m['handle_table_bytes'] / 2**20:.1f} MiB + "
        f"request arena {m['request_arena_bytes'] / 2**20:.0f} MiB (and what rounding leaves)")
    # saturated throughput: a backlog of requests all arriving at t = 0
    warm = poisson_requests(8, 1e9, list(processes), seed=7)
    Scheduler(ex, n_slots, ex.arena_bytes).run([r._replace(arrival=0.0) for r in warm])
    sat_reqs = [r._replace(arrival=0.0) for r in poisson_requests(64, 1e9, list(processes), seed=2)]
    t = time.perf_counter()
    sch = Scheduler(ex, n_slots, ex.arena_bytes)
    done = sch.run(sat_reqs)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t
    ev = sum(c.req.n_evt for c in done if c.ok)
    sat_req_rate = len(done) / dt
    out = {"processes": list(processes), "slots": n_slots, "large_process_slots": ex.n_large,
           "saturated": {"requests_per_s": sat_req_rate, "MEs_per_s": ev / dt,
                         "admissions_waited_for_memory": sch.waited_for_memory}}
    log(f"serving: saturated {sat_req_rate:.1f} req/s, {ev / dt:.4g} MEs/s, "
        f"{sch.waited_for_memory} admissions waited for memory")
    for load in loads:
        rate = load * sat_req_rate
        n = max(20, int(rate * duration_s))
        reqs = poisson_requests(n, rate, list(processes), seed=1)
        sch = Scheduler(ex, n_slots, ex.arena_bytes)
        t = time.perf_counter()
        done = sch.run(reqs, progress=lambda el, nd, nt: log(f"serving load {load}: {el:.0f} s, {nd}/{nt} done"))
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        st = latency_stats(done)
        st.update({"offered_load": load, "requests": n, "MEs_per_s": sum(c.req.n_evt for c in done if c.ok) / dt,
                   "max_in_flight": sch.max_in_flight, "max_busy_slots": sch.max_busy_slots,
                   "failed": sum(1 for c in done if not c.ok),
                   "admissions_waited_for_memory": sch.waited_for_memory,
                   "per_process": latency_by_process(done)})
        out[f"load_{load}"] = st
        per = ", ".join(f"{p} p99 {v.get('p99_ms', 0):.1f} ms" for p, v in st["per_process"].items())
        log(f"serving load {load}: {n} requests, p50 {st.get('p50_ms', 0):.2f} ms, p99 {st.get('p99_ms', 0):.2f} ms "
            f"({per}), {st['MEs_per_s']:.4g} MEs/s, {sch.waited_for_memory} waited for memory")
    out["memory"] = ex.memory_report()
    return out
