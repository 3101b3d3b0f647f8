"""Serving loop: matrix-element requests of mixed processes and sizes, admitted
continuously onto concurrent HIP streams.

Requests arrive as an MC integrator's channels issue them (here: a Poisson process).  The
server keeps one library handle per process resident (colour matrices, helicity masks,
couplings on the device) and S slots, each a HIP stream with its own jamp scratch.  A
pending request is admitted, in arrival order, as soon as a slot is free and its HBM
footprint (momenta + output + its share of the slot's jamp scratch) fits the remaining
budget; requests on different slots run concurrently on the device.  Completion is polled
through HIP events; latency = completion time - arrival time on the host monotonic clock.

The scheduling logic is independent of the executor: ``GpuExecutor`` runs me_sigma on the
GPU, ``FakeExecutor`` (tests on the CPU) completes a request after a time proportional to
its cost, so admission, ordering and failure handling can be checked without a GPU.
"""
import collections
import heapq
import math
import time

import numpy as np

Request = collections.namedtuple("Request", "rid process n_evt seed arrival")


class Completed:
    __slots__ = ("req", "slot", "t_admit", "t_done", "ok", "error", "result")

    def __init__(self, req, slot, t_admit):
        self.req, self.slot, self.t_admit = req, slot, t_admit
        self.t_done, self.ok, self.error, self.result = None, None, None, None


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


class Scheduler:
    """Admission and completion bookkeeping over an executor with `n_slots` slots and an
    HBM budget in bytes."""

    def __init__(self, executor, n_slots, hbm_budget):
        self.ex = executor
        self.n_slots = n_slots
        self.budget = hbm_budget
        self.used = 0
        self.free_slots = list(range(n_slots))
        self.pending = collections.deque()
        self.running = {}
        self.done = []
        self.max_in_flight = 0

    def footprint(self, req):
        return self.ex.footprint(req)

    def submit(self, req):
        fp = self.footprint(req)
        if fp > self.budget:
            c = Completed(req, None, None)
            c.ok, c.error, c.t_done = False, f"footprint {fp} B exceeds the HBM budget {self.budget} B", \
                self.ex.now()
            self.done.append(c)
            return
        self.pending.append(req)

    def _admit(self):
        while self.pending and self.free_slots:
            req = self.pending[0]
            fp = self.footprint(req)
            if self.used + fp > self.budget:
                break  # FIFO: the head waits for memory; later requests do not overtake it
            self.pending.popleft()
            slot = self.free_slots.pop()
            self.used += fp
            c = Completed(req, slot, self.ex.now())
            try:
                token = self.ex.launch(req, slot)
            except Exception as e:  # a failed launch completes with an error and frees its slot
                c.ok, c.error, c.t_done = False, str(e), self.ex.now()
                self.used -= fp
                self.free_slots.append(slot)
                self.done.append(c)
                continue
            self.running[slot] = (c, token, fp)
            self.max_in_flight = max(self.max_in_flight, len(self.running))

    def _poll(self):
        for slot in list(self.running):
            c, token, fp = self.running[slot]
            st = self.ex.poll(token)
            if st is None:
                continue
            c.t_done = self.ex.now()
            c.ok = st is True
            if c.ok:
                c.result = self.ex.result(token)
            else:
                c.error = str(st)
            del self.running[slot]
            self.used -= fp
            self.free_slots.append(slot)
            self.done.append(c)

    def run(self, requests, keep_results=False, progress=None, progress_every=20.0):
        """Drive the requests (sorted by arrival, times relative to the start) to
        completion; returns the list of Completed.  progress(elapsed, done, total) is
        called every progress_every seconds of the executor's clock."""
        reqs = sorted(requests, key=lambda r: r.arrival)
        t0 = self.ex.now()
        next_report = progress_every
        i = 0
        while i < len(reqs) or self.pending or self.running:
            now = self.ex.now() - t0
            if progress is not None and now >= next_report:
                progress(now, len(self.done), len(reqs))
                next_report += progress_every
            while i < len(reqs) and reqs[i].arrival <= now:
                r = reqs[i]
                self.submit(r._replace(arrival=t0 + r.arrival))
                i += 1
            self._poll()
            self._admit()
            if not keep_results:
                for c in self.done:
                    c.result = None
            self.ex.idle(reqs[i].arrival - now if i < len(reqs) else None, bool(self.running))
        return self.done


def latency_stats(done):
    lat = np.array([c.t_done - c.req.arrival for c in done if c.ok])
    if len(lat) == 0:
        return {"n": 0}
    return {"n": int(len(lat)), "p50_ms": float(np.quantile(lat, 0.5) * 1e3),
            "p99_ms": float(np.quantile(lat, 0.99) * 1e3), "mean_ms": float(lat.mean() * 1e3),
            "max_ms": float(lat.max() * 1e3)}


# ----------------------------------------------------------------------------------------
# executors


class FakeExecutor:
    """CPU stand-in: a request 'runs' for cost(process) * n_evt seconds of simulated time on
    its slot; slots run concurrently.  Simulated clock, no sleeping."""

    def __init__(self, cost_per_event, bytes_per_event, fail=None):
        self.cost = cost_per_event
        self.bpe = bytes_per_event
        self.fail = fail or set()
        self.t = 0.0
        self.finish = {}

    def now(self):
        return self.t

    def footprint(self, req):
        return self.bpe[req.process] * req.n_evt

    def launch(self, req, slot):
        if req.rid in self.fail:
            raise RuntimeError(f"injected failure of request {req.rid}")
        tok = (req.rid, slot)
        self.finish[tok] = (self.t + self.cost[req.process] * req.n_evt, req)
        return tok

    def poll(self, tok):
        return True if self.t >= self.finish[tok][0] else None

    def result(self, tok):
        req = self.finish[tok][1]
        return np.full(req.n_evt, float(req.rid))

    def idle(self, until_next_arrival, busy):
        nxt = [f for f, _ in self.finish.values() if f > self.t]
        cands = ([min(nxt)] if nxt and busy else []) + \
            ([self.t + until_next_arrival] if until_next_arrival is not None else [])
        self.t = max(self.t, min(cands)) if cands else self.t + 1e-6


class GpuExecutor:
    """Runs me_sigma on one HIP stream per slot.  Momenta of a request are generated on its
    slot's stream by the library's RAMBO from the request's seed (in a serving deployment
    they would come from the integrator)."""

    def __init__(self, processes, n_slots, precision="fp64", sqrt_s=None, params=None):
        import torch
        from .binding import Process
        self.torch = torch
        params = params or {}
        self.handles = {p: Process(p, precision=precision, **params) for p in processes}
        self.streams = [torch.cuda.Stream() for _ in range(n_slots)]
        self.sqrt_s = sqrt_s or {p: (500.0 if p == "ee_mumu" else 1500.0) for p in processes}
        self.live = {}

    def now(self):
        return time.perf_counter()

    def footprint(self, req):
        h = self.handles[req.process]
        info = h.info
        mom = req.n_evt * info["n_par"] * 32
        out = req.n_evt * 8
        scratch = min(req.n_evt + 63, info["chunk_events"]) * info["bytes_per_event_scratch"]
        if info["n_partial_slots"] > 0 and req.n_evt > info["chunk_events"]:
            scratch *= 2   # the library's two internal streams, a chunk of scratch each
        return mom + out + scratch

    def launch(self, req, slot):
        torch = self.torch
        h = self.handles[req.process]
        st = self.streams[slot]
        with torch.cuda.stream(st):
            x = torch.empty((req.n_evt, h.n_par, 4), dtype=torch.float64, device="cuda")
            out = torch.empty(req.n_evt, dtype=torch.float64, device="cuda")
            h.rambo(req.seed, self.sqrt_s[req.process], req.n_evt, out=x, stream=st)
            h.sigma(x, out=out, stream=st)
            ev = torch.cuda.Event()
            ev.record(st)
        tok = (req.rid, slot)
        self.live[tok] = (ev, x, out)
        return tok

    def poll(self, tok):
        ev = self.live[tok][0]
        return True if ev.query() else None

    def result(self, tok):
        ev, x, out = self.live.pop(tok)
        return out

    def idle(self, until_next_arrival, busy):
        # short spin: completions are polled, the device keeps working meanwhile
        if until_next_arrival is not None and until_next_arrival > 0 and not busy:
            time.sleep(min(until_next_arrival, 1e-3))


def run_alone(executor, requests):
    """each request alone on slot 0, one after the other: results by request id"""
    out = {}
    for r in requests:
        tok = executor.launch(r, 0)
        while executor.poll(tok) is None:
            pass
        out[r.rid] = executor.result(tok)
    return out


def bench_serving(duration_s=10.0, processes=("gg_tt", "gg_ttg", "gg_ttgg"), n_slots=4,
                  hbm_budget=32 << 30, loads=(0.5, 0.9), log=print):
    """Measure the saturated mix throughput, then run Poisson arrivals at the given
    fractions of it; report p50/p99 latency and achieved throughput per load."""
    import torch
    ex = GpuExecutor(list(processes), n_slots)
    # saturated throughput: a backlog of requests all arriving at t = 0
    warm = poisson_requests(8, 1e9, list(processes), seed=7)
    Scheduler(ex, n_slots, hbm_budget).run([r._replace(arrival=0.0) for r in warm])
    sat_reqs = [r._replace(arrival=0.0) for r in poisson_requests(64, 1e9, list(processes), seed=2)]
    t = time.perf_counter()
    done = Scheduler(ex, n_slots, hbm_budget).run(sat_reqs)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t
    ev = sum(c.req.n_evt for c in done if c.ok)
    sat_req_rate = len(done) / dt
    out = {"processes": list(processes), "slots": n_slots, "hbm_budget_bytes": hbm_budget,
           "saturated": {"requests_per_s": sat_req_rate, "MEs_per_s": ev / dt}}
    log(f"serving: saturated {sat_req_rate:.1f} req/s, {ev / dt:.4g} MEs/s")
    for load in loads:
        rate = load * sat_req_rate
        n = max(20, int(rate * duration_s))
        reqs = poisson_requests(n, rate, list(processes), seed=1)
        sch = Scheduler(ex, n_slots, hbm_budget)
        t = time.perf_counter()
        done = sch.run(reqs, progress=lambda el, nd, nt: log(f"serving load {load}: {el:.0f} s, {nd}/{nt} done"))
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        st = latency_stats(done)
        st.update({"offered_load": load, "requests": n, "MEs_per_s": sum(c.req.n_evt for c in done if c.ok) / dt,
                   "max_in_flight": sch.max_in_flight, "failed": sum(1 for c in done if not c.ok)})
        out[f"load_{load}"] = st
        log(f"serving load {load}: {n} requests, p50 {st.get('p50_ms', 0):.2f} ms, p99 {st.get('p99_ms', 0):.2f} ms, "
            f"{st['MEs_per_s']:.4g} MEs/s, max in flight {sch.max_in_flight}")
    return out
