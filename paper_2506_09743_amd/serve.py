"""Continuous-batching server for VMC blocks.

A request asks for one Metropolis block (``steps`` all-electron moves of
``walkers`` walkers) of one molecule at one geometry, in FP64 or the mixed
form, and gets back its mean local energy (the Monte Carlo estimate of the
variational energy, the paper's Introduction), its variance, the acceptance
and its latency.

Scheduling.  One host thread runs the loop; every admitted request owns a
HIP stream (default priority) and its walker state stays resident in HBM
until it retires.  Each loop iteration

  1. admits queued requests in arrival order while their device footprint
     (walkers x ``qmc_bytes_per_walker`` plus a bound on the system tables)
     fits the HBM budget and a stream slot is free.  The budget is the
     device's free HBM when the server starts (``hipMemGetInfo`` through
     torch) minus a reserve, unless the caller sets it; the server counts
     how many requests had to wait for memory and how many for a stream
     slot.  A request's initial walkers are drawn on its stream from its own
     seeded generator, and its system's drawn tables come from a
     per-molecule cache, so admission costs the scheduler thread little
     host time;
  2. launches the next chunk of ``chunk_steps`` Metropolis steps for every
     active request whose previous chunk has finished, each on its own
     stream, so chunks of different molecules overlap on the device;
  3. retires requests whose last chunk finished: reduces the per-walker
     accumulators on the device in an order fixed by the walker count
     (``qmc_reduce_accumulators``), copies the five sums to the host, frees
     the state and fulfils the future.  Walker-steps whose state had no
     finite log|Psi| or E_L are counted and left out of the mean.  The system's device tables (under 1 MiB
     each) are freed in batches, when the server is idle or 64 have piled
     up, so a retirement never waits on other requests' work.

A request's numbers depend only on its own inputs (system, walker seed,
Philox seed, request-local walker ids), never on what else is in flight, so
a result is identical alone and in the mix.
"""
from __future__ import annotations

import collections
import queue
import threading
import time
from concurrent.futures import Future
from dataclasses import dataclass, field

import numpy as np

from . import qmc, synth


@dataclass
class Request:
    id: int
    name: str                 # H2, LiH, Li2 or CO
    bond_scale: float
    walkers: int
    steps: int
    precision: str = "fp64"   # "fp64" or "fp32"
    walker_seed: int = 0
    philox_seed: int = 0
    sigma: float = 0.2
    arrival: float = 0.0      # host clock (perf_counter) at submission
    keep_walkers: bool = False  # return the initial walkers and per-walker sums (checks)


@dataclass
class Result:
    id: int
    name: str
    walkers: int
    steps: int
    precision: str
    mean_energy: float        # mean of E_L over the finite walker-steps
    energy_variance: float
    acceptance: float
    latency_s: float          # arrival -> result
    queue_s: float            # arrival -> admission
    footprint_bytes: int
    nonfinite_steps: int = 0  # walker-steps left out of the mean
    nonfinite_walkers: int = 0
    waited_for: str = ""      # "", "memory" or "slot": what first held its admission
    # with keep_walkers: the initial walkers [W][N_e][3] and the per-walker
    # accumulators [W][4] (sum E_L, sum E_L^2, accepted, non-finite)
    initial_walkers: np.ndarray = field(repr=False, default=None)
    acc: np.ndarray = field(repr=False, default=None)


class AdmissionError(RuntimeError):
    pass


def block_statistics(sums, walkers: int, steps: int):
    """Mean energy, variance, acceptance and non-finite counts from the five
    device sums of qmc_reduce_accumulators (sum E_L, sum E_L^2, accepted,
    non-finite steps, walkers with non-finite steps)."""
    s1, s2, s3, bad, bad_w = (float(v) for v in sums)
    n_all = walkers * steps
    n = n_all - bad
    mean = s1 / n if n > 0 else float("nan")
    var = s2 / n - mean * mean if n > 0 else float("nan")
    return mean, var, s3 / n_all if n_all else float("nan"), int(bad), int(bad_w)


class _Active:
    def __init__(self, req, fut, system, state, acc, stream, footprint, admitted):
        self.req, self.fut, self.system = req, fut, system
        self.state, self.acc, self.stream = state, acc, stream
        self.footprint, self.admitted = footprint, admitted
        self.done_steps = 0
        self.events = collections.deque()  # chunks in flight on this stream


class Server:
    """Single-GPU VMC request server with footprint admission."""

    # HBM kept back from the admission budget: torch's caching allocator,
    # the runtime and fragmentation
    RESERVE_BYTES = 4 << 30
    RESERVE_FRACTION = 0.05
    # bound on one request's system tables (a few hundred KB at most here)
    SYSTEM_TABLE_BYTES = 1 << 20

    def __init__(self, device: int = 0, hbm_budget_bytes: int = None, chunk_steps: int = 25,
                 max_active: int = 8):
        import torch
        self.torch = torch
        self.device = torch.device(f"cuda:{device}")
        self.dev_index = device
        if hbm_budget_bytes is None:
            free, total = torch.cuda.mem_get_info(device)
            hbm_budget_bytes = max(0, free - max(self.RESERVE_BYTES, int(self.RESERVE_FRACTION * total)))
        self.budget = int(hbm_budget_bytes)
        self.chunk = int(chunk_steps)
        self.max_active = int(max_active)
        self.q: "queue.Queue" = queue.Queue()
        self.pending: "collections.deque" = collections.deque()
        self.active: list = []
        self.used = 0
        self.results: list = []
        self._retired_systems: list = []  # destroyed once the server is idle
        self.peak_active = 0
        self.peak_used = 0
        self.overlap_samples = 0
        self.overlap_active_sum = 0
        self.waits_memory = 0      # requests whose admission first waited for HBM
        self.waits_slot = 0        # ... for a free stream slot
        self._bpw = {}             # bytes per walker by molecule (from the C ABI)
        self._free_streams = None  # created on the scheduler thread

    # -- public ---------------------------------------------------------------
    def footprint(self, req: Request) -> int:
        """Device bytes a request holds while active: walkers x
        qmc_bytes_per_walker (positions, log|Psi|, sign, E_L and the four
        accumulators) plus the bound on its system tables.  Runs on the
        scheduler thread (it may create the molecule's reference handle)."""
        if getattr(req, "_footprint", None) is None:
            if req.name not in self._bpw:
                ref = qmc.System(synth.make_system(req.name), device=self.dev_index)
                self._bpw[req.name] = ref.bytes_per_walker(req.precision)
                ref.close()
            req._footprint = req.walkers * self._bpw[req.name] + self.SYSTEM_TABLE_BYTES
        return req._footprint

    def submit(self, req: Request) -> Future:
        """Queues a request (any thread); a request that could never fit the
        budget fails with AdmissionError when the scheduler reaches it."""
        fut: Future = Future()
        if req.arrival == 0.0:
            req.arrival = time.perf_counter()
        self.q.put((req, fut))
        return fut

    def run(self, stop_when_idle: bool = True, producer: threading.Thread = None,
            poll_s: float = 2e-4) -> list:
        """Scheduler loop; returns the results in completion order."""
        torch = self.torch
        torch.cuda.set_device(self.dev_index)
        if self._free_streams is None:
            self._free_streams = [torch.cuda.Stream(device=self.device) for _ in range(self.max_active)]
        while True:
            # read before draining the queue: once the producer has ended,
            # everything it submitted is in the queue when it is drained
            producer_done = producer is None or not producer.is_alive()
            self._drain_queue()
            self._admit()
            self._launch()
            retired = self._retire()
            idle = not self.active and not self.pending and self.q.empty()
            if idle or len(self._retired_systems) > 64:
                self._destroy_retired()
            if idle and stop_when_idle and producer_done:
                break
            if not retired:
                time.sleep(poll_s)
        return self.results

    # -- internals ---------------------------------------------------------------
    def _destroy_retired(self):
        """Frees retired systems' device tables; deferred so that a retirement
        never waits on the other requests' work in flight."""
        for system in self._retired_systems:
            system.close()
        self._retired_systems = []

    def _drain_queue(self):
        while True:
            try:
                self.pending.append(self.q.get_nowait())
            except queue.Empty:
                return

    def _admit(self):
        torch = self.torch
        while self.pending:
            req, fut = self.pending[0]
            need = self.footprint(req)
            if need > self.budget:
                self.pending.popleft()
                fut.set_exception(AdmissionError(
                    f"request {req.id} needs {need} B > budget {self.budget} B"))
                continue
            if self.used + need > self.budget:
                self._note_wait(req, "memory")
                return  # wait for memory: requests are admitted in arrival order
            if not self._free_streams:
                self._note_wait(req, "slot")
                return
            self.pending.popleft()
            stream = self._free_streams.pop()
            sysd = synth.make_system(req.name, bond_scale=req.bond_scale)
            system = qmc.System(sysd, device=self.dev_index)
            with torch.cuda.stream(stream):
                # drawn on the device: no host generation or copy on the scheduler thread
                X = synth.init_walkers_device(sysd, req.walkers, req.walker_seed, self.device)
                X0 = X.clone() if req.keep_walkers else None
                lp, sg, el = system.eval(X, precision=req.precision)
                acc = torch.zeros((req.walkers, qmc.ACC_COLS), dtype=torch.float64, device=self.device)
                sums = torch.empty(5, dtype=torch.float64, device=self.device)
            a = _Active(req, fut, system, [X, lp, sg, el], acc, stream, need, time.perf_counter())
            a.initial, a.sums = X0, sums
            self.used += need
            self.active.append(a)
            self.peak_active = max(self.peak_active, len(self.active))
            self.peak_used = max(self.peak_used, self.used)

    def _note_wait(self, req, why: str):
        """Admission is in arrival order: when the head of the queue waits,
        every queued request waits for the same reason; each is counted once,
        for the first reason it waited."""
        for r, _ in self.pending:
            if not getattr(r, "_waited", ""):
                r._waited = why
                if why == "memory":
                    self.waits_memory += 1
                else:
                    self.waits_slot += 1

    def _launch(self):
        """Keeps up to two chunks queued per request so its stream never
        drains between scheduler iterations."""
        torch = self.torch
        running = 0
        for a in self.active:
            while a.events and a.events[0].query():
                a.events.popleft()
            while len(a.events) < 2 and a.done_steps < a.req.steps:
                n = min(self.chunk, a.req.steps - a.done_steps)
                with torch.cuda.stream(a.stream):
                    a.system.metropolis(*a.state, n, a.req.sigma, a.req.philox_seed,
                                        step0=a.done_steps, acc=a.acc, precision=a.req.precision)
                    if a.done_steps + n >= a.req.steps:
                        # the last chunk: reduce the accumulators on the device
                        qmc.qmc_reduce_accumulators(a.acc, a.sums)
                    ev = torch.cuda.Event()
                    ev.record(a.stream)
                a.events.append(ev)
                a.done_steps += n
            if a.events:
                running += 1
        if running:
            self.overlap_samples += 1
            self.overlap_active_sum += running

    def _retire(self) -> int:
        n = 0
        keep = []
        for a in self.active:
            while a.events and a.events[0].query():
                a.events.popleft()
            if a.done_steps >= a.req.steps and not a.events:
                sums = a.sums.cpu().numpy()  # five doubles; the stream has finished
                mean, var, accr, bad, bad_w = block_statistics(sums, a.req.walkers, a.req.steps)
                now = time.perf_counter()
                r = Result(a.req.id, a.req.name, a.req.walkers, a.req.steps, a.req.precision, mean, var,
                           accr, now - a.req.arrival, a.admitted - a.req.arrival, a.footprint,
                           nonfinite_steps=bad, nonfinite_walkers=bad_w,
                           waited_for=getattr(a.req, "_waited", ""))
                if a.req.keep_walkers:
                    r.initial_walkers = a.initial.cpu().numpy()
                    r.acc = a.acc.cpu().numpy()
                self._retired_systems.append(a.system)
                a.system = a.state = a.acc = a.initial = a.sums = None
                self.used -= a.footprint
                self._free_streams.append(a.stream)
                self.results.append(r)
                a.fut.set_result(r)
                n += 1
            else:
                keep.append(a)
        self.active = keep
        return n


def requests_from_stream(stream: list) -> list:
    """(unit-mean gap, Request) pairs from ``synth.serving_request_stream``."""
    return [(r["gap"], Request(id=r["id"], name=r["name"], bond_scale=r["bond_scale"],
                               walkers=r["walkers"], steps=r["steps"], precision=r["precision"],
                               walker_seed=r["walker_seed"], philox_seed=r["philox_seed"]))
            for r in stream]


def poisson_producer(server: Server, timed_requests: list, rate_hz: float) -> threading.Thread:
    """Submits (gap, Request) pairs with exponential inter-arrival times of
    mean 1 / rate_hz (each gap is a unit-mean exponential draw)."""

    def run():
        t = time.perf_counter()
        for gap, req in timed_requests:
            t += gap / rate_hz
            delay = t - time.perf_counter()
            if delay > 0:
                time.sleep(delay)
            req.arrival = 0.0
            server.submit(req)

    th = threading.Thread(target=run, daemon=True)
    th.start()
    return th


def latency_summary(results: list, wall_s: float) -> dict:
    lat = np.array([r.latency_s for r in results])
    ws = sum(r.walkers * r.steps for r in results)
    return {"requests": len(results), "p50_s": float(np.percentile(lat, 50)),
            "p99_s": float(np.percentile(lat, 99)), "mean_s": float(lat.mean()),
            "walker_steps_per_s": ws / wall_s, "wall_s": wall_s}
