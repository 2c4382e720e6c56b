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
     (walker state from ``qmc_bytes_per_walker`` plus the system tables)
     fits the HBM budget and a stream slot is free; a request's initial
     walkers are drawn on its stream from its own seeded generator, and
     its system's drawn tables come from a per-molecule cache, so admission
     costs the scheduler thread little host time;
  2. launches the next chunk of ``chunk_steps`` Metropolis steps for every
     active request whose previous chunk has finished, each on its own
     stream, so chunks of different molecules overlap on the device;
  3. retires requests whose last chunk finished: copies the per-walker
     accumulators to the host, reduces them in a fixed order, frees the
     state and fulfils the future.  The system's device tables (under 1 MiB
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


@dataclass
class Result:
    id: int
    name: str
    walkers: int
    steps: int
    precision: str
    mean_energy: float        # mean of E_L over walkers and steps
    energy_variance: float
    acceptance: float
    latency_s: float          # arrival -> result
    queue_s: float            # arrival -> admission
    footprint_bytes: int
    acc: np.ndarray = field(repr=False, default=None)  # per-walker (sum E_L, sum E_L^2, accepted)


class AdmissionError(RuntimeError):
    pass


def reduce_accumulators(acc: np.ndarray, steps: int):
    """Fixed-order reduction of the per-walker accumulators (numpy's pairwise
    summation: the same order for the same walker count, so a request's
    result does not depend on what else runs)."""
    n = acc.shape[0] * steps
    s1, s2, s3 = (float(v) for v in np.sum(np.ascontiguousarray(acc.T), axis=1))
    mean = s1 / n
    var = s2 / n - mean * mean
    return mean, var, s3 / n


class _Active:
    def __init__(self, req, fut, system, state, acc, stream, footprint, admitted):
        self.req, self.fut, self.system = req, fut, system
        self.state, self.acc, self.stream = state, acc, stream
        self.footprint, self.admitted = footprint, admitted
        self.done_steps = 0
        self.events = collections.deque()  # chunks in flight on this stream


class Server:
    """Single-GPU VMC request server with footprint admission."""

    def __init__(self, device: int = 0, hbm_budget_bytes: int = 8 << 30, chunk_steps: int = 25,
                 max_active: int = 8):
        import torch
        self.torch = torch
        self.device = torch.device(f"cuda:{device}")
        self.dev_index = device
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
        self.overlap_samples = 0
        self.overlap_active_sum = 0
        self._free_streams = None  # created on the scheduler thread

    # -- public ---------------------------------------------------------------
    @staticmethod
    def footprint(req: Request) -> int:
        """Device bytes a request holds while active: its walker state (the
        same per-walker count qmc_bytes_per_walker reports: positions,
        log|Psi|, sign, E_L and three accumulators, FP64) plus 1 MiB bounding
        the system tables."""
        if getattr(req, "_footprint", None) is None:
            n_e = synth.n_elec(synth.make_system(req.name, bond_scale=req.bond_scale))
            req._footprint = req.walkers * (3 * n_e + 6) * 8 + (1 << 20)
        return req._footprint

    def submit(self, req: Request) -> Future:
        fut: Future = Future()
        if req.arrival == 0.0:
            req.arrival = time.perf_counter()
        if self.footprint(req) > self.budget:
            fut.set_exception(AdmissionError(
                f"request {req.id} needs {self.footprint(req)} B > budget {self.budget} B"))
            return fut
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
            self._drain_queue()
            self._admit()
            self._launch()
            retired = self._retire()
            idle = not self.active and not self.pending and self.q.empty()
            if idle or len(self._retired_systems) > 64:
                self._destroy_retired()
            if idle and stop_when_idle and (producer is None or not producer.is_alive()):
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
        while self.pending and self._free_streams:
            req, fut = self.pending[0]
            need = self.footprint(req)
            if self.used + need > self.budget:
                return  # wait for memory: requests are admitted in arrival order
            self.pending.popleft()
            stream = self._free_streams.pop()
            sysd = synth.make_system(req.name, bond_scale=req.bond_scale)
            system = qmc.System(sysd, device=self.dev_index)
            with torch.cuda.stream(stream):
                # drawn on the device: no host generation or copy on the scheduler thread
                X = synth.init_walkers_device(sysd, req.walkers, req.walker_seed, self.device)
                lp, sg, el = system.eval(X, precision=req.precision)
                acc = torch.zeros((req.walkers, 3), dtype=torch.float64, device=self.device)
            a = _Active(req, fut, system, [X, lp, sg, el], acc, stream, need, time.perf_counter())
            self.used += need
            self.active.append(a)
            self.peak_active = max(self.peak_active, len(self.active))

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
                acc = a.acc.cpu().numpy()
                mean, var, accr = reduce_accumulators(acc, a.req.steps)
                now = time.perf_counter()
                r = Result(a.req.id, a.req.name, a.req.walkers, a.req.steps, a.req.precision, mean, var,
                           accr, now - a.req.arrival, a.admitted - a.req.arrival, a.footprint, acc)
                self._retired_systems.append(a.system)
                a.system = a.state = a.acc = None
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
