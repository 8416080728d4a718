"""Continuous-batching HOTRG solve server on one GPU.

Requests (model, q, T, D, steps) arrive over time.  The scheduler admits a
request when a stream slot is free and its device footprint
(hotrg_workspace_bytes: dominated by the two D^5 intermediates) fits the
memory budget, keeps every admitted solve's tensors resident in its own
workspace, and advances the active solves one coarse-graining step at a time,
round-robin, each on its own HIP stream, so that the steps of different solves
overlap on the device (iteration-level scheduling, not run-to-completion).  A
solve completes when the event recorded after its last step has fired; its
ln Z / N is read, its latency recorded, and its memory and slot are released
for the next request.  All device work goes through the C ABI (binding.py);
this module only schedules.  The steps themselves are whole steps (every
eigensolver pass up to the cap enqueued), host-polled steps driven by this
loop, or host-polled steps driven by the library's progress thread
(`stepping`); the results are bitwise the same.

Results do not depend on the mix: each solve's kernels use fixed-order
reductions and no atomics, so a solve gives bitwise the same ln Z / N alone
and among others.
"""
from __future__ import annotations

import collections
import time
from dataclasses import dataclass, field

import torch

from . import accounting, binding


@dataclass
class Completed:
    rid: int
    model: str
    q: int
    temperature: float
    dmax: int
    nsteps: int
    precision: str
    lnz_per_site: float
    arrival: float        # seconds since the start of the run
    admitted: float
    finished: float
    footprint: int
    flops: float
    stage_ms: dict | None = None

    @property
    def latency(self) -> float:
        return self.finished - self.arrival

    @property
    def free_energy(self) -> float:
        return -self.temperature * self.lnz_per_site


@dataclass
class _Active:
    req: object
    solve: binding.Solve
    stream: object
    workspace: torch.Tensor
    footprint: int
    admitted: float
    slot: int = -1
    enqueued: int = 0
    pending: bool = False     # a host-polled step waits for its eigensolve
    mode: str = "whole"       # how this solve's steps are enqueued
    events: collections.deque = field(default_factory=collections.deque)


class Server:
    """Schedules HOTRG solves on one device.

    slots       maximum number of solves in flight (one HIP stream each)
    budget      bytes of device memory the solves' workspaces may hold
    depth       coarse-graining steps a solve may have enqueued ahead of the
                device (keeps every stream busy without flooding the host)
    precision   contraction precision of every solve
    timing      record per-stage HIP events of every solve (hotrg_stage_times)
    stepping    "whole": whole steps (hotrg_coarse_grain_batch), every
                eigensolver pass up to the cap enqueued; "polled": host-
                polled steps (hotrg_step_begin / hotrg_step_poll) driven by
                this loop, a step's products enqueued once the host has seen
                its eigensolve stop, so no pass after convergence is
                enqueued; "engine": the same steps driven by the library's
                own progress thread (hotrg_coarse_grain_async), this loop
                only admitting and completing solves; "hybrid": "engine" for
                solves with D <= hybrid_dmax, "whole" for the others
    poll_extra  passes beyond a solve's history in a polled step's first group
    idle_sleep  seconds the scheduling loop sleeps when a round enqueued nothing
    """

    STEPPINGS = ("whole", "polled", "engine", "hybrid")

    def __init__(self, slots: int = 8, budget: int = 64 << 30, depth: int = 2,
                 precision: str = "fp64", device: str = "cuda:0", timing: bool = False,
                 stepping: str = "whole", poll_extra: int = 0, idle_sleep: float = 2e-4,
                 hybrid_dmax: int = 32):
        if stepping not in self.STEPPINGS:
            raise ValueError(f"stepping must be one of {self.STEPPINGS}")
        binding.load()
        self.timing = timing
        self.stepping = stepping
        self.hybrid_dmax = hybrid_dmax
        self.poll_extra = poll_extra
        self.idle_sleep = idle_sleep
        self.device = torch.device(device)
        self.slots = slots
        self.budget = budget
        self.depth = depth
        self.precision = precision
        self.streams = [torch.cuda.Stream(device=self.device) for _ in range(slots)]
        self.free_streams = list(range(slots))
        self.in_use = 0
        self.peak_in_use = 0
        self.queue: collections.deque = collections.deque()
        self.active: list[_Active] = []
        self.done: list[Completed] = []
        self.admission_log: list = []   # (rid, footprint, bytes in use after admission)
        self.t0 = None

    # -- footprint -------------------------------------------------------
    def footprint(self, req) -> int:
        return binding.workspace_bytes(model=req.model, q=req.q, temperature=req.temperature,
                                       dmax=req.dmax, precision=self.precision, max_steps=req.nsteps)

    # -- scheduling ------------------------------------------------------
    def _now(self) -> float:
        return time.perf_counter() - self.t0

    def _admit(self):
        while self.queue and self.free_streams:
            req = self.queue[0]
            fp = self.footprint(req)
            if fp == 0:
                raise ValueError(f"request {req.rid} has an invalid parameter set")
            if fp > self.budget:
                raise ValueError(f"request {req.rid} needs {fp} bytes, more than the whole budget")
            if self.in_use + fp > self.budget:
                break   # wait for memory; requests are admitted in arrival order
            self.queue.popleft()
            si = self.free_streams.pop()
            stream = self.streams[si]
            ws = torch.empty(fp, dtype=torch.uint8, device=self.device)
            solve = binding.Solve(model=req.model, q=req.q, temperature=req.temperature, dmax=req.dmax,
                                  precision=self.precision, stream=stream, workspace=ws, max_steps=req.nsteps)
            self.in_use += fp
            self.peak_in_use = max(self.peak_in_use, self.in_use)
            self.admission_log.append((req.rid, fp, self.in_use))
            if self.timing:
                solve.set_timing(True)
            a = _Active(req=req, solve=solve, stream=stream, workspace=ws, footprint=fp, admitted=self._now(),
                        slot=si)
            a.mode = self.stepping
            if a.mode == "hybrid":
                a.mode = "engine" if req.dmax <= self.hybrid_dmax else "whole"
            if a.mode == "engine":
                solve.coarse_grain_async(req.nsteps, extra=self.poll_extra)
                a.enqueued = req.nsteps
                a.pending = True
            self.active.append(a)

    def _stepped(self, a: _Active):
        ev = torch.cuda.Event()
        ev.record(a.stream)
        a.events.append(ev)

    def _advance_polled(self) -> bool:
        """Poll every solve's pending step (enqueueing more eigensolver passes
        or the step's products), and begin the next step of a solve that has
        none pending and room on its stream; True if anything was enqueued."""
        progressed = False
        for a in self.active:
            if a.mode != "polled":
                continue
            while a.events and a.events[0].query():
                a.events.popleft()
            if a.pending:
                st = a.solve.step_poll()
                if st == binding.POLL_RUNNING:
                    continue
                progressed = True
                if st == binding.POLL_PASSES:
                    continue
                a.pending = False          # POLL_STEPPED
                self._stepped(a)
            if a.enqueued < a.req.nsteps and len(a.events) < self.depth:
                a.enqueued += 1
                a.pending = a.solve.step_begin(extra=self.poll_extra)
                if not a.pending:
                    self._stepped(a)
                progressed = True
        return progressed

    def _advance_engine(self) -> bool:
        """A solve whose steps the progress thread has all enqueued gets the
        event its completion waits for."""
        progressed = False
        for a in self.active:
            if a.mode == "engine" and a.pending and not a.solve.async_busy():
                a.pending = False
                self._stepped(a)
                progressed = True
        return progressed

    def _advance(self) -> bool:
        """Enqueue at most one step per active solve, as one grouped call over
        the solves that have room; returns True if any step was enqueued."""
        progressed = self._advance_polled()
        progressed = self._advance_engine() or progressed
        ready = []
        for a in self.active:
            if a.mode != "whole":
                continue
            while a.events and a.events[0].query():
                a.events.popleft()
            if a.enqueued < a.req.nsteps and len(a.events) < self.depth:
                ready.append(a)
        if not ready:
            return progressed
        binding.coarse_grain_batch([a.solve for a in ready], 1)
        for a in ready:
            a.enqueued += 1
            ev = torch.cuda.Event()
            ev.record(a.stream)
            a.events.append(ev)
        return True

    def _complete(self):
        still = []
        for a in self.active:
            if a.enqueued == a.req.nsteps and not a.pending and all(e.query() for e in a.events):
                lnz = a.solve.log_z()          # its stream is idle: returns at once
                st = a.solve.stage_times()[0] if self.timing else None
                r = a.req
                self.done.append(Completed(
                    rid=r.rid, model=r.model, q=r.q, temperature=r.temperature, dmax=r.dmax, nsteps=r.nsteps,
                    precision=self.precision, lnz_per_site=lnz, arrival=r.arrival, admitted=a.admitted,
                    finished=self._now(), footprint=a.footprint,
                    flops=accounting.solve_flops(r.q, r.dmax, r.nsteps), stage_ms=st))
                a.solve.close()
                self.in_use -= a.footprint
                self.free_streams.append(a.slot)
                del a.workspace
            else:
                still.append(a)
        self.active = still

    def run(self, requests, realtime: bool = True, progress=None, horizon: float | None = None) -> list[Completed]:
        """Serve `requests` (objects with rid, arrival, model, q, temperature,
        dmax, nsteps).  realtime: requests become visible at their arrival
        time; otherwise all are queued at once (a closed batch).  horizon:
        stop serving that many seconds after the start; solves still in
        flight are then drained and released without a result, and
        `self.unfinished` holds the (rid, arrival) of every request without
        one (in flight, queued or not yet arrived)."""
        reqs = sorted(requests, key=lambda r: r.arrival)
        self.t0 = time.perf_counter()
        self.unfinished = []
        i = 0
        n_total = len(reqs)
        n_before = len(self.done)
        last_report = 0.0
        while len(self.done) - n_before < n_total:
            now = self._now()
            if horizon is not None and now >= horizon:
                self._abandon(reqs[i:])
                break
            while i < n_total and (not realtime or reqs[i].arrival <= now):
                self.queue.append(reqs[i])
                i += 1
            self._complete()
            self._admit()
            progressed = self._advance()
            if progress and now - last_report >= 5.0:
                progress(now, len(self.done) - n_before, n_total, len(self.active), len(self.queue))
                last_report = now
            if not progressed and self.idle_sleep > 0:
                time.sleep(self.idle_sleep)
        torch.cuda.synchronize(self.device)
        return sorted(self.done[n_before:], key=lambda c: c.rid)

    def _abandon(self, not_arrived):
        """End of a horizon: wait for the enqueued work of the solves in
        flight, release them and forget the queue."""
        torch.cuda.synchronize(self.device)
        for a in self.active:
            self.unfinished.append((a.req.rid, a.req.arrival))
            a.solve.close()
            self.in_use -= a.footprint
            self.free_streams.append(a.slot)
            del a.workspace
        self.active = []
        self.unfinished += [(r.rid, r.arrival) for r in self.queue]
        self.queue.clear()
        self.unfinished += [(r.rid, r.arrival) for r in not_arrived]


def percentile(xs, p):
    xs = sorted(xs)
    if not xs:
        return float("nan")
    k = (len(xs) - 1) * p / 100.0
    lo, hi = int(k), min(int(k) + 1, len(xs) - 1)
    return xs[lo] + (xs[hi] - xs[lo]) * (k - lo)


def summarize(done: list[Completed], wall: float) -> dict:
    lat = [c.latency for c in done]
    flops = sum(c.flops for c in done)
    return {
        "solves": len(done),
        "wall_s": wall,
        "solves_per_s": len(done) / wall if wall > 0 else None,
        "served_tflops": flops / wall / 1e12 if wall > 0 else None,
        "p50_latency_s": percentile(lat, 50),
        "p99_latency_s": percentile(lat, 99),
        "max_latency_s": max(lat) if lat else None,
    }
