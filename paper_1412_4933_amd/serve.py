"""Serving form: continuous batching of independent scenarios on one GPU.

Requests (a scenario plus a step count) arrive over time. The server keeps a
batch of resident scenarios on the device and repeats:
  1. admit   queued requests in arrival order while a batch slot is free and
             the resident state fits the HBM budget (planes + scratch); a new
             request's planes are uploaded and validated on a side stream
             while the previous quantum is still running;
  2. advance every resident scenario by min(quantum, its remaining steps)
             in shared launches of the batch kernel;
  3. harvest scenarios that finished: their counters (and optionally final
             planes) are read, their slot and memory are released.
Latency of a request = completion time - arrival time. Every scenario's
result is bit-identical to running it alone (the random words depend only on
the scenario's seed, step and agent number).
"""
from __future__ import annotations

import dataclasses
import heapq
import time
from typing import Callable, List, Optional

import numpy as np

from . import pedsim, scenarios


@dataclasses.dataclass
class Request:
    rid: int
    arrival: float          # seconds after the start of the run
    steps: int
    build: Callable[[], "scenarios.Scenario"]  # makes the initial state on the host
    nbytes: int             # device bytes the request holds while resident
    agents: int
    scenario: Optional["scenarios.Scenario"] = None  # the initial state, when it came with the request
    mode: Optional[int] = None  # SIM_MODE_* of the scenario (None: read from its initial state)


@dataclasses.dataclass
class Result:
    rid: int
    arrival: float
    admitted: float
    finished: float
    steps: int
    agents: int
    stats: dict
    state: Optional[tuple] = None  # (code, ids, tau) with keep_state
    tour: Optional[np.ndarray] = None  # tour matrix of a tour-variant request, with keep_state

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


def resident_bytes(W: int, H: int, mode: int, agents: int = 0) -> int:
    """Device bytes one scenario holds: code + id planes, pheromone planes
    (ACO and the tour variant), the tour matrix and its ping-pong half (tour
    variant, 4 B each per agent), and the library's scratch."""
    p = pedsim.SimParams(W, H, 0, 0, 0.1, 1.0, 1, 2, 0, 0)
    aco = mode in (scenarios.MODE_ACO, scenarios.MODE_ACO_TOUR)
    tour = 8 * agents if mode == scenarios.MODE_ACO_TOUR else 0
    return W * H * (1 + 4 + (8 if aco else 0)) + tour + pedsim.sim_scratch_bytes(p)


def prebuild(requests: List[Request]) -> None:
    """Attach each request's initial state (host arrays), as a request that
    arrives with its payload; the serving loop then only uploads it."""
    for r in requests:
        if r.scenario is None:
            r.scenario = r.build()


def _initial_state(req: Request) -> "scenarios.Scenario":
    return req.scenario if req.scenario is not None else req.build()


def _request_mode(req: Request) -> int:
    return req.mode if req.mode is not None else _initial_state(req).mode


def poisson_requests(specs, rate: float, seed: int = 0) -> List[Request]:
    """specs: (W, H, N, band, mode, steps, seed) tuples; arrivals of a Poisson
    process with `rate` requests per second."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for rid, (W, H, N, band, mode, steps, sseed) in enumerate(specs):
        t += float(rng.exponential(1.0 / rate))

        def build(W=W, H=H, N=N, band=band, mode=mode, sseed=sseed):
            return scenarios.make_scenario(W, H, N // 2, N - N // 2, band_a=band, seed=sseed, mode=mode)

        out.append(Request(rid, t, steps, build, resident_bytes(W, H, mode, N), N, mode=mode))
    return out


class Server:
    def __init__(self, capacity: int = 256, budget_bytes: int = 2 << 30, quantum: int = 200,
                 device: str = "cuda", keep_state: bool = False, tuning=None):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.stream = torch.cuda.Stream(self.device)
        self.side = torch.cuda.Stream(self.device)
        self.batch = pedsim.Batch(capacity, device=device, stream=self.stream)
        self.tuning = tuning
        if tuning is not None:
            self.batch.set_tuning(*tuning)
        self.capacity = capacity
        self.budget = budget_bytes
        self.quantum = quantum
        self.keep_state = keep_state
        self.used = 0
        self.live = {}  # slot -> [request, remaining, admitted_time]

    def _admit(self, req: Request, now: float) -> None:
        scn = _initial_state(req)
        with self.torch.cuda.stream(self.side):
            res = pedsim._Resident(scn, self.device)
        self.side.synchronize()
        slot = pedsim.sim_batch_add(self.batch.b, res.params, scn.mode, res.code, res.ids, res.tau,
                                    res.scratch, res.scratch_bytes, self.side)
        if res.tour is not None and res.tour.numel():
            pedsim.sim_batch_attach_tour(self.batch.b, slot, res.tour, res.tour_shadow, self.side)
        self.batch.members[slot] = res
        self.live[slot] = [req, req.steps, now]
        self.used += req.nbytes

    def run(self, requests: List[Request], clock=time.perf_counter) -> List[Result]:
        if self.tuning is None and not self.live and any(
                _request_mode(r) == scenarios.MODE_ACO_TOUR for r in requests):
            # tour-variant scenarios run on the batch's LDS form only
            self.batch.set_tuning(*pedsim.LDS_BATCH_TUNING)
        pending = sorted(requests, key=lambda r: r.arrival)
        queue: List[Request] = []
        results: List[Result] = []
        t0 = clock()
        i = 0
        while i < len(pending) or queue or self.live:
            now = clock() - t0
            while i < len(pending) and pending[i].arrival <= now:
                queue.append(pending[i])
                i += 1
            if not self.live and not queue:  # idle until the next arrival
                time.sleep(max(0.0, pending[i].arrival - now))
                continue
            # advance the resident scenarios by one quantum (asynchronous)
            steps = [0] * self.capacity
            for slot, (req, remaining, _) in self.live.items():
                steps[slot] = min(self.quantum, remaining)
            if any(steps):
                pedsim.sim_batch_step_slots(self.batch.b, steps, self.stream)
            # admit arrivals while the quantum runs
            while queue and len(self.live) < self.capacity and self.used + queue[0].nbytes <= self.budget:
                req = queue.pop(0)
                if req.nbytes > self.budget:
                    raise ValueError(f"request {req.rid} alone exceeds the memory budget")
                self._admit(req, clock() - t0)
            self.stream.synchronize()
            done_time = clock() - t0
            for slot, k in enumerate(steps):
                if k == 0 or slot not in self.live:
                    continue
                entry = self.live[slot]
                entry[1] -= k
                if entry[1] == 0:
                    req = entry[0]
                    stats = pedsim.sim_batch_stats(self.batch.b, slot, self.stream)
                    res = self.batch.members[slot]
                    state = res.state() if self.keep_state else None
                    tour = res.tour.cpu().numpy() if self.keep_state and res.tour is not None else None
                    results.append(Result(req.rid, req.arrival, entry[2], done_time, req.steps, req.agents,
                                          stats, state, tour))
                    self.batch.remove(slot)
                    del self.live[slot]
                    self.used -= req.nbytes
            if queue and not self.live and self.used == 0 and queue[0].nbytes > self.budget:
                raise ValueError(f"request {queue[0].rid} alone exceeds the memory budget")
        return results

    def close(self) -> None:
        self.batch.close()


def summarize(results: List[Result], wall: float) -> dict:
    lat = np.array([r.latency for r in results])
    work = sum(r.agents * r.steps for r in results)
    return {"requests": len(results), "p50_latency_s": float(np.percentile(lat, 50)),
            "p99_latency_s": float(np.percentile(lat, 99)), "mean_latency_s": float(lat.mean()),
            "agent_steps": work, "wall_s": wall, "agent_steps_per_s": work / wall}


def run_back_to_back(requests: List[Request], device: str = "cuda", clock=time.perf_counter) -> dict:
    """The same requests, one after another through the plain single-scenario
    path (upload, create, run, read counters, release)."""
    import torch
    stream = torch.cuda.Stream(torch.device(device))
    work = 0
    t0 = clock()
    for req in sorted(requests, key=lambda r: r.arrival):
        scn = _initial_state(req)
        sim = pedsim.Sim(scn, device=device, stream=stream)
        sim.step(req.steps)
        sim.stats()
        sim.close()
        work += req.agents * req.steps
    wall = clock() - t0
    return {"requests": len(requests), "agent_steps": work, "wall_s": wall, "agent_steps_per_s": work / wall}
