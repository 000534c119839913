"""Continuous-batching job server for many independent simulations.

Requests (a grid and a number of steps each) arrive over time.  The server
keeps every admitted job's populations resident on the device, admits new
arrivals between quanta as long as their device footprint fits the memory
budget and a batch slot is free, and advances all admitted jobs together,
one batched launch pair per step (`lbm_step_batched`), a quantum of steps at
a time.  A job finishing leaves the batch at the next quantum boundary and
frees its memory for the queue.

The scheduler only talks to an engine object, so the same loop runs on the
GPU (`GpuEngine`) and on a virtual clock with a cost model (`FakeEngine`),
which is how its admission, ordering and accounting are tested without a
device.  `serve_one_at_a_time` is the plain single-job path on the same
arrivals, for comparison.

Times are seconds on the engine's clock; time-to-solution is completion
minus arrival.
"""
from __future__ import annotations

import collections
import dataclasses
import math
import time
from typing import Callable, Dict, List, Optional, Sequence

import numpy as np


@dataclasses.dataclass
class Request:
    job_id: int
    arrival: float          # seconds on the engine clock
    nx: int
    ny: int
    steps: int
    make: Callable          # () -> workloads.Workload with the initial state


@dataclasses.dataclass
class Result:
    job_id: int
    arrival: float
    admitted: float
    finished: float
    nodes: int
    steps: int
    status: int = 0         # 0, or the lbm_status that stopped the job

    @property
    def time_to_solution(self) -> float:
        return self.finished - self.arrival


@dataclasses.dataclass
class Report:
    results: List[Result]
    makespan: float
    peak_bytes: int
    quanta: int

    def summary(self) -> Dict:
        ok = [r for r in self.results if r.status == 0]
        tts = np.array([r.time_to_solution for r in ok]) if ok else np.zeros(1)
        work = sum(r.nodes * r.steps for r in ok)
        return dict(jobs=len(self.results), failed=len(self.results) - len(ok),
                    p50_s=float(np.percentile(tts, 50)), p99_s=float(np.percentile(tts, 99)),
                    mean_s=float(tts.mean()),
                    mean_wait_s=float(np.mean([r.admitted - r.arrival for r in ok])) if ok else 0.0,
                    makespan_s=self.makespan,
                    mlups=work / self.makespan / 1e6 if self.makespan > 0 else 0.0,
                    jobs_per_s=len(ok) / self.makespan if self.makespan > 0 else 0.0,
                    peak_bytes=self.peak_bytes, quanta=self.quanta)


# --------------------------------------------------------------- scheduler
def serve(requests: Sequence[Request], engine, memory_budget: int, quantum: int = 50,
          max_batch: int = 1024, on_finish: Optional[Callable] = None) -> Report:
    """Continuous batching.  Between quanta: admit, in arrival order, every
    arrived request whose footprint fits what is left of memory_budget (a
    request that does not fit waits, and so do the ones behind it: no
    overtaking); then advance every admitted job by min(quantum, steps left)
    steps in one batched call.  A request larger than the whole budget is
    refused (status -2 in its result)."""
    pending = collections.deque(sorted(requests, key=lambda r: (r.arrival, r.job_id)))
    active: List[Dict] = []
    results: List[Result] = []
    used = peak = 0
    quanta = 0
    t0 = engine.now()
    while pending or active:
        now = engine.now() - t0
        while pending and pending[0].arrival <= now and len(active) < max_batch:
            req = pending[0]
            need = engine.footprint(req)
            if need > memory_budget:
                pending.popleft()
                results.append(Result(req.job_id, req.arrival, now, now, req.nx * req.ny, 0, -2))
                continue
            if used + need > memory_budget:
                break
            pending.popleft()
            handle = engine.start(req)
            used += need
            peak = max(peak, used)
            active.append(dict(req=req, handle=handle, left=req.steps, need=need,
                               admitted=engine.now() - t0))
        if not active:
            if pending:
                engine.wait_until(t0 + pending[0].arrival)
            continue
        steps = [min(quantum, a["left"]) for a in active]
        statuses = engine.run([a["handle"] for a in active], steps)
        quanta += 1
        now = engine.now() - t0
        still = []
        for a, k, st in zip(active, steps, statuses):
            a["left"] -= k
            if a["left"] == 0 or st != 0:
                req = a["req"]
                if on_finish is not None and st == 0:
                    on_finish(req, a["handle"])
                results.append(Result(req.job_id, req.arrival, a["admitted"], now,
                                      req.nx * req.ny, req.steps, st))
                engine.release(a["handle"])
                used -= a["need"]
            else:
                still.append(a)
        active = still
    return Report(sorted(results, key=lambda r: r.job_id), engine.now() - t0, peak, quanta)


def serve_one_at_a_time(requests: Sequence[Request], engine,
                        on_finish: Optional[Callable] = None) -> Report:
    """The plain path: one job at a time in arrival order, each run to the
    end with the single-context step call."""
    results = []
    t0 = engine.now()
    peak = 0
    for req in sorted(requests, key=lambda r: (r.arrival, r.job_id)):
        now = engine.now() - t0
        if now < req.arrival:
            engine.wait_until(t0 + req.arrival)
        admitted = engine.now() - t0
        handle = engine.start(req)
        peak = max(peak, engine.footprint(req))
        st = engine.run_alone(handle, req.steps)
        if on_finish is not None and st == 0:
            on_finish(req, handle)
        results.append(Result(req.job_id, req.arrival, admitted, engine.now() - t0,
                              req.nx * req.ny, req.steps, st))
        engine.release(handle)
    return Report(results, engine.now() - t0, peak, len(results))


# ----------------------------------------------------------------- engines
class GpuEngine:
    """Jobs as `Sim` contexts on one device and one stream; batched steps
    through `lbm_step_batched`.  Every context copies the initial-guess table
    of one template context instead of building its own.

    schedule "auto": the batched launches use the autotuner's batched-step
    schedule and the one-job-at-a-time path each job's size-class schedule
    (both from the cache; `prepare` tunes the missing ones before serving,
    so that tuning never falls in served time).  None: library defaults."""

    def __init__(self, precision: str = "fp32", device=None, schedule: Optional[str] = None):
        import torch
        from . import Sim, lib, make_config, workspace_bytes, _check
        self.torch = torch
        self.Sim, self.lib, self._check = Sim, lib, _check
        self.make_config, self.workspace_bytes = make_config, workspace_bytes
        self.precision = precision
        self.device = torch.device("cuda" if device is None else device)
        self.stream = torch.cuda.current_stream(self.device)
        self.template = Sim(8, 8, device=self.device, stream=self.stream, precision=precision)
        self.auto = schedule == "auto"
        self.batch_schedule = None

    def prepare(self, requests: Sequence[Request]):
        """Tunes (or reads from the cache) every schedule the requests need."""
        if not self.auto:
            return
        from . import autotune
        self.batch_schedule = autotune.batched_schedule_for(self.precision, device=self.device)
        for key in sorted({(r.nx, r.ny) for r in requests}):
            autotune.schedule_for(self.precision, *key, device=self.device)

    def now(self) -> float:
        return time.perf_counter()

    def wait_until(self, t: float):
        d = t - time.perf_counter()
        if d > 0:
            time.sleep(d)

    def footprint(self, req: Request) -> int:
        """Workspace bytes plus the FP64 initial fields held during init."""
        cfg = self.make_config(req.nx, req.ny, precision=self.precision)
        return self.workspace_bytes(cfg) + 4 * 8 * req.nx * req.ny

    def start(self, req: Request):
        sim = self.Sim.from_workload(req.make(), precision=self.precision, device=self.device,
                                     stream=self.stream, like=self.template)
        if self.batch_schedule:
            sim.schedule = self.batch_schedule
        return sim

    def run(self, sims, steps) -> List[int]:
        import ctypes as C
        n = len(sims)
        arr = (C.c_void_p * n)(*[s.handle.value for s in sims])
        ks = (C.c_int32 * n)(*[int(k) for k in steps])
        st = self.lib.lbm_step_batched(arr, ks, n)
        if st == 0:
            return [0] * n
        return [int(self.lib.lbm_sync(s.handle)) for s in sims]

    def run_alone(self, sim, steps: int) -> int:
        if self.auto:
            from . import autotune
            sched = autotune.schedule_for(self.precision, sim.nx, sim.ny, tune_missing=False)
            if sched:
                sim.schedule = sched
        return int(self.lib.lbm_step(sim.handle, int(steps)))

    def release(self, sim):
        sim.close()
        sim.workspace = None


class FakeEngine:
    """Virtual clock and a cost model: a batched quantum costs a fixed launch
    overhead per step plus the node updates at a fixed rate; nothing runs."""

    def __init__(self, rate_nodes_per_s: float = 5e9, launch_s: float = 20e-6,
                 start_s: float = 1e-3, bytes_per_node: int = 400, fail: Sequence[int] = ()):
        self.t = 0.0
        self.rate, self.launch, self.start_cost = rate_nodes_per_s, launch_s, start_s
        self.bpn = bytes_per_node
        self.fail = set(fail)
        self.log: List = []

    def now(self) -> float:
        return self.t

    def wait_until(self, t: float):
        self.t = max(self.t, t)

    def footprint(self, req: Request) -> int:
        return self.bpn * req.nx * req.ny

    def start(self, req: Request):
        self.t += self.start_cost
        self.log.append(("start", req.job_id, self.t))
        return req

    def run(self, reqs, steps) -> List[int]:
        most = max(steps)
        work = sum(r.nx * r.ny * k for r, k in zip(reqs, steps))
        self.t += most * 2 * self.launch + work / self.rate
        self.log.append(("run", tuple(r.job_id for r in reqs), tuple(steps), self.t))
        return [1 if r.job_id in self.fail else 0 for r in reqs]

    def run_alone(self, req, steps: int) -> int:
        self.t += steps * 2 * self.launch + req.nx * req.ny * steps / self.rate
        return 1 if req.job_id in self.fail else 0

    def release(self, req):
        self.log.append(("release", req.job_id, self.t))


# --------------------------------------------------------------- workloads
def requests_from_specs(specs, rate: float, prebuild: bool = False) -> List[Request]:
    """Requests for job specs (workloads.JobSpec): arrival times are the
    cumulative unit-rate gaps divided by `rate` (jobs per second); rate
    math.inf puts every arrival at 0.  With prebuild, each request carries
    its initial fields already drawn (as a client would send them), so that
    drawing them is not part of the served time."""
    out, t = [], 0.0
    for sp in specs:
        if math.isfinite(rate):
            t += sp.interarrival / rate
        make = sp.build
        if prebuild:
            wl = sp.build()
            make = (lambda w=wl: w)
        out.append(Request(sp.job_id, t if math.isfinite(rate) else 0.0, sp.side, sp.side,
                           sp.steps, make))
    return out
