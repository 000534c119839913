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
        """p50/p99/mean time-to-solution over the jobs that completed, and
        p50_all/p99_all over every job, a failed one counted at the time its
        failure was reported (its time to a final answer)."""
        ok = [r for r in self.results if r.status == 0]
        tts = np.array([r.time_to_solution for r in ok]) if ok else np.zeros(1)
        tall = np.array([r.time_to_solution for r in self.results]) if self.results \
            else np.zeros(1)
        work = sum(r.nodes * r.steps for r in ok)
        return dict(jobs=len(self.results), failed=len(self.results) - len(ok),
                    p50_s=float(np.percentile(tts, 50)), p99_s=float(np.percentile(tts, 99)),
                    p50_all_s=float(np.percentile(tall, 50)),
                    p99_all_s=float(np.percentile(tall, 99)),
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
    refused (status -2 in its result).  The batch never holds more jobs than
    the engine takes in one call (engine.max_batch)."""
    max_batch = min(max_batch, getattr(engine, "max_batch", max_batch))
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
# Statuses of a job that stopped on its own numbers (a failed equilibrium
# solve, a non-physical state): the job fails, the batch goes on.
NUMERICAL_FAILURES = (-5, -6)  # lbm_status LBM_ERR_NEWTON, LBM_ERR_NONPHYSICAL


class BatchError(RuntimeError):
    """A batched call failed for a reason other than a job's numerics (bad
    argument, HIP error, call out of order): no job can be trusted to have
    advanced, so the server stops instead of retiring them as done."""

    def __init__(self, status: int):
        super().__init__(f"batched step failed with status {status}")
        self.status = status


def batch_statuses(status: int, n: int, job_status: Callable[[int], int]) -> List[int]:
    """Per-job statuses after a batched call that returned `status`: all 0
    on success; on a numerical failure, each job's own status (job_status(k)
    reads job k's device error word); any other status raises BatchError."""
    if status == 0:
        return [0] * n
    if status in NUMERICAL_FAILURES:
        return [int(job_status(k)) for k in range(n)]
    raise BatchError(status)


class GpuEngine:
    """Jobs as `Sim` contexts on one device and one stream; batched steps
    through `lbm_step_batched`.  Every context copies the initial-guess table
    of one template context instead of building its own.

    schedule "auto": the batched launches use the autotuner's batched-step
    schedule and the one-job-at-a-time path each job's size-class schedule
    (both from the cache; `prepare` tunes the missing ones before serving,
    so that tuning never falls in served time).  None: library defaults."""

    def __init__(self, precision: str = "fp32", device=None, schedule: Optional[str] = None,
                 graph: bool = False):
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
        self.graph = graph          # quanta as replays of a HIP graph (lbm_step_batched_graph)
        self.graph_builds = self.graph_replays = 0
        # jobs that took the fallback equilibrium (lbm_config.fallback), and
        # the collisions and rebuilt links that did, over released jobs
        self.fallback_jobs = self.fallback_solves = 0

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

    max_batch = 1024  # contexts per lbm_step_batched call

    def run(self, sims, steps) -> List[int]:
        import ctypes as C
        n = len(sims)
        arr = (C.c_void_p * n)(*[s.handle.value for s in sims])
        ks = (C.c_int32 * n)(*[int(k) for k in steps])
        if self.graph:
            built = C.c_int32(0)
            st = self.lib.lbm_step_batched_graph(arr, ks, n, C.byref(built))
            if st == 0:
                self.graph_builds += built.value
                self.graph_replays += 1 - built.value
        else:
            st = self.lib.lbm_step_batched(arr, ks, n)
        return batch_statuses(int(st), n, lambda k: self.lib.lbm_sync(sims[k].handle))

    def run_alone(self, sim, steps: int) -> int:
        if self.auto:
            from . import autotune
            sched = autotune.schedule_for(self.precision, sim.nx, sim.ny, tune_missing=False)
            if sched:
                sim.schedule = sched
        return int(self.lib.lbm_step(sim.handle, int(steps)))

    def release(self, sim):
        if sim.cfg.fallback:
            k = sim.diag()["fallback_solves"]
            self.fallback_jobs += int(k > 0)
            self.fallback_solves += k
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


class Prefetcher:
    """Draws the jobs' initial fields ahead of their arrivals on a host
    thread, in arrival order, at most `ahead` jobs in advance (a client that
    has its fields ready when it submits); `make(k)` blocks until job k's
    fields are drawn."""

    def __init__(self, specs, ahead: int = 256):
        import threading
        self.specs = list(specs)
        self.ready: Dict[int, object] = {}
        self.cv = threading.Condition()
        self.next = 0
        self.ahead = ahead
        self.taken = 0
        self.thread = threading.Thread(target=self._run, daemon=True)
        self.thread.start()

    def _run(self):
        for k, sp in enumerate(self.specs):
            with self.cv:
                while k - self.taken >= self.ahead:
                    self.cv.wait()
            wl = sp.build()
            with self.cv:
                self.ready[k] = wl
                self.cv.notify_all()

    def make(self, k: int):
        with self.cv:
            while k not in self.ready:
                self.cv.wait()
            wl = self.ready.pop(k)
            self.taken = max(self.taken, k + 1)
            self.cv.notify_all()
        return wl


def requests_prefetched(specs, rate: float, ahead: int = 256) -> List[Request]:
    """As requests_from_specs, with the fields drawn ahead by a Prefetcher."""
    pf = Prefetcher(specs, ahead)
    out, t = [], 0.0
    for k, sp in enumerate(specs):
        if math.isfinite(rate):
            t += sp.interarrival / rate
        out.append(Request(sp.job_id, t if math.isfinite(rate) else 0.0, sp.side, sp.side,
                           sp.steps, (lambda k=k: pf.make(k))))
    return out


def main(argv=None):
    """The seeded serving mix through the batched server: capacity with the
    first --capacity-jobs jobs queued at t = 0, then --jobs Poisson arrivals
    at --load times that capacity.  Prints progress and one JSON summary.

      python -m paper_2009_13426_amd.serve --jobs 10000 --capacity-jobs 2000
    """
    import argparse
    import json
    import os
    import sys
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=10000)
    ap.add_argument("--capacity-jobs", type=int, default=2000)
    ap.add_argument("--load", type=float, default=0.8)
    ap.add_argument("--quantum", type=int, default=50)
    ap.add_argument("--precision", default="fp32")
    ap.add_argument("--budget-frac", type=float, default=0.6)
    ap.add_argument("--graph", action="store_true",
                    help="quanta as replays of a HIP graph (lbm_step_batched_graph)")
    ap.add_argument("--out", default="")
    args = ap.parse_args(argv)
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    if root not in sys.path:
        sys.path.insert(0, root)
    import torch
    import workloads as W
    from . import autotune
    torch.cuda.set_device(0)
    specs = W.serving_jobs(args.jobs)
    eng = GpuEngine(precision=args.precision, graph=args.graph)
    eng.batch_schedule = autotune.batched_schedule_for(args.precision, device=eng.device)
    free, _ = torch.cuda.mem_get_info()
    budget = int(args.budget_frac * free)
    t0 = time.time()

    def progress(tag, total):
        done = [0]

        def on_finish(req, handle):
            done[0] += 1
            if done[0] % 250 == 0 or done[0] == total:
                print(f"[serve] {tag}: {done[0]}/{total} jobs done, {time.time() - t0:.0f} s",
                      flush=True)
        return on_finish

    cap_specs = specs[:args.capacity_jobs]
    cap = serve(requests_prefetched(cap_specs, math.inf), eng, budget, args.quantum,
                on_finish=progress("capacity", len(cap_specs))).summary()
    rate = args.load * cap["jobs_per_s"]
    print(f"[serve] capacity {cap['jobs_per_s']:.2f} jobs/s on {len(cap_specs)} jobs; "
          f"arrivals at {rate:.2f} jobs/s", flush=True)
    eng.fallback_jobs = eng.fallback_solves = 0
    rep = serve(requests_prefetched(specs, rate), eng, budget, args.quantum,
                on_finish=progress("trace", len(specs)))
    summ = rep.summary()
    failed = [dict(job=r.job_id, status=r.status) for r in rep.results if r.status != 0]
    out = dict(jobs=args.jobs, capacity_jobs=args.capacity_jobs,
               capacity_jobs_per_s=cap["jobs_per_s"], capacity_mlups=cap["mlups"],
               load=args.load, rate_jobs_per_s=rate, quantum=args.quantum,
               precision=args.precision, memory_budget_bytes=budget,
               batched_schedule=eng.batch_schedule, summary=summ, failed_jobs=failed,
               fallback_jobs=eng.fallback_jobs, fallback_solves=eng.fallback_solves,
               graph=args.graph, graph_builds=eng.graph_builds,
               graph_replays=eng.graph_replays, wall_s=time.time() - t0)
    line = json.dumps(out)
    print(line, flush=True)
    if args.out:
        with open(args.out, "w") as f:
            f.write(line + "\n")


if __name__ == "__main__":
    main()
