"""The continuous-batching scheduler on a virtual clock (no device): admission
order and memory budget, continuous admission while others run, failures,
refusals, and the accounting of time-to-solution."""
import math

import numpy as np
import pytest

import workloads as W
from conftest import ensure_library

ensure_library()
from paper_2009_13426_amd import serve as S  # noqa: E402


def reqs(specs):
    return [S.Request(i, t, n, n, k, None) for i, (t, n, k) in enumerate(specs)]


def replay_memory(engine, requests, budget):
    """Footprint in use after every start/release in the engine log."""
    size = {r.job_id: engine.footprint(r) for r in requests}
    used, trace = 0, []
    for ev in engine.log:
        if ev[0] == "start":
            used += size[ev[1]]
        elif ev[0] == "release":
            used -= size[ev[1]]
        trace.append(used)
    return trace


def test_every_job_runs_its_steps_once():
    rq = reqs([(0.0, 64, 100), (0.0, 128, 300), (0.01, 96, 50), (0.5, 64, 1000)])
    eng = S.FakeEngine()
    rep = S.serve(rq, eng, memory_budget=10**12, quantum=40)
    steps_run = {r.job_id: 0 for r in rq}
    for ev in eng.log:
        if ev[0] == "run":
            for j, k in zip(ev[1], ev[2]):
                steps_run[j] += k
    assert steps_run == {r.job_id: r.steps for r in rq}
    assert [r.job_id for r in rep.results] == [0, 1, 2, 3]
    assert all(r.status == 0 and r.finished >= r.admitted >= r.arrival for r in rep.results)


def test_admission_is_fifo_and_within_budget():
    rq = reqs([(0.001 * i, 64 + 32 * (i % 5), 200) for i in range(30)])
    eng = S.FakeEngine(bytes_per_node=400)
    budget = 400 * (3 * 128 * 128)
    rep = S.serve(rq, eng, memory_budget=budget, quantum=25)
    starts = [ev[1] for ev in eng.log if ev[0] == "start"]
    assert starts == sorted(starts)           # arrival order, no overtaking
    assert max(replay_memory(eng, rq, budget)) <= budget
    assert rep.peak_bytes <= budget
    assert len(rep.results) == 30 and all(r.status == 0 for r in rep.results)


def test_arrivals_join_a_running_batch():
    # job 1 arrives while job 0 (long) runs: it must be admitted before job 0 ends
    rq = reqs([(0.0, 256, 2000), (0.002, 64, 100)])
    eng = S.FakeEngine(rate_nodes_per_s=1e9)
    rep = S.serve(rq, eng, memory_budget=10**12, quantum=20)
    r0, r1 = rep.results
    assert r1.admitted < r0.finished
    assert r1.finished < r0.finished
    mixed = [ev for ev in eng.log if ev[0] == "run" and set(ev[1]) == {0, 1}]
    assert mixed, "the two jobs never shared a batched call"


def test_oversized_request_is_refused_and_others_served():
    rq = reqs([(0.0, 64, 10), (0.0, 4096, 10), (0.0, 64, 10)])
    eng = S.FakeEngine(bytes_per_node=400)
    rep = S.serve(rq, eng, memory_budget=400 * 200 * 200, quantum=5)
    st = {r.job_id: r.status for r in rep.results}
    assert st == {0: 0, 1: -2, 2: 0}


def test_failed_job_is_retired_and_the_rest_continue():
    rq = reqs([(0.0, 64, 100), (0.0, 64, 100), (0.0, 64, 100)])
    eng = S.FakeEngine(fail=[1])
    rep = S.serve(rq, eng, memory_budget=10**12, quantum=30)
    st = {r.job_id: r.status for r in rep.results}
    assert st[1] != 0 and st[0] == 0 and st[2] == 0
    s = rep.summary()
    assert s["failed"] == 1 and s["jobs"] == 3


def test_percentiles_and_throughput_accounting():
    res = [S.Result(i, 0.0, 0.0, float(i + 1), 100, 10) for i in range(100)]
    rep = S.Report(res, makespan=100.0, peak_bytes=0, quanta=1)
    s = rep.summary()
    assert s["p50_s"] == pytest.approx(np.percentile(np.arange(1, 101), 50))
    assert s["p99_s"] == pytest.approx(np.percentile(np.arange(1, 101), 99))
    assert s["mlups"] == pytest.approx(100 * 100 * 10 / 100.0 / 1e6)


def test_one_at_a_time_path_is_sequential():
    rq = reqs([(0.0, 64, 100), (0.0, 64, 100), (0.3, 64, 100)])
    eng = S.FakeEngine()
    rep = S.serve_one_at_a_time(rq, eng)
    r = rep.results
    assert r[1].admitted >= r[0].finished and r[2].admitted >= max(r[1].finished, 0.3)


def test_batching_beats_one_at_a_time_on_small_jobs():
    # launch-bound small grids: one launch pair per step for all jobs vs per job
    specs = W.serving_jobs(40)
    small = [S.Request(i, 0.0, 64, 64, 400, None) for i in range(40)]
    b = S.serve(small, S.FakeEngine(), memory_budget=10**12, quantum=50).summary()
    a = S.serve_one_at_a_time(small, S.FakeEngine()).summary()
    assert b["makespan_s"] < a["makespan_s"]
    assert b["p50_s"] < a["p50_s"]
    assert len(specs) == 40


def test_requests_from_specs_arrival_times():
    specs = W.serving_jobs(20)
    rq = S.requests_from_specs(specs, rate=10.0)
    gaps = np.diff([0.0] + [r.arrival for r in rq])
    assert np.allclose(gaps, [sp.interarrival / 10.0 for sp in specs])
    rq0 = S.requests_from_specs(specs, rate=math.inf)
    assert all(r.arrival == 0.0 for r in rq0)
    assert all(r.nx == sp.side and r.steps == sp.steps for r, sp in zip(rq, specs))


def test_batch_statuses_only_numerical_failures_fall_back():
    """A job's own numerical failure (LBM_ERR_NEWTON -5, NONPHYSICAL -6)
    gives each job its status; any other error of the batched call (bad
    argument -1, HIP -3, out of order -4) stops the server instead of
    retiring every job as if it had advanced."""
    own = {0: 0, 1: -5, 2: 0}
    assert S.batch_statuses(0, 3, own.__getitem__) == [0, 0, 0]
    assert S.batch_statuses(-5, 3, own.__getitem__) == [0, -5, 0]
    assert S.batch_statuses(-6, 3, own.__getitem__) == [0, -5, 0]
    for st in (-1, -2, -3, -4):
        with pytest.raises(S.BatchError):
            S.batch_statuses(st, 3, own.__getitem__)


class _LimitEngine(S.FakeEngine):
    max_batch = 4


def test_batch_never_exceeds_the_engines_limit():
    rq = reqs([(0.0, 64, 100) for _ in range(10)])
    eng = _LimitEngine()
    rep = S.serve(rq, eng, memory_budget=10**12, quantum=50, max_batch=1024)
    sizes = [len(ev[1]) for ev in eng.log if ev[0] == "run"]
    assert max(sizes) == 4
    assert len(rep.results) == 10 and all(r.status == 0 for r in rep.results)
