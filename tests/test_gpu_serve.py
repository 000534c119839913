"""The job server on the GPU: jobs that arrive while others run are admitted
into the running batch, and every job's result is the same in the mix as
alone (bitwise: the batched launches run the same per-node code on the same
inputs)."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def serve():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2009_13426_amd import serve
    return serve


def small_mix():
    """Vortex and quadrant jobs of uneven sides and step counts, arriving
    over ~40 ms so that later ones join a running batch."""
    specs = []
    sides = [48, 80, 64, 96, 56, 72]
    steps = [60, 25, 90, 40, 70, 30]
    for j, (n, k) in enumerate(zip(sides, steps)):
        kind = "vortex" if j % 2 == 0 else "quadrant"
        specs.append(W.JobSpec(j, kind, n, 1.0 + 0.3 * j, k, 1.0))
    return specs


def macros_of(sim):
    m = sim.macros()
    return {k: v.cpu().numpy() for k, v in m.items()}


@pytest.mark.parametrize("precision,schedule", [("fp32", None), ("fp64", None), ("fp32", "auto")])
def test_mix_equals_alone(serve, precision, schedule, tmp_path, monkeypatch):
    import paper_2009_13426_amd as lbm
    from paper_2009_13426_amd import autotune
    monkeypatch.setenv(autotune.CACHE_ENV, str(tmp_path / "schedules.json"))
    specs = small_mix()
    reqs = serve.requests_from_specs(specs, rate=150.0)
    eng = serve.GpuEngine(precision=precision, schedule=schedule)
    eng.prepare(reqs)
    if schedule:
        print("batched schedule", eng.batch_schedule, flush=True)
    got = {}
    rep = serve.serve(reqs, eng, memory_budget=1 << 34, quantum=10,
                      on_finish=lambda req, sim: got.__setitem__(req.job_id, macros_of(sim)))
    s = rep.summary()
    print(f"{precision}: {s['jobs']} jobs, {s['quanta']} quanta, p50 {s['p50_s'] * 1e3:.1f} ms, "
          f"p99 {s['p99_s'] * 1e3:.1f} ms, failed {s['failed']}", flush=True)
    assert s["failed"] == 0
    assert sorted(got) == [sp.job_id for sp in specs]
    for sp in specs:
        sim = lbm.Sim.from_workload(sp.build(), precision=precision)
        sim.step(sp.steps)
        alone = macros_of(sim)
        sim.close()
        for k in ("rho", "ux", "uy", "T", "Ux", "Uy"):
            assert np.array_equal(alone[k], got[sp.job_id][k]), (sp.job_id, k)


def test_late_arrivals_join_the_running_batch(serve):
    # job 1 arrives just after job 0 started; with a small quantum it must be
    # admitted while job 0 still runs, and finish first (it is much shorter)
    specs = [W.JobSpec(0, "quadrant", 256, 1.5, 400, 0.0),
             W.JobSpec(1, "vortex", 64, 1.0, 20, 0.0)]
    reqs = serve.requests_from_specs(specs, rate=1e9)
    reqs[1].arrival = 0.005
    eng = serve.GpuEngine(precision="fp32")
    rep = serve.serve(reqs, eng, memory_budget=1 << 34, quantum=5)
    r0, r1 = rep.results
    print(f"job0 admitted {r0.admitted * 1e3:.1f} ms finished {r0.finished * 1e3:.1f} ms; "
          f"job1 admitted {r1.admitted * 1e3:.1f} ms finished {r1.finished * 1e3:.1f} ms", flush=True)
    assert r0.status == 0 and r1.status == 0
    assert r1.admitted < r0.finished and r1.finished < r0.finished


def test_many_jobs_in_one_batch_equal_alone(serve):
    """A batch of up to 300 small jobs (more than one job per thread in the
    batched rebuild's block-wide scan of the jobs' receiver chunks), of
    uneven sides and step counts, some on one fixed lattice (no rebuilt
    links) and some finishing before others: every job's fields after the
    batch equal the job run alone, bit for bit.  Draws whose flow leaves the
    equilibrium's envelope when run alone (a few small quadrant grids) are
    left out of the batch."""
    import paper_2009_13426_amd as lbm
    rng = np.random.Generator(np.random.PCG64(23))
    jobs, alone = [], []
    for j in range(300):
        n = int(rng.integers(8, 40))
        if j % 7 == 3:
            wl = W.uniform(n, n, 1.0, 0.4, -0.2, 0.8, shift_mode=1, fixed_U=(0, 0))
        elif j % 2 == 0:
            wl = W.four_quadrant(n, 20, sub=j + 1, mach=0.5 + (j % 5) * 0.2)
        else:
            wl = W.isentropic_vortex(n, steps=20, mach=0.5 + (j % 4) * 0.5)
        k = int(rng.integers(1, 13))
        a = lbm.Sim.from_workload(wl, precision="fp32")
        try:
            a.step(k)
        except lbm.LBMError:
            a.close()
            continue
        jobs.append((wl, k))
        alone.append(macros_of(a))
        a.close()
    assert len(jobs) > 256
    sims = [lbm.Sim.from_workload(wl, precision="fp32") for wl, _ in jobs]
    lbm.step_batched(sims, [k for _, k in jobs])
    for (wl, k), s, want in zip(jobs, sims, alone):
        got = macros_of(s)
        for key in ("rho", "ux", "uy", "T", "Ux", "Uy"):
            assert np.array_equal(got[key], want[key]), (wl.name, k, key)
        s.close()


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_graph_replayed_quanta_equal_plain_batched(serve, precision):
    """Batched quanta replayed as a HIP graph (lbm_step_batched_graph) give
    the populations of plain batched launches bit for bit: three quanta on
    the same batch (recorded once, then replayed with a fresh job table),
    then a quantum with one job fewer (the launch shape changes: recorded
    again)."""
    import paper_2009_13426_amd as lbm
    wls = [W.four_quadrant(48 + 11 * k, 40, sub=k + 5) for k in range(3)] + \
          [W.isentropic_vortex(56, steps=40)]
    plain = [lbm.Sim.from_workload(wl, precision=precision) for wl in wls]
    graph = [lbm.Sim.from_workload(wl, precision=precision) for wl in wls]
    built = []
    for q, steps in enumerate([[10, 10, 10, 10], [10, 7, 10, 4], [10, 10, 10, 10]]):
        lbm.step_batched(plain, steps)
        built.append(lbm.step_batched(graph, steps, graph=True))
    lbm.step_batched(plain[:3], [6, 6, 6])
    built.append(lbm.step_batched(graph[:3], [6, 6, 6], graph=True))
    print(f"{precision}: graph recorded per quantum {built}", flush=True)
    assert built == [1, 0, 0, 1]
    for a, b in zip(plain, graph):
        fa, ga = a.populations()
        fb, gb = b.populations()
        assert bool((fa == fb).all()) and bool((ga == gb).all())
    for s in plain + graph:
        s.close()
