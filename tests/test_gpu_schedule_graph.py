"""Launch schedules, HIP-graph replay and the autotuner on the GPU.

A schedule only changes how nodes map to workgroups, and a graph replays
the same launches: results must be bitwise the same as the default plain
launches, on grids whose node count is a multiple of no tile size (ragged
last tile), in both storage forms.  Graph replays are checked after every
call, with eager launches and host synchronisation between the calls, and
across both buffer parities.  A failure inside a replay must report its true
step (the same as the plain path and the oracle)."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

FIELDS = ("rho", "ux", "uy", "T", "Ux", "Uy")


@pytest.fixture(scope="module")
def lbm():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2009_13426_amd as lbm
    return lbm


def host(sim):
    return {k: v.cpu().numpy() for k, v in sim.macros().items()}


def same(a, b):
    return all(np.array_equal(a[k], b[k]) for k in FIELDS)


def ragged():
    # 97 x 83 = 8051 nodes: no multiple of 64, 128 or 256
    wl = W.four_quadrant(97, 12)
    wl.ny = 83
    wl.rho, wl.ux, wl.uy, wl.T = (a[:83] for a in (wl.rho, wl.ux, wl.uy, wl.T))
    return wl


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_every_schedule_gives_the_same_bits(lbm, precision):
    from paper_2009_13426_amd import autotune
    wl = ragged()
    steps = 12
    ref = lbm.Sim.from_workload(wl, precision=precision)
    print(f"{precision} default schedule {ref.schedule}", flush=True)
    ref.step(steps)
    want = host(ref)
    assert ref.diag()["status"] == 0
    ref.close()
    cands = [dict(c, rebuild_blocks=0) for c in autotune.step_candidates(precision)]
    cands += [dict(step_block=64, tiles_per_block=1, xcd_remap=1, rebuild_blocks=r)
              for r in (1, 7, 256, 8192)]
    for c in cands:
        sim = lbm.Sim.from_workload(wl, precision=precision, schedule=c)
        sim.step(steps)
        got = host(sim)
        sim.close()
        assert same(got, want), c


def test_invalid_schedules_are_refused(lbm):
    sim = lbm.Sim.from_workload(W.four_quadrant(32, 4), precision="fp64")
    before = sim.schedule
    for bad in (dict(step_block=256), dict(step_block=96), dict(tiles_per_block=0),
                dict(tiles_per_block=65), dict(xcd_remap=2), dict(rebuild_blocks=-1)):
        with pytest.raises(lbm.LBMError) as e:
            sim.schedule = bad
        assert e.value.status == lbm.ERR_ARG
        assert sim.schedule == before
    sim.close()


def test_batched_step_with_a_wider_block(lbm):
    specs = [W.JobSpec(j, "quadrant" if j % 2 else "vortex", n, 1.0 + 0.4 * j, 20, 0.0)
             for j, n in enumerate((40, 72, 57))]
    alone = []
    for sp in specs:
        s = lbm.Sim.from_workload(sp.build(), precision="fp32")
        s.step(sp.steps)
        alone.append(host(s))
        s.close()
    sims = [lbm.Sim.from_workload(sp.build(), precision="fp32") for sp in specs]
    sims[0].schedule = dict(step_block=256, xcd_remap=0)
    lbm.step_batched(sims, [sp.steps for sp in specs])
    for s, a, sp in zip(sims, alone, specs):
        assert same(host(s), a), sp.job_id
        s.close()


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_graph_replays_match_plain_launches(lbm, precision):
    wl = ragged()
    plain = lbm.Sim.from_workload(wl, precision=precision)
    graph = lbm.Sim.from_workload(wl, precision=precision)
    # (plain steps, graph call: steps, chunk); odd plain counts flip the
    # buffer parity, so graphs of both parities are built and replayed
    plan = [(0, 20, 4), (0, 20, 4), (1, 9, 4), (0, 16, 8), (3, 40, 8), (0, 7, 2)]
    done = 0
    for k, (p, n, chunk) in enumerate(plan):
        if p:
            graph.step(p)
        graph.step_graph(n, chunk)
        plain.step(p + n)
        done += p + n
        a, b = host(graph), host(plain)       # eager work between replays
        assert same(a, b), (k, p, n, chunk)
        assert graph.diag()["steps_done"] == plain.diag()["steps_done"] == done
    assert plain.diag()["status"] == 0
    plain.close()
    graph.close()


def accelerating_pulse():
    """1D density pulse (+20 %, width 40) on a uniform flow at u = 1.45, T = 1:
    the flow passes u = 1.5 at step 15, where the selected lattice U = 2
    leaves the admissible range |U| <= 1 (seen on the oracle)."""
    nx = 256
    x = np.arange(nx)[None, :]
    rho = 1.0 + 0.2 * np.exp(-((x - nx / 2) / 40.0) ** 2)
    return W.Workload("pulse", nx, 1, rho, np.full((1, nx), 1.45), np.zeros((1, nx)),
                      np.ones((1, nx)), 0.01, 40)


def test_failure_in_a_replay_reports_its_step(lbm):
    import oracle
    wl = accelerating_pulse()
    ref = oracle.Sim.from_workload(wl, max_abs_shift=1)
    fail_oracle = None
    for k in range(1, 41):
        try:
            ref.step(1)
        except oracle.OracleError as e:
            assert e.rc == oracle.ERR_NONPHYSICAL
            fail_oracle = k
            break
    assert fail_oracle is not None and fail_oracle > 8
    sim = lbm.Sim.from_workload(wl, precision="fp64", max_abs_shift=1)
    with pytest.raises(lbm.LBMError) as e:
        sim.step(40)
    assert e.value.status == lbm.ERR_NONPHYSICAL
    fail_plain = sim.diag()["fail_step"]
    sim.close()
    sim = lbm.Sim.from_workload(wl, precision="fp64", max_abs_shift=1)
    sim.step(3)
    with pytest.raises(lbm.LBMError) as e:
        sim.step_graph(36, 4)
    assert e.value.status == lbm.ERR_NONPHYSICAL
    fail_graph = sim.diag()["fail_step"]
    sim.close()
    print(f"failure step: oracle {fail_oracle}, plain {fail_plain}, graph {fail_graph}", flush=True)
    assert fail_plain == fail_graph == fail_oracle


def test_autotuned_schedule_is_cached_and_used(lbm, tmp_path, monkeypatch):
    from paper_2009_13426_amd import autotune
    path = str(tmp_path / "schedules.json")
    monkeypatch.setenv(autotune.CACHE_ENV, path)
    wl = W.four_quadrant(128, 10)
    entry = autotune.tune_workload(wl, precision="fp32", steps=3, repeats=1, advance=5)
    print("tuned 128^2 fp32:", entry["schedule"], f"step {entry['step_ms']:.4f} ms",
          f"rebuild {entry['rebuild_ms']:.4f} ms", flush=True)
    assert autotune.load_cache()["fp32/128"]["schedule"] == entry["schedule"]
    a = lbm.Sim.from_workload(wl, precision="fp32", schedule="auto")
    want = dict(entry["schedule"])
    got = a.schedule
    assert all(got[k] == v for k, v in want.items() if k != "rebuild_blocks" or v)
    a.step(10)
    b = lbm.Sim.from_workload(wl, precision="fp32")
    b.step(10)
    assert same(host(a), host(b))
    a.close()
    b.close()


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_copied_state_continues_bitwise(lbm, precision):
    wl = ragged()
    a = lbm.Sim.from_workload(wl, precision=precision)
    a.step(7)
    b = lbm.Sim.from_workload(wl, precision=precision, like=a)
    b.step(3)                                  # its own state is overwritten
    b.copy_state_from(a)
    assert b.diag()["steps_done"] == 7
    a.step(9)
    b.step(9)
    assert same(host(a), host(b))
    # configurations must match; the source must be initialised
    c = lbm.Sim.from_workload(wl, precision=precision, nu=2 * wl.nu)
    with pytest.raises(lbm.LBMError) as e:
        c.copy_state_from(a)
    assert e.value.status == lbm.ERR_ARG
    fresh = lbm.Sim(wl.nx, wl.ny, precision=precision, nu=wl.nu, sensor=wl.sensor)
    with pytest.raises(lbm.LBMError) as e:
        a.copy_state_from(fresh)
    assert e.value.status == lbm.ERR_STATE
    for s in (a, b, c, fresh):
        s.close()


def test_neighbourhood_mode_runs_the_default_schedule_only(lbm):
    wl = W.four_quadrant(48, 4)
    wl.shift_mode, wl.halfwidth = 3, 0.9
    sim = lbm.Sim.from_workload(wl, precision="fp32")
    with pytest.raises(lbm.LBMError) as e:
        sim.schedule = dict(step_block=128)
    assert e.value.status == lbm.ERR_ARG
    with pytest.raises(lbm.LBMError) as e:
        lbm.step_batched([sim], [2])
    assert e.value.status == lbm.ERR_ARG
    sim.step_graph(8, 4)                      # graphs are fine
    auto = lbm.Sim.from_workload(wl, precision="fp32", schedule="auto")
    assert auto.schedule["step_block"] == 64
    auto.close()
    sim.close()
