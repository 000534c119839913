"""Throughput of the adaptive D2Q21 step on one MI355X.

Workload: the seeded four-quadrant Riemann problem on a 4096 x 4096 periodic
grid (densities in [0.5, 1.5], pressures in [0.03, 1.5], common velocity up
to Mach 3), Knudsen sensor on, nu = 1e-3, adaptive lattice shifts.  A step is
one pass of the whole hot path over every node (pull, Grad rebuild at shift
interfaces, moments, shift selection, Newton equilibrium, BGK, store).

The headline value is MLUPS (million lattice-node updates per second) of
the FP32-storage form (FP32 populations and collision, FP64 moments and
Newton); the FP64 form is timed the same way and reported beside it.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--size L] [--no-cpu]

One JSON line on stdout.  Inputs are resident on the GPU before timing
starts.  The launch schedule is the autotuner's choice for the grid's size
class (tuned and cached before any timing on a miss; --schedule default
keeps the library's).  Before timing, --settle plain steps (default 200)
carry the draw into its developed state, and warm-up replays of the HIP
graph (at least one chunk) build the graph the timed region replays.  The
timed region is K steps between two synchronisations, replayed as HIP
graphs of --graph-chunk steps; a second pass of K steps with HIP events
around every launch on the stream the library launches on gives the step
kernel's and the link-rebuild kernel's own durations.

`roofline` is the HBM one, the target the step kernel is measured against:
the algorithmic bytes of a node update (read and write 2 x 21 populations:
336 B in FP32 storage, 672 B in FP64) times the nodes of one launch, over
the step kernel's event-timed duration, against 8 TB/s and against the
measured ceiling of the library's own streaming copy kernel.  Its `traffic`
is the HBM bytes one launch moves (FETCH_SIZE + WRITE_SIZE, calibrated on
a copy), reported only while the committed profile summary was taken on
the current kernel sources.  The kernel spends most of its time in FP64
Newton arithmetic, so `roofline.alu` gives beside it the FP64 flops and
VALU instructions per node (from the same summary), the achieved FP64 rate
against the 78.6 TFLOP/s vector peak and the VALU issue fraction, at
2.4 GHz and at the engine clock the summary measured during that kernel.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
FP64_PEAK_TFLOPS = 78.6        # MI355X FP64 vector (256 CUs x 4 SIMDs x 16 lanes x 2 x 2.4 GHz)
VALU_ISSUE_PEAK = 256 * 4 * 64 / 4 * 2.4e9   # wave64 VALU instructions: lanes per second
Q = 21
PROFILE = os.path.join(ROOT, "profiles", "step_kernel_four_quadrant_4096.txt")


def bytes_per_node(precision):
    """Algorithmic HBM bytes per node update of the step kernel: read and
    write 2 x 21 populations, read and write the node's lattice tag and its
    rebuilt-link mask (4 bytes each), write the four moments of the
    collision that the next step's link rebuild reads.  "ref49": the same
    for the reference model (2 x 49 FP64 populations, 8-byte link mask)."""
    if precision == "ref49":
        return 2 * 2 * 49 * 8 + 2 * 4 + 2 * 8 + 4 * 8
    es = 8 if precision == "fp64" else 4
    return 2 * 2 * Q * es + 2 * 4 + 2 * 4 + 4 * es


def algorithmic_bytes(precision):
    """Bytes per node update the method must move (read and write the 2 x 21
    populations), the per-node figure the HBM roofline is taken on: 336 in
    FP32 storage, 672 in FP64."""
    if precision == "ref49":
        return 2 * 2 * 49 * 8
    return 2 * 2 * Q * (8 if precision == "fp64" else 4)


def kernel_sources_digest():
    """sha256 over the HIP sources (the counter figures in the profile are
    valid only for the kernels they were taken on)."""
    import glob
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2009_13426_amd", "csrc")
    for path in sorted(glob.glob(os.path.join(csrc, "*.hpp")) + glob.glob(os.path.join(csrc, "*.hip"))):
        with open(path, "rb") as f:
            h.update(os.path.basename(path).encode() + b"\0" + f.read())
    return h.hexdigest()


def profile_figures():
    """Per-form counter figures of the step kernel from the committed
    rocprofv3 summary: lines 'key: value', keys '<form>.<name>'."""
    out = {}
    try:
        with open(PROFILE) as f:
            for line in f:
                if ":" in line and not line.startswith("#"):
                    k, v = line.split(":", 1)
                    out[k.strip()] = v.strip()
    except OSError:
        return {}
    return out


def time_form(lbm, torch, wl, precision, steps, warmup, schedule=None, chunk=10, settle=0,
              **over):
    """Untimed: `settle` plain steps that carry the draw into its developed
    state (more shift interfaces, hence more rebuilt links, than the first
    steps), then warm-up replays of a HIP graph of `chunk` steps, at least one
    chunk, so that the graph the timed region replays is built before it.
    Timed region: `steps` steps between two synchronisations, as replays of
    that graph (plus plain launches for a remainder).  A second pass of
    `steps` steps with HIP events around every launch on the library's stream
    gives the step and link-rebuild kernels' own durations."""
    sim = lbm.Sim.from_workload(wl, precision=precision, schedule=schedule, **over)
    sched = sim.schedule
    if settle:
        sim.step(settle)
    graph_warm = max(chunk, warmup + (-warmup) % chunk)
    sim.step_graph(graph_warm, chunk)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step_graph_async(steps, chunk)
    sim.sync()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_rebuild, ms_step = sim.step_profiled(steps)
    d = sim.diag()
    nodes = wl.nx * wl.ny
    out = dict(ms_per_step=wall * 1e3 / steps, kernel_ms=ms_step / steps,
               rebuild_ms=ms_rebuild / steps, mlups=nodes * steps / wall / 1e6,
               conserved=d["conserved"], status=d["status"], schedule=sched,
               untimed_steps=settle + graph_warm)
    sim.close()
    return out


def stats_pass(lbm, wl, precision, steps, settle=0):
    """Newton iterations per solve and rebuilt links per node over a window
    of `steps` steps after the same settling as the timed run."""
    sim = lbm.Sim.from_workload(wl, precision=precision, stats=True)
    if settle:
        sim.step(settle)
    d0 = sim.diag()
    sim.step(steps)
    d = sim.diag()
    nodes = wl.nx * wl.ny * steps
    sim.close()
    calls = d["newton_calls"] - d0["newton_calls"]
    iters = d["newton_iters"] - d0["newton_iters"]
    links = d["mismatched_links"] - d0["mismatched_links"]
    return dict(newton_iters_per_solve=iters / max(calls, 1), solves_per_node=calls / nodes,
                rebuilt_links_per_node=links / nodes, window_steps=steps, after_steps=settle)


def copy_bandwidth(torch, lbm, mib=2048, reps=5):
    """Practical HBM ceiling: the library's streaming copy kernel (16-byte
    nontemporal loads and stores) over 2 GiB, far beyond the caches, timed
    with HIP events on the stream it is launched on; bytes read + written per
    second, the best of a few."""
    n = (mib << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    stream = torch.cuda.current_stream()
    lbm.stream_copy(src, dst, stream)
    best = float("inf")
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        lbm.stream_copy(src, dst, stream)
        b.record(stream)
        b.synchronize()
        best = min(best, a.elapsed_time(b) * 1e-3)
    ok = bool(torch.equal(src[:1024], dst[:1024])) and bool(torch.equal(src[-1024:], dst[-1024:]))
    del src, dst
    torch.cuda.empty_cache()
    if not ok:
        raise RuntimeError("stream copy produced wrong data")
    return 2 * (mib << 20) / best / 1e9


def host_cpu():
    """Model, sockets and physical cores of the host (from /proc/cpuinfo).
    Where the model name is generic (virtual machines report "AMD EPYC"),
    the CPUID family, model and stepping identify the part."""
    model, phys = "", set()
    ident = {}
    cur = {}
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if ":" not in line:
                    if cur:
                        phys.add((cur.get("physical id"), cur.get("core id")))
                    cur = {}
                    continue
                k, v = (t.strip() for t in line.split(":", 1))
                cur[k] = v
                if k == "model name" and not model:
                    model = v
                if k in ("cpu family", "model", "stepping") and k not in ident:
                    ident[k] = v
        if cur:
            phys.add((cur.get("physical id"), cur.get("core id")))
    except OSError:
        pass
    sockets = len({p for p, _ in phys if p is not None}) or None
    cores = len(phys) if phys and None not in {c for _, c in phys} else None
    if ident:
        model = (f"{model} (family {ident.get('cpu family', '?')}, model "
                 f"{ident.get('model', '?')}, stepping {ident.get('stepping', '?')})")
    return dict(model=model, sockets=sockets, physical_cores=cores,
                logical_cpus=os.cpu_count(), affinity_cpus=len(os.sched_getaffinity(0)))


def cpu_baseline(wl_full, seconds_target=15.0, max_steps=40):
    """The FP64 oracle, as it is, on a bounded sample of the same workload:
    a 641 x 641 periodic crop around the quadrant corner, stepped until about
    seconds_target have passed (at most max_steps, which keeps the crop
    clear of the wave collisions its smaller periodic box would bring)."""
    import oracle
    half = 320
    sample = wl_full.window(wl_full.nx // 2, wl_full.ny // 2, half)
    threads = int(os.environ.get("OMP_NUM_THREADS", len(os.sched_getaffinity(0))))
    s = oracle.Sim.from_workload(sample)
    n = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds_target and n < max_steps:
        s.step(2)
        n += 2
    dt = time.perf_counter() - t0
    nodes = sample.nx * sample.ny
    cpu = host_cpu()
    return dict(value=round(nodes * n / dt / 1e6, 4), unit="MLUPS", cores=threads,
                kind="oracle", cpu=cpu["model"], sockets=cpu["sockets"],
                physical_cores=cpu["physical_cores"], logical_cpus=cpu["logical_cpus"],
                threads=threads,
                sample=f"{sample.nx}x{sample.ny} periodic crop of the same initial field, "
                       f"{n} steps, FP64, {dt:.1f} s, OpenMP threads {threads}")


SERVE_JOBS = 128


def serving_pass(torch, W, n_jobs=SERVE_JOBS, quantum=50, schedule="auto"):
    """The first n_jobs of the seeded serving mix (vortex / quadrant flows,
    side log-uniform in [64, 1024], Mach in [0.5, 3], 100-2000 steps), FP32
    storage.  Capacity = jobs per second with every job queued at t = 0 on
    the batched server; then Poisson arrivals at 80 % of capacity, served by
    the continuous-batching loop and by the one-job-at-a-time path."""
    from paper_2009_13426_amd import serve as S
    specs = W.serving_jobs(n_jobs)
    free, _ = torch.cuda.mem_get_info()
    budget = int(0.6 * free)
    eng = S.GpuEngine(precision="fp32", schedule=schedule)
    eng.prepare(S.requests_from_specs(specs, float("inf")))
    cap = S.serve(S.requests_from_specs(specs, float("inf"), prebuild=True), eng, budget,
                  quantum).summary()
    rate = 0.8 * cap["jobs_per_s"]
    reqs = S.requests_from_specs(specs, rate, prebuild=True)
    batched = S.serve(reqs, eng, budget, quantum).summary()
    alone = S.serve_one_at_a_time(reqs, eng).summary()
    keep = ("p50_s", "p99_s", "p50_all_s", "p99_all_s", "mean_s", "mean_wait_s", "mlups",
            "makespan_s", "failed")
    return dict(jobs=n_jobs, sample=f"a sample: the first {n_jobs} jobs of the seeded 10,000-job "
                                    "mix (the full trace runs through python -m "
                                    "paper_2009_13426_amd.serve); p50/p99 over completed jobs, "
                                    "p50_all/p99_all with failed jobs at their failure time",
                capacity_jobs_per_s=round(cap["jobs_per_s"], 3), rate_jobs_per_s=round(rate, 3),
                quantum_steps=quantum, memory_budget_bytes=budget,
                batched_schedule=eng.batch_schedule,
                batched={k: round(batched[k], 4) for k in keep},
                one_at_a_time={k: round(alone[k], 4) for k in keep})


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--size", type=int, default=4096)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--schedule", default="auto", choices=("auto", "default"),
                    help="launch schedule: the autotuner's choice for the grid's size class "
                         "(cached; tuned before the timed region on a miss) or the library "
                         "default")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip timing the four-constraint equilibrium variant (FP32 storage), "
                         "the flexible-Prandtl collision (FP32, Pr = 0.71) and the reference "
                         "model (D2Q49, 13 constraints, FP64)")
    ap.add_argument("--graph-chunk", type=int, default=10,
                    help="steps per HIP graph replayed in the timed region (even)")
    ap.add_argument("--forms", default="fp32,fp64")
    ap.add_argument("--no-serve", action="store_true",
                    help="skip the job-server pass (p50/p99 time-to-solution)")
    ap.add_argument("--no-counters", action="store_true",
                    help="skip the extra run with Newton and rebuild counters")
    ap.add_argument("--settle", type=int, default=200,
                    help="untimed plain steps before the warm-up, which carry the draw into "
                         "its developed state (shift interfaces grown from the quadrant lines)")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="only run a plain device copy of this many MiB three times "
                         "(calibrates the HBM byte counters) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU "
              "slab decomposition is a design, not a build.", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2009_13426_amd as lbm
    import workloads as W

    torch.cuda.set_device(0)
    if args.copy_mib:
        n = args.copy_mib << 20
        src = torch.ones(n // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            lbm.stream_copy(src, dst)
        torch.cuda.synchronize()
        print(json.dumps(dict(copy_bytes=n, launches=3)), flush=True)
        return
    wl = W.four_quadrant(args.size, args.settle + args.warmup + args.steps)
    res = {}
    for form in args.forms.split(","):
        print(f"[bench] timing {form} {args.size}^2, warmup {args.warmup}, steps {args.steps}",
              file=sys.stderr, flush=True)
        sched = None
        if args.schedule == "auto":
            from paper_2009_13426_amd import autotune
            sched = autotune.schedule_for(form, args.size, args.size)
        res[form] = time_form(lbm, torch, wl, form, args.steps, args.warmup, sched,
                              args.graph_chunk, settle=args.settle)
        print(f"[bench] {form}: {res[form]['mlups']:.1f} MLUPS, step kernel "
              f"{res[form]['kernel_ms']:.3f} ms, rebuild kernel {res[form]['rebuild_ms']:.3f} ms",
              file=sys.stderr, flush=True)
    variants = {}
    if not args.no_variants:
        print("[bench] timing the four-constraint variant (fp32)", file=sys.stderr, flush=True)
        v = time_form(lbm, torch, wl, "fp32", args.steps, args.warmup, None, args.graph_chunk,
                      settle=args.settle, constraints=4)
        variants["fp32_constraints4"] = dict(
            mlups=round(v["mlups"], 2), kernel_ms=round(v["kernel_ms"], 4),
            rebuild_ms=round(v["rebuild_ms"], 4), status=v["status"],
            equilibrium="mass, momentum and energy constraints only (4 x 4 solve)")
        print(f"[bench] fp32 four constraints: {v['mlups']:.1f} MLUPS", file=sys.stderr,
              flush=True)
        print("[bench] timing the flexible-Prandtl collision (fp32, Pr = 0.71)",
              file=sys.stderr, flush=True)
        v = time_form(lbm, torch, wl, "fp32", args.steps, args.warmup, None, args.graph_chunk,
                      settle=args.settle, prandtl=0.71)
        variants["fp32_prandtl_0.71"] = dict(
            mlups=round(v["mlups"], 2), kernel_ms=round(v["kernel_ms"], 4),
            rebuild_ms=round(v["rebuild_ms"], 4), status=v["status"],
            collision="eq. (Shakhov) at Pr = 0.71, 8 constraints")
        print(f"[bench] fp32 Pr = 0.71: {v['mlups']:.1f} MLUPS", file=sys.stderr, flush=True)
        # the reference model is about ten times slower per node: fewer steps
        rsteps, rwarm = min(args.steps, 20), min(args.warmup, 4)
        print(f"[bench] timing the reference model (D2Q49, 13 constraints, fp64), "
              f"{rsteps} steps", file=sys.stderr, flush=True)
        v = time_form(lbm, torch, wl, "fp64", rsteps, rwarm, None, 2, constraints=13)
        variants["fp64_reference_d2q49_constraints13"] = dict(
            mlups=round(v["mlups"], 2), kernel_ms=round(v["kernel_ms"], 4),
            rebuild_ms=round(v["rebuild_ms"], 4), status=v["status"], steps=rsteps,
            warmup=rwarm,
            equilibrium="D2Q49 lattice, 13 constraints up to the contracted fourth-order "
                        "moments (13 x 13 solve), FP64 storage")
        print(f"[bench] reference model: {v['mlups']:.1f} MLUPS", file=sys.stderr, flush=True)
    head = "fp32" if "fp32" in res else next(iter(res))
    counters = {f: {} for f in res}
    if not args.no_counters:
        print("[bench] counters pass", file=sys.stderr, flush=True)
        counters = {f: stats_pass(lbm, wl, f, args.steps, args.settle) for f in res}

    nodes = wl.nx * wl.ny
    copy_gbs = copy_bandwidth(torch, lbm)
    prof = profile_figures()
    fresh = prof.get("source_sha256") == kernel_sources_digest() and \
        prof.get("size") == str(args.size)
    t_step = res[head]["kernel_ms"] * 1e-3
    flops = float(prof.get(f"{head}.fp64_flops_per_node", "nan"))
    valu = float(prof.get(f"{head}.valu_insts_per_node", "nan"))
    # the engine clock the profile measured during this kernel (GRBM_GUI_ACTIVE
    # per XCC over the dispatch time): the VALU issue limit at that clock
    clk = float(prof[f"{head}.engine_clock_ghz"]) if f"{head}.engine_clock_ghz" in prof else None
    traffic = None
    if fresh:
        traffic = round(float(prof[f"{head}.fetch_bytes_per_launch"]) +
                        float(prof[f"{head}.write_bytes_per_launch"]))
    ach = flops * nodes / t_step / 1e12
    hbm = algorithmic_bytes(head) * nodes / t_step / 1e9
    roofline = dict(bound="hbm", achieved=round(hbm, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(hbm / HBM_PEAK_GBS, 4), traffic=traffic,
                    kernel="step_kernel", bytes_per_node=algorithmic_bytes(head),
                    counters_match_kernel=fresh,
                    copy_gbs=round(copy_gbs, 1), frac_of_copy=round(hbm / copy_gbs, 4),
                    with_side_arrays=dict(
                        bytes_per_node=bytes_per_node(head),
                        achieved=round(bytes_per_node(head) * nodes / t_step / 1e9, 1)),
                    alu=dict(fp64_flops_per_node=flops, achieved=round(ach, 2),
                             peak=FP64_PEAK_TFLOPS, unit="TFLOP/s",
                             frac=round(ach / FP64_PEAK_TFLOPS, 4),
                             valu_insts_per_node=valu,
                             valu_issue_frac=round(valu * nodes / t_step / VALU_ISSUE_PEAK, 4),
                             engine_clock_ghz=clk,
                             valu_issue_frac_at_clock=round(
                                 valu * nodes / t_step / (VALU_ISSUE_PEAK * clk / 2.4), 4)
                             if clk else None))
    serving = None
    if not args.no_serve:
        print("[bench] serving mix", file=sys.stderr, flush=True)
        serving = serving_pass(torch, W, schedule="auto" if args.schedule == "auto" else None)
        print(f"[bench] serving: {json.dumps(serving)}", file=sys.stderr, flush=True)
    cpu = None
    if not args.no_cpu:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        cpu = cpu_baseline(wl)

    line = dict(
        metric="MLUPS of D2Q21 adaptive step (FP64 vs FP32-store); p50/p99 job latency",
        value=round(res[head]["mlups"], 2), unit="MLUPS", n_gpus=1, steps=args.steps,
        warmup=args.warmup, ms_per_step=round(res[head]["ms_per_step"], 4),
        higher_is_better=True, scaling="weak", vs_baseline=None,
        dtype="f32-store/f64-newton" if head == "fp32" else "f64", data="synthetic",
        config=dict(workload=f"four-quadrant Riemann {args.size}x{args.size}, D2Q21 adaptive "
                             f"shifts, Knudsen sensor, nu={wl.nu:g}, seeded draw",
                    nodes=nodes, precision=head, schedule=res[head]["schedule"],
                    graph_chunk=args.graph_chunk, settle_steps=args.settle,
                    untimed_steps_before_timing=res[head]["untimed_steps"]),
        roofline=roofline, cpu_baseline=cpu, serving=serving, variants=variants or None,
        forms={f: dict(mlups=round(r["mlups"], 2), kernel_ms=round(r["kernel_ms"], 4),
                       rebuild_ms=round(r["rebuild_ms"], 4), schedule=r["schedule"],
                       hbm_gbs=round(algorithmic_bytes(f) * nodes / (r["kernel_ms"] * 1e-3) / 1e9, 1),
                       hbm_frac=round(algorithmic_bytes(f) * nodes / (r["kernel_ms"] * 1e-3) / 1e9
                                      / HBM_PEAK_GBS, 4),
                       frac_of_copy=round(algorithmic_bytes(f) * nodes / (r["kernel_ms"] * 1e-3)
                                          / 1e9 / copy_gbs, 4),
                       bytes_per_node=algorithmic_bytes(f), **counters[f])
               for f, r in res.items()},
    )
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
