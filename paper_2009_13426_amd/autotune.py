"""Autotuner of the step loop's launch schedule.

The per-node work of a step is fixed; what can be chosen is how nodes map to
workgroups (`lbm_schedule`): lanes per workgroup of the step kernel, nodes
per lane (a workgroup runs that many consecutive tiles one after the other,
each lane taking one node of every tile in turn: `tiles_per_block`), the
XCD-aware tile order, and the workgroup count of the link-rebuild launch.
Every schedule gives bitwise the same results, so the choice is by time
alone.

The tuner times each candidate on a throw-away simulation (its steps are
never part of a user's run), restored before every timing to one state of
the developed flow (lbm_copy_state), with `lbm_step_profiled`, which brackets every launch with HIP events, and keeps
the fastest: first the step schedule on
the summed step-launch time, then the rebuild workgroup count on the
rebuild-launch time.  Results are cached in a JSON file keyed by storage
precision and grid-size bucket (the power of two nearest to the square root
of the node count), so that one tuning serves every grid of that size
class.
"""
from __future__ import annotations

import json
import math
import os
import tempfile
from typing import Callable, Dict, Iterable, List, Optional, Tuple

CACHE_ENV = "LBM_SCHEDULE_CACHE"
STEP_BLOCKS = {"fp64": (64, 128), "fp32": (64, 128, 256)}
TILES = (1, 2, 4, 8)   # nodes per lane (tiles per workgroup)
REMAPS = (1, 0)
REBUILD_BLOCKS = (0, 256, 1024, 8192)
MARGIN = 0.02   # relative gain a candidate needs over the best so far


def default_cache_path() -> str:
    return os.environ.get(CACHE_ENV) or os.path.join(
        os.path.expanduser("~"), ".cache", "paper_2009_13426_amd", "schedules.json")


def _precision_name(precision) -> str:
    return "fp64" if precision in ("fp64", 0) else "fp32"


def bucket(nx: int, ny: int) -> int:
    """Side of the size class: the power of two nearest (in log scale) to
    sqrt(nx * ny)."""
    return 1 << max(0, int(math.floor(0.5 * math.log2(max(1, nx * ny)) + 0.5)))


def cache_key(precision, nx: int, ny: int) -> str:
    return f"{_precision_name(precision)}/{bucket(nx, ny)}"


def step_candidates(precision) -> List[Dict[str, int]]:
    return [dict(step_block=b, tiles_per_block=t, xcd_remap=r)
            for b in STEP_BLOCKS[_precision_name(precision)] for t in TILES for r in REMAPS]


def rebuild_candidates() -> List[Dict[str, int]]:
    return [dict(rebuild_blocks=r) for r in REBUILD_BLOCKS]


def load_cache(path: Optional[str] = None) -> Dict[str, dict]:
    path = path or default_cache_path()
    try:
        with open(path) as f:
            data = json.load(f)
    except (OSError, ValueError):
        return {}
    return data if isinstance(data, dict) else {}


def save_cache(entries: Dict[str, dict], path: Optional[str] = None):
    """Writes the cache atomically (temporary file, then rename)."""
    path = path or default_cache_path()
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    fd, tmp = tempfile.mkstemp(dir=os.path.dirname(os.path.abspath(path)), suffix=".tmp")
    with os.fdopen(fd, "w") as f:
        json.dump(entries, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def time_schedule(sim, sched: Dict[str, int], steps: int, repeats: int,
                  reset: Optional[Callable] = None, warm: int = 2) -> Tuple[float, float]:
    """(rebuild ms, step ms) per step under `sched`: the best of `repeats`
    runs of `steps` steps, each after reset() (back to the initial state,
    so that every candidate is timed on the same steps of the same flow)
    and `warm` untimed steps."""
    sim.schedule = sched
    best_r = best_s = math.inf
    for _ in range(repeats):
        if reset is not None:
            reset()
        if warm:
            sim.step(warm)
        r, s = sim.step_profiled(steps)
        best_r, best_s = min(best_r, r / steps), min(best_s, s / steps)
    return best_r, best_s


def choose(sim, precision, steps: int = 8, repeats: int = 2,
           timer: Callable = time_schedule, reset: Optional[Callable] = None,
           step_cands: Optional[Iterable[dict]] = None,
           rebuild_cands: Optional[Iterable[dict]] = None, margin: float = MARGIN) -> dict:
    """Times the candidates on `sim` and returns {"schedule": {...},
    "step_ms": t, "rebuild_ms": t, "trials": [...]}.  A candidate replaces
    the best so far only if faster by more than `margin` (relative), so
    that timing noise does not move the choice away from the first
    (default) candidate."""
    trials = []
    best, best_t = None, math.inf
    for cand in (step_cands if step_cands is not None else step_candidates(precision)):
        r, s = timer(sim, dict(cand, rebuild_blocks=0), steps, repeats, reset)
        trials.append(dict(cand, rebuild_blocks=0, nodes_per_lane=cand.get("tiles_per_block", 1),
                           step_ms=s, rebuild_ms=r))
        if s < best_t * (1.0 - margin):
            best, best_t = dict(cand), s
    best_rb, best_rt = 0, math.inf
    for cand in (rebuild_cands if rebuild_cands is not None else rebuild_candidates()):
        r, s = timer(sim, dict(best, **cand), steps, repeats, reset)
        trials.append(dict(best, **cand, step_ms=s, rebuild_ms=r))
        if r < best_rt * (1.0 - margin):
            best_rb, best_rt = cand["rebuild_blocks"], r
    return dict(schedule=dict(best, rebuild_blocks=best_rb), step_ms=best_t, rebuild_ms=best_rt,
                trials=trials)


def tune_workload(wl, precision="fp32", steps: int = 8, repeats: int = 3, advance: int = 100,
                  cache_path: Optional[str] = None, store: bool = True, device=None) -> dict:
    """Tunes on throw-away simulations of workload `wl`: a reference run is
    advanced `advance` steps (so that the flow has developed its shift
    interfaces and rebuild lists), and every candidate is timed on a probe
    restored from that state (lbm_copy_state) before each repeat.  Stores
    the result under the workload's cache key and returns the entry."""
    from . import Sim
    ref = Sim.from_workload(wl, precision=precision, device=device)
    probe = None
    try:
        ref.step(advance)
        probe = Sim.from_workload(wl, precision=precision, device=device, like=ref)
        entry = choose(probe, precision, steps=steps, repeats=repeats,
                       reset=lambda: probe.copy_state_from(ref))
    finally:
        ref.close()
        if probe is not None:
            probe.close()
    entry["grid"] = [wl.nx, wl.ny]
    entry["advance"] = advance
    if store:
        entries = load_cache(cache_path)
        entries[cache_key(precision, wl.nx, wl.ny)] = entry
        save_cache(entries, cache_path)
    return entry


def schedule_for(precision, nx: int, ny: int, cache_path: Optional[str] = None,
                 tune_missing: bool = True, device=None) -> Optional[Dict[str, int]]:
    """The cached schedule of the size class of nx x ny; on a miss, tunes on
    a seeded four-quadrant flow of the bucket's side (if tune_missing), else
    None (the library default then applies)."""
    entries = load_cache(cache_path)
    key = cache_key(precision, nx, ny)
    if key in entries:
        return dict(entries[key]["schedule"])
    if not tune_missing:
        return None
    import workloads as W
    side = max(16, bucket(nx, ny))
    entry = tune_workload(W.four_quadrant(side, 100), precision=precision,
                          cache_path=cache_path, device=device)
    return dict(entry["schedule"])


def batched_candidates(precision) -> List[Dict[str, int]]:
    """The batched step launch takes step_block and xcd_remap from its first
    context and runs one tile per workgroup."""
    return [dict(step_block=b, xcd_remap=r) for b in STEP_BLOCKS[_precision_name(precision)]
            for r in REMAPS]


def tune_batched(wls, precision="fp32", steps: int = 10, repeats: int = 2,
                 cache_path: Optional[str] = None, store: bool = True, device=None) -> dict:
    """Tunes the schedule of the batched step (lbm_step_batched) on a batch
    of workloads: each candidate is set on the first context, every context
    is reset to its initial state, and `steps` batched steps are timed
    between two synchronisations (best of `repeats`).  Stored under
    "<precision>/batched"."""
    import time

    import torch
    from . import Sim, step_batched
    sims = [Sim.from_workload(wl, precision=precision, device=device) for wl in wls]
    fields = [[torch.as_tensor(a, dtype=torch.float64, device=s.device).reshape(wl.ny, wl.nx)
               .contiguous() for a in wl.fields()] for s, wl in zip(sims, wls)]
    n = len(sims)
    trials = []
    best, best_t = None, math.inf
    try:
        for cand in batched_candidates(precision):
            sims[0].schedule = cand
            t = math.inf
            for _ in range(repeats):
                for s, f in zip(sims, fields):
                    s.init(*f)
                step_batched(sims, [2] * n)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                step_batched(sims, [steps] * n)
                t = min(t, (time.perf_counter() - t0) * 1e3 / steps)
            trials.append(dict(cand, ms_per_step=t))
            if t < best_t * (1.0 - MARGIN):
                best, best_t = dict(cand), t
    finally:
        for s in sims:
            s.close()
    entry = dict(schedule=best, ms_per_step=best_t, trials=trials,
                 grids=[[wl.nx, wl.ny] for wl in wls])
    if store:
        entries = load_cache(cache_path)
        entries[f"{_precision_name(precision)}/batched"] = entry
        save_cache(entries, cache_path)
    return entry


def batched_schedule_for(precision, cache_path: Optional[str] = None, tune_missing: bool = True,
                         device=None, jobs: int = 16) -> Optional[Dict[str, int]]:
    """The cached batched-step schedule; on a miss, tunes on the first
    `jobs` flows of the seeded serving mix (if tune_missing), else None."""
    entries = load_cache(cache_path)
    key = f"{_precision_name(precision)}/batched"
    if key in entries:
        return dict(entries[key]["schedule"])
    if not tune_missing:
        return None
    import workloads as W
    wls = [sp.build() for sp in W.serving_jobs(jobs)]
    return dict(tune_batched(wls, precision=precision, cache_path=cache_path,
                             device=device)["schedule"])
