"""The schedule autotuner's host logic (no device): size classes, candidate
sets, the choice from timings, and the JSON cache."""
import json
import math

import pytest

from conftest import ensure_library

ensure_library()
from paper_2009_13426_amd import autotune as A  # noqa: E402


def test_size_classes():
    assert A.bucket(4096, 4096) == 4096
    assert A.bucket(1024, 1024) == 1024
    assert A.bucket(2048, 4) == 128          # sqrt(8192) = 2^6.5, halves round up
    assert A.bucket(256, 1) == 16
    assert A.bucket(1, 1) == 1
    assert A.cache_key("fp32", 4000, 4100) == "fp32/4096"
    assert A.cache_key(0, 64, 64) == "fp64/64"


def test_candidates_respect_what_is_built():
    c64 = A.step_candidates("fp64")
    c32 = A.step_candidates("fp32")
    assert {c["step_block"] for c in c64} == {64, 128}
    assert {c["step_block"] for c in c32} == {64, 128, 256}
    assert len(c32) == 3 * len(A.TILES) * len(A.REMAPS)
    assert all(set(c) == {"step_block", "tiles_per_block", "xcd_remap"} for c in c32)


class FakeSim:
    def __init__(self):
        self.applied = []


def test_choice_is_the_fastest_step_then_the_fastest_rebuild():
    # step time depends on the step schedule only, rebuild time on the
    # rebuild workgroups only
    def step_ms(s):
        return 1.0 + 0.1 * s["tiles_per_block"] + (0.0 if s["step_block"] == 128 else 0.05) + \
            0.01 * (1 - s["xcd_remap"])

    def timer(sim, sched, steps, repeats, reset):
        sim.applied.append(dict(sched))
        rb = {0: 0.3, 256: 0.25, 1024: 0.2, 8192: 0.4}[sched["rebuild_blocks"]]
        return rb, step_ms(sched)

    sim = FakeSim()
    out = A.choose(sim, "fp32", timer=timer)
    assert out["schedule"] == dict(step_block=128, tiles_per_block=1, xcd_remap=1,
                                   rebuild_blocks=1024)
    assert out["step_ms"] == pytest.approx(1.1)
    assert out["rebuild_ms"] == pytest.approx(0.2)
    n_step = len(A.step_candidates("fp32"))
    assert len(out["trials"]) == n_step + len(A.rebuild_candidates())
    # the rebuild sweep runs on the chosen step schedule
    assert all(t["step_block"] == 128 and t["tiles_per_block"] == 1
               for t in out["trials"][n_step:])


def test_noise_below_the_margin_keeps_the_first_candidate():
    def timer(sim, sched, steps, repeats, reset):
        # the second candidate is 1.5 % faster: within the margin
        return 0.2, 1.0 - (0.015 if sched["xcd_remap"] == 0 and sched["step_block"] == 64
                           and sched["tiles_per_block"] == 1 else 0.0)
    out = A.choose(FakeSim(), "fp64", timer=timer)
    assert out["schedule"]["step_block"] == 64 and out["schedule"]["xcd_remap"] == 1
    assert out["schedule"]["rebuild_blocks"] == 0


def test_cache_round_trip(tmp_path):
    path = str(tmp_path / "sub" / "schedules.json")
    assert A.load_cache(path) == {}
    entry = dict(schedule=dict(step_block=64, tiles_per_block=1, xcd_remap=1, rebuild_blocks=512),
                 step_ms=2.1, rebuild_ms=0.2, trials=[])
    A.save_cache({"fp32/4096": entry}, path)
    assert json.load(open(path))["fp32/4096"]["schedule"]["rebuild_blocks"] == 512
    assert A.schedule_for("fp32", 4096, 4096, cache_path=path) == entry["schedule"]
    assert A.schedule_for("fp32", 3900, 4000, cache_path=path) == entry["schedule"]
    # a miss without tuning leaves the library default
    assert A.schedule_for("fp64", 4096, 4096, cache_path=path, tune_missing=False) is None
    # a corrupt cache reads as empty
    open(path, "w").write("{not json")
    assert A.load_cache(path) == {}


def test_default_cache_path_follows_the_environment(monkeypatch, tmp_path):
    monkeypatch.setenv(A.CACHE_ENV, str(tmp_path / "x.json"))
    assert A.default_cache_path() == str(tmp_path / "x.json")
    monkeypatch.delenv(A.CACHE_ENV)
    assert A.default_cache_path().endswith("schedules.json")
    assert math.isfinite(len(A.default_cache_path()))
