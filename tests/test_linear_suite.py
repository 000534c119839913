"""The linear-regime cases of Sec. IV.B on the oracle: the stored oracle
figures (tests/golden/linear_suite_oracle.json, written by
make_linear_suite.py) against the paper's printed values, and cheap
re-runs showing that the stored figures are the oracle's.

Soft pins: the paper's figures depend on its velocity set, which it does not
print (the D2Q21 set here is a reading), so they are held to within a few
tenths of a percent (entropy spot) or to the paper's own claim (shear wave:
below 1 %)."""
import json
import os
import sys

import numpy as np
import pytest

import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))
import make_linear_suite as M  # noqa: E402

GOLD = json.load(open(os.path.join(HERE, "golden", "paper_values.json")))
LIN = json.load(open(os.path.join(HERE, "golden", "linear_suite_oracle.json")))


def test_steps_are_fifteen_flow_through_times():
    g = GOLD["shear_wave_nu_num_percent"]
    assert [W.linear_steps(u) for u in g["u0"]] == g["steps"]
    s = GOLD["entropy_spot_loss_percent"]
    assert [W.linear_steps(u) for u in s["u0"]] == s["steps"]
    with pytest.raises(ValueError):
        W.linear_steps(2.2)


def test_shear_wave_below_one_percent():
    for u0, paper in zip(GOLD["shear_wave_nu_num_percent"]["u0"],
                         GOLD["shear_wave_nu_num_percent"]["value"]):
        v = LIN["shear_wave"][str(u0)]["nu_num_percent"]
        assert 0.0 <= v < 1.0, (u0, v, paper)


def test_entropy_spot_loss_near_the_paper():
    g = GOLD["entropy_spot_loss_percent"]
    for u0, paper in zip(g["u0"], g["value"]):
        v = LIN["entropy_spot"][str(u0)]["peak_loss_percent"]
        assert abs(v - paper) < 0.4, (u0, v, paper)


def test_acoustic_pulse_is_galilean_invariant():
    # the pulse moved back by u0 * 30 nodes matches the pulse at rest to 1 %
    for u0, rec in LIN["acoustic_pulse"].items():
        assert rec["recentred_max_diff"] < 0.01, (u0, rec)


@pytest.mark.parametrize("u0", [3.0])
def test_stored_shear_figure_is_the_oracle(orc, u0):
    m = M.run(W.shear_wave(u0))
    assert M.shear_nu_num(m) == pytest.approx(LIN["shear_wave"][str(u0)]["nu_num_percent"],
                                              rel=1e-9, abs=1e-12)


def test_stored_acoustic_figure_is_the_oracle(orc):
    ref = M.recentred(M.acoustic_dp(M.run(W.acoustic_pulse(0.0))), 0.0)
    dp = M.recentred(M.acoustic_dp(M.run(W.acoustic_pulse(1.3))), 1.3)
    rec = LIN["acoustic_pulse"]["1.3"]
    assert float(dp.max()) == pytest.approx(rec["max_dp"], rel=1e-12)
    assert float(np.abs(dp - ref).max() / np.abs(ref).max()) == pytest.approx(
        rec["recentred_max_diff"], rel=1e-9)


def test_relative_velocity_half_grows_an_inviscid_mode(orc):
    """At u0 = 2.5 every node sits at relative velocity 1/2 in its lattice
    (the edge of the shift range); with nu = 0 (tau = 1/2) a small
    perturbation of the entropy spot then grows (about tenfold per 100
    steps once it has organised), while at u0 = 2 (relative velocity 0) it
    stays at its seeded size.  This is why the FP32 storage form cannot
    carry the u0 = 2.5 spot over 15 t_c: its rounding seeds the mode at
    ~1e-8 (see test_gpu_linear_suite.py)."""
    rng = np.random.default_rng(1)
    growth = {}
    for u0 in (2.5, 2.0):
        clean = W.entropy_spot(u0, L=50)
        noisy = W.entropy_spot(u0, L=50)
        noisy.rho = noisy.rho * (1 + 1e-8 * rng.standard_normal(noisy.rho.shape))
        a, b = orc.Sim.from_workload(clean), orc.Sim.from_workload(noisy)
        a.step(400)
        b.step(400)
        growth[u0] = float(np.abs(a.macros()["rho"] - b.macros()["rho"]).max()) / 1e-8
    assert growth[2.5] > 10.0 and growth[2.0] < 3.0, growth
