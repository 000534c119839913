"""Writes linear_suite_oracle.json: the oracle's figures for the linear-regime
cases of Sec. IV.B (shear wave, entropy spot, acoustic pulse), computed with
the CPU oracle only.  Run from the repository root:

    python tests/golden/make_linear_suite.py

Figures (same definitions in the GPU tests):
  shear wave     nu_num = |A - max u_y| / A in percent after 15 t_c
                 (Sec. IV.B.1; the reference peak is the initial amplitude A)
  entropy spot   loss of the temperature peak, 1 - max(T - T0) / (A T0), in
                 percent after 15 t_c (Sec. IV.B.2)
  acoustic pulse pressure fluctuation dP = (rho T - P0) / (A P0) after 30
                 steps; the field at u0 > 0 moved back by u0 * 30 nodes is
                 compared with the u0 = 0 field: max |difference| / max dP(u0=0)
                 (Sec. IV.B.3; the paper shows these fields, no number)
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads as W  # noqa: E402

SHEAR_U0 = (2.0, 2.5, 3.0)
SPOT_U0 = (2.0, 2.5, 3.0)
ACOUSTIC_U0 = (0.0, 1.3, 2.6, 3.9)


def run(wl):
    s = oracle.Sim.from_workload(wl)
    s.step(wl.steps)
    return s.macros()


def shear_nu_num(m):
    return abs(W.LINEAR_A - float(m["uy"].max())) / W.LINEAR_A * 100.0


def spot_loss(m):
    dT = (m["T"] - W.T0) / (W.LINEAR_A * W.T0)
    return (1.0 - float(dT.max())) * 100.0


def acoustic_dp(m):
    P0 = W.RHO0 * W.T0
    return (m["rho"] * m["T"] - P0) / (W.LINEAR_A * P0)


def recentred(dp, u0, steps=W.ACOUSTIC_STEPS):
    shift = int(round(u0 * steps))
    return np.roll(dp, -shift, axis=1)


def main():
    out = {"_about": "Oracle figures for the linear-regime cases of Sec. IV.B, written by "
                     "tests/golden/make_linear_suite.py (CPU oracle only)."}
    out["shear_wave"] = {}
    for u0 in SHEAR_U0:
        wl = W.shear_wave(u0)
        m = run(wl)
        out["shear_wave"][str(u0)] = dict(steps=wl.steps, nu_num_percent=shear_nu_num(m))
        print("shear", u0, out["shear_wave"][str(u0)], flush=True)
    out["entropy_spot"] = {}
    for u0 in SPOT_U0:
        wl = W.entropy_spot(u0)
        m = run(wl)
        out["entropy_spot"][str(u0)] = dict(steps=wl.steps, peak_loss_percent=spot_loss(m))
        print("spot", u0, out["entropy_spot"][str(u0)], flush=True)
    out["acoustic_pulse"] = {}
    ref = None
    for u0 in ACOUSTIC_U0:
        dp = recentred(acoustic_dp(run(W.acoustic_pulse(u0))), u0)
        if ref is None:
            ref = dp
        out["acoustic_pulse"][str(u0)] = dict(
            steps=W.ACOUSTIC_STEPS, max_dp=float(dp.max()),
            recentred_max_diff=float(np.abs(dp - ref).max() / np.abs(ref).max()))
        print("acoustic", u0, out["acoustic_pulse"][str(u0)], flush=True)
    with open(os.path.join(HERE, "linear_suite_oracle.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
