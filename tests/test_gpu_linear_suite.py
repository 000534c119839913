"""The linear-regime cases of Sec. IV.B on the GPU (inviscid, tau = 1/2,
hysteresis half-width 0.51), through the C ABI: parity with the oracle over
the paper's full horizons, and the figures the paper reports (shear-wave
dissipation, entropy-spot peak loss) equal to the oracle's stored ones
(tests/golden/linear_suite_oracle.json).  Metrics and tolerances as in
test_gpu_parity.py: FP64 1e-12, FP32 storage 1e-5 (no sensor here).

The figures measure a perturbation of relative size A = 1e-3 on a mean
state, so a field error bounded by TOL relative to the mean moves them by
up to TOL / A of the perturbation: FP32 rounding (TOL 1e-5) can move the
shear-wave figure by up to 100 * 1e-5 * max|u| / A percentage points and
the entropy-spot figure by up to 100 * 1e-5 / A; those derived bounds are
the ones asserted for FP32, with the FP64 ones at 1e-7 points.

At u0 = 2.5 every node sits at relative velocity 1/2 in its lattice (the
edge of the shift range), where the inviscid scheme (tau = 1/2) has a weakly
unstable two-dimensional mode: on the oracle alone, noise of 1e-8 seeded in
the density grows tenfold per 100 steps after step 200 (the one-dimensional
shear wave shows no growth).  Seeded by FP64 rounding it stays near 1e-10
over the 600 steps, so the FP64 entropy spot at 2.5 is held to 1e-9 (field)
and 1e-4 points (figure); seeded by FP32 storage rounding it reaches the
size of the spot itself, so the FP32 form cannot carry that case over 15 t_c
(strict expected failure) and is checked over 200 steps instead.

The acoustic pulse at u0 = 0 has no mean flow, so velocity errors are taken
relative to the sound speed sqrt(gamma T0) instead of max |u| (which is
there the pulse's own ~1e-4 velocity)."""
import json
import os
import sys

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))
import make_linear_suite as M  # noqa: E402

LIN = json.load(open(os.path.join(HERE, "golden", "linear_suite_oracle.json")))
TOL = {"fp64": 1e-12, "fp32": 1e-5}


@pytest.fixture(scope="module")
def lbm():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2009_13426_amd as lbm
    return lbm


def gpu(lbm, wl, precision):
    sim = lbm.Sim.from_workload(wl, precision=precision)
    sim.step(wl.steps)
    m = {k: v.cpu().numpy() for k, v in sim.macros().items()}
    sim.close()
    return m


def errors(orc, got, ref, u_scale=0.0):
    """D-20 metrics; velocity errors relative to max(max |u_ref|, u_scale)."""
    du = np.hypot(got["ux"] - ref["ux"], got["uy"] - ref["uy"]).max()
    um = max(float(np.hypot(ref["ux"], ref["uy"]).max()), u_scale)
    return dict(rho=orc.rel_err_scalar(got["rho"], ref["rho"]), u=float(du / um),
                T=orc.rel_err_scalar(got["T"], ref["T"]))


SOUND_SPEED = (W.GAMMA * W.T0) ** 0.5
UNSTABLE_FP32 = pytest.mark.xfail(
    strict=True, reason="u0 = 2.5 puts every node at relative velocity 1/2, where the inviscid "
                        "scheme has a weakly unstable mode that FP32 storage rounding seeds "
                        "(grows tenfold per 100 steps); the FP32 form cannot carry it over 15 t_c")
# field bound (relative) at the full horizon: u0 = 2.5 grows FP64 rounding to ~1e-10
SPOT_FP64_FIELD = {2.0: 1e-12, 2.5: 1e-9, 3.0: 1e-12}


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("u0", [2.0, 2.5, 3.0])
def test_shear_wave(lbm, orc, u0, precision):
    wl = W.shear_wave(u0)
    got = gpu(lbm, wl, precision)
    ref = M.run(wl)
    e = errors(orc, got, ref)
    nu = M.shear_nu_num(got)
    print(f"shear u0={u0} {precision} ({wl.steps} steps): {e}, nu_num {nu:.5f} % "
          f"(oracle {LIN['shear_wave'][str(u0)]['nu_num_percent']:.5f} %)", flush=True)
    assert max(e.values()) <= TOL[precision], e
    assert np.array_equal(got["Ux"], ref["Ucx"]) and np.array_equal(got["Uy"], ref["Ucy"])
    want = LIN["shear_wave"][str(u0)]["nu_num_percent"]
    bound = 1e-7 if precision == "fp64" else \
        100 * TOL["fp32"] * float(np.hypot(ref["ux"], ref["uy"]).max()) / W.LINEAR_A
    assert abs(nu - want) <= bound, (nu, want, bound)


@pytest.mark.parametrize("u0,precision", [
    (2.0, "fp64"), (2.5, "fp64"), (3.0, "fp64"), (2.0, "fp32"),
    pytest.param(2.5, "fp32", marks=UNSTABLE_FP32), (3.0, "fp32")])
def test_entropy_spot_peak_loss(lbm, u0, precision):
    wl = W.entropy_spot(u0)
    got = gpu(lbm, wl, precision)
    loss = M.spot_loss(got)
    want = LIN["entropy_spot"][str(u0)]["peak_loss_percent"]
    print(f"entropy spot u0={u0} {precision}: peak loss {loss:.6f} % (oracle {want:.6f} %)",
          flush=True)
    field = SPOT_FP64_FIELD[u0] if precision == "fp64" else TOL["fp32"]
    bound = 100 * field / W.LINEAR_A
    assert abs(loss - want) <= bound, (loss, want, bound)


@pytest.mark.parametrize("u0", [2.0, 2.5])
def test_entropy_spot_field_parity(lbm, orc, u0):
    wl = W.entropy_spot(u0)
    got = gpu(lbm, wl, "fp64")
    ref = M.run(wl)
    e = errors(orc, got, ref)
    print(f"entropy spot u0={u0} fp64 ({wl.steps} steps): {e}", flush=True)
    assert max(e.values()) <= SPOT_FP64_FIELD[u0], e


def test_entropy_spot_fp32_before_the_mode_grows(lbm, orc):
    wl = W.entropy_spot(2.5, steps=200)
    got = gpu(lbm, wl, "fp32")
    ref = M.run(wl)
    e = errors(orc, got, ref)
    print(f"entropy spot u0=2.5 fp32 (200 steps): {e}", flush=True)
    assert max(e.values()) <= TOL["fp32"], e


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_acoustic_pulse(lbm, orc, precision):
    base = None
    for u0 in M.ACOUSTIC_U0:
        wl = W.acoustic_pulse(u0)
        got = gpu(lbm, wl, precision)
        ref = M.run(wl)
        e = errors(orc, got, ref, u_scale=SOUND_SPEED)
        dp = M.recentred(M.acoustic_dp(got), u0)
        if base is None:
            base = dp
        diff = float(np.abs(dp - base).max() / np.abs(base).max())
        want = LIN["acoustic_pulse"][str(u0)]["recentred_max_diff"]
        print(f"acoustic u0={u0} {precision}: {e}, recentred diff {diff:.6e} (oracle {want:.6e})",
              flush=True)
        assert max(e.values()) <= TOL[precision], e
        bound = 1e-9 if precision == "fp64" else 2 * TOL["fp32"] / W.LINEAR_A / float(base.max())
        assert abs(diff - want) <= bound, (diff, want, bound)
