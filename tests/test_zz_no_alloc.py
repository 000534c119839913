"""The allocation-free batched step (lbm_step_batched_noalloc: job table and
failure words in the library's fixed device array) against lbm_step_batched
(job table in the first context's workspace), through the C ABI: the same
populations bit for bit, on two calls in a row, the second with fewer and
smaller jobs, and sizes beyond the array refused."""
import ctypes as C

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lbm():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2009_13426_amd as lbm
    return lbm


def _call(lbm, fn, sims, steps):
    n = len(sims)
    arr = (C.c_void_p * n)(*[s.handle.value for s in sims])
    st = (C.c_int32 * n)(*[int(k) for k in steps])
    return getattr(lbm.lib, fn)(arr, st, n)


def _fields(sims):
    out = []
    for s in sims:
        f, g = s.populations()
        out.append((f.cpu().numpy(), g.cpu().numpy()))
    return out


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_noalloc_batched_equals_batched(lbm, precision):
    rounds = [
        # first call: four uneven jobs; second call: two smaller ones
        ([W.four_quadrant(72, 12, sub=1), W.isentropic_vortex(64, steps=12),
          W.four_quadrant(45, 12, sub=2), W.four_quadrant(96, 12, sub=3)], [12, 9, 12, 5]),
        ([W.four_quadrant(33, 8, sub=4), W.isentropic_vortex(40, steps=8)], [8, 6]),
    ]
    for r, (wls, steps) in enumerate(rounds):
        ref = [lbm.Sim.from_workload(wl, precision=precision) for wl in wls]
        got = [lbm.Sim.from_workload(wl, precision=precision) for wl in wls]
        print(f"{precision} call {r}: {len(wls)} jobs, sides {[wl.nx for wl in wls]}, "
              f"steps {steps}", flush=True)
        assert _call(lbm, "lbm_step_batched", ref, steps) == lbm.OK
        assert _call(lbm, "lbm_step_batched_noalloc", got, steps) == lbm.OK
        for (fa, ga), (fb, gb) in zip(_fields(ref), _fields(got)):
            assert np.array_equal(fa, fb) and np.array_equal(ga, gb)
        for s in ref + got:
            s.close()


def test_noalloc_batched_limits(lbm):
    sim = lbm.Sim.from_workload(W.four_quadrant(16, 1), precision="fp32")
    arr = (C.c_void_p * 1)(sim.handle.value)
    st = (C.c_int32 * 1)(1)
    assert lbm.lib.lbm_step_batched_noalloc(arr, st, 1025) == lbm.ERR_ARG
    assert lbm.lib.lbm_step_batched_noalloc(arr, st, -1) == lbm.ERR_ARG
    assert lbm.lib.lbm_step_batched_noalloc(arr, st, 0) == lbm.OK
    assert lbm.lib.lbm_step_batched_noalloc(arr, st, 1) == lbm.OK
    sim.close()
