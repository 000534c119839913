"""Pins of the exact ideal-gas Riemann solver (oracle/riemann.py) to the
jump conditions, the isentropic relations and tabulated textbook values."""
import json
import math
import os

import numpy as np
import pytest

from oracle import riemann as R

TORO = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "sod_textbook.json")))
G = 1.4
L, Rt = (1.0, 0.0, 1.0), (0.125, 0.0, 0.1)


def test_sod_star_state_matches_table():
    st = R.star_state(L, Rt, G)
    assert abs(st.p - TORO["p_star"]) < 1e-5
    assert abs(st.u - TORO["u_star"]) < 1e-5
    assert abs(st.rho_L - TORO["rho_star_L"]) < 1e-5
    assert abs(st.rho_R - TORO["rho_star_R"]) < 1e-5
    assert not st.shock_L and st.shock_R


@pytest.mark.parametrize("left,right", [(L, Rt), ((1.0, 0.3, 1.0), (0.5, -0.4, 0.4)),
                                        ((0.8, 2.0, 0.6), (1.3, 1.1, 1.2))])
def test_rankine_hugoniot_and_isentropes(left, right):
    st = R.star_state(left, right, G)
    for side, (rk, uk, pk), rs in [("L", left, st.rho_L), ("R", right, st.rho_R)]:
        shock = st.shock_L if side == "L" else st.shock_R
        if shock:
            S = R.shock_speed(left, right, G, side)
            m0, m1 = rk * (uk - S), rs * (st.u - S)             # mass flux
            assert abs(m0 - m1) < 1e-12 * max(1, abs(m0))
            assert abs(m0 * (uk - S) + pk - (m1 * (st.u - S) + st.p)) < 1e-12
            e0 = pk / (rk * (G - 1)) + 0.5 * (uk - S) ** 2 + pk / rk
            e1 = st.p / (rs * (G - 1)) + 0.5 * (st.u - S) ** 2 + st.p / rs
            assert abs(e0 - e1) < 1e-12 * abs(e0)              # total enthalpy
        else:
            assert abs(pk / rk ** G - st.p / rs ** G) < 1e-12 * pk / rk ** G
            a0, a1 = math.sqrt(G * pk / rk), math.sqrt(G * st.p / rs)
            sgn = 1 if side == "L" else -1                        # Riemann invariants
            assert abs((uk + sgn * 2 * a0 / (G - 1)) - (st.u + sgn * 2 * a1 / (G - 1))) < 1e-12


def test_rarefaction_fan_is_isentropic_and_continuous():
    xi = np.linspace(-1.5, 0.0, 301)
    rho, u, p = R.sample(L, Rt, xi, G)
    assert np.allclose(p / rho ** G, 1.0, rtol=1e-12)
    a = np.sqrt(G * p / rho)
    assert np.allclose(u + 2 * a / (G - 1), 2 * math.sqrt(G) / (G - 1), rtol=1e-12)
    assert np.all(np.diff(rho) <= 1e-15)


def test_periodic_profile_has_both_problems():
    rho, u, p = R.periodic_sod_profile(256, 20, 128, (1, 1), (0.125, 0.1))
    assert rho[128 + 25] == pytest.approx(R.star_state(L, Rt).rho_R)   # between contact and shock
    assert rho[128 + 10] == pytest.approx(R.star_state(L, Rt).rho_L)   # between fan and contact
    assert u[5] < 0 and u[150] > 0          # mirrored problem at the seam moves left
    assert rho[60] == 1.0 and rho[200] == 0.125
