"""The oracle against a second, independent implementation of the same model
on the simplest flow that exercises every part of a step in one lattice: a
vectorised numpy D2Q21 DDF-BGK on a periodic line of 100 nodes (Sec. IV.B.1,
the shear wave), written here from the paper's definitions and sharing no
code with the oracle.

What differs from the oracle: the populations are held node x velocity and
streamed with np.roll in the frame of the lattice (so its fields are the
oracle's translated by U per step: the Galilean shift, Sec. III.A); the
equilibrium is plain Newton from the lattice Maxwellian with a dense solve
(np.linalg.solve), not Gaussian elimination with Armijo steps; the targets
are the continuous Maxwellian's moments of the 8-moment set (eqs.
G0_8mom-G3yaa_8mom).  Common to both, as the model itself: the velocity set
of reading D-1, g_eq = (2 Cv - D) T f_eq (eq. gEq), tau = 1/2 at nu = 0
and the collision of eq. (coll).

A dropped or mis-signed term in the oracle's moments, targets, Hessian,
streaming or collision moves these fields by far more than the 1e-10 (of
the wave's amplitude) the two agree to."""
import json
import math
import os

import numpy as np
import pytest

import oracle
import workloads as W

# D2Q21 (reading D-1): rest, then the +- pairs of (1,0) (0,1) (1,1) (1,-1)
# (2,0) (0,2) (2,2) (2,-2) (3,0) (0,3)
PAIRS = [(1, 0), (0, 1), (1, 1), (1, -1), (2, 0), (0, 2), (2, 2), (2, -2), (3, 0), (0, 3)]
CX = np.array([0.0] + [s * p[0] for p in PAIRS for s in (1, -1)])
CY = np.array([0.0] + [s * p[1] for p in PAIRS for s in (1, -1)])
SQ = CX * CX + CY * CY
PHI = np.stack([np.ones(21), CX, CY, CX * CX, CX * CY, CY * CY, CX * SQ, CY * SQ], 1)
GAMMA = 1.4
CV = 1.0 / (GAMMA - 1.0)   # per unit mass, R = 1
D = 2


def maxwellian_targets(ux, uy, T):
    """Per-unit-density moments of the 2D Maxwellian for phi = (1, x, y, x^2,
    xy, y^2, x|xi|^2, y|xi|^2): <xi_a xi_b> = u_a u_b + T delta_ab and
    <xi_a |xi|^2> = u_a (|u|^2 + (D + 2) T)."""
    u2 = ux * ux + uy * uy
    return np.stack([np.ones_like(ux), ux, uy, ux * ux + T, ux * uy, uy * uy + T,
                     ux * (u2 + (D + 2) * T), uy * (u2 + (D + 2) * T)], 1)


def equilibrium_weights(ux, uy, T, tol=1e-12):
    """w_i = exp(-lambda . phi_i) with sum_i w_i phi_i = targets, by Newton
    from the lattice Maxwellian (one final step after the tolerance)."""
    m = maxwellian_targets(ux, uy, T)
    lam = np.zeros((ux.size, 8))
    lam[:, 1], lam[:, 2] = -ux / T, -uy / T
    lam[:, 3] = lam[:, 5] = 0.5 / T
    lam[:, 0] = np.log(np.exp(-(lam[:, 1:] @ PHI[:, 1:].T)).sum(1))
    for _ in range(50):
        w = np.exp(-(lam @ PHI.T))
        G = w @ PHI - m
        H = np.einsum("ni,ia,ib->nab", w, PHI, PHI)
        lam = lam + np.linalg.solve(H, G[..., None])[..., 0]
        if np.abs(G).max() <= tol:
            return np.exp(-(lam @ PHI.T))
    raise RuntimeError("Newton did not converge")


def line_run(u0, steps, L=100):
    """Shear wave of workloads.shear_wave in the lattice U = ceil(u0 - 1/2),
    populations in that lattice's frame; returns (rho, u_x, u_y, T) in
    absolute velocities, translated back by U per step."""
    wl = W.shear_wave(u0, L, steps)
    U = math.ceil(u0 - 0.5)
    rho = wl.rho.ravel().copy()
    ux = wl.ux.ravel() - U
    uy = wl.uy.ravel().copy()
    T = wl.T.ravel().copy()
    f = rho[:, None] * equilibrium_weights(ux, uy, T)
    g = (2 * CV - D) * T[:, None] * f
    shift = CX.astype(int)
    for _ in range(steps):
        f = np.stack([np.roll(f[:, k], shift[k]) for k in range(21)], 1)
        g = np.stack([np.roll(g[:, k], shift[k]) for k in range(21)], 1)
        rho = f.sum(1)
        ux, uy = (f @ CX) / rho, (f @ CY) / rho
        T = (f @ SQ + g.sum(1) - rho * (ux * ux + uy * uy)) / (2 * rho * CV)
        fe = rho[:, None] * equilibrium_weights(ux, uy, T)
        ge = (2 * CV - D) * T[:, None] * fe
        f, g = 2.0 * fe - f, 2.0 * ge - g       # tau = 1/2 (nu = 0)
    back = lambda a: np.roll(a, U * steps)   # the lattice moved by U per step
    return back(rho), back(ux) + U, back(uy), back(T)


@pytest.mark.parametrize("u0", [2.0, 2.5, 3.0])
def test_independent_line_solver_matches_the_oracle(u0):
    steps = 50
    wl = W.shear_wave(u0, steps=steps)
    s = oracle.Sim.from_workload(wl)
    s.step(steps)
    m = {k: v.ravel() for k, v in s.macros().items()}
    rho, ux, uy, T = line_run(u0, steps)
    A = wl.meta["A"]
    err = dict(rho=np.abs(rho - m["rho"]).max(), T=np.abs(T - m["T"]).max() / W.T0,
               ux=np.abs(ux - m["ux"]).max() / u0, uy=np.abs(uy - m["uy"]).max() / A)
    print(u0, {k: f"{v:.1e}" for k, v in err.items()})
    assert max(err.values()) <= 1e-10, err
    # the wave itself is there (a translation error would flip it)
    assert np.abs(m["uy"]).max() > 0.99 * A


def test_independent_line_solver_reproduces_the_stored_dissipation():
    """nu_num of Sec. IV.B.1 after 15 t_c, against the oracle's stored
    figures (tests/golden/linear_suite_oracle.json) to 1e-3 relative."""
    path = os.path.join(os.path.dirname(__file__), "golden", "linear_suite_oracle.json")
    stored = json.load(open(path))["shear_wave"]
    for u0 in (2.0, 2.5, 3.0):
        steps = W.linear_steps(u0)
        _, _, uy, _ = line_run(u0, steps)
        nu = 100 * abs(W.LINEAR_A - uy.max()) / W.LINEAR_A
        want = stored[str(u0)]["nu_num_percent"]
        print(u0, steps, f"{nu:.5f} % (oracle {want:.5f} %)")
        assert abs(nu - want) <= 1e-3 * want, (u0, nu, want)
