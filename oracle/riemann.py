"""Exact solution of the one-dimensional Riemann problem for an ideal gas.

Test infrastructure (see the package docstring).  This is the textbook
construction the paper compares its Sod-tube results with (Sec. IV.C.1):
the star pressure solves f_L(p) + f_R(p) + (u_R - u_L) = 0, where f_K is the
shock (Rankine-Hugoniot) branch for p > p_K and the rarefaction (isentropic)
branch for p <= p_K; the solution is then sampled along x / t.

Units are the lattice units of the method: p = rho T with unit gas constant,
sound speed a = sqrt(gamma p / rho).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


@dataclass
class Star:
    p: float
    u: float
    rho_L: float
    rho_R: float
    shock_L: bool
    shock_R: bool


def _f_and_df(p, rho, pk, gamma):
    a = math.sqrt(gamma * pk / rho)
    if p > pk:  # shock branch
        A = 2.0 / ((gamma + 1.0) * rho)
        B = (gamma - 1.0) / (gamma + 1.0) * pk
        s = math.sqrt(A / (p + B))
        f = (p - pk) * s
        df = s * (1.0 - 0.5 * (p - pk) / (p + B))
    else:       # rarefaction branch
        e = (gamma - 1.0) / (2.0 * gamma)
        f = 2.0 * a / (gamma - 1.0) * ((p / pk) ** e - 1.0)
        df = 1.0 / (rho * a) * (p / pk) ** (-(gamma + 1.0) / (2.0 * gamma))
    return f, df


def star_state(left, right, gamma=1.4, tol=1e-15, max_iter=200) -> Star:
    """left/right = (rho, u, p).  Newton on the pressure function, started from
    the two-rarefaction approximation, then bisection-safeguarded."""
    rl, ul, pl = left
    rr, ur, pr = right
    al = math.sqrt(gamma * pl / rl)
    ar = math.sqrt(gamma * pr / rr)
    if 2.0 * (al + ar) / (gamma - 1.0) <= ur - ul:
        raise ValueError("vacuum is generated")
    z = (gamma - 1.0) / (2.0 * gamma)
    p = ((al + ar - 0.5 * (gamma - 1.0) * (ur - ul)) /
         (al / pl ** z + ar / pr ** z)) ** (1.0 / z)
    lo, hi = 0.0, max(pl, pr) * 1e3 + 1.0
    for _ in range(max_iter):
        fl, dl = _f_and_df(p, rl, pl, gamma)
        fr, dr = _f_and_df(p, rr, pr, gamma)
        F = fl + fr + ur - ul
        if F > 0:
            hi = min(hi, p)
        else:
            lo = max(lo, p)
        pn = p - F / (dl + dr)
        if not (lo < pn < hi):
            pn = 0.5 * (lo + hi)
        if abs(pn - p) <= tol * 0.5 * (pn + p):
            p = pn
            break
        p = pn
    fl, _ = _f_and_df(p, rl, pl, gamma)
    fr, _ = _f_and_df(p, rr, pr, gamma)
    u = 0.5 * (ul + ur) + 0.5 * (fr - fl)
    g1 = (gamma - 1.0) / (gamma + 1.0)

    def rho_star(rk, pk, shock):
        if shock:
            return rk * ((p / pk + g1) / (g1 * p / pk + 1.0))
        return rk * (p / pk) ** (1.0 / gamma)

    return Star(p, u, rho_star(rl, pl, p > pl), rho_star(rr, pr, p > pr), p > pl, p > pr)


def sample(left, right, xi, gamma=1.4, star: Star | None = None):
    """Primitive variables (rho, u, p) at similarity coordinates xi = x / t."""
    rl, ul, pl = left
    rr, ur, pr = right
    st = star or star_state(left, right, gamma)
    al = math.sqrt(gamma * pl / rl)
    ar = math.sqrt(gamma * pr / rr)
    xi = np.asarray(xi, dtype=np.float64)
    rho = np.empty_like(xi)
    u = np.empty_like(xi)
    p = np.empty_like(xi)
    g1 = (gamma - 1.0) / (gamma + 1.0)
    for k, s in np.ndenumerate(xi):
        if s <= st.u:  # left of the contact
            if st.shock_L:
                S = ul - al * math.sqrt((gamma + 1) / (2 * gamma) * st.p / pl +
                                        (gamma - 1) / (2 * gamma))
                val = (rl, ul, pl) if s <= S else (st.rho_L, st.u, st.p)
            else:
                a_star = al * (st.p / pl) ** ((gamma - 1) / (2 * gamma))
                head, tail = ul - al, st.u - a_star
                if s <= head:
                    val = (rl, ul, pl)
                elif s >= tail:
                    val = (st.rho_L, st.u, st.p)
                else:
                    fac = 2 / (gamma + 1) + (gamma - 1) / ((gamma + 1) * al) * (ul - s)
                    r = rl * fac ** (2 / (gamma - 1))
                    uu = 2 / (gamma + 1) * (al + (gamma - 1) / 2 * ul + s)
                    pp = pl * fac ** (2 * gamma / (gamma - 1))
                    val = (r, uu, pp)
        else:          # right of the contact
            if st.shock_R:
                S = ur + ar * math.sqrt((gamma + 1) / (2 * gamma) * st.p / pr +
                                        (gamma - 1) / (2 * gamma))
                val = (rr, ur, pr) if s >= S else (st.rho_R, st.u, st.p)
            else:
                a_star = ar * (st.p / pr) ** ((gamma - 1) / (2 * gamma))
                head, tail = ur + ar, st.u + a_star
                if s >= head:
                    val = (rr, ur, pr)
                elif s <= tail:
                    val = (st.rho_R, st.u, st.p)
                else:
                    fac = 2 / (gamma + 1) - (gamma - 1) / ((gamma + 1) * ar) * (ur - s)
                    r = rr * fac ** (2 / (gamma - 1))
                    uu = 2 / (gamma + 1) * (-ar + (gamma - 1) / 2 * ur + s)
                    pp = pr * fac ** (2 * gamma / (gamma - 1))
                    val = (r, uu, pp)
        rho[k], u[k], p[k] = val
    return rho, u, p


def shock_speed(left, right, gamma=1.4, side="R"):
    st = star_state(left, right, gamma)
    rl, ul, pl = left
    rr, ur, pr = right
    if side == "R":
        ar = math.sqrt(gamma * pr / rr)
        return ur + ar * math.sqrt((gamma + 1) / (2 * gamma) * st.p / pr + (gamma - 1) / (2 * gamma))
    al = math.sqrt(gamma * pl / rl)
    return ul - al * math.sqrt((gamma + 1) / (2 * gamma) * st.p / pl + (gamma - 1) / (2 * gamma))


def periodic_sod_profile(nx, t, x0, left, right, gamma=1.4, u0=0.0):
    """Exact fields at time t on a periodic row of nodes x = 0..nx-1 whose
    initial data is `left` = (rho, p) for x < x0 and `right` otherwise, both
    moving at velocity u0.  Two Riemann problems start at x0 - 1/2 and at the
    seam -1/2; the result is valid while their waves have not met."""
    L = (left[0], u0, left[1])
    R = (right[0], u0, right[1])
    x = np.arange(nx, dtype=np.float64)

    def rel(pos):  # displacement from an advected discontinuity, nearest image
        d = x - (pos + u0 * t)
        return (d + 0.5 * nx) % nx - 0.5 * nx

    da, db = rel(x0 - 0.5), rel(-0.5)
    ra, ua, pa = sample(L, R, u0 + da / t, gamma)
    rb, ub, pb = sample(R, L, u0 + db / t, gamma)
    use_a = np.abs(da) <= np.abs(db)
    return (np.where(use_a, ra, rb), np.where(use_a, ua, ub), np.where(use_a, pa, pb))
