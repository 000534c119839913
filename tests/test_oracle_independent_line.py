"""The oracle against a second, independent implementation of the same model:
a vectorised numpy D2Q21 DDF-BGK on periodic grids, written here from the
paper's definitions and sharing no code with the oracle.  First on the
shear wave in one lattice (Sec. IV.B.1), then with lattices that follow the
flow, rebuilt links and the sensor (a1-a6 of the step) on lines and on
small 2D grids, with every constraint set (8 and 4 on D2Q21, 13 on
D2Q49), shift mode and the flexible-Prandtl collision.

What differs from the oracle: the populations are held node x velocity and
streamed with np.roll (in the one-lattice case in the frame of the lattice,
so its fields are the oracle's translated by U per step: the Galilean shift,
Sec. III.A); the equilibrium is Newton from the lattice Maxwellian with a
dense solve (np.linalg.solve) and step halving on the dual, not Gaussian
elimination with Armijo steps; the targets are the continuous Maxwellian's
moments of the 8-moment set (eqs. G0_8mom-G3yaa_8mom).  Common to both, as
the model itself and its readings: the velocity set of reading D-1, g_eq =
(2 Cv - D) T f_eq (eq. gEq), tau = 1/2 + nu/T and the collision of eq.
(coll), the one-step lag of the lattice choice (reading D-4), Grad's
rebuild with phi_g as printed (reading D-6) and the source's tau (reading
D-RB), the sensor's alpha (reading D-S).

A dropped or mis-signed term in the oracle's moments, targets, Hessian,
streaming, rebuild or collision moves these fields by far more than the
1e-10 the two agree to."""
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
# the reference model's lattice (App. C): D2Q49 = {0, +-1, +-2, +-3}^2
CX49 = np.array([float(x) for y in range(-3, 4) for x in range(-3, 4)])
CY49 = np.array([float(y) for y in range(-3, 4) for x in range(-3, 4)])


def lattice(Q):
    """(c_x, c_y, |c|^2) of D2Q21 or D2Q49."""
    cx, cy = (CX, CY) if Q == 21 else (CX49, CY49)
    return cx, cy, cx * cx + cy * cy
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


def equilibrium_weights(ux, uy, T, tol=1e-12, constraints=8):
    """w_i = exp(-lambda . phi_i) with sum_i w_i phi_i = targets: Newton from
    the lattice Maxwellian on the convex dual Psi = sum_i w_i + lambda . m,
    each step halved while it raises Psi (one final full step after the
    tolerance)."""
    if constraints == 8:
        phi, m = PHI, maxwellian_targets(ux, uy, T)
        lam = np.zeros((ux.size, 8))
        lam[:, 3] = lam[:, 5] = 0.5 / T
    elif constraints == 13:
        # eqs. (G0)-(G4yyaa) on D2Q49: moments up to the third order and the
        # contracted fourth ones, E = |u|^2 / 2 + T
        cx, cy, sq = lattice(49)
        phi = np.stack([np.ones(49), cx, cy, cx * cx, cx * cy, cy * cy, cx ** 3, cx * cx * cy,
                        cx * cy * cy, cy ** 3, cx * cx * sq, cx * cy * sq, cy * cy * sq], 1)
        E = 0.5 * (ux * ux + uy * uy) + T
        m = np.stack([np.ones_like(ux), ux, uy, ux * ux + T, ux * uy, uy * uy + T,
                      ux * (ux * ux + 3 * T), (ux * ux + T) * uy, ux * (uy * uy + T),
                      uy * (uy * uy + 3 * T), 2 * ((E + 2 * T) * ux * ux + (E + T) * T),
                      2 * (E + 2 * T) * ux * uy, 2 * ((E + 2 * T) * uy * uy + (E + T) * T)], 1)
        lam = np.zeros((ux.size, 13))
        lam[:, 3] = lam[:, 5] = 0.5 / T
    else:  # mass, momentum and energy only (eq. feqNum_4Mom)
        phi = np.stack([np.ones(21), CX, CY, SQ], 1)
        m = np.stack([np.ones_like(ux), ux, uy, ux * ux + uy * uy + D * T], 1)
        lam = np.zeros((ux.size, 4))
        lam[:, 3] = 0.5 / T
    lam[:, 1], lam[:, 2] = -ux / T, -uy / T
    lam[:, 0] = np.log(np.exp(-(lam[:, 1:] @ phi[:, 1:].T)).sum(1))
    psi = lambda l: np.exp(-(l @ phi.T)).sum(1) + (l * m).sum(1)
    done = np.zeros(ux.size, dtype=bool)
    for _ in range(200):
        w = np.exp(-(lam @ phi.T))
        G = w @ phi - m
        H = np.einsum("ni,ia,ib->nab", w, phi, phi)
        d = np.linalg.solve(H, G[..., None])[..., 0]
        conv = np.abs(G).max(1) <= tol
        step = np.ones(ux.size)
        p0 = psi(lam)
        for _ in range(60):       # backtracking where the full step raises Psi
            # (a rise within rounding of Psi is no rise: near the root Psi
            # changes by |G|^2, far below its last bit; an overflow is a rise)
            bad = ~conv & ~done & ~(psi(lam + step[:, None] * d) <= p0 + 1e-13 * np.abs(p0))
            if not bad.any():
                break
            step = np.where(bad, 0.5 * step, step)
        lam = np.where(done[:, None], lam, lam + step[:, None] * d)
        done |= conv
        if done.all():
            return np.exp(-(lam @ phi.T))
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


# --------------------------------------------------- adaptive line (a1-a6)
# The same independent model with lattices that follow the flow: each node
# pulls in the lattice it selected at its last collision (reading D-4), a
# link whose source collided in another lattice is rebuilt by Grad's ansatz
# (eqs. GradGeneral, GradGeneral_f, GradGeneral_g; phi_g as printed, reading
# D-6) from the source's moments and the central differences of its
# neighbours', post-collision with the source's tau = 1/2 + nu/T (reading
# D-RB), and the next lattice is ceil(u - 1/2) unless u stays within the
# half-width of the current one (eq. criterion, Sec. III.A.2).  On a line
# one node tall every y-difference is zero.

def sensor_alpha(eps):
    """Reading D-S: 1 up to 1e-2, then the levels 1.05, 1.35 and 2 from 1e-2,
    1e-1 and 1 on, each reached by a linear ramp over the first tenth of its
    decade."""
    a = np.ones_like(eps)
    for lo, below, level in ((1e-2, 1.0, 1.05), (1e-1, 1.05, 1.35), (1.0, 1.35, 2.0)):
        ramp = below + (eps - lo) / (0.1 * lo) * (level - below)
        a = np.where(eps > lo, np.minimum(ramp, level), a)
    return a


def grad_pops(rho, ux, uy, T, du, dT, Lx, Ly, nu, k, constraints=8, pr=1.0, post_tau=None):
    """h_eq (1 + k phi_h) of eqs. (GradGeneral_f), (GradGeneral_g) in lattice
    (Lx, Ly) at absolute (rho, u, T); du = (d_x u_x, d_y u_x, d_x u_y,
    d_y u_y), dT = (d_x T, d_y T); mu = rho nu, kappa = rho Cp nu (unit
    Prandtl number)."""
    Cp = GAMMA * CV
    w = equilibrium_weights(ux - Lx, uy - Ly, T, constraints=constraints)
    CXq, CYq, _ = lattice(w.shape[1])
    cx = CXq[None, :] + Lx[:, None] - ux[:, None]
    cy = CYq[None, :] + Ly[:, None] - uy[:, None]
    mu = rho * nu
    div = du[0] + du[3]
    sxx = -mu * (2.0 * du[0] - (2.0 / D) * div)
    syy = -mu * (2.0 * du[3] - (2.0 / D) * div)
    sxy = -mu * (du[1] + du[2])
    kappa = rho * Cp * nu / pr
    qc = -kappa[:, None] * (dT[0][:, None] * cx + dT[1][:, None] * cy)
    c2 = cx * cx + cy * cy
    r, t = rho[:, None], T[:, None]
    phif = (sxx[:, None] * cx * cx + 2 * sxy[:, None] * cx * cy + syy[:, None] * cy * cy) \
        / (2 * r * t * t) + qc / (r * Cp * t * t) * (c2 / (2 * t) - Cp)
    phig = 2.0 * qc / (r * Cp)
    feq = r * w
    geq = (2 * CV - D) * t * feq
    k = np.broadcast_to(np.asarray(k, dtype=np.float64), rho.shape)[:, None]
    if pr != 1.0 and post_tau is not None:
        # eq. (Shakhov) applied to the Grad populations (App. E): their heat
        # flux in the receiver's frame, then each link's share of the term
        fg, gg = feq * (1 + phif), geq * (1 + phig)
        upx, upy = ux - Lx, uy - Ly
        qx, qy = heat_flux(fg, gg, upx, upy)
        sf, sg = shakhov_shapes(feq, upx, upy, rho, T, qx, qy)
        tau = post_tau
        ks = (1.0 / tau - 1.0 / (0.5 + (tau - 0.5) / pr))[:, None]
        return feq + k * (fg - feq) + ks * feq * sf, geq + k * (gg - geq) + ks * geq * sg
    return feq * (1 + k * phif), geq * (1 + k * phig)


def shakhov_shapes(feq, upx, upy, rho, T, qx, qy):
    """Reading D-Pr of eq. (Shakhov): phi_S,f = q.cbar / (rho Cp T^2)
    (|cbar|^2 / (2T) - (D + 2)/2), phi_S,g = q.cbar / (rho Cp T^2), cbar =
    xi - u' in the lattice's frame, with f_eq phi_S,f made free of mass,
    momentum and energy by removing its f_eq-weighted projection on (1,
    cbar_x, cbar_y, |cbar|^2)."""
    Cp = GAMMA * CV
    CXq, CYq, _ = lattice(feq.shape[1])
    cx = CXq[None, :] - upx[:, None]
    cy = CYq[None, :] - upy[:, None]
    c2 = cx * cx + cy * cy
    a = (qx[:, None] * cx + qy[:, None] * cy) / (rho * Cp * T * T)[:, None]
    sf = a * (c2 / (2 * T[:, None]) - 0.5 * (D + 2))
    e = np.stack([np.ones_like(cx), cx, cy, c2], 2)                 # n x 21 x 4
    gram = np.einsum("ni,nij,nik->njk", feq, e, e)
    r = np.einsum("ni,ni,nij->nj", feq, sf, e)
    beta = np.linalg.solve(gram, r[..., None])[..., 0]
    return sf - np.einsum("nij,nj->ni", e, beta), a


def heat_flux(f, g, upx, upy):
    """q = (1/2) sum_i cbar_i (|cbar_i|^2 f_i + g_i), cbar = xi - u'."""
    CXq, CYq, _ = lattice(f.shape[1])
    cx = CXq[None, :] - upx[:, None]
    cy = CYq[None, :] - upy[:, None]
    h = (cx * cx + cy * cy) * f + g
    return 0.5 * (cx * h).sum(1), 0.5 * (cy * h).sum(1)


def central(a, nx, ny):
    """Periodic central differences of a field stored row-major (ny rows of
    nx nodes): (d_x a, d_y a), flattened."""
    a = a.reshape(ny, nx)
    return (0.5 * (np.roll(a, -1, 1) - np.roll(a, 1, 1))).ravel(), \
        (0.5 * (np.roll(a, -1, 0) - np.roll(a, 1, 0))).ravel()


def gradients(ux, uy, T, nx, ny):
    (uxx, uxy), (uyx, uyy), (Tx, Ty) = (central(a, nx, ny) for a in (ux, uy, T))
    return (uxx, uxy, uyx, uyy), (Tx, Ty)


class AdaptiveGrid:
    """The adaptive model on a periodic nx x ny grid (row-major nodes)."""

    def __init__(self, wl, constraints=8, shift_mode=None, halfwidth=None, prandtl=1.0):
        self.nu, self.sensor, self.pr = wl.nu, wl.sensor, prandtl
        self.hw = wl.halfwidth if halfwidth is None else halfwidth
        self.mode = wl.shift_mode if shift_mode is None else shift_mode
        self.M = constraints
        self.nx, self.ny = wl.nx, wl.ny
        rho, ux, uy, T = (a.ravel().copy() for a in (wl.rho, wl.ux, wl.uy, wl.T))
        if self.mode == 2:      # static lattice map (Sec. IV.C.1)
            self.static = tuple(np.asarray(a).ravel().astype(int) for a in wl.static_U)
            Lx, Ly = self.static
        elif self.mode == 1:    # one fixed lattice
            Lx = np.full(rho.size, wl.fixed_U[0])
            Ly = np.full(rho.size, wl.fixed_U[1])
        else:
            Lx = np.ceil(ux - 0.5).astype(int)
            Ly = np.ceil(uy - 0.5).astype(int)
        # Grad initial condition (Sec. IV.A.1, reading: pre-collision), then a collision
        du, dT = gradients(ux, uy, T, self.nx, self.ny)
        f, g = grad_pops(rho, ux, uy, T, du, dT, Lx, Ly, self.nu, 1.0, self.M, self.pr)
        self.collide(f, g, Lx, Ly)

    def select(self, u, L):
        keep = (u > L - self.hw) & (u <= L + self.hw)
        return np.where(keep, L, np.ceil(u - 0.5).astype(int))

    def select_next(self, ux, uy, Lx, Ly):
        """The lattice of the next pull.  Mode 0: eq. (criterion) with the
        half-width kept around the current lattice; 1 and 2: the fixed or
        static one; 3 (reading of Sec. III.A.2 for overlapping ranges, half-
        width below 1): among the admissible pairs (n - w < u <= n + w per
        axis) the one the most of the four nearest neighbours collide in at
        this step, ties to the current lattice, then to ceil(u - 1/2), then
        to the first pair by increasing x and then y shift."""
        if self.mode == 1:
            return Lx, Ly
        if self.mode == 2:
            return self.static
        if self.mode == 0:
            return self.select(ux, Lx), self.select(uy, Ly)
        grid = lambda a: a.reshape(self.ny, self.nx)
        nbs = [(np.roll(grid(Lx), sh, ax).ravel(), np.roll(grid(Ly), sh, ax).ravel())
               for ax in (0, 1) for sh in (1, -1)]
        px, py = np.ceil(ux - 0.5).astype(int), np.ceil(uy - 0.5).astype(int)
        best = np.full(ux.size, -1)
        bx, by = px.copy(), py.copy()
        for dx in (-1, 0, 1):
            cx = px + dx
            okx = (ux > cx - self.hw) & (ux <= cx + self.hw)
            for dy in (-1, 0, 1):
                cy = py + dy
                ok = okx & (uy > cy - self.hw) & (uy <= cy + self.hw)
                score = sum(((nx_ == cx) & (ny_ == cy)).astype(int) for nx_, ny_ in nbs)
                rank = 4 * score + 2 * ((cx == Lx) & (cy == Ly)) + ((cx == px) & (cy == py))
                take = ok & (rank > best)
                best = np.where(take, rank, best)
                bx, by = np.where(take, cx, bx), np.where(take, cy, by)
        return bx, by

    def collide(self, f, g, Lx, Ly):
        cxq, cyq, sqq = lattice(f.shape[1])
        rho = f.sum(1)
        upx, upy = (f @ cxq) / rho, (f @ cyq) / rho
        T = (f @ sqq + g.sum(1) - rho * (upx * upx + upy * upy)) / (2 * rho * CV)
        ux, uy = upx + Lx, upy + Ly
        feq = rho[:, None] * equilibrium_weights(upx, upy, T, constraints=self.M)
        geq = (2 * CV - D) * T[:, None] * feq
        tau = 0.5 + self.nu / T
        if self.sensor:
            tau = tau * sensor_alpha(np.mean(np.abs(f - feq) / feq, axis=1))
        f1 = f - (f - feq) / tau[:, None]
        g1 = g - (g - geq) / tau[:, None]
        if self.pr != 1.0:
            # eq. (Shakhov): BGK plus (1/tau - 1/tau_Pr) h_eq phi_S, with q the
            # heat flux of the populations being collided
            qx, qy = heat_flux(f, g, upx, upy)
            sf, sg = shakhov_shapes(feq, upx, upy, rho, T, qx, qy)
            ks = (1.0 / tau - 1.0 / (0.5 + (tau - 0.5) / self.pr))[:, None]
            f1 = f1 + ks * feq * sf
            g1 = g1 + ks * geq * sg
        self.f, self.g = f1, g1
        self.mac = (rho, ux, uy, T)
        self.Uc = (Lx, Ly)
        self.Un = self.select_next(ux, uy, Lx, Ly)
        return self

    def step(self):
        Lx, Ly = self.Un
        n = np.arange(self.nx * self.ny)
        x, y = n % self.nx, n // self.nx
        cxq, cyq, _ = lattice(self.f.shape[1])
        sx = (x[:, None] - (cxq.astype(int)[None, :] + Lx[:, None])) % self.nx
        sy = (y[:, None] - (cyq.astype(int)[None, :] + Ly[:, None])) % self.ny
        src = sy * self.nx + sx                                   # node x plane
        same = (self.Uc[0][src] == Lx[:, None]) & (self.Uc[1][src] == Ly[:, None])
        planes = np.arange(cxq.size)[None, :]
        f = np.where(same, self.f[src, planes], 0.0)
        g = np.where(same, self.g[src, planes], 0.0)
        nodes, ks = np.nonzero(~same)
        if nodes.size:
            s = src[nodes, ks]
            rho, ux, uy, T = (a[s] for a in self.mac)
            du, dT = gradients(*self.mac[1:], self.nx, self.ny)
            hf, hg = grad_pops(rho, ux, uy, T, [d[s] for d in du], [d[s] for d in dT],
                               Lx[nodes], Ly[nodes], self.nu, 1.0 - 1.0 / (0.5 + self.nu / T),
                               self.M, self.pr, post_tau=0.5 + self.nu / T)
            f[nodes, ks] = hf[np.arange(nodes.size), ks]
            g[nodes, ks] = hg[np.arange(nodes.size), ks]
        self.rebuilt = nodes.size
        return self.collide(f, g, Lx, Ly)


ADAPTIVE_CASES = {
    # advected Sod (Mach 2 of the driver state), half-width 0.6, sensor on
    # (without it both implementations' equilibrium fails at step 5 on a
    # rebuilt link at |u'| = 2.1): about 80 rebuilt links a step
    "advected_sod_sensor": lambda steps: W.config1(256, 1, steps, halfwidth=0.6),
    # Sod on a flow at u = 1.45, next to the lattice boundary 1.5, nu = 1e-2,
    # plain criterion, no sensor: about 280 rebuilt links a step
    "sod_at_lattice_boundary": lambda steps: W.sod(256, 1, u0=1.45, nu=1e-2, shift_mode=0,
                                                   halfwidth=0.5, sensor=0, steps=steps),
    # 2D: the four-quadrant draw of the benchmark at 64^2, the Table 1
    # Riemann problem at 48^2 and the advected vortex at 48^2 (sensor on,
    # y-gradients, shear stress and heat flux in both directions); 1 000 to
    # 6 000 rebuilt links a step
    "four_quadrant_64": lambda steps: W.four_quadrant(64, steps),
    "riemann_table1_48": lambda steps: W.riemann_table1(48, steps=steps),
    "vortex_48": lambda steps: W.config2(48, steps),
}
ADAPTIVE_STEPS = {"four_quadrant_64": 20, "riemann_table1_48": 20, "vortex_48": 20,
                  "four_quadrant_64_four_constraints": 20}
# the four-constraint set (next item f3, eq. feqNum_4Mom) on the same draw
ADAPTIVE_CASES["four_quadrant_64_four_constraints"] = lambda steps: W.four_quadrant(64, steps)
CONSTRAINTS = {"four_quadrant_64_four_constraints": 4}
# the static lattice map of the paper's static Sod (Sec. IV.C.1, Fig. 7) and
# the neighbourhood choice (next item f4) on the quadrant draw at half-width 0.9
ADAPTIVE_CASES["sod_static_shift"] = lambda steps: W.sod_static_shift(256, 1, steps)
# (its 32 steps: at step 38 a rebuilt link at u' = -1.77, T = 1.24 has no
# 8-moment equilibrium, the dual being unbounded, in both implementations)
ADAPTIVE_STEPS["sod_static_shift"] = 32
ADAPTIVE_CASES["four_quadrant_64_neighbourhood"] = lambda steps: W.four_quadrant(64, steps)
ADAPTIVE_STEPS["four_quadrant_64_neighbourhood"] = 20
OPTIONS = {"four_quadrant_64_neighbourhood": dict(shift_mode=3, halfwidth=0.9)}
# the flexible-Prandtl collision (next item f4, reading D-Pr) at Pr = 0.71 on the
# quadrant draw and on the advected Sod line
ADAPTIVE_CASES["four_quadrant_64_prandtl"] = lambda steps: W.four_quadrant(64, steps)
ADAPTIVE_STEPS["four_quadrant_64_prandtl"] = 20
OPTIONS["four_quadrant_64_prandtl"] = dict(prandtl=0.71)
ADAPTIVE_CASES["advected_sod_prandtl"] = ADAPTIVE_CASES["advected_sod_sensor"]
OPTIONS["advected_sod_prandtl"] = dict(prandtl=0.71)
# the reference model (next item f3): D2Q49 with 13 constraints on the
# quadrant draw at 32^2
ADAPTIVE_CASES["four_quadrant_32_reference_model"] = lambda steps: W.four_quadrant(32, steps)
ADAPTIVE_STEPS["four_quadrant_32_reference_model"] = 10
CONSTRAINTS["four_quadrant_32_reference_model"] = 13


@pytest.mark.parametrize("case", list(ADAPTIVE_CASES))
def test_independent_adaptive_line_matches_the_oracle(case):
    """After 40 steps (20 on the 2D grids) the two agree to 1e-10 on every
    node, select the same lattices and rebuild the same number of links."""
    steps = ADAPTIVE_STEPS.get(case, 40)
    wl = ADAPTIVE_CASES[case](steps)
    M = CONSTRAINTS.get(case, 8)
    opts = OPTIONS.get(case, {})
    line = AdaptiveGrid(wl, M, **opts)
    rebuilt = 0
    for _ in range(steps):
        line.step()
        rebuilt += line.rebuilt
    s = oracle.Sim.from_workload(wl, constraints=M, **opts)
    s.step(steps)
    m = {k: v.ravel() for k, v in s.macros().items()}
    rho, ux, uy, T = line.mac
    uscale = np.hypot(m["ux"], m["uy"]).max()
    err = dict(rho=(np.abs(rho - m["rho"]) / m["rho"]).max(),
               T=(np.abs(T - m["T"]) / m["T"]).max(),
               u=(np.hypot(ux - m["ux"], uy - m["uy"]) / uscale).max())
    print(f"{case}: rebuilt links {rebuilt} (oracle {s.stats()['mismatched_links']}), "
          + ", ".join(f"{k} {v:.1e}" for k, v in err.items()))
    assert rebuilt == s.stats()["mismatched_links"] > 20 * steps
    assert np.array_equal(line.Uc[0], m["Ucx"]) and np.array_equal(line.Uc[1], m["Ucy"])
    assert max(err.values()) <= 1e-10, err
    if "prandtl" in opts:   # the term moves these fields well beyond the agreement
        b = oracle.Sim.from_workload(wl, constraints=M)
        b.step(steps)
        assert np.abs(b.macros()["T"].ravel() - m["T"]).max() > 1e-6
