/*
 * Plain FP64 CPU oracle for the interpolation-free, state-adaptive
 * compressible lattice Boltzmann method of Coreixas & Latt (arXiv 2009.13426):
 * D2Q21 lattice, 8-constraint numerical (maximum-entropy) equilibrium,
 * double-distribution BGK collision, on-grid pull streaming with Grad
 * reconstruction where neighbouring lattice shifts differ; and the paper's
 * reference model on the same framework, D2Q49 with 13 constraints (App. C).
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the slow, obviously-correct
 * reference the GPU implementation is checked against.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark may load it.  It
 * shares no code with the GPU path and must never be used as a fallback for it.
 *
 * Parity unpinned (the paper does not fix them, so the tests pin only their
 * stated properties): the D2Q21 velocity table (orc_velocities), the printed
 * coefficient of the Grad g-deviation, and the values of the sensor's
 * relaxation-time factor (orc_sensor_alpha).
 *
 * Conventions
 *  - Grid nx * ny, periodic in x and y; node n = y * nx + x.
 *  - Populations are stored SoA: h[i * N + n], i in [0, Q), Q = 21 (or 49
 *    for the 13-constraint model).
 *  - Fields passed in or out are float64 arrays of N values, row-major [ny][nx].
 *  - All arithmetic is IEEE double, built with -ffp-contract=off.
 */
#ifndef LBM_ORACLE_H
#define LBM_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_Q 21          /* discrete velocities of D2Q21 */
#define ORC_Q49 49        /* discrete velocities of D2Q49 */
#define ORC_QMAX 49
#define ORC_M 8           /* constraints of the 8-moment equilibrium */
#define ORC_MMAX 13
#define ORC_D 2           /* physical dimensions */
#define ORC_HIST 128      /* Newton-iteration histogram bins */

enum {
  ORC_OK = 0,
  ORC_ERR_ARG = -1,
  ORC_ERR_NEWTON = -5,       /* the equilibrium solve did not converge */
  ORC_ERR_NONPHYSICAL = -6   /* rho <= 0, T <= 0, non-finite, or |U| too large */
};

typedef struct {
  int nx, ny;
  double gamma;          /* heat capacity ratio; Cv = 1/(gamma-1), Cp = gamma Cv */
  double nu;             /* kinematic viscosity; tau = 1/2 + nu / T per node */
  int shift_mode;        /* 0: adaptive criterion; 1: one fixed lattice (fixed_ux, fixed_uy);
                            2: static per-node map set by orc_set_static_shift;
                            3: overlapping ranges of half-width halfwidth (< 1),
                               shift chosen by the four nearest neighbours */
  int fixed_ux, fixed_uy;
  double halfwidth;      /* 0.5 reproduces the criterion exactly; > 0.5 adds hysteresis */
  double newton_tol;     /* max |G_a| per unit density; 1e-12 */
  int newton_max_iter;
  int max_abs_shift;     /* |U_alpha| above this is reported as non-physical */
  int sensor;            /* 1: Knudsen sensor scales tau by alpha(eps_Kn) */
  int constraints;       /* 8 (or 0): eq. (8moments); 4: mass, momentum and energy
                            only, eq. (feqNum_4Mom); 13: eqs. (G0)-(G4yyaa) on the
                            D2Q49 lattice (the paper's reference model) */
  double prandtl;        /* 0 or 1: BGK collision, eq. (coll); otherwise the
                            flexible-Prandtl collision of eq. (Shakhov) with
                            Pr = nu / (thermal diffusivity) */
  int fallback;          /* 0: a state whose 8-moment equilibrium has no solution
                            stops the run (ORC_ERR_NEWTON); 1: that collision or
                            rebuilt link takes the four-constraint equilibrium
                            of the same state instead (a reading: the paper does
                            not treat the case); BGK only; without effect for
                            4 or 13 constraints */
} orc_params;

typedef struct {
  long newton_calls;
  long newton_iters;
  long mismatched_links;
  long hist[ORC_HIST];
  long fail_node;        /* first failing node (lowest index), -1 if none */
  long steps;
  long fallbacks;        /* collisions and rebuilt links that took the four-
                            constraint equilibrium (initial condition included) */
} orc_stats;

typedef struct orc_sim orc_sim;

/* Velocity table: writes 21 integer components each. */
void orc_velocities(int* cx, int* cy);
/* Velocities of lattice Q (21 or 49); orc_lattice_of(M) is the lattice a
 * constraint count is solved on (49 for M = 13, else 21). */
void orc_velocities_q(int Q, int* cx, int* cy);
int orc_lattice_of(int M);

/* Numerical equilibrium per unit density in the frame of the lattice:
 * minimises sum_i w_i ln(w_i) under the 8 moment constraints for peculiar
 * velocity (ux, uy) and temperature T.  lam0 (nullable) is an initial guess
 * for the 8 multipliers.  Outputs w[21], lam[8], Newton iterations used.
 * Returns ORC_OK, ORC_ERR_NEWTON or ORC_ERR_NONPHYSICAL. */
int orc_equilibrium(double ux, double uy, double T, const double* lam0,
                    double tol, int max_iter, double* w, double* lam, int* iters);

/* Exact targets m[8] of the 8 constraints per unit density. */
void orc_targets(double ux, double uy, double T, double* m);

/* As orc_equilibrium / orc_targets for M = 8, 4 or 13 constraints (M = 4:
 * phi = (1, xi_x, xi_y, |xi|^2), targets (1, u_x, u_y, 2E); M = 13: the
 * monomials up to third order and the contracted fourth-order ones on
 * D2Q49, w then holds 49 weights); lam and m hold M values.  ORC_ERR_ARG for
 * another M. */
int orc_equilibrium_m(int M, double ux, double uy, double T, const double* lam0,
                      double tol, int max_iter, double* w, double* lam, int* iters);
void orc_targets_m(int M, double ux, double uy, double T, double* m);

/* Grad populations h = h_eq (1 + phi) for lattice shift (Lx, Ly) at a state
 * with gradients du = (dux/dx, dux/dy, duy/dx, duy/dy), dT = (dT/dx, dT/dy).
 * post != 0 returns post-collision h_eq (1 + (1 - 1/tau) phi) instead.
 * Writes f[Q], g[Q] (Q of the constraint set in p). */
int orc_grad_populations(const orc_params* p, double rho, double ux, double uy,
                         double T, const double* du, const double* dT, int Lx,
                         int Ly, int post, double* f, double* g);

/* Lattice shift along one axis for velocity u, previous shift Uprev and
 * selection half-width (0.5 = eq. criterion without history). */
int orc_select(double u, int Uprev, double halfwidth);

/* Relaxation-time factor alpha(eps) of the kinetic sensor, eq. (DeltaAvg)
 * (a reading: the paper does not print alpha; see lbm_oracle.c). */
double orc_sensor_alpha(double eps);

orc_sim* orc_create(const orc_params* p);
void orc_destroy(orc_sim* s);
int orc_init(orc_sim* s, const double* rho, const double* ux, const double* uy,
             const double* T);
/* Per-node lattice shifts for shift_mode 2 (the paper's 'static' Sod
 * configuration, Sec. IV.C.1); call before orc_init. */
int orc_set_static_shift(orc_sim* s, const int* Ux, const int* Uy);
int orc_step(orc_sim* s, int nsteps);
/* Macros at the current time: rho, absolute u, T; lattice tags of the stored
 * populations (Uc) and of the next pull (Un); any pointer may be NULL. */
void orc_macros(const orc_sim* s, double* rho, double* ux, double* uy, double* T,
                int* Ucx, int* Ucy, int* Unx, int* Uny);
/* Post-collision populations, [i * N + n]. */
void orc_populations(const orc_sim* s, double* f, double* g);
/* Sums over the grid of mass, x/y momentum and total energy
 * (1/2) sum_i (|c_i|^2 f_i + g_i) of the stored populations. */
void orc_conserved(const orc_sim* s, double* out4);
void orc_get_stats(const orc_sim* s, orc_stats* out);

#ifdef __cplusplus
}
#endif
#endif
