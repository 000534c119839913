/*
 * Plain FP64 CPU oracle of the adaptive D2Q21 compressible LBM (and of the
 * paper's reference model, D2Q49 with 13 constraints)
 * (Coreixas & Latt, arXiv 2009.13426).  TEST INFRASTRUCTURE ONLY: see
 * lbm_oracle.h.  Each function follows the passage of the paper cited above
 * it; readings of passages the paper leaves open are marked "Reading".
 *
 * No blocking, fusion or reordering beyond what the paper's algorithm states:
 * one time iteration is, in order (Sec. IV.A.4, "Algorithm overview"),
 *   streaming in pull form with Grad reconstruction of populations whose
 *   source node lives in another lattice (eqs. stream, GradGeneral),
 *   macroscopic moments (eq. polyTemp),
 *   lattice selection from the local velocity (eq. criterion),
 *   numerical equilibrium f_eq (eq. feqNum_8Mom), g_eq (eq. gEq),
 *   BGK collision (eq. coll).
 * Storing post-collision populations makes "streaming" the first pass of each
 * call; the cycle is the paper's.
 */
#include "lbm_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ---------------------------------------------------------------- lattice
 * D2Q21 (Sec. I, Fig. 1; lattice of Zhang et al.).  The velocity table is not
 * printed in the paper.  Reading: the rest velocity, (+-1,0) and (0,+-1),
 * (+-1,+-1), (+-2,0) and (0,+-2), (+-2,+-2), (+-3,0) and (0,+-3).  This set
 * is symmetric under the square's symmetry group and contains the reference
 * populations (0,0), (-1,0), (1,1) named in the caption of Fig. 1. */
static const int XI[ORC_Q][2] = {
    {0, 0},
    {1, 0},  {-1, 0},  {0, 1},  {0, -1},
    {1, 1},  {-1, 1},  {-1, -1}, {1, -1},
    {2, 0},  {-2, 0},  {0, 2},  {0, -2},
    {2, 2},  {-2, 2},  {-2, -2}, {2, -2},
    {3, 0},  {-3, 0},  {0, 3},  {0, -3}};

/* D2Q49 (Sec. I and App. C, the paper's reference lattice): the tensor
 * product {-3, ..., 3}^2, velocity i = (i mod 7 - 3, i div 7 - 3). */
static int cx_of(int Q, int i) { return Q == ORC_Q49 ? i % 7 - 3 : XI[i][0]; }
static int cy_of(int Q, int i) { return Q == ORC_Q49 ? i / 7 - 3 : XI[i][1]; }

/* Lattice of a constraint count: the 13-constraint set is solved on D2Q49,
 * the 8- and 4-constraint sets on D2Q21. */
int orc_lattice_of(int M) { return M == 13 ? ORC_Q49 : ORC_Q; }

void orc_velocities_q(int Q, int* cx, int* cy) {
  for (int i = 0; i < Q; ++i) {
    cx[i] = cx_of(Q, i);
    cy[i] = cy_of(Q, i);
  }
}

void orc_velocities(int* cx, int* cy) { orc_velocities_q(ORC_Q, cx, cy); }

/* ------------------------------------------------ numerical equilibrium
 * Eq. (feqNum_8Mom): f_i^eq = rho exp[-(1 + lambda . phi(xi_i))] with the
 * monomials of the 8-moment set, eq. (8moments):
 *   phi = (1, xi_x, xi_y, xi_x^2, xi_x xi_y, xi_y^2, xi_x |xi|^2, xi_y |xi|^2).
 * Reading: the constraints are written in the frame of the lattice, i.e.
 * with the integer-valued xi_i and the peculiar velocity u - U; the span of
 * phi is invariant under integer translations, so this is the same
 * equilibrium as the one written with c_i = xi_i + U and u. */
static void basis8(double x, double y, double phi[ORC_MMAX]) {
  double s = x * x + y * y;
  phi[0] = 1.0;
  phi[1] = x;
  phi[2] = y;
  phi[3] = x * x;
  phi[4] = x * y;
  phi[5] = y * y;
  phi[6] = x * s;
  phi[7] = y * s;
}

/* Sec. "Reduced models", eq. (feqNum_4Mom): the four constraints of mass,
 * momentum and total energy, phi = (1, xi_x, xi_y, |xi|^2). */
static void basis4(double x, double y, double phi[ORC_MMAX]) {
  phi[0] = 1.0;
  phi[1] = x;
  phi[2] = y;
  phi[3] = x * x + y * y;
}

/* App. C, eqs. (G0)-(G4yyaa) and (feqNum_13Mom): the 13 constraints of the
 * reference model, up to the third-order moments and the contracted
 * fourth-order ones, phi = (1, xi_x, xi_y, xi_x^2, xi_x xi_y, xi_y^2,
 * xi_x^3, xi_x^2 xi_y, xi_x xi_y^2, xi_y^3, xi_x^2 |xi|^2, xi_x xi_y |xi|^2,
 * xi_y^2 |xi|^2).  Reading: the printed exponent of eq. (feqNum_13Mom) lists
 * twelve multipliers and leaves out the one of xi_x^3, although G_3,xxx is
 * among the constraints; it is taken as a dropped term (13 constraints, 13
 * multipliers). */
static void basis13(double x, double y, double phi[ORC_MMAX]) {
  double s = x * x + y * y;
  phi[0] = 1.0;
  phi[1] = x;
  phi[2] = y;
  phi[3] = x * x;
  phi[4] = x * y;
  phi[5] = y * y;
  phi[6] = x * x * x;
  phi[7] = x * x * y;
  phi[8] = x * y * y;
  phi[9] = y * y * y;
  phi[10] = x * x * s;
  phi[11] = x * y * s;
  phi[12] = y * y * s;
}

/* Monomials of velocity i of the lattice of constraint set M. */
static void basis(int M, int i, double phi[ORC_MMAX]) {
  int Q = orc_lattice_of(M);
  double x = cx_of(Q, i), y = cy_of(Q, i);
  if (M == 4)
    basis4(x, y, phi);
  else if (M == 13)
    basis13(x, y, phi);
  else
    basis8(x, y, phi);
}

/* Constraint targets per unit density, eqs. (G0_8mom)-(G3yaa_8mom), with the
 * energy 2E = u_x^2 + u_y^2 + D T (App. C, D = 2). */
void orc_targets_m(int M, double ux, double uy, double T, double* m) {
  double E = 0.5 * (ux * ux + uy * uy + ORC_D * T);
  if (M == 4) { /* G_0, G_1x, G_1y, G_2aa of the four-constraint set */
    m[0] = 1.0;
    m[1] = ux;
    m[2] = uy;
    m[3] = 2.0 * E;
    return;
  }
  if (M == 13) { /* eqs. (G0)-(G4yyaa) */
    m[0] = 1.0;
    m[1] = ux;
    m[2] = uy;
    m[3] = ux * ux + T;
    m[4] = ux * uy;
    m[5] = uy * uy + T;
    m[6] = ux * (ux * ux + 3.0 * T);
    m[7] = (ux * ux + T) * uy;
    m[8] = ux * (uy * uy + T);
    m[9] = uy * (uy * uy + 3.0 * T);
    m[10] = 2.0 * ((E + 2.0 * T) * ux * ux + (E + T) * T);
    m[11] = 2.0 * (E + 2.0 * T) * ux * uy;
    m[12] = 2.0 * ((E + 2.0 * T) * uy * uy + (E + T) * T);
    return;
  }
  m[0] = 1.0;
  m[1] = ux;
  m[2] = uy;
  m[3] = ux * ux + T;
  m[4] = ux * uy;
  m[5] = uy * uy + T;
  m[6] = 2.0 * ux * (E + T);
  m[7] = 2.0 * uy * (E + T);
}

void orc_targets(double ux, double uy, double T, double* m) { orc_targets_m(8, ux, uy, T, m); }

/* Weights w_i = exp(-(1 + lambda.phi_i)), constraint residuals
 * G_a = sum_i w_i phi_a(xi_i) - m_a (eq. constraints) and the value of the
 * convex dual Psi(lambda) = sum_i w_i + lambda.m, whose gradient is -G and
 * whose Hessian is H = sum_i w_i phi phi^T (positive definite since phi has
 * rank 8 on the lattice).  Minimising Psi is the entropy problem of
 * eqs. (Hfunction)-(exponential) with prefactor a = rho. */
static double evaluate(int M, const double lam[ORC_MMAX], const double m[ORC_MMAX],
                       double w[ORC_QMAX], double G[ORC_MMAX]) {
  double phi[ORC_MMAX];
  double psi = 0.0;
  const int Q = orc_lattice_of(M);
  for (int a = 0; a < M; ++a) G[a] = -m[a];
  for (int i = 0; i < Q; ++i) {
    basis(M, i, phi);
    double e = 1.0;
    for (int a = 0; a < M; ++a) e += lam[a] * phi[a];
    w[i] = exp(-e);
    for (int a = 0; a < M; ++a) G[a] += w[i] * phi[a];
    psi += w[i];
  }
  for (int a = 0; a < M; ++a) psi += lam[a] * m[a];
  return psi;
}

static void hessian(int M, const double w[ORC_QMAX], double H[ORC_MMAX][ORC_MMAX]) {
  double phi[ORC_MMAX];
  const int Q = orc_lattice_of(M);
  memset(H, 0, sizeof(double) * ORC_MMAX * ORC_MMAX);
  for (int i = 0; i < Q; ++i) {
    basis(M, i, phi);
    for (int a = 0; a < M; ++a)
      for (int b = 0; b < M; ++b) H[a][b] += w[i] * phi[a] * phi[b];
  }
}

/* Gaussian elimination with partial pivoting for H d = G (leading M x M). */
static int solve(int M, double Hin[ORC_MMAX][ORC_MMAX], const double G[ORC_MMAX],
                 double d[ORC_MMAX]) {
  double A[ORC_MMAX][ORC_MMAX + 1];
  for (int r = 0; r < M; ++r) {
    for (int c = 0; c < M; ++c) A[r][c] = Hin[r][c];
    A[r][M] = G[r];
  }
  for (int c = 0; c < M; ++c) {
    int p = c;
    for (int r = c + 1; r < M; ++r)
      if (fabs(A[r][c]) > fabs(A[p][c])) p = r;
    if (!(fabs(A[p][c]) > 0.0)) return -1;
    if (p != c)
      for (int k = 0; k <= M; ++k) {
        double t = A[c][k];
        A[c][k] = A[p][k];
        A[p][k] = t;
      }
    for (int r = c + 1; r < M; ++r) {
      double f = A[r][c] / A[c][c];
      for (int k = c; k <= M; ++k) A[r][k] -= f * A[c][k];
    }
  }
  for (int r = M - 1; r >= 0; --r) {
    double acc = A[r][M];
    for (int k = r + 1; k < M; ++k) acc -= A[r][k] * d[k];
    d[r] = acc / A[r][r];
  }
  return 0;
}

static double maxabs(const double* v, int n) {
  double r = 0.0;
  for (int k = 0; k < n; ++k) {
    double a = fabs(v[k]);
    if (!(a <= r)) r = a; /* propagates NaN */
  }
  return r;
}

/* Initial guess: the lattice-normalised Maxwellian, lambda_1 = -u/T,
 * lambda_2 = I / (2T) (for M = 4 the |xi|^2 multiplier 1/(2T)), cross and
 * third-order multipliers zero, lambda_0 such that sum_i w_i = 1. */
static void maxwellian_guess(int M, double ux, double uy, double T, double lam[ORC_MMAX]) {
  double phi[ORC_MMAX];
  const int Q = orc_lattice_of(M);
  for (int a = 0; a < ORC_MMAX; ++a) lam[a] = 0.0;
  lam[1] = -ux / T;
  lam[2] = -uy / T;
  lam[3] = 0.5 / T;
  if (M != 4) lam[5] = 0.5 / T;
  double z = 0.0;
  for (int i = 0; i < Q; ++i) {
    basis(M, i, phi);
    double e = 0.0;
    for (int a = 1; a < M; ++a) e += lam[a] * phi[a];
    z += exp(-e);
  }
  lam[0] = log(z) - 1.0;
}

/* Root finding for the multipliers (App. C; the paper uses a globalised
 * Newton method with a 1e-12 criterion).  Newton steps d = H^{-1} G on the
 * convex dual, globalised by backtracking on Psi (a full step is also
 * accepted when it halves the residual, since near the root the change of Psi
 * falls below its rounding).  Stop when max_a |G_a| <= tol, then apply one
 * more plain Newton step so that the constraints hold to rounding.
 * Reading: the polishing step. */
int orc_equilibrium_m(int M, double ux, double uy, double T, const double* lam0,
                      double tol, int max_iter, double* w, double* lam, int* iters) {
  double m[ORC_MMAX], l[ORC_MMAX], G[ORC_MMAX], d[ORC_MMAX], H[ORC_MMAX][ORC_MMAX];
  double wt[ORC_QMAX], lt[ORC_MMAX], Gt[ORC_MMAX];
  if (iters) *iters = 0;
  if (M != 4 && M != 8 && M != 13) return ORC_ERR_ARG;
  if (!(T > 0.0) || !isfinite(T) || !isfinite(ux) || !isfinite(uy))
    return ORC_ERR_NONPHYSICAL;
  orc_targets_m(M, ux, uy, T, m);
  for (int a = 0; a < ORC_MMAX; ++a) l[a] = 0.0;
  if (lam0)
    memcpy(l, lam0, sizeof(double) * M);
  else
    maxwellian_guess(M, ux, uy, T, l);
  double psi = evaluate(M, l, m, w, G);
  for (int it = 0; it < max_iter; ++it) {
    double r = maxabs(G, M);
    if (!isfinite(r) || !isfinite(psi)) return ORC_ERR_NEWTON;
    hessian(M, w, H);
    if (solve(M, H, G, d)) return ORC_ERR_NEWTON;
    if (r <= tol) { /* converged: one polishing Newton step */
      for (int a = 0; a < M; ++a) l[a] += d[a];
      evaluate(M, l, m, w, G);
      if (!isfinite(maxabs(G, M))) return ORC_ERR_NEWTON;
      memcpy(lam, l, sizeof(double) * M);
      if (iters) *iters = it + 1;
      return ORC_OK;
    }
    double slope = 0.0; /* directional derivative of Psi along d: -G.d < 0 */
    for (int a = 0; a < M; ++a) slope -= G[a] * d[a];
    double t = 1.0, psit;
    for (;;) {
      for (int a = 0; a < M; ++a) lt[a] = l[a] + t * d[a];
      psit = evaluate(M, lt, m, wt, Gt);
      if (isfinite(psit)) {
        if (psit <= psi + 1e-4 * t * slope) break;
        if (t == 1.0 && maxabs(Gt, M) < 0.5 * r) break;
      }
      t *= 0.5;
      if (t < 1e-12) return ORC_ERR_NEWTON;
    }
    memcpy(l, lt, sizeof l);
    memcpy(w, wt, sizeof(double) * orc_lattice_of(M));
    memcpy(G, Gt, sizeof Gt);
    psi = psit;
  }
  return ORC_ERR_NEWTON;
}

int orc_equilibrium(double ux, double uy, double T, const double* lam0,
                    double tol, int max_iter, double* w, double* lam, int* iters) {
  return orc_equilibrium_m(8, ux, uy, T, lam0, tol, max_iter, w, lam, iters);
}

/* Constraint count of a simulation: 8 (eq. 8moments) unless set to 4 or 13;
 * its lattice follows (D2Q49 for 13, else D2Q21). */
static int constraints_of(const orc_params* p) {
  return p->constraints == 4 || p->constraints == 13 ? p->constraints : 8;
}
static int lattice_of(const orc_params* p) { return orc_lattice_of(constraints_of(p)); }

/* ------------------------------------------------------ Grad populations
 * Eqs. (GradGeneral), (GradGeneral_f), (GradGeneral_g):
 *   h ~ h_eq (1 + phi_h),
 *   phi_f = sigma:cbar cbar / (2 rho T^2)
 *           + q.cbar / (rho Cp T^2) (|cbar|^2 / (2T) - Cp),
 *   phi_g = 2 q.cbar / (rho Cp)            (Reading: as printed),
 *   -sigma = mu [grad u + grad u^T - (2/D) div u I],  mu = rho nu,
 *   q = -kappa grad T,  cbar = c_i - u,  c_i = xi_i + U.
 * Reading: kappa = rho Cp nu (unit Prandtl number of BGK, Sec. IV.A.1),
 * Cp = gamma / (gamma - 1).  Post-collision populations follow from
 * h* = h_eq + (1 - 1/tau) h_neq with h_neq = h_eq phi_h (Sec. III.B.2),
 * tau = 1/2 + nu / T (App. E). */
#define ORC_GRAD_G_COEFF 2.0

/* Prandtl number of a simulation: 1 (BGK) unless set. */
static double prandtl_of(const orc_params* p) { return p->prandtl > 0.0 ? p->prandtl : 1.0; }

/* Heat flux of populations f, g of lattice Q in the frame moving with the
 * fluid: q_a = (1/2) sum_i cbar_ia (|cbar_i|^2 f_i + g_i), cbar_i = xi_i - u'
 * (lattice frame, u' the peculiar velocity). */
static void heat_flux(int Q, const double* f, const double* g, double upx, double upy,
                      double q[2]) {
  q[0] = 0.0;
  q[1] = 0.0;
  for (int i = 0; i < Q; ++i) {
    double cx = cx_of(Q, i) - upx, cy = cy_of(Q, i) - upy;
    double h = (cx * cx + cy * cy) * f[i] + g[i];
    q[0] += 0.5 * cx * h;
    q[1] += 0.5 * cy * h;
  }
}

/* Flexible-Prandtl collision, eq. (Shakhov) (App. E, Rykov's model with
 * elastic collisions): BGK plus (1/tau - 1/tau_Pr) h_eq phi_S, with q the
 * heat flux of the populations being collided.  Reading: the printed term
 * shapes are the monatomic ones with Cp put in place of the translational
 * (D + 2)/2 and an extra factor 2 T^2 in the g term; as printed the f term
 * carries momentum (2 - Cp)/(Cp T) q and the pair carries a fraction of q.
 * Here
 *   phi_S,f = q.cbar / (rho Cp T^2) (|cbar|^2 / (2T) - (D + 2)/2),
 *   phi_S,g = q.cbar / (rho Cp T^2),
 * which, with the Maxwellian's moments (up to sixth order), carry no mass,
 * momentum or energy and together the heat flux q (the f term 2/Cp of it,
 * the g term (Cv - 1)/Cp), so that the heat flux relaxes with tau_Pr; they
 * equal the printed ones for a monatomic gas (Cp = 2, g_eq = 0).  On a
 * lattice whose equilibrium moments differ from the Maxwellian's beyond the
 * enforced ones, f_eq phi_S,f is made free of mass, momentum and energy by
 * subtracting its projection on 1, cbar_x, cbar_y, |cbar|^2 in the inner
 * product weighted by f_eq (D2Q21 with 8 constraints fixes moments up to
 * the third order; D2Q49 with 13 up to the contracted fourth, so there
 * only the energy part, a fifth-order moment, is left); the g term needs none
 * (g carries no momentum, and its mass and energy vanish with the first
 * moment of f_eq).  tau_Pr = 1/2 + (tau - 1/2)/Pr, i.e. 1/2 + nu/(Pr T)
 * without the sensor. */
static void shakhov_terms(const orc_params* p, int Q, const double* w, double upx, double upy,
                          double rho, double T, const double q[2], double* sf, double* sg) {
  double Cp = p->gamma / (p->gamma - 1.0);
  double G[ORC_MMAX][ORC_MMAX], r[ORC_MMAX], beta[ORC_MMAX];
  memset(G, 0, sizeof G);
  memset(r, 0, sizeof r);
  for (int i = 0; i < Q; ++i) {
    double cx = cx_of(Q, i) - upx, cy = cy_of(Q, i) - upy, c2 = cx * cx + cy * cy;
    double a = (q[0] * cx + q[1] * cy) / (rho * Cp * T * T);
    double e[4] = {1.0, cx, cy, c2};
    sf[i] = a * (c2 / (2.0 * T) - 0.5 * (ORC_D + 2));
    sg[i] = a;
    double feq = rho * w[i];
    for (int j = 0; j < 4; ++j) {
      r[j] += feq * sf[i] * e[j];
      for (int k = 0; k < 4; ++k) G[j][k] += feq * e[j] * e[k];
    }
  }
  if (solve(4, G, r, beta)) return; /* singular only for a degenerate f_eq */
  for (int i = 0; i < Q; ++i) {
    double cx = cx_of(Q, i) - upx, cy = cy_of(Q, i) - upy;
    sf[i] -= beta[0] + beta[1] * cx + beta[2] * cy + beta[3] * (cx * cx + cy * cy);
  }
}

static void grad_phi(const orc_params* p, int i, double rho, double ux, double uy,
                     double T, const double* du, const double* dT, int Lx, int Ly,
                     double* phif, double* phig) {
  double Cv = 1.0 / (p->gamma - 1.0), Cp = p->gamma * Cv;
  const int Q = lattice_of(p);
  double cbx = (double)(cx_of(Q, i) + Lx) - ux;
  double cby = (double)(cy_of(Q, i) + Ly) - uy;
  double mu = rho * p->nu;
  double div = du[0] + du[3];
  double sxx = -mu * (2.0 * du[0] - (2.0 / ORC_D) * div);
  double syy = -mu * (2.0 * du[3] - (2.0 / ORC_D) * div);
  double sxy = -mu * (du[1] + du[2]);
  double kappa = rho * Cp * p->nu / prandtl_of(p);
  double qx = -kappa * dT[0], qy = -kappa * dT[1];
  double qc = qx * cbx + qy * cby;
  double c2 = cbx * cbx + cby * cby;
  *phif = (sxx * cbx * cbx + 2.0 * sxy * cbx * cby + syy * cby * cby) / (2.0 * rho * T * T) +
          qc / (rho * Cp * T * T) * (c2 / (2.0 * T) - Cp);
  *phig = ORC_GRAD_G_COEFF * qc / (rho * Cp);
}

/* The equilibrium of the constraint set of p at (ux, uy, T) in the lattice's
 * frame.  Reading (the paper leaves the case open): with p->fallback set,
 * where the 8-moment problem has no solution (the Newton solve fails, e.g.
 * a rebuilt link whose source moves at |u'| ~ 1.6 in the receiver's
 * lattice), the four-constraint equilibrium of the same state stands in,
 * eq. (feqNum_4Mom): it conserves mass, momentum and energy and exists for
 * every velocity inside the lattice.  *fell_back (nullable) is set to 1
 * when it was taken. */
static int equilibrium_of(const orc_params* p, double ux, double uy, double T, double* w,
                          double* lam, int* iters, int* fell_back) {
  int it = 0;
  int rc = orc_equilibrium_m(constraints_of(p), ux, uy, T, NULL, p->newton_tol,
                             p->newton_max_iter, w, lam, &it);
  if (fell_back) *fell_back = 0;
  if (rc == ORC_ERR_NEWTON && p->fallback && constraints_of(p) == 8) {
    int it4 = 0;
    rc = orc_equilibrium_m(4, ux, uy, T, NULL, p->newton_tol, p->newton_max_iter, w, lam,
                           &it4);
    it += it4;
    if (rc == ORC_OK && fell_back) *fell_back = 1;
  }
  if (iters) *iters = it;
  return rc;
}

static int grad_populations(const orc_params* p, double rho, double ux, double uy,
                            double T, const double* du, const double* dT, int Lx,
                            int Ly, int post, double* f, double* g, int* fell_back) {
  double w[ORC_QMAX], lam[ORC_MMAX];
  double Cv = 1.0 / (p->gamma - 1.0);
  const int Q = lattice_of(p);
  if (fell_back) *fell_back = 0;
  if (!(rho > 0.0) || !isfinite(rho)) return ORC_ERR_NONPHYSICAL;
  int rc = equilibrium_of(p, ux - Lx, uy - Ly, T, w, lam, NULL, fell_back);
  if (rc) return rc;
  double tau = 0.5 + p->nu / T;
  double k = post ? (1.0 - 1.0 / tau) : 1.0;
  double Pr = prandtl_of(p);
  if (post && Pr != 1.0) {
    /* eq. (Shakhov) applied to the Grad populations (App. E) */
    double fg[ORC_QMAX] = {0}, gg[ORC_QMAX] = {0}, q[2];
    double upx = ux - Lx, upy = uy - Ly;
    for (int i = 0; i < Q; ++i) {
      double phif, phig;
      grad_phi(p, i, rho, ux, uy, T, du, dT, Lx, Ly, &phif, &phig);
      double feq = rho * w[i];
      double geq = (2.0 * Cv - ORC_D) * T * feq;
      fg[i] = feq * (1.0 + phif);
      gg[i] = geq * (1.0 + phig);
    }
    heat_flux(Q, fg, gg, upx, upy, q);
    double tpr = 0.5 + (tau - 0.5) / Pr;
    double ks = 1.0 / tau - 1.0 / tpr;
    double sf[ORC_QMAX], sg[ORC_QMAX];
    shakhov_terms(p, Q, w, upx, upy, rho, T, q, sf, sg);
    for (int i = 0; i < Q; ++i) {
      double feq = rho * w[i];
      double geq = (2.0 * Cv - ORC_D) * T * feq;
      f[i] = feq + k * (fg[i] - feq) + ks * feq * sf[i];
      g[i] = geq + k * (gg[i] - geq) + ks * geq * sg[i];
    }
    return ORC_OK;
  }
  for (int i = 0; i < Q; ++i) {
    double phif, phig;
    grad_phi(p, i, rho, ux, uy, T, du, dT, Lx, Ly, &phif, &phig);
    double feq = rho * w[i];
    double geq = (2.0 * Cv - ORC_D) * T * feq; /* eq. (gEq) */
    f[i] = feq * (1.0 + k * phif);
    g[i] = geq * (1.0 + k * phig);
  }
  return ORC_OK;
}

int orc_grad_populations(const orc_params* p, double rho, double ux, double uy,
                         double T, const double* du, const double* dT, int Lx,
                         int Ly, int post, double* f, double* g) {
  return grad_populations(p, rho, ux, uy, T, du, dT, Lx, Ly, post, f, g, NULL);
}

/* ------------------------------------------------------------ simulation */
struct orc_sim {
  orc_params p;
  long N;
  int Q;                 /* velocities of the lattice */
  double *f, *g;         /* post-collision populations at time t */
  double *fp, *gp;       /* streamed (pre-collision) populations at t+1 */
  double *mac, *mac1;    /* rho, ux, uy, T per node */
  int *Uc, *Un, *Uc1, *Un1;
  int* Us;               /* static per-node shifts (shift_mode 2) */
  orc_stats st;
};

static long wrap(long v, long n) {
  v %= n;
  return v < 0 ? v + n : v;
}

/* Eq. (criterion): n - 1/2 < u <= n + 1/2  <=>  U = n, i.e. U = ceil(u - 1/2).
 * Reading of the overlapping-range remark (Sec. III.A.2): with a half-width
 * w > 1/2 the previous shift is kept while U_prev - w < u <= U_prev + w. */
static int select_axis(double u, int Uprev, double w) {
  if (u > Uprev - w && u <= Uprev + w) return Uprev;
  return (int)ceil(u - 0.5);
}

int orc_select(double u, int Uprev, double halfwidth) {
  return select_axis(u, Uprev, halfwidth);
}

/* Reading of the neighbourhood choice among overlapping ranges (Sec.
 * III.A.2: where the ranges of half-width w > 1/2 overlap, the shift can be
 * chosen by the cell's neighbourhood to reduce the number of interface
 * cells).  Per axis the admissible shifts are the n with n - w < u <= n + w
 * (one or two of them for w < 1); among the admissible pairs the node takes
 * the one that the most of its four nearest neighbours are colliding in at
 * this step; ties go to its own current lattice, then to the plain
 * criterion ceil(u - 1/2), then to the first pair in the order of
 * increasing x and then y shift. */
static void select_neighbourhood(const orc_sim* s, long n, double ux, double uy, int* nUx,
                                 int* nUy) {
  const orc_params* p = &s->p;
  const double w = p->halfwidth;
  long nx = p->nx, ny = p->ny;
  long x = n % nx, y = n / nx;
  long nb[4] = {y * nx + wrap(x + 1, nx), y * nx + wrap(x - 1, nx),
                wrap(y + 1, ny) * nx + x, wrap(y - 1, ny) * nx + x};
  int cand[2][2], nc[2];
  double u[2] = {ux, uy};
  for (int a = 0; a < 2; ++a) {
    int c = (int)ceil(u[a] - 0.5);
    nc[a] = 0;
    for (int d = -1; d <= 1; ++d) {
      int m = c + d;
      if (u[a] > m - w && u[a] <= m + w) cand[a][nc[a]++] = m;
    }
  }
  int Ux = s->Un[2 * n], Uy = s->Un[2 * n + 1];
  int cx0 = (int)ceil(ux - 0.5), cy0 = (int)ceil(uy - 0.5);
  int best = -1, bx = 0, by = 0;
  for (int i = 0; i < nc[0]; ++i)
    for (int j = 0; j < nc[1]; ++j) {
      int cx = cand[0][i], cy = cand[1][j];
      int score = 0;
      for (int k = 0; k < 4; ++k)
        score += (s->Un[2 * nb[k]] == cx && s->Un[2 * nb[k] + 1] == cy);
      /* rank: neighbours first, then history, then the plain criterion */
      int rank = 4 * score + 2 * (cx == Ux && cy == Uy) + (cx == cx0 && cy == cy0);
      if (rank > best) {
        best = rank;
        bx = cx;
        by = cy;
      }
    }
  *nUx = bx;
  *nUy = by;
}

orc_sim* orc_create(const orc_params* p) {
  if (!p || p->nx < 1 || p->ny < 1 || !(p->gamma > 1.0) || !(p->nu >= 0.0) ||
      p->newton_max_iter < 1 || !(p->halfwidth >= 0.5) ||
      (p->constraints != 0 && p->constraints != 4 && p->constraints != 8 &&
       p->constraints != 13) ||
      p->shift_mode < 0 || p->shift_mode > 3 ||
      (p->shift_mode == 3 && !(p->halfwidth < 1.0)) || !(p->prandtl >= 0.0) ||
      !(p->prandtl < 1e3) || (p->fallback != 0 && p->fallback != 1) ||
      (p->fallback && prandtl_of(p) != 1.0))
    return NULL;
  orc_sim* s = (orc_sim*)calloc(1, sizeof(orc_sim));
  if (!s) return NULL;
  s->p = *p;
  s->N = (long)p->nx * p->ny;
  s->Q = lattice_of(p);
  long N = s->N;
  size_t QN = (size_t)s->Q * N;
  s->f = (double*)calloc(QN, sizeof(double));
  s->g = (double*)calloc(QN, sizeof(double));
  s->fp = (double*)calloc(QN, sizeof(double));
  s->gp = (double*)calloc(QN, sizeof(double));
  s->mac = (double*)calloc((size_t)4 * N, sizeof(double));
  s->mac1 = (double*)calloc((size_t)4 * N, sizeof(double));
  s->Uc = (int*)calloc((size_t)2 * N, sizeof(int));
  s->Un = (int*)calloc((size_t)2 * N, sizeof(int));
  s->Uc1 = (int*)calloc((size_t)2 * N, sizeof(int));
  s->Un1 = (int*)calloc((size_t)2 * N, sizeof(int));
  s->Us = (int*)calloc((size_t)2 * N, sizeof(int));
  if (!s->f || !s->g || !s->fp || !s->gp || !s->mac || !s->mac1 || !s->Uc || !s->Un ||
      !s->Uc1 || !s->Un1 || !s->Us) {
    orc_destroy(s);
    return NULL;
  }
  s->st.fail_node = -1;
  return s;
}

void orc_destroy(orc_sim* s) {
  if (!s) return;
  free(s->f); free(s->g); free(s->fp); free(s->gp);
  free(s->mac); free(s->mac1);
  free(s->Uc); free(s->Un); free(s->Uc1); free(s->Un1); free(s->Us);
  free(s);
}

/* Keeps the lowest failing node index of a pass and its status code. */
static void record_failure(orc_sim* s, long n, int rc, int* err) {
#pragma omp critical(orc_fail)
  {
    if (*err == 0 || n < s->st.fail_node) {
      *err = rc;
      s->st.fail_node = n;
    }
  }
}

/* Relaxation-time factor alpha(eps) of the kinetic sensor (Sec. IV.A.2).
 * The paper states that dissipation is added above eps = 0.01 but does not
 * print alpha.  Reading: three levels of added dissipation, alpha = 1.05,
 * 1.35 and 2 from eps = 0.01, 0.1 and 1 on, each reached by a linear ramp
 * over the first tenth of its decade (from 1 at eps = 0.01 to 1.05 at
 * 0.011, from 1.05 at 0.1 to 1.35 at 0.11, from 1.35 at 1 to 2 at 1.1), and
 * 1 up to 0.01.  alpha is continuous and non-decreasing, so a rounding-level
 * change of eps changes tau by a rounding-level amount. */
double orc_sensor_alpha(double eps) {
  static const double ke[6] = {0.01, 0.011, 0.1, 0.11, 1.0, 1.1};
  static const double ka[6] = {1.0, 1.05, 1.05, 1.35, 1.35, 2.0};
  if (!(eps > ke[0])) return 1.0;
  for (int j = 1; j < 6; ++j)
    if (eps <= ke[j])
      return ka[j - 1] + (ka[j] - ka[j - 1]) * (eps - ke[j - 1]) / (ke[j] - ke[j - 1]);
  return ka[5];
}

/* Kinetic sensor, eq. (DeltaAvg): eps = (1/V) sum_i |f_i - f_i^eq| / f_i^eq,
 * with tau_f -> tau_f alpha(eps) (Sec. IV.A.2). */
static double sensor_alpha(int Q, const double* f, double rho, const double* w) {
  double eps = 0.0;
  for (int i = 0; i < Q; ++i) {
    double feq = rho * w[i];
    eps += fabs(f[i] - feq) / feq;
  }
  eps /= Q;
  return orc_sensor_alpha(eps);
}

/* Moments, lattice selection, equilibrium and collision for every node.
 * Input: pre-collision populations fp, gp living in lattice Un.
 * Output: post-collision f, g in lattice Un (now Uc), macros, next lattice. */
static int collide_all(orc_sim* s) {
  const orc_params* p = &s->p;
  const long N = s->N;
  const double Cv = 1.0 / (p->gamma - 1.0);
  const int Q = s->Q;
  int err = 0;
  long calls = 0, iters = 0, fallbacks = 0;
  long hist[ORC_HIST];
  memset(hist, 0, sizeof hist);
#pragma omp parallel for schedule(static) reduction(+ : calls, iters, fallbacks)
  for (long n = 0; n < N; ++n) {
    const int Ux = s->Un[2 * n], Uy = s->Un[2 * n + 1];
    double f[ORC_QMAX], g[ORC_QMAX];
    for (int i = 0; i < Q; ++i) {
      f[i] = s->fp[i * N + n];
      g[i] = s->gp[i * N + n];
    }
    /* moments in the frame of the lattice, eq. (polyTemp) */
    double rho = 0.0, jx = 0.0, jy = 0.0, e = 0.0;
    for (int i = 0; i < Q; ++i) {
      const int x = cx_of(Q, i), y = cy_of(Q, i);
      rho += f[i];
      jx += f[i] * x;
      jy += f[i] * y;
      e += (double)(x * x + y * y) * f[i] + g[i];
    }
    double upx = jx / rho, upy = jy / rho;
    double T = (e - rho * (upx * upx + upy * upy)) / (2.0 * rho * Cv);
    if (!(rho > 0.0) || !(T > 0.0) || !isfinite(rho) || !isfinite(T) ||
        !isfinite(upx) || !isfinite(upy)) {
      record_failure(s, n, ORC_ERR_NONPHYSICAL, &err);
      continue;
    }
    double ux = upx + Ux, uy = upy + Uy;
    /* decomposition for the next streaming, eq. (criterion) */
    int nUx, nUy;
    if (p->shift_mode == 1) {
      nUx = p->fixed_ux;
      nUy = p->fixed_uy;
    } else if (p->shift_mode == 2) {
      nUx = s->Us[2 * n];
      nUy = s->Us[2 * n + 1];
    } else if (p->shift_mode == 3) {
      select_neighbourhood(s, n, ux, uy, &nUx, &nUy);
    } else {
      nUx = select_axis(ux, Ux, p->halfwidth);
      nUy = select_axis(uy, Uy, p->halfwidth);
    }
    if (abs(nUx) > p->max_abs_shift || abs(nUy) > p->max_abs_shift) {
      record_failure(s, n, ORC_ERR_NONPHYSICAL, &err);
      continue;
    }
    /* numerical equilibrium in the current lattice, eqs. (feqNum_8Mom), (gEq) */
    double w[ORC_QMAX], lam[ORC_MMAX];
    int it = 0, fb = 0;
    int rc = equilibrium_of(p, upx, upy, T, w, lam, &it, &fb);
    calls += 1;
    iters += it;
    fallbacks += fb;
    if (rc) {
      record_failure(s, n, rc, &err);
      continue;
    }
#pragma omp atomic
    hist[it < ORC_HIST ? it : ORC_HIST - 1] += 1;
    /* BGK collision, eq. (coll), tau = 1/2 + nu / T (App. E) */
    double tau = 0.5 + p->nu / T;
    if (p->sensor) tau *= sensor_alpha(Q, f, rho, w);
    if (prandtl_of(p) != 1.0) {
      /* flexible Prandtl number, eq. (Shakhov) */
      double q[2];
      heat_flux(Q, f, g, upx, upy, q);
      double tpr = 0.5 + (tau - 0.5) / prandtl_of(p);
      double ks = 1.0 / tau - 1.0 / tpr;
      double sf[ORC_QMAX], sg[ORC_QMAX];
      shakhov_terms(p, Q, w, upx, upy, rho, T, q, sf, sg);
      for (int i = 0; i < Q; ++i) {
        double feq = rho * w[i];
        double geq = (2.0 * Cv - ORC_D) * T * feq;
        s->f[i * N + n] = f[i] - (f[i] - feq) / tau + ks * feq * sf[i];
        s->g[i * N + n] = g[i] - (g[i] - geq) / tau + ks * geq * sg[i];
      }
    } else {
      for (int i = 0; i < Q; ++i) {
        double feq = rho * w[i];
        double geq = (2.0 * Cv - ORC_D) * T * feq;
        s->f[i * N + n] = f[i] - (f[i] - feq) / tau;
        s->g[i * N + n] = g[i] - (g[i] - geq) / tau;
      }
    }
    s->mac1[4 * n + 0] = rho;
    s->mac1[4 * n + 1] = ux;
    s->mac1[4 * n + 2] = uy;
    s->mac1[4 * n + 3] = T;
    s->Uc1[2 * n] = Ux;
    s->Uc1[2 * n + 1] = Uy;
    s->Un1[2 * n] = nUx;
    s->Un1[2 * n + 1] = nUy;
  }
  s->st.newton_calls += calls;
  s->st.newton_iters += iters;
  s->st.fallbacks += fallbacks;
  for (int k = 0; k < ORC_HIST; ++k) s->st.hist[k] += hist[k];
  if (err) return err;
  double* t = s->mac; s->mac = s->mac1; s->mac1 = t;
  int* u = s->Uc; s->Uc = s->Uc1; s->Uc1 = u;
  u = s->Un; s->Un = s->Un1; s->Un1 = u;
  return ORC_OK;
}

/* Central differences (Reading: second-order FD of Sec. IV.A.1 are centred,
 * periodic) of absolute velocity and temperature around node n, taken from
 * per-node values v[4 * m + k] with k = 1, 2 (u) and 3 (T). */
static void gradients(const orc_sim* s, const double* v, long n, double du[4],
                      double dT[2]) {
  long nx = s->p.nx, ny = s->p.ny;
  long x = n % nx, y = n / nx;
  long xp = y * nx + wrap(x + 1, nx), xm = y * nx + wrap(x - 1, nx);
  long yp = wrap(y + 1, ny) * nx + x, ym = wrap(y - 1, ny) * nx + x;
  du[0] = 0.5 * (v[4 * xp + 1] - v[4 * xm + 1]);
  du[1] = 0.5 * (v[4 * yp + 1] - v[4 * ym + 1]);
  du[2] = 0.5 * (v[4 * xp + 2] - v[4 * xm + 2]);
  du[3] = 0.5 * (v[4 * yp + 2] - v[4 * ym + 2]);
  dT[0] = 0.5 * (v[4 * xp + 3] - v[4 * xm + 3]);
  dT[1] = 0.5 * (v[4 * yp + 3] - v[4 * ym + 3]);
}

/* Eq. (GradGeneral) applied to a missing post-collision population
 * (Sec. IV.A.4): macros and gradients at the source x - c_i, equilibrium in
 * the lattice of the receiving node. */
static int reconstruct(const orc_sim* s, long src, int Lx, int Ly, int i, double* fi,
                       double* gi, int* fell_back) {
  double du[4], dT[2], f[ORC_QMAX], g[ORC_QMAX];
  const double* m = s->mac + 4 * src;
  gradients(s, s->mac, src, du, dT);
  int rc = grad_populations(&s->p, m[0], m[1], m[2], m[3], du, dT, Lx, Ly, 1, f, g,
                            fell_back);
  *fi = f[i];
  *gi = g[i];
  return rc;
}

int orc_init(orc_sim* s, const double* rho, const double* ux, const double* uy,
             const double* T) {
  const orc_params* p = &s->p;
  const long N = s->N;
  int err = 0;
  /* Grad initial condition (Sec. IV.A.1): h(0) = h_eq (1 + phi_h) in the
   * lattice each node selects, gradients of the input fields by central
   * differences.  Reading: these are pre-collision populations, followed by
   * a collision, so the stored state is h*(0). */
  double* v = (double*)malloc(sizeof(double) * 4 * N);
  if (!v) return ORC_ERR_ARG;
  for (long n = 0; n < N; ++n) {
    v[4 * n] = rho[n];
    v[4 * n + 1] = ux[n];
    v[4 * n + 2] = uy[n];
    v[4 * n + 3] = T[n];
  }
  memset(&s->st, 0, sizeof s->st);
  s->st.fail_node = -1;
  long fallbacks = 0;
#pragma omp parallel for schedule(static) reduction(+ : fallbacks)
  for (long n = 0; n < N; ++n) {
    int Ux, Uy;
    if (p->shift_mode == 1) {
      Ux = p->fixed_ux;
      Uy = p->fixed_uy;
    } else if (p->shift_mode == 2) {
      Ux = s->Us[2 * n];
      Uy = s->Us[2 * n + 1];
    } else {
      Ux = (int)ceil(ux[n] - 0.5);
      Uy = (int)ceil(uy[n] - 0.5);
    }
    if (!isfinite(ux[n]) || !isfinite(uy[n]) || abs(Ux) > p->max_abs_shift ||
        abs(Uy) > p->max_abs_shift) {
      record_failure(s, n, ORC_ERR_NONPHYSICAL, &err);
      continue;
    }
    double du[4], dT[2], f[ORC_QMAX], g[ORC_QMAX];
    gradients(s, v, n, du, dT);
    int fb = 0;
    int rc = grad_populations(p, rho[n], ux[n], uy[n], T[n], du, dT, Ux, Uy, 0, f, g, &fb);
    fallbacks += fb;
    if (rc) {
      record_failure(s, n, rc, &err);
      continue;
    }
    for (int i = 0; i < s->Q; ++i) {
      s->fp[i * N + n] = f[i];
      s->gp[i * N + n] = g[i];
    }
    s->Un[2 * n] = Ux;
    s->Un[2 * n + 1] = Uy;
  }
  free(v);
  s->st.fallbacks = fallbacks;
  if (err) return err;
  return collide_all(s);
}

int orc_set_static_shift(orc_sim* s, const int* Ux, const int* Uy) {
  for (long n = 0; n < s->N; ++n) {
    s->Us[2 * n] = Ux[n];
    s->Us[2 * n + 1] = Uy[n];
  }
  return ORC_OK;
}

int orc_step(orc_sim* s, int nsteps) {
  const long N = s->N;
  const long nx = s->p.nx, ny = s->p.ny;
  const int Q = s->Q;
  for (int k = 0; k < nsteps; ++k) {
    int err = 0;
    long mism = 0, fallbacks = 0;
    /* streaming, eq. (stream), pull form: h_i(x, t+1) = h*_i(x - c_i, t) when
     * x and x - c_i use the same lattice, otherwise eq. (GradGeneral) with
     * macros and gradients at x - c_i (Sec. IV.A.4). */
#pragma omp parallel for schedule(static) reduction(+ : mism, fallbacks)
    for (long n = 0; n < N; ++n) {
      const long x = n % nx, y = n / nx;
      const int Ux = s->Un[2 * n], Uy = s->Un[2 * n + 1];
      for (int i = 0; i < Q; ++i) {
        long sx = wrap(x - (cx_of(Q, i) + Ux), nx);
        long sy = wrap(y - (cy_of(Q, i) + Uy), ny);
        long src = sy * nx + sx;
        if (s->Uc[2 * src] == Ux && s->Uc[2 * src + 1] == Uy) {
          s->fp[i * N + n] = s->f[i * N + src];
          s->gp[i * N + n] = s->g[i * N + src];
        } else {
          mism += 1;
          int fb = 0;
          int rc = reconstruct(s, src, Ux, Uy, i, &s->fp[i * N + n], &s->gp[i * N + n], &fb);
          fallbacks += fb;
          if (rc) record_failure(s, n, rc, &err);
        }
      }
    }
    s->st.mismatched_links += mism;
    s->st.fallbacks += fallbacks;
    if (err) return err;
    int rc = collide_all(s);
    if (rc) return rc;
    s->st.steps += 1;
  }
  return ORC_OK;
}

void orc_macros(const orc_sim* s, double* rho, double* ux, double* uy, double* T,
                int* Ucx, int* Ucy, int* Unx, int* Uny) {
  for (long n = 0; n < s->N; ++n) {
    if (rho) rho[n] = s->mac[4 * n];
    if (ux) ux[n] = s->mac[4 * n + 1];
    if (uy) uy[n] = s->mac[4 * n + 2];
    if (T) T[n] = s->mac[4 * n + 3];
    if (Ucx) Ucx[n] = s->Uc[2 * n];
    if (Ucy) Ucy[n] = s->Uc[2 * n + 1];
    if (Unx) Unx[n] = s->Un[2 * n];
    if (Uny) Uny[n] = s->Un[2 * n + 1];
  }
}

void orc_populations(const orc_sim* s, double* f, double* g) {
  size_t bytes = sizeof(double) * s->Q * (size_t)s->N;
  if (f) memcpy(f, s->f, bytes);
  if (g) memcpy(g, s->g, bytes);
}

void orc_conserved(const orc_sim* s, double* out4) {
  long double m = 0, px = 0, py = 0, en = 0;
  const long N = s->N;
  for (long n = 0; n < N; ++n) {
    for (int i = 0; i < s->Q; ++i) {
      long double f = s->f[i * N + n], g = s->g[i * N + n];
      long double cx = cx_of(s->Q, i) + s->Uc[2 * n], cy = cy_of(s->Q, i) + s->Uc[2 * n + 1];
      m += f;
      px += f * cx;
      py += f * cy;
      en += 0.5L * ((cx * cx + cy * cy) * f + g);
    }
  }
  out4[0] = (double)m;
  out4[1] = (double)px;
  out4[2] = (double)py;
  out4[3] = (double)en;
}

void orc_get_stats(const orc_sim* s, orc_stats* out) { *out = s->st; }
