// Numerical (maximum-entropy) equilibrium of the 8-moment set on D2Q21,
// solved per lane in FP64 registers.
//
// f_i^eq = rho w_i, w_i = exp(-(1 + lambda . phi(xi_i))) with
// phi = (1, x, y, x^2, xy, y^2, x|xi|^2, y|xi|^2) (eq. feqNum_8Mom), and the
// multipliers chosen so that sum_i w_i phi(xi_i) equals the per-unit-density
// targets of eqs. (G0_8mom)-(G3yaa_8mom), written in the frame of the
// lattice (peculiar velocity u - U).
//
// Newton on G(lambda) = sum_i w_i phi_i - m with Jacobian -H,
// H = sum_i w_i phi_i phi_i^T (symmetric positive definite): lambda += H^-1 G.
// Every entry of G and H is one of the 28 monomial moments
// M_pq = sum_i w_i x_i^p y_i^q, p + q <= 6; with the +- pairing the even ones
// come from S_p = w+ + w- and the odd ones from D_p = w+ - w-, and all
// velocity components are compile-time constants.  H is factored by LDL^T.
// The loop stops when max_a |G_a| <= tol and then applies the final Newton
// correction to the weights to first order (w_i *= 1 - delta . phi_i), which
// leaves the constraints satisfied to rounding.
#pragma once

#include "lattice.hpp"

namespace lbm {

struct Weights {
  double wp[kPairs];  // w at +v_p
  double wm[kPairs];  // w at -v_p
  double w0;          // rest
};

// even part: base + l0 + l3 x^2 + l4 xy + l5 y^2 ; odd part: l1 x + l2 y + s (l6 x + l7 y)
template <int p>
__device__ __forceinline__ void pair_exponent(const double (&l)[kM], double base, double& even,
                                              double& odd) {
  constexpr int x = kPX[p], y = kPY[p], s = x * x + y * y;
  even = cmad<y * y>(cmad<x * y>(cmad<x * x>(base + l[0], l[3]), l[4]), l[5]);
  odd = cmad<s * y>(cmad<s * x>(cmad<y>(cmad<x>(0.0, l[1]), l[2]), l[6]), l[7]);
}

template <int p = 0>
__device__ __forceinline__ void eval_weights(const double (&l)[kM], Weights& w) {
  if constexpr (p == 0) w.w0 = exp(-(1.0 + l[0]));
  if constexpr (p < kPairs) {
    double e, o;
    pair_exponent<p>(l, 1.0, e, o);
    w.wp[p] = exp(-(e + o));
    w.wm[p] = exp(-(e - o));
    eval_weights<p + 1>(l, w);
  }
}

// w_i *= 1 - d . phi_i  (first-order update for a tiny final correction d)
template <int p = 0>
__device__ __forceinline__ void linear_update(const double (&d)[kM], Weights& w) {
  if constexpr (p == 0) w.w0 = __builtin_fma(-w.w0, d[0], w.w0);
  if constexpr (p < kPairs) {
    double e, o;
    pair_exponent<p>(d, 0.0, e, o);
    w.wp[p] = __builtin_fma(-w.wp[p], e + o, w.wp[p]);
    w.wm[p] = __builtin_fma(-w.wm[p], e - o, w.wm[p]);
    linear_update<p + 1>(d, w);
  }
}

template <int P, int Qy, int p = 0>
__device__ __forceinline__ double mom_acc(double acc, const double (&S)[kPairs],
                                          const double (&D)[kPairs]) {
  if constexpr (p == kPairs) {
    return acc;
  } else {
    constexpr int c = ipow(kPX[p], P) * ipow(kPY[p], Qy);
    if constexpr ((P + Qy) % 2 == 0)
      return mom_acc<P, Qy, p + 1>(cmad<c>(acc, S[p]), S, D);
    else
      return mom_acc<P, Qy, p + 1>(cmad<c>(acc, D[p]), S, D);
  }
}

template <int P, int Qy>
__device__ __forceinline__ double mom(const double (&S)[kPairs], const double (&D)[kPairs],
                                      double w0) {
  return mom_acc<P, Qy>((P + Qy == 0) ? w0 : 0.0, S, D);
}

struct NewtonOut {
  int iters;  // residual evaluations, including the converged one
  bool ok;
};

// Solves for the weights at peculiar velocity (ux, uy) and temperature T.
__device__ __forceinline__ NewtonOut solve_equilibrium(double ux, double uy, double T,
                                                       double tol, int max_iter, Weights& w) {
  NewtonOut out{0, false};
  const double E = 0.5 * (ux * ux + uy * uy + 2.0 * T);  // 2E = u^2 + D T, D = 2
  const double m[kM] = {1.0,         ux, uy, ux * ux + T, ux * uy, uy * uy + T,
                        2.0 * ux * (E + T), 2.0 * uy * (E + T)};
  // initial guess: lattice-normalised Maxwellian (lambda_1 = -u/T,
  // lambda_2 = I/(2T)); the normalisation is folded into the weights.
  const double iT = 1.0 / T;
  double l[kM] = {-1.0, -ux * iT, -uy * iT, 0.5 * iT, 0.0, 0.5 * iT, 0.0, 0.0};
  eval_weights(l, w);
  {
    double Z = w.w0;
#pragma unroll
    for (int p = 0; p < kPairs; ++p) Z += w.wp[p] + w.wm[p];
    const double iZ = 1.0 / Z;
    w.w0 *= iZ;
#pragma unroll
    for (int p = 0; p < kPairs; ++p) {
      w.wp[p] *= iZ;
      w.wm[p] *= iZ;
    }
    l[0] = log(Z) - 1.0;
  }
  for (int it = 0; it < max_iter; ++it) {
    double S[kPairs], D[kPairs];
#pragma unroll
    for (int p = 0; p < kPairs; ++p) {
      S[p] = w.wp[p] + w.wm[p];
      D[p] = w.wp[p] - w.wm[p];
    }
    const double w0 = w.w0;
    const double M00 = mom<0, 0>(S, D, w0), M10 = mom<1, 0>(S, D, w0), M01 = mom<0, 1>(S, D, w0);
    const double M20 = mom<2, 0>(S, D, w0), M11 = mom<1, 1>(S, D, w0), M02 = mom<0, 2>(S, D, w0);
    const double M30 = mom<3, 0>(S, D, w0), M21 = mom<2, 1>(S, D, w0), M12 = mom<1, 2>(S, D, w0);
    const double M03 = mom<0, 3>(S, D, w0);
    double G[kM] = {M00 - m[0], M10 - m[1], M01 - m[2], M20 - m[3],
                    M11 - m[4], M02 - m[5], M30 + M12 - m[6], M21 + M03 - m[7]};
    double r = 0.0;
#pragma unroll
    for (int a = 0; a < kM; ++a) r = fmax(r, fabs(G[a]));
    out.iters = it + 1;
    if (!(r < 1e300)) return out;  // NaN or overflow
    const double M40 = mom<4, 0>(S, D, w0), M31 = mom<3, 1>(S, D, w0), M22 = mom<2, 2>(S, D, w0);
    const double M13 = mom<1, 3>(S, D, w0), M04 = mom<0, 4>(S, D, w0);
    const double M50 = mom<5, 0>(S, D, w0), M41 = mom<4, 1>(S, D, w0), M32 = mom<3, 2>(S, D, w0);
    const double M23 = mom<2, 3>(S, D, w0), M14 = mom<1, 4>(S, D, w0), M05 = mom<0, 5>(S, D, w0);
    const double M60 = mom<6, 0>(S, D, w0), M51 = mom<5, 1>(S, D, w0), M42 = mom<4, 2>(S, D, w0);
    const double M33 = mom<3, 3>(S, D, w0), M24 = mom<2, 4>(S, D, w0), M15 = mom<1, 5>(S, D, w0);
    const double M06 = mom<0, 6>(S, D, w0);
    // Hessian, lower triangle, basis (1, x, y, x2, xy, y2, x|xi|^2, y|xi|^2)
    double H[kM][kM];
    H[0][0] = M00;
    H[1][0] = M10; H[1][1] = M20;
    H[2][0] = M01; H[2][1] = M11; H[2][2] = M02;
    H[3][0] = M20; H[3][1] = M30; H[3][2] = M21; H[3][3] = M40;
    H[4][0] = M11; H[4][1] = M21; H[4][2] = M12; H[4][3] = M31; H[4][4] = M22;
    H[5][0] = M02; H[5][1] = M12; H[5][2] = M03; H[5][3] = M22; H[5][4] = M13; H[5][5] = M04;
    H[6][0] = M30 + M12; H[6][1] = M40 + M22; H[6][2] = M31 + M13; H[6][3] = M50 + M32;
    H[6][4] = M41 + M23; H[6][5] = M32 + M14; H[6][6] = M60 + 2.0 * M42 + M24;
    H[7][0] = M21 + M03; H[7][1] = M31 + M13; H[7][2] = M22 + M04; H[7][3] = M41 + M23;
    H[7][4] = M32 + M14; H[7][5] = M23 + M05; H[7][6] = M51 + 2.0 * M33 + M15;
    H[7][7] = M42 + 2.0 * M24 + M06;
    // LDL^T: Ld[i][j] = L[i][j] d[j]
    double L[kM][kM], Ld[kM][kM], id[kM];
    bool spd = true;
#pragma unroll
    for (int j = 0; j < kM; ++j) {
      double dj = H[j][j];
#pragma unroll
      for (int k = 0; k < j; ++k) dj -= L[j][k] * Ld[j][k];
      spd = spd && (dj > 0.0);
      id[j] = 1.0 / dj;
#pragma unroll
      for (int i = j + 1; i < kM; ++i) {
        double v = H[i][j];
#pragma unroll
        for (int k = 0; k < j; ++k) v -= L[i][k] * Ld[j][k];
        Ld[i][j] = v;
        L[i][j] = v * id[j];
      }
    }
    if (!spd) return out;
    double d[kM];
#pragma unroll
    for (int i = 0; i < kM; ++i) {
      double v = G[i];
#pragma unroll
      for (int k = 0; k < i; ++k) v -= L[i][k] * d[k];
      d[i] = v;
    }
#pragma unroll
    for (int i = 0; i < kM; ++i) d[i] *= id[i];
#pragma unroll
    for (int i = kM - 1; i >= 0; --i) {
      double v = d[i];
#pragma unroll
      for (int k = i + 1; k < kM; ++k) v -= L[k][i] * d[k];
      d[i] = v;
    }
    if (r <= tol) {
      linear_update(d, w);
      out.ok = true;
      return out;
    }
    // limit the step (max norm 1) far from the root
    double dmax = 0.0;
#pragma unroll
    for (int a = 0; a < kM; ++a) dmax = fmax(dmax, fabs(d[a]));
    const double sc = dmax > 1.0 ? 1.0 / dmax : 1.0;
#pragma unroll
    for (int a = 0; a < kM; ++a) l[a] = __builtin_fma(sc, d[a], l[a]);
    eval_weights(l, w);
  }
  return out;
}

}  // namespace lbm
