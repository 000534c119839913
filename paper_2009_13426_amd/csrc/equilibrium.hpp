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
// velocity components are compile-time constants.  H is factored in place by
// LDL^T.  The loop stops when max_a |G_a| <= tol and then applies the final
// Newton correction to the weights to first order (w_i *= 1 - delta . phi_i),
// which leaves the constraints satisfied to rounding.
//
// Two drivers share these pieces:
//   solve_robust  lattice-Maxwellian start, weights always recomputed from
//                 the multipliers with the library exp (table build);
//   solve_fast    start from an interpolated table of lambda - lambda_Maxwell,
//                 weights carried (not multipliers): later updates
//                 w *= exp(-delta . phi) by Taylor polynomials of degree 3
//                 (every |delta . phi| of the wave < 1e-5) or 7 (< 0.03) and
//                 by exp_cw otherwise; H is accumulated straight from the
//                 weights, one +- pair at a time, and the factors of the last
//                 step stay in registers for the final correction.
// Both stop on the same criterion, so both reach the unique root to rounding.
#pragma once

#include "lattice.hpp"

namespace lbm {

// e^x by Cody and Waite's argument reduction, x = k ln2 + r with k the
// nearest integer to x / ln2 and ln2 split in a head with trailing zero bits
// (exact k * head for |k| < 2^20) and a tail, then e^r from its Taylor
// polynomial of degree 13 on |r| <= ln2 / 2 (truncation below 5e-18
// relative) and the exact scaling by 2^k.  Finite arguments of magnitude up
// to ~700; NaN propagates.  Error within a few units in the last place.
__device__ __forceinline__ double exp_cw(double x) {
  constexpr double kLog2e = 1.4426950408889634074;
  constexpr double kLn2Hi = 6.93147180369123816490e-01;
  constexpr double kLn2Lo = 1.90821492927058770002e-10;
  const double k = __builtin_rint(x * kLog2e);
  double r = __builtin_fma(-k, kLn2Hi, x);
  r = __builtin_fma(-k, kLn2Lo, r);
  double p = 1.0 / 6227020800.0;  // 1/13!
  p = __builtin_fma(p, r, 1.0 / 479001600.0);
  p = __builtin_fma(p, r, 1.0 / 39916800.0);
  p = __builtin_fma(p, r, 1.0 / 3628800.0);
  p = __builtin_fma(p, r, 1.0 / 362880.0);
  p = __builtin_fma(p, r, 1.0 / 40320.0);
  p = __builtin_fma(p, r, 1.0 / 5040.0);
  p = __builtin_fma(p, r, 1.0 / 720.0);
  p = __builtin_fma(p, r, 1.0 / 120.0);
  p = __builtin_fma(p, r, 1.0 / 24.0);
  p = __builtin_fma(p, r, 1.0 / 6.0);
  p = __builtin_fma(p, r, 0.5);
  p = __builtin_fma(p, r, 1.0);
  p = __builtin_fma(p, r, 1.0);
  return __builtin_amdgcn_ldexp(p, static_cast<int>(k));
}

// exp(-z) as used for the weights: exp_cw, or the library exp when
// LBM_EXP_CW is 0.
#ifndef LBM_EXP_CW
#define LBM_EXP_CW 1
#endif
__device__ __forceinline__ double exp_neg(double z) {
#if LBM_EXP_CW
  return exp_cw(-z);
#else
  return exp(-z);
#endif
}

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
  if constexpr (p == 0) w.w0 = exp_neg(1.0 + l[0]);
  if constexpr (p < kPairs) {
    double e, o;
    pair_exponent<p>(l, 1.0, e, o);
    w.wp[p] = exp_neg(e + o);
    w.wm[p] = exp_neg(e - o);
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

// exp(-z) for |z| < 0.03 by its Taylor polynomial of degree 7.
__device__ __forceinline__ double expm_small(double z) {
  const double t = -z;
  double p = 1.0 / 5040.0;
  p = __builtin_fma(p, t, 1.0 / 720.0);
  p = __builtin_fma(p, t, 1.0 / 120.0);
  p = __builtin_fma(p, t, 1.0 / 24.0);
  p = __builtin_fma(p, t, 1.0 / 6.0);
  p = __builtin_fma(p, t, 0.5);
  p = __builtin_fma(p, t, 1.0);
  p = __builtin_fma(p, t, 1.0);
  return p;
}

// exp(-z) for |z| < 1e-5 by its Taylor polynomial of degree 3 (truncation
// below 1e-21 relative).
__device__ __forceinline__ double expm_tiny(double z) {
  const double t = -z;
  double p = 1.0 / 6.0;
  p = __builtin_fma(p, t, 0.5);
  p = __builtin_fma(p, t, 1.0);
  return __builtin_fma(p, t, 1.0);
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

__device__ __forceinline__ void pair_sums(const Weights& w, double (&S)[kPairs],
                                          double (&D)[kPairs]) {
#pragma unroll
  for (int p = 0; p < kPairs; ++p) {
    S[p] = w.wp[p] + w.wm[p];
    D[p] = w.wp[p] - w.wm[p];
  }
}

// Moments up to third order and the residual G; returns max |G_a|.
struct LowMoments {
  double M00, M10, M01, M20, M11, M02, M30, M21, M12, M03;
};

__device__ __forceinline__ double residual(const double (&S)[kPairs], const double (&D)[kPairs],
                                           double w0, const double (&m)[kM], LowMoments& L,
                                           double (&G)[kM]) {
  L.M00 = mom<0, 0>(S, D, w0);
  L.M10 = mom<1, 0>(S, D, w0);
  L.M01 = mom<0, 1>(S, D, w0);
  L.M20 = mom<2, 0>(S, D, w0);
  L.M11 = mom<1, 1>(S, D, w0);
  L.M02 = mom<0, 2>(S, D, w0);
  L.M30 = mom<3, 0>(S, D, w0);
  L.M21 = mom<2, 1>(S, D, w0);
  L.M12 = mom<1, 2>(S, D, w0);
  L.M03 = mom<0, 3>(S, D, w0);
  G[0] = L.M00 - m[0];
  G[1] = L.M10 - m[1];
  G[2] = L.M01 - m[2];
  G[3] = L.M20 - m[3];
  G[4] = L.M11 - m[4];
  G[5] = L.M02 - m[5];
  G[6] = L.M30 + L.M12 - m[6];
  G[7] = L.M21 + L.M03 - m[7];
  double r = 0.0;
#pragma unroll
  for (int a = 0; a < kM; ++a) r = fmax(r, fabs(G[a]));
  return r;
}

// Packed lower triangle of the symmetric 8x8 matrix: (i, j), j <= i.
__host__ __device__ constexpr int tri(int i, int j) { return i * (i + 1) / 2 + j; }
constexpr int kTri = kM * (kM + 1) / 2;

// Hessian in the basis (1, x, y, x2, xy, y2, x|xi|^2, y|xi|^2).
__device__ __forceinline__ void hessian(const double (&S)[kPairs], const double (&D)[kPairs],
                                        double w0, const LowMoments& L, double (&A)[kTri]) {
  const double M40 = mom<4, 0>(S, D, w0), M31 = mom<3, 1>(S, D, w0), M22 = mom<2, 2>(S, D, w0);
  const double M13 = mom<1, 3>(S, D, w0), M04 = mom<0, 4>(S, D, w0);
  const double M50 = mom<5, 0>(S, D, w0), M41 = mom<4, 1>(S, D, w0), M32 = mom<3, 2>(S, D, w0);
  const double M23 = mom<2, 3>(S, D, w0), M14 = mom<1, 4>(S, D, w0), M05 = mom<0, 5>(S, D, w0);
  const double M60 = mom<6, 0>(S, D, w0), M51 = mom<5, 1>(S, D, w0), M42 = mom<4, 2>(S, D, w0);
  const double M33 = mom<3, 3>(S, D, w0), M24 = mom<2, 4>(S, D, w0), M15 = mom<1, 5>(S, D, w0);
  const double M06 = mom<0, 6>(S, D, w0);
  A[tri(0, 0)] = L.M00;
  A[tri(1, 0)] = L.M10; A[tri(1, 1)] = L.M20;
  A[tri(2, 0)] = L.M01; A[tri(2, 1)] = L.M11; A[tri(2, 2)] = L.M02;
  A[tri(3, 0)] = L.M20; A[tri(3, 1)] = L.M30; A[tri(3, 2)] = L.M21; A[tri(3, 3)] = M40;
  A[tri(4, 0)] = L.M11; A[tri(4, 1)] = L.M21; A[tri(4, 2)] = L.M12; A[tri(4, 3)] = M31;
  A[tri(4, 4)] = M22;
  A[tri(5, 0)] = L.M02; A[tri(5, 1)] = L.M12; A[tri(5, 2)] = L.M03; A[tri(5, 3)] = M22;
  A[tri(5, 4)] = M13; A[tri(5, 5)] = M04;
  A[tri(6, 0)] = L.M30 + L.M12; A[tri(6, 1)] = M40 + M22; A[tri(6, 2)] = M31 + M13;
  A[tri(6, 3)] = M50 + M32; A[tri(6, 4)] = M41 + M23; A[tri(6, 5)] = M32 + M14;
  A[tri(6, 6)] = M60 + 2.0 * M42 + M24;
  A[tri(7, 0)] = L.M21 + L.M03; A[tri(7, 1)] = M31 + M13; A[tri(7, 2)] = M22 + M04;
  A[tri(7, 3)] = M41 + M23; A[tri(7, 4)] = M32 + M14; A[tri(7, 5)] = M23 + M05;
  A[tri(7, 6)] = M51 + 2.0 * M33 + M15; A[tri(7, 7)] = M42 + 2.0 * M24 + M06;
}

// 1/x to full double precision: hardware estimate plus two Newton-Raphson steps.
__device__ __forceinline__ double rcp64(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = __builtin_fma(__builtin_fma(-x, r, 1.0), r, r);
  r = __builtin_fma(__builtin_fma(-x, r, 1.0), r, r);
  return r;
}

// In-place LDL^T: strict lower part of A becomes L, id holds 1/D.
__device__ __forceinline__ bool ldl_factor(double (&A)[kTri], double (&id)[kM]) {
  bool spd = true;
#pragma unroll
  for (int j = 0; j < kM; ++j) {
    double t[kM];
#pragma unroll
    for (int k = 0; k < j; ++k) t[k] = A[tri(j, k)] * A[tri(k, k)];  // L_jk d_k
    double dj = A[tri(j, j)];
#pragma unroll
    for (int k = 0; k < j; ++k) dj = __builtin_fma(-A[tri(j, k)], t[k], dj);
    spd = spd && (dj > 0.0);
    A[tri(j, j)] = dj;
    id[j] = rcp64(dj);
#pragma unroll
    for (int i = j + 1; i < kM; ++i) {
      double v = A[tri(i, j)];
#pragma unroll
      for (int k = 0; k < j; ++k) v = __builtin_fma(-A[tri(i, k)], t[k], v);
      A[tri(i, j)] = v * id[j];
    }
  }
  return spd;
}

__device__ __forceinline__ void ldl_solve(const double (&A)[kTri], const double (&id)[kM],
                                          const double (&G)[kM], double (&d)[kM]) {
#pragma unroll
  for (int i = 0; i < kM; ++i) {
    double v = G[i];
#pragma unroll
    for (int k = 0; k < i; ++k) v = __builtin_fma(-A[tri(i, k)], d[k], v);
    d[i] = v;
  }
#pragma unroll
  for (int i = 0; i < kM; ++i) d[i] *= id[i];
#pragma unroll
  for (int i = kM - 1; i >= 0; --i) {
    double v = d[i];
#pragma unroll
    for (int k = i + 1; k < kM; ++k) v = __builtin_fma(-A[tri(k, i)], d[k], v);
    d[i] = v;
  }
}

__device__ __forceinline__ void targets(double ux, double uy, double T, double (&m)[kM]) {
  const double E = 0.5 * (ux * ux + uy * uy + 2.0 * T);  // 2E = u^2 + D T, D = 2
  m[0] = 1.0;
  m[1] = ux;
  m[2] = uy;
  m[3] = ux * ux + T;
  m[4] = ux * uy;
  m[5] = uy * uy + T;
  m[6] = 2.0 * ux * (E + T);
  m[7] = 2.0 * uy * (E + T);
}

struct NewtonOut {
  int iters;  // residual evaluations, including the converged one
  bool ok;
};

// Lattice-Maxwellian start (lambda_1 = -u/T, lambda_2 = I/(2T), the rest 0;
// lambda_0 from the normalisation), weights always recomputed from the
// multipliers.  Newton steps on the convex dual
// Psi(lambda) = sum_i w_i(lambda) + lambda . m (gradient -G, Hessian H),
// globalised by backtracking until Psi decreases by at least 1e-4 of the
// linear prediction (a full step is also taken when it halves max |G|, since
// near the root the change of Psi drops below its rounding).  lam returns
// the multipliers of the converged weights (before the final first-order
// step).
__device__ __forceinline__ NewtonOut solve_robust(double ux, double uy, double T, double tol,
                                                  int max_iter, Weights& w, double (&l)[kM]) {
  NewtonOut out{0, false};
  double m[kM];
  targets(ux, uy, T, m);
  const double iT = 1.0 / T;
  l[0] = -1.0;
  l[1] = -ux * iT;
  l[2] = -uy * iT;
  l[3] = 0.5 * iT;
  l[4] = 0.0;
  l[5] = 0.5 * iT;
  l[6] = 0.0;
  l[7] = 0.0;
  eval_weights(l, w);
  {
    double Z = w.w0;
#pragma unroll
    for (int p = 0; p < kPairs; ++p) Z += w.wp[p] + w.wm[p];
    if (!(Z < 1e300) || !(Z > 1e-300)) return out;
    const double iZ = 1.0 / Z;
    w.w0 *= iZ;
#pragma unroll
    for (int p = 0; p < kPairs; ++p) {
      w.wp[p] *= iZ;
      w.wm[p] *= iZ;
    }
    l[0] = log(Z) - 1.0;
  }
  auto dual = [&](const Weights& v, const double (&lv)[kM]) {
    double psi = v.w0;
#pragma unroll
    for (int p = 0; p < kPairs; ++p) psi += v.wp[p] + v.wm[p];
#pragma unroll
    for (int a = 0; a < kM; ++a) psi = __builtin_fma(lv[a], m[a], psi);
    return psi;
  };
  double psi = dual(w, l);
  for (int it = 0; it < max_iter; ++it) {
    double S[kPairs], D[kPairs], G[kM], A[kTri], id[kM], d[kM];
    LowMoments LM;
    pair_sums(w, S, D);
    const double r = residual(S, D, w.w0, m, LM, G);
    out.iters = it + 1;
    if (!(r < 1e300) || !(psi < 1e300)) return out;
    hessian(S, D, w.w0, LM, A);
    if (!ldl_factor(A, id)) return out;
    ldl_solve(A, id, G, d);
    if (r <= tol) {
      linear_update(d, w);
      out.ok = true;
      return out;
    }
    double slope = 0.0;  // directional derivative of Psi along d: -G . d < 0
#pragma unroll
    for (int a = 0; a < kM; ++a) slope = __builtin_fma(-G[a], d[a], slope);
    double t = 1.0;
    for (;;) {
      double lt[kM];
#pragma unroll
      for (int a = 0; a < kM; ++a) lt[a] = __builtin_fma(t, d[a], l[a]);
      Weights wt;
      eval_weights(lt, wt);
      const double pt = dual(wt, lt);
      bool take = pt < 1e300 && pt <= psi + 1e-4 * t * slope;
      if (!take && t == 1.0 && pt < 1e300) {
        double St[kPairs], Dt[kPairs], Gt[kM];
        LowMoments Lt;
        pair_sums(wt, St, Dt);
        take = residual(St, Dt, wt.w0, m, Lt, Gt) < 0.5 * r;
      }
      if (take) {
#pragma unroll
        for (int a = 0; a < kM; ++a) l[a] = lt[a];
        w = wt;
        psi = pt;
        break;
      }
      t *= 0.5;
      if (t < 1e-12) return out;
    }
  }
  return out;
}

// Geometry of the initial-guess table: dlambda = lambda - lambda_Maxwell
// for lambda_1 .. lambda_7 (lambda_0 follows from the normalisation) on a
// regular grid over a = |u_x|, b = |u_y| in [0, umax] and s = 1/T in
// [smin, smax]; 8 floats per point (7 values and a validity slot that holds
// NaN where the solve failed).
struct GuessTable {
  const float* data;  // [ns][nu][nu][8]
  int nu, ns;
  float umax, smin, smax, inv_hu, inv_hs;
};

// The table's part of a guess at (ux, uy, 1/T): the eight corners of the
// cell around (|u_x|, |u_y|, 1/T), clamped so that every read stays inside
// the table, and the interpolation weights.  Split from the interpolation
// so that a caller can issue the sixteen loads early and use them later.
struct GuessFetch {
  float4 v[8][2];
  float ta, tb, ts;
  bool inside;
};

__device__ __forceinline__ GuessFetch table_fetch(const GuessTable& tb, double ux, double uy,
                                                  double iT) {
  GuessFetch g;
  const float a = fabsf(static_cast<float>(ux)), b = fabsf(static_cast<float>(uy));
  const float s = static_cast<float>(iT);
  g.inside = a <= tb.umax && b <= tb.umax && s >= tb.smin && s <= tb.smax;
  const float fa = fminf(a, tb.umax) * tb.inv_hu, fb = fminf(b, tb.umax) * tb.inv_hu;
  const float fs = (fminf(fmaxf(s, tb.smin), tb.smax) - tb.smin) * tb.inv_hs;
  const int ia = min(static_cast<int>(fa), tb.nu - 2);
  const int ib = min(static_cast<int>(fb), tb.nu - 2);
  const int is = min(static_cast<int>(fs), tb.ns - 2);
  g.ta = fa - ia;
  g.tb = fb - ib;
  g.ts = fs - is;
  // all sixteen loads in flight before the first is used
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    const int da = c & 1, db = (c >> 1) & 1, ds = c >> 2;
    const float4* p = reinterpret_cast<const float4*>(
        tb.data + (((static_cast<long>(is + ds) * tb.nu + (ib + db)) * tb.nu + (ia + da)) << 3));
    g.v[c][0] = p[0];
    g.v[c][1] = p[1];
  }
  return g;
}

// lambda guess at (ux, uy, T) from a fetched cell; returns false (and
// leaves the lattice Maxwellian in l) when the state is outside the table.
__device__ __forceinline__ bool table_guess_from(const GuessFetch& g, double ux, double uy,
                                                 double iT, double (&l)[kM]) {
  l[0] = 0.0;
  l[1] = -ux * iT;
  l[2] = -uy * iT;
  l[3] = 0.5 * iT;
  l[4] = 0.0;
  l[5] = 0.5 * iT;
  l[6] = 0.0;
  l[7] = 0.0;
  float acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    const int da = c & 1, db = (c >> 1) & 1, ds = c >> 2;
    const float wgt = (da ? g.ta : 1.0f - g.ta) * (db ? g.tb : 1.0f - g.tb) * (ds ? g.ts : 1.0f - g.ts);
    acc[0] = __builtin_fmaf(wgt, g.v[c][0].x, acc[0]);
    acc[1] = __builtin_fmaf(wgt, g.v[c][0].y, acc[1]);
    acc[2] = __builtin_fmaf(wgt, g.v[c][0].z, acc[2]);
    acc[3] = __builtin_fmaf(wgt, g.v[c][0].w, acc[3]);
    acc[4] = __builtin_fmaf(wgt, g.v[c][1].x, acc[4]);
    acc[5] = __builtin_fmaf(wgt, g.v[c][1].y, acc[5]);
    acc[6] = __builtin_fmaf(wgt, g.v[c][1].z, acc[6]);
    acc[7] = __builtin_fmaf(wgt, g.v[c][1].w, acc[7]);
  }
  // outside the table, or a corner that failed to converge: Maxwellian start
  const bool ok = g.inside && fabsf(acc[7]) < 1e30f;
  const double sx = ux < 0.0 ? -1.0 : 1.0, sy = uy < 0.0 ? -1.0 : 1.0;
#pragma unroll
  for (int k = 0; k < 7; ++k) acc[k] = ok ? acc[k] : 0.0f;
  // unfold the reflections u_x -> -u_x, u_y -> -u_y
  l[1] += sx * acc[0];
  l[2] += sy * acc[1];
  l[3] += acc[2];
  l[4] += sx * sy * acc[3];
  l[5] += acc[4];
  l[6] += sx * acc[5];
  l[7] += sy * acc[6];
  return ok;
}

__device__ __forceinline__ bool table_guess(const GuessTable& tb, double ux, double uy, double iT,
                                            double (&l)[kM]) {
  return table_guess_from(table_fetch(tb, ux, uy, iT), ux, uy, iT, l);
}

// H accumulated directly from the weights, one +- pair at a time: the pair
// adds phi_a(v) phi_b(v) (w+ + w- or w+ - w-, by the parity of phi_a phi_b).
// Column 0 of H is sum_i w_i phi_a(xi_i), the constrained moments themselves.
template <int p, int a, int b>
__device__ __forceinline__ void hess_pair_entry(double (&A)[kTri], double S, double D) {
  constexpr int x = kPX[p], y = kPY[p], s = x * x + y * y;
  constexpr int phi[kM] = {1, x, y, x * x, x * y, y * y, x * s, y * s};
  constexpr int par[kM] = {1, -1, -1, 1, 1, 1, -1, -1};  // phi(-v) = par * phi(v)
  constexpr int c = phi[a] * phi[b];
  if constexpr (par[a] * par[b] > 0)
    A[tri(a, b)] = cmad<c>(A[tri(a, b)], S);
  else
    A[tri(a, b)] = cmad<c>(A[tri(a, b)], D);
}

template <int p, int idx = 0>
__device__ __forceinline__ void hess_pair(double (&A)[kTri], double S, double D) {
  if constexpr (idx < kTri) {
    constexpr int a = [] { int r = 0; while ((r + 1) * (r + 2) / 2 <= idx) ++r; return r; }();
    constexpr int b = idx - a * (a + 1) / 2;
    if constexpr (b > 0) hess_pair_entry<p, a, b>(A, S, D);
    hess_pair<p, idx + 1>(A, S, D);
  }
}

// H with column 0 taken from the constraint sums c; the other 28 entries
// accumulated pair by pair (the rest velocity adds to entry (0, 0) only).
template <int p = 0>
__device__ __forceinline__ void hessian_direct(const Weights& w, const double (&c)[kM],
                                               double (&A)[kTri]) {
  if constexpr (p == 0) {
#pragma unroll
    for (int k = 0; k < kTri; ++k) A[k] = 0.0;
  }
  if constexpr (p < kPairs) {
    const double S = w.wp[p] + w.wm[p], D = w.wp[p] - w.wm[p];
    hess_pair<p, 1>(A, S, D);
    hessian_direct<p + 1>(w, c, A);
  } else {
#pragma unroll
    for (int a = 0; a < kM; ++a) A[tri(a, 0)] = c[a];
  }
}

// In-place LDL^T; on return the diagonal holds 1/D (one reciprocal per
// pivot: the pivots themselves are kept aside while later columns need them).
__device__ __forceinline__ bool ldl_factor_inplace(double (&A)[kTri]) {
  bool spd = true;
  double dg[kM];
#pragma unroll
  for (int j = 0; j < kM; ++j) {
    double t[kM];
#pragma unroll
    for (int k = 0; k < j; ++k) t[k] = A[tri(j, k)] * dg[k];  // L_jk d_k
    double dj = A[tri(j, j)];
#pragma unroll
    for (int k = 0; k < j; ++k) dj = __builtin_fma(-A[tri(j, k)], t[k], dj);
    spd = spd && (dj > 0.0);
    dg[j] = dj;
    const double idj = rcp64(dj);
#pragma unroll
    for (int i = j + 1; i < kM; ++i) {
      double v = A[tri(i, j)];
#pragma unroll
      for (int k = 0; k < j; ++k) v = __builtin_fma(-A[tri(i, k)], t[k], v);
      A[tri(i, j)] = v * idj;
    }
    A[tri(j, j)] = idj;
  }
  return spd;
}

// Solves in place: G holds the right-hand side on entry, the step on return.
__device__ __forceinline__ void ldl_solve_inplace(const double (&A)[kTri], double (&G)[kM]) {
#pragma unroll
  for (int i = 0; i < kM; ++i) {
#pragma unroll
    for (int k = 0; k < i; ++k) G[i] = __builtin_fma(-A[tri(i, k)], G[k], G[i]);
  }
#pragma unroll
  for (int i = 0; i < kM; ++i) G[i] *= A[tri(i, i)];
#pragma unroll
  for (int i = kM - 1; i >= 0; --i) {
#pragma unroll
    for (int k = i + 1; k < kM; ++k) G[i] = __builtin_fma(-A[tri(k, i)], G[k], G[i]);
  }
}

// Even and odd parts of d . phi over the +- pairs (z = e +- o), computed
// once per step for the update and for its largest magnitude.
template <int p = 0>
__device__ __forceinline__ void step_exponents(const double (&d)[kM], double (&e)[kPairs],
                                               double (&o)[kPairs]) {
  if constexpr (p < kPairs) {
    pair_exponent<p>(d, 0.0, e[p], o[p]);
    step_exponents<p + 1>(d, e, o);
  }
}

// w_i *= F(z_i) for one of the exp(-z) evaluators below.
template <typename F>
__device__ __forceinline__ void scale_weights(double d0, const double (&e)[kPairs],
                                              const double (&o)[kPairs], Weights& w, F f) {
  w.w0 *= f(d0);
#pragma unroll
  for (int p = 0; p < kPairs; ++p) {
    w.wp[p] *= f(e[p] + o[p]);
    w.wm[p] *= f(e[p] - o[p]);
  }
}

// w_i *= exp(-d . phi_i): the degree-3 polynomial when every |d . phi_i| of
// every lane of the wave is below 1e-5, the degree-7 one below 0.03, exp
// otherwise.  The choice is made for the whole wave (a ballot), so that
// lanes never split over two evaluators: each one is exact over its range,
// and a wave runs one of them.
__device__ __forceinline__ void exp_update(const double (&d)[kM], Weights& w) {
  double e[kPairs], o[kPairs];
  step_exponents(d, e, o);
  double big = fabs(d[0]);
#pragma unroll
  for (int p = 0; p < kPairs; ++p) big = fmax(big, fabs(e[p]) + fabs(o[p]));
  if (__ballot(!(big < 0.03))) {
    scale_weights(d[0], e, o, w, [](double z) { return exp_neg(z); });
  } else if (__ballot(!(big < 1e-5))) {
    scale_weights(d[0], e, o, w, [](double z) { return expm_small(z); });
  } else {
    scale_weights(d[0], e, o, w, [](double z) { return expm_tiny(z); });
  }
}

// Sums sum_i w_i phi_a(xi_i), a = 0..7 (column 0 of H), from the +- pairs.
template <int p = 0>
__device__ __forceinline__ void constraint_moments(const Weights& w, double (&c)[kM]) {
  if constexpr (p == 0) {
    c[0] = w.w0;
#pragma unroll
    for (int a = 1; a < kM; ++a) c[a] = 0.0;
  }
  if constexpr (p < kPairs) {
    constexpr int x = kPX[p], y = kPY[p], sq = x * x + y * y;
    const double S = w.wp[p] + w.wm[p], D = w.wp[p] - w.wm[p];
    c[0] += S;
    c[1] = cmad<x>(c[1], D);
    c[2] = cmad<y>(c[2], D);
    c[3] = cmad<x * x>(c[3], S);
    c[4] = cmad<x * y>(c[4], S);
    c[5] = cmad<y * y>(c[5], S);
    c[6] = cmad<x * sq>(c[6], D);
    c[7] = cmad<y * sq>(c[7], D);
    constraint_moments<p + 1>(w, c);
  }
}

// Table start, then Newton steps applied to the weights multiplicatively (no
// multipliers are carried).  Stops on max |G| <= tol with a first-order
// final correction, solved with the factors of the last step, which are
// kept in registers: the residual is at the tolerance, so factors of a
// Hessian that moved by the size of that step take it to round-off.
// g: the table cell of (ux, uy, iT = 1/T), fetched by the caller.
__device__ __forceinline__ NewtonOut solve_fast(const GuessFetch& g, double iT, double ux,
                                                double uy, double T, double tol, int max_iter,
                                                Weights& w) {
  NewtonOut out{0, false};
  {
    // The first weights must be of exponential form to full FP64 accuracy:
    // the multiplicative updates below never touch components outside the
    // span of phi, so any noise introduced here would survive to the end.
    double l[kM];
    table_guess_from(g, ux, uy, iT, l);
    l[0] = -1.0;
    eval_weights(l, w);
  }
  {
    double Z = w.w0;
#pragma unroll
    for (int p = 0; p < kPairs; ++p) Z += w.wp[p] + w.wm[p];
    if (!(Z < 1e300) || !(Z > 1e-300)) return out;
    const double iZ = rcp64(Z);
    w.w0 *= iZ;
#pragma unroll
    for (int p = 0; p < kPairs; ++p) {
      w.wp[p] *= iZ;
      w.wm[p] *= iZ;
    }
  }
  const double ET = 0.5 * (ux * ux + uy * uy + 2.0 * T) + T;  // E + T
  // constraint targets, recomputed where used (cheaper than keeping them live)
  auto target = [&](int a) {
    return a == 0 ? 1.0
         : a == 1 ? ux
         : a == 2 ? uy
         : a == 3 ? ux * ux + T
         : a == 4 ? ux * uy
         : a == 5 ? uy * uy + T
         : a == 6 ? 2.0 * ux * ET
                  : 2.0 * uy * ET;
  };
  double A[kTri];  // factors of the last step's Hessian
  for (int it = 0; it < max_iter; ++it) {
    double G[kM];
    constraint_moments(w, G);
#pragma unroll
    for (int a = 0; a < kM; ++a) G[a] -= target(a);
    double r = 0.0;
#pragma unroll
    for (int a = 0; a < kM; ++a) r = fmax(r, fabs(G[a]));
    out.iters = it + 1;
    if (!(r < 1e300)) return out;
    if (r <= tol && it > 0) {
      // final correction with the last step's factors
      ldl_solve_inplace(A, G);
      linear_update(G, w);
      out.ok = true;
      return out;
    }
    {
      // column 0 of H is the constraint sums, G + m up to rounding
      double c[kM];
#pragma unroll
      for (int a = 0; a < kM; ++a) c[a] = G[a] + target(a);
      hessian_direct(w, c, A);
    }
    if (!ldl_factor_inplace(A)) return out;
    ldl_solve_inplace(A, G);  // G now holds the step
    if (r <= tol) {
      linear_update(G, w);
      out.ok = true;
      return out;
    }
    double dmax = 0.0;
#pragma unroll
    for (int a = 0; a < kM; ++a) dmax = fmax(dmax, fabs(G[a]));
    if (dmax > 1.0) {
      const double sc = 1.0 / dmax;
#pragma unroll
      for (int a = 0; a < kM; ++a) G[a] *= sc;
    }
    exp_update(G, w);
  }
  return out;
}

// solve_fast with its own fetch of the table cell.
__device__ __forceinline__ NewtonOut solve_fast(const GuessTable& tb, double ux, double uy,
                                                double T, double tol, int max_iter, Weights& w) {
  const double iT = rcp64(T);
  return solve_fast(table_fetch(tb, ux, uy, iT), iT, ux, uy, T, tol, max_iter, w);
}

// solve_fast from a cell fetched by the caller (table_fetch at iT = 1/T),
// and where it fails (a state far from the table or a start from which plain
// Newton steps do not converge) the globalised solve_robust.
__device__ __forceinline__ NewtonOut solve_equilibrium(const GuessFetch& g, double iT, double ux,
                                                       double uy, double T, double tol,
                                                       int max_iter, Weights& w) {
  NewtonOut out = solve_fast(g, iT, ux, uy, T, tol, max_iter, w);
  if (!out.ok) {
    double l[kM];
    const NewtonOut r = solve_robust(ux, uy, T, tol, max_iter, w, l);
    out.iters += r.iters;
    out.ok = r.ok;
  }
  return out;
}

// solve_fast, and where it fails (a state far from the table or a start
// from which plain Newton steps do not converge) the globalised solve_robust.
__device__ __forceinline__ NewtonOut solve_equilibrium(const GuessTable& tb, double ux, double uy,
                                                       double T, double tol, int max_iter,
                                                       Weights& w) {
  NewtonOut out = solve_fast(tb, ux, uy, T, tol, max_iter, w);
  if (!out.ok) {
    double l[kM];
    const NewtonOut r = solve_robust(ux, uy, T, tol, max_iter, w, l);
    out.iters += r.iters;
    out.ok = r.ok;
  }
  return out;
}

}  // namespace lbm
