// Numerical equilibrium with the four constraints of mass, momentum and
// total energy (Sec. "Reduced models", eq. feqNum_4Mom), solved per lane in
// FP64 registers:
//
//   f_i^eq = rho w_i,  w_i = exp(-(1 + l0 + l1x x_i + l1y y_i + l2 |xi_i|^2)),
//   sum_i w_i (1, x_i, y_i, |xi_i|^2) = (1, u'_x, u'_y, |u'|^2 + D T)
//
// in the frame of the lattice (peculiar velocity u' = u - U; the span of the
// four monomials is invariant under integer translations).  Compared with
// the 8-moment set it leaves the pressure tensor and the heat flux free, so
// it costs a 4 x 4 solve instead of 8 x 8 but does not recover the
// convective terms at non-zero u' (the paper's reason for the 8-moment set).
//
// Newton on G(l) = sum_i w_i phi_i - m with H = sum_i w_i phi_i phi_i^T
// (the Hessian of the strictly convex dual Psi(l) = sum_i w_i(l) + l . m)
// from a guess near the root (the lattice Maxwellian l1 = -u'/T,
// l2 = 1/(2T) corrected by a table); stop at
// max_a |G_a| <= tol, then one more step so that the constraints hold to
// rounding.  The start is interpolated in a table of solutions built on the
// device; where plain steps fail, steps halved until Psi decreases.
#pragma once

#include "equilibrium.hpp"

namespace lbm {

constexpr int kM4 = 4;

// Weights for multipliers l (l[0] includes the 1 of the exponent) and the
// dual's value sum_i w_i.
__device__ __forceinline__ double weights4(const double (&l)[kM4], Weights& w) {
  w.w0 = exp_cw(-(1.0 + l[0]));
  double z = w.w0;
  static_for<0, kPairs>([&](auto pc) {
    constexpr int p = decltype(pc)::value;
    constexpr int x = kPX[p], y = kPY[p], s = x * x + y * y;
    const double even = cmad<s>(1.0 + l[0], l[3]);
    const double odd = cmad<y>(cmad<x>(0.0, l[1]), l[2]);
    w.wp[p] = exp_cw(-(even + odd));
    w.wm[p] = exp_cw(-(even - odd));
    z += w.wp[p] + w.wm[p];
  });
  return z;
}

// G = sum_i w_i phi_i - m and the 10 entries of H (row-major upper
// triangle: 00 01 02 03 11 12 13 22 23 33).
__device__ __forceinline__ void moments4(const Weights& w, const double (&m)[kM4],
                                         double (&G)[kM4], double (&H)[10]) {
  double s0 = w.w0, sx = 0.0, sy = 0.0, ss = 0.0;
  double xx = 0.0, xy = 0.0, xs = 0.0, yy = 0.0, ys = 0.0, s2 = 0.0;
  static_for<0, kPairs>([&](auto pc) {
    constexpr int p = decltype(pc)::value;
    constexpr int x = kPX[p], y = kPY[p], s = x * x + y * y;
    const double S = w.wp[p] + w.wm[p];
    const double D = w.wp[p] - w.wm[p];
    s0 += S;
    sx = cmad<x>(sx, D);
    sy = cmad<y>(sy, D);
    ss = cmad<s>(ss, S);
    xx = cmad<x * x>(xx, S);
    xy = cmad<x * y>(xy, S);
    xs = cmad<x * s>(xs, D);
    yy = cmad<y * y>(yy, S);
    ys = cmad<y * s>(ys, D);
    s2 = cmad<s * s>(s2, S);
  });
  G[0] = s0 - m[0];
  G[1] = sx - m[1];
  G[2] = sy - m[2];
  G[3] = ss - m[3];
  H[0] = s0; H[1] = sx; H[2] = sy; H[3] = ss;
  H[4] = xx; H[5] = xy; H[6] = xs;
  H[7] = yy; H[8] = ys;
  H[9] = s2;
}

// Solves H d = G by LDL^T of the symmetric 4 x 4 matrix; false if a pivot
// is not positive (H is positive definite for finite weights).
__device__ __forceinline__ bool solve4(const double (&H)[10], const double (&G)[kM4],
                                       double (&d)[kM4]) {
  // L (unit lower) and D of H = L D L^T
  const double d0 = H[0];
  if (!(d0 > 0.0)) return false;
  const double i0 = rcp64(d0);
  const double l10 = H[1] * i0, l20 = H[2] * i0, l30 = H[3] * i0;
  const double d1 = H[4] - l10 * H[1];
  if (!(d1 > 0.0)) return false;
  const double i1 = rcp64(d1);
  const double l21 = (H[5] - l20 * H[1]) * i1;
  const double l31 = (H[6] - l30 * H[1]) * i1;
  const double d2 = H[7] - l20 * H[2] - l21 * l21 * d1;
  if (!(d2 > 0.0)) return false;
  const double i2 = rcp64(d2);
  const double l32 = (H[8] - l30 * H[2] - l31 * l21 * d1) * i2;
  const double d3 = H[9] - l30 * H[3] - l31 * l31 * d1 - l32 * l32 * d2;
  if (!(d3 > 0.0)) return false;
  const double i3 = rcp64(d3);
  // L y = G, D z = y, L^T d = z
  const double y0 = G[0];
  const double y1 = G[1] - l10 * y0;
  const double y2 = G[2] - l20 * y0 - l21 * y1;
  const double y3 = G[3] - l30 * y0 - l31 * y1 - l32 * y2;
  d[3] = y3 * i3;
  d[2] = y2 * i2 - l32 * d[3];
  d[1] = y1 * i1 - l21 * d[2] - l31 * d[3];
  d[0] = y0 * i0 - l10 * d[1] - l20 * d[2] - l30 * d[3];
  return true;
}

// Globalised solve: Newton with backtracking on the dual, weights always
// recomputed from the multipliers.
__device__ __forceinline__ NewtonOut solve_robust4(const double (&m)[kM4], double T, double tol,
                                                   int max_iter, Weights& w, double (&l)[kM4]) {
  NewtonOut out{0, false};
  {
    const double iT = rcp64(T);
    l[0] = 0.0;
    l[1] = -m[1] * iT;
    l[2] = -m[2] * iT;
    l[3] = 0.5 * iT;
    // normalise: sum_i w_i = 1
    const double z = weights4(l, w);
    if (!(z > 1e-300) || !(z < 1e300)) return out;
    l[0] = log(z);
  }
  double psi = weights4(l, w);
#pragma unroll
  for (int a = 0; a < kM4; ++a) psi += l[a] * m[a];
  for (int it = 0; it < max_iter; ++it) {
    double G[kM4], H[10], d[kM4];
    moments4(w, m, G, H);
    double r = 0.0;
#pragma unroll
    for (int a = 0; a < kM4; ++a) r = fmax(r, fabs(G[a]));
    out.iters = it + 1;
    if (!(r < 1e300) || !(psi < 1e300)) return out;
    if (!solve4(H, G, d)) return out;
    if (r <= tol) {
#pragma unroll
      for (int a = 0; a < kM4; ++a) l[a] += d[a];
      weights4(l, w);
      out.ok = true;
      return out;
    }
    // the dual decreases along d at rate -G . d < 0
    double slope = 0.0;
#pragma unroll
    for (int a = 0; a < kM4; ++a) slope -= G[a] * d[a];
    double t = 1.0;
    for (int k = 0; k < 60; ++k) {
      double lt[kM4];
#pragma unroll
      for (int a = 0; a < kM4; ++a) lt[a] = __builtin_fma(t, d[a], l[a]);
      double pt = weights4(lt, w);
#pragma unroll
      for (int a = 0; a < kM4; ++a) pt += lt[a] * m[a];
      bool accept = pt <= psi + 1e-4 * t * slope;
      if (!accept && t == 1.0 && pt < 1e300) {
        // a full step that halves the residual is taken even where the
        // dual's decrease falls below its rounding
        double Gt[kM4], Ht[10];
        moments4(w, m, Gt, Ht);
        double rt = 0.0;
#pragma unroll
        for (int a = 0; a < kM4; ++a) rt = fmax(rt, fabs(Gt[a]));
        accept = rt < 0.5 * r;
      }
      if (accept) {
#pragma unroll
        for (int a = 0; a < kM4; ++a) l[a] = lt[a];
        psi = pt;
        break;
      }
      t *= 0.5;
      if (k == 59) return out;
    }
  }
  return out;
}

// Targets per unit density: (1, u'_x, u'_y, 2E) with 2E = |u'|^2 + D T, D = 2.
__device__ __forceinline__ void targets4(double ux, double uy, double T, double (&m)[kM4]) {
  m[0] = 1.0;
  m[1] = ux;
  m[2] = uy;
  m[3] = ux * ux + uy * uy + 2.0 * T;
}

// Multipliers guessed from a table of the four-constraint solution over
// (|u'_x|, |u'_y|, 1/T) (the same grid and record layout as the 8-moment
// table; each record holds l1x + |u'_x|/T, l1y + |u'_y|/T, l2 - 1/(2T), 1 in
// its first four floats), trilinear, odd multipliers unfolded by the
// reflections; the lattice Maxwellian outside the table or next to a corner
// that did not converge.  l[0] is left for the normalisation.
__device__ __forceinline__ void table_guess4(const GuessTable& tb, double ux, double uy,
                                             double iT, double (&l)[kM4]) {
  l[0] = 0.0;
  l[1] = -ux * iT;
  l[2] = -uy * iT;
  l[3] = 0.5 * iT;
  const float a = fabsf(static_cast<float>(ux)), b = fabsf(static_cast<float>(uy));
  const float s = static_cast<float>(iT);
  const bool inside = a <= tb.umax && b <= tb.umax && s >= tb.smin && s <= tb.smax;
  const float fa = fminf(a, tb.umax) * tb.inv_hu, fb = fminf(b, tb.umax) * tb.inv_hu;
  const float fs = (fminf(fmaxf(s, tb.smin), tb.smax) - tb.smin) * tb.inv_hs;
  const int ia = min(static_cast<int>(fa), tb.nu - 2);
  const int ib = min(static_cast<int>(fb), tb.nu - 2);
  const int is = min(static_cast<int>(fs), tb.ns - 2);
  const float ta = fa - ia, tb_ = fb - ib, ts = fs - is;
  float4 v[8];
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    const int da = c & 1, db = (c >> 1) & 1, ds = c >> 2;
    v[c] = *reinterpret_cast<const float4*>(
        tb.data + (((static_cast<long>(is + ds) * tb.nu + (ib + db)) * tb.nu + (ia + da)) << 3));
  }
  float acc[4] = {0, 0, 0, 0};
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    const int da = c & 1, db = (c >> 1) & 1, ds = c >> 2;
    const float wgt = (da ? ta : 1.0f - ta) * (db ? tb_ : 1.0f - tb_) * (ds ? ts : 1.0f - ts);
    acc[0] = __builtin_fmaf(wgt, v[c].x, acc[0]);
    acc[1] = __builtin_fmaf(wgt, v[c].y, acc[1]);
    acc[2] = __builtin_fmaf(wgt, v[c].z, acc[2]);
    acc[3] = __builtin_fmaf(wgt, v[c].w, acc[3]);
  }
  const bool ok = inside && fabsf(acc[3]) < 1e30f;
  const double sx = ux < 0.0 ? -1.0 : 1.0, sy = uy < 0.0 ? -1.0 : 1.0;
  l[1] += ok ? sx * acc[0] : 0.0;
  l[2] += ok ? sy * acc[1] : 0.0;
  l[3] += ok ? acc[2] : 0.0;
}

// Plain Newton from the table guess with the weights carried and
// updated multiplicatively, w_i *= exp(-d . phi_i), by the same tiered
// polynomials / exp_cw as the 8-moment solve (a step (d0, d1x, d1y, d2) of
// the four multipliers is the step (d0, d1x, d1y, d2, 0, d2, 0, 0) of the
// eight, since |xi|^2 = x^2 + y^2); the globalised solve_robust4 where it
// fails.
__device__ __forceinline__ NewtonOut solve_equilibrium4(const GuessTable& tb, double ux,
                                                        double uy, double T, double tol,
                                                        int max_iter, Weights& w) {
  NewtonOut out{0, false};
  if (!(T > 0.0) || !(T < 1e300)) return out;
  double m[kM4];
  targets4(ux, uy, T, m);
  {
    double l[kM4];
    table_guess4(tb, ux, uy, rcp64(T), l);
    const double z = weights4(l, w);
    if (!(z > 1e-300) || !(z < 1e300)) return out;
    const double iz = rcp64(z);
    w.w0 *= iz;
#pragma unroll
    for (int p = 0; p < kPairs; ++p) {
      w.wp[p] *= iz;
      w.wm[p] *= iz;
    }
  }
  bool ok = false;
  for (int it = 0; it < max_iter; ++it) {
    double G[kM4], H[10], d4[kM4];
    moments4(w, m, G, H);
    double r = 0.0;
#pragma unroll
    for (int a = 0; a < kM4; ++a) r = fmax(r, fabs(G[a]));
    out.iters = it + 1;
    if (!(r < 1e300) || !solve4(H, G, d4)) break;
    double d[kM] = {d4[0], d4[1], d4[2], d4[3], 0.0, d4[3], 0.0, 0.0};
    if (r <= tol) {
      linear_update(d, w);
      ok = true;
      break;
    }
    double dmax = 0.0;
#pragma unroll
    for (int a = 0; a < kM4; ++a) dmax = fmax(dmax, fabs(d4[a]));
    if (dmax > 1.0) {
      const double sc = 1.0 / dmax;
#pragma unroll
      for (int a = 0; a < kM; ++a) d[a] *= sc;
    }
    exp_update(d, w);
  }
  if (ok) {
    out.ok = true;
    return out;
  }
  double l[kM4];
  const NewtonOut rb = solve_robust4(m, T, tol, max_iter, w, l);
  out.iters += rb.iters;
  out.ok = rb.ok;
  return out;
}

}  // namespace lbm
