// Numerical equilibrium of the paper's reference model (App. C): the D2Q49
// lattice {-3, ..., 3}^2 with 13 constraints, eqs. (G0)-(G4yyaa), solved per
// lane in FP64 registers:
//
//   w_i = exp(-l . phi(xi_i)),  sum_i w_i phi(xi_i) = m(u', T),
//   phi = (1, x, y, x^2, xy, y^2, x^3, x^2 y, x y^2, y^3,
//          x^2 |xi|^2, xy |xi|^2, y^2 |xi|^2)
//
// in the frame of the lattice (peculiar velocity u' = u - U; every monomial
// of degree <= 3 is in the span, so the span is invariant under integer
// translations).  l[0] includes the 1 of the exponent.  The printed
// exponent of eq. (feqNum_13Mom) lists no multiplier for x^3 although G_3,xxx
// is a constraint; it is taken as a dropped term (13 multipliers).
//
// Newton on G(l) = sum_i w_i phi_i - m with H = sum_i w_i phi_i phi_i^T, the
// Hessian of the strictly convex dual Psi(l) = sum_i w_i(l) + l . m, from
// the lattice Maxwellian, steps halved until Psi decreases (a full step is
// also taken when it halves the residual); stop at max_a |G_a| <= tol, then
// one more step so that the constraints hold to rounding.
//
// G and H need only the 45 power moments mu(p, q) = sum_i w_i x^p y^q,
// p + q <= 8; they are taken row by row, the rows and columns of the
// lattice folded by their +- symmetry (odd powers from differences, even
// powers from sums).
#pragma once

#include "equilibrium.hpp"

namespace lbm {

constexpr int kQ49 = 49;
constexpr int kM13 = 13;
constexpr int kTri13 = kM13 * (kM13 + 1) / 2;

// Storage plane k of D2Q49: velocity (k mod 7 - 3, k div 7 - 3).
__host__ __device__ constexpr int cx49(int k) { return k % 7 - 3; }
__host__ __device__ constexpr int cy49(int k) { return k / 7 - 3; }

// Monomial a as a sum of one or two terms x^p y^q.
constexpr int kNT13[kM13] = {1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 2, 2, 2};
constexpr int kTP13[kM13][2] = {{0, 0}, {1, 0}, {0, 0}, {2, 0}, {1, 0}, {0, 0}, {3, 0},
                                {2, 0}, {1, 0}, {0, 0}, {4, 2}, {3, 1}, {2, 0}};
constexpr int kTQ13[kM13][2] = {{0, 0}, {0, 0}, {1, 0}, {0, 0}, {1, 0}, {2, 0}, {0, 0},
                                {1, 0}, {2, 0}, {3, 0}, {0, 2}, {1, 3}, {2, 4}};

__host__ __device__ constexpr int phi13(int a, int x, int y) {
  int v = 0;
  for (int t = 0; t < kNT13[a]; ++t) v += ipow(x, kTP13[a][t]) * ipow(y, kTQ13[a][t]);
  return v;
}

// Exponent l . phi(x, y) of velocity (x, y), coefficients folded in.
template <int X, int Y>
__device__ __forceinline__ double exponent13(const double (&l)[kM13]) {
  double e = l[0];
  static_for<1, kM13>([&](auto ac) {
    constexpr int a = decltype(ac)::value;
    e = cmad<phi13(a, X, Y)>(e, l[a]);
  });
  return e;
}

// Weight of plane k for multipliers l.
template <int K>
__device__ __forceinline__ double weight13(const double (&l)[kM13]) {
  return exp_cw(-exponent13<cx49(K), cy49(K)>(l));
}

// Power moments mu[p][q], p + q <= 8, of the weights of l (mu[0][0] is
// sum_i w_i).  Along a row y the exponent splits into a part even in x,
// A(y) + x^2 B(y) + x^4 l10, and an odd one, x C(y) + x^3 D(y), so that
// each +-x pair costs two products and a sum and a difference.
__device__ __forceinline__ void power_moments13(const double (&l)[kM13], double (&mu)[9][9]) {
  static_for<0, 9>([&](auto pc) {
    constexpr int p = decltype(pc)::value;
    static_for<0, 9 - p>([&](auto qc) { mu[p][decltype(qc)::value] = 0.0; });
  });
  const double l1012 = l[10] + l[12];
  // r[p] = sum_x x^p w(x, y) of row y, for the rows y and -y together
  static_for<0, 4>([&](auto yc) {
    constexpr int y = decltype(yc)::value;
    double rp[9], rm[9];
    static_for<0, (y == 0 ? 1 : 2)>([&](auto sc) {
      constexpr int yy = decltype(sc)::value == 0 ? y : -y;
      double r[9];
      // l0 + l2 y + l5 y^2 + l9 y^3 + l12 y^4; l3 + l7 y + (l10 + l12) y^2;
      // l1 + l4 y + l8 y^2 + l11 y^3; l6 + l11 y
      const double A = cmad<yy * yy * yy * yy>(
          cmad<yy * yy * yy>(cmad<yy * yy>(cmad<yy>(l[0], l[2]), l[5]), l[9]), l[12]);
      const double B = cmad<yy * yy>(cmad<yy>(l[3], l[7]), l1012);
      const double C = cmad<yy * yy * yy>(cmad<yy * yy>(cmad<yy>(l[1], l[4]), l[8]), l[11]);
      const double Dd = cmad<yy>(l[6], l[11]);
      const double w0 = exp_cw(-A);
      double S[4], D[4];
      static_for<1, 4>([&](auto xc) {
        constexpr int x = decltype(xc)::value;
        const double even = __builtin_fma(static_cast<double>(x * x * x * x), l[10],
                                          __builtin_fma(static_cast<double>(x * x), B, A));
        const double odd = __builtin_fma(static_cast<double>(x * x * x), Dd,
                                         static_cast<double>(x) * C);
        const double wp = exp_cw(-(even + odd));
        const double wm = exp_cw(-(even - odd));
        S[x] = wp + wm;
        D[x] = wp - wm;
      });
      static_for<0, 9>([&](auto pc) {
        constexpr int p = decltype(pc)::value;
        double acc = p == 0 ? w0 : 0.0;
        static_for<1, 4>([&](auto xc) {
          constexpr int x = decltype(xc)::value;
          acc = cmad<ipow(x, p)>(acc, (p & 1) ? D[x] : S[x]);
        });
        r[p] = acc;
      });
      static_for<0, 9>([&](auto pc) {
        constexpr int p = decltype(pc)::value;
        if constexpr (decltype(sc)::value == 0)
          rp[p] = r[p];
        else
          rm[p] = r[p];
      });
    });
    static_for<0, 9>([&](auto pc) {
      constexpr int p = decltype(pc)::value;
      if constexpr (y == 0) {
        mu[p][0] += rp[p];
      } else {
        const double s = rp[p] + rm[p], d = rp[p] - rm[p];
        static_for<0, 9 - p>([&](auto qc) {
          constexpr int q = decltype(qc)::value;
          mu[p][q] = cmad<ipow(y, q)>(mu[p][q], (q & 1) ? d : s);
        });
      }
    });
  });
}

// Targets per unit density, eqs. (G0)-(G4yyaa), 2E = |u'|^2 + D T, D = 2.
__device__ __forceinline__ void targets13(double ux, double uy, double T, double (&m)[kM13]) {
  const double E = 0.5 * (ux * ux + uy * uy + 2.0 * T);
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
}

__host__ __device__ constexpr int tri13(int i, int j) { return i * (i + 1) / 2 + j; }

// G_a = sum of mu over the terms of monomial a, minus m_a; lower triangle
// of H from the products of terms.
__device__ __forceinline__ void residual13(const double (&mu)[9][9], const double (&m)[kM13],
                                           double (&G)[kM13]) {
  static_for<0, kM13>([&](auto ac) {
    constexpr int a = decltype(ac)::value;
    double g = mu[kTP13[a][0]][kTQ13[a][0]];
    if constexpr (kNT13[a] == 2) g += mu[kTP13[a][1]][kTQ13[a][1]];
    G[a] = g - m[a];
  });
}

__device__ __forceinline__ void hessian13(const double (&mu)[9][9], double (&H)[kTri13]) {
  static_for<0, kM13>([&](auto ac) {
    constexpr int a = decltype(ac)::value;
    static_for<0, a + 1>([&](auto bc) {
      constexpr int b = decltype(bc)::value;
      double h = 0.0;
      static_for<0, kNT13[a]>([&](auto sc) {
        constexpr int s = decltype(sc)::value;
        static_for<0, kNT13[b]>([&](auto tc) {
          constexpr int t = decltype(tc)::value;
          h += mu[kTP13[a][s] + kTP13[b][t]][kTQ13[a][s] + kTQ13[b][t]];
        });
      });
      H[tri13(a, b)] = h;
    });
  });
}

// Solves H d = G by an in-place LDL^T of the symmetric positive definite
// 13 x 13 matrix (lower triangle, row-major); false on a non-positive pivot.
__device__ __forceinline__ bool solve13(double (&A)[kTri13], const double (&G)[kM13],
                                        double (&d)[kM13]) {
  double inv[kM13];
#pragma unroll
  for (int j = 0; j < kM13; ++j) {
    // A(j, k) for k < j holds L(j, k) D(k); turn row j into L and D
#pragma unroll
    for (int k = 0; k < j; ++k) {
      const double ljk = A[tri13(j, k)] * inv[k];
      A[tri13(j, j)] -= ljk * A[tri13(j, k)];
#pragma unroll
      for (int i = j + 1; i < kM13; ++i) A[tri13(i, j)] -= A[tri13(i, k)] * ljk;
      A[tri13(j, k)] = ljk;
    }
    const double dj = A[tri13(j, j)];
    if (!(dj > 0.0)) return false;
    inv[j] = rcp64(dj);
  }
  double y[kM13];
#pragma unroll
  for (int i = 0; i < kM13; ++i) {
    double v = G[i];
#pragma unroll
    for (int k = 0; k < i; ++k) v -= A[tri13(i, k)] * y[k];
    y[i] = v;
  }
#pragma unroll
  for (int i = kM13 - 1; i >= 0; --i) {
    double v = y[i] * inv[i];
#pragma unroll
    for (int k = i + 1; k < kM13; ++k) v -= A[tri13(k, i)] * d[k];
    d[i] = v;
  }
  return true;
}

// Guess table of the 13-constraint solution over (|u'_x|, |u'_y|, 1/T), the
// grid of the D2Q21 table, 16 floats per point: l_1 .. l_12 minus the
// lattice Maxwellian's (l_1 + |u'_x|/T, l_2 + |u'_y|/T, l_3 - 1/(2T), l_4,
// l_5 - 1/(2T), l_6 .. l_12), 1 (NaN where the solve failed), zeros.
constexpr int kRec13 = 16;

__global__ __launch_bounds__(256) void table13_kernel(float* out, int nu, int ns, float umax,
                                                      float smin, float smax, double tol,
                                                      int max_iter);

// Trilinear guess from the table, multipliers odd in x (odd in y) unfolded
// by the sign of u'_x (u'_y); the lattice Maxwellian outside the table or
// next to a corner that did not converge.  l[0] is left for the
// normalisation.
__device__ __forceinline__ void table_guess13(const GuessTable& tb, double ux, double uy,
                                              double iT, double (&l)[kM13]) {
#pragma unroll
  for (int a = 0; a < kM13; ++a) l[a] = 0.0;
  l[1] = -ux * iT;
  l[2] = -uy * iT;
  l[3] = 0.5 * iT;
  l[5] = 0.5 * iT;
  if (tb.data == nullptr) return;
  const float a = fabsf(static_cast<float>(ux)), b = fabsf(static_cast<float>(uy));
  const float s = static_cast<float>(iT);
  const bool inside = a <= tb.umax && b <= tb.umax && s >= tb.smin && s <= tb.smax;
  const float fa = fminf(a, tb.umax) * tb.inv_hu, fb = fminf(b, tb.umax) * tb.inv_hu;
  const float fs = (fminf(fmaxf(s, tb.smin), tb.smax) - tb.smin) * tb.inv_hs;
  const int ia = min(static_cast<int>(fa), tb.nu - 2);
  const int ib = min(static_cast<int>(fb), tb.nu - 2);
  const int is = min(static_cast<int>(fs), tb.ns - 2);
  const float ta = fa - ia, tb_ = fb - ib, ts = fs - is;
  float acc[kRec13 - 3];
#pragma unroll
  for (int k = 0; k < kRec13 - 3; ++k) acc[k] = 0.0f;
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    const int da = c & 1, db = (c >> 1) & 1, ds = c >> 2;
    const float4* p = reinterpret_cast<const float4*>(
        tb.data + (((static_cast<long>(is + ds) * tb.nu + (ib + db)) * tb.nu + (ia + da)) << 4));
    const float wgt = (da ? ta : 1.0f - ta) * (db ? tb_ : 1.0f - tb_) * (ds ? ts : 1.0f - ts);
    float v[kRec13 - 3];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const float4 r = p[q];
      if (4 * q + 0 < kRec13 - 3) v[4 * q + 0] = r.x;
      if (4 * q + 1 < kRec13 - 3) v[4 * q + 1] = r.y;
      if (4 * q + 2 < kRec13 - 3) v[4 * q + 2] = r.z;
      if (4 * q + 3 < kRec13 - 3) v[4 * q + 3] = r.w;
    }
#pragma unroll
    for (int k = 0; k < kRec13 - 3; ++k) acc[k] = __builtin_fmaf(wgt, v[k], acc[k]);
  }
  if (!inside || !(fabsf(acc[12]) < 1e30f)) return;
  const double sx = ux < 0.0 ? -1.0 : 1.0, sy = uy < 0.0 ? -1.0 : 1.0;
  // signs under x -> -x and y -> -y of l_1 .. l_12
  constexpr int kOddX[kM13] = {0, 1, 0, 0, 1, 0, 1, 0, 1, 0, 0, 1, 0};
  constexpr int kOddY[kM13] = {0, 0, 1, 0, 1, 0, 0, 1, 0, 1, 0, 1, 0};
#pragma unroll
  for (int k = 1; k < kM13; ++k) {
    double v = acc[k - 1];
    if (kOddX[k]) v *= sx;
    if (kOddY[k]) v *= sy;
    l[k] += v;
  }
}

// Multipliers of the equilibrium at (u', T); the weights follow from
// weight13<k>(l).  The start: the table guess (tb.data non-null) or the
// lattice Maxwellian.
__device__ __forceinline__ NewtonOut solve_equilibrium13(const GuessTable& tb, double ux,
                                                         double uy, double T, double tol,
                                                         int max_iter, double (&l)[kM13]) {
  NewtonOut out{0, false};
  if (!(T > 0.0) || !(T < 1e300) || !(fabs(ux) < 1e300) || !(fabs(uy) < 1e300)) return out;
  double m[kM13];
  targets13(ux, uy, T, m);
  double mu[9][9];
  {
    table_guess13(tb, ux, uy, rcp64(T), l);
    power_moments13(l, mu);
    const double z = mu[0][0];
    if (!(z > 1e-300) || !(z < 1e300)) return out;
    l[0] = log(z);  // sum_i w_i = 1: every moment scales by 1 / z
    const double iz = rcp64(z);
    static_for<0, 9>([&](auto pc) {
      constexpr int p = decltype(pc)::value;
      static_for<0, 9 - p>([&](auto qc) { mu[p][decltype(qc)::value] *= iz; });
    });
  }
  double psi = mu[0][0];
#pragma unroll
  for (int a = 0; a < kM13; ++a) psi += l[a] * m[a];
  for (int it = 0; it < max_iter; ++it) {
    double G[kM13], H[kTri13], d[kM13];
    residual13(mu, m, G);
    hessian13(mu, H);
    double r = 0.0;
#pragma unroll
    for (int a = 0; a < kM13; ++a) r = fmax(r, fabs(G[a]));
    out.iters = it + 1;
    if (!(r < 1e300) || !(psi < 1e300)) return out;
    if (!solve13(H, G, d)) return out;
    if (r <= tol) {
#pragma unroll
      for (int a = 0; a < kM13; ++a) l[a] += d[a];
      out.ok = true;
      return out;
    }
    // the dual decreases along d at rate -G . d < 0
    double slope = 0.0;
#pragma unroll
    for (int a = 0; a < kM13; ++a) slope -= G[a] * d[a];
    double t = 1.0;
    bool moved = false;
    for (int k = 0; k < 60; ++k) {
      double lt[kM13];
#pragma unroll
      for (int a = 0; a < kM13; ++a) lt[a] = __builtin_fma(t, d[a], l[a]);
      power_moments13(lt, mu);
      double pt = mu[0][0];
#pragma unroll
      for (int a = 0; a < kM13; ++a) pt += lt[a] * m[a];
      bool accept = pt <= psi + 1e-4 * t * slope;
      if (!accept && t == 1.0 && pt < 1e300) {
        double Gt[kM13];
        residual13(mu, m, Gt);
        double rt = 0.0;
#pragma unroll
        for (int a = 0; a < kM13; ++a) rt = fmax(rt, fabs(Gt[a]));
        accept = rt < 0.5 * r;
      }
      if (accept) {
#pragma unroll
        for (int a = 0; a < kM13; ++a) l[a] = lt[a];
        psi = pt;
        moved = true;
        break;
      }
      t *= 0.5;
    }
    if (!moved) return out;
    // mu now holds the moments of the accepted point
  }
  return out;
}

}  // namespace lbm

namespace lbm {

// One lane per table point: the solve from the lattice Maxwellian.
__global__ __launch_bounds__(256) void table13_kernel(float* out, int nu, int ns, float umax,
                                                      float smin, float smax, double tol,
                                                      int max_iter) {
  const int idx = blockIdx.x * 256 + threadIdx.x;
  if (idx >= nu * nu * ns) return;
  const int ia = idx % nu, ib = (idx / nu) % nu, is = idx / (nu * nu);
  const double a = umax * static_cast<double>(ia) / (nu - 1);
  const double b = umax * static_cast<double>(ib) / (nu - 1);
  const double s = smin + (smax - smin) * static_cast<double>(is) / (ns - 1);
  double l[kM13];
  const GuessTable none{nullptr, 0, 0, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
  const NewtonOut no = solve_equilibrium13(none, a, b, 1.0 / s, tol, max_iter, l);
  float* o = out + static_cast<long>(kRec13) * idx;
  for (int k = 0; k < kRec13; ++k) o[k] = 0.0f;
  if (!no.ok) {
    o[12] = __builtin_nanf("");
    return;
  }
  o[0] = static_cast<float>(l[1] + a * s);
  o[1] = static_cast<float>(l[2] + b * s);
  o[2] = static_cast<float>(l[3] - 0.5 * s);
  o[3] = static_cast<float>(l[4]);
  o[4] = static_cast<float>(l[5] - 0.5 * s);
  for (int k = 6; k < kM13; ++k) o[k - 1] = static_cast<float>(l[k]);
  o[12] = 1.0f;
}

}  // namespace lbm
