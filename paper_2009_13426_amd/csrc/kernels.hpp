// Device kernels of the adaptive D2Q21 step (gfx950, wave64).
//
//   step_kernel<S, STREAM>  fused pull / rebuild / moments / shift / Newton /
//                           BGK / store, one node per lane (STREAM = false is
//                           the collide-only pass of the initial condition)
//   init_kernel<S>          Grad initial condition h(0) = h_eq (1 + phi)
//   macros_kernel<S>        moments of the stored populations
//   widen_kernel<S>         populations to FP64 for export
//   conserved_kernel<S>     per-block sums of mass, momentum, energy
//   reduce_partials_kernel  fixed-order final sum
//
// S is the storage type of the populations: double (FP64 form) or float
// (FP32 storage and collision, FP64 moments and Newton).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "equilibrium.hpp"
#include "equilibrium4.hpp"
#include "lattice.hpp"

#ifndef LBM_HIST_BINS
#define LBM_HIST_BINS 32
#endif
// Waves per SIMD the step kernel is compiled for (caps its registers): FP64
// storage and FP32 storage.
#ifndef LBM_STEP_WAVES_PER_EU
#define LBM_STEP_WAVES_PER_EU 2
#endif
#ifndef LBM_STEP_WAVES_PER_EU_F32
#define LBM_STEP_WAVES_PER_EU_F32 2
#endif

namespace lbm {

constexpr int kBlock = 256;
constexpr int kWaves = kBlock / 64;

struct DevDiag {
  unsigned long long fail_key;  // (step << 34) | (node << 3) | code, ~0 when clean
  unsigned long long newton_calls;
  unsigned long long newton_iters;
  unsigned long long mismatched;
  unsigned long long hist[LBM_HIST_BINS];
  unsigned long long step_base;  // added to the step of a failure (graph replays)
  unsigned long long fallbacks;  // solves that took the four-constraint equilibrium
};

enum : unsigned { kCodeNewton = 1, kCodeNonphysical = 2 };

struct Phys {
  double nu, Cv, Cp, halfwidth, tol;
  int max_iter, shift_mode, fixed_ux, fixed_uy, max_abs_shift, sensor, stats;
  int fallback;   // 1: four-constraint equilibrium where the 8-moment one fails
  double inv_pr;  // 1 / Prandtl number (1: BGK)
};

struct Grid {
  long long N;
  int nx, ny;
  int fast_x, fast_y;  // wrap by one conditional add/sub (grid wider than any reach)
};

// Per-node side arrays carried from one step to the next.
struct Carry {
  unsigned* mask;      // links of the node's next pull whose source collided in another lattice
  void* mac;           // [4][N] of S: rho, u'x, u'y, T of the last collision (lattice frame)
  int* list;           // nodes with a non-zero mask (first counters[parity] entries)
  unsigned* counters;  // [4]: list lengths (0, 1) and pair-queue lengths (2, 3),
                       // alternating with the step parity
  // D2Q21: the links to rebuild as (source node, receiver lattice) pairs,
  // each pair once: pairs[i] = source | (lattice16 << 32), at most pair_cap
  // entries; seen[s] marks the receiver lattices already queued for source
  // s (bit (dUx + 3) * 7 + (dUy + 3) of the lattice difference)
  unsigned long long* pairs;
  unsigned long long* seen;
  long long pair_cap;
};

enum : unsigned { kCodeQueueFull = 3 };

struct StepArgs {
  const void* fin;
  const void* gin;
  void* fout;  // on entry: the rebuilt links, each in its receiver's own slot
  void* gout;
  const int* tin;
  int* tout;
  Carry carry;
  Grid grid;
  Phys phys;
  GuessTable table;
  int step;
  DevDiag* diag;
  int ntiles;  // tiles of BLOCK nodes
  int tiles;   // tiles per workgroup, run one after the other
  int remap;   // 1: workgroups mapped to tiles by XCD (xcd_remap)
};

struct RebuildArgs {
  void* fout;       // buffer the coming step writes; rebuilt links go to their receiver's slot
  void* gout;
  const int* tags;  // current tags: Uc of every node, Un = lattice of its next pull
  Carry carry;
  Grid grid;
  Phys phys;
  GuessTable table;
  int step;  // index of the coming step
  DevDiag* diag;
};

struct InitArgs {
  const double* rho;
  const double* ux;
  const double* uy;
  const double* T;
  const int8_t* sux;
  const int8_t* suy;
  void* fout;
  void* gout;
  int* tout;
  Grid grid;
  Phys phys;
  GuessTable table;
  DevDiag* diag;
};

// ------------------------------------------------------------ helpers

__device__ __forceinline__ int wrapc(int v, int n, int fast) {
  if (fast) {
    v += (v < 0) ? n : 0;
    v -= (v >= n) ? n : 0;
    return v;
  }
  v %= n;
  return v < 0 ? v + n : v;
}

// Element idx of one population plane, addressed by a 32-bit byte offset
// from the plane's (wave-uniform) base; the host admits only grids whose
// planes are below 4 GiB.
template <typename S>
__device__ __forceinline__ const S& plane_at(const S* plane, unsigned idx) {
  return *reinterpret_cast<const S*>(reinterpret_cast<const char*>(plane) +
                                     idx * static_cast<unsigned>(sizeof(S)));
}
template <typename S>
__device__ __forceinline__ S& plane_at(S* plane, unsigned idx) {
  return *reinterpret_cast<S*>(reinterpret_cast<char*>(plane) +
                               idx * static_cast<unsigned>(sizeof(S)));
}

// Collided populations are written once per step and read once by the
// next, long after the caches have turned over: stored nontemporal.  (The
// pull's loads stay cached: a cache line of a source row serves the pulls
// of two neighbouring waves; nontemporal loads fetched 5 % more bytes for
// the same time.)
template <typename S>
__device__ __forceinline__ void stream_store(S* plane, unsigned idx, S v) {
  __builtin_nontemporal_store(v, &plane_at(plane, idx));
}

// Consecutive blocks are dispatched round-robin over the 8 XCDs; remap so
// that each XCD (own L2) works on one contiguous range of nodes.
__device__ __forceinline__ int xcd_remap(int b, int G) {
  const int q = G >> 3, r = G & 7, xcd = b & 7, idx = b >> 3;
  return xcd < r ? xcd * (q + 1) + idx : r * (q + 1) + (xcd - r) * q + idx;
}

__device__ __forceinline__ void record_failure(DevDiag* d, int step, long long node,
                                               unsigned code) {
  const unsigned long long key = ((static_cast<unsigned long long>(step) + d->step_base) << 34) |
                                 (static_cast<unsigned long long>(node) << 3) | code;
  atomicMin(&d->fail_key, key);
}

// Eq. (criterion) with optional hysteresis half-width hw >= 1/2.
__device__ __forceinline__ int select_axis(double u, int uprev, double hw) {
  if (u > uprev - hw && u <= uprev + hw) return uprev;
  return static_cast<int>(ceil(u - 0.5));
}

// Overlapping ranges of half-width hw in [1/2, 1) chosen by the
// neighbourhood (Sec. III.A.2): per axis the admissible shifts are the n
// with n - hw < u <= n + hw; among the admissible pairs, the one that the
// most of the four nearest neighbours collide in (nb16: the Un halves of
// their tags), ties to the node's own lattice, then to ceil(u - 1/2), then
// to the first pair in increasing x and then y order.
__device__ __forceinline__ void select_neighbourhood(double ux, double uy, int ucx, int ucy,
                                                     const int (&nb16)[4], double hw, int& nx,
                                                     int& ny) {
  const int c0x = static_cast<int>(ceil(ux - 0.5)), c0y = static_cast<int>(ceil(uy - 0.5));
  int best = -1;
  nx = c0x;
  ny = c0y;
  for (int dx = -1; dx <= 1; ++dx) {
    const int cx = c0x + dx;
    if (!(ux > cx - hw && ux <= cx + hw)) continue;
    for (int dy = -1; dy <= 1; ++dy) {
      const int cy = c0y + dy;
      if (!(uy > cy - hw && uy <= cy + hw)) continue;
      const int c16 = (cx & 0xFF) | ((cy & 0xFF) << 8);
      const int score = (nb16[0] == c16) + (nb16[1] == c16) + (nb16[2] == c16) + (nb16[3] == c16);
      const int rank = 4 * score + 2 * (cx == ucx && cy == ucy) + (dx == 0 && dy == 0);
      if (rank > best) {
        best = rank;
        nx = cx;
        ny = cy;
      }
    }
  }
}

template <int k>
__device__ __forceinline__ double weight_of(const Weights& w) {
  if constexpr (k == 0)
    return w.w0;
  else if constexpr (((k - 1) & 1) == 0)
    return w.wp[(k - 1) >> 1];
  else
    return w.wm[(k - 1) >> 1];
}

// Moments of one node's stored populations in its own lattice frame (all
// 42 loads issued before the first is used).
template <typename S>
__device__ __forceinline__ void node_moments(const S* f, const S* g, long long N, long long s,
                                             double& rho, double& upx, double& upy, double& T,
                                             double Cv) {
  S fv[kQ], gv[kQ];
  static_for<0, kQ>([&](auto kc) {
    constexpr int k = decltype(kc)::value;
    fv[k] = plane_at(f + k * N, static_cast<unsigned>(s));
    gv[k] = plane_at(g + k * N, static_cast<unsigned>(s));
  });
  double r = 0.0, jx = 0.0, jy = 0.0, e = 0.0;
  static_for<0, kQ>([&](auto kc) {
    constexpr int k = decltype(kc)::value;
    constexpr int cx = plane_cx(k), cy = plane_cy(k);
    const double fk = static_cast<double>(fv[k]);
    const double gk = static_cast<double>(gv[k]);
    r += fk;
    jx = cmad<cx>(jx, fk);
    jy = cmad<cy>(jy, fk);
    e = cmad<cx * cx + cy * cy>(e, fk) + gk;
  });
  rho = r;
  upx = jx / r;
  upy = jy / r;
  T = (e - r * (upx * upx + upy * upy)) / (2.0 * r * Cv);
}

// Grad deviations phi_f, phi_g (eqs. GradGeneral_f, GradGeneral_g) of
// velocity c = (cx, cy) (absolute) at (rho, u, T) with gradients
// du = (dux/dx, dux/dy, duy/dx, duy/dy), dT = (dT/dx, dT/dy).
struct GradState {
  double sxx, sxy, syy, qx, qy;  // sigma and q
  double rho, ux, uy, T;
};

__device__ __forceinline__ GradState grad_state(double rho, double ux, double uy, double T,
                                                const double (&du)[4], const double (&dT)[2],
                                                const Phys& P) {
  GradState s;
  const double mu = rho * P.nu;
  const double div = du[0] + du[3];
  s.sxx = -mu * (2.0 * du[0] - div);  // 2/D = 1
  s.syy = -mu * (2.0 * du[3] - div);
  s.sxy = -mu * (du[1] + du[2]);
  const double kappa = rho * P.Cp * P.nu * P.inv_pr;  // rho Cp nu / Pr
  s.qx = -kappa * dT[0];
  s.qy = -kappa * dT[1];
  s.rho = rho;
  s.ux = ux;
  s.uy = uy;
  s.T = T;
  return s;
}

// phi_g is used as printed in the paper: 2 q.cbar / (rho Cp).
constexpr double kGradGCoeff = 2.0;

__device__ __forceinline__ void grad_phi(const GradState& s, double cx, double cy,
                                         const Phys& P, double& phif, double& phig) {
  const double cbx = cx - s.ux, cby = cy - s.uy;
  const double qc = s.qx * cbx + s.qy * cby;
  const double c2 = cbx * cbx + cby * cby;
  const double T2 = s.T * s.T;
  phif = (s.sxx * cbx * cbx + 2.0 * s.sxy * cbx * cby + s.syy * cby * cby) / (2.0 * s.rho * T2) +
         qc / (s.rho * P.Cp * T2) * (c2 / (2.0 * s.T) - P.Cp);
  phig = kGradGCoeff * qc / (s.rho * P.Cp);
}

// Flexible-Prandtl collision (eq. Shakhov, App. E) on D2Q21 with the
// 8-moment equilibrium (and on D2Q49 with 13 constraints, which enforce
// the same low moments): BGK plus (1/tau - 1/tau_Pr) h_eq phi_S with q the
// heat flux (1/2) sum_i cbar_i (|cbar_i|^2 f_i + g_i), cbar = xi - u', of the
// populations being collided, and
//   phi_S,f = t - (b0 + b1 cbar_x + b2 cbar_y + b3 |cbar|^2),
//   t = q.cbar / (rho Cp T^2) (|cbar|^2 / (2T) - 2),  phi_S,g = q.cbar / (rho Cp T^2):
// t is the monatomic heat-flux shape (the printed one carries momentum with
// the polyatomic Cp), and the b's remove its projection on the collision
// invariants in the f_eq-weighted inner product, so that the collision
// conserves mass, momentum and energy on the lattice.  The Gram matrix of
// (1, cbar_x, cbar_y, |cbar|^2) is rho [[1, 0, 0, 2T], [0, T, 0, 0],
// [0, 0, T, 0], [2T, 0, 0, S4 / rho]] by the enforced moments up to the
// third order, S4 = sum_i f_eq |cbar|^4.
struct ShakhovCoef {
  double qx, qy, s0, b0, b1, b2, b3;
  double qu, bu, uu, upx, upy, h;  // q.u', b1 u'x + b2 u'y, |u'|^2, u', 1 / (2T)
};

// Velocity set of a lattice for the code shared by D2Q21 and D2Q49.
struct Lattice21 {
  static constexpr int Q = kQ;
  static constexpr int cx(int k) { return plane_cx(k); }
  static constexpr int cy(int k) { return plane_cy(k); }
};

// Coefficients from the equilibrium weights (wk(k) for the velocities of
// lattice L), the node's (rho, u', T) and its heat flux q.
template <class L = Lattice21, typename WeightOf>
__device__ __forceinline__ ShakhovCoef shakhov_coef(WeightOf&& wk, double rho, double upx,
                                                    double upy, double T, double qx, double qy,
                                                    const Phys& P) {
  ShakhovCoef c;
  c.qx = qx;
  c.qy = qy;
  c.s0 = 1.0 / (rho * P.Cp * T * T);
  const double h = 0.5 / T;
  double r0 = 0.0, r1 = 0.0, r2 = 0.0, r3 = 0.0, s4 = 0.0;
  static_for<0, L::Q>([&](auto kc) {
    constexpr int k = decltype(kc)::value;
    const double cx = L::cx(k) - upx, cy = L::cy(k) - upy;
    const double c2 = cx * cx + cy * cy;
    const double feq = rho * wk(kc);
    const double ft = feq * (c.s0 * (qx * cx + qy * cy) * __builtin_fma(c2, h, -2.0));
    r0 += ft;
    r1 = __builtin_fma(ft, cx, r1);
    r2 = __builtin_fma(ft, cy, r2);
    r3 = __builtin_fma(ft, c2, r3);
    s4 = __builtin_fma(feq * c2, c2, s4);
  });
  const double rT = rho * T;
  c.b1 = r1 / rT;
  c.b2 = r2 / rT;
  const double det = rho * s4 - 4.0 * rT * rT;
  c.b0 = (s4 * r0 - 2.0 * rT * r3) / det;
  c.b3 = (rho * r3 - 2.0 * rT * r0) / det;
  c.qu = qx * upx + qy * upy;
  c.bu = c.b1 * upx + c.b2 * upy;
  c.uu = upx * upx + upy * upy;
  c.upx = upx;
  c.upy = upy;
  c.h = h;
  return c;
}

// phi_S,f and phi_S,g of lattice velocity (CX, CY), cbar = c - u'; the
// products with cbar are expanded in c (integer) so that nothing is shared
// with the moments pass of shakhov_coef, whose per-velocity values would
// otherwise stay live into the collision.
template <int CX, int CY>
__device__ __forceinline__ void shakhov_phi(const ShakhovCoef& c, double& sf, double& sg) {
  const double c2 = static_cast<double>(CX * CX + CY * CY) -
                    2.0 * (CX * c.upx + CY * c.upy) + c.uu;
  const double a = c.s0 * (c.qx * CX + c.qy * CY - c.qu);
  sf = a * __builtin_fma(c2, c.h, -2.0) -
       (c.b0 + (c.b1 * CX + c.b2 * CY - c.bu) + c.b3 * c2);
  sg = a;
}

// Storage type of the carried moments for population storage type S: S
// itself (default), or FP64 in both forms with LBM_CARRY_FP64.
#ifndef LBM_CARRY_FP64
#define LBM_CARRY_FP64 0
#endif
template <typename S>
using CarryT = typename std::conditional<LBM_CARRY_FP64 != 0, double, S>::type;

// Absolute velocity and temperature of node s from the carried moments.
template <typename S>
__device__ __forceinline__ void carried_uT(const S* mac, const int* tags, long long N, long long s,
                                           double& ux, double& uy, double& T) {
  const int t = tags[s];
  ux = static_cast<double>(mac[N + s]) + tag_ucx(t);
  uy = static_cast<double>(mac[2 * N + s]) + tag_ucy(t);
  T = static_cast<double>(mac[3 * N + s]);
}

// The numerical equilibrium of the context's constraint set: the 8-moment
// set (eq. feqNum_8Mom, default) or mass, momentum and energy only (M = 4,
// eq. feqNum_4Mom).
template <int M>
__device__ __forceinline__ NewtonOut solve_of(const GuessTable& tb, double ux, double uy,
                                              double T, const Phys& P, Weights& w) {
  if constexpr (M == 4)
    return solve_equilibrium4(tb, ux, uy, T, P.tol, P.max_iter, w);
  else
    return solve_equilibrium(tb, ux, uy, T, P.tol, P.max_iter, w);
}

// solve_of, and with P.fallback set, where the 8-moment problem has no
// solution (its solve fails, e.g. a rebuilt link whose source moves at |u'|
// ~ 1.6 in the receiver's lattice), the four-constraint equilibrium of the
// same state, eq. (feqNum_4Mom), from the lattice Maxwellian with
// backtracking: it conserves mass, momentum and energy and exists for every
// velocity inside the lattice.  The paper leaves the case open; such a
// solve adds `uses` (the collision, or the rebuilt links it serves) to
// diag->fallbacks.
struct FallbackOut {
  Weights w;
  NewtonOut no;
};

// A call, not inlined: the rare path stays out of the register allocation of
// the kernels' common path.
__device__ __noinline__ FallbackOut solve_fallback4(double ux, double uy, double T, double tol,
                                                    int max_iter) {
  FallbackOut r;
  double m4[kM4], l4[kM4];
  targets4(ux, uy, T, m4);
  r.no = solve_robust4(m4, T, tol, max_iter, r.w, l4);
  return r;
}

// With P.fallback set, a failed 8-moment solve (no) is replaced by the
// four-constraint one of the same state.
__device__ __forceinline__ void fallback_if_failed(NewtonOut& no, double ux, double uy, double T,
                                                   const Phys& P, Weights& w, DevDiag* diag,
                                                   unsigned uses) {
  if (!no.ok && P.fallback) {
    const FallbackOut f = solve_fallback4(ux, uy, T, P.tol, P.max_iter);
    no.iters += f.no.iters;
    no.ok = f.no.ok;
    if (f.no.ok) {
      w = f.w;
      atomicAdd(&diag->fallbacks, static_cast<unsigned long long>(uses));
    }
  }
}

template <int M>
__device__ __forceinline__ NewtonOut solve_node(const GuessTable& tb, double ux, double uy,
                                                double T, const Phys& P, Weights& w,
                                                DevDiag* diag, unsigned uses = 1u) {
  NewtonOut no = solve_of<M>(tb, ux, uy, T, P, w);
  if constexpr (M == kM) fallback_if_failed(no, ux, uy, T, P, w, diag, uses);
  return no;
}

// The same for the 8-moment set from a table cell the caller fetched
// (table_fetch at iT = 1/T) ahead of the solve.
__device__ __forceinline__ NewtonOut solve_node(const GuessFetch& g, double iT, double ux,
                                                double uy, double T, const Phys& P, Weights& w,
                                                DevDiag* diag) {
  NewtonOut no = solve_equilibrium(g, iT, ux, uy, T, P.tol, P.max_iter, w);
  fallback_if_failed(no, ux, uy, T, P, w, diag, 1u);
  return no;
}

// The rebuilt links of one queued pair: source node s, receiver lattice
// (Lx, Ly).  Every receiver r = s + c_k + (Lx, Ly) whose next pull is in
// that lattice and whose link k is marked in its mask gets, in its own slot
// of the buffer the coming step writes, the post-collision population of
// plane k built by Grad's ansatz from the moments of s's last collision and
// central differences of its neighbours' (eq. GradGeneral with h* = h_eq +
// (1 - 1/tau) h_neq, tau = 1/2 + nu / T(s)), in the receiver's lattice at
// the source's state.  One equilibrium solve serves all the links of the
// pair.  Clears s's seen mask for the coming step's queue.
template <typename S, int M, bool PR = false>
__device__ __forceinline__ void rebuild_pair(const RebuildArgs& a, unsigned long long entry) {
  const CarryT<S>* mac = static_cast<const CarryT<S>*>(a.carry.mac);
  const long long N = a.grid.N;
  const int nx = a.grid.nx, ny = a.grid.ny;
  const Phys& P = a.phys;
  const unsigned s = static_cast<unsigned>(entry & 0xFFFFFFFFull);
  const int L16 = static_cast<int>((entry >> 32) & 0xFFFFull);
  const int Lx = static_cast<int8_t>(L16 & 0xFF), Ly = static_cast<int8_t>((L16 >> 8) & 0xFF);
  a.carry.seen[s] = 0ull;
  const int ys = static_cast<int>(s / static_cast<unsigned>(nx));
  const int xs = static_cast<int>(s - static_cast<unsigned>(ys) * static_cast<unsigned>(nx));
  // receivers of the pair: lattice L and link k marked (their indices are
  // recomputed at the writes rather than held across the solve)
  const auto receiver = [&](int k, int x0, int y0) {
    const int xr = wrapc(x0 + plane_cx(k) + Lx, nx, a.grid.fast_x);
    const int yr = wrapc(y0 + plane_cy(k) + Ly, ny, a.grid.fast_y);
    return static_cast<unsigned>(yr) * static_cast<unsigned>(nx) + static_cast<unsigned>(xr);
  };
  unsigned take = 0u;
  {
    int tg[kQ];
    unsigned mk[kQ];
    static_for<0, kQ>([&](auto kc) {
      constexpr int k = decltype(kc)::value;
      const unsigned r = receiver(k, xs, ys);
      tg[k] = a.tags[r];
      mk[k] = a.carry.mask[r];
    });
    static_for<0, kQ>([&](auto kc) {
      constexpr int k = decltype(kc)::value;
      if (tag_un16(tg[k]) == L16 && ((mk[k] >> k) & 1u)) take |= 1u << k;
    });
    // take is settled here: the gathered tags and masks die before the solve
    asm volatile("" : "+v"(take));
  }
  const double rho = static_cast<double>(mac[s]);
  double ux, uy, T;
  carried_uT<CarryT<S>>(mac, a.tags, N, s, ux, uy, T);
  if (!(rho > 0.0) || !(T > 0.0) || !(rho < 1e300) || !(T < 1e300)) {
    record_failure(a.diag, a.step, s, kCodeNonphysical);
    return;
  }
  Weights w;
  const NewtonOut no =
      solve_node<M>(a.table, ux - Lx, uy - Ly, T, P, w, a.diag, static_cast<unsigned>(__popc(take)));
  if (P.stats) {
    atomicAdd(&a.diag->newton_calls, 1ull);
    atomicAdd(&a.diag->newton_iters, static_cast<unsigned long long>(no.iters));
    atomicAdd(&a.diag->hist[no.iters < LBM_HIST_BINS ? no.iters : LBM_HIST_BINS - 1], 1ull);
    atomicAdd(&a.diag->mismatched, static_cast<unsigned long long>(__popc(take)));
  }
  if (!no.ok) {
    record_failure(a.diag, a.step, s, kCodeNewton);
    return;
  }
  // central differences of the neighbours' moments (loaded after the
  // solve, which then has their registers)
  double du[4] = {0.0, 0.0, 0.0, 0.0}, dT[2] = {0.0, 0.0};
  if (P.nu > 0.0) {
    const long long xp = (long long)ys * nx + wrapc(xs + 1, nx, a.grid.fast_x);
    const long long xm = (long long)ys * nx + wrapc(xs - 1, nx, a.grid.fast_x);
    const long long yp = (long long)wrapc(ys + 1, ny, a.grid.fast_y) * nx + xs;
    const long long ym = (long long)wrapc(ys - 1, ny, a.grid.fast_y) * nx + xs;
    double uxp, uyp, Tp, uxm, uym, Tm, vxp, vyp, Sp, vxm, vym, Sm;
    carried_uT<CarryT<S>>(mac, a.tags, N, xp, uxp, uyp, Tp);
    carried_uT<CarryT<S>>(mac, a.tags, N, xm, uxm, uym, Tm);
    carried_uT<CarryT<S>>(mac, a.tags, N, yp, vxp, vyp, Sp);
    carried_uT<CarryT<S>>(mac, a.tags, N, ym, vxm, vym, Sm);
    du[0] = 0.5 * (uxp - uxm);
    du[2] = 0.5 * (uyp - uym);
    dT[0] = 0.5 * (Tp - Tm);
    du[1] = 0.5 * (vxp - vxm);
    du[3] = 0.5 * (vyp - vym);
    dT[1] = 0.5 * (Sp - Sm);
  }
  const GradState gs = grad_state(rho, ux, uy, T, du, dT, P);
  const double tau = 0.5 + P.nu / T;
  const double kf = 1.0 - 1.0 / tau;
  const double gfac = (2.0 * P.Cv - 2.0) * T;
  ShakhovCoef sc{};
  double ks = 0.0;
  if constexpr (PR) {
    // eq. (Shakhov) applied to the Grad populations h = h_eq (1 + phi) of
    // the source (App. E): their heat flux in the receiver's frame, then
    // each link's share of the term
    const double upx = ux - Lx, upy = uy - Ly;
    double qx = 0.0, qy = 0.0;
    static_for<0, kQ>([&](auto kc) {
      constexpr int kk = decltype(kc)::value;
      double pf, pg;
      grad_phi(gs, static_cast<double>(plane_cx(kk) + Lx), static_cast<double>(plane_cy(kk) + Ly),
               P, pf, pg);
      const double fe = rho * weight_of<kk>(w);
      const double hf = fe * (1.0 + pf), hg = gfac * fe * (1.0 + pg);
      const double cx = plane_cx(kk) - upx, cy = plane_cy(kk) - upy;
      const double e = (cx * cx + cy * cy) * hf + hg;
      qx = __builtin_fma(0.5 * cx, e, qx);
      qy = __builtin_fma(0.5 * cy, e, qy);
    });
    sc = shakhov_coef([&](auto kc) { return weight_of<decltype(kc)::value>(w); }, rho, upx, upy,
                      T, qx, qy, P);
    const double tpr = 0.5 + (tau - 0.5) * P.inv_pr;
    ks = 1.0 / tau - 1.0 / tpr;
  }
  S* fout = static_cast<S*>(a.fout);
  S* gout = static_cast<S*>(a.gout);
  // an opaque copy of the source's position: the compiler would otherwise
  // keep the gather's receiver indices alive (spilled) across the solve
  int xw = xs, yw = ys;
  asm volatile("" : "+v"(xw), "+v"(yw));
  static_for<0, kQ>([&](auto kc) {
    constexpr int k = decltype(kc)::value;
    if ((take >> k) & 1u) {
      double phif, phig;
      grad_phi(gs, static_cast<double>(plane_cx(k) + Lx), static_cast<double>(plane_cy(k) + Ly), P,
               phif, phig);
      const double feq = rho * weight_of<k>(w);
      const double geq = gfac * feq;
      double rf = feq * (1.0 + kf * phif);
      double rg = geq * (1.0 + kf * phig);
      if constexpr (PR) {
        double sf, sg;
        shakhov_phi<plane_cx(k), plane_cy(k)>(sc, sf, sg);
        rf += ks * feq * sf;
        rg += ks * geq * sg;
      }
      const unsigned r = receiver(k, xw, yw);
      plane_at(fout + k * N, r) = static_cast<S>(rf);
      plane_at(gout + k * N, r) = static_cast<S>(rg);
    }
  });
}

// Relaxation-time factor alpha of the kinetic sensor eps = (1/V) sum_i
// |f_i - f_i^eq| / f_i^eq (eq. DeltaAvg).  The paper adds dissipation above
// eps = 0.01 without printing alpha; here alpha is 1 up to 0.01 and takes the
// levels 1.05, 1.35 and 2 from 0.01, 0.1 and 1 on, each reached by a linear
// ramp over the first tenth of its decade.  alpha is continuous, so a
// rounding-level change of eps changes tau by a rounding-level amount.
__device__ __forceinline__ double sensor_alpha(double eps) {
  if (!(eps > 1e-2)) return 1.0;
  if (eps <= 1.1e-2) return __builtin_fma(eps - 1e-2, 0.05 / 1e-3, 1.0);
  if (eps <= 1e-1) return 1.05;
  if (eps <= 1.1e-1) return __builtin_fma(eps - 1e-1, 0.30 / 1e-2, 1.05);
  if (eps <= 1.0) return 1.35;
  if (eps <= 1.1) return __builtin_fma(eps - 1.0, 0.65 / 0.1, 1.35);
  return 2.0;
}

// Wrapped source columns and row offsets of node (x, y) for a pull in
// lattice (ux, uy): link k's source is (x - cx - ux, y - cy - uy) and the
// offsets cx + ux, cy + uy take seven values each (cx, cy in [-3, 3]).
// Lattice tags read through a buffer resource: one descriptor and a 32-bit
// byte offset per load (plain loads of the tag array took a 64-bit address
// per lane and load).  Offsets stay below the n tags the descriptor covers.
struct TagReader {
  __amdgpu_buffer_rsrc_t r;
  __device__ __forceinline__ TagReader(const int* tags, long long n)
      : r(__builtin_amdgcn_make_buffer_rsrc(const_cast<int*>(tags), static_cast<short>(0),
                                            static_cast<int>(n * 4), 0x00020000)) {}
  __device__ __forceinline__ int operator()(unsigned idx) const {
    return static_cast<int>(
        __builtin_amdgcn_raw_buffer_load_b32(r, static_cast<int>(idx * 4u), 0, 0));
  }
};

struct PullMap {
  int col[7], row[7];
  __device__ __forceinline__ void build(int x, int y, int ux, int uy, const Grid& g) {
    static_for<0, 7>([&](auto ic) {
      constexpr int c = decltype(ic)::value - 3;
      col[c + 3] = wrapc(x - (c + ux), g.nx, g.fast_x);
      row[c + 3] = wrapc(y - (c + uy), g.ny, g.fast_y) * g.nx;
    });
  }
  template <int k>
  __device__ __forceinline__ unsigned source() const {
    return static_cast<unsigned>(row[plane_cy(k) + 3] + col[plane_cx(k) + 3]);
  }
};

// Lattice difference dU (receiver minus source) as a bit of the source's
// seen mask; -1 outside [-3, 3]^2 (such pairs are queued without the check:
// a duplicate pair writes the same values twice).
__device__ __forceinline__ int seen_bit(int dux, int duy) {
  return (dux >= -3 && dux <= 3 && duy >= -3 && duy <= 3) ? (dux + 3) * 7 + (duy + 3) : -1;
}

__device__ __forceinline__ unsigned long long pair_entry(unsigned s, int Lx, int Ly) {
  return static_cast<unsigned long long>(s) |
         (static_cast<unsigned long long>((Lx & 0xFF) | ((Ly & 0xFF) << 8)) << 32);
}

// For every set link k of receiver (x, y)'s pull mask (its lattice (Lx,
// Ly)): source s_k = (x, y) - c_k - (Lx, Ly); the pair (s_k, lattice) joins
// the queue unless the source's seen mask already holds the lattice.  tags:
// the step's input tags (the Un half of a source is the lattice it
// collided in).  Every lane of the wave calls this: one queue atomic per
// wave (a single counter takes every append, so appends are gathered);
// lanes with an empty mask only take part in the wave's prefix sum.
__device__ __forceinline__ void queue_pairs(const Carry& carry, const Grid& grid, const int* tags,
                                            int step, DevDiag* diag, int x, int y, int Lx,
                                            int Ly, unsigned mask) {
  PullMap pm;
  if (mask) pm.build(x, y, Lx, Ly, grid);
  // mark the lattice in each source's seen mask (returning atomics, all in
  // flight before the first result is used); fresh: the links whose pair
  // this receiver saw first
  unsigned long long old[kQ];
  int bit[kQ];
  static_for<0, kQ>([&](auto kc) {
    constexpr int k = decltype(kc)::value;
    bit[k] = -1;
    old[k] = 0ull;
    if ((mask >> k) & 1u) {
      const unsigned sidx = pm.template source<k>();
      const int t = tags[sidx];
      bit[k] = seen_bit(Lx - tag_unx(t), Ly - tag_uny(t));
      if (bit[k] >= 0) old[k] = atomicOr(&carry.seen[sidx], 1ull << bit[k]);
    }
  });
  unsigned fresh = 0u;
  static_for<0, kQ>([&](auto kc) {
    constexpr int k = decltype(kc)::value;
    if (((mask >> k) & 1u) && (bit[k] < 0 || !((old[k] >> bit[k]) & 1ull))) fresh |= 1u << k;
  });
  // wave prefix sum of the append counts, one atomic for the wave
  const int lane = threadIdx.x & 63;
  const unsigned cnt = static_cast<unsigned>(__popc(fresh));
  unsigned incl = cnt;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const unsigned t = __shfl_up(incl, d, 64);
    if (lane >= d) incl += t;
  }
  const unsigned total = __shfl(incl, 63, 64);
  if (total == 0u) return;
  unsigned base = 0u;
  if (lane == 0) base = atomicAdd(&carry.counters[2 + (step & 1)], total);
  long long i = static_cast<long long>(__shfl(base, 0, 64)) + (incl - cnt);
  static_for<0, kQ>([&](auto kc) {
    constexpr int k = decltype(kc)::value;
    if ((fresh >> k) & 1u) {
      const unsigned sidx = pm.template source<k>();
      if (i < carry.pair_cap)
        carry.pairs[i] = pair_entry(sidx, Lx, Ly);
      else
        record_failure(diag, step, sidx, kCodeQueueFull);
      ++i;
    }
  });
}

// ------------------------------------------------------------ fused step
// One node per lane; BLOCK lanes per workgroup.  The pulled populations are
// parked in LDS (plane-major, conflict-free) while the Newton solve holds
// the registers, then read back for the collision.  Links whose source
// collided in another lattice were rebuilt beforehand (rebuild_kernel) into
// the node's own slot of the output buffer and are read from there.  The
// tail prepares the next step: moments of this collision, the mask of the
// next pull's rebuilt links, and the list of nodes that have any.
template <typename S, bool STREAM, int BLOCK, int M, bool NBH = false, bool PR = false>
__device__ __forceinline__ void step_body(const StepArgs& a, int b) {
  __shared__ S sh_pop[2 * kQ][BLOCK];
  __shared__ unsigned long long sh_stat[2 + LBM_HIST_BINS];

  const int tid = threadIdx.x;
  const long long N = a.grid.N;
  const int nx = a.grid.nx;
  const long long n = static_cast<long long>(b) * BLOCK + tid;
  const bool active = n < N;
  const Phys& P = a.phys;
  // the wave issues its loads ahead of the SIMD's other wave, then yields
  __builtin_amdgcn_s_setprio(2);
  const S* fin = static_cast<const S*>(a.fin);
  const S* gin = static_cast<const S*>(a.gin);
  S* fout = static_cast<S*>(a.fout);
  S* gout = static_cast<S*>(a.gout);

  if (P.stats) {
    for (int i = tid; i < 2 + LBM_HIST_BINS; i += BLOCK) sh_stat[i] = 0ull;
    __syncthreads();
  }

  int x = 0, y = 0, tag = 0;
  unsigned mism = 0u;
  if (active) {
    y = static_cast<int>(n / nx);
    x = static_cast<int>(n - static_cast<long long>(y) * nx);
    tag = a.tin[n];
    if constexpr (STREAM) mism = a.carry.mask[n];
  }
  // Shifts used for addressing are clamped to the admissible range, so no
  // tag content can move a pull outside the grid.
  const int unx = min(max(tag_unx(tag), -P.max_abs_shift), P.max_abs_shift);
  const int uny = min(max(tag_uny(tag), -P.max_abs_shift), P.max_abs_shift);

  // a1 and a3: every link loaded (all loads in flight at once) from its
  // source, or from this node's slot of the output buffer where rebuilt;
  // parked in LDS; moments in the frame of the node's lattice (eq. polyTemp)
  double rho = 0.0, jx = 0.0, jy = 0.0, e = 0.0;
  PullMap pm;  // sources of this pull; the next pull reuses them unless the lattice changes
  int st[kQ];  // tags of the next pull's sources, loaded with this pull's populations
  const TagReader tag_at(a.tin, N);
  if (active) {
    S fv[kQ], gv[kQ];
    if constexpr (STREAM) {
      pm.build(x, y, unx, uny, a.grid);
      static_for<0, kQ>([&](auto kc) {
        constexpr int k = decltype(kc)::value;
        const unsigned i = pm.template source<k>();
        fv[k] = plane_at(fin + k * N, i);
        gv[k] = plane_at(gin + k * N, i);
      });
      if (P.shift_mode != 1) {
        static_for<0, kQ>([&](auto kc) {
          constexpr int k = decltype(kc)::value;
          st[k] = tag_at(pm.template source<k>());
        });
      }
      __builtin_amdgcn_s_setprio(0);
      // rebuilt links (rare: a wave-uniform test skips this for most waves)
      if (__ballot(mism != 0u)) {
        static_for<0, kQ>([&](auto kc) {
          constexpr int k = decltype(kc)::value;
          if ((mism >> k) & 1u) {
            fv[k] = plane_at(static_cast<const S*>(fout) + k * N, static_cast<unsigned>(n));
            gv[k] = plane_at(static_cast<const S*>(gout) + k * N, static_cast<unsigned>(n));
          }
        });
      }
    } else {
      static_for<0, kQ>([&](auto kc) {
        constexpr int k = decltype(kc)::value;
        fv[k] = plane_at(fin + k * N, static_cast<unsigned>(n));
        gv[k] = plane_at(gin + k * N, static_cast<unsigned>(n));
      });
    }
    static_for<0, kQ>([&](auto kc) {
      constexpr int k = decltype(kc)::value;
      constexpr int cx = plane_cx(k), cy = plane_cy(k);
      sh_pop[k][tid] = fv[k];
      sh_pop[kQ + k][tid] = gv[k];
      const double fd = static_cast<double>(fv[k]);
      rho += fd;
      jx = cmad<cx>(jx, fd);
      jy = cmad<cy>(jy, fd);
      e = cmad<cx * cx + cy * cy>(e, fd) + static_cast<double>(gv[k]);
    });
  }
  // the populations now live in LDS only; the solve gets the registers
  asm volatile("" ::: "memory");

  unsigned next_mask = 0u;
  if (active) {
    // exact divisions, as the oracle takes them, in both forms: at tau close
    // to 1/2 the flows carry small differences a long way (a reciprocal of
    // rho here together with solves stopped without their final correction
    // moved the FP32 form's 256^2 vortex by 1e-3 to 4e-3 after 1250 steps,
    // against 3e-5)
    const double upx = jx / rho, upy = jy / rho;
    const double T = (e - rho * (upx * upx + upy * upy)) / (2.0 * rho * P.Cv);
    unsigned code = 0;
    int nux = unx, nuy = uny;
    Weights w;
    int iters = 0;
    const bool physical = rho > 0.0 && T > 0.0 && rho < 1e300 && T < 1e300 &&
                          fabs(upx) < 1e300 && fabs(upy) < 1e300;
    // the guess table's cell, loaded now so that its latency is spent on
    // the lattice choice and the next-pull mask below (8-moment set)
    GuessFetch gf;
    double iT = 0.0;
    if constexpr (M == kM) {
      if (physical) {
        iT = rcp64(T);
        __builtin_amdgcn_s_setprio(2);
        gf = table_fetch(a.table, upx, upy, iT);
        __builtin_amdgcn_s_setprio(0);
      }
    }
    if (!physical) {
      code = kCodeNonphysical;
    } else if (NBH ? P.shift_mode == 3 : P.shift_mode == 0) {
      // a4: lattice of the next pull (the neighbourhood choice, shift mode 3,
      // is compiled into its own kernels: NBH)
      if constexpr (!NBH) {
        nux = select_axis(upx + unx, unx, P.halfwidth);
        nuy = select_axis(upy + uny, uny, P.halfwidth);
      } else {
        const int ny_ = a.grid.ny;
        int nb16[4];
        nb16[0] = tag_un16(a.tin[static_cast<long long>(y) * nx + wrapc(x + 1, nx, a.grid.fast_x)]);
        nb16[1] = tag_un16(a.tin[static_cast<long long>(y) * nx + wrapc(x - 1, nx, a.grid.fast_x)]);
        nb16[2] = tag_un16(a.tin[static_cast<long long>(wrapc(y + 1, ny_, a.grid.fast_y)) * nx + x]);
        nb16[3] = tag_un16(a.tin[static_cast<long long>(wrapc(y - 1, ny_, a.grid.fast_y)) * nx + x]);
        select_neighbourhood(upx + unx, upy + uny, unx, uny, nb16, P.halfwidth, nux, nuy);
      }
      if (abs(nux) > P.max_abs_shift || abs(nuy) > P.max_abs_shift) {
        code = kCodeNonphysical;
        nux = unx;  // keep every stored shift in range: later pulls stay in bounds
        nuy = uny;
      }
    }
    // links of the next pull whose source collides in another lattice this
    // step (the source's lattice of this step is the Un half of its tag)
    if (P.shift_mode != 1) {
      if (!STREAM || nux != unx || nuy != uny) {
        // the lattice changes (or nothing was pulled): other sources
        pm.build(x, y, nux, nuy, a.grid);
        static_for<0, kQ>([&](auto kc) {
          constexpr int k = decltype(kc)::value;
          st[k] = tag_at(pm.template source<k>());
        });
      }
      const int nun16 = (nux & 0xFF) | ((nuy & 0xFF) << 8);
      static_for<0, kQ>([&](auto kc) {
        constexpr int k = decltype(kc)::value;
        if (tag_un16(st[k]) != nun16) next_mask |= 1u << k;
      });
    }
    if (physical) {
      // a5: numerical equilibrium
      NewtonOut no;
      if constexpr (M == kM)
        no = solve_node(gf, iT, upx, upy, T, P, w, a.diag);
      else
        no = solve_node<M>(a.table, upx, upy, T, P, w, a.diag);
      iters = no.iters;
      if (!no.ok && !code) code = kCodeNewton;
    }
    if (P.stats) {
      atomicAdd(&sh_stat[0], 1ull);
      atomicAdd(&sh_stat[1], static_cast<unsigned long long>(iters));
      atomicAdd(&sh_stat[2 + (iters < LBM_HIST_BINS ? iters : LBM_HIST_BINS - 1)], 1ull);
    }
    if (code) {
      record_failure(a.diag, a.step, n, code);
      static_for<0, kQ>([&](auto kc) {
        constexpr int k = decltype(kc)::value;
        plane_at(fout + k * N, static_cast<unsigned>(n)) = sh_pop[k][tid];
        plane_at(gout + k * N, static_cast<unsigned>(n)) = sh_pop[kQ + k][tid];
      });
    } else {
      // a6: collision, eq. (coll), with g_eq = (2 Cv - D) T f_eq (eq. gEq)
      Weights fe;  // f_eq = rho w, shared by the sensor and the collision
      fe.w0 = rho * w.w0;
#pragma unroll
      for (int p = 0; p < kPairs; ++p) {
        fe.wp[p] = rho * w.wp[p];
        fe.wm[p] = rho * w.wm[p];
      }
      // FP32-storage form (BGK): f_eq rounded to FP32 once for the collision,
      // which runs in FP32 arithmetic (as it did before this array).  The sensor stays FP64 in both forms:
      // at tau close to 1/2 the viscosity it adds, (alpha tau - 1/2) T, is
      // sensitive to alpha (FP32 sums of eps moved the 256^2 vortex by 6e-4
      // after 1250 steps, against 3e-5 in FP64)
      constexpr bool k32 = std::is_same<S, float>::value && !PR;
      float fe32[k32 ? kQ : 1];
      if constexpr (k32) {
        static_for<0, kQ>([&](auto kc) {
          constexpr int k = decltype(kc)::value;
          fe32[k] = static_cast<float>(weight_of<k>(fe));
        });
      }
      double tau = 0.5 + P.nu / T;
      if (P.sensor) {
        double eps = 0.0;
        static_for<0, kQ>([&](auto kc) {
          constexpr int k = decltype(kc)::value;
          const double feq = weight_of<k>(fe);
          // one Newton-Raphson step on the hardware reciprocal: ~1e-14 relative
          const double r0 = __builtin_amdgcn_rcp(feq);
          const double ifeq = __builtin_fma(__builtin_fma(-feq, r0, 1.0), r0, r0);
          eps += fabs(static_cast<double>(sh_pop[k][tid]) - feq) * ifeq;
        });
        tau *= sensor_alpha(eps * (1.0 / kQ));
      }
      const double om = rcp64(tau);
      const double gfac = (2.0 * P.Cv - 2.0) * T;
      if constexpr (PR) {
        // flexible Prandtl number, eq. (Shakhov): heat flux of the pulled
        // populations, then BGK plus the projected term
        double qx = 0.0, qy = 0.0;
        static_for<0, kQ>([&](auto kc) {
          constexpr int k = decltype(kc)::value;
          const double cx = plane_cx(k) - upx, cy = plane_cy(k) - upy;
          const double e = (cx * cx + cy * cy) * static_cast<double>(sh_pop[k][tid]) +
                           static_cast<double>(sh_pop[kQ + k][tid]);
          qx = __builtin_fma(0.5 * cx, e, qx);
          qy = __builtin_fma(0.5 * cy, e, qy);
        });
        const ShakhovCoef sc =
            shakhov_coef([&](auto kc) { return weight_of<decltype(kc)::value>(w); }, rho, upx,
                         upy, T, qx, qy, P);
        const double tpr = 0.5 + (tau - 0.5) * P.inv_pr;
        const double ks = om - rcp64(tpr);
        static_for<0, kQ>([&](auto kc) {
          constexpr int k = decltype(kc)::value;
          const double feq = weight_of<k>(fe);
          const double geq = gfac * feq;
          double sf, sg;
          shakhov_phi<plane_cx(k), plane_cy(k)>(sc, sf, sg);
          const double fk = static_cast<double>(sh_pop[k][tid]);
          const double gk = static_cast<double>(sh_pop[kQ + k][tid]);
          plane_at(fout + k * N, static_cast<unsigned>(n)) =
              static_cast<S>(__builtin_fma(om, feq - fk, fk) + ks * feq * sf);
          plane_at(gout + k * N, static_cast<unsigned>(n)) =
              static_cast<S>(__builtin_fma(om, geq - gk, gk) + ks * geq * sg);
        });
      } else
      static_for<0, kQ>([&](auto kc) {
        constexpr int k = decltype(kc)::value;
        const S fk = sh_pop[k][tid], gk = sh_pop[kQ + k][tid];
        if constexpr (std::is_same<S, double>::value) {
          const double feq = weight_of<k>(fe);
          const double geq = gfac * feq;
          stream_store(fout + k * N, static_cast<unsigned>(n), __builtin_fma(om, feq - fk, fk));
          stream_store(gout + k * N, static_cast<unsigned>(n), __builtin_fma(om, geq - gk, gk));
        } else {
          // g_eq from the FP64 product, rounded once: a product of rounded
          // FP32 factors is biased the same way at every node of a state, and
          // that bias accumulates over the steps (it moved the 256^2 vortex
          // by 1e-3 after 1250 steps)
          const float omf = static_cast<float>(om);
          const float geq = static_cast<float>(gfac * weight_of<k>(fe));
          stream_store(fout + k * N, static_cast<unsigned>(n), __builtin_fmaf(omf, fe32[k] - fk, fk));
          stream_store(gout + k * N, static_cast<unsigned>(n), __builtin_fmaf(omf, geq - gk, gk));
        }
      });
    }
    a.tout[n] = tag_pack(unx, uny, nux, nuy);
    a.carry.mask[n] = next_mask;
    CarryT<S>* mac = static_cast<CarryT<S>*>(a.carry.mac);
    mac[n] = static_cast<CarryT<S>>(rho);
    mac[N + n] = static_cast<CarryT<S>>(upx);
    mac[2 * N + n] = static_cast<CarryT<S>>(upy);
    mac[3 * N + n] = static_cast<CarryT<S>>(T);
  }

  // nodes with rebuilt links next step go to the list (one atomic per wave)
  {
    const unsigned long long bal = __ballot(next_mask != 0u);
    if (bal) {
      const int lane = tid & 63;
      const int leader = __ffsll(static_cast<long long>(bal)) - 1;
      unsigned base = 0;
      if (lane == leader)
        base = atomicAdd(&a.carry.counters[a.step & 1], static_cast<unsigned>(__popcll(bal)));
      base = __shfl(base, leader, 64);
      if (next_mask)
        a.carry.list[base + __popcll(bal & ((1ull << lane) - 1ull))] = static_cast<int>(n);
    }
  }

  if (P.stats) {
    __syncthreads();
    if (tid < 2 + LBM_HIST_BINS && sh_stat[tid]) {
      unsigned long long* dst = tid == 0   ? &a.diag->newton_calls
                                : tid == 1 ? &a.diag->newton_iters
                                           : &a.diag->hist[tid - 2];
      atomicAdd(dst, sh_stat[tid]);
    }
  }
}

// TILED: each workgroup runs a.tiles consecutive tiles in a loop (the loop
// keeps kernel arguments live across the body, which costs spills); else
// one tile per workgroup.
template <typename S>
constexpr int kStepWaves =
    std::is_same<S, float>::value ? LBM_STEP_WAVES_PER_EU_F32 : LBM_STEP_WAVES_PER_EU;

template <typename S, bool STREAM, int BLOCK, bool TILED, int M = kM, bool NBH = false,
          bool PR = false>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(kStepWaves<S>)))
void step_kernel(StepArgs a) {
  const int g = a.remap ? xcd_remap(blockIdx.x, gridDim.x) : static_cast<int>(blockIdx.x);
  if constexpr (TILED) {
    for (int t = 0; t < a.tiles; ++t) {
      const int b = g * a.tiles + t;
      if (b >= a.ntiles) break;
      step_body<S, STREAM, BLOCK, M, NBH, PR>(a, b);
    }
  } else {
    step_body<S, STREAM, BLOCK, M, NBH, PR>(a, g);
  }
}

// ------------------------------------------------------------ rebuild
// a2 in two launches before a step.  queue: every receiver of the list the
// previous step wrote turns its marked links into (source, receiver
// lattice) pairs, each pair queued once; it also clears the other list
// counter for the coming step's appends.  rebuild: one lane per queued
// pair (rebuild_pair), grid-stride, clearing the other queue counter.
// Entry i of a receiver list of `count` (i past the end: an empty mask,
// the lane only joins the wave's ballots).
__device__ __forceinline__ void queue_entry(const Carry& carry, const Grid& grid, const int* tags,
                                            int step, DevDiag* diag, int max_shift, long long i,
                                            unsigned count) {
  int x = 0, y = 0, Lx = 0, Ly = 0;
  unsigned mask = 0u;
  if (i < count) {
    const int r = carry.list[i];
    mask = carry.mask[r];
    const int t = tags[r];
    Lx = min(max(tag_unx(t), -max_shift), max_shift);
    Ly = min(max(tag_uny(t), -max_shift), max_shift);
    y = r / grid.nx;
    x = r - y * grid.nx;
  }
  queue_pairs(carry, grid, tags, step, diag, x, y, Lx, Ly, mask);
}

__device__ __forceinline__ void queue_body(const RebuildArgs& a, long long i0, long long stride) {
  const unsigned count = a.carry.counters[(a.step - 1) & 1];
  if (blockIdx.x == 0 && threadIdx.x == 0) a.carry.counters[a.step & 1] = 0u;
  // whole waves go round the loop together (the queue uses wave ballots)
  const long long n = (static_cast<long long>(count) + 63) / 64 * 64;
  for (long long i = i0; i < n; i += stride)
    queue_entry(a.carry, a.grid, a.tags, a.step, a.diag, a.phys.max_abs_shift, i, count);
}

__global__ __launch_bounds__(kBlock) void queue_kernel(RebuildArgs a) {
  queue_body(a, static_cast<long long>(blockIdx.x) * kBlock + threadIdx.x,
             static_cast<long long>(gridDim.x) * kBlock);
}

template <typename S, int M, bool PR = false>
__device__ __forceinline__ void rebuild_body(const RebuildArgs& a) {
  const unsigned count = a.carry.counters[2 + (a.step & 1)];
  if (blockIdx.x == 0 && threadIdx.x == 0) a.carry.counters[2 + ((a.step + 1) & 1)] = 0u;
  const long long n = min(static_cast<long long>(count), a.carry.pair_cap);
  const long long stride = static_cast<long long>(gridDim.x) * kBlock;
  for (long long i = static_cast<long long>(blockIdx.x) * kBlock + threadIdx.x; i < n; i += stride)
    rebuild_pair<S, M, PR>(a, a.carry.pairs[i]);
}

template <typename S, int M = kM, bool PR = false>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(LBM_STEP_WAVES_PER_EU)))
void rebuild_kernel(RebuildArgs a) {
  rebuild_body<S, M, PR>(a);
}

// ------------------------------------------------------------ batched
// One context's share of a batched launch: many independent grids (uneven
// sizes, one storage type) advanced by one rebuild launch and one step
// launch per step.  Buffer parity and step index follow from the state at
// the batch start and the batch step s.
struct JobArgs {
  void* pop[2];  // f planes of population buffer 0 / 1; g planes follow 21 N values on
  int* tag[2];
  Carry carry;
  Grid grid;
  Phys phys;
  GuessTable table;
  DevDiag* diag;
  int cur;     // buffer holding the state at the batch start
  int step0;   // steps done at the batch start
  int nsteps;  // steps of this job in the batch
  int block0;  // first block of this job in a step launch (jobs in block order)
  int nblocks;
};

template <typename S>
__device__ __forceinline__ StepArgs job_step_args(const JobArgs& j, int s) {
  const int src = (j.cur + s) & 1, dst = src ^ 1;
  StepArgs a;
  a.fin = j.pop[src];
  a.gin = static_cast<const S*>(j.pop[src]) + kQ * j.grid.N;
  a.fout = j.pop[dst];
  a.gout = static_cast<S*>(j.pop[dst]) + kQ * j.grid.N;
  a.tin = j.tag[src];
  a.tout = j.tag[dst];
  a.carry = j.carry;
  a.grid = j.grid;
  a.phys = j.phys;
  a.table = j.table;
  a.step = j.step0 + s + 1;
  a.diag = j.diag;
  a.ntiles = j.nblocks;
  a.tiles = 1;
  a.remap = 0;
  return a;
}

// Step s of a batch: the grid covers every job's blocks; a block finds its
// job by binary search over the jobs' first blocks.
template <typename S, int BLOCK, int M = kM>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(LBM_STEP_WAVES_PER_EU)))
void step_batched_kernel(const JobArgs* jobs, int njobs, int s, int remap) {
  const int gb = remap ? xcd_remap(blockIdx.x, gridDim.x) : static_cast<int>(blockIdx.x);
  int lo = 0, hi = njobs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (jobs[mid].block0 <= gb) lo = mid;
    else hi = mid - 1;
  }
  const JobArgs& j = jobs[lo];
  if (s >= j.nsteps || gb - j.block0 >= j.nblocks) return;
  step_body<S, true, BLOCK, M>(job_step_args<S>(j, s), gb - j.block0);
}

// Failure words of every job of a batch, gathered for one copy to the host.
__global__ __launch_bounds__(kBlock) void gather_fail_keys_kernel(const JobArgs* jobs, int njobs,
                                                                 unsigned long long* out) {
  const int k = blockIdx.x * kBlock + threadIdx.x;
  if (k < njobs) out[k] = jobs[k].diag->fail_key;
}

constexpr int kMaxJobs = 1024;

// Exclusive prefix over a batch's jobs of count(job, step) for step s (0 for
// a job past its steps or on a fixed lattice), a block-wide scan in LDS:
// sh_first[k] for job k, sh_first[kMaxJobs] the total, which it returns.
// Every lane of the block calls it.
template <typename F>
__device__ __forceinline__ unsigned job_prefix(const JobArgs* jobs, int njobs, int s, F count,
                                               unsigned* sh_first, unsigned* sh_part) {
  const int tid = threadIdx.x;
  constexpr int kPer = kMaxJobs / kBlock;
  unsigned local[kPer], sum = 0;
#pragma unroll
  for (int q = 0; q < kPer; ++q) {
    const int k = tid * kPer + q;
    unsigned c = 0;
    if (k < njobs) {
      const JobArgs& j = jobs[k];
      if (s < j.nsteps && j.phys.shift_mode != 1) c = count(j, j.step0 + s + 1);
    }
    local[q] = c;
    sum += c;
  }
  sh_part[tid] = sum;
  __syncthreads();
  for (int d = 1; d < kBlock; d <<= 1) {
    const unsigned t = tid >= d ? sh_part[tid - d] : 0u;
    __syncthreads();
    sh_part[tid] += t;
    __syncthreads();
  }
  unsigned run = sh_part[tid] - sum;  // exclusive prefix of this thread's jobs
#pragma unroll
  for (int q = 0; q < kPer; ++q) {
    sh_first[tid * kPer + q] = run;
    run += local[q];
  }
  if (tid == kBlock - 1) sh_first[kMaxJobs] = sh_part[kBlock - 1];
  __syncthreads();
  return sh_first[kMaxJobs];
}

// Last job whose first item is <= g (jobs with no items are skipped: their
// first equals the next job's).
__device__ __forceinline__ int job_of(const unsigned* sh_first, int njobs, unsigned g) {
  int lo = 0, hi = njobs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (sh_first[mid] <= g) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// The queue pass of step s for every job of a batch: the jobs' receiver
// lists cut into waves of 64 entries, numbered job after job, grid-stride
// over the waves (a wave works on one job, as the pair appends need).
__global__ __launch_bounds__(kBlock) void queue_batched_kernel(const JobArgs* jobs, int njobs,
                                                               int s) {
  __shared__ unsigned sh_first[kMaxJobs + 1];  // first wave of each job
  __shared__ unsigned sh_part[kBlock];
  const unsigned total = job_prefix(
      jobs, njobs, s,
      [](const JobArgs& j, int step) {
        const unsigned c = j.carry.counters[(step - 1) & 1];
        if (blockIdx.x == 0) j.carry.counters[step & 1] = 0u;
        return (c + 63u) / 64u;
      },
      sh_first, sh_part);
  constexpr unsigned kWaves = kBlock / 64;
  const unsigned lane = threadIdx.x & 63;
  for (unsigned w = blockIdx.x * kWaves + threadIdx.x / 64; w < total; w += gridDim.x * kWaves) {
    const int jb = job_of(sh_first, njobs, w);
    const JobArgs& j = jobs[jb];
    const int step = j.step0 + s + 1;
    const int src = (j.cur + s) & 1;
    const unsigned count = j.carry.counters[(step - 1) & 1];
    const long long i = static_cast<long long>(w - sh_first[jb]) * 64 + lane;
    queue_entry(j.carry, j.grid, j.tag[src], step, j.diag, j.phys.max_abs_shift, i, count);
  }
}

// Rebuilds of step s for every job of a batch as one flat index space: the
// queued (source, lattice) pairs of every job, numbered job after job,
// grid-stride over the lanes; a lane finds its pair's job by binary search.
// Small jobs do not leave the grid idle while each job's queue is taken in
// turn.
template <typename S, int M = kM>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(LBM_STEP_WAVES_PER_EU)))
void rebuild_batched_kernel(const JobArgs* jobs, int njobs, int s) {
  __shared__ unsigned sh_first[kMaxJobs + 1];  // first global pair of each job
  __shared__ unsigned sh_part[kBlock];
  const unsigned total = job_prefix(
      jobs, njobs, s,
      [](const JobArgs& j, int step) {
        const unsigned c = static_cast<unsigned>(
            min(static_cast<long long>(j.carry.counters[2 + (step & 1)]), j.carry.pair_cap));
        if (blockIdx.x == 0) j.carry.counters[2 + ((step + 1) & 1)] = 0u;
        return c;
      },
      sh_first, sh_part);
  const unsigned lanes = gridDim.x * kBlock;
  for (unsigned g = blockIdx.x * kBlock + threadIdx.x; g < total; g += lanes) {
    const int lo = job_of(sh_first, njobs, g);
    const JobArgs& j = jobs[lo];
    const int src = (j.cur + s) & 1, dst = src ^ 1;
    RebuildArgs a;
    a.fout = j.pop[dst];
    a.gout = static_cast<S*>(j.pop[dst]) + kQ * j.grid.N;
    a.tags = j.tag[src];
    a.carry = j.carry;
    a.grid = j.grid;
    a.phys = j.phys;
    a.table = j.table;
    a.step = j.step0 + s + 1;
    a.diag = j.diag;
    rebuild_pair<S, M>(a, j.carry.pairs[g - sh_first[lo]]);
  }
}

// Default lanes per workgroup of the step kernel: one wave.  The LDS parking
// area is 42 x BLOCK values (10.5 KB FP32, 21 KB FP64 per wave); single-wave
// blocks let the LDS-bound FP64 form fit 7 waves per CU instead of 6.  The
// kernels are also built for 128 lanes, and for 256 in FP32 storage.
template <typename S>
constexpr int step_block() {
  return 64;
}

// Builds the initial-guess table: one lane per grid point, Maxwellian-start
// Newton in FP64, stores lambda_1..7 minus the lattice Maxwellian's.
__global__ __launch_bounds__(256) void table_kernel(float* out, int nu, int ns, float umax,
                                                    float smin, float smax, double tol,
                                                    int max_iter) {
  const int idx = blockIdx.x * 256 + threadIdx.x;
  if (idx >= nu * nu * ns) return;
  const int ia = idx % nu, ib = (idx / nu) % nu, is = idx / (nu * nu);
  const double a = umax * static_cast<double>(ia) / (nu - 1);
  const double b = umax * static_cast<double>(ib) / (nu - 1);
  const double s = smin + (smax - smin) * static_cast<double>(is) / (ns - 1);
  const double T = 1.0 / s;
  Weights w;
  double l[kM];
  const NewtonOut no = solve_robust(a, b, T, tol, max_iter, w, l);
  float* o = out + 8l * idx;
  if (!no.ok) {
    for (int k = 0; k < 8; ++k) o[k] = __builtin_nanf("");
    return;
  }
  o[0] = static_cast<float>(l[1] + a * s);  // lambda_1x - (-u_x / T)
  o[1] = static_cast<float>(l[2] + b * s);
  o[2] = static_cast<float>(l[3] - 0.5 * s);
  o[3] = static_cast<float>(l[4]);
  o[4] = static_cast<float>(l[5] - 0.5 * s);
  o[5] = static_cast<float>(l[6]);
  o[6] = static_cast<float>(l[7]);
  o[7] = 1.0f;
}

// The guess table of the four-constraint set: the same grid and records,
// first four floats l1x + a s, l1y + b s, l2 - s / 2, 1 (NaN where the
// globalised solve did not converge), the rest zero.
__global__ __launch_bounds__(256) void table4_kernel(float* out, int nu, int ns, float umax,
                                                     float smin, float smax, double tol,
                                                     int max_iter) {
  const int idx = blockIdx.x * 256 + threadIdx.x;
  if (idx >= nu * nu * ns) return;
  const int ia = idx % nu, ib = (idx / nu) % nu, is = idx / (nu * nu);
  const double a = umax * static_cast<double>(ia) / (nu - 1);
  const double b = umax * static_cast<double>(ib) / (nu - 1);
  const double s = smin + (smax - smin) * static_cast<double>(is) / (ns - 1);
  const double T = 1.0 / s;
  double m[kM4], l[kM4];
  targets4(a, b, T, m);
  Weights w;
  const NewtonOut no = solve_robust4(m, T, tol, max_iter, w, l);
  float* o = out + 8l * idx;
  for (int k = 0; k < 8; ++k) o[k] = 0.0f;
  if (!no.ok) {
    o[3] = __builtin_nanf("");
    return;
  }
  o[0] = static_cast<float>(l[1] + a * s);
  o[1] = static_cast<float>(l[2] + b * s);
  o[2] = static_cast<float>(l[3] - 0.5 * s);
  o[3] = 1.0f;
}

// ------------------------------------------------------------ init
// Grad initial condition: lattice from u (or fixed / static), equilibrium
// there, central differences of the input fields, h(0) = h_eq (1 + phi).
template <typename S, int M = kM>
__global__ __launch_bounds__(kBlock) void init_kernel(InitArgs a) {
  const long long n = static_cast<long long>(blockIdx.x) * kBlock + threadIdx.x;
  const long long N = a.grid.N;
  if (n >= N) return;
  const int nx = a.grid.nx, ny = a.grid.ny;
  const int y = static_cast<int>(n / nx), x = static_cast<int>(n - static_cast<long long>(y) * nx);
  const Phys& P = a.phys;
  const double rho = a.rho[n], ux = a.ux[n], uy = a.uy[n], T = a.T[n];
  int Ux, Uy;
  if (P.shift_mode == 1) {
    Ux = P.fixed_ux;
    Uy = P.fixed_uy;
  } else if (P.shift_mode == 2) {
    Ux = a.sux[n];
    Uy = a.suy[n];
  } else {
    Ux = (fabs(ux) < 1e9) ? static_cast<int>(ceil(ux - 0.5)) : 1 << 20;
    Uy = (fabs(uy) < 1e9) ? static_cast<int>(ceil(uy - 0.5)) : 1 << 20;
  }
  S* fo = static_cast<S*>(a.fout);
  S* go = static_cast<S*>(a.gout);
  unsigned code = 0;
  if (abs(Ux) > P.max_abs_shift || abs(Uy) > P.max_abs_shift || !(rho > 0.0) || !(T > 0.0) ||
      !(rho < 1e300) || !(T < 1e300))
    code = kCodeNonphysical;
  if (abs(Ux) > P.max_abs_shift || abs(Uy) > P.max_abs_shift) Ux = Uy = 0;  // stored tags stay in range
  a.tout[n] = tag_pack(Ux, Uy, Ux, Uy);
  Weights w;
  if (!code) {
    const NewtonOut no = solve_node<M>(a.table, ux - Ux, uy - Uy, T, P, w, a.diag);
    if (!no.ok) code = kCodeNewton;
  }
  if (code) {
    record_failure(a.diag, 0, n, code);
    for (int k = 0; k < kQ; ++k) {
      fo[k * N + n] = S(0);
      go[k * N + n] = S(0);
    }
    return;
  }
  const long long xp = (long long)y * nx + wrapc(x + 1, nx, a.grid.fast_x);
  const long long xm = (long long)y * nx + wrapc(x - 1, nx, a.grid.fast_x);
  const long long yp = (long long)wrapc(y + 1, ny, a.grid.fast_y) * nx + x;
  const long long ym = (long long)wrapc(y - 1, ny, a.grid.fast_y) * nx + x;
  const double du[4] = {0.5 * (a.ux[xp] - a.ux[xm]), 0.5 * (a.ux[yp] - a.ux[ym]),
                        0.5 * (a.uy[xp] - a.uy[xm]), 0.5 * (a.uy[yp] - a.uy[ym])};
  const double dT[2] = {0.5 * (a.T[xp] - a.T[xm]), 0.5 * (a.T[yp] - a.T[ym])};
  const GradState gs = grad_state(rho, ux, uy, T, du, dT, P);
  const double gfac = (2.0 * P.Cv - 2.0) * T;
  static_for<0, kQ>([&](auto kc) {
    constexpr int k = decltype(kc)::value;
    double phif, phig;
    grad_phi(gs, static_cast<double>(plane_cx(k) + Ux), static_cast<double>(plane_cy(k) + Uy), P,
             phif, phig);
    const double feq = rho * weight_of<k>(w);
    fo[k * N + n] = static_cast<S>(feq * (1.0 + phif));
    go[k * N + n] = static_cast<S>(gfac * feq * (1.0 + phig));
  });
}

// ------------------------------------------------------------ copy
// Streaming device copy: the practical HBM ceiling the step kernels are
// measured against.  Each lane moves kCopyUnroll 16-byte words per pass
// (all loads in flight before the first store), nontemporal so that the
// stream does not displace anything else from the caches; grid-stride.
constexpr int kCopyUnroll = 4;
typedef float CopyWord __attribute__((ext_vector_type(4)));  // 16 bytes

__global__ __launch_bounds__(kBlock) void stream_copy_kernel(const CopyWord* __restrict__ src,
                                                             CopyWord* __restrict__ dst,
                                                             long long words) {
  const long long stride = static_cast<long long>(gridDim.x) * kBlock * kCopyUnroll;
  for (long long base = static_cast<long long>(blockIdx.x) * kBlock * kCopyUnroll + threadIdx.x;
       base < words; base += stride) {
    CopyWord v[kCopyUnroll];
#pragma unroll
    for (int u = 0; u < kCopyUnroll; ++u) {
      const long long i = base + static_cast<long long>(u) * kBlock;
      if (i < words) v[u] = __builtin_nontemporal_load(src + i);
    }
#pragma unroll
    for (int u = 0; u < kCopyUnroll; ++u) {
      const long long i = base + static_cast<long long>(u) * kBlock;
      if (i < words) __builtin_nontemporal_store(v[u], dst + i);
    }
  }
}

__global__ __launch_bounds__(kBlock) void copy_tail_kernel(const unsigned char* src,
                                                           unsigned char* dst, long long n) {
  const long long i = static_cast<long long>(blockIdx.x) * kBlock + threadIdx.x;
  if (i < n) dst[i] = src[i];
}

// ------------------------------------------------------------ exports
template <typename S>
__global__ __launch_bounds__(kBlock) void macros_kernel(const S* f, const S* g, const int* tags,
                                                        long long N, double Cv, double* rho,
                                                        double* ux, double* uy, double* T,
                                                        int8_t* Ux, int8_t* Uy) {
  const long long n = static_cast<long long>(blockIdx.x) * kBlock + threadIdx.x;
  if (n >= N) return;
  double r, upx, upy, t;
  node_moments<S>(f, g, N, n, r, upx, upy, t, Cv);
  const int tg = tags[n];
  rho[n] = r;
  ux[n] = upx + tag_ucx(tg);
  uy[n] = upy + tag_ucy(tg);
  T[n] = t;
  if (Ux) Ux[n] = static_cast<int8_t>(tag_ucx(tg));
  if (Uy) Uy[n] = static_cast<int8_t>(tag_ucy(tg));
}

template <typename S>
__global__ __launch_bounds__(kBlock) void widen_kernel(const S* src, double* dst, long long count) {
  const long long i = static_cast<long long>(blockIdx.x) * kBlock + threadIdx.x;
  if (i < count) dst[i] = static_cast<double>(src[i]);
}

// Per-block sums of mass, momentum (absolute velocities c = xi + Uc) and
// total energy (1/2) sum (|c|^2 f + g); reduced in a fixed order.
template <typename S>
__global__ __launch_bounds__(kBlock) void conserved_kernel(const S* f, const S* g,
                                                           const int* tags, long long N,
                                                           double* partials) {
  __shared__ double sh[4][kBlock];
  const int tid = threadIdx.x;
  const long long n = static_cast<long long>(blockIdx.x) * kBlock + tid;
  double m = 0.0, px = 0.0, py = 0.0, en = 0.0;
  if (n < N) {
    const int tg = tags[n];
    const int ucx = tag_ucx(tg), ucy = tag_ucy(tg);
    static_for<0, kQ>([&](auto kc) {
      constexpr int k = decltype(kc)::value;
      const double fk = static_cast<double>(f[k * N + n]);
      const double gk = static_cast<double>(g[k * N + n]);
      const double cx = plane_cx(k) + ucx, cy = plane_cy(k) + ucy;
      m += fk;
      px += fk * cx;
      py += fk * cy;
      en += 0.5 * ((cx * cx + cy * cy) * fk + gk);
    });
  }
  sh[0][tid] = m;
  sh[1][tid] = px;
  sh[2][tid] = py;
  sh[3][tid] = en;
  __syncthreads();
  for (int s = kBlock / 2; s > 0; s >>= 1) {
    if (tid < s)
      for (int c = 0; c < 4; ++c) sh[c][tid] += sh[c][tid + s];
    __syncthreads();
  }
  if (tid < 4) partials[4ll * blockIdx.x + tid] = sh[tid][0];
}

__global__ __launch_bounds__(kBlock) void reduce_partials_kernel(const double* partials,
                                                                 int nparts, double* out) {
  __shared__ double sh[4][kBlock];
  const int tid = threadIdx.x;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int b = tid; b < nparts; b += kBlock)
    for (int c = 0; c < 4; ++c) acc[c] += partials[4ll * b + c];
  for (int c = 0; c < 4; ++c) sh[c][tid] = acc[c];
  __syncthreads();
  for (int s = kBlock / 2; s > 0; s >>= 1) {
    if (tid < s)
      for (int c = 0; c < 4; ++c) sh[c][tid] += sh[c][tid + s];
    __syncthreads();
  }
  if (tid < 4) out[tid] = sh[tid][0];
}

}  // namespace lbm
