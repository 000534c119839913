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
#include "lattice.hpp"

#ifndef LBM_HIST_BINS
#define LBM_HIST_BINS 32
#endif
// Waves per SIMD the step kernel is compiled for (caps its registers).
#ifndef LBM_STEP_WAVES_PER_EU
#define LBM_STEP_WAVES_PER_EU 2
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
};

enum : unsigned { kCodeNewton = 1, kCodeNonphysical = 2 };

struct Phys {
  double nu, Cv, Cp, halfwidth, tol;
  int max_iter, shift_mode, fixed_ux, fixed_uy, max_abs_shift, sensor, stats;
};

struct Grid {
  long long N;
  int nx, ny;
  int fast_x, fast_y;  // wrap by one conditional add/sub (grid wider than any reach)
};

struct StepArgs {
  const void* fin;
  const void* gin;
  void* fout;
  void* gout;
  const int* tin;
  int* tout;
  Grid grid;
  Phys phys;
  GuessTable table;
  int step;
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
template <int K, int N, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (K < N) {
    f(std::integral_constant<int, K>{});
    static_for<K + 1, N>(f);
  }
}

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

// Consecutive blocks are dispatched round-robin over the 8 XCDs; remap so
// that each XCD (own L2) works on one contiguous range of nodes.
__device__ __forceinline__ int xcd_remap(int b, int G) {
  const int q = G >> 3, r = G & 7, xcd = b & 7, idx = b >> 3;
  return xcd < r ? xcd * (q + 1) + idx : r * (q + 1) + (xcd - r) * q + idx;
}

__device__ __forceinline__ void record_failure(DevDiag* d, int step, long long node,
                                               unsigned code) {
  const unsigned long long key = (static_cast<unsigned long long>(step) << 34) |
                                 (static_cast<unsigned long long>(node) << 3) | code;
  atomicMin(&d->fail_key, key);
}

// Eq. (criterion) with optional hysteresis half-width hw >= 1/2.
__device__ __forceinline__ int select_axis(double u, int uprev, double hw) {
  if (u > uprev - hw && u <= uprev + hw) return uprev;
  return static_cast<int>(ceil(u - 0.5));
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
  const double kappa = rho * P.Cp * P.nu;  // unit Prandtl number
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

// Absolute macroscopic velocity and temperature of node s.
template <typename S>
__device__ __forceinline__ void node_uT(const S* f, const S* g, const int* tags, long long N,
                                        long long s, double Cv, double& ux, double& uy,
                                        double& T) {
  double rho, upx, upy;
  node_moments<S>(f, g, N, s, rho, upx, upy, T, Cv);
  const int t = tags[s];
  ux = upx + tag_ucx(t);
  uy = upy + tag_ucy(t);
}

// Post-collision population of velocity plane k in lattice (Lx, Ly) at
// source node s, rebuilt by Grad's ansatz from the moments and central
// gradients at s (eq. GradGeneral with h* = h_eq + (1 - 1/tau) h_neq).
template <typename S>
__device__ __forceinline__ unsigned rebuild_link(const StepArgs& a, int s, int Lx, int Ly, int k,
                                              double& rf, double& rg, int& iters) {
  const S* f = static_cast<const S*>(a.fin);
  const S* g = static_cast<const S*>(a.gin);
  const long long N = a.grid.N;
  const int nx = a.grid.nx, ny = a.grid.ny;
  const Phys& P = a.phys;
  double rho, upx, upy, T;
  node_moments<S>(f, g, N, s, rho, upx, upy, T, P.Cv);
  const int ts = a.tin[s];
  const double ux = upx + tag_ucx(ts), uy = upy + tag_ucy(ts);
  rf = 0.0;
  rg = 0.0;
  iters = 0;
  if (!(rho > 0.0) || !(T > 0.0) || !(rho < 1e300) || !(T < 1e300)) return kCodeNonphysical;
  double du[4] = {0.0, 0.0, 0.0, 0.0}, dT[2] = {0.0, 0.0};
  if (P.nu > 0.0) {
    const int ys = s / nx, xs = s - ys * nx;
    const long long xp = (long long)ys * nx + wrapc(xs + 1, nx, a.grid.fast_x);
    const long long xm = (long long)ys * nx + wrapc(xs - 1, nx, a.grid.fast_x);
    const long long yp = (long long)wrapc(ys + 1, ny, a.grid.fast_y) * nx + xs;
    const long long ym = (long long)wrapc(ys - 1, ny, a.grid.fast_y) * nx + xs;
    double uxp, uyp, Tp, uxm, uym, Tm;
    node_uT<S>(f, g, a.tin, N, xp, P.Cv, uxp, uyp, Tp);
    node_uT<S>(f, g, a.tin, N, xm, P.Cv, uxm, uym, Tm);
    du[0] = 0.5 * (uxp - uxm);
    du[2] = 0.5 * (uyp - uym);
    dT[0] = 0.5 * (Tp - Tm);
    node_uT<S>(f, g, a.tin, N, yp, P.Cv, uxp, uyp, Tp);
    node_uT<S>(f, g, a.tin, N, ym, P.Cv, uxm, uym, Tm);
    du[1] = 0.5 * (uxp - uxm);
    du[3] = 0.5 * (uyp - uym);
    dT[1] = 0.5 * (Tp - Tm);
  }
  Weights w;
  const NewtonOut no = solve_fast(a.table, ux - Lx, uy - Ly, T, P.tol, P.max_iter, w);
  iters = no.iters;
  if (!no.ok) return kCodeNewton;
  double wk = 0.0, cxk = 0.0, cyk = 0.0;
  static_for<0, kQ>([&](auto kc) {
    constexpr int kk = decltype(kc)::value;
    if (k == kk) {
      wk = weight_of<kk>(w);
      cxk = plane_cx(kk);
      cyk = plane_cy(kk);
    }
  });
  const GradState gs = grad_state(rho, ux, uy, T, du, dT, P);
  double phif, phig;
  grad_phi(gs, cxk + Lx, cyk + Ly, P, phif, phig);
  const double tau = 0.5 + P.nu / T;
  const double kf = 1.0 - 1.0 / tau;
  const double feq = rho * wk;
  const double geq = (2.0 * P.Cv - 2.0) * T * feq;
  rf = feq * (1.0 + kf * phif);
  rg = geq * (1.0 + kf * phig);
  return 0;
}

// Kinetic sensor eps = (1/V) sum_i |f_i - f_i^eq| / f_i^eq and the relaxation
// time factor alpha(eps) (eq. DeltaAvg; alpha is not printed in the paper:
// piecewise constant 1 / 1.05 / 1.35 / 2 with breaks at 1e-2, 1e-1, 1).
__device__ __forceinline__ double sensor_alpha(double eps) {
  return eps < 1e-2 ? 1.0 : (eps < 1e-1 ? 1.05 : (eps < 1.0 ? 1.35 : 2.0));
}

// ------------------------------------------------------------ fused step
// One node per lane; BLOCK lanes per workgroup.  The pulled populations are
// parked in LDS (plane-major, conflict-free) while the Newton solve holds
// the registers, then read back for the collision.
template <typename S, bool STREAM, int BLOCK>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(LBM_STEP_WAVES_PER_EU)))
void step_kernel(StepArgs a) {
  constexpr int WAVES = BLOCK / 64;
  __shared__ S sh_pop[2 * kQ][BLOCK];
  __shared__ int sh_cnt[WAVES];
  __shared__ int sh_src[BLOCK];
  __shared__ int sh_meta[BLOCK];
  __shared__ double sh_rf[BLOCK];
  __shared__ double sh_rg[BLOCK];
  __shared__ unsigned long long sh_stat[3 + LBM_HIST_BINS];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int b = xcd_remap(blockIdx.x, gridDim.x);
  const long long N = a.grid.N;
  const int nx = a.grid.nx, ny = a.grid.ny;
  const long long n = static_cast<long long>(b) * BLOCK + tid;
  const bool active = n < N;
  const Phys& P = a.phys;
  const S* fin = static_cast<const S*>(a.fin);
  const S* gin = static_cast<const S*>(a.gin);

  if (P.stats) {
    for (int i = tid; i < 3 + LBM_HIST_BINS; i += BLOCK) sh_stat[i] = 0ull;
    __syncthreads();
  }

  int x = 0, y = 0, tag = 0;
  if (active) {
    y = static_cast<int>(n / nx);
    x = static_cast<int>(n - static_cast<long long>(y) * nx);
    tag = a.tin[n];
  }
  // Shifts used for addressing are clamped to the admissible range, so no
  // tag content can move a pull outside the grid.
  const int unx = min(max(tag_unx(tag), -P.max_abs_shift), P.max_abs_shift);
  const int uny = min(max(tag_uny(tag), -P.max_abs_shift), P.max_abs_shift);
  const int un16 = tag_un16(tag);

  // Source node of link k is (x - cx - Ux, y - cy - Uy): with cx, cy in
  // [-3, 3] the wrapped columns and row offsets take seven values each.
  int col[7], row[7];
  if constexpr (STREAM) {
    static_for<0, 7>([&](auto ic) {
      constexpr int c = decltype(ic)::value - 3;
      col[c + 3] = wrapc(x - (c + unx), nx, a.grid.fast_x);
      row[c + 3] = wrapc(y - (c + uny), ny, a.grid.fast_y) * nx;
    });
  }
  auto source = [&](auto kc) -> unsigned {
    constexpr int k = decltype(kc)::value;
    if constexpr (STREAM)
      return static_cast<unsigned>(row[plane_cy(k) + 3] + col[plane_cx(k) + 3]);
    else
      return static_cast<unsigned>(n);
  };

  // a1 (first half): which links have their source in another lattice
  unsigned mism = 0u;
  if constexpr (STREAM) {
    if (active) {
      int st[kQ];
      static_for<0, kQ>([&](auto kc) {
        constexpr int k = decltype(kc)::value;
        st[k] = plane_at(a.tin, source(kc));
      });
      static_for<0, kQ>([&](auto kc) {
        constexpr int k = decltype(kc)::value;
        if (tag_uc16(st[k]) != un16) mism |= 1u << k;
      });
    }

    // a2: those links are rebuilt by Grad's ansatz.  The block's
    // (lane, link) items are packed and handed out one per lane, so a block
    // pays ceil(items / BLOCK) rebuild rounds instead of one per distinct
    // link; results go straight to the owner's LDS slots.
    const int cnt = __popc(mism);
    int v = cnt;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const int t = __shfl_up(v, d, 64);
      if (lane >= d) v += t;
    }
    if (lane == 63) sh_cnt[wave] = v;
    __syncthreads();
    int total = 0, wbase = 0;
#pragma unroll
    for (int w = 0; w < WAVES; ++w) {
      const int c = sh_cnt[w];
      wbase += (w < wave) ? c : 0;
      total += c;
    }
    const int off = wbase + v - cnt;
    for (int r0 = 0; r0 < total; r0 += BLOCK) {
      const bool mine = cnt > 0 && off < r0 + BLOCK && off + cnt > r0;
      if (mine) {
        int j = off;
        static_for<0, kQ>([&](auto kc) {
          constexpr int k = decltype(kc)::value;
          if (mism & (1u << k)) {
            if (j >= r0 && j < r0 + BLOCK) {
              sh_src[j - r0] = static_cast<int>(source(kc));
              sh_meta[j - r0] = k | ((unx & 0xFF) << 8) | ((uny & 0xFF) << 16);
            }
            ++j;
          }
        });
      }
      __syncthreads();
      if (r0 + tid < total) {
        const int meta = sh_meta[tid];
        double rf, rg;
        int it;
        const unsigned code =
            rebuild_link<S>(a, sh_src[tid], static_cast<int8_t>((meta >> 8) & 0xFF),
                            static_cast<int8_t>((meta >> 16) & 0xFF), meta & 0xFF, rf, rg, it);
        if (code) record_failure(a.diag, a.step, sh_src[tid], code);
        sh_rf[tid] = rf;
        sh_rg[tid] = rg;
        if (P.stats) {
          atomicAdd(&sh_stat[0], 1ull);
          atomicAdd(&sh_stat[1], static_cast<unsigned long long>(it));
          atomicAdd(&sh_stat[3 + (it < LBM_HIST_BINS ? it : LBM_HIST_BINS - 1)], 1ull);
        }
      }
      __syncthreads();
      if (mine) {
        int j = off;
        static_for<0, kQ>([&](auto kc) {
          constexpr int k = decltype(kc)::value;
          if (mism & (1u << k)) {
            if (j >= r0 && j < r0 + BLOCK) {
              sh_pop[k][tid] = static_cast<S>(sh_rf[j - r0]);
              sh_pop[kQ + k][tid] = static_cast<S>(sh_rg[j - r0]);
            }
            ++j;
          }
        });
      }
      __syncthreads();
    }
    if (P.stats && cnt) atomicAdd(&sh_stat[2], static_cast<unsigned long long>(cnt));
  }

  // a1 (second half) and a3: every link is loaded (all loads in flight at
  // once), rebuilt links then replace theirs from LDS by a select; the
  // merged populations are parked in LDS and their moments taken in the
  // frame of the node's lattice (eq. polyTemp)
  double rho = 0.0, jx = 0.0, jy = 0.0, e = 0.0;
  if (active) {
    S fv[kQ], gv[kQ];
    static_for<0, kQ>([&](auto kc) {
      constexpr int k = decltype(kc)::value;
      const unsigned s = source(kc);
      fv[k] = plane_at(fin + k * N, s);
      gv[k] = plane_at(gin + k * N, s);
    });
    static_for<0, kQ>([&](auto kc) {
      constexpr int k = decltype(kc)::value;
      constexpr int cx = plane_cx(k), cy = plane_cy(k);
      S fk = fv[k], gk = gv[k];
      if constexpr (STREAM) {
        const bool m = (mism >> k) & 1u;
        const S rf = sh_pop[k][tid], rg = sh_pop[kQ + k][tid];
        fk = m ? rf : fk;
        gk = m ? rg : gk;
      }
      sh_pop[k][tid] = fk;
      sh_pop[kQ + k][tid] = gk;
      const double fd = static_cast<double>(fk);
      rho += fd;
      jx = cmad<cx>(jx, fd);
      jy = cmad<cy>(jy, fd);
      e = cmad<cx * cx + cy * cy>(e, fd) + static_cast<double>(gk);
    });
  }
  // the populations now live in LDS only; the solve gets the registers
  asm volatile("" ::: "memory");

  if (active) {
    const double upx = jx / rho, upy = jy / rho;
    const double T = (e - rho * (upx * upx + upy * upy)) / (2.0 * rho * P.Cv);
    unsigned code = 0;
    int nux = unx, nuy = uny;
    Weights w;
    int iters = 0;
    if (!(rho > 0.0) || !(T > 0.0) || !(rho < 1e300) || !(T < 1e300) || !(fabs(upx) < 1e300) ||
        !(fabs(upy) < 1e300)) {
      code = kCodeNonphysical;
    } else {
      // a4: lattice of the next pull
      if (P.shift_mode == 0) {
        nux = select_axis(upx + unx, unx, P.halfwidth);
        nuy = select_axis(upy + uny, uny, P.halfwidth);
        if (abs(nux) > P.max_abs_shift || abs(nuy) > P.max_abs_shift) {
          code = kCodeNonphysical;
          nux = unx;  // keep every stored shift in range: later pulls stay in bounds
          nuy = uny;
        }
      }
      // a5: numerical equilibrium
      const NewtonOut no = solve_fast(a.table, upx, upy, T, P.tol, P.max_iter, w);
      iters = no.iters;
      if (!no.ok && !code) code = kCodeNewton;
    }
    if (P.stats) {
      atomicAdd(&sh_stat[0], 1ull);
      atomicAdd(&sh_stat[1], static_cast<unsigned long long>(iters));
      atomicAdd(&sh_stat[3 + (iters < LBM_HIST_BINS ? iters : LBM_HIST_BINS - 1)], 1ull);
    }
    S* fout = static_cast<S*>(a.fout);
    S* gout = static_cast<S*>(a.gout);
    if (code) {
      record_failure(a.diag, a.step, n, code);
      static_for<0, kQ>([&](auto kc) {
        constexpr int k = decltype(kc)::value;
        plane_at(fout + k * N, static_cast<unsigned>(n)) = sh_pop[k][tid];
        plane_at(gout + k * N, static_cast<unsigned>(n)) = sh_pop[kQ + k][tid];
      });
    } else {
      // a6: collision, eq. (coll), with g_eq = (2 Cv - D) T f_eq (eq. gEq)
      double tau = 0.5 + P.nu / T;
      if (P.sensor) {
        double eps = 0.0;
        static_for<0, kQ>([&](auto kc) {
          constexpr int k = decltype(kc)::value;
          const double feq = rho * weight_of<k>(w);
          // one Newton-Raphson step on the hardware reciprocal: ~1e-14 relative
          const double r0 = __builtin_amdgcn_rcp(feq);
          const double ifeq = __builtin_fma(__builtin_fma(-feq, r0, 1.0), r0, r0);
          eps += fabs(static_cast<double>(sh_pop[k][tid]) - feq) * ifeq;
        });
        tau *= sensor_alpha(eps * (1.0 / kQ));
      }
      const double om = rcp64(tau);
      const double gfac = (2.0 * P.Cv - 2.0) * T;
      static_for<0, kQ>([&](auto kc) {
        constexpr int k = decltype(kc)::value;
        const double feq = rho * weight_of<k>(w);
        const double geq = gfac * feq;
        const S fk = sh_pop[k][tid], gk = sh_pop[kQ + k][tid];
        if constexpr (std::is_same<S, double>::value) {
          plane_at(fout + k * N, static_cast<unsigned>(n)) = __builtin_fma(om, feq - fk, fk);
          plane_at(gout + k * N, static_cast<unsigned>(n)) = __builtin_fma(om, geq - gk, gk);
        } else {
          const float omf = static_cast<float>(om);
          plane_at(fout + k * N, static_cast<unsigned>(n)) = __builtin_fmaf(omf, static_cast<float>(feq) - fk, fk);
          plane_at(gout + k * N, static_cast<unsigned>(n)) = __builtin_fmaf(omf, static_cast<float>(geq) - gk, gk);
        }
      });
    }
    a.tout[n] = tag_pack(unx, uny, nux, nuy);
  }

  if (P.stats) {
    __syncthreads();
    if (tid < 3 + LBM_HIST_BINS && sh_stat[tid]) {
      unsigned long long* dst = tid == 0   ? &a.diag->newton_calls
                                : tid == 1 ? &a.diag->newton_iters
                                : tid == 2 ? &a.diag->mismatched
                                           : &a.diag->hist[tid - 3];
      atomicAdd(dst, sh_stat[tid]);
    }
  }
}

// Population storage type -> lanes per workgroup of the step kernel (the
// LDS parking area is 42 x BLOCK values: 43 KB either way).
template <typename S>
constexpr int step_block() {
  return std::is_same<S, double>::value ? 128 : 256;
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

// ------------------------------------------------------------ init
// Grad initial condition: lattice from u (or fixed / static), equilibrium
// there, central differences of the input fields, h(0) = h_eq (1 + phi).
template <typename S>
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
    const NewtonOut no = solve_fast(a.table, ux - Ux, uy - Uy, T, P.tol, P.max_iter, w);
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
