// Kernels of the paper's reference model on the same adaptive framework:
// D2Q49 with the 13-constraint equilibrium (App. C), FP64 storage.  The
// step is the one of the D2Q21 model (Sec. IV.A.4: pull with Grad rebuild
// of links whose source collided in another lattice, moments, lattice
// selection, equilibrium, BGK), over 2 x 49 planes:
//
//   step49_kernel<STREAM, PR>  (PR: flexible-Prandtl collision)
//                          one node per lane, 64 lanes per workgroup; the
//                          98 pulled populations are parked in LDS (50 KB)
//                          while the 13 x 13 Newton solve (from the guess
//                          table of table13_kernel) holds the
//                          registers; weights are recomputed per plane from
//                          the multipliers for the collision
//   rebuild49_kernel       the links of the next pull whose source collided
//                          in another lattice (64-bit link masks)
//   init49_kernel          Grad initial condition h(0) = h_eq (1 + phi)
//   macros49_kernel, conserved49_kernel
//
// The carried arrays, tags, lists and diagnostics are those of the D2Q21
// kernels; the per-node link mask is 64 bits wide here.
#pragma once

#include "equilibrium13.hpp"
#include "kernels.hpp"

namespace lbm {

constexpr int kBlock49 = 64;

struct Lattice49 {
  static constexpr int Q = kQ49;
  static constexpr int cx(int k) { return cx49(k); }
  static constexpr int cy(int k) { return cy49(k); }
};

// Wrapped source of plane K for a pull in lattice (ux, uy) at (x, y).
struct PullMap49 {
  int col[7], row[7];
  __device__ __forceinline__ void build(int x, int y, int ux, int uy, const Grid& g) {
    static_for<0, 7>([&](auto ic) {
      constexpr int c = decltype(ic)::value - 3;
      col[c + 3] = wrapc(x - (c + ux), g.nx, g.fast_x);
      row[c + 3] = wrapc(y - (c + uy), g.ny, g.fast_y) * g.nx;
    });
  }
  template <int K>
  __device__ __forceinline__ unsigned source() const {
    return static_cast<unsigned>(row[cy49(K) + 3] + col[cx49(K) + 3]);
  }
};

__device__ __forceinline__ unsigned long long* mask64(const Carry& c) {
  return reinterpret_cast<unsigned long long*>(c.mask);
}

// PR: the flexible-Prandtl collision (eq. Shakhov) in place of BGK.
template <bool STREAM, bool PR = false>
__global__ __launch_bounds__(kBlock49) void step49_kernel(StepArgs a) {
  __shared__ double sh_pop[2 * kQ49][kBlock49];
  __shared__ unsigned long long sh_stat[2 + LBM_HIST_BINS];
  const int tid = threadIdx.x;
  const int b = a.remap ? xcd_remap(blockIdx.x, gridDim.x) : static_cast<int>(blockIdx.x);
  const long long N = a.grid.N;
  const int nx = a.grid.nx;
  const long long n = static_cast<long long>(b) * kBlock49 + tid;
  const bool active = n < N;
  const Phys& P = a.phys;
  const double* fin = static_cast<const double*>(a.fin);
  const double* gin = static_cast<const double*>(a.gin);
  double* fout = static_cast<double*>(a.fout);
  double* gout = static_cast<double*>(a.gout);
  unsigned long long* mask = mask64(a.carry);

  if (P.stats) {
    for (int i = tid; i < 2 + LBM_HIST_BINS; i += kBlock49) sh_stat[i] = 0ull;
    __syncthreads();
  }

  int x = 0, y = 0, tag = 0;
  unsigned long long mism = 0ull;
  if (active) {
    y = static_cast<int>(n / nx);
    x = static_cast<int>(n - static_cast<long long>(y) * nx);
    tag = a.tin[n];
    if constexpr (STREAM) mism = mask[n];
  }
  const int unx = min(max(tag_unx(tag), -P.max_abs_shift), P.max_abs_shift);
  const int uny = min(max(tag_uny(tag), -P.max_abs_shift), P.max_abs_shift);

  // pull (or the rebuilt value in this node's slot), park, moments
  double rho = 0.0, jx = 0.0, jy = 0.0, e = 0.0;
  if (active) {
    PullMap49 pm;
    if constexpr (STREAM) pm.build(x, y, unx, uny, a.grid);
    static_for<0, kQ49>([&](auto kc) {
      constexpr int k = decltype(kc)::value;
      constexpr int cx = cx49(k), cy = cy49(k);
      double fk, gk;
      if constexpr (STREAM) {
        const bool rebuilt = (mism >> k) & 1ull;
        const unsigned i = rebuilt ? static_cast<unsigned>(n) : pm.template source<k>();
        fk = plane_at(rebuilt ? static_cast<const double*>(fout) + k * N : fin + k * N, i);
        gk = plane_at(rebuilt ? static_cast<const double*>(gout) + k * N : gin + k * N, i);
      } else {
        fk = plane_at(fin + k * N, static_cast<unsigned>(n));
        gk = plane_at(gin + k * N, static_cast<unsigned>(n));
      }
      sh_pop[k][tid] = fk;
      sh_pop[kQ49 + k][tid] = gk;
      rho += fk;
      jx = cmad<cx>(jx, fk);
      jy = cmad<cy>(jy, fk);
      e = cmad<cx * cx + cy * cy>(e, fk) + gk;
    });
  }
  asm volatile("" ::: "memory");

  unsigned long long next_mask = 0ull;
  if (active) {
    const double upx = jx / rho, upy = jy / rho;
    const double T = (e - rho * (upx * upx + upy * upy)) / (2.0 * rho * P.Cv);
    unsigned code = 0;
    int nux = unx, nuy = uny;
    int iters = 0;
    double l[kM13];
    const bool physical = rho > 0.0 && T > 0.0 && rho < 1e300 && T < 1e300 &&
                          fabs(upx) < 1e300 && fabs(upy) < 1e300;
    if (!physical) {
      code = kCodeNonphysical;
    } else if (P.shift_mode == 0) {
      nux = select_axis(upx + unx, unx, P.halfwidth);
      nuy = select_axis(upy + uny, uny, P.halfwidth);
      if (abs(nux) > P.max_abs_shift || abs(nuy) > P.max_abs_shift) {
        code = kCodeNonphysical;
        nux = unx;
        nuy = uny;
      }
    }
    if (P.shift_mode != 1) {
      PullMap49 pm;
      pm.build(x, y, nux, nuy, a.grid);
      const int nun16 = (nux & 0xFF) | ((nuy & 0xFF) << 8);
      static_for<0, kQ49>([&](auto kc) {
        constexpr int k = decltype(kc)::value;
        if (tag_un16(plane_at(a.tin, pm.template source<k>())) != nun16)
          next_mask |= 1ull << k;
      });
    }
    if (physical) {
      const NewtonOut no = solve_equilibrium13(a.table, upx, upy, T, P.tol, P.max_iter, l);
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
      static_for<0, kQ49>([&](auto kc) {
        constexpr int k = decltype(kc)::value;
        plane_at(fout + k * N, static_cast<unsigned>(n)) = sh_pop[k][tid];
        plane_at(gout + k * N, static_cast<unsigned>(n)) = sh_pop[kQ49 + k][tid];
      });
    } else {
      double tau = 0.5 + P.nu / T;
      if (P.sensor) {
        double eps = 0.0;
        static_for<0, kQ49>([&](auto kc) {
          constexpr int k = decltype(kc)::value;
          const double feq = rho * weight13<k>(l);
          eps += fabs(sh_pop[k][tid] - feq) / feq;
        });
        tau *= sensor_alpha(eps * (1.0 / kQ49));
      }
      const double om = rcp64(tau);
      const double gfac = (2.0 * P.Cv - 2.0) * T;
      if constexpr (PR) {
        // heat flux of the pulled populations, then BGK plus the term
        double qx = 0.0, qy = 0.0;
        static_for<0, kQ49>([&](auto kc) {
          constexpr int k = decltype(kc)::value;
          const double cx = cx49(k) - upx, cy = cy49(k) - upy;
          const double e = (cx * cx + cy * cy) * sh_pop[k][tid] + sh_pop[kQ49 + k][tid];
          qx = __builtin_fma(0.5 * cx, e, qx);
          qy = __builtin_fma(0.5 * cy, e, qy);
        });
        const ShakhovCoef sc = shakhov_coef<Lattice49>(
            [&](auto kc) { return weight13<decltype(kc)::value>(l); }, rho, upx, upy, T, qx, qy, P);
        const double ks = om - rcp64(0.5 + (tau - 0.5) * P.inv_pr);
        static_for<0, kQ49>([&](auto kc) {
          constexpr int k = decltype(kc)::value;
          const double feq = rho * weight13<k>(l);
          const double geq = gfac * feq;
          double sf, sg;
          shakhov_phi<cx49(k), cy49(k)>(sc, sf, sg);
          const double fk = sh_pop[k][tid], gk = sh_pop[kQ49 + k][tid];
          plane_at(fout + k * N, static_cast<unsigned>(n)) =
              __builtin_fma(om, feq - fk, fk) + ks * feq * sf;
          plane_at(gout + k * N, static_cast<unsigned>(n)) =
              __builtin_fma(om, geq - gk, gk) + ks * geq * sg;
        });
      } else {
        static_for<0, kQ49>([&](auto kc) {
          constexpr int k = decltype(kc)::value;
          const double feq = rho * weight13<k>(l);
          const double geq = gfac * feq;
          const double fk = sh_pop[k][tid], gk = sh_pop[kQ49 + k][tid];
          plane_at(fout + k * N, static_cast<unsigned>(n)) = __builtin_fma(om, feq - fk, fk);
          plane_at(gout + k * N, static_cast<unsigned>(n)) = __builtin_fma(om, geq - gk, gk);
        });
      }
    }
    a.tout[n] = tag_pack(unx, uny, nux, nuy);
    mask[n] = next_mask;
    double* mac = static_cast<double*>(a.carry.mac);
    mac[n] = rho;
    mac[N + n] = upx;
    mac[2 * N + n] = upy;
    mac[3 * N + n] = T;
  }

  {
    const unsigned long long bal = __ballot(next_mask != 0ull);
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

// Post-collision population of plane k in the receiver's lattice (Lx, Ly),
// rebuilt at source s by Grad's ansatz (eq. GradGeneral) from the moments
// of s's last collision and central differences of its neighbours'.
template <bool PR>
__device__ __forceinline__ unsigned rebuild_link49(const RebuildArgs& a, long long s, int Lx,
                                                   int Ly, int k, double& rf, double& rg,
                                                   int& iters) {
  const double* mac = static_cast<const double*>(a.carry.mac);
  const long long N = a.grid.N;
  const int nx = a.grid.nx, ny = a.grid.ny;
  const Phys& P = a.phys;
  const double rho = mac[s];
  double ux, uy, T;
  carried_uT<double>(mac, a.tags, N, s, ux, uy, T);
  rf = 0.0;
  rg = 0.0;
  iters = 0;
  if (!(rho > 0.0) || !(T > 0.0) || !(rho < 1e300) || !(T < 1e300)) return kCodeNonphysical;
  double du[4] = {0.0, 0.0, 0.0, 0.0}, dT[2] = {0.0, 0.0};
  if (P.nu > 0.0) {
    const int ys = static_cast<int>(s / nx), xs = static_cast<int>(s - static_cast<long long>(ys) * nx);
    const long long xp = (long long)ys * nx + wrapc(xs + 1, nx, a.grid.fast_x);
    const long long xm = (long long)ys * nx + wrapc(xs - 1, nx, a.grid.fast_x);
    const long long yp = (long long)wrapc(ys + 1, ny, a.grid.fast_y) * nx + xs;
    const long long ym = (long long)wrapc(ys - 1, ny, a.grid.fast_y) * nx + xs;
    double uxp, uyp, Tp, uxm, uym, Tm, vxp, vyp, Sp, vxm, vym, Sm;
    carried_uT<double>(mac, a.tags, N, xp, uxp, uyp, Tp);
    carried_uT<double>(mac, a.tags, N, xm, uxm, uym, Tm);
    carried_uT<double>(mac, a.tags, N, yp, vxp, vyp, Sp);
    carried_uT<double>(mac, a.tags, N, ym, vxm, vym, Sm);
    du[0] = 0.5 * (uxp - uxm);
    du[2] = 0.5 * (uyp - uym);
    dT[0] = 0.5 * (Tp - Tm);
    du[1] = 0.5 * (vxp - vxm);
    du[3] = 0.5 * (vyp - vym);
    dT[1] = 0.5 * (Sp - Sm);
  }
  double l[kM13];
  const NewtonOut no = solve_equilibrium13(a.table, ux - Lx, uy - Ly, T, P.tol, P.max_iter, l);
  iters = no.iters;
  if (!no.ok) return kCodeNewton;
  double wk = 0.0;
  static_for<0, kQ49>([&](auto kc) {
    constexpr int kk = decltype(kc)::value;
    if (k == kk) wk = weight13<kk>(l);
  });
  const GradState gs = grad_state(rho, ux, uy, T, du, dT, P);
  double phif, phig;
  grad_phi(gs, static_cast<double>(cx49(k) + Lx), static_cast<double>(cy49(k) + Ly), P, phif,
           phig);
  const double tau = 0.5 + P.nu / T;
  const double kf = 1.0 - 1.0 / tau;
  const double feq = rho * wk;
  const double geq = (2.0 * P.Cv - 2.0) * T * feq;
  rf = feq * (1.0 + kf * phif);
  rg = geq * (1.0 + kf * phig);
  if constexpr (PR) {
    // eq. (Shakhov) applied to the source's Grad populations (App. E)
    const double upx = ux - Lx, upy = uy - Ly;
    const double gf = (2.0 * P.Cv - 2.0) * T;
    double qx = 0.0, qy = 0.0;
    static_for<0, kQ49>([&](auto kc) {
      constexpr int kk = decltype(kc)::value;
      double pf, pg;
      grad_phi(gs, static_cast<double>(cx49(kk) + Lx), static_cast<double>(cy49(kk) + Ly), P,
               pf, pg);
      const double fe = rho * weight13<kk>(l);
      const double cx = cx49(kk) - upx, cy = cy49(kk) - upy;
      const double e = (cx * cx + cy * cy) * fe * (1.0 + pf) + gf * fe * (1.0 + pg);
      qx = __builtin_fma(0.5 * cx, e, qx);
      qy = __builtin_fma(0.5 * cy, e, qy);
    });
    const ShakhovCoef sc = shakhov_coef<Lattice49>(
        [&](auto kc) { return weight13<decltype(kc)::value>(l); }, rho, upx, upy, T, qx, qy, P);
    const double ks = 1.0 / tau - 1.0 / (0.5 + (tau - 0.5) * P.inv_pr);
    double sf = 0.0, sg = 0.0;
    static_for<0, kQ49>([&](auto kc) {
      constexpr int kk = decltype(kc)::value;
      if (k == kk) shakhov_phi<cx49(kk), cy49(kk)>(sc, sf, sg);
    });
    rf += ks * feq * sf;
    rg += ks * geq * sg;
  }
  return 0;
}

// Every (receiver, link) item of the list, one per lane (the receivers'
// 64-bit masks expanded wave by wave, as in rebuild_kernel).
template <bool PR = false>
__global__ __launch_bounds__(kBlock) void rebuild49_kernel(RebuildArgs a) {
  __shared__ int sh_node[kWaves][64];
  __shared__ int sh_k[kWaves][64];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const unsigned count = a.carry.counters[(a.step - 1) & 1];
  if (blockIdx.x == 0 && tid == 0) a.carry.counters[a.step & 1] = 0u;
  const Phys& P = a.phys;
  const long long N = a.grid.N;
  const int nx = a.grid.nx;
  double* fout = static_cast<double*>(a.fout);
  double* gout = static_cast<double*>(a.gout);
  const unsigned long long* mask = mask64(a.carry);
  constexpr int kChunk = 8;
  const long long waves = static_cast<long long>(gridDim.x) * kWaves;
  for (long long base = (static_cast<long long>(blockIdx.x) * kWaves + wave) * kChunk; base < count;
       base += waves * kChunk) {
    const long long i = base + lane;
    int node = 0;
    unsigned long long msk = 0ull;
    if (lane < kChunk && i < count) {
      node = a.carry.list[i];
      msk = mask[node];
    }
    const int cnt = __popcll(msk);
    int v = cnt;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const int t = __shfl_up(v, d, 64);
      if (lane >= d) v += t;
    }
    const int total = __shfl(v, 63, 64);
    const int off = v - cnt;
    for (int r0 = 0; r0 < total; r0 += 64) {
      if (cnt > 0 && off < r0 + 64 && off + cnt > r0) {
        int j = off;
        unsigned long long m = msk;
        while (m) {
          const int k = __ffsll(static_cast<long long>(m)) - 1;
          m &= m - 1ull;
          if (j >= r0 && j < r0 + 64) {
            sh_node[wave][j - r0] = node;
            sh_k[wave][j - r0] = k;
          }
          ++j;
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      if (r0 + lane < total) {
        const int xn = sh_node[wave][lane];
        const int k = sh_k[wave][lane];
        const int t = a.tags[xn];
        const int Lx = min(max(tag_unx(t), -P.max_abs_shift), P.max_abs_shift);
        const int Ly = min(max(tag_uny(t), -P.max_abs_shift), P.max_abs_shift);
        const int yx = xn / nx, xx = xn - yx * nx;
        const long long s =
            static_cast<long long>(wrapc(yx - (cy49(k) + Ly), a.grid.ny, a.grid.fast_y)) * nx +
            wrapc(xx - (cx49(k) + Lx), nx, a.grid.fast_x);
        double rf, rg;
        int it;
        const unsigned code = rebuild_link49<PR>(a, s, Lx, Ly, k, rf, rg, it);
        if (code) record_failure(a.diag, a.step, s, code);
        plane_at(fout + k * N, static_cast<unsigned>(xn)) = rf;
        plane_at(gout + k * N, static_cast<unsigned>(xn)) = rg;
        if (P.stats) {
          atomicAdd(&a.diag->mismatched, 1ull);
          atomicAdd(&a.diag->newton_calls, 1ull);
          atomicAdd(&a.diag->newton_iters, static_cast<unsigned long long>(it));
          atomicAdd(&a.diag->hist[it < LBM_HIST_BINS ? it : LBM_HIST_BINS - 1], 1ull);
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
  }
}

// Grad initial condition of the reference model.
__global__ __launch_bounds__(kBlock) void init49_kernel(InitArgs a) {
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
  double* fo = static_cast<double*>(a.fout);
  double* go = static_cast<double*>(a.gout);
  unsigned code = 0;
  if (abs(Ux) > P.max_abs_shift || abs(Uy) > P.max_abs_shift || !(rho > 0.0) || !(T > 0.0) ||
      !(rho < 1e300) || !(T < 1e300))
    code = kCodeNonphysical;
  if (abs(Ux) > P.max_abs_shift || abs(Uy) > P.max_abs_shift) Ux = Uy = 0;
  a.tout[n] = tag_pack(Ux, Uy, Ux, Uy);
  double l[kM13];
  if (!code) {
    const NewtonOut no = solve_equilibrium13(a.table, ux - Ux, uy - Uy, T, P.tol, P.max_iter, l);
    if (!no.ok) code = kCodeNewton;
  }
  if (code) {
    record_failure(a.diag, 0, n, code);
    for (int k = 0; k < kQ49; ++k) {
      fo[k * N + n] = 0.0;
      go[k * N + n] = 0.0;
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
  static_for<0, kQ49>([&](auto kc) {
    constexpr int k = decltype(kc)::value;
    double phif, phig;
    grad_phi(gs, static_cast<double>(cx49(k) + Ux), static_cast<double>(cy49(k) + Uy), P, phif,
             phig);
    const double feq = rho * weight13<k>(l);
    fo[k * N + n] = feq * (1.0 + phif);
    go[k * N + n] = gfac * feq * (1.0 + phig);
  });
}

__global__ __launch_bounds__(kBlock) void macros49_kernel(const double* f, const double* g,
                                                          const int* tags, long long N, double Cv,
                                                          double* rho, double* ux, double* uy,
                                                          double* T, int8_t* Ux, int8_t* Uy) {
  const long long n = static_cast<long long>(blockIdx.x) * kBlock + threadIdx.x;
  if (n >= N) return;
  double r = 0.0, jx = 0.0, jy = 0.0, e = 0.0;
  static_for<0, kQ49>([&](auto kc) {
    constexpr int k = decltype(kc)::value;
    constexpr int cx = cx49(k), cy = cy49(k);
    const double fk = f[k * N + n];
    r += fk;
    jx = cmad<cx>(jx, fk);
    jy = cmad<cy>(jy, fk);
    e = cmad<cx * cx + cy * cy>(e, fk) + g[k * N + n];
  });
  const double upx = jx / r, upy = jy / r;
  const int tg = tags[n];
  rho[n] = r;
  ux[n] = upx + tag_ucx(tg);
  uy[n] = upy + tag_ucy(tg);
  T[n] = (e - r * (upx * upx + upy * upy)) / (2.0 * r * Cv);
  if (Ux) Ux[n] = static_cast<int8_t>(tag_ucx(tg));
  if (Uy) Uy[n] = static_cast<int8_t>(tag_ucy(tg));
}

__global__ __launch_bounds__(kBlock) void conserved49_kernel(const double* f, const double* g,
                                                             const int* tags, long long N,
                                                             double* partials) {
  __shared__ double sh[4][kBlock];
  const int tid = threadIdx.x;
  const long long n = static_cast<long long>(blockIdx.x) * kBlock + tid;
  double m = 0.0, px = 0.0, py = 0.0, en = 0.0;
  if (n < N) {
    const int tg = tags[n];
    const int ucx = tag_ucx(tg), ucy = tag_ucy(tg);
    static_for<0, kQ49>([&](auto kc) {
      constexpr int k = decltype(kc)::value;
      const double fk = f[k * N + n], gk = g[k * N + n];
      const double cx = cx49(k) + ucx, cy = cy49(k) + ucy;
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

}  // namespace lbm
