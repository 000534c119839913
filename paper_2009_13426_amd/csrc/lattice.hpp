// D2Q21 velocity set and the compile-time helpers the kernels are built on.
//
// Velocity set (Sec. I, Fig. 1; the paper defers the table to Zhang et al.
// and does not print it): the rest velocity and the ten +- pairs
// (1,0) (0,1) (1,1) (1,-1) (2,0) (0,2) (2,2) (2,-2) (3,0) (0,3).
// Storage plane k: 0 = rest, 1 + 2p = +v_p, 2 + 2p = -v_p.  Pairing +-v lets
// every odd moment be taken from w+ - w- and every even one from w+ + w-.
#pragma once

#include <cstdint>
#include <type_traits>

namespace lbm {

// f(integral_constant<int, K>) ... f(integral_constant<int, N - 1>), unrolled
// at compile time (velocity components become constants).
template <int K, int N, typename F>
__host__ __device__ __forceinline__ void static_for(F&& f) {
  if constexpr (K < N) {
    f(std::integral_constant<int, K>{});
    static_for<K + 1, N>(f);
  }
}

constexpr int kQ = 21;
constexpr int kPairs = 10;
constexpr int kM = 8;  // constraints of the 8-moment equilibrium
constexpr int kPX[kPairs] = {1, 0, 1, 1, 2, 0, 2, 2, 3, 0};
constexpr int kPY[kPairs] = {0, 1, 1, -1, 0, 2, 2, -2, 0, 3};

__host__ __device__ constexpr int plane_cx(int k) {
  return k == 0 ? 0 : (((k - 1) & 1) ? -kPX[(k - 1) >> 1] : kPX[(k - 1) >> 1]);
}
__host__ __device__ constexpr int plane_cy(int k) {
  return k == 0 ? 0 : (((k - 1) & 1) ? -kPY[(k - 1) >> 1] : kPY[(k - 1) >> 1]);
}
__host__ __device__ constexpr int ipow(int b, int e) {
  int r = 1;
  for (int i = 0; i < e; ++i) r *= b;
  return r;
}

// acc + C * v with the multiplication folded away for C in {0, 1, -1}.
template <int C>
__device__ __forceinline__ double cmad(double acc, double v) {
  if constexpr (C == 0)
    return acc;
  else if constexpr (C == 1)
    return acc + v;
  else if constexpr (C == -1)
    return acc - v;
  else
    return __builtin_fma(static_cast<double>(C), v, acc);
}

// Lattice tags: one int32 per node holding two int8 shifts each for the
// lattice of the stored populations (Uc, low half) and the lattice of the
// node's next pull (Un, high half).
__host__ __device__ __forceinline__ int tag_pack(int ucx, int ucy, int unx, int uny) {
  return (ucx & 0xFF) | ((ucy & 0xFF) << 8) | ((unx & 0xFF) << 16) |
         (static_cast<int>(static_cast<unsigned>(uny & 0xFF) << 24));
}
__host__ __device__ __forceinline__ int tag_ucx(int t) { return static_cast<int8_t>(t & 0xFF); }
__host__ __device__ __forceinline__ int tag_ucy(int t) { return static_cast<int8_t>((t >> 8) & 0xFF); }
__host__ __device__ __forceinline__ int tag_unx(int t) { return static_cast<int8_t>((t >> 16) & 0xFF); }
__host__ __device__ __forceinline__ int tag_uny(int t) { return static_cast<int8_t>((t >> 24) & 0xFF); }
__host__ __device__ __forceinline__ int tag_uc16(int t) { return t & 0xFFFF; }
__host__ __device__ __forceinline__ int tag_un16(int t) { return (t >> 16) & 0xFFFF; }

}  // namespace lbm
