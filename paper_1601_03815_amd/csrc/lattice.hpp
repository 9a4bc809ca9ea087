// D3Q19 lattice constants for the GPU kernels (compile-time).
//
// Velocity set and weights: Sec. II.A (D3Q19).  MRT transformation: the
// row formulas of Sec. II.B, evaluated here at compile time as integers.
// Population order is the ABI order documented in include/dhit.h.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>
#include <utility>

namespace dhit {

constexpr int kQ = 19;

constexpr int kCx[kQ] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
constexpr int kCy[kQ] = {0, 0, 0, 1, -1, 0, 0, 1, 1, -1, -1, 0, 0, 0, 0, 1, -1, 1, -1};
constexpr int kCz[kQ] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, 1, -1, -1, 1, 1, -1, -1};

constexpr int cdir(int q, int d) { return d == 0 ? kCx[q] : (d == 1 ? kCy[q] : kCz[q]); }
constexpr int speed2(int q) { return kCx[q] * kCx[q] + kCy[q] * kCy[q] + kCz[q] * kCz[q]; }

// Weights as exact rationals 1/3, 1/18, 1/36 (Sec. II.A).
constexpr double kWeight(int q) { return speed2(q) == 0 ? 1.0 / 3.0 : (speed2(q) == 1 ? 1.0 / 18.0 : 1.0 / 36.0); }

// Index of the population with the opposite velocity.
constexpr int opposite(int q) {
  for (int p = 0; p < kQ; ++p)
    if (kCx[p] == -kCx[q] && kCy[p] == -kCy[q] && kCz[p] == -kCz[q]) return p;
  return -1;
}

// Entry M[k][a] of the D3Q19 MRT matrix (Sec. II.B), all integers.
constexpr int mrt_entry(int k, int a) {
  const int x = kCx[a], y = kCy[a], z = kCz[a];
  const int s = x * x + y * y + z * z;
  switch (k) {
    case 0: return 1;
    case 1: return 19 * s - 30;
    case 2: return (21 * s * s - 53 * s + 24) / 2;
    case 3: return x;
    case 4: return (5 * s - 9) * x;
    case 5: return y;
    case 6: return (5 * s - 9) * y;
    case 7: return z;
    case 8: return (5 * s - 9) * z;
    case 9: return 3 * x * x - s;
    case 10: return (3 * s - 5) * (3 * x * x - s);
    case 11: return y * y - z * z;
    case 12: return (3 * s - 5) * (y * y - z * z);
    case 13: return x * y;
    case 14: return y * z;
    case 15: return x * z;
    case 16: return (y * y - z * z) * x;
    case 17: return (z * z - x * x) * y;
    case 18: return (x * x - y * y) * z;
  }
  return 0;
}

// Squared norm of row k (the rows are mutually orthogonal, so
// M^-1 = M^T diag(1/norm)).
constexpr int mrt_norm(int k) {
  int s = 0;
  for (int a = 0; a < kQ; ++a) s += mrt_entry(k, a) * mrt_entry(k, a);
  return s;
}

// Rows whose moments the collision conserves (drho, jx, jy, jz).
constexpr bool mrt_conserved(int k) { return k == 0 || k == 3 || k == 5 || k == 7; }

// Compile-time loop: calls f(std::integral_constant<int, i>) for i = 0..N-1.
template <class F, int... I>
__host__ __device__ __forceinline__ void static_for_impl(F &&f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, I>{}), ...);
}
template <int N, class F>
__host__ __device__ __forceinline__ void static_for(F &&f) {
  static_for_impl(f, std::make_integer_sequence<int, N>{});
}

}  // namespace dhit
