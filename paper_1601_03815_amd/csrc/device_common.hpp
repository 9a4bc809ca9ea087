// Device helpers shared by the LBE, DUGKS and diagnostics kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "lattice.hpp"

namespace dhit {

constexpr int kBlock = 256;            // threads per block of the streaming kernels
constexpr int kWaves = kBlock / 64;    // 64-wide wavefronts per block
constexpr int kNumSums = 5;            // sum drho, sum jx, sum jy, sum jz, 1/2 sum |u|^2

// Compensated summation (Kahan): s carries the running sum and c the
// rounding error of the last addition (with its sign reversed), which is
// fed back into the next term, so that the error of a sum of m terms is
// about 2 eps sum |x_i| instead of (m - 1) eps sum |x_i|.  Used for the
// per-cell moment sums of FP32 boxes.
template <typename Real>
struct CompSum {
  Real s = Real(0), c = Real(0);
  __device__ __forceinline__ void add(Real x) {
    const Real y = x - c;
    const Real t = s + y;
    c = (t - s) - y;
    s = t;
  }
  __device__ __forceinline__ void sub(Real x) { add(-x); }
  __device__ __forceinline__ Real value() const { return s - c; }
};

// Moments of one cell: drho = sum f, j = sum xi f (Sec. II.A / II.B).
// Double: plain sums.  Float: compensated sums.
template <typename Real>
__device__ __forceinline__ void cell_moments(const Real (&f)[kQ], Real &drho, Real &jx, Real &jy, Real &jz) {
  if constexpr (std::is_same<Real, double>::value) {
    double r = 0, ax = 0, ay = 0, az = 0;
    static_for<kQ>([&](auto q) {
      r += f[q];
      if constexpr (kCx[q] == 1) ax += f[q];
      if constexpr (kCx[q] == -1) ax -= f[q];
      if constexpr (kCy[q] == 1) ay += f[q];
      if constexpr (kCy[q] == -1) ay -= f[q];
      if constexpr (kCz[q] == 1) az += f[q];
      if constexpr (kCz[q] == -1) az -= f[q];
    });
    drho = r; jx = ax; jy = ay; jz = az;
  } else {
    CompSum<Real> r, ax, ay, az;
    static_for<kQ>([&](auto q) {
      r.add(f[q]);
      if constexpr (kCx[q] == 1) ax.add(f[q]);
      if constexpr (kCx[q] == -1) ax.sub(f[q]);
      if constexpr (kCy[q] == 1) ay.add(f[q]);
      if constexpr (kCy[q] == -1) ay.sub(f[q]);
      if constexpr (kCz[q] == 1) az.add(f[q]);
      if constexpr (kCz[q] == -1) az.sub(f[q]);
    });
    drho = r.value(); jx = ax.value(); jy = ay.value(); jz = az.value();
  }
}

// Discrete incompressible equilibrium of Sec. II.A with RT = 1/3:
// f_q^eq = W_q [drho + rho0 (3 xi.u + 9/2 (xi.u)^2 - 3/2 |u|^2)], u = j/rho0,
// evaluated as W_q (base + 9/2 rho0 (xi.u)^2) + L_q rho0 xi.u with
// base = drho - 3/2 rho0 |u|^2 and L_q = 3 W_q (1/6 on the axes, 1/12 on the
// diagonals).  The momentum of the linear term is u sum_q L_q xi_qx^2 =
// u (2 L_axis + 8 L_diag); with 3 W_q rounded to the working precision that
// factor is 1 + d (d = 7e-9 in FP32), and a BGK or DUGKS collision then adds
// a fixed fraction of d j to the momentum at every step (a steady energy
// drift, 3e-8 per DUGKS step in FP32).  L_diag is rounded and L_axis taken as
// (1 - 8 L_diag)/2, which is exact, so that the factor is exactly 1.
template <typename Real>
constexpr Real kLinDiag = Real(1.0 / 12.0);
template <typename Real>
constexpr Real kLinAxis = (Real(1) - Real(8) * kLinDiag<Real>) / Real(2);

// xi_q . u
template <int Q, typename Real>
__device__ __forceinline__ Real xi_dot(Real ux, Real uy, Real uz) {
  Real xu = Real(0);
  if constexpr (kCx[Q] == 1) xu += ux;
  if constexpr (kCx[Q] == -1) xu -= ux;
  if constexpr (kCy[Q] == 1) xu += uy;
  if constexpr (kCy[Q] == -1) xu -= uy;
  if constexpr (kCz[Q] == 1) xu += uz;
  if constexpr (kCz[Q] == -1) xu -= uz;
  return xu;
}

// f_Q^eq from base and xu = xi_Q . u (see above).
template <int Q, typename Real>
__device__ __forceinline__ Real equilibrium_q(Real base, Real xu, Real rho0) {
  constexpr Real w = Real(kWeight(Q));
  constexpr Real l = speed2(Q) == 0 ? Real(0) : (speed2(Q) == 1 ? kLinAxis<Real> : kLinDiag<Real>);
  const Real even = w * (base + Real(4.5) * rho0 * xu * xu);
  if constexpr (Q == 0)
    return even;
  else
    return even + l * rho0 * xu;
}

template <typename Real>
__device__ __forceinline__ void equilibrium(Real drho, Real jx, Real jy, Real jz, Real rho0, Real inv_rho0,
                                            Real (&feq)[kQ]) {
  const Real ux = jx * inv_rho0, uy = jy * inv_rho0, uz = jz * inv_rho0;
  const Real uu = ux * ux + uy * uy + uz * uz;
  const Real base = drho - Real(1.5) * rho0 * uu;
  static_for<kQ>([&](auto q) { feq[q] = equilibrium_q<q, Real>(base, xi_dot<q>(ux, uy, uz), rho0); });
}

// Sum of five doubles over the block; thread 0 gets the block total.
// Deterministic: fixed shuffle tree inside each wavefront, then the
// wavefront totals in wavefront order.
__device__ __forceinline__ void block_sum5(double (&v)[kNumSums], double (*smem)[kNumSums]) {
  static_for<kNumSums>([&](auto i) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v[i] += __shfl_down(v[i], off, 64);
  });
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) {
    static_for<kNumSums>([&](auto i) { smem[wave][i] = v[i]; });
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    static_for<kNumSums>([&](auto i) {
      double s = smem[0][i];
      for (int w = 1; w < (int)(blockDim.x >> 6); ++w) s += smem[w][i];
      v[i] = s;
    });
  }
}

// Per-cell contributions to the five global sums, accumulated in FP64 from
// the stored values (exact for FP32 populations, which double represents).
template <typename Real>
__device__ __forceinline__ void sums_of_populations(const Real (&f)[kQ], double inv_rho0, double (&v)[kNumSums]) {
  double r = 0, ax = 0, ay = 0, az = 0;
  static_for<kQ>([&](auto q) {
    const double x = (double)f[q];
    r += x;
    if constexpr (kCx[q] == 1) ax += x;
    if constexpr (kCx[q] == -1) ax -= x;
    if constexpr (kCy[q] == 1) ay += x;
    if constexpr (kCy[q] == -1) ay -= x;
    if constexpr (kCz[q] == 1) az += x;
    if constexpr (kCz[q] == -1) az -= x;
  });
  v[0] += r;
  v[1] += ax;
  v[2] += ay;
  v[3] += az;
  v[4] += 0.5 * (ax * ax + ay * ay + az * az) * inv_rho0 * inv_rho0;
}

// Per-cell contributions to the five global sums.
template <typename Real>
__device__ __forceinline__ void sums_of_cell(Real drho, Real jx, Real jy, Real jz, double inv_rho0,
                                             double (&v)[kNumSums]) {
  const double x = (double)jx, y = (double)jy, z = (double)jz;
  v[0] += (double)drho;
  v[1] += x;
  v[2] += y;
  v[3] += z;
  v[4] += 0.5 * (x * x + y * y + z * z) * inv_rho0 * inv_rho0;
}

// Pointer into global memory.  The device functions that stream population
// fields take these, so that their accesses compile to global instructions
// also where a kernel reads the field pointers from a device table (through
// a generic pointer they would compile to flat instructions, which count
// against the LDS counter as well: every LDS wait would also wait for memory).
template <typename T>
using global_t = __attribute__((address_space(1))) T;
template <typename T>
__device__ __forceinline__ global_t<T> *to_global(T *p) {
  return (global_t<T> *)p;
}

// Writes the block's five sums to partials laid out [5][nblocks], using
// smem (at least one row of five doubles per wavefront of the block) for
// the reduction.
__device__ __forceinline__ void write_block_partials(double (&v)[kNumSums], double *partials, int nblocks, int block,
                                                     double (*smem)[kNumSums]) {
  block_sum5(v, smem);
  if (threadIdx.x == 0) {
    static_for<kNumSums>([&](auto i) { to_global(partials)[(int64_t)i * nblocks + block] = v[i]; });
  }
}
__device__ __forceinline__ void write_block_partials(double (&v)[kNumSums], double *partials, int nblocks,
                                                     int block) {
  __shared__ double smem[kBlock / 64][kNumSums];
  write_block_partials(v, partials, nblocks, block, smem);
}

// Flat-index offsets of the +-1 neighbours along one axis with periodic
// wrap: up = offset of coordinate+1, dn = offset of coordinate-1.
struct AxisOff {
  int up, dn;
};
__device__ __forceinline__ AxisOff axis_offsets(int c, int n, int unit) {
  AxisOff o;
  o.up = (c == n - 1) ? -(n - 1) * unit : unit;
  o.dn = (c == 0) ? (n - 1) * unit : -unit;
  return o;
}

}  // namespace dhit
