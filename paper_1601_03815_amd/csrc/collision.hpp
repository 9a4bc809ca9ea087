// LBE collision operators on one cell held in registers.
//
// BGK:  f <- f - omega (f - f^eq), omega = 1/tau.
// MRT:  f <- f - M^-1 S (M f - m^eq)  (Sec. II.B evolution equation), with
//       the sparse integer rows of M expanded at compile time and
//       M^-1 = M^T diag(1/norm) folded into the rates r_k = s_k / norm_k.
#pragma once

#include "device_common.hpp"
#include "runtime.hpp"

namespace dhit {

enum Coll { kBGK = 0, kMRT = 1 };

template <typename Real>
__device__ __forceinline__ void collide_bgk(Real (&f)[kQ], Real drho, Real jx, Real jy, Real jz,
                                            const StepParams &p) {
  Real feq[kQ];
  equilibrium<Real>(drho, jx, jy, jz, Real(p.rho0), Real(p.inv_rho0), feq);
  const Real om = Real(p.omega);
  static_for<kQ>([&](auto q) { f[q] = f[q] - om * (f[q] - feq[q]); });
}

// Equilibrium value of moment k (Sec. II.B), for non-conserved rows.
template <int K, typename Real>
__device__ __forceinline__ Real mrt_meq(Real drho, Real jx, Real jy, Real jz, Real inv_rho0, Real jj,
                                        const StepParams &p) {
  if constexpr (K == 1) return Real(-11) * drho + Real(19) * jj;
  else if constexpr (K == 2) return Real(p.w_eps) * drho + Real(p.w_epsj) * jj;
  else if constexpr (K == 4) return Real(-2.0 / 3.0) * jx;
  else if constexpr (K == 6) return Real(-2.0 / 3.0) * jy;
  else if constexpr (K == 8) return Real(-2.0 / 3.0) * jz;
  else if constexpr (K == 9) return (Real(2) * jx * jx - jy * jy - jz * jz) * inv_rho0;
  else if constexpr (K == 10) return Real(p.w_xx) * ((Real(2) * jx * jx - jy * jy - jz * jz) * inv_rho0);
  else if constexpr (K == 11) return (jy * jy - jz * jz) * inv_rho0;
  else if constexpr (K == 12) return Real(p.w_xx) * ((jy * jy - jz * jz) * inv_rho0);
  else if constexpr (K == 13) return jx * jy * inv_rho0;
  else if constexpr (K == 14) return jy * jz * inv_rho0;
  else if constexpr (K == 15) return jx * jz * inv_rho0;
  else return Real(0);  // 16, 17, 18
}

template <typename Real>
__device__ __forceinline__ void collide_mrt(Real (&f)[kQ], Real drho, Real jx, Real jy, Real jz,
                                            const StepParams &p) {
  const Real inv_rho0 = Real(p.inv_rho0);
  const Real jj = (jx * jx + jy * jy + jz * jz) * inv_rho0;
  Real dm[kQ];
  static_for<kQ>([&](auto k) {
    if constexpr (!mrt_conserved(k)) {
      Real m = Real(0);
      static_for<kQ>([&](auto a) {
        constexpr int e = mrt_entry(k, a);
        if constexpr (e == 1) m += f[a];
        else if constexpr (e == -1) m -= f[a];
        else if constexpr (e != 0) m += Real(e) * f[a];
      });
      dm[k] = Real(p.r[k]) * (m - mrt_meq<k, Real>(drho, jx, jy, jz, inv_rho0, jj, p));
    }
  });
  static_for<kQ>([&](auto a) {
    Real acc = Real(0);
    static_for<kQ>([&](auto k) {
      if constexpr (!mrt_conserved(k)) {
        constexpr int e = mrt_entry(k, a);
        if constexpr (e == 1) acc += dm[k];
        else if constexpr (e == -1) acc -= dm[k];
        else if constexpr (e != 0) acc += Real(e) * dm[k];
      }
    });
    f[a] -= acc;
  });
}

template <int C, typename Real>
__device__ __forceinline__ void collide(Real (&f)[kQ], Real drho, Real jx, Real jy, Real jz,
                                        const StepParams &p) {
  if constexpr (C == kBGK) collide_bgk<Real>(f, drho, jx, jy, jz, p);
  else collide_mrt<Real>(f, drho, jx, jy, jz, p);
}

// MRT equilibrium in population space, f = M^-1 m^eq: the fixed point of
// the MRT collision for the given conserved moments.
template <typename Real>
__device__ __forceinline__ void mrt_equilibrium_populations(Real drho, Real jx, Real jy, Real jz,
                                                            const StepParams &p, Real (&f)[kQ]) {
  const Real inv_rho0 = Real(p.inv_rho0);
  const Real jj = (jx * jx + jy * jy + jz * jz) * inv_rho0;
  Real meq[kQ];
  static_for<kQ>([&](auto k) {
    if constexpr (k == 0) meq[k] = drho;
    else if constexpr (k == 3) meq[k] = jx;
    else if constexpr (k == 5) meq[k] = jy;
    else if constexpr (k == 7) meq[k] = jz;
    else meq[k] = mrt_meq<k, Real>(drho, jx, jy, jz, inv_rho0, jj, p);
  });
  static_for<kQ>([&](auto a) {
    Real acc = Real(0);
    static_for<kQ>([&](auto k) {
      constexpr int e = mrt_entry(k, a);
      if constexpr (e != 0) acc += Real(double(e) / double(mrt_norm(k))) * meq[k];
    });
    f[a] = acc;
  });
}

}  // namespace dhit
