// DUGKS time step (Sec. II.A finite-volume update).
//
// With tau = nu/RT, h = dt/2, the tracked field is f~.  Per cell:
//   moments of f~ -> f^eq -> fbp = a f~ + b f^eq, a = (2tau-h)/(2tau+dt),
//   b = 3h/(2tau+dt);  f~+ = 4/3 fbp - 1/3 f~.
// Per face between L and R = L + e_d, for all 19 populations:
//   fbar = (fbp_L + fbp_R)/2 - h [xi_d (fbp_R - fbp_L)
//          + sum_{t != d} xi_t (G_t(L) + G_t(R))/4],  G_t(c) = fbp(c+e_t) - fbp(c-e_t)
//   face moments of fbar -> f^eq_face -> f_face = alpha fbar + beta f^eq_face,
//   alpha = 2tau/(2tau+h), beta = h/(2tau+h).
// Update: f~(t+dt) = f~+ - dt sum_d xi_d (f_face(+d) - f_face(-d))   (dx = 1).
//
// This file holds the two-pass form (DHIT_VARIANT_TWO_PASS): a transform
// kernel writes fbp to a scratch field, then a face kernel evaluates the six
// faces of each cell from that field (through the caches) and writes the
// update.  It follows the face-by-face description directly and serves as a
// cross-check of the fused kernel (dugks_fused.hip), which is the default.
//
// It also holds the stretched-mesh form (set_mesh): the same two passes
// with the reconstruction written for cell widths w that vary along each
// axis (Sec. II.A's interpolation with x_b - x_L = w_L/2 and the gradient
// over c_R - c_L; tangential central differences over c_{k+1} - c_{k-1},
// interpolated to the face with the value's weight):
//   fbar = fbp_L + lam sd - h [xi_d sd / gap + sum_t xi_t (G_t(L) + lam (G_t(R) - G_t(L))) / span_t],
//   lam = w_L/(w_L + w_R), gap = (w_L + w_R)/2, sd = fbp_R - fbp_L,
// and the update f~(t+dt) = f~+ - dt sum_d xi_d (f_face(+d) - f_face(-d)) / w_d.
#include "collision.hpp"

namespace dhit {

template <typename Real>
__global__ __launch_bounds__(kBlock) void dugks_transform_kernel(const Real *__restrict__ ft, Real *__restrict__ fbp,
                                                                 StepParams p, int ncell) {
  const int cell = blockIdx.x * kBlock + threadIdx.x;
  if (cell >= ncell) return;
  const int64_t stride = p.stride;
  Real f[kQ];
  static_for<kQ>([&](auto q) { f[q] = ft[(int64_t)q * stride + cell]; });
  Real drho, jx, jy, jz, feq[kQ];
  cell_moments<Real>(f, drho, jx, jy, jz);
  equilibrium<Real>(drho, jx, jy, jz, Real(p.rho0), Real(p.inv_rho0), feq);
  // fbp = a f~ + b f^eq with a + b = 1, written as f^eq + a (f~ - f^eq) so
  // that an equilibrium cell maps to itself exactly in any precision
  const Real a = Real(p.a_bp);
  static_for<kQ>([&](auto q) { fbp[(int64_t)q * stride + cell] = feq[q] + a * (f[q] - feq[q]); });
}

// Block numbering for the face kernels: blocks are dealt to the eight XCDs
// in turn (block b runs on XCD b mod 8), so block b takes the row range
// that puts consecutive rows, and so a cell's y and z neighbour rows, on
// the same XCD and its L2.  A bijection of [0, nblocks) for any nblocks.
__device__ __forceinline__ int xcd_block(int b, int nblocks) {
  const int xcd = b & 7, per = nblocks >> 3, extra = nblocks & 7;
  return xcd * per + (xcd < extra ? xcd : extra) + (b >> 3);
}

// Offsets of the 3x3x3 neighbourhood of a cell: off(dx,dy,dz) = X[dx] + Y[dy] + Z[dz].
struct Nbr {
  int X[3], Y[3], Z[3];  // index 0 = -1, 1 = 0, 2 = +1
  __device__ __forceinline__ int at(int dx, int dy, int dz) const { return X[dx + 1] + Y[dy + 1] + Z[dz + 1]; }
};

// Face f (all fluxing populations) of the face at side s (+1 / -1) of the
// cell along axis D; accumulates s * xi_D * f_face into acc.  Off32 as in
// face_accumulate_mesh.
template <int D, int S, bool Off32, typename Real>
__device__ __forceinline__ void face_accumulate(const Real *__restrict__ fbp, int cell, const Nbr &nb,
                                                const StepParams &p, Real (&acc)[kQ]) {
  const int64_t stride = p.stride;
  // L = cell + (S == -1 ? -e_D : 0), R = L + e_D
  constexpr int l = (S == -1) ? -1 : 0;
  constexpr int r = l + 1;
  auto off = [&](int a, int tb, int tc) {  // offset of (a along D, tb, tc along the two tangents)
    int d[3] = {0, 0, 0};
    d[D] = a;
    constexpr int T1 = (D + 1) % 3, T2 = (D + 2) % 3;
    d[T1] = tb;
    d[T2] = tc;
    return nb.at(d[0], d[1], d[2]);
  };
  constexpr int T1 = (D + 1) % 3, T2 = (D + 2) % 3;
  const Real h = Real(p.h);
  Real fbar[kQ];
  static_for<kQ>([&](auto q) {
    const Real *fq = fbp + (int64_t)q * stride + cell;
    const uint32_t qoff = (uint32_t)q * (uint32_t)stride + (uint32_t)cell;
    auto ld = [&](int o) {
      if constexpr (Off32)
        return *reinterpret_cast<const Real *>(reinterpret_cast<const char *>(fbp) +
                                               (uint32_t)(qoff + (uint32_t)o) * (uint32_t)sizeof(Real));
      else
        return fq[o];
    };
    const Real fl = ld(off(l, 0, 0)), fr = ld(off(r, 0, 0));
    const Real sd = fr - fl;
    Real tang = Real(0);
    if constexpr (cdir(q, T1) != 0) {
      const Real st = Real(0.25) * ((ld(off(l, 1, 0)) - ld(off(l, -1, 0))) + (ld(off(r, 1, 0)) - ld(off(r, -1, 0))));
      tang += Real(cdir(q, T1)) * st;
    }
    if constexpr (cdir(q, T2) != 0) {
      const Real st = Real(0.25) * ((ld(off(l, 0, 1)) - ld(off(l, 0, -1))) + (ld(off(r, 0, 1)) - ld(off(r, 0, -1))));
      tang += Real(cdir(q, T2)) * st;
    }
    fbar[q] = (fl + Real(0.5) * sd) - h * (Real(cdir(q, D)) * sd + tang);
    if constexpr (std::is_same<Real, double>::value && q % 2 == 1) __builtin_amdgcn_sched_barrier(0);
  });
  Real drho, jx, jy, jz, feq[kQ];
  cell_moments<Real>(fbar, drho, jx, jy, jz);
  equilibrium<Real>(drho, jx, jy, jz, Real(p.rho0), Real(p.inv_rho0), feq);
  const Real al = Real(p.alpha), be = Real(p.beta);
  static_for<kQ>([&](auto q) {
    if constexpr (cdir(q, D) != 0) {
      const Real ff = al * fbar[q] + be * feq[q];
      if constexpr (S * cdir(q, D) > 0) acc[q] += ff;
      else acc[q] -= ff;
    }
  });
}

template <typename Real, bool Off32>
__global__ __launch_bounds__(kBlock) void dugks_face_kernel(const Real *__restrict__ ft, const Real *__restrict__ fbp,
                                                            Real *__restrict__ out, StepParams p, int ncell,
                                                            double *__restrict__ partials) {
  const int n = p.n;
  const int block = xcd_block(blockIdx.x, gridDim.x);
  const int cell = block * kBlock + threadIdx.x;
  double v[kNumSums] = {0, 0, 0, 0, 0};
  if (cell < ncell) {
    const int x = cell % n;
    const int t = cell / n;
    const int y = t % n;
    const int z = t / n;
    const AxisOff ox = axis_offsets(x, n, 1), oy = axis_offsets(y, n, n), oz = axis_offsets(z, n, n * n);
    Nbr nb;
    nb.X[0] = ox.dn; nb.X[1] = 0; nb.X[2] = ox.up;
    nb.Y[0] = oy.dn; nb.Y[1] = 0; nb.Y[2] = oy.up;
    nb.Z[0] = oz.dn; nb.Z[1] = 0; nb.Z[2] = oz.up;
    Real acc[kQ];
    static_for<kQ>([&](auto q) { acc[q] = Real(0); });
    face_accumulate<0, 1, Off32, Real>(fbp, cell, nb, p, acc);
    if constexpr (std::is_same<Real, double>::value) __builtin_amdgcn_sched_barrier(0);
    face_accumulate<0, -1, Off32, Real>(fbp, cell, nb, p, acc);
    if constexpr (std::is_same<Real, double>::value) __builtin_amdgcn_sched_barrier(0);
    face_accumulate<1, 1, Off32, Real>(fbp, cell, nb, p, acc);
    if constexpr (std::is_same<Real, double>::value) __builtin_amdgcn_sched_barrier(0);
    face_accumulate<1, -1, Off32, Real>(fbp, cell, nb, p, acc);
    if constexpr (std::is_same<Real, double>::value) __builtin_amdgcn_sched_barrier(0);
    face_accumulate<2, 1, Off32, Real>(fbp, cell, nb, p, acc);
    if constexpr (std::is_same<Real, double>::value) __builtin_amdgcn_sched_barrier(0);
    face_accumulate<2, -1, Off32, Real>(fbp, cell, nb, p, acc);
    const int64_t stride = p.stride;
    const Real dt = Real(p.dt);
    Real o[kQ];
    static_for<kQ>([&](auto q) {
      const Real bp = fbp[(int64_t)q * stride + cell];
      const Real tl = ft[(int64_t)q * stride + cell];
      // f~+ = 4/3 fbp - 1/3 f~ = fbp + (fbp - f~)/3 (exact when fbp = f~)
      o[q] = (bp + (bp - tl) * Real(1.0 / 3.0)) - dt * acc[q];
      out[(int64_t)q * stride + cell] = o[q];
    });
    sums_of_populations<Real>(o, p.inv_rho0, v);
  }
  write_block_partials(v, partials, gridDim.x, block);
}

// Face at side S of the cell along axis D on a stretched mesh; adds
// S xi_D f_face / w_D(cell) to acc.  pos = the cell's (x, y, z).
// Off32: address the field with 32-bit byte offsets from its base (valid
// when the whole field is below 4 GB; fewer live address registers).
template <int D, int S, bool Off32, typename Real>
__device__ __forceinline__ void face_accumulate_mesh(const Real *__restrict__ fbp, int cell, const Nbr &nb,
                                                     const int (&pos)[3], const double *__restrict__ mesh,
                                                     const StepParams &p, Real (&acc)[kQ]) {
  const int64_t stride = p.stride;
  const int n = p.n;
  constexpr int l = (S == -1) ? -1 : 0;
  constexpr int r = l + 1;
  constexpr int T1 = (D + 1) % 3, T2 = (D + 2) % 3;
  auto off = [&](int a, int tb, int tc) {
    int d[3] = {0, 0, 0};
    d[D] = a;
    d[T1] = tb;
    d[T2] = tc;
    return nb.at(d[0], d[1], d[2]);
  };
  auto table = [&](int axis, int t, int i) { return mesh[((int64_t)axis * kMeshTables + t) * n + i]; };
  const int iL = (S == -1) ? (pos[D] == 0 ? n - 1 : pos[D] - 1) : pos[D];
  const Real lam = Real(table(D, kMeshLam, iL)), inv_gap = Real(table(D, kMeshInvGap, iL));
  const Real inv_span1 = Real(table(T1, kMeshInvSpan, pos[T1]));
  const Real inv_span2 = Real(table(T2, kMeshInvSpan, pos[T2]));
  const Real inv_w = Real(table(D, kMeshInvWidth, pos[D]));
  const Real h = Real(p.h);
  Real fbar[kQ];
  static_for<kQ>([&](auto q) {
    const Real *fq = fbp + (int64_t)q * stride + cell;
    const uint32_t qoff = (uint32_t)q * (uint32_t)stride + (uint32_t)cell;
    auto ld = [&](int o) {
      if constexpr (Off32)  // element q*stride + cell + o, as a byte offset (wraps back into range for o < 0)
        return *reinterpret_cast<const Real *>(reinterpret_cast<const char *>(fbp) +
                                               (uint32_t)(qoff + (uint32_t)o) * (uint32_t)sizeof(Real));
      else
        return fq[o];
    };
    const Real fl = ld(off(l, 0, 0)), fr = ld(off(r, 0, 0));
    const Real sd = fr - fl;
    Real tang = Real(0);
    if constexpr (cdir(q, T1) != 0) {
      const Real gl = ld(off(l, 1, 0)) - ld(off(l, -1, 0)), gr = ld(off(r, 1, 0)) - ld(off(r, -1, 0));
      tang += Real(cdir(q, T1)) * (inv_span1 * (gl + lam * (gr - gl)));
    }
    if constexpr (cdir(q, T2) != 0) {
      const Real gl = ld(off(l, 0, 1)) - ld(off(l, 0, -1)), gr = ld(off(r, 0, 1)) - ld(off(r, 0, -1));
      tang += Real(cdir(q, T2)) * (inv_span2 * (gl + lam * (gr - gl)));
    }
    fbar[q] = (fl + lam * sd) - h * (Real(cdir(q, D)) * (sd * inv_gap) + tang);
    // FP64: keep the scheduler from hoisting the loads of the whole face: with
    // them in flight at once the kernel needs more than 256 registers (one
    // wave per SIMD); in pairs of populations it runs two.  FP32 fits
    // two waves without this and is faster with the full face in flight.
    if constexpr (std::is_same<Real, double>::value && q % 2 == 1) __builtin_amdgcn_sched_barrier(0);
  });
  Real drho, jx, jy, jz, feq[kQ];
  cell_moments<Real>(fbar, drho, jx, jy, jz);
  equilibrium<Real>(drho, jx, jy, jz, Real(p.rho0), Real(p.inv_rho0), feq);
  const Real al = Real(p.alpha), be = Real(p.beta);
  static_for<kQ>([&](auto q) {
    if constexpr (cdir(q, D) != 0) {
      const Real ff = (al * fbar[q] + be * feq[q]) * inv_w;
      if constexpr (S * cdir(q, D) > 0) acc[q] += ff;
      else acc[q] -= ff;
    }
  });
}

// Face kernel of the stretched mesh; the five sums are weighted by the
// cell volumes w_x w_y w_z.
template <typename Real, bool Off32>
__global__ __launch_bounds__(kBlock) void dugks_mesh_face_kernel(const Real *__restrict__ ft,
                                                                 const Real *__restrict__ fbp, Real *__restrict__ out,
                                                                 StepParams p, int ncell,
                                                                 const double *__restrict__ mesh,
                                                                 double *__restrict__ partials) {
  const int n = p.n;
  const int block = xcd_block(blockIdx.x, gridDim.x);
  const int cell = block * kBlock + threadIdx.x;
  double v[kNumSums] = {0, 0, 0, 0, 0};
  if (cell < ncell) {
    const int x = cell % n;
    const int t = cell / n;
    const int y = t % n;
    const int z = t / n;
    const int pos[3] = {x, y, z};
    const AxisOff ox = axis_offsets(x, n, 1), oy = axis_offsets(y, n, n), oz = axis_offsets(z, n, n * n);
    Nbr nb;
    nb.X[0] = ox.dn; nb.X[1] = 0; nb.X[2] = ox.up;
    nb.Y[0] = oy.dn; nb.Y[1] = 0; nb.Y[2] = oy.up;
    nb.Z[0] = oz.dn; nb.Z[1] = 0; nb.Z[2] = oz.up;
    Real acc[kQ];
    static_for<kQ>([&](auto q) { acc[q] = Real(0); });
    // FP64: one face at a time (see the register note in face_accumulate_mesh)
    face_accumulate_mesh<0, 1, Off32, Real>(fbp, cell, nb, pos, mesh, p, acc);
    if constexpr (std::is_same<Real, double>::value) __builtin_amdgcn_sched_barrier(0);
    face_accumulate_mesh<0, -1, Off32, Real>(fbp, cell, nb, pos, mesh, p, acc);
    if constexpr (std::is_same<Real, double>::value) __builtin_amdgcn_sched_barrier(0);
    face_accumulate_mesh<1, 1, Off32, Real>(fbp, cell, nb, pos, mesh, p, acc);
    if constexpr (std::is_same<Real, double>::value) __builtin_amdgcn_sched_barrier(0);
    face_accumulate_mesh<1, -1, Off32, Real>(fbp, cell, nb, pos, mesh, p, acc);
    if constexpr (std::is_same<Real, double>::value) __builtin_amdgcn_sched_barrier(0);
    face_accumulate_mesh<2, 1, Off32, Real>(fbp, cell, nb, pos, mesh, p, acc);
    if constexpr (std::is_same<Real, double>::value) __builtin_amdgcn_sched_barrier(0);
    face_accumulate_mesh<2, -1, Off32, Real>(fbp, cell, nb, pos, mesh, p, acc);
    const int64_t stride = p.stride;
    const Real dt = Real(p.dt);
    Real o[kQ];
    static_for<kQ>([&](auto q) {
      const Real bp = fbp[(int64_t)q * stride + cell];
      const Real tl = ft[(int64_t)q * stride + cell];
      o[q] = (bp + (bp - tl) * Real(1.0 / 3.0)) - dt * acc[q];
      out[(int64_t)q * stride + cell] = o[q];
    });
    double c[kNumSums] = {0, 0, 0, 0, 0};
    sums_of_populations<Real>(o, p.inv_rho0, c);
    const double vol = mesh[(0 * kMeshTables + kMeshWidth) * n + x] * mesh[(1 * kMeshTables + kMeshWidth) * n + y] *
                       mesh[(2 * kMeshTables + kMeshWidth) * n + z];
    static_for<kNumSums>([&](auto i) { v[i] = vol * c[i]; });
  }
  write_block_partials(v, partials, gridDim.x, block);
}

template <typename Real>
static void dugks_mesh_two_pass(dhit_box &b, const void *src, void *dst, double *sums_out) {
  const int blocks = cell_blocks(b.ncell);
  const Real *s = static_cast<const Real *>(src);
  Real *d = static_cast<Real *>(dst);
  Real *bp = static_cast<Real *>(b.scratch);
  {
    TimedLaunch t(b, DHIT_K_DUGKS_TRANSFORM);
    hipLaunchKernelGGL((dugks_transform_kernel<Real>), dim3(blocks), dim3(kBlock), 0, b.stream, s, bp, b.sp,
                       (int)b.ncell);
    DHIT_HIP(hipGetLastError());
    t.done();
  }
  {
    TimedLaunch t(b, DHIT_K_DUGKS_FACE);
    // 32-bit byte offsets when the whole field (19 padded arrays) is below 4 GB
    const bool off32 = (uint64_t)kQ * (uint64_t)b.stride * sizeof(Real) < (uint64_t(1) << 32);
    if (off32)
      hipLaunchKernelGGL((dugks_mesh_face_kernel<Real, true>), dim3(blocks), dim3(kBlock), 0, b.stream, s, bp, d,
                         b.sp, (int)b.ncell, b.mesh, b.partials);
    else
      hipLaunchKernelGGL((dugks_mesh_face_kernel<Real, false>), dim3(blocks), dim3(kBlock), 0, b.stream, s, bp, d,
                         b.sp, (int)b.ncell, b.mesh, b.partials);
    DHIT_HIP(hipGetLastError());
    t.done();
  }
  launch_finalize_sums(b, b.partials, blocks, sums_out);
}

template <typename Real>
static void dugks_two_pass(dhit_box &b, const void *src, void *dst, double *sums_out) {
  const int blocks = cell_blocks(b.ncell);
  const Real *s = static_cast<const Real *>(src);
  Real *d = static_cast<Real *>(dst);
  Real *bp = static_cast<Real *>(b.scratch);
  {
    TimedLaunch t(b, DHIT_K_DUGKS_TRANSFORM);
    hipLaunchKernelGGL((dugks_transform_kernel<Real>), dim3(blocks), dim3(kBlock), 0, b.stream, s, bp, b.sp,
                       (int)b.ncell);
    DHIT_HIP(hipGetLastError());
    t.done();
  }
  {
    TimedLaunch t(b, DHIT_K_DUGKS_FACE);
    const bool off32 = (uint64_t)kQ * (uint64_t)b.stride * sizeof(Real) < (uint64_t(1) << 32);
    if (off32)
      hipLaunchKernelGGL((dugks_face_kernel<Real, true>), dim3(blocks), dim3(kBlock), 0, b.stream, s, bp, d, b.sp,
                         (int)b.ncell, b.partials);
    else
      hipLaunchKernelGGL((dugks_face_kernel<Real, false>), dim3(blocks), dim3(kBlock), 0, b.stream, s, bp, d, b.sp,
                         (int)b.ncell, b.partials);
    DHIT_HIP(hipGetLastError());
    t.done();
  }
  launch_finalize_sums(b, b.partials, blocks, sums_out);
}

void launch_dugks_step(dhit_box &b, const void *src, void *dst, double *sums_out) {
  if (b.mesh) {
    if (b.p.precision == DHIT_FP64)
      dugks_mesh_two_pass<double>(b, src, dst, sums_out);
    else
      dugks_mesh_two_pass<float>(b, src, dst, sums_out);
    return;
  }
  if (b.p.variant == DHIT_VARIANT_DEFAULT) {
    launch_dugks_fused(b, src, dst, sums_out);
    return;
  }
  if (b.p.precision == DHIT_FP64)
    dugks_two_pass<double>(b, src, dst, sums_out);
  else
    dugks_two_pass<float>(b, src, dst, sums_out);
}

}  // namespace dhit
