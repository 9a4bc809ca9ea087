// DUGKS time step in one kernel (Sec. II.A), LDS-tiled, marching in z.
//
// Arithmetic.  With B = fbar+ (the cell transform of f~), h = dt/2 and the
// face distribution f_face = alpha fbar_face + beta f^eq_face, the update
//   f~(t+dt) = f~+ - dt sum_d xi_d (f_face(+d) - f_face(-d))
// splits, because fbar_face is linear in B, into
//   f~(t+dt)_q = f~+_q - dt [alpha L_q + beta E_q]
//   L_q = sum_d xi_qd (fbar_face,q(+d) - fbar_face,q(-d))   a fixed stencil of B_q
//   E_q = sum_d xi_qd (f^eq_q(face +d) - f^eq_q(face -d)).
// With the face value (B_L + B_R)/2 - h [xi_d (B_R - B_L) + sum_{t != d}
// xi_t (G_t(L) + G_t(R))/4] and G_t(c) = B(c+e_t) - B(c-e_t):
//   axis population along d, sign s:
//     L = s/2 (B(+d) - B(-d)) - h (B(+d) - 2 B(0) + B(-d))
//   diagonal population in (d1, d2), signs s1, s2:
//     L = s1/2 (B(+d1) - B(-d1)) + s2/2 (B(+d2) - B(-d2))
//         - h (B(+d1) + B(-d1) + B(+d2) + B(-d2) - 4 B(0))
//         - h/2 s1 s2 (B(+d1+d2) - B(+d1-d2) - B(-d1+d2) + B(-d1-d2)).
// The face moments (drho_b = sum fbar_face, j_b = sum xi fbar_face) are the
// same linear reconstruction applied to the cell moment fields of B:
//   R0 = sum B = drho, J = sum xi B = j, P = sum xi xi B
//      = a Pi(f~) + b (drho/3 I + j j / rho0),
// so only 10 moment fields (not 19 populations) are read per face.
//
// Tiling.  A block of 32 x 8 threads owns 32 x 8 (x, y) columns, of which
// the inner 30 x 6 are updated and the outer ring is the halo, and marches
// over a chunk of z.  Each thread keeps the loads of its column's cell two
// planes ahead in flight, computes moments, B and f~+ of the next plane and
// writes the fields its neighbours need to LDS:
//   group A, three-plane ring (z-1, z, z+1): B of the populations moving in
//     z (q5, q6, q11..q18) and Jz, Pxz, Pyz, Pzz;
//   group B, two-plane ring (z, z+1): B of q1..q4, q7..q10 and R0, Jx, Jy,
//     Pxx, Pxy, Pyy.
// The z-face below the centre plane is the z-face above the previous centre
// and is carried in registers, so group B is never needed at z-1.
// HBM traffic per updated cell: 19 loads + 19 stores, plus the halo ring
// (a factor 256/180 on loads, mostly served by the caches).
#include "collision.hpp"

namespace dhit {
namespace fused {

// Column tile of a block: W x 8 columns, the inner (W-2) x 6 updated.
template <int W>
struct Tile {
  static constexpr int TX = W, TY = 8, NT = TX * TY, IX = TX - 2, IY = TY - 2;
};

// Field ids: 0..18 populations of B; moment fields after them.
enum : int { kR0 = 19, kJx, kJy, kJz, kPxx, kPxy, kPxz, kPyy, kPyz, kPzz };
constexpr int kNA = 14, kNB = 14;

constexpr int a_index(int id) {
  switch (id) {
    case 5: return 0;
    case 6: return 1;
    case 11: return 2;
    case 12: return 3;
    case 13: return 4;
    case 14: return 5;
    case 15: return 6;
    case 16: return 7;
    case 17: return 8;
    case 18: return 9;
    case kJz: return 10;
    case kPxz: return 11;
    case kPyz: return 12;
    case kPzz: return 13;
  }
  return -1;
}
constexpr int b_index(int id) {
  switch (id) {
    case 1: return 0;
    case 2: return 1;
    case 3: return 2;
    case 4: return 3;
    case 7: return 4;
    case 8: return 5;
    case 9: return 6;
    case 10: return 7;
    case kR0: return 8;
    case kJx: return 9;
    case kJy: return 10;
    case kPxx: return 11;
    case kPxy: return 12;
    case kPyy: return 13;
  }
  return -1;
}
constexpr int jid(int a) { return kJx + a; }
constexpr int pid(int a, int b) {
  const int lo = a < b ? a : b, hi = a < b ? b : a;
  return lo == 0 ? (hi == 0 ? kPxx : (hi == 1 ? kPxy : kPxz)) : (lo == 1 ? (hi == 1 ? kPyy : kPyz) : kPzz);
}

template <typename Real, int W>
struct Ctx {
  static constexpr int TX = Tile<W>::TX, NT = Tile<W>::NT;
  const Real *A;  // [3][kNA][NT]
  const Real *B;  // [2][kNB][NT]
  int sa[3];      // A slots of planes centre-1, centre, centre+1
  int sb[3];      // B slots of planes centre-1, centre, centre+1 (two are valid at a time)
  int tid;
  template <int ID, int DZ, int DX, int DY>
  __device__ __forceinline__ Real at() const {
    constexpr int ia = a_index(ID), ib = b_index(ID);
    static_assert(ia >= 0 || ib >= 0, "unknown field");
    const int idx = tid + DY * TX + DX;
    if constexpr (ia >= 0)
      return A[(sa[DZ + 1] * kNA + ia) * NT + idx];
    else
      return B[(sb[DZ + 1] * kNB + ib) * NT + idx];
  }
};

template <int T>
struct Unit {
  static constexpr int x = T == 0, y = T == 1, z = T == 2;
};

// Face moments (drho_b, j_b) of the face between L = centre + (LX, LY, LZ)
// and R = L + e_D.
template <int D, int LX, int LY, int LZ, typename Real, int W>
__device__ __forceinline__ void face_moments(const Ctx<Real, W> &c, Real h, Real &rho_b, Real (&jb)[3]) {
  constexpr int RX = LX + Unit<D>::x, RY = LY + Unit<D>::y, RZ = LZ + Unit<D>::z;
  Real tang = Real(0);
  static_for<3>([&](auto t) {
    if constexpr (t != D) {
      constexpr int ex = Unit<t>::x, ey = Unit<t>::y, ez = Unit<t>::z;
      tang += (c.template at<jid(t), LZ + ez, LX + ex, LY + ey>() - c.template at<jid(t), LZ - ez, LX - ex, LY - ey>()) +
              (c.template at<jid(t), RZ + ez, RX + ex, RY + ey>() - c.template at<jid(t), RZ - ez, RX - ex, RY - ey>());
    }
  });
  const Real r0l = c.template at<kR0, LZ, LX, LY>(), r0r = c.template at<kR0, RZ, RX, RY>();
  const Real jdl = c.template at<jid(D), LZ, LX, LY>(), jdr = c.template at<jid(D), RZ, RX, RY>();
  rho_b = (r0l + Real(0.5) * (r0r - r0l)) - h * ((jdr - jdl) + Real(0.25) * tang);
  static_for<3>([&](auto a) {
    Real tg = Real(0);
    static_for<3>([&](auto t) {
      if constexpr (t != D) {
        constexpr int ex = Unit<t>::x, ey = Unit<t>::y, ez = Unit<t>::z;
        constexpr int P = pid(a, t);
        tg += (c.template at<P, LZ + ez, LX + ex, LY + ey>() - c.template at<P, LZ - ez, LX - ex, LY - ey>()) +
              (c.template at<P, RZ + ez, RX + ex, RY + ey>() - c.template at<P, RZ - ez, RX - ex, RY - ey>());
      }
    });
    constexpr int PN = pid(a, D);
    const Real jl = c.template at<jid(a), LZ, LX, LY>(), jr = c.template at<jid(a), RZ, RX, RY>();
    const Real pl = c.template at<PN, LZ, LX, LY>(), pr = c.template at<PN, RZ, RX, RY>();
    jb[a] = (jl + Real(0.5) * (jr - jl)) - h * ((pr - pl) + Real(0.25) * tg);
  });
}

// Index of the population with velocity (x, y, z).
constexpr int pop_of(int x, int y, int z) {
  for (int q = 0; q < kQ; ++q)
    if (kCx[q] == x && kCy[q] == y && kCz[q] == z) return q;
  return -1;
}

// acc_q -= dt beta S xi_qD f^eq_q(face) for the ten populations crossing a
// D-face (the face-equilibrium part of the flux difference, subtracted from
// f~+ as each face is evaluated).  With u = j_b/rho0 and
// f^eq_q = W_q [rho_b - 3/2 rho0 |u|^2 + 3 rho0 (xi.u) + 9/2 rho0 (xi.u)^2],
// opposite velocities share the even part and flip the odd part, so each
// pair is formed from one even and one odd term.
template <int D, int S, typename Real>
__device__ __forceinline__ void sub_face_equilibrium(Real rho_b, const Real (&jb)[3], const StepParams &p, Real dtbe,
                                                     Real (&acc)[kQ]) {
  const Real rho0 = Real(p.rho0), ir = Real(p.inv_rho0);
  const Real u[3] = {jb[0] * ir, jb[1] * ir, jb[2] * ir};
  const Real base = rho_b - Real(1.5) * rho0 * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
  const Real c3 = Real(3) * rho0, c45 = Real(4.5) * rho0;
  const Real k1 = Real(S) * dtbe * Real(1.0 / 18.0), k2 = Real(S) * dtbe * Real(1.0 / 36.0);
  const Real ud = u[D];
  {
    const Real ev = base + c45 * ud * ud, od = c3 * ud;
    constexpr int qp = pop_of(Unit<D>::x, Unit<D>::y, Unit<D>::z);
    constexpr int qm = pop_of(-Unit<D>::x, -Unit<D>::y, -Unit<D>::z);
    acc[qp] -= k1 * (ev + od);   // xi_D = +1
    acc[qm] += k1 * (ev - od);   // xi_D = -1
  }
  static_for<3>([&](auto t) {
    if constexpr (t != D) {
      const Real ut = u[t];
      const Real up = ud + ut, um = ud - ut;
      const Real ep = base + c45 * up * up, op = c3 * up;
      const Real em = base + c45 * um * um, om = c3 * um;
      constexpr int x = Unit<D>::x, y = Unit<D>::y, z = Unit<D>::z;
      constexpr int tx = Unit<t>::x, ty = Unit<t>::y, tz = Unit<t>::z;
      constexpr int q_pp = pop_of(x + tx, y + ty, z + tz);      // xi.u = ud + ut
      constexpr int q_pm = pop_of(x - tx, y - ty, z - tz);      // xi.u = ud - ut
      constexpr int q_mp = pop_of(-x + tx, -y + ty, -z + tz);   // xi.u = -(ud - ut)
      constexpr int q_mm = pop_of(-x - tx, -y - ty, -z - tz);   // xi.u = -(ud + ut)
      acc[q_pp] -= k2 * (ep + op);
      acc[q_pm] -= k2 * (em + om);
      acc[q_mp] += k2 * (em - om);
      acc[q_mm] += k2 * (ep - op);
    }
  });
}

// Linear part L_q of the flux difference (stencil of B_q).
template <int Q, typename Real, int W>
__device__ __forceinline__ Real linear_part(const Ctx<Real, W> &c, Real h) {
  constexpr int sx = kCx[Q], sy = kCy[Q], sz = kCz[Q];
  constexpr int nz = (sx != 0) + (sy != 0) + (sz != 0);
  const Real b0 = c.template at<Q, 0, 0, 0>();
  if constexpr (nz == 1) {
    constexpr int ex = sx != 0, ey = sy != 0, ez = sz != 0;
    constexpr int s = sx + sy + sz;
    const Real bp = c.template at<Q, ez, ex, ey>(), bm = c.template at<Q, -ez, -ex, -ey>();
    return Real(0.5 * s) * (bp - bm) - h * ((bp + bm) - Real(2) * b0);
  } else {
    // the two nonzero directions d1 < d2 with signs s1, s2
    constexpr int d1 = sx != 0 ? 0 : 1;
    constexpr int d2 = sz != 0 ? 2 : 1;
    constexpr int s1 = cdir(Q, d1), s2 = cdir(Q, d2);
    constexpr int x1 = Unit<d1>::x, y1 = Unit<d1>::y, z1 = Unit<d1>::z;
    constexpr int x2 = Unit<d2>::x, y2 = Unit<d2>::y, z2 = Unit<d2>::z;
    const Real p1 = c.template at<Q, z1, x1, y1>(), m1 = c.template at<Q, -z1, -x1, -y1>();
    const Real p2 = c.template at<Q, z2, x2, y2>(), m2 = c.template at<Q, -z2, -x2, -y2>();
    const Real pp = c.template at<Q, z1 + z2, x1 + x2, y1 + y2>();
    const Real pm = c.template at<Q, z1 - z2, x1 - x2, y1 - y2>();
    const Real mp = c.template at<Q, -z1 + z2, -x1 + x2, -y1 + y2>();
    const Real mm = c.template at<Q, -z1 - z2, -x1 - x2, -y1 - y2>();
    return (Real(0.5 * s1) * (p1 - m1) + Real(0.5 * s2) * (p2 - m2)) -
           h * (((p1 + m1) + (p2 + m2)) - Real(4) * b0) - Real(0.5 * s1 * s2) * h * (((pp - pm) - mp) + mm);
  }
}

// Issues the loads of the 19 f~ of the column's cell in plane `plane`
// (periodic in z).  The values are consumed one loop iteration later, so the
// loads overlap the work on the centre plane.
template <typename Real>
__device__ __forceinline__ void load_raw(const Real *__restrict__ ft, int64_t stride, int n, int col, int plane,
                                         Real (&f)[kQ]) {
  const int z = plane < 0 ? plane + n : (plane >= n ? plane - n : plane);
  const int cell = z * n * n + col;
  static_for<kQ>([&](auto q) { f[q] = ft[(int64_t)q * stride + cell]; });
}

// From the 19 f~ of a cell: moments, B = a f~ + b f^eq, the moment fields of
// B; writes the fields its neighbours need to the LDS slots (sa, sb) and
// returns f~+ = 4/3 B - 1/3 f~.
template <typename Real, int W>
__device__ __forceinline__ void publish_cell(const Real (&f)[kQ], int sa, int sb, Real *A, Real *B, int tid,
                                             const StepParams &p, Real (&ftp)[kQ]) {
  constexpr int NT = Tile<W>::NT;
  Real drho, jx, jy, jz, feq[kQ];
  cell_moments<Real>(f, drho, jx, jy, jz);
  equilibrium<Real>(drho, jx, jy, jz, Real(p.rho0), Real(p.inv_rho0), feq);
  // second moments of f~
  Real pxx = 0, pyy = 0, pzz = 0, pxy = 0, pxz = 0, pyz = 0;
  static_for<kQ>([&](auto q) {
    constexpr int x = kCx[q], y = kCy[q], z = kCz[q];
    if constexpr (x != 0) pxx += f[q];
    if constexpr (y != 0) pyy += f[q];
    if constexpr (z != 0) pzz += f[q];
    if constexpr (x * y == 1) pxy += f[q];
    if constexpr (x * y == -1) pxy -= f[q];
    if constexpr (x * z == 1) pxz += f[q];
    if constexpr (x * z == -1) pxz -= f[q];
    if constexpr (y * z == 1) pyz += f[q];
    if constexpr (y * z == -1) pyz -= f[q];
  });
  // B = a f~ + b f^eq with a + b = 1 is formed as f^eq + a (f~ - f^eq) and
  // f~+ = 4/3 B - 1/3 f~ as B + (B - f~)/3, so that an equilibrium cell maps
  // to itself exactly in any precision (rounded 4/3 and 1/3, or a and b,
  // would otherwise scale the state by 1 + O(ulp) every step)
  const Real a = Real(p.a_bp);
  const Real ir = Real(p.inv_rho0);
  const Real d3 = drho * Real(1.0 / 3.0);
  Real fld[29];
  static_for<kQ>([&](auto q) {
    const Real bp = feq[q] + a * (f[q] - feq[q]);
    fld[q] = bp;
    ftp[q] = bp + (bp - f[q]) * Real(1.0 / 3.0);
  });
  fld[kR0] = drho;
  fld[kJx] = jx;
  fld[kJy] = jy;
  fld[kJz] = jz;
  // P = a Pi(f~) + b Pi(f^eq), Pi(f^eq) = drho/3 I + j j / rho0, in the same form
  const Real exx = d3 + jx * jx * ir, eyy = d3 + jy * jy * ir, ezz = d3 + jz * jz * ir;
  const Real exy = jx * jy * ir, exz = jx * jz * ir, eyz = jy * jz * ir;
  fld[kPxx] = exx + a * (pxx - exx);
  fld[kPyy] = eyy + a * (pyy - eyy);
  fld[kPzz] = ezz + a * (pzz - ezz);
  fld[kPxy] = exy + a * (pxy - exy);
  fld[kPxz] = exz + a * (pxz - exz);
  fld[kPyz] = eyz + a * (pyz - eyz);
  static_for<29>([&](auto id) {
    constexpr int ia = a_index(id), ib = b_index(id);
    if constexpr (ia >= 0) A[(sa * kNA + ia) * NT + tid] = fld[id];
    if constexpr (ib >= 0) B[(sb * kNB + ib) * NT + tid] = fld[id];
  });
}

// The z-march of one tile (bx, by) over the z-chunk bz of a box; adds the
// moments of the updated cells to v.  A and B are the block's LDS rings.
template <typename Real, int W>
__device__ __forceinline__ void fused_tile(const Real *__restrict__ ft, Real *__restrict__ out, const StepParams &p,
                                           int bx, int by, int bz, int nz_chunk, Real *A, Real *B,
                                           double (&v)[kNumSums]) {
  constexpr int TX = Tile<W>::TX, TY = Tile<W>::TY, IX = Tile<W>::IX, IY = Tile<W>::IY;
  const int n = p.n;
  const int64_t stride = p.stride;
  const int tid = threadIdx.x;
  const int tx = tid % TX, ty = tid / TX;
  const int x0 = bx * IX, y0 = by * IY, z0 = bz * nz_chunk;
  const int z1 = min(z0 + nz_chunk, n);
  int gx = x0 - 1 + tx, gy = y0 - 1 + ty;
  gx = gx < 0 ? gx + n : (gx >= n ? gx % n : gx);
  gy = gy < 0 ? gy + n : (gy >= n ? gy % n : gy);
  const int col = gy * n + gx;
  const bool inner = tx >= 1 && tx <= TX - 2 && ty >= 1 && ty <= TY - 2 && (x0 + tx - 1) < n && (y0 + ty - 1) < n;
  const Real h = Real(p.h), dt = Real(p.dt);
  const Real dtal = dt * Real(p.alpha), dtbe = dt * Real(p.beta);

  auto slot3 = [](int z) { return (z + 3) % 3; };
  auto slot2 = [](int z) { return (z + 2) % 2; };

  Real pf[kQ], acc[kQ], ftp_next[kQ];
  Real rho_zm = Real(0), jzm[3] = {Real(0), Real(0), Real(0)};

  // prologue: planes z0-1 and z0 published, plane z0+1 in flight, and the
  // z-face between z0-1 and z0
  load_raw<Real>(ft, stride, n, col, z0 - 1, pf);
  publish_cell<Real, W>(pf, slot3(z0 - 1), slot2(z0 - 1), A, B, tid, p, acc);
  load_raw<Real>(ft, stride, n, col, z0, pf);
  publish_cell<Real, W>(pf, slot3(z0), slot2(z0), A, B, tid, p, acc);
  load_raw<Real>(ft, stride, n, col, z0 + 1, pf);
  __syncthreads();
  {
    Ctx<Real, W> c{A, B, {slot3(z0 - 1), slot3(z0), slot3(z0 + 1)}, {slot2(z0 - 1), slot2(z0), slot2(z0 + 1)}, tid};
    if (inner && z0 < z1) face_moments<2, 0, 0, -1, Real>(c, h, rho_zm, jzm);
  }
  __syncthreads();

  for (int z = z0; z < z1; ++z) {
    // acc holds f~+ of the centre plane z; publish plane z+1, prefetch z+2
    publish_cell<Real, W>(pf, slot3(z + 1), slot2(z + 1), A, B, tid, p, ftp_next);
    if (z + 1 < z1) load_raw<Real>(ft, stride, n, col, z + 2, pf);
    __syncthreads();
    if (inner) {
      Ctx<Real, W> c{A, B, {slot3(z - 1), slot3(z), slot3(z + 1)}, {slot2(z - 1), slot2(z), slot2(z + 1)}, tid};
      {
        Real rb, jb[3];
        face_moments<0, 0, 0, 0, Real>(c, h, rb, jb);
        sub_face_equilibrium<0, 1, Real>(rb, jb, p, dtbe, acc);
        face_moments<0, -1, 0, 0, Real>(c, h, rb, jb);
        sub_face_equilibrium<0, -1, Real>(rb, jb, p, dtbe, acc);
        face_moments<1, 0, 0, 0, Real>(c, h, rb, jb);
        sub_face_equilibrium<1, 1, Real>(rb, jb, p, dtbe, acc);
        face_moments<1, 0, -1, 0, Real>(c, h, rb, jb);
        sub_face_equilibrium<1, -1, Real>(rb, jb, p, dtbe, acc);
        sub_face_equilibrium<2, -1, Real>(rho_zm, jzm, p, dtbe, acc);
        face_moments<2, 0, 0, 0, Real>(c, h, rho_zm, jzm);  // the z-face above, carried to the next plane
        sub_face_equilibrium<2, 1, Real>(rho_zm, jzm, p, dtbe, acc);
      }
      static_for<kQ>([&](auto q) {
        if constexpr (q != 0) acc[q] -= dtal * linear_part<q, Real>(c, h);
      });
      const int cell = z * n * n + col;
      static_for<kQ>([&](auto q) { __builtin_nontemporal_store(acc[q], &out[(int64_t)q * stride + cell]); });
      sums_of_populations<Real>(acc, p.inv_rho0, v);
    }
    static_for<kQ>([&](auto q) { acc[q] = ftp_next[q]; });
    __syncthreads();
  }
}

template <typename Real, int W>
__global__ __launch_bounds__(Tile<W>::NT) void dugks_fused_kernel(const Real *__restrict__ ft, Real *__restrict__ out,
                                                                  StepParams p, int tiles_x, int tiles_y,
                                                                  int nz_chunk, double *__restrict__ partials) {
  __shared__ Real A[3 * kNA * Tile<W>::NT];
  __shared__ Real B[2 * kNB * Tile<W>::NT];
  const int bx = blockIdx.x % tiles_x;
  const int by = (blockIdx.x / tiles_x) % tiles_y;
  const int bz = blockIdx.x / (tiles_x * tiles_y);
  double v[kNumSums] = {0, 0, 0, 0, 0};
  fused_tile<Real, W>(ft, out, p, bx, by, bz, nz_chunk, A, B, v);
  write_block_partials(v, partials, gridDim.x, blockIdx.x);
}

// Many boxes in one persistent launch: work item = one tile z-chunk of one
// box, numbered as the blocks of that box's single-box launch.
template <typename Real, int W>
__global__ __launch_bounds__(Tile<W>::NT) void dugks_batch_kernel(BatchBox *__restrict__ boxes, int nbox,
                                                                  int total_items) {
  __shared__ Real A[3 * kNA * Tile<W>::NT];
  __shared__ Real B[2 * kNB * Tile<W>::NT];
  for (int it = blockIdx.x; it < total_items; it += gridDim.x) {
    const int b = find_batch_box(boxes, nbox, it);
    const BatchBox &d = boxes[b];
    const int local = it - d.item_begin;
    const int bx = local % d.tiles_x;
    const int by = (local / d.tiles_x) % d.tiles_y;
    const int bz = local / (d.tiles_x * d.tiles_y);
    double v[kNumSums] = {0, 0, 0, 0, 0};
    fused_tile<Real, W>(static_cast<const Real *>(d.f[d.cur]), static_cast<Real *>(d.f[d.cur ^ 1]), d.sp, bx, by, bz,
                        d.nz_chunk, A, B, v);
    write_block_partials(v, d.partials, d.items, local);
    __syncthreads();
  }
}

}  // namespace fused

// Default tile width by precision: FP64 tiles of 16 x 8 columns use 72 KB of
// LDS, so two blocks share a compute unit; FP32 tiles of 32 x 8 use 72 KB too.
constexpr int fused_tile_width(int precision) { return precision == DHIT_FP64 ? 16 : 32; }

int fused_default_chunk(int n) { return n >= 128 ? 32 : (n >= 32 ? 16 : n); }

int fused_dugks_items(int n, int precision, int chunk, int *tiles_x, int *tiles_y) {
  const int ix = fused_tile_width(precision) - 2, iy = 8 - 2;
  const int tx = (n + ix - 1) / ix;
  const int ty = (n + iy - 1) / iy;
  if (tiles_x) *tiles_x = tx;
  if (tiles_y) *tiles_y = ty;
  return tx * ty * ((n + chunk - 1) / chunk);
}

// Blocks of a single-box fused launch with the box's tile width and z-chunk.
int fused_dugks_blocks(const dhit_params &p, int *width, int *tiles_x, int *tiles_y, int *nz_chunk) {
  const int n = p.n;
  const int w = p.tile_width ? p.tile_width : fused_tile_width(p.precision);
  const int ix = w - 2, iy = 8 - 2;
  const int tx = (n + ix - 1) / ix;
  const int ty = (n + iy - 1) / iy;
  const int cz = p.z_chunk ? p.z_chunk : fused_default_chunk(n);
  const int nzc = (n + cz - 1) / cz;
  if (width) *width = w;
  if (tiles_x) *tiles_x = tx;
  if (tiles_y) *tiles_y = ty;
  if (nz_chunk) *nz_chunk = cz;
  return tx * ty * nzc;
}

template <typename Real, int W>
static void fused_launch(dhit_box &b, const void *src, void *dst, int blocks, int tx, int ty, int cz) {
  hipLaunchKernelGGL((fused::dugks_fused_kernel<Real, W>), dim3(blocks), dim3(fused::Tile<W>::NT), 0, b.stream,
                     static_cast<const Real *>(src), static_cast<Real *>(dst), b.sp, tx, ty, cz, b.partials);
}

template <typename Real>
static void fused_step(dhit_box &b, const void *src, void *dst, double *sums_out) {
  int w, tx, ty, cz;
  const int blocks = fused_dugks_blocks(b.p, &w, &tx, &ty, &cz);
  {
    TimedLaunch t(b, DHIT_K_DUGKS_FUSED);
    if (w == 16)
      fused_launch<Real, 16>(b, src, dst, blocks, tx, ty, cz);
    else
      fused_launch<Real, 32>(b, src, dst, blocks, tx, ty, cz);
    DHIT_HIP(hipGetLastError());
    t.done();
  }
  launch_finalize_sums(b, b.partials, blocks, sums_out);
}

int fused_tile_width_of(int precision) { return fused_tile_width(precision); }

void launch_dugks_batch(hipStream_t s, int precision, BatchBox *d_boxes, int nbox, int total_items, int grid) {
  if (precision == DHIT_FP64) {
    constexpr int W = fused_tile_width(DHIT_FP64);
    hipLaunchKernelGGL((fused::dugks_batch_kernel<double, W>), dim3(grid), dim3(fused::Tile<W>::NT), 0, s, d_boxes,
                       nbox, total_items);
  } else {
    constexpr int W = fused_tile_width(DHIT_FP32);
    hipLaunchKernelGGL((fused::dugks_batch_kernel<float, W>), dim3(grid), dim3(fused::Tile<W>::NT), 0, s, d_boxes,
                       nbox, total_items);
  }
  DHIT_HIP(hipGetLastError());
}

void launch_dugks_fused(dhit_box &b, const void *src, void *dst, double *sums_out) {
  if (b.p.precision == DHIT_FP64)
    fused_step<double>(b, src, dst, sums_out);
  else
    fused_step<float>(b, src, dst, sums_out);
}

}  // namespace dhit
