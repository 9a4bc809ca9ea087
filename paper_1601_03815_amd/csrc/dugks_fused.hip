// DUGKS time step in one kernel (Sec. II.A), marching in z with one plane
// of cell data in LDS at a time.
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
// Plane-by-plane evaluation.  Every term above is a sum of pieces that each
// involve one z-plane only (a plane's own cell and its in-plane
// neighbours).  When plane p is in LDS, each thread adds the pieces of
// plane p to the three centres that use it:
//   centre p-1 (p is its z+1 plane): the z+1 terms of the z-moving
//     populations and the upper half of the face between p-1 and p;
//   centre p: the in-plane terms of the populations and the lower half of
//     the face between p and p+1;
//   centre p+1 (p is its z-1 plane): the z-1 terms of the z-moving
//     populations.
// The x- and y-faces of centre p-1 are formed in the same iteration from
// the moment fields of planes p-2, p-1 and p, after which centre p-1 is
// complete and stored.  Each in-plane face is formed once, by one of its two
// cells, and handed to the other: across lanes for the x-faces (a tile row
// is 32 consecutive lanes) and through LDS for the y-faces (in the FP32
// march the upper cell applies it, and is stored, after the barrier that
// ends the iteration).  Between planes a thread carries the running
// results of centres p and p+1 in registers.  LDS holds the populations of
// plane p only, the in-plane moment fields (R0, Jx, Jy, Pxx, Pxy, Pyy) of
// planes p-1 and p, and the fields the x/y-faces differentiate in z (Jz,
// Pxz, Pyz, Pzz) of planes p-2, p-1 and p: 16 + 12 + 12 values per column.
//
// Two marches implement this.  fused_tile (FP32): one thread per column,
// 44 values of LDS per column (44 KB for a 32 x 8 tile, two blocks per
// compute unit).  split_tile (FP64): two threads per column, one in each of
// two groups that hold about half of the populations each (see below), so
// that a thread's registers fit two waves per SIMD; 70 values per column.
// LDS reads are gathered (see gathered()) so that each chunk of work waits
// for LDS once.
//
// Tiling.  A block owns W x 8 (x, y) columns, of which the inner (W-2) x 6
// are updated and the outer ring is the halo, and marches over a chunk of
// z.  HBM traffic per updated cell: 19 loads + 19 stores, plus the halo
// ring (loads only).  Blocks are numbered so that the tiles one XCD (one L2)
// works on at a time are neighbours, whose halo columns then come from that
// L2.
#include <array>
#include <cstring>
#include <map>
#include <mutex>

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

// LDS buffers: populations (one plane) other than 0, 5, 6 (the rest
// population has no stencil, q5 and q6 only use their own column); the
// in-plane moment fields (two planes); the fields differentiated in z
// across x/y-faces (three planes).
constexpr int kNPop = 16, kNQ = 6, kNZ = 4;
constexpr int kLdsValues = kNPop + 2 * kNQ + 3 * kNZ;  // per column
// The one-thread march adds the ten face-equilibrium terms of the y-face
// between each column and the next row (read back by the column above as
// its lower y-face).
constexpr int kFusedValues = kLdsValues + 10;
constexpr int pop_index(int id) { return (id >= 1 && id <= 4) ? id - 1 : ((id >= 7 && id <= 18) ? id - 3 : -1); }
constexpr int q_index(int id) {
  switch (id) {
    case kR0: return 0;
    case kJx: return 1;
    case kJy: return 2;
    case kPxx: return 3;
    case kPxy: return 4;
    case kPyy: return 5;
  }
  return -1;
}
constexpr int z_index(int id) {
  switch (id) {
    case kJz: return 0;
    case kPxz: return 1;
    case kPyz: return 2;
    case kPzz: return 3;
  }
  return -1;
}
constexpr int jid(int a) { return kJx + a; }
constexpr int pid(int a, int b) {
  const int lo = a < b ? a : b, hi = a < b ? b : a;
  return lo == 0 ? (hi == 0 ? kPxx : (hi == 1 ? kPxy : kPxz)) : (lo == 1 ? (hi == 1 ? kPyy : kPyz) : kPzz);
}
// Position of a z-moving population among the ten (q5, q6, q11..q18).
constexpr int zslot(int q) { return q == 5 ? 0 : (q == 6 ? 1 : q - 9); }
constexpr bool is_diag_z(int q) { return q >= 11; }

// Column of the tile (row-major, ty * W + tx) that thread t of a march
// handles.  In the 32-wide tile a wavefront covers two rows; the two rows
// made only of halo columns (0 and 7) are put together in the last
// wavefront, so that the work of the updated cells (stencils, faces,
// stores), which halo rows skip, runs on three wavefronts instead of four:
// wavefronts 0..2 take rows (1, 2), (3, 4), (5, 6) and wavefront 3 rows 0
// and 7.  A row stays 32 consecutive lanes, as the x-face lane shift needs.
// Other widths keep row-major order.
template <int W>
__device__ __forceinline__ int tile_column(int t) {
  if constexpr (W == 32) {
    const int w = t >> 6, half = (t >> 5) & 1, tx = t & 31;
    const int ty = w < 3 ? 2 * w + 1 + half : (half ? 7 : 0);
    return ty * 32 + tx;
  } else {
    return t;
  }
}

// Compiler-only memory fence between the phases of a plane's work: LDS
// values are re-read after it instead of being kept live in registers
// across phases, which bounds register pressure.  No instruction is emitted.
__device__ __forceinline__ void phase() { asm volatile("" ::: "memory"); }

template <int T>
struct Unit {
  static constexpr int x = T == 0, y = T == 1, z = T == 2;
};

// Value of the previous lane of the wavefront (lane 0 gets 0): a DPP
// whole-wavefront shift right by one lane, one move per 32 bits.
__device__ __forceinline__ int from_previous_lane(int v) { return __builtin_amdgcn_update_dpp(0, v, 0x138, 0xf, 0xf, false); }
__device__ __forceinline__ float from_previous_lane(float v) {
  return __builtin_bit_cast(float, from_previous_lane(__builtin_bit_cast(int, v)));
}
__device__ __forceinline__ double from_previous_lane(double v) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = from_previous_lane((int)b), hi = from_previous_lane((int)(b >> 32));
  return __builtin_bit_cast(double, ((long long)hi << 32) | (long long)(unsigned)lo);
}

// Reads of one plane: populations from P, in-plane moment fields from Q,
// z-differentiated fields from Z (each offset to the thread's column; a
// plane whose populations or Q fields are no longer held has null there).
template <typename Real, int W>
struct Plane {
  const Real *P;
  const Real *Q;
  const Real *Z;
  template <int ID, int DX, int DY>
  __device__ __forceinline__ Real at() const {
    constexpr int NT = Tile<W>::NT, off = DY * W + DX;
    constexpr int ip = pop_index(ID), iq = q_index(ID), iz = z_index(ID);
    static_assert(ip >= 0 || iq >= 0 || iz >= 0, "field not in LDS");
    if constexpr (ip >= 0)
      return P[ip * NT + off];
    else if constexpr (iq >= 0)
      return Q[iq * NT + off];
    else
      return Z[iz * NT + off];
  }
};

// In-plane central difference of field ID along in-plane axis t (0 or 1)
// at the column offset (DX, DY).
template <int ID, int T, int DX, int DY, class P>
__device__ __forceinline__ auto dif(const P &c) {
  return c.template at<ID, DX + Unit<T>::x, DY + Unit<T>::y>() - c.template at<ID, DX - Unit<T>::x, DY - Unit<T>::y>();
}

// Reads gathered ahead of their use.  A computation written against a
// plane is run twice: once on a Load view, which issues every LDS read the
// computation makes (its arithmetic is discarded), then on a Use view, which
// replays it on the gathered values.  All reads of a chunk of work are thus
// in flight together and their latencies overlap, instead of one read being
// waited for before the next is issued.
constexpr int kNumIds = 29;
template <typename Real>
struct Gathered {
  Real v[kNumIds][3][3];  // field id, dy + 1, dx + 1
};
template <typename Real, int W, bool kLoad>
struct GView {
  static constexpr bool use = !kLoad;
  const Plane<Real, W> &src;
  Gathered<Real> &g;
  template <int ID, int DX, int DY>
  __device__ __forceinline__ Real at() const {
    if constexpr (kLoad) {
      g.v[ID][DY + 1][DX + 1] = src.template at<ID, DX, DY>();
      return Real(0);
    } else {
      return g.v[ID][DY + 1][DX + 1];
    }
  }
};
// f(view0, view1) with views of planes c0 and c1; f must change state only
// when view0.use is true.
template <typename Real, int W, class F>
__device__ __forceinline__ void gathered(const Plane<Real, W> &c0, const Plane<Real, W> &c1, F &&f) {
  Gathered<Real> g0, g1;
  f(GView<Real, W, true>{c0, g0}, GView<Real, W, true>{c1, g1});
  __builtin_amdgcn_sched_barrier(0);
  f(GView<Real, W, false>{c0, g0}, GView<Real, W, false>{c1, g1});
  phase();
}

// In-plane part of the moments of the D-face (D = 0 or 1) between
// L = (LX, LY) and R = L + e_D in the current plane: everything but the
// z-tangential gradients.  Face moment of field pair (value field V,
// normal-flux field N, in-plane tangential field T):
//   V_L + (V_R - V_L)/2 - h [(N_R - N_L) + (T(L+e_t) - T(L-e_t) + T(R+e_t) - T(R-e_t))/4]
template <int D, int LX, int LY, typename Real, class P>
__device__ __forceinline__ void face_inplane(const P &c, Real h, Real (&m)[4]) {
  constexpr int t = 1 - D;
  constexpr int RX = LX + Unit<D>::x, RY = LY + Unit<D>::y;
  {
    const Real tang = dif<jid(t), t, LX, LY>(c) + dif<jid(t), t, RX, RY>(c);
    const Real vl = c.template at<kR0, LX, LY>(), vr = c.template at<kR0, RX, RY>();
    const Real nl = c.template at<jid(D), LX, LY>(), nr = c.template at<jid(D), RX, RY>();
    m[0] = (vl + Real(0.5) * (vr - vl)) - h * ((nr - nl) + Real(0.25) * tang);
  }
  static_for<3>([&](auto a) {
    constexpr int PN = pid(a, D), PT = pid(a, t);
    const Real tang = dif<PT, t, LX, LY>(c) + dif<PT, t, RX, RY>(c);
    const Real vl = c.template at<jid(a), LX, LY>(), vr = c.template at<jid(a), RX, RY>();
    const Real nl = c.template at<PN, LX, LY>(), nr = c.template at<PN, RX, RY>();
    m[1 + a] = (vl + Real(0.5) * (vr - vl)) - h * ((nr - nl) + Real(0.25) * tang);
  });
}

// z-tangential part of an x/y-face moment pair sum: for the face between
// L = (LX, LY) and R, the fields (Jz, Pxz, Pyz, Pzz) summed over L and R.
template <int D, int LX, int LY, typename Real, class P>
__device__ __forceinline__ void face_zsum(const P &c, Real (&s)[4]) {
  constexpr int RX = LX + Unit<D>::x, RY = LY + Unit<D>::y;
  s[0] = c.template at<kJz, LX, LY>() + c.template at<kJz, RX, RY>();
  s[1] = c.template at<kPxz, LX, LY>() + c.template at<kPxz, RX, RY>();
  s[2] = c.template at<kPyz, LX, LY>() + c.template at<kPyz, RX, RY>();
  s[3] = c.template at<kPzz, LX, LY>() + c.template at<kPzz, RX, RY>();
}

// Half of the moments of a z-face that comes from one plane (the cell of
// the column and its in-plane neighbours).  For the plane below the face
// (S = +1) and the plane above it (S = -1):
//   R0/2 + S h Jz - h/4 (dJx/dx + dJy/dy) and, for component a,
//   J_a/2 + S h P_az - h/4 (dP_ax/dx + dP_ay/dy)   (central differences).
template <int S, typename Real, class P>
__device__ __forceinline__ void zface_half(const P &c, Real h, Real (&m)[4]) {
  {
    const Real tang = dif<kJx, 0, 0, 0>(c) + dif<kJy, 1, 0, 0>(c);
    m[0] = Real(0.5) * c.template at<kR0, 0, 0>() + Real(S) * h * c.template at<kJz, 0, 0>() - Real(0.25) * h * tang;
  }
  static_for<3>([&](auto a) {
    const Real tang = dif<pid(a, 0), 0, 0, 0>(c) + dif<pid(a, 1), 1, 0, 0>(c);
    m[1 + a] = Real(0.5) * c.template at<jid(a), 0, 0>() + Real(S) * h * c.template at<pid(a, 2), 0, 0>() -
               Real(0.25) * h * tang;
  });
}

// Index of the population with velocity (x, y, z).
constexpr int pop_of(int x, int y, int z) {
  for (int q = 0; q < kQ; ++q)
    if (kCx[q] == x && kCy[q] == y && kCz[q] == z) return q;
  return -1;
}

// Face-equilibrium terms of a D-face: calls put(q, v) for the ten
// populations crossing it, v = dt beta xi_qD f^eq_q(face).  With
// u = j_b/rho0 and f^eq_q = W_q [rho_b - 3/2 rho0 |u|^2 + 3 rho0 (xi.u)
// + 9/2 rho0 (xi.u)^2], opposite velocities share the even part and flip
// the odd part, so each pair is formed from one even and one odd term.
template <int D, typename Real, class Put>
__device__ __forceinline__ void face_equilibrium(const Real (&m)[4], const StepParams &p, Real dtbe, Put &&put) {
  const Real rho0 = Real(p.rho0), ir = Real(p.inv_rho0);
  const Real u[3] = {m[1] * ir, m[2] * ir, m[3] * ir};
  const Real base = m[0] - Real(1.5) * rho0 * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
  const Real c3 = Real(3) * rho0, c45 = Real(4.5) * rho0;
  const Real k1 = dtbe * Real(1.0 / 18.0), k2 = dtbe * Real(1.0 / 36.0);
  const Real ud = u[D];
  {
    const Real ev = base + c45 * ud * ud, od = c3 * ud;
    put(std::integral_constant<int, pop_of(Unit<D>::x, Unit<D>::y, Unit<D>::z)>{}, k1 * (ev + od));
    put(std::integral_constant<int, pop_of(-Unit<D>::x, -Unit<D>::y, -Unit<D>::z)>{}, -(k1 * (ev - od)));
  }
  static_for<3>([&](auto t) {
    if constexpr (t != D) {
      const Real ut = u[t];
      const Real up = ud + ut, um = ud - ut;
      const Real ep = base + c45 * up * up, op = c3 * up;
      const Real em = base + c45 * um * um, om = c3 * um;
      constexpr int x = Unit<D>::x, y = Unit<D>::y, z = Unit<D>::z;
      constexpr int tx = Unit<t>::x, ty = Unit<t>::y, tz = Unit<t>::z;
      put(std::integral_constant<int, pop_of(x + tx, y + ty, z + tz)>{}, k2 * (ep + op));      // xi.u = ud + ut
      put(std::integral_constant<int, pop_of(x - tx, y - ty, z - tz)>{}, k2 * (em + om));      // xi.u = ud - ut
      put(std::integral_constant<int, pop_of(-x + tx, -y + ty, -z + tz)>{}, -(k2 * (em - om)));  // -(ud - ut)
      put(std::integral_constant<int, pop_of(-x - tx, -y - ty, -z - tz)>{}, -(k2 * (ep - op)));  // -(ud + ut)
    }
  });
}

// Slot of population q among the ten that cross a D-face (increasing q).
template <int D>
constexpr int cross_slot(int q) {
  int k = 0;
  for (int r = 0; r < q; ++r) k += cdir(r, D) != 0;
  return k;
}

// The ten face-equilibrium terms of a D-face, v[cross_slot<D>(q)] =
// dt beta xi_qD f^eq_q(face) (face_equilibrium), formed once for both of the
// face's cells.
template <int D, typename Real>
__device__ __forceinline__ void face_terms(const Real (&m)[4], const StepParams &p, Real dtbe, Real (&v)[10]) {
  face_equilibrium<D, Real>(m, p, dtbe, [&](auto q, Real val) { v[cross_slot<D>(q)] = val; });
}

// acc_q -= S v_q for the face terms of a D-face (S = +1: the centre's upper
// face, -1: its lower face).
template <int D, int S, typename Real>
__device__ __forceinline__ void apply_terms(const Real (&v)[10], Real (&acc)[kQ]) {
  static_for<kQ>([&](auto q) {
    if constexpr (cdir(q, D) != 0) {
      if constexpr (S > 0)
        acc[q] -= v[cross_slot<D>(q)];
      else
        acc[q] += v[cross_slot<D>(q)];
    }
  });
}

// acc_q -= S v_q for the populations crossing a D-face of the centre
// (S = +1 for its upper face, -1 for its lower face).
template <int D, int S, typename Real>
__device__ __forceinline__ void sub_face(const Real (&m)[4], const StepParams &p, Real dtbe, Real (&acc)[kQ]) {
  face_equilibrium<D, Real>(m, p, dtbe, [&](auto q, Real v) {
    if constexpr (S > 0)
      acc[q] -= v;
    else
      acc[q] += v;
  });
}

// Cell idx of the population array that starts at qbase.  With O32 the
// byte offset is formed in 32 bits (every population array of the box is
// below 4 GB), so that the access can go through the array's uniform base
// in scalar registers with a 32-bit lane offset, with no 64-bit address
// arithmetic per access.
template <bool O32, typename T>
__device__ __forceinline__ T *at_cell(T *qbase, int idx) {
  if constexpr (O32) {
    using Byte = std::conditional_t<std::is_const<T>::value, const global_t<char>, global_t<char>>;
    return reinterpret_cast<T *>(reinterpret_cast<Byte *>(qbase) + (uint32_t)idx * (uint32_t)sizeof(T));
  } else {
    return qbase + idx;
  }
}

// Issues the loads of the 19 f~ of the column's cell in plane `plane`
// (periodic in z).
template <typename Real, bool O32>
__device__ __forceinline__ void load_raw(const global_t<Real> *__restrict__ ft, int64_t stride, int n, int col, int plane,
                                         Real (&f)[kQ]) {
  const int z = plane < 0 ? plane + n : (plane >= n ? plane - n : plane);
  const int idx = z * n * n + col;
  static_for<kQ>([&](auto q) { f[q] = *at_cell<O32>(ft + (int64_t)q * stride, idx); });
}

// The ten moments drho, j, Pi of a cell (or of the populations get(q)
// yields for q in a set closed under q -> -q), formed from opposite-velocity
// pairs: with s = f_q + f_-q and d = f_q - f_-q over the pairs (q < -q),
//   drho = f_0 + sum s,  j = sum xi_q d,  Pi_ab = sum xi_qa xi_qb s.
// FP32: drho and j are compensated sums over the pair terms.
// m = {drho, jx, jy, jz, Pxx, Pyy, Pzz, Pxy, Pxz, Pyz}.
template <typename Real, class Has, class Get>
__device__ __forceinline__ void pair_moments(Has has, Get get, Real (&m)[10]) {
  CompSum<Real> r, ax, ay, az;
  Real pxx = 0, pyy = 0, pzz = 0, pxy = 0, pxz = 0, pyz = 0;
  constexpr bool plain = std::is_same<Real, double>::value;
  auto acc = [&](CompSum<Real> &c, Real x) {
    if constexpr (plain)
      c.s += x;
    else
      c.add(x);
  };
  if constexpr (has(0)) acc(r, get(std::integral_constant<int, 0>{}));
  static_for<kQ>([&](auto q) {
    constexpr int qb = opposite(q);
    if constexpr (q != 0 && q < qb && has(q)) {
      const Real fq = get(q), fb = get(std::integral_constant<int, qb>{});
      const Real sm = fq + fb, df = fq - fb;
      constexpr int x = kCx[q], y = kCy[q], z = kCz[q];
      acc(r, sm);
      if constexpr (x != 0) acc(ax, x > 0 ? df : -df);
      if constexpr (y != 0) acc(ay, y > 0 ? df : -df);
      if constexpr (z != 0) acc(az, z > 0 ? df : -df);
      if constexpr (x != 0) pxx += sm;
      if constexpr (y != 0) pyy += sm;
      if constexpr (z != 0) pzz += sm;
      if constexpr (x * y == 1) pxy += sm;
      if constexpr (x * y == -1) pxy -= sm;
      if constexpr (x * z == 1) pxz += sm;
      if constexpr (x * z == -1) pxz -= sm;
      if constexpr (y * z == 1) pyz += sm;
      if constexpr (y * z == -1) pyz -= sm;
    }
  });
  m[0] = r.value(); m[1] = ax.value(); m[2] = ay.value(); m[3] = az.value();
  m[4] = pxx; m[5] = pyy; m[6] = pzz; m[7] = pxy; m[8] = pxz; m[9] = pyz;
}

// From the 19 f~ of a cell: moments, B = a f~ + b f^eq and f~+ =
// 4/3 B - 1/3 f~, and the moment fields of B; writes the fields other
// columns read to the plane's LDS buffers P, Q, Z (offset to the thread's
// column) and hands each population's (B, f~+) to
// use(q, B_q, f~+_q) as soon as it is formed.
template <typename Real, int W, class Use>
__device__ __forceinline__ void publish_cell(const Real (&f)[kQ], Real *P, Real *Q, Real *Z, const StepParams &p,
                                             Use &&use) {
  constexpr int NT = Tile<W>::NT;
  Real mom[10];
  pair_moments<Real>([](int) constexpr { return true; }, [&](auto q) { return f[q]; }, mom);
  const Real drho = mom[0], jx = mom[1], jy = mom[2], jz = mom[3];
  const Real pxx = mom[4], pyy = mom[5], pzz = mom[6], pxy = mom[7], pxz = mom[8], pyz = mom[9];
  const Real rho0 = Real(p.rho0), ir = Real(p.inv_rho0);
  const Real a = Real(p.a_bp);
  const Real d3 = drho * Real(1.0 / 3.0);
  // P = a Pi(f~) + b Pi(f^eq), Pi(f^eq) = drho/3 I + j j / rho0, formed as
  // Pi(f^eq) + a (Pi(f~) - Pi(f^eq)) (see below)
  {
    const Real exx = d3 + jx * jx * ir, eyy = d3 + jy * jy * ir, ezz = d3 + jz * jz * ir;
    const Real exy = jx * jy * ir, exz = jx * jz * ir, eyz = jy * jz * ir;
    Q[q_index(kR0) * NT] = drho;
    Q[q_index(kJx) * NT] = jx;
    Q[q_index(kJy) * NT] = jy;
    Q[q_index(kPxx) * NT] = exx + a * (pxx - exx);
    Q[q_index(kPxy) * NT] = exy + a * (pxy - exy);
    Q[q_index(kPyy) * NT] = eyy + a * (pyy - eyy);
    Z[z_index(kJz) * NT] = jz;
    Z[z_index(kPxz) * NT] = exz + a * (pxz - exz);
    Z[z_index(kPyz) * NT] = eyz + a * (pyz - eyz);
    Z[z_index(kPzz) * NT] = ezz + a * (pzz - ezz);
  }
  // B = a f~ + b f^eq with a + b = 1 is formed as f^eq + a (f~ - f^eq) and
  // f~+ = 4/3 B - 1/3 f~ as B + (B - f~)/3, so that an equilibrium cell maps
  // to itself exactly in any precision (rounded 4/3 and 1/3, or a and b,
  // would otherwise scale the state by 1 + O(ulp) every step).  f^eq is the
  // equilibrium of Sec. II.A, evaluated as in equilibrium().
  const Real ux = jx * ir, uy = jy * ir, uz = jz * ir;
  const Real base = drho - Real(1.5) * rho0 * (ux * ux + uy * uy + uz * uz);
  static_for<kQ>([&](auto q) {
    const Real feq = equilibrium_q<q, Real>(base, xi_dot<q>(ux, uy, uz), rho0);
    const Real b = feq + a * (f[q] - feq);
    if constexpr (pop_index(q) >= 0) P[pop_index(q) * NT] = b;
    use(q, b, b + (b - f[q]) * Real(1.0 / 3.0));
  });
}

// The z-march of one tile (bx, by) over the planes [z0, z1) of a box; adds
// the moments of the updated cells to v.  L is the block's LDS, kFusedValues
// values per column: P [kNPop][NT], Q [2][kNQ][NT], Z [3][kNZ][NT].
template <typename Real, int W, bool O32>
__device__ __forceinline__ void fused_tile(const global_t<Real> *__restrict__ ft, global_t<Real> *__restrict__ out, const StepParams &p,
                                           int bx, int by, int z0, int z1, Real *L, double (&v)[kNumSums]) {
  constexpr int TX = Tile<W>::TX, TY = Tile<W>::TY, IX = Tile<W>::IX, IY = Tile<W>::IY, NT = Tile<W>::NT;
  const int n = p.n;
  const int64_t stride = p.stride;
  const int tid = tile_column<W>(threadIdx.x);  // column of the tile
  const int tx = tid % TX, ty = tid / TX;
  const int x0 = bx * IX, y0 = by * IY;
  int gx = x0 - 1 + tx, gy = y0 - 1 + ty;
  gx = gx < 0 ? gx + n : (gx >= n ? gx % n : gx);
  gy = gy < 0 ? gy + n : (gy >= n ? gy % n : gy);
  const int col = gy * n + gx;
  const bool inner = tx >= 1 && tx <= TX - 2 && ty >= 1 && ty <= TY - 2 && (x0 + tx - 1) < n && (y0 + ty - 1) < n;
  const bool xface = tx <= TX - 2 && ty >= 1 && ty <= TY - 2;  // forms the x+ face (see below)
  const bool yface = tx >= 1 && tx <= TX - 2 && ty <= TY - 2;  // forms the y+ face
  const Real h = Real(p.h), dt = Real(p.dt);
  const Real dtal = dt * Real(p.alpha), dtbe = dt * Real(p.beta);
  Real *const LP = L + tid;
  Real *const LQ = L + kNPop * NT + tid;
  Real *const LZ = L + (kNPop + 2 * kNQ) * NT + tid;
  Real *const LY = L + kLdsValues * NT + tid;

  Real pf[kQ];        // f~ of the plane being published (loaded one plane ahead)
  // A centre's result is f~+ plus the stencil and face terms, which are
  // small beside it: they are summed apart (acc) and f~+ (fp) is added once,
  // when the centre is stored, so that the result is rounded at the scale of
  // f~ once instead of at every term (in FP32 this more than halves the
  // rounding noise the march adds per step).
  Real acc_c[kQ];     // terms of centre p-1, completed in this iteration
  Real acc_p[kQ];     // terms of centre p
  Real fp_c[kQ];      // f~+ of centre p-1
  Real fp_p[kQ];      // f~+ of centre p
  Real nxt[10];       // z-1 terms of the z-moving populations of centre p+1
  Real zl[4];         // lower half of the z-face above the previous plane
  static_for<kQ>([&](auto q) { acc_p[q] = Real(0); fp_p[q] = Real(0); });
  static_for<10>([&](auto i) { nxt[i] = Real(0); });
  static_for<4>([&](auto i) { zl[i] = Real(0); });

  // Completes centre `plane` (acc_c): its lower y-face, read from the slot
  // of the column W before, the store and the sums.  Runs after the barrier
  // that ends the iteration which formed the faces.
  auto finish = [&](int plane) {
    Real fym[10];
    static_for<10>([&](auto k) { fym[k] = LY[k * NT - W]; });
    apply_terms<1, -1>(fym, acc_c);
    const int cell = plane * n * n + col;
    // plain (L2-allocating) stores: a tile row's 30 updated cells do not
    // fill whole 128-byte lines, and L2 merges them with the neighbouring
    // tiles' rows before they are written back
    Real res[kQ];
    static_for<kQ>([&](auto q) {
      res[q] = fp_c[q] + acc_c[q];
      *at_cell<O32>(out + (int64_t)q * stride, cell) = res[q];
    });
    sums_of_populations<Real>(res, p.inv_rho0, v);
  };

  load_raw<Real, O32>(ft, stride, n, col, z0 - 1, pf);
  int q2 = 0, q3 = 0;  // Q slot and Z slot of plane p
  // One iteration past the chunk's end only finishes its last centre, so
  // that every centre is completed by the same code (and rounds the same
  // whatever the chunk length).
  for (int p_ = z0 - 1; p_ <= z1 + 1; ++p_) {
    if (p_ - 1 > z0 && inner) finish(p_ - 2);  // the centre the last iteration formed
    if (p_ > z1) break;
    const bool has_prev = p_ > z0;          // centre p-1 is in the chunk
    const bool has_cur = p_ >= z0 && p_ < z1;
    const int q2m = q2 ^ 1, q3m = q3 == 0 ? 2 : q3 - 1, q3mm = q3 == 2 ? 0 : q3 + 1;
    const Plane<Real, W> c{LP, LQ + q2 * (kNQ * NT), LZ + q3 * (kNZ * NT)};        // plane p
    const Plane<Real, W> c1{nullptr, LQ + q2m * (kNQ * NT), LZ + q3m * (kNZ * NT)};  // plane p-1
    const Plane<Real, W> c2{nullptr, nullptr, LZ + q3mm * (kNZ * NT)};              // plane p-2

    // centre p-1 becomes the completed centre
    static_for<kQ>([&](auto q) { acc_c[q] = acc_p[q]; fp_c[q] = fp_p[q]; });
    // own-column pieces of plane p: z+1 terms of centre p-1, the centre
    // terms and initial value of centre p, z-1 terms of centre p+1 (formed
    // by halo columns too, which never store them)
    publish_cell<Real, W>(pf, LP, LQ + q2 * (kNQ * NT), LZ + q3 * (kNZ * NT), p, [&](auto q, Real bq, Real ftq) {
      if constexpr (kCz[q] != 0) acc_c[q] -= dtal * ((Real(0.5 * kCz[q]) - h) * bq);
      Real r = Real(0);
      if constexpr (kCz[q] != 0) r = nxt[zslot(q)];
      if constexpr (q != 0) r -= dtal * (Real(speed2(q) == 1 ? 2 : 4) * h * bq);
      acc_p[q] = r;
      fp_p[q] = ftq;
      if constexpr (kCz[q] != 0) nxt[zslot(q)] = -(dtal * ((Real(-0.5 * kCz[q]) - h) * bq));
    });
    __syncthreads();

    if (inner) {
      // face between p-1 and p (upper half from plane p, lower half carried
      // from plane p-1) and the lower half of the face between p and p+1
      gathered<Real, W>(c, c, [&](const auto &g, const auto &) {
        Real m[4], lo[4];
        zface_half<-1>(g, h, m);
        zface_half<1>(g, h, lo);
        if constexpr (std::decay_t<decltype(g)>::use) {
          static_for<4>([&](auto i) { m[i] += zl[i]; });
          face_equilibrium<2, Real>(m, p, dtbe, [&](auto q, Real val) {
            acc_c[q] -= val;   // upper face of centre p-1
            acc_p[q] += val;   // lower face of centre p
          });
          static_for<4>([&](auto i) { zl[i] = lo[i]; });
        }
      });
      // diagonal z-moving populations: the in-plane differences D = B(+d1)
      // - B(-d1) and sums S = B(+d1) + B(-d1) of plane p enter centre p-1
      // (z+1 mixed term), centre p (in-plane terms) and centre p+1 (z-1
      // mixed term)
      gathered<Real, W>(c, c, [&](const auto &g, const auto &) {
        static_for<kQ>([&](auto q) {
          if constexpr (is_diag_z(q)) {
            constexpr int d1 = kCx[q] != 0 ? 0 : 1, s1 = kCx[q] + kCy[q];
            constexpr Real k = Real(0.5 * s1 * kCz[q]);
            const Real bp_ = g.template at<q, Unit<d1>::x, Unit<d1>::y>();
            const Real bm_ = g.template at<q, -Unit<d1>::x, -Unit<d1>::y>();
            if constexpr (std::decay_t<decltype(g)>::use) {
              const Real dd = bp_ - bm_;
              acc_c[q] += dtal * (k * h * dd);
              acc_p[q] -= dtal * (Real(0.5 * s1) * dd - h * (bp_ + bm_));
              nxt[zslot(q)] -= dtal * (k * h * dd);
            }
          }
        });
      });
    }
    if (has_prev) {
      // x- and y-faces of centre p-1: in-plane part from plane p-1, the
      // z-tangential gradients -h/4 [(M_L + M_R)(p) - (M_L + M_R)(p-2)]
      const Real hq = Real(0.25) * h;
      auto face_moments = [&](auto D, auto LX, auto LY, Real (&m)[4]) {
        gathered<Real, W>(c1, c1, [&](const auto &g, const auto &) {
          Real t[4];
          face_inplane<D, LX, LY>(g, h, t);
          if constexpr (std::decay_t<decltype(g)>::use) static_for<4>([&](auto i) { m[i] = t[i]; });
        });
        gathered<Real, W>(c, c2, [&](const auto &g, const auto &g2) {
          Real s1[4], s0[4];
          face_zsum<D, LX, LY>(g, s1);
          face_zsum<D, LX, LY>(g2, s0);
          if constexpr (std::decay_t<decltype(g)>::use) static_for<4>([&](auto i) { m[i] -= hq * (s1[i] - s0[i]); });
        });
      };
      using I0 = std::integral_constant<int, 0>;
      using I1 = std::integral_constant<int, 1>;
      using Im1 = std::integral_constant<int, -1>;
      // Each x-face is formed once: every column of an interior row but the
      // last (the halo column 0 too) forms its x+ face and that face's ten
      // equilibrium terms, and a column's x- terms are the x+ terms of the
      // column before it, the previous lane (a tile row is 32 consecutive
      // lanes of one wavefront).  The lane shift runs with every lane active.
      Real mxp[4] = {Real(0), Real(0), Real(0), Real(0)};
      if (xface) face_moments(I0{}, I0{}, I0{}, mxp);
      Real fxp[10], fxm[10];
      face_terms<0>(mxp, p, dtbe, fxp);
      static_for<10>([&](auto k) { fxm[k] = from_previous_lane(fxp[k]); });
      // The y-face between the column and the next row is formed once too,
      // by every interior column of every row but the last (halo row 0
      // too); its ten terms are left in LY for the column above, which
      // applies them as its lower face in finish() after the barrier that
      // ends this iteration.
      if (yface) {
        Real my[4], fy[10];
        face_moments(I1{}, I0{}, I0{}, my);
        face_terms<1>(my, p, dtbe, fy);
        static_for<10>([&](auto k) { LY[k * NT] = fy[k]; });
        if (inner) apply_terms<1, 1>(fy, acc_c);    // y+
      }
      if (inner) {
        apply_terms<0, 1>(fxp, acc_c);   // x+
        apply_terms<0, -1>(fxm, acc_c);  // x-
      }
    }

    phase();
    // the next plane's loads overlap the rest of this one (issued right
    // after publishing they took the same time and fetched 33% more bytes
    // from HBM)
    if (p_ < z1) load_raw<Real, O32>(ft, stride, n, col, p_ + 1, pf);

    if (inner && has_cur) {
      // in-plane terms of the in-plane populations of centre p (the centre
      // value was added before)
      //   axis: L = s/2 (B(+d) - B(-d)) - h (B(+d) + B(-d))
      gathered<Real, W>(c, c, [&](const auto &g, const auto &) {
        static_for<5>([&](auto q) {
          if constexpr (q >= 1) {
            constexpr int d = kCx[q] != 0 ? 0 : 1, s = kCx[q] + kCy[q];
            const Real bp_ = g.template at<q, Unit<d>::x, Unit<d>::y>();
            const Real bm_ = g.template at<q, -Unit<d>::x, -Unit<d>::y>();
            if constexpr (std::decay_t<decltype(g)>::use)
              acc_p[q] -= dtal * (Real(0.5 * s) * (bp_ - bm_) - h * (bp_ + bm_));
          }
        });
      });
      //   diagonal in the plane, in the (x, y) frame of its own signs
      auto diag_xy = [&](auto q, const auto &g) {
        constexpr int sx = kCx[q], sy = kCy[q];
        const Real p1 = g.template at<q, 1, 0>(), m1 = g.template at<q, -1, 0>();
        const Real p2 = g.template at<q, 0, 1>(), m2 = g.template at<q, 0, -1>();
        const Real pp = g.template at<q, sx, sy>(), pm = g.template at<q, sx, -sy>();
        const Real mp = g.template at<q, -sx, sy>(), mm = g.template at<q, -sx, -sy>();
        if constexpr (std::decay_t<decltype(g)>::use) {
          const Real a1 = sx > 0 ? (p1 - m1) : (m1 - p1);
          const Real a2 = sy > 0 ? (p2 - m2) : (m2 - p2);
          acc_p[q] -= dtal * ((Real(0.5) * a1 + Real(0.5) * a2) - h * ((p1 + m1) + (p2 + m2)) -
                              Real(0.5) * h * (((pp - pm) - mp) + mm));
        }
      };
      gathered<Real, W>(c, c, [&](const auto &g, const auto &) {
        diag_xy(std::integral_constant<int, 7>{}, g);
        diag_xy(std::integral_constant<int, 8>{}, g);
      });
      gathered<Real, W>(c, c, [&](const auto &g, const auto &) {
        diag_xy(std::integral_constant<int, 9>{}, g);
        diag_xy(std::integral_constant<int, 10>{}, g);
      });
    }
    q2 ^= 1;
    q3 = q3 == 2 ? 0 : q3 + 1;
    __syncthreads();
  }
}

// Register budget of the one-thread march: in FP32, 256 registers, two
// waves per SIMD.  (Without the separate f~+ of two centres it fits 168
// registers and three waves, 10% faster, but its rounding noise then puts
// the FP32 spectrum's weakest resolved shells at ~1e-4 of FP64.)  FP64
// tiles use the split march.
template <typename Real>
constexpr int kWavesPerSimd = sizeof(Real) == 4 ? 2 : 1;

// Tile and planes of work item `local` of a box.  Items are tile z-chunks,
// numbered by tile (x fastest, then y), then by chunk.  With tail_split =
// m > 1 (a box launched alone, one block per item, blocks dealt to the 8
// XCDs in turn): the first tail_from chunk items fill whole rounds of the
// device; each of the t chunks left over is cut in z into m parts of
// ceil(chunk planes / m) planes (the last parts may be short or empty),
// numbered part by part so that the parts of neighbouring tiles run side by
// side.  The work of each XCD (a contiguous eighth of the items, see
// xcd_tile) is its eighth of the whole chunks followed by its eighth of the
// parts (slots past the last part are empty), so that every XCD's last
// round is made of parts and fills its compute units for a fraction of a
// chunk's time.
// (Host and device code: the library's work-split query runs it on the host.)
__host__ __device__ constexpr int imin(int a, int b) { return a < b ? a : b; }
struct ItemPlanes {
  int tile, z0, left;
  __host__ __device__ __forceinline__ ItemPlanes(const BatchBox &d, int local) {
    const int n = d.sp.n, c = d.nz_chunk, tiles = d.tiles_x * d.tiles_y;
    int item = local, part = 0, parts = 1;
    if (d.tail_split > 1) {
      const int t = tiles * ((n + c - 1) / c) - d.tail_from;
      const int pieces = t * d.tail_split;
      const int fx = d.tail_from / 8, px = (pieces + 7) / 8;
      const int x = local / (fx + px), j = local - x * (fx + px);
      if (j < fx) {
        item = x * fx + j;
      } else {
        const int piece = x * px + (j - fx);
        if (piece >= pieces) {  // an empty slot of the last XCD
          tile = z0 = left = 0;
          return;
        }
        part = piece / t;
        item = d.tail_from + (piece - part * t);
        parts = d.tail_split;
      }
    }
    tile = item % tiles;
    const int zc = item / tiles * c, zc1 = imin(zc + c, n);
    const int len = (zc1 - zc + parts - 1) / parts;
    z0 = imin(zc1, zc + part * len);
    left = imin(zc1, z0 + len) - z0;
  }
};

// Tile of a block, numbered so that the blocks one XCD runs (blocks are
// dealt to the eight XCDs in turn) take consecutive tiles: block b of a
// launch of `padded` blocks (a multiple of 8) takes tile
// (b mod 8) * padded/8 + b/8.
__device__ __forceinline__ int xcd_tile(int b, int padded) { return (b & 7) * (padded >> 3) + (b >> 3); }

// One launch advances one or many boxes: work item = one tile z-chunk of
// one box of the device table `boxes` (sorted by item_begin), numbered as
// the tiles of that box's own launch.  Round r of the grid takes items
// [r G, (r+1) G), dealt to the XCDs in contiguous eighths.  A single box is
// a table of one entry, so a box stepped alone and the same box stepped in
// a batch run the same machine code and give the same bits.
template <typename Real, int W, bool O32>
__global__ __launch_bounds__(Tile<W>::NT, kWavesPerSimd<Real>) void dugks_fused_kernel(const BatchBox *__restrict__ boxes, int nbox,
                                                                  int total_items) {
  __shared__ Real L[kFusedValues * Tile<W>::NT];
  const int G = gridDim.x;
  for (int base = 0; base < total_items; base += G) {
    const int it = base + xcd_tile(blockIdx.x, G);
    if (it >= total_items) continue;
    const int b = find_batch_box(boxes, nbox, it);
    const BatchBox &d = boxes[b];
    const int local = it - d.item_begin;
    double v[kNumSums] = {0, 0, 0, 0, 0};
    const global_t<Real> *src = to_global(static_cast<const Real *>(d.f[d.cur]));
    global_t<Real> *dst = to_global(static_cast<Real *>(d.f[d.cur ^ 1]));
    const ItemPlanes ip(d, local);
    // the march ends with a barrier: L is free for the block reduction
    if (ip.left > 0)
      fused_tile<Real, W, O32>(src, dst, d.sp, ip.tile % d.tiles_x, ip.tile / d.tiles_x, ip.z0, ip.z0 + ip.left, L, v);
    write_block_partials(v, d.partials, d.items, local, reinterpret_cast<double (*)[kNumSums]>(L));
    __syncthreads();
  }
}


// ---------------------------------------------------------------------------
// Split-population march.  Two thread groups share each column of the
// tile: group A (the first NT threads) holds the ten z-moving populations
// (5, 6, 11..18), group B the other nine.  Each step is done by one group:
// A the z-moving stencils and the x-face moments, B the in-plane stencils,
// the z-face and y-face moments and the global sums; each applies the face
// equilibria to its own populations.  The groups exchange the partial
// moment sums of each published cell, the face moments and A's part of the
// stored cells' sums through LDS.  A thread carries the state of about half
// a column, so each compute unit holds twice the waves of the
// one-thread-per-column march.
constexpr int kPopsA[10] = {5, 6, 11, 12, 13, 14, 15, 16, 17, 18};
constexpr int kPopsB[9] = {0, 1, 2, 3, 4, 7, 8, 9, 10};
template <int G>
struct Group {
  static constexpr int N = G == 0 ? 10 : 9;
  static constexpr int pop(int i) { return G == 0 ? kPopsA[i] : kPopsB[i]; }
};
constexpr int group_of(int q) { return (q == 5 || q == 6 || q >= 11) ? 0 : 1; }
constexpr int local_of(int q) {
  for (int i = 0; i < 10; ++i)
    if (kPopsA[i] == q) return i;
  for (int i = 0; i < 9; ++i)
    if (kPopsB[i] == q) return i;
  return -1;
}
// LDS per column after the plane buffers:
//   RA [12]: A's partial moments (read by B after the first barrier of an
//            iteration), then the z-face moments [8..12), formed by B (read
//            by A after the third);
//   RB [10]: B's partial moments, then the x-face moments [0..8) formed by A;
//   SA [4]:  A's part of the sums of its last stored cell (read by B in the
//            next iteration);
//   RY [4]:  the moments of the y-face between the column and the next row,
//            formed by B in the third phase and read after the third barrier
//            by both threads of the column above (its lower y-face).
// RA, RB and SA of a column are used only by the two threads of that
// column, so every reuse is separated from the previous reads by a barrier
// or by program order within one thread.  RY is read by another column,
// at the end of an iteration, without a barrier before that column's next
// partial moments are written: it has slots of its own, next written after
// the second barrier of the next iteration.
constexpr int kRA = kNPop + 2 * kNQ + 3 * kNZ, kRB = kRA + 12, kSA = kRB + 10, kRY = kSA + 4;
constexpr int kSplitValues = kRY + 4;

// Loads of the group's populations of the column's cell in plane `plane`.
template <typename Real, int G, bool O32>
__device__ __forceinline__ void load_group(const global_t<Real> *__restrict__ ft, int64_t stride, int n, int col, int plane,
                                           Real (&f)[Group<G>::N]) {
  const int z = plane < 0 ? plane + n : (plane >= n ? plane - n : plane);
  const int idx = z * n * n + col;
  static_for<Group<G>::N>([&](auto i) { f[i] = *at_cell<O32>(ft + (int64_t)Group<G>::pop(i) * stride, idx); });
}

// Partial moment sums over the group's populations (both groups' sets are
// closed under q -> -q): drho, jx, jy, jz, Pi_xx, Pi_yy, Pi_zz, Pi_xy,
// Pi_xz, Pi_yz, formed as in pair_moments().
template <typename Real, int G>
__device__ __forceinline__ void partial_moments(const Real (&f)[Group<G>::N], Real (&m)[10]) {
  pair_moments<Real>([](int q) constexpr { return group_of(q) == G; }, [&](auto q) { return f[local_of(q)]; }, m);
}

// The rest of publishing a cell, from its full moment sums m: B and f~+ of
// the group's populations (handed to use(q, B_q, f~+_q)), their LDS
// entries, and the group's moment fields (A: Jz, Pxz, Pyz, Pzz; B: R0, Jx,
// Jy, Pxx, Pxy, Pyy), in the equilibrium-exact forms of publish_cell().
template <typename Real, int W, int G, class Use>
__device__ __forceinline__ void publish_group(const Real (&f)[Group<G>::N], const Real (&m)[10], Real *P, Real *Q,
                                              Real *Z, const StepParams &p, Use &&use) {
  constexpr int NT = Tile<W>::NT;
  const Real drho = m[0], jx = m[1], jy = m[2], jz = m[3];
  const Real rho0 = Real(p.rho0), ir = Real(p.inv_rho0);
  const Real a = Real(p.a_bp);
  const Real d3 = drho * Real(1.0 / 3.0);
  if constexpr (G == 0) {
    const Real ezz = d3 + jz * jz * ir, exz = jx * jz * ir, eyz = jy * jz * ir;
    Z[z_index(kJz) * NT] = jz;
    Z[z_index(kPxz) * NT] = exz + a * (m[8] - exz);
    Z[z_index(kPyz) * NT] = eyz + a * (m[9] - eyz);
    Z[z_index(kPzz) * NT] = ezz + a * (m[6] - ezz);
  } else {
    const Real exx = d3 + jx * jx * ir, eyy = d3 + jy * jy * ir, exy = jx * jy * ir;
    Q[q_index(kR0) * NT] = drho;
    Q[q_index(kJx) * NT] = jx;
    Q[q_index(kJy) * NT] = jy;
    Q[q_index(kPxx) * NT] = exx + a * (m[4] - exx);
    Q[q_index(kPxy) * NT] = exy + a * (m[7] - exy);
    Q[q_index(kPyy) * NT] = eyy + a * (m[5] - eyy);
  }
  const Real ux = jx * ir, uy = jy * ir, uz = jz * ir;
  const Real base = drho - Real(1.5) * rho0 * (ux * ux + uy * uy + uz * uz);
  static_for<Group<G>::N>([&](auto i) {
    constexpr int q = Group<G>::pop(i);
    const Real feq = equilibrium_q<q, Real>(base, xi_dot<q>(ux, uy, uz), rho0);
    const Real b = feq + a * (f[i] - feq);
    if constexpr (pop_index(q) >= 0) P[pop_index(q) * NT] = b;
    use(std::integral_constant<int, q>{}, b, b + (b - f[i]) * Real(1.0 / 3.0));
  });
}

// The z-march of group G of a tile over the planes [z0, z1) (see above).
// L: the block's LDS, kSplitValues values per column.
template <typename Real, int W, int G, bool O32>
__device__ __forceinline__ void split_tile(const global_t<Real> *__restrict__ ft, global_t<Real> *__restrict__ out, const StepParams &p,
                                           int bx, int by, int z0, int z1, Real *L, double (&v)[kNumSums]) {
  constexpr int TX = Tile<W>::TX, TY = Tile<W>::TY, IX = Tile<W>::IX, IY = Tile<W>::IY, NT = Tile<W>::NT;
  constexpr int NG = Group<G>::N;
  const int n = p.n;
  const int64_t stride = p.stride;
  const int c = tile_column<W>(threadIdx.x - G * NT);  // column of the tile
  const int tx = c % TX, ty = c / TX;
  const int x0 = bx * IX, y0 = by * IY;
  int gx = x0 - 1 + tx, gy = y0 - 1 + ty;
  gx = gx < 0 ? gx + n : (gx >= n ? gx % n : gx);
  gy = gy < 0 ? gy + n : (gy >= n ? gy % n : gy);
  const int col = gy * n + gx;
  const bool inner = tx >= 1 && tx <= TX - 2 && ty >= 1 && ty <= TY - 2 && (x0 + tx - 1) < n && (y0 + ty - 1) < n;
  const bool xface = tx <= TX - 2 && ty >= 1 && ty <= TY - 2;  // A: forms an x+ face
  const bool yface = tx >= 1 && tx <= TX - 2 && ty <= TY - 2;  // B: forms a y+ face
  const Real h = Real(p.h), dt = Real(p.dt);
  const Real dtal = dt * Real(p.alpha), dtbe = dt * Real(p.beta);
  const double ir = p.inv_rho0;
  Real *const LP = L + c;
  Real *const LQ = L + kNPop * NT + c;
  Real *const LZ = L + (kNPop + 2 * kNQ) * NT + c;
  Real *const RA = L + kRA * NT + c;
  Real *const RB = L + kRB * NT + c;
  Real *const SA = L + kSA * NT + c;
  Real *const RY = L + kRY * NT + c;

  Real pf[NG];            // the group's f~ of the plane being published
  Real acc_c[NG];         // centre p-1
  Real acc_p[NG];         // centre p
  Real nxt[10];           // A: z-1 terms of centre p+1 (all of A's populations move in z)
  Real zl[4];             // B: lower half of the z-face above the previous plane
  double jb[3] = {0, 0, 0};  // B: its part of the momentum of the last stored cell
  static_for<NG>([&](auto i) { acc_p[i] = Real(0); });
  static_for<10>([&](auto i) { nxt[i] = Real(0); });
  static_for<4>([&](auto i) { zl[i] = Real(0); });

  load_group<Real, G, O32>(ft, stride, n, col, z0 - 1, pf);
  int q2 = 0, q3 = 0;
  for (int p_ = z0 - 1; p_ <= z1; ++p_) {
    const bool has_prev = p_ > z0;
    const bool has_cur = p_ >= z0 && p_ < z1;
    const bool stored_last = p_ - 1 > z0;  // a cell was stored in the previous iteration
    const int q2m = q2 ^ 1, q3m = q3 == 0 ? 2 : q3 - 1, q3mm = q3 == 2 ? 0 : q3 + 1;
    const Plane<Real, W> pc{LP, LQ + q2 * (kNQ * NT), LZ + q3 * (kNZ * NT)};
    const Plane<Real, W> pc1{nullptr, LQ + q2m * (kNQ * NT), LZ + q3m * (kNZ * NT)};
    const Plane<Real, W> pc2{nullptr, nullptr, LZ + q3mm * (kNZ * NT)};

    static_for<NG>([&](auto i) { acc_c[i] = acc_p[i]; });
    // partial moments of this group's populations, exchanged with the other group
    Real m[10];
    partial_moments<Real, G>(pf, m);
    static_for<10>([&](auto k) { (G == 0 ? RA : RB)[k * NT] = m[k]; });
    __syncthreads();
    static_for<10>([&](auto k) { m[k] = G == 0 ? m[k] + RB[k * NT] : RA[k * NT] + m[k]; });
    if constexpr (G == 1) {
      if (inner && stored_last) {
        const double ra = (double)SA[0], xa = (double)SA[NT], ya = (double)SA[2 * NT], za = (double)SA[3 * NT];
        v[0] += ra; v[1] += xa; v[2] += ya; v[3] += za;
        const double x = jb[0] + xa, y = jb[1] + ya, z = jb[2] + za;
        v[4] += 0.5 * (x * x + y * y + z * z) * ir * ir;
      }
    }
    // own-column pieces of plane p (see fused_tile)
    publish_group<Real, W, G>(pf, m, LP, LQ + q2 * (kNQ * NT), LZ + q3 * (kNZ * NT), p, [&](auto q, Real bq, Real ftq) {
      constexpr int i = local_of(q);
      if constexpr (kCz[q] != 0) acc_c[i] -= dtal * ((Real(0.5 * kCz[q]) - h) * bq);
      Real r = ftq;
      if constexpr (kCz[q] != 0) r += nxt[i];
      if constexpr (q != 0) r -= dtal * (Real(speed2(q) == 1 ? 2 : 4) * h * bq);
      acc_p[i] = r;
      if constexpr (kCz[q] != 0) nxt[i] = -(dtal * ((Real(-0.5 * kCz[q]) - h) * bq));
    });
    __syncthreads();

    Real fx[2][4];  // the faces this group forms: A x+ and x-, B y+ and y-
    if (inner) {
      if constexpr (G == 0) {
        // diagonal z-moving populations: in-plane differences D = B(+d1) -
        // B(-d1) and sums S = B(+d1) + B(-d1) of plane p enter centre p-1
        // (z+1 mixed term), centre p (in-plane terms), centre p+1 (z-1 mixed term)
        gathered<Real, W>(pc, pc, [&](const auto &g, const auto &) {
          static_for<kQ>([&](auto q) {
            if constexpr (is_diag_z(q)) {
              constexpr int d1 = kCx[q] != 0 ? 0 : 1, s1 = kCx[q] + kCy[q];
              constexpr Real k = Real(0.5 * s1 * kCz[q]);
              constexpr int i = local_of(q);
              const Real bp_ = g.template at<q, Unit<d1>::x, Unit<d1>::y>();
              const Real bm_ = g.template at<q, -Unit<d1>::x, -Unit<d1>::y>();
              if constexpr (std::decay_t<decltype(g)>::use) {
                const Real dd = bp_ - bm_;
                acc_c[i] += dtal * (k * h * dd);
                acc_p[i] -= dtal * (Real(0.5 * s1) * dd - h * (bp_ + bm_));
                nxt[i] -= dtal * (k * h * dd);
              }
            }
          });
        });
      } else {
        // face between p-1 and p (upper half from plane p, lower half
        // carried from plane p-1) for A, and the lower half of the next one
        gathered<Real, W>(pc, pc, [&](const auto &g, const auto &) {
          Real mm[4], lo[4];
          zface_half<-1>(g, h, mm);
          zface_half<1>(g, h, lo);
          if constexpr (std::decay_t<decltype(g)>::use) {
            static_for<4>([&](auto i) { RA[(8 + i) * NT] = mm[i] + zl[i]; });
            static_for<4>([&](auto i) { zl[i] = lo[i]; });
          }
        });
        if (has_cur) {
          gathered<Real, W>(pc, pc, [&](const auto &g, const auto &) {
            static_for<5>([&](auto q) {
              if constexpr (q >= 1) {
                constexpr int d = kCx[q] != 0 ? 0 : 1, s = kCx[q] + kCy[q];
                const Real bp_ = g.template at<q, Unit<d>::x, Unit<d>::y>();
                const Real bm_ = g.template at<q, -Unit<d>::x, -Unit<d>::y>();
                if constexpr (std::decay_t<decltype(g)>::use)
                  acc_p[local_of(q)] -= dtal * (Real(0.5 * s) * (bp_ - bm_) - h * (bp_ + bm_));
              }
            });
          });
          auto diag_xy = [&](auto q, const auto &g) {
            constexpr int sx = kCx[q], sy = kCy[q];
            const Real p1 = g.template at<q, 1, 0>(), m1 = g.template at<q, -1, 0>();
            const Real p2 = g.template at<q, 0, 1>(), m2 = g.template at<q, 0, -1>();
            const Real pp = g.template at<q, sx, sy>(), pm = g.template at<q, sx, -sy>();
            const Real mp = g.template at<q, -sx, sy>(), mm = g.template at<q, -sx, -sy>();
            if constexpr (std::decay_t<decltype(g)>::use) {
              const Real a1 = sx > 0 ? (p1 - m1) : (m1 - p1);
              const Real a2 = sy > 0 ? (p2 - m2) : (m2 - p2);
              acc_p[local_of(q)] -= dtal * ((Real(0.5) * a1 + Real(0.5) * a2) - h * ((p1 + m1) + (p2 + m2)) -
                                            Real(0.5) * h * (((pp - pm) - mp) + mm));
            }
          };
          gathered<Real, W>(pc, pc, [&](const auto &g, const auto &) {
            diag_xy(std::integral_constant<int, 7>{}, g);
            diag_xy(std::integral_constant<int, 8>{}, g);
          });
          gathered<Real, W>(pc, pc, [&](const auto &g, const auto &) {
            diag_xy(std::integral_constant<int, 9>{}, g);
            diag_xy(std::integral_constant<int, 10>{}, g);
          });
        }
      }
    }
    if (has_prev) {
      {
        // the group's two faces of centre p-1: in-plane part from plane
        // p-1, z-tangential gradients -h/4 [(M_L + M_R)(p) - (M_L + M_R)(p-2)];
        // written for the other group (A's into RB, B's into RA)
        constexpr int D = G == 0 ? 0 : 1;
        const Real hq = Real(0.25) * h;
        auto face = [&](auto LX, auto LY, Real (&fm)[4]) {
          gathered<Real, W>(pc1, pc1, [&](const auto &g, const auto &) {
            Real t[4];
            face_inplane<D, LX, LY>(g, h, t);
            if constexpr (std::decay_t<decltype(g)>::use) static_for<4>([&](auto i) { fm[i] = t[i]; });
          });
          gathered<Real, W>(pc, pc2, [&](const auto &g, const auto &g2) {
            Real s1[4], s0[4];
            face_zsum<D, LX, LY>(g, s1);
            face_zsum<D, LX, LY>(g2, s0);
            if constexpr (std::decay_t<decltype(g)>::use) static_for<4>([&](auto i) { fm[i] -= hq * (s1[i] - s0[i]); });
          });
        };
        using I0 = std::integral_constant<int, 0>;
        using Im1 = std::integral_constant<int, -1>;
        if constexpr (G == 0) {
          // each x-face formed once, as in fused_tile: x+ by every column of
          // an interior row but the last, x- from the previous lane
          Real xp[4] = {Real(0), Real(0), Real(0), Real(0)};
          if (xface) face(I0{}, I0{}, xp);
          static_for<4>([&](auto i) {
            fx[0][i] = xp[i];
            fx[1][i] = from_previous_lane(xp[i]);
          });
        } else {
          // y+ faces only, by every interior column of every row but the
          // last (halo row 0 too); the y- face is read back from the row below
          if (yface) {
            face(I0{}, I0{}, fx[0]);
            static_for<4>([&](auto i) { RY[i * NT] = fx[0][i]; });
          }
        }
        if constexpr (G == 0) {
          if (inner) static_for<2>([&](auto f) { static_for<4>([&](auto i) { RB[(f * 4 + i) * NT] = fx[f][i]; }); });
        }
      }
    }
    phase();
    if (p_ < z1) load_group<Real, G, O32>(ft, stride, n, col, p_ + 1, pf);
    if (p_ >= z0) {
      __syncthreads();
      if (inner) {
        using I0 = std::integral_constant<int, 0>;
        using I1 = std::integral_constant<int, 1>;
        auto put_face = [&](const Real (&fm)[4], auto D, auto S) {
          face_equilibrium<D, Real>(fm, p, dtbe, [&](auto q, Real val) {
            if constexpr (group_of(q) == G) {
              if constexpr (S > 0)
                acc_c[local_of(q)] -= val;
              else
                acc_c[local_of(q)] += val;
            }
          });
        };
        if constexpr (G == 0) {
          // the z-face between p-1 and p: upper face of centre p-1, lower of centre p
          Real zf[4];
          static_for<4>([&](auto i) { zf[i] = RA[(8 + i) * NT]; });
          face_equilibrium<2, Real>(zf, p, dtbe, [&](auto q, Real val) {
            acc_c[local_of(q)] -= val;
            acc_p[local_of(q)] += val;
          });
        }
        if (has_prev) {
          // equilibrium parts of the four x/y-faces of centre p-1 for this
          // group's populations: its own two faces and the other group's
          Real fo[2][4];
          if constexpr (G == 0) {
            static_for<4>([&](auto i) { fo[0][i] = RY[i * NT]; fo[1][i] = RY[i * NT - W]; });
          } else {
            static_for<2>([&](auto f) { static_for<4>([&](auto i) { fo[f][i] = RB[(f * 4 + i) * NT]; }); });
            static_for<4>([&](auto i) { fx[1][i] = RY[i * NT - W]; });
          }
          using Ip = std::integral_constant<int, 1>;
          using Im = std::integral_constant<int, -1>;
          if constexpr (G == 0) {
            put_face(fx[0], I0{}, Ip{}); put_face(fx[1], I0{}, Im{});
            put_face(fo[0], I1{}, Ip{}); put_face(fo[1], I1{}, Im{});
          } else {
            put_face(fo[0], I0{}, Ip{}); put_face(fo[1], I0{}, Im{});
            put_face(fx[0], I1{}, Ip{}); put_face(fx[1], I1{}, Im{});
          }
          const int cell = (p_ - 1) * n * n + col;
          double r = 0, ax = 0, ay = 0, az = 0;
          static_for<NG>([&](auto i) {
            constexpr int q = Group<G>::pop(i);
            *at_cell<O32>(out + (int64_t)q * stride, cell) = acc_c[i];  // plain stores, as in fused_tile
            const double x = (double)acc_c[i];
            r += x;
            if constexpr (kCx[q] != 0) ax += kCx[q] * x;
            if constexpr (kCy[q] != 0) ay += kCy[q] * x;
            if constexpr (kCz[q] != 0) az += kCz[q] * x;
          });
          if constexpr (G == 0) {
            SA[0] = Real(r); SA[NT] = Real(ax); SA[2 * NT] = Real(ay); SA[3 * NT] = Real(az);
          } else {
            v[0] += r; v[1] += ax; v[2] += ay; v[3] += az;
            jb[0] = ax; jb[1] = ay; jb[2] = az;
          }
        }
      }
    }
    q2 ^= 1;
    q3 = q3 == 2 ? 0 : q3 + 1;
  }
  // A's part of the sums of the last stored cell
  __syncthreads();
  if constexpr (G == 1) {
    if (inner) {
      const double ra = (double)SA[0], xa = (double)SA[NT], ya = (double)SA[2 * NT], za = (double)SA[3 * NT];
      v[0] += ra; v[1] += xa; v[2] += ya; v[3] += za;
      const double x = jb[0] + xa, y = jb[1] + ya, z = jb[2] + za;
      v[4] += 0.5 * (x * x + y * y + z * z) * ir * ir;
    }
  }
  __syncthreads();
}

// Work-list kernel of the split march (see dugks_fused_kernel).
template <typename Real, int W, bool O32>
__global__ __launch_bounds__(2 * Tile<W>::NT) void dugks_split_kernel(const BatchBox *__restrict__ boxes, int nbox,
                                                                      int total_items) {
  __shared__ Real L[kSplitValues * Tile<W>::NT];
  const int G = gridDim.x;
  for (int base = 0; base < total_items; base += G) {
    const int it = base + xcd_tile(blockIdx.x, G);
    if (it >= total_items) continue;
    const int b = find_batch_box(boxes, nbox, it);
    const BatchBox &d = boxes[b];
    const int local = it - d.item_begin;
    double v[kNumSums] = {0, 0, 0, 0, 0};
    const global_t<Real> *src = to_global(static_cast<const Real *>(d.f[d.cur]));
    global_t<Real> *dst = to_global(static_cast<Real *>(d.f[d.cur ^ 1]));
    const ItemPlanes ip(d, local);
    if (ip.left > 0) {
      const int bx = ip.tile % d.tiles_x, by = ip.tile / d.tiles_x, z1 = ip.z0 + ip.left;
      if (threadIdx.x < Tile<W>::NT)
        split_tile<Real, W, 0, O32>(src, dst, d.sp, bx, by, ip.z0, z1, L, v);
      else
        split_tile<Real, W, 1, O32>(src, dst, d.sp, bx, by, ip.z0, z1, L, v);
    }
    write_block_partials(v, d.partials, d.items, local, reinterpret_cast<double (*)[kNumSums]>(L));
    __syncthreads();
  }
}

// Writes table entries given by value (the launch carries them in its
// arguments), for callers that must not copy from host memory.
__global__ void store_table_kernel(BatchBox e0, BatchBox e1, BatchBox *__restrict__ dst) {
  if (threadIdx.x == 0) {
    dst[0] = e0;
    dst[1] = e1;
  }
}

}  // namespace fused

// Default tile: 32 x 8 columns in both precisions (rows of 256 B in FP64).
// FP64 (split march, 512 threads): 140 KB of LDS, one block per compute
// unit; FP32 (256 threads): 51 KB of LDS, two blocks per compute unit
// (two waves per SIMD).
constexpr int fused_tile_width(int) { return 32; }

int fused_default_chunk(int n) { return n >= 128 ? 32 : (n >= 32 ? 16 : n); }

// Chunk items of a box (tiles x z-chunks) at tile width w and z-chunk
// `chunk` planes, and its tiling.
int fused_dugks_items(int n, int w, int chunk, int *tiles_x, int *tiles_y) {
  const int ix = w - 2, iy = 8 - 2;
  const int tx = (n + ix - 1) / ix;
  const int ty = (n + iy - 1) / iy;
  if (tiles_x) *tiles_x = tx;
  if (tiles_y) *tiles_y = ty;
  return tx * ty * ((n + chunk - 1) / chunk);
}

// Shortest z-chunk the balanced choice below takes (shorter chunks re-read
// the two halo planes too often).
constexpr int kMinAutoChunk = 8;

// Parts each chunk of a launch's last round is cut into: `chunks` items of
// `chunk` planes run in rounds of `slots` blocks; when at least one round
// is full and the t items left over fill at most half a round, each is cut
// into parts of ceil(chunk / min(slots / t, chunk)) planes, as many as that
// length needs (1: no cut).
static int tail_parts(int chunks, int slots, int chunk) {
  const int full = chunks / slots, t = chunks - full * slots;
  if (full < 1 || t == 0) return 1;
  const int m = std::min(slots / t, chunk);
  if (m < 2) return 1;
  const int len = (chunk + m - 1) / m;
  return (chunk + len - 1) / len;
}

static int fused_slots(int precision, int w);

FusedPlan fused_plan_for(const dhit_params &p, int slots) {
  FusedPlan f{};
  const int n = p.n;
  f.width = p.tile_width ? p.tile_width : fused_tile_width(p.precision);
  // an unresolved setting (0) gets the shortest automatic chunk: an upper
  // bound on the items, for sizing buffers
  f.chunk = p.z_chunk > 0 ? p.z_chunk : (p.z_chunk < 0 ? -p.z_chunk : std::min(n, kMinAutoChunk));
  const int chunks = fused_dugks_items(n, f.width, f.chunk, &f.tiles_x, &f.tiles_y);
  f.items = f.tail_from = f.grid = chunks;
  f.tail_split = 1;
  if (p.z_chunk < 0 && slots > 0) {
    const int m = tail_parts(chunks, slots, f.chunk);
    if (m > 1 && slots % 8 == 0) {
      f.tail_from = chunks / slots * slots;
      f.tail_split = m;
      // per XCD: its eighth of the whole chunks, then its eighth of the parts
      const int pieces = (chunks - f.tail_from) * m;
      f.items = f.grid = 8 * (f.tail_from / 8 + (pieces + 7) / 8);
    }
  }
  return f;
}

FusedPlan fused_plan(const dhit_params &p) {
  return fused_plan_for(p, p.z_chunk < 0 ? fused_slots(p.precision, p.tile_width ? p.tile_width : fused_tile_width(p.precision)) : 0);
}

void fused_item_planes(const FusedPlan &f, int n, int item, int *tile, int *z0, int *planes) {
  BatchBox d;
  std::memset(&d, 0, sizeof(d));
  d.sp.n = n;
  d.tiles_x = f.tiles_x;
  d.tiles_y = f.tiles_y;
  d.nz_chunk = f.chunk;
  d.tail_from = f.tail_from;
  d.tail_split = f.tail_split;
  const fused::ItemPlanes ip(d, item);
  *tile = ip.tile;
  *z0 = ip.z0;
  *planes = ip.left;
}

// Work items of a box's fused launch (and its tiling).  With z_chunk = 0
// (not yet resolved) an upper bound for sizing buffers: twice the items of
// the shortest automatic chunk and 8 (a cut last round adds at most a
// round's items, rounded up to a multiple of 8, to at least one full round).
int fused_dugks_blocks(const dhit_params &p, int *width, int *tiles_x, int *tiles_y, int *nz_chunk) {
  const FusedPlan f = fused_plan(p);
  if (width) *width = f.width;
  if (tiles_x) *tiles_x = f.tiles_x;
  if (tiles_y) *tiles_y = f.tiles_y;
  if (nz_chunk) *nz_chunk = f.chunk;
  return p.z_chunk == 0 ? 2 * f.items + 8 : f.items;
}

// FP64 tiles use the split-population march (two thread groups per
// column), FP32 tiles one thread per column.
template <typename Real>
constexpr bool kSplit = sizeof(Real) == 8;

template <typename Real, int W, bool O32>
static void list_launch(hipStream_t s, const BatchBox *d_boxes, int nbox, int total_items, int grid) {
  grid = (grid + 7) / 8 * 8;  // the XCD numbering of work items needs a multiple of 8
  if constexpr (kSplit<Real>)
    hipLaunchKernelGGL((fused::dugks_split_kernel<Real, W, O32>), dim3(grid), dim3(2 * fused::Tile<W>::NT), 0, s,
                       d_boxes, nbox, total_items);
  else
    hipLaunchKernelGGL((fused::dugks_fused_kernel<Real, W, O32>), dim3(grid), dim3(fused::Tile<W>::NT), 0, s, d_boxes,
                       nbox, total_items);
}

// Whether 32-bit byte offsets reach every cell of one population array of
// an n^3 box (n^3 elements of `elem` bytes below 4 GB).
static bool offsets32(int max_n, int precision) {
  const uint64_t elem = precision == DHIT_FP64 ? 8 : 4;
  return (uint64_t)max_n * max_n * max_n * elem < (uint64_t(1) << 32);
}

void launch_dugks_batch(hipStream_t s, int precision, int w, int max_n, const BatchBox *d_boxes, int nbox,
                        int total_items, int grid) {
  if (w != 16 && w != 32) throw Error(DHIT_EINVAL, "fused DUGKS tile width must be 16 or 32");
  const bool o32 = offsets32(max_n, precision);
  if (precision == DHIT_FP64) {
    if (w == 16) o32 ? list_launch<double, 16, true>(s, d_boxes, nbox, total_items, grid)
                     : list_launch<double, 16, false>(s, d_boxes, nbox, total_items, grid);
    else o32 ? list_launch<double, 32, true>(s, d_boxes, nbox, total_items, grid)
             : list_launch<double, 32, false>(s, d_boxes, nbox, total_items, grid);
  } else {
    if (w == 16) o32 ? list_launch<float, 16, true>(s, d_boxes, nbox, total_items, grid)
                     : list_launch<float, 16, false>(s, d_boxes, nbox, total_items, grid);
    else o32 ? list_launch<float, 32, true>(s, d_boxes, nbox, total_items, grid)
             : list_launch<float, 32, false>(s, d_boxes, nbox, total_items, grid);
  }
  DHIT_HIP(hipGetLastError());
}

// The two one-box tables of a box: entry c steps from f[c] to f[1 - c].
void fused_table_entries(const dhit_box &b, BatchBox (&e)[2]) {
  const FusedPlan f = fused_plan(b.p);
  for (int c = 0; c < 2; ++c) {
    std::memset(&e[c], 0, sizeof(BatchBox));
    e[c].f[0] = b.f[0];
    e[c].f[1] = b.f[1];
    e[c].sp = b.sp;
    e[c].ncell = (int)b.ncell;
    e[c].item_begin = 0;
    e[c].items = f.items;
    e[c].tiles_x = f.tiles_x;
    e[c].tiles_y = f.tiles_y;
    e[c].nz_chunk = f.chunk;
    e[c].tail_from = f.tail_from;
    e[c].tail_split = f.tail_split;
    e[c].partials = b.partials;
    e[c].hist = b.hist;
    e[c].cur = c;
  }
}

void launch_store_table(hipStream_t s, const BatchBox (&e)[2], BatchBox *dst) {
  hipLaunchKernelGGL(fused::store_table_kernel, dim3(1), dim3(64), 0, s, e[0], e[1], dst);
  DHIT_HIP(hipGetLastError());
}

static void fused_step(dhit_box &b, const void *src, void *dst, double *sums_out) {
  if (!b.step_table) throw Error(DHIT_EINVAL, "box has no fused-step table");
  int entry;
  if (src == b.f[0] && dst == b.f[1]) entry = 0;
  else if (src == b.f[1] && dst == b.f[0]) entry = 1;
  else throw Error(DHIT_EINVAL, "fused DUGKS step between buffers that are not the box's");
  const FusedPlan f = fused_plan(b.p);
  {
    TimedLaunch t(b, DHIT_K_DUGKS_FUSED);
    launch_dugks_batch(b.stream, b.p.precision, f.width, b.n, b.step_table + entry, 1, f.items, f.grid);
    t.done();
  }
  launch_finalize_sums(b, b.partials, f.items, sums_out);
}

int fused_tile_width_of(int precision) { return fused_tile_width(precision); }

// Blocks of the fused kernel of this precision and tile width that one
// compute unit holds at once (registers and LDS decide: one for the FP64
// split march, two for FP32 at width 32).
static int fused_resident_blocks(int precision, int w) {
  int nb = 0;
  hipError_t e;
  if (precision == DHIT_FP64)
    e = w == 16 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(
                      &nb, reinterpret_cast<const void *>(&fused::dugks_split_kernel<double, 16, true>), 2 * fused::Tile<16>::NT, 0)
                : hipOccupancyMaxActiveBlocksPerMultiprocessor(
                      &nb, reinterpret_cast<const void *>(&fused::dugks_split_kernel<double, 32, true>), 2 * fused::Tile<32>::NT, 0);
  else
    e = w == 16 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(
                      &nb, reinterpret_cast<const void *>(&fused::dugks_fused_kernel<float, 16, true>), fused::Tile<16>::NT, 0)
                : hipOccupancyMaxActiveBlocksPerMultiprocessor(
                      &nb, reinterpret_cast<const void *>(&fused::dugks_fused_kernel<float, 32, true>), fused::Tile<32>::NT, 0);
  return e == hipSuccess && nb > 0 ? nb : 1;
}

int fused_resident_blocks_of(int precision, int w) { return fused_resident_blocks(precision, w); }

// Blocks of the fused kernel that the current device holds at once
// (compute units x resident blocks), kept per device.
static int fused_slots(int precision, int w) {
  int dev = 0;
  DHIT_HIP(hipGetDevice(&dev));
  static std::mutex mu;
  static std::map<std::array<int, 3>, int> known;
  std::lock_guard<std::mutex> lock(mu);
  const std::array<int, 3> key{dev, precision, w};
  const auto it = known.find(key);
  if (it != known.end()) return it->second;
  int cus = 0;
  DHIT_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  const int slots = std::max(cus, 1) * fused_resident_blocks(precision, w);
  known[key] = slots;
  return slots;
}

// z-chunk that balances a launch.  Its blocks run in rounds of `slots`
// (compute units x resident blocks); a block marching c planes costs about
// c + 2 plane iterations (the two halo planes), so a launch of K chunk items
// costs about ceil(K / slots) (c + 2); with its last, partly filled round
// cut into m parts per chunk (tail_parts) it costs floor(K / slots) (c + 2)
// + ceil(c / m) + 2.  Among the chunks ceil(n / k) of at least kMinAutoChunk
// planes (or n, if smaller), each with and without the cut, the cheapest is
// taken (the cut one is returned as -c), the longest and the uncut of equal
// ones.  At 256^3 in FP64 (1 block per unit, 387 column tiles): chunks of
// 37 planes cost 11 rounds of 39 iterations (the last round 58% full: 429);
// chunks of 128 planes, 3 full rounds of 130 and 6 chunks left over that
// are cut into 32 parts of 4 planes, 396.
int fused_balanced_chunk(int n, int tiles_xy, int slots) {
  const int cmin = std::min(n, kMinAutoChunk);
  int best = n;
  int64_t best_cost = INT64_MAX;
  for (int k = 1; (n + k - 1) / k >= cmin; ++k) {
    const int c = (n + k - 1) / k;
    if (k > 1 && c == (n + k - 2) / (k - 1)) continue;  // same chunk as k - 1
    const int64_t blocks = (int64_t)tiles_xy * ((n + c - 1) / c);
    const int64_t cost = (blocks + slots - 1) / slots * (c + 2);
    if (cost < best_cost) {
      best_cost = cost;
      best = c;
    }
    if (blocks <= INT32_MAX) {
      const int m = tail_parts((int)blocks, slots, c);
      const int64_t cut = blocks / slots * (c + 2) + (c + m - 1) / m + 2;
      if (m > 1 && cut < best_cost) {
        best_cost = cut;
        best = -c;
      }
    }
  }
  return best;
}

// Default z-chunk of a box on the current device.
int fused_auto_chunk(const dhit_params &p) {
  dhit_params q = p;
  q.z_chunk = 0;
  const FusedPlan f = fused_plan(q);
  return fused_balanced_chunk(p.n, f.tiles_x * f.tiles_y, fused_slots(p.precision, f.width));
}

void launch_dugks_fused(dhit_box &b, const void *src, void *dst, double *sums_out) { fused_step(b, src, dst, sums_out); }

}  // namespace dhit
