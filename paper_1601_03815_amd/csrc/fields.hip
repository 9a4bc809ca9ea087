// Field kernels around the time steps: initial equilibrium state, moments,
// conversion between the stored state and host-order double arrays, and
// the deterministic finalisation of the per-step global sums.
#include "collision.hpp"

namespace dhit {

// f = f^eq(drho, rho0 u) (BGK-LBE, DUGKS) or f = M^-1 m^eq (MRT-LBE).
template <typename Real, bool Mrt>
__global__ __launch_bounds__(kBlock) void init_kernel(const double *__restrict__ u, const double *__restrict__ drho,
                                                      Real *__restrict__ f, StepParams p, int ncell) {
  const int cell = blockIdx.x * kBlock + threadIdx.x;
  if (cell >= ncell) return;
  const Real r = drho ? Real(drho[cell]) : Real(0);
  const Real jx = Real(p.rho0 * u[cell]);
  const Real jy = Real(p.rho0 * u[(int64_t)ncell + cell]);
  const Real jz = Real(p.rho0 * u[2 * (int64_t)ncell + cell]);
  Real fe[kQ];
  if constexpr (Mrt)
    mrt_equilibrium_populations<Real>(r, jx, jy, jz, p, fe);
  else
    equilibrium<Real>(r, jx, jy, jz, Real(p.rho0), Real(p.inv_rho0), fe);
  static_for<kQ>([&](auto q) { f[(int64_t)q * p.stride + cell] = fe[q]; });
}

// Consistent initial state of a DUGKS box (Sec. IV.A): the equilibrium of
// Sec. II.A plus the first-order Chapman-Enskog non-equilibrium part of the
// BGK model, f1_q = -(tau rho0 / RT) W_q (xi_qa xi_qb - RT delta_ab) G_ab
// with G_ab = d_a u_b, in the tracked variable f~ = f - dt/2 Omega, i.e.
// f~ = f^eq + (1 + dt/(2 tau)) f1 = f^eq - 3 rho0 (tau + dt/2) W_q
// (xi_qa xi_qb - delta_ab/3) G_ab.  Evaluated in double, rounded once.
template <typename Real>
__global__ __launch_bounds__(kBlock) void ce_init_kernel(const double *__restrict__ u, const double *__restrict__ drho,
                                                         const double *__restrict__ grad, Real *__restrict__ f,
                                                         StepParams p, int ncell) {
  const int cell = blockIdx.x * kBlock + threadIdx.x;
  if (cell >= ncell) return;
  const double r = drho ? drho[cell] : 0.0;
  const double jx = p.rho0 * u[cell], jy = p.rho0 * u[(int64_t)ncell + cell], jz = p.rho0 * u[2 * (int64_t)ncell + cell];
  double G[3][3];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) G[a][b] = grad[(int64_t)(3 * a + b) * ncell + cell];
  double fe[kQ];
  equilibrium<double>(r, jx, jy, jz, p.rho0, p.inv_rho0, fe);
  const double coef = -3.0 * p.rho0 * (p.tau + 0.5 * p.dt);
  static_for<kQ>([&](auto q) {
    double s = 0.0;
    static_for<3>([&](auto a) {
      static_for<3>([&](auto b) {
        constexpr double qab = double(cdir(q, a) * cdir(q, b)) - (a == b ? 1.0 / 3.0 : 0.0);
        if constexpr (qab != 0.0) s += qab * G[a][b];
      });
    });
    f[(int64_t)q * p.stride + cell] = Real(fe[q] + coef * kWeight(q) * s);
  });
}

// One pass of the initial-state iteration of an LBE box (Sec. IV.A: the
// kinetic schemes start from the density fluctuation and non-equilibrium
// part that belong to the initial velocity, found by running the scheme
// with the velocity held at its initial value).  After each time step, every
// cell's momentum is put back to rho0 u while its density and its
// non-equilibrium part are kept: f += E(drho, rho0 u) - E(drho, j), with E
// the state init_kernel builds.  Both collisions conserve drho and j and
// relax only f - E, so the update gives the same result on the stored
// post-collision state as on the pre-collision one.
// drho_out (optional) receives drho; with drho_prev and block_max given,
// block b stores the largest |drho - drho_prev| of its cells in block_max[b].
template <typename Real, bool Mrt>
__global__ __launch_bounds__(kBlock) void hold_velocity_kernel(Real *__restrict__ f, const double *__restrict__ u,
                                                               double *__restrict__ drho_out,
                                                               const double *__restrict__ drho_prev,
                                                               double *__restrict__ block_max, StepParams p,
                                                               int ncell) {
  __shared__ double wave_max[kWaves];
  const int cell = blockIdx.x * kBlock + threadIdx.x;
  double dev = 0.0;
  if (cell < ncell) {
    Real g[kQ];
    static_for<kQ>([&](auto q) { g[q] = f[(int64_t)q * p.stride + cell]; });
    Real r, jx, jy, jz;
    cell_moments<Real>(g, r, jx, jy, jz);
    const Real hx = Real(p.rho0 * u[cell]);
    const Real hy = Real(p.rho0 * u[(int64_t)ncell + cell]);
    const Real hz = Real(p.rho0 * u[2 * (int64_t)ncell + cell]);
    Real held[kQ], now[kQ];
    if constexpr (Mrt) {
      mrt_equilibrium_populations<Real>(r, hx, hy, hz, p, held);
      mrt_equilibrium_populations<Real>(r, jx, jy, jz, p, now);
    } else {
      equilibrium<Real>(r, hx, hy, hz, Real(p.rho0), Real(p.inv_rho0), held);
      equilibrium<Real>(r, jx, jy, jz, Real(p.rho0), Real(p.inv_rho0), now);
    }
    static_for<kQ>([&](auto q) { f[(int64_t)q * p.stride + cell] = g[q] + (held[q] - now[q]); });
    if (drho_out) drho_out[cell] = (double)r;
    if (drho_prev) {
      dev = fabs((double)r - drho_prev[cell]);
      if (!(dev < INFINITY)) dev = INFINITY;  // a NaN must survive the fmax reduction
    }
  }
  if (!block_max) return;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) dev = fmax(dev, __shfl_down(dev, off, 64));
  if ((threadIdx.x & 63) == 0) wave_max[threadIdx.x >> 6] = dev;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = wave_max[0];
    for (int w = 1; w < kWaves; ++w) m = fmax(m, wave_max[w]);
    block_max[blockIdx.x] = m;
  }
}

// Moments of every cell and the five global sums (weighted by the cell
// volumes w_x w_y w_z when a stretched mesh is given).
template <typename Real>
__global__ __launch_bounds__(kBlock) void moments_kernel(const Real *__restrict__ f, double *__restrict__ drho,
                                                         double *__restrict__ j, StepParams p, int ncell,
                                                         const double *__restrict__ mesh,
                                                         double *__restrict__ partials) {
  const int cell = blockIdx.x * kBlock + threadIdx.x;
  double v[kNumSums] = {0, 0, 0, 0, 0};
  if (cell < ncell) {
    Real g[kQ];
    static_for<kQ>([&](auto q) { g[q] = f[(int64_t)q * p.stride + cell]; });
    Real r, jx, jy, jz;
    cell_moments<Real>(g, r, jx, jy, jz);
    if (drho) drho[cell] = (double)r;
    if (j) {
      j[cell] = (double)jx;
      j[(int64_t)ncell + cell] = (double)jy;
      j[2 * (int64_t)ncell + cell] = (double)jz;
    }
    sums_of_cell<Real>(r, jx, jy, jz, p.inv_rho0, v);
    if (mesh) {
      const int n = p.n, x = cell % n, y = (cell / n) % n, z = cell / (n * n);
      const double vol = mesh[(0 * kMeshTables + kMeshWidth) * n + x] *
                         mesh[(1 * kMeshTables + kMeshWidth) * n + y] *
                         mesh[(2 * kMeshTables + kMeshWidth) * n + z];
      static_for<kNumSums>([&](auto i) { v[i] *= vol; });
    }
  }
  write_block_partials(v, partials, gridDim.x, blockIdx.x);
}

// u = j / rho0 as double [3][ncell].
template <typename Real>
__global__ __launch_bounds__(kBlock) void velocity_kernel(const Real *__restrict__ f, double *__restrict__ u,
                                                          StepParams p, int ncell) {
  const int cell = blockIdx.x * kBlock + threadIdx.x;
  if (cell >= ncell) return;
  Real g[kQ];
  static_for<kQ>([&](auto q) { g[q] = f[(int64_t)q * p.stride + cell]; });
  Real r, jx, jy, jz;
  cell_moments<Real>(g, r, jx, jy, jz);
  u[cell] = (double)jx * p.inv_rho0;
  u[(int64_t)ncell + cell] = (double)jy * p.inv_rho0;
  u[2 * (int64_t)ncell + cell] = (double)jz * p.inv_rho0;
}

template <typename Real>
__global__ __launch_bounds__(kBlock) void pack_kernel(const Real *__restrict__ f, double *__restrict__ out,
                                                      int64_t stride, int64_t ncell) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= ncell * kQ) return;
  const int64_t q = i / ncell, c = i - q * ncell;
  out[i] = (double)f[q * stride + c];
}

template <typename Real>
__global__ __launch_bounds__(kBlock) void unpack_kernel(const double *__restrict__ in, Real *__restrict__ f,
                                                        int64_t stride, int64_t ncell) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= ncell * kQ) return;
  const int64_t q = i / ncell, c = i - q * ncell;
  f[q * stride + c] = (Real)in[i];
}

// Sums the [5][nblocks] partials in a fixed order: thread t takes blocks
// t, t + 1024, ... in order, then a fixed tree over the threads.
__global__ __launch_bounds__(1024) void finalize_sums_kernel(const double *__restrict__ partials, int nblocks,
                                                             double *__restrict__ out) {
  __shared__ double smem[16][kNumSums];
  double v[kNumSums] = {0, 0, 0, 0, 0};
  for (int b = threadIdx.x; b < nblocks; b += 1024) {
    static_for<kNumSums>([&](auto i) { v[i] += partials[(int64_t)i * nblocks + b]; });
  }
  block_sum5(v, smem);
  if (threadIdx.x == 0) {
    static_for<kNumSums>([&](auto i) { out[i] = v[i]; });
  }
}

// Per-box finalisation of a batched step: block b sums box b's partials in
// the order of finalize_sums_kernel, writes the sums to the history slot of
// the box's step (commit) or to its trial slot, then (commit) advances the
// step and flips the buffer index.
__global__ __launch_bounds__(1024) void finalize_batch_kernel(BatchBox *__restrict__ boxes, int commit) {
  __shared__ double smem[16][kNumSums];
  BatchBox &d = boxes[blockIdx.x];
  const int nblocks = d.items;
  double v[kNumSums] = {0, 0, 0, 0, 0};
  for (int b = threadIdx.x; b < nblocks; b += 1024) {
    static_for<kNumSums>([&](auto i) { v[i] += d.partials[(int64_t)i * nblocks + b]; });
  }
  block_sum5(v, smem);
  if (threadIdx.x == 0) {
    double *out = commit ? d.hist + (d.step % kHistoryCap) * kNumSums : d.trial;
    static_for<kNumSums>([&](auto i) { out[i] = v[i]; });
    if (commit) {
      d.step = d.step + 1;
      d.cur = d.cur ^ 1;
    }
  }
}

void launch_finalize_batch(hipStream_t s, BatchBox *d_boxes, int nbox, int commit) {
  hipLaunchKernelGGL(finalize_batch_kernel, dim3(nbox), dim3(1024), 0, s, d_boxes, commit);
  DHIT_HIP(hipGetLastError());
}

// The same sums spread over G blocks when there are many partials: block g
// sums its contiguous slice [g * per, (g + 1) * per) in a fixed order into
// level[g], and the block that finishes last (an agent-scope counter) adds
// level[0..G) in order and resets the counter for the next launch.  The
// result does not depend on which block is last.  level: kFinalizeLevels x 5
// doubles, then the counter at a fixed place whatever G is (launches of
// different G share the work space; zero before the first launch).
__global__ __launch_bounds__(kBlock) void finalize_sums_wide_kernel(const double *__restrict__ partials, int nblocks,
                                                                    int per, double *__restrict__ level,
                                                                    double *__restrict__ out) {
  __shared__ double smem[kWaves][kNumSums];
  __shared__ int last;
  const int lo = blockIdx.x * per, hi = min(nblocks, lo + per);
  double v[kNumSums] = {0, 0, 0, 0, 0};
  for (int b = lo + (int)threadIdx.x; b < hi; b += kBlock) {
    static_for<kNumSums>([&](auto i) { v[i] += partials[(int64_t)i * nblocks + b]; });
  }
  block_sum5(v, smem);
  unsigned *counter = reinterpret_cast<unsigned *>(level + kFinalizeLevels * kNumSums);
  if (threadIdx.x == 0) {
    static_for<kNumSums>([&](auto i) {
      __hip_atomic_store(&level[(int64_t)blockIdx.x * kNumSums + i], v[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    });
    const unsigned done = __hip_atomic_fetch_add(counter, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    last = done == gridDim.x - 1;
  }
  __syncthreads();
  if (last && threadIdx.x < kNumSums) {
    double s = 0.0;
    for (unsigned g = 0; g < gridDim.x; ++g)
      s += __hip_atomic_load(&level[(int64_t)g * kNumSums + threadIdx.x], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    out[threadIdx.x] = s;
    if (threadIdx.x == 0) __hip_atomic_store(counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// Partials one block of the wide finalisation sums.
constexpr int kFinalizePer = 4096;

void launch_finalize_sums(dhit_box &b, const double *partials, int nblocks, double *out) {
  TimedLaunch t(b, DHIT_K_FINALIZE);
  const int g = (nblocks + kFinalizePer - 1) / kFinalizePer;
  if (g > 1 && b.reduce_level && g <= kFinalizeLevels)
    hipLaunchKernelGGL(finalize_sums_wide_kernel, dim3(g), dim3(kBlock), 0, b.stream, partials, nblocks, kFinalizePer,
                       b.reduce_level, out);
  else
    hipLaunchKernelGGL(finalize_sums_kernel, dim3(1), dim3(1024), 0, b.stream, partials, nblocks, out);
  DHIT_HIP(hipGetLastError());
  t.done();
}

void launch_init_equilibrium(dhit_box &b, const double *d_u, const double *d_drho, void *dst) {
  const int blocks = cell_blocks(b.ncell);
  const bool mrt = b.p.method == DHIT_LBE_MRT;
  if (b.p.precision == DHIT_FP64) {
    if (mrt)
      hipLaunchKernelGGL((init_kernel<double, true>), dim3(blocks), dim3(kBlock), 0, b.stream, d_u, d_drho,
                         static_cast<double *>(dst), b.sp, (int)b.ncell);
    else
      hipLaunchKernelGGL((init_kernel<double, false>), dim3(blocks), dim3(kBlock), 0, b.stream, d_u, d_drho,
                         static_cast<double *>(dst), b.sp, (int)b.ncell);
  } else {
    if (mrt)
      hipLaunchKernelGGL((init_kernel<float, true>), dim3(blocks), dim3(kBlock), 0, b.stream, d_u, d_drho,
                         static_cast<float *>(dst), b.sp, (int)b.ncell);
    else
      hipLaunchKernelGGL((init_kernel<float, false>), dim3(blocks), dim3(kBlock), 0, b.stream, d_u, d_drho,
                         static_cast<float *>(dst), b.sp, (int)b.ncell);
  }
  DHIT_HIP(hipGetLastError());
}

void launch_ce_init(dhit_box &b, const double *d_u, const double *d_drho, const double *d_grad, void *dst) {
  const int blocks = cell_blocks(b.ncell);
  if (b.p.precision == DHIT_FP64)
    hipLaunchKernelGGL((ce_init_kernel<double>), dim3(blocks), dim3(kBlock), 0, b.stream, d_u, d_drho, d_grad,
                       static_cast<double *>(dst), b.sp, (int)b.ncell);
  else
    hipLaunchKernelGGL((ce_init_kernel<float>), dim3(blocks), dim3(kBlock), 0, b.stream, d_u, d_drho, d_grad,
                       static_cast<float *>(dst), b.sp, (int)b.ncell);
  DHIT_HIP(hipGetLastError());
}

void launch_hold_velocity(dhit_box &b, void *f, const double *d_u, double *d_drho_out, const double *d_drho_prev,
                          double *d_block_max) {
  const int blocks = cell_blocks(b.ncell);
  const bool mrt = b.p.method == DHIT_LBE_MRT;
  const int n = (int)b.ncell;
  if (b.p.precision == DHIT_FP64) {
    double *g = static_cast<double *>(f);
    if (mrt)
      hipLaunchKernelGGL((hold_velocity_kernel<double, true>), dim3(blocks), dim3(kBlock), 0, b.stream, g, d_u,
                         d_drho_out, d_drho_prev, d_block_max, b.sp, n);
    else
      hipLaunchKernelGGL((hold_velocity_kernel<double, false>), dim3(blocks), dim3(kBlock), 0, b.stream, g, d_u,
                         d_drho_out, d_drho_prev, d_block_max, b.sp, n);
  } else {
    float *g = static_cast<float *>(f);
    if (mrt)
      hipLaunchKernelGGL((hold_velocity_kernel<float, true>), dim3(blocks), dim3(kBlock), 0, b.stream, g, d_u,
                         d_drho_out, d_drho_prev, d_block_max, b.sp, n);
    else
      hipLaunchKernelGGL((hold_velocity_kernel<float, false>), dim3(blocks), dim3(kBlock), 0, b.stream, g, d_u,
                         d_drho_out, d_drho_prev, d_block_max, b.sp, n);
  }
  DHIT_HIP(hipGetLastError());
}

void launch_moments(dhit_box &b, const void *f, double *d_drho, double *d_j, double *d_sums) {
  const int blocks = cell_blocks(b.ncell);
  if (b.p.precision == DHIT_FP64)
    hipLaunchKernelGGL((moments_kernel<double>), dim3(blocks), dim3(kBlock), 0, b.stream,
                       static_cast<const double *>(f), d_drho, d_j, b.sp, (int)b.ncell, b.mesh, b.partials);
  else
    hipLaunchKernelGGL((moments_kernel<float>), dim3(blocks), dim3(kBlock), 0, b.stream,
                       static_cast<const float *>(f), d_drho, d_j, b.sp, (int)b.ncell, b.mesh, b.partials);
  DHIT_HIP(hipGetLastError());
  launch_finalize_sums(b, b.partials, blocks, d_sums);
}

void launch_velocity(dhit_box &b, const void *f, double *d_u) {
  const int blocks = cell_blocks(b.ncell);
  if (b.p.precision == DHIT_FP64)
    hipLaunchKernelGGL((velocity_kernel<double>), dim3(blocks), dim3(kBlock), 0, b.stream,
                       static_cast<const double *>(f), d_u, b.sp, (int)b.ncell);
  else
    hipLaunchKernelGGL((velocity_kernel<float>), dim3(blocks), dim3(kBlock), 0, b.stream,
                       static_cast<const float *>(f), d_u, b.sp, (int)b.ncell);
  DHIT_HIP(hipGetLastError());
}

void launch_pack(dhit_box &b, const void *f, double *d_out) {
  const int64_t total = b.ncell * kQ;
  const int blocks = (int)((total + kBlock - 1) / kBlock);
  if (b.p.precision == DHIT_FP64)
    hipLaunchKernelGGL((pack_kernel<double>), dim3(blocks), dim3(kBlock), 0, b.stream,
                       static_cast<const double *>(f), d_out, b.stride, b.ncell);
  else
    hipLaunchKernelGGL((pack_kernel<float>), dim3(blocks), dim3(kBlock), 0, b.stream,
                       static_cast<const float *>(f), d_out, b.stride, b.ncell);
  DHIT_HIP(hipGetLastError());
}

void launch_unpack(dhit_box &b, const double *d_in, void *f) {
  const int64_t total = b.ncell * kQ;
  const int blocks = (int)((total + kBlock - 1) / kBlock);
  if (b.p.precision == DHIT_FP64)
    hipLaunchKernelGGL((unpack_kernel<double>), dim3(blocks), dim3(kBlock), 0, b.stream, d_in,
                       static_cast<double *>(f), b.stride, b.ncell);
  else
    hipLaunchKernelGGL((unpack_kernel<float>), dim3(blocks), dim3(kBlock), 0, b.stream, d_in,
                       static_cast<float *>(f), b.stride, b.ncell);
  DHIT_HIP(hipGetLastError());
}

// Plain streaming copy: 16 bytes per thread, non-temporal loads and stores
// (the fastest plain copy form measured on MI355X).
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
__global__ __launch_bounds__(kBlock) void copy_kernel(const u32x4 *__restrict__ src, u32x4 *__restrict__ dst,
                                                      int64_t n16) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n16) __builtin_nontemporal_store(__builtin_nontemporal_load(&src[i]), &dst[i]);
}

}  // namespace dhit

extern "C" int32_t device_copy(void *dst, const void *src, int64_t bytes, void *stream) {
  (void)hipGetLastError();
  if (!dst || !src || bytes < 0 || (bytes & 15) || ((reinterpret_cast<uintptr_t>(dst) | reinterpret_cast<uintptr_t>(src)) & 15))
    return DHIT_EINVAL;
  const int64_t n16 = bytes / 16;
  if (n16 == 0) return DHIT_OK;
  const int64_t blocks = (n16 + dhit::kBlock - 1) / dhit::kBlock;
  if (blocks > 0x7fffffff) return DHIT_EINVAL;
  hipLaunchKernelGGL(dhit::copy_kernel, dim3((unsigned)blocks), dim3(dhit::kBlock), 0,
                     static_cast<hipStream_t>(stream), static_cast<const dhit::u32x4 *>(src),
                     static_cast<dhit::u32x4 *>(dst), n16);
  return hipGetLastError() == hipSuccess ? DHIT_OK : DHIT_EDEVICE;
}
