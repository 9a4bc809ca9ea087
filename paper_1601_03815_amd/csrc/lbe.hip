// LBE time step: fused pull streaming + collision (Sec. II.B evolution
// equation; BGK or MRT collision), one cell per thread.
//
// Data layout: 19 population arrays of `stride` elements each (SoA), cell
// index x fastest.  A wavefront covers 64 consecutive cells, so each of the
// 19 gathers and 19 stores is one contiguous 64-element run (the pull of a
// population moving in +-x is shifted by one element, still one run).
//
// Phase: the buffer holds post-collision populations.  Thread (cell x)
// gathers g_q(x) = f*_q(x - xi_q), which is the pre-collision state of the
// next time level, takes its moments, collides, and stores f*_q(x).  The
// moments of the new level are reduced per block into `partials` for the
// global FP64 sums.
#include "collision.hpp"

namespace dhit {

// Update of one cell; adds its moments to the block's sums v.
template <int C, typename Real>
__device__ __forceinline__ void lbe_cell(const global_t<Real> *__restrict__ src, global_t<Real> *__restrict__ dst, const StepParams &p,
                                         int cell, double (&v)[kNumSums]) {
  const int n = p.n;
  const int64_t stride = p.stride;
  const int x = cell % n;
  const int t = cell / n;
  const int y = t % n;
  const int z = t / n;
  const AxisOff ox = axis_offsets(x, n, 1), oy = axis_offsets(y, n, n), oz = axis_offsets(z, n, n * n);
  Real f[kQ];
  static_for<kQ>([&](auto q) {
    // source cell x - xi_q
    int off = 0;
    if constexpr (kCx[q] == 1) off += ox.dn;
    if constexpr (kCx[q] == -1) off += ox.up;
    if constexpr (kCy[q] == 1) off += oy.dn;
    if constexpr (kCy[q] == -1) off += oy.up;
    if constexpr (kCz[q] == 1) off += oz.dn;
    if constexpr (kCz[q] == -1) off += oz.up;
    f[q] = src[(int64_t)q * stride + (cell + off)];
  });
  Real drho, jx, jy, jz;
  cell_moments<Real>(f, drho, jx, jy, jz);
  sums_of_cell<Real>(drho, jx, jy, jz, p.inv_rho0, v);
  collide<C, Real>(f, drho, jx, jy, jz, p);
  // the new state is read only by the next step: stream it past the caches
  static_for<kQ>([&](auto q) { __builtin_nontemporal_store(f[q], &dst[(int64_t)q * stride + cell]); });
}

template <int C, typename Real>
__global__ __launch_bounds__(kBlock) void lbe_pull_kernel(const Real *__restrict__ src, Real *__restrict__ dst,
                                                          StepParams p, int ncell, double *__restrict__ partials) {
  const int cell = blockIdx.x * kBlock + threadIdx.x;
  double v[kNumSums] = {0, 0, 0, 0, 0};
  if (cell < ncell) lbe_cell<C, Real>(to_global(src), to_global(dst), p, cell, v);
  write_block_partials(v, partials, gridDim.x, blockIdx.x);
}

// Many boxes in one persistent launch: work item i is block-sized run of
// cells of one box (the same grouping as the single-box launch, so the
// per-item partial sums equal that launch's block partials).
template <int C, typename Real>
__global__ __launch_bounds__(kBlock) void lbe_batch_kernel(BatchBox *__restrict__ boxes, int nbox, int total_items) {
  for (int it = blockIdx.x; it < total_items; it += gridDim.x) {
    const int b = find_batch_box(boxes, nbox, it);
    const BatchBox &d = boxes[b];
    const int local = it - d.item_begin;
    const int cell = local * kBlock + threadIdx.x;
    double v[kNumSums] = {0, 0, 0, 0, 0};
    if (cell < d.ncell)
      lbe_cell<C, Real>(to_global(static_cast<const Real *>(d.f[d.cur])), to_global(static_cast<Real *>(d.f[d.cur ^ 1])), d.sp,
                        cell, v);
    write_block_partials(v, d.partials, d.items, local);
    __syncthreads();
  }
}

void launch_lbe_batch(hipStream_t s, int method, int precision, BatchBox *d_boxes, int nbox, int total_items,
                      int grid) {
  if (precision == DHIT_FP64) {
    if (method == DHIT_LBE_BGK)
      hipLaunchKernelGGL((lbe_batch_kernel<kBGK, double>), dim3(grid), dim3(kBlock), 0, s, d_boxes, nbox, total_items);
    else
      hipLaunchKernelGGL((lbe_batch_kernel<kMRT, double>), dim3(grid), dim3(kBlock), 0, s, d_boxes, nbox, total_items);
  } else {
    if (method == DHIT_LBE_BGK)
      hipLaunchKernelGGL((lbe_batch_kernel<kBGK, float>), dim3(grid), dim3(kBlock), 0, s, d_boxes, nbox, total_items);
    else
      hipLaunchKernelGGL((lbe_batch_kernel<kMRT, float>), dim3(grid), dim3(kBlock), 0, s, d_boxes, nbox, total_items);
  }
  DHIT_HIP(hipGetLastError());
}

template <typename Real>
static void lbe_step_typed(dhit_box &b, const void *src, void *dst, double *sums_out) {
  const int blocks = cell_blocks(b.ncell);
  const Real *s = static_cast<const Real *>(src);
  Real *d = static_cast<Real *>(dst);
  TimedLaunch t(b, DHIT_K_LBE);
  if (b.p.method == DHIT_LBE_BGK)
    hipLaunchKernelGGL((lbe_pull_kernel<kBGK, Real>), dim3(blocks), dim3(kBlock), 0, b.stream, s, d, b.sp,
                       (int)b.ncell, b.partials);
  else
    hipLaunchKernelGGL((lbe_pull_kernel<kMRT, Real>), dim3(blocks), dim3(kBlock), 0, b.stream, s, d, b.sp,
                       (int)b.ncell, b.partials);
  DHIT_HIP(hipGetLastError());
  t.done();
  launch_finalize_sums(b, b.partials, blocks, sums_out);
}

void launch_lbe_step(dhit_box &b, const void *src, void *dst, double *sums_out) {
  if (b.p.precision == DHIT_FP64)
    lbe_step_typed<double>(b, src, dst, sums_out);
  else
    lbe_step_typed<float>(b, src, dst, sums_out);
}

}  // namespace dhit
