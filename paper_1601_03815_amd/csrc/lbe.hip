// LBE time step: fused pull streaming + collision (Sec. II.B evolution
// equation; BGK or MRT collision), two cells of a row per thread in FP64
// (one 16-byte access per population; one cell if n is odd), one in FP32.
//
// Data layout: 19 population arrays of `stride` elements each (SoA), cell
// index x fastest.  A wavefront covers 64 consecutive runs, so each of the
// 19 gathers and 19 stores is one contiguous access (the pull of a
// population moving in +-x is shifted by one element, still one run; the
// lanes where a two-cell run wraps around the periodic row fix one element
// up).
//
// Phase: the buffer holds post-collision populations.  Thread (cell x)
// gathers g_q(x) = f*_q(x - xi_q), which is the pre-collision state of the
// next time level, takes its moments, collides, and stores f*_q(x).  The
// moments of the new level are reduced per block into `partials` for the
// global FP64 sums.
#include <cstring>

#include "collision.hpp"

namespace dhit {

// Cells a thread updates.  FP64: two consecutive cells of a row, so that
// each population moves as one 16-byte access per lane (measured 0.962
// against 0.980 ms per 256^3 MRT step with one cell); boxes with odd n run
// one cell per thread.  FP32: one cell (runs of 2 or 4 cells measured 15%
// slower: the registers of several cells' collisions cost occupancy that the
// wider accesses do not win back).
template <typename Real>
constexpr int kRunCells = sizeof(Real) == 8 ? 2 : 1;

template <typename Real, int C>
struct Run {
  Real v[C];
};

// Values of one population at the C cells x - SX .. x - SX + C - 1 of a row
// (periodic in x; x is a multiple of C, SX = xi_x of the population), where
// `row` points at element 0 of the source row.  One vector access per lane;
// the lanes at the row's ends, where the run wraps, fix one element up with
// an extra scalar load.
template <int SX, int C, typename Real>
__device__ __forceinline__ Run<Real, C> load_run(const global_t<Real> *row, int x, int n) {
  Run<Real, C> r;
  if constexpr (C == 1) {
    int s = x - SX;
    s = s < 0 ? s + n : (s >= n ? s - n : s);
    r.v[0] = row[s];
  } else if constexpr (SX == 0) {
    __builtin_memcpy(&r, row + x, sizeof(r));
  } else {
    // a wrapping run starts at x (SX = +1, x = 0) or ends at n - 1 (SX = -1)
    const bool wrap = SX > 0 ? x == 0 : x + C == n;
    Run<Real, C> a;
    __builtin_memcpy(&a, row + (wrap ? x : x - SX), sizeof(a));
    if (wrap) {
      const Real e = SX > 0 ? row[n - 1] : row[0];
#pragma unroll
      for (int k = 0; k < C; ++k) {
        if constexpr (SX > 0)
          r.v[k] = k == 0 ? e : a.v[k - 1];
        else
          r.v[k] = k == C - 1 ? e : a.v[k + 1];
      }
    } else {
      r = a;
    }
  }
  return r;
}

// Update of the C cells starting at `cell` (same row); adds their moments
// to the block's sums v.
template <int K, int C, typename Real>
__device__ __forceinline__ void lbe_run(const global_t<Real> *__restrict__ src, global_t<Real> *__restrict__ dst,
                                        const StepParams &p, int cell, double (&v)[kNumSums]) {
  const int n = p.n;
  const int64_t stride = p.stride;
  const int x = cell % n;
  const int t = cell / n;
  const int y = t % n;
  const int z = t / n;
  const int row = cell - x;
  const AxisOff oy = axis_offsets(y, n, n), oz = axis_offsets(z, n, n * n);
  Real f[C][kQ];
  static_for<kQ>([&](auto q) {
    // source row of the cells - xi_q
    int off = row;
    if constexpr (kCy[q] == 1) off += oy.dn;
    if constexpr (kCy[q] == -1) off += oy.up;
    if constexpr (kCz[q] == 1) off += oz.dn;
    if constexpr (kCz[q] == -1) off += oz.up;
    const Run<Real, C> r = load_run<kCx[q], C>(src + (int64_t)q * stride + off, x, n);
#pragma unroll
    for (int k = 0; k < C; ++k) f[k][q] = r.v[k];
  });
#pragma unroll
  for (int k = 0; k < C; ++k) {
    Real drho, jx, jy, jz;
    cell_moments<Real>(f[k], drho, jx, jy, jz);
    sums_of_cell<Real>(drho, jx, jy, jz, p.inv_rho0, v);
    collide<K, Real>(f[k], drho, jx, jy, jz, p);
  }
  // the new state is read only by the next step: stream it past the caches
  static_for<kQ>([&](auto q) {
    global_t<Real> *d = dst + (int64_t)q * stride + cell;
    if constexpr (C == 1) {
      __builtin_nontemporal_store(f[0][q], d);
    } else {
      typedef Real Vec __attribute__((ext_vector_type(C)));
      Vec w;
#pragma unroll
      for (int k = 0; k < C; ++k) w[k] = f[k][q];
      __builtin_nontemporal_store(w, reinterpret_cast<global_t<Vec> *>(d));
    }
  });
}

// One launch advances one or many boxes: work item = a run of kBlock * C
// cells of one box of the device table `boxes` (sorted by item_begin),
// where C is 1 or kRunCells<Real> for the whole launch.  A single box is a
// table of one entry.  The per-item partial sums are laid out as a block
// launch's would be.
template <int K, typename Real, int C>
__global__ __launch_bounds__(kBlock) void lbe_kernel(const BatchBox *__restrict__ boxes, int nbox, int total_items) {
  for (int it = blockIdx.x; it < total_items; it += gridDim.x) {
    const int b = find_batch_box(boxes, nbox, it);
    const BatchBox &d = boxes[b];
    const int local = it - d.item_begin;
    const int cell = (local * kBlock + threadIdx.x) * C;
    double v[kNumSums] = {0, 0, 0, 0, 0};
    if (cell < d.ncell)
      lbe_run<K, C, Real>(to_global(static_cast<const Real *>(d.f[d.cur])), to_global(static_cast<Real *>(d.f[d.cur ^ 1])),
                          d.sp, cell, v);
    write_block_partials(v, d.partials, d.items, local);
    __syncthreads();
  }
}

int lbe_cells_per_thread(int n, int precision) {
  const int c = precision == DHIT_FP64 ? kRunCells<double> : kRunCells<float>;
  return n % c == 0 ? c : 1;
}

int lbe_items(int64_t ncell, int cells_per_thread) {
  return (int)((ncell / cells_per_thread + kBlock - 1) / kBlock);
}

template <typename Real, int C>
static void lbe_launch_typed(hipStream_t s, int method, const BatchBox *d_boxes, int nbox, int total_items, int grid) {
  if (method == DHIT_LBE_BGK)
    hipLaunchKernelGGL((lbe_kernel<kBGK, Real, C>), dim3(grid), dim3(kBlock), 0, s, d_boxes, nbox, total_items);
  else
    hipLaunchKernelGGL((lbe_kernel<kMRT, Real, C>), dim3(grid), dim3(kBlock), 0, s, d_boxes, nbox, total_items);
}

void launch_lbe_batch(hipStream_t s, int method, int precision, int cells_per_thread, const BatchBox *d_boxes,
                      int nbox, int total_items, int grid) {
  if (precision == DHIT_FP64) {
    if (cells_per_thread == kRunCells<double>)
      lbe_launch_typed<double, kRunCells<double>>(s, method, d_boxes, nbox, total_items, grid);
    else
      lbe_launch_typed<double, 1>(s, method, d_boxes, nbox, total_items, grid);
  } else {
    if (cells_per_thread == kRunCells<float>)
      lbe_launch_typed<float, kRunCells<float>>(s, method, d_boxes, nbox, total_items, grid);
    else
      lbe_launch_typed<float, 1>(s, method, d_boxes, nbox, total_items, grid);
  }
  DHIT_HIP(hipGetLastError());
}

// The two one-box tables of an LBE box (entry c steps from f[c] to f[1 - c]).
void lbe_table_entries(const dhit_box &b, BatchBox (&e)[2]) {
  const int cpt = lbe_cells_per_thread(b.n, b.p.precision);
  for (int c = 0; c < 2; ++c) {
    std::memset(&e[c], 0, sizeof(BatchBox));
    e[c].f[0] = b.f[0];
    e[c].f[1] = b.f[1];
    e[c].sp = b.sp;
    e[c].ncell = (int)b.ncell;
    e[c].item_begin = 0;
    e[c].items = lbe_items(b.ncell, cpt);
    e[c].partials = b.partials;
    e[c].hist = b.hist;
    e[c].cur = c;
  }
}

void launch_lbe_step(dhit_box &b, const void *src, void *dst, double *sums_out) {
  if (!b.step_table) throw Error(DHIT_EINVAL, "box has no step table");
  int entry;
  if (src == b.f[0] && dst == b.f[1]) entry = 0;
  else if (src == b.f[1] && dst == b.f[0]) entry = 1;
  else throw Error(DHIT_EINVAL, "LBE step between buffers that are not the box's");
  const int cpt = lbe_cells_per_thread(b.n, b.p.precision);
  const int items = lbe_items(b.ncell, cpt);
  {
    TimedLaunch t(b, DHIT_K_LBE);
    launch_lbe_batch(b.stream, b.p.method, b.p.precision, cpt, b.step_table + entry, 1, items, items);
    t.done();
  }
  launch_finalize_sums(b, b.partials, items, sums_out);
}

}  // namespace dhit
