// Host-side runtime of the library: the box object and the launchers that
// the C ABI (box.hip) calls.  Not part of the public interface.
#pragma once

#include <hip/hip_runtime.h>
#include <hipfft/hipfft.h>

#include <cstdint>
#include <stdexcept>
#include <string>

#include "../../include/dhit.h"

namespace dhit {

// Error carrying an ABI status code; converted at the C boundary.
struct Error : std::runtime_error {
  int32_t code;
  Error(int32_t c, const std::string &m) : std::runtime_error(m), code(c) {}
};

#define DHIT_HIP(expr)                                                                       \
  do {                                                                                       \
    hipError_t e_ = (expr);                                                                  \
    if (e_ != hipSuccess)                                                                    \
      throw ::dhit::Error(DHIT_EDEVICE, std::string(#expr " failed: ") + hipGetErrorString(e_)); \
  } while (0)

// Parameters of the collision / update passed to kernels by value.
struct StepParams {
  int n;
  int64_t stride;      // elements between consecutive population arrays
  double rho0, inv_rho0;
  // BGK-LBE: omega = 1/tau
  double omega;
  // MRT-LBE: r[k] = s_k / norm_k (0 for conserved rows), equilibrium constants
  double r[19];
  double w_eps, w_epsj, w_xx;
  // DUGKS: tau, dt, h and the combination coefficients
  double tau, dt, h;
  double a_bp, b_bp;   // fbp = a_bp f~ + b_bp f^eq   (2tau-h)/(2tau+dt), 3h/(2tau+dt)
  double alpha, beta;  // f_face = alpha fbar + beta f^eq   2tau/(2tau+h), h/(2tau+h)
};

constexpr int kHistoryCap = 4096;
// Blocks of the wide finalisation of the per-step sums at most (each sums
// 4096 block partials); its work space is kFinalizeLevels * 5 doubles and a
// counter that must be zero before the first launch.
constexpr int kFinalizeLevels = 64;
constexpr int kFinalizeDoubles = kFinalizeLevels * 5 + 8;

// Geometry tables of a stretched DUGKS mesh (set_mesh), laid out
// [axis][table][n] doubles; for cell i of an axis with widths w:
//   width w_i, 1/w_i; for the face between i and i+1: lam = w_i/(w_i + w_{i+1})
//   (position of the face between the two centres) and 1/(c_{i+1} - c_i)
//   = 2/(w_i + w_{i+1}); 1/(c_{i+1} - c_{i-1}) for the central difference.
enum MeshTable { kMeshWidth = 0, kMeshInvWidth, kMeshLam, kMeshInvGap, kMeshInvSpan, kMeshTables };

// One box of a batched launch (device-resident table entry).  `cur` and
// `step` live on the device so that a captured graph can be replayed for
// any number of steps: the per-box finalisation writes the history slot of
// `step`, then advances `step` and flips `cur`.
struct BatchBox {
  void *f[2];          // population buffers; f[cur] holds the state
  StepParams sp;
  int ncell;
  int item_begin;      // first work item of the box in the batch
  int items;           // work items of the box (= blocks of its single-box launch)
  int tiles_x, tiles_y, nz_chunk;  // DUGKS tiling
  // DUGKS: with tail_split > 1 the chunk items from tail_from on are each
  // cut into tail_split parts in z (see ItemPlanes in dugks_fused.hip)
  int tail_from, tail_split;
  double *partials;    // the box's per-item partial sums, [5][items]
  double *hist;        // the box's history of global sums, [kHistoryCap][5]
  double *trial;       // where a trial (uncommitted) step writes its sums, [5]
  int cur;
  int pad_;
  int64_t step;
};

// Box of work item `it`: the last box whose first item is <= it.
__device__ __forceinline__ int find_batch_box(const BatchBox *boxes, int nbox, int it) {
  int lo = 0, hi = nbox - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (boxes[mid].item_begin <= it) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

struct SpectrumWork;  // spectrum.hip

// Ring of event pairs bracketing kernel launches (see set_kernel_timing).
struct KernelTimer {
  static constexpr int kCap = 8192;
  bool enabled = false;
  hipEvent_t start[kCap] = {}, stop[kCap] = {};
  int kind[kCap] = {};
  bool created = false;
  int64_t count = 0;  // launches recorded since the last read
};

}  // namespace dhit

struct dhit_box {
  dhit_params p{};
  int n = 0;
  int64_t ncell = 0;
  int64_t stride = 0;        // padded per-population array length (elements)
  size_t elem = 8;           // bytes per stored value
  void *f[2] = {nullptr, nullptr};
  bool own_f = false;
  int cur = 0;               // f[cur] holds the state
  hipStream_t stream = nullptr;
  bool own_stream = false;
  double *partials = nullptr;  // [5][max_blocks]
  double *reduce_level = nullptr;  // work space of the wide finalisation (kFinalizeDoubles), NULL: one block
  int max_blocks = 0;
  double *hist = nullptr;      // [kHistoryCap][5]
  int64_t steps = 0;
  void *scratch = nullptr;     // DUGKS two-pass transform field
  double *mesh = nullptr;      // stretched-mesh tables [3][kMeshTables][n] (DUGKS), NULL = unit cells
  dhit::BatchBox *step_table = nullptr;  // LBE and fused DUGKS steps: the box as a one-entry table per buffer phase [2]
  bool own_step_table = false;
  dhit::StepParams sp{};
  dhit::SpectrumWork *spec = nullptr;
  dhit::KernelTimer *timer = nullptr;
};

namespace dhit {

// Sets the thread's message returned by dhit_last_error().
void set_last_error(const std::string &m);

// Launchers (each enqueues on b.stream; src/dst are population buffers).
void launch_lbe_step(dhit_box &b, const void *src, void *dst, double *sums_out);
void launch_dugks_step(dhit_box &b, const void *src, void *dst, double *sums_out);
void launch_dugks_fused(dhit_box &b, const void *src, void *dst, double *sums_out);
// Blocks of the fused DUGKS launch for an n^3 box (and its tiling).
int fused_dugks_blocks(const dhit_params &p, int *width, int *tiles_x, int *tiles_y, int *nz_chunk);
// Work split of a box's fused DUGKS launch: tile width, tiling, z-chunk,
// work items (the chunk items, or with a cut last round tail_from whole
// chunks and the (chunk items - tail_from) * tail_split parts, laid out
// per XCD) and grid (one block per item).
struct FusedPlan {
  int width, tiles_x, tiles_y, chunk, items, tail_from, tail_split, grid;
};
FusedPlan fused_plan(const dhit_params &p);
// The same for a device holding `slots` blocks of the kernel at once (no
// device query), and the tile and planes [z0, z0 + planes) of one item.
FusedPlan fused_plan_for(const dhit_params &p, int slots);
void fused_item_planes(const FusedPlan &f, int n, int item, int *tile, int *z0, int *planes);
void launch_init_equilibrium(dhit_box &b, const double *d_u, const double *d_drho, void *dst);
void launch_moments(dhit_box &b, const void *f, double *d_drho, double *d_j, double *d_sums);
// One pass of the LBE initial-state iteration on state f (in place): momentum
// back to rho0 u, density and non-equilibrium kept; optional drho output and
// per-block largest |drho - drho_prev| (cell_blocks(ncell) entries).
void launch_hold_velocity(dhit_box &b, void *f, const double *d_u, double *d_drho_out, const double *d_drho_prev,
                          double *d_block_max);
void launch_pack(dhit_box &b, const void *f, double *d_out);     // state -> [19][ncell] double
void launch_unpack(dhit_box &b, const double *d_in, void *f);    // [19][ncell] double -> state
void launch_finalize_sums(dhit_box &b, const double *partials, int nblocks, double *out);
void timer_free(dhit_box &b);
void launch_velocity(dhit_box &b, const void *f, double *d_u);   // u = j / rho0, [3][ncell]

// Batched launches (batch.hip drives them).  LBE: one launch over the work
// items (runs of kBlock * cells_per_thread cells) of a device table of boxes;
// cells_per_thread is lbe_cells_per_thread() of every box of the launch, or 1.
void launch_lbe_batch(hipStream_t s, int method, int precision, int cells_per_thread, const BatchBox *d_boxes,
                      int nbox, int total_items, int grid);
int lbe_cells_per_thread(int n, int precision);
int lbe_items(int64_t ncell, int cells_per_thread);
void lbe_table_entries(const dhit_box &b, BatchBox (&e)[2]);
// One launch of the fused DUGKS kernel (tile width w) over the work items
// of a device table of boxes (the largest of side max_n); a single box is a
// table of one entry.
void launch_dugks_batch(hipStream_t s, int precision, int w, int max_n, const BatchBox *d_boxes, int nbox,
                        int total_items, int grid);
// The two one-entry tables of a box (entry c steps from f[c] to f[1 - c]),
// and a launch that writes two entries given by value to device memory.
void fused_table_entries(const dhit_box &b, BatchBox (&e)[2]);
void launch_store_table(hipStream_t s, const BatchBox (&e)[2], BatchBox *dst);
void launch_finalize_batch(hipStream_t s, BatchBox *d_boxes, int nbox, int commit);
int fused_tile_width_of(int precision);
// Blocks of the fused DUGKS kernel of this precision and tile width that
// one compute unit holds at once.
int fused_resident_blocks_of(int precision, int w);
int fused_default_chunk(int n);
int fused_balanced_chunk(int n, int tiles_xy, int slots);
int fused_auto_chunk(const dhit_params &p);
int fused_dugks_items(int n, int w, int chunk, int *tiles_x, int *tiles_y);

// Spectrum (spectrum.hip)
void spectrum_compute(dhit_box &b, double *E_host, int kmax, double *stats_host);
void spectrum_free(dhit_box &b);
int64_t spectrum_work_bytes(int n);  // arrays + hipFFT work areas of an n^3 box's spectrum work space
void vorticity_compute(dhit_box &b, double *omega_host);  // omega = curl(j/rho0), host [3][ncell]
void pressure_compute(dhit_box &b, const double *u_host, double *drho_host);  // drho = 3 p of a host u
// Spectral velocity gradient of a device field u[3][ncell] into
// grad[3 a + b][ncell] = d_a u_b (device).
void gradient_compute(dhit_box &b, const double *d_u, double *d_grad);
// DUGKS consistent start: f~ = f^eq(drho, rho0 u) + (1 + dt/(2 tau)) f1 with
// the first-order Chapman-Enskog part f1 of the velocity gradient (device
// fields: u [3][ncell], drho [ncell] or NULL, grad [9][ncell]).
void launch_ce_init(dhit_box &b, const double *d_u, const double *d_drho, const double *d_grad, void *dst);

// Event bracket around one kernel launch when timing is enabled:
//   TimedLaunch t(b, DHIT_K_LBE); hipLaunchKernelGGL(...); t.done();
struct TimedLaunch {
  dhit_box &b;
  int slot = -1;
  TimedLaunch(dhit_box &box, int kind);
  void done();
};

// Number of blocks of a one-cell-per-thread launch over the box.
inline int cell_blocks(int64_t ncell) { return (int)((ncell + 255) / 256); }

}  // namespace dhit
