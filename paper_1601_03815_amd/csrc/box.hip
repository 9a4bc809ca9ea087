// C ABI of the library (declared in include/dhit.h): parameter handling,
// box lifetime, buffers, and the step loops.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "lattice.hpp"
#include "runtime.hpp"

namespace {

thread_local std::string g_last_error;

void set_error(const std::string &m) { g_last_error = m; }

}  // namespace

void dhit::set_last_error(const std::string &m) { set_error(m); }

namespace {

// hipGetLastError() reports the last failing HIP call of the thread, including
// calls made outside this library (by the host program or another library
// sharing the runtime) and calls whose status is deliberately ignored during
// clean-up.  Every entry point clears that state first, so a launch check
// inside the library reports the library's own launch.  DHIT_DEBUG=1 prints
// what was cleared.
void clear_stale_hip_error() {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess && std::getenv("DHIT_DEBUG"))
    std::fprintf(stderr, "dhit: cleared a pending HIP error at entry: %s\n", hipGetErrorString(e));
}

template <class F>
int32_t guarded(F &&f) {
  try {
    g_last_error.clear();
    clear_stale_hip_error();
    return f();
  } catch (const dhit::Error &e) {
    set_error(e.what());
    return e.code;
  } catch (const std::bad_alloc &) {
    set_error("host allocation failed");
    return DHIT_ENOMEM;
  } catch (const std::exception &e) {
    set_error(e.what());
    return DHIT_EINVAL;
  }
}

[[noreturn]] void fail(int32_t code, const std::string &m) { throw dhit::Error(code, m); }

// Elements between consecutive population arrays: the cell count rounded up
// to 256 bytes' worth of elements plus a shift, so that the 19 arrays start
// at staggered offsets modulo large powers of two (cell counts such as 256^3
// would otherwise place all 19 streams on the same memory channels).  The
// shift suits each kernel's access pattern (measured at 256^3): 3 KiB for the
// LBE, whose 19 streams advance together (in sweeps of 0.5 to 9 KiB the FP64
// step was fastest at 3 KiB: 1% faster than at 1 KiB, 4% than at 4 KiB;
// FP32 alike within 1%), 16 KiB for the DUGKS march (1 KiB made it 4% slower).
int64_t padded_stride(int64_t ncell, size_t elem, int method) {
  const int64_t align = 256 / (int64_t)elem;
  const int64_t shift = (method == DHIT_DUGKS ? 16384 : 3072) / (int64_t)elem;
  return ((ncell + align - 1) / align) * align + shift;
}

void validate(const dhit_params &p) {
  if (p.n < 4 || p.n > 1024) fail(DHIT_EINVAL, "n must be in [4, 1024]");
  if (p.method < DHIT_LBE_BGK || p.method > DHIT_DUGKS) fail(DHIT_EINVAL, "unknown method");
  if (p.precision != DHIT_FP64 && p.precision != DHIT_FP32) fail(DHIT_EINVAL, "unknown precision");
  if (p.variant != DHIT_VARIANT_DEFAULT && p.variant != DHIT_VARIANT_TWO_PASS) fail(DHIT_EINVAL, "unknown variant");
  if (p.tile_width != 0 && p.tile_width != 16 && p.tile_width != 32) fail(DHIT_EINVAL, "tile_width must be 0, 16 or 32");
  if (p.z_chunk < -p.n || p.z_chunk > p.n) fail(DHIT_EINVAL, "z_chunk must be in [-n, n]");
  if (!(p.nu > 0) || !std::isfinite(p.nu)) fail(DHIT_EINVAL, "nu must be positive and finite");
  if (!(p.rho0 > 0) || !std::isfinite(p.rho0)) fail(DHIT_EINVAL, "rho0 must be positive and finite");
  if (p.method == DHIT_DUGKS) {
    if (!(p.dt > 0) || p.dt * std::sqrt(2.0) > 1.0 + 1e-12)
      fail(DHIT_EINVAL, "DUGKS needs 0 < dt and CFL dt*sqrt(2) <= 1");
  } else if (p.dt != 1.0) {
    fail(DHIT_EINVAL, "LBE requires dt = 1 (dt = dx in lattice units)");
  }
  if ((p.f_a == nullptr) != (p.f_b == nullptr)) fail(DHIT_EINVAL, "f_a and f_b must both be given or both NULL");
  if (p.f_a && ((reinterpret_cast<uintptr_t>(p.f_a) | reinterpret_cast<uintptr_t>(p.f_b)) & 255))
    fail(DHIT_EINVAL, "caller buffers must be 256-byte aligned");
  const double rates[] = {p.s1, p.s2, p.s4, p.s9, p.s10, p.s13, p.s16};
  if (p.method == DHIT_LBE_MRT)
    for (double s : rates)
      if (!(s > 0 && s < 2)) fail(DHIT_EINVAL, "MRT rates must lie in (0, 2)");
}

void derive_step_params(dhit_box &b) {
  const dhit_params &p = b.p;
  dhit::StepParams &s = b.sp;
  std::memset(&s, 0, sizeof(s));
  s.n = b.n;
  s.stride = b.stride;
  s.rho0 = p.rho0;
  s.inv_rho0 = 1.0 / p.rho0;
  // BGK-LBE: nu = (tau - 1/2)/3 with dt = 1
  s.omega = 1.0 / (3.0 * p.nu + 0.5);
  // MRT: diagonal of S in the order of Sec. II.B, divided by the row norms
  const double S[19] = {0, p.s1, p.s2, 0, p.s4, 0, p.s4, 0, p.s4, p.s9, p.s10, p.s9, p.s10,
                        p.s13, p.s13, p.s13, p.s16, p.s16, p.s16};
  for (int k = 0; k < 19; ++k) s.r[k] = dhit::mrt_conserved(k) ? 0.0 : S[k] / (double)dhit::mrt_norm(k);
  s.w_eps = p.w_eps;
  s.w_epsj = p.w_epsj;
  s.w_xx = p.w_xx;
  // DUGKS: tau = nu / RT
  s.tau = 3.0 * p.nu;
  s.dt = p.dt;
  s.h = 0.5 * p.dt;
  s.a_bp = (2.0 * s.tau - s.h) / (2.0 * s.tau + s.dt);
  s.b_bp = 3.0 * s.h / (2.0 * s.tau + s.dt);
  s.alpha = 2.0 * s.tau / (2.0 * s.tau + s.h);
  s.beta = s.h / (2.0 * s.tau + s.h);
}

// DUGKS transform field, needed by the two-pass variant only.
int64_t scratch_bytes_of(const dhit_params &p, int64_t pop_bytes) {
  return (p.method == DHIT_DUGKS && p.variant == DHIT_VARIANT_TWO_PASS) ? pop_bytes : 0;
}

// The step's one-box tables of an LBE box or a fused-DUGKS box (the box as
// a table of one entry for each buffer phase, see lbe_table_entries and
// fused_table_entries).
int64_t step_table_bytes(const dhit_params &p) {
  return (p.method != DHIT_DUGKS || p.variant == DHIT_VARIANT_DEFAULT) ? 2 * (int64_t)sizeof(dhit::BatchBox) : 0;
}

// Blocks (and so partial-sum slots) of the largest per-step launch.
int64_t reduction_blocks(const dhit_params &p) {
  const int64_t ncell = (int64_t)p.n * p.n * p.n;
  int64_t blocks = (ncell + 255) / 256;
  if (p.method == DHIT_DUGKS) {
    const int64_t f = dhit::fused_dugks_blocks(p, nullptr, nullptr, nullptr, nullptr);
    if (f > blocks) blocks = f;
  }
  return blocks;
}

void check_finite(const double *s, int count) {
  for (int i = 0; i < count; ++i)
    if (!std::isfinite(s[i])) fail(DHIT_ENONFINITE, "a global reduction is not finite (the run blew up)");
}

void require_box(const dhit_box *b) {
  if (!b) fail(DHIT_EINVAL, "null box");
}

}  // namespace

// Work space of step_noalloc: the per-block partial sums of one step's
// global reduction, plus a slot where the finalisation writes the sums when
// the caller wants none.  A file-scope device array, so that the entry point
// allocates nothing; every GPU the library runs on holds its own copy until
// the process ends.  In host code `scratch` names a host-side stand-in: the
// device address comes from hipGetSymbolAddress, taken once per device with
// that device current and kept in g_scratch_ptr.
constexpr int64_t kNoallocPartials = 131072;                                 // block partial slots
constexpr int64_t kNoallocLevel = 5 * kNoallocPartials;                        // wide finalisation work space
constexpr int64_t kNoallocDiscard = kNoallocLevel + dhit::kFinalizeDoubles;    // sums nobody asked for
constexpr int64_t kNoallocTable = kNoallocDiscard + 8;                         // the step tables
constexpr int64_t kNoallocDoubles = kNoallocTable + (2 * sizeof(dhit::BatchBox) + 7) / 8;
static __device__ __align__(256) double scratch[kNoallocDoubles];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device.
double *scratch_on_current_device() {
  int dev = 0;
  DHIT_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) fail(DHIT_EDEVICE, "device index out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *ptr = nullptr;
    DHIT_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) fail(DHIT_EDEVICE, "no device address for the step_noalloc work space");
    g_scratch_ptr[dev] = static_cast<double *>(ptr);
  }
  return g_scratch_ptr[dev];
}

}  // namespace

extern "C" {

int32_t default_params(int32_t n, int32_t method, int32_t precision, double nu, dhit_params *out) {
  return guarded([&]() -> int32_t {
    if (!out) fail(DHIT_EINVAL, "null output");
    dhit_params p;
    std::memset(&p, 0, sizeof(p));
    p.n = n;
    p.method = method;
    p.precision = precision;
    p.variant = DHIT_VARIANT_DEFAULT;
    p.nu = nu;
    p.rho0 = 1.0;
    p.dt = method == DHIT_DUGKS ? 0.5 : 1.0;
    p.s1 = 1.19;
    p.s2 = 1.4;
    p.s4 = 1.2;
    p.s9 = 1.0 / (3.0 * nu + 0.5);
    p.s10 = 1.4;
    p.s13 = p.s9;
    p.s16 = 1.98;
    p.w_eps = 0.0;
    p.w_epsj = -475.0 / 63.0;
    p.w_xx = 0.0;
    *out = p;
    return DHIT_OK;
  });
}

int64_t population_buffer_bytes(const dhit_params *p) {
  int64_t r = 0;
  int32_t st = guarded([&]() -> int32_t {
    if (!p) fail(DHIT_EINVAL, "null params");
    if (p->n < 4 || p->n > 1024) fail(DHIT_EINVAL, "n must be in [4, 1024]");
    const size_t elem = p->precision == DHIT_FP32 ? 4 : 8;
    const int64_t ncell = (int64_t)p->n * p->n * p->n;
    r = 19 * padded_stride(ncell, elem, p->method) * (int64_t)elem;
    return DHIT_OK;
  });
  return st == DHIT_OK ? r : st;
}

int64_t box_bytes(const dhit_params *p) {
  int64_t pop = population_buffer_bytes(p);
  if (pop < 0) return pop;
  return 2 * pop + (reduction_blocks(*p) * 5 + dhit::kFinalizeDoubles) * 8 + dhit::kHistoryCap * 5 * 8 +
         scratch_bytes_of(*p, pop) +
         step_table_bytes(*p);
}

int64_t spectrum_bytes(const dhit_params *p) {
  int64_t r = 0;
  int32_t st = guarded([&]() -> int32_t {
    if (!p) fail(DHIT_EINVAL, "null params");
    if (p->n < 4 || p->n > 1024) fail(DHIT_EINVAL, "n must be in [4, 1024]");
    r = dhit::spectrum_work_bytes(p->n);
    return DHIT_OK;
  });
  return st == DHIT_OK ? r : st;
}

int32_t create_box(const dhit_params *pp, dhit_box **out) {
  return guarded([&]() -> int32_t {
    if (!pp || !out) fail(DHIT_EINVAL, "null argument");
    *out = nullptr;
    validate(*pp);
    dhit_box *b = new dhit_box();
    try {
      b->p = *pp;
      if (b->p.method == DHIT_DUGKS && b->p.z_chunk == 0) b->p.z_chunk = dhit::fused_auto_chunk(b->p);
      b->n = pp->n;
      b->ncell = (int64_t)pp->n * pp->n * pp->n;
      b->elem = pp->precision == DHIT_FP32 ? 4 : 8;
      b->stride = padded_stride(b->ncell, b->elem, b->p.method);
      const int64_t pop = 19 * b->stride * (int64_t)b->elem;
      if (pp->stream) {
        b->stream = static_cast<hipStream_t>(pp->stream);
      } else {
        DHIT_HIP(hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking));
        b->own_stream = true;
      }
      if (pp->f_a) {
        b->f[0] = pp->f_a;
        b->f[1] = pp->f_b;
        b->own_f = false;
      } else {
        b->own_f = true;
        if (hipMalloc(&b->f[0], pop) != hipSuccess || hipMalloc(&b->f[1], pop) != hipSuccess)
          fail(DHIT_ENOMEM, "cannot allocate population buffers");
      }
      b->max_blocks = (int)reduction_blocks(b->p);
      // block partials, then the wide finalisation's level sums and counter
      if (hipMalloc(&b->partials, ((size_t)b->max_blocks * 5 + dhit::kFinalizeDoubles) * sizeof(double)) != hipSuccess ||
          hipMalloc(&b->hist, (size_t)dhit::kHistoryCap * 5 * sizeof(double)) != hipSuccess)
        fail(DHIT_ENOMEM, "cannot allocate reduction buffers");
      if (scratch_bytes_of(*pp, pop) > 0) {
        if (hipMalloc(&b->scratch, scratch_bytes_of(*pp, pop)) != hipSuccess)
          fail(DHIT_ENOMEM, "cannot allocate DUGKS scratch field");
      }
      b->reduce_level = b->partials + (size_t)b->max_blocks * 5;
      DHIT_HIP(hipMemsetAsync(b->reduce_level, 0, dhit::kFinalizeDoubles * sizeof(double), b->stream));
      derive_step_params(*b);
      if (step_table_bytes(b->p) > 0) {
        if (hipMalloc(&b->step_table, (size_t)step_table_bytes(b->p)) != hipSuccess)
          fail(DHIT_ENOMEM, "cannot allocate the step table");
        b->own_step_table = true;
        dhit::BatchBox e[2];
        if (b->p.method == DHIT_DUGKS)
          dhit::fused_table_entries(*b, e);
        else
          dhit::lbe_table_entries(*b, e);
        DHIT_HIP(hipMemcpy(b->step_table, e, sizeof(e), hipMemcpyHostToDevice));
      }
      // zero state until initialised
      DHIT_HIP(hipMemsetAsync(b->f[0], 0, pop, b->stream));
      DHIT_HIP(hipMemsetAsync(b->hist, 0, (size_t)dhit::kHistoryCap * 5 * sizeof(double), b->stream));
      DHIT_HIP(hipStreamSynchronize(b->stream));
    } catch (...) {
      destroy_box(b);
      throw;
    }
    *out = b;
    return DHIT_OK;
  });
}

int32_t destroy_box(dhit_box *b) {
  if (!b) return DHIT_OK;
  if (b->stream) (void)hipStreamSynchronize(b->stream);
  dhit::spectrum_free(*b);
  dhit::timer_free(*b);
  if (b->own_f) {
    if (b->f[0]) (void)hipFree(b->f[0]);
    if (b->f[1]) (void)hipFree(b->f[1]);
  }
  if (b->partials) (void)hipFree(b->partials);
  if (b->hist) (void)hipFree(b->hist);
  if (b->scratch) (void)hipFree(b->scratch);
  if (b->mesh) (void)hipFree(b->mesh);
  if (b->own_step_table && b->step_table) (void)hipFree(b->step_table);
  if (b->own_stream && b->stream) (void)hipStreamDestroy(b->stream);
  delete b;
  return DHIT_OK;
}

int32_t init_velocity_field_device(dhit_box *b, const double *u, const double *drho) {
  return guarded([&]() -> int32_t {
    require_box(b);
    if (!u) fail(DHIT_EINVAL, "null velocity field");
    b->cur = 0;
    dhit::launch_init_equilibrium(*b, u, drho, b->f[0]);
    b->steps = 0;
    return DHIT_OK;
  });
}

int32_t init_velocity_field(dhit_box *b, const double *u, const double *drho) {
  return guarded([&]() -> int32_t {
    require_box(b);
    if (!u) fail(DHIT_EINVAL, "null velocity field");
    const size_t bytes = (size_t)b->ncell * sizeof(double);
    double *du = nullptr, *dr = nullptr;
    if (hipMalloc(&du, 3 * bytes) != hipSuccess) fail(DHIT_ENOMEM, "cannot allocate upload buffer");
    try {
      if (drho && hipMalloc(&dr, bytes) != hipSuccess) fail(DHIT_ENOMEM, "cannot allocate upload buffer");
      DHIT_HIP(hipMemcpyAsync(du, u, 3 * bytes, hipMemcpyHostToDevice, b->stream));
      if (drho) DHIT_HIP(hipMemcpyAsync(dr, drho, bytes, hipMemcpyHostToDevice, b->stream));
      b->cur = 0;
      dhit::launch_init_equilibrium(*b, du, dr, b->f[0]);
      DHIT_HIP(hipStreamSynchronize(b->stream));
    } catch (...) {
      (void)hipStreamSynchronize(b->stream);
      (void)hipFree(du);
      if (dr) (void)hipFree(dr);
      throw;
    }
    (void)hipFree(du);
    if (dr) (void)hipFree(dr);
    b->steps = 0;
    return DHIT_OK;
  });
}

int32_t set_mesh(dhit_box *b, const double *widths) {
  return guarded([&]() -> int32_t {
    require_box(b);
    if (b->p.method != DHIT_DUGKS) fail(DHIT_EMETHOD, "set_mesh applies to DUGKS boxes");
    DHIT_HIP(hipStreamSynchronize(b->stream));
    if (!widths) {
      if (b->mesh) (void)hipFree(b->mesh);
      b->mesh = nullptr;
      return DHIT_OK;
    }
    const int n = b->n;
    double wmin = INFINITY;
    for (int i = 0; i < 3 * n; ++i) {
      if (!(widths[i] > 0.0) || !std::isfinite(widths[i])) fail(DHIT_EINVAL, "cell widths must be finite and > 0");
      wmin = std::min(wmin, widths[i]);
    }
    // the fastest particles move sqrt(2) per unit time: CFL = sqrt(2) dt / w_min
    if (std::sqrt(2.0) * b->p.dt > wmin) fail(DHIT_EINVAL, "dt exceeds CFL 1 on the smallest cell");
    std::vector<double> t((size_t)3 * dhit::kMeshTables * n);
    for (int a = 0; a < 3; ++a) {
      const double *w = widths + (size_t)a * n;
      double *row = t.data() + (size_t)a * dhit::kMeshTables * n;
      for (int i = 0; i < n; ++i) {
        const double wm = w[(i + n - 1) % n], wi = w[i], wp = w[(i + 1) % n];
        row[dhit::kMeshWidth * n + i] = wi;
        row[dhit::kMeshInvWidth * n + i] = 1.0 / wi;
        row[dhit::kMeshLam * n + i] = wi / (wi + wp);
        row[dhit::kMeshInvGap * n + i] = 2.0 / (wi + wp);
        row[dhit::kMeshInvSpan * n + i] = 1.0 / (0.5 * wm + wi + 0.5 * wp);
      }
    }
    if (!b->scratch) {
      const int64_t bytes = population_buffer_bytes(&b->p);
      if (hipMalloc(&b->scratch, (size_t)bytes) != hipSuccess) fail(DHIT_ENOMEM, "cannot allocate DUGKS scratch field");
    }
    if (!b->mesh && hipMalloc(&b->mesh, t.size() * sizeof(double)) != hipSuccess)
      fail(DHIT_ENOMEM, "cannot allocate mesh tables");
    DHIT_HIP(hipMemcpy(b->mesh, t.data(), t.size() * sizeof(double), hipMemcpyHostToDevice));
    return DHIT_OK;
  });
}

int32_t init_consistent(dhit_box *b, const double *u, const double *drho, int32_t iters, double *residual) {
  return guarded([&]() -> int32_t {
    require_box(b);
    if (!u) fail(DHIT_EINVAL, "null velocity field");
    if (iters < 0) fail(DHIT_EINVAL, "iters must be >= 0");
    const size_t bytes = (size_t)b->ncell * sizeof(double);
    if (b->p.method == DHIT_DUGKS) {
      // first-order Chapman-Enskog start from the spectral velocity gradient
      if (b->mesh) fail(DHIT_EMETHOD, "the spectral velocity gradient needs unit cells (this box has a stretched mesh)");
      double *du = nullptr, *dr = nullptr, *dg = nullptr;
      auto cleanup = [&]() {
        (void)hipStreamSynchronize(b->stream);
        if (du) (void)hipFree(du);
        if (dr) (void)hipFree(dr);
        if (dg) (void)hipFree(dg);
      };
      try {
        if (hipMalloc(&du, 3 * bytes) != hipSuccess || hipMalloc(&dg, 9 * bytes) != hipSuccess)
          fail(DHIT_ENOMEM, "cannot allocate the velocity and gradient buffers");
        if (drho && hipMalloc(&dr, bytes) != hipSuccess) fail(DHIT_ENOMEM, "cannot allocate upload buffer");
        DHIT_HIP(hipMemcpyAsync(du, u, 3 * bytes, hipMemcpyHostToDevice, b->stream));
        if (drho) DHIT_HIP(hipMemcpyAsync(dr, drho, bytes, hipMemcpyHostToDevice, b->stream));
        dhit::gradient_compute(*b, du, dg);
        b->cur = 0;
        dhit::launch_ce_init(*b, du, dr, dg, b->f[0]);
        DHIT_HIP(hipStreamSynchronize(b->stream));
      } catch (...) {
        cleanup();
        b->steps = 0;
        throw;
      }
      cleanup();
      if (residual) *residual = 0.0;
      b->steps = 0;
      return DHIT_OK;
    }
    const int blocks = dhit::cell_blocks(b->ncell);
    double *du = nullptr, *dr = nullptr, *dprev = nullptr, *dmax = nullptr;
    auto cleanup = [&]() {
      (void)hipStreamSynchronize(b->stream);
      if (du) (void)hipFree(du);
      if (dr) (void)hipFree(dr);
      if (dprev) (void)hipFree(dprev);
      if (dmax) (void)hipFree(dmax);
    };
    try {
      if (hipMalloc(&du, 3 * bytes) != hipSuccess) fail(DHIT_ENOMEM, "cannot allocate upload buffer");
      if (drho && hipMalloc(&dr, bytes) != hipSuccess) fail(DHIT_ENOMEM, "cannot allocate upload buffer");
      if (iters > 0 && (hipMalloc(&dprev, bytes) != hipSuccess ||
                        hipMalloc(&dmax, (size_t)blocks * sizeof(double)) != hipSuccess))
        fail(DHIT_ENOMEM, "cannot allocate iteration buffers");
      DHIT_HIP(hipMemcpyAsync(du, u, 3 * bytes, hipMemcpyHostToDevice, b->stream));
      if (drho) DHIT_HIP(hipMemcpyAsync(dr, drho, bytes, hipMemcpyHostToDevice, b->stream));
      b->cur = 0;
      dhit::launch_init_equilibrium(*b, du, dr, b->f[0]);
      if (iters > 0) {
        // drho before the first pass is the initial field (the equilibrium state carries it exactly)
        if (dr)
          DHIT_HIP(hipMemcpyAsync(dprev, dr, bytes, hipMemcpyDeviceToDevice, b->stream));
        else
          DHIT_HIP(hipMemsetAsync(dprev, 0, bytes, b->stream));
      }
      for (int32_t k = 0; k < iters; ++k) {
        const bool last = k == iters - 1;
        double *slot = b->hist + (k % dhit::kHistoryCap) * 5;
        dhit::launch_lbe_step(*b, b->f[b->cur], b->f[1 - b->cur], slot);
        b->cur = 1 - b->cur;
        dhit::launch_hold_velocity(*b, b->f[b->cur], du, last ? nullptr : dprev, last ? dprev : nullptr,
                                   last ? dmax : nullptr);
      }
      double res = 0.0;
      if (iters > 0) {
        std::vector<double> h(blocks);
        DHIT_HIP(hipMemcpyAsync(h.data(), dmax, (size_t)blocks * sizeof(double), hipMemcpyDeviceToHost, b->stream));
        DHIT_HIP(hipStreamSynchronize(b->stream));
        for (double v : h) res = std::max(res, v);
      }
      DHIT_HIP(hipStreamSynchronize(b->stream));
      if (!std::isfinite(res)) fail(DHIT_ENONFINITE, "initial-state iteration produced a non-finite density");
      if (residual) *residual = res;
    } catch (...) {
      cleanup();
      b->steps = 0;
      throw;
    }
    cleanup();
    b->steps = 0;
    return DHIT_OK;
  });
}

static int32_t step_common(dhit_box *b, int32_t nsteps, bool lbe) {
  return guarded([&]() -> int32_t {
    require_box(b);
    if (nsteps < 0) fail(DHIT_EINVAL, "nsteps must be >= 0");
    const bool is_lbe = b->p.method != DHIT_DUGKS;
    if (is_lbe != lbe) fail(DHIT_EMETHOD, lbe ? "step_lbe called on a DUGKS box" : "step_dugks called on an LBE box");
    for (int32_t s = 0; s < nsteps; ++s) {
      double *slot = b->hist + (b->steps % dhit::kHistoryCap) * 5;
      const void *src = b->f[b->cur];
      void *dst = b->f[1 - b->cur];
      if (lbe)
        dhit::launch_lbe_step(*b, src, dst, slot);
      else
        dhit::launch_dugks_step(*b, src, dst, slot);
      b->cur = 1 - b->cur;
      b->steps++;
    }
    return DHIT_OK;
  });
}

int32_t step_lbe(dhit_box *b, int32_t nsteps) { return step_common(b, nsteps, true); }
int32_t step_dugks(dhit_box *b, int32_t nsteps) { return step_common(b, nsteps, false); }

int32_t moments(dhit_box *b, double *drho, double *j, double *sums) {
  return guarded([&]() -> int32_t {
    require_box(b);
    const size_t bytes = (size_t)b->ncell * sizeof(double);
    double *dd = nullptr, *dj = nullptr, *ds = nullptr;
    auto cleanup = [&]() {
      if (dd) (void)hipFree(dd);
      if (dj) (void)hipFree(dj);
      if (ds) (void)hipFree(ds);
    };
    try {
      if (drho && hipMalloc(&dd, bytes) != hipSuccess) fail(DHIT_ENOMEM, "cannot allocate moments buffer");
      if (j && hipMalloc(&dj, 3 * bytes) != hipSuccess) fail(DHIT_ENOMEM, "cannot allocate moments buffer");
      if (hipMalloc(&ds, 5 * sizeof(double)) != hipSuccess) fail(DHIT_ENOMEM, "cannot allocate moments buffer");
      dhit::launch_moments(*b, b->f[b->cur], dd, dj, ds);
      double hs[5];
      DHIT_HIP(hipMemcpyAsync(hs, ds, sizeof(hs), hipMemcpyDeviceToHost, b->stream));
      if (drho) DHIT_HIP(hipMemcpyAsync(drho, dd, bytes, hipMemcpyDeviceToHost, b->stream));
      if (j) DHIT_HIP(hipMemcpyAsync(j, dj, 3 * bytes, hipMemcpyDeviceToHost, b->stream));
      DHIT_HIP(hipStreamSynchronize(b->stream));
      if (sums) std::memcpy(sums, hs, sizeof(hs));
      cleanup();
      check_finite(hs, 5);
    } catch (...) {
      (void)hipStreamSynchronize(b->stream);
      cleanup();
      throw;
    }
    return DHIT_OK;
  });
}

int32_t sums_history(dhit_box *b, double *out, int32_t count) {
  return guarded([&]() -> int32_t {
    require_box(b);
    if (count < 0 || (count > 0 && !out)) fail(DHIT_EINVAL, "bad output");
    if (count > b->steps || count > dhit::kHistoryCap) fail(DHIT_EINVAL, "count exceeds the recorded history");
    DHIT_HIP(hipStreamSynchronize(b->stream));
    for (int32_t i = 0; i < count; ++i) {
      const int64_t step = b->steps - count + i;
      DHIT_HIP(hipMemcpy(out + 5 * i, b->hist + (step % dhit::kHistoryCap) * 5, 5 * sizeof(double),
                         hipMemcpyDeviceToHost));
    }
    check_finite(out, 5 * count);
    return DHIT_OK;
  });
}

int32_t energy_spectrum(dhit_box *b, double *E, int32_t kmax, double *stats) {
  return guarded([&]() -> int32_t {
    require_box(b);
    if (kmax < 0 || !E) fail(DHIT_EINVAL, "need E and kmax >= 0");
    if (b->mesh) fail(DHIT_EMETHOD, "spectral diagnostics need unit cells (this box has a stretched mesh)");
    dhit::spectrum_compute(*b, E, kmax, stats);
    return DHIT_OK;
  });
}

int32_t initial_pressure(dhit_box *b, const double *u, double *drho) {
  return guarded([&]() -> int32_t {
    require_box(b);
    if (!u || !drho) fail(DHIT_EINVAL, "null velocity or output");
    dhit::pressure_compute(*b, u, drho);
    return DHIT_OK;
  });
}

int32_t vorticity(dhit_box *b, double *omega) {
  return guarded([&]() -> int32_t {
    require_box(b);
    if (!omega) fail(DHIT_EINVAL, "null output");
    if (b->mesh) fail(DHIT_EMETHOD, "spectral diagnostics need unit cells (this box has a stretched mesh)");
    dhit::vorticity_compute(*b, omega);
    return DHIT_OK;
  });
}

int32_t get_populations(dhit_box *b, double *f) {
  return guarded([&]() -> int32_t {
    require_box(b);
    if (!f) fail(DHIT_EINVAL, "null output");
    const size_t bytes = (size_t)b->ncell * 19 * sizeof(double);
    double *d = nullptr;
    if (hipMalloc(&d, bytes) != hipSuccess) fail(DHIT_ENOMEM, "cannot allocate download buffer");
    try {
      dhit::launch_pack(*b, b->f[b->cur], d);
      DHIT_HIP(hipMemcpyAsync(f, d, bytes, hipMemcpyDeviceToHost, b->stream));
      DHIT_HIP(hipStreamSynchronize(b->stream));
    } catch (...) {
      (void)hipStreamSynchronize(b->stream);
      (void)hipFree(d);
      throw;
    }
    (void)hipFree(d);
    return DHIT_OK;
  });
}

int32_t set_populations(dhit_box *b, const double *f) {
  return guarded([&]() -> int32_t {
    require_box(b);
    if (!f) fail(DHIT_EINVAL, "null input");
    const size_t bytes = (size_t)b->ncell * 19 * sizeof(double);
    double *d = nullptr;
    if (hipMalloc(&d, bytes) != hipSuccess) fail(DHIT_ENOMEM, "cannot allocate upload buffer");
    try {
      DHIT_HIP(hipMemcpyAsync(d, f, bytes, hipMemcpyHostToDevice, b->stream));
      b->cur = 0;
      dhit::launch_unpack(*b, d, b->f[0]);
      DHIT_HIP(hipStreamSynchronize(b->stream));
    } catch (...) {
      (void)hipStreamSynchronize(b->stream);
      (void)hipFree(d);
      throw;
    }
    (void)hipFree(d);
    b->steps = 0;
    return DHIT_OK;
  });
}

int64_t steps_taken(const dhit_box *b) { return b ? b->steps : DHIT_EINVAL; }

int32_t box_synchronize(dhit_box *b) {
  return guarded([&]() -> int32_t {
    require_box(b);
    DHIT_HIP(hipStreamSynchronize(b->stream));
    if (b->steps > 0) {
      double s[5];
      DHIT_HIP(hipMemcpy(s, b->hist + ((b->steps - 1) % dhit::kHistoryCap) * 5, sizeof(s), hipMemcpyDeviceToHost));
      check_finite(s, 5);
    }
    return DHIT_OK;
  });
}

int32_t step_noalloc(const dhit_params *pp, const void *src, void *dst, double *sums) {
  return guarded([&]() -> int32_t {
    if (!pp || !src || !dst) fail(DHIT_EINVAL, "null argument");
    dhit_params p = *pp;
    p.f_a = p.f_b = nullptr;  // the caller's buffers come as src and dst
    validate(p);
    if (p.method == DHIT_DUGKS && p.variant != DHIT_VARIANT_DEFAULT)
      fail(DHIT_EINVAL, "step_noalloc runs the fused DUGKS step only (the two-pass form needs a field-sized work space)");
    if ((reinterpret_cast<uintptr_t>(src) | reinterpret_cast<uintptr_t>(dst)) & 255)
      fail(DHIT_EINVAL, "population buffers must be 256-byte aligned");
    if (src == dst) fail(DHIT_EINVAL, "src and dst must be different buffers");
    if (p.method == DHIT_DUGKS && p.z_chunk == 0) p.z_chunk = dhit::fused_auto_chunk(p);
    const int64_t blocks = reduction_blocks(p);
    if (blocks > kNoallocPartials)
      fail(DHIT_EINVAL, "box too large for step_noalloc: its reduction needs " + std::to_string(blocks) +
                            " block partials, the static work space holds " + std::to_string(kNoallocPartials) +
                            " (LBE: n <= 322)");
    double *ws = scratch_on_current_device();
    dhit_box b;  // host-side view of the caller's buffers; owns nothing
    b.p = p;
    b.n = p.n;
    b.ncell = (int64_t)p.n * p.n * p.n;
    b.elem = p.precision == DHIT_FP32 ? 4 : 8;
    b.stride = padded_stride(b.ncell, b.elem, p.method);
    b.f[0] = const_cast<void *>(src);
    b.f[1] = dst;
    b.stream = static_cast<hipStream_t>(p.stream);
    b.partials = ws;
    b.max_blocks = (int)kNoallocPartials;
    // its counter starts at zero (the array is zero when the library is
    // loaded) and every launch that uses it leaves it at zero
    b.reduce_level = ws + kNoallocLevel;
    derive_step_params(b);
    double *out = sums ? sums : ws + kNoallocDiscard;
    // the step reads the box as a table in device memory: written into the
    // work space by a launch that carries the entries by value
    dhit::BatchBox e[2];
    if (p.method == DHIT_DUGKS)
      dhit::fused_table_entries(b, e);
    else
      dhit::lbe_table_entries(b, e);
    b.step_table = reinterpret_cast<dhit::BatchBox *>(ws + kNoallocTable);
    dhit::launch_store_table(b.stream, e, b.step_table);
    if (p.method == DHIT_DUGKS)
      dhit::launch_dugks_step(b, src, dst, out);
    else
      dhit::launch_lbe_step(b, src, dst, out);
    return DHIT_OK;
  });
}

int32_t current_populations(const dhit_box *b, void **ptr, int64_t *stride) {
  return guarded([&]() -> int32_t {
    require_box(b);
    if (ptr) *ptr = b->f[b->cur];
    if (stride) *stride = b->stride;
    return DHIT_OK;
  });
}

namespace {
// The fused DUGKS launch of params p on a device holding `slots` blocks of
// the kernel at once, with an automatic z-chunk resolved for that device
// (the resolved setting in *z_chunk).
dhit::FusedPlan work_split_plan(const dhit_params *pp, int32_t slots, int32_t *z_chunk) {
  if (!pp) fail(DHIT_EINVAL, "null params");
  validate(*pp);
  if (pp->method != DHIT_DUGKS || pp->variant != DHIT_VARIANT_DEFAULT)
    fail(DHIT_EMETHOD, "the work split is that of the fused DUGKS step");
  if (slots < 1) fail(DHIT_EINVAL, "slots must be positive");
  dhit_params p = *pp;
  if (p.z_chunk == 0) {
    const dhit::FusedPlan t = dhit::fused_plan_for(p, slots);
    p.z_chunk = dhit::fused_balanced_chunk(p.n, t.tiles_x * t.tiles_y, slots);
  }
  *z_chunk = p.z_chunk;
  return dhit::fused_plan_for(p, slots);
}
}  // namespace

int32_t fused_work_items(const dhit_params *p, int32_t slots, int32_t *z_chunk) {
  int32_t items = 0;
  const int32_t st = guarded([&]() -> int32_t {
    int32_t zc = 0;
    const dhit::FusedPlan f = work_split_plan(p, slots, &zc);
    items = f.items;
    if (z_chunk) *z_chunk = zc;
    return DHIT_OK;
  });
  return st == DHIT_OK ? items : st;
}

int32_t fused_work_item(const dhit_params *p, int32_t slots, int32_t item, int32_t *tile, int32_t *z0,
                        int32_t *planes) {
  return guarded([&]() -> int32_t {
    if (!tile || !z0 || !planes) fail(DHIT_EINVAL, "null argument");
    int32_t zc = 0;
    const dhit::FusedPlan f = work_split_plan(p, slots, &zc);
    if (item < 0 || item >= f.items) fail(DHIT_EINVAL, "item out of range");
    int t, z, k;
    dhit::fused_item_planes(f, p->n, item, &t, &z, &k);
    *tile = t;
    *z0 = z;
    *planes = k;
    return DHIT_OK;
  });
}

const char *dhit_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
