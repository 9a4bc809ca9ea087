// Energy spectrum and velocity-derivative statistics of a box (Sec. III):
//   u = j/rho0 -> u_hat = DFT(u)/n^3 (hipFFT, real-to-complex, batch of 3)
//   -> shell binning of 1/2 |u_hat|^2 and of |kappa|^2 1/2 |u_hat|^2
//      (exact integer sums, so E(k) is the same bits on every run)
//   -> spectral derivatives i kappa_a u_hat_a (inverse transforms)
//   -> <(d_a u_a)^m>, m = 2, 3, 4 -> K, eps, S, F.
#include <cmath>
#include <cstring>
#include <vector>

#include "device_common.hpp"
#include "runtime.hpp"

namespace dhit {

struct SpectrumWork {
  int n = 0;
  int nshell = 0;
  int64_t nhalf = 0;  // modes of one real-to-complex transform, n*n*(n/2+1)
  double *u = nullptr;
  hipfftDoubleComplex *uh = nullptr;
  hipfftDoubleComplex *tmp = nullptr;
  unsigned long long *shells = nullptr;  // [2][kShellParts][nshell]: digit sums of E and kappa^2-weighted E
  int *overflow = nullptr;               // set when a shell term is out of range or not finite
  double *partials = nullptr;  // [5][blocks]
  double *dstats = nullptr;    // [3][5]
  hipfftHandle fwd = 0, inv = 0;
  bool have_fwd = false, have_inv = false;
};

#define DHIT_FFT(expr)                                                                               \
  do {                                                                                               \
    hipfftResult r_ = (expr);                                                                        \
    if (r_ != HIPFFT_SUCCESS) throw ::dhit::Error(DHIT_EDEVICE, std::string(#expr " failed, code ") + std::to_string((int)r_)); \
  } while (0)

// Signed integer wavenumber of FFT index i (numpy fftfreq order).
__device__ __forceinline__ int signed_k(int i, int n) { return (i <= (n - 1) / 2) ? i : i - n; }

// Shell sums are accumulated exactly, so that E(k) does not depend on the
// order in which threads add their modes: a term e (>= 0) is taken as the
// integer floor(e 2^kShellFrac), split into three kShellDigit-bit digits,
// and each digit is summed with integer atomic adds (associative, so the
// order does not matter).  The host joins the digits in 128-bit integers
// and rounds once.  Terms below 2^-kShellFrac (3e-27) in absolute value are
// truncated; a term of 2^8 or more (or not finite; velocities of order one
// in lattice units already mean a blown-up run) raises the overflow flag.
// With 34-bit digits a digit sum stays below 2^64, and the joined value
// below 2^126, for up to 2^30 modes (n <= 1024).
constexpr int kShellFrac = 88, kShellDigit = 34, kShellParts = 3;

__device__ __forceinline__ void shell_digits(double e, unsigned long long (&d)[kShellParts], bool &over) {
  if (!(e >= 0.0 && e < 256.0)) {
    over = true;
    d[0] = d[1] = d[2] = 0;
    return;
  }
  const double x = e * 0x1p88;                 // exact: a power of two, x < 2^96
  const double hi = floor(x * 0x1p-68);        // < 2^28
  const double r = x - hi * 0x1p68;            // exact: a multiple of ulp(x) below 2^68
  const double mid = floor(r * 0x1p-34);       // < 2^34
  const double lo = floor(r - mid * 0x1p34);   // < 2^34; drops bits below 2^-88 of e
  d[2] = (unsigned long long)hi;
  d[1] = (unsigned long long)mid;
  d[0] = (unsigned long long)lo;
}

// One thread per mode of the half spectrum; block histogram of the digits
// in LDS, then one integer atomic add per digit, shell and block.  Modes
// 0 < kx < n/2 stand for their Hermitian partners too (weight 2).
// shells: [2][kShellParts][nshell] digit sums of E and of kappa^2 E.
__global__ __launch_bounds__(256) void bin_kernel(const hipfftDoubleComplex *__restrict__ uh, int n, int64_t nhalf,
                                                  int nshell, double inv_n6, unsigned long long *__restrict__ shells,
                                                  int *__restrict__ overflow) {
  extern __shared__ unsigned long long hist[];  // [2][kShellParts][nshell]
  const int nh = 2 * kShellParts * nshell;
  for (int i = threadIdx.x; i < nh; i += blockDim.x) hist[i] = 0ull;
  __syncthreads();
  const int nxh = n / 2 + 1;
  const double kfac = 2.0 * M_PI / n;
  bool over = false;
  for (int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; m < nhalf; m += (int64_t)gridDim.x * blockDim.x) {
    const int kxh = (int)(m % nxh);
    const int64_t r = m / nxh;
    const int iy = (int)(r % n), iz = (int)(r / n);
    const int kx = kxh, ky = signed_k(iy, n), kz = signed_k(iz, n);
    double e = 0.0;
    for (int c = 0; c < 3; ++c) {
      const hipfftDoubleComplex v = uh[(int64_t)c * nhalf + m];
      e += v.x * v.x + v.y * v.y;
    }
    const bool self = (kx == 0) || (2 * kx == n);
    e *= 0.5 * inv_n6 * (self ? 1.0 : 2.0);
    const int k2 = kx * kx + ky * ky + kz * kz;
    const int s = (int)rint(sqrt((double)k2));
    unsigned long long d[kShellParts], dk[kShellParts];
    shell_digits(e, d, over);
    shell_digits(kfac * kfac * (double)k2 * e, dk, over);
    for (int j = 0; j < kShellParts; ++j) {
      if (d[j]) atomicAdd(&hist[j * nshell + s], d[j]);
      if (dk[j]) atomicAdd(&hist[(kShellParts + j) * nshell + s], dk[j]);
    }
  }
  if (over) atomicOr(overflow, 1);
  __syncthreads();
  for (int i = threadIdx.x; i < nh; i += blockDim.x)
    if (hist[i] != 0ull) atomicAdd(&shells[i], hist[i]);
}

// tmp = i kappa_a u_hat_a on the half spectrum; the Nyquist wavenumber of
// the derivative direction is set to zero.
__global__ __launch_bounds__(256) void deriv_kernel(const hipfftDoubleComplex *__restrict__ uha,
                                                    hipfftDoubleComplex *__restrict__ out, int n, int64_t nhalf,
                                                    int axis) {
  const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= nhalf) return;
  const int nxh = n / 2 + 1;
  const int kxh = (int)(m % nxh);
  const int64_t r = m / nxh;
  const int iy = (int)(r % n), iz = (int)(r / n);
  int k = axis == 0 ? kxh : (axis == 1 ? signed_k(iy, n) : signed_k(iz, n));
  if ((n % 2 == 0) && (2 * k == n || 2 * k == -n)) k = 0;
  const double kap = 2.0 * M_PI / n * k;
  const hipfftDoubleComplex v = uha[m];
  hipfftDoubleComplex o;
  o.x = -kap * v.y;
  o.y = kap * v.x;
  out[m] = o;
}

// Component a of the vorticity on the half spectrum, scaled by `scale`:
// out = scale i (kappa_b u_hat_c - kappa_c u_hat_b), (a, b, c) cyclic; the
// Nyquist wavenumber of each derivative direction is set to zero, as in
// deriv_kernel.
__global__ __launch_bounds__(256) void curl_kernel(const hipfftDoubleComplex *__restrict__ uh,
                                                   hipfftDoubleComplex *__restrict__ out, int n, int64_t nhalf,
                                                   int a, double scale) {
  const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= nhalf) return;
  const int nxh = n / 2 + 1;
  const int64_t r = m / nxh;
  int k[3] = {(int)(m % nxh), signed_k((int)(r % n), n), signed_k((int)(r / n), n)};
  for (int i = 0; i < 3; ++i)
    if ((n % 2 == 0) && (2 * k[i] == n || 2 * k[i] == -n)) k[i] = 0;
  const int b = (a + 1) % 3, c = (a + 2) % 3;
  const double kb = 2.0 * M_PI / n * k[b], kc = 2.0 * M_PI / n * k[c];
  const hipfftDoubleComplex ub = uh[(int64_t)b * nhalf + m], uc = uh[(int64_t)c * nhalf + m];
  // i (kb uc - kc ub)
  const double re = kb * uc.x - kc * ub.x, im = kb * uc.y - kc * ub.y;
  hipfftDoubleComplex o;
  o.x = -im * scale;
  o.y = re * scale;
  out[m] = o;
}

// Spectrum of the velocity-gradient component d_a u_b, scaled by `scale`:
// out = scale i kappa_a u_hat_b on the half spectrum, the Nyquist
// wavenumber of the derivative direction set to zero (as deriv_kernel).
__global__ __launch_bounds__(256) void gradient_kernel(const hipfftDoubleComplex *__restrict__ uhb,
                                                       hipfftDoubleComplex *__restrict__ out, int n, int64_t nhalf,
                                                       int a, double scale) {
  const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= nhalf) return;
  const int nxh = n / 2 + 1;
  const int64_t r = m / nxh;
  int k = a == 0 ? (int)(m % nxh) : (a == 1 ? signed_k((int)(r % n), n) : signed_k((int)(r / n), n));
  if ((n % 2 == 0) && (2 * k == n || 2 * k == -n)) k = 0;
  const double kap = 2.0 * M_PI / n * k * scale;
  const hipfftDoubleComplex v = uhb[m];
  hipfftDoubleComplex o;
  o.x = -kap * v.y;
  o.y = kap * v.x;
  out[m] = o;
}

// Products of velocity components for the pressure source: set 0 gives
// (u u, v v, w w), set 1 gives (u v, v w, w u), into three fields of out.
__global__ __launch_bounds__(256) void products_kernel(const double *__restrict__ u, double *__restrict__ out,
                                                       int64_t ncell, int set) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ncell) return;
  const double a = u[i], b = u[ncell + i], c = u[2 * ncell + i];
  if (set == 0) {
    out[i] = a * a;
    out[ncell + i] = b * b;
    out[2 * ncell + i] = c * c;
  } else {
    out[i] = a * b;
    out[ncell + i] = b * c;
    out[2 * ncell + i] = c * a;
  }
}

// acc (half spectrum) (=, set 0) or (+=, set 1) sum over the three
// transformed products ph of their weights: set 0 k_a^2 for (aa),
// set 1 2 k_a k_b for (ab) = (xy, yz, zx); k the integer wavevector with the
// Nyquist component of each derivative factor dropped.
__global__ __launch_bounds__(256) void pressure_source_kernel(const hipfftDoubleComplex *__restrict__ ph,
                                                              hipfftDoubleComplex *__restrict__ acc, int n,
                                                              int64_t nhalf, int set) {
  const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= nhalf) return;
  const int nxh = n / 2 + 1;
  const int64_t r = m / nxh;
  int k[3] = {(int)(m % nxh), signed_k((int)(r % n), n), signed_k((int)(r / n), n)};
  for (int i = 0; i < 3; ++i)
    if ((n % 2 == 0) && (2 * k[i] == n || 2 * k[i] == -n)) k[i] = 0;
  double re = 0.0, im = 0.0;
  for (int c = 0; c < 3; ++c) {
    const double w = set == 0 ? (double)k[c] * k[c] : 2.0 * (double)k[c] * k[(c + 1) % 3];
    const hipfftDoubleComplex v = ph[(int64_t)c * nhalf + m];
    re += w * v.x;
    im += w * v.y;
  }
  if (set == 0) {
    acc[m].x = re;
    acc[m].y = im;
  } else {
    acc[m].x += re;
    acc[m].y += im;
  }
}

// acc <- scale acc / |k|^2 (full integer |k|^2; the k = 0 mode set to 0).
__global__ __launch_bounds__(256) void inverse_laplacian_kernel(hipfftDoubleComplex *__restrict__ acc, int n,
                                                                int64_t nhalf, double scale) {
  const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= nhalf) return;
  const int nxh = n / 2 + 1;
  const int64_t r = m / nxh;
  const int kx = (int)(m % nxh), ky = signed_k((int)(r % n), n), kz = signed_k((int)(r / n), n);
  const int k2 = kx * kx + ky * ky + kz * kz;
  const double f = k2 == 0 ? 0.0 : scale / (double)k2;
  acc[m].x *= f;
  acc[m].y *= f;
}

// Sums of d^2, d^3, d^4 of a real field scaled by `scale`.
__global__ __launch_bounds__(kBlock) void power_sums_kernel(const double *__restrict__ d, int64_t ncell, double scale,
                                                            double *__restrict__ partials) {
  double v[kNumSums] = {0, 0, 0, 0, 0};
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < ncell; i += (int64_t)gridDim.x * kBlock) {
    const double x = d[i] * scale;
    const double x2 = x * x;
    v[0] += x2;
    v[1] += x2 * x;
    v[2] += x2 * x2;
  }
  write_block_partials(v, partials, gridDim.x, blockIdx.x);
}

static void ensure_work(dhit_box &b) {
  if (b.spec) return;
  SpectrumWork *w = new SpectrumWork();
  b.spec = w;
  const int n = b.n;
  w->n = n;
  w->nhalf = (int64_t)n * n * (n / 2 + 1);
  w->nshell = (int)std::floor(std::sqrt(3.0) * (n / 2 + 1)) + 2;
  if (hipMalloc(&w->u, 3 * b.ncell * sizeof(double)) != hipSuccess ||
      hipMalloc(&w->uh, 3 * w->nhalf * sizeof(hipfftDoubleComplex)) != hipSuccess ||
      hipMalloc(&w->tmp, w->nhalf * sizeof(hipfftDoubleComplex)) != hipSuccess ||
      hipMalloc(&w->shells, 2 * kShellParts * w->nshell * sizeof(unsigned long long)) != hipSuccess ||
      hipMalloc(&w->overflow, sizeof(int)) != hipSuccess ||
      hipMalloc(&w->partials, 5 * 1024 * sizeof(double)) != hipSuccess ||
      hipMalloc(&w->dstats, 3 * 5 * sizeof(double)) != hipSuccess)
    throw Error(DHIT_ENOMEM, "cannot allocate spectrum work space");
  int dims[3] = {n, n, n};
  DHIT_FFT(hipfftPlanMany(&w->fwd, 3, dims, nullptr, 1, (int)b.ncell, nullptr, 1, (int)w->nhalf, HIPFFT_D2Z, 3));
  w->have_fwd = true;
  DHIT_FFT(hipfftPlanMany(&w->inv, 3, dims, nullptr, 1, (int)w->nhalf, nullptr, 1, (int)b.ncell, HIPFFT_Z2D, 1));
  w->have_inv = true;
}

// Device bytes of the spectrum work space of an n^3 box: the arrays of
// ensure_work and the work areas of its two hipFFT plans (made here with
// automatic allocation off, so nothing is allocated).
int64_t spectrum_work_bytes(int n) {
  const int64_t ncell = (int64_t)n * n * n, nhalf = (int64_t)n * n * (n / 2 + 1);
  const int64_t nshell = (int64_t)std::floor(std::sqrt(3.0) * (n / 2 + 1)) + 2;
  int64_t bytes = 3 * ncell * (int64_t)sizeof(double) + 4 * nhalf * (int64_t)sizeof(hipfftDoubleComplex) +
                  2 * kShellParts * nshell * (int64_t)sizeof(unsigned long long) + (int64_t)sizeof(int) +
                  5 * 1024 * (int64_t)sizeof(double) + 15 * (int64_t)sizeof(double);
  int dims[3] = {n, n, n};
  for (int dir = 0; dir < 2; ++dir) {
    hipfftHandle h = 0;
    DHIT_FFT(hipfftCreate(&h));
    size_t work = 0;
    hipfftResult r = hipfftSetAutoAllocation(h, 0);
    if (r == HIPFFT_SUCCESS)
      r = dir == 0 ? hipfftMakePlanMany(h, 3, dims, nullptr, 1, (int)ncell, nullptr, 1, (int)nhalf, HIPFFT_D2Z, 3, &work)
                   : hipfftMakePlanMany(h, 3, dims, nullptr, 1, (int)nhalf, nullptr, 1, (int)ncell, HIPFFT_Z2D, 1, &work);
    hipfftDestroy(h);
    if (r != HIPFFT_SUCCESS) throw Error(DHIT_EDEVICE, "hipfftMakePlanMany failed, code " + std::to_string((int)r));
    bytes += (int64_t)work;
  }
  return bytes;
}

void spectrum_free(dhit_box &b) {
  SpectrumWork *w = b.spec;
  if (!w) return;
  if (w->have_fwd) hipfftDestroy(w->fwd);
  if (w->have_inv) hipfftDestroy(w->inv);
  if (w->u) (void)hipFree(w->u);
  if (w->uh) (void)hipFree(w->uh);
  if (w->tmp) (void)hipFree(w->tmp);
  if (w->shells) (void)hipFree(w->shells);
  if (w->overflow) (void)hipFree(w->overflow);
  if (w->partials) (void)hipFree(w->partials);
  if (w->dstats) (void)hipFree(w->dstats);
  delete w;
  b.spec = nullptr;
}

void spectrum_compute(dhit_box &b, double *E_host, int kmax, double *stats_host) {
  ensure_work(b);
  SpectrumWork &w = *b.spec;
  const int n = b.n;
  DHIT_FFT(hipfftSetStream(w.fwd, b.stream));
  DHIT_FFT(hipfftSetStream(w.inv, b.stream));
  launch_velocity(b, b.f[b.cur], w.u);
  DHIT_FFT(hipfftExecD2Z(w.fwd, w.u, w.uh));
  const size_t shell_words = 2 * kShellParts * (size_t)w.nshell;
  DHIT_HIP(hipMemsetAsync(w.shells, 0, shell_words * sizeof(unsigned long long), b.stream));
  DHIT_HIP(hipMemsetAsync(w.overflow, 0, sizeof(int), b.stream));
  const double inv_n3 = 1.0 / ((double)n * n * n);
  {
    const int blocks = (int)std::min<int64_t>((w.nhalf + 255) / 256, 2048);
    hipLaunchKernelGGL(bin_kernel, dim3(blocks), dim3(256), shell_words * sizeof(unsigned long long), b.stream, w.uh,
                       n, w.nhalf, w.nshell, inv_n3 * inv_n3, w.shells, w.overflow);
    DHIT_HIP(hipGetLastError());
  }
  for (int a = 0; a < 3; ++a) {
    const int blocks = (int)((w.nhalf + 255) / 256);
    hipLaunchKernelGGL(deriv_kernel, dim3(blocks), dim3(256), 0, b.stream, w.uh + a * w.nhalf, w.tmp, n, w.nhalf, a);
    DHIT_HIP(hipGetLastError());
    DHIT_FFT(hipfftExecZ2D(w.inv, w.tmp, w.u));  // overwrites u[0 .. ncell)
    const int rb = (int)std::min<int64_t>((b.ncell + kBlock - 1) / kBlock, 1024);
    hipLaunchKernelGGL(power_sums_kernel, dim3(rb), dim3(kBlock), 0, b.stream, w.u, b.ncell, inv_n3, w.partials);
    DHIT_HIP(hipGetLastError());
    launch_finalize_sums(b, w.partials, rb, w.dstats + 5 * a);
  }
  std::vector<unsigned long long> dig(shell_words);
  double ds[15];
  int over = 0;
  DHIT_HIP(hipMemcpyAsync(dig.data(), w.shells, shell_words * sizeof(unsigned long long), hipMemcpyDeviceToHost,
                          b.stream));
  DHIT_HIP(hipMemcpyAsync(ds, w.dstats, sizeof(ds), hipMemcpyDeviceToHost, b.stream));
  DHIT_HIP(hipMemcpyAsync(&over, w.overflow, sizeof(int), hipMemcpyDeviceToHost, b.stream));
  DHIT_HIP(hipStreamSynchronize(b.stream));
  if (over) throw Error(DHIT_ENONFINITE, "velocity field is not finite (or a spectral term exceeds 2^8)");
  // join the digits of each shell: sum_j digit_j 2^(34 j), then times 2^-88
  std::vector<double> sh(2 * w.nshell);
  for (int q = 0; q < 2; ++q)
    for (int k = 0; k < w.nshell; ++k) {
      unsigned __int128 v = 0;
      for (int j = kShellParts - 1; j >= 0; --j)
        v = (v << kShellDigit) + (unsigned __int128)dig[((size_t)q * kShellParts + j) * w.nshell + k];
      sh[(size_t)q * w.nshell + k] = std::ldexp((double)v, -kShellFrac);
    }
  for (int k = 0; k <= kmax; ++k) E_host[k] = k < w.nshell ? sh[k] : 0.0;
  if (stats_host) {
    double K = 0, D = 0;
    for (int k = 0; k < w.nshell; ++k) {
      K += sh[k];
      D += sh[w.nshell + k];
    }
    double num3 = 0, den3 = 0, num4 = 0, den4 = 0;
    for (int a = 0; a < 3; ++a) {
      const double m2 = ds[5 * a + 0] * inv_n3, m3 = ds[5 * a + 1] * inv_n3, m4 = ds[5 * a + 2] * inv_n3;
      num3 += m3;
      num4 += m4;
      den3 += std::pow(m2, 1.5);
      den4 += m2 * m2;
    }
    stats_host[0] = K;
    stats_host[1] = 2.0 * b.p.nu * D;
    stats_host[2] = den3 > 0 ? num3 / den3 : 0.0;
    stats_host[3] = den4 > 0 ? num4 / den4 : 0.0;
  }
  for (int i = 0; i < 15; ++i)
    if (!std::isfinite(ds[i])) throw Error(DHIT_ENONFINITE, "velocity field is not finite");
}

void pressure_compute(dhit_box &b, const double *u_host, double *drho_host) {
  ensure_work(b);
  SpectrumWork &w = *b.spec;
  const int n = b.n;
  DHIT_FFT(hipfftSetStream(w.fwd, b.stream));
  DHIT_FFT(hipfftSetStream(w.inv, b.stream));
  double *du = nullptr;
  if (hipMalloc(&du, 3 * b.ncell * sizeof(double)) != hipSuccess)
    throw Error(DHIT_ENOMEM, "cannot allocate the velocity upload buffer");
  try {
    DHIT_HIP(hipMemcpyAsync(du, u_host, 3 * b.ncell * sizeof(double), hipMemcpyHostToDevice, b.stream));
    const int cb = (int)((b.ncell + 255) / 256), mb = (int)((w.nhalf + 255) / 256);
    for (int set = 0; set < 2; ++set) {
      hipLaunchKernelGGL(products_kernel, dim3(cb), dim3(256), 0, b.stream, du, w.u, (int64_t)b.ncell, set);
      DHIT_HIP(hipGetLastError());
      DHIT_FFT(hipfftExecD2Z(w.fwd, w.u, w.uh));
      hipLaunchKernelGGL(pressure_source_kernel, dim3(mb), dim3(256), 0, b.stream, w.uh, w.tmp, n, w.nhalf, set);
      DHIT_HIP(hipGetLastError());
    }
    // p_hat = -rho0 rhs / |k|^2; drho = 3 p; both transforms are unnormalised
    const double scale = -3.0 * b.p.rho0 / ((double)n * n * n);
    hipLaunchKernelGGL(inverse_laplacian_kernel, dim3(mb), dim3(256), 0, b.stream, w.tmp, n, w.nhalf, scale);
    DHIT_HIP(hipGetLastError());
    DHIT_FFT(hipfftExecZ2D(w.inv, w.tmp, w.u));
    DHIT_HIP(hipMemcpyAsync(drho_host, w.u, b.ncell * sizeof(double), hipMemcpyDeviceToHost, b.stream));
    DHIT_HIP(hipStreamSynchronize(b.stream));
  } catch (...) {
    (void)hipStreamSynchronize(b.stream);
    (void)hipFree(du);
    throw;
  }
  (void)hipFree(du);
}

void gradient_compute(dhit_box &b, const double *d_u, double *d_grad) {
  ensure_work(b);
  SpectrumWork &w = *b.spec;
  const int n = b.n;
  DHIT_FFT(hipfftSetStream(w.fwd, b.stream));
  DHIT_FFT(hipfftSetStream(w.inv, b.stream));
  DHIT_HIP(hipMemcpyAsync(w.u, d_u, 3 * b.ncell * sizeof(double), hipMemcpyDeviceToDevice, b.stream));
  DHIT_FFT(hipfftExecD2Z(w.fwd, w.u, w.uh));
  const double inv_n3 = 1.0 / ((double)n * n * n);  // both transforms are unnormalised
  const int blocks = (int)((w.nhalf + 255) / 256);
  for (int a = 0; a < 3; ++a)
    for (int c = 0; c < 3; ++c) {
      hipLaunchKernelGGL(gradient_kernel, dim3(blocks), dim3(256), 0, b.stream, w.uh + (int64_t)c * w.nhalf, w.tmp, n,
                         w.nhalf, a, inv_n3);
      DHIT_HIP(hipGetLastError());
      DHIT_FFT(hipfftExecZ2D(w.inv, w.tmp, d_grad + (int64_t)(3 * a + c) * b.ncell));
    }
}

void vorticity_compute(dhit_box &b, double *omega_host) {
  ensure_work(b);
  SpectrumWork &w = *b.spec;
  const int n = b.n;
  DHIT_FFT(hipfftSetStream(w.fwd, b.stream));
  DHIT_FFT(hipfftSetStream(w.inv, b.stream));
  launch_velocity(b, b.f[b.cur], w.u);
  DHIT_FFT(hipfftExecD2Z(w.fwd, w.u, w.uh));
  const double inv_n3 = 1.0 / ((double)n * n * n);  // both transforms are unnormalised
  const int blocks = (int)((w.nhalf + 255) / 256);
  for (int a = 0; a < 3; ++a) {
    hipLaunchKernelGGL(curl_kernel, dim3(blocks), dim3(256), 0, b.stream, w.uh, w.tmp, n, w.nhalf, a, inv_n3);
    DHIT_HIP(hipGetLastError());
    DHIT_FFT(hipfftExecZ2D(w.inv, w.tmp, w.u + (int64_t)a * b.ncell));
  }
  DHIT_HIP(hipMemcpyAsync(omega_host, w.u, 3 * b.ncell * sizeof(double), hipMemcpyDeviceToHost, b.stream));
  DHIT_HIP(hipStreamSynchronize(b.stream));
}

}  // namespace dhit
