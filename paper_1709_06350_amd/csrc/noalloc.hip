// Residual of a given potential without a context and without any device allocation, for callers
// that cannot allocate (code under HIP graph capture, tight serving loops, harnesses that forbid
// hipMalloc). It computes what mr_residual computes (Sec. II.A.1, Eq. 15 with the mean projection)
// directly on the caller's natural-order arrays; the only device memory beyond the inputs and the
// output is the file-scope array `scratch` below: per-block partial sums, their arrival counter and
// the reduced totals. Every call on a device shares that device's copy of the array, so calls that
// overlap on one device race; the counter and totals are cleared at the start of every call.
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>

#include "mr.h"
#include "mr_ctx.h"
#include "mr_device.h"

namespace mr {
namespace {

constexpr int kNaBlocks = 2048;   // blocks of each reducing launch (rows of the mesh dealt to them)
constexpr int kNaThreads = 256;
constexpr int kNaValues = 4;
constexpr int kNaMaxDevices = 64;
// scratch layout (doubles): partial sums [kNaBlocks * kNaValues], totals of pass 1 [4] and pass 2 [4],
// then the arrival counter (an unsigned int in the first bytes of its own 256-byte slot)
constexpr size_t kNaTotals1 = (size_t)kNaBlocks * kNaValues;
constexpr size_t kNaTotals2 = kNaTotals1 + 4;
constexpr size_t kNaCounter = kNaTotals1 + 32;
constexpr size_t kNaDoubles = kNaCounter + 32;   // 65 792 + 512 bytes

}  // namespace

static __device__ __align__(256) double scratch[kNaDoubles];

namespace {

std::mutex g_na_mu;
double* g_na_ptr[kNaMaxDevices] = {};

// Device address of this device's scratch (hipGetSymbolAddress once per device, with the device current).
int na_scratch(double** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "mr_residual_noalloc: device");
  if (dev < 0 || dev >= kNaMaxDevices) return fail(MR_EINVAL, "mr_residual_noalloc: device %d out of range", dev);
  std::lock_guard<std::mutex> lk(g_na_mu);
  if (!g_na_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "mr_residual_noalloc: scratch");
    g_na_ptr[dev] = static_cast<double*>(p);
  }
  *out = g_na_ptr[dev];
  return MR_OK;
}

}  // namespace

// Zeroes the counter and the totals (a fill kernel rather than a memset node, for graph capture).
__global__ void na_clear_kernel(double* __restrict__ s) {
  const int t = threadIdx.x;
  if (t < 64) s[kNaTotals1 + t] = 0.0;
}

// Pass 1: sum Sigma(0), sum Sigma(0)^2 and sum Sigma(theta) over the mesh (natural order).
__global__ void __launch_bounds__(kNaThreads) na_sigma_kernel(const double* __restrict__ delta,
                                                              const double* __restrict__ theta, int n,
                                                              double* __restrict__ s) {
  double a0 = 0.0, a1 = 0.0, a2 = 0.0;
  const Nb18 zero{};
  for (int row = blockIdx.x; row < n * n; row += gridDim.x) {
    const int i = row / n, j = row - i * n;
    for (int k = threadIdx.x; k < n; k += blockDim.x) {
      const size_t c = ((size_t)i * n + j) * n + k;
      const double opd = 1.0 + delta[c];
      double S;
      const double s0 = sigma_cell(zero, opd, 1.0, S);
      Nb18 t;
      gather18(theta, n, i, j, k, t);
      const double st = sigma_cell(t, opd, 1.0, S);
      a0 += s0;
      a1 += s0 * s0;
      a2 += st;
    }
  }
  double v[4] = {a0, a1, a2, 0.0};
  unsigned* counter = reinterpret_cast<unsigned*>(s + kNaCounter);
  grid_sum<4>(v, s, counter, s + kNaTotals1, gridDim.x, blockIdx.x);
}

// Pass 2: r = nabla^2 theta - (Sigma - <Sigma>) into r_out (may be null); sum r, sum r^2.
__global__ void __launch_bounds__(kNaThreads) na_residual_kernel(const double* __restrict__ delta,
                                                                 const double* __restrict__ theta, int n,
                                                                 double* __restrict__ r_out, double* __restrict__ s) {
  const double cells = (double)n * n * n;
  const double msig = s[kNaTotals1 + 2] / cells;
  double a0 = 0.0, a1 = 0.0;
  for (int row = blockIdx.x; row < n * n; row += gridDim.x) {
    const int i = row / n, j = row - i * n;
    for (int k = threadIdx.x; k < n; k += blockDim.x) {
      const size_t c = ((size_t)i * n + j) * n + k;
      Nb18 t;
      gather18(theta, n, i, j, k, t);
      double S;
      const double sig = sigma_cell(t, 1.0 + delta[c], 1.0, S);
      const double r = (S - 6.0 * theta[c]) - (sig - msig);
      if (r_out) r_out[c] = r;
      a0 += r;
      a1 += r * r;
    }
  }
  double v[4] = {a0, a1, 0.0, 0.0};
  unsigned* counter = reinterpret_cast<unsigned*>(s + kNaCounter);
  grid_sum<4>(v, s, counter, s + kNaTotals2, gridDim.x, blockIdx.x);
}

}  // namespace mr

using namespace mr;

extern "C" int mr_residual_noalloc(int n, const double* delta, const double* theta, double* r_out, double* rel_out,
                                   double* msum_out, void* hip_stream) {
  if (!delta || !theta) return fail(MR_EINVAL, "mr_residual_noalloc: null argument");
  if (n < 4 || n > 1024)
    return fail(MR_EINVAL, "mr_residual_noalloc: n = %d outside 4..1024 (the scratch holds the sums of %d blocks)", n,
                kNaBlocks);
  double* s = nullptr;
  int rc = na_scratch(&s);
  if (rc != MR_OK) return rc;
  hipStream_t st = (hipStream_t)hip_stream;
  const int rows = n * n;
  const unsigned blocks = (unsigned)(rows < kNaBlocks ? rows : kNaBlocks);
  const unsigned threads = (unsigned)(n < kNaThreads ? ((n + 63) / 64) * 64 : kNaThreads);
  hipLaunchKernelGGL(na_clear_kernel, dim3(1), dim3(64), 0, st, s);
  hipLaunchKernelGGL(na_sigma_kernel, dim3(blocks), dim3(threads), 0, st, delta, theta, n, s);
  hipLaunchKernelGGL(na_residual_kernel, dim3(blocks), dim3(threads), 0, st, delta, theta, n, r_out, s);
  hipError_t e = hipGetLastError();
  double tot[8];
  if (e == hipSuccess) e = hipMemcpyAsync(tot, s + kNaTotals1, sizeof tot, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(e, "mr_residual_noalloc");
  const double cells = (double)n * n * n;
  const double v0 = tot[1] - tot[0] * tot[0] / cells;   // ||Sigma(0) - <Sigma(0)>||^2
  const double v1 = tot[5] - tot[4] * tot[4] / cells;   // ||r - <r>||^2 (<r> = 0 up to rounding)
  const double r0 = std::sqrt(v0 > 0.0 ? v0 : 0.0), r1 = std::sqrt(v1 > 0.0 ? v1 : 0.0);
  if (rel_out) *rel_out = r0 > 0.0 ? r1 / r0 : r1;
  if (msum_out) *msum_out = tot[2] / cells;
  return MR_OK;
}
