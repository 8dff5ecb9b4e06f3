// Grid-transfer, residual, layout and reduction kernels of the FAS cycle (Sec. II.A.3), FP64.
//
// Fields are colour-split (mr_device.h) unless named "natural". Streaming kernels use a 3D grid
// (k within a row, then j, then i) so no index division is needed; reducing kernels walk rows
// with a capped 1D grid and the deterministic grid_sum.
#include "mr_device.h"
#include "mr_kernels.h"

namespace mr {

constexpr int kReduceGrid = 4096;

__device__ __forceinline__ double shift_value(const ShiftRef& c) {
  return (c.c_sum ? (c.c_sum[0] + c.c_sum[1]) * c.c_scale : 0.0) + c.c_add;
}

// f = nabla^2 th - Sigma(th) - rd (FAS coarse right-hand side, Eq. 19); result = (sum of
// Sigma + f, 0), the running sums of the two colours that seed the coarse relaxation's shift.
__global__ void __launch_bounds__(256) tau_kernel(const double* __restrict__ th,
    const double* __restrict__ delta, const double* rd, double* f, int n, double ih2, Reduce red) {
  double acc = 0.0;
  const int rows = n * n;
  const int rpb = (rows + gridDim.x - 1) / gridDim.x;
  const int r0 = xcd_remap(blockIdx.x, gridDim.x) * rpb;
  const int r1 = r0 + rpb < rows ? r0 + rpb : rows;
  for (int row = r0; row < r1; ++row) {
    const int i = row / n, j = row - (row / n) * n;
    for (int k = threadIdx.x; k < n; k += blockDim.x) {
      const unsigned e = split_idx(n, i, j, k);
      Nb18 t;
      gather18_split(th, n, i, j, k, t);
      double S;
      const double sig = sigma_cell(t, 1.0 + delta[e], ih2, S);
      const double fv = (S - 6.0 * th[e]) * ih2 - sig - rd[e];
      f[e] = fv;
      acc += sig + fv;
    }
  }
  double v[2] = {acc, 0.0};
  grid_sum<2>(v, red.partials, red.counter, red.result, gridDim.x, blockIdx.x);
}

__global__ void __launch_bounds__(256) residual_kernel(const double* __restrict__ theta,
    const double* __restrict__ delta, int n, double ih2, ShiftRef sref, double* __restrict__ r_nat,
    Reduce red) {
  const double sh = shift_value(sref);
  double a0 = 0.0, a1 = 0.0;
  const int rows = n * n;
  const int rpb = (rows + gridDim.x - 1) / gridDim.x;
  const int r0 = xcd_remap(blockIdx.x, gridDim.x) * rpb;
  const int r1 = r0 + rpb < rows ? r0 + rpb : rows;
  for (int row = r0; row < r1; ++row) {
    const int i = row / n, j = row - (row / n) * n;
    for (int k = threadIdx.x; k < n; k += blockDim.x) {
      const unsigned e = split_idx(n, i, j, k);
      Nb18 t = {};
      double b;
      if (theta) {
        gather18_split(theta, n, i, j, k, t);
        double S;
        const double sig = sigma_cell(t, 1.0 + delta[e], ih2, S);
        b = (S - 6.0 * theta[e]) * ih2 - sig + sh;
      } else {
        double S;
        b = -sigma_cell(t, 1.0 + delta[e], ih2, S) + sh;
      }
      if (r_nat) r_nat[((size_t)i * n + j) * n + k] = b;
      a0 += b;
      a1 += b * b;
    }
  }
  double v[2] = {a0, a1};
  grid_sum<2>(v, red.partials, red.counter, red.result, gridDim.x, blockIdx.x);
}

// that <- tc - that on the coarse mesh (the coarse correction, formed once before prolongation).
__global__ void __launch_bounds__(256) coarse_diff_kernel(const double* __restrict__ tc, double* __restrict__ that,
                                                          size_t cells) {
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < cells; e += (size_t)gridDim.x * blockDim.x)
    that[e] = tc[e] - that[e];
}

// theta += P(ec) with ec = tc - that: trilinear between cell centres, 3/4 on the own coarse cell
// and 1/4 on the neighbour on the side of the fine cell, per axis (Eq. 20). A thread owns the
// cell pair k = 2m, 2m+1 of row (i, j), which share coarse column K = m; k = 2m takes its
// k-neighbour at K - 1, k = 2m + 1 at K + 1. The two cells lie in the two colour halves at the
// same offset.
__device__ __forceinline__ void prolong_correct_row(const double* __restrict__ ec, double* __restrict__ theta, int n,
                                                    int row, int m) {
  const int nh = n >> 1;
  const int i = row / n, j = row - i * n;
  const int nc = n >> 1;
  const int I = i >> 1, J = j >> 1, K = m;
  const int I2 = wrapi((i & 1) ? I + 1 : I - 1, nc);
  const int J2 = wrapi((j & 1) ? J + 1 : J - 1, nc);
  const int Km = wrapi(K - 1, nc), Kp = wrapi(K + 1, nc);
  const double wI[2] = {0.75, 0.25};
  double lo = 0.0, hi = 0.0;   // cells k = 2m (neighbour K - 1) and k = 2m + 1 (neighbour K + 1)
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const int ii = (s & 2) ? I2 : I, jj = (s & 1) ? J2 : J;
    const double w = wI[(s >> 1) & 1] * wI[s & 1];
    const double ek = ec[split_idx(nc, ii, jj, K)];
    lo += w * (0.75 * ek + 0.25 * ec[split_idx(nc, ii, jj, Km)]);
    hi += w * (0.75 * ek + 0.25 * ec[split_idx(nc, ii, jj, Kp)]);
  }
  const unsigned half = (unsigned)n * (unsigned)n * (unsigned)nh;
  const unsigned off = ((unsigned)i * n + j) * (unsigned)nh + m;
  // cell k = 2m has colour (i + j) & 1, cell k = 2m + 1 the other one
  const int c0 = (i + j) & 1;
  theta[c0 * half + off] += lo;
  theta[(1 - c0) * half + off] += hi;
}

// Each block handles a contiguous range of rows (blocks are mapped XCD-aware), a thread one
// column m of every row in it.
__global__ void __launch_bounds__(512) prolong_correct_kernel(const double* __restrict__ ec,
    double* __restrict__ theta, int n, int rows_per_block) {
  const int nh = n >> 1;
  const int r0 = xcd_remap(blockIdx.x, gridDim.x) * rows_per_block;
  const int r1 = min(r0 + rows_per_block, n * n);
  for (int row = r0; row < r1; ++row)
    for (int m = threadIdx.x; m < nh; m += blockDim.x) prolong_correct_row(ec, theta, n, row, m);
}

__global__ void __launch_bounds__(512) restrict_kernel(const double* __restrict__ fine,
    double* __restrict__ coarse, int n) {
  const int m = n >> 1;
  const int row = xcd_remap(blockIdx.x, gridDim.x);
  const int I = row / m, J = row - I * m;
  const int K = threadIdx.x;
  if (K >= m) return;
  double s = 0.0;
#pragma unroll
  for (int q = 0; q < 8; ++q)
    s += fine[split_idx(n, 2 * I + (q >> 2), 2 * J + ((q >> 1) & 1), 2 * K + (q & 1))];
  coarse[split_idx(m, I, J, K)] = 0.125 * s;
}

__global__ void __launch_bounds__(1024) to_split_kernel(const double* __restrict__ nat,
    double* __restrict__ sp, int n) {
  const int row = xcd_remap(blockIdx.x, gridDim.x);
  const int i = row / n, j = row - i * n;
  const int k = threadIdx.x;
  if (k >= n) return;
  sp[split_idx(n, i, j, k)] = nat[((size_t)i * n + j) * n + k];
}

__global__ void __launch_bounds__(1024) from_split_kernel(const double* __restrict__ sp,
    double* __restrict__ nat, int n, const double* sum, double scale) {
  const int row = xcd_remap(blockIdx.x, gridDim.x);
  const int i = row / n, j = row - i * n;
  const int k = threadIdx.x;
  if (k >= n) return;
  const double mshift = sum ? (*sum) * scale : 0.0;
  nat[((size_t)i * n + j) * n + k] = sp[split_idx(n, i, j, k)] - mshift;
}

__global__ void __launch_bounds__(256) validate_kernel(const double* __restrict__ delta, size_t cells, Reduce red) {
  double bad = 0.0;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < cells; e += (size_t)gridDim.x * blockDim.x) {
    const double v = 1.0 + delta[e];
    if (!(v > 0.0) || !__builtin_isfinite(v)) bad += 1.0;
  }
  double v[1] = {bad};
  grid_sum<1>(v, red.partials, red.counter, red.result, gridDim.x, blockIdx.x);
}

__global__ void __launch_bounds__(256) sum_kernel(const double* __restrict__ a, size_t cells, Reduce red) {
  double s = 0.0;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < cells; e += (size_t)gridDim.x * blockDim.x)
    s += a[e];
  double v[1] = {s};
  grid_sum<1>(v, red.partials, red.counter, red.result, gridDim.x, blockIdx.x);
}

// ---- launchers ----------------------------------------------------------------------------

// One block per row (i, j) of the mesh; n <= 1024 so a row fits one block.
static dim3 rows_of(int n) { return dim3((unsigned)n * (unsigned)n); }
static int rows_grid(int n) { return n * n < kReduceGrid ? n * n : kReduceGrid; }
static int lin_grid(size_t cells) {
  size_t b = (cells + 255) / 256;
  return (int)(b < 1 ? 1 : (b > (size_t)kReduceGrid ? kReduceGrid : b));
}
static int row_threads(int n) { return n < 64 ? 64 : (n < 256 ? n : 256); }

hipError_t launch_tau(const double* th, const double* delta, const double* rd, double* f, int n,
                      double h, Reduce red, hipStream_t s) {
  bool done = false;
  hipError_t e = launch_tau_pipe(th, delta, rd, f, n, h, red, s, &done);
  if (e != hipSuccess || done) return e;
  hipLaunchKernelGGL(tau_kernel, dim3(rows_grid(n)), dim3(row_threads(n)), 0, s, th, delta, rd, f, n,
                     1.0 / (h * h), red);
  return hipGetLastError();
}

hipError_t launch_prolong_correct(const double* tc, double* that, double* theta, int n, hipStream_t s) {
  const size_t cc = (size_t)(n / 2) * (n / 2) * (n / 2);
  hipLaunchKernelGGL(coarse_diff_kernel, dim3(lin_grid(cc)), dim3(256), 0, s, tc, that, cc);
  const int rows = n * n;
  const int rpb = rows > 16384 ? (rows + 8191) / 8192 : 1;
  const int blocks = (rows + rpb - 1) / rpb;
  hipLaunchKernelGGL(prolong_correct_kernel, dim3(blocks), dim3(n / 2 < 512 ? n / 2 : 512), 0, s, that, theta, n, rpb);
  return hipGetLastError();
}

hipError_t launch_restrict(const double* fine, double* coarse, int n, hipStream_t s) {
  const int m = n / 2;
  hipLaunchKernelGGL(restrict_kernel, rows_of(m), dim3(m), 0, s, fine, coarse, n);
  return hipGetLastError();
}

hipError_t launch_residual(const double* theta, const double* delta, int n, double h, ShiftRef shift,
                           double* r_natural, Reduce red, hipStream_t s) {
  hipLaunchKernelGGL(residual_kernel, dim3(rows_grid(n)), dim3(row_threads(n)), 0, s, theta, delta, n,
                     1.0 / (h * h), shift, r_natural, red);
  return hipGetLastError();
}

hipError_t launch_to_split(const double* natural, double* split, int n, hipStream_t s) {
  hipLaunchKernelGGL(to_split_kernel, rows_of(n), dim3(n), 0, s, natural, split, n);
  return hipGetLastError();
}

hipError_t launch_from_split(const double* split, double* natural, int n, const double* sum, double scale,
                             hipStream_t s) {
  hipLaunchKernelGGL(from_split_kernel, rows_of(n), dim3(n), 0, s, split, natural, n, sum, scale);
  return hipGetLastError();
}

hipError_t launch_validate(const double* delta, size_t cells, Reduce red, hipStream_t s) {
  hipLaunchKernelGGL(validate_kernel, dim3(lin_grid(cells)), dim3(256), 0, s, delta, cells, red);
  return hipGetLastError();
}

hipError_t launch_sum(const double* a, size_t cells, Reduce red, hipStream_t s) {
  hipLaunchKernelGGL(sum_kernel, dim3(lin_grid(cells)), dim3(256), 0, s, a, cells, red);
  return hipGetLastError();
}

}  // namespace mr
