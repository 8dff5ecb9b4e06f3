// Grid-transfer, residual and reduction kernels of the FAS V-cycle (Sec. II.A.3), FP64.
//
// All are single passes over HBM with neighbour reuse through L1/L2. Kernels that reduce use
// grid-stride loops over a capped grid and the deterministic grid_sum of mr_device.h.
#include "mr_device.h"
#include "mr_kernels.h"

namespace mr {

__device__ __forceinline__ double shift_value(const ShiftRef& c) {
  return (c.c_sum ? (*c.c_sum) * c.c_scale : 0.0) + c.c_add;
}

// One thread per coarse cell: the 8 son defects d = nabla^2 theta - Sigma - f + C (Eq. 18 with
// the level's uniform shift) and the 8-son means of d and theta (restriction R).
__global__ void __launch_bounds__(256) defect_restrict_kernel(const double* __restrict__ theta,
    const double* __restrict__ delta, const double* __restrict__ f, int n, double h2, double ih2,
    ShiftRef cref, double* __restrict__ theta_c, double* __restrict__ theta_c2,
    double* __restrict__ dr) {
  const int m = n >> 1;
  const size_t mc = (size_t)m * m * m;
  const double C = shift_value(cref);
  const size_t N = (size_t)n;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < mc; e += (size_t)gridDim.x * blockDim.x) {
    const int K = (int)(e % m), J = (int)((e / m) % m), I = (int)(e / ((size_t)m * m));
    double sd = 0.0, st = 0.0;
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      const int i = 2 * I + (s >> 2), j = 2 * J + ((s >> 1) & 1), k = 2 * K + (s & 1);
      const size_t g = ((size_t)i * N + j) * N + k;
      Nb18 t;
      gather18(theta, n, i, j, k, t);
      double S;
      const double sig = sigma_cell(t, 1.0 + delta[g], ih2, S);
      const double tc = theta[g];
      const double d = (S - 6.0 * tc) * ih2 - sig - (f ? f[g] : 0.0) + C;
      sd += d;
      st += tc;
    }
    theta_c[e] = 0.125 * st;
    if (theta_c2) theta_c2[e] = 0.125 * st;
    dr[e] = 0.125 * sd;
  }
}

// f = nabla^2 th - Sigma(th) - rd (FAS coarse right-hand side, Eq. 19); sums Sigma + f.
__global__ void __launch_bounds__(256) tau_kernel(const double* __restrict__ th,
    const double* __restrict__ delta, const double* rd, double* f, int n, double ih2, Reduce red) {
  const size_t cells = (size_t)n * n * n;
  double acc = 0.0;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < cells; e += (size_t)gridDim.x * blockDim.x) {
    const int k = (int)(e % n), j = (int)((e / n) % n), i = (int)(e / ((size_t)n * n));
    Nb18 t;
    gather18(th, n, i, j, k, t);
    double S;
    const double sig = sigma_cell(t, 1.0 + delta[e], ih2, S);
    const double fv = (S - 6.0 * th[e]) * ih2 - sig - rd[e];
    f[e] = fv;
    acc += sig + fv;
  }
  double v[1] = {acc};
  grid_sum<1>(v, red.partials, red.counter, red.result, gridDim.x, blockIdx.x);
}

// theta += P(tc - that): trilinear between cell centres, 3/4 on the own coarse cell and 1/4 on
// the neighbour on the side of the fine cell, per axis (Eq. 20).
__global__ void __launch_bounds__(256) prolong_correct_kernel(const double* __restrict__ tc,
    const double* __restrict__ that, double* __restrict__ theta, int n) {
  const int m = n >> 1;
  const size_t cells = (size_t)n * n * n;
  const size_t M = (size_t)m;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < cells; e += (size_t)gridDim.x * blockDim.x) {
    const int k = (int)(e % n), j = (int)((e / n) % n), i = (int)(e / ((size_t)n * n));
    const int I = i >> 1, J = j >> 1, K = k >> 1;
    const int I2 = wrapi((i & 1) ? I + 1 : I - 1, m);
    const int J2 = wrapi((j & 1) ? J + 1 : J - 1, m);
    const int K2 = wrapi((k & 1) ? K + 1 : K - 1, m);
    double acc = 0.0;
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      const int ii = (s & 4) ? I2 : I, jj = (s & 2) ? J2 : J, kk = (s & 1) ? K2 : K;
      const double w = ((s & 4) ? 0.25 : 0.75) * ((s & 2) ? 0.25 : 0.75) * ((s & 1) ? 0.25 : 0.75);
      const size_t g = ((size_t)ii * M + jj) * M + kk;
      acc += w * (tc[g] - that[g]);
    }
    theta[e] += acc;
  }
}

__global__ void __launch_bounds__(256) restrict_kernel(const double* __restrict__ fine,
    double* __restrict__ coarse, int n) {
  const int m = n >> 1;
  const size_t mc = (size_t)m * m * m;
  const size_t N = (size_t)n;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < mc; e += (size_t)gridDim.x * blockDim.x) {
    const int K = (int)(e % m), J = (int)((e / m) % m), I = (int)(e / ((size_t)m * m));
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int i = 2 * I + (q >> 2), j = 2 * J + ((q >> 1) & 1), k = 2 * K + (q & 1);
      s += fine[((size_t)i * N + j) * N + k];
    }
    coarse[e] = 0.125 * s;
  }
}

__global__ void __launch_bounds__(256) residual_kernel(const double* __restrict__ theta,
    const double* __restrict__ delta, int n, double ih2, ShiftRef sref, double* __restrict__ r_out,
    Reduce red) {
  const size_t cells = (size_t)n * n * n;
  const double sh = shift_value(sref);
  double a0 = 0.0, a1 = 0.0;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < cells; e += (size_t)gridDim.x * blockDim.x) {
    double b;
    if (theta) {
      const int k = (int)(e % n), j = (int)((e / n) % n), i = (int)(e / ((size_t)n * n));
      Nb18 t;
      gather18(theta, n, i, j, k, t);
      double S;
      const double sig = sigma_cell(t, 1.0 + delta[e], ih2, S);
      b = (S - 6.0 * theta[e]) * ih2 - sig + sh;
    } else {
      Nb18 t = {};
      double S;
      b = -sigma_cell(t, 1.0 + delta[e], ih2, S) + sh;
    }
    if (r_out) r_out[e] = b;
    a0 += b;
    a1 += b * b;
  }
  double v[2] = {a0, a1};
  grid_sum<2>(v, red.partials, red.counter, red.result, gridDim.x, blockIdx.x);
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

__global__ void __launch_bounds__(256) shift_copy_kernel(const double* in, double* out, size_t cells,
                                                         const double* sum, double scale) {
  const double m = (*sum) * scale;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < cells; e += (size_t)gridDim.x * blockDim.x)
    out[e] = in[e] - m;
}

// ---- launchers ----------------------------------------------------------------------------

static int grid_for(size_t work, int max_blocks) {
  size_t b = (work + 255) / 256;
  if (b < 1) b = 1;
  if (b > (size_t)max_blocks) b = (size_t)max_blocks;
  return (int)b;
}

hipError_t launch_defect_restrict(const double* theta, const double* delta, const double* f,
                                  int n, double h, ShiftRef c, double* theta_c, double* theta_c2,
                                  double* dr, hipStream_t s) {
  const size_t mc = (size_t)(n / 2) * (n / 2) * (n / 2);
  hipLaunchKernelGGL(defect_restrict_kernel, dim3(grid_for(mc, 1 << 20)), dim3(256), 0, s, theta,
                     delta, f, n, h * h, 1.0 / (h * h), c, theta_c, theta_c2, dr);
  return hipGetLastError();
}

hipError_t launch_tau(const double* th, const double* delta, const double* rd, double* f, int n,
                      double h, Reduce red, int max_blocks, hipStream_t s) {
  const size_t cells = (size_t)n * n * n;
  hipLaunchKernelGGL(tau_kernel, dim3(grid_for(cells, max_blocks)), dim3(256), 0, s, th, delta, rd, f,
                     n, 1.0 / (h * h), red);
  return hipGetLastError();
}

hipError_t launch_prolong_correct(const double* tc, const double* that, double* theta, int n,
                                  hipStream_t s) {
  const size_t cells = (size_t)n * n * n;
  hipLaunchKernelGGL(prolong_correct_kernel, dim3(grid_for(cells, 1 << 20)), dim3(256), 0, s, tc,
                     that, theta, n);
  return hipGetLastError();
}

hipError_t launch_restrict(const double* fine, double* coarse, int n, hipStream_t s) {
  const size_t mc = (size_t)(n / 2) * (n / 2) * (n / 2);
  hipLaunchKernelGGL(restrict_kernel, dim3(grid_for(mc, 1 << 20)), dim3(256), 0, s, fine, coarse, n);
  return hipGetLastError();
}

hipError_t launch_residual(const double* theta, const double* delta, int n, double h,
                           ShiftRef shift, double* r_out, Reduce red, int max_blocks, hipStream_t s) {
  const size_t cells = (size_t)n * n * n;
  hipLaunchKernelGGL(residual_kernel, dim3(grid_for(cells, max_blocks)), dim3(256), 0, s, theta,
                     delta, n, 1.0 / (h * h), shift, r_out, red);
  return hipGetLastError();
}

hipError_t launch_validate(const double* delta, size_t cells, Reduce red, int max_blocks, hipStream_t s) {
  hipLaunchKernelGGL(validate_kernel, dim3(grid_for(cells, max_blocks)), dim3(256), 0, s, delta, cells, red);
  return hipGetLastError();
}

hipError_t launch_sum(const double* a, size_t cells, Reduce red, int max_blocks, hipStream_t s) {
  hipLaunchKernelGGL(sum_kernel, dim3(grid_for(cells, max_blocks)), dim3(256), 0, s, a, cells, red);
  return hipGetLastError();
}

hipError_t launch_shift_copy(const double* in, double* out, size_t cells, const double* sum,
                             double scale, hipStream_t s) {
  hipLaunchKernelGGL(shift_copy_kernel, dim3(grid_for(cells, 1 << 20)), dim3(256), 0, s, in, out,
                     cells, sum, scale);
  return hipGetLastError();
}

}  // namespace mr
