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

// Trilinear prolongation with correction, t += P(ec - mu) (mu = 0 unless SHIFT), a thread per
// coarse cell (I, J, K): it loads the 3 x 3 x 3 coarse neighbourhood once and updates the 8 fine
// sons, fine rows i = 2I + a, j = 2J + b and the cell pair k = 2K, 2K + 1 (both colours at column
// K), issuing all 8 fine loads before any store. A fine cell takes 3/4 of its own coarse parent
// and 1/4 of the neighbour towards it in each direction, the weights multiplied across x, y, z
// (Eq. 20).
template <bool SHIFT>
__global__ void __launch_bounds__(256) prolong_quad_kernel(const double* __restrict__ ec, const double* mu_sum,
                                                          double mu_scale, double* __restrict__ theta, int n) {
  const int nc = n >> 1, nh = nc;
  const long total = (long)nc * nc * nc;
  const long gid = (long)xcd_remap(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (gid >= total) return;
  const int K = (int)(gid % nc);
  const long rest = gid / nc;
  const int J = (int)(rest % nc), I = (int)(rest / nc);
  const double mu = SHIFT && mu_sum ? (mu_sum[0] + mu_sum[1]) * mu_scale : 0.0;
  // e[a][b][c]: coarse cell (I - 1 + a, J - 1 + b, K - 1 + c)
  double e[3][3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const double v = ec[split_idx(nc, wrapi(I - 1 + a, nc), wrapi(J - 1 + b, nc), wrapi(K - 1 + c, nc))];
        e[a][b][c] = SHIFT ? v - mu : v;
      }
  const unsigned half = (unsigned)n * (unsigned)n * (unsigned)nh;
  unsigned off[2][2];
  int c0[2][2];
  double t[2][2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const int i = 2 * I + a, j = 2 * J + b;
      off[a][b] = ((unsigned)i * n + j) * (unsigned)nh + K;
      c0[a][b] = (i + j) & 1;
      t[a][b][0] = theta[c0[a][b] * half + off[a][b]];
      t[a][b][1] = theta[(1 - c0[a][b]) * half + off[a][b]];
    }
  const double wI[2] = {0.75, 0.25};
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      // neighbour plane / row of the fine cell: I - 1 for even i, I + 1 for odd (index 0 or 2)
      const int a2 = a ? 2 : 0, b2 = b ? 2 : 0;
      double lo = 0.0, hi = 0.0;   // cells k = 2K (neighbour K - 1) and k = 2K + 1 (neighbour K + 1)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int ia = (q & 2) ? a2 : 1, jb = (q & 1) ? b2 : 1;
        const double w = wI[(q >> 1) & 1] * wI[q & 1];
        const double ek = e[ia][jb][1];
        lo += w * (0.75 * ek + 0.25 * e[ia][jb][0]);
        hi += w * (0.75 * ek + 0.25 * e[ia][jb][2]);
      }
      theta[c0[a][b] * half + off[a][b]] = t[a][b][0] + lo;
      theta[(1 - c0[a][b]) * half + off[a][b]] = t[a][b][1] + hi;
    }
}

// The same update with the coarse neighbourhood staged in LDS: a block of 256 threads covers coarse
// plane I, rows J0 .. J0 + R - 1 (R = 256 / nc) and every column K; it first copies the coarse rows
// I-1..I+1 x J0-1..J0+R of both colours into LDS in natural k order (coalesced along each colour),
// then each thread reads its 3 x 3 x 3 neighbourhood from LDS. Requires nc = n / 2 to divide 256
// and R <= nc (16 <= nc <= 256).
template <bool SHIFT>
__global__ void __launch_bounds__(256) prolong_rows_kernel(const double* __restrict__ ec, const double* mu_sum,
                                                           double mu_scale, double* __restrict__ theta, int n) {
  __shared__ double cl[3 * (256 + 2 * 256)];   // 3 planes x (R + 2) rows x nc = 3 (256 + 2 nc), nc <= 256
  const int nc = n >> 1, nh = nc, nch = nc >> 1;
  const int R = 256 / nc;
  const int groups = nc / R;
  const int blk = xcd_remap(blockIdx.x, gridDim.x);
  const int I = blk / groups, J0 = (blk - I * groups) * R;
  const int tid = threadIdx.x;
  const double mu = SHIFT && mu_sum ? (mu_sum[0] + mu_sum[1]) * mu_scale : 0.0;
  const unsigned halfc = (unsigned)nc * (unsigned)nc * (unsigned)nch;
  // loader: LDS row w = a * (R + 2) + b holds coarse row (I - 1 + a, J0 - 1 + b); element index
  // x = w * nc + c * nch + m (colour-major inside a row) goes to position k = 2m + ((ii + jj + c) & 1)
  const int rows = 3 * (R + 2);
  for (int x = tid; x < rows * nc; x += 256) {
    const int w = x / nc, pos = x - w * nc;
    const int a = w / (R + 2), b = w - a * (R + 2);
    const int c = pos / nch, m = pos - c * nch;
    const int ii = wrapi(I - 1 + a, nc), jj = wrapi(J0 - 1 + b, nc);
    const double v = ec[(unsigned)c * halfc + ((unsigned)ii * nc + jj) * (unsigned)nch + m];
    cl[w * nc + 2 * m + ((ii + jj + c) & 1)] = SHIFT ? v - mu : v;
  }
  __syncthreads();
  const int r = tid / nc, K = tid - r * nc;
  const int J = J0 + r;
  const int km = K == 0 ? nc - 1 : K - 1, kp = K == nc - 1 ? 0 : K + 1;
  double e[3][3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      const double* row = cl + (a * (R + 2) + r + b) * nc;
      e[a][b][0] = row[km];
      e[a][b][1] = row[K];
      e[a][b][2] = row[kp];
    }
  const unsigned half = (unsigned)n * (unsigned)n * (unsigned)nh;
  unsigned off[2][2];
  int c0[2][2];
  double t[2][2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const int i = 2 * I + a, j = 2 * J + b;
      off[a][b] = ((unsigned)i * n + j) * (unsigned)nh + K;
      c0[a][b] = (i + j) & 1;
      t[a][b][0] = theta[c0[a][b] * half + off[a][b]];
      t[a][b][1] = theta[(1 - c0[a][b]) * half + off[a][b]];
    }
  const double wI[2] = {0.75, 0.25};
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const int a2 = a ? 2 : 0, b2 = b ? 2 : 0;
      double lo = 0.0, hi = 0.0;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int ia = (q & 2) ? a2 : 1, jb = (q & 1) ? b2 : 1;
        const double w = wI[(q >> 1) & 1] * wI[q & 1];
        const double ek = e[ia][jb][1];
        lo += w * (0.75 * ek + 0.25 * e[ia][jb][0]);
        hi += w * (0.75 * ek + 0.25 * e[ia][jb][2]);
      }
      theta[c0[a][b] * half + off[a][b]] = t[a][b][0] + lo;
      theta[(1 - c0[a][b]) * half + off[a][b]] = t[a][b][1] + hi;
    }
}

hipError_t launch_prolong_add(const double* ec, const double* mu_sum, double mu_scale, double* theta, int n,
                              hipStream_t s) {
  const long total = (long)(n / 2) * (n / 2) * (n / 2);
  const unsigned blocks = (unsigned)((total + 255) / 256);
  const int nc = n / 2;
  if (nc >= 16 && nc <= 256 && 256 % nc == 0) {   // blocks = nc^3 / 256: whole row groups
    if (mu_sum)
      hipLaunchKernelGGL((prolong_rows_kernel<true>), dim3(blocks), dim3(256), 0, s, ec, mu_sum, mu_scale, theta, n);
    else
      hipLaunchKernelGGL((prolong_rows_kernel<false>), dim3(blocks), dim3(256), 0, s, ec, mu_sum, mu_scale, theta, n);
    return hipGetLastError();
  }
  if (mu_sum)
    hipLaunchKernelGGL((prolong_quad_kernel<true>), dim3(blocks), dim3(256), 0, s, ec, mu_sum, mu_scale, theta, n);
  else
    hipLaunchKernelGGL((prolong_quad_kernel<false>), dim3(blocks), dim3(256), 0, s, ec, mu_sum, mu_scale, theta, n);
  return hipGetLastError();
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
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? launch_prolong_add(that, nullptr, 0.0, theta, n, s) : e;
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
