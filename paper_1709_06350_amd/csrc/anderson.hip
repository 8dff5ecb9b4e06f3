// Anderson acceleration of the FAS V-cycle (an addition to the paper's method, for inputs on
// which the plain cycle converges slowly: near-empty cells, where the coarse-grid correction
// contributes little). With y_k = V(x_k) the result of one V-cycle from x_k and f_k = y_k - x_k,
// the next iterate is x_{k+1} = y_k - sum_i gamma_i (y_{i+1} - y_i) over the last m steps, where
// gamma minimises |f_k - sum_i gamma_i (f_{i+1} - f_i)|_2 (Anderson mixing with unit damping).
// The fixed point, and so the solution, is that of the plain V-cycle.
//
// Device side: one pass records f_k (in FP32: it only enters the small least-squares problem) and
// y_k (FP64) into the history ring and forms the dot products of f_k with every stored f
// (deterministic: per-block partials, added in block order by one block);
// one pass forms x_{k+1} as a linear combination of stored y. The small least-squares problem is
// solved on the host from the Gram matrix of the stored f.
#include <algorithm>
#include <cmath>
#include <vector>

#include "mr.h"
#include "mr_ctx.h"
#include "mr_device.h"
#include "mr_kernels.h"

namespace mr {

constexpr int kAAMaxRing = kAAMaxDepth + 1;
constexpr int kAABlocks = 8192;

struct AAPtrs {
  const double* p[kAAMaxRing];
};
struct AAPtrsF {
  const float* p[kAAMaxRing];
};

// f = y - x (rounded to FP32) into f_out, y into y_out; partials[block][j] = sum over the block's
// cells of f * ring_j (ring_j == f_out gives |f|^2).
// f_out is one of the ring entries, so it is not declared __restrict__; its own dot product uses
// the value in registers.
__global__ void __launch_bounds__(256) aa_record_kernel(const double* __restrict__ x, const double* __restrict__ y,
                                                        float* f_out, double* __restrict__ y_out, AAPtrsF ring,
                                                        int nr, size_t cells, double* __restrict__ partials) {
  __shared__ double red[4][kAAMaxRing];
  double acc[kAAMaxRing];
#pragma unroll
  for (int j = 0; j < kAAMaxRing; ++j) acc[j] = 0.0;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < cells; e += (size_t)gridDim.x * blockDim.x) {
    const double yv = y[e];
    const float f = (float)(yv - x[e]);
    f_out[e] = f;
    y_out[e] = yv;
#pragma unroll
    for (int j = 0; j < kAAMaxRing; ++j)
      if (j < nr) acc[j] += (double)f * (double)(ring.p[j] == f_out ? f : ring.p[j][e]);
  }
  block_sum<kAAMaxRing>(acc, red, threadIdx.x, blockDim.x);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int j = 0; j < kAAMaxRing; ++j) partials[(size_t)blockIdx.x * kAAMaxRing + j] = acc[j];
  }
}

// The same record for an iteration whose step is a known FP32 correction (the mixed-precision outer
// iteration theta -> theta + e): f = e exactly and y = theta + e, so the update pass is not needed.
__global__ void __launch_bounds__(256) aa_record_e_kernel(const double* __restrict__ theta, const float* __restrict__ e,
                                                          float* f_out, double* __restrict__ y_out, AAPtrsF ring, int nr,
                                                          size_t cells, double* __restrict__ partials) {
  __shared__ double red[4][kAAMaxRing];
  double acc[kAAMaxRing];
#pragma unroll
  for (int j = 0; j < kAAMaxRing; ++j) acc[j] = 0.0;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < cells; i += (size_t)gridDim.x * blockDim.x) {
    const float f = e[i];
    f_out[i] = f;
    y_out[i] = theta[i] + (double)f;
#pragma unroll
    for (int j = 0; j < kAAMaxRing; ++j)
      if (j < nr) acc[j] += (double)f * (double)(ring.p[j] == f_out ? f : ring.p[j][i]);
  }
  block_sum<kAAMaxRing>(acc, red, threadIdx.x, blockDim.x);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int j = 0; j < kAAMaxRing; ++j) partials[(size_t)blockIdx.x * kAAMaxRing + j] = acc[j];
  }
}

// out[j] = sum over blocks of partials[block][j], in block order (one block).
__global__ void __launch_bounds__(256) aa_sum_kernel(const double* __restrict__ partials, int nblocks,
                                                     double* __restrict__ out) {
  __shared__ double red[4][kAAMaxRing];
  double acc[kAAMaxRing];
#pragma unroll
  for (int j = 0; j < kAAMaxRing; ++j) acc[j] = 0.0;
  for (int b = threadIdx.x; b < nblocks; b += blockDim.x)
#pragma unroll
    for (int j = 0; j < kAAMaxRing; ++j) acc[j] += partials[(size_t)b * kAAMaxRing + j];
  block_sum<kAAMaxRing>(acc, red, threadIdx.x, blockDim.x);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int j = 0; j < kAAMaxRing; ++j) out[j] = acc[j];
  }
}

struct AACoef {
  double c[kAAMaxRing];
};

// out = out2 = sum_j c_j ring_j (the new iterate, and its copy kept as x for the next step; out2
// may be null).
__global__ void __launch_bounds__(256) aa_combine_kernel(AAPtrs ring, AACoef c, int nr, size_t cells,
                                                         double* __restrict__ out, double* __restrict__ out2) {
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < cells; e += (size_t)gridDim.x * blockDim.x) {
    double v = 0.0;
#pragma unroll
    for (int j = 0; j < kAAMaxRing; ++j)
      if (j < nr) v += c.c[j] * ring.p[j][e];
    out[e] = v;
    if (out2) out2[e] = v;
  }
}

int Ctx::aa_reserve(int depth) {
  const size_t cells = lv[0].cells;
  if (aa_mem && aa_ring >= depth + 1) return MR_OK;
  if (aa_mem) {
    (void)hipFree(aa_mem);
    aa_mem = nullptr;
  }
  const int ring = depth + 1;
  // x save, ring of y (FP64), ring of f (FP32, counted in doubles), partials, dot results
  const size_t count = cells * (1 + (size_t)ring) + (cells * (size_t)ring + 1) / 2 + (size_t)kAABlocks * kAAMaxRing +
                       kAAMaxRing;
  hipError_t e = hipMalloc((void**)&aa_mem, count * sizeof(double));
  if (e != hipSuccess) {
    aa_mem = nullptr;
    return fail(MR_ENOMEM, "Anderson history (%d steps): %s", depth, hipGetErrorString(e));
  }
  aa_ring = ring;
  return MR_OK;
}

void Ctx::aa_release() {
  if (aa_mem) (void)hipFree(aa_mem);
  aa_mem = nullptr;
  aa_ring = 0;
}

AAState::AAState(int depth_, int ring_) : depth(depth_), ring(ring_), gram((size_t)ring_ * ring_, 0.0) {}

// Solves the small dense system a z = b (n <= kAAMaxDepth) by Gaussian elimination with partial
// pivoting; false if a pivot is negligible against the largest diagonal entry.
static bool solve_small(std::vector<double> a, std::vector<double> b, int n, std::vector<double>& z) {
  double scale = 0.0;
  for (int i = 0; i < n; ++i) scale = std::fmax(scale, std::fabs(a[i * n + i]));
  if (!(scale > 0.0)) return false;
  for (int k = 0; k < n; ++k) {
    int p = k;
    for (int i = k + 1; i < n; ++i)
      if (std::fabs(a[i * n + k]) > std::fabs(a[p * n + k])) p = i;
    if (!(std::fabs(a[p * n + k]) > 1e-13 * scale)) return false;
    if (p != k) {
      for (int j = 0; j < n; ++j) std::swap(a[k * n + j], a[p * n + j]);
      std::swap(b[k], b[p]);
    }
    for (int i = k + 1; i < n; ++i) {
      const double m = a[i * n + k] / a[k * n + k];
      for (int j = k; j < n; ++j) a[i * n + j] -= m * a[k * n + j];
      b[i] -= m * b[k];
    }
  }
  z.assign(n, 0.0);
  for (int i = n - 1; i >= 0; --i) {
    double s = b[i];
    for (int j = i + 1; j < n; ++j) s -= a[i * n + j] * z[j];
    z[i] = s / a[i * n + i];
  }
  return true;
}

// Called after a V-cycle took x (st.x_prev: the saved start of the first cycle, the previous
// combination, or the previous cycle's result in the y ring) to y = the level-0 iterate. Records
// the step, then overwrites the iterate with the Anderson combination (also kept as the next x).
// With `correction` (the mixed outer iteration) the iterate is x itself, not yet updated, and the
// step is y = x + correction: the record forms y, and the iterate receives the combination or y.
int Ctx::aa_step(AAState& st, double* iterate, const float* correction) {
  const size_t cells = lv[0].cells;
  double* xsave = aa_mem;
  double* Y = aa_mem + cells;
  double* part = Y + cells * (size_t)aa_ring;
  double* dots = part + (size_t)kAABlocks * kAAMaxRing;
  float* F = reinterpret_cast<float*>(dots + kAAMaxRing);
  const int slot = (int)(st.steps % st.ring);
  st.order.push_back(slot);
  if ((int)st.order.size() > st.depth + 1) st.order.erase(st.order.begin());
  const int nr = (int)st.order.size();
  AAPtrsF rp{};
  for (int j = 0; j < nr; ++j) rp.p[j] = F + cells * (size_t)st.order[j];
  const int nb = (int)std::min<size_t>((cells + 255) / 256, (size_t)kAABlocks);
  if (correction)
    hipLaunchKernelGGL(aa_record_e_kernel, dim3(nb), dim3(256), 0, stream, iterate, correction,
                       F + cells * (size_t)slot, Y + cells * (size_t)slot, rp, nr, cells, part);
  else
    hipLaunchKernelGGL(aa_record_kernel, dim3(nb), dim3(256), 0, stream, st.x_prev ? st.x_prev : xsave, iterate,
                       F + cells * (size_t)slot, Y + cells * (size_t)slot, rp, nr, cells, part);
  hipLaunchKernelGGL(aa_sum_kernel, dim3(1), dim3(256), 0, stream, part, nb, dots);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "Anderson record");
  double d[kAAMaxRing];
  e = hipMemcpyAsync(d, dots, nr * sizeof(double), hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return hip_fail(e, "Anderson dots");
  for (int j = 0; j < nr; ++j) {
    st.gram[(size_t)slot * st.ring + st.order[j]] = d[j];
    st.gram[(size_t)st.order[j] * st.ring + slot] = d[j];
  }
  ++st.steps;
  const int m = nr - 1;  // differences available
  AACoef cf{};
  bool mixed = false;
  if (m >= 1) {
    auto G = [&](int a, int b) { return st.gram[(size_t)st.order[a] * st.ring + st.order[b]]; };
    std::vector<double> M((size_t)m * m), b(m), gam;
    double tr = 0.0;
    for (int i = 0; i < m; ++i) {
      for (int j = 0; j < m; ++j) M[(size_t)i * m + j] = G(i + 1, j + 1) - G(i + 1, j) - G(i, j + 1) + G(i, j);
      b[i] = G(i + 1, m) - G(i, m);
      tr += M[(size_t)i * m + i];
    }
    for (int i = 0; i < m; ++i) M[(size_t)i * m + i] += 1e-12 * tr / m;  // small Tikhonov term
    if (solve_small(M, b, m, gam)) {
      for (int j = 0; j < nr; ++j) cf.c[j] = 0.0;
      cf.c[m] = 1.0;
      for (int i = 0; i < m; ++i) {
        cf.c[i + 1] -= gam[i];
        cf.c[i] += gam[i];
      }
      mixed = true;
    } else {
      // ill-conditioned history: restart from this step
      st.order.erase(st.order.begin(), st.order.end() - 1);
    }
  }
  if (!mixed) {  // x_{k+1} = y_k: stored in the y ring (and already the iterate without a correction)
    st.x_prev = Y + cells * (size_t)slot;
    if (correction) {
      e = hipMemcpyAsync(iterate, Y + cells * (size_t)slot, cells * sizeof(double), hipMemcpyDeviceToDevice, stream);
      if (e != hipSuccess) return hip_fail(e, "Anderson step");
    }
    return MR_OK;
  }
  AAPtrs yp{};
  for (int j = 0; j < nr; ++j) yp.p[j] = Y + cells * (size_t)st.order[j];
  hipLaunchKernelGGL(aa_combine_kernel, dim3(nb), dim3(256), 0, stream, yp, cf, nr, cells, iterate,
                     correction ? (double*)nullptr : xsave);
  st.x_prev = xsave;
  e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "Anderson combine");
  return MR_OK;
}

hipError_t aa_save(const Ctx& c, const double* iterate) {
  return hipMemcpyAsync(c.aa_mem, iterate, c.lv[0].cells * sizeof(double), hipMemcpyDeviceToDevice, c.stream);
}

}  // namespace mr
