// Mixed-precision form of the solve: an FP64 defect-correction (Newton) outer loop on the finest
// mesh around an FP32 linear multigrid for the Jacobian of the mean-projected operator.
//
// Outer step: r = -F(theta) in FP64 (F the mean-projected operator of Sec. II.A.1, Eq. 15; the
// residual also decides convergence), then J_p e = r is solved approximately by FP32 V-cycles,
// and theta += e in FP64. Representing e separately keeps FP32 rounding out of theta itself.
//
// Linearisation (differentiating the physical root of the cubic, Sec. II, Eqs. 8-10):
// dSigma(e) = tr(W dMbar(e)), W = (9 s Mbar - 27 Mbar^2) / (3 s^2 + p), so with the traceless
// part Wbar of W, h^2 dSigma(e) = sum_a Wbar_aa S_a(e) + sum_{a<b} W_ab D_ab(e) / 2 (S_a the pair
// sum along axis a, D_ab the cross difference of e). The Jacobian J_p e = nabla^2 e - dSigma(e)
// + <dSigma(e)> keeps the -6/h^2 diagonal of the nonlinear operator, so the inner smoother is the
// same red-black point update with the source replaced by dSigma(e) and no root finding:
//     e_c <- (sum of 6 face neighbours of e - h^2 (dSigma_c(e) + rhs_c - C)) / 6.
// W is rebuilt on the fly in every sweep from an FP32 copy of the base potential (both colours in
// LDS with e) and the FP32 base root s; coarse meshes use the restricted base potential and
// their own root (rediscretisation).
#include <algorithm>
#include <map>
#include <mutex>
#include <type_traits>
#include <utility>
#include <vector>

#include "mr_ctx.h"
#include "mr_device.h"
#include "mr_kernels.h"
#include "mixed_device.h"
#include "tuning.h"

namespace mr {

// Compiled tile shapes (tm columns of m, tj rows) of the FP32 linear sweeps.
#define MR_LIN_TILES(X) X(64, 8) X(64, 4) X(64, 16) X(32, 16) X(32, 8) X(16, 16) X(8, 16) X(4, 8) X(2, 4)

template <int TM, int TJ>
__global__ void __launch_bounds__(TM * TJ) lin_half_sweep_tiled(LinSweepArgs a) {
  __shared__ float lds[LinTile<TM, TJ>::LDS];
  lin_sweep_body<TM, TJ>(a, xcd_remap(blockIdx.x, gridDim.x), blockIdx.x, gridDim.x, lds);
}

__global__ void __launch_bounds__(256) mixed_resid64_kernel(const double* __restrict__ theta,
    const double* __restrict__ delta, int n, ShiftRef cref, float* __restrict__ rhs32, int* __restrict__ baseq,
    const double* __restrict__ bq, float* __restrict__ sb32, Reduce red) {
  mixed_resid64_body(theta, delta, n, cref, rhs32, baseq, bq, sb32, red, blockIdx.x, gridDim.x);
}

__global__ void __launch_bounds__(256) base_root_kernel(const int* __restrict__ baseq, const double* __restrict__ bq,
    const double* __restrict__ delta, int n, double ih2, float* __restrict__ sb32) {
  base_root_body(baseq, bq, delta, n, ih2, sb32, blockIdx.x, gridDim.x);
}

__global__ void __launch_bounds__(512) restrictq_kernel(const int* __restrict__ fine, int* __restrict__ coarse, int n) {
  restrictq_body(fine, coarse, n, blockIdx.x, gridDim.x);
}

__global__ void __launch_bounds__(256) absmax_kernel(const double* __restrict__ a, size_t cells, double* tmax) {
  absmax_body(a, cells, tmax, blockIdx.x, gridDim.x);
}

__global__ void base_scale_kernel(double* tmax, double* bq) {
  if (threadIdx.x == 0) base_scale_body(tmax, bq);
}

__global__ void __launch_bounds__(256) quantise_kernel(const double* __restrict__ src, int* __restrict__ dst, size_t cells,
                                                       const double* __restrict__ bq) {
  const double qs = bq[1];
  for (size_t x = blockIdx.x * (size_t)blockDim.x + threadIdx.x; x < cells; x += (size_t)gridDim.x * blockDim.x)
    dst[x] = base_quantise(src[x], qs);
}

__global__ void __launch_bounds__(256) lin_resid_restrict_kernel(const float* __restrict__ e,
    const int* __restrict__ baseq, const double* __restrict__ bq, const float* __restrict__ sb,
    const float* __restrict__ rhs, int n, float ih2, ShiftRef cref, float* __restrict__ rhs_c, Reduce red) {
  lin_resid_restrict_body(e, baseq, bq, sb, rhs, n, ih2, cref, rhs_c, red, blockIdx.x, gridDim.x);
}

__global__ void __launch_bounds__(256) prolong_add32_kernel(const float* __restrict__ ec, float* __restrict__ e, int n) {
  prolong_add32_body(ec, e, n, blockIdx.x, gridDim.x);
}

__global__ void __launch_bounds__(256) lin_coarsest_kernel(float* __restrict__ e, const int* __restrict__ baseq,
    const double* __restrict__ bq, const float* __restrict__ sb, const float* __restrict__ rhs, int n, int nsweeps,
    float h2, float ih2, const double* c_sum, double c_scale) {
  __shared__ LinCoarsestShared sh;
  lin_coarsest_body(e, baseq, bq, sb, rhs, n, nsweeps, h2, ih2, c_sum, c_scale, sh);
}

__global__ void __launch_bounds__(kTailThreads) lin_tail_kernel(LinTailArgs a) {
  __shared__ LinTailShared sh;
  lin_tail_body(a, sh);
}

__global__ void __launch_bounds__(256) update64_kernel(double* __restrict__ theta, const float* __restrict__ e, size_t cells,
                                                       double* tmax) {
  update64_body(theta, e, cells, blockIdx.x, gridDim.x, tmax);
}

__global__ void __launch_bounds__(256) fill32_kernel(float* __restrict__ a, float v, size_t cells) {
  fill32_body(a, v, cells, blockIdx.x, gridDim.x);
}

template <int TM, int TJ, int COL, bool ZB = false>
__global__ void __launch_bounds__(TM * TJ) lin_sweep_pipe(LinSweepArgs a) {
  __shared__ float lds[LinTile<TM, TJ>::LDS];
  lin_sweep_pipe_body<TM, TJ, COL, ZB>(a, xcd_remap(blockIdx.x, gridDim.x), blockIdx.x, gridDim.x, lds);
}

// (J z)_c = nabla^2 z - dSigma(z) at every cell (rows of the mesh dealt to blocks), FP32.
__global__ void __launch_bounds__(256) lin_apply_row_kernel(const float* __restrict__ z, const int* __restrict__ baseq,
    const double* __restrict__ bq, const float* __restrict__ sb, int n, float ih2, float* __restrict__ w) {
  const float* __restrict__ base = reinterpret_cast<const float*>(baseq);
  const float bscl = (float)bq[0];
  for (int row = blockIdx.x; row < n * n; row += gridDim.x) {
    const int i = row / n, j = row - i * n;
    for (int k = threadIdx.x; k < n; k += blockDim.x) {
      const unsigned g = split_idx(n, i, j, k);
      Nb18f te, tb;
      gather18_split_t(z, n, i, j, k, te);
      gather18_split_t(base, n, i, j, k, tb);
      float Se;
      const float src = lin_source(tb, base[g], bscl, sb[g], ih2, te, Se) * ih2;
      w[g] = (Se - 6.0f * z[g]) * ih2 - src;
    }
  }
}

template <int K>
__global__ void __launch_bounds__(256) kry_dots_kernel(const float* __restrict__ w, KryPtrs v, size_t cells,
                                                       double* partials, unsigned* counter, double* result) {
  kry_dots_body<K>(w, v, cells, partials, counter, result, blockIdx.x, gridDim.x);
}

template <int TM, int TJ, int K>
__global__ void __launch_bounds__(2 * TM * TJ) lin_apply_dots(LinApplyArgs a) {
  __shared__ float lds[LinTile<TM, TJ>::LDS];
  lin_apply_dots_body<TM, TJ, K>(a, xcd_remap(blockIdx.x, gridDim.x), blockIdx.x, gridDim.x, lds);
}

__global__ void __launch_bounds__(256) kry_orth_kernel(const float* __restrict__ w, KryPtrs v, KryCoef c, int k,
                                                       size_t cells, float* __restrict__ out) {
  kry_orth_body(w, v, c, k, cells, out, blockIdx.x, gridDim.x);
}

__global__ void __launch_bounds__(256) kry_update_kernel(double* __restrict__ theta, KryPtrs z, KryCoef y, int m,
                                                         size_t cells, double* tmax) {
  kry_update_body(theta, z, y, m, cells, tmax, blockIdx.x, gridDim.x);
}

// Red half of a sweep from e = 0: with e = 0 the source dSigma(e) and the face sum vanish, so
// e_red = -h^2 (rhs_red - C) / 6; also zeroes the black half of e_zero (the black snapshot of the
// black half-sweep that follows) unless that pointer is null (a black half-sweep that does not
// read the snapshot), and reduces sum rhs_red (the red sum of the sweep) into *sum_out.
__global__ void __launch_bounds__(1024) lin_red_zero_kernel(const float* __restrict__ rhs, size_t half, float h2,
    const double* c_sum, double c_scale, float* __restrict__ e_red, float* __restrict__ e_zero_black,
    double* partials, unsigned* counter, double* sum_out) {
  const float C = (float)(c_sum ? (c_sum[0] + c_sum[1]) * c_scale : 0.0);
  const float g = -h2 * (1.0f / 6.0f);
  double acc = 0.0;
  // half is a multiple of 4 (n even): four cells per thread and pass
  const size_t q = half >> 2;
  typedef float v4f __attribute__((ext_vector_type(4)));
  const v4f* __restrict__ r4 = reinterpret_cast<const v4f*>(rhs);
  v4f* __restrict__ e4 = reinterpret_cast<v4f*>(e_red);
  v4f* __restrict__ z4 = reinterpret_cast<v4f*>(e_zero_black);
  for (size_t x = blockIdx.x * (size_t)blockDim.x + threadIdx.x; x < q; x += (size_t)gridDim.x * blockDim.x) {
    const v4f r = __builtin_nontemporal_load(r4 + x);
    v4f o;
    o.x = g * (r.x - C);
    o.y = g * (r.y - C);
    o.z = g * (r.z - C);
    o.w = g * (r.w - C);
    e4[x] = o;
    if (z4) __builtin_nontemporal_store((v4f){0.0f, 0.0f, 0.0f, 0.0f}, z4 + x);
    acc += ((double)r.x + (double)r.y) + ((double)r.z + (double)r.w);
  }
  double v[1] = {acc};
  grid_sum<1>(v, partials, counter, sum_out, gridDim.x, blockIdx.x);
}

__global__ void zero_scalars_kernel(double* p, int count) {
  if ((int)threadIdx.x < count) p[threadIdx.x] = 0.0;
}

// Compiled tile shapes of the one-launch FP32 sweep.
#define MR_LF_TILES(X) X(32, 16) X(64, 8) X(64, 16) X(16, 16) X(32, 8) X(16, 8) X(8, 8) X(4, 8)

template <int TM, int TJ>
__global__ void __launch_bounds__(TM * TJ) lin_fused_kernel(LinFusedArgs a) {
  __shared__ float lds[LinFusedTile<TM, TJ>::LDS];
  lin_fused_body<TM, TJ>(a, xcd_remap(blockIdx.x, gridDim.x), blockIdx.x, gridDim.x, lds);
}

template <int TM, int TJ>
__global__ void __launch_bounds__(TM * TJ / 2) lin_resid_restrict_tiled(LinRRArgs a) {
  __shared__ float lds[4 * 4 * (TJ + 2) * (TM + 2)];
  lin_resid_restrict_tiled_body<TM, TJ>(a, xcd_remap(blockIdx.x, gridDim.x), blockIdx.x, gridDim.x, lds);
}

template <int TM, int TJ>
__global__ void __launch_bounds__(TM * TJ) mixed_resid64_tiled(ResidTiledArgs a) {
  __shared__ double lds[2 * 4 * (TJ + 2) * (TM + 2)];
  mixed_resid64_tiled_body<TM, TJ>(a, xcd_remap(blockIdx.x, gridDim.x), blockIdx.x, gridDim.x, lds);
}

#define MR_RR_TILES(X) X(64, 8) X(32, 8) X(16, 8) X(8, 8) X(4, 8)

static const void* rr_tiled_kernel(int tm, int tj) {
#define MR_RR_PTR(TM, TJ) \
  if (tm == TM && tj == TJ) return reinterpret_cast<const void*>(&lin_resid_restrict_tiled<TM, TJ>);
  MR_RR_TILES(MR_RR_PTR)
#undef MR_RR_PTR
  return nullptr;
}

#define MR_RT_TILES(X) X(64, 8) X(32, 8) X(16, 8) X(8, 8) X(4, 8)

static const void* resid_tiled_kernel(int tm, int tj) {
#define MR_RT_PTR(TM, TJ) \
  if (tm == TM && tj == TJ) return reinterpret_cast<const void*>(&mixed_resid64_tiled<TM, TJ>);
  MR_RT_TILES(MR_RT_PTR)
#undef MR_RT_PTR
  return nullptr;
}

// Tile and chunking of a 2.5D kernel for an n^3 mesh: the largest tile (tm x tj of (m, j),
// threads = tm * tj / per) that divides the mesh, the plane axis split in units of 4 planes so
// that the grid fills whole waves of the device's resident block slots as well as possible.
// Returns false when no tile applies.
static const int kPref8[][2] = {{64, 8}, {32, 8}, {16, 8}, {8, 8}, {4, 8}};

template <typename Get, size_t NP>
static bool tiled_cfg(int n, Get get, int per, int& tm, int& tj, int& nchunks, const int (&pref)[NP][2]) {
  if (n % 8 != 0) return false;
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
    return false;
  for (const auto& t : pref) {
    if ((n / 2) % t[0] != 0 || n % t[1] != 0) continue;
    int bpc = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&bpc, get(t[0], t[1]), t[0] * t[1] / per, 0) != hipSuccess ||
        bpc < 1)
      continue;
    const long tiles = (long)(n / t[1]) * (n / 2 / t[0]);
    const long cap = (long)cus * bpc;
    double best = -1.0;
    int bc = 1;
    for (int c = 1; c <= n / 4; ++c) {
      const long blocks = tiles * c;
      if (blocks > kMaxReduceBlocks) break;
      const long rounds = (blocks + cap - 1) / cap;
      const double fill = (double)blocks / (double)(rounds * cap);
      const double ci = (double)n / c;
      const double eff = fill * ci / (ci + 3.0);
      if (eff > best + 1e-9) {
        best = eff;
        bc = c;
      }
    }
    tm = t[0];
    tj = t[1];
    nchunks = bc;
    return true;
  }
  return false;
}

static bool resid_tiled_cfg(int n, int& tm, int& tj, int& nchunks) {
  return tiled_cfg(n, resid_tiled_kernel, 1, tm, tj, nchunks, kPref8);
}

// Inner shift of level 0 from the outer residual sums: (sum of rhs, 0) = (-sum b, 0).
__global__ void inner_shift_kernel(const double* __restrict__ res, double* __restrict__ lsum0) {
  if (threadIdx.x == 0) {
    lsum0[0] = -res[2];
    lsum0[1] = 0.0;
  }
}

// FP64 colour-split field -> FP32 copy (same layout).
__global__ void __launch_bounds__(256) cast32_kernel(const double* __restrict__ src, float* __restrict__ dst, size_t cells) {
  for (size_t x = blockIdx.x * (size_t)blockDim.x + threadIdx.x; x < cells; x += (size_t)gridDim.x * blockDim.x)
    dst[x] = (float)src[x];
}

// Defect of the linear level equation at every cell, in FP64 for the caller (the arithmetic is the
// FP32 operator of the inner solve): r = rhs + dSigma(e) - nabla^2 e - cshift. Rows of the mesh
// dealt to blocks; result[0] = sum r.
__global__ void __launch_bounds__(256) lin_residual_kernel(const float* __restrict__ e, const int* __restrict__ baseq,
    const double* __restrict__ bq, const float* __restrict__ sb, const float* __restrict__ rhs, int n, float ih2,
    float cshift, double* __restrict__ r_out) {
  const float* __restrict__ base = reinterpret_cast<const float*>(baseq);
  const float bscl = (float)bq[0];
  for (int row = blockIdx.x; row < n * n; row += gridDim.x) {
    const int i = row / n, j = row - i * n;
    for (int k = threadIdx.x; k < n; k += blockDim.x) {
      const unsigned g = split_idx(n, i, j, k);
      Nb18f te, tb;
      gather18_split_t(e, n, i, j, k, te);
      gather18_split_t(base, n, i, j, k, tb);
      float Se;
      const float src = lin_source(tb, base[g], bscl, sb[g], ih2, te, Se) * ih2;
      const float lap = (Se - 6.0f * e[g]) * ih2;
      r_out[g] = (double)((rhs ? rhs[g] : 0.0f) + src - lap - cshift);
    }
  }
}

// FP32 colour-split field -> FP64 copy (same layout).
__global__ void __launch_bounds__(256) widen64_kernel(const float* __restrict__ src, double* __restrict__ dst, size_t cells) {
  for (size_t x = blockIdx.x * (size_t)blockDim.x + threadIdx.x; x < cells; x += (size_t)gridDim.x * blockDim.x)
    dst[x] = (double)src[x];
}

// Level-0 shift of the inner solve from a sum of the right-hand side: (sum rhs, 0).
__global__ void set_shift_kernel(const double* __restrict__ sum, double* __restrict__ lsum0) {
  if (threadIdx.x == 0) {
    lsum0[0] = sum[0];
    lsum0[1] = 0.0;
  }
}

// ---- launchers ----------------------------------------------------------------------------

static int lin_blocks(size_t cells) {
  size_t b = (cells + 255) / 256;
  return (int)(b < 1 ? 1 : (b > 4096 ? 4096 : b));
}
static int rows_blocks(int n) { return n * n < 4096 ? n * n : 4096; }
static int row_threads(int n) { return n < 64 ? 64 : (n < 256 ? n : 256); }


bool lin_tile_supported(int tm, int tj) {
#define MR_LIN_MATCH(TM, TJ) if (tm == TM && tj == TJ) return true;
  MR_LIN_TILES(MR_LIN_MATCH)
#undef MR_LIN_MATCH
  return false;
}

hipError_t launch_lin_half_sweep(const LinSweepArgs& a, const TileCfg& t, hipStream_t s) {
  const long blocks_l = (long)t.tiles_j * t.tiles_m * (a.n / std::max(t.ci, 1));
  if (blocks_l < 1 || blocks_l > kMaxReduceBlocks || t.tj * t.tiles_j != a.n || t.tm * t.tiles_m != a.n / 2 ||
      t.ci < 1 || a.n % t.ci != 0)
    return hipErrorInvalidValue;
  LinSweepArgs b = a;
  b.tiles_j = t.tiles_j;
  b.tiles_m = t.tiles_m;
  b.ci = t.ci;
  const int blocks = (int)blocks_l;
  if (t.pipe) {
    if (b.ci % 4 != 0 || (a.colour == 1 && !a.e_red_new)) return hipErrorInvalidValue;
#define MR_LP_LAUNCH(TM, TJ)                                                                          \
    if (t.tm == TM && t.tj == TJ) {                                                                   \
      if (a.colour == 0)                                                                              \
        hipLaunchKernelGGL((lin_sweep_pipe<TM, TJ, 0>), dim3(blocks), dim3(TM * TJ), 0, s, b);        \
      else if (a.zero_black)                                                                          \
        hipLaunchKernelGGL((lin_sweep_pipe<TM, TJ, 1, true>), dim3(blocks), dim3(TM * TJ), 0, s, b);  \
      else                                                                                            \
        hipLaunchKernelGGL((lin_sweep_pipe<TM, TJ, 1>), dim3(blocks), dim3(TM * TJ), 0, s, b);        \
      return hipGetLastError();                                                                       \
    }
    MR_LIN_TILES(MR_LP_LAUNCH)
#undef MR_LP_LAUNCH
    return hipErrorInvalidValue;
  }
#define MR_LIN_LAUNCH(TM, TJ)                                                                  \
  if (t.tm == TM && t.tj == TJ) {                                                              \
    hipLaunchKernelGGL((lin_half_sweep_tiled<TM, TJ>), dim3(blocks), dim3(TM * TJ), 0, s, b);  \
    return hipGetLastError();                                                                  \
  }
  MR_LIN_TILES(MR_LIN_LAUNCH)
#undef MR_LIN_LAUNCH
  return hipErrorInvalidValue;
}

bool lin_fused_supported(int tm, int tj) {
#define MR_LF_MATCH(TM, TJ) if (tm == TM && tj == TJ) return true;
  MR_LF_TILES(MR_LF_MATCH)
#undef MR_LF_MATCH
  return false;
}

hipError_t launch_lin_fused(const LinFusedArgs& a, const LinFusedCfg& t, hipStream_t s) {
  const long blocks = (long)(a.n / t.tj) * (a.n / 2 / t.tm) * t.nchunks;
  if (t.tm < 1 || t.tj < 1 || a.n % t.tj != 0 || (a.n / 2) % t.tm != 0 || t.nchunks < 1 || a.n % t.nchunks != 0 ||
      a.n / t.nchunks < 2 || blocks > kMaxReduceBlocks || a.e_in == a.e_out)
    return hipErrorInvalidValue;
  LinFusedArgs b = a;
  b.tiles_j = a.n / t.tj;
  b.tiles_m = a.n / 2 / t.tm;
  b.nchunks = t.nchunks;
#define MR_LF_LAUNCH(TM, TJ)                                                                           \
  if (t.tm == TM && t.tj == TJ) {                                                                      \
    hipLaunchKernelGGL((lin_fused_kernel<TM, TJ>), dim3((unsigned)blocks), dim3(TM * TJ), 0, s, b);    \
    return hipGetLastError();                                                                          \
  }
  MR_LF_TILES(MR_LF_LAUNCH)
#undef MR_LF_LAUNCH
  return hipErrorInvalidValue;
}

// w = J z on an n^3 mesh (both colours) and the sums w v_j (j < k), w, w^2 into result[0 .. k + 1]:
// one pipelined launch with the projections fused where a 64 x 8 tile fits (at most kKryBlocks
// blocks), otherwise the row kernel followed by the dot-product kernel.
hipError_t launch_lin_apply_dots(const float* z, const int* baseq, const double* bq, const float* sb, int n, double h,
                                 float* w, const KryPtrs& v, int k, double* partials, unsigned* counter, double* result,
                                 hipStream_t s) {
  constexpr int TM = 64, TJ = 8;
  if (k < 1 || k > kKryMax) return hipErrorInvalidValue;
  if ((n / 2) % TM == 0 && n % TJ == 0 && n % 4 == 0) {
    const int tiles = (n / TJ) * (n / 2 / TM);
    // up to one block per CU: more blocks cost more in the per-block release of the reduction
    // than they gain in occupancy (the blocks have 16 waves each)
    int nch = 1;
    while (tiles * nch * 2 <= kApplyBlocks && (n / (nch * 2)) % 4 == 0 && n / (nch * 2) >= 16) nch *= 2;
    if (tiles * nch <= kKryBlocks && (n / nch) % 4 == 0) {
      LinApplyArgs a{};
      a.z = z;
      a.base = baseq;
      a.bq = bq;
      a.sb = sb;
      a.w = w;
      a.n = n;
      a.ih2 = (float)(1.0 / (h * h));
      a.tiles_j = n / TJ;
      a.tiles_m = n / 2 / TM;
      a.ci = n / nch;
      a.v = v;
      a.partials = partials;
      a.counter = counter;
      a.result = result;
      const unsigned blocks = (unsigned)(tiles * nch);
      switch (k) {
#define MR_AD_CASE(KK)                                                                                          \
        case KK:                                                                                                \
          hipLaunchKernelGGL((lin_apply_dots<TM, TJ, KK>), dim3(blocks), dim3(2 * TM * TJ), 0, s, a);          \
          break;
        MR_AD_CASE(1) MR_AD_CASE(2) MR_AD_CASE(3) MR_AD_CASE(4) MR_AD_CASE(5) MR_AD_CASE(6) MR_AD_CASE(7)
        MR_AD_CASE(8)
#undef MR_AD_CASE
      }
      return hipGetLastError();
    }
  }
  hipLaunchKernelGGL(lin_apply_row_kernel, dim3(rows_blocks(n)), dim3(row_threads(n)), 0, s, z, baseq, bq, sb, n,
                     (float)(1.0 / (h * h)), w);
  const size_t cells = (size_t)n * n * n;
  const int nb = (int)std::min<size_t>((cells / 4 + 255) / 256, (size_t)kKryBlocks);
  switch (k) {
#define MR_KD_CASE(KK)                                                                                            \
    case KK:                                                                                                      \
      hipLaunchKernelGGL((kry_dots_kernel<KK>), dim3(nb), dim3(256), 0, s, (const float*)w, v, cells, partials, counter, \
                         result);                                                                                 \
      break;
    MR_KD_CASE(1) MR_KD_CASE(2) MR_KD_CASE(3) MR_KD_CASE(4) MR_KD_CASE(5) MR_KD_CASE(6) MR_KD_CASE(7) MR_KD_CASE(8)
#undef MR_KD_CASE
  }
  return hipGetLastError();
}

hipError_t launch_mixed_resid64(const double* theta, const double* delta, int n, ShiftRef C, float* rhs32, int* baseq,
                                const double* bq, float* sb32, Reduce red, hipStream_t s) {
  int tm = 0, tj = 0, nch = 0;
  if (resid_tiled_cfg(n, tm, tj, nch)) {
    ResidTiledArgs a{theta, delta, n, C, rhs32, baseq, bq, sb32, red, n / tj, n / 2 / tm, nch};
    const unsigned blocks = (unsigned)(a.tiles_j * a.tiles_m * nch);
#define MR_RT_LAUNCH(TM, TJ)                                                                   \
    if (tm == TM && tj == TJ) {                                                                \
      hipLaunchKernelGGL((mixed_resid64_tiled<TM, TJ>), dim3(blocks), dim3(TM * TJ), 0, s, a); \
      return hipGetLastError();                                                                \
    }
    MR_RT_TILES(MR_RT_LAUNCH)
#undef MR_RT_LAUNCH
  }
  hipLaunchKernelGGL(mixed_resid64_kernel, dim3(rows_blocks(n)), dim3(row_threads(n)), 0, s, theta, delta, n, C, rhs32,
                     baseq, bq, sb32, red);
  return hipGetLastError();
}

hipError_t launch_base_root(const int* baseq, const double* bq, const double* delta, int n, double h, float* sb32,
                            hipStream_t s) {
  hipLaunchKernelGGL(base_root_kernel, dim3((unsigned)n * n), dim3(n < 256 ? n : 256), 0, s, baseq, bq, delta, n,
                     1.0 / (h * h), sb32);
  return hipGetLastError();
}

hipError_t launch_restrictq(const int* fine, int* coarse, int n, hipStream_t s) {
  const int m = n / 2;
  hipLaunchKernelGGL(restrictq_kernel, dim3((unsigned)m * m), dim3(m), 0, s, fine, coarse, n);
  return hipGetLastError();
}

hipError_t launch_absmax(const double* a, size_t cells, double* tmax, hipStream_t s) {
  hipLaunchKernelGGL(absmax_kernel, dim3(lin_blocks(cells)), dim3(256), 0, s, a, cells, tmax);
  return hipGetLastError();
}

hipError_t launch_base_scale(double* tmax, double* bq, hipStream_t s) {
  hipLaunchKernelGGL(base_scale_kernel, dim3(1), dim3(64), 0, s, tmax, bq);
  return hipGetLastError();
}

hipError_t launch_quantise(const double* src, int* dst, size_t cells, const double* bq, hipStream_t s) {
  hipLaunchKernelGGL(quantise_kernel, dim3(lin_blocks(cells)), dim3(256), 0, s, src, dst, cells, bq);
  return hipGetLastError();
}

// With tm0 > 0 the tile (tm0, tj0) and nch0 chunks (a timed choice); otherwise the largest tile that
// fits with chunks from the occupancy model.
static hipError_t launch_lin_rr(const float* e, const int* baseq, const double* bq, const float* sb, const float* rhs,
                                int n, double h, ShiftRef c, float* rhs_c, Reduce red, hipStream_t s, int tm0, int tj0,
                                int nch0) {
  int tm = 0, tj = 0, nch = 0;
  bool tiled = false;
  if (tm0 > 0) {
    tm = tm0;
    tj = tj0;
    nch = nch0;
    tiled = (n / 2) % tm == 0 && n % tj == 0 && nch >= 1 && nch <= n / 4;
  } else {
    tiled = tiled_cfg(n, rr_tiled_kernel, 2, tm, tj, nch, kPref8);
  }
  if (tiled) {
    LinRRArgs a{e, baseq, bq, sb, rhs, n, (float)(1.0 / (h * h)), c, rhs_c, red, n / tj, n / 2 / tm, nch};
    const unsigned blocks = (unsigned)(a.tiles_j * a.tiles_m * nch);
#define MR_RR_LAUNCH(TM, TJ)                                                                           \
    if (tm == TM && tj == TJ) {                                                                        \
      hipLaunchKernelGGL((lin_resid_restrict_tiled<TM, TJ>), dim3(blocks), dim3(TM * TJ / 2), 0, s, a); \
      return hipGetLastError();                                                                        \
    }
    MR_RR_TILES(MR_RR_LAUNCH)
#undef MR_RR_LAUNCH
  }
  const int m = n / 2;
  hipLaunchKernelGGL(lin_resid_restrict_kernel, dim3(rows_blocks(m)), dim3(row_threads(m)), 0, s, e, baseq, bq, sb, rhs,
                     n, (float)(1.0 / (h * h)), c, rhs_c, red);
  return hipGetLastError();
}

hipError_t launch_lin_resid_restrict(const float* e, const int* baseq, const double* bq, const float* sb, const float* rhs,
                                     int n, double h, ShiftRef c, float* rhs_c, Reduce red, hipStream_t s) {
  return launch_lin_rr(e, baseq, bq, sb, rhs, n, h, c, rhs_c, red, s, 0, 0, 0);
}

__global__ void __launch_bounds__(256) prolong_rows32_kernel(const float* __restrict__ ec, float* __restrict__ e, int n) {
  __shared__ float cl[kProlongRowsLds];
  prolong_rows32_body(ec, e, n, xcd_remap(blockIdx.x, gridDim.x), cl);
}

__global__ void __launch_bounds__(1024) prolong_pipe32_kernel(const float* __restrict__ ec, float* __restrict__ e, int n,
                                                               int nchunks) {
  __shared__ float cl[kProlongPipeLds];
  prolong_pipe32_body(ec, e, n, xcd_remap(blockIdx.x, gridDim.x), nchunks, cl);
}

hipError_t launch_prolong_add32(const float* ec, float* e, int n, hipStream_t s) {
  const long cc = (long)(n / 2) * (n / 2) * (n / 2);   // one thread per coarse cell
  if (prolong_pipe_ok(n)) {   // 1024-thread blocks of 1024 / nc coarse rows, about 512 blocks
    const int nc = n / 2, tiles = nc * nc / 1024;
    const int nchunks = std::min(nc / 8, std::max(1, 512 / tiles));
    hipLaunchKernelGGL(prolong_pipe32_kernel, dim3((unsigned)(tiles * nchunks)), dim3(1024), 0, s, ec, e, n, nchunks);
    return hipGetLastError();
  }
  if (prolong_rows_ok(n)) {   // cc / 256 whole row groups
    hipLaunchKernelGGL(prolong_rows32_kernel, dim3((unsigned)(cc / 256)), dim3(256), 0, s, ec, e, n);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(prolong_add32_kernel, dim3((unsigned)((cc + 255) / 256)), dim3(256), 0, s, ec, e, n);
  return hipGetLastError();
}

hipError_t launch_lin_coarsest(float* e, const int* baseq, const double* bq, const float* sb, const float* rhs, int n,
                               int nsweeps, double h, const double* c_sum, double c_scale, hipStream_t s) {
  if ((long)n * n * n > kMaxCoarsest) return hipErrorInvalidValue;
  hipLaunchKernelGGL(lin_coarsest_kernel, dim3(1), dim3(256), 0, s, e, baseq, bq, sb, rhs, n, nsweeps, (float)(h * h),
                     (float)(1.0 / (h * h)), c_sum, c_scale);
  return hipGetLastError();
}

hipError_t launch_update64(double* theta, const float* e, size_t cells, double* tmax, hipStream_t s) {
  hipLaunchKernelGGL(update64_kernel, dim3(lin_blocks(cells)), dim3(256), 0, s, theta, e, cells, tmax);
  return hipGetLastError();
}

hipError_t launch_fill32(float* a, float v, size_t cells, hipStream_t s) {
  hipLaunchKernelGGL(fill32_kernel, dim3(lin_blocks(cells)), dim3(256), 0, s, a, v, cells);
  return hipGetLastError();
}

hipError_t launch_cast32(const double* src, float* dst, size_t cells, hipStream_t s) {
  hipLaunchKernelGGL(cast32_kernel, dim3(lin_blocks(cells)), dim3(256), 0, s, src, dst, cells);
  return hipGetLastError();
}

hipError_t launch_widen64(const float* src, double* dst, size_t cells, hipStream_t s) {
  hipLaunchKernelGGL(widen64_kernel, dim3(lin_blocks(cells)), dim3(256), 0, s, src, dst, cells);
  return hipGetLastError();
}

hipError_t launch_lin_residual(const float* e, const int* baseq, const double* bq, const float* sb, const float* rhs,
                               int n, double h, double cshift, double* r_out, hipStream_t s) {
  hipLaunchKernelGGL(lin_residual_kernel, dim3(rows_blocks(n)), dim3(row_threads(n)), 0, s, e, baseq, bq, sb, rhs, n,
                     (float)(1.0 / (h * h)), (float)cshift, r_out);
  return hipGetLastError();
}

// ---- driver -------------------------------------------------------------------------------

// FP32 buffers of one level of the inner linear multigrid (colour-split).
struct LinLevel {
  float* e[2] = {nullptr, nullptr};
  int cur = 0;
  float* rhs = nullptr;
  int* base = nullptr;   // fixed-point base potential (scale in the context's kSlotBase scalars)
  float* sb = nullptr;
  TileCfg sw;            // two-launch schedule
  bool fused = false;    // the one-launch sweep (schedule fz) won the tuner
  LinFusedCfg fz;
  int rr_tm = 0, rr_tj = 0, rr_nch = 0;   // timed defect + restriction tile (rr_tm == 0: default)
};

// Krylov space of the inner solve on the finest mesh: V[0..m] orthonormal mean-free vectors,
// Z[0..m-1] their preconditioned images, W the operator's product, S a spare e buffer, and the
// reduction buffers of the dot products.
struct KryState {
  int m = 0;
  std::vector<float*> V, Z;
  float *W = nullptr, *S = nullptr;
  double *partials = nullptr, *result = nullptr;
  unsigned* counter = nullptr;
};

// The coarse part of an inner V-cycle (levels 1 .. coarsest, from zero), captured once in a HIP graph
// and replayed: its launches are short and latency-bound, and between V-cycles only buffer contents
// change. cur_in / cur_out: the ping-pong state of the coarse levels before and after one cycle.
struct CoarseGraph {
  hipStream_t cs = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<int> cur_in, cur_out;
  int npre = -1, npost = -1, ncoarse = -1;
};

struct MixedState {
  std::vector<LinLevel> lv;
  std::vector<void*> owned;
  KryState kry;
  std::vector<void*> kry_owned;
  CoarseGraph cg;
};

static TileCfg lin_tiles(int n) {
  TileCfg t;
  const int nh = n / 2;
  int tm = 64;
  while (tm > 2 && (nh % tm != 0 || tm > nh)) tm /= 2;
  static const int pref[][2] = {{64, 4}, {32, 8}, {16, 16}, {8, 16}, {4, 8}, {2, 4}};
  t.tm = 0;
  for (const auto& p : pref)
    if (p[0] == tm && n % p[1] == 0 && p[1] <= n) {
      t.tm = p[0];
      t.tj = p[1];
      break;
    }
  if (t.tm == 0) return t;
  t.tiles_j = n / t.tj;
  t.tiles_m = nh / t.tm;
  const long tiles = (long)t.tiles_j * t.tiles_m;
  t.ci = n;
  while (t.ci % 2 == 0 && t.ci / 2 >= 8 && tiles * (n / t.ci) < 1024) t.ci /= 2;
  while (tiles * (n / t.ci) > kMaxReduceBlocks && t.ci * 2 <= n && n % (t.ci * 2) == 0) t.ci *= 2;
  t.pipe = t.ci % 4 == 0;
  return t;
}

struct LinSched {
  TileCfg two;
  bool fused = false;
  LinFusedCfg fz;
};
static std::mutex g_lin_tune_mu;
static std::map<std::pair<int, int>, LinSched> g_lin_tuned;   // (device, n)

// Times both colours of a linear sweep for the default tile and for the pipelined kernel on every
// compiled tile with chunks of 16 to 256 planes, on the level's (zeroed) buffers, and keeps the
// fastest. Cached per (device, n).
static int tune_lin_sweep(Ctx* c, int l, LinSched* out) {
  const int n = c->lv[l].n, nh = n / 2;
  LinLevel& L = c->mixed->lv[l];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return hip_fail(hipErrorInvalidDevice, "linear sweep tuner");
  {
    std::lock_guard<std::mutex> lk(g_lin_tune_mu);
    static int gen = -1;
    tuning_sync(gen, g_lin_tuned);
    auto it = g_lin_tuned.find({dev, n});
    if (it != g_lin_tuned.end()) {
      *out = it->second;
      return MR_OK;
    }
  }
  std::vector<TileCfg> cand{lin_tiles(n)};
  auto add = [&](int tm, int tj) {
    if (nh % tm != 0 || n % tj != 0 || tj > n || tm > nh) return;
    for (int ci = 16; ci <= 256 && ci <= n; ci *= 2) {
      TileCfg t;
      t.tm = tm;
      t.tj = tj;
      t.cpt = 1;
      t.ci = ci;
      t.tiles_j = n / tj;
      t.tiles_m = nh / tm;
      t.pipe = true;
      if (n % ci == 0 && (long)t.tiles_j * t.tiles_m * (n / ci) <= kMaxReduceBlocks) cand.push_back(t);
    }
  };
#define MR_LIN_ADD(TM, TJ) add(TM, TJ);
  MR_LIN_TILES(MR_LIN_ADD)
#undef MR_LIN_ADD
  const size_t cells = c->lv[l].cells;
  hipError_t e = hipSuccess;
  for (void* b : {(void*)L.e[0], (void*)L.e[1], (void*)L.base, (void*)L.sb, (void*)L.rhs})
    if (e == hipSuccess) e = hipMemsetAsync(b, 0, cells * sizeof(float), c->stream);
  LinSweepArgs a{};
  a.e_in = L.e[0];
  a.e_out = L.e[1];
  a.base = L.base;
  a.bq = c->scal + kSlotBase;
  a.sb = L.sb;
  a.rhs = L.rhs;
  a.n = n;
  a.h2 = 1.0f;
  a.ih2 = 1.0f;
  a.partials = c->partials;
  a.counter = c->counter;
  a.sum_out = c->scal + kSlotAux;
  auto run = [&](const TileCfg& t) {
    LinSweepArgs r = a;
    r.colour = 0;
    hipError_t x = launch_lin_half_sweep(r, t, c->stream);
    r.colour = 1;
    r.e_red_new = L.e[1];
    return x == hipSuccess ? launch_lin_half_sweep(r, t, c->stream) : x;
  };
  const int reps = cells >= ((size_t)1 << 24) ? 2 : 4;
  // the default tile can be unsupported on tiny meshes (tm == 0): it is then never picked
  std::vector<LinSched> ok;
  for (const TileCfg& t : cand)
    if (t.tm != 0) ok.push_back(LinSched{t, false, LinFusedCfg{}});
  // one-launch candidates: every compiled tile that fits, chunks of 16 to 256 planes
  auto add_fused = [&](int tm, int tj) {
    if (nh % tm != 0 || n % tj != 0 || tj > n || tm > nh) return;
    for (int ci = 16; ci <= 256 && ci <= n; ci *= 2) {
      const long blocks = (long)(n / tj) * (nh / tm) * (n / ci);
      if (n % ci == 0 && blocks <= kMaxReduceBlocks) ok.push_back(LinSched{cand[0], true, LinFusedCfg{tm, tj, n / ci}});
    }
  };
#define MR_LF_ADD(TM, TJ) add_fused(TM, TJ);
  MR_LF_TILES(MR_LF_ADD)
#undef MR_LF_ADD
  LinFusedArgs fa{};
  fa.e_in = L.e[0];
  fa.e_out = L.e[1];
  fa.base = L.base;
  fa.bq = c->scal + kSlotBase;
  fa.sb = L.sb;
  fa.rhs = L.rhs;
  fa.n = n;
  fa.h2 = 1.0f;
  fa.ih2 = 1.0f;
  fa.sum_out = c->scal + kSlotAux;
  fa.partials = c->partials;
  fa.counter = c->counter;
  auto run_any = [&](size_t i) {
    return ok[i].fused ? launch_lin_fused(fa, ok[i].fz, c->stream) : run(ok[i].two);
  };
  auto code = [](const LinSched& t) {
    std::vector<int> v{t.fused ? 1 : 0};
    for (int x : tile_code(t.two)) v.push_back(x);
    for (int x : {t.fz.tm, t.fz.tj, t.fz.nchunks}) v.push_back(x);
    return v;
  };
  size_t bi = 0;
  bool recorded = false;
  {
    std::vector<int> rec;
    if (tuning_lookup("lin32.v1", dev, n, rec))
      for (size_t i = 0; i < ok.size() && !recorded; ++i)
        if (code(ok[i]) == rec) {
          bi = i;
          recorded = true;
        }
  }
  if (e == hipSuccess && !ok.empty() && !recorded) e = pick_fastest(ok.size(), reps, c->stream, run_any, &bi);
  LinSched best_t;
  if (!ok.empty()) best_t = ok[bi];
  else best_t.two = cand[0];
  if (e != hipSuccess) return hip_fail(e, "linear sweep tuner");
  {
    std::lock_guard<std::mutex> lk(g_lin_tune_mu);
    g_lin_tuned[{dev, n}] = best_t;
  }
  if (!ok.empty() && !recorded) tuning_record("lin32.v1", dev, n, code(best_t));
  *out = best_t;
  return MR_OK;
}

static std::mutex g_rr_tune_mu;
static std::map<std::pair<int, int>, std::vector<int>> g_rr_tuned;   // (device, n) -> (tm, tj, nchunks)

// Times the FP32 defect + restriction of level l (< coarsest) on every compiled tile with 1 to n/4
// chunks (powers of two) and the occupancy-model default, on the level's zeroed buffers (the kernel
// only reads them and writes the coarse right-hand side); keeps and records the fastest.
static int tune_lin_rr(Ctx* c, int l, int* tm, int* tj, int* nch) {
  const int n = c->lv[l].n, nh = n / 2;
  *tm = *tj = *nch = 0;
  if (n % 8 != 0) return MR_OK;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return hip_fail(hipErrorInvalidDevice, "defect tuner");
  {
    std::lock_guard<std::mutex> lk(g_rr_tune_mu);
    static int gen = -1;
    tuning_sync(gen, g_rr_tuned);
    auto it = g_rr_tuned.find({dev, n});
    if (it != g_rr_tuned.end()) {
      *tm = it->second[0];
      *tj = it->second[1];
      *nch = it->second[2];
      return MR_OK;
    }
  }
  std::vector<std::vector<int>> cand{{0, 0, 0}};
  auto add = [&](int TM, int TJ) {
    if (nh % TM != 0 || n % TJ != 0) return;
    for (int k = 1; k <= n / 4; k *= 2)
      if ((long)(n / TJ) * (nh / TM) * k <= kMaxReduceBlocks) cand.push_back({TM, TJ, k});
  };
#define MR_RR_ADD(TM, TJ) add(TM, TJ);
  MR_RR_TILES(MR_RR_ADD)
#undef MR_RR_ADD
  size_t bi = 0;
  bool recorded = false;
  {
    std::vector<int> rec;
    if (tuning_lookup("linrr32.v1", dev, n, rec))
      for (size_t i = 0; i < cand.size() && !recorded; ++i)
        if (cand[i] == rec) {
          bi = i;
          recorded = true;
        }
  }
  LinLevel& L = c->mixed->lv[l];
  LinLevel& Lc = c->mixed->lv[l + 1];
  const Level& F = c->lv[l];
  const int reps = F.cells >= ((size_t)1 << 24) ? 2 : 4;
  hipError_t e = hipSuccess;
  if (!recorded)
    e = pick_fastest(cand.size(), reps, c->stream, [&](size_t i) {
      return launch_lin_rr(L.e[0], L.base, c->scal + kSlotBase, L.sb, L.rhs, F.n, F.h, ShiftRef{nullptr, 0.0, 0.0}, Lc.rhs,
                           c->reducer(kSlotAux), c->stream, cand[i][0], cand[i][1], cand[i][2]);
    }, &bi);
  if (e != hipSuccess) return hip_fail(e, "defect tuner");
  {
    std::lock_guard<std::mutex> lk(g_rr_tune_mu);
    g_rr_tuned[{dev, n}] = cand[bi];
  }
  if (!recorded) tuning_record("linrr32.v1", dev, n, cand[bi]);
  *tm = cand[bi][0];
  *tj = cand[bi][1];
  *nch = cand[bi][2];
  return MR_OK;
}

static int mixed_alloc(Ctx* c) {
  if (c->mixed) return MR_OK;
  MixedState* m = new MixedState();
  c->mixed = m;
  m->lv.resize(c->nlev);
  for (int l = 0; l < c->nlev; ++l) {
    const size_t cells = c->lv[l].cells;
    LinLevel& L = m->lv[l];
    void** bufs[] = {(void**)&L.e[0], (void**)&L.e[1], (void**)&L.rhs, (void**)&L.base, (void**)&L.sb};
    for (void** b : bufs) {
      hipError_t e = hipMalloc(b, cells * sizeof(float));
      if (e != hipSuccess) return fail(MR_ENOMEM, "mixed precision buffers: %s", hipGetErrorString(e));
      m->owned.push_back(*b);
    }
  }
  // linear sweep schedule per level, timed on the level's buffers
  for (int l = 0; l + 1 < c->nlev; ++l) {
    LinSched ls;
    int rc = tune_lin_sweep(c, l, &ls);
    if (rc != MR_OK) return rc;
    m->lv[l].sw = ls.two;
    m->lv[l].fused = ls.fused;
    m->lv[l].fz = ls.fz;
    if ((rc = tune_lin_rr(c, l, &m->lv[l].rr_tm, &m->lv[l].rr_tj, &m->lv[l].rr_nch)) != MR_OK) return rc;
  }
  return MR_OK;
}

void Ctx::release_extra() {
  if (dep_mem) {
    (void)hipFree(dep_mem);
    dep_mem = nullptr;
    dep_bytes = 0;
  }
  if (cic_grid) {
    (void)hipFree(cic_grid);
    cic_grid = nullptr;
  }
  if (mixed) {
    for (void* p : mixed->owned) (void)hipFree(p);
    for (void* p : mixed->kry_owned) (void)hipFree(p);
    CoarseGraph& g = mixed->cg;
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
    if (g.graph) (void)hipGraphDestroy(g.graph);
    if (g.cs) (void)hipStreamDestroy(g.cs);
    delete mixed;
    mixed = nullptr;
  }
  release_adjoint();
  aa_release();
}

double* Ctx::linsum(int l) { return scal + kSlotLin + 3 * l; }

int Ctx::lin_sweep(int l, bool zero_start) {
  LinLevel& L = mixed->lv[l];
  Level& F = lv[l];
  double* cs = linsum(l);
  if (zero_start && L.sw.tm == 0) {   // no two-launch tile on this mesh: clear e and sweep as usual
    hipError_t e = launch_fill32(L.e[L.cur], 0.0f, F.cells, stream);
    if (e != hipSuccess) return hip_fail(e, "fill");
    zero_start = false;
  }
  if (zero_start) {
    // e = 0 on entry: the red half needs no neighbours; the black half-sweep then runs as usual on
    // the new red values and a zero black snapshot
    const size_t half = F.cells / 2;
    const int ev = (l == 0) ? timer.begin(stream) : -1;
    // few large blocks: each block's counter release costs an L2 writeback, so the grid stays at
    // one block per CU (16 waves each) however large the level
    const int nbz = (int)std::min<size_t>(256, (half / 4 + 1023) / 1024);
    // the pipelined black half-sweep takes the zero black snapshot as given; the others read it
    const bool zb = L.sw.pipe;
    hipLaunchKernelGGL(lin_red_zero_kernel, dim3(nbz), dim3(1024), 0, stream, (const float*)L.rhs, half,
                       (float)(F.h * F.h), (const double*)cs, 1.0 / (double)F.cells, L.e[L.cur ^ 1],
                       zb ? nullptr : L.e[L.cur] + half, partials, counter, cs + 2);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "linear red half-sweep from zero");
    LinSweepArgs a{};
    a.e_in = L.e[L.cur];
    a.e_red_new = L.e[L.cur ^ 1];
    a.e_out = L.e[L.cur ^ 1];
    a.base = L.base;
    a.bq = scal + kSlotBase;
    a.sb = L.sb;
    a.rhs = L.rhs;
    a.n = F.n;
    a.colour = 1;
    a.h2 = (float)(F.h * F.h);
    a.ih2 = (float)(1.0 / (F.h * F.h));
    a.c_sum = cs;
    a.c_scale = 1.0 / (double)F.cells;
    a.sum_out = cs + 1;
    a.copy_from = cs + 2;
    a.copy_to = cs + 0;
    a.partials = partials;
    a.counter = counter;
    a.zero_black = zb ? 1 : 0;
    e = launch_lin_half_sweep(a, L.sw, stream);
    if (e != hipSuccess) return hip_fail(e, "linear black half-sweep");
    timer.end(1, ev, stream);
    L.cur ^= 1;
    return MR_OK;
  }
  if (L.fused && !(opts.flags & MR_FLAG_TWO_PASS)) {
    LinFusedArgs a{};
    a.e_in = L.e[L.cur];
    a.e_out = L.e[L.cur ^ 1];
    a.base = L.base;
    a.bq = scal + kSlotBase;
    a.sb = L.sb;
    a.rhs = L.rhs;
    a.n = F.n;
    a.h2 = (float)(F.h * F.h);
    a.ih2 = (float)(1.0 / (F.h * F.h));
    a.c_sum = cs;
    a.c_scale = 1.0 / (double)F.cells;
    a.sum_out = cs;   // (red sum, black sum): the shift of the next sweep
    a.partials = partials;
    a.counter = counter;
    const int ev = (l == 0) ? timer.begin(stream) : -1;
    hipError_t e = launch_lin_fused(a, L.fz, stream);
    if (e != hipSuccess) return hip_fail(e, "linear fused sweep");
    timer.end(1, ev, stream);
    L.cur ^= 1;
    return MR_OK;
  }
  LinSweepArgs a{};
  a.e_in = L.e[L.cur];
  a.e_red_new = nullptr;
  a.e_out = L.e[L.cur ^ 1];
  a.base = L.base;
  a.bq = scal + kSlotBase;
  a.sb = L.sb;
  a.rhs = L.rhs;
  a.n = F.n;
  a.colour = 0;
  a.h2 = (float)(F.h * F.h);
  a.ih2 = (float)(1.0 / (F.h * F.h));
  a.c_sum = cs;
  a.c_scale = 1.0 / (double)F.cells;
  a.sum_out = cs + 2;
  a.partials = partials;
  a.counter = counter;
  const int ev = (l == 0) ? timer.begin(stream) : -1;
  hipError_t e = launch_lin_half_sweep(a, L.sw, stream);
  if (e != hipSuccess) return hip_fail(e, "linear red half-sweep");
  a.colour = 1;
  a.e_red_new = L.e[L.cur ^ 1];
  a.sum_out = cs + 1;
  a.copy_from = cs + 2;
  a.copy_to = cs + 0;
  e = launch_lin_half_sweep(a, L.sw, stream);
  if (e != hipSuccess) return hip_fail(e, "linear black half-sweep");
  timer.end(1, ev, stream);
  L.cur ^= 1;
  return MR_OK;
}

// Linear V-cycle on level l; zero: e of the level is zero on entry (it is then not read: the first
// pre-smoothing sweep starts from zero, or the coarsest level is cleared first).
int Ctx::lin_vcycle(int l, bool zero) {
  LinLevel& L = mixed->lv[l];
  Level& F = lv[l];
  hipError_t e;
  if (l > 0 && zero && F.n <= kTailMaxN && nlev - l <= kTailMaxLev) {
    // this level and all coarser ones in one workgroup
    LinTailArgs a{};
    a.e_out = L.e[L.cur];
    a.rhs = L.rhs;
    for (int t = 0; t < nlev - l; ++t) {
      a.base[t] = mixed->lv[l + t].base;
      a.sb[t] = mixed->lv[l + t].sb;
    }
    a.bq = scal + kSlotBase;
    a.c_sum = linsum(l);
    a.n0 = F.n;
    a.levels = nlev - l;
    a.npre = opts.npre;
    a.npost = opts.npost;
    a.ncoarse = opts.ncoarse;
    a.h0 = (float)F.h;
    hipLaunchKernelGGL(lin_tail_kernel, dim3(1), dim3(kTailThreads), 0, stream, a);
    e = hipGetLastError();
    return e == hipSuccess ? MR_OK : hip_fail(e, "linear V-cycle tail");
  }
  if (l == nlev - 1) {
    e = zero ? launch_fill32(L.e[L.cur], 0.0f, F.cells, stream) : hipSuccess;
    if (e == hipSuccess)
      e = launch_lin_coarsest(L.e[L.cur], L.base, scal + kSlotBase, L.sb, L.rhs, F.n, opts.ncoarse, F.h, linsum(l),
                              1.0 / (double)F.cells, stream);
    return e == hipSuccess ? MR_OK : hip_fail(e, "linear coarsest");
  }
  int rc;
  if (zero && opts.npre == 0 && (e = launch_fill32(L.e[L.cur], 0.0f, F.cells, stream)) != hipSuccess)
    return hip_fail(e, "fill");
  for (int s = 0; s < opts.npre; ++s)
    if ((rc = lin_sweep(l, zero && s == 0)) != MR_OK) return rc;
  LinLevel& Lc = mixed->lv[l + 1];
  e = launch_lin_rr(L.e[L.cur], L.base, scal + kSlotBase, L.sb, L.rhs, F.n, F.h,
                    ShiftRef{linsum(l), 1.0 / (double)F.cells, 0.0}, Lc.rhs, Reduce{partials, counter, linsum(l + 1)},
                    stream, L.rr_tm, L.rr_tj, L.rr_nch);
  if (e != hipSuccess) return hip_fail(e, "linear restriction");
  if ((rc = (l == 0 ? lin_coarse_cycle() : lin_vcycle(l + 1, true))) != MR_OK) return rc;
  e = launch_prolong_add32(Lc.e[Lc.cur], L.e[L.cur], F.n, stream);
  if (e != hipSuccess) return hip_fail(e, "linear prolongation");
  for (int s = 0; s < opts.npost; ++s)
    if ((rc = lin_sweep(l)) != MR_OK) return rc;
  return MR_OK;
}

// lin_vcycle(1, true) through the captured graph (captured on first use, or again when the cycle
// options change). The coarse levels start from zero, so their buffers' contents on entry do not
// matter: each replay first puts the host-side ping-pong state back to the captured one.
int Ctx::lin_coarse_cycle() {
  CoarseGraph& g = mixed->cg;
  hipError_t e = hipSuccess;
  if (!g.exec || g.npre != opts.npre || g.npost != opts.npost || g.ncoarse != opts.ncoarse) {
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
    if (g.graph) (void)hipGraphDestroy(g.graph);
    g.exec = nullptr;
    g.graph = nullptr;
    if (!g.cs && (e = hipStreamCreateWithFlags(&g.cs, hipStreamNonBlocking)) != hipSuccess) return hip_fail(e, "stream");
    g.cur_in.assign(nlev, 0);
    for (int l = 1; l < nlev; ++l) g.cur_in[l] = mixed->lv[l].cur;
    hipStream_t keep = stream;
    stream = g.cs;
    e = hipStreamBeginCapture(g.cs, hipStreamCaptureModeThreadLocal);
    int rc = e == hipSuccess ? lin_vcycle(1, true) : hip_fail(e, "capture");
    hipError_t e2 = hipStreamEndCapture(g.cs, &g.graph);
    stream = keep;
    if (rc != MR_OK) return rc;
    if (e2 != hipSuccess) return hip_fail(e2, "capture");
    if ((e = hipGraphInstantiate(&g.exec, g.graph, nullptr, nullptr, 0)) != hipSuccess) return hip_fail(e, "graph");
    g.cur_out.assign(nlev, 0);
    for (int l = 1; l < nlev; ++l) g.cur_out[l] = mixed->lv[l].cur;
    g.npre = opts.npre;
    g.npost = opts.npost;
    g.ncoarse = opts.ncoarse;
  }
  for (int l = 1; l < nlev; ++l) mixed->lv[l].cur = g.cur_in[l];
  if ((e = hipGraphLaunch(g.exec, stream)) != hipSuccess) return hip_fail(e, "graph launch");
  for (int l = 1; l < nlev; ++l) mixed->lv[l].cur = g.cur_out[l];
  return MR_OK;
}

int Ctx::lin_schedule(int l, int sched[4]) {
  int rc = mixed_alloc(this);
  if (rc != MR_OK) return rc;
  const LinLevel& L = mixed->lv[l];
  if (L.fused && !(opts.flags & MR_FLAG_TWO_PASS)) {
    sched[0] = MR_SCHED_FUSED;
    sched[1] = L.fz.tm;
    sched[2] = L.fz.tj;
    sched[3] = L.fz.nchunks;
  } else {
    sched[0] = L.sw.pipe ? MR_SCHED_PIPELINED : MR_SCHED_TILED;
    sched[1] = L.sw.tm;
    sched[2] = L.sw.tj;
    sched[3] = L.sw.ci > 0 ? lv[l].n / L.sw.ci : 0;
  }
  return MR_OK;
}

int Ctx::mixed_ready() { return mixed_alloc(this); }

// Base potential and root of every coarse level of the inner linear multigrid from those of the
// finest level: base = R base (8-son mean), root from the coarse base and R delta at the level's h.
int Ctx::lin_base_hierarchy() {
  for (int l = 1; l < nlev; ++l) {
    hipError_t e = launch_restrictq(mixed->lv[l - 1].base, mixed->lv[l].base, lv[l - 1].n, stream);
    if (e == hipSuccess)
      e = launch_base_root(mixed->lv[l].base, scal + kSlotBase, lv[l].delta, lv[l].n, lv[l].h, mixed->lv[l].sb, stream);
    if (e != hipSuccess) return hip_fail(e, "linear base hierarchy");
  }
  return MR_OK;
}

// Inner solve of J_p e = rhs on level 0 from e = 0 with ncycles linear V-cycles; the level-0
// shift (linsum(0)) must hold (sum rhs, 0). The result is in mixed->lv[0].e[cur].
int Ctx::lin_solve(int ncycles) {
  LinLevel& M0 = mixed->lv[0];
  M0.cur = 0;
  int rc;
  for (int k = 0; k < ncycles; ++k)
    if ((rc = lin_vcycle(0, k == 0)) != MR_OK) return rc;
  return MR_OK;
}

// Building block: k inner V-cycles on J_p(theta_base) e = rhs, all inputs colour-split on level 0
// (delta already in lv[0].delta and the hierarchy prepared); the FP32 base, root and right-hand
// side of level 0 come from the same residual pass as in the solve, the right-hand side then
// replaced by the caller's.
int Ctx::lin_vcycles_split(const double* theta_split, const double* rhs_split, int ncycles, float** e_out) {
  int rc = mixed_alloc(this);
  if (rc != MR_OK) return rc;
  LinLevel& M0 = mixed->lv[0];
  Level& L0 = lv[0];
  const double N3 = (double)L0.cells;
  if ((rc = write_scalar(kSlotRes, 0.0)) != MR_OK) return rc;
  if ((rc = write_scalar(kSlotRes + 1, 0.0)) != MR_OK) return rc;
  if ((rc = write_scalar(kSlotTmax, 0.0)) != MR_OK) return rc;
  hipError_t e = launch_absmax(theta_split, L0.cells, scal + kSlotTmax, stream);
  if (e == hipSuccess) e = launch_base_scale(scal + kSlotTmax, scal + kSlotBase, stream);
  if (e == hipSuccess)
    e = launch_mixed_resid64(theta_split, L0.delta, L0.n, ShiftRef{scal + kSlotRes, 1.0 / N3, 0.0}, M0.rhs, M0.base,
                             scal + kSlotBase, M0.sb, reducer(kSlotRes), stream);
  if (e == hipSuccess) e = launch_cast32(rhs_split, M0.rhs, L0.cells, stream);
  if (e == hipSuccess) e = launch_sum(rhs_split, L0.cells, reducer(kSlotAux), stream);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(set_shift_kernel, dim3(1), dim3(64), 0, stream, (const double*)(scal + kSlotAux), linsum(0));
    e = hipGetLastError();
  }
  if (e != hipSuccess) return hip_fail(e, "linear building block");
  if ((rc = lin_base_hierarchy()) != MR_OK) return rc;
  if ((rc = lin_solve(ncycles)) != MR_OK) return rc;
  *e_out = M0.e[M0.cur];
  return MR_OK;
}

// Krylov storage for a space of m vectors (kept with the context, grown on demand).
static int kry_reserve(Ctx* c, int m) {
  MixedState& ms = *c->mixed;
  KryState& k = ms.kry;
  if (k.m >= m) return MR_OK;
  for (void* p : ms.kry_owned) (void)hipFree(p);
  ms.kry_owned.clear();
  k = KryState{};
  const size_t bytes = c->lv[0].cells * sizeof(float);
  auto get = [&](size_t b) -> void* {
    void* p = nullptr;
    if (hipMalloc(&p, b) != hipSuccess) return nullptr;
    ms.kry_owned.push_back(p);
    return p;
  };
  for (int i = 0; i <= m; ++i) k.V.push_back((float*)get(bytes));
  for (int i = 0; i < m; ++i) k.Z.push_back((float*)get(bytes));
  k.W = (float*)get(bytes);
  k.S = (float*)get(bytes);
  k.partials = (double*)get((size_t)kKryBlocks * kKryNV * sizeof(double));
  k.result = (double*)get(kKryNV * sizeof(double));
  k.counter = (unsigned*)get(64 * sizeof(unsigned));
  bool ok = k.W && k.S && k.partials && k.result && k.counter;
  for (float* p : k.V) ok = ok && p;
  for (float* p : k.Z) ok = ok && p;
  if (!ok || hipMemsetAsync(k.counter, 0, 64 * sizeof(unsigned), c->stream) != hipSuccess) {
    for (void* p : ms.kry_owned) (void)hipFree(p);
    ms.kry_owned.clear();
    k = KryState{};
    return fail(MR_ENOMEM, "Krylov space of %d vectors: allocation failed", m);
  }
  k.m = m;
  return MR_OK;
}

// Least squares min |beta e_1 - H y| for the (k + 1) x k upper Hessenberg H (row-major, ld kKryMax + 1
// columns... stored as h[row][col]) by Givens rotations; returns y.
static void hessenberg_ls(std::vector<std::vector<double>> H, double beta, int k, std::vector<double>& y) {
  std::vector<double> g(k + 1, 0.0);
  g[0] = beta;
  for (int i = 0; i < k; ++i) {
    const double a = H[i][i], b = H[i + 1][i];
    const double r = std::hypot(a, b);
    const double cs = r > 0.0 ? a / r : 1.0, sn = r > 0.0 ? b / r : 0.0;
    for (int j = i; j < k; ++j) {
      const double u = H[i][j], v = H[i + 1][j];
      H[i][j] = cs * u + sn * v;
      H[i + 1][j] = -sn * u + cs * v;
    }
    const double u = g[i], v = g[i + 1];
    g[i] = cs * u + sn * v;
    g[i + 1] = -sn * u + cs * v;
  }
  y.assign(k, 0.0);
  for (int i = k - 1; i >= 0; --i) {
    double s = g[i];
    for (int j = i + 1; j < k; ++j) s -= H[i][j] * y[j];
    y[i] = H[i][i] != 0.0 ? s / H[i][i] : 0.0;
  }
}

// One inner solve of the mixed outer step by flexible GMRES(m) on J_p e = rhs (rhs in the level-0
// rhs buffer, FP32; rhs_sum and rhs_sq the sums of its FP64 values), preconditioned by one linear
// V-cycle per iteration, from e = 0; then theta64 += e (and max |theta| into kSlotTmax). The
// Krylov vectors are mean-free: J_p maps onto mean-free fields and annihilates constants, so the
// mean of the right-hand side is removed and the Gram-Schmidt step removes the mean of J z.
int Ctx::kry_step(double* theta64, int m, double rhs_sum, double rhs_sq, double eta, int* used) {
  int rc = kry_reserve(this, m);
  if (rc != MR_OK) return rc;
  LinLevel& M0 = mixed->lv[0];
  KryState& K = mixed->kry;
  const size_t cells = lv[0].cells;
  const double N = (double)cells;
  const double mean_b = rhs_sum / N;
  const double beta2 = rhs_sq - rhs_sum * rhs_sum / N;
  const double beta = std::sqrt(beta2 > 0.0 ? beta2 : 0.0);
  if (!(beta > 0.0)) return MR_OK;   // nothing to correct
  const int nbu = lin_blocks(cells);
  KryPtrs vp{}, zp{};
  KryCoef cf{};
  cf.c[0] = mean_b;
  cf.c[1] = 1.0 / beta;
  hipLaunchKernelGGL(kry_orth_kernel, dim3(nbu), dim3(256), 0, stream, (const float*)M0.rhs, vp, cf, 0, cells, K.V[0]);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "Krylov start");
  float* rhs_own = M0.rhs;
  float* e_own[2] = {M0.e[0], M0.e[1]};
  std::vector<std::vector<double>> H(m + 1, std::vector<double>(m, 0.0));
  // Givens rotations applied so far and the rotated right-hand side: |g[i + 1]| is the residual norm
  // of the least-squares solution after i + 1 iterations
  std::vector<double> gcs(m, 1.0), gsn(m, 0.0), gg(m + 1, 0.0);
  gg[0] = beta;
  int k = 0;
  for (int i = 0; i < m; ++i) {
    // z_i = one V-cycle on J_p z = v_i from z = 0 (v_i is mean-free: the level-0 shift starts at 0)
    M0.rhs = K.V[i];
    M0.e[0] = K.Z[i];
    M0.e[1] = K.S;
    M0.cur = 0;
    hipLaunchKernelGGL(zero_scalars_kernel, dim3(1), dim3(64), 0, stream, linsum(0), 2);
    e = hipGetLastError();
    if (e != hipSuccess) rc = hip_fail(e, "Krylov cycle start");
    if (rc == MR_OK) rc = lin_vcycle(0, true);
    if (rc == MR_OK && M0.cur == 1) std::swap(K.Z[i], K.S);   // the result ended in the spare buffer
    M0.rhs = rhs_own;
    M0.e[0] = e_own[0];
    M0.e[1] = e_own[1];
    if (rc != MR_OK) return rc;
    // w = J z_i, with its projections on v_0 .. v_i, its sum and its square
    for (int j = 0; j <= i; ++j) vp.p[j] = K.V[j];
    e = launch_lin_apply_dots(K.Z[i], M0.base, scal + kSlotBase, M0.sb, lv[0].n, lv[0].h, K.W, vp, i + 1, K.partials,
                              K.counter, K.result, stream);
    double d[kKryNV];
    if (e == hipSuccess) e = hipMemcpyAsync(d, K.result, (i + 3) * sizeof(double), hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return hip_fail(e, "Krylov dot products");
    const double sum_w = d[i + 1], sq_w = d[i + 2];
    const double mean_w = sum_w / N;
    double hh = sq_w - N * mean_w * mean_w;
    for (int j = 0; j <= i; ++j) {
      H[j][i] = d[j];
      hh -= d[j] * d[j];
    }
    const double hn = std::sqrt(hh > 0.0 ? hh : 0.0);
    H[i + 1][i] = hn;
    k = i + 1;
    {
      std::vector<double> col(i + 2);
      for (int r2 = 0; r2 <= i + 1; ++r2) col[r2] = H[r2][i];
      for (int r2 = 0; r2 < i; ++r2) {
        const double u = col[r2], v = col[r2 + 1];
        col[r2] = gcs[r2] * u + gsn[r2] * v;
        col[r2 + 1] = -gsn[r2] * u + gcs[r2] * v;
      }
      const double rr = std::hypot(col[i], col[i + 1]);
      gcs[i] = rr > 0.0 ? col[i] / rr : 1.0;
      gsn[i] = rr > 0.0 ? col[i + 1] / rr : 0.0;
      gg[i + 1] = -gsn[i] * gg[i];
      gg[i] = gcs[i] * gg[i];
    }
    // stop when the inner residual is below eta of the right-hand side, when the space is exhausted
    // (the next vector would be rounding noise) or after m iterations
    if (std::fabs(gg[i + 1]) <= eta * beta || hn <= 1e-6 * std::sqrt(sq_w > 0.0 ? sq_w : 0.0) || i + 1 == m) break;
    for (int j = 0; j <= i; ++j) cf.c[j] = d[j];
    cf.c[i + 1] = mean_w;
    cf.c[i + 2] = 1.0 / hn;
    hipLaunchKernelGGL(kry_orth_kernel, dim3(nbu), dim3(256), 0, stream, (const float*)K.W, vp, cf, i + 1, cells,
                       K.V[i + 1]);
    if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "Krylov orthogonalisation");
  }
  std::vector<double> y;
  std::vector<std::vector<double>> Hk(k + 1, std::vector<double>(k, 0.0));
  for (int r = 0; r <= k; ++r)
    for (int c2 = 0; c2 < k; ++c2) Hk[r][c2] = H[r][c2];
  hessenberg_ls(Hk, beta, k, y);
  KryPtrs zz{};
  KryCoef yy{};
  for (int j = 0; j < k; ++j) {
    zz.p[j] = K.Z[j];
    yy.c[j] = y[j];
  }
  hipLaunchKernelGGL(kry_update_kernel, dim3(nbu), dim3(256), 0, stream, theta64, zz, yy, k, cells, scal + kSlotTmax);
  e = hipGetLastError();
  if (used) *used = k;
  return e == hipSuccess ? MR_OK : hip_fail(e, "Krylov update");
}

int Ctx::solve_mixed(const double* delta, double* theta, mr_info* info, int aa_depth) {
  auto t0 = std::chrono::steady_clock::now();
  int rc = mixed_alloc(this);
  if (rc != MR_OK) return rc;
  if ((rc = prepare(delta)) != MR_OK) return rc;
  if (aa_depth > 0 && (rc = aa_reserve(aa_depth)) != MR_OK) return rc;
  AAState aa(aa_depth, aa_depth + 1);
  Level& L0 = lv[0];
  const double N3 = (double)L0.cells;
  L0.cur = 0;
  hipError_t e = opts.warm_start ? launch_to_split(theta, L0.th[0], L0.n, stream)
                                 : hipMemsetAsync(L0.th[0], 0, L0.cells * sizeof(double), stream);
  // max |theta| of the start, for the scale of the fixed-point base (kSlotTmax is zero between uses)
  if (e == hipSuccess && (rc = write_scalar(kSlotTmax, 0.0)) != MR_OK) return rc;
  if (e == hipSuccess && opts.warm_start) e = launch_absmax(L0.th[0], L0.cells, scal + kSlotTmax, stream);
  if (e != hipSuccess) return hip_fail(e, "initial theta");
  // reference norm: the residual at theta = 0. From a cold start the first outer residual is that
  // residual (its variance does not depend on the shift it is evaluated with), so it is not
  // evaluated twice.
  const bool cold = !opts.warm_start;
  double r0 = 1.0, m0 = 0.0;
  if (!cold) {
    if ((rc = finest_norm(nullptr, ShiftRef{nullptr, 0.0, 0.0}, &r0, &m0)) != MR_OK) return rc;
    if (r0 == 0.0) r0 = 1.0;
  }
  // running sum of Sigma for the shift of the outer residual: (sum Sigma, 0) at theta = 0
  if ((rc = write_scalar(kSlotRes, m0 * N3)) != MR_OK) return rc;
  if ((rc = write_scalar(kSlotRes + 1, 0.0)) != MR_OK) return rc;
  mr_info loc{};
  loc.r0_norm = r0;
  int it = 0, status = MR_OK;
  double rel = 1.0, best = 1e300, msig = m0, rel_prev = 0.0, eta_prev = 0.5;
  LinLevel& M0 = mixed->lv[0];
  for (;;) {
    e = launch_base_scale(scal + kSlotTmax, scal + kSlotBase, stream);
    if (e == hipSuccess)
      e = launch_mixed_resid64(L0.th[0], L0.delta, L0.n, ShiftRef{scal + kSlotRes, 1.0 / N3, 0.0}, M0.rhs, M0.base,
                               scal + kSlotBase, M0.sb, reducer(kSlotRes), stream);
    if (e != hipSuccess) return hip_fail(e, "mixed residual");
    double r[4];
    if ((rc = read_scalars(kSlotRes, 4, r)) != MR_OK) return rc;
    const double var = r[3] - r[2] * r[2] / N3;
    if (cold && it == 0) {
      r0 = std::sqrt(var > 0.0 ? var : 0.0);
      if (r0 == 0.0) r0 = 1.0;
      loc.r0_norm = r0;
    }
    rel = std::sqrt(var > 0.0 ? var : 0.0) / r0;
    msig = r[0] / N3;
    if (it < 128) loc.history[it] = rel;
    if (!std::isfinite(rel) || rel > 1e6 * (best < 1.0 ? 1.0 : best)) {
      status = fail(MR_EDIVERGED, "residual diverged at outer iteration %d (%g)", it, rel);
      break;
    }
    if (rel < best) best = rel;
    if (rel <= opts.tol || it >= opts.max_cycles) break;
    if ((rc = lin_base_hierarchy()) != MR_OK) return rc;
    if (aa_depth == 0 && !(opts.flags & MR_FLAG_PLAIN_INNER)) {
      // Krylov-accelerated inner solve (inexact Newton): the inner residual is reduced to eta of the
      // outer one, eta from the last outer reduction (Eisenstat and Walker's second choice,
      // 0.9 (rel_k / rel_k-1)^2, safeguarded and at most 0.5) but not below what the tolerance
      // needs (half of tol / rel); at most inner_cycles V-cycles. The rhs -b has sum -r[2] and
      // square sum r[3].
      double eta = 0.5;
      if (it > 0 && rel_prev > 0.0) {
        const double ratio = rel / rel_prev;
        eta = 0.9 * ratio * ratio;
        const double safe = 0.9 * eta_prev * eta_prev;
        if (safe > 0.1) eta = std::max(eta, safe);
      }
      eta = std::min(0.5, std::max(eta, 0.5 * opts.tol / rel));
      int used = 0;
      if ((rc = kry_step(L0.th[0], opts.inner_cycles, -r[2], r[3], eta, &used)) != MR_OK) return rc;
      loc.inner_cycles += used;
      rel_prev = rel;
      eta_prev = eta;
      ++it;
      continue;
    }
    // inner solve from e = 0; the shift starts at <rhs> = -<b>
    hipLaunchKernelGGL(inner_shift_kernel, dim3(1), dim3(64), 0, stream, (const double*)(scal + kSlotRes), linsum(0));
    if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "inner shift");
    if ((rc = lin_solve(opts.inner_cycles)) != MR_OK) return rc;
    loc.inner_cycles += opts.inner_cycles;
    if (aa_depth > 0) {
      // Anderson mixing of the outer iteration theta -> theta + e(theta): the step forms theta + e
      // itself and writes the mixed (or plain) new iterate
      if ((rc = aa_step(aa, L0.th[0], M0.e[M0.cur])) != MR_OK) return rc;
      if ((e = launch_absmax(L0.th[0], L0.cells, scal + kSlotTmax, stream)) != hipSuccess) return hip_fail(e, "max");
    } else if ((e = launch_update64(L0.th[0], M0.e[M0.cur], L0.cells, scal + kSlotTmax, stream)) != hipSuccess) {
      return hip_fail(e, "update");
    }
    ++it;
  }
  if (status == MR_OK && rel > opts.tol) {
    status = MR_NOT_CONVERGED;
    fail(MR_NOT_CONVERGED, "not converged after %d outer iterations (rel residual %g)", it, rel);
  }
  e = launch_sum(L0.th[0], L0.cells, reducer(kSlotGauge), stream);
  if (e == hipSuccess) e = launch_from_split(L0.th[0], theta, L0.n, scal + kSlotGauge, 1.0 / N3, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return hip_fail(e, "gauge");
  loc.status = status;
  loc.cycles = it;
  loc.rel_residual = rel;
  loc.m_shift = msig;
  loc.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (info) *info = loc;
  return status;
}

}  // namespace mr
