// Batched mixed-precision solve of many independent periodic boxes of uneven sizes.
//
// Every phase of the outer iteration (FP64 residual, base hierarchy, FP32 linear V-cycle levels,
// FP64 update; the same steps as the one-mesh mixed form) is one kernel launch over all boxes of
// a size class: block b of a launch works on box table[b / bpb], share b % bpb, every box reduces
// into its own partial slots and counter, and a box whose residual is below the tolerance (or
// which has used its iterations) switches itself off on the device, so that the later phases of
// the same pass and all later passes skip it. One outer iteration -- all phases of all size
// classes -- is captured once into a HIP graph and replayed until no box is left; the host reads
// a small status array after each replay. Tile shapes of the FP32 sweep come from a tuner that
// times the compiled shapes per mesh size on the device and caches the choice.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <vector>

#include "mr.h"
#include "mr_ctx.h"
#include "mr_device.h"
#include "mr_kernels.h"
#include "mixed_device.h"
#include "tuning.h"

namespace mr {

constexpr int kBoxPartials = 4096;   // partial-sum slots per box (x kMaxNV values)

struct BLevel {
  float* e[2];
  float* rhs;
  int* base;        // fixed-point base potential (scale: the box's res[5], res[6])
  float* sb;
  const double* delta;
  double* lsum;     // 3 doubles: inner running sums of this level
};

// Convergence state of one box, written by the last block of its residual reduction.
struct BStat {
  int active;       // 1 while the box iterates
  int iters;        // outer updates applied so far
  int maxit;
  int status;       // MR_OK or MR_EDIVERGED
  double r0, tol, rel, best;
  double hist[128]; // relative residual before update 0, 1, ...
};

// Anderson mixing of a box's outer iteration (MR_FLAG_ANDERSON, depth 2): with theta_k the
// iterate after update k and e_k = theta_k - x_k the FP32 correction of that update, the next
// start is sum_j c_j theta_j over the last three updates, c from the least squares on the e's. The
// state lives on the device and is advanced by one thread per box, so the mixing stays inside the
// captured outer iteration.
constexpr int kBAARing = 3;
struct BAAState {
  long long steps;          // updates recorded since the last restart
  int nr, mix;              // entries used by the last combination; 1 if it mixes
  int order[kBAARing];      // ring slots of those entries, oldest first
  double gram[kBAARing * kBAARing];
  double c[kBAARing];
};

struct BBox {
  BLevel lv[kMaxLevels];
  double* theta;    // FP64 colour-split potential (finest)
  double* aaY;      // Anderson history (null without MR_FLAG_ANDERSON): kBAARing iterates
  float* aaF;       // ... and their corrections
  double* aaPart;   // ... per-block partial dot products (256 x kBAARing)
  BAAState* aa;
  double* res;      // 8 doubles: (sum Sigma, 0, sum b, sum b^2) of the last outer residual; [4] max |theta|
                    // (bits; zero between uses), [5] 2^-s and [6] 2^s of the fixed-point base scale
  double* partials;
  unsigned int* counter;
  BStat* st;
};

__device__ __forceinline__ bool box_of(const BBox* boxes, const int* cls, int bpb, int& b, int& t) {
  const int L = xcd_remap(blockIdx.x, gridDim.x);
  b = cls[L / bpb];
  t = L % bpb;
  return boxes[b].st->active != 0;
}

// Convergence bookkeeping of one box after its residual reduction (last block, one thread).
__device__ void box_check(const BBox& x, double N3) {
  BStat& st = *x.st;
  const double var = x.res[3] - x.res[2] * x.res[2] / N3;
  const double rel = sqrt(var > 0.0 ? var : 0.0) / st.r0;
  if (st.iters < 128) st.hist[st.iters] = rel;
  st.rel = rel;
  if (!__builtin_isfinite(rel) || rel > 1e6 * (st.best < 1.0 ? 1.0 : st.best)) {
    st.status = MR_EDIVERGED;
    st.active = 0;
  } else {
    if (rel < st.best) st.best = rel;
    if (rel <= st.tol || st.iters >= st.maxit)
      st.active = 0;
    else
      st.iters += 1;
  }
}

__global__ void __launch_bounds__(256) b_resid64_kernel(const BBox* boxes, const int* cls, int bpb, int n) {
  int b, t;
  if (!box_of(boxes, cls, bpb, b, t)) return;
  const BBox& x = boxes[b];
  const double N3 = (double)n * n * n;
  const bool last = mixed_resid64_body(x.theta, x.lv[0].delta, n, ShiftRef{x.res, 1.0 / N3, 0.0}, x.lv[0].rhs,
                                       x.lv[0].base, x.res + 5, x.lv[0].sb, Reduce{x.partials, x.counter, x.res}, t,
                                       bpb);
  if (last && threadIdx.x == 0) box_check(x, N3);
}

// Tiled FP64 residual of every box of a size class: bpb = tiles_j * tiles_m * nchunks blocks per box.
template <int TM, int TJ>
__global__ void __launch_bounds__(TM * TJ) b_resid64_tiled_kernel(const BBox* boxes, const int* cls, int bpb, int n,
                                                                  int tiles_j, int tiles_m, int nchunks) {
  __shared__ double lds[2 * 4 * (TJ + 2) * (TM + 2)];
  int b, t;
  if (!box_of(boxes, cls, bpb, b, t)) return;
  const BBox& x = boxes[b];
  const double N3 = (double)n * n * n;
  ResidTiledArgs a{x.theta, x.lv[0].delta, n, ShiftRef{x.res, 1.0 / N3, 0.0}, x.lv[0].rhs, x.lv[0].base, x.res + 5,
                   x.lv[0].sb, Reduce{x.partials, x.counter, x.res}, tiles_j, tiles_m, nchunks};
  const bool last = mixed_resid64_tiled_body<TM, TJ>(a, t, t, bpb, lds);
  if (last && threadIdx.x == 0) box_check(x, N3);
}

__global__ void __launch_bounds__(512) b_base_kernel(const BBox* boxes, const int* cls, int bpb, int l, int nf, double ihc2) {
  int b, t;
  if (!box_of(boxes, cls, bpb, b, t)) return;
  const BBox& x = boxes[b];
  restrictq_body(x.lv[l].base, x.lv[l + 1].base, nf, t, bpb);
}

__global__ void __launch_bounds__(512) b_root_kernel(const BBox* boxes, const int* cls, int bpb, int l, int n, double ih2) {
  int b, t;
  if (!box_of(boxes, cls, bpb, b, t)) return;
  const BBox& x = boxes[b];
  base_root_body(x.lv[l].base, x.res + 5, x.lv[l].delta, n, ih2, x.lv[l].sb, t, bpb);
}

__global__ void __launch_bounds__(256) b_fill_kernel(const BBox* boxes, const int* cls, int bpb, int l, int which,
                                                     size_t cells) {
  int b, t;
  if (!box_of(boxes, cls, bpb, b, t)) return;
  fill32_body(boxes[b].lv[l].e[which], 0.0f, cells, t, bpb);
}

// Fixed-point base scale of every active box of a size class from its max |theta| (one thread per box).
__global__ void b_scale_kernel(const BBox* boxes, const int* cls, int nb) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nb) return;
  const BBox& x = boxes[cls[i]];
  if (!x.st->active) return;
  base_scale_body(x.res + 4, x.res + 5);
}

__global__ void b_inner_shift_kernel(const BBox* boxes, const int* cls, int nb) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nb) return;
  const BBox& x = boxes[cls[i]];
  if (!x.st->active) return;
  x.lv[0].lsum[0] = -x.res[2];
  x.lv[0].lsum[1] = 0.0;
}

template <int TM, int TJ, int COL>
__global__ void __launch_bounds__(TM * TJ) b_lin_sweep_kernel(const BBox* boxes, const int* cls, int bpb, int l, int cur,
                                                              int n, float h2, float ih2, int tiles_j, int tiles_m,
                                                              int ci) {
  __shared__ float lds[LinTile<TM, TJ>::LDS];
  int b, t;
  if (!box_of(boxes, cls, bpb, b, t)) return;
  const BBox& x = boxes[b];
  const BLevel& L = x.lv[l];
  LinSweepArgs a{};
  a.e_in = L.e[cur];
  a.e_red_new = COL ? L.e[cur ^ 1] : nullptr;
  a.e_out = L.e[cur ^ 1];
  a.base = L.base;
  a.bq = x.res + 5;
  a.sb = L.sb;
  a.rhs = L.rhs;
  a.n = n;
  a.colour = COL;
  a.h2 = h2;
  a.ih2 = ih2;
  a.c_sum = L.lsum;
  a.c_scale = 1.0 / ((double)n * n * n);
  a.sum_out = COL ? L.lsum + 1 : L.lsum + 2;
  a.copy_from = COL ? L.lsum + 2 : nullptr;
  a.copy_to = COL ? L.lsum : nullptr;
  a.partials = x.partials;
  a.counter = x.counter;
  a.tiles_j = tiles_j;
  a.tiles_m = tiles_m;
  a.ci = ci;
  lin_sweep_pipe_body<TM, TJ, COL>(a, t, t, bpb, lds);
}

__global__ void __launch_bounds__(256) b_resid_restrict_kernel(const BBox* boxes, const int* cls, int bpb, int l, int cur,
                                                               int n, float ih2) {
  int b, t;
  if (!box_of(boxes, cls, bpb, b, t)) return;
  const BBox& x = boxes[b];
  const BLevel& L = x.lv[l];
  lin_resid_restrict_body(L.e[cur], L.base, x.res + 5, L.sb, L.rhs, n, ih2,
                          ShiftRef{L.lsum, 1.0 / ((double)n * n * n), 0.0}, x.lv[l + 1].rhs,
                          Reduce{x.partials, x.counter, x.lv[l + 1].lsum}, t, bpb);
}

template <int TM, int TJ>
__global__ void __launch_bounds__(TM * TJ / 2) b_resid_restrict_tiled_kernel(const BBox* boxes, const int* cls, int bpb,
    int l, int cur, int n, float ih2, int tiles_j, int tiles_m, int nchunks) {
  __shared__ float lds[4 * 4 * (TJ + 2) * (TM + 2)];
  int b, t;
  if (!box_of(boxes, cls, bpb, b, t)) return;
  const BBox& x = boxes[b];
  const BLevel& L = x.lv[l];
  LinRRArgs a{L.e[cur], L.base, x.res + 5, L.sb, L.rhs, n, ih2, ShiftRef{L.lsum, 1.0 / ((double)n * n * n), 0.0},
              x.lv[l + 1].rhs, Reduce{x.partials, x.counter, x.lv[l + 1].lsum}, tiles_j, tiles_m, nchunks};
  lin_resid_restrict_tiled_body<TM, TJ>(a, t, t, bpb, lds);
}

__global__ void __launch_bounds__(512) b_prolong_kernel(const BBox* boxes, const int* cls, int bpb, int l, int cur_c,
                                                        int cur_f, int n) {
  int b, t;
  if (!box_of(boxes, cls, bpb, b, t)) return;
  const BBox& x = boxes[b];
  prolong_add32_body(x.lv[l + 1].e[cur_c], x.lv[l].e[cur_f], n, t, bpb);
}

// Sizes with prolong_rows_ok: bpb = (n/2)^3 / 256 row groups per box, 256 threads each.
__global__ void __launch_bounds__(256) b_prolong_rows_kernel(const BBox* boxes, const int* cls, int bpb, int l,
                                                             int cur_c, int cur_f, int n) {
  __shared__ float cl[kProlongRowsLds];
  int b, t;
  if (!box_of(boxes, cls, bpb, b, t)) return;
  const BBox& x = boxes[b];
  prolong_rows32_body(x.lv[l + 1].e[cur_c], x.lv[l].e[cur_f], n, t, cl);
}

__global__ void __launch_bounds__(256) b_coarsest_kernel(const BBox* boxes, const int* cls, int l, int cur, int n,
                                                         int nsweeps, float h2, float ih2) {
  extern __shared__ unsigned char smem[];
  const BBox& x = boxes[cls[blockIdx.x]];
  if (!x.st->active) return;
  const BLevel& L = x.lv[l];
  lin_coarsest_body(L.e[cur], L.base, x.res + 5, L.sb, L.rhs, n, nsweeps, h2, ih2, L.lsum, 1.0 / ((double)n * n * n),
                    *reinterpret_cast<LinCoarsestShared*>(smem));
}

__global__ void __launch_bounds__(256) b_update_kernel(const BBox* boxes, const int* cls, int bpb, int cur0, size_t cells) {
  int b, t;
  if (!box_of(boxes, cls, bpb, b, t)) return;
  update64_body(boxes[b].theta, boxes[b].lv[0].e[cur0], cells, t, bpb, boxes[b].res + 4);
}

// Slots of the history entries after recording update number `steps` (0-based), oldest first.
__device__ __forceinline__ void baa_order(long long steps, int& nr, int (&order)[kBAARing]) {
  nr = (int)(steps < kBAARing - 1 ? steps : kBAARing - 1) + 1;
  for (int j = 0; j < kBAARing; ++j) order[j] = j < nr ? (int)((steps - (nr - 1) + j) % kBAARing) : 0;
}

// Records theta and e of the update just applied and the dot products of e with the stored e's
// (per-block partials; bpb = 256 blocks per box, the partition of b_update_kernel).
__global__ void __launch_bounds__(256) b_aa_record_kernel(const BBox* boxes, const int* cls, int bpb, int cur0,
                                                          size_t cells) {
  __shared__ double red[4][kBAARing];
  int b, t;
  if (!box_of(boxes, cls, bpb, b, t)) return;
  const BBox& x = boxes[b];
  int nr, order[kBAARing];
  baa_order(x.aa->steps, nr, order);
  const int slot = order[nr - 1];
  const float* __restrict__ e = x.lv[0].e[cur0];
  float* fnew = x.aaF + (size_t)slot * cells;
  double* ynew = x.aaY + (size_t)slot * cells;
  double acc[kBAARing] = {0.0, 0.0, 0.0};
  for (size_t i = t * (size_t)blockDim.x + threadIdx.x; i < cells; i += (size_t)bpb * blockDim.x) {
    const float f = e[i];
    fnew[i] = f;
    ynew[i] = x.theta[i];
#pragma unroll
    for (int j = 0; j < kBAARing; ++j)
      if (j < nr) acc[j] += (double)f * (double)(order[j] == slot ? f : x.aaF[(size_t)order[j] * cells + i]);
  }
  block_sum<kBAARing>(acc, red, threadIdx.x, blockDim.x);
  if (threadIdx.x == 0)
    for (int j = 0; j < kBAARing; ++j) x.aaPart[(size_t)t * kBAARing + j] = acc[j];
}

// One block per box of a size class: adds the partials in block order, updates the Gram matrix
// and solves the 1x1 or 2x2 least-squares problem (a 1e-12 relative Tikhonov term; a negligible
// determinant restarts the history).
__global__ void __launch_bounds__(256) b_aa_solve_kernel(const BBox* boxes, const int* cls, int nparts) {
  __shared__ double red[4][kBAARing];
  const BBox& x = boxes[cls[blockIdx.x]];
  if (!x.st->active) return;
  double acc[kBAARing] = {0.0, 0.0, 0.0};
  for (int p = threadIdx.x; p < nparts; p += blockDim.x)
#pragma unroll
    for (int j = 0; j < kBAARing; ++j) acc[j] += x.aaPart[(size_t)p * kBAARing + j];
  block_sum<kBAARing>(acc, red, threadIdx.x, blockDim.x);
  if (threadIdx.x != 0) return;
  BAAState& st = *x.aa;
  int nr, order[kBAARing];
  baa_order(st.steps, nr, order);
  const int slot = order[nr - 1];
  for (int j = 0; j < nr; ++j) {
    st.gram[slot * kBAARing + order[j]] = acc[j];
    st.gram[order[j] * kBAARing + slot] = acc[j];
  }
  auto G = [&](int a, int c) { return st.gram[order[a] * kBAARing + order[c]]; };
  const int m = nr - 1;
  double gam[2] = {0.0, 0.0};
  bool mix = false;
  if (m == 1) {
    const double M = G(1, 1) - 2.0 * G(1, 0) + G(0, 0);
    const double r = G(1, 1) - G(0, 1);
    if (M > 0.0) {
      gam[0] = r / (M * (1.0 + 1e-12));
      mix = true;
    }
  } else if (m == 2) {
    double M00 = G(1, 1) - G(1, 0) - G(0, 1) + G(0, 0);
    const double M01 = G(1, 2) - G(1, 1) - G(0, 2) + G(0, 1);
    double M11 = G(2, 2) - G(2, 1) - G(1, 2) + G(1, 1);
    const double b0 = G(1, 2) - G(0, 2), b1 = G(2, 2) - G(1, 2);
    const double reg = 1e-12 * 0.5 * (M00 + M11);
    M00 += reg;
    M11 += reg;
    const double det = M00 * M11 - M01 * M01;
    if (det > 1e-13 * M00 * M11) {
      gam[0] = (b0 * M11 - b1 * M01) / det;
      gam[1] = (M00 * b1 - M01 * b0) / det;
      mix = true;
    }
  }
  st.nr = nr;
  for (int j = 0; j < kBAARing; ++j) {
    st.order[j] = order[j];
    st.c[j] = 0.0;
  }
  if (mix) {
    *(x.res + 4) = 0.0;   // the combination replaces theta: its maximum is taken again by the combine
    st.c[m] = 1.0;
    for (int i = 0; i < m; ++i) {
      st.c[i + 1] -= gam[i];
      st.c[i] += gam[i];
    }
    st.mix = 1;
    st.steps += 1;
  } else {
    st.mix = 0;
    st.steps = m >= 1 ? 0 : st.steps + 1;   // an unusable history restarts; the first step has none
  }
}

// theta = sum_j c_j theta_j for the boxes whose last solve mixes.
__global__ void __launch_bounds__(256) b_aa_combine_kernel(const BBox* boxes, const int* cls, int bpb, size_t cells) {
  int b, t;
  if (!box_of(boxes, cls, bpb, b, t)) return;
  const BBox& x = boxes[b];
  const BAAState& st = *x.aa;
  if (!st.mix) return;
  double mx = 0.0;
  for (size_t i = t * (size_t)blockDim.x + threadIdx.x; i < cells; i += (size_t)bpb * blockDim.x) {
    double v = 0.0;
#pragma unroll
    for (int j = 0; j < kBAARing; ++j)
      if (j < st.nr) v += st.c[j] * x.aaY[(size_t)st.order[j] * cells + i];
    x.theta[i] = v;
    mx = fmax(mx, fabs(v));
  }
  block_absmax_to(mx, x.res + 4);
}

// ---- FP32 sweep tile tuner ----------------------------------------------------------------

#define MR_BLIN_TILES(X) X(64, 16) X(64, 8) X(64, 4) X(32, 8) X(16, 16) X(8, 16) X(4, 8) X(2, 4)
#define MR_BRT_TILES(X) X(64, 8) X(32, 8) X(16, 8) X(8, 8) X(4, 8)

static hipError_t launch_b_lin_sweep(const BBox* boxes, const int* cls, int nb, const TileCfg& t, int l, int colour, int cur,
                                     int n, double h, hipStream_t s) {
  const int bpb = t.tiles_j * t.tiles_m * (n / t.ci);
  if (t.ci % 4 != 0) return hipErrorInvalidValue;
  const float h2 = (float)(h * h), ih2 = (float)(1.0 / (h * h));
#define MR_BLIN_LAUNCH(TM, TJ)                                                                                   \
  if (t.tm == TM && t.tj == TJ) {                                                                                \
    if (colour == 0)                                                                                             \
      hipLaunchKernelGGL((b_lin_sweep_kernel<TM, TJ, 0>), dim3(nb * bpb), dim3(TM * TJ), 0, s, boxes, cls, bpb, l, \
                         cur, n, h2, ih2, t.tiles_j, t.tiles_m, t.ci);                                           \
    else                                                                                                         \
      hipLaunchKernelGGL((b_lin_sweep_kernel<TM, TJ, 1>), dim3(nb * bpb), dim3(TM * TJ), 0, s, boxes, cls, bpb, l, \
                         cur, n, h2, ih2, t.tiles_j, t.tiles_m, t.ci);                                           \
    return hipGetLastError();                                                                                    \
  }
  MR_BLIN_TILES(MR_BLIN_LAUNCH)
#undef MR_BLIN_LAUNCH
  return hipErrorInvalidValue;
}

// Candidate shapes and chunk lengths: tiles of at least 128 threads and chunks of at least 8
// planes where the mesh allows them (smaller ones only on meshes too small for those).
static std::vector<TileCfg> lin_candidates(int n) {
  std::vector<TileCfg> out;
  const int nh = n / 2;
  static const int shapes[][2] = {{64, 16}, {64, 8}, {64, 4}, {32, 8}, {16, 16}, {8, 16}, {4, 8}, {2, 4}};
  auto fits = [&](const int* sh) { return nh % sh[0] == 0 && sh[0] <= nh && n % sh[1] == 0 && sh[1] <= n; };
  bool big = false;
  for (const auto& sh : shapes) big = big || (fits(sh) && sh[0] * sh[1] >= 128);
  const int min_ci = n >= 16 ? 8 : 4;
  for (const auto& sh : shapes) {
    if (!fits(sh) || (big && sh[0] * sh[1] < 128)) continue;
    for (int ci : {4, 8, 16, 32, 64, 128, 256}) {
      if (ci > n || n % ci != 0 || ci < min_ci) continue;
      TileCfg t;
      t.tm = sh[0];
      t.tj = sh[1];
      t.ci = ci;
      t.tiles_j = n / t.tj;
      t.tiles_m = nh / t.tm;
      const long bpb = (long)t.tiles_j * t.tiles_m * (n / ci);
      if (bpb > kBoxPartials) continue;
      out.push_back(t);
    }
  }
  return out;
}

static std::mutex g_tune_mu;
static std::map<std::pair<int, int>, std::pair<TileCfg, float>> g_tuned;   // (device, n) -> (tile, ms)

// Times every compiled FP32 sweep shape and chunk length on nb synthetic n^3 boxes (red + black
// half-sweeps of all of them in one launch each, as the batched solve launches a size class) and
// keeps the fastest: with many boxes in a launch the best tile is larger and the chunks longer
// than for one box. The box count is a fixed function of n (as many boxes as fill 2^25 cells,
// 1 to 64), not the batch's, so a box's schedule and hence its result do not depend on the other
// boxes of a batch. Cached per (device, n).
int tune_lin_tiles(int n, hipStream_t s, TileCfg* out, float* ms_out) {
  int dev = 0;
  (void)hipGetDevice(&dev);
  const size_t cells = (size_t)n * n * n;
  const int nb = (int)std::max<size_t>(1, std::min<size_t>(64, ((size_t)1 << 25) / cells));
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    static int gen = -1;
    tuning_sync(gen, g_tuned);
    auto it = g_tuned.find({dev, n});
    if (it != g_tuned.end()) {
      *out = it->second.first;
      if (ms_out) *ms_out = it->second.second;
      return MR_OK;
    }
  }
  // a recorded choice that is still a candidate: the tile and the time of one sweep (float bits)
  {
    std::vector<int> rec;
    if (tuning_lookup("blin32.v1", dev, n, rec) && rec.size() == 8)
      for (const TileCfg& t : lin_candidates(n)) {
        std::vector<int> code = tile_code(t);
        if (!std::equal(code.begin(), code.end(), rec.begin())) continue;
        float ms = 0.0f;
        std::memcpy(&ms, &rec[7], sizeof ms);
        {
          std::lock_guard<std::mutex> lk(g_tune_mu);
          g_tuned[{dev, n}] = {t, ms};
        }
        *out = t;
        if (ms_out) *ms_out = ms;
        return MR_OK;
      }
  }
  std::vector<void*> mem;
  auto get = [&](size_t bytes) -> void* {
    void* p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) return nullptr;
    mem.push_back(p);
    return p;
  };
  std::vector<BBox> hb(nb);
  bool ok = true;
  for (int k = 0; k < nb && ok; ++k) {
    float *e0 = (float*)get(cells * 4), *e1 = (float*)get(cells * 4), *rhs = (float*)get(cells * 4),
          *sb = (float*)get(cells * 4);
    int* base = (int*)get(cells * 4);
    double* aux = (double*)get(64 * 8);
    double* part = (double*)get((size_t)kBoxPartials * kMaxNV * 8);
    unsigned* cnt = (unsigned*)get(64 * 4);
    BStat* dst = (BStat*)get(sizeof(BStat));
    ok = e0 && e1 && rhs && base && sb && aux && part && cnt && dst;
    if (!ok) break;
    hb[k] = BBox{};
    hb[k].lv[0].e[0] = e0;
    hb[k].lv[0].e[1] = e1;
    hb[k].lv[0].rhs = rhs;
    hb[k].lv[0].base = base;
    hb[k].lv[0].sb = sb;
    hb[k].lv[0].lsum = aux;
    hb[k].res = aux + 16;   // zero: base scale 0 (flat base)
    hb[k].partials = part;
    hb[k].counter = cnt;
    hb[k].st = dst;
  }
  BBox* dbox = ok ? (BBox*)get(sizeof(BBox) * nb) : nullptr;
  int* dcls = ok ? (int*)get(sizeof(int) * nb) : nullptr;
  int rc = MR_OK;
  std::vector<TileCfg> cand = lin_candidates(n);
  size_t bi = 0;
  float best_ms = 0.0f;
  if (!ok || !dbox || !dcls || cand.empty()) {
    rc = fail(MR_ENOMEM, "tile tuner: allocation failed or no candidate shape for n = %d", n);
  } else {
    // benign synthetic state: e = 0, rhs = 0, flat base potential, base root 3
    hipError_t e = hipSuccess;
    BStat hs{};
    hs.active = 1;
    std::vector<int> idx(nb);
    for (int k = 0; k < nb && e == hipSuccess; ++k) {
      const BLevel& L = hb[k].lv[0];
      for (void* f : {(void*)L.e[0], (void*)L.e[1], (void*)L.rhs, (void*)L.base})
        if (e == hipSuccess) e = hipMemsetAsync(f, 0, cells * 4, s);
      if (e == hipSuccess) e = launch_fill32(L.sb, 3.0f, cells, s);
      if (e == hipSuccess) e = hipMemsetAsync(L.lsum, 0, 64 * 8, s);
      if (e == hipSuccess) e = hipMemsetAsync(hb[k].counter, 0, 64 * 4, s);
      if (e == hipSuccess) e = hipMemcpyAsync(hb[k].st, &hs, sizeof hs, hipMemcpyHostToDevice, s);
      idx[k] = k;
    }
    if (e == hipSuccess) e = hipMemcpyAsync(dbox, hb.data(), sizeof(BBox) * nb, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(dcls, idx.data(), sizeof(int) * nb, hipMemcpyHostToDevice, s);
    auto run = [&](size_t i) {
      hipError_t x = launch_b_lin_sweep(dbox, dcls, nb, cand[i], 0, 0, 0, n, 1.0, s);
      return x == hipSuccess ? launch_b_lin_sweep(dbox, dcls, nb, cand[i], 0, 1, 0, n, 1.0, s) : x;
    };
    if (e == hipSuccess) e = pick_fastest(cand.size(), 4, s, run, &bi);
    // time of the winner alone (reported)
    hipEvent_t ea = nullptr, eb = nullptr;
    if (e == hipSuccess) e = hipEventCreate(&ea);
    if (e == hipSuccess) e = hipEventCreate(&eb);
    if (e == hipSuccess) e = hipEventRecord(ea, s);
    for (int r = 0; r < 4 && e == hipSuccess; ++r) e = run(bi);
    if (e == hipSuccess) e = hipEventRecord(eb, s);
    if (e == hipSuccess) e = hipEventSynchronize(eb);
    if (e == hipSuccess) e = hipEventElapsedTime(&best_ms, ea, eb);
    best_ms /= 4.0f * nb;
    if (ea) (void)hipEventDestroy(ea);
    if (eb) (void)hipEventDestroy(eb);
    if (e != hipSuccess) rc = hip_fail(e, "tile tuner");
  }
  (void)hipStreamSynchronize(s);
  for (void* p : mem) (void)hipFree(p);
  if (rc != MR_OK) return rc;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tuned[{dev, n}] = {cand[bi], best_ms};
  }
  {
    std::vector<int> code = tile_code(cand[bi]);
    int bits = 0;
    std::memcpy(&bits, &best_ms, sizeof bits);
    code.push_back(bits);
    tuning_record("blin32.v1", dev, n, code);
  }
  *out = cand[bi];
  if (ms_out) *ms_out = best_ms;
  return MR_OK;
}

// ---- batched driver -----------------------------------------------------------------------

namespace {

// Tile of a 2.5D residual kernel for one size class (tm x tj of (m, j), nch chunks of planes).
struct BTile {
  bool ok = false;
  int tm = 0, tj = 0, tiles_j = 0, tiles_m = 0, nch = 0;
  int bpb() const { return tiles_j * tiles_m * nch; }
};

struct SizeClass {
  int n = 0, nlev = 0;
  std::vector<int> boxes;   // global box indices
  int* d_boxes = nullptr;
  std::vector<int> ns;
  std::vector<double> hs;
  std::vector<TileCfg> tiles;
  BTile resid;              // FP64 outer residual (finest level)
  std::vector<BTile> rr;    // linear residual + restriction per level
};

// The largest compiled tile that divides an n^3 mesh (n a multiple of 8), and a chunk count (in
// units of 4 planes, chunks of at least 8 planes) that gives each box about 64 blocks. It depends on
// n only, so a box is reduced in the same order whatever else is in the batch.
BTile pick_btile(int n) {
  static const int pref[][2] = {{64, 8}, {32, 8}, {16, 8}, {8, 8}, {4, 8}};
  BTile t;
  if (n % 8 != 0) return t;
  for (const auto& p : pref) {
    if ((n / 2) % p[0] != 0 || n % p[1] != 0) continue;
    t.tm = p[0];
    t.tj = p[1];
    t.tiles_j = n / p[1];
    t.tiles_m = n / 2 / p[0];
    const long tiles = (long)t.tiles_j * t.tiles_m;
    long nch = (64 + tiles - 1) / tiles;
    nch = std::max(1L, std::min(nch, (long)(n / 8)));
    while (nch > 1 && tiles * nch > kBoxPartials) --nch;
    if (tiles * nch > kBoxPartials) return BTile{};
    t.nch = (int)nch;
    t.ok = true;
    return t;
  }
  return t;
}

// Device memory of one batched call: a single allocation carved into 256-byte aligned pieces. The
// carving runs twice: once to measure (reserve), once on the allocation (get).
struct BatchMem {
  char* base = nullptr;
  size_t size = 0, used = 0;
  bool measuring = true;
  ~BatchMem() {
    if (base) (void)hipFree(base);
  }
  template <typename T>
  T* get(size_t count) {
    const size_t bytes = (count * sizeof(T) + 255) & ~(size_t)255;
    if (measuring) {
      size += bytes;
      return reinterpret_cast<T*>(static_cast<uintptr_t>(256));   // placeholder, never dereferenced
    }
    if (!base || used + bytes > size) return nullptr;
    T* p = reinterpret_cast<T*>(base + used);
    used += bytes;
    return p;
  }
  bool allocate() {
    measuring = false;
    used = 0;
    return hipMalloc((void**)&base, size) == hipSuccess;
  }
};

int rows_grid_b(int rows) { return rows < 1024 ? rows : 1024; }

}  // namespace

static int record_iteration(std::vector<SizeClass>& cls, BBox* dboxes, const mr_opts& o, hipStream_t s) {
  hipError_t e = hipSuccess;
  auto ok = [&]() { return e == hipSuccess ? (e = hipGetLastError()) == hipSuccess : false; };
  int maxlev = 0;
  for (auto& c : cls) maxlev = std::max(maxlev, c.nlev);
  std::vector<std::vector<int>> cur(cls.size(), std::vector<int>(kMaxLevels, 0));
  // 1. FP64 residual of every box (also the base state of level 0, fixed-point with the scale of max |theta|)
  for (auto& c : cls) {
    const int nb = (int)c.boxes.size();
    hipLaunchKernelGGL(b_scale_kernel, dim3((nb + 63) / 64), dim3(64), 0, s, dboxes, c.d_boxes, nb);
    if (c.resid.ok) {
      const BTile& t = c.resid;
      const int bpb = t.bpb();
#define MR_BRT_LAUNCH(TM, TJ)                                                                                     \
      if (t.tm == TM && t.tj == TJ)                                                                               \
        hipLaunchKernelGGL((b_resid64_tiled_kernel<TM, TJ>), dim3(nb * bpb), dim3(TM * TJ), 0, s, dboxes, c.d_boxes, \
                           bpb, c.n, t.tiles_j, t.tiles_m, t.nch);
      MR_BRT_TILES(MR_BRT_LAUNCH)
#undef MR_BRT_LAUNCH
    } else {
      const int bpb = rows_grid_b(c.n * c.n / 8 > 0 ? c.n * c.n / 8 : 1);
      hipLaunchKernelGGL(b_resid64_kernel, dim3(nb * bpb), dim3(c.n < 256 ? (c.n < 64 ? 64 : c.n) : 256), 0, s, dboxes,
                         c.d_boxes, bpb, c.n);
    }
    if (!ok()) return hip_fail(e, "batched residual");
  }
  // 2. base hierarchy
  for (auto& c : cls) {
    const int nb = (int)c.boxes.size();
    for (int l = 1; l < c.nlev; ++l) {
      const int m = c.ns[l];
      const int bpb = rows_grid_b(m * m);
      hipLaunchKernelGGL(b_base_kernel, dim3(nb * bpb), dim3(m < 512 ? m : 512), 0, s, dboxes, c.d_boxes, bpb, l - 1,
                         c.ns[l - 1], 0.0);
      hipLaunchKernelGGL(b_root_kernel, dim3(nb * bpb), dim3(m < 256 ? (m < 64 ? 64 : m) : 256), 0, s, dboxes, c.d_boxes,
                         bpb, l, m, 1.0 / (c.hs[l] * c.hs[l]));
      if (!ok()) return hip_fail(e, "batched base hierarchy");
    }
  }
  // 3. inner linear V-cycles
  for (auto& c : cls) {
    const int nb = (int)c.boxes.size();
    const size_t cells = (size_t)c.n * c.n * c.n;
    hipLaunchKernelGGL(b_fill_kernel, dim3(nb * 64), dim3(256), 0, s, dboxes, c.d_boxes, 64, 0, 0, cells);
    hipLaunchKernelGGL(b_inner_shift_kernel, dim3((nb + 63) / 64), dim3(64), 0, s, dboxes, c.d_boxes, nb);
    if (!ok()) return hip_fail(e, "batched inner start");
  }
  for (int k = 0; k < o.inner_cycles; ++k) {
    // down
    for (int l = 0; l < maxlev; ++l) {
      for (size_t ci = 0; ci < cls.size(); ++ci) {
        SizeClass& c = cls[ci];
        const int nb = (int)c.boxes.size();
        if (l >= c.nlev) continue;
        const int n = c.ns[l];
        const double h = c.hs[l];
        if (l == c.nlev - 1) {
          hipLaunchKernelGGL(b_coarsest_kernel, dim3(nb), dim3(256), sizeof(LinCoarsestShared), s, dboxes, c.d_boxes, l,
                             cur[ci][l], n, o.ncoarse, (float)(h * h), (float)(1.0 / (h * h)));
          if (!ok()) return hip_fail(e, "batched coarsest");
          continue;
        }
        for (int sw = 0; sw < o.npre; ++sw) {
          e = launch_b_lin_sweep(dboxes, c.d_boxes, nb, c.tiles[l], l, 0, cur[ci][l], n, h, s);
          if (e == hipSuccess) e = launch_b_lin_sweep(dboxes, c.d_boxes, nb, c.tiles[l], l, 1, cur[ci][l], n, h, s);
          if (e != hipSuccess) return hip_fail(e, "batched sweep");
          cur[ci][l] ^= 1;
        }
        const int m = n / 2;
        if (c.rr[l].ok) {
          const BTile& t = c.rr[l];
          const int bpb = t.bpb();
#define MR_BRR_LAUNCH(TM, TJ)                                                                                  \
          if (t.tm == TM && t.tj == TJ)                                                                        \
            hipLaunchKernelGGL((b_resid_restrict_tiled_kernel<TM, TJ>), dim3(nb * bpb), dim3(TM * TJ / 2), 0, s, \
                               dboxes, c.d_boxes, bpb, l, cur[ci][l], n, (float)(1.0 / (h * h)), t.tiles_j,      \
                               t.tiles_m, t.nch);
          MR_BRT_TILES(MR_BRR_LAUNCH)
#undef MR_BRR_LAUNCH
        } else {
          const int bpb = rows_grid_b(m * m / 4 > 0 ? m * m / 4 : 1);
          hipLaunchKernelGGL(b_resid_restrict_kernel, dim3(nb * bpb), dim3(m < 256 ? (m < 64 ? 64 : m) : 256), 0, s,
                             dboxes, c.d_boxes, bpb, l, cur[ci][l], n, (float)(1.0 / (h * h)));
        }
        cur[ci][l + 1] = 0;
        const size_t cc = (size_t)m * m * m;
        hipLaunchKernelGGL(b_fill_kernel, dim3(nb * 64), dim3(256), 0, s, dboxes, c.d_boxes, 64, l + 1, 0, cc);
        if (!ok()) return hip_fail(e, "batched restriction");
      }
    }
    // up
    for (int l = maxlev - 2; l >= 0; --l) {
      for (size_t ci = 0; ci < cls.size(); ++ci) {
        SizeClass& c = cls[ci];
        const int nb = (int)c.boxes.size();
        if (l >= c.nlev - 1) continue;
        const int n = c.ns[l];
        const double h = c.hs[l];
        if (prolong_rows_ok(n)) {
          const int bpb = (n / 2) * (n / 2) * (n / 2) / 256;
          hipLaunchKernelGGL(b_prolong_rows_kernel, dim3(nb * bpb), dim3(256), 0, s, dboxes, c.d_boxes, bpb, l,
                             cur[ci][l + 1], cur[ci][l], n);
        } else {
          const int bpb = rows_grid_b(n * n);
          hipLaunchKernelGGL(b_prolong_kernel, dim3(nb * bpb), dim3(n / 2 < 512 ? n / 2 : 512), 0, s, dboxes, c.d_boxes,
                             bpb, l, cur[ci][l + 1], cur[ci][l], n);
        }
        if (!ok()) return hip_fail(e, "batched prolongation");
        for (int sw = 0; sw < o.npost; ++sw) {
          e = launch_b_lin_sweep(dboxes, c.d_boxes, nb, c.tiles[l], l, 0, cur[ci][l], n, h, s);
          if (e == hipSuccess) e = launch_b_lin_sweep(dboxes, c.d_boxes, nb, c.tiles[l], l, 1, cur[ci][l], n, h, s);
          if (e != hipSuccess) return hip_fail(e, "batched sweep");
          cur[ci][l] ^= 1;
        }
      }
    }
    // a further inner cycle restarts from the current level-0 correction: nothing to reset
  }
  // 4. theta += e, then (MR_FLAG_ANDERSON) the mixing of the box's last updates
  for (size_t ci = 0; ci < cls.size(); ++ci) {
    SizeClass& c = cls[ci];
    const int nb = (int)c.boxes.size();
    const size_t cells = (size_t)c.n * c.n * c.n;
    hipLaunchKernelGGL(b_update_kernel, dim3(nb * 256), dim3(256), 0, s, dboxes, c.d_boxes, 256, cur[ci][0], cells);
    if (!ok()) return hip_fail(e, "batched update");
    if (o.flags & MR_FLAG_ANDERSON) {
      hipLaunchKernelGGL(b_aa_record_kernel, dim3(nb * 256), dim3(256), 0, s, dboxes, c.d_boxes, 256, cur[ci][0], cells);
      hipLaunchKernelGGL(b_aa_solve_kernel, dim3(nb), dim3(256), 0, s, dboxes, c.d_boxes, 256);
      hipLaunchKernelGGL(b_aa_combine_kernel, dim3(nb * 256), dim3(256), 0, s, dboxes, c.d_boxes, 256, cells);
      if (!ok()) return hip_fail(e, "batched Anderson mixing");
    }
  }
  return MR_OK;
}

// A batch: the size classes of its boxes, their tiles, one device allocation for every box's
// working set, the descriptors, and the captured outer iteration. Everything a solve needs is made
// once here; a solve then allocates no device memory and captures nothing.
struct Batch {
  int nbox = 0;
  std::vector<int> n;
  mr_opts o{};
  hipStream_t s = nullptr;   // the caller's stream: set-up, inputs and outputs
  BatchMem mem;
  std::vector<BBox> hb;
  std::map<int, int> cls_of_n;
  std::vector<SizeClass> cls;
  BStat* dstat = nullptr;
  BBox* dboxes = nullptr;
  double* scratch = nullptr;
  unsigned* scounter = nullptr;
  double* resall = nullptr;   // 8 doubles per box: the residual sums of its outer iteration
  double* rbuf = nullptr;     // 8 doubles per box: results of the set-up and final reductions
  hipStream_t cs = nullptr;   // the replay stream
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  ~Batch() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (cs) (void)hipStreamDestroy(cs);
  }
};

static int batch_create(Batch& B) {
  const int nbox = B.nbox;
  const int* n = B.n.data();
  const mr_opts& o = B.o;
  hipStream_t s = B.s;
  BatchMem& mem = B.mem;
  std::vector<BBox>& hb = B.hb;
  std::map<int, int>& cls_of_n = B.cls_of_n;
  std::vector<SizeClass>& cls = B.cls;
  hb.resize(nbox);
  for (int b = 0; b < nbox; ++b) {
    if (cls_of_n.find(n[b]) == cls_of_n.end()) {
      cls_of_n[n[b]] = (int)cls.size();
      SizeClass c;
      c.n = n[b];
      c.ns = level_sizes(n[b]);
      c.nlev = (int)c.ns.size();
      if (c.nlev < 2) return fail(MR_EINVAL, "batched: box size %d has a single level", n[b]);
      for (int l = 0; l < c.nlev; ++l) c.hs.push_back(std::ldexp(1.0, l));
      cls.push_back(c);
    }
    cls[cls_of_n[n[b]]].boxes.push_back(b);
  }
  // FP32 sweep tile per level (timed once per device and size)
  for (auto& c : cls)
    for (int l = 0; l < c.nlev; ++l) {
      TileCfg t;
      if (l < c.nlev - 1) {
        int rc = tune_lin_tiles(c.ns[l], s, &t, nullptr);
        if (rc != MR_OK) return rc;
      }
      c.tiles.push_back(t);
    }
  for (auto& c : cls) {
    c.resid = pick_btile(c.n);
    c.rr.assign(c.nlev, BTile{});
    for (int l = 0; l + 1 < c.nlev; ++l) c.rr[l] = pick_btile(c.ns[l]);
  }
  // per-box memory and descriptors, carved from one allocation (measured first)
  BStat*& dstat = B.dstat;
  BBox*& dboxes = B.dboxes;
  double*& scratch = B.scratch;
  unsigned*& scounter = B.scounter;
  double*& resall = B.resall;
  double*& rbuf = B.rbuf;
  auto carve = [&]() -> int {
  dstat = mem.get<BStat>(nbox);
  resall = mem.get<double>(8 * (size_t)nbox);
  rbuf = mem.get<double>(8 * (size_t)nbox);
  if (!dstat || !resall || !rbuf) return fail(MR_ENOMEM, "batched: status array");
  for (int b = 0; b < nbox; ++b) {
    const SizeClass& c = cls[cls_of_n[n[b]]];
    BBox& x = hb[b];
    x = BBox{};
    x.theta = mem.get<double>((size_t)c.n * c.n * c.n);
    x.res = resall + 8 * (size_t)b;
    x.partials = mem.get<double>((size_t)kBoxPartials * kMaxNV);
    x.counter = mem.get<unsigned>(16);
    x.st = dstat + b;
    if (!x.theta || !x.res || !x.partials || !x.counter) return fail(MR_ENOMEM, "batched: box buffers");
    if (o.flags & MR_FLAG_ANDERSON) {
      const size_t cells = (size_t)c.n * c.n * c.n;
      x.aaY = mem.get<double>(kBAARing * cells);
      x.aaF = mem.get<float>(kBAARing * cells);
      x.aaPart = mem.get<double>(256 * kBAARing);
      x.aa = mem.get<BAAState>(1);
      if (!x.aaY || !x.aaF || !x.aaPart || !x.aa) return fail(MR_ENOMEM, "batched: Anderson history");
    }
    for (int l = 0; l < c.nlev; ++l) {
      const size_t cells = (size_t)c.ns[l] * c.ns[l] * c.ns[l];
      BLevel& L = x.lv[l];
      L.e[0] = mem.get<float>(cells);
      L.e[1] = mem.get<float>(cells);
      L.rhs = mem.get<float>(cells);
      L.base = mem.get<int>(cells);
      L.sb = mem.get<float>(cells);
      double* d = mem.get<double>(cells);
      L.delta = d;
      L.lsum = mem.get<double>(4);
      if (!L.e[0] || !L.e[1] || !L.rhs || !L.base || !L.sb || !d || !L.lsum) return fail(MR_ENOMEM, "batched: level buffers");
    }
  }
  dboxes = mem.get<BBox>(nbox);
  if (!dboxes) return fail(MR_ENOMEM, "batched: descriptors");
  for (auto& c : cls) {
    c.d_boxes = mem.get<int>(c.boxes.size());
    if (!c.d_boxes) return fail(MR_ENOMEM, "batched: work table");
  }
  scratch = mem.get<double>((size_t)kMaxReduceBlocks * kMaxNV + 64);
  scounter = mem.get<unsigned>(16);
  if (!scratch || !scounter) return fail(MR_ENOMEM, "batched: scratch");
  return MR_OK;
  };
  int crc = carve();
  if (crc != MR_OK) return crc;
  if (!mem.allocate()) return fail(MR_ENOMEM, "batched: %.1f MiB of device memory", mem.size / 1048576.0);
  if ((crc = carve()) != MR_OK) return crc;
  hipError_t e = hipSuccess;
  for (auto& c : cls)
    if (e == hipSuccess) e = hipMemcpy(c.d_boxes, c.boxes.data(), c.boxes.size() * sizeof(int), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemsetAsync(scounter, 0, 16 * sizeof(unsigned), s);
  if (e == hipSuccess) e = hipMemcpyAsync(dboxes, hb.data(), nbox * sizeof(BBox), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "batched setup");
  // capture one outer iteration (the kernels read the descriptors and per-box state from device
  // memory, so the graph stays valid for every solve of the batch)
  const bool eager = (o.flags & MR_FLAG_EAGER) != 0;
  e = hipStreamCreateWithFlags(&B.cs, hipStreamNonBlocking);
  if (e != hipSuccess) return hip_fail(e, "stream");
  if (eager) return MR_OK;
  e = hipStreamBeginCapture(B.cs, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return hip_fail(e, "graph capture");
  int rc = record_iteration(cls, dboxes, o, B.cs);
  hipError_t e2 = hipStreamEndCapture(B.cs, &B.graph);
  if (rc != MR_OK) return rc;
  if (e2 != hipSuccess) return hip_fail(e2, "graph capture");
  e = hipGraphInstantiate(&B.exec, B.graph, nullptr, nullptr, 0);
  if (e != hipSuccess) return hip_fail(e, "graph instantiate");
  return MR_OK;
}

static int batch_solve(Batch& B, const double* const* delta, double* const* theta, mr_info* infos) {
  auto t0 = std::chrono::steady_clock::now();
  const int nbox = B.nbox;
  const int* n = B.n.data();
  const mr_opts& o = B.o;
  hipStream_t s = B.s;
  std::vector<BBox>& hb = B.hb;
  std::map<int, int>& cls_of_n = B.cls_of_n;
  std::vector<SizeClass>& cls = B.cls;
  BStat* dstat = B.dstat;
  double* scratch = B.scratch;
  unsigned* scounter = B.scounter;
  double* resall = B.resall;
  double* rbuf = B.rbuf;
  hipStream_t cs = B.cs;
  hipError_t e = hipSuccess;
  // Inputs: validate, convert, delta hierarchy, theta = 0. The residual at theta = 0 gives the
  // normalisation r0 and the running sum of Sigma that sets the shift of the first outer residual.
  // Every box reduces into its own result slots, so each phase needs one synchronisation.
  std::vector<double> rh(8 * (size_t)nbox, 0.0);
  for (int b = 0; b < nbox && e == hipSuccess; ++b) {
    const size_t cells = (size_t)n[b] * n[b] * n[b];
    e = launch_validate(delta[b], cells, Reduce{scratch + 64, scounter, rbuf + 8 * (size_t)b}, s);
  }
  if (e == hipSuccess) e = hipMemcpyAsync(rh.data(), rbuf, rh.size() * sizeof(double), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "batched setup");
  for (int b = 0; b < nbox; ++b)
    if (rh[8 * (size_t)b] != 0.0) return fail(MR_EDOMAIN, "batched: box %d has a non-finite value or 1 + delta <= 0", b);
  for (int b = 0; b < nbox && e == hipSuccess; ++b) {
    const SizeClass& c = cls[cls_of_n[n[b]]];
    const size_t cells = (size_t)c.n * c.n * c.n;
    BBox& x = hb[b];
    e = launch_to_split(delta[b], const_cast<double*>(x.lv[0].delta), c.n, s);
    for (int l = 1; l < c.nlev && e == hipSuccess; ++l)
      e = launch_restrict(x.lv[l - 1].delta, const_cast<double*>(x.lv[l].delta), c.ns[l - 1], s);
    if (e == hipSuccess) e = hipMemsetAsync(x.theta, 0, cells * sizeof(double), s);
    for (int l = 0; l < c.nlev && e == hipSuccess; ++l) e = hipMemsetAsync(x.lv[l].lsum, 0, 4 * sizeof(double), s);
    if (e == hipSuccess) e = hipMemsetAsync(x.counter, 0, 16 * sizeof(unsigned), s);
    if (e == hipSuccess)
      e = launch_residual(nullptr, x.lv[0].delta, c.n, 1.0, ShiftRef{nullptr, 0.0, 0.0}, nullptr,
                          Reduce{scratch + 64, scounter, rbuf + 8 * (size_t)b}, s);
  }
  if (e == hipSuccess) e = hipMemcpyAsync(rh.data(), rbuf, rh.size() * sizeof(double), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "batched setup");
  std::vector<BStat> hs(nbox);
  std::vector<double> resinit(8 * (size_t)nbox, 0.0);
  for (int b = 0; b < nbox; ++b) {
    const double cells = (double)n[b] * n[b] * n[b];
    const double s0 = rh[8 * (size_t)b], s1 = rh[8 * (size_t)b + 1];
    const double var = s1 - s0 * s0 / cells;
    BStat& st = hs[b];
    st = BStat{};
    st.active = 1;
    st.maxit = o.max_cycles;
    st.status = MR_OK;
    st.r0 = std::sqrt(var > 0.0 ? var : 0.0);
    if (st.r0 == 0.0) st.r0 = 1.0;
    st.tol = o.tol;
    st.rel = 1.0;
    st.best = 1e300;
    resinit[8 * (size_t)b] = -s0;   // b = -Sigma at theta = 0: running sum of Sigma
  }
  e = hipMemcpy(resall, resinit.data(), resinit.size() * sizeof(double), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(dstat, hs.data(), nbox * sizeof(BStat), hipMemcpyHostToDevice);
  if (o.flags & MR_FLAG_ANDERSON) {
    const BAAState zero{};
    for (int b = 0; b < nbox && e == hipSuccess; ++b) e = hipMemcpy(hb[b].aa, &zero, sizeof(BAAState), hipMemcpyHostToDevice);
  }
  if (e != hipSuccess) return hip_fail(e, "batched setup");
  const bool eager = (o.flags & MR_FLAG_EAGER) != 0;
  int rc = MR_OK;
  // Replay until no box is active; each replay measures every active box once, so max_cycles + 1
  // replays always suffice.
  for (int rep = 0; rc == MR_OK && rep <= o.max_cycles; ++rep) {
    if (eager) {
      rc = record_iteration(cls, B.dboxes, o, cs);
      if (rc != MR_OK) break;
    } else {
      e = hipGraphLaunch(B.exec, cs);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(cs);
    if (e == hipSuccess) e = hipMemcpy(hs.data(), dstat, nbox * sizeof(BStat), hipMemcpyDeviceToHost);
    if (e != hipSuccess) {
      rc = hip_fail(e, "graph replay");
      break;
    }
    bool any = false;
    for (int b = 0; b < nbox; ++b) any = any || hs[b].active;
    if (!any) break;
  }
  if (rc != MR_OK) return rc;
  // final residual of the returned potentials, gauge, output (one synchronisation)
  for (int b = 0; b < nbox && e == hipSuccess; ++b) {
    const SizeClass& c = cls[cls_of_n[n[b]]];
    const size_t cells = (size_t)c.n * c.n * c.n;
    BBox& x = hb[b];
    double* r = rbuf + 8 * (size_t)b;
    e = launch_residual(x.theta, x.lv[0].delta, c.n, 1.0, ShiftRef{nullptr, 0.0, 0.0}, nullptr,
                        Reduce{scratch + 64, scounter, r}, s);
    if (e == hipSuccess) e = launch_sum(x.theta, cells, Reduce{scratch + 64, scounter, r + 2}, s);
    if (e == hipSuccess) e = launch_from_split(x.theta, theta[b], c.n, r + 2, 1.0 / (double)cells, s);
  }
  if (e == hipSuccess) e = hipMemcpyAsync(rh.data(), rbuf, rh.size() * sizeof(double), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "batched output");
  int status = MR_OK;
  for (int b = 0; b < nbox; ++b) {
    const double N3 = (double)n[b] * n[b] * n[b];
    const double s0 = rh[8 * (size_t)b], s1 = rh[8 * (size_t)b + 1];
    const double var = s1 - s0 * s0 / N3;
    const double relf = std::sqrt(var > 0.0 ? var : 0.0) / hs[b].r0;
    int st = hs[b].status;
    if (st == MR_OK && !std::isfinite(relf)) st = MR_EDIVERGED;
    if (st == MR_OK && !(relf <= o.tol)) st = MR_NOT_CONVERGED;
    if (st != MR_OK && (status == MR_OK || (status == MR_NOT_CONVERGED && st < 0))) status = st;
    if (infos) {
      mr_info& inf = infos[b];
      inf = mr_info{};
      inf.status = st;
      inf.cycles = hs[b].iters;
      inf.rel_residual = relf;
      inf.r0_norm = hs[b].r0;
      inf.m_shift = -s0 / N3;
      const int nh = std::min(hs[b].iters + 1, 128);
      for (int k = 0; k < nh; ++k) inf.history[k] = hs[b].hist[k];
      inf.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
  }
  if (status == MR_NOT_CONVERGED) fail(MR_NOT_CONVERGED, "batched: not every box reached the tolerance");
  if (status == MR_EDIVERGED) fail(MR_EDIVERGED, "batched: the residual of at least one box diverged");
  return status;
}

}  // namespace mr

static int batch_check(int nbox, const int* n, const mr_opts* opts, mr_opts& o) {
  if (nbox < 1 || !n) return mr::fail(MR_EINVAL, "batched: bad arguments");
  mr_default_opts(&o);
  if (opts) o = *opts;
  int rc = mr::check_opts(o);
  if (rc != MR_OK) return rc;
  for (int b = 0; b < nbox; ++b) {
    if (n[b] < 8 || n[b] % 2 || n[b] > 1024) return mr::fail(MR_EINVAL, "batched: box size %d not supported", n[b]);
    const auto s = mr::level_sizes(n[b]);
    if ((long)s.back() * s.back() * s.back() > mr::kMaxCoarsest || (int)s.size() > mr::kMaxLevels)
      return mr::fail(MR_EINVAL, "batched: box size %d not supported", n[b]);
  }
  return MR_OK;
}

static int batch_check_io(int nbox, const double* const* delta, double* const* theta) {
  if (!delta || !theta) return mr::fail(MR_EINVAL, "batched: null pointer array");
  for (int b = 0; b < nbox; ++b)
    if (!delta[b] || !theta[b]) return mr::fail(MR_EINVAL, "batched: null box pointer");
  return MR_OK;
}

extern "C" int mr_solve_batched(int nbox, const int* n, const double* const* delta, double* const* theta,
                                const mr_opts* opts, mr_info* infos, void* hip_stream) {
  mr_opts o;
  int rc = batch_check(nbox, n, opts, o);
  if (rc == MR_OK) rc = batch_check_io(nbox, delta, theta);
  if (rc != MR_OK) return rc;
  mr::Batch B;
  B.nbox = nbox;
  B.n.assign(n, n + nbox);
  B.o = o;
  B.s = (hipStream_t)hip_stream;
  rc = mr::batch_create(B);
  if (rc != MR_OK) return rc;
  return mr::batch_solve(B, delta, theta, infos);
}

struct mr_batch {
  mr::Batch b;
};

extern "C" int mr_batch_create(mr_batch** out, int nbox, const int* n, const mr_opts* opts, void* hip_stream) {
  if (!out) return mr::fail(MR_EINVAL, "mr_batch_create: null out");
  *out = nullptr;
  mr_opts o;
  int rc = batch_check(nbox, n, opts, o);
  if (rc != MR_OK) return rc;
  mr_batch* h = new (std::nothrow) mr_batch();
  if (!h) return mr::fail(MR_ENOMEM, "mr_batch_create: host memory");
  h->b.nbox = nbox;
  h->b.n.assign(n, n + nbox);
  h->b.o = o;
  h->b.s = (hipStream_t)hip_stream;
  rc = mr::batch_create(h->b);
  if (rc != MR_OK) {
    delete h;
    return rc;
  }
  *out = h;
  return MR_OK;
}

extern "C" int mr_batch_solve(mr_batch* h, const double* const* delta, double* const* theta, mr_info* infos) {
  if (!h) return mr::fail(MR_EINVAL, "mr_batch_solve: null batch");
  int rc = batch_check_io(h->b.nbox, delta, theta);
  if (rc != MR_OK) return rc;
  return mr::batch_solve(h->b, delta, theta, infos);
}

extern "C" int mr_batch_destroy(mr_batch* h) {
  if (!h) return MR_OK;
  if (h->b.s) (void)hipStreamSynchronize(h->b.s);
  if (h->b.cs) (void)hipStreamSynchronize(h->b.cs);
  delete h;
  return MR_OK;
}

extern "C" int mr_tune_lin_tiles(int n, void* hip_stream, int* tm, int* tj, int* ci, float* ms) {
  if (n < 8 || n % 4 || n > 1024) return mr::fail(MR_EINVAL, "mr_tune_lin_tiles: size %d not supported", n);
  mr::TileCfg t;
  int rc = mr::tune_lin_tiles(n, (hipStream_t)hip_stream, &t, ms);
  if (rc != MR_OK) return rc;
  if (tm) *tm = t.tm;
  if (tj) *tj = t.tj;
  if (ci) *ci = t.ci;
  return MR_OK;
}
