// Kernel argument blocks and launchers (internal to the library).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <utility>
#include <vector>
#include <stddef.h>
#include <stdint.h>

namespace mr {

constexpr int kMaxCoarsest = 12 * 12 * 12;
constexpr int kMaxReduceBlocks = 16384;  // partial-sum slots (blocks of a reducing launch)
constexpr int kMaxNV = 4;                // values reduced per launch

// Tile of the 2.5D kernels: tm columns (m = k >> 1) x tj rows (j), chunks of ci planes (i).
struct TileCfg {
  int tm = 64, tj = 4, ci = 32, tiles_j = 1, tiles_m = 1, cpt = 1;   // cpt: cells per thread per plane
  bool pipe = false;   // one-colour sweeps: the pipelined kernel (cpt 1, ci % 4 == 0)
};

// The uniform shift subtracted from the source in a relaxation or defect is
// C = (c_sum ? (c_sum[0] + c_sum[1]) * c_scale : 0) + c_add: either device-resident running sums
// of (Sigma + f) of the two colours from the previous sweep, or an explicit value.
struct ShiftRef {
  const double* c_sum;
  double c_scale;
  double c_add;
};

// One colour's half-sweep. th_in holds both colours of the snapshot; for the black half-sweep
// th_red_new points at the new red values (colour 0 half of th_out). Writes colour `colour` of
// th_out. sum_out receives sum over the colour of (Sigma + f); after that, the last block copies
// *copy_from to *copy_to when copy_to is set.
struct HalfSweepArgs {
  const double* th_in;
  const double* th_red_new;
  double* th_out;
  const double* delta;
  const double* f;        // may be null
  int n, colour;
  double h2, ih2;
  const double* c_sum;
  double c_scale, c_add;
  double* sum_out;
  const double* copy_from;
  double* copy_to;
  double* partials;
  unsigned int* counter;
  int tj, tiles_j, tiles_m, ci;
  // 0: update every row of the colour. 4 + 2 (i & 1) + (j & 1): update only the rows (i, j) of
  // that parity and copy the others (a sub-sweep of the 4-class ordering; tiled kernel only).
  int row_filter;
};

// Fused defect + restriction: theta_c (and theta_c2) = R theta, dr = R d with
// d = nabla^2 theta - Sigma - f + C; sums_out[0..1] = sum d, sum d^2 over the fine mesh.
struct DefectArgs {
  const double* theta;
  const double* delta;
  const double* f;        // may be null
  int n;
  double ih2;
  const double* c_sum;
  double c_scale, c_add;
  double* theta_c;
  double* theta_c2;       // may be null
  double* dr;
  double* sums_out;
  double* partials;
  unsigned int* counter;
  int tj, tiles_j, tiles_m, ci;
};

// Fused red-black sweep (one launch): th_in holds both colours of the old iterate, th_out
// receives both colours of the new one. sum_out[0] / sum_out[1] receive the sums of Sigma + f over
// the red / black cells as evaluated during the sweep.
struct FusedSweepArgs {
  const double* th_in;
  double* th_out;
  const double* delta;
  const double* f;        // may be null
  int n;
  double h2, ih2;
  const double* c_sum;
  double c_scale, c_add;
  double* sum_out;
  double* partials;
  unsigned int* counter;
  int tiles_j, tiles_m, nchunks;
};

// Tile of the fused sweep: tm x tj cells of (m, j) per block, the i axis split into nchunks
// chunks of (nearly) equal length; blocks = tiles_j * tiles_m * nchunks.
struct FusedCfg {
  int tm = 0, tj = 0, tiles_j = 0, tiles_m = 0, nchunks = 0;
};

struct CoarsestArgs {
  double* theta;
  const double* delta;
  const double* f;
  int n, nsweeps;
  double h2, ih2;
  const double* c_sum;
  double c_scale, c_add;
  double* c_sum_out;      // may be null; receives (sum, 0)
};

// FP32 half-sweep of the linearised operator (mixed precision): e colour `colour` from the
// snapshot e_in (black half-sweep: red from e_red_new), base potential / root / rhs colour-split.
struct LinSweepArgs {
  const float* e_in;
  const float* e_red_new;
  float* e_out;
  const int* base;      // fixed-point base potential (value bq[0] * q)
  const double* bq;     // [0] 2^-s, [1] 2^s of the base's fixed-point scale
  const float* sb;
  const float* rhs;
  int n, colour;
  float h2, ih2;
  const double* c_sum;
  double c_scale, c_add;
  double* sum_out;
  const double* copy_from;
  double* copy_to;
  double* partials;
  unsigned int* counter;
  int tiles_j, tiles_m, ci;
  int zero_black;       // black half-sweep whose old black values are all zero (not read)
};

struct Reduce {
  double* partials;
  unsigned int* counter;
  double* result;         // device, up to 4 values
};

size_t tile_lds_bytes(int tj, int tm);
hipError_t launch_half_sweep(const HalfSweepArgs& a, const TileCfg& t, hipStream_t s);
bool half_sweep_tile_supported(int tm, int tj, int cpt);
bool half_sweep_pipe_supported(int tm, int tj);
hipError_t launch_defect_restrict_tiled(const DefectArgs& a, const TileCfg& t, hipStream_t s);
hipError_t launch_coarsest(const CoarsestArgs& a, hipStream_t s);
// Chooses a fused-sweep tile for an n^3 mesh on the current device by occupancy (false: no
// compiled tile fits).
bool pick_fused(int n, FusedCfg& cfg);

// Picks the fastest of ncand launch candidates; run(i) launches candidate i once on stream s.
// First pass: one warm-up and `reps` timed launches of every candidate; second pass: the four
// fastest again with 3 x reps launches, in two interleaved rounds (close candidates are a few
// percent apart, and a single short timing can misorder them). *best receives the index.
template <class Run>
hipError_t pick_fastest(size_t ncand, int reps, hipStream_t s, Run&& run, size_t* best) {
  *best = 0;
  if (ncand == 0) return hipSuccess;
  hipEvent_t ea = nullptr, eb = nullptr;
  hipError_t e = hipEventCreate(&ea);
  if (e == hipSuccess) e = hipEventCreate(&eb);
  auto time_it = [&](size_t i, int r, float* ms) -> hipError_t {
    hipError_t x = hipEventRecord(ea, s);
    for (int k = 0; k < r && x == hipSuccess; ++k) x = run(i);
    if (x == hipSuccess) x = hipEventRecord(eb, s);
    if (x == hipSuccess) x = hipEventSynchronize(eb);
    if (x == hipSuccess) x = hipEventElapsedTime(ms, ea, eb);
    return x;
  };
  std::vector<std::pair<float, size_t>> first;
  for (size_t i = 0; i < ncand && e == hipSuccess; ++i) {
    float ms = 0.0f;
    e = run(i);   // warm-up
    if (e == hipSuccess) e = time_it(i, reps, &ms);
    if (e == hipSuccess) first.push_back({ms, i});
  }
  if (e == hipSuccess) {
    std::stable_sort(first.begin(), first.end(),
                     [](const std::pair<float, size_t>& a, const std::pair<float, size_t>& b) { return a.first < b.first; });
    const size_t top = std::min<size_t>(4, first.size());
    std::vector<float> tot(top, 0.0f);
    for (int round = 0; round < 2 && e == hipSuccess; ++round)
      for (size_t k = 0; k < top && e == hipSuccess; ++k) {
        float ms = 0.0f;
        e = time_it(first[k].second, 3 * reps, &ms);
        tot[k] += ms;
      }
    size_t bk = 0;
    for (size_t k = 1; k < top; ++k)
      if (tot[k] < tot[bk]) bk = k;
    if (top > 0) *best = first[bk].second;
  }
  if (ea) (void)hipEventDestroy(ea);
  if (eb) (void)hipEventDestroy(eb);
  return e;
}

bool fused_tile_supported(int tm, int tj);
// Times the fused candidates and the two-launch sweep (tiles *two, general and pipelined kernel)
// on the given n^3 buffers, which it overwrites; *use_fused tells whether the fused launch is
// fastest, *cfg its configuration, *two the faster two-launch variant. The result is cached per
// device and n. Returns an MR_ status code.
// Times the pipelined defect + restriction configurations for a's mesh on a's buffers; cached.
int tune_defect(const DefectArgs& a, hipStream_t s);
int tune_sweep(int n, double* th_a, double* th_b, double* delta, double* partials, unsigned* counter, double* sums,
               TileCfg* two, hipStream_t s, bool* use_fused, FusedCfg* cfg);
// One schedule of the FP64 relaxation of a level: two launches per sweep (tile `two`, general or
// pipelined kernel) or the fused red-black launch (tile fz).
struct SweepCand {
  bool fused;
  TileCfg two;
  FusedCfg fz;
};
// The schedules tune_sweep times for an n^3 level (two: the default two-launch tile).
std::vector<SweepCand> sweep_candidates(int n, const TileCfg& two);
// The cached tuning result for n on the current device (false: not tuned or two launches won).
bool tuned_sweep(int n, FusedCfg* cfg);
hipError_t launch_sweep_fused(const FusedSweepArgs& a, const FusedCfg& cfg, hipStream_t s);

// All fields below are colour-split unless named "natural".
// f = nabla^2 th - Sigma(th) - rd on an n^3 mesh (f may alias rd); result[0..1] = (sum(Sigma + f), 0).
hipError_t launch_tau(const double* th, const double* delta, const double* rd, double* f, int n,
                      double h, Reduce red, hipStream_t s);
// The tiled kernel for launch_tau where a tile fits n (*done false: nothing launched).
hipError_t launch_tau_pipe(const double* th, const double* delta, const double* rd, double* f, int n, double h,
                           Reduce red, hipStream_t s, bool* done);
// theta += P(tc - that) from the (n/2)^3 mesh onto the n^3 mesh; that is overwritten with tc - that.
hipError_t launch_prolong_correct(const double* tc, double* that, double* theta, int n, hipStream_t s);
// theta += P(ec - mu) on the fine mesh n (mu = (mu_sum[0] + mu_sum[1]) * mu_scale, 0 if mu_sum is null)
hipError_t launch_prolong_add(const double* ec, const double* mu_sum, double mu_scale, double* theta, int n,
                              hipStream_t s);
// coarse = 8-son mean of fine (fine n^3).
hipError_t launch_restrict(const double* fine, double* coarse, int n, hipStream_t s);
// b = nabla^2 theta - Sigma + shift (theta == null means theta = 0); result[0] = sum b,
// result[1] = sum b^2; r_natural (may be null) receives b in natural order.
hipError_t launch_residual(const double* theta, const double* delta, int n, double h, ShiftRef shift,
                           double* r_natural, Reduce red, hipStream_t s);
// natural -> colour-split and back; from_split subtracts (*sum) * scale when sum is given.
hipError_t launch_to_split(const double* natural, double* split, int n, hipStream_t s);
hipError_t launch_from_split(const double* split, double* natural, int n, const double* sum, double scale,
                             hipStream_t s);
// result[0] = number of entries with a non-finite value or 1 + value <= 0.
hipError_t launch_validate(const double* delta, size_t cells, Reduce red, hipStream_t s);
// result[0] = sum of a (size cells).
hipError_t launch_sum(const double* a, size_t cells, Reduce red, hipStream_t s);
hipError_t launch_cast32(const double* src, float* dst, size_t cells, hipStream_t s);
// fixed-point copy q = round(src bq[1]) of an FP64 field (same layout)
hipError_t launch_quantise(const double* src, int* dst, size_t cells, const double* bq, hipStream_t s);
hipError_t launch_widen64(const float* src, double* dst, size_t cells, hipStream_t s);
hipError_t launch_lin_residual(const float* e, const int* baseq, const double* bq, const float* sb, const float* rhs,
                               int n, double h,
                               double cshift, double* r_out, hipStream_t s);

// ---- mixed precision (FP32 linearised multigrid) ----
// One-launch FP32 sweep schedule: tile tm x tj of (m, j), nchunks equal chunks of planes.
struct LinFusedCfg {
  int tm = 0, tj = 0, nchunks = 0;
};
struct LinFusedArgs {
  const float* e_in;     // both colours of the snapshot
  float* e_out;          // both colours of the result (must not alias e_in)
  const int* base;       // fixed-point base potential
  const double* bq;      // its scale: [0] 2^-s
  const float* sb;       // base root, both colours
  const float* rhs;      // right-hand side, both colours
  int n;
  float h2, ih2;
  const double* c_sum;   // running sums (red, black) of g + rhs of the previous sweep, or null
  double c_scale, c_add;
  double* sum_out;       // receives (red sum, black sum) of this sweep
  double* partials;
  unsigned int* counter;
  int tiles_j, tiles_m, nchunks;
};

bool lin_fused_supported(int tm, int tj);
hipError_t launch_lin_fused(const LinFusedArgs& a, const LinFusedCfg& t, hipStream_t s);
bool lin_tile_supported(int tm, int tj);
hipError_t launch_lin_half_sweep(const LinSweepArgs& a, const TileCfg& t, hipStream_t s);
hipError_t launch_mixed_resid64(const double* theta, const double* delta, int n, ShiftRef C, float* rhs32, int* baseq,
                                const double* bq,
                                float* sb32, Reduce red, hipStream_t s);
hipError_t launch_base_root(const int* baseq, const double* bq, const double* delta, int n, double h, float* sb32,
                            hipStream_t s);
hipError_t launch_restrictq(const int* fine, int* coarse, int n, hipStream_t s);
// max |a| over cells into *tmax (atomic maximum on its bits; *tmax must start at or below it).
hipError_t launch_absmax(const double* a, size_t cells, double* tmax, hipStream_t s);
// bq[0] = 2^-s, bq[1] = 2^s for max |theta| = *tmax; returns *tmax to zero.
hipError_t launch_base_scale(double* tmax, double* bq, hipStream_t s);
hipError_t launch_lin_resid_restrict(const float* e, const int* baseq, const double* bq, const float* sb, const float* rhs,
                                     int n, double h,
                                     ShiftRef c, float* rhs_c, Reduce red, hipStream_t s);
hipError_t launch_prolong_add32(const float* ec, float* e, int n, hipStream_t s);
hipError_t launch_lin_coarsest(float* e, const int* baseq, const double* bq, const float* sb, const float* rhs, int n,
                               int nsweeps, double h,
                               const double* c_sum, double c_scale, hipStream_t s);
hipError_t launch_update64(double* theta, const float* e, size_t cells, double* tmax, hipStream_t s);
hipError_t launch_fill32(float* a, float v, size_t cells, hipStream_t s);

}  // namespace mr
