// Solver context (internal to the library).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <string>
#include <vector>

#include "mr.h"
#include "mr_kernels.h"

namespace mr {

// Device scalar slots: running sums of (Sigma + f) per level, reduction results, gauge.
constexpr int kSlotLevel = 0;    // 0..31
constexpr int kSlotRes = 32;     // 4 values
constexpr int kSlotGauge = 36;
constexpr int kSlotAux = 40;     // 8 values for the mixed / adjoint drivers
constexpr int kSlotCount = 64;
constexpr int kHostSlots = 80;

struct TileCfg {
  int tk = 64, tj = 8, ci = 32, tiles_j = 1, tiles_k = 1;
};

struct Level {
  int n = 0;
  size_t cells = 0;
  double h = 1.0;
  double* th[2] = {nullptr, nullptr};
  int cur = 0;
  double* that = nullptr;
  const double* delta = nullptr;
  double* delta_own = nullptr;
  double* f = nullptr;
  TileCfg tile;
};

struct MixedState;
struct AdjointState;

struct Ctx {
  int n = 0, nlev = 0, device = 0, max_lds = 65536;
  hipStream_t stream = nullptr;
  mr_opts opts{};
  std::vector<Level> lv;
  double* ws_theta0 = nullptr;
  double* scal = nullptr;
  double* partials = nullptr;
  unsigned int* counter = nullptr;
  double* host = nullptr;
  std::vector<void*> owned;
  MixedState* mixed = nullptr;
  AdjointState* adj = nullptr;

  int dev_alloc(double** p, size_t count);
  Reduce reducer(int slot);
  int read_scalars(int slot, int count, double* out);
  int write_scalar(int slot, double v);
  int sweep(int l);
  int vcycle(int l);
  int finest_norm(const double* theta, ShiftRef sh, double* nrm, double* msig);
  int prepare(const double* delta, double* theta);
  int solve_fp64(const double* delta, double* theta, mr_info* info);
  int solve_mixed(const double* delta, double* theta, mr_info* info);
  void release_extra();
};

int fail(int code, const char* fmt, ...);
int hip_fail(hipError_t e, const char* where);
std::vector<int> level_sizes(int n);
TileCfg choose_tiles(int n, int max_lds);

}  // namespace mr
