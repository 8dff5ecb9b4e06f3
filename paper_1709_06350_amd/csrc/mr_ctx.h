// Solver context (internal to the library).
#pragma once

#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstdarg>
#include <string>
#include <vector>

#include "mr.h"
#include "mr_kernels.h"

namespace mr {

// Device scalar slots: per level the running sums (red, black) of Sigma + f of the last sweep
// and a staging slot; reduction results; gauge; scratch for the mixed / adjoint drivers.
constexpr int kSlotLevel = 0;    // 3 per level: [0] red sum, [1] black sum, [2] staging
constexpr int kMaxLevels = 10;
constexpr int kSlotRes = 32;     // 4 values
constexpr int kSlotGauge = 36;
constexpr int kSlotAux = 40;     // 16 values
constexpr int kSlotLin = 64;     // 3 per level: running sums of the linear (FP32 / adjoint) smoother
constexpr int kSlotBase = 112;   // 2 values: 2^-s, 2^s of the fixed-point base of the mixed form
constexpr int kSlotTmax = 114;   // max |theta| (as the bits of a non-negative double; zero between uses)
constexpr int kSlotCount = 128;
constexpr int kHostSlots = 80;

// One mesh of the hierarchy. All fields colour-split; th[0], th[1] are the ping-pong buffers
// (both colours each), th[cur] the current iterate.
struct Level {
  int n = 0;
  size_t cells = 0;
  double h = 1.0;
  double* th[2] = {nullptr, nullptr};
  int cur = 0;
  double* that = nullptr;   // R theta_hat saved for the correction (levels >= 1)
  double* delta = nullptr;
  double* f = nullptr;      // FAS right-hand side (levels >= 1)
  TileCfg sw, df;           // tiles of the half-sweep and of the defect + restriction
  FusedCfg fz;              // tile of the fused red-black sweep (has_fz: one fits)
  bool has_fz = false;
};

struct EventTimer {
  bool on = false;
  std::vector<hipEvent_t> pool;
  std::vector<std::pair<int, int>> pending[2];   // [0] fp64 sweeps, [1] fp32 sweeps
  double ms[2] = {0.0, 0.0};
  int64_t count[2] = {0, 0};
  size_t next = 0;
  int begin(hipStream_t s);                      // returns event index or -1
  void end(int kind, int start, hipStream_t s);
  int resolve();
  void reset();
  void destroy();
};

struct MixedState;
struct AdjointState;

constexpr int kAAMaxDepth = 8;   // longest Anderson history (steps)

// Host side of one Anderson-accelerated solve: the chronological ring slots in use and the Gram
// matrix of the stored fixed-point residuals f (indexed by slot).
struct AAState {
  int depth, ring;
  long long steps = 0;
  std::vector<int> order;
  std::vector<double> gram;
  const double* x_prev = nullptr;   // start of the current cycle (null: the saved first iterate)
  AAState(int depth_, int ring_);
};

struct Ctx {
  int n = 0, nlev = 0, device = 0, max_lds = 65536;
  hipStream_t stream = nullptr;
  mr_opts opts{};
  std::vector<Level> lv;
  double* scal = nullptr;
  double* partials = nullptr;
  unsigned int* counter = nullptr;
  double* host = nullptr;
  std::vector<void*> owned;
  EventTimer timer;
  unsigned long long* cic_grid = nullptr;   // fixed-point CIC accumulation grid (allocated on first use)
  void* dep_mem = nullptr;                   // tile-sorted deposit: counts, offsets, sorted particles, boxes
  size_t dep_bytes = 0;
  MixedState* mixed = nullptr;
  AdjointState* adj = nullptr;
  double* aa_mem = nullptr;   // Anderson history (x save, f and y rings, partials), on first use
  int aa_ring = 0;

  int dev_alloc(double** p, size_t count);
  Reduce reducer(int slot);
  int read_scalars(int slot, int count, double* out);
  int write_scalar(int slot, double v);
  double* lsum(int l) { return scal + kSlotLevel + 3 * l; }
  int sweep(int l);
  int down(int l, double* norm_sums);
  int up(int l);
  int vcycle(int l);
  int finest_norm(const double* theta_split, ShiftRef sh, double* nrm, double* msig);
  int prepare(const double* delta_natural);
  int solve_fp64(const double* delta, double* theta, mr_info* info, int aa_depth = 0);
  int aa_reserve(int depth);
  int aa_step(AAState& st, double* iterate, const float* correction = nullptr);
  void aa_release();
  int solve_mixed(const double* delta, double* theta, mr_info* info, int aa_depth = 0);
  int deposit(const double* pos, long long np, double mass, int scheme, double* delta_out);
  int lagrangian(const double* theta, const double* pos, long long np, double* disp_out, double* psi_out);
  int adjoint_solve(const double* delta, const double* theta_star, const double* g, double* grad, mr_info* info,
                    int aa_depth = 0);
  int adj_sweep(int l);
  int adj_vcycle(int l, double* norm2);
  double adj_last_norm = 0.0, adj_stop = 0.0;
  double* linsum(int l);
  int lin_sweep(int l, bool zero_start = false);
  int lin_vcycle(int l, bool zero = false);
  int lin_coarse_cycle();
  int mixed_ready();
  int lin_schedule(int l, int sched[4]);
  int lin_base_hierarchy();
  int lin_solve(int ncycles);
  int lin_vcycles_split(const double* theta_split, const double* rhs_split, int ncycles, float** e_out);
  int kry_step(double* theta64, int m, double rhs_sum, double rhs_sq, double eta, int* used);
  void release_extra();
  void release_adjoint();
};

int fail(int code, const char* fmt, ...);
int hip_fail(hipError_t e, const char* where);
std::vector<int> level_sizes(int n);
int check_opts(const mr_opts& o);
TileCfg sweep_tiles(int n);
TileCfg defect_tiles(int n);
hipError_t aa_save(const Ctx& c, const double* iterate);

}  // namespace mr
