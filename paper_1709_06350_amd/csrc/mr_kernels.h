// Kernel argument blocks and launchers (internal to the library).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace mr {

constexpr int kMaxCoarsest = 12 * 12 * 12;
constexpr int kMaxReduceBlocks = 8192;   // partial-sum slots (blocks of a reducing launch)
constexpr int kMaxNV = 4;                // values reduced per launch

// The uniform shift subtracted from the source in a relaxation or defect is
// C = (c_sum ? *c_sum * c_scale : 0) + c_add: either a device-resident running sum of
// (Sigma + f) from the previous pass, or an explicit value.
struct ShiftRef {
  const double* c_sum;
  double c_scale;
  double c_add;
};

struct SweepArgs {
  const double* th_in;
  double* th_out;
  const double* delta;
  const double* f;        // may be null
  int n;
  double h2, ih2;
  const double* c_sum;
  double c_scale, c_add;
  double* sum_out;        // device: sum over cells of (Sigma + f)
  double* partials;
  unsigned int* counter;
  int tj, tiles_j, tiles_k, ci;
};

struct CoarsestArgs {
  double* theta;
  const double* delta;
  const double* f;
  int n, nsweeps;
  double h2, ih2;
  const double* c_sum;
  double c_scale, c_add;
  double* c_sum_out;      // may be null
};

struct Reduce {
  double* partials;
  unsigned int* counter;
  double* result;         // device, up to 4 values
};

size_t sweep_lds_bytes(int tj, int tk);
hipError_t launch_sweep(const SweepArgs& a, int tk, hipStream_t s);
hipError_t launch_coarsest(const CoarsestArgs& a, hipStream_t s);

// theta_c = R theta, dr = R (nabla^2 theta - Sigma - f + C) on the coarse mesh.
hipError_t launch_defect_restrict(const double* theta, const double* delta, const double* f,
                                  int n, double h, ShiftRef c, double* theta_c, double* theta_c2,
                                  double* dr, hipStream_t s);
// f = nabla^2 th - Sigma(th) - rd on an n^3 mesh (f may alias rd); result[0] = sum(Sigma + f).
hipError_t launch_tau(const double* th, const double* delta, const double* rd, double* f, int n,
                      double h, Reduce red, int max_blocks, hipStream_t s);
// theta += P(tc - that) from the (n/2)^3 mesh onto the n^3 mesh.
hipError_t launch_prolong_correct(const double* tc, const double* that, double* theta, int n,
                                  hipStream_t s);
// coarse = 8-son mean of fine (fine n^3).
hipError_t launch_restrict(const double* fine, double* coarse, int n, hipStream_t s);
// b = nabla^2 theta - Sigma + shift on the n^3 mesh (theta == null means theta = 0);
// result[0] = sum b, result[1] = sum b^2; r_out (may be null) receives b.
hipError_t launch_residual(const double* theta, const double* delta, int n, double h,
                           ShiftRef shift, double* r_out, Reduce red, int max_blocks, hipStream_t s);
// result[0] = number of cells with a non-finite delta or 1 + delta <= 0.
hipError_t launch_validate(const double* delta, size_t cells, Reduce red, int max_blocks, hipStream_t s);
// result[0] = sum of a (size cells).
hipError_t launch_sum(const double* a, size_t cells, Reduce red, int max_blocks, hipStream_t s);
// out = in - (*sum) * scale (in and out may alias).
hipError_t launch_shift_copy(const double* in, double* out, size_t cells, const double* sum,
                             double scale, hipStream_t s);

}  // namespace mr
