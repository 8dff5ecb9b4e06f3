/*
 * mr.h -- C ABI of the MI355X (gfx950) library for the nonlinear multigrid solve of the
 * mass-conservation (Monge-Ampere-type) equation used for initial-density reconstruction
 * (Shi, Cautun & Li, "New method for initial density reconstruction").
 *
 * Equation (Sec. II, Eqs. 2-10 and 15): find the periodic displacement potential theta on an
 * n^3 mesh (grid units, h = 1) such that, in every cell,
 *
 *     nabla^2 theta - (Sigma - <Sigma>) = 0,    Sigma = s* - 3,
 *
 * where s* is the largest real root of s^3 + p s + q = 0 with p = -(9/2) tr(Mbar^2),
 * q = 9 tr(Mbar^3) - 27 (1 + delta), Mbar the traceless part of the second-order
 * finite-difference Hessian (Eqs. 11-14). <Sigma> is the uniform shift that makes the periodic
 * problem compatible (it vanishes for every exact discrete solution); it is reported as m_shift.
 * The solution is normalised to <theta> = 0. The solver is the FAS V-cycle of Sec. II.A.3 with
 * red-black Newton-Gauss-Seidel relaxation (Sec. II.A.2, Eq. 17).
 *
 * Conventions shared by every call:
 *  - Arrays are contiguous C-order [n][n][n] (k fastest), periodic, in DEVICE memory owned by
 *    the caller, unless the argument says "host".
 *  - Work is enqueued on the HIP stream given at creation (NULL = default stream). Calls that
 *    return a host scalar synchronise that stream before returning.
 *  - Return codes: MR_OK (0); MR_NOT_CONVERGED (1: outputs are valid but the tolerance was not
 *    reached); MR_EINVAL (-1: null pointer, unsupported size, bad option); MR_EDOMAIN (-2: a
 *    non-finite delta or 1 + delta <= 0); MR_EDIVERGED (-3: non-finite or growing residual);
 *    MR_EHIP (-4: a HIP runtime error); MR_ENOMEM (-5). mr_last_error() returns a
 *    thread-local description of the last failure.
 *  - Supported sizes: n even, n >= 4, and the coarsest mesh reached by halving while the
 *    result stays even and >= 4 must be at most 16 cells wide (4^3 for powers of two,
 *    6^3 for 96^3, 12^3 for 48 * 2^k ...).
 */
#ifndef MR_H
#define MR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  MR_OK = 0,
  MR_NOT_CONVERGED = 1,
  MR_EINVAL = -1,
  MR_EDOMAIN = -2,
  MR_EDIVERGED = -3,
  MR_EHIP = -4,
  MR_ENOMEM = -5
};

enum { MR_PREC_FP64 = 0, MR_PREC_MIXED = 1 };

/* Solver options. tol is the relative residual ||r(theta)||_2 / ||r(0)||_2 on the finest mesh
 * (the paper stops on the rms residual, Sec. II.A.2). npre/npost are red-black sweeps before and
 * after the coarse correction, ncoarse the sweeps on the coarsest mesh (Sec. II.A.3).
 * precision: MR_PREC_FP64, or MR_PREC_MIXED (FP32 relaxation and coarse grids on the linearised
 * operator inside an FP64 defect-correction loop; the FP64 residual decides convergence).
 * inner_cycles: FP32 V-cycles per outer step in mixed precision. warm_start: non-zero to start
 * from the theta passed in instead of theta = 0. flags: MR_FLAG_* bits (0 by default). */
typedef struct {
  double tol;
  int max_cycles;
  int npre;
  int npost;
  int ncoarse;
  int precision;
  int inner_cycles;
  int warm_start;
  int flags;
} mr_opts;

/* MR_FLAG_EAGER (mr_solve_batched only): launch every pass directly on the stream instead of
 * replaying the captured graph (same kernels and arguments; for checking the graph against direct
 * launches). MR_FLAG_TWO_PASS: relax with one launch per colour (red, then black from the new
 * red values) instead of the fused red-black launch; both compute the same update.
 * MR_FLAG_ADJ_ROWS / MR_FLAG_ADJ_TILED (mr_adjoint_solve): relax the adjoint with the untiled
 * row kernel on every level, or with the tiled plane-marching kernel on every level a compiled
 * tile fits, instead of the per-level timed choice; all compute the same update up to rounding
 * order. Setting both is an error.
 * MR_FLAG_ORDER4 (FP64 relaxation: mr_solve at MR_PREC_FP64 and mr_sweep): split each sweep into
 * 4 sub-sweeps instead of the red and black ones (the alternative ordering suggested in
 * Sec. II.A.2). Sub-sweep c = 0..3 updates the cells with 2 ((j + k) mod 2) + ((i + k) mod 2) = c;
 * no cell of the 19-point stencil shares its centre's class, so the sources of a sub-sweep stay
 * fixed while it runs and the update is exact Gauss-Seidel. Each sub-sweep costs about as much as
 * a red-black sweep (row-filtered per-colour launches); the coarsest mesh keeps red-black. The
 * fixed point is the same as with red-black.
 * MR_FLAG_ANDERSON (mr_solve_batched only): mix each box's outer iterations as mr_solve_anderson
 * does, with depth 2 (the state stays on the device, inside the replayed graph); not in the paper,
 * same solutions.
 * MR_FLAG_DEPOSIT_SCATTER (mr_deposit): deposit CIC and TSC with the atomic scatter kernels instead
 * of sorting the particles by mesh tile; both give the same result bit for bit (the same rounded
 * contribution per particle and mesh point, summed exactly in 64-bit fixed point).
 * MR_FLAG_PLAIN_INNER (mr_solve at MR_PREC_MIXED): the inner solve of each outer step is
 * inner_cycles plain linear V-cycles instead of flexible GMRES with inner_cycles V-cycles as the
 * preconditioner (the default; mr_solve_anderson at MR_PREC_MIXED always uses plain cycles). */
enum {
  MR_FLAG_EAGER = 1,
  MR_FLAG_TWO_PASS = 2,
  MR_FLAG_ADJ_ROWS = 4,
  MR_FLAG_ADJ_TILED = 8,
  MR_FLAG_ORDER4 = 16,
  MR_FLAG_ANDERSON = 32,
  MR_FLAG_PLAIN_INNER = 64,
  MR_FLAG_DEPOSIT_SCATTER = 128
};

/* Per-solve report. history[c] is the relative residual after cycle c (history[0] = start).
 * inner_cycles: total linear V-cycles of the inner solves of a mixed-precision solve (0 otherwise). */
typedef struct {
  int status;
  int cycles;
  double rel_residual;
  double r0_norm;
  double m_shift;
  double seconds;
  double history[128];
  int inner_cycles;
} mr_info;

typedef struct mr_ctx mr_ctx;

/* Fills *opts with the defaults: tol 1e-10, max_cycles 100, npre = npost = 2, ncoarse 20,
 * FP64, inner_cycles 1, cold start. */
void mr_default_opts(mr_opts* opts);

/* Creates a solver context for an n^3 mesh: allocates the level hierarchy (about 1/7 of the
 * finest arrays per field) plus one finest-level ping-pong buffer on the current HIP device.
 * opts may be NULL (defaults). hip_stream is a hipStream_t (NULL = default stream).
 * Returns MR_EINVAL for an unsupported n, MR_ENOMEM if allocation fails. */
int mr_create(mr_ctx** out, int n, const mr_opts* opts, void* hip_stream);

/* Releases the context and its device memory (NULL is ignored). */
void mr_destroy(mr_ctx* ctx);

/* Replaces the options of an existing context (same validation as mr_create). */
int mr_set_opts(mr_ctx* ctx, const mr_opts* opts);

/* Mesh size and level count of a context. */
int mr_size(const mr_ctx* ctx);
int mr_levels(const mr_ctx* ctx);

/* FP64 relaxation schedule of one level (0 = finest .. mr_levels - 2; the coarsest level has none):
 * sched[0] = kind (MR_SCHED_TILED: two launches per sweep, general tiled kernel;
 * MR_SCHED_PIPELINED: two launches, plane-pipelined kernel; MR_SCHED_FUSED: one launch for both
 * colours), sched[1] = tile width in columns m (cells of one colour along k), sched[2] = tile
 * height in rows j, sched[3] = number of chunks the planes i are split into. mr_create picks each
 * level's schedule by timing the candidates on this device; all schedules compute the same update
 * and differ only in the rounding order of the sums of Sigma. For callers that need the schedule
 * the solve ran (reports, profiling of one configuration) or identical schedules in several
 * processes (bitwise-equal results): mr_get_schedule reads it, mr_set_schedule pins it (not a
 * passage of the paper). Host-only, no device work. Returns MR_EINVAL for a NULL argument, a level
 * out of range, or a schedule the library has no kernel for (set: the tile must be compiled and
 * divide the level's mesh, chunks must hold at least 4 planes each (MR_SCHED_FUSED splits the
 * planes into nearly equal chunks; the two-launch kinds need equal whole chunks, a multiple of 4
 * planes for MR_SCHED_PIPELINED) and the grid must fit the reduction buffers). */
enum { MR_SCHED_TILED = 0, MR_SCHED_PIPELINED = 1, MR_SCHED_FUSED = 2 };
int mr_get_schedule(const mr_ctx* ctx, int level, int sched[4]);
int mr_set_schedule(mr_ctx* ctx, int level, const int sched[4]);

/* Lists the schedules mr_create's tuner times for one level (0 .. mr_levels - 2), in the format of
 * mr_get_schedule, into sched[4 * i .. 4 * i + 3] for i < max_count, and returns how many there are
 * (the count may exceed max_count; max_count = 0 with sched = NULL only counts). Any of them can be
 * pinned with mr_set_schedule. For callers that check or profile every schedule the tuner may pick
 * (not a passage of the paper). Host-only. Returns MR_EINVAL for a NULL context, a level out of range,
 * max_count < 0, or sched = NULL with max_count > 0. */
int mr_schedule_candidates(const mr_ctx* ctx, int level, int* sched, int max_count);

/* The FP32 sweep schedule of the mixed-precision form on a level (the tuner's choice, see the
 * persistent record of tuner choices below), in the (kind, tm, tj, nchunks) form of
 * mr_get_schedule; the first call allocates the context's mixed-precision buffers (and times the
 * candidates unless a recorded choice applies). Returns MR_EINVAL for a NULL argument or a level
 * without a sweep (the coarsest), MR_ENOMEM if the buffers cannot be allocated. */
int mr_get_lin_schedule(mr_ctx* ctx, int level, int sched[4]);

/* Density assignment (the paper's footnote on density assignment, Sec. I, allows NGP, CIC or TSC).
 * pos: device, np x 3 doubles (x, y, z) in cell units, any finite real value (wrapped
 * periodically); mesh points sit at integer coordinates. Per axis, with b = floor(x) and
 * f = x - b: MR_DEPOSIT_NGP gives weight 1 to the nearest point (b, or b + 1 when f >= 1/2);
 * MR_DEPOSIT_CIC gives 1 - f to b and f to b + 1; MR_DEPOSIT_TSC, with i the NGP point and
 * d = x - i, gives (1/2 - d)^2 / 2, 3/4 - d^2 and (1/2 + d)^2 / 2 to i - 1, i and i + 1. A particle
 * deposits mass times the product of its three axis weights on each point. delta_out: device
 * n^3, receives rho / <rho> - 1 with <rho> = np * mass / n^3 (mass > 0). Accumulation is in
 * unsigned 64-bit fixed point (each weight rounded to a multiple of 2^-40 of a particle's mass
 * before the sum), so the result is bitwise reproducible and independent of the particles' order.
 * CIC and TSC on meshes with n a multiple of 32 up to 512 first sort the particles by mesh tile
 * (16 x 16 x 32 points; counting sort on the device) and accumulate each tile in LDS, without global
 * atomics; this needs 24 bytes per particle and about 11 bytes per mesh point of device memory,
 * kept with the context. NGP, other meshes and MR_FLAG_DEPOSIT_SCATTER use atomic scatter kernels
 * into a 64-bit grid; both ways give the same result bit for bit. Returns MR_EINVAL for a NULL argument,
 * np < 1, a mass that is not positive and finite, an unknown scheme, or particles with a
 * non-finite coordinate (then delta_out is left unchanged); a cell can hold at most 2^24
 * particles' worth of weight, and an overflow (detected from the total) returns MR_EINVAL. */
enum { MR_DEPOSIT_NGP = 0, MR_DEPOSIT_CIC = 1, MR_DEPOSIT_TSC = 2 };
int mr_deposit(mr_ctx* ctx, const double* pos, int64_t np, double mass, int scheme, double* delta_out);

/* Cloud-in-cell density assignment: mr_deposit with MR_DEPOSIT_CIC. */
int mr_deposit_cic(mr_ctx* ctx, const double* pos, int64_t np, double mass, double* delta_out);

/* Lagrangian mapping (the step after the solve). With Theta = Theta_0 + theta and
 * Theta_0 = |x|^2 / 2 (Sec. II), the Lagrangian coordinate is q = grad Theta = x + grad theta, so the
 * displacement is psi = grad theta (x - q = -grad theta, Sec. III). theta: device n^3 in natural
 * order (e.g. the output of mr_solve). On the mesh psi is the second-order central difference
 * (theta(i+1) - theta(i-1)) / 2 per axis (cell units; the discretisation section), periodic; at
 * each particle (pos: device np x 3 doubles in cell units, any real value, wrapped as in
 * mr_deposit_cic) it is interpolated with the CIC weights of mr_deposit_cic (the transpose of the
 * deposit). disp_out: device np x 3, receives psi(x_p), so that q_p = x_p + disp_p. psi_out: device
 * n^3 x 3 doubles laid out [i][j][k][axis], receives the mesh field, or NULL (then the differences
 * at the 8 mesh points around each particle are formed from theta directly, with the same
 * operations, so disp_out is bitwise the same; nothing is allocated). The call synchronizes the
 * context's stream. Returns MR_EINVAL for a NULL argument, np < 1 or a particle with a non-finite
 * coordinate (such a particle's output is NaN, the others are computed). */
int mr_lagrangian(mr_ctx* ctx, const double* theta, const double* pos, int64_t np, double* disp_out,
                  double* psi_out);

/* Residual of a given theta (Sec. II.A.1, Eq. 15 with the mean projection):
 * r = nabla^2 theta - (Sigma - <Sigma>). r_out: device n^3 or NULL. rel_out: host, receives
 * ||r||_2 / ||r(theta = 0)||_2 (NULL allowed). msum_out: host, receives <Sigma> (NULL allowed). */
int mr_residual(mr_ctx* ctx, const double* delta, const double* theta, double* r_out,
                double* rel_out, double* msum_out);

/* mr_residual without a context and without device allocation, for callers that cannot allocate
 * (code under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc). n: 4..1024;
 * delta, theta: device n^3 natural order; r_out (device n^3, may be NULL), rel_out and msum_out (host,
 * may be NULL) as for mr_residual. Work is enqueued on hip_stream (a hipStream_t, NULL = default
 * stream) and the call synchronises it before returning the host scalars. The only device memory
 * used beyond the arguments is a fixed array of about 66 KB that the library holds on every device
 * it runs on until the process ends (per-block partial sums, an arrival counter and the totals);
 * it is shared by every call on a device, so calls that overlap on one device race. Nothing is
 * allocated. Returns MR_EINVAL for a NULL delta or theta or n outside 4..1024, MR_EHIP on a HIP
 * error. */
int mr_residual_noalloc(int n, const double* delta, const double* theta, double* r_out,
                        double* rel_out, double* msum_out, void* hip_stream);

/* FP64 or mixed-precision solve (per opts.precision) for theta given delta (Sec. II.A).
 * theta: device n^3, input guess iff opts.warm_start, output the solution with <theta> = 0.
 * delta is validated (finite, 1 + delta > 0). info: host, may be NULL. */
int mr_solve(mr_ctx* ctx, const double* delta, double* theta, mr_info* info);

/* mr_solve with Anderson acceleration of the V-cycle, for inputs on which the plain
 * cycle converges slowly (cells close to empty, 1 + delta << 1, where the coarse-grid correction
 * contributes little). This is an addition to the paper's method (Sec. II.A.3 runs plain V-cycles);
 * the fixed point, and so the solution, is the same. With y_k the iterate after one V-cycle from
 * x_k and f_k = y_k - x_k, the next iterate is y_k - sum_i gamma_i (y_{i+1} - y_i) over the last
 * `depth` steps (1..8), gamma minimising |f_k - sum_i gamma_i (f_{i+1} - f_i)|_2 (solved from the
 * Gram matrix of the stored f on the host; an ill-conditioned history restarts). The convergence
 * test, tolerances, warm start and the returned info are those of mr_solve. Needs depth + 2 extra
 * fields of n^3 doubles and depth + 1 of floats, allocated on first use and kept with the context.
 * At MR_PREC_MIXED
 * the mixed outer iteration theta -> theta + e(theta) is accelerated the same way. Returns MR_EINVAL
 * for a NULL argument or a depth outside 1..8; otherwise as mr_solve. */
int mr_solve_anderson(mr_ctx* ctx, const double* delta, double* theta, int depth, mr_info* info);

/* Gradient of a loss through the solve. Given delta, the converged theta_star = solve(delta)
 * and g = dLoss/dtheta (device n^3 each), writes grad_delta = dLoss/ddelta (device n^3):
 * solves J_p^T lambda = g - <g> (J_p the Jacobian of the mean-projected operator, obtained by
 * differentiating the physical root of the cubic of Sec. II, Eqs. 8-10) with a linear multigrid
 * on the transposed operator, coefficients rebuilt per level from theta_star and delta, then
 * grad = (dSigma/ddelta) * (lambda - <lambda>). tol/max_cycles/npre/npost from the context
 * options. info may be NULL. */
int mr_adjoint_solve(mr_ctx* ctx, const double* delta, const double* theta_star,
                     const double* g, double* grad_delta, mr_info* info);

/* mr_adjoint_solve with Anderson mixing of lambda between the transposed V-cycles, as
 * mr_solve_anderson does for theta (not in the paper; same solution). depth 1..8; the history is
 * the one of mr_solve_anderson (shared). Returns MR_EINVAL for
 * a NULL argument or a depth outside 1..8; otherwise as mr_adjoint_solve. */
int mr_adjoint_solve_anderson(mr_ctx* ctx, const double* delta, const double* theta_star, const double* g,
                              double* grad_delta, int depth, mr_info* info);

/* Batched solve of nbox independent periodic boxes of possibly different sizes (the one-mesh
 * solve applied box by box, Sec. II.A, in the mixed-precision form). n: host array of nbox box
 * sizes (each even, 8..1024, coarsest level at most 12^3). delta, theta: host arrays of nbox
 * device pointers, delta[b] and theta[b] of n[b]^3 doubles in natural order; theta[b] is
 * written (zero mean), every box starts from theta = 0. opts: as for mr_create (NULL: the
 * defaults); precision and warm_start are ignored. Each phase of an outer iteration is one
 * launch per distinct box size covering all boxes of that size; one outer iteration is captured
 * in a HIP graph and replayed until every box has reached opts->tol or used opts->max_cycles
 * iterations (a box that has stops being updated). FP32 sweep tiles per size come from
 * mr_tune_lin_tiles. infos: host array of nbox reports (may be NULL); history[k] is the relative
 * residual before update k, rel_residual the one of the returned potential. Device memory is
 * allocated for the call and freed before it returns; the call synchronizes hip_stream.
 * Returns MR_OK, MR_NOT_CONVERGED or MR_EDIVERGED (the worst box), MR_EDOMAIN for an invalid
 * delta, or an argument / HIP / memory error. */
int mr_solve_batched(int nbox, const int* n, const double* const* delta, double* const* theta,
                     const mr_opts* opts, mr_info* infos, void* hip_stream);

/* Reusable batch: the work of mr_solve_batched split into a set-up that is done once and solves
 * that repeat it on new inputs. mr_batch_create groups the nbox sizes n[] into size classes, picks
 * the tiles, allocates one device block for every box's working set (all levels, the descriptors,
 * the status array) and captures one outer iteration in a HIP graph, on hip_stream; opts as for
 * mr_solve_batched. mr_batch_solve solves the boxes for delta[b] into theta[b] (host arrays of
 * nbox device pointers to n[b]^3 doubles, natural order) exactly as mr_solve_batched does, with
 * no device allocation and no graph capture; it synchronises the batch's stream and returns as
 * mr_solve_batched. mr_batch_destroy frees the batch (NULL is a no-op). A batch is not thread
 * safe: calls on one batch must not overlap. Device memory per box: 28 bytes per cell on every
 * level (two FP32 corrections, the FP32 right-hand side, the fixed-point base and its root, FP64
 * delta), about 1.15 x that over the hierarchy, plus the FP64 potential (8 bytes per finest cell);
 * with MR_FLAG_ANDERSON, 12 bytes more per finest cell and history slot. */
typedef struct mr_batch mr_batch;
int mr_batch_create(mr_batch** out, int nbox, const int* n, const mr_opts* opts, void* hip_stream);
int mr_batch_solve(mr_batch* batch, const double* const* delta, double* const* theta, mr_info* infos);
int mr_batch_destroy(mr_batch* batch);

/* Tile tuner of the FP32 linear sweep used by mr_solve_batched: times every compiled tile shape
 * and plane-chunk length on a launch over several synthetic n^3 boxes (as many as fill 2^25 cells,
 * 1 to 64: the batched solve launches all boxes of a size together) on the current device, and
 * returns (and caches per device and n) the fastest: tm cells along z/2, tj rows, ci planes per
 * block, ms the time of one red+black sweep per box. Any output pointer may be NULL.
 * n: multiple of 4, 8..1024. */
int mr_tune_lin_tiles(int n, void* hip_stream, int* tm, int* tj, int* ci, float* ms);

/* Persistent tuner choices. Every tuner of the library (FP64 sweep and defect schedules, the FP32
 * sweep of the mixed form, the batched FP32 sweep tiles, the adjoint sweep) times its candidates
 * once per device and mesh size; the choice is kept for the process and recorded in a text file
 * so that later processes on the same kind of device make the same choice without timing. A
 * record is a list of integers under (tuner kind with a format version, architecture name,
 * device (its memory size, "<GiB>GiB"), compute-unit count, n). A tuner uses a recorded choice only if it is among its
 * current candidates, and times again otherwise. The file is $MR_TUNING_FILE if that variable is
 * set (an empty value: no file), else $XDG_CACHE_HOME/paper_1709_06350_amd/tuning.txt, else
 * $HOME/.cache/paper_1709_06350_amd/tuning.txt; it is read on first use and rewritten (through a
 * temporary file and a rename) when a choice is recorded. A file that cannot be written is not an
 * error for the tuners. A key the file does not hold is looked up in the choices shipped with the
 * library, tuning_defaults.txt in the directory of libmr.so (or $MR_TUNING_DEFAULTS; an empty value:
 * none), which is read but never written (a choice taken from it is copied into the record file).
 * Host code only; no device is needed for these four calls.
 *
 * mr_tuning_file: use path from now on (NULL: back to the default above; "": no file) and forget
 * the choices read so far (the shipped ones are read again too). mr_tuning_file_path: the file in
 * use ("" if none; the pointer is valid until the next mr_tuning_file). mr_tuning_store: record count
 * (1..64) values under the key and write the file (MR_EINVAL if it cannot be written).
 * mr_tuning_lookup: the values recorded under the key (else the shipped ones) into vals (at most
 * max_count), their number into *count (0 if none). */
int mr_tuning_file(const char* path);
const char* mr_tuning_file_path(void);
int mr_tuning_store(const char* kind, const char* arch, const char* device, int cus, int n, const int* vals,
                    int count);
int mr_tuning_lookup(const char* kind, const char* arch, const char* device, int cus, int n, int* vals, int max_count,
                     int* count);

/* ---- Building blocks of the cycle, exported so that each can be checked in isolation. ----
 * All act on one mesh of size nl (any level of a hierarchy) with cell size h, on the context's
 * stream, and write only their outputs. */

/* One red-black Newton-Gauss-Seidel sweep (Sec. II.A.2, Eq. 17): red cells ((i+j+k) even)
 * are updated from theta_in, then black cells from the red results and theta_in's black values:
 *     theta_c <- (sum of 6 face neighbours - h^2 (Sigma_c + f_c - cshift)) / 6.
 * f may be NULL (zero). theta_out must not alias theta_in. sum_out (host, may be NULL)
 * receives sum over all cells of (Sigma_c + f_c) as evaluated during the sweep. When nl is the mesh
 * size of a relaxed level of the context, the sweep runs that level's schedule (the one the solve
 * uses, as read by mr_get_schedule and pinned by mr_set_schedule; with MR_FLAG_TWO_PASS the level's
 * two-launch tile). Other sizes run the fused red-black kernel, or the two per-colour launches
 * (the pipelined kernel where the default tile allows it) when the context's opts.flags has
 * MR_FLAG_TWO_PASS. With MR_FLAG_ORDER4 it runs the four
 * class sub-sweeps instead (cells of class 0, then 1, 2, 3, each from the previous result) and
 * sum_out is the sum evaluated during the last sub-sweep. */
int mr_sweep(mr_ctx* ctx, int nl, double h, const double* delta, const double* f, double cshift,
             const double* theta_in, double* theta_out, double* sum_out);

/* Defect and restriction (Sec. II.A.3, Eq. 18 and the 8-son average R):
 * d = nabla^2 theta - Sigma - f + cshift on the nl^3 mesh; writes theta_c = R theta and
 * dr_c = R d on the (nl/2)^3 mesh. f may be NULL. */
int mr_defect_restrict(mr_ctx* ctx, int nl, double h, const double* delta, const double* f,
                       double cshift, const double* theta, double* theta_c, double* dr_c);

/* Coarse right-hand side of the FAS equation (Sec. II.A.3, Eq. 19): on the nl^3 mesh with
 * cell size h, f = nabla^2 theta_hat - Sigma(theta_hat) - rd (in place on rd_f allowed:
 * pass the same pointer for rd and f_out). sum_out (host, may be NULL): sum of Sigma + f. */
int mr_tau_rhs(mr_ctx* ctx, int nl, double h, const double* delta, const double* theta_hat,
               const double* rd, double* f_out, double* sum_out);

/* Correction (Sec. II.A.3, Eq. 20): theta += P(theta_c - theta_hat_c), P trilinear between
 * cell centres (weights 3/4, 1/4 per axis); theta is the nl^3 mesh, the others (nl/2)^3. */
int mr_prolong_correct(mr_ctx* ctx, int nl, const double* theta_c, const double* theta_hat_c,
                       double* theta);

/* 8-son average R from an nl^3 to an (nl/2)^3 mesh (Sec. II.A.3). */
int mr_restrict(mr_ctx* ctx, int nl, const double* fine, double* coarse);

/* ---- Building blocks of the FP32 inner solve of the mixed-precision form. ----
 * The inner operator is the Jacobian of the mean-projected operator at a base potential theta_b
 * (differentiating the physical root s of the cubic of Sec. II, Eqs. 8-10, with the discrete
 * Hessian of Eqs. 11-14):
 *     J_p e = nabla^2 e - dSigma(e) + <dSigma(e)>,   dSigma(e) = tr(W dMbar(e)),
 *     W = (9 s Mbar - 27 Mbar^2) / (3 s^2 + p),
 * Mbar, p and s those of theta_b (cell size h). It is evaluated in FP32: theta_b is rounded to
 * FP32, and s is the largest real root computed (in FP64) from the FP32 theta_b and delta, as on
 * the coarse levels of the inner solve. Arrays are natural-order doubles on the device. */

/* Defect of the linear level equation J e = rhs - cshift (the uniform shift as in mr_sweep):
 * r_out = rhs + dSigma(e) - nabla^2 e - cshift on the nl^3 mesh with cell size h (with
 * cshift = <rhs + dSigma(e)> this is (rhs - <rhs>) - J_p e). rhs may be NULL (zero). r_out receives
 * the FP32 result widened to FP64. Returns MR_EINVAL for a NULL argument, an unsupported nl or
 * h <= 0. */
int mr_lin_residual(mr_ctx* ctx, int nl, double h, const double* delta, const double* theta_base,
                    const double* e, const double* rhs, double cshift, double* r_out);

/* The inner solve's fused defect and restriction (the linear counterpart of mr_defect_restrict,
 * Sec. II.A.3 Eq. 18 and R): rc_out = R(rhs + dSigma(e) - nabla^2 e - cshift) on the (nl/2)^3 mesh,
 * computed by the kernel the inner V-cycle runs. rhs may be NULL. Returns MR_EINVAL for a NULL
 * argument, nl not a multiple of 4 or h <= 0. */
int mr_lin_defect_restrict(mr_ctx* ctx, int nl, double h, const double* delta, const double* theta_base,
                           const double* e, const double* rhs, double cshift, double* rc_out);

/* One red-black sweep of the inner solve's smoother on the nl^3 mesh (cell size h): red cells
 * ((i + j + k) even) from e_in, then black cells from the new red values, each by
 *     e_c <- (sum of 6 face neighbours of e - h^2 (dSigma_c(e) + rhs_c - cshift)) / 6
 * (the linear level equation nabla^2 e - dSigma(e) = rhs - cshift solved at the cell; dSigma does not
 * depend on e_c). rhs may be NULL (zero). sched: (kind, tm, tj, nchunks) as for mr_set_schedule --
 * MR_SCHED_FUSED runs the one-launch kernel of both colours, MR_SCHED_PIPELINED / MR_SCHED_TILED the
 * two one-colour launches -- or NULL for a default two-launch schedule. e_out receives the FP32
 * result widened to FP64 (e_out must not alias e_in). Returns MR_EINVAL for a NULL argument, nl not a
 * multiple of 4, h <= 0, or a schedule the library has no kernel for. */
int mr_lin_sweep(mr_ctx* ctx, int nl, double h, const double* delta, const double* theta_base,
                 const double* e_in, const double* rhs, double cshift, const int* sched, double* e_out);

/* The inner solve's coarse-to-fine correction (Sec. II.A.3, the prolongation P of the V-cycle, in
 * FP32): e_out = e_in + P ec on the nl^3 mesh, ec on the (nl/2)^3 mesh, P the cell-centred
 * trilinear interpolation (per axis, fine cell 2I takes 3/4 of coarse cell I and 1/4 of I-1, fine
 * cell 2I+1 3/4 of I and 1/4 of I+1, periodic). Computed by the kernel the inner V-cycle runs at
 * this size, with ec and e_in rounded to FP32; e_out receives the result widened to FP64. Arrays
 * are natural-order doubles on the device; e_out may alias e_in. Returns MR_EINVAL for a NULL
 * argument or nl not a multiple of 4 in 4..1024. */
int mr_lin_prolong_add(mr_ctx* ctx, int nl, const double* ec, const double* e_in, double* e_out);

/* ncycles (1..64) inner linear V-cycles of the mixed-precision solve on the context's mesh, from
 * e = 0, for J_p e = rhs at the base theta_base (the finest level's FP32 base and root come from
 * the same FP64 residual pass as in mr_solve; coarse levels restrict the base and take their own
 * root, as in the solve). e_out receives e (its mean is not fixed: J_p annihilates constants).
 * The options' npre, npost and ncoarse apply. delta is validated as for mr_solve. */
int mr_lin_vcycles(mr_ctx* ctx, const double* delta, const double* theta_base, const double* rhs,
                   int ncycles, double* e_out);

/* Kernel timing with HIP events on the context's stream, for benchmarking. mr_timing_enable
 * resets the counters and turns recording on (on != 0) or off. Recorded: every finest-mesh
 * relaxation sweep launch (FP64 sweep, and the FP32 sweep of the mixed-precision form).
 * mr_timing_read synchronises the stream and reports totals since the last enable. */
typedef struct {
  double sweep64_ms;          /* summed duration of finest-mesh FP64 sweep launches */
  int64_t sweep64_launches;
  double sweep32_ms;          /* summed duration of finest-mesh FP32 sweep launches */
  int64_t sweep32_launches;
  int64_t finest_cells;       /* cells of the finest mesh (cell updates per sweep) */
} mr_timing;

int mr_timing_enable(mr_ctx* ctx, int on);
int mr_timing_read(mr_ctx* ctx, mr_timing* out);

/* HBM bandwidth probe (not part of the method): the ceiling that the memory-bound kernels are
 * judged against, measured with hand-written streaming kernels on the current device.
 * MR_STREAM_COPY: c[i] = a[i] (16 B per element); MR_STREAM_READ: per-block partial sums of a into
 * c[0 .. blocks-1] (8 B per element); MR_STREAM_TRIAD: c[i] = a[i] + b[i] / 2 (24 B per element, the
 * traffic of one FP64 relaxation update: two reads and one write). count doubles (even, >= 2) per
 * array, device memory; nontemporal != 0 uses non-temporal loads and stores. The grid is
 * blocks_per_cu (1..64) blocks of 256 threads per compute unit. ms_out (host, may be NULL) receives
 * the launch's duration from HIP events on hip_stream (the call then synchronises the event).
 * Returns MR_EINVAL for a bad argument (for MR_STREAM_READ, c must hold one value per block). */
enum { MR_STREAM_COPY = 0, MR_STREAM_READ = 1, MR_STREAM_TRIAD = 2 };
int mr_hbm_stream(int kind, int nontemporal, const double* a, const double* b, double* c, size_t count,
                  int blocks_per_cu, void* hip_stream, float* ms_out);

const char* mr_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* MR_H */
