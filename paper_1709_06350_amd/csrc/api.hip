// Host side of the library: context and level hierarchy, the FAS V-cycle driver (Sec. II.A.3)
// and the C ABI declared in include/mr.h. Inside the solver all fields are colour-split
// (mr_device.h); the caller's arrays are in natural C order and are converted at the boundary.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "mr.h"
#include "mr_ctx.h"
#include "mr_kernels.h"

namespace mr {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

int hip_fail(hipError_t e, const char* where) {
  return fail(MR_EHIP, "%s: %s", where, hipGetErrorString(e));
}

std::vector<int> level_sizes(int n) {
  std::vector<int> s{n};
  while (s.back() % 2 == 0 && s.back() / 2 >= 4 && (s.back() / 2) % 2 == 0) s.push_back(s.back() / 2);
  return s;
}

int check_size(int n) {
  if (n < 4 || n % 2 != 0) return fail(MR_EINVAL, "n = %d: must be even and >= 4", n);
  if (n > 1024) return fail(MR_EINVAL, "n = %d: larger than 1024", n);
  const auto s = level_sizes(n);
  if ((long)s.back() * s.back() * s.back() > kMaxCoarsest)
    return fail(MR_EINVAL, "n = %d: coarsest mesh %d^3 exceeds 12^3", n, s.back());
  if ((int)s.size() > kMaxLevels) return fail(MR_EINVAL, "n = %d: too many levels", n);
  return MR_OK;
}

int check_opts(const mr_opts& o) {
  if (!(o.tol >= 0.0) || o.max_cycles < 1 || o.max_cycles > 127 || o.npre < 0 || o.npost < 0 ||
      o.npre + o.npost < 1 || o.ncoarse < 1 ||
      (o.precision != MR_PREC_FP64 && o.precision != MR_PREC_MIXED) || o.inner_cycles < 1 ||
      o.inner_cycles > 8 ||
      (o.flags & ~(MR_FLAG_EAGER | MR_FLAG_TWO_PASS | MR_FLAG_ADJ_ROWS | MR_FLAG_ADJ_TILED | MR_FLAG_ORDER4 |
                   MR_FLAG_ANDERSON | MR_FLAG_PLAIN_INNER | MR_FLAG_DEPOSIT_SCATTER)) != 0 ||
      (o.flags & MR_FLAG_ADJ_ROWS && o.flags & MR_FLAG_ADJ_TILED))
    return fail(MR_EINVAL, "invalid options");
  return MR_OK;
}

static int pow2_divisor(int v, int cap) {
  int t = cap;
  while (t > 1 && (v % t != 0 || t > v)) t /= 2;
  return t;
}

static void pick_chunk(TileCfg& t, int n, bool even, int target_blocks, int min_ci) {
  const long tiles = (long)t.tiles_j * t.tiles_m;
  t.ci = n;
  while (t.ci % 2 == 0 && t.ci / 2 >= min_ci && (!even || (t.ci / 2) % 2 == 0) &&
         tiles * (n / t.ci) < target_blocks)
    t.ci /= 2;
  while (tiles * (n / t.ci) > kMaxReduceBlocks && t.ci * 2 <= n && n % (t.ci * 2) == 0) t.ci *= 2;
}

// Half-sweep tile: the widest column count (power of two, <= 64) dividing n/2, then the first
// compiled (tm, tj, cpt) shape whose rows divide n; chunks of >= 8 planes.
struct TileChoice {
  int tm, tj, cpt;
};
static const TileChoice kSweepPref[] = {{64, 8, 1}, {64, 4, 1}, {32, 16, 2}, {32, 8, 1}, {16, 32, 2},
                                        {16, 16, 1}, {8, 16, 1},  {8, 8, 1},   {4, 8, 1},   {4, 16, 2},
                                        {2, 4, 1},   {2, 8, 1}};

TileCfg sweep_tiles(int n) {
  TileCfg t;
  const int nh = n / 2;
  const int tm = pow2_divisor(nh, 64);
  t.tm = 0;
  for (const auto& c : kSweepPref) {
    if (c.tm == tm && n % c.tj == 0 && c.tj <= n && half_sweep_tile_supported(c.tm, c.tj, c.cpt)) {
      t.tm = c.tm;
      t.tj = c.tj;
      t.cpt = c.cpt;
      break;
    }
  }
  if (t.tm == 0) return t;  // unsupported: launch will fail with an invalid-value error
  t.tiles_j = n / t.tj;
  t.tiles_m = nh / t.tm;
  pick_chunk(t, n, false, 1024, 8);
  return t;
}

// Defect + restriction tile: even rows; a thread owns two rows, 256 threads.
TileCfg defect_tiles(int n) {
  TileCfg t;
  const int nh = n / 2;
  t.tm = pow2_divisor(nh, 64);
  if (t.tm < 2) t.tm = 2;
  t.tj = pow2_divisor(n, 512 / t.tm);
  if (t.tj < 2) t.tj = 2;
  t.tiles_j = n / t.tj;
  t.tiles_m = nh / t.tm;
  pick_chunk(t, n, true, 1024, 8);
  return t;
}

int Ctx::dev_alloc(double** p, size_t count) {
  hipError_t e = hipMalloc((void**)p, count * sizeof(double));
  if (e != hipSuccess) {
    *p = nullptr;
    return fail(MR_ENOMEM, "hipMalloc of %zu bytes failed: %s", count * sizeof(double), hipGetErrorString(e));
  }
  owned.push_back(*p);
  return MR_OK;
}

Reduce Ctx::reducer(int slot) { return Reduce{partials, counter, scal + slot}; }

int Ctx::read_scalars(int slot, int count, double* out) {
  if (count > kHostSlots - 16) return fail(MR_EINVAL, "read_scalars: too many values");
  hipError_t e = hipMemcpyAsync(host, scal + slot, count * sizeof(double), hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return hip_fail(e, "read back");
  for (int i = 0; i < count; ++i) out[i] = host[i];
  return MR_OK;
}

int Ctx::write_scalar(int slot, double v) {
  host[kHostSlots - 1] = v;
  hipError_t e = hipMemcpyAsync(scal + slot, host + kHostSlots - 1, sizeof(double), hipMemcpyHostToDevice, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return hip_fail(e, "write scalar");
  return MR_OK;
}

// ---- event timing of finest-mesh sweeps ----------------------------------------------------

int EventTimer::begin(hipStream_t s) {
  if (!on) return -1;
  if (next + 2 > pool.size()) {
    if (pool.size() >= 8192) return -1;  // drop samples beyond the pool
    for (int i = 0; i < 256; ++i) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return -1;
      pool.push_back(e);
    }
  }
  const int idx = (int)next;
  next += 2;
  if (hipEventRecord(pool[idx], s) != hipSuccess) return -1;
  return idx;
}

void EventTimer::end(int kind, int start, hipStream_t s) {
  if (start < 0) return;
  if (hipEventRecord(pool[start + 1], s) != hipSuccess) return;
  pending[kind].push_back({start, start + 1});
}

int EventTimer::resolve() {
  for (int k = 0; k < 2; ++k) {
    for (auto& pr : pending[k]) {
      if (hipEventSynchronize(pool[pr.second]) != hipSuccess) return MR_EHIP;
      float t = 0.0f;
      if (hipEventElapsedTime(&t, pool[pr.first], pool[pr.second]) != hipSuccess) return MR_EHIP;
      ms[k] += t;
      count[k] += 1;
    }
    pending[k].clear();
  }
  next = 0;
  return MR_OK;
}

void EventTimer::reset() {
  for (int k = 0; k < 2; ++k) {
    pending[k].clear();
    ms[k] = 0.0;
    count[k] = 0;
  }
  next = 0;
}

void EventTimer::destroy() {
  for (auto e : pool) (void)hipEventDestroy(e);
  pool.clear();
}

// ---- FP64 sweep / V-cycle on the level hierarchy --------------------------------------------

// The two per-colour launches of a sweep (or of one 4-class sub-sweep): colour 0 from the current
// iterate, colour 1 from the new colour-0 values and the old colour-1 values; both use the shift
// of the previous (sub-)sweep. The colour-0 sum goes to the staging slot, the colour-1 sum to slot
// [1]; the colour-1 launch then moves staging to [0]. filter0 / filter1: row filters of the two
// launches (0: every row).
static int colour_pair(Ctx& c, int l, const TileCfg& t, int filter0, int filter1) {
  Level& L = c.lv[l];
  double* cs = c.lsum(l);
  HalfSweepArgs a{};
  a.th_in = L.th[L.cur];
  a.th_red_new = nullptr;
  a.th_out = L.th[L.cur ^ 1];
  a.delta = L.delta;
  a.f = (l == 0) ? nullptr : L.f;
  a.n = L.n;
  a.colour = 0;
  a.h2 = L.h * L.h;
  a.ih2 = 1.0 / a.h2;
  a.c_sum = cs;
  a.c_scale = 1.0 / (double)L.cells;
  a.c_add = 0.0;
  a.sum_out = cs + 2;
  a.copy_from = nullptr;
  a.copy_to = nullptr;
  a.partials = c.partials;
  a.counter = c.counter;
  a.row_filter = filter0;
  hipError_t e = launch_half_sweep(a, t, c.stream);
  if (e != hipSuccess) return hip_fail(e, "colour-0 half-sweep");
  a.colour = 1;
  a.th_red_new = L.th[L.cur ^ 1];
  a.sum_out = cs + 1;
  a.copy_from = cs + 2;
  a.copy_to = cs + 0;
  a.row_filter = filter1;
  e = launch_half_sweep(a, t, c.stream);
  if (e != hipSuccess) return hip_fail(e, "colour-1 half-sweep");
  L.cur ^= 1;
  return MR_OK;
}

// Row filters of the two colour launches of 4-class sub-sweep cls. The class of cell (i, j, k) is
// 2 ((j + k) mod 2) + ((i + k) mod 2); with A = cls >> 1 and B = cls & 1 its cells of colour 0
// ((i + j + k) even) lie in the rows with (i, j) parity (A, B) and its cells of colour 1 in the
// rows with parity (1 - A, 1 - B), one colour row each.
static void class_filters(int cls, int& filter0, int& filter1) {
  const int A = cls >> 1, B = cls & 1;
  filter0 = 4 + 2 * A + B;
  filter1 = 4 + 2 * (A ^ 1) + (B ^ 1);
}

// One sweep on level l: the fused red-black launch, the two per-colour launches, or (with
// MR_FLAG_ORDER4) four class sub-sweeps of two row-filtered tiled launches each.
int Ctx::sweep(int l) {
  Level& L = lv[l];
  double* cs = lsum(l);
  const bool order4 = (opts.flags & MR_FLAG_ORDER4) != 0;
  if (!order4 && L.has_fz && !(opts.flags & MR_FLAG_TWO_PASS)) {
    FusedSweepArgs a{};
    a.th_in = L.th[L.cur];
    a.th_out = L.th[L.cur ^ 1];
    a.delta = L.delta;
    a.f = (l == 0) ? nullptr : L.f;
    a.n = L.n;
    a.h2 = L.h * L.h;
    a.ih2 = 1.0 / a.h2;
    a.c_sum = cs;
    a.c_scale = 1.0 / (double)L.cells;
    a.c_add = 0.0;
    a.sum_out = cs;   // red sum, black sum: the shift of the next sweep
    a.partials = partials;
    a.counter = counter;
    const int ev = (l == 0) ? timer.begin(stream) : -1;
    hipError_t e = launch_sweep_fused(a, L.fz, stream);
    if (e != hipSuccess) return hip_fail(e, "fused sweep");
    timer.end(0, ev, stream);
    L.cur ^= 1;
    return MR_OK;
  }
  const int ev = (l == 0) ? timer.begin(stream) : -1;
  int rc = MR_OK;
  if (!order4) {
    rc = colour_pair(*this, l, L.sw, 0, 0);
  } else {
    const TileCfg t = sweep_tiles(L.n);
    for (int cls = 0; cls < 4 && rc == MR_OK; ++cls) {
      int f0, f1;
      class_filters(cls, f0, f1);
      rc = colour_pair(*this, l, t, f0, f1);
    }
  }
  if (rc != MR_OK) return rc;
  timer.end(0, ev, stream);
  return MR_OK;
}

// Pre-relaxation on level l, then the fused defect + restriction onto level l+1 (theta_c into
// the coarse iterate and the saved copy, R d into the coarse f). norm_sums (device, 2 values)
// receives sum d and sum d^2 of level l when given.
int Ctx::down(int l, double* norm_sums) {
  int rc;
  for (int s = 0; s < opts.npre; ++s)
    if ((rc = sweep(l)) != MR_OK) return rc;
  Level& L = lv[l];
  Level& Lc = lv[l + 1];
  DefectArgs a{};
  a.theta = L.th[L.cur];
  a.delta = L.delta;
  a.f = (l == 0) ? nullptr : L.f;
  a.n = L.n;
  a.ih2 = 1.0 / (L.h * L.h);
  a.c_sum = lsum(l);
  a.c_scale = 1.0 / (double)L.cells;
  a.c_add = 0.0;
  a.theta_c = Lc.th[Lc.cur];
  a.theta_c2 = Lc.that;
  a.dr = Lc.f;
  a.sums_out = norm_sums ? norm_sums : scal + kSlotAux + 14;
  a.partials = partials;
  a.counter = counter;
  hipError_t e = launch_defect_restrict_tiled(a, L.df, stream);
  return e == hipSuccess ? MR_OK : hip_fail(e, "defect_restrict");
}

// Coarse-grid correction of level l from level l+1 and post-relaxation on level l.
int Ctx::up(int l) {
  Level& L = lv[l];
  Level& Lc = lv[l + 1];
  hipError_t e = launch_tau(Lc.that, Lc.delta, Lc.f, Lc.f, Lc.n, Lc.h, reducer(kSlotLevel + 3 * (l + 1)), stream);
  if (e != hipSuccess) return hip_fail(e, "tau");
  int rc;
  if ((rc = vcycle(l + 1)) != MR_OK) return rc;
  e = launch_prolong_correct(Lc.th[Lc.cur], Lc.that, L.th[L.cur], L.n, stream);
  if (e != hipSuccess) return hip_fail(e, "prolong_correct");
  for (int s = 0; s < opts.npost; ++s)
    if ((rc = sweep(l)) != MR_OK) return rc;
  return MR_OK;
}

int Ctx::vcycle(int l) {
  Level& L = lv[l];
  if (l == nlev - 1) {
    CoarsestArgs a{};
    a.theta = L.th[L.cur];
    a.delta = L.delta;
    a.f = (l == 0) ? nullptr : L.f;
    a.n = L.n;
    a.nsweeps = opts.ncoarse;
    a.h2 = L.h * L.h;
    a.ih2 = 1.0 / a.h2;
    a.c_sum = lsum(l);
    a.c_scale = 1.0 / (double)L.cells;
    a.c_sum_out = lsum(l);
    hipError_t e = launch_coarsest(a, stream);
    return e == hipSuccess ? MR_OK : hip_fail(e, "coarsest");
  }
  int rc;
  if ((rc = down(l, nullptr)) != MR_OK) return rc;
  return up(l);
}

// Residual of the finest level with a given shift: b = nabla^2 theta - Sigma + shift;
// ||r|| = sqrt(sum b^2 - (sum b)^2 / N^3) is the norm of the mean-projected residual and
// <Sigma> = shift - <b>.
int Ctx::finest_norm(const double* theta_split, ShiftRef sh, double* nrm, double* msig) {
  Level& L = lv[0];
  hipError_t e = launch_residual(theta_split, L.delta, L.n, 1.0, sh, nullptr, reducer(kSlotRes), stream);
  if (e != hipSuccess) return hip_fail(e, "residual");
  double r[kSlotRes + 2];
  int rc = read_scalars(0, kSlotRes + 2, r);
  if (rc != MR_OK) return rc;
  const double N3 = (double)L.cells;
  const double var = r[kSlotRes + 1] - r[kSlotRes] * r[kSlotRes] / N3;
  *nrm = std::sqrt(var > 0.0 ? var : 0.0);
  const double shv = (sh.c_sum ? (r[sh.c_sum - scal] + r[sh.c_sum - scal + 1]) * sh.c_scale : 0.0) + sh.c_add;
  *msig = shv - r[kSlotRes] / N3;
  return MR_OK;
}

// Validate delta, convert it to the colour-split layout and build its hierarchy.
int Ctx::prepare(const double* delta) {
  Level& L0 = lv[0];
  hipError_t e = launch_validate(delta, L0.cells, reducer(kSlotRes), stream);
  if (e != hipSuccess) return hip_fail(e, "validate");
  double bad;
  int rc = read_scalars(kSlotRes, 1, &bad);
  if (rc != MR_OK) return rc;
  if (bad != 0.0) return fail(MR_EDOMAIN, "delta has %.0f cells with a non-finite value or 1 + delta <= 0", bad);
  e = launch_to_split(delta, L0.delta, L0.n, stream);
  if (e != hipSuccess) return hip_fail(e, "to_split");
  for (int l = 1; l < nlev; ++l) {
    e = launch_restrict(lv[l - 1].delta, lv[l].delta, lv[l - 1].n, stream);
    if (e != hipSuccess) return hip_fail(e, "restrict delta");
  }
  return MR_OK;
}

int Ctx::solve_fp64(const double* delta, double* theta, mr_info* info, int aa_depth) {
  auto t0 = std::chrono::steady_clock::now();
  int rc = prepare(delta);
  if (rc != MR_OK) return rc;
  if (aa_depth > 0 && (rc = aa_reserve(aa_depth)) != MR_OK) return rc;
  AAState aa(aa_depth, aa_depth + 1);
  Level& L0 = lv[0];
  const double N3 = (double)L0.cells;
  hipError_t e;
  L0.cur = 0;
  if (opts.warm_start) e = launch_to_split(theta, L0.th[0], L0.n, stream);
  else e = hipMemsetAsync(L0.th[0], 0, L0.cells * sizeof(double), stream);
  if (e != hipSuccess) return hip_fail(e, "initial theta");
  double r0, m0, nrm, msig;
  if ((rc = finest_norm(nullptr, ShiftRef{nullptr, 0.0, 0.0}, &r0, &m0)) != MR_OK) return rc;
  if (opts.warm_start) {
    if ((rc = finest_norm(L0.th[0], ShiftRef{nullptr, 0.0, 0.0}, &nrm, &msig)) != MR_OK) return rc;
  } else {
    nrm = r0;
    msig = m0;
  }
  if (r0 == 0.0) r0 = 1.0;
  // Running sums of the finest level, so that the first sweep uses the exact <Sigma>.
  if ((rc = write_scalar(kSlotLevel + 0, msig * N3)) != MR_OK) return rc;
  if ((rc = write_scalar(kSlotLevel + 1, 0.0)) != MR_OK) return rc;
  double rel = nrm / r0;
  mr_info loc{};
  loc.r0_norm = r0;
  loc.history[0] = rel;
  int cyc = 0;
  int status = MR_OK;
  double best = rel;
  // Each cycle: pre-relaxation, then the defect pass, whose sums give the residual norm of the
  // current iterate (convergence test); if not converged, coarse correction and post-relaxation.
  while (rel > opts.tol && cyc < opts.max_cycles) {
    if (aa_depth > 0 && aa.steps == 0) {   // later cycles start from a state aa_step keeps
      e = aa_save(*this, L0.th[L0.cur]);
      if (e != hipSuccess) return hip_fail(e, "Anderson save");
    }
    if ((rc = down(0, scal + kSlotRes)) != MR_OK) return rc;
    double r[kSlotRes + 2];
    if ((rc = read_scalars(0, kSlotRes + 2, r)) != MR_OK) return rc;
    const double var = r[kSlotRes + 1] - r[kSlotRes] * r[kSlotRes] / N3;
    nrm = std::sqrt(var > 0.0 ? var : 0.0);
    msig = (r[0] + r[1]) / N3 - r[kSlotRes] / N3;
    rel = nrm / r0;
    ++cyc;
    if (cyc < 128) loc.history[cyc] = rel;
    if (!std::isfinite(rel) || rel > 1e6 * (best > 1.0 ? best : 1.0)) {
      status = fail(MR_EDIVERGED, "residual diverged at cycle %d (%g)", cyc, rel);
      break;
    }
    if (rel < best) best = rel;
    if (rel <= opts.tol || cyc >= opts.max_cycles) break;
    if ((rc = up(0)) != MR_OK) return rc;
    if (aa_depth > 0 && (rc = aa_step(aa, L0.th[L0.cur])) != MR_OK) return rc;
  }
  if (status == MR_OK && rel > opts.tol) {
    status = MR_NOT_CONVERGED;
    fail(MR_NOT_CONVERGED, "not converged after %d cycles (rel residual %g)", cyc, rel);
  }
  // Gauge <theta> = 0, result into the caller's buffer in natural order.
  e = launch_sum(L0.th[L0.cur], L0.cells, reducer(kSlotGauge), stream);
  if (e == hipSuccess) e = launch_from_split(L0.th[L0.cur], theta, L0.n, scal + kSlotGauge, 1.0 / N3, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return hip_fail(e, "gauge");
  loc.status = status;
  loc.cycles = cyc;
  loc.rel_residual = rel;
  loc.m_shift = msig;
  loc.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (info) *info = loc;
  return status;
}

}  // namespace mr

using namespace mr;

namespace {

// Device temporaries for the building-block entry points (freed on scope exit).
struct Temps {
  std::vector<void*> ptrs;
  hipStream_t s;
  explicit Temps(hipStream_t st) : s(st) {}
  double* get(size_t count) {
    void* p = nullptr;
    if (hipMalloc(&p, count * sizeof(double)) != hipSuccess) return nullptr;
    ptrs.push_back(p);
    return (double*)p;
  }
  ~Temps() {
    if (s) (void)hipStreamSynchronize(s);
    else (void)hipDeviceSynchronize();
    for (void* p : ptrs) (void)hipFree(p);
  }
};

}  // namespace

extern "C" {

void mr_default_opts(mr_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof *o);
  o->tol = 1e-10;
  o->max_cycles = 100;
  o->npre = 2;
  o->npost = 2;
  o->ncoarse = 20;
  o->precision = MR_PREC_FP64;
  o->inner_cycles = 1;
  o->warm_start = 0;
}

const char* mr_last_error(void) { return g_err.c_str(); }

int mr_create(mr_ctx** out, int n, const mr_opts* opts, void* hip_stream) {
  if (!out) return fail(MR_EINVAL, "mr_create: null out");
  *out = nullptr;
  int rc = check_size(n);
  if (rc != MR_OK) return rc;
  mr_opts o;
  mr_default_opts(&o);
  if (opts) o = *opts;
  if ((rc = check_opts(o)) != MR_OK) return rc;
  Ctx* c = new Ctx();
  c->n = n;
  c->opts = o;
  c->stream = (hipStream_t)hip_stream;
  (void)hipGetDevice(&c->device);
  const auto sizes = level_sizes(n);
  c->nlev = (int)sizes.size();
  c->lv.resize(sizes.size());
  for (size_t l = 0; l < sizes.size(); ++l) {
    Level& L = c->lv[l];
    L.n = sizes[l];
    L.cells = (size_t)L.n * L.n * L.n;
    L.h = std::ldexp(1.0, (int)l);
    if ((int)l < c->nlev - 1) {
      L.sw = sweep_tiles(L.n);
      L.df = defect_tiles(L.n);
    }
    if ((rc = c->dev_alloc(&L.th[0], L.cells)) != MR_OK || (rc = c->dev_alloc(&L.th[1], L.cells)) != MR_OK ||
        (rc = c->dev_alloc(&L.delta, L.cells)) != MR_OK) {
      mr_destroy(reinterpret_cast<mr_ctx*>(c));
      return rc;
    }
    if (l == 0) continue;
    if ((rc = c->dev_alloc(&L.that, L.cells)) != MR_OK || (rc = c->dev_alloc(&L.f, L.cells)) != MR_OK) {
      mr_destroy(reinterpret_cast<mr_ctx*>(c));
      return rc;
    }
  }
  if ((rc = c->dev_alloc(&c->scal, kSlotCount)) != MR_OK ||
      (rc = c->dev_alloc(&c->partials, (size_t)kMaxReduceBlocks * kMaxNV)) != MR_OK) {
    mr_destroy(reinterpret_cast<mr_ctx*>(c));
    return rc;
  }
  hipError_t e = hipMalloc((void**)&c->counter, 64 * sizeof(unsigned));
  if (e == hipSuccess) c->owned.push_back(c->counter);
  if (e == hipSuccess) e = hipMemset(c->counter, 0, 64 * sizeof(unsigned));
  if (e == hipSuccess) e = hipMemset(c->scal, 0, kSlotCount * sizeof(double));
  if (e == hipSuccess) e = hipHostMalloc((void**)&c->host, kHostSlots * sizeof(double), hipHostMallocDefault);
  if (e != hipSuccess) {
    rc = hip_fail(e, "mr_create");
    mr_destroy(reinterpret_cast<mr_ctx*>(c));
    return rc;
  }
  // Relaxation schedule per level: the fused red-black launch or the two per-colour launches,
  // whichever is faster on this device (timed on the level's own buffers before any use).
  if (!(o.flags & MR_FLAG_TWO_PASS)) {
    for (int l = 0; l < c->nlev - 1; ++l) {
      Level& L = c->lv[l];
      rc = tune_sweep(L.n, L.th[0], L.th[1], L.delta, c->partials, c->counter, c->scal + kSlotAux, &L.sw, c->stream,
                      &L.has_fz, &L.fz);
      // defect + restriction of the level, on the synthetic state the sweep tuner left in th[0]
      // and delta (f zeroed on coarse levels; outputs into the coarse level's buffers)
      Level& Lc = c->lv[l + 1];
      if (rc == MR_OK && l > 0 && hipMemsetAsync(L.f, 0, L.cells * sizeof(double), c->stream) != hipSuccess)
        rc = hip_fail(hipErrorInvalidValue, "mr_create");
      if (rc == MR_OK) {
        DefectArgs a{};
        a.theta = L.th[0];
        a.delta = L.delta;
        a.f = (l == 0) ? nullptr : L.f;
        a.n = L.n;
        a.ih2 = 1.0;
        a.theta_c = Lc.th[0];
        a.dr = Lc.th[1];
        a.sums_out = c->scal + kSlotAux;
        a.partials = c->partials;
        a.counter = c->counter;
        rc = tune_defect(a, c->stream);
      }
      if (rc != MR_OK) {
        mr_destroy(reinterpret_cast<mr_ctx*>(c));
        return rc;
      }
    }
    if ((e = hipMemsetAsync(c->scal, 0, kSlotCount * sizeof(double), c->stream)) == hipSuccess)
      e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
      rc = hip_fail(e, "mr_create");
      mr_destroy(reinterpret_cast<mr_ctx*>(c));
      return rc;
    }
  }
  *out = reinterpret_cast<mr_ctx*>(c);
  return MR_OK;
}

void mr_destroy(mr_ctx* h) {
  if (!h) return;
  Ctx* c = reinterpret_cast<Ctx*>(h);
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  else (void)hipDeviceSynchronize();
  c->release_extra();
  c->timer.destroy();
  for (void* p : c->owned) (void)hipFree(p);
  if (c->host) (void)hipHostFree(c->host);
  delete c;
}

int mr_set_opts(mr_ctx* h, const mr_opts* opts) {
  if (!h || !opts) return fail(MR_EINVAL, "mr_set_opts: null argument");
  int rc = check_opts(*opts);
  if (rc != MR_OK) return rc;
  reinterpret_cast<Ctx*>(h)->opts = *opts;
  return MR_OK;
}

int mr_size(const mr_ctx* h) { return h ? reinterpret_cast<const Ctx*>(h)->n : 0; }
int mr_levels(const mr_ctx* h) { return h ? reinterpret_cast<const Ctx*>(h)->nlev : 0; }

int mr_get_schedule(const mr_ctx* h, int level, int sched[4]) {
  if (!h || !sched) return fail(MR_EINVAL, "mr_get_schedule: null argument");
  const Ctx* c = reinterpret_cast<const Ctx*>(h);
  if (level < 0 || level >= c->nlev - 1) return fail(MR_EINVAL, "mr_get_schedule: level %d has no sweep schedule", level);
  const Level& L = c->lv[level];
  const bool fused = L.has_fz && !(c->opts.flags & MR_FLAG_TWO_PASS);
  if (fused) {
    sched[0] = MR_SCHED_FUSED;
    sched[1] = L.fz.tm;
    sched[2] = L.fz.tj;
    sched[3] = L.fz.nchunks;
  } else {
    sched[0] = L.sw.pipe ? MR_SCHED_PIPELINED : MR_SCHED_TILED;
    sched[1] = L.sw.tm;
    sched[2] = L.sw.tj;
    sched[3] = L.n / L.sw.ci;
  }
  return MR_OK;
}

int mr_get_lin_schedule(mr_ctx* h, int level, int sched[4]) {
  if (!h || !sched) return fail(MR_EINVAL, "mr_get_lin_schedule: null argument");
  Ctx* c = reinterpret_cast<Ctx*>(h);
  if (level < 0 || level >= c->nlev - 1)
    return fail(MR_EINVAL, "mr_get_lin_schedule: level %d has no sweep schedule", level);
  return c->lin_schedule(level, sched);
}

int mr_set_schedule(mr_ctx* h, int level, const int sched[4]) {
  if (!h || !sched) return fail(MR_EINVAL, "mr_set_schedule: null argument");
  Ctx* c = reinterpret_cast<Ctx*>(h);
  if (level < 0 || level >= c->nlev - 1) return fail(MR_EINVAL, "mr_set_schedule: level %d has no sweep schedule", level);
  Level& L = c->lv[level];
  const int n = L.n, nh = n / 2, kind = sched[0], tm = sched[1], tj = sched[2], nch = sched[3];
  // the fused launch splits the planes into nch nearly equal chunks; the two-launch kernels need equal ones
  if (tm < 1 || tj < 1 || nh % tm != 0 || n % tj != 0 || nch < 1 || (kind != MR_SCHED_FUSED && n % nch != 0) ||
      n / nch < 4 || (long)(nh / tm) * (n / tj) * nch > kMaxReduceBlocks)
    return fail(MR_EINVAL, "mr_set_schedule: tile %d x %d, %d chunks do not fit the %d^3 level", tm, tj, nch, n);
  if (kind == MR_SCHED_FUSED) {
    if (!fused_tile_supported(tm, tj)) return fail(MR_EINVAL, "mr_set_schedule: no fused kernel for tile %d x %d", tm, tj);
    L.fz.tm = tm;
    L.fz.tj = tj;
    L.fz.tiles_j = n / tj;
    L.fz.tiles_m = nh / tm;
    L.fz.nchunks = nch;
    L.has_fz = true;
    return MR_OK;
  }
  TileCfg t;
  t.tm = tm;
  t.tj = tj;
  t.cpt = 1;
  t.ci = n / nch;
  t.tiles_j = n / tj;
  t.tiles_m = nh / tm;
  if (kind == MR_SCHED_PIPELINED) {
    if (!half_sweep_pipe_supported(tm, tj) || t.ci % 4 != 0)
      return fail(MR_EINVAL, "mr_set_schedule: no pipelined kernel for tile %d x %d, %d-plane chunks", tm, tj, t.ci);
    t.pipe = true;
  } else if (kind == MR_SCHED_TILED) {
    // the general kernel is compiled with 1, 2 or 4 cells per thread and plane depending on the tile
    t.cpt = 0;
    for (int cpt : {1, 2, 4})
      if (t.cpt == 0 && half_sweep_tile_supported(tm, tj, cpt)) t.cpt = cpt;
    if (t.cpt == 0) return fail(MR_EINVAL, "mr_set_schedule: no tiled kernel for tile %d x %d", tm, tj);
  } else {
    return fail(MR_EINVAL, "mr_set_schedule: unknown kind %d", kind);
  }
  L.sw = t;
  L.has_fz = false;
  return MR_OK;
}

int mr_schedule_candidates(const mr_ctx* h, int level, int* sched, int max_count) {
  if (!h || (!sched && max_count > 0) || max_count < 0) return fail(MR_EINVAL, "mr_schedule_candidates: bad argument");
  const Ctx* c = reinterpret_cast<const Ctx*>(h);
  if (level < 0 || level >= c->nlev - 1)
    return fail(MR_EINVAL, "mr_schedule_candidates: level %d has no sweep schedule", level);
  const int n = c->lv[level].n;
  const std::vector<SweepCand> all = sweep_candidates(n, sweep_tiles(n));
  int k = 0;
  for (const SweepCand& x : all) {
    if (k < max_count) {
      int* o = sched + 4 * k;
      if (x.fused) {
        o[0] = MR_SCHED_FUSED;
        o[1] = x.fz.tm;
        o[2] = x.fz.tj;
        o[3] = x.fz.nchunks;
      } else {
        o[0] = x.two.pipe ? MR_SCHED_PIPELINED : MR_SCHED_TILED;
        o[1] = x.two.tm;
        o[2] = x.two.tj;
        o[3] = n / x.two.ci;
      }
    }
    ++k;
  }
  return k;
}

int mr_timing_enable(mr_ctx* h, int on) {
  if (!h) return fail(MR_EINVAL, "mr_timing_enable: null context");
  Ctx* c = reinterpret_cast<Ctx*>(h);
  hipError_t e = c->stream ? hipStreamSynchronize(c->stream) : hipDeviceSynchronize();
  if (e != hipSuccess) return hip_fail(e, "mr_timing_enable");
  c->timer.reset();
  c->timer.on = on != 0;
  return MR_OK;
}

int mr_timing_read(mr_ctx* h, mr_timing* out) {
  if (!h || !out) return fail(MR_EINVAL, "mr_timing_read: null argument");
  Ctx* c = reinterpret_cast<Ctx*>(h);
  hipError_t e = c->stream ? hipStreamSynchronize(c->stream) : hipDeviceSynchronize();
  if (e != hipSuccess) return hip_fail(e, "mr_timing_read");
  if (c->timer.resolve() != MR_OK) return fail(MR_EHIP, "mr_timing_read: event query failed");
  out->sweep64_ms = c->timer.ms[0];
  out->sweep64_launches = c->timer.count[0];
  out->sweep32_ms = c->timer.ms[1];
  out->sweep32_launches = c->timer.count[1];
  out->finest_cells = (int64_t)c->lv[0].cells;
  return MR_OK;
}

int mr_residual(mr_ctx* h, const double* delta, const double* theta, double* r_out, double* rel_out,
                double* msum_out) {
  if (!h || !delta || !theta) return fail(MR_EINVAL, "mr_residual: null argument");
  Ctx* c = reinterpret_cast<Ctx*>(h);
  Level& L0 = c->lv[0];
  hipError_t e = launch_to_split(delta, L0.delta, L0.n, c->stream);
  if (e == hipSuccess) e = launch_to_split(theta, L0.th[1], L0.n, c->stream);
  if (e != hipSuccess) return hip_fail(e, "mr_residual");
  int rc;
  double r0, m0, n1, m1;
  if ((rc = c->finest_norm(nullptr, ShiftRef{nullptr, 0.0, 0.0}, &r0, &m0)) != MR_OK) return rc;
  if ((rc = c->finest_norm(L0.th[1], ShiftRef{nullptr, 0.0, 0.0}, &n1, &m1)) != MR_OK) return rc;
  // second pass with the mean of Sigma, writing r in natural order
  e = launch_residual(L0.th[1], L0.delta, L0.n, 1.0, ShiftRef{nullptr, 0.0, m1}, r_out, c->reducer(kSlotRes),
                      c->stream);
  if (e != hipSuccess) return hip_fail(e, "residual");
  double r[2];
  if ((rc = c->read_scalars(kSlotRes, 2, r)) != MR_OK) return rc;
  const double var = r[1] - r[0] * r[0] / (double)L0.cells;
  const double n2 = std::sqrt(var > 0 ? var : 0.0);
  if (rel_out) *rel_out = (r0 > 0.0) ? n2 / r0 : n2;
  if (msum_out) *msum_out = m1;
  return MR_OK;
}

int mr_solve_anderson(mr_ctx* h, const double* delta, double* theta, int depth, mr_info* info) {
  if (!h || !delta || !theta) return fail(MR_EINVAL, "mr_solve_anderson: null argument");
  if (depth < 1 || depth > kAAMaxDepth) return fail(MR_EINVAL, "mr_solve_anderson: depth %d not in 1..%d", depth, kAAMaxDepth);
  Ctx* c = reinterpret_cast<Ctx*>(h);
  if (c->opts.precision == MR_PREC_MIXED) return c->solve_mixed(delta, theta, info, depth);
  return c->solve_fp64(delta, theta, info, depth);
}

int mr_solve(mr_ctx* h, const double* delta, double* theta, mr_info* info) {
  if (!h || !delta || !theta) return fail(MR_EINVAL, "mr_solve: null argument");
  Ctx* c = reinterpret_cast<Ctx*>(h);
  if (c->opts.precision == MR_PREC_MIXED) return c->solve_mixed(delta, theta, info);
  return c->solve_fp64(delta, theta, info);
}

// ---- building blocks (natural-order arguments; temporaries allocated per call) -------------

static int check_level(int nl, bool coarsen) {
  if (nl < 4 || nl % 2 != 0 || nl > 1024) return fail(MR_EINVAL, "level size %d not supported", nl);
  if (coarsen && nl % 4 != 0) return fail(MR_EINVAL, "level size %d: must be a multiple of 4", nl);
  return MR_OK;
}

int mr_sweep(mr_ctx* h, int nl, double hcell, const double* delta, const double* f, double cshift,
             const double* theta_in, double* theta_out, double* sum_out) {
  if (!h || !delta || !theta_in || !theta_out || theta_in == theta_out)
    return fail(MR_EINVAL, "mr_sweep: bad pointers");
  int rc = check_level(nl, true);
  if (rc != MR_OK) return rc;
  Ctx* c = reinterpret_cast<Ctx*>(h);
  const size_t cells = (size_t)nl * nl * nl;
  Temps tmp(c->stream);
  double *ds = tmp.get(cells), *fs = f ? tmp.get(cells) : nullptr, *tin = tmp.get(cells), *tout = tmp.get(cells);
  if (!ds || !tin || !tout || (f && !fs)) return fail(MR_ENOMEM, "mr_sweep: temporaries");
  hipError_t e = launch_to_split(delta, ds, nl, c->stream);
  if (e == hipSuccess && f) e = launch_to_split(f, fs, nl, c->stream);
  if (e == hipSuccess) e = launch_to_split(theta_in, tin, nl, c->stream);
  if (e != hipSuccess) return hip_fail(e, "mr_sweep");
  FusedCfg fz;
  const bool order4 = (c->opts.flags & MR_FLAG_ORDER4) != 0;
  const bool two_pass = (c->opts.flags & MR_FLAG_TWO_PASS) != 0;
  // a mesh size that is a relaxed level of this context runs that level's schedule
  const Level* lev = nullptr;
  for (int l = 0; l + 1 < c->nlev; ++l)
    if (c->lv[l].n == nl) lev = &c->lv[l];
  double* final_out = tout;
  bool use_fused = false;
  TileCfg two;
  if (lev) {
    use_fused = lev->has_fz && !two_pass;
    fz = lev->fz;
    two = lev->sw;
  } else {
    use_fused = !two_pass && (tuned_sweep(nl, &fz) || pick_fused(nl, fz));
    two = sweep_tiles(nl);
    two.pipe = two.cpt == 1 && two.ci % 4 == 0 && half_sweep_pipe_supported(two.tm, two.tj);
  }
  if (order4) {
    // four class sub-sweeps, each two row-filtered tiled launches, ping-ponging tin and tout
    const TileCfg t = sweep_tiles(nl);
    double* bufs[2] = {tin, tout};
    for (int cls = 0; cls < 4 && e == hipSuccess; ++cls) {
      int f0, f1;
      class_filters(cls, f0, f1);
      HalfSweepArgs a{};
      a.th_in = bufs[cls & 1];
      a.th_out = bufs[(cls & 1) ^ 1];
      a.delta = ds;
      a.f = fs;
      a.n = nl;
      a.h2 = hcell * hcell;
      a.ih2 = 1.0 / a.h2;
      a.c_add = cshift;
      a.partials = c->partials;
      a.counter = c->counter;
      a.colour = 0;
      a.row_filter = f0;
      a.sum_out = c->scal + kSlotAux + 0;
      e = launch_half_sweep(a, t, c->stream);
      a.colour = 1;
      a.row_filter = f1;
      a.th_red_new = a.th_out;
      a.sum_out = c->scal + kSlotAux + 1;
      if (e == hipSuccess) e = launch_half_sweep(a, t, c->stream);
    }
    final_out = bufs[0];   // four sub-sweeps: the last one wrote back into the first buffer
  } else if (use_fused) {
    FusedSweepArgs a{};
    a.th_in = tin;
    a.th_out = tout;
    a.delta = ds;
    a.f = fs;
    a.n = nl;
    a.h2 = hcell * hcell;
    a.ih2 = 1.0 / a.h2;
    a.c_add = cshift;
    a.sum_out = c->scal + kSlotAux;
    a.partials = c->partials;
    a.counter = c->counter;
    if (e == hipSuccess) e = launch_sweep_fused(a, fz, c->stream);
  } else {
    const TileCfg& t = two;
    HalfSweepArgs a{};
    a.th_in = tin;
    a.th_out = tout;
    a.delta = ds;
    a.f = fs;
    a.n = nl;
    a.h2 = hcell * hcell;
    a.ih2 = 1.0 / a.h2;
    a.c_add = cshift;
    a.partials = c->partials;
    a.counter = c->counter;
    a.colour = 0;
    a.sum_out = c->scal + kSlotAux + 0;
    if (e == hipSuccess) e = launch_half_sweep(a, t, c->stream);
    a.colour = 1;
    a.th_red_new = tout;
    a.sum_out = c->scal + kSlotAux + 1;
    if (e == hipSuccess) e = launch_half_sweep(a, t, c->stream);
  }
  if (e == hipSuccess) e = launch_from_split(final_out, theta_out, nl, nullptr, 0.0, c->stream);
  if (e != hipSuccess) return hip_fail(e, "mr_sweep");
  double s[2];
  if ((rc = c->read_scalars(kSlotAux, 2, s)) != MR_OK) return rc;
  if (sum_out) *sum_out = s[0] + s[1];
  return MR_OK;
}

int mr_defect_restrict(mr_ctx* h, int nl, double hcell, const double* delta, const double* f,
                       double cshift, const double* theta, double* theta_c, double* dr_c) {
  if (!h || !delta || !theta || !theta_c || !dr_c) return fail(MR_EINVAL, "mr_defect_restrict: null argument");
  int rc = check_level(nl, true);
  if (rc != MR_OK) return rc;
  Ctx* c = reinterpret_cast<Ctx*>(h);
  const size_t cells = (size_t)nl * nl * nl, cc = cells / 8;
  Temps tmp(c->stream);
  double *ds = tmp.get(cells), *fs = f ? tmp.get(cells) : nullptr, *ts = tmp.get(cells), *tcs = tmp.get(cc),
         *drs = tmp.get(cc);
  if (!ds || !ts || !tcs || !drs || (f && !fs)) return fail(MR_ENOMEM, "mr_defect_restrict: temporaries");
  hipError_t e = launch_to_split(delta, ds, nl, c->stream);
  if (e == hipSuccess && f) e = launch_to_split(f, fs, nl, c->stream);
  if (e == hipSuccess) e = launch_to_split(theta, ts, nl, c->stream);
  DefectArgs a{};
  a.theta = ts;
  a.delta = ds;
  a.f = fs;
  a.n = nl;
  a.ih2 = 1.0 / (hcell * hcell);
  a.c_add = cshift;
  a.theta_c = tcs;
  a.dr = drs;
  a.sums_out = c->scal + kSlotAux;
  a.partials = c->partials;
  a.counter = c->counter;
  if (e == hipSuccess) e = launch_defect_restrict_tiled(a, defect_tiles(nl), c->stream);
  if (e == hipSuccess) e = launch_from_split(tcs, theta_c, nl / 2, nullptr, 0.0, c->stream);
  if (e == hipSuccess) e = launch_from_split(drs, dr_c, nl / 2, nullptr, 0.0, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  return e == hipSuccess ? MR_OK : hip_fail(e, "mr_defect_restrict");
}

int mr_tau_rhs(mr_ctx* h, int nl, double hcell, const double* delta, const double* theta_hat,
               const double* rd, double* f_out, double* sum_out) {
  if (!h || !delta || !theta_hat || !rd || !f_out) return fail(MR_EINVAL, "mr_tau_rhs: null argument");
  int rc = check_level(nl, false);
  if (rc != MR_OK) return rc;
  Ctx* c = reinterpret_cast<Ctx*>(h);
  const size_t cells = (size_t)nl * nl * nl;
  Temps tmp(c->stream);
  double *ds = tmp.get(cells), *ts = tmp.get(cells), *rs = tmp.get(cells);
  if (!ds || !ts || !rs) return fail(MR_ENOMEM, "mr_tau_rhs: temporaries");
  hipError_t e = launch_to_split(delta, ds, nl, c->stream);
  if (e == hipSuccess) e = launch_to_split(theta_hat, ts, nl, c->stream);
  if (e == hipSuccess) e = launch_to_split(rd, rs, nl, c->stream);
  if (e == hipSuccess) e = launch_tau(ts, ds, rs, rs, nl, hcell, c->reducer(kSlotAux), c->stream);
  if (e == hipSuccess) e = launch_from_split(rs, f_out, nl, nullptr, 0.0, c->stream);
  if (e != hipSuccess) return hip_fail(e, "mr_tau_rhs");
  double s;
  if ((rc = c->read_scalars(kSlotAux, 1, &s)) != MR_OK) return rc;
  if (sum_out) *sum_out = s;
  return MR_OK;
}

int mr_prolong_correct(mr_ctx* h, int nl, const double* theta_c, const double* theta_hat_c, double* theta) {
  if (!h || !theta_c || !theta_hat_c || !theta) return fail(MR_EINVAL, "mr_prolong_correct: null argument");
  int rc = check_level(nl, true);
  if (rc != MR_OK) return rc;
  Ctx* c = reinterpret_cast<Ctx*>(h);
  const size_t cells = (size_t)nl * nl * nl, cc = cells / 8;
  Temps tmp(c->stream);
  double *a = tmp.get(cc), *b = tmp.get(cc), *t = tmp.get(cells);
  if (!a || !b || !t) return fail(MR_ENOMEM, "mr_prolong_correct: temporaries");
  hipError_t e = launch_to_split(theta_c, a, nl / 2, c->stream);
  if (e == hipSuccess) e = launch_to_split(theta_hat_c, b, nl / 2, c->stream);
  if (e == hipSuccess) e = launch_to_split(theta, t, nl, c->stream);
  if (e == hipSuccess) e = launch_prolong_correct(a, b, t, nl, c->stream);
  if (e == hipSuccess) e = launch_from_split(t, theta, nl, nullptr, 0.0, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  return e == hipSuccess ? MR_OK : hip_fail(e, "mr_prolong_correct");
}

// Inputs of the linear building blocks on an nl^3 mesh: delta, base potential, e and rhs (rhs NULL:
// zero) converted to colour-split FP32 where the inner solve keeps them, and the base root at
// cell size h from the FP32 base (as on the coarse levels of the inner solve).
namespace {
struct LinInputs {
  double* ds = nullptr;
  int* base = nullptr;
  const double* bq = nullptr;
  float *sb = nullptr, *e = nullptr, *rhs = nullptr;
};
}  // namespace

static int lin_inputs(Ctx* c, Temps& tmp, int nl, double hcell, const double* delta, const double* theta_base,
                      const double* e, const double* rhs, LinInputs& in) {
  const size_t cells = (size_t)nl * nl * nl, fw = (cells + 1) / 2;   // doubles holding cells floats
  double* t64 = tmp.get(cells);
  in.ds = tmp.get(cells);
  in.base = (int*)tmp.get(fw);
  in.bq = c->scal + kSlotBase;
  in.sb = (float*)tmp.get(fw);
  in.e = (float*)tmp.get(fw);
  in.rhs = (float*)tmp.get(fw);
  if (!t64 || !in.ds || !in.base || !in.sb || !in.e || !in.rhs) return fail(MR_ENOMEM, "linear building block: temporaries");
  hipError_t x = launch_to_split(delta, in.ds, nl, c->stream);
  if (x == hipSuccess) x = launch_to_split(theta_base, t64, nl, c->stream);
  // fixed-point base with the scale of max |theta_base| (the solve's representation)
  if (x == hipSuccess) x = launch_absmax(t64, cells, c->scal + kSlotTmax, c->stream);
  if (x == hipSuccess) x = launch_base_scale(c->scal + kSlotTmax, c->scal + kSlotBase, c->stream);
  if (x == hipSuccess) x = launch_quantise(t64, in.base, cells, in.bq, c->stream);
  if (x == hipSuccess) x = launch_to_split(e, t64, nl, c->stream);
  if (x == hipSuccess) x = launch_cast32(t64, in.e, cells, c->stream);
  if (x == hipSuccess && rhs) x = launch_to_split(rhs, t64, nl, c->stream);
  if (x == hipSuccess && rhs) x = launch_cast32(t64, in.rhs, cells, c->stream);
  if (x == hipSuccess && !rhs) x = launch_fill32(in.rhs, 0.0f, cells, c->stream);
  if (x == hipSuccess) x = launch_base_root(in.base, in.bq, in.ds, nl, hcell, in.sb, c->stream);
  return x == hipSuccess ? MR_OK : hip_fail(x, "linear building block");
}

int mr_lin_residual(mr_ctx* h, int nl, double hcell, const double* delta, const double* theta_base, const double* e,
                    const double* rhs, double cshift, double* r_out) {
  if (!h || !delta || !theta_base || !e || !r_out) return fail(MR_EINVAL, "mr_lin_residual: null argument");
  int rc = check_level(nl, false);
  if (rc != MR_OK) return rc;
  if (!(hcell > 0.0)) return fail(MR_EINVAL, "mr_lin_residual: cell size must be positive");
  Ctx* c = reinterpret_cast<Ctx*>(h);
  const size_t cells = (size_t)nl * nl * nl;
  Temps tmp(c->stream);
  LinInputs in;
  if ((rc = lin_inputs(c, tmp, nl, hcell, delta, theta_base, e, rhs, in)) != MR_OK) return rc;
  double* rs = tmp.get(cells);
  if (!rs) return fail(MR_ENOMEM, "mr_lin_residual: temporaries");
  hipError_t x = launch_lin_residual(in.e, in.base, in.bq, in.sb, in.rhs, nl, hcell, cshift, rs, c->stream);
  if (x == hipSuccess) x = launch_from_split(rs, r_out, nl, nullptr, 0.0, c->stream);
  if (x == hipSuccess) x = hipStreamSynchronize(c->stream);
  return x == hipSuccess ? MR_OK : hip_fail(x, "mr_lin_residual");
}

int mr_lin_defect_restrict(mr_ctx* h, int nl, double hcell, const double* delta, const double* theta_base,
                           const double* e, const double* rhs, double cshift, double* rc_out) {
  if (!h || !delta || !theta_base || !e || !rc_out) return fail(MR_EINVAL, "mr_lin_defect_restrict: null argument");
  int rc = check_level(nl, true);
  if (rc != MR_OK) return rc;
  if (!(hcell > 0.0)) return fail(MR_EINVAL, "mr_lin_defect_restrict: cell size must be positive");
  Ctx* c = reinterpret_cast<Ctx*>(h);
  const size_t cc = (size_t)(nl / 2) * (nl / 2) * (nl / 2);
  Temps tmp(c->stream);
  LinInputs in;
  if ((rc = lin_inputs(c, tmp, nl, hcell, delta, theta_base, e, rhs, in)) != MR_OK) return rc;
  float* rc32 = (float*)tmp.get((cc + 1) / 2);
  double* rcs = tmp.get(cc);
  if (!rc32 || !rcs) return fail(MR_ENOMEM, "mr_lin_defect_restrict: temporaries");
  hipError_t x = launch_lin_resid_restrict(in.e, in.base, in.bq, in.sb, in.rhs, nl, hcell, ShiftRef{nullptr, 0.0, cshift}, rc32,
                                           c->reducer(kSlotAux), c->stream);
  if (x == hipSuccess) x = launch_widen64(rc32, rcs, cc, c->stream);
  if (x == hipSuccess) x = launch_from_split(rcs, rc_out, nl / 2, nullptr, 0.0, c->stream);
  if (x == hipSuccess) x = hipStreamSynchronize(c->stream);
  return x == hipSuccess ? MR_OK : hip_fail(x, "mr_lin_defect_restrict");
}

int mr_lin_prolong_add(mr_ctx* h, int nl, const double* ec, const double* e_in, double* e_out) {
  if (!h || !ec || !e_in || !e_out) return fail(MR_EINVAL, "mr_lin_prolong_add: null argument");
  int rc = check_level(nl, true);
  if (rc != MR_OK) return rc;
  Ctx* c = reinterpret_cast<Ctx*>(h);
  const size_t cells = (size_t)nl * nl * nl, cc = cells / 8;
  Temps tmp(c->stream);
  double* t64 = tmp.get(cells);
  float* e32 = (float*)tmp.get((cells + 1) / 2);
  float* ec32 = (float*)tmp.get((cc + 1) / 2);
  if (!t64 || !e32 || !ec32) return fail(MR_ENOMEM, "mr_lin_prolong_add: temporaries");
  hipError_t x = launch_to_split(ec, t64, nl / 2, c->stream);
  if (x == hipSuccess) x = launch_cast32(t64, ec32, cc, c->stream);
  if (x == hipSuccess) x = launch_to_split(e_in, t64, nl, c->stream);
  if (x == hipSuccess) x = launch_cast32(t64, e32, cells, c->stream);
  if (x == hipSuccess) x = launch_prolong_add32(ec32, e32, nl, c->stream);
  if (x == hipSuccess) x = launch_widen64(e32, t64, cells, c->stream);
  if (x == hipSuccess) x = launch_from_split(t64, e_out, nl, nullptr, 0.0, c->stream);
  if (x == hipSuccess) x = hipStreamSynchronize(c->stream);
  return x == hipSuccess ? MR_OK : hip_fail(x, "mr_lin_prolong_add");
}

int mr_lin_sweep(mr_ctx* h, int nl, double hcell, const double* delta, const double* theta_base, const double* e_in,
                 const double* rhs, double cshift, const int* sched, double* e_out) {
  if (!h || !delta || !theta_base || !e_in || !e_out || e_in == e_out) return fail(MR_EINVAL, "mr_lin_sweep: bad pointers");
  int rc = check_level(nl, true);
  if (rc != MR_OK) return rc;
  if (!(hcell > 0.0)) return fail(MR_EINVAL, "mr_lin_sweep: cell size must be positive");
  const int nh = nl / 2;
  int kind = MR_SCHED_PIPELINED, tm = 0, tj = 0, nch = 0;
  if (sched) {
    kind = sched[0];
    tm = sched[1];
    tj = sched[2];
    nch = sched[3];
  } else {
    static const int pref[][2] = {{64, 4}, {64, 8}, {32, 8}, {16, 16}, {8, 16}, {4, 8}, {2, 4}};
    for (const auto& p : pref)
      if (tm == 0 && nh % p[0] == 0 && nl % p[1] == 0) {
        tm = p[0];
        tj = p[1];
      }
    nch = nl % 8 == 0 ? nl / 8 : 1;
    kind = (nl / nch) % 4 == 0 ? MR_SCHED_PIPELINED : MR_SCHED_TILED;
  }
  if (tm < 1 || tj < 1 || nh % tm != 0 || nl % tj != 0 || nch < 1 || nl % nch != 0 ||
      (long)(nh / tm) * (nl / tj) * nch > kMaxReduceBlocks)
    return fail(MR_EINVAL, "mr_lin_sweep: tile %d x %d, %d chunks do not fit the %d^3 mesh", tm, tj, nch, nl);
  if (kind == MR_SCHED_FUSED ? !lin_fused_supported(tm, tj) || nl / nch < 2
                             : !lin_tile_supported(tm, tj) || (kind == MR_SCHED_PIPELINED && (nl / nch) % 4 != 0) ||
                                   (kind != MR_SCHED_PIPELINED && kind != MR_SCHED_TILED))
    return fail(MR_EINVAL, "mr_lin_sweep: no kernel for schedule %d (%d x %d, %d chunks)", kind, tm, tj, nch);
  Ctx* c = reinterpret_cast<Ctx*>(h);
  const size_t cells = (size_t)nl * nl * nl;
  Temps tmp(c->stream);
  LinInputs in;
  if ((rc = lin_inputs(c, tmp, nl, hcell, delta, theta_base, e_in, rhs, in)) != MR_OK) return rc;
  float* eo = (float*)tmp.get((cells + 1) / 2);
  double* es = tmp.get(cells);
  if (!eo || !es) return fail(MR_ENOMEM, "mr_lin_sweep: temporaries");
  hipError_t x = hipSuccess;
  if (kind == MR_SCHED_FUSED) {
    LinFusedArgs a{};
    a.e_in = in.e;
    a.e_out = eo;
    a.base = in.base;
    a.bq = in.bq;
    a.sb = in.sb;
    a.rhs = in.rhs;
    a.n = nl;
    a.h2 = (float)(hcell * hcell);
    a.ih2 = (float)(1.0 / (hcell * hcell));
    a.c_add = cshift;
    a.sum_out = c->scal + kSlotAux;
    a.partials = c->partials;
    a.counter = c->counter;
    x = launch_lin_fused(a, LinFusedCfg{tm, tj, nch}, c->stream);
  } else {
    TileCfg t;
    t.tm = tm;
    t.tj = tj;
    t.ci = nl / nch;
    t.tiles_j = nl / tj;
    t.tiles_m = nh / tm;
    t.pipe = kind == MR_SCHED_PIPELINED;
    LinSweepArgs a{};
    a.e_in = in.e;
    a.e_out = eo;
    a.base = in.base;
    a.bq = in.bq;
    a.sb = in.sb;
    a.rhs = in.rhs;
    a.n = nl;
    a.colour = 0;
    a.h2 = (float)(hcell * hcell);
    a.ih2 = (float)(1.0 / (hcell * hcell));
    a.c_add = cshift;
    a.sum_out = c->scal + kSlotAux;
    a.partials = c->partials;
    a.counter = c->counter;
    x = launch_lin_half_sweep(a, t, c->stream);
    a.colour = 1;
    a.e_red_new = eo;
    a.sum_out = c->scal + kSlotAux + 1;
    if (x == hipSuccess) x = launch_lin_half_sweep(a, t, c->stream);
  }
  if (x == hipSuccess) x = launch_widen64(eo, es, cells, c->stream);
  if (x == hipSuccess) x = launch_from_split(es, e_out, nl, nullptr, 0.0, c->stream);
  if (x == hipSuccess) x = hipStreamSynchronize(c->stream);
  return x == hipSuccess ? MR_OK : hip_fail(x, "mr_lin_sweep");
}

int mr_lin_vcycles(mr_ctx* h, const double* delta, const double* theta_base, const double* rhs, int ncycles,
                   double* e_out) {
  if (!h || !delta || !theta_base || !rhs || !e_out) return fail(MR_EINVAL, "mr_lin_vcycles: null argument");
  if (ncycles < 1 || ncycles > 64) return fail(MR_EINVAL, "mr_lin_vcycles: ncycles %d not in 1..64", ncycles);
  Ctx* c = reinterpret_cast<Ctx*>(h);
  int rc = c->mixed_ready();
  if (rc != MR_OK) return rc;
  if ((rc = c->prepare(delta)) != MR_OK) return rc;
  const int n = c->n;
  const size_t cells = c->lv[0].cells;
  Temps tmp(c->stream);
  double *ts = tmp.get(cells), *rs = tmp.get(cells);
  if (!ts || !rs) return fail(MR_ENOMEM, "mr_lin_vcycles: temporaries");
  hipError_t x = launch_to_split(theta_base, ts, n, c->stream);
  if (x == hipSuccess) x = launch_to_split(rhs, rs, n, c->stream);
  if (x != hipSuccess) return hip_fail(x, "mr_lin_vcycles");
  float* e32 = nullptr;
  if ((rc = c->lin_vcycles_split(ts, rs, ncycles, &e32)) != MR_OK) return rc;
  x = launch_widen64(e32, ts, cells, c->stream);
  if (x == hipSuccess) x = launch_from_split(ts, e_out, n, nullptr, 0.0, c->stream);
  if (x == hipSuccess) x = hipStreamSynchronize(c->stream);
  return x == hipSuccess ? MR_OK : hip_fail(x, "mr_lin_vcycles");
}

int mr_restrict(mr_ctx* h, int nl, const double* fine, double* coarse) {
  if (!h || !fine || !coarse) return fail(MR_EINVAL, "mr_restrict: null argument");
  int rc = check_level(nl, true);
  if (rc != MR_OK) return rc;
  Ctx* c = reinterpret_cast<Ctx*>(h);
  const size_t cells = (size_t)nl * nl * nl, cc = cells / 8;
  Temps tmp(c->stream);
  double *a = tmp.get(cells), *b = tmp.get(cc);
  if (!a || !b) return fail(MR_ENOMEM, "mr_restrict: temporaries");
  hipError_t e = launch_to_split(fine, a, nl, c->stream);
  if (e == hipSuccess) e = launch_restrict(a, b, nl, c->stream);
  if (e == hipSuccess) e = launch_from_split(b, coarse, nl / 2, nullptr, 0.0, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  return e == hipSuccess ? MR_OK : hip_fail(e, "mr_restrict");
}

}  // extern "C"
