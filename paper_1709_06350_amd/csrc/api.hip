// Host side of the library: context and level hierarchy, the FAS V-cycle driver (Sec. II.A.3)
// and the C ABI declared in include/mr.h.
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
  const auto s = level_sizes(n);
  if ((long)s.back() * s.back() * s.back() > kMaxCoarsest)
    return fail(MR_EINVAL, "n = %d: coarsest mesh %d^3 exceeds 12^3", n, s.back());
  if (n > 2048) return fail(MR_EINVAL, "n = %d: too large", n);
  return MR_OK;
}

int check_opts(const mr_opts& o) {
  if (!(o.tol >= 0.0) || o.max_cycles < 1 || o.max_cycles > 127 || o.npre < 0 || o.npost < 0 ||
      o.ncoarse < 1 || (o.precision != MR_PREC_FP64 && o.precision != MR_PREC_MIXED) ||
      o.inner_cycles < 1 || o.inner_cycles > 8)
    return fail(MR_EINVAL, "invalid options");
  return MR_OK;
}

TileCfg choose_tiles(int n, int max_lds) {
  TileCfg t;
  t.tk = 64;
  while (t.tk > 4 && (n % t.tk != 0 || t.tk > n)) t.tk /= 2;
  t.tj = 16;
  while (t.tj > 2 && (n % t.tj != 0 || t.tj > n)) t.tj /= 2;
  while (t.tj > 2 && sweep_lds_bytes(t.tj, t.tk) > (size_t)max_lds) t.tj /= 2;
  t.tiles_j = n / t.tj;
  t.tiles_k = n / t.tk;
  const long tiles = (long)t.tiles_j * t.tiles_k;
  t.ci = n;
  while (t.ci % 2 == 0 && t.ci > 4 && tiles * (n / t.ci) < 2048) t.ci /= 2;
  while (tiles * (n / t.ci) > kMaxReduceBlocks && t.ci * 2 <= n && n % (t.ci * 2) == 0) t.ci *= 2;
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

// ---- one FP64 sweep / V-cycle on the level hierarchy ----------------------------------------

int Ctx::sweep(int l) {
  Level& L = lv[l];
  SweepArgs a{};
  a.th_in = L.th[L.cur];
  a.th_out = L.th[L.cur ^ 1];
  a.delta = L.delta;
  a.f = (l == 0) ? nullptr : L.f;
  a.n = L.n;
  a.h2 = L.h * L.h;
  a.ih2 = 1.0 / a.h2;
  a.c_sum = scal + kSlotLevel + l;
  a.c_scale = 1.0 / (double)L.cells;
  a.c_add = 0.0;
  a.sum_out = scal + kSlotLevel + l;
  a.partials = partials;
  a.counter = counter;
  a.tj = L.tile.tj;
  a.tiles_j = L.tile.tiles_j;
  a.tiles_k = L.tile.tiles_k;
  a.ci = L.tile.ci;
  hipError_t e = launch_sweep(a, L.tile.tk, stream);
  if (e != hipSuccess) return hip_fail(e, "sweep");
  L.cur ^= 1;
  return MR_OK;
}

int Ctx::vcycle(int l) {
  Level& L = lv[l];
  hipError_t e;
  if (l == nlev - 1) {
    CoarsestArgs a{};
    a.theta = L.th[L.cur];
    a.delta = L.delta;
    a.f = (l == 0) ? nullptr : L.f;
    a.n = L.n;
    a.nsweeps = opts.ncoarse;
    a.h2 = L.h * L.h;
    a.ih2 = 1.0 / a.h2;
    a.c_sum = scal + kSlotLevel + l;
    a.c_scale = 1.0 / (double)L.cells;
    a.c_sum_out = scal + kSlotLevel + l;
    e = launch_coarsest(a, stream);
    return e == hipSuccess ? MR_OK : hip_fail(e, "coarsest");
  }
  int rc;
  for (int s = 0; s < opts.npre; ++s)
    if ((rc = sweep(l)) != MR_OK) return rc;
  Level& Lc = lv[l + 1];
  ShiftRef c{scal + kSlotLevel + l, 1.0 / (double)L.cells, 0.0};
  e = launch_defect_restrict(L.th[L.cur], L.delta, (l == 0) ? nullptr : L.f, L.n, L.h, c,
                             Lc.th[Lc.cur], Lc.that, Lc.f, stream);
  if (e != hipSuccess) return hip_fail(e, "defect_restrict");
  e = launch_tau(Lc.that, Lc.delta, Lc.f, Lc.f, Lc.n, Lc.h,
                 Reduce{partials, counter, scal + kSlotLevel + l + 1}, kMaxReduceBlocks, stream);
  if (e != hipSuccess) return hip_fail(e, "tau");
  if ((rc = vcycle(l + 1)) != MR_OK) return rc;
  e = launch_prolong_correct(Lc.th[Lc.cur], Lc.that, L.th[L.cur], L.n, stream);
  if (e != hipSuccess) return hip_fail(e, "prolong_correct");
  for (int s = 0; s < opts.npost; ++s)
    if ((rc = sweep(l)) != MR_OK) return rc;
  return MR_OK;
}

// Residual norm of the finest level: b = nabla^2 theta - Sigma + shift with the given shift;
// ||r|| = sqrt(sum b^2 - (sum b)^2 / N^3) is the norm of the mean-projected residual and
// <Sigma> = shift - <b>. shv is the host value of the shift.
int Ctx::finest_norm(const double* theta, ShiftRef sh, double* nrm, double* msig) {
  Level& L = lv[0];
  hipError_t e = launch_residual(theta, L.delta, L.n, 1.0, sh, nullptr, reducer(kSlotRes), kMaxReduceBlocks, stream);
  if (e != hipSuccess) return hip_fail(e, "residual");
  double r[kSlotRes + 2];
  int rc = read_scalars(0, kSlotRes + 2, r);
  if (rc != MR_OK) return rc;
  const double N3 = (double)L.cells;
  const double var = r[kSlotRes + 1] - r[kSlotRes] * r[kSlotRes] / N3;
  *nrm = std::sqrt(var > 0.0 ? var : 0.0);
  const double shv = (sh.c_sum ? r[sh.c_sum - scal] * sh.c_scale : 0.0) + sh.c_add;
  *msig = shv - r[kSlotRes] / N3;
  return MR_OK;
}

int Ctx::prepare(const double* delta, double* theta) {
  Level& L0 = lv[0];
  L0.delta = delta;
  L0.th[0] = theta;
  L0.th[1] = ws_theta0;
  L0.cur = 0;
  hipError_t e = launch_validate(delta, L0.cells, reducer(kSlotRes), kMaxReduceBlocks, stream);
  if (e != hipSuccess) return hip_fail(e, "validate");
  double bad;
  int rc = read_scalars(kSlotRes, 1, &bad);
  if (rc != MR_OK) return rc;
  if (bad != 0.0) return fail(MR_EDOMAIN, "delta has %.0f cells with a non-finite value or 1 + delta <= 0", bad);
  for (int l = 1; l < nlev; ++l) {
    e = launch_restrict(lv[l - 1].delta, lv[l].delta_own, lv[l - 1].n, stream);
    if (e != hipSuccess) return hip_fail(e, "restrict delta");
  }
  return MR_OK;
}

int Ctx::solve_fp64(const double* delta, double* theta, mr_info* info) {
  auto t0 = std::chrono::steady_clock::now();
  int rc = prepare(delta, theta);
  if (rc != MR_OK) return rc;
  Level& L0 = lv[0];
  hipError_t e;
  if (!opts.warm_start) {
    e = hipMemsetAsync(theta, 0, L0.cells * sizeof(double), stream);
    if (e != hipSuccess) return hip_fail(e, "memset");
  }
  double r0, m0, nrm, msig;
  if ((rc = finest_norm(nullptr, ShiftRef{nullptr, 0.0, 0.0}, &r0, &m0)) != MR_OK) return rc;
  if (r0 == 0.0) r0 = 1.0;
  if (opts.warm_start) {
    if ((rc = finest_norm(theta, ShiftRef{nullptr, 0.0, 0.0}, &nrm, &msig)) != MR_OK) return rc;
  } else {
    nrm = r0 == 1.0 ? 0.0 : r0;
    msig = m0;
  }
  // Running sum of Sigma on the finest level, so that the first sweep uses the exact <Sigma>.
  if ((rc = write_scalar(kSlotLevel + 0, msig * (double)L0.cells)) != MR_OK) return rc;
  double rel = nrm / r0;
  mr_info loc{};
  loc.r0_norm = r0;
  loc.history[0] = rel;
  int cyc = 0;
  int status = MR_OK;
  double best = rel;
  while (rel > opts.tol && cyc < opts.max_cycles) {
    if ((rc = vcycle(0)) != MR_OK) return rc;
    ++cyc;
    if ((rc = finest_norm(L0.th[L0.cur], ShiftRef{scal + kSlotLevel + 0, 1.0 / (double)L0.cells, 0.0}, &nrm, &msig)) != MR_OK)
      return rc;
    rel = nrm / r0;
    if (cyc < 128) loc.history[cyc] = rel;
    if (!std::isfinite(rel) || rel > 1e6 * (best > 1.0 ? best : 1.0)) {
      status = fail(MR_EDIVERGED, "residual diverged at cycle %d (%g)", cyc, rel);
      break;
    }
    if (rel < best) best = rel;
  }
  if (status == MR_OK && rel > opts.tol) {
    status = MR_NOT_CONVERGED;
    fail(MR_NOT_CONVERGED, "not converged after %d cycles (rel residual %g)", cyc, rel);
  }
  // Gauge <theta> = 0, result into the caller's buffer.
  e = launch_sum(L0.th[L0.cur], L0.cells, reducer(kSlotGauge), kMaxReduceBlocks, stream);
  if (e == hipSuccess)
    e = launch_shift_copy(L0.th[L0.cur], theta, L0.cells, scal + kSlotGauge, 1.0 / (double)L0.cells, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return hip_fail(e, "gauge");
  L0.cur = 0;
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
  int max_lds = 65536;
  c->max_lds = max_lds;
  const auto sizes = level_sizes(n);
  c->nlev = (int)sizes.size();
  c->lv.resize(sizes.size());
  for (size_t l = 0; l < sizes.size(); ++l) {
    Level& L = c->lv[l];
    L.n = sizes[l];
    L.cells = (size_t)L.n * L.n * L.n;
    L.h = std::ldexp(1.0, (int)l);
    L.tile = choose_tiles(L.n, max_lds);
    if (l == 0) continue;
    if ((rc = c->dev_alloc(&L.th[0], L.cells)) != MR_OK ||
        (rc = c->dev_alloc(&L.th[1], L.cells)) != MR_OK ||
        (rc = c->dev_alloc(&L.that, L.cells)) != MR_OK ||
        (rc = c->dev_alloc(&L.f, L.cells)) != MR_OK ||
        (rc = c->dev_alloc(&L.delta_own, L.cells)) != MR_OK) {
      mr_destroy(reinterpret_cast<mr_ctx*>(c));
      return rc;
    }
    L.delta = L.delta_own;
  }
  if ((rc = c->dev_alloc(&c->ws_theta0, c->lv[0].cells)) != MR_OK ||
      (rc = c->dev_alloc(&c->scal, kSlotCount)) != MR_OK ||
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
  *out = reinterpret_cast<mr_ctx*>(c);
  return MR_OK;
}

void mr_destroy(mr_ctx* h) {
  if (!h) return;
  Ctx* c = reinterpret_cast<Ctx*>(h);
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  else (void)hipDeviceSynchronize();
  for (void* p : c->owned) (void)hipFree(p);
  if (c->host) (void)hipHostFree(c->host);
  c->release_extra();
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

int mr_residual(mr_ctx* h, const double* delta, const double* theta, double* r_out, double* rel_out,
                double* msum_out) {
  if (!h || !delta || !theta) return fail(MR_EINVAL, "mr_residual: null argument");
  Ctx* c = reinterpret_cast<Ctx*>(h);
  Level& L0 = c->lv[0];
  L0.delta = delta;
  int rc;
  double r0, m0, n1, m1, n2, m2;
  if ((rc = c->finest_norm(nullptr, ShiftRef{nullptr, 0.0, 0.0}, &r0, &m0)) != MR_OK) return rc;
  if ((rc = c->finest_norm(theta, ShiftRef{nullptr, 0.0, 0.0}, &n1, &m1)) != MR_OK) return rc;
  // second pass with the exact mean of Sigma, writing r
  hipError_t e = launch_residual(theta, delta, L0.n, 1.0, ShiftRef{nullptr, 0.0, m1}, r_out,
                                 c->reducer(kSlotRes), kMaxReduceBlocks, c->stream);
  if (e != hipSuccess) return hip_fail(e, "residual");
  double r[2];
  if ((rc = c->read_scalars(kSlotRes, 2, r)) != MR_OK) return rc;
  const double var = r[1] - r[0] * r[0] / (double)L0.cells;
  n2 = std::sqrt(var > 0 ? var : 0.0);
  m2 = m1;
  if (rel_out) *rel_out = (r0 > 0.0) ? n2 / r0 : n2;
  if (msum_out) *msum_out = m2;
  (void)m0;
  (void)n1;
  return MR_OK;
}

int mr_solve(mr_ctx* h, const double* delta, double* theta, mr_info* info) {
  if (!h || !delta || !theta) return fail(MR_EINVAL, "mr_solve: null argument");
  Ctx* c = reinterpret_cast<Ctx*>(h);
  if (c->opts.precision == MR_PREC_MIXED) return c->solve_mixed(delta, theta, info);
  return c->solve_fp64(delta, theta, info);
}

// ---- building blocks ----------------------------------------------------------------------

static int check_level_size(Ctx* c, int nl) {
  (void)c;
  if (nl < 4 || nl % 4 != 0) return fail(MR_EINVAL, "level size %d: must be a multiple of 4", nl);
  return MR_OK;
}

int mr_sweep(mr_ctx* h, int nl, double hcell, const double* delta, const double* f, double cshift,
             const double* theta_in, double* theta_out, double* sum_out) {
  if (!h || !delta || !theta_in || !theta_out || theta_in == theta_out)
    return fail(MR_EINVAL, "mr_sweep: bad pointers");
  Ctx* c = reinterpret_cast<Ctx*>(h);
  int rc = check_level_size(c, nl);
  if (rc != MR_OK) return rc;
  TileCfg t = choose_tiles(nl, c->max_lds);
  SweepArgs a{};
  a.th_in = theta_in;
  a.th_out = theta_out;
  a.delta = delta;
  a.f = f;
  a.n = nl;
  a.h2 = hcell * hcell;
  a.ih2 = 1.0 / a.h2;
  a.c_sum = nullptr;
  a.c_scale = 0.0;
  a.c_add = cshift;
  a.sum_out = c->scal + kSlotRes;
  a.partials = c->partials;
  a.counter = c->counter;
  a.tj = t.tj;
  a.tiles_j = t.tiles_j;
  a.tiles_k = t.tiles_k;
  a.ci = t.ci;
  hipError_t e = launch_sweep(a, t.tk, c->stream);
  if (e != hipSuccess) return hip_fail(e, "sweep");
  double s;
  if ((rc = c->read_scalars(kSlotRes, 1, &s)) != MR_OK) return rc;
  if (sum_out) *sum_out = s;
  return MR_OK;
}

int mr_defect_restrict(mr_ctx* h, int nl, double hcell, const double* delta, const double* f,
                       double cshift, const double* theta, double* theta_c, double* dr_c) {
  if (!h || !delta || !theta || !theta_c || !dr_c) return fail(MR_EINVAL, "mr_defect_restrict: null argument");
  Ctx* c = reinterpret_cast<Ctx*>(h);
  if (nl < 4 || nl % 2) return fail(MR_EINVAL, "bad level size");
  hipError_t e = launch_defect_restrict(theta, delta, f, nl, hcell, ShiftRef{nullptr, 0.0, cshift},
                                        theta_c, nullptr, dr_c, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  return e == hipSuccess ? MR_OK : hip_fail(e, "defect_restrict");
}

int mr_tau_rhs(mr_ctx* h, int nl, double hcell, const double* delta, const double* theta_hat,
               const double* rd, double* f_out, double* sum_out) {
  if (!h || !delta || !theta_hat || !rd || !f_out) return fail(MR_EINVAL, "mr_tau_rhs: null argument");
  Ctx* c = reinterpret_cast<Ctx*>(h);
  if (nl < 2 || nl % 2) return fail(MR_EINVAL, "bad level size");
  hipError_t e = launch_tau(theta_hat, delta, rd, f_out, nl, hcell, c->reducer(kSlotRes), kMaxReduceBlocks, c->stream);
  if (e != hipSuccess) return hip_fail(e, "tau");
  double s;
  int rc = c->read_scalars(kSlotRes, 1, &s);
  if (rc == MR_OK && sum_out) *sum_out = s;
  return rc;
}

int mr_prolong_correct(mr_ctx* h, int nl, const double* theta_c, const double* theta_hat_c, double* theta) {
  if (!h || !theta_c || !theta_hat_c || !theta) return fail(MR_EINVAL, "mr_prolong_correct: null argument");
  Ctx* c = reinterpret_cast<Ctx*>(h);
  if (nl < 4 || nl % 2) return fail(MR_EINVAL, "bad level size");
  hipError_t e = launch_prolong_correct(theta_c, theta_hat_c, theta, nl, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  return e == hipSuccess ? MR_OK : hip_fail(e, "prolong_correct");
}

int mr_restrict(mr_ctx* h, int nl, const double* fine, double* coarse) {
  if (!h || !fine || !coarse) return fail(MR_EINVAL, "mr_restrict: null argument");
  Ctx* c = reinterpret_cast<Ctx*>(h);
  if (nl < 2 || nl % 2) return fail(MR_EINVAL, "bad level size");
  hipError_t e = launch_restrict(fine, coarse, nl, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  return e == hipSuccess ? MR_OK : hip_fail(e, "restrict");
}

}  // extern "C"
