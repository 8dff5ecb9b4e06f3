// Host-side checks of libmr, built with the host half of the HIP sources instrumented by
// AddressSanitizer and UndefinedBehaviorSanitizer (the device code is not instrumented).
//
// Without a device: argument validation of every entry point that checks before touching the
// device (level sizes of batched boxes, option checks, buffer sizes), the on-disk record of tuner
// choices (store, reload, malformed lines, long keys) and error strings. With a device (--gpu and
// one present): contexts of several mesh sizes (level hierarchies, schedule tuners and their
// candidate lists, the mixed form's buffers and Krylov space), small FP64, mixed and batched
// solves, a deposit, and the reusable batch; a sanitizer report or a failed check exits non-zero.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "mr.h"

static int g_fail = 0;
#define CHECK(cond)                                                            \
  do {                                                                         \
    if (!(cond)) {                                                             \
      std::fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #cond); \
      ++g_fail;                                                                \
    }                                                                          \
  } while (0)

static void host_only(const char* tmpdir) {
  mr_opts o;
  mr_default_opts(&o);
  CHECK(o.npre == 2 && o.npost == 2 && o.max_cycles == 100);
  mr_ctx* c = nullptr;
  CHECK(mr_create(nullptr, 32, &o, nullptr) == MR_EINVAL);
  for (int n : {0, 2, 7, 9, 2000, -8}) CHECK(mr_create(&c, n, &o, nullptr) == MR_EINVAL && c == nullptr);
  mr_opts bad = o;
  bad.npre = -1;
  CHECK(mr_create(&c, 32, &bad, nullptr) == MR_EINVAL);
  bad = o;
  bad.flags = 1 << 20;
  CHECK(mr_create(&c, 32, &bad, nullptr) == MR_EINVAL);
  bad = o;
  bad.inner_cycles = 99;
  CHECK(mr_create(&c, 32, &bad, nullptr) == MR_EINVAL);
  CHECK(std::strlen(mr_last_error()) > 0);
  // batched: box sizes are checked (level hierarchy per size) before any device work
  const double* dp[3] = {nullptr, nullptr, nullptr};
  double* tp[3] = {nullptr, nullptr, nullptr};
  for (int nb : {10, 7, 2048, 6, 0}) {
    int ns[3] = {16, nb, 32};
    CHECK(mr_solve_batched(3, ns, dp, tp, &o, nullptr, nullptr) == MR_EINVAL);
    mr_batch* b = nullptr;
    CHECK(mr_batch_create(&b, 3, ns, &o, nullptr) == MR_EINVAL && b == nullptr);
  }
  CHECK(mr_solve_batched(0, nullptr, dp, tp, &o, nullptr, nullptr) == MR_EINVAL);
  CHECK(mr_batch_create(nullptr, 1, nullptr, &o, nullptr) == MR_EINVAL);
  CHECK(mr_batch_solve(nullptr, dp, tp, nullptr) == MR_EINVAL);
  CHECK(mr_batch_destroy(nullptr) == MR_OK);
  CHECK(mr_tune_lin_tiles(7, nullptr, nullptr, nullptr, nullptr, nullptr) == MR_EINVAL);
  CHECK(mr_tune_lin_tiles(2048, nullptr, nullptr, nullptr, nullptr, nullptr) == MR_EINVAL);
  CHECK(mr_hbm_stream(5, 0, nullptr, nullptr, nullptr, 16, 4, nullptr, nullptr) == MR_EINVAL);
  CHECK(mr_residual_noalloc(7, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr) == MR_EINVAL);
  CHECK(mr_deposit(nullptr, nullptr, 1, 1.0, MR_DEPOSIT_CIC, nullptr) == MR_EINVAL);
  CHECK(mr_lagrangian(nullptr, nullptr, nullptr, 1, nullptr, nullptr) == MR_EINVAL);
  CHECK(mr_solve(nullptr, nullptr, nullptr, nullptr) == MR_EINVAL);
  CHECK(mr_get_schedule(nullptr, 0, nullptr) == MR_EINVAL);
  CHECK(mr_get_lin_schedule(nullptr, 0, nullptr) == MR_EINVAL);
  // the record of tuner choices: store, reload from the file, malformed lines, long keys
  const std::string path = std::string(tmpdir) + "/sub/dir/tuning.txt";
  CHECK(mr_tuning_file(path.c_str()) == MR_OK);
  CHECK(std::string(mr_tuning_file_path()) == path);
  std::string longname(5000, 'x');
  longname[100] = '|';
  const int v1[5] = {1, -2, 3, 2147483647, -2147483647};
  CHECK(mr_tuning_store("k.v1", "gfx950", longname.c_str(), 256, 512, v1, 5) == MR_OK);
  int out[64] = {0}, cnt = -1;
  CHECK(mr_tuning_file(path.c_str()) == MR_OK);   // forget, read the file again
  CHECK(mr_tuning_lookup("k.v1", "gfx950", longname.c_str(), 256, 512, out, 64, &cnt) == MR_OK && cnt == 5);
  CHECK(std::memcmp(out, v1, sizeof v1) == 0);
  CHECK(mr_tuning_lookup("k.v1", "gfx950", longname.c_str(), 256, 512, out, 2, &cnt) == MR_EINVAL);
  CHECK(mr_tuning_lookup("absent", "a", "b", 1, 1, out, 64, &cnt) == MR_OK && cnt == 0);
  {
    FILE* f = std::fopen(path.c_str(), "w");
    CHECK(f != nullptr);
    if (f) {
      std::fputs("#\n|||||\nk|a|b|1|2|\nk|a|b|1|3|1,,2\nk|a|b|1|4|99999999999999999999\nk|a|b|1|5|7,8\n", f);
      std::fclose(f);
    }
  }
  CHECK(mr_tuning_file(path.c_str()) == MR_OK);
  CHECK(mr_tuning_lookup("k", "a", "b", 1, 5, out, 64, &cnt) == MR_OK && cnt == 2 && out[0] == 7 && out[1] == 8);
  CHECK(mr_tuning_lookup("k", "a", "b", 1, 3, out, 64, &cnt) == MR_OK && cnt == 0);
  CHECK(mr_tuning_file("") == MR_OK);
  CHECK(std::string(mr_tuning_file_path()).empty());
  CHECK(mr_tuning_file(nullptr) == MR_OK);
}

static std::vector<double> smooth_delta(int n, double amp) {
  std::vector<double> d((size_t)n * n * n);
  const double k = 2.0 * M_PI / n;
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j)
      for (int l = 0; l < n; ++l)
        d[((size_t)i * n + j) * n + l] = amp * (std::sin(k * i) * std::cos(2 * k * j) + 0.5 * std::sin(k * (l + i)));
  return d;
}

static double* to_dev(const std::vector<double>& h) {
  double* p = nullptr;
  if (hipMalloc(&p, h.size() * sizeof(double)) != hipSuccess) return nullptr;
  (void)hipMemcpy(p, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice);
  return p;
}

static void with_device() {
  mr_opts o;
  mr_default_opts(&o);
  for (int n : {8, 12, 48, 64, 96}) {
    mr_ctx* c = nullptr;
    CHECK(mr_create(&c, n, &o, nullptr) == MR_OK);
    if (!c) continue;
    const int nl = mr_levels(c);
    CHECK(nl >= 2);
    for (int l = 0; l + 1 < nl; ++l) {
      int sched[4];
      CHECK(mr_get_schedule(c, l, sched) == MR_OK);
      const int cnt = mr_schedule_candidates(c, l, nullptr, 0);
      CHECK(cnt >= 1);
      std::vector<int> all(4 * (size_t)(cnt > 0 ? cnt : 1));
      CHECK(mr_schedule_candidates(c, l, all.data(), cnt) == cnt);
      CHECK(mr_set_schedule(c, l, all.data()) == MR_OK);
      CHECK(mr_get_lin_schedule(c, l, sched) == MR_OK);
    }
    CHECK(mr_get_schedule(c, nl - 1, nullptr) == MR_EINVAL);
    std::vector<double> dh = smooth_delta(n, 0.3);
    double* d = to_dev(dh);
    double* th = to_dev(std::vector<double>(dh.size(), 0.0));
    mr_info info;
    o.tol = 1e-9;
    for (int prec : {MR_PREC_FP64, MR_PREC_MIXED}) {
      o.precision = prec;
      o.inner_cycles = prec == MR_PREC_MIXED ? 4 : 1;
      CHECK(mr_set_opts(c, &o) == MR_OK);
      CHECK(mr_solve(c, d, th, &info) == MR_OK && info.rel_residual <= 1e-9);
    }
    // a deposit of a few particles
    std::vector<double> ph = {0.5, 1.25, 2.0, n - 0.5, 0.0, 3.75, 1e-9, n - 1e-9, 0.5};
    double* pos = to_dev(ph);
    CHECK(mr_deposit(c, pos, 3, 1.0, MR_DEPOSIT_TSC, th) == MR_OK);
    CHECK(mr_deposit(c, pos, 3, 1.0, MR_DEPOSIT_CIC, th) == MR_OK);
    (void)hipFree(pos);
    (void)hipFree(d);
    (void)hipFree(th);
    mr_destroy(c);
  }
  // batched, one-shot and reusable
  const int ns[4] = {16, 24, 32, 16};
  std::vector<double*> ds, ts;
  for (int b = 0; b < 4; ++b) {
    ds.push_back(to_dev(smooth_delta(ns[b], 0.2 + 0.1 * b)));
    ts.push_back(to_dev(std::vector<double>((size_t)ns[b] * ns[b] * ns[b], 0.0)));
  }
  mr_opts ob;
  mr_default_opts(&ob);
  ob.tol = 1e-8;
  mr_info infos[4];
  CHECK(mr_solve_batched(4, ns, ds.data(), ts.data(), &ob, infos, nullptr) == MR_OK);
  mr_batch* b = nullptr;
  CHECK(mr_batch_create(&b, 4, ns, &ob, nullptr) == MR_OK);
  for (int rep = 0; rep < 2 && b; ++rep) CHECK(mr_batch_solve(b, ds.data(), ts.data(), infos) == MR_OK);
  CHECK(mr_batch_destroy(b) == MR_OK);
  for (int k = 0; k < 4; ++k) {
    (void)hipFree(ds[k]);
    (void)hipFree(ts[k]);
  }
}

int main(int argc, char** argv) {
  const char* tmpdir = argc > 1 ? argv[1] : "/tmp";
  const bool want_gpu = argc > 2 && std::strcmp(argv[2], "--gpu") == 0;
  host_only(tmpdir);
  int count = 0;
  if (want_gpu && hipGetDeviceCount(&count) == hipSuccess && count > 0) with_device();
  std::printf("host checks: %d failed%s\n", g_fail, want_gpu ? (count > 0 ? " (with device)" : " (no device)") : "");
  return g_fail == 0 ? 0 : 1;
}
