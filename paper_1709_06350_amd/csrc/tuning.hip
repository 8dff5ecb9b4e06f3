// Persistent record of the tuners' choices: an in-memory map backed by a text file.
//
// File format: lines "kind|arch|device|cus|n|v0,v1,..."; lines starting with '#' are comments.
// The file is read once (on the first lookup after the path is set) and rewritten as a whole,
// through a temporary file and a rename, whenever a choice is recorded.
#include <hip/hip_runtime.h>

#include <dlfcn.h>
#include <sys/stat.h>
#include <unistd.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "mr.h"
#include "mr_ctx.h"
#include "tuning.h"

namespace mr {
namespace {

std::mutex g_mu;
std::map<std::string, std::vector<int>> g_store;
bool g_loaded = false;
// choices shipped beside the library (tuning_defaults.txt next to libmr.so, or $MR_TUNING_DEFAULTS):
// consulted when the record file has no entry for a key; never written
std::map<std::string, std::vector<int>> g_defaults;
bool g_defaults_loaded = false;
bool g_path_set = false;   // mr_tuning_file was called
int g_generation = 0;
std::string g_path;        // the file in use when g_path_set ("" = none)

struct DevKey {
  std::string arch, name;
  int cus = 0;
};
std::map<int, DevKey> g_devs;

std::string default_path() {
  const char* env = std::getenv("MR_TUNING_FILE");
  if (env) return std::string(env);   // "" turns the file off
  const char* xdg = std::getenv("XDG_CACHE_HOME");
  if (xdg && *xdg) return std::string(xdg) + "/paper_1709_06350_amd/tuning.txt";
  const char* home = std::getenv("HOME");
  if (home && *home) return std::string(home) + "/.cache/paper_1709_06350_amd/tuning.txt";
  return std::string();
}

const std::string& path_locked() {
  if (!g_path_set) {
    g_path = default_path();
    g_path_set = true;
  }
  return g_path;
}

// '|' and newlines would break a record: replace them in the free-text parts
std::string clean(const std::string& s) {
  std::string o = s;
  for (char& c : o)
    if (c == '|' || c == '\n' || c == '\r') c = ' ';
  return o;
}

std::string make_key(const std::string& kind, const std::string& arch, const std::string& dev, int cus, int n) {
  return clean(kind) + "|" + clean(arch) + "|" + clean(dev) + "|" + std::to_string(cus) + "|" + std::to_string(n);
}

void parse_file(const std::string& p, std::map<std::string, std::vector<int>>& store);

std::string defaults_path() {
  const char* env = std::getenv("MR_TUNING_DEFAULTS");
  if (env) return std::string(env);   // "" turns the defaults off
  Dl_info info;
  if (dladdr(reinterpret_cast<void*>(&default_path), &info) == 0 || !info.dli_fname) return std::string();
  std::string lib = info.dli_fname;
  const size_t slash = lib.rfind('/');
  return (slash == std::string::npos ? std::string(".") : lib.substr(0, slash)) + "/tuning_defaults.txt";
}

void load_locked() {
  if (!g_defaults_loaded) {
    g_defaults_loaded = true;
    const std::string d = defaults_path();
    if (!d.empty()) parse_file(d, g_defaults);
  }
  if (g_loaded) return;
  g_loaded = true;
  const std::string& p = path_locked();
  if (p.empty()) return;
  parse_file(p, g_store);
}

void parse_file(const std::string& p, std::map<std::string, std::vector<int>>& store) {
  std::ifstream f(p);
  std::string line;
  while (std::getline(f, line)) {
    if (line.empty() || line[0] == '#') continue;
    const size_t bar = line.rfind('|');
    if (bar == std::string::npos) continue;
    // the key is the first five fields
    size_t nbar = 0;
    for (char c : line.substr(0, bar)) nbar += (c == '|');
    if (nbar != 4) continue;
    std::vector<int> vals;
    std::stringstream ss(line.substr(bar + 1));
    std::string tok;
    bool ok = true;
    while (std::getline(ss, tok, ',')) {
      char* end = nullptr;
      const long v = std::strtol(tok.c_str(), &end, 10);
      if (end == tok.c_str() || *end != '\0') {
        ok = false;
        break;
      }
      vals.push_back((int)v);
    }
    if (ok && !vals.empty()) store[line.substr(0, bar)] = vals;
  }
}

void mkdirs(const std::string& file) {
  for (size_t i = 1; i < file.size(); ++i)
    if (file[i] == '/') (void)mkdir(file.substr(0, i).c_str(), 0755);
}

bool save_locked() {
  const std::string& p = path_locked();
  if (p.empty()) return true;
  mkdirs(p);
  const std::string tmp = p + ".tmp." + std::to_string((long)getpid());
  {
    std::ofstream f(tmp, std::ios::trunc);
    if (!f) return false;
    f << "# tuner choices of libmr: kind|arch|device|compute units|n|values\n";
    for (const auto& kv : g_store) {
      f << kv.first << "|";
      for (size_t i = 0; i < kv.second.size(); ++i) f << (i ? "," : "") << kv.second[i];
      f << "\n";
    }
    if (!f) return false;
  }
  return std::rename(tmp.c_str(), p.c_str()) == 0;
}

bool dev_key(int dev, DevKey& k) {
  {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_devs.find(dev);
    if (it != g_devs.end()) {
      k = it->second;
      return true;
    }
  }
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return false;
  // the device is named by its memory size rather than its product name, which is empty in
  // some environments (under a profiler) and would make the same device look like another
  k.arch = prop.gcnArchName;
  k.name = std::to_string((long long)((prop.totalGlobalMem + (1ull << 29)) >> 30)) + "GiB";
  k.cus = prop.multiProcessorCount;
  std::lock_guard<std::mutex> lk(g_mu);
  g_devs[dev] = k;
  return true;
}

bool lookup_key(const std::string& key, std::vector<int>& vals) {
  std::lock_guard<std::mutex> lk(g_mu);
  load_locked();
  auto it = g_store.find(key);
  if (it != g_store.end()) {
    vals = it->second;
    return true;
  }
  it = g_defaults.find(key);
  if (it == g_defaults.end()) return false;
  vals = it->second;
  // the record file lists every choice in use, shipped ones included
  g_store[key] = vals;
  (void)save_locked();
  return true;
}

bool record_key(const std::string& key, const std::vector<int>& vals) {
  std::lock_guard<std::mutex> lk(g_mu);
  load_locked();
  g_store[key] = vals;
  return save_locked();
}

}  // namespace

bool tuning_lookup(const char* kind, int dev, int n, std::vector<int>& vals) {
  DevKey k;
  if (!dev_key(dev, k)) return false;
  return lookup_key(make_key(kind, k.arch, k.name, k.cus, n), vals);
}

void tuning_record(const char* kind, int dev, int n, const std::vector<int>& vals) {
  DevKey k;
  if (!dev_key(dev, k)) return;
  (void)record_key(make_key(kind, k.arch, k.name, k.cus, n), vals);   // a file that cannot be written is not an error
}

int tuning_generation() {
  std::lock_guard<std::mutex> lk(g_mu);
  return g_generation;
}

}  // namespace mr

extern "C" {

int mr_tuning_file(const char* path) {
  std::lock_guard<std::mutex> lk(mr::g_mu);
  mr::g_store.clear();
  mr::g_loaded = false;
  mr::g_defaults.clear();
  mr::g_defaults_loaded = false;
  ++mr::g_generation;
  if (path) {
    mr::g_path = path;
    mr::g_path_set = true;
  } else {
    mr::g_path_set = false;   // back to the default location, resolved on next use
  }
  return MR_OK;
}

const char* mr_tuning_file_path(void) {
  std::lock_guard<std::mutex> lk(mr::g_mu);
  return mr::path_locked().c_str();
}

int mr_tuning_store(const char* kind, const char* arch, const char* device, int cus, int n, const int* vals,
                    int count) {
  if (!kind || !arch || !device || !vals || count < 1 || count > 64 || n < 1 || cus < 0)
    return mr::fail(MR_EINVAL, "mr_tuning_store: bad argument");
  const std::vector<int> v(vals, vals + count);
  if (!mr::record_key(mr::make_key(kind, arch, device, cus, n), v))
    return mr::fail(MR_EINVAL, "mr_tuning_store: cannot write %s", mr_tuning_file_path());
  return MR_OK;
}

int mr_tuning_lookup(const char* kind, const char* arch, const char* device, int cus, int n, int* vals, int max_count,
                     int* count) {
  if (!kind || !arch || !device || !count || (max_count > 0 && !vals) || max_count < 0)
    return mr::fail(MR_EINVAL, "mr_tuning_lookup: bad argument");
  std::vector<int> v;
  *count = 0;
  if (!mr::lookup_key(mr::make_key(kind, arch, device, cus, n), v)) return MR_OK;
  if ((int)v.size() > max_count) return mr::fail(MR_EINVAL, "mr_tuning_lookup: %d values do not fit", (int)v.size());
  for (size_t i = 0; i < v.size(); ++i) vals[i] = v[i];
  *count = (int)v.size();
  return MR_OK;
}

}  // extern "C"
