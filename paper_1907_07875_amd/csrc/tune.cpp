// Tuning cache and candidate timing (see tune.hpp).
#include "tune.hpp"

#include <sys/stat.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <set>
#include <sstream>

namespace gft {

uint64_t fnv1a(const void *data, size_t n, uint64_t h) {
  const unsigned char *p = static_cast<const unsigned char *>(data);
  for (size_t i = 0; i < n; ++i) {
    h ^= p[i];
    h *= 1099511628211ull;
  }
  return h;
}

std::string device_tag(int dev) {
  hipDeviceProp_t prop;
  std::string arch = "unknown";
  if (hipGetDeviceProperties(&prop, dev) == hipSuccess) {
    arch = prop.gcnArchName;
    const size_t colon = arch.find(':');   // drop feature suffixes (":sramecc+:xnack-")
    if (colon != std::string::npos) arch.resize(colon);
  }
  int cus = 0;
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  return arch + ":" + std::to_string(cus);
}

namespace {

std::mutex g_mu;
std::map<std::string, std::vector<int32_t>> g_mem;
std::set<std::string> g_loaded;                             // cache files read into g_mem
std::set<std::pair<std::string, std::string>> g_in_file;   // (file, key) already in that file

// The cache file, or "" for memory only.
std::string cache_path() {
  const char *env = std::getenv("GFT_TUNE_CACHE");
  if (env) return (!*env || !std::strcmp(env, "off")) ? std::string() : std::string(env);
  const char *home = std::getenv("HOME");
  if (!home || !*home) return std::string();
  return std::string(home) + "/.cache/libgft/tuning-v2.txt";
}

void make_parent_dirs(const std::string &path) {
  for (size_t i = 1; i < path.size(); ++i)
    if (path[i] == '/') (void)mkdir(path.substr(0, i).c_str(), 0755);
}

// Append "key v0 v1 ..." to the cache file once per (file, key).  Caller holds g_mu.
void write_line(const std::string &path, const std::string &key, const std::vector<int32_t> &values) {
  if (path.empty() || g_in_file.count({path, key})) return;
  make_parent_dirs(path);
  FILE *f = std::fopen(path.c_str(), "a");
  if (!f) return;   // an unwritable cache only costs re-timing
  std::fprintf(f, "%s", key.c_str());
  for (int32_t v : values) std::fprintf(f, " %d", v);
  std::fprintf(f, "\n");
  std::fclose(f);
  g_in_file.insert({path, key});
}

// Lines "key v0 v1 ...": later lines win.  Caller holds g_mu.
void load_file(const std::string &path) {
  if (path.empty() || g_loaded.count(path)) return;
  g_loaded.insert(path);
  FILE *f = std::fopen(path.c_str(), "r");
  if (!f) return;
  char line[1024];
  while (std::fgets(line, sizeof line, f)) {
    std::istringstream is(line);
    std::string key;
    if (!(is >> key)) continue;
    std::vector<int32_t> v;
    int32_t x;
    while (is >> x) v.push_back(x);
    if (!v.empty()) {
      g_mem[key] = v;
      g_in_file.insert({path, key});
    }
  }
  std::fclose(f);
}

}  // namespace

bool tune_cache_get(const std::string &key, std::vector<int32_t> &values) {
  std::lock_guard<std::mutex> lock(g_mu);
  const std::string path = cache_path();
  load_file(path);
  auto it = g_mem.find(key);
  if (it == g_mem.end()) return false;
  values = it->second;
  write_line(path, key, values);   // a choice made under another cache file
  return true;
}

void tune_cache_put(const std::string &key, const std::vector<int32_t> &values) {
  std::lock_guard<std::mutex> lock(g_mu);
  const std::string path = cache_path();
  load_file(path);
  g_mem[key] = values;
  g_in_file.erase({path, key});
  write_line(path, key, values);
}

int time_candidates(int ncand, int base, const std::function<hipError_t(int, hipStream_t)> &launch,
                    hipStream_t st) {
  if (ncand <= 0 || base < 0 || base >= ncand) return -1;
  hipEvent_t ev[2] = {nullptr, nullptr};
  bool okay = hipEventCreate(&ev[0]) == hipSuccess && hipEventCreate(&ev[1]) == hipSuccess;
  std::vector<float> best(ncand, 0.0f);
  for (int w = 0; w < 6 && okay; ++w)   // warm-up: clocks, code, caches
    okay = launch(base, st) == hipSuccess;
  for (int round = 0; round < 4 && okay; ++round)
    for (int c = 0; c < ncand && okay; ++c) {
      okay = hipEventRecord(ev[0], st) == hipSuccess;
      for (int r = 0; r < 2 && okay; ++r) okay = launch(c, st) == hipSuccess;
      float ms = 0.0f;
      okay = okay && hipEventRecord(ev[1], st) == hipSuccess && hipEventSynchronize(ev[1]) == hipSuccess &&
             hipEventElapsedTime(&ms, ev[0], ev[1]) == hipSuccess;
      if (okay && (best[c] == 0.0f || ms < best[c])) best[c] = ms;
    }
  for (hipEvent_t e : ev)
    if (e) (void)hipEventDestroy(e);
  if (!okay) {
    (void)hipGetLastError();
    return -1;
  }
  int pick = base;
  for (int c = 0; c < ncand; ++c)
    if (best[c] < 0.97f * best[pick]) pick = c;
  return pick;
}

}  // namespace gft
