// Tuning cache of the uneven-batch plans: the launch configuration that the
// autotuner picked for a size class, keyed by the device and by what
// describes the class (kind, number of right-hand sides, instance count,
// smallest, largest and summed order), kept in process memory and written
// to / read from a plain text file so that a later process skips the
// timing runs.  Host code only; every entry point takes the table's mutex.
//
// File format (one entry per line, '#' starts a comment line):
//   arch cus kind nrhs count nmin nmax nsum cfg ms
// arch is the device's architecture name (no blanks), cus its compute-unit
// count, cfg the configuration value of blasfeo_hip_plan_config and ms the
// time the autotuner measured for it (informative).
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>

#include "plan.hpp"

namespace bh {
namespace {

using Key = std::tuple<std::string, int, int, int, int, int, int, long long>;
struct Val {
  int cfg;
  float ms;
};

std::mutex &mu() {
  static std::mutex m;
  return m;
}
std::map<Key, Val> &table() {
  static std::map<Key, Val> t;
  return t;
}
long long g_hits = 0, g_misses = 0;

Key to_key(const TuneKey &k) {
  return Key(k.arch, k.cus, k.kind, k.nrhs, k.count, k.nmin, k.nmax, k.nsum);
}

}  // namespace

int tune_key_device(TuneKey &k) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return -1;
  hipDeviceProp_t pr;
  if (hipGetDeviceProperties(&pr, dev) != hipSuccess) return -1;
  std::string a(pr.gcnArchName);
  for (char &c : a)
    if (c == ' ' || c == '\t') c = '_';
  k.arch = a.empty() ? "unknown" : a;
  k.cus = pr.multiProcessorCount;
  return 0;
}

bool tune_lookup(const TuneKey &k, int *cfg) {
  std::lock_guard<std::mutex> g(mu());
  auto it = table().find(to_key(k));
  if (it == table().end()) {
    ++g_misses;
    return false;
  }
  ++g_hits;
  *cfg = it->second.cfg;
  return true;
}

void tune_store(const TuneKey &k, int cfg, float ms) {
  std::lock_guard<std::mutex> g(mu());
  table()[to_key(k)] = Val{cfg, ms};
}

}  // namespace bh

extern "C" {

int blasfeo_hip_tune_cache_load(const char *path) {
  if (!path) return -1;
  FILE *f = std::fopen(path, "r");
  if (!f) return 0;  // no file yet: an empty cache
  std::map<bh::Key, bh::Val> got;
  char line[512];
  int bad = 0;
  while (std::fgets(line, sizeof line, f)) {
    const size_t len = std::strlen(line);
    if (len + 1 == sizeof line && line[len - 1] != '\n') {
      bad = 1;
      break;
    }
    const char *s = line;
    while (*s == ' ' || *s == '\t') ++s;
    if (*s == '#' || *s == '\n' || *s == '\0') continue;
    char arch[256];
    int cus, kind, nrhs, count, nmin, nmax, cfg, used = 0;
    long long nsum;
    float ms;
    if (std::sscanf(s, "%255s %d %d %d %d %d %d %lld %d %f %n", arch, &cus, &kind, &nrhs,
                    &count, &nmin, &nmax, &nsum, &cfg, &ms, &used) != 10 ||
        s[used] != '\0' || !bh::tune_cfg_valid(kind, cfg) || cus < 1 || nrhs < 0 ||
        count < 1 || nmin < 1 || nmax < nmin) {
      bad = 1;
      break;
    }
    got[bh::Key(arch, cus, kind, nrhs, count, nmin, nmax, nsum)] = bh::Val{cfg, ms};
  }
  std::fclose(f);
  if (bad) return -2;
  std::lock_guard<std::mutex> g(bh::mu());
  for (const auto &e : got) bh::table()[e.first] = e.second;
  return (int)got.size();
}

int blasfeo_hip_tune_cache_save(const char *path) {
  if (!path) return -1;
  std::lock_guard<std::mutex> g(bh::mu());
  const std::string tmp = std::string(path) + ".tmp";
  FILE *f = std::fopen(tmp.c_str(), "w");
  if (!f) return -2;
  int ok = std::fprintf(f, "# arch cus kind nrhs count nmin nmax nsum cfg ms\n") > 0;
  for (const auto &e : bh::table()) {
    const bh::Key &k = e.first;
    ok = ok && std::fprintf(f, "%s %d %d %d %d %d %d %lld %d %.4f\n", std::get<0>(k).c_str(),
                            std::get<1>(k), std::get<2>(k), std::get<3>(k), std::get<4>(k),
                            std::get<5>(k), std::get<6>(k), std::get<7>(k), e.second.cfg,
                            e.second.ms) > 0;
  }
  ok = (std::fclose(f) == 0) && ok;
  if (!ok || std::rename(tmp.c_str(), path) != 0) {
    std::remove(tmp.c_str());
    return -2;
  }
  return (int)bh::table().size();
}

int blasfeo_hip_tune_cache_clear(void) {
  std::lock_guard<std::mutex> g(bh::mu());
  bh::table().clear();
  bh::g_hits = bh::g_misses = 0;
  return 0;
}

int blasfeo_hip_tune_cache_stats(long long *entries, long long *hits, long long *misses) {
  std::lock_guard<std::mutex> g(bh::mu());
  if (entries) *entries = (long long)bh::table().size();
  if (hits) *hits = bh::g_hits;
  if (misses) *misses = bh::g_misses;
  return 0;
}

}  // extern "C"
