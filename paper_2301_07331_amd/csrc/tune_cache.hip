// tune_cache.hip -- the autotuner's cache (see tune_cache.hpp).
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "tune_cache.hpp"

namespace hlc {
namespace {

std::mutex g_mu;
std::vector<std::pair<std::string, std::vector<double>>> g_tune;
bool g_loaded = false;

// Reads {"key": [numbers] or number, ...}; anything it does not understand
// ends the read (the cache is then only what was read so far).
void load_locked() {
  if (g_loaded) return;
  g_loaded = true;
  const char* path = std::getenv("HLC_TUNE_CACHE");
  if (!path) return;
  FILE* f = std::fopen(path, "r");
  if (!f) return;
  std::string t;
  char buf[4096];
  size_t n;
  while ((n = std::fread(buf, 1, sizeof buf, f)) > 0) t.append(buf, n);
  std::fclose(f);
  size_t i = 0;
  auto skip = [&]() {
    while (i < t.size() && (t[i] == ' ' || t[i] == '\n' || t[i] == '\r' || t[i] == '\t' || t[i] == ','))
      ++i;
  };
  auto number = [&](double* v) {
    const char* s = t.c_str() + i;
    char* e = nullptr;
    *v = std::strtod(s, &e);
    if (e == s) return false;
    i += (size_t)(e - s);
    return true;
  };
  skip();
  if (i >= t.size() || t[i] != '{') return;
  ++i;
  while (true) {
    skip();
    if (i >= t.size() || t[i] != '"') return;
    const size_t a = i + 1, b = t.find('"', a);
    if (b == std::string::npos) return;
    std::string key = t.substr(a, b - a);
    i = b + 1;
    skip();
    if (i >= t.size() || t[i] != ':') return;
    ++i;
    skip();
    std::vector<double> vals;
    if (i < t.size() && t[i] == '[') {
      ++i;
      while (true) {
        skip();
        if (i < t.size() && t[i] == ']') {
          ++i;
          break;
        }
        double v;
        if (!number(&v)) return;
        vals.push_back(v);
      }
    } else {
      double v;
      if (!number(&v)) return;
      vals.push_back(v);
    }
    g_tune.emplace_back(std::move(key), std::move(vals));
  }
}

void save_locked() {
  const char* path = std::getenv("HLC_TUNE_CACHE");
  if (!path) return;
  FILE* f = std::fopen(path, "w");
  if (!f) return;
  std::fprintf(f, "{\n");
  for (size_t k = 0; k < g_tune.size(); ++k) {
    std::fprintf(f, "  \"%s\": [", g_tune[k].first.c_str());
    for (size_t j = 0; j < g_tune[k].second.size(); ++j)
      std::fprintf(f, "%s%.9g", j ? ", " : "", g_tune[k].second[j]);
    std::fprintf(f, "]%s\n", k + 1 < g_tune.size() ? "," : "");
  }
  std::fprintf(f, "}\n");
  std::fclose(f);
}

}  // namespace

bool tune_lookup(const std::string& bucket, std::vector<double>* values) {
  std::lock_guard<std::mutex> lk(g_mu);
  load_locked();
  for (auto& kv : g_tune)
    if (kv.first == bucket) {
      *values = kv.second;
      return true;
    }
  return false;
}

void tune_store(const std::string& bucket, const std::vector<double>& values) {
  std::lock_guard<std::mutex> lk(g_mu);
  load_locked();
  bool found = false;
  for (auto& kv : g_tune)
    if (kv.first == bucket) {
      kv.second = values;
      found = true;
    }
  if (!found) g_tune.emplace_back(bucket, values);
  save_locked();
}

std::string tune_device_tag() {
  // the properties query is slow: once per device
  constexpr int MAXDEV = 64;
  static std::string tags[MAXDEV];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    (void)hipGetLastError();
    return "unknown|cu0";
  }
  std::lock_guard<std::mutex> lk(g_mu);
  if (dev >= 0 && dev < MAXDEV && !tags[dev].empty()) return tags[dev];
  hipDeviceProp_t p;
  if (hipGetDeviceProperties(&p, dev) != hipSuccess) {
    (void)hipGetLastError();
    return "unknown|cu0";
  }
  std::string arch = p.gcnArchName;
  const size_t colon = arch.find(':');  // drop target features (":sramecc+:xnack-")
  if (colon != std::string::npos) arch.resize(colon);
  std::string tag = arch + "|cu" + std::to_string(p.multiProcessorCount);
  if (dev >= 0 && dev < MAXDEV) tags[dev] = tag;
  return tag;
}

}  // namespace hlc
