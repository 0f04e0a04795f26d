// Persistent store of the tuners' choices (see tune_cache.h).
#include "tune_cache.h"

#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <sstream>
#include <string>

namespace rfk {

namespace {

std::mutex g_mu;
std::map<std::string, std::vector<int>> g_table;
bool g_loaded = false;

std::string arch_name() {
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
    return "unknown";
  std::string a = prop.gcnArchName;
  const size_t colon = a.find(':');
  return colon == std::string::npos ? a : a.substr(0, colon);
}

std::string make_key(const char* kind, const std::vector<int64_t>& key) {
  std::ostringstream s;
  s << arch_name() << ' ' << kind;
  for (int64_t v : key) s << ' ' << v;
  return s.str();
}

// Reads the file once (caller holds g_mu).
void load_file() {
  if (g_loaded) return;
  g_loaded = true;
  const char* path = getenv("REFINE_TUNE_CACHE");
  if (!path || !*path) return;
  FILE* f = fopen(path, "r");
  if (!f) return;
  char line[512];
  while (fgets(line, sizeof line, f)) {
    char* sep = strchr(line, ':');
    if (!sep) continue;
    *sep = '\0';
    std::string k(line);
    while (!k.empty() && k.back() == ' ') k.pop_back();
    std::istringstream vs(sep + 1);
    std::vector<int> v;
    int x;
    while (vs >> x) v.push_back(x);
    if (!k.empty() && !v.empty()) g_table[k] = v;
  }
  fclose(f);
}

}  // namespace

bool tune_cache_get(const char* kind, const std::vector<int64_t>& key, std::vector<int>* value) {
  const std::string k = make_key(kind, key);
  std::lock_guard<std::mutex> lock(g_mu);
  load_file();
  auto it = g_table.find(k);
  if (it == g_table.end()) return false;
  *value = it->second;
  if (getenv("REFINE_LOG")) fprintf(stderr, "refine: tuning cache hit: %s\n", k.c_str());
  return true;
}

void tune_cache_put(const char* kind, const std::vector<int64_t>& key,
                    const std::vector<int>& value) {
  const std::string k = make_key(kind, key);
  std::lock_guard<std::mutex> lock(g_mu);
  load_file();
  g_table[k] = value;
  const char* path = getenv("REFINE_TUNE_CACHE");
  if (!path || !*path) return;
  FILE* f = fopen(path, "a");
  if (!f) return;
  fprintf(f, "%s :", k.c_str());
  for (int v : value) fprintf(f, " %d", v);
  fprintf(f, "\n");
  fclose(f);
}

}  // namespace rfk
