// Launch-shape registry for the pair kernels: built-in defaults, shapes chosen
// by the autotuner (abacus_nf_autotune in api.hip), and an optional on-disk
// cache (ABACUS_NF_TUNE_CACHE) so a tuned shape survives the process.
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>

#include "nf_internal.h"

namespace anf {

KernelConfig default_config(int kernel) {
  KernelConfig c;
  c.unroll = kernel == 0 ? 4 : 2;
  c.pipeline = 0;
  c.span = kDefaultSpan;
  c.grid_mult = 1;
  c.split = 1;
  return c;
}

bool config_valid(int kernel, const KernelConfig& c) {
  const bool unroll_ok = kernel == 0 ? (c.unroll == 2 || c.unroll == 4 || c.unroll == 8)
                                     : (c.unroll == 2 || c.unroll == 3 || c.unroll == 4);
  return unroll_ok && (c.pipeline == 0 || c.pipeline == 1) && c.span >= 1 &&
         c.span <= kMaxSpan && (c.grid_mult == 1 || c.grid_mult == 2) &&
         (c.split == 0 || c.split == 1);
}

namespace {

using Key = std::tuple<std::string, int, uint32_t, int, int64_t, int64_t, uint64_t>;

std::mutex g_mu;
std::map<Key, KernelConfig> g_table;
bool g_cache_loaded = false;

// Architecture name of the current device (cached per device; "unknown" if
// there is no device).  Called with g_mu held.
std::string device_arch() {
  static std::map<int, std::string> names;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return "unknown";
  auto it = names.find(dev);
  if (it != names.end()) return it->second;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
  std::string a = prop.gcnArchName;
  const size_t colon = a.find(':');
  a = colon == std::string::npos ? a : a.substr(0, colon);
  names[dev] = a;
  return a;
}

Key make_key(const TuneKey& k) {
  return Key(device_arch(), k.kernel, k.mode, k.nboxes, k.n_total, k.cells_total, k.shape_hash);
}

const char* cache_path() {
  const char* p = std::getenv("ABACUS_NF_TUNE_CACHE");
  return (p && *p) ? p : nullptr;
}

// One line per entry: arch kernel mode nboxes n cells hash unroll pipeline span grid split
void load_cache_locked() {
  if (g_cache_loaded) return;
  g_cache_loaded = true;
  const char* path = cache_path();
  if (!path) return;
  FILE* f = std::fopen(path, "r");
  if (!f) return;
  char arch[64];
  int kernel, nboxes;
  unsigned mode;
  long long n, cells;
  unsigned long long hash;
  KernelConfig c;
  while (std::fscanf(f, "%63s %d %u %d %lld %lld %llu %d %d %d %d %d", arch, &kernel, &mode,
                     &nboxes, &n, &cells, &hash, &c.unroll, &c.pipeline, &c.span, &c.grid_mult,
                     &c.split) == 12) {
    if (config_valid(kernel, c))
      g_table[Key(arch, kernel, mode, nboxes, n, cells, hash)] = c;
  }
  std::fclose(f);
}

}  // namespace

KernelConfig lookup_config(const TuneKey& k) {
  std::lock_guard<std::mutex> lock(g_mu);
  load_cache_locked();
  auto it = g_table.find(make_key(k));
  return it == g_table.end() ? default_config(k.kernel) : it->second;
}

void store_config(const TuneKey& k, const KernelConfig& c, bool persist) {
  std::lock_guard<std::mutex> lock(g_mu);
  load_cache_locked();
  const Key key = make_key(k);
  g_table[key] = c;
  const char* path = persist ? cache_path() : nullptr;
  if (!path) return;
  FILE* f = std::fopen(path, "a");
  if (!f) return;
  std::fprintf(f, "%s %d %u %d %lld %lld %llu %d %d %d %d %d\n", std::get<0>(key).c_str(),
               k.kernel, k.mode, k.nboxes, (long long)k.n_total, (long long)k.cells_total,
               (unsigned long long)k.shape_hash, c.unroll, c.pipeline, c.span, c.grid_mult,
               c.split);
  std::fclose(f);
}

void clear_config(const TuneKey& k) {
  std::lock_guard<std::mutex> lock(g_mu);
  load_cache_locked();
  g_table.erase(make_key(k));
}

}  // namespace anf
