// Tile choices picked by measurement.  The NaivePT contraction and the fused
// reconstruction split the voxels of every relabelling group into `nc`
// chunks (one workgroup each); the planners start from a rule of thumb (about
// 1,280 workgroups) and the autotuner times the candidates around it on the
// caller's own shape, keeping the fastest in a table keyed by kernel and
// shape.  The table can be written to and read from a text file; a file named
// by the RPT_TUNE_CACHE environment variable is read on first use.
#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>
#include <tuple>

#include "rpt_internal.h"

namespace rpt {

namespace {
using Key = std::tuple<int, int64_t, int64_t, int, int>;  // kernel, v, L, dim, variant
std::mutex g_tune_mu;
std::map<Key, int> g_tuned;
bool g_env_read = false;

int load_file(const char* path) {  // caller holds g_tune_mu
  FILE* f = std::fopen(path, "r");
  if (!f) return -1;
  int count = 0;
  int kernel, dim, variant, nc;
  long long v, L;
  while (std::fscanf(f, "%d %lld %lld %d %d %d", &kernel, &v, &L, &dim, &variant, &nc) == 6) {
    if (nc >= 8 && nc % 8 == 0) {
      g_tuned[Key(kernel, v, L, dim, variant)] = nc;
      ++count;
    }
  }
  std::fclose(f);
  return count;
}

void read_env_once() {  // caller holds g_tune_mu
  if (g_env_read) return;
  g_env_read = true;
  const char* path = std::getenv("RPT_TUNE_CACHE");
  if (path && *path) (void)load_file(path);
}
}  // namespace

int chunk_candidates(int64_t nc_heur, int64_t ncmax, int* out) {
  int m = 0;
  for (int64_t f : {1, 2, 4, 8, 16, 32}) {  // nc / 2, nc, 2 nc, ..., 16 nc
    int64_t c = round_up(nc_heur * f / 2, 8);
    if (c > ncmax) c = ncmax;
    if (c < 8) c = 8;
    if (m == 0 || out[m - 1] != c) out[m++] = static_cast<int>(c);
  }
  return m;
}

int64_t chunk_cap(int64_t nc_heur, int64_t ncmax) {
  int c[kMaxChunkCandidates];
  const int m = chunk_candidates(nc_heur, ncmax, c);
  return c[m - 1];
}

int tuned_chunks(int kernel, int64_t v, int64_t L, int dim, int variant) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  read_env_once();
  auto it = g_tuned.find(Key(kernel, v, L, dim, variant));
  return it == g_tuned.end() ? 0 : it->second;
}

void set_tuned_chunks(int kernel, int64_t v, int64_t L, int dim, int variant, int nc) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  read_env_once();
  g_tuned[Key(kernel, v, L, dim, variant)] = nc;
}

}  // namespace rpt

using namespace rpt;

extern "C" {

int rpt_autotune_save(const char* path) {
  if (!path) return -1;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  FILE* f = std::fopen(path, "w");
  if (!f) return -1;
  int count = 0;
  for (const auto& kv : g_tuned) {
    std::fprintf(f, "%d %lld %lld %d %d %d\n", std::get<0>(kv.first), static_cast<long long>(std::get<1>(kv.first)),
                 static_cast<long long>(std::get<2>(kv.first)), std::get<3>(kv.first), std::get<4>(kv.first),
                 kv.second);
    ++count;
  }
  std::fclose(f);
  return count;
}

int rpt_autotune_load(const char* path) {
  if (!path) return -1;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_env_read = true;
  return load_file(path);
}

void rpt_autotune_clear(void) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_env_read = true;
  g_tuned.clear();
}

int rpt_autotune_count(void) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  read_env_once();
  return static_cast<int>(g_tuned.size());
}

}  // extern "C"
