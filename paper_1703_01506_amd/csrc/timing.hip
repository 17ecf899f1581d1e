// Per-stage timing: while enabled, every kernel stage records a pair of HIP
// events on the caller's stream; queries wait for those events and sum their
// elapsed times.  Off by default (no events are created when disabled);
// events are pooled and reused after a reset.
#include <map>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "rpt_internal.h"

namespace rpt {

namespace {
std::mutex g_mu;
bool g_on = false;
std::map<std::string, std::vector<std::pair<hipEvent_t, hipEvent_t>>> g_ev;
std::vector<hipEvent_t> g_pool;  // events of earlier rounds, reused (creating one is not cheap)

hipEvent_t take_event() {  // caller holds g_mu
  if (!g_pool.empty()) {
    hipEvent_t e = g_pool.back();
    g_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  return hipEventCreate(&e) == hipSuccess ? e : nullptr;
}
}  // namespace

StageScope::StageScope(const char* name, hipStream_t s) : name_(name), s_(s), start_(nullptr) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_on) return;
  start_ = take_event();
  if (start_ && hipEventRecord(start_, s_) != hipSuccess) {
    g_pool.push_back(start_);
    start_ = nullptr;
  }
}

StageScope::~StageScope() {
  if (!start_) return;
  std::lock_guard<std::mutex> lk(g_mu);
  hipEvent_t end = take_event();
  if (!end || hipEventRecord(end, s_) != hipSuccess) {
    g_pool.push_back(start_);
    if (end) g_pool.push_back(end);
    return;
  }
  g_ev[name_].emplace_back(start_, end);
}

}  // namespace rpt

using namespace rpt;

extern "C" {

void rpt_timing_enable(int on) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_on = on != 0;
}

void rpt_timing_reset(void) {
  std::lock_guard<std::mutex> lk(g_mu);
  for (auto& kv : g_ev)
    for (auto& pr : kv.second) {
      (void)hipEventSynchronize(pr.second);
      g_pool.push_back(pr.first);
      g_pool.push_back(pr.second);
    }
  g_ev.clear();
}

int rpt_timing_query(const char* stage, double* total_ms, int64_t* count) {
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_ev.find(stage ? stage : "");
  if (it == g_ev.end()) return -1;
  double tot = 0.0;
  for (auto& pr : it->second) {
    float ms = 0.0f;
    if (hipEventSynchronize(pr.second) != hipSuccess) return -2;
    if (hipEventElapsedTime(&ms, pr.first, pr.second) != hipSuccess) return -2;
    tot += ms;
  }
  if (total_ms) *total_ms = tot;
  if (count) *count = static_cast<int64_t>(it->second.size());
  return 0;
}

int rpt_timing_stages(char* buf, size_t len) {
  std::lock_guard<std::mutex> lk(g_mu);
  std::string all;
  for (auto& kv : g_ev) {
    if (!all.empty()) all += ",";
    all += kv.first;
  }
  if (buf && len) {
    const size_t n = all.size() < len - 1 ? all.size() : len - 1;
    all.copy(buf, n);
    buf[n] = '\0';
  }
  return static_cast<int>(all.size());
}

}  // extern "C"
