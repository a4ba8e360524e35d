// stats.cpp -- optional per-kernel timing of the library's own launches.
//
// When enabled, each launch is bracketed by two HIP events recorded on the
// launch's stream; ntt_stats_collect() waits for the recorded events and
// returns, per kernel name, the launch count, the coefficient words covered and
// the summed device time.  Disabled (the default), a launch costs one atomic
// load more.
#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "ntt_internal.hpp"

namespace {

struct Pending {
  std::string name;
  uint64_t words;
  hipEvent_t a, b;
};

struct Agg {
  uint64_t launches = 0;
  uint64_t words = 0;
  double ms = 0.0;
};

std::atomic<bool> g_on{false};
std::mutex g_mu;
std::vector<Pending> g_pending;
std::map<std::string, Agg> g_agg;
std::vector<hipEvent_t> g_pool;

hipEvent_t take_event() {
  if (!g_pool.empty()) {
    hipEvent_t e = g_pool.back();
    g_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

}  // namespace

namespace nttk {

bool stats_enabled() { return g_on.load(std::memory_order_relaxed); }

LaunchTimer::LaunchTimer(const char* kind, const char* cls, int size_log, bool inv, bool two_pass,
                         uint64_t words, hipStream_t s) {
  if (!kind || !stats_enabled()) return;
  char name[96];
  snprintf(name, sizeof(name), "%s_%s_%s_log%d%s", kind, inv ? "inv" : "fwd", cls, size_log,
           two_pass ? "_2pass" : "");
  std::lock_guard<std::mutex> lk(g_mu);
  hipEvent_t a = take_event(), b = take_event();
  if (!a || !b) return;
  if (hipEventRecord(a, s) != hipSuccess) return;
  g_pending.push_back(Pending{name, words, a, b});
  slot_ = (int)g_pending.size() - 1;
  s_ = s;
  on_ = true;
}

LaunchTimer::~LaunchTimer() {
  if (!on_) return;
  std::lock_guard<std::mutex> lk(g_mu);
  if (slot_ >= 0 && slot_ < (int)g_pending.size()) (void)hipEventRecord(g_pending[slot_].b, s_);
}

}  // namespace nttk

extern "C" {

ntt_status ntt_stats_enable(int on) {
  g_on.store(on != 0);
  return NTT_OK;
}

ntt_status ntt_stats_reset(void) {
  std::lock_guard<std::mutex> lk(g_mu);
  for (auto& p : g_pending) {
    (void)hipEventSynchronize(p.b);
    g_pool.push_back(p.a);
    g_pool.push_back(p.b);
  }
  g_pending.clear();
  g_agg.clear();
  return NTT_OK;
}

ntt_status ntt_stats_collect(ntt_kernel_stat* out, uint32_t cap, uint32_t* count) {
  if (!count) return nttk::fail(NTT_EINVAL, "null count");
  std::lock_guard<std::mutex> lk(g_mu);
  for (auto& p : g_pending) {
    hipError_t e = hipEventSynchronize(p.b);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, p.a, p.b);
    if (e != hipSuccess) return nttk::hip_fail(e, "stats event");
    Agg& g = g_agg[p.name];
    g.launches += 1;
    g.words += p.words;
    g.ms += ms;
    g_pool.push_back(p.a);
    g_pool.push_back(p.b);
  }
  g_pending.clear();
  uint32_t i = 0;
  for (const auto& kv : g_agg) {
    if (out && i < cap) {
      std::memset(&out[i], 0, sizeof(out[i]));
      std::strncpy(out[i].name, kv.first.c_str(), sizeof(out[i].name) - 1);
      out[i].launches = kv.second.launches;
      out[i].words = kv.second.words;
      out[i].total_ms = kv.second.ms;
    }
    ++i;
  }
  *count = i;
  return NTT_OK;
}

}  // extern "C"
