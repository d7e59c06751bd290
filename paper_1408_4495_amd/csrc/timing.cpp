// Optional per-kernel timing: when enabled, every launch made through
// LSP_LAUNCH carries two HIP events that the runtime records at the kernel's
// start and end on the launch's own stream; lsp_timing_get() waits for them
// and reports, per kernel name and element size, the summed kernel time and
// the launch count.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "lsp_common.h"

namespace lsp {

namespace {

struct Pending {
  std::string key;
  hipEvent_t a, b;
};

struct Registry {
  std::mutex mu;
  std::atomic<bool> on{false};
  std::vector<hipEvent_t> pool;
  std::vector<Pending> pending;
  std::map<std::string, std::pair<double, long long>> totals;
  std::vector<std::string> order;

  hipEvent_t take() {
    if (!pool.empty()) { hipEvent_t e = pool.back(); pool.pop_back(); return e; }
    hipEvent_t e;
    LSP_HIP(hipEventCreate(&e));
    return e;
  }
  void collect() {
    for (auto& p : pending) {
      LSP_HIP(hipEventSynchronize(p.b));
      float ms = 0.f;
      LSP_HIP(hipEventElapsedTime(&ms, p.a, p.b));
      auto it = totals.find(p.key);
      if (it == totals.end()) { totals[p.key] = {ms, 1}; order.push_back(p.key); }
      else { it->second.first += ms; it->second.second += 1; }
      pool.push_back(p.a);
      pool.push_back(p.b);
    }
    pending.clear();
  }
};

Registry& reg() {
  static Registry r;
  return r;
}

}  // namespace

KTimer::KTimer(const char* name, int esize, hipStream_t st) : st_(st), a_(nullptr), b_(nullptr) {
  Registry& r = reg();
  if (!r.on.load(std::memory_order_relaxed)) return;
  std::lock_guard<std::mutex> g(r.mu);
  key_ = std::string(name) + (esize == 16 ? " [c128]" : esize == 8 ? " [c64]" : "");
  a_ = r.take();
  b_ = r.take();
}

KTimer::~KTimer() {
  if (!a_) return;
  Registry& r = reg();
  std::lock_guard<std::mutex> g(r.mu);
  if (launched_) {
    r.pending.push_back({key_, a_, b_});
  } else {  // the launch failed: the events were never recorded
    r.pool.push_back(a_);
    r.pool.push_back(b_);
  }
}

}  // namespace lsp

extern "C" {

lsp_status lsp_timing_enable(int enable) {
  lsp::reg().on.store(enable != 0);
  return LSP_OK;
}

lsp_status lsp_timing_reset(void) {
  lsp::Registry& r = lsp::reg();
  std::lock_guard<std::mutex> g(r.mu);
  try {
    r.collect();
  } catch (const lsp::Error& e) {
    return e.status;
  }
  r.totals.clear();
  r.order.clear();
  return LSP_OK;
}

int lsp_timing_count(void) {
  lsp::Registry& r = lsp::reg();
  std::lock_guard<std::mutex> g(r.mu);
  try {
    r.collect();
  } catch (const lsp::Error&) {
    return -1;
  }
  return (int)r.order.size();
}

lsp_status lsp_timing_get(int i, char* name, size_t len, double* total_ms, long long* launches) {
  lsp::Registry& r = lsp::reg();
  std::lock_guard<std::mutex> g(r.mu);
  if (i < 0 || i >= (int)r.order.size()) return LSP_ERR_ARG;
  const std::string& k = r.order[i];
  if (name && len > 0) {
    size_t n = std::min(len - 1, k.size());
    std::memcpy(name, k.data(), n);
    name[n] = 0;
  }
  if (total_ms) *total_ms = r.totals[k].first;
  if (launches) *launches = r.totals[k].second;
  return LSP_OK;
}

}  // extern "C"
