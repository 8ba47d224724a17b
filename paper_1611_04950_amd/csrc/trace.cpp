// Kernel tracing (see trace.h) and its C entry points.
#include "trace.h"

#include <atomic>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "slepian.h"

namespace slp {
namespace {

struct Rec {
  const char *name;
  hipEvent_t a, b;
};

std::atomic<bool> g_on{false};
std::mutex g_mu;
std::vector<Rec> g_open;      // records with both events enqueued
std::vector<hipEvent_t> g_pool;
Rec g_cur{nullptr, nullptr, nullptr};

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

bool trace_enabled() { return g_on.load(std::memory_order_relaxed); }

void trace_mark_begin(const char *name, hipStream_t st) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_cur.name = name;
  g_cur.a = take_event();
  g_cur.b = take_event();
  if (g_cur.a) (void)hipEventRecord(g_cur.a, st);
}

void trace_mark_end(hipStream_t st) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_cur.a || !g_cur.b) return;
  (void)hipEventRecord(g_cur.b, st);
  g_open.push_back(g_cur);
  g_cur = Rec{nullptr, nullptr, nullptr};
}

}  // namespace slp

extern "C" {

int slepian_trace_enable(int on) {
  slp::g_on.store(on != 0, std::memory_order_relaxed);
  return SLEPIAN_OK;
}

int slepian_trace_read(slepian_kernel_stat *stats, int cap, int *count, int reset) {
  if (!count || cap < 0 || (cap > 0 && !stats)) return SLEPIAN_EINVAL;
  std::lock_guard<std::mutex> lk(slp::g_mu);
  struct Acc {
    int64_t n = 0;
    double tot = 0, mn = 1e300, mx = 0;
  };
  std::map<std::string, Acc> acc;
  for (const slp::Rec &r : slp::g_open) {
    if (hipEventSynchronize(r.b) != hipSuccess) return SLEPIAN_EHIP;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) return SLEPIAN_EHIP;
    Acc &a = acc[r.name];
    a.n += 1;
    a.tot += ms;
    a.mn = ms < a.mn ? ms : a.mn;
    a.mx = ms > a.mx ? ms : a.mx;
  }
  int i = 0;
  for (const auto &kv : acc) {
    if (i < cap) {
      slepian_kernel_stat &s = stats[i];
      std::memset(&s, 0, sizeof(s));
      std::strncpy(s.name, kv.first.c_str(), sizeof(s.name) - 1);
      s.launches = kv.second.n;
      s.total_ms = kv.second.tot;
      s.min_ms = kv.second.mn;
      s.max_ms = kv.second.mx;
    }
    ++i;
  }
  *count = i;
  if (reset) {
    for (const slp::Rec &r : slp::g_open) {
      slp::g_pool.push_back(r.a);
      slp::g_pool.push_back(r.b);
    }
    slp::g_open.clear();
  }
  return SLEPIAN_OK;
}

}  // extern "C"
