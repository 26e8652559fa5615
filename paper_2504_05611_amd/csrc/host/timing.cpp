// Kernel timing registry (tracing aid behind tmcs_timing_*).
#include "timing.h"

#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "internal.h"

namespace tmcs {

namespace {
struct Rec {
  std::string name;
  hipEvent_t a, b;
};
std::mutex g_mu;
bool g_on = false;
std::vector<Rec*> g_recs;
}  // namespace

bool timing_on() { return g_on; }

void timing_begin(const char* name, hipStream_t s, void** token) {
  Rec* r = new Rec{name, nullptr, nullptr};
  // timing only: no system-scope fence (cache writeback and invalidation) per record
  if (hipEventCreateWithFlags(&r->a, hipEventDisableSystemFence) != hipSuccess ||
      hipEventCreateWithFlags(&r->b, hipEventDisableSystemFence) != hipSuccess) {
    delete r;
    *token = nullptr;
    return;
  }
  (void)hipEventRecord(r->a, s);
  *token = r;
}

void timing_end(void* token, hipStream_t s) {
  Rec* r = (Rec*)token;
  (void)hipEventRecord(r->b, s);
  std::lock_guard<std::mutex> g(g_mu);
  g_recs.push_back(r);
}

static void clear_locked() {
  for (Rec* r : g_recs) {
    (void)hipEventDestroy(r->a);
    (void)hipEventDestroy(r->b);
    delete r;
  }
  g_recs.clear();
}

}  // namespace tmcs

using namespace tmcs;

extern "C" {

tmcs_status tmcs_timing_enable(int on) {
  std::lock_guard<std::mutex> g(g_mu);
  g_on = on != 0;
  return TMCS_OK;
}

tmcs_status tmcs_timing_reset(void) {
  std::lock_guard<std::mutex> g(g_mu);
  clear_locked();
  return TMCS_OK;
}

tmcs_status tmcs_timing_report(char* buf, size_t cap, size_t* len) {
  std::lock_guard<std::mutex> g(g_mu);
  std::map<std::string, std::pair<long, double>> agg;
  for (Rec* r : g_recs) {
    if (hipEventSynchronize(r->b) != hipSuccess) return fail(TMCS_EDEVICE, "timing event");
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, r->a, r->b);
    auto& e = agg[r->name];
    e.first += 1;
    e.second += ms;
  }
  std::string s = "{";
  bool first = true;
  for (auto& kv : agg) {
    if (!first) s += ", ";
    first = false;
    char tmp[128];
    snprintf(tmp, sizeof tmp, "\"%s\": [%ld, %.6f]", kv.first.c_str(), kv.second.first, kv.second.second);
    s += tmp;
  }
  s += "}";
  if (len) *len = s.size();
  if (buf && cap) {
    const size_t n = s.size() < cap - 1 ? s.size() : cap - 1;
    std::memcpy(buf, s.data(), n);
    buf[n] = 0;
  }
  return TMCS_OK;
}

}  // extern "C"
