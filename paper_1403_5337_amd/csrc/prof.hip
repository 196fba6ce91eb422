// Optional per-kernel timing with HIP events recorded on the launch stream.
// Off by default; when on, every wrapped launch records an event pair, and
// hodlr_prof_query sums the elapsed times of one kernel name.
#include <mutex>
#include <string>
#include <vector>

#include "hodlr_internal.h"

namespace hodlr {

namespace {
struct Rec {
  const char* name;
  hipEvent_t a, b;
};
std::mutex g_mu;
bool g_on = false;
std::vector<Rec> g_recs;
std::vector<hipEvent_t> g_pool;

hipEvent_t get_event() {
  if (!g_pool.empty()) {
    hipEvent_t e = g_pool.back();
    g_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  // no system-scope release at the marker: the timed kernels write device
  // memory only, and the fence would add to every measured interval
  if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return nullptr;
  return e;
}

void release_all() {
  for (auto& r : g_recs) {
    if (r.a) g_pool.push_back(r.a);
    if (r.b) g_pool.push_back(r.b);
  }
  g_recs.clear();
}
}  // namespace

thread_local bool t_suspended = false;

bool prof_on() { return g_on && !t_suspended; }
void prof_suspend(bool on) { t_suspended = on; }

void prof_mark(const char* name, hipStream_t s, bool begin) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_on) return;
  hipEvent_t e = get_event();
  if (!e) return;
  (void)hipEventRecord(e, s);
  if (begin) {
    g_recs.push_back(Rec{name, e, nullptr});
  } else {
    for (auto it = g_recs.rbegin(); it != g_recs.rend(); ++it)
      if (it->b == nullptr && std::string(it->name) == name) {
        it->b = e;
        return;
      }
    g_pool.push_back(e);
  }
}

}  // namespace hodlr

extern "C" {

int hodlr_prof_enable(int on) {
  std::lock_guard<std::mutex> lk(hodlr::g_mu);
  hodlr::release_all();
  hodlr::g_on = on != 0;
  return HODLR_OK;
}

int hodlr_prof_query(const char* name, int* launches, double* total_ms) {
  if (!name || !launches || !total_ms) return hodlr::fail(HODLR_EINVAL, "NULL pointer");
  std::lock_guard<std::mutex> lk(hodlr::g_mu);
  int cnt = 0;
  double tot = 0.0;
  for (auto& r : hodlr::g_recs) {
    if (!r.b || std::string(r.name) != name) continue;
    HODLR_HIP(hipEventSynchronize(r.b));
    float ms = 0.f;
    HODLR_HIP(hipEventElapsedTime(&ms, r.a, r.b));
    tot += ms;
    ++cnt;
  }
  *launches = cnt;
  *total_ms = tot;
  return HODLR_OK;
}

}  // extern "C"
