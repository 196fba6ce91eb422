// Optional per-kernel timing with HIP events recorded on the launch stream.
// Off by default; when on, every wrapped launch records an event pair, and
// hodlr_prof_query sums the elapsed times of one kernel name.
#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "hodlr_internal.h"

namespace hodlr {

namespace {
struct Rec {
  const char* name;
  hipEvent_t a, b;
  std::thread::id tid;  // the recording thread
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
thread_local bool t_no_tune = false;  // tune_choice keeps to choices already made (no timing)

bool prof_on() { return g_on && !t_suspended; }
void prof_suspend(bool on) { t_suspended = on; }
void tune_freeze(bool on) { t_no_tune = on; }

size_t prof_count() {
  std::lock_guard<std::mutex> lk(g_mu);
  return g_recs.size();
}
void prof_drop_from(size_t first) {  // this thread's records only
  std::lock_guard<std::mutex> lk(g_mu);
  const std::thread::id me = std::this_thread::get_id();
  size_t keep = std::min(first, g_recs.size());
  for (size_t i = keep; i < g_recs.size(); ++i) {
    Rec& r = g_recs[i];
    if (r.tid == me) {
      if (r.a) g_pool.push_back(r.a);
      if (r.b) g_pool.push_back(r.b);
    } else {
      g_recs[keep++] = r;
    }
  }
  g_recs.resize(keep);
}
void prof_mark(const char* name, hipStream_t s, bool begin) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_on) return;
  hipEvent_t e = get_event();
  if (!e) return;
  (void)hipEventRecord(e, s);
  if (begin) {
    g_recs.push_back(Rec{name, e, nullptr, std::this_thread::get_id()});
  } else {
    for (auto it = g_recs.rbegin(); it != g_recs.rend(); ++it)
      if (it->b == nullptr && std::string(it->name) == name) {
        it->b = e;
        return;
      }
    g_pool.push_back(e);
  }
}

// ---------------------------------------------------------------------------
// Autotuning of launch variants (tune_choice): the first call for a key times
// every candidate on the caller's stream (one warm launch, then kTuneReps
// timed launches each, the profiler suspended), keeps the fastest for the
// process and launches it once more, so the call's outputs are the chosen
// variant's.  Later calls launch the kept choice; other threads asking while
// a key is being tuned wait for it.  Under stream capture, or with
// HODLR_TUNE=0 in the environment, the fallback runs untimed.  A choice
// changes only how work is split (e.g. the order of partial sums).
// ---------------------------------------------------------------------------
namespace {
constexpr int kTuneReps = 3;
std::mutex g_tune_mu;
std::map<std::string, int> g_tune;
}  // namespace

bool tune_known(const std::string& key) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  return g_tune.count(key) != 0;
}

int tune_choice(const std::string& key, int ncand, int fallback, const std::function<int(int)>& launch,
                hipStream_t s, int* pick) {
  // one thread tunes a key while the others wait for its choice
  std::unique_lock<std::mutex> lk(g_tune_mu);
  auto it = g_tune.find(key);
  if (it != g_tune.end()) {
    *pick = it->second;
    lk.unlock();
    return launch(*pick);
  }
  const char* env = std::getenv("HODLR_TUNE");
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  HODLR_HIP(hipStreamIsCapturing(s, &cs));
  if ((env && env[0] == '0') || cs != hipStreamCaptureStatusNone || ncand < 2 || t_no_tune) {
    lk.unlock();
    *pick = fallback;
    return launch(fallback);
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HODLR_HIP(hipEventCreate(&e0));
  HODLR_HIP(hipEventCreate(&e1));
  const bool was = t_suspended;
  t_suspended = true;
  int best = fallback, st = HODLR_OK;
  float best_ms = 0.f;
  for (int c = 0; c < ncand && st == HODLR_OK; ++c) {
    st = launch(c);
    if (st == HODLR_OK && hipEventRecord(e0, s) != hipSuccess) st = fail(HODLR_EHIP, "hipEventRecord");
    for (int r = 0; r < kTuneReps && st == HODLR_OK; ++r) st = launch(c);
    if (st != HODLR_OK) break;
    if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
      st = fail(HODLR_EHIP, "tuning events");
      break;
    }
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    if (c == 0 || ms < best_ms) {
      best_ms = ms;
      best = c;
    }
  }
  t_suspended = was;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != HODLR_OK) return st;
  g_tune[key] = best;
  lk.unlock();
  *pick = best;
  return launch(best);
}

std::string tune_report() {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  std::string out;
  for (auto& kv : g_tune) out += kv.first + "=" + std::to_string(kv.second) + "\n";
  return out;
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

extern "C" int hodlr_tune_report(char* buf, int len) {
  if (!buf || len < 1) return hodlr::fail(HODLR_EINVAL, "buf is NULL or len < 1");
  const std::string r = hodlr::tune_report();
  const size_t k = std::min((size_t)len - 1, r.size());
  std::memcpy(buf, r.data(), k);
  buf[k] = 0;
  return r.size() < (size_t)len ? HODLR_OK : hodlr::fail(HODLR_EINVAL, "buffer too short for the report");
}
