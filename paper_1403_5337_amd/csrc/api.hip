// C ABI entry points: argument validation, handle lifetime, tree set-up.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <cstdint>
#include <map>
#include <memory>
#include <condition_variable>
#include <cstdlib>
#include <functional>
#include <mutex>
#include <thread>
#include <string>

#include "gemm.h"
#include "hodlr_internal.h"

namespace hodlr {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

int fail(int code, const std::string& msg) {
  set_error(msg);
  return code;
}

// ---------------------------------------------------------------------------
// Caching device allocator.  Freed blocks go to a per-device free list and
// are handed out again for requests between half their size and their size,
// so repeated builds and solves do not call hipMalloc / hipFree (which also
// synchronizes the device).  Blocks are returned only by
// hodlr_release_memory().  A block is reused by later work on any stream, so
// a temporary is released either after the work that used it has been
// synchronized, or behind an event on the stream of that work
// (dev_free_after): such a block joins the free list only once its event has
// completed, which allocations check without waiting.
// ---------------------------------------------------------------------------
namespace {
std::mutex g_alloc_mu;
std::multimap<size_t, void*> g_free[64];
struct PendingBlock {
  size_t bytes;
  void* p;
  hipEvent_t ev;
  int dev;
};
std::vector<PendingBlock> g_pending;  // released behind an event, not yet reusable
std::vector<hipEvent_t> g_event_pool;
int cur_device() {
  int d = 0;
  (void)hipGetDevice(&d);
  return d < 0 ? 0 : (d > 63 ? 63 : d);
}
// moves the pending blocks whose event has completed (all of them with
// wait) to the free lists; g_alloc_mu held
void collect_pending(bool wait) {
  size_t keep = 0;
  for (size_t i = 0; i < g_pending.size(); ++i) {
    PendingBlock& b = g_pending[i];
    const bool done = wait ? hipEventSynchronize(b.ev) == hipSuccess : hipEventQuery(b.ev) == hipSuccess;
    if (done || wait) {
      g_free[b.dev].emplace(b.bytes, b.p);
      g_event_pool.push_back(b.ev);
    } else {
      g_pending[keep++] = b;
    }
  }
  g_pending.resize(keep);
  (void)hipGetLastError();  // a not-ready query leaves no error behind
}
}  // namespace

int dev_alloc(size_t nbytes, void** out) {
  nbytes = (nbytes + 255) / 256 * 256;
  {
    std::lock_guard<std::mutex> lk(g_alloc_mu);
    if (!g_pending.empty()) collect_pending(false);
    auto& fl = g_free[cur_device()];
    auto it = fl.lower_bound(nbytes);
    if (it != fl.end() && it->first <= 2 * nbytes) {
      *out = it->second;
      fl.erase(it);
      return HODLR_OK;
    }
  }
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, nbytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    // give the cache back to the runtime once and retry
    release_cached_memory();
    e = hipMalloc(&p, nbytes);
    if (e != hipSuccess)
      return fail(HODLR_ENOMEM, std::string("hipMalloc(") + std::to_string(nbytes) +
                                    "): " + hipGetErrorString(e));
  }
  *out = p;
  return HODLR_OK;
}

namespace {
std::mutex g_pin_mu;
std::multimap<size_t, void*> g_pin_free;  // size -> block
}  // namespace

int pinned_alloc(size_t nbytes, void** out, size_t* got) {
  nbytes = std::max<size_t>(4096, (nbytes + 4095) / 4096 * 4096);
  {
    std::lock_guard<std::mutex> lk(g_pin_mu);
    auto it = g_pin_free.lower_bound(nbytes);
    if (it != g_pin_free.end() && it->first <= 4 * nbytes) {
      *out = it->second;
      *got = it->first;
      g_pin_free.erase(it);
      return HODLR_OK;
    }
  }
  void* p = nullptr;
  HODLR_HIP(hipHostMalloc(&p, nbytes));
  *out = p;
  *got = nbytes;
  return HODLR_OK;
}

void pinned_free(void* p, size_t nbytes) {
  if (!p) return;
  std::lock_guard<std::mutex> lk(g_pin_mu);
  g_pin_free.emplace(nbytes, p);
}

void dev_free(void* p, size_t nbytes) {
  if (!p) return;
  nbytes = (nbytes + 255) / 256 * 256;
  std::lock_guard<std::mutex> lk(g_alloc_mu);
  g_free[cur_device()].emplace(nbytes, p);
}

void dev_free_after(void* p, size_t nbytes, hipStream_t s) {
  if (!p) return;
  nbytes = (nbytes + 255) / 256 * 256;
  hipEvent_t ev = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_alloc_mu);
    if (!g_event_pool.empty()) {
      ev = g_event_pool.back();
      g_event_pool.pop_back();
    }
  }
  if (!ev && hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) ev = nullptr;
  if (!ev || hipEventRecord(ev, s) != hipSuccess) {
    // no event: fall back to waiting for the stream
    (void)hipGetLastError();
    (void)hipStreamSynchronize(s);
    dev_free(p, nbytes);
    if (ev) {
      std::lock_guard<std::mutex> lk(g_alloc_mu);
      g_event_pool.push_back(ev);
    }
    return;
  }
  std::lock_guard<std::mutex> lk(g_alloc_mu);
  g_pending.push_back({nbytes, p, ev, cur_device()});
}

int event_take(hipEvent_t* out) {
  {
    std::lock_guard<std::mutex> lk(g_alloc_mu);
    if (!g_event_pool.empty()) {
      *out = g_event_pool.back();
      g_event_pool.pop_back();
      return HODLR_OK;
    }
  }
  HODLR_HIP(hipEventCreateWithFlags(out, hipEventDisableTiming));
  return HODLR_OK;
}

void event_give(hipEvent_t e) {
  if (!e) return;
  std::lock_guard<std::mutex> lk(g_alloc_mu);
  g_event_pool.push_back(e);
}

void release_cached_memory() {
  std::lock_guard<std::mutex> lk(g_alloc_mu);
  int dev = cur_device();
  (void)hipDeviceSynchronize();
  collect_pending(true);
  for (auto& kv : g_free[dev]) (void)hipFree(kv.second);
  g_free[dev].clear();
}

void DevBuf::release() {
  if (p) dev_free(p, bytes);
  p = nullptr;
  bytes = 0;
}

void DevBuf::release_after(hipStream_t s) {
  if (p) dev_free_after(p, bytes, s);
  p = nullptr;
  bytes = 0;
}

int DevBuf::ensure(size_t nbytes) {
  if (nbytes <= bytes && p) return HODLR_OK;
  release();
  if (nbytes == 0) nbytes = 256;
  void* q = nullptr;
  HODLR_TRY(dev_alloc(nbytes, &q));
  p = q;
  bytes = (nbytes + 255) / 256 * 256;
  return HODLR_OK;
}

void Tree::build(int n_, int leaf_) {
  n = n_;
  leaf = leaf_;
  L = 0;
  while ((n + (1 << L) - 1) / (1 << L) > leaf) ++L;
  lo.assign((2 << L) - 1, 0);
  hi.assign((2 << L) - 1, 0);
  lo[0] = 0;
  hi[0] = n;
  for (int p = 0; p < L; ++p) {
    for (int i = 0; i < (1 << p); ++i) {
      int id = node_id(p, i);
      int mid = lo[id] + (hi[id] - lo[id]) / 2;
      int a = node_id(p + 1, 2 * i), b = node_id(p + 1, 2 * i + 1);
      lo[a] = lo[id];
      hi[a] = mid;
      lo[b] = mid;
      hi[b] = hi[id];
    }
  }
}

int Tree::min_size(int p) const {
  int m = n;
  for (int i = 0; i < (1 << p); ++i) m = std::min(m, size(node_id(p, i)));
  return m;
}

int Tree::max_size(int p) const {
  int m = 0;
  for (int i = 0; i < (1 << p); ++i) m = std::max(m, size(node_id(p, i)));
  return m;
}

// Common set-up of a new handle once the tree is known.
// The status words are cleared on the build's stream: the handle's blocks
// come from the caching allocator (recycled memory), and a clear on the null
// stream is not ordered before work on a non-blocking stream (the worker
// streams of the batched calls).
static int init_handle(hodlr_s* h, int n, int leaf, int precision, hipStream_t stream) {
  h->tree.build(n, leaf);
  h->precision = precision;
  h->esize = precision == 64 ? 8 : 4;
  HODLR_HIP(hipGetDevice(&h->device));
  const Tree& t = h->tree;
  h->nleaf = 1 << t.L;
  h->bmax = t.max_size(t.L);
  int nn = t.nnodes();
  h->rank.assign(nn, 0);
  HODLR_TRY(h->d_lo.ensure(nn * sizeof(int)));
  HODLR_TRY(h->d_hi.ensure(nn * sizeof(int)));
  HODLR_TRY(h->d_rank.ensure(nn * sizeof(int)));
  // the node ranges from the process-wide copy of this tree's ranges on the
  // device, by copies ordered on the stream (no host round trip)
  const int *dlo = nullptr, *dhi = nullptr;
  HODLR_TRY(device_tree_ranges(t, &dlo, &dhi));
  HODLR_HIP(hipMemcpyAsync(h->d_lo.p, dlo, nn * sizeof(int), hipMemcpyDeviceToDevice, stream));
  HODLR_HIP(hipMemcpyAsync(h->d_hi.p, dhi, nn * sizeof(int), hipMemcpyDeviceToDevice, stream));
  HODLR_TRY(h->status.ensure(4 * sizeof(int)));
  HODLR_HIP(hipMemsetAsync(h->status.p, 0, 4 * sizeof(int), stream));
  HODLR_TRY(h->Kinv.ensure((size_t)h->nleaf * h->bmax * h->bmax * h->esize));
  return HODLR_OK;
}

// The solve's correction operators: level q's block is 2 r_q wide.
int alloc_E(hodlr_s* h) {
  const Tree& t = h->tree;
  h->offE.assign(t.L, 0);
  int RE = 0;
  for (int q = 1; q <= t.L; ++q) {
    h->offE[q - 1] = RE;
    RE += 2 * h->rcols[q - 1];
  }
  return h->E.ensure((size_t)t.n * std::max(RE, 1) * h->esize);
}

// Column layout from the per-node ranks: level q's block is as wide as the
// largest rank at that level.
int set_layout_from_ranks(hodlr_s* h) {
  const Tree& t = h->tree;
  h->rcols.assign(t.L, 0);
  h->off.assign(t.L, 0);
  int R = 0;
  for (int q = 1; q <= t.L; ++q) {
    int rq = 0;
    for (int i = 0; i < (1 << q); ++i) rq = std::max(rq, h->rank[node_id(q, i)]);
    h->rcols[q - 1] = rq;
    h->off[q - 1] = R;
    R += rq;
  }
  h->R = R;
  HODLR_TRY(h->Y.ensure((size_t)t.n * std::max(R, 1) * h->esize));
  HODLR_TRY(h->W.ensure((size_t)t.n * std::max(R, 1) * h->esize));
  HODLR_TRY(alloc_E(h));
  // inverse capacitance matrices, per parent level p: 2^p nodes of (2 r_{p+1})^2
  h->sinv_off.assign(t.L, 0);
  size_t tot = 0;
  for (int p = 0; p < t.L; ++p) {
    h->sinv_off[p] = tot;
    size_t rq = h->rcols[p];
    tot += (size_t)(1 << p) * (2 * rq) * (2 * rq);
  }
  HODLR_TRY(h->Sinv.ensure(std::max<size_t>(tot, 1) * h->esize));
  return ensure_work(h, 8);
}

int side_stream(int which, hipStream_t* out) {
  // per host thread, so concurrent builds do not queue behind each other
  static thread_local hipStream_t streams[2] = {nullptr, nullptr};
  if (which < 0 || which > 1) return fail(HODLR_EINVAL, "side stream index");
  if (!streams[which]) HODLR_HIP(hipStreamCreateWithFlags(&streams[which], hipStreamNonBlocking));
  *out = streams[which];
  return HODLR_OK;
}

// ---------------------------------------------------------------------------
// Worker pool of the batched calls: threads started on first use and kept for
// the process, each with its own stream; a call hands out its items through
// a shared counter and waits for all of them.
// ---------------------------------------------------------------------------
class Workers {
 public:
  static Workers& get() {
    static Workers* w = new Workers();  // kept for the process
    return *w;
  }
  // fn(item, stream) for every item in [0, nitems); returns the code of the
  // lowest failing item and its message in *msg
  int run(int nitems, const std::function<int(int, hipStream_t)>& fn, hipStream_t caller, std::string* msg) {
    std::lock_guard<std::mutex> serial(call_mu_);  // one batched call at a time
    int dev = 0;
    HODLR_HIP(hipGetDevice(&dev));
    hipEvent_t start = nullptr;
    HODLR_HIP(hipEventCreateWithFlags(&start, hipEventDisableTiming));
    const hipError_t er = hipEventRecord(start, caller);
    if (er != hipSuccess) {
      (void)hipEventDestroy(start);
      return fail(HODLR_EHIP, std::string("hipEventRecord: ") + hipGetErrorString(er));
    }
    std::vector<int> codes(nitems, HODLR_OK);
    std::vector<std::string> msgs(nitems);
    {
      std::unique_lock<std::mutex> lk(mu_);
      job_ = [&, dev, start](int i) {
        hipStream_t s = nullptr;
        int st = worker_stream(dev, &s);
        if (st == HODLR_OK) {
          const hipError_t e = hipStreamWaitEvent(s, start, 0);
          st = e == hipSuccess ? fn(i, s) : fail(HODLR_EHIP, std::string("hipStreamWaitEvent: ") +
                                                                 hipGetErrorString(e));
          if (s) {
            const hipError_t e2 = hipStreamSynchronize(s);
            if (st == HODLR_OK && e2 != hipSuccess)
              st = fail(HODLR_EHIP, std::string("hipStreamSynchronize: ") + hipGetErrorString(e2));
          }
        }
        codes[i] = st;
        if (st != HODLR_OK) msgs[i] = hodlr_last_error();
      };
      next_ = 0;
      count_ = nitems;
      remaining_ = nitems;
      ++generation_;
      start_threads();
    }
    cv_.notify_all();
    {
      std::unique_lock<std::mutex> lk(mu_);
      done_cv_.wait(lk, [&] { return remaining_ == 0; });
      job_ = nullptr;
    }
    (void)hipEventDestroy(start);
    for (int i = 0; i < nitems; ++i)
      if (codes[i] != HODLR_OK) {
        *msg = msgs[i];
        return codes[i];
      }
    return HODLR_OK;
  }

 private:
  static int worker_stream(int dev, hipStream_t* out) {
    static thread_local hipStream_t s = nullptr;
    static thread_local int sdev = -1;
    HODLR_HIP(hipSetDevice(dev));
    if (!s || sdev != dev) {
      HODLR_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
      sdev = dev;
    }
    *out = s;
    return HODLR_OK;
  }
  void start_threads() {  // under mu_
    if (!threads_.empty()) return;
    int nt = 8;
    if (const char* e = std::getenv("HODLR_THREADS")) nt = std::max(1, std::min(64, std::atoi(e)));
    for (int k = 0; k < nt; ++k) threads_.emplace_back([this] { loop(); });
  }
  void loop() {
    unsigned long long seen = 0;
    for (;;) {
      std::function<void(int)> job;
      int i = -1;
      {
        std::unique_lock<std::mutex> lk(mu_);
        cv_.wait(lk, [&] { return generation_ != seen && next_ < count_; });
        i = next_++;
        if (next_ >= count_) seen = generation_;
        job = job_;
      }
      job(i);
      {
        std::lock_guard<std::mutex> lk(mu_);
        if (--remaining_ == 0) done_cv_.notify_all();
      }
    }
  }
  std::mutex call_mu_, mu_;
  std::condition_variable cv_, done_cv_;
  std::vector<std::thread> threads_;
  std::function<void(int)> job_;
  int next_ = 0, count_ = 0, remaining_ = 0;
  unsigned long long generation_ = 0;
};

// ESINGULAR for the status words of a factorization (0: flag, 1: node).
int singular_status(const int* st) {
  return fail(HODLR_ESINGULAR, st[0] == 1 ? "singular leaf block " + std::to_string(st[1])
                                          : "singular capacitance matrix at node " + std::to_string(st[1]));
}

int mark_inflight(hodlr_s* h, hipStream_t s) {
  size_t keep = 0;
  for (hipEvent_t e : h->inflight) {
    if (hipEventQuery(e) == hipSuccess)
      event_give(e);
    else
      h->inflight[keep++] = e;
  }
  h->inflight.resize(keep);
  (void)hipGetLastError();  // a not-ready query leaves no error behind
  if (h->inflight.size() >= 16) {
    HODLR_HIP(hipEventSynchronize(h->inflight.front()));
    event_give(h->inflight.front());
    h->inflight.erase(h->inflight.begin());
  }
  hipEvent_t e = nullptr;
  HODLR_TRY(event_take(&e));
  h->inflight.push_back(e);
  HODLR_HIP(hipEventRecord(e, s));
  return HODLR_OK;
}

int settle_factor_status(hodlr_s* h) {
  if (!h->status_pending) return HODLR_OK;
  HODLR_HIP(hipEventSynchronize(h->status_ev));
  h->status_pending = false;
  if (h->pin_status[0]) {
    h->factored = false;
    return singular_status(h->pin_status);
  }
  return HODLR_OK;
}

}  // namespace hodlr

using namespace hodlr;

extern "C" {

void hodlr_default_opts(hodlr_opts* o) {
  if (!o) return;
  o->leaf = 128;
  o->tol = 1e-4;
  o->method = HODLR_ACA;
  o->bdlr_depth = 1;
  o->max_rank = 0;
  o->precision = 32;
  o->skel_k = 0;
  o->mlp_params = nullptr;
  o->seed = 0;
  o->skel_tol = 0.0;
  o->bdlr_max_skel = 0;
  o->symmetric = 0;
  o->bdlr_max_depth = 0;
}

const char* hodlr_last_error(void) { return g_last_error.c_str(); }

static int check_opts(const hodlr_opts& o) {
  if (o.leaf < 1 || o.leaf > kLeafMax)
    return fail(HODLR_EINVAL, "opts.leaf must be in [1, " + std::to_string(kLeafMax) + "]");
  if (!(o.tol >= 0.0) || !std::isfinite(o.tol)) return fail(HODLR_EINVAL, "opts.tol must be >= 0");
  if (o.method != HODLR_ACA && o.method != HODLR_BDLR && o.method != HODLR_LEARNED)
    return fail(HODLR_EINVAL, "opts.method must be HODLR_ACA, HODLR_BDLR or HODLR_LEARNED");
  if (o.method == HODLR_LEARNED && (!o.mlp_params || o.skel_k < 0))
    return fail(HODLR_EINVAL, "HODLR_LEARNED needs opts.mlp_params and opts.skel_k >= 0");
  if (o.method == HODLR_LEARNED && o.skel_k == 0 && (o.bdlr_depth < 1 || o.bdlr_depth > 250))
    return fail(HODLR_EINVAL, "HODLR_LEARNED with skel_k 0 sizes by opts.bdlr_depth, which must be in [1, 250]");
  if (!(o.skel_tol >= 0.0) || !std::isfinite(o.skel_tol)) return fail(HODLR_EINVAL, "opts.skel_tol must be >= 0");
  if (o.bdlr_max_skel < 0) return fail(HODLR_EINVAL, "opts.bdlr_max_skel must be >= 0");
  if (o.symmetric != 0 && o.symmetric != 1) return fail(HODLR_EINVAL, "opts.symmetric must be 0 or 1");
  if (o.bdlr_max_depth != 0 && (o.bdlr_max_depth < o.bdlr_depth || o.bdlr_max_depth > 250))
    return fail(HODLR_EINVAL, "opts.bdlr_max_depth must be 0 or in [bdlr_depth, 250]");
  if (o.precision != 32 && o.precision != 64)
    return fail(HODLR_EINVAL, "opts.precision must be 32 or 64");
  if (o.leaf > leaf_cap(o.precision))
    return fail(HODLR_EINVAL, "opts.leaf must be <= " + std::to_string(leaf_cap(o.precision)) +
                                  " at this precision");
  if (o.max_rank < 0) return fail(HODLR_EINVAL, "opts.max_rank must be >= 0");
  if (o.method == HODLR_BDLR && (o.bdlr_depth < 1 || o.bdlr_depth > 250))
    return fail(HODLR_EINVAL, "opts.bdlr_depth must be in [1, 250]");
  return HODLR_OK;
}

// dst[0, na) = a, dst[na, na + 4) = b, dst[na + 4, na + 8) = c (zeros if c
// is NULL); dst is pinned host memory, made visible to the host before the
// kernel ends.
__global__ void k_export_ints(const int* __restrict__ a, int na, const int* __restrict__ b,
                              const int* __restrict__ c, int* dst) {
  for (int i = threadIdx.x; i < na + 8; i += blockDim.x) {
    int v = 0;
    if (i < na) v = a[i];
    else if (i < na + 4) v = b[i - na];
    else if (c) v = c[i - na - 4];
    dst[i] = v;
  }
  __threadfence_system();
}

static int build_impl(const double* K, int n, int ldk, const int* g_rowptr, const int* g_col,
                      const float* coords, const hodlr_opts* opts, hipStream_t stream, hodlr_t* out,
                      int* piv_export) {
  if (!out) return fail(HODLR_EINVAL, "out is NULL");
  *out = nullptr;
  hodlr_opts o;
  hodlr_default_opts(&o);
  if (opts) o = *opts;
  if (!K) return fail(HODLR_EINVAL, "K is NULL");
  if (n < 1 || n > kMaxN) return fail(HODLR_EINVAL, "n out of range");
  if (ldk < n) return fail(HODLR_EINVAL, "ldk < n");
  HODLR_TRY(check_opts(o));
  if (o.method != HODLR_ACA && (!g_rowptr || !g_col))
    return fail(HODLR_EINVAL, "BDLR and learned skeletons need the separator graph (g_rowptr, g_col)");
  if (o.method == HODLR_LEARNED && !coords) return fail(HODLR_EINVAL, "learned skeletons need coords");
  if (n > 16384) return fail(HODLR_EINVAL, "hodlr_build supports n <= 16384 (block sides <= 8192)");
  std::unique_ptr<hodlr_s> h(new hodlr_s());
  h->method = o.method;
  h->depth = o.bdlr_depth;
  h->max_rank = o.max_rank;
  h->tol = o.tol;
  HODLR_TRY(init_handle(h.get(), n, o.leaf, o.precision, stream));
  const Tree& t = h->tree;
  // a1: leaf blocks to the factorization precision
  HODLR_TRY(launch_stage_leaves_from_K(h.get(), K, ldk, stream));
  // The leaf inverses need only the staged diagonal blocks: they run on a
  // second stream beside the compression (not beside ACA, whose cooperative
  // launch wants every compute unit).  The guard joins that stream before any
  // return, so no kernel outlives the handle's buffers.
  struct Fork {
    hipStream_t side = nullptr;
    hipEvent_t ev[2] = {nullptr, nullptr};
    ~Fork() {
      if (side) (void)hipStreamSynchronize(side);
      for (auto e : ev) event_give(e);
    }
  } fork;
  if (o.method != HODLR_ACA) {
    HODLR_TRY(side_stream(0, &fork.side));
    for (auto& e : fork.ev) HODLR_TRY(event_take(&e));
    HODLR_HIP(hipEventRecord(fork.ev[0], stream));
    HODLR_HIP(hipStreamWaitEvent(fork.side, fork.ev[0], 0));
    HODLR_TRY(h->lstatus.ensure(4 * sizeof(int)));
    HODLR_TRY(launch_leaf_inverse(h.get(), h->lstatus.as<int>(), fork.side));
    HODLR_HIP(hipEventRecord(fork.ev[1], fork.side));
  }
  if (t.L > 0) {
    int cap = rank_cap(o.precision);
    if (o.max_rank > 0) cap = std::min(cap, o.max_rank);
    std::vector<int> capq(t.L), capoff(t.L);
    int C = 0;
    for (int q = 1; q <= t.L; ++q) {
      capq[q - 1] = std::min(cap, t.max_size(q));
      capoff[q - 1] = C;
      C += capq[q - 1];
    }
    DevBuf Ucap, Vcap;
    HODLR_TRY(Ucap.ensure((size_t)n * C * h->esize));
    HODLR_TRY(Vcap.ensure((size_t)n * C * h->esize));
    HODLR_HIP(hipMemsetAsync(Ucap.p, 0, (size_t)n * C * h->esize, stream));
    HODLR_HIP(hipMemsetAsync(Vcap.p, 0, (size_t)n * C * h->esize, stream));
    // compression of every off-diagonal block
    if (o.method == HODLR_BDLR && o.bdlr_max_depth > 0)
      HODLR_TRY(launch_bdlr_adaptive(h.get(), K, ldk, g_rowptr, g_col, o.bdlr_max_depth, o.bdlr_max_skel, o.seed,
                                     o.skel_tol > 0.0 ? o.skel_tol : 30.0 * o.tol, Ucap.p, Vcap.p, capoff, capq,
                                     stream));
    else if (o.method == HODLR_BDLR)
      HODLR_TRY(launch_bdlr(h.get(), K, ldk, g_rowptr, g_col, Ucap.p, Vcap.p, capoff, capq, stream,
                            o.bdlr_max_skel, piv_export));
    else if (o.method == HODLR_LEARNED)
      HODLR_TRY(launch_learned(h.get(), K, ldk, g_rowptr, g_col, coords, o.mlp_params, o.skel_k, o.seed,
                               o.skel_tol > 0.0 ? o.skel_tol : 30.0 * o.tol, Ucap.p, Vcap.p, capoff, capq,
                               stream));
    else if (o.symmetric) {
      // only the left children's blocks; their siblings' are their transposes
      std::vector<int> left;
      for (int q = 1; q <= t.L; ++q)
        for (int i = 0; i < (1 << q); i += 2) left.push_back(node_id(q, i));
      HODLR_TRY(launch_aca(h.get(), K, ldk, Ucap.p, Vcap.p, capoff, capq, stream, &left, piv_export));
    } else {
      HODLR_TRY(launch_aca(h.get(), K, ldk, Ucap.p, Vcap.p, capoff, capq, stream, nullptr, piv_export));
    }
    // the ranks, the compression's status words and those of the leaf
    // inverses come back together, written into pinned host memory by one
    // kernel, behind the build's one synchronization
    if (fork.side) HODLR_HIP(hipStreamWaitEvent(stream, fork.ev[1], 0));
    const int nn = t.nnodes();
    void* pin = nullptr;
    size_t pin_bytes = 0;
    HODLR_TRY(pinned_alloc((size_t)(nn + 8) * sizeof(int), &pin, &pin_bytes));
    struct PinGuard {
      void* p;
      size_t b;
      ~PinGuard() { pinned_free(p, b); }
    } pin_guard{pin, pin_bytes};
    int* dpin = nullptr;
    HODLR_HIP(hipHostGetDevicePointer(reinterpret_cast<void**>(&dpin), pin, 0));
    k_export_ints<<<1, kBlock, 0, stream>>>(h->d_rank.as<int>(), nn, h->status.as<int>(),
                                            fork.side ? h->lstatus.as<int>() : nullptr, dpin);
    HODLR_HIP(hipGetLastError());
    HODLR_HIP(hipStreamSynchronize(stream));
    const int* hp = static_cast<const int*>(pin);
    std::copy(hp, hp + nn, h->rank.begin());
    if (hp[nn + 2]) return fail(HODLR_EHIP, "ACA workgroup barrier timed out");
    if (fork.side) {
      h->leaves_inverted = true;
      if (hp[nn + 4]) h->leaf_singular = hp[nn + 5];
    }
    h->rank[0] = 0;
    if (o.symmetric)  // a right child (even id >= 2) takes its left sibling's rank
      for (int id = 2; id < nn; id += 2) h->rank[id] = h->rank[id - 1];
    HODLR_TRY(set_layout_from_ranks(h.get()));
    HODLR_TRY(launch_repack(h.get(), Ucap.p, Vcap.p, n, capoff, stream));
    if (o.symmetric) HODLR_TRY(launch_mirror(h.get(), stream));
    // the capped panels go back to the allocator once the repack has run
    Ucap.release_after(stream);
    Vcap.release_after(stream);
    HODLR_TRY(mark_inflight(h.get(), stream));
    *out = h.release();
    return HODLR_OK;
  }
  HODLR_TRY(set_layout_from_ranks(h.get()));
  if (fork.side) {
    HODLR_HIP(hipStreamWaitEvent(stream, fork.ev[1], 0));
    HODLR_HIP(hipStreamSynchronize(stream));
    int ls[4];
    HODLR_HIP(hipMemcpy(ls, h->lstatus.p, sizeof(ls), hipMemcpyDeviceToHost));
    h->leaves_inverted = true;
    if (ls[0]) h->leaf_singular = ls[1];
  }
  HODLR_TRY(mark_inflight(h.get(), stream));
  *out = h.release();
  return HODLR_OK;
}

int hodlr_build(const double* K, int n, int ldk, const int* g_rowptr, const int* g_col, const float* coords,
                const hodlr_opts* opts, hipStream_t stream, hodlr_t* out) {
  return build_impl(K, n, ldk, g_rowptr, g_col, coords, opts, stream, out, nullptr);
}

int hodlr_build_from_factors(int n, int leaf, int precision, const double* leaves,
                             const double* Upanel, const double* Vpanel, const int* ranks,
                             const int* rcols, int nlevels, hipStream_t stream, hodlr_t* out) {
  if (!out) return fail(HODLR_EINVAL, "out is NULL");
  *out = nullptr;
  if (n < 1 || n > kMaxN) return fail(HODLR_EINVAL, "n out of range");
  if (leaf < 1 || leaf > kLeafMax) return fail(HODLR_EINVAL, "leaf out of range");
  if (precision != 32 && precision != 64) return fail(HODLR_EINVAL, "precision must be 32 or 64");
  if (leaf > leaf_cap(precision)) return fail(HODLR_EINVAL, "leaf too large for this precision");
  if (!leaves) return fail(HODLR_EINVAL, "leaves is NULL");
  {
    Tree t0;
    t0.build(n, leaf);
    if (nlevels != t0.L)
      return fail(HODLR_EINVAL, "nlevels = " + std::to_string(nlevels) + " but the tree has " +
                                    std::to_string(t0.L) + " levels");
    if (t0.L > 0 && (!Upanel || !Vpanel || !ranks || !rcols))
      return fail(HODLR_EINVAL, "panels, ranks and rcols are required when L > 0");
  }
  std::unique_ptr<hodlr_s> h(new hodlr_s());
  HODLR_TRY(init_handle(h.get(), n, leaf, precision, stream));
  const Tree& t = h->tree;
  int cap = rank_cap(precision);
  for (int q = 1; q <= t.L; ++q) {
    if (rcols[q - 1] < 0 || rcols[q - 1] > cap || rcols[q - 1] > t.max_size(q))
      return fail(HODLR_EINVAL, "rcols out of range at level " + std::to_string(q));
    for (int i = 0; i < (1 << q); ++i) {
      int r = ranks[node_id(q, i) - 1];
      if (r < 0 || r > rcols[q - 1] || r > std::min(t.size(node_id(q, i)), t.size(node_id(q, i ^ 1))))
        return fail(HODLR_EINVAL, "rank out of range at node " + std::to_string(node_id(q, i)));
      h->rank[node_id(q, i)] = r;
    }
  }
  // layout = the caller's column widths (they bound the ranks)
  h->rcols.assign(rcols, rcols + t.L);
  h->off.assign(t.L, 0);
  int R = 0;
  for (int q = 1; q <= t.L; ++q) {
    h->off[q - 1] = R;
    R += h->rcols[q - 1];
  }
  h->R = R;
  HODLR_TRY(h->Y.ensure((size_t)n * std::max(R, 1) * h->esize));
  HODLR_TRY(h->W.ensure((size_t)n * std::max(R, 1) * h->esize));
  HODLR_TRY(alloc_E(h.get()));
  h->sinv_off.assign(t.L, 0);
  size_t tot = 0;
  for (int p = 0; p < t.L; ++p) {
    h->sinv_off[p] = tot;
    tot += (size_t)(1 << p) * (2 * (size_t)h->rcols[p]) * (2 * (size_t)h->rcols[p]);
  }
  HODLR_TRY(h->Sinv.ensure(std::max<size_t>(tot, 1) * h->esize));
  HODLR_TRY(ensure_work(h.get(), 8));
  HODLR_HIP(hipMemcpyAsync(h->d_rank.p, h->rank.data(), t.nnodes() * sizeof(int),
                           hipMemcpyHostToDevice, stream));
  HODLR_TRY(launch_stage_leaves_packed(h.get(), leaves, stream));
  if (t.L > 0) HODLR_TRY(launch_from_f64_panels(h.get(), Upanel, Vpanel, stream));
  HODLR_HIP(hipStreamSynchronize(stream));
  *out = h.release();
  return HODLR_OK;
}

static int factor_checks(hodlr_t h) {
  if (!h) return fail(HODLR_EINVAL, "handle is NULL");
  if (h->factored) return fail(HODLR_EINVAL, "handle is already factorized");
  if (h->leaf_singular >= 0) return fail(HODLR_ESINGULAR, "singular leaf block " + std::to_string(h->leaf_singular));
  return HODLR_OK;
}

int hodlr_factor(hodlr_t h, hipStream_t stream) {
  HODLR_TRY(factor_checks(h));
  HODLR_TRY(factor_impl(h, stream));
  // the status words come back through pinned host memory, written by a
  // kernel behind the factorization, with one synchronization
  void* pin = nullptr;
  size_t pin_bytes = 0;
  HODLR_TRY(pinned_alloc(16 * sizeof(int), &pin, &pin_bytes));
  struct PinGuard {
    void* p;
    size_t b;
    ~PinGuard() { pinned_free(p, b); }
  } pin_guard{pin, pin_bytes};
  int* dpin = nullptr;
  HODLR_HIP(hipHostGetDevicePointer(reinterpret_cast<void**>(&dpin), pin, 0));
  k_export_ints<<<1, 64, 0, stream>>>(h->status.as<int>(), 4, h->status.as<int>(), nullptr, dpin);
  HODLR_HIP(hipGetLastError());
  HODLR_HIP(hipStreamSynchronize(stream));
  const int* st = static_cast<const int*>(pin);
  if (st[0]) return singular_status(st);
  h->factored = true;
  return HODLR_OK;
}

int hodlr_factor_async(hodlr_t h, hipStream_t stream) {
  HODLR_TRY(factor_checks(h));
  if (!h->pin_status) {
    void* pin = nullptr;
    HODLR_TRY(pinned_alloc(16 * sizeof(int), &pin, &h->pin_status_bytes));
    h->pin_status = static_cast<int*>(pin);
  }
  if (!h->status_ev) HODLR_TRY(event_take(&h->status_ev));
  HODLR_TRY(factor_impl(h, stream));
  int* dpin = nullptr;
  HODLR_HIP(hipHostGetDevicePointer(reinterpret_cast<void**>(&dpin), h->pin_status, 0));
  k_export_ints<<<1, 64, 0, stream>>>(h->status.as<int>(), 4, h->status.as<int>(), nullptr, dpin);
  HODLR_HIP(hipGetLastError());
  HODLR_HIP(hipEventRecord(h->status_ev, stream));
  h->factored = true;
  h->status_pending = true;
  return HODLR_OK;
}

int hodlr_factor_wait(hodlr_t h) {
  if (!h) return fail(HODLR_EINVAL, "handle is NULL");
  return settle_factor_status(h);
}

// one stream per front of a batch (default priority), kept for the process
static std::mutex g_pool_mu;
static std::vector<hipStream_t> g_pool;

static int stream_pool(int count, std::vector<hipStream_t>* out) {
  std::lock_guard<std::mutex> lk(g_pool_mu);
  while ((int)g_pool.size() < count) {
    hipStream_t s = nullptr;
    HODLR_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    g_pool.push_back(s);
  }
  out->assign(g_pool.begin(), g_pool.begin() + count);
  return HODLR_OK;
}

int hodlr_factor_batched(hodlr_t* hs, int nh, hipStream_t stream) {
  if (!hs || nh < 1) return fail(HODLR_EINVAL, "need at least one handle");
  if (nh > 4096) return fail(HODLR_EINVAL, "at most 4096 handles per batch");
  for (int f = 0; f < nh; ++f) {
    if (!hs[f]) return fail(HODLR_EINVAL, "handle " + std::to_string(f) + " is NULL");
    if (hs[f]->factored) return fail(HODLR_EINVAL, "handle " + std::to_string(f) + " is already factorized");
    if (hs[f]->leaf_singular >= 0)
      return fail(HODLR_ESINGULAR, "front " + std::to_string(f) + ": singular leaf block " +
                                       std::to_string(hs[f]->leaf_singular));
    for (int g = 0; g < f; ++g)
      if (hs[g] == hs[f]) return fail(HODLR_EINVAL, "a handle appears twice in the batch");
  }
  // first pass outside the capture: everything is sized, so the captured pass
  // allocates and synchronizes nothing
  for (int f = 0; f < nh; ++f) {
    hodlr_s* h = hs[f];
    if (h->tree.L > 0 && h->R > 0) {
      HODLR_TRY(ensure_work(h, 64));
      size_t tb = 0, wb = 0;
      for (int q = 1; q <= h->tree.L; ++q) {
        const size_t rq = h->rcols[q - 1], zc = h->off[q - 1] + rq, nq = (size_t)1 << q;
        tb += 3 * gemm_table_bound((int)nq) + 2 * gemm_table_bound((int)nq / 2);
        wb += nq * rq * zc * (size_t)std::max(1, h->tree.max_size(q) / 128) * h->esize + 256;
      }
      HODLR_TRY(gemm_prepare(h, tb, wb, stream));
    }
  }
  HODLR_HIP(hipStreamSynchronize(stream));
  // the graph is recorded on a pool stream (the caller's may be the legacy
  // default stream, which cannot capture) and launched on the caller's
  std::vector<hipStream_t> ss;
  HODLR_TRY(stream_pool(nh + 1, &ss));
  hipStream_t cs = ss[nh];
  std::vector<hipEvent_t> ev(nh + 1, nullptr);
  for (auto& e : ev) HODLR_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  struct Cleanup {
    std::vector<hipEvent_t>& ev;
    hodlr_t* hs;
    int nh;
    ~Cleanup() {
      for (auto e : ev)
        if (e) (void)hipEventDestroy(e);
      for (int f = 0; f < nh; ++f) hs[f]->capturing = false;
      prof_suspend(false);
    }
  } cleanup{ev, hs, nh};
  prof_suspend(true);
  HODLR_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
  int st = HODLR_OK;
  st = hipEventRecord(ev[nh], cs) == hipSuccess ? HODLR_OK : fail(HODLR_EHIP, "event record");
  // every front on its own stream: independent branches of one graph
  for (int f = 0; f < nh && st == HODLR_OK; ++f) {
    hodlr_s* h = hs[f];
    if (hipStreamWaitEvent(ss[f], ev[nh], 0) != hipSuccess) {
      st = fail(HODLR_EHIP, "stream wait");
      break;
    }
    h->capturing = true;
    st = factor_impl(h, ss[f]);
    h->capturing = false;
    if (st != HODLR_OK) break;
    if (hipEventRecord(ev[f], ss[f]) != hipSuccess || hipStreamWaitEvent(cs, ev[f], 0) != hipSuccess)
      st = fail(HODLR_EHIP, "event join");
  }
  hipGraph_t graph = nullptr;
  const hipError_t ec = hipStreamEndCapture(cs, &graph);
  if (st != HODLR_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return st;
  }
  if (ec != hipSuccess) return fail(HODLR_EHIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(ec));
  hipGraphExec_t exec = nullptr;
  const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  if (ei != hipSuccess) {
    (void)hipGraphDestroy(graph);
    return fail(HODLR_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(ei));
  }
  {
    ProfScope prof("factor_graph", stream);
    const hipError_t el = hipGraphLaunch(exec, stream);
    if (el != hipSuccess) st = fail(HODLR_EHIP, std::string("hipGraphLaunch: ") + hipGetErrorString(el));
  }
  const hipError_t es = hipStreamSynchronize(stream);
  (void)hipGraphExecDestroy(exec);
  (void)hipGraphDestroy(graph);
  if (st != HODLR_OK) return st;
  if (es != hipSuccess) return fail(HODLR_EHIP, std::string("hipStreamSynchronize: ") + hipGetErrorString(es));
  for (int f = 0; f < nh; ++f) {
    int sv[4];
    HODLR_HIP(hipMemcpy(sv, hs[f]->status.p, sizeof(sv), hipMemcpyDeviceToHost));
    if (sv[0])
      return fail(HODLR_ESINGULAR, "front " + std::to_string(f) + ": " +
                                       (sv[0] == 1 ? "singular leaf block " : "singular capacitance matrix at node ") +
                                       std::to_string(sv[1]));
  }
  for (int f = 0; f < nh; ++f) hs[f]->factored = true;
  return HODLR_OK;
}

int hodlr_solve(hodlr_t h, const void* B, int nrhs, int ldb, void* X, int ldx,
                hipStream_t stream) {
  if (!h) return fail(HODLR_EINVAL, "handle is NULL");
  if (!h->factored) return fail(HODLR_EINVAL, "call hodlr_factor first");
  if (h->status_pending) HODLR_HIP(hipStreamWaitEvent(stream, h->status_ev, 0));
  int n = h->tree.n;
  if (nrhs < 0) return fail(HODLR_EINVAL, "nrhs < 0");
  if (nrhs == 0) return HODLR_OK;
  if (!B || !X) return fail(HODLR_EINVAL, "B or X is NULL");
  if (ldb < n || ldx < n) return fail(HODLR_EINVAL, "ldb or ldx < n");
  if (B != X) {
    HODLR_HIP(hipMemcpy2DAsync(X, (size_t)ldx * h->esize, B, (size_t)ldb * h->esize,
                               (size_t)n * h->esize, nrhs, hipMemcpyDeviceToDevice, stream));
  } else if (ldb != ldx) {
    return fail(HODLR_EINVAL, "aliased B and X need ldb == ldx");
  }
  HODLR_TRY(apply_impl(h, X, ldx, nrhs, stream));
  return mark_inflight(h, stream);
}

int gmres_solve(const double* K, int n, int ldk, hodlr_t precond, const double* B, int nrhs,
                int ldb, double* X, int ldx, double tol, int maxit, int restart, int* iters,
                double* relres, hipStream_t stream) {
  if (!K || !B || !X) return fail(HODLR_EINVAL, "K, B or X is NULL");
  if (n < 1 || n > kMaxN) return fail(HODLR_EINVAL, "n out of range");
  if (ldk < n || ldb < n || ldx < n) return fail(HODLR_EINVAL, "leading dimension < n");
  if (nrhs < 1 || nrhs > 64) return fail(HODLR_EINVAL, "nrhs must be in [1, 64]");
  if (!(tol > 0.0)) return fail(HODLR_EINVAL, "tol must be > 0");
  if (maxit < 1 || restart < 1) return fail(HODLR_EINVAL, "maxit and restart must be >= 1");
  if (!iters || !relres) return fail(HODLR_EINVAL, "iters or relres is NULL");
  if (precond) {
    if (!precond->factored) return fail(HODLR_EINVAL, "preconditioner is not factorized");
    if (precond->tree.n != n) return fail(HODLR_EINVAL, "preconditioner size differs from n");
  }
  const int st = gmres_impl(K, n, ldk, precond, B, nrhs, ldb, X, ldx, tol, maxit, restart, iters, relres,
                    stream);
  // (an error return may leave work queued behind the preconditioner)
  if (precond && st != HODLR_OK && st != HODLR_ENOCONV) (void)mark_inflight(precond, stream);
  return st;
}

int gmres_solve_noalloc(const double* K, int n, int ldk, hodlr_t precond, const double* B, int nrhs, int ldb,
                        double* X, int ldx, double tol, int maxit, int restart, int* iters, double* relres,
                        hipStream_t stream) {
  if (!K || !B || !X) return fail(HODLR_EINVAL, "K, B or X is NULL");
  if (n < 1 || n > kMaxN) return fail(HODLR_EINVAL, "n out of range");
  if (ldk < n || ldb < n || ldx < n) return fail(HODLR_EINVAL, "leading dimension < n");
  if (nrhs < 1 || nrhs > 64) return fail(HODLR_EINVAL, "nrhs must be in [1, 64]");
  if (!(tol > 0.0)) return fail(HODLR_EINVAL, "tol must be > 0");
  if (maxit < 1 || restart < 1) return fail(HODLR_EINVAL, "maxit and restart must be >= 1");
  if (!iters || !relres) return fail(HODLR_EINVAL, "iters or relres is NULL");
  if (precond) {
    if (!precond->factored) return fail(HODLR_EINVAL, "preconditioner is not factorized");
    if (precond->tree.n != n) return fail(HODLR_EINVAL, "preconditioner size differs from n");
  }
  const size_t need = gmres_noalloc_bytes(n, nrhs, restart, precond ? precond->precision : 0);
  if (need > gmres_noalloc_limit())
    return fail(HODLR_EINVAL, "gmres_solve_noalloc: n x nrhs x (restart + 1) needs " + std::to_string(need) +
                                  " bytes of workspace, above the fixed " + std::to_string(gmres_noalloc_limit()) +
                                  " bytes");
  const int st = gmres_impl(K, n, ldk, precond, B, nrhs, ldb, X, ldx, tol, maxit, restart, iters, relres, stream, true);
  // (an error return may leave work queued behind the preconditioner)
  if (precond && st != HODLR_OK && st != HODLR_ENOCONV) (void)mark_inflight(precond, stream);
  return st;
}

int cg_solve(const double* K, int n, int ldk, hodlr_t precond, const double* B, int nrhs, int ldb, double* X,
             int ldx, double tol, int maxit, int* iters, double* relres, hipStream_t stream) {
  if (!K || !B || !X) return fail(HODLR_EINVAL, "K, B or X is NULL");
  if (n < 1 || n > kMaxN) return fail(HODLR_EINVAL, "n out of range");
  if (ldk < n || ldb < n || ldx < n) return fail(HODLR_EINVAL, "leading dimension < n");
  if (nrhs < 1 || nrhs > 64) return fail(HODLR_EINVAL, "nrhs must be in [1, 64]");
  if (!(tol > 0.0)) return fail(HODLR_EINVAL, "tol must be > 0");
  if (maxit < 1) return fail(HODLR_EINVAL, "maxit must be >= 1");
  if (!iters || !relres) return fail(HODLR_EINVAL, "iters or relres is NULL");
  if (precond) {
    if (!precond->factored) return fail(HODLR_EINVAL, "preconditioner is not factorized");
    if (precond->tree.n != n) return fail(HODLR_EINVAL, "preconditioner size differs from n");
  }
  const int st = cg_impl(K, n, ldk, precond, B, nrhs, ldb, X, ldx, tol, maxit, iters, relres, stream);
  // (an error return may leave work queued behind the preconditioner)
  if (precond && st != HODLR_OK && st != HODLR_ENOCONV) (void)mark_inflight(precond, stream);
  return st;
}

int hodlr_build_batched(int nf, const double* const* K, const int* n, const int* ldk,
                        const int* const* g_rowptr, const int* const* g_col, const float* const* coords,
                        const hodlr_opts* opts, hipStream_t stream, hodlr_t* out) {
  if (nf < 1 || nf > 65536) return fail(HODLR_EINVAL, "nf must be in [1, 65536]");
  if (!K || !n || !ldk || !out) return fail(HODLR_EINVAL, "K, n, ldk or out is NULL");
  for (int f = 0; f < nf; ++f) out[f] = nullptr;
  std::string msg;
  const int st = Workers::get().run(
      nf,
      [&](int f, hipStream_t s) {
        return hodlr_build(K[f], n[f], ldk[f], g_rowptr ? g_rowptr[f] : nullptr, g_col ? g_col[f] : nullptr,
                           coords ? coords[f] : nullptr, opts, s, &out[f]);
      },
      stream, &msg);
  if (st != HODLR_OK) {
    for (int f = 0; f < nf; ++f) {
      if (out[f]) hodlr_destroy(out[f]);
      out[f] = nullptr;
    }
    return fail(st, msg);
  }
  return HODLR_OK;
}

int hodlr_order_batched(int nf, const float* const* coords, const int* n, int leaf, const double* const* K,
                        const int* ldk, const int* const* g_rowptr, const int* const* g_col, int* const* perm,
                        double* const* Kout, const int* ldo, int* const* rowptr_out, int* const* col_out,
                        hipStream_t stream) {
  if (nf < 1 || nf > 65536) return fail(HODLR_EINVAL, "nf must be in [1, 65536]");
  if (!coords || !n || !K || !ldk || !perm || !Kout || !ldo) return fail(HODLR_EINVAL, "NULL argument array");
  if (g_rowptr && (!g_col || !rowptr_out || !col_out)) return fail(HODLR_EINVAL, "graph arrays incomplete");
  std::string msg;
  const int st = Workers::get().run(
      nf,
      [&](int f, hipStream_t s) -> int {
        HODLR_TRY(hodlr_order_rcb(coords[f], n[f], leaf, perm[f], s));
        HODLR_TRY(hodlr_permute(K[f], n[f], ldk[f], perm[f], Kout[f], ldo[f], s));
        if (g_rowptr)
          HODLR_TRY(hodlr_permute_graph(g_rowptr[f], g_col[f], n[f], perm[f], rowptr_out[f], col_out[f], s));
        return HODLR_OK;
      },
      stream, &msg);
  if (st != HODLR_OK) return fail(st, msg);
  return HODLR_OK;
}

int gmres_solve_batched(int nf, const double* const* K, const int* n, const int* ldk, const hodlr_t* precond,
                        const double* const* B, int nrhs, const int* ldb, double* const* X, const int* ldx,
                        double tol, int maxit, int restart, int* iters, double* relres, hipStream_t stream) {
  if (nf < 1 || nf > 65536) return fail(HODLR_EINVAL, "nf must be in [1, 65536]");
  if (!K || !n || !ldk || !B || !ldb || !X || !ldx || !iters || !relres)
    return fail(HODLR_EINVAL, "NULL argument array");
  std::string msg;
  const int st = Workers::get().run(
      nf,
      [&](int f, hipStream_t s) {
        return gmres_solve(K[f], n[f], ldk[f], precond ? precond[f] : nullptr, B[f], nrhs, ldb[f], X[f], ldx[f],
                           tol, maxit, restart, iters + (size_t)f * nrhs, relres + (size_t)f * nrhs, s);
      },
      stream, &msg);
  if (st != HODLR_OK) return fail(st, msg);
  return HODLR_OK;
}

int hodlr_order_rcb(const float* coords, int n, int leaf, int* perm, hipStream_t stream) {
  if (!coords || !perm) return fail(HODLR_EINVAL, "coords or perm is NULL");
  if (n < 1 || n > 16384) return fail(HODLR_EINVAL, "n must be in [1, 16384]");
  if (leaf < 1) return fail(HODLR_EINVAL, "leaf must be >= 1");
  Tree t;
  t.build(n, leaf);
  return launch_rcb(coords, n, t, perm, stream);
}

int hodlr_permute(const double* Kin, int n, int ldi, const int* perm, double* Kout, int ldo,
                  hipStream_t stream) {
  if (!Kin || !Kout || !perm) return fail(HODLR_EINVAL, "NULL pointer");
  if (n < 1 || ldi < n || ldo < n) return fail(HODLR_EINVAL, "bad size");
  if (Kin == Kout) return fail(HODLR_EINVAL, "Kin and Kout must not overlap");
  return launch_permute(Kin, n, ldi, perm, Kout, ldo, stream);
}

int hodlr_permute_rows(const float* in, int n, int width, const int* perm, float* out, hipStream_t stream) {
  if (!in || !perm || !out) return fail(HODLR_EINVAL, "NULL pointer");
  if (n < 1 || width < 1 || width > 16) return fail(HODLR_EINVAL, "n < 1 or width not in [1, 16]");
  if (in == out) return fail(HODLR_EINVAL, "in and out must not overlap");
  return launch_permute_rows(in, n, width, perm, out, stream);
}

int hodlr_permute_graph(const int* rowptr, const int* col, int n, const int* perm,
                        int* rowptr_out, int* col_out, hipStream_t stream) {
  if (!rowptr || !col || !perm || !rowptr_out || !col_out) return fail(HODLR_EINVAL, "NULL pointer");
  if (n < 1) return fail(HODLR_EINVAL, "n < 1");
  return launch_permute_graph(rowptr, col, n, perm, rowptr_out, col_out, stream);
}

int hodlr_stats(hodlr_t h, int* nlevels, int* ranks, int* rcols) {
  if (!h) return fail(HODLR_EINVAL, "handle is NULL");
  const Tree& t = h->tree;
  if (nlevels) *nlevels = t.L;
  if (ranks)
    for (int id = 1; id < t.nnodes(); ++id) ranks[id - 1] = h->rank[id];
  if (rcols)
    for (int q = 0; q < t.L; ++q) rcols[q] = h->rcols[q];
  return HODLR_OK;
}

int hodlr_get_factors(hodlr_t h, double* Upanel, double* Vpanel, hipStream_t stream) {
  if (!h) return fail(HODLR_EINVAL, "handle is NULL");
  if (h->factored) return fail(HODLR_EINVAL, "factors are overwritten by hodlr_factor");
  if (!Upanel || !Vpanel) return fail(HODLR_EINVAL, "NULL pointer");
  if (h->tree.L == 0 || h->R == 0) return HODLR_OK;
  HODLR_TRY(launch_to_f64_panels(h, Upanel, Vpanel, stream));
  return mark_inflight(h, stream);
}

int hodlr_skel_info(hodlr_t h, int* kused) {
  if (!h) return fail(HODLR_EINVAL, "handle is NULL");
  if (!kused) return fail(HODLR_EINVAL, "kused is NULL");
  const Tree& t = h->tree;
  for (int id = 1; id < t.nnodes(); ++id) kused[id - 1] = h->skel_k.empty() ? -1 : h->skel_k[id];
  return HODLR_OK;
}

int hodlr_skel_features(const int* g_rowptr, const int* g_col, const float* coords, const double* K, int n,
                        int ldk, int leaf, float* feats, hipStream_t stream) {
  if (!g_rowptr || !g_col || !coords || !K || !feats) return fail(HODLR_EINVAL, "NULL pointer argument");
  if (n < 2 || n > 16384) return fail(HODLR_EINVAL, "n must be in [2, 16384]");
  if (ldk < n) return fail(HODLR_EINVAL, "ldk < n");
  if (leaf < 1 || leaf > kLeafMax) return fail(HODLR_EINVAL, "leaf out of range");
  if (reinterpret_cast<uintptr_t>(feats) % 16) return fail(HODLR_EINVAL, "feats must be 16-byte aligned");
  Tree t;
  t.build(n, leaf);
  if (t.L == 0) return fail(HODLR_EINVAL, "n <= leaf: the tree has no off-diagonal blocks");
  return launch_skel_features(g_rowptr, g_col, coords, K, ldk, skel_blocks(t), feats, stream);
}

int hodlr_skel_labels(const double* K, int n, int ldk, const int* g_rowptr, const int* g_col, int leaf,
                      double tol, int precision, int source, int depth, float* labels, hipStream_t stream) {
  if (!K || !labels) return fail(HODLR_EINVAL, "NULL pointer argument");
  if (n < 2 || n > 16384) return fail(HODLR_EINVAL, "n must be in [2, 16384]");
  if (source != 0 && source != 1) return fail(HODLR_EINVAL, "source must be 0 (ACA) or 1 (skeleton LU)");
  hodlr_opts o;
  hodlr_default_opts(&o);
  o.leaf = leaf;
  o.tol = tol;
  o.precision = precision;
  o.method = source == 0 ? HODLR_ACA : HODLR_BDLR;
  o.bdlr_depth = depth;
  HODLR_TRY(check_opts(o));
  Tree t;
  t.build(n, leaf);
  if (t.L == 0) return fail(HODLR_EINVAL, "n <= leaf: the tree has no off-diagonal blocks");
  const int kcap = source == 0 ? rank_cap(precision) : skel_stride(precision);
  DevBuf piv;
  HODLR_TRY(piv.ensure((size_t)t.nnodes() * 2 * kcap * sizeof(int)));
  hodlr_t h = nullptr;
  HODLR_TRY(build_impl(K, n, ldk, g_rowptr, g_col, nullptr, &o, stream, &h, piv.as<int>()));
  std::unique_ptr<hodlr_s> hold(h);
  return launch_skel_labels(skel_blocks(t), piv.as<int>(), kcap, h->d_rank.as<int>(), labels, stream);
}

int hodlr_mlp_forward(const float* feats, int N, const float* params, int bf16, float* logits,
                      hipStream_t stream) {
  if (!feats || !params || !logits) return fail(HODLR_EINVAL, "NULL pointer argument");
  if (N < 0) return fail(HODLR_EINVAL, "N < 0");
  return launch_mlp_forward(feats, N, params, bf16 ? 1 : 0, logits, stream);
}

int hodlr_mlp_grad(const float* feats, const float* labels, int N, const float* params, int bf16,
                   float pos_weight, float* grad, float* loss, hipStream_t stream) {
  if (!feats || !labels || !params || !grad) return fail(HODLR_EINVAL, "NULL pointer argument");
  if (N < 1) return fail(HODLR_EINVAL, "N must be >= 1");
  return launch_mlp_grad(feats, labels, N, const_cast<float*>(params), bf16 ? 1 : 0, pos_weight, grad, loss,
                         nullptr, nullptr, 0, 0.f, 0.f, 0.f, 0.f, stream);
}

int hodlr_mlp_adam_step(const float* feats, const float* labels, int N, float* params, float* m, float* v,
                        int step, float lr, float pos_weight, float* loss, hipStream_t stream) {
  if (!feats || !labels || !params || !m || !v) return fail(HODLR_EINVAL, "NULL pointer argument");
  if (N < 1) return fail(HODLR_EINVAL, "N must be >= 1");
  if (step < 1) return fail(HODLR_EINVAL, "step must be >= 1");
  return launch_mlp_grad(feats, labels, N, params, 1, pos_weight, nullptr, loss, m, v, step, lr, 0.9f, 0.999f,
                         1e-8f, stream);
}

int hodlr_destroy(hodlr_t h) {
  if (!h) return HODLR_OK;
  // the handle's blocks go back to the allocator cache: work still queued on
  // them must finish first (the calls that leave work queued recorded events)
  bool busy = h->status_pending && hipEventQuery(h->status_ev) != hipSuccess;
  for (hipEvent_t e : h->inflight) busy = busy || hipEventQuery(e) != hipSuccess;
  (void)hipGetLastError();  // a not-ready query leaves no error behind
  if (busy) HODLR_HIP(hipDeviceSynchronize());
  delete h;
  return HODLR_OK;
}

int hodlr_release_memory(void) {
  release_cached_memory();
  return HODLR_OK;
}

}  // extern "C"
