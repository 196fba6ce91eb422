// Batched small dense products for the factorization (Sec. 4.3.1): the panel
// products V^T Z, the capacitance blocks of eq. SchurSum and the correction
// operators.  Each task is one C = alpha op(A) B (+ C or + I) with op(A) = A
// or A^T; all tasks of a call go out in one launch, 64 x 64 output tiles per
// workgroup, and a long inner dimension can be split over workgroups whose
// partial tiles are summed by a second launch in a fixed order.
#include <algorithm>
#include <cstring>
#include <vector>

#include "gemm.h"
#include "hodlr_internal.h"

namespace hodlr {

namespace {

constexpr int kTile = 64, kKc = 32;  // tile side; K splits are multiples of kKc
// K chunk staged in LDS per step: 32 (float), 16 (double)
template <typename T> constexpr int chunk_k() { return sizeof(T) == 8 ? 16 : 32; }

struct TaskDev {
  const void* A;
  const void* B;
  void* C;
  int m, n, k, lda, ldb, ldc, transA, mode;
  double alpha;
  int tiles_m, tiles_n, ksplit, kchunk;
  long long cstride;
  int tile0;
};

// C tile (64 x 64) = alpha op(A) B over k in [kb, ke); thread (tx, ty) owns
// rows tx + 16 u and columns ty + 16 v.  The next K chunk is loaded into
// registers while the current one is multiplied out of LDS.
template <typename T>
__global__ void __launch_bounds__(kBlock)
    k_gemm_batched(const TaskDev* __restrict__ tasks, int ntask) {
  constexpr int KC = chunk_k<T>(), NL = kTile * KC / kBlock;
  __shared__ T As[2][KC][kTile + 1];
  __shared__ T Bs[2][KC][kTile + 1];
  __shared__ int s_task;
  const int t = threadIdx.x, tx = t & 15, ty = t >> 4;
  if (t == 0) {
    int lo = 0, hi = ntask - 1;
    while (lo < hi) {  // last task with tile0 <= blockIdx.x
      const int mid = (lo + hi + 1) >> 1;
      if (tasks[mid].tile0 <= (int)blockIdx.x) lo = mid;
      else hi = mid - 1;
    }
    s_task = lo;
  }
  __syncthreads();
  const TaskDev tk = tasks[s_task];
  int rem = blockIdx.x - tk.tile0;
  const int tm = rem % tk.tiles_m;
  rem /= tk.tiles_m;
  const int tn = rem % tk.tiles_n;
  const int ks = rem / tk.tiles_n;
  const int i0 = tm * kTile, j0 = tn * kTile;
  const int kb = ks * tk.kchunk, ke = min(tk.k, kb + tk.kchunk);
  const T* A = static_cast<const T*>(tk.A);
  const T* B = static_cast<const T*>(tk.B);
  T* C = static_cast<T*>(tk.C) + (size_t)ks * tk.cstride;
  // loads: 64 x KC of op(A) and KC x 64 of B, NL elements each per thread
  T av[NL], bv[NL];
  auto load = [&](int k0) {
#pragma unroll
    for (int u = 0; u < NL; ++u) {
      const int e = t + u * kBlock;
      if (tk.transA) {  // op(A)(i, kk) = A[kk + i lda]: contiguous along kk
        const int kk = e % KC, i = e / KC;
        av[u] = (i0 + i < tk.m && k0 + kk < ke) ? A[(size_t)(i0 + i) * tk.lda + k0 + kk] : T(0);
      } else {  // A[i + kk lda]: contiguous along i
        const int i = e % kTile, kk = e / kTile;
        av[u] = (i0 + i < tk.m && k0 + kk < ke) ? A[(size_t)(k0 + kk) * tk.lda + i0 + i] : T(0);
      }
      const int kk = e % KC, j = e / KC;
      bv[u] = (j0 + j < tk.n && k0 + kk < ke) ? B[(size_t)(j0 + j) * tk.ldb + k0 + kk] : T(0);
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int u = 0; u < NL; ++u) {
      const int e = t + u * kBlock;
      if (tk.transA) As[buf][e % KC][e / KC] = av[u];
      else As[buf][e / kTile][e % kTile] = av[u];
      Bs[buf][e % KC][e / KC] = bv[u];
    }
  };
  T acc[4][4];
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[u][v] = T(0);
  int buf = 0;
  if (kb < ke) {
    load(kb);
    store(0);
  }
  __syncthreads();
  for (int k0 = kb; k0 < ke; k0 += KC) {
    const bool more = k0 + KC < ke;
    if (more) load(k0 + KC);
#pragma unroll 8
    for (int kk = 0; kk < KC; ++kk) {
      T a[4], b[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        a[u] = As[buf][kk][tx + 16 * u];
        b[u] = Bs[buf][kk][ty + 16 * u];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[u][v] = fma(a[u], b[v], acc[u][v]);
    }
    if (more) store(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }
  const T alpha = (T)tk.alpha;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int j = j0 + ty + 16 * v;
    if (j >= tk.n) continue;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int i = i0 + tx + 16 * u;
      if (i >= tk.m) continue;
      T* cp = C + i + (size_t)j * tk.ldc;
      T val = alpha * acc[u][v];
      if (tk.ksplit == 1) {
        if (tk.mode == kGemmAccumulate) val += *cp;
        else if (tk.mode == kGemmAddIdentity && i == j) val += T(1);
      }
      *cp = val;
    }
  }
}

// C = sum over the split slices (+ C or + I), one thread per element.
template <typename T>
__global__ void __launch_bounds__(kBlock)
    k_gemm_reduce(const TaskDev* __restrict__ tasks, const void* const* __restrict__ parts) {
  const TaskDev tk = tasks[blockIdx.y];
  if (tk.ksplit == 1) return;
  const T* P = static_cast<const T*>(parts[blockIdx.y]);
  T* C = static_cast<T*>(tk.C);
  for (int e = blockIdx.x * kBlock + threadIdx.x; e < tk.m * tk.n; e += gridDim.x * kBlock) {
    const int i = e % tk.m, j = e / tk.m;
    T s = T(0);
    for (int q = 0; q < tk.ksplit; ++q) s += P[(size_t)q * tk.cstride + i + (size_t)j * tk.ldc];
    T* cp = C + i + (size_t)j * tk.ldc;
    if (tk.mode == kGemmAccumulate) s += *cp;
    else if (tk.mode == kGemmAddIdentity && i == j) s += T(1);
    *cp = s;
  }
}

// Reserves `bytes` (256-aligned) of an arena.  Growing it first drains the
// stream, since earlier launches may still read the old block; under stream
// capture that is impossible, so the arenas must have been sized beforehand
// (gemm_prepare).
static int arena_take(hodlr_s* h, DevBuf& buf, size_t& used, size_t bytes, hipStream_t s, void** out) {
  bytes = (bytes + 255) & ~(size_t)255;
  if (used + bytes > buf.bytes) {
    if (h->capturing) return fail(HODLR_EINVAL, "batched-product arena too small under graph capture");
    HODLR_HIP(hipStreamSynchronize(s));
    HODLR_TRY(buf.ensure(std::max(2 * buf.bytes, used + bytes + (1 << 16))));
    used = 0;
  }
  *out = static_cast<char*>(buf.p) + used;
  used += bytes;
  return HODLR_OK;
}

// Task tables are written to pinned host staging at the same offset as their
// device copy, so an asynchronous (or captured) copy reads memory that stays
// valid until the next factorization of the handle.
static int stage_tables(hodlr_s* h, const void* src, size_t bytes, void* dev, hipStream_t s) {
  const size_t off = static_cast<char*>(dev) - static_cast<char*>(h->gemm_tab.p);
  if (h->gemm_host_bytes < h->gemm_tab.bytes) {
    if (h->capturing) return fail(HODLR_EINVAL, "batched-product staging too small under graph capture");
    HODLR_HIP(hipStreamSynchronize(s));
    if (h->gemm_host) HODLR_HIP(hipHostFree(h->gemm_host));
    h->gemm_host = nullptr;
    h->gemm_host_bytes = 0;
    HODLR_HIP(hipHostMalloc(&h->gemm_host, h->gemm_tab.bytes));
    h->gemm_host_bytes = h->gemm_tab.bytes;
  }
  char* hp = static_cast<char*>(h->gemm_host) + off;
  std::memcpy(hp, src, bytes);
  HODLR_HIP(hipMemcpyAsync(dev, hp, bytes, hipMemcpyHostToDevice, s));
  return HODLR_OK;
}

template <typename T>
int gemm_batched_t(hodlr_s* h, const std::vector<GemmTask>& in, hipStream_t s) {
  std::vector<TaskDev> tasks;
  int tiles = 0, maxmn = 0, nsplit = 0;
  size_t work_elems = 0;
  for (const GemmTask& g : in) {
    if (g.m <= 0 || g.n <= 0) continue;
    TaskDev d{};
    d.A = g.A;
    d.B = g.B;
    d.C = g.C;
    d.m = g.m;
    d.n = g.n;
    d.k = g.k;
    d.lda = g.lda;
    d.ldb = g.ldb;
    d.ldc = g.ldc;
    d.transA = g.transA;
    d.mode = g.mode;
    d.alpha = g.alpha;
    d.tiles_m = (g.m + kTile - 1) / kTile;
    d.tiles_n = (g.n + kTile - 1) / kTile;
    const int ks = std::max(1, std::min(g.ksplit, (g.k + kKc - 1) / kKc));
    d.kchunk = std::max(kKc, ((g.k + ks - 1) / ks + kKc - 1) / kKc * kKc);
    d.ksplit = g.k > 0 ? (g.k + d.kchunk - 1) / d.kchunk : 1;
    d.tile0 = tiles;
    tiles += d.tiles_m * d.tiles_n * d.ksplit;
    if (d.ksplit > 1) {
      // partial tiles: slices laid out like C (ld ldc), summed by k_gemm_reduce
      d.cstride = (long long)g.ldc * g.n;
      work_elems += (size_t)d.cstride * d.ksplit;
      maxmn = std::max(maxmn, d.m * d.n);
      ++nsplit;
    }
    tasks.push_back(d);
  }
  if (tasks.empty()) return HODLR_OK;
  std::vector<TaskDev> red;
  std::vector<const void*> parts;
  if (nsplit) {
    void* w = nullptr;
    HODLR_TRY(arena_take(h, h->gemm_work, h->gemm_work_used, work_elems * sizeof(T), s, &w));
    T* wp = static_cast<T*>(w);
    for (TaskDev& d : tasks) {
      if (d.ksplit == 1) continue;
      TaskDev r = d;  // the sum goes to the caller's C
      red.push_back(r);
      parts.push_back(wp);
      d.C = wp;
      wp += (size_t)d.cstride * d.ksplit;
    }
  }
  // one block of the table arena: tasks, then the sums' tasks and their parts
  const size_t b0 = tasks.size() * sizeof(TaskDev), b1 = red.size() * sizeof(TaskDev);
  const size_t o1 = (b0 + 255) & ~(size_t)255, o2 = o1 + ((b1 + 255) & ~(size_t)255);
  void* tab = nullptr;
  HODLR_TRY(arena_take(h, h->gemm_tab, h->gemm_tab_used, o2 + parts.size() * sizeof(void*), s, &tab));
  char* tb = static_cast<char*>(tab);
  HODLR_TRY(stage_tables(h, tasks.data(), b0, tb, s));
  k_gemm_batched<T><<<tiles, kBlock, 0, s>>>(reinterpret_cast<const TaskDev*>(tb), (int)tasks.size());
  HODLR_HIP(hipGetLastError());
  if (nsplit) {
    HODLR_TRY(stage_tables(h, red.data(), b1, tb + o1, s));
    HODLR_TRY(stage_tables(h, parts.data(), parts.size() * sizeof(void*), tb + o2, s));
    k_gemm_reduce<T><<<dim3(std::min(64, (maxmn + kBlock - 1) / kBlock), (unsigned)red.size()), kBlock, 0, s>>>(
        reinterpret_cast<const TaskDev*>(tb + o1), reinterpret_cast<const void* const*>(tb + o2));
    HODLR_HIP(hipGetLastError());
  }
  return HODLR_OK;
}

}  // namespace

int gemm_batched(hodlr_s* h, const std::vector<GemmTask>& tasks, hipStream_t s) {
  return h->precision == 64 ? gemm_batched_t<double>(h, tasks, s) : gemm_batched_t<float>(h, tasks, s);
}

void gemm_reset(hodlr_s* h) {
  h->gemm_tab_used = 0;
  h->gemm_work_used = 0;
}

size_t gemm_table_bound(int ntasks) {
  const size_t t = ((size_t)ntasks * sizeof(TaskDev) + 255) & ~(size_t)255;
  return 2 * t + (((size_t)ntasks * sizeof(void*) + 255) & ~(size_t)255) + 256;
}

int gemm_prepare(hodlr_s* h, size_t tab_bytes, size_t work_bytes, hipStream_t s) {
  if (h->gemm_tab.bytes < tab_bytes || h->gemm_work.bytes < work_bytes || h->gemm_host_bytes < tab_bytes) {
    HODLR_HIP(hipStreamSynchronize(s));
    if (h->gemm_tab.bytes < tab_bytes) HODLR_TRY(h->gemm_tab.ensure(tab_bytes));
    if (h->gemm_work.bytes < work_bytes) HODLR_TRY(h->gemm_work.ensure(work_bytes));
    if (h->gemm_host_bytes < h->gemm_tab.bytes) {
      if (h->gemm_host) HODLR_HIP(hipHostFree(h->gemm_host));
      h->gemm_host = nullptr;
      h->gemm_host_bytes = 0;
      HODLR_HIP(hipHostMalloc(&h->gemm_host, h->gemm_tab.bytes));
      h->gemm_host_bytes = h->gemm_tab.bytes;
    }
  }
  return HODLR_OK;
}

}  // namespace hodlr
