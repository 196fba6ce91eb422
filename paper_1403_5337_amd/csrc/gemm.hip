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

// A zero word for the loads of entries outside an operand (never written).
__device__ double g_gemm_zero[2];

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

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

// A wave's 32 x 32 accumulator on the matrix cores.  step() multiplies the
// LDS chunks A(k, i) = As[k ld + i] and B(k, j) = Bs[k ld + j] (k < KC) into
// rows wm.., columns wn.. of the tile; coord() names the (row, column) within
// the quarter of accumulator slot q of a lane.
template <typename T> struct MfmaAcc;

template <> struct MfmaAcc<float> {
  static constexpr int kN = 16;
  f32x16 d;
  __device__ void zero() { d = f32x16{}; }
  template <int KC>
  __device__ __forceinline__ void step(const float* As, const float* Bs, int ld, int wm, int wn, int lane) {
    const int ml = lane & 31, kl = lane >> 5;
#pragma unroll
    for (int k = 0; k < KC; k += 2)  // v_mfma_f32_32x32x2f32: A(m = l % 32, k = l / 32), B(k = l / 32, n = l % 32)
      d = __builtin_amdgcn_mfma_f32_32x32x2f32(As[(k + kl) * ld + wm + ml], Bs[(k + kl) * ld + wn + ml], d, 0, 0, 0);
  }
  // slot q of lane l: row 8 (q / 4) + 4 (l / 32) + q % 4, column l % 32
  __device__ static void coord(int q, int lane, int& i, int& j) {
    i = 8 * (q >> 2) + 4 * (lane >> 5) + (q & 3);
    j = lane & 31;
  }
  __device__ float get(int q) const { return d[q]; }
};

template <> struct MfmaAcc<double> {
  static constexpr int kN = 16;
  f64x4 d[2][2];
  __device__ void zero() {
    for (int x = 0; x < 2; ++x)
      for (int y = 0; y < 2; ++y) d[x][y] = f64x4{};
  }
  template <int KC>
  __device__ __forceinline__ void step(const double* As, const double* Bs, int ld, int wm, int wn, int lane) {
    const int ml = lane & 15, kl = lane >> 4;
#pragma unroll
    for (int k = 0; k < KC; k += 4) {  // v_mfma_f64_16x16x4f64: A(m = l % 16, k = l / 16), B(k = l / 16, n = l % 16)
      double a[2], b[2];
#pragma unroll
      for (int x = 0; x < 2; ++x) {
        a[x] = As[(k + kl) * ld + wm + 16 * x + ml];
        b[x] = Bs[(k + kl) * ld + wn + 16 * x + ml];
      }
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) d[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[x], b[y], d[x][y], 0, 0, 0);
    }
  }
  // slot q = 8 x + 4 y + v of lane l: block (x, y), row l / 16 + 4 v, column l % 16
  __device__ static void coord(int q, int lane, int& i, int& j) {
    const int x = q >> 3, y = (q >> 2) & 1, v = q & 3;
    i = 16 * x + (lane >> 4) + 4 * v;
    j = 16 * y + (lane & 15);
  }
  __device__ double get(int q) const { return d[q >> 3][(q >> 2) & 1][q & 3]; }
};

// C tile (64 x 64) = alpha op(A) B over k in [kb, ke), each wave a 32 x 32
// quarter on the matrix cores.  The next K chunk is loaded into registers
// while the current one is multiplied out of LDS.
template <typename T>
__global__ void __launch_bounds__(kBlock)
    k_gemm_batched(const TaskDev* __restrict__ tasks, int ntask) {
  constexpr int KC = chunk_k<T>(), NL = kTile * KC / kBlock;
  __shared__ T As[2][KC][kTile + 1];
  __shared__ T Bs[2][KC][kTile + 1];
  __shared__ int s_task;
  const int t = threadIdx.x;
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
  // the operands as global-memory pointers (the task table only holds
  // generic ones), so that their loads count on the vector-memory counter
  // alone and do not wait behind LDS traffic
  typedef const __attribute__((address_space(1))) T* GP;
  typedef __attribute__((address_space(1))) T* GPW;
  const GP A = (GP)tk.A;
  const GP B = (GP)tk.B;
  const GPW C = (GPW)tk.C + (size_t)ks * tk.cstride;
  // loads: 64 x KC of op(A) and KC x 64 of B, NL elements each per thread.
  // An entry outside the operand reads a zero word instead: the address is
  // chosen, not the value, so no load sits behind a branch and all of them
  // are in flight together.
  const GP Z = (GP)(const void*)g_gemm_zero;
  T av[NL], bv[NL];
  auto load = [&](int k0) {
    if (tk.transA) {  // op(A)(i, kk) = A[kk + i lda]: contiguous along kk
#pragma unroll
      for (int u = 0; u < NL; ++u) {
        const int e = t + u * kBlock, kk = e % KC, i = e / KC;
        const bool in = i0 + i < tk.m && k0 + kk < ke;
        av[u] = *(in ? A + (size_t)(i0 + i) * tk.lda + k0 + kk : Z);
      }
    } else {  // A[i + kk lda]: contiguous along i
#pragma unroll
      for (int u = 0; u < NL; ++u) {
        const int e = t + u * kBlock, i = e % kTile, kk = e / kTile;
        const bool in = i0 + i < tk.m && k0 + kk < ke;
        av[u] = *(in ? A + (size_t)(k0 + kk) * tk.lda + i0 + i : Z);
      }
    }
#pragma unroll
    for (int u = 0; u < NL; ++u) {
      const int e = t + u * kBlock, kk = e % KC, j = e / KC;
      const bool in = j0 + j < tk.n && k0 + kk < ke;
      bv[u] = *(in ? B + (size_t)(j0 + j) * tk.ldb + k0 + kk : Z);
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
  // each wave owns a 32 x 32 quarter of the tile, on the matrix cores
  const int lane = t & 63, wv = t >> 6, wm = (wv & 1) * 32, wn = (wv >> 1) * 32;
  MfmaAcc<T> acc;
  acc.zero();
  int buf = 0;
  if (kb < ke) {
    load(kb);
    store(0);
  }
  __syncthreads();
  for (int k0 = kb; k0 < ke; k0 += KC) {
    const bool more = k0 + KC < ke;
    if (more) load(k0 + KC);
    acc.template step<KC>(&As[buf][0][0], &Bs[buf][0][0], kTile + 1, wm, wn, lane);
    if (more) store(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }
  const T alpha = (T)tk.alpha;
  for (int q = 0; q < MfmaAcc<T>::kN; ++q) {
    int ii, jj;
    MfmaAcc<T>::coord(q, lane, ii, jj);
    const int i = i0 + wm + ii, j = j0 + wn + jj;
    if (i >= tk.m || j >= tk.n) continue;
    const GPW cp = C + i + (size_t)j * tk.ldc;
    T val = alpha * acc.get(q);
    if (tk.ksplit == 1) {
      if (tk.mode == kGemmAccumulate) val += *cp;
      else if (tk.mode == kGemmAddIdentity && i == j) val += T(1);
    }
    *cp = val;
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
    if (h->gemm_mode == kGemmRecord) h->gemm_replan = true;  // earlier records point into the old block
  }
  *out = static_cast<char*>(buf.p) + used;
  used += bytes;
  return HODLR_OK;
}

// Task tables are written to pinned host staging at the same offset as their
// device copy, so an asynchronous (or captured) copy reads memory that stays
// valid until the next factorization of the handle.  In record mode the copy
// is left to gemm_upload.
static int stage_tables(hodlr_s* h, const void* src, size_t bytes, void* dev, hipStream_t s) {
  const size_t off = static_cast<char*>(dev) - static_cast<char*>(h->gemm_tab.p);
  if (h->gemm_host_bytes < h->gemm_tab.bytes) {
    if (h->capturing) return fail(HODLR_EINVAL, "batched-product staging too small under graph capture");
    HODLR_HIP(hipStreamSynchronize(s));
    if (h->gemm_host) pinned_free(h->gemm_host, h->gemm_host_bytes);
    h->gemm_host = nullptr;
    h->gemm_host_bytes = 0;
    HODLR_TRY(pinned_alloc(h->gemm_tab.bytes, &h->gemm_host, &h->gemm_host_bytes));
    if (h->gemm_mode == kGemmRecord) h->gemm_replan = true;  // the tables staged so far are gone
  }
  char* hp = static_cast<char*>(h->gemm_host) + off;
  std::memcpy(hp, src, bytes);
  if (h->gemm_mode == kGemmRecord) {
    h->gemm_staged = std::max(h->gemm_staged, off + bytes);
    return HODLR_OK;
  }
  HODLR_HIP(hipMemcpyAsync(dev, hp, bytes, hipMemcpyHostToDevice, s));
  return HODLR_OK;
}

}  // namespace

int gemm_upload(hodlr_s* h, hipStream_t s) {
  if (h->gemm_staged > 0)
    HODLR_HIP(hipMemcpyAsync(h->gemm_tab.p, h->gemm_host, h->gemm_staged, hipMemcpyHostToDevice, s));
  h->gemm_staged = 0;
  return HODLR_OK;
}

template <typename T>
static int gemm_launch(const GemmRec& r, hipStream_t s) {
  k_gemm_batched<T><<<r.tiles, kBlock, 0, s>>>(reinterpret_cast<const TaskDev*>(r.tb), r.ntasks);
  HODLR_HIP(hipGetLastError());
  if (r.nred) {
    k_gemm_reduce<T><<<dim3(std::min(64, (r.maxmn + kBlock - 1) / kBlock), (unsigned)r.nred), kBlock, 0, s>>>(
        reinterpret_cast<const TaskDev*>(r.tb + r.o1), reinterpret_cast<const void* const*>(r.tb + r.o2));
    HODLR_HIP(hipGetLastError());
  }
  return HODLR_OK;
}

template <typename T>
int gemm_batched_t(hodlr_s* h, const std::vector<GemmTask>& in, hipStream_t s) {
  if (h->gemm_mode == kGemmReplay) {
    if (h->gemm_rec_pos >= h->gemm_recs.size()) return fail(HODLR_EINVAL, "batched product beyond the recorded sequence");
    return gemm_launch<T>(h->gemm_recs[h->gemm_rec_pos++], s);
  }
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
  // one block of the table arena: tasks, then the sums' tasks and their parts,
  // staged with one copy
  const size_t b0 = tasks.size() * sizeof(TaskDev), b1 = red.size() * sizeof(TaskDev);
  const size_t o1 = (b0 + 255) & ~(size_t)255, o2 = o1 + ((b1 + 255) & ~(size_t)255);
  const size_t nb = nsplit ? o2 + parts.size() * sizeof(void*) : b0;
  void* tab = nullptr;
  HODLR_TRY(arena_take(h, h->gemm_tab, h->gemm_tab_used, o2 + parts.size() * sizeof(void*), s, &tab));
  std::vector<char> blk(nb, 0);
  std::memcpy(blk.data(), tasks.data(), b0);
  if (nsplit) {
    std::memcpy(blk.data() + o1, red.data(), b1);
    std::memcpy(blk.data() + o2, parts.data(), parts.size() * sizeof(void*));
  }
  HODLR_TRY(stage_tables(h, blk.data(), nb, tab, s));
  GemmRec r;
  r.tb = static_cast<const char*>(tab);
  r.ntasks = (int)tasks.size();
  r.tiles = tiles;
  r.nred = (int)red.size();
  r.maxmn = maxmn;
  r.o1 = o1;
  r.o2 = o2;
  if (h->gemm_mode == kGemmRecord) {
    h->gemm_recs.push_back(r);
    return HODLR_OK;
  }
  return gemm_launch<T>(r, s);
}

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
    // a buffer being replaced may still be read by queued products (a
    // handle's first factorization has none to replace)
    if (h->gemm_tab.p || h->gemm_work.p || h->gemm_host) HODLR_HIP(hipStreamSynchronize(s));
    if (h->gemm_tab.bytes < tab_bytes) HODLR_TRY(h->gemm_tab.ensure(tab_bytes));
    if (h->gemm_work.bytes < work_bytes) HODLR_TRY(h->gemm_work.ensure(work_bytes));
    if (h->gemm_host_bytes < h->gemm_tab.bytes) {
      if (h->gemm_host) pinned_free(h->gemm_host, h->gemm_host_bytes);
      h->gemm_host = nullptr;
      h->gemm_host_bytes = 0;
      HODLR_TRY(pinned_alloc(h->gemm_tab.bytes, &h->gemm_host, &h->gemm_host_bytes));
    }
  }
  return HODLR_OK;
}

}  // namespace hodlr
