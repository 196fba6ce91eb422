// Dof ordering for the HODLR index halving, and relabelling of a front.
//
// The HODLR tree halves index ranges (Sec. 4.1), so neighbouring dofs must be
// close in the order; the paper takes the order from SCOTCH (Sec. 6).  Here a
// recursive coordinate bisection follows the tree itself: for every node,
// from the root down, its dofs are sorted by the coordinate of largest
// extent (first axis on ties; equal keys keep their current order) and the
// left child takes the first floor(len/2).  One workgroup sorts one node with
// a bitonic sort of (key, position) pairs, which is stable by construction
// because positions break ties; the pairs stay in registers except for the
// strides that cross waves.
#include <algorithm>
#include <cfloat>
#include <climits>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "device_util.h"
#include "hodlr_internal.h"

namespace hodlr {

constexpr int kRcbMax = 16384;
constexpr int kRcbThreads = 1024;

// (k, p) becomes the smaller (take_min) or the larger of itself and (ko, po)
// in the order "key, then position".
__device__ __forceinline__ void rcb_pick(float& k, int& p, float ko, int po, bool take_min) {
  const bool o_less = (ko < k) | ((ko == k) & (po < p));
  const bool take = take_min ? o_less : !o_less;
  k = take ? ko : k;
  p = take ? po : p;
}

// Bitonic sort of P (a power of two, <= 1024 E) (key, position) pairs held
// E per thread: element e = t E + r.  Strides below E stay in registers,
// strides below 64 E pair lanes of one wave, larger strides go through LDS.
template <int E>
__device__ void rcb_sort(float (&key)[E], int (&pos)[E], int P, float* skey, int* spos) {
  const int t = threadIdx.x;
  const bool live = t * E < P;
  for (int k = 2; k <= P; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      if (j < E) {
#pragma unroll
        for (int jj = E / 2; jj >= 1; jj >>= 1) {
          if (jj != j) continue;
#pragma unroll
          for (int r = 0; r < E; ++r) {
            const int rr = r ^ jj;
            if (rr < r) continue;
            const bool up = (((t * E + r) & k) == 0);
            const float ka = key[r], kb = key[rr];
            const int pa = pos[r], pb = pos[rr];
            const bool a_gt_b = (ka > kb) | ((ka == kb) & (pa > pb));
            if (a_gt_b == up) {
              key[r] = kb;
              key[rr] = ka;
              pos[r] = pb;
              pos[rr] = pa;
            }
          }
        }
      } else if (j < 64 * E) {
        const int m = j / E;  // partner lane: t ^ m
        const bool lower = (t & m) == 0;
#pragma unroll
        for (int r = 0; r < E; ++r) {
          const float ko = __shfl_xor(key[r], m, 64);
          const int po = __shfl_xor(pos[r], m, 64);
          const bool up = (((t * E + r) & k) == 0);
          rcb_pick(key[r], pos[r], ko, po, lower == up);
        }
      } else {
        if (live)
#pragma unroll
          for (int r = 0; r < E; ++r) {
            skey[t * E + r] = key[r];
            spos[t * E + r] = pos[r];
          }
        __syncthreads();
        if (live)
#pragma unroll
          for (int r = 0; r < E; ++r) {
            const int e = t * E + r, x = e ^ j;
            const bool up = ((e & k) == 0);
            rcb_pick(key[r], pos[r], skey[x], spos[x], ((e & j) == 0) == up);
          }
        __syncthreads();
      }
    }
  }
}

template <int E>
__device__ void rcb_node(const float* __restrict__ coords, int* __restrict__ perm, int l0, int len, int P,
                         int ax, float* skey, int* spos) {
  const int t = threadIdx.x;
  float key[E];
  int pos[E];
  // every load issued unconditionally (addresses clamped into the node), the
  // vertex ids first, then their coordinates, so each batch is one round trip
  int v[E];
#pragma unroll
  for (int r = 0; r < E; ++r) v[r] = perm[l0 + min(t * E + r, len - 1)];
#pragma unroll
  for (int r = 0; r < E; ++r) key[r] = coords[3 * (size_t)v[r] + ax];
#pragma unroll
  for (int r = 0; r < E; ++r) {
    const int e = t * E + r;
    pos[r] = e < len ? e : INT_MAX;
    key[r] = e < len ? key[r] : INFINITY;
  }
  rcb_sort<E>(key, pos, P, skey, spos);
  // perm(l0 + e) <- perm(l0 + pos(e)); the old entries go through LDS
  int* old = spos;
#pragma unroll
  for (int r = 0; r < E; ++r) v[r] = perm[l0 + min(t + r * (int)blockDim.x, len - 1)];
#pragma unroll
  for (int r = 0; r < E; ++r) {
    const int e = t + r * (int)blockDim.x;
    if (e < len) old[e] = v[r];
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < E; ++r) {
    const int e = t * E + r;
    if (e < len && pos[r] < len) perm[l0 + e] = old[pos[r]];
  }
}

__global__ void __launch_bounds__(kRcbThreads)
    k_rcb_level(const float* __restrict__ coords, int* __restrict__ perm, const int* __restrict__ lo,
                const int* __restrict__ hi, int id0) {
  __shared__ float skey[kRcbMax];
  __shared__ int spos[kRcbMax];
  __shared__ float red[6][kRcbThreads / 64];
  __shared__ int s_axis;
  const int node = blockIdx.x, id = id0 + node, t = threadIdx.x, nt = blockDim.x;
  const int l0 = lo[id], len = hi[id] - l0;
  if (len <= 1) return;
  int P = 1;
  while (P < len) P <<= 1;
  float mn[3] = {FLT_MAX, FLT_MAX, FLT_MAX}, mx[3] = {-FLT_MAX, -FLT_MAX, -FLT_MAX};
  // batches of 8 entries per thread: the vertex ids, then their coordinates,
  // each batch of loads in flight together (addresses clamped into the node)
  constexpr int kB = 8;
  for (int e0 = 0; e0 < len; e0 += kB * nt) {
    int v[kB];
#pragma unroll
    for (int u = 0; u < kB; ++u) v[u] = perm[l0 + min(e0 + t + u * nt, len - 1)];
    float c[kB][3];
#pragma unroll
    for (int u = 0; u < kB; ++u)
#pragma unroll
      for (int a = 0; a < 3; ++a) c[u][a] = coords[3 * (size_t)v[u] + a];
#pragma unroll
    for (int u = 0; u < kB; ++u)
      if (e0 + t + u * nt < len)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          mn[a] = fminf(mn[a], c[u][a]);
          mx[a] = fmaxf(mx[a], c[u][a]);
        }
  }
#pragma unroll
  for (int a = 0; a < 3; ++a)
    for (int o = 32; o > 0; o >>= 1) {
      mn[a] = fminf(mn[a], __shfl_xor(mn[a], o, 64));
      mx[a] = fmaxf(mx[a], __shfl_xor(mx[a], o, 64));
    }
  const int w = t >> 6, nw = nt >> 6;
  if ((t & 63) == 0)
    for (int a = 0; a < 3; ++a) {
      red[a][w] = mn[a];
      red[3 + a][w] = mx[a];
    }
  __syncthreads();
  if (t == 0) {
    float ext[3];
    for (int a = 0; a < 3; ++a) {
      float lo_a = red[a][0], hi_a = red[3 + a][0];
      for (int k = 1; k < nw; ++k) {
        lo_a = fminf(lo_a, red[a][k]);
        hi_a = fmaxf(hi_a, red[3 + a][k]);
      }
      ext[a] = hi_a - lo_a;
    }
    int ax = 0;
    if (ext[1] > ext[ax]) ax = 1;
    if (ext[2] > ext[ax]) ax = 2;
    s_axis = ax;
  }
  __syncthreads();
  const int ax = s_axis;
  if (P <= kRcbThreads) rcb_node<1>(coords, perm, l0, len, P, ax, skey, spos);
  else if (P <= 2 * kRcbThreads) rcb_node<2>(coords, perm, l0, len, P, ax, skey, spos);
  else if (P <= 4 * kRcbThreads) rcb_node<4>(coords, perm, l0, len, P, ax, skey, spos);
  else if (P <= 8 * kRcbThreads) rcb_node<8>(coords, perm, l0, len, P, ax, skey, spos);
  else rcb_node<16>(coords, perm, l0, len, P, ax, skey, spos);
}

__global__ void k_iota(int* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = i;
}

// Node ranges of the tree of (n, leaf) on the current device, uploaded once
// and kept for the process (a few KB each), so the ordering never waits for
// the stream to drain before releasing them.
int device_tree_ranges(const Tree& t, const int** lo, const int** hi) {
  static std::mutex mu;
  static std::map<std::tuple<int, int, int>, std::pair<int*, int*>> cache;
  int dev = 0;
  HODLR_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(mu);
  auto key = std::make_tuple(dev, t.n, t.leaf);
  auto it = cache.find(key);
  if (it == cache.end()) {
    const size_t nn = t.nnodes();
    int* d = nullptr;
    HODLR_HIP(hipMalloc(&d, 2 * nn * sizeof(int)));
    std::vector<int> h(2 * nn);
    std::copy(t.lo.begin(), t.lo.end(), h.begin());
    std::copy(t.hi.begin(), t.hi.end(), h.begin() + nn);
    const hipError_t e = hipMemcpy(d, h.data(), 2 * nn * sizeof(int), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      (void)hipFree(d);
      return fail(HODLR_EHIP, std::string("hipMemcpy: ") + hipGetErrorString(e));
    }
    it = cache.emplace(key, std::make_pair(d, d + nn)).first;
  }
  *lo = it->second.first;
  *hi = it->second.second;
  return HODLR_OK;
}

int launch_rcb(const float* coords, int n, const Tree& t, int* perm, hipStream_t s) {
  k_iota<<<(n + kBlock - 1) / kBlock, kBlock, 0, s>>>(perm, n);
  HODLR_HIP(hipGetLastError());
  if (t.L == 0) return HODLR_OK;
  const int *dlo = nullptr, *dhi = nullptr;
  HODLR_TRY(device_tree_ranges(t, &dlo, &dhi));
  for (int p = 0; p < t.L; ++p) {
    k_rcb_level<<<1 << p, kRcbThreads, 0, s>>>(coords, perm, dlo, dhi, node_id(p, 0));
    HODLR_HIP(hipGetLastError());
  }
  return HODLR_OK;
}

// ---------------------------------------------------------------------------
__global__ void k_permute(const double* __restrict__ Kin, int n, int ldi, const int* __restrict__ perm,
                          double* __restrict__ Kout, int ldo) {
  const int j = blockIdx.y;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int pj = perm[j];
  Kout[(size_t)j * ldo + i] = Kin[(size_t)pj * ldi + perm[i]];
}

// Column j of the output through LDS: input column perm[j] arrives with
// contiguous asynchronous copies, rows are gathered inside LDS, and the
// output column is written contiguously (n <= kPermLds).
constexpr int kPermLds = 16384;

__global__ void __launch_bounds__(kBlock)
    k_permute_lds(const double* __restrict__ Kin, int n, int ldi, const int* __restrict__ perm,
                  double* __restrict__ Kout, int ldo) {
  extern __shared__ __align__(16) unsigned char smem[];
  double* col = reinterpret_cast<double*>(smem);
  const int j = blockIdx.x, t = threadIdx.x, w = t >> 6, nw = blockDim.x >> 6;
  const double* src = Kin + (size_t)perm[j] * ldi;
  const int part = (n + nw - 1) / nw;
  const int c0 = min(n, w * part), c1 = min(n, c0 + part);
  dma_span(col + c0, src + c0, c1 - c0);
  dma_wait();
  double* dst = Kout + (size_t)j * ldo;
  for (int i0 = 0; i0 < n; i0 += 4 * kBlock) {
    int p[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int i = i0 + t + u * kBlock;
      p[u] = i < n ? perm[i] : 0;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int i = i0 + t + u * kBlock;
      if (i < n) dst[i] = col[p[u]];
    }
  }
}

int launch_permute(const double* Kin, int n, int ldi, const int* perm, double* Kout, int ldo,
                   hipStream_t s) {
  if (n <= kPermLds) {
    const size_t lds = (size_t)n * sizeof(double);
    if (lds > 64 * 1024)
      HODLR_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(k_permute_lds),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    k_permute_lds<<<n, kBlock, lds, s>>>(Kin, n, ldi, perm, Kout, ldo);
  } else {
    k_permute<<<dim3((n + kBlock - 1) / kBlock, n), kBlock, 0, s>>>(Kin, n, ldi, perm, Kout, ldo);
  }
  HODLR_HIP(hipGetLastError());
  return HODLR_OK;
}

// ---------------------------------------------------------------------------
// Graph relabelling: new vertex i = old vertex perm[i].
__global__ void k_inverse_perm(const int* __restrict__ perm, int* __restrict__ inv, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) inv[perm[i]] = i;
}

__global__ void k_new_degree(const int* __restrict__ rowptr, const int* __restrict__ perm,
                             int* __restrict__ deg, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) deg[i] = rowptr[perm[i] + 1] - rowptr[perm[i]];
}

// Exclusive scan of deg into rowptr_out[0..n] by one workgroup: thread t sums
// its contiguous chunk, the 256 chunk sums are scanned in LDS, and each
// thread writes its chunk's running sums.
__global__ void __launch_bounds__(kBlock) k_scan(const int* __restrict__ deg, int* __restrict__ out, int n) {
  __shared__ int part[kBlock];
  const int t = threadIdx.x;
  const int per = (n + kBlock - 1) / kBlock;
  const int b = min(n, t * per), e = min(n, b + per);
  int sum = 0;
#pragma unroll 8
  for (int i = b; i < e; ++i) sum += deg[i];
  part[t] = sum;
  __syncthreads();
  for (int o = 1; o < kBlock; o <<= 1) {
    const int add = t >= o ? part[t - o] : 0;
    __syncthreads();
    part[t] += add;
    __syncthreads();
  }
  int run = t > 0 ? part[t - 1] : 0;
  for (int i = b; i < e; ++i) {
    out[i] = run;
    run += deg[i];
  }
  if (t == kBlock - 1) out[n] = part[kBlock - 1];
}

// One wave per new row i: the row's new column ids, each placed at its rank
// (the entries below it, equal entries by their old order), so the row is
// sorted ascending.  The entries are taken 64 at a time, one per lane; a
// rank counts over all chunks of the row.
__global__ void __launch_bounds__(kBlock)
    k_fill_sorted(const int* __restrict__ rowptr, const int* __restrict__ col, const int* __restrict__ perm,
                  const int* __restrict__ inv, const int* __restrict__ rowptr_out, int* __restrict__ col_out,
                  int n) {
  const int lane = threadIdx.x & 63;
  const int i = __builtin_amdgcn_readfirstlane(blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6));
  if (i >= n) return;
  const int src = perm[i], b = rowptr[src], deg = rowptr[src + 1] - b, o = rowptr_out[i];
  for (int cx = 0; cx < deg; cx += 64) {
    const int x = cx + lane;
    const int v = x < deg ? inv[col[b + x]] : INT_MAX;
    int rank = 0;
    for (int cy = 0; cy < deg; cy += 64) {
      const int y = cy + lane;
      const int u = cy == cx ? v : (y < deg ? inv[col[b + y]] : INT_MAX);
      const int ny = min(64, deg - cy);
      for (int j = 0; j < ny; ++j) {
        const int uj = __builtin_amdgcn_readlane(u, j);
        rank += (uj < v || (uj == v && cy + j < x)) ? 1 : 0;
      }
    }
    if (x < deg) col_out[o + rank] = v;
  }
}

int launch_permute_graph(const int* rowptr, const int* col, int n, const int* perm,
                         int* rowptr_out, int* col_out, hipStream_t s) {
  // the two scratch arrays are allocated and freed in stream order, so the
  // call returns without waiting for its kernels
  int* scratch = nullptr;
  HODLR_HIP(hipMallocAsync(reinterpret_cast<void**>(&scratch), 2 * (size_t)n * sizeof(int), s));
  int* inv = scratch;
  int* deg = scratch + n;
  const int g = (n + kBlock - 1) / kBlock;
  k_inverse_perm<<<g, kBlock, 0, s>>>(perm, inv, n);
  k_new_degree<<<g, kBlock, 0, s>>>(rowptr, perm, deg, n);
  k_scan<<<1, kBlock, 0, s>>>(deg, rowptr_out, n);
  k_fill_sorted<<<(n + kBlock / 64 - 1) / (kBlock / 64), kBlock, 0, s>>>(rowptr, col, perm, inv, rowptr_out,
                                                                        col_out, n);
  const hipError_t le = hipGetLastError();
  HODLR_HIP(hipFreeAsync(scratch, s));
  if (le != hipSuccess) return fail(HODLR_EHIP, std::string("graph permutation launch: ") + hipGetErrorString(le));
  return HODLR_OK;
}

// ---------------------------------------------------------------------------
// out(i, :) = in(perm[i], :) for row-major n x width float arrays (dof
// coordinates follow the dofs into the new order).
__global__ void k_permute_rows(const float* __restrict__ in, int n, int width, const int* __restrict__ perm,
                               float* __restrict__ out) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)n * width) return;
  const int i = (int)(e / width), c = (int)(e % width);
  out[e] = in[(size_t)perm[i] * width + c];
}

int launch_permute_rows(const float* in, int n, int width, const int* perm, float* out, hipStream_t s) {
  const long total = (long)n * width;
  k_permute_rows<<<(int)((total + kBlock - 1) / kBlock), kBlock, 0, s>>>(in, n, width, perm, out);
  HODLR_HIP(hipGetLastError());
  return HODLR_OK;
}

}  // namespace hodlr
