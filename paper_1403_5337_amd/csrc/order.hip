// Dof ordering for the HODLR index halving, and relabelling of a front.
//
// The HODLR tree halves index ranges (Sec. 4.1), so neighbouring dofs must be
// close in the order; the paper takes the order from SCOTCH (Sec. 6).  Here a
// recursive coordinate bisection follows the tree itself: for every node,
// from the root down, its dofs are sorted by the coordinate of largest
// extent (first axis on ties; equal keys keep their current order) and the
// left child takes the first floor(len/2).  One workgroup sorts one node with
// a stable LSD radix sort (four 8-bit passes) of monotone integer keys made
// from the coordinates, through LDS.
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

// Sort key of a coordinate: the float's bits made monotone as an unsigned
// integer (negative values bit-inverted, the sign bit set on the others), with
// -0 taken as +0 and every NaN as one value above +inf, so that integer order
// is the order of the values and equal values (and all NaNs, last) keep their
// positions, as a stable sort by value does.
__device__ __forceinline__ unsigned rcb_key(float x) {
  unsigned u = __float_as_uint(x);
  if (u == 0x80000000u) u = 0u;
  if ((u & 0x7fffffffu) > 0x7f800000u) return 0xfffffffeu;
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

// Stable LSD radix sort (four passes of 8-bit digits) of the node's keys,
// followed by perm(l0 + e) <- perm(l0 + position of the e-th smallest).
// Positions are laid out wave-major: wave w holds positions w 64 E + 64 r +
// lane (r < E), so a wave's elements are contiguous and each of its E rows
// is in lane order.  Padding positions (>= len) take the key 0xffffffff and
// stay behind every real key.  A pass: each wave ranks its elements by digit
// row by row (lanes of equal digit found by eight ballots; the wave's running
// count per digit in LDS), one scan over (digit, wave) gives every group its
// first destination, and the elements are scattered through LDS.
template <int E>
__device__ void rcb_radix_node(const float* __restrict__ coords, int* __restrict__ perm, int l0, int len, int ax,
                               unsigned* sk, int* sv, int* cnt, int* wsum) {
  constexpr int kW = kRcbThreads / 64;  // waves
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const unsigned long long below = (1ull << lane) - 1ull;
  unsigned key[E];
  int val[E];
  {
    int v[E];
#pragma unroll
    for (int r = 0; r < E; ++r) v[r] = perm[l0 + min(w * 64 * E + 64 * r + lane, len - 1)];
#pragma unroll
    for (int r = 0; r < E; ++r) {
      const int e = w * 64 * E + 64 * r + lane;
      const float c = coords[3 * (size_t)v[r] + ax];
      key[r] = e < len ? rcb_key(c) : 0xffffffffu;
      val[r] = e;
    }
  }
  for (int shift = 0; shift < 32; shift += 8) {
    int* wc = cnt + w * 256;  // this wave's running counts per digit
#pragma unroll
    for (int q = 0; q < 4; ++q) wc[lane + 64 * q] = 0;
    int dst[E];
#pragma unroll
    for (int r = 0; r < E; ++r) {
      const unsigned d = (key[r] >> shift) & 255u;
      unsigned long long m = ~0ull;
#pragma unroll
      for (int bit = 0; bit < 8; ++bit) {
        const unsigned long long bal = __ballot((d >> bit) & 1u);
        m &= ((d >> bit) & 1u) ? bal : ~bal;
      }
      const int base = wc[d];
      const int lead = __ffsll((long long)m) - 1;
      if (lane == lead) wc[d] = base + __popcll(m);
      dst[r] = base + __popcll(m & below);  // rank among this wave's equal digits so far
    }
    __syncthreads();
    // exclusive prefix over (digit, wave) in digit-major order: thread t takes
    // entries 4 t .. 4 t + 3 (digit t / 4, waves 4 (t % 4) .. + 3)
    {
      const int d = t >> 2, w0 = (t & 3) * 4;
      int c[4], tot = 0;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        c[q] = cnt[(w0 + q) * 256 + d];
        tot += c[q];
      }
      int inc = tot;  // inclusive scan of the thread totals within the wave
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(inc, o, 64);
        if (lane >= o) inc += y;
      }
      if (lane == 63) wsum[w] = inc;
      __syncthreads();
      int before = 0;
#pragma unroll
      for (int k = 0; k < kW; ++k) before += k < w ? wsum[k] : 0;
      int run = before + inc - tot;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        cnt[(w0 + q) * 256 + d] = run;
        run += c[q];
      }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < E; ++r) {
      const int o = cnt[w * 256 + ((key[r] >> shift) & 255u)] + dst[r];
      sk[o] = key[r];
      sv[o] = val[r];
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < E; ++r) {
      const int e = w * 64 * E + 64 * r + lane;
      key[r] = sk[e];
      val[r] = sv[e];
    }
    __syncthreads();
  }
  // perm(l0 + e) <- perm(l0 + val(e)); the old entries go through LDS
  int* old = sv;
  {
    int v[E];
#pragma unroll
    for (int r = 0; r < E; ++r) v[r] = perm[l0 + min(t + r * kRcbThreads, len - 1)];
#pragma unroll
    for (int r = 0; r < E; ++r)
      if (t + r * kRcbThreads < len) old[t + r * kRcbThreads] = v[r];
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < E; ++r) {
    const int e = w * 64 * E + 64 * r + lane;
    if (e < len) perm[l0 + e] = old[val[r]];
  }
}

__global__ void __launch_bounds__(kRcbThreads)
    k_rcb_level(const float* __restrict__ coords, int* __restrict__ perm, const int* __restrict__ lo,
                const int* __restrict__ hi, int id0) {
  __shared__ unsigned skey[kRcbMax];
  __shared__ int spos[kRcbMax];
  __shared__ int scnt[kRcbThreads / 64 * 256];
  __shared__ int swsum[kRcbThreads / 64];
  __shared__ float red[6][kRcbThreads / 64];
  __shared__ int s_axis;
  const int node = blockIdx.x, id = id0 + node, t = threadIdx.x, nt = blockDim.x;
  const int l0 = lo[id], len = hi[id] - l0;
  if (len <= 1) return;
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
  if (len <= kRcbThreads) rcb_radix_node<1>(coords, perm, l0, len, ax, skey, spos, scnt, swsum);
  else if (len <= 2 * kRcbThreads) rcb_radix_node<2>(coords, perm, l0, len, ax, skey, spos, scnt, swsum);
  else if (len <= 4 * kRcbThreads) rcb_radix_node<4>(coords, perm, l0, len, ax, skey, spos, scnt, swsum);
  else if (len <= 8 * kRcbThreads) rcb_radix_node<8>(coords, perm, l0, len, ax, skey, spos, scnt, swsum);
  else rcb_radix_node<16>(coords, perm, l0, len, ax, skey, spos, scnt, swsum);
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
