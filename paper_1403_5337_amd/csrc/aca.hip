// Partial-pivoting adaptive cross approximation of every off-diagonal block
// (Sec. 5.1), all levels in one launch.
//
// ACA is a chain of dependent pivot steps (a row residual, its largest entry,
// a column residual, its largest entry), so each block is worked on by a
// group of G workgroups that split its rows and columns into slices of at
// most SLICE entries.  Each workgroup keeps its slice of the growing U and V
// in LDS, so the residual rows/columns and the inner products of the norm
// estimate are LDS-bandwidth work; the pivot choices are exchanged through
// small per-workgroup records in global memory between two group barriers
// per step.  All workgroups of a group read the same records in the same
// order, so they take identical decisions.  The launch is cooperative (all
// workgroups resident), and every barrier wait is bounded: a timeout sets an
// abort flag that every workgroup checks, so the kernel always drains.
//
// Readings (same as the FP64 reference): first pivot row 0; column pivot =
// largest |residual| among unused columns, next row = largest |u| among
// unused rows, ties to the lowest index; a residual row with no nonzero
// unused entry moves to the lowest unused row; the cross is accepted, then
// the iteration stops when |u_k|^2 |v_k|^2 <= eps^2 |U V^T|_F^2, the norm
// being updated with the inner products of the new cross with the old ones.
#include <algorithm>
#include <climits>
#include <numeric>

#include "device_util.h"
#include "hodlr_internal.h"

namespace hodlr {

struct AcaTask {
  int node;          // node id of the block's row set
  int row0, m;       // block rows: global [row0, row0 + m)
  int col0, nc;      // block columns: global [col0, col0 + nc)
  int g0, G;         // first workgroup (global index) and group size
  int capcol, kmax;  // column of the capped panels, rank cap
};

constexpr int kMaxBlockDim = 8192;  // largest block side (n <= 16384)
constexpr unsigned kSpinLimit = 1u << 21;

// Device-scope (agent) atomic loads and stores: coherent across the XCDs
// without L2 write-back or invalidation.  The pivot records are only ever
// accessed through these.
__device__ __forceinline__ void st_agent(float* p, float v) {
  __hip_atomic_store(reinterpret_cast<unsigned*>(p), __float_as_uint(v), __ATOMIC_RELAXED,
                     __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_agent(double* p, double v) {
  __hip_atomic_store(reinterpret_cast<unsigned long long*>(p),
                     (unsigned long long)__double_as_longlong(v), __ATOMIC_RELAXED,
                     __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ float ld_agent(const float* p) {
  return __uint_as_float(__hip_atomic_load(reinterpret_cast<unsigned*>(const_cast<float*>(p)),
                                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
}
__device__ __forceinline__ double ld_agent(const double* p) {
  return __longlong_as_double((long long)__hip_atomic_load(
      reinterpret_cast<unsigned long long*>(const_cast<double*>(p)), __ATOMIC_RELAXED,
      __HIP_MEMORY_SCOPE_AGENT));
}

// Barrier of the G workgroups of one group.  Every record store is a
// device-scope atomic store; each thread waits for its own stores to
// complete (s_waitcnt), the workgroup meets, one thread bumps the group
// counter and spins on it, and the records are then read with device-scope
// atomic loads.  Returns false (uniformly) if the wait timed out or another
// workgroup aborted.
__device__ bool group_barrier(unsigned* bar, unsigned target, int* abort_flag, int* s_ok) {
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0) {
    __hip_atomic_fetch_add(bar, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    int ok = 1;
    unsigned spins = 0;
    while (__hip_atomic_load(bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
      if (__hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
        ok = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
      if (++spins > kSpinLimit) {
        __hip_atomic_store(abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        ok = 0;
        break;
      }
    }
    __builtin_amdgcn_s_waitcnt(0);
    *s_ok = ok;
  }
  __syncthreads();
  return *s_ok != 0;
}

__device__ __forceinline__ bool bit_get(const unsigned* b, int i) { return (b[i >> 5] >> (i & 31)) & 1u; }

template <typename T, int KCAP, int SLICE>
__global__ void __launch_bounds__(kBlock)
    k_aca(const double* __restrict__ K, int ldk, const AcaTask* __restrict__ tasks,
          const int* __restrict__ wg_task, int wg_base, T* __restrict__ Ucap, T* __restrict__ Vcap,
          int ldu, T* rec, int rec_stride, unsigned* bars,
          int* __restrict__ rank_out, int* __restrict__ status, T eps, int* __restrict__ piv_out_rec) {
  constexpr int LD = SLICE + 1;
  extern __shared__ __align__(16) unsigned char smem[];
  T* Us = reinterpret_cast<T*>(smem);           // KCAP x LD: U slice, column l at l*LD
  T* Vs = Us + KCAP * LD;                       // KCAP x LD: V slice
  T* rown = Vs + KCAP * LD;                     // SLICE: residual row on own columns
  T* urow = rown + SLICE;                       // KCAP: U(i*, :)
  T* vrow = urow + KCAP;                        // KCAP: V(j*, :)
  T* dsum = vrow + KCAP;                        // 2 KCAP + 2: inner products
  unsigned* rowused = reinterpret_cast<unsigned*>(dsum + 2 * KCAP + 2);
  unsigned* colused = rowused + kMaxBlockDim / 32;
  __shared__ T sv[kBlock / 64];
  __shared__ int si[kBlock / 64];
  __shared__ T s_bv, s_piv;
  __shared__ int s_j, s_i, s_done, s_k, s_ok;

  const int wg = wg_base + blockIdx.x;
  const AcaTask tk = tasks[wg_task[wg]];
  const int t = threadIdx.x, nt = blockDim.x;
  const int g = wg - tk.g0, G = tk.G;
  const int Sr = (tk.m + G - 1) / G, Sc = (tk.nc + G - 1) / G;
  const int rlo = g * Sr, rn = max(0, min(tk.m, rlo + Sr) - rlo);
  const int clo = g * Sc, cn = max(0, min(tk.nc, clo + Sc) - clo);
  unsigned* bar = bars + tk.g0;  // one counter per group
  int* abort_flag = status + 2;
  auto recp = [&](int slot, int gg) { return rec + ((size_t)(tk.g0 + gg) * 2 + slot) * rec_stride; };

  for (int w = t; w < kMaxBlockDim / 32; w += nt) {
    rowused[w] = 0u;
    colused[w] = 0u;
  }
  if (t == 0) {
    s_done = 0;
    s_k = 0;
    s_i = 0;
  }
  __syncthreads();
  int k = 0, istar = 0;
  unsigned nb = 0;   // group barriers passed
  T norm2 = T(0);    // thread 0 only
  bool aborted = false;

  while (true) {
    // ---------------- phase A: residual of row istar on own columns
    if (t == 0) rowused[istar >> 5] |= 1u << (istar & 31);
    T best = T(-1);
    int bj = INT_MAX;
    if (t < cn) {
      const int j = clo + t;
      T r = (T)K[(size_t)(tk.col0 + j) * ldk + tk.row0 + istar];
      for (int l = 0; l < k; ++l) r -= urow[l] * Vs[l * LD + t];
      rown[t] = r;
      if (!bit_get(colused, j)) argmax_merge(best, bj, dabs(r), j);
    }
    T bv;
    int bjj;
    block_argmax(best, bj, sv, si, bv, bjj);
    const bool have = (bjj != INT_MAX);
    if (G > 1) {
      T* R = recp(nb & 1, g);
      if (t == 0) {
        st_agent(R + 0, have ? bv : T(-1));
        st_agent(R + 1, have ? T(bjj) : T(-1));
        st_agent(R + 2, have ? rown[bjj - clo] : T(0));
      }
      for (int l = t; l < k; l += nt) st_agent(R + 3 + l, have ? Vs[l * LD + (bjj - clo)] : T(0));
      if (!group_barrier(bar, (unsigned)G * (nb + 1), abort_flag, &s_ok)) {
        aborted = true;
        break;
      }
      // one candidate record per workgroup, read in parallel after the fence
      T hv = T(-2);
      int hg = INT_MAX;
      if (t < G) {
        hv = ld_agent(recp(nb & 1, t));
        hg = t;
      }
      T wv;
      int win;
      block_argmax(hv, hg, sv, si, wv, win);
      const T* Rw = recp(nb & 1, win);
      if (t == 0) {
        s_bv = wv;
        s_j = (int)ld_agent(Rw + 1);
        s_piv = ld_agent(Rw + 2);
      }
      for (int l = t; l < k; l += nt) vrow[l] = ld_agent(Rw + 3 + l);
      ++nb;
    } else {
      if (t == 0) {
        s_bv = have ? bv : T(-1);
        s_j = have ? bjj : -1;
        s_piv = have ? rown[bjj - clo] : T(0);
      }
      for (int l = t; l < k; l += nt) vrow[l] = have ? Vs[l * LD + (bjj - clo)] : T(0);
    }
    __syncthreads();
    if (!(s_bv > T(0))) {
      // no nonzero residual on an unused column: next unused row, if any
      if (t == 0) {
        int nxt = -1;
        for (int w = 0; w < (tk.m + 31) / 32 && nxt < 0; ++w) {
          unsigned free_bits = ~rowused[w];
          if (w == (tk.m - 1) / 32 && (tk.m & 31)) free_bits &= (1u << (tk.m & 31)) - 1u;
          if (free_bits) nxt = w * 32 + __builtin_ctz(free_bits);
        }
        s_done = (nxt < 0);
        s_i = nxt;
      }
      __syncthreads();
      if (s_done) break;
      istar = s_i;
      __syncthreads();
      continue;
    }
    // ---------------- phase B: new cross
    const int jstar = s_j;
    const T piv = s_piv;
    if (t == 0) colused[jstar >> 5] |= 1u << (jstar & 31);
    if (piv_out_rec && g == 0 && t == 0) {  // pivot row and column of cross k
      piv_out_rec[(size_t)(tk.node - 1) * 2 * KCAP + k] = istar;
      piv_out_rec[(size_t)(tk.node - 1) * 2 * KCAP + KCAP + k] = jstar;
    }
    if (t < cn) {
      const T v = rown[t] / piv;
      Vs[k * LD + t] = v;
      Vcap[(size_t)(tk.capcol + k) * ldu + tk.col0 + clo + t] = v;
    }
    if (t < rn) {
      const int i = rlo + t;
      T u = (T)K[(size_t)(tk.col0 + jstar) * ldk + tk.row0 + i];
      for (int l = 0; l < k; ++l) u -= Us[l * LD + t] * vrow[l];
      Us[k * LD + t] = u;
      Ucap[(size_t)(tk.capcol + k) * ldu + tk.row0 + i] = u;
    }
    __syncthreads();
    for (int idx = t; idx < 2 * k + 2; idx += nt) {
      T s = T(0);
      if (idx < k) {
        for (int x = 0; x < rn; ++x) s += Us[k * LD + x] * Us[idx * LD + x];
      } else if (idx < 2 * k) {
        for (int x = 0; x < cn; ++x) s += Vs[k * LD + x] * Vs[(idx - k) * LD + x];
      } else if (idx == 2 * k) {
        for (int x = 0; x < rn; ++x) s += Us[k * LD + x] * Us[k * LD + x];
      } else {
        for (int x = 0; x < cn; ++x) s += Vs[k * LD + x] * Vs[k * LD + x];
      }
      dsum[idx] = s;
    }
    best = T(-1);
    int bi = INT_MAX;
    if (t < rn) {
      const int i = rlo + t;
      if (!bit_get(rowused, i)) argmax_merge(best, bi, dabs(Us[k * LD + t]), i);
    }
    T bu;
    int bii;
    block_argmax(best, bi, sv, si, bu, bii);  // (synchronizes dsum too)
    const bool haverow = (bii != INT_MAX);
    if (G > 1) {
      T* R = recp(nb & 1, g);
      if (t == 0) {
        st_agent(R + 0, haverow ? bu : T(-1));
        st_agent(R + 1, haverow ? T(bii) : T(-1));
      }
      for (int l = t; l <= k; l += nt) st_agent(R + 3 + l, haverow ? Us[l * LD + (bii - rlo)] : T(0));
      for (int idx = t; idx < 2 * k + 2; idx += nt) st_agent(R + 3 + KCAP + idx, dsum[idx]);
      if (!group_barrier(bar, (unsigned)G * (nb + 1), abort_flag, &s_ok)) {
        aborted = true;
        break;
      }
      for (int idx = t; idx < 2 * k + 2; idx += nt) {
        // issue up to 16 record loads before waiting on any of them
        T acc = T(0);
        for (int g0 = 0; g0 < G; g0 += 16) {
          T v[16];
#pragma unroll
          for (int u = 0; u < 16; ++u)
            v[u] = (g0 + u < G) ? ld_agent(recp(nb & 1, g0 + u) + 3 + KCAP + idx) : T(0);
#pragma unroll
          for (int u = 0; u < 16; ++u) acc += v[u];
        }
        dsum[idx] = acc;
      }
      T hv = T(-2);
      int hg = INT_MAX;
      if (t < G) {
        hv = ld_agent(recp(nb & 1, t));
        hg = t;
      }
      T wv;
      int win;
      block_argmax(hv, hg, sv, si, wv, win);
      const T* Rw = recp(nb & 1, win);
      if (t == 0) {
        s_bv = wv;
        s_i = (int)ld_agent(Rw + 1);
      }
      for (int l = t; l <= k; l += nt) urow[l] = ld_agent(Rw + 3 + l);
      ++nb;
    } else {
      if (t == 0) {
        s_bv = haverow ? bu : T(-1);
        s_i = haverow ? bii : -1;
      }
      for (int l = t; l <= k; l += nt) urow[l] = haverow ? Us[l * LD + (bii - rlo)] : T(0);
    }
    __syncthreads();
    if (t == 0) {
      T cross = T(0);
      for (int l = 0; l < k; ++l) cross += dsum[l] * dsum[k + l];
      const T uu = dsum[2 * k], vv = dsum[2 * k + 1];
      norm2 += T(2) * cross + uu * vv;
      const int k1 = k + 1;
      s_done = (uu * vv <= eps * eps * norm2) || (k1 >= tk.kmax) || !(s_bv >= T(0)) || s_i < 0;
      s_k = k1;
    }
    __syncthreads();
    k = s_k;
    if (s_done) break;
    istar = s_i;
    __syncthreads();
  }
  if (g == 0 && t == 0) rank_out[tk.node] = aborted ? 0 : k;
}

// Occupancy-limited cooperative launches over contiguous ranges of groups.
template <typename T, int KCAP, int SLICE>
static int aca_t(hodlr_s* h, const double* K, int ldk, T* Ucap, T* Vcap,
                 const std::vector<int>& capoff, const std::vector<int>& cap, hipStream_t s,
                 const std::vector<int>* nodes, int* piv) {
  const Tree& tr = h->tree;
  if (tr.n > 2 * kMaxBlockDim) return fail(HODLR_EINVAL, "ACA supports n <= 16384");
  // blocks, largest first
  std::vector<AcaTask> tasks;
  std::vector<char> want(tr.nnodes(), nodes ? 0 : 1);
  if (nodes)
    for (int c : *nodes) want[c] = 1;
  for (int q = 1; q <= tr.L; ++q)
    for (int i = 0; i < (1 << q); ++i) {
      const int c = node_id(q, i), sib = node_id(q, i ^ 1);
      if (!want[c]) continue;
      AcaTask tk{};
      tk.node = c;
      tk.row0 = tr.lo[c];
      tk.m = tr.size(c);
      tk.col0 = tr.lo[sib];
      tk.nc = tr.size(sib);
      tk.G = (std::max(tk.m, tk.nc) + SLICE - 1) / SLICE;
      tk.capcol = capoff[q - 1];
      tk.kmax = std::min(std::min(tk.m, tk.nc), std::min(cap[q - 1], KCAP));
      tasks.push_back(tk);
    }
  if (tasks.empty()) return HODLR_OK;
  int total = 0;
  for (auto& tk : tasks) {
    tk.g0 = total;
    total += tk.G;
  }
  std::vector<int> wg_task(total);
  for (size_t x = 0; x < tasks.size(); ++x)
    for (int g = 0; g < tasks[x].G; ++g) wg_task[tasks[x].g0 + g] = (int)x;

  const size_t lds = sizeof(T) * ((size_t)2 * KCAP * (SLICE + 1) + SLICE + 2 * KCAP + 2 * KCAP + 2) +
                     sizeof(unsigned) * 2 * (kMaxBlockDim / 32);
  auto kern = k_aca<T, KCAP, SLICE>;
  HODLR_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  int per_cu = 0, ncu = 0, dev = 0;
  HODLR_HIP(hipGetDevice(&dev));
  HODLR_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  HODLR_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(kern),
                                                         kBlock, lds));
  const int resident = per_cu * ncu;
  if (resident < 1) return fail(HODLR_EHIP, "ACA kernel cannot be resident");
  for (auto& tk : tasks)
    if (tk.G > resident) return fail(HODLR_EINVAL, "ACA block needs more workgroups than fit");

  const int rec_stride = 3 + KCAP + 2 * KCAP + 2;
  DevBuf d_tasks, d_wg;
  HODLR_TRY(d_tasks.ensure(tasks.size() * sizeof(AcaTask)));
  HODLR_TRY(d_wg.ensure(total * sizeof(int)));
  const size_t rec_bytes = ((size_t)total * 2 * rec_stride * sizeof(T) + 255) / 256 * 256;
  DevBuf d_rec;
  HODLR_TRY(d_rec.ensure(rec_bytes + total * sizeof(unsigned)));
  void* uc = d_rec.p;
  HODLR_HIP(hipMemcpyAsync(d_tasks.p, tasks.data(), tasks.size() * sizeof(AcaTask),
                           hipMemcpyHostToDevice, s));
  HODLR_HIP(hipMemcpyAsync(d_wg.p, wg_task.data(), total * sizeof(int), hipMemcpyHostToDevice, s));
  T* p_rec = static_cast<T*>(uc);
  unsigned* p_bars = reinterpret_cast<unsigned*>(static_cast<char*>(uc) + rec_bytes);
  HODLR_HIP(hipMemsetAsync(p_bars, 0, total * sizeof(unsigned), s));
  if (!nodes) HODLR_HIP(hipMemsetAsync(h->d_rank.p, 0, tr.nnodes() * sizeof(int), s));

  const AcaTask* p_tasks = d_tasks.as<AcaTask>();
  const int* p_wg = d_wg.as<int>();
  int* p_rank = h->d_rank.as<int>();
  int* p_status = h->status.as<int>();
  T teps = (T)h->tol;
  int ldu = tr.n;
  // contiguous ranges of whole groups that fit on the device at once
  {
  ProfScope prof("aca", s);
  size_t x = 0;
  while (x < tasks.size()) {
    int wg_base = tasks[x].g0, cnt = 0;
    while (x < tasks.size() && cnt + tasks[x].G <= resident) {
      cnt += tasks[x].G;
      ++x;
    }
    void* args[] = {(void*)&K,     (void*)&ldk,        (void*)&p_tasks, (void*)&p_wg,
                    (void*)&wg_base, (void*)&Ucap,     (void*)&Vcap,    (void*)&ldu,
                    (void*)&p_rec, (void*)&rec_stride, (void*)&p_bars,  (void*)&p_rank,
                    (void*)&p_status, (void*)&teps,    (void*)&piv};
    HODLR_HIP(hipLaunchCooperativeKernel(reinterpret_cast<const void*>(kern), dim3(cnt),
                                         dim3(kBlock), args, (unsigned)lds, s));
  }
  }
  // the scratch goes back to the allocator once s is past the kernels
  for (DevBuf* b : {&d_tasks, &d_wg, &d_rec}) b->release_after(s);
  return HODLR_OK;
}

int launch_aca(hodlr_s* h, const double* K, int ldk, void* Ucap, void* Vcap,
               const std::vector<int>& capoff, const std::vector<int>& cap, hipStream_t s,
               const std::vector<int>* nodes, int* piv) {
  if (h->precision == 64)
    return aca_t<double, kRankCap64, kAcaSlice64>(h, K, ldk, static_cast<double*>(Ucap),
                                                  static_cast<double*>(Vcap), capoff, cap, s, nodes, piv);
  return aca_t<float, kRankCap32, kAcaSlice32>(h, K, ldk, static_cast<float*>(Ucap),
                                               static_cast<float*>(Vcap), capoff, cap, s, nodes, piv);
}

}  // namespace hodlr
