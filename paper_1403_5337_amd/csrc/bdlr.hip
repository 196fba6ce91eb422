// Boundary-distance low-rank approximation, BDLR (Sec. 5.3, eq. Ahat), of
// every off-diagonal block, all levels at once.
//
// For block K(I, J) (I = the node's rows, J = its sibling's, both contiguous
// index ranges after the ordering) three launches, one workgroup per block:
//   select  boundary sets (vertices with an edge into the other set), a
//           level-synchronous breadth-first search inside each set up to
//           depth-1, and the picked rows/columns: distance < depth, nearest
//           the boundary first and at most max_skel of them, listed in
//           increasing position;
//   lu      Ahat = K(rows, cols) gathered into LDS, LU with full pivoting
//           (largest |entry| of the remaining Schur complement, ties to the
//           lowest row-major position), kept while |pivot| >= eps |first
//           pivot| (Sec. 7.1), giving rank r; then the r x r leading factors
//           are inverted in place (U11^-1 and L11^-1);
//   factors C~ = K(I, pivot columns) U11^-1 and R~^T = K(pivot rows, J)^T
//           L11^-T as gathered panels times the small inverses, written as
//           U = C~ and V = R~^T into the capped panels.
#include <algorithm>
#include <climits>
#include <cstdint>

#include "device_util.h"
#include "hodlr_internal.h"

namespace hodlr {

constexpr int kBdlrMaxSide = 8192;  // largest block side (n <= 16384)
constexpr int kSkel32 = 192;        // max picked rows (columns): Ahat fits in LDS
constexpr int kSkel64 = 128;

struct BdlrTask {
  int node, row0, m, col0, nc;
  int capcol, kmax;
  int sel_off;   // ints: rows at sel_off, columns at sel_off + max_skel
  size_t inv_off;  // elements: U11^-1 then L11^-T, max_skel^2 each
  size_t cg_off;   // elements: C panel (m x kmax) then R^T panel (nc x kmax)
};

// exclusive prefix over the 256 per-thread values v; returns this thread's
// offset and, in *total, the sum
__device__ int block_exclusive_scan(int v, int* buf, int* total) {
  const int t = threadIdx.x;
  buf[t] = v;
  __syncthreads();
  for (int o = 1; o < kBlock; o <<= 1) {
    const int add = t >= o ? buf[t - o] : 0;
    __syncthreads();
    buf[t] += add;
    __syncthreads();
  }
  const int incl = buf[t];
  *total = buf[kBlock - 1];
  __syncthreads();
  return incl - v;
}

// Picks (in increasing position) of one side from its distances d[0..len).
__device__ void pick_side(const uint8_t* d, int len, int depth, int max_skel, int* out, int* count,
                          int* cnt, int* buf, int* s_cut) {
  const int t = threadIdx.x;
  for (int l = t; l < 256; l += kBlock) cnt[l] = 0;
  __syncthreads();
  for (int i = t; i < len; i += kBlock)
    if (d[i] < depth) atomicAdd(&cnt[d[i]], 1);
  __syncthreads();
  if (t == 0) {
    int cum = 0, dcut = depth, take = 0;
    for (int l = 0; l < depth; ++l) {
      if (cum + cnt[l] > max_skel) {
        dcut = l;
        take = max_skel - cum;
        break;
      }
      cum += cnt[l];
    }
    s_cut[0] = dcut;
    s_cut[1] = take;
  }
  __syncthreads();
  const int dcut = s_cut[0], take = s_cut[1];
  const int seg = (len + kBlock - 1) / kBlock, b0 = min(len, t * seg), b1 = min(len, b0 + seg);
  int tot;
  // rank of each d == dcut entry among those, in position order
  int ne = 0;
  for (int i = b0; i < b1; ++i) ne += (d[i] == dcut);
  int eq = block_exclusive_scan(ne, buf, &tot);
  int ns = 0;
  for (int i = b0, e = eq; i < b1; ++i) {
    const bool ise = d[i] == dcut;
    ns += (d[i] < dcut) || (ise && e < take);
    e += ise;
  }
  int pos = block_exclusive_scan(ns, buf, &tot);
  for (int i = b0, e = eq; i < b1; ++i) {
    const bool ise = d[i] == dcut;
    if ((d[i] < dcut) || (ise && e < take)) out[pos++] = i;
    e += ise;
  }
  if (t == 0) *count = tot;
  __syncthreads();
}

__global__ void __launch_bounds__(kBlock)
    k_bdlr_select(const int* __restrict__ rowptr, const int* __restrict__ col,
                  const BdlrTask* __restrict__ tasks, int depth, int max_skel, int* __restrict__ sel,
                  int* __restrict__ counts) {
  __shared__ uint8_t dI[kBdlrMaxSide], dJ[kBdlrMaxSide];
  __shared__ int cnt[256], buf[kBlock], s_cut[2];
  const BdlrTask tk = tasks[blockIdx.x];
  const int t = threadIdx.x;
  const int r0 = tk.row0, r1 = tk.row0 + tk.m, c0 = tk.col0, c1 = tk.col0 + tk.nc;
  // boundary sets: an edge into the other set
  for (int i = t; i < tk.m; i += kBlock) {
    const int v = r0 + i;
    uint8_t dv = 255;
    for (int e = rowptr[v]; e < rowptr[v + 1]; ++e) {
      const int u = col[e];
      if (u >= c0 && u < c1) {
        dv = 0;
        break;
      }
    }
    dI[i] = dv;
  }
  for (int j = t; j < tk.nc; j += kBlock) {
    const int v = c0 + j;
    uint8_t dv = 255;
    for (int e = rowptr[v]; e < rowptr[v + 1]; ++e) {
      const int u = col[e];
      if (u >= r0 && u < r1) {
        dv = 0;
        break;
      }
    }
    dJ[j] = dv;
  }
  __syncthreads();
  // breadth-first layers inside each set
  for (int lvl = 0; lvl + 1 < depth; ++lvl) {
    for (int i = t; i < tk.m; i += kBlock) {
      if (dI[i] != 255) continue;
      const int v = r0 + i;
      for (int e = rowptr[v]; e < rowptr[v + 1]; ++e) {
        const int u = col[e];
        if (u >= r0 && u < r1 && dI[u - r0] == lvl) {
          dI[i] = (uint8_t)(lvl + 1);
          break;
        }
      }
    }
    for (int j = t; j < tk.nc; j += kBlock) {
      if (dJ[j] != 255) continue;
      const int v = c0 + j;
      for (int e = rowptr[v]; e < rowptr[v + 1]; ++e) {
        const int u = col[e];
        if (u >= c0 && u < c1 && dJ[u - c0] == lvl) {
          dJ[j] = (uint8_t)(lvl + 1);
          break;
        }
      }
    }
    __syncthreads();
  }
  pick_side(dI, tk.m, depth, max_skel, sel + tk.sel_off, counts + 2 * blockIdx.x, cnt, buf, s_cut);
  pick_side(dJ, tk.nc, depth, max_skel, sel + tk.sel_off + max_skel, counts + 2 * blockIdx.x + 1, cnt,
            buf, s_cut);
}

template <typename T, int SKEL>
__global__ void __launch_bounds__(kBlock)
    k_bdlr_lu(const double* __restrict__ K, int ldk, const BdlrTask* __restrict__ tasks,
              const int* __restrict__ sel, const int* __restrict__ counts, T eps,
              int* __restrict__ piv_out, T* __restrict__ inv, int* __restrict__ rank_out,
              int* __restrict__ rank_task) {
  extern __shared__ __align__(16) unsigned char smem[];
  T* A = reinterpret_cast<T*>(smem);
  __shared__ int prow[SKEL], pcol[SKEL];
  __shared__ T tmp[SKEL];
  __shared__ T sv[kBlock / 64];
  __shared__ int si[kBlock / 64];
  __shared__ int s_r;
  const int task = blockIdx.x, t = threadIdx.x;
  const BdlrTask tk = tasks[task];
  const int nr = counts[2 * task], nc = counts[2 * task + 1], ld = nr + 1;
  const int* rows = sel + tk.sel_off;
  const int* cols = sel + tk.sel_off + SKEL;
  for (int e0 = 0; e0 < nr * nc; e0 += 8 * kBlock) {
    T v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = e0 + t + u * kBlock, i = e % max(nr, 1), j = e / max(nr, 1);
      v[u] = e < nr * nc ? (T)K[(size_t)(tk.col0 + cols[j]) * ldk + tk.row0 + rows[i]] : T(0);
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = e0 + t + u * kBlock;
      if (e < nr * nc) A[e % nr + (e / nr) * ld] = v[u];
    }
  }
  for (int i = t; i < SKEL; i += kBlock) {
    prow[i] = i;
    pcol[i] = i;
  }
  __syncthreads();
  const int kmax = min(min(nr, nc), tk.kmax);
  T first = T(0);
  int r = 0;
  for (int k = 0; k < kmax; ++k) {
    // largest |entry| of the trailing block; ties to the lowest row-major position
    T bv = T(-1);
    int bi = INT_MAX;
    const int w = nc - k, tot = (nr - k) * w;
    for (int e = t; e < tot; e += kBlock) {
      const int i = k + e / w, j = k + e % w;
      argmax_merge(bv, bi, dabs(A[i + j * ld]), e);
    }
    T pv;
    int flat;
    block_argmax(bv, bi, sv, si, pv, flat);
    if (k == 0) first = pv;
    if (!(pv > T(0)) || pv < eps * first || !(pv < T(INFINITY))) break;
    const int pi = k + flat / w, pj = k + flat % w;
    if (pi != k) {
      for (int j = t; j < nc; j += kBlock) {
        const T x = A[k + j * ld];
        A[k + j * ld] = A[pi + j * ld];
        A[pi + j * ld] = x;
      }
      if (t == 0) {
        const int x = prow[k];
        prow[k] = prow[pi];
        prow[pi] = x;
      }
    }
    __syncthreads();
    if (pj != k) {
      for (int i = t; i < nr; i += kBlock) {
        const T x = A[i + k * ld];
        A[i + k * ld] = A[i + pj * ld];
        A[i + pj * ld] = x;
      }
      if (t == 0) {
        const int x = pcol[k];
        pcol[k] = pcol[pj];
        pcol[pj] = x;
      }
    }
    __syncthreads();
    const T rp = T(1) / A[k + k * ld];
    for (int i = k + 1 + t; i < nr; i += kBlock) A[i + k * ld] *= rp;
    __syncthreads();
    const int h = nr - k - 1;
    for (int e = t; e < h * (nc - k - 1); e += kBlock) {
      const int i = k + 1 + e % h, j = k + 1 + e / h;
      A[i + j * ld] -= A[i + k * ld] * A[k + j * ld];
    }
    __syncthreads();
    r = k + 1;
  }
  if (t == 0) {
    s_r = r;
    rank_out[tk.node] = r;
    rank_task[task] = r;
  }
  for (int l = t; l < r; l += kBlock) {
    piv_out[tk.sel_off + l] = rows[prow[l]];         // picked rows in pivot order
    piv_out[tk.sel_off + SKEL + l] = cols[pcol[l]];  // picked columns in pivot order
  }
  __syncthreads();
  // In-place inverse of U11 (upper), column by column:
  // Uinv(0:j, j) = -Uinv(0:j, 0:j) U(0:j, j) / U(j, j)
  for (int j = 0; j < r; ++j) {
    const T ujj = T(1) / A[j + j * ld];
    for (int i = t; i < j; i += kBlock) {
      T s = T(0);
      for (int l = i; l < j; ++l) s += A[i + l * ld] * A[l + j * ld];
      tmp[i] = -s * ujj;
    }
    __syncthreads();
    for (int i = t; i < j; i += kBlock) A[i + j * ld] = tmp[i];
    if (t == 0) A[j + j * ld] = ujj;
    __syncthreads();
  }
  // In-place inverse of the unit lower L11, from the last column back:
  // Linv(j+1:r, j) = -Linv(j+1:r, j+1:r) L(j+1:r, j)
  for (int j = r - 2; j >= 0; --j) {
    for (int i = j + 1 + t; i < r; i += kBlock) {
      T s = A[i + j * ld];
      for (int l = j + 1; l < i; ++l) s += A[i + l * ld] * A[l + j * ld];
      tmp[i] = -s;
    }
    __syncthreads();
    for (int i = j + 1 + t; i < r; i += kBlock) A[i + j * ld] = tmp[i];
    __syncthreads();
  }
  T* Ui = inv + tk.inv_off;               // r x r, ld r: U11^-1
  T* LiT = inv + tk.inv_off + SKEL * SKEL;  // r x r, ld r: (L11^-1)^T
  for (int e = t; e < r * r; e += kBlock) {
    const int i = e % r, j = e / r;
    Ui[i + (size_t)j * r] = (i <= j) ? A[i + j * ld] : T(0);
    // (L^-1)^T (i, j) = L^-1 (j, i): unit lower -> unit upper
    LiT[i + (size_t)j * r] = (i < j) ? A[j + i * ld] : (i == j ? T(1) : T(0));
  }
}

// Gathers the panels: side 0: C(i, l) = K(row0 + i, pivot column l);
// side 1: Rt(j, l) = K(pivot row l, col0 + j).
template <typename T, int SKEL>
__global__ void __launch_bounds__(kBlock)
    k_bdlr_gather(const double* __restrict__ K, int ldk, const BdlrTask* __restrict__ tasks,
                  const int* __restrict__ piv, const int* __restrict__ rank_task, T* __restrict__ cg) {
  const int task = blockIdx.x, side = blockIdx.z, t = threadIdx.x;
  const BdlrTask tk = tasks[task];
  const int r = rank_task[task];
  const int len = side == 0 ? tk.m : tk.nc;
  const int i = blockIdx.y * kBlock + t;
  if (i >= len || r == 0) return;
  T* out = cg + tk.cg_off + (side == 0 ? 0 : (size_t)tk.m * tk.kmax);
  const int* pv = piv + tk.sel_off + (side == 0 ? SKEL : 0);
  for (int l0 = 0; l0 < r; l0 += 8) {
    T v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int l = l0 + u;
      if (l < r) {
        const int p = pv[l];
        v[u] = side == 0 ? (T)K[(size_t)(tk.col0 + p) * ldk + tk.row0 + i]
                         : (T)K[(size_t)(tk.col0 + i) * ldk + tk.row0 + p];
      } else {
        v[u] = T(0);
      }
    }
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (l0 + u < r) out[i + (size_t)(l0 + u) * len] = v[u];
  }
}

// U(rows of I) = C U11^-1 ; V(rows of J) = Rt L11^-T, 256 rows per workgroup.
template <typename T, int SKEL>
__global__ void __launch_bounds__(kBlock)
    k_bdlr_factors(const BdlrTask* __restrict__ tasks, const int* __restrict__ rank_task,
                   const T* __restrict__ cg, const T* __restrict__ inv, T* __restrict__ Ucap,
                   T* __restrict__ Vcap, int ldu) {
  __shared__ T As[32 * 33], Bs[32 * 33];
  const int task = blockIdx.x, side = blockIdx.z;
  const BdlrTask tk = tasks[task];
  const int r = rank_task[task];
  const int len = side == 0 ? tk.m : tk.nc;
  const int i0 = blockIdx.y * 256, rn = min(256, len - i0);
  if (rn <= 0 || r == 0) return;
  const T* P = cg + tk.cg_off + (side == 0 ? 0 : (size_t)tk.m * tk.kmax) + i0;
  const T* Mi = inv + tk.inv_off + (side == 0 ? 0 : (size_t)SKEL * SKEL);
  T* out = (side == 0 ? Ucap + tk.row0 : Vcap + tk.col0) + i0 + (size_t)tk.capcol * ldu;
  wg_gemm(rn, r, r, T(1), P, len, Mi, r, T(0), out, ldu, As, Bs);
}

// One task per node below the root, in level order (level 1 left to right,
// then level 2, ...); sel holds 2 * skel ints per task.
template <typename T>
static std::vector<BdlrTask> make_tasks(const Tree& tr, const std::vector<int>& capoff,
                                        const std::vector<int>& cap, int skel, size_t* inv_elems,
                                        size_t* cg_elems) {
  std::vector<BdlrTask> tasks;
  size_t cgo = 0, invo = 0;
  int selo = 0;
  for (int q = 1; q <= tr.L; ++q)
    for (int i = 0; i < (1 << q); ++i) {
      const int c = node_id(q, i), sib = node_id(q, i ^ 1);
      BdlrTask tk{};
      tk.node = c;
      tk.row0 = tr.lo[c];
      tk.m = tr.size(c);
      tk.col0 = tr.lo[sib];
      tk.nc = tr.size(sib);
      tk.capcol = capoff.empty() ? 0 : capoff[q - 1];
      tk.kmax = std::min(std::min(tk.m, tk.nc), skel);
      if (!cap.empty()) tk.kmax = std::min(tk.kmax, cap[q - 1]);
      tk.sel_off = selo;
      tk.inv_off = invo;
      tk.cg_off = cgo;
      selo += 2 * skel;
      invo += 2 * (size_t)skel * skel;
      cgo += (size_t)(tk.m + tk.nc) * tk.kmax;
      tasks.push_back(tk);
    }
  *inv_elems = invo;
  *cg_elems = cgo;
  return tasks;
}

template <typename T, int SKEL>
static int bdlr_t(hodlr_s* h, const double* K, int ldk, const int* rowptr, const int* col, T* Ucap,
                  T* Vcap, const std::vector<int>& capoff, const std::vector<int>& cap, hipStream_t s) {
  const Tree& tr = h->tree;
  if (tr.n > 2 * kBdlrMaxSide) return fail(HODLR_EINVAL, "BDLR supports n <= 16384");
  if (h->depth > 250) return fail(HODLR_EINVAL, "bdlr_depth must be <= 250");
  size_t invo = 0, cgo = 0;
  const std::vector<BdlrTask> tasks = make_tasks<T>(tr, capoff, cap, SKEL, &invo, &cgo);
  const int selo = 2 * SKEL * (int)tasks.size();
  const int nt = (int)tasks.size();
  int maxside = 0;
  for (auto& tk : tasks) maxside = std::max(maxside, std::max(tk.m, tk.nc));
  DevBuf d_tasks, d_sel, d_piv, d_cnt, d_rt, d_inv, d_cg;
  HODLR_TRY(d_tasks.ensure(nt * sizeof(BdlrTask)));
  HODLR_TRY(d_sel.ensure((size_t)selo * sizeof(int)));
  HODLR_TRY(d_piv.ensure((size_t)selo * sizeof(int)));
  HODLR_TRY(d_cnt.ensure((size_t)2 * nt * sizeof(int)));
  HODLR_TRY(d_rt.ensure((size_t)nt * sizeof(int)));
  HODLR_TRY(d_inv.ensure(std::max<size_t>(invo, 1) * sizeof(T)));
  HODLR_TRY(d_cg.ensure(std::max<size_t>(cgo, 1) * sizeof(T)));
  HODLR_HIP(hipMemcpyAsync(d_tasks.p, tasks.data(), nt * sizeof(BdlrTask), hipMemcpyHostToDevice, s));
  HODLR_HIP(hipMemsetAsync(h->d_rank.p, 0, tr.nnodes() * sizeof(int), s));
  {
    ProfScope prof("bdlr_select", s);
    k_bdlr_select<<<nt, kBlock, 0, s>>>(rowptr, col, d_tasks.as<BdlrTask>(), h->depth, SKEL,
                                        d_sel.as<int>(), d_cnt.as<int>());
  }
  HODLR_HIP(hipGetLastError());
  const size_t lds = (size_t)SKEL * (SKEL + 1) * sizeof(T);
  HODLR_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(k_bdlr_lu<T, SKEL>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  {
    ProfScope prof("bdlr_lu", s);
    k_bdlr_lu<T, SKEL><<<nt, kBlock, lds, s>>>(K, ldk, d_tasks.as<BdlrTask>(), d_sel.as<int>(),
                                              d_cnt.as<int>(), (T)h->tol, d_piv.as<int>(), d_inv.as<T>(),
                                              h->d_rank.as<int>(), d_rt.as<int>());
  }
  HODLR_HIP(hipGetLastError());
  const int nch = (maxside + kBlock - 1) / kBlock;
  {
    ProfScope prof("bdlr_factors", s);
    k_bdlr_gather<T, SKEL><<<dim3(nt, nch, 2), kBlock, 0, s>>>(K, ldk, d_tasks.as<BdlrTask>(), d_piv.as<int>(),
                                                              d_rt.as<int>(), d_cg.as<T>());
    k_bdlr_factors<T, SKEL><<<dim3(nt, nch, 2), kBlock, 0, s>>>(d_tasks.as<BdlrTask>(), d_rt.as<int>(),
                                                               d_cg.as<T>(), d_inv.as<T>(), Ucap, Vcap,
                                                               tr.n);
  }
  HODLR_HIP(hipGetLastError());
  HODLR_HIP(hipStreamSynchronize(s));  // scratch goes back to the allocator cache
  return HODLR_OK;
}

int launch_bdlr(hodlr_s* h, const double* K, int ldk, const int* rowptr, const int* col, void* Ucap,
                void* Vcap, const std::vector<int>& capoff, const std::vector<int>& cap, hipStream_t s) {
  if (h->precision == 64)
    return bdlr_t<double, kSkel64>(h, K, ldk, rowptr, col, static_cast<double*>(Ucap),
                                   static_cast<double*>(Vcap), capoff, cap, s);
  return bdlr_t<float, kSkel32>(h, K, ldk, rowptr, col, static_cast<float*>(Ucap),
                                static_cast<float*>(Vcap), capoff, cap, s);
}

}  // namespace hodlr

using namespace hodlr;

extern "C" int hodlr_bdlr_select(const int* g_rowptr, const int* g_col, int n, int leaf, int depth,
                                 int max_skel, int* picks, int* counts, hipStream_t stream) {
  if (n < 2 || n > 2 * kBdlrMaxSide) return fail(HODLR_EINVAL, "n must be in [2, 16384]");
  if (leaf < 1 || leaf > kLeafMax) return fail(HODLR_EINVAL, "leaf out of range");
  if (depth < 1 || depth > 250) return fail(HODLR_EINVAL, "depth must be in [1, 250]");
  if (max_skel < 1 || max_skel > kBdlrMaxSide) return fail(HODLR_EINVAL, "max_skel out of range");
  if (!g_rowptr || !g_col || !picks || !counts) return fail(HODLR_EINVAL, "NULL pointer argument");
  Tree tr;
  tr.build(n, leaf);
  if (tr.L == 0) return fail(HODLR_EINVAL, "n <= leaf: the tree has no off-diagonal blocks");
  size_t invo = 0, cgo = 0;
  const std::vector<BdlrTask> tasks = make_tasks<float>(tr, {}, {}, max_skel, &invo, &cgo);
  const int nt = (int)tasks.size();
  DevBuf d_tasks;
  HODLR_TRY(d_tasks.ensure(nt * sizeof(BdlrTask)));
  HODLR_HIP(hipMemcpyAsync(d_tasks.p, tasks.data(), nt * sizeof(BdlrTask), hipMemcpyHostToDevice, stream));
  k_bdlr_select<<<nt, kBlock, 0, stream>>>(g_rowptr, g_col, d_tasks.as<BdlrTask>(), depth, max_skel, picks,
                                           counts);
  HODLR_HIP(hipGetLastError());
  HODLR_HIP(hipStreamSynchronize(stream));  // the task table goes back to the allocator cache
  return HODLR_OK;
}
