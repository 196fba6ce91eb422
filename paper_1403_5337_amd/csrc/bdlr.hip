// Boundary-distance low-rank approximation, BDLR (Sec. 5.3, eq. Ahat), of
// every off-diagonal block, all levels at once.
//
// For block K(I, J) (I = the node's rows, J = its sibling's, both contiguous
// index ranges after the ordering), one workgroup per block in each of:
//   select  boundary sets (vertices with an edge into the other set), a
//           level-synchronous breadth-first search inside each set up to
//           depth-1, and the picked rows/columns: distance < depth, nearest
//           the boundary first and at most max_skel of them, listed in
//           increasing position;
//   lu      Ahat = K(rows, cols) held in registers, LU with full pivoting
//           (largest |entry| of the remaining Schur complement, ties to the
//           lowest (row, column) of Ahat), kept while |pivot| >= eps |first
//           pivot| (Sec. 7.1), giving rank r and the pivot rows and columns;
//           then G = Ahat11^-1 for the r x r submatrix on them;
//   gather  C = K(I, pivot columns) and V = K(pivot rows, J)^T;
//   factors U = C G.
// U V^T = C Ahat11^-1 R = (C Q)(:, 1:r) U11^-1 L11^-1 (P R)(1:r, :) is the
// pseudo-skeleton C~ R~ of eq. Ahat; the split between the two factors
// differs (one r x r inverse and one panel product instead of two of each).
#include <algorithm>
#include <cstring>
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
  int samp0;     // first sample of the block in the learned proposer's numbering
  int capcol, kmax;
  int sel_off;   // ints: rows at sel_off, columns at sel_off + max_skel
  size_t inv_off;  // elements: G = Ahat11^-1 (r x r, column-major), max_skel^2 reserved
  size_t cg_off;   // elements: C panel (m x kmax) then R^T panel (nc x kmax)
  int task;        // position in the build's whole task list (attempt loops)
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

constexpr int kSelNb = 8;  // neighbour indices loaded together

__global__ void __launch_bounds__(kBlock)
    k_bdlr_select(const int* __restrict__ rowptr, const int* __restrict__ col,
                  const BdlrTask* __restrict__ tasks, int depth, int max_skel, int stride, int* __restrict__ sel,
                  int* __restrict__ counts) {
  __shared__ uint8_t dI[kBdlrMaxSide], dJ[kBdlrMaxSide];
  __shared__ int cnt[256], buf[kBlock], s_cut[2];
  const BdlrTask tk = tasks[blockIdx.x];
  const int t = threadIdx.x;
  const int r0 = tk.row0, r1 = tk.row0 + tk.m, c0 = tk.col0, c1 = tk.col0 + tk.nc;
  // boundary sets: an edge into the other set (neighbour lists read
  // kSelNb entries at a time, the loads issued together)
  for (int sd = 0; sd < 2; ++sd) {
    const int s0 = sd == 0 ? r0 : c0, len = sd == 0 ? tk.m : tk.nc;
    const int o0 = sd == 0 ? c0 : r0, o1 = sd == 0 ? c1 : r1;
    uint8_t* d = sd == 0 ? dI : dJ;
    for (int i = t; i < len; i += kBlock) {
      const int v = s0 + i, e1 = rowptr[v + 1];
      uint8_t dv = 255;
      for (int e0 = rowptr[v]; e0 < e1 && dv != 0; e0 += kSelNb) {
        int u[kSelNb];
#pragma unroll
        for (int k = 0; k < kSelNb; ++k) u[k] = e0 + k < e1 ? col[e0 + k] : -1;
#pragma unroll
        for (int k = 0; k < kSelNb; ++k)
          if (u[k] >= o0 && u[k] < o1) dv = 0;
      }
      d[i] = dv;
    }
  }
  __syncthreads();
  // breadth-first layers inside each set: the vertices of layer lvl mark
  // their unmarked out-neighbours in the same set (benign races: every
  // writer of a vertex writes the same layer number)
  for (int lvl = 0; lvl + 1 < depth; ++lvl) {
    for (int sd = 0; sd < 2; ++sd) {
      const int s0 = sd == 0 ? r0 : c0, s1 = sd == 0 ? r1 : c1, len = s1 - s0;
      uint8_t* d = sd == 0 ? dI : dJ;
      for (int i = t; i < len; i += kBlock) {
        if (d[i] != lvl) continue;
        const int v = s0 + i, e1 = rowptr[v + 1];
        for (int e0 = rowptr[v]; e0 < e1; e0 += kSelNb) {
          int u[kSelNb];
#pragma unroll
          for (int k = 0; k < kSelNb; ++k) u[k] = e0 + k < e1 ? col[e0 + k] : -1;
#pragma unroll
          for (int k = 0; k < kSelNb; ++k)
            if (u[k] >= s0 && u[k] < s1 && d[u[k] - s0] == 255) d[u[k] - s0] = (uint8_t)(lvl + 1);
        }
      }
    }
    __syncthreads();
  }
  pick_side(dI, tk.m, depth, max_skel, sel + tk.sel_off, counts + 2 * blockIdx.x, cnt, buf, s_cut);
  pick_side(dJ, tk.nc, depth, max_skel, sel + tk.sel_off + stride, counts + 2 * blockIdx.x + 1, cnt,
            buf, s_cut);
}

// Full-pivot elimination of Ahat held in registers: thread (lane, w) of the
// NW waves owns rows lane + 64 a and columns w + NW b of the tile.  Nothing
// moves: a pivot column and a pivot row are retired (a wave-uniform column
// bit, a per-lane row bit) and drop out of the pivot search, which is the
// largest |entry| of the Schur complement (ties: lowest row, then lowest
// column).  A step tracks only the per-row maxima during the update; the
// waves' maxima are combined across one barrier, then the one wave holding
// the maximum finds its position (the lowest row by a ballot per register
// row, then the lowest column by a ballot per register column) and
// publishes the pivot column before the second barrier.  Equal maxima in
// several waves take a third barrier to agree on the lowest position.  The
// pivot sequence is kept (prow, pcol: positions in Ahat).  Sixteen waves
// (four per SIMD) keep the VALU busy while each wave waits on its own chain
// of cross-lane steps; eight wider waves measured slower.
//
// Every step is also the exchange (Gauss-Jordan) step on the retired rows and
// columns, so the inverse of the pivot block comes out of the same sweep.
// With pivot p at (pr, pc), multipliers l = x(:, pc) / p and pivot row v =
// x(pr, :), the exchange step sets every other entry to x - l v, the pivot
// column to l, the pivot row to -v / p and the pivot to 1 / p.  Here the
// pivot row is kept as v with -1 at the pivot, i.e. -p times its exchanged
// value (its multiplier is taken as 0): the later steps act on each row
// linearly, so the row keeps that factor, and it is divided out once at the
// end.  After r steps the entry at (pivot row k, pivot column l), divided by
// -p_k, is Ahat11^-1 (k, l), with Ahat11 = Ahat(pivot rows, pivot columns)
// in pivot order; it is written to G (r x r, column-major).  The retired
// entries are updated on every step, so the update covers all columns.
// The multipliers are x(:, pc) times the rounded reciprocal of p.
constexpr int kLuWaves = 16;
constexpr int kLuBlock = 64 * kLuWaves;

// Position 256 i + j of the first entry (lowest row i, then lowest column j)
// of this wave with |x| == M over the active columns; M must be the wave's
// own maximum, so some row maximum ma[a] equals it.  One ballot per register
// row, then one per register column of the chosen row.
template <typename T, int RA, int CB, int NW>
__device__ __forceinline__ int first_position(const T (&x)[RA][CB], const T (&ma)[RA], T M, unsigned cact,
                                              int w) {
  int as = -1, ls = 0;
#pragma unroll
  for (int a = 0; a < RA; ++a) {
    const unsigned long long bal = __ballot(ma[a] == M);
    if (as < 0 && bal) {
      as = a;
      ls = __ffsll((long long)bal) - 1;
    }
  }
  as = __builtin_amdgcn_readfirstlane(as);
  ls = __builtin_amdgcn_readfirstlane(ls);
  int bs = 0;
#pragma unroll
  for (int a = 0; a < RA; ++a)
    if (a == as) {
#pragma unroll
      for (int b = CB - 1; b >= 0; --b)  // the lowest matching column wins
        if ((cact >> b) & 1u) {
          const unsigned long long bal = __ballot(fabs(x[a][b]) == M);
          if ((bal >> ls) & 1ull) bs = b;
        }
    }
  return ((ls + 64 * max(as, 0)) << 8) + w + NW * bs;
}

template <typename T, int RA, int CB, int NW>
__device__ int full_pivot_steps(const double* __restrict__ Kb, int ldk, const int* srow, const int* scol,
                                int nr, int nc, int kmax, T eps, int* prow, int* pcol, T* pval, T* colv,
                                T (*sv)[NW], int (*si)[NW], int* spos, T* __restrict__ G, int* rpos, int* cpos,
                                bool* bad) {
  static_assert(NW <= 16, "the maxima of the waves are combined inside one 16-lane row");
  static_assert(CB <= 32, "one bit per register column");
  const int t = threadIdx.x, lane = t & 63;
  const int w = __builtin_amdgcn_readfirstlane(t >> 6);
  unsigned cact = 0;  // per wave: bit b = column w + NW b still active
#pragma unroll
  for (int b = 0; b < CB; ++b) cact |= (w + NW * b < nc ? 1u : 0u) << b;
  unsigned ract = 0;  // per lane: bit a = row lane + 64 a still active
#pragma unroll
  for (int a = 0; a < RA; ++a) ract |= (lane + 64 * a < nr ? 1u : 0u) << a;
  T x[RA][CB];
#pragma unroll
  for (int a = 0; a < RA; ++a) {
    const int i = lane + 64 * a;
    const int ri = srow[i];
#pragma unroll
    for (int b = 0; b < CB; ++b) {
      const int j = w + NW * b;
      x[a][b] = (i < nr && j < nc) ? (T)Kb[(size_t)scol[j] * ldk + ri] : T(0);
    }
  }
  T ma[RA];  // per register row: largest |entry| over the active columns (0 on a retired row)
#pragma unroll
  for (int a = 0; a < RA; ++a) {
    ma[a] = T(0);
#pragma unroll
    for (int b = 0; b < CB; ++b)
      if ((cact >> b) & 1u) ma[a] = fmax(ma[a], fabs(x[a][b]));
  }
  T first = T(0);
  int r = 0;
  for (int k = 0; k < kmax; ++k) {
    const int par = k & 1;
    T lm = ma[0];
#pragma unroll
    for (int a = 1; a < RA; ++a) lm = fmax(lm, ma[a]);
    const T wm = wave_max(lm);
    if (lane == 0) sv[par][w] = wm;
    __syncthreads();
    // the waves' maxima, combined inside the first 16-lane row
    const T pv = lane < NW ? sv[par][lane] : T(-1);
    T M = pv;
    M = sel_max(M, dpp_move<0xB1>(M));
    M = sel_max(M, dpp_move<0x4E>(M));
    M = sel_max(M, dpp_move<0x141>(M));
    M = sel_max(M, dpp_move<0x140>(M));
    M = lane_value(M, 0);
    if (k == 0) first = M;
    if (!(M > T(0)) || M < eps * first || !(M < T(INFINITY))) break;
    const unsigned long long who = __ballot(lane < NW && pv == M);  // waves holding the maximum
    int enc = -1;  // the pivot position, in the wave that holds its column
    if (__popcll(who) == 1) {
      if (w == __ffsll((long long)who) - 1) enc = first_position<T, RA, CB, NW>(x, ma, M, cact, w);
    } else {
      if ((who >> w) & 1ull) {
        const int e = first_position<T, RA, CB, NW>(x, ma, M, cact, w);
        if (lane == 0) si[par][w] = e;
      }
      __syncthreads();
      int e = (lane < NW && ((who >> lane) & 1ull)) ? si[par][lane] : INT_MAX;
      e = min(e, dpp_move<0xB1>(e));
      e = min(e, dpp_move<0x4E>(e));
      e = min(e, dpp_move<0x141>(e));
      e = min(e, dpp_move<0x140>(e));
      e = __builtin_amdgcn_readlane(e, 0);
      if ((e & 255) % NW == w) enc = e;
    }
    enc = __builtin_amdgcn_readfirstlane(enc);
    if (enc >= 0) {
      // publish the pivot column
      const int bs = (enc & 255) / NW;
#pragma unroll
      for (int b = 0; b < CB; ++b)
        if (b == bs) {
#pragma unroll
          for (int a = 0; a < RA; ++a) colv[lane + 64 * a] = x[a][b];
        }
      if (lane == 0) {
        spos[par] = enc;
        prow[k] = enc >> 8;
        pcol[k] = enc & 255;
      }
    }
    __syncthreads();
    const int pi = __builtin_amdgcn_readfirstlane(spos[par]), pr = pi >> 8, pc = pi & 255;
    const int pl = pr & 63, ap = pr >> 6;
    const int bp = pc % NW == w ? pc / NW : -1;  // the pivot column's register column in this wave, or -1
    const T p = colv[pr], pinv = T(1) / p;
    if (t == 0) pval[k] = p;
    T l[RA];
#pragma unroll
    for (int a = 0; a < RA; ++a) l[a] = (a == ap && lane == pl) ? T(0) : colv[lane + 64 * a] * pinv;
    // the pivot row's entries, from the lane that holds them
    T rv[CB];
#pragma unroll
    for (int a = 0; a < RA; ++a)
      if (a == ap) {
#pragma unroll
        for (int b = 0; b < CB; ++b) rv[b] = lane_value(x[a][b], pl);
      }
    if (lane == pl) ract &= ~(1u << ap);
    if (bp >= 0) cact &= ~(1u << bp);
#pragma unroll
    for (int a = 0; a < RA; ++a) ma[a] = T(0);
#pragma unroll
    for (int b = 0; b < CB; ++b) {
      if ((cact >> b) & 1u) {
#pragma unroll
        for (int a = 0; a < RA; ++a) {
          x[a][b] = fma(-l[a], rv[b], x[a][b]);
          ma[a] = fmax(ma[a], fabs(x[a][b]));
        }
      } else {
#pragma unroll
        for (int a = 0; a < RA; ++a) x[a][b] = fma(-l[a], rv[b], x[a][b]);
      }
    }
    // the pivot column takes the multipliers, the pivot -1
#pragma unroll
    for (int b = 0; b < CB; ++b)
      if (b == bp) {
#pragma unroll
        for (int a = 0; a < RA; ++a) x[a][b] = (a == ap && lane == pl) ? T(-1) : l[a];
      }
#pragma unroll
    for (int a = 0; a < RA; ++a)
      if (!((ract >> a) & 1u)) ma[a] = T(0);
    r = k + 1;
  }
  if (G) {
    // Ahat11^-1 (k, l) = x(prow[k], pcol[l]) / -pval[k]: the steps of the
    // rows and columns, then one store per owned entry of the pivot block
    __syncthreads();
    for (int q = t; q < 64 * RA; q += blockDim.x) rpos[q] = -1;
    for (int q = t; q < NW * CB; q += blockDim.x) cpos[q] = -1;
    __syncthreads();
    for (int q = t; q < r; q += blockDim.x) {
      rpos[prow[q]] = q;
      cpos[pcol[q]] = q;
    }
    __syncthreads();
    int nonfinite = 0;
#pragma unroll
    for (int a = 0; a < RA; ++a) {
      const int rk = rpos[lane + 64 * a];
      if (rk < 0) continue;
      const T d = -pval[rk];
#pragma unroll
      for (int b = 0; b < CB; ++b) {
        const int cl = cpos[w + NW * b];
        if (cl >= 0) {
          const T g = x[a][b] / d;
          G[rk + (size_t)cl * r] = g;
          nonfinite |= !(fabs(g) < T(INFINITY)) ? 1 : 0;
        }
      }
    }
    *bad = __syncthreads_or(nonfinite) != 0;
  }
  return r;
}

// Pivots of every block, and (inv given) G = Ahat11^-1 with Ahat11 =
// Ahat(pivot rows, pivot columns) in pivot order (r x r, column-major at
// inv + inv_off): C(:, pivot columns) G R(pivot rows, :) is the pseudo-
// skeleton C~ R~ of eq. Ahat.  The elimination runs on the smallest register
// tile (64, 128 or SKEL square) that holds Ahat.  rank_out / rank_task
// receive the number of pivots; a non-finite entry of G drops the block
// (rank 0).
template <typename T, int SKEL>
__global__ void __launch_bounds__(kLuBlock)
    k_bdlr_lu(const double* __restrict__ K, int ldk, const BdlrTask* __restrict__ tasks,
              const int* __restrict__ sel, const int* __restrict__ counts, T eps, int rcap,
              int* __restrict__ piv_out, T* __restrict__ inv, int* __restrict__ rank_out,
              int* __restrict__ rank_task, const int* __restrict__ skip) {
  static_assert(SKEL % 64 == 0 && SKEL <= 256 && SKEL % kLuWaves == 0, "tile shape");
  constexpr int NW = kLuWaves;
  __shared__ int srow[SKEL], scol[SKEL], prow[SKEL], pcol[SKEL], rpos[SKEL], cpos[SKEL];
  __shared__ T pval[SKEL], colv[SKEL];
  __shared__ T sv[2][NW];
  __shared__ int si[2][NW], spos[2];
  const int task = blockIdx.x, t = threadIdx.x;
  if (skip && skip[task]) return;
  const BdlrTask tk = tasks[task];
  const int nr = counts[2 * task], nc = counts[2 * task + 1];
  for (int x = t; x < SKEL; x += blockDim.x) {
    srow[x] = x < nr ? sel[tk.sel_off + x] : 0;
    scol[x] = x < nc ? sel[tk.sel_off + SKEL + x] : 0;
  }
  __syncthreads();
  const double* Kb = K + (size_t)tk.col0 * ldk + tk.row0;
  const int kmax = min(min(nr, nc), min(tk.kmax, rcap));
  const int side = max(nr, nc);
  T* G = inv ? inv + tk.inv_off : nullptr;
  bool bad = false;
  int r;
  if (side <= 64)
    r = full_pivot_steps<T, 1, 64 / NW, NW>(Kb, ldk, srow, scol, nr, nc, kmax, eps, prow, pcol, pval, colv, sv,
                                            si, spos, G, rpos, cpos, &bad);
  else if (side <= 128 || SKEL <= 128)
    r = full_pivot_steps<T, 2, 128 / NW, NW>(Kb, ldk, srow, scol, nr, nc, kmax, eps, prow, pcol, pval, colv, sv,
                                             si, spos, G, rpos, cpos, &bad);
  else
    r = full_pivot_steps<T, SKEL / 64, SKEL / NW, NW>(Kb, ldk, srow, scol, nr, nc, kmax, eps, prow, pcol, pval,
                                                      colv, sv, si, spos, G, rpos, cpos, &bad);
  __syncthreads();
  for (int q = t; q < r; q += blockDim.x) {
    piv_out[tk.sel_off + q] = srow[prow[q]];         // picked rows in pivot order
    piv_out[tk.sel_off + SKEL + q] = scol[pcol[q]];  // picked columns in pivot order
  }
  if (t == 0) {
    rank_out[tk.node] = bad ? 0 : r;
    rank_task[task] = bad ? 0 : r;
  }
}

// The pivots and G of ns blocks.
template <typename T, int SKEL>
static int launch_bdlr_lu(const double* K, int ldk, const BdlrTask* tasks, int ns, const int* sel, const int* cnt,
                          T eps, int rcap, int* piv, T* inv, int* rank_out, int* rank_task, hipStream_t s,
                          const int* skip = nullptr) {
  k_bdlr_lu<T, SKEL><<<ns, kLuBlock, 0, s>>>(K, ldk, tasks, sel, cnt, eps, rcap, piv, inv, rank_out, rank_task,
                                              skip);
  HODLR_HIP(hipGetLastError());
  return HODLR_OK;
}

// Gathers the panels: side 0: C(i, l) = K(row0 + i, pivot column l) into the
// work panel; side 1: V(j, l) = K(pivot row l, col0 + j) straight into the
// capped V panel.
template <typename T, int SKEL>
__global__ void __launch_bounds__(kBlock)
    k_bdlr_gather(const double* __restrict__ K, int ldk, const BdlrTask* __restrict__ tasks,
                  const int* __restrict__ piv, const int* __restrict__ rank_task, T* __restrict__ cg,
                  T* __restrict__ Ucap, T* __restrict__ Vcap, int ldu, const int* __restrict__ skip) {
  __shared__ int spv[SKEL];  // the side's pivots, read once per workgroup
  const int task = blockIdx.x, side = blockIdx.z, t = threadIdx.x;
  if (skip && skip[task]) return;
  const BdlrTask tk = tasks[task];
  const int r = rank_task[task];
  const int len = side == 0 ? tk.m : tk.nc;
  if ((int)blockIdx.y * kBlock >= len) return;  // (uniform)
  const int i = blockIdx.y * kBlock + t;
  const bool act = i < len;
  if (act) {  // the factor columns past the rank are zero (an earlier attempt may have written them)
    T* z = (side == 0 ? Ucap + tk.row0 : Vcap + tk.col0) + (size_t)tk.capcol * ldu + i;
    for (int l = r; l < tk.kmax; ++l) z[(size_t)l * ldu] = T(0);
  }
  if (r == 0) return;  // (uniform)
  const int* pv = piv + tk.sel_off + (side == 0 ? SKEL : 0);
  for (int l = t; l < r; l += kBlock) spv[l] = pv[l];
  __syncthreads();
  if (!act) return;
  T* out = side == 0 ? cg + tk.cg_off : Vcap + (size_t)tk.capcol * ldu + tk.col0;
  const int ldo = side == 0 ? len : ldu;
  // side 0 reads column pcol_l from row row0 + i, side 1 row prow_l from
  // column col0 + i; kB entries per batch with their loads in flight together
  // (the pivot index clamped into the rank, the store only below it)
  const double* base = side == 0 ? K + tk.row0 + i : K + (size_t)(tk.col0 + i) * ldk + tk.row0;
  const size_t stride = side == 0 ? (size_t)ldk : 1;
  constexpr int kB = 16;
  for (int l0 = 0; l0 < r; l0 += kB) {
    T v[kB];
#pragma unroll
    for (int u = 0; u < kB; ++u) {
      const int p = spv[min(l0 + u, r - 1)];
      v[u] = (T)base[(size_t)(side == 0 ? tk.col0 + p : p) * stride];
    }
#pragma unroll
    for (int u = 0; u < kB; ++u)
      if (l0 + u < r) out[i + (size_t)(l0 + u) * ldo] = v[u];
  }
}

// U(rows of I) = C G, 256 rows per workgroup.
// U(rows of the block, 0:r) = C G, one 64 x 64 tile of U per workgroup
// (blockIdx.y: row tile, blockIdx.z: column tile), on the matrix cores: each
// wave owns a 32 x 32 quarter.  The tile's 64 rows of C (all r columns) and
// 64 columns of G go to LDS in one round of asynchronous copies; the inner
// dimension is padded with zeros to the MFMA depth.
template <typename T> constexpr int mfma_depth() { return sizeof(T) == 4 ? 2 : 4; }
template <typename T> constexpr int factors_kmax() { return sizeof(T) == 4 ? kRankCap32 : kRankCap64; }

template <typename T>
struct FactorsSmem {
  static constexpr int kK = (factors_kmax<T>() + 3) / 4 * 4;  // padded inner dimension
  static constexpr int kLdA = 65, kLdB = kK + 1;
  T A[kK * kLdA];   // C(i0 + i, k) at A[k kLdA + i]
  T B[64 * kLdB];   // G(k, j0 + j) at B[j kLdB + k]
};

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

template <typename T>
__global__ void __launch_bounds__(kBlock)
    k_bdlr_factors(const BdlrTask* __restrict__ tasks, const int* __restrict__ rank_task,
                   const T* __restrict__ cg, const T* __restrict__ inv, T* __restrict__ Ucap, int ldu,
                   const int* __restrict__ skip) {
  using S = FactorsSmem<T>;
  __shared__ S sm;
  const int task = blockIdx.x, t = threadIdx.x, lane = t & 63, w = t >> 6;
  if (skip && skip[task]) return;
  const BdlrTask tk = tasks[task];
  const int r = rank_task[task];
  const int i0 = blockIdx.y * 64, j0 = blockIdx.z * 64;
  const int rn = min(64, tk.m - i0), cn = min(64, r - j0);
  if (rn <= 0 || cn <= 0) return;
  constexpr int D = mfma_depth<T>();
  const int kp = (r + D - 1) / D * D;
  // zero the padding of the inner dimension
  for (int e = t; e < (kp - r) * 64; e += kBlock) {
    const int k = r + e / 64, i = e % 64;
    sm.A[k * S::kLdA + i] = T(0);
    sm.B[i * S::kLdB + k] = T(0);
  }
  const T* C = cg + tk.cg_off + i0;  // column k at C + k m
  const T* G = inv + tk.inv_off + (size_t)j0 * r;
  for (int k = w; k < r; k += kBlock / 64) dma_span(sm.A + k * S::kLdA, C + (size_t)k * tk.m, rn);
  for (int j = w; j < cn; j += kBlock / 64) dma_span(sm.B + j * S::kLdB, G + (size_t)j * r, r);
  dma_wait();
  const int wm = (w & 1) * 32, wn = (w >> 1) * 32;
  T* U = Ucap + tk.row0 + i0 + (size_t)(tk.capcol + j0) * ldu;
  if constexpr (sizeof(T) == 4) {
    f32x16 acc = {};
    const int am = wm + (lane & 31), bn = wn + (lane & 31), kl = lane >> 5;
    for (int k = 0; k < kp; k += 2) {
      const float a = sm.A[(k + kl) * S::kLdA + am];
      const float b = sm.B[bn * S::kLdB + k + kl];
      acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, acc, 0, 0, 0);
    }
    // D(v) at lane l: row 8 (v / 4) + 4 (l / 32) + v % 4, column l % 32
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int i = wm + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3), j = wn + (lane & 31);
      if (i < rn && j < cn) U[i + (size_t)j * ldu] = acc[v];
    }
  } else {
    f64x4 acc[2][2] = {};
    const int ml = lane & 15, kl = lane >> 4;
    for (int k = 0; k < kp; k += 4) {
      double a[2], b[2];
#pragma unroll
      for (int x = 0; x < 2; ++x) {
        a[x] = sm.A[(k + kl) * S::kLdA + wm + 16 * x + ml];
        b[x] = sm.B[(wn + 16 * x + ml) * S::kLdB + k + kl];
      }
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) acc[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[x], b[y], acc[x][y], 0, 0, 0);
    }
    // D(v) at lane l: row l / 16 + 4 v, column l % 16
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int y = 0; y < 2; ++y)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int i = wm + 16 * x + (lane >> 4) + 4 * v, j = wn + 16 * y + (lane & 15);
          if (i < rn && j < cn) U[i + (size_t)j * ldu] = acc[x][y][v];
        }
  }
}

// One task per node below the root, in level order (level 1 left to right,
// then level 2, ...); sel holds 2 * skel ints per task.
template <typename T>
static std::vector<BdlrTask> make_tasks(const Tree& tr, const std::vector<int>& capoff,
                                        const std::vector<int>& cap, int skel, size_t* inv_elems,
                                        size_t* cg_elems) {
  std::vector<BdlrTask> tasks;
  size_t cgo = 0, invo = 0;
  int selo = 0, samp = 0;
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
      tk.samp0 = samp;
      samp += tk.m + tk.nc;
      selo += 2 * skel;
      invo += (size_t)skel * skel;
      cgo += (size_t)tk.m * tk.kmax;
      tasks.push_back(tk);
    }
  *inv_elems = invo;
  *cg_elems = cgo;
  return tasks;
}

template <typename T, int SKEL>
static int bdlr_t(hodlr_s* h, const double* K, int ldk, const int* rowptr, const int* col, T* Ucap,
                  T* Vcap, const std::vector<int>& capoff, const std::vector<int>& cap, hipStream_t s,
                  int max_skel, int* piv_export) {
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
    const int ms = max_skel > 0 ? std::min(max_skel, SKEL) : SKEL;
    k_bdlr_select<<<nt, kBlock, 0, s>>>(rowptr, col, d_tasks.as<BdlrTask>(), h->depth, ms, SKEL,
                                        d_sel.as<int>(), d_cnt.as<int>());
  }
  HODLR_HIP(hipGetLastError());
  const int rcap = h->precision == 64 ? kRankCap64 : kRankCap32;
  {
    ProfScope prof("bdlr_lu", s);
    k_bdlr_lu<T, SKEL><<<nt, kLuBlock, 0, s>>>(K, ldk, d_tasks.as<BdlrTask>(), d_sel.as<int>(), d_cnt.as<int>(),
                                                (T)h->tol, rcap, d_piv.as<int>(), d_inv.as<T>(), h->d_rank.as<int>(),
                                                d_rt.as<int>(), nullptr);
  }
  HODLR_HIP(hipGetLastError());
  const int nch = (maxside + kBlock - 1) / kBlock;
  {
    ProfScope prof("bdlr_gather", s);
    k_bdlr_gather<T, SKEL><<<dim3(nt, nch, 2), kBlock, 0, s>>>(K, ldk, d_tasks.as<BdlrTask>(), d_piv.as<int>(),
                                                              d_rt.as<int>(), d_cg.as<T>(), Ucap, Vcap, tr.n,
                                                              nullptr);
  }
  HODLR_HIP(hipGetLastError());
  {
    ProfScope prof("bdlr_factors", s);
    k_bdlr_factors<T><<<dim3(nt, (maxside + 63) / 64, (rcap + 63) / 64), kBlock, 0, s>>>(
        d_tasks.as<BdlrTask>(), d_rt.as<int>(), d_cg.as<T>(), d_inv.as<T>(), Ucap, tr.n, nullptr);
  }
  HODLR_HIP(hipGetLastError());
  if (piv_export)
    HODLR_HIP(hipMemcpyAsync(piv_export, d_piv.p, (size_t)selo * sizeof(int), hipMemcpyDeviceToDevice, s));
  // the scratch goes back to the allocator once s is past its last reader
  for (DevBuf* b : {&d_tasks, &d_sel, &d_piv, &d_cnt, &d_rt, &d_inv, &d_cg}) b->release_after(s);
  return HODLR_OK;
}

// ---------------------------------------------------------------------------
// Learned proposals: the k highest-scoring rows and columns of every block
// replace the boundary-distance picks; the skeleton is formed as above, its
// error is sampled on rows and columns outside the skeleton, and a block that
// misses the tolerance retries with twice the k, then falls back to ACA.
// ---------------------------------------------------------------------------

// larger score -> larger key; NaN lowest
__device__ __forceinline__ unsigned score_key(float x) {
  if (x != x) return 0u;
  const unsigned u = __float_as_uint(x);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

// |K(I, J)|_F^2 of every block.  The blocks are cut into chunks of whole
// columns of about kNormEntries entries, numbered across all blocks (block x
// owns chunks c0[x] .. c0[x + 1] - 1), one workgroup per chunk, so the work
// per workgroup is the same for every block size.  A thread walks the
// chunk's entries in column-major order with a stride of the workgroup size
// (row and column advanced incrementally, no division per load), eight
// loads in flight.  k_norm_total then adds a block's chunks in order into
// norm2[x], the slot the checks read; the chunk sums sit after the nt totals.
constexpr int kNormEntries = 16384;
__global__ void __launch_bounds__(kBlock)
    k_block_norm2(const double* __restrict__ K, int ldk, const BdlrTask* __restrict__ tasks,
                  const int* __restrict__ c0, int nt, double* __restrict__ part) {
  __shared__ double red[kBlock / 64];
  const int c = blockIdx.x, t = threadIdx.x;
  int lo = 0, hi = nt;  // the block of chunk c: the last x with c0[x] <= c
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (c0[mid] <= c) lo = mid;
    else hi = mid;
  }
  const BdlrTask tk = tasks[lo];
  const int m = tk.m, cols = max(1, kNormEntries / m);
  const int j0 = (c - c0[lo]) * cols, ncol = min(tk.nc, j0 + cols) - j0;
  const double* B = K + (size_t)(tk.col0 + j0) * ldk + tk.row0;
  const int di = kBlock % m, dj = kBlock / m;
  int i = t % m, j = t / m;
  constexpr int kU = 8;
  double acc = 0.0;
  while (j < ncol) {
    double v[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      v[u] = j < ncol ? B[(size_t)j * ldk + i] : 0.0;
      i += di;
      j += dj;
      if (i >= m) {
        i -= m;
        ++j;
      }
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) acc += v[u] * v[u];
  }
  acc = block_sum(acc, red);
  if (t == 0) part[c] = acc;
}

// One wave per block: lane l adds chunks l, l + 64, ... in order, then the
// lanes are combined by a fixed butterfly.
__global__ void __launch_bounds__(64)
    k_norm_total(const int* __restrict__ c0, const double* __restrict__ part, double* __restrict__ norm2) {
  const int x = blockIdx.x, lane = threadIdx.x;
  double s = 0.0;
  for (int c = c0[x] + lane; c < c0[x + 1]; c += 64) s += part[c];
  for (int o = 1; o < 64; o <<= 1) s += __shfl_xor(s, o, 64);
  if (lane == 0) norm2[x] = s;
}

// Estimated relative Frobenius error of U V^T on the block: the residual on
// the sampled rows (whole rows), scaled by (rows outside the skeleton) /
// (rows sampled), over |K(I, J)|_F^2; the same over columns; the larger of
// the two (float64).  samp: per task 2 * ns entries (rows, then columns; -1 =
// unused), ns <= 16; counts: rows and columns picked per task; norm2: per
// task of the whole list (BdlrTask::task), |K(I, J)|_F^2.
//
// A zero word for loads of entries outside the data (never written).
__device__ double g_bdlr_zero[2];

// k_skel_check: workgroup (task, chunk, group) sums the squared residual of
// the group's rows over its chunk of kCheckX columns (and of the group's
// columns over its chunk of kCheckX rows) into part: lane l takes position
// l of the chunk, and the four waves split the rank, their partial products
// added in wave order through LDS.  The factors' entries are loaded 16 at a
// time.  A task has gridDim.z groups of 2 ns positions (one group: the
// samples) and gridDim.y = check_chunks(tasks) chunks (chunks past a side's
// end write 0).  k_skel_err then adds a task's chunks in order and forms the
// estimate, so the result does not depend on timing.
constexpr int kCheckX = 64;
constexpr int kCheckWaves = kBlock / 64;

static int check_chunks(const std::vector<BdlrTask>& tasks) {
  int mx = 1;
  for (const BdlrTask& t : tasks) mx = std::max(mx, std::max(t.m, t.nc));
  return (mx + kCheckX - 1) / kCheckX;
}

template <typename T>
__global__ void __launch_bounds__(kBlock)
    k_skel_check(const double* __restrict__ K, int ldk, const BdlrTask* __restrict__ tasks,
                 const int* __restrict__ rank_task, const T* __restrict__ Ucap, const T* __restrict__ Vcap,
                 int ldu, const int* __restrict__ samp, int ns, double* __restrict__ part,
                 const int* __restrict__ skip) {
  constexpr int RC = sizeof(T) == 8 ? kRankCap64 : kRankCap32, NS = 16, kL = 16;
  constexpr int kStage = (NS * RC + kBlock - 1) / kBlock;  // staged entries per thread
  static_assert(NS == 4 * kCheckWaves, "each wave finishes four positions");
  __shared__ T uv[NS][RC];
  __shared__ double acc[kCheckWaves][NS][64];
  __shared__ int sp[2 * NS];
  __shared__ double red[kBlock / 64];
  if (skip && skip[blockIdx.x]) return;
  const BdlrTask tk = tasks[blockIdx.x];
  const int r = rank_task[blockIdx.x], t = threadIdx.x, lane = t & 63, w = t >> 6;
  const size_t grp = (size_t)blockIdx.x * gridDim.z + blockIdx.z;  // position group of this task
  const size_t slot = (grp * gridDim.y + blockIdx.y) * 2;
  if (t < 2 * NS) sp[t] = (t % NS) < ns ? samp[grp * 2 * ns + (t / NS) * ns + t % NS] : -1;
  __syncthreads();
  const T* U = Ucap + (size_t)tk.capcol * ldu;
  const T* V = Vcap + (size_t)tk.capcol * ldu;
  for (int side = 0; side < 2; ++side) {
    const int len = side == 0 ? tk.nc : tk.m;
    const int x0 = blockIdx.y * kCheckX;
    if (x0 >= len) {  // (uniform over the workgroup)
      if (t == 0) part[slot + side] = 0.0;
      continue;
    }
    // the fixed factor's sampled rows: U(row0 + p, :) (side 0) or V(col0 + p, :)
    const T* F = side == 0 ? U + tk.row0 : V + tk.col0;
    const T* O = side == 0 ? V + tk.col0 : U + tk.row0;
    {
      T v[kStage];
#pragma unroll
      for (int k = 0; k < kStage; ++k) {
        const int e = t + k * kBlock, q = e % NS, l = e / NS;
        const int p = e < NS * r ? sp[side * NS + q] : -1;
        // the address is chosen, not the value (a zero word for the entries
        // outside), so the loads are in flight together
        v[k] = *(p >= 0 ? F + (size_t)l * ldu + p : reinterpret_cast<const T*>(g_bdlr_zero));
      }
#pragma unroll
      for (int k = 0; k < kStage; ++k) {
        const int e = t + k * kBlock;
        if (e < NS * r) uv[e % NS][e / NS] = v[k];
      }
    }
    __syncthreads();
    const int x = x0 + lane;
    const bool in = x < len;
    const int rq = (r + kCheckWaves - 1) / kCheckWaves, l0 = min(r, w * rq), l1 = min(r, l0 + rq);
    double a[NS];
#pragma unroll
    for (int q = 0; q < NS; ++q) a[q] = 0.0;
    if (in) {
      int l = l0;
      for (; l + kL <= l1; l += kL) {
        // the kL loads from one base, all issued before the first use
        const T* Ob = O + (size_t)l * ldu + x;
        T o[kL];
#pragma unroll
        for (int u = 0; u < kL; ++u) o[u] = Ob[u * ldu];
#pragma unroll
        for (int u = 0; u < kL; ++u) {
          const double ou = (double)o[u];
#pragma unroll
          for (int q = 0; q < NS; ++q) a[q] += (double)uv[q][l + u] * ou;
        }
      }
      for (; l < l1; ++l) {
        const double o = (double)O[(size_t)l * ldu + x];
#pragma unroll
        for (int q = 0; q < NS; ++q) a[q] += (double)uv[q][l] * o;
      }
    }
#pragma unroll
    for (int q = 0; q < NS; ++q) acc[w][q][lane] = a[q];
    __syncthreads();
    // thread (lane, w): positions 4 w .. 4 w + 3 at x
    double num = 0.0;
    if (in) {
      double b[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int p = sp[side * NS + 4 * w + u];
        b[u] = *(p < 0 ? g_bdlr_zero
                       : side == 0 ? K + (size_t)(tk.col0 + x) * ldk + tk.row0 + p
                                   : K + (size_t)(tk.col0 + p) * ldk + tk.row0 + x);
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int q = 4 * w + u;
        if (sp[side * NS + q] >= 0) {
          double s = acc[0][q][lane];
#pragma unroll
          for (int k = 1; k < kCheckWaves; ++k) s += acc[k][q][lane];
          num += (b[u] - s) * (b[u] - s);
        }
      }
    }
    num = block_sum(num, red);
    if (t == 0) part[slot + side] = num;
    __syncthreads();
  }
}

__global__ void k_skel_err(const BdlrTask* __restrict__ tasks, int ntask, const int* __restrict__ counts,
                           const double* __restrict__ norm2, const int* __restrict__ samp, int ns,
                           const double* __restrict__ part, int nch, double* __restrict__ err,
                           const int* __restrict__ skip) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= ntask || (skip && skip[x])) return;
  const BdlrTask tk = tasks[x];
  // both sides' chunk sums (adjacent in part) in chunk order, kB chunks per
  // batch with their loads in flight together (addresses clamped into range)
  constexpr int kB = 16;
  double num[2] = {0.0, 0.0};
  const double2* pp = reinterpret_cast<const double2*>(part) + (size_t)x * nch;
  for (int c0 = 0; c0 < nch; c0 += kB) {
    double2 v[kB];
#pragma unroll
    for (int u = 0; u < kB; ++u) v[u] = pp[min(c0 + u, nch - 1)];
#pragma unroll
    for (int u = 0; u < kB; ++u)
      if (c0 + u < nch) {
        num[0] += v[u].x;
        num[1] += v[u].y;
      }
  }
  int used[2] = {0, 0};
  for (int q0 = 0; q0 < 2 * ns; q0 += kB) {
    int sv[kB];
#pragma unroll
    for (int u = 0; u < kB; ++u) sv[u] = samp[(size_t)x * 2 * ns + min(q0 + u, 2 * ns - 1)];
#pragma unroll
    for (int u = 0; u < kB; ++u)
      if (q0 + u < 2 * ns) used[(q0 + u) / ns] += sv[u] >= 0;
  }
  double est = 0.0;
  for (int side = 0; side < 2; ++side) {
    const int outside = (side == 0 ? tk.m : tk.nc) - counts[2 * x + side];
    if (used[side] > 0) est = fmax(est, num[side] * (double)outside / (double)used[side]);
  }
  const double nb = norm2[tk.task];  // the block's total (k_norm_total)
  err[x] = nb > 0.0 ? sqrt(est / nb) : sqrt(est);
}

// splitmix64 (Steele, Lea & Flood 2014): the sample stream of a block.  The
// state advances by a fixed increment per draw, so draw c (from 0) of the
// stream seeded with x0 is the mix of x0 + (c + 1) * increment, which lets
// every draw be computed on its own lane.
constexpr unsigned long long kSplitmixGamma = 0x9E3779B97F4A7C15ull;
__device__ __forceinline__ unsigned long long splitmix64_draw(unsigned long long x0, unsigned long long c) {
  unsigned long long z = x0 + (c + 1) * kSplitmixGamma;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Position p of the list of [0, len) without the picks (sorted ascending,
// distinct): p + k, k = the number of picks below the answer = the number of
// i with picked[i] - i <= p (non-decreasing in i), by binary search.
__device__ __forceinline__ int avail_at(const int* picked, int npick, int p) {
  int lo = 0, hi = npick;  // first i with picked[i] - i > p
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (picked[mid] - mid <= p) lo = mid + 1;
    else hi = mid;
  }
  return p + lo;
}

constexpr int kSkelSamples = 16;  // sampled rows (columns) per block side

// NS positions of [0, len) outside the picks, without replacement: the first
// NS steps of a Fisher-Yates shuffle of the list of unpicked positions.  Step
// x swaps list entries x and j[x] (j[x] = x + draw mod (navail - x), drawn
// beforehand, as are the entries' initial values ax[x] and aj[x]); the list
// itself is never built: the entries the swaps moved are kept in fixed
// register slots, 2x for position x and 2x + 1 for the position j swapped
// with it at step x, and a lookup takes the latest slot holding the position.
// Every loop is unrolled, so the slots stay in registers.
template <int NS>
__device__ void draw_side(int navail, const int* j_of, const int* ax, const int* aj, int* out) {
  int opos[2 * NS], oval[2 * NS];
#pragma unroll
  for (int k = 0; k < 2 * NS; ++k) opos[k] = -1;
#pragma unroll
  for (int x = 0; x < NS; ++x) {
    if (navail - x <= 0) {
      out[x] = -1;
      continue;
    }
    const int j = j_of[x];
    int vx = -1, vj = -1;
#pragma unroll
    for (int k = 2 * x - 1; k >= 0; --k) {  // latest first
      if (vx < 0 && opos[k] == x) vx = oval[k];
      if (vj < 0 && opos[k] == j) vj = oval[k];
    }
    if (vx < 0) vx = ax[x];
    if (vj < 0) vj = aj[x];
    opos[2 * x] = x;
    oval[2 * x] = vj;
    opos[2 * x + 1] = j;
    oval[2 * x + 1] = (j == x) ? vj : vx;
    out[x] = vj;
  }
}

// One wave per block of the attempt: the picks go to LDS; one stream seeded
// by the block's node and the attempt gives the row draws, then the column
// draws.  Lane q < 2 NS computes draw q % NS of side q / NS and the two list
// entries it swaps; then lane 0 (rows) and lane 1 (columns) run the swaps.
constexpr int kDrawPicks = 256;  // >= the largest skeleton (192 / 128)
struct DrawLds {
  int pk[2][kDrawPicks];
  int jv[2][kSkelSamples], ax[2][kSkelSamples], aj[2][kSkelSamples];
};
// The draws of one task by the first wave of the calling workgroup (the
// picks sel / cnt of the task at x are final); out: 2 ns ints.
__device__ void draw_task(const BdlrTask& tk, int x, const int* __restrict__ sel, const int* __restrict__ cnt,
                          int skel, unsigned long long seed, int attempt, int ns, int* __restrict__ out,
                          DrawLds& d) {
  constexpr int NS = kSkelSamples;
  const int t = threadIdx.x;
  const int np[2] = {min(cnt[2 * x], kDrawPicks), min(cnt[2 * x + 1], kDrawPicks)};
  if (t < 64) {
    for (int i = t; i < np[0]; i += 64) d.pk[0][i] = sel[tk.sel_off + i];
    for (int i = t; i < np[1]; i += 64) d.pk[1][i] = sel[tk.sel_off + skel + i];
  }
  __syncthreads();
  const unsigned long long st = seed ^ (0xD1B54A32D192ED03ull * (unsigned long long)tk.node) ^
                                (0x8CB92BA72F3D8DD7ull * (unsigned long long)(attempt + 1));
  const int navail[2] = {tk.m - np[0], tk.nc - np[1]};
  if (t < 2 * NS) {
    const int sd = t / NS, q = t % NS, na = navail[sd] - q;
    if (na > 0) {
      // the row side draws once per step with a nonempty list
      const int c = (sd == 0 ? 0 : min(NS, max(0, navail[0]))) + q;
      const int j = q + (int)(splitmix64_draw(st, (unsigned long long)c) % (unsigned long long)na);
      d.jv[sd][q] = j;
      d.ax[sd][q] = avail_at(d.pk[sd], np[sd], q);
      d.aj[sd][q] = avail_at(d.pk[sd], np[sd], j);
    }
  }
  __syncthreads();
  if (t < 2) draw_side<NS>(navail[t], d.jv[t], d.ax[t], d.aj[t], out + t * ns);
}

__global__ void __launch_bounds__(64)
    k_draw_samples(const BdlrTask* __restrict__ tasks, const int* __restrict__ sel, const int* __restrict__ cnt,
                   int skel, unsigned long long seed, int attempt, int ns, int* __restrict__ samp,
                   const int* __restrict__ skip) {
  __shared__ DrawLds d;
  const int x = blockIdx.x;
  if (skip && skip[x]) return;
  draw_task(tasks[x], x, sel, cnt, skel, seed, attempt, ns, samp + (size_t)x * 2 * ns, d);
}

// Scratch of the attempt loops (learned proposals, adaptive BDLR depth).
struct SkelScratch {
  DevBuf tasks, sel, piv, cnt, rt, inv, cg, samp, err, norm, part;
  int nch = 1;  // check chunks per side (check_chunks of the build's tasks)
  int ensure(int nt, int selo, size_t invo, size_t cgo, size_t esize, int nchunks) {
    nch = nchunks;
    HODLR_TRY(tasks.ensure(nt * sizeof(BdlrTask)));
    HODLR_TRY(sel.ensure((size_t)selo * sizeof(int)));
    HODLR_TRY(piv.ensure((size_t)selo * sizeof(int)));
    HODLR_TRY(cnt.ensure((size_t)2 * nt * sizeof(int)));
    HODLR_TRY(rt.ensure((size_t)nt * sizeof(int)));
    HODLR_TRY(inv.ensure(std::max<size_t>(invo, 1) * esize));
    HODLR_TRY(cg.ensure(std::max<size_t>(cgo, 1) * esize));
    HODLR_TRY(samp.ensure((size_t)nt * 2 * kSkelSamples * sizeof(int)));
    HODLR_TRY(err.ensure((size_t)nt * sizeof(double)));
    HODLR_TRY(part.ensure((size_t)nt * nch * 2 * sizeof(double)));
    return HODLR_OK;  // norm: sized by block_norms
  }
};

// |K(I, J)|_F^2 of every block of the build, once (the attempts read them by
// BdlrTask::task); the task list goes through sc.tasks, which each attempt
// then overwrites with its own.
// Uploads the task records and the chunk numbering (one copy on s); the
// norm kernels follow on run (which must be ordered after s's copy).
// staging (optional): pinned host memory of norm_upload_bytes(nt) bytes that
// stays valid until the stream is past the copy; without it the tables are
// copied from pageable memory.
static size_t norm_upload_bytes(int nt) { return (size_t)nt * sizeof(BdlrTask) + ((size_t)nt + 1) * sizeof(int); }

static int norm_upload(const std::vector<BdlrTask>& tasks, SkelScratch& sc, hipStream_t s, int* nchunk_out,
                       void* staging = nullptr) {
  const int nt = (int)tasks.size();
  // chunk numbering (c0, nt + 1 ints) after the task records in one upload
  std::vector<int> c0(nt + 1, 0);
  for (int x = 0; x < nt; ++x) {
    const int cols = std::max(1, kNormEntries / std::max(tasks[x].m, 1));
    c0[x + 1] = c0[x] + (tasks[x].nc + cols - 1) / cols;
  }
  const int nchunk = c0[nt];
  const size_t tb = (size_t)nt * sizeof(BdlrTask), ub = norm_upload_bytes(nt);
  std::vector<unsigned char> up;
  unsigned char* hp = static_cast<unsigned char*>(staging);
  if (!hp) {
    up.resize(ub);
    hp = up.data();
  }
  std::memcpy(hp, tasks.data(), tb);
  std::memcpy(hp + tb, c0.data(), (nt + 1) * sizeof(int));
  HODLR_TRY(sc.tasks.ensure(ub));
  HODLR_TRY(sc.norm.ensure(((size_t)nt + nchunk) * sizeof(double)));
  HODLR_HIP(hipMemcpyAsync(sc.tasks.p, hp, ub, hipMemcpyHostToDevice, s));
  *nchunk_out = nchunk;
  return HODLR_OK;
}

static int norm_launch(const double* K, int ldk, int nt, int nchunk, SkelScratch& sc, hipStream_t run) {
  const int* d_c0 = reinterpret_cast<const int*>(static_cast<unsigned char*>(sc.tasks.p) + (size_t)nt * sizeof(BdlrTask));
  ProfScope prof("skel_check", run);
  if (nchunk > 0) {
    k_block_norm2<<<nchunk, kBlock, 0, run>>>(K, ldk, sc.tasks.as<BdlrTask>(), d_c0, nt, sc.norm.as<double>() + nt);
    HODLR_HIP(hipGetLastError());
  }
  k_norm_total<<<nt, 64, 0, run>>>(d_c0, sc.norm.as<double>() + nt, sc.norm.as<double>());
  HODLR_HIP(hipGetLastError());
  return HODLR_OK;
}

static int block_norms(const double* K, int ldk, const std::vector<BdlrTask>& tasks, SkelScratch& sc, hipStream_t s) {
  int nchunk = 0;
  HODLR_TRY(norm_upload(tasks, sc, s, &nchunk));
  return norm_launch(K, ldk, (int)tasks.size(), nchunk, sc, s);
}

// One attempt over the ns blocks whose tasks are in sc.tasks and picks in
// sc.sel / sc.cnt: the pivot-block LU and inverse, the factors into Ucap /
// Vcap, then the sampled error of every block (samples drawn on the device
// outside its picks, from a stream seeded by the block and the attempt) into
// sc.err.  Blocks with skip[x] != 0 (skip may be NULL) are left untouched.
// The per-task arrays of an attempt launch, offset to its first task (a
// launch covers ns consecutive tasks of sc.tasks); the picks, pivots,
// inverses, panels and norms are reached through the task records
// (sel_off, inv_off, cg_off, task) and are shared by every launch.
struct AttemptView {
  const BdlrTask* tasks;
  int *cnt, *rt, *samp;
  double *part, *err;
};
static AttemptView attempt_view(SkelScratch& sc, int x0) {
  return {sc.tasks.as<BdlrTask>() + x0,
          sc.cnt.as<int>() + 2 * x0,
          sc.rt.as<int>() + x0,
          sc.samp.as<int>() + (size_t)x0 * 2 * kSkelSamples,
          sc.part.as<double>() + (size_t)x0 * sc.nch * 2,
          sc.err.as<double>() + x0};
}

template <typename T, int SKEL>
static int skel_attempt_launch(hodlr_s* h, const double* K, int ldk, int ns, int maxside, SkelScratch& sc,
                               const AttemptView& v, T* Ucap, T* Vcap, unsigned long long seed, int attempt,
                               const int* skip, hipStream_t s, bool own_draw_err = true) {
  const Tree& tr = h->tree;
  const int rcap = h->precision == 64 ? kRankCap64 : kRankCap32;
  {
    ProfScope prof("bdlr_lu", s);
    HODLR_TRY((launch_bdlr_lu<T, SKEL>(K, ldk, v.tasks, ns, sc.sel.as<int>(), v.cnt, (T)h->tol, rcap,
                                       sc.piv.as<int>(), sc.inv.as<T>(), h->d_rank.as<int>(), v.rt, s, skip)));
  }
  const int nch = (maxside + kBlock - 1) / kBlock;
  {
    ProfScope prof("bdlr_gather", s);
    k_bdlr_gather<T, SKEL><<<dim3(ns, nch, 2), kBlock, 0, s>>>(K, ldk, v.tasks, sc.piv.as<int>(), v.rt, sc.cg.as<T>(),
                                                              Ucap, Vcap, tr.n, skip);
    k_bdlr_factors<T><<<dim3(ns, (maxside + 63) / 64, (rcap + 63) / 64), kBlock, 0, s>>>(
        v.tasks, v.rt, sc.cg.as<T>(), sc.inv.as<T>(), Ucap, tr.n, skip);
  }
  HODLR_HIP(hipGetLastError());
  static_assert(SKEL <= kDrawPicks, "the picks of a side must fit the sampler's LDS");
  if (own_draw_err) {  // (else the caller's pick kernel drew them)
    k_draw_samples<<<ns, 64, 0, s>>>(v.tasks, sc.sel.as<int>(), v.cnt, SKEL, seed, attempt, kSkelSamples, v.samp,
                                     skip);
    HODLR_HIP(hipGetLastError());
  }
  {
    ProfScope prof("skel_check", s);
    k_skel_check<T><<<dim3(ns, sc.nch), kBlock, 0, s>>>(K, ldk, v.tasks, v.rt, Ucap, Vcap, tr.n, v.samp,
                                                         kSkelSamples, v.part, skip);
    if (own_draw_err)  // (else the caller's decision kernel forms the estimates)
      k_skel_err<<<(ns + kBlock - 1) / kBlock, kBlock, 0, s>>>(v.tasks, ns, v.cnt, sc.norm.as<double>(), v.samp,
                                                              kSkelSamples, v.part, sc.nch, v.err, skip);
  }
  HODLR_HIP(hipGetLastError());
  return HODLR_OK;
}

// skel_attempt_launch for every block of sub, then the errors and pick counts
// (rows, columns per block) to the host: one stream synchronization.
template <typename T, int SKEL>
static int skel_attempt(hodlr_s* h, const double* K, int ldk, const std::vector<BdlrTask>& sub, int maxside,
                        SkelScratch& sc, T* Ucap, T* Vcap, unsigned long long seed, int attempt,
                        std::vector<double>& err, std::vector<int>& cnt, hipStream_t s) {
  const int ns = (int)sub.size();
  HODLR_TRY((skel_attempt_launch<T, SKEL>(h, K, ldk, ns, maxside, sc, attempt_view(sc, 0), Ucap, Vcap, seed,
                                          attempt, nullptr, s)));
  err.assign(ns, 0.0);
  cnt.assign(2 * ns, 0);
  HODLR_HIP(hipMemcpyAsync(err.data(), sc.err.p, ns * sizeof(double), hipMemcpyDeviceToHost, s));
  HODLR_HIP(hipMemcpyAsync(cnt.data(), sc.cnt.p, 2 * ns * sizeof(int), hipMemcpyDeviceToHost, s));
  HODLR_HIP(hipStreamSynchronize(s));
  return HODLR_OK;
}

// ---------------------------------------------------------------------------
// Learned proposals, decided on the device.  State per block: 0 pending, 1
// accepted, 2 failed (the largest size tried is above the acceptance), 3
// failed at the caps (keeps its skeleton); the
// per-side budgets (rows, columns) double after every failing attempt, up to
// the skeleton cap; kused: the budget that passed.
// ---------------------------------------------------------------------------
constexpr int kLearnedAttempts = 4;

// First budgets: kinit per side, or (kinit == 0) the side's BDLR pick count
// at the build's depth (dcount), at least 1 and at most the cap and the side.
__global__ void k_learned_init(const BdlrTask* __restrict__ tasks, int nt, const int* __restrict__ dcount, int kinit,
                               int skel, int* __restrict__ budget, int* __restrict__ state,
                               int* __restrict__ kused) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= nt) return;
  const BdlrTask tk = tasks[x];
  for (int sd = 0; sd < 2; ++sd) {
    const int len = sd == 0 ? tk.m : tk.nc;
    const int k0 = kinit > 0 ? kinit : dcount[2 * x + sd];
    budget[2 * x + sd] = max(1, min(k0, min(skel, len)));
  }
  state[x] = 0;
  kused[x] = 0;
}

// After an attempt, for each pending block: its error estimate (as
// k_skel_err), then the decision: it passes at err <= accept; otherwise its
// budgets double (capped), and it fails when they cannot grow or on the last
// attempt: state 2 (the ACA fallback runs), or state 3 when its budgets are
// at the pick cap and its rank at the rank cap (ACA is held to the same rank
// cap; the block keeps its skeleton).
__global__ void k_err_decide(const BdlrTask* __restrict__ tasks, int nt, const int* __restrict__ counts,
                             const double* __restrict__ norm2, const int* __restrict__ samp, int ns,
                             const double* __restrict__ part, int nch, double* __restrict__ err, double accept,
                             int skel, int rcap, int last, const int* __restrict__ rank_task, int* __restrict__ budget,
                             int* __restrict__ state, int* __restrict__ kused) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= nt || state[x] != 0) return;
  const BdlrTask tk = tasks[x];
  // both sides' chunk sums (adjacent in part) in chunk order, kB chunks per
  // batch with their loads in flight together (addresses clamped into range)
  constexpr int kB = 16;
  double num[2] = {0.0, 0.0};
  const double2* pp = reinterpret_cast<const double2*>(part) + (size_t)x * nch;
  for (int c0 = 0; c0 < nch; c0 += kB) {
    double2 v[kB];
#pragma unroll
    for (int u = 0; u < kB; ++u) v[u] = pp[min(c0 + u, nch - 1)];
#pragma unroll
    for (int u = 0; u < kB; ++u)
      if (c0 + u < nch) {
        num[0] += v[u].x;
        num[1] += v[u].y;
      }
  }
  int used[2] = {0, 0};
  for (int q0 = 0; q0 < 2 * ns; q0 += kB) {
    int sv[kB];
#pragma unroll
    for (int u = 0; u < kB; ++u) sv[u] = samp[(size_t)x * 2 * ns + min(q0 + u, 2 * ns - 1)];
#pragma unroll
    for (int u = 0; u < kB; ++u)
      if (q0 + u < 2 * ns) used[(q0 + u) / ns] += sv[u] >= 0;
  }
  double est = 0.0;
  for (int side = 0; side < 2; ++side) {
    const int outside = (side == 0 ? tk.m : tk.nc) - counts[2 * x + side];
    if (used[side] > 0) est = fmax(est, num[side] * (double)outside / (double)used[side]);
  }
  const double nb = norm2[tk.task];
  const double e = nb > 0.0 ? sqrt(est / nb) : sqrt(est);
  err[x] = e;
  const int br = budget[2 * x], bc = budget[2 * x + 1];
  if (e <= accept) {
    state[x] = 1;
    kused[x] = max(br, bc);
    return;
  }
  const int nr = min(2 * br, min(skel, tk.m)), nc = min(2 * bc, min(skel, tk.nc));
  if (last || (nr == br && nc == bc)) {
    const bool capped = nr == br && nc == bc && rank_task[x] >= min(rcap, tk.kmax);
    state[x] = capped ? 3 : 2;
    kused[x] = -max(br, bc);
    return;
  }
  budget[2 * x] = nr;
  budget[2 * x + 1] = nc;
}

// Learned picks by mesh node.  On each side, dofs at consecutive positions
// with equal coordinates form one node (at most kRunMax dofs: later equal
// positions count as nodes of their own); a node scores the largest score of
// its dofs.  A side with budget k and longest node of g dofs takes the k / g
// best nodes (ties to the lower first position) and lists all their dofs in
// increasing position, so at most k picks.
constexpr int kRunMax = 8;

__device__ __forceinline__ bool same_point(const float* __restrict__ xyz, int u, int v) {
  return xyz[3 * u] == xyz[3 * v] && xyz[3 * u + 1] == xyz[3 * v + 1] && xyz[3 * u + 2] == xyz[3 * v + 2];
}

constexpr int kTopBlock = 1024, kTopWaves = kTopBlock / 64;

// Inclusive prefix over the workgroup's per-thread values (in thread order);
// *total receives the sum.  Two barriers.
__device__ int top_scan(int v, int* wsum, int* total) {
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  int x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) wsum[w] = x;
  __syncthreads();
  int before = 0, tot = 0;
#pragma unroll
  for (int k = 0; k < kTopWaves; ++k) {
    const int c = wsum[k];
    before += k < w ? c : 0;
    tot += c;
  }
  *total = tot;
  __syncthreads();
  return before + x;
}

// Workgroup maximum and sum of two per-thread values.  Two barriers.
__device__ void top_reduce(int& mx, int& sum, int (*red)[2]) {
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  for (int o = 32; o > 0; o >>= 1) {
    mx = max(mx, __shfl_xor(mx, o, 64));
    sum += __shfl_xor(sum, o, 64);
  }
  if (lane == 0) {
    red[w][0] = mx;
    red[w][1] = sum;
  }
  __syncthreads();
  mx = 0;
  sum = 0;
  for (int k = 0; k < kTopWaves; ++k) {
    mx = max(mx, red[k][0]);
    sum += red[k][1];
  }
  __syncthreads();
}

// One workgroup per block; per side: equal-point flags, the node runs and
// keys, the knode-th largest key by a radix select on 8-bit digits, then the
// chosen nodes' dofs listed in increasing position.  Then the attempt's
// sample draws of the block (as k_draw_samples).
__global__ void __launch_bounds__(kTopBlock)
    k_skel_topk_nodes(const float* __restrict__ score, const float* __restrict__ xyz,
                      const BdlrTask* __restrict__ tasks, const int* __restrict__ budget,
                      const int* __restrict__ skip, int skel, int* __restrict__ sel, int* __restrict__ counts,
                      unsigned long long seed, int attempt, int* __restrict__ samp) {
  __shared__ DrawLds dl;
  __shared__ unsigned key[kBdlrMaxSide];
  __shared__ float sco[kBdlrMaxSide];
  __shared__ unsigned char eqp[kBdlrMaxSide];  // position i has the point of position i - 1
  __shared__ unsigned char run[kBdlrMaxSide];  // dofs of the node starting here, 0 elsewhere
  __shared__ unsigned char flag[kBdlrMaxSide];
  __shared__ int hist[256];
  __shared__ int wsum[kTopWaves], red[kTopWaves][2];
  __shared__ unsigned s_digit, s_need;
  const int x = blockIdx.x, t = threadIdx.x;
  if (skip && skip[x]) return;
  const BdlrTask tk = tasks[x];
  for (int side = 0; side < 2; ++side) {
    const int len = side == 0 ? tk.m : tk.nc, v0 = side == 0 ? tk.row0 : tk.col0;
    const int off = tk.samp0 + (side == 0 ? 0 : tk.m);
    for (int i = t; i < len; i += kTopBlock) {
      eqp[i] = i > 0 && same_point(xyz, v0 + i, v0 + i - 1) ? 1 : 0;
      sco[i] = score[off + i];
      flag[i] = 0;
    }
    __syncthreads();
    // equal points form an equivalence (exact comparison), so position j has
    // the point of position i < j iff eqp holds on (i, j]
    auto back = [&](int i) {  // equal predecessors, counted up to kRunMax
      int c = 0;
      while (c < kRunMax && i - c > 0 && eqp[i - c]) ++c;
      return c;
    };
    int longest = 0, nstart = 0;
    for (int i = t; i < len; i += kTopBlock) {
      const int bk = back(i);
      const bool start = bk == 0 || bk >= kRunMax;
      int g = 0;
      float best = -INFINITY;
      if (start) {
        g = 1;
        best = sco[i];
        // a dof with kRunMax equal predecessors starts a node of its own
        while (g < kRunMax && i + g < len && eqp[i + g] && back(i + g) < kRunMax) {
          best = fmaxf(best, sco[i + g]);
          ++g;
        }
      }
      run[i] = (unsigned char)g;
      key[i] = start ? max(score_key(best), 1u) : 0u;
      longest = max(longest, g);
      nstart += start ? 1 : 0;
    }
    top_reduce(longest, nstart, red);
    const int k = min(budget[2 * x + side], min(skel, len));
    const int knode = min(nstart, max(1, k / max(1, longest)));
    // the knode-th largest key thr, digit by digit from the top; take = the
    // number of keys equal to thr that are chosen (the lowest positions)
    unsigned thr = 0u, mask = 0u;
    int take = knode;
    const bool all = knode >= len;
    if (!all) {
      for (int shift = 24; shift >= 0; shift -= 8) {
        for (int q = t; q < 256; q += kTopBlock) hist[q] = 0;
        __syncthreads();
        for (int i = t; i < len; i += kTopBlock) {
          const unsigned kv = key[i];
          if ((kv & mask) == thr) atomicAdd(&hist[(kv >> shift) & 255u], 1);
        }
        __syncthreads();
        if (t < 64) {
          // lane l holds digits 255 - 4 l .. 252 - 4 l; suffix sums from the top
          int c[4], cs = 0;
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            c[u] = hist[255 - 4 * t - u];
            cs += c[u];
          }
          int incl = cs;
#pragma unroll
          for (int o = 1; o < 64; o <<= 1) {
            const int y = __shfl_up(incl, o, 64);
            if (t >= o) incl += y;
          }
          int above = incl - cs;  // keys in the digits above this lane's four
          for (int u = 0; u < 4; ++u) {
            if (above < take && above + c[u] >= take) {
              s_digit = 255u - 4u * t - u;
              s_need = (unsigned)(take - above);
            }
            above += c[u];
          }
        }
        __syncthreads();
        // (the next write of s_digit comes two barriers later, and hist was
        // read before the barrier above)
        thr |= s_digit << shift;
        mask |= 255u << shift;
        take = (int)s_need;
      }
    }
    // positions of the keys equal to thr, in order, pick the first take
    const int seg = (len + kTopBlock - 1) / kTopBlock, b0 = min(len, t * seg), b1 = min(len, b0 + seg);
    int ne = 0, tot;
    if (!all)
      for (int i = b0; i < b1; ++i) ne += key[i] == thr ? 1 : 0;
    int e = top_scan(ne, wsum, &tot) - ne;
    for (int i = b0; i < b1; ++i) {
      const unsigned kv = key[i];
      const bool ise = !all && kv == thr;
      if (kv != 0u && (all || kv > thr || (ise && e < take)))
        for (int j = 0; j < run[i]; ++j) flag[i + j] = 1;
      e += ise ? 1 : 0;
    }
    __syncthreads();
    // the flagged positions in increasing order
    int nf = 0;
    for (int i = b0; i < b1; ++i) nf += flag[i];
    int pos = top_scan(nf, wsum, &tot) - nf;
    int* out = sel + tk.sel_off + side * skel;
    for (int i = b0; i < b1; ++i)
      if (flag[i]) out[pos++] = i;
    if (t == 0) counts[2 * x + side] = tot;
    __syncthreads();
  }
  // the attempt's sample draws for this block, from its final picks
  draw_task(tk, x, sel, counts, skel, seed, attempt, kSkelSamples, samp + (size_t)x * 2 * kSkelSamples, dl);
}

// The per-task rank of the fallback (ACA) approximation of failed blocks,
// and the skip mask of the blocks that did not fail.
__global__ void k_fallback_prep(const BdlrTask* __restrict__ tasks, int nt, const int* __restrict__ state,
                                const int* __restrict__ rank, int* __restrict__ rank2, int* __restrict__ skip2) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= nt) return;
  const bool failed = state[x] == 2;
  skip2[x] = failed ? 0 : 1;
  rank2[x] = failed ? rank[tasks[x].node] : 0;
}

// A failed block keeps the approximation with the smaller sampled error: the
// fallback's (its factors copied from U2 / V2, the rank it wrote) or its own
// last skeleton (whose rank is restored); kused then is 0 or minus the size.
template <typename T>
__global__ void __launch_bounds__(kBlock)
    k_fallback_choose(const BdlrTask* __restrict__ tasks, const int* __restrict__ state,
                      const double* __restrict__ err, const double* __restrict__ err2,
                      const int* __restrict__ rank_task, const T* __restrict__ U2, const T* __restrict__ V2,
                      T* __restrict__ Ucap, T* __restrict__ Vcap, int ldu, int* __restrict__ rank,
                      int* __restrict__ kused) {
  const int x = blockIdx.x, t = threadIdx.x;
  if (state[x] != 2) return;
  const BdlrTask tk = tasks[x];
  const bool aca = err2[x] < err[x];
  if (!aca) {
    if (t == 0) rank[tk.node] = rank_task[x];
    return;
  }
  if (t == 0) kused[x] = 0;
  for (int side = 0; side < 2; ++side) {
    const int len = side == 0 ? tk.m : tk.nc, r0 = side == 0 ? tk.row0 : tk.col0;
    const T* src = (side == 0 ? U2 : V2) + (size_t)tk.capcol * ldu + r0;
    T* dst = (side == 0 ? Ucap : Vcap) + (size_t)tk.capcol * ldu + r0;
    for (int e = blockIdx.y * kBlock + t; e < len * tk.kmax; e += gridDim.y * kBlock) {
      const int i = e % len, l = e / len;
      dst[i + (size_t)l * ldu] = src[i + (size_t)l * ldu];
    }
  }
}

// The fallback's comparison: each candidate's squared residual, exact on the
// rows (columns) the skeleton picked plus the sampled rows (columns) outside
// them scaled by (outside / sampled), over |K(I, J)|_F^2, the larger of the
// two sides.  Positions per task: G groups of 2 x 16 (rows, then columns):
// groups 0 .. G-2 hold the picks 16 at a time, group G-1 the samples.
__global__ void k_cand_positions(const BdlrTask* __restrict__ tasks, int nt, const int* __restrict__ sel,
                                 const int* __restrict__ cnt, int skel, const int* __restrict__ samp, int G,
                                 const int* __restrict__ skip, int* __restrict__ pos) {
  const int x = blockIdx.x, t = threadIdx.x;
  if (x >= nt || (skip && skip[x])) return;
  const BdlrTask tk = tasks[x];
  for (int e = t; e < G * 2 * kSkelSamples; e += blockDim.x) {
    const int g = e / (2 * kSkelSamples), side = (e / kSkelSamples) & 1, q = e % kSkelSamples;
    int v;
    if (g == G - 1) {
      v = samp[(size_t)x * 2 * kSkelSamples + side * kSkelSamples + q];
    } else {
      const int k = 16 * g + q;
      v = k < cnt[2 * x + side] ? sel[tk.sel_off + side * skel + k] : -1;
    }
    pos[(size_t)x * G * 2 * kSkelSamples + e] = v;
  }
}

__global__ void k_cand_err(const BdlrTask* __restrict__ tasks, int nt, const int* __restrict__ cnt,
                           const double* __restrict__ norm2, const int* __restrict__ pos, int G,
                           const double* __restrict__ part, int nch, const int* __restrict__ skip,
                           double* __restrict__ err) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= nt || (skip && skip[x])) return;
  const BdlrTask tk = tasks[x];
  double est = 0.0;
  for (int side = 0; side < 2; ++side) {
    double exact = 0.0, sampled = 0.0;
    for (int g = 0; g < G; ++g)
      for (int c = 0; c < nch; ++c) {
        const double v = part[(((size_t)x * G + g) * nch + c) * 2 + side];
        if (g == G - 1) sampled += v;
        else exact += v;
      }
    int used = 0;
    for (int q = 0; q < kSkelSamples; ++q)
      used += pos[((size_t)x * G + G - 1) * 2 * kSkelSamples + side * kSkelSamples + q] >= 0;
    const int outside = (side == 0 ? tk.m : tk.nc) - cnt[2 * x + side];
    const double e = exact + (used > 0 ? sampled * (double)outside / (double)used : 0.0);
    est = fmax(est, e);
  }
  const double nb = norm2[tk.task];  // the block's total (k_norm_total)
  err[x] = nb > 0.0 ? sqrt(est / nb) : sqrt(est);
}

template <typename T, int SKEL>
static int learned_t(hodlr_s* h, const double* K, int ldk, const int* rowptr, const int* col, const float* xyz,
                     const float* params, int kinit, unsigned long long seed, double accept, T* Ucap, T* Vcap,
                     const std::vector<int>& capoff, const std::vector<int>& cap, hipStream_t s) {
  const Tree& tr = h->tree;
  if (tr.n > 2 * kBdlrMaxSide) return fail(HODLR_EINVAL, "learned skeletons support n <= 16384");
  size_t invo = 0, cgo = 0;
  std::vector<BdlrTask> tasks = make_tasks<T>(tr, capoff, cap, SKEL, &invo, &cgo);
  const int nt = (int)tasks.size(), selo = 2 * SKEL * nt;
  for (int x = 0; x < nt; ++x) tasks[x].task = x;
  const std::vector<SkelBlock> blocks = skel_blocks(tr);
  const int N = 2 * tr.n * tr.L;  // every vertex is a row of one block and a column of another, per level
  int maxside = 0;
  for (auto& tk : tasks) maxside = std::max(maxside, std::max(tk.m, tk.nc));
  DevBuf d_feat, d_score, d_dcnt, d_budget, d_state, d_blk;
  HODLR_TRY(d_feat.ensure((size_t)N * 8 * sizeof(float)));
  HODLR_TRY(d_score.ensure((size_t)N * sizeof(float)));
  HODLR_TRY(d_dcnt.ensure((size_t)2 * nt * sizeof(int)));
  HODLR_TRY(d_budget.ensure((size_t)2 * nt * sizeof(int)));
  // block states, then the picks each block used: one read-back
  HODLR_TRY(d_state.ensure((size_t)2 * nt * sizeof(int)));
  int* const dstate = d_state.as<int>();
  int* const dkused = dstate + nt;
  SkelScratch sc;
  HODLR_TRY(sc.ensure(nt, selo, invo, cgo, sizeof(T), check_chunks(tasks)));
  // The attempts are queued in two batches (the host reads the block states
  // once in between); blocks already decided skip an attempt's kernels.  A
  // block's attempts depend only on its own decisions, so the
  // blocks of levels 1 and 2 (the largest picks, so the longest
  // eliminations) run their attempts on a side stream beside those of the
  // other levels, and the build waits for the longer of the two chains.  The
  // side stream first computes the block norms while the features and the
  // scores are computed on the build's stream.
  struct Group {
    int x0, n, maxside;
    hipStream_t st;
  };
  std::vector<Group> groups;
  {
    int nA = 0;
    while (nA < nt && 31 - __builtin_clz(tasks[nA].node + 1) <= 2) ++nA;
    for (int g = 0; g < 2; ++g) {
      const int x0 = g == 0 ? 0 : nA, x1 = g == 0 ? nA : nt;
      if (x1 <= x0) continue;
      int ms = 0;
      for (int x = x0; x < x1; ++x) ms = std::max(ms, std::max(tasks[x].m, tasks[x].nc));
      groups.push_back({x0, x1 - x0, ms, s});
    }
  }
  // The guards below wait for the streams on every return, so the scratch
  // and the pinned block outlive their work; "synced" skips the wait when a
  // read-back has just synchronized the build stream behind the side
  // stream's join and nothing was queued since.
  struct Join {
    hipStream_t side = nullptr;
    hipEvent_t e[4] = {nullptr, nullptr, nullptr, nullptr};
    bool synced = false;
    ~Join() {
      if (side && !synced) (void)hipStreamSynchronize(side);
      for (auto x : e) event_give(x);
    }
  } join;
  // One pinned block for this build's uploads (task and chunk tables, the
  // feature block table) and its read-back of the block states: the copies
  // are then asynchronous, and the block outlives them (it is returned after
  // the read-back's synchronization, or after the guards' on an early return).
  const size_t ub = (norm_upload_bytes(nt) + 255) & ~(size_t)255;
  const size_t bb = (blocks.size() * sizeof(SkelBlock) + 255) & ~(size_t)255;
  void* pin = nullptr;
  size_t pin_bytes = 0;
  HODLR_TRY(pinned_alloc(ub + bb + (size_t)2 * nt * sizeof(int), &pin, &pin_bytes));
  struct PinGuard {
    void* p;
    size_t b;
    hipStream_t s;
    bool synced;
    ~PinGuard() {
      if (!synced) (void)hipStreamSynchronize(s);
      pinned_free(p, b);
    }
  } pin_guard{pin, pin_bytes, s, false};
  unsigned char* const pin_up = static_cast<unsigned char*>(pin);
  unsigned char* const pin_blk = pin_up + ub;
  int* const pin_rb = reinterpret_cast<int*>(pin_blk + bb);
  int nchunk = 0;
  HODLR_TRY(norm_upload(tasks, sc, s, &nchunk, pin_up));  // (the task table for every kernel below)
  HODLR_TRY(d_blk.ensure(blocks.size() * sizeof(SkelBlock)));
  std::memcpy(pin_blk, blocks.data(), blocks.size() * sizeof(SkelBlock));
  HODLR_HIP(hipMemcpyAsync(d_blk.p, pin_blk, blocks.size() * sizeof(SkelBlock), hipMemcpyHostToDevice, s));
  if (groups.size() == 2) {
    HODLR_TRY(side_stream(1, &groups[0].st));
    join.side = groups[0].st;
    for (auto& x : join.e) HODLR_TRY(event_take(&x));
    HODLR_HIP(hipEventRecord(join.e[0], s));
    HODLR_HIP(hipStreamWaitEvent(join.side, join.e[0], 0));
    HODLR_TRY(norm_launch(K, ldk, nt, nchunk, sc, join.side));
    HODLR_HIP(hipEventRecord(join.e[2], join.side));
  } else {
    HODLR_TRY(norm_launch(K, ldk, nt, nchunk, sc, s));
  }
  {
    ProfScope prof("skel_features", s);
    HODLR_TRY(launch_skel_features(rowptr, col, xyz, K, ldk, blocks, d_feat.as<float>(), s, h->depth,
                                   d_dcnt.as<int>(), d_blk.as<SkelBlock>()));
  }
  {
    ProfScope prof("skel_score", s);
    HODLR_TRY(launch_mlp_forward(d_feat.as<float>(), N, params, 1, d_score.as<float>(), s));
  }
  HODLR_HIP(hipMemsetAsync(h->d_rank.p, 0, tr.nnodes() * sizeof(int), s));
  const int g1 = (nt + kBlock - 1) / kBlock;
  k_learned_init<<<g1, kBlock, 0, s>>>(sc.tasks.as<BdlrTask>(), nt, d_dcnt.as<int>(), kinit, SKEL,
                                       d_budget.as<int>(), dstate, dkused);
  HODLR_HIP(hipGetLastError());
  if (join.side) {
    // the side stream's attempts need the budgets; the build's need the norms
    HODLR_HIP(hipEventRecord(join.e[3], s));
    HODLR_HIP(hipStreamWaitEvent(join.side, join.e[3], 0));
    HODLR_HIP(hipStreamWaitEvent(s, join.e[2], 0));
  }
  auto queue = [&](int a0, int a1) -> int {
    join.synced = pin_guard.synced = false;
    for (int attempt = a0; attempt < a1; ++attempt)
      for (const Group& g : groups) {
        const AttemptView v = attempt_view(sc, g.x0);
        int* state_g = dstate + g.x0;
        int* budget_g = d_budget.as<int>() + 2 * g.x0;
        {
          ProfScope prof("skel_topk", g.st);
          k_skel_topk_nodes<<<g.n, kTopBlock, 0, g.st>>>(d_score.as<float>(), xyz, v.tasks, budget_g, state_g, SKEL,
                                                         sc.sel.as<int>(), v.cnt, seed, attempt, v.samp);
        }
        HODLR_HIP(hipGetLastError());
        HODLR_TRY((skel_attempt_launch<T, SKEL>(h, K, ldk, g.n, g.maxside, sc, v, Ucap, Vcap, seed, attempt,
                                                state_g, g.st, false)));
        k_err_decide<<<(g.n + kBlock - 1) / kBlock, kBlock, 0, g.st>>>(
            v.tasks, g.n, v.cnt, sc.norm.as<double>(), v.samp, kSkelSamples, v.part, sc.nch, v.err, accept, SKEL,
            h->precision == 64 ? kRankCap64 : kRankCap32, attempt == kLearnedAttempts - 1 ? 1 : 0, v.rt, budget_g,
            state_g, dkused + g.x0);
        HODLR_HIP(hipGetLastError());
      }
    if (join.side) {
      HODLR_HIP(hipEventRecord(join.e[1], join.side));
      HODLR_HIP(hipStreamWaitEvent(s, join.e[1], 0));
    }
    return HODLR_OK;
  };
  // The decisions stay on the device; the host reads the states once after
  // the first two attempts (most blocks are decided by then) and queues the
  // last two only if a block is still pending, instead of queueing launches
  // that would find nothing to do.
  std::vector<int> state(nt), kused(nt);
  constexpr int kFirstBatch = 2;
  auto read_back = [&]() -> int {
    HODLR_HIP(hipMemcpyAsync(pin_rb, dstate, 2 * nt * sizeof(int), hipMemcpyDeviceToHost, s));
    HODLR_HIP(hipStreamSynchronize(s));
    join.synced = pin_guard.synced = true;
    const int* hp = pin_rb;
    std::copy(hp, hp + nt, state.begin());
    std::copy(hp + nt, hp + 2 * nt, kused.begin());
    return HODLR_OK;
  };
  HODLR_TRY(queue(0, std::min(kFirstBatch, kLearnedAttempts)));
  HODLR_TRY(read_back());
  if (std::any_of(state.begin(), state.end(), [](int v) { return v == 0; }) && kFirstBatch < kLearnedAttempts) {
    HODLR_TRY(queue(kFirstBatch, kLearnedAttempts));
    HODLR_TRY(read_back());
  }
  std::vector<int> nodes;
  for (int x = 0; x < nt; ++x)
    if (state[x] == 2) nodes.push_back(tasks[x].node);
  if (!nodes.empty()) {
    join.synced = pin_guard.synced = false;
    // fallback: ACA on the failed blocks into panels of their own; the block
    // keeps whichever of the two approximations has the smaller estimate
    int C = 0;
    for (int q = 0; q < tr.L; ++q) C = std::max(C, capoff[q] + cap[q]);
    DevBuf U2, V2, rank2, skip2, err2, pos2, part2;
    {
      constexpr int G = (SKEL + kSkelSamples - 1) / kSkelSamples + 1;
      HODLR_TRY(pos2.ensure((size_t)nt * G * 2 * kSkelSamples * sizeof(int)));
      HODLR_TRY(part2.ensure((size_t)nt * G * sc.nch * 2 * sizeof(double)));
    }
    HODLR_TRY(U2.ensure((size_t)tr.n * C * sizeof(T)));
    HODLR_TRY(V2.ensure((size_t)tr.n * C * sizeof(T)));
    HODLR_TRY(rank2.ensure((size_t)nt * sizeof(int)));
    HODLR_TRY(skip2.ensure((size_t)nt * sizeof(int)));
    HODLR_TRY(err2.ensure((size_t)nt * sizeof(double)));
    HODLR_HIP(hipMemsetAsync(U2.p, 0, (size_t)tr.n * C * sizeof(T), s));
    HODLR_HIP(hipMemsetAsync(V2.p, 0, (size_t)tr.n * C * sizeof(T), s));
    HODLR_TRY(launch_aca(h, K, ldk, U2.p, V2.p, capoff, cap, s, &nodes));
    k_fallback_prep<<<g1, kBlock, 0, s>>>(sc.tasks.as<BdlrTask>(), nt, dstate, h->d_rank.as<int>(),
                                          rank2.as<int>(), skip2.as<int>());
    HODLR_HIP(hipGetLastError());
    // both candidates measured on the same positions: the skeleton's last
    // picks (exactly) and 16 fresh samples per side outside them (stream
    // attempt kLearnedAttempts, scaled); a sample of the whole block alone
    // would favour ACA, whose error gathers near the boundary the picks cover
    k_draw_samples<<<nt, 64, 0, s>>>(sc.tasks.as<BdlrTask>(), sc.sel.as<int>(), sc.cnt.as<int>(), SKEL, seed,
                                     kLearnedAttempts, kSkelSamples, sc.samp.as<int>(), skip2.as<int>());
    HODLR_HIP(hipGetLastError());
    constexpr int G = (SKEL + kSkelSamples - 1) / kSkelSamples + 1;
    k_cand_positions<<<nt, 256, 0, s>>>(sc.tasks.as<BdlrTask>(), nt, sc.sel.as<int>(), sc.cnt.as<int>(), SKEL,
                                        sc.samp.as<int>(), G, skip2.as<int>(), pos2.as<int>());
    HODLR_HIP(hipGetLastError());
    {
      ProfScope prof("skel_check", s);
      for (int cand = 0; cand < 2; ++cand) {
        k_skel_check<T><<<dim3(nt, sc.nch, G), kBlock, 0, s>>>(
            K, ldk, sc.tasks.as<BdlrTask>(), cand ? rank2.as<int>() : sc.rt.as<int>(), cand ? U2.as<T>() : Ucap,
            cand ? V2.as<T>() : Vcap, tr.n, pos2.as<int>(), kSkelSamples, part2.as<double>(), skip2.as<int>());
        k_cand_err<<<g1, kBlock, 0, s>>>(sc.tasks.as<BdlrTask>(), nt, sc.cnt.as<int>(), sc.norm.as<double>(),
                                         pos2.as<int>(), G, part2.as<double>(), sc.nch, skip2.as<int>(),
                                         cand ? err2.as<double>() : sc.err.as<double>());
      }
    }
    HODLR_HIP(hipGetLastError());
    k_fallback_choose<T><<<dim3(nt, 8), kBlock, 0, s>>>(sc.tasks.as<BdlrTask>(), dstate,
                                                        sc.err.as<double>(), err2.as<double>(), sc.rt.as<int>(),
                                                        U2.as<T>(), V2.as<T>(), Ucap, Vcap, tr.n,
                                                        h->d_rank.as<int>(), dkused);
    HODLR_HIP(hipGetLastError());
    HODLR_HIP(hipMemcpyAsync(kused.data(), dkused, nt * sizeof(int), hipMemcpyDeviceToHost, s));
    HODLR_HIP(hipStreamSynchronize(s));
  }
  h->skel_k.assign(tr.nnodes(), -1);
  for (int x = 0; x < nt; ++x) h->skel_k[tasks[x].node] = kused[x];
  // the stream (joined with the side stream) was synchronized above, so no
  // queued work reads the scratch: it goes back to the allocator at once,
  // without an event per buffer
  for (DevBuf* b : {&d_feat, &d_score, &d_dcnt, &d_budget, &d_state, &d_blk}) b->release();
  for (DevBuf* b : {&sc.tasks, &sc.sel, &sc.piv, &sc.cnt, &sc.rt, &sc.inv, &sc.cg, &sc.samp, &sc.err, &sc.norm,
                    &sc.part})
    b->release();
  return HODLR_OK;
}

// BDLR with the error monitor of Sec. 5.3: every block starts at the handle's
// depth; a block whose sampled error is above accept takes one more distance
// layer, up to max_depth (or until its picks stop growing).  A block that
// never passes keeps its deepest skeleton.  h->skel_k receives the depth each
// block ended at.
template <typename T, int SKEL>
static int adaptive_t(hodlr_s* h, const double* K, int ldk, const int* rowptr, const int* col, int max_depth,
                      int max_skel, unsigned long long seed, double accept, T* Ucap, T* Vcap,
                      const std::vector<int>& capoff, const std::vector<int>& cap, hipStream_t s) {
  const Tree& tr = h->tree;
  if (tr.n > 2 * kBdlrMaxSide) return fail(HODLR_EINVAL, "BDLR supports n <= 16384");
  size_t invo = 0, cgo = 0;
  std::vector<BdlrTask> tasks = make_tasks<T>(tr, capoff, cap, SKEL, &invo, &cgo);
  const int nt = (int)tasks.size(), selo = 2 * SKEL * nt;
  for (int x = 0; x < nt; ++x) tasks[x].task = x;
  int maxside = 0;
  for (auto& tk : tasks) maxside = std::max(maxside, std::max(tk.m, tk.nc));
  SkelScratch sc;
  HODLR_TRY(sc.ensure(nt, selo, invo, cgo, sizeof(T), check_chunks(tasks)));
  HODLR_TRY(block_norms(K, ldk, tasks, sc, s));
  HODLR_HIP(hipMemsetAsync(h->d_rank.p, 0, tr.nnodes() * sizeof(int), s));
  h->skel_k.assign(tr.nnodes(), -1);
  const int ms = max_skel > 0 ? std::min(max_skel, SKEL) : SKEL;
  std::vector<int> pending(nt), last(nt, -1);  // picks (rows + columns) of a block's previous attempt
  for (int x = 0; x < nt; ++x) pending[x] = x;
  std::vector<double> err;
  std::vector<int> cnt;
  for (int depth = h->depth, attempt = 0;; ++depth, ++attempt) {
    std::vector<BdlrTask> sub;
    for (int x : pending) sub.push_back(tasks[x]);
    const int ns = (int)sub.size();
    HODLR_HIP(hipMemcpyAsync(sc.tasks.p, sub.data(), ns * sizeof(BdlrTask), hipMemcpyHostToDevice, s));
    {
      ProfScope prof("bdlr_select", s);
      k_bdlr_select<<<ns, kBlock, 0, s>>>(rowptr, col, sc.tasks.as<BdlrTask>(), depth, ms, SKEL, sc.sel.as<int>(),
                                          sc.cnt.as<int>());
    }
    HODLR_HIP(hipGetLastError());
    HODLR_TRY((skel_attempt<T, SKEL>(h, K, ldk, sub, maxside, sc, Ucap, Vcap, seed, attempt, err, cnt, s)));
    std::vector<int> next;
    for (int x = 0; x < ns; ++x) {
      const int b = pending[x], picks = cnt[2 * x] + cnt[2 * x + 1];
      h->skel_k[sub[x].node] = depth;
      // a block stops when it passes, or when one more layer added no pick
      // (its picks are capped or cover both sides)
      if (err[x] > accept && picks > last[b]) next.push_back(b);
      last[b] = picks;
    }
    pending.swap(next);
    if (pending.empty() || depth >= max_depth) break;
  }
  HODLR_HIP(hipStreamSynchronize(s));  // scratch goes back to the allocator cache
  return HODLR_OK;
}

int launch_bdlr_adaptive(hodlr_s* h, const double* K, int ldk, const int* rowptr, const int* col, int max_depth,
                         int max_skel, unsigned long long seed, double accept, void* Ucap, void* Vcap,
                         const std::vector<int>& capoff, const std::vector<int>& cap, hipStream_t s) {
  if (h->precision == 64)
    return adaptive_t<double, kSkel64>(h, K, ldk, rowptr, col, max_depth, max_skel, seed, accept,
                                       static_cast<double*>(Ucap), static_cast<double*>(Vcap), capoff, cap, s);
  return adaptive_t<float, kSkel32>(h, K, ldk, rowptr, col, max_depth, max_skel, seed, accept,
                                    static_cast<float*>(Ucap), static_cast<float*>(Vcap), capoff, cap, s);
}

int launch_learned(hodlr_s* h, const double* K, int ldk, const int* rowptr, const int* col, const float* xyz,
                   const float* params, int kinit, unsigned long long seed, double accept, void* Ucap, void* Vcap,
                   const std::vector<int>& capoff, const std::vector<int>& cap, hipStream_t s) {
  if (h->precision == 64)
    return learned_t<double, kSkel64>(h, K, ldk, rowptr, col, xyz, params, kinit, seed, accept,
                                      static_cast<double*>(Ucap), static_cast<double*>(Vcap), capoff, cap, s);
  return learned_t<float, kSkel32>(h, K, ldk, rowptr, col, xyz, params, kinit, seed, accept,
                                   static_cast<float*>(Ucap), static_cast<float*>(Vcap), capoff, cap, s);
}

int launch_bdlr(hodlr_s* h, const double* K, int ldk, const int* rowptr, const int* col, void* Ucap,
                void* Vcap, const std::vector<int>& capoff, const std::vector<int>& cap, hipStream_t s,
                int max_skel, int* piv_export) {
  if (h->precision == 64)
    return bdlr_t<double, kSkel64>(h, K, ldk, rowptr, col, static_cast<double*>(Ucap),
                                   static_cast<double*>(Vcap), capoff, cap, s, max_skel, piv_export);
  return bdlr_t<float, kSkel32>(h, K, ldk, rowptr, col, static_cast<float*>(Ucap),
                                static_cast<float*>(Vcap), capoff, cap, s, max_skel, piv_export);
}

int skel_stride(int precision) { return precision == 64 ? kSkel64 : kSkel32; }

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
  k_bdlr_select<<<nt, kBlock, 0, stream>>>(g_rowptr, g_col, d_tasks.as<BdlrTask>(), depth, max_skel, max_skel,
                                           picks, counts);
  HODLR_HIP(hipGetLastError());
  HODLR_HIP(hipStreamSynchronize(stream));  // the task table goes back to the allocator cache
  return HODLR_OK;
}

namespace {
// The sampled error check of the learned and adaptive builds on given
// factors (hodlr_sampled_error): block norms, draws, residuals, estimates.
template <typename T>
int sampled_error_t(const double* K, int ldk, const Tree& tr, const T* U, const T* V, const int* ranks,
                    const int* rcols, const int* picks, const int* counts, int max_skel, unsigned long long seed,
                    int attempt, int* samples, double* err, hipStream_t s) {
  std::vector<int> capoff(tr.L), cap(rcols, rcols + tr.L);
  for (int q = 0, o = 0; q < tr.L; o += rcols[q], ++q) capoff[q] = o;
  size_t invo = 0, cgo = 0;
  std::vector<BdlrTask> tasks = make_tasks<T>(tr, capoff, cap, max_skel, &invo, &cgo);
  const int nt = (int)tasks.size();
  for (int x = 0; x < nt; ++x) tasks[x].task = x;
  SkelScratch sc;
  HODLR_TRY(sc.tasks.ensure(nt * sizeof(BdlrTask)));
  HODLR_TRY(sc.rt.ensure(nt * sizeof(int)));
  const int nch = check_chunks(tasks);
  HODLR_TRY(sc.part.ensure((size_t)nt * nch * 2 * sizeof(double)));
  HODLR_HIP(hipMemcpyAsync(sc.rt.p, ranks, nt * sizeof(int), hipMemcpyHostToDevice, s));
  HODLR_TRY(block_norms(K, ldk, tasks, sc, s));
  k_draw_samples<<<nt, 64, 0, s>>>(sc.tasks.as<BdlrTask>(), picks, counts, max_skel, seed, attempt, kSkelSamples,
                                   samples, nullptr);
  HODLR_HIP(hipGetLastError());
  k_skel_check<T><<<dim3(nt, nch), kBlock, 0, s>>>(K, ldk, sc.tasks.as<BdlrTask>(), sc.rt.as<int>(), U, V,
                                                             tr.n, samples, kSkelSamples, sc.part.as<double>(),
                                                             nullptr);
  HODLR_HIP(hipGetLastError());
  k_skel_err<<<(nt + kBlock - 1) / kBlock, kBlock, 0, s>>>(sc.tasks.as<BdlrTask>(), nt, counts, sc.norm.as<double>(),
                                                          samples, kSkelSamples, sc.part.as<double>(), nch, err,
                                                          nullptr);
  HODLR_HIP(hipGetLastError());
  HODLR_HIP(hipStreamSynchronize(s));  // the scratch goes back to the allocator cache
  return HODLR_OK;
}
}  // namespace

extern "C" int hodlr_sampled_error(const double* K, int n, int ldk, int leaf, int precision, const void* Upanel,
                                   const void* Vpanel, const int* ranks, const int* rcols, const int* picks,
                                   const int* counts, int max_skel, unsigned long long seed, int attempt,
                                   int* samples, double* err, hipStream_t stream) {
  if (n < 2 || n > 2 * kBdlrMaxSide) return fail(HODLR_EINVAL, "n must be in [2, 16384]");
  if (leaf < 1 || leaf > kLeafMax) return fail(HODLR_EINVAL, "leaf out of range");
  if (ldk < n) return fail(HODLR_EINVAL, "ldk < n");
  if (precision != 32 && precision != 64) return fail(HODLR_EINVAL, "precision must be 32 or 64");
  if (!K || !Upanel || !Vpanel || !ranks || !rcols || !picks || !counts || !samples || !err)
    return fail(HODLR_EINVAL, "NULL pointer argument");
  if (attempt < 0) return fail(HODLR_EINVAL, "attempt must be >= 0");
  const int skel = skel_stride(precision);
  if (max_skel < 1 || max_skel > skel) return fail(HODLR_EINVAL, "max_skel must be in [1, 192 / 128]");
  Tree tr;
  tr.build(n, leaf);
  if (tr.L == 0) return fail(HODLR_EINVAL, "n <= leaf: the tree has no off-diagonal blocks");
  const int rc = rank_cap(precision);
  for (int q = 1, x = 0; q <= tr.L; ++q) {
    if (rcols[q - 1] < 0 || rcols[q - 1] > rc) return fail(HODLR_EINVAL, "rcols out of range");
    for (int i = 0; i < (1 << q); ++i, ++x)
      if (ranks[x] < 0 || ranks[x] > rcols[q - 1]) return fail(HODLR_EINVAL, "rank above its level's width");
  }
  if (precision == 64)
    return sampled_error_t<double>(K, ldk, tr, static_cast<const double*>(Upanel),
                                   static_cast<const double*>(Vpanel), ranks, rcols, picks, counts, max_skel, seed,
                                   attempt, samples, err, stream);
  return sampled_error_t<float>(K, ldk, tr, static_cast<const float*>(Upanel), static_cast<const float*>(Vpanel),
                                ranks, rcols, picks, counts, max_skel, seed, attempt, samples, err, stream);
}
