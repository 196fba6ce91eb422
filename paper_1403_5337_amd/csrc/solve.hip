// HODLR solve x = Ktilde^-1 b (Sec. 4.3.2) for few right-hand sides, fused
// into L + 1 launches: the GMRES preconditioner.
//
// The factorization leaves, per node c of level q with parent P = (a, b),
//   E_c = d_c S_P^-1(rows of y that multiply d_c, :)        (|c| x (r_a + r_b))
// so the level-q step of the solve is  x_c -= E_c t_P  with
//   t_P = [V_b^T x_a; V_a^T x_b] = [W(rows a)^T x_a; W(rows b)^T x_b],
// (eq. y followed by the back-substitution of Sec. 4.2, applied from the
// leaves up as in Sec. 4.3.2).
//
// Rows are processed in units of kRows = 64 rows, one workgroup per unit.
// Launch "leaf" computes x = Kinv_leaf x for its unit; launch "level q"
// applies x -= E t_P to its unit.  Both then form the unit's partial products
// W(unit rows, block of the next level)^T x into one slot per unit.  The next
// launch reads the slots of its parent's two children along with its other
// loads.  Where those reads would be large (wide blocks of many units), a
// small launch in between first adds each node's slots into its first slot
// (k_sum_units, a fixed summation order), and the next launch reads one slot
// per child.
//
// Every workgroup issues its HBM reads together: the operand columns (E or the
// leaf inverse, then W) go to LDS by asynchronous global-to-LDS copies while
// the right-hand side and the group sums are read into registers.  The
// contraction over the rank splits the rank range across 4 waves per column
// group (one row per lane), or across all 16 waves for a single right-hand
// column, and adds the parts in order at the end.
#include <algorithm>

#include "device_util.h"
#include "hodlr_internal.h"

namespace hodlr {

constexpr int kRows = 64;        // rows per unit
constexpr int kSolveThreads = 1024;  // 16 waves: four per SIMD
// The 16 waves of a unit split a contraction into kZP parts of the rank (or
// row) range times kGroups column groups of kC columns: 4 x 4 for blocks of
// 4 or more right-hand columns, all 16 waves on the range for one column.
template <int SM>
struct SolveSplit {
  static constexpr int kZP = SM >= 4 ? 4 : 16 / SM;
  static constexpr int kGroups = 16 / kZP;
  static constexpr int kC = SM / kGroups;
  static_assert(kZP * kGroups == 16 && kC * kGroups == SM, "16 waves");
};
// alignment of a wave's kC consecutive columns in an [z][SM] block
template <typename T, int SM>
constexpr int split_align() { return SolveSplit<SM>::kC * sizeof(T) >= 8 ? 8 : (int)sizeof(T); }
constexpr int kLdW = kRows + 1;  // LDS column stride of staged W columns (read across columns)
// LDS column stride of the staged E / leaf-inverse columns (read 4 rows at a
// time, so 16-byte aligned)
template <typename T> constexpr int lda_lds() { return sizeof(T) == 4 ? kRows + 4 : kRows + 2; }

template <typename T> struct SolveCfg;
// kArena: operand columns staged at once; kT: rows of the right-hand block
// (>= 2 x rank cap, >= leaf cap, >= 256 for the cross-wave sums)
template <> struct SolveCfg<float> { static constexpr int kArena = 480, kT = 2 * kRankCap32; };
template <> struct SolveCfg<double> { static constexpr int kArena = 224, kT = 2 * kRankCap64; };

// Operand columns staged at once.  A single right-hand column leaves room for
// more of them (the widest float level, 2 x 184 E columns plus the parent's
// 184 W columns, then stages in one round).
template <typename T, int SM>
constexpr int arena_cols() { return sizeof(T) == 4 && SM == 1 ? 560 : SolveCfg<T>::kArena; }

template <typename T, int SM>
struct SolveSmem {
  alignas(16) T arena[arena_cols<T, SM>() * lda_lds<T>()];  // staged operand columns
  // right-hand block (z x SM), then the waves' partial sums (kZP x SM x 64)
  alignas(16) T tb[SolveCfg<T>::kT * SM > SolveSplit<SM>::kZP * SM * kRows ? SolveCfg<T>::kT * SM
                                                                          : SolveSplit<SM>::kZP * SM * kRows];
  alignas(16) T xs[kRows * SM];                 // x of the unit (i x SM)
};

// Asynchronous copy of columns [0, cn) of a 64-row column-major panel (first
// row at src, leading dimension ld; rows >= rn are not read) into LDS columns
// dst + c * ldl.  One wave instruction moves 256 bytes of one column; the
// copies complete at dma_wait().
template <typename T>
__device__ __forceinline__ void dma_columns(T* dst, int ldl, const T* __restrict__ src, size_t ld, int rn, int cn) {
  constexpr int kParts = sizeof(T) / 4;
  constexpr int kRowsPart = kRows / kParts;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int row = lane / kParts;
  for (int j = wave; j < cn * kParts; j += nw) {
    const int c = j / kParts, p = j - c * kParts;
    if (p * kRowsPart + row < rn) {
      const char* g = reinterpret_cast<const char*>(src + (size_t)c * ld + p * kRowsPart) + lane * 4;
      __builtin_amdgcn_global_load_lds((gptr_t)g, (lptr_t)(dst + c * ldl + p * kRowsPart), 4, 0, 0);
    }
  }
}

// Stage operand columns [j0, j0 + jn) of the stream "A columns 0..ra-1, then
// W columns 0..": A and W are 64-row panels (first row at A / Wp).  In the
// arena the chunk's A columns come first (stride lda_lds), then its W
// columns (stride kLdW).
template <typename T>
__device__ __forceinline__ void stage_stream(T* arena, const T* A, size_t lda, int ra, const T* Wp, size_t ldw,
                                             int j0, int jn, int rn) {
  const int j1 = j0 + jn;
  if (j0 < ra) dma_columns(arena, lda_lds<T>(), A + (size_t)j0 * lda, lda, rn, min(j1, ra) - j0);
  if (j1 > ra) {
    const int w0 = max(j0, ra);
    dma_columns(arena + (w0 - j0) * lda_lds<T>(), kLdW, Wp + (size_t)(w0 - ra) * ldw, ldw, rn, j1 - w0);
  }
}

// acc[cj] += sum_z A(lane, z - a0) B(z, cb + cj) over this wave's share of
// [z0, z1): wave w takes part w % kZP of the range and the column group
// cb = (w / kZP) kC.  A in LDS with column stride lda_lds, B in LDS as
// [z][SM].  The loads of kU consecutive z are issued together; the sum runs
// in z order.
template <typename T, int SM>
__device__ __forceinline__ void contract(const T* A, int a0, const T* B, int z0, int z1,
                                         T (&acc)[SolveSplit<SM>::kC]) {
  constexpr int kC = SolveSplit<SM>::kC, kZP = SolveSplit<SM>::kZP, kU = 8, kL = lda_lds<T>();
  constexpr int kAl = split_align<T, SM>();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int zp = wave % kZP, cb = (wave / kZP) * kC;
  const int per = (z1 - z0 + kZP - 1) / kZP;
  const int zb = z0 + zp * per, ze = min(z1, zb + per);
  int z = zb;
  for (; z + kU <= ze; z += kU) {
    T a[kU], b[kU][kC];
#pragma unroll
    for (int k = 0; k < kU; ++k) {
      a[k] = A[(z + k - a0) * kL + lane];
      const T* bp = static_cast<const T*>(__builtin_assume_aligned(B + (z + k) * SM + cb, kAl));
#pragma unroll
      for (int cj = 0; cj < kC; ++cj) b[k][cj] = bp[cj];
    }
#pragma unroll
    for (int k = 0; k < kU; ++k)
#pragma unroll
      for (int cj = 0; cj < kC; ++cj) acc[cj] += a[k] * b[k][cj];
  }
  for (; z < ze; ++z) {
    const T a = A[(z - a0) * kL + lane];
    const T* bp = static_cast<const T*>(__builtin_assume_aligned(B + z * SM + cb, kAl));
#pragma unroll
    for (int cj = 0; cj < kC; ++cj) acc[cj] += a * bp[cj];
  }
}

// x(i, c) = xr - (sum of the kZP rank parts, in order) (sub) or the sum itself;
// written to Xout (rows i < rn, c < nc) and to xs (zero elsewhere).  Thread
// (lane, wave) finishes row lane of column wave (waves >= SM idle here).
template <typename T, int SM>
__device__ __forceinline__ void finalize_x(SolveSmem<T, SM>& sm, const T (&acc)[SolveSplit<SM>::kC], T xr,
                                           bool sub, int rn, int nc, T* Xout, size_t ldxo) {
  constexpr int kC = SolveSplit<SM>::kC, kZP = SolveSplit<SM>::kZP;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int zp = wave % kZP, cb = (wave / kZP) * kC;
  __syncthreads();  // every wave is done with tb
#pragma unroll
  for (int cj = 0; cj < kC; ++cj) sm.tb[(zp * SM + cb + cj) * kRows + lane] = acc[cj];
  __syncthreads();
  if (wave < SM) {
    const int c = wave;
    T s = sm.tb[c * kRows + lane];
#pragma unroll
    for (int p = 1; p < kZP; ++p) s += sm.tb[(p * SM + c) * kRows + lane];
    const bool ok = lane < rn && c < nc;
    const T v = ok ? (sub ? xr - s : s) : T(0);
    if (ok) Xout[(size_t)c * ldxo + lane] = v;
    sm.xs[lane * SM + c] = v;
  }
  __syncthreads();
}

// Pu(r0 + r, c) = sum_{i < rn} Wl(i, r) xs(i, c) for r < nw, c < nc (Pu has
// leading dimension rp); Wl in LDS with column stride kLdW.  Lane = r.  Per
// 64-column block of Wl the 16 waves split as kZP row parts x kGroups column
// groups of kC; the parts are added in order through red (LDS,
// kZP x SM x 64).
template <typename T, int SM>
__device__ __forceinline__ void unit_partials(const T* Wl, T* red, const T* xs, int rn, int nw, int nc, T* Pu,
                                              int r0, int rp) {
  constexpr int kC = SolveSplit<SM>::kC, kZP = SolveSplit<SM>::kZP, kU = 4;
  constexpr int kAl = split_align<T, SM>();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int part = wave % kZP, cb = (wave / kZP) * kC;
  const int per = ((rn + kZP - 1) / kZP + kU - 1) / kU * kU;
  const int i0 = part * per, i1 = min(rn, i0 + per);
  for (int b0 = 0; b0 < nw; b0 += 64) {
    const int r = b0 + lane, rc = min(r, nw - 1);
    const T* wc = Wl + rc * kLdW;
    T acc[kC];
#pragma unroll
    for (int cj = 0; cj < kC; ++cj) acc[cj] = T(0);
    int i = i0;
    for (; i + kU <= i1; i += kU) {
      T w[kU], x[kU][kC];
#pragma unroll
      for (int k = 0; k < kU; ++k) {
        w[k] = wc[i + k];
        const T* xp = static_cast<const T*>(__builtin_assume_aligned(xs + (i + k) * SM + cb, kAl));
#pragma unroll
        for (int cj = 0; cj < kC; ++cj) x[k][cj] = xp[cj];
      }
#pragma unroll
      for (int k = 0; k < kU; ++k)
#pragma unroll
        for (int cj = 0; cj < kC; ++cj) acc[cj] += w[k] * x[k][cj];
    }
    for (; i < i1; ++i) {
      const T w = wc[i];
      const T* xp = static_cast<const T*>(__builtin_assume_aligned(xs + i * SM + cb, kAl));
#pragma unroll
      for (int cj = 0; cj < kC; ++cj) acc[cj] += w * xp[cj];
    }
#pragma unroll
    for (int cj = 0; cj < kC; ++cj) red[(part * SM + cb + cj) * 64 + lane] = acc[cj];
    __syncthreads();
    if (wave < SM) {
      const int c = wave;
      T v = red[c * 64 + lane];
#pragma unroll
      for (int p = 1; p < kZP; ++p) v += red[(p * SM + c) * 64 + lane];
      if (r < nw && c < nc) Pu[(size_t)(r0 + r) + (size_t)c * rp] = v;
    }
    __syncthreads();
  }
}

// P holds nnodes x upn slots of usz elements; slot 0 of each node receives
// the sum of the node's upn slots.  kLanes consecutive lanes share an
// element: lane j adds units j, j + kLanes, ... in order, then the lanes are
// combined by a fixed butterfly, so the result does not depend on timing.
constexpr int kSumLanes = 8;

template <typename T>
__global__ void __launch_bounds__(kBlock) k_sum_units(T* __restrict__ P, int nnodes, int upn, int usz) {
  const long gid = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long el = gid / kSumLanes;
  const int j = (int)(gid % kSumLanes);
  const bool live = el < (long)nnodes * usz;
  const int node = live ? (int)(el / usz) : 0, e = live ? (int)(el % usz) : 0;
  T* base = P + (size_t)node * upn * usz + e;
  T s = T(0);
  if (live) {
    int u = j;
    for (; u + 3 * kSumLanes < upn; u += 4 * kSumLanes) {
      T v[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) v[k] = base[(size_t)(u + k * kSumLanes) * usz];
#pragma unroll
      for (int k = 0; k < 4; ++k) s += v[k];
    }
    for (; u < upn; u += kSumLanes) s += base[(size_t)u * usz];
  }
#pragma unroll
  for (int o = 1; o < kSumLanes; o <<= 1) s += __shfl_xor(s, o, 64);
  if (live && j == 0) base[0] = s;
}

// The unit's pipeline after its right-hand block is in sm.tb: stream the
// operand columns (A: ra columns, then W: nwc columns), contract, form x, and
// the partial products of W.
template <typename T, int SM>
__device__ __forceinline__ void unit_pipeline(SolveSmem<T, SM>& sm, const T* A, size_t lda, int ra, const T* Wp,
                                              size_t ldw, int nwc, int rn, int nc, T xr, bool sub,
                                              T* Xout, size_t ldxo, T* Pu, int rp, int jn) {
  constexpr int kA = arena_cols<T, SM>();
  const int total = ra + nwc;
  T acc[SolveSplit<SM>::kC];
#pragma unroll
  for (int cj = 0; cj < SolveSplit<SM>::kC; ++cj) acc[cj] = T(0);
  bool done = false;
  for (int j0 = 0;;) {
    dma_wait();
    const int j1 = j0 + jn;
    if (j0 < ra) contract<T, SM>(sm.arena, j0, sm.tb, j0, min(j1, ra), acc);
    if (!done && ra <= j1) {
      finalize_x<T, SM>(sm, acc, xr, sub, rn, nc, Xout, ldxo);
      done = true;
    }
    if (j1 > ra) {
      const int w0 = max(j0, ra);
      unit_partials<T, SM>(sm.arena + (w0 - j0) * lda_lds<T>(), sm.tb, sm.xs, rn, j1 - w0, nc, Pu, w0 - ra, rp);
    }
    if (j1 >= total) break;
    __syncthreads();  // the arena is reused
    j0 = j1;
    jn = min(kA, total - j0);
    stage_stream(sm.arena, A, lda, ra, Wp, ldw, j0, jn, rn);
  }
}

template <typename T, int SM>
__global__ void __launch_bounds__(kSolveThreads)
    k_solve_leaf(const T* __restrict__ Kinv, int bmax, const int* __restrict__ lo, const int* __restrict__ hi,
                 int idL, const T* __restrict__ Xin, int ldxi, T* __restrict__ Xout, int ldxo, int nc,
                 const T* __restrict__ W, int ldw, int offL, int rL, int nchL, T* __restrict__ P,
                 const int* __restrict__ gate) {
  if (gate_closed(gate, nc)) return;
  __shared__ SolveSmem<T, SM> sm;
  const int leaf = blockIdx.x, ch = blockIdx.y, id = idL + leaf, t = threadIdx.x;
  const int l0 = lo[id], b = hi[id] - l0, row0 = ch * kRows, rn = min(kRows, b - row0);
  const int flat = leaf * nchL + ch;
  T* Pu = P ? P + (size_t)flat * rL * nc : nullptr;
  if (rn <= 0) {
    if (Pu)
      for (int e = t; e < rL * nc; e += blockDim.x) Pu[e] = T(0);
    return;
  }
  const T* Ki = Kinv + (size_t)leaf * bmax * bmax + row0;
  const T* Wu = W + (size_t)offL * ldw + l0 + row0;
  const int nwc = Pu ? rL : 0;
  const int jn = min(arena_cols<T, SM>(), b + nwc);
  stage_stream(sm.arena, Ki, (size_t)bmax, b, Wu, (size_t)ldw, 0, jn, rn);
  // right-hand block: the leaf's rows of x, as [k][SM]
  for (int e0 = 0; e0 < b * SM; e0 += 4 * kSolveThreads) {
    T v[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      const int e = e0 + t + a * kSolveThreads, k = e % b, c = e / b;
      v[a] = (e < b * SM && c < nc) ? Xin[(size_t)c * ldxi + l0 + k] : T(0);
    }
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      const int e = e0 + t + a * kSolveThreads;
      if (e < b * SM) sm.tb[(e % b) * SM + e / b] = v[a];
    }
  }
  unit_pipeline<T, SM>(sm, Ki, (size_t)bmax, b, Wu, (size_t)ldw, nwc, rn, nc, T(0), false,
                       Xout + l0 + row0, (size_t)ldxo, Pu, rL, jn);
}

template <typename T, int SM>
__global__ void __launch_bounds__(kSolveThreads)
    k_solve_level(int q, const int* __restrict__ lo, const int* __restrict__ hi, const int* __restrict__ rank,
                  const T* Xin, int ldxi, T* Xout, int ldxo, int nc, const T* __restrict__ E, int ldE, int offE,
                  int rq, const T* __restrict__ Pin, int upn, int gin, int nch, const T* __restrict__ W, int ldw,
                  int offp, int rp, T* __restrict__ Pout, const int* __restrict__ gate) {
  if (gate_closed(gate, nc)) return;
  __shared__ SolveSmem<T, SM> sm;
  const int c = blockIdx.x, ch = blockIdx.y, t = threadIdx.x;
  const int par = c >> 1, id = node_id(q, c);
  const int ra = rank[node_id(q, 2 * par)], rb = rank[node_id(q, 2 * par + 1)], r = ra + rb;
  const int row0 = lo[id] + ch * kRows, rn = min(kRows, hi[id] - row0);
  const int flat = c * nch + ch;
  T* Pu = Pout ? Pout + (size_t)flat * rp * nc : nullptr;
  if (rn <= 0) {
    if (Pu)
      for (int e = t; e < rp * nc; e += blockDim.x) Pu[e] = T(0);
    return;
  }
  const T* Eu = E + (size_t)offE * ldE + row0;
  const T* Wu = W + (size_t)offp * ldw + row0;
  const int nwc = Pu ? rp : 0;
  const int jn = min(arena_cols<T, SM>(), r + nwc);
  stage_stream(sm.arena, Eu, (size_t)ldE, r, Wu, (size_t)ldw, 0, jn, rn);
  // x of the unit: thread (lane, wave) holds row lane of column wave
  const int lane = t & 63, cw = t >> 6;
  const T xr = (lane < rn && cw < nc) ? Xin[(size_t)cw * ldxi + row0 + lane] : T(0);
  // t_P = [W(rows a)^T x_a (r_b entries); W(rows b)^T x_b (r_a entries)] from
  // the group sums of both children, as [z][SM]: entry e = z + r c (c < nc)
  // adds its ng slots in slot order with up to kJ loads in one round trip
  // (issued in batches of 4; a batch past the last slot is skipped, and the
  // addresses are clamped into range).  Columns c >= nc are zero.
  const size_t usz = (size_t)rq * nc, gstride = (size_t)gin * usz;
  const int ng = upn / gin;
  constexpr int kJ = sizeof(T) == 8 ? 16 : SM <= 8 ? 48 : 32;
  for (int e = t; e < r * SM; e += kSolveThreads) {
    const int z = e % r, cc = e / r;
    T sum = T(0);
    if (cc < nc) {
      const int node = (z < rb) ? 2 * par : 2 * par + 1, zz = (z < rb) ? z : z - rb;
      const T* p0 = Pin + (size_t)node * upn * usz + zz + (size_t)cc * rq;
      for (int j0 = 0; j0 < ng; j0 += kJ) {
        T v[kJ];
#pragma unroll
        for (int bq = 0; bq < kJ; bq += 4)
          if (j0 + bq < ng) {
#pragma unroll
            for (int j = bq; j < bq + 4; ++j) v[j] = p0[(size_t)min(j0 + j, ng - 1) * gstride];
          }
#pragma unroll
        for (int j = 0; j < kJ; ++j)
          if (j0 + j < ng) sum += v[j];
      }
    }
    sm.tb[z * SM + cc] = sum;
  }
  unit_pipeline<T, SM>(sm, Eu, (size_t)ldE, r, Wu, (size_t)ldw, nwc, rn, nc, xr, true, Xout + row0,
                       (size_t)ldxo, Pu, rp, jn);
}

// ---------------------------------------------------------------------------
static inline int cdiv(int a, int b) { return (a + b - 1) / b; }

// Units per level-q node: q = L -> its own units; q < L -> its children's.
static int units_per_node(const Tree& t, int q) {
  return q == t.L ? cdiv(t.max_size(t.L), kRows) : 2 * cdiv(t.max_size(q + 1), kRows);
}

// A level-q workgroup reads the upn slots of both children of its parent.
// While those reads stay within kDirectBytes they ride along with the unit's
// other loads; beyond that k_sum_units first adds each node's slots (one more
// launch, one more round trip to memory).
constexpr size_t kDirectBytes = 96 * 1024;

static bool sum_first(const hodlr_s* h, int q, int nc) {
  return 2 * (size_t)h->rcols[q - 1] * nc * units_per_node(h->tree, q) * h->esize > kDirectBytes;
}

size_t solve_partial_elems(const hodlr_s* h) {
  const Tree& t = h->tree;
  size_t mx = 1;
  for (int q = 1; q <= t.L; ++q) {
    const size_t rq = h->rcols[q - 1];
    const size_t units = ((size_t)1 << q) * units_per_node(t, q);
    mx = std::max(mx, units * rq * 16);
  }
  return mx;
}

template <typename T, int SM>
static int solve_t(hodlr_s* h, T* X, int ldx, int nc, hipStream_t s, const int* gate) {
  const Tree& t = h->tree;
  const int n = t.n, L = t.L;
  T* P[2] = {h->G.as<T>(), h->G.as<T>() + h->p_half};
  T* Xt = h->Xtmp.as<T>();
  const int rL = L > 0 ? h->rcols[L - 1] : 0, offL = L > 0 ? h->off[L - 1] : 0;
  const int nchL = cdiv(h->bmax, kRows);
  {
    ProfScope prof_("apply_leaf", s);
    k_solve_leaf<T, SM><<<dim3(h->nleaf, nchL), kSolveThreads, 0, s>>>(
        h->Kinv.as<T>(), h->bmax, h->d_lo.as<int>(), h->d_hi.as<int>(), node_id(L, 0), X, ldx, Xt, n, nc,
        h->W.as<T>(), n, offL, rL, nchL, L > 0 ? P[0] : nullptr, gate);
  }
  HODLR_HIP(hipGetLastError());
  int cur = 0;
  for (int q = L; q >= 1; --q) {
    const int rq = h->rcols[q - 1];
    const int nch = cdiv(t.max_size(q), kRows);
    const int rp = q > 1 ? h->rcols[q - 2] : 0, offp = q > 1 ? h->off[q - 2] : 0;
    T* Xo = (q == 1) ? X : Xt;
    const int ldo = (q == 1) ? ldx : n;
    const int upn = units_per_node(t, q);
    int gin = 1;
    if (sum_first(h, q, nc)) {
      const long threads = (long)(1 << q) * rq * nc * kSumLanes;
      {
        ProfScope prof_("apply_sum", s);
        k_sum_units<T><<<(int)((threads + kBlock - 1) / kBlock), kBlock, 0, s>>>(P[cur], 1 << q, upn, rq * nc);
      }
      HODLR_HIP(hipGetLastError());
      gin = upn;
    }
    {
      ProfScope prof_("apply_level", s);
      k_solve_level<T, SM><<<dim3(1 << q, nch), kSolveThreads, 0, s>>>(
          q, h->d_lo.as<int>(), h->d_hi.as<int>(), h->d_rank.as<int>(), Xt, n, Xo, ldo, nc, h->E.as<T>(), n,
          h->offE[q - 1], rq, P[cur], upn, gin, nch, h->W.as<T>(), n, offp, rp, q > 1 ? P[cur ^ 1] : nullptr,
          gate);
    }
    HODLR_HIP(hipGetLastError());
    cur ^= 1;
  }
  if (L == 0)
    HODLR_HIP(hipMemcpy2DAsync(X, (size_t)ldx * sizeof(T), Xt, (size_t)n * sizeof(T), (size_t)n * sizeof(T),
                               nc, hipMemcpyDeviceToDevice, s));
  return HODLR_OK;
}

template <typename T>
static int apply_t(hodlr_s* h, T* X, int ldx, int nrhs, hipStream_t s, const int* gate) {
  for (int c0 = 0; c0 < nrhs; c0 += 16) {
    const int nc = std::min(16, nrhs - c0);
    T* Xc = X + (size_t)c0 * ldx;
    const int* g = gate ? gate + c0 : nullptr;  // this block's columns
    if (nc == 1) HODLR_TRY((solve_t<T, 1>(h, Xc, ldx, nc, s, g)));
    else if (nc <= 8) HODLR_TRY((solve_t<T, 8>(h, Xc, ldx, nc, s, g)));
    else HODLR_TRY((solve_t<T, 16>(h, Xc, ldx, nc, s, g)));
  }
  return HODLR_OK;
}

int apply_impl(hodlr_s* h, void* X, int ldx, int nrhs, hipStream_t s, const int* gate) {
  return h->precision == 64 ? apply_t<double>(h, static_cast<double*>(X), ldx, nrhs, s, gate)
                            : apply_t<float>(h, static_cast<float*>(X), ldx, nrhs, s, gate);
}

}  // namespace hodlr
