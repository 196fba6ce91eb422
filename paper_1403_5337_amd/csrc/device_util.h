// Device helpers shared by the kernels: reductions and in-LDS Gauss-Jordan.
#pragma once

#include <hip/hip_runtime.h>

#include <climits>

namespace hodlr {

template <typename T> __device__ __forceinline__ T dabs(T x) { return x < T(0) ? -x : x; }

// Keep the larger value; ties go to the lower index.  NaN never wins.
// Written without branches so that it compiles to compares and selects.
template <typename T>
__device__ __forceinline__ void argmax_merge(T& v, int& i, T v2, int i2) {
  const bool take = (v2 > v) | ((v2 == v) & (i2 < i));
  v = take ? v2 : v;
  i = take ? i2 : i;
}

template <typename T> __device__ __forceinline__ T wave_sum(T v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Block-wide argmax over (v, i); every thread gets the result.  sv/si hold
// at least blockDim.x / 64 entries.
template <typename T>
__device__ void block_argmax(T v, int i, T* sv, int* si, T& ov, int& oi) {
  for (int o = 32; o > 0; o >>= 1) {
    T v2 = __shfl_xor(v, o, 64);
    int i2 = __shfl_xor(i, o, 64);
    argmax_merge(v, i, v2, i2);
  }
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, nw = (blockDim.x + 63) >> 6;
  __syncthreads();
  if (lane == 0) {
    sv[w] = v;
    si[w] = i;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    T bv = sv[0];
    int bi = si[0];
    for (int k = 1; k < nw; ++k) argmax_merge(bv, bi, sv[k], si[k]);
    sv[0] = bv;
    si[0] = bi;
  }
  __syncthreads();
  ov = sv[0];
  oi = si[0];
  __syncthreads();
}

template <typename T> __device__ T block_sum(T v, T* sv) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, nw = (blockDim.x + 63) >> 6;
  __syncthreads();
  if (lane == 0) sv[w] = v;
  __syncthreads();
  T s = 0;
  for (int k = 0; k < nw; ++k) s += sv[k];
  __syncthreads();
  return s;
}

// ---------------------------------------------------------------------------
// Asynchronous global-to-LDS copies: each wave instruction moves 64 dwords
// (lane l takes dword l) to consecutive LDS addresses from a wave-uniform
// base.  They complete at dma_wait().
// ---------------------------------------------------------------------------
typedef __attribute__((address_space(1))) const void* gptr_t;
typedef __attribute__((address_space(3))) void* lptr_t;

// The calling wave copies count contiguous elements from src to LDS dst.
template <typename T>
__device__ __forceinline__ void dma_span(T* dst, const T* __restrict__ src, int count) {
  const int lane = threadIdx.x & 63;
  const int nd = count * (int)(sizeof(T) / 4);
  for (int d0 = 0; d0 < nd; d0 += 64)
    if (d0 + lane < nd)
      __builtin_amdgcn_global_load_lds((gptr_t)(reinterpret_cast<const char*>(src) + 4 * (d0 + lane)),
                                       (lptr_t)(reinterpret_cast<char*>(dst) + 4 * d0), 4, 0, 0);
}

__device__ __forceinline__ void dma_wait() {
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
}

// ---------------------------------------------------------------------------
// Cross-lane moves inside a wavefront through DPP (no LDS round trip).
// ---------------------------------------------------------------------------
template <int CTRL> __device__ __forceinline__ int dpp_move(int v) {
  return __builtin_amdgcn_mov_dpp(v, CTRL, 0xF, 0xF, true);
}
template <int CTRL> __device__ __forceinline__ float dpp_move(float v) {
  return __int_as_float(dpp_move<CTRL>(__float_as_int(v)));
}
template <int CTRL> __device__ __forceinline__ double dpp_move(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = dpp_move<CTRL>((int)(b & 0xffffffffll)), hi = dpp_move<CTRL>((int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__device__ __forceinline__ float lane_value(float x, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), l));
}
__device__ __forceinline__ double lane_value(double x, int l) {
  const long long v = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_readlane((int)(v & 0xffffffffll), l);
  const int hi = __builtin_amdgcn_readlane((int)(v >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Wave-wide argmax over (v, i), ties to the lower index; every lane gets the
// result.  Pairs lanes by xor 1 and xor 2 (quad permutes), then mirrors
// within 8 and 16 lanes (DPP), then xor 16 and xor 32.
template <typename T> __device__ __forceinline__ void wave_argmax(T& v, int& i) {
  argmax_merge(v, i, dpp_move<0xB1>(v), dpp_move<0xB1>(i));
  argmax_merge(v, i, dpp_move<0x4E>(v), dpp_move<0x4E>(i));
  argmax_merge(v, i, dpp_move<0x141>(v), dpp_move<0x141>(i));
  argmax_merge(v, i, dpp_move<0x140>(v), dpp_move<0x140>(i));
  argmax_merge(v, i, __shfl_xor(v, 16, 64), __shfl_xor(i, 16, 64));
  argmax_merge(v, i, __shfl_xor(v, 32, 64), __shfl_xor(i, 32, 64));
}

// The same argmax with a wave-uniform result and no LDS traffic: the four DPP
// stages leave every lane of a 16-lane row holding its row's result, and the
// four row results are read with readlane and merged in row order.
template <typename T> __device__ __forceinline__ void wave_argmax_uniform(T& v, int& i) {
  argmax_merge(v, i, dpp_move<0xB1>(v), dpp_move<0xB1>(i));
  argmax_merge(v, i, dpp_move<0x4E>(v), dpp_move<0x4E>(i));
  argmax_merge(v, i, dpp_move<0x141>(v), dpp_move<0x141>(i));
  argmax_merge(v, i, dpp_move<0x140>(v), dpp_move<0x140>(i));
  T bv = lane_value(v, 0);
  int bi = __builtin_amdgcn_readlane(i, 0);
#pragma unroll
  for (int r = 1; r < 4; ++r) argmax_merge(bv, bi, lane_value(v, 16 * r), __builtin_amdgcn_readlane(i, 16 * r));
  v = bv;
  i = bi;
}

// Row of the largest candidate cv[a] (row lane + 64 a), ties to the lowest
// row, and that candidate (best), both wave-uniform.  The maximum is reduced
// with DPP inside each 16-lane row and across the four rows by readlane;
// then the lowest row holding it comes from one ballot per register.  Returns
// -1 if no candidate equals the maximum (a NaN maximum).
template <typename T> __device__ __forceinline__ T sel_max(T a, T b) { return b > a ? b : a; }

template <typename T> __device__ __forceinline__ T wave_max(T m) {
  m = sel_max(m, dpp_move<0xB1>(m));
  m = sel_max(m, dpp_move<0x4E>(m));
  m = sel_max(m, dpp_move<0x141>(m));
  m = sel_max(m, dpp_move<0x140>(m));
  return sel_max(sel_max(lane_value(m, 0), lane_value(m, 16)), sel_max(lane_value(m, 32), lane_value(m, 48)));
}

template <typename T, int RA>
__device__ __forceinline__ int wave_argmax_rows(const T (&cv)[RA], T& best) {
  T m = cv[0];
#pragma unroll
  for (int a = 1; a < RA; ++a) m = sel_max(m, cv[a]);
  best = wave_max(m);
#pragma unroll
  for (int a = 0; a < RA; ++a) {
    const unsigned long long bal = __ballot(cv[a] == best);
    if (bal) return 64 * a + __ffsll((long long)bal) - 1;
  }
  return -1;
}

// ---------------------------------------------------------------------------
// Blocked Gauss-Jordan inversion with partial pivoting (gj_threads<T>() threads).
//
// The matrix sits in LDS.  Every kGjNb = 8 pivot steps form a block.  Wave 0
// factors the block's 8 columns (the panel) on its own, without barriers: the
// pivot of each step is the largest |entry| of the current column among the
// rows not yet used (ties to the lower row); the pivot row is scaled, the
// other rows are eliminated, and the column is replaced by the multipliers,
// which is the in-place Gauss-Jordan step.  The block's steps applied to any
// other column j amount to X(:, j) += C X_old(P, j), with P the block's pivot
// rows and C = Z - I(:, P) for the factored panel Z: one rank-8 update.
//
// Look-ahead: while waves 1-15 apply block b's update to the other columns
// (small tiles per thread), wave 0 applies it to the next panel's columns in
// its registers and factors that panel, so the updates run under the chain
// of pivot steps.  Rows are never swapped: with p_k the pivot row of step k
// the array ends as (P A)^-1, i.e. A^-1(r, c) = X(p_r, pinv(c)).
// ---------------------------------------------------------------------------
constexpr int kGjNb = 8;
// A single wave issues a VALU op only every ~8 cycles, so the tile updates
// need as many waves as a workgroup can hold to keep up with the panel wave;
// the kernels that invert hold the whole CU (LDS) anyway.  Double precision
// takes 8 waves, which leaves it 256 registers per lane.
template <typename T>
constexpr int gj_threads() {
  return sizeof(T) == 8 ? 512 : 1024;
}

template <typename T, int NMAX>
struct GjScratch {
  static constexpr int kLd = (NMAX + 7) / 8 * 8;  // column stride of X and C
  alignas(16) T X[NMAX * kLd];                    // the matrix, column-major
  alignas(16) T C[2][kGjNb * kLd];                // C = Z - I(:, P) of two blocks, column-major
  alignas(16) T R[NMAX * kGjNb];                  // pivot rows of the other columns, [j][s]
  int p[2][kGjNb];                                // pivot rows of two blocks
  int pinv[NMAX];                                 // step at which a row was the pivot row
  int prow[NMAX];                                 // pivot row of each step
  int bad;
};

// Wave 0: loads the panel X(:, k0 : k0 + nbk) into registers (rows of lane l
// are l + 64 a, a < RA), first applying the previous block's update (Cp, with
// the panel's pivot-row values at R[(jr + j) * kGjNb]) if Cp is not NULL,
// then runs the panel's pivot steps and stores Z, C and the pivots.  used:
// per lane, bit a = row used or beyond n.
template <typename T, int RA, int NMAX>
__device__ bool gj_panel(GjScratch<T, NMAX>& s, int n, int k0, int nbk, int buf, const T* Cp, int jr,
                         unsigned& used) {
  constexpr int ld = GjScratch<T, NMAX>::kLd;
  const int lane = threadIdx.x & 63;
  T P[RA][kGjNb];
#pragma unroll
  for (int a = 0; a < RA; ++a)
#pragma unroll
    for (int j = 0; j < kGjNb; ++j) {
      const int i = lane + 64 * a;
      P[a][j] = (i < n && j < nbk) ? s.X[(k0 + j) * ld + i] : T(0);
    }
  if (Cp) {
#pragma unroll
    for (int a = 0; a < RA; ++a) {
      const int i = min(lane + 64 * a, ld - 1);
      T c[kGjNb];
#pragma unroll
      for (int q = 0; q < kGjNb; ++q) c[q] = Cp[q * ld + i];
#pragma unroll
      for (int j = 0; j < kGjNb; ++j) {
        const T* rp = static_cast<const T*>(__builtin_assume_aligned(s.R + (jr + j) * kGjNb, 16));
#pragma unroll
        for (int q = 0; q < kGjNb; ++q) P[a][j] = fma(c[q], rp[q], P[a][j]);
      }
    }
  }
  int pv[kGjNb];
  bool ok = true;
  // pivot candidates of the current column
  T cv[RA];
#pragma unroll
  for (int a = 0; a < RA; ++a) cv[a] = ((used >> a) & 1u) ? T(-1) : fabs(P[a][0]);
#pragma unroll
  for (int j = 0; j < kGjNb; ++j) {
    pv[j] = -1;
    if (j >= nbk || !ok) continue;
    T bv;
    const int pr = __builtin_amdgcn_readfirstlane(wave_argmax_rows<T, RA>(cv, bv));
    if (pr < 0 || pr >= n || !(bv > T(0)) || !(bv < T(INFINITY))) {
      ok = false;
      continue;
    }
    const int pl = pr & 63, ap = pr >> 6;
    T rs[kGjNb];
#pragma unroll
    for (int j2 = 0; j2 < kGjNb; ++j2) {
      T v = P[0][j2];
#pragma unroll
      for (int a = 1; a < RA; ++a) v = ap == a ? P[a][j2] : v;
      rs[j2] = lane_value(v, pl);
    }
    const T inv = T(1) / rs[j];
#pragma unroll
    for (int j2 = 0; j2 < kGjNb; ++j2) rs[j2] *= inv;
    if (lane == pl) used |= 1u << ap;
#pragma unroll
    for (int a = 0; a < RA; ++a) {
      const bool isp = lane + 64 * a == pr;
      const T f = P[a][j];
#pragma unroll
      for (int j2 = 0; j2 < kGjNb; ++j2)
        if (j2 != j) P[a][j2] = isp ? rs[j2] : fma(-f, rs[j2], P[a][j2]);
      P[a][j] = isp ? inv : -f * inv;
      if (j + 1 < kGjNb) cv[a] = ((used >> a) & 1u) ? T(-1) : fabs(P[a][j + 1]);
    }
    pv[j] = pr;
    if (lane == 0) {
      s.p[buf][j] = pr;
      s.pinv[pr] = k0 + j;
      s.prow[k0 + j] = pr;
    }
  }
  if (!ok) return false;
#pragma unroll
  for (int a = 0; a < RA; ++a) {
    const int i = lane + 64 * a;
    if (i < n)
#pragma unroll
      for (int j = 0; j < kGjNb; ++j)
        if (j < nbk) {
          s.X[(k0 + j) * ld + i] = P[a][j];
          s.C[buf][j * ld + i] = i == pv[j] ? P[a][j] - T(1) : P[a][j];
        }
  }
  return true;
}

template <typename T, int NMAX>
__device__ __forceinline__ bool gj_panel_any(GjScratch<T, NMAX>& s, int n, int k0, int nbk, int buf, const T* Cp,
                                             int jr, unsigned& used) {
  if (n <= 64) return gj_panel<T, 1, NMAX>(s, n, k0, nbk, buf, Cp, jr, used);
  if (NMAX <= 128 || n <= 128) return gj_panel<T, 2, NMAX>(s, n, k0, nbk, buf, Cp, jr, used);
  return gj_panel<T, (NMAX + 63) / 64, NMAX>(s, n, k0, nbk, buf, Cp, jr, used);
}

// X(0 : n8, j) += C X_old(P, j) for the m columns listed by t' -> jj = t' < k0
// ? t' : t' + skip (column j = jj < k0 ? jj : jj + nbk, R row jj), in TR x 2
// tiles taken by threads tid, tid + nthr, ... (TR = 8 rows for float, 4 for
// double, so the C tile stays in 64 registers).
template <typename T, int NMAX>
__device__ __forceinline__ void gj_tiles(GjScratch<T, NMAX>& s, const T* Cb, int n8, int m, int k0, int skip,
                                         int nbk, int tid, int nthr) {
  constexpr int ld = GjScratch<T, NMAX>::kLd;
  constexpr int TR = sizeof(T) == 8 ? 4 : 8, TC = 2;
  const int nti = n8 / TR, ntj = (m + TC - 1) / TC;
  for (int tile = tid; tile < nti * ntj; tile += nthr) {
    const int ti = tile % nti, tj = tile / nti, i0 = ti * TR;
    T c[TR][kGjNb];
#pragma unroll
    for (int q = 0; q < kGjNb; ++q) {
      const T* cp = static_cast<const T*>(__builtin_assume_aligned(Cb + q * ld + i0, 16));
#pragma unroll
      for (int r = 0; r < TR; ++r) c[r][q] = cp[r];
    }
#pragma unroll
    for (int u = 0; u < TC; ++u) {
      const int tp = tj * TC + u;
      if (tp >= m) break;
      const int jj = tp < k0 ? tp : tp + skip, j = jj < k0 ? jj : jj + nbk;
      const T* rp = static_cast<const T*>(__builtin_assume_aligned(s.R + jj * kGjNb, 16));
      T rv[kGjNb];
#pragma unroll
      for (int q = 0; q < kGjNb; ++q) rv[q] = rp[q];
      T* xp = static_cast<T*>(__builtin_assume_aligned(s.X + j * ld + i0, 16));
      T x[TR];
#pragma unroll
      for (int r = 0; r < TR; ++r) x[r] = xp[r];
#pragma unroll
      for (int r = 0; r < TR; ++r)
#pragma unroll
        for (int q = 0; q < kGjNb; ++q) x[r] = fma(c[r][q], rv[q], x[r]);
#pragma unroll
      for (int r = 0; r < TR; ++r) xp[r] = x[r];
    }
  }
}

// load(i, j) returns A(i, j) for i, j < n <= NMAX; out (column-major, ld ldo,
// any address space) receives A^-1 and may hold A itself, since every element
// is read before the first barrier.  Returns false (uniformly) on a zero or
// non-finite pivot.
template <typename T, int NMAX, typename Load>
__device__ bool gj_invert(Load load, int n, T* out, int ldo, GjScratch<T, NMAX>& s) {
  static_assert(NMAX <= 192, "three rows per lane at most");
  constexpr int ld = GjScratch<T, NMAX>::kLd;
  const int t = threadIdx.x, nt = blockDim.x, lane = t & 63;
  const int n8 = (n + 7) & ~7;  // rows touched by the 8-row tiles
  // 16 loads per thread in flight at a time
  constexpr int kLoads = 16;
  for (int e0 = 0; e0 < n * n8; e0 += kLoads * nt) {
    T v[kLoads];
#pragma unroll
    for (int u = 0; u < kLoads; ++u) {
      const int e = e0 + t + u * nt, i = e % n8, j = e / n8;
      v[u] = (e < n * n8 && i < n) ? load(i, j) : T(0);
    }
#pragma unroll
    for (int u = 0; u < kLoads; ++u) {
      const int e = e0 + t + u * nt;
      if (e < n * n8) s.X[(e / n8) * ld + e % n8] = v[u];
    }
  }
  for (int e = t; e < 2 * kGjNb * n8; e += nt) {
    const int b = e / (kGjNb * n8), r = e % (kGjNb * n8);
    s.C[b][(r / n8) * ld + r % n8] = T(0);
  }
  if (t == 0) s.bad = 0;
  unsigned used = 0;
#pragma unroll
  for (int a = 0; a < 3; ++a) used |= (lane + 64 * a >= n ? 1u : 0u) << a;
  __syncthreads();
  if (t < 64 && !gj_panel_any<T, NMAX>(s, n, 0, min(kGjNb, n), 0, nullptr, 0, used) && t == 0) s.bad = 1;
  for (int k0 = 0, buf = 0;; k0 += kGjNb, buf ^= 1) {
    __syncthreads();
    if (s.bad) return false;
    const int nbk = min(kGjNb, n - k0), ncols = n - nbk;
    const int k1 = k0 + nbk, nbk1 = k1 < n ? min(kGjNb, n - k1) : 0;
    // block buf's pivot rows of every other column, before its update
    for (int e = t; e < ncols * kGjNb; e += nt) {
      const int jj = e / kGjNb, q = e % kGjNb, j = jj < k0 ? jj : jj + nbk;
      s.R[e] = q < nbk ? s.X[j * ld + s.p[buf][q]] : T(0);
    }
    __syncthreads();
    if (t < 64) {
      if (nbk1 > 0 && !gj_panel_any<T, NMAX>(s, n, k1, nbk1, buf ^ 1, s.C[buf], k0, used) && t == 0) s.bad = 1;
    } else {
      gj_tiles<T, NMAX>(s, s.C[buf], n8, ncols - nbk1, k0, nbk1, nbk, t - 64, nt - 64);
    }
    if (nbk1 == 0) break;
  }
  __syncthreads();
  for (int e = t; e < n * n; e += nt) {
    const int i = e % n, j = e / n;
    out[s.pinv[i] + (size_t)s.prow[j] * ldo] = s.X[j * ld + i];
  }
  return true;
}

}  // namespace hodlr
