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

// Wave-uniform maximum: DPP inside each 16-lane row, then the four row
// results by readlane.  NaN never wins a comparison.
template <typename T> __device__ __forceinline__ T sel_max(T a, T b) { return b > a ? b : a; }

// A launch gated on per-column activity flags (gate[0..ngate), any nonzero:
// work to do) does nothing once every column has stopped.  Every thread reads
// the same flags, so the answer is the same across the workgroup.
__device__ __forceinline__ bool gate_closed(const int* gate, int ngate) {
  if (!gate) return false;
  int any = 0;
  for (int k = 0; k < ngate; ++k) any |= gate[k];
  return any == 0;
}

template <typename T> __device__ __forceinline__ T wave_max(T m) {
  m = sel_max(m, dpp_move<0xB1>(m));
  m = sel_max(m, dpp_move<0x4E>(m));
  m = sel_max(m, dpp_move<0x141>(m));
  m = sel_max(m, dpp_move<0x140>(m));
  return sel_max(sel_max(lane_value(m, 0), lane_value(m, 16)), sel_max(lane_value(m, 32), lane_value(m, 48)));
}

// ---------------------------------------------------------------------------
// Blocked Gauss-Jordan inversion with partial pivoting (gj_threads<T>() threads).
//
// The matrix sits in LDS.  Every kGjNb = 8 pivot steps form a block.  Wave 0
// factors the block's 8 columns (the panel) in its registers (rows lane +
// 64 a) without barriers: the pivot row is scaled, the other rows are
// eliminated, and the column is replaced by the multipliers, which is the
// in-place Gauss-Jordan step.  The block's steps applied to any other column
// j amount to X(:, j) += C X_old(P, j), with P the block's pivot rows and
// C = Z - I(:, P) for the factored panel Z: one rank-8 update.
//
// Pivot choice: the rows not yet used are compared on a 32-bit key, the
// leading bits of |x| (float: sign-cleared bits with the low byte dropped,
// i.e. 15 of the 23 mantissa bits; double: the high word likewise, 12 of
// 52) with 255 - row in the low byte, so that one unsigned maximum (DPP in
// each 16-lane row, readlane across rows) gives the largest magnitude and,
// among magnitudes equal to that precision, the lowest row.  A NaN or
// infinite candidate wins and fails the step, as does a zero pivot.  The
// step has no branch, so the whole panel is one scheduling region.
//
// Look-ahead: while wave 0 applies block b's update to the next panel's
// columns and factors that panel, waves 1.. apply block b's update to every
// other column on the matrix cores (v_mfma_*_16x16x4: A = 16 rows of C, K =
// the block's 4 + 4 pivot steps, B = the pivot rows of 16 columns).  A wave
// owns whole 16-column strips, so it reads their pivot-row values before it
// writes any of them and no barrier separates the two.  Rows are never
// swapped: with p_k the pivot row of step k the array ends as (P A)^-1, i.e.
// A^-1(r, c) = X(p_r, pinv(c)).
// ---------------------------------------------------------------------------
constexpr int kGjNb = 8;
// Double precision takes 8 waves, which leaves it 256 registers per lane for
// the panel wave.
template <typename T>
constexpr int gj_threads() {
  return sizeof(T) == 8 ? 512 : 1024;
}

template <typename T, int NMAX>
struct GjScratch {
  // column stride: 16 bytes past a multiple of 8 entries, so that the 16
  // lanes of an MFMA tile row (16 columns) hit different LDS banks
  static constexpr int kLd = (NMAX + 7) / 8 * 8 + 16 / (int)sizeof(T);
  alignas(16) T X[NMAX * kLd];      // the matrix, column-major
  alignas(16) T C[2][kGjNb * kLd];  // C = Z - I(:, P) of two blocks, column-major
  int p[2][kGjNb];                  // pivot rows of two blocks
  int pinv[NMAX];                   // step at which a row was the pivot row
  int prow[NMAX];                   // pivot row of each step
  int bad;
};

__device__ __forceinline__ unsigned gj_key_bits(float x) { return __float_as_uint(x); }
__device__ __forceinline__ unsigned gj_key_bits(double x) {
  return (unsigned)((unsigned long long)__double_as_longlong(x) >> 32);
}

template <int CTRL> __device__ __forceinline__ unsigned dpp_max_u32(unsigned v) {
  const unsigned o = (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, 0xF, 0xF, false);
  return v > o ? v : o;
}

__device__ __forceinline__ unsigned wave_max_u32(unsigned m) {
  m = dpp_max_u32<0xB1>(m);
  m = dpp_max_u32<0x4E>(m);
  m = dpp_max_u32<0x141>(m);
  m = dpp_max_u32<0x140>(m);
  const unsigned a = __builtin_amdgcn_readlane(m, 0), b = __builtin_amdgcn_readlane(m, 16);
  const unsigned c = __builtin_amdgcn_readlane(m, 32), d = __builtin_amdgcn_readlane(m, 48);
  const unsigned ab = a > b ? a : b, cd = c > d ? c : d;
  return ab > cd ? ab : cd;
}

// 1 / p: the hardware estimate refined by Newton steps (one for float, two
// for double, from the estimate's ~2^-26 relative error)
__device__ __forceinline__ float gj_recip(float p) {
  const float r = __builtin_amdgcn_rcpf(p);
  return fmaf(fmaf(-p, r, 1.f), r, r);
}
__device__ __forceinline__ double gj_recip(double p) {
  double r = __builtin_amdgcn_rcp(p);
  r = fma(fma(-p, r, 1.0), r, r);
  return fma(fma(-p, r, 1.0), r, r);
}

// Wave 0: loads the panel X(:, k0 : k0 + nbk) into registers, applies the
// previous block's update to it if upd (C and pivots in buffer buf ^ 1, the
// pivot-row values read from the panel's own columns before any write),
// runs the panel's pivot steps and stores Z, C and the pivots in buffer buf.
// used: per lane, bit a = row lane + 64 a used or beyond n.  FULL: nbk = 8.
template <typename T, int RA, int NMAX, bool FULL>
__device__ bool gj_panel(GjScratch<T, NMAX>& s, int n, int k0, int nbk, int buf, bool upd, unsigned& used) {
  constexpr int ld = GjScratch<T, NMAX>::kLd;
  const int lane = threadIdx.x & 63;
  T P[RA][kGjNb];
#pragma unroll
  for (int a = 0; a < RA; ++a)
#pragma unroll
    for (int j = 0; j < kGjNb; ++j) {
      const int i = lane + 64 * a;
      P[a][j] = (i < n && (FULL || j < nbk)) ? s.X[(k0 + j) * ld + i] : T(0);
    }
  if (upd) {
    const T* Cp = s.C[buf ^ 1];
    int pq[kGjNb];
#pragma unroll
    for (int q = 0; q < kGjNb; ++q) pq[q] = __builtin_amdgcn_readfirstlane(s.p[buf ^ 1][q]);
    T c[RA][kGjNb];
#pragma unroll
    for (int a = 0; a < RA; ++a) {
      const int i = min(lane + 64 * a, ld - 1);
#pragma unroll
      for (int q = 0; q < kGjNb; ++q) c[a][q] = Cp[q * ld + i];
    }
#pragma unroll
    for (int j = 0; j < kGjNb; ++j) {
      if (!FULL && j >= nbk) break;
      T r[kGjNb];
#pragma unroll
      for (int q = 0; q < kGjNb; ++q) r[q] = s.X[(k0 + j) * ld + pq[q]];
#pragma unroll
      for (int a = 0; a < RA; ++a)
#pragma unroll
        for (int q = 0; q < kGjNb; ++q) P[a][j] = fma(c[a][q], r[q], P[a][j]);
    }
  }
  int pv[kGjNb];
#pragma unroll
  for (int j = 0; j < kGjNb; ++j) pv[j] = 0;
  bool ok = true;
#pragma unroll
  for (int j = 0; j < kGjNb; ++j) {
    if (!FULL && j >= nbk) break;
    unsigned m = 0;
#pragma unroll
    for (int a = 0; a < RA; ++a) {
      const unsigned k = ((used >> a) & 1u) ? 0u
                                            : ((gj_key_bits(P[a][j]) & 0x7fffff00u) | (unsigned)(255 - (lane + 64 * a)));
      m = k > m ? k : m;
    }
    const unsigned key = wave_max_u32(m);
    const int pr = key ? 255 - (int)(key & 255u) : 0;
    const int ap = pr >> 6, pl = pr & 63;
    T rs[kGjNb];
#pragma unroll
    for (int j2 = 0; j2 < kGjNb; ++j2) {
      T v = P[0][j2];
#pragma unroll
      for (int a = 1; a < RA; ++a) v = ap == a ? P[a][j2] : v;
      rs[j2] = lane_value(v, pl);
    }
    const T av = fabs(rs[j]);
    ok = ok && key != 0u && av > T(0) && av < T(INFINITY);
    const T inv = gj_recip(rs[j]);
#pragma unroll
    for (int j2 = 0; j2 < kGjNb; ++j2) rs[j2] *= inv;
    used |= lane == pl ? 1u << ap : 0u;
#pragma unroll
    for (int a = 0; a < RA; ++a) {
      const bool isp = lane + 64 * a == pr;
      const T f = P[a][j];
#pragma unroll
      for (int j2 = 0; j2 < kGjNb; ++j2)
        if (j2 != j) P[a][j2] = isp ? rs[j2] : fma(-f, rs[j2], P[a][j2]);
      P[a][j] = isp ? inv : -f * inv;
    }
    pv[j] = pr;
  }
  if (!ok) return false;
  int mine = pv[0];
#pragma unroll
  for (int j = 1; j < kGjNb; ++j) mine = lane == j ? pv[j] : mine;
  if (lane < nbk) {
    s.p[buf][lane] = mine;
    s.pinv[mine] = k0 + lane;
    s.prow[k0 + lane] = mine;
  }
#pragma unroll
  for (int a = 0; a < RA; ++a) {
    const int i = lane + 64 * a;
    if (i < n)
#pragma unroll
      for (int j = 0; j < kGjNb; ++j)
        if (FULL || j < nbk) {
          s.X[(k0 + j) * ld + i] = P[a][j];
          s.C[buf][j * ld + i] = i == pv[j] ? P[a][j] - T(1) : P[a][j];
        }
  }
  return true;
}

template <typename T, int NMAX>
__device__ __forceinline__ bool gj_panel_any(GjScratch<T, NMAX>& s, int n, int k0, int nbk, int buf, bool upd,
                                             unsigned& used) {
  constexpr int RMAX = (NMAX + 63) / 64;
  if (nbk == kGjNb) {
    if (n <= 64) return gj_panel<T, 1, NMAX, true>(s, n, k0, nbk, buf, upd, used);
    if (NMAX <= 128 || n <= 128) return gj_panel<T, 2, NMAX, true>(s, n, k0, nbk, buf, upd, used);
    return gj_panel<T, RMAX, NMAX, true>(s, n, k0, nbk, buf, upd, used);
  }
  if (n <= 64) return gj_panel<T, 1, NMAX, false>(s, n, k0, nbk, buf, upd, used);
  if (NMAX <= 128 || n <= 128) return gj_panel<T, 2, NMAX, false>(s, n, k0, nbk, buf, upd, used);
  return gj_panel<T, RMAX, NMAX, false>(s, n, k0, nbk, buf, upd, used);
}

typedef float gj_f4 __attribute__((ext_vector_type(4)));
typedef double gj_d4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ gj_f4 gj_mfma(float a, float b, gj_f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ gj_d4 gj_mfma(double a, double b, gj_d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
template <typename T> struct GjVec;
template <> struct GjVec<float> { typedef gj_f4 t; };
template <> struct GjVec<double> { typedef gj_d4 t; };

// Block buf's steps applied to the m columns outside both panels (column
// t' < m is jj = t' < k0 ? t' : t' + skip, j = jj < k0 ? jj : jj + nbk), in
// 16-column strips, strip wt, wt + nwt, ... for this wave.  Lane (cl, kg) =
// (lane % 16, lane / 16) holds column cl of the strip; the MFMA's A operand
// is C(m0 + cl, kg [+ 4]) and its B operand the column's value in pivot row
// p_kg [p_kg+4], read once per strip before the first write.
template <typename T, int NMAX>
__device__ void gj_strips(GjScratch<T, NMAX>& s, int buf, int n, int nbk, int m, int k0, int skip, int wt, int nwt) {
  constexpr int ld = GjScratch<T, NMAX>::kLd;
  typedef typename GjVec<T>::t v4;
  const int lane = threadIdx.x & 63, cl = lane & 15, kg = lane >> 4;
  const T* Cb = s.C[buf];
  const int q0 = s.p[buf][kg], q1 = s.p[buf][kg + 4];
  const bool h0 = kg < nbk, h1 = kg + 4 < nbk;
  const int ntr = (n + 15) >> 4;
  for (int strip = wt; strip * 16 < m; strip += nwt) {
    const int tp = strip * 16 + cl;
    const bool vc = tp < m;
    const int jj = tp < k0 ? tp : tp + skip, j = vc ? (jj < k0 ? jj : jj + nbk) : 0;
    T* col = s.X + j * ld;
    const T b0 = (vc && h0) ? col[q0] : T(0), b1 = (vc && h1) ? col[q1] : T(0);
    for (int ti = 0; ti < ntr; ++ti) {
      const int m0 = 16 * ti, ra = min(m0 + cl, ld - 1);
      v4 acc;
      if constexpr (sizeof(T) == 4) {
        // float: output register v of lane (cl, kg) is row 4 kg + v, column cl
        const int row0 = m0 + 4 * kg;
        const bool st = vc && row0 < n;  // rows row0 .. row0 + 3 < ld
        if (st)
          acc = *reinterpret_cast<const v4*>(col + row0);
        else
          acc = v4{0, 0, 0, 0};
        acc = gj_mfma(Cb[kg * ld + ra], b0, acc);
        acc = gj_mfma(Cb[(kg + 4) * ld + ra], b1, acc);
        if (st) *reinterpret_cast<v4*>(col + row0) = acc;
      } else {
        // double: output register v of lane (cl, kg) is row 4 v + kg, column cl
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[v] = (vc && m0 + 4 * v + kg < n) ? col[m0 + 4 * v + kg] : T(0);
        acc = gj_mfma(Cb[kg * ld + ra], b0, acc);
        acc = gj_mfma(Cb[(kg + 4) * ld + ra], b1, acc);
#pragma unroll
        for (int v = 0; v < 4; ++v)
          if (vc && m0 + 4 * v + kg < n) col[m0 + 4 * v + kg] = acc[v];
      }
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
  const int wv = __builtin_amdgcn_readfirstlane(t >> 6), nwv = nt >> 6;
  const int n8 = (n + 7) & ~7;
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
  for (int e = t; e < 2 * kGjNb * ld; e += nt) (&s.C[0][0])[e] = T(0);
  if (t < 2 * kGjNb) (&s.p[0][0])[t] = 0;
  if (t == 0) s.bad = 0;
  unsigned used = 0;
#pragma unroll
  for (int a = 0; a < 3; ++a) used |= (lane + 64 * a >= n ? 1u : 0u) << a;
  __syncthreads();
  if (wv == 0 && !gj_panel_any<T, NMAX>(s, n, 0, min(kGjNb, n), 0, false, used) && t == 0) s.bad = 1;
  for (int k0 = 0, buf = 0;; k0 += kGjNb, buf ^= 1) {
    __syncthreads();
    if (s.bad) return false;
    const int nbk = min(kGjNb, n - k0), ncols = n - nbk;
    const int k1 = k0 + nbk, nbk1 = k1 < n ? min(kGjNb, n - k1) : 0;
    if (wv == 0) {
      if (nbk1 > 0 && !gj_panel_any<T, NMAX>(s, n, k1, nbk1, buf ^ 1, true, used) && t == 0) s.bad = 1;
    } else {
      gj_strips<T, NMAX>(s, buf, n, nbk, ncols - nbk1, k0, nbk1, wv - 1, nwv - 1);
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
