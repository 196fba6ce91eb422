// Device helpers shared by the kernels: reductions and in-LDS Gauss-Jordan.
#pragma once

#include <hip/hip_runtime.h>

#include <climits>

namespace hodlr {

template <typename T> __device__ __forceinline__ T dabs(T x) { return x < T(0) ? -x : x; }

// Keep the larger value; ties go to the lower index.  NaN never wins.
template <typename T>
__device__ __forceinline__ void argmax_merge(T& v, int& i, T v2, int i2) {
  if (v2 > v || (v2 == v && i2 < i)) {
    v = v2;
    i = i2;
  }
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

// In-place Gauss-Jordan inversion with partial (row) pivoting of the b x b
// matrix A (LDS, column-major, leading dimension ld, b <= kGjMax).  On return
// A holds the inverse of the row-permuted matrix; src[j] names the column of
// A that is column j of the inverse of the original matrix.  Returns false
// (uniformly) if a zero or non-finite pivot is met.
//
// Each pivot step costs three workgroup barriers: one wave finds the pivot
// row p of column k; every thread snapshots row p, row k and column k; then
// every thread rewrites the elements it owns as the row swap, the scaling of
// the pivot row and the elimination of the other rows at once.
constexpr int kGjMax = 256;

template <typename T>
struct GjScratch {
  int ipiv[kGjMax], src[kGjMax];
  T colk[kGjMax], prow[kGjMax], krow[kGjMax];
  T pv;
  int p;
};

template <typename T>
__device__ bool gj_inverse(T* A, int b, int ld, GjScratch<T>& w) {
  const int t = threadIdx.x, nt = blockDim.x;
  int lb = 0;
  while ((1 << lb) < b) ++lb;
  // thread t owns row (t & (bp-1)) of every (nt/bp)-th column: no div/mod
  const int bp = 1 << lb, ri = t & (bp - 1), cstep = nt >> lb, c0 = t >> lb;
  const bool owner = cstep > 0 && ri < b;
  bool ok = true;
  for (int k = 0; k < b; ++k) {
    if (t < 64) {
      T v = T(-1);
      int idx = INT_MAX;
      for (int i = k + t; i < b; i += 64) argmax_merge(v, idx, dabs(A[i + k * ld]), i);
      for (int o = 32; o > 0; o >>= 1) {
        const T v2 = __shfl_xor(v, o, 64);
        const int i2 = __shfl_xor(idx, o, 64);
        argmax_merge(v, idx, v2, i2);
      }
      if (t == 0) {
        w.pv = v;
        w.p = idx;
        w.ipiv[k] = idx;
      }
    }
    __syncthreads();
    const int p = w.p;
    const T pv = w.pv;
    if (!(pv > T(0)) || !(pv < T(INFINITY)) || p >= b) {
      ok = false;
      break;
    }
    const T inv = T(1) / A[p + k * ld];
    // snapshot: scaled pivot row, old row k, column k
    for (int j = t; j < b; j += nt) {
      w.prow[j] = A[p + j * ld] * inv;
      w.krow[j] = A[k + j * ld];
    }
    for (int i = t; i < b; i += nt) w.colk[i] = A[i + k * ld];
    __syncthreads();
    if (owner) {
      T* Ai = A + ri;
      const T* pr = w.prow;
      if (ri == k) {
#pragma unroll 4
        for (int j = c0; j < b; j += cstep) Ai[j * ld] = pr[j];
      } else if (ri == p) {  // old row k lands here
        const T f = w.krow[k];
        const T* kr = w.krow;
#pragma unroll 4
        for (int j = c0; j < b; j += cstep) Ai[j * ld] = kr[j] - f * pr[j];
      } else {
        const T f = w.colk[ri];
#pragma unroll 4
        for (int j = c0; j < b; j += cstep) Ai[j * ld] -= f * pr[j];
      }
      if (((k - c0) & (cstep - 1)) == 0 && k >= c0) {
        // column k holds the multipliers: inv on the pivot row, -f * inv elsewhere
        const T f = (ri == p) ? w.krow[k] : w.colk[ri];
        Ai[k * ld] = (ri == k) ? inv : -f * inv;
      }
    }
    __syncthreads();
  }
  if (ok) {
    if (t == 0) {
      for (int j = 0; j < b; ++j) w.src[j] = j;
      for (int k = b - 1; k >= 0; --k) {
        const int p = w.ipiv[k];
        const int x = w.src[k];
        w.src[k] = w.src[p];
        w.src[p] = x;
      }
    }
    __syncthreads();
  }
  return ok;
}

// ---------------------------------------------------------------------------
// Cross-lane moves inside a wavefront through DPP (no LDS round trip).
// ---------------------------------------------------------------------------
template <int CTRL> __device__ __forceinline__ int dpp_move(int v) {
  return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, false);
}
template <int CTRL> __device__ __forceinline__ float dpp_move(float v) {
  return __int_as_float(dpp_move<CTRL>(__float_as_int(v)));
}
template <int CTRL> __device__ __forceinline__ double dpp_move(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = dpp_move<CTRL>((int)(b & 0xffffffffll)), hi = dpp_move<CTRL>((int)(b >> 32));
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

__device__ __forceinline__ float lane_value(float x, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), l));
}
__device__ __forceinline__ double lane_value(double x, int l) {
  const long long v = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_readlane((int)(v & 0xffffffffll), l);
  const int hi = __builtin_amdgcn_readlane((int)(v >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// ---------------------------------------------------------------------------
// Gauss-Jordan inversion with partial pivoting, matrix held in registers.
//
// 256 threads (4 waves); thread (lane, w) holds rows lane + 64 a (a < RA) of
// the columns w + 4 c assigned to its registers, so n <= min(64 RA, 4 CB).
// Step k eliminates column k: the wave holding it finds the pivot row p
// (largest |entry| among rows not yet used, ties to the lower row) and
// publishes the column in LDS; after the one barrier of the step every wave
// reads the pivot row from lane p & 63 of itself, and every element is
// updated at once (rows are never swapped; row p is scaled, the others get
// x -= f * (pivot row) / pivot, and column k receives the multipliers).  With
// P the row order of the pivots the array ends as (P A)^-1 in place, i.e.
// A^-1(r, c) = X(p_r, pinv(c)).  The register columns rotate by one after
// every 4 steps, so the pivot column is always register column 0 of its
// wave and no register is addressed by a run-time index.
// ---------------------------------------------------------------------------
template <typename T, int RA, int CB>
struct GjRegScratch {
  T colv[2][64 * RA];
  int p[2];
  int pinv[64 * RA];  // step at which a row was the pivot row
  int prow[4 * CB];   // pivot row of each step
};

// load(i, j) returns A(i, j) for i, j < n; out (column-major, ld ldo, any
// address space) receives A^-1 and may hold A itself, since every element is
// read before the first barrier.  Returns false (uniformly) on a zero or
// non-finite pivot.
template <typename T, int RA, int CB, typename Load>
__device__ bool gj_invert_regs(Load load, int n, T* out, int ldo, GjRegScratch<T, RA, CB>& s) {
  const int t = threadIdx.x, lane = t & 63;
  const int w = __builtin_amdgcn_readfirstlane(t >> 6);
  T x[RA][CB];
#pragma unroll
  for (int a = 0; a < RA; ++a)
#pragma unroll
    for (int c = 0; c < CB; ++c) {
      const int i = lane + 64 * a, j = w + 4 * c;
      x[a][c] = (i < n && j < n) ? load(i, j) : T(0);
    }
  unsigned used = 0;  // rows that were pivots, or lie beyond n
#pragma unroll
  for (int a = 0; a < RA; ++a) used |= (lane + 64 * a >= n ? 1u : 0u) << a;
  bool ok = true;
  int rot = 0;  // register column c holds column w + 4 ((c + rot) mod CB)
  for (int k0 = 0; k0 < n && ok; k0 += 4) {
    for (int wq = 0; wq < 4; ++wq) {
      const int k = k0 + wq;
      if (k >= n) break;
      const int par = k & 1;
      if (w == wq) {
        T bv = T(-1);
        int bi = INT_MAX;
#pragma unroll
        for (int a = 0; a < RA; ++a) {
          const T v = ((used >> a) & 1u) ? T(-1) : fabs(x[a][0]);
          if (v > bv) {
            bv = v;
            bi = lane + 64 * a;
          }
        }
        wave_argmax(bv, bi);
        if (lane == 0) s.p[par] = bi;
#pragma unroll
        for (int a = 0; a < RA; ++a) s.colv[par][lane + 64 * a] = x[a][0];
      }
      __syncthreads();
      const int p = __builtin_amdgcn_readfirstlane(s.p[par]);
      if (p < 0 || p >= n) {
        ok = false;
        break;
      }
      const T piv = s.colv[par][p];
      if (!(fabs(piv) > T(0)) || !(fabs(piv) < T(INFINITY))) {
        ok = false;
        break;
      }
      const T inv = T(1) / piv;
      const int pl = p & 63, ap = p >> 6;
      if (t == 0) {
        s.pinv[p] = k;
        s.prow[k] = p;
      }
      T f[RA];
#pragma unroll
      for (int a = 0; a < RA; ++a) f[a] = (lane + 64 * a == p) ? T(0) : s.colv[par][lane + 64 * a];
#pragma unroll
      for (int c = 0; c < CB; ++c) {
        T v = x[0][c];
#pragma unroll
        for (int a = 1; a < RA; ++a)
          if (ap == a) v = x[a][c];
        const T rs = lane_value(v, pl) * inv;
#pragma unroll
        for (int a = 0; a < RA; ++a) x[a][c] = fma(-f[a], rs, x[a][c]);
      }
      // the pivot row is scaled (its f is 0, so the update left it as it was)
      const T sc = lane == pl ? inv : T(1);
#pragma unroll
      for (int a = 0; a < RA; ++a)
        if (a == ap) {
#pragma unroll
          for (int c = 0; c < CB; ++c) x[a][c] *= sc;
        }
      // column k: the multipliers
      if (w == wq) {
#pragma unroll
        for (int a = 0; a < RA; ++a)
          x[a][0] = (lane + 64 * a == p) ? inv : -s.colv[par][lane + 64 * a] * inv;
      }
      if (lane == pl) used |= 1u << ap;
    }
    // rotate the register columns by one
#pragma unroll
    for (int a = 0; a < RA; ++a) {
      const T x0 = x[a][0];
#pragma unroll
      for (int c = 0; c + 1 < CB; ++c) x[a][c] = x[a][c + 1];
      x[a][CB - 1] = x0;
    }
    ++rot;
  }
  __syncthreads();
  if (!ok) return false;
#pragma unroll
  for (int a = 0; a < RA; ++a)
#pragma unroll
    for (int c = 0; c < CB; ++c) {
      int cc = c + rot;
      while (cc >= CB) cc -= CB;
      const int i = lane + 64 * a, j = w + 4 * cc;
      if (i < n && j < n) out[s.pinv[i] + (size_t)s.prow[j] * ldo] = x[a][c];
    }
  return true;
}

// Size classes of gj_invert_regs for n <= 64, 128 and NMAX (184 or 128).
template <typename T, int NMAX>
union GjRegScratchAll {
  GjRegScratch<T, 1, 16> s1;
  GjRegScratch<T, 2, 32> s2;
  GjRegScratch<T, (NMAX + 63) / 64, (NMAX + 3) / 4> s3;
};

template <typename T, int NMAX, typename Load>
__device__ bool gj_invert(Load load, int n, T* out, int ldo, GjRegScratchAll<T, NMAX>& s) {
  if (n <= 64) return gj_invert_regs<T, 1, 16>(load, n, out, ldo, s.s1);
  if (n <= 128 || NMAX <= 128) return gj_invert_regs<T, 2, 32>(load, n, out, ldo, s.s2);
  return gj_invert_regs<T, (NMAX + 63) / 64, (NMAX + 3) / 4>(load, n, out, ldo, s.s3);
}

// C = alpha * A * B + beta * C for column-major operands (any address space)
// computed by the whole workgroup through 32 x 32 LDS tiles.  As, Bs: LDS,
// 32 * 33 elements each.  beta == 0 does not read C.  C must not alias A, B.
template <typename T>
__device__ void wg_gemm(int m, int n, int k, T alpha, const T* A, int lda, const T* B, int ldb, T beta,
                        T* C, int ldc, T* As, T* Bs) {
  const int t = threadIdx.x, nt = blockDim.x, tx = t & 15, ty = (t >> 4) & 15;
  const bool active = t < 256;
  for (int i0 = 0; i0 < m; i0 += 32)
    for (int j0 = 0; j0 < n; j0 += 32) {
      T acc[2][2] = {{T(0), T(0)}, {T(0), T(0)}};
      for (int k0 = 0; k0 < k; k0 += 32) {
        // all loads of the two tiles are issued before any is stored
        T av[4], bv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int e = t + u * 256;
          const int ii = e & 31, kk = e >> 5;
          av[u] = (e < 1024 && i0 + ii < m && k0 + kk < k) ? A[(i0 + ii) + (size_t)(k0 + kk) * lda] : T(0);
          bv[u] = (e < 1024 && k0 + ii < k && j0 + kk < n) ? B[(k0 + ii) + (size_t)(j0 + kk) * ldb] : T(0);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int e = t + u * 256;
          if (e < 1024 && t < 256) {
            As[(e >> 5) * 33 + (e & 31)] = av[u];
            Bs[(e >> 5) * 33 + (e & 31)] = bv[u];
          }
        }
        __syncthreads();
        if (active) {
#pragma unroll 8
          for (int kk = 0; kk < 32; ++kk) {
            const T a0 = As[kk * 33 + tx], a1 = As[kk * 33 + tx + 16];
            const T b0 = Bs[ty * 33 + kk], b1 = Bs[(ty + 16) * 33 + kk];
            acc[0][0] += a0 * b0;
            acc[0][1] += a0 * b1;
            acc[1][0] += a1 * b0;
            acc[1][1] += a1 * b1;
          }
        }
        __syncthreads();
      }
      if (active) {
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
          for (int c = 0; c < 2; ++c) {
            const int i = i0 + tx + 16 * a, j = j0 + ty + 16 * c;
            if (i < m && j < n) {
              T* cp = C + i + (size_t)j * ldc;
              *cp = (beta == T(0) ? T(0) : beta * *cp) + alpha * acc[a][c];
            }
          }
      }
      __syncthreads();
    }
}

}  // namespace hodlr
