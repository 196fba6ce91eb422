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
// matrix A (LDS, column-major, leading dimension ld).  On return A holds the
// inverse of the row-permuted matrix; src[j] (LDS, b ints) names the column
// of A that is column j of the inverse of the original matrix.  Returns false
// (uniformly) if a zero or non-finite pivot is met.  ipiv, colk: LDS scratch
// of b entries; sv/si: reduction scratch.
template <typename T>
__device__ bool gj_inverse(T* A, int b, int ld, int* ipiv, int* src, T* colk, T* sv, int* si) {
  const int t = threadIdx.x, nt = blockDim.x;
  bool ok = true;
  for (int k = 0; k < b; ++k) {
    T v = T(-1);
    int idx = INT_MAX;
    for (int i = k + t; i < b; i += nt) argmax_merge(v, idx, dabs(A[i + k * ld]), i);
    T pv;
    int p;
    block_argmax(v, idx, sv, si, pv, p);
    if (!(pv > T(0)) || !(pv < T(INFINITY)) || p >= b) {
      ok = false;
      break;
    }
    if (t == 0) ipiv[k] = p;
    if (p != k) {
      for (int j = t; j < b; j += nt) {
        T x = A[k + j * ld];
        A[k + j * ld] = A[p + j * ld];
        A[p + j * ld] = x;
      }
    }
    __syncthreads();
    const T inv = T(1) / A[k + k * ld];
    for (int i = t; i < b; i += nt) colk[i] = A[i + k * ld];
    __syncthreads();
    for (int j = t; j < b; j += nt) A[k + j * ld] = (j == k) ? inv : A[k + j * ld] * inv;
    __syncthreads();
    for (int e = t; e < b * b; e += nt) {
      const int i = e % b, j = e / b;
      if (i != k) {
        const T rk = A[k + j * ld];
        A[i + j * ld] = (j == k ? T(0) : A[i + j * ld]) - colk[i] * rk;
      }
    }
    __syncthreads();
  }
  if (ok) {
    if (t == 0) {
      for (int j = 0; j < b; ++j) src[j] = j;
      for (int k = b - 1; k >= 0; --k) {
        int p = ipiv[k];
        int x = src[k];
        src[k] = src[p];
        src[p] = x;
      }
    }
    __syncthreads();
  }
  return ok;
}

}  // namespace hodlr
