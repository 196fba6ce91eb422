// HODLR factorization and solve (Sec. 4.3), level by level on the GPU.
//
// Storage (T = float or double, column-major, leading dimension n):
//   Y  n x R  column block q (offset off[q-1], width rcols[q-1]) holds, in the
//             rows of each level-q node c, U_c; the factorization overwrites
//             it with d_c = K_c^-1 U_c and, in the columns of the blocks
//             above q, with the partially solved ancestor panels.
//   W  n x R  column block q holds, in the rows of the sibling of c, V_c, so
//             K(c, sibling) = U_c V_c^T.
//   Kinv      leaf inverses from an LU with partial pivoting (Gauss-Jordan).
//   Sinv      per internal node, the inverse of the capacitance matrix
//             S = [[I, V_b^T d_a], [V_a^T d_b, I]] (eq. SchurSum), stored for
//             the ranks (r_b + r_a) with leading dimension 2 r_q.
//
// With the leaf inverses applied to every column of Y at once (the stacked
// right-hand sides Z = [U | ancestor U] of Sec. 4.3.1 step 2-3), each level q,
// from the leaves up, needs for every node c of level q the products
// G_c = W_c^T Y_c (giving V^T d and V^T c at once), then per parent the
// capacitance inverse and y = S^-1 [V_b^T c_a; V_a^T c_b], and finally the
// corrections c_a -= d_a y_b, c_b -= d_b y_a (step 5).  The solve (Sec. 4.3.2)
// runs the same three kernels on the right-hand side after the leaf solve.
#include <algorithm>
#include <string>
#include <vector>

#include "device_util.h"
#include "gemm.h"
#include "hodlr_internal.h"

namespace hodlr {

// ---------------------------------------------------------------------------
// Staging
// ---------------------------------------------------------------------------
template <typename T>
__global__ void k_stage_leaves_K(const double* __restrict__ K, int ldk, const int* __restrict__ lo,
                                 const int* __restrict__ hi, int id0, int bmax, T* __restrict__ out) {
  const int leaf = blockIdx.y, id = id0 + leaf;
  const int l0 = lo[id], b = hi[id] - l0;
  T* o = out + (size_t)leaf * bmax * bmax;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < b * b; e += gridDim.x * blockDim.x) {
    const int i = e % b, j = e / b;
    o[i + (size_t)j * bmax] = (T)K[(size_t)(l0 + j) * ldk + l0 + i];
  }
}

template <typename T>
__global__ void k_stage_leaves_packed(const double* __restrict__ leaves, const int* __restrict__ lo,
                                      const int* __restrict__ hi, int id0, int bmax,
                                      T* __restrict__ out) {
  const int leaf = blockIdx.y, id = id0 + leaf;
  size_t base = 0;
  for (int k = 0; k < leaf; ++k) {
    const size_t bk = hi[id0 + k] - lo[id0 + k];
    base += bk * bk;
  }
  const int b = hi[id] - lo[id];
  T* o = out + (size_t)leaf * bmax * bmax;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < b * b; e += gridDim.x * blockDim.x) {
    const int i = e % b, j = e / b;
    o[i + (size_t)j * bmax] = (T)leaves[base + i + (size_t)j * b];
  }
}

template <typename S, typename D>
__global__ void k_convert(const S* __restrict__ src, D* __restrict__ dst, size_t count) {
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < count;
       e += (size_t)gridDim.x * blockDim.x)
    dst[e] = (D)src[e];
}

// ---------------------------------------------------------------------------
// Leaf LU (partial pivoting) kept as the explicit inverse
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(gj_threads<T>())
    k_leaf_inverse(T* __restrict__ Kinv, int bmax, const int* __restrict__ lo,
                   const int* __restrict__ hi, int id0, int* __restrict__ status) {
  __shared__ GjScratch<T, (sizeof(T) == 8 ? kRankCap64 : kRankCap32)> gw;
  const int leaf = blockIdx.x, id = id0 + leaf, t = threadIdx.x;
  const int b = hi[id] - lo[id];
  T* Gm = Kinv + (size_t)leaf * bmax * bmax;
  const bool ok = gj_invert(
      [&](int i, int j) { return Gm[i + (size_t)j * bmax]; }, b, Gm, bmax, gw);
  if (!ok && t == 0) {
    atomicExch(status + 0, 1);
    atomicExch(status + 1, id);
  }
}

// Z(rows of leaf, c0 : c0+CT) = Kinv_leaf * Z(rows of leaf, c0 : c0+CT), in place.
template <typename T, int CT>
__global__ void __launch_bounds__(kBlock)
    k_leaf_apply(const T* __restrict__ Kinv, int bmax, const int* __restrict__ lo,
                 const int* __restrict__ hi, int id0, T* __restrict__ Z, int ldz, int ncols) {
  __shared__ T Zt[kLeafMax * CT];
  const int leaf = blockIdx.x, c0 = blockIdx.y * CT, id = id0 + leaf, t = threadIdx.x;
  const int l0 = lo[id], b = hi[id] - l0;
  const int nc = min(CT, ncols - c0);
  const T* Ki = Kinv + (size_t)leaf * bmax * bmax;
  for (int e = t; e < b * CT; e += blockDim.x) {
    const int i = e % b, c = e / b;
    Zt[i + c * b] = (c < nc) ? Z[(size_t)(c0 + c) * ldz + l0 + i] : T(0);
  }
  __syncthreads();
  for (int i = t; i < b; i += blockDim.x) {
    T acc[CT];
#pragma unroll
    for (int c = 0; c < CT; ++c) acc[c] = T(0);
    int kk = 0;
    for (; kk + 8 <= b; kk += 8) {
      T a[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) a[u] = Ki[i + (size_t)(kk + u) * bmax];
#pragma unroll
      for (int u = 0; u < 8; ++u)
#pragma unroll
        for (int c = 0; c < CT; ++c) acc[c] += a[u] * Zt[kk + u + c * b];
    }
    for (; kk < b; ++kk) {
      const T a = Ki[i + (size_t)kk * bmax];
#pragma unroll
      for (int c = 0; c < CT; ++c) acc[c] += a * Zt[kk + c * b];
    }
    for (int c = 0; c < nc; ++c) Z[(size_t)(c0 + c) * ldz + l0 + i] = acc[c];
  }
}

// The same product in float32 on the matrix cores (v_mfma_f32_32x32x2f32):
// one workgroup per (leaf, 64-column tile of Z); the leaf inverse and the
// tile go to LDS by asynchronous copies (inner dimension padded to even with
// zeros, inverse rows to a multiple of 32), each of the four waves computes
// up to three 32 x 32 output quarters, and the tile is written back in place
// (every read of it precedes the writes).  Used while both fit in LDS.
typedef float f32x16 __attribute__((ext_vector_type(16)));

static size_t leaf_apply_mfma_lds(int bmax) {
  const int nrt = (bmax + 31) / 32, bp = (bmax + 7) & ~7, ld = 32 * nrt + 1;
  return (size_t)(bp + 64) * ld * sizeof(float);
}

__global__ void __launch_bounds__(kBlock)
    k_leaf_apply_mfma(const float* __restrict__ Kinv, int bmax, const int* __restrict__ lo,
                      const int* __restrict__ hi, int id0, float* __restrict__ Z, int ldz, int ncols) {
  extern __shared__ __align__(16) float lsm[];
  const int leaf = blockIdx.x, c0 = blockIdx.y * 64, id = id0 + leaf, t = threadIdx.x;
  const int lane = t & 63, w = t >> 6, kl = lane >> 5, r32 = lane & 31;
  const int l0 = lo[id], b = hi[id] - l0, nc = min(64, ncols - c0);
  // inner dimension padded to a multiple of 8 (four MFMA steps per round)
  const int nrt = (b + 31) / 32, bp = (b + 7) & ~7, ld = 32 * nrt + 1;
  float* Ks = lsm;            // column k at Ks + k ld, rows [0, 32 nrt)
  float* Zs = lsm + bp * ld;  // column j at Zs + j ld, rows [0, bp)
  const float* Ki = Kinv + (size_t)leaf * bmax * bmax;
  for (int k = w; k < b; k += kBlock / 64) dma_span(Ks + (size_t)k * ld, Ki + (size_t)k * bmax, b);
  for (int j = w; j < nc; j += kBlock / 64) dma_span(Zs + (size_t)j * ld, Z + (size_t)(c0 + j) * ldz + l0, b);
  // zeros outside what the copies fill
  const int tail = 32 * nrt - b;
  for (int e = t; e < b * tail; e += kBlock) Ks[(size_t)(e / tail) * ld + b + e % tail] = 0.f;
  for (int e = t; e < (bp - b) * 32 * nrt; e += kBlock) Ks[(size_t)(b + e / (32 * nrt)) * ld + e % (32 * nrt)] = 0.f;
  for (int e = t; e < nc * (bp - b); e += kBlock) Zs[(size_t)(e / (bp - b)) * ld + b + e % (bp - b)] = 0.f;
  for (int e = t; e < (64 - nc) * bp; e += kBlock) Zs[(size_t)(nc + e / bp) * ld + e % bp] = 0.f;
  dma_wait();
  // wave w: quarters w, w + 4, w + 8 (row tiles w / 2, w / 2 + 2, w / 2 + 4,
  // all in column tile w % 2), updated together so their products overlap
  const int ct = w & 1, rt0 = w >> 1;
  const int nq = min(3, (nrt - rt0 + 1) / 2);
  if (nq <= 0) return;
  f32x16 acc[3] = {f32x16{}, f32x16{}, f32x16{}};
  const float* Bp = Zs + (size_t)(32 * ct + r32) * ld + kl;
  const float* Ap = Ks + 32 * rt0 + r32 + (size_t)kl * ld;
  for (int k = 0; k < bp; k += 8) {
    float bv[4], av[3][4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      bv[u] = Bp[k + 2 * u];
#pragma unroll
      for (int qi = 0; qi < 3; ++qi) av[qi][u] = qi < nq ? Ap[(size_t)(k + 2 * u) * ld + 64 * qi] : 0.f;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int qi = 0; qi < 3; ++qi)
        if (qi < nq) acc[qi] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[qi][u], bv[u], acc[qi], 0, 0, 0);
  }
  // D(v) at lane l: row 8 (v / 4) + 4 (l / 32) + v % 4, column l % 32
#pragma unroll
  for (int qi = 0; qi < 3; ++qi) {
    if (qi >= nq) break;
    const int rt = rt0 + 2 * qi;
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int i = 32 * rt + 8 * (v >> 2) + 4 * kl + (v & 3), j = 32 * ct + r32;
      if (i < b && j < nc) Z[(size_t)(c0 + j) * ldz + l0 + i] = acc[qi][v];
    }
  }
}

__global__ void k_fill_int(int* p, int n, int v) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = v;
}

// ---------------------------------------------------------------------------
// Capacitance inverse per parent of level q.  With A = V_b^T d_a (r_b x r_a)
// and B = V_a^T d_b (r_a x r_b), S = [[I, A], [B, I]] (eq. SchurSum) and, with
// M = I - B A,
//   S^-1 = [[I + A M^-1 B, -A M^-1], [-M^-1 B, M^-1]].
// M is formed in the S22 block by a batched product; this kernel inverts it
// in place; the other three blocks follow as batched products.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(gj_threads<T>())
    k_capacitance_inverse(const int* __restrict__ rank, int q, int rq, T* __restrict__ Sinv,
                          int* __restrict__ status) {
  __shared__ GjScratch<T, (sizeof(T) == 8 ? kRankCap64 : kRankCap32)> gw;
  const int i = blockIdx.x;
  const int ra = rank[node_id(q, 2 * i)], rb = rank[node_id(q, 2 * i + 1)], lds = 2 * rq;
  if (ra == 0) return;
  T* S22 = Sinv + (size_t)i * lds * lds + rb + (size_t)rb * lds;
  const bool ok = gj_invert([&](int r, int c) { return S22[r + (size_t)c * lds]; }, ra, S22, lds, gw);
  if (!ok && threadIdx.x == 0) {
    atomicExch(status + 0, 2);
    atomicExch(status + 1, node_id(q - 1, i));
  }
}

// y = S^-1 [t_a; t_b] for every parent of level q: t_a = G_a(0:r_b, 0:ccols),
// t_b = G_b(0:r_a, 0:ccols).  Y is (2 rq) x ccols per parent (ld 2 rq).
// Workgroup (parent, CT-column chunk), one thread per row of S.
template <typename T, int CT>
__global__ void __launch_bounds__(kBlock)
    k_schur_apply(const T* __restrict__ G, int rq, int gcols, int ccols, int nchunk,
                  const int* __restrict__ rank, int q, const T* __restrict__ Sinv, T* __restrict__ Yb) {
  __shared__ T Tc[2 * kRankCap32 * CT];
  const int i = blockIdx.x, c0 = blockIdx.y * CT, t = threadIdx.x, nt = blockDim.x;
  const int ra = rank[node_id(q, 2 * i)], rb = rank[node_id(q, 2 * i + 1)], r = ra + rb;
  const int lds = 2 * rq, nc = min(CT, ccols - c0);
  const size_t cs = (size_t)rq * gcols;  // one chunk's products
  const T* Ga = G + (size_t)(2 * i) * nchunk * cs;
  const T* Gb = G + (size_t)(2 * i + 1) * nchunk * cs;
  for (int e = t; e < r * CT; e += nt) {
    const int z = e % r, c = e / r;
    T v = T(0);
    if (c < nc) {
      const T* Gx = (z < rb) ? Ga + z : Gb + (z - rb);
      for (int ch = 0; ch < nchunk; ++ch) v += Gx[ch * cs + (size_t)(c0 + c) * rq];
    }
    Tc[z + c * r] = v;
  }
  __syncthreads();
  const T* S = Sinv + (size_t)i * lds * lds;
  T* Y = Yb + (size_t)i * lds * ccols;
  for (int x = t; x < r; x += nt) {
    T acc[CT];
#pragma unroll
    for (int c = 0; c < CT; ++c) acc[c] = T(0);
    int z = 0;
    for (; z + 8 <= r; z += 8) {
      T sv[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) sv[u] = S[x + (size_t)(z + u) * lds];
#pragma unroll
      for (int u = 0; u < 8; ++u)
#pragma unroll
        for (int c = 0; c < CT; ++c) acc[c] += sv[u] * Tc[z + u + c * r];
    }
    for (; z < r; ++z) {
      const T s = S[x + (size_t)z * lds];
#pragma unroll
      for (int c = 0; c < CT; ++c) acc[c] += s * Tc[z + c * r];
    }
    for (int c = 0; c < nc; ++c) Y[x + (size_t)(c0 + c) * lds] = acc[c];
  }
}

// k_schur_apply for levels of few parents and column chunks, where one
// thread per row leaves most of the GPU idle and each thread's inner loop is
// one long latency chain.  Workgroup (parent, CT-column chunk, row tiles z,
// z + gridDim.z, ... of 64
// rows of S): lane = row, the four waves take quarters of the inner range
// (16 loads of S in flight per thread), and their sums are added in quarter
// order through LDS.  The right-hand block T is gathered first, four entries
// by four split-K chunks per batch (each entry summed in chunk order).
template <typename T, int CT>
__global__ void __launch_bounds__(kBlock)
    k_schur_apply_tiles(const T* __restrict__ G, int rq, int gcols, int ccols, int nchunk,
                  const int* __restrict__ rank, int q, const T* __restrict__ Sinv, T* __restrict__ Yb) {
  static_assert(kBlock == 256, "four waves");
  constexpr int kU = 16, kE = 4, kH = 4;
  __shared__ T Tc[2 * kRankCap32 * CT];
  __shared__ T part[4][CT][64];
  const int i = blockIdx.x, c0 = blockIdx.y * CT, t = threadIdx.x, nt = blockDim.x;
  const int ra = rank[node_id(q, 2 * i)], rb = rank[node_id(q, 2 * i + 1)], r = ra + rb;
  if ((int)blockIdx.z * 64 >= r) return;  // (uniform)
  const int lds = 2 * rq, nc = min(CT, ccols - c0);
  const size_t cs = (size_t)rq * gcols;  // one chunk's products
  const T* Ga = G + (size_t)(2 * i) * nchunk * cs;
  const T* Gb = G + (size_t)(2 * i + 1) * nchunk * cs;
  const int ne = r * CT;
  for (int e0 = 0; e0 < ne; e0 += kE * nt) {
    const T* src[kE];
    bool ok[kE];
#pragma unroll
    for (int k = 0; k < kE; ++k) {
      const int e = min(e0 + t + k * nt, ne - 1), z = e % r, c = e / r;
      ok[k] = e0 + t + k * nt < ne && c < nc;
      src[k] = ((z < rb) ? Ga + z : Gb + (z - rb)) + (size_t)(c0 + min(c, nc - 1)) * rq;
    }
    T v[kE];
#pragma unroll
    for (int k = 0; k < kE; ++k) v[k] = T(0);
    for (int h0 = 0; h0 < nchunk; h0 += kH) {
      T g[kE][kH];
#pragma unroll
      for (int k = 0; k < kE; ++k)
#pragma unroll
        for (int u = 0; u < kH; ++u) g[k][u] = src[k][(size_t)min(h0 + u, nchunk - 1) * cs];
#pragma unroll
      for (int k = 0; k < kE; ++k)
#pragma unroll
        for (int u = 0; u < kH; ++u)
          if (h0 + u < nchunk) v[k] += g[k][u];
    }
#pragma unroll
    for (int k = 0; k < kE; ++k) {
      const int e = e0 + t + k * nt;
      if (e < ne) Tc[e] = ok[k] ? v[k] : T(0);  // Tc[z + c r] with e = z + c r
    }
  }
  __syncthreads();
  const int lane = t & 63, w = t >> 6;
  const int per = (r + 3) / 4, z0 = w * per, z1 = min(r, z0 + per);
  for (int x0 = blockIdx.z * 64; x0 < r; x0 += gridDim.z * 64) {  // (uniform)
    const int x = x0 + lane;
    const T* S = Sinv + (size_t)i * lds * lds + min(x, r - 1);
    T acc[CT];
#pragma unroll
    for (int c = 0; c < CT; ++c) acc[c] = T(0);
    for (int zb = z0; zb < z1; zb += kU) {
      T sv[kU];
#pragma unroll
      for (int u = 0; u < kU; ++u) sv[u] = S[(size_t)min(zb + u, z1 - 1) * lds];
#pragma unroll
      for (int u = 0; u < kU; ++u)
        if (zb + u < z1) {
#pragma unroll
          for (int c = 0; c < CT; ++c) acc[c] += sv[u] * Tc[zb + u + c * r];
        }
    }
#pragma unroll
    for (int c = 0; c < CT; ++c) part[w][c][lane] = acc[c];
    __syncthreads();
    if (w == 0 && x < r) {
      T* Y = Yb + (size_t)i * lds * ccols + x;
      for (int c = 0; c < nc; ++c)
        Y[(size_t)(c0 + c) * lds] = ((part[0][c][lane] + part[1][c][lane]) + part[2][c][lane]) + part[3][c][lane];
    }
    __syncthreads();  // part is rewritten by the next tile
  }
}

// Z(rows c, 0:zcols) -= d_c * y_other for every node c of level q, where d_c =
// Y(rows c, offq : offq + r_c) and y_other is the part of the parent's y that
// multiplies it: y_b (rows r_b .. r_b + r_a) for a left child, y_a (rows
// 0 .. r_b) for a right child.
template <typename T, int CT>
__global__ void __launch_bounds__(kBlock)
    k_correct(const T* __restrict__ Yd, int ldy, int offq, T* __restrict__ Z, int ldz, int zcols,
              const T* __restrict__ Yb, int rq, const int* __restrict__ lo,
              const int* __restrict__ hi, const int* __restrict__ rank, int q) {
  __shared__ T Yo[kRankCap32 * CT];
  const int c = blockIdx.x, par = c >> 1, left = (c & 1) == 0, t = threadIdx.x;
  const int id = node_id(q, c);
  const int ra = rank[node_id(q, 2 * par)], rb = rank[node_id(q, 2 * par + 1)];
  const int rc = left ? ra : rb, yoff = left ? rb : 0, lds = 2 * rq;
  const int c0 = blockIdx.z * CT, nc = min(CT, zcols - c0);
  const T* Yp = Yb + (size_t)par * lds * zcols;
  for (int e = t; e < rc * CT; e += blockDim.x) {
    const int l = e % rc, k = e / rc;
    Yo[l + k * rc] = (k < nc) ? Yp[(yoff + l) + (size_t)(c0 + k) * lds] : T(0);
  }
  __syncthreads();
  const int row = lo[id] + blockIdx.y * blockDim.x + t;
  if (row >= hi[id] || rc == 0) return;
  T acc[CT];
#pragma unroll
  for (int k = 0; k < CT; ++k) acc[k] = T(0);
  int l = 0;
  for (; l + 8 <= rc; l += 8) {
    T d[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) d[u] = Yd[(size_t)(offq + l + u) * ldy + row];
#pragma unroll
    for (int u = 0; u < 8; ++u)
#pragma unroll
      for (int k = 0; k < CT; ++k) acc[k] += d[u] * Yo[l + u + k * rc];
  }
  for (; l < rc; ++l) {
    const T d = Yd[(size_t)(offq + l) * ldy + row];
#pragma unroll
    for (int k = 0; k < CT; ++k) acc[k] += d * Yo[l + k * rc];
  }
  for (int k = 0; k < nc; ++k) Z[(size_t)(c0 + k) * ldz + row] -= acc[k];
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
static inline int cdiv(int a, int b) { return (a + b - 1) / b; }

template <typename F>
static int allow_lds(F kernel, size_t bytes) {
  if (bytes > 64 * 1024)
    HODLR_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
  return HODLR_OK;
}

int ensure_work(hodlr_s* h, int ncols) {
  const Tree& t = h->tree;
  ncols = std::max(ncols, 64);
  size_t g = 1, y = 1;
  for (int q = 1; q <= t.L; ++q) {
    size_t rq = h->rcols.empty() ? 0 : h->rcols[q - 1];
    size_t offq = h->off.empty() ? 0 : h->off[q - 1];
    g = std::max(g, (size_t)(1 << q) * rq * (offq + rq));
    y = std::max(y, (size_t)(1 << (q - 1)) * 2 * rq * std::max<size_t>(offq, ncols));
  }
  // the fused solve keeps two buffers of unit partial products in G
  h->p_half = solve_partial_elems(h);
  g = std::max(g, 2 * h->p_half);
  HODLR_TRY(h->Xtmp.ensure((size_t)t.n * 16 * h->esize));
  HODLR_TRY(h->G.ensure(g * h->esize));
  HODLR_TRY(h->Ybuf.ensure(y * h->esize));
  return HODLR_OK;
}

int launch_leaf_inverse(hodlr_s* h, int* status, hipStream_t s) {
  const Tree& t = h->tree;
  k_fill_int<<<1, 64, 0, s>>>(status, 4, 0);
  HODLR_HIP(hipGetLastError());
  ProfScope prof_("leaf_inverse", s);
  if (h->precision == 64)
    k_leaf_inverse<double><<<h->nleaf, gj_threads<double>(), 0, s>>>(h->Kinv.as<double>(), h->bmax, h->d_lo.as<int>(),
                                                       h->d_hi.as<int>(), node_id(t.L, 0), status);
  else
    k_leaf_inverse<float><<<h->nleaf, gj_threads<float>(), 0, s>>>(h->Kinv.as<float>(), h->bmax, h->d_lo.as<int>(),
                                                      h->d_hi.as<int>(), node_id(t.L, 0), status);
  HODLR_HIP(hipGetLastError());
  return HODLR_OK;
}

template <typename T>
static int stage_from_K(hodlr_s* h, const double* K, int ldk, hipStream_t s) {
  const Tree& t = h->tree;
  dim3 grid(cdiv(h->bmax * h->bmax, kBlock), h->nleaf);
  k_stage_leaves_K<T><<<grid, kBlock, 0, s>>>(K, ldk, h->d_lo.as<int>(), h->d_hi.as<int>(),
                                              node_id(t.L, 0), h->bmax, h->Kinv.as<T>());
  HODLR_HIP(hipGetLastError());
  return HODLR_OK;
}

int launch_stage_leaves_from_K(hodlr_s* h, const double* K, int ldk, hipStream_t s) {
  return h->precision == 64 ? stage_from_K<double>(h, K, ldk, s) : stage_from_K<float>(h, K, ldk, s);
}

template <typename T>
static int stage_packed(hodlr_s* h, const double* leaves, hipStream_t s) {
  const Tree& t = h->tree;
  dim3 grid(cdiv(h->bmax * h->bmax, kBlock), h->nleaf);
  k_stage_leaves_packed<T><<<grid, kBlock, 0, s>>>(leaves, h->d_lo.as<int>(), h->d_hi.as<int>(),
                                                   node_id(t.L, 0), h->bmax, h->Kinv.as<T>());
  HODLR_HIP(hipGetLastError());
  return HODLR_OK;
}

int launch_stage_leaves_packed(hodlr_s* h, const double* leaves, hipStream_t s) {
  return h->precision == 64 ? stage_packed<double>(h, leaves, s) : stage_packed<float>(h, leaves, s);
}

// Copies every level's rq columns of the capped panels (column block capoff,
// leading dimension ldcap) into the packed panels Y / W (column block off,
// leading dimension n): workgroup row y is packed column y, z picks U or V.
constexpr int kRepackLevels = 32;
struct RepackCols {
  int L;
  int off[kRepackLevels], cap[kRepackLevels];
};

template <typename T>
__global__ void __launch_bounds__(kBlock)
    k_repack(const T* __restrict__ Ucap, const T* __restrict__ Vcap, int ldcap, T* __restrict__ Y,
             T* __restrict__ W, int n, const RepackCols rc) {
  const int j = blockIdx.y;
  int q = 0;
  while (q + 1 < rc.L && j >= rc.off[q + 1]) ++q;
  const size_t src = (size_t)(rc.cap[q] + j - rc.off[q]) * ldcap;
  const T* sp = blockIdx.z ? Vcap : Ucap;
  T* dp = (blockIdx.z ? W : Y) + (size_t)j * n;
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) dp[i] = sp[src + i];
}

int launch_repack(hodlr_s* h, const void* Ucap, const void* Vcap, int ldcap,
                  const std::vector<int>& capoff, hipStream_t s) {
  const Tree& t = h->tree;
  if (t.L > kRepackLevels) return fail(HODLR_EINVAL, "tree deeper than the repack supports");
  if (h->R == 0) return HODLR_OK;
  RepackCols rc{};
  rc.L = t.L;
  for (int q = 1; q <= t.L; ++q) {
    rc.off[q - 1] = h->off[q - 1];
    rc.cap[q - 1] = capoff[q - 1];
  }
  const dim3 grid(std::min(cdiv(t.n, kBlock), 16), h->R, 2);
  if (h->precision == 64)
    k_repack<double><<<grid, kBlock, 0, s>>>(static_cast<const double*>(Ucap), static_cast<const double*>(Vcap),
                                            ldcap, h->Y.as<double>(), h->W.as<double>(), t.n, rc);
  else
    k_repack<float><<<grid, kBlock, 0, s>>>(static_cast<const float*>(Ucap), static_cast<const float*>(Vcap), ldcap,
                                           h->Y.as<float>(), h->W.as<float>(), t.n, rc);
  HODLR_HIP(hipGetLastError());
  return HODLR_OK;
}

// Symmetric build: the block of every right child s is the transpose of its
// left sibling c's, K(s, c) = K(c, s)^T ~ V_c U_c^T, so U_s = V_c and
// V_s = U_c.  In the panels U_s sits in Y and V_c in W at the rows of s, V_s
// in W and U_c in Y at the rows of c.  For column j of level p: rows of a
// right child take Y(i, j) = W(i, j), rows of a left child W(i, j) = Y(i, j),
// for j - off_p < rank(c); the level's other columns become zero there.  The
// first workgroup also gives every right child its sibling's rank.
template <typename T>
__global__ void __launch_bounds__(kBlock)
    k_mirror(T* __restrict__ Y, T* __restrict__ W, int n, const int* __restrict__ lo, int* __restrict__ rank,
             int nnodes, const RepackCols rc) {
  const int j = blockIdx.y;
  if (j == 0 && blockIdx.x == 0)
    for (int id = 2 + 2 * threadIdx.x; id < nnodes; id += 2 * kBlock) rank[id] = rank[id - 1];
  int q = 0;
  while (q + 1 < rc.L && j >= rc.off[q + 1]) ++q;
  const int p = q + 1, jj = j - rc.off[q];
  const int first = node_id(p, 0), cnt = 1 << p;
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
    // the node of level p holding row i: the last one with lo <= i
    int a = 0, b = cnt - 1;
    while (a < b) {
      const int m = (a + b + 1) >> 1;
      if (lo[first + m] <= i) a = m;
      else b = m - 1;
    }
    const bool keep = jj < rank[first + (a & ~1)];
    const size_t e = (size_t)j * n + i;
    if (a & 1) Y[e] = keep ? W[e] : T(0);
    else W[e] = keep ? Y[e] : T(0);
  }
}

int launch_mirror(hodlr_s* h, hipStream_t s) {
  const Tree& t = h->tree;
  if (t.L > kRepackLevels) return fail(HODLR_EINVAL, "tree deeper than the repack supports");
  if (h->R == 0) return HODLR_OK;
  RepackCols rc{};
  rc.L = t.L;
  for (int q = 1; q <= t.L; ++q) rc.off[q - 1] = h->off[q - 1];
  const dim3 grid(std::min(cdiv(t.n, kBlock), 16), h->R);
  if (h->precision == 64)
    k_mirror<double><<<grid, kBlock, 0, s>>>(h->Y.as<double>(), h->W.as<double>(), t.n, h->d_lo.as<int>(),
                                            h->d_rank.as<int>(), t.nnodes(), rc);
  else
    k_mirror<float><<<grid, kBlock, 0, s>>>(h->Y.as<float>(), h->W.as<float>(), t.n, h->d_lo.as<int>(),
                                           h->d_rank.as<int>(), t.nnodes(), rc);
  HODLR_HIP(hipGetLastError());
  return HODLR_OK;
}

template <typename S, typename D>
static int convert(const S* src, D* dst, size_t count, hipStream_t s) {
  if (count == 0) return HODLR_OK;
  const int grid = (int)std::min<size_t>((count + kBlock - 1) / kBlock, 4096);
  k_convert<S, D><<<grid, kBlock, 0, s>>>(src, dst, count);
  HODLR_HIP(hipGetLastError());
  return HODLR_OK;
}

int launch_from_f64_panels(hodlr_s* h, const double* Up, const double* Vp, hipStream_t s) {
  const size_t cnt = (size_t)h->tree.n * h->R;
  if (h->precision == 64) {
    HODLR_HIP(hipMemcpyAsync(h->Y.p, Up, cnt * 8, hipMemcpyDeviceToDevice, s));
    HODLR_HIP(hipMemcpyAsync(h->W.p, Vp, cnt * 8, hipMemcpyDeviceToDevice, s));
    return HODLR_OK;
  }
  HODLR_TRY(convert(Up, h->Y.as<float>(), cnt, s));
  return convert(Vp, h->W.as<float>(), cnt, s);
}

int launch_to_f64_panels(hodlr_s* h, double* Up, double* Vp, hipStream_t s) {
  const size_t cnt = (size_t)h->tree.n * h->R;
  if (h->precision == 64) {
    HODLR_HIP(hipMemcpyAsync(Up, h->Y.p, cnt * 8, hipMemcpyDeviceToDevice, s));
    HODLR_HIP(hipMemcpyAsync(Vp, h->W.p, cnt * 8, hipMemcpyDeviceToDevice, s));
    return HODLR_OK;
  }
  HODLR_TRY(convert(h->Y.as<float>(), Up, cnt, s));
  return convert(h->W.as<float>(), Vp, cnt, s);
}

constexpr int kCT = 8;  // columns per workgroup in the leaf / Woodbury kernels

template <typename T>
static int level_solve(hodlr_s* h, int q, T* Z, int ldz, int zcols, const T* G, int gcols,
                       int nchunk, hipStream_t s) {
  // y = S^-1 t for every parent, then the corrections of the level-q nodes
  const Tree& t = h->tree;
  const int rq = h->rcols[q - 1], offq = h->off[q - 1];
  const T* Sinv = h->Sinv.as<T>() + h->sinv_off[q - 1];
  T* Yb = h->Ybuf.as<T>();
  {
    ProfScope prof_("schur_apply", s);
    // few parents x column chunks: rows split over 64-row tiles and inner
    // quarters (measured faster below 256 workgroups, slower above)
    const dim3 grid(1 << (q - 1), cdiv(zcols, kCT));
    if (grid.x * grid.y < 256)
      k_schur_apply_tiles<T, kCT><<<dim3(grid.x, grid.y, cdiv(2 * rq, 64)), kBlock, 0, s>>>(
          G, rq, gcols, zcols, nchunk, h->d_rank.as<int>(), q, Sinv, Yb);
    else
      k_schur_apply<T, kCT><<<grid, kBlock, 0, s>>>(G, rq, gcols, zcols, nchunk, h->d_rank.as<int>(), q, Sinv, Yb);
  }
  HODLR_HIP(hipGetLastError());
  {
    ProfScope prof_("correct", s);
    k_correct<T, kCT><<<dim3(1 << q, cdiv(t.max_size(q), kBlock), cdiv(zcols, kCT)), kBlock, 0, s>>>(
        h->Y.as<T>(), t.n, offq, Z, ldz, zcols, Yb, rq, h->d_lo.as<int>(), h->d_hi.as<int>(),
        h->d_rank.as<int>(), q);
  }
  HODLR_HIP(hipGetLastError());
  return HODLR_OK;
}

// The Woodbury steps of every level, leaves up (Sec. 4.2-4.3).  With rec the
// pass only records the batched products (their task tables), launching
// nothing; the launching pass then replays them in the same order.
template <typename T>
static int factor_levels(hodlr_s* h, hipStream_t s, bool rec) {
  const Tree& t = h->tree;
  const int n = t.n, L = t.L;
  T* Y = h->Y.as<T>();
  const T* W = h->W.as<T>();
  for (int q = L; q >= 1; --q) {
    const int rq = h->rcols[q - 1], offq = h->off[q - 1];
    if (rq == 0) continue;
    const int zc = offq + rq, lds = 2 * rq, np = 1 << (q - 1);
    T* G = h->G.as<T>();
    T* Sq = h->Sinv.as<T>() + h->sinv_off[q - 1];
    std::vector<GemmTask> gt;
    // panel products G_c = V_sib^T Z_c (V of the sibling is stored in c's rows)
    {
      int tiles = 0, kmax = 1;
      for (int c = 0; c < (1 << q); ++c) {
        const int rs = h->rank[node_id(q, c ^ 1)];
        tiles += ((rs + 63) / 64) * ((zc + 63) / 64);
        kmax = std::max(kmax, t.size(node_id(q, c)));
      }
      const int ks = std::max(1, std::min((256 + tiles - 1) / std::max(tiles, 1), kmax / 128));
      for (int c = 0; c < (1 << q); ++c) {
        const int id = node_id(q, c);
        GemmTask g;
        g.A = W + (size_t)offq * n + t.lo[id];
        g.lda = n;
        g.transA = 1;
        g.B = Y + t.lo[id];
        g.ldb = n;
        g.C = G + (size_t)c * rq * zc;
        g.ldc = rq;
        g.m = h->rank[node_id(q, c ^ 1)];
        g.n = zc;
        g.k = t.size(id);
        g.ksplit = ks;
        gt.push_back(g);
      }
      ProfScope prof_("panel_tn", s, !rec);
      HODLR_TRY(gemm_batched(h, gt, s));
    }
    // S22 <- M = I - B A, then M^-1 in place
    gt.clear();
    for (int i = 0; i < np; ++i) {
      const int ra = h->rank[node_id(q, 2 * i)], rb = h->rank[node_id(q, 2 * i + 1)];
      T* S = Sq + (size_t)i * lds * lds;
      GemmTask g;
      g.A = G + (size_t)(2 * i + 1) * rq * zc + (size_t)offq * rq;  // B: r_a x r_b
      g.lda = rq;
      g.B = G + (size_t)(2 * i) * rq * zc + (size_t)offq * rq;      // A: r_b x r_a
      g.ldb = rq;
      g.C = S + rb + (size_t)rb * lds;
      g.ldc = lds;
      g.m = ra;
      g.n = ra;
      g.k = rb;
      g.alpha = -1.0;
      g.mode = kGemmAddIdentity;
      gt.push_back(g);
    }
    {
      {
        ProfScope prof_("schur_form", s, !rec);
        HODLR_TRY(gemm_batched(h, gt, s));
      }
      if (!rec) {
        ProfScope prof_("cap_inverse", s);
        k_capacitance_inverse<T><<<np, gj_threads<T>(), 0, s>>>(h->d_rank.as<int>(), q, rq, Sq, h->status.as<int>());
        HODLR_HIP(hipGetLastError());
      }
      ProfScope prof_("schur_form", s, !rec);
      // S21 = -M^-1 B, S12 = -A M^-1
      gt.clear();
      for (int i = 0; i < np; ++i) {
        const int ra = h->rank[node_id(q, 2 * i)], rb = h->rank[node_id(q, 2 * i + 1)];
        T* S = Sq + (size_t)i * lds * lds;
        const T* Am = G + (size_t)(2 * i) * rq * zc + (size_t)offq * rq;
        const T* Bm = G + (size_t)(2 * i + 1) * rq * zc + (size_t)offq * rq;
        const T* S22 = S + rb + (size_t)rb * lds;
        GemmTask g;
        g.alpha = -1.0;
        g.A = S22;
        g.lda = lds;
        g.B = Bm;
        g.ldb = rq;
        g.C = S + rb;
        g.ldc = lds;
        g.m = ra;
        g.n = rb;
        g.k = ra;
        gt.push_back(g);
        g.A = Am;
        g.lda = rq;
        g.B = S22;
        g.ldb = lds;
        g.C = S + (size_t)rb * lds;
        g.m = rb;
        g.n = ra;
        g.k = ra;
        gt.push_back(g);
      }
      HODLR_TRY(gemm_batched(h, gt, s));
      // S11 = I - A S21
      gt.clear();
      for (int i = 0; i < np; ++i) {
        const int ra = h->rank[node_id(q, 2 * i)], rb = h->rank[node_id(q, 2 * i + 1)];
        T* S = Sq + (size_t)i * lds * lds;
        GemmTask g;
        g.alpha = -1.0;
        g.mode = kGemmAddIdentity;
        g.A = G + (size_t)(2 * i) * rq * zc + (size_t)offq * rq;
        g.lda = rq;
        g.B = S + rb;
        g.ldb = lds;
        g.C = S;
        g.ldc = lds;
        g.m = rb;
        g.n = rb;
        g.k = ra;
        gt.push_back(g);
      }
      HODLR_TRY(gemm_batched(h, gt, s));
    }
    // E_c = d_c S^-1(y rows of c, :): rows r_b.. for a left child, 0.. for a right one
    gt.clear();
    for (int c = 0; c < (1 << q); ++c) {
      const int par = c >> 1, left = (c & 1) == 0, id = node_id(q, c);
      const int ra = h->rank[node_id(q, 2 * par)], rb = h->rank[node_id(q, 2 * par + 1)];
      const int rc = left ? ra : rb, yoff = left ? rb : 0;
      if (ra + rb == 0) continue;
      GemmTask g;
      g.A = Y + (size_t)offq * n + t.lo[id];
      g.lda = n;
      g.B = Sq + (size_t)par * lds * lds + yoff;
      g.ldb = lds;
      g.C = h->E.as<T>() + (size_t)h->offE[q - 1] * n + t.lo[id];
      g.ldc = n;
      g.m = t.size(id);
      g.n = ra + rb;
      g.k = rc;
      gt.push_back(g);
    }
    {
      ProfScope prof_("form_E", s, !rec);
      HODLR_TRY(gemm_batched(h, gt, s));
    }
    if (offq > 0 && !rec) HODLR_TRY(level_solve<T>(h, q, Y, n, offq, G, zc, 1, s));
  }
  return HODLR_OK;
}

// Restores direct batched products when a factorization ends, also on error.
struct GemmModeGuard {
  hodlr_s* h;
  ~GemmModeGuard() {
    h->gemm_mode = kGemmDirect;
    h->gemm_recs.clear();
    h->gemm_rec_pos = 0;
    h->gemm_staged = 0;
  }
};

template <typename T>
static int factor_t(hodlr_s* h, hipStream_t s) {
  const Tree& t = h->tree;  // (tree)
  const int n = t.n, L = t.L;
  // The leaf work needs no batched-product table: it is queued first, so the
  // GPU runs it while the host plans the products of every level.
  k_fill_int<<<1, 64, 0, s>>>(h->status.as<int>(), 4, 0);
  HODLR_HIP(hipGetLastError());
  if (!h->leaves_inverted) {  // (the build may have run them beside the compression)
    ProfScope prof_("leaf_inverse", s);
    k_leaf_inverse<T><<<h->nleaf, gj_threads<T>(), 0, s>>>(h->Kinv.as<T>(), h->bmax, h->d_lo.as<int>(),
                                                         h->d_hi.as<int>(), node_id(L, 0),
                                                         h->status.as<int>());
  }
  HODLR_HIP(hipGetLastError());
  if (L == 0 || h->R == 0) return HODLR_OK;
  T* Y = h->Y.as<T>();
  {
    ProfScope prof_("leaf_apply", s);
    const size_t lds = leaf_apply_mfma_lds(h->bmax);
    if (sizeof(T) == 4 && lds <= 160 * 1024) {
      HODLR_TRY(allow_lds(k_leaf_apply_mfma, lds));
      k_leaf_apply_mfma<<<dim3(h->nleaf, cdiv(h->R, 64)), kBlock, lds, s>>>(
          reinterpret_cast<const float*>(h->Kinv.p), h->bmax, h->d_lo.as<int>(), h->d_hi.as<int>(), node_id(L, 0),
          reinterpret_cast<float*>(Y), n, h->R);
    } else {
      k_leaf_apply<T, kCT><<<dim3(h->nleaf, cdiv(h->R, kCT)), kBlock, 0, s>>>(
          h->Kinv.as<T>(), h->bmax, h->d_lo.as<int>(), h->d_hi.as<int>(), node_id(L, 0), Y, n, h->R);
    }
  }
  // every buffer is sized before the first product: the sequence below has
  // no allocation, synchronization or pageable copy once the buffers are
  // sized, so it can be recorded into a graph (hodlr_factor_batched, which
  // sizes them first)
  if (L > 0 && h->R > 0) {
    HODLR_TRY(ensure_work(h, 64));
    size_t tb = 0, wb = 0;
    for (int q = 1; q <= L; ++q) {
      const size_t rq = h->rcols[q - 1], zc = h->off[q - 1] + rq, nq = (size_t)1 << q;
      tb += 3 * gemm_table_bound((int)nq) + 2 * gemm_table_bound((int)nq / 2);
      wb += nq * rq * zc * (size_t)std::max(1, t.max_size(q) / 128) * h->esize + 256;
    }
    HODLR_TRY(gemm_prepare(h, tb, wb, s));
  }
  GemmModeGuard guard_{h};
  // record every batched product of the factorization, then move all their
  // task tables with one copy
  for (int attempt = 0;; ++attempt) {
    gemm_reset(h);
    h->gemm_recs.clear();
    h->gemm_staged = 0;
    h->gemm_replan = false;
    h->gemm_mode = kGemmRecord;
    if (L > 0 && h->R > 0) HODLR_TRY(factor_levels<T>(h, s, true));
    if (!h->gemm_replan) break;
    if (attempt >= 3) return fail(HODLR_EINVAL, "batched-product arenas keep growing");
  }
  HODLR_TRY(gemm_upload(h, s));
  h->gemm_mode = kGemmReplay;
  h->gemm_rec_pos = 0;
  HODLR_HIP(hipGetLastError());
  HODLR_TRY(factor_levels<T>(h, s, false));
  if (h->gemm_rec_pos != h->gemm_recs.size()) return fail(HODLR_EINVAL, "batched products replayed out of step");
  return HODLR_OK;
}

int factor_impl(hodlr_s* h, hipStream_t s) {
  return h->precision == 64 ? factor_t<double>(h, s) : factor_t<float>(h, s);
}

}  // namespace hodlr
