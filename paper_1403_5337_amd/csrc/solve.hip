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
// Rows are processed in units of kRows = 64 rows.  Launch "leaf" computes
// x = Kinv_leaf x for one unit and writes the unit's partial products
// W(unit rows, level-L block)^T x; launch "level q" (one workgroup per
// level-q node and unit) adds the partial products of both siblings into
// t_P, applies x -= E t_P to its unit, and writes the unit's partial products
// for level q-1.  Every operand tile goes through LDS with all its loads in
// flight together.
#include <algorithm>

#include "device_util.h"
#include "hodlr_internal.h"

namespace hodlr {

constexpr int kRows = 64;          // rows per unit
constexpr int kTileC = 64;         // columns per staged tile
constexpr int kLdT = kRows + 1;    // LDS leading dimension of a tile
constexpr int kLeafLds = 192;      // >= largest leaf

// dst(i, c) = src(i, c) for i < rn, c < cn (zero elsewhere); src column-major
// with leading dimension ld; dst in LDS with leading dimension kLdT.
template <typename T>
__device__ __forceinline__ void stage_tile(T* dst, const T* __restrict__ src, size_t ld, int rn, int cn) {
  constexpr int total = kRows * kTileC;
  constexpr int per = total / kBlock;  // 16 loads per thread, issued together
  const int t = threadIdx.x;
  T v[per];
#pragma unroll
  for (int u = 0; u < per; ++u) {
    const int e = t + u * kBlock, i = e & (kRows - 1), c = e / kRows;
    v[u] = (i < rn && c < cn) ? src[i + (size_t)c * ld] : T(0);
  }
#pragma unroll
  for (int u = 0; u < per; ++u) {
    const int e = t + u * kBlock;
    dst[(e & (kRows - 1)) + (e / kRows) * kLdT] = v[u];
  }
}

// Pu(r, c) = sum_i W(row0 + i, r) xs(i, c) for r < rp, c < nc: the unit's
// partial products.  Wsrc points at W(row0, first column of the block).
template <typename T, int SM>
__device__ void unit_out(T* tile, const T* xs, const T* __restrict__ Wsrc, size_t ldw, int rn, int rp,
                         int nc, T* __restrict__ Pu) {
  const int t = threadIdx.x, rr = t & (kRows - 1), cg = t / kRows;
  for (int r0 = 0; r0 < rp; r0 += kTileC) {
    const int cn = min(kTileC, rp - r0);
    stage_tile(tile, Wsrc + (size_t)r0 * ldw, ldw, rn, cn);
    __syncthreads();
    if (rr < cn) {
      T acc[SM / 4];
#pragma unroll
      for (int u = 0; u < SM / 4; ++u) acc[u] = T(0);
      for (int i = 0; i < kRows; ++i) {
        const T w = tile[i + rr * kLdT];
#pragma unroll
        for (int u = 0; u < SM / 4; ++u) acc[u] += w * xs[(cg + 4 * u) * kRows + i];
      }
#pragma unroll
      for (int u = 0; u < SM / 4; ++u) {
        const int c = cg + 4 * u;
        if (c < nc) Pu[(r0 + rr) + (size_t)c * rp] = acc[u];
      }
    }
    __syncthreads();
  }
}

template <typename T, int SM>
__global__ void __launch_bounds__(kBlock)
    k_solve_leaf(const T* __restrict__ Kinv, int bmax, const int* __restrict__ lo,
                 const int* __restrict__ hi, int idL, const T* __restrict__ Xin, int ldxi,
                 T* __restrict__ Xout, int ldxo, int nc, const T* __restrict__ W, int ldw, int offL,
                 int rL, int nchL, T* __restrict__ P) {
  __shared__ T xs[SM * kLeafLds];
  __shared__ T tile[kLdT * kTileC];
  __shared__ T ys[SM * kRows];
  const int leaf = blockIdx.x, ch = blockIdx.y, id = idL + leaf, t = threadIdx.x;
  const int l0 = lo[id], b = hi[id] - l0, row0 = ch * kRows, rn = min(kRows, b - row0);
  T* Pu = P + ((size_t)leaf * nchL + ch) * rL * nc;
  if (rn <= 0) {
    for (int e = t; e < rL * nc; e += blockDim.x) Pu[e] = T(0);
    return;
  }
  for (int e0 = 0; e0 < SM * kLeafLds; e0 += 8 * kBlock) {
    T v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = e0 + t + u * kBlock, i = e % kLeafLds, c = e / kLeafLds;
      v[u] = (e < SM * kLeafLds && i < b && c < nc) ? Xin[(size_t)c * ldxi + l0 + i] : T(0);
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = e0 + t + u * kBlock;
      if (e < SM * kLeafLds) xs[e] = v[u];
    }
  }
  const T* Ki = Kinv + (size_t)leaf * bmax * bmax + row0;
  const int ii = t & (kRows - 1), cg = t / kRows;
  T acc[SM / 4];
#pragma unroll
  for (int u = 0; u < SM / 4; ++u) acc[u] = T(0);
  for (int k0 = 0; k0 < b; k0 += kTileC) {
    const int kn = min(kTileC, b - k0);
    stage_tile(tile, Ki + (size_t)k0 * bmax, bmax, rn, kn);
    __syncthreads();
    for (int kk = 0; kk < kn; ++kk) {
      const T a = tile[ii + kk * kLdT];
#pragma unroll
      for (int u = 0; u < SM / 4; ++u) acc[u] += a * xs[(cg + 4 * u) * kLeafLds + k0 + kk];
    }
    __syncthreads();
  }
#pragma unroll
  for (int u = 0; u < SM / 4; ++u) {
    const int c = cg + 4 * u;
    const bool ok = ii < rn && c < nc;
    if (ok) Xout[(size_t)c * ldxo + l0 + row0 + ii] = acc[u];
    ys[c * kRows + ii] = ok ? acc[u] : T(0);
  }
  __syncthreads();
  if (rL > 0) unit_out<T, SM>(tile, ys, W + (size_t)offL * ldw + l0 + row0, ldw, rn, rL, nc, Pu);
}

template <typename T, int SM>
__global__ void __launch_bounds__(kBlock)
    k_solve_level(int q, const int* __restrict__ lo, const int* __restrict__ hi,
                  const int* __restrict__ rank, const T* Xin, int ldxi, T* Xout, int ldxo, int nc,
                  const T* __restrict__ E, int ldE, int offE, int rq, const T* __restrict__ Pin, int upn,
                  int nch, const T* __restrict__ W, int ldw, int offp, int rp, T* __restrict__ Pout) {
  constexpr int RC = sizeof(T) == 8 ? kRankCap64 : kRankCap32;
  __shared__ T tcat[2 * RC * SM];
  __shared__ T tile[kLdT * kTileC];
  __shared__ T xs[SM * kRows];
  const int c = blockIdx.x, ch = blockIdx.y, t = threadIdx.x, nt = blockDim.x;
  const int par = c >> 1, id = node_id(q, c);
  const int ra = rank[node_id(q, 2 * par)], rb = rank[node_id(q, 2 * par + 1)], r = ra + rb;
  const int row0 = lo[id] + ch * kRows, rn = min(kRows, hi[id] - row0);
  T* Pu = Pout ? Pout + ((size_t)c * nch + ch) * rp * nc : nullptr;
  if (rn <= 0) {
    if (Pu)
      for (int e = t; e < rp * nc; e += nt) Pu[e] = T(0);
    return;
  }
  // t_P = [W(rows a)^T x_a (r_b entries); W(rows b)^T x_b (r_a entries)]
  const size_t us = (size_t)rq * nc;
  for (int e = t; e < r * nc; e += nt) {
    const int z = e % r, cc = e / r;
    const int node = (z < rb) ? 2 * par : 2 * par + 1;
    const int zz = (z < rb) ? z : z - rb;
    const T* P0 = Pin + (size_t)node * upn * us + zz + (size_t)cc * rq;
    T v = T(0);
    int u = 0;
    for (; u + 8 <= upn; u += 8) {
      T pv[8];
#pragma unroll
      for (int x = 0; x < 8; ++x) pv[x] = P0[(u + x) * us];
#pragma unroll
      for (int x = 0; x < 8; ++x) v += pv[x];
    }
    for (; u < upn; ++u) v += P0[u * us];
    tcat[z + cc * r] = v;
  }
  // x(unit) -= E(unit, :) t_P
  const int ii = t & (kRows - 1), cg = t / kRows;
  T acc[SM / 4];
#pragma unroll
  for (int u = 0; u < SM / 4; ++u) acc[u] = T(0);
  const T* Eu = E + (size_t)offE * ldE + row0;
  for (int z0 = 0; z0 < r; z0 += kTileC) {
    const int zn = min(kTileC, r - z0);
    stage_tile(tile, Eu + (size_t)z0 * ldE, ldE, rn, zn);
    __syncthreads();
    for (int zz = 0; zz < zn; ++zz) {
      const T e = tile[ii + zz * kLdT];
#pragma unroll
      for (int u = 0; u < SM / 4; ++u) acc[u] += e * tcat[z0 + zz + (cg + 4 * u) * r];
    }
    __syncthreads();
  }
#pragma unroll
  for (int u = 0; u < SM / 4; ++u) {
    const int cc = cg + 4 * u;
    T v = T(0);
    if (ii < rn && cc < nc) {
      v = Xin[(size_t)cc * ldxi + row0 + ii] - acc[u];
      Xout[(size_t)cc * ldxo + row0 + ii] = v;
    }
    xs[cc * kRows + ii] = v;
  }
  __syncthreads();
  if (Pu && rp > 0) unit_out<T, SM>(tile, xs, W + (size_t)offp * ldw + row0, ldw, rn, rp, nc, Pu);
}

// ---------------------------------------------------------------------------
static inline int cdiv(int a, int b) { return (a + b - 1) / b; }

// Units per level-q node: q = L -> its own units; q < L -> its children's.
static int units_per_node(const Tree& t, int q) {
  return q == t.L ? cdiv(t.max_size(t.L), kRows) : 2 * cdiv(t.max_size(q + 1), kRows);
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
static int solve_t(hodlr_s* h, T* X, int ldx, int nc, hipStream_t s) {
  const Tree& t = h->tree;
  const int n = t.n, L = t.L;
  T* P[2] = {h->G.as<T>(), h->G.as<T>() + h->p_half};
  T* Xt = h->Xtmp.as<T>();
  const int rL = L > 0 ? h->rcols[L - 1] : 0, offL = L > 0 ? h->off[L - 1] : 0;
  const int nchL = cdiv(h->bmax, kRows);
  {
    ProfScope prof_("apply_leaf", s);
    k_solve_leaf<T, SM><<<dim3(h->nleaf, nchL), kBlock, 0, s>>>(
        h->Kinv.as<T>(), h->bmax, h->d_lo.as<int>(), h->d_hi.as<int>(), node_id(L, 0), X, ldx, Xt, n, nc,
        h->W.as<T>(), n, offL, rL, nchL, P[0]);
  }
  HODLR_HIP(hipGetLastError());
  int cur = 0;
  for (int q = L; q >= 1; --q) {
    const int rq = h->rcols[q - 1];
    const int nch = cdiv(t.max_size(q), kRows);
    const int rp = q > 1 ? h->rcols[q - 2] : 0, offp = q > 1 ? h->off[q - 2] : 0;
    T* Xo = (q == 1) ? X : Xt;
    const int ldo = (q == 1) ? ldx : n;
    {
      ProfScope prof_("apply_level", s);
      k_solve_level<T, SM><<<dim3(1 << q, nch), kBlock, 0, s>>>(
          q, h->d_lo.as<int>(), h->d_hi.as<int>(), h->d_rank.as<int>(), Xt, n, Xo, ldo, nc, h->E.as<T>(), n,
          h->offE[q - 1], rq, P[cur], units_per_node(t, q), nch, h->W.as<T>(), n, offp, rp,
          q > 1 ? P[cur ^ 1] : nullptr);
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
static int apply_t(hodlr_s* h, T* X, int ldx, int nrhs, hipStream_t s) {
  for (int c0 = 0; c0 < nrhs; c0 += 16) {
    const int nc = std::min(16, nrhs - c0);
    T* Xc = X + (size_t)c0 * ldx;
    if (nc <= 8) HODLR_TRY((solve_t<T, 8>(h, Xc, ldx, nc, s)));
    else HODLR_TRY((solve_t<T, 16>(h, Xc, ldx, nc, s)));
  }
  return HODLR_OK;
}

int apply_impl(hodlr_s* h, void* X, int ldx, int nrhs, hipStream_t s) {
  return h->precision == 64 ? apply_t<double>(h, static_cast<double*>(X), ldx, nrhs, s)
                            : apply_t<float>(h, static_cast<float*>(X), ldx, nrhs, s);
}

}  // namespace hodlr
