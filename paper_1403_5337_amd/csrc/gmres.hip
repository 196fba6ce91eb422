// Flexible right-preconditioned GMRES in float64 (Sec. 3), s right-hand sides
// at once, each with its own Krylov basis and its own convergence.
//
// Per step j, for every still-active right-hand side k:
//   z_j = M^-1 v_j   (HODLR solve in the handle's precision, in place on the
//                     z_j slot, which the previous step filled with v_j)
//   w   = K z_j      (float64 split-K matrix product)
//   classical Gram-Schmidt applied twice against v_0..v_j, the Hessenberg
//   column, one Givens rotation, the residual estimate |g_{j+1}|;
//   v_{j+1} = w / h_{j+1,j}.
// A right-hand side stops taking steps when |g_{j+1}| <= tol |b| (or maxit,
// or breakdown); at the end of a cycle x += Z y with H y = g, and the true
// residual b - K x decides whether it restarts.
//
// Storage, all column-major with leading dimension n: basis vector j of
// right-hand side k at V + (j s + k) n (so the s vectors of step j form one
// n x s matrix), preconditioned vectors likewise in Z.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <mutex>

#include "device_util.h"
#include "hodlr_internal.h"

namespace hodlr {

constexpr int kRowsPerWG = 256;
constexpr int kMatvecCols = 128;     // default columns of K per workgroup (split-K)
constexpr int kMatvecColsMin = 64;   // narrowest split the tuner tries (sizes the partial sums)
constexpr int kMaxRestart = 512;
constexpr int kFlagInts = 384;       // host-visible flag block (layout at GmresPtrs::dev_flags)

// part[(sp s + k) n + i] = sum over the columns c of split sp of K(i, c)
// src(c, k), with the matrix cores doing the multiply-adds.  Wave w of
// workgroup (x, sp) takes rows 64 x + 16 w .. + 16 and the 128 columns of
// split sp; its 32 loads of K (one 16 x 4 block each, 128 contiguous bytes
// per column) are all in flight at once, z (as float64, zero-padded to 16 NB
// columns) comes from LDS, and v_mfma_f64_16x16x4f64 accumulates the
// 16 x 16 NB block.  The product stays bound by the K traffic; the matrix
// cores only keep the instruction count per byte low.  K is read with
// ordinary (cached) loads: the 256 MB last-level cache then keeps much of a
// 134 MB K between the products of one solve.
typedef double f64x4 __attribute__((ext_vector_type(4)));

template <typename TZ, int NB, int COLS>
__global__ void __launch_bounds__(kRowsPerWG)
    k_matvec_mfma(const double* __restrict__ K, int ldk, int n, const TZ* __restrict__ src, int lds, int s,
                  double* __restrict__ part, int rev, const int* __restrict__ gate) {
  if (gate_closed(gate, s)) return;
  constexpr int kQ = COLS / 4;
  __shared__ double zs[COLS * 16 * NB];  // z(c, k) at zs[c 16 NB + k]
  const int t = threadIdx.x, lane = t & 63, w = t >> 6, sp = rev ? gridDim.y - 1 - blockIdx.y : blockIdx.y;
  const int c0 = sp * COLS, cn = min(COLS, n - c0);
  const int m = lane & 15, kl = lane >> 4;
  const int row = blockIdx.x * 64 + 16 * w + m;
  // z first: its loads precede those of K in the (in-order) load queue, so
  // staging it waits for z alone, and the products below start on the first
  // blocks of K while the later ones are still arriving
  constexpr int kZ = COLS * 16 * NB / kRowsPerWG;
  double zv[kZ];
  // (addresses are clamped into range so that no load sits behind a branch;
  // the entries outside become zero afterwards)
#pragma unroll
  for (int u = 0; u < kZ; ++u) {
    const int e = t + u * kRowsPerWG, c = e / (16 * NB), k = e % (16 * NB);
    zv[u] = (double)src[(size_t)min(k, s - 1) * lds + c0 + min(c, cn - 1)];
  }
  double a[kQ];
  const int rowc = min(row, n - 1);
#pragma unroll
  for (int q = 0; q < kQ; ++q) {
    const int c = min(4 * q + kl, cn - 1);
    a[q] = K[(size_t)(c0 + c) * ldk + rowc];
  }
  __builtin_amdgcn_sched_barrier(0);  // every load is issued before the wait for z
#pragma unroll
  for (int u = 0; u < kZ; ++u) {
    const int e = t + u * kRowsPerWG, c = e / (16 * NB), k = e % (16 * NB);
    zs[e] = (c < cn && k < s) ? zv[u] : 0.0;
  }
  __syncthreads();
  f64x4 acc[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b) acc[b] = f64x4{};
#pragma unroll
  for (int q = 0; q < kQ; ++q)
#pragma unroll
    for (int b = 0; b < NB; ++b)  // A(m = l % 16, k = l / 16), B(k = l / 16, n = l % 16)
      acc[b] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[q], zs[(4 * q + kl) * 16 * NB + 16 * b + m], acc[b], 0, 0, 0);
  // slot v of lane l: row l / 16 + 4 v, column l % 16
  const int r0 = blockIdx.x * 64 + 16 * w + (lane >> 4);
#pragma unroll
  for (int b = 0; b < NB; ++b)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = r0 + 4 * v, k = 16 * b + m;
      if (r < n && k < s) part[((size_t)sp * s + k) * n + r] = acc[b][v];
    }
}

// The same product with CH consecutive 128-column chunks per workgroup:
// workgroup (x, sp) loads chunk c + 1 of its row block while chunk c goes
// through the matrix cores, and writes one partial for all CH chunks, so
// the partial sums shrink CH-fold and the grid fits the chip in one round.
// z for all chunks is staged in LDS first (CH * 128 * 16 NB doubles).
template <typename TZ, int NB, int CH>
__global__ void __launch_bounds__(kRowsPerWG)
    k_matvec_chunks(const double* __restrict__ K, int ldk, int n, const TZ* __restrict__ src, int lds, int s,
                    double* __restrict__ part, int rev, const int* __restrict__ gate) {
  if (gate_closed(gate, s)) return;
  constexpr int COLS = 128, kQ = COLS / 4, WD = CH * COLS;
  __shared__ double zs[WD * 16 * NB];  // z(c, k) at zs[c 16 NB + k]
  const int t = threadIdx.x, lane = t & 63, w = t >> 6, sp = rev ? gridDim.y - 1 - blockIdx.y : blockIdx.y;
  const int c0 = sp * WD, cn = min(WD, n - c0);
  const int m = lane & 15, kl = lane >> 4;
  const int row = blockIdx.x * 64 + 16 * w + m;
  const int rowc = min(row, n - 1);
  constexpr int kZ = WD * 16 * NB / kRowsPerWG;
  double zv[kZ];
#pragma unroll
  for (int u = 0; u < kZ; ++u) {
    const int e = t + u * kRowsPerWG, c = e / (16 * NB), k = e % (16 * NB);
    zv[u] = (double)src[(size_t)min(k, s - 1) * lds + c0 + min(c, cn - 1)];
  }
  double a[2][kQ];
#pragma unroll
  for (int q = 0; q < kQ; ++q)
    a[0][q] = K[(size_t)(c0 + min(4 * q + kl, cn - 1)) * ldk + rowc];
  __builtin_amdgcn_sched_barrier(0);  // every load is issued before the wait for z
#pragma unroll
  for (int u = 0; u < kZ; ++u) {
    const int e = t + u * kRowsPerWG, c = e / (16 * NB), k = e % (16 * NB);
    zs[e] = (c < cn && k < s) ? zv[u] : 0.0;
  }
  __syncthreads();
  f64x4 acc[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b) acc[b] = f64x4{};
#pragma unroll
  for (int c = 0; c < CH; ++c) {
    if (c + 1 < CH) {
#pragma unroll
      for (int q = 0; q < kQ; ++q)
        a[(c + 1) & 1][q] = K[(size_t)(c0 + min((c + 1) * COLS + 4 * q + kl, cn - 1)) * ldk + rowc];
    }
#pragma unroll
    for (int q = 0; q < kQ; ++q)
#pragma unroll
      for (int b = 0; b < NB; ++b)  // A(m = l % 16, k = l / 16), B(k = l / 16, n = l % 16)
        acc[b] = __builtin_amdgcn_mfma_f64_16x16x4f64(
            a[c & 1][q], zs[(c * COLS + 4 * q + kl) * 16 * NB + 16 * b + m], acc[b], 0, 0, 0);
  }
  const int r0 = blockIdx.x * 64 + 16 * w + (lane >> 4);
#pragma unroll
  for (int b = 0; b < NB; ++b)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = r0 + 4 * v, k = 16 * b + m;
      if (r < n && k < s) part[((size_t)sp * s + k) * n + r] = acc[b][v];
    }
}

// PASS 0: w = sum of the split-K partials (minus b when residual != 0), dots
//         of w with v_0..v_j into hout
// PASS 1: h = sum of hin over chunks; w -= V h; hcol = h; dots into hout
// PASS 2: h = sum of hin; w -= V h; hcol += h; |w|^2 partial into npart
// (the residual variant of PASS 0 takes no dots; it writes |b - K x|^2)
template <int PASS>
__global__ void __launch_bounds__(kRowsPerWG)
    k_orth(int n, int s, int j, int m1, const double* __restrict__ V, double* __restrict__ w,
           const double* __restrict__ part, int nsplit, const double* __restrict__ b, int ldb,
           const double* __restrict__ hin, double* __restrict__ hout, double* __restrict__ hcol,
           double* __restrict__ npart, const int* __restrict__ active) {
  __shared__ double ws[kRowsPerWG];
  __shared__ double hs[kMaxRestart + 1];
  __shared__ double red[kRowsPerWG / 64];
  const int k = blockIdx.y, ch = blockIdx.x, t = threadIdx.x, nt = blockDim.x;
  if (!active[k]) return;
  const int nch = gridDim.x;
  const int i = ch * kRowsPerWG + t;
  const bool valid = i < n;
  double wi = 0.0;
  if (PASS == 0) {
    if (valid) {
      int sp = 0;
      for (; sp + 8 <= nsplit; sp += 8) {
        double pv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) pv[u] = part[((size_t)(sp + u) * s + k) * n + i];
#pragma unroll
        for (int u = 0; u < 8; ++u) wi += pv[u];
      }
      for (; sp < nsplit; ++sp) wi += part[((size_t)sp * s + k) * n + i];
      if (b) wi = b[(size_t)k * ldb + i] - wi;
      w[(size_t)k * n + i] = wi;
    }
  } else {
    for (int l = t; l <= j; l += nt) {
      double h = 0.0;
      int c = 0;
      for (; c + 8 <= nch; c += 8) {
        double hv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) hv[u] = hin[((size_t)(c + u) * s + k) * m1 + l];
#pragma unroll
        for (int u = 0; u < 8; ++u) h += hv[u];
      }
      for (; c < nch; ++c) h += hin[((size_t)c * s + k) * m1 + l];
      hs[l] = h;
    }
    __syncthreads();
    if (ch == 0) {
      for (int l = t; l <= j; l += nt) {
        if (PASS == 1) hcol[(size_t)k * m1 + l] = hs[l];
        else hcol[(size_t)k * m1 + l] += hs[l];
      }
    }
    if (valid) {
      wi = w[(size_t)k * n + i];
      int l = 0;
      for (; l + 8 <= j + 1; l += 8) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = V[((size_t)(l + u) * s + k) * n + i];
#pragma unroll
        for (int u = 0; u < 8; ++u) wi -= v[u] * hs[l + u];
      }
      for (; l <= j; ++l) wi -= V[((size_t)l * s + k) * n + i] * hs[l];
      w[(size_t)k * n + i] = wi;
    }
  }
  if (PASS == 2 || (PASS == 0 && b)) {
    const double sq = block_sum(valid ? wi * wi : 0.0, red);
    if (t == 0) npart[(size_t)ch * s + k] = sq;
    return;
  }
  ws[t] = valid ? wi : 0.0;
  __syncthreads();
  const int wave = t >> 6, lane = t & 63, nw = nt >> 6;
  const int r0 = ch * kRowsPerWG;
  // two basis vectors per wave at a time, all loads issued before reducing
  for (int l = wave; l <= j; l += 2 * nw) {
    const int l1 = l + nw;
    const bool two = l1 <= j;
    double v0[kRowsPerWG / 64], v1[kRowsPerWG / 64];
#pragma unroll
    for (int r = 0; r < kRowsPerWG / 64; ++r) {
      const int row = r0 + lane + 64 * r;
      v0[r] = row < n ? V[((size_t)l * s + k) * n + row] : 0.0;
      v1[r] = (two && row < n) ? V[((size_t)l1 * s + k) * n + row] : 0.0;
    }
    double d0 = 0.0, d1 = 0.0;
#pragma unroll
    for (int r = 0; r < kRowsPerWG / 64; ++r) {
      d0 += v0[r] * ws[lane + 64 * r];
      d1 += v1[r] * ws[lane + 64 * r];
    }
    d0 = wave_sum(d0);
    d1 = wave_sum(d1);
    if (lane == 0) {
      hout[((size_t)ch * s + k) * m1 + l] = d0;
      if (two) hout[((size_t)ch * s + k) * m1 + l1] = d1;
    }
  }
}

// End of step j, one launch: the Hessenberg column j, its Givens rotation,
// the residual estimate and the convergence decision per right-hand side,
// then v_{j+1} = w / |w| (and its copy, rounded to TP, as the next
// preconditioner input; zero for a column that stops).  Every workgroup of
// column k works the rotation out itself from data no workgroup writes in
// this step (the earlier rotations, the running residual grun_in, the flags
// act_in, the cycle's starting count tstart), so they all take the same
// decision; workgroup 0 alone writes the results: H, the rotation, g, the
// next running residual, the counts, the next flags act_out, and the flags
// into host memory (pinned, read by the host after the stream event).
template <typename TP>
__global__ void __launch_bounds__(kBlock)
    k_step_end(int n, int s, int j, int m, int nch, const double* __restrict__ hcol,
               const double* __restrict__ npart, double* __restrict__ H, double* __restrict__ cs,
               double* __restrict__ sn, double* __restrict__ g, const double* __restrict__ grun_in,
               double* __restrict__ grun_out, double* __restrict__ scal, const double* __restrict__ bnorm,
               const int* __restrict__ act_in, int* __restrict__ act_out, int* __restrict__ steps,
               int* __restrict__ total, const int* __restrict__ tstart, double tol, int maxit,
               const double* __restrict__ w, double* __restrict__ V, TP* __restrict__ Z, int* host_slot) {
  __shared__ double s_hn;
  __shared__ int s_go;
  __shared__ double s_col[kMaxRestart + 1], s_c[kMaxRestart], s_s[kMaxRestart], s_n2;
  const int k = blockIdx.y, lead = blockIdx.x == 0, t = threadIdx.x;
  const bool live = act_in[k] != 0;
  const int m1 = m + 1;
  if (live) {
    // the column, the earlier rotations and the norm partials, all loaded at
    // once by the workgroup
    for (int l = t; l <= j; l += blockDim.x) s_col[l] = hcol[(size_t)k * m1 + l];
    for (int l = t; l < j; l += blockDim.x) {
      s_c[l] = cs[(size_t)k * m + l];
      s_s[l] = sn[(size_t)k * m + l];
    }
    if (t < 64) {
      double v = 0.0;
      for (int c = t; c < nch; c += 64) v += npart[(size_t)c * s + k];
      v = wave_sum(v);
      if (t == 0) s_n2 = v;
    }
  }
  __syncthreads();
  if (t == 0) {
    int go = 0;
    double hn = 1.0;
    if (live) {
      hn = sqrt(s_n2);
      double* Hk = H + (size_t)k * m1 * m + (size_t)j * m1;
      // the earlier rotations applied down the column, one running entry
      double cur = s_col[0];
      for (int l = 0; l < j; ++l) {
        const double b = s_col[l + 1];
        const double o = s_c[l] * cur + s_s[l] * b;
        cur = -s_s[l] * cur + s_c[l] * b;
        if (lead) Hk[l] = o;
      }
      double c = 1.0, sv = 0.0;
      if (hn != 0.0) {
        const double r = hypot(cur, hn);
        c = cur / r;
        sv = hn / r;
      }
      const double g0 = grun_in[k], g1 = -sv * g0;
      const int tot = tstart[k] + j + 1;
      const bool conv = fabs(g1) <= tol * bnorm[k];
      go = !(conv || tot >= maxit || !(hn > 0.0) || j + 1 >= m);
      if (lead) {
        cs[(size_t)k * m + j] = c;
        sn[(size_t)k * m + j] = sv;
        Hk[j] = c * cur + sv * hn;
        Hk[j + 1] = 0.0;
        g[(size_t)k * m1 + j] = c * g0;
        g[(size_t)k * m1 + j + 1] = g1;
        grun_out[k] = g1;
        scal[k] = hn;
        steps[k] = j + 1;
        total[k] = tot;
      }
    }
    if (lead) {
      act_out[k] = go;
      host_slot[k] = go;
      __threadfence_system();
    }
    s_hn = hn;
    s_go = go;
  }
  __syncthreads();
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const size_t o = ((size_t)(j + 1) * s + k) * n + i;
  if (s_go) {
    const double v = w[(size_t)k * n + i] / s_hn;
    V[o] = v;
    if (Z) Z[o] = (TP)v;
  } else if (Z) {
    Z[o] = TP(0);
  }
}

// v_0(k) = w(k) / scal(k) for active k, copied (rounded to TP) into the z
// slot 0 as the first preconditioner input.  Inactive columns of the z slot
// are zeroed.
template <typename TP>
__global__ void k_normalize(int n, int s, const double* __restrict__ w, const double* __restrict__ scal,
                            const int* __restrict__ active, double* __restrict__ V, TP* __restrict__ Z) {
  const int k = blockIdx.y;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const size_t o = (size_t)k * n + i;
  if (active[k]) {
    const double v = w[(size_t)k * n + i] / scal[k];
    V[o] = v;
    if (Z) Z[o] = (TP)v;
  } else if (Z) {
    Z[o] = TP(0);
  }
}

// Start of a cycle: true residual norms, decide who iterates, g = beta e_1
// (and the running residual), the count at the start; the flags also go to
// host memory (pinned).
__global__ void k_cycle_init(int s, int m, int nch, const double* __restrict__ npart,
                             const double* __restrict__ bnorm, double* __restrict__ scal,
                             double* __restrict__ g, double* __restrict__ grun, double* __restrict__ relres,
                             int* __restrict__ active, int* __restrict__ steps,
                             const int* __restrict__ total, int* __restrict__ tstart, double tol, int maxit,
                             int* host_slot) {
  const int k = threadIdx.x;
  if (k >= s) return;
  double r2 = 0.0;
  for (int c = 0; c < nch; ++c) r2 += npart[(size_t)c * s + k];
  const double beta = sqrt(r2);
  const double rr = bnorm[k] > 0.0 ? beta / bnorm[k] : 0.0;
  relres[k] = rr;
  const int go = (bnorm[k] > 0.0) && (rr > tol) && (total[k] < maxit) && (beta > 0.0);
  // the steps so far and the true relative residual, beside the flag: after
  // the cycle start that stops every column they are the call's results
  host_slot[192 + k] = total[k];
  reinterpret_cast<double*>(host_slot + 256)[k] = rr;
  active[k] = go;
  steps[k] = 0;
  tstart[k] = total[k];
  scal[k] = go ? beta : 1.0;
  for (int l = 0; l <= m; ++l) g[(size_t)k * (m + 1) + l] = 0.0;
  g[(size_t)k * (m + 1)] = beta;
  grun[k] = beta;
  host_slot[k] = go;
  __threadfence_system();
}

__global__ void k_bnorm(int s, int nch, const double* __restrict__ npart, double* __restrict__ bnorm) {
  const int k = threadIdx.x;
  if (k >= s) return;
  double r2 = 0.0;
  for (int c = 0; c < nch; ++c) r2 += npart[(size_t)c * s + k];
  bnorm[k] = sqrt(r2);
}

__global__ void __launch_bounds__(kRowsPerWG)
    k_sqnorm(int n, int s, const double* __restrict__ B, int ldb, double* __restrict__ npart) {
  __shared__ double red[kRowsPerWG / 64];
  const int k = blockIdx.y, i = blockIdx.x * kRowsPerWG + threadIdx.x;
  const double v = i < n ? B[(size_t)k * ldb + i] : 0.0;
  const double sq = block_sum(v * v, red);
  if (threadIdx.x == 0) npart[(size_t)blockIdx.x * s + k] = sq;
}

// Back substitution H y = g per right-hand side (H upper triangular after
// the rotations), one thread each.
__global__ void k_trisolve(int s, int m, const double* __restrict__ H, const double* __restrict__ g,
                           const int* __restrict__ steps, double* __restrict__ y) {
  const int k = threadIdx.x;
  if (k >= s) return;
  const int m1 = m + 1, nk = steps[k];
  const double* Hk = H + (size_t)k * m1 * m;
  double* yk = y + (size_t)k * m;
  for (int l = nk - 1; l >= 0; --l) {
    double v = g[(size_t)k * m1 + l];
    for (int c = l + 1; c < nk; ++c) v -= Hk[l + (size_t)c * m1] * yk[c];
    yk[l] = v / Hk[l + (size_t)l * m1];
  }
}

template <typename TZ>
__global__ void k_xupdate(int n, int s, int m, double* __restrict__ X, int ldx, const TZ* __restrict__ Z,
                          const double* __restrict__ y, const int* __restrict__ steps) {
  const int k = blockIdx.y, i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int nk = steps[k];
  if (nk == 0) return;
  double acc = 0.0;
  int l = 0;
  for (; l + 8 <= nk; l += 8) {
    double z[8], yy[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      z[u] = (double)Z[((size_t)(l + u) * s + k) * n + i];
      yy[u] = y[(size_t)k * m + l + u];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) acc += z[u] * yy[u];
  }
  for (; l < nk; ++l) acc += (double)Z[((size_t)l * s + k) * n + i] * y[(size_t)k * m + l];
  X[(size_t)k * ldx + i] += acc;
}

// ---------------------------------------------------------------------------
// The workspace of one solve, carved in this order from one arena (every
// piece 256-byte aligned); its size depends only on (n, s, m, type of z).
struct GmresPtrs {
  double *V, *w, *part, *hA, *hB, *hcol, *H, *cs, *sn, *g, *grun, *y, *npart, *scal, *bnorm, *relres;
  void* Z;
  int* ints;
  int* dev_flags;  // kFlagInts ints: [0, 64) cycle start, [64, 192) two step slots,
                   // [192, 256) steps taken, [256, 384) relative residuals (double)
};

static size_t gmres_layout(int n, int s, int m, size_t zsize, bool precond, unsigned char* base, GmresPtrs* p) {
  const size_t m1 = m + 1, ns = (size_t)n * s, nch = (n + kRowsPerWG - 1) / kRowsPerWG;
  const size_t nsplit_max = (n + kMatvecColsMin - 1) / kMatvecColsMin;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    void* q = base ? base + off : nullptr;
    off += (bytes + 255) / 256 * 256;
    return q;
  };
  GmresPtrs t{};
  t.V = static_cast<double*>(take(ns * m1 * sizeof(double)));
  t.Z = precond ? take(ns * m1 * zsize) : nullptr;
  t.w = static_cast<double*>(take(ns * sizeof(double)));
  t.part = static_cast<double*>(take(ns * nsplit_max * sizeof(double)));
  t.hA = static_cast<double*>(take(nch * s * m1 * sizeof(double)));
  t.hB = static_cast<double*>(take(nch * s * m1 * sizeof(double)));
  t.hcol = static_cast<double*>(take((size_t)s * m1 * sizeof(double)));
  t.H = static_cast<double*>(take((size_t)s * m1 * m * sizeof(double)));
  t.cs = static_cast<double*>(take((size_t)s * m * sizeof(double)));
  t.sn = static_cast<double*>(take((size_t)s * m * sizeof(double)));
  t.g = static_cast<double*>(take((size_t)s * m1 * sizeof(double)));
  t.grun = static_cast<double*>(take(2 * 64 * sizeof(double)));
  t.y = static_cast<double*>(take((size_t)s * m * sizeof(double)));
  t.npart = static_cast<double*>(take(nch * s * sizeof(double)));
  t.scal = static_cast<double*>(take(s * sizeof(double)));
  t.bnorm = static_cast<double*>(take(s * sizeof(double)));
  t.relres = static_cast<double*>(take(s * sizeof(double)));
  t.ints = static_cast<int*>(take(5 * 64 * sizeof(int)));
  t.dev_flags = static_cast<int*>(take(kFlagInts * sizeof(int)));
  if (p) *p = t;
  return off;
}

struct GmresWork {
  DevBuf arena;
  int* host_flags = nullptr;  // pinned: the kernels write the step flags here
  int* dev_flags = nullptr;   // the same memory as the device addresses it
  hipEvent_t ev[2] = {nullptr, nullptr};
};

// One workspace per host thread, so solves on different threads (each on its
// own stream) run side by side; it lives as long as its thread.
static GmresWork& work() {
  static thread_local GmresWork* ws = new GmresWork();
  return *ws;
}

// ---------------------------------------------------------------------------
// The workspace of gmres_solve_noalloc: a fixed array in device memory, one
// copy per GPU, whose address is looked up once per device.  Calls that
// overlap on one GPU share it and race.
// ---------------------------------------------------------------------------
constexpr size_t kNoallocScratchBytes = (size_t)192 << 20;
static __device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];

static int noalloc_scratch(unsigned char** out) {
  static std::mutex mu;
  static void* ptr[64] = {};
  int dev = 0;
  HODLR_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) return fail(HODLR_EINVAL, "device index above 63");
  std::lock_guard<std::mutex> lk(mu);
  if (!ptr[dev]) {
    void* q = nullptr;
    const hipError_t e = hipGetSymbolAddress(&q, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !q)
      return fail(HODLR_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    ptr[dev] = q;
  }
  *out = static_cast<unsigned char*>(ptr[dev]);
  return HODLR_OK;
}

size_t gmres_noalloc_bytes(int n, int s, int restart, int precision) {
  const int m = std::min(restart, kMaxRestart);
  return gmres_layout(n, s, m, precision == 32 ? sizeof(float) : sizeof(double), precision != 0, nullptr, nullptr);
}

size_t gmres_noalloc_limit() { return kNoallocScratchBytes; }

template <typename TZ, int COLS>
static int launch_matvec_cols(const double* K, int ldk, int n, const TZ* src, int lds, int s, double* part,
                              hipStream_t st, int rev, const int* gate) {
  const dim3 grid((n + 63) / 64, (n + COLS - 1) / COLS);
#define HODLR_MV(NB) \
  k_matvec_mfma<TZ, NB, COLS><<<grid, kRowsPerWG, 0, st>>>(K, ldk, n, src, lds, s, part, rev, gate)
  if (s <= 16) HODLR_MV(1);
  else if (s <= 32) HODLR_MV(2);
  else HODLR_MV(4);
#undef HODLR_MV
  HODLR_HIP(hipGetLastError());
  return HODLR_OK;
}

template <typename TZ, int CH>
static int launch_matvec_chunks(const double* K, int ldk, int n, const TZ* src, int lds, int s, double* part,
                                hipStream_t st, int rev, const int* gate) {
  const dim3 grid((n + 63) / 64, (n + 128 * CH - 1) / (128 * CH));
  if (s <= 16)
    k_matvec_chunks<TZ, 1, CH><<<grid, kRowsPerWG, 0, st>>>(K, ldk, n, src, lds, s, part, rev, gate);
  else if (s <= 32)
    k_matvec_chunks<TZ, 2, CH><<<grid, kRowsPerWG, 0, st>>>(K, ldk, n, src, lds, s, part, rev, gate);
  else
    return fail(HODLR_EINVAL, "chunked product: too many right-hand sides for the staged z");
  HODLR_HIP(hipGetLastError());
  return HODLR_OK;
}

// Split widths the tuner chooses from (columns of K per partial sum): a
// narrower split gives more workgroups and more loads in flight, a wider one
// writes fewer partial sums; 512 walks 4 chunks of 128 columns per
// workgroup, with z staged for all of them (up to 32 right-hand sides).
constexpr int kMatvecChoices[4] = {64, 128, 256, 512};

static int matvec_choices(int s) { return s <= 32 ? 4 : 3; }

template <typename TZ>
static int launch_matvec(const double* K, int ldk, int n, const TZ* src, int lds, int s, double* part, int cols,
                         hipStream_t st, const int* gate = nullptr) {
  ProfScope prof("matvec", st);
  // successive products sweep K in opposite directions (column splits in
  // increasing, then decreasing order), so that each one starts on the part
  // of K the previous one read last, which the last-level cache still holds
  // when K is larger than the cache; each split writes its own partial sums,
  // so the result does not depend on the direction
  static std::atomic<unsigned> calls{0};
  const int rev = (int)(calls.fetch_add(1, std::memory_order_relaxed) & 1u);
  if (cols == 64) return launch_matvec_cols<TZ, 64>(K, ldk, n, src, lds, s, part, st, rev, gate);
  if (cols == 256) return launch_matvec_cols<TZ, 256>(K, ldk, n, src, lds, s, part, st, rev, gate);
  if (cols == 512) return launch_matvec_chunks<TZ, 4>(K, ldk, n, src, lds, s, part, st, rev, gate);
  return launch_matvec_cols<TZ, 128>(K, ldk, n, src, lds, s, part, st, rev, gate);
}

// The split width for (n, right-hand-side block, type of z): chosen on the
// first product of that shape by timing each width (tune_choice), kept for
// the process.  gate (s column flags, may be NULL): the product does nothing
// once every column has stopped; the launches that time the widths are not
// gated.
template <typename TZ>
static int matvec_cols(const double* K, int ldk, int n, const TZ* src, int lds, int s, double* part,
                       hipStream_t st, int* cols, const int* gate = nullptr) {
  const std::string key = "matvec:" + std::to_string(n) + ":" + std::to_string((s + 15) / 16) + ":" +
                          std::to_string(sizeof(TZ));
  int pick = 1;
  const int* g = gate && tune_known(key) ? gate : nullptr;
  HODLR_TRY(tune_choice(key, matvec_choices(s), 1, [&](int c) {
    return launch_matvec<TZ>(K, ldk, n, src, lds, s, part, kMatvecChoices[c], st, g);
  }, st, &pick));
  *cols = kMatvecChoices[pick];
  return HODLR_OK;
}

// noalloc: the workspace is the fixed device array, the step flags are read
// back by a copy and a stream synchronization per step, and the matvec width
// is the tuner's kept choice or the default (nothing is allocated).
template <typename TP>
static int gmres_t(const double* K, int n, int ldk, hodlr_s* M, const double* B, int s, int ldb,
                   double* X, int ldx, double tol, int maxit, int m, int* iters, double* relres,
                   hipStream_t st, bool noalloc) {
  const int m1 = m + 1;
  const int nch = (n + kRowsPerWG - 1) / kRowsPerWG;
  int cols_d = kMatvecCols, cols_p = kMatvecCols;
  const size_t ns = (size_t)n * s;
  const size_t need = gmres_layout(n, s, m, sizeof(TP), M != nullptr, nullptr, nullptr);
  GmresPtrs wp{};
  int* host_flags = nullptr;
  int local_flags[kFlagInts];
  hipEvent_t ev[2] = {nullptr, nullptr};
  if (noalloc) {
    if (need > kNoallocScratchBytes)
      return fail(HODLR_EINVAL, "gmres_solve_noalloc: the workspace needs " + std::to_string(need) +
                                    " bytes, above its " + std::to_string(kNoallocScratchBytes) + "-byte scratch");
    unsigned char* base = nullptr;
    HODLR_TRY(noalloc_scratch(&base));
    gmres_layout(n, s, m, sizeof(TP), M != nullptr, base, &wp);
    host_flags = local_flags;
  } else {
    GmresWork& ws = work();
    HODLR_TRY(ws.arena.ensure(need));
    gmres_layout(n, s, m, sizeof(TP), M != nullptr, ws.arena.as<unsigned char>(), &wp);
    if (!ws.host_flags) {
      HODLR_HIP(hipHostMalloc(reinterpret_cast<void**>(&ws.host_flags), kFlagInts * sizeof(int)));
      HODLR_HIP(hipHostGetDevicePointer(reinterpret_cast<void**>(&ws.dev_flags), ws.host_flags, 0));
    }
    for (int e = 0; e < 2; ++e)
      // no system-scope release at the step markers: the flags the host reads
      // after them are already released by k_step_end's system fence
      if (!ws.ev[e]) HODLR_HIP(hipEventCreateWithFlags(&ws.ev[e], hipEventDisableTiming | hipEventDisableSystemFence));
    wp.dev_flags = ws.dev_flags;
    host_flags = ws.host_flags;
    ev[0] = ws.ev[0];
    ev[1] = ws.ev[1];
  }
  struct Freeze {  // the tuner times nothing inside a no-allocation call
    bool on;
    explicit Freeze(bool o) : on(o) {
      if (on) tune_freeze(true);
    }
    ~Freeze() {
      if (on) tune_freeze(false);
    }
  } freeze(noalloc);
  // flags written by the kernels at dev_flags + off, visible at host_flags + off
  auto fetch = [&](int off, int cnt) -> int {
    if (noalloc) {
      HODLR_HIP(hipMemcpyAsync(host_flags + off, wp.dev_flags + off, cnt * sizeof(int), hipMemcpyDeviceToHost, st));
      HODLR_HIP(hipStreamSynchronize(st));
    }
    return HODLR_OK;
  };
  double* V = wp.V;
  TP* Z = M ? static_cast<TP*>(wp.Z) : nullptr;
  double* w = wp.w;
  double* part = wp.part;
  // flags of the columns still iterating, two arrays: step j reads act[j & 1]
  // and its last kernel writes act[(j + 1) & 1]
  int* act[2] = {wp.ints, wp.ints + 64};
  int* active = act[0];
  int* steps = act[0] + 128;
  int* total = act[0] + 192;
  int* tstart = act[0] + 256;
  double* grun[2] = {wp.grun, wp.grun + 64};
  // behind a factorization queued without waiting, possibly on another stream
  if (M && M->status_pending) HODLR_HIP(hipStreamWaitEvent(st, M->status_ev, 0));
  HODLR_HIP(hipMemsetAsync(total, 0, s * sizeof(int), st));

  const dim3 gch(nch, s), gvec((n + kBlock - 1) / kBlock, s);
  k_sqnorm<<<gch, kRowsPerWG, 0, st>>>(n, s, B, ldb, wp.npart);
  k_bnorm<<<1, 64, 0, st>>>(s, nch, wp.npart, wp.bnorm);
  HODLR_HIP(hipGetLastError());

  // The first cycle's start is not waited for (except without pinned
  // memory): its steps are queued at once, so the host prepares them while
  // the GPU still runs the work queued before the call (a factorization
  // queued without waiting, say).  The steps of a column that is not active
  // do nothing, so the cycle start's flags are read with step 0's, behind its
  // event.
  bool defer = !noalloc;
  while (true) {
    // true residual of the current x, start of a cycle
    HODLR_TRY(matvec_cols<double>(K, ldk, n, X, ldx, s, part, st, &cols_d));
    HODLR_HIP(hipMemsetAsync(active, 0xff, s * sizeof(int), st));  // nonzero: every column
    k_orth<0><<<gch, kRowsPerWG, 0, st>>>(n, s, 0, m1, V, w, part, (n + cols_d - 1) / cols_d, B, ldb, nullptr, nullptr,
                                          nullptr, wp.npart, active);
    k_cycle_init<<<1, 64, 0, st>>>(s, m, nch, wp.npart, wp.bnorm, wp.scal, wp.g, grun[0], wp.relres, active, steps,
                                   total, tstart, tol, maxit, wp.dev_flags);
    HODLR_HIP(hipGetLastError());
    // the cycle start's flags (and a singular block of a factorization
    // queued without waiting) are read here, or behind step 0 when deferred
    auto start_check = [&](bool* any) -> int {
      if (M) HODLR_TRY(settle_factor_status(M));
      *any = false;
      for (int k = 0; k < s; ++k) *any |= host_flags[k] != 0;
      return HODLR_OK;
    };
    const bool deferred = defer;
    defer = false;
    if (!deferred) {
      HODLR_HIP(hipStreamSynchronize(st));
      HODLR_TRY(fetch(0, s));
      bool any;
      HODLR_TRY(start_check(&any));
      if (!any) break;
    }
    bool idle = false;  // a deferred start found no active column
    k_normalize<TP><<<gvec, kBlock, 0, st>>>(n, s, w, wp.scal, active, V, Z);
    // profiler records before each step: a step found afterwards to have been
    // queued with no active column did nothing, and its records are dropped
    size_t mark[2] = {prof_count(), 0};
    for (int j = 0; j < m; ++j) {
      mark[j & 1] = prof_count();
      const double* src_d = V + (size_t)j * ns;
      if (M) {
        TP* zj = Z + (size_t)j * ns;
        // (the preconditioner and the product of a step taken after every
        // column has stopped do nothing: gated on the step's flags)
        HODLR_TRY(apply_impl(M, zj, n, s, st, act[j & 1]));
        HODLR_TRY(matvec_cols<TP>(K, ldk, n, zj, n, s, part, st, &cols_p, act[j & 1]));
      } else {
        HODLR_TRY(matvec_cols<double>(K, ldk, n, src_d, n, s, part, st, &cols_p, act[j & 1]));
      }
      const int nsplit = (n + cols_p - 1) / cols_p;
      {
        ProfScope po("orth", st);
        k_orth<0><<<gch, kRowsPerWG, 0, st>>>(n, s, j, m1, V, w, part, nsplit, nullptr, 0, nullptr, wp.hA, nullptr,
                                              nullptr, act[j & 1]);
      }
      {
        ProfScope po("orth", st);
        k_orth<1><<<gch, kRowsPerWG, 0, st>>>(n, s, j, m1, V, w, part, nsplit, nullptr, 0, wp.hA, wp.hB, wp.hcol,
                                              nullptr, act[j & 1]);
      }
      {
        ProfScope po("orth", st);
        k_orth<2><<<gch, kRowsPerWG, 0, st>>>(n, s, j, m1, V, w, part, nsplit, nullptr, 0, wp.hB, nullptr, wp.hcol,
                                              wp.npart, act[j & 1]);
      }
      // flags of step j go straight to a pinned slot, read after the event;
      // the host waits for the flags of step j-1 only, so step j is already
      // queued (a step taken after every column has stopped does no work:
      // the kernels read the device flags).  Without pinned memory (noalloc)
      // the host copies step j's flags back and waits for them.
      k_step_end<TP><<<gvec, kBlock, 0, st>>>(n, s, j, m, nch, wp.hcol, wp.npart, wp.H, wp.cs, wp.sn, wp.g,
                                              grun[j & 1], grun[(j + 1) & 1], wp.scal, wp.bnorm, act[j & 1],
                                              act[(j + 1) & 1], steps, total, tstart, tol, maxit, w, V, Z,
                                              wp.dev_flags + 64 + 64 * (j & 1));
      HODLR_HIP(hipGetLastError());
      if (noalloc) {
        HODLR_TRY(fetch(64 + 64 * (j & 1), s));
        bool more = false;
        for (int k = 0; k < s; ++k) more |= host_flags[64 + 64 * (j & 1) + k] != 0;
        if (!more) break;
        continue;
      }
      HODLR_HIP(hipEventRecord(ev[j & 1], st));
      if (deferred && (j == 1 || m == 1)) {
        HODLR_HIP(hipEventSynchronize(ev[0]));
        bool any = false;
        const int rc = start_check(&any);
        if (rc != HODLR_OK || !any) {
          // the steps queued behind the start use the workspace: let them end
          HODLR_HIP(hipStreamSynchronize(st));
          if (rc != HODLR_OK) return rc;
          prof_drop_from(mark[0]);
          idle = true;
          break;
        }
      }
      if (j > 0) {
        HODLR_HIP(hipEventSynchronize(ev[(j - 1) & 1]));
        const int* prev = host_flags + 64 + 64 * ((j - 1) & 1);
        bool more = false;
        for (int k = 0; k < s; ++k) more |= prev[k] != 0;
        if (!more) {
          prof_drop_from(mark[j & 1]);  // step j was queued behind columns that had all stopped
          break;
        }
      }
    }
    if (idle) break;
    k_trisolve<<<1, 64, 0, st>>>(s, m, wp.H, wp.g, steps, wp.y);
    if (M)
      k_xupdate<TP><<<gvec, kBlock, 0, st>>>(n, s, m, X, ldx, Z, wp.y, steps);
    else
      k_xupdate<double><<<gvec, kBlock, 0, st>>>(n, s, m, X, ldx, V, wp.y, steps);
    HODLR_HIP(hipGetLastError());
  }
  // the loop ends after a synchronized cycle start, which wrote the steps
  // and residuals to the pinned block (copied back here without it)
  HODLR_TRY(fetch(192, 192));
  const double* rr = reinterpret_cast<const double*>(host_flags + 256);
  bool conv = true;
  for (int k = 0; k < s; ++k) {
    iters[k] = host_flags[192 + k];
    relres[k] = rr[k];
    conv &= relres[k] <= tol;
  }
  if (!conv) return fail(HODLR_ENOCONV, "GMRES reached maxit above tol");
  return HODLR_OK;
}

int gmres_impl(const double* K, int n, int ldk, hodlr_s* M, const double* B, int nrhs, int ldb,
               double* X, int ldx, double tol, int maxit, int restart, int* iters,
               double* relres, hipStream_t s, bool noalloc) {
  const int m = std::min(restart, kMaxRestart);
  if (M && M->precision == 32)
    return gmres_t<float>(K, n, ldk, M, B, nrhs, ldb, X, ldx, tol, maxit, m, iters, relres, s, noalloc);
  return gmres_t<double>(K, n, ldk, M, B, nrhs, ldb, X, ldx, tol, maxit, m, iters, relres, s, noalloc);
}

}  // namespace hodlr

namespace hodlr {

// The float64 product K src (s columns, leading dimension lds) as split-K
// partial sums, with the tuned split width; *nsplit receives the number of
// partials per element (part[(sp s + k) n + i]).
int matvec_partials(const double* K, int ldk, int n, const double* src, int lds, int s, double* part,
                    hipStream_t st, int* nsplit) {
  int cols = kMatvecCols;
  HODLR_TRY(matvec_cols<double>(K, ldk, n, src, lds, s, part, st, &cols));
  *nsplit = (n + cols - 1) / cols;
  return HODLR_OK;
}

size_t matvec_partial_elems(int n, int s) {
  return (size_t)n * s * ((n + kMatvecColsMin - 1) / kMatvecColsMin);
}

}  // namespace hodlr
