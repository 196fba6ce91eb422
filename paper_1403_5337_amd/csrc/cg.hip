// Preconditioned conjugate gradients in float64 for a symmetric positive
// definite K, s right-hand sides at once, each with its own scalars and its
// own convergence.  Sec. 3 notes that the HODLR solve can precondition any
// Krylov method and names conjugate gradients (Hestenes & Stiefel) beside
// GMRES; the fronts of the diffusion and elasticity problems are SPD.
//
// A cycle starts from the true residual r = b - K x with p = z = M r.  Per
// step of every right-hand side still iterating:
//   q = K p                        (the float64 split-K product of GMRES)
//   alpha = (r^T z) / (p^T q);  x += alpha p;  r -= alpha q
//   stop the cycle when |r| <= tol |b|, at maxit, or when p^T q <= 0
//   z' = M r                       (HODLR solve in the handle's precision)
//   beta = r^T (z' - z) / (r^T z)  (flexible form: a float32 solve is only
//                                   nearly a fixed symmetric operator; for
//                                   a fixed symmetric M it is the classical
//                                   coefficient, since then r^T z = 0)
//   p = z' + beta p
// When every column's cycle has ended, the true residual decides who
// restarts; a column whose last cycle took no step stops for good.
//
// In the vector kernels one workgroup owns one right-hand side, so every
// inner product is summed in one fixed order.  The per-step flags go to
// pinned host memory; the host waits for the flags of the step before the
// one it has just queued, as in GMRES.
#include <algorithm>
#include <cmath>

#include "device_util.h"
#include "hodlr_internal.h"

namespace hodlr {

constexpr int kCgThreads = 1024;
constexpr int kCgMaxRhs = 64;

// Each thread takes elements t, t + kCgThreads, ... of its column, kE of them
// per round with all their loads issued together; the sums run in element
// order, so the result does not depend on the batching.
constexpr int kE = 4;

// q(i) of column k: the sum of the nsplit partial products of K p, in split
// order, loaded 8 at a time
__device__ __forceinline__ double cg_q(const double* __restrict__ part, int nsplit, int s, int n, int k, int i) {
  const double* pp = part + (size_t)k * n + i;
  const size_t st = (size_t)s * n;
  double q = 0.0;
  int sp = 0;
  for (; sp + 8 <= nsplit; sp += 8) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = pp[(size_t)(sp + u) * st];
#pragma unroll
    for (int u = 0; u < 8; ++u) q += v[u];
  }
  for (; sp < nsplit; ++sp) q += pp[(size_t)sp * st];
  return q;
}

__global__ void __launch_bounds__(kCgThreads)
    k_cg_bnorm(int n, const double* __restrict__ B, int ldb, double* __restrict__ bnorm) {
  __shared__ double red[kCgThreads / 64];
  const int k = blockIdx.x;
  double v = 0.0;
  for (int i = threadIdx.x; i < n; i += kCgThreads) {
    const double b = B[(size_t)k * ldb + i];
    v += b * b;
  }
  v = block_sum(v, red);
  if (threadIdx.x == 0) bnorm[k] = sqrt(v);
}

// Start of a cycle: r = b - K x (K x from the partial products), its norm
// against |b|, who iterates, and z's slot = r (rounded to TP) as the first
// preconditioner input (zero for a column that does not iterate).
template <typename TP>
__global__ void __launch_bounds__(kCgThreads)
    k_cg_start(int n, int s, const double* __restrict__ B, int ldb, const double* __restrict__ part, int nsplit,
               double* __restrict__ R, TP* __restrict__ Z, double* __restrict__ rz,
               const double* __restrict__ bnorm, double* __restrict__ relres, int* __restrict__ act,
               const int* __restrict__ total, int* __restrict__ tstart, double tol, int maxit,
               int* host_flags) {
  __shared__ double red[kCgThreads / 64];
  const int k = blockIdx.x, t = threadIdx.x;
  double v = 0.0;
  for (int i0 = t; i0 < n; i0 += kE * kCgThreads) {
    double r[kE];
#pragma unroll
    for (int e = 0; e < kE; ++e) {
      const int i = i0 + e * kCgThreads;
      r[e] = i < n ? B[(size_t)k * ldb + i] - cg_q(part, nsplit, s, n, k, i) : 0.0;
    }
#pragma unroll
    for (int e = 0; e < kE; ++e) {
      const int i = i0 + e * kCgThreads;
      if (i < n) {
        R[(size_t)k * n + i] = r[e];
        Z[(size_t)k * n + i] = (TP)r[e];
      }
      v += r[e] * r[e];
    }
  }
  v = block_sum(v, red);
  const double bn = bnorm[k], rel = bn > 0.0 ? sqrt(v) / bn : 0.0;
  // a column whose previous cycle took no step (a breakdown) stops
  const bool go = bn > 0.0 && rel > tol && total[k] < maxit && total[k] != tstart[k];
  if (!go)
    for (int i = t; i < n; i += kCgThreads) Z[(size_t)k * n + i] = TP(0);
  if (t == 0) {
    relres[k] = rel;
    act[k] = go ? 1 : 0;
    rz[k] = 0.0;  // marks the first direction of the cycle
    tstart[k] = total[k];
    host_flags[k] = go ? 1 : 0;
    __threadfence_system();
  }
}

// New direction: beta from r^T z' and r^T z (the z of the previous step, in
// Zold), p = z' + beta p, Zold = z'.  The cycle's first direction is p = z'.
template <typename TP>
__global__ void __launch_bounds__(kCgThreads)
    k_cg_dir(int n, const double* __restrict__ R, const TP* __restrict__ Z, TP* __restrict__ Zold,
             double* __restrict__ P, double* __restrict__ rz, int* __restrict__ act) {
  __shared__ double red[kCgThreads / 64];
  const int k = blockIdx.x, t = threadIdx.x;
  if (!act[k]) return;
  const double* r = R + (size_t)k * n;
  const TP* z = Z + (size_t)k * n;
  TP* zo = Zold + (size_t)k * n;
  double* p = P + (size_t)k * n;
  const double rz_old = rz[k];
  const bool first = rz_old == 0.0;
  double a = 0.0, b = 0.0;
  for (int i0 = t; i0 < n; i0 += kE * kCgThreads) {
    double rv[kE], zv[kE], ov[kE];
#pragma unroll
    for (int e = 0; e < kE; ++e) {
      const int i = i0 + e * kCgThreads;
      const bool in = i < n;
      rv[e] = in ? r[i] : 0.0;
      zv[e] = in ? (double)z[i] : 0.0;
      ov[e] = (in && !first) ? (double)zo[i] : 0.0;
    }
#pragma unroll
    for (int e = 0; e < kE; ++e) {
      a += rv[e] * zv[e];
      b += rv[e] * ov[e];
    }
  }
  const double rzn = block_sum(a, red);
  const double rzo = first ? 0.0 : block_sum(b, red);
  if (!(rzn > 0.0)) {  // M not positive definite in floating point: end the cycle
    if (t == 0) act[k] = 0;
    return;
  }
  const double beta = first ? 0.0 : (rzn - rzo) / rz_old;
  for (int i0 = t; i0 < n; i0 += kE * kCgThreads) {
    TP zv[kE];
    double pv[kE];
#pragma unroll
    for (int e = 0; e < kE; ++e) {
      const int i = i0 + e * kCgThreads;
      const bool in = i < n;
      zv[e] = in ? z[i] : TP(0);
      pv[e] = (in && !first) ? p[i] : 0.0;
    }
#pragma unroll
    for (int e = 0; e < kE; ++e) {
      const int i = i0 + e * kCgThreads;
      if (i < n) {
        p[i] = first ? (double)zv[e] : (double)zv[e] + beta * pv[e];
        zo[i] = zv[e];
      }
    }
  }
  if (t == 0) rz[k] = rzn;
}

// The step: alpha = r^T z / p^T q, x += alpha p, r -= alpha q, z's slot = r
// (rounded to TP) for the next preconditioner solve, the recurrence residual
// and the decision; the flag also goes to the host slot.
template <typename TP>
__global__ void __launch_bounds__(kCgThreads)
    k_cg_step(int n, int s, const double* __restrict__ part, int nsplit, const double* __restrict__ P,
              double* __restrict__ X, int ldx, double* __restrict__ R, TP* __restrict__ Z,
              const double* __restrict__ rz, const double* __restrict__ bnorm, int* __restrict__ act,
              int* __restrict__ total, double tol, int maxit, int* host_slot) {
  __shared__ double red[kCgThreads / 64];
  const int k = blockIdx.x, t = threadIdx.x;
  int go = act[k];
  if (go) {
    const double* p = P + (size_t)k * n;
    // q kept in registers for the update when the column is short enough
    constexpr int kKeep = 4;
    double qk[kKeep][kE];
    const bool keep = n <= kKeep * kE * kCgThreads;
    double v = 0.0;
    for (int i0 = t, c = 0; i0 < n; i0 += kE * kCgThreads, ++c) {
      double pv[kE], qv[kE];
#pragma unroll
      for (int e = 0; e < kE; ++e) {
        const int i = i0 + e * kCgThreads;
        const bool in = i < n;
        pv[e] = in ? p[i] : 0.0;
        qv[e] = in ? cg_q(part, nsplit, s, n, k, i) : 0.0;
      }
#pragma unroll
      for (int e = 0; e < kE; ++e) {
        v += pv[e] * qv[e];
        if (keep) {
#pragma unroll
          for (int cc = 0; cc < kKeep; ++cc)
            if (cc == c) qk[cc][e] = qv[e];
        }
      }
    }
    const double pq = block_sum(v, red);
    if (!(pq > 0.0)) {
      go = 0;  // K not positive definite along p: end the cycle
    } else {
      const double alpha = rz[k] / pq;
      double* x = X + (size_t)k * ldx;
      double* r = R + (size_t)k * n;
      TP* z = Z + (size_t)k * n;
      double w = 0.0;
      for (int i0 = t, c = 0; i0 < n; i0 += kE * kCgThreads, ++c) {
        double pv[kE], qv[kE], xv[kE], rv[kE];
#pragma unroll
        for (int e = 0; e < kE; ++e) {
          const int i = i0 + e * kCgThreads;
          const bool in = i < n;
          double qq = 0.0;
          if (keep) {
#pragma unroll
            for (int cc = 0; cc < kKeep; ++cc)
              if (cc == c) qq = qk[cc][e];
          } else if (in) {
            qq = cg_q(part, nsplit, s, n, k, i);
          }
          qv[e] = in ? qq : 0.0;
          pv[e] = in ? p[i] : 0.0;
          xv[e] = in ? x[i] : 0.0;
          rv[e] = in ? r[i] : 0.0;
        }
#pragma unroll
        for (int e = 0; e < kE; ++e) {
          const int i = i0 + e * kCgThreads;
          const double ri = rv[e] - alpha * qv[e];
          if (i < n) {
            x[i] = xv[e] + alpha * pv[e];
            r[i] = ri;
            z[i] = (TP)ri;
          }
          w += (i < n) ? ri * ri : 0.0;
        }
      }
      const double rr = block_sum(w, red);
      const int tot = total[k] + 1;
      go = (sqrt(rr) > tol * bnorm[k] && tot < maxit) ? 1 : 0;
      if (t == 0) total[k] = tot;
    }
  }
  if (t == 0) {
    act[k] = go;
    host_slot[k] = go;
    __threadfence_system();
  }
}

// ---------------------------------------------------------------------------
struct CgWork {
  DevBuf R, P, Z, Zold, part, dbl, ints;
  int* host_flags = nullptr;  // pinned: [0, 64) cycle start, [64, 192) two step slots
  int* dev_flags = nullptr;
  hipEvent_t ev[2] = {nullptr, nullptr};
};

// one workspace per host thread (solves on different threads run side by side)
static CgWork& cg_work() {
  static thread_local CgWork* ws = new CgWork();
  return *ws;
}

template <typename TP>
static int cg_t(const double* K, int n, int ldk, hodlr_s* M, const double* B, int s, int ldb, double* X,
                int ldx, double tol, int maxit, int* iters, double* relres, hipStream_t st) {
  CgWork& ws = cg_work();
  const size_t ns = (size_t)n * s;
  HODLR_TRY(ws.R.ensure(ns * sizeof(double)));
  HODLR_TRY(ws.P.ensure(ns * sizeof(double)));
  HODLR_TRY(ws.Z.ensure(ns * sizeof(TP)));
  HODLR_TRY(ws.Zold.ensure(ns * sizeof(TP)));
  HODLR_TRY(ws.part.ensure(matvec_partial_elems(n, s) * sizeof(double)));
  HODLR_TRY(ws.dbl.ensure(4 * kCgMaxRhs * sizeof(double)));
  HODLR_TRY(ws.ints.ensure(3 * kCgMaxRhs * sizeof(int)));
  if (!ws.host_flags) {
    HODLR_HIP(hipHostMalloc(reinterpret_cast<void**>(&ws.host_flags), 192 * sizeof(int)));
    HODLR_HIP(hipHostGetDevicePointer(reinterpret_cast<void**>(&ws.dev_flags), ws.host_flags, 0));
  }
  for (int e = 0; e < 2; ++e)
    if (!ws.ev[e]) HODLR_HIP(hipEventCreateWithFlags(&ws.ev[e], hipEventDisableTiming));
  double* R = ws.R.as<double>();
  double* P = ws.P.as<double>();
  TP* Z = ws.Z.as<TP>();
  TP* Zold = ws.Zold.as<TP>();
  double* part = ws.part.as<double>();
  double* rz = ws.dbl.as<double>();
  double* bnorm = rz + kCgMaxRhs;
  double* rel = rz + 2 * kCgMaxRhs;
  int* act = ws.ints.as<int>();
  int* total = act + kCgMaxRhs;
  int* tstart = act + 2 * kCgMaxRhs;
  // behind a factorization queued without waiting, possibly on another stream
  if (M && M->status_pending) HODLR_HIP(hipStreamWaitEvent(st, M->status_ev, 0));
  HODLR_HIP(hipMemsetAsync(total, 0, s * sizeof(int), st));
  HODLR_HIP(hipMemsetAsync(tstart, 0xff, s * sizeof(int), st));  // -1: no cycle yet
  k_cg_bnorm<<<s, kCgThreads, 0, st>>>(n, B, ldb, bnorm);
  HODLR_HIP(hipGetLastError());
  while (true) {
    int nsplit = 0;
    HODLR_TRY(matvec_partials(K, ldk, n, X, ldx, s, part, st, &nsplit));
    k_cg_start<TP><<<s, kCgThreads, 0, st>>>(n, s, B, ldb, part, nsplit, R, Z, rz, bnorm, rel, act, total, tstart,
                                              tol, maxit, ws.dev_flags);
    HODLR_HIP(hipGetLastError());
    HODLR_HIP(hipStreamSynchronize(st));
    if (M) HODLR_TRY(settle_factor_status(M));  // (a factorization queued without waiting)
    bool any = false;
    for (int k = 0; k < s; ++k) any |= ws.host_flags[k] != 0;
    if (!any) break;
    for (int j = 0;; ++j) {
      // z = M r in place (without a preconditioner z's slot already holds r)
      if (M) HODLR_TRY(apply_impl(M, Z, n, s, st));
      {
        ProfScope po("cg_vec", st);
        k_cg_dir<TP><<<s, kCgThreads, 0, st>>>(n, R, Z, Zold, P, rz, act);
      }
      HODLR_HIP(hipGetLastError());
      HODLR_TRY(matvec_partials(K, ldk, n, P, n, s, part, st, &nsplit));
      {
        ProfScope po("cg_vec", st);
        k_cg_step<TP><<<s, kCgThreads, 0, st>>>(n, s, part, nsplit, P, X, ldx, R, Z, rz, bnorm, act, total, tol,
                                                 maxit, ws.dev_flags + 64 + 64 * (j & 1));
      }
      HODLR_HIP(hipGetLastError());
      HODLR_HIP(hipEventRecord(ws.ev[j & 1], st));
      if (j > 0) {
        HODLR_HIP(hipEventSynchronize(ws.ev[(j - 1) & 1]));
        const int* prev = ws.host_flags + 64 + 64 * ((j - 1) & 1);
        bool more = false;
        for (int k = 0; k < s; ++k) more |= prev[k] != 0;
        if (!more) break;
      }
    }
  }
  HODLR_HIP(hipMemcpyAsync(relres, rel, s * sizeof(double), hipMemcpyDeviceToHost, st));
  HODLR_HIP(hipMemcpyAsync(ws.host_flags, total, s * sizeof(int), hipMemcpyDeviceToHost, st));
  HODLR_HIP(hipStreamSynchronize(st));
  bool conv = true;
  for (int k = 0; k < s; ++k) {
    iters[k] = ws.host_flags[k];
    conv &= relres[k] <= tol;
  }
  if (!conv) return fail(HODLR_ENOCONV, "CG stopped above tol (maxit or a breakdown)");
  return HODLR_OK;
}

int cg_impl(const double* K, int n, int ldk, hodlr_s* M, const double* B, int nrhs, int ldb, double* X, int ldx,
            double tol, int maxit, int* iters, double* relres, hipStream_t s) {
  if (M && M->precision == 32) return cg_t<float>(K, n, ldk, M, B, nrhs, ldb, X, ldx, tol, maxit, iters, relres, s);
  return cg_t<double>(K, n, ldk, M, B, nrhs, ldb, X, ldx, tol, maxit, iters, relres, s);
}

}  // namespace hodlr
