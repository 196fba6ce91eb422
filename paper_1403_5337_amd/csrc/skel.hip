// Learned skeleton proposer: per-vertex block features, their training labels
// (the pivots ACA picks), and the 8-64-64-1 scorer with its gradient and
// Adam update.  Not in the paper: it proposes the rows and columns of the
// pseudo-skeleton of Sec. 5.3 (eq. Ahat) that BDLR picks by boundary
// distance; a block whose sampled error stays above the tolerance falls back
// to ACA (Sec. 5.1) in the build.
//
// Samples: the blocks of the tree in level order (node 1, 2, ...); for the
// block of node c (rows I = c, columns J = its sibling) its |I| row vertices,
// then its |J| column vertices.  Features are 8 floats per sample (row-major).
//
// Scorer parameters (float32, kMlpParams values): W1 (64 x 8, row-major),
// b1 (64), W2 (64 x 64, row-major), b2 (64), w3 (64), b3 (1).  The forward
// pass and the gradient run with the weights rounded to bfloat16 (nearest,
// ties to even) unless asked for float32, and always accumulate in float32.
#include <algorithm>
#include <climits>
#include <cstdint>
#include <vector>

#include "device_util.h"
#include "hodlr_internal.h"

namespace hodlr {

namespace {

constexpr int NF = 8, HD = 64;
constexpr int OW1 = 0, OB1 = OW1 + HD * NF, OW2 = OB1 + HD, OB2 = OW2 + HD * HD, OW3 = OB2 + HD,
              OB3 = OW3 + HD, NP = OB3 + 1;
static_assert(NP == kMlpParams, "parameter count");
constexpr int kSideMax = 8192;

__device__ __forceinline__ float bf16_round(float x) {
  unsigned u = __float_as_uint(x);
  if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x7fffffu)) return x;  // NaN stays
  u += 0x7fffu + ((u >> 16) & 1u);
  return __uint_as_float(u & 0xffff0000u);
}

// ---------------------------------------------------------------------------
// Features
// ---------------------------------------------------------------------------
// One workgroup per (block, side): the side's breadth-first distances from
// its boundary, its statistics and its vertices' features.  The side is a
// contiguous range of vertex ids, so its row pointers are one slice, staged
// in LDS; a vertex's neighbour list is read kNb entries at a time with the
// loads issued together (one round trip to the cache for most vertices of a
// 3-dof mesh).
constexpr int kFeatBlock = 1024, kFeatWaves = kFeatBlock / 64;
constexpr int kNb = 32;
constexpr int kStats = 15;  // own: dmax, degree, |K_vv|, -lo[3], hi[3]; other side: -lo[3], hi[3]
constexpr unsigned kUnreached = 0xffffffffu;
constexpr int kMaxLayer = kSideMax;  // a side of len vertices has at most len layers

// dcount (optional): per block, the number of row and of column vertices at
// distance < cnt_depth (the picks of BDLR at that depth before any cap).
__global__ void __launch_bounds__(kFeatBlock)
    k_skel_features(const int* __restrict__ rowptr, const int* __restrict__ col, const float* __restrict__ xyz,
                    const double* __restrict__ K, int ldk, const SkelBlock* __restrict__ blocks,
                    float* __restrict__ feats, int cnt_depth, int* __restrict__ dcount) {
  __shared__ unsigned dist[kSideMax];  // kUnreached = not reached
  __shared__ int rp[kSideMax + 1];
  __shared__ float red[kFeatWaves][kStats];
  __shared__ float st[kStats];
  __shared__ int flag[3], cnt;
  const SkelBlock b = blocks[blockIdx.x];
  const int sd = blockIdx.y, t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int s0 = sd == 0 ? b.row0 : b.col0, len = sd == 0 ? b.m : b.nc;
  const int o0 = sd == 0 ? b.col0 : b.row0, olen = sd == 0 ? b.nc : b.m;
  for (int i = t; i <= len; i += kFeatBlock) rp[i] = rowptr[s0 + i];
  if (t < 3) flag[t] = 0;
  if (t == 0) cnt = 0;
  __syncthreads();
  // the boundary: vertices with an edge into the other side
  for (int i = t; i < len; i += kFeatBlock) {
    const int e1 = rp[i + 1];
    unsigned d = kUnreached;
    for (int e0 = rp[i]; e0 < e1 && d != 0; e0 += kNb) {
      int u[kNb];
#pragma unroll
      for (int k = 0; k < kNb; ++k) u[k] = e0 + k < e1 ? col[e0 + k] : -1;
#pragma unroll
      for (int k = 0; k < kNb; ++k)
        if ((unsigned)(u[k] - o0) < (unsigned)olen) d = 0;
    }
    dist[i] = d;
  }
  __syncthreads();
  // layer lvl lowers its neighbours inside the side to lvl + 1 (LDS atomic
  // minima without return, so the loads of a neighbour list go out together
  // and nothing waits on LDS).  A vertex first lowered in layer lvl is at
  // distance lvl + 1, and no later layer lowers it further.  One barrier per
  // layer: a thread that found a vertex of layer lvl sets flag[lvl % 3];
  // thread 0 clears the flag of layer lvl + 1 before the barrier of layer
  // lvl, after every reader of that slot (layer lvl - 2) has passed the
  // barrier of lvl - 1.  The search ends at the first empty layer.
  for (int lvl = 0; lvl < kMaxLayer; ++lvl) {
    int found = 0;
    for (int i = t; i < len; i += kFeatBlock) {
      if (dist[i] != (unsigned)lvl) continue;
      found = 1;
      const int e1 = rp[i + 1];
      for (int e0 = rp[i]; e0 < e1; e0 += kNb) {
        int u[kNb];
#pragma unroll
        for (int k = 0; k < kNb; ++k) u[k] = e0 + k < e1 ? col[e0 + k] : -1;
#pragma unroll
        for (int k = 0; k < kNb; ++k) {
          const int j = u[k] - s0;
          if ((unsigned)j < (unsigned)len) atomicMin(&dist[j], (unsigned)(lvl + 1));
        }
      }
    }
    if (found) flag[lvl % 3] = 1;
    if (t == 0) flag[(lvl + 1) % 3] = 0;
    __syncthreads();
    if (!flag[lvl % 3]) break;
  }
  // statistics, all as maxima (minima negated)
  float v[kStats];
  for (int q = 0; q < kStats; ++q) v[q] = -INFINITY;
  v[0] = v[1] = v[2] = 0.f;
  int c = 0;
  for (int i = t; i < len; i += kFeatBlock) {
    const int x = s0 + i;
    const unsigned d = dist[i];
    if (d != kUnreached) v[0] = fmaxf(v[0], (float)d);
    c += d < (unsigned)max(cnt_depth, 0) ? 1 : 0;
    v[1] = fmaxf(v[1], (float)(rp[i + 1] - rp[i]));
    v[2] = fmaxf(v[2], (float)fabs(K[(size_t)x * ldk + x]));
    for (int a = 0; a < 3; ++a) {
      const float p = xyz[3 * x + a];
      v[3 + a] = fmaxf(v[3 + a], -p);
      v[6 + a] = fmaxf(v[6 + a], p);
    }
  }
  for (int i = t; i < olen; i += kFeatBlock)
    for (int a = 0; a < 3; ++a) {
      const float p = xyz[3 * (o0 + i) + a];
      v[9 + a] = fmaxf(v[9 + a], -p);
      v[12 + a] = fmaxf(v[12 + a], p);
    }
#pragma unroll
  for (int q = 0; q < kStats; ++q)
    for (int o = 32; o > 0; o >>= 1) v[q] = fmaxf(v[q], __shfl_xor(v[q], o, 64));
  for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
  if (lane == 0) {
    for (int q = 0; q < kStats; ++q) red[w][q] = v[q];
    if (c) atomicAdd(&cnt, c);
  }
  __syncthreads();
  if (t < kStats) {
    float r = red[0][t];
    for (int k = 1; k < kFeatWaves; ++k) r = fmaxf(r, red[k][t]);
    st[t] = r;
  }
  __syncthreads();
  if (dcount && t == 0) dcount[2 * blockIdx.x + sd] = cnt;
  const float dmax = st[0], dgmax = st[1], kdmax = st[2];
  float lo[3], ext[3], olo[3], ohi[3], diag2 = 0.f;
  for (int a = 0; a < 3; ++a) {
    lo[a] = -st[3 + a];
    ext[a] = st[6 + a] - lo[a];
    olo[a] = -st[9 + a];
    ohi[a] = st[12 + a];
    diag2 += ext[a] * ext[a];
  }
  const float diag = sqrtf(diag2);
  float* F = feats + (size_t)(b.samp0 + (sd == 0 ? 0 : b.m)) * NF;
  for (int i = t; i < len; i += kFeatBlock) {
    const int x = s0 + i;
    const float d = dist[i] == kUnreached ? dmax + 1.f : (float)dist[i];
    float f[NF];
    f[0] = d / (dmax + 1.f);
    f[1] = 1.f / (1.f + d);
    f[2] = dgmax > 0.f ? (float)(rp[i + 1] - rp[i]) / dgmax : 0.f;
    float g2 = 0.f;
    for (int a = 0; a < 3; ++a) {
      const float p = xyz[3 * x + a];
      f[3 + a] = ext[a] > 0.f ? (p - lo[a]) / ext[a] : 0.f;
      const float gap = fmaxf(0.f, fmaxf(olo[a] - p, p - ohi[a]));
      g2 += gap * gap;
    }
    f[6] = kdmax > 0.f ? (float)fabs(K[(size_t)x * ldk + x]) / kdmax : 0.f;
    f[7] = (olen > 0 && diag > 0.f) ? fminf(1.f, sqrtf(g2) / diag) : 0.f;
    float4* o = reinterpret_cast<float4*>(F + (size_t)i * NF);
    o[0] = make_float4(f[0], f[1], f[2], f[3]);
    o[1] = make_float4(f[4], f[5], f[6], f[7]);
  }
}

// labels of every sample of a block: 1 on the ACA pivot rows / columns
__global__ void __launch_bounds__(kBlock)
    k_skel_labels(const SkelBlock* __restrict__ blocks, const int* __restrict__ piv, int kcap,
                  const int* __restrict__ rank, float* __restrict__ labels) {
  const SkelBlock b = blocks[blockIdx.x];
  const int t = threadIdx.x;
  for (int i = t; i < b.m + b.nc; i += kBlock) labels[b.samp0 + i] = 0.f;
  __syncthreads();
  const int r = rank[b.node];
  const int* p = piv + (size_t)(b.node - 1) * 2 * kcap;
  for (int l = t; l < r; l += kBlock) {
    labels[b.samp0 + p[l]] = 1.f;
    labels[b.samp0 + b.m + p[kcap + l]] = 1.f;
  }
}

// ---------------------------------------------------------------------------
// Scorer
// ---------------------------------------------------------------------------
__device__ void stage_params(const float* __restrict__ P, int bf16, float* W) {
  for (int i = threadIdx.x; i < NP; i += blockDim.x) W[i] = bf16 ? bf16_round(P[i]) : P[i];
  __syncthreads();
}

// logits of N samples, grid-stride over samples
// Forward pass on the matrix cores (v_mfma_f32_32x32x2f32, float32 products
// and accumulation), one wave per 32 samples, computed transposed so that no
// layer's output has to be re-laid out: layer 1 is W1 (64 x 8) times X^T
// (8 x 32 samples); in the result lane l holds, for sample l % 32, the
// hidden units 32 t + 8 (v / 4) + 4 (l / 32) + v % 4 of its registers v.
// Layer 2 (W2 times H1^T) takes those registers directly as its B operand:
// at step (t, v) lanes < 32 supply hidden unit 32 t + 8 (v / 4) + v % 4 and
// lanes >= 32 the unit 4 above it, so A supplies W2's column of the same
// unit, lane by lane.  Layer 3 is a dot product per lane, the two lanes of
// a sample added at the end.  The weights sit in LDS with padded rows.
typedef float f32x16 __attribute__((ext_vector_type(16)));

__global__ void __launch_bounds__(kBlock)
    k_mlp_forward(const float* __restrict__ X, int N, const float* __restrict__ P, int bf16,
                  float* __restrict__ z_out) {
  __shared__ float W1s[HD][NF + 1], W2s[HD][HD + 1], b1s[HD], b2s[HD], w3s[HD], b3s;
  const int t = threadIdx.x, lane = t & 63, kl = lane >> 5, r32 = lane & 31;
  for (int e = t; e < HD * NF; e += kBlock) {
    const float w = P[OW1 + e];
    W1s[e / NF][e % NF] = bf16 ? bf16_round(w) : w;
  }
  for (int e = t; e < HD * HD; e += kBlock) {
    const float w = P[OW2 + e];
    W2s[e / HD][e % HD] = bf16 ? bf16_round(w) : w;
  }
  if (t < HD) {
    b1s[t] = bf16 ? bf16_round(P[OB1 + t]) : P[OB1 + t];
    b2s[t] = bf16 ? bf16_round(P[OB2 + t]) : P[OB2 + t];
    w3s[t] = bf16 ? bf16_round(P[OW3 + t]) : P[OW3 + t];
  }
  if (t == 0) b3s = bf16 ? bf16_round(P[OB3]) : P[OB3];
  __syncthreads();
  const int waves = gridDim.x * (kBlock / 64);
  for (int tile = blockIdx.x * (kBlock / 64) + (t >> 6); tile * 32 < N; tile += waves) {
    const int sm = tile * 32 + r32;
    const bool live = sm < N;
    f32x16 acc1[2] = {f32x16{}, f32x16{}};
#pragma unroll
    for (int step = 0; step < NF / 2; ++step) {
      const int f = 2 * step + kl;
      const float b = live ? X[(size_t)sm * NF + f] : 0.f;
#pragma unroll
      for (int tt = 0; tt < 2; ++tt) acc1[tt] = __builtin_amdgcn_mfma_f32_32x32x2f32(W1s[32 * tt + r32][f], b, acc1[tt], 0, 0, 0);
    }
#pragma unroll
    for (int tt = 0; tt < 2; ++tt)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int h = 32 * tt + 8 * (v >> 2) + 4 * kl + (v & 3);
        acc1[tt][v] = fmaxf(acc1[tt][v] + b1s[h], 0.f);
      }
    f32x16 acc2[2] = {f32x16{}, f32x16{}};
#pragma unroll
    for (int tt = 0; tt < 2; ++tt)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int h = 32 * tt + 8 * (v >> 2) + 4 * kl + (v & 3);
        const float b = acc1[tt][v];
#pragma unroll
        for (int ot = 0; ot < 2; ++ot)
          acc2[ot] = __builtin_amdgcn_mfma_f32_32x32x2f32(W2s[32 * ot + r32][h], b, acc2[ot], 0, 0, 0);
      }
    float zp = 0.f;
#pragma unroll
    for (int ot = 0; ot < 2; ++ot)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int o = 32 * ot + 8 * (v >> 2) + 4 * kl + (v & 3);
        zp = fmaf(w3s[o], fmaxf(acc2[ot][v] + b2s[o], 0.f), zp);
      }
    zp += __shfl_xor(zp, 32, 64);
    if (kl == 0 && live) z_out[sm] = zp + b3s;
  }
}

__device__ __forceinline__ float sigmoidf_(float z) {
  const float e = expf(-fabsf(z));
  return z >= 0.f ? 1.f / (1.f + e) : e / (1.f + e);
}
__device__ __forceinline__ float softplusf_(float z) { return fmaxf(z, 0.f) + log1pf(expf(-fabsf(z))); }

constexpr int kSB = 128;  // samples per workgroup of the gradient

// Partial gradient (and loss) of the mean weighted logistic loss over the
// workgroup's 128 samples; partial[wg][0..NP) and partial[wg][NP] = loss sum.
__global__ void __launch_bounds__(kBlock)
    k_mlp_grad(const float* __restrict__ X, const float* __restrict__ Y, int N, const float* __restrict__ P,
               int bf16, float pos_weight, float inv_n, float* __restrict__ partial) {
  __shared__ float W[NP];
  __shared__ float Xs[kSB][NF];
  __shared__ float H1[kSB][HD + 1];  // h1, later dl/da1
  __shared__ float A2[kSB][HD + 1];  // a2, later dl/da2
  __shared__ float dz[kSB], lz[kSB];
  stage_params(P, bf16, W);
  const int t = threadIdx.x, s0 = blockIdx.x * kSB;
  float* out = partial + (size_t)blockIdx.x * (NP + 1);
  if (t < kSB) {
    const int s = s0 + t;
    const bool ok = s < N;
    float x[NF], h1[HD];
#pragma unroll
    for (int a = 0; a < NF; ++a) {
      x[a] = ok ? X[(size_t)s * NF + a] : 0.f;
      Xs[t][a] = x[a];
    }
#pragma unroll
    for (int o = 0; o < HD; ++o) {
      float a1 = W[OB1 + o];
#pragma unroll
      for (int a = 0; a < NF; ++a) a1 = fmaf(W[OW1 + o * NF + a], x[a], a1);
      h1[o] = ok ? fmaxf(a1, 0.f) : 0.f;
      H1[t][o] = h1[o];
    }
    float z = W[OB3];
    for (int o = 0; o < HD; ++o) {
      float a2 = W[OB2 + o];
#pragma unroll
      for (int i = 0; i < HD; ++i) a2 = fmaf(W[OW2 + o * HD + i], h1[i], a2);
      A2[t][o] = ok ? a2 : 0.f;
      z = fmaf(W[OW3 + o], fmaxf(a2, 0.f), z);
    }
    const float y = ok ? Y[s] : 0.f;
    dz[t] = ok ? (-pos_weight * y * sigmoidf_(-z) + (1.f - y) * sigmoidf_(z)) * inv_n : 0.f;
    lz[t] = ok ? (pos_weight * y * softplusf_(-z) + (1.f - y) * softplusf_(z)) * inv_n : 0.f;
  }
  __syncthreads();
  // w3, b3 and the loss
  if (t < HD) {
    float g = 0.f;
    for (int s = 0; s < kSB; ++s) g = fmaf(dz[s], fmaxf(A2[s][t], 0.f), g);
    out[OW3 + t] = g;
  } else if (t == HD) {
    float g = 0.f, l = 0.f;
    for (int s = 0; s < kSB; ++s) {
      g += dz[s];
      l += lz[s];
    }
    out[OB3] = g;
    out[NP] = l;
  }
  __syncthreads();
  for (int e = t; e < kSB * HD; e += kBlock) {
    const int s = e / HD, o = e % HD;
    A2[s][o] = A2[s][o] > 0.f ? dz[s] * W[OW3 + o] : 0.f;
  }
  __syncthreads();
  // W2: 16 outputs per thread; b2
  {
    const int o = t >> 2, i0 = (t & 3) * 16;
    float acc[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) acc[u] = 0.f;
    float gb = 0.f;
    for (int s = 0; s < kSB; ++s) {
      const float d = A2[s][o];
      gb += d;
#pragma unroll
      for (int u = 0; u < 16; ++u) acc[u] = fmaf(d, H1[s][i0 + u], acc[u]);
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) out[OW2 + o * HD + i0 + u] = acc[u];
    if ((t & 3) == 0) out[OB2 + o] = gb;
  }
  __syncthreads();
  // dl/da1 = (h1 > 0) * (dl/da2 W2), in place of h1
  {
    const int s = t & (kSB - 1), i0 = (t >> 7) * 32;
    float acc[32];
#pragma unroll
    for (int u = 0; u < 32; ++u) acc[u] = 0.f;
    for (int o = 0; o < HD; ++o) {
      const float d = A2[s][o];
#pragma unroll
      for (int u = 0; u < 32; ++u) acc[u] = fmaf(d, W[OW2 + o * HD + i0 + u], acc[u]);
    }
#pragma unroll
    for (int u = 0; u < 32; ++u) H1[s][i0 + u] = H1[s][i0 + u] > 0.f ? acc[u] : 0.f;
  }
  __syncthreads();
  // W1: 2 outputs per thread; b1
  {
    const int o = t >> 2, a0 = (t & 3) * 2;
    float g0 = 0.f, g1 = 0.f, gb = 0.f;
    for (int s = 0; s < kSB; ++s) {
      const float d = H1[s][o];
      gb += d;
      g0 = fmaf(d, Xs[s][a0], g0);
      g1 = fmaf(d, Xs[s][a0 + 1], g1);
    }
    out[OW1 + o * NF + a0] = g0;
    out[OW1 + o * NF + a0 + 1] = g1;
    if ((t & 3) == 0) out[OB1 + o] = gb;
  }
}

// Sums the partial gradients in workgroup order; optionally one Adam step.
__global__ void __launch_bounds__(kBlock)
    k_mlp_reduce(const float* __restrict__ partial, int nwg, float* __restrict__ grad, float* __restrict__ loss,
                 float* __restrict__ P, float* __restrict__ M, float* __restrict__ V, int step, float lr,
                 float beta1, float beta2, float eps) {
  const int p = blockIdx.x * kBlock + threadIdx.x;
  if (p > NP) return;
  float g = 0.f;
  for (int w = 0; w < nwg; ++w) g += partial[(size_t)w * (NP + 1) + p];
  if (p == NP) {
    if (loss) *loss = g;
    return;
  }
  if (grad) grad[p] = g;
  if (P) {
    const float m = beta1 * M[p] + (1.f - beta1) * g;
    const float v = beta2 * V[p] + (1.f - beta2) * g * g;
    M[p] = m;
    V[p] = v;
    const float mh = m / (1.f - powf(beta1, (float)step));
    const float vh = v / (1.f - powf(beta2, (float)step));
    P[p] -= lr * mh / (sqrtf(vh) + eps);
  }
}

}  // namespace

std::vector<SkelBlock> skel_blocks(const Tree& t) {
  std::vector<SkelBlock> out;
  int samp = 0;
  for (int q = 1; q <= t.L; ++q)
    for (int i = 0; i < (1 << q); ++i) {
      const int c = node_id(q, i), sib = node_id(q, i ^ 1);
      SkelBlock b{c, t.lo[c], t.size(c), t.lo[sib], t.size(sib), samp};
      samp += b.m + b.nc;
      out.push_back(b);
    }
  return out;
}

int launch_skel_features(const int* rowptr, const int* col, const float* xyz, const double* K, int ldk,
                         const std::vector<SkelBlock>& blocks, float* feats, hipStream_t s, int cnt_depth,
                         int* dcount, const SkelBlock* d_blocks) {
  if (blocks.empty()) return HODLR_OK;
  for (const SkelBlock& b : blocks)
    if (b.m > kSideMax || b.nc > kSideMax) return fail(HODLR_EINVAL, "block side above 8192");
  DevBuf d;
  if (!d_blocks) {
    HODLR_TRY(d.ensure(blocks.size() * sizeof(SkelBlock)));
    HODLR_HIP(hipMemcpyAsync(d.p, blocks.data(), blocks.size() * sizeof(SkelBlock), hipMemcpyHostToDevice, s));
    d_blocks = d.as<SkelBlock>();
  }
  k_skel_features<<<dim3((unsigned)blocks.size(), 2), kFeatBlock, 0, s>>>(rowptr, col, xyz, K, ldk, d_blocks,
                                                                         feats, cnt_depth, dcount);
  HODLR_HIP(hipGetLastError());
  if (d.p) d.release_after(s);  // the block table goes back to the cache once the kernel has read it
  return HODLR_OK;
}

int launch_skel_labels(const std::vector<SkelBlock>& blocks, const int* piv, int kcap, const int* rank,
                       float* labels, hipStream_t s) {
  if (blocks.empty()) return HODLR_OK;
  DevBuf d;
  HODLR_TRY(d.ensure(blocks.size() * sizeof(SkelBlock)));
  HODLR_HIP(hipMemcpyAsync(d.p, blocks.data(), blocks.size() * sizeof(SkelBlock), hipMemcpyHostToDevice, s));
  k_skel_labels<<<(unsigned)blocks.size(), kBlock, 0, s>>>(d.as<SkelBlock>(), piv, kcap, rank, labels);
  HODLR_HIP(hipGetLastError());
  HODLR_HIP(hipStreamSynchronize(s));
  return HODLR_OK;
}

int launch_mlp_forward(const float* X, int N, const float* P, int bf16, float* z, hipStream_t s) {
  if (N <= 0) return HODLR_OK;
  const int tiles = (N + 31) / 32, per_wg = kBlock / 64;
  const int grid = std::min(2048, (tiles + per_wg - 1) / per_wg);
  k_mlp_forward<<<grid, kBlock, 0, s>>>(X, N, P, bf16, z);
  HODLR_HIP(hipGetLastError());
  return HODLR_OK;
}

int launch_mlp_grad(const float* X, const float* Y, int N, float* P, int bf16, float pos_weight, float* grad,
                    float* loss, float* M, float* V, int step, float lr, float beta1, float beta2, float eps,
                    hipStream_t s) {
  if (N <= 0) return fail(HODLR_EINVAL, "N must be >= 1");
  const int nwg = (N + kSB - 1) / kSB;
  DevBuf part;
  HODLR_TRY(part.ensure((size_t)nwg * (NP + 1) * sizeof(float)));
  k_mlp_grad<<<nwg, kBlock, 0, s>>>(X, Y, N, P, bf16, pos_weight, 1.f / (float)N, part.as<float>());
  HODLR_HIP(hipGetLastError());
  k_mlp_reduce<<<(NP + 1 + kBlock - 1) / kBlock, kBlock, 0, s>>>(part.as<float>(), nwg, grad, loss,
                                                                  M ? P : nullptr, M, V, step, lr, beta1,
                                                                  beta2, eps);
  HODLR_HIP(hipGetLastError());
  HODLR_HIP(hipStreamSynchronize(s));  // the partials go back to the cache
  return HODLR_OK;
}

}  // namespace hodlr
