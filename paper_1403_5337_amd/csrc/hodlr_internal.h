// Internal declarations shared by the HIP translation units of libhodlr.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <functional>
#include <string>
#include <vector>

#include "hodlr.h"
#include "gemm.h"

namespace hodlr {

// ---------------------------------------------------------------------------
// Errors
// ---------------------------------------------------------------------------
void set_error(const std::string& msg);
int fail(int code, const std::string& msg);

#define HODLR_HIP(call)                                                                    \
  do {                                                                                     \
    hipError_t e_ = (call);                                                                \
    if (e_ != hipSuccess)                                                                  \
      return ::hodlr::fail(HODLR_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

#define HODLR_TRY(call)          \
  do {                           \
    int s_ = (call);             \
    if (s_ != HODLR_OK) return s_; \
  } while (0)

// ---------------------------------------------------------------------------
// Limits.  Off-diagonal ranks are capped so that the per-node capacitance
// matrix and the ACA working slices fit in the 160 KB of LDS of one CU.
// ---------------------------------------------------------------------------
constexpr int kBlock = 256;          // threads per workgroup for most kernels
constexpr int kRankCap32 = 184;      // float: 184*185*4 B = 133 KB
constexpr int kRankCap64 = 128;      // double: 128*129*8 B = 132 KB
constexpr int kAcaSlice32 = 96;      // ACA rows/cols per workgroup (float)
constexpr int kAcaSlice64 = 64;      // (double)
constexpr int kLeafMax = 256;        // largest leaf block
constexpr int kMaxN = 1 << 20;

inline int rank_cap(int precision) { return precision == 64 ? kRankCap64 : kRankCap32; }
// the leaf inverse keeps a leaf in LDS: leaf <= 184 (float) / 128 (double)
inline int leaf_cap(int precision) { return precision == 64 ? kRankCap64 : kRankCap32; }

// ---------------------------------------------------------------------------
// Tree: node id of (level p, index i) is (1 << p) - 1 + i.
// ---------------------------------------------------------------------------
__host__ __device__ inline int node_id(int p, int i) { return (1 << p) - 1 + i; }

struct Tree {
  int n = 0, leaf = 0, L = 0;
  std::vector<int> lo, hi;  // per node id
  void build(int n_, int leaf_);
  int nnodes() const { return (2 << L) - 1; }
  int size(int id) const { return hi[id] - lo[id]; }
  int min_size(int p) const;
  int max_size(int p) const;
};

// caching device allocator (api.hip)
int dev_alloc(size_t nbytes, void** out);
void dev_free(void* p, size_t nbytes);
// released once the work queued so far on stream s is done, without waiting
void dev_free_after(void* p, size_t nbytes, hipStream_t s);
void release_cached_memory();
// pinned host blocks, kept in a process-wide cache (api.hip): pinning and
// unpinning memory are slow driver calls, so freed blocks are reused.  A block
// must not be returned while a copy from it may still be pending.
int pinned_alloc(size_t nbytes, void** out, size_t* got);
void pinned_free(void* p, size_t nbytes);
// events (no timing) from a process-wide pool: taking one creates it only if
// the pool is empty; an event goes back once no wait on it is still to be
// queued (a wait already queued is not affected by a later record)
int event_take(hipEvent_t* out);
void event_give(hipEvent_t e);

// ---------------------------------------------------------------------------
// Device buffer (RAII over the caching allocator)
// ---------------------------------------------------------------------------
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() { release(); }
  void release();             // back to the allocator cache
  void release_after(hipStream_t s);  // back to the cache once s's queued work is done
  int ensure(size_t nbytes);  // grow-only; contents not preserved
  template <typename T> T* as() const { return static_cast<T*>(p); }
};

}  // namespace hodlr

// ---------------------------------------------------------------------------
// The handle
// ---------------------------------------------------------------------------
struct hodlr_s {
  hodlr::Tree tree;
  int precision = 32;
  size_t esize = 4;  // bytes per element of the factorization
  int method = HODLR_ACA;
  int depth = 1;
  int max_rank = 0;
  double tol = 1e-4;
  int device = 0;

  std::vector<int> rank;   // per node id (root 0)
  std::vector<int> rcols;  // per level q = 1..L at index q-1: column width
  std::vector<int> off;    // per level q at index q-1: column offset
  int R = 0;               // total columns of the panels
  int bmax = 0;            // largest leaf
  int nleaf = 0;

  hodlr::DevBuf d_lo, d_hi, d_rank;
  hodlr::DevBuf Y;      // n x R: U panels, then the factorization (d / c)
  hodlr::DevBuf W;      // n x R: V panels
  hodlr::DevBuf E;      // n x RE: solve correction operators E_c = d_c S^-1(rows, :)
  std::vector<int> offE;  // per level q at index q-1: column offset in E (width 2 rq)
  hodlr::DevBuf Xtmp;   // n x 16: solve work vector
  hodlr::DevBuf Kinv;   // nleaf x bmax x bmax: leaf inverses
  hodlr::DevBuf Sinv;   // per internal node: (2 rq)^2 inverse capacitance
  std::vector<size_t> sinv_off;  // per parent level p = 0..L-1 (elements)
  hodlr::DevBuf G;      // work: per-node panel products
  size_t p_half = 0;    // elements of one partial-product buffer of the solve
  hodlr::DevBuf Ybuf;   // work: per-node Woodbury solutions
  hodlr::DevBuf status; // int[4]: 0 singular flag, 1 node, 2 abort
  hodlr::DevBuf gemm_tab, gemm_work;  // arenas of the batched products
  std::vector<int> skel_k;  // learned build, per node: skeleton size kept, 0 = ACA fallback
  size_t gemm_tab_used = 0, gemm_work_used = 0;
  void* gemm_host = nullptr;  // pinned staging of the task tables
  size_t gemm_host_bytes = 0;
  int gemm_mode = hodlr::kGemmDirect;    // direct, record or replay (gemm.h)
  std::vector<hodlr::GemmRec> gemm_recs;  // the recorded products, in call order
  size_t gemm_rec_pos = 0;               // next product to replay
  size_t gemm_staged = 0;                // bytes of recorded tables in the staging
  bool gemm_replan = false;              // an arena grew while recording: record again
  bool capturing = false;     // launches are being recorded into a graph
  hodlr::DevBuf lstatus;      // int[4]: status of the leaf inverses run by the build
  bool leaves_inverted = false;  // the build already inverted the leaf blocks
  int leaf_singular = -1;        // node id of a singular leaf found by the build
  bool factored = false;
  // hodlr_factor_async: the status words go to pinned memory behind the
  // factorization (status_ev recorded after them) and are read by the next
  // call that waits on the handle (settle_factor_status)
  bool status_pending = false;
  int* pin_status = nullptr;
  size_t pin_status_bytes = 0;
  hipEvent_t status_ev = nullptr;
  // events recorded behind work that calls leave queued on the handle's
  // buffers (hodlr_destroy waits only if one has not completed)
  std::vector<hipEvent_t> inflight;
  hodlr_s() = default;
  hodlr_s(const hodlr_s&) = delete;
  hodlr_s& operator=(const hodlr_s&) = delete;
  ~hodlr_s() {
    if (gemm_host) hodlr::pinned_free(gemm_host, gemm_host_bytes);
    if (pin_status) hodlr::pinned_free(pin_status, pin_status_bytes);
    if (status_ev) hodlr::event_give(status_ev);
    for (hipEvent_t e : inflight) hodlr::event_give(e);
  }
};

namespace hodlr {

// A factorization queued by hodlr_factor_async: waits for its status words
// (status_ev) and returns ESINGULAR as hodlr_factor does (the handle is then
// no longer factorized); HODLR_OK when nothing is pending (api.hip).
int settle_factor_status(hodlr_s* h);
// Records an event on s behind work just queued on the handle's buffers
// (completed events are recycled first; at most 16 are kept).
int mark_inflight(hodlr_s* h, hipStream_t s);
int singular_status(const int* st);

// ---------------------------------------------------------------------------
// Kernel launchers (one translation unit each)
// ---------------------------------------------------------------------------
// order.hip
int launch_rcb(const float* coords, int n, const Tree& t, int* perm, hipStream_t s);
// the tree's node ranges (lo, then hi) on the current device, uploaded once
// per (device, n, leaf) and kept for the process
int device_tree_ranges(const Tree& t, const int** lo, const int** hi);
int launch_permute(const double* Kin, int n, int ldi, const int* perm, double* Kout, int ldo,
                   hipStream_t s);
int launch_permute_rows(const float* in, int n, int width, const int* perm, float* out, hipStream_t s);
int launch_permute_graph(const int* rowptr, const int* col, int n, const int* perm,
                         int* rowptr_out, int* col_out, hipStream_t s);

// aca.hip: compress every off-diagonal block (or only the blocks of the
// listed nodes) into capped panels; piv (optional, 2 * rank cap ints per node
// below the root, level order) receives the pivot rows, then the pivot
// columns, of every cross.
int launch_aca(hodlr_s* h, const double* K, int ldk, void* Ucap, void* Vcap,
               const std::vector<int>& capoff, const std::vector<int>& cap, hipStream_t s,
               const std::vector<int>* nodes = nullptr, int* piv = nullptr);

// bdlr.hip: boundary-distance skeletons of every off-diagonal block
// max_skel: cap on picked rows (columns) per side (0 = the library's 192 /
// 128); piv_export (optional, 2 skel_stride ints per node below the root,
// level order) receives the skeleton's pivot rows, then columns
int launch_bdlr(hodlr_s* h, const double* K, int ldk, const int* rowptr, const int* col, void* Ucap,
                void* Vcap, const std::vector<int>& capoff, const std::vector<int>& cap, hipStream_t s,
                int max_skel = 0, int* piv_export = nullptr);
int skel_stride(int precision);

// bdlr.hip: BDLR with the sampled error monitor of Sec. 5.3: blocks above
// accept take one more distance layer, up to max_depth
int launch_bdlr_adaptive(hodlr_s* h, const double* K, int ldk, const int* rowptr, const int* col, int max_depth,
                         int max_skel, unsigned long long seed, double accept, void* Ucap, void* Vcap,
                         const std::vector<int>& capoff, const std::vector<int>& cap, hipStream_t s);

// bdlr.hip: learned proposals with sampled-error check and ACA fallback
int launch_learned(hodlr_s* h, const double* K, int ldk, const int* rowptr, const int* col, const float* xyz,
                   const float* params, int kinit, unsigned long long seed, double accept, void* Ucap, void* Vcap,
                   const std::vector<int>& capoff, const std::vector<int>& cap, hipStream_t s);

// factor.hip
int launch_stage_leaves_from_K(hodlr_s* h, const double* K, int ldk, hipStream_t s);
int launch_stage_leaves_packed(hodlr_s* h, const double* leaves, hipStream_t s);
int launch_repack(hodlr_s* h, const void* Ucap, const void* Vcap, int ldcap,
                  const std::vector<int>& capoff, hipStream_t s);
// symmetric build: right children's panels and ranks from their left siblings
int launch_mirror(hodlr_s* h, hipStream_t s);
int launch_from_f64_panels(hodlr_s* h, const double* Up, const double* Vp, hipStream_t s);
int launch_to_f64_panels(hodlr_s* h, double* Up, double* Vp, hipStream_t s);
int factor_impl(hodlr_s* h, hipStream_t s);
// leaf inverses in place (status: int[4], zeroed here; [0] = 1 and [1] = node
// id for a singular leaf)
int launch_leaf_inverse(hodlr_s* h, int* status, hipStream_t s);
int ensure_work(hodlr_s* h, int ncols);

// solve.hip
// in place; gate (nrhs column flags, may be NULL): every launch does nothing
// once all columns have stopped
int apply_impl(hodlr_s* h, void* X, int ldx, int nrhs, hipStream_t s, const int* gate = nullptr);
size_t solve_partial_elems(const hodlr_s* h);

// api.hip: streams for work that runs beside the caller's stream (default
// priority, one pair per host thread, created on first use)
int side_stream(int which, hipStream_t* out);

// prof.hip: event timing of wrapped launches (hodlr_prof_enable)
bool prof_on();
void prof_suspend(bool on);  // this thread records nothing while suspended
void tune_freeze(bool on);   // this thread's tune_choice uses kept choices or the fallback, timing nothing
void prof_mark(const char* name, hipStream_t s, bool begin);
// records so far, and dropping the records from a count on: launches known
// afterwards to have done nothing (a step queued after its columns stopped)
// are kept out of the per-kernel times
size_t prof_count();
void prof_drop_from(size_t first);
// launch(c) for candidate c < ncand, the choice for `key` found by timing on
// first use (see prof.hip); *pick receives it
bool tune_known(const std::string& key);  // a choice is kept for key
int tune_choice(const std::string& key, int ncand, int fallback, const std::function<int(int)>& launch,
                hipStream_t s, int* pick);
std::string tune_report();
struct ProfScope {
  const char* name;
  hipStream_t s;
  bool on;
  ProfScope(const char* n, hipStream_t st, bool enabled = true) : name(n), s(st), on(enabled && prof_on()) {
    if (on) prof_mark(name, s, true);
  }
  ~ProfScope() {
    if (on) prof_mark(name, s, false);
  }
};

// skel.hip: learned skeleton proposer (features, labels, scorer)
constexpr int kMlpParams = 64 * 8 + 64 + 64 * 64 + 64 + 64 + 1;
struct SkelBlock {
  int node, row0, m, col0, nc, samp0;  // samp0: first sample (rows, then columns)
};
std::vector<SkelBlock> skel_blocks(const Tree& t);  // level order; samples total 2 n L
// dcount (optional, 2 ints per block): row and column vertices at distance < cnt_depth
// d_blocks (optional): the block table already on the device (else it is
// uploaded here)
int launch_skel_features(const int* rowptr, const int* col, const float* xyz, const double* K, int ldk,
                         const std::vector<SkelBlock>& blocks, float* feats, hipStream_t s, int cnt_depth = 0,
                         int* dcount = nullptr, const SkelBlock* d_blocks = nullptr);
int launch_skel_labels(const std::vector<SkelBlock>& blocks, const int* piv, int kcap, const int* rank,
                       float* labels, hipStream_t s);
int launch_mlp_forward(const float* X, int N, const float* P, int bf16, float* z, hipStream_t s);
// gradient (grad, loss may be NULL); with M, V non-NULL also one Adam step on P
int launch_mlp_grad(const float* X, const float* Y, int N, float* P, int bf16, float pos_weight, float* grad,
                    float* loss, float* M, float* V, int step, float lr, float beta1, float beta2, float eps,
                    hipStream_t s);

// gmres.hip: the float64 product of GMRES, as split-K partial sums
int matvec_partials(const double* K, int ldk, int n, const double* src, int lds, int s, double* part,
                    hipStream_t st, int* nsplit);
size_t matvec_partial_elems(int n, int s);  // elements of part for (n, s)

// cg.hip
int cg_impl(const double* K, int n, int ldk, hodlr_s* M, const double* B, int nrhs, int ldb, double* X, int ldx,
            double tol, int maxit, int* iters, double* relres, hipStream_t s);

// gmres.hip: workspace bytes of gmres_solve_noalloc for (n, s, restart,
// preconditioner precision 32 / 64, 0 for none) and the fixed limit
size_t gmres_noalloc_bytes(int n, int s, int restart, int precision);
size_t gmres_noalloc_limit();
int gmres_impl(const double* K, int n, int ldk, hodlr_s* M, const double* B, int nrhs, int ldb,
               double* X, int ldx, double tol, int maxit, int restart, int* iters,
               double* relres, hipStream_t s, bool noalloc = false);

}  // namespace hodlr
