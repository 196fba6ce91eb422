// Batched small dense products (gemm.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

struct hodlr_s;

namespace hodlr {

enum { kGemmOverwrite = 0, kGemmAccumulate = 1, kGemmAddIdentity = 2 };

// C (m x n, ld ldc) = alpha op(A) B, then + C (kGemmAccumulate) or + I
// (kGemmAddIdentity).  op(A) is A (m x k, ld lda) or, with transA, the
// transpose of A stored k x m (ld lda).  B is k x n (ld ldb).  Column-major,
// element type of the handle's precision.  ksplit > 1 splits k over that many
// workgroups per tile and sums the partial tiles afterwards.
struct GemmTask {
  const void* A = nullptr;
  const void* B = nullptr;
  void* C = nullptr;
  int m = 0, n = 0, k = 0, lda = 0, ldb = 0, ldc = 0;
  int transA = 0, mode = kGemmOverwrite, ksplit = 1;
  double alpha = 1.0;
};

// All tasks in one launch (plus one for the split sums).  Task tables and
// split partials live in per-handle arenas that the caller resets (gemm_reset)
// once the stream has drained.
int gemm_batched(hodlr_s* h, const std::vector<GemmTask>& tasks, hipStream_t s);

// Recording.  In kGemmRecord mode a call only writes its task tables to the
// handle's pinned staging (no copy, no launch) and keeps what its launches
// need; gemm_upload then moves every recorded table to the device with one
// copy, and in kGemmReplay mode each call launches the next recorded product
// (its task list is not looked at again).  A factorization records its whole
// product sequence first, so its tables cost one copy instead of one per call.
enum { kGemmDirect = 0, kGemmRecord = 1, kGemmReplay = 2 };
struct GemmRec {
  const char* tb = nullptr;  // device table block: tasks, then the sums' tasks (o1) and parts (o2)
  int ntasks = 0, tiles = 0, nred = 0, maxmn = 0;
  size_t o1 = 0, o2 = 0;
};
int gemm_upload(hodlr_s* h, hipStream_t s);
void gemm_reset(hodlr_s* h);
// sizes the arenas (and the pinned staging of the task tables) up front, so
// that a factorization needs no growth (required under graph capture)
int gemm_prepare(hodlr_s* h, size_t tab_bytes, size_t work_bytes, hipStream_t s);
size_t gemm_table_bound(int ntasks);  // table-arena bytes one call with ntasks tasks may take

}  // namespace hodlr
