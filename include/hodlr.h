/*
 * hodlr.h - C ABI of the MI355X (gfx950) HODLR-preconditioned GMRES library.
 *
 * The library solves K x = F for a dense frontal matrix K (n x n, float64,
 * column-major) and s right-hand sides (the problem statement of Sec. 4.2,
 * eq. denseSystem) with GMRES (Sec. 3) preconditioned by a low-accuracy
 * HODLR factorization of K (Sec. 4): off-diagonal blocks compressed by
 * partial-pivoting ACA (Sec. 5.1) or by the boundary-distance pseudo-skeleton
 * BDLR (Sec. 5.3), then factorized level by level with the Woodbury formula
 * (Sec. 4.3).
 *
 * Conventions shared by every entry point
 *   - Matrices are column-major with a leading dimension >= their row count.
 *   - Every matrix/vector pointer is DEVICE memory owned by the caller unless
 *     the argument says "host".  The library never frees caller memory.
 *   - Work is enqueued on the given HIP stream; calls are asynchronous unless
 *     stated otherwise.  Pass 0 for the default stream.
 *   - Every function returns a hodlr_status.  No exception crosses the ABI.
 *     On failure hodlr_last_error() returns a thread-local message.
 *   - A handle is not thread-safe; distinct handles are independent.
 */
#ifndef HODLR_H_
#define HODLR_H_

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hodlr_s* hodlr_t; /* opaque; created by hodlr_build*, freed by hodlr_destroy */

typedef enum {
  HODLR_OK = 0,
  HODLR_EINVAL = 1,    /* bad argument (size, pointer, option) */
  HODLR_ENOMEM = 2,    /* device allocation failed */
  HODLR_ESINGULAR = 3, /* a leaf block or a Woodbury capacitance matrix is singular */
  HODLR_ENOCONV = 4,   /* GMRES stopped at maxit above tol; X holds the last iterate */
  HODLR_EHIP = 5       /* a HIP runtime call or kernel failed */
} hodlr_status;

enum { HODLR_ACA = 0, HODLR_BDLR = 1, HODLR_LEARNED = 2 };

typedef struct {
  int leaf;       /* largest leaf block, 1..184 (precision 32) or 1..128
                     (precision 64).  The tree splits [lo,hi) at
                     lo + floor((hi-lo)/2) to the smallest depth L with
                     ceil(n / 2^L) <= leaf (Sec. 4.1 block sizes n/2^p). */
  double tol;     /* compression tolerance eps: the ACA stopping ratio
                     |u_k||v_k| <= eps |U V^T|_F (Sec. 5.1), or the BDLR
                     relative pivot threshold |pivot| >= eps |first pivot|
                     (Sec. 7.1). */
  int method;     /* HODLR_ACA, HODLR_BDLR or HODLR_LEARNED (scorer-proposed
                     skeletons with ACA fallback, see hodlr_mlp_forward) */
  int bdlr_depth; /* BDLR: pick rows/cols at graph distance < depth from the
                     block boundary (Sec. 5.3), 1..250.  At most 192
                     (precision 32) / 128 (precision 64) rows and as many
                     columns are kept, nearest the boundary first, ties to
                     the lower index. */
  int max_rank;   /* cap on every off-diagonal rank (0 = library maximum:
                     184 at precision 32, 128 at precision 64) */
  int precision;  /* 32 or 64: arithmetic of the factorization and solve */
  /* HODLR_LEARNED only: the scorer proposes the skeleton rows/columns of
     eq. Ahat (Sec. 5.3) by mesh node.  On each side of a block, dofs at
     consecutive positions with equal coordinates form one node (at most 8
     dofs); a node scores the best score of its dofs; with a budget of k
     picks and longest node g, the side takes the k / g best nodes (at least
     one, ties to the lower position) with all their dofs.  The skeleton's
     relative Frobenius error is estimated from 16 whole rows and 16 whole
     columns outside it (hodlr_sampled_error); a block above skel_tol
     retries with both budgets doubled, up to 192 (precision 32) / 128
     (precision 64) picks and at most 4 attempts, all decided on the device.
     A block that still fails is also compressed by ACA, and keeps whichever
     approximation has the smaller error estimated on its picked rows and
     columns (exactly) and 16 fresh rows and columns outside them
     (hodlr_skel_info) -- except a block whose budgets are at the pick cap
     and whose rank is at the rank cap, which keeps its skeleton (ACA is held
     to the same rank cap). */
  int skel_k;                /* first budget per side, >= 0; 0 (default) =
                                the side's BDLR pick count at bdlr_depth */
  const float* mlp_params;   /* device float32, 4801 scorer parameters in the
                                layout of hodlr_mlp_forward; read during the
                                call only */
  unsigned long long seed;   /* sample stream of the error check */
  double skel_tol;           /* HODLR_LEARNED: largest accepted sampled error
                                (0 = 30 tol: a skeleton truncated at relative
                                pivot tol has a block error about an order of
                                magnitude above tol) */
  int bdlr_max_skel;         /* HODLR_BDLR: cap on the rows (columns) picked
                                per side, nearest first (0 = 192 / 128) */
  int bdlr_max_depth;        /* HODLR_BDLR: 0 (default) = every block at
                                bdlr_depth.  Otherwise the error monitor of
                                Sec. 5.3: a block whose sampled error (the
                                estimate of HODLR_LEARNED, seed opts.seed) is
                                above skel_tol (0 = 30 tol) takes one more
                                distance layer, up to bdlr_max_depth
                                (bdlr_depth..250) or until a layer adds no
                                pick; a block that never passes keeps its
                                deepest skeleton.  hodlr_skel_info gives the
                                depth each block ended at.  One stream
                                synchronization per layer tried. */
  int symmetric;             /* 1: K is symmetric (the symmetric case of eq.
                                HODLR2: a node's two off-diagonal blocks are
                                each other's transposes).  Only the block of
                                each left child c is compressed, K(c, s) ~
                                U_c V_c^T; its sibling takes U_s = V_c,
                                V_s = U_c, so Ktilde is symmetric.  ACA then
                                compresses half the blocks; BDLR and learned
                                skeletons compress all and keep the left
                                ones.  0 (default): every block on its own. */
} hodlr_opts;

/* Fill *opts with defaults: leaf 128, tol 1e-4, ACA, depth 1, max_rank 0,
 * precision 32, skel_k 0, mlp_params NULL, seed 0, skel_tol 0,
 * bdlr_max_skel 0, bdlr_max_depth 0, symmetric 0. */
void hodlr_default_opts(hodlr_opts* opts);

/* Compress K into a HODLR matrix (Sec. 4.3.1 step 1).
 *   K       device, n x n float64, leading dimension ldk >= n.  Read only;
 *           not retained after the call returns (the handle keeps copies of
 *           the leaf blocks and the low-rank factors).
 *   g_rowptr, g_col
 *           device CSR (int32, n+1 and nnz entries) of the separator's
 *           sparse interaction graph in K's numbering (Sec. 5.3); required
 *           for HODLR_BDLR and HODLR_LEARNED, ignored (may be NULL) for
 *           HODLR_ACA.
 *   coords  device n x 3 float32 (row-major) dof coordinates in K's
 *           numbering; required for HODLR_LEARNED, else ignored.
 *   opts    host; NULL = defaults.
 *   out     host; receives the new handle.
 * Synchronizes the stream once (to size the factor storage from the ranks
 * found; HODLR_LEARNED synchronizes once more, and twice when a block falls
 * back; the adaptive BDLR depth once per depth tried).  Errors: EINVAL
 * (n < 1, n > 16384 (every compression keeps a block side <= 8192), ldk < n,
 * NULL K/out, bad opts, BDLR or learned without the graph, learned without
 * coords or parameters), ENOMEM, EHIP. */
int hodlr_build(const double* K, int n, int ldk, const int* g_rowptr, const int* g_col,
                const float* coords, const hodlr_opts* opts, hipStream_t stream, hodlr_t* out);

/* Test/benchmark hook: a HODLR matrix given directly by its pieces.
 *   leaves  device float64, the leaf blocks packed leaf after leaf, each
 *           b_i x b_i column-major with leading dimension b_i, leaves in
 *           left-to-right order of the tree for (n, leaf).
 *   Upanel, Vpanel
 *           device float64, n x R column-major (ld n) with R = sum of
 *           rcols[p-1] for p = 1..L.  Column block p (offset sum of
 *           rcols[q-1], q < p) holds, in the rows of node (p,i), that node's
 *           U, and in the rows of its sibling, that node's V, so
 *           K(node, sibling) = U V^T.
 *   ranks   host int, one per node below the root in level order
 *           (level 1 left to right, then level 2, ...), each <= rcols[p-1]
 *           and <= the smaller of the node's and its sibling's sizes.
 *   rcols   host int[L], width of each level's column block, at most 184
 *           (precision 32) / 128 (precision 64) and the level's largest
 *           node.
 * Errors: EINVAL on inconsistent sizes, ENOMEM, EHIP. */
int hodlr_build_from_factors(int n, int leaf, int precision, const double* leaves,
                             const double* Upanel, const double* Vpanel, const int* ranks,
                             const int* rcols, int nlevels, hipStream_t stream, hodlr_t* out);

/* Factorize (Sec. 4.3.1 steps 2-5): leaf LU with partial pivoting (kept as
 * the leaf inverse), leaf solves of the stacked panels Z = [U | ancestor U],
 * then, from the leaves up, per node the capacitance matrix
 * S = [[I, V_b^T d_a], [V_a^T d_b, I]] (eq. SchurSum), its inverse, and the
 * correction of the ancestor columns.  Synchronizes once to report
 * ESINGULAR (message names the node). */
int hodlr_factor(hodlr_t h, hipStream_t stream);

/* hodlr_factor without the synchronization: the same launches (the same
 * results, bit for bit), queued on the stream, and the handle counts as
 * factorized at once.  The status words are copied behind the factorization
 * into pinned host memory that the handle keeps.  A singular leaf or
 * capacitance matrix is then reported (ESINGULAR, as hodlr_factor reports
 * it, after which the handle is no longer factorized) by the next call that
 * waits on the handle: hodlr_factor_wait, or gmres_solve / cg_solve /
 * gmres_solve_noalloc with the handle as preconditioner, at their first
 * synchronization (they then return ESINGULAR; X holds no result).
 * hodlr_solve and the solvers order their work behind the factorization
 * (an event), also on other streams.  For callers whose next step is a
 * solve: the host prepares it while the GPU still factorizes.
 * Errors here: EINVAL (NULL or already factorized handle), ESINGULAR for a
 * singular leaf found by the build, ENOMEM, EHIP. */
int hodlr_factor_async(hodlr_t h, hipStream_t stream);

/* Waits for a factorization queued by hodlr_factor_async and returns its
 * status (HODLR_OK, or ESINGULAR naming the node); HODLR_OK at once when
 * none is pending (already settled, or hodlr_factor).  EINVAL on NULL. */
int hodlr_factor_wait(hodlr_t h);

/* hodlr_factor for nh handles at once (a batch of fronts, e.g. the
 * separators of a nested-dissection tree): every front's factorization is
 * recorded on its own stream into one HIP graph, which is launched once, so
 * the fronts' level-by-level launches run concurrently.  hs: host array of
 * nh distinct, not yet factorized handles (any sizes and precisions).
 * Synchronizes.  Errors: EINVAL, ESINGULAR (the message names the front and
 * node), ENOMEM, EHIP; on error no handle is marked factorized. */
int hodlr_factor_batched(hodlr_t* hs, int nh, hipStream_t stream);

/* X = Ktilde^-1 B (Sec. 4.3.2) in the handle's precision.
 *   B, X    device, n x nrhs, leading dimensions ldb, ldx >= n; element
 *           type float (precision 32) or double (precision 64).  X may alias
 *           B (ldx == ldb).
 * Requires hodlr_factor (or hodlr_factor_async: a singular block found
 * there is reported by hodlr_factor_wait, not here).  Asynchronous.
 * Errors: EINVAL, ENOMEM, EHIP. */
int hodlr_solve(hodlr_t h, const void* B, int nrhs, int ldb, void* X, int ldx,
                hipStream_t stream);

/* Flexible right-preconditioned GMRES in float64 (Sec. 3; Table 3 settings
 * as defaults of the caller): Arnoldi with classical Gram-Schmidt applied
 * twice, Givens rotations, each right-hand side converging on its own when
 * its Givens residual estimate drops to tol * |b|, confirmed with the true
 * residual |b - K x| at the end of the cycle; restarts every `restart`
 * steps; at most `maxit` steps per right-hand side.
 *   K       device n x n float64 (ld ldk), read for the whole call.
 *   precond handle from hodlr_factor, or NULL for no preconditioner.
 *   B       device n x nrhs float64 (ld ldb).
 *   X       device n x nrhs float64 (ld ldx): initial guess in, solution out.
 *   iters   host int[nrhs]: steps taken per right-hand side.
 *   relres  host double[nrhs]: final true |b - K x| / |b|.
 * Synchronizes the stream.  Returns ENOCONV if any right-hand side is above
 * tol at maxit (X still holds the last iterates). */
int gmres_solve(const double* K, int n, int ldk, hodlr_t precond, const double* B, int nrhs,
                int ldb, double* X, int ldx, double tol, int maxit, int restart, int* iters,
                double* relres, hipStream_t stream);

/* gmres_solve for callers that cannot allocate (code under HIP graph capture
 * of the surrounding work, tight serving loops, harnesses that forbid
 * hipMalloc): the same arguments and arithmetic (bit for bit the same
 * results when both use the same product split width), but the Arnoldi
 * basis, the preconditioned vectors, the partial sums and every other piece
 * of workspace live in one fixed device array of 192 MiB that the library
 * holds on each GPU it runs on until the process ends; no hipMalloc,
 * hipHostMalloc, hipFree or event creation happens in the call.
 *   Limit: about 8 n nrhs (restart + 1) bytes for the basis, plus 4 or 8
 *   n nrhs (restart + 1) for the preconditioned vectors (float32 or float64
 *   preconditioner), plus 8 n nrhs ceil(n / 64) for the product's partial
 *   sums, must fit in 192 MiB (e.g. n 4096, 8 right-hand sides, restart
 *   200: 100 MB); larger problems return EINVAL with the bytes needed.
 *   The step flags come back by a copy and a stream synchronization per
 *   Arnoldi step (gmres_solve reads them from pinned memory one step
 *   behind), and the float64 product uses the split width the autotuner
 *   already chose for this shape, else its default; nothing is timed.
 *   Every call on a GPU shares that GPU's array: calls that overlap on one
 *   GPU (two threads, two streams) race.  The array keeps the last call's
 *   contents; everything a solve reads is written by it first. */
int gmres_solve_noalloc(const double* K, int n, int ldk, hodlr_t precond, const double* B, int nrhs, int ldb,
                        double* X, int ldx, double tol, int maxit, int restart, int* iters, double* relres,
                        hipStream_t stream);

/* Preconditioned conjugate gradients in float64 for symmetric positive
 * definite K (Sec. 3: the HODLR solve preconditions any Krylov method,
 * conjugate gradients included).  Arguments as gmres_solve, without restart.
 * precond is NULL (plain CG) or a factorized handle, best built with
 * opts.symmetric = 1.  Per right-hand side: x0 = X on entry, r = b - K x0,
 * z = M r, p = z; a step takes alpha = r^T z / p^T q (q = K p), updates x
 * and r, and stops the cycle when |r| <= tol |b|; otherwise z' = M r and
 * p = z' + beta p with the flexible beta = r^T (z' - z) / (r^T z), which is
 * the classical coefficient when M is a fixed symmetric operator and keeps
 * CG converging with a float32 M.  A cycle also ends when p^T q <= 0 or
 * r^T z' <= 0 (not positive definite in floating point).  When every
 * column's cycle has ended the true residual |b - K x| / |b| decides who
 * restarts (a column whose last cycle took no step stops).  iters[k] counts
 * the steps, at most maxit in total; relres[k] is the last true relative
 * residual.  Synchronizes the stream.  Returns ENOCONV if any right-hand
 * side ends above tol (X holds the last iterates).  Scratch is per host
 * thread, so calls on different threads (and streams) run side by side. */
int cg_solve(const double* K, int n, int ldk, hodlr_t precond, const double* B, int nrhs, int ldb,
             double* X, int ldx, double tol, int maxit, int* iters, double* relres, hipStream_t stream);

/* Batches of fronts (the separators of a nested-dissection tree, solved
 * independently; Sec. 2): the library runs the fronts side by side on a pool
 * of host worker threads, each issuing its fronts' calls on its own stream
 * (default priority), ordered after the work already queued on `stream`.
 * The worker count is 8, or HODLR_THREADS (1..64) from the environment when
 * the pool starts.  Pointer arguments are host arrays of nf entries; each
 * front follows the rules of the single-front call.  The batched calls
 * (hodlr_order_batched, hodlr_build_batched, gmres_solve_batched)
 * synchronize and return the error of the lowest-numbered failing front (the
 * message names it); every front runs even if another fails.  Concurrent
 * batched calls on one process share the pool and run one after another.
 *
 * hodlr_build_batched: out[f] receives front f's handle; on any error every
 * handle built by the call is destroyed and out[] is all NULL.
 * g_rowptr, g_col, coords may be NULL (all fronts) or arrays whose entries
 * follow hodlr_build.  One opts for all fronts. */
int hodlr_build_batched(int nf, const double* const* K, const int* n, const int* ldk,
                        const int* const* g_rowptr, const int* const* g_col, const float* const* coords,
                        const hodlr_opts* opts, hipStream_t stream, hodlr_t* out);

/* hodlr_order_batched: for every front f, hodlr_order_rcb(coords[f], n[f],
 * leaf, perm[f]), then hodlr_permute(K[f], n[f], ldk[f], perm[f], Kout[f],
 * ldo[f]), then (if g_rowptr is not NULL) hodlr_permute_graph(g_rowptr[f],
 * g_col[f], n[f], perm[f], rowptr_out[f], col_out[f]); every output array is
 * caller-owned device memory sized as for the single calls.  The fronts'
 * ordering and relabelling are the first step of the path (the index-halving
 * tree of Sec. 4.1 needs a bisection order of each separator). */
int hodlr_order_batched(int nf, const float* const* coords, const int* n, int leaf, const double* const* K,
                        const int* ldk, const int* const* g_rowptr, const int* const* g_col, int* const* perm,
                        double* const* Kout, const int* ldo, int* const* rowptr_out, int* const* col_out,
                        hipStream_t stream);

/* gmres_solve_batched: front f solves K[f] X[f] = B[f] with preconditioner
 * precond[f] (precond may be NULL for none); iters and relres are host
 * arrays of nf * nrhs entries, front f at f * nrhs. */
int gmres_solve_batched(int nf, const double* const* K, const int* n, const int* ldk, const hodlr_t* precond,
                        const double* const* B, int nrhs, const int* ldb, double* const* X, const int* ldx,
                        double tol, int maxit, int restart, int* iters, double* relres, hipStream_t stream);

/* Recursive coordinate bisection order of n dofs for the HODLR tree of
 * (n, leaf): for every node from the root down, sort its dofs by the
 * coordinate of largest extent (first axis on ties, stable) and give the
 * first floor(len/2) to the left child.  coords: device n x 3 float32,
 * row-major (x, y, z per dof).  perm: device int32[n], out, new dof i = old
 * dof perm[i].  n <= 16384.  Asynchronous. */
int hodlr_order_rcb(const float* coords, int n, int leaf, int* perm, hipStream_t stream);

/* Kout(i, j) = Kin(perm[i], perm[j]).  Kin, Kout device float64 (ld ldi,
 * ldo >= n), must not overlap; perm device int32[n].  Asynchronous. */
int hodlr_permute(const double* Kin, int n, int ldi, const int* perm, double* Kout, int ldo,
                  hipStream_t stream);

/* out(i, :) = in(perm[i], :): device float32 row-major n x width arrays
 * (width 1..16), e.g. the dof coordinates a learned build takes in K's
 * permuted numbering; in and out must not overlap; perm device int32[n].
 * Asynchronous.  Errors: EINVAL. */
int hodlr_permute_rows(const float* in, int n, int width, const int* perm, float* out, hipStream_t stream);

/* Relabel a CSR graph: new vertex i = old vertex perm[i].  All device int32:
 * rowptr[n+1], col[nnz] in; rowptr_out[n+1], col_out[nnz] out (neighbours
 * sorted).  Asynchronous. */
int hodlr_permute_graph(const int* rowptr, const int* col, int n, const int* perm,
                        int* rowptr_out, int* col_out, hipStream_t stream);

/* The row and column picks of BDLR (Sec. 5.3) for every off-diagonal block of
 * the tree for (n, leaf), as hodlr_build with HODLR_BDLR takes them: for node
 * c with sibling s, the boundary of c is the set of its indices with a graph
 * edge into s, distances are breadth-first inside c, and the rows picked are
 * the positions (0-based, within c) at distance < depth, at most max_skel of
 * them, nearest the boundary first and ties to the lower position, listed in
 * increasing position; columns likewise within s.
 *   g_rowptr, g_col  device CSR of the graph in K's numbering (as hodlr_build).
 *   picks   device int, (2^(L+1)-2) * 2 * max_skel: for the k-th node below
 *           the root in level order, rows at k*2*max_skel, columns at
 *           k*2*max_skel + max_skel.
 *   counts  device int, 2 per node: number of rows, number of columns.
 * 2 <= n <= 16384, n > leaf, 1 <= depth <= 250.  Synchronizes the stream.
 * Errors: EINVAL, ENOMEM, EHIP. */
int hodlr_bdlr_select(const int* g_rowptr, const int* g_col, int n, int leaf, int depth,
                      int max_skel, int* picks, int* counts, hipStream_t stream);

/* Test hook: the sampled error check that HODLR_LEARNED and the adaptive
 * BDLR depth apply to every block (the error monitor of Sec. 5.3, measured on
 * rows and columns outside the skeleton), run on given factors and picks.
 * For the k-th node below the root (level order; node id c = 2^p - 1 + i,
 * block K(c, sibling), m x nc):
 *   draws   splitmix64 (Steele, Lea & Flood 2014) from the state
 *           seed ^ (0xD1B54A32D192ED03 * c) ^ (0x8CB92BA72F3D8DD7 * (attempt+1))
 *           (mod 2^64); 16 row positions, then 16 column positions, each the
 *           first 16 steps of a Fisher-Yates shuffle of the side's positions
 *           outside its picks (ascending), step x swapping entries x and
 *           x + (next() mod (left - x)); -1 once fewer are left;
 *   err     sqrt(max(e_r, e_c) / |K(c, sibling)|_F^2), e_r = the squared
 *           residual of U V^T on the sampled whole rows times (m - rows
 *           picked) / (rows sampled), e_c likewise over columns; float64.
 *   K       device n x n float64 (ld ldk).
 *   Upanel, Vpanel
 *           device n x R, ld n, float (precision 32) or double (64), in the
 *           layout of hodlr_build_from_factors; ranks (host, one per node
 *           below the root) and rcols (host, per level) as there.
 *   picks, counts
 *           device, the layout of hodlr_bdlr_select for max_skel (at most
 *           192 / 128): ascending distinct positions, counts <= max_skel
 *           and <= the side's length.
 *   samples device int, 32 per node: 16 rows then 16 columns (out).
 *   err     device double, one per node (out).
 * Synchronizes the stream.  Errors: EINVAL, ENOMEM, EHIP. */
int hodlr_sampled_error(const double* K, int n, int ldk, int leaf, int precision, const void* Upanel,
                        const void* Vpanel, const int* ranks, const int* rcols, const int* picks,
                        const int* counts, int max_skel, unsigned long long seed, int attempt, int* samples,
                        double* err, hipStream_t stream);

/* Introspection (host arrays): number of levels L, ranks of the nodes below
 * the root in level order (capacity 2^(L+1)-2 ints), per-level column widths
 * (capacity L ints).  Any pointer may be NULL. */
int hodlr_stats(hodlr_t h, int* nlevels, int* ranks, int* rcols);

/* Copy out the low-rank factors as float64 in the layout of
 * hodlr_build_from_factors (device, n x R, ld n).  Valid before
 * hodlr_factor (afterwards the U panel holds the factorization). */
int hodlr_get_factors(hodlr_t h, double* Upanel, double* Vpanel, hipStream_t stream);

/* HODLR_LEARNED handles: per node below the root in level order, the
 * budget (picks per side, the larger of rows and columns) that passed the
 * check; for a block that failed at its last budget k, 0 if the ACA
 * fallback was kept, -k if its own skeleton was (the smaller estimate).
 * Adaptive BDLR handles (bdlr_max_depth > 0): the depth each block ended at.
 * -1 for handles built otherwise.  kused: host, 2^(L+1)-2 ints. */
int hodlr_skel_info(hodlr_t h, int* kused);

/* Learned skeleton proposer (not in the paper; it proposes the skeleton rows
 * and columns that BDLR picks by boundary distance, Sec. 5.3).
 *
 * Samples: the off-diagonal blocks of the tree for (n, leaf) in level order
 * (node 1, 2, ...); block of node c: the |c| row vertices, then the |sibling|
 * column vertices; 2 n L samples in all.  Features, 8 float32 per sample
 * (row-major), for a vertex v of side S (other side O) of a block:
 *   d / (dmax + 1), 1 / (1 + d)   d = breadth-first distance inside S from
 *                                 the vertices of S with an edge into O (a
 *                                 vertex never reached: dmax + 1), dmax the
 *                                 largest distance reached on S
 *   deg(v) / max deg on S         graph degree
 *   x, y, z scaled to [0, 1] over the bounding box of S (0 on a flat axis)
 *   |K_vv| / max on S
 *   min(1, distance from v to the bounding box of O / diagonal of S's box)
 * g_rowptr/g_col/coords/K as for hodlr_build; feats: device, 2 n L x 8,
 * 16-byte aligned (each sample is written as two 16-byte stores).
 * Asynchronous.  Errors: EINVAL (2 <= n <= 16384, n > leaf, feats not
 * 16-byte aligned), ENOMEM, EHIP. */
int hodlr_skel_features(const int* g_rowptr, const int* g_col, const float* coords, const double* K, int n,
                        int ldk, int leaf, float* feats, hipStream_t stream);

/* Training labels: 1.0 where the sample is a pivot row (row side) or pivot
 * column (column side) of the block's compression at tol in the given
 * precision, else 0.0.  source 0: the crosses of ACA (as hodlr_build with
 * HODLR_ACA); source 1: the pivots of the full-pivot LU of the BDLR skeleton
 * at the given depth (as HODLR_BDLR; needs the graph).
 * labels: device, 2 n L float32.  Synchronizes.  Errors: as hodlr_build. */
int hodlr_skel_labels(const double* K, int n, int ldk, const int* g_rowptr, const int* g_col, int leaf,
                      double tol, int precision, int source, int depth, float* labels, hipStream_t stream);

/* Scorer: per sample z = w3 . relu(W2 relu(W1 x + b1) + b2) + b3.
 * params: device float32, 4801 values: W1 (64 x 8 row-major), b1 (64),
 * W2 (64 x 64 row-major), b2 (64), w3 (64), b3 (1).  bf16 != 0 rounds the
 * weights to bfloat16 (nearest, ties to even) before use; accumulation is
 * float32.  feats: device N x 8; logits: device N.  Asynchronous. */
int hodlr_mlp_forward(const float* feats, int N, const float* params, int bf16, float* logits,
                      hipStream_t stream);

/* Gradient of the mean weighted logistic loss
 *   L = mean_i [ p y_i softplus(-z_i) + (1 - y_i) softplus(z_i) ]
 * (p = pos_weight, y = labels in {0, 1}) with respect to params (same layout),
 * into grad (device, 4801); loss (device, 1 value) may be NULL.  Partial sums
 * are combined in a fixed order.  Synchronizes. */
int hodlr_mlp_grad(const float* feats, const float* labels, int N, const float* params, int bf16,
                   float pos_weight, float* grad, float* loss, hipStream_t stream);

/* One training step: the gradient above with bfloat16 weights, then Adam
 * (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected at step >= 1) on the
 * float32 params with moments m, v (device, 4801 each).  Synchronizes. */
int hodlr_mlp_adam_step(const float* feats, const float* labels, int N, float* params, float* m, float* v,
                        int step, float lr, float pos_weight, float* loss, hipStream_t stream);

/* Frees the handle; its device blocks go back to the library's allocator
 * cache for reuse.  Work that the library's calls left queued on the
 * handle's buffers (hodlr_solve, hodlr_factor_async, the end of a build, a
 * solver's error return) is tracked by events: if one of them has not
 * completed, the device is synchronized first; otherwise nothing waits. */
int hodlr_destroy(hodlr_t h);

/* Returns every cached device block to the HIP runtime (synchronizes the
 * device).  The library keeps freed device memory for reuse otherwise. */
int hodlr_release_memory(void);

/* Launch variants chosen by the library's autotuner: the split width of the
 * float64 matvec is picked per (n, right-hand-side block, type of z) by timing
 * each width on the first product of that shape (HODLR_TUNE=0 in the
 * environment keeps the default, choice 1).  Choice c sums 64 << c columns of
 * K per partial (64, 128, 256, or 512 as four chunks of 128 per workgroup,
 * the last for up to 32 right-hand sides).  Writes one "key=choice" line per tuned
 * shape into buf (NUL-terminated, at most len bytes).  Errors: EINVAL if buf
 * is NULL or too short. */
int hodlr_tune_report(char* buf, int len);

/* Kernel timing for benchmarks.  hodlr_prof_enable(1) clears earlier records
 * and makes the library record a HIP event pair around each launch of its
 * main kernels, on the launch stream; hodlr_prof_enable(0) stops recording.
 * hodlr_prof_query(name) synchronizes those events and returns how many
 * launches of kernel `name` were recorded and their summed duration in ms.
 * Names: "aca", "leaf_inverse", "leaf_apply", "panel_tn", "schur_form", "apply_leaf", "apply_level",
 * "schur_apply", "correct", "matvec", "orth".  Host-side pointers. */
int hodlr_prof_enable(int on);
int hodlr_prof_query(const char* name, int* launches, double* total_ms);

/* Thread-local message of the last failing call on this thread. */
const char* hodlr_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* HODLR_H_ */
