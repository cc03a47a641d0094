/*
 * ffpluq -- exact rank-profile-revealing PLUQ over Z/pZ on AMD Instinct MI355X (gfx950).
 *
 * C ABI of the shared library libffpluq.so.  Paper: J-G. Dumas, T. Gautier,
 * C. Pernet, Z. Sultan, "Parallel computation of echelon forms"
 * (arXiv:1402.3501).  Section 2.1 defines the four routines this library
 * exports (gemm, trsm, laswp, getrf/PLUQ); Section 3.1 the delayed modular
 * reduction; Section 4.1 the pivoting that reveals the row and column rank
 * profiles and the four-quadrant tile recursion.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Matrices are row-major int32 with leading dimension ld >= number of
 *    columns (ld >= 1).  Entries are canonical residues in [0, p).  Results
 *    are canonical residues in [0, p).
 *  - Every matrix / vector pointer is a DEVICE pointer owned by the caller;
 *    the library never frees or retains caller memory.  Workspace `ws` is a
 *    caller-owned device buffer of at least the bytes the matching
 *    *_workspace() query returns (it may be NULL when the query returns 0).
 *  - `stream` is a hipStream_t (NULL = the null stream).  Calls are
 *    asynchronous with respect to the host unless stated otherwise.
 *  - p must be prime.  Path limits: FP64 needs p <= FFP_P_MAX_FP64; INT8
 *    needs p <= FFP_P_MAX_INT8.  Rank deficiency is not an error.
 *  - Indices are 0-based int32.
 *  - Return value: FFP_OK (0), -i when the i-th argument is invalid
 *    (LAPACK convention, 1-based), or one of the FFP_E_* codes.  On error
 *    no device memory has been modified unless the code is FFP_E_HIP.
 *  - The library is thread-compatible: concurrent calls on different
 *    streams are safe; calls sharing one workspace must not overlap.
 */
#ifndef FFPLUQ_H
#define FFPLUQ_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef void *ffp_stream_t; /* hipStream_t */

#define FFP_OK 0
#define FFP_E_NOTPRIME (-101)    /* p is not prime */
#define FFP_E_P_RANGE (-102)     /* p too large for the requested path */
#define FFP_E_WORKSPACE (-103)   /* workspace missing or too small */
#define FFP_E_HIP (-104)         /* a HIP runtime call failed */
#define FFP_E_RANGE (-105)       /* an input entry lies outside [0, p) (ffp_check_range only) */
#define FFP_E_UNSUPPORTED (-106) /* valid request the library does not implement */
#define FFP_E_NODEVICE (-107)    /* no gfx950 device / kernels failed to load */
#define FFP_E_INTERNAL (-108)    /* internal consistency check failed; A is restored */
#define FFP_E_SCRATCH (-109)     /* request exceeds the fixed scratch of ffp_fgemm_noalloc */

/* Largest p of each arithmetic path (see ffp_fgemm). */
#define FFP_P_MAX_FP64 94906249u /* largest prime with (p-1)^2 + p < 2^53 */
#define FFP_P_MAX_INT8 16711421u /* largest prime whose centred residues fit 3 signed 8-bit limbs */

typedef enum {
    FFP_PATH_AUTO = 0, /* fastest exact path for (p, shape) */
    FFP_PATH_FP64 = 1, /* residues embedded in FP64, FP64 matrix cores */
    FFP_PATH_INT8 = 2  /* centred residues split in signed 8-bit limbs, INT8 matrix cores */
} ffp_path;

/* Human-readable name of an error code (static storage). */
const char *ffp_error_string(int code);
/* Library version string, e.g. "ffpluq 0.1 gfx950". */
const char *ffp_version(void);
/* 1 if p is prime (deterministic Miller-Rabin for 32-bit p), else 0. */
int ffp_is_prime(uint32_t p);
/* Number of limbs the INT8 path uses for p (0 if p exceeds FFP_P_MAX_INT8). */
int ffp_int8_limbs(uint32_t p);
/* Path FFP_PATH_AUTO resolves to for a product of the given size. */
int ffp_auto_path(uint32_t p, int64_t m, int64_t n, int64_t k);

/* --------------------------------------------------------------------------
 * fgemm -- Section 2.1 (gemm): C <- alpha * op(A) * op(B) + beta * C mod p,
 * with the delayed modular reduction of Section 3.1: products are summed
 * exactly (FP64: |partial sum| < 2^53; INT8 limbs: |partial sum| < 2^31) and
 * reduced once at the end, or once per chunk of the inner dimension when k
 * exceeds the exactness bound.
 *   transA/transB: 0 = as stored, 1 = transposed.  op(A) is m x k (A stored
 *   m x k, or k x m when transposed), op(B) is k x n, C is m x n.
 *   alpha, beta: residues in [0, p).  beta = 0 means C is not read.
 *   path: ffp_path.  FP64 requires p <= FFP_P_MAX_FP64, INT8 p <= FFP_P_MAX_INT8.
 * The INT8 path splits A and B into limbs in the workspace; when the grid
 * of 128 x 128 output blocks is too small to fill the device it also splits
 * the inner dimension over up to 4 workgroups per block, with their partial
 * results (at most 4 m n int32, capped at 32 MiB) in the workspace and one
 * more launch to combine them.  The workspace query includes that room.
 * A product with m + n beyond about 4.19e6 (65535 grid rows of 64 limb
 * rows) runs on the FP64 path whatever the path argument (the same bits),
 * or returns FFP_E_UNSUPPORTED when p is beyond that path.
 * -------------------------------------------------------------------------- */
size_t ffp_fgemm_workspace(int transA, int transB, int64_t m, int64_t n, int64_t k, uint32_t p,
                           int path);
int ffp_fgemm(int transA, int transB, int64_t m, int64_t n, int64_t k, uint32_t p, uint32_t alpha,
              const int32_t *A, int64_t lda, const int32_t *B, int64_t ldb, uint32_t beta, int32_t *C,
              int64_t ldc, int path, void *ws, size_t ws_bytes, ffp_stream_t stream);

/* --------------------------------------------------------------------------
 * fgemm_wino -- Section 2.1: the sequential fgemm runs recursive steps of
 * Winograd's variant of Strassen's algorithm over the plain product
 * (Sections 2.3 and 3.2 discuss its gain and crossover).  Same arguments and
 * the same result as ffp_fgemm, plus:
 *   levels: number of Winograd steps (0 = the plain product, at most
 *     FFP_WINO_MAX_LEVELS), or FFP_WINO_AUTO for the levels this library
 *     measured to pay on MI355X for the size and path.
 * Each step splits op(A), op(B), C into 2 x 2 blocks (odd dimensions peeled
 * off and finished by thin products) and forms C from 7 block products and
 * 15 block additions; every addition is reduced mod p as it is formed, so
 * the block products keep the exactness bound of the plain product.
 * Temporaries (4 (m k + k n + m n) / 4 int32 per step) come from the
 * workspace, ffp_fgemm_wino_workspace bytes.  An invalid `levels` is
 * argument 16.
 * -------------------------------------------------------------------------- */
#define FFP_WINO_AUTO (-1)
#define FFP_WINO_MAX_LEVELS 6
size_t ffp_fgemm_wino_workspace(int transA, int transB, int64_t m, int64_t n, int64_t k, uint32_t p, int path,
                                int levels);
int ffp_fgemm_wino(int transA, int transB, int64_t m, int64_t n, int64_t k, uint32_t p, uint32_t alpha,
                   const int32_t *A, int64_t lda, const int32_t *B, int64_t ldb, uint32_t beta, int32_t *C,
                   int64_t ldc, int path, int levels, void *ws, size_t ws_bytes, ffp_stream_t stream);

/* --------------------------------------------------------------------------
 * fgemm_noalloc -- for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, hosts that forbid
 * allocation): the same product as ffp_fgemm, same arguments and the same
 * bits, minus the workspace.  The INT8 path takes its limb planes (and
 * split-K partial results) from a fixed device array of
 * FFP_NOALLOC_SCRATCH_BYTES that the library holds on every GPU it runs on
 * until the process ends; the call itself never allocates or frees.
 *   An INT8 product whose ffp_fgemm_workspace exceeds that size returns
 *   FFP_E_SCRATCH (nothing is launched); with FFP_PATH_AUTO such a product
 *   runs on the FP64 path instead (no workspace, same result).
 * All calls on one GPU share the array, so calls that overlap on one GPU
 * (different streams or host threads) race: the caller serialises them.
 * -------------------------------------------------------------------------- */
#define FFP_NOALLOC_SCRATCH_BYTES (64u << 20)
size_t ffp_noalloc_scratch_bytes(void);
int ffp_fgemm_noalloc(int transA, int transB, int64_t m, int64_t n, int64_t k, uint32_t p, uint32_t alpha,
                      const int32_t *A, int64_t lda, const int32_t *B, int64_t ldb, uint32_t beta, int32_t *C,
                      int64_t ldc, int path, ffp_stream_t stream);

/* --------------------------------------------------------------------------
 * ftrsm -- Section 2.1 (trsm): triangular solve mod p.
 *   side 0 (left):  B <- alpha * op(T)^-1 * B,  T is m x m;
 *   side 1 (right): B <- alpha * B * op(T)^-1,  T is n x n;
 *   uplo 0 lower / 1 upper (the triangle of T that is read),
 *   trans 0: op(T) = T, 1: op(T) = T^T,
 *   diag 0 non-unit / 1 unit (the diagonal of T is then not read).
 * Block recursion onto fgemm (Section 2.1: trsm reduces most work to gemm).
 * A zero diagonal entry of a non-unit T gives an unspecified result.
 * -------------------------------------------------------------------------- */
size_t ffp_ftrsm_workspace(int side, int uplo, int trans, int diag, int64_t m, int64_t n,
                           uint32_t p, int path);
int ffp_ftrsm(int side, int uplo, int trans, int diag, int64_t m, int64_t n, uint32_t p,
              uint32_t alpha, const int32_t *T, int64_t ldt, int32_t *B, int64_t ldb, int path,
              void *ws, size_t ws_bytes, ffp_stream_t stream);

/* --------------------------------------------------------------------------
 * flaswp -- Section 2.1 (laswp): permute the rows (dim 0) or columns (dim 1)
 * of the m x n matrix A in place, given as an index vector rather than a
 * sequence of swaps (ffp_swaps_to_perm converts):
 *   dim 0, inverse 0: new row i = old row perm[i]      (perm has m entries)
 *   dim 0, inverse 1: new row perm[i] = old row i
 *   dim 1: the same for columns (perm has n entries).
 * perm must be a permutation (not checked on the device).  Out of place
 * through the workspace, then copied back.
 * -------------------------------------------------------------------------- */
size_t ffp_flaswp_workspace(int dim, int64_t m, int64_t n);
int ffp_flaswp(int dim, int64_t m, int64_t n, int32_t *A, int64_t lda, const int32_t *perm,
               int inverse, void *ws, size_t ws_bytes, ffp_stream_t stream);

/* --------------------------------------------------------------------------
 * pluq -- Section 2.1 (getrf): A = P L U Q with L and U in place of A,
 * revealing the rank and the row and column rank profiles (Section 4.1),
 * computed by the four-quadrant tile recursion (Section 4.1, tiled
 * recursive elimination) with dynamic pivot blocks.
 * Output (canonical, bit-identical to the reference convention):
 *   P[i] = original row at position i, Q[j] = original column at position j,
 *   so A[P[i]][Q[j]] = sum_t L[i][t] U[t][j]; the r pivots come first, in the
 *   order of the quadrant recursion (top-left, top-right, bottom-left,
 *   bottom-right, halves rounded down), then the non-pivot rows / columns in
 *   increasing index.  A holds L strictly below the diagonal of its first r
 *   columns (unit diagonal implied), U on and above the diagonal of its first
 *   r rows, and zeros in [r:, r:].
 *   rank_dev: device int64 receiving r (may be NULL);
 *   rank_host: host int64 receiving r (may be NULL; the call then returns
 *     after the factorisation has completed on `stream`);
 *   rrp / crp: device int32 arrays of min(m, n) entries receiving the sorted
 *     row / column rank profile in their first r entries (may be NULL).
 * The host drives the recursion and reads each sub-block's rank back, so
 * the call synchronises with `stream` internally and cannot be captured in
 * a graph; ffp_lu_nopiv (generic rank profile) and ffp_pluq_batched are the
 * asynchronous, capturable alternatives.  Within a node of the
 * general recursion the solve E = C1 U1^-1 and its product run on a second
 * stream that the library owns (one per device, default priority, shared by
 * all calls on the device), ordered against `stream` with events and joined
 * back into it before the node's next step; the generic attempt below runs
 * on `stream` alone.
 * A first attempt assumes a generic rank profile (all leading minors
 * nonzero: plain block LU, no rank read-backs) on a copy kept in the
 * workspace; a zero pivot restores A and runs the general recursion.  The
 * attempt reads its flag back once at the end and, on large inputs, at up to
 * two checkpoints on the way (after the leading blocks of order about 1024
 * and 4096), stopping early when a zero pivot was met.  The index of the
 * first zero pivot (every leading minor below it is nonzero) lets the
 * general recursion factor leading tiles within that order as plain LU, and
 * sub-blocks found zero (one reduction and read-back) skip their recursion.
 * The output is the same either way.
 * -------------------------------------------------------------------------- */
size_t ffp_pluq_workspace(int64_t m, int64_t n, uint32_t p, int path);
int ffp_pluq(int64_t m, int64_t n, uint32_t p, int32_t *A, int64_t lda, int32_t *P, int32_t *Q,
             int64_t *rank_dev, int64_t *rank_host, int32_t *rrp, int32_t *crp, int path, void *ws,
             size_t ws_bytes, ffp_stream_t stream);

/* --------------------------------------------------------------------------
 * lu_nopiv -- the PLUQ of Section 2.1 (getrf) for an input of generic rank
 * profile (every leading principal minor nonzero, the assumption Section 3
 * makes for its reduction counts): then R_A is the leading diagonal, P and Q
 * are the identity and A = L U without pivoting, so no rank ever has to be
 * read back.  Fully asynchronous on `stream` (no host synchronisation, no
 * allocation: graph-capturable), unlike ffp_pluq.
 *   info_dev: device int32 receiving 0 when every pivot was nonzero (A then
 *     holds L\U exactly as ffp_pluq returns it, rank min(m, n), P = Q = id),
 *     otherwise 1 + the diagonal index of the first zero pivot (A is then
 *     left in an unspecified state: keep a copy to fall back on ffp_pluq).
 * Workspace: ffp_lu_nopiv_workspace bytes.
 * -------------------------------------------------------------------------- */
size_t ffp_lu_nopiv_workspace(int64_t m, int64_t n, uint32_t p, int path);
int ffp_lu_nopiv(int64_t m, int64_t n, uint32_t p, int32_t *A, int64_t lda, int32_t *info_dev, int path,
                 void *ws, size_t ws_bytes, ffp_stream_t stream);

/* --------------------------------------------------------------------------
 * pluq_slab -- the slab-recursive PLUQ of Section 4.1 ("Pivoting
 * strategies"): the row-major pivot search (rows in order, a row with no
 * nonzero left skipped, otherwise its leftmost remaining nonzero is the next
 * pivot) as a recursion on halves of the rows.  Same arguments, outputs and
 * layout as ffp_pluq, except the pivot order: pivots in increasing row
 * order, so P[0:r] is the row rank profile itself; the pivot pairs are the
 * same rank profile matrix, rrp / crp the same profiles, and non-pivot rows
 * and columns ascend.  At most FFP_SLAB_MAX_COLS columns (argument 2 else).
 * Synchronises `stream` once per slab of 32 rows (rank read-back).
 * Workspace: ffp_pluq_slab_workspace bytes.
 * -------------------------------------------------------------------------- */
#define FFP_SLAB_MAX_COLS 65536
size_t ffp_pluq_slab_workspace(int64_t m, int64_t n, uint32_t p, int path);
int ffp_pluq_slab(int64_t m, int64_t n, uint32_t p, int32_t *A, int64_t lda, int32_t *P, int32_t *Q, int64_t *rank_dev,
                  int64_t *rank_host, int32_t *rrp, int32_t *crp, int path, void *ws, size_t ws_bytes,
                  ffp_stream_t stream);

/* --------------------------------------------------------------------------
 * lu_tiled -- the tile-iterative block LU of Section 3.1 (Table 1) in one of
 * its three orders, for an input of generic rank profile (the assumption of
 * Section 3): variant FFP_LU_RIGHT (right-looking), FFP_LU_CROUT or
 * FFP_LU_LEFT (left-looking), with k x k diagonal tiles (k >= 1; the last one
 * may be smaller).  The result, when every pivot is nonzero, is the unique LU
 * without pivoting, bit-identical to what ffp_pluq returns for such an input
 * (P = Q = identity).  Asynchronous (no host synchronisation):
 *   info_dev: device int32 receiving 0, or 1 + the diagonal index of the
 *     first zero pivot (A is then left in an unspecified state).
 * Workspace: ffp_lu_tiled_workspace bytes.
 *
 * reduction_count -- host only, no device: the number of modular reductions
 * the model of Section 3.1 charges an n x n factorisation (a product m x k
 * by k x n: m n; a unit triangular solve m x m with n right-hand sides:
 * (m - 1) n; a non-unit one: (2 m - 1) n; a k x k base case: 3/2 k^2 -
 * 7/2 k + 3, the unblocked Crout count).  For FFP_LU_RIGHT / CROUT / LEFT it
 * runs the loops of ffp_lu_tiled with tile k without launching anything;
 * FFP_LU_TILE_RECURSIVE and FFP_LU_SLAB_RECURSIVE are the halving recursions
 * of the four-quadrant and the row-slab algorithms (k ignored).
 * -------------------------------------------------------------------------- */
#define FFP_LU_RIGHT 0
#define FFP_LU_CROUT 1
#define FFP_LU_LEFT 2
#define FFP_LU_TILE_RECURSIVE 3
#define FFP_LU_SLAB_RECURSIVE 4
size_t ffp_lu_tiled_workspace(int variant, int64_t m, int64_t n, int64_t k, uint32_t p, int path);
int ffp_lu_tiled(int variant, int64_t m, int64_t n, uint32_t p, int32_t *A, int64_t lda, int64_t k, int32_t *info_dev,
                 int path, void *ws, size_t ws_bytes, ffp_stream_t stream);
int ffp_reduction_count(int algorithm, int64_t n, int64_t k, double *count);

/* --------------------------------------------------------------------------
 * Consumers of the rank profile (Section 1, "Pivoting strategies and rank
 * deficiencies": the pivoting that reveals the rank profile reveals the
 * echelon form).  They take the output of ffp_pluq as it stands: LU (m x n,
 * leading dimension ld, L\U in place), P (m), Q (n) and the rank r (host
 * value), all device memory, none modified.  Asynchronous on `stream`; the
 * workspace queries give the bytes each call takes.
 *
 * echelon -- form 0: the reduced row echelon form of A, E (r x n, leading
 *   dimension lde >= n): E[:, crp] = I, row t has its leading 1 in column
 *   crp[t] (the column rank profile, ascending), and the rows span the row
 *   space of A.  form 1: the reduced column echelon form, E (m x r, lde >=
 *   r), the transpose of the row form of A^T: E[rrp, :] = I.
 * nullspace -- side 0: N (n x (n - r), ldn >= n - r) with A N = 0 and N = I
 *   on the non-pivot columns (ascending); side 1: N ((m - r) x m, ldn >= m)
 *   with N A = 0 and N = I on the non-pivot rows.  Both bases are unique.
 * solve -- A X = B for B (m x nrhs, ldb >= nrhs): consistent[j] (device
 *   int32[nrhs]) = 1 when column j of B lies in the column space of A, and
 *   then X[:, j] (X is n x nrhs, ldx >= nrhs) is the solution that is zero
 *   on the non-pivot columns; otherwise consistent[j] = 0 and X[:, j] = 0.
 * Arguments are numbered from form / side = 1 (ffp_solve from m = 1).
 * -------------------------------------------------------------------------- */
size_t ffp_echelon_workspace(int form, int64_t m, int64_t n, int64_t r, uint32_t p, int path);
int ffp_echelon(int form, int64_t m, int64_t n, uint32_t p, const int32_t *LU, int64_t ld, const int32_t *P,
                const int32_t *Q, int64_t r, int32_t *E, int64_t lde, int path, void *ws, size_t ws_bytes,
                ffp_stream_t stream);
size_t ffp_nullspace_workspace(int side, int64_t m, int64_t n, int64_t r, uint32_t p, int path);
int ffp_nullspace(int side, int64_t m, int64_t n, uint32_t p, const int32_t *LU, int64_t ld, const int32_t *P,
                  const int32_t *Q, int64_t r, int32_t *N, int64_t ldn, int path, void *ws, size_t ws_bytes,
                  ffp_stream_t stream);
size_t ffp_solve_workspace(int64_t m, int64_t n, int64_t r, int64_t nrhs, uint32_t p, int path);
int ffp_solve(int64_t m, int64_t n, uint32_t p, const int32_t *LU, int64_t ld, const int32_t *P, const int32_t *Q,
              int64_t r, int64_t nrhs, const int32_t *B, int64_t ldb, int32_t *X, int64_t ldx, int32_t *consistent,
              int path, void *ws, size_t ws_bytes, ffp_stream_t stream);

/* --------------------------------------------------------------------------
 * check_range -- the validating call: FFP_E_RANGE if some entry of the m x n
 * matrix A (device, leading dimension lda) lies outside [0, p), else FFP_OK.
 * The other entry points take canonical residues without checking them
 * (an entry >= p gives unspecified bits); callers that cannot vouch for
 * their input run this first.  Synchronises `stream` (one read-back).
 * -------------------------------------------------------------------------- */
int ffp_check_range(int64_t m, int64_t n, uint32_t p, const int32_t *A, int64_t lda, ffp_stream_t stream);

/* --------------------------------------------------------------------------
 * pluq_batched -- the same factorisation for `batch` independent matrices of
 * uneven shapes (the heterogeneous pivot blocks of Section 4.1), in one
 * persistent kernel launch with no host synchronisation (graph-capturable).
 *   m_arr, n_arr: device int32[batch] shapes (each 0 <= m, n <= FFP_BATCH_MAX_DIM);
 *   A_off: device int64[batch] element offsets of each row-major matrix
 *     (leading dimension n_i) in A_packed; P_off / Q_off: device int64[batch]
 *     offsets of each P (m_i entries) / Q (n_i entries) in P_packed / Q_packed;
 *   rank_arr: device int32[batch]; rrp_packed / crp_packed use P_off / Q_off
 *     and receive the sorted profiles in their first r_i entries (may be NULL).
 *   max_m, max_n: host upper bounds of the shapes (used to size the launch
 *     and the workspace).  A matrix whose m_i or n_i lies outside [0, max_m]
 *     or [0, max_n] is not touched and its rank_arr entry reads -1.
 * Every output equals what ffp_pluq returns for that matrix alone.
 * -------------------------------------------------------------------------- */
#define FFP_BATCH_MAX_DIM 1024
size_t ffp_pluq_batched_workspace(int32_t batch, int32_t max_m, int32_t max_n, uint32_t p, int path);
int ffp_pluq_batched(int32_t batch, const int32_t *m_arr, const int32_t *n_arr, int32_t max_m,
                     int32_t max_n, uint32_t p, int32_t *A_packed, const int64_t *A_off,
                     int32_t *P_packed, const int64_t *P_off, int32_t *Q_packed,
                     const int64_t *Q_off, int32_t *rank_arr, int32_t *rrp_packed,
                     int32_t *crp_packed, int path, void *ws, size_t ws_bytes,
                     ffp_stream_t stream);

/* --------------------------------------------------------------------------
 * pluq_batched_tune -- autotuning of the batched launch: the same call as
 * ffp_pluq_batched, run once with each of the library's FFP_BATCH_SHAPES
 * launch shapes (workgroup size x workgroups per compute unit), each timed
 * with HIP events on `stream`, the batch restored from a copy in the
 * workspace before each run.  The fastest shape is kept for later
 * ffp_pluq_batched calls with the same (device, batch, max_m, max_n); on
 * return the batch is factored exactly as by ffp_pluq_batched.  Synchronises
 * `stream` (call it before capturing the batched call in a graph).
 *   a_elems: number of entries of A_packed (all matrices);
 *   shape_out: host int receiving the chosen shape index (may be NULL);
 *   ms_out: host float[FFP_BATCH_SHAPES] receiving each shape's time (may be NULL).
 * -------------------------------------------------------------------------- */
#define FFP_BATCH_SHAPES 4
/* Record launch shape `shape` (0 .. FFP_BATCH_SHAPES - 1) for batches with
 * this (batch, max_m, max_n) on the current device, as the tuner does:
 * for callers that know the best shape already (e.g. from an earlier run). */
int ffp_pluq_batched_set_shape(int32_t batch, int32_t max_m, int32_t max_n, int shape);
size_t ffp_pluq_batched_tune_workspace(int32_t batch, int32_t max_m, int32_t max_n, int64_t a_elems);
int ffp_pluq_batched_tune(int32_t batch, const int32_t *m_arr, const int32_t *n_arr, int32_t max_m,
                          int32_t max_n, uint32_t p, int32_t *A_packed, int64_t a_elems, const int64_t *A_off,
                          int32_t *P_packed, const int64_t *P_off, int32_t *Q_packed, const int64_t *Q_off,
                          int32_t *rank_arr, int32_t *rrp_packed, int32_t *crp_packed, int path, int *shape_out,
                          float *ms_out, void *ws, size_t ws_bytes, ffp_stream_t stream);

/* --------------------------------------------------------------------------
 * Host helpers (host pointers): Section 2.1 describes laswp as applying a
 * sequence of swaps, while this library's permutations are index vectors
 * (order-preserving rotations, see ffp_flaswp).  These convert between the
 * two: ipiv is the LAPACK laswp form (for i = 0..len-1, swap entries i and
 * ipiv[i]), perm[i] = original index placed at position i.  Return -2 when
 * the input is not a permutation / not a valid swap sequence.
 * -------------------------------------------------------------------------- */
int ffp_perm_to_swaps(int64_t len, const int32_t *perm, int32_t *ipiv);
int ffp_swaps_to_perm(int64_t len, const int32_t *ipiv, int32_t *perm);

/* --------------------------------------------------------------------------
 * Kernel timing (for benchmarks): when enabled, the library brackets each
 * launch of its kernels with HIP events on the launching stream and
 * accumulates, per kernel family ("kind", 1 .. FFP_PROFILE_KINDS - 1), the
 * number of launches, the summed event time, the summed algorithmic work in
 * field operations (2 m n k per product, d^2 nv per triangular solve of a
 * d x d triangle with nv vectors, 2 m n k - (m + n) k^2 + 2 k^3 / 3 per
 * elimination of rank k plus the products fused into a leaf) and the summed
 * algorithmic bytes (operands read once, results written once).  Kind 1 is
 * the FP64 product kernels and kind 2 the INT8 product kernel (FFP_PATH_FP64
 * and FFP_PATH_INT8); ffp_profile_kind_name names every kind after its
 * kernels.  Reading synchronises the recorded events.
 * -------------------------------------------------------------------------- */
#define FFP_PROFILE_KINDS 11
int ffp_profile_enable(int on);
int ffp_profile_reset(void);
int ffp_profile_read(int kind, int64_t *launches, double *milliseconds, double *field_ops);
int ffp_profile_read_bytes(int kind, double *bytes);
/* name of the kernel family `kind` (static storage), NULL outside the range */
const char *ffp_profile_kind_name(int kind);

#ifdef __cplusplus
}
#endif
#endif /* FFPLUQ_H */
