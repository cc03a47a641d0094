// Internal declarations of the gfx950 library (not part of the C ABI).
//
// Field elements travel as int32 canonical residues in [0, p).  Kernels embed
// them as *centred* residues c in [-(p-1)/2, (p-1)/2] (FP64 path) or as
// signed 8-bit limbs of c (INT8 path), accumulate exactly and reduce once
// (the delayed reduction of Section 3.1 of the paper).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include "../../include/ffpluq.h"

namespace ffp {

// ------------------------------------------------------------------ errors
#define FFP_HIP_CHECK(expr)                                  \
    do {                                                     \
        hipError_t _e = (expr);                              \
        if (_e != hipSuccess) return ::ffp::hip_fail(_e, #expr, __FILE__, __LINE__); \
    } while (0)

#define FFP_CHECK(expr)          \
    do {                         \
        int _r = (expr);         \
        if (_r != FFP_OK) return _r; \
    } while (0)

int hip_fail(hipError_t e, const char *what, const char *file, int line);

// ------------------------------------------------------------------ field
struct Field {
    uint32_t p;
    double pd;      // p as double
    double pinv;    // 1/p rounded
    int64_t half;   // (p-1)/2: residues above it are centred to r - p
    int64_t kexact; // largest k such that 2p + k*half^2 < 2^53 (FP64 exact accumulation)
    int limbs;      // INT8 limbs (0 if p exceeds the INT8 path)
    explicit Field(uint32_t p_);
};

bool is_prime_u32(uint32_t p);
int int8_limbs(uint32_t p);

// ------------------------------------------------------------------ workspace
// Bump allocator over the caller's workspace (256-byte aligned slices).
struct Arena {
    char *base = nullptr;
    size_t cap = 0, used = 0, peak = 0;
    bool counting = false;  // size query mode: hand out nullptr, only count
    void *take(size_t bytes);
    size_t mark() const { return used; }
    void release(size_t m) { used = m; }
};

// ------------------------------------------------------------------ profiling
// Kernel families timed by the optional launch events (ffp_profile_*): each
// launch site brackets its kernel with a ProfScope of its family, giving
// the launch's algorithmic work (field operations: 2 m n k for a product,
// d^2 nv for a triangular solve, 2 m n k - (m + n) k^2 + 2 k^3 / 3 for an
// elimination of rank k) and its algorithmic bytes.
enum ProfKind {
    PK_FGEMM_F64 = 1,   // FP64 matrix-core products (all shapes)
    PK_FGEMM_I8 = 2,    // INT8 matrix-core products (the product kernel alone)
    PK_I8_SPLIT = 3,    // limb split of the INT8 operands
    PK_I8_COMBINE = 4,  // split-K combining pass
    PK_LEAF_GEN = 5,    // generic-rank-profile leaves (with their fused solves / update)
    PK_LEAF = 6,        // leaves of the general recursion
    PK_TRSM = 7,        // triangular-solve base cases and block inverses
    PK_PERMUTE = 8,     // out-of-place and in-LDS permutations
    PK_BATCHED = 9,     // the persistent batched factorisation
    PK_WINOGRAD = 10,   // pre- and post-additions of the Strassen-Winograd products
};
constexpr int kProfKinds = 11;
struct ProfScope {
    int kind;
    double ops, bytes;
    hipStream_t s;
    void *ev0 = nullptr, *ev1 = nullptr;
    ProfScope(int kind_, double ops_, hipStream_t s_, double bytes_ = 0.0);
    ~ProfScope();
};
const char *profile_kind_name(int kind);

// ------------------------------------------------------------------ kernels (launchers)
// All return FFP_OK or an error code; all are asynchronous on `s`.

// C <- alpha op(A) op(B) + beta C  (FP64 matrix cores)
int fgemm_f64(const Field &F, int ta, int tb, int64_t m, int64_t n, int64_t k, uint32_t alpha,
              const int32_t *A, int64_t lda, const int32_t *B, int64_t ldb, uint32_t beta,
              int32_t *C, int64_t ldc, hipStream_t s);

// two products C_i <- alpha A_i B_i + beta C_i (no transposes, the same k) in
// one launch when both are small-product shapes, else one after the other
int fgemm_f64_pair(const Field &F, int64_t m0, int64_t n0, const int32_t *A0, int64_t lda0, const int32_t *B0,
                   int64_t ldb0, int32_t *C0, int64_t ldc0, int64_t m1, int64_t n1, const int32_t *A1, int64_t lda1,
                   const int32_t *B1, int64_t ldb1, int32_t *C1, int64_t ldc1, int64_t k, uint32_t alpha,
                   uint32_t beta, hipStream_t s);

// same result through signed 8-bit limbs on INT8 matrix cores (workspace from the arena)
size_t fgemm_i8_ws(const Field &F, int64_t m, int64_t n, int64_t k);
// optional workspace of the split-K partial results (see fgemm_i8.hip)
size_t fgemm_i8_split_ws(int64_t m, int64_t n);
int fgemm_i8(const Field &F, int ta, int tb, int64_t m, int64_t n, int64_t k, uint32_t alpha,
             const int32_t *A, int64_t lda, const int32_t *B, int64_t ldb, uint32_t beta,
             int32_t *C, int64_t ldc, Arena &ws, hipStream_t s);
// two independent products of the same k (no transposes) in one split and one product launch
int fgemm_i8_pair(const Field &F, int64_t k, uint32_t alpha, uint32_t beta, int64_t m0, int64_t n0,
                  const int32_t *A0, int64_t lda0, const int32_t *B0, int64_t ldb0, int32_t *C0, int64_t ldc0,
                  int64_t m1, int64_t n1, const int32_t *A1, int64_t lda1, const int32_t *B1, int64_t ldb1, int32_t *C1,
                  int64_t ldc1, Arena &ws, hipStream_t s);

// dispatch on path (FFP_PATH_FP64 / FFP_PATH_INT8, AUTO already resolved)
int fgemm_any(int path, const Field &F, int ta, int tb, int64_t m, int64_t n, int64_t k,
              uint32_t alpha, const int32_t *A, int64_t lda, const int32_t *B, int64_t ldb,
              uint32_t beta, int32_t *C, int64_t ldc, Arena &ws, hipStream_t s);
int resolve_path(int path, uint32_t p, int64_t m, int64_t n, int64_t k);
// argument checks of ffp_fgemm (negative argument index or FFP_E_*), and the
// path the product runs on
int fgemm_validate(int transA, int transB, int64_t m, int64_t n, int64_t k, uint32_t p, uint32_t alpha,
                   const int32_t *A, int64_t lda, const int32_t *B, int64_t ldb, uint32_t beta, const int32_t *C,
                   int64_t ldc, int path, int *eff);

// Strassen-Winograd levels over fgemm_any (winograd.hip); levels = 0 is the
// plain product.  Block products below kWinoMinDim* in some dimension are
// not split further by the automatic level choice.
constexpr int64_t kWinoMinDimF64 = 4096;
constexpr int64_t kWinoMinDimI8 = 4096;
size_t fgemm_wino_ws(int path, const Field &F, int levels, int64_t m, int64_t n, int64_t k);
int fgemm_wino(int path, const Field &F, int levels, int ta, int tb, int64_t m, int64_t n, int64_t k,
               uint32_t alpha, const int32_t *A, int64_t lda, const int32_t *B, int64_t ldb, uint32_t beta,
               int32_t *C, int64_t ldc, Arena &ws, hipStream_t s);
int wino_auto_levels(int path, const Field &F, int64_t m, int64_t n, int64_t k);

// consumers of a PLUQ (echelon.hip): reduced row (form 0, r x n) or column
// (form 1, m x r) echelon form, right (side 0) or left (side 1) nullspace,
// and A X = B with per-column consistency flags; workspace by counting mode
int echelon_run(int form, int path, const Field &F, int64_t m, int64_t n, const int32_t *LU, int64_t ld,
                const int32_t *P, const int32_t *Q, int64_t r, int32_t *E, int64_t lde, Arena &ws, hipStream_t s);
int nullspace_run(int side, int path, const Field &F, int64_t m, int64_t n, const int32_t *LU, int64_t ld,
                  const int32_t *P, const int32_t *Q, int64_t r, int32_t *N, int64_t ldn, Arena &ws, hipStream_t s);
int solve_run(int path, const Field &F, int64_t m, int64_t n, const int32_t *LU, int64_t ld, const int32_t *P,
              const int32_t *Q, int64_t r, int64_t nrhs, const int32_t *B, int64_t ldb, int32_t *X, int64_t ldx,
              int32_t *ok, Arena &ws, hipStream_t s);

// triangular solve (recursive onto fgemm_any); alpha applied first
int ftrsm_run(int path, const Field &F, int side, int uplo, int trans, int diag, int64_t m,
              int64_t n, uint32_t alpha, const int32_t *T, int64_t ldt, int32_t *B, int64_t ldb,
              Arena &ws, hipStream_t s);
// workspace bytes of ftrsm_run (block inverses + products of the given path)
size_t ftrsm_ws(int path, const Field &F, int side, int64_t m, int64_t n);
// solve with the inverses of the diagonal 64 x 64 blocks of op(T) = T already
// formed (W: ceil(d / 64) blocks of 64 x 64 centred doubles); alpha = 1
// the two panel solves D = L^-1 Bd (lower, unit, h x nvd) and E = Be U^-1
// (upper, nve x h) of a generic block LU node on one stream, each base-case
// pair in one launch; T is the factored h x h diagonal block, Li / Ui its
// 64-block inverses
int ftrsm_pair_gen(int path, const Field &F, int64_t h, const int32_t *T, int64_t ldt, int64_t nvd, int32_t *Bd,
                   int64_t nve, int32_t *Be, int64_t ldb, const double *Li, const double *Ui, Arena &ws,
                   hipStream_t s);
int ftrsm_with_inverses(int path, const Field &F, int side, bool lower, int64_t m, int64_t n,
                        const int32_t *T, int64_t ldt, int32_t *B, int64_t ldb, const double *W, Arena &ws,
                        hipStream_t s);

// B <- alpha * B mod p
int scale_mat(const Field &F, int64_t m, int64_t n, uint32_t alpha, int32_t *B, int64_t ldb,
              hipStream_t s);

// Permutation described either by an index array or by up to kMaxSeg
// contiguous segments: destination index d in segment i reads source index
// src[i] + (d - dst[i]).
constexpr int kMaxSeg = 8;
struct SegPerm {
    int nseg;
    int64_t dst[kMaxSeg], src[kMaxSeg], len[kMaxSeg];
};
struct PermSpec {
    const int32_t *idx = nullptr;  // if set: dst d reads src idx[d] + idx_base
    int64_t idx_base = 0;
    SegPerm seg{};                  // used when idx == nullptr and seg.nseg > 0
    bool identity() const { return idx == nullptr && seg.nseg == 0; }
};

// dst[i][j] = src[rp(i)][cp(j)] for an m x n block (out of place)
int permute_copy(int64_t m, int64_t n, const int32_t *src, int64_t lds, int32_t *dst,
                 int64_t ldd, const PermSpec &rp, const PermSpec &cp, hipStream_t s);
// in place through a workspace slice (copy out permuted, copy back)
int permute_inplace(int64_t m, int64_t n, int32_t *A, int64_t lda, const PermSpec &rp,
                    const PermSpec &cp, Arena &ws, hipStream_t s);
// 2-D copy on the stream
int copy2d(int64_t m, int64_t n, const int32_t *src, int64_t lds, int32_t *dst, int64_t ldd,
           hipStream_t s);

// PLUQ leaf for blocks of at most 64 x 64 (one wave; rank to rank_dev); with
// gflag non-null: plain LU leaf of the generic-rank-profile attempt (a zero
// pivot sets *gflag; P, Q and rank are not written; with Linv / Uinv
// non-null, the 64 x 64 inverses of its L and U blocks are stored there).
// Generic leaf only, when 64-term sums need no reduction: He / Hd first
// update the block, A <- A - He Hd (He: m x 64, Hd: 64 x n, leading
// dimension lda); Pd / Pe (a full 64 x 64 block with inverses) are replaced
// after it by L^-1 Pd (64 x pdn) and Pe U^-1 (pem x 64).  A zero pivot sets
// *gflag = 1 + its index on the whole diagonal (diag0: the block's offset).
// General leaf with gen_done non-null: the generic leaf ran first with that
// flag; if it stayed clear only P, Q and the rank are written.
int leaf64_launch(const Field &F, int64_t m, int64_t n, int32_t *A, int64_t lda, int32_t *P, int32_t *Q,
                  int64_t *rank_dev, int *gflag, double *Linv, double *Uinv, hipStream_t s,
                  const int32_t *He = nullptr, const int32_t *Hd = nullptr, int32_t *Pd = nullptr,
                  int64_t pdn = 0, int32_t *Pe = nullptr, int64_t pem = 0, int64_t diag0 = 0,
                  const int *gen_done = nullptr);

// PLUQ (host recursion); P, Q device outputs (local indices); returns rank via *r
int pluq_run(int path, const Field &F, int64_t m, int64_t n, int32_t *A, int64_t lda, int32_t *P,
             int32_t *Q, int64_t *r, Arena &ws, hipStream_t s);
size_t pluq_ws(int64_t m, int64_t n, const Field &F, int path);
// plain LU of a generic-rank-profile input, asynchronous; *info (device) = 0
// or 1 + the diagonal index of the first zero pivot
int lu_nopiv_run(int path, const Field &F, int64_t m, int64_t n, int32_t *A, int64_t lda, int *info, Arena &ws,
                 hipStream_t s);
// generic-rank-profile LU of one block at diagonal offset d0, sharing the
// zero-pivot flag *info with other blocks (set only if still clear)
int lu_block_generic(int path, const Field &F, int64_t m, int64_t n, int32_t *A, int64_t lda, int *info, int64_t d0,
                     Arena &ws, hipStream_t s);
// tile-iterative LU (tiled.hip): variant FFP_LU_RIGHT / CROUT / LEFT, tile k;
// *reductions = the modular-reduction count of the model of Section 3.1
int lu_tiled_run(int variant, int path, const Field &F, int64_t m, int64_t n, int64_t k, int32_t *A, int64_t lda,
                 int *info, Arena &ws, hipStream_t s, double *reductions);
size_t lu_tiled_ws(int variant, int path, const Field &F, int64_t m, int64_t n, int64_t k);
int reduction_count(int algorithm, int64_t n, int64_t k, double *count);
// *ok = every entry of the block lies in [0, p) (synchronises s)
int check_range_run(int64_t m, int64_t n, uint32_t p, const int32_t *A, int64_t lda, hipStream_t s, bool *ok);
// slab-recursive PLUQ (slab.hip): pivots in the order of the row-major search
size_t pluq_slab_ws(int64_t m, int64_t n, const Field &F, int path);
int pluq_slab_run(int path, const Field &F, int64_t m, int64_t n, int32_t *A, int64_t lda, int32_t *P, int32_t *Q,
                  int64_t *r, Arena &ws, hipStream_t s);
int pluq_batched_set_shape(int32_t batch, int32_t max_m, int32_t max_n, int shape);
// a pinned, device-visible host word for one rank / flag read-back (pooled)
struct RankWord {
    int64_t *host = nullptr, *dev = nullptr;
};
int rank_word_get(RankWord *w);
void rank_word_put(const RankWord &w);
// sorted rank profiles from P[0:r] (device); r is a host value
int rank_profiles(int64_t m, int64_t n, const int32_t *P, const int32_t *Q, int64_t r,
                  int32_t *rrp, int32_t *crp, Arena &ws, hipStream_t s);

// batched persistent PLUQ
size_t pluq_batched_ws(int32_t batch, int32_t max_m, int32_t max_n);
int pluq_batched_run(const Field &F, int32_t batch, const int32_t *m_arr, const int32_t *n_arr,
                     int32_t max_m, int32_t max_n, int32_t *A, const int64_t *A_off, int32_t *P,
                     const int64_t *P_off, int32_t *Q, const int64_t *Q_off, int32_t *rank,
                     int32_t *rrp, int32_t *crp, Arena &ws, hipStream_t s);
int pluq_batched_tune(const Field &F, int32_t batch, const int32_t *m_arr, const int32_t *n_arr, int32_t max_m,
                      int32_t max_n, int32_t *A, int64_t a_elems, const int64_t *A_off, int32_t *P,
                      const int64_t *P_off, int32_t *Q, const int64_t *Q_off, int32_t *rank, int32_t *rrp,
                      int32_t *crp, Arena &ws, hipStream_t s, int *chosen, float *ms_out);

}  // namespace ffp
