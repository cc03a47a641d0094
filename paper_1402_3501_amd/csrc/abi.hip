// Exported C ABI (include/ffpluq.h): argument validation, path selection,
// workspace accounting, and the host-side permutation helpers.
#include <cstring>
#include <functional>
#include <vector>

#include "ffp_internal.hpp"

namespace ffp {
int profile_enable(int on);
int profile_reset();
int profile_read(int path, int64_t *launches, double *ms, double *ops);
int profile_read_bytes(int path, double *bytes);

int resolve_path(int path, uint32_t p, int64_t m, int64_t n, int64_t k) {
    if (path != FFP_PATH_AUTO) return path;
    const int L = int8_limbs(p);
    if (L == 0) return FFP_PATH_FP64;
    // one limb: one INT8 product replaces one FP64 product at 64x the peak;
    // several limbs: L^2 INT8 products, still several times the FP64 peak,
    // once the product amortises the limb split (one more launch, ~16 us of
    // fixed cost in all).  Measured on MI355X (p = 131071 and 8388593,
    // whole-call time, FP64 / INT8): 256 x 4096 x 256 21 / 16 us, 1024 x 1024
    // x 256 21 / 17 us, 512 x 1024 x 512 19 / 20 us, 768^3 36 / 20 us, 512^3
    // 12 / 21 us, 256 x 2048 x 256 12 / 17 us: they cross near 0.5 * 10^9
    // field operations.
    if (L == 1) return (k >= 128 && m * n >= 256 * 256) ? FFP_PATH_INT8 : FFP_PATH_FP64;
    return 2.0 * (double)m * (double)n * (double)k >= 0.5e9 ? FFP_PATH_INT8 : FFP_PATH_FP64;
}

int fgemm_any(int path, const Field &F, int ta, int tb, int64_t m, int64_t n, int64_t k, uint32_t alpha,
              const int32_t *A, int64_t lda, const int32_t *B, int64_t ldb, uint32_t beta, int32_t *C,
              int64_t ldc, Arena &ws, hipStream_t s) {
    if (ws.counting) {
        if (path == FFP_PATH_INT8) ws.take(fgemm_i8_ws(F, m, n, k));
        return FFP_OK;
    }
    int eff = path == FFP_PATH_AUTO ? resolve_path(path, F.p, m, n, k) : path;
    // the limb split runs one grid row per 64 plane rows (at most 65535): a
    // taller product runs on the FP64 path (the same bits), or is refused
    // when p is beyond that path
    if (eff == FFP_PATH_INT8 && (m + n) / 64 + 8 > 65535) {
        if (F.p > FFP_P_MAX_FP64) return FFP_E_UNSUPPORTED;
        eff = FFP_PATH_FP64;
    }
    if (eff == FFP_PATH_INT8 && F.limbs > 0 && k > 0)
        return fgemm_i8(F, ta, tb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, ws, s);
    return fgemm_f64(F, ta, tb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, s);
}

static int check_field(uint32_t p, int path, int arg_p, int arg_path) {
    if (path < 0 || path > 2) return -arg_path;
    if (p < 2) return -arg_p;
    if (!is_prime_u32(p)) return FFP_E_NOTPRIME;
    if (path == FFP_PATH_FP64 && p > FFP_P_MAX_FP64) return FFP_E_P_RANGE;
    if (path == FFP_PATH_INT8 && int8_limbs(p) == 0) return FFP_E_P_RANGE;
    if (path == FFP_PATH_AUTO && p > FFP_P_MAX_FP64) return FFP_E_P_RANGE;
    return FFP_OK;
}

// path used for the products of a whole factorisation
static int pluq_path(int path, uint32_t p, int64_t m, int64_t n) {
    if (path != FFP_PATH_AUTO) return path;
    const int64_t k = (m < n ? m : n) / 2;
    return resolve_path(FFP_PATH_AUTO, p, m / 2, n / 2, k);
}

__global__ void k_set64(int64_t *dst, int64_t v) { *dst = v; }
__global__ void k_invperm(const int32_t *__restrict__ perm, int64_t n, int32_t *__restrict__ inv) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        inv[perm[i]] = (int32_t)i;
}

// Argument checks of ffp_fgemm (LAPACK numbering of its arguments), shared
// with the allocation-free variant; *eff = the path the product runs on.
int fgemm_validate(int transA, int transB, int64_t m, int64_t n, int64_t k, uint32_t p, uint32_t alpha,
                   const int32_t *A, int64_t lda, const int32_t *B, int64_t ldb, uint32_t beta, const int32_t *C,
                   int64_t ldc, int path, int *eff) {
    if (transA != 0 && transA != 1) return -1;
    if (transB != 0 && transB != 1) return -2;
    if (m < 0) return -3;
    if (n < 0) return -4;
    if (k < 0) return -5;
    FFP_CHECK(check_field(p, path, 6, 15));
    if (alpha >= p) return -7;
    if (beta >= p) return -12;
    *eff = resolve_path(path, p, m, n, k);
    if (m == 0 || n == 0) return FFP_OK;
    const int64_t acols = transA ? m : k, bcols = transB ? k : n;
    if (k > 0 && (!A || lda < (acols > 1 ? acols : 1))) return A ? -9 : -8;
    if (k > 0 && (!B || ldb < (bcols > 1 ? bcols : 1))) return B ? -11 : -10;
    if (!C || ldc < (n > 1 ? n : 1)) return C ? -14 : -13;
    return FFP_OK;
}

}  // namespace ffp

using namespace ffp;

extern "C" {

const char *ffp_error_string(int code) {
    switch (code) {
        case FFP_OK: return "success";
        case FFP_E_NOTPRIME: return "p is not prime";
        case FFP_E_P_RANGE: return "p too large for the requested arithmetic path";
        case FFP_E_WORKSPACE: return "workspace missing or too small";
        case FFP_E_HIP: return "HIP runtime error";
        case FFP_E_RANGE: return "input entry outside [0, p)";
        case FFP_E_UNSUPPORTED: return "unsupported request";
        case FFP_E_NODEVICE: return "no usable gfx950 device";
        case FFP_E_INTERNAL: return "internal consistency check failed";
        case FFP_E_SCRATCH: return "request exceeds the fixed scratch of the allocation-free entry point";
        default: return code < 0 && code > -64 ? "invalid argument" : "unknown error";
    }
}

const char *ffp_version(void) { return "ffpluq 0.1 gfx950"; }

int ffp_is_prime(uint32_t p) { return is_prime_u32(p) ? 1 : 0; }

int ffp_int8_limbs(uint32_t p) { return int8_limbs(p); }

int ffp_auto_path(uint32_t p, int64_t m, int64_t n, int64_t k) {
    return resolve_path(FFP_PATH_AUTO, p, m, n, k);
}

// ------------------------------------------------------------------ fgemm
size_t ffp_fgemm_workspace(int transA, int transB, int64_t m, int64_t n, int64_t k, uint32_t p, int path) {
    (void)transA;
    (void)transB;
    if (p < 2 || m < 0 || n < 0 || k < 0) return 0;
    const int eff = resolve_path(path, p, m, n, k);
    if (eff != FFP_PATH_INT8 || int8_limbs(p) == 0) return 0;
    Field F(p);
    return fgemm_i8_ws(F, m, n, k) + fgemm_i8_split_ws(m, n) + 256;
}

int ffp_fgemm(int transA, int transB, int64_t m, int64_t n, int64_t k, uint32_t p, uint32_t alpha,
              const int32_t *A, int64_t lda, const int32_t *B, int64_t ldb, uint32_t beta, int32_t *C,
              int64_t ldc, int path, void *ws, size_t ws_bytes, ffp_stream_t stream) {
    int eff = 0;
    FFP_CHECK(fgemm_validate(transA, transB, m, n, k, p, alpha, A, lda, B, ldb, beta, C, ldc, path, &eff));
    if (m == 0 || n == 0) return FFP_OK;
    const size_t need = ffp_fgemm_workspace(transA, transB, m, n, k, p, eff);
    if (need > 0 && (!ws || ws_bytes < need)) return FFP_E_WORKSPACE;
    Field F(p);
    Arena ar;
    ar.base = (char *)ws;
    ar.cap = ws_bytes;
    return fgemm_any(eff, F, transA, transB, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, ar,
                     (hipStream_t)stream);
}

// ------------------------------------------------------------------ fgemm, Winograd
static int wino_levels(int levels, int eff, const Field &F, int64_t m, int64_t n, int64_t k) {
    return levels == FFP_WINO_AUTO ? wino_auto_levels(eff, F, m, n, k) : levels;
}

size_t ffp_fgemm_wino_workspace(int transA, int transB, int64_t m, int64_t n, int64_t k, uint32_t p, int path,
                                int levels) {
    (void)transA;
    (void)transB;
    if (p < 2 || m < 0 || n < 0 || k < 0 || levels < FFP_WINO_AUTO || levels > FFP_WINO_MAX_LEVELS) return 0;
    Field F(p);
    const int lv = wino_levels(levels, path, F, m, n, k);
    return fgemm_wino_ws(path, F, lv, m, n, k) + 256;
}

int ffp_fgemm_wino(int transA, int transB, int64_t m, int64_t n, int64_t k, uint32_t p, uint32_t alpha,
                   const int32_t *A, int64_t lda, const int32_t *B, int64_t ldb, uint32_t beta, int32_t *C,
                   int64_t ldc, int path, int levels, void *ws, size_t ws_bytes, ffp_stream_t stream) {
    int eff = 0;
    FFP_CHECK(fgemm_validate(transA, transB, m, n, k, p, alpha, A, lda, B, ldb, beta, C, ldc, path, &eff));
    if (levels < FFP_WINO_AUTO || levels > FFP_WINO_MAX_LEVELS) return -16;
    if (m == 0 || n == 0) return FFP_OK;
    const size_t need = ffp_fgemm_wino_workspace(transA, transB, m, n, k, p, path, levels);
    if (need > 0 && (!ws || ws_bytes < need)) return FFP_E_WORKSPACE;
    Field F(p);
    const int lv = wino_levels(levels, path, F, m, n, k);
    Arena ar;
    ar.base = (char *)ws;
    ar.cap = ws_bytes;
    return fgemm_wino(path, F, lv, transA, transB, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, ar,
                      (hipStream_t)stream);
}

// ------------------------------------------------------------------ tile-iterative LU
size_t ffp_lu_tiled_workspace(int variant, int64_t m, int64_t n, int64_t k, uint32_t p, int path) {
    if (p < 2 || m < 0 || n < 0 || k < 1 || variant < FFP_LU_RIGHT || variant > FFP_LU_LEFT) return 0;
    Field F(p);
    return lu_tiled_ws(variant, pluq_path(path, p, m, n), F, m, n, k);
}

int ffp_lu_tiled(int variant, int64_t m, int64_t n, uint32_t p, int32_t *A, int64_t lda, int64_t k, int32_t *info_dev,
                 int path, void *ws, size_t ws_bytes, ffp_stream_t stream) {
    if (variant < FFP_LU_RIGHT || variant > FFP_LU_LEFT) return -1;
    if (m < 0 || m > INT32_MAX) return -2;
    if (n < 0 || n > INT32_MAX) return -3;
    FFP_CHECK(check_field(p, path, 4, 9));
    if (m > 0 && n > 0 && !A) return -5;
    if (lda < (n > 1 ? n : 1)) return -6;
    if (k < 1) return -7;
    if (!info_dev) return -8;
    const size_t need = ffp_lu_tiled_workspace(variant, m, n, k, p, path);
    if (!ws || ws_bytes < need) return FFP_E_WORKSPACE;
    Field F(p);
    Arena ar;
    ar.base = (char *)ws;
    ar.cap = ws_bytes;
    return lu_tiled_run(variant, pluq_path(path, p, m, n), F, m, n, k, A, lda, (int *)info_dev, ar,
                        (hipStream_t)stream, nullptr);
}

int ffp_reduction_count(int algorithm, int64_t n, int64_t k, double *count) {
    if (algorithm < FFP_LU_RIGHT || algorithm > FFP_LU_SLAB_RECURSIVE) return -1;
    if (n < 0) return -2;
    if (k < 1 && algorithm <= FFP_LU_LEFT) return -3;
    if (!count) return -4;
    return reduction_count(algorithm, n, k, count);
}

// ------------------------------------------------------------------ echelon forms
// Common checks of the PLUQ-consumer calls: sizes, field, factor pointers and
// the rank.  Their arguments (m, n, p, LU, ld, P, Q, r) sit at positions
// off + 1 .. off + 8; the path is argument arg_path.
static int check_factors(int64_t m, int64_t n, uint32_t p, const int32_t *LU, int64_t ld, const int32_t *P,
                         const int32_t *Q, int64_t r, int path, int off, int arg_path) {
    if (m < 0 || m > INT32_MAX) return -(off + 1);
    if (n < 0 || n > INT32_MAX) return -(off + 2);
    FFP_CHECK(check_field(p, path, off + 3, arg_path));
    if (m > 0 && n > 0 && !LU) return -(off + 4);
    if (ld < (n > 1 ? n : 1)) return -(off + 5);
    if (m > 0 && !P) return -(off + 6);
    if (n > 0 && !Q) return -(off + 7);
    if (r < 0 || r > (m < n ? m : n)) return -(off + 8);
    return FFP_OK;
}

static size_t count_ws(const std::function<int(Arena &)> &f) {
    Arena ar;
    ar.counting = true;
    f(ar);
    return ar.peak + 512;
}

size_t ffp_echelon_workspace(int form, int64_t m, int64_t n, int64_t r, uint32_t p, int path) {
    if (p < 2 || m < 0 || n < 0 || r < 0 || r > (m < n ? m : n) || (form != 0 && form != 1)) return 0;
    Field F(p);
    const int32_t dummy = 0;
    return count_ws([&](Arena &ar) {
        return echelon_run(form, path, F, m, n, &dummy, n > 1 ? n : 1, &dummy, &dummy, r, nullptr, 1, ar, nullptr);
    });
}

int ffp_echelon(int form, int64_t m, int64_t n, uint32_t p, const int32_t *LU, int64_t ld, const int32_t *P,
                const int32_t *Q, int64_t r, int32_t *E, int64_t lde, int path, void *ws, size_t ws_bytes,
                ffp_stream_t stream) {
    if (form != 0 && form != 1) return -1;
    FFP_CHECK(check_factors(m, n, p, LU, ld, P, Q, r, path, 1, 12));
    if (r == 0) return FFP_OK;
    if (!E) return -10;
    if (lde < (form == 0 ? n : r)) return -11;
    const size_t need = ffp_echelon_workspace(form, m, n, r, p, path);
    if (!ws || ws_bytes < need) return FFP_E_WORKSPACE;
    Field F(p);
    Arena ar;
    ar.base = (char *)ws;
    ar.cap = ws_bytes;
    return echelon_run(form, path, F, m, n, LU, ld, P, Q, r, E, lde, ar, (hipStream_t)stream);
}

size_t ffp_nullspace_workspace(int side, int64_t m, int64_t n, int64_t r, uint32_t p, int path) {
    if (p < 2 || m < 0 || n < 0 || r < 0 || r > (m < n ? m : n) || (side != 0 && side != 1)) return 0;
    Field F(p);
    const int32_t dummy = 0;
    return count_ws([&](Arena &ar) {
        return nullspace_run(side, path, F, m, n, &dummy, n > 1 ? n : 1, &dummy, &dummy, r, nullptr, 1, ar, nullptr);
    });
}

int ffp_nullspace(int side, int64_t m, int64_t n, uint32_t p, const int32_t *LU, int64_t ld, const int32_t *P,
                  const int32_t *Q, int64_t r, int32_t *N, int64_t ldn, int path, void *ws, size_t ws_bytes,
                  ffp_stream_t stream) {
    if (side != 0 && side != 1) return -1;
    FFP_CHECK(check_factors(m, n, p, LU, ld, P, Q, r, path, 1, 12));
    const int64_t rows = side == 0 ? n : m - r, cols = side == 0 ? n - r : m;
    if (rows == 0 || cols == 0) return FFP_OK;
    if (!N) return -10;
    if (ldn < cols) return -11;
    const size_t need = ffp_nullspace_workspace(side, m, n, r, p, path);
    if (!ws || ws_bytes < need) return FFP_E_WORKSPACE;
    Field F(p);
    Arena ar;
    ar.base = (char *)ws;
    ar.cap = ws_bytes;
    return nullspace_run(side, path, F, m, n, LU, ld, P, Q, r, N, ldn, ar, (hipStream_t)stream);
}

size_t ffp_solve_workspace(int64_t m, int64_t n, int64_t r, int64_t nrhs, uint32_t p, int path) {
    if (p < 2 || m < 0 || n < 0 || r < 0 || r > (m < n ? m : n) || nrhs < 0) return 0;
    Field F(p);
    const int32_t dummy = 0;
    return count_ws([&](Arena &ar) {
        return solve_run(path, F, m, n, &dummy, n > 1 ? n : 1, &dummy, &dummy, r, nrhs, &dummy, nrhs > 1 ? nrhs : 1,
                         nullptr, 1, nullptr, ar, nullptr);
    });
}

int ffp_solve(int64_t m, int64_t n, uint32_t p, const int32_t *LU, int64_t ld, const int32_t *P, const int32_t *Q,
              int64_t r, int64_t nrhs, const int32_t *B, int64_t ldb, int32_t *X, int64_t ldx, int32_t *consistent,
              int path, void *ws, size_t ws_bytes, ffp_stream_t stream) {
    FFP_CHECK(check_factors(m, n, p, LU, ld, P, Q, r, path, 0, 15));
    if (nrhs < 0) return -9;
    if (nrhs == 0) return FFP_OK;
    if (m > 0 && !B) return -10;
    if (ldb < nrhs) return -11;
    if (n > 0 && !X) return -12;
    if (ldx < nrhs) return -13;
    if (!consistent) return -14;
    const size_t need = ffp_solve_workspace(m, n, r, nrhs, p, path);
    if (!ws || ws_bytes < need) return FFP_E_WORKSPACE;
    Field F(p);
    Arena ar;
    ar.base = (char *)ws;
    ar.cap = ws_bytes;
    return solve_run(path, F, m, n, LU, ld, P, Q, r, nrhs, B, ldb, X, ldx, consistent, ar, (hipStream_t)stream);
}

// ------------------------------------------------------------------ ftrsm
size_t ffp_ftrsm_workspace(int side, int uplo, int trans, int diag, int64_t m, int64_t n, uint32_t p, int path) {
    if (p < 2 || m < 0 || n < 0) return 0;
    const int64_t d = side == 0 ? m : n, nv = side == 0 ? n : m;
    const int eff = resolve_path(path, p, d / 2, nv, d / 2);
    Field F(p);
    Arena ar;
    ar.counting = true;
    ftrsm_run(eff, F, side, uplo, trans, diag, m, n, 1, nullptr, 1, nullptr, 1, ar, nullptr);
    return ar.peak + 256;
}

int ffp_ftrsm(int side, int uplo, int trans, int diag, int64_t m, int64_t n, uint32_t p, uint32_t alpha,
              const int32_t *T, int64_t ldt, int32_t *B, int64_t ldb, int path, void *ws, size_t ws_bytes,
              ffp_stream_t stream) {
    if (side != 0 && side != 1) return -1;
    if (uplo != 0 && uplo != 1) return -2;
    if (trans != 0 && trans != 1) return -3;
    if (diag != 0 && diag != 1) return -4;
    if (m < 0) return -5;
    if (n < 0) return -6;
    FFP_CHECK(check_field(p, path, 7, 13));
    if (alpha >= p) return -8;
    const int64_t d = side == 0 ? m : n;
    if (m == 0 || n == 0) return FFP_OK;
    if (!T) return -9;
    if (ldt < (d > 1 ? d : 1)) return -10;
    if (!B) return -11;
    if (ldb < (n > 1 ? n : 1)) return -12;
    const int64_t nv = side == 0 ? n : m;
    const int eff = resolve_path(path, p, d / 2, nv, d / 2);
    const size_t need = ffp_ftrsm_workspace(side, uplo, trans, diag, m, n, p, path);
    if (need > 0 && (!ws || ws_bytes < need)) return FFP_E_WORKSPACE;
    Field F(p);
    Arena ar;
    ar.base = (char *)ws;
    ar.cap = ws_bytes;
    return ftrsm_run(eff, F, side, uplo, trans, diag, m, n, alpha, T, ldt, B, ldb, ar, (hipStream_t)stream);
}

// ------------------------------------------------------------------ flaswp
size_t ffp_flaswp_workspace(int dim, int64_t m, int64_t n) {
    if (m <= 0 || n <= 0) return 0;
    const int64_t len = dim == 0 ? m : n;
    return (((size_t)m * (size_t)n * 4 + 255) & ~(size_t)255) + (size_t)len * 4 + 512;
}

int ffp_flaswp(int dim, int64_t m, int64_t n, int32_t *A, int64_t lda, const int32_t *perm, int inverse, void *ws,
               size_t ws_bytes, ffp_stream_t stream) {
    if (dim != 0 && dim != 1) return -1;
    if (m < 0) return -2;
    if (n < 0) return -3;
    if (m == 0 || n == 0) return FFP_OK;
    if (!A) return -4;
    if (lda < (n > 1 ? n : 1)) return -5;
    if (!perm) return -6;
    if (inverse != 0 && inverse != 1) return -7;
    const size_t need = ffp_flaswp_workspace(dim, m, n);
    if (!ws || ws_bytes < need) return FFP_E_WORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    Arena ar;
    ar.base = (char *)ws;
    ar.cap = ws_bytes;
    const int64_t len = dim == 0 ? m : n;
    const int32_t *g = perm;
    if (inverse) {
        int32_t *inv = (int32_t *)ar.take((size_t)len * 4);
        unsigned grid = (unsigned)((len + 255) / 256 < 1024 ? (len + 255) / 256 : 1024);
        hipLaunchKernelGGL(k_invperm, dim3(grid), dim3(256), 0, s, perm, len, inv);
        FFP_HIP_CHECK(hipGetLastError());
        g = inv;
    }
    PermSpec ps;
    ps.idx = g;
    return dim == 0 ? permute_inplace(m, n, A, lda, ps, PermSpec(), ar, s)
                    : permute_inplace(m, n, A, lda, PermSpec(), ps, ar, s);
}

// ------------------------------------------------------------------ pluq
size_t ffp_pluq_workspace(int64_t m, int64_t n, uint32_t p, int path) {
    if (p < 2 || m < 0 || n < 0) return 0;
    Field F(p);
    const int eff = pluq_path(path, p, m, n);
    return pluq_ws(m, n, F, eff == FFP_PATH_INT8 && int8_limbs(p) > 0 ? FFP_PATH_INT8 : FFP_PATH_FP64) +
           (size_t)(m + n) * 4 + 4096;
}

int ffp_pluq(int64_t m, int64_t n, uint32_t p, int32_t *A, int64_t lda, int32_t *P, int32_t *Q, int64_t *rank_dev,
             int64_t *rank_host, int32_t *rrp, int32_t *crp, int path, void *ws, size_t ws_bytes,
             ffp_stream_t stream) {
    if (m < 0) return -1;
    if (n < 0) return -2;
    FFP_CHECK(check_field(p, path, 3, 12));
    if (m > 0 && n > 0 && !A) return -4;
    if (lda < (n > 1 ? n : 1)) return -5;
    if (m > 0 && !P) return -6;
    if (n > 0 && !Q) return -7;
    if (m > INT32_MAX || n > INT32_MAX) return -1;
    const size_t need = ffp_pluq_workspace(m, n, p, path);
    if (!ws || ws_bytes < need) return FFP_E_WORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    Field F(p);
    Arena ar;
    ar.base = (char *)ws;
    ar.cap = ws_bytes;
    int64_t r = 0;
    // with FFP_PATH_AUTO every product inside the factorisation picks its own path
    FFP_CHECK(pluq_run(path, F, m, n, A, lda, P, Q, &r, ar, s));
    if (rank_dev) {
        hipLaunchKernelGGL(k_set64, dim3(1), dim3(1), 0, s, rank_dev, r);
        FFP_HIP_CHECK(hipGetLastError());
    }
    FFP_CHECK(rank_profiles(m, n, P, Q, r, rrp, crp, ar, s));
    if (rank_host) {
        FFP_HIP_CHECK(hipStreamSynchronize(s));
        *rank_host = r;
    }
    return FFP_OK;
}

// ------------------------------------------------------------------ slab-recursive PLUQ
size_t ffp_pluq_slab_workspace(int64_t m, int64_t n, uint32_t p, int path) {
    if (p < 2 || m < 0 || n < 0) return 0;
    Field F(p);
    const int eff = pluq_path(path, p, m, n);
    return pluq_slab_ws(m, n, F, eff == FFP_PATH_INT8 && int8_limbs(p) > 0 ? FFP_PATH_INT8 : FFP_PATH_FP64) +
           (size_t)(m + n) * 4 + 4096;
}

int ffp_pluq_slab(int64_t m, int64_t n, uint32_t p, int32_t *A, int64_t lda, int32_t *P, int32_t *Q, int64_t *rank_dev,
                  int64_t *rank_host, int32_t *rrp, int32_t *crp, int path, void *ws, size_t ws_bytes,
                  ffp_stream_t stream) {
    if (m < 0 || m > INT32_MAX) return -1;
    if (n < 0 || n > FFP_SLAB_MAX_COLS) return -2;
    FFP_CHECK(check_field(p, path, 3, 12));
    if (m > 0 && n > 0 && !A) return -4;
    if (lda < (n > 1 ? n : 1)) return -5;
    if (m > 0 && !P) return -6;
    if (n > 0 && !Q) return -7;
    const size_t need = ffp_pluq_slab_workspace(m, n, p, path);
    if (!ws || ws_bytes < need) return FFP_E_WORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    Field F(p);
    Arena ar;
    ar.base = (char *)ws;
    ar.cap = ws_bytes;
    int64_t r = 0;
    FFP_CHECK(pluq_slab_run(path, F, m, n, A, lda, P, Q, &r, ar, s));
    if (rank_dev) {
        hipLaunchKernelGGL(k_set64, dim3(1), dim3(1), 0, s, rank_dev, r);
        FFP_HIP_CHECK(hipGetLastError());
    }
    FFP_CHECK(rank_profiles(m, n, P, Q, r, rrp, crp, ar, s));
    if (rank_host) {
        FFP_HIP_CHECK(hipStreamSynchronize(s));
        *rank_host = r;
    }
    return FFP_OK;
}

// ------------------------------------------------------------------ lu_nopiv
size_t ffp_lu_nopiv_workspace(int64_t m, int64_t n, uint32_t p, int path) {
    if (p < 2 || m < 0 || n < 0) return 0;
    Field F(p);
    const int eff = pluq_path(path, p, m, n);
    return pluq_ws(m, n, F, eff == FFP_PATH_INT8 && int8_limbs(p) > 0 ? FFP_PATH_INT8 : FFP_PATH_FP64) + 4096;
}

int ffp_lu_nopiv(int64_t m, int64_t n, uint32_t p, int32_t *A, int64_t lda, int32_t *info_dev, int path, void *ws,
                 size_t ws_bytes, ffp_stream_t stream) {
    if (m < 0 || m > INT32_MAX) return -1;
    if (n < 0 || n > INT32_MAX) return -2;
    FFP_CHECK(check_field(p, path, 3, 7));
    if (m > 0 && n > 0 && !A) return -4;
    if (lda < (n > 1 ? n : 1)) return -5;
    if (!info_dev) return -6;
    const size_t need = ffp_lu_nopiv_workspace(m, n, p, path);
    if (!ws || ws_bytes < need) return FFP_E_WORKSPACE;
    Field F(p);
    Arena ar;
    ar.base = (char *)ws;
    ar.cap = ws_bytes;
    return lu_nopiv_run(path, F, m, n, A, lda, (int *)info_dev, ar, (hipStream_t)stream);
}

// ------------------------------------------------------------------ check_range
int ffp_check_range(int64_t m, int64_t n, uint32_t p, const int32_t *A, int64_t lda, ffp_stream_t stream) {
    if (m < 0) return -1;
    if (n < 0) return -2;
    if (p < 2) return -3;
    if (m > 0 && n > 0 && !A) return -4;
    if (lda < (n > 1 ? n : 1)) return -5;
    bool ok = true;
    FFP_CHECK(check_range_run(m, n, p, A, lda, (hipStream_t)stream, &ok));
    return ok ? FFP_OK : FFP_E_RANGE;
}

// ------------------------------------------------------------------ batched
size_t ffp_pluq_batched_workspace(int32_t batch, int32_t max_m, int32_t max_n, uint32_t p, int path) {
    (void)p;
    (void)path;
    if (batch <= 0) return 0;
    return pluq_batched_ws(batch, max_m, max_n);
}

int ffp_pluq_batched(int32_t batch, const int32_t *m_arr, const int32_t *n_arr, int32_t max_m, int32_t max_n,
                     uint32_t p, int32_t *A_packed, const int64_t *A_off, int32_t *P_packed, const int64_t *P_off,
                     int32_t *Q_packed, const int64_t *Q_off, int32_t *rank_arr, int32_t *rrp_packed,
                     int32_t *crp_packed, int path, void *ws, size_t ws_bytes, ffp_stream_t stream) {
    if (batch < 0) return -1;
    if (batch == 0) return FFP_OK;
    if (!m_arr) return -2;
    if (!n_arr) return -3;
    if (max_m < 0 || max_m > FFP_BATCH_MAX_DIM) return -4;
    if (max_n < 0 || max_n > FFP_BATCH_MAX_DIM) return -5;
    FFP_CHECK(check_field(p, path, 6, 16));
    if (!A_packed) return -7;
    if (!A_off) return -8;
    if (!P_packed) return -9;
    if (!P_off) return -10;
    if (!Q_packed) return -11;
    if (!Q_off) return -12;
    if (!rank_arr) return -13;
    const size_t need = ffp_pluq_batched_workspace(batch, max_m, max_n, p, path);
    if (need > 0 && (!ws || ws_bytes < need)) return FFP_E_WORKSPACE;
    Field F(p);
    Arena ar;
    ar.base = (char *)ws;
    ar.cap = ws_bytes;
    return pluq_batched_run(F, batch, m_arr, n_arr, max_m, max_n, A_packed, A_off, P_packed, P_off, Q_packed,
                            Q_off, rank_arr, rrp_packed, crp_packed, ar, (hipStream_t)stream);
}

int ffp_pluq_batched_set_shape(int32_t batch, int32_t max_m, int32_t max_n, int shape) {
    if (batch < 0) return -1;
    if (max_m < 0 || max_m > FFP_BATCH_MAX_DIM) return -2;
    if (max_n < 0 || max_n > FFP_BATCH_MAX_DIM) return -3;
    return pluq_batched_set_shape(batch, max_m, max_n, shape);
}

size_t ffp_pluq_batched_tune_workspace(int32_t batch, int32_t max_m, int32_t max_n, int64_t a_elems) {
    if (batch <= 0) return 0;
    return pluq_batched_ws(batch, max_m, max_n) + (size_t)(a_elems > 0 ? a_elems : 0) * 4 + 512;
}

int ffp_pluq_batched_tune(int32_t batch, const int32_t *m_arr, const int32_t *n_arr, int32_t max_m, int32_t max_n,
                          uint32_t p, int32_t *A_packed, int64_t a_elems, const int64_t *A_off, int32_t *P_packed,
                          const int64_t *P_off, int32_t *Q_packed, const int64_t *Q_off, int32_t *rank_arr,
                          int32_t *rrp_packed, int32_t *crp_packed, int path, int *shape_out, float *ms_out,
                          void *ws, size_t ws_bytes, ffp_stream_t stream) {
    if (batch < 0) return -1;
    if (batch == 0) return FFP_OK;
    if (!m_arr) return -2;
    if (!n_arr) return -3;
    if (max_m < 0 || max_m > FFP_BATCH_MAX_DIM) return -4;
    if (max_n < 0 || max_n > FFP_BATCH_MAX_DIM) return -5;
    FFP_CHECK(check_field(p, path, 6, 17));
    if (!A_packed) return -7;
    if (a_elems < 0) return -8;
    if (!A_off) return -9;
    if (!P_packed) return -10;
    if (!P_off) return -11;
    if (!Q_packed) return -12;
    if (!Q_off) return -13;
    if (!rank_arr) return -14;
    const size_t need = ffp_pluq_batched_tune_workspace(batch, max_m, max_n, a_elems);
    if (!ws || ws_bytes < need) return FFP_E_WORKSPACE;
    Field F(p);
    Arena ar;
    ar.base = (char *)ws;
    ar.cap = ws_bytes;
    return pluq_batched_tune(F, batch, m_arr, n_arr, max_m, max_n, A_packed, a_elems, A_off, P_packed, P_off,
                             Q_packed, Q_off, rank_arr, rrp_packed, crp_packed, ar, (hipStream_t)stream, shape_out,
                             ms_out);
}

// ------------------------------------------------------------------ host helpers
int ffp_perm_to_swaps(int64_t len, const int32_t *perm, int32_t *ipiv) {
    if (len < 0) return -1;
    if (len > 0 && !perm) return -2;
    if (len > 0 && !ipiv) return -3;
    std::vector<int32_t> cur(len), pos(len);
    std::vector<char> seen(len, 0);
    for (int64_t i = 0; i < len; ++i) {
        if (perm[i] < 0 || perm[i] >= len || seen[perm[i]]) return -2;
        seen[perm[i]] = 1;
        cur[i] = (int32_t)i;
        pos[i] = (int32_t)i;
    }
    for (int64_t i = 0; i < len; ++i) {
        const int32_t j = pos[perm[i]];
        ipiv[i] = j;
        const int32_t a = cur[i], b = cur[j];
        cur[i] = b;
        cur[j] = a;
        pos[b] = (int32_t)i;
        pos[a] = j;
    }
    return FFP_OK;
}

int ffp_swaps_to_perm(int64_t len, const int32_t *ipiv, int32_t *perm) {
    if (len < 0) return -1;
    if (len > 0 && !ipiv) return -2;
    if (len > 0 && !perm) return -3;
    for (int64_t i = 0; i < len; ++i) {
        if (ipiv[i] < 0 || ipiv[i] >= len) return -2;
        perm[i] = (int32_t)i;
    }
    for (int64_t i = 0; i < len; ++i) {
        const int32_t j = ipiv[i];
        const int32_t t = perm[i];
        perm[i] = perm[j];
        perm[j] = t;
    }
    return FFP_OK;
}

// ------------------------------------------------------------------ profiling
int ffp_profile_enable(int on) { return profile_enable(on); }
int ffp_profile_reset(void) { return profile_reset(); }
int ffp_profile_read(int path, int64_t *launches, double *milliseconds, double *field_ops) {
    return profile_read(path, launches, milliseconds, field_ops);
}
int ffp_profile_read_bytes(int path, double *bytes) { return profile_read_bytes(path, bytes); }
const char *ffp_profile_kind_name(int kind) { return profile_kind_name(kind); }

}  // extern "C"
