// Tile-iterative block LU, in the three orders of Section 3.1 (Table 1):
// right-looking, Crout and left-looking, for inputs of generic rank profile
// (Section 3 assumes no rank deficiency in any diagonal block), with the
// modular-reduction count of Section 3.1 kept along the way.
//
// With tiles of k rows / columns and the diagonal block i at offset
// i0 = (i - 1) k (kb = k, or less for the last one), the main loops issue:
//
//   right-looking:  pluq(kb); utrsm(kb, kb, n - i0 - kb); trsm(kb, kb, m - i0 - kb);
//                   gemm(m - i0 - kb, kb, n - i0 - kb)
//   Crout:          gemm(m - i0, i0, kb); gemm(kb, i0, n - i0 - kb)  (i > 1);
//                   pluq(kb); utrsm(kb, kb, n - i0 - kb); trsm(kb, kb, m - i0 - kb)
//   left-looking:   utrsm(i0, i0, kb); gemm(m - i0, i0, kb)  (i > 1);
//                   pluq(kb); trsm(kb, kb, m - i0 - kb)
//                   (and, for a wide matrix, one last utrsm of the columns
//                   right of the last diagonal block)
//
// utrsm is the unit lower solve from the left (U blocks), trsm the upper
// solve from the right (L blocks), gemm the Schur update C -= A B, pluq the
// generic LU of the diagonal block.  Every call is also charged the number
// of modular reductions the model of Section 3.1 gives it: a product of an
// m x k by a k x n matrix costs m n, a unit triangular solve with an m x m
// triangle and n right-hand sides (m - 1) n, a non-unit one (2 m - 1) n, and
// the k x k base case the count of the unblocked Crout elimination,
// 3/2 k^2 - 7/2 k + 3.  Run in counting mode (no device), the same loops
// give the totals that Table 2 states in closed form.
#include <cmath>

#include "ffp_internal.hpp"

namespace ffp {

namespace {
__global__ void k_clear_info(int *info) { *info = 0; }

// reduction counts of the model of Section 3.1
double r_gemm(int64_t m, int64_t k, int64_t n) { return (m > 0 && k > 0 && n > 0) ? (double)m * (double)n : 0.0; }
double r_utrsm(int64_t m, int64_t n) { return (m > 0 && n > 0) ? (double)(m - 1) * (double)n : 0.0; }
double r_trsm(int64_t m, int64_t n) { return (m > 0 && n > 0) ? (double)(2 * m - 1) * (double)n : 0.0; }
double r_base(int64_t k) { return k > 0 ? 1.5 * (double)k * (double)k - 3.5 * (double)k + 3.0 : 0.0; }

struct Tiled {
    int path;
    const Field &F;
    int32_t *A;
    int64_t lda;
    int *info;
    Arena &ws;
    hipStream_t s;
    double count = 0.0;

    int32_t *at(int64_t i, int64_t j) const { return A ? A + i * lda + j : nullptr; }

    // generic LU of the kb x kb diagonal block at offset i0
    int base(int64_t i0, int64_t kb) {
        count += r_base(kb);
        if (ws.counting) {
            ws.take(pluq_ws(kb, kb, F, path));
            return FFP_OK;
        }
        return lu_block_generic(path, F, kb, kb, at(i0, i0), lda, info, i0, ws, s);
    }
    // B (d x nv at (r0, c0)) <- L^-1 B, L the unit lower d x d block at (t0, t0)
    int utrsm(int64_t t0, int64_t d, int64_t r0, int64_t c0, int64_t nv) {
        if (d <= 0 || nv <= 0) return FFP_OK;
        count += r_utrsm(d, nv);
        return ftrsm_run(resolve_path(path, F.p, d / 2, nv, d / 2), F, 0, 0, 0, 1, d, nv, 1, at(t0, t0), lda,
                         at(r0, c0), lda, ws, s);
    }
    // B (nv x d at (r0, c0)) <- B U^-1, U the upper d x d block at (t0, t0)
    int trsm(int64_t t0, int64_t d, int64_t r0, int64_t c0, int64_t nv) {
        if (d <= 0 || nv <= 0) return FFP_OK;
        count += r_trsm(d, nv);
        return ftrsm_run(resolve_path(path, F.p, d / 2, nv, d / 2), F, 1, 1, 0, 0, nv, d, 1, at(t0, t0), lda,
                         at(r0, c0), lda, ws, s);
    }
    // C (m x n at (ci, cj)) -= A (m x k at (ai, aj)) B (k x n at (bi, bj))
    int gemm(int64_t m, int64_t n, int64_t k, int64_t ai, int64_t aj, int64_t bi, int64_t bj, int64_t ci, int64_t cj) {
        if (m <= 0 || n <= 0 || k <= 0) return FFP_OK;
        count += r_gemm(m, k, n);
        return fgemm_any(resolve_path(path, F.p, m, n, k), F, 0, 0, m, n, k, F.p - 1, at(ai, aj), lda, at(bi, bj),
                         lda, 1, at(ci, cj), lda, ws, s);
    }
};
}  // namespace

int lu_tiled_run(int variant, int path, const Field &F, int64_t m, int64_t n, int64_t k, int32_t *A, int64_t lda,
                 int *info, Arena &ws, hipStream_t s, double *reductions) {
    Tiled t{path, F, A, lda, info, ws, s};
    if (!ws.counting) {
        hipLaunchKernelGGL(k_clear_info, dim3(1), dim3(1), 0, s, info);
        FFP_HIP_CHECK(hipGetLastError());
    }
    const int64_t K = m < n ? m : n;
    for (int64_t i0 = 0; i0 < K; i0 += k) {
        const int64_t kb = K - i0 < k ? K - i0 : k, e = i0 + kb;
        if (variant == FFP_LU_RIGHT) {
            FFP_CHECK(t.base(i0, kb));
            FFP_CHECK(t.utrsm(i0, kb, i0, e, n - e));
            FFP_CHECK(t.trsm(i0, kb, e, i0, m - e));
            FFP_CHECK(t.gemm(m - e, n - e, kb, e, i0, i0, e, e, e));
        } else if (variant == FFP_LU_CROUT) {
            // the block column (diagonal block and below) and the block row
            // right of it, updated by all earlier steps at once
            FFP_CHECK(t.gemm(m - i0, kb, i0, i0, 0, 0, i0, i0, i0));
            FFP_CHECK(t.gemm(kb, n - e, i0, i0, 0, 0, e, i0, e));
            FFP_CHECK(t.base(i0, kb));
            FFP_CHECK(t.utrsm(i0, kb, i0, e, n - e));
            FFP_CHECK(t.trsm(i0, kb, e, i0, m - e));
        } else {
            // the U block above the diagonal block, then the block column
            // (diagonal block and below) updated by all earlier steps
            FFP_CHECK(t.utrsm(0, i0, 0, i0, kb));
            FFP_CHECK(t.gemm(m - i0, kb, i0, i0, 0, 0, i0, i0, i0));
            FFP_CHECK(t.base(i0, kb));
            FFP_CHECK(t.trsm(i0, kb, e, i0, m - e));
        }
    }
    // left-looking never touched the columns right of the last diagonal block
    if (variant == FFP_LU_LEFT && n > K) FFP_CHECK(t.utrsm(0, K, 0, K, n - K));
    if (reductions) *reductions = t.count;
    return FFP_OK;
}

size_t lu_tiled_ws(int variant, int path, const Field &F, int64_t m, int64_t n, int64_t k) {
    Arena ar;
    ar.counting = true;
    lu_tiled_run(variant, path, F, m, n, k, nullptr, n > 1 ? n : 1, nullptr, ar, nullptr, nullptr);
    return ar.peak + 1024;
}

// The reductions of the two recursive algorithms of Table 2 under the same
// model, for an n x n input of generic rank profile split in halves down to
// single rows / columns:
//   tile recursive (four quadrants): R(n) = 2 R(n/2) + utrsm(n/2, n/2, n/2)
//     + trsm(n/2, n/2, n/2) + gemm(n/2, n/2, n/2), R(1) = 1 (the 1 x 1 base
//     case of the Crout count);
//   slab recursive (row halves, each slab as wide as the rest of the
//     matrix): S(m, w) = S(m/2, w) + trsm(m/2, m/2, m/2)
//     + gemm(m/2, m/2, w - m/2) + S(m/2, w - m/2), S(1, w) = 0 (a single row
//     is its own U row).
static double r_tile_rec(int64_t n) {
    if (n <= 1) return n == 1 ? 1.0 : 0.0;
    const int64_t h = n / 2;
    return r_tile_rec(h) + r_tile_rec(n - h) + r_utrsm(h, n - h) + r_trsm(h, n - h) + r_gemm(n - h, h, n - h);
}
static double r_slab_rec(int64_t m, int64_t w) {
    if (m <= 1) return 0.0;
    const int64_t h = m / 2;
    return r_slab_rec(h, w) + r_trsm(h, m - h) + r_gemm(m - h, h, w - h) + r_slab_rec(m - h, w - h);
}

int reduction_count(int algorithm, int64_t n, int64_t k, double *count) {
    if (algorithm == FFP_LU_TILE_RECURSIVE) {
        *count = r_tile_rec(n);
        return FFP_OK;
    }
    if (algorithm == FFP_LU_SLAB_RECURSIVE) {
        *count = r_slab_rec(n, n);
        return FFP_OK;
    }
    Field F(65521);
    Arena ar;
    ar.counting = true;
    return lu_tiled_run(algorithm, FFP_PATH_FP64, F, n, n, k, nullptr, n > 1 ? n : 1, nullptr, ar, nullptr, count);
}

}  // namespace ffp
