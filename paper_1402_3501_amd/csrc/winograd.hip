// Strassen-Winograd layer over fgemm (Section 2.1: the sequential fgemm runs
// recursive steps of Winograd's variant of Strassen's algorithm on top of the
// plain product; Sections 2.3 and 3.2 discuss its gain and crossover).
//
// One level splits op(A) (m x k), op(B) (k x n) and C into 2 x 2 blocks of
// half size and forms the product from 7 block products instead of 8:
//
//   S1 = A21 + A22   S2 = S1 - A11   S3 = A11 - A21   S4 = A12 - S2
//   T1 = B12 - B11   T2 = B22 - T1   T3 = B22 - B12   T4 = T2 - B21
//   P1 = A11 B11  P2 = A12 B21  P3 = S4 B22  P4 = A22 T4
//   P5 = S1 T1    P6 = S2 T2    P7 = S3 T3
//   C11 = P1 + P2             C12 = P1 + P6 + P5 + P3
//   C21 = P1 + P6 + P7 - P4   C22 = P1 + P6 + P7 + P5
//
// Every pre- and post-addition is reduced mod p as it is formed: they are
// memory-bound elementwise passes, so the reduction is free, and the block
// products then see canonical residues exactly like a plain product, with
// the same exactness bound (no growth of the intermediates to track).
// alpha is applied inside the block products (P4 with -alpha), beta where a
// block product first writes its C block (C11 <- alpha P2 + beta C11,
// C12 <- alpha P3 + beta C12, C21 <- -alpha P4 + beta C21) and in the final
// pass for C22.  Odd dimensions are peeled: the core runs on the leading
// even part, then one rank-1 product adds the last inner index and two thin
// products fill the last row and column.
#include "ffp_internal.hpp"
#include "ffp_device.hpp"

namespace ffp {

// ------------------------------------------------------------------ kernels
__device__ __forceinline__ int32_t madd(int32_t a, int32_t b, int32_t p) {
    const int32_t s = a + b;
    return s >= p ? s - p : s;
}
__device__ __forceinline__ int32_t msub(int32_t a, int32_t b, int32_t p) {
    const int32_t s = a - b;
    return s < 0 ? s + p : s;
}

struct Quad {
    const int32_t *x11, *x12, *x21, *x22;  // the operand's logical quadrants (as stored)
    int64_t ld;
};

// Pre-additions on the four stored quadrants of one operand (all rows x cols,
// row stride q.ld); outputs contiguous with row stride cols.  OPB = 0: the S
// sums of the left operand, 1: the T sums of the right operand.
template <int OPB>
__global__ __launch_bounds__(256) void k_wino_pre(int64_t rows, int64_t cols, Quad q, int32_t *__restrict__ o1,
                                                  int32_t *__restrict__ o2, int32_t *__restrict__ o3,
                                                  int32_t *__restrict__ o4, int32_t p) {
    for (int64_t i = blockIdx.y; i < rows; i += gridDim.y)
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < cols; j += (int64_t)gridDim.x * blockDim.x) {
        const int64_t s = i * q.ld + j, d = i * cols + j;
        const int32_t a11 = q.x11[s], a12 = q.x12[s], a21 = q.x21[s], a22 = q.x22[s];
        if (OPB == 0) {
            const int32_t s1 = madd(a21, a22, p), s2 = msub(s1, a11, p);
            o1[d] = s1;
            o2[d] = s2;
            o3[d] = msub(a11, a21, p);
            o4[d] = msub(a12, s2, p);
        } else {
            const int32_t t1 = msub(a12, a11, p), t2 = msub(a22, t1, p);
            o1[d] = t1;
            o2[d] = t2;
            o3[d] = msub(a22, a12, p);
            o4[d] = msub(t2, a21, p);
        }
    }
}

// Post-additions: q1 = alpha P1, q5 = alpha P5, q6 = alpha P6, q7 = alpha P7
// (contiguous, row stride cols); the C blocks already hold C11 = alpha P2 +
// beta C11, C12 = alpha P3 + beta C12, C21 = -alpha P4 + beta C21.
__global__ __launch_bounds__(256) void k_wino_post(int64_t rows, int64_t cols, const int32_t *__restrict__ q1,
                                                   const int32_t *__restrict__ q5, const int32_t *__restrict__ q6,
                                                   const int32_t *__restrict__ q7, int32_t *__restrict__ c11,
                                                   int32_t *__restrict__ c12, int32_t *__restrict__ c21,
                                                   int32_t *__restrict__ c22, int64_t ldc, double beta, double pd,
                                                   double pinv) {
    const int32_t p = (int32_t)pd;
    for (int64_t i = blockIdx.y; i < rows; i += gridDim.y)
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < cols; j += (int64_t)gridDim.x * blockDim.x) {
        const int64_t s = i * cols + j, d = i * ldc + j;
        const int32_t p1 = q1[s], p5 = q5[s];
        const int32_t u2 = madd(p1, q6[s], p), u3 = madd(u2, q7[s], p);
        c11[d] = madd(c11[d], p1, p);
        c12[d] = madd(c12[d], madd(u2, p5, p), p);
        c21[d] = madd(c21[d], u3, p);
        int32_t c = madd(u3, p5, p);
        if (beta != 0.0) {
            const int32_t old = c22[d];
            const int32_t bc = beta == 1.0 ? old : (int32_t)mod_canon(beta * (double)old, pd, pinv);
            c = madd(c, bc, p);
        }
        c22[d] = c;
    }
}

static dim3 ew_grid(int64_t rows, int64_t cols) {
    const int64_t gx = (cols + 255) / 256;
    return dim3((unsigned)(gx < 16 ? gx : 16), (unsigned)(rows < 65535 ? rows : 65535));
}

// ------------------------------------------------------------------ host side
static bool wino_splits(int levels, int64_t m, int64_t n, int64_t k) { return levels > 0 && m >= 2 && n >= 2 && k >= 2; }

static size_t base_ws(int path, const Field &F, int64_t m, int64_t n, int64_t k) {
    const int eff = resolve_path(path, F.p, m, n, k);
    if (eff != FFP_PATH_INT8 || F.limbs == 0) return 0;
    return fgemm_i8_ws(F, m, n, k) + fgemm_i8_split_ws(m, n) + 256;
}

size_t fgemm_wino_ws(int path, const Field &F, int levels, int64_t m, int64_t n, int64_t k) {
    if (!wino_splits(levels, m, n, k)) return base_ws(path, F, m, n, k);
    const int64_t hm = m / 2, hn = n / 2, hk = k / 2;
    const size_t temps = 4 * ((size_t)hm * hk + (size_t)hk * hn + (size_t)hm * hn) * 4 + 12 * 256;
    size_t child = fgemm_wino_ws(path, F, levels - 1, hm, hn, hk);
    // peeled last row / column / inner index (run after the temporaries are released)
    size_t peel = base_ws(path, F, 2 * hm, 2 * hn, 1);
    const size_t r = base_ws(path, F, 1, n, k), c = base_ws(path, F, 2 * hm, 1, k);
    peel = peel > r ? peel : r;
    peel = peel > c ? peel : c;
    return (temps + child > peel ? temps + child : peel) + 256;
}

int fgemm_wino(int path, const Field &F, int levels, int ta, int tb, int64_t m, int64_t n, int64_t k,
               uint32_t alpha, const int32_t *A, int64_t lda, const int32_t *B, int64_t ldb, uint32_t beta,
               int32_t *C, int64_t ldc, Arena &ws, hipStream_t s) {
    if (m <= 0 || n <= 0) return FFP_OK;
    if (!wino_splits(levels, m, n, k))
        return fgemm_any(resolve_path(path, F.p, m, n, k), F, ta, tb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc,
                         ws, s);
    const int64_t hm = m / 2, hn = n / 2, hk = k / 2;
    // logical quadrant (i, j) of op(A) / op(B), as stored
    auto qa = [&](int i, int j) { return ta ? A + (j * hk) * lda + i * hm : A + (i * hm) * lda + j * hk; };
    auto qb = [&](int i, int j) { return tb ? B + (j * hn) * ldb + i * hk : B + (i * hk) * ldb + j * hn; };
    // stored shapes of the quadrants and of their sums
    const int64_t ar = ta ? hk : hm, ac = ta ? hm : hk, br = tb ? hn : hk, bc = tb ? hk : hn;
    const size_t mk = ws.mark();
    int32_t *S[4], *T[4], *Q[4];
    for (auto &x : S) x = (int32_t *)ws.take((size_t)hm * hk * 4);
    for (auto &x : T) x = (int32_t *)ws.take((size_t)hk * hn * 4);
    for (auto &x : Q) x = (int32_t *)ws.take((size_t)hm * hn * 4);
    for (int i = 0; i < 4; ++i)
        if (!S[i] || !T[i] || !Q[i]) return FFP_E_WORKSPACE;
    {
        ProfScope prof(PK_WINOGRAD, 0.0, s, 32.0 * ((double)hm * hk + (double)hk * hn));
        const Quad qA{qa(0, 0), qa(0, 1), qa(1, 0), qa(1, 1), lda};
        const Quad qB{qb(0, 0), qb(0, 1), qb(1, 0), qb(1, 1), ldb};
        hipLaunchKernelGGL(k_wino_pre<0>, ew_grid(ar, ac), dim3(256), 0, s, ar, ac, qA, S[0], S[1], S[2], S[3],
                           (int32_t)F.p);
        hipLaunchKernelGGL(k_wino_pre<1>, ew_grid(br, bc), dim3(256), 0, s, br, bc, qB, T[0], T[1], T[2], T[3],
                           (int32_t)F.p);
        FFP_HIP_CHECK(hipGetLastError());
    }
    const int64_t lS = ac, lT = bc;  // row strides of the stored sums
    const uint32_t nalpha = alpha == 0 ? 0 : F.p - alpha;
    int32_t *C11 = C, *C12 = C + hn, *C21 = C + hm * ldc, *C22 = C + hm * ldc + hn;
    const int L1 = levels - 1;
    // Q1 = alpha P1, C11 = alpha P2 + beta C11
    FFP_CHECK(fgemm_wino(path, F, L1, ta, tb, hm, hn, hk, alpha, qa(0, 0), lda, qb(0, 0), ldb, 0, Q[0], hn, ws, s));
    FFP_CHECK(fgemm_wino(path, F, L1, ta, tb, hm, hn, hk, alpha, qa(0, 1), lda, qb(1, 0), ldb, beta, C11, ldc, ws, s));
    // Q5 = alpha S1 T1, Q6 = alpha S2 T2, Q7 = alpha S3 T3
    FFP_CHECK(fgemm_wino(path, F, L1, ta, tb, hm, hn, hk, alpha, S[0], lS, T[0], lT, 0, Q[1], hn, ws, s));
    FFP_CHECK(fgemm_wino(path, F, L1, ta, tb, hm, hn, hk, alpha, S[1], lS, T[1], lT, 0, Q[2], hn, ws, s));
    FFP_CHECK(fgemm_wino(path, F, L1, ta, tb, hm, hn, hk, alpha, S[2], lS, T[2], lT, 0, Q[3], hn, ws, s));
    // C12 = alpha S4 B22 + beta C12, C21 = -alpha A22 T4 + beta C21
    FFP_CHECK(fgemm_wino(path, F, L1, ta, tb, hm, hn, hk, alpha, S[3], lS, qb(1, 1), ldb, beta, C12, ldc, ws, s));
    FFP_CHECK(fgemm_wino(path, F, L1, ta, tb, hm, hn, hk, nalpha, qa(1, 1), lda, T[3], lT, beta, C21, ldc, ws, s));
    {
        ProfScope prof(PK_WINOGRAD, 0.0, s, 4.0 * (double)hm * hn * (beta != 0 ? 12.0 : 11.0));
        hipLaunchKernelGGL(k_wino_post, ew_grid(hm, hn), dim3(256), 0, s, hm, hn, Q[0], Q[1], Q[2], Q[3], C11, C12,
                           C21, C22, ldc, (double)beta, F.pd, F.pinv);
        FFP_HIP_CHECK(hipGetLastError());
    }
    ws.release(mk);
    // peeling of odd dimensions
    const int64_t mm = 2 * hm, nn = 2 * hn, kk = 2 * hk;
    if (k > kk) {
        const int32_t *Acol = ta ? A + kk * lda : A + kk;
        const int32_t *Brow = tb ? B + kk : B + kk * ldb;
        FFP_CHECK(fgemm_any(resolve_path(path, F.p, mm, nn, 1), F, ta, tb, mm, nn, 1, alpha, Acol, lda, Brow, ldb, 1,
                            C, ldc, ws, s));
    }
    if (m > mm) {
        const int32_t *Arow = ta ? A + mm : A + mm * lda;
        FFP_CHECK(fgemm_any(resolve_path(path, F.p, 1, n, k), F, ta, tb, 1, n, k, alpha, Arow, lda, B, ldb, beta,
                            C + mm * ldc, ldc, ws, s));
    }
    if (n > nn) {
        const int32_t *Bcol = tb ? B + nn * ldb : B + nn;
        FFP_CHECK(fgemm_any(resolve_path(path, F.p, mm, 1, k), F, ta, tb, mm, 1, k, alpha, A, lda, Bcol, ldb, beta,
                            C + nn, ldc, ws, s));
    }
    return FFP_OK;
}

// Levels taken by FFP_WINO_AUTO: one level per halving while the block
// products stay at least `min_dim` in every dimension, where min_dim is the
// measured size below which a level no longer pays on MI355X.  Measured
// (whole call, ms; levels 0 / 1 / 2 / 3): FP64 8192^3 18.6 / 16.8 / 18.1 /
// 24.6, 16384^3 148 / 131 / 119 / 128; INT8 with 3 limbs 8192^3 4.37 / 4.16
// / 5.00 / 13.6, 16384^3 31.9 / 29.6 / 29.8 / 36.5.  With one limb the
// product is so cheap that the additions never pay (16384^3: 6.96 / 7.88 /
// 10.5 ms), so that path takes no level.
int wino_auto_levels(int path, const Field &F, int64_t m, int64_t n, int64_t k) {
    const int eff = resolve_path(path, F.p, m, n, k);
    if (eff == FFP_PATH_INT8 && F.limbs == 1) return 0;
    const int64_t min_dim = eff == FFP_PATH_INT8 ? kWinoMinDimI8 : kWinoMinDimF64;
    int lv = 0;
    int64_t a = m, b = n, c = k;
    while (lv < 4 && a / 2 >= min_dim && b / 2 >= min_dim && c / 2 >= min_dim) {
        a /= 2;
        b /= 2;
        c /= 2;
        ++lv;
    }
    return lv;
}

}  // namespace ffp
