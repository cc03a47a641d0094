/*
 * Plain CPU oracle for exact linear algebra over Z/pZ: the modular matrix
 * product, the triangular solve, the row/column permutation and the
 * rank-profile-revealing PLUQ factorisation.
 *
 * TEST INFRASTRUCTURE.  This file is the independent checker of the GPU
 * library: only the test-suite, the smoke check and the benchmark's
 * CPU-baseline leg load it.  It shares no code, header, table or helper with
 * the GPU path, and the GPU path never calls it.
 *
 * Everything is computed the slow, obvious way: int64 (or wider) integers,
 * every intermediate reduced to the canonical representative in [0, p),
 * no blocking and no delayed reduction.  The only concession to size is an
 * OpenMP loop over independent rows inside each rank-one update.
 *
 * Paper: J-G. Dumas, T. Gautier, C. Pernet, Z. Sultan, "Parallel computation
 * of echelon forms" (arXiv:1402.3501).  Section 2.1 defines the four
 * routines (gemm, trsm, laswp, getrf with A = PLUQ, L and U in place);
 * Section 4.1 ("Pivoting strategies") defines the row-major pivot search and
 * the four-quadrant tile recursion whose pivot order this oracle reproduces.
 *
 * Parity status of each function is stated in its header comment.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OK 0
#define ORC_E_ARG -1
#define ORC_E_NOTPRIME -2
#define ORC_E_RANGE -3
#define ORC_E_SINGULAR -4   /* zero diagonal entry in a non-unit triangle */
#define ORC_E_CONVENTION -5 /* pivot order does not yield an LU (see pluq) */
#define ORC_E_SELFCHECK -6
#define ORC_E_NOMEM -7

/* ------------------------------------------------------------------ */
/* Scalar arithmetic: canonical floor-mod, product, inverse, primality */
/* ------------------------------------------------------------------ */

static inline int64_t md(int64_t a, int64_t p) {
    int64_t r = a % p;
    return r < 0 ? r + p : r;
}

/* a*b mod p for |a|, |b| < 2^31 (the product fits in int64). */
static inline int64_t mulmod(int64_t a, int64_t b, int64_t p) {
    return md(a * b, p);
}

/* Inverse of a (a != 0 mod p) by the extended Euclidean algorithm. */
int64_t orc_inv(int64_t a, int64_t p) {
    int64_t r0 = p, r1 = md(a, p), s0 = 0, s1 = 1;
    if (r1 == 0) return 0;
    while (r1 != 0) {
        int64_t q = r0 / r1, t;
        t = r0 - q * r1; r0 = r1; r1 = t;
        t = s0 - q * s1; s0 = s1; s1 = t;
    }
    return r0 == 1 ? md(s0, p) : 0;
}

static uint64_t powmod_u64(uint64_t b, uint64_t e, uint64_t m) {
    unsigned __int128 r = 1, x = b % m;
    while (e) {
        if (e & 1) r = (r * x) % m;
        x = (x * x) % m;
        e >>= 1;
    }
    return (uint64_t)r;
}

/* Deterministic Miller-Rabin for 32-bit integers (bases 2, 7, 61 cover all
 * n < 4,759,123,141). */
int orc_is_prime(uint64_t n) {
    if (n < 2) return 0;
    static const uint64_t small[] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
    for (int i = 0; i < 12; i++) {
        if (n == small[i]) return 1;
        if (n % small[i] == 0) return 0;
    }
    uint64_t d = n - 1; int s = 0;
    while ((d & 1) == 0) { d >>= 1; s++; }
    static const uint64_t bases[] = {2, 7, 61};
    for (int i = 0; i < 3; i++) {
        uint64_t a = bases[i] % n;
        if (a == 0) continue;
        uint64_t x = powmod_u64(a, d, n);
        if (x == 1 || x == n - 1) continue;
        int comp = 1;
        for (int r = 1; r < s; r++) {
            x = (uint64_t)(((unsigned __int128)x * x) % n);
            if (x == n - 1) { comp = 0; break; }
        }
        if (comp) return 0;
    }
    return 1;
}

static int check_field(uint32_t p) {
    if (p < 2 || p > 0x7fffffffu) return ORC_E_ARG;
    return orc_is_prime(p) ? ORC_OK : ORC_E_NOTPRIME;
}

static int check_entries(int64_t m, int64_t n, const int32_t *A, int64_t lda, uint32_t p) {
    for (int64_t i = 0; i < m; i++)
        for (int64_t j = 0; j < n; j++) {
            int32_t v = A[i * lda + j];
            if (v < 0 || (uint32_t)v >= p) return ORC_E_RANGE;
        }
    return ORC_OK;
}

int orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_threads(int t) {
#ifdef _OPENMP
    if (t > 0) omp_set_num_threads(t);
#else
    (void)t;
#endif
}

/* ------------------------------------------------------------------ */
/* gemm over Z/pZ (Section 2.1): C <- alpha*op(A)*op(B) + beta*C.       */
/* Plain definition: every product reduced, every sum reduced.          */
/* Pinned in tests by Python big-integer products.                      */
/* ------------------------------------------------------------------ */
int orc_fgemm(int transA, int transB, int64_t m, int64_t n, int64_t k, uint32_t p,
              uint32_t alpha, const int32_t *A, int64_t lda, const int32_t *B, int64_t ldb,
              uint32_t beta, int32_t *C, int64_t ldc) {
    int e = check_field(p);
    if (e) return e;
    if (m < 0 || n < 0 || k < 0 || alpha >= p || beta >= p) return ORC_E_ARG;
    const int64_t P = p;
#pragma omp parallel for schedule(dynamic, 4) if (m * n * k > (1 << 22))
    for (int64_t i = 0; i < m; i++) {
        for (int64_t j = 0; j < n; j++) {
            int64_t s = 0;
            for (int64_t t = 0; t < k; t++) {
                int64_t a = transA ? A[t * lda + i] : A[i * lda + t];
                int64_t b = transB ? B[j * ldb + t] : B[t * ldb + j];
                s = md(s + mulmod(a, b, P), P);
            }
            int64_t c = C[i * ldc + j];
            C[i * ldc + j] = (int32_t)md(mulmod(alpha, s, P) + mulmod(beta, md(c, P), P), P);
        }
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* trsm over Z/pZ (Section 2.1): solve with a triangular matrix.        */
/*   side 0: B <- alpha * op(T)^-1 * B   (T is m x m)                   */
/*   side 1: B <- alpha * B * op(T)^-1   (T is n x n)                   */
/*   uplo 0 lower / 1 upper, trans 0 op(T)=T / 1 op(T)=T^T,             */
/*   diag 0 non-unit / 1 unit (diagonal of T not read).                 */
/* Plain forward / back substitution with exact inverses.               */
/* Pinned in tests by the residual op(T)*X == alpha*B.                  */
/* ------------------------------------------------------------------ */
int orc_ftrsm(int side, int uplo, int trans, int diag, int64_t m, int64_t n, uint32_t p,
              uint32_t alpha, const int32_t *T, int64_t ldt, int32_t *B, int64_t ldb) {
    int e = check_field(p);
    if (e) return e;
    if (m < 0 || n < 0 || alpha >= p) return ORC_E_ARG;
    const int64_t P = p;
    const int64_t d = side == 0 ? m : n;
    /* effective triangle after transposition: op(T)[i][j] */
    const int lower = (uplo == 0) ^ (trans != 0);
    int64_t *dinv = (int64_t *)malloc(sizeof(int64_t) * (d ? d : 1));
    if (!dinv) return ORC_E_NOMEM;
    for (int64_t i = 0; i < d; i++) {
        if (diag) { dinv[i] = 1; continue; }
        int64_t t = T[i * ldt + i];
        if (md(t, P) == 0) { free(dinv); return ORC_E_SINGULAR; }
        dinv[i] = orc_inv(t, P);
    }
#define OPT(i, j) ((int64_t)(trans ? T[(j) * ldt + (i)] : T[(i) * ldt + (j)]))
    if (side == 0) {
        /* columns of B are independent: solve op(T) x = alpha b per column */
#pragma omp parallel for schedule(dynamic, 8) if (m * m * n > (1 << 22))
        for (int64_t c = 0; c < n; c++) {
            for (int64_t s = 0; s < m; s++) {
                int64_t i = lower ? s : m - 1 - s;
                int64_t acc = mulmod(alpha, B[i * ldb + c], P);
                if (lower)
                    for (int64_t t = 0; t < i; t++)
                        acc = md(acc - mulmod(OPT(i, t), B[t * ldb + c], P), P);
                else
                    for (int64_t t = i + 1; t < m; t++)
                        acc = md(acc - mulmod(OPT(i, t), B[t * ldb + c], P), P);
                B[i * ldb + c] = (int32_t)mulmod(acc, dinv[i], P);
            }
        }
    } else {
        /* rows of B are independent: solve x op(T) = alpha b per row */
#pragma omp parallel for schedule(dynamic, 8) if (m * n * n > (1 << 22))
        for (int64_t r = 0; r < m; r++) {
            for (int64_t s = 0; s < n; s++) {
                /* x_j depends on x_t for t<j if op(T) upper, t>j if lower */
                int64_t j = lower ? n - 1 - s : s;
                int64_t acc = mulmod(alpha, B[r * ldb + j], P);
                if (lower)
                    for (int64_t t = j + 1; t < n; t++)
                        acc = md(acc - mulmod(B[r * ldb + t], OPT(t, j), P), P);
                else
                    for (int64_t t = 0; t < j; t++)
                        acc = md(acc - mulmod(B[r * ldb + t], OPT(t, j), P), P);
                B[r * ldb + j] = (int32_t)mulmod(acc, dinv[j], P);
            }
        }
    }
#undef OPT
    free(dinv);
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Pass 1 -- pivot discovery by the row-major search of Section 4.1:    */
/* rows are visited in order; a row whose remaining part is zero is     */
/* skipped, otherwise its leftmost nonzero not yet in a pivot column    */
/* becomes the next pivot and is eliminated from all later rows.        */
/* Because non-pivot rows and columns keep their relative order (the    */
/* permutations are rotations), "current position" equals "original    */
/* index among the remaining ones", so the search runs in place.        */
/* Output: pivot pairs (prow[t], pcol[t]) in increasing row order;      */
/* these are the nonzero positions of the rank profile matrix R_A.      */
/* If W is non-NULL it receives the eliminated matrix (multipliers in   */
/* the pivot columns of later rows), i.e. the LU for the row-sorted     */
/* pivot order, in original positions.                                  */
/* Pinned in tests by ranks of leading blocks (minor enumeration).      */
/* ------------------------------------------------------------------ */
int orc_pivots(int64_t m, int64_t n, uint32_t p, const int32_t *A, int64_t lda,
               int32_t *prow, int32_t *pcol, int64_t *rank, int64_t *Wout) {
    int e = check_field(p);
    if (e) return e;
    if (m < 0 || n < 0) return ORC_E_ARG;
    if ((e = check_entries(m, n, A, lda, p))) return e;
    const int64_t P = p;
    int64_t *W = Wout ? Wout : (int64_t *)malloc(sizeof(int64_t) * (m > 0 && n > 0 ? m * n : 1));
    int64_t *act = (int64_t *)malloc(sizeof(int64_t) * (n ? n : 1)); /* active columns */
    if (!W || !act) { if (!Wout) free(W); free(act); return ORC_E_NOMEM; }
    for (int64_t i = 0; i < m; i++)
        for (int64_t j = 0; j < n; j++) W[i * n + j] = A[i * lda + j];
    int64_t na = n;
    for (int64_t j = 0; j < n; j++) act[j] = j;
    int64_t r = 0;
    for (int64_t x = 0; x < m && na > 0; x++) {
        int64_t q = -1;
        for (int64_t a = 0; a < na; a++)
            if (W[x * n + act[a]] != 0) { q = a; break; }
        if (q < 0) continue;
        const int64_t j = act[q];
        prow[r] = (int32_t)x; pcol[r] = (int32_t)j; r++;
        for (int64_t a = q; a + 1 < na; a++) act[a] = act[a + 1];
        na--;
        const int64_t inv = orc_inv(W[x * n + j], P);
        const int64_t *rowx = W + x * n;
#pragma omp parallel for schedule(static) if ((m - x) * na > (1 << 16))
        for (int64_t i = x + 1; i < m; i++) {
            int64_t *rowi = W + i * n;
            int64_t l = mulmod(rowi[j], inv, P);
            rowi[j] = l;
            if (l == 0) continue;
            for (int64_t a = 0; a < na; a++) {
                int64_t c = act[a];
                rowi[c] = md(rowi[c] - mulmod(l, rowx[c], P), P);
            }
        }
    }
    *rank = r;
    free(act);
    if (!Wout) free(W);
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Pivot order of the four-quadrant tile recursion (Section 4.1, tiled  */
/* recursive elimination).  Index manipulation only.                    */
/* ORDER(rows, cols) on ascending index lists:                          */
/*   empty list -> nothing; one row or one column -> the pivot of R_A   */
/*   lying in the region, if any; otherwise with m1 = |rows|/2 and      */
/*   n1 = |cols|/2 (floor):                                             */
/*     top-left     ORDER(rows[:m1], cols[:n1])                         */
/*     top-right    ORDER(rows[:m1] w/o top-left pivots, cols[n1:])     */
/*     bottom-left  ORDER(rows[m1:], cols[:n1] w/o top-left pivots)     */
/*     bottom-right ORDER(rows[m1:] w/o bottom-left pivots,             */
/*                        cols[n1:] w/o top-right pivots)               */
/* The top-right block is eliminated before the bottom-left one; the    */
/* two are independent, so only the position of the cross term depends */
/* on this choice.  Non-pivot indices keep their relative order.        */
/* This order is a convention (the paper fixes no example of it); it   */
/* is pinned in tests against a direct block implementation of the      */
/* recursion, exhaustively on small inputs.                             */
/* ------------------------------------------------------------------ */
typedef struct {
    const int32_t *pc_of_row; /* pivot column of row x, or -1 */
    const int32_t *pr_of_col; /* pivot row of column y, or -1 */
    char *rdone, *cdone;
    int32_t *orow, *ocol;
    int64_t cnt;
} order_ctx;

static int in_sorted(const int32_t *v, int64_t len, int32_t x) {
    int64_t lo = 0, hi = len;
    while (lo < hi) {
        int64_t mid = (lo + hi) / 2;
        if (v[mid] < x) lo = mid + 1; else hi = mid;
    }
    return lo < len && v[lo] == x;
}

static void emit(order_ctx *c, int32_t x, int32_t y) {
    c->orow[c->cnt] = x; c->ocol[c->cnt] = y; c->cnt++;
    c->rdone[x] = 1; c->cdone[y] = 1;
}

static int32_t *filter(const int32_t *v, int64_t len, const char *done, int64_t *outlen) {
    int32_t *o = (int32_t *)malloc(sizeof(int32_t) * (len ? len : 1));
    int64_t k = 0;
    for (int64_t i = 0; i < len; i++) if (!done[v[i]]) o[k++] = v[i];
    *outlen = k;
    return o;
}

static void order_rec(order_ctx *c, const int32_t *rows, int64_t nr, const int32_t *cols, int64_t nc) {
    if (nr == 0 || nc == 0) return;
    if (nr == 1) {
        int32_t y = c->pc_of_row[rows[0]];
        if (y >= 0 && in_sorted(cols, nc, y)) emit(c, rows[0], y);
        return;
    }
    if (nc == 1) {
        int32_t x = c->pr_of_col[cols[0]];
        if (x >= 0 && in_sorted(rows, nr, x)) emit(c, x, cols[0]);
        return;
    }
    const int64_t m1 = nr / 2, n1 = nc / 2;
    int64_t lf, lg, lhr, lhc;
    order_rec(c, rows, m1, cols, n1);                           /* top-left */
    int32_t *fr = filter(rows, m1, c->rdone, &lf);
    order_rec(c, fr, lf, cols + n1, nc - n1);                   /* top-right */
    int32_t *gc = filter(cols, n1, c->cdone, &lg);
    order_rec(c, rows + m1, nr - m1, gc, lg);                   /* bottom-left */
    int32_t *hr = filter(rows + m1, nr - m1, c->rdone, &lhr);
    int32_t *hc = filter(cols + n1, nc - n1, c->cdone, &lhc);
    order_rec(c, hr, lhr, hc, lhc);                             /* bottom-right */
    free(fr); free(gc); free(hr); free(hc);
}

/* Given the pivot pairs (any order), write the ordered pairs. Returns the
 * number of pairs emitted (equals r when the pairs form R_A). */
int64_t orc_order(int64_t m, int64_t n, int64_t r, const int32_t *prow, const int32_t *pcol,
                  int32_t *orow, int32_t *ocol) {
    int32_t *pc = (int32_t *)malloc(sizeof(int32_t) * (m ? m : 1));
    int32_t *pr = (int32_t *)malloc(sizeof(int32_t) * (n ? n : 1));
    char *rd = (char *)calloc(m ? m : 1, 1), *cd = (char *)calloc(n ? n : 1, 1);
    int32_t *rows = (int32_t *)malloc(sizeof(int32_t) * (m ? m : 1));
    int32_t *cols = (int32_t *)malloc(sizeof(int32_t) * (n ? n : 1));
    for (int64_t i = 0; i < m; i++) { pc[i] = -1; rows[i] = (int32_t)i; }
    for (int64_t j = 0; j < n; j++) { pr[j] = -1; cols[j] = (int32_t)j; }
    for (int64_t t = 0; t < r; t++) { pc[prow[t]] = pcol[t]; pr[pcol[t]] = prow[t]; }
    order_ctx c = {pc, pr, rd, cd, orow, ocol, 0};
    order_rec(&c, rows, m, cols, n);
    free(pc); free(pr); free(rd); free(cd); free(rows); free(cols);
    return c.cnt;
}

/* ------------------------------------------------------------------ */
/* getrf / PLUQ over Z/pZ (Section 2.1: (P,L,U,Q) with L and U in place */
/* of A and A = PLUQ), revealing rank, row and column rank profiles     */
/* (Section 4.1).                                                       */
/*                                                                      */
/* Output convention (in place, row-major, ld = lda):                   */
/*   P[i] = original row placed at position i, Q[j] = original column   */
/*   placed at position j, so that A[P[i]][Q[j]] = sum_t L[i][t]U[t][j]. */
/*   P = ordered pivot rows then non-pivot rows ascending; same for Q.  */
/*   Strictly lower part of columns < r: L (unit diagonal implied);     */
/*   rows < r, columns >= row: U; the block [r:, r:] is zero.           */
/*   rrp / crp: sorted pivot rows / columns (first r entries).          */
/*                                                                      */
/* Steps: pass 1 (pivot set), ORDER (pivot order), pass 2 (plain LU of  */
/* the permuted matrix with no search; a zero pivot or a nonzero Schur  */
/* complement is reported as ORC_E_CONVENTION).  When the ordered pivots */
/* coincide with the row-sorted ones, the LU of pass 1 is reused.       */
/* selfcheck: 1 = verify A == PLUQ exactly; 0 = skip.                   */
/* Pinned in tests: A == PLUQ, triangular structure, R_A against minor  */
/* enumeration, special cases (identity, permutation, zero, rank one,   */
/* generic rank profile), and a direct block recursion on small inputs. */
/* ------------------------------------------------------------------ */
int orc_pluq(int64_t m, int64_t n, uint32_t p, int32_t *A, int64_t lda, int32_t *Pout,
             int32_t *Qout, int64_t *rank, int32_t *rrp, int32_t *crp, int selfcheck) {
    int e = check_field(p);
    if (e) return e;
    if (m < 0 || n < 0 || lda < (n > 0 ? n : 0)) return ORC_E_ARG;
    if ((e = check_entries(m, n, A, lda, p))) return e;
    const int64_t P = p;
    const int64_t mn = m < n ? m : n;
    int32_t *prow = (int32_t *)malloc(sizeof(int32_t) * (mn ? mn : 1));
    int32_t *pcol = (int32_t *)malloc(sizeof(int32_t) * (mn ? mn : 1));
    int32_t *orow = (int32_t *)malloc(sizeof(int32_t) * (mn ? mn : 1));
    int32_t *ocol = (int32_t *)malloc(sizeof(int32_t) * (mn ? mn : 1));
    int64_t *W = (int64_t *)malloc(sizeof(int64_t) * (m > 0 && n > 0 ? m * n : 1));
    if (!prow || !pcol || !orow || !ocol || !W) {
        free(prow); free(pcol); free(orow); free(ocol); free(W);
        return ORC_E_NOMEM;
    }
    int64_t r = 0;
    e = orc_pivots(m, n, p, A, lda, prow, pcol, &r, W);
    if (e) goto done;
    if (orc_order(m, n, r, prow, pcol, orow, ocol) != r) { e = ORC_E_CONVENTION; goto done; }

    /* permutations: ordered pivots, then non-pivots ascending */
    {
        char *rp = (char *)calloc(m ? m : 1, 1), *cp = (char *)calloc(n ? n : 1, 1);
        for (int64_t t = 0; t < r; t++) {
            Pout[t] = orow[t]; Qout[t] = ocol[t];
            rp[orow[t]] = 1; cp[ocol[t]] = 1;
        }
        int64_t k = r;
        for (int64_t i = 0; i < m; i++) if (!rp[i]) Pout[k++] = (int32_t)i;
        k = r;
        for (int64_t j = 0; j < n; j++) if (!cp[j]) Qout[k++] = (int32_t)j;
        free(rp); free(cp);
    }
    int same = 1;
    for (int64_t t = 0; t < r; t++)
        if (orow[t] != prow[t] || ocol[t] != pcol[t]) { same = 0; break; }

    if (same) {
        /* pass-1 elimination already is the LU for this order: gather it */
        int64_t *G = (int64_t *)malloc(sizeof(int64_t) * (m > 0 && n > 0 ? m * n : 1));
        for (int64_t i = 0; i < m; i++)
            for (int64_t j = 0; j < n; j++) G[i * n + j] = W[(int64_t)Pout[i] * n + Qout[j]];
        free(W);
        W = G;
    } else {
        /* pass 2: plain LU of A[P][:,Q] in the prescribed order */
        for (int64_t i = 0; i < m; i++)
            for (int64_t j = 0; j < n; j++) W[i * n + j] = A[(int64_t)Pout[i] * lda + Qout[j]];
        for (int64_t k = 0; k < r; k++) {
            int64_t piv = W[k * n + k];
            if (piv == 0) { e = ORC_E_CONVENTION; goto done; }
            const int64_t inv = orc_inv(piv, P);
            const int64_t *rowk = W + k * n;
#pragma omp parallel for schedule(static) if ((m - k) * (n - k) > (1 << 16))
            for (int64_t i = k + 1; i < m; i++) {
                int64_t *rowi = W + i * n;
                int64_t l = mulmod(rowi[k], inv, P);
                rowi[k] = l;
                if (l == 0) continue;
                for (int64_t c = k + 1; c < n; c++) rowi[c] = md(rowi[c] - mulmod(l, rowk[c], P), P);
            }
        }
    }
    for (int64_t i = r; i < m; i++)
        for (int64_t j = r; j < n; j++)
            if (W[i * n + j] != 0) { e = ORC_E_CONVENTION; goto done; }

    if (selfcheck) {
        /* exact A[P[i]][Q[j]] == sum_{t <= min(i, j, r-1)} L[i][t] U[t][j] */
        int bad = 0;
#pragma omp parallel for schedule(dynamic, 4) reduction(| : bad) if (m * n * r > (1 << 22))
        for (int64_t i = 0; i < m; i++) {
            for (int64_t j = 0; j < n; j++) {
                int64_t lim = i < j ? i : j;
                if (lim > r - 1) lim = r - 1;
                int64_t s = 0;
                for (int64_t t = 0; t <= lim; t++) {
                    int64_t l = (t == i) ? 1 : W[i * n + t];
                    s = md(s + mulmod(l, W[t * n + j], P), P);
                }
                if (s != A[(int64_t)Pout[i] * lda + Qout[j]]) bad = 1;
            }
        }
        if (bad) { e = ORC_E_SELFCHECK; goto done; }
    }
    for (int64_t i = 0; i < m; i++)
        for (int64_t j = 0; j < n; j++) A[i * lda + j] = (int32_t)W[i * n + j];
    *rank = r;
    for (int64_t t = 0; t < r; t++) { rrp[t] = Pout[t]; crp[t] = Qout[t]; }
    /* sort the profiles (insertion into counting arrays) */
    {
        char *rm = (char *)calloc(m ? m : 1, 1), *cm = (char *)calloc(n ? n : 1, 1);
        for (int64_t t = 0; t < r; t++) { rm[rrp[t]] = 1; cm[crp[t]] = 1; }
        int64_t k = 0;
        for (int64_t i = 0; i < m; i++) if (rm[i]) rrp[k++] = (int32_t)i;
        k = 0;
        for (int64_t j = 0; j < n; j++) if (cm[j]) crp[k++] = (int32_t)j;
        free(rm); free(cm);
    }
done:
    free(prow); free(pcol); free(orow); free(ocol); free(W);
    return e;
}

/* ------------------------------------------------------------------ */
/* Echelon forms and the consumers of a rank profile (Section 1,       */
/* "Pivoting strategies and rank deficiencies": the pivoting strategies */
/* that reveal the rank profile reveal the echelon form).  All three    */
/* come from the textbook Gauss-Jordan elimination below, written out   */
/* on its own (no use of the PLUQ above).                               */
/* ------------------------------------------------------------------ */

/* Gauss-Jordan on the m x w matrix W (int64, ld w), pivoting only in the
 * first n columns: columns are visited left to right; the first row at or
 * below the current rank with a nonzero in the column is swapped up, scaled
 * to a unit pivot, and the column is cleared in every other row.  Returns
 * the rank; piv[t] receives the column of pivot t. */
static int64_t gauss_jordan(int64_t m, int64_t n, int64_t w, int64_t *W, int64_t P, int32_t *piv) {
    int64_t r = 0;
    for (int64_t c = 0; c < n && r < m; c++) {
        int64_t i0 = -1;
        for (int64_t i = r; i < m; i++)
            if (W[i * w + c] != 0) { i0 = i; break; }
        if (i0 < 0) continue;
        if (i0 != r)
            for (int64_t j = 0; j < w; j++) {
                int64_t t = W[i0 * w + j]; W[i0 * w + j] = W[r * w + j]; W[r * w + j] = t;
            }
        const int64_t inv = orc_inv(W[r * w + c], P);
        for (int64_t j = 0; j < w; j++) W[r * w + j] = mulmod(W[r * w + j], inv, P);
        const int64_t *rowr = W + r * w;
#pragma omp parallel for schedule(static) if (m * w > (1 << 16))
        for (int64_t i = 0; i < m; i++) {
            if (i == r) continue;
            int64_t *rowi = W + i * w;
            const int64_t f = rowi[c];
            if (f == 0) continue;
            for (int64_t j = 0; j < w; j++) rowi[j] = md(rowi[j] - mulmod(f, rowr[j], P), P);
        }
        piv[r++] = (int32_t)c;
    }
    return r;
}

/* Reduced row echelon form: R (m x n, ld n) receives the RREF of A (rows
 * r..m-1 zero), pivcols[0..r) its pivot columns (ascending: the column rank
 * profile).  Pinned in tests by the characterisation of the RREF: R[:,
 * pivcols] = I, the leading entry of row t in column pivcols[t], and
 * A = A[:, pivcols] R (the row spaces agree). */
int orc_rref(int64_t m, int64_t n, uint32_t p, const int32_t *A, int64_t lda, int32_t *R, int32_t *pivcols,
             int64_t *rank) {
    int e = check_field(p);
    if (e) return e;
    if (m < 0 || n < 0) return ORC_E_ARG;
    if ((e = check_entries(m, n, A, lda, p))) return e;
    int64_t *W = (int64_t *)malloc(sizeof(int64_t) * (m * n > 0 ? m * n : 1));
    if (!W) return ORC_E_NOMEM;
    for (int64_t i = 0; i < m; i++)
        for (int64_t j = 0; j < n; j++) W[i * n + j] = A[i * lda + j];
    *rank = gauss_jordan(m, n, n, W, p, pivcols);
    for (int64_t i = 0; i < m * n; i++) R[i] = (int32_t)W[i];
    free(W);
    return ORC_OK;
}

/* Right nullspace: N (n x (n - r), ld n - r) with A N = 0, one column per
 * non-pivot column f_j of the RREF (ascending): N[f_j][j] = 1, zero on the
 * other non-pivot columns, -R[t][f_j] on pivot column pivcols[t].
 * Pinned in tests by A N = 0 and N = I on the non-pivot rows (which
 * determines a basis of the kernel uniquely). */
int orc_nullspace(int64_t m, int64_t n, uint32_t p, const int32_t *A, int64_t lda, int32_t *N, int64_t *rank) {
    int e = check_field(p);
    if (e) return e;
    if (m < 0 || n < 0) return ORC_E_ARG;
    int32_t *R = (int32_t *)malloc(sizeof(int32_t) * (m * n > 0 ? m * n : 1));
    int32_t *pc = (int32_t *)malloc(sizeof(int32_t) * (n > 0 ? n : 1));
    char *isp = (char *)calloc(n > 0 ? n : 1, 1);
    if (!R || !pc || !isp) { free(R); free(pc); free(isp); return ORC_E_NOMEM; }
    int64_t r = 0;
    e = orc_rref(m, n, p, A, lda, R, pc, &r);
    if (!e) {
        const int64_t d = n - r, P = p;
        for (int64_t t = 0; t < r; t++) isp[pc[t]] = 1;
        for (int64_t i = 0; i < n * d; i++) N[i] = 0;
        int64_t j = 0;
        for (int64_t f = 0; f < n; f++) {
            if (isp[f]) continue;
            N[f * d + j] = 1;
            for (int64_t t = 0; t < r; t++) N[(int64_t)pc[t] * d + j] = (int32_t)md(-(int64_t)R[t * n + f], P);
            j++;
        }
        *rank = r;
    }
    free(R); free(pc); free(isp);
    return e;
}

/* Linear system A X = B (A m x n, B m x nrhs): Gauss-Jordan on [A | B]
 * pivoting in A's columns only.  consistent[j] = 1 when column j of B lies
 * in the column space of A (no nonzero left in rows r.. of the reduced B);
 * then X[:, j] is the solution that is zero on the non-pivot columns (X[
 * pivcols[t]][j] = reduced B[t][j]); otherwise X[:, j] = 0.
 * Pinned in tests by A X = B, X zero off the pivot columns, and
 * inconsistency exactly when rank([A b]) > rank(A). */
int orc_solve(int64_t m, int64_t n, uint32_t p, const int32_t *A, int64_t lda, int64_t nrhs, const int32_t *B,
              int64_t ldb, int32_t *X, int64_t ldx, int32_t *consistent, int64_t *rank) {
    int e = check_field(p);
    if (e) return e;
    if (m < 0 || n < 0 || nrhs < 0) return ORC_E_ARG;
    if ((e = check_entries(m, n, A, lda, p)) || (e = check_entries(m, nrhs, B, ldb, p))) return e;
    const int64_t w = n + nrhs;
    int64_t *W = (int64_t *)malloc(sizeof(int64_t) * (m * w > 0 ? m * w : 1));
    int32_t *pc = (int32_t *)malloc(sizeof(int32_t) * (n > 0 ? n : 1));
    if (!W || !pc) { free(W); free(pc); return ORC_E_NOMEM; }
    for (int64_t i = 0; i < m; i++) {
        for (int64_t j = 0; j < n; j++) W[i * w + j] = A[i * lda + j];
        for (int64_t j = 0; j < nrhs; j++) W[i * w + n + j] = B[i * ldb + j];
    }
    const int64_t r = gauss_jordan(m, n, w, W, p, pc);
    for (int64_t j = 0; j < nrhs; j++) {
        int ok = 1;
        for (int64_t i = r; i < m; i++)
            if (W[i * w + n + j] != 0) { ok = 0; break; }
        consistent[j] = ok;
        for (int64_t c = 0; c < n; c++) X[c * ldx + j] = 0;
        if (ok)
            for (int64_t t = 0; t < r; t++) X[(int64_t)pc[t] * ldx + j] = (int32_t)W[t * w + n + j];
    }
    *rank = r;
    free(W); free(pc);
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* PLUQ in the order of the row-major search itself (Section 4.1: the   */
/* pivoting of the slab algorithms, rows visited in order, a row with   */
/* no nonzero left skipped): pivots in increasing row order, each       */
/* paired with the leftmost remaining nonzero column of its row;        */
/* non-pivot rows and columns ascending.  This is exactly pass 1 above, */
/* gathered into P, Q order: A[P[i]][Q[j]] = sum_t L[i][t] U[t][j].     */
/* Pinned in tests: the pivots are R_A (minor enumeration, as pass 1),  */
/* the pivot rows ascend, A == PLUQ exactly, triangular structure.      */
/* ------------------------------------------------------------------ */
int orc_pluq_rowmajor(int64_t m, int64_t n, uint32_t p, int32_t *A, int64_t lda, int32_t *Pout, int32_t *Qout,
                      int64_t *rank, int32_t *rrp, int32_t *crp) {
    int e = check_field(p);
    if (e) return e;
    if (m < 0 || n < 0 || lda < (n > 0 ? n : 0)) return ORC_E_ARG;
    const int64_t mn = m < n ? m : n;
    int32_t *prow = (int32_t *)malloc(sizeof(int32_t) * (mn ? mn : 1));
    int32_t *pcol = (int32_t *)malloc(sizeof(int32_t) * (mn ? mn : 1));
    int64_t *W = (int64_t *)malloc(sizeof(int64_t) * (m > 0 && n > 0 ? m * n : 1));
    char *rp = (char *)calloc(m ? m : 1, 1), *cp = (char *)calloc(n ? n : 1, 1);
    if (!prow || !pcol || !W || !rp || !cp) { e = ORC_E_NOMEM; goto done; }
    int64_t r = 0;
    e = orc_pivots(m, n, p, A, lda, prow, pcol, &r, W);
    if (e) goto done;
    for (int64_t t = 0; t < r; t++) {
        Pout[t] = prow[t]; Qout[t] = pcol[t];
        rp[prow[t]] = 1; cp[pcol[t]] = 1;
    }
    {
        int64_t k = r;
        for (int64_t i = 0; i < m; i++) if (!rp[i]) Pout[k++] = (int32_t)i;
        k = r;
        for (int64_t j = 0; j < n; j++) if (!cp[j]) Qout[k++] = (int32_t)j;
    }
    for (int64_t i = 0; i < m; i++)
        for (int64_t j = 0; j < n; j++) A[i * lda + j] = (int32_t)W[(int64_t)Pout[i] * n + Qout[j]];
    *rank = r;
    {
        int64_t k = 0;
        for (int64_t i = 0; i < m; i++) if (rp[i]) rrp[k++] = (int32_t)i;
        k = 0;
        for (int64_t j = 0; j < n; j++) if (cp[j]) crp[k++] = (int32_t)j;
    }
done:
    free(prow); free(pcol); free(W); free(rp); free(cp);
    return e;
}
