// Echelon forms and the other consumers of a rank-profile-revealing PLUQ
// (Section 1, "Pivoting strategies and rank deficiencies": only pivoting
// strategies that reveal the rank profile reveal the echelon form, which is
// what Gaussian elimination is used for in Groebner-basis and number-theory
// codes).  Everything here starts from the output of ffp_pluq,
// A = P [L1; L2] [U1 U2] Q with L1, U1 r x r, and runs on the library's own
// triangular solves, products and permutations:
//
//   row echelon form (reduced):    R = Pi^T [I  U1^-1 U2] Q      (r x n)
//   column echelon form (reduced): C = P [I; L2 L1^-1] Pi'^T     (m x r)
//   right nullspace:               N = Q^T [-U1^-1 U2; I]        (n x (n - r))
//   left nullspace:                N = [-L2 L1^-1  I] P^T        ((m - r) x m)
//   solve A X = B:                 Y = L1^-1 (P^T B)[0:r], consistent iff
//                                  (P^T B)[r:m] = L2 Y, X = Q^T [U1^-1 Y; 0]
//
// where Pi (Pi') sorts the pivot columns (rows): the rows of R follow the
// ascending column rank profile and the columns of C the ascending row rank
// profile.  Since the pivots of ffp_pluq are the rank profile matrix, the
// pivot columns are the column rank profile and [I X] Q is the unique
// reduced row echelon form of A; the nullspace bases are the unique ones
// that are the identity on the non-pivot columns (rows), and the solution
// is the unique one that vanishes off the pivot columns.
#include "ffp_internal.hpp"

namespace ffp {

namespace {
PermSpec idx_perm(const int32_t *idx) {
    PermSpec ps;
    ps.idx = idx;
    return ps;
}

__global__ void k_inv_index(const int32_t *__restrict__ perm, int64_t n, int32_t *__restrict__ inv) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        inv[perm[i]] = (int32_t)i;
}

// out[t] = inv[sel[t]] (positions of the sorted pivot indices)
__global__ void k_gather_index(const int32_t *__restrict__ inv, const int32_t *__restrict__ sel, int64_t r,
                               int32_t *__restrict__ out) {
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < r; t += (int64_t)gridDim.x * blockDim.x)
        out[t] = inv[sel[t]];
}

// rows x cols block: the identity block at column offset c0 (value 1 where
// j - c0 == i), zero elsewhere
__global__ void k_eye(int64_t rows, int64_t cols, int64_t c0, int32_t *__restrict__ D, int64_t ldd) {
    for (int64_t i = blockIdx.y; i < rows; i += gridDim.y)
        for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < cols; j += (int64_t)gridDim.x * blockDim.x)
            D[i * ldd + j] = (j - c0 == i) ? 1 : 0;
}

// consistent[j] = 1 iff column j of the (m - r) x nrhs residual is zero
__global__ void k_fill_int(int32_t *v, int64_t n, int32_t x) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) v[i] = x;
}
__global__ void k_mark_inconsistent(int64_t rows, int64_t nrhs, const int32_t *__restrict__ Rz, int64_t ldr,
                                    int32_t *__restrict__ ok) {
    for (int64_t i = blockIdx.y; i < rows; i += gridDim.y)
        for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < nrhs; j += (int64_t)gridDim.x * blockDim.x)
            if (Rz[i * ldr + j] != 0) ok[j] = 0;  // every writer stores the same value
}

// X[c][j] = Z[qinv[c]][j] when qinv[c] < r and column j is consistent, else 0
__global__ void k_solve_scatter(int64_t n, int64_t nrhs, int64_t r, const int32_t *__restrict__ qinv,
                                const int32_t *__restrict__ Z, int64_t ldz, const int32_t *__restrict__ ok,
                                int32_t *__restrict__ X, int64_t ldx) {
    for (int64_t c = blockIdx.y; c < n; c += gridDim.y) {
        const int64_t i = qinv[c];
        for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < nrhs; j += (int64_t)gridDim.x * blockDim.x)
            X[c * ldx + j] = (i < r && ok[j]) ? Z[i * ldz + j] : 0;
    }
}

dim3 grid2(int64_t rows, int64_t cols) {
    const int64_t gx = (cols + 255) / 256;
    return dim3((unsigned)(gx < 16 ? (gx > 0 ? gx : 1) : 16), (unsigned)(rows < 65535 ? (rows > 0 ? rows : 1) : 65535));
}
unsigned grid1(int64_t n) { return (unsigned)((n + 255) / 256 < 1024 ? ((n + 255) / 256 > 0 ? (n + 255) / 256 : 1) : 1024); }

// inverse of a length-len index vector, into the arena
int32_t *inverse_of(const int32_t *perm, int64_t len, Arena &ws, hipStream_t s) {
    int32_t *inv = (int32_t *)ws.take((size_t)(len > 0 ? len : 1) * 4);
    if (!inv || ws.counting || len <= 0) return inv;
    hipLaunchKernelGGL(k_inv_index, dim3(grid1(len)), dim3(256), 0, s, perm, len, inv);
    return inv;
}

// positions (in the factorisation's order) of the ascending pivot indices:
// out[t] = inv[sorted(idx[0:r])[t]]
int32_t *sorted_positions(int64_t len, const int32_t *idx, const int32_t *inv, int64_t r, bool rows, Arena &ws,
                          hipStream_t s) {
    int32_t *sorted = (int32_t *)ws.take((size_t)(r > 0 ? r : 1) * 4);
    int32_t *out = (int32_t *)ws.take((size_t)(r > 0 ? r : 1) * 4);
    if (ws.counting) {
        // rank_profiles' own flag buffer
        const size_t mk = ws.mark();
        ws.take((size_t)(len > 0 ? len : 1));
        ws.release(mk);
        return out;
    }
    if (!sorted || !out || r <= 0) return out;
    // rank_profiles sorts the first r entries of its index vector(s)
    if (rows) {
        if (rank_profiles(len, 1, idx, nullptr, r, sorted, nullptr, ws, s) != FFP_OK) return nullptr;
    } else {
        if (rank_profiles(1, len, nullptr, idx, r, nullptr, sorted, ws, s) != FFP_OK) return nullptr;
    }
    hipLaunchKernelGGL(k_gather_index, dim3(grid1(r)), dim3(256), 0, s, inv, sorted, r, out);
    return out;
}

// rows x cols identity-at-offset block (skipped when counting)
void eye(int64_t rows, int64_t cols, int64_t c0, int32_t *D, int64_t ldd, const Arena &ws, hipStream_t s) {
    if (ws.counting || rows <= 0 || cols <= 0) return;
    hipLaunchKernelGGL(k_eye, grid2(rows, cols), dim3(256), 0, s, rows, cols, c0, D, ldd);
}
}  // namespace

// X = alpha U1^-1 U2 (r x (n - r), row stride ldx) from the in-place factors
static int upper_solve(int path, const Field &F, int64_t n, const int32_t *LU, int64_t ld, int64_t r, uint32_t alpha,
                       int32_t *X, int64_t ldx, Arena &ws, hipStream_t s) {
    if (r <= 0 || n - r <= 0) return FFP_OK;
    path = resolve_path(path, F.p, r / 2, n - r, r / 2);
    if (!ws.counting) FFP_CHECK(copy2d(r, n - r, LU + r, ld, X, ldx, s));
    return ftrsm_run(path, F, 0, 1, 0, 0, r, n - r, alpha, LU, ld, X, ldx, ws, s);
}

// Y = alpha L2 L1^-1 ((m - r) x r, row stride ldy)
static int lower_solve(int path, const Field &F, int64_t m, const int32_t *LU, int64_t ld, int64_t r, uint32_t alpha,
                       int32_t *Y, int64_t ldy, Arena &ws, hipStream_t s) {
    if (r <= 0 || m - r <= 0) return FFP_OK;
    path = resolve_path(path, F.p, r / 2, m - r, r / 2);
    if (!ws.counting) FFP_CHECK(copy2d(m - r, r, LU + r * ld, ld, Y, ldy, s));
    return ftrsm_run(path, F, 1, 0, 0, 1, m - r, r, alpha, LU, ld, Y, ldy, ws, s);
}

int echelon_run(int form, int path, const Field &F, int64_t m, int64_t n, const int32_t *LU, int64_t ld,
                const int32_t *P, const int32_t *Q, int64_t r, int32_t *E, int64_t lde, Arena &ws, hipStream_t s) {
    if (r <= 0) return FFP_OK;
    const size_t mk = ws.mark();
    if (form == 0) {
        // W = [I X] (r x n), X = U1^-1 U2; E[t][c] = W[pi[t]][qinv[c]]
        int32_t *W = (int32_t *)ws.take((size_t)r * n * 4);
        if (!W && !ws.counting) return FFP_E_WORKSPACE;
        eye(r, r, 0, W, n, ws, s);
        FFP_CHECK(upper_solve(path, F, n, LU, ld, r, 1, W + r, n, ws, s));
        int32_t *qinv = inverse_of(Q, n, ws, s);
        int32_t *pi = sorted_positions(n, Q, qinv, r, false, ws, s);
        if (ws.counting) { ws.release(mk); return FFP_OK; }
        if (!qinv || !pi) return FFP_E_WORKSPACE;
        FFP_CHECK(permute_copy(r, n, W, n, E, lde, idx_perm(pi), idx_perm(qinv), s));
    } else {
        // V = [I; Y] (m x r), Y = L2 L1^-1; E[x][t] = V[pinv[x]][pi'[t]]
        int32_t *V = (int32_t *)ws.take((size_t)m * r * 4);
        if (!V && !ws.counting) return FFP_E_WORKSPACE;
        eye(r, r, 0, V, r, ws, s);
        FFP_CHECK(lower_solve(path, F, m, LU, ld, r, 1, V + r * r, r, ws, s));
        int32_t *pinv = inverse_of(P, m, ws, s);
        int32_t *pi = sorted_positions(m, P, pinv, r, true, ws, s);
        if (ws.counting) { ws.release(mk); return FFP_OK; }
        if (!pinv || !pi) return FFP_E_WORKSPACE;
        FFP_CHECK(permute_copy(m, r, V, r, E, lde, idx_perm(pinv), idx_perm(pi), s));
    }
    FFP_HIP_CHECK(hipGetLastError());
    ws.release(mk);
    return FFP_OK;
}

int nullspace_run(int side, int path, const Field &F, int64_t m, int64_t n, const int32_t *LU, int64_t ld,
                  const int32_t *P, const int32_t *Q, int64_t r, int32_t *N, int64_t ldn, Arena &ws, hipStream_t s) {
    const uint32_t neg1 = F.p - 1;
    const size_t mk = ws.mark();
    if (side == 0) {
        // Z = [-X; I] (n x d), N[c][j] = Z[qinv[c]][j]
        const int64_t d = n - r;
        if (d <= 0) return FFP_OK;
        int32_t *Z = (int32_t *)ws.take((size_t)n * d * 4);
        if (!Z && !ws.counting) return FFP_E_WORKSPACE;
        eye(d, d, 0, ws.counting ? nullptr : Z + r * d, d, ws, s);
        FFP_CHECK(upper_solve(path, F, n, LU, ld, r, neg1, Z, d, ws, s));
        int32_t *qinv = inverse_of(Q, n, ws, s);
        if (ws.counting) { ws.release(mk); return FFP_OK; }
        if (!qinv) return FFP_E_WORKSPACE;
        FFP_CHECK(permute_copy(n, d, Z, d, N, ldn, idx_perm(qinv), PermSpec(), s));
    } else {
        // Z = [-Y I] (d x m), N[j][x] = Z[j][pinv[x]]
        const int64_t d = m - r;
        if (d <= 0) return FFP_OK;
        int32_t *Z = (int32_t *)ws.take((size_t)d * m * 4);
        if (!Z && !ws.counting) return FFP_E_WORKSPACE;
        eye(d, d, 0, ws.counting ? nullptr : Z + r, m, ws, s);
        FFP_CHECK(lower_solve(path, F, m, LU, ld, r, neg1, Z, m, ws, s));
        int32_t *pinv = inverse_of(P, m, ws, s);
        if (ws.counting) { ws.release(mk); return FFP_OK; }
        if (!pinv) return FFP_E_WORKSPACE;
        FFP_CHECK(permute_copy(d, m, Z, m, N, ldn, PermSpec(), idx_perm(pinv), s));
    }
    FFP_HIP_CHECK(hipGetLastError());
    ws.release(mk);
    return FFP_OK;
}

int solve_run(int path, const Field &F, int64_t m, int64_t n, const int32_t *LU, int64_t ld, const int32_t *P,
              const int32_t *Q, int64_t r, int64_t nrhs, const int32_t *B, int64_t ldb, int32_t *X, int64_t ldx,
              int32_t *ok, Arena &ws, hipStream_t s) {
    if (nrhs <= 0) return FFP_OK;
    const size_t mk = ws.mark();
    int32_t *Y = (int32_t *)ws.take((size_t)(m > 0 ? m : 1) * nrhs * 4);
    int32_t *qinv = inverse_of(Q, n, ws, s);
    if (!ws.counting) {
        if (!Y || !qinv) return FFP_E_WORKSPACE;
        hipLaunchKernelGGL(k_fill_int, dim3(grid1(nrhs)), dim3(256), 0, s, ok, nrhs, 1);
        // Y = P^T B
        if (m > 0) FFP_CHECK(permute_copy(m, nrhs, B, ldb, Y, nrhs, idx_perm(P), PermSpec(), s));
    }
    if (r > 0) {
        const int tpath = resolve_path(path, F.p, r / 2, nrhs, r / 2);
        // Y[0:r] <- L1^-1 Y[0:r]
        FFP_CHECK(ftrsm_run(tpath, F, 0, 0, 0, 1, r, nrhs, 1, LU, ld, Y, nrhs, ws, s));
        // Y[r:m] <- Y[r:m] - L2 Y[0:r]: the residual of the equations below the pivots
        if (m > r)
            FFP_CHECK(fgemm_any(resolve_path(path, F.p, m - r, nrhs, r), F, 0, 0, m - r, nrhs, r, F.p - 1,
                                LU + r * ld, ld, Y, nrhs, 1, ws.counting ? nullptr : Y + r * nrhs, nrhs, ws, s));
        // Y[0:r] <- U1^-1 Y[0:r]
        FFP_CHECK(ftrsm_run(tpath, F, 0, 1, 0, 0, r, nrhs, 1, LU, ld, Y, nrhs, ws, s));
    }
    if (ws.counting) { ws.release(mk); return FFP_OK; }
    if (m > r)
        hipLaunchKernelGGL(k_mark_inconsistent, grid2(m - r, nrhs), dim3(256), 0, s, m - r, nrhs, Y + r * nrhs, nrhs,
                           ok);
    if (n > 0)
        hipLaunchKernelGGL(k_solve_scatter, grid2(n, nrhs), dim3(256), 0, s, n, nrhs, r, qinv, Y, nrhs, ok, X, ldx);
    FFP_HIP_CHECK(hipGetLastError());
    ws.release(mk);
    return FFP_OK;
}

}  // namespace ffp
