// Slab-recursive PLUQ (Section 4.1, "Pivoting strategies"): the row-major
// pivot search (rows visited in order, a row with nothing left skipped,
// otherwise its leftmost remaining nonzero becomes the next pivot) turned
// into a recursion that splits the rows in halves, as in the sequential
// slab algorithm the paper cites.  Pivots come out in increasing row order,
// each paired with the leftmost remaining nonzero of its row; with
// order-preserving rotations these are the rank profile matrix, so the call
// reveals the row rank profile in the order of P and the column rank
// profile as the set of Q's first r entries.
//
// For a slab of m rows (width w), with h = m / 2:
//   1. factor the top h rows (the whole width): P1, Q1, rank r1;
//   2. permute the bottom rows' columns by Q1: [C1 C2];
//   3. E = C1 U1^-1 (triangular solve), H = C2 - E V1 (fgemm);
//   4. factor H (m - h rows, w - r1 columns): P2, Q2, rank r2;
//   5. apply Q2 to V1's columns and P2 to E's rows, and rotate the bottom
//      pivot rows up past the top non-pivot rows.
// Rows then read [top pivots | bottom pivots | top non-pivots | bottom
// non-pivots], columns [Q1 pivots | Q2 pivots | the rest ascending].
// Slabs of at most 32 rows are eliminated by one workgroup (k_slab_leaf)
// in the row-major order itself; each leaf's rank is read back once.
#include <climits>

#include "ffp_internal.hpp"
#include "ffp_device.hpp"

namespace ffp {

namespace {
constexpr int kSlabRows = 32;           // rows of a leaf slab
constexpr int kSlabT = 1024;            // threads of a leaf
constexpr int kSlabMaxW = FFP_SLAB_MAX_COLS;  // columns: LDS bitmap of the active columns

__device__ int slab_block_min(int v, int *red) {
    for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    int r = red[0];
#pragma unroll
    for (int i = 1; i < kSlabT / 64; ++i) r = min(r, red[i]);
    __syncthreads();
    return r;
}

// Row-major elimination of an m x w slab (m <= 32) in place, in original
// positions: for each row x in order, its leftmost nonzero among the active
// columns (c) is the next pivot; every later row i gets its multiplier l_i
// = A[i][c] / A[x][c] stored at A[i][c] and row x times l_i removed from its
// active columns.  Thread t owns columns t, t + 1024, ...  Outputs the
// local row order P (pivot rows, then the others ascending), the local
// column order Q (pivot columns in pivot order, then the active columns
// ascending) and the rank (to a device-visible word).
__global__ __launch_bounds__(kSlabT) void k_slab_leaf(int m, int w, int32_t *__restrict__ A, int64_t lda,
                                                      int32_t *__restrict__ P, int32_t *__restrict__ Q,
                                                      int64_t *__restrict__ rank_out, double p, double pinv,
                                                      int32_t pi) {
    __shared__ uint32_t act[kSlabMaxW / 32];
    __shared__ double lmul[kSlabRows];
    __shared__ int red[kSlabT / 64];
    __shared__ int prow[kSlabRows], pcol[kSlabRows];
    __shared__ double s_inv;
    __shared__ int cnt[kSlabT];
    const int tid = threadIdx.x;
    const int nw = (w + 31) >> 5;
    for (int i = tid; i < nw; i += kSlabT) act[i] = (i == nw - 1 && (w & 31)) ? ((1u << (w & 31)) - 1u) : 0xffffffffu;
    __syncthreads();
    int r = 0;
    for (int x = 0; x < m; ++x) {
        const int32_t *rowx = A + (int64_t)x * lda;
        int best = INT_MAX;
        for (int j = tid; j < w; j += kSlabT)
            if (((act[j >> 5] >> (j & 31)) & 1u) && rowx[j] != 0) {
                best = j;
                break;
            }
        const int c = slab_block_min(best, red);
        if (c == INT_MAX) continue;  // uniform: nothing left in this row
        if (tid == 0) {
            prow[r] = x;
            pcol[r] = c;
            act[c >> 5] &= ~(1u << (c & 31));
            s_inv = (double)inv_mod(rowx[c], pi);
        }
        __syncthreads();
        const int below = m - x - 1;
        if (tid < below) {
            int32_t *ri = A + (int64_t)(x + 1 + tid) * lda;
            const double l = mod_canon((double)ri[c] * s_inv, p, pinv);
            ri[c] = (int32_t)l;
            lmul[tid] = l;
        }
        __syncthreads();
        for (int j = tid; j < w; j += kSlabT) {
            if (!((act[j >> 5] >> (j & 31)) & 1u)) continue;
            const double u = (double)rowx[j];
            if (u == 0.0) continue;
            for (int t = 0; t < below; ++t) {
                const double l = lmul[t];
                if (l == 0.0) continue;
                int32_t *e = A + (int64_t)(x + 1 + t) * lda + j;
                *e = (int32_t)mod_canon(fma(-l, u, (double)*e), p, pinv);
            }
        }
        __syncthreads();
        ++r;
    }
    if (tid == 0) {
        int k = 0;
        for (int t = 0; t < r; ++t) P[k++] = prow[t];
        for (int i = 0; i < m; ++i) {
            bool piv = false;
            for (int t = 0; t < r; ++t) piv |= prow[t] == i;
            if (!piv) P[k++] = i;
        }
        *(volatile int64_t *)rank_out = r;
    }
    if (tid < r) Q[tid] = pcol[tid];
    // the active columns ascending after the pivots: each thread compacts a
    // contiguous chunk, offsets by an exclusive scan of the chunk counts
    const int chunk = (w + kSlabT - 1) / kSlabT;
    const int j0 = tid * chunk < w ? tid * chunk : w, j1 = j0 + chunk < w ? j0 + chunk : w;
    int c0 = 0;
    for (int j = j0; j < j1; ++j) c0 += (act[j >> 5] >> (j & 31)) & 1u;
    cnt[tid] = c0;
    __syncthreads();
    if (tid == 0) {
        int s = 0;
        for (int t = 0; t < kSlabT; ++t) {
            const int v = cnt[t];
            cnt[t] = s;
            s += v;
        }
    }
    __syncthreads();
    int pos = r + cnt[tid];
    for (int j = j0; j < j1; ++j)
        if ((act[j >> 5] >> (j & 31)) & 1u) Q[pos++] = j;
}

// P of a node from its halves' orders (Pin: top order in [0, h), bottom
// order in [h, m), each local): [top pivots | bottom pivots | top
// non-pivots | bottom non-pivots], bottom entries shifted by h
__global__ void k_slab_compose_p(int64_t m, int64_t h, int64_t r1, int64_t r2, const int32_t *__restrict__ Pin,
                                 int32_t *__restrict__ Pout) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x) {
        int32_t v;
        if (i < r1) v = Pin[i];
        else if (i < r1 + r2) v = (int32_t)h + Pin[h + (i - r1)];
        else if (i < h + r2) v = Pin[r1 + (i - r1 - r2)];
        else v = (int32_t)h + Pin[i];
        Pout[i] = v;
    }
}

// Q of a node: Q1 on the first r1 positions, Q1 composed with Q2 after
__global__ void k_slab_compose_q(int64_t w, int64_t r1, const int32_t *__restrict__ Q1, const int32_t *__restrict__ Q2,
                                 int32_t *__restrict__ Qout) {
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < w; j += (int64_t)gridDim.x * blockDim.x)
        Qout[j] = j < r1 ? Q1[j] : Q1[r1 + Q2[j - r1]];
}

// rotation of len rows by `shift`: destination d reads source (d + shift) mod len
__global__ void k_slab_rot(int64_t len, int64_t shift, int32_t *__restrict__ idx) {
    for (int64_t d = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; d < len; d += (int64_t)gridDim.x * blockDim.x)
        idx[d] = (int32_t)((d + shift) % len);
}

__global__ void k_slab_iota(int32_t *v, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        v[i] = (int32_t)i;
}

unsigned g1(int64_t n) { return (unsigned)((n + 255) / 256 < 1024 ? ((n + 255) / 256 > 0 ? (n + 255) / 256 : 1) : 1024); }

PermSpec idx_spec(const int32_t *idx) {
    PermSpec ps;
    ps.idx = idx;
    return ps;
}

struct SCtx {
    int path;
    const Field &F;
    Arena &ws;
    hipStream_t s;
    RankWord rw;
};

// one rank read-back through the pinned word
int read_word(SCtx &c, int64_t *out) {
    FFP_HIP_CHECK(hipStreamSynchronize(c.s));
    *out = *(const volatile int64_t *)c.rw.host;
    return FFP_OK;
}

int slab_rec(SCtx &c, int64_t m, int64_t w, int32_t *A, int64_t lda, int32_t *P, int32_t *Q, int64_t *rank) {
    const Field &F = c.F;
    Arena &ws = c.ws;
    hipStream_t s = c.s;
    if (m <= 0 || w <= 0) {
        if (m > 0) hipLaunchKernelGGL(k_slab_iota, dim3(g1(m)), dim3(256), 0, s, P, m);
        if (w > 0) hipLaunchKernelGGL(k_slab_iota, dim3(g1(w)), dim3(256), 0, s, Q, w);
        FFP_HIP_CHECK(hipGetLastError());
        *rank = 0;
        return FFP_OK;
    }
    if (m <= kSlabRows) {
        {
            ProfScope prof(PK_LEAF, 0.0, s, 8.0 * (double)m * (double)w);
            hipLaunchKernelGGL(k_slab_leaf, dim3(1), dim3(kSlabT), 0, s, (int)m, (int)w, A, lda, P, Q, c.rw.dev, F.pd,
                               F.pinv, (int32_t)F.p);
            FFP_HIP_CHECK(hipGetLastError());
        }
        FFP_CHECK(read_word(c, rank));
        return permute_inplace(m, w, A, lda, idx_spec(P), idx_spec(Q), ws, s);
    }
    const int64_t h = m / 2;
    const size_t mk = ws.mark();
    int32_t *Q1 = (int32_t *)ws.take((size_t)w * 4);
    int32_t *Q2 = (int32_t *)ws.take((size_t)w * 4);
    int32_t *Pt = (int32_t *)ws.take((size_t)m * 4);
    int32_t *rot = (int32_t *)ws.take((size_t)m * 4);
    if (!Q1 || !Q2 || !Pt || !rot) return FFP_E_WORKSPACE;
    int64_t r1 = 0, r2 = 0;
    FFP_CHECK(slab_rec(c, h, w, A, lda, P, Q1, &r1));
    int32_t *Ab = A + h * lda;
    FFP_CHECK(permute_inplace(m - h, w, Ab, lda, PermSpec(), idx_spec(Q1), ws, s));
    if (r1 > 0) {
        FFP_CHECK(ftrsm_run(resolve_path(c.path, F.p, r1 / 2, m - h, r1 / 2), F, 1, 1, 0, 0, m - h, r1, 1, A, lda, Ab,
                            lda, ws, s));
        if (w > r1)
            FFP_CHECK(fgemm_any(resolve_path(c.path, F.p, m - h, w - r1, r1), F, 0, 0, m - h, w - r1, r1, F.p - 1, Ab,
                                lda, A + r1, lda, 1, Ab + r1, lda, ws, s));
    }
    FFP_CHECK(slab_rec(c, m - h, w - r1, Ab + r1, lda, P + h, Q2, &r2));
    if (r1 > 0) {
        if (w > r1) FFP_CHECK(permute_inplace(r1, w - r1, A + r1, lda, PermSpec(), idx_spec(Q2), ws, s));
        FFP_CHECK(permute_inplace(m - h, r1, Ab, lda, idx_spec(P + h), PermSpec(), ws, s));
    }
    if (h > r1 && r2 > 0) {
        const int64_t len = h - r1 + r2;
        hipLaunchKernelGGL(k_slab_rot, dim3(g1(len)), dim3(256), 0, s, len, h - r1, rot);
        FFP_HIP_CHECK(hipGetLastError());
        FFP_CHECK(permute_inplace(len, w, A + r1 * lda, lda, idx_spec(rot), PermSpec(), ws, s));
    }
    hipLaunchKernelGGL(k_slab_compose_p, dim3(g1(m)), dim3(256), 0, s, m, h, r1, r2, P, Pt);
    hipLaunchKernelGGL(k_slab_compose_q, dim3(g1(w)), dim3(256), 0, s, w, r1, Q1, Q2, Q);
    FFP_HIP_CHECK(hipGetLastError());
    FFP_HIP_CHECK(hipMemcpyAsync(P, Pt, (size_t)m * 4, hipMemcpyDeviceToDevice, s));
    *rank = r1 + r2;
    ws.release(mk);
    return FFP_OK;
}
}  // namespace

size_t pluq_slab_ws(int64_t m, int64_t n, const Field &F, int path) {
    int64_t depth = 2;
    for (int64_t x = m; x > kSlabRows; x >>= 1) ++depth;
    size_t b = (size_t)m * (size_t)n * 4 + 1024;                   // largest out-of-place permutation
    b += (size_t)depth * ((size_t)(2 * n + 2 * m) * 4 + 4 * 256);  // index vectors along one path
    if (path == FFP_PATH_INT8 || path == FFP_PATH_AUTO)
        b += fgemm_i8_ws(F, m, n, (m + 1) / 2) + fgemm_i8_split_ws(m, n);
    b += ftrsm_ws(FFP_PATH_INT8, F, 1, m, (m + 1) / 2) + ftrsm_ws(FFP_PATH_FP64, F, 1, m, (m + 1) / 2);
    b += (size_t)(m > n ? m : n) + 4096;                           // rank profiles
    return b;
}

int pluq_slab_run(int path, const Field &F, int64_t m, int64_t n, int32_t *A, int64_t lda, int32_t *P, int32_t *Q,
                  int64_t *r, Arena &ws, hipStream_t s) {
    RankWord rw;
    FFP_CHECK(rank_word_get(&rw));
    struct WordBack {
        RankWord w;
        ~WordBack() { rank_word_put(w); }
    } word_back{rw};
    SCtx c{path, F, ws, s, rw};
    return slab_rec(c, m, n, A, lda, P, Q, r);
}

}  // namespace ffp
