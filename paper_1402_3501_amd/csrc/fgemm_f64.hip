// fgemm over Z/pZ on the FP64 matrix cores of gfx950 (v_mfma_f64_16x16x4_f64).
//
// Section 2.1 (gemm) with the delayed reduction of Section 3.1: residues are
// embedded in doubles as centred integers |c| <= (p-1)/2, so a sum of k
// products is an exact integer while p + k ((p-1)/2)^2 < 2^53.  The K loop
// runs on the matrix cores with no reduction at all when k is below that
// bound (every workload here except p = 8388593), and otherwise brings the
// accumulators back to (-p, p) every `kchunk` products.  The single final
// reduction, alpha, beta and the int32 store are fused into the epilogue.
//
// Tiling: 256 threads (4 wave64s in a 2 x 2 grid), block tile BM x BN x 16,
// operands converted int32 -> centred FP64 on their way to LDS, double
// buffered (one barrier per K tile), global loads of tile t+1 in flight
// while tile t is multiplied.
#include "ffp_internal.hpp"
#include "ffp_device.hpp"

namespace ffp {

typedef double v4d __attribute__((ext_vector_type(4)));

template <int BM, int BN, bool TA, bool TB, bool RED>
__global__ __launch_bounds__(256) void k_fgemm_f64(int64_t m, int64_t n, int64_t k,
                                                   const int32_t *__restrict__ A, int64_t lda,
                                                   const int32_t *__restrict__ B, int64_t ldb,
                                                   int32_t *__restrict__ C, int64_t ldc, double p,
                                                   double pinv, int32_t half, double alpha,
                                                   double beta, int kchunk_steps, int ntx, int nty) {
    constexpr int BK = 16;
    constexpr int PAD = 2;
    constexpr int WM = BM / 2, WN = BN / 2;
    constexpr int FM = WM / 16, FN = WN / 16;
    constexpr int A_PER = BM * BK / 256;
    constexpr int B_PER = BN * BK / 256;
    __shared__ double As[2][BK][BM + PAD];
    __shared__ double Bs[2][BK][BN + PAD];

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wm0 = (wave >> 1) * WM, wn0 = (wave & 1) * WN;
    int ty, tx;
    xcd_tile(blockIdx.x, ntx, nty, ty, tx);
    const int64_t m0 = (int64_t)ty * BM, n0 = (int64_t)tx * BN;

    int32_t ra[A_PER], rb[B_PER];

    // element e of this thread in the A tile: (row i, inner kk); coalesced
    // along the stored contiguous dimension
    auto a_coord = [&](int e, int &i, int &kk) {
        int idx = tid + e * 256;
        if (!TA) { kk = idx % BK; i = idx / BK; }
        else { i = idx % BM; kk = idx / BM; }
    };
    auto b_coord = [&](int e, int &kk, int &j) {
        int idx = tid + e * 256;
        if (!TB) { j = idx % BN; kk = idx / BN; }
        else { kk = idx % BK; j = idx / BK; }
    };
    auto load = [&](int64_t k0) {
#pragma unroll
        for (int e = 0; e < A_PER; ++e) {
            int i, kk;
            a_coord(e, i, kk);
            int64_t gi = m0 + i, gk = k0 + kk;
            int32_t v = 0;
            if (gi < m && gk < k) v = TA ? A[gk * lda + gi] : A[gi * lda + gk];
            ra[e] = v;
        }
#pragma unroll
        for (int e = 0; e < B_PER; ++e) {
            int kk, j;
            b_coord(e, kk, j);
            int64_t gj = n0 + j, gk = k0 + kk;
            int32_t v = 0;
            if (gj < n && gk < k) v = TB ? B[gj * ldb + gk] : B[gk * ldb + gj];
            rb[e] = v;
        }
    };
    auto store = [&](int buf) {
#pragma unroll
        for (int e = 0; e < A_PER; ++e) {
            int i, kk;
            a_coord(e, i, kk);
            As[buf][kk][i] = centre(ra[e], p, half);
        }
#pragma unroll
        for (int e = 0; e < B_PER; ++e) {
            int kk, j;
            b_coord(e, kk, j);
            Bs[buf][kk][j] = centre(rb[e], p, half);
        }
    };

    v4d acc[FM][FN];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) acc[i][j] = v4d{0.0, 0.0, 0.0, 0.0};

    const int64_t ntiles = (k + BK - 1) / BK;
    int steps = 0;
    if (ntiles > 0) {
        load(0);
        store(0);
    }
    __syncthreads();
    for (int64_t t = 0; t < ntiles; ++t) {
        const int buf = (int)(t & 1);
        if (t + 1 < ntiles) load((t + 1) * BK);
#pragma unroll
        for (int ks = 0; ks < BK / 4; ++ks) {
            double a[FM], b[FN];
            const int kr = ks * 4 + (lane >> 4);
#pragma unroll
            for (int i = 0; i < FM; ++i) a[i] = As[buf][kr][wm0 + i * 16 + (lane & 15)];
#pragma unroll
            for (int j = 0; j < FN; ++j) b[j] = Bs[buf][kr][wn0 + j * 16 + (lane & 15)];
#pragma unroll
            for (int i = 0; i < FM; ++i)
#pragma unroll
                for (int j = 0; j < FN; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
            if (RED) {
                if (++steps == kchunk_steps) {
                    steps = 0;
#pragma unroll
                    for (int i = 0; i < FM; ++i)
#pragma unroll
                        for (int j = 0; j < FN; ++j)
#pragma unroll
                            for (int v = 0; v < 4; ++v) acc[i][j][v] = mod_near(acc[i][j][v], p, pinv);
                }
            }
        }
        if (t + 1 < ntiles) store(buf ^ 1);
        __syncthreads();
    }

    // epilogue: in each 16x16 FP64 result block, lane l holds rows l/16 + 4v
    // (v = 0..3) of column l%16
#pragma unroll
    for (int i = 0; i < FM; ++i) {
#pragma unroll
        for (int j = 0; j < FN; ++j) {
            const int64_t gj = n0 + wn0 + j * 16 + (lane & 15);
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int64_t gi = m0 + wm0 + i * 16 + (lane >> 4) + 4 * v;
                if (gi < m && gj < n) {
                    double r = mod_canon(acc[i][j][v], p, pinv);
                    if (alpha != 1.0) r = mod_canon(alpha * r, p, pinv);
                    if (beta != 0.0) {
                        double c = (double)C[gi * ldc + gj];
                        if (beta != 1.0) c = mod_canon(beta * c, p, pinv);
                        r += c;
                        if (r >= p) r -= p;
                    }
                    C[gi * ldc + gj] = (int32_t)r;
                }
            }
        }
    }
}

// Small and medium products (up to a few hundred 64 x 64 output tiles): the
// same arithmetic with K staged 64 at a time, so a product with k <= 64 makes
// a single round trip to memory for its operands (the C tile for beta != 0
// is fetched alongside), and longer K overlaps the next 64-slice with the
// current one.  Operands sit in LDS as centred int32 (converted to FP64 as
// the matrix-core fragments are read).
template <bool TA, bool TB, bool RED>
__global__ __launch_bounds__(256) void k_fgemm_f64_k64(int64_t m, int64_t n, int64_t k,
                                                       const int32_t *__restrict__ A, int64_t lda,
                                                       const int32_t *__restrict__ B, int64_t ldb,
                                                       int32_t *__restrict__ C, int64_t ldc, double p, double pinv,
                                                       int32_t half, double alpha, double beta, int kchunk_steps) {
    constexpr int T = 64;
    __shared__ int32_t As[2][T][T + 1];  // [kk][i]
    __shared__ int32_t Bs[2][T][T + 1];  // [kk][j]
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm0 = (wave >> 1) * 32, wn0 = (wave & 1) * 32;
    const int64_t m0 = (int64_t)blockIdx.y * T, n0 = (int64_t)blockIdx.x * T;
    const int32_t ip = (int32_t)p;
    int32_t ra[16], rb[16];
    // loads are unconditional (addresses clamped into the operand) so that
    // they are all in flight together; out-of-range elements are zeroed after
    auto load = [&](int64_t k0) {
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            const int idx = tid + e * 256, x = idx % T, y = idx / T;  // x along the contiguous dimension
            {
                const int i = TA ? x : y, kk = TA ? y : x;
                const int64_t gi = m0 + i, gk = k0 + kk;
                const int64_t ci = gi < m ? gi : m - 1, ck = gk < k ? gk : k - 1;
                ra[e] = TA ? A[ck * lda + ci] : A[ci * lda + ck];
            }
            {
                const int j = TB ? y : x, kk = TB ? x : y;
                const int64_t gj = n0 + j, gk = k0 + kk;
                const int64_t cj = gj < n ? gj : n - 1, ck = gk < k ? gk : k - 1;
                rb[e] = TB ? B[cj * ldb + ck] : B[ck * ldb + cj];
            }
        }
    };
    auto mask = [&](int64_t k0) {
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            const int idx = tid + e * 256, x = idx % T, y = idx / T;
            {
                const int i = TA ? x : y, kk = TA ? y : x;
                if (!(m0 + i < m && k0 + kk < k)) ra[e] = 0;
            }
            {
                const int j = TB ? y : x, kk = TB ? x : y;
                if (!(n0 + j < n && k0 + kk < k)) rb[e] = 0;
            }
        }
    };
    auto store = [&](int buf, int64_t k0) {
        mask(k0);
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            const int idx = tid + e * 256, x = idx % T, y = idx / T;
            As[buf][TA ? y : x][TA ? x : y] = ra[e] > half ? ra[e] - ip : ra[e];
            Bs[buf][TB ? x : y][TB ? y : x] = rb[e] > half ? rb[e] - ip : rb[e];
        }
    };
    // C tile prefetch (beta != 0); lane l holds rows l/16 + 4v of column l%16
    int32_t cpre[2][2][4];
    if (beta != 0.0) {
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int64_t gi = m0 + wm0 + i * 16 + (lane >> 4) + 4 * v, gj = n0 + wn0 + j * 16 + (lane & 15);
                    cpre[i][j][v] = C[(gi < m ? gi : m - 1) * ldc + (gj < n ? gj : n - 1)];
                }
    }
    v4d acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = v4d{0.0, 0.0, 0.0, 0.0};
    const int64_t nt = (k + T - 1) / T;
    int steps = 0;
    if (nt > 0) {
        load(0);
        store(0, 0);
    }
    __syncthreads();
    for (int64_t t = 0; t < nt; ++t) {
        const int buf = (int)(t & 1);
        if (t + 1 < nt) load((t + 1) * T);
#pragma unroll
        for (int ks = 0; ks < T / 4; ++ks) {
            const int kr = ks * 4 + (lane >> 4);
            double a[2], b[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) a[i] = (double)As[buf][kr][wm0 + i * 16 + (lane & 15)];
#pragma unroll
            for (int j = 0; j < 2; ++j) b[j] = (double)Bs[buf][kr][wn0 + j * 16 + (lane & 15)];
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
            if (RED && ++steps == kchunk_steps) {
                steps = 0;
#pragma unroll
                for (int i = 0; i < 2; ++i)
#pragma unroll
                    for (int j = 0; j < 2; ++j)
#pragma unroll
                        for (int v = 0; v < 4; ++v) acc[i][j][v] = mod_near(acc[i][j][v], p, pinv);
            }
        }
        if (t + 1 < nt) store(buf ^ 1, (t + 1) * T);
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int64_t gi = m0 + wm0 + i * 16 + (lane >> 4) + 4 * v, gj = n0 + wn0 + j * 16 + (lane & 15);
                if (gi < m && gj < n) {
                    double r = mod_canon(acc[i][j][v], p, pinv);
                    if (alpha != 1.0) r = mod_canon(alpha * r, p, pinv);
                    if (beta != 0.0) {
                        double c = (double)cpre[i][j][v];
                        if (beta != 1.0) c = mod_canon(beta * c, p, pinv);
                        r += c;
                        if (r >= p) r -= p;
                    }
                    C[gi * ldc + gj] = (int32_t)r;
                }
            }
}

// Small products: one 32 x 32 output tile per workgroup of four waves that
// split K (wave w takes the 32-deep K stages w, w + 4, ...), so a product of
// a few 64 x 64 blocks keeps the matrix cores of four SIMDs busy on each of
// many compute units instead of one long wave.  Operands go straight from
// global memory to registers, one stage ahead: at k-step s of a stage, lane
// l supplies row l % 16 and the reduction index 8 (l / 16) + s (the order of
// the sum is free), so each lane reads 8 consecutive entries of a row-major
// operand (two 16-byte loads when aligned) and the other operand is read
// with 16 lanes along its contiguous dimension.  Loads are unconditional
// with clamped 32-bit indices and masked after arrival.  The four partial
// tiles, each reduced to |x| <= p/2, are summed through LDS; for alpha = +-1
// and beta in {0, 1} the epilogue is one reduction of +-acc + C.
template <bool TA, bool TB, bool RED>
__device__ __forceinline__ void sk_body(int m0, int n0, int m, int n, int k, const int32_t *__restrict__ A,
                                        uint32_t lda, const int32_t *__restrict__ B, uint32_t ldb,
                                        int32_t *__restrict__ C, uint32_t ldc, double p, double pinv, int32_t half,
                                        double alpha, double beta, int kchunk_steps, int vecA, int vecB) {
    constexpr int T = 32, KD = 32, NWV = 4;
    __shared__ double part[NWV][T][T + 1];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int r16 = lane & 15, kq = lane >> 4;
    const int32_t ip = (int32_t)p;
    const int nst = (k + KD - 1) / KD;
    // one operand's 2 x 8 entries of a stage: rows (or columns) 16 u + r16
    // of the tile, reduction indices k0 + 8 kq + s
    auto load_op = [&](const int32_t *__restrict__ X, uint32_t ldx, bool kcontig, int vec, int base, int lim, int k0,
                       int32_t (&r)[2][8]) {
        const int kb = k0 + 8 * kq;
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int g = min(base + 16 * u + r16, lim - 1);
            if (kcontig) {
                const int32_t *row = X + (uint64_t)g * ldx;
                if (vec && kb + 8 <= k) {
                    const int4 x = *(const int4 *)(row + kb), y = *(const int4 *)(row + kb + 4);
                    r[u][0] = x.x; r[u][1] = x.y; r[u][2] = x.z; r[u][3] = x.w;
                    r[u][4] = y.x; r[u][5] = y.y; r[u][6] = y.z; r[u][7] = y.w;
                } else {
#pragma unroll
                    for (int t = 0; t < 8; ++t) r[u][t] = row[min(kb + t, k - 1)];
                }
            } else {
#pragma unroll
                for (int t = 0; t < 8; ++t) r[u][t] = X[(uint64_t)min(kb + t, k - 1) * ldx + g];
            }
        }
    };
    auto load = [&](int k0, int32_t (&ra)[2][8], int32_t (&rb)[2][8]) {
        load_op(A, lda, !TA, vecA, m0, m, k0, ra);
        load_op(B, ldb, TB, vecB, n0, n, k0, rb);
    };
    // this thread's four entries of C for the epilogue, read up front
    int32_t cv[T * T / 256];
#pragma unroll
    for (int e = 0; e < T * T / 256; ++e) {
        const int idx = tid + 256 * e;
        cv[e] = beta != 0.0 ? C[(uint64_t)min(m0 + (idx >> 5), m - 1) * ldc + min(n0 + (idx & 31), n - 1)] : 0;
    }
    v4d acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = v4d{0.0, 0.0, 0.0, 0.0};
    int steps = 0;
    auto compute = [&](int k0, const int32_t (&ra)[2][8], const int32_t (&rb)[2][8]) {
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            const bool kin = k0 + 8 * kq + t < k;
            double a[2], b[2];
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const int32_t va = (kin && m0 + 16 * u + r16 < m) ? ra[u][t] : 0;
                const int32_t vb = (kin && n0 + 16 * u + r16 < n) ? rb[u][t] : 0;
                a[u] = (double)(va > half ? va - ip : va);
                b[u] = (double)(vb > half ? vb - ip : vb);
            }
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
            if (RED && ++steps == kchunk_steps) {
                steps = 0;
#pragma unroll
                for (int i = 0; i < 2; ++i)
#pragma unroll
                    for (int j = 0; j < 2; ++j)
#pragma unroll
                        for (int v = 0; v < 4; ++v) acc[i][j][v] = mod_near(acc[i][j][v], p, pinv);
            }
        }
    };
    {
        int32_t a0[2][8], b0[2][8], a1[2][8], b1[2][8];
        int st = wave;
        if (st < nst) load(st * KD, a0, b0);
        while (st < nst) {
            if (st + NWV < nst) load((st + NWV) * KD, a1, b1);
            compute(st * KD, a0, b0);
            st += NWV;
            if (st >= nst) break;
            if (st + NWV < nst) load((st + NWV) * KD, a0, b0);
            compute(st * KD, a1, b1);
            st += NWV;
        }
    }
    // lane l holds rows l/16 + 4v of column l%16 of each 16 x 16 block
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v)
                part[wave][i * 16 + kq + 4 * v][j * 16 + r16] = mod_near(acc[i][j][v], p, pinv);
    __syncthreads();
    const double sgn = alpha == 1.0 ? 1.0 : (alpha == p - 1.0 ? -1.0 : 0.0);
    const bool fast = sgn != 0.0 && (beta == 0.0 || beta == 1.0);
#pragma unroll
    for (int e = 0; e < T * T / 256; ++e) {
        const int idx = tid + 256 * e, li = idx >> 5, lj = idx & 31;
        const int gi = m0 + li, gj = n0 + lj;
        const double x = part[0][li][lj] + part[1][li][lj] + part[2][li][lj] + part[3][li][lj];
        double r;
        if (fast) {
            r = mod_canon(fma(sgn, x, (double)cv[e]), p, pinv);
        } else {
            r = mod_canon(x, p, pinv);
            if (alpha != 1.0) r = mod_canon(alpha * r, p, pinv);
            if (beta != 0.0) {
                double c = (double)cv[e];
                if (beta != 1.0) c = mod_canon(beta * c, p, pinv);
                r += c;
                if (r >= p) r -= p;
            }
        }
        if (gi < m && gj < n) C[(uint64_t)gi * ldc + gj] = (int32_t)r;
    }
}

template <bool TA, bool TB, bool RED>
__global__ __launch_bounds__(256) void k_fgemm_f64_sk(int m, int n, int k, const int32_t *__restrict__ A,
                                                      uint32_t lda, const int32_t *__restrict__ B, uint32_t ldb,
                                                      int32_t *__restrict__ C, uint32_t ldc, double p, double pinv,
                                                      int32_t half, double alpha, double beta, int kchunk_steps,
                                                      int vecA, int vecB) {
    sk_body<TA, TB, RED>((int)blockIdx.y * 32, (int)blockIdx.x * 32, m, n, k, A, lda, B, ldb, C, ldc, p, pinv, half,
                         alpha, beta, kchunk_steps, vecA, vecB);
}

// Two independent small products with the same k, alpha and beta (the two
// updates between the levels of a pair of panel solves) in one launch: the
// first o0.nblk workgroups take the first product's 32 x 32 tiles, the rest
// the second's.
struct SkOp {
    int m, n;
    const int32_t *A;
    uint32_t lda;
    const int32_t *B;
    uint32_t ldb;
    int32_t *C;
    uint32_t ldc;
    int vecA, vecB, ntx, nblk;
};
template <bool RED>
__global__ __launch_bounds__(256) void k_fgemm_f64_sk_pair(SkOp o0, SkOp o1, int k, double p, double pinv,
                                                           int32_t half, double alpha, double beta,
                                                           int kchunk_steps) {
    const bool second = (int)blockIdx.x >= o0.nblk;
    const SkOp o = second ? o1 : o0;
    const int b = second ? (int)blockIdx.x - o0.nblk : (int)blockIdx.x;
    sk_body<false, false, RED>((b / o.ntx) * 32, (b % o.ntx) * 32, o.m, o.n, k, o.A, o.lda, o.B, o.ldb, o.C, o.ldc,
                               p, pinv, half, alpha, beta, kchunk_steps, o.vecA, o.vecB);
}

template <int BM, int BN, bool RED>
static void launch_tiles(int ta, int tb, dim3 grid, hipStream_t s, int64_t m, int64_t n, int64_t k,
                         const int32_t *A, int64_t lda, const int32_t *B, int64_t ldb, int32_t *C,
                         int64_t ldc, double p, double pinv, int32_t half, double alpha,
                         double beta, int ksteps) {
    const int ntx = (int)grid.x, nty = (int)grid.y;
    const dim3 g1((unsigned)(ntx * nty));
#define FFP_LAUNCH(TA_, TB_)                                                                  \
    hipLaunchKernelGGL((k_fgemm_f64<BM, BN, TA_, TB_, RED>), g1, dim3(256), 0, s, m, n, k, A, \
                       lda, B, ldb, C, ldc, p, pinv, half, alpha, beta, ksteps, ntx, nty)
    if (!ta && !tb) FFP_LAUNCH(false, false);
    else if (ta && !tb) FFP_LAUNCH(true, false);
    else if (!ta && tb) FFP_LAUNCH(false, true);
    else FFP_LAUNCH(true, true);
#undef FFP_LAUNCH
}

// the small-product kernel takes a product with fewer than 192 tiles of
// 128 and (fewer than 256 tiles of 64 or k <= 256), with 32-bit indices
static bool takes_sk(int64_t m, int64_t n, int64_t k, int64_t lda, int64_t ldb, int64_t ldc) {
    const int64_t big_tiles = ((m + 127) / 128) * ((n + 127) / 128);
    return big_tiles < 192 && (((m + 63) / 64) * ((n + 63) / 64) < 256 || k <= 256) && m < (1ll << 30) &&
           n < (1ll << 30) && k < (1ll << 30) && lda < (1ll << 31) && ldb < (1ll << 31) && ldc < (1ll << 31);
}

int fgemm_f64_pair(const Field &F, int64_t m0, int64_t n0, const int32_t *A0, int64_t lda0, const int32_t *B0,
                   int64_t ldb0, int32_t *C0, int64_t ldc0, int64_t m1, int64_t n1, const int32_t *A1, int64_t lda1,
                   const int32_t *B1, int64_t ldb1, int32_t *C1, int64_t ldc1, int64_t k, uint32_t alpha,
                   uint32_t beta, hipStream_t s) {
    if (m0 <= 0 || n0 <= 0 || m1 <= 0 || n1 <= 0 || k <= 0 || !takes_sk(m0, n0, k, lda0, ldb0, ldc0) ||
        !takes_sk(m1, n1, k, lda1, ldb1, ldc1)) {
        FFP_CHECK(fgemm_f64(F, 0, 0, m0, n0, k, alpha, A0, lda0, B0, ldb0, beta, C0, ldc0, s));
        return fgemm_f64(F, 0, 0, m1, n1, k, alpha, A1, lda1, B1, ldb1, beta, C1, ldc1, s);
    }
    const bool red = k > F.kexact;
    const int ksteps = (int)(F.kexact / 4 > (1 << 30) ? (1 << 30) : (F.kexact / 4 < 1 ? 1 : F.kexact / 4));
    auto op = [](int64_t m, int64_t n, const int32_t *A, int64_t lda, const int32_t *B, int64_t ldb, int32_t *C,
                 int64_t ldc) {
        SkOp o;
        o.m = (int)m;
        o.n = (int)n;
        o.A = A;
        o.lda = (uint32_t)lda;
        o.B = B;
        o.ldb = (uint32_t)ldb;
        o.C = C;
        o.ldc = (uint32_t)ldc;
        o.vecA = ((((uintptr_t)A) | (uintptr_t)(lda * 4)) & 15) == 0;
        o.vecB = ((((uintptr_t)B) | (uintptr_t)(ldb * 4)) & 15) == 0;
        o.ntx = (int)((n + 31) / 32);
        o.nblk = o.ntx * (int)((m + 31) / 32);
        return o;
    };
    const SkOp o0 = op(m0, n0, A0, lda0, B0, ldb0, C0, ldc0), o1 = op(m1, n1, A1, lda1, B1, ldb1, C1, ldc1);
    const double mn = (double)m0 * (double)n0 + (double)m1 * (double)n1;
    ProfScope prof(PK_FGEMM_F64, 2.0 * mn * (double)k, s,
                   4.0 * ((double)(m0 + m1) * (double)k + (double)k * (double)(n0 + n1) + (beta != 0 ? 2.0 : 1.0) * mn));
    const dim3 grid((unsigned)(o0.nblk + o1.nblk));
    if (red)
        hipLaunchKernelGGL((k_fgemm_f64_sk_pair<true>), grid, dim3(256), 0, s, o0, o1, (int)k, F.pd, F.pinv,
                           (int32_t)F.half, (double)alpha, (double)beta, ksteps);
    else
        hipLaunchKernelGGL((k_fgemm_f64_sk_pair<false>), grid, dim3(256), 0, s, o0, o1, (int)k, F.pd, F.pinv,
                           (int32_t)F.half, (double)alpha, (double)beta, ksteps);
    FFP_HIP_CHECK(hipGetLastError());
    return FFP_OK;
}

int fgemm_f64(const Field &F, int ta, int tb, int64_t m, int64_t n, int64_t k, uint32_t alpha,
              const int32_t *A, int64_t lda, const int32_t *B, int64_t ldb, uint32_t beta,
              int32_t *C, int64_t ldc, hipStream_t s) {
    if (m <= 0 || n <= 0) return FFP_OK;
    const bool red = k > F.kexact;
    const int ksteps = (int)(F.kexact / 4 > (1 << 30) ? (1 << 30) : (F.kexact / 4 < 1 ? 1 : F.kexact / 4));
    const double p = F.pd, pinv = F.pinv, a = (double)alpha, b = (double)beta;
    const int32_t half = (int32_t)F.half;
    const int64_t big_tiles = ((m + 127) / 128) * ((n + 127) / 128);
    ProfScope prof(PK_FGEMM_F64, 2.0 * (double)m * (double)n * (double)k, s,
                   4.0 * ((double)m * (double)k + (double)k * (double)n + (beta != 0 ? 2.0 : 1.0) * (double)m * (double)n));
    if (big_tiles >= 192) {
        dim3 grid((unsigned)((n + 127) / 128), (unsigned)((m + 127) / 128));
        if (red) launch_tiles<128, 128, true>(ta, tb, grid, s, m, n, k, A, lda, B, ldb, C, ldc, p, pinv, half, a, b, ksteps);
        else launch_tiles<128, 128, false>(ta, tb, grid, s, m, n, k, A, lda, B, ldb, C, ldc, p, pinv, half, a, b, ksteps);
    } else if (takes_sk(m, n, k, lda, ldb, ldc)) {
        dim3 grid((unsigned)((n + 31) / 32), (unsigned)((m + 31) / 32));
        // 16-byte loads along K need 16-byte aligned rows
        const int vA = ((((uintptr_t)A) | (uintptr_t)(lda * 4)) & 15) == 0;
        const int vB = ((((uintptr_t)B) | (uintptr_t)(ldb * 4)) & 15) == 0;
#define FFP_T32(TA_, TB_, R_)                                                                               \
    hipLaunchKernelGGL((k_fgemm_f64_sk<TA_, TB_, R_>), grid, dim3(256), 0, s, (int)m, (int)n, (int)k, A,    \
                       (uint32_t)lda, B, (uint32_t)ldb, C, (uint32_t)ldc, p, pinv, half, a, b, ksteps, vA, vB)
#define FFP_T32R(R_)                                          \
    if (!ta && !tb) FFP_T32(false, false, R_);                 \
    else if (ta && !tb) FFP_T32(true, false, R_);              \
    else if (!ta && tb) FFP_T32(false, true, R_);              \
    else FFP_T32(true, true, R_);
        if (red) { FFP_T32R(true) } else { FFP_T32R(false) }
#undef FFP_T32R
#undef FFP_T32
    } else {
        dim3 grid((unsigned)((n + 63) / 64), (unsigned)((m + 63) / 64));
#define FFP_K64(TA_, TB_, R_)                                                                                  \
    hipLaunchKernelGGL((k_fgemm_f64_k64<TA_, TB_, R_>), grid, dim3(256), 0, s, m, n, k, A, lda, B, ldb, C, ldc, \
                       p, pinv, half, a, b, ksteps)
#define FFP_K64R(R_)                                          \
    if (!ta && !tb) FFP_K64(false, false, R_);                 \
    else if (ta && !tb) FFP_K64(true, false, R_);              \
    else if (!ta && tb) FFP_K64(false, true, R_);              \
    else FFP_K64(true, true, R_);
        if (red) { FFP_K64R(true) } else { FFP_K64R(false) }
#undef FFP_K64R
#undef FFP_K64
    }
    FFP_HIP_CHECK(hipGetLastError());
    return FFP_OK;
}

}  // namespace ffp
