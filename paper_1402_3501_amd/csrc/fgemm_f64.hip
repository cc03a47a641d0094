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
                                                   double beta, int kchunk_steps) {
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
    const int64_t m0 = (int64_t)blockIdx.y * BM, n0 = (int64_t)blockIdx.x * BN;

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

template <int BM, int BN, bool RED>
static void launch_tiles(int ta, int tb, dim3 grid, hipStream_t s, int64_t m, int64_t n, int64_t k,
                         const int32_t *A, int64_t lda, const int32_t *B, int64_t ldb, int32_t *C,
                         int64_t ldc, double p, double pinv, int32_t half, double alpha,
                         double beta, int ksteps) {
#define FFP_LAUNCH(TA_, TB_)                                                                  \
    hipLaunchKernelGGL((k_fgemm_f64<BM, BN, TA_, TB_, RED>), grid, dim3(256), 0, s, m, n, k, A, \
                       lda, B, ldb, C, ldc, p, pinv, half, alpha, beta, ksteps)
    if (!ta && !tb) FFP_LAUNCH(false, false);
    else if (ta && !tb) FFP_LAUNCH(true, false);
    else if (!ta && tb) FFP_LAUNCH(false, true);
    else FFP_LAUNCH(true, true);
#undef FFP_LAUNCH
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
    ProfScope prof(FFP_PATH_FP64, 2.0 * (double)m * (double)n * (double)k, s);
    if (big_tiles >= 192) {
        dim3 grid((unsigned)((n + 127) / 128), (unsigned)((m + 127) / 128));
        if (red) launch_tiles<128, 128, true>(ta, tb, grid, s, m, n, k, A, lda, B, ldb, C, ldc, p, pinv, half, a, b, ksteps);
        else launch_tiles<128, 128, false>(ta, tb, grid, s, m, n, k, A, lda, B, ldb, C, ldc, p, pinv, half, a, b, ksteps);
    } else {
        dim3 grid((unsigned)((n + 63) / 64), (unsigned)((m + 63) / 64));
        if (red) launch_tiles<64, 64, true>(ta, tb, grid, s, m, n, k, A, lda, B, ldb, C, ldc, p, pinv, half, a, b, ksteps);
        else launch_tiles<64, 64, false>(ta, tb, grid, s, m, n, k, A, lda, B, ldb, C, ldc, p, pinv, half, a, b, ksteps);
    }
    FFP_HIP_CHECK(hipGetLastError());
    return FFP_OK;
}

}  // namespace ffp
