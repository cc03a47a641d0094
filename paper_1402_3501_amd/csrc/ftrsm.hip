// ftrsm over Z/pZ: triangular solves, Section 2.1 (trsm).  As in the paper,
// the solve is block recursive so that almost all of its work is fgemm; the
// base case (triangles of at most kTB rows) runs in LDS with exact inverses
// of the diagonal and one delayed reduction per solved component
// (the R_trsm count of Section 3.1: one reduction for the dot product, one
// for the division by a non-unit diagonal).
#include "ffp_internal.hpp"
#include "ffp_device.hpp"

namespace ffp {

constexpr int kTB = 64;   // base-case triangle size
constexpr int kTV = 128;  // vectors per workgroup (one per thread)

// Solve, for each of nv independent vectors, x_i = (b_i - sum_{t before i} c(i,t) x_t) / diag_i
// for i in processing order (ascending if FWD, else descending), where
//   c(i,t) = swap ? T[t][i] : T[i][t]   and   diag_i = unit ? 1 : T[i][i].
// Vector v, component i lives at B[i][v] (COLS) or B[v][i].
// One thread per vector.  The coefficients sit in LDS in processing order
// (zero padded to 64, read as broadcasts).  Components are solved in four
// groups of 16 held in registers: a group first takes the contributions of
// the solved groups (kept in LDS, one column per thread), then solves its
// 16 x 16 diagonal block in registers.
template <bool RED, bool FWD, bool COLS>
__global__ __launch_bounds__(kTV) void k_trsm_base(int d, int64_t nv, const int32_t *__restrict__ T,
                                                   int64_t ldt, int32_t *__restrict__ B, int64_t ldb,
                                                   int swap, int unit, double p, double pinv, int32_t half,
                                                   int kchunk) {
    constexpr int G = 16;
    __shared__ __attribute__((aligned(16))) double Ts[kTB][kTB];
    __shared__ double Dinv[kTB];
    __shared__ double Xs[kTB][kTV + 1];
    const int tid = threadIdx.x;
    const int32_t ip = (int32_t)p;

    {
        // issue all coefficient loads before any use (out-of-triangle and
        // padding entries read T[0][0] and are zeroed afterwards)
        constexpr int PER = kTB * kTB / kTV;
        int32_t cv[PER];
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int e = tid + q * kTV, a = e / kTB, b = e % kTB;
            const bool in = b < a && a < d;
            const int i = in ? (FWD ? a : d - 1 - a) : 0, t = in ? (FWD ? b : d - 1 - b) : 0;
            cv[q] = swap ? T[(int64_t)t * ldt + i] : T[(int64_t)i * ldt + t];
        }
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int e = tid + q * kTV, a = e / kTB, b = e % kTB;
            Ts[a][b] = (b < a && a < d) ? centre(cv[q], p, half) : 0.0;
        }
    }
    for (int a = tid; a < kTB; a += kTV) {
        double dv = 1.0;
        if (a < d && !unit) {
            const int i = FWD ? a : d - 1 - a;
            dv = (double)inv_mod(T[(int64_t)i * ldt + i], ip);
        }
        Dinv[a] = dv;
    }
    __syncthreads();
    const int64_t v = (int64_t)blockIdx.x * kTV + tid;
    if (v >= nv) return;
    int32_t *base = COLS ? B + v : B + v * ldb;
    const int64_t step = COLS ? ldb : 1;
    const int ngroups = (d + G - 1) / G;
#pragma unroll 1
    for (int J = 0; J < ngroups; ++J) {
        const int a0 = J * G;
        double bj[G], acc[G], xg[G];
#pragma unroll
        for (int j = 0; j < G; ++j) {
            const int a = a0 + j;
            const int i = a < d ? (FWD ? a : d - 1 - a) : 0;
            bj[j] = (double)base[i * step];
            acc[j] = 0.0;
        }
        // contributions of the groups already solved
#pragma unroll 1
        for (int I = 0; I < J; ++I) {
#pragma unroll
            for (int t = 0; t < G; ++t) {
                const double xt = Xs[I * G + t][tid];
#pragma unroll
                for (int j = 0; j < G; ++j) acc[j] = fma(Ts[a0 + j][I * G + t], xt, acc[j]);
                if (RED && ((t + 1) % kchunk == 0)) {
#pragma unroll
                    for (int j = 0; j < G; ++j) acc[j] = mod_near(acc[j], p, pinv);
                }
            }
            if (RED) {
#pragma unroll
                for (int j = 0; j < G; ++j) acc[j] = mod_near(acc[j], p, pinv);
            }
        }
        // diagonal block
#pragma unroll
        for (int j = 0; j < G; ++j) {
            double sdiag = 0.0;
#pragma unroll
            for (int t = 0; t < j; ++t) {
                sdiag = fma(Ts[a0 + j][a0 + t], xg[t], sdiag);
                if (RED && ((t + 1) % kchunk == 0)) sdiag = mod_near(sdiag, p, pinv);
            }
            double sj = bj[j] - mod_near(acc[j], p, pinv);
            sj = mod_canon(sj - sdiag, p, pinv);
            const double xa = mod_canon(sj * Dinv[a0 + j], p, pinv);
            bj[j] = xa;
            xg[j] = xa > (double)half ? xa - p : xa;
        }
#pragma unroll
        for (int j = 0; j < G; ++j) {
            Xs[a0 + j][tid] = xg[j];
            const int a = a0 + j;
            if (a < d) base[(FWD ? a : d - 1 - a) * step] = (int32_t)bj[j];
        }
    }
}

static int trsm_base(const Field &F, int d, int64_t nv, const int32_t *T, int64_t ldt, int32_t *B,
                     int64_t ldb, bool fwd, bool swap, bool unit, bool cols_are_vectors, hipStream_t s) {
    if (d <= 0 || nv <= 0) return FFP_OK;
    // exact while 2p + (terms per sum) * half^2 < 2^53: a sum takes at most 48
    // terms unreduced, else is reduced every kchunk of its terms
    const bool red = F.kexact < 48;
    const int kchunk = (int)(F.kexact < 1 ? 1 : (F.kexact > kTB ? kTB : F.kexact));
    dim3 grid((unsigned)((nv + kTV - 1) / kTV));
#define FFP_TB(R_, F_, C_)                                                                                    \
    hipLaunchKernelGGL((k_trsm_base<R_, F_, C_>), grid, dim3(kTV), 0, s, d, nv, T, ldt, B, ldb, (int)swap, \
                       (int)unit, F.pd, F.pinv, (int32_t)F.half, kchunk)
#define FFP_TB2(R_)                                  \
    if (fwd) {                                       \
        if (cols_are_vectors) FFP_TB(R_, true, true); \
        else FFP_TB(R_, true, false);                \
    } else {                                         \
        if (cols_are_vectors) FFP_TB(R_, false, true); \
        else FFP_TB(R_, false, false);               \
    }
    if (red) { FFP_TB2(true) } else { FFP_TB2(false) }
#undef FFP_TB2
#undef FFP_TB
    FFP_HIP_CHECK(hipGetLastError());
    return FFP_OK;
}

// op(T) = trans ? T^T : T.  eff_lower: op(T) is lower triangular.
static int trsm_rec(int path, const Field &F, int side, bool eff_lower, int trans, bool unit, int64_t d,
                    int64_t nv, const int32_t *T, int64_t ldt, int32_t *B, int64_t ldb, Arena &ws,
                    hipStream_t s) {
    if (d <= 0 || nv <= 0) return FFP_OK;
    const uint32_t minus1 = F.p - 1;
    if (d <= kTB) {
        // left: x_i uses op(T)[i][t]; right: x_j uses op(T)[t][j]
        const bool fwd = side == 0 ? eff_lower : !eff_lower;
        const bool swap = (side == 1) != (trans != 0);
        return trsm_base(F, (int)d, nv, T, ldt, B, ldb, fwd, swap, unit, side == 0, s);
    }
    int64_t d1 = ((d / 2 + kTB - 1) / kTB) * kTB;
    if (d1 >= d) d1 = d / 2;
    const int64_t d2 = d - d1;
    const int32_t *T11 = T, *T22 = T + d1 * ldt + d1;
    // op(T)21 (d2 x d1) and op(T)12 (d1 x d2) as (pointer, transposed?) of the stored T
    const int32_t *op21 = trans ? T + d1 : T + d1 * ldt;   // trans: (T[0:d1, d1:d])^T
    const int32_t *op12 = trans ? T + d1 * ldt : T + d1;   // trans: (T[d1:d, 0:d1])^T
    if (side == 0) {
        int32_t *B1 = B, *B2 = B + d1 * ldb;
        if (eff_lower) {
            FFP_CHECK(trsm_rec(path, F, side, eff_lower, trans, unit, d1, nv, T11, ldt, B1, ldb, ws, s));
            FFP_CHECK(fgemm_any(path, F, trans, 0, d2, nv, d1, minus1, op21, ldt, B1, ldb, 1, B2, ldb, ws, s));
            FFP_CHECK(trsm_rec(path, F, side, eff_lower, trans, unit, d2, nv, T22, ldt, B2, ldb, ws, s));
        } else {
            FFP_CHECK(trsm_rec(path, F, side, eff_lower, trans, unit, d2, nv, T22, ldt, B2, ldb, ws, s));
            FFP_CHECK(fgemm_any(path, F, trans, 0, d1, nv, d2, minus1, op12, ldt, B2, ldb, 1, B1, ldb, ws, s));
            FFP_CHECK(trsm_rec(path, F, side, eff_lower, trans, unit, d1, nv, T11, ldt, B1, ldb, ws, s));
        }
    } else {
        int32_t *B1 = B, *B2 = B + d1;
        if (!eff_lower) {
            FFP_CHECK(trsm_rec(path, F, side, eff_lower, trans, unit, d1, nv, T11, ldt, B1, ldb, ws, s));
            FFP_CHECK(fgemm_any(path, F, 0, trans, nv, d2, d1, minus1, B1, ldb, op12, ldt, 1, B2, ldb, ws, s));
            FFP_CHECK(trsm_rec(path, F, side, eff_lower, trans, unit, d2, nv, T22, ldt, B2, ldb, ws, s));
        } else {
            FFP_CHECK(trsm_rec(path, F, side, eff_lower, trans, unit, d2, nv, T22, ldt, B2, ldb, ws, s));
            FFP_CHECK(fgemm_any(path, F, 0, trans, nv, d1, d2, minus1, B2, ldb, op21, ldt, 1, B1, ldb, ws, s));
            FFP_CHECK(trsm_rec(path, F, side, eff_lower, trans, unit, d1, nv, T11, ldt, B1, ldb, ws, s));
        }
    }
    return FFP_OK;
}

int ftrsm_run(int path, const Field &F, int side, int uplo, int trans, int diag, int64_t m, int64_t n,
              uint32_t alpha, const int32_t *T, int64_t ldt, int32_t *B, int64_t ldb, Arena &ws,
              hipStream_t s) {
    if (m <= 0 || n <= 0) return FFP_OK;
    if (!ws.counting) FFP_CHECK(scale_mat(F, m, n, alpha, B, ldb, s));
    const bool eff_lower = (uplo == 0) != (trans != 0);
    const int64_t d = side == 0 ? m : n, nv = side == 0 ? n : m;
    if (ws.counting) {
        // the recursion's products on the INT8 path need limb workspace for at most d/2 x max(d, nv)
        if (path == FFP_PATH_INT8) ws.take(fgemm_i8_ws(F, d, nv > d ? nv : d, d));
        return FFP_OK;
    }
    return trsm_rec(path, F, side, eff_lower, trans, diag != 0, d, nv, T, ldt, B, ldb, ws, s);
}

}  // namespace ffp
