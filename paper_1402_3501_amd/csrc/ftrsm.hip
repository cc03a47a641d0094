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
constexpr int kTV = 64;   // vectors per workgroup (one per thread)

// Solve, for each of nv independent vectors, x_i = (b_i - sum_{t before i} c(i,t) x_t) / diag_i
// for i in processing order (ascending if fwd, else descending), where
//   c(i,t) = swap ? T[t][i] : T[i][t]   and   diag_i = unit ? 1 : T[i][i].
// Vector v, component i lives at B[i][v] (cols_are_vectors) or B[v][i].
template <bool RED>
__global__ __launch_bounds__(kTV) void k_trsm_base(int d, int64_t nv, const int32_t *__restrict__ T,
                                                   int64_t ldt, int32_t *__restrict__ B, int64_t ldb,
                                                   int fwd, int swap, int unit, int cols_are_vectors,
                                                   double p, double pinv, int32_t half, int kchunk) {
    __shared__ double Ts[kTB][kTB];
    __shared__ double Xs[kTB][kTV + 1];
    __shared__ double Dinv[kTB];
    const int tid = threadIdx.x;
    const int64_t v = (int64_t)blockIdx.x * kTV + tid;
    const int32_t ip = (int32_t)p;

    // coefficients in "processing order" positions: row a (a-th processed) holds
    // c(i_a, i_b) at column b for b < a
    for (int e = tid; e < d * d; e += kTV) {
        const int a = e / d, b = e % d;
        double val = 0.0;
        if (b < a) {
            const int i = fwd ? a : d - 1 - a, t = fwd ? b : d - 1 - b;
            const int32_t c = swap ? T[(int64_t)t * ldt + i] : T[(int64_t)i * ldt + t];
            val = centre(c, p, half);
        }
        Ts[a][b] = val;
    }
    for (int a = tid; a < d; a += kTV) {
        const int i = fwd ? a : d - 1 - a;
        Dinv[a] = unit ? 1.0 : (double)inv_mod(T[(int64_t)i * ldt + i], ip);
    }
    __syncthreads();
    if (v < nv) {
        for (int a = 0; a < d; ++a) {
            const int i = fwd ? a : d - 1 - a;
            const int64_t off = cols_are_vectors ? (int64_t)i * ldb + v : v * ldb + i;
            double acc = 0.0;
            if (!RED) {
                for (int b = 0; b < a; ++b) acc = fma(Ts[a][b], Xs[b][tid], acc);
            } else {
                int cnt = 0;
                for (int b = 0; b < a; ++b) {
                    acc = fma(Ts[a][b], Xs[b][tid], acc);
                    if (++cnt == kchunk) { acc = mod_near(acc, p, pinv); cnt = 0; }
                }
            }
            double x = mod_canon((double)B[off] - acc, p, pinv);
            x = mod_canon(x * Dinv[a], p, pinv);
            B[off] = (int32_t)x;
            Xs[a][tid] = x > (double)half ? x - p : x;
        }
    }
}

static int trsm_base(const Field &F, int d, int64_t nv, const int32_t *T, int64_t ldt, int32_t *B,
                     int64_t ldb, bool fwd, bool swap, bool unit, bool cols_are_vectors, hipStream_t s) {
    if (d <= 0 || nv <= 0) return FFP_OK;
    const bool red = F.kexact < kTB;
    const int kchunk = (int)(F.kexact < 1 ? 1 : (F.kexact > kTB ? kTB : F.kexact));
    dim3 grid((unsigned)((nv + kTV - 1) / kTV));
    if (red)
        hipLaunchKernelGGL((k_trsm_base<true>), grid, dim3(kTV), 0, s, d, nv, T, ldt, B, ldb, (int)fwd,
                           (int)swap, (int)unit, (int)cols_are_vectors, F.pd, F.pinv, (int32_t)F.half, kchunk);
    else
        hipLaunchKernelGGL((k_trsm_base<false>), grid, dim3(kTV), 0, s, d, nv, T, ldt, B, ldb, (int)fwd,
                           (int)swap, (int)unit, (int)cols_are_vectors, F.pd, F.pinv, (int32_t)F.half, kchunk);
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
