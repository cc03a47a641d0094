// Inversion of a lower triangular 64 x 64 block mod p held in LDS, by
// doubling: with the inverses of the 1 x 1 diagonal blocks in place, the
// inverse of [M11 0; M21 M22] is [W11 0; -W22 (M21 W11), W22] for s x s
// blocks, s = 1, 2, .., 32.  Every dot product has at most 32 terms of
// centred residues and is exact (or reduced every kchunk terms when p is
// large).  Used by the triangular solves (block inverses of a triangle) and by
// the generic-rank-profile leaf (inverses of its own L and U).
#pragma once

#include "ffp_device.hpp"

namespace ffp {

constexpr int kTri = 64;

// centred residue of an integer-valued double |x| < 2^53
__device__ __forceinline__ double cmod(double x, double p, double pinv, double half) {
    const double c = mod_canon(x, p, pinv);
    return c > half ? c - p : c;
}

// One doubling step on SZ x SZ diagonal blocks: for each pair,
// Ts = M21 W11, then W21 = -W22 Ts.  W11 and W22 are lower triangular with
// zeros stored above the diagonal, so the dot products run over all SZ terms
// (fixed trip counts, fully unrolled).  A group of 256 threads (tid =
// 0..255 within the group) takes 32 SZ / 256 outputs each; every thread of
// the workgroup must call it (it contains workgroup barriers).
template <int SZ, bool RED>
__device__ __forceinline__ void inv_level(int tid, const int32_t (*Ms)[kTri + 1], double (*Ws)[kTri + 1], double *Ts,
                                          double p, double pinv, double hd, int kchunk) {
    constexpr int N2 = SZ * SZ, TOT = (kTri / 2) * SZ, PER = TOT < 256 ? 1 : TOT / 256;
    if (tid < TOT) {
        double acc[PER];
#pragma unroll
        for (int e = 0; e < PER; ++e) acc[e] = 0.0;
#pragma unroll
        for (int t = 0; t < SZ; ++t) {
#pragma unroll
            for (int e = 0; e < PER; ++e) {
                const int idx = tid + e * 256, q = idx / N2, i = (idx / SZ) % SZ, j = idx % SZ, r0 = 2 * SZ * q;
                acc[e] = fma((double)Ms[r0 + SZ + i][r0 + t], Ws[r0 + t][r0 + j], acc[e]);
            }
            if (RED && (t + 1) % kchunk == 0) {
#pragma unroll
                for (int e = 0; e < PER; ++e) acc[e] = mod_near(acc[e], p, pinv);
            }
        }
#pragma unroll
        for (int e = 0; e < PER; ++e) Ts[tid + e * 256] = cmod(acc[e], p, pinv, hd);
    }
    __syncthreads();
    if (tid < TOT) {
        double acc[PER];
#pragma unroll
        for (int e = 0; e < PER; ++e) acc[e] = 0.0;
#pragma unroll
        for (int t = 0; t < SZ; ++t) {
#pragma unroll
            for (int e = 0; e < PER; ++e) {
                const int idx = tid + e * 256, q = idx / N2, i = (idx / SZ) % SZ, j = idx % SZ, r0 = 2 * SZ * q;
                acc[e] = fma(Ws[r0 + SZ + i][r0 + SZ + t], Ts[q * N2 + t * SZ + j], acc[e]);
            }
            if (RED && (t + 1) % kchunk == 0) {
#pragma unroll
                for (int e = 0; e < PER; ++e) acc[e] = mod_near(acc[e], p, pinv);
            }
        }
#pragma unroll
        for (int e = 0; e < PER; ++e) {
            const int idx = tid + e * 256, q = idx / N2, i = (idx / SZ) % SZ, j = idx % SZ, r0 = 2 * SZ * q;
            Ws[r0 + SZ + i][r0 + j] = cmod(-acc[e], p, pinv, hd);
        }
    }
    __syncthreads();
}

typedef double v4d_t __attribute__((ext_vector_type(4)));

// The same doubling step for SZ = 16 or 32 on the FP64 matrix cores: each
// of the (32 / SZ) pairs needs (SZ / 16)^2 output tiles of 16 x 16 per
// product, one tile per wave of the group (4 waves; gw = wave in group).
// A 16 x 16 x 4 step sums 4 products, which is exact for every p the FP64
// embedding takes; with RED the accumulator is reduced every ksteps steps.
template <int SZ, bool RED>
__device__ __forceinline__ void inv_level_mfma(int tid, const int32_t (*Ms)[kTri + 1], double (*Ws)[kTri + 1],
                                               double *Ts, double p, double pinv, double hd, int ksteps) {
    constexpr int TPP = (SZ / 16) * (SZ / 16), JOBS = (32 / SZ) * TPP, N2 = SZ * SZ;
    const int gw = tid >> 6, lane = tid & 63, r16 = lane & 15, k4 = lane >> 4;
    const int job = gw, q = job / TPP, ti = (job % TPP) / (SZ / 16), tj = (job % TPP) % (SZ / 16);
    const int r0 = 2 * SZ * q;
    // Ts[q] = M21 W11 (rows r0 + SZ + 16 ti, columns r0 + 16 tj)
    if (job < JOBS) {
        v4d_t acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int ks = 0; ks < SZ / 4; ++ks) {
            const int t = ks * 4 + k4;
            const double a = (double)Ms[r0 + SZ + 16 * ti + r16][r0 + t];
            const double b = Ws[r0 + t][r0 + 16 * tj + r16];
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
            if (RED && (ks + 1) % ksteps == 0)
                for (int v = 0; v < 4; ++v) acc[v] = mod_near(acc[v], p, pinv);
        }
        // lane l holds rows l/16 + 4v of column l%16
#pragma unroll
        for (int v = 0; v < 4; ++v)
            Ts[q * N2 + (16 * ti + k4 + 4 * v) * SZ + 16 * tj + r16] = cmod(acc[v], p, pinv, hd);
    }
    __syncthreads();
    // W21 = -W22 Ts
    if (job < JOBS) {
        v4d_t acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int ks = 0; ks < SZ / 4; ++ks) {
            const int t = ks * 4 + k4;
            const double a = Ws[r0 + SZ + 16 * ti + r16][r0 + SZ + t];
            const double b = Ts[q * N2 + t * SZ + 16 * tj + r16];
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
            if (RED && (ks + 1) % ksteps == 0)
                for (int v = 0; v < 4; ++v) acc[v] = mod_near(acc[v], p, pinv);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v)
            Ws[r0 + SZ + 16 * ti + k4 + 4 * v][r0 + 16 * tj + r16] = cmod(-acc[v], p, pinv, hd);
    }
    __syncthreads();
}

// All six levels; Ws must hold the inverted diagonal and zeros elsewhere,
// Ms the strictly lower part (centred), Ts 1024 doubles of scratch.
// kchunk: terms per exact partial sum (scalar levels).
template <bool RED>
__device__ __forceinline__ void tri_inverse_levels(int tid, const int32_t (*Ms)[kTri + 1], double (*Ws)[kTri + 1],
                                                   double *Ts, double p, double pinv, double hd, int kchunk) {
    inv_level<1, RED>(tid, Ms, Ws, Ts, p, pinv, hd, kchunk);
    inv_level<2, RED>(tid, Ms, Ws, Ts, p, pinv, hd, kchunk);
    inv_level<4, RED>(tid, Ms, Ws, Ts, p, pinv, hd, kchunk);
    inv_level<8, RED>(tid, Ms, Ws, Ts, p, pinv, hd, kchunk);
    const int ksteps = kchunk / 4 < 1 ? 1 : kchunk / 4;
    inv_level_mfma<16, RED>(tid, Ms, Ws, Ts, p, pinv, hd, ksteps);
    inv_level_mfma<32, RED>(tid, Ms, Ws, Ts, p, pinv, hd, ksteps);
}

}  // namespace ffp
