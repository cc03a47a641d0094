// ftrsm over Z/pZ: triangular solves, Section 2.1 (trsm).  As in the paper,
// the solve is block recursive so that almost all of its work is fgemm.  The
// base case differs from a substitution: the inverses of all diagonal 64 x 64
// blocks are formed at once (one workgroup per block), and each base case is
// then a 64 x 64 by 64 x nv product on the FP64 matrix cores, in place.  The
// result is the same (arithmetic is exact); the chain of dependent steps of a
// solve is one inversion launch plus one product per base block.
#include "ffp_internal.hpp"
#include "ffp_device.hpp"
#include "trinv.hpp"

namespace ffp {

constexpr int kTB = 64;  // base-case triangle size

// Inverses of the diagonal 64 x 64 blocks of op(T), one workgroup per block.
// The stored triangle is read as a lower triangular Lm (transposed when the
// upper triangle is stored; rows and columns past the end are identity
// padding) and inverted by doubling: the 1 x 1 blocks are the inverses of
// the diagonal, and the inverse of [M11 0; M21 M22] is
// [W11 0; -W22 (M21 W11), W22] for s x s blocks, s = 1, 2, .., 32.  Every
// dot product has at most 32 terms of centred residues and is exact (or
// reduced every kchunk terms when p is large).  The terms of Ts = M21 W11
// with t < j and of W22 Ts with t > i are zero and are summed anyway.  op(T)^-1 is Lm^-1 when op(T)
// is lower triangular and its transpose otherwise; it is stored as 64 x 64
// centred doubles, zero outside the block.
template <bool RED>
__global__ __launch_bounds__(256) void k_trsm_inv(int64_t d, const int32_t *__restrict__ T, int64_t ldt,
                                                  int upper_stored, int unit, int eff_lower,
                                                  double *__restrict__ Winv, double p, double pinv,
                                                  int32_t half, int kchunk) {
    __shared__ int32_t Ms[kTB][kTB + 1];
    __shared__ double Ws[kTB][kTB + 1];
    __shared__ double Ts[kTB * kTB / 4];
    const int tid = threadIdx.x;
    const int64_t o = (int64_t)blockIdx.x * kTB;
    const int db = (int)(d - o < kTB ? d - o : kTB);
    const double hd = (double)half;
    {
        constexpr int PER = kTB * kTB / 256;
        int32_t v[PER];
#pragma unroll
        for (int e = 0; e < PER; ++e) {
            // coalesced along the stored row: (a, b) = (stored row, stored column)
            // unconditional (clamped) loads, all in flight together
            const int idx = tid + e * 256, a = idx / kTB, b = idx % kTB;
            v[e] = T[(o + (a < db ? a : db - 1)) * ldt + o + (b < db ? b : db - 1)];
        }
#pragma unroll
        for (int e = 0; e < PER; ++e) {
            const int idx = tid + e * 256, a = idx / kTB, b = idx % kTB;
            const bool in = a < db && b < db && (upper_stored ? b > a : b < a);
            if (!in) v[e] = 0;
            const int32_t c = v[e] > half ? v[e] - (int32_t)p : v[e];
            if (upper_stored) Ms[b][a] = c;
            else Ms[a][b] = c;
        }
    }
    for (int idx = tid; idx < kTB * kTB; idx += 256) Ws[idx / kTB][idx % kTB] = 0.0;
    __syncthreads();
    if (tid < kTB) {
        double w = 1.0;
        if (tid < db && !unit) {
            const int32_t t = T[(o + tid) * ldt + o + tid];
            const int32_t ip = (int32_t)p;
            w = (double)(p < 16777216.0 ? inv_mod_small(t, ip) : inv_mod(t, ip));
            if (w > hd) w -= p;
        }
        Ws[tid][tid] = w;
    }
    __syncthreads();
    tri_inverse_levels<RED>(tid, Ms, Ws, Ts, p, pinv, hd, kchunk);
    double *out = Winv + (int64_t)blockIdx.x * kTB * kTB;
    for (int idx = tid; idx < kTB * kTB; idx += 256) {
        const int i = idx / kTB, j = idx % kTB;
        out[idx] = (i < db && j < db) ? (eff_lower ? Ws[i][j] : Ws[j][i]) : 0.0;
    }
}

typedef double v4d __attribute__((ext_vector_type(4)));

// Base case: X = W B_b (left: B_b is db rows x nv vectors) or X = B_b W
// (right: nv vector rows x db), in place, with W the block inverse.  One
// workgroup per 64 vectors: the 64 x 64 slab is read whole into LDS, then
// multiplied on the FP64 matrix cores (4 waves, 32 x 32 each) and written
// back; slabs of different workgroups are disjoint.
template <bool LEFT, bool RED>
__device__ __forceinline__ void trsm_apply_body(int bid, int db, int64_t nv, const double *__restrict__ W,
                                                int32_t *__restrict__ B, int64_t ldb, double p, double pinv,
                                                int32_t half, int ksteps) {
    __shared__ double Ws[kTB][kTB + 2];
    __shared__ int32_t Ss[kTB][kTB + 1];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t v0 = (int64_t)bid * kTB;
    {
        constexpr int PER = kTB * kTB / 256;
        double w[PER];
        int32_t b[PER];
#pragma unroll
        for (int e = 0; e < PER; ++e) {
            const int idx = tid + e * 256, a = idx / kTB, c = idx % kTB;
            w[e] = W[idx];
            // LEFT: slab element (component a, vector c); right: (vector a, component c);
            // unconditional (clamped) loads, zeroed below when out of range
            const int ac = LEFT ? (a < db ? a : db - 1) : (v0 + a < nv ? a : (int)(nv - 1 - v0));
            const int cc = LEFT ? (v0 + c < nv ? c : (int)(nv - 1 - v0)) : (c < db ? c : db - 1);
            b[e] = LEFT ? B[ac * ldb + v0 + cc] : B[(v0 + ac) * ldb + cc];
        }
#pragma unroll
        for (int e = 0; e < PER; ++e) {
            const int idx = tid + e * 256, a = idx / kTB, c = idx % kTB;
            const bool in = LEFT ? (a < db && v0 + c < nv) : (v0 + a < nv && c < db);
            if (!in) b[e] = 0;
            Ws[a][c] = w[e];
            Ss[a][c] = b[e] > half ? b[e] - (int32_t)p : b[e];
        }
    }
    __syncthreads();
    const int wm0 = (wave >> 1) * 32, wn0 = (wave & 1) * 32;
    v4d acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = v4d{0.0, 0.0, 0.0, 0.0};
    const int nks = (db + 3) / 4;
    int steps = 0;
    for (int ks = 0; ks < nks; ++ks) {
        const int kr = ks * 4 + (lane >> 4);
        double a[2], b[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const int r = wm0 + i * 16 + (lane & 15);
            a[i] = LEFT ? Ws[r][kr] : (double)Ss[r][kr];
        }
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int c = wn0 + j * 16 + (lane & 15);
            b[j] = LEFT ? (double)Ss[kr][c] : Ws[kr][c];
        }
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
        if (RED && ++steps == ksteps) {
            steps = 0;
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
#pragma unroll
                    for (int v = 0; v < 4; ++v) acc[i][j][v] = mod_near(acc[i][j][v], p, pinv);
        }
    }
    // lane l holds rows l/16 + 4v of column l%16 of each 16 x 16 block
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int r = wm0 + i * 16 + (lane >> 4) + 4 * v, c = wn0 + j * 16 + (lane & 15);
                const int32_t x = (int32_t)mod_canon(acc[i][j][v], p, pinv);
                if (LEFT) {
                    if (r < db && v0 + c < nv) B[r * ldb + v0 + c] = x;
                } else {
                    if (v0 + r < nv && c < db) B[(v0 + r) * ldb + c] = x;
                }
            }
}

template <bool LEFT, bool RED>
__global__ __launch_bounds__(256) void k_trsm_apply(int db, int64_t nv, const double *__restrict__ W,
                                                    int32_t *__restrict__ B, int64_t ldb, double p, double pinv,
                                                    int32_t half, int ksteps) {
    trsm_apply_body<LEFT, RED>(blockIdx.x, db, nv, W, B, ldb, p, pinv, half, ksteps);
}

constexpr int kTBB = 256;  // fused base case: up to four 64-blocks

// Fused base case for triangles of up to 256: one workgroup per 16 vectors
// keeps its slab (d components x 16 vectors, centred int32) in LDS and runs
// the block substitution
//   X_t = W_t (B_t - sum_{s solved} M(t, s) X_s)
// over the 64-blocks t in dependency order, every product on the FP64
// matrix cores: 1 + 2 + .. + nb products of 64 x 16 x 64 in one launch
// instead of nb applications and nb - 1 products in separate launches.  A
// product is one 16 x 16 output tile per wave (wave w: components
// 16 w .. 16 w + 15 of the block); narrow slabs spread a solve over many
// compute units, which is what bounds these small products.  The right-side
// solve is the same computation on the transposed slab (operands
// transposed).  Each wave reads its A-operand fragments straight from global
// memory into registers, three products ahead of the one that runs.
//   M(t, s)[i][k] = direct ? T[64t + i][64s + k] : T[64s + k][64t + i]
//   W_t = op(T)_tt^-1 (64 x 64 centred doubles), taken as is (left) or
//   transposed (right).
constexpr int kVB = 16;  // vectors per workgroup of the fused base case
constexpr int kWideGroups = 1024;  // 16-wide groups from which the paired base runs 32 wide

// NBT > 0: d == 64 NBT and T's rows are 16-byte aligned (host-checked), so
// that the item count and every load's form are compile-time: no branch
// between a fragment load and its use, and the loads of several items stay in
// flight together (a branch join makes the wait conservative).
// VB vectors per workgroup (16 or 32): each wave then computes VB / 16
// output tiles of 16 x 16 from the same operand fragments.
template <bool LEFT, bool RED, int NBT = 0, int VB = kVB>
__device__ __forceinline__ void trsm_blk_body(int32_t (&S)[kTBB][VB + 1], int bid, int d, int64_t nv,
                                              const int32_t *__restrict__ T, int64_t ldt, int direct, int fwd,
                                              const double *__restrict__ W, int32_t *__restrict__ B, int64_t ldb,
                                              double p, double pinv, int32_t half, int ksteps) {
    constexpr int KS = kTB / 4;  // k-steps per 64 x 16 x 64 product
    constexpr int CT = VB / 16;  // column tiles per wave
    // S: the slab in LDS, [component][vector]
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int r16 = lane & 15, k4 = lane >> 4;
    const int64_t v0 = (int64_t)bid * VB;
    const int nb = NBT > 0 ? NBT : (d + kTB - 1) / kTB;
    const double hd = (double)half;
    const int32_t ip = (int32_t)p;
    // items: for q = 0.., the sources r < q then the inverse of block q
    const int nitems = nb * (nb + 1) / 2;
    auto item = [&](int it, int &q, int &r) {
        q = 0;
        while ((q + 1) * (q + 2) / 2 <= it) ++q;
        r = it - q * (q + 1) / 2;
    };
    auto blk = [&](int x) { return fwd ? x : nb - 1 - x; };
    // A fragments of this lane: row 16 wave + r16 of the block, and the
    // reduction index k = 16 k4 + ks at k-step ks (the sum over k may run in
    // any order as long as the S operand uses the same one), so that each
    // lane reads 16 consecutive entries of a row of T or W
    const int arow = 16 * wave + r16;
    const bool vec = NBT > 0 || (((uintptr_t)T | (uintptr_t)(ldt * 4)) & 15) == 0;
    // operand fragments in flight: a ring of PD raw slots (16 int32 entries
    // of T, or 16 doubles of W as 32 words), filled PD items ahead so that
    // several global reads overlap the products
    constexpr int PD = RED ? 1 : 3;  // the reducing variant has no registers to spare
    constexpr int MAXIT = (kTBB / kTB) * (kTBB / kTB + 1) / 2;
    uint32_t ring[PD][2 * KS];
    auto prefetch = [&](int it, uint32_t(&sl)[2 * KS]) {
        int q, r;
        item(it, q, r);
        const int t = blk(q);
        if (r < q) {
            const int sb = blk(r);
            if (direct) {
                const int a = 64 * t + arow, b0 = 64 * sb + 16 * k4;
                const int32_t *row = T + (int64_t)(a < d ? a : d - 1) * ldt;
                if (NBT > 0 || (vec && b0 + KS <= d)) {
#pragma unroll
                    for (int v = 0; v < KS / 4; ++v) {
                        const uint4 x = *(const uint4 *)(row + b0 + 4 * v);
                        sl[4 * v] = x.x;
                        sl[4 * v + 1] = x.y;
                        sl[4 * v + 2] = x.z;
                        sl[4 * v + 3] = x.w;
                    }
                } else {
#pragma unroll
                    for (int ks = 0; ks < KS; ++ks) {
                        const int b = b0 + ks;
                        sl[ks] = (uint32_t)row[b < d ? b : d - 1];
                    }
                }
            } else {
                const int b = 64 * t + arow;
                const int bc = b < d ? b : d - 1;
#pragma unroll
                for (int ks = 0; ks < KS; ++ks) {
                    const int a = 64 * sb + 16 * k4 + ks;
                    sl[ks] = (uint32_t)T[(int64_t)(a < d ? a : d - 1) * ldt + bc];
                }
            }
        } else {
            const double *Wt = W + (int64_t)t * kTB * kTB;
            if (LEFT) {
                const uint4 *w4 = (const uint4 *)(Wt + arow * kTB + 16 * k4);
#pragma unroll
                for (int v = 0; v < KS / 2; ++v) {
                    const uint4 x = w4[v];
                    sl[4 * v] = x.x;
                    sl[4 * v + 1] = x.y;
                    sl[4 * v + 2] = x.z;
                    sl[4 * v + 3] = x.w;
                }
            } else {
#pragma unroll
                for (int ks = 0; ks < KS; ++ks) {
                    const uint2 x = *(const uint2 *)(Wt + (16 * k4 + ks) * kTB + arow);
                    sl[2 * ks] = x.x;
                    sl[2 * ks + 1] = x.y;
                }
            }
        }
    };
    v4d acc[CT];
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) acc[ct] = v4d{0.0, 0.0, 0.0, 0.0};
    // ac += A S[row0 .. row0 + 63][*], A in registers, for each column tile
    auto product = [&](const double (&av)[KS], int row0, v4d (&ac)[CT]) {
        int32_t bv[CT][KS];
#pragma unroll
        for (int ct = 0; ct < CT; ++ct)
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) bv[ct][ks] = S[row0 + 16 * k4 + ks][16 * ct + r16];
        int steps = 0;
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
#pragma unroll
            for (int ct = 0; ct < CT; ++ct)
                ac[ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[ks], (double)bv[ct][ks], ac[ct], 0, 0, 0);
            if (RED && ++steps == ksteps) {
                steps = 0;
#pragma unroll
                for (int ct = 0; ct < CT; ++ct)
#pragma unroll
                    for (int v = 0; v < 4; ++v) ac[ct][v] = mod_near(ac[ct][v], p, pinv);
            }
        }
        // keep partial sums bounded across several products
#pragma unroll
        for (int ct = 0; ct < CT; ++ct)
#pragma unroll
            for (int v = 0; v < 4; ++v) ac[ct][v] = mod_near(ac[ct][v], p, pinv);
    };
#pragma unroll
    for (int j = 0; j < PD; ++j)
        if (j < nitems) prefetch(j, ring[j]);
    // (the slab's loads go out after the first operands': one wait covers both)
    // ---- slab in (clamped loads, zero outside)
    {
        constexpr int PER = kTBB * VB / 256;
        int32_t v[PER];
#pragma unroll
        for (int e = 0; e < PER; ++e) {
            const int idx = tid + e * 256;
            const int c = LEFT ? idx / VB : idx % kTBB, w = LEFT ? idx % VB : idx / kTBB;
            const int cc = c < d ? c : d - 1;
            const int64_t vv = v0 + w < nv ? v0 + w : nv - 1;
            v[e] = LEFT ? B[(int64_t)cc * ldb + vv] : B[vv * ldb + cc];
        }
#pragma unroll
        for (int e = 0; e < PER; ++e) {
            const int idx = tid + e * 256;
            const int c = LEFT ? idx / VB : idx % kTBB, w = LEFT ? idx % VB : idx / kTBB;
            const int32_t x = (c < d && v0 + w < nv) ? v[e] : 0;
            S[c][w] = x > half ? x - ip : x;
        }
    }
    __syncthreads();
    auto run_item = [&](int it, uint32_t(&sl)[2 * KS]) {
        int q, r;
        item(it, q, r);
        const int t = blk(q);
        // this item's operand (its slot is refilled below)
        double av[KS];
        if (r < q) {
            const int sb = blk(r);
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) {
                const bool in = 64 * t + arow < d && 64 * sb + 16 * k4 + ks < d;
                const int32_t x = in ? (int32_t)sl[ks] : 0;
                av[ks] = x > half ? (double)(x - ip) : (double)x;
            }
        } else {
#pragma unroll
            for (int ks = 0; ks < KS; ++ks)
                av[ks] = __builtin_bit_cast(double, ((uint64_t)sl[2 * ks + 1] << 32) | sl[2 * ks]);
        }
        if (it + PD < nitems) prefetch(it + PD, sl);
        if (r < q) {
            product(av, 64 * blk(r), acc);
        } else {
            // lane l holds rows l/16 + 4v of column l%16 of the wave's tile
            if (q > 0) {
                // S_t <- S_t - (sum of the source products)
#pragma unroll
                for (int ct = 0; ct < CT; ++ct)
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int row = 64 * t + 16 * wave + k4 + 4 * v;
                        S[row][16 * ct + r16] = (int32_t)cmod((double)S[row][16 * ct + r16] - acc[ct][v], p, pinv, hd);
                        acc[ct][v] = 0.0;
                    }
                __syncthreads();
            }
            v4d x2[CT];
#pragma unroll
            for (int ct = 0; ct < CT; ++ct) x2[ct] = v4d{0.0, 0.0, 0.0, 0.0};
            product(av, 64 * t, x2);
            __syncthreads();  // every read of S_t is done
#pragma unroll
            for (int ct = 0; ct < CT; ++ct)
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    S[64 * t + 16 * wave + k4 + 4 * v][16 * ct + r16] = (int32_t)cmod(x2[ct][v], p, pinv, hd);
            __syncthreads();
        }
    };
    if constexpr (PD == 1) {
        for (int it = 0; it < nitems; ++it) run_item(it, ring[0]);
    } else {
        // fully unrolled (guards, no break) so that every ring slot is a
        // fixed set of registers
#pragma unroll
        for (int it = 0; it < MAXIT; ++it)
            if (it < nitems) run_item(it, ring[it % PD]);
    }
    // ---- slab out
    for (int idx = tid; idx < kTBB * VB; idx += 256) {
        const int c = LEFT ? idx / VB : idx % kTBB, w = LEFT ? idx % VB : idx / kTBB;
        if (c < d && v0 + w < nv) {
            const int32_t x = S[c][w];
            const int32_t y = x < 0 ? x + ip : x;
            if (LEFT) B[(int64_t)c * ldb + v0 + w] = y;
            else B[(v0 + w) * ldb + c] = y;
        }
    }
}

template <bool LEFT, bool RED>
__global__ __launch_bounds__(256) void k_trsm_blk(int d, int64_t nv, const int32_t *__restrict__ T, int64_t ldt,
                                                  int direct, int fwd, const double *__restrict__ W,
                                                  int32_t *__restrict__ B, int64_t ldb, double p, double pinv,
                                                  int32_t half, int ksteps) {
    __shared__ int32_t S[kTBB][kVB + 1];
    trsm_blk_body<LEFT, RED>(S, blockIdx.x, d, nv, T, ldt, direct, fwd, W, B, ldb, p, pinv, half, ksteps);
}

// The two panel solves of a generic block LU node in one launch, for a
// leading block of h <= 256 (one base case each): D = L^-1 B (left, lower,
// forward) on the first gd workgroups and E = C U^-1 (right, upper, forward)
// on the rest; they read the same diagonal block and write disjoint panels.
template <bool RED>
__global__ __launch_bounds__(256) void k_trsm_apply_pair(int h, int gd, int64_t nvd, int32_t *__restrict__ Bd,
                                                         int64_t nve, int32_t *__restrict__ Be, int64_t ldb,
                                                         const double *__restrict__ Li,
                                                         const double *__restrict__ Ui, double p, double pinv,
                                                         int32_t half, int ksteps) {
    if ((int)blockIdx.x < gd) trsm_apply_body<true, RED>(blockIdx.x, h, nvd, Li, Bd, ldb, p, pinv, half, ksteps);
    else trsm_apply_body<false, RED>(blockIdx.x - gd, h, nve, Ui, Be, ldb, p, pinv, half, ksteps);
}
template <bool RED, int NBT, int VB>
__global__ __launch_bounds__(256) void k_trsm_blk_pair(int h, int gd, int64_t nvd, int32_t *__restrict__ Bd,
                                                       int64_t nve, int32_t *__restrict__ Be, int64_t ldb,
                                                       const int32_t *__restrict__ T, int64_t ldt,
                                                       const double *__restrict__ Li, const double *__restrict__ Ui,
                                                       double p, double pinv, int32_t half, int ksteps) {
    __shared__ int32_t S[kTBB][VB + 1];  // one slab for either side
    if ((int)blockIdx.x < gd)
        trsm_blk_body<true, RED, NBT, VB>(S, blockIdx.x, h, nvd, T, ldt, 1, 1, Li, Bd, ldb, p, pinv, half, ksteps);
    else
        trsm_blk_body<false, RED, NBT, VB>(S, blockIdx.x - gd, h, nve, T, ldt, 0, 1, Ui, Be, ldb, p, pinv, half,
                                           ksteps);
}

static int trsm_blk(const Field &F, int side, int d, int64_t nv, const int32_t *T, int64_t ldt, bool direct,
                    bool fwd, const double *W, int32_t *B, int64_t ldb, hipStream_t s) {
    if (d <= 0 || nv <= 0) return FFP_OK;
    const bool red = F.kexact < kTB;
    const int ksteps = (int)(F.kexact / 4 < 1 ? 1 : (F.kexact / 4 > 16 ? 16 : F.kexact / 4));
    dim3 grid((unsigned)((nv + kVB - 1) / kVB));
    ProfScope prof(PK_TRSM, (double)d * (double)d * (double)nv, s, 4.0 * (double)d * (double)d / 2.0 + 8.0 * (double)d * (double)nv);
#define FFP_TBK(L_, R_)                                                                                          \
    hipLaunchKernelGGL((k_trsm_blk<L_, R_>), grid, dim3(256), 0, s, d, nv, T, ldt, (int)direct, (int)fwd, W, B, ldb, \
                       F.pd, F.pinv, (int32_t)F.half, ksteps)
    if (side == 0) {
        if (red) FFP_TBK(true, true);
        else FFP_TBK(true, false);
    } else {
        if (red) FFP_TBK(false, true);
        else FFP_TBK(false, false);
    }
#undef FFP_TBK
    FFP_HIP_CHECK(hipGetLastError());
    return FFP_OK;
}

static int trsm_apply(const Field &F, int side, int db, int64_t nv, const double *W, int32_t *B, int64_t ldb,
                      hipStream_t s) {
    if (db <= 0 || nv <= 0) return FFP_OK;
    // a k-step adds 4 products; exact while 2p + terms * half^2 < 2^53
    const bool red = F.kexact < db;
    const int ksteps = (int)(F.kexact / 4 < 1 ? 1 : (F.kexact / 4 > 16 ? 16 : F.kexact / 4));
    dim3 grid((unsigned)((nv + kTB - 1) / kTB));
    ProfScope prof(PK_TRSM, (double)db * (double)db * (double)nv, s, 8.0 * (double)db * (double)nv);
#define FFP_TA(L_, R_)                                                                                    \
    hipLaunchKernelGGL((k_trsm_apply<L_, R_>), grid, dim3(256), 0, s, db, nv, W, B, ldb, F.pd, F.pinv, \
                       (int32_t)F.half, ksteps)
    if (side == 0) {
        if (red) FFP_TA(true, true);
        else FFP_TA(true, false);
    } else {
        if (red) FFP_TA(false, true);
        else FFP_TA(false, false);
    }
#undef FFP_TA
    FFP_HIP_CHECK(hipGetLastError());
    return FFP_OK;
}

// op(T) = trans ? T^T : T.  eff_lower: op(T) is lower triangular.  Split
// points are multiples of 256 from the origin of the top-level triangle, so
// every base case is made of whole diagonal 64-blocks, whose inverses are W.
static int trsm_rec(int path, const Field &F, int side, bool eff_lower, int trans, int64_t d, int64_t nv,
                    const int32_t *T, int64_t ldt, int32_t *B, int64_t ldb, const double *W, Arena &ws,
                    hipStream_t s) {
    if (d <= 0 || nv <= 0) return FFP_OK;
    const uint32_t minus1 = F.p - 1;
    if (d <= kTB) return trsm_apply(F, side, (int)d, nv, W, B, ldb, s);
    if (d <= kTBB) {
        const bool fwd = side == 0 ? eff_lower : !eff_lower;
        const bool direct = (side == 0) == (trans == 0);
        return trsm_blk(F, side, (int)d, nv, T, ldt, direct, fwd, W, B, ldb, s);
    }
    // split at a multiple of 256 (the fused base) below d
    const int64_t d1 = ((d / 2 + kTBB - 1) / kTBB) * kTBB < d ? ((d / 2 + kTBB - 1) / kTBB) * kTBB : kTBB;
    const int64_t d2 = d - d1;
    const int32_t *T11 = T, *T22 = T + d1 * ldt + d1;
    const double *W1 = W, *W2 = W + (d1 / kTB) * kTB * kTB;
    // op(T)21 (d2 x d1) and op(T)12 (d1 x d2) as (pointer, transposed?) of the stored T
    const int32_t *op21 = trans ? T + d1 : T + d1 * ldt;   // trans: (T[0:d1, d1:d])^T
    const int32_t *op12 = trans ? T + d1 * ldt : T + d1;   // trans: (T[d1:d, 0:d1])^T
    if (side == 0) {
        int32_t *B1 = B, *B2 = B + d1 * ldb;
        if (eff_lower) {
            FFP_CHECK(trsm_rec(path, F, side, eff_lower, trans, d1, nv, T11, ldt, B1, ldb, W1, ws, s));
            FFP_CHECK(fgemm_any(path, F, trans, 0, d2, nv, d1, minus1, op21, ldt, B1, ldb, 1, B2, ldb, ws, s));
            FFP_CHECK(trsm_rec(path, F, side, eff_lower, trans, d2, nv, T22, ldt, B2, ldb, W2, ws, s));
        } else {
            FFP_CHECK(trsm_rec(path, F, side, eff_lower, trans, d2, nv, T22, ldt, B2, ldb, W2, ws, s));
            FFP_CHECK(fgemm_any(path, F, trans, 0, d1, nv, d2, minus1, op12, ldt, B2, ldb, 1, B1, ldb, ws, s));
            FFP_CHECK(trsm_rec(path, F, side, eff_lower, trans, d1, nv, T11, ldt, B1, ldb, W1, ws, s));
        }
    } else {
        int32_t *B1 = B, *B2 = B + d1;
        if (!eff_lower) {
            FFP_CHECK(trsm_rec(path, F, side, eff_lower, trans, d1, nv, T11, ldt, B1, ldb, W1, ws, s));
            FFP_CHECK(fgemm_any(path, F, 0, trans, nv, d2, d1, minus1, B1, ldb, op12, ldt, 1, B2, ldb, ws, s));
            FFP_CHECK(trsm_rec(path, F, side, eff_lower, trans, d2, nv, T22, ldt, B2, ldb, W2, ws, s));
        } else {
            FFP_CHECK(trsm_rec(path, F, side, eff_lower, trans, d2, nv, T22, ldt, B2, ldb, W2, ws, s));
            FFP_CHECK(fgemm_any(path, F, 0, trans, nv, d1, d2, minus1, B2, ldb, op21, ldt, 1, B1, ldb, ws, s));
            FFP_CHECK(trsm_rec(path, F, side, eff_lower, trans, d1, nv, T11, ldt, B1, ldb, W1, ws, s));
        }
    }
    return FFP_OK;
}

int ftrsm_run(int path, const Field &F, int side, int uplo, int trans, int diag, int64_t m, int64_t n,
              uint32_t alpha, const int32_t *T, int64_t ldt, int32_t *B, int64_t ldb, Arena &ws,
              hipStream_t s) {
    if (m <= 0 || n <= 0) return FFP_OK;
    const bool eff_lower = (uplo == 0) != (trans != 0);
    const int64_t d = side == 0 ? m : n, nv = side == 0 ? n : m;
    const int64_t nblk = (d + kTB - 1) / kTB;
    const size_t mk = ws.mark();
    double *W = (double *)ws.take((size_t)nblk * kTB * kTB * sizeof(double));
    if (ws.counting) {
        // the recursion's products on the INT8 path need limb workspace for at most d/2 x max(d, nv)
        if (path == FFP_PATH_INT8) ws.take(fgemm_i8_ws(F, d, nv > d ? nv : d, d));
        ws.release(mk);
        return FFP_OK;
    }
    if (!W) return FFP_E_WORKSPACE;
    FFP_CHECK(scale_mat(F, m, n, alpha, B, ldb, s));
    // dot products of the inversion take at most 32 terms
    const bool red = F.kexact < 32;
    const int kchunk = (int)(F.kexact < 1 ? 1 : (F.kexact > 32 ? 32 : F.kexact));
    ProfScope prof(PK_TRSM, 0.0, s, 4.0 * (double)d * (double)d / 2.0 + 8.0 * (double)nblk * kTB * kTB);
#define FFP_TI(R_)                                                                                          \
    hipLaunchKernelGGL((k_trsm_inv<R_>), dim3((unsigned)nblk), dim3(256), 0, s, d, T, ldt, uplo, diag, \
                       (int)eff_lower, W, F.pd, F.pinv, (int32_t)F.half, kchunk)
    if (red) FFP_TI(true);
    else FFP_TI(false);
#undef FFP_TI
    FFP_HIP_CHECK(hipGetLastError());
    FFP_CHECK(trsm_rec(path, F, side, eff_lower, trans, d, nv, T, ldt, B, ldb, W, ws, s));
    ws.release(mk);
    return FFP_OK;
}

int ftrsm_with_inverses(int path, const Field &F, int side, bool lower, int64_t m, int64_t n,
                        const int32_t *T, int64_t ldt, int32_t *B, int64_t ldb, const double *W, Arena &ws,
                        hipStream_t s) {
    if (m <= 0 || n <= 0) return FFP_OK;
    const int64_t d = side == 0 ? m : n, nv = side == 0 ? n : m;
    return trsm_rec(path, F, side, lower, 0, d, nv, T, ldt, B, ldb, W, ws, s);
}

static int trsm_pair_base(const Field &F, int64_t h, const int32_t *T, int64_t ldt, int64_t nvd, int32_t *Bd,
                          int64_t nve, int32_t *Be, int64_t ldb, const double *Li, const double *Ui, hipStream_t s) {
    if (h <= 0 || h > kTBB || (nvd <= 0 && nve <= 0)) return FFP_OK;
    const int ksteps = (int)(F.kexact / 4 < 1 ? 1 : (F.kexact / 4 > 16 ? 16 : F.kexact / 4));
    ProfScope prof(PK_TRSM, (double)h * (double)h * (double)(nvd + nve), s,
                   4.0 * (double)h * (double)h + 8.0 * (double)h * (double)(nvd + nve));
    if (h <= kTB) {
        const bool red = F.kexact < h;
        const int gd = (int)((nvd + kTB - 1) / kTB), ge = (int)((nve + kTB - 1) / kTB);
#define FFP_AP(R_)                                                                                          \
    hipLaunchKernelGGL((k_trsm_apply_pair<R_>), dim3((unsigned)(gd + ge)), dim3(256), 0, s, (int)h, gd, nvd, Bd, \
                       nve, Be, ldb, Li, Ui, F.pd, F.pinv, (int32_t)F.half, ksteps)
        if (red) FFP_AP(true);
        else FFP_AP(false);
#undef FFP_AP
    } else {
        const bool red = F.kexact < kTB;
        // 32 vectors per workgroup once the 16-wide grid holds at least
        // kWideGroups groups: each operand fragment then feeds two MFMA tiles
        const bool wide = (nvd + kVB - 1) / kVB + (nve + kVB - 1) / kVB >= kWideGroups;
        const int vb = wide ? 2 * kVB : kVB;
        const int gd = (int)((nvd + vb - 1) / vb), ge = (int)((nve + vb - 1) / vb);
        // whole 64-blocks and aligned rows: the item count is a template argument
        const bool aligned = (((uintptr_t)T | (uintptr_t)(ldt * 4)) & 15) == 0;
        const int nbt = (aligned && h % kTB == 0) ? (int)(h / kTB) : 0;
#define FFP_BP(R_, N_, V_)                                                                                   \
    hipLaunchKernelGGL((k_trsm_blk_pair<R_, N_, V_>), dim3((unsigned)(gd + ge)), dim3(256), 0, s, (int)h, gd, \
                       nvd, Bd, nve, Be, ldb, T, ldt, Li, Ui, F.pd, F.pinv, (int32_t)F.half, ksteps)
#define FFP_BPN(R_, V_)                   \
    switch (nbt) {                        \
        case 2: FFP_BP(R_, 2, V_); break; \
        case 3: FFP_BP(R_, 3, V_); break; \
        case 4: FFP_BP(R_, 4, V_); break; \
        default: FFP_BP(R_, 0, V_); break; \
    }
        if (wide) {
            if (red) FFP_BPN(true, 2 * kVB)
            else FFP_BPN(false, 2 * kVB)
        } else {
            if (red) FFP_BPN(true, kVB)
            else FFP_BPN(false, kVB)
        }
#undef FFP_BPN
#undef FFP_BP
    }
    FFP_HIP_CHECK(hipGetLastError());
    return FFP_OK;
}

// Both solves recurse in step (forward, the same 256-multiple splits): each
// level's two base cases share one launch, and the two products between them
// run back to back on the same stream.
int ftrsm_pair_gen(int path, const Field &F, int64_t h, const int32_t *T, int64_t ldt, int64_t nvd, int32_t *Bd,
                   int64_t nve, int32_t *Be, int64_t ldb, const double *Li, const double *Ui, Arena &ws,
                   hipStream_t s) {
    if (h <= 0 || (nvd <= 0 && nve <= 0)) return FFP_OK;
    if (h <= kTBB) return trsm_pair_base(F, h, T, ldt, nvd, Bd, nve, Be, ldb, Li, Ui, s);
    const uint32_t minus1 = F.p - 1;
    const int64_t d1 = ((h / 2 + kTBB - 1) / kTBB) * kTBB < h ? ((h / 2 + kTBB - 1) / kTBB) * kTBB : kTBB;
    const int64_t d2 = h - d1, off = (d1 / kTB) * kTB * kTB;
    FFP_CHECK(ftrsm_pair_gen(path, F, d1, T, ldt, nvd, Bd, nve, Be, ldb, Li, Ui, ws, s));
    // D2 -= L21 D1 (rows d1.. of the left panel), E2 -= E1 U12 (columns d1.. of the right one);
    // both on the FP64 path: one launch
    auto on_fp64 = [&](int64_t mm, int64_t nn) {
        const int eff = path == FFP_PATH_AUTO ? resolve_path(path, F.p, mm, nn, d1) : path;
        return !(eff == FFP_PATH_INT8 && F.limbs > 0);
    };
    if (!ws.counting && nvd > 0 && nve > 0 && on_fp64(d2, nvd) && on_fp64(nve, d2)) {
        FFP_CHECK(fgemm_f64_pair(F, d2, nvd, T + d1 * ldt, ldt, Bd, ldb, Bd + d1 * ldb, ldb, nve, d2, Be, ldb, T + d1,
                                 ldt, Be + d1, ldb, d1, minus1, 1, s));
    } else if (nvd > 0 && nve > 0 && F.limbs > 0 && !on_fp64(d2, nvd) && !on_fp64(nve, d2)) {
        // both on INT8: one limb split and one product grid for the two
        FFP_CHECK(fgemm_i8_pair(F, d1, minus1, 1, d2, nvd, T + d1 * ldt, ldt, Bd, ldb, Bd + d1 * ldb, ldb, nve, d2,
                                Be, ldb, T + d1, ldt, Be + d1, ldb, ws, s));
    } else {
        if (nvd > 0)
            FFP_CHECK(fgemm_any(path, F, 0, 0, d2, nvd, d1, minus1, T + d1 * ldt, ldt, Bd, ldb, 1, Bd + d1 * ldb, ldb,
                                ws, s));
        if (nve > 0)
            FFP_CHECK(fgemm_any(path, F, 0, 0, nve, d2, d1, minus1, Be, ldb, T + d1, ldt, 1, Be + d1, ldb, ws, s));
    }
    return ftrsm_pair_gen(path, F, d2, T + d1 * ldt + d1, ldt, nvd, Bd + d1 * ldb, nve, Be + d1, ldb, Li + off,
                          Ui + off, ws, s);
}

size_t ftrsm_ws(int path, const Field &F, int side, int64_t m, int64_t n) {
    Arena a;
    a.counting = true;
    ftrsm_run(path, F, side, 0, 0, 0, m, n, 1, nullptr, 1, nullptr, 1, a, nullptr);
    return a.peak;
}

}  // namespace ffp
