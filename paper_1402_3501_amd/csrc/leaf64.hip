// PLUQ leaf for blocks of at most 64 x 64, one wave64 per block.
//
// Same result as the tile recursion of Section 4.1 applied to the block (see
// pluq.hip): the quadrant recursion is walked with an explicit stack to find
// each pivot (first nonzero of a one-row region, or of a one-column region),
// and each pivot is applied at once as a rank-one update of the remaining
// block.  The block lives in LDS as FP64-embedded centred residues with
// delayed reduction (one reduction per element only when the bound of
// Section 3.1 is reached); lane c owns column c.  Row / column sets are
// 64-bit masks; the stack is spread over the lanes (lane d holds the frame
// at depth d) and read with uniform lane indices, so the walk runs on the
// scalar unit.  The pivot search is one ballot, the inverse one extended
// Euclid on the pivot.
#include <type_traits>

#include "ffp_internal.hpp"
#include "ffp_device.hpp"
#include "trinv.hpp"

namespace ffp {

__device__ __forceinline__ uint64_t rl64(uint64_t v, int lane) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, lane);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), lane);
    return ((uint64_t)hi << 32) | lo;
}
__device__ __forceinline__ double rld(double v, int lane) {
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    return __builtin_bit_cast(double, rl64(b, lane));
}
// the first k set bits of x (0 <= k <= popcount(x))
__device__ __forceinline__ uint64_t first_k64(uint64_t x, int k) {
    if (k <= 0) return 0;
    int pos = 0;
    uint64_t y = x;
#pragma unroll
    for (int w = 32; w >= 1; w >>= 1) {
        const int c = __popcll(y & ((1ull << w) - 1ull));
        if (k > c) { k -= c; y >>= w; pos += w; }
    }
    return pos >= 63 ? x : (x & ((2ull << pos) - 1ull));
}

enum { B_NONE = 0, B_ROW = 1, B_COL = 2 };

// centred residue of an integer-valued double |x| < 2^53
__device__ __forceinline__ double cen(double x, double p, double pinv, double hd) {
    const double c = mod_canon(x, p, pinv);
    return c > hd ? c - p : c;
}

// gen_done non-null: the generic leaf ran on the block just before, with
// *gen_done as its zero-pivot flag; when it stayed clear the block holds its
// LU already (identity permutations, full rank) and only P, Q and the rank
// are written here, otherwise the block is untouched and factored below.
template <bool RED, bool SMALLP>
__global__ __launch_bounds__(64) void k_leaf64(int mb, int nb, int32_t *__restrict__ A, int64_t lda,
                                              int32_t *__restrict__ P, int32_t *__restrict__ Q,
                                              int64_t *__restrict__ rank_out, double p, double pinv, int32_t half,
                                              int64_t kexact, const int *__restrict__ gen_done) {
    __shared__ double W[64][65];
    __shared__ double Lc[64];
    __shared__ int rord[64], cord[64];
    const int lane = threadIdx.x;
    if (gen_done && __builtin_amdgcn_readfirstlane(*(volatile const int *)gen_done) == 0) {
        if (lane < mb) P[lane] = lane;
        if (lane < nb) Q[lane] = lane;
        // rank, with both permutations flagged as the identity (bits 40, 41)
        if (lane == 0) *(volatile int64_t *)rank_out = (int64_t)(mb < nb ? mb : nb) | (3ll << 40);
        return;
    }
    const uint64_t allr = mb >= 64 ? ~0ull : ((1ull << mb) - 1ull);
    const uint64_t allc = nb >= 64 ? ~0ull : ((1ull << nb) - 1ull);
    {
        // all 64 loads in flight before the first LDS store
        int32_t av[64];
        const int cl = lane < nb ? lane : 0;
#pragma unroll
        for (int i = 0; i < 64; ++i) av[i] = A[(int64_t)(i < mb ? i : 0) * lda + cl];
#pragma unroll
        for (int i = 0; i < 64; ++i) W[i][lane] = (i < mb && lane < nb) ? centre(av[i], p, half) : 0.0;
    }

    uint64_t rowdone = 0, coldone = 0;
    int r = 0;
    int64_t cnt = 0;
    __syncthreads();

    // ---- generic rank profile: if every diagonal pivot of the unpivoted
    // elimination is nonzero, the leading minors are all nonzero, the pivots
    // are (k, k) and the quadrant order is the identity, so no walk and no
    // search are needed.  A zero pivot sends the block to the general walk.
    // (skipped when the generic leaf already found a zero pivot in this block)
    const int kd = mb < nb ? mb : nb;
    const bool try_generic_pass = gen_done == nullptr;
    bool generic = try_generic_pass;
    for (int k = 0; k < (try_generic_pass ? kd : 0); ++k) {
        double u = 0.0;
        if (lane < nb && lane >= k) {
            const double c = mod_canon(W[k][lane], p, pinv);
            u = c > (double)half ? c - p : c;
            W[k][lane] = u;
        }
        double pv = rld(u, k);
        if (pv < 0.0) pv += p;
        if (pv == 0.0) { generic = false; break; }
        const double inv = SMALLP ? (double)inv_mod_uniform((int32_t)pv, (int32_t)p)
                                  : (double)inv_mod((int32_t)pv, (int32_t)p);
        double l = 0.0;
        if (lane > k && lane < mb) {
            const double c = mod_canon(W[lane][k], p, pinv);
            const double t = mod_canon(c * inv, p, pinv);
            l = t > (double)half ? t - p : t;
            W[lane][k] = l;
        }
        Lc[lane] = l;
        if (lane == 0) { rord[k] = k; cord[k] = k; }
        __syncthreads();
        const double uu = (lane > k && lane < nb) ? u : 0.0;
        const uint64_t act = allr & ~((2ull << k) - 1ull);
#pragma unroll
        for (int g = 0; g < 64; g += 32) {
            if (!((act >> g) & 0xffffffffull)) continue;
            double wv[32], lv[32];
#pragma unroll
            for (int q = 0; q < 32; ++q) {
                wv[q] = W[g + q][lane];
                lv[q] = Lc[g + q];
            }
#pragma unroll
            for (int q = 0; q < 32; ++q) wv[q] = fma(-lv[q], uu, wv[q]);
#pragma unroll
            for (int q = 0; q < 32; ++q) W[g + q][lane] = wv[q];
        }
        if (RED) {
            if (++cnt >= kexact) {
                cnt = 0;
                if (lane > k && lane < nb) {
                    for (int i = k + 1; i < mb; ++i) W[i][lane] = mod_near(W[i][lane], p, pinv);
                }
            }
        }
        __syncthreads();
    }
    if (generic) {
        r = kd;
        rowdone = kd >= 64 ? ~0ull : ((1ull << kd) - 1ull);
        coldone = rowdone;
    } else if (try_generic_pass) {
        // restart from the untouched input with the general walk
        cnt = 0;
        int32_t av[64];
        const int cl = lane < nb ? lane : 0;
#pragma unroll
        for (int i = 0; i < 64; ++i) av[i] = A[(int64_t)(i < mb ? i : 0) * lda + cl];
#pragma unroll
        for (int i = 0; i < 64; ++i) W[i][lane] = (i < mb && lane < nb) ? centre(av[i], p, half) : 0.0;
        __syncthreads();
    }
    uint64_t f_rows = lane == 0 ? allr : 0, f_cols = lane == 0 ? allc : 0, f_top = 0, f_left = 0;
    int f_stage = 0;
    int sp = generic ? 0 : 1;
    // nonzero entries of the active block, one row mask per column (lane);
    // the block changes only at a pivot, so the masks are rebuilt at most
    // once per pivot, when the walk next asks.  A region of the walk holds a
    // pivot exactly when it holds a nonzero entry: zero regions (the whole
    // rest of a rank-deficient block, typically) are skipped with one ballot
    // instead of being walked down to their one-row / one-column pieces.
    uint64_t nzm = 0;
    bool nz_valid = false;
    auto region_nz = [&](uint64_t rows, uint64_t cols) {
        if (!nz_valid) {
            uint64_t mk = 0;
            if (lane < nb && !((coldone >> lane) & 1ull)) {
#pragma unroll
                for (int g = 0; g < 64; g += 32) {
                    double wv[32];
#pragma unroll
                    for (int q = 0; q < 32; ++q) wv[q] = W[g + q][lane];
#pragma unroll
                    for (int q = 0; q < 32; ++q)
                        if (mod_canon(wv[q], p, pinv) != 0.0) mk |= 1ull << (g + q);
                }
            }
            nzm = mk & allr & ~rowdone;
            nz_valid = true;
        }
        return __ballot(((cols >> lane) & 1ull) && (nzm & rows) != 0) != 0;
    };

    while (true) {
        // ---- walk the quadrant recursion to the next one-row / one-column region
        int type = B_NONE, bx = 0;
        uint64_t bmask = 0;
        while (sp > 0) {
            const int t = sp - 1;
            const uint64_t rows = rl64(f_rows, t), cols = rl64(f_cols, t);
            const int stage = __builtin_amdgcn_readlane(f_stage, t);
            if (stage == 0) {
                if (!region_nz(rows, cols)) { --sp; continue; }
                const int nr = __popcll(rows), nc = __popcll(cols);
                if (nr == 1) { type = B_ROW; bx = __ffsll((long long)rows) - 1; bmask = cols; --sp; break; }
                if (nc == 1) { type = B_COL; bx = __ffsll((long long)cols) - 1; bmask = rows; --sp; break; }
                const uint64_t top = first_k64(rows, nr >> 1), left = first_k64(cols, nc >> 1);
                if (lane == t) { f_top = top; f_left = left; f_stage = 1; }
                if (lane == t + 1) { f_rows = top; f_cols = left; f_stage = 0; }
                ++sp;
                continue;
            }
            // stages 1..3: push the next non-empty child, or pop when none is left
            const uint64_t top = rl64(f_top, t), left = rl64(f_left, t);
            bool pushed = false;
            for (int st = stage; st <= 3 && !pushed; ++st) {
                uint64_t cr, cc;
                if (st == 1) { cr = top & ~rowdone; cc = cols & ~left; }
                else if (st == 2) { cr = rows & ~top; cc = left & ~coldone; }
                else { cr = rows & ~top & ~rowdone; cc = cols & ~left & ~coldone; }
                if (cr && cc && region_nz(cr, cc)) {
                    if (lane == t) f_stage = st + 1;
                    if (lane == t + 1) { f_rows = cr; f_cols = cc; f_stage = 0; }
                    ++sp;
                    pushed = true;
                }
            }
            if (!pushed) --sp;
        }
        if (type == B_NONE) break;

        // ---- search: first nonzero of the region
        int x, y;
        if (type == B_ROW) {
            const double v = lane < nb ? W[bx][lane] : 0.0;
            const bool nz = ((bmask >> lane) & 1ull) && mod_canon(v, p, pinv) != 0.0;
            const uint64_t b = __ballot(nz);
            if (!b) continue;
            x = bx;
            y = __ffsll((long long)b) - 1;
        } else {
            const double v = lane < mb ? W[lane][bx] : 0.0;
            const bool nz = ((bmask >> lane) & 1ull) && mod_canon(v, p, pinv) != 0.0;
            const uint64_t b = __ballot(nz);
            if (!b) continue;
            x = __ffsll((long long)b) - 1;
            y = bx;
        }

        // ---- pivot row (final U entries, reduced and centred)
        const bool cact = lane < nb && !((coldone >> lane) & 1ull);
        double u = 0.0;
        if (cact) {
            const double c = mod_canon(W[x][lane], p, pinv);
            u = c > (double)half ? c - p : c;
            W[x][lane] = u;
        }
        double pv = rld(u, y);
        if (pv < 0.0) pv += p;
        const double inv = SMALLP ? (double)inv_mod_uniform((int32_t)pv, (int32_t)p)
                                  : (double)inv_mod((int32_t)pv, (int32_t)p);
        // ---- multipliers (final L entries)
        const bool ract = lane < mb && lane != x && !((rowdone >> lane) & 1ull);
        double l = 0.0;
        if (ract) {
            const double c = mod_canon(W[lane][y], p, pinv);
            const double t = mod_canon(c * inv, p, pinv);
            l = t > (double)half ? t - p : t;
            W[lane][y] = l;
        }
        Lc[lane] = l;
        if (lane == 0) { rord[x] = r; cord[y] = r; }
        __syncthreads();
        // ---- rank-one update of the active block, 32 rows at a time: all
        // loads of a half are issued before any of its stores
        // every updated entry is reduced to (-p, p) on the spot, so that the
        // nonzero-row masks of the walk come out of the update itself (the
        // masks of rows outside the update are zero: they are done)
        const double uu = (cact && lane != y) ? u : 0.0;
        const uint64_t act = allr & ~rowdone & ~(1ull << x);
        uint64_t mk = 0;
#pragma unroll
        for (int g = 0; g < 64; g += 32) {
            if (!((act >> g) & 0xffffffffull)) continue;
            double wv[32], lv[32];
#pragma unroll
            for (int q = 0; q < 32; ++q) {
                wv[q] = W[g + q][lane];
                lv[q] = Lc[g + q];
            }
#pragma unroll
            for (int q = 0; q < 32; ++q) {
                wv[q] = mod_near(fma(-lv[q], uu, wv[q]), p, pinv);
                mk |= (uint64_t)(wv[q] != 0.0) << (g + q);
            }
#pragma unroll
            for (int q = 0; q < 32; ++q) W[g + q][lane] = wv[q];
        }
        if (RED) {
            if (++cnt >= kexact) {
                cnt = 0;
                if (cact && lane != y) {
                    uint64_t a2 = act;
                    while (a2) {
                        const int i = __ffsll((long long)a2) - 1;
                        a2 &= a2 - 1;
                        W[i][lane] = mod_near(W[i][lane], p, pinv);
                    }
                }
            }
        }
        rowdone |= 1ull << x;
        coldone |= 1ull << y;
        ++r;
        nzm = cact && lane != y ? (mk & act) : 0ull;
        nz_valid = true;
        __syncthreads();
    }

    // ---- outputs: pivots in order, then the other rows / columns ascending
    if (lane < mb && !((rowdone >> lane) & 1ull))
        rord[lane] = r + __popcll(~rowdone & allr & ((1ull << lane) - 1ull));
    if (lane < nb && !((coldone >> lane) & 1ull))
        cord[lane] = r + __popcll(~coldone & allc & ((1ull << lane) - 1ull));
    __syncthreads();
    if (lane < nb) {
        const int cp = cord[lane];
        for (int i = 0; i < mb; ++i) A[(int64_t)rord[i] * lda + cp] = (int32_t)mod_canon(W[i][lane], p, pinv);
        Q[cp] = lane;
    }
    if (lane < mb) P[rord[lane]] = lane;
    // the rank, with bit 40 / 41 set when P / Q is the identity
    const bool pid = __ballot(lane < mb && rord[lane] != lane) == 0ull;
    const bool qid = __ballot(lane < nb && cord[lane] != lane) == 0ull;
    if (lane == 0) *rank_out = (int64_t)r | ((int64_t)pid << 40) | ((int64_t)qid << 41);
}

// Leaf of the generic-rank-profile factorisation (plain LU: pivots (k, k)),
// fraction free: step k multiplies each remaining row by the pivot instead of
// dividing the pivot row by it,
//   W[i][c] <- q_k W[i][c] - W[i][k] W[k][c]   (i, c > k),   q_k = W[k][k],
// so the steps need no inverse.  Row i then holds s_i times the row of the
// ordinary elimination, s_k = q_0 ... q_{k-1}, hence (all exact mod p)
//   L[i][k] = W[i][k] / q_k   and   U[k][c] = W[k][c] / s_k,
// and all 64 inverses (one per lane) and the prefix products s_k^-1 are
// formed once at the end.  A pivot is zero exactly when the ordinary one is.
//
// NW waves; lane c owns column c and wave w owns rows w, w + NW, ..., held in
// registers, so the updates stay balanced as the active block shrinks.  Per
// step the owner of row k publishes it through LDS (double buffered, one
// barrier); each wave first reads all its multipliers W[i][k] from lane k,
// then runs the row updates side by side.
// Entries are brought back to |W| <= (p-1)/2 + 3 every step (rounded
// quotient), so q W - a u stays below 2^53 for every p the FP64 embedding
// takes, and a pivot is zero mod p exactly when it is 0.0.  SMALLP selects
// the inverse routine.  LAZY (4 (half + 3)^3 < 2^53): the rows below a block
// of pivots are reduced every second step only; one unreduced step leaves
// |x| <= 2 B^2 (B = half + 3 bounds every reduced entry), the next one
// <= 4 B^3, and every product in both steps is an exact integer below 2^53.  A zero pivot sets *gflag to 1 + its index on the
// whole diagonal (diag0 = the block's offset there) and leaves A untouched
// (A is written only at the end); nothing runs once *gflag is set.
// With Linv / Uinv non-null the leaf also stores L^-1 and U^-1 of its k x k
// diagonal block (k = min(mb, nb); 64 x 64 centred doubles, zero outside),
// the base-case inverses of later triangular solves with these blocks.
// Fused neighbours (generic node of at most 128 x 128 whose two halves are
// leaves; host ensures 64 x (p/2)^2 sums are exact, i.e. no reduction):
//  - He / Hd non-null: the block is first updated, A <- A - He Hd, with He
//    the mb x 64 and Hd the 64 x nb operand (leading dimension lda);
//  - Pd / Pe non-null (needs Linv): after the factorisation the 64 x pdn
//    panel right of the block becomes L^-1 Pd and the pem x 64 panel below
//    it Pe U^-1 (the two solves of the node).
template <bool SMALLP, int NW, bool LAZY>
__global__ __launch_bounds__(64 * NW) void k_leaf_gen(int mb, int nb, int32_t *__restrict__ A, int64_t lda,
                                                      double p, double pinv, int32_t half, int *__restrict__ gflag,
                                                      double *__restrict__ Linv, double *__restrict__ Uinv,
                                                      int inv_red, int kchunk, const int32_t *__restrict__ He,
                                                      const int32_t *__restrict__ Hd, int32_t *__restrict__ Pd,
                                                      int pdn, int32_t *__restrict__ Pe, int pem, int diag0) {
    static_assert(NW == 8, "four pivot rows per block share one row slot; two 256-thread inversion groups");
    constexpr int RPW = 64 / NW;  // rows per wave
    constexpr int KB = 4;         // elimination steps per barrier
    if (__builtin_amdgcn_readfirstlane(*(volatile int *)gflag) != 0) return;
    // the pivot-row buffer is dead once the elimination is over and shares
    // its space with the buffers of the inverse stage
    struct InvBufs {
        int32_t Ms[2][kTri][kTri + 1];  // [0] L (unit lower), [1] U^T (lower)
        double Ws[2][kTri][kTri + 1];
        double Ts[2][kTri * kTri / 4];
    };
    __shared__ union {
        double rowbuf[2][KB][64];
        InvBufs v;
    } sh;
    __shared__ double qv[64], QI[64], SI[64];
    const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const double hd = (double)half;
    double R[RPW];
    {
        int32_t av[RPW];
        const int cl = lane < nb ? lane : 0;
#pragma unroll
        for (int e = 0; e < RPW; ++e) {
            const int i = wave + NW * e;
            av[e] = A[(int64_t)(i < mb ? i : 0) * lda + cl];
        }
#pragma unroll
        for (int e = 0; e < RPW; ++e) {
            const int i = wave + NW * e;
            R[e] = (i < mb && lane < nb) ? centre(av[e], p, half) : 0.0;
        }
    }
    const int kd = mb < nb ? mb : nb;
    if (He) {
        // H = He Hd on the matrix cores, wave w: output tiles (w % 4, 2 (w / 4) + t);
        // reduction index 16 (lane / 16) + s at k-step s, as for every operand here
        const int tr = wave & 3, tcb = 2 * (wave >> 2), r16 = lane & 15, kq = lane >> 4;
        int32_t ev[16], dv[2][16];
#pragma unroll
        for (int sidx = 0; sidx < 16; ++sidx) {
            const int k = 16 * kq + sidx, i = 16 * tr + r16;
            ev[sidx] = He[(int64_t)(i < mb ? i : 0) * lda + k];
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                const int c = 16 * (tcb + t) + r16;
                dv[t][sidx] = Hd[(int64_t)k * lda + (c < nb ? c : 0)];
            }
        }
        v4d_t acc[2] = {v4d_t{0.0, 0.0, 0.0, 0.0}, v4d_t{0.0, 0.0, 0.0, 0.0}};
#pragma unroll
        for (int sidx = 0; sidx < 16; ++sidx) {
            const double a = centre(ev[sidx], p, half);
#pragma unroll
            for (int t = 0; t < 2; ++t)
                acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, centre(dv[t][sidx], p, half), acc[t], 0, 0, 0);
        }
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
            for (int v = 0; v < 4; ++v) sh.v.Ws[0][16 * tr + kq + 4 * v][16 * (tcb + t) + r16] = acc[t][v];
        __syncthreads();
#pragma unroll
        for (int e = 0; e < RPW; ++e) {
            const int i = wave + NW * e;
            if (i < mb && lane < nb) R[e] = mod_near(R[e] - sh.v.Ws[0][i][lane], p, pinv);
        }
        __syncthreads();  // the staging area is the pivot-row buffer below
    }
    // one fraction-free step on a row x held lane-wise: pivot row um (zero in
    // columns <= k), pivot q, step k.  Columns <= k are multiplied by q
    // instead of being left alone (no select); the final scaling divides the
    // extra factors out again (see below).
    auto step = [&](double x, double um, double q, int k) {
        const double a = rld(x, k);
        return mod_near(fma(-a, um, q * x), p, pinv);
    };
    auto step_raw = [&](double x, double um, double q, int k) { return fma(-rld(x, k), um, q * x); };
    // blocks of KB steps: rows kb .. kb + KB - 1 are rows e = kb / NW of waves
    // kb % NW .. kb % NW + KB - 1 (KB divides NW)
#pragma unroll
    for (int kb = 0; kb < 64; kb += KB) {
        if (kb < kd) {  // a guard, not a break: the loop must unroll (R[kb / NW])
        const int nbk = kd - kb < KB ? kd - kb : KB;
        const int eb = kb / NW, w0 = kb % NW;
        const int buf = (kb / KB) & 1;
        if (wave >= w0 && wave < w0 + nbk) sh.rowbuf[buf][wave - w0][lane] = R[eb];
        __syncthreads();
        // every wave eliminates the block's KB x 64 pivot rows among themselves
        double u[KB], um[KB], q[KB];
#pragma unroll
        for (int j = 0; j < KB; ++j) u[j] = j < nbk ? sh.rowbuf[buf][j][lane] : 0.0;
        int zj = -1;  // first zero pivot of the block
#pragma unroll
        for (int j = 0; j < KB; ++j) {
#pragma unroll
            for (int jj = 0; jj < j; ++jj) u[j] = step(u[j], um[jj], q[jj], kb + jj);
            q[j] = rld(u[j], kb + j);
            um[j] = lane > kb + j ? u[j] : 0.0;
            if (j < nbk && q[j] == 0.0 && zj < 0) zj = j;
        }
        if (zj >= 0) {
            // every wave sees the same pivots and leaves here; the flag
            // records 1 + the pivot's index on the diagonal of the whole
            // factorisation (every leading minor below that order is nonzero)
            if (tid == 0) *gflag = 1 + diag0 + kb + zj;
            return;
        }
        if (tid < nbk) {
            double qt = q[0];
#pragma unroll
            for (int j = 1; j < KB; ++j) qt = tid == j ? q[j] : qt;
            qv[kb + tid] = qt;
        }
        // own rows: below the block, KB steps; in the block, the final pivot row
        // (copies of the row loop for full blocks and the last partial one: a
        // uniform branch per block, none per row)
        auto own_rows = [&](auto lazy_c, auto full_c) {
            constexpr bool LZ = decltype(lazy_c)::value, FULL = decltype(full_c)::value;
            const int nbr = FULL ? KB : nbk;
#pragma unroll
            for (int e = eb; e < RPW; ++e) {
                const bool inblk = e == eb && wave >= w0 && wave < w0 + nbr;
                const bool below = e > eb || wave >= w0 + nbr;  // rows after the block's pivots
                if (inblk) {
                    const int j = wave - w0;
                    double ut = u[0];
#pragma unroll
                    for (int jj = 1; jj < KB; ++jj) ut = j == jj ? u[jj] : ut;
                    R[e] = ut;
                } else if (below) {
                    double x = R[e];
#pragma unroll
                    for (int j = 0; j < KB; ++j) {
                        if (LZ) x = (j & 1) == 0 ? step_raw(x, um[j], q[j], kb + j) : step(x, um[j], q[j], kb + j);
                        else if (FULL || j < nbk) x = step(x, um[j], q[j], kb + j);
                    }
                    R[e] = x;
                }
            }
        };
        // a full block (KB even) ends on a reducing step
        if (nbk == KB) own_rows(std::integral_constant<bool, LAZY>{}, std::true_type{});
        else own_rows(std::false_type{}, std::false_type{});
        }
    }
    __syncthreads();
    const bool want_inv = Linv != nullptr;
    if (wave == 0) {
        // q_t^-1, s_t = q_0 .. q_{t-1} and s_t^-1 from one inverse (Montgomery):
        // P_t = q_0 .. q_t, 1 / P_t = (1 / P_{k-1}) q_{t+1} .. q_{k-1}
        double qc = 1.0;
        if (lane < kd) {
            qc = qv[lane];  // |qc| < p
            qc = cen(qc, p, pinv, hd);
        }
        double pre = qc, suf = qc;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const double o = __shfl_up(pre, off), o2 = __shfl_down(suf, off);
            if (lane >= off) pre = cen(pre * o, p, pinv, hd);
            if (lane + off < 64) suf = cen(suf * o2, p, pinv, hd);
        }
        // pre = P_t (inclusive), suf = q_t .. q_63 (inclusive; q = 1 past k)
        double total = rld(pre, 63);
        if (total < 0.0) total += p;
        double itot = SMALLP ? (double)inv_mod_uniform((int32_t)total, (int32_t)p)
                             : (double)inv_mod((int32_t)total, (int32_t)p);
        double sx = __shfl_down(suf, 1);   // q_{t+1} .. q_63
        if (lane == 63) sx = 1.0;
        const double invP = cen(itot * sx, p, pinv, hd);  // 1 / P_t
        double pprev = __shfl_up(pre, 1), iprev = __shfl_up(invP, 1);
        if (lane == 0) {
            pprev = 1.0;
            iprev = 1.0;
        }
        const double qi = cen(pprev * invP, p, pinv, hd);  // q_t^-1 = P_{t-1} / P_t
        QI[lane] = cen(qi * pprev, p, pinv, hd);           // q_t^-1 s_t = U[t][t]^-1
        SI[lane] = iprev;                                  // s_t^-1 = 1 / P_{t-1}
    }
    __syncthreads();
    // Row i ends as s_i times its ordinary row in the columns c >= i (U part);
    // its column c < min(i, k) holds the multiplier of step c times q_c ...
    // q_{min(i,k)-1} (it was multiplied by every later pivot while i was below
    // the pivot row), so L[i][c] = W[i][c] (q_c^-1 s_c) s_i^-1, with
    // s_i = q_0 .. q_{min(i,k)-1}.
#pragma unroll
    for (int e = 0; e < RPW; ++e) {
        const int i = wave + NW * e;
        const int lim = i < kd ? i : kd;
        const double f = lane < lim ? cen(QI[lane] * SI[i], p, pinv, hd) : SI[i];
        const double v = mod_canon(R[e] * f, p, pinv);
        if (i < mb && lane < nb) A[(int64_t)i * lda + lane] = (int32_t)v;
        if (want_inv) {
            // the k x k blocks, written whole (no separate clearing): L strictly
            // below the diagonal, U^T likewise; W holds the diagonal inverses
            const double cv = v > hd ? v - p : v;
            const bool ink = i < kd && lane < kd;
            sh.v.Ms[0][i][lane] = (ink && lane < i) ? (int32_t)cv : 0;
            sh.v.Ms[1][lane][i] = (ink && lane > i) ? (int32_t)cv : 0;
            const double ud = i < kd ? QI[i] : 1.0;  // U[i][i]^-1 = q_i^-1 s_i
            sh.v.Ws[0][i][lane] = lane == i ? 1.0 : 0.0;
            sh.v.Ws[1][i][lane] = lane == i ? ud : 0.0;
        }
    }
    if (!want_inv) return;
    __syncthreads();
    {
        const int g = __builtin_amdgcn_readfirstlane(tid >> 8), t = tid & 255;
        if (inv_red) tri_inverse_levels<true>(t, sh.v.Ms[g], sh.v.Ws[g], sh.v.Ts[g], p, pinv, hd, kchunk);
        else tri_inverse_levels<false>(t, sh.v.Ms[g], sh.v.Ws[g], sh.v.Ts[g], p, pinv, hd, kchunk);
    }
    // L^-1 and U^-1 = ((U^T)^-1)^T, zero outside the k x k block
    for (int idx = tid; idx < kTri * kTri; idx += 64 * NW) {
        const int i = idx / kTri, j = idx % kTri;
        const bool in = i < kd && j < kd;
        Linv[idx] = in ? sh.v.Ws[0][i][j] : 0.0;
        Uinv[idx] = in ? sh.v.Ws[1][j][i] : 0.0;
    }
    if (Pd) {
        // D = L^-1 Pd (64 x pdn) and E = Pe U^-1 (pem x 64), in place: every
        // wave reads its operands, then all write (tiles share source rows
        // and columns)
        __syncthreads();
        const int tr = wave & 3, tcb = 2 * (wave >> 2), r16 = lane & 15, kq = lane >> 4;
        v4d_t accd[2] = {v4d_t{0.0, 0.0, 0.0, 0.0}, v4d_t{0.0, 0.0, 0.0, 0.0}};
        v4d_t acce[2] = {v4d_t{0.0, 0.0, 0.0, 0.0}, v4d_t{0.0, 0.0, 0.0, 0.0}};
        {
            int32_t bv[2][16], cv[16];
#pragma unroll
            for (int sidx = 0; sidx < 16; ++sidx) {
                const int k = 16 * kq + sidx, i = 16 * tr + r16;
                cv[sidx] = Pe[(int64_t)(i < pem ? i : 0) * lda + k];
#pragma unroll
                for (int t = 0; t < 2; ++t) {
                    const int c = 16 * (tcb + t) + r16;
                    bv[t][sidx] = Pd[(int64_t)k * lda + (c < pdn ? c : 0)];
                }
            }
#pragma unroll
            for (int sidx = 0; sidx < 16; ++sidx) {
                const int k = 16 * kq + sidx;
                const double li = sh.v.Ws[0][16 * tr + r16][k];
                const double ce = centre(cv[sidx], p, half);
#pragma unroll
                for (int t = 0; t < 2; ++t) {
                    // U^-1[k][c] = (U^T)^-1[c][k]
                    const double ui = sh.v.Ws[1][16 * (tcb + t) + r16][k];
                    accd[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(li, centre(bv[t][sidx], p, half), accd[t], 0, 0, 0);
                    acce[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(ce, ui, acce[t], 0, 0, 0);
                }
            }
        }
        __syncthreads();
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int i = 16 * tr + kq + 4 * v, c = 16 * (tcb + t) + r16;
                if (c < pdn) Pd[(int64_t)i * lda + c] = (int32_t)mod_canon(accd[t][v], p, pinv);
                if (i < pem) Pe[(int64_t)i * lda + c] = (int32_t)mod_canon(acce[t][v], p, pinv);
            }
    }
}

constexpr int kGenWaves = 8;

int leaf64_launch(const Field &F, int64_t m, int64_t n, int32_t *A, int64_t lda, int32_t *P, int32_t *Q,
                  int64_t *rank_dev, int *gflag, double *Linv, double *Uinv, hipStream_t s, const int32_t *He,
                  const int32_t *Hd, int32_t *Pd, int64_t pdn, int32_t *Pe, int64_t pem, int64_t diag0,
                  const int *gen_done) {
    const bool red = F.kexact < 64;
    const bool small = F.p < (1u << 24);
#define FFP_L64(R_, S_)                                                                                    \
    hipLaunchKernelGGL((k_leaf64<R_, S_>), dim3(1), dim3(64), 0, s, (int)m, (int)n, A, lda, P, Q, rank_dev, \
                       F.pd, F.pinv, (int32_t)F.half, F.kexact, gen_done)
#define FFP_SEL(X_)                                     \
    if (red) {                                          \
        if (small) X_(true, true); else X_(true, false); \
    } else {                                            \
        if (small) X_(false, true); else X_(false, false); \
    }
    if (gflag) {
        // dot products of the block inversion take at most 32 terms
        const int inv_red = F.kexact < 32;
        const int kchunk = (int)(F.kexact < 1 ? 1 : (F.kexact > 32 ? 32 : F.kexact));
        // the fused products sum 64 terms unreduced
        if ((He || Pd) && (F.kexact < 64 || (Pd && (!Linv || m != 64 || n != 64 || pdn > 64 || pem > 64)) ||
                           (He && (!Hd || m > 64 || n > 64))))
            return FFP_E_INTERNAL;
        // two unreduced steps stay exact: 4 B^3 < 2^53 with B = half + 3
        const double B = (double)F.half + 3.0;
        const bool lazy = 4.0 * B * B * B < 9007199254740992.0;
#define FFP_LG(S_, L_)                                                                                              \
    hipLaunchKernelGGL((k_leaf_gen<S_, kGenWaves, L_>), dim3(1), dim3(64 * kGenWaves), 0, s, (int)m, (int)n, A, lda, \
                       F.pd, F.pinv, (int32_t)F.half, gflag, Linv, Uinv, inv_red, kchunk, He, Hd, Pd, (int)pdn, Pe,   \
                       (int)pem, (int)diag0)
        const double kk = (double)(m < n ? m : n);
        ProfScope prof(PK_LEAF_GEN,
                       2.0 * (double)m * (double)n * kk - (double)(m + n) * kk * kk + 2.0 * kk * kk * kk / 3.0 +
                           (He ? 2.0 * (double)m * (double)n * 64.0 : 0.0) +
                           (Pd ? 64.0 * 64.0 * (double)(pdn + pem) : 0.0),
                       s, 8.0 * (double)m * (double)n);
        if (lazy) FFP_LG(true, true);
        else if (small) FFP_LG(true, false);
        else FFP_LG(false, false);
#undef FFP_LG
    } else {
        ProfScope prof(PK_LEAF, 0.0, s, 8.0 * (double)m * (double)n);
        FFP_SEL(FFP_L64)
    }
#undef FFP_SEL
#undef FFP_L64
    FFP_HIP_CHECK(hipGetLastError());
    return FFP_OK;
}

}  // namespace ffp
