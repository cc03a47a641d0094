// Batched PLUQ: many independent matrices of uneven shapes and ranks in one
// persistent launch (the heterogeneous, rank-dependent pivot blocks of
// Section 4.1 are exactly why the work per matrix cannot be known ahead).
//
// Each workgroup repeatedly takes the next matrix from an atomic counter (no
// host synchronisation; graph-capturable), copies it into its workspace
// slot, and factors it with the same pivot order as the tile recursion of
// Section 4.1: the quadrant recursion is walked with an explicit stack to
// find each pivot (first nonzero of a one-row or one-column region) and the
// pivot is applied at once as a rank-one update.  Eager and deferred updates
// give the same Schur complements, so the result equals what ffp_pluq
// returns for the matrix alone.  The factors are then written back with the
// final row and column order, together with P, Q, the rank and the sorted
// rank profiles.
#include <algorithm>
#include <climits>
#include <map>
#include <mutex>
#include <tuple>
#include <type_traits>

#include "ffp_internal.hpp"
#include "ffp_device.hpp"

namespace ffp {

constexpr int kBMax = FFP_BATCH_MAX_DIM;      // max rows / columns
constexpr int kBW = kBMax / 32;               // mask words
constexpr int kBStack = 24;

struct BFrame {
    uint32_t rows[kBW], cols[kBW], top[kBW], left[kBW];
    int stage;
};

struct BShared {
    uint32_t rowdone[kBW], coldone[kBW], mask[kBW];
    uint32_t nz[kBW];  // row i has a nonzero in the active columns
    BFrame st[kBStack];
    int sp, type, bx, piv, r, job;
    int rord[kBMax], cord[kBMax];
    int upiv;  // the pivot's value
    int wcnt[kBW + 1];
    // rows (nonzero multiplier) and columns (active, not the pivot's) of the
    // next rank-one update, the columns in increasing order
    short rl[kBMax], cl[kBMax];
    int nrl, ncl, wtot[16];
    int np;  // pending pivots not yet applied to the active block
};

enum { BT_FIN = 0, BT_ROW = 1, BT_COL = 2 };

__device__ __forceinline__ bool bbit(const uint32_t *m, int i) { return (m[i >> 5] >> (i & 31)) & 1u; }

// Walk to the next one-row / one-column region (or finish), by one wave:
// lane w holds word w of every row / column mask, so each mask operation of
// a frame is a handful of wave-wide instructions (popcounts by shuffle
// reduction, "first k set bits" by a prefix scan of the words' popcounts)
// rather than a loop of dependent scalar LDS accesses (one thread doing the
// same walk cost ~50 us per pivot).  Regions none of whose active rows has a
// nonzero in the active columns hold no pivot and are skipped whole (S.nz);
// this only prunes the walk, the regions that are visited and their order
// are those of the recursion.  Called by all 64 lanes of wave 0.
// The masks have at most kBW <= 32 words, held by lanes 0..31 (two DPP rows
// of 16 lanes; the other lanes hold zeros), so sums and scans run within
// the rows on DPP lane moves (a few cycles each) and join the two rows by
// lane reads, rather than through LDS-routed shuffles.
static_assert(kBW <= 32, "mask words fit two DPP rows of 16 lanes");
constexpr int kDppRowShr = 0x110, kDppRowRor = 0x120;  // + shift 1..15
template <int CTRL>
__device__ __forceinline__ int dpp_move(int v) {
    // lanes whose source lies outside the row read 0
    return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xf, 0xf, true);
}
// sum over lanes 0..31, the same value returned to every lane
__device__ __forceinline__ int wsum(int v) {
    v += dpp_move<kDppRowRor + 8>(v);
    v += dpp_move<kDppRowRor + 4>(v);
    v += dpp_move<kDppRowRor + 2>(v);
    v += dpp_move<kDppRowRor + 1>(v);
    return __builtin_amdgcn_readlane(v, 0) + __builtin_amdgcn_readlane(v, 16);
}
// the k lowest set bits of the wave-distributed mask x (k <= popcount)
__device__ __forceinline__ uint32_t wfirst_k(uint32_t x, int k, int lane) {
    const int c = __popc(x);
    int incl = c;  // inclusive prefix sum of the words' popcounts over lanes 0..31
    incl += dpp_move<kDppRowShr + 1>(incl);
    incl += dpp_move<kDppRowShr + 2>(incl);
    incl += dpp_move<kDppRowShr + 4>(incl);
    incl += dpp_move<kDppRowShr + 8>(incl);
    const int row0 = __builtin_amdgcn_readlane(incl, 15);
    if (lane >= 16 && lane < 32) incl += row0;
    const int excl = incl - c;
    if (incl <= k) return x;
    if (excl >= k) return 0u;
    uint32_t o = 0;
    for (int t = k - excl; t > 0; --t) {
        const uint32_t low = x & (~x + 1u);
        o |= low;
        x ^= low;
    }
    return o;
}
// index of the lowest set bit of the wave-distributed mask x (x != 0)
__device__ __forceinline__ int wfirst(uint32_t x) {
    const uint64_t b = __ballot(x != 0u);
    const int w = __ffsll((long long)b) - 1;
    const uint32_t xw = (uint32_t)__builtin_amdgcn_readlane((int)x, w);
    return w * 32 + __ffs(xw) - 1;
}

__device__ __noinline__ static void bwalk_w(BShared &S, int nwr, int nwc, int lane) {
    const bool lr = lane < nwr, lc = lane < nwc;
    const uint32_t rd = lr ? S.rowdone[lane] : 0u, cd = lc ? S.coldone[lane] : 0u, nz = lr ? S.nz[lane] : 0u;
    int sp = S.sp;
    int type = BT_FIN, bx = 0;
    while (sp > 0) {
        BFrame &f = S.st[sp - 1];
        const int stage = f.stage;
        const uint32_t rows = lr ? f.rows[lane] : 0u, cols = lc ? f.cols[lane] : 0u;
        if (stage == 0) {
            const int nr = wsum(__popc(rows)), nc = wsum(__popc(cols));
            if (nr == 0 || nc == 0) { --sp; continue; }
            // no active row of the region has a nonzero left: no pivot in it
            if (__ballot((rows & ~rd & nz) != 0u) == 0ull) { --sp; continue; }
            if (nr == 1) {
                type = BT_ROW;
                bx = wfirst(rows);
                if (lc) S.mask[lane] = cols;
                --sp;
                break;
            }
            if (nc == 1) {
                type = BT_COL;
                bx = wfirst(cols);
                if (lr) S.mask[lane] = rows;
                --sp;
                break;
            }
            const uint32_t top = wfirst_k(rows, nr / 2, lane), left = wfirst_k(cols, nc / 2, lane);
            BFrame &c = S.st[sp];
            if (lr) { f.top[lane] = top; c.rows[lane] = top; }
            if (lc) { f.left[lane] = left; c.cols[lane] = left; }
            if (lane == 0) { f.stage = 1; c.stage = 0; }
            ++sp;
            continue;
        }
        const uint32_t top = lr ? f.top[lane] : 0u, left = lc ? f.left[lane] : 0u;
        const uint32_t bot = rows & ~top, right = cols & ~left;
        bool pushed = false;
        for (int st = stage; st <= 3 && !pushed; ++st) {
            const uint32_t cr = st == 1 ? (top & ~rd) : st == 2 ? bot : (bot & ~rd);
            const uint32_t cc = st == 1 ? right : st == 2 ? (left & ~cd) : (right & ~cd);
            if (__ballot(cr != 0u) != 0ull && __ballot(cc != 0u) != 0ull) {
                BFrame &c = S.st[sp];
                if (lr) c.rows[lane] = cr;
                if (lc) c.cols[lane] = cc;
                if (lane == 0) { f.stage = st + 1; c.stage = 0; }
                ++sp;
                pushed = true;
            }
        }
        if (!pushed) --sp;
    }
    if (lane == 0) {
        S.sp = sp;
        S.type = type;
        S.bx = bx;
    }
}

__global__ void k_batch_reset(int *counter) { *counter = 0; }

// Longest-processing-time order of the queue: jobs sorted by decreasing
// bucket of m n min(m, n) (the elimination's work), one workgroup, counting
// sort over 1024 logarithmic buckets (32 per doubling).  Large matrices are
// taken first so that the last ones to finish are small.
__global__ __launch_bounds__(1024) void k_batch_order(int32_t batch, const int32_t *__restrict__ m_arr,
                                                      const int32_t *__restrict__ n_arr, int32_t *__restrict__ order) {
    __shared__ int hist[1024];
    const int tid = threadIdx.x;
    hist[tid] = 0;
    __syncthreads();
    auto bucket = [&](int j) {
        const double m = m_arr[j], n = n_arr[j];
        const double w = m > 0 && n > 0 ? m * n * (m < n ? m : n) : 0.0;
        const int b = w >= 1.0 ? (int)(log2(w) * 32.0) : 0;
        return 1023 - (b < 0 ? 0 : (b > 1023 ? 1023 : b));  // largest first
    };
    for (int j = tid; j < batch; j += 1024) atomicAdd(&hist[bucket(j)], 1);
    __syncthreads();
    if (tid == 0) {
        int acc = 0;
        for (int b = 0; b < 1024; ++b) {
            const int c = hist[b];
            hist[b] = acc;
            acc += c;
        }
    }
    __syncthreads();
    for (int j = tid; j < batch; j += 1024) order[atomicAdd(&hist[bucket(j)], 1)] = j;
}

// Current Schur-complement value of an entry whose stored value w has not
// yet received the np pending pivots: w - sum_t L[t] U[t] (L: the row's
// pending multipliers, U: the pending pivot rows at the entry's column,
// stride ldu; both centred, held as PT: int16_t when p < 2^16, else int32_t),
// exact in FP64 with a reduction every kred terms; canonical result.
template <typename PT>
__device__ __forceinline__ double schur_val(int32_t w, const PT *L, const PT *U, int ldu, int np, int kred,
                                            double p, double pinv) {
    double acc = (double)w;
    int k = 0;
    for (int t = 0; t < np; ++t) {
        acc = fma(-(double)L[t], (double)U[t * ldu], acc);
        if (++k == kred) {
            acc = mod_near(acc, p, pinv);
            k = 0;
        }
    }
    return mod_canon(acc, p, pinv);
}

// Ordered compaction helper: the number of set flags of lanes below this one
// in the wave, and the wave's total
__device__ __forceinline__ int wprefix(bool f, int lane, int *tot) {
    const uint64_t b = __ballot(f);
    *tot = __popcll(b);
    return __popcll(b & ((lane ? (~0ull >> (64 - lane)) : 0ull)));
}

// NARROW (p < 2^16): the working copy holds canonical residues as uint16_t
// and the pending pivots centred ones as int16_t, halving their bytes;
// otherwise both are int32_t.
template <int kBT, bool NARROW>
__global__ __launch_bounds__(kBT) void k_pluq_batched(int32_t batch, const int32_t *__restrict__ m_arr,
                                                      const int32_t *__restrict__ n_arr, int32_t *__restrict__ A,
                                                      const int64_t *__restrict__ A_off, int32_t *__restrict__ P,
                                                      const int64_t *__restrict__ P_off, int32_t *__restrict__ Q,
                                                      const int64_t *__restrict__ Q_off, int32_t *__restrict__ rank,
                                                      int32_t *__restrict__ rrp, int32_t *__restrict__ crp,
                                                      int *__restrict__ counter, const int32_t *__restrict__ order,
                                                      int32_t *__restrict__ slots, int64_t slot_elems, int32_t max_m,
                                                      int32_t max_n, double p, double pinv, int32_t half, int nb,
                                                      int kred) {
    __shared__ BShared S;
    // pending pivots (delayed rank-one updates): L[i][t] at Lb[i nb + t],
    // U[t][j] at Ub[t ldu + j], centred residues
    using PT = typename std::conditional<NARROW, int16_t, int32_t>::type;
    using WT = typename std::conditional<NARROW, uint16_t, int32_t>::type;
    extern __shared__ __attribute__((aligned(16))) int32_t pend[];
    PT *Lb = (PT *)pend, *Ub = Lb + (size_t)max_m * nb;
    const int ldu = max_n > 0 ? max_n : 1;
    const int tid = threadIdx.x;
    WT *W = (WT *)slots + (int64_t)blockIdx.x * slot_elems;
    while (true) {
        if (tid == 0) {
            const int t = atomicAdd(counter, 1);
            S.job = t < batch ? order[t] : batch;
        }
        __syncthreads();
        const int job = S.job;
        if (job >= batch) break;  // uniform: every wave of the workgroup exits
        const int m = m_arr[job], n = n_arr[job];
        // a shape beyond the bounds the workspace slots and the LDS masks were
        // sized for is not factored: its rank reads -1 (uniform branch)
        if (m < 0 || n < 0 || m > max_m || n > max_n) {
            if (tid == 0) rank[job] = -1;
            __syncthreads();
            continue;
        }
        int32_t *Aj = A + A_off[job];
        const int nwr = (m + 31) >> 5, nwc = (n + 31) >> 5;
        // workspace copy (leading dimension n), and the nonzero-row mask
        if (tid < kBW) S.nz[tid] = 0u;
        __syncthreads();
        {
            const int wv = tid >> 6, ln = tid & 63;
            for (int i = wv; i < m; i += kBT / 64) {
                bool any = false;
                for (int c = ln; c < n; c += 64) {
                    const int32_t v = Aj[(int64_t)i * n + c];
                    W[(int64_t)i * n + c] = (WT)v;
                    any |= v != 0;
                }
                if (__ballot(any) != 0ull && ln == 0) atomicOr(&S.nz[i >> 5], 1u << (i & 31));
            }
        }
        if (tid == 0) {
            for (int w = 0; w < kBW; ++w) { S.rowdone[w] = 0; S.coldone[w] = 0; }
            BFrame &f = S.st[0];
            for (int w = 0; w < nwr; ++w) {
                const int c = m - w * 32;
                f.rows[w] = c >= 32 ? 0xffffffffu : ((1u << c) - 1u);
            }
            for (int w = 0; w < nwc; ++w) {
                const int c = n - w * 32;
                f.cols[w] = c >= 32 ? 0xffffffffu : ((1u << c) - 1u);
            }
            f.stage = 0;
            S.sp = (m > 0 && n > 0) ? 1 : 0;
            S.r = 0;
        }
        __syncthreads();
        // the first region
        if (tid < 64) bwalk_w(S, nwr, nwc, tid);
        if (tid == 0) S.np = 0;
        __syncthreads();
        constexpr int NWV = kBT / 64;
        static_assert(NWV >= 2, "the walk wave and at least one other wave");
        const int wv = tid >> 6, ln = tid & 63;
        while (true) {
            const int type = S.type, bx = S.bx, np = S.np;
            if (type == BT_FIN) break;
            if (tid == 0) S.piv = INT_MAX;
            __syncthreads();
            // search the region for its first nonzero of the current Schur
            // complement (stored value minus the pending pivots' terms)
            if (type == BT_ROW) {
                if (bbit(S.nz, bx))
                    for (int c = tid; c < n; c += kBT)
                        if (bbit(S.mask, c) &&
                            schur_val(W[(int64_t)bx * n + c], Lb + bx * nb, Ub + c, ldu, np, kred, p, pinv) != 0.0) {
                            atomicMin(&S.piv, c);
                            break;
                        }
            } else {
                for (int i = tid; i < m; i += kBT)
                    if (bbit(S.mask, i) && bbit(S.nz, i) &&
                        schur_val(W[(int64_t)i * n + bx], Lb + i * nb, Ub + bx, ldu, np, kred, p, pinv) != 0.0) {
                        atomicMin(&S.piv, i);
                        break;
                    }
            }
            __syncthreads();
            const int pv = S.piv;
            if (pv != INT_MAX) {
            const int x = type == BT_ROW ? bx : pv, y = type == BT_ROW ? pv : bx;
            // the pivot row's final U entries (pending terms applied), kept as
            // pending row np (centred) for the later corrections
            for (int c = tid; c < n; c += kBT)
                if (!bbit(S.coldone, c)) {
                    const double u = schur_val(W[(int64_t)x * n + c], Lb + x * nb, Ub + c, ldu, np, kred, p, pinv);
                    if (c == y) S.upiv = (int32_t)u;
                    W[(int64_t)x * n + c] = (WT)u;
                    Ub[np * ldu + c] = (PT)centre((int32_t)u, p, half);
                }
            __syncthreads();
            if (wv == 0) {
                // wave 0 records the pivot and walks to the next region while
                // the others form the L column (the walk reads the done masks
                // and the nonzero-row bits, which stay a superset of the true ones)
                if (ln == 0) {
                    S.rowdone[x >> 5] |= 1u << (x & 31);
                    S.coldone[y >> 5] |= 1u << (y & 31);
                    S.rord[x] = S.r;
                    S.cord[y] = S.r;
                    S.r += 1;
                    S.np = np + 1;
                }
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                bwalk_w(S, nwr, nwc, ln);
            } else {
                // the pivot column's final L entries, kept as pending column np:
                // each thread's rows are read and corrected first, so that the
                // pivot's inverse is computed while those loads are in flight
                constexpr int LR = (kBMax + kBT - 65) / (kBT - 64);  // rows per thread
                double sv[LR];
#pragma unroll
                for (int e = 0; e < LR; ++e) {
                    const int i = tid - 64 + e * (kBT - 64);
                    sv[e] = (i < m && i != x && !bbit(S.rowdone, i))
                                ? schur_val(W[(int64_t)i * n + y], Lb + i * nb, Ub + y, ldu, np, kred, p, pinv)
                                : 0.0;
                }
                const int32_t piv = S.upiv;
                const double inv =
                    (double)(p < 16777216.0 ? inv_mod_small(piv, (int32_t)p) : inv_mod(piv, (int32_t)p));
#pragma unroll
                for (int e = 0; e < LR; ++e) {
                    const int i = tid - 64 + e * (kBT - 64);
                    if (i < m && i != x && !bbit(S.rowdone, i)) {
                        const double l = mod_canon(sv[e] * inv, p, pinv);
                        W[(int64_t)i * n + y] = (WT)l;
                        Lb[i * nb + np] = (PT)centre((int32_t)l, p, half);
                    }
                }
            }
            __syncthreads();
            }
            // ---- flush: apply the pending pivots to the active block at once
            // when nb are pending, or when a region turned out empty (the
            // nonzero-row bits are refreshed only here, so an empty region
            // means they may be stale: refreshed, they prune the walk again)
            const int npf = S.np;
            if (npf >= nb || (pv == INT_MAX && npf > 0)) {
            // ---- flush: apply the pending pivots to the active block at
            // once (one read and one write per entry for nb pivots); the rows
            // with a nonzero pending multiplier and the active columns compacted
            int wt_r = 0, wt_c = 0;
#pragma unroll
            for (int k = 0; k < (kBMax + kBT - 1) / kBT; ++k) {
                const int i = tid + k * kBT;
                bool f = false;
                if (i < m && !bbit(S.rowdone, i)) {
                    for (int t = 0; t < npf; ++t) f |= Lb[i * nb + t] != 0;
                }
                int t;
                const int pr = wprefix(f, ln, &t);
                wt_r = t;
                const bool fc = i < n && !bbit(S.coldone, i);
                const int pc = wprefix(fc, ln, &t);
                wt_c = t;
                if (ln == 0) S.wtot[wv] = wt_r | (wt_c << 16);
                __syncthreads();
                if (tid == 0) {
                    int ar = k == 0 ? 0 : S.nrl, ac = k == 0 ? 0 : S.ncl;
                    for (int w = 0; w < NWV; ++w) {
                        const int v = S.wtot[w];
                        S.wtot[w] = ar | (ac << 16);
                        ar += v & 0xffff;
                        ac += v >> 16;
                    }
                    S.nrl = ar;
                    S.ncl = ac;
                }
                __syncthreads();
                const int base = S.wtot[wv];
                if (f) S.rl[(base & 0xffff) + pr] = (short)i;
                if (fc) S.cl[(base >> 16) + pc] = (short)i;
                __syncthreads();
            }
            {
                // each wave takes RB listed rows at a time and CH chunks of 64
                // listed columns: RB x CH loads in flight per lane, and every
                // pending entry read from LDS serves RB (U) or CH (L) updates.
                // Per entry the same fma chain as schur_val, so the same bits.
                const int nrl = S.nrl, ncl = S.ncl;
                constexpr int CH = 4, RB = kBT >= 1024 ? 2 : 4;
                const int nch = (ncl + 63) >> 6;
                for (int q0 = wv * RB; q0 < nrl; q0 += NWV * RB) {
                    int ii[RB];
                    bool rok[RB], nzr[RB];
#pragma unroll
                    for (int rb = 0; rb < RB; ++rb) {
                        rok[rb] = q0 + rb < nrl;
                        ii[rb] = S.rl[rok[rb] ? q0 + rb : q0];
                        nzr[rb] = false;
                    }
                    for (int ch0 = 0; ch0 < nch; ch0 += CH) {
                        int col[CH];
                        bool ok[CH];
#pragma unroll
                        for (int cc = 0; cc < CH; ++cc) {
                            const int qq = ln + 64 * (ch0 + cc);
                            ok[cc] = qq < ncl;
                            col[cc] = S.cl[ok[cc] ? qq : ncl - 1];
                        }
                        double a[RB][CH];
#pragma unroll
                        for (int rb = 0; rb < RB; ++rb)
#pragma unroll
                            for (int cc = 0; cc < CH; ++cc) a[rb][cc] = (double)W[(int64_t)ii[rb] * n + col[cc]];
                        int k = 0;
                        for (int t = 0; t < npf; ++t) {
                            double u[CH], l[RB];
#pragma unroll
                            for (int cc = 0; cc < CH; ++cc) u[cc] = (double)Ub[t * ldu + col[cc]];
#pragma unroll
                            for (int rb = 0; rb < RB; ++rb) l[rb] = (double)Lb[ii[rb] * nb + t];
#pragma unroll
                            for (int rb = 0; rb < RB; ++rb)
#pragma unroll
                                for (int cc = 0; cc < CH; ++cc) a[rb][cc] = fma(-l[rb], u[cc], a[rb][cc]);
                            if (++k == kred) {
#pragma unroll
                                for (int rb = 0; rb < RB; ++rb)
#pragma unroll
                                    for (int cc = 0; cc < CH; ++cc) a[rb][cc] = mod_near(a[rb][cc], p, pinv);
                                k = 0;
                            }
                        }
#pragma unroll
                        for (int rb = 0; rb < RB; ++rb)
#pragma unroll
                            for (int cc = 0; cc < CH; ++cc)
                                if (rok[rb] && ok[cc]) {
                                    const int32_t nv = (int32_t)mod_canon(a[rb][cc], p, pinv);
                                    W[(int64_t)ii[rb] * n + col[cc]] = (WT)nv;
                                    nzr[rb] |= nv != 0;
                                }
                    }
                    // a listed row's active entries are the listed columns
#pragma unroll
                    for (int rb = 0; rb < RB; ++rb) {
                        const bool any = __ballot(nzr[rb]) != 0ull;
                        if (ln == 0 && rok[rb]) {
                            const int i = ii[rb];
                            if (any) atomicOr(&S.nz[i >> 5], 1u << (i & 31));
                            else atomicAnd(&S.nz[i >> 5], ~(1u << (i & 31)));
                        }
                    }
                }
            }
            if (tid == 0) S.np = 0;
            __syncthreads();
            }
            if (pv == INT_MAX) {
                // no pivot in the region: walk on to the next one
                if (tid < 64) bwalk_w(S, nwr, nwc, tid);
                __syncthreads();
            }
        }
        // ---- output order: pivots in order, then the rest ascending
        const int r = S.r;
        if (tid == 0) {
            int acc = 0;
            for (int w = 0; w < nwr; ++w) {
                S.wcnt[w] = acc;
                const int c = m - w * 32;
                acc += __popc(~S.rowdone[w] & (c >= 32 ? 0xffffffffu : ((1u << c) - 1u)));
            }
        }
        __syncthreads();
        for (int i = tid; i < m; i += kBT) {
            if (!bbit(S.rowdone, i)) {
                const uint32_t below = (i & 31) ? (~S.rowdone[i >> 5] & ((1u << (i & 31)) - 1u)) : 0u;
                S.rord[i] = r + S.wcnt[i >> 5] + __popc(below);
            }
        }
        __syncthreads();
        if (tid == 0) {
            int acc = 0;
            for (int w = 0; w < nwc; ++w) {
                S.wcnt[w] = acc;
                const int c = n - w * 32;
                acc += __popc(~S.coldone[w] & (c >= 32 ? 0xffffffffu : ((1u << c) - 1u)));
            }
        }
        __syncthreads();
        for (int c = tid; c < n; c += kBT) {
            if (!bbit(S.coldone, c)) {
                const uint32_t below = (c & 31) ? (~S.coldone[c >> 5] & ((1u << (c & 31)) - 1u)) : 0u;
                S.cord[c] = r + S.wcnt[c >> 5] + __popc(below);
            }
        }
        __syncthreads();
        // the block of non-pivot rows and columns is zero in the final
        // factorisation (every pivot has been found); the slot may still hold
        // its entries without the last pending pivots' terms
        for (int64_t e = tid; e < (int64_t)m * n; e += kBT) {
            const int i = (int)(e / n), c = (int)(e % n);
            const bool keep = bbit(S.rowdone, i) || bbit(S.coldone, c);
            Aj[(int64_t)S.rord[i] * n + S.cord[c]] = keep ? (int32_t)W[e] : 0;
        }
        int32_t *Pj = P + P_off[job], *Qj = Q + Q_off[job];
        for (int i = tid; i < m; i += kBT) Pj[S.rord[i]] = i;
        for (int c = tid; c < n; c += kBT) Qj[S.cord[c]] = c;
        if (tid == 0) {
            rank[job] = r;
            if (rrp) {
                int k = 0;
                for (int i = 0; i < m; ++i)
                    if (bbit(S.rowdone, i)) rrp[P_off[job] + k++] = i;
            }
            if (crp) {
                int k = 0;
                for (int c = 0; c < n; ++c)
                    if (bbit(S.coldone, c)) crp[Q_off[job] + k++] = c;
            }
        }
        __syncthreads();
    }
}

// Launch shapes (threads per workgroup, workgroups per compute unit): one
// 1024-thread workgroup per CU (sixteen waves on each matrix, the default),
// or several smaller workgroups per CU (more matrices in flight, whose
// latency-bound pivot chains then overlap, fewer waves on each).  ffp_pluq_batched_tune times them on the
// caller's batch and keeps the faster one for batches of that description.
struct BShape {
    int threads, per_cu;
};
constexpr BShape kShapes[] = {{1024, 1}, {512, 2}, {256, 3}, {256, 2}};
constexpr int kNShapes = sizeof(kShapes) / sizeof(kShapes[0]);
static_assert(kNShapes == FFP_BATCH_SHAPES, "the header states the number of launch shapes");

std::mutex g_tune_mu;
std::map<std::tuple<int, int, int, int>, int> g_tuned;  // (device, batch, max_m, max_n) -> shape

static int device_cus() {
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    return cus > 0 ? cus : 256;
}
static int batched_grid(int32_t batch, int shape) {
    const int g = device_cus() * kShapes[shape].per_cu;
    return batch < g ? batch : g;
}
static int max_grid(int32_t batch) {
    int g = 0;
    for (int i = 0; i < kNShapes; ++i) g = std::max(g, batched_grid(batch, i));
    return g;
}

size_t pluq_batched_ws(int32_t batch, int32_t max_m, int32_t max_n) {
    const size_t slot = (size_t)(max_m > 0 ? max_m : 1) * (size_t)(max_n > 0 ? max_n : 1);
    return 256 + (size_t)(batch > 0 ? batch : 0) * 4 + 256 + (size_t)max_grid(batch) * slot * 4 + 256;
}

static int tuned_shape(int32_t batch, int32_t max_m, int32_t max_n) {
    int dev = 0;
    (void)hipGetDevice(&dev);
    std::lock_guard<std::mutex> g(g_tune_mu);
    auto it = g_tuned.find(std::make_tuple(dev, batch, max_m, max_n));
    return it == g_tuned.end() ? 0 : it->second;
}

static int launch_shape(int shape, const Field &F, int32_t batch, const int32_t *m_arr, const int32_t *n_arr,
                        int32_t max_m, int32_t max_n, int32_t *A, const int64_t *A_off, int32_t *P,
                        const int64_t *P_off, int32_t *Q, const int64_t *Q_off, int32_t *rank, int32_t *rrp,
                        int32_t *crp, Arena &ws, hipStream_t s) {
    const size_t mk = ws.mark();
    int *counter = (int *)ws.take(256);
    int32_t *order = (int32_t *)ws.take((size_t)batch * 4);
    const int grid = batched_grid(batch, shape);
    const int64_t slot = (int64_t)(max_m > 0 ? max_m : 1) * (int64_t)(max_n > 0 ? max_n : 1);
    int32_t *slots = (int32_t *)ws.take((size_t)grid * (size_t)slot * 4);
    if (!counter || !order || !slots) return FFP_E_WORKSPACE;
    // pending-pivot buffers in LDS: as many pivots as the shape's share of
    // the compute unit's 160 KiB leaves room for (at most 16, or 32 with
    // 16-bit entries: centred residues of p < 2^16 fit an int16_t)
    const bool narrow = F.p < 65536u;
    const int64_t budget = (int64_t)(160 * 1024) / kShapes[shape].per_cu - (int64_t)sizeof(BShared) - 1024;
    const int64_t per = (narrow ? 2 : 4) * (int64_t)((max_m > 0 ? max_m : 1) + (max_n > 0 ? max_n : 1));
    int nb = (int)std::min<int64_t>(narrow ? 32 : 16, budget / per);
    if (nb < 1) nb = 1;
    const int kred = (int)std::min<int64_t>(nb, F.kexact > 0 ? F.kexact : 1);
    const size_t dyn = (size_t)nb * (size_t)per;
    // counter cleared by a kernel (not a memset) so that the sequence can be captured in a graph
    hipLaunchKernelGGL(k_batch_reset, dim3(1), dim3(1), 0, s, counter);
    hipLaunchKernelGGL(k_batch_order, dim3(1), dim3(1024), 0, s, batch, m_arr, n_arr, order);
    ProfScope prof(PK_BATCHED, 0.0, s, 0.0);
#define FFP_BAT(T_, PT_)                                                                                         \
    hipLaunchKernelGGL((k_pluq_batched<T_, PT_>), dim3(grid), dim3(T_), dyn, s, batch, m_arr, n_arr, A, A_off, P, P_off, \
                       Q, Q_off, rank, rrp, crp, counter, order, slots, slot, max_m, max_n, F.pd, F.pinv,        \
                       (int32_t)F.half, nb, kred)
    if (narrow) {
        if (kShapes[shape].threads == 1024) FFP_BAT(1024, true);
        else if (kShapes[shape].threads == 512) FFP_BAT(512, true);
        else FFP_BAT(256, true);
    } else {
        if (kShapes[shape].threads == 1024) FFP_BAT(1024, false);
        else if (kShapes[shape].threads == 512) FFP_BAT(512, false);
        else FFP_BAT(256, false);
    }
#undef FFP_BAT
    FFP_HIP_CHECK(hipGetLastError());
    ws.release(mk);
    return FFP_OK;
}

int pluq_batched_run(const Field &F, int32_t batch, const int32_t *m_arr, const int32_t *n_arr, int32_t max_m,
                     int32_t max_n, int32_t *A, const int64_t *A_off, int32_t *P, const int64_t *P_off, int32_t *Q,
                     const int64_t *Q_off, int32_t *rank, int32_t *rrp, int32_t *crp, Arena &ws, hipStream_t s) {
    if (batch <= 0) return FFP_OK;
    return launch_shape(tuned_shape(batch, max_m, max_n), F, batch, m_arr, n_arr, max_m, max_n, A, A_off, P, P_off,
                        Q, Q_off, rank, rrp, crp, ws, s);
}

int pluq_batched_tune(const Field &F, int32_t batch, const int32_t *m_arr, const int32_t *n_arr, int32_t max_m,
                      int32_t max_n, int32_t *A, int64_t a_elems, const int64_t *A_off, int32_t *P,
                      const int64_t *P_off, int32_t *Q, const int64_t *Q_off, int32_t *rank, int32_t *rrp,
                      int32_t *crp, Arena &ws, hipStream_t s, int *chosen, float *ms_out) {
    if (batch <= 0) return FFP_OK;
    // the pristine batch, restored before each timed run
    int32_t *keep = (int32_t *)ws.take((size_t)a_elems * 4);
    if (!keep) return FFP_E_WORKSPACE;
    FFP_HIP_CHECK(hipMemcpyAsync(keep, A, (size_t)a_elems * 4, hipMemcpyDeviceToDevice, s));
    hipEvent_t e0, e1;
    FFP_HIP_CHECK(hipEventCreate(&e0));
    FFP_HIP_CHECK(hipEventCreate(&e1));
    int best = 0;
    float best_ms = 0.f;
    int rc = FFP_OK;
    for (int sh = 0; sh < kNShapes && rc == FFP_OK; ++sh) {
        if ((rc = (int)hipMemcpyAsync(A, keep, (size_t)a_elems * 4, hipMemcpyDeviceToDevice, s)) != 0) {
            rc = FFP_E_HIP;
            break;
        }
        (void)hipEventRecord(e0, s);
        rc = launch_shape(sh, F, batch, m_arr, n_arr, max_m, max_n, A, A_off, P, P_off, Q, Q_off, rank, rrp, crp, ws, s);
        (void)hipEventRecord(e1, s);
        if (rc != FFP_OK) break;
        if (hipEventSynchronize(e1) != hipSuccess) { rc = FFP_E_HIP; break; }
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        if (ms_out) ms_out[sh] = ms;
        if (sh == 0 || ms < best_ms) { best = sh; best_ms = ms; }
    }
    // leave the batch factored by the chosen shape
    if (rc == FFP_OK && best != kNShapes - 1) {
        if (hipMemcpyAsync(A, keep, (size_t)a_elems * 4, hipMemcpyDeviceToDevice, s) != hipSuccess) rc = FFP_E_HIP;
        else rc = launch_shape(best, F, batch, m_arr, n_arr, max_m, max_n, A, A_off, P, P_off, Q, Q_off, rank, rrp,
                               crp, ws, s);
    }
    (void)hipStreamSynchronize(s);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != FFP_OK) return rc;
    int dev = 0;
    (void)hipGetDevice(&dev);
    {
        std::lock_guard<std::mutex> g(g_tune_mu);
        g_tuned[std::make_tuple(dev, batch, max_m, max_n)] = best;
    }
    if (chosen) *chosen = best;
    return FFP_OK;
}

// Record a launch shape for batches of this description (what the tuner
// stores after timing): later ffp_pluq_batched calls with the same (device,
// batch, max_m, max_n) use it.
int pluq_batched_set_shape(int32_t batch, int32_t max_m, int32_t max_n, int shape) {
    if (shape < 0 || shape >= kNShapes) return -4;
    int dev = 0;
    FFP_HIP_CHECK(hipGetDevice(&dev));
    std::lock_guard<std::mutex> g(g_tune_mu);
    g_tuned[std::make_tuple(dev, batch, max_m, max_n)] = shape;
    return FFP_OK;
}

}  // namespace ffp
