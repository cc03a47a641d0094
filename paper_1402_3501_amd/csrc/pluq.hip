// Tile-recursive PLUQ over Z/pZ (Section 4.1, "Tiled recursive elimination"):
// split rows and columns in halves, factor the top-left tile, update the
// other three, factor the top-right and bottom-left remainders (independent
// when the top-left tile is rank deficient), update and factor the
// bottom-right remainder, then restore the echelon layout with
// order-preserving block rotations.  Block sizes depend on the ranks found
// at run time (the dynamic splitting of Section 4.1), so the host drives the
// recursion and reads each sub-block's rank back.
//
// Leaf: a block small enough for one workgroup is factored by a kernel that
// keeps the block in registers (an 8 x 8 tile of FP64-embedded residues per
// thread), walks the same quadrant recursion with an explicit stack to pick
// each pivot (first nonzero of a one-row region / one-column region), and
// applies every pivot eagerly as a rank-one update with delayed reduction.
// Eager and deferred updates give the same Schur complements, so the leaf
// returns exactly what the block recursion would.
#include <algorithm>
#include <cstdlib>
#include <climits>
#include <cstring>
#include <mutex>
#include <vector>

#include "ffp_internal.hpp"
#include "ffp_device.hpp"

namespace ffp {

// ===================================================================== leaf
constexpr int kLT = 256;        // threads
constexpr int kLTile = 8;       // per-thread register tile edge
constexpr int kLMaxDim = 1024;  // max rows / columns of a leaf
constexpr int kLW = kLMaxDim / 32;
constexpr int kLStack = 24;

// blocks up to 64 x 64 go to the single-wave leaf; the register-tiled
// workgroup leaf takes skinny blocks (one side at most 32) that fit it
static inline bool leaf64_fits(int64_t m, int64_t n) { return m >= 1 && n >= 1 && m <= 64 && n <= 64; }
static inline bool leaf_fits(int64_t m, int64_t n) {
    return m >= 1 && n >= 1 && m <= kLMaxDim && n <= kLMaxDim && (m <= 32 || n <= 32) &&
           ((m + kLTile - 1) / kLTile) * ((n + kLTile - 1) / kLTile) <= kLT;
}

struct LFrame {
    uint32_t rows[kLW], cols[kLW], top[kLW], left[kLW];
    int stage;
};

struct LeafShared {
    uint32_t rowdone[kLW], coldone[kLW];
    uint32_t mask[kLW];  // base region: columns (row base) or rows (column base)
    LFrame st[kLStack];
    int sp, type, bx, piv, r, pend_x, pend_y;
    int prow[kLMaxDim], pcol[kLMaxDim];
    int rpos[kLMaxDim], cpos[kLMaxDim];
    double urow[kLMaxDim], vcol[kLMaxDim];
    int wcnt[kLW + 1];
};

enum { LT_FINISHED = 0, LT_ROW = 1, LT_COL = 2 };

__device__ __forceinline__ bool bit(const uint32_t *m, int i) { return (m[i >> 5] >> (i & 31)) & 1u; }

__device__ static int popc_mask(const uint32_t *m, int nw) {
    int c = 0;
    for (int w = 0; w < nw; ++w) c += __popc(m[w]);
    return c;
}
__device__ static int first_bit(const uint32_t *m, int nw) {
    for (int w = 0; w < nw; ++w)
        if (m[w]) return w * 32 + __ffs(m[w]) - 1;
    return -1;
}
// out = the first k set bits of m
__device__ static void first_k(const uint32_t *m, int nw, int k, uint32_t *out) {
    for (int w = 0; w < nw; ++w) {
        uint32_t x = m[w];
        int c = __popc(x);
        if (k >= c) { out[w] = x; k -= c; }
        else {
            uint32_t o = 0;
            while (k > 0) { uint32_t low = x & (~x + 1u); o |= low; x ^= low; --k; }
            out[w] = o;
        }
    }
}

// single-thread walk of the quadrant recursion to the next one-row / one-column region
__device__ static void leaf_advance(LeafShared &S, int nwr, int nwc) {
    if (S.pend_x >= 0) {
        const int x = S.pend_x, y = S.pend_y;
        S.rowdone[x >> 5] |= 1u << (x & 31);
        S.coldone[y >> 5] |= 1u << (y & 31);
        S.prow[S.r] = x;
        S.pcol[S.r] = y;
        S.r += 1;
        S.pend_x = -1;
    }
    while (S.sp > 0) {
        LFrame &f = S.st[S.sp - 1];
        if (f.stage == 0) {
            const int nr = popc_mask(f.rows, nwr), nc = popc_mask(f.cols, nwc);
            if (nr == 0 || nc == 0) { S.sp--; continue; }
            if (nr == 1) {
                S.type = LT_ROW;
                S.bx = first_bit(f.rows, nwr);
                for (int w = 0; w < nwc; ++w) S.mask[w] = f.cols[w];
                S.sp--;
                return;
            }
            if (nc == 1) {
                S.type = LT_COL;
                S.bx = first_bit(f.cols, nwc);
                for (int w = 0; w < nwr; ++w) S.mask[w] = f.rows[w];
                S.sp--;
                return;
            }
            first_k(f.rows, nwr, nr / 2, f.top);
            first_k(f.cols, nwc, nc / 2, f.left);
            f.stage = 1;
            LFrame &c = S.st[S.sp++];
            for (int w = 0; w < nwr; ++w) c.rows[w] = f.top[w];
            for (int w = 0; w < nwc; ++w) c.cols[w] = f.left[w];
            c.stage = 0;
            continue;
        }
        if (f.stage <= 3) {
            const int st = f.stage;
            f.stage = st + 1;
            LFrame &c = S.st[S.sp++];
            for (int w = 0; w < nwr; ++w) {
                const uint32_t top = f.top[w], bot = f.rows[w] & ~f.top[w];
                c.rows[w] = st == 1 ? (top & ~S.rowdone[w]) : st == 2 ? bot : (bot & ~S.rowdone[w]);
            }
            for (int w = 0; w < nwc; ++w) {
                const uint32_t left = f.left[w], right = f.cols[w] & ~f.left[w];
                c.cols[w] = st == 1 ? right : st == 2 ? (left & ~S.coldone[w]) : (right & ~S.coldone[w]);
            }
            c.stage = 0;
            continue;
        }
        S.sp--;
    }
    S.type = LT_FINISHED;
}

template <bool RED>
__global__ __launch_bounds__(kLT) void k_pluq_leaf(int mb, int nb, int32_t *__restrict__ A, int64_t lda,
                                                   int32_t *__restrict__ P, int32_t *__restrict__ Q,
                                                   int64_t *__restrict__ rank_out, double p, double pinv,
                                                   int32_t half, int64_t kexact) {
    __shared__ LeafShared S;
    const int tid = threadIdx.x;
    const int TC = (nb + kLTile - 1) / kLTile, TR = (mb + kLTile - 1) / kLTile;
    const bool owner = tid < TR * TC;
    const int i0 = owner ? (tid / TC) * kLTile : 0, c0 = owner ? (tid % TC) * kLTile : 0;
    const int nwr = (mb + 31) >> 5, nwc = (nb + 31) >> 5;

    double w[kLTile][kLTile];
#pragma unroll
    for (int a = 0; a < kLTile; ++a)
#pragma unroll
        for (int b = 0; b < kLTile; ++b) {
            const int i = i0 + a, c = c0 + b;
            w[a][b] = (owner && i < mb && c < nb) ? centre(A[(int64_t)i * lda + c], p, half) : 0.0;
        }

    if (tid == 0) {
        for (int x = 0; x < kLW; ++x) { S.rowdone[x] = 0; S.coldone[x] = 0; }
        LFrame &f = S.st[0];
        for (int x = 0; x < nwr; ++x) {
            const int lo = x * 32, cnt = mb - lo >= 32 ? 32 : mb - lo;
            f.rows[x] = cnt >= 32 ? 0xffffffffu : ((1u << cnt) - 1u);
        }
        for (int x = 0; x < nwc; ++x) {
            const int lo = x * 32, cnt = nb - lo >= 32 ? 32 : nb - lo;
            f.cols[x] = cnt >= 32 ? 0xffffffffu : ((1u << cnt) - 1u);
        }
        f.stage = 0;
        S.sp = 1;
        S.r = 0;
        S.pend_x = -1;
    }
    int64_t cnt = 0;
    __syncthreads();

    while (true) {
        if (tid == 0) {
            leaf_advance(S, nwr, nwc);
            S.piv = INT_MAX;
        }
        __syncthreads();
        const int type = S.type;
        if (type == LT_FINISHED) break;
        const int bx = S.bx;
        // ---- search: first nonzero of the one-row / one-column region
        if (owner) {
            if (type == LT_ROW && bx >= i0 && bx < i0 + kLTile) {
                const int xa = bx - i0;
                int best = INT_MAX;
#pragma unroll
                for (int a = 0; a < kLTile; ++a) {
                    if (a != xa) continue;
#pragma unroll
                    for (int b = kLTile - 1; b >= 0; --b) {
                        const int c = c0 + b;
                        if (c < nb && bit(S.mask, c) && mod_canon(w[a][b], p, pinv) != 0.0) best = c;
                    }
                }
                if (best != INT_MAX) atomicMin(&S.piv, best);
            } else if (type == LT_COL && bx >= c0 && bx < c0 + kLTile) {
                const int yb = bx - c0;
                int best = INT_MAX;
#pragma unroll
                for (int b = 0; b < kLTile; ++b) {
                    if (b != yb) continue;
#pragma unroll
                    for (int a = kLTile - 1; a >= 0; --a) {
                        const int i = i0 + a;
                        if (i < mb && bit(S.mask, i) && mod_canon(w[a][b], p, pinv) != 0.0) best = i;
                    }
                }
                if (best != INT_MAX) atomicMin(&S.piv, best);
            }
        }
        __syncthreads();
        if (S.piv == INT_MAX) continue;  // no pivot in this region (uniform)
        const int x = type == LT_ROW ? bx : S.piv;
        const int y = type == LT_ROW ? S.piv : bx;
        // ---- pivot row (reduced, centred: final U entries) and pivot column to LDS
        if (owner) {
            if (x >= i0 && x < i0 + kLTile) {
#pragma unroll
                for (int a = 0; a < kLTile; ++a) {
                    if (a != x - i0) continue;
#pragma unroll
                    for (int b = 0; b < kLTile; ++b) {
                        const int c = c0 + b;
                        if (c < nb && !bit(S.coldone, c)) {
                            double u = mod_canon(w[a][b], p, pinv);
                            u = u > (double)half ? u - p : u;
                            w[a][b] = u;
                            S.urow[c] = u;
                        }
                    }
                }
            }
            if (y >= c0 && y < c0 + kLTile) {
#pragma unroll
                for (int b = 0; b < kLTile; ++b) {
                    if (b != y - c0) continue;
#pragma unroll
                    for (int a = 0; a < kLTile; ++a) {
                        const int i = i0 + a;
                        if (i < mb && !bit(S.rowdone, i) && i != x) S.vcol[i] = mod_canon(w[a][b], p, pinv);
                    }
                }
            }
        }
        __syncthreads();
        // ---- multipliers and rank-one update of the active block
        if (owner) {
            double piv = S.urow[y];
            if (piv < 0.0) piv += p;
            const double inv = (double)inv_mod((int32_t)piv, (int32_t)p);
            bool colact[kLTile];
            double u[kLTile];
#pragma unroll
            for (int b = 0; b < kLTile; ++b) {
                const int c = c0 + b;
                colact[b] = c < nb && c != y && !bit(S.coldone, c);
                u[b] = colact[b] ? S.urow[c] : 0.0;
            }
#pragma unroll
            for (int a = 0; a < kLTile; ++a) {
                const int i = i0 + a;
                if (i >= mb || i == x || bit(S.rowdone, i)) continue;
                double l = mod_canon(S.vcol[i] * inv, p, pinv);
                l = l > (double)half ? l - p : l;
#pragma unroll
                for (int b = 0; b < kLTile; ++b) {
                    if (c0 + b == y) w[a][b] = l;
                    else if (colact[b]) w[a][b] = fma(-l, u[b], w[a][b]);
                }
            }
            if (RED) {
                if (++cnt >= kexact) {
                    cnt = 0;
#pragma unroll
                    for (int a = 0; a < kLTile; ++a) {
                        const int i = i0 + a;
                        if (i >= mb || i == x || bit(S.rowdone, i)) continue;
#pragma unroll
                        for (int b = 0; b < kLTile; ++b)
                            if (colact[b]) w[a][b] = mod_near(w[a][b], p, pinv);
                    }
                }
            }
        }
        if (tid == 0) {
            S.pend_x = x;
            S.pend_y = y;
        }
        __syncthreads();
    }

    // ---- output positions: pivots in order, then the others ascending
    const int r = S.r;
    if (tid == 0) {
        int acc = 0;
        for (int x = 0; x < nwr; ++x) {
            S.wcnt[x] = acc;
            acc += __popc(~S.rowdone[x] & (x * 32 + 32 <= mb ? 0xffffffffu : ((1u << (mb - x * 32)) - 1u)));
        }
    }
    __syncthreads();
    for (int i = tid; i < mb; i += kLT) {
        if (!bit(S.rowdone, i)) {
            const uint32_t below = (i & 31) ? (~S.rowdone[i >> 5] & ((1u << (i & 31)) - 1u)) : 0u;
            S.rpos[i] = r + S.wcnt[i >> 5] + __popc(below);
        }
    }
    for (int k = tid; k < r; k += kLT) S.rpos[S.prow[k]] = k;
    __syncthreads();
    if (tid == 0) {
        int acc = 0;
        for (int x = 0; x < nwc; ++x) {
            S.wcnt[x] = acc;
            acc += __popc(~S.coldone[x] & (x * 32 + 32 <= nb ? 0xffffffffu : ((1u << (nb - x * 32)) - 1u)));
        }
    }
    __syncthreads();
    for (int c = tid; c < nb; c += kLT) {
        if (!bit(S.coldone, c)) {
            const uint32_t below = (c & 31) ? (~S.coldone[c >> 5] & ((1u << (c & 31)) - 1u)) : 0u;
            S.cpos[c] = r + S.wcnt[c >> 5] + __popc(below);
        }
    }
    for (int k = tid; k < r; k += kLT) S.cpos[S.pcol[k]] = k;
    __syncthreads();
    if (owner) {
#pragma unroll
        for (int a = 0; a < kLTile; ++a) {
            const int i = i0 + a;
            if (i >= mb) continue;
            const int64_t ro = (int64_t)S.rpos[i] * lda;
#pragma unroll
            for (int b = 0; b < kLTile; ++b) {
                const int c = c0 + b;
                if (c < nb) A[ro + S.cpos[c]] = (int32_t)mod_canon(w[a][b], p, pinv);
            }
        }
    }
    for (int i = tid; i < mb; i += kLT) P[S.rpos[i]] = i;
    for (int c = tid; c < nb; c += kLT) Q[S.cpos[c]] = c;
    if (tid == 0) *rank_out = r;
}

// ===================================================================== index bookkeeping
// Composes the local permutation of a recursion node from its children's and
// applies the final rotation (see the layout comment in pluq_rec).
struct NodeDims {
    int64_t m, n, m1, n1, r1, r2, r3, r4;
};

__device__ __forceinline__ int32_t node_index(const NodeDims &d, int64_t t, const int32_t *Pcur, const int32_t *P2,
                                              const int32_t *P3, const int32_t *P4, const int32_t *Qcur,
                                              const int32_t *Q2, const int32_t *Q3, const int32_t *Q4) {
    if (t < d.m) {
        // destination order [a f g R f' rest] -> source position in the current layout
        const int64_t i = t;
        const int64_t a = d.r1, f = d.r2, g = d.r3, R = d.r4, fp = d.m1 - d.r1 - d.r2;
        int64_t s;
        if (i < a + f) s = i;
        else if (i < a + f + g) s = d.m1 + (i - a - f);
        else if (i < a + f + g + R) s = d.m1 + d.r3 + (i - a - f - g);
        else if (i < a + f + g + R + fp) s = d.r1 + d.r2 + (i - a - f - g - R);
        else s = d.m1 + d.r3 + d.r4 + (i - a - f - g - R - fp);
        // composed row id of current position s
        int64_t v;
        if (s < d.r1) v = Pcur[s];
        else if (s < d.m1) v = Pcur[d.r1 + P2[s - d.r1]];
        else if (s < d.m1 + d.r3) v = d.m1 + P3[s - d.m1];
        else v = d.m1 + P3[d.r3 + P4[s - d.m1 - d.r3]];
        return (int32_t)v;
    } else {
        const int64_t j = t - d.m;
        const int64_t a = d.r1, f = d.r2, g = d.r3, R = d.r4, gp = d.n1 - d.r1 - d.r3;
        int64_t s;
        if (j < a) s = j;
        else if (j < a + f) s = d.n1 + (j - a);
        else if (j < a + f + g) s = d.r1 + (j - a - f);
        else if (j < a + f + g + R) s = d.n1 + d.r2 + (j - a - f - g);
        else if (j < a + f + g + R + gp) s = d.r1 + d.r3 + (j - a - f - g - R);
        else s = d.n1 + d.r2 + d.r4 + (j - a - f - g - R - gp);
        int64_t v;
        if (s < d.r1) v = Qcur[s];
        else if (s < d.n1) v = Qcur[d.r1 + Q3[s - d.r1]];
        else if (s < d.n1 + d.r2) v = d.n1 + Q2[s - d.n1];
        else v = d.n1 + Q2[d.r2 + Q4[s - d.n1 - d.r2]];
        return (int32_t)v;
    }
}
__global__ void k_node_index(NodeDims d, const int32_t *__restrict__ Pcur, const int32_t *__restrict__ P2,
                             const int32_t *__restrict__ P3, const int32_t *__restrict__ P4,
                             const int32_t *__restrict__ Qcur, const int32_t *__restrict__ Q2,
                             const int32_t *__restrict__ Q3, const int32_t *__restrict__ Q4,
                             int32_t *__restrict__ Pnew, int32_t *__restrict__ Qnew) {
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t < d.m + d.n) {
        const int32_t v = node_index(d, t, Pcur, P2, P3, P4, Qcur, Q2, Q3, Q4);
        if (t < d.m) Pnew[t] = v;
        else Qnew[t - d.m] = v;
    }
}
// the same for a small node in place, one workgroup, through LDS
__global__ __launch_bounds__(1024) void k_node_index_lds(NodeDims d, int32_t *__restrict__ P,
                                                         const int32_t *__restrict__ P2,
                                                         const int32_t *__restrict__ P3,
                                                         const int32_t *__restrict__ P4, int32_t *__restrict__ Q,
                                                         const int32_t *__restrict__ Q2,
                                                         const int32_t *__restrict__ Q3,
                                                         const int32_t *__restrict__ Q4) {
    extern __shared__ int32_t ibuf[];
    const int64_t tot = d.m + d.n;
    for (int64_t t = threadIdx.x; t < tot; t += blockDim.x) ibuf[t] = node_index(d, t, P, P2, P3, P4, Q, Q2, Q3, Q4);
    __syncthreads();
    for (int64_t t = threadIdx.x; t < tot; t += blockDim.x) {
        if (t < d.m) P[t] = ibuf[t];
        else Q[t - d.m] = ibuf[t];
    }
}

__global__ void k_iota(int32_t *__restrict__ v, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        v[i] = (int32_t)i;
}

__global__ void k_set_int(int *dst, int v) { *dst = v; }

static int iota(int32_t *v, int64_t n, hipStream_t s) {
    if (n <= 0) return FFP_OK;
    unsigned g = (unsigned)((n + 255) / 256);
    if (g > 1024) g = 1024;
    hipLaunchKernelGGL(k_iota, dim3(g), dim3(256), 0, s, v, n);
    FFP_HIP_CHECK(hipGetLastError());
    return FFP_OK;
}

// ===================================================================== host recursion
// Host words the leaves of the general recursion write their rank into
// directly (pinned, coherent, device-visible): the host reads a rank after
// one stream synchronisation, with no copy on the stream.  One word per
// concurrent call, taken from a pool and kept for the life of the process.
namespace {
std::mutex g_pin_mu;
std::vector<RankWord> g_rank_pool;
}  // namespace

int rank_word_get(RankWord *w) {
    std::lock_guard<std::mutex> g(g_pin_mu);
    if (!g_rank_pool.empty()) {
        *w = g_rank_pool.back();
        g_rank_pool.pop_back();
        return FFP_OK;
    }
    FFP_HIP_CHECK(hipHostMalloc((void **)&w->host, 64, hipHostMallocMapped | hipHostMallocCoherent));
    FFP_HIP_CHECK(hipHostGetDevicePointer((void **)&w->dev, w->host, 0));
    return FFP_OK;
}
void rank_word_put(const RankWord &w) {
    std::lock_guard<std::mutex> g(g_pin_mu);
    g_rank_pool.push_back(w);
}

namespace {

// A second stream (one per device, default priority) for the triangular
// solve E = C1 U1^-1 and the product G -= E V1, which are independent of
// D = L1^-1 B1: the two latency-bound solve chains then overlap.
std::mutex g_side_mu;
hipStream_t g_side[64];
std::vector<hipEvent_t> g_evpool;

int side_stream(hipStream_t *out) {
    int dev = 0;
    FFP_HIP_CHECK(hipGetDevice(&dev));
    std::lock_guard<std::mutex> g(g_side_mu);
    if (dev < 0 || dev >= 64) return FFP_E_UNSUPPORTED;
    if (!g_side[dev]) FFP_HIP_CHECK(hipStreamCreateWithFlags(&g_side[dev], hipStreamNonBlocking));
    *out = g_side[dev];
    return FFP_OK;
}
int ev_get(hipEvent_t *e) {
    std::lock_guard<std::mutex> g(g_side_mu);
    if (!g_evpool.empty()) {
        *e = g_evpool.back();
        g_evpool.pop_back();
        return FFP_OK;
    }
    FFP_HIP_CHECK(hipEventCreateWithFlags(e, hipEventDisableTiming));
    return FFP_OK;
}
void ev_put(hipEvent_t e) {
    std::lock_guard<std::mutex> g(g_side_mu);
    g_evpool.push_back(e);
}

PermSpec by_index(const int32_t *idx) {
    PermSpec ps;
    ps.idx = idx;
    return ps;
}

struct Ctx {
    int path;
    const Field *F;
    Arena *ws;
    hipStream_t s;
    int64_t *rank_dev;   // device address of a pinned host word the leaves write their rank to
    int64_t *rank_host;  // the same word for the host
    int *flag_dev;       // device word: generic-attempt flag, zero-block flag
    int64_t gen_k = 0;   // order of the running generic attempt
};

int read_rank(const Ctx &c, int64_t *out) {
    FFP_HIP_CHECK(hipStreamSynchronize(c.s));
    *out = *(const volatile int64_t *)c.rank_host;
    return FFP_OK;
}

int fgemm_sub(Ctx &c, int64_t m, int64_t n, int64_t k, const int32_t *A, int64_t lda, const int32_t *B,
              int64_t ldb, int32_t *C, int64_t ldc) {
    if (m <= 0 || n <= 0 || k <= 0) return FFP_OK;
    return fgemm_any(c.path, *c.F, 0, 0, m, n, k, c.F->p - 1, A, lda, B, ldb, 1, C, ldc, *c.ws, c.s);
}

int trsm_sub(Ctx &c, int side, int uplo, int diag, int64_t m, int64_t n, const int32_t *T, int64_t ldt,
             int32_t *B, int64_t ldb) {
    if (m <= 0 || n <= 0) return FFP_OK;
    return ftrsm_run(c.path, *c.F, side, uplo, 0, diag, m, n, 1, T, ldt, B, ldb, *c.ws, c.s);
}

// D = L1^-1 B1 (main stream), E = C1 U1^-1 then G -= E V1 (side stream),
// then [F; H] -= [M1; E] D after both (A1 = L1\U1 holds r1 pivots).
int node_updates(Ctx &c, int64_t m, int64_t n, int64_t m1, int64_t n1, int64_t r1, int32_t *A, int64_t lda) {
    if (r1 <= 0) return FFP_OK;
    const Field &F = *c.F;
    Arena &ws = *c.ws;
    hipStream_t s2;
    FFP_CHECK(side_stream(&s2));
    // workspace of the side stream, reserved until the join
    const bool i8 = c.path != FFP_PATH_FP64 && F.limbs > 0;
    size_t need = ftrsm_ws(i8 ? FFP_PATH_INT8 : FFP_PATH_FP64, F, 1, m - m1, r1);
    if (i8) {
        const size_t b = fgemm_i8_ws(F, m - m1, n1 - r1, r1);
        need = need > b ? need : b;
    }
    need += 1024;
    const size_t mk = ws.mark();
    Arena a2;
    a2.base = (char *)ws.take(need);
    a2.cap = need;
    if (!a2.base) return FFP_E_WORKSPACE;
    hipEvent_t fork, join;
    FFP_CHECK(ev_get(&fork));
    FFP_CHECK(ev_get(&join));
    FFP_HIP_CHECK(hipEventRecord(fork, c.s));
    FFP_HIP_CHECK(hipStreamWaitEvent(s2, fork, 0));
    Ctx c2 = c;
    c2.s = s2;
    c2.ws = &a2;
    FFP_CHECK(trsm_sub(c2, 1, 1, 0, m - m1, r1, A, lda, A + m1 * lda, lda));                         // E
    FFP_CHECK(fgemm_sub(c2, m - m1, n1 - r1, r1, A + m1 * lda, lda, A + r1, lda, A + m1 * lda + r1, lda));  // G
    FFP_HIP_CHECK(hipEventRecord(join, s2));
    FFP_CHECK(trsm_sub(c, 0, 0, 1, r1, n - n1, A, lda, A + n1, lda));                                // D
    FFP_HIP_CHECK(hipStreamWaitEvent(c.s, join, 0));
    FFP_CHECK(fgemm_sub(c, m - r1, n - n1, r1, A + r1 * lda, lda, A + n1, lda, A + r1 * lda + n1, lda));  // F, H
    ev_put(fork);
    ev_put(join);
    ws.release(mk);
    return FFP_OK;
}

int rows_perm(Ctx &c, int64_t m, int64_t n, int32_t *A, int64_t lda, const int32_t *perm) {
    return permute_inplace(m, n, A, lda, by_index(perm), PermSpec(), *c.ws, c.s);
}
int cols_perm(Ctx &c, int64_t m, int64_t n, int32_t *A, int64_t lda, const int32_t *perm) {
    return permute_inplace(m, n, A, lda, PermSpec(), by_index(perm), *c.ws, c.s);
}

// segment permutation from (dst-order list of (src start, len)); returns false if identity
bool make_seg(SegPerm &sp, const int64_t (*segs)[2], int nseg, int64_t lo, int64_t hi) {
    sp.nseg = 0;
    int64_t d = 0;
    bool ident = true;
    for (int i = 0; i < nseg; ++i) {
        const int64_t src = segs[i][0], len = segs[i][1];
        if (len <= 0) continue;
        if (src != d) ident = false;
        if (d + len > lo && d < hi) {
            sp.dst[sp.nseg] = d - lo;
            sp.src[sp.nseg] = src - lo;
            sp.len[sp.nseg] = len;
            sp.nseg++;
        }
        d += len;
    }
    return !ident;
}

}  // namespace
int try_generic(Ctx &c, int64_t m, int64_t n, int32_t *A, int64_t lda, bool *ok, int64_t *k0);
int read_flag(const Ctx &c, int64_t *out);
namespace {

// any nonzero entry in an m x n block: *flag |= 1 (entries are canonical)
__global__ __launch_bounds__(256) void k_any_nonzero(int64_t m, int64_t n, const int32_t *__restrict__ A, int64_t lda,
                                                     int *__restrict__ flag) {
    bool nz = false;
    for (int64_t i = blockIdx.x; i < m; i += gridDim.x) {
        const int32_t *row = A + i * lda;
        for (int64_t j = threadIdx.x; j < n; j += 256) nz |= row[j] != 0;
    }
    if (__syncthreads_or(nz) && threadIdx.x == 0) atomicOr(flag, 1);
}

// A sub-block of a rank-deficient input is often zero (its rank spent
// above): one reduction and one read-back then replace its whole
// recursion (every leaf of which would read a rank back).
constexpr int64_t kZeroCheckMin = 128 * 128;

int block_is_zero(Ctx &c, int64_t m, int64_t n, const int32_t *A, int64_t lda, bool *zero) {
    *zero = false;
    if (m * n < kZeroCheckMin) return FFP_OK;
    hipLaunchKernelGGL(k_set_int, dim3(1), dim3(1), 0, c.s, c.flag_dev, 0);
    const unsigned g = (unsigned)(m < 1024 ? m : 1024);
    hipLaunchKernelGGL(k_any_nonzero, dim3(g), dim3(256), 0, c.s, m, n, A, lda, c.flag_dev);
    FFP_HIP_CHECK(hipGetLastError());
    int64_t f = 0;
    FFP_CHECK(read_flag(c, &f));
    *zero = f == 0;
    return FFP_OK;
}

// *pid / *qid: set when the block's P / Q came out as the identity, so that
// the parent can skip applying them
int pluq_sub(Ctx &c, int64_t m, int64_t n, int32_t *A, int64_t lda, int32_t *P, int32_t *Q, int64_t *rank, bool *pid,
             bool *qid);

// gen_ok: every leading minor of this block up to that order is known to be
// nonzero (from a failed generic attempt on a block with the same top-left
// corner); a leading tile within that order is then factored as a plain LU.
int pluq_rec(Ctx &c, int64_t m, int64_t n, int32_t *A, int64_t lda, int32_t *P, int32_t *Q, int64_t *rank,
             int64_t gen_ok, bool *pid, bool *qid) {
    hipStream_t s = c.s;
    Arena &ws = *c.ws;
    *pid = false;
    *qid = false;
    if (m == 0 || n == 0) {
        FFP_CHECK(iota(P, m, s));
        FFP_CHECK(iota(Q, n, s));
        *rank = 0;
        *pid = *qid = true;
        return FFP_OK;
    }
    const Field &F = *c.F;
    if (leaf64_fits(m, n)) {
        // most blocks of an input whose rank profile is generic almost
        // everywhere (a uniform matrix mod a small prime) are themselves
        // generic: the eight-wave generic leaf is tried first (it writes the
        // block only when every pivot is nonzero), the one-wave general leaf
        // then only writes P, Q and the rank, or factors the untouched block
        const int *gen_done = nullptr;
        if (m >= 16 && n >= 16) {
            hipLaunchKernelGGL(k_set_int, dim3(1), dim3(1), 0, s, c.flag_dev, 0);
            FFP_CHECK(leaf64_launch(F, m, n, A, lda, nullptr, nullptr, nullptr, c.flag_dev, nullptr, nullptr, s));
            gen_done = c.flag_dev;
        }
        FFP_CHECK(leaf64_launch(F, m, n, A, lda, P, Q, c.rank_dev, nullptr, nullptr, nullptr, s, nullptr, nullptr,
                                nullptr, 0, nullptr, 0, 0, gen_done));
        int64_t word = 0;
        FFP_CHECK(read_rank(c, &word));
        *rank = word & ((1ll << 40) - 1);
        *pid = (word >> 40) & 1;
        *qid = (word >> 41) & 1;
        return FFP_OK;
    }
    if (leaf_fits(m, n)) {
        const bool red = F.kexact < kLMaxDim;
        ProfScope prof(PK_LEAF, 0.0, s, 8.0 * (double)m * (double)n);
        if (red)
            hipLaunchKernelGGL((k_pluq_leaf<true>), dim3(1), dim3(kLT), 0, s, (int)m, (int)n, A, lda, P, Q,
                               c.rank_dev, F.pd, F.pinv, (int32_t)F.half, F.kexact);
        else
            hipLaunchKernelGGL((k_pluq_leaf<false>), dim3(1), dim3(kLT), 0, s, (int)m, (int)n, A, lda, P, Q,
                               c.rank_dev, F.pd, F.pinv, (int32_t)F.half, F.kexact);
        FFP_HIP_CHECK(hipGetLastError());
        return read_rank(c, rank);
    }
    const int64_t m1 = m / 2, n1 = n / 2;
    // ---- 1. top-left tile (same corner: same leading minors)
    int64_t r1 = 0;
    bool p1id = false, q1id = false;
    {
        const int64_t k1 = m1 < n1 ? m1 : n1;
        bool gen = false;
        int64_t k0 = 0;
        if (k1 > 64 && k1 <= gen_ok) FFP_CHECK(try_generic(c, m1, n1, A, lda, &gen, &k0));
        if (gen) {
            FFP_CHECK(iota(P, m1, s));
            FFP_CHECK(iota(Q, n1, s));
            r1 = k1;
            p1id = q1id = true;
        } else {
            FFP_CHECK(pluq_rec(c, m1, n1, A, lda, P, Q, &r1, gen_ok, &p1id, &q1id));
        }
    }
    // ---- 2. [B1; B2] = P1^T A2,  [C1 C2] = A3 Q1^T  (identities skipped)
    if (!p1id) FFP_CHECK(rows_perm(c, m1, n - n1, A + n1, lda, P));
    if (!q1id) FFP_CHECK(cols_perm(c, m - m1, n1, A + m1 * lda, lda, Q));
    // ---- 3. D = L1^-1 B1, E = C1 U1^-1, [F; H] -= [M1; E] D, G = C2 - E V1
    FFP_CHECK(node_updates(c, m, n, m1, n1, r1, A, lda));
    // ---- 4. factor F (top-right remainder) and G (bottom-left remainder)
    const size_t mk = ws.mark();
    int32_t *P2 = (int32_t *)ws.take((size_t)(m1 - r1) * 4);
    int32_t *Q2 = (int32_t *)ws.take((size_t)(n - n1) * 4);
    int32_t *P3 = (int32_t *)ws.take((size_t)(m - m1) * 4);
    int32_t *Q3 = (int32_t *)ws.take((size_t)(n1 - r1) * 4);
    if ((!P2 && m1 - r1 > 0) || (!Q2 && n - n1 > 0) || (!P3 && m - m1 > 0) || (!Q3 && n1 - r1 > 0))
        return FFP_E_WORKSPACE;
    int64_t r2 = 0, r3 = 0;
    bool p2id = false, q2id = false, p3id = false, q3id = false;
    FFP_CHECK(pluq_sub(c, m1 - r1, n - n1, A + r1 * lda + n1, lda, P2, Q2, &r2, &p2id, &q2id));
    FFP_CHECK(pluq_sub(c, m - m1, n1 - r1, A + m1 * lda + r1, lda, P3, Q3, &r3, &p3id, &q3id));
    // ---- 5. carry the sub-permutations to the rest of their rows / columns
    if (r1 > 0) {
        if (!p2id) FFP_CHECK(rows_perm(c, m1 - r1, r1, A + r1 * lda, lda, P2));   // M1
        if (!q3id) FFP_CHECK(cols_perm(c, r1, n1 - r1, A + r1, lda, Q3));         // V1
        if (!p3id) FFP_CHECK(rows_perm(c, m - m1, r1, A + m1 * lda, lda, P3));    // E
        if (!q2id) FFP_CHECK(cols_perm(c, r1, n - n1, A + n1, lda, Q2));          // D
    }
    if (!p3id || !q2id)                                                           // H
        FFP_CHECK(permute_inplace(m - m1, n - n1, A + m1 * lda + n1, lda, p3id ? PermSpec() : by_index(P3),
                                  q2id ? PermSpec() : by_index(Q2), ws, s));
    // ---- 6. [I; K] = [H1; H3] U2^-1, O = L3^-1 (H2 - I V2), R = H4 - K V2 - M3 O
    int32_t *const H = A + m1 * lda + n1;
    if (r2 > 0) FFP_CHECK(trsm_sub(c, 1, 1, 0, m - m1, r2, A + r1 * lda + n1, lda, H, lda));
    if (r3 > 0) {
        FFP_CHECK(fgemm_sub(c, r3, n - n1 - r2, r2, H, lda, A + r1 * lda + n1 + r2, lda, H + r2, lda));
        FFP_CHECK(trsm_sub(c, 0, 0, 1, r3, n - n1 - r2, A + m1 * lda + r1, lda, H + r2, lda));
    }
    int32_t *const R = H + r3 * lda + r2;
    FFP_CHECK(fgemm_sub(c, m - m1 - r3, n - n1 - r2, r2, H + r3 * lda, lda, A + r1 * lda + n1 + r2, lda, R, lda));
    FFP_CHECK(fgemm_sub(c, m - m1 - r3, n - n1 - r2, r3, A + (m1 + r3) * lda + r1, lda, H + r2, lda, R, lda));
    // ---- 7. factor R
    int32_t *P4 = (int32_t *)ws.take((size_t)(m - m1 - r3) * 4);
    int32_t *Q4 = (int32_t *)ws.take((size_t)(n - n1 - r2) * 4);
    if ((!P4 && m - m1 - r3 > 0) || (!Q4 && n - n1 - r2 > 0)) return FFP_E_WORKSPACE;
    int64_t r4 = 0;
    bool p4id = false, q4id = false;
    FFP_CHECK(pluq_sub(c, m - m1 - r3, n - n1 - r2, R, lda, P4, Q4, &r4, &p4id, &q4id));
    if (!p4id) FFP_CHECK(rows_perm(c, m - m1 - r3, n1 + r2, A + (m1 + r3) * lda, lda, P4));
    if (!q4id) FFP_CHECK(cols_perm(c, m1 + r3, n - n1 - r2, A + n1 + r2, lda, Q4));
    // ---- 8. final rotations: rows [a f f' g R r'] -> [a f g R f' r'],
    //         columns [a g g' f R c'] -> [a f g R g' c']
    {
        const int64_t rseg[6][2] = {{0, r1}, {r1, r2}, {m1, r3}, {m1 + r3, r4}, {r1 + r2, m1 - r1 - r2},
                                    {m1 + r3 + r4, m - m1 - r3 - r4}};
        const int64_t lo = r1 + r2, hi = m1 + r3 + r4;
        PermSpec rp;
        if (hi > lo && make_seg(rp.seg, rseg, 6, lo, hi))
            FFP_CHECK(permute_inplace(hi - lo, n, A + lo * lda, lda, rp, PermSpec(), ws, s));
        const int64_t cseg[6][2] = {{0, r1}, {n1, r2}, {r1, r3}, {n1 + r2, r4}, {r1 + r3, n1 - r1 - r3},
                                    {n1 + r2 + r4, n - n1 - r2 - r4}};
        const int64_t clo = r1, chi = n1 + r2 + r4;
        PermSpec cp;
        if (chi > clo && make_seg(cp.seg, cseg, 6, clo, chi))
            FFP_CHECK(permute_inplace(m, chi - clo, A + clo, lda, PermSpec(), cp, ws, s));
    }
    // ---- 9. local permutations of this node
    {
        NodeDims d{m, n, m1, n1, r1, r2, r3, r4};
        const int64_t tot = m + n;
        if (tot <= 16384) {
            hipLaunchKernelGGL(k_node_index_lds, dim3(1), dim3(1024), (size_t)tot * 4, s, d, P, P2, P3, P4, Q, Q2,
                               Q3, Q4);
            FFP_HIP_CHECK(hipGetLastError());
        } else {
            int32_t *Pn = (int32_t *)ws.take((size_t)(m + n) * 4);
            if (!Pn) return FFP_E_WORKSPACE;
            hipLaunchKernelGGL(k_node_index, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, d, P, P2, P3,
                               P4, Q, Q2, Q3, Q4, Pn, Pn + m);
            FFP_HIP_CHECK(hipGetLastError());
            FFP_HIP_CHECK(hipMemcpyAsync(P, Pn, (size_t)m * 4, hipMemcpyDeviceToDevice, s));
            FFP_HIP_CHECK(hipMemcpyAsync(Q, Pn + m, (size_t)n * 4, hipMemcpyDeviceToDevice, s));
        }
    }
    ws.release(mk);
    *rank = r1 + r2 + r3 + r4;
    // the node's rows keep their order when A1 has full row rank (F has no
    // rows) and every sub-block's row order is the identity; columns alike
    *pid = r1 == m1 && p1id && p3id && p4id;
    *qid = r1 == n1 && q1id && q2id && q4id;
    return FFP_OK;
}

// F, G and R of a node: a zero block is factored by its identity permutations
int pluq_sub(Ctx &c, int64_t m, int64_t n, int32_t *A, int64_t lda, int32_t *P, int32_t *Q, int64_t *rank, bool *pid,
             bool *qid) {
    bool zero = false;
    if (m > 0 && n > 0) FFP_CHECK(block_is_zero(c, m, n, A, lda, &zero));
    if (zero) {
        FFP_CHECK(iota(P, m, c.s));
        FFP_CHECK(iota(Q, n, c.s));
        *rank = 0;
        *pid = *qid = true;
        return FFP_OK;
    }
    return pluq_rec(c, m, n, A, lda, P, Q, rank, 0, pid, qid);
}
}  // namespace

// ---------------------------------------------------------------- generic speculation
// When every leading minor of A is nonzero (generic rank profile) the rank
// profile matrix is the diagonal, the quadrant order is the identity and the
// PLUQ decomposition is the LU decomposition without pivoting, P = Q = I:
// every permutation and rotation is the identity and no rank has to be read
// back.  That decomposition is unique, so it may be computed with any block
// split: lu_generic splits off a leading square block whose size is a
// multiple of 64,
//   [A1 B1; C1 A4] = [L1 0; E L3] [U1 D; 0 U3],
//   D = L1^-1 B1,  E = C1 U1^-1,  L3 U3 = A4 - E D,
// so that every diagonal leaf is an aligned 64 x 64 block (the last one may
// be smaller).  Each leaf stores the inverses of its L and U blocks, which
// are exactly the base-case inverses of the later solves with L1 and U1.
// Leaves raise *gflag on the first zero pivot (A is then not generic), and
// the caller restores A and runs the general recursion.  The result, when the flag stays clear, is
// bit-identical to the general one.
namespace {
constexpr int64_t kBlk = 64 * 64;  // doubles per stored block inverse

// D = L1^-1 B1 and E = C1 U1^-1 recurse in step on the caller's stream with
// each pair of base cases in one launch (measured on MI355X: faster at every
// size than two streams joined by events), then H = A4 - E D.
int node_updates_gen(Ctx &c, int64_t m, int64_t n, int64_t h, int32_t *A, int64_t lda, const double *Li,
                     const double *Ui) {
    FFP_CHECK(ftrsm_pair_gen(c.path, *c.F, h, A, lda, n - h, A + h, m - h, A + h * lda, lda, Li, Ui, *c.ws, c.s));
    return fgemm_sub(c, m - h, n - h, h, A + h * lda, lda, A + h, lda, A + h * lda + h, lda);
}

// returned (never to callers of the library) when a checkpoint of the
// generic attempt finds a zero pivot: the rest of the attempt was not enqueued
constexpr int kGenAbort = -1000;

// Li / Ui: block-inverse slots from this block's diagonal offset on
int lu_generic(Ctx &c, int64_t m, int64_t n, int32_t *A, int64_t lda, int *gflag, double *Li, double *Ui,
               int64_t d0) {
    if (m == 0 || n == 0) return FFP_OK;
    if (leaf64_fits(m, n))
        return leaf64_launch(*c.F, m, n, A, lda, nullptr, nullptr, nullptr, gflag, Li, Ui, c.s, nullptr, nullptr,
                             nullptr, 0, nullptr, 0, d0);
    const int64_t k = m < n ? m : n;
    const int64_t h = k <= 64 ? k : 64 * ((k + 127) / 128);
    if (h == 64 && m <= 128 && n <= 128 && c.F->kexact >= 64) {
        // both halves are leaves: the node's two solves run at the end of the
        // first leaf and its update H = A4 - E D at the start of the second
        FFP_CHECK(leaf64_launch(*c.F, 64, 64, A, lda, nullptr, nullptr, nullptr, gflag, Li, Ui, c.s, nullptr,
                                nullptr, A + 64, n - 64, A + 64 * lda, m - 64, d0));
        return leaf64_launch(*c.F, m - 64, n - 64, A + 64 * lda + 64, lda, nullptr, nullptr, nullptr, gflag,
                             Li + kBlk, Ui + kBlk, c.s, A + 64 * lda, A + 64, nullptr, 0, nullptr, 0, d0 + 64);
    }
    FFP_CHECK(lu_generic(c, h, h, A, lda, gflag, Li, Ui, d0));
    // checkpoints on the leading corner, once the leading block of order
    // 1024..2047 and then of order 4096..8191 is factored, where at least
    // three quarters of the attempt remain: one read-back each, and an input
    // that is not generic that far skips the rest
    if (d0 == 0 && c.gen_k >= 4 * h && ((h >= 1024 && h < 2048) || (h >= 4096 && h < 8192))) {
        int64_t f = 0;
        FFP_CHECK(read_flag(c, &f));
        if (f != 0) return kGenAbort;
    }
    FFP_CHECK(node_updates_gen(c, m, n, h, A, lda, Li, Ui));
    const int64_t off = (h / 64) * kBlk;  // h is a multiple of 64 whenever the rest is non-empty
    return lu_generic(c, m - h, n - h, A + h * lda + h, lda, gflag, Li + off, Ui + off, d0 + h);
}
}  // namespace

size_t pluq_ws(int64_t m, int64_t n, const Field &F, int path) {
    // largest out-of-place permutation (the whole block) + index arrays along
    // one root-to-leaf path + the rank word + limb planes of the largest
    // product + the backup copy of A for the generic speculation
    int64_t depth = 2;
    for (int64_t x = (m > n ? m : n); x > 1; x >>= 1) ++depth;
    size_t b = (size_t)m * (size_t)n * 4 + 256;
    b += (size_t)depth * ((size_t)(m + n) * 4 * 3 + 4 * 256);
    b += 512;
    if (path == FFP_PATH_INT8 || path == FFP_PATH_AUTO) b += fgemm_i8_ws(F, m, n, (m < n ? m : n));
    b += (size_t)m * (size_t)n * 4 + 512;
    // inverses of the triangular solves' diagonal blocks (two solves at once),
    // and the leaves' L and U block inverses of the generic attempt
    b += 2 * ((size_t)(((m < n ? m : n) + 63) / 64) + 2) * 64 * 64 * 8 + 4096;
    b += 2 * ((size_t)(((m < n ? m : n) + 63) / 64)) * 64 * 64 * 8 + 1024;
    return b;
}

// Flag words through the pinned host word: one small copy kernel, one
// stream synchronisation.
__global__ void k_flag_to_word(const int *flag, int64_t *word) { *word = *flag; }
int read_flag(const Ctx &c, int64_t *out) {
    hipLaunchKernelGGL(k_flag_to_word, dim3(1), dim3(1), 0, c.s, c.flag_dev, c.rank_dev);
    FFP_HIP_CHECK(hipGetLastError());
    return read_rank(c, out);
}

// The generic attempt on an m x n block (a copy kept to fall back): *ok when
// every pivot was nonzero (A then holds the LU factors, P = Q = identity);
// otherwise A is restored and *k0 receives the order of the first vanishing
// leading minor minus one (all leading minors up to order k0 are nonzero).
int try_generic(Ctx &c, int64_t m, int64_t n, int32_t *A, int64_t lda, bool *ok, int64_t *k0) {
    Arena &ws = *c.ws;
    hipStream_t s = c.s;
    const size_t mk = ws.mark();
    int32_t *backup = (int32_t *)ws.take((size_t)m * (size_t)n * 4);
    const size_t nblk = (size_t)(((m < n ? m : n) + 63) / 64);
    double *Li = (double *)ws.take(nblk * kBlk * sizeof(double));
    double *Ui = (double *)ws.take(nblk * kBlk * sizeof(double));
    if (!backup || !Li || !Ui) return FFP_E_WORKSPACE;
    FFP_CHECK(copy2d(m, n, A, lda, backup, n, s));
    hipLaunchKernelGGL(k_set_int, dim3(1), dim3(1), 0, s, c.flag_dev, 0);
    FFP_HIP_CHECK(hipGetLastError());
    {
        c.gen_k = m < n ? m : n;
        const int rc = lu_generic(c, m, n, A, lda, c.flag_dev, Li, Ui, 0);
        if (rc != FFP_OK && rc != kGenAbort) return rc;
    }
    int64_t flag = 0;
    FFP_CHECK(read_flag(c, &flag));
    *ok = flag == 0;
    *k0 = flag - 1;
    if (!*ok) FFP_CHECK(copy2d(m, n, backup, n, A, lda, s));
    ws.release(mk);
    // leaves only ever write 1 + a diagonal index: anything else is an internal error
    if (flag < 0 || flag > (m < n ? m : n)) {
        FFP_HIP_CHECK(hipStreamSynchronize(s));
        return FFP_E_INTERNAL;
    }
    return FFP_OK;
}

int pluq_run(int path, const Field &F, int64_t m, int64_t n, int32_t *A, int64_t lda, int32_t *P, int32_t *Q,
             int64_t *r, Arena &ws, hipStream_t s) {
    int *flag_dev = (int *)ws.take(256);
    if (!flag_dev) return FFP_E_WORKSPACE;
    RankWord rw;
    FFP_CHECK(rank_word_get(&rw));
    struct WordBack {
        RankWord w;
        ~WordBack() { rank_word_put(w); }
    } word_back{rw};
    Ctx c{path, &F, &ws, s, rw.dev, rw.host, flag_dev};
    int64_t gen_ok = 0;
    if (m > 64 && n > 64 && !getenv("FFP_PLUQ_GENERAL_ONLY")) {
        // speculate that A has generic rank profile
        bool ok = false;
        FFP_CHECK(try_generic(c, m, n, A, lda, &ok, &gen_ok));
        if (ok) {
            FFP_CHECK(iota(P, m, s));
            FFP_CHECK(iota(Q, n, s));
            *r = m < n ? m : n;
            return FFP_OK;
        }
    }
    bool pid = false, qid = false;
    return pluq_rec(c, m, n, A, lda, P, Q, r, gen_ok, &pid, &qid);
}

// Plain LU of an input of generic rank profile, asynchronous (ffp_lu_nopiv):
// the generic attempt without its checkpoints (they read the flag back) and
// without the backup copy; *info = 1 + the first zero pivot's diagonal index.
int lu_nopiv_run(int path, const Field &F, int64_t m, int64_t n, int32_t *A, int64_t lda, int *info, Arena &ws,
                 hipStream_t s) {
    hipLaunchKernelGGL(k_set_int, dim3(1), dim3(1), 0, s, info, 0);
    FFP_HIP_CHECK(hipGetLastError());
    if (m == 0 || n == 0) return FFP_OK;
    const size_t mk = ws.mark();
    const size_t nblk = (size_t)(((m < n ? m : n) + 63) / 64);
    double *Li = (double *)ws.take(nblk * kBlk * sizeof(double));
    double *Ui = (double *)ws.take(nblk * kBlk * sizeof(double));
    if (!Li || !Ui) return FFP_E_WORKSPACE;
    Ctx c{path, &F, &ws, s, nullptr, nullptr, info};
    c.gen_k = 0;
    FFP_CHECK(lu_generic(c, m, n, A, lda, info, Li, Ui, 0));
    ws.release(mk);
    return FFP_OK;
}

// The generic-rank-profile LU of one block at diagonal offset d0 (the base
// case of the tile-iterative variants): a zero pivot sets *info = 1 + its
// index on the whole diagonal unless *info is already set (later leaves then
// return at once).  Asynchronous.
int lu_block_generic(int path, const Field &F, int64_t m, int64_t n, int32_t *A, int64_t lda, int *info, int64_t d0,
                     Arena &ws, hipStream_t s) {
    if (m == 0 || n == 0) return FFP_OK;
    const size_t mk = ws.mark();
    const size_t nblk = (size_t)(((m < n ? m : n) + 63) / 64);
    double *Li = (double *)ws.take(nblk * kBlk * sizeof(double));
    double *Ui = (double *)ws.take(nblk * kBlk * sizeof(double));
    if (!Li || !Ui) return FFP_E_WORKSPACE;
    Ctx c{path, &F, &ws, s, nullptr, nullptr, info};
    c.gen_k = 0;
    FFP_CHECK(lu_generic(c, m, n, A, lda, info, Li, Ui, d0));
    ws.release(mk);
    return FFP_OK;
}

// ffp_check_range: one pass over the block, any entry outside [0, p) stores
// 1 into a pinned host word (all writers store the same value)
__global__ __launch_bounds__(256) void k_range(int64_t m, int64_t n, const int32_t *__restrict__ A, int64_t lda,
                                               int32_t p, int64_t *__restrict__ word) {
    bool bad = false;
    for (int64_t i = blockIdx.x; i < m; i += gridDim.x) {
        const int32_t *row = A + i * lda;
        for (int64_t j = threadIdx.x; j < n; j += 256) bad |= (uint32_t)row[j] >= (uint32_t)p;
    }
    if (__syncthreads_or(bad) && threadIdx.x == 0) *(volatile int64_t *)word = 1;
}

int check_range_run(int64_t m, int64_t n, uint32_t p, const int32_t *A, int64_t lda, hipStream_t s, bool *ok) {
    *ok = true;
    if (m <= 0 || n <= 0) return FFP_OK;
    RankWord rw;
    FFP_CHECK(rank_word_get(&rw));
    struct WordBack {
        RankWord w;
        ~WordBack() { rank_word_put(w); }
    } word_back{rw};
    *(volatile int64_t *)rw.host = 0;
    const unsigned g = (unsigned)(m < 2048 ? m : 2048);
    hipLaunchKernelGGL(k_range, dim3(g), dim3(256), 0, s, m, n, A, lda, (int32_t)p, rw.dev);
    FFP_HIP_CHECK(hipGetLastError());
    FFP_HIP_CHECK(hipStreamSynchronize(s));
    *ok = *(const volatile int64_t *)rw.host == 0;
    return FFP_OK;
}

// ===================================================================== rank profiles
__global__ void k_mark(const int32_t *__restrict__ idx, int64_t r, uint8_t *__restrict__ flag) {
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < r; t += (int64_t)gridDim.x * blockDim.x)
        flag[idx[t]] = 1;
}
__global__ void k_zero8(uint8_t *__restrict__ f, int64_t n) {
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x)
        f[t] = 0;
}
// single workgroup: compact the flagged indices in increasing order
__global__ __launch_bounds__(1024) void k_compact(const uint8_t *__restrict__ flag, int64_t n, int32_t *__restrict__ out) {
    __shared__ int64_t sums[1024];
    const int tid = threadIdx.x;
    const int64_t chunk = (n + 1023) / 1024;
    const int64_t lo = tid * chunk, hi = lo + chunk < n ? lo + chunk : n;
    int64_t cnt = 0;
    for (int64_t i = lo; i < hi; ++i) cnt += flag[i];
    sums[tid] = cnt;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        int64_t v = tid >= off ? sums[tid - off] : 0;
        __syncthreads();
        sums[tid] += v;
        __syncthreads();
    }
    int64_t pos = sums[tid] - cnt;
    for (int64_t i = lo; i < hi; ++i)
        if (flag[i]) out[pos++] = (int32_t)i;
}

int rank_profiles(int64_t m, int64_t n, const int32_t *P, const int32_t *Q, int64_t r, int32_t *rrp, int32_t *crp,
                  Arena &ws, hipStream_t s) {
    if (r <= 0) return FFP_OK;
    const size_t mk = ws.mark();
    uint8_t *fl = (uint8_t *)ws.take((size_t)(m > n ? m : n));
    if (!fl) return FFP_E_WORKSPACE;
    for (int which = 0; which < 2; ++which) {
        int32_t *out = which == 0 ? rrp : crp;
        if (!out) continue;
        const int64_t len = which == 0 ? m : n;
        hipLaunchKernelGGL(k_zero8, dim3((unsigned)std::min<int64_t>((len + 255) / 256, 1024)), dim3(256), 0, s, fl, len);
        hipLaunchKernelGGL(k_mark, dim3((unsigned)std::min<int64_t>((r + 255) / 256, 1024)), dim3(256), 0, s,
                           which == 0 ? P : Q, r, fl);
        hipLaunchKernelGGL(k_compact, dim3(1), dim3(1024), 0, s, fl, len, out);
        FFP_HIP_CHECK(hipGetLastError());
    }
    ws.release(mk);
    return FFP_OK;
}

}  // namespace ffp
