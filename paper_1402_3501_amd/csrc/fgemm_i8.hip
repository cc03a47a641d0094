// fgemm over Z/pZ on the INT8 matrix cores of gfx950 (v_mfma_i32_16x16x64_i8).
//
// The delayed reduction of Section 3.1, carried to 8-bit integers: a
// canonical residue r is centred (c = r or r - p, |c| <= (p-1)/2) and written
// in L balanced base-256 digits c = sum_i 256^i c_i with c_i in [-128, 127]
// (L = 1 for p <= 255, 3 up to p = 16711421).  Then
//     sum_k a_k b_k = sum_s 256^s S_s,   S_s = sum_{i+j=s} sum_k a_{k,i} b_{k,j},
// and every S_s is an exact int32 sum of 8-bit products while
// k * (products per class) * 2^14 < 2^31.  The L^2 digit products run on the
// INT8 matrix cores with one int32 accumulator per shift class s; the
// epilogue reduces each S_s, recombines with 256^s mod p, and applies alpha,
// beta and the store.  Inner dimensions beyond the int32 bound are processed
// in chunks, each ending in a reduction (beta = 1 for the later chunks).
//
// Data path: a split kernel writes the digits of op(A) and op(B) into
// zero-padded planes [digit][row][k] (k contiguous, so that each lane's
// 16-byte MFMA operand is one contiguous load); the product kernel computes
// a 128 x 128 block of C per workgroup, streaming 64-deep K tiles of all L
// digit planes of both operands into LDS with the direct global-to-LDS loads
// (three buffers, each tile requested two tiles ahead) and from there into 8
// wave64s, each owning a 32 x 64 sub-block; products too small to fill the
// chip with such blocks take 64 x 64 blocks of 4 waves, and one-limb products
// large enough take 256 x 256 blocks of 8 waves (64 x 128 each).  Products with too few output blocks to
// fill the chip split K over several workgroups per block (each writes its
// reduced partial result, a second kernel sums them mod p and applies alpha
// and beta).
#include "ffp_internal.hpp"
#include "ffp_device.hpp"

namespace ffp {

typedef int v4i __attribute__((ext_vector_type(4)));

constexpr int kI8BM = 128, kI8BN = 128, kI8BK = 64;
constexpr int kI8Threads = 512;
// products whose grid of 128 x 128 blocks would not fill the chip run on
// 64 x 64 blocks of four waves (two workgroups per compute unit)
constexpr int kI8SmallB = 64, kI8SmallThreads = 256;
// one limb (one accumulator set) leaves the registers for 256 x 256 blocks of
// eight waves with 64 x 128 wave tiles: four times the products per barrier
constexpr int kI8WideB = 256;
// split-K: at most 4 parts, partial results at most 32 MiB
constexpr int kI8MaxSplit = 4;
constexpr int64_t kI8SplitBytes = (int64_t)32 << 20;

static inline int64_t rup(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

// ------------------------------------------------------------------ split
// dst[d][r][kk] = digit d of centre(src(r, kk)), src(r, kk) = X[r*sr + kk*sk],
// zero outside rows < R, kk < K.  Tile 64 x 64 through LDS so that both the
// read (along the stored contiguous dimension) and the write (along kk) are
// coalesced.
// one operand to split: rows of length K (row stride sr, element stride sk)
struct SplitSrc {
    const int32_t *X;
    int64_t sr, sk, R, plane;
    int8_t *dst;
};

// The operands of one product, or of two with the same K, in one launch:
// operand i takes the row tiles [end[i - 1], end[i]) of the grid (end[-1] = 0).
struct SplitSet {
    SplitSrc src[4];
    int64_t end[4];
};
template <int L>
__global__ __launch_bounds__(256) void k_split(SplitSet set, int64_t K, int64_t Kp, int32_t half, int32_t p) {
    const int64_t by = blockIdx.y;
    const int i = by < set.end[0] ? 0 : (by < set.end[1] ? 1 : (by < set.end[2] ? 2 : 3));
    const SplitSrc &sc = set.src[i];
    const int32_t *__restrict__ X = sc.X;
    const int64_t sr = sc.sr, sk = sc.sk, R = sc.R, plane = sc.plane;
    int8_t *__restrict__ dst = sc.dst;
    __shared__ int32_t tile[64][65];
    const int tid = threadIdx.x;
    const int64_t r0 = (by - (i > 0 ? set.end[i - 1] : 0)) * 64, k0 = (int64_t)blockIdx.x * 64;
    const bool along_k = sk == 1;
    // unconditional loads (addresses clamped into the operand) so that all 16
    // are in flight together; out-of-range elements are zeroed afterwards
    int32_t v[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        const int idx = tid + e * 256;
        const int a = idx & 63, b = idx >> 6;   // a runs along the contiguous source dimension
        const int rr = along_k ? b : a, kk = along_k ? a : b;
        const int64_t gr = r0 + rr, gk = k0 + kk;
        v[e] = X[(gr < R ? gr : R - 1) * sr + (gk < K ? gk : K - 1) * sk];
    }
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        const int idx = tid + e * 256;
        const int a = idx & 63, b = idx >> 6;
        const int rr = along_k ? b : a, kk = along_k ? a : b;
        const bool in = r0 + rr < R && k0 + kk < K;
        const int32_t c = v[e] > half ? v[e] - p : v[e];  // centred
        tile[rr][kk] = in ? c : 0;
    }
    __syncthreads();
    // 64 rows x 16 words (4 digits of consecutive kk per word) per digit plane
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int idx = tid + e * 256;
        const int w = idx & 15, rr = idx >> 4;
        uint32_t packed[L];
#pragma unroll
        for (int d = 0; d < L; ++d) packed[d] = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            int32_t c = tile[rr][w * 4 + q];
#pragma unroll
            for (int d = 0; d < L; ++d) {
                const int32_t dig = (d == L - 1) ? c : (((c + 128) & 255) - 128);
                packed[d] |= ((uint32_t)(dig & 255)) << (8 * q);
                c = (c - dig) >> 8;
            }
        }
        const int64_t gr = r0 + rr;
        uint32_t *out = (uint32_t *)(dst + gr * Kp + k0) + w;
#pragma unroll
        for (int d = 0; d < L; ++d) out[(int64_t)d * (plane >> 2)] = packed[d];
    }
}

// ------------------------------------------------------------------ product
// epilogue: lane l holds rows 4*(l/16)+v, column l%16 of each 16x16 block
// of the wave tile at (r0, c0).  The shift classes S_s (|S_s| < 2^31) are
// recombined by Horner's rule, t = (..(S_{NS-1} 256 + S_{NS-2}) 256 ..) + S_0,
// exact in doubles with one reduction after the third class when there are
// five (2^31 256^2 < 2^48 before it, (p/2 + p) 256^2 + 2^31 256 < 2^48 after
// it), then reduced; alpha = p - 1 (the C - A B of the factorisations) is a
// negation; then beta and the store (or the partial result of K part z)
template <int NS, int FM, int FN>
__device__ __forceinline__ void i8_epilogue(const v4i (&acc)[NS][FM][FN], int64_t r0, int64_t c0, int lane, int64_t m,
                                            int64_t n, int32_t *__restrict__ C, int64_t ldc, double p, double pinv,
                                            double alpha, double beta, int z, int32_t *__restrict__ part) {
    const bool negate = alpha == p - 1.0;
#pragma unroll
    for (int i = 0; i < FM; ++i) {
#pragma unroll
        for (int j = 0; j < FN; ++j) {
            const int64_t gj = c0 + j * 16 + (lane & 15);
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int64_t gi = r0 + i * 16 + (lane >> 4) * 4 + v;
                if (gi < m && gj < n) {
                    double t = (double)acc[NS - 1][i][j][v];
#pragma unroll
                    for (int s = NS - 2; s >= 0; --s) {
                        t = fma(t, 256.0, (double)acc[s][i][j][v]);
                        if (NS == 5 && s == 2) t = mod_near(t, p, pinv);
                    }
                    double rres = mod_canon(t, p, pinv);
                    if (part) {
                        part[((int64_t)z * m + gi) * n + gj] = (int32_t)rres;
                        continue;
                    }
                    if (negate && beta == 1.0) {
                        // C - A B: both terms canonical, one correction
                        const double r = (double)C[gi * ldc + gj] - rres;
                        C[gi * ldc + gj] = (int32_t)(r < 0.0 ? r + p : r);
                        continue;
                    }
                    if (negate) rres = rres == 0.0 ? 0.0 : p - rres;
                    else if (alpha != 1.0) rres = mod_canon(alpha * rres, p, pinv);
                    if (beta != 0.0) {
                        double c = (double)C[gi * ldc + gj];
                        if (beta != 1.0) c = mod_canon(beta * c, p, pinv);
                        rres += c;
                        if (rres >= p) rres -= p;
                    }
                    C[gi * ldc + gj] = (int32_t)rres;
                }
            }
        }
    }
}

// One wave-wide direct load: lane l's 16 bytes at base + off (base
// wave-uniform, off this lane's byte offset) go to LDS byte lds + 16 l.
// Written as an instruction here (the builtin makes the compiler wait for
// every such load before any later LDS read, which would serialise the
// buffers): it has no result register, its LDS writes are covered by the
// hand-counted waits of the caller, and the memory clobber keeps the
// compiler's own LDS accesses on their side of it.  The compiler reserves
// m0 (it warns about the clobber): none of the code it emits for these
// kernels reads m0, so the value written here is never one it relies on.
__device__ __forceinline__ void lds_load16(const int8_t *base, uint32_t off, uint32_t lds) {
    asm volatile("s_mov_b32 m0, %2\n\tglobal_load_lds_dwordx4 %0, %1"
                 :
                 : "v"(off), "s"(base), "s"(lds)
                 : "memory", "m0");
}
// LDS byte address of a shared object
template <typename T>
__device__ __forceinline__ uint32_t lds_addr(T &x) {
    return __builtin_amdgcn_readfirstlane((uint32_t)(uintptr_t)(__attribute__((address_space(3))) char *)&x);
}

// The product: a BM x BN block of C per workgroup of NT threads, wave tiles
// of WM rows.  The K tiles come into LDS by the direct loads of gfx950
// (global_load_lds_dwordx4: one wave instruction writes 64 consecutive
// 16-byte chunks, 1 KiB = 16 rows of 64 bytes), three buffers deep: tile
// t + 2 is requested in the step of tile t, right after its first fragment
// reads, so every tile's loads have two tiles' products to arrive, and no
// registers stage them.  Rows are unpadded; chunk q of tile row r sits at
// position q ^ ((r / 4) % 4), so that each 16-lane group of a fragment read
// (16 rows, one chunk) covers all 64 banks once.  The wait before each
// barrier counts this wave's loads: at most one tile's (the next) may still
// be in flight.
// One grid may run two products of the same K (the two panel products of a
// generic node's solves): workgroups [0, g0) take P0, the rest P1.
struct I8Prod {
    const int8_t *A, *B;  // limb planes
    int64_t planeA, planeB, m, n;
    int32_t *C;
    int64_t ldc;
    int ntx, nty;  // output blocks
};
template <int L, int BM, int BN, int NT, int WM>
__global__ __launch_bounds__(NT) void k_fgemm_i8(I8Prod P0, I8Prod P1, int g0, int64_t Kp, double p, double pinv,
                                                 double alpha, double beta, int64_t kt_per,
                                                 int32_t *__restrict__ part) {
    constexpr int BK = 64;
    constexpr int NS = 2 * L - 1;
    constexpr int NW = NT / 64;
    constexpr int WGM = BM / WM, WGN = NW / WGM, WN = BN / WGN;
    static_assert(WGM * WGN == NW && WN % 16 == 0, "wave grid covers the block");
    constexpr int FM = WM / 16, FN = WN / 16;
    // 16-row chunks of a tile per operand, and per wave
    constexpr int CHA = L * BM / 16, CHB = L * BN / 16;
    static_assert(CHA % NW == 0 && CHB % NW == 0, "every wave loads the same number of chunks");
    constexpr int PWA = CHA / NW, PWB = CHB / NW, CHW = PWA + PWB;
    static_assert(CHW <= 63, "wait count");
    typedef int8_t TileA[L][BM][BK];
    typedef int8_t TileB[L][BN][BK];
    // the three buffers of each operand
    __shared__ __attribute__((aligned(1024))) TileA A0, A1, A2;
    __shared__ __attribute__((aligned(1024))) TileB B0, B1, B2;

    const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wm0 = (wave / WGN) * WM, wn0 = (wave % WGN) * WN;
    const bool second = (int)blockIdx.x >= g0;
    const int bid = second ? (int)blockIdx.x - g0 : (int)blockIdx.x;
    const int8_t *__restrict__ Ad = second ? P1.A : P0.A;
    const int8_t *__restrict__ Bd = second ? P1.B : P0.B;
    const int64_t planeA = second ? P1.planeA : P0.planeA, planeB = second ? P1.planeB : P0.planeB;
    const int64_t m = second ? P1.m : P0.m, n = second ? P1.n : P0.n, ldc = second ? P1.ldc : P0.ldc;
    int32_t *__restrict__ C = second ? P1.C : P0.C;
    const int ntx = second ? P1.ntx : P0.ntx, nty = second ? P1.nty : P0.nty;
    // part != nullptr (one product only): workgroup b computes K tiles
    // [kt_per z, kt_per (z + 1)) of output block b % (ntx nty), z = b / (ntx nty), into part[z] (m x n)
    const int tiles = ntx * nty;
    const int z = part ? bid / tiles : 0;
    int ty, tx;
    xcd_tile(part ? bid % tiles : bid, ntx, nty, ty, tx);
    const int64_t m0 = (int64_t)ty * BM, n0 = (int64_t)tx * BN;
    const int64_t t0 = part ? kt_per * z : 0;
    const int64_t nt = part ? ((Kp / BK - t0) < kt_per ? Kp / BK - t0 : kt_per) : Kp / BK;

    // lane -> (row lane / 4 of a 16-row chunk, position lane % 4): it loads
    // the global 16 bytes that belong at that position; the same byte
    // offset serves both operands (rows of Kp bytes)
    const int crow = lane >> 2, cq = (lane & 3) ^ ((crow >> 2) & 3);
    const uint32_t voff = (uint32_t)(crow * Kp + 16 * cq);
    const uint32_t la[3] = {lds_addr(A0), lds_addr(A1), lds_addr(A2)};
    const uint32_t lb[3] = {lds_addr(B0), lds_addr(B1), lds_addr(B2)};
    // K tile t into buffer q (t clamped to the last tile: every step issues
    // the same number of loads, so the wait counts hold; a clamped load only
    // refills a buffer that is not read again)
    auto issue = [&](int64_t t, int q) {
        const int64_t k0 = (t0 + (t < nt ? t : nt - 1)) * BK;
#pragma unroll
        for (int e = 0; e < PWA; ++e) {
            const int c = wave + NW * e;  // wave-uniform
            const int d = c / (BM / 16), rb = (c % (BM / 16)) * 16;
            lds_load16(Ad + d * planeA + (m0 + rb) * Kp + k0, voff, la[q] + (uint32_t)((d * BM + rb) * BK));
        }
#pragma unroll
        for (int e = 0; e < PWB; ++e) {
            const int c = wave + NW * e;
            const int d = c / (BN / 16), rb = (c % (BN / 16)) * 16;
            lds_load16(Bd + d * planeB + (n0 + rb) * Kp + k0, voff, lb[q] + (uint32_t)((d * BN + rb) * BK));
        }
    };

    v4i acc[NS][FM][FN];
#pragma unroll
    for (int s = 0; s < NS; ++s)
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int j = 0; j < FN; ++j) acc[s][i][j] = v4i{0, 0, 0, 0};

    // fragment reads: lane reads row r = lane % 16 of its 16-row block, the
    // 16 bytes of reduction chunk lane / 16 (rows start at multiples of 16)
    const int r = lane & 15, fpos = 16 * ((lane >> 4) ^ ((r >> 2) & 3));
    // vmcnt(n), expcnt and lgkmcnt left alone
    constexpr int kWaitNext = (CHW & 15) | ((CHW >> 4) << 14) | (0x7 << 4) | (0xF << 8);
    // step on tile t in buffer (Ac, Bc); the loads of tile t + 2 go to buffer qn
    auto step = [&](int64_t t, const TileA &Ac, const TileB &Bc, int qn) {
        __builtin_amdgcn_s_waitcnt(kWaitNext);  // tile t is in (this wave's part)
        __builtin_amdgcn_s_barrier();           // every wave's part; every read of buffer qn is done
        asm volatile("" ::: "memory");
        v4i a[L][FM];
#pragma unroll
        for (int d = 0; d < L; ++d)
#pragma unroll
            for (int i = 0; i < FM; ++i) a[d][i] = *(const v4i *)&Ac[d][wm0 + i * 16 + r][fpos];
#pragma unroll
        for (int db = 0; db < L; ++db) {
            v4i b[FN];
#pragma unroll
            for (int j = 0; j < FN; ++j) b[j] = *(const v4i *)&Bc[db][wn0 + j * 16 + r][fpos];
            if (db == 0) issue(t + 2, qn);  // after the first fragment reads are on their way
#pragma unroll
            for (int da = 0; da < L; ++da)
#pragma unroll
                for (int i = 0; i < FM; ++i)
#pragma unroll
                    for (int j = 0; j < FN; ++j)
                        acc[da + db][i][j] =
                            __builtin_amdgcn_mfma_i32_16x16x64_i8(a[da][i], b[j], acc[da + db][i][j], 0, 0, 0);
        }
    };
    issue(0, 0);
    issue(1, 1);
    for (int64_t t = 0; t < nt; t += 3) {
        step(t, A0, B0, 2);
        if (t + 1 < nt) step(t + 1, A1, B1, 0);
        if (t + 2 < nt) step(t + 2, A2, B2, 1);
    }
    // no load may still write the LDS when the workgroup ends
    __builtin_amdgcn_s_waitcnt((0x7 << 4) | (0xF << 8));
    i8_epilogue<NS, FM, FN>(acc, m0 + wm0, n0 + wn0, lane, m, n, C, ldc, p, pinv, alpha, beta, z, part);
}

// C <- alpha * (sum of the nz partial results) + beta * C, all mod p (each
// partial is canonical, the sum of at most kI8MaxSplit of them is exact);
// row gi = blockIdx.y (only products of at most 65535 rows are split)
__global__ __launch_bounds__(256) void k_i8_combine(int64_t m, int64_t n, int nz, const int32_t *__restrict__ part,
                                                    int32_t *__restrict__ C, int64_t ldc, double p, double pinv,
                                                    double alpha, double beta) {
    const int64_t gi = blockIdx.y, gj = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (gj >= n) return;
    const int64_t idx = gi * n + gj;
    double t = 0.0;
    for (int zz = 0; zz < nz; ++zz) t += (double)part[(int64_t)zz * m * n + idx];
    double rres = mod_canon(t, p, pinv);
    if (alpha != 1.0) rres = mod_canon(alpha * rres, p, pinv);
    if (beta != 0.0) {
        double c = (double)C[gi * ldc + gj];
        if (beta != 1.0) c = mod_canon(beta * c, p, pinv);
        rres += c;
        if (rres >= p) rres -= p;
    }
    C[gi * ldc + gj] = (int32_t)rres;
}

// ------------------------------------------------------------------ host side
static int64_t kchunk_for(int L) { return L == 1 ? 131072 : (L == 2 ? 65536 : 32768); }

// rows of the limb planes: zero-padded to whole blocks of the largest tile
static int64_t plane_rows(int L, int64_t r) { return rup(r, L == 1 ? kI8WideB : kI8BM); }
// and columns: zero-padded to whole K tiles
static int64_t plane_k(int) { return kI8BK; }

size_t fgemm_i8_ws(const Field &F, int64_t m, int64_t n, int64_t k) {
    const int L = F.limbs > 0 ? F.limbs : 3;
    const int64_t kc = k < kchunk_for(L) ? k : kchunk_for(L);
    const int64_t Kp = rup(kc > 0 ? kc : 1, plane_k(L));
    return (size_t)L * (size_t)(plane_rows(L, m) + plane_rows(L, n)) * (size_t)Kp + 1024;
}

// The split-K partial results are optional workspace: a product splits K
// only when the arena still has room for them after the limb planes (the
// workspace sizes of the factorisations leave it), otherwise it runs
// unsplit.  A caller that wants the split for a lone product adds this.
size_t fgemm_i8_split_ws(int64_t m, int64_t n) {
    const int64_t b = (int64_t)kI8MaxSplit * rup(m, kI8BM) * rup(n, kI8BN) * 4;
    return (size_t)(b < kI8SplitBytes ? b : kI8SplitBytes) + 256;
}

// K parts for a product of `tiles` output blocks and nt K tiles: enough to
// bring the grid to the chip's 256 compute units, each part at least 4 K
// tiles, the partial results within kI8SplitBytes
static int i8_split(int64_t tiles, int64_t nt, int64_t m, int64_t n) {
    int z = 1;
    if (m > 65535) return 1;  // the combining pass runs one grid row per output row
    while (z < kI8MaxSplit && tiles * z * 2 <= 256 && nt / (z * 2) >= 4 && (int64_t)(z * 2) * m * n * 4 <= kI8SplitBytes)
        z *= 2;
    return z;
}

// One product C = alpha op(A) op(B) + beta C of a run (op as ta / tb).
struct I8Call {
    int64_t m, n;
    const int32_t *A;
    int64_t lda;
    const int32_t *B;
    int64_t ldb;
    int32_t *C;
    int64_t ldc;
};

// nc = 1 or 2 products of the same k, alpha, beta and transposes: their limb
// splits share one launch and their products one grid (two products never
// split K).
template <int L>
static int run_i8(const Field &F, int ta, int tb, int64_t k, uint32_t alpha, uint32_t beta, const I8Call *cs,
                  int nc, Arena &ws, hipStream_t s) {
    const int64_t KC = kchunk_for(L);
    int64_t Mp[2], Np[2];
    for (int i = 0; i < nc; ++i) {
        Mp[i] = plane_rows(L, cs[i].m);
        Np[i] = plane_rows(L, cs[i].n);
    }
    // output blocks: 128 x 128 when they fill the chip's 256 compute units,
    // else 64 x 64 (measured on MI355X: 1024^3 with three limbs 31 us against
    // 36 us, the 16384 factorisation 34.3 against 35.0 ms); one limb takes
    // 256 x 256 blocks whenever they fill the chip
    int64_t t256 = 0, t128 = 0;
    for (int i = 0; i < nc; ++i) {
        t256 += (rup(cs[i].n, kI8WideB) / kI8WideB) * (rup(cs[i].m, kI8WideB) / kI8WideB);
        t128 += (rup(cs[i].n, kI8BN) / kI8BN) * (rup(cs[i].m, kI8BM) / kI8BM);
    }
    const bool wide = L == 1 && t256 >= 256;
    const bool small = !wide && t128 < 256;
    const int bs = wide ? kI8WideB : (small ? kI8SmallB : kI8BM);
    for (int64_t kc0 = 0; kc0 < k; kc0 += KC) {
        const int64_t kc = k - kc0 < KC ? k - kc0 : KC;
        const int64_t Kp = rup(kc, plane_k(L));
        const size_t mk = ws.mark();
        SplitSet set;
        I8Prod P[2];
        int64_t rows = 0;
        double split_bytes = 0.0, ops = 0.0, prod_bytes = 0.0;
        for (int i = 0; i < nc; ++i) {
            const I8Call &c = cs[i];
            const int64_t planeA = Mp[i] * Kp, planeB = Np[i] * Kp;
            int8_t *Ad = (int8_t *)ws.take((size_t)L * planeA);
            int8_t *Bd = (int8_t *)ws.take((size_t)L * planeB);
            if (!Ad || !Bd) return FFP_E_WORKSPACE;
            // op(A)[i][kk] and op(B)[kk][j] as (row, k) accessors
            const int32_t *Ab = ta ? c.A + kc0 * c.lda : c.A + kc0;
            const int32_t *Bb = tb ? c.B + kc0 : c.B + kc0 * c.ldb;
            const int64_t asr = ta ? 1 : c.lda, ask = ta ? c.lda : 1;
            const int64_t bsr = tb ? c.ldb : 1, bsk = tb ? 1 : c.ldb;
            set.src[2 * i] = SplitSrc{Ab, asr, ask, c.m, planeA, Ad};
            set.src[2 * i + 1] = SplitSrc{Bb, bsr, bsk, c.n, planeB, Bd};
            set.end[2 * i] = (rows += Mp[i] / 64);
            set.end[2 * i + 1] = (rows += Np[i] / 64);
            split_bytes += 4.0 * (double)kc * (double)(c.m + c.n) + (double)L * (double)Kp * (double)(Mp[i] + Np[i]);
            P[i] = I8Prod{Ad, Bd, planeA, planeB, c.m, c.n, c.C, c.ldc, (int)(rup(c.n, bs) / bs),
                          (int)(rup(c.m, bs) / bs)};
        }
        for (int j = 2 * nc; j < 4; ++j) {
            set.src[j] = set.src[2 * nc - 1];
            set.end[j] = rows;
        }
        {
            ProfScope prof(PK_I8_SPLIT, 0.0, s, split_bytes);
            hipLaunchKernelGGL((k_split<L>), dim3((unsigned)(Kp / 64), (unsigned)rows), dim3(256), 0, s, set, kc, Kp,
                               (int32_t)F.half, (int32_t)F.p);
        }
        const double be = kc0 == 0 ? (double)beta : 1.0;
        const int64_t nt = Kp / kI8BK;
        const int64_t m0 = cs[0].m, n0 = cs[0].n;
        int nz = nc == 1 ? i8_split((int64_t)P[0].ntx * P[0].nty, nt, m0, n0) : 1;
        int64_t kt_per = (nt + nz - 1) / nz;
        nz = (int)((nt + kt_per - 1) / kt_per);  // every part non-empty
        // optional: without room for the partial results the product runs unsplit
        int32_t *part = nullptr;
        if (nz > 1) {
            const size_t bytes = (size_t)nz * (size_t)m0 * (size_t)n0 * 4;
            if (ws.used + bytes + 256 <= ws.cap) part = (int32_t *)ws.take(bytes);
        }
        if (!part) {
            nz = 1;
            kt_per = nt;
        }
        // algorithmic bytes: the limb planes read once, the result written
        // once (and C read once when beta != 0)
        for (int i = 0; i < nc; ++i) {
            const double m = (double)cs[i].m, n = (double)cs[i].n;
            ops += 2.0 * m * n * (double)kc;
            prod_bytes += (double)L * (m + n) * (double)kc + 4.0 * (part ? (double)nz : (be != 0.0 ? 2.0 : 1.0)) * m * n;
        }
        const int g0 = P[0].ntx * P[0].nty * nz;
        const int grid = g0 + (nc == 2 ? P[1].ntx * P[1].nty : 0);
        const I8Prod &P1 = P[nc - 1];
        {
            ProfScope prof(PK_FGEMM_I8, ops, s, prod_bytes);
            if constexpr (L == 1) {
                if (wide)
                    hipLaunchKernelGGL((k_fgemm_i8<1, kI8WideB, kI8WideB, kI8Threads, 64>), dim3((unsigned)grid),
                                       dim3(kI8Threads), 0, s, P[0], P1, g0, Kp, F.pd, F.pinv, (double)alpha, be,
                                       kt_per, part);
            }
            if (wide) {
            } else if (small)
                hipLaunchKernelGGL((k_fgemm_i8<L, kI8SmallB, kI8SmallB, kI8SmallThreads, 32>), dim3((unsigned)grid),
                                   dim3(kI8SmallThreads), 0, s, P[0], P1, g0, Kp, F.pd, F.pinv, (double)alpha, be,
                                   kt_per, part);
            else
                hipLaunchKernelGGL((k_fgemm_i8<L, kI8BM, kI8BN, kI8Threads, 32>), dim3((unsigned)grid),
                                   dim3(kI8Threads), 0, s, P[0], P1, g0, Kp, F.pd, F.pinv, (double)alpha, be,
                                   kt_per, part);
        }
        if (part) {
            ProfScope prof(PK_I8_COMBINE, 0.0, s, 4.0 * ((double)nz + (be != 0.0 ? 2.0 : 1.0)) * (double)m0 * (double)n0);
            hipLaunchKernelGGL(k_i8_combine, dim3((unsigned)((n0 + 255) / 256), (unsigned)m0), dim3(256), 0, s, m0,
                               n0, nz, part, cs[0].C, cs[0].ldc, F.pd, F.pinv, (double)alpha, be);
        }
        FFP_HIP_CHECK(hipGetLastError());
        ws.release(mk);
    }
    return FFP_OK;
}

static int run_i8_any(const Field &F, int ta, int tb, int64_t k, uint32_t alpha, uint32_t beta, const I8Call *cs,
                      int nc, Arena &ws, hipStream_t s) {
    switch (F.limbs) {
        case 1: return run_i8<1>(F, ta, tb, k, alpha, beta, cs, nc, ws, s);
        case 2: return run_i8<2>(F, ta, tb, k, alpha, beta, cs, nc, ws, s);
        case 3: return run_i8<3>(F, ta, tb, k, alpha, beta, cs, nc, ws, s);
        default: return FFP_E_P_RANGE;
    }
}

int fgemm_i8(const Field &F, int ta, int tb, int64_t m, int64_t n, int64_t k, uint32_t alpha,
             const int32_t *A, int64_t lda, const int32_t *B, int64_t ldb, uint32_t beta, int32_t *C,
             int64_t ldc, Arena &ws, hipStream_t s) {
    if (m <= 0 || n <= 0) return FFP_OK;
    if (k <= 0) return fgemm_f64(F, ta, tb, m, n, 0, alpha, A, lda, B, ldb, beta, C, ldc, s);
    const I8Call c{m, n, A, lda, B, ldb, C, ldc};
    return run_i8_any(F, ta, tb, k, alpha, beta, &c, 1, ws, s);
}

// Two independent products C_i = alpha A_i B_i + beta C_i of the same k
// (no transposes) in one limb-split launch and one product grid, when both
// are small enough for the split's grid and k for one chunk; otherwise one
// after the other.
int fgemm_i8_pair(const Field &F, int64_t k, uint32_t alpha, uint32_t beta, int64_t m0, int64_t n0,
                  const int32_t *A0, int64_t lda0, const int32_t *B0, int64_t ldb0, int32_t *C0, int64_t ldc0,
                  int64_t m1, int64_t n1, const int32_t *A1, int64_t lda1, const int32_t *B1, int64_t ldb1, int32_t *C1,
                  int64_t ldc1, Arena &ws, hipStream_t s) {
    const int L = F.limbs;
    if (ws.counting) {
        ws.take(fgemm_i8_ws(F, m0, n0, k));
        ws.take(fgemm_i8_ws(F, m1, n1, k));
        return FFP_OK;
    }
    const int64_t rows = (plane_rows(L, m0) + plane_rows(L, n0) + plane_rows(L, m1) + plane_rows(L, n1)) / 64;
    if (m0 <= 0 || n0 <= 0 || m1 <= 0 || n1 <= 0 || k <= 0 || k > kchunk_for(L) || rows > 65535) {
        FFP_CHECK(fgemm_any(FFP_PATH_INT8, F, 0, 0, m0, n0, k, alpha, A0, lda0, B0, ldb0, beta, C0, ldc0, ws, s));
        return fgemm_any(FFP_PATH_INT8, F, 0, 0, m1, n1, k, alpha, A1, lda1, B1, ldb1, beta, C1, ldc1, ws, s);
    }
    const I8Call cs[2] = {{m0, n0, A0, lda0, B0, ldb0, C0, ldc0}, {m1, n1, A1, lda1, B1, ldb1, C1, ldc1}};
    return run_i8_any(F, 0, 0, k, alpha, beta, cs, 2, ws, s);
}

}  // namespace ffp
