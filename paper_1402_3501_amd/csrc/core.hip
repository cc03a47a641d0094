// Library infrastructure: field constants, workspace arena, HIP error
// reporting, kernel timing, and the memory-bound helper kernels
// (scaling, order-preserving permutations = the laswp of Section 2.1).
#include <mutex>
#include <vector>
#include <cstdio>
#include <cstdlib>

#include "ffp_internal.hpp"
#include "ffp_device.hpp"

namespace ffp {

// ------------------------------------------------------------------ errors
int hip_fail(hipError_t e, const char *what, const char *file, int line) {
    if (getenv("FFP_DEBUG"))
        fprintf(stderr, "ffpluq: %s failed (%s) at %s:%d\n", what, hipGetErrorString(e), file, line);
    return FFP_E_HIP;
}

// ------------------------------------------------------------------ field
static uint64_t powmod(uint64_t b, uint64_t e, uint64_t m) {
    unsigned __int128 r = 1, x = b % m;
    while (e) {
        if (e & 1) r = (r * x) % m;
        x = (x * x) % m;
        e >>= 1;
    }
    return (uint64_t)r;
}

bool is_prime_u32(uint32_t n) {
    if (n < 2) return false;
    for (uint32_t d : {2u, 3u, 5u, 7u, 11u, 13u, 17u, 19u, 23u, 29u, 31u, 37u}) {
        if (n == d) return true;
        if (n % d == 0) return false;
    }
    uint64_t d = n - 1;
    int s = 0;
    while (!(d & 1)) { d >>= 1; ++s; }
    for (uint64_t a : {2ull, 7ull, 61ull}) {
        uint64_t x = powmod(a % n, d, n);
        if (x == 1 || x == n - 1 || a % n == 0) continue;
        bool comp = true;
        for (int i = 1; i < s && comp; ++i) {
            x = (uint64_t)(((unsigned __int128)x * x) % n);
            if (x == n - 1) comp = false;
        }
        if (comp) return false;
    }
    return true;
}

int int8_limbs(uint32_t p) {
    // centred residues |c| <= (p-1)/2 must fit L balanced base-256 digits in [-128, 127]:
    // the largest such magnitude is 127 * (1 + 256 + ... + 256^(L-1))
    const uint64_t h = (p - 1) / 2;
    if (h <= 127ull) return 1;
    if (h <= 127ull * 257ull) return 2;
    if (h <= 127ull * 65793ull) return 3;
    return 0;
}

Field::Field(uint32_t p_) : p(p_) {
    pd = (double)p;
    pinv = 1.0 / pd;
    half = (p - 1) / 2;
    const double two53 = 9007199254740992.0;
    // 2p + k * half^2 < 2^53 keeps every partial sum of centred products exact
    // when it starts from a value reduced to |x| < 2p
    long double h2 = (long double)(half > 0 ? half : 1) * (long double)(half > 0 ? half : 1);
    long double kk = ((long double)two53 - 1.0L - 2.0L * (long double)p) / h2;
    kexact = kk > 4.0e18L ? (int64_t)4e18 : (int64_t)kk;
    if (half == 0) kexact = (int64_t)4e18;  // p = 2: every product is 0 or 1
    limbs = int8_limbs(p);
}

// ------------------------------------------------------------------ arena
void *Arena::take(size_t bytes) {
    size_t b = (bytes + 255) & ~(size_t)255;
    size_t off = used;
    used += b;
    if (used > peak) peak = used;
    if (counting) return nullptr;
    if (used > cap) return nullptr;
    return base + off;
}

// ------------------------------------------------------------------ profiling
namespace {
struct ProfRec {
    int kind;
    double ops, bytes;
    hipEvent_t e0, e1;
};
std::mutex g_prof_mu;
bool g_prof_on = false;
std::vector<ProfRec> g_prof;
std::vector<hipEvent_t> g_pool;  // recycled events (creation is the costly part)
struct ProfTotals {
    int64_t launches = 0;
    double ms = 0.0, ops = 0.0, bytes = 0.0;
} g_tot[kProfKinds];

hipEvent_t pool_get() {
    if (!g_pool.empty()) {
        hipEvent_t e = g_pool.back();
        g_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

void drain_locked() {
    for (auto &r : g_prof) {
        float ms = 0.f;
        (void)hipEventSynchronize(r.e1);
        (void)hipEventElapsedTime(&ms, r.e0, r.e1);
        if (r.kind >= 0 && r.kind < kProfKinds) {
            g_tot[r.kind].launches += 1;
            g_tot[r.kind].ms += ms;
            g_tot[r.kind].ops += r.ops;
            g_tot[r.kind].bytes += r.bytes;
        }
        g_pool.push_back(r.e0);
        g_pool.push_back(r.e1);
    }
    g_prof.clear();
}
}  // namespace

ProfScope::ProfScope(int kind_, double ops_, hipStream_t s_, double bytes_)
    : kind(kind_), ops(ops_), bytes(bytes_), s(s_) {
    if (!g_prof_on) return;
    std::lock_guard<std::mutex> g(g_prof_mu);
    hipEvent_t a = pool_get(), b = pool_get();
    if (!a || !b) {
        if (a) g_pool.push_back(a);
        if (b) g_pool.push_back(b);
        return;
    }
    (void)hipEventRecord(a, s);
    ev0 = a;
    ev1 = b;
}

ProfScope::~ProfScope() {
    if (!ev0) return;
    (void)hipEventRecord((hipEvent_t)ev1, s);
    std::lock_guard<std::mutex> g(g_prof_mu);
    g_prof.push_back({kind, ops, bytes, (hipEvent_t)ev0, (hipEvent_t)ev1});
}

int profile_enable(int on) {
    std::lock_guard<std::mutex> g(g_prof_mu);
    g_prof_on = on != 0;
    return FFP_OK;
}
int profile_reset() {
    std::lock_guard<std::mutex> g(g_prof_mu);
    drain_locked();
    for (auto &t : g_tot) t = ProfTotals();
    return FFP_OK;
}
int profile_read(int kind, int64_t *launches, double *ms, double *ops) {
    std::lock_guard<std::mutex> g(g_prof_mu);
    drain_locked();
    if (kind < 0 || kind >= kProfKinds) return -1;
    if (launches) *launches = g_tot[kind].launches;
    if (ms) *ms = g_tot[kind].ms;
    if (ops) *ops = g_tot[kind].ops;
    return FFP_OK;
}
int profile_read_bytes(int kind, double *bytes) {
    std::lock_guard<std::mutex> g(g_prof_mu);
    drain_locked();
    if (kind < 0 || kind >= kProfKinds) return -1;
    if (bytes) *bytes = g_tot[kind].bytes;
    return FFP_OK;
}
const char *profile_kind_name(int kind) {
    static const char *names[kProfKinds] = {"",
                                            "k_fgemm_f64",
                                            "k_fgemm_i8",
                                            "k_split",
                                            "k_i8_combine",
                                            "k_leaf_gen",
                                            "k_leaf64",
                                            "k_trsm",
                                            "k_permute",
                                            "k_pluq_batched",
                                            "k_winograd_add"};
    return kind > 0 && kind < kProfKinds ? names[kind] : nullptr;
}

// ------------------------------------------------------------------ scaling
__global__ void k_scale(int64_t m, int64_t n, int32_t *B, int64_t ldb, double a, double p, double pinv) {
    const int64_t i = blockIdx.y;
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x)
        B[i * ldb + j] = (int32_t)mod_canon(a * (double)B[i * ldb + j], p, pinv);
}

int scale_mat(const Field &F, int64_t m, int64_t n, uint32_t alpha, int32_t *B, int64_t ldb,
              hipStream_t s) {
    if (m <= 0 || n <= 0 || alpha == 1) return FFP_OK;
    for (int64_t r0 = 0; r0 < m; r0 += 65535) {
        int64_t rows = m - r0 < 65535 ? m - r0 : 65535;
        dim3 grid((unsigned)((n + 255) / 256 < 64 ? (n + 255) / 256 : 64), (unsigned)rows);
        hipLaunchKernelGGL(k_scale, grid, dim3(256), 0, s, rows, n, B + r0 * ldb, ldb, (double)alpha,
                           F.pd, F.pinv);
    }
    FFP_HIP_CHECK(hipGetLastError());
    return FFP_OK;
}

// ------------------------------------------------------------------ permutations
__device__ __forceinline__ int64_t perm_apply(const PermSpec &ps, int64_t d) {
    if (ps.idx) return ps.idx_base + (int64_t)ps.idx[d];
    for (int s = 0; s < ps.seg.nseg; ++s)
        if (d >= ps.seg.dst[s] && d < ps.seg.dst[s] + ps.seg.len[s]) return ps.seg.src[s] + (d - ps.seg.dst[s]);
    return d;
}

// dst[i][j] = src[rp(i)][cp(j)]; grid.y walks rows, block x walks columns
__global__ __launch_bounds__(256) void k_permute(int64_t m, int64_t n, const int32_t *__restrict__ src,
                                                 int64_t lds, int32_t *__restrict__ dst, int64_t ldd,
                                                 PermSpec rp, PermSpec cp, int64_t row0) {
    const int64_t i = row0 + blockIdx.y;
    if (i >= m) return;
    const int64_t si = perm_apply(rp, i);
    const int32_t *srow = src + si * lds;
    int32_t *drow = dst + i * ldd;
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x)
        drow[j] = srow[perm_apply(cp, j)];
}

int permute_copy(int64_t m, int64_t n, const int32_t *src, int64_t lds, int32_t *dst, int64_t ldd,
                 const PermSpec &rp, const PermSpec &cp, hipStream_t s) {
    if (m <= 0 || n <= 0) return FFP_OK;
    unsigned gx = (unsigned)((n + 255) / 256);
    if (gx > 16) gx = 16;
    ProfScope prof(PK_PERMUTE, 0.0, s, 8.0 * (double)m * (double)n);
    for (int64_t r0 = 0; r0 < m; r0 += 65535) {
        int64_t rows = m - r0 < 65535 ? m - r0 : 65535;
        hipLaunchKernelGGL(k_permute, dim3(gx, (unsigned)rows), dim3(256), 0, s, m, n, src, lds, dst, ldd,
                           rp, cp, r0);
    }
    FFP_HIP_CHECK(hipGetLastError());
    return FFP_OK;
}

int copy2d(int64_t m, int64_t n, const int32_t *src, int64_t lds, int32_t *dst, int64_t ldd,
           hipStream_t s) {
    if (m <= 0 || n <= 0) return FFP_OK;
    FFP_HIP_CHECK(hipMemcpy2DAsync(dst, (size_t)ldd * 4, src, (size_t)lds * 4, (size_t)n * 4, (size_t)m,
                                   hipMemcpyDeviceToDevice, s));
    return FFP_OK;
}

// Small blocks in place through LDS, one workgroup: every source entry is
// read before any is written, so one launch replaces the gather and the copy
// back (the recursion permutes many small blocks).
constexpr int64_t kPermLds = 16384;  // entries (64 KiB of LDS)

__global__ __launch_bounds__(1024) void k_permute_lds(int64_t m, int64_t n, int32_t *__restrict__ A, int64_t lda,
                                                      PermSpec rp, PermSpec cp) {
    extern __shared__ int32_t pbuf[];
    const int64_t tot = m * n;
    for (int64_t e = threadIdx.x; e < tot; e += blockDim.x) {
        const int64_t i = e / n, j = e % n;
        pbuf[e] = A[perm_apply(rp, i) * lda + perm_apply(cp, j)];
    }
    __syncthreads();
    for (int64_t e = threadIdx.x; e < tot; e += blockDim.x) A[(e / n) * lda + e % n] = pbuf[e];
}

int permute_inplace(int64_t m, int64_t n, int32_t *A, int64_t lda, const PermSpec &rp,
                    const PermSpec &cp, Arena &ws, hipStream_t s) {
    if (m <= 0 || n <= 0 || (rp.identity() && cp.identity())) return FFP_OK;
    if (m * n <= kPermLds) {
        if (ws.counting) return FFP_OK;
        ProfScope prof(PK_PERMUTE, 0.0, s, 8.0 * (double)m * (double)n);
        hipLaunchKernelGGL(k_permute_lds, dim3(1), dim3(1024), (size_t)(m * n) * 4, s, m, n, A, lda, rp, cp);
        FFP_HIP_CHECK(hipGetLastError());
        return FFP_OK;
    }
    const size_t mk = ws.mark();
    int32_t *tmp = (int32_t *)ws.take((size_t)m * (size_t)n * 4);
    if (ws.counting) { ws.release(mk); return FFP_OK; }
    if (!tmp) return FFP_E_WORKSPACE;
    FFP_CHECK(permute_copy(m, n, A, lda, tmp, n, rp, cp, s));
    FFP_CHECK(copy2d(m, n, tmp, n, A, lda, s));
    ws.release(mk);
    return FFP_OK;
}

}  // namespace ffp
