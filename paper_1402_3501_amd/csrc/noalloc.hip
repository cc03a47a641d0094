// Allocation-free fgemm: the product of ffp_fgemm with its workspace taken
// from a fixed device array that the library owns, for callers that cannot
// allocate device memory (code under graph capture, serving loops, hosts
// that forbid allocation).
//
// The array lives in the library's code object, so each GPU the library runs
// on holds its own copy from the moment the code object is loaded on it
// until the process ends.  Its device address is looked up once per device
// (with that device current) and kept; host code never passes the array's
// name itself, which on the host is only a stand-in for the symbol.
//
// Every call on one GPU uses the same array: calls that overlap on one GPU
// (two streams, two host threads) race on it and must be serialised by the
// caller.  Nothing in the array has to start at zero: the limb split writes
// every byte of the planes the product reads (padding included), and every
// split-K part writes its whole partial result before the combining pass
// reads it.
#include <mutex>

#include "ffp_internal.hpp"

namespace ffp {

constexpr size_t kScratchBytes = (size_t)FFP_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) char scratch[kScratchBytes];

namespace {
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices];  // device address of `scratch` on each device

// device address of this device's copy of the array (looked up on the first
// call made with the device current)
int scratch_ptr(void **out) {
    int dev = 0;
    FFP_HIP_CHECK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return FFP_E_NODEVICE;
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        FFP_HIP_CHECK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr) return FFP_E_NODEVICE;
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return FFP_OK;
}
}  // namespace

}  // namespace ffp

using namespace ffp;

extern "C" {

size_t ffp_noalloc_scratch_bytes(void) { return kScratchBytes; }

int ffp_fgemm_noalloc(int transA, int transB, int64_t m, int64_t n, int64_t k, uint32_t p, uint32_t alpha,
                      const int32_t *A, int64_t lda, const int32_t *B, int64_t ldb, uint32_t beta, int32_t *C,
                      int64_t ldc, int path, ffp_stream_t stream) {
    int eff = 0;
    FFP_CHECK(fgemm_validate(transA, transB, m, n, k, p, alpha, A, lda, B, ldb, beta, C, ldc, path, &eff));
    if (m == 0 || n == 0) return FFP_OK;
    size_t need = ffp_fgemm_workspace(transA, transB, m, n, k, p, eff);
    if (need > kScratchBytes) {
        // the limb planes of an INT8 product do not fit: an explicit INT8
        // request is refused; AUTO runs the product on the FP64 path, which
        // needs no workspace and gives the same bits
        if (path == FFP_PATH_INT8) return FFP_E_SCRATCH;
        eff = FFP_PATH_FP64;
        need = 0;
    }
    void *base = nullptr;
    if (need > 0) FFP_CHECK(scratch_ptr(&base));
    Field F(p);
    Arena ar;
    ar.base = (char *)base;
    ar.cap = need > 0 ? kScratchBytes : 0;
    return fgemm_any(eff, F, transA, transB, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, ar, (hipStream_t)stream);
}

}  // extern "C"
