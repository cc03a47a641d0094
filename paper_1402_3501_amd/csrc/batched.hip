// Batched persistent PLUQ.
#include "ffp_internal.hpp"

namespace ffp {

size_t pluq_batched_ws(int32_t batch, int32_t max_m, int32_t max_n) {
    (void)batch; (void)max_m; (void)max_n;
    return 0;
}

int pluq_batched_run(const Field &F, int32_t batch, const int32_t *m_arr, const int32_t *n_arr,
                     int32_t max_m, int32_t max_n, int32_t *A, const int64_t *A_off, int32_t *P,
                     const int64_t *P_off, int32_t *Q, const int64_t *Q_off, int32_t *rank,
                     int32_t *rrp, int32_t *crp, Arena &ws, hipStream_t s) {
    return FFP_E_UNSUPPORTED;
}

}  // namespace ffp
