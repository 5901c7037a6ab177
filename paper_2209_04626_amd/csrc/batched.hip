// placeholder, replaced by the persistent batched kernel
#include "../../include/mpjsvd.h"
#include <stdlib.h>
extern "C" int svd_batched_plan_create(int batch, const int *h_m, const int *h_n,
                                       const svd_opts *o, void **plan, size_t *work_bytes) {
    (void)batch; (void)h_m; (void)h_n; (void)o; (void)plan; (void)work_bytes;
    return SVD_ERR_HIP;
}
extern "C" int svd_batched(void *plan, const double *A_base, double *S_base, double *U_base,
                           double *V_base, void *work, size_t work_bytes, svd_batch_info *info,
                           void *stream) {
    (void)plan; (void)A_base; (void)S_base; (void)U_base; (void)V_base; (void)work;
    (void)work_bytes; (void)info; (void)stream;
    return SVD_ERR_HIP;
}
extern "C" void svd_batched_plan_destroy(void *plan) { (void)plan; }
