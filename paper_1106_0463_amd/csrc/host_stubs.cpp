// Batch and GEMM plan entry points (placeholders until implemented).
#include "lc_internal.h"

namespace lc {
lc_status fail_status(lc_status s, const std::string &msg);
void destroy_gemm(lc_plan_s *) {}
void info_gemm(lc_plan_s *, lc_plan_desc *) {}
lc_status nodes_gemm(lc_plan_s *, const double **, int64_t *, int32_t *) { return LC_ERR_UNSUPPORTED; }
}  // namespace lc

extern "C" {
lc_status lc_plan_gemm(int32_t, int64_t, int64_t, lc_gemm_mode, lc_plan_t *) {
    return lc::fail_status(LC_ERR_UNSUPPORTED, "not built yet");
}
lc_status lc_execute_gemm(lc_plan_t, const double *, int32_t, double *, hipStream_t) {
    return lc::fail_status(LC_ERR_UNSUPPORTED, "not built yet");
}
lc_status lc_plan_gemm_reserve(lc_plan_t, int32_t) { return lc::fail_status(LC_ERR_UNSUPPORTED, "not built yet"); }
lc_status lc_plan_gemm_matrix(lc_plan_t, const double **) { return lc::fail_status(LC_ERR_UNSUPPORTED, "not built yet"); }
lc_status lc_autotune(lc_plan_t, hipStream_t) { return lc::fail_status(LC_ERR_UNSUPPORTED, "not built yet"); }
}
