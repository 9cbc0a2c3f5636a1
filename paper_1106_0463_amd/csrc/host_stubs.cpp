// Autotuner entry point (placeholder until implemented).
#include "lc_internal.h"

namespace lc {
lc_status fail_status(lc_status s, const std::string &msg);
}  // namespace lc

extern "C" {
lc_status lc_autotune(lc_plan_t, hipStream_t) { return lc::fail_status(LC_ERR_UNSUPPORTED, "lc_autotune: not built yet"); }
}
