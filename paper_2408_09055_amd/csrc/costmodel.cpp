// Learned cost model hooks used by the planner.
#include "plan.hpp"

namespace qk {

bool learned_available(qk_ctx* ctx, int dtype)
{
    (void)ctx; (void)dtype;
    return false;
}

int learned_predict(qk_ctx* ctx, int dtype, const float* feats, int64_t cnt, float* out)
{
    (void)ctx; (void)dtype; (void)feats; (void)cnt; (void)out;
    return fail(QK_EUNSUPPORTED, "learned cost model not loaded");
}

}  // namespace qk
