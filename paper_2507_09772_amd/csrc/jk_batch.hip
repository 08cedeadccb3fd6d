// jk_batch.hip -- batched many-molecule builds (placeholder until the
// persistent queue kernel lands).
#include <hip/hip_runtime.h>

#include "../../include/jk.h"

extern "C" int jk_batch_create(jk_plan *const *, int32_t, int32_t, int32_t, double, jk_batch **out) {
    if (out) *out = nullptr;
    return JK_EUNSUPPORTED;
}
extern "C" int jk_batch_execute(jk_batch *, const double *const *, double *const *, double *const *, void *) {
    return JK_EUNSUPPORTED;
}
extern "C" void jk_batch_destroy(jk_batch *) {}
