// Batches of independent products (placeholder until the persistent kernel lands).
#include <hip/hip_runtime.h>

#include "qmm_internal.h"

using namespace qmm;

struct qmm_batched {
    int64_t count;
};

extern "C" qmm_status qmm_batched_create(int64_t count, const qmm_problem *probs, uint32_t flags, qmm_batched **out) {
    (void)count; (void)probs; (void)flags;
    if (out) *out = nullptr;
    return fail(QMM_EUNSUPPORTED, "batched products are not built yet");
}
extern "C" qmm_status qmm_gemm_mod_p_batched(qmm_batched *batch, void *stream) {
    (void)batch; (void)stream;
    return fail(QMM_EUNSUPPORTED, "batched products are not built yet");
}
extern "C" qmm_status qmm_batched_plan(const qmm_batched *batch, int64_t i, qmm_plan *out) {
    (void)batch; (void)i; (void)out;
    return fail(QMM_EUNSUPPORTED, "batched products are not built yet");
}
extern "C" qmm_status qmm_batched_destroy(qmm_batched *batch) {
    delete batch;
    return QMM_OK;
}
