// qai_batch.hip -- batched form (placeholder entry points until the
// persistent kernel lands): every call reports QAI_ESTATE.
#include "qai.h"

extern "C" {

size_t qai_batch_workspace_bytes(int, const int64_t (*)[3]) { return 0; }

int qai_batch_plan_create(int, const float* const*, const int64_t (*)[3], const float*, float* const*,
                          const qai_params*, void*, size_t, void*, qai_batch_plan** plan)
{
    if (plan)
        *plan = nullptr;
    return QAI_ESTATE;
}

int qai_batch_plan_launch(qai_batch_plan*, void*) { return QAI_ESTATE; }
int qai_batch_plan_launch_per_field(qai_batch_plan*, void*) { return QAI_ESTATE; }
void qai_batch_plan_destroy(qai_batch_plan*) {}

} // extern "C"
