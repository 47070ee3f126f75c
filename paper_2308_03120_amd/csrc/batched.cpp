// Batched evaluation of many matrices' expressions in one persistent launch.
#include "internal.h"
#include "runtime.h"

namespace coot {
void batch_destroy_all() {}
}  // namespace coot

extern "C" {
int coot_batch_create(const coot_batch*, void*, coot_batch_plan**)
{
    coot::set_error(COOT_ERR_UNSUPPORTED, "batched evaluation not built yet");
    return COOT_ERR_UNSUPPORTED;
}
int coot_batch_run(coot_batch_plan*, void*) { return COOT_ERR_UNSUPPORTED; }
int coot_batch_destroy(coot_batch_plan*) { return COOT_OK; }
}
