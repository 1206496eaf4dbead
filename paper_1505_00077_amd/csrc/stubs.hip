// Entry points not yet implemented: they validate nothing and report
// BF_EUNSUPPORTED.
#include "../../include/bfgp.h"

extern "C" {
int bf_gp_plan_batched(const bf_gp_item *, int, unsigned, void **) { return BF_EUNSUPPORTED; }
size_t bf_gp_plan_workspace_bytes(const void *) { return 0; }
int bf_gp_plan_upload(void *, void *, size_t, void *) { return BF_EUNSUPPORTED; }
int bf_gp_forward_batched(void *, void *, size_t, void *) { return BF_EUNSUPPORTED; }
void bf_gp_plan_free(void *) {}
}
