// Fused matrix-core step (placeholder until the kernel lands).
#include "fe_plan.h"

namespace fe {
bool fused_supported(int, int) { return false; }
hipError_t fused_upload(const float *, const float *, int, int, FusedBank *) { return hipSuccess; }
void fused_release(FusedBank *) {}
void make_plan(int, const fe_job *, int, Plan *) {}
hipError_t run_fused(const FusedBank &, const Plan &, const fe_job *, int, float **, float **,
                     void *, hipStream_t) { return hipErrorNotSupported; }
}  // namespace fe
