// rad_batched.hip -- independent blocks in one persistent launch (placeholder until implemented).
#include "rad_host.h"

using namespace vr;

extern "C" size_t rad_batched_workspace_bytes(int, const rad_block_desc_t *, const rad_params_t *) { return 0; }
extern "C" int rad_plan_batched(int, const rad_block_desc_t *, const rad_params_t *, void *, size_t, void *, rad_plan *out)
{
    if (out) *out = nullptr;
    return fail(RAD_ENOTIMPL, "batched path not built yet");
}
extern "C" size_t rad_autotune_scratch_bytes(rad_plan) { return 0; }
extern "C" int rad_autotune_batched(rad_plan, double *, double *, double *, const void *, const void *, const void *,
                                    const void *, void *, size_t, void *)
{
    return fail(RAD_ENOTIMPL, "batched path not built yet");
}
extern "C" int rad_step_batched(rad_plan, double *, double *, double *, const void *, const void *, const void *,
                                const void *, rad_stats_t *, void *)
{
    return fail(RAD_ENOTIMPL, "batched path not built yet");
}
extern "C" void rad_plan_destroy(rad_plan) {}
