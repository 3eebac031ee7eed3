// Entry points whose kernels are not built yet: they report UNSUPPORTED.
#include "hvms.h"

extern "C" {
int hvms_cdf_forward(const float *, const float *, float *, int64_t, void *) { return HVMS_ERR_UNSUPPORTED; }
int64_t hvms_cdf_workspace_bytes(int64_t) { return HVMS_ERR_UNSUPPORTED; }
int hvms_cdf_backward(const float *, const float *, const float *, float *, float *, int64_t, void *,
                      size_t, void *)
{
    return HVMS_ERR_UNSUPPORTED;
}
int hvms_cdf_adam_step(float *, float *, float *, const float *, int32_t, float, float, float, float,
                       void *)
{
    return HVMS_ERR_UNSUPPORTED;
}
int64_t hvms_cdf_train_workspace_bytes(int64_t) { return HVMS_ERR_UNSUPPORTED; }
int hvms_cdf_train(float *, float *, float *, const int32_t *, int64_t, int64_t, int32_t, float,
                   uint64_t, void *, size_t, void *)
{
    return HVMS_ERR_UNSUPPORTED;
}
}
