// wbp.hip -- weighted (unrolled) BP forward and adjoint kernels.
#include "internal.h"

using namespace pbp;

extern "C" {
size_t wbp_workspace_bytes(const pc_code *code, int64_t F, int32_t T_unroll) {
    (void)code; (void)F; (void)T_unroll;
    return 0;
}
int wbp_forward(const pc_code *, const float *, int64_t, const float *, int32_t,
                const pc_pp_params *, float *, void *, size_t, void *) {
    return fail(PC_ENOTSUP, "weighted BP not built yet");
}
int wbp_backward(const pc_code *, const float *, int64_t, const float *, int32_t,
                 const pc_pp_params *, const float *, float *, void *, size_t, void *) {
    return fail(PC_ENOTSUP, "weighted BP not built yet");
}
}
