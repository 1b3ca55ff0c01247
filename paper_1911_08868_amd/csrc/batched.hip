// batched.hip -- persistent mixed-length decoding from a device work queue.
#include "internal.h"

using namespace pbp;

extern "C" {
size_t polar_batched_workspace_bytes(int32_t n_codes) { (void)n_codes; return 0; }
int pp_mt_bp_decode_batched(const pc_code *const *, int32_t, const int32_t *, const int64_t *,
                            const float *, int64_t, const int32_t *, const pc_bp_params *,
                            const pc_pp_params *, uint8_t *, const int64_t *, int32_t *,
                            uint8_t *, void *, size_t, const pc_launch_cfg *, void *) {
    return fail(PC_ENOTSUP, "batched decoding not built yet");
}
}
