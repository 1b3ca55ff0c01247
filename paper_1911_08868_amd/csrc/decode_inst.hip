// One block length's decode kernels; built once per PBP_NLOG = 1..12 for each
// kernel family PBP_VARIANT (0 min-sum, 1 with decision history, 2 exact
// boxplus, 3 with noise injection).
#include "decode_inst.h"

#define PBP_CAT2(a, b) a##b
#define PBP_CAT(a, b) PBP_CAT2(a, b)

namespace pbp {
#if PBP_VARIANT == 1
int PBP_CAT(run_decode_trace_n, PBP_NLOG)(const DecodeLaunch &L) { return run_decode_n<PBP_NLOG, 1>(L); }
#elif PBP_VARIANT == 2
int PBP_CAT(run_decode_exact_n, PBP_NLOG)(const DecodeLaunch &L) { return run_decode_n<PBP_NLOG, 2>(L); }
#elif PBP_VARIANT == 3
int PBP_CAT(run_decode_noise_n, PBP_NLOG)(const DecodeLaunch &L) { return run_decode_n<PBP_NLOG, 3>(L); }
#else
int PBP_CAT(run_decode_n, PBP_NLOG)(const DecodeLaunch &L) { return run_decode_n<PBP_NLOG, 0>(L); }
#endif
}  // namespace pbp
