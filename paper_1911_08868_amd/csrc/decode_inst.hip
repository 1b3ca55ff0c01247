// One block length's decode kernels; built once per PBP_NLOG = 1..12, and
// once more with PBP_TRACE=1 for the decision-history kernels.
#include "decode_inst.h"

#define PBP_CAT2(a, b) a##b
#define PBP_CAT(a, b) PBP_CAT2(a, b)

namespace pbp {
#if PBP_TRACE
int PBP_CAT(run_decode_trace_n, PBP_NLOG)(const DecodeLaunch &L) { return run_decode_n<PBP_NLOG, true>(L); }
#else
int PBP_CAT(run_decode_n, PBP_NLOG)(const DecodeLaunch &L) { return run_decode_n<PBP_NLOG, false>(L); }
#endif
}  // namespace pbp
