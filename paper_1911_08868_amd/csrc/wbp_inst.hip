// One block length's weighted-BP kernels; built once per PBP_NLOG = 4..10.
#include "wbp_inst.h"

#define PBP_CAT2(a, b) a##b
#define PBP_CAT(a, b) PBP_CAT2(a, b)

namespace pbp {
int PBP_CAT(run_wbp_n, PBP_NLOG)(const WbpLaunch &L) { return run_wbp_n<PBP_NLOG>(L); }
}  // namespace pbp
