// One block length's decode kernels; built once per PBP_NLOG = 1..12.
#include "decode_inst.h"

#define PBP_CAT2(a, b) a##b
#define PBP_CAT(a, b) PBP_CAT2(a, b)

namespace pbp {
int PBP_CAT(run_decode_n, PBP_NLOG)(const DecodeLaunch &L) { return run_decode_n<PBP_NLOG>(L); }
}  // namespace pbp
