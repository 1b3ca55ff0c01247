// decode_inst.h -- launch of the decode kernel for one block length.  Each
// decode_nXX.hip includes this with its own NLOG so the instantiations build
// in parallel translation units.
#pragma once

#include "decode_kernel.h"
#include "internal.h"

namespace pbp {

struct DecodeLaunch {
    DecodeArgs args;
    int kp = 0;
    bool scaled = false, gmode = false;
    bool trace = false;  // decision-history kernels (rho 2 only)
    int rho = 2, slots = 0, grid = 0;
    int64_t F = 0;
    hipStream_t stream = nullptr;
};

template <int NLOG, int KP, int RHO, bool SC, bool GM, bool TR>
int run_decode(const DecodeLaunch &L) {
    using P = Plan<NLOG, KP, RHO>;
    const int TPS = P::TPS;
    int S = L.slots;
    if (S <= 0) S = TPS >= 256 ? 1 : 256 / TPS;
    constexpr int LB = TPS > 256 ? TPS : 256;  // the kernel's launch bound
    if (S * TPS > LB) return fail(PC_EINVAL, "slots * threads per frame exceeds the launch bound");
    const size_t lds = DecodeLds<P>::bytes(S);
    if (lds > 160 * 1024) return fail(PC_EINVAL, "LDS budget exceeded for this launch shape");
    auto kern = k_decode<NLOG, KP, RHO, SC, GM, TR>;
    int grid = L.grid;
    if (grid <= 0) {
        int per_cu = 0;
        hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, S * TPS, lds);
        if (e != hipSuccess) return hip_fail(e, "occupancy query");
        if (per_cu < 1) per_cu = 1;
        grid = per_cu * device_cu_count();
    }
    const int64_t need = (L.F + S - 1) / S;
    if (grid > need) grid = (int)need;
    if (grid < 1) grid = 1;
    hipLaunchKernelGGL(kern, dim3(grid), dim3(S * TPS), lds, L.stream, L.args);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "decode launch");
    return PC_OK;
}

template <int NLOG, int KP, int RHO, bool TR>
int run_decode_flags(const DecodeLaunch &L) {
    if constexpr (KP == 0) {
        if (L.gmode)
            return L.scaled ? run_decode<NLOG, KP, RHO, true, true, TR>(L)
                            : run_decode<NLOG, KP, RHO, false, true, TR>(L);
        return L.scaled ? run_decode<NLOG, KP, RHO, true, false, TR>(L)
                        : run_decode<NLOG, KP, RHO, false, false, TR>(L);
    } else {
        if (L.gmode) return fail(PC_ENOTSUP, "the G test is only built for the original graph");
        return L.scaled ? run_decode<NLOG, KP, RHO, true, false, TR>(L)
                        : run_decode<NLOG, KP, RHO, false, false, TR>(L);
    }
}

template <int NLOG, int RHO, bool TR>
int run_decode_kp(const DecodeLaunch &L) {
    if (L.kp == 0) return run_decode_flags<NLOG, 0, RHO, TR>(L);
    if (L.kp == NLOG) {
        if constexpr (NLOG >= 2) return run_decode_flags<NLOG, NLOG, RHO, TR>(L);
    }
    switch (L.kp) {
        case 2: if constexpr (NLOG > 2) return run_decode_flags<NLOG, 2, RHO, TR>(L); break;
        case 3: if constexpr (NLOG > 3) return run_decode_flags<NLOG, 3, RHO, TR>(L); break;
        case 4: if constexpr (NLOG > 4) return run_decode_flags<NLOG, 4, RHO, TR>(L); break;
        case 5: if constexpr (NLOG > 5) return run_decode_flags<NLOG, 5, RHO, TR>(L); break;
        default: break;
    }
    return fail(PC_ENOTSUP, "permuted range k must be 2..5 or n in this build");
}

// TR: the decision-history kernels, built with two rows per thread only
template <int NLOG, bool TR>
int run_decode_n(const DecodeLaunch &L) {
    if constexpr (NLOG == 1) {
        return run_decode_kp<1, 1, TR>(L);
    } else {
        if (L.rho == 3) {
            if constexpr (NLOG >= 3 && !TR) return run_decode_kp<NLOG, 3, TR>(L);
            return fail(TR ? PC_ENOTSUP : PC_EINVAL, TR ? "decision history is built for rho 2" : "rho exceeds log2 N");
        }
        if (L.rho != 2) return fail(PC_EINVAL, "rho must be 2 or 3");
        return run_decode_kp<NLOG, 2, TR>(L);
    }
}

}  // namespace pbp

namespace pbp {
// dispatch on log2 N to the per-length translation units
int launch_decode_n(int n, const DecodeLaunch &L);
}  // namespace pbp
